"""The C ABI library loads on the host and exports every entry point that
include/mxfft.h declares; host-side argument checks reject bad input before
any device call (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2512_04317_amd import mxfft

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mxfft.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mxfft_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = mxfft.lib()
    decl = declared_functions()
    assert decl, "no declarations found"
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(mxfft.EXPORTS) == decl


def test_defaults_and_strings():
    p = mxfft.default_params()
    assert p.struct_size == ctypes.sizeof(mxfft.Params)
    assert (p.format, p.block, p.target, p.tau_pct, p.tau_min) == (mxfft.E4M3, 32, 128.0, 5.0, 2.0 ** -6)
    assert (p.k_min, p.k_max, p.flags) == (mxfft.INT32_MIN, mxfft.INT32_MAX, 0)
    assert mxfft.status_string(mxfft.ENONFINITE) == "non-finite input"
    assert mxfft.lib().mxfft_version() >= 100


def plan_status(n, max_batch, **kw):
    p = mxfft.make_params(**kw)
    h = ctypes.c_void_p()
    return mxfft.lib().mxfft_plan(ctypes.byref(h), n, max_batch, ctypes.byref(p), None)


@pytest.mark.parametrize("n,mb,kw,st", [
    (63, 1, {}, mxfft.EINVAL),                       # not a power of two
    (1, 1, {}, mxfft.EINVAL),
    (8192, 1, {}, mxfft.EINVAL),                     # above 4096
    (64, 0, {}, mxfft.EINVAL),
    (64, 1, dict(block=48), mxfft.EINVAL),
    (64, 1, dict(block=1), mxfft.EINVAL),
    (16, 1, dict(block=32), mxfft.EINVAL),           # B > n
    (512, 1, dict(block=256), mxfft.EUNSUPPORTED),   # B > 128 not built
    (64, 1, dict(fmt="fp16", tau=-1.0), mxfft.EINVAL),
    (64, 1, dict(fmt=9), mxfft.EINVAL),
    (64, 1, dict(tau=101.0), mxfft.EINVAL),
    (64, 1, dict(target=0.0), mxfft.EINVAL),
    (64, 1, dict(target=float("nan")), mxfft.EINVAL),
    (64, 1, dict(tau_min=0.3), mxfft.EUNSUPPORTED),  # tau_min must be a power of two
    (64, 1, dict(k_min=3, k_max=2), mxfft.EINVAL),
    (64, 1, dict(flags=0x80), mxfft.EINVAL),
])
def test_plan_argument_checks(n, mb, kw, st):
    assert plan_status(n, mb, **kw) == st


def test_bad_struct_size_and_nulls():
    p = mxfft.default_params()
    p.struct_size = 12
    h = ctypes.c_void_p()
    assert mxfft.lib().mxfft_plan(ctypes.byref(h), 64, 1, ctypes.byref(p), None) == mxfft.EINVAL
    assert mxfft.lib().mxfft_plan(None, 64, 1, ctypes.byref(mxfft.default_params()), None) == mxfft.EINVAL
    assert mxfft.lib().mxfft_forward(None, None, None, 1, None, None) == mxfft.EINVAL
    assert mxfft.lib().mxfft_inverse(None, None, None, 1, None, None) == mxfft.EINVAL
    assert mxfft.lib().mxfft_roundtrip(None, None, None, 1, None, None) == mxfft.EINVAL
    assert mxfft.lib().mxfft_plan_last_status(None, None) == mxfft.EINVAL
    assert mxfft.lib().mxfft_plan_destroy(None) == mxfft.OK
