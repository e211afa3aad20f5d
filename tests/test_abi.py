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
    (512, 1, dict(block=1024), mxfft.EINVAL),        # B > n
    (64, 1, dict(fmt="fp16", tau=-1.0), mxfft.EINVAL),
    (64, 1, dict(fmt=9), mxfft.EINVAL),
    (64, 1, dict(fmt="e2m3", block=48), mxfft.EINVAL),   # MXFP6 blocks follow the MX rules
    (64, 1, dict(fmt="e3m2", block=256), mxfft.EINVAL),
    (64, 1, dict(tau=101.0), mxfft.EINVAL),
    (64, 1, dict(target=0.0), mxfft.EINVAL),
    (64, 1, dict(target=float("nan")), mxfft.EINVAL),
    (64, 1, dict(tau_min=0.0), mxfft.EINVAL),       # tau_min > 0
    (64, 1, dict(tau_min=float("inf")), mxfft.EINVAL),
    (64, 1, dict(k_min=3, k_max=2), mxfft.EINVAL),
    (64, 1, dict(flags=0x80), mxfft.EINVAL),
    (64, 1, dict(flags=0x40), mxfft.EINVAL),
    (64, 1, dict(fmt="fp16", flags=mxfft.DEBUG_CAPTURE), mxfft.EINVAL),   # capture: MX formats only
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


def test_tune_cache_lookup_host(tmp_path):
    """The tuning cache is plain text, one entry per line; lookups match on
    (arch, n, format, block), block counting only for the MX formats, and
    skip malformed lines."""
    path = tmp_path / "tune.json"
    path.write_text(
        '{"arch": "gfx950:sramecc+:xnack-", "n": 256, "format": 0, "block": 32, "lines": 8, "ms": 0.25}\n'
        'not an entry\n'
        '{"arch": "gfx950:sramecc+:xnack-", "n": 256, "format": 0, "block": 16, "lines": 4, "ms": 0.5}\n'
        '{"arch": "gfx942", "n": 256, "format": 0, "block": 32, "lines": 2, "ms": 1.0}\n'
        '{"arch": "gfx950:sramecc+:xnack-", "n": 64, "format": 2, "block": 0, "lines": 16, "ms": 0.125}\n'
        '{"arch": "gfx950:sramecc+:xnack-", "n": 32, "format": 0, "block": 32, "lines": 8, "ms": 0.1, "single": 1}\n')
    arch = "gfx950:sramecc+:xnack-"
    off = {"single": False, "stats": 0, "chunks": 0}
    assert mxfft.tune_cache_lookup(str(path), arch, 256) == dict(off, lines=8, ms=0.25)
    assert mxfft.tune_cache_lookup(str(path), arch, 256, block=16) == dict(off, lines=4, ms=0.5)
    assert mxfft.tune_cache_lookup(str(path), "gfx942", 256) == dict(off, lines=2, ms=1.0)
    assert mxfft.tune_cache_lookup(str(path), arch, 64, fmt="fp16", block=8) == dict(off, lines=16, ms=0.125)
    # n <= 64: the single-launch choice (entries without the key keep the line kernels)
    assert mxfft.tune_cache_lookup(str(path), arch, 32) == dict(off, lines=8, ms=0.1, single=True)
    assert mxfft.tune_cache_lookup(str(path), arch, 128) is None
    assert mxfft.tune_cache_lookup(str(path), arch, 256, fmt="e5m2") is None
    assert mxfft.tune_cache_lookup(str(tmp_path / "missing.json"), arch, 256) is None


def batch_status(groups, **kw):
    p = mxfft.make_params(**kw)
    arr = (mxfft.Group * max(1, len(groups)))(*[mxfft.Group(*g) for g in groups])
    h = ctypes.c_void_p()
    return mxfft.lib().mxfft_batch_create(ctypes.byref(h), arr, len(groups), ctypes.byref(p), None, None)


@pytest.mark.parametrize("groups", [
    [],                                          # no group
    [(63, 1, 0)],                                # not a power of two
    [(64, 0, 0)],                                # empty group
    [(8192, 1, 0)],                              # above 4096
    [(64, 2, 0), (32, 1, 64 * 64)],              # second group starts inside the first
    [(16, 1, 1000), (16, 4, 800)],               # overlap in the other order
])
def test_batch_create_rejects_bad_groups(groups):
    """Group lists are checked on the host before any device call."""
    assert batch_status(groups) == mxfft.EINVAL


def test_plan_bytes_host():
    """The device-memory estimate runs on the host (no HIP call) and follows
    the workspace of each path: the MX intermediate (2 + 2/B bytes per value)
    and the 16-bit one (4 bytes per value) at n = 128 .. 1024,
    none for the generic line kernels; invalid arguments fail like mxfft_plan."""
    per = lambda n, **kw: (mxfft.plan_bytes(n, 8, **kw) - mxfft.plan_bytes(n, 4, **kw)) // 4   # noqa: E731
    mx = per(512, fmt="e4m3", block=32)
    assert 512 * 512 * (2 + 2 / 32) <= mx < 512 * 512 * (2 + 2 / 32) + 64 * 1024
    h = per(512, fmt="fp16")
    assert 512 * 512 * 4 <= h < 512 * 512 * 4 + 64 * 1024
    m256 = per(256, fmt="e4m3", block=32)
    assert 256 * 256 * (2 + 2 / 32) <= m256 < 256 * 256 * (2 + 2 / 32) + 64 * 1024
    m1k = per(1024, fmt="e5m2", block=16)
    assert 1024 * 1024 * (2 + 2 / 16) <= m1k < 1024 * 1024 * (2 + 2 / 16) + 64 * 1024
    assert per(64, fmt="e4m3", block=32) < 64 * 1024        # generic line kernels: no intermediate
    h1k = per(1024, fmt="bf16")
    assert 1024 * 1024 * 4 <= h1k < 1024 * 1024 * 4 + 64 * 1024
    assert per(64, fmt="fp16") < 64 * 1024
    assert per(512, fmt="fp32") < 64 * 1024
    # the 6-bit formats ride in 8-bit containers: the same buffers as MXFP8
    # wherever they take the register-resident path (blocks of 16 and 32)
    for n in (128, 256, 512, 1024):
        for f6, f8 in (("e2m3", "e4m3"), ("e3m2", "e5m2")):
            for blk in (16, 32):
                assert mxfft.plan_bytes(n, 3, fmt=f6, block=blk) == mxfft.plan_bytes(n, 3, fmt=f8, block=blk), (n, f6, blk)
    assert per(512, fmt="e2m3", block=8) < 64 * 1024        # blocks of 8: line kernels
    for bad in (dict(n=63), dict(n=64, max_batch=0), dict(n=64, block=48)):
        n, mb = bad.pop("n"), bad.pop("max_batch", 1)
        with pytest.raises(mxfft.MxfftError):
            mxfft.plan_bytes(n, mb, **bad)


def test_blocks_up_to_n_are_accepted():
    """Any power-of-two B from 2 to n (host check, no GPU)."""
    for n, b in ((256, 256), (512, 512), (1024, 1024), (4096, 4096), (2048, 256)):
        assert mxfft.plan_bytes(n, 1, block=b) > 0


def test_quantize_output_flag_is_known():
    """MXFFT_QUANTIZE_OUTPUT is accepted for every format (host check, no GPU)."""
    for fmt in ("e4m3", "e2m3", "fp16", "fp32"):
        assert mxfft.plan_bytes(256, 2, fmt=fmt, flags=mxfft.QUANTIZE_OUTPUT) > 0


def test_any_positive_tau_min_is_accepted():
    """Alg. 1 takes any tail floor: plans with tau_min not a power of two are
    valid (checked host-side through mxfft_plan_bytes, no GPU call)."""
    for t in (0.3, 1e-3, 3.0 * 2.0 ** -7, 314572.8):
        assert mxfft.plan_bytes(256, 4, tau_min=t) > 0
