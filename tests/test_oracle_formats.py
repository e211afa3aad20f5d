"""Pins of the oracle's number formats (OCP FP8 E4M3 / E5M2, FP16, BF16).

Each check compares the oracle's quantiser with something it does not use: the
format's code table searched by brute force, facts of the OCP 8-bit format
definition, and the independent casts of numpy and torch.
"""
import numpy as np
import pytest
import torch

import oracle as O


def finite_table(f):
    """All finite code values of an 8-bit format, decoded one code at a time."""
    codes = [c for c in range(256)]
    vals = np.array([O.decode_code(f, c) for c in codes])
    keep = np.isfinite(vals)
    return np.array(codes)[keep], vals[keep]


@pytest.mark.parametrize("f", [O.E4M3, O.E5M2])
def test_code_roundtrip_exhaustive(f):
    codes, vals = finite_table(f)
    for c, v in zip(codes, vals):
        assert O.quantize(f, [v])[0] == v
        assert O.encode_code(f, v) == c


def test_format_landmarks():
    # OCP 8-bit float definitions: E4M3 has no infinities and one NaN pattern
    # per sign; E5M2 follows IEEE-754 conventions.
    assert O.decode_code(O.E4M3, 0x7E) == 448.0
    assert np.isnan(O.decode_code(O.E4M3, 0x7F))
    assert O.decode_code(O.E4M3, 0x78) == 256.0
    assert O.decode_code(O.E4M3, 0x01) == 2.0 ** -9
    assert O.decode_code(O.E4M3, 0x08) == 2.0 ** -6
    assert O.decode_code(O.E5M2, 0x7B) == 57344.0
    assert O.decode_code(O.E5M2, 0x7C) == np.inf
    assert np.isnan(O.decode_code(O.E5M2, 0x7D))
    assert O.decode_code(O.E5M2, 0x01) == 2.0 ** -16
    assert O.decode_code(O.E5M2, 0x04) == 2.0 ** -14
    assert O.decode_code(O.E4M3, 0x80) == 0.0 and np.signbit(O.decode_code(O.E4M3, 0x80))
    _, v4 = finite_table(O.E4M3)
    _, v5 = finite_table(O.E5M2)
    assert len(set(v4)) == 253 and len(set(v5)) == 247   # +-0 share a value


def brute_force_nearest(x, codes, vals, maxval):
    """Nearest finite code value, ties to the code with an even last bit,
    saturating above the largest finite value."""
    out = np.empty_like(x)
    for n, xi in enumerate(x):
        if abs(xi) >= maxval:
            out[n] = np.copysign(maxval, xi)
            continue
        d = np.abs(vals - xi)
        best = d.min()
        cand = [(c, v) for c, v, di in zip(codes, vals, d) if di == best]
        if len(cand) > 1:
            even = [cv for cv in cand if cv[0] % 2 == 0]
            cand = even
        v = cand[0][1]
        if v == 0.0:
            v = np.copysign(0.0, xi)
        out[n] = v
    return out


@pytest.mark.parametrize("f", [O.E4M3, O.E5M2])
def test_quantize_vs_brute_force(f):
    codes, vals = finite_table(f)
    mx = vals.max()
    rng = np.random.default_rng(1)
    x = np.concatenate([
        rng.uniform(-1.2 * mx, 1.2 * mx, 3000),
        np.exp(rng.uniform(np.log(2.0 ** -20), np.log(mx), 3000)) * rng.choice([-1, 1], 3000),
    ])
    # every midpoint between neighbouring values (ties) and a hair either side
    sv = np.unique(vals)
    mids = (sv[:-1] + sv[1:]) / 2
    x = np.concatenate([x, mids, np.nextafter(mids, np.inf), np.nextafter(mids, -np.inf), sv,
                        [mx + 1, -mx - 1, 1e30, -1e30]])
    got = O.quantize(f, x)
    exp = brute_force_nearest(x, codes, vals, mx)
    np.testing.assert_array_equal(got, exp)
    assert np.array_equal(np.signbit(got), np.signbit(exp))


@pytest.mark.parametrize("f,tdt,lim", [(O.E4M3, torch.float8_e4m3fn, 448.0),
                                       (O.E5M2, torch.float8_e5m2, 57344.0)])
def test_quantize_vs_torch_cast_in_range(f, tdt, lim):
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.uniform(-lim, lim, 200000),
                        np.exp(rng.uniform(-30, np.log(lim), 200000)) * rng.choice([-1, 1], 200000)])
    x = x.astype(np.float32)
    ref = torch.from_numpy(x).to(tdt).to(torch.float32).numpy()
    got = O.quantize(f, x.astype(np.float64))
    np.testing.assert_array_equal(got, ref.astype(np.float64))


def test_fp16_vs_numpy_cast():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(0, 1e4, 100000), np.exp(rng.uniform(-25, 12, 100000)),
                        [65519.99, 65520.0, 65536.0, 1e6, -1e6]]).astype(np.float32)
    with np.errstate(over="ignore"):
        ref = x.astype(np.float16).astype(np.float64)
    got = O.quantize(O.FP16, x.astype(np.float64))
    np.testing.assert_array_equal(got, ref)


def test_bf16_vs_torch_cast():
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.normal(0, 1e4, 100000), np.exp(rng.uniform(-80, 80, 100000))]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    got = O.quantize(O.BF16, x.astype(np.float64))
    np.testing.assert_array_equal(got, ref)


def test_e8m0_scale_values_vs_torch():
    # block scales 2^E, E in [-127, 127], are exactly the E8M0 values
    e = np.arange(-127, 128)
    vals = torch.from_numpy(np.ldexp(1.0, e).astype(np.float32)).to(torch.float8_e8m0fnu).to(torch.float32)
    np.testing.assert_array_equal(vals.numpy().astype(np.float64), np.ldexp(1.0, e))
