"""Pins of the oracle's MX block codec and MX butterfly (Sec. 2.2, Alg. 2).

The expected values below are worked out by hand from the OCP MX rule (shared
exponent floor(log2 amax) - emax_elem, element rounding to nearest even with
saturation) and from Alg. 2; each derivation is written next to its case.
"""
import math

import numpy as np
import pytest

import oracle as O


def test_block_exponent_rule():
    # amax = 1: floor(log2 1) = 0 -> E = 0 - 8 = -8 (E4M3), 0 - 15 = -15 (E5M2)
    assert O.mx_encode(O.E4M3, [1.0, 0.0])[0] == -8
    assert O.mx_encode(O.E5M2, [1.0, 0.0])[0] == -15
    # amax just below 1 falls in binade -1
    assert O.mx_encode(O.E4M3, [0.999, -0.5])[0] == -9
    # all-zero block: E = 0 and the zeros keep their signs
    E, m = O.mx_encode(O.E4M3, [0.0, -0.0, 0.0, -0.0])
    assert E == 0 and list(np.signbit(m)) == [False, True, False, True]
    # E8M0 clamp at -127: amax = 2^-140 -> floor - 8 = -148 -> -127
    E, m = O.mx_encode(O.E4M3, [2.0 ** -140, 0.0])
    assert E == -127
    # 2^-140 * 2^127 = 2^-13 is below half the smallest E4M3 subnormal 2^-9 -> 0
    assert m[0] == 0.0


def test_worked_twiddle_examples():
    s = math.sqrt(0.5)
    # E4M3: amax = s -> E = -1 - 8 = -9; s * 512 = 362.04 on grid 32 -> 352 -> 0.6875
    E, m = O.mx_encode(O.E4M3, [s, -s])
    assert E == -9 and list(m) == [352.0, -352.0]
    # E5M2: E = -1 - 15 = -16; s * 65536 = 46341 on grid 8192 -> 49152 -> 0.75
    E, m = O.mx_encode(O.E5M2, [s, -s])
    assert E == -16 and list(m) == [49152.0, -49152.0]
    # saturation: amax = cos(2 pi 16/1024) = 0.99518 -> E = -9; 509.5 rounds to
    # 512 which saturates to 448 -> 0.875 (12% low)
    c = math.cos(2 * math.pi * 16 / 1024)
    E, m = O.mx_encode(O.E4M3, [c, 0.1])
    assert E == -9 and m[0] == 448.0
    # and the same twiddle in a block that also holds 1: E = -8, 254.8 -> 256
    E, m = O.mx_encode(O.E4M3, [1.0, 0.0, c, 0.1])
    assert E == -8 and m[2] == 256.0


@pytest.mark.parametrize("f", [O.E4M3, O.E5M2])
def test_encode_postconditions_and_equivariance(f):
    info = O.fmt_info(f)
    rng = np.random.default_rng(5)
    for trial in range(300):
        n = int(rng.choice([2, 4, 8, 16, 32, 64]))
        v = (rng.normal(size=n) * np.exp(rng.normal(0, 4, size=n))).astype(np.float32).astype(np.float64)
        E, m = O.mx_encode(f, v)
        top = np.abs(m).max()
        # the block maximum lands in [2^emax, M_max] (saturation caps it)
        assert 2.0 ** info["emax"] <= top <= info["maxval"]
        np.testing.assert_array_equal(m, O.quantize(f, np.ldexp(v, -E)))
        j = int(rng.integers(-20, 20))
        E2, m2 = O.mx_encode(f, np.ldexp(v, j))
        assert E2 == E + j
        np.testing.assert_array_equal(m2, m)


def twiddle_block(f, js, m_size, inverse=False):
    w = np.array([O.twiddle64(j, m_size, inverse) for j in js])
    flat = np.empty(2 * len(w))
    flat[0::2], flat[1::2] = w.real, w.imag
    E, mant = O.mx_encode(f, flat)
    return mant[0::2] + 1j * mant[1::2], E


def test_butterfly_unit_twiddle_is_exact():
    # w = 1: x = 256 + 0i with Ew = -8.  The product 256*y has max in
    # [2^16, 448*2^8], so kr = 8 and the re-quantised product is y itself:
    # w*v equals the MX-encoded v exactly and y0/y1 are exact FP32 sums.
    rng = np.random.default_rng(6)
    for cb in (1, 2, 4, 16, 32):
        x, Ew = twiddle_block(O.E4M3, [0] * cb, 2)
        assert Ew == -8
        u = (rng.normal(size=cb) + 1j * rng.normal(size=cb)).astype(np.complex64)
        v = (rng.normal(size=cb) + 1j * rng.normal(size=cb)).astype(np.complex64)
        y0, y1, (Ev, kr, Eo) = O.mx_butterfly(O.E4M3, u, v, x, Ew)
        flat = np.empty(2 * cb)
        flat[0::2], flat[1::2] = v.real, v.imag
        E, mv = O.mx_encode(O.E4M3, flat)
        vq = np.ldexp(mv[0::2], E) + 1j * np.ldexp(mv[1::2], E)
        assert kr == 8 and Ev == E and Eo == Ew + Ev + kr
        np.testing.assert_array_equal(y0, (u.astype(np.complex128) + vq).astype(np.complex64))
        np.testing.assert_array_equal(y1, (u.astype(np.complex128) - vq).astype(np.complex64))


def test_butterfly_hand_traced():
    # One block of two butterflies, E4M3, twiddles [1, -i] (x = 256, -256i; Ew = -8),
    # u = [2, 0], v = [2.125, -0.125] (real).
    # v block: amax 2.125 -> Ev = 1 - 8 = -7; 2.125*128 = 272 on grid 32 is a tie
    # between 256 and 288 -> even -> 256; -0.125*128 = -16 exact.  y = [256, -16].
    # products: 256*256 = 65536 and -i*256*(-16) = +4096 i -> amax 65536 > 448,
    # kr = ceil(log2(65536/448)) = 8 -> p' = [256, 16 i], exact; Eout = -8-7+8 = -7
    # wv = [2, 0.125 i] -> y0 = [4, 0.125 i], y1 = [0, -0.125 i].
    x = np.array([256 + 0j, -256j])
    u = np.array([2, 0], np.complex64)
    v = np.array([2.125, -0.125], np.complex64)
    y0, y1, tr = O.mx_butterfly(O.E4M3, u, v, x, -8)
    assert tr == (-7, 8, -7)
    np.testing.assert_array_equal(y0, np.array([4, 0.125j], np.complex64))
    np.testing.assert_array_equal(y1, np.array([0, -0.125j], np.complex64))


def test_butterfly_renorm_postcondition():
    # after renormalisation the largest product magnitude lies in (M/2, M]
    rng = np.random.default_rng(7)
    for f in (O.E4M3, O.E5M2):
        M = O.fmt_info(f)["maxval"]
        for trial in range(200):
            cb = int(rng.choice([1, 2, 4, 8, 16, 32]))
            msize = int(rng.choice([4, 8, 64, 512]))
            j0 = int(rng.integers(0, msize // 2))
            x, Ew = twiddle_block(f, [(j0 + k) % (msize // 2) for k in range(cb)], msize)
            u = np.zeros(cb, np.complex64)
            v = (rng.normal(size=cb) + 1j * rng.normal(size=cb)).astype(np.complex64) * np.float32(
                np.exp(rng.normal(0, 5)))
            y0, y1, (Ev, kr, Eo) = O.mx_butterfly(f, u, v, x, Ew)
            flat = np.empty(2 * cb)
            flat[0::2], flat[1::2] = v.real, v.imag
            _, yv = O.mx_encode(f, flat)
            yv = yv[0::2] + 1j * yv[1::2]
            p = x * yv                                  # exact in FP64 for 8-bit elements
            a = max(np.abs(p.real).max(), np.abs(p.imag).max())
            assert kr >= 1 and M / 2 < a / 2.0 ** kr <= M
            # wv = y0 - u = y0: its value is a quantised product at scale 2^Eo
            q = np.ldexp(y0.astype(np.complex128).real, -Eo)
            np.testing.assert_array_equal(O.quantize(f, q), q)


def test_butterfly_zero_block():
    x, Ew = twiddle_block(O.E4M3, [0, 1, 2, 3], 16)
    u = np.array([1, 2, 3, 4], np.complex64)
    v = np.zeros(4, np.complex64)
    y0, y1, (Ev, kr, Eo) = O.mx_butterfly(O.E4M3, u, v, x, Ew)
    assert Ev == 0 and kr == 0
    np.testing.assert_array_equal(y0, u)
    np.testing.assert_array_equal(y1, u)


@pytest.mark.parametrize("f", [O.E4M3, O.E5M2])
def test_twiddle_codes_are_robust(f):
    """No twiddle element sits within 1e-9 (relative) of a rounding boundary of
    its block's grid, so any correctly computed FP64 cos/sin gives the same
    codes; the GPU plan generates its tables independently."""
    info = O.fmt_info(f)
    for L in range(1, 13):
        m = 1 << L
        h = m // 2
        for cb in (1, 2, 4, 8, 16, 32, 64):
            for j0 in range(0, h, max(cb, 1)) if cb <= h else [0]:
                js = list(range(j0, j0 + min(cb, h)))
                w = np.array([O.twiddle64(j, m) for j in js])
                flat = np.concatenate([w.real, w.imag])
                E, mant = O.mx_encode(f, flat)
                s = np.ldexp(np.abs(flat), -E)
                nz = s[(s > 0)]
                e = np.maximum(np.floor(np.log2(nz)), info["emin"])
                ulp = np.ldexp(1.0, (e - info["mbits"]).astype(int))
                frac = nz / ulp - np.floor(nz / ulp)
                exact = (frac == 0)
                assert np.all(exact | (np.abs(frac - 0.5) > 1e-9 * nz / ulp))
