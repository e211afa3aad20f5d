"""Pins of the oracle's global power-of-two prescale (Sec. 2.1, Alg. 1).

k1 = round(log2(T / amax)), k2 = ceil(log2(tau_min / p_tau)), k = max(k1, k2)
clipped; the cases below are worked by hand, or checked against exact rational
arithmetic (Python's Fraction) and numpy's percentile away from ties.
"""
from fractions import Fraction
import math

import numpy as np
import pytest

import oracle as O


def one(vals):
    return np.asarray(vals, np.complex64)


def test_hand_cases():
    # amax = 100, T = 2^7: log2(1.28) = 0.36 -> k1 = 0; tail 100 -> k2 = ceil(log2(2^-6/100)) < 0
    assert O.prescale(one([100]), target=2.0 ** 7)[1] == 0
    # amax = 2^10: log2(2^7 / 2^10) = -3 exactly
    assert O.prescale(one([2 ** 10, 1]), target=2.0 ** 7, tau_min=2.0 ** -20)[1] == -3
    # all zeros: k = 0
    assert O.prescale(np.zeros(16, np.complex64)) == (O.OK, 0)
    # k2 wins: values 1..21 (n = 21); tau = 5 -> pos = 20*5/100 = 1 -> p = 2;
    # tau_min = 2^10 -> k2 = ceil(log2(1024/2)) = 9; k1 = round(log2(128/21)) = 3
    st, k = O.prescale(one(np.arange(1, 22)), target=2.0 ** 7, tau=5.0, tau_min=2.0 ** 10)
    assert (st, k) == (O.OK, 9)
    # same with a floor of 2^2: k2 = ceil(log2(4/2)) = 1 < k1 = 3
    assert O.prescale(one(np.arange(1, 22)), tau=5.0, tau_min=4.0)[1] == 3


def test_percentile_interpolation():
    # 1..5 at tau = 30: pos = 4*30/100 = 1.2 -> p = 2 + 0.2*(3-2) = 2.2;
    # tau_min = 16: k2 = ceil(log2(16/2.2)) = ceil(2.86) = 3 (T = 2^-10 keeps k1 low)
    assert O.prescale(one([5, 4, 3, 2, 1]), target=2.0 ** -10, tau=30.0, tau_min=16.0)[1] == 3
    # tau = 37.5: pos = 1.5 -> p = 2.5; tau_min = 20: 20/2.5 = 8 = 2^3 exactly -> k2 = 3
    assert O.prescale(one([1, 2, 3, 4, 5]), target=2.0 ** -10, tau=37.5, tau_min=20.0)[1] == 3
    # a hair above 20 needs one more doubling
    assert O.prescale(one([1, 2, 3, 4, 5]), target=2.0 ** -10, tau=37.5, tau_min=20.000001)[1] == 4


def test_round_half_boundary_is_sqrt2():
    # k1 = t - e - [f > sqrt 2] for amax = f 2^e: the rounding boundary of
    # round(log2(T/amax)) sits at f = sqrt(2).  float32 values either side of it:
    a32 = np.float32(1.4142135)
    b32 = np.float32(1.4142137)
    assert Fraction(float(a32)) ** 2 < 2 < Fraction(float(b32)) ** 2
    assert O.prescale(one([a32]), target=2.0 ** 7, tau_min=2.0 ** -30)[1] == 7
    assert O.prescale(one([b32]), target=2.0 ** 7, tau_min=2.0 ** -30)[1] == 6


def exact_k(x, T, tau, tmin, kmin=None, kmax=None):
    """Reference built from exact rationals and numpy's order statistics."""
    m = np.sqrt(x.real.astype(np.float64) ** 2 + x.imag.astype(np.float64) ** 2).ravel()
    nz = np.sort(m[m > 0])
    if nz.size == 0:
        return 0
    amax = Fraction(max(float(nz[-1]), 1e-30))
    # k1: nearest integer to log2(T/amax): the k with 2^(2k-1) < (T/amax)^2 < 2^(2k+1)
    r2 = (Fraction(T) / amax) ** 2
    k1 = math.floor(math.log2(float(Fraction(T) / amax)))
    while not (Fraction(2) ** (2 * k1 - 1) < r2):
        k1 -= 1
    while not (r2 < Fraction(2) ** (2 * k1 + 1)):
        k1 += 1
    pos = ((nz.size - 1) * tau) / 100.0
    i = int(math.floor(pos))
    f = pos - i
    hi = nz[min(i + 1, nz.size - 1)]
    p = nz[i] + f * (hi - nz[i])
    P = Fraction(max(p, 1e-30))
    k2 = math.ceil(math.log2(float(Fraction(tmin) / P)))
    while Fraction(2) ** k2 * P < Fraction(tmin):
        k2 += 1
    while Fraction(2) ** (k2 - 1) * P >= Fraction(tmin):
        k2 -= 1
    k = max(k1, k2)
    if kmin is not None:
        k = max(k, kmin)
    if kmax is not None:
        k = min(k, kmax)
    return k


@pytest.mark.parametrize("seed", range(12))
def test_random_slices_vs_rationals(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 3000))
    x = (rng.normal(size=n) + 1j * rng.normal(size=n)) * np.exp(rng.normal(0, 6, size=n))
    x[rng.random(n) < 0.1] = 0
    x = x.astype(np.complex64)
    T = float(2.0 ** rng.integers(-8, 12)) * float(rng.choice([1.0, 0.7, 1.3]))
    tau = float(rng.choice([0.0, 5.0, 12.5, 50.0, 100.0]))
    tmin = float(2.0 ** rng.integers(-20, 4)) * float(rng.choice([1.0, 0.9]))
    st, k = O.prescale(x, target=T, tau=tau, tau_min=tmin)
    assert st == O.OK
    assert k == exact_k(x, T, tau, tmin)


def test_numpy_percentile_agrees_away_from_ties():
    rng = np.random.default_rng(11)
    x = (rng.normal(size=4096) + 1j * rng.normal(size=4096)).astype(np.complex64) * np.float32(37.0)
    m = np.abs(x.astype(np.complex128))
    p = np.percentile(m[m > 0], 5.0)
    k2_np = math.ceil(math.log2(2.0 ** -6 / p))
    k1_np = round(math.log2(2.0 ** 7 / m.max()))
    assert O.prescale(x)[1] == max(k1_np, k2_np)


def test_clip_and_errors():
    x = one([3.0, 1e-3])
    assert O.prescale(x, k_min=10)[1] == 10
    assert O.prescale(x, k_max=-2)[1] == -2
    st, k = O.prescale(one([1.0, np.inf]))
    assert st == O.ENONFINITE and k == O.INT32_MIN
    st, k = O.prescale(one([np.nan, 1.0]))
    assert st == O.ENONFINITE
    # component 2^100 shifted by k >= 28 overflows FP32
    st, k = O.prescale(one([2.0 ** 100]), k_min=28)
    assert st == O.ERANGE and k == O.INT32_MIN
    st, k = O.prescale(one([2.0 ** 100]), k_min=27)
    assert st == O.OK and k == 27
