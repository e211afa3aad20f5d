"""Pins of the oracle's root-sum-of-squares coil combine (Eq. 1) and of its
mean SSIM (the image metric the paper reports, in the form of Wang et al.
2004), against hand-worked values, closed forms, invariants and an
independent evaluation with a library correlation."""
import numpy as np
import pytest

import oracle as O

scipy_signal = pytest.importorskip("scipy.signal")


def test_rss_hand_values():
    """Sec. 2.3, Eq. 1: x_RSS = (sum_c |T_c|^2)^(1/2)."""
    one = lambda vals: np.array([[[v]] for v in vals], np.complex64)   # noqa: E731  coils x 1 x 1
    assert O.rss(one([3 + 4j]), 1)[0, 0, 0] == 5.0
    assert O.rss(one([5 - 12j]), 1)[0, 0, 0] == 13.0
    assert O.rss(one([1, 1j, -1, -1j]), 4)[0, 0, 0] == 2.0       # every coil counts
    assert O.rss(one([3, 4j]), 2)[0, 0, 0] == 5.0                 # parts of different coils
    assert O.rss(one([0, 0, 0]), 3)[0, 0, 0] == 0.0
    assert np.isnan(O.rss(one([1, complex(np.nan, 0)]), 2)[0, 0, 0])
    # two reconstructions of two coils: coil-minor layout
    T = np.array([[[3]], [[4]], [[6j]], [[8]]], np.complex64)
    np.testing.assert_array_equal(O.rss(T, 2)[:, 0, 0], [5.0, 10.0])


def test_rss_error_bound_and_scaling():
    """Within the FP32 rounding bound of the exact value, and exactly
    equivariant under power-of-two scaling (every FP32 step is)."""
    rng = np.random.default_rng(11)
    C, n = 7, 16
    T = ((rng.standard_normal((3 * C, n, n)) + 1j * rng.standard_normal((3 * C, n, n))) * 10.0).astype(np.complex64)
    r = O.rss(T, C).astype(np.float64)
    exact = np.sqrt((np.abs(T.astype(np.complex128)) ** 2).reshape(3, C, n, n).sum(axis=1))
    assert np.all(np.abs(r - exact) <= (C + 3) * 2.0 ** -24 * exact)
    for k in (-20, 7):
        np.testing.assert_array_equal(O.rss(T * np.float32(2.0 ** k), C), O.rss(T, C) * np.float32(2.0 ** k))


def gaussian_window():
    i = np.arange(11) - 5
    w = np.exp(-(i[:, None] ** 2 + i[None, :] ** 2) / (2 * 1.5 ** 2))
    return w / w.sum()


def ssim_by_correlation(x, y, L):
    """Independent evaluation of the same definition: local statistics by a
    library 2-D correlation ('valid' region) of the window with each field."""
    x = x.astype(np.float64)
    y = y.astype(np.float64)
    w = gaussian_window()
    f = lambda a: scipy_signal.correlate2d(a, w, mode="valid")   # noqa: E731
    mx, my = f(x), f(y)
    sx, sy, sxy = f(x * x) - mx ** 2, f(y * y) - my ** 2, f(x * y) - mx * my
    C1, C2 = (0.01 * L) ** 2, (0.03 * L) ** 2
    return float((((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx ** 2 + my ** 2 + C1) * (sx + sy + C2))).mean())


def test_ssim_identity_and_closed_form():
    rng = np.random.default_rng(3)
    x = rng.random((40, 40)).astype(np.float32) * 5
    assert O.ssim(x, x) == 1.0
    # constant images a, b: the variance terms vanish,
    # SSIM = (2ab + C1) / (a^2 + b^2 + C1)
    a, b, L = 0.25, 0.75, 1.0
    C1 = (0.01 * L) ** 2
    s = O.ssim(np.full((24, 24), a, np.float32), np.full((24, 24), b, np.float32), L=L)
    assert s == pytest.approx((2 * a * b + C1) / (a * a + b * b + C1), abs=1e-12)


def test_ssim_matches_library_correlation():
    rng = np.random.default_rng(5)
    y = np.abs(rng.standard_normal((48, 48))).astype(np.float32)
    x = (y + 0.1 * rng.standard_normal((48, 48))).astype(np.float32)
    L = float(y.max())
    assert O.ssim(x, y) == pytest.approx(ssim_by_correlation(x, y, L), abs=1e-12)
    # symmetric in its arguments for a fixed range, and below 1 for a noisy copy
    assert O.ssim(y, x, L=L) == pytest.approx(O.ssim(x, y, L=L), abs=1e-12)
    assert O.ssim(x, y) < 0.99
    # only windows that contain a changed pixel change: a border pixel outside
    # every window centre's reach but the corner one
    z = y.copy()
    z[0, 0] += 3.0
    n_windows = (48 - 10) ** 2
    assert 0 < (O.ssim(y, y) - O.ssim(z, y)) * n_windows < 1.0
