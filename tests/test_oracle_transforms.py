"""Pins of the oracle's 1D and 2D transforms.

FP64 mode against the O(N^2) DFT (pins bit reversal, stage indexing, twiddle
sign); FP32 mode against numpy's FFT; MX mode against closed forms that are
exact under quantisation (impulse, constant), hand-traced 4-point cases, the
structural identity MX(e6m23) == FP32, scale equivariance, conjugate symmetry
and batch independence.
"""
import numpy as np
import pytest

import oracle as O
from paper_2512_04317_amd import synth


def dft_matrix(N, inverse=False):
    n = np.arange(N)
    sgn = 1 if inverse else -1
    return np.exp(sgn * 2j * np.pi * np.outer(n, n) / N)


def nrmse(y, r):
    return np.linalg.norm((y - r).ravel()) / np.linalg.norm(r.ravel())


@pytest.mark.parametrize("N", [2, 4, 8, 16, 32, 64])
def test_fp64_line_vs_dft(N):
    x = synth.random_complex((3, N), seed=N).astype(np.complex128)
    for inv in (False, True):
        got = O.fft1_f64(x, inverse=inv)
        ref = x @ dft_matrix(N, inv).T
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("N", [2, 4, 16, 32])
def test_fp64_2d_vs_separable_dft(N):
    x = synth.random_complex((2, N, N), seed=100 + N).astype(np.complex128)
    F = dft_matrix(N)
    ref = np.einsum("ij,bjk,lk->bil", F, x, F)
    got = O.fft2_f64(x)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    np.testing.assert_allclose(got, np.fft.fft2(x), rtol=0, atol=1e-10 * np.abs(ref).max())


@pytest.mark.parametrize("N", [4, 64, 256])
def test_fp32_plain_vs_numpy(N):
    x = synth.random_complex((2, N, N), seed=200 + N)
    st, y, k = O.transform(x, mode=O.MODE_FP32, flags=O.NO_PRESCALE)
    ref = np.fft.fft2(x.astype(np.complex128))
    assert st == O.OK and nrmse(y, ref) < 1e-6
    # Parseval: sum |Y|^2 = N^2 sum |x|^2
    e_y = np.sum(np.abs(y.astype(np.complex128)) ** 2)
    e_x = N * N * np.sum(np.abs(x.astype(np.complex128)) ** 2)
    assert abs(e_y / e_x - 1) < 1e-5
    st, rt, _ = O.transform(x, op=O.ROUNDTRIP, mode=O.MODE_FP32)
    assert nrmse(rt, x) < 1e-6


@pytest.mark.parametrize("f", [O.E4M3, O.E5M2])
@pytest.mark.parametrize("N,B", [(4, 2), (16, 4), (64, 32), (128, 64)])
def test_mx_impulse_gives_ones(f, N, B):
    # every v block of every stage is zero, so each butterfly copies u: exact
    x = np.zeros((N, N), np.complex64)
    x[0, 0] = 1
    st, y, k = O.transform(x, fmt=f, B=B)
    assert st == O.OK and k[0] == 7
    np.testing.assert_array_equal(y, np.ones((N, N), np.complex64))


@pytest.mark.parametrize("f", [O.E4M3, O.E5M2])
@pytest.mark.parametrize("N,B", [(4, 4), (32, 8), (64, 32)])
def test_mx_constant_gives_scaled_impulse(f, N, B):
    # values stay powers of two; twiddles met by nonzero v are 1 only
    x = np.ones((N, N), np.complex64)
    st, y, k = O.transform(x, fmt=f, B=B)
    ref = np.zeros((N, N), np.complex64)
    ref[0, 0] = N * N
    np.testing.assert_array_equal(y, ref)


def test_mx_four_point_hand_traced():
    # Row pass of x = [0, 0, 3.9, 4], E4M3, no prescale.
    # B = 4 (2 complex per block): input blocks {0,0} and {3.9, 4}: amax 4 ->
    #   E = 2-8 = -6; 3.9*64 = 249.6 -> 256 (grid 16) -> 4.0.  x' = [0,0,4,4].
    #   bit reversal [0,4,0,4]; stage 1 (w = 1): [4,-4,4,-4]; stage 2 block
    #   v = [4, -4], w = [1, -i]: exact -> X = [8, -4+4i, 0, -4-4i].
    # B = 2 (one complex per block): 3.9 alone: E = 1-8 = -7; 3.9*128 = 499.2
    #   -> 512 -> saturates to 448 -> 3.5.  x' = [0,0,3.5,4]; stage 1 ->
    #   [3.5,-3.5,4,-4]; stage 2 -> X = [7.5, -3.5+4i, -0.5, -3.5-4i].
    x = np.array([[0, 0, 3.9, 4]], np.complex64)
    y4 = O.pass_lines(x, fmt=O.E4M3, B=4)
    np.testing.assert_array_equal(y4[0], np.array([8, -4 + 4j, 0, -4 - 4j], np.complex64))
    y2 = O.pass_lines(x, fmt=O.E4M3, B=2)
    np.testing.assert_array_equal(y2[0], np.array([7.5, -3.5 + 4j, -0.5, -3.5 - 4j], np.complex64))
    # x = [1, 1, 1, 1.1], B = 4: input {1,1} exact; {1, 1.1}: E = -8, 281.6 -> 288
    #   -> 1.125.  Stage 1: [2, 0, 2.125, -0.125].  Stage 2 block v = [2.125,
    #   -0.125]: E = -7, 272 is a tie between 256 and 288 -> 256 -> 2.0;
    #   -16 exact.  X = [2+2, 0 + 0.125i, 2-2, 0 - 0.125i].
    y = O.pass_lines(np.array([[1, 1, 1, 1.1]], np.complex64), fmt=O.E4M3, B=4)
    np.testing.assert_array_equal(y[0], np.array([4, 0.125j, 0, -0.125j], np.complex64))
    # Two points, B = 2: a = 1 + 0.3i -> E = -8: 76.8 -> 80 (grid 8) -> 0.3125;
    # b = 0.1 - 2i -> E = -7: 12.8 -> 13 -> 0.1015625.  X = [a'+b', a'-b'].
    y = O.pass_lines(np.array([[1 + 0.3j, 0.1 - 2j]], np.complex64), fmt=O.E4M3, B=2)
    np.testing.assert_array_equal(y[0], np.array([1.1015625 - 1.6875j, 0.8984375 + 2.3125j], np.complex64))


def test_mx_trace_kr_and_exponents():
    # the butterfly trace of a row: stage 1 (w = 1) always renormalises by
    # exactly emax for nonzero v blocks, and Eout = Ew + Ev + kr
    x = synth.random_complex((1, 64), seed=7)
    _, tr = O.pass_lines(x, fmt=O.E4M3, B=16, trace=True)
    assert np.all(tr[0, :, 1] == 8)
    assert np.all(tr[0, :, 2] == -8 + tr[0, :, 0] + 8)


@pytest.mark.parametrize("N,B", [(16, 4), (64, 32), (128, 8)])
def test_mx_wide_element_equals_fp32(N, B):
    """MX with a 23-bit-mantissa element (e6m23) reproduces the FP32 plain
    form bit for bit: a power-of-two scale commutes with rounding, so every
    MX encode is the identity and the mantissa-space product equals the FP32
    product.  Pins the MX data flow (operand order, exponent bookkeeping)."""
    x = synth.random_complex((2, N, N), seed=300 + N)
    st, ymx, _ = O.transform(x, fmt=O.E6M23, B=B)
    st2, y32, _ = O.transform(x, mode=O.MODE_FP32)
    np.testing.assert_array_equal(ymx, y32)
    st, ymx, _ = O.transform(x, op=O.INVERSE, fmt=O.E6M23, B=B)
    st2, y32, _ = O.transform(x, op=O.INVERSE, mode=O.MODE_FP32)
    np.testing.assert_array_equal(ymx, y32)


@pytest.mark.parametrize("f", [O.E4M3, O.E5M2])
def test_mx_scale_equivariance(f):
    x = synth.random_complex((2, 32, 32), seed=400)
    _, y, _ = O.transform(x, fmt=f, B=16, flags=O.NO_PRESCALE)
    for j in (-9, 5, 31):
        xs = np.ldexp(x.real, j) + 1j * np.ldexp(x.imag, j)
        _, ys, _ = O.transform(xs.astype(np.complex64), fmt=f, B=16, flags=O.NO_PRESCALE)
        np.testing.assert_array_equal(ys, (np.ldexp(y.real, j) + 1j * np.ldexp(y.imag, j)).astype(np.complex64))
    # hence prescale on or off gives the same de-scaled output
    _, yp, k = O.transform(x, fmt=f, B=16)
    assert k[0] != 0
    np.testing.assert_array_equal(yp, y)


@pytest.mark.parametrize("f", [O.E4M3, O.E5M2])
def test_mx_conjugate_symmetry(f):
    x = synth.kspace_batch(32, 1, 1, 1)
    _, yi, ki = O.transform(x, op=O.INVERSE, fmt=f, B=8)
    _, yf, kf = O.transform(np.conj(x), fmt=f, B=8)
    np.testing.assert_array_equal(yi, np.conj(yf))
    assert ki[0] == kf[0]


def test_batch_independence_and_determinism():
    x = synth.kspace_batch(32, 2, 2, 3)
    _, yb, kb = O.transform(x, fmt=O.E5M2, B=8, nthreads=3)
    for s in range(x.shape[0]):
        _, ys, ks = O.transform(x[s], fmt=O.E5M2, B=8)
        np.testing.assert_array_equal(yb[s], ys)
        assert kb[s] == ks[0]
    _, yb2, _ = O.transform(x, fmt=O.E5M2, B=8, nthreads=1)
    np.testing.assert_array_equal(yb, yb2)


def test_roundtrip_uses_one_prescale():
    # round trip = forward keeping 2^k, inverse with the same k, then 2^(-k-2L)
    x = synth.kspace_batch(32, 1, 1, 2)
    _, rt, k = O.transform(x, op=O.ROUNDTRIP, fmt=O.E4M3, B=32)
    _, mid, k1 = O.transform(x, fmt=O.E4M3, B=32, flags=O.KEEP_SCALE)
    _, back, _ = O.transform(mid, op=O.INVERSE, fmt=O.E4M3, B=32, kp=k1, flags=O.NORMALIZE)
    np.testing.assert_array_equal(rt, back)
    np.testing.assert_array_equal(k, k1)


def test_fp16_bf16_controls_are_accurate():
    x = synth.kspace_batch(64, 1, 1, 1)
    ref = np.fft.fft2(x.astype(np.complex128))
    _, y16, _ = O.transform(x, mode=O.MODE_FP16)
    _, yb16, _ = O.transform(x, mode=O.MODE_BF16)
    assert nrmse(y16, ref) < 5e-3 and nrmse(yb16, ref) < 3e-2


def test_fp16_overflow_follows_ieee():
    """Infinities from the half form's overflow propagate as IEEE FP32 sums
    do: -inf + finite = -inf, never NaN.  Hand-worked 2 x 2 case (forward, no
    prescale): row 0 sums to -120000, which rounds to -inf in half; the column
    butterfly then adds and subtracts the finite 2 of row 1."""
    x = np.array([[[-60000.0, -60000.0], [1.0, 1.0]]], np.complex64)
    st, y, _ = O.transform(x, mode=O.MODE_FP16, flags=O.NO_PRESCALE)
    assert st == O.OK
    assert y[0, 0, 0].real == -np.inf and y[0, 1, 0].real == -np.inf
    assert not np.isnan(y).any()
    assert y[0, 0, 1].real == 0.0 and y[0, 1, 1].real == 0.0


def test_errors():
    x = np.zeros((8, 8), np.complex64)
    assert O.transform(x, B=16)[0] == O.EINVAL            # B > N
    assert O.transform(x, B=6)[0] == O.EINVAL             # not a power of two
    x[1, 1] = np.nan
    st, y, k = O.transform(x, B=4)
    assert st == O.ENONFINITE and k[0] == O.INT32_MIN


def test_paper_orderings_on_phantom():
    """Orderings the paper reports (Sec. 3, Sec. 4): E4M3 beats E5M2; the round
    trip is worse than the forward transform; small blocks (B = 2) are worse
    than B = 32.  Measured on the synthetic phantom against FP64."""
    x = synth.kspace_batch(64, 1, 4, 1)
    ref = np.fft.fft2(x.astype(np.complex128))
    e = {}
    for name, f in (("e4m3", O.E4M3), ("e5m2", O.E5M2)):
        for B in (2, 32):
            _, y, _ = O.transform(x, fmt=f, B=B)
            e[name, B] = nrmse(y, ref)
        _, rt, _ = O.transform(x, op=O.ROUNDTRIP, fmt=f, B=32)
        e[name, "rt"] = nrmse(rt, x)
    print({k: round(v, 4) for k, v in e.items()})
    assert e["e4m3", 32] < e["e5m2", 32]
    assert e["e4m3", 32] < e["e4m3", "rt"]
    assert e["e4m3", 32] <= e["e4m3", 2] and e["e5m2", 32] <= e["e5m2", 2]
