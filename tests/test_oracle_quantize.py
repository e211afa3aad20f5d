"""The oracle's quantised output (flag QUANTIZE_OUT, MX formats): the final
de-scaled output MX-encoded in blocks of B/2 consecutive rows of one column
(Alg. 2's EncodeBlockMX; Sec. 2.2 states quantised outputs for the 16-bit
control).  Pinned here against the element sets built from the OCP format
definitions (E4M3: bias 7, 3 mantissa bits, no infinities, 448 the largest;
E5M2: bias 15, 2 mantissa bits, 57344 the largest), the OCP shared exponent
E = floor(log2 amax) - emax_elem computed with numpy, nearest-element
rounding with saturation, idempotence and exactly representable outputs."""
import numpy as np
import pytest

import oracle as O
from paper_2512_04317_amd import synth


def element_grid(fmt):
    """Every finite element value of the format (both signs), sorted, and emax."""
    if fmt == O.E4M3:
        bias, top = 7, 15
        vals = [(1 + m / 8) * 2.0 ** (e - bias) for e in range(1, top + 1) for m in range(8) if not (e == 15 and m == 7)]
        vals += [(m / 8) * 2.0 ** (1 - bias) for m in range(8)]
        emax = 8
    else:
        bias, top = 15, 30
        vals = [(1 + m / 4) * 2.0 ** (e - bias) for e in range(1, top + 1) for m in range(4)]
        vals += [(m / 4) * 2.0 ** (1 - bias) for m in range(4)]
        emax = 15
    g = np.array(sorted(set(vals) | {-v for v in vals}))
    return g, emax


def expected_quantised(y, fmt, B):
    """Column blocks of B/2 rows: E from the block maximum, each component the
    nearest element of y / 2^E (either neighbour on an exact tie), times 2^E
    rounded once to FP32.  Returns (lo, hi) candidates per component."""
    grid, emax = element_grid(fmt)
    cb = B // 2
    yb = y.astype(np.complex128)
    S, N, _ = y.shape
    blocks = yb.reshape(S, N // cb, cb, N)                     # [slice][row block][row][column]
    amax = np.maximum(np.abs(blocks.real), np.abs(blocks.imag)).max(axis=2, keepdims=True)
    with np.errstate(divide="ignore"):
        _, e2 = np.frexp(amax)                                  # amax = f 2^e2, f in [1/2, 1)
    E = np.where(amax > 0, np.clip(e2 - 1 - emax, -127, 127), 0)
    out = []
    for part in (blocks.real, blocks.imag):
        t = np.ldexp(part, -E)                                  # exact: power-of-two scaling in FP64
        hi_i = np.clip(np.searchsorted(grid, t), 0, len(grid) - 1)
        lo_i = np.clip(hi_i - 1, 0, len(grid) - 1)
        dlo, dhi = np.abs(grid[lo_i] - t), np.abs(grid[hi_i] - t)
        best_lo = np.where(dlo <= dhi, grid[lo_i], grid[hi_i])
        best_hi = np.where(dhi <= dlo, grid[hi_i], grid[lo_i])
        out.append((np.ldexp(best_lo, E).astype(np.float32).reshape(S, N, N),
                    np.ldexp(best_hi, E).astype(np.float32).reshape(S, N, N)))
    return out


@pytest.mark.parametrize("op", [O.FORWARD, O.INVERSE, O.ROUNDTRIP])
@pytest.mark.parametrize("fmt", [O.E4M3, O.E5M2])
@pytest.mark.parametrize("B", [2, 4, 16, 32])
def test_quantised_output_is_the_column_block_encode(fmt, B, op):
    x = synth.kspace_batch(max(16, B), 3, 1, 2)               # B <= N
    st, y, k = O.transform(x, op=op, fmt=fmt, B=B, nthreads=4)
    stq, yq, kq = O.transform(x, op=op, fmt=fmt, B=B, flags=O.QUANTIZE_OUT, nthreads=4)
    assert st == stq == O.OK
    np.testing.assert_array_equal(k, kq)
    (re_lo, re_hi), (im_lo, im_hi) = expected_quantised(y, fmt, B)
    ok_re = (yq.real == re_lo) | (yq.real == re_hi)
    ok_im = (yq.imag == im_lo) | (yq.imag == im_hi)
    assert ok_re.all() and ok_im.all(), "%d components off the column-block grid" % ((~ok_re).sum() + (~ok_im).sum())
    assert not np.array_equal(yq, y)                            # it does quantise
    # the row-block reading (blocks along the contiguous axis) differs
    (rr_lo, _), _ = expected_quantised(np.swapaxes(y, 1, 2).copy(), fmt, B)
    rows = np.swapaxes(rr_lo, 1, 2)
    assert not np.array_equal(yq.real, rows) or B == 2


def test_quantised_output_is_idempotent_and_keeps_exact_outputs():
    x = synth.kspace_batch(32, 4, 1, 1)
    _, yq, _ = O.transform(x, fmt=O.E4M3, B=8, flags=O.QUANTIZE_OUT)
    (lo, hi), (ilo, ihi) = expected_quantised(yq[None] if yq.ndim == 2 else yq, O.E4M3, 8)
    yq3 = yq.reshape(lo.shape)
    assert ((yq3.real == lo) | (yq3.real == hi)).all() and ((yq3.imag == ilo) | (yq3.imag == ihi)).all()
    assert (lo == hi).all() and (lo == yq3.real).all()          # already on the grid: unchanged
    imp = np.zeros((1, 16, 16), np.complex64)
    imp[0, 0, 0] = 1.0
    st, y1, _ = O.transform(imp, fmt=O.E4M3, B=16, flags=O.QUANTIZE_OUT)
    assert st == O.OK and (y1 == 1.0).all()                     # impulse -> ones, exactly representable


def test_quantised_output_flag_leaves_other_forms():
    x = synth.kspace_batch(16, 3, 1, 1)
    for mode in (O.MODE_FP16, O.MODE_BF16, O.MODE_FP32):
        st, y, _ = O.transform(x, mode=mode)
        stq, yq, _ = O.transform(x, mode=mode, flags=O.QUANTIZE_OUT)
        assert st == stq == O.OK
        assert np.array_equal(y.view(np.uint32), yq.view(np.uint32))
