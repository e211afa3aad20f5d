"""Hand-worked pins of two oracle readings that no closed form or invariant
fixes: the butterfly-block geometry of Alg. 2 for stages with fewer
butterflies per group than per block, and the per-operation rounding of the
16-bit positive control (Sec. 2.2).  Every expected value below is derived by
hand in the comments (exact binary fractions); the alternative readings'
values are derived too and must differ, so a plausible slip in either oracle
function fails here.  CPU only."""
import numpy as np

import oracle as O


def _line(vals):
    return np.array([vals], np.complex64)


def test_mx_block_geometry_t_ordered_blocks_across_groups():
    # E4M3, N = 8, B = 4 (two complex per block), one 1D pass, no prescale.
    # x = [0, 0, 0, 0, 256, 0, c, 0] with c = 9 * 2^-10 = 1.125 * 2^-7.
    # Input encode, blocks {x4, x5}: amax 256 -> E = 8 - 8 = 0, 256 exact;
    #   {x6, x7}: amax c -> E = -7 - 8 = -15, c * 2^15 = 288 = 1.125 * 2^8
    #   exact.  The input is unchanged.
    # Bit reversal: a = [x0, x4, x2, x6, x1, x5, x3, x7] = [0, 256, 0, c, 0..].
    # Stage 1 (h = 1, every twiddle 1; twiddle block (1, 0, 1, 0): Ew = -8,
    #   element 256).  Butterflies t = 0, 1 (groups 0 and 1) form ONE block:
    #   v = (256, c): amax 256 -> Ev = 0; c * 2^0 is on the E4M3 subnormal grid
    #   2^-9: c / 2^-9 = 4.5 -> 4 (ties to even) -> y = 2^-7.
    #   Products 256 * 256 = 65536, 256 * 2^-7 = 2; a = 65536 > 448:
    #   kr = 8 (448 * 2^7 < 65536 <= 448 * 2^8), Eout = -8 + 0 + 8 = 0;
    #   Q(65536 / 2^8) = 256, Q(2 / 2^8) = 2^-7 (subnormal, exact).
    #   a = [256, -256, 2^-7, -2^-7, 0, 0, 0, 0].
    # Stage 2 (h = 2 = B/2): block v = (2^-7, -2^-7), w = (1, -i): Ev = -15,
    #   y = (256, -256); products (65536, 0) and (+0, 65536): kr = 8, Eout =
    #   -15, w v = (2^-7, 0), (0, 2^-7).  a = [256 + 2^-7, -256 + 2^-7 i,
    #   256 - 2^-7, -256 - 2^-7 i, 0, 0, 0, 0] (each sum exact in FP32).
    # Stage 3: every v is zero, so y0 = y1 = u.
    # X = [256 + d, -256 + d i, 256 - d, -256 - d i] twice, d = 2^-7.
    # Per-group blocks (min(B/2, h) = 1 butterfly at stage 1) would encode c
    # alone (Ev = -15, exact) and give d = c = 9 * 2^-10, the exact DFT.
    c = 9.0 * 2.0 ** -10
    x = _line([0, 0, 0, 0, 256, 0, c, 0])
    y = O.pass_lines(x, fmt=O.E4M3, B=4)[0]
    d = 2.0 ** -7
    want = np.array([256 + d, -256 + d * 1j, 256 - d, -256 - d * 1j] * 2, np.complex64)
    np.testing.assert_array_equal(y, want)
    per_group = np.array([256 + c, -256 + c * 1j, 256 - c, -256 - c * 1j] * 2, np.complex64)
    assert not np.array_equal(y, per_group)
    # the exponent trace of stage 1, block 0: Ev = 0 (the block maximum is
    # 256, not c), kr = 8, Eout = 0
    _, tr = O.pass_lines(x, fmt=O.E4M3, B=4, trace=True)
    assert tuple(tr[0, 0]) == (0, 8, 0)


def test_fp16_per_operation_rounding_hand_worked():
    # FP16, N = 8, one 1D pass per line.  Only x1 and x5 are nonzero, exact
    # halves.  Bit reversal puts them at a4, a5; stage 1 (w = 1) gives
    # a4 = x1 + x5, a5 = x1 - x5 (FP32, exact here); stage 2 meets v = 0 and
    # copies them to a6, a7.  Stage 3 has u = 0, so X[j] = p_j, X[j + 4] = -p_j
    # with p_j the product of w_j and v = a4 (j = 0, 2) or a5 (j = 1, 3).
    # w_1 = fl16(sqrt(1/2)) (1 - i) = 181/256 (1 - i), w_3 = -181/256 (1 + i).
    #
    # Line A: x1 = 129.625 + 0.625i, x5 = 128: a4 = 257.625 + 0.625i,
    # a5 = 1.625 + 0.625i.
    #  j = 0 (w = 1): p = fl16(257.625) = 257.5 (a tie between 257.5 and
    #   257.75 -> even) + 0.625i.
    #  j = 1: wr vr = 181/256 * 13/8 = 2353/2048 = 1176.5 * 2^-10 -> tie ->
    #   1.1484375; wi vi = -905/2048 = -0.44189453125 (exact half).
    #   pr = fl16(1.1484375 + 0.44189453125 = 1628.5 * 2^-10) -> tie ->
    #   1.58984375.  pi = fl16(0.44189453125 - 1.1484375) = -0.70654296875
    #   (exact).  ONE rounding of the exact sums would give 181/256 * 18/8 =
    #   1.5908203125 and 181/256 * (-1) = -0.70703125.
    #  j = 2 (w = -i): 0.625 - 257.5i.  j = 3: pr = fl16(-1.1484375 +
    #   0.44189453125) = -0.70654296875, pi = fl16(-0.44189453125 - 1.1484375)
    #   = -1.58984375.
    x = _line([0, 129.625 + 0.625j, 0, 0, 0, 128, 0, 0])
    y = O.pass_lines(x, mode=O.MODE_FP16, fmt=O.FP16)[0]
    p = [257.5 + 0.625j, 1.58984375 - 0.70654296875j, 0.625 - 257.5j, -0.70654296875 - 1.58984375j]
    np.testing.assert_array_equal(y, np.array(p + [-v for v in p], np.complex64))
    assert y[1] != np.complex64(1.5908203125 - 0.70703125j)     # single rounding
    # Line B: x5 = -128 instead: a4 = 1.625 + 0.625i, a5 = 257.625 + 0.625i,
    # so the twiddle w_1 meets a v that is not a half.
    #  v rounded first: v = 257.5 + 0.625i.  wr vr = 181 * 257.5 / 256 =
    #   182.060546875 -> fl16 (spacing 1/8 on [128, 256)) 182; wi vi =
    #   -0.44189453125.  pr = fl16(182.44189453125) = 182.5 (1459.54 / 8 ->
    #   1460 / 8); pi = fl16(0.44189453125 - 182) = fl16(-181.55810546875) =
    #   -181.5.  Unrounded v (257.625) would give wr vr = 182.1489... -> 182.125
    #   and X[1] = 182.625 - 181.625i.
    #  j = 0: 1.625 + 0.625i.  j = 2: 0.625 - 1.625i.  j = 3: pr =
    #   fl16(-182 + 0.44189453125) = -181.5, pi = fl16(-0.44189453125 - 182)
    #   = -182.5.
    x = _line([0, 129.625 + 0.625j, 0, 0, 0, -128, 0, 0])
    y = O.pass_lines(x, mode=O.MODE_FP16, fmt=O.FP16)[0]
    p = [1.625 + 0.625j, 182.5 - 181.5j, 0.625 - 1.625j, -181.5 - 182.5j]
    np.testing.assert_array_equal(y, np.array(p + [-v for v in p], np.complex64))
    assert y[1] != np.complex64(182.625 - 181.625j)             # v not rounded


def test_bf16_per_operation_rounding_hand_worked():
    # BF16 (8 significant bits), the same 8-point probe as the FP16 test:
    # w_1 = fl_bf16(sqrt(1/2)) (1 - i) = 181/256 (1 - i).
    # Line A: x1 = 1.75 + 16.625i, x5 = 16i: a4 = 1.75 + 32.625i,
    # a5 = 1.75 + 0.625i.
    #  j = 0 (w = 1): 32.625 lies between 32.5 and 32.75 (spacing 0.25), a
    #   tie -> 32.5.  X[0] = 1.75 + 32.5i.
    #  j = 1, v = 7/4 + 5/8 i: wr vr = 1267/1024 = 158.375/128 -> 1.234375;
    #   wi vi = -905/2048 = -226.25/512 -> -0.44140625.  pr = fl(1.67578125 =
    #   214.5/128) -> tie -> 1.671875; pi = fl(0.44140625 - 1.234375) =
    #   -0.79296875 (exact).  One rounding of the exact sums: 181/256 * 19/8
    #   = 1.67919921875 -> 1.6796875 and 181/256 * (-9/8) -> -0.796875.
    #  j = 2: 32.5 - 1.75i.  j = 3: pr = fl(-1.234375 + 0.44140625) =
    #   -0.79296875, pi = fl(-0.44140625 - 1.234375) -> -1.671875.
    x = _line([0, 1.75 + 16.625j, 0, 0, 0, 16j, 0, 0])
    y = O.pass_lines(x, mode=O.MODE_BF16, fmt=O.BF16)[0]
    p = [1.75 + 32.5j, 1.671875 - 0.79296875j, 32.5 - 1.75j, -0.79296875 - 1.671875j]
    np.testing.assert_array_equal(y, np.array(p + [-v for v in p], np.complex64))
    assert y[1] != np.complex64(1.6796875 - 0.796875j)          # single rounding
    # Line B: x5 = -16i: a4 = 1.75 + 0.625i, a5 = 1.75 + 32.625i -> v rounded
    # to 1.75 + 32.5i before the product with w_1:
    #  wr vr -> 1.234375; wi vi = -181 * 32.5 / 256 = -22.978515625 -> -23
    #   (spacing 1/8 on [16, 32)); pr = fl(24.234375) = 24.25; wr vi -> 23,
    #   pi = fl(23 - 1.234375 = 21.765625) = 21.75.  Unrounded v would give
    #   wi vi = -23.06689453125 -> -23.125 and pr = fl(24.359375) = 24.375.
    #  j = 0: 1.75 + 0.625i; j = 2: 0.625 - 1.75i; j = 3: pr = fl(-1.234375 +
    #   23) = 21.75, pi = fl(-23 - 1.234375) = -24.25.
    x = _line([0, 1.75 + 16.625j, 0, 0, 0, -16j, 0, 0])
    y = O.pass_lines(x, mode=O.MODE_BF16, fmt=O.BF16)[0]
    p = [1.75 + 0.625j, 24.25 + 21.75j, 0.625 - 1.75j, 21.75 - 24.25j]
    np.testing.assert_array_equal(y, np.array(p + [-v for v in p], np.complex64))
    assert y[1].real != np.float32(24.375)                      # v not rounded


def test_16bit_twiddles_rounded_once_from_fp64():
    # The 16-bit twiddles are FP64 values rounded once to the format.  For
    # every n <= 4096 rounding through FP32 first gives the same values (no
    # twiddle part falls on a midpoint of either format after rounding to
    # FP32), so the two readings cannot differ on any supported size; this
    # checks that over all stages, with the quantiser against numpy's own
    # float16 cast and a bfloat16 cast by truncation with round-half-even.
    import torch
    for L in range(1, 13):
        m = 1 << L
        js = np.arange(m // 2)
        tw = [O.twiddle64(int(j), m) for j in js]
        w = np.array([[t.real, t.imag] for t in tw], np.float64).reshape(-1)
        q16 = O.quantize(O.FP16, w)
        np.testing.assert_array_equal(q16, w.astype(np.float16).astype(np.float64))
        np.testing.assert_array_equal(q16, w.astype(np.float32).astype(np.float16).astype(np.float64))
        qb = O.quantize(O.BF16, w)
        tb = torch.from_numpy(w.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
        np.testing.assert_array_equal(qb, tb)
    # the value both 16-bit formats give sqrt(1/2): 181/256
    assert O.quantize(O.FP16, np.array([np.sqrt(0.5)]))[0] == 181 / 256
    assert O.quantize(O.BF16, np.array([np.sqrt(0.5)]))[0] == 181 / 256
