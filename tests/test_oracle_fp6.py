"""Pins of the oracle's OCP 6-bit MX elements (MXFP6 E2M3 and E3M2, which the
paper evaluates beside MXFP8 in Sec. 3): every code's value from the format
definition, round-to-nearest-even at midpoints, saturation, the MX block
exponent, and an end-to-end FFT against FP64."""
import numpy as np
import pytest

import oracle as O
from paper_2512_04317_amd import synth

# positive values of each format, written out from the OCP definitions:
# E2M3 (bias 1): subnormals k/8, then 1 + m/8 for exponents 0, 1, 2
E2M3_POS = [k / 8 for k in range(8)] + [(8 + m) / 8 * 2.0 ** e for e in (0, 1, 2) for m in range(8)]
# E3M2 (bias 3): subnormals k/16, then 1 + m/4 for exponents -2 .. 4
E3M2_POS = [k / 16 for k in range(4)] + [(4 + m) / 4 * 2.0 ** e for e in range(-2, 5) for m in range(4)]


@pytest.mark.parametrize("f,pos,ebits,mbits", [(O.E2M3, E2M3_POS, 2, 3), (O.E3M2, E3M2_POS, 3, 2)])
def test_fp6_codes(f, pos, ebits, mbits):
    assert len(pos) == 32 and pos[-1] == O.fmt_info(f)["maxval"]
    for c in range(64):
        v = O.decode_code(f, c)
        mag = pos[c & 31]
        assert v == (-mag if c & 32 else mag), (c, v)
        assert np.isfinite(v)
        if v != 0 or not (c & 32):
            assert O.encode_code(f, v) == c
    # every representable value quantises to itself
    for v in pos:
        assert O.quantize(f, np.array([v, -v])).tolist() == [v, -v]


def test_fp6_rounding_and_saturation():
    q2 = lambda x: O.quantize(O.E2M3, np.array([x]))[0]   # noqa: E731
    q3 = lambda x: O.quantize(O.E3M2, np.array([x]))[0]   # noqa: E731
    assert q2(1.0625) == 1.0        # midpoint of 1.0 and 1.125: even mantissa
    assert q2(1.1875) == 1.25       # midpoint of 1.125 and 1.25: even is 1.25
    assert q2(0.0625) == 0.0        # half the smallest subnormal: ties to zero
    assert q2(0.0626) == 0.125
    assert q2(7.75) == 7.5 and q2(1e30) == 7.5 and q2(-1e30) == -7.5   # saturation
    assert q2(np.inf) == 7.5
    assert q3(0.09375) == 0.125     # midpoint of 0.0625 and 0.125: even (2 * 2^-4)
    assert q3(26.0) == 24.0 and q3(26.5) == 28.0 and q3(1e9) == 28.0
    assert q3(0.03125) == 0.0 and q3(-0.04) == -0.0625


def test_fp6_block_exponent():
    """EncodeBlockMX: E = floor(log2 amax) - emax (2 for E2M3, 4 for E3M2)."""
    E, m = O.mx_encode(O.E2M3, [3.0, -0.5, 0.01, 6.9])
    assert E == 2 - 2 and m.tolist() == [3.0, -0.5, 0.0, 7.0]
    E, m = O.mx_encode(O.E3M2, [100.0, 1.0, -0.3])
    assert E == 6 - 4 and m.tolist() == [24.0, 0.25, -0.0625]


def test_fp6_fft_against_fp64():
    """The MXFP6 FFT of k-space data is close to FP64, and E2M3 (three
    mantissa bits) is closer than E3M2 (two), as the paper finds."""
    x = synth.kspace_batch(64, 1, 1, 2)
    ref = np.fft.fft2(x.astype(np.complex128))
    err = {}
    for f in (O.E2M3, O.E3M2):
        st, y, k = O.transform(x, fmt=f, B=32)
        assert st == O.OK
        err[f] = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    assert err[O.E2M3] < err[O.E3M2] < 0.6
    assert err[O.E2M3] > 0.01
