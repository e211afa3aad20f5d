"""Pins of the oracle's fused round trip (the encode -> F -> F^-1 -> decode
the paper proposes in its discussion, Sec. 4): the forward result enters the
inverse transform's row stages without the inverse's input MX encode."""
import numpy as np

import oracle as O
from paper_2512_04317_amd import synth


def rt(x, fmt=O.E4M3, B=32, flags=0):
    st, y, k = O.transform(x, op=O.ROUNDTRIP, fmt=fmt, B=B, flags=flags)
    assert st == O.OK
    return y, k


def test_fused_equals_plain_when_the_encode_is_exact():
    """A delta's forward result is a constant, which every MX block holds
    exactly: skipping its re-encode changes nothing."""
    d = np.zeros((2, 32, 32), np.complex64)
    d[0, 0, 0] = 1.0
    d[1, 0, 0] = -3.0 + 0.5j
    a, ka = rt(d)
    b, kb = rt(d, flags=O.FUSED_RT)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32)) and np.array_equal(ka, kb)
    np.testing.assert_array_equal(a, d)


def test_fused_changes_only_the_round_trip_and_reduces_its_loss():
    x = synth.kspace_batch(64, 1, 1, 4)
    img = np.fft.ifft2(x.astype(np.complex128)).astype(np.complex64)   # coil images, as Eq. 1 takes them
    for op in (O.FORWARD, O.INVERSE):
        s1, y1, _ = O.transform(img, op=op, fmt=O.E4M3, B=32)
        s2, y2, _ = O.transform(img, op=op, fmt=O.E4M3, B=32, flags=O.FUSED_RT)
        assert np.array_equal(y1.view(np.uint32), y2.view(np.uint32))
    for f in (O.E4M3, O.E5M2):
        a, _ = rt(img, fmt=f)
        b, _ = rt(img, fmt=f, flags=O.FUSED_RT)
        assert (a.view(np.uint32) != b.view(np.uint32)).mean() > 0.5
        ea = np.linalg.norm(a - img) / np.linalg.norm(img)
        eb = np.linalg.norm(b - img) / np.linalg.norm(img)
        assert eb < ea, (f, ea, eb)
