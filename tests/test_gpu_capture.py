"""The MX intermediate itself: the column pass's input as the GPU encodes it
(MXFFT_DEBUG_CAPTURE), element values and shared exponents bit for bit
against the oracle's EncodeBlockMX (Alg. 2) of its own row pass of the
prescaled slice.  Covers the generic line kernels (the column pass encodes
on load), the register-resident passes (the row pass stores FP8 codes and
E8M0 bytes in its swizzled layout) and the fused statistics (exponents stored
unscaled and offset by k, or the literal redo for out-of-window slices)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2512_04317_amd import mxfft, synth

pytestmark = pytest.mark.gpu

FMTS = {"e4m3": O.E4M3, "e5m2": O.E5M2, "e2m3": O.E2M3, "e3m2": O.E3M2}


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield


def oracle_column_input(x, fmt, B):
    """Oracle: k of Alg. 1, the row pass of 2^k x, then EncodeBlockMX of each
    column's blocks of B/2 rows."""
    st, k = O.prescale(x)
    assert st == O.OK
    xs = np.ldexp(x.view(np.float32), k).astype(np.float32).view(np.complex64)
    a = O.pass_lines(xs, mode=O.MODE_MX, fmt=FMTS[fmt], B=B)
    mant, E = O.column_encode(a, fmt=FMTS[fmt], B=B)
    return k, mant.astype(np.complex64), E


@pytest.mark.parametrize("N,fmt,B", [
    (4, "e4m3", 4), (8, "e5m2", 8), (64, "e4m3", 32), (64, "e2m3", 8),      # line kernels
    (128, "e4m3", 32), (256, "e5m2", 16), (256, "e3m2", 32),                # register-resident, literal statistics
    (512, "e4m3", 32), (512, "e2m3", 16), (1024, "e5m2", 8),                # fused statistics
    (256, "e5m2", 64), (512, "e4m3", 64),                                   # blocks of 64: 32-line row tiles
    (256, "e4m3", 256),                                                     # blocks above 128: line kernels
])
def test_column_pass_input_matches_oracle_encode(N, fmt, B):
    batch = 3
    x = synth.kspace_batch(N, 8, 1, batch)
    x[1] *= np.float32(2.0 ** -100)        # outside the fused statistics' window: literal redo
    print("capture case: N=%d %s B=%d batch=%d" % (N, fmt, B, batch), flush=True)
    with mxfft.Plan(N, batch, fmt=fmt, block=B, flags=mxfft.DEBUG_CAPTURE) as plan:
        xd = torch.from_numpy(x).cuda()
        _, k = plan.forward(xd)
        assert plan.last_status() == mxfft.OK
        mant, exps = plan.capture(batch)
        torch.cuda.synchronize()
        kg, mg, eg = k.cpu().numpy(), mant.cpu().numpy(), exps.cpu().numpy()
    for s in range(batch):
        ko, mo, Eo = oracle_column_input(x[s], fmt, B)
        assert kg[s] == ko, (s, kg[s], ko)
        np.testing.assert_array_equal(eg[s], Eo, err_msg="slice %d exponents" % s)
        bad = mg[s].view(np.uint32) != mo.view(np.uint32)
        assert not bad.any(), "slice %d: %d element values differ, first at %s" % (
            s, bad.sum(), np.argwhere(bad)[:3].tolist())


@pytest.mark.parametrize("N,fmt,B,single", [(8, "e4m3", 4, True), (64, "e5m2", 16, True), (64, "e4m3", 32, False),
                                            (128, "e2m3", 16, True), (256, "e3m2", 8, False),
                                            (256, "e4m3", 256, False)])
def test_stage_exponents_match_oracle_trace(N, fmt, B, single):
    """Alg. 2's block exponents at every stage (E_v, k_r, E_out) of row 0's
    row pass, recorded by the single-launch kernel and the line kernels, bit
    for bit against the oracle's trace of its own row pass."""
    batch = 3
    x = synth.kspace_batch(N, 8, 1, batch)
    x[2] *= np.float32(2.0 ** -100)
    print("trace case: N=%d %s B=%d single=%s" % (N, fmt, B, single), flush=True)
    with mxfft.Plan(N, batch, fmt=fmt, block=B, flags=mxfft.DEBUG_CAPTURE) as plan:
        plan.set_tuning(0, single=single)
        xd = torch.from_numpy(x).cuda()
        _, k = plan.forward(xd)
        assert plan.last_status() == mxfft.OK
        _, _, tr = plan.capture(batch, trace=True)
        torch.cuda.synchronize()
        trg = tr.cpu().numpy()
    for s in range(batch):
        st, ko = O.prescale(x[s])
        xs = np.ldexp(x[s].view(np.float32), ko).astype(np.float32).view(np.complex64)
        _, tro = O.pass_lines(xs[:1], mode=O.MODE_MX, fmt=FMTS[fmt], B=B, trace=True)
        np.testing.assert_array_equal(trg[s], tro, err_msg="slice %d stage exponents" % s)


@pytest.mark.parametrize("B", [32, 64])
def test_trace_needs_the_line_or_single_kernels(B):
    with mxfft.Plan(256, 1, fmt="e4m3", block=B, flags=mxfft.DEBUG_CAPTURE) as plan:
        plan.forward(torch.from_numpy(synth.kspace_batch(256, 8, 1, 1)).cuda())
        plan.capture(1)                                    # the register-resident intermediate: fine
        with pytest.raises(mxfft.MxfftError) as e:
            plan.capture(1, trace=True)
        assert e.value.status == mxfft.EUNSUPPORTED


def test_capture_needs_the_flag_and_a_call():
    with mxfft.Plan(64, 2, fmt="e4m3", block=32) as plan:
        with pytest.raises(mxfft.MxfftError):
            plan.capture(1)
    with mxfft.Plan(64, 2, fmt="e4m3", block=32, flags=mxfft.DEBUG_CAPTURE) as plan:
        with pytest.raises(mxfft.MxfftError):
            plan.capture(1)            # no forward call yet
        x = torch.from_numpy(synth.kspace_batch(64, 8, 1, 2)).cuda()
        plan.forward(x)
        with pytest.raises(mxfft.MxfftError):
            plan.capture(3)            # more than the call's batch
        plan.capture(2)
