"""The fused root-sum-of-squares coil combine (Eq. 1) on the GPU, through
the C ABI: each reconstruction's image equals the oracle's combine of the
oracle's per-coil transforms bit for bit (FP32 form: to tolerance)."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_2512_04317_amd import mxfft, synth  # noqa: E402

pytestmark = pytest.mark.gpu
NTHREADS = min(16, os.cpu_count() or 1)
MODES = {"fp32": O.MODE_FP32, "fp16": O.MODE_FP16, "bf16": O.MODE_BF16}
FMTS = {"e4m3": O.E4M3, "e5m2": O.E5M2, "e2m3": O.E2M3, "e3m2": O.E3M2}


def oracle_rss(x, coils, op, fmt, block):
    mode = MODES.get(fmt, O.MODE_MX)
    st, y, k = O.transform(x, op=O.FORWARD if op == mxfft.FORWARD else O.ROUNDTRIP, mode=mode,
                           fmt=FMTS.get(fmt, O.E4M3), B=block, nthreads=NTHREADS)
    assert st == O.OK
    return O.rss(y, coils), k


@pytest.mark.parametrize("op", [mxfft.FORWARD, mxfft.ROUNDTRIP])
@pytest.mark.parametrize("N,fmt,block", [(128, "e4m3", 32), (512, "e4m3", 32), (512, "e5m2", 8), (1024, "e4m3", 16),
                                         (512, "e2m3", 32), (256, "e3m2", 16), (256, "e4m3", 64), (512, "e5m2", 64),
                                         (256, "fp16", 0), (512, "bf16", 0), (1024, "fp16", 0)])
def test_rss_matches_oracle(N, fmt, block, op):
    coils = 3
    x = synth.kspace_batch(N, 2, 2, coils)                  # 2 reconstructions x 3 coils
    print("rss N=%d %s B=%d op=%d" % (N, fmt, block, op), flush=True)
    kw = dict(fmt=fmt, block=block) if block else dict(fmt=fmt)
    plan = mxfft.Plan(N, x.shape[0], **kw)
    xd = torch.from_numpy(x).cuda()
    rss, k = plan.rss(xd, coils, op=op)
    assert plan.last_status() == mxfft.OK
    ro, ko = oracle_rss(x, coils, op, fmt, block or 32)
    np.testing.assert_array_equal(k.cpu().numpy(), ko)
    r = rss.cpu().numpy()
    bad = r.view(np.uint32) != ro.view(np.uint32)
    assert not bad.any(), "%d of %d differ; first %s: gpu %s oracle %s" % (
        bad.sum(), bad.size, np.argwhere(bad)[:3].tolist(), r[bad][:3], ro[bad][:3])
    plan.close()


def test_rss_fp32_form_and_arguments():
    """FP32 form at 512^2 (its FFT may contract multiply-adds: held to the
    plain form's tolerance); the input stays untouched for the forward;
    argument errors and sizes without the fused epilogue."""
    coils = 4
    x = synth.kspace_batch(512, 2, 1, coils)
    plan = mxfft.Plan(512, coils, fmt="fp32", flags=mxfft.NO_PRESCALE)
    xd = torch.from_numpy(x).cuda()
    rss, _ = plan.rss(xd, coils)
    ref = np.sqrt((np.abs(np.fft.fft2(x.astype(np.complex128))) ** 2).sum(axis=0))
    err = np.linalg.norm(rss.cpu().numpy()[0] - ref) / np.linalg.norm(ref)
    assert err < 2e-6, err
    assert np.array_equal(xd.cpu().numpy().view(np.uint32), x.view(np.uint32))
    with pytest.raises(ValueError):
        plan.rss(xd, 3)                                     # not whole reconstructions
    # the FP32 form needs the scratch buffer for its intermediate: refused on the host without one
    out = torch.empty((1, 512, 512), dtype=torch.float32, device="cuda")
    assert mxfft.lib().mxfft_rss(plan.handle, mxfft.FORWARD, mxfft._ptr(xd), None, mxfft._ptr(out), 1, coils, None,
                                 mxfft._stream(None)) == mxfft.EINVAL
    plan.close()


@pytest.mark.parametrize("op", [mxfft.FORWARD, mxfft.ROUNDTRIP])
@pytest.mark.parametrize("N,fmt,block", [(64, "e4m3", 32), (512, "e2m3", 8), (256, "e3m2", 8)])
def test_rss_generic_kernels(N, fmt, block, op):
    """Plans without the fused epilogue (generic line kernels: small sizes,
    MXFP6 blocks of 8) transform into the scratch buffer and combine separately, with the
    same arithmetic: bit for bit against the oracle."""
    coils = 2
    x = synth.kspace_batch(N, 4, 2, coils)
    plan = mxfft.Plan(N, x.shape[0], fmt=fmt, block=block)
    assert not plan.tuning()["fast"]
    rss, k = plan.rss(torch.from_numpy(x).cuda(), coils, op=op)
    assert plan.last_status() == mxfft.OK
    fo = {"e4m3": O.E4M3, "e2m3": O.E2M3, "e3m2": O.E3M2}[fmt]
    st, y, ko = O.transform(x, op=O.FORWARD if op == mxfft.FORWARD else O.ROUNDTRIP, fmt=fo, B=block,
                            nthreads=NTHREADS)
    assert st == O.OK
    np.testing.assert_array_equal(k.cpu().numpy(), ko)
    np.testing.assert_array_equal(rss.cpu().numpy().view(np.uint32), O.rss(y, coils).view(np.uint32))
    with pytest.raises(mxfft.MxfftError) as e:              # the scratch buffer is required here
        out = torch.empty((2, N, N), dtype=torch.float32, device="cuda")
        st = mxfft.lib().mxfft_rss(plan.handle, int(op), mxfft._ptr(torch.from_numpy(x).cuda()), None,
                                   mxfft._ptr(out), 2, coils, None, mxfft._stream(None))
        if st != mxfft.OK:
            raise mxfft.MxfftError(st, "mxfft_rss")
    assert e.value.status == mxfft.EINVAL
    plan.close()


def test_ssim_kernel_against_oracle():
    """Mean SSIM of RSS images: against the oracle's FP64 evaluation of the
    same definition (different summation order: 1e-9), exactly 1 for an image
    against itself."""
    coils = 4
    x = synth.kspace_batch(256, 2, 2, coils)
    plan = mxfft.Plan(256, x.shape[0], fmt="e5m2", block=8)
    rss, _ = plan.rss(torch.from_numpy(x).cuda(), coils)
    ref = np.sqrt((np.abs(np.fft.fft2(x.astype(np.complex128))) ** 2).reshape(2, coils, 256, 256).sum(axis=1))
    ref = ref.astype(np.float32)
    s = mxfft.ssim(rss, torch.from_numpy(ref).cuda()).cpu().numpy()
    r = rss.cpu().numpy()
    for i in range(2):
        assert s[i] == pytest.approx(O.ssim(r[i], ref[i]), abs=1e-9)
        assert 0.2 < s[i] < 1.0
    same = mxfft.ssim(rss, rss).cpu().numpy()
    assert np.all(same == 1.0)
    plan.close()
