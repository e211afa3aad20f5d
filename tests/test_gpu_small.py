"""The single-launch kernel of small slices (n <= 128: Alg. 1, the row and
column passes and both halves of a round trip in one work-group's LDS)
against the oracle, bit for bit, and against the line kernels of the same
plan (same arithmetic, several launches), for every format, operation and
flag, and at batches that change its work-group size."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2512_04317_amd import mxfft, synth

pytestmark = pytest.mark.gpu

FMTS = {"e4m3": O.E4M3, "e5m2": O.E5M2, "e2m3": O.E2M3, "e3m2": O.E3M2}
OPS = {"forward": O.FORWARD, "inverse": O.INVERSE, "roundtrip": O.ROUNDTRIP}


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield


def bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


def run(plan, op, xd, k_in=None):
    if op == "forward":
        y, k = plan.forward(xd)
    elif op == "inverse":
        y, k = plan.inverse(xd, k_in=k_in), None
    else:
        y, k = plan.roundtrip(xd)
    st = plan.last_status()
    torch.cuda.synchronize()
    return y.cpu().numpy(), None if k is None else k.cpu().numpy(), st


def oracle(x, op, fmt, B, flags=0, k_in=None):
    if fmt == "fp32":
        mode, f = O.MODE_FP32, O.E4M3
    elif fmt in ("fp16", "bf16"):
        mode, f = (O.MODE_FP16 if fmt == "fp16" else O.MODE_BF16), O.E4M3
    else:
        mode, f = O.MODE_MX, FMTS[fmt]
    return O.transform(x, op=OPS[op], mode=mode, fmt=f, B=B, kp=k_in, flags=flags, nthreads=8)


def batch_of(N, seed):
    """Synthetic k-space, heavy-tailed random data, an all-zero slice and a
    tiny one."""
    x = np.concatenate([synth.kspace_batch(N, 5, 1, 2) if N >= 8 else
                        synth.random_complex((2, N, N), seed=seed + 1, dist="lognormal"),
                        synth.random_complex((2, N, N), seed=seed, dist="lognormal")])
    x = np.concatenate([x, np.zeros((1, N, N), np.complex64), x[:1] * np.float32(2.0 ** -100)])
    return np.ascontiguousarray(x)


CASES = [(2, "e4m3", 2), (4, "e5m2", 4), (8, "e4m3", 8), (16, "e2m3", 8), (32, "e3m2", 32), (64, "e4m3", 32),
         (64, "e5m2", 64), (16, "fp16", 0), (32, "bf16", 0), (64, "fp32", 0), (64, "fp16", 0)]


@pytest.mark.parametrize("op", ["forward", "inverse", "roundtrip"])
@pytest.mark.parametrize("N,fmt,B", CASES)
def test_single_launch_matches_oracle_and_line_kernels(N, fmt, B, op):
    x = batch_of(N, N)
    kw = dict(fmt=fmt) if B == 0 else dict(fmt=fmt, block=B)
    flags = mxfft.NO_PRESCALE if fmt == "fp32" else 0
    print("single-launch case: N=%d %s B=%d %s" % (N, fmt, B, op), flush=True)
    xd = torch.from_numpy(x).cuda()
    with mxfft.Plan(N, x.shape[0], flags=flags, **kw) as plan:
        assert plan.tuning()["single"]
        ys, ks, sts = run(plan, op, xd)
        plan.set_tuning(0, single=False)
        assert not plan.tuning()["single"]
        yl, kl, stl = run(plan, op, xd)
    assert sts == stl == mxfft.OK
    assert np.array_equal(bits(ys), bits(yl)), "single launch and line kernels differ"
    if ks is not None:
        np.testing.assert_array_equal(ks, kl)
    so, yo, ko = oracle(x, op, fmt, max(B, 2), flags=O.NO_PRESCALE if fmt == "fp32" else 0)
    assert so == O.OK
    if ks is not None:
        np.testing.assert_array_equal(ks, ko)
    if fmt == "fp32":
        err = np.linalg.norm(ys - yo) / max(np.linalg.norm(yo), 1e-30)
        assert err <= 1e-6, err
    else:
        bad = bits(ys) != bits(yo)
        bad &= ~(np.isnan(ys.view(np.float32)) & np.isnan(yo.view(np.float32)))
        assert not bad.any(), "%d words differ from the oracle" % bad.sum()


@pytest.mark.parametrize("fmt,B", [("e4m3", 16), ("e3m2", 8), ("bf16", 0)])
def test_single_launch_flags_and_given_k(fmt, B):
    """KEEP_SCALE forward, then the inverse with that k (k_in) and NORMALIZE;
    the fused round trip (MX); no prescale."""
    N = 32
    x = batch_of(N, 7)
    kw = dict(fmt=fmt) if B == 0 else dict(fmt=fmt, block=B)
    xd = torch.from_numpy(x).cuda()
    print("single-launch flags case: %s B=%d" % (fmt, B), flush=True)
    with mxfft.Plan(N, x.shape[0], flags=mxfft.KEEP_SCALE, **kw) as fwd, \
            mxfft.Plan(N, x.shape[0], flags=mxfft.NORMALIZE, **kw) as inv:
        y, k = fwd.forward(xd)
        z = inv.inverse(y, k_in=k)
        assert fwd.last_status() == mxfft.OK
        torch.cuda.synchronize()
        yg, kg, zg = y.cpu().numpy(), k.cpu().numpy(), z.cpu().numpy()
    so, yo, ko = oracle(x, "forward", fmt, max(B, 2), flags=O.KEEP_SCALE)
    np.testing.assert_array_equal(kg, ko)
    assert np.array_equal(bits(yg), bits(yo))
    so, zo, _ = oracle(yo, "inverse", fmt, max(B, 2), flags=O.NORMALIZE, k_in=ko)
    assert np.array_equal(bits(zg), bits(zo))
    if B:
        with mxfft.Plan(N, x.shape[0], flags=mxfft.FUSED_ROUNDTRIP, **kw) as rt:
            r, _ = rt.roundtrip(xd)
            torch.cuda.synchronize()
            so, ro, _ = oracle(x, "roundtrip", fmt, B, flags=O.FUSED_RT)
            assert np.array_equal(bits(r.cpu().numpy()), bits(ro))
    with mxfft.Plan(N, x.shape[0], flags=mxfft.NO_PRESCALE, **kw) as nop:
        y, k = nop.forward(xd)
        torch.cuda.synchronize()
        so, yo, ko = oracle(x, "forward", fmt, max(B, 2), flags=O.NO_PRESCALE)
        assert (k.cpu().numpy() == 0).all()
        assert np.array_equal(bits(y.cpu().numpy()), bits(yo))


def test_single_launch_large_batch_with_errors():
    """Many 64^2 slices in one launch, with a non-finite slice: its k is
    INT32_MIN and the call reports it; the other slices are exact."""
    N = 64
    x = synth.random_complex((300, N, N), seed=11, dist="lognormal")
    x[123, 4, 5] = np.float32(np.inf)
    xd = torch.from_numpy(x).cuda()
    print("single-launch case: 300 x 64^2 with an infinity", flush=True)
    with mxfft.Plan(N, 300, fmt="e4m3", block=32) as plan:
        y, k = plan.forward(xd)
        assert plan.last_status() == mxfft.ENONFINITE
        torch.cuda.synchronize()
        yg, kg = y.cpu().numpy(), k.cpu().numpy()
    assert kg[123] == mxfft.INT32_MIN
    keep = [i for i in range(300) if i != 123][::23]
    so, yo, ko = oracle(x[keep], "forward", "e4m3", 32)
    np.testing.assert_array_equal(kg[keep], ko)
    assert np.array_equal(bits(yg[keep]), bits(yo))


def test_tuner_times_the_single_launch():
    """n <= 64: the tuner weighs the single-launch kernel against the line
    kernels and a plan takes either choice."""
    t = mxfft.tune(64, sample=16, force=True)
    assert not t["fast"] and t["lines"] >= 1 and t["ms"] > 0
    with mxfft.Plan(64, 4) as pl:
        pl.set_tuning(t["lines"], single=t["single"])
        assert pl.tuning()["single"] == t["single"]
    with mxfft.Plan(256, 1) as big:
        with pytest.raises(mxfft.MxfftError):
            big.set_tuning(0, single=True)                   # n > 128 has no single-launch kernel


@pytest.mark.parametrize("op", ["forward", "inverse", "roundtrip"])
@pytest.mark.parametrize("fmt,B", [("e4m3", 32), ("e2m3", 16), ("fp16", 0), ("e5m2", 64), ("fp32", 0), ("e2m3", 8)])
def test_single_launch_at_128(fmt, B, op):
    """n = 128 (132 KiB of LDS per slice; a tuning choice beside the
    register-resident passes, the default without them) against the other
    kernels of the plan and the oracle, bit for bit."""
    N = 128
    x = batch_of(N, 3)
    kw = dict(fmt=fmt) if B == 0 else dict(fmt=fmt, block=B)
    xd = torch.from_numpy(x).cuda()
    print("single-launch case: N=128 %s B=%d %s" % (fmt, B, op), flush=True)
    with mxfft.Plan(N, x.shape[0], **kw) as plan:
        # the default where the plan has no register-resident passes
        assert plan.tuning()["single"] == (not plan.tuning()["fast"])
        plan.set_tuning(0, single=False)
        yd, kd, std = run(plan, op, xd)
        plan.set_tuning(0, single=True)
        assert plan.tuning()["single"]
        ys, ks, sts = run(plan, op, xd)
    assert std == sts == mxfft.OK
    assert np.array_equal(bits(ys), bits(yd))
    if ks is not None:
        np.testing.assert_array_equal(ks, kd)
    so, yo, ko = oracle(x, op, fmt, max(B, 2))
    if fmt == "fp32":
        fin = np.isfinite(yo)
        err = np.linalg.norm(ys[fin] - yo[fin]) / max(np.linalg.norm(yo[fin]), 1e-30)
        assert err <= 1e-6, err
        return
    bad = bits(ys) != bits(yo)
    bad &= ~(np.isnan(ys.view(np.float32)) & np.isnan(yo.view(np.float32)))
    assert not bad.any(), "%d words differ from the oracle" % bad.sum()


@pytest.mark.parametrize("N,batch,fmt,B", [(16, 4096, "e4m3", 16), (32, 4096, "e5m2", 32), (32, 1024, "fp16", 0),
                                           (64, 1024, "e4m3", 32), (64, 2048, "e2m3", 16), (64, 4096, "fp32", 0)])
def test_single_launch_work_group_sizes(N, batch, fmt, B):
    """Batches that hold several slices per CU give the single launch smaller
    work-groups (down to one wave per slice, each thread looping over several
    butterflies of a stage): bit for bit against the line kernels on every
    slice and against the oracle on sampled slices."""
    x = synth.random_complex((batch, N, N), seed=N + batch, dist="lognormal")
    x[batch // 3] *= np.float32(2.0 ** -100)
    kw = dict(fmt=fmt) if B == 0 else dict(fmt=fmt, block=B)
    xd = torch.from_numpy(x).cuda()
    print("single-launch case: %d x %d^2 %s B=%d" % (batch, N, fmt, B), flush=True)
    with mxfft.Plan(N, batch, **kw) as plan:
        assert plan.tuning()["single"]
        ys, ks, sts = run(plan, "roundtrip", xd)
        plan.set_tuning(0, single=False)
        yl, kl, stl = run(plan, "roundtrip", xd)
    assert sts == stl == mxfft.OK
    np.testing.assert_array_equal(ks, kl)
    assert np.array_equal(bits(ys), bits(yl)), "single launch and line kernels differ"
    pick = sorted({0, batch // 3, batch - 1} | set(range(7, batch, batch // 5)))
    so, yo, ko = oracle(x[pick], "roundtrip", fmt, max(B, 2))
    assert so == O.OK
    np.testing.assert_array_equal(ks[pick], ko)
    if fmt == "fp32":
        err = np.linalg.norm(ys[pick] - yo) / np.linalg.norm(yo)
        assert err <= 1e-6, err
    else:
        assert np.array_equal(bits(ys[pick]), bits(yo))
