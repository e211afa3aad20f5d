"""mxfft_forward_static (the forward transform whose workspace is the static
device array, for callers that cannot allocate) against mxfft_forward on the
same plan and data: outputs, prescale exponents and status bit for bit, on two
calls in a row, the second with a smaller batch (and other data), for each
kind of launch sequence (fused statistics, literal statistics, 16-bit and FP32
forms, generic line kernels)."""
import numpy as np
import pytest
import torch

from paper_2512_04317_amd import mxfft, synth

pytestmark = pytest.mark.gpu

CASES = [
    # (n, first batch, second batch, params): launch sequence covered
    (512, 8, 3, dict(fmt="e4m3", block=32)),                # row pass with statistics, column pass
    (1024, 6, 2, dict(fmt="e5m2", block=16)),               # same at 1024^2
    (256, 9, 4, dict(fmt="e4m3", block=8)),                 # literal statistics, register-resident passes
    (128, 12, 5, dict(fmt="e2m3", block=32)),               # MXFP6 on the register-resident passes
    (512, 5, 2, dict(fmt="fp16")),                          # 16-bit intermediate
    (512, 5, 2, dict(fmt="bf16")),
    (512, 4, 2, dict(fmt="fp32", flags=mxfft.NO_PRESCALE)),  # FP32 form, no statistics
    (64, 16, 7, dict(fmt="e4m3", block=32)),                # single launch
    (256, 6, 3, dict(fmt="e5m2", block=64)),                # B = 64: 32-line row tiles
    (512, 4, 2, dict(fmt="e4m3", block=64)),                # B = 64 with the statistics on the row pass
    (256, 4, 2, dict(fmt="e4m3", block=256)),               # line kernels, blocks above 128 (LDS maxima)
    (128, 6, 2, dict(fmt="e5m2", block=16, flags=mxfft.QUANTIZE_OUTPUT)),   # quantised output
]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield


def data(n, batch, seed):
    x = synth.kspace_batch(n, 7, 1, batch).reshape(batch, n, n)
    rng = np.random.default_rng([seed, n, batch])
    # a slice of tiny magnitudes sends the fused statistics to the literal redo
    if batch > 2:
        x[1] *= np.float32(2.0 ** -100)
    return np.ascontiguousarray(x[rng.permutation(batch)])


def run_pair(plan, n, batch, seed):
    x = torch.from_numpy(data(n, batch, seed)).cuda()
    y0 = torch.empty_like(x)
    k0 = torch.full((batch,), 12345, dtype=torch.int32, device="cuda")
    plan.forward(x, out=y0, k_out=k0)
    st0 = plan.last_status()
    y1 = torch.full_like(x, float("nan"))
    k1 = torch.full((batch,), -777, dtype=torch.int32, device="cuda")
    plan.forward_static(x, out=y1, k_out=k1)
    st1 = plan.last_status()
    torch.cuda.synchronize()
    assert st0 == st1 == mxfft.OK
    a, b = y0.cpu().numpy(), y1.cpu().numpy()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), "outputs differ"
    assert np.array_equal(k0.cpu().numpy(), k1.cpu().numpy()), "prescale exponents differ"


@pytest.mark.parametrize("n,b1,b2,kw", CASES)
def test_static_matches_forward_twice(n, b1, b2, kw):
    print("no-alloc case: n=%d batches %d then %d %s" % (n, b1, b2, kw), flush=True)
    with mxfft.Plan(n, b1, **kw) as plan:
        run_pair(plan, n, b1, 1)
        run_pair(plan, n, b2, 2)


def test_static_batch_beyond_plan_capacity():
    """The plan's max_batch bounds its own workspace only: a plan for one slice
    transforms 8 through the static workspace, as a plan for 8 does."""
    n, batch = 512, 8
    print("no-alloc case: n=512 batch 8 on a plan of max_batch 1", flush=True)
    x = torch.from_numpy(data(n, batch, 3)).cuda()
    with mxfft.Plan(n, batch, fmt="e4m3", block=32) as big, mxfft.Plan(n, 1, fmt="e4m3", block=32) as small:
        y0, k0 = big.forward(x)
        y1 = torch.empty_like(x)
        k1 = torch.empty(batch, dtype=torch.int32, device="cuda")
        small.forward_static(x, out=y1, k_out=k1)
        assert small.last_status() == mxfft.OK
        torch.cuda.synchronize()
        assert np.array_equal(y0.cpu().numpy().view(np.uint32), y1.cpu().numpy().view(np.uint32))
        assert np.array_equal(k0.cpu().numpy(), k1.cpu().numpy())


def test_static_status_and_limits():
    """A non-finite slice is reported through the static status words, and a
    batch whose workspace exceeds the array is refused before any launch."""
    n = 256
    print("no-alloc case: n=256 status words and the size limit", flush=True)
    x = data(n, 4, 4)
    x[2, 5, 7] = np.float32(np.nan)
    xd = torch.from_numpy(x).cuda()
    with mxfft.Plan(n, 4, fmt="e4m3", block=32) as plan:
        y = torch.empty_like(xd)
        k = torch.empty(4, dtype=torch.int32, device="cuda")
        plan.forward_static(xd, out=y, k_out=k)
        assert plan.last_status() == mxfft.ENONFINITE
        kk = k.cpu().numpy()
        assert kk[2] == mxfft.INT32_MIN and (kk[[0, 1, 3]] != mxfft.INT32_MIN).all()
    with mxfft.Plan(1024, 1, fmt="e4m3", block=32) as plan:
        big = torch.zeros((64, 1024, 1024), dtype=torch.complex64, device="cuda")
        kb = torch.empty(64, dtype=torch.int32, device="cuda")
        with pytest.raises(mxfft.MxfftError) as e:
            plan.forward_static(big, out=big, k_out=kb)
        assert e.value.status == mxfft.EBUDGET
