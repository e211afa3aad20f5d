"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

MX results are compared bit for bit (outputs, prescale exponents); the FP32
plain form within NRMSE 1e-6 of the oracle's FP32 form (it may contract
multiply-adds).  Inputs are the seeded synthetic k-space and seeded random
data with heavy-tailed magnitudes.
"""
import os

import numpy as np
import pytest
import torch

import oracle as O
from paper_2512_04317_amd import mxfft, synth

pytestmark = pytest.mark.gpu

NTHREADS = min(16, os.cpu_count() or 1)
FMTS = {"e4m3": O.E4M3, "e5m2": O.E5M2, "e2m3": O.E2M3, "e3m2": O.E3M2}


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield


def gpu_run(x, op="forward", n_batch=None, k_in=None, **params):
    x = np.ascontiguousarray(x.reshape(-1, x.shape[-2], x.shape[-1]))
    batch, N = x.shape[0], x.shape[-1]
    print("gpu case: op=%s N=%d batch=%d %s" % (op, N, batch, params), flush=True)
    plan = mxfft.Plan(N, n_batch or batch, **params)
    xd = torch.from_numpy(x).cuda()
    k = None
    if op == "forward":
        y, k = plan.forward(xd)
    elif op == "inverse":
        kd = None if k_in is None else torch.from_numpy(np.asarray(k_in, np.int32)).cuda()
        y = plan.inverse(xd, k_in=kd)
    else:
        y, k = plan.roundtrip(xd)
    st = plan.last_status()
    torch.cuda.synchronize()
    out = (y.cpu().numpy(), None if k is None else k.cpu().numpy(), st)
    plan.close()
    return out


def orc_run(x, op="forward", fmt="e4m3", block=32, k_in=None, flags=0, **kw):
    opcode = {"forward": O.FORWARD, "inverse": O.INVERSE, "roundtrip": O.ROUNDTRIP}[op]
    if fmt == "fp32":
        mode, f = O.MODE_FP32, O.E4M3
    elif fmt in ("fp16", "bf16"):
        mode, f = (O.MODE_FP16 if fmt == "fp16" else O.MODE_BF16), O.E4M3
    else:
        mode, f = O.MODE_MX, FMTS[fmt]
    return O.transform(x, op=opcode, mode=mode, fmt=f, B=block, kp=k_in, flags=flags, nthreads=NTHREADS, **kw)


def nrmse(y, r):
    return float(np.linalg.norm((y - r).ravel()) / max(np.linalg.norm(r.ravel()), 1e-300))


def assert_bitexact(yg, yo, what=""):
    """Bit for bit; a NaN matches any NaN (payloads carry no meaning)."""
    yg = np.ascontiguousarray(yg).reshape(yo.shape)
    bad = yg.view(np.uint32) != yo.view(np.uint32)
    bad &= ~(np.isnan(yg.view(np.float32)) & np.isnan(yo.view(np.float32)))
    if bad.any():
        idx = np.argwhere(bad)[:5]
        raise AssertionError("%s: %d of %d words differ (NRMSE %.3g); first at %s: gpu %s oracle %s"
                             % (what, bad.sum(), bad.size, nrmse(yg, yo), idx.tolist(),
                                yg.view(np.float32).ravel()[bad.ravel()][:4],
                                yo.view(np.float32).ravel()[bad.ravel()][:4]))


def small_cases():
    out = []
    for N in (2, 4, 8, 16, 32, 64, 128):
        for fmt in ("e4m3", "e5m2"):
            for B in (2, 4, 8, 16, 32, 64, 128):
                if B <= N:
                    out.append((N, fmt, B))
    return out


@pytest.mark.parametrize("N,fmt,B", small_cases())
def test_forward_small(N, fmt, B):
    x = synth.random_complex((3, N, N), seed=N * 1000 + B, dist="lognormal")
    yg, kg, st = gpu_run(x, fmt=fmt, block=B)
    so, yo, ko = orc_run(x, fmt=fmt, block=B)
    assert st == mxfft.OK and so == O.OK
    np.testing.assert_array_equal(kg, ko)
    assert_bitexact(yg, yo, "forward N=%d %s B=%d" % (N, fmt, B))


@pytest.mark.parametrize("fmt", ["e4m3", "e5m2"])
@pytest.mark.parametrize("B", [8, 16, 32, 64])
def test_forward_kspace_256(fmt, B):
    x = synth.kspace_batch(256, 2, 1, 8)
    yg, kg, st = gpu_run(x, fmt=fmt, block=B)
    so, yo, ko = orc_run(x, fmt=fmt, block=B)
    np.testing.assert_array_equal(kg, ko)
    assert_bitexact(yg, yo, "kspace256 %s B=%d" % (fmt, B))


@pytest.mark.parametrize("fmt", ["e4m3", "e5m2"])
@pytest.mark.parametrize("N", [64, 256])
def test_inverse_and_roundtrip(fmt, N):
    x = synth.kspace_batch(N, 2, 1, 4)
    # inverse with its own prescale
    yg, _, st = gpu_run(x, op="inverse", fmt=fmt, block=32)
    so, yo, _ = orc_run(x, op="inverse", fmt=fmt, block=32)
    assert_bitexact(yg, yo, "inverse")
    # inverse of a KEEP_SCALE forward output with the forward's k, normalised
    so, mid, k = orc_run(x, fmt=fmt, block=32, flags=O.KEEP_SCALE)
    yg, _, st = gpu_run(mid, op="inverse", k_in=k, fmt=fmt, block=32, flags=mxfft.NORMALIZE)
    so, yo, _ = orc_run(mid, op="inverse", fmt=fmt, block=32, k_in=k, flags=O.NORMALIZE)
    assert_bitexact(yg, yo, "inverse with k_in")
    # the round trip of Eq. 1
    yg, kg, st = gpu_run(x, op="roundtrip", fmt=fmt, block=32)
    so, yo, ko = orc_run(x, op="roundtrip", fmt=fmt, block=32)
    np.testing.assert_array_equal(kg, ko)
    assert_bitexact(yg, yo, "roundtrip")


@pytest.mark.parametrize("N", [4, 64, 256, 512])
def test_fp32_plain(N):
    x = synth.kspace_batch(N, 2, 1, 2) if N >= 64 else synth.random_complex((2, N, N), seed=5)
    yg, kg, st = gpu_run(x, fmt="fp32")
    so, yo, ko = orc_run(x, fmt="fp32")
    np.testing.assert_array_equal(kg, ko)
    assert nrmse(yg, yo) <= 1e-6
    ref = np.fft.fft2(x.astype(np.complex128))
    assert nrmse(yg, ref) <= 2e-6
    yg, _, _ = gpu_run(x, op="roundtrip", fmt="fp32")
    assert nrmse(yg, x) <= 1e-6


def prescale_cases():
    rng = np.random.default_rng(77)
    N = 32
    cases = []
    cases.append(("zeros", np.zeros((N, N), np.complex64), {}))
    one = np.zeros((N, N), np.complex64)
    one[3, 5] = 3.0 - 4.0j
    cases.append(("single", one, {}))
    cases.append(("lognormal", synth.random_complex((N, N), seed=9, dist="lognormal"), {}))
    cases.append(("kspace", synth.kspace_batch(N, 1, 1, 1)[0], {}))
    cases.append(("tiny", (synth.random_complex((N, N), seed=10) * np.float32(1e-30)), {}))
    cases.append(("clip", synth.random_complex((N, N), seed=11), dict(k_min=-2, k_max=1)))
    cases.append(("target", synth.random_complex((N, N), seed=12), dict(target=300.0, tau=37.0, tau_min=2.0 ** 3)))
    # order statistics either side of a power of two: refinement path
    st = np.full(N * N, 1.1, np.float32)
    st[:2] = 0.9
    rng.shuffle(st)
    cases.append(("straddle", st.reshape(N, N).astype(np.complex64), dict(tau=0.15, tau_min=2.0 ** 10)))
    st2 = np.full(N * N, 3.0, np.float32)
    st2[:40] = 1.75
    cases.append(("straddle2", st2.reshape(N, N).astype(np.complex64), dict(tau=3.85, tau_min=2.0 ** 10)))
    return cases


@pytest.mark.parametrize("name,x,kw", prescale_cases(), ids=[c[0] for c in prescale_cases()])
def test_prescale_exponent(name, x, kw):
    so, yo, ko = orc_run(x[None], fmt="e4m3", block=32, **kw)
    yg, kg, st = gpu_run(x[None], fmt="e4m3", block=32, **kw)
    assert st == mxfft.OK and so == O.OK
    np.testing.assert_array_equal(kg, ko)
    assert_bitexact(yg, yo, "prescale case " + name)


def test_flags_no_prescale_keep_scale():
    x = synth.kspace_batch(64, 2, 1, 2)
    for flags in (mxfft.NO_PRESCALE, mxfft.KEEP_SCALE):
        yg, kg, st = gpu_run(x, fmt="e5m2", block=16, flags=flags)
        so, yo, ko = orc_run(x, fmt="e5m2", block=16, flags=flags)
        np.testing.assert_array_equal(kg, ko)
        assert_bitexact(yg, yo, "flags %d" % flags)


def test_nonfinite_and_range_errors():
    x = synth.kspace_batch(32, 1, 1, 3)
    x[1, 4, 4] = np.nan
    yg, kg, st = gpu_run(x, fmt="e4m3", block=8)
    assert st == mxfft.ENONFINITE
    assert kg[1] == mxfft.INT32_MIN and kg[0] != mxfft.INT32_MIN and kg[2] != mxfft.INT32_MIN
    so, yo, ko = orc_run(x, fmt="e4m3", block=8)
    assert_bitexact(yg[[0, 2]], yo[[0, 2]], "finite slices beside a non-finite one")
    # largest component 215.09 = 1.68 * 2^7: 2^120 still fits FP32, 2^121 overflows
    x = synth.kspace_batch(32, 1, 1, 1)
    yg, kg, st = gpu_run(x, fmt="e4m3", block=8, k_min=120)
    assert st == mxfft.OK and kg[0] == 120 and O.prescale(x[0], k_min=120) == (O.OK, 120)
    yg, kg, st = gpu_run(x, fmt="e4m3", block=8, k_min=121)
    assert st == mxfft.ERANGE and kg[0] == mxfft.INT32_MIN
    assert O.prescale(x[0], k_min=121) == (O.ERANGE, O.INT32_MIN)


@pytest.mark.parametrize("N,kw", [(128, dict(fmt="e4m3", block=32)), (512, dict(fmt="e2m3", block=32)),
                                  (1024, dict(fmt="e3m2", block=16)), (512, dict(fmt="bf16")),
                                  (512, dict(fmt="fp32", flags=mxfft.NO_PRESCALE))])
def test_in_place_batch_independence_determinism(N, kw):
    """Repeated calls give the same bits; in place (out = in) equals out of
    place; a slice transformed alone equals the same slice in a batch."""
    x = synth.kspace_batch(N, 2, 2, 3)
    print("in-place / batch case N=%d %s" % (N, kw), flush=True)
    plan = mxfft.Plan(N, 8, **kw)
    xd = torch.from_numpy(x).cuda()
    y1, k1 = plan.forward(xd)
    y2, k2 = plan.forward(xd)
    xi = xd.clone()
    y3, k3 = plan.forward(xi, out=xi)
    y4, k4 = plan.forward(xd[2:3].contiguous())
    torch.cuda.synchronize()
    a = y1.cpu().numpy()
    assert np.array_equal(a.view(np.uint32), y2.cpu().numpy().view(np.uint32))
    assert np.array_equal(a.view(np.uint32), y3.cpu().numpy().view(np.uint32))
    assert np.array_equal(a[2:3].view(np.uint32), y4.cpu().numpy().view(np.uint32))
    plan.close()


def test_plan_as_context_manager():
    """A plan used in a with-block works inside it and is released at its end."""
    x = torch.from_numpy(synth.kspace_batch(64, 1, 1, 2)).cuda()
    with mxfft.Plan(64, 2, fmt="e4m3", block=32) as plan:
        y, k = plan.forward(x)
        torch.cuda.synchronize()
        assert plan.last_status() == mxfft.OK and plan.handle
    assert plan.handle is None


@pytest.fixture(scope="module")
def full_workload():
    w = synth.WORKLOADS["kspace512_64x16"]
    x = synth.kspace_batch(w["N"], w["config"], w["slices"], w["coils"], workers=NTHREADS)
    return x


def test_full_size_sampled(full_workload):
    """The benchmark's launch: 1024 slices of 512^2, MXFP8-E4M3, B = 32.
    Every 16th slice's k against the oracle's Alg. 1; three whole slices bit
    for bit."""
    x = full_workload
    plan = mxfft.Plan(512, x.shape[0], fmt="e4m3", block=32)
    xd = torch.from_numpy(x).cuda()
    print("gpu case: full size 1024 x 512^2 e4m3 B=32", flush=True)
    y, k = plan.forward(xd)
    assert plan.last_status() == mxfft.OK
    kg = k.cpu().numpy()
    for s in range(0, x.shape[0], 16):
        st, ko = O.prescale(x[s])
        assert kg[s] == ko, s
    pick = [0, 517, x.shape[0] - 1]
    so, yo, ko = orc_run(x[pick], fmt="e4m3", block=32)
    yg = y[pick].cpu().numpy()
    assert_bitexact(yg, yo, "full-size sampled slices")
    plan.close()


@pytest.mark.parametrize("op", ["forward", "inverse", "roundtrip"])
@pytest.mark.parametrize("fmt", ["e4m3", "e5m2"])
@pytest.mark.parametrize("B", [2, 4, 8, 16, 32, 64])
def test_n512_all_blocks(op, fmt, B):
    """512^2 slices take the register-resident kernels for 4 <= B <= 64 and
    the generic kernels otherwise; every combination is bit-exact."""
    x = synth.kspace_batch(512, 3, 1, 2)
    yg, kg, st = gpu_run(x, op=op, fmt=fmt, block=B)
    so, yo, ko = orc_run(x, op=op, fmt=fmt, block=B)
    assert st == mxfft.OK and so == O.OK
    if kg is not None:
        np.testing.assert_array_equal(kg, ko)
    assert_bitexact(yg, yo, "512^2 %s %s B=%d" % (op, fmt, B))


@pytest.mark.parametrize("op", ["forward", "inverse", "roundtrip"])
@pytest.mark.parametrize("fmt", ["e4m3", "e5m2"])
@pytest.mark.parametrize("B", [2, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("N", [128, 256, 1024])
def test_fast_sizes_all_blocks(N, op, fmt, B):
    """128^2, 256^2 and 1024^2 slices take the register-resident kernels of
    their size for 4 <= B <= 32 and, at 256^2 and 1024^2, B = 64 (all with the
    statistics on the row pass), the single launch or the generic kernels
    otherwise."""
    x = synth.kspace_batch(N, 3, 1, 2)
    yg, kg, st = gpu_run(x, op=op, fmt=fmt, block=B)
    so, yo, ko = orc_run(x, op=op, fmt=fmt, block=B)
    assert st == mxfft.OK and so == O.OK
    if kg is not None:
        np.testing.assert_array_equal(kg, ko)
    assert_bitexact(yg, yo, "%d^2 %s %s B=%d" % (N, op, fmt, B))


@pytest.mark.parametrize("op", ["forward", "inverse", "roundtrip"])
@pytest.mark.parametrize("fmt", ["e2m3", "e3m2"])
@pytest.mark.parametrize("N,B,fast", [(16, 8, False), (64, 32, False), (128, 32, True), (256, 16, True),
                                      (512, 32, True), (512, 8, False), (1024, 16, True)])
def test_fp6_forms(N, B, fast, fmt, op):
    """MXFP6 elements (E2M3, E3M2) bit for bit, on the generic line kernels and
    on the register-resident passes (blocks of 16 and 32 at 128^2 .. 1024^2,
    which carry the 6-bit codes in the 8-bit conversions)."""
    pl = mxfft.Plan(N, 1, fmt=fmt, block=B)
    assert pl.tuning()["fast"] == fast
    pl.close()
    x = synth.kspace_batch(N, 3, 1, 2) if N >= 64 else synth.random_complex((3, N, N), seed=N, dist="lognormal")
    yg, kg, st = gpu_run(x, op=op, fmt=fmt, block=B)
    so, yo, ko = orc_run(x, op=op, fmt=fmt, block=B)
    assert st == mxfft.OK and so == O.OK
    if kg is not None:
        np.testing.assert_array_equal(kg, ko)
    assert_bitexact(yg, yo, "%d^2 %s %s B=%d" % (N, op, fmt, B))


@pytest.mark.parametrize("fmt,B", [("e4m3", 32), ("e5m2", 8), ("e2m3", 32), ("e5m2", 64)])
@pytest.mark.parametrize("N", [64, 128, 512, 1024])
def test_fused_roundtrip(N, fmt, B):
    """The fused round trip (no re-encode between the transforms) on every
    kind of pass: bit for bit against the oracle's fused round trip."""
    x = synth.kspace_batch(N, 2, 1, 2)
    img = np.fft.ifft2(x.astype(np.complex128)).astype(np.complex64)
    yg, kg, st = gpu_run(img, op="roundtrip", fmt=fmt, block=B, flags=mxfft.FUSED_ROUNDTRIP)
    so, yo, ko = orc_run(img, op="roundtrip", fmt=fmt, block=B, flags=O.FUSED_RT)
    assert st == mxfft.OK and so == O.OK
    np.testing.assert_array_equal(kg, ko)
    assert_bitexact(yg, yo, "fused round trip %d^2 %s B=%d" % (N, fmt, B))


def mixed_512_batch(N=512):
    """Slices inside and outside the window where the statistics ride on the
    unscaled row pass: k-space, tiny, all-zero, huge, single value, heavy-tailed."""
    ks = synth.kspace_batch(N, 4, 1, 2)
    one = np.zeros((N, N), np.complex64)
    one[7, 3 * N // 5] = 2.5 - 1.0j
    return np.stack([ks[0],
                     ks[1] * np.float32(1e-30),
                     np.zeros((N, N), np.complex64),
                     ks[1] * np.float32(1e25),
                     one,
                     synth.random_complex((N, N), seed=41, dist="lognormal")]).astype(np.complex64)


@pytest.mark.parametrize("op", ["forward", "roundtrip"])
@pytest.mark.parametrize("N,B", [(128, 32), (256, 32), (1024, 32), (256, 64), (1024, 64)])
def test_fast_sizes_prescale_paths(N, B, op):
    """The mixed batch at 128^2, 256^2 and 1024^2 (statistics on the row
    pass: 4, 16 and 32 histogram copies), out-of-window slices redone
    literally, for blocks of 32 and of 64 (32-line row tiles)."""
    x = mixed_512_batch(N)
    yg, kg, st = gpu_run(x, op=op, fmt="e4m3", block=B)
    so, yo, ko = orc_run(x, op=op, fmt="e4m3", block=B)
    assert st == mxfft.OK and so == O.OK
    np.testing.assert_array_equal(kg, ko)
    assert_bitexact(yg, yo, "%d^2 mixed %s B=%d" % (N, op, B))


@pytest.mark.parametrize("op", ["forward", "roundtrip"])
@pytest.mark.parametrize("fmt,B", [("e2m3", 32), ("e3m2", 16)])
@pytest.mark.parametrize("N", [256, 512, 1024])
def test_fp6_prescale_paths(N, fmt, B, op):
    """MXFP6 on the passes that gather the prescale statistics on the row
    pass: the mixed batch, slices inside and outside the window."""
    x = mixed_512_batch(N)
    yg, kg, st = gpu_run(x, op=op, fmt=fmt, block=B)
    so, yo, ko = orc_run(x, op=op, fmt=fmt, block=B)
    assert st == mxfft.OK and so == O.OK
    np.testing.assert_array_equal(kg, ko)
    assert_bitexact(yg, yo, "%d^2 mixed %s %s B=%d" % (N, op, fmt, B))


def fp6_range_batch(N):
    """Unprescaled slices whose block exponents reach past 127 - OFF (2^OFF
    the factor between the 6-bit element and its 8-bit carrier): impulses near
    2^125 (a plane wave of the same magnitude after each pass, no growth), two
    impulses in one slice, a tiny impulse and tiny noise."""
    x = np.zeros((6, N, N), np.complex64)
    x[0, 3, 5] = np.float32(2.0 ** 125 * 1.3) - 1j * np.float32(2.0 ** 124)
    x[1, N // 2, 7] = np.float32(-(2.0 ** 121) * 1.9)
    x[2, 1, 1] = np.float32(2.0 ** 123)
    x[2, N - 3, N // 3] = 1j * np.float32(2.0 ** 122 * 1.7)
    x[3, 5, N - 2] = np.float32(2.0 ** 118) + 1j * np.float32(2.0 ** 117)
    x[4, 9, 9] = np.float32(2.0 ** -120) - 1j * np.float32(2.0 ** -121)
    rng = np.random.default_rng(N)
    x[5] = ((rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))) * 1e-38).astype(np.complex64)
    return x


@pytest.mark.parametrize("fmt,B", [("e2m3", 32), ("e3m2", 16), ("e2m3", 8)])
@pytest.mark.parametrize("N", [128, 512])
def test_fp6_scale_range_edges(N, fmt, B):
    """Blocks whose scale 2^(E + OFF) would leave the E8M0 range: encoded
    with 2^E and the values times 2^-OFF, decoded times 2^OFF, on the
    register-resident passes (B = 16, 32) and the line kernels (B = 8).  No
    round trip: its unnormalised inverse of the forward overflows FP32 here."""
    x = fp6_range_batch(N)
    for op in ("forward", "inverse"):
        yg, kg, st = gpu_run(x, op=op, fmt=fmt, block=B, flags=mxfft.NO_PRESCALE)
        so, yo, ko = orc_run(x, op=op, fmt=fmt, block=B, flags=O.NO_PRESCALE)
        assert st == mxfft.OK and so == O.OK
        assert np.isfinite(yo).all() and np.abs(yo).max() > 2.0 ** 124
        assert_bitexact(yg, yo, "%d^2 %s %s B=%d range edges" % (N, op, fmt, B))


def fp8_range_batch(N):
    """Slices at both ends of the E8M0 scale range for MXFP8 (no prescale, or
    a prescale clipped to keep them there): an impulse near 2^125 and two
    near 2^122 (a plane wave of the same size after each pass), FP32-subnormal
    noise and a tiny impulse (block exponents clamped at -127 and product
    scales 2^(E_w + E_v + k_r) below 2^-127, which the kernels apply with
    ldexp), a subnormal impulse that quantises to zero, and an ordinary slice
    with a few rows of tiny values beside its normal ones."""
    x = np.zeros((6, N, N), np.complex64)
    x[0, 3, 5] = np.float32(2.0 ** 125 * 1.3) - 1j * np.float32(2.0 ** 124)
    x[1, 1, 1] = np.float32(2.0 ** 122)
    x[1, N - 3, N // 3] = 1j * np.float32(2.0 ** 121 * 1.7)
    rng = np.random.default_rng([N, 8])
    x[2] = ((rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))) * 1e-38).astype(np.complex64)
    x[3, 9, 9] = np.float32(2.0 ** -120) - 1j * np.float32(2.0 ** -121)
    x[4, 2, N - 1] = np.float32(2.0 ** -140)
    x[5] = ((rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)))).astype(np.complex64)
    x[5, ::7] *= np.float32(2.0 ** -125)
    return x


@pytest.mark.parametrize("fmt,B", [("e4m3", 32), ("e5m2", 16), ("e4m3", 64), ("e5m2", 64)])
@pytest.mark.parametrize("N", [128, 512])
def test_fp8_scale_range_edges(N, fmt, B):
    """MXFP8 blocks at the E8M0 limits: block exponents clamped at -127, and
    product scales below 2^-127 (the decode-then-ldexp branch of the butterfly),
    on the register-resident passes (B = 16, 32, and 64 at 512^2) and the
    single launch (B = 64 at 128^2); forward and inverse without the
    prescale, and the forward with a prescale clipped at k_max = 0 (the fused
    statistics then redo every tiny slice literally at 512^2)."""
    x = fp8_range_batch(N)
    for op in ("forward", "inverse"):
        yg, kg, st = gpu_run(x, op=op, fmt=fmt, block=B, flags=mxfft.NO_PRESCALE)
        so, yo, ko = orc_run(x, op=op, fmt=fmt, block=B, flags=O.NO_PRESCALE)
        assert st == mxfft.OK and so == O.OK
        assert np.isfinite(yo).all() and np.abs(yo).max() > 2.0 ** 124
        assert_bitexact(yg, yo, "%d^2 %s %s B=%d E8M0 edges" % (N, op, fmt, B))
    yg, kg, st = gpu_run(x, fmt=fmt, block=B, k_max=0)
    so, yo, ko = orc_run(x, fmt=fmt, block=B, k_max=0)
    assert st == mxfft.OK and so == O.OK
    np.testing.assert_array_equal(kg, ko)
    assert (ko[2:5] == 0).all()
    assert_bitexact(yg, yo, "%d^2 forward %s B=%d k_max=0" % (N, fmt, B))


def tau_min_batch(N, rng):
    """Slices for Alg. 1 with a tail floor that is not a power of two
    (tau_min = 0.3 * 2^20, mantissa 0.6): the percentile (tau = 5) between
    two values a < T' <= b of one binade, T' = 0.6 * 2^(lp + 1) the floor's
    threshold in that binade, with p = a + f (b - a) on either side of T';
    the same with both order statistics below T'; synthetic k-space; and a
    slice of values near 1e-30 (Alg. 1's guard max(p, 1e-30))."""
    nn = N * N
    ri = int(np.floor((nn - 1) * 5.0 / 100.0))
    out = []
    for a, b in ((0.14, 0.16), (0.14, 0.151), (0.13, 0.14)):
        v = np.full(nn, b, np.float32)
        v[:ri + 1] = a
        rng.shuffle(v)
        out.append(v.reshape(N, N).astype(np.complex64))
    out.append(synth.kspace_batch(N, 6, 1, 1)[0])
    tiny = (9e-31 * (1.0 + 0.01 * rng.random((N, N)))).astype(np.float32)
    out.append(tiny.astype(np.complex64))
    return np.stack(out)


@pytest.mark.parametrize("N,fmt,B", [(512, "e4m3", 32), (256, "e5m2", 16), (64, "e4m3", 32), (512, "fp16", 32)])
def test_tau_min_not_a_power_of_two(N, fmt, B):
    """Alg. 1 with tau_min = 0.3 * 2^20 (and 0.3, where the 1e-30 guard
    decides): k bit for bit against the oracle on the fused statistics (512^2
    MX), the literal statistics (256^2, the 16-bit form) and the line kernels
    (64^2), with the outputs; the floor's mantissa matters (the power-of-two
    floor 2^18 gives another k for some of the first three slices)."""
    rng = np.random.default_rng([N, 9])
    x = tau_min_batch(N, rng)
    for tm, tgt in ((0.3 * 2.0 ** 20, 2.0 ** 7), (0.3, 2.0 ** -90)):
        yg, kg, st = gpu_run(x, fmt=fmt, block=B, tau_min=tm, target=tgt)
        so, yo, ko = orc_run(x, fmt=fmt, block=B, tau_min=tm, target=tgt)
        assert st == mxfft.OK and so == O.OK
        np.testing.assert_array_equal(kg, ko)
        assert_bitexact(yg, yo, "%d^2 %s tau_min=%g" % (N, fmt, tm))
    k_pow2 = [O.prescale(x[i], tau_min=2.0 ** 18)[1] for i in range(3)]
    k_gen = [O.prescale(x[i], tau_min=0.3 * 2.0 ** 20)[1] for i in range(3)]
    assert any(g != q for g, q in zip(k_gen, k_pow2)), (k_gen, k_pow2)


@pytest.mark.parametrize("op", ["forward", "inverse", "roundtrip"])
@pytest.mark.parametrize("fmt,B", [("e4m3", 32), ("e5m2", 8), ("e4m3", 64)])
def test_n512_prescale_paths(op, fmt, B):
    """512^2 with the prescale: slices whose block exponents stay inside the
    equivariance window and slices redone literally, in one batch."""
    x = mixed_512_batch()
    yg, kg, st = gpu_run(x, op=op, fmt=fmt, block=B)
    so, yo, ko = orc_run(x, op=op, fmt=fmt, block=B)
    assert st == mxfft.OK and so == O.OK
    if kg is not None:
        np.testing.assert_array_equal(kg, ko)
    assert_bitexact(yg, yo, "512^2 mixed %s %s B=%d" % (op, fmt, B))


def test_n512_prescale_limits_and_errors():
    """k pushed outside the window for every slice (k_min), a refinement case,
    and the non-finite / range errors on the 512^2 path."""
    ks = synth.kspace_batch(512, 4, 1, 2)
    yg, kg, st = gpu_run(ks, fmt="e4m3", block=32, k_min=60)
    so, yo, ko = orc_run(ks, fmt="e4m3", block=32, k_min=60)
    assert st == mxfft.OK and so == O.OK and (kg == 60).all()
    np.testing.assert_array_equal(kg, ko)
    assert_bitexact(yg, yo, "512^2 k_min=60")
    # order statistics either side of a power of two (refinement) at 512^2
    st2 = np.full(512 * 512, 3.0, np.float32)
    st2[:8913] = 1.75              # S[8912] = 1.75 and S[8913] = 3.0 straddle a power of two
    np.random.default_rng(5).shuffle(st2)
    xs = st2.reshape(1, 512, 512).astype(np.complex64)
    yg, kg, st = gpu_run(xs, fmt="e4m3", block=16, tau=3.4, tau_min=2.0 ** 10)
    so, yo, ko = orc_run(xs, fmt="e4m3", block=16, tau=3.4, tau_min=2.0 ** 10)
    assert st == mxfft.OK and so == O.OK
    np.testing.assert_array_equal(kg, ko)
    assert_bitexact(yg, yo, "512^2 refinement")
    # non-finite value in one slice; its neighbours unaffected
    xn = ks.copy()
    xn[1, 100, 200] = np.inf
    yg, kg, st = gpu_run(xn, fmt="e4m3", block=32)
    assert st == mxfft.ENONFINITE and kg[1] == mxfft.INT32_MIN and kg[0] != mxfft.INT32_MIN
    so, yo, ko = orc_run(xn[:1], fmt="e4m3", block=32)
    assert_bitexact(yg[:1], yo, "512^2 finite slice beside a non-finite one")
    # largest component near 2^k limit: ERANGE exactly where the oracle says so
    kmax_ok = 127 - int(np.floor(np.log2(np.abs(ks[0].view(np.float32)).max())))
    yg, kg, st = gpu_run(ks[:1], fmt="e4m3", block=32, k_min=kmax_ok)
    assert st == mxfft.OK and O.prescale(ks[0], k_min=kmax_ok)[0] == O.OK
    yg, kg, st = gpu_run(ks[:1], fmt="e4m3", block=32, k_min=kmax_ok + 1)
    assert st == mxfft.ERANGE and O.prescale(ks[0], k_min=kmax_ok + 1)[0] == O.ERANGE


def test_n512_redo_list_longer_than_grid():
    """80 slices pushed outside the equivariance window (k_min = 100: the
    largest block exponents, about 2^9 above the scale of the data, plus k
    pass 90): the redo pass's work-groups (64 slices' tiles) stride over the
    longer list."""
    x = synth.kspace_batch(512, 3, 5, 16)
    yg, kg, st = gpu_run(x, fmt="e4m3", block=32, k_min=100)
    so, yo, ko = orc_run(x, fmt="e4m3", block=32, k_min=100)
    assert st == mxfft.OK and so == O.OK and x.shape[0] == 80 and (kg == 100).all()
    assert np.isfinite(yo).all()
    np.testing.assert_array_equal(kg, ko)
    assert_bitexact(yg, yo, "512^2 redo list of 80 slices")


@pytest.mark.parametrize("fmt", ["fp16", "bf16"])
@pytest.mark.parametrize("N", [2, 8, 32, 64, 128, 256, 512, 1024])
def test_16bit_forms(fmt, N):
    """The 16-bit forms (Sec. 2.3): rounding of every pass input, v operand,
    product and sum to the format, bit for bit against the oracle; forward
    with the prescale, inverse with its own prescale, round trip."""
    if N >= 64:
        x = synth.kspace_batch(N, 5, 1, 2)
    else:
        x = synth.random_complex((3, N, N), seed=N + 7, dist="lognormal")
    for op in ("forward", "inverse", "roundtrip"):
        yg, kg, st = gpu_run(x, op=op, fmt=fmt)
        so, yo, ko = orc_run(x, op=op, fmt=fmt)
        assert st == mxfft.OK and so == O.OK
        if kg is not None:
            np.testing.assert_array_equal(kg, ko)
        assert_bitexact(yg, yo, "%s N=%d %s" % (fmt, N, op))


@pytest.mark.parametrize("N", [32, 128, 512, 1024])
@pytest.mark.parametrize("fmt", ["fp16", "bf16"])
def test_16bit_range_edges(fmt, N):
    """Values that overflow the half range and bfloat16 products below the
    FP32 normal range (no prescale, so the data reaches the kernels as is).
    At N >= 128 the bfloat16 waves that meet such products redo their lines
    with exact products; the big slices of the same batch do not."""
    rng = np.random.default_rng(3)
    big = (rng.standard_normal((2, N, N)) + 1j * rng.standard_normal((2, N, N))) * 3e4
    tiny = (rng.standard_normal((2, N, N)) + 1j * rng.standard_normal((2, N, N))) * 3e-39
    # a slice of ordinary values with one row of tiny ones: only the waves
    # that hold that row (row pass) or meet its values (column pass) redo
    mixed = rng.standard_normal((1, N, N)) + 1j * rng.standard_normal((1, N, N))
    mixed[0, N // 3] *= 3e-39
    x = np.concatenate([big, tiny, mixed]).astype(np.complex64)
    yg, kg, st = gpu_run(x, fmt=fmt, flags=mxfft.NO_PRESCALE)
    so, yo, ko = orc_run(x, fmt=fmt, flags=O.NO_PRESCALE)
    # overflow makes NaN (inf - inf) in the half form: NaNs must sit at the
    # same places (their payloads are not compared); every other value bit for bit
    yg = np.ascontiguousarray(yg).reshape(yo.shape)
    ng, no = np.isnan(yg), np.isnan(yo)
    np.testing.assert_array_equal(ng, no)
    assert_bitexact(np.where(ng, 0, yg), np.where(no, 0, yo), "%s range edges" % fmt)
    if fmt == "bf16":
        assert np.count_nonzero(yo[2:4]) > 0           # the subnormal products left a trace


@pytest.mark.parametrize("N,fmt,fast", [(128, "e4m3", False), (256, "e4m3", True), (512, "e5m2", True),
                                        (1024, "e4m3", True)])
def test_block_64_paths(N, fmt, fast):
    """MXFP8 B = 64 takes the register-resident passes at 256^2 .. 1024^2
    (blocks of 32 butterflies split over two or four lanes, row tiles of 32
    lines so that a column block's 32 rows are encoded in one work-group) and
    the single launch at 128^2.  Forward keeping k, the inverse with that k
    and the fused round trip on k-space and a heavy-tailed slice, bit for
    bit."""
    with mxfft.Plan(N, 2, fmt=fmt, block=64) as pl:
        t = pl.tuning()
        assert t["fast"] == fast
        assert t["single"] == (not fast)
    x = np.concatenate([synth.kspace_batch(N, 5, 1, 1),
                        synth.random_complex((1, N, N), seed=N + 64, dist="lognormal")]).astype(np.complex64)
    print("B=64 case: N=%d %s" % (N, fmt), flush=True)
    yg, kg, st = gpu_run(x, fmt=fmt, block=64, flags=mxfft.KEEP_SCALE)
    so, yo, ko = orc_run(x, fmt=fmt, block=64, flags=O.KEEP_SCALE)
    assert st == mxfft.OK and so == O.OK
    np.testing.assert_array_equal(kg, ko)
    assert_bitexact(yg, yo, "%d^2 %s B=64 forward, k kept" % (N, fmt))
    zg, _, st = gpu_run(yo, op="inverse", fmt=fmt, block=64, k_in=ko, flags=mxfft.NORMALIZE)
    so, zo, _ = orc_run(yo, op="inverse", fmt=fmt, block=64, k_in=ko, flags=O.NORMALIZE)
    assert_bitexact(zg, zo, "%d^2 %s B=64 inverse with k_in" % (N, fmt))
    rg, _, st = gpu_run(x, op="roundtrip", fmt=fmt, block=64, flags=mxfft.FUSED_ROUNDTRIP)
    so, ro, _ = orc_run(x, op="roundtrip", fmt=fmt, block=64, flags=O.FUSED_RT)
    assert_bitexact(rg, ro, "%d^2 %s B=64 fused round trip" % (N, fmt))


@pytest.mark.parametrize("op", ["forward", "inverse", "roundtrip"])
@pytest.mark.parametrize("N,fmt,B", [(64, "e4m3", 32), (256, "e5m2", 16), (512, "e4m3", 64), (512, "e2m3", 8),
                                     (1024, "e3m2", 32), (128, "e5m2", 128)])
def test_quantized_output(N, fmt, B, op):
    """MXFFT_QUANTIZE_OUTPUT: the output MX-encoded in blocks of B/2 rows of
    each column after the last pass, on the single launch (64^2, 128^2 with
    B = 128), the register-resident passes (256^2 .. 1024^2, fused
    statistics and blocks of 64 included) and the line kernels (MXFP6 B = 8):
    bit for bit against the oracle's quantised output."""
    x = synth.kspace_batch(N, 3, 1, 2)
    yg, kg, st = gpu_run(x, op=op, fmt=fmt, block=B, flags=mxfft.QUANTIZE_OUTPUT)
    so, yo, ko = orc_run(x, op=op, fmt=fmt, block=B, flags=O.QUANTIZE_OUT)
    assert st == mxfft.OK and so == O.OK
    if kg is not None:
        np.testing.assert_array_equal(kg, ko)
    assert_bitexact(yg, yo, "%d^2 %s %s B=%d quantised output" % (N, op, fmt, B))


def test_quantized_output_flag_elsewhere():
    """No effect on the 16-bit forms (their output is rounded to the format
    anyway); RSS refuses an MX plan with the flag."""
    x = synth.kspace_batch(128, 3, 1, 2)
    a, _, _ = gpu_run(x, fmt="fp16")
    b, _, _ = gpu_run(x, fmt="fp16", flags=mxfft.QUANTIZE_OUTPUT)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    with mxfft.Plan(128, 2, fmt="e4m3", block=32, flags=mxfft.QUANTIZE_OUTPUT) as pl:
        with pytest.raises(mxfft.MxfftError) as e:
            pl.rss(torch.from_numpy(x).cuda(), 2)
        assert e.value.status == mxfft.EUNSUPPORTED


@pytest.mark.parametrize("op", ["forward", "inverse", "roundtrip"])
@pytest.mark.parametrize("N,fmt,B,lines", [(256, "e4m3", 256, 0), (256, "e5m2", 256, 1), (512, "e5m2", 512, 0),
                                           (512, "e2m3", 256, 2), (1024, "e4m3", 1024, 0), (1024, "e3m2", 512, 4)])
def test_blocks_above_128(N, fmt, B, lines, op):
    """MX blocks of more than 64 butterflies (B = 256 .. n) on the line
    kernels, whose block maxima then go through LDS (a block spans several
    waves, or several steps of a thread's loop), with the default and with
    small line counts per work-group: bit for bit against the oracle."""
    x = synth.kspace_batch(N, 3, 1, 2)
    print("big-block case: N=%d %s B=%d lines=%d %s" % (N, fmt, B, lines, op), flush=True)
    with mxfft.Plan(N, 2, fmt=fmt, block=B) as pl:
        assert not pl.tuning()["fast"]
        if lines:
            pl.set_tuning(lines)
        xd = torch.from_numpy(x).cuda()
        if op == "forward":
            y, k = pl.forward(xd)
        elif op == "inverse":
            y, k = pl.inverse(xd), None
        else:
            y, k = pl.roundtrip(xd)
        st = pl.last_status()
        torch.cuda.synchronize()
        yg, kg = y.cpu().numpy(), None if k is None else k.cpu().numpy()
    so, yo, ko = orc_run(x, op=op, fmt=fmt, block=B)
    assert st == mxfft.OK and so == O.OK
    if kg is not None:
        np.testing.assert_array_equal(kg, ko)
    assert_bitexact(yg, yo, "%d^2 %s %s B=%d lines=%d" % (N, op, fmt, B, lines))


@pytest.mark.parametrize("N,fmt,B", [(128, "e4m3", 32), (256, "e5m2", 16), (256, "e4m3", 64), (1024, "e4m3", 32),
                                     (512, "e2m3", 32)])
def test_fused_statistics_nonfinite(N, fmt, B):
    """The row pass that gathers Alg. 1's statistics finds non-finite parts
    through its histogram (Inf/NaN land in their own bin, zeros in another):
    a NaN real part, a -Inf imaginary part and a NaN beside zeros each fail
    their own slice with ENONFINITE and k = INT32_MIN, and the finite slices
    around them (one of them mostly zeros) keep their k and output, bit for
    bit against the oracle."""
    ks = synth.kspace_batch(N, 2, 1, 5)
    sparse = np.zeros((N, N), np.complex64)
    sparse[3, 5] = 1.5 - 2.0j
    sparse[N - 2, N // 3] = 0.25j
    x = np.stack([ks[0], ks[1], sparse, ks[0], sparse]).astype(np.complex64)
    x[1, N // 2, 7] = np.complex64(complex(np.nan, 1.0))
    x[3, 1, N - 1] = np.complex64(complex(2.0, -np.inf))
    x[4, 0, 0] = np.complex64(complex(np.nan, 0.0))
    yg, kg, st = gpu_run(x, fmt=fmt, block=B)
    assert st == mxfft.ENONFINITE
    bad = [1, 3, 4]
    assert all(kg[i] == mxfft.INT32_MIN for i in bad)
    good = [0, 2]
    so, yo, ko = orc_run(x[good], fmt=fmt, block=B)
    assert so == O.OK
    np.testing.assert_array_equal(kg[good], ko)
    assert_bitexact(np.asarray(yg)[good], yo, "%d^2 %s B=%d finite slices beside non-finite ones" % (N, fmt, B))
    for i in bad:
        assert O.prescale(x[i])[0] == O.ENONFINITE
