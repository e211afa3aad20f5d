"""Uneven batches and launch tuning on the GPU, through the C ABI.

An uneven batch (groups of slices of different sizes in one pool, executed
as one HIP graph launch) must give every slice exactly the result of a
single-plan call, which the parity tests pin to the oracle; a few groups are
also compared with the oracle directly here.  Graph replays are checked
against the eager result with the program's own work in between."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_2512_04317_amd import mxfft, synth  # noqa: E402

pytestmark = pytest.mark.gpu
NTHREADS = min(16, os.cpu_count() or 1)


def bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


def pool_of(batch, xs):
    pool = np.zeros(batch.pool_elems, np.complex64)
    for (n, c, o), x in zip(batch.groups, xs):
        pool[o:o + c * n * n] = x.reshape(-1)
    return pool


# sizes of the uneven workload plus the small sizes; groups listed out of
# memory order (explicit offsets), one size twice
GROUPS = [(256, 3), (64, 5), (512, 2), (16, 7), (64, 2), (128, 4)]


def layout(groups):
    """Explicit offsets in reverse order of the list (gaps of 96 values)."""
    out, off = [], 0
    for n, c in reversed(groups):
        out.append((n, c, off))
        off += c * n * n + 96
    return list(reversed(out))


@pytest.mark.parametrize("fmt,block", [("e4m3", 16), ("e5m2", 8), ("fp16", 32)])
def test_uneven_batch_matches_single_plans(fmt, block):
    groups = layout(GROUPS)
    print("uneven batch %s B=%d groups=%s" % (fmt, block, groups), flush=True)
    b = mxfft.Batch(groups, fmt=fmt, block=block)
    xs = [synth.random_complex((c, n, n), seed=10 * i + n, dist="lognormal") for i, (n, c, _) in enumerate(groups)]
    pool = torch.from_numpy(pool_of(b, xs)).cuda()
    for op in (mxfft.FORWARD, mxfft.INVERSE, mxfft.ROUNDTRIP):
        out, k = b.execute(op, pool)
        assert b.last_status() == mxfft.OK
        yb = b.views(out.cpu())
        kb = None if k is None else k.cpu().numpy()
        for gi, ((n, c, _), x) in enumerate(zip(groups, xs)):
            pl = mxfft.Plan(n, c, fmt=fmt, block=block)
            xd = torch.from_numpy(x).cuda()
            if op == mxfft.FORWARD:
                y, ks = pl.forward(xd)
            elif op == mxfft.INVERSE:
                y, ks = pl.inverse(xd), None
            else:
                y, ks = pl.roundtrip(xd)
            torch.cuda.synchronize()
            assert np.array_equal(bits(yb[gi].numpy()), bits(y.cpu().numpy())), "group %d op %d" % (gi, op)
            if ks is not None:
                kbase = sum(cc for _, cc, _ in groups[:gi])
                assert np.array_equal(kb[kbase:kbase + c], ks.cpu().numpy())
            pl.close()
    # the groups' outputs stay in their ranges: the gaps are untouched
    out = torch.full_like(pool, 7 + 7j)
    b.execute(mxfft.FORWARD, pool, out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    mask = np.ones(o.size, bool)
    for n, c, off in groups:
        mask[off:off + c * n * n] = False
    assert np.all(o[mask] == 7 + 7j)
    b.close()


@pytest.mark.parametrize("fmt,block,flags", [("e4m3", 64, 0), ("e5m2", 64, mxfft.QUANTIZE_OUTPUT),
                                             ("e4m3", 256, 0)])
def test_uneven_batch_large_blocks(fmt, block, flags):
    """Work lists with MXFP8 blocks of 64 (single launch at 128^2, 32-line row
    tiles at 256^2 .. 1024^2, fused statistics from 256^2), of 256 (line
    kernels with LDS block maxima; sizes from 256^2) and with the quantised output: every
    group bit for bit as a single-plan call, forward and round trip; one
    group against the oracle."""
    sizes = [(512, 2), (128, 3), (1024, 1), (256, 4)] if block <= 128 else [(512, 2), (256, 3), (1024, 1)]   # B <= n
    groups = layout(sizes)
    print("uneven batch %s B=%d flags=%d" % (fmt, block, flags), flush=True)
    b = mxfft.Batch(groups, fmt=fmt, block=block, flags=flags)
    xs = [synth.kspace_batch(n, 3, 1, c) for n, c, _ in groups]
    pool = torch.from_numpy(pool_of(b, xs)).cuda()
    for op in (mxfft.FORWARD, mxfft.ROUNDTRIP):
        out, k = b.execute(op, pool)
        assert b.last_status() == mxfft.OK
        yb = b.views(out.cpu())
        kb = k.cpu().numpy()
        kbase = 0
        for gi, ((n, c, _), x) in enumerate(zip(groups, xs)):
            with mxfft.Plan(n, c, fmt=fmt, block=block, flags=flags) as pl:
                xd = torch.from_numpy(x).cuda()
                y, ks = pl.forward(xd) if op == mxfft.FORWARD else pl.roundtrip(xd)
                torch.cuda.synchronize()
                assert np.array_equal(bits(yb[gi].numpy()), bits(y.cpu().numpy())), "group %d op %d" % (gi, op)
                assert np.array_equal(kb[kbase:kbase + c], ks.cpu().numpy())
            kbase += c
        fo = O.E4M3 if fmt == "e4m3" else O.E5M2
        oflags = O.QUANTIZE_OUT if flags else 0
        st, yo, ko = O.transform(xs[1], op=O.FORWARD if op == mxfft.FORWARD else O.ROUNDTRIP, fmt=fo, B=block,
                                 flags=oflags, nthreads=NTHREADS)
        assert st == O.OK
        assert np.array_equal(bits(yb[1].numpy()), bits(yo)), "group 1 vs oracle"
    b.close()


def test_uneven_batch_against_oracle():
    groups = [(64, 3), (256, 2), (512, 1)]
    b = mxfft.Batch(groups, fmt="e4m3", block=32)
    xs = [synth.kspace_batch(n, 2, 1, c) for n, c in groups]
    pool = torch.from_numpy(pool_of(b, xs)).cuda()
    out, k = b.forward(pool)
    assert b.last_status() == mxfft.OK
    yb = b.views(out.cpu())
    kb = k.cpu().numpy()
    kbase = 0
    for gi, ((n, c), x) in enumerate(zip(groups, xs)):
        st, yo, ko = O.transform(x, fmt=O.E4M3, B=32, nthreads=NTHREADS)
        assert st == O.OK
        assert np.array_equal(bits(yb[gi].numpy()), bits(yo)), "group %d" % gi
        assert np.array_equal(kb[kbase:kbase + c], ko)
        kbase += c
    b.close()


def test_uneven_batch_graph_replays():
    """Replays of the captured graph, with eager work and synchronisation in
    between, each equal the first result; a new output pointer re-captures."""
    groups = [(128, 3), (512, 2), (32, 6)]
    b = mxfft.Batch(groups, fmt="e4m3", block=32)
    xs = [synth.random_complex((c, n, n), seed=n, dist="lognormal") for n, c in groups]
    pool = torch.from_numpy(pool_of(b, xs)).cuda()
    out, k = b.forward(pool)
    torch.cuda.synchronize()
    ref, kref = out.cpu().numpy().copy(), k.cpu().numpy().copy()
    other = mxfft.Plan(64, 4, fmt="e5m2", block=8)
    junk = torch.from_numpy(synth.random_complex((4, 64, 64), seed=3)).cuda()
    for rep in range(4):
        out.fill_(0)
        other.forward(junk)                       # eager work of the program between replays
        torch.cuda.synchronize()
        b.forward(pool, out, k)
        torch.cuda.synchronize()
        assert np.array_equal(bits(out.cpu().numpy()), bits(ref)), "replay %d" % rep
        assert np.array_equal(k.cpu().numpy(), kref)
    out2, k2 = b.forward(pool)                    # other buffers: captured again
    torch.cuda.synchronize()
    assert np.array_equal(bits(out2.cpu().numpy()), bits(ref))
    other.close()
    b.close()


def test_tuner_cache_round_trip(tmp_path):
    """The tuner measures the candidates on a miss, records the winner, and
    answers from the file afterwards; the chosen launch is bit-identical to
    the default one."""
    cache = str(tmp_path / "tune.json")
    t1 = mxfft.tune(64, sample=8, cache=cache)
    assert not t1["fast"] and t1["lines"] >= 1 and t1["ms"] > 0
    assert os.path.exists(cache)
    arch = torch.cuda.get_device_properties(0).gcnArchName
    hit = mxfft.tune_cache_lookup(cache, arch, 64)
    assert hit is not None and hit["lines"] == t1["lines"]
    t2 = mxfft.tune(64, sample=8, cache=cache)
    assert t2["lines"] == t1["lines"] and t2["ms"] == pytest.approx(hit["ms"])
    t3 = mxfft.tune(64, sample=8, cache=cache, fmt="e5m2", block=8)    # another key, same file
    assert mxfft.tune_cache_lookup(cache, arch, 64) is not None
    assert mxfft.tune_cache_lookup(cache, arch, 64, fmt="e5m2", block=8)["lines"] == t3["lines"]
    assert mxfft.tune(512, sample=2, cache=cache)["fast"]              # register-resident: nothing to tune
    x = torch.from_numpy(synth.random_complex((3, 64, 64), seed=5, dist="lognormal")).cuda()
    pl = mxfft.Plan(64, 3)
    y0, k0 = pl.forward(x)
    y0 = y0.cpu().numpy().copy()
    for r in (1, 2, 8, 32, 64):
        pl.set_tuning(r)
        assert pl.tuning()["lines"] == r
        y, k = pl.forward(x)
        torch.cuda.synchronize()
        assert np.array_equal(bits(y.cpu().numpy()), bits(y0)), "lines %d" % r
    with pytest.raises(mxfft.MxfftError):
        pl.set_tuning(3)
    with pytest.raises(mxfft.MxfftError):
        pl.set_tuning(128)                         # more lines than the slice has
    pl.close()


def test_per_reconstruction_work_list():
    """Reconstructions in arrival order, each its coils contiguous at its own
    offset, sizes interleaved (so each size's branch addresses its slices
    through the offset table): every slice bit for bit against a single-plan
    call, a sample against the oracle, k in the callers' order; a tiny coil
    takes the fused statistics' literal redo, a non-finite one fails alone."""
    rng = np.random.default_rng([20251204, 41])
    sizes = rng.choice([32, 64, 128, 256, 512], size=24)
    coils = rng.integers(1, 4, size=24)
    groups, off = [], 0
    for n, c in zip(sizes.tolist(), coils.tolist()):
        groups.append((n, c, off))
        off += c * n * n + 8
    print("work list: %d reconstructions, %s" % (len(groups), groups), flush=True)
    xs = [synth.kspace_batch(n, 4, 1, c) for n, c, _ in groups]
    big = [i for i, (n, _, _) in enumerate(groups) if n == 512]
    xs[big[0]][0] *= np.float32(2.0 ** -110)            # outside the fused statistics' window
    bad = [i for i, (n, _, _) in enumerate(groups) if n == 128][0]
    xs[bad][-1, 3, 3] = np.float32(np.nan)
    b = mxfft.Batch(groups, fmt="e4m3", block=32)
    pool = torch.from_numpy(pool_of(b, xs)).cuda()
    for op in (mxfft.FORWARD, mxfft.ROUNDTRIP):
        out, k = b.execute(op, pool)
        assert b.last_status() == mxfft.ENONFINITE
        yb = b.views(out.cpu())
        kb = k.cpu().numpy()
        kbase = 0
        for gi, ((n, c, _), x) in enumerate(zip(groups, xs)):
            with mxfft.Plan(n, c, fmt="e4m3", block=32) as pl:
                xd = torch.from_numpy(x).cuda()
                y, ks = pl.forward(xd) if op == mxfft.FORWARD else pl.roundtrip(xd)
                torch.cuda.synchronize()
                ks = ks.cpu().numpy()
                assert np.array_equal(kb[kbase:kbase + c], ks), "group %d k" % gi
                ok = ks != mxfft.INT32_MIN
                assert np.array_equal(bits(yb[gi].numpy()[ok]), bits(y.cpu().numpy()[ok])), "group %d op %d" % (gi, op)
            kbase += c
        assert kb[sum(c for _, c, _ in groups[:bad]) + groups[bad][1] - 1] == mxfft.INT32_MIN
        for gi in (big[0], 0, len(groups) - 1):
            st, yo, ko = O.transform(xs[gi], op=O.FORWARD if op == mxfft.FORWARD else O.ROUNDTRIP, fmt=O.E4M3, B=32,
                                     nthreads=NTHREADS)
            if gi != bad:
                assert st == O.OK and np.array_equal(bits(yb[gi].numpy()), bits(yo)), "group %d vs oracle" % gi
    b.close()


@pytest.mark.parametrize("n,fmt,block", [(512, "e4m3", 32), (1024, "e5m2", 16), (256, "e4m3", 8), (512, "fp16", 32)])
def test_register_resident_tuning_choices_are_bit_identical(n, fmt, block):
    """The tuned choices of the register-resident passes (Alg. 1 gathered by
    the row pass or read separately, work-groups per slice of that read) give
    the same bits and k; the tuner records its pick."""
    x = synth.kspace_batch(n, 4, 1, 5)
    x[2] *= np.float32(2.0 ** -110)                      # a literal redo under the fused statistics
    xd = torch.from_numpy(x).cuda()
    print("tuning choices: %d^2 %s B=%d" % (n, fmt, block), flush=True)
    with mxfft.Plan(n, 5, fmt=fmt, block=block) as pl:
        y0, k0 = pl.forward(xd)
        y0, k0 = y0.cpu().numpy().copy(), k0.cpu().numpy().copy()
        for stats, chunks in ((1, 0), (1, 1), (1, 4), (0, 16)):
            pl.set_tuning(stats=stats, chunks=chunks)
            assert pl.tuning()["chunks"] == chunks
            y, k = pl.forward(xd)
            assert pl.last_status() == mxfft.OK
            torch.cuda.synchronize()
            assert np.array_equal(bits(y.cpu().numpy()), bits(y0)), (stats, chunks)
            assert np.array_equal(k.cpu().numpy(), k0)
        with pytest.raises(mxfft.MxfftError):
            pl.set_tuning(chunks=3)
    t = mxfft.tune(n, sample=8, force=True, fmt=fmt, block=block)
    assert t["fast"] and t["stats"] in (0, 1) and t["ms"] > 0
