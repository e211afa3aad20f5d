"""Serving on the GPU, through the C ABI: results bit-identical to the oracle
and to a single plan, alone, in a mixed stream of requests and when queued
requests share one launch; plans never shared across block sizes (MXFP8 and
MXFP6); admission under a device-memory budget; a request with non-finite
input failing alone (its neighbours unaffected)."""
import os
import threading

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_2512_04317_amd import mxfft, synth  # noqa: E402

pytestmark = pytest.mark.gpu
GiB = 1 << 30
NTHREADS = min(16, os.cpu_count() or 1)
ORC_FMT = {"e4m3": (O.MODE_MX, O.E4M3), "e5m2": (O.MODE_MX, O.E5M2), "e2m3": (O.MODE_MX, O.E2M3),
           "e3m2": (O.MODE_MX, O.E3M2), "fp16": (O.MODE_FP16, O.E4M3), "bf16": (O.MODE_BF16, O.E4M3)}


def oracle_of(x, op, fmt="e4m3", block=32):
    """The oracle's result for a request (default prescale parameters)."""
    mode, f = ORC_FMT[fmt]
    opcode = {mxfft.FORWARD: O.FORWARD, mxfft.INVERSE: O.INVERSE, mxfft.ROUNDTRIP: O.ROUNDTRIP}[op]
    st, y, k = O.transform(x.cpu().numpy(), op=opcode, mode=mode, fmt=f, B=block, nthreads=NTHREADS)
    assert st == O.OK
    return y, (None if op == mxfft.INVERSE else k)


def bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


def alone(x, op, **params):
    """The request's result from a single plan of its own (the reference)."""
    pl = mxfft.Plan(x.shape[1], x.shape[0], **params)
    if op == mxfft.FORWARD:
        y, k = pl.forward(x)
    elif op == mxfft.INVERSE:
        y, k = pl.inverse(x), None
    else:
        y, k = pl.roundtrip(x)
    torch.cuda.synchronize()
    out = (y.cpu().numpy().copy(), None if k is None else k.cpu().numpy().copy())
    pl.close()
    return out


def mixed_requests(count, seed=7):
    rng = np.random.default_rng(seed)
    fmts = [dict(fmt="e4m3", block=32), dict(fmt="e5m2", block=16), dict(fmt="fp16"), dict(fmt="e4m3", block=8)]
    reqs = []
    for i in range(count):
        n = int(rng.choice([32, 64, 128, 256, 512]))
        coils = int(rng.integers(1, 6))
        op = int(rng.choice([mxfft.FORWARD, mxfft.INVERSE, mxfft.ROUNDTRIP]))
        params = fmts[int(rng.integers(len(fmts)))]
        x = torch.from_numpy(synth.random_complex((coils, n, n), seed=100 + i, dist="lognormal")).cuda()
        reqs.append((x, op, params))
    return reqs


def test_serve_mixed_requests_match_alone():
    reqs = mixed_requests(24)
    print("serve: %d mixed requests" % len(reqs), flush=True)
    srv = mxfft.Server(8 * GiB, slots=4)
    outs, ks, tickets = [], [], [None] * len(reqs)

    def submit(lo, hi):
        for i in range(lo, hi):
            x, op, params = reqs[i]
            tickets[i] = srv.submit(x, outs[i], ks[i], op=op, **params)

    for x, op, _ in reqs:
        outs.append(torch.empty_like(x))
        ks.append(torch.full((x.shape[0],), 12345, dtype=torch.int32, device="cuda"))
    # two submitting threads
    th = [threading.Thread(target=submit, args=(0, 12)), threading.Thread(target=submit, args=(12, 24))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    results = [srv.wait(t) for t in tickets]
    st = srv.stats()
    assert st["submitted"] == st["admitted"] == st["completed"] == 24 and st["rejected"] == 0
    assert st["queued"] == 0 and st["in_flight"] == 0
    assert st["peak_plan_bytes"] <= 8 * GiB
    for i, ((x, op, params), r) in enumerate(zip(reqs, results)):
        assert r["status"] == mxfft.OK, (i, r)
        assert r["t_submit_ms"] <= r["t_start_ms"] <= r["t_done_ms"]
        got = bits(outs[i].cpu().numpy())
        y, k = alone(x, op, **params)
        assert np.array_equal(got, bits(y)), "request %d (%s)" % (i, params)
        yo, ko = oracle_of(x, op, **params)
        assert np.array_equal(got, bits(yo)), "request %d (%s) vs oracle" % (i, params)
        if k is not None:
            assert np.array_equal(ks[i].cpu().numpy(), k)
            assert np.array_equal(ks[i].cpu().numpy(), ko)
    with pytest.raises(mxfft.MxfftError):
        srv.wait(tickets[0])                   # answered once
    srv.close()


def test_serve_budget_admission():
    """A budget that holds one plan at a time: five requests that each need a
    plan of their own still all complete, one after another, with eviction of
    the idle plans; the pooled plans never exceed the budget; a request whose
    plan alone exceeds the budget is rejected at submission."""
    kinds = [dict(fmt="fp16"), dict(fmt="bf16"), dict(fmt="fp16", target=64.0), dict(fmt="bf16", target=64.0),
             dict(fmt="fp16", target=32.0)]
    need = max(mxfft.plan_bytes(512, 32, **p) for p in kinds)     # pooled plans hold at least 32 slices
    budget = need + need // 2
    srv = mxfft.Server(budget, slots=3)
    xs = [torch.from_numpy(synth.random_complex((3, 512, 512), seed=i, dist="lognormal")).cuda() for i in range(5)]
    outs = [torch.empty_like(x) for x in xs]
    tickets = [srv.submit(x, o, op=mxfft.FORWARD, **p) for x, o, p in zip(xs, outs, kinds)]
    big = torch.empty((128, 512, 512), dtype=torch.complex64, device="cuda")
    with pytest.raises(mxfft.MxfftError) as e:
        srv.submit(big, big, fmt="fp16")          # its workspace alone is above the budget
    assert e.value.status == mxfft.EBUDGET
    res = [srv.wait(t) for t in tickets]
    st = srv.stats()
    assert st["rejected"] == 1 and st["completed"] == 5 and st["submitted"] == 6
    assert st["peak_plan_bytes"] <= budget
    assert st["plans_created"] == 5 and st["plans_evicted"] == 4
    for x, o, p, r in zip(xs, outs, kinds, res):
        assert r["status"] == mxfft.OK
        y, _ = alone(x, mxfft.FORWARD, **p)
        assert np.array_equal(bits(o.cpu().numpy()), bits(y))
    # one request at a time, in arrival order
    for a, b in zip(res, res[1:]):
        assert b["t_start_ms"] >= a["t_done_ms"]
    srv.close()


def test_serve_nonfinite_request_fails_alone():
    srv = mxfft.Server(4 * GiB, slots=2)
    xs = [torch.from_numpy(synth.random_complex((2, 64, 64), seed=s, dist="lognormal")).cuda() for s in range(3)]
    xs[1][1, 5, 7] = complex(float("nan"), 0.0)
    outs = [torch.empty_like(x) for x in xs]
    tickets = [srv.submit(x, o, op=mxfft.FORWARD, fmt="e4m3", block=32) for x, o in zip(xs, outs)]
    res = [srv.wait(t) for t in tickets]
    assert [r["status"] for r in res] == [mxfft.OK, mxfft.ENONFINITE, mxfft.OK]
    for i in (0, 2):
        y, _ = alone(xs[i], mxfft.FORWARD, fmt="e4m3", block=32)
        assert np.array_equal(bits(outs[i].cpu().numpy()), bits(y))
    srv.close()


@pytest.mark.parametrize("fmt,blocks", [("e2m3", (16, 32)), ("e3m2", (8, 32)), ("e4m3", (16, 32))])
def test_serve_plans_keep_their_block_size(fmt, blocks):
    """Requests of one MX element format that differ only in the block size
    (same n, coil count and prescale parameters) each get a plan of their
    own block size: the second arrives when the first request's plan is idle
    in the pool, and must not be handed it.  Both results against the oracle,
    bit for bit (MXFP6 blocks of 8 run on the generic kernels, 16 and 32 on
    the register-resident passes)."""
    srv = mxfft.Server(4 * GiB, slots=2)
    for b in blocks + blocks[:1]:
        x = torch.from_numpy(synth.random_complex((2, 128, 128), seed=40 + b, dist="lognormal")).cuda()
        out = torch.empty_like(x)
        k = torch.empty(2, dtype=torch.int32, device="cuda")
        print("serve case: %s B=%d" % (fmt, b), flush=True)
        r = srv.wait(srv.submit(x, out, k, op=mxfft.FORWARD, fmt=fmt, block=b))
        assert r["status"] == mxfft.OK
        yo, ko = oracle_of(x, mxfft.FORWARD, fmt=fmt, block=b)
        assert np.array_equal(bits(out.cpu().numpy()), bits(yo)), "%s B=%d" % (fmt, b)
        assert np.array_equal(k.cpu().numpy(), ko)
    st = srv.stats()
    # one plan per block size; the repeat of the first block reuses its plan
    assert st["plans_created"] == len(blocks) and st["completed"] == len(blocks) + 1
    srv.close()


def test_serve_waits_for_input_written_on_the_submitting_stream():
    """The input is produced by a kernel still queued on the submitting torch
    stream when the request is submitted; the request runs after it (its
    stream waits on the event submit() records) and matches the oracle."""
    x0 = torch.from_numpy(synth.random_complex((4, 256, 256), seed=5, dist="lognormal")).cuda()
    x = torch.empty_like(x0)
    out = torch.empty_like(x0)
    srv = mxfft.Server(4 * GiB, slots=2)
    torch.cuda.synchronize()
    torch.cuda._sleep(20_000_000)      # keeps the stream busy for a while before the copy
    x.copy_(x0)
    r = srv.wait(srv.submit(x, out, op=mxfft.FORWARD, fmt="e4m3", block=32))
    assert r["status"] == mxfft.OK
    yo, _ = oracle_of(x0, mxfft.FORWARD)
    assert np.array_equal(bits(out.cpu().numpy()), bits(yo))
    srv.close()


def test_serve_coalesces_queued_requests():
    """Requests queued while admissions are held, then released onto one
    slot: those of the same size, parameters and operation share launches
    (counted), the others run on their own; interleaved, with an in-place
    request, one without k_out and one with a non-finite slice.  Nothing is
    admitted while held.  Every result bit for bit as the request alone and
    as the oracle, k included; the non-finite request fails alone."""
    import time
    srv = mxfft.Server(8 * GiB, slots=1)
    rng = np.random.default_rng(5)
    reqs = []
    for i in range(14):
        coils = int(rng.integers(1, 5))
        x = torch.from_numpy(synth.random_complex((coils, 128, 128), seed=200 + i, dist="lognormal")).cuda()
        op, params = mxfft.FORWARD, dict(fmt="e4m3", block=32)
        if i % 5 == 3:
            op = mxfft.ROUNDTRIP
        if i % 7 == 6:
            params = dict(fmt="e5m2", block=16)
        if i == 9:
            x[coils - 1, 3, 4] = complex(float("inf"), 0.0)
        reqs.append((x, op, params))
    x_ref = [x.clone() for x, _, _ in reqs]
    outs = [x if i == 4 else torch.empty_like(x) for i, (x, _, _) in enumerate(reqs)]   # request 4 in place
    ks = [None if i == 2 else torch.full((x.shape[0],), 777, dtype=torch.int32, device="cuda")
          for i, (x, _, _) in enumerate(reqs)]
    torch.cuda.synchronize()
    print("serve coalescing: %d requests queued while held" % len(reqs), flush=True)
    srv.hold(True)
    tickets = [srv.submit(x, o, k, op=op, **p) for (x, op, p), o, k in zip(reqs, outs, ks)]
    time.sleep(0.05)
    st = srv.stats()
    assert st["admitted"] == 0 and st["queued"] == len(reqs), st
    srv.hold(False)
    res = [srv.wait(t) for t in tickets]
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["in_flight"] == 0 and st["queued"] == 0
    # forward e4m3 (10 requests) and round trip e4m3 (2) share launches
    assert st["coalesced_launches"] >= 2 and st["coalesced_requests"] >= 5, st
    for i, ((_, op, params), r) in enumerate(zip(reqs, res)):
        x0 = x_ref[i]
        if i == 9:
            assert r["status"] == mxfft.ENONFINITE, r
            continue
        assert r["status"] == mxfft.OK, (i, r)
        got = bits(outs[i].cpu().numpy())
        y, k = alone(x0, op, **params)
        assert np.array_equal(got, bits(y)), "request %d" % i
        yo, ko = oracle_of(x0, op, **params)
        assert np.array_equal(got, bits(yo)), "request %d vs oracle" % i
        if ks[i] is not None:
            assert np.array_equal(ks[i].cpu().numpy(), ko), "request %d k" % i
    # a server destroyed while held still runs what it has queued
    srv.hold(True)
    x, op, params = reqs[0]
    out = torch.empty_like(x)
    srv.submit(x_ref[0], out, op=op, **params)
    srv.close()
    y, _ = alone(x_ref[0], op, **params)
    assert np.array_equal(bits(out.cpu().numpy()), bits(y))


def test_serve_quantized_output_requests_share_launches():
    """Requests with the quantised output (MX) queued while held share a
    launch with each other but not with plain requests of the same size:
    each result bit for bit as the oracle's."""
    srv = mxfft.Server(4 * GiB, slots=1)
    xs = [torch.from_numpy(synth.random_complex((c, 256, 256), seed=300 + c, dist="lognormal")).cuda()
          for c in (2, 3, 1, 2)]
    flags = [mxfft.QUANTIZE_OUTPUT, 0, mxfft.QUANTIZE_OUTPUT, 0]
    outs = [torch.empty_like(x) for x in xs]
    srv.hold(True)
    tickets = [srv.submit(x, o, op=mxfft.FORWARD, fmt="e4m3", block=32, flags=f) for x, o, f in zip(xs, outs, flags)]
    srv.hold(False)
    res = [srv.wait(t) for t in tickets]
    st = srv.stats()
    assert st["coalesced_launches"] == 2 and st["coalesced_requests"] == 4, st
    for x, o, f, r in zip(xs, outs, flags, res):
        assert r["status"] == mxfft.OK
        mode, fo = ORC_FMT["e4m3"]
        s2, yo, _ = O.transform(x.cpu().numpy(), mode=mode, fmt=fo, B=32, flags=O.QUANTIZE_OUT if f else 0,
                                nthreads=NTHREADS)
        assert s2 == O.OK
        assert np.array_equal(bits(o.cpu().numpy()), bits(yo))
    srv.close()
