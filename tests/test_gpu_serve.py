"""Serving on the GPU, through the C ABI: results bit-identical alone and in a
mixed stream of requests, admission under a device-memory budget, and a
request with non-finite input failing alone (its neighbours unaffected)."""
import threading

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2512_04317_amd import mxfft, synth  # noqa: E402

pytestmark = pytest.mark.gpu
GiB = 1 << 30


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
        y, k = alone(x, op, **params)
        assert np.array_equal(bits(outs[i].cpu().numpy()), bits(y)), "request %d (%s)" % (i, params)
        if k is not None:
            assert np.array_equal(ks[i].cpu().numpy(), k)
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
    need = max(mxfft.plan_bytes(512, 4, **p) for p in kinds)
    budget = need + need // 2
    srv = mxfft.Server(budget, slots=3)
    xs = [torch.from_numpy(synth.random_complex((3, 512, 512), seed=i, dist="lognormal")).cuda() for i in range(5)]
    outs = [torch.empty_like(x) for x in xs]
    tickets = [srv.submit(x, o, op=mxfft.FORWARD, **p) for x, o, p in zip(xs, outs, kinds)]
    big = torch.empty((64, 512, 512), dtype=torch.complex64, device="cuda")
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
