#!/usr/bin/env python3
"""Benchmark of the MX-scaled mixed-precision 2D FFT on one MI355X.

Default workload: 1024 slices (64 slices x 16 coils) of 512 x 512 complex64
synthetic k-space, MXFP8-E4M3 with B = 32, forward transform with the Alg. 1
prescale (T = 2^7, tau = 5 %, tau_min = 2^-6).  A step is one forward call over
the whole resident batch.  Also timed: the plain FP32 form of the same FFT on
the same batch, the other formats of the precision sweep (the other MX element
format, FP16, BF16; forward, slices/s and accuracy against FP64 each), and the
CPU oracle on a bounded sample (host cores), a device copy and rocFFT's FP32
FFT of the same batch (context), one graph launch over an uneven work list
of 128^2..1024^2 slices, a served stream of Poisson-arriving requests, and
Eq. 1's RSS images (SSIM / PSNR / NMSE per format, fused combine timing).

Prints one JSON line (rank 0).  Usage:
    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--workload kspace512_64x16]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MX-FP8 2D FFT slices/s vs FP32 at stated NRMSE; % HBM roofline; p50/p99 latency"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
ALG_BYTES_PER_ELEM = 16.0      # complex64 read once + complex64 written once per transform
# VALU issue rate: 256 compute units x 64 lanes, one lane operation per lane
# and cycle (non-packed FP32 and integer VALU), at the published 2.4 GHz peak
# clock, and at the clock the counters measured for the kernel under this
# load (GRBM_GUI_ACTIVE over its duration, recorded beside the HBM traffic in
# profiles/traffic_<workload>_<format>.json; 2.1 to 2.36 GHz on different
# machines)
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# algorithmic operations per radix-2 butterfly of the MX path: one complex
# product and two complex sums (10 flops) plus the four quantise/dequantise
# operations of Alg. 2 (encode v, encode the product, decode both)
ALG_OPS_PER_BUTTERFLY = 14.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="kspace512_64x16")
    ap.add_argument("--fmt", default="e4m3", choices=["e4m3", "e5m2"])
    ap.add_argument("--block", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip the other formats (E5M2/E4M3, FP16, BF16, FP32)")
    ap.add_argument("--no-context", action="store_true", help="skip the device copy and rocFFT context timings")
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven work list (sizes 128..1024)")
    ap.add_argument("--no-serving", action="store_true", help="skip the served request stream")
    ap.add_argument("--no-rss", action="store_true", help="skip the RSS-image quality and the fused RSS timing")
    ap.add_argument("--no-blocks", action="store_true",
                    help="skip the block-size table (256^2, 32 slices x 8 coils, E4M3/E5M2, B = 8..64)")
    ap.add_argument("--no-small", action="store_true", help="skip the single 64^2 slice (latency, accuracy)")
    ap.add_argument("--cpu-sample", type=int, default=256, help="slices the CPU oracle transforms per run")
    ap.add_argument("--cpu-runs", type=int, default=3, help="timed oracle runs (median reported)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one device copy of the input (known bytes) to scale HBM counters")
    return ap.parse_args()


def kernel_source_sha():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2512_04317_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def timed_steps(fn, steps, warmup, torch):
    """Wall time of `steps` calls after `warmup` untimed ones, bracketed by
    device synchronisation, plus per-step event durations (current stream)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        starts[i].record()
        fn()
        ends[i].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])
    return wall, per


def uneven_workload(seed=20251204):
    """The uneven work list: 512 reconstructions whose sizes follow 4:3:2:1
    over 128^2, 256^2, 512^2, 1024^2 (largest-remainder counts 205, 154, 102,
    51), shuffled, each with U{1..16} coils.  Returns [(n, coils)] in order."""
    rng = np.random.default_rng([seed, 4])
    sizes = [128] * 205 + [256] * 154 + [512] * 102 + [1024] * 51
    rng.shuffle(sizes)
    coils = rng.integers(1, 17, size=len(sizes))
    return list(zip(sizes, coils.tolist()))


def uneven_batch(args, torch, mxfft, synth):
    """One graph launch over the uneven work list, laid out per
    reconstruction: the 512 reconstructions in arrival order, each its coils
    contiguous at its own offset of one pool.  The library runs one branch
    per size over that size's slices (through a per-slice offset table), the
    branches side by side.  Also timed: each size's branch alone (the same
    slices, in a batch of that size only) and the same slices grouped by size
    in the pool, to show what the concurrent branches gain and what the
    per-reconstruction layout costs.  The data: 16 synthetic phantom coil
    slices per size, each use times its own random complex factor (uniform
    phase, amplitude 2^U(-3, 3)), so every slice of the list is distinct."""
    recon = uneven_workload()
    groups, off = [], 0
    for n, c in recon:
        groups.append((n, c, off))
        off += c * n * n
    b = mxfft.Batch(groups, fmt=args.fmt, block=args.block)
    pool = torch.empty(b.pool_elems, dtype=torch.complex64, device="cuda")
    D = 16
    distinct = {n: torch.from_numpy(synth.kspace_batch(n, 4, 1, D)).cuda() for n in (128, 256, 512, 1024)}
    rng = np.random.default_rng([20251205, 4])
    for i, (n, c, o) in enumerate(b.groups):
        idx = torch.tensor([(i + j) % D for j in range(c)], device="cuda")
        f = np.exp(1j * rng.uniform(0, 2 * np.pi, c)) * 2.0 ** rng.uniform(-3, 3, c)
        fac = torch.from_numpy(f.astype(np.complex64)).cuda().view(c, 1, 1)
        pool[o:o + c * n * n].view(c, n, n).copy_(distinct[n].index_select(0, idx) * fac)
    out = torch.empty_like(pool)
    k = torch.empty(b.slices, dtype=torch.int32, device="cuda")
    wall, per = timed_steps(lambda: b.forward(pool, out, k), args.steps, args.warmup, torch)
    assert b.last_status() == mxfft.OK
    elems = sum(n * n * c for n, c, _ in groups)
    sizes = sorted(set(n for n, _, _ in groups))
    tuning = {n: b.group_tuning(next(i for i, g in enumerate(groups) if g[0] == n)) for n in sizes}
    b.close()
    # each size's branch alone (same pool positions), then the sum
    alone = {}
    for n in sizes:
        sub = [g for g in groups if g[0] == n]
        with mxfft.Batch(sub, fmt=args.fmt, block=args.block) as bn:
            kk = torch.empty(bn.slices, dtype=torch.int32, device="cuda")
            w_n, _ = timed_steps(lambda: bn.forward(pool, out, kk), args.steps, args.warmup, torch)
            alone[n] = {"slices": bn.slices, "ms": round(1e3 * w_n / args.steps, 4)}
    # the same slices grouped by size (one contiguous group per size)
    grouped, off = [], 0
    for n in sizes:
        c = sum(cc for nn, cc, _ in groups if nn == n)
        grouped.append((n, c, off))
        off += c * n * n
    with mxfft.Batch(grouped, fmt=args.fmt, block=args.block) as bg:
        pg = torch.empty(bg.pool_elems, dtype=torch.complex64, device="cuda")
        for n, c, o in bg.groups:             # the same slices, in size order
            dst = pg[o:o + c * n * n].view(c, n, n)
            at = 0
            for nn, cc, oo in groups:
                if nn == n:
                    dst[at:at + cc].copy_(pool[oo:oo + cc * n * n].view(cc, n, n))
                    at += cc
        og = torch.empty_like(pg)
        kg = torch.empty(bg.slices, dtype=torch.int32, device="cuda")
        w_g, _ = timed_steps(lambda: bg.forward(pg, og, kg), args.steps, args.warmup, torch)
        del pg, og
    ms = 1e3 * wall / args.steps
    sum_alone = sum(v["ms"] for v in alone.values())
    return {"metric": "slices/s of one graph launch over the uneven work list (per-reconstruction layout)",
            "value": round(sum(c for _, c, _ in groups) * args.steps / wall, 1),
            "unit": "slices/s", "ms_per_step": round(ms, 4),
            "latency_ms": {"p50": round(float(np.percentile(per, 50)), 4), "p99": round(float(np.percentile(per, 99)), 4)},
            "hbm_frac_algorithmic": round(elems * 16.0 * args.steps / wall / (HBM_PEAK_GBS * 1e9), 4),
            "reconstructions": len(recon), "slices": sum(c for _, c, _ in groups),
            "sizes": {str(n): dict(alone[n], tuning=tuning[n]) for n in sizes},
            "sum_of_branches_alone_ms": round(sum_alone, 4),
            "concurrency_gain": round(sum_alone / ms, 3),
            "grouped_by_size_ms": round(1e3 * w_g / args.steps, 4),
            "format": args.fmt, "block": args.block, "direction": "forward",
            "data": "synthetic: 16 phantom coil slices per size, each use with its own random complex factor "
                    "(every slice distinct)"}


def nrmse_psnr(y, ref):
    """Per-slice NRMSE and PSNR of y against ref (both [batch, n, n])."""
    y = y.astype(np.complex128)
    ref = ref.astype(np.complex128)
    b = y.shape[0]
    err = np.linalg.norm((y - ref).reshape(b, -1), axis=1) / np.linalg.norm(ref.reshape(b, -1), axis=1)
    mse = np.mean(np.abs(y - ref) ** 2, axis=(1, 2))
    psnr = 20 * np.log10(np.abs(ref).max(axis=(1, 2)) / np.sqrt(mse))
    return err, psnr


def block_table(args, torch, mxfft, synth):
    """The block-size trade-off (the paper's Table 2, Sec. 4.2) on the
    256^2 workload: 32 slices x 8 coils of synthetic k-space, MXFP8 E4M3 and
    E5M2 at B = 8, 16, 32, 64, forward and round trip, Alg. 1 prescale.
    Per entry: slices/s (one call over the 256 coil slices), the HBM fraction
    of the algorithmic 16 B per element per call, and NRMSE / PSNR against
    FP64 over every slice (forward: numpy's complex128 fft2; round trip: the
    input itself)."""
    w = synth.WORKLOADS["kspace256_32x8"]
    N, batch = w["N"], w["slices"] * w["coils"]
    x = synth.kspace_batch(N, w["config"], w["slices"], w["coils"], workers=min(16, os.cpu_count() or 1))
    ref_f = np.fft.fft2(x.astype(np.complex128))
    xd = torch.from_numpy(x).cuda()
    out = torch.empty_like(xd)
    k = torch.empty(batch, dtype=torch.int32, device="cuda")
    rows = []
    steps = max(5, args.steps // 2)
    for fmt in ("e4m3", "e5m2"):
        for B in (8, 16, 32, 64):
            with mxfft.Plan(N, batch, fmt=fmt, block=B) as pl:
                fast = pl.tuning()["fast"]
                for op, name, ref in ((mxfft.FORWARD, "forward", ref_f), (mxfft.ROUNDTRIP, "roundtrip", x)):
                    fn = (lambda: pl.forward(xd, out=out, k_out=k)) if op == mxfft.FORWARD else \
                         (lambda: pl.roundtrip(xd, out=out, k_out=k))
                    wall, per = timed_steps(fn, steps, args.warmup, torch)
                    assert pl.last_status() == mxfft.OK
                    err, psnr = nrmse_psnr(out.cpu().numpy(), ref)
                    sps = batch * steps / wall
                    rows.append({"format": fmt, "block": B, "direction": name, "register_resident": bool(fast),
                                 "slices_per_s": round(sps, 1), "ms_per_call": round(1e3 * wall / steps, 4),
                                 "hbm_frac_algorithmic": round(sps * N * N * ALG_BYTES_PER_ELEM / (HBM_PEAK_GBS * 1e9), 4),
                                 "nrmse_vs_fp64": {"mean": float("%.4g" % err.mean()), "max": float("%.4g" % err.max())},
                                 "psnr_db_vs_fp64": round(float(psnr.mean()), 2)})
    return {"workload": "kspace256_32x8: %d coil slices (32 x 8) of %dx%d complex64 k-space" % (batch, N, N),
            "reference": "FP64: numpy complex128 fft2 (forward), the input (round trip)", "steps": steps,
            "rows": rows}


def small_slice(args, torch, mxfft, synth):
    """The single 64^2 slice (one coil): latency of one forward call (HIP
    events, many calls), bit parity with the oracle, NRMSE / PSNR against the
    FP64 brute-force DFT, and the oracle's single-threaded time."""
    import oracle
    w = synth.WORKLOADS["kspace64_1x1"]
    N = w["N"]
    x = synth.kspace_batch(N, w["config"], 1, 1)
    xd = torch.from_numpy(x).cuda()
    out = torch.empty_like(xd)
    k = torch.empty(1, dtype=torch.int32, device="cuda")
    with mxfft.Plan(N, 1, fmt="e4m3", block=32) as pl:
        fn = lambda: pl.forward(xd, out=out, k_out=k)   # noqa: E731
        wall, per = timed_steps(fn, 200, 20, torch)
        assert pl.last_status() == mxfft.OK
        y = out.cpu().numpy()
        kern = {}
        pl.profile(True)
        for _ in range(50):
            fn()
        for name, (n, t) in pl.kernel_times().items():
            kern[name] = round(1e3 * t / n, 2)
        pl.profile(False)
    t0 = time.perf_counter()
    st, yo, ko = oracle.transform(x, fmt=oracle.E4M3, B=32, nthreads=1)
    t_orc = time.perf_counter() - t0
    # FP64 brute-force DFT: separable O(N^3) matrix products in complex128
    j = np.arange(N)
    Fm = np.exp(-2j * np.pi * np.outer(j, j) / N)
    ref = Fm @ x[0].astype(np.complex128) @ Fm.T
    err, psnr = nrmse_psnr(y, ref[None])
    return {"workload": "kspace64_1x1: one 64x64 complex64 k-space slice, MXFP8-E4M3 B=32, forward, Alg. 1 prescale",
            "latency_us": {"p50": round(1e3 * float(np.percentile(per, 50)), 2),
                           "p99": round(1e3 * float(np.percentile(per, 99)), 2),
                           "what": "HIP events around one mxfft_forward call, 200 calls"},
            "kernel_us": kern,
            "bit_exact_vs_oracle": bool(st == oracle.OK and np.array_equal(y.view(np.uint32), yo.view(np.uint32))
                                        and int(k.cpu().numpy()[0]) == int(ko[0])),
            "nrmse_vs_fp64_dft": float("%.4g" % err[0]), "psnr_db_vs_fp64_dft": round(float(psnr[0]), 2),
            "oracle_s": round(t_orc, 4), "oracle_threads": 1}


def serving_workload(count, seed=20251204):
    """Requests of the serving workload: Poisson arrivals at 2000 per second
    (seeded exponential gaps), size uniform over 128^2..1024^2, U{1..32}
    coils, forward or round trip 50/50, format E4M3 / E5M2 / FP16 uniform.
    Returns [(t_arrival_s, n, coils, op, fmt)]."""
    rng = np.random.default_rng([seed, 5])
    t = np.cumsum(rng.exponential(1.0 / 2000.0, size=count))
    n = rng.choice([128, 256, 512, 1024], size=count)
    coils = rng.integers(1, 33, size=count)
    op = rng.choice([0, 2], size=count)
    fmt = rng.choice(["e4m3", "e5m2", "fp16"], size=count)
    return [(float(t[i]), int(n[i]), int(coils[i]), int(op[i]), str(fmt[i])) for i in range(count)]


def serving(args, torch, mxfft, synth, count=1000, slots=4, budget=64 << 30):
    """Serve the request stream through mxfft_serve_* and report latency
    (submission to completion seen by the scheduler) and throughput.  Inputs
    are pre-staged device pools (8 distinct synthetic coil slices per size,
    repeated to 32 coils); outputs rotate over 16 device buffers per size.
    The stream runs twice: the first pass warms the plan pool up."""
    reqs = serving_workload(count)
    pools, outs = {}, {}
    for n in (128, 256, 512, 1024):
        d = torch.from_numpy(synth.kspace_batch(n, 5, 1, 8)).cuda()
        pools[n] = d.repeat(4, 1, 1).contiguous()
        outs[n] = [torch.empty_like(pools[n]) for _ in range(16)]
    srv = mxfft.Server(budget, slots=slots)
    slices = sum(c for _, _, c, _, _ in reqs)

    def run(paced):
        tickets = []
        before = srv.stats()
        if not paced:
            srv.hold(True)        # the whole stream queued first: the server's own sustainable rate
        t0 = time.perf_counter()
        for i, (ta, n, c, op, fmt) in enumerate(reqs):
            while paced and time.perf_counter() - t0 < ta:
                pass
            kw = dict(fmt=fmt) if fmt == "fp16" else dict(fmt=fmt, block=args.block)
            tickets.append(srv.submit(pools[n][:c], outs[n][i % 16][:c], op=op, **kw))
        if not paced:
            srv.hold(False)
        res = [srv.wait(t) for t in tickets]
        assert all(r["status"] == mxfft.OK for r in res)
        lat = np.array([r["t_done_ms"] - r["t_submit_ms"] for r in res])
        # from the first submission (paced) or the first start (queued at once) to the last completion
        t_first = min(r["t_submit_ms"] if paced else r["t_start_ms"] for r in res)
        span_s = (max(r["t_done_ms"] for r in res) - t_first) / 1e3
        after = srv.stats()
        return {"p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "mean_ms": round(float(lat.mean()), 3), "slices_per_s": round(slices / span_s, 1),
                "requests_per_s": round(count / span_s, 1),
                # launches that served several queued requests of the same size, format and operation
                "shared_launches": after["coalesced_launches"] - before["coalesced_launches"],
                "requests_in_shared_launches": after["coalesced_requests"] - before["coalesced_requests"]}

    st0 = srv.stats()
    cold = run(True)              # plans created as requests need them
    st1 = srv.stats()
    warm = run(True)              # plan pool warm
    sat = run(False)              # every request submitted at once: the sustainable rate
    st = srv.stats()
    srv.close()
    return {"metric": "p50/p99 latency of Poisson-arriving requests (submission to completion)",
            "p50_ms": warm["p50_ms"], "p99_ms": warm["p99_ms"], "mean_ms": warm["mean_ms"],
            "requests": count, "arrival_rate_per_s": 2000,
            "slices_per_s": warm["slices_per_s"], "requests_per_s": warm["requests_per_s"],
            "cold": dict(cold, plans_created=st1["plans_created"] - st0["plans_created"]),
            "warm": dict(warm, plans_created=st["plans_created"] - st1["plans_created"]),
            "saturated": dict(sat, what="the same 1000 requests all queued (admissions held while submitting), then "
                                         "released: slices/s from the first start to the last completion; latency "
                                         "from submission includes the queueing"),
            "slots": slots, "budget_GB": budget / 2 ** 30, "admitted": st["admitted"], "rejected": st["rejected"],
            "peak_plan_MB": round(st["peak_plan_bytes"] / 2 ** 20, 1), "plans_created": st["plans_created"],
            "plans_evicted": st.get("plans_evicted"),
            "data": "pre-staged device pools; host-to-device transfer excluded"}


def rss_quality(args, torch, mxfft, x, xd, N, recon=8, coils=16):
    """Eq. 1 on RSS images, as the paper reports its quality (Sec. 3): the
    first `recon` reconstructions of the batch (16 coils each), forward and
    round trip, every format; SSIM (GPU kernel) and PSNR / NMSE against the
    FP64 reference image (forward: RSS of numpy's complex128 fft2; round trip:
    RSS of the input itself).  Also the time of the fused forward + RSS over
    the whole batch against the plain forward."""
    n_sl = recon * coils
    xk = x[:n_sl].astype(np.complex128)
    # forward: the k-space coil slices; round trip: the image-domain coil
    # images x_c (their inverse transforms), as Eq. 1 takes them
    xi = np.fft.ifft2(xk).astype(np.complex64)
    inputs = {mxfft.FORWARD: xd[:n_sl], mxfft.ROUNDTRIP: torch.from_numpy(xi).cuda()}
    ref_f = np.sqrt((np.abs(np.fft.fft2(xk)) ** 2).reshape(recon, coils, N, N).sum(axis=1))
    ref_r = np.sqrt((np.abs(xi.astype(np.complex128)) ** 2).reshape(recon, coils, N, N).sum(axis=1))
    refs = {mxfft.FORWARD: ref_f, mxfft.ROUNDTRIP: ref_r}
    refs_d = {k: torch.from_numpy(v.astype(np.float32)).cuda() for k, v in refs.items()}
    out = {}
    # the FP16 round trip uses T = 2^-3 and tau_min = 2^-24: its forward
    # result grows by up to N^2 and overflows half precision at T = 2^7, and on
    # image-domain data Alg. 1's tail term (tau_min over the 5th percentile)
    # would lift the maximum far above T
    kinds = [("e4m3_b%d" % args.block, dict(fmt="e4m3", block=args.block), {}),
             ("e5m2_b%d" % args.block, dict(fmt="e5m2", block=args.block), {}),
             ("e2m3_b%d" % args.block, dict(fmt="e2m3", block=args.block), {}),
             ("e3m2_b%d" % args.block, dict(fmt="e3m2", block=args.block), {}),
             ("fp16", dict(fmt="fp16"), {mxfft.ROUNDTRIP: dict(target=2.0 ** -3, tau_min=2.0 ** -24)}),
             ("bf16", dict(fmt="bf16"), {}), ("fp32", dict(fmt="fp32", flags=mxfft.NO_PRESCALE), {})]
    fin = lambda v, nd: round(float(v), nd) if np.isfinite(v) else None   # noqa: E731
    for name, kw, over in kinds:
        row = {}
        for op, opn in ((mxfft.FORWARD, "forward"), (mxfft.ROUNDTRIP, "roundtrip")):
            pkw = dict(kw, **over.get(op, {}))
            pl = mxfft.Plan(N, n_sl, **pkw)
            img, _ = pl.rss(inputs[op], coils, op=op)
            ss = mxfft.ssim(img, refs_d[op]).cpu().numpy()
            y = img.cpu().numpy().astype(np.float64)
            r = refs[op]
            mse = ((y - r) ** 2).mean(axis=(1, 2))
            psnr = 20 * np.log10(r.max(axis=(1, 2)) / np.sqrt(mse))
            nmse = ((y - r) ** 2).sum(axis=(1, 2)) / (r ** 2).sum(axis=(1, 2))
            row[opn] = {"ssim": fin(ss.mean(), 5), "psnr_db": fin(psnr.mean(), 2), "nmse": fin(nmse.mean(), 6)}
            if over.get(op):
                row[opn]["prescale"] = {"target": pkw["target"], "tau_min": pkw["tau_min"]}
            pl.close()
        if name[:2] == "e4" or name[:2] == "e5" or name[:2] == "e2" or name[:2] == "e3":
            # the fused round trip of the paper's discussion (no re-encode between F and F^-1)
            pl = mxfft.Plan(N, n_sl, flags=mxfft.FUSED_ROUNDTRIP, **kw)
            img, _ = pl.rss(inputs[mxfft.ROUNDTRIP], coils, op=mxfft.ROUNDTRIP)
            ss = mxfft.ssim(img, refs_d[mxfft.ROUNDTRIP]).cpu().numpy()
            y = img.cpu().numpy().astype(np.float64)
            r = refs[mxfft.ROUNDTRIP]
            mse = ((y - r) ** 2).mean(axis=(1, 2))
            row["roundtrip_fused"] = {"ssim": fin(ss.mean(), 5),
                                      "psnr_db": fin((20 * np.log10(r.max(axis=(1, 2)) / np.sqrt(mse))).mean(), 2),
                                      "nmse": fin((((y - r) ** 2).sum(axis=(1, 2)) / (r ** 2).sum(axis=(1, 2))).mean(), 6)}
            pl.close()
        out[name] = row
    # fused combine over the whole batch (64 reconstructions x 16 coils) against the plain forward
    plan = mxfft.Plan(N, xd.shape[0], fmt=args.fmt, block=args.block)
    img = torch.empty((xd.shape[0] // coils, N, N), dtype=torch.float32, device="cuda")
    k = torch.empty(xd.shape[0], dtype=torch.int32, device="cuda")
    wall, _ = timed_steps(lambda: plan.rss(xd, coils, out=img, k_out=k), args.steps, args.warmup, torch)
    plan.close()
    return {"images": recon, "coils": coils, "reference": "FP64 (numpy complex128 fft2; the input for the round trip)",
            "metrics": out,
            "fused_forward_rss": {"ms_per_step": round(1e3 * wall / args.steps, 4),
                                  "value": round(xd.shape[0] * args.steps / wall, 1), "unit": "coil slices/s",
                                  "output_bytes_per_slice": N * N * 4 / coils}}


def apply_tuning(mxfft, plan, n, batch, kw):
    """Run the autotuner for this plan's shape on the batch size and apply its
    pick; returns the choice."""
    t = mxfft.tune(n, sample=batch, force=True, **kw)
    plan.set_tuning(t["lines"], single=t["single"], stats=t["stats"], chunks=t["chunks"])
    return {k: t[k] for k in ("fast", "lines", "single", "stats", "chunks")}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args, x, batch):
    """The CPU oracle (exact MX emulation, one slice per thread) on the first
    cpu_sample slices of the same batch and parameters, timed cpu_runs times;
    the median is reported.  Threads: the host cores this process may use,
    at most 16 (the host cores one GPU is given)."""
    import oracle
    ns = min(args.cpu_sample, batch)
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    nth = max(1, min(16, avail))
    fmt = oracle.E4M3 if args.fmt == "e4m3" else oracle.E5M2
    times = []
    for _ in range(max(1, args.cpu_runs)):
        t0 = time.perf_counter()
        st, _, _ = oracle.transform(x[:ns], fmt=fmt, B=args.block, nthreads=nth)
        times.append(time.perf_counter() - t0)
        assert st == oracle.OK
    dt = float(np.median(times))
    return {"value": round(ns / dt, 3), "unit": "slices/s", "cores": nth, "kind": "oracle",
            "sample": "first %d of %d slices, same input and parameters; median of %d runs (%s s)"
                      % (ns, batch, len(times), ", ".join("%.2f" % t for t in times)),
            "host": {"cpu_model": cpu_model(), "nproc": os.cpu_count(), "affinity": avail}}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the transform runs on one GPU only (--gpus 1). Slices are independent, so a "
              "batch would shard across GPUs with no communication; no multi-GPU path is built.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2512_04317_amd import mxfft, synth

    mxfft.lib()   # fails loudly when the HIP library is not built
    w = synth.WORKLOADS[args.workload]
    N, batch = w["N"], w["slices"] * w["coils"]
    workers = min(16, os.cpu_count() or 1)
    x = synth.kspace_batch(N, w["config"], w["slices"], w["coils"], workers=workers)
    xd = torch.from_numpy(x).cuda()
    out = torch.empty_like(xd)
    kout = torch.empty(batch, dtype=torch.int32, device=xd.device)

    if args.copy_calibration:
        # a plain copy of the whole input: reads and writes exactly batch * N * N * 8 bytes
        out.copy_(xd)
        torch.cuda.synchronize()

    plan = mxfft.Plan(N, batch, fmt=args.fmt, block=args.block)
    # the library's autotuner picks the launch choices for this batch (every
    # choice gives the same bits); its pick is part of the configuration
    tuned = apply_tuning(mxfft, plan, N, batch, dict(fmt=args.fmt, block=args.block))
    fwd = lambda: plan.forward(xd, out=out, k_out=kout)   # noqa: E731
    for _ in range(args.warmup):
        fwd()
    assert plan.last_status() == mxfft.OK
    # which kernel dominates (three profiled steps, every launch timed)
    plan.profile(True)
    for _ in range(3):
        fwd()
    pre = plan.kernel_times()
    plan.profile(False)
    dom = max(pre, key=lambda k: pre[k][1])
    # timed region: only the dominant kernel's launches carry event pairs
    plan.profile(True, roles=[dom])
    wall, per_step = timed_steps(fwd, args.steps, 0, torch)
    ktimes = plan.kernel_times()
    plan.profile(False)
    slices_per_s = batch * args.steps / wall
    ms_per_step = 1e3 * wall / args.steps

    # accuracy of this run against FP64 (numpy), on a sample of slices
    pick = list(range(0, batch, max(1, batch // 16)))[:16]
    y = out[pick].cpu().numpy().astype(np.complex128)
    ref = np.fft.fft2(x[pick].astype(np.complex128))
    errs = np.linalg.norm((y - ref).reshape(len(pick), -1), axis=1) / np.linalg.norm(ref.reshape(len(pick), -1), axis=1)
    mse = np.mean(np.abs(y - ref) ** 2, axis=(1, 2))
    psnr = 20 * np.log10(np.abs(ref).max(axis=(1, 2)) / np.sqrt(mse))

    # Dominant kernel and its roofline against HBM: the transform's
    # algorithmic 16 B per element split over the two passes (the row pass
    # owns the complex64 input read, the column pass the complex64 output
    # write: 8 B per element each) over the launch's event-timed duration.
    # The passes are VALU-bound in fact (counters: VALU busy near 90%), so a
    # VALU view rides beside it: algorithmic operations per launch (14 per
    # butterfly, N^2 L / 2 butterflies per slice and pass) against the lane
    # issue rate at the published and at the measured clock.
    elems = batch * N * N
    logn = N.bit_length() - 1
    alg_ops = {"row_pass": ALG_OPS_PER_BUTTERFLY * batch * N * N * logn / 2,
               "column_pass": ALG_OPS_PER_BUTTERFLY * batch * N * N * logn / 2}
    alg_bytes = {"row_pass": 8.0 * elems, "column_pass": 8.0 * elems, "prescale_stats": 0.0}
    n_dom, t_dom = ktimes[dom]
    avg_s = t_dom / n_dom * 1e-3
    traffic, clock_ghz = None, None
    tfile = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (args.workload, args.fmt))
    if os.path.exists(tfile):
        t = json.load(open(tfile))
        if t.get("source_sha") == kernel_source_sha() and dom in t.get("kernels", {}):
            traffic = t["kernels"][dom]["hbm_bytes_per_launch"]
            clock_ghz = t["kernels"][dom].get("clock_GHz")
    achieved_ops = alg_ops.get(dom, 0.0) / avg_s / 1e12
    achieved_gbs = alg_bytes.get(dom, 0.0) / avg_s / 1e9
    clock_peak = 256 * 64 * clock_ghz * 1e9 / 1e12 if clock_ghz else None
    roofline = {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved_gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                "kernel_avg_ms": round(avg_s * 1e3, 4), "launches_timed": n_dom,
                "alg_bytes_per_launch": alg_bytes.get(dom, 0.0),
                "alg_bytes_per_elem": 8.0, "elems_per_launch": elems,
                "valu": {"achieved": round(achieved_ops, 3), "unit": "Tops/s",
                         "alg_ops_per_launch": alg_ops.get(dom, 0.0),
                         "peak_2.4GHz": round(ALU_PEAK_TOPS, 3), "frac_2.4GHz": round(achieved_ops / ALU_PEAK_TOPS, 4),
                         "clock_GHz_measured": clock_ghz,
                         "peak_measured_clock": round(clock_peak, 3) if clock_peak else None,
                         "frac_measured_clock": round(achieved_ops / clock_peak, 4) if clock_peak else None}}
    kern = {k: {"launches": n, "avg_ms": t / n} for k, (n, t) in pre.items()}
    step_frac = slices_per_s * N * N * ALG_BYTES_PER_ELEM / (HBM_PEAK_GBS * 1e9)

    result = {
        "metric": METRIC, "value": round(slices_per_s, 1), "unit": "slices/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "mxfp8_%s_b%d/f32" % (args.fmt, args.block), "data": "synthetic",
        "config": {"workload": "%s: %d slices (%d x %d coils) of %dx%d complex64 k-space, MXFP8-%s B=%d, "
                               "forward with Alg. 1 prescale" % (args.workload, batch, w["slices"], w["coils"],
                                                                  N, N, args.fmt.upper(), args.block),
                   "n": N, "batch": batch, "format": args.fmt, "block": args.block, "direction": "forward",
                   "tuning": tuned,
                   "prescale": {"target": 128.0, "tau_pct": 5.0, "tau_min": 2.0 ** -6}},
        "roofline": roofline,
        "hbm_frac_whole_step": round(step_frac, 4),
        "latency_ms": {"p50": round(float(np.percentile(per_step, 50)), 4),
                       "p99": round(float(np.percentile(per_step, 99)), 4)},
        "kernels_profiled_steps": {k: {"launches": v["launches"], "avg_ms": round(v["avg_ms"], 4)} for k, v in kern.items()},
        "nrmse_vs_fp64": {"mean": round(float(errs.mean()), 5), "max": round(float(errs.max()), 5)},
        "psnr_db_vs_fp64": round(float(psnr.mean()), 2),
    }

    if not args.no_sweep:
        # Precision sweep on the same batch: the other MXFP8 element format, the
        # MXFP6 elements (register-resident passes, 6-bit codes in 8-bit
        # conversions), the 16-bit forms (literal prescale pass: not
        # scale-equivariant) and plain FP32 (no prescale: its result is
        # scale-equivariant).  Same step count.
        sweep = {"%s_b%d" % (args.fmt, args.block): {
            "value": result["value"], "ms_per_step": result["ms_per_step"],
            "nrmse_vs_fp64": result["nrmse_vs_fp64"], "psnr_db_vs_fp64": result["psnr_db_vs_fp64"]}}
        other = "e5m2" if args.fmt == "e4m3" else "e4m3"
        for name, kw in ((other + "_b%d" % args.block, dict(fmt=other, block=args.block)),
                         ("e2m3_b%d" % args.block, dict(fmt="e2m3", block=args.block)),
                         ("e3m2_b%d" % args.block, dict(fmt="e3m2", block=args.block)),
                         ("fp16", dict(fmt="fp16")), ("bf16", dict(fmt="bf16")),
                         ("fp32", dict(fmt="fp32", flags=mxfft.NO_PRESCALE))):
            pl = mxfft.Plan(N, batch, **kw)
            t_sw = apply_tuning(mxfft, pl, N, batch, kw)
            fn = lambda: pl.forward(xd, out=out, k_out=kout)   # noqa: E731
            wall_f, _ = timed_steps(fn, args.steps, args.warmup, torch)
            assert pl.last_status() == mxfft.OK, name
            yf = out[pick].cpu().numpy().astype(np.complex128)
            ef = np.linalg.norm((yf - ref).reshape(len(pick), -1), axis=1) / np.linalg.norm(ref.reshape(len(pick), -1), axis=1)
            msef = np.mean(np.abs(yf - ref) ** 2, axis=(1, 2))
            psf = 20 * np.log10(np.abs(ref).max(axis=(1, 2)) / np.sqrt(msef))
            sweep[name] = {"value": round(batch * args.steps / wall_f, 1), "ms_per_step": round(1e3 * wall_f / args.steps, 4),
                           "nrmse_vs_fp64": {"mean": float("%.4g" % ef.mean()), "max": float("%.4g" % ef.max())},
                           "psnr_db_vs_fp64": round(float(psf.mean()), 2), "tuning": t_sw}
            pl.close()
        result["precision_sweep"] = {"unit": "slices/s", "direction": "forward", "formats": sweep}
        result["speedup_vs_fp32"] = round(slices_per_s / sweep["fp32"]["value"], 3)

    if not args.no_context:
        # Context, not the product: a device copy of the batch (measured HBM
        # bandwidth) and the FP32 C2C FFT of the vendor library (torch.fft on
        # ROCm calls rocFFT) on the same batch.
        wall_c, _ = timed_steps(lambda: out.copy_(xd), args.steps, args.warmup, torch)
        copy_gbs = 2.0 * xd.numel() * 8 * args.steps / wall_c / 1e9
        wall_r, _ = timed_steps(lambda: torch.fft.fft2(xd, out=out), args.steps, args.warmup, torch)
        result["context"] = {
            "device_copy": {"GB_per_s": round(copy_gbs, 1), "frac_of_peak": round(copy_gbs / HBM_PEAK_GBS, 4),
                            "what": "out.copy_(in) of the 2 GiB batch: read + write"},
            "rocfft_fp32_c2c": {"value": round(batch * args.steps / wall_r, 1), "unit": "slices/s",
                                "ms_per_step": round(1e3 * wall_r / args.steps, 4),
                                "what": "torch.fft.fft2 (rocFFT) on the same batch, FP32"}}

    if not args.no_rss:
        result["rss"] = rss_quality(args, torch, mxfft, x, xd, N)

    if not args.no_blocks:
        result["block_table"] = block_table(args, torch, mxfft, synth)

    if not args.no_small:
        result["small_64"] = small_slice(args, torch, mxfft, synth)

    if not args.no_uneven:
        result["uneven_batch"] = uneven_batch(args, torch, mxfft, synth)

    if not args.no_serving:
        result["serving"] = serving(args, torch, mxfft, synth)

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(args, x, batch)
    plan.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
