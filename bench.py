#!/usr/bin/env python3
"""Benchmark of the M2NuFFT hot path on one MI355X.

One step = the whole path for one gapped series: GPSS tapers by the GEP at the
nominal band (validation of t, R(B) = I detected on the lattice, R(A0) by its
quadrature factor, the Gram matrix and its top-K eigen-solve, normalisation
and sign), then the type-1 NuFFT of the K tapered sequences onto the I band
centres fused with the multitaper average P and the suboptimality estimate
Ehat.  Inputs are resident in HBM before the timed region.

Workload (default): 20,480-sample unit grid with periodic 64-of-320 gaps and
5 % random dropouts (N observed ~ 15.5k), AR(2) + 5 sinusoids, f_w = 4/20480,
K = 7, I = 2^18 bands; NuFFT in FP32 at tolerance 1e-6, GEP in FP64.

value = N K I / (seconds per step) / 1e6   (NUDFT-equivalent Mpts*tapers*bands/s)
plus PSDs/s, step latency p50/p99, the NuFFT-only rate, the dominant kernel's
roofline (HIP events on the launch stream over a second timed pass) and the
CPU FP64 oracle timed on a bounded sample of the same workload (all threads
and one thread).  `legs` repeats the step on the FP64 path of the same
workload, on the 256-sample series (FP64) and on the 81,920-sample series
(FP32), each with its parity against the oracle on sampled bands.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# the sources each kernel family is built from: measured HBM traffic of a
# kernel is reported only while the hash of its family's sources matches the
# one recorded with the counters
NUFFT_SOURCES = ["paper_2407_01943_amd/csrc/nufft.hip", "paper_2407_01943_amd/csrc/fft_lds.hpp",
                 "paper_2407_01943_amd/csrc/m2n_common.hpp"]
GEP_SOURCES = ["paper_2407_01943_amd/csrc/gep.hip", "paper_2407_01943_amd/csrc/fft_lds.hpp",
               "paper_2407_01943_amd/csrc/m2n_common.hpp"]
TRAFFIC_FILE = "profiles/hbm_traffic_gapped_20k.md"


def sources_sha256(paths):
    import hashlib
    h = hashlib.sha256()
    for q in paths:
        with open(os.path.join(ROOT, q), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def kernel_sources(kernel):
    """The source family that defines `kernel` (a __global__ function name),
    or None."""
    import re
    pat = re.compile(r"void\s+" + re.escape(kernel) + r"\s*\(")
    for fam in (NUFFT_SOURCES, GEP_SOURCES):
        with open(os.path.join(ROOT, fam[0])) as f:
            if pat.search(f.read()):
                return fam
    return None


# kernels profiled under another kernel's label (same role in the step)
LABEL_OF = {"k_pass2w": "k_pass2"}


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when there is none or the kernel's sources changed since.  Of
    several instances under one label, the one dispatched most often in the
    profiled run (the timed step's own)."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    fam = kernel_sources(kernel)
    if not os.path.exists(path) or fam is None:
        return None
    rec = None
    with open(path) as f:
        for line in f:
            if line.startswith("<!-- traffic "):
                r = json.loads(line[len("<!-- traffic "):].rsplit("-->", 1)[0])
                if r.get("kernel") == kernel and (rec is None or r.get("dispatches", 0) > rec.get("dispatches", 0)):
                    rec = r
    if rec is None or rec.get("sources_sha256") != sources_sha256(fam):
        return None
    return rec["bytes_per_launch"]


def _short(name):
    import re
    name = name.replace("m2n::(anonymous namespace)::", "").replace("void ", "")
    return re.sub(r"\(.*", "", name)


def profile_summary(a):
    """Markdown summaries of rocprofv3 databases: the kernel trace, and the
    HBM bytes per dispatch from FETCH_SIZE and WRITE_SIZE runs calibrated by
    the 256 MiB device copy that --calib-copy performs."""
    import collections
    import sqlite3
    trace_db, fetch_db, write_db = a.profile_summary
    out = []
    con = sqlite3.connect(trace_db)
    durs = collections.defaultdict(list)
    for name, du in con.execute("select name, duration from kernels"):
        durs[_short(name)].append(du)
    out.append(f"# {a.summary_title}\n")
    out.append("Commands (from the repository root on the MI355X; R = repository root):\n")
    out.append("```\n" + a.summary_cmd.replace("\\n", "\n") + "\n```\n")
    out.append("## Kernel trace (rocprofv3 --kernel-trace --stats)\n")
    out.append("| kernel | dispatches | avg us | total us |\n|---|---:|---:|---:|")
    for k, v in sorted(durs.items(), key=lambda kv: -sum(kv[1])):
        out.append(f"| {k} | {len(v)} | {sum(v) / len(v) / 1e3:.2f} | {sum(v) / 1e3:.1f} |")

    def load(db):
        c = sqlite3.connect(db)
        d = collections.defaultdict(list)
        for name, val in c.execute("select name, counter_value from pmc_events"):
            d[_short(name)].append(val)
        return d

    F, W = load(fetch_db), load(write_db)
    calib = 256 * 1024.0   # KiB the copy reads and writes
    cf = calib / max(F["__amd_rocclr_copyBuffer"])
    cw = calib / max(W["__amd_rocclr_copyBuffer"])
    out.append("\n## HBM traffic (rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE)\n")
    out.append(f"Calibration by a 256 MiB device-to-device copy: FETCH_SIZE x {cf:.4f}, "
               f"WRITE_SIZE x {cw:.4f} (counter KiB per dispatch to bytes moved).\n")
    out.append("| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | calibrated MB per dispatch |")
    out.append("|---|---:|---:|---:|---:|")
    recs = []
    for k in sorted(F, key=lambda k: -sum(F[k]) / len(F[k])):
        if k.startswith("__amd"):
            continue
        f = sum(F[k]) / len(F[k])
        w = sum(W.get(k, [0.0])) / max(1, len(W.get(k, [0.0])))
        byts = (f * cf + w * cw) * 1024.0
        out.append(f"| {k} | {len(F[k])} | {f:.1f} | {w:.1f} | {byts / 1e6:.3f} |")
        fam = kernel_sources(k.split("<")[0])
        if fam is not None:
            # records are keyed by the launch's profiling label: the
            # wavefront-row form of pass 2 is profiled as k_pass2
            label = LABEL_OF.get(k.split("<")[0], k.split("<")[0])
            recs.append({"kernel": label, "instance": k, "dispatches": len(F[k]), "bytes_per_launch": round(byts),
                         "fetch_kib": round(f, 1), "write_kib": round(w, 1),
                         "fetch_factor": round(cf, 4), "write_factor": round(cw, 4),
                         "sources_sha256": sources_sha256(fam)})
    out.append("")
    for r in recs:
        out.append("<!-- traffic " + json.dumps(r) + " -->")
    with open(a.summary_out, "w") as f:
        f.write("\n".join(out) + "\n")
    print(f"wrote {a.summary_out}")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="gapped_20k",
                    choices=["gapped_20k", "gapped_82k", "small_gapped"])
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-bands", type=int, default=16384,
                    help="bands in the oracle's timed NUDFT sample")
    ap.add_argument("--batch-series", type=int, default=512,
                    help="series in the batched-form measurement (0: skip)")
    ap.add_argument("--served-seconds", type=float, default=60.0,
                    help="length of the served-form Poisson arrival trace (0: skip)")
    ap.add_argument("--served-rate", type=float, default=200.0, help="arrivals per second")
    ap.add_argument("--gep-stress-n", type=int, default=16384,
                    help="N of the dense jittered GEP stress solve (0: skip)")
    ap.add_argument("--multiband-n", type=int, default=4096,
                    help="samples of the multiband form (0 skips it)")
    ap.add_argument("--no-idpss", action="store_true", help="skip the interpolated-DPSS form")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the other workloads' step legs (FP64 gapped_20k, small_gapped, gapped_82k)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 256 MiB device-to-device copy (byte-counter calibration)")
    ap.add_argument("--profile-summary", nargs=3, metavar=("TRACE_DB", "FETCH_DB", "WRITE_DB"),
                    help="write a markdown summary of rocprofv3 results instead of benchmarking")
    ap.add_argument("--summary-out", default=TRAFFIC_FILE)
    ap.add_argument("--summary-title", default="Kernel trace and HBM traffic")
    ap.add_argument("--summary-cmd", default="")
    return ap.parse_args()


def served_form(m2n, torch, workloads, ctx, rate, seconds):
    """Poisson arrivals through the request queue (continuous batching, FP32
    NuFFT) against the unbatched per-series FP64 path on one stream, same
    arrival trace and requests."""
    import threading
    import numpy as np
    arr = workloads.poisson_arrivals(rate, seconds)
    reqs = [workloads.served_request(r) for r in range(len(arr))]
    n = len(reqs)
    # results (P, Ehat, lambda; the tapers are not returned) are copied from
    # the device straight into pinned host buffers; the request arrays are
    # borrowed until the results are collected (reqs keeps them alive)
    q = m2n.Queue(ctx, prec=m2n.M2N_FP32, pinned_outputs=True, borrow_inputs=True)
    warm = [reqs[0]] + [r for r in reqs if r.I == 2 ** 20][:1]
    for r in warm:
        q.wait(q.submit(r.t, r.x, r.fmax, r.fw, r.K, r.f_lo, r.df, r.I, want_w=False))

    def run_trace(qq, arr_, reqs_, tag):
        # a submitter thread replays the arrivals; this thread collects
        m = len(reqs_)
        tickets = [None] * m
        ready = [threading.Event() for _ in range(m)]
        start = time.perf_counter() + 0.05

        def submitter():
            for i, ta in enumerate(arr_):
                dt = start + ta - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
                r = reqs_[i]
                tickets[i] = qq.submit(r.t, r.x, r.fmax, r.fw, r.K, r.f_lo, r.df, r.I, want_w=False)
                ready[i].set()

        th = threading.Thread(target=submitter)
        th.start()
        lat, bsz, fails = [], [], 0
        for i in range(m):
            ready[i].wait()
            try:
                res = qq.wait(tickets[i])
                lat.append(res["latency_us"] / 1e3)
                bsz.append(res["batch_size"])
            except m2n.M2NError:
                fails += 1
            if (i + 1) % 2000 == 0:
                print(f"bench: {tag} {i + 1}/{m}", file=sys.stderr, flush=True)
        end = time.perf_counter()
        th.join()
        return end - start, np.array(lat), bsz, fails

    wall, lat, bsz, fails = run_trace(q, arr, reqs, "served")
    # saturation: the first requests submitted at once, so that the queue
    # forms batches as fast as the device drains them
    nb = min(n, 2000)
    # output buffers of the burst: views of one pinned pool, made once (a
    # server keeps such a pool and reuses it)
    rdt_t = torch.float32
    # P and E of each request in turn, eigenvalues in a pool of their own,
    # so that the queue copies each kind of a batch back in one piece
    tot = sum(2 * r.I for r in reqs[:nb])
    pool = torch.empty(tot, dtype=rdt_t, pin_memory=True).numpy()
    lam_pool = torch.empty(sum(r.K for r in reqs[:nb]), dtype=torch.float64, pin_memory=True).numpy()
    outs, o, ol = [], 0, 0
    for r in reqs[:nb]:
        outs.append({"P": pool[o:o + r.I], "E": pool[o + r.I:o + 2 * r.I], "lam": lam_pool[ol:ol + r.K],
                     "w": None})
        o += 2 * r.I
        ol += r.K

    def burst(qq, pinned):
        t0_ = time.perf_counter()
        if pinned:
            tks = [qq.submit(r.t, r.x, r.fmax, r.fw, r.K, r.f_lo, r.df, r.I, want_w=False, out=ob)
                   for r, ob in zip(reqs[:nb], outs)]
        else:
            tks = [qq.submit(r.t, r.x, r.fmax, r.fw, r.K, r.f_lo, r.df, r.I) for r in reqs[:nb]]
        res_ = [qq.wait(tk) for tk in tks]
        return time.perf_counter() - t0_, res_

    def bursts(qq, pinned, reps=3):
        # once to warm the slots' arenas, then the median of `reps` timed
        # bursts (single bursts vary with host scheduling)
        burst(qq, pinned)
        runs = sorted((burst(qq, pinned) for _ in range(reps)), key=lambda wr: wr[0])
        return runs[len(runs) // 2][0], runs[len(runs) // 2][1], [nb / wr[0] for wr in runs]

    b_wall, bres, b_all = bursts(q, True)
    q.close()
    # the inputs copied at submit instead of borrowed
    q = m2n.Queue(ctx, prec=m2n.M2N_FP32, pinned_outputs=True)
    c_wall, cres, c_all = bursts(q, True)
    q.close()
    # the same burst with the staging path (any host memory, tapers returned)
    q = m2n.Queue(ctx, prec=m2n.M2N_FP32)
    s_wall, sres, s_all = bursts(q, False)
    q.close()
    # and with an HBM budget of 256 MiB for the requests in flight
    budget = 256 << 20
    q = m2n.Queue(ctx, hbm_budget_bytes=budget, prec=m2n.M2N_FP32, pinned_outputs=True, borrow_inputs=True)
    g_wall, gres, g_all = bursts(q, True)
    q.close()
    print(f"bench: served trace done, burst of {nb} in {b_wall:.2f} s", file=sys.stderr, flush=True)

    # baseline: per-series FP64 GPU path, FIFO on one stream, same arrivals
    dev = torch.device("cuda:0")

    def serve_one(r):
        t = torch.from_numpy(r.t).to(dev)
        x = torch.from_numpy(r.x).to(dev)
        w, lam = m2n.gpss_tapers(ctx, t, r.fmax, r.fw, r.K)
        out = m2n.m2nufft_psd(ctx, t, x, w, lam, r.fmax, r.fw, r.f_lo, r.df, r.I,
                              prec=m2n.M2N_FP64, check=False)
        return lam.cpu(), out["P"].cpu(), out["E"].cpu()

    for r in warm:
        serve_one(r)
    torch.cuda.synchronize()

    def run_baseline(arr_, reqs_, tag):
        blat = []
        b0 = time.perf_counter() + 0.05
        for i, r in enumerate(reqs_):
            dt = b0 + arr_[i] - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            serve_one(r)
            blat.append((time.perf_counter() - (b0 + arr_[i])) * 1e3)
            if (i + 1) % 2000 == 0:
                print(f"bench: {tag} {i + 1}/{len(reqs_)}", file=sys.stderr, flush=True)
        return time.perf_counter() - b0, np.array(blat)

    bwall, blat = run_baseline(arr, reqs, "baseline")
    # a loaded trace: the first requests again at 5,000 arrivals/s for one
    # second, where batching matters (at 200/s the GPU idles between requests)
    lrate, lsec = 5000.0, 1.0
    larr = workloads.poisson_arrivals(lrate, lsec, seed=5)
    nl = min(len(larr), n)
    larr, lreqs = larr[:nl], reqs[:nl]
    q = m2n.Queue(ctx, prec=m2n.M2N_FP32, pinned_outputs=True, borrow_inputs=True)
    for r in warm:
        q.wait(q.submit(r.t, r.x, r.fmax, r.fw, r.K, r.f_lo, r.df, r.I, want_w=False))
    l_wall, l_lat, l_bsz, l_fails = run_trace(q, larr, lreqs, "loaded")
    q.close()
    lb_wall, lb_lat = run_baseline(larr, lreqs, "loaded baseline")
    print(f"bench: loaded trace {nl} requests: queue p99 {np.percentile(l_lat, 99):.2f} ms, "
          f"per series p99 {np.percentile(lb_lat, 99):.2f} ms", file=sys.stderr, flush=True)
    return {"requests": n, "rate_per_s": rate, "seconds": seconds,
            "long_requests": int(sum(r.I == 2 ** 20 for r in reqs)), "failed": fails,
            "psds_per_s": round(n / wall, 1), "latency_ms": {
                "p50": round(float(np.percentile(lat, 50)), 3),
                "p99": round(float(np.percentile(lat, 99)), 3)},
            "mean_batch": round(float(np.mean(bsz)), 2), "max_batch": int(np.max(bsz)),
            "burst": {"requests": nb, "psds_per_s": round(nb / b_wall, 1), "timed_bursts": 3,
                      "psds_per_s_range": [round(min(b_all), 1), round(max(b_all), 1)],
                      "mean_batch": round(float(np.mean([r["batch_size"] for r in bres])), 1),
                      "outputs": "a reused pool of pinned host buffers, P + Ehat + lambda",
                      "inputs": "borrowed until the results are collected"},
            "burst_copied_inputs": {"requests": nb, "psds_per_s": round(nb / c_wall, 1),
                                    "psds_per_s_range": [round(min(c_all), 1), round(max(c_all), 1)],
                                    "mean_batch": round(float(np.mean([r["batch_size"] for r in cres])), 1),
                                    "inputs": "copied at submit"},
            "burst_staged_outputs": {"requests": nb, "psds_per_s": round(nb / s_wall, 1),
                                     "psds_per_s_range": [round(min(s_all), 1), round(max(s_all), 1)],
                                     "mean_batch": round(float(np.mean([r["batch_size"] for r in sres])), 1),
                                     "outputs": "pageable host buffers through a pinned staging "
                                                "block, tapers included"},
            "burst_hbm_budget": {"budget_bytes": budget, "requests": nb, "psds_per_s": round(nb / g_wall, 1),
                                 "psds_per_s_range": [round(min(g_all), 1), round(max(g_all), 1)],
                                 "mean_batch": round(float(np.mean([r["batch_size"] for r in gres])), 1),
                                 "max_batch": int(np.max([r["batch_size"] for r in gres]))},
            "baseline_fp64_per_series": {
                "psds_per_s": round(n / bwall, 1), "latency_ms": {
                    "p50": round(float(np.percentile(blat, 50)), 3),
                    "p99": round(float(np.percentile(blat, 99)), 3)}},
            "loaded": {
                "rate_per_s": lrate, "seconds": lsec, "requests": nl, "failed": l_fails,
                "psds_per_s": round(nl / l_wall, 1),
                "latency_ms": {"p50": round(float(np.percentile(l_lat, 50)), 3),
                               "p99": round(float(np.percentile(l_lat, 99)), 3)},
                "mean_batch": round(float(np.mean(l_bsz)), 2), "max_batch": int(np.max(l_bsz)),
                "baseline_fp64_per_series": {
                    "psds_per_s": round(nl / lb_wall, 1), "latency_ms": {
                        "p50": round(float(np.percentile(lb_lat, 50)), 3),
                        "p99": round(float(np.percentile(lb_lat, 99)), 3)}}}}


def batched_form(m2n, torch, workloads, ctx, nser, reps=5):
    """The 512-series batched form (one m2n_batch_psd call per batch) against
    the per-series calls on the same stream, same series."""
    import numpy as np
    series = [workloads.batched_series(s) for s in range(nser)]
    dev = torch.device("cuda:0")
    specs = []
    for s in series:
        specs.append({"t": torch.from_numpy(s.t).to(dev), "x": torch.from_numpy(s.x).to(dev),
                      "fmax": s.fmax, "fw": s.fw, "K": s.K, "f_lo": s.f_lo, "df": s.df,
                      "I": s.I,
                      "w": torch.empty((s.K, s.N), dtype=torch.float64, device=dev),
                      "lam": torch.empty((s.K,), dtype=torch.float64, device=dev),
                      "P": torch.empty((s.I,), dtype=torch.float32, device=dev),
                      "E": torch.empty((s.I,), dtype=torch.float32, device=dev)})
    work = float(sum(s.N * s.K * s.I for s in series))
    # the descriptor array is built once, like the resident inputs
    prep = m2n.batch_descriptors(specs, prec=m2n.M2N_FP32)
    m2n.m2n_batch_psd(ctx, specs, prec=m2n.M2N_FP32, check=False, prepared=prep)
    torch.cuda.synchronize()
    ctx.check()
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        m2n.m2n_batch_psd(ctx, specs, prec=m2n.M2N_FP32, check=False, prepared=prep)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    tb = float(np.median(times))
    P_batch = [sp["P"].clone() for sp in specs[:8]]
    # per-kernel times of one batch (HIP events inside the library) and the
    # HBM roofline of the two NuFFT passes: every taper's grid of nf FP32
    # complex values is written once by pass 1 and read once by pass 2
    ctx.profile_reset()
    ctx.profile(True)
    m2n.m2n_batch_psd(ctx, specs, prec=m2n.M2N_FP32, check=False, prepared=prep)
    torch.cuda.synchronize()
    ctx.profile(False)
    ks = ctx.profile_read()
    kern = {k: round(v[0], 3) for k, v in sorted(ks.items(), key=lambda kv: -kv[1][0])}
    nf = 1
    while nf < 2 * series[0].I:
        nf *= 2
    grid_bytes = float(sum(s.K for s in series)) * nf * 8
    pts = float(sum(s.N * (4 + 4 + 8 + 4) + s.K * s.N * 8 for s in series))
    roof = []
    for name, byts in (("k_pass1", grid_bytes + pts), ("k_pass2", grid_bytes + 2 * 4 * series[0].I * nser)):
        if name in ks:
            ms = ks[name][0]
            ach = byts / (ms * 1e-3) / 1e9
            roof.append({"kernel": name, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "algorithmic_bytes": byts,
                         "ms": round(ms, 4), "launches": ks[name][1]})

    def per_series():
        for sp in specs:
            m2n.gpss_tapers(ctx, sp["t"], sp["fmax"], sp["fw"], sp["K"], out=(sp["w"], sp["lam"]))
            m2n.m2nufft_psd(ctx, sp["t"], sp["x"], sp["w"], sp["lam"], sp["fmax"], sp["fw"],
                            sp["f_lo"], sp["df"], sp["I"], prec=m2n.M2N_FP32,
                            out=(sp["P"], sp["E"], None), check=False)
    per_series()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per_series()
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    dP = max(float((a.double() - sp["P"].double()).abs().max() / sp["P"].double().abs().max())
             for a, sp in zip(P_batch, specs[:8]))
    # the replayable batch: one HIP graph per batch, NuFFT schedule by the
    # autotuner or the default rule, against the same launches issued eagerly
    replay = {}
    for label, graph, tune in (("graph_tuned", True, True), ("graph_default", True, False),
                               ("eager_tuned", False, True)):
        bspecs = [{k: v for k, v in sp.items() if k not in ("w", "lam", "P", "E")} for sp in specs]
        b = m2n.Batch(ctx, bspecs, prec=m2n.M2N_FP32, graph=graph, tune=tune)
        b.launch()
        torch.cuda.synchronize()
        tt = []
        for _ in range(reps):
            t0 = time.perf_counter()
            b.launch()
            torch.cuda.synchronize()
            tt.append(time.perf_counter() - t0)
        tm = float(np.median(tt))
        inf = b.info()
        dPg = max(float((o["P"].double() - a.double()).abs().max() / a.double().abs().max())
                  for o, a in zip(b.outputs[:8], P_batch))
        b.close()
        replay[label] = {"ms_per_batch": round(tm * 1e3, 3), "psds_per_s": round(nser / tm, 1),
                         "value": round(work / tm / 1e6, 1), "P_rel_vs_batch_psd": dPg,
                         "graph_nodes": inf["graph_nodes"], "tuned": bool(inf["tuned"]),
                         "schedule": {"log2_N1": inf["l1"], "B": inf["B"], "M": inf["M"]}
                         if inf["tuned"] else "default rule",
                         "tuner": {"from_cache": bool(inf["from_cache"]), "candidates": inf["candidates"],
                                   "nufft_ms_default": round(inf["nufft_ms_default"], 4),
                                   "nufft_ms_tuned": round(inf["nufft_ms_tuned"], 4)} if inf["tuned"] else None}
    return {"series": nser, "N_range": [min(s.N for s in series), max(s.N for s in series)],
            "K_range": [min(s.K for s in series), max(s.K for s in series)], "I": series[0].I,
            "ms_per_batch": round(tb * 1e3, 3), "psds_per_s": round(nser / tb, 1),
            "value": round(work / tb / 1e6, 1), "unit": "Mpts*tapers*bands/s",
            "per_series_ms": round(ts * 1e3, 3), "per_series_psds_per_s": round(nser / ts, 1),
            "speedup_vs_per_series": round(ts / tb, 2),
            "batch_vs_per_series_P_rel": dP, "kernels_ms": kern, "roofline_nufft": roof,
            "replayable": replay}


FP64_PEAK_TFLOPS = 78.6
# the NuFFT settings of each precision (the library's defaults at tolerance 0:
# kernel width ceil(-log10 tol) + 1, oversampling 2)
NUFFT_LABEL = {"fp32": "fp32 tol 1e-6 w7 sigma2", "fp64": "fp64 tol 1e-12 w13 sigma2"}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def step_leg(m2n, torch, workloads, ctx, name, prec_name, steps, warmup, oracle_bands=1024):
    """The per-series step (tapers, P and Ehat in one fused call) on one workload and
    precision: step time over `steps` steps queued back to back after `warmup`
    (and the latency of steps run one at a time), and
    P on sampled bands (both ends, uniform draws, the largest-P bands) and
    lambda against the oracle (its own tapers through its direct NUDFT)."""
    import numpy as np
    s = getattr(workloads, name)()
    prec = m2n.M2N_FP32 if prec_name == "fp32" else m2n.M2N_FP64
    dev = torch.device("cuda:0")
    t = torch.from_numpy(s.t).to(dev)
    x = torch.from_numpy(s.x).to(dev)
    w = torch.empty((s.K, s.N), dtype=torch.float64, device=dev)
    lam = torch.empty((s.K,), dtype=torch.float64, device=dev)
    rdt = torch.float32 if prec == m2n.M2N_FP32 else torch.float64
    P = torch.empty((s.I,), dtype=rdt, device=dev)
    E = torch.empty((s.I,), dtype=rdt, device=dev)

    spec = [{"t": t, "x": x, "fmax": s.fmax, "fw": s.fw, "K": s.K, "f_lo": s.f_lo, "df": s.df, "I": s.I,
             "w": w, "lam": lam, "P": P, "E": E}]
    prepared = m2n.batch_descriptors(spec, prec, True, False, False)

    def step():
        m2n.m2n_batch_psd(ctx, spec, prec=prec, prepared=prepared, check=False)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.check()
    # throughput: steps back to back between two synchronisations; latency:
    # one step at a time from an idle device
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    lat = []
    for _ in range(steps):
        t0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    out = {"workload": name, "N": s.N, "K": s.K, "I": s.I, "prec": prec_name,
           "nufft": NUFFT_LABEL[prec_name], "steps": steps, "ms_per_step": round(ms, 4),
           "value": round(s.N * s.K * s.I / (ms * 1e-3) / 1e6, 1), "unit": "Mpts*tapers*bands/s",
           "psds_per_s": round(1e3 / ms, 1),
           "latency_ms": {"p50": round(1e3 * float(np.percentile(lat, 50)), 4),
                          "p99": round(1e3 * float(np.percentile(lat, 99)), 4)}}
    import oracle
    Pg = P.double().cpu().numpy()
    rng = np.random.default_rng(5 + s.N)
    nb = min(oracle_bands, s.I)
    bands = np.unique(np.concatenate([[0, s.I - 1], rng.integers(0, s.I, nb),
                                      np.argsort(Pg)[-min(64, s.I):]])).astype(np.int64)
    w_o, lam_o = oracle.gpss_tapers(s.t, s.fmax, s.fw, s.K)
    P_o = oracle.psd(oracle.nudft(s.t, s.x, w_o, s.f_lo, s.df, bands=bands))
    E_o, _ = oracle.ehat(s.t, w_o, lam_o, s.fmax, s.fw, s.f_lo, s.df, bands=bands[:64]) \
        if s.N <= 4096 else (None, None)
    gate = 1e-5 if prec == m2n.M2N_FP32 else 1e-10
    err = float(np.max(np.abs(Pg[bands] - P_o)) / np.max(P_o))
    par = {"bands": int(bands.size), "P_rel_err": err,
           "lambda_abs_err": float(np.max(np.abs(lam.cpu().numpy() - lam_o))), "gate": gate}
    if E_o is not None:
        par["Ehat_abs_err"] = float(np.max(np.abs(E.double().cpu().numpy()[bands[:64]] - E_o)))
    par["pass"] = bool(err < gate and par["lambda_abs_err"] < 1e-12 and par.get("Ehat_abs_err", 0.0) < gate)
    out["parity"] = par
    return out


def gep_stress(m2n, torch, workloads, ctx, n, reps=3):
    """Dense GEP on a jittered grid t_n = n + z_n, z ~ N(0, 0.1^2): R(B) is a
    dense, well-conditioned matrix, factored by the tiled FP64 Cholesky whose
    trailing updates run on MFMA.  Reports the solve time, the Cholesky's
    flop rate against the FP64 matrix peak and, from dense FP64 products on
    the device, the tapers' R(B)-orthonormality and GEP residual."""
    s = workloads.jitter_stress(n=n)
    dev = torch.device("cuda:0")
    t = torch.from_numpy(s.t).to(dev)
    K = s.K
    w = torch.empty((K, s.N), dtype=torch.float64, device=dev)
    lam = torch.empty((K,), dtype=torch.float64, device=dev)
    m2n.gpss_tapers(ctx, t, s.fmax, s.fw, K, out=(w, lam))       # workspace, tables
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        m2n.gpss_tapers(ctx, t, s.fmax, s.fw, K, out=(w, lam))
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ctx.profile_reset()
    ctx.profile(True)
    m2n.gpss_tapers(ctx, t, s.fmax, s.fw, K, out=(w, lam))
    torch.cuda.synchronize()
    ctx.profile(False)
    ks = ctx.profile_read()
    kern = {k: round(v[0], 3) for k, v in sorted(ks.items(), key=lambda kv: -kv[1][0])[:8]}
    # algorithmic flops: Cholesky N^3/3; its trailing updates (64-wide
    # panels): sum over panels of 64 M (M + 1), M = rows below the panel
    Np = (s.N + 63) // 64 * 64
    chol = s.N ** 3 / 3.0
    syrk = sum(64.0 * M * (M + 1) for M in range(Np - 64, 0, -64))
    syrk_ms = ks.get("k_syrk", (0.0, 1))[0]
    # checks with dense FP64 products (verification only, not the solve)
    tt = t.double()
    tau = tt[:, None] - tt[None, :]

    def sinc_band(f):
        m = torch.sin(2 * math.pi * f * tau) / (math.pi * tau)
        m.fill_diagonal_(2 * f)
        return m

    RB = sinc_band(s.fmax)
    wT = w.T.contiguous()
    RBw = RB @ wT
    del RB
    orth = float((w @ RBw / (2 * s.fw) - torch.eye(K, device=dev, dtype=torch.float64)).abs().max())
    RA = sinc_band(s.fw)
    RAw = RA @ wT
    del RA, tau
    res = float(((RAw - RBw * lam[None, :]).norm(dim=0) / (RBw * lam[None, :]).norm(dim=0)).max())
    del RAw, RBw
    torch.cuda.empty_cache()
    return {"workload": f"jitter_{s.N}", "N": s.N, "K": K, "fw": s.fw, "fmax": s.fmax,
            "ms_per_solve": round(ms, 3), "reps": reps,
            "cholesky_flops": chol, "cholesky_tflops_per_s": round(chol / (ms * 1e-3) / 1e12, 2),
            "frac_fp64_peak": round(chol / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4),
            "k_syrk": {"ms": round(syrk_ms, 3), "flops": syrk,
                       "tflops_per_s": round(syrk / (syrk_ms * 1e-3) / 1e12, 2) if syrk_ms else None,
                       "peak": FP64_PEAK_TFLOPS,
                       "frac": round(syrk / (syrk_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4) if syrk_ms else None},
            "kernels_ms": kern, "lambda": [round(float(v), 12) for v in lam.cpu()],
            "RB_orthonormality": orth, "gep_residual": res}


def multiband_form(m2n, torch, workloads, ctx, n, I, reps=3):
    """The multiband partition on a band-pass sampled series (two sub-bands
    [0, 1/4] and [1/4, 1/2] of f_max = 1/2, nominal centres 1/8 and 3/8):
    per sub-band, the complex taper solve (dense FP64 Cholesky of the
    sub-band matrix, complex Hermitian reduction) and the relative-frequency
    PSD in FP32.  Reports times, the trailing update's FP64 MFMA rate, the
    one-solve kernel times, and from dense FP64 products on the device the
    tapers' R(B^q)-orthonormality and GEP residual."""
    s, sbs = workloads.multiband(n=n, I=I)
    dev = torch.device("cuda:0")
    t = torch.from_numpy(s.t).to(dev)
    x = torch.from_numpy(s.x).to(dev)
    K, N = s.K, s.N
    Np = (N + 63) // 64 * 64
    syrk = sum(64.0 * M * (M + 1) for M in range(Np - 64, 0, -64))
    out = []
    kern_all = {}
    stream = torch.cuda.current_stream()
    for sb in sbs:
        w = torch.empty((2 * K, N), dtype=torch.float64, device=dev)
        lam = torch.empty((K,), dtype=torch.float64, device=dev)
        P = torch.empty((I,), dtype=torch.float32, device=dev)
        m2n.gpss_tapers_subband(ctx, t, sb.fmin, sb.fmax, s.fw, sb.fc0, K, out=(w, lam))
        m2n.m2nufft_psd_subband(ctx, t, x, w, s.f_lo, s.df, I, prec=m2n.M2N_FP32, out=(P, None))
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            m2n.gpss_tapers_subband(ctx, t, sb.fmin, sb.fmax, s.fw, sb.fc0, K, out=(w, lam))
        e1.record(stream)
        torch.cuda.synchronize()
        ms_tap = e0.elapsed_time(e1) / reps
        e0.record(stream)
        for _ in range(10 * reps):
            m2n.m2nufft_psd_subband(ctx, t, x, w, s.f_lo, s.df, I, prec=m2n.M2N_FP32, out=(P, None),
                                    check=False)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_psd = e0.elapsed_time(e1) / (10 * reps)
        ctx.profile_reset()
        ctx.profile(True)
        m2n.gpss_tapers_subband(ctx, t, sb.fmin, sb.fmax, s.fw, sb.fc0, K, out=(w, lam))
        m2n.m2nufft_psd_subband(ctx, t, x, w, s.f_lo, s.df, I, prec=m2n.M2N_FP32, out=(P, None))
        torch.cuda.synchronize()
        ctx.profile(False)
        ks = ctx.profile_read()
        for k, v in ks.items():
            kern_all[k] = kern_all.get(k, 0.0) + v[0]
        syrk_ms = ks.get("k_syrk", (0.0, 1))[0]
        # checks with dense FP64 products (verification only)
        wc = torch.complex(w[:K], w[K:])
        tau = t[:, None] - t[None, :]
        ntau = torch.where(tau == 0, torch.ones_like(tau), tau)
        RB = torch.where(tau == 0, torch.full_like(tau, 2 * (sb.fmax - sb.fmin)),
                         2 * torch.cos(math.pi * (sb.fmax + sb.fmin) * tau)
                         * torch.sin(math.pi * (sb.fmax - sb.fmin) * tau) / (math.pi * ntau))
        RBw = RB.to(torch.complex128) @ wc.T
        del RB
        orth = float((wc.conj() @ RBw / (2 * s.fw) - torch.eye(K, device=dev)).abs().max())
        RA = torch.where(tau == 0, torch.full_like(tau, 2 * s.fw),
                         torch.sin(2 * math.pi * s.fw * tau) / (math.pi * ntau)).to(torch.complex128)
        RA = RA * torch.exp(2j * math.pi * sb.fc0 * tau)
        RAw = RA @ wc.T
        del RA, tau, ntau
        lamc = lam.to(torch.complex128)
        res = float(((RAw - RBw * lamc[None, :]).norm(dim=0) / (RBw * lamc[None, :]).norm(dim=0)).max())
        del RAw, RBw
        torch.cuda.empty_cache()
        out.append({"fmin": sb.fmin, "fmax": sb.fmax, "fc0": sb.fc0,
                    "tapers_ms": round(ms_tap, 3), "psd_ms": round(ms_psd, 4),
                    "psd_value": round(N * K * I / (ms_psd * 1e-3) / 1e6, 1),
                    "k_syrk": {"ms": round(syrk_ms, 3), "flops": syrk,
                               "tflops_per_s": round(syrk / (syrk_ms * 1e-3) / 1e12, 2) if syrk_ms else None,
                               "frac": round(syrk / (syrk_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4)
                               if syrk_ms else None},
                    "k_herm_jacobi_ms": round(ks.get("k_herm_jacobi", (0.0, 1))[0], 4),
                    "lambda": [round(float(v), 12) for v in lam.cpu()],
                    "RB_orthonormality": orth, "gep_residual": res})
    kern = {k: round(v / len(sbs), 4) for k, v in sorted(kern_all.items(), key=lambda kv: -kv[1])[:10]}
    # the sub-bands are independent: all taper solves at once, each on a
    # child context and stream of its own (gpss_tapers_multiband)
    bands = [(sb.fmin, sb.fmax, sb.fc0) for sb in sbs]
    res = m2n.gpss_tapers_multiband(ctx, t, bands, s.fw, K)
    conc = []
    for _ in range(reps):
        torch.cuda.synchronize()
        h0 = time.perf_counter()
        res = m2n.gpss_tapers_multiband(ctx, t, bands, s.fw, K)
        torch.cuda.synchronize()
        conc.append((time.perf_counter() - h0) * 1e3)
    same = all(max(abs(float(a) - b) for a, b in zip(res[i][1].cpu(), out[i]["lambda"])) < 1e-11
               for i in range(len(sbs)))
    return {"workload": s.name, "N": N, "Q": len(sbs), "K": K, "fw": s.fw, "I": I,
            "tapers_multiband_ms": round(min(conc), 3), "tapers_sequential_ms":
            round(sum(o["tapers_ms"] for o in out), 3), "multiband_lambda_ok": same,
            "psd_prec": "fp32", "unit_psd_value": "Mpts*tapers*bands/s (complex tapers)",
            "ms_all_subbands": round(sum(o["tapers_ms"] + o["psd_ms"] for o in out), 3),
            "subbands": out, "kernels_ms_per_subband": kern}


def idpss_form(m2n, torch, workloads, ctx, s_main, reps=5):
    """Interpolated-DPSS tapers (Table 3 step 3 for fc0 = 0) next to the GEP
    branch: on the main workload (a gapped unit grid, so R(B) = I and the
    scale is O(N)) and on the jittered grid of the GEP stress (R(B) dense, the
    scale an O(N^2) FP64 quadratic form).  Reports both solve times, the
    kernel times of one interpolated solve, and the concentration
    w^T R(A0) w / w^T R(B) w of each interpolated taper on the actual grid next
    to the GEP eigenvalues: the suboptimality the paper trades for speed."""
    dev = torch.device("cuda:0")
    out = {}
    for name, s in (("main", s_main), ("jitter", workloads.jitter_stress(n=16384))):
        t = torch.from_numpy(s.t).to(dev)
        K = s.K
        w = torch.empty((K, s.N), dtype=torch.float64, device=dev)
        lam = torch.empty((K,), dtype=torch.float64, device=dev)
        wg = torch.empty_like(w)
        lg = torch.empty_like(lam)
        m2n.idpss_tapers(ctx, t, s.fmax, s.fw, K, out=(w, lam))
        m2n.gpss_tapers(ctx, t, s.fmax, s.fw, K, out=(wg, lg))
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        times = {}
        for label, fn, r in (("idpss", lambda: m2n.idpss_tapers(ctx, t, s.fmax, s.fw, K, out=(w, lam)), reps),
                             ("gep", lambda: m2n.gpss_tapers(ctx, t, s.fmax, s.fw, K, out=(wg, lg)),
                              reps if name == "main" else 1)):
            e0.record(stream)
            for _ in range(r):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            times[label] = e0.elapsed_time(e1) / r
        ctx.profile_reset()
        ctx.profile(True)
        m2n.idpss_tapers(ctx, t, s.fmax, s.fw, K, out=(w, lam))
        torch.cuda.synchronize()
        ctx.profile(False)
        ks = ctx.profile_read()
        # concentration of each interpolated taper on the actual grid,
        # w^T R(A0) w / w^T R(B) w, by dense FP64 products in row chunks
        # (verification only); the GEP tapers reach lambda
        qa = torch.zeros(K, dtype=torch.float64, device=dev)
        qb = torch.zeros(K, dtype=torch.float64, device=dev)
        for r0 in range(0, s.N, 2048):
            tau = t[r0:r0 + 2048, None] - t[None, :]
            ntau = torch.where(tau == 0, torch.ones_like(tau), tau)
            for f, q in ((s.fw, qa), (s.fmax, qb)):
                R = torch.where(tau == 0, torch.full_like(tau, 2 * f),
                                torch.sin(2 * math.pi * f * tau) / (math.pi * ntau))
                q += (w[:, r0:r0 + 2048] * (R @ w.T).T).sum(dim=1)
            del tau, ntau, R
        conc = (qa / qb).cpu().numpy()
        torch.cuda.empty_cache()
        out[name] = {"workload": s.name, "N": s.N, "K": K, "fw": s.fw,
                     "idpss_ms": round(times["idpss"], 4), "gep_ms": round(times["gep"], 4),
                     "kernels_ms": {k: round(v[0], 4) for k, v in sorted(ks.items(), key=lambda kv: -kv[1][0])[:8]},
                     "concentration_idpss": [round(float(v), 9) for v in conc],
                     "lambda_gep": [round(float(v), 9) for v in lg.cpu()]}
    return out


def psd_at_form(m2n, torch, ctx, s, w, n_centres=4096, reps=10):
    """P at an arbitrary list of band centres on the main workload's tapers:
    the direct FP64 summation (time per call and the rate in sample-centre
    pairs per second, each pair one reduced sincos and 2K FMAs) and the
    type-3 NuFFT at the same and at 2^18 centres."""
    import numpy as np
    dev = torch.device("cuda:0")
    t = torch.from_numpy(s.t).to(dev)
    x = torch.from_numpy(s.x).to(dev)
    rng = np.random.default_rng(7)
    freqs = torch.from_numpy(rng.uniform(-0.5, 0.5, n_centres)).to(dev)
    m2n.m2nufft_psd_at(ctx, t, x, w, freqs, check=False)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        m2n.m2nufft_psd_at(ctx, t, x, w, freqs, check=False)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    pairs = float(s.N) * n_centres
    out = {"workload": s.name, "N": s.N, "K": int(w.shape[0]), "centres": n_centres, "ms": round(ms, 4),
           "pairs_per_s": round(pairs / (ms * 1e-3), 1)}
    # the type-3 NuFFT (m2nufft_psd_freqs) at the same and at many more
    # centres; wall time per call (it reads the span back: one round trip)
    t3 = []
    for nc in (n_centres, 2 ** 18):
        fr = torch.from_numpy(np.random.default_rng(8).uniform(-0.5, 0.5, nc)).to(dev)
        for prec in (m2n.M2N_FP32, m2n.M2N_FP64):
            m2n.m2nufft_psd_freqs(ctx, t, x, w, fr, prec=prec, check=False)
            torch.cuda.synchronize()
            tt = []
            for _ in range(reps):
                t0 = time.perf_counter()
                m2n.m2nufft_psd_freqs(ctx, t, x, w, fr, prec=prec, check=False)
                torch.cuda.synchronize()
                tt.append(time.perf_counter() - t0)
            msn = 1e3 * float(np.median(tt))
            t3.append({"centres": nc, "prec": "fp32" if prec == m2n.M2N_FP32 else "fp64",
                       "ms": round(msn, 4), "centres_per_s": round(nc / (msn * 1e-3), 1)})
    out["type3"] = t3
    return out


def algorithmic_bytes(name, s, N, K, I, plan, prec_bytes):
    """Bytes each kernel must move per launch (its compulsory traffic)."""
    cs = 2 * prec_bytes                      # one complex grid value
    nf = plan["nf"]
    if name == "k_pass1":
        # write the K column-transformed grids; read the binned points
        # (cell, offset, FP64 complex pre-phased sample, index) and the FP64
        # tapers, each once
        return K * nf * cs + N * (4 + prec_bytes + 16 + 4) + K * N * 8
    if name == "k_pass2":
        # read the K grids; write P and Ehat
        return K * nf * cs + I * 2 * prec_bytes
    return None


def main():
    a = parse()
    if a.profile_summary:
        profile_summary(a)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                          "(the multi-GPU sharding is described, not built)"}))
        sys.exit(2)
    import numpy as np
    import torch
    import workloads
    import paper_2407_01943_amd as m2n

    s = getattr(workloads, a.workload)()
    prec = m2n.M2N_FP32 if a.prec == "fp32" else m2n.M2N_FP64
    dev = torch.device("cuda:0")
    N, K, I = s.N, s.K, s.I
    print(f"bench: workload={s.name} N={N} K={K} I={I} prec={a.prec}", file=sys.stderr, flush=True)
    ctx = m2n.Context(0)
    t = torch.from_numpy(s.t).to(dev)
    x = torch.from_numpy(s.x).to(dev)
    w = torch.empty((K, N), dtype=torch.float64, device=dev)
    lam = torch.empty((K,), dtype=torch.float64, device=dev)
    rdt = torch.float32 if prec == m2n.M2N_FP32 else torch.float64
    P = torch.empty((I,), dtype=rdt, device=dev)
    E = torch.empty((I,), dtype=rdt, device=dev)
    stream = torch.cuda.current_stream()

    # one step: the fused boundary call (t check, tapers, NuFFT, P and Ehat)
    # on a batch of this one series
    spec = [{"t": t, "x": x, "fmax": s.fmax, "fw": s.fw, "K": K, "f_lo": s.f_lo, "df": s.df, "I": I,
             "w": w, "lam": lam, "P": P, "E": E}]
    prepared = m2n.batch_descriptors(spec, prec, True, False, False)

    def step():
        m2n.m2n_batch_psd(ctx, spec, prec=prec, prepared=prepared, check=False)

    def nufft_only():
        m2n.m2nufft_psd(ctx, t, x, w, lam, s.fmax, s.fw, s.f_lo, s.df, I, prec=prec,
                        want_E=True, out=(P, E, None), check=False)

    if a.calib_copy:
        # a plain copy of known size: the HBM byte counters of the kernel
        # that performs it calibrate the counters of the path's kernels
        src = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    ctx.check()
    print("bench: warmup done", file=sys.stderr, flush=True)

    # ---- timed pass 1: K whole steps back to back on the stream (the call
    # waits for nothing in between, so step i + 1 is queued while step i runs),
    # bracketed by synchronisations: whole-job throughput
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = 1e3 * elapsed / a.steps
    # ---- latency: the same steps one at a time, each from an idle device to
    # its results
    lat = []
    for _ in range(a.steps):
        ts = time.perf_counter()
        step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
    lat_ms = np.array(lat) * 1e3

    # ---- NuFFT + average only (tapers resident), HIP events on the stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(a.steps, 20)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        nufft_only()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_nufft = e0.elapsed_time(e1) / reps
    print(f"bench: step {ms_step:.3f} ms (p50 latency {float(np.percentile(lat_ms, 50)):.3f} ms), "
          f"nufft {ms_nufft:.4f} ms", file=sys.stderr, flush=True)

    # ---- the same with the Thomson F-statistic fused into the average
    Fb = torch.empty((I,), dtype=rdt, device=dev)

    def nufft_ftest():
        m2n.m2nufft_psd(ctx, t, x, w, lam, s.fmax, s.fw, s.f_lo, s.df, I, prec=prec,
                        want_E=True, out=(P, E, None, Fb), check=False)

    nufft_ftest()
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        nufft_ftest()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_nufft_f = e0.elapsed_time(e1) / reps

    # ---- timed pass 2: per-kernel HIP events inside the library
    ctx.profile_reset()
    ctx.profile(True)
    torch.cuda.synchronize()
    for _ in range(a.steps):
        step()
    torch.cuda.synchronize()
    ctx.profile(False)
    kstats = ctx.profile_read()
    per_step = {k: v[0] / a.steps for k, v in kstats.items()}
    dom = max(per_step, key=per_step.get)
    nf = 1
    while nf < 2 * I:
        nf *= 2
    plan = {"nf": nf}
    pb = 4 if prec == m2n.M2N_FP32 else 8
    # roofline of the dominant kernel.  The lattice GEP's eigen-solver
    # (k_sym_topk: one workgroup on the Q x Q quadrature Gram matrix) is
    # FP64 ALU work priced against the chip's FP64 vector peak, with the
    # textbook flop count of a dense symmetric top-K eigenproblem
    # (Householder tridiagonalisation 4/3 Q^3 plus the back-transformation
    # of K vectors 4 Q^2 K), whatever method the kernel uses; HBM-bound
    # kernels are priced by their algorithmic bytes.
    def roof(name):
        ms_k, cnt_k = kstats[name]
        avg = ms_k / cnt_k
        if name.startswith("k_sym_topk"):
            span = float(s.t[-1] - s.t[0])
            Q = math.ceil(0.7 * 2 * math.pi * s.fw * span) + 14
            Q = max(Q, K + 2)
            Q += Q & 1
            fl = 4.0 / 3.0 * Q ** 3 + 4.0 * Q * Q * K
            ach = fl / (avg * 1e-3) / 1e12
            return {"kernel": name, "bound": "alu", "achieved": round(ach, 6),
                    "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(ach / FP64_PEAK_TFLOPS, 8), "traffic": measured_traffic(name),
                    "algorithmic_flops": fl, "Q": Q, "avg_ms": round(avg, 5), "launches": cnt_k,
                    "note": "one workgroup of four wavefronts (4 of 1024 SIMDs): latency of the serial eigen-solve"}
        byts = algorithmic_bytes(name, s, N, K, I, plan, pb)
        ach = byts / (avg * 1e-3) / 1e9
        tr = measured_traffic(name)
        return {"kernel": name, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": tr,
                "algorithmic_bytes": byts, "avg_ms": round(avg, 5), "launches": cnt_k}

    roofline = roof(dom) if (dom.startswith("k_sym_topk") or dom in ("k_pass1", "k_pass2")) else None
    roofline_nufft = [roof(k) for k in ("k_pass1", "k_pass2") if k in kstats]

    # ---- parity gate and CPU baseline (oracle, bounded sample)
    cpu = None
    parity = None
    if not a.no_cpu_baseline:
        import oracle
        nb = min(a.cpu_bands, I)
        bands = np.linspace(0, I - 1, nb).round().astype(np.int64)
        tc0 = time.perf_counter()
        w_o, lam_o = oracle.gpss_tapers(s.t, s.fmax, s.fw, K)
        tc1 = time.perf_counter()
        J_o = oracle.nudft(s.t, s.x, w_o, s.f_lo, s.df, bands=bands)
        P_o = oracle.psd(J_o)
        tc2 = time.perf_counter()
        t_gep, t_nudft = tc1 - tc0, tc2 - tc1
        t_full = t_gep + t_nudft * I / nb
        # the same on one thread, on a quarter of the bands
        nthreads = oracle.num_threads()
        oracle.set_threads(1)
        nb1 = max(1, nb // 4)
        tc3 = time.perf_counter()
        oracle.gpss_tapers(s.t, s.fmax, s.fw, K)
        tc4 = time.perf_counter()
        oracle.nudft(s.t, s.x, w_o, s.f_lo, s.df, bands=bands[::4][:nb1])
        tc5 = time.perf_counter()
        oracle.set_threads(nthreads)
        t1_full = (tc4 - tc3) + (tc5 - tc4) * I / nb1
        cpu = {"value": round(N * K * I / t_full / 1e6, 3), "unit": "Mpts*tapers*bands/s",
               "cores": nthreads, "kind": "oracle", "cpu_model": cpu_model(),
               "sample": (f"GEP by Lanczos with the lattice Toeplitz operator on the full series "
                          f"({t_gep:.2f} s) + direct NUDFT and average on {nb} of {I} bands "
                          f"({t_nudft:.2f} s), extrapolated to all bands"),
               "seconds_per_psd": round(t_full, 3),
               "single_thread": {"value": round(N * K * I / t1_full / 1e6, 3),
                                 "seconds_per_psd": round(t1_full, 3),
                                 "sample": (f"GEP {tc4 - tc3:.2f} s + NUDFT on {nb1} bands "
                                            f"{tc5 - tc4:.2f} s, extrapolated")}}
        Pg = P.double().cpu().numpy()[bands]
        err = float(np.max(np.abs(Pg - P_o)) / np.max(P_o))
        lam_err = float(np.max(np.abs(lam.cpu().numpy() - lam_o)))
        parity = {"P_rel_err_sampled": err, "lambda_abs_err": lam_err,
                  "gate": 1e-5 if prec == m2n.M2N_FP32 else 1e-10,
                  "pass": bool(err < (1e-5 if prec == m2n.M2N_FP32 else 1e-10))}

    batched = None
    if a.batch_series > 0:
        print("bench: batched form", file=sys.stderr, flush=True)
        batched = batched_form(m2n, torch, workloads, ctx, a.batch_series)
        print(f"bench: batched {batched['ms_per_batch']} ms per {a.batch_series} series",
              file=sys.stderr, flush=True)

    served = None
    if a.served_seconds > 0:
        print("bench: served form", file=sys.stderr, flush=True)
        served = served_form(m2n, torch, workloads, ctx, a.served_rate, a.served_seconds)
        print(f"bench: served p50 {served['latency_ms']['p50']} ms p99 {served['latency_ms']['p99']} ms",
              file=sys.stderr, flush=True)

    stress = None
    if a.gep_stress_n > 0:
        print("bench: GEP stress", file=sys.stderr, flush=True)
        stress = gep_stress(m2n, torch, workloads, ctx, a.gep_stress_n)
        print(f"bench: GEP stress {stress['ms_per_solve']} ms, k_syrk {stress['k_syrk']['tflops_per_s']} TF/s",
              file=sys.stderr, flush=True)

    multiband = None
    if a.multiband_n > 0:
        print("bench: multiband", file=sys.stderr, flush=True)
        multiband = multiband_form(m2n, torch, workloads, ctx, a.multiband_n, 2 ** 15)
        print(f"bench: multiband {multiband['ms_all_subbands']} ms for {multiband['Q']} sub-bands",
              file=sys.stderr, flush=True)

    idpss = None
    if not a.no_idpss:
        print("bench: interpolated DPSS", file=sys.stderr, flush=True)
        idpss = idpss_form(m2n, torch, workloads, ctx, s)
        print(f"bench: idpss {idpss['main']['idpss_ms']} ms (GEP {idpss['main']['gep_ms']} ms) on {s.name}",
              file=sys.stderr, flush=True)

    print("bench: band-centre list", file=sys.stderr, flush=True)
    wl = torch.empty((s.K, s.N), dtype=torch.float64, device=torch.device("cuda:0"))
    ll = torch.empty((s.K,), dtype=torch.float64, device=torch.device("cuda:0"))
    m2n.gpss_tapers(ctx, torch.from_numpy(s.t).cuda(), s.fmax, s.fw, s.K, out=(wl, ll))
    psd_at = psd_at_form(m2n, torch, ctx, s, wl)
    print(f"bench: band-centre list {psd_at['ms']} ms for {psd_at['centres']} centres", file=sys.stderr, flush=True)

    legs = []
    if not a.no_legs:
        for wl, pr, st_, wu in (("gapped_20k", "fp64", 20, 5), ("small_gapped", "fp64", 50, 10),
                                ("gapped_82k", "fp32", 10, 3)):
            print(f"bench: leg {wl} {pr}", file=sys.stderr, flush=True)
            legs.append(step_leg(m2n, torch, workloads, ctx, wl, pr, st_, wu))
            print(f"bench: leg {wl} {pr} {legs[-1]['ms_per_step']} ms per step, "
                  f"parity {legs[-1]['parity']['pass']}", file=sys.stderr, flush=True)

    value = N * K * I / (ms_step * 1e-3) / 1e6
    line = {
        "metric": "tapered NuFFT Mpts*tapers*bands/s + PSDs/s at 1e-5 rel err; p50/p99 latency",
        "value": round(value, 3),
        "unit": "Mpts*tapers*bands/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == m2n.M2N_FP32 else "f64",
        "data": "synthetic",
        "config": {"workload": s.name, "N": N, "grid_len": s.grid_len, "K": K, "I": I,
                   "fw": s.fw, "fmax": s.fmax, "nufft": NUFFT_LABEL[a.prec],
                   "gep": "fp64"},
        "psds_per_s": round(1e3 / ms_step, 2),
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 4),
                       "p99": round(float(np.percentile(lat_ms, 99)), 4)},
        "ftest": {"nufft_ms_with_F": round(ms_nufft_f, 5),
                  "extra_ms": round(ms_nufft_f - ms_nufft, 5),
                  "note": "Thomson F-statistic fused into the band average (pass 2)"},
        "nufft_only": {"ms": round(ms_nufft, 5),
                       "value": round(N * K * I / (ms_nufft * 1e-3) / 1e6, 1),
                       # bytes the NuFFT cannot avoid (read t, x and the K
                       # tapers once, write P and Ehat once) over its time:
                       # how far the two-pass grid round trip is from them
                       "compulsory": {"bytes": N * (8 + 8 + 8 * K) + I * 2 * (4 if a.prec == "fp32" else 8),
                                      "GB_per_s": round((N * (8 + 8 + 8 * K) + I * 2 * (4 if a.prec == "fp32" else 8))
                                                        / (ms_nufft * 1e-3) / 1e9, 1),
                                      "frac_of_8TBps": round((N * (8 + 8 + 8 * K) + I * 2 * (4 if a.prec == "fp32" else 8))
                                                             / (ms_nufft * 1e-3) / 8e12, 5)}},
        "kernels_ms_per_step": {k: round(v, 5) for k, v in sorted(per_step.items(), key=lambda kv: -kv[1])},
        "dominant_kernel": dom,
        "roofline": roofline,
        "roofline_nufft": roofline_nufft,
        "cpu_baseline": cpu,
        "parity": parity,
        "batched_form": batched,
        "served_form": served,
        "gep_stress": stress,
        "multiband": multiband,
        "idpss": idpss,
        "psd_at": psd_at,
        "legs": legs,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
