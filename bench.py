"""Benchmark of the k-center hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-mrg]

Workload (one "step"): Gonzalez's traversal with k = 1000 on n = 1,000,000
synthetic integer-grid points in d = 10 (five coordinates uniform in {1..4},
five in {1..13}, stored FP32), first center 0, through kcenter_gonzalez:
all k steps, the FP64 radius trace and the exact FP64 radius.  The points
are resident in HBM before the timed region.

Prints ONE JSON line: value = n*k distance updates per second over the K
timed steps, plus
  roofline      the dominant kernel (live HIP-event timing from the library,
                on the stream it launches on) against its MI355X peak;
  cpu_baseline  the FP64 oracle on the host cores, 1 thread and all cores;
  configs       the other workloads: c1 (Gonzalez, 20,000 uniform 2-D
                points, k = 20: microseconds per call), c2_k100 (the step's
                workload at k = 100), c4_assign (the n x k assignment of the
                5,000,000 x 41 workload against its BF16 MFMA peak), c5_batch
                (the 256-instance mixed batch);
  mrg           two-round MRG on n = 8,000,000, d = 16, m = 64 Dirichlet
                partitions, k = 200: FP32 vs BF16+rescore wall time and
                whether the centers agree;
  gon_bf16      Gonzalez k = 500 on the 5,000,000 x 41 workload, FP32 vs
                BF16 stream + exact FP32 rescoring.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP32_PEAK_TFLOPS = 157.3     # MI355X FP32 vector peak (dense)
BF16_MFMA_PEAK_TFLOPS = 2500.0
FP32_MFMA_PEAK_TFLOPS = 157.3
# VALU issue ceiling of MI355X: the FP32 vector peak of 157.3 TFLOP/s is
# 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz FMA lane-operations x 2 flop, so
# one FP32 VALU instruction retires at most 32 lanes per cycle per SIMD
# (measured: sub/FMA distance chains reach 0.75 of this with 8 waves per
# SIMD, 0.57 with 2).  Reported beside the FLOP fraction.
VALU_PEAK_TOPS = 256 * 4 * 32 * 2.4e9 / 1e12
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--k", type=int, default=1000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mrg", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip configs 1, 2 (k = 100), 4's assignment and 5")
    ap.add_argument("--engine", choices=["auto", "stream"], default="auto")
    ap.add_argument("--mrg-only", action="store_true",
                    help="only the MRG FP32 vs BF16 comparison")
    ap.add_argument("--eim-study", action="store_true",
                    help="EIM's runtime / solution trade-off over phi and k on "
                         "Gaussian data (n = 200,000, 25 clusters) and exit")
    ap.add_argument("--quality-sweep", action="store_true",
                    help="covering radius of MRG (m = 50), EIM (eps 0.1, "
                         "phi 6) and Gonzalez over k on the Unif / Gau / UnB "
                         "graph types and exit")
    ap.add_argument("--batch-only", action="store_true",
                    help="time kcenter_batch on the 256-instance mixed batch "
                         "(GON / MRG / EIM, d in {2, 8, 32}) and exit")
    ap.add_argument("--assign-only", action="store_true",
                    help="time config 4's assignment (5,000,000 x 41 points, "
                         "500 centers) in FP32 and BF16 and exit")
    ap.add_argument("--copy-probe", action="store_true",
                    help="copy 1 GiB device-to-device 5 times (calibrates "
                         "the FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def copy_probe():
    import torch
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    # read-only reference: torch's sum over the same 1 GiB
    acc = src.sum()
    e0.record()
    for _ in range(5):
        acc = src.sum()
    e1.record()
    torch.cuda.synchronize()
    ms_r = e0.elapsed_time(e1) / 5
    print(json.dumps({"copy_probe_bytes_read": nbytes,
                      "copy_probe_bytes_written": nbytes, "launches": 5,
                      "ms_per_copy": ms,
                      "copy_GBps": 2 * nbytes / (ms * 1e-3) / 1e9,
                      "ms_per_sum": ms_r,
                      "sum_read_GBps": nbytes / (ms_r * 1e-3) / 1e9}))


def kernel_source_hash(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_1604_03228_amd", "csrc", f),
                      "rb").read())
    return h.hexdigest()[:16]


def _median_time(fn, runs=3, cap_s=60.0):
    """Median wall time of `runs` calls (one call when it exceeds cap_s)."""
    ts = []
    for _ in range(runs):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
        if ts[-1] > cap_s:
            break
    return float(np.median(ts)), len(ts)


def cpu_baseline(X, k):
    """The FP64 oracle's Gonzalez on the step's points: on all host cores
    (OpenMP over the per-point update loop) for the full k, and on one thread
    for the first 100 centers (a bounded sample, the paper's sequential
    setting); each the median of 3 runs."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    used = oracle.set_threads(cores)
    dt, runs = _median_time(lambda: oracle.gon(X, k, 0))
    out = {"value": len(X) * k / dt, "unit": "dist-updates/s",
           "cores": used, "kind": "oracle",
           "sample": "full workload (n=%d, d=%d, k=%d), median of %d runs, "
                     "%.2f s each" % (len(X), X.shape[1], k, runs, dt)}
    k1 = min(k, 100)
    oracle.set_threads(1)
    dt1, runs1 = _median_time(lambda: oracle.gon(X, k1, 0))
    out["one_thread"] = {"value": len(X) * k1 / dt1, "unit": "dist-updates/s",
                         "cores": 1,
                         "sample": "n=%d, d=%d, first %d centers, median of %d "
                                   "runs, %.2f s each" % (len(X), X.shape[1],
                                                          k1, runs1, dt1)}
    oracle.set_threads(used)
    return out


def stored_traffic(kernel, workload, sources):
    """HBM bytes per launch measured by the FETCH_SIZE / WRITE_SIZE counters
    (scaled by the copy-probe factor), as recorded in profiles/traffic.json;
    None when absent or when the kernel's sources changed since."""
    try:
        t = json.load(open(PROFILE_TRAFFIC))
        e = t.get(kernel + "|" + workload)
        if e is None or e.get("source_hash") != kernel_source_hash(sources):
            return None
        return e["bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        return None


def bench_mrg(kc, torch, steps):
    """Two-round MRG on the 8,000,000 x 16 Gaussian mixture, m = 64, k = 200.
    `fp32` / `bf16` are the library's paths (round 1 register-resident in
    both when the partitions fit); `*_stream` force the streaming engines
    (option resident = 0), FP32 against BF16 + exact rescoring."""
    from paper_1604_03228_amd import workloads as W
    X, off = W.config3()
    Xd = torch.from_numpy(X).cuda()
    B = torch.from_numpy(W.to_bf16_rne(X).view(np.int16)).cuda()
    k = W.CONFIG3["k"]
    out = {}
    cents = {}
    for mode in ("fp32", "bf16", "fp32_stream", "bf16_stream"):
        h = kc.Handle(resident=not mode.endswith("_stream"))
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            bf = B if mode.startswith("bf16") else None
            for _ in range(2):
                r = kc.mrg(Xd, off, k, bf16=bf, handle=h)
            st.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(steps):
                r = kc.mrg(Xd, off, k, bf16=bf, handle=h)
            e1.record(st)
            st.synchronize()
        out[mode + "_ms"] = e0.elapsed_time(e1) / steps
        cents[mode] = r[0].cpu().numpy()
        out[mode + "_radius"] = float(r[2].item())
        if mode == "bf16_stream":
            out["bf16_rescored_per_step"] = h.counter("bf16_rescored") / k
            out["bf16_listed_per_step"] = h.counter("bf16_listed") / k
        h.close()
    out["same_centers"] = bool(all(np.array_equal(cents["fp32"], c)
                                   for c in cents.values()))
    # Algorithm 1 with its loop: capacity 250,000 points per machine (32
    # blocks of 250,000, then 32 x 200 = 6,400 centers in one last round)
    h = kc.Handle()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        for _ in range(2):
            r = kc.mrg_rounds(Xd, k, 250_000, handle=h)
        st.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(steps):
            r = kc.mrg_rounds(Xd, k, 250_000, handle=h)
        e1.record(st)
        st.synchronize()
    out["rounds_c250000_ms"] = e0.elapsed_time(e1) / steps
    out["rounds_c250000_rounds"] = r[3]
    out["rounds_c250000_radius"] = float(r[2].item())
    h.close()
    out["workload"] = "mrg_gauss50_n8000000_d16_m64_k200"
    # every partition fits the register-resident grid, so round 1 runs the
    # same FP32 resident kernel in both modes: the BF16 comparison proper is
    # the streamed pair
    out["resident_rows_same_kernel"] = True
    out["speedup_bf16"] = out["fp32_ms"] / out["bf16_ms"]
    out["speedup_bf16_stream"] = out["fp32_stream_ms"] / out["bf16_stream_ms"]
    return out


def bench_batch(kc, torch, steps):
    """kcenter_batch on the 256-instance mixed batch: wall time per call with
    the points resident in HBM, and the Gonzalez / MRG-round-1 distance
    updates it performs (EIM instances counted by their final Gonzalez
    only, as a lower bound)."""
    from paper_1604_03228_amd import workloads as W
    insts = W.config5_instances()
    probs = []
    upd = 0
    for inst in insts:
        X, off = W.config5_points(inst)
        pr = dict(X=torch.from_numpy(X).cuda(), algo=inst["algo"], k=inst["k"])
        if off is not None:
            pr["offsets"] = off
            upd += int(sum(min(inst["k"], int(b - a)) * int(b - a)
                           for a, b in zip(off[:-1], off[1:])))
        elif inst["algo"] == "gon":
            upd += inst["n"] * inst["k"]
        if inst["algo"] == "eim":
            pr.update(eps=inst["eps"], phi=inst["phi"], seed=inst["seed"])
        probs.append(pr)
    h = kc.Handle()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        for _ in range(2):
            kc.batch(probs, handle=h)
        st.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(steps):
            kc.batch(probs, handle=h)
        e1.record(st)
        st.synchronize()
    ms = e0.elapsed_time(e1) / steps
    # the same batch planned once (kcenter_batch_plan) and run repeatedly
    plan = kc.BatchPlan(probs, handle=h)
    with torch.cuda.stream(st):
        for _ in range(2):
            plan.run()
        st.synchronize()
        e0.record(st)
        for _ in range(steps):
            plan.run()
        e1.record(st)
        st.synchronize()
    plan_ms = e0.elapsed_time(e1) / steps
    plan.close()
    status = h.device_status()
    h.close()
    eim_pass = bench_eim_pass(kc, torch, insts, probs)
    algos = [i["algo"] for i in insts]
    return {"workload": "batch256_unbalanced_gon_mrg_eim", "ms": ms, "plan_run_ms": plan_ms,
            "eim_pass": eim_pass,
            "instances": len(insts), "gon": algos.count("gon"),
            "mrg": algos.count("mrg"), "eim": algos.count("eim"),
            "points": int(sum(i["n"] for i in insts)),
            "gon_mrg1_updates": upd,
            "gon_mrg1_updates_per_s": upd / (ms * 1e-3), "status": status}


def bench_eim_pass(kc, torch, insts, probs):
    """EIM's distance pass on the batch's largest d = 32 instance, alone on a
    tuned handle: the pass's kernel time (timing spans), the MFMA work it
    does (K padded to 32; three products per pair in the split mode) against
    the peak of the chosen MFMA, and how many candidates needed the canonical
    FP32 refinement and FP64; plus the same counts over every d = 32 EIM
    instance of the batch."""
    big = max((i for i, t in enumerate(insts) if t["algo"] == "eim" and t["d"] == 32),
              key=lambda i: insts[i]["n"])
    pr = probs[big]
    h = kc.Handle()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        for _ in range(2):   # tune, warm
            kc.eim(pr["X"], pr["k"], pr["eps"], pr["phi"], pr["seed"], handle=h)
        st.synchronize()
        h.set_option("timing", 1)
        res = kc.eim(pr["X"], pr["k"], pr["eps"], pr["phi"], pr["seed"], handle=h)
        st.synchronize()
    dist_ms, launches, _ = h.timing_read("eim_dist")
    its = res[4]
    rep = h.tune_report()
    var = [v[0] for key, v in rep.items() if key.startswith("eim/32/")]
    split = bool(var) and var[-1] >= 2
    pairs = sum((it["r_size"] - it["ds_size"]) * it["ds_size"] for it in its)
    flop = 2.0 * pairs * 32 * (3 if split else 1)
    peak = BF16_MFMA_PEAK_TFLOPS if split else FP32_MFMA_PEAK_TFLOPS
    achieved = flop / (dist_ms * 1e-3) / 1e12 if dist_ms > 0 else None
    out = {"workload": "eim_gauss25_n%d_d32_k%d" % (insts[big]["n"], insts[big]["k"]),
           "iterations": len(its), "pairs": pairs, "dist_ms": dist_ms,
           "dist_launches": launches,
           "kernel": "k_mindist_mfma (%s)" % ("split BF16 16x16x32, 3 products" if split
                                               else "FP32 16x16x4"),
           "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak,
                        "unit": "TFLOP/s", "frac": achieved / peak if achieved else None},
           "refined_fp32": h.counter("eim_refined"), "decided_fp64": h.counter("eim_exact")}
    h.close()
    # every d = 32 EIM instance: candidates refined and decided in FP64
    ref = exact = cands = 0
    h = kc.Handle()
    with torch.cuda.stream(st):
        for i, t in enumerate(insts):
            if t["algo"] != "eim" or t["d"] != 32:
                continue
            p = probs[i]
            r = kc.eim(p["X"], p["k"], p["eps"], p["phi"], p["seed"], handle=h)
            st.synchronize()
            ref += h.counter("eim_refined")
            exact += h.counter("eim_exact")
            cands += sum(it["r_size"] - it["ds_size"] for it in r[4])
    h.close()
    out["d32_instances"] = {"candidates": cands, "refined_fp32": ref, "decided_fp64": exact}
    return out


def eim_study(kc, torch, seeds=5):
    """EIM with phi in {1, 4, 6, 8} and k in {2, 5, 10, 25, 50, 100}, eps 0.1,
    on Gaussian data shaped like the paper's parameter study: n = 200,000,
    d = 2, 25 clusters with centers uniform in [0, 100]^2 and sigma 0.1.
    Per (k, phi): mean covering radius, mean wall time per call (the call
    synchronises once per iteration), mean iterations and sample size over
    `seeds` data sets; Gonzalez's radius on the same data for reference."""
    import time
    from paper_1604_03228_amd import workloads as W
    ks = (2, 5, 10, 25, 50, 100)
    phis = (1.0, 4.0, 6.0, 8.0)
    acc = {}
    gon = {k: 0.0 for k in ks}
    h = kc.Handle()
    for sd in range(seeds):
        X = W.points_gauss_mixture(200_000, 2, 25, 0.0, 100.0, 0.1, 0.1, seed=600 + sd)
        Xd = torch.from_numpy(X).cuda()
        for k in ks:
            c, tr, nc = kc.gonzalez(Xd, k, 0, handle=h)
            gon[k] += float(tr[int(nc.item()) - 1].item()) / seeds
            for phi in phis:
                kc.eim(Xd, k, 0.1, phi, 7 * 2**32 + sd, handle=h)   # warm
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                c, nc, r, smp, its = kc.eim(Xd, k, 0.1, phi, 7 * 2**32 + sd,
                                            want_sample=False, handle=h)
                rr = float(r.item())
                dt = time.perf_counter() - t0
                a = acc.setdefault((k, phi), [0.0, 0.0, 0.0, 0.0])
                a[0] += rr / seeds
                a[1] += dt * 1e3 / seeds
                a[2] += len(its) / seeds
                a[3] += (its[-1]["s_size"] if its else 0) / seeds
    h.close()
    rows = [{"k": k, "phi": phi, "radius": v[0], "ms": v[1], "iterations": v[2],
             "sample_S": v[3], "gon_radius": gon[k]}
            for (k, phi), v in sorted(acc.items())]
    return {"workload": "eim_study_gau_n200000_d2_k25clusters_eps0.1",
            "seeds": seeds, "rows": rows}


def quality_sweep(kc, torch, sets=3):
    """The solution-value comparison of the paper's Tables 2-4 on seeded
    stand-ins: for each graph type (Unif n = 100,000; Gau n = 1,000,000 and
    UnB n = 200,000, 25 clusters) and k in {2, 5, 10, 25, 50, 100}, the mean
    covering radius of MRG (m = 50 equal partitions), EIM (eps = 0.1,
    phi = 6; two Philox seeds per data set) and Gonzalez (first center 0)
    over `sets` data sets, with the wall time per call."""
    import time
    from paper_1604_03228_amd import workloads as W
    ks = (2, 5, 10, 25, 50, 100)
    h = kc.Handle()
    out = {}
    for kind in ("gau", "unif", "unb"):
        acc = {}
        for sd in range(sets):
            X = W.quality_points(kind, 900 + sd)
            n = len(X)
            Xd = torch.from_numpy(X).cuda()
            off = W.equal_offsets(n, 50)
            for k in ks:
                runs = [("gon", lambda: kc.gonzalez(Xd, k, 0, handle=h)),
                        ("mrg", lambda: kc.mrg(Xd, off, k, handle=h))]
                for e in range(2):
                    runs.append(("eim", lambda e=e: kc.eim(
                        Xd, k, 0.1, 6.0, 9 * 2**32 + 2 * sd + e,
                        want_sample=False, handle=h)))
                for name, fn in runs:
                    fn()   # warm
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    r = fn()
                    if name == "gon":
                        rad = float(r[1][int(r[2].item()) - 1].item())
                    else:
                        rad = float(r[2].item())
                    dt = (time.perf_counter() - t0) * 1e3
                    a = acc.setdefault((k, name), [0.0, 0.0, 0])
                    a[0] += rad
                    a[1] += dt
                    a[2] += 1
        rows = []
        for k in ks:
            row = {"k": k}
            for name in ("mrg", "eim", "gon"):
                a = acc[(k, name)]
                row[name] = a[0] / a[2]
                row[name + "_ms"] = a[1] / a[2]
            row["mrg_over_gon"] = row["mrg"] / row["gon"]
            row["eim_over_gon"] = row["eim"] / row["gon"]
            rows.append(row)
        out[kind] = {"n": int(W.QUALITY_SETS[kind]), "sets": sets, "rows": rows}
    h.close()
    return out


def bench_assign(kc, torch, Xd, B, centers, steps):
    """kcenter_assign (labels and exact radius) of every point to `centers`,
    in FP32 and with BF16 MFMA distances: ms per call, and the MFMA distance
    kernel's time from the library's own timing spans."""
    n, d = Xd.shape
    k = centers.numel()
    out = {}
    labs = {}
    for mode, bf in (("bf16", B), ("fp32", None)):
        h = kc.Handle()
        h.set_option("timing", 1)
        st = torch.cuda.Stream()
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            for _ in range(2):
                kc.assign(Xd, centers, bf16=bf, handle=h)
            st.synchronize()
            h.timing_read("assign_mfma")
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(steps):
                lab, rad = kc.assign(Xd, centers, bf16=bf, handle=h)
            e1.record(st)
            st.synchronize()
        kms, kl, _ = h.timing_read("assign_mfma")
        out[mode + "_rescored_fp64"] = h.counter("assign_rescored")
        out[mode + "_ms"] = e0.elapsed_time(e1) / steps
        out[mode + "_mfma_kernel_ms"] = kms / max(kl, 1)
        out[mode + "_radius"] = float(rad.item())
        labs[mode] = lab.cpu().numpy()
        h.close()
    flops = 2.0 * n * k * d
    per = out["bf16_mfma_kernel_ms"]
    ach = flops / (per * 1e-3) / 1e12
    kpad = -(-d // 32) * 32          # BF16 16x16x32 MFMA: K padded to 32
    out.update({"n": n, "k": k, "d": d, "same_labels": bool(
        np.array_equal(labs["bf16"], labs["fp32"])),
        "roofline": {"kernel": "k_mindist_mfma (BF16 16x16x32)", "bound": "mfma",
                     "achieved": ach, "peak": BF16_MFMA_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": ach / BF16_MFMA_PEAK_TFLOPS,
                     "work_per_launch": "2*n*k*d = %.4g flop (%.4g with K "
                                        "padded to %d)" % (flops, 2.0 * n * k * kpad, kpad),
                     "avg_launch_ms": per}})
    return out


def bench_gon_bf16(kc, torch, steps, cfg=None):
    """Gonzalez k=500 on the 5,000,000 x 41 mixed-scale workload, FP32 vs
    BF16 stream + exact FP32 rescoring (same centers required); with `cfg`,
    also the n x k assignment to those centers (cfg["c4_assign"])."""
    from paper_1604_03228_amd import workloads as W
    X, Xb = W.config4()
    Xd = torch.from_numpy(X).cuda()
    B = torch.from_numpy(Xb.view(np.int16)).cuda()
    k = W.CONFIG4["k"]
    out = {"workload": "gon_mixed41_n5000000_k500"}
    cents = {}
    for mode in ("fp32", "bf16"):
        h = kc.Handle()
        st = torch.cuda.Stream()
        bf = B if mode == "bf16" else None
        with torch.cuda.stream(st):
            for _ in range(2):
                r = kc.gonzalez(Xd, k, 0, bf16=bf, handle=h)
            st.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(steps):
                r = kc.gonzalez(Xd, k, 0, bf16=bf, handle=h)
            e1.record(st)
            st.synchronize()
        out[mode + "_ms"] = e0.elapsed_time(e1) / steps
        cents[mode] = r[0].cpu().numpy()
        out[mode + "_radius"] = float(r[1][-1].item())
        if mode == "bf16":
            out["bf16_rescored_per_step"] = h.counter("bf16_rescored") / k
            out["bf16_listed_per_step"] = h.counter("bf16_listed") / k
        h.close()
    out["same_centers"] = bool(np.array_equal(cents["fp32"], cents["bf16"]))
    out["speedup_bf16"] = out["fp32_ms"] / out["bf16_ms"]
    out["dist_updates_per_s_bf16"] = len(X) * k / (out["bf16_ms"] * 1e-3)
    if cfg is not None:
        a = bench_assign(kc, torch, Xd, B, torch.from_numpy(cents["fp32"]).cuda(), steps)
        a["workload"] = "assign_mixed41_n5000000_k500"
        a["radius_matches_gonzalez"] = a["bf16_radius"] == out["fp32_radius"]
        cfg["c4_assign"] = a
    return out


def bench_assign_only(kc, torch, steps):
    """Config 4's assignment alone: the 500 centers of one Gonzalez run on
    the BF16 copy (with rescoring, the FP32 path's centers), then
    bench_assign."""
    from paper_1604_03228_amd import workloads as W
    X, Xb = W.config4()
    Xd = torch.from_numpy(X).cuda()
    B = torch.from_numpy(Xb.view(np.int16)).cuda()
    h = kc.Handle()
    c, _, _ = kc.gonzalez(Xd, W.CONFIG4["k"], 0, bf16=B, handle=h)
    torch.cuda.synchronize()
    h.close()
    a = bench_assign(kc, torch, Xd, B, c, steps)
    a["workload"] = "assign_mixed41_n5000000_k500"
    return a


def time_gon(kc, torch, Xd, k, steps, warmup, resident=True):
    """kcenter_gonzalez on the HBM-resident points Xd, timed over `steps`
    calls on a non-default stream (so the library's HIP graphs apply), with
    the library's own timing spans of the dominant kernel."""
    h = kc.Handle(resident=resident)
    h.set_option("timing", 1)
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    with torch.cuda.stream(st):
        for _ in range(warmup):
            kc.gonzalez(Xd, k, 0, handle=h)
        st.synchronize()
        for name in ("gon_resident", "gon_step", "gon_block"):
            h.timing_read(name)           # drop warm-up spans
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        w0 = time.perf_counter()
        e0.record(st)
        for _ in range(steps):
            kc.gonzalez(Xd, k, 0, handle=h)
        e1.record(st)
        st.synchronize()
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
    nint = h.counter("resident_integer")   # read before the status clears it
    status = h.device_status()
    if status:
        raise SystemExit("device status 0x%x" % status)
    out = {"ms": e0.elapsed_time(e1) / steps, "wall": wall}
    res_ms, res_l, _ = h.timing_read("gon_resident")
    stp_ms, stp_l, _ = h.timing_read("gon_step")
    blk_ms, blk_l, _ = h.timing_read("gon_block")
    if blk_l > 0:
        out.update(engine="k_gon_block", kern_ms=blk_ms, launches=blk_l,
                   sources=["kc_block.hip", "kc_device.h"])
    elif res_l > 0:
        out.update(engine="k_gon_resident", kern_ms=res_ms, launches=res_l,
                   sources=["kc_resident.hip", "kc_device.h"], integer_form=nint > 0)
    else:
        out.update(engine="k_gon_step", kern_ms=stp_ms, launches=stp_l,
                   sources=["kc_gon.hip", "kc_device.h"])
    h.close()
    return out


def gon_roofline(n, d, k, g):
    """Roofline of the dominant Gonzalez kernel.  Register-resident: bound by
    FP32 vector arithmetic, 3d flop per update (a subtraction and a fused
    multiply-add per coordinate) against the 157.3 TFLOP/s FP32 peak, with
    the VALU issue-rate fraction beside it: 2d + 1 instructions per update
    (one integer min) in the canonical form, d + 1 in the resident engine's
    exact-integer form (d fused multiply-adds and the min).  Streamed: bound by HBM, 4d + 8 bytes per point and
    step against 8 TB/s."""
    kern = g["engine"]
    if kern in ("k_gon_resident", "k_gon_block"):
        per = g["kern_ms"] / g["launches"]
        flops = n * k * 3 * d
        ach = flops / (per * 1e-3) / 1e12
        opu = d + 1 if g.get("integer_form") else 2 * d + 1
        ops = n * k * opu
        issue = ops / (per * 1e-3) / 1e12
        roof = {"kernel": kern, "bound": "alu", "achieved": ach,
                "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / FP32_PEAK_TFLOPS,
                "avg_launch_ms": per, "launches": g["launches"],
                "work_per_launch": "%d updates x %d flop" % (n * k, 3 * d),
                "issue_rate": {"achieved": issue, "peak": VALU_PEAK_TOPS,
                               "unit": "T VALU lane-ops/s",
                               "frac": issue / VALU_PEAK_TOPS,
                               "ops_per_update": opu,
                               "form": "exact-integer" if g.get("integer_form") else "canonical"}}
    else:
        per = g["kern_ms"] / g["launches"]
        byt = n * (4 * d + 8)             # read d coords + mind, write mind
        ach = byt / (per * 1e-3) / 1e9
        roof = {"kernel": kern, "bound": "hbm", "achieved": ach,
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS,
                "avg_launch_ms": per, "launches": g["launches"],
                "work_per_launch": "%d points x %d B" % (n, 4 * d + 8)}
    return kern, roof


def bench_c1(kc, torch, W, steps=200):
    """Gonzalez on 20,000 uniform 2-D points, k = 20 (latency-bound: report
    microseconds per call and per step)."""
    X = W.config1()
    Xd = torch.from_numpy(X).cuda()
    g = time_gon(kc, torch, Xd, 20, steps, 10)
    return {"workload": "gon_uniform_n20000_d2_k20", "engine": g["engine"],
            "us_per_call": g["ms"] * 1e3, "us_per_step": g["ms"] * 1e3 / 20,
            "kernel_us_per_call": g["kern_ms"] / steps * 1e3,
            "launches_per_call": g["launches"] / steps,
            "dist_updates_per_s": len(X) * 20 / (g["ms"] * 1e-3)}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py: measures one GPU only (the hot path runs "
              "on a single MI355X); --gpus %d is not supported" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    if a.copy_probe:
        copy_probe()
        return
    import torch
    import paper_1604_03228_amd as kc
    from paper_1604_03228_amd import workloads as W

    if a.eim_study:
        print(json.dumps({"eim_study": eim_study(kc, torch)}))
        return
    if a.quality_sweep:
        print(json.dumps({"quality": quality_sweep(kc, torch)}))
        return
    if a.batch_only:
        print(json.dumps({"batch": bench_batch(kc, torch, max(2, a.steps))}))
        return
    if a.assign_only:
        print(json.dumps({"c4_assign": bench_assign_only(kc, torch, max(2, a.steps))}))
        return
    if a.mrg_only:
        print(json.dumps({"mrg": bench_mrg(kc, torch, max(2, a.steps)),
                          "gon_bf16": bench_gon_bf16(kc, torch, max(2, a.steps))}))
        return

    n, d, k = 1_000_000, 10, a.k
    X = W.config2(n)
    Xd = torch.from_numpy(X).cuda()
    g = time_gon(kc, torch, Xd, k, a.steps, a.warmup, resident=(a.engine == "auto"))
    ms, wall = g["ms"], g["wall"]
    value = n * k / (ms * 1e-3)
    kern, roof = gon_roofline(n, d, k, g)
    roof["traffic"] = stored_traffic(kern, "gon_intgrid_n1000000_d10_k%d" % k,
                                     g["sources"])

    line = {"metric": "n*k dist-updates/s (Gonzalez, 1 GPU)",
            "value": value, "unit": "dist-updates/s", "n_gpus": 1,
            "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms,
            "wall_s": wall, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32",
            "data": "synthetic (seeded integer grid, stands in for the "
                    "Poker Hand schema)",
            "config": {"workload": "gon_intgrid_n1000000_d10_k%d" % k,
                       "n": n, "d": d, "k": k, "first": 0,
                       "engine": kern},
            "roofline": roof}
    cfg = {}
    if not a.no_configs:
        cfg["c1"] = bench_c1(kc, torch, W)
        g100 = time_gon(kc, torch, Xd, 100, a.steps, a.warmup)
        kern100, roof100 = gon_roofline(n, d, 100, g100)
        cfg["c2_k100"] = {"workload": "gon_intgrid_n1000000_d10_k100",
                          "ms": g100["ms"],
                          "dist_updates_per_s": n * 100 / (g100["ms"] * 1e-3),
                          "roofline": roof100}
    del Xd
    if not a.no_mrg:
        try:
            line["mrg"] = bench_mrg(kc, torch, max(2, min(a.steps, 5)))
            line["gon_bf16"] = bench_gon_bf16(kc, torch, max(2, min(a.steps, 5)),
                                              cfg if not a.no_configs else None)
        except kc.KCenterError as e:
            line["mrg"] = {"error": str(e)}
    if not a.no_configs:
        b = bench_batch(kc, torch, 3)
        cfg["c5_batch"] = b
    if cfg:
        line["configs"] = cfg
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline(X, k)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
