"""Throughput of the (T) correction on one MI355X.

One step is one whole (T) job on the synthetic o=40, v=400, naux=1200
workload with the inputs already in HBM: staging from the factors
(integral assembly, padded layouts, precision copies), the W build over every
occupied triple, the fused V/D/energy consumer and the reductions, ending
with E(T) on the host. FP64 is the headline and runs the whole job. FP32 and
the split-BF16 modes run the same step over a fixed leading slice of the
triple list (--secondary-frac, default 10%) and report |dE(T)| against the
FP64 partials of the same triples.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precisions fp64,fp32,...]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "(T) TFLOP/s at o=40,v=400 FP64 vs FP32/split; jobs/s + p99; |dE| vs FP64"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0, "bf16x2": 2500.0, "fp16x2": 2500.0}
ISSUED = {"fp64": 1, "fp32": 1, "bf16x3": 6, "bf16x2": 3, "fp16x2": 3}   # MFMA products per algorithmic one


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def wbuild_source_hash() -> str:
    """First 16 hex digits of the SHA-256 over the W-build sources (shared
    device header, then the kernel file)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("te_device.h", "te_wbuild.hip"):
        h.update(open(os.path.join(ROOT, "paper_2512_01055_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel source has changed since the counters were taken."""
    import glob
    h = wbuild_source_hash()
    for path in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        for line in open(path):
            if line.startswith("traffic_bytes_per_launch:"):
                f = line.split()
                d = dict(zip(f[0::2], f[1::2]))
                if (d.get("kernel:") == kernel and d.get("workload:") == workload
                        and d.get("source_sha256_16:") == h):
                    return float(d["traffic_bytes_per_launch:"])
    return None


def cpu_baseline(P, triples):
    """The CPU oracle as it stands, on a bounded sample of the same workload."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max((d.get("num_threads", 1) for d in threadpool_info()), default=1)
    except Exception:
        cores = os.cpu_count() or 1
    ints = oracle.DFIntegrals(P.B_oo, P.B_ov, P.B_vv, max_cached=6)
    t0 = time.perf_counter()
    E, parts = oracle.energy(P.eps_occ, P.eps_vir, P.t1, P.t2, ints, triple_subset=triples)
    dt = time.perf_counter() - t0
    fl = len(triples) * 12.0 * P.v ** 3 * (P.v + P.o)
    return {"value": fl / dt / 1e12, "unit": "TFLOP/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{len(triples)} occupied triples {', '.join(str(tuple(t)) for t in triples)} "
                      f"of o={P.o} v={P.v} naux={P.naux}, including their (vv|vo) slice assembly "
                      f"from the factors; {dt:.1f} s"}, {tuple(p[:3]): p[3] for p in parts}


def bench_huge(args) -> int:
    """o=100 v=800 naux=2400 with (vv|vo) assembled on the fly from the
    factors: a fixed seeded subset of triples is timed and the full job is
    extrapolated (per-triple time x N_t, plus the slice assemblies the
    full-job schedule performs at the same cache size)."""
    import torch
    from paper_2512_01055_amd import te
    from paper_2512_01055_amd.inputs import make_problem_device, sample_triples
    o, v, naux, seed = 100, 800, 2400, 5
    t0 = time.time()
    P = make_problem_device(o, v, naux, seed)
    log(f"inputs o={o} v={v} naux={naux} seed={seed} formed on the device in {time.time() - t0:.1f} s")
    if args.t2_host:
        # every array to host memory: the factors are staged by te_init, t2
        # stays there and reaches the device as panels of the slice cache
        for name in ("eps_occ", "eps_vir", "t1", "t2", "B_oo", "B_ov", "B_vv"):
            setattr(P, name, getattr(P, name).cpu().numpy())
        torch.cuda.empty_cache()
        log(f"inputs moved to host memory (t2 {P.t2.nbytes / 1e9:.1f} GB stays there)")
    sample = sample_triples(o, args.sample, seed)
    n = len(sample)
    n_full = int(te.lib().te_num_triples(o))
    fpt = te.flops_per_triple(o, v)
    res = {}
    for prec in args.precisions.split(","):
        job = te.Job(P, device=0, x_mode="on_the_fly", x_cache_slices=args.cache,
                     t2_host=args.t2_host)
        torch.cuda.synchronize()
        # the subset in chunks on one job: the slice cache stays warm across
        # chunks, and each finished chunk prints a progress line
        tot = {"seconds": 0.0, "assemble_seconds": 0.0, "slices_assembled": 0,
               "w_kernel_seconds": 0.0, "stage_seconds": 0.0}
        E = 0.0
        t1 = time.perf_counter()
        for c0 in range(0, n, args.chunk):
            Ec, _, st = job.energy_triples(sample[c0:c0 + args.chunk], prec)
            E += Ec
            for k_ in tot:
                tot[k_] += st[k_]
            log(f"[{prec}] triples {min(c0 + args.chunk, n)}/{n}: {time.perf_counter() - t1:.1f} s, "
                f"W kernel {st['w_kernel_seconds']:.2f} s, {st['slices_assembled']} slices assembled")
        dt = time.perf_counter() - t1
        S = int(st["cache_slices"])
        job.free()
        loads_full = int(te.lib().te_plan_slice_loads(o, S, 1))
        t_asm = tot["assemble_seconds"] / max(tot["slices_assembled"], 1)
        # one-off set-up of the job (operand conversion, cache allocation,
        # planning), then per-triple time, then the slice assemblies of the
        # full-job schedule at this cache size
        t_stage = tot["stage_seconds"]
        per_tr = max(dt - tot["assemble_seconds"] - t_stage, 1e-9) / n
        full = t_stage + n_full * per_tr + loads_full * t_asm
        res[prec] = {"subset_triples": n, "subset_seconds": round(dt, 3), "E_subset": E,
                     "w_kernel_tflops": round(n * fpt / tot["w_kernel_seconds"] / 1e12, 3),
                     "subset_tflops_excl_assembly": round(n * fpt / (n * per_tr) / 1e12, 3),
                     "setup_seconds": round(t_stage, 3),
                     "slices_assembled_subset": int(tot["slices_assembled"]),
                     "assemble_seconds_subset": round(tot["assemble_seconds"], 3),
                     "seconds_per_slice": round(t_asm, 4), "cache_slices": S,
                     "full_job_slice_loads": loads_full,
                     "full_job_extrapolated_seconds": round(full, 1),
                     "full_job_extrapolated_tflops": round(n_full * fpt / full / 1e12, 3)}
        log(f"[{prec}] {json.dumps(res[prec])}")
    if "fp64" in res:
        for p_, r in res.items():
            if p_ != "fp64":
                r["dE_subset_vs_fp64"] = abs(r["E_subset"] - res["fp64"]["E_subset"])
                r["dE_subset_rel"] = r["dE_subset_vs_fp64"] / abs(res["fp64"]["E_subset"])
    head = res.get("fp64") or next(iter(res.values()))
    print(json.dumps({"metric": "(T) o=100 v=800 naux=2400, (vv|vo) on the fly: extrapolated "
                                "full-job TFLOP/s", "value": head["full_job_extrapolated_tflops"],
                      "unit": "TFLOP/s", "n_gpus": 1, "data": "synthetic",
                      "config": {"workload": f"(T) o={o} v={v} naux={naux} seed {seed}, "
                                             f"{n} of {n_full} triples timed"
                                             + (", t2 in host memory" if args.t2_host else "")},
                      "precisions": res}), flush=True)
    return 0


def bench_serving(args) -> int:
    """Mixed-size (T) jobs arriving as a Poisson process: the packed server
    against sequential plain solves (te_init + te_energy + te_free, one job
    at a time) on the same arrival trace. Reports jobs/s and p50/p99 latency
    (arrival to result)."""
    import threading
    from paper_2512_01055_amd import te
    from paper_2512_01055_amd.inputs import make_problem
    rng = np.random.default_rng(4)
    os_ = rng.integers(args.omin, args.omax + 1, size=args.jobs)
    pool = {}
    t0 = time.time()
    for o in sorted(set(int(x) for x in os_)):
        pool[o] = make_problem(o, 8 * o, 24 * o, 1000 + o)
    log(f"serving: {args.jobs} jobs, o in [{args.omin},{args.omax}], pool of {len(pool)} problems "
        f"drawn in {time.time() - t0:.1f} s")
    work = sum(te.lib().te_num_triples(int(o)) * te.flops_per_triple(int(o), 8 * int(o)) for o in os_)

    def run_seq(arrivals):
        lat = []
        t_start = time.perf_counter()
        for o, a in zip(os_, arrivals):
            now = time.perf_counter() - t_start
            if now < a:
                time.sleep(a - now)
            with te.Job(pool[int(o)], device=0) as job:
                job.energy(args.precision)
            lat.append(time.perf_counter() - t_start - a)
            log(f"  sequential: job {len(lat)}/{len(os_)} (o={int(o)}) done at "
                f"{time.perf_counter() - t_start:.1f} s")
        return time.perf_counter() - t_start, lat

    def run_srv(arrivals):
        lat = [None] * len(os_)
        with te.Server(device=0, borrow_inputs=True, staging_threads=args.staging_threads) as srv:
            t_start = time.perf_counter()
            tickets = []
            for q, (o, a) in enumerate(zip(os_, arrivals)):
                now = time.perf_counter() - t_start
                if now < a:
                    time.sleep(a - now)
                tickets.append(srv.submit(pool[int(o)], args.precision))
            for q, t in enumerate(tickets):
                E, st = srv.wait(t)
                lat[q] = st["seconds"]
                log(f"  packed: job {q + 1}/{len(tickets)} (o={int(os_[q])}) collected at "
                    f"{time.perf_counter() - t_start:.1f} s")
            span = time.perf_counter() - t_start
        return span, lat

    def summary(span, lat):
        lat = np.sort(np.asarray(lat))
        return {"jobs_per_s": round(len(lat) / span, 4), "makespan_s": round(span, 2),
                "p50_s": round(float(np.percentile(lat, 50)), 3),
                "p99_s": round(float(np.percentile(lat, 99)), 3)}

    out = {}
    sat = np.zeros(args.jobs)
    log("serving: saturated arrivals, sequential")
    span_seq, lat_seq = run_seq(sat)
    out["saturated"] = {"sequential": summary(span_seq, lat_seq)}
    log("serving: saturated arrivals, packed server")
    span_p, lat_p = run_srv(sat)
    out["saturated"]["packed"] = summary(span_p, lat_p)
    cap = args.jobs / span_seq
    rate = 0.8 * cap
    arr = np.cumsum(rng.exponential(1.0 / rate, size=args.jobs))
    if args.arrivals == "both":
        log(f"serving: Poisson arrivals at {rate:.3f} jobs/s (0.8 x sequential capacity)")
        span_seq2, lat_seq2 = run_seq(arr)
        span_p2, lat_p2 = run_srv(arr)
        out["poisson"] = {"rate_jobs_per_s": round(rate, 4),
                          "sequential": summary(span_seq2, lat_seq2),
                          "packed": summary(span_p2, lat_p2)}
    print(json.dumps({"metric": "(T) serving mix: jobs/s and p50/p99 latency, packed vs sequential",
                      "value": out["saturated"]["packed"]["jobs_per_s"], "unit": "jobs/s",
                      "n_gpus": 1, "data": "synthetic", "precision": args.precision,
                      "config": {"workload": f"{args.jobs} (T) jobs, o ~ U{{{args.omin}..{args.omax}}}, "
                                             f"v = 8 o, naux = 3 v, seed 4; {work:.3e} flop in total"},
                      "results": out}), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--precisions", default="fp64,fp32,bf16x3,bf16x2,fp16x2")
    ap.add_argument("--o", type=int, default=40)
    ap.add_argument("--v", type=int, default=400)
    ap.add_argument("--naux", type=int, default=1200)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--secondary-frac", type=float, default=0.1,
                    help="fraction of the triple list (leading slice) the non-FP64 precisions time")
    ap.add_argument("--cpu-triples", type=int, default=4)
    ap.add_argument("--max-triples", type=int, default=0,
                    help="exploration only: evaluate the first N triples per step")
    ap.add_argument("--workload", choices=("large", "huge", "serving"), default="large")
    ap.add_argument("--sample", type=int, default=2000, help="huge: triples timed")
    ap.add_argument("--cache", type=int, default=0, help="huge: slice cache size (0: auto)")
    ap.add_argument("--chunk", type=int, default=100, help="huge: triples per call (progress)")
    ap.add_argument("--t2-host", action="store_true",
                    help="huge: leave t2 in host memory (panels streamed into the slice cache)")
    ap.add_argument("--jobs", type=int, default=256, help="serving: number of jobs")
    ap.add_argument("--omin", type=int, default=8)
    ap.add_argument("--omax", type=int, default=40)
    ap.add_argument("--precision", default="fp64", help="serving: precision of every job")
    ap.add_argument("--staging-threads", type=int, default=2, help="serving: concurrent staging")
    ap.add_argument("--arrivals", choices=("both", "saturated"), default="both",
                    help="serving: saturated only, or also Poisson at 0.8 x sequential capacity")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first copy this many MiB device to device (a known-size copy "
                         "kernel for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path shards by "
              "occupied triples across GPUs, which is not launched here", file=sys.stderr)
        return 2
    if args.workload == "huge":
        return bench_huge(args)
    if args.workload == "serving":
        return bench_serving(args)

    import torch
    from paper_2512_01055_amd import te
    from paper_2512_01055_amd.inputs import make_problem

    if args.calib_copy_mib:
        x = torch.ones(args.calib_copy_mib << 17, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calib_copy_mib} MiB read, {args.calib_copy_mib} MiB written")
        del x, y

    o, v, naux, seed = args.o, args.v, args.naux, args.seed
    t0 = time.time()
    P = make_problem(o, v, naux, seed)
    log(f"inputs o={o} v={v} naux={naux} seed={seed} drawn in {time.time() - t0:.1f} s")
    dev = torch.device("cuda:0")
    names = ("eps_occ", "eps_vir", "t1", "t2", "B_oo", "B_ov", "B_vv")
    D = type("DevProblem", (), {})()
    for n in names:
        setattr(D, n, torch.from_numpy(getattr(P, n)).to(dev))
    D.o, D.v, D.naux = o, v, naux
    torch.cuda.synchronize()
    n_tr = int(te.lib().te_num_triples(o))
    subset = None
    if args.max_triples and args.max_triples < n_tr:
        subset = te.triple_list(o)[:args.max_triples]
        n_tr = len(subset)
    fl_job = n_tr * te.flops_per_triple(o, v)
    stream = torch.cuda.current_stream()

    results = {}
    precs = args.precisions.split(",")
    head = "fp64" if "fp64" in precs else precs[0]
    # secondary precisions time a fixed leading slice of the triple list
    n_sec = n_tr if args.secondary_frac >= 1.0 else max(1, int(round(n_tr * args.secondary_frac)))
    sec_subset = (subset if subset is not None else te.triple_list(o))[:n_sec]
    head_pt = None
    for prec in precs:
        is_head = prec == head
        n_this = n_tr if is_head else n_sec
        fl_this = n_this * te.flops_per_triple(o, v)

        def step():
            nonlocal head_pt
            job = te.Job(D, device=0, stream=stream)
            if is_head and subset is None:
                E, st, pt = job.energy(prec, per_triple=True)
            elif is_head:
                E, pt, st = job.energy_triples(subset, prec)
            else:
                E, pt, st = job.energy_triples(sec_subset, prec)
            job.free()
            if is_head:
                head_pt = pt
            return E, st
        for w in range(args.warmup):
            log(f"[{prec}] warmup {w + 1}/{args.warmup}")
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sts = []
        E = None
        for s in range(args.steps):
            E, st = step()
            sts.append(st)
            log(f"[{prec}] step {s + 1}/{args.steps}: E(T) = {E:.12e} Eh, "
                f"{st['tflops']:.2f} TFLOP/s in te_energy, W kernel "
                f"{st['w_kernel_seconds']:.2f} s over {st['w_launches']} launches")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        wsec = sum(s_["w_kernel_seconds"] for s_ in sts)
        wl = sum(s_["w_launches"] for s_ in sts)
        results[prec] = {
            "E": E, "triples": n_this, "seconds": dt, "ms_per_step": dt / args.steps * 1e3,
            "tflops": fl_this * args.steps / dt / 1e12,
            "w_kernel_avg_ms": wsec / max(wl, 1) * 1e3,
            "w_flops_per_launch": fl_this * args.steps / max(wl, 1),
            "e_kernel_seconds": sum(s_["e_kernel_seconds"] for s_ in sts),
            "energy_seconds": sum(s_["seconds"] for s_ in sts),
        }

    r = results[head]
    achieved = r["w_flops_per_launch"] / (r["w_kernel_avg_ms"] * 1e-3) / 1e12
    out = {
        "metric": METRIC, "value": round(r["tflops"], 4), "unit": "TFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3", "bf16x2": "bf16x2",
                  "fp16x2": "fp16x2"}[head],
        "data": "synthetic",
        "config": {"workload": f"(T) of closed-shell CCSD(T), o={o} v={v} naux={naux}, "
                               f"seeded synthetic DF factors and MP2-like amplitudes (seed {seed}), "
                               f"{n_tr} occupied triples, {fl_job:.4e} algorithmic flop per job",
                   "precision": head},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3),
                     "peak": PEAK_TFLOPS[head], "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_TFLOPS[head], 4),
                     "traffic": measured_traffic(f"wbuild_kernel<{head}>", f"o{o}_v{v}"),
                     "traffic_unit": "bytes/launch",
                     "kernel": f"wbuild_kernel<{head}>",
                     "avg_launch_ms": round(r["w_kernel_avg_ms"], 4),
                     "sustained_mfma_tflops": round(te.mfma_sustained(head if head in ("fp64", "fp32", "bf16x3") else "bf16x3", 2.0), 2)},
    }
    precs_out = {}
    for p_, rr in results.items():
        d = {"tflops": round(rr["tflops"], 4), "ms_per_step": round(rr["ms_per_step"], 3),
             "triples": rr["triples"], "E": rr["E"],
             "w_kernel_tflops": round(rr["w_flops_per_launch"] / (rr["w_kernel_avg_ms"] * 1e-3) / 1e12, 3),
             "issued_mfma_tflops": round(ISSUED[p_] * rr["w_flops_per_launch"]
                                         / (rr["w_kernel_avg_ms"] * 1e-3) / 1e12, 3),
             "peak": PEAK_TFLOPS[p_]}
        if p_ != head and head == "fp64" and head_pt is not None:
            # same triples in FP64, summed in list order from the FP64 run
            E64 = float(np.sum(head_pt[:rr["triples"]]))
            dE = abs(rr["E"] - E64)
            d["E_fp64_same_triples"] = E64
            d["dE_vs_fp64"] = dE
            d["dE_rel"] = dE / abs(E64)
        precs_out[p_] = d
    out["precisions"] = precs_out
    if not args.no_cpu:
        from paper_2512_01055_amd.inputs import triple_list
        tl = triple_list(o)
        sample = [tuple(int(x) for x in t) for t in tl[1:1 + args.cpu_triples]]
        log(f"cpu baseline: oracle on {sample}")
        cb, _ = cpu_baseline(P, sample)
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
