"""Throughput of the (T) correction on one MI355X.

The workload is one whole FP64 (T) job on the synthetic o=40, v=400,
naux=1200 problem with the inputs already in HBM: staging from the factors
(integral assembly, padded layouts), the W build over all 11,440 occupied
triples, the fused V/D/energy consumer and the reductions. The job is timed
as --steps steps (default 20): step 0 also stages the job (te_init), step s
evaluates the s-th contiguous piece of the i-major triple list, and the last
step also frees the job, so the steps together are exactly one job. Warmup
steps run the first pieces on a job of their own. FP32 and the split 16-bit
modes then run a fixed leading piece of the list (--secondary-frac, default
10%) and report |dE(T)| against the FP64 partials of the same triples.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precisions fp64,fp32,...]
    python bench.py --workload huge      # o=100 v=800, (vv|vo) on the fly, subset
    python bench.py --workload serving   # mixed-size jobs, packed server vs sequential
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


def cpu_info():
    """CPU model and the number of logical CPUs this process may run on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return model, n


def cpu_baseline(P, triples, single):
    """The CPU oracle as it stands, on a bounded sample of the same workload:
    `triples` on the BLAS thread pool (every core it uses), and `single`
    (one triple) on one thread. Both include the (vv|vo) slice assembly
    from the factors that their triples need."""
    import oracle
    from threadpoolctl import threadpool_info, threadpool_limits
    model, ncpu = cpu_info()
    threads = max((d.get("num_threads", 1) for d in threadpool_info()), default=1)
    fpt = 12.0 * P.v ** 3 * (P.v + P.o)

    def run(sample):
        ints = oracle.DFIntegrals(P.B_oo, P.B_ov, P.B_vv, max_cached=6)
        t0 = time.perf_counter()
        E, parts = oracle.energy(P.eps_occ, P.eps_vir, P.t1, P.t2, ints, triple_subset=sample)
        return time.perf_counter() - t0, parts
    dt, parts = run(triples)
    with threadpool_limits(limits=1):
        dt1, parts1 = run(single)
    desc = lambda ts: ", ".join(str(tuple(int(x) for x in t)) for t in ts)  # noqa: E731
    return {"value": len(triples) * fpt / dt / 1e12, "unit": "TFLOP/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{len(triples)} occupied triples {desc(triples)} of o={P.o} v={P.v} "
                      f"naux={P.naux} in {dt:.1f} s on {threads} BLAS threads, including their "
                      f"(vv|vo) slice assembly from the factors; numpy FP64",
            "cpu_model": model, "nproc": ncpu,
            "single_thread_value": fpt * len(single) / dt1 / 1e12,
            "single_thread_sample": f"{desc(single)} in {dt1:.1f} s on one thread, with its "
                                    f"slice assembly"}, {tuple(p[:3]): p[3] for p in parts + parts1}


def bench_huge(args) -> int:
    """o=100 v=800 naux=2400 with (vv|vo) assembled on the fly from the
    factors. A fixed seeded subset of triples gives the energies (and their
    spread against FP64) and the time per slice assembly; the time per triple
    with every slice already in the cache comes from triples within the first
    few occupied indices, run twice on one job with the second run timed. The
    full job is extrapolated as set-up + N_t x that time + the slice
    assemblies of the full-job schedule at the same cache size, counted as if
    none overlapped a W build (slices are filled on a stream of their own,
    beside the W builds)."""
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
    # triples within the first q occupied indices (q slices, all cached)
    q = 8
    warm = np.array([(i, j, k) for i in range(q) for j in range(i, q) for k in range(j, q)
                     if not i == j == k], dtype=np.int32)
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
        # per-triple time with the slices cached: the warm set twice
        job.energy_triples(warm, prec)
        t2_ = time.perf_counter()
        _, _, sw_ = job.energy_triples(warm, prec)
        dtw = time.perf_counter() - t2_
        if sw_["slices_assembled"]:
            raise SystemExit(f"warm set assembled {sw_['slices_assembled']} slices; cache {S}")
        log(f"[{prec}] {len(warm)} cached triples in {dtw:.2f} s, "
            f"W kernel {sw_['w_kernel_seconds']:.2f} s")
        job.free()
        loads_full = int(te.lib().te_plan_slice_loads(o, S, 1))
        t_asm = tot["assemble_seconds"] / max(tot["slices_assembled"], 1)
        t_stage = tot["stage_seconds"]
        # from the call's first launch to its result: the call's own set-up
        # (scratch allocation, planning) and the release of its scratch are
        # paid once per call, and the full job is one call (its set-up is in
        # t_stage)
        per_tr = max(sw_["seconds"] - sw_["stage_seconds"], 1e-9) / len(warm)
        full = t_stage + n_full * per_tr + loads_full * t_asm
        res[prec] = {"subset_triples": n, "subset_seconds": round(dt, 3), "E_subset": E,
                     "w_kernel_tflops": round(len(warm) * fpt / sw_["w_kernel_seconds"] / 1e12, 3),
                     "cached_triples": len(warm), "cached_seconds": round(dtw, 3),
                     "cached_setup_seconds": round(sw_["stage_seconds"], 3),
                     "cached_tflops": round(len(warm) * fpt / (len(warm) * per_tr) / 1e12, 3),
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
        """Submit each job at its arrival time and collect results as they
        complete (every job is reported when it finishes)."""
        lat = [None] * len(os_)
        with te.Server(device=0, borrow_inputs=True, staging_threads=args.staging_threads) as srv:
            t_start = time.perf_counter()
            pending = {}
            nsub, ndone = 0, 0
            while ndone < len(os_):
                now = time.perf_counter() - t_start
                while nsub < len(os_) and arrivals[nsub] <= now:
                    pending[nsub] = srv.submit(pool[int(os_[nsub])], args.precision)
                    nsub += 1
                for q in list(pending):
                    r = srv.poll(pending[q])
                    if r is not None:
                        lat[q] = r[1]["seconds"]
                        del pending[q]
                        ndone += 1
                        log(f"  packed: job {q + 1} (o={int(os_[q])}) done at "
                            f"{time.perf_counter() - t_start:.1f} s ({ndone}/{len(os_)})")
                time.sleep(0.005)
            span = time.perf_counter() - t_start
        return span, lat

    def summary(span, lat):
        lat = np.sort(np.asarray(lat))
        return {"jobs_per_s": round(len(lat) / span, 4), "makespan_s": round(span, 2),
                "p50_s": round(float(np.percentile(lat, 50)), 3),
                "p99_s": round(float(np.percentile(lat, 99)), 3)}

    out = {}
    if args.arrivals == "poisson":
        if args.rate <= 0:
            raise SystemExit("--arrivals poisson needs --rate")
        arr = np.cumsum(rng.exponential(1.0 / args.rate, size=args.jobs))
        log(f"serving: Poisson arrivals at {args.rate:.3f} jobs/s, sequential")
        span_seq2, lat_seq2 = run_seq(arr)
        log("serving: Poisson arrivals, packed server")
        span_p2, lat_p2 = run_srv(arr)
        out["poisson"] = {"rate_jobs_per_s": round(args.rate, 4),
                          "sequential": summary(span_seq2, lat_seq2),
                          "packed": summary(span_p2, lat_p2)}
        print(json.dumps({"metric": "(T) serving mix: jobs/s and p50/p99 latency, packed vs "
                                    "sequential", "value": out["poisson"]["packed"]["jobs_per_s"],
                          "unit": "jobs/s", "n_gpus": 1, "data": "synthetic",
                          "precision": args.precision,
                          "config": {"workload": f"{args.jobs} (T) jobs, o ~ U{{{args.omin}.."
                                                 f"{args.omax}}}, v = 8 o, naux = 3 v, seed 4; "
                                                 f"{work:.3e} flop in total"},
                          "results": out}), flush=True)
        return 0
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
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precisions", default="fp64,fp32,bf16x3,bf16x2,fp16x2")
    ap.add_argument("--o", type=int, default=40)
    ap.add_argument("--v", type=int, default=400)
    ap.add_argument("--naux", type=int, default=1200)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--secondary-frac", type=float, default=0.1,
                    help="fraction of the triple list (leading slice) the non-FP64 precisions time")
    ap.add_argument("--cpu-triples", type=int, default=3)
    ap.add_argument("--max-triples", type=int, default=0,
                    help="exploration only: a job of the first N triples")
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
    ap.add_argument("--arrivals", choices=("both", "saturated", "poisson"), default="both",
                    help="serving: saturated only, also Poisson at 0.8 x sequential capacity, "
                         "or Poisson only at --rate")
    ap.add_argument("--rate", type=float, default=0.0,
                    help="serving, --arrivals poisson: arrival rate in jobs/s")
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

    return bench_large(args)


def step_slices(n_triples: int, steps: int):
    """Contiguous pieces [start, stop) of the i-major triple list, one per
    step: together the steps evaluate every triple exactly once."""
    if steps < 1:
        raise ValueError("need at least one step")
    edges = np.linspace(0, n_triples, steps + 1).round().astype(np.int64)
    return [(int(edges[s]), int(edges[s + 1])) for s in range(steps)]


def bench_large(args) -> int:
    """One whole FP64 (T) job at o=40, v=400, naux=1200, timed as `steps`
    steps: step 0 stages the job (te_init), step s evaluates the s-th
    contiguous piece of the triple list, and the last step also frees the
    job. The value is the job's algorithmic flops over the total."""
    import math

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
    D = type("DevProblem", (), {})()
    for n in ("eps_occ", "eps_vir", "t1", "t2", "B_oo", "B_ov", "B_vv"):
        setattr(D, n, torch.from_numpy(getattr(P, n)).to(dev))
    D.o, D.v, D.naux = o, v, naux
    torch.cuda.synchronize()
    tl = te.triple_list(o)
    if args.max_triples:
        tl = tl[:args.max_triples]
    n_tr = len(tl)
    fpt = te.flops_per_triple(o, v)
    fl_job = n_tr * fpt
    pieces = step_slices(n_tr, args.steps)
    stream = torch.cuda.current_stream()

    # warmup: a job of its own, evaluating the first pieces
    if args.warmup:
        job = te.Job(D, device=0, stream=stream)
        for w in range(args.warmup):
            a, b = pieces[w % len(pieces)]
            job.energy_triples(tl[a:b], "fp64")
            log(f"[fp64] warmup {w + 1}/{args.warmup}: triples {a}..{b - 1}")
        job.free()
    torch.cuda.synchronize()

    # timed: te_init, every piece in order, te_free
    pts, sts, step_s = [], [], []
    t_start = time.perf_counter()
    job = te.Job(D, device=0, stream=stream)
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t_start
    for s, (a, b) in enumerate(pieces):
        ts = time.perf_counter()
        _, pt, st = job.energy_triples(tl[a:b], "fp64")
        if s == len(pieces) - 1:
            job.free()
        torch.cuda.synchronize()
        step_s.append(time.perf_counter() - ts + (t_init if s == 0 else 0.0))
        pts.append(pt)
        sts.append(st)
        log(f"[fp64] step {s + 1}/{len(pieces)}: triples {a}..{b - 1} in {step_s[-1]:.3f} s, "
            f"W kernel {st['w_kernel_seconds']:.3f} s over {st['w_launches']} launches")
    total = time.perf_counter() - t_start
    pt64 = np.concatenate(pts)
    E64 = math.fsum(pt64.tolist())
    wsec = sum(x["w_kernel_seconds"] for x in sts)
    wl = sum(x["w_launches"] for x in sts)
    w_flops_per_launch = fl_job / max(wl, 1)
    achieved = w_flops_per_launch / (wsec / max(wl, 1)) / 1e12
    log(f"[fp64] job: E(T) = {E64:.12e} Eh in {total:.2f} s (te_init {t_init:.3f} s), "
        f"{fl_job / total / 1e12:.2f} TFLOP/s; W kernel {achieved:.2f} TFLOP/s")

    precs_out = {"fp64": {"tflops": round(fl_job / total / 1e12, 4), "triples": n_tr, "E": E64,
                          "seconds": round(total, 3), "init_seconds": round(t_init, 4),
                          "w_kernel_tflops": round(achieved, 3),
                          "w_kernel_avg_ms": round(wsec / max(wl, 1) * 1e3, 4),
                          "e_kernel_seconds": round(sum(x["e_kernel_seconds"] for x in sts), 3),
                          "issued_mfma_tflops": round(achieved, 3), "peak": PEAK_TFLOPS["fp64"]}}

    # the other precisions on a fixed leading piece of the same list, on a
    # job of their own; |dE| against the FP64 partials of the same triples
    n_sec = max(1, int(round(n_tr * args.secondary_frac)))
    sec = [p_ for p_ in args.precisions.split(",") if p_ != "fp64"]
    if sec:
        job = te.Job(D, device=0, stream=stream)
        for prec in sec:
            ts = time.perf_counter()
            E, pt, st = job.energy_triples(tl[:n_sec], prec)
            dt = time.perf_counter() - ts
            Eref = math.fsum(pt64[:n_sec].tolist())
            Es = math.fsum(pt.tolist())
            wr = n_sec * fpt / st["w_kernel_seconds"] / 1e12
            precs_out[prec] = {
                "tflops": round(n_sec * fpt / dt / 1e12, 4), "triples": n_sec, "E": Es,
                "seconds": round(dt, 3), "setup_seconds": round(st["stage_seconds"], 3),
                "w_kernel_tflops": round(wr, 3), "issued_mfma_tflops": round(ISSUED[prec] * wr, 3),
                "peak": PEAK_TFLOPS[prec], "E_fp64_same_triples": Eref,
                "dE_vs_fp64": abs(Es - Eref), "dE_rel": abs(Es - Eref) / abs(Eref)}
            log(f"[{prec}] {n_sec} triples in {dt:.2f} s (operand conversion "
                f"{st['stage_seconds']:.2f} s): W kernel {wr:.1f} TFLOP/s, "
                f"|dE| vs FP64 {abs(Es - Eref):.3e} Eh ({abs(Es - Eref) / abs(Eref):.2e} rel)")
        job.free()
    del D
    torch.cuda.empty_cache()

    out = {
        "metric": METRIC, "value": round(fl_job / total / 1e12, 4), "unit": "TFLOP/s",
        "n_gpus": 1, "steps": len(pieces), "warmup": args.warmup,
        "ms_per_step": round(total / len(pieces) * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"(T) of closed-shell CCSD(T), o={o} v={v} naux={naux}, "
                               f"seeded synthetic DF factors and MP2-like amplitudes (seed {seed}); "
                               f"one whole job ({n_tr} occupied triples, {fl_job:.4e} algorithmic "
                               f"flop) split into {len(pieces)} steps of consecutive triples, "
                               f"te_init in the first step",
                   "precision": "fp64"},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3),
                     "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_TFLOPS["fp64"], 4),
                     "traffic": measured_traffic("wbuild_kernel<fp64>", f"o{o}_v{v}"),
                     "traffic_unit": "bytes/launch",
                     "kernel": "wbuild_kernel<fp64>",
                     "launches": int(wl), "w_flops_per_launch": w_flops_per_launch,
                     "avg_launch_ms": round(wsec / max(wl, 1) * 1e3, 4)},
        "step_seconds": [round(x, 4) for x in step_s],
        "precisions": precs_out,
    }
    if not args.no_cpu:
        # all cores on three triples (three slices assembled), one thread on one
        sample = [tuple(int(x) for x in t) for t in tl[1:1 + args.cpu_triples]]
        single = [tuple(int(x) for x in tl[0])]
        log(f"cpu baseline: oracle on {sample} (all cores) and {single} (one thread)")
        cb, ref = cpu_baseline(P, sample, single)
        out["cpu_baseline"] = cb
        # the oracle's values of those triples against the device's
        pos = {tuple(int(x) for x in t): q for q, t in enumerate(tl)}
        out["cpu_baseline"]["max_rel_diff_vs_device"] = max(
            abs(pt64[pos[k]] - e) / abs(e) for k, e in ref.items())
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
