"""Write stored oracle values for the GPU parity tests.

Calls only the CPU oracle (and the seeded generators): nothing here comes
from the device library.

    python tests/golden/make_golden.py medium       # all 1520 triples, o=20 v=200
    python tests/golden/make_golden.py medium_phys  # the same at physical scale
    python tests/golden/make_golden.py large        # 64 stratified triples, o=40 v=400
    python tests/golden/make_golden.py large_phys   # the same at physical scale
    python tests/golden/make_golden.py serving      # every job of the serving tests
    python tests/golden/make_golden.py huge [dir]   # sampled triples, o=100 v=800
                                                    # (t2 formed lazily; ~40 GB RAM)

Physical scale: a smaller factor spread b_std, chosen so that |E(T)| of the
whole job is about 0.5 Eh (E[4] scales as b_std^8, E[5] as b_std^6), where
the absolute tolerances of the method apply literally.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import numpy as np  # noqa: E402

from paper_2512_01055_amd.inputs import (HUGE, LARGE, MEDIUM, LazyDoubles,  # noqa: E402
                                         draw_factors, make_problem, triple_list)

HERE = os.path.dirname(os.path.abspath(__file__))
HUGE_TRIPLES = [(0, 0, 1), (3, 50, 99), (10, 11, 12), (98, 99, 99)]

# factor spreads of the physical-scale variants (|E(T)| about 0.5 Eh)
MEDIUM_PHYS_STD = 0.0059
LARGE_PHYS_STD = 0.0027

# jobs of the serving tests, (o, v = 8 o, naux = 3 v, seed): small ones, and
# one from the middle of the serving workload's range
SERVING_JOBS = [(8, 64, 192, 101), (5, 40, 120, 102), (10, 80, 240, 103), (8, 64, 192, 104),
                (6, 48, 144, 105), (12, 96, 288, 106), (7, 56, 168, 107), (9, 72, 216, 108),
                (24, 192, 576, 109)]


def stratified_triples(o, n=64, seed=11):
    """n triples of o occupied orbitals, in list order: the corners (first
    and last orbitals, each kind of repeated index), then seeded draws of 16
    i=j<k, 16 i<j=k and the rest i<j<k triples."""
    corners = {(0, 0, 1), (0, 1, 1), (0, 1, 2), (o - 3, o - 2, o - 1), (o - 2, o - 1, o - 1),
               (o - 2, o - 2, o - 1), (0, 0, o - 1), (0, o - 1, o - 1)}
    allt = [tuple(int(x) for x in t) for t in triple_list(o)]
    rng = np.random.default_rng(seed)
    pools = [[t for t in allt if t[0] == t[1] and t not in corners],
             [t for t in allt if t[1] == t[2] and t not in corners],
             [t for t in allt if t[0] < t[1] < t[2] and t not in corners]]
    want = [16, 16, n - len(corners) - 32]
    pick = set(corners)
    for pool, m in zip(pools, want):
        for q in rng.choice(len(pool), size=m, replace=False):
            pick.add(pool[int(q)])
    return [t for t in allt if t in pick]


def run(name, shape, b_std, triples=None):
    o, v, naux, seed = shape
    P = make_problem(o, v, naux, seed, b_std=b_std)
    ints = oracle.DFIntegrals(P.B_oo, P.B_ov, P.B_vv, max_cached=o if o <= 24 else 4)
    t0 = time.time()
    E, parts = oracle.energy(P.eps_occ, P.eps_vir, P.t1, P.t2, ints, triple_subset=triples)
    out = {
        "generator": "paper_2512_01055_amd.inputs.make_problem",
        "o": o, "v": v, "naux": naux, "seed": seed, "b_std": b_std,
        "complete": triples is None,
        "E": E,
        "triples": [[int(p[0]), int(p[1]), int(p[2])] for p in parts],
        "e": [p[3] for p in parts],
        "oracle_seconds": time.time() - t0,
    }
    path = os.path.join(HERE, f"{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print(f"{path}: E = {E:.16e} over {len(parts)} triples in {out['oracle_seconds']:.1f} s",
          flush=True)
    return out


def run_serving():
    """Every triple of every serving-test job: the whole-job E(T) a served
    job must reproduce."""
    jobs = []
    for (o, v, naux, seed) in SERVING_JOBS:
        P = make_problem(o, v, naux, seed)
        ints = oracle.DFIntegrals(P.B_oo, P.B_ov, P.B_vv, max_cached=o)
        t0 = time.time()
        E, parts = oracle.energy(P.eps_occ, P.eps_vir, P.t1, P.t2, ints)
        jobs.append({"o": o, "v": v, "naux": naux, "seed": seed, "b_std": 0.05, "E": E,
                     "n_triples": len(parts), "oracle_seconds": time.time() - t0})
        print(f"serving job {(o, v, naux, seed)}: E = {E:.16e} over {len(parts)} triples "
              f"in {jobs[-1]['oracle_seconds']:.1f} s", flush=True)
    path = os.path.join(HERE, "serving_jobs.json")
    with open(path, "w") as f:
        json.dump({"generator": "paper_2512_01055_amd.inputs.make_problem", "jobs": jobs}, f,
                  indent=0)
    print(f"{path}: {len(jobs)} jobs")


def run_huge(outdir):
    o, v, naux, seed = HUGE
    eo, ev, t1, B_oo, B_ov, B_vv = draw_factors(o, v, naux, seed)
    t2 = LazyDoubles(eo, ev, B_ov)
    ints = oracle.DFIntegrals(B_oo, B_ov, B_vv, max_cached=3)
    t0 = time.time()
    parts = []

    def say(msg):
        print(f"{msg} ({time.time() - t0:.0f} s)", flush=True)
    for (i, j, k) in HUGE_TRIPLES:             # one at a time, reporting progress
        for p in sorted({i, j, k}):
            ints.ovvv(p)
            say(f"slice {p} assembled")
        e = oracle.triple_energy(i, j, k, eo, ev, t1, t2, ints, progress=say)
        parts.append((i, j, k, e))
        say(f"triple {(i, j, k)}: e = {e:.16e}")
    E = sum(p[3] for p in parts)
    out = {"generator": "paper_2512_01055_amd.inputs.draw_factors + LazyDoubles",
           "o": o, "v": v, "naux": naux, "seed": seed, "b_std": 0.05, "complete": False,
           "E": E, "triples": [[int(p[0]), int(p[1]), int(p[2])] for p in parts],
           "e": [p[3] for p in parts], "oracle_seconds": time.time() - t0}
    path = os.path.join(outdir, "huge_o100_v800_seed5_sample.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print(f"{path}: {len(parts)} triples in {out['oracle_seconds']:.1f} s")


if __name__ == "__main__":
    if sys.argv[1:2] == ["huge"]:
        run_huge(sys.argv[2] if len(sys.argv) > 2 else HERE)
        sys.exit(0)
    which = sys.argv[1:] or ["medium", "large"]
    if "serving" in which:
        run_serving()
    if "large" in which:
        run("large_o40_v400_seed3_sample", LARGE, 0.05, stratified_triples(LARGE[0]))
    if "large_phys" in which:
        run("large_o40_v400_seed3_phys_sample", LARGE, LARGE_PHYS_STD,
            stratified_triples(LARGE[0]))
    if "medium" in which:
        run("medium_o20_v200_seed2", MEDIUM, 0.05)
    if "medium_phys" in which:
        run("medium_o20_v200_seed2_phys", MEDIUM, MEDIUM_PHYS_STD)
