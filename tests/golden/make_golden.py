"""Write stored oracle values for the GPU parity tests.

Calls only the CPU oracle (and the seeded generators): nothing here comes
from the device library.

    python tests/golden/make_golden.py medium     # all 1520 triples, o=20 v=200
    python tests/golden/make_golden.py large      # sampled triples, o=40 v=400
    python tests/golden/make_golden.py huge [dir] # sampled triples, o=100 v=800
                                                  # (t2 formed lazily; ~50 GB RAM)
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2512_01055_amd.inputs import (HUGE, LARGE, MEDIUM, LazyDoubles,  # noqa: E402
                                         draw_factors, make_problem)

HERE = os.path.dirname(os.path.abspath(__file__))
HUGE_TRIPLES = [(0, 0, 1), (3, 50, 99), (98, 99, 99)]

# triples of the large workload checked one by one: both i=j<k and i<j=k
# kinds, first and last occupied orbitals, a generic triple
LARGE_TRIPLES = [(0, 0, 1), (0, 1, 1), (5, 17, 33), (38, 39, 39), (2, 21, 39)]


def run(name, shape, b_std, triples=None):
    o, v, naux, seed = shape
    P = make_problem(o, v, naux, seed, b_std=b_std)
    ints = oracle.DFIntegrals(P.B_oo, P.B_ov, P.B_vv, max_cached=o if o <= 20 else 4)
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
    print(f"{path}: E = {E:.16e} over {len(parts)} triples in {out['oracle_seconds']:.1f} s")


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
    if "medium" in which:
        run("medium_o20_v200_seed2", MEDIUM, 0.05)
    if "medium_phys" in which:
        run("medium_o20_v200_seed2_phys", MEDIUM, 0.0067)
    if "large" in which:
        run("large_o40_v400_seed3_sample", LARGE, 0.05, LARGE_TRIPLES)
    if "large_phys" in which:
        run("large_o40_v400_seed3_phys_sample", LARGE, 0.0028, LARGE_TRIPLES)
