"""Seeded synthetic (T) problems.

This module only draws inputs; it computes no part of the triples correction.
Both the CPU oracle (through the tests) and the device library consume what it
returns, so it must stay free of either side's arithmetic.

The recipe stands in for the converged CCSD amplitudes and Cholesky/DF
factors of the paper's molecules, which are not available:

* occupied orbital energies ~ U[-1.5, -0.3] Eh, virtual ones ~ U[0.1, 3.0] Eh
  (left unsorted);
* DF factors B^Q_pq ~ N(0, b_std^2), symmetric in the orbital pair: the
  elements with p <= q are drawn i.i.d. and mirrored, so every element keeps
  the same spread. Each draw is rounded to a multiple of 2^-20 (a relative
  change of ~1e-5 at b_std = 0.05). Products of two such values are
  multiples of 2^-40, and while max|B|^2 naux < 2^13 every partial sum of
  (pq|rs) = sum_Q B^Q_pq B^Q_rs is a multiple of 2^-40 below 2^13, which
  FP64 holds exactly: every integral, and so the doubles below, come out
  bitwise the same whatever the summation order (numpy or torch, host or
  device, any BLAS);
* MP2-like doubles t_ij^ab = (ia|jb) / (e_i + e_j - e_a - e_b) with
  (ia|jb) = sum_Q B^Q_ia B^Q_jb, so t_ij^ab = t_ji^ba holds exactly;
* singles t_i^a ~ N(0, t1_std^2).

Layouts are row-major FP64: eps_occ[o], eps_vir[v], t1[o][v], t2[o][o][v][v],
B_oo[naux][o][o], B_ov[naux][o][v], B_vv[naux][v][v].
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Problem:
    o: int
    v: int
    naux: int
    eps_occ: np.ndarray
    eps_vir: np.ndarray
    t1: np.ndarray
    t2: np.ndarray
    B_oo: np.ndarray
    B_ov: np.ndarray
    B_vv: np.ndarray
    seed: int = 0

    @property
    def n_triples(self) -> int:
        o = self.o
        return o * (o + 1) * (o + 2) // 6 - o


# Shapes of the synthetic workloads: (o, v, naux, seed).
SMALL = (6, 30, 90, 1)          # every triple checked against the oracle
MEDIUM = (20, 200, 600, 2)      # single job, full (vv|vo) resident
LARGE = (40, 400, 1200, 3)      # the throughput workload
HUGE = (100, 800, 2400, 5)      # (vv|vo) assembled on the fly


# Factor values are drawn on this grid (see the module docstring).
GRID = 2.0 ** 20


def _on_grid(x: np.ndarray) -> np.ndarray:
    """x rounded to the nearest multiple of 1 / GRID (in place)."""
    x *= GRID
    np.rint(x, out=x)
    x *= 1.0 / GRID
    return x


def _sym_normal(rng: np.random.Generator, naux: int, n: int, std: float) -> np.ndarray:
    """naux symmetric n x n matrices; p<=q drawn i.i.d., mirrored below."""
    out = np.empty((naux, n, n))
    iu = np.triu_indices(n)
    for q in range(naux):
        m = np.zeros((n, n))
        m[iu] = _on_grid(rng.standard_normal(len(iu[0])) * std)
        out[q] = m + np.triu(m, 1).T
    return out


def _check_exact(naux: int, *factors: np.ndarray) -> None:
    """The factor integrals are exact in FP64 only while every partial sum
    stays below 2^13 (2^53 grid units of 2^-40)."""
    m = max(float(np.abs(f).max()) for f in factors if f.size)
    if m * m * naux >= 2.0 ** 13:
        raise ValueError(f"factors too large for exact integrals: max|B| = {m}, naux = {naux}")


def make_problem(o: int, v: int, naux: int, seed: int, *, b_std: float = 0.05,
                 t1_std: float = 1e-3, with_t1: bool = True) -> Problem:
    """Draw one synthetic closed-shell (T) problem."""
    if o < 1 or v < 1 or naux < 1:
        raise ValueError("o, v and naux must be positive")
    rng = np.random.default_rng(seed)
    eps_occ = rng.uniform(-1.5, -0.3, o)
    eps_vir = rng.uniform(0.1, 3.0, v)
    B_oo = _sym_normal(rng, naux, o, b_std)
    B_ov = _on_grid(rng.standard_normal((naux, o, v)) * b_std)
    B_vv = _sym_normal(rng, naux, v, b_std)
    _check_exact(naux, B_oo, B_ov, B_vv)
    t1 = rng.standard_normal((o, v)) * t1_std
    if not with_t1:
        t1[:] = 0.0
    t2 = mp2_doubles(eps_occ, eps_vir, B_ov)
    return Problem(o, v, naux, eps_occ, eps_vir, t1, t2, B_oo, B_ov, B_vv, seed)


def mp2_doubles(eps_occ: np.ndarray, eps_vir: np.ndarray, B_ov: np.ndarray) -> np.ndarray:
    """t2[i][j][a][b] = (ia|jb) / (e_i + e_j - e_a - e_b)."""
    naux, o, v = B_ov.shape
    L = B_ov.reshape(naux, o * v)
    M = L.T @ L
    M += M.T           # exact symmetry (ia|jb) = (jb|ia), whatever BLAS rounding did
    M *= 0.5
    t2 = np.ascontiguousarray(M.reshape(o, v, o, v).transpose(0, 2, 1, 3))
    del M
    # (e_i + e_j) - (e_a + e_b): both sums commute, so t_ij^ab = t_ji^ba bitwise
    den = ((eps_occ[:, None, None, None] + eps_occ[None, :, None, None])
           - (eps_vir[None, None, :, None] + eps_vir[None, None, None, :]))
    t2 /= den
    return t2


def triple_list(o: int) -> np.ndarray:
    """Occupied triples i<=j<=k, i=j=k left out, i-major; int32 [N_t][3]."""
    out = [(i, j, k) for i in range(o) for j in range(i, o) for k in range(j, o)
           if not (i == j == k)]
    return np.asarray(out, dtype=np.int32).reshape(-1, 3)


def sample_triples(o: int, n: int, seed: int) -> np.ndarray:
    """A fixed seeded subset of n triples that always holds both
    i=j<k and i<j=k kinds when they exist; returned in list order."""
    allt = triple_list(o)
    n = min(n, len(allt))
    rng = np.random.default_rng(seed)
    idx = set(rng.choice(len(allt), size=n, replace=False).tolist())
    eq_ij = np.nonzero((allt[:, 0] == allt[:, 1]))[0]
    eq_jk = np.nonzero((allt[:, 1] == allt[:, 2]))[0]
    for pool in (eq_ij, eq_jk):
        if len(pool) and not idx.intersection(pool.tolist()):
            idx.pop()
            idx.add(int(pool[rng.integers(len(pool))]))
    return allt[sorted(idx)]


def draw_factors(o: int, v: int, naux: int, seed: int, *, b_std: float = 0.05,
                 t1_std: float = 1e-3):
    """The random draws of make_problem (same stream, same values) without
    forming the doubles: returns (eps_occ, eps_vir, t1, B_oo, B_ov, B_vv)."""
    rng = np.random.default_rng(seed)
    eps_occ = rng.uniform(-1.5, -0.3, o)
    eps_vir = rng.uniform(0.1, 3.0, v)
    B_oo = _sym_normal(rng, naux, o, b_std)
    B_ov = _on_grid(rng.standard_normal((naux, o, v)) * b_std)
    B_vv = _sym_normal(rng, naux, v, b_std)
    _check_exact(naux, B_oo, B_ov, B_vv)
    t1 = rng.standard_normal((o, v)) * t1_std
    return eps_occ, eps_vir, t1, B_oo, B_ov, B_vv


class LazyDoubles:
    """Host view of t2 = (ia|jb)/(e_i+e_j-e_a-e_b) that forms only what is
    indexed: t2[i, j] -> [v][v] and t2[:, j] -> [o][v][v]. Same definition as
    mp2_doubles, for problems whose full t2 does not fit host memory."""

    def __init__(self, eps_occ, eps_vir, B_ov):
        self.eo, self.ev, self.B = eps_occ, eps_vir, B_ov
        naux, o, v = B_ov.shape
        self.shape = (o, o, v, v)

    def _pair(self, i, j):
        X = self.B[:, i, :].T @ self.B[:, j, :]          # (ia|jb)
        Y = self.B[:, j, :].T @ self.B[:, i, :]          # (jb|ia)
        M = 0.5 * (X + Y.T)
        den = (self.eo[i] + self.eo[j]) - (self.ev[:, None] + self.ev[None, :])
        return M / den

    def __getitem__(self, key):
        i, j = key
        if isinstance(i, slice):
            return np.stack([self._pair(q, j) for q in range(self.shape[0])[i]])
        return self._pair(i, j)


def make_problem_device(o: int, v: int, naux: int, seed: int, device="cuda:0", *,
                        b_std: float = 0.05, t1_std: float = 1e-3):
    """make_problem with the doubles formed on the device (torch, FP64), for
    sizes whose o^2 v^2 array is too large to build on the host. The draws
    are identical to make_problem's, and since the factors sit on the exact
    grid, so is t2, bit for bit: (ia|jb) is exact in any summation order,
    and the symmetrisation, the denominators and the one division are the
    same IEEE operations as on the host. Returns an object with torch
    tensors (on `device`) eps_occ, eps_vir, t1, t2, B_oo, B_ov, B_vv and
    o, v, naux."""
    import torch
    eo, ev, t1, B_oo, B_ov, B_vv = draw_factors(o, v, naux, seed, b_std=b_std, t1_std=t1_std)
    dev = torch.device(device)
    out = type("DeviceProblem", (), {})()
    out.o, out.v, out.naux, out.seed = o, v, naux, seed
    for name, x in (("eps_occ", eo), ("eps_vir", ev), ("t1", t1), ("B_oo", B_oo),
                    ("B_ov", B_ov), ("B_vv", B_vv)):
        setattr(out, name, torch.from_numpy(x).to(dev))
    del B_vv
    L = out.B_ov.reshape(naux, o * v)
    t2 = torch.empty((o, o, v, v), dtype=torch.float64, device=dev)
    for i in range(o):                                  # (ia|jb) for all j, row block i
        t2[i] = (L[:, i * v:(i + 1) * v].T @ L).reshape(v, o, v).permute(1, 0, 2)
    t2 += t2.permute(1, 0, 3, 2).clone()
    t2 *= 0.5
    e_o, e_v = out.eps_occ, out.eps_vir
    for i in range(o):
        den = (e_o[i] + e_o)[:, None, None] - (e_v[:, None] + e_v[None, :])[None]
        t2[i] /= den
    out.t2 = t2
    if dev.type == "cuda":
        torch.cuda.synchronize()
        torch.cuda.empty_cache()     # return the temporaries to the device
    return out
