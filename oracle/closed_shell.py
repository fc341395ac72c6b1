"""Closed-shell (T) energy, plain FP64 on the CPU.

TEST INFRASTRUCTURE ONLY. This is the reference the device library is
checked against. Only the tests, the smoke check and the benchmark's CPU
baseline may import it; the library never does.

Every function follows one passage of Fajen, Kelly, Hohenstein, Martinez,
"Accelerating CCSD(T) on GPUs" (arXiv 2512.01055), section "Implementation
Details", Eqs. 1-6, under the readings listed below. Contractions use numpy's
einsum/matmul as plain steps; nothing is blocked, fused or reordered beyond
what the equations state.

Readings (where the text is ambiguous or inconsistent):

R1  G^{rs}_{pq} is the physicists' integral <pq|rs> = (pr|qs) in chemists'
    notation, so G^{ab}_{if} = (ia|bf), G^{al}_{ij} = (ia|jl),
    G^{bc}_{jk} = (jb|kc).
R2  t^{xy}_{pq}: x pairs with p, y with q; t^{ab}_{ij} = t^{ba}_{ji}.
R3  The denominator is D = e_i + e_j + e_k - e_a - e_b - e_c (negative for a
    bound reference). Eq. 4 prints the opposite sign; the energy-kernel
    figure uses this one, and only this one gives E[4] <= 0.
R4  Eq. 1 restricted to a>=b>=c with weight (2 - d_ab - d_bc) equals one third
    of the unrestricted sum over all abc and ijk, and equals the occupied
    restricted form sum_{i<=j<=k} (2 - d_ij - d_jk) sum_{abc}; this module
    evaluates the last one (``energy``) and the printed one
    (``energy_eq1_form``) so that the two can be compared.
R6  The paper's V (Eq. 3) is the singles term only; the energy uses W + V.
R7  Canonical orbitals: no f_ov term.

Integral access goes through an ``Integrals`` object with three methods:
  ovvv(p)   -> [v][v][v]   element [x][y][f] = (p x|y f)
  ovoo(p)   -> [v][o][o]   element [x][q][l] = (p x|q l)
  ovov(p,q) -> [v][v]      element [x][y]    = (p x|q y)
"""
from __future__ import annotations

import numpy as np

# The six simultaneous (occupied, virtual) pair permutations of Eq. 5, as
# position maps: term s takes occupied (o[P[0]], o[P[1]], o[P[2]]) together
# with virtual (u[P[0]], u[P[1]], u[P[2]]), u = (a, b, c).
EQ5_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 1, 0), (2, 0, 1))


class ExplicitIntegrals:
    """Integrals given in full: (ia|bc) [o][v][v][v], (ia|jk) [o][v][o][o],
    (ia|jb) [o][v][o][v]."""

    def __init__(self, ovvv: np.ndarray, ovoo: np.ndarray, ovov: np.ndarray):
        self._ovvv, self._ovoo, self._ovov = ovvv, ovoo, ovov

    def ovvv(self, p: int) -> np.ndarray:
        return self._ovvv[p]

    def ovoo(self, p: int) -> np.ndarray:
        return self._ovoo[p]

    def ovov(self, p: int, q: int) -> np.ndarray:
        return self._ovov[p, :, q, :]


class DFIntegrals:
    """Integrals rebuilt from factors, Eq. 6: (pq|rs) = sum_Q B^Q_pq B^Q_rs.

    Slices are formed when first asked for and kept, so large problems never
    hold the full o*v^3 array.
    """

    def __init__(self, B_oo: np.ndarray, B_ov: np.ndarray, B_vv: np.ndarray,
                 max_cached: int = 8):
        self.B_oo, self.B_ov, self.B_vv = B_oo, B_ov, B_vv
        self._cache: dict = {}
        self._order: list = []
        self._max = max_cached

    def _keep(self, key, val):
        self._cache[key] = val
        self._order.append(key)
        while len(self._order) > self._max:
            self._cache.pop(self._order.pop(0), None)
        return val

    def ovvv(self, p: int) -> np.ndarray:
        key = ("ovvv", p)
        if key not in self._cache:
            naux, v = self.B_vv.shape[0], self.B_vv.shape[1]
            # (p x|y f) = sum_Q B^Q_px B^Q_yf
            val = (self.B_ov[:, p, :].T @ self.B_vv.reshape(naux, v * v)).reshape(v, v, v)
            return self._keep(key, val)
        return self._cache[key]

    def ovoo(self, p: int) -> np.ndarray:
        # (p x|q l) = sum_Q B^Q_px B^Q_ql
        return np.einsum("Qx,Qql->xql", self.B_ov[:, p, :], self.B_oo)

    def ovov(self, p: int, q: int) -> np.ndarray:
        # (p x|q y) = sum_Q B^Q_px B^Q_qy
        return np.einsum("Qx,Qy->xy", self.B_ov[:, p, :], self.B_ov[:, q, :])


def integrals_from_df(B_oo, B_ov, B_vv):
    """Full (ia|bc), (ia|jk), (ia|jb) from the factors (Eq. 6); small cases."""
    ovvv = np.einsum("Qia,Qbc->iabc", B_ov, B_vv)
    ovoo = np.einsum("Qia,Qjk->iajk", B_ov, B_oo)
    ovov = np.einsum("Qia,Qjb->iajb", B_ov, B_ov)
    return ovvv, ovoo, ovov


def w_tensor(i: int, j: int, k: int, ints, t2: np.ndarray) -> np.ndarray:
    """W^{abc}_{ijk} for fixed (i, j, k) as a [v][v][v] array (Eqs. 2 and 5).

    Eq. 2 for one ordering (p, q, r; x, y, z) of the pairs is
        A^{xyz}_{pqr} = sum_f (px|yf) t^{zf}_{rq} - sum_l (px|ql) t^{yz}_{lr},
    and Eq. 5 adds it over the six simultaneous pair permutations.
    """
    occ = (i, j, k)
    v = t2.shape[2]
    W = np.zeros((v, v, v))
    for P in EQ5_PERMS:
        p, q, r = occ[P[0]], occ[P[1]], occ[P[2]]
        # A[x, y, z] for all x, y, z
        o = t2.shape[0]
        # sum_f (px|yf) t^{zf}_{rq}: rows (x, y) of the slice times rows z of t_rq
        A = (ints.ovvv(p).reshape(v * v, v) @ t2[r, q].T).reshape(v, v, v)
        # sum_l (px|ql) t^{yz}_{lr}: rows x of (px|q.) times t_{lr} over l
        A -= (ints.ovoo(p)[:, q, :] @ t2[:, r].reshape(o, v * v)).reshape(v, v, v)
        # W[u0, u1, u2] += A[u_P0, u_P1, u_P2]
        inv = tuple(int(np.argsort(P)[d]) for d in range(3))
        W += A.transpose(inv)
    return W


def v_tensor(i: int, j: int, k: int, ints, t1: np.ndarray) -> np.ndarray:
    """Singles term of Eq. 3: t_i^a (jb|kc) + t_j^b (ia|kc) + t_k^c (ia|jb)."""
    Vt = (t1[i][:, None, None] * ints.ovov(j, k)[None, :, :]
          + t1[j][None, :, None] * ints.ovov(i, k)[:, None, :]
          + t1[k][None, None, :] * ints.ovov(i, j)[:, :, None])
    return Vt


def d_tensor(i: int, j: int, k: int, eps_occ, eps_vir) -> np.ndarray:
    """Denominator (Eq. 4, sign per reading R3): e_i+e_j+e_k-e_a-e_b-e_c."""
    ev = eps_vir
    return (eps_occ[i] + eps_occ[j] + eps_occ[k]
            - ev[:, None, None] - ev[None, :, None] - ev[None, None, :])


def z_tensor(W: np.ndarray) -> np.ndarray:
    """4 W^abc + W^bca + W^cab - 2 W^acb - 2 W^bac - 2 W^cba (Eq. 1, with the
    occupied permutations of the printed form moved onto the virtual labels,
    reading R4)."""
    return (4.0 * W + _permuted(W, "bca") + _permuted(W, "cab")
            - 2.0 * _permuted(W, "acb") - 2.0 * _permuted(W, "bac")
            - 2.0 * _permuted(W, "cba"))


def _permuted(W: np.ndarray, s: str) -> np.ndarray:
    """Array X with X[a,b,c] = W[s0, s1, s2] where s names which of a, b, c
    goes in each slot, e.g. s = 'bca' gives X[a,b,c] = W[b,c,a]."""
    pos = {"a": 0, "b": 1, "c": 2}
    # W's axis d is indexed by X's axis pos[s[d]]  ->  X = W.transpose(perm)
    # with X's axis e = W's axis perm[e]; perm[pos[s[d]]] = d.
    perm = [0, 0, 0]
    for d in range(3):
        perm[pos[s[d]]] = d
    return W.transpose(perm)


def triple_weight(i: int, j: int, k: int) -> float:
    """(2 - d_ij - d_jk) for i <= j <= k (reading R4)."""
    return 2.0 - (i == j) - (j == k)


def triple_energy(i: int, j: int, k: int, eps_occ, eps_vir, t1, t2, ints,
                  split: bool = False, progress=None):
    """e_ijk = w_ijk * sum_abc (W + V) Z / D for one occupied triple i<=j<=k.

    With split=True returns (e4, e5): the part from W alone and the part
    from V (E = e4 + e5). progress, if given, is called with a short string
    after each stage (long runs report that they are alive).
    """
    W = w_tensor(i, j, k, ints, t2)
    if progress:
        progress(f"W of {(i, j, k)} formed")
    Vt = v_tensor(i, j, k, ints, t1)
    D = d_tensor(i, j, k, eps_occ, eps_vir)
    Z = z_tensor(W)
    if progress:
        progress(f"V, D, Z of {(i, j, k)} formed")
    w = triple_weight(i, j, k)
    if split:
        return w * _fsum((W * Z / D).ravel()), w * _fsum((Vt * Z / D).ravel())
    return w * _fsum(((W + Vt) * Z / D).ravel())


def _fsum(x: np.ndarray) -> float:
    """Sum with float error compensation (math.fsum is exact-rounded)."""
    import math
    return math.fsum(x.tolist()) if x.size <= 1 << 20 else float(
        math.fsum(np.add.reduceat(x, np.arange(0, x.size, 4096)).tolist()))


def triples(o: int):
    """i <= j <= k, i = j = k left out (their Z vanishes), i-major order."""
    return [(i, j, k) for i in range(o) for j in range(i, o) for k in range(j, o)
            if not (i == j == k)]


def energy(eps_occ, eps_vir, t1, t2, ints, triple_subset=None, split=False):
    """E(T) and the per-triple partials, summed over i<=j<=k (Eq. 1, R4).

    Returns (E, [(i, j, k, e_ijk), ...]); with split=True each entry holds
    (i, j, k, e4, e5) and E is the pair (E4, E5).
    """
    o = len(eps_occ)
    tl = triples(o) if triple_subset is None else [tuple(int(x) for x in t) for t in triple_subset]
    parts = []
    for (i, j, k) in tl:
        if split:
            e4, e5 = triple_energy(i, j, k, eps_occ, eps_vir, t1, t2, ints, split=True)
            parts.append((i, j, k, e4, e5))
        else:
            parts.append((i, j, k, triple_energy(i, j, k, eps_occ, eps_vir, t1, t2, ints)))
    import math
    if split:
        return (math.fsum(p[3] for p in parts), math.fsum(p[4] for p in parts)), parts
    return math.fsum(p[3] for p in parts), parts


def energy_eq1_form(eps_occ, eps_vir, t1, t2, ints):
    """Eq. 1 as printed: sum over a>=b>=c with weight (2 - d_ab - d_bc) and
    over all i, j, k of (W + V)^{abc}_{ijk} times the occupied-permuted
    combination, divided by D. Builds the full 6-index W; tiny sizes only."""
    o, v = t1.shape
    Wf = np.zeros((o, o, o, v, v, v))
    Vf = np.zeros((o, o, o, v, v, v))
    for i in range(o):
        for j in range(o):
            for k in range(o):
                Wf[i, j, k] = w_tensor(i, j, k, ints, t2)
                Vf[i, j, k] = v_tensor(i, j, k, ints, t1)
    total = 0.0
    terms = []
    for a in range(v):
        for b in range(a + 1):
            for c in range(b + 1):
                wabc = 2.0 - (a == b) - (b == c)
                for i in range(o):
                    for j in range(o):
                        for k in range(o):
                            D = (eps_occ[i] + eps_occ[j] + eps_occ[k]
                                 - eps_vir[a] - eps_vir[b] - eps_vir[c])
                            Zo = (4 * Wf[i, j, k, a, b, c] + Wf[j, k, i, a, b, c]
                                  + Wf[k, i, j, a, b, c] - 2 * Wf[j, i, k, a, b, c]
                                  - 2 * Wf[i, k, j, a, b, c] - 2 * Wf[k, j, i, a, b, c])
                            terms.append(wabc * (Wf[i, j, k, a, b, c] + Vf[i, j, k, a, b, c]) * Zo / D)
    import math
    total = math.fsum(terms)
    return total


def energy_all_form(eps_occ, eps_vir, t1, t2, ints):
    """One third of the sum over all i, j, k and all a, b, c (reading R4)."""
    o, v = t1.shape
    import math
    terms = []
    for i in range(o):
        for j in range(o):
            for k in range(o):
                W = w_tensor(i, j, k, ints, t2)
                Vt = v_tensor(i, j, k, ints, t1)
                D = d_tensor(i, j, k, eps_occ, eps_vir)
                terms.append(_fsum(((W + Vt) * z_tensor(W) / D).ravel()))
    return math.fsum(terms) / 3.0
