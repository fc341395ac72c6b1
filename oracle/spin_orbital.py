"""Spin-orbital (T) by brute force, for tiny problems only.

TEST INFRASTRUCTURE ONLY (see closed_shell.py).

This is the textbook spin-orbital expression of the perturbative triples
correction of Raghavachari, Trucks, Pople and Head-Gordon (the paper's
ref. 3), in the form given by Crawford and Schaefer (Rev. Comput. Chem. 14,
2000), written out with explicit 6-index arrays. It shares nothing with the
closed-shell formula of the paper except the inputs, so agreement between the
two pins the closed-shell oracle's index bookkeeping, signs and weights.

  D t_c(ijk,abc) = P(i/jk) P(a/bc) [ sum_e t_jk^ae <ei||bc> - sum_m t_im^bc <ma||jk> ]
  D t_d(ijk,abc) = P(i/jk) P(a/bc) t_i^a <jk||bc>
  E(T)  = (1/36) sum t_c D (t_c + t_d),   D = f_ii + f_jj + f_kk - f_aa - f_bb - f_cc
  P(i/jk) f(ijk) = f(ijk) - f(jik) - f(kji)
  <pq|rs> = (pr|qs) d(s_p, s_r) d(s_q, s_s),  <pq||rs> = <pq|rs> - <pq|sr>

Spin-orbital amplitudes from closed-shell spatial ones:
  t_I^A = t_i^a d(s_I, s_A)
  t_IJ^AB = t_ij^ab d(s_I,s_A) d(s_J,s_B) - t_ij^ba d(s_I,s_B) d(s_J,s_A)
"""
from __future__ import annotations

import numpy as np


def mo_eri_from_df(B_oo, B_ov, B_vv):
    """Full spatial (pq|rs) over all o+v orbitals from symmetric factors."""
    naux, o, v = B_ov.shape
    n = o + v
    B = np.zeros((naux, n, n))
    B[:, :o, :o] = B_oo
    B[:, :o, o:] = B_ov
    B[:, o:, :o] = B_ov.transpose(0, 2, 1)
    B[:, o:, o:] = B_vv
    return np.einsum("Qpq,Qrs->pqrs", B, B)


def so_energy(eps_occ, eps_vir, t1, t2, eri, split=False):
    """(T) energy from explicit spin-orbital arrays.

    eri: spatial (pq|rs) over o occupied then v virtual orbitals.
    With split=True returns (E[4] part, E[5] part).
    """
    o, v = t1.shape
    n = o + v
    # spin orbital P = 2 p + s ; occupied ones first (p < o)
    nso = 2 * n
    spin = np.arange(nso) % 2
    sp = np.arange(nso) // 2
    # <PQ|RS> = (pr|qs) d(sP,sR) d(sQ,sS)
    g = eri[np.ix_(sp, sp, sp, sp)].transpose(0, 2, 1, 3).copy()
    same_pr = spin[:, None] == spin[None, :]
    g *= same_pr[:, None, :, None] * same_pr[None, :, None, :]
    asym = g - g.transpose(0, 1, 3, 2)          # <PQ||RS>

    O = 2 * o
    occ = slice(0, O)
    vir = slice(O, nso)
    f = np.concatenate([np.repeat(eps_occ, 2), np.repeat(eps_vir, 2)])
    fo, fv = f[occ], f[vir]
    so_o = spin[occ]
    so_v = spin[vir]
    io = sp[occ]
    av = sp[vir] - o

    dIA = (so_o[:, None] == so_v[None, :]).astype(float)
    T1 = t1[np.ix_(io, av)] * dIA
    t2a = t2[np.ix_(io, io, av, av)]
    t2b = t2[np.ix_(io, io, av, av)].transpose(0, 1, 3, 2)  # t_ij^ba
    T2 = (t2a * dIA[:, None, :, None] * dIA[None, :, None, :]
          - t2b * dIA[:, None, None, :] * dIA[None, :, :, None])

    # <ei||bc> as [e][i][b][c]; <ma||jk> as [m][a][j][k]; <jk||bc> as [j][k][b][c]
    vovv = asym[vir, occ, vir, vir]
    ovoo = asym[occ, vir, occ, occ]
    oovv = asym[occ, occ, vir, vir]

    # X[i,j,k,a,b,c] = sum_e t_jk^ae <ei||bc> - sum_m t_im^bc <ma||jk>
    X = (np.einsum("jkae,eibc->ijkabc", T2, vovv)
         - np.einsum("imbc,majk->ijkabc", T2, ovoo))
    Y = np.einsum("ia,jkbc->ijkabc", T1, oovv)

    def P_occ(A):  # f(ijk) - f(jik) - f(kji)
        return A - A.transpose(1, 0, 2, 3, 4, 5) - A.transpose(2, 1, 0, 3, 4, 5)

    def P_vir(A):  # f(abc) - f(bac) - f(cba)
        return A - A.transpose(0, 1, 2, 4, 3, 5) - A.transpose(0, 1, 2, 5, 4, 3)

    D = (fo[:, None, None, None, None, None] + fo[None, :, None, None, None, None]
         + fo[None, None, :, None, None, None] - fv[None, None, None, :, None, None]
         - fv[None, None, None, None, :, None] - fv[None, None, None, None, None, :])
    tc = P_occ(P_vir(X)) / D
    td = P_occ(P_vir(Y)) / D
    e4 = np.sum(tc * D * tc) / 36.0
    e5 = np.sum(tc * D * td) / 36.0
    if split:
        return e4, e5
    return e4 + e5
