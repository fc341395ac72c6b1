"""CPU check of the W-build kernel's index table: the twelve terms of Eq. 2
under the six pair permutations of Eq. 5, grouped into three GEMMs by the
virtual index that stands alone, add up to the oracle's W.

The table (X slice, T2 rows, occupied panels and In rows of each GEMM's four
K segments) is read from make_setup in the kernel source, so an edit there
that breaks the grouping fails here without a GPU; the GEMMs themselves are
plain numpy products over the same operand definitions the kernel uses.
"""
import os
import re

import numpy as np
import pytest

import oracle
from paper_2512_01055_amd.inputs import make_problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2512_01055_amd", "csrc", "te_wbuild.hip")
FIELDS = ("xa", "tq", "tr", "op", "om", "ix", "iy")
POSITION = ("xa", "tr", "op")        # index into (i, j, k); tq, ix, iy name i / j / k


def kernel_table():
    """{g: {field: (expr0, expr1)}} from make_setup's three branches."""
    src = open(SRC).read()
    body = re.search(r"make_setup\(int g, int i, int j, int k\)\s*\{(.*?)return s;", src,
                     re.S).group(1)
    branches = re.split(r"if \(g == 0\)|else if \(g == 1\)|else", body)[1:]
    assert len(branches) == 3
    table = {}
    for g, br in enumerate(branches):
        ent = dict(((f, int(q)), e) for f, q, e in
                   re.findall(r"s\.(\w+)\[(\d)\]\s*=\s*(\w+)\s*;", br))
        table[g] = {f: (ent[(f, 0)], ent[(f, 1)]) for f in FIELDS}
    return table


def _resolve(table, g, i, j, k):
    env = {"i": i, "j": j, "k": k}
    occ = (i, j, k)
    s = {}
    for f in FIELDS:
        vals = [int(env.get(e, e)) for e in table[g][f]]
        s[f] = tuple(occ[x] for x in vals) if f in POSITION else tuple(vals)
    return s


def w_from_table(table, i, j, k, X, In, t2):
    """W = G_c + G_a + G_b built as the kernel's three GEMMs:
    C[m][n] = X-segment 0 + transposed X-segment 1 + two occupied segments,
    m over the paired virtual indices, n over the lone one."""
    o, v = t2.shape[0], t2.shape[2]
    W = np.zeros((v, v, v))
    for g in range(3):
        s = _resolve(table, g, i, j, k)
        A0 = X[s["xa"][0]].reshape(v * v, v)
        A1 = X[s["xa"][1]].transpose(1, 0, 2).reshape(v * v, v)
        B0 = t2[s["tq"][0], s["tr"][0]]
        B1 = t2[s["tq"][1], s["tr"][1]]
        C = A0 @ B0.T + A1 @ B1.T
        for seg in range(2):
            p = s["op"][seg]
            panel = t2[p] if s["om"][seg] == 0 else t2[:, p]     # [l][y][z]
            A = panel.reshape(o, v * v).T                          # [m][l]
            B = In[s["ix"][seg], :, s["iy"][seg], :]               # [n][l]
            C += A @ B.T
        C = C.reshape(v, v, v)                                     # [p0][p1][n]
        if g == 0:
            W += C                                                 # a=p0 b=p1 c=n
        elif g == 1:
            W += C.transpose(2, 0, 1)                              # a=n b=p0 c=p1
        else:
            W += C.transpose(0, 2, 1)                              # a=p0 b=n c=p1
    return W


@pytest.fixture(scope="module")
def problem():
    P = make_problem(4, 7, 11, 91, b_std=0.3)
    ovvv, ovoo, _ = oracle.integrals_from_df(P.B_oo, P.B_ov, P.B_vv)
    ints = oracle.DFIntegrals(P.B_oo, P.B_ov, P.B_vv)
    return P, ovvv, -ovoo, ints


TRIPLES = [(0, 0, 1), (0, 1, 1), (0, 1, 2), (1, 2, 3), (2, 2, 3), (0, 3, 3)]


def test_kernel_grouping_reproduces_the_oracle_w(problem):
    P, X, In, ints = problem
    table = kernel_table()
    for (i, j, k) in TRIPLES:
        W = w_from_table(table, i, j, k, X, In, P.t2)
        Wo = oracle.closed_shell.w_tensor(i, j, k, ints, P.t2)
        err = np.abs(W - Wo).max() / np.abs(Wo).max()
        assert err <= 1e-13, ((i, j, k), err)


def test_every_table_entry_matters(problem):
    """Changing any one entry of the table (to another occupied position,
    value or panel orientation) breaks the sum for a triple of distinct
    indices."""
    P, X, In, ints = problem
    table = kernel_table()
    i, j, k = 0, 1, 3
    Wo = oracle.closed_shell.w_tensor(i, j, k, ints, P.t2)
    n = 0
    for g in range(3):
        for f in FIELDS:
            for seg in range(2):
                cur = table[g][f][seg]
                alts = (["0", "1"] if f == "om" else
                        ["0", "1", "2"] if f in POSITION else ["i", "j", "k"])
                for alt in alts:
                    if alt == cur:
                        continue
                    bad = {gg: dict(t) for gg, t in table.items()}
                    e = list(bad[g][f])
                    e[seg] = alt
                    bad[g][f] = tuple(e)
                    W = w_from_table(bad, i, j, k, X, In, P.t2)
                    err = np.abs(W - Wo).max() / np.abs(Wo).max()
                    assert err > 1e-3, (g, f, seg, alt, err)
                    n += 1
    assert n == 3 * 2 * (3 * 2 + 3 * 2 + 1)       # 78 single-entry mutations
