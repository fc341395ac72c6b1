"""CPU check of the energy kernel's sextet logic: the permutation tables, the
slots it reads the five permuted W values from, and the coefficients of its
Z expression (Eq. 1), all read from the kernel source, rebuild the oracle's
Z box by box and visit every (a, b, c) exactly once.

Slot s of a sextet (A >= B >= C box indices) holds box
(T[P_s[0]], T[P_s[1]], T[P_s[2]]); a slot whose box repeats an earlier one is
not loaded and its readers use the earlier slot.
"""
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2512_01055_amd", "csrc", "te_kernels.hip")
BOX = 8


def _ints(block):
    block = re.sub(r"//[^\n]*", "", block)
    return [int(x) for x in re.findall(r"-?\d+", block)]


def kernel_tables():
    src = open(SRC).read()
    perm = np.array(_ints(re.search(r"c_perm\[6\]\[3\] = \{(.*?)\};", src, re.S).group(1)))
    comp = np.array(_ints(re.search(r"c_comp\[6\]\[6\] = \{(.*?)\};", src, re.S).group(1)))
    slots = {n: int(q) for n, q in
             re.findall(r"const int (s[b-f]) = canon\[c_comp\[s\]\[(\d)\]\] \* BX_S;", src)}
    zexpr = re.search(r"const double z = (.*?);", src, re.S).group(1)
    terms = []
    for sign, coef, _, slot, *order in re.findall(
            r"([+-]?)\s*(?:(\d+\.\d+)\s*\*\s*)?(w0|box\[(s[b-f])\s*\+\s*bxi\((x\d),\s*(x\d),"
            r"\s*(x\d)\)\])", zexpr):
        c = float(coef or 1.0) * (-1.0 if sign == "-" else 1.0)
        if not slot:                                   # w0: the slot's own element
            terms.append((c, None, (0, 1, 2)))
        else:
            terms.append((c, slot, tuple(int(x[1]) for x in order)))
    return perm.reshape(6, 3), comp.reshape(6, 6), slots, terms


def z_by_sextets(W, perm, comp, slots, terms):
    """Z assembled as the kernel does it; returns Z and the visit count of
    every padded (a, b, c)."""
    v = W.shape[0]
    nT = (v + BOX - 1) // BOX
    vp = nT * BOX
    Wp = np.zeros((vp, vp, vp))
    Wp[:v, :v, :v] = W
    Z = np.zeros_like(Wp)
    seen = np.zeros(Wp.shape, dtype=np.int64)
    x = np.indices((BOX, BOX, BOX))
    for A in range(nT):
        for B in range(A + 1):
            for C in range(B + 1):
                T = (A, B, C)
                bx = [tuple(T[perm[s][d]] for d in range(3)) for s in range(6)]
                canon = [next(q for q in range(s + 1) if bx[q] == bx[s]) for s in range(6)]
                box = [Wp[b[0] * BOX:(b[0] + 1) * BOX, b[1] * BOX:(b[1] + 1) * BOX,
                          b[2] * BOX:(b[2] + 1) * BOX] for b in bx]
                for s in range(6):
                    if canon[s] != s:
                        continue
                    z = np.zeros((BOX, BOX, BOX))
                    for c, slot, order in terms:
                        t = s if slot is None else canon[comp[s][slots[slot]]]
                        z += c * box[t][x[order[0]], x[order[1]], x[order[2]]]
                    sl = tuple(slice(b * BOX, (b + 1) * BOX) for b in bx[s])
                    Z[sl] = z
                    seen[sl] += 1
    return Z[:v, :v, :v], seen


def test_tables_follow_their_definition():
    perm, comp, slots, terms = kernel_tables()
    assert sorted(map(tuple, perm)) == sorted(
        {(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)})
    for s in range(6):
        for q in range(6):
            want = tuple(perm[s][perm[q][d]] for d in range(3))
            assert tuple(perm[comp[s][q]]) == want, (s, q)
    assert len(slots) == 5 and len(terms) == 6
    assert sorted(c for c, _, _ in terms) == [-2.0, -2.0, -2.0, 1.0, 1.0, 4.0]


@pytest.mark.parametrize("v", [16, 21, 24])
def test_sextets_rebuild_the_oracle_z(v):
    perm, comp, slots, terms = kernel_tables()
    W = np.random.default_rng(v).standard_normal((v, v, v))
    Z, seen = z_by_sextets(W, perm, comp, slots, terms)
    assert np.all(seen == 1)
    Zo = oracle.closed_shell.z_tensor(W)
    assert np.abs(Z - Zo).max() <= 1e-13 * np.abs(Zo).max()


def test_every_used_table_entry_matters():
    """A wrong entry in any column of the composition table the kernel reads,
    or a wrong slot for any of the five permuted values, changes Z."""
    perm, comp, slots, terms = kernel_tables()
    W = np.random.default_rng(5).standard_normal((24, 24, 24))
    Zo = oracle.closed_shell.z_tensor(W)
    n = 0
    for s in range(6):
        for q in sorted(set(slots.values())):
            for alt in range(6):
                if alt == comp[s][q]:
                    continue
                bad = comp.copy()
                bad[s][q] = alt
                Z, _ = z_by_sextets(W, perm, bad, slots, terms)
                assert np.abs(Z - Zo).max() > 1e-3 * np.abs(Zo).max(), (s, q, alt)
                n += 1
    assert n == 6 * 5 * 5
    for name in slots:
        for q in range(6):
            if q == slots[name]:
                continue
            Z, _ = z_by_sextets(W, perm, comp, dict(slots, **{name: q}), terms)
            assert np.abs(Z - Zo).max() > 1e-3 * np.abs(Zo).max(), (name, q)
