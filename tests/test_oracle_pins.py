"""Pins for the CPU oracle: things the oracle must satisfy that do not come
from the oracle itself (the textbook spin-orbital formula, algebraic
invariants, closed forms and special cases), plus planted mistakes that at
least one pin must catch."""
import math

import numpy as np
import pytest

import oracle
from oracle import closed_shell as cs
from paper_2512_01055_amd.inputs import make_problem, mp2_doubles

TINY = [(2, 3, 5, 11), (3, 4, 6, 12), (3, 5, 7, 13), (4, 5, 9, 14), (4, 6, 8, 15)]


def _cs_energy(P, split=False, ints=None):
    ints = ints or oracle.DFIntegrals(P.B_oo, P.B_ov, P.B_vv)
    E, parts = oracle.energy(P.eps_occ, P.eps_vir, P.t1, P.t2, ints, split=split)
    return E


def _so_energy(P, split=False):
    eri = oracle.mo_eri_from_df(P.B_oo, P.B_ov, P.B_vv)
    return oracle.so_energy(P.eps_occ, P.eps_vir, P.t1, P.t2, eri, split=split)


@pytest.mark.parametrize("o,v,naux,seed", TINY)
def test_closed_shell_equals_spin_orbital(o, v, naux, seed):
    P = make_problem(o, v, naux, seed, b_std=0.3)
    (e4, e5) = _cs_energy(P, split=True)
    (s4, s5) = _so_energy(P, split=True)
    assert abs(e4 - s4) <= 1e-12 * abs(s4)
    assert abs(e5 - s5) <= 1e-11 * abs(s4)
    assert abs(e5) > 1e-6 * abs(e4)      # the singles term is really exercised


@pytest.mark.parametrize("o,v,naux,seed", TINY[:3])
def test_three_summation_forms_agree(o, v, naux, seed):
    P = make_problem(o, v, naux, seed, b_std=0.3)
    ints = oracle.DFIntegrals(P.B_oo, P.B_ov, P.B_vv)
    E = _cs_energy(P, ints=ints)
    Eall = oracle.energy_all_form(P.eps_occ, P.eps_vir, P.t1, P.t2, ints)
    Eeq1 = oracle.energy_eq1_form(P.eps_occ, P.eps_vir, P.t1, P.t2, ints)
    assert abs(E - Eall) <= 1e-12 * abs(E)
    assert abs(E - Eeq1) <= 1e-12 * abs(E)


def test_doubles_scaling_and_bilinearity():
    P = make_problem(4, 6, 10, 21, b_std=0.3)
    (e4, e5) = _cs_energy(P, split=True)
    lam, mu = 0.5, -1.7
    Q = make_problem(4, 6, 10, 21, b_std=0.3)
    Q.t2 = lam * P.t2
    Q.t1 = mu * P.t1
    E = _cs_energy(Q)
    assert abs(E - (lam ** 2 * e4 + lam * mu * e5)) <= 1e-12 * abs(e4)
    Q.t1 = 0.0 * P.t1
    E0 = _cs_energy(Q)
    assert abs(E0 / e4 - lam ** 2) <= 1e-13


def test_integral_scaling():
    """B -> kB with fixed amplitudes: E -> k^4 E. With amplitudes regenerated
    from kB (t2 ~ k^2): E[4] -> k^8 E[4], E[5] -> k^6 E[5]."""
    P = make_problem(3, 5, 8, 22, b_std=0.3)
    (e4, e5) = _cs_energy(P, split=True)
    k = 0.7
    Q = make_problem(3, 5, 8, 22, b_std=0.3)
    Q.B_oo, Q.B_ov, Q.B_vv = k * P.B_oo, k * P.B_ov, k * P.B_vv
    E = _cs_energy(Q)
    assert abs(E - k ** 4 * (e4 + e5)) <= 1e-12 * abs(e4)
    Q.t2 = mp2_doubles(P.eps_occ, P.eps_vir, Q.B_ov)
    (f4, f5) = _cs_energy(Q, split=True)
    assert abs(f4 - k ** 8 * e4) <= 1e-12 * abs(f4)
    assert abs(f5 - k ** 6 * e5) <= 1e-11 * abs(f4)


@pytest.mark.parametrize("seed", [31, 32, 33])
def test_fourth_order_part_is_never_positive(seed):
    P = make_problem(4, 6, 10, seed, b_std=0.3, with_t1=False)
    ints = oracle.DFIntegrals(P.B_oo, P.B_ov, P.B_vv)
    E, parts = oracle.energy(P.eps_occ, P.eps_vir, P.t1, P.t2, ints)
    assert E < 0
    assert all(p[3] <= 0 for p in parts)


def _relabel(P, po, pv):
    Q = make_problem(P.o, P.v, P.naux, P.seed, b_std=0.3)
    Q.eps_occ = P.eps_occ[po]
    Q.eps_vir = P.eps_vir[pv]
    Q.t1 = P.t1[np.ix_(po, pv)]
    Q.t2 = P.t2[np.ix_(po, po, pv, pv)]
    Q.B_oo = P.B_oo[:, po][:, :, po]
    Q.B_ov = P.B_ov[:, po][:, :, pv]
    Q.B_vv = P.B_vv[:, pv][:, :, pv]
    return Q


def test_relabelling_invariance():
    P = make_problem(4, 6, 10, 41, b_std=0.3)
    E = _cs_energy(P)
    rng = np.random.default_rng(5)
    for _ in range(3):
        Q = _relabel(P, rng.permutation(P.o), rng.permutation(P.v))
        assert abs(_cs_energy(Q) - E) <= 1e-13 * abs(E)


def _rotate(P, U, Vr):
    Q = make_problem(P.o, P.v, P.naux, P.seed, b_std=0.3)
    Q.eps_occ, Q.eps_vir = P.eps_occ.copy(), P.eps_vir.copy()
    Q.B_oo = np.einsum("Qij,ik,jl->Qkl", P.B_oo, U, U)
    Q.B_ov = np.einsum("Qia,ik,ab->Qkb", P.B_ov, U, Vr)
    Q.B_vv = np.einsum("Qab,ac,bd->Qcd", P.B_vv, Vr, Vr)
    Q.t1 = U.T @ P.t1 @ Vr
    Q.t2 = np.einsum("ijab,ik,jl,ac,bd->klcd", P.t2, U, U, Vr, Vr)
    return Q


def _block_rotation(n, idx, seed):
    rng = np.random.default_rng(seed)
    R = np.eye(n)
    q, _ = np.linalg.qr(rng.standard_normal((len(idx), len(idx))))
    R[np.ix_(idx, idx)] = q
    return R


def test_degenerate_rotation_invariance_and_its_teeth():
    P = make_problem(4, 6, 10, 51, b_std=0.3)
    P.eps_occ[1] = P.eps_occ[0]
    P.eps_vir[2] = P.eps_vir[1] = P.eps_vir[0]
    P.t2 = mp2_doubles(P.eps_occ, P.eps_vir, P.B_ov)
    E = _cs_energy(P)
    U = _block_rotation(4, [0, 1], 1)
    Vr = _block_rotation(6, [0, 1, 2], 2)
    Q = _rotate(P, U, Vr)
    assert abs(_cs_energy(Q) - E) <= 1e-12 * abs(E)
    # the same kind of rotation across non-degenerate orbitals must change E
    U2 = _block_rotation(4, [2, 3], 3)
    Q2 = _rotate(P, U2, np.eye(6))
    assert abs(_cs_energy(Q2) - E) > 1e-4 * abs(E)


def test_special_cases_vanish():
    P = make_problem(1, 5, 7, 61, b_std=0.3)        # only i=j=k exists
    assert _cs_energy(P) == 0.0
    assert abs(_so_energy(P)) <= 1e-14
    P = make_problem(3, 1, 7, 62, b_std=0.3)        # a=b=c only: Z = 0
    assert abs(_cs_energy(P)) <= 1e-14
    assert abs(_so_energy(P)) <= 1e-14


def test_df_and_explicit_integrals_agree():
    P = make_problem(3, 5, 8, 71, b_std=0.3)
    E_df = _cs_energy(P)
    ints = oracle.ExplicitIntegrals(*oracle.integrals_from_df(P.B_oo, P.B_ov, P.B_vv))
    E_ex = _cs_energy(P, ints=ints)
    assert abs(E_df - E_ex) <= 1e-13 * abs(E_df)


def test_generator_symmetries_and_reproducibility():
    P = make_problem(4, 7, 9, 81)
    assert np.array_equal(P.t2, P.t2.transpose(1, 0, 3, 2))
    assert np.array_equal(P.B_vv, P.B_vv.transpose(0, 2, 1))
    assert np.array_equal(P.B_oo, P.B_oo.transpose(0, 2, 1))
    Q = make_problem(4, 7, 9, 81)
    for name in ("eps_occ", "eps_vir", "t1", "t2", "B_oo", "B_ov", "B_vv"):
        assert np.array_equal(getattr(P, name), getattr(Q, name))
    assert np.all(P.eps_occ < -0.3 + 1e-12) and np.all(P.eps_vir > 0.1 - 1e-12)


# ---- planted mistakes: each mutated oracle must miss the spin-orbital pin ----

def _w_wrong_amplitude_order(i, j, k, ints, t2):
    occ = (i, j, k)
    v = t2.shape[2]
    o = t2.shape[0]
    W = np.zeros((v, v, v))
    for P in cs.EQ5_PERMS:
        p, q, r = occ[P[0]], occ[P[1]], occ[P[2]]
        A = (ints.ovvv(p).reshape(v * v, v) @ t2[q, r].T).reshape(v, v, v)   # t_qr not t_rq
        A -= (ints.ovoo(p)[:, q, :] @ t2[:, r].reshape(o, v * v)).reshape(v, v, v)
        W += A.transpose(tuple(int(np.argsort(P)[d]) for d in range(3)))
    return W


def _w_no_vooo(i, j, k, ints, t2):
    occ = (i, j, k)
    v = t2.shape[2]
    W = np.zeros((v, v, v))
    for P in cs.EQ5_PERMS:
        p, q, r = occ[P[0]], occ[P[1]], occ[P[2]]
        A = (ints.ovvv(p).reshape(v * v, v) @ t2[r, q].T).reshape(v, v, v)
        W += A.transpose(tuple(int(np.argsort(P)[d]) for d in range(3)))
    return W


def _w_forward_transpose(i, j, k, ints, t2):
    occ = (i, j, k)
    v = t2.shape[2]
    o = t2.shape[0]
    W = np.zeros((v, v, v))
    for P in cs.EQ5_PERMS:
        p, q, r = occ[P[0]], occ[P[1]], occ[P[2]]
        A = (ints.ovvv(p).reshape(v * v, v) @ t2[r, q].T).reshape(v, v, v)
        A -= (ints.ovoo(p)[:, q, :] @ t2[:, r].reshape(o, v * v)).reshape(v, v, v)
        W += A.transpose(P)              # P instead of its inverse
    return W


def _v_swapped(i, j, k, ints, t1):
    return (t1[i][:, None, None] * ints.ovov(j, k)[None, :, :]
            + t1[j][None, :, None] * ints.ovov(i, k)[:, None, :]
            + t1[k][None, None, :] * ints.ovov(j, i)[:, :, None])


MUTATIONS = {
    "drop_one_eq5_term": ("EQ5_PERMS", cs.EQ5_PERMS[:5]),
    "eq4_sign_as_printed": ("d_tensor", None),      # filled in the test
    "amplitude_pair_order": ("w_tensor", _w_wrong_amplitude_order),
    "no_occupied_term": ("w_tensor", _w_no_vooo),
    "forward_permutation": ("w_tensor", _w_forward_transpose),
    "unit_weights": ("triple_weight", lambda i, j, k: 2.0),
    "singles_integral_swapped": ("v_tensor", _v_swapped),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    attr, val = MUTATIONS[name]
    if name == "eq4_sign_as_printed":
        orig = cs.d_tensor
        val = lambda i, j, k, eo, ev: -orig(i, j, k, eo, ev)   # noqa: E731
    caught = False
    for (o, v, naux, seed) in TINY[1:4]:
        P = make_problem(o, v, naux, seed, b_std=0.3)
        ref = _so_energy(P)
        with monkeypatch.context() as m:
            m.setattr(cs, attr, val)
            E = _cs_energy(P)
        if not math.isfinite(E) or abs(E - ref) > 1e-6 * abs(ref):
            caught = True
    assert caught, f"mutation {name} slipped past the spin-orbital pin"


def test_compensated_sum_of_large_arrays():
    """Above 2^20 elements (every triple with v >= 102) the oracle's per-triple
    sum adds 4096-element blocks in order and then sums the block totals
    exactly. Against math.fsum of the whole array (exactly rounded) it must
    stay within the error bound of one block's sequential sum, 4096 u sum|x|.
    The array cancels heavily, has a ragged last block holding its largest
    element, and every element is far above the bound, so a block, an
    element or the tail left out is caught (the last check plants that)."""
    rng = np.random.default_rng(5)
    n = (1 << 21) + 1237
    x = rng.choice([-1.0, 1.0], n) * rng.uniform(1e-3, 2e-3, n)
    big = rng.choice(n - 1, 64, replace=False)
    x[big[:32]] = rng.uniform(1e2, 1e3, 32)         # large values that cancel in pairs
    x[big[32:]] = -x[big[:32]]
    x[-1] = 2.5e3
    exact = math.fsum(x.tolist())
    bound = 4096 * 2.0 ** -53 * float(np.abs(x).sum())
    assert np.abs(x).min() > 1e3 * bound
    got = cs._fsum(x)
    assert abs(got - exact) <= bound
    # the same with the array length a multiple of the block size
    y = x[:1 << 21]
    assert abs(cs._fsum(y) - math.fsum(y.tolist())) <= bound
    # small arrays take math.fsum itself: exactly rounded
    z = x[:1 << 20]
    assert cs._fsum(z) == math.fsum(z.tolist())
    # planted mistake: the ragged last block dropped
    full = n // 4096 * 4096
    dropped = math.fsum(x[:full].reshape(-1, 4096).sum(1).tolist())
    assert abs(dropped - exact) > 1e3 * bound
