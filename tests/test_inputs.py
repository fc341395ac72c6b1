"""CPU checks of the seeded input recipe: the orbital-energy ranges, the
spreads of the factors and singles, the MP2-like doubles, and the triple
lists both sides iterate over."""
import numpy as np

from paper_2512_01055_amd import inputs


def test_recipe_ranges_and_spreads():
    P = inputs.make_problem(12, 60, 180, 21)
    assert np.all((P.eps_occ >= -1.5) & (P.eps_occ <= -0.3))
    assert np.all((P.eps_vir >= 0.1) & (P.eps_vir <= 3.0))
    # 129,600 draws: the sample spread is within 1% of 0.05
    assert abs(P.B_ov.std() - 0.05) < 5e-4 and abs(P.B_ov.mean()) < 5e-4
    iu = np.triu_indices(P.v)
    up = P.B_vv[:, iu[0], iu[1]]
    assert abs(up.std() - 0.05) < 5e-4
    # 720 draws: within 10% of 1e-3
    assert abs(P.t1.std() - 1e-3) < 1e-4
    Q = inputs.make_problem(12, 60, 180, 21, with_t1=False)
    assert not Q.t1.any() and np.array_equal(Q.t2, P.t2)


def test_doubles_are_mp2_like():
    P = inputs.make_problem(5, 14, 30, 22)
    iajb = np.einsum("Qia,Qjb->ijab", P.B_ov, P.B_ov)
    den = (P.eps_occ[:, None, None, None] + P.eps_occ[None, :, None, None]
           - P.eps_vir[None, None, :, None] - P.eps_vir[None, None, None, :])
    ref = iajb / den
    assert np.abs(P.t2 - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.all(den < 0)          # occupied below virtual: no vanishing denominator


def test_triple_lists():
    for o in (1, 2, 3, 7):
        t = inputs.triple_list(o)
        assert len(t) == o * (o + 1) * (o + 2) // 6 - o
        assert all(i <= j <= k and not (i == j == k) for i, j, k in t)
        assert len({tuple(x) for x in t}) == len(t)
        keys = [tuple(x) for x in t]
        assert keys == sorted(keys)                         # i-major order
    s = inputs.sample_triples(9, 8, 3)
    allt = [tuple(x) for x in inputs.triple_list(9)]
    pos = [allt.index(tuple(x)) for x in s]
    assert len(s) == 8 and pos == sorted(set(pos))
    assert any(i == j < k for i, j, k in s) and any(i < j == k for i, j, k in s)


def test_factors_sit_on_the_exact_grid():
    P = inputs.make_problem(6, 20, 40, 31)
    for B in (P.B_oo, P.B_ov, P.B_vv):
        scaled = B * inputs.GRID
        assert np.array_equal(scaled, np.rint(scaled))
    with np.testing.assert_raises(ValueError):     # sums could leave the exact range
        inputs.make_problem(2, 3, 40, 31, b_std=20.0)


def test_integrals_do_not_depend_on_summation_order():
    """(ia|jb) from a BLAS product, from a left-to-right loop and from a
    right-to-left loop are the same bits, and equal the exactly rounded sum."""
    import math
    P = inputs.make_problem(3, 9, 50, 32)
    L = P.B_ov.reshape(P.naux, -1)
    blas = L.T @ L
    fwd = np.zeros_like(blas)
    for q in range(P.naux):
        fwd += np.outer(L[q], L[q])
    bwd = np.zeros_like(blas)
    for q in reversed(range(P.naux)):
        bwd += np.outer(L[q], L[q])
    assert np.array_equal(blas, fwd) and np.array_equal(blas, bwd)
    for (x, y) in ((0, 0), (4, 17), (26, 3)):
        assert blas[x, y] == math.fsum(L[:, x] * L[:, y])


def test_doubles_formed_three_ways_are_bitwise_equal():
    """The host recipe, the on-demand pairs and the torch formation used for
    problems too large for host memory (run here on the CPU) agree bit for
    bit."""
    o, v, naux, seed = 5, 24, 60, 33
    P = inputs.make_problem(o, v, naux, seed)
    lazy = inputs.LazyDoubles(P.eps_occ, P.eps_vir, P.B_ov)
    for (i, j) in ((0, 0), (1, 3), (4, 2)):
        assert np.array_equal(lazy[i, j], P.t2[i, j])
    assert np.array_equal(lazy[:, 2], P.t2[:, 2])
    D = inputs.make_problem_device(o, v, naux, seed, device="cpu")
    assert np.array_equal(D.t2.numpy(), P.t2)
    for n in ("eps_occ", "eps_vir", "t1", "B_oo", "B_ov", "B_vv"):
        assert np.array_equal(getattr(D, n).numpy(), getattr(P, n))
