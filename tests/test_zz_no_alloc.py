"""te_energy_triples_noalloc (scratch in a static device array) against
te_energy_triples (scratch allocated per call), through the C ABI."""
import numpy as np
import pytest

from paper_2512_01055_amd.inputs import make_problem, triple_list

pytestmark = pytest.mark.gpu


def _te():
    from paper_2512_01055_amd import te
    return te


def test_noalloc_equals_allocating_entry_point_on_two_calls():
    """A larger problem, then a smaller one: the second call reuses the
    array the first one filled. Both must give bitwise the allocating path's
    partials and sum, in FP64 and in a reduced precision."""
    import torch
    te = _te()
    for (o, v, naux, seed) in ((7, 72, 40, 31), (4, 40, 24, 32)):
        print(f"\n[noalloc o={o} v={v} naux={naux} seed={seed}]", flush=True)
        P = make_problem(o, v, naux, seed)
        tl = triple_list(o)
        with te.Job(P, device=0) as job:
            for prec in ("fp64", "bf16x2"):
                E_a, pt_a, _ = job.energy_triples(tl, prec)      # converts the operands
                E_n, pt_n, st = job.energy_triples_noalloc(tl, prec)
                free0 = torch.cuda.mem_get_info(0)[0]
                E_n2, pt_n2, _ = job.energy_triples_noalloc(tl[::-1], prec)
                free1 = torch.cuda.mem_get_info(0)[0]
                print(f"{prec}: E {E_a:.15e} noalloc {E_n:.15e}; free memory "
                      f"{free0} -> {free1}", flush=True)
                assert st["n_triples"] == len(tl)
                assert np.array_equal(pt_n, pt_a)
                assert E_n == E_a
                assert np.array_equal(pt_n2, pt_a[::-1])
                # the array is in place after the first call: later calls take
                # no device memory
                assert free1 == free0


def test_noalloc_subset_and_errors():
    te = _te()
    P = make_problem(6, 30, 90, 1)
    tl = triple_list(6)
    with te.Job(P, device=0) as job:
        sub = tl[5:17]
        _, pt_a, _ = job.energy_triples(sub, "fp64")
        _, pt_n, _ = job.energy_triples_noalloc(sub, "fp64")
        assert np.array_equal(pt_a, pt_n)
        # no FP32 copy exists yet: the no-allocation path will not make one
        with pytest.raises(te.TeError) as ei:
            job.energy_triples_noalloc(sub, "fp32")
        assert ei.value.status == -1
        # bad triples are rejected like te_energy_triples rejects them
        with pytest.raises(te.TeError):
            job.energy_triples_noalloc([[2, 1, 3]], "fp64")
        # an empty list gives zero
        E0, pt0, _ = job.energy_triples_noalloc(np.zeros((0, 3), np.int32), "fp64")
        assert E0 == 0.0 and len(pt0) == 0


def test_noalloc_rejects_problems_beyond_the_array():
    """v = 288 in FP64: one triple's W shares (3 * 288^3 * 8 bytes) exceed the
    512 MiB array; the call fails with TE_EINVAL and allocates nothing."""
    te = _te()
    P = make_problem(2, 288, 8, 33)
    with te.Job(P, device=0) as job:
        with pytest.raises(te.TeError) as ei:
            job.energy_triples_noalloc([[0, 0, 1]], "fp64")
        assert ei.value.status == -1
        assert "too large" in str(ei.value)
