"""The allocation-free kinetic-energy entry point (static device scratch)
against lsd_kinetic_energy with caller scratch: the same kernels and order,
so results are equal bit for bit.  Two calls in a row, the second on a
smaller input, check that nothing left in the shared array by the first call
leaks into the second; the capacity limit is rejected cleanly."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _inputs(n_replicas, seed):
    from paper_2606_02455_amd import workloads as W
    w = W.triatomic_replicas(n_replicas=n_replicas, seed=seed)
    off = np.asarray(w.atom_offsets, np.int32)
    p = w.momenta.T.astype(np.float32).copy()
    return p, w.species.astype(np.int32), w.species_mass, off


def _both(p, sp, masses, off):
    import torch
    from paper_2606_02455_amd import lsd
    pt = torch.tensor(p, device="cuda")
    st = torch.tensor(sp, device="cuda")
    ot = torch.tensor(off, device="cuda")
    nmax = int(np.diff(off).max())
    ref = lsd.kinetic_energy(pt, st, masses, ot, nmax).cpu().numpy()
    out = torch.full((off.shape[0] - 1,), float("nan"), dtype=torch.float64, device="cuda")
    got = lsd.kinetic_energy_noalloc(pt, st, masses, ot, nmax, out).cpu().numpy()
    return got, ref


def test_noalloc_equals_scratch_variant_on_two_calls_in_a_row():
    p, sp, m, off = _inputs(48, 21)
    got, ref = _both(p, sp, m, off)
    assert np.array_equal(got, ref)
    assert np.all(ref > 0)
    # second call: fewer replicas, and fewer atoms, than the first
    p2, sp2, m2, off2 = _inputs(5, 22)
    assert off2.shape[0] < off.shape[0] and off2[-1] < off[-1]
    got2, ref2 = _both(p2, sp2, m2, off2)
    assert np.array_equal(got2, ref2)


def test_noalloc_large_system_spans_several_chunks():
    from paper_2606_02455_amd import workloads as W
    w = W.config("c5")
    p = w.momenta.T.astype(np.float32).copy()
    off = np.asarray(w.atom_offsets, np.int32)
    got, ref = _both(p, w.species.astype(np.int32), w.species_mass, off)
    assert np.array_equal(got, ref)


def test_noalloc_rejects_requests_beyond_its_array():
    import torch
    from paper_2606_02455_amd import lsd
    # 33 replicas of up to 2000 chunks of 2048 atoms: 66 000 partial sums,
    # above the 65 536 the static array holds; rejected on the host with
    # CAPACITY before any launch (the offsets are never read)
    n = 2048 * 2000
    p = torch.zeros((3, n), dtype=torch.float32, device="cuda")
    off = torch.zeros((34,), dtype=torch.int32, device="cuda")
    out = torch.zeros((33,), dtype=torch.float64, device="cuda")
    with pytest.raises(lsd.LSDError) as e:
        lsd.kinetic_energy_noalloc(p, None, [1.0], off, n, out)
    assert e.value.status == -4  # LSD_ERR_CAPACITY
    # the entry point still works after the rejected call
    p2, sp2, m2, off2 = _inputs(3, 23)
    got, ref = _both(p2, sp2, m2, off2)
    assert np.array_equal(got, ref)
