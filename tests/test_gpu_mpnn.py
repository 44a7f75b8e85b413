"""GPU parity of the message-passing target (batched over the K frames of a
window) against the FP64 oracle, on identical binary32 frames.

Tolerance: the network is evaluated in binary32 through three layers and
their reverse pass (128-term products, 16-term radial products, sums over
~30 messages); forces are required to agree to 1e-4 of the largest oracle
force component and energies to 1e-5 relative."""
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from paper_2606_02455_amd import workloads as W

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
FORCE_TOL = 1e-4
ENERGY_TOL = 1e-5


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no GPU")
    return T


@pytest.fixture(scope="module")
def lsd(torch):
    from paper_2606_02455_amd import lsd as L
    L.load()
    return L


def c3_scale():
    for line in open(os.path.join(HERE, "golden", "mpnn_c3_scale.txt")):
        if line.startswith("scale"):
            return float(line.split("=")[1])
    raise RuntimeError("scale missing")


def _target(scale):
    return dict(kind="mpnn", rc=5.0, weights=W.mpnn_weights(3, seed=17), n_model_species=3,
                scale=scale)


def _zero_draft(w):
    return dict(kind="harmonic", k=0.0, anchor=w.positions)


def _atom_box(w):
    """Box edge of every atom's replica, [N, 1]."""
    return np.repeat(np.asarray(w.box, np.float64), np.diff(w.atom_offsets))[:, None]


def _frames(w, K, seed, amp=0.05):
    rng = np.random.default_rng(seed)
    L = _atom_box(w)
    fr = W.f32(np.mod(w.positions[None] + rng.uniform(-amp, amp, (K,) + w.positions.shape), L))
    fr = np.where(fr >= L[None], 0.0, fr)
    return fr


def _inject(g, torch, qm, pd, fd):
    win = g.window()
    K, N = qm.shape[:2]
    L = _atom_box(g.w)[None]
    qc = qm.copy()
    qc[1:] -= L * np.round((qc[1:] - qc[0][None]) / L)
    q4 = np.zeros((K, N, 4), np.float32)
    q4[:, :, :3] = qc
    win["q_mid"][:K].copy_(torch.tensor(q4))
    win["p_draft"][:K + 1].copy_(torch.tensor(np.transpose(pd, (0, 2, 1)).astype(np.float32)))
    win["f_draft"][:K].copy_(torch.tensor(np.transpose(fd, (0, 2, 1)).astype(np.float32)))
    torch.cuda.synchronize()


def _check_frames(torch, lsd, ora, w, K, scale, seed):
    from oracle.mpnn import MPNN
    net = MPNN(W.mpnn_weights(3, seed=17), 3, rc=5.0, scale=scale)
    g = lsd.LSDSystem(w, mode="lsd", target=_target(scale), draft=_zero_draft(w), k_max=K)
    qm = _frames(w, K, seed)
    rng = np.random.default_rng(seed + 1)
    sig = np.sqrt(w.masses() * w.kT * w.force_unit)[:, None]
    pd = W.f32(rng.normal(size=(K + 1,) + w.positions.shape) * sig)
    fd = np.zeros_like(qm)
    _inject(g, torch, qm, pd, fd)
    g.mark_drafted(K)
    g.verify_window()
    g.accept_rollback(sync=True)
    assert g.status() == 0
    ft = g.window()["f_target"][:K].cpu().numpy().transpose(0, 2, 1).astype(np.float64)
    en = g.energy.cpu().numpy()[0]
    inv = g.window()["frame_invalid"].cpu().numpy()[0]
    assert not inv[:K].any()
    L = float(w.box[0])
    with ThreadPoolExecutor(max_workers=min(K, 16)) as ex:
        refs = list(ex.map(lambda k: net.energy_forces(w.species, qm[k], L), range(K)))
    worst = 0.0
    for k, (E, F) in enumerate(refs):
        err = np.abs(ft[k] - F).max() / np.abs(F).max()
        worst = max(worst, err)
        assert err <= FORCE_TOL, (k, err)
        assert abs(en[k] - E) <= ENERGY_TOL * abs(E), (k, en[k], E)
    _say(f"  worst force error / max|F| = {worst:.2e}")
    g.destroy()


def _check_replica_frames(torch, lsd, ora, w, K, scale, seed, amp=0.05):
    """Per replica and frame: forces and energies of the batched evaluation
    against the oracle's evaluation of that replica alone."""
    from oracle.mpnn import MPNN
    net = MPNN(W.mpnn_weights(3, seed=17), 3, rc=5.0, scale=scale)
    g = lsd.LSDSystem(w, mode="lsd", target=_target(scale), draft=_zero_draft(w), k_max=K)
    qm = _frames(w, K, seed, amp)
    rng = np.random.default_rng(seed + 1)
    sig = np.sqrt(w.masses() * w.kT * w.force_unit)[:, None]
    pd = W.f32(rng.normal(size=(K + 1,) + w.positions.shape) * sig)
    _inject(g, torch, qm, pd, np.zeros_like(qm))
    g.mark_drafted(K)
    g.verify_window()
    g.accept_rollback(sync=True)
    assert g.status() == 0
    ft = g.window()["f_target"][:K].cpu().numpy().transpose(0, 2, 1).astype(np.float64)
    en = g.energy.cpu().numpy()
    inv = g.window()["frame_invalid"].cpu().numpy()
    assert not inv[:, :K].any()
    jobs = [(r, k) for r in range(w.n_replicas) for k in range(K)]

    def ref(job):
        r, k = job
        sl = w.replica_slice(r)
        return net.energy_forces(w.species[sl], qm[k, sl], float(w.box[r]))

    with ThreadPoolExecutor(max_workers=16) as ex:
        refs = list(ex.map(ref, jobs))
    worst = 0.0
    for (r, k), (E, F) in zip(jobs, refs):
        sl = w.replica_slice(r)
        err = np.abs(ft[k, sl] - F).max() / np.abs(F).max()
        worst = max(worst, err)
        assert err <= FORCE_TOL, (r, k, err)
        assert abs(en[r, k] - E) <= ENERGY_TOL * abs(E), (r, k, en[r, k], E)
    _say(f"  {len(jobs)} replica frames, worst force error / max|F| = {worst:.2e}")
    g.destroy()


def test_mpnn_target_small_system(torch, lsd, ora):
    _say("mpnn 96 atoms")
    w = W.triatomic_liquid(32, seed=8, K=4)
    _check_frames(torch, lsd, ora, w, 4, c3_scale(), seed=2)


def test_mpnn_target_full_c3_window(torch, lsd, ora):
    _say("mpnn c3 window")
    w = W.config("c3")
    _check_frames(torch, lsd, ora, w, w.K, c3_scale(), seed=3)


def test_mpnn_plain_stepping(torch, lsd, ora):
    _say("mpnn plain steps")
    from oracle.mpnn import MPNN
    w = W.triatomic_liquid(32, seed=9, K=4)
    scale = c3_scale()
    g = lsd.LSDSystem(w, mode="plain", target=_target(scale))
    g.draft_steps(2)
    torch.cuda.synchronize()
    win = g.window()
    q0 = win["q_mid"][0, :, :3].cpu().numpy().astype(np.float64)
    fd0 = win["f_draft"][0].cpu().numpy().T.astype(np.float64)
    L = float(w.box[0])
    net = MPNN(W.mpnn_weights(3, seed=17), 3, rc=5.0, scale=scale)
    E, F = net.energy_forces(w.species, np.mod(q0, L), L)
    assert np.abs(fd0 - F).max() <= FORCE_TOL * np.abs(F).max()
    g.accept_rollback(sync=True)
    g.run_windows(3, 4)
    st = g.state()
    assert np.isfinite(st["p"]).all() and int(st["step"][0]) >= 3
    g.destroy()


def test_mpnn_target_ragged_replicas_with_images(torch, lsd, ora):
    # the batched-replica regime: boxes of 8-20 molecules (7.3-9.9 A edges,
    # under 2 rc), so every replica is one cell with 27 images, edges reach
    # periodic copies of the neighbours and of the atom itself, and tiles and
    # edge blocks straddle replicas of uneven size
    _say("mpnn ragged replicas (multi-image)")
    w = W.triatomic_replicas(24, n_mol_lo=8, n_mol_hi=20, seed=44, K=3)
    assert (np.asarray(w.box) < 10.0).all()
    _check_replica_frames(torch, lsd, ora, w, 3, c3_scale(), seed=5, amp=0.04)


def test_mpnn_target_full_size_c5_frames(torch, lsd, ora):
    # the precision-at-scale system (24 576 atoms), two frames
    _say("mpnn c5 size, 2 frames")
    w = W.config("c5")
    _check_frames(torch, lsd, ora, w, 2, c3_scale(), seed=6)


def test_network_launch_shapes_give_identical_results(torch, lsd):
    # the autotuner's candidates for the network evaluation (blocks of the
    # pair-filter kernel x rows per row-chain block) change only which block
    # computes what: forces and energies are equal bit for bit
    _say("mpnn launch shapes")
    w = W.triatomic_replicas(n_replicas=3, n_mol_lo=10, n_mol_hi=20, seed=51, K=4)
    K = 4
    scale = c3_scale()
    qm = _frames(w, K, 52)
    rng = np.random.default_rng(53)
    sig = np.sqrt(w.masses() * w.kT * w.force_unit)[:, None]
    pd = W.f32(rng.normal(size=(K + 1,) + w.positions.shape) * sig)
    ref = None
    for c in range(9):
        g = lsd.LSDSystem(w, mode="lsd", target=_target(scale), draft=_zero_draft(w), k_max=K)
        g.set_verify_variant(K, c)
        _inject(g, torch, qm, pd, np.zeros_like(qm))
        g.mark_drafted(K)
        g.verify_window()
        g.accept_rollback(sync=True)
        assert g.status() == 0
        out = (g.window()["f_target"][:K].cpu().numpy().copy(), g.energy.cpu().numpy().copy(),
               g.log_ratio.cpu().numpy().copy())
        if ref is None:
            ref = out
        else:
            for x, y in zip(out, ref):
                assert np.array_equal(x, y), c
        g.destroy()


def test_network_autotuned_windows_equal_untuned(torch, lsd):
    _say("mpnn autotuned vs untuned windows")
    w = W.triatomic_replicas(n_replicas=3, n_mol_lo=8, n_mol_hi=16, seed=54, K=4)
    tgt = dict(kind="mpnn", rc=5.0, weights=W.mpnn_weights(3, seed=17), n_model_species=3,
               scale=0.1 * W.MPNN_C3_SCALE)
    a = lsd.LSDSystem(w, mode="lsd", target=tgt, draft=_zero_draft(w), error_correction=2)
    b = lsd.LSDSystem(w, mode="lsd", target=tgt, draft=_zero_draft(w), error_correction=2)
    chosen, us = b.autotune_verify(4, repeats=2)
    assert 0 <= chosen < 9 and len(us) == 9 and all(v > 0 for v in us.values())
    b.verify_window()
    b.accept_rollback()
    a.draft_steps(4)
    a.verify_window()
    a.accept_rollback()
    for rep in range(3):
        a.run_windows(4, 4)
        b.run_windows(4, 4)
        sa, sb = a.state(), b.state()
        for k in ("q", "p", "img", "step"):
            assert np.array_equal(sa[k], sb[k]), (rep, k)
        assert np.array_equal(a.counters(), b.counters())
    assert a.counters()[:, 1].sum() > a.counters()[:, 0].sum()
    a.destroy()
    b.destroy()
