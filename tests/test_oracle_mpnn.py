"""Oracle pins of the message-passing target (random-init weights).

The network is a stand-in for the paper's external interatomic potentials;
its forces are pinned by the definition F = -dU/dq (Sec. 2.1) through
central finite differences, by the invariances of an interatomic
potential, by smoothness at the cutoff, and by the isolated-atom closed
form of the readout."""
import numpy as np
import pytest

from paper_2606_02455_amd import workloads as W


@pytest.fixture(scope="module")
def net(ora):
    from oracle.mpnn import MPNN
    return MPNN(W.mpnn_weights(3, seed=17), 3, rc=5.0, scale=1.0)


def _small_liquid(n_mol=16, seed=5):
    w = W.triatomic_liquid(n_mol, seed=seed)
    return w.positions, w.species, float(w.box[0])


def test_mpnn_forces_are_minus_energy_gradient(net):
    x, sp, L = _small_liquid()
    E, F = net.energy_forces(sp, x, L)
    rng = np.random.default_rng(0)
    h = 1e-5
    for _ in range(10):
        i, a = int(rng.integers(len(x))), int(rng.integers(3))
        xp, xm = x.copy(), x.copy()
        xp[i, a] += h
        xm[i, a] -= h
        fd = -(net.energy_forces(sp, xp, L, False)[0] - net.energy_forces(sp, xm, L, False)[0]) / (2 * h)
        assert fd == pytest.approx(F[i, a], rel=1e-6, abs=1e-8 * np.abs(F).max())


def test_mpnn_invariances(net):
    x, sp, L = _small_liquid()
    E, F = net.energy_forces(sp, x, L)
    assert np.abs(F.sum(0)).max() < 1e-10 * np.abs(F).max()
    ax = [1, 2, 0]
    E2, F2 = net.energy_forces(sp, x[:, ax], L)
    assert E2 == pytest.approx(E, rel=1e-12)
    assert np.allclose(F2, F[:, ax], rtol=1e-9, atol=1e-10 * np.abs(F).max())
    perm = np.random.default_rng(3).permutation(len(x))
    E3, F3 = net.energy_forces(sp[perm], x[perm], L)
    assert E3 == pytest.approx(E, rel=1e-12)
    assert np.allclose(F3, F[perm], rtol=1e-9, atol=1e-10 * np.abs(F).max())
    t = np.mod(x + np.array([1.3, -2.1, 0.7]), L)
    E4, F4 = net.energy_forces(sp, t, L)
    assert E4 == pytest.approx(E, rel=1e-11)


def test_mpnn_isolated_atoms_closed_form(net):
    # atoms farther apart than the cutoff: no messages, h = embedding, so E is
    # the readout of the embeddings and every force vanishes
    sp = np.array([0, 1, 2, 1], np.int32)
    L = 40.0
    x = np.array([[1.0, 1.0, 1.0], [11.0, 1.0, 1.0], [1.0, 11.0, 1.0], [11.0, 11.0, 21.0]])
    E, F = net.energy_forces(sp, x, L)
    shapes = dict(W.mpnn_weight_shapes(3))
    off, parts = 0, {}
    for name, shp in W.mpnn_weight_shapes(3):
        k = int(np.prod(shp))
        parts[name] = net.w[off:off + k].reshape(shp)
        off += k
    h = parts["W_emb"][sp]
    y = h @ parts["W1"].T + parts["b1"]
    silu = y / (1 + np.exp(-y))
    E_ref = float((silu @ parts["w2"] + parts["b2"][0]).sum())
    assert E == pytest.approx(E_ref, rel=1e-12)
    assert np.all(F == 0.0)


def test_mpnn_smooth_at_cutoff(net):
    # a pair crossing the cutoff changes E continuously (f_c(rc) = 0)
    sp = np.array([0, 2], np.int32)
    L = 40.0
    Es = []
    for r in (5.0 - 1e-6, 5.0 + 1e-6):
        x = np.array([[10.0, 10.0, 10.0], [10.0 + r, 10.0, 10.0]])
        Es.append(net.energy_forces(sp, x, L)[0])
    assert abs(Es[0] - Es[1]) < 1e-9


def test_mpnn_energy_scales_linearly(ora):
    from oracle.mpnn import MPNN
    x, sp, L = _small_liquid(8)
    a = MPNN(W.mpnn_weights(3, seed=17), 3, scale=1.0).energy_forces(sp, x, L)
    b = MPNN(W.mpnn_weights(3, seed=17), 3, scale=2.5).energy_forces(sp, x, L)
    assert b[0] == pytest.approx(2.5 * a[0], rel=1e-14)
    assert np.allclose(b[1], 2.5 * a[1], rtol=1e-13, atol=0)


def _special_weights():
    """Weights under which one layer and the readout reduce to a short
    scalar expression: only hidden channels 3, 7 and 9 and basis index 5
    (b = 6) carry signal, and every matrix used is off-diagonal, so a
    transposed operand or a shifted basis index changes the result."""
    parts = {name: np.zeros(shp) for name, shp in W.mpnn_weight_shapes(3)}
    parts["W_emb"][0, 7], parts["W_emb"][0, 9] = 0.8, -0.3
    parts["W_emb"][2, 7], parts["W_emb"][2, 9] = 0.5, 1.1
    parts["W_emb"][1, 7], parts["W_emb"][1, 9] = -0.6, 0.4
    parts["A1_0"][3, 5] = 1.0            # hidden 3 <- basis b = 6
    parts["a1_0"][3] = 0.2
    parts["A2_0"][7, 3], parts["A2_0"][9, 3] = 2.0, -1.5
    parts["a2_0"][7] = 0.25
    parts["B_0"][7, 9], parts["B_0"][9, 7] = 1.3, 0.7
    parts["C1_0"][7, 9], parts["C1_0"][9, 7] = 0.9, 1.2
    parts["c1_0"][9] = -0.1
    parts["C2_0"][7, 7], parts["C2_0"][9, 9] = 1.0, -0.8
    parts["c2_0"][7] = 0.05
    parts["W1"][0, 7], parts["W1"][1, 9] = 1.0, 1.0
    parts["b1"][0] = 0.05
    parts["w2"][0], parts["w2"][1] = 1.0, 0.5
    parts["b2"][0] = 0.1
    return np.concatenate([parts[n].ravel() for n, _ in W.mpnn_weight_shapes(3)])


def _silu(x):
    return x / (1.0 + np.exp(-x))


def _special_energy(sp, x, rc, scale):
    # scalar form of the network under _special_weights (no periodic images)
    emb = {0: (0.8, -0.3), 1: (-0.6, 0.4), 2: (0.5, 1.1)}
    E = 0.0
    for i in range(len(x)):
        h7, h9 = emb[int(sp[i])]
        m7 = m9 = 0.0
        for j in range(len(x)):
            r = np.linalg.norm(x[j] - x[i])
            if j == i or r >= rc:
                continue
            e6 = np.sqrt(2.0 / rc) * np.sin(6 * np.pi * r / rc) / r
            s = _silu(e6 + 0.2)
            fc = 0.5 * (np.cos(np.pi * r / rc) + 1.0)
            g7, g9 = emb[int(sp[j])]
            m7 += fc * (2.0 * s + 0.25) * (1.3 * g9)
            m9 += fc * (-1.5 * s) * (0.7 * g7)
        n7 = h7 + 1.0 * _silu(0.9 * m9) + 0.05
        n9 = h9 - 0.8 * _silu(1.2 * m7 - 0.1)
        E += _silu(n7 + 0.05) + 0.5 * _silu(n9) + 0.1
    return scale * E


def test_mpnn_special_weights_reduce_to_scalar_form(ora):
    from oracle.mpnn import MPNN
    net = MPNN(_special_weights(), 3, rc=5.0, scale=1.7)
    L = 40.0
    sp = np.array([0, 2, 1, 0], np.int32)
    rng = np.random.default_rng(11)
    for trial in range(5):
        # four atoms within a few Angstrom: some pairs inside, some outside rc
        x = 10.0 + rng.uniform(0.0, 6.0, size=(4, 3))
        E, F = net.energy_forces(sp, x, L)
        assert E == pytest.approx(_special_energy(sp, x, 5.0, 1.7), rel=1e-12, abs=1e-12)
        h = 1e-6
        for i in range(4):
            for a in range(3):
                xp, xm = x.copy(), x.copy()
                xp[i, a] += h
                xm[i, a] -= h
                fd = -(_special_energy(sp, xp, 5.0, 1.7) - _special_energy(sp, xm, 5.0, 1.7)) / (2 * h)
                assert F[i, a] == pytest.approx(fd, rel=1e-5, abs=1e-7)


def test_workload_energy_scale_is_the_golden_value():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "mpnn_c3_scale.txt")
    val = [float(l.split("=")[1]) for l in open(path) if l.startswith("scale")][0]
    assert W.MPNN_C3_SCALE == val
