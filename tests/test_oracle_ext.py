"""The oracle's integrator and window code driving force fields of the other
oracle files (the message-passing target, the pair and learned drafts)
through its external kind: the plumbing hands back each field's own forces
bit for bit, and the window pins hold with them (Alg. 1 with a draft equal
to the target is plain Langevin of Eq. aboba; the step-keyed stream makes
the committed trajectory independent of K)."""
import numpy as np


def _liquid():
    from paper_2606_02455_amd import workloads as W
    return W.triatomic_replicas(n_replicas=1, seed=5)  # 138 atoms, box over 2 rc


def _net():
    from oracle.mpnn import MPNN
    from paper_2606_02455_amd import workloads as W
    return MPNN(W.mpnn_weights(3, seed=17), 3, rc=5.0, scale=1.0)


def _system(ora, w):
    return ora.System(w.n_atoms, float(w.box[0]), w.masses(), w.dt, w.gamma, w.kT,
                      w.force_unit)


def _drafts(w, seed=3, B=8):
    from oracle.net import NetDraft
    from oracle.pair import PairDraft
    rng = np.random.default_rng(seed)
    pair = PairDraft(3, B, 4.0, w=rng.normal(size=(6, B)) * 0.05)
    net = NetDraft(3, B, 4.0, rng.normal(size=NetDraft.count(3, B)) * 0.02)
    return pair, net


def test_external_fields_return_the_fields_own_forces(ora):
    w = _liquid()
    L = float(w.box[0])
    x = w.positions
    net = _net()
    E, F = net.energy_forces(w.species, x, L)
    E2, F2 = ora.energy_forces(ora.Potential.mpnn(net, w.species), x, L)
    assert E2 == E and np.array_equal(F2, F)
    pair, nd = _drafts(w)
    _, Fp = ora.energy_forces(ora.Potential.pair_draft(pair, w.species), x, L)
    assert np.array_equal(Fp, pair.forces(w.species, x, L))
    _, Fn = ora.energy_forces(ora.Potential.net_draft(nd, w.species), x, L)
    assert np.array_equal(Fn, nd.forces(w.species, x, L))
    assert np.abs(F).max() > 0 and np.abs(Fp).max() > 0 and np.abs(Fn).max() > 0


def test_network_target_as_its_own_draft_is_plain_langevin(ora):
    w = _liquid()
    sysm = _system(ora, w)
    T = ora.Potential.mpnn(_net(), w.species)
    n = w.n_atoms
    q1, p1, i1 = w.positions.copy(), w.momenta.copy(), np.zeros((n, 3), np.int32)
    st, tq, tp = ora.lsd_run(sysm, T, T, q1, p1, i1, seed=4, replica=0, step0=0, n_steps=8,
                             K=4, record=True)
    assert st["rejections"] == 0 and st["committed"] == 8
    q2, p2, i2 = w.positions.copy(), w.momenta.copy(), np.zeros((n, 3), np.int32)
    _, pq, pp = ora.plain_run(sysm, T, q2, p2, i2, seed=4, replica=0, step0=0, n_steps=8,
                              record=True)
    assert np.array_equal(tq, pq) and np.array_equal(tp, pp) and np.array_equal(i1, i2)


def test_learned_draft_windows_do_not_depend_on_the_window_length(ora):
    w = _liquid()
    sysm = _system(ora, w)
    T = ora.Potential.mpnn(_net(), w.species)
    _, nd = _drafts(w)
    D = ora.Potential.net_draft(nd, w.species)
    n = w.n_atoms
    runs = []
    for K in (1, 3):
        q, p, img = w.positions.copy(), w.momenta.copy(), np.zeros((n, 3), np.int32)
        st, tq, tp = ora.lsd_run(sysm, T, D, q, p, img, seed=6, replica=0, step0=0, n_steps=6,
                                 K=K, record=True)
        assert st["committed"] == 6
        runs.append((st["rejections"], tq, tp, img))
    assert runs[0][0] == runs[1][0] and runs[0][0] > 0
    for a, b in zip(runs[0][1:], runs[1][1:]):
        assert np.array_equal(a, b)
