"""Oracle pins of the learned many-body draft (a one-layer direct-force
network over a species-resolved radial descriptor) and of its training.

The forces are pinned by the pair draft they reduce to when the network's
edge coefficients vanish (the pair oracle has its own pins), by closed forms
of a dimer and of a trimer whose middle atom sees both ends, by Newton's
third law, and by translation, permutation and lattice-rotation symmetry.
The loss gradient is pinned by central finite differences of the loss, which
use only the forward pass; the Adam step by its first-step and
constant-gradient closed forms."""
import numpy as np
import pytest

from paper_2606_02455_amd import workloads as W

H = 32


@pytest.fixture(scope="module")
def net(ora):
    from oracle import net as N
    return N


def _random_params(N, S, B, seed, scale=0.3, w2=0.2):
    P = N.NetDraft.count(S, B)
    rng = np.random.default_rng(seed)
    p = rng.normal(scale=scale, size=P)
    d = N.NetDraft(S, B, 4.0, p)
    W1, b1, W2, c = d.split(p)
    W1 *= 1.0 / np.sqrt(S * B)
    W2 *= w2 / scale / np.sqrt(H)
    return p


def _silu(z):
    return z / (1.0 + np.exp(-z))


def _e(r, rc, b=1):
    return 0.5 * (np.cos(np.pi * r / rc) + 1.0) * np.sin(b * np.pi * r / rc) / r


def test_zero_edge_coefficients_give_the_pair_draft(net, ora):
    from oracle.pair import PairDraft
    w = W.triatomic_liquid(64, seed=21)
    S, B, rc, L = 3, 8, 4.0, float(w.box[0])
    p = _random_params(net, S, B, seed=1)
    d = net.NetDraft(S, B, rc, p)
    W1, b1, W2, c = d.split()
    W2[:] = 0.0
    F = d.forces(w.species, w.positions, L)
    ref = PairDraft(S, B, rc, c.copy()).forces(w.species, w.positions, L)
    assert np.max(np.abs(F - ref)) <= 1e-13 * np.max(np.abs(ref))
    assert np.max(np.abs(ref)) > 0.1


def test_dimer_closed_form(net):
    # B = 1; every hidden unit sees the neighbour density with weight alpha,
    # every edge coefficient reads the hidden layer with weight beta
    rc, r, alpha, beta, c0 = 4.0, 1.7, 0.8, -0.05, 0.6
    d = net.NetDraft(1, 1, rc, np.zeros(net.NetDraft.count(1, 1)))
    W1, b1, W2, c = d.split()
    W1[:] = alpha
    W2[:] = beta
    c[:] = c0
    x = np.array([[5.0, 5.0, 5.0], [5.0 + r, 5.0, 5.0]])
    F = d.forces(np.zeros(2, np.int32), x, 30.0)
    e = _e(r, rc)
    v = H * beta * _silu(alpha * e)
    f = e * (c0 + 2.0 * v)     # pushes atom 1 along +x
    assert F[1] == pytest.approx([f, 0.0, 0.0], rel=1e-13, abs=1e-15)
    assert F[0] == pytest.approx([-f, 0.0, 0.0], rel=1e-13, abs=1e-15)


def test_trimer_descriptor_blocks_by_neighbour_species(net):
    # atoms 0 (species 0), 1, 2 (species 1) on a line; 0 and 2 are out of
    # range of each other.  Only the species-1 block of the descriptor is
    # read, so atom 0 sees e(r01), atom 1 sees e(r12) (its species-0
    # neighbour is ignored) and atom 2 sees e(r12)
    rc, r01, r12, alpha, beta = 4.0, 2.0, 2.4, 1.3, 0.07
    S, B = 2, 1
    d = net.NetDraft(S, B, rc, np.zeros(net.NetDraft.count(S, B)))
    W1, b1, W2, c = d.split()
    W1[:, 1] = alpha
    W2[:] = beta
    x = np.array([[5.0, 5.0, 5.0], [5.0 + r01, 5.0, 5.0], [5.0 + r01 + r12, 5.0, 5.0]])
    sp = np.array([0, 1, 1], np.int32)
    F = d.forces(sp, x, 30.0)
    e01, e12 = _e(r01, rc), _e(r12, rc)
    v0 = H * beta * _silu(alpha * e01)
    v1 = H * beta * _silu(alpha * e12)
    v2 = v1
    f01 = e01 * (v0 + v1)
    f12 = e12 * (v1 + v2)
    assert F[0, 0] == pytest.approx(-f01, rel=1e-13)
    assert F[2, 0] == pytest.approx(f12, rel=1e-13)
    assert F[1, 0] == pytest.approx(f01 - f12, rel=1e-12)


def test_symmetries(net):
    w = W.triatomic_liquid(64, seed=22)
    S, B, rc, L = 3, 8, 4.0, float(w.box[0])
    d = net.NetDraft(S, B, rc, _random_params(net, S, B, seed=2))
    x, sp = w.positions, w.species
    F = d.forces(sp, x, L)
    scale = np.max(np.abs(F))
    # Newton's third law: the pair coefficient is symmetric in i and j
    assert np.max(np.abs(F.sum(0))) <= 1e-12 * scale * len(x)
    # translation (with wrapping)
    xs = np.mod(x + np.array([1.3, -2.2, 0.7]), L)
    assert np.max(np.abs(d.forces(sp, xs, L) - F)) <= 1e-11 * scale
    # permutation
    perm = np.random.default_rng(3).permutation(len(x))
    assert np.max(np.abs(d.forces(sp[perm], x[perm], L) - F[perm])) <= 1e-11 * scale
    # a quarter turn about z maps the periodic lattice onto itself
    xr = np.stack([np.mod(-x[:, 1], L), x[:, 0], x[:, 2]], 1)
    Fr = d.forces(sp, xr, L)
    assert np.max(np.abs(Fr - np.stack([-F[:, 1], F[:, 0], F[:, 2]], 1))) <= 1e-11 * scale


def test_gradient_matches_finite_differences(net):
    w = W.triatomic_liquid(16, seed=23)
    S, B, rc, L = 3, 4, 4.0, float(w.box[0])
    p = _random_params(net, S, B, seed=4, w2=0.5)
    d = net.NetDraft(S, B, rc, p)
    Y = np.random.default_rng(5).normal(size=(w.n_atoms, 3))
    sse, g = d.sse_grad(w.species, w.positions, L, Y)
    assert sse == pytest.approx(np.sum((d.forces(w.species, w.positions, L) - Y) ** 2), rel=1e-14)
    h = 1e-5
    fd = np.zeros_like(p)
    for k in range(p.size):
        old = p[k]
        p[k] = old + h
        d.params = p
        up, _ = d.sse_grad(w.species, w.positions, L, Y)
        p[k] = old - h
        dn, _ = d.sse_grad(w.species, w.positions, L, Y)
        p[k] = old
        fd[k] = (up - dn) / (2 * h)
    d.params = p
    # every block of parameters carries gradient
    W1g, b1g, W2g, cg = d.split(g)
    assert min(np.abs(W1g).max(), np.abs(b1g).max(), np.abs(W2g).max(), np.abs(cg).max()) > 1e-3
    assert np.max(np.abs(fd - g)) <= 1e-6 * np.max(np.abs(g)), np.max(np.abs(fd - g))
    # gradients of several frames add
    _, g2 = d.sse_grad(w.species, w.positions, L, Y, grad=g.copy())
    assert np.max(np.abs(g2 - 2 * g)) <= 1e-12 * np.max(np.abs(g))


def test_difference_loss_gradient_matches_finite_differences(net):
    # the loss of the force changes between consecutive frames, with its
    # gradient assembled from per-frame backward passes
    w = W.triatomic_liquid(12, seed=25)
    S, B, rc, L = 3, 4, 4.0, float(w.box[0])
    p = _random_params(net, S, B, seed=9, w2=0.5)
    d = net.NetDraft(S, B, rc, p)
    rng = np.random.default_rng(10)
    frames = [np.mod(w.positions + rng.normal(scale=0.03, size=w.positions.shape), L)
              for _ in range(3)]
    Ys = [rng.normal(size=(w.n_atoms, 3)) for _ in frames]
    sse, g = d.diff_sse_grad(w.species, frames, L, Ys)
    F = [d.forces(w.species, x, L) for x in frames]
    want = sum(np.sum(((F[k + 1] - F[k]) - (Ys[k + 1] - Ys[k])) ** 2) for k in range(2))
    assert sse == pytest.approx(want, rel=1e-13)
    h = 1e-5
    for k in np.random.default_rng(11).choice(p.size, 60, replace=False):
        old = p[k]
        p[k] = old + h
        d.params = p
        up, _ = d.diff_sse_grad(w.species, frames, L, Ys)
        p[k] = old - h
        d.params = p
        dn, _ = d.diff_sse_grad(w.species, frames, L, Ys)
        p[k] = old
        d.params = p
        assert (up - dn) / (2 * h) == pytest.approx(g[k], abs=1e-6 * np.max(np.abs(g))), k
    # with one frame there is no difference and no gradient
    s0, g0 = d.diff_sse_grad(w.species, frames[:1], L, Ys[:1])
    assert s0 == 0.0 and not g0.any()


def test_adam_closed_forms(net):
    lr, eps = 0.01, 1e-8
    p0 = np.array([1.0, -2.0, 0.5, 3.0])
    g = np.array([0.3, -4.0, 0.0, 1e-3])
    p, m, v = p0.copy(), np.zeros(4), np.zeros(4)
    # step 1: bias-corrected moments are g and g^2
    net.adam(p, m, v, g, lr, 1, eps=eps)
    assert np.allclose(p, p0 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    # a constant gradient keeps the corrected moments at g and g^2: equal steps
    for t in range(2, 7):
        net.adam(p, m, v, g, lr, t, eps=eps)
    assert np.allclose(p, p0 - 6 * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-13)
    # the gradient flips sign at step 2: bias-corrected moments in closed form
    p, m, v = p0.copy(), np.zeros(4), np.zeros(4)
    b1, b2 = 0.9, 0.999
    net.adam(p, m, v, g, lr, 1, eps=eps)
    net.adam(p, m, v, -g, lr, 2, eps=eps)
    mh = ((1 - b1) * b1 * g - (1 - b1) * g) / (1 - b1 ** 2)
    vh = ((1 - b2) * b2 * g * g + (1 - b2) * g * g) / (1 - b2 ** 2)
    want = p0 - lr * g / (np.abs(g) + eps) - lr * mh / (np.sqrt(vh) + eps)
    assert np.allclose(p, want, rtol=0, atol=1e-14)


def test_training_recovers_a_teacher(net):
    w = W.triatomic_liquid(16, seed=24)
    S, B, rc, L = 3, 4, 4.0, float(w.box[0])
    teacher = net.NetDraft(S, B, rc, _random_params(net, S, B, seed=6, w2=0.5))
    rng = np.random.default_rng(7)
    frames = [np.mod(w.positions + rng.normal(scale=0.05, size=w.positions.shape), L)
              for _ in range(4)]
    Ys = [teacher.forces(w.species, x, L) for x in frames]
    p = teacher.params + np.random.default_rng(8).normal(scale=0.05, size=teacher.P)
    student = net.NetDraft(S, B, rc, p)
    m, v = np.zeros_like(p), np.zeros_like(p)

    def loss_grad():
        g = np.zeros_like(p)
        sse = sum(student.sse_grad(w.species, x, L, Y, grad=g)[0] for x, Y in zip(frames, Ys))
        return sse, g

    first, _ = loss_grad()
    for t in range(1, 301):
        _, g = loss_grad()
        net.adam(p, m, v, g, 2e-3, t)
        student.params = p
    last, _ = loss_grad()
    assert last < 0.05 * first, (first, last)
