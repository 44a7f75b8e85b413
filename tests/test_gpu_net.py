"""GPU parity of the learned many-body draft and of its training against the
FP64 oracle, through the C ABI.

Tolerances:
  * binary32 node pass: forces are binary32 sums of ~20 pair terms whose
    coefficients come through two dense layers; 2e-5 of the largest force
    component.
  * bfloat16 node pass (matrix cores): D, h, W1 and W2 are rounded to
    bfloat16 (unit roundoff u = 2^-8) with binary32 accumulation.  Per atom,
    |dz| <= 2.01 u sum |W1||D|, |dh| <= 1.1 |dz| + 1.01 u |h| (silu' <= 1.1),
    |dv| <= sum |W2| (|dh| + 1.01 u |h|), and the force error is at most
    sum over the atom's pairs of sum_b |e_b| (|dv_i| + |dv_j|).  The test
    evaluates this bound from the oracle's intermediates and allows 1.5x it
    plus the binary32 tolerance.
  * FP8 node pass (OCP e4m3, 3 mantissa bits, u = 2^-4, one scale s per
    tensor): each quantised operand errs by at most u |x| + 2^-10 s (half
    the subnormal spacing); the same propagation through the two layers
    bounds the force error, again with 1.5x the bound plus the binary32
    tolerance.
  * training gradient: binary32 forward and backward passes reduced in
    binary64; 1e-4 of the largest gradient entry.
  * Adam: moments from identical binary64 inputs are bitwise equal; the
    binary32 parameters, rounded once per step, within half an ulp of each
    step's result summed over the steps.
"""
import sys

import numpy as np
import pytest

from paper_2606_02455_amd import workloads as W

pytestmark = pytest.mark.gpu
S_, B_, RC = 3, 8, 4.0
H = 32


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


def _params(lsd, seed, w2=0.05, c=0.3, nb=B_):
    """Random learned-draft parameters (float32) whose edge coefficients
    matter next to the pair part."""
    P = lsd.net_param_count(S_, nb)
    rng = np.random.default_rng(seed)
    p = np.zeros(P)
    o1 = H * S_ * nb
    o2 = o1 + S_ * H
    o3 = o2 + nb * H
    p[:o1] = rng.normal(scale=1.0 / np.sqrt(S_ * nb), size=o1)
    p[o1:o2] = rng.normal(scale=0.2, size=o2 - o1)
    p[o2:o3] = rng.normal(scale=w2, size=o3 - o2)
    p[o3:] = rng.normal(scale=c, size=P - o3) / (1.0 + np.arange(nb))[None, :].repeat(6, 0).ravel()
    return W.f32(p)


def _tether(w):
    return dict(kind="harmonic", k=1.0, anchor=w.positions)


def _midpoints(w):
    L = float(w.box[0])
    m = w.species_mass[w.species][:, None]
    x = W.f32(w.positions) + 0.5 * w.dt / m * W.f32(w.momenta)
    x = x - L * np.floor(x / L)
    x = W.f32(x)
    x[x >= L] = 0.0
    return x


def _bf16_bound(ora_net, species, x, L, D, z, v, rc=RC, nb=B_):
    """Force error bound of the bfloat16 node pass (module docstring)."""
    u = 2.0 ** -8
    W1, b1, W2, c = ora_net.split()
    h = z / (1.0 + np.exp(-z))
    dz = 2.01 * u * (np.abs(D) @ np.abs(W1).T)
    dh = 1.1 * dz + 1.01 * u * np.abs(h)
    dv = (dh + 1.01 * u * np.abs(h)) @ np.abs(W2).T
    return _pair_sum(x, L, species, dv, rc, nb)


def _pair_sum(x, L, species, dv, rc=RC, nb=B_):
    """Per atom, sum over its pairs of sum_b |e_b| (dv_i[b] + dv_j[b])."""
    from oracle import pairs
    rec = pairs(x, L, rc, method="cells" if np.floor(L / rc) >= 3 else "brute")
    i, j = rec[:, 0], rec[:, 1]
    d = x[j] + L * rec[:, 2:5] - x[i]
    r = np.linalg.norm(d, axis=1)
    b = np.arange(1, nb + 1)
    e = (0.5 * (np.cos(np.pi * r / rc) + 1.0))[:, None] * np.sin(np.pi * np.outer(r, b) / rc) / r[:, None]
    per = np.sum(np.abs(e) * (dv[i] + dv[j]), axis=1)
    out = np.zeros(len(x))
    np.add.at(out, i, per)
    return out[:, None]


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_net_draft_forces_match_oracle(torch, lsd, ora, precision):
    _say(f"learned draft forces ({precision})")
    from oracle.net import NetDraft
    w = W.triatomic_liquid(64, seed=31, K=2)
    L = float(w.box[0])
    p = _params(lsd, 3)
    draft = dict(kind="net", rc=RC, weights=p, n_basis=B_, n_model_species=S_,
                 precision=precision)
    g = lsd.LSDSystem(w, mode="lsd", target=_tether(w), draft=draft)
    g.draft_steps(1)
    torch.cuda.synchronize()
    win = g.window()
    x0 = win["q_mid"][0, :, :3].double().cpu().numpy()
    fd = win["f_draft"][0].double().cpu().numpy().T
    xm = _midpoints(w)
    assert np.array_equal(x0, xm)
    ref_net = NetDraft(S_, B_, RC, p.astype(np.float64))
    ref, D, z, v = ref_net.forward(w.species, xm, L, intermediates=True)
    scale = np.max(np.abs(ref))
    # the edge coefficients carry a real share of the force
    o2 = H * S_ * B_ + S_ * H
    no_w2 = p.astype(np.float64)
    no_w2[o2:o2 + B_ * H] = 0.0
    pair_only = NetDraft(S_, B_, RC, no_w2)
    assert np.max(np.abs(ref - pair_only.forces(w.species, xm, L))) > 0.2 * scale
    err = np.abs(fd - ref)
    tol32 = 2e-5 * scale
    if precision == "fp32":
        assert np.max(err) <= tol32, np.max(err) / scale
    else:
        bound = _bf16_bound(ref_net, w.species, xm, L, D, z, v)
        assert np.all(err <= 1.5 * bound + tol32), np.max(err / (1.5 * bound + tol32))
        assert np.max(err) > tol32  # the bfloat16 path really ran
    assert g.status() == 0
    g.destroy()


@pytest.mark.parametrize("rc,nb", [(6.5, 8), (4.0, 16)])
def test_net_draft_bf16_long_rows_and_full_basis(torch, lsd, ora, rc, nb):
    # the bfloat16 node pass stages each atom's list entries 64 at a time
    # with one lane per radial function: a 6.5 A cutoff gives rows of more
    # than 64 entries (several stages, the lanes past the basis idle), and
    # 16 radial functions use every lane
    _say(f"learned draft, bfloat16, rc {rc}, {nb} radial functions")
    from oracle.net import NetDraft
    w = W.triatomic_liquid(64, seed=33, K=2)
    L = float(w.box[0])
    p = _params(lsd, 5, nb=nb)
    draft = dict(kind="net", rc=rc, weights=p, n_basis=nb, n_model_species=S_, precision="bf16")
    g = lsd.LSDSystem(w, mode="lsd", target=_tether(w), draft=draft)
    g.draft_steps(1)
    torch.cuda.synchronize()
    if rc > 6.0:
        cnt = g.neighbor_lists("draft")[0]
        assert int(cnt.max()) > 64, int(cnt.max())
    win = g.window()
    fd = win["f_draft"][0].double().cpu().numpy().T
    xm = _midpoints(w)
    ref_net = NetDraft(S_, nb, rc, p.astype(np.float64))
    ref, D, z, v = ref_net.forward(w.species, xm, L, intermediates=True)
    scale = np.max(np.abs(ref))
    err = np.abs(fd - ref)
    tol32 = 2e-5 * scale
    bound = _bf16_bound(ref_net, w.species, xm, L, D, z, v, rc, nb)
    assert np.all(err <= 1.5 * bound + tol32), np.max(err / (1.5 * bound + tol32))
    assert g.status() == 0
    g.destroy()


def _fp8_bound(ora_net, species, x, L, D, z, amax):
    """Force error bound of the FP8 node pass (module docstring)."""
    u, a = 2.0 ** -4, 2.0 ** -10
    W1, b1, W2, c = ora_net.split()
    sD, sh = amax[0] / 448.0, amax[1] / 448.0
    sW1, sW2 = np.abs(W1).max() / 448.0, np.abs(W2).max() / 448.0
    eD = u * np.abs(D) + a * sD
    eW1 = u * np.abs(W1) + a * sW1
    dz = eD @ np.abs(W1).T + np.abs(D) @ eW1.T + eD @ eW1.T
    h = z / (1.0 + np.exp(-z))
    dh = 1.1 * dz
    dh = dh + u * (np.abs(h) + dh) + a * sh
    eW2 = u * np.abs(W2) + a * sW2
    dv = dh @ np.abs(W2).T + np.abs(h) @ eW2.T + dh @ eW2.T
    return _pair_sum(x, L, species, dv)


def test_net_draft_fp8_within_rounding_bound(torch, lsd, ora):
    _say("learned draft forces (fp8) and activation calibration")
    from oracle.net import NetDraft
    w = W.triatomic_liquid(64, seed=31, K=2)
    L = float(w.box[0])
    p = _params(lsd, 3)
    xm = _midpoints(w)
    ref_net = NetDraft(S_, B_, RC, p.astype(np.float64))
    ref, D, z, v = ref_net.forward(w.species, xm, L, intermediates=True)
    h = z / (1.0 + np.exp(-z))
    amax = (np.abs(D).max() * 1.0001, np.abs(h).max() * 1.0001)
    pt = torch.tensor(p, dtype=torch.float32, device="cuda")
    draft = dict(kind="net", rc=RC, weights=pt, n_basis=B_, n_model_species=S_,
                 precision="fp8", act_amax=amax)
    target = dict(kind="mpnn", rc=5.0, weights=W.mpnn_weights(3, seed=17), n_model_species=3,
                  scale=1.0)
    g = lsd.LSDSystem(w, mode="lsd", target=target, draft=draft)
    g.draft_steps(1)
    torch.cuda.synchronize()
    win = g.window()
    assert np.array_equal(win["q_mid"][0, :, :3].double().cpu().numpy(), xm)
    fd = win["f_draft"][0].double().cpu().numpy().T
    scale = np.max(np.abs(ref))
    err = np.abs(fd - ref)
    bound = 1.5 * _fp8_bound(ref_net, w.species, xm, L, D, z, amax) + 2e-5 * scale
    assert np.all(err <= bound), np.max(err / bound)
    # FP8 rounds far more than bfloat16: the error is visible but bounded
    assert np.max(err) > 1e-3 * scale
    # the calibration pass returns the maxima of the valid frame exactly up
    # to binary32 evaluation
    got = g.net_activation_amax(dict(draft, weights=pt))
    assert got[0] == pytest.approx(amax[0] / 1.0001, rel=1e-5)
    assert got[1] == pytest.approx(amax[1] / 1.0001, rel=1e-5)
    assert g.status() == 0
    g.destroy()


def test_net_draft_graph_replays_equal_eager(torch, lsd):
    _say("learned draft: graph vs eager")
    w = W.triatomic_liquid(64, seed=32, K=4)
    p = torch.tensor(_params(lsd, 4, w2=0.01, c=0.05), dtype=torch.float32, device="cuda")
    draft = dict(kind="net", rc=RC, weights=p, n_basis=B_, n_model_species=S_)
    a = lsd.LSDSystem(w, mode="lsd", target=_tether(w), draft=draft)
    b = lsd.LSDSystem(w, mode="lsd", target=_tether(w), draft=draft)
    b.set_graphs(False)
    for rep in range(4):
        a.run_windows(3, 4)
        b.run_windows(3, 4)
        sa, sb = a.state(), b.state()
        for k in ("q", "p", "img", "step"):
            assert np.array_equal(sa[k], sb[k]), (rep, k)
    cn = a.counters()
    assert cn[0, 1] > 0
    assert a.status() == 0
    a.destroy()
    b.destroy()


@pytest.mark.parametrize("skin", [1.0, 0.05])
def test_net_draft_tail_equals_per_step_launches(torch, lsd, skin):
    """Draft steps from first_step on in one launch (node and force passes
    block by block with grid barriers) give the trajectory and counters of
    one launch per step: graph and eager windows, three first steps, a skin
    long enough for whole windows and one that ends windows inside the
    chain."""
    _say(f"learned draft: one-launch chain vs per-step launches, skin {skin}")
    w = W.triatomic_liquid(64, seed=33, K=8)
    p = torch.tensor(_params(lsd, 4, w2=0.01, c=0.05), dtype=torch.float32, device="cuda")
    draft = dict(kind="net", rc=RC, weights=p, n_basis=B_, n_model_species=S_, precision="bf16")
    ref = lsd.LSDSystem(w, mode="lsd", target=_tether(w), draft=draft, skin=skin)
    ref.set_draft_tail(0)
    systems = []
    for first, graphs in ((1, True), (3, True), (5, True), (3, False)):
        g = lsd.LSDSystem(w, mode="lsd", target=_tether(w), draft=draft, skin=skin)
        g.set_draft_tail(first)
        g.set_graphs(graphs)
        systems.append(g)
    for rep in range(3):
        ref.run_windows(4, 8)
        sr = ref.state()
        for g in systems:
            g.run_windows(4, 8)
            sg = g.state()
            for k in ("q", "p", "img", "step"):
                assert np.array_equal(sr[k], sg[k]), (rep, k)
            assert np.array_equal(ref.counters(), g.counters()), rep
            assert g.status() == 0
    cn = ref.counters()[0]
    frames_per_window = cn[3] / cn[0]
    if skin == 1.0:
        assert frames_per_window > 5, frames_per_window  # the chain runs valid steps
    else:
        assert frames_per_window < 8, frames_per_window  # windows end inside the chain
    for g in [ref] + systems:
        g.destroy()


def _training_window(torch, lsd, w, K, net_p):
    """A system whose window holds K caller frames (small perturbations of
    the wrapped start) with forces y of a teacher net, written as the
    stepping forces."""
    from oracle.net import NetDraft
    L = float(w.box[0])
    rng = np.random.default_rng(11)
    base = W.f32(np.mod(w.positions, L))
    base[base >= L] = 0.0
    frames = [base] + [W.f32(np.clip(base + rng.normal(scale=0.02, size=base.shape), 0, L * (1 - 1e-6)))
                       for _ in range(K - 1)]
    frames = np.stack(frames)
    teacher = NetDraft(S_, B_, RC, net_p.astype(np.float64))
    ys = W.f32(np.stack([teacher.forces(w.species, x, L) for x in frames]))
    target = dict(kind="mpnn", rc=5.0, weights=W.mpnn_weights(3, seed=17), n_model_species=3,
                  scale=1.0)
    g = lsd.LSDSystem(w, mode="lsd", target=target,
                      draft=dict(kind="harmonic", k=0.0, anchor=w.positions))
    g.set_state(w.positions, np.zeros_like(w.positions))
    win = g.window()
    N = w.n_atoms
    q4 = np.zeros((K, N, 4), np.float32)
    q4[:, :, :3] = frames
    win["q_mid"][:K].copy_(torch.tensor(q4))
    win["p_draft"][:K + 1].zero_()
    win["f_draft"][:K].copy_(torch.tensor(np.transpose(ys, (0, 2, 1)).copy(), dtype=torch.float32))
    torch.cuda.synchronize()
    g.mark_drafted(K)
    return g, frames, ys


def test_net_training_gradient_matches_oracle(torch, lsd, ora):
    _say("learned draft training gradient")
    from oracle.net import NetDraft
    w = W.triatomic_liquid(64, seed=33, K=4)
    K, L = w.K, float(w.box[0])
    g, frames, ys = _training_window(torch, lsd, w, K, _params(lsd, 5))
    student = _params(lsd, 6)
    P = student.size
    pt = torch.tensor(student, dtype=torch.float32, device="cuda")
    grad = torch.zeros(P + 2, dtype=torch.float64, device="cuda")
    net = dict(kind="net", rc=RC, weights=pt, n_basis=B_, n_model_species=S_)
    scratch = g.net_train_accumulate(net, grad)
    torch.cuda.synchronize()
    assert int(g.window()["frame_invalid"][0, :K].sum()) == 0
    gg = grad.cpu().numpy()
    ref = NetDraft(S_, B_, RC, student.astype(np.float64))
    gr = np.zeros(P)
    sse = sum(ref.sse_grad(w.species, x, L, y, grad=gr)[0] for x, y in zip(frames, ys))
    assert gg[P + 1] == K * w.n_atoms
    assert gg[P] == pytest.approx(sse, rel=1e-4)
    assert np.max(np.abs(gg[:P] - gr)) <= 1e-4 * np.max(np.abs(gr)), \
        np.max(np.abs(gg[:P] - gr)) / np.max(np.abs(gr))
    # the loss of force changes between consecutive frames
    gd = torch.zeros(P + 2, dtype=torch.float64, device="cuda")
    g.net_train_accumulate(net, gd, scratch=scratch, differences=True)
    torch.cuda.synchronize()
    gdd = gd.cpu().numpy()
    sd, grd = ref.diff_sse_grad(w.species, frames, L, ys)
    assert gdd[P + 1] == (K - 1) * w.n_atoms
    assert gdd[P] == pytest.approx(sd, rel=1e-4)
    # differences of binary32 forces lose digits: 1e-3 of the largest entry
    assert np.max(np.abs(gdd[:P] - grd)) <= 1e-3 * np.max(np.abs(grd)), \
        np.max(np.abs(gdd[:P] - grd)) / np.max(np.abs(grd))
    # a second call accumulates; an Adam step consumes and clears the buffer
    g.net_train_accumulate(net, grad, scratch=scratch)
    torch.cuda.synchronize()
    assert np.allclose(grad.cpu().numpy(), 2 * gg, rtol=1e-12, atol=1e-12 * np.max(np.abs(gg)))
    m = torch.zeros(P, dtype=torch.float64, device="cuda")
    v = torch.zeros(P, dtype=torch.float64, device="cuda")
    lsd.net_adam_step(torch, pt, m, v, grad, 1e-3, 1)
    torch.cuda.synchronize()
    assert not grad.any().item()
    g.destroy()


def test_net_adam_matches_oracle(torch, lsd, ora):
    _say("learned draft Adam step")
    from oracle.net import adam
    rng = np.random.default_rng(12)
    P = lsd.net_param_count(S_, B_)
    p0 = W.f32(rng.normal(size=P))
    rows = 321.0
    grads = [rng.normal(size=P) * 10.0 ** rng.uniform(-3, 2, size=P) for _ in range(2)]
    pt = torch.tensor(p0, dtype=torch.float32, device="cuda")
    m = torch.zeros(P, dtype=torch.float64, device="cuda")
    v = torch.zeros(P, dtype=torch.float64, device="cuda")
    po, mo, vo = p0.astype(np.float64), np.zeros(P), np.zeros(P)
    # each step rounds the parameters to binary32 once: after two steps the
    # GPU is within half an ulp of the first result plus half an ulp of the
    # second (of the oracle's binary64 values) of the oracle
    tol = np.zeros(P)
    for t, gsum in enumerate(grads, start=1):
        buf = torch.tensor(np.concatenate([gsum, [1.0, rows]]), dtype=torch.float64, device="cuda")
        lsd.net_adam_step(torch, pt, m, v, buf, 1e-2, t, beta1=0.9, beta2=0.99, eps=1e-8)
        adam(po, mo, vo, gsum * (1.0 / (3.0 * rows)), 1e-2, t, beta1=0.9, beta2=0.99, eps=1e-8)
        tol += 0.5 * np.spacing(np.abs(po).astype(np.float32)).astype(np.float64)
        torch.cuda.synchronize()
        assert not buf.any().item()
        assert np.array_equal(m.cpu().numpy(), mo) and np.array_equal(v.cpu().numpy(), vo)
    got = pt.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - po) <= 1.01 * tol), np.max(np.abs(got - po) / tol)
    # an empty buffer (no atom frames) changes nothing
    before = pt.clone()
    lsd.net_adam_step(torch, pt, m, v, torch.zeros(P + 2, dtype=torch.float64, device="cuda"),
                      1e-2, 3)
    torch.cuda.synchronize()
    assert torch.equal(before, pt)


def test_net_training_reduces_the_force_error(torch, lsd):
    _say("learned draft training loop")
    w = W.triatomic_liquid(64, seed=34, K=4)
    g, frames, ys = _training_window(torch, lsd, w, w.K, _params(lsd, 7))
    P = lsd.net_param_count(S_, B_)
    pt = torch.tensor(lsd.net_init_params(S_, B_, seed=1), device="cuda")
    net = dict(kind="net", rc=RC, weights=pt, n_basis=B_, n_model_species=S_)
    grad = torch.zeros(P + 2, dtype=torch.float64, device="cuda")
    m = torch.zeros(P, dtype=torch.float64, device="cuda")
    v = torch.zeros(P, dtype=torch.float64, device="cuda")
    scratch = None
    losses = []
    for t in range(1, 201):
        scratch = g.net_train_accumulate(net, grad, scratch=scratch)
        if t in (1, 200):
            torch.cuda.synchronize()
            losses.append(grad[P].item() / grad[P + 1].item())
        lsd.net_adam_step(torch, pt, m, v, grad, 1e-2, t)
    assert losses[1] < 0.2 * losses[0], losses
    g.destroy()


def _replica_frames(w, K, seed):
    """K frames per replica: the wrapped start and small perturbations of it,
    each replica in its own box."""
    rng = np.random.default_rng(seed)
    frames = np.zeros((K, w.n_atoms, 3))
    for r in range(w.n_replicas):
        sl = w.replica_slice(r)
        L = float(w.box[r])
        base = W.f32(np.mod(w.positions[sl], L))
        base[base >= L] = 0.0
        frames[0, sl] = base
        for k in range(1, K):
            frames[k, sl] = W.f32(np.clip(base + rng.normal(scale=0.02, size=base.shape), 0,
                                          L * (1 - 1e-6)))
    return frames


def test_net_on_ragged_replicas(torch, lsd, ora):
    # replicas of 21..39 atoms: the 16-atom node blocks and 64-atom training
    # blocks straddle replicas, each box is small enough for 27 images
    _say("learned draft on ragged replicas")
    from oracle.net import NetDraft
    w = W.triatomic_replicas(3, n_mol_lo=7, n_mol_hi=13, seed=35, K=3)
    assert w.n_atoms % 16 != 0
    p = _params(lsd, 8)
    ref_net = NetDraft(S_, B_, RC, p.astype(np.float64))
    # drafting forces at the first midpoints, replica by replica
    g = lsd.LSDSystem(w, mode="lsd", target=dict(kind="harmonic", k=1.0, anchor=w.positions),
                      draft=dict(kind="net", rc=RC, weights=p, n_basis=B_, n_model_species=S_,
                                 precision="fp32"))
    g.draft_steps(1)
    torch.cuda.synchronize()
    x0 = g.window()["q_mid"][0, :, :3].double().cpu().numpy()
    fd = g.window()["f_draft"][0].double().cpu().numpy().T
    for r in range(w.n_replicas):
        sl = w.replica_slice(r)
        L = float(w.box[r])
        ref = ref_net.forces(w.species[sl], np.mod(x0[sl], L), L)
        assert np.max(np.abs(fd[sl] - ref)) <= 2e-5 * np.max(np.abs(ref)), r
    g.destroy()
    # training gradient over caller frames of every replica
    K = w.K
    frames = _replica_frames(w, K, seed=36)
    teacher = NetDraft(S_, B_, RC, _params(lsd, 9).astype(np.float64))
    ys = np.zeros_like(frames)
    for r in range(w.n_replicas):
        sl = w.replica_slice(r)
        for k in range(K):
            ys[k, sl] = teacher.forces(w.species[sl], frames[k, sl], float(w.box[r]))
    ys = W.f32(ys)
    target = dict(kind="mpnn", rc=5.0, weights=W.mpnn_weights(3, seed=17), n_model_species=3,
                  scale=1.0)
    g = lsd.LSDSystem(w, mode="lsd", target=target,
                      draft=dict(kind="harmonic", k=0.0, anchor=w.positions))
    g.set_state(w.positions, np.zeros_like(w.positions))
    win = g.window()
    q4 = np.zeros((K, w.n_atoms, 4), np.float32)
    q4[:, :, :3] = frames
    win["q_mid"][:K].copy_(torch.tensor(q4))
    win["p_draft"][:K + 1].zero_()
    win["f_draft"][:K].copy_(torch.tensor(np.transpose(ys, (0, 2, 1)).copy(), dtype=torch.float32))
    torch.cuda.synchronize()
    g.mark_drafted(K)
    pt = torch.tensor(p, dtype=torch.float32, device="cuda")
    net = dict(kind="net", rc=RC, weights=pt, n_basis=B_, n_model_species=S_)
    P = p.size
    for diff in (False, True):
        grad = torch.zeros(P + 2, dtype=torch.float64, device="cuda")
        g.net_train_accumulate(net, grad, differences=diff)
        torch.cuda.synchronize()
        assert int(win["frame_invalid"][:, :K].sum()) == 0
        gg = grad.cpu().numpy()
        gr, sse = np.zeros(P), 0.0
        for r in range(w.n_replicas):
            sl = w.replica_slice(r)
            L = float(w.box[r])
            if diff:
                sse += ref_net.diff_sse_grad(w.species[sl], frames[:, sl], L, ys[:, sl], grad=gr)[0]
            else:
                for k in range(K):
                    sse += ref_net.sse_grad(w.species[sl], frames[k, sl], L, ys[k, sl], grad=gr)[0]
        assert gg[P + 1] == (K - 1 if diff else K) * w.n_atoms
        assert gg[P] == pytest.approx(sse, rel=1e-4)
        tol = (1e-3 if diff else 1e-4) * np.max(np.abs(gr))
        assert np.max(np.abs(gg[:P] - gr)) <= tol, (diff, np.max(np.abs(gg[:P] - gr)) / tol)
    g.destroy()
