"""GPU parity of the force-matched pair draft and of its force-matching
normal equations against the FP64 oracle, on identical binary32 inputs.

Tolerances: draft forces are binary32 sums of ~60 pair terms whose radial
profile comes from a Chebyshev recurrence (16 terms); they must agree to
1e-5 of the largest force component.  The normal equations are binary64
sums of products of binary32 design entries: 1e-5 relative to the largest
entry."""
import sys

import numpy as np
import pytest

from paper_2606_02455_amd import workloads as W

pytestmark = pytest.mark.gpu
NB, RC = 16, 4.0


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


def _target():
    return dict(kind="mpnn", rc=5.0, weights=W.mpnn_weights(3, seed=17), n_model_species=3,
                scale=1.0)


def _weights(seed=6):
    rng = np.random.default_rng(seed)
    # a smooth profile per type: decaying coefficients
    return W.f32(rng.normal(size=(6, NB)) / (1.0 + np.arange(NB))[None, :])


def _midpoints(w):
    """First midpoints of the committed state: (A) in binary64, wrapped, then
    rounded to binary32 (the integrator's half step, Eq. aboba)."""
    L = float(w.box[0])
    m = w.species_mass[w.species][:, None]
    x = W.f32(w.positions) + 0.5 * w.dt / m * W.f32(w.momenta)
    x = x - L * np.floor(x / L)
    x = W.f32(x)
    x[x >= L] = 0.0
    return x


def test_pair_draft_forces_match_oracle(torch, lsd, ora):
    _say("pair draft forces")
    from oracle.pair import PairDraft
    w = W.triatomic_liquid(64, seed=12, K=2)
    wt = _weights()
    draft = dict(kind="pair", rc=RC, weights=wt, n_basis=NB, n_model_species=3)
    g = lsd.LSDSystem(w, mode="lsd", target=_target(), draft=draft)
    g.draft_steps(1)
    torch.cuda.synchronize()
    win = g.window()
    x0 = win["q_mid"][0, :, :3].double().cpu().numpy()
    fd = win["f_draft"][0].double().cpu().numpy().T
    xm = _midpoints(w)
    assert np.array_equal(x0, xm)
    ref = PairDraft(3, NB, RC, wt).forces(w.species, xm, float(w.box[0]))
    assert np.max(np.abs(fd - ref)) <= 1e-5 * np.max(np.abs(ref)), np.max(np.abs(fd - ref))
    assert g.status() == 0
    g.destroy()


def test_fit_normal_equations_match_oracle(torch, lsd, ora):
    _say("pair fit normal equations")
    from oracle.pair import PairDraft
    w = W.triatomic_liquid(64, seed=13, K=4)
    K, N, L = w.K, w.n_atoms, float(w.box[0])
    wt = _weights(7)
    ref_draft = PairDraft(3, NB, RC, wt)
    rng = np.random.default_rng(1)
    base = W.f32(np.mod(w.positions, L))
    base[base >= L] = 0.0
    frames = [base]
    for k in range(1, K):
        frames.append(W.f32(base + rng.normal(scale=0.02, size=base.shape)))
    frames = np.stack(frames)
    forces = W.f32(np.stack([ref_draft.forces(w.species, x, L) for x in frames]))
    g = lsd.LSDSystem(w, mode="lsd", target=_target(), draft=_target_free_draft(w))
    g.set_state(w.positions, np.zeros_like(w.positions))
    win = g.window()
    q4 = np.zeros((K, N, 4), np.float32)
    q4[:, :, :3] = frames
    win["q_mid"][:K].copy_(torch.tensor(q4))
    win["p_draft"][:K + 1].zero_()
    win["f_draft"][:K].copy_(torch.tensor(np.transpose(forces, (0, 2, 1)).copy()))
    torch.cuda.synchronize()
    g.mark_drafted(K)
    P = 6 * NB
    gram = torch.zeros((P + 1, P + 1), dtype=torch.float64, device="cuda")
    g.fit_pair_accumulate(NB, RC, gram)
    torch.cuda.synchronize()
    assert int(win["frame_invalid"][0, :K].sum()) == 0
    G = gram.cpu().numpy()
    Ae = np.concatenate([np.concatenate([ref_draft.design(w.species, x, L), f.reshape(-1, 1)], 1)
                         for x, f in zip(frames, forces)])
    G_ref = Ae.T @ Ae
    G_ref[P, P] = 0.0
    scale = np.max(np.abs(G_ref))
    assert np.max(np.abs(G - G_ref)) <= 1e-5 * scale, np.max(np.abs(G - G_ref)) / scale
    # the forces were made by known weights: the fitted weights reproduce
    # them (the weights themselves are ill-determined: the basis is nearly
    # collinear over the sampled distances)
    got = lsd.fit_pair_solve(G, ridge=1e-12)
    y = np.concatenate([f.ravel() for f in forces])
    A = Ae[:, :P]
    res = np.linalg.norm(A @ got - y) / np.linalg.norm(y)
    assert res < 1e-4, res
    # a second call accumulates
    g.fit_pair_accumulate(NB, RC, gram)
    torch.cuda.synchronize()
    assert np.allclose(gram.cpu().numpy(), 2 * G, rtol=0, atol=1e-12 * scale)
    # differences of consecutive frames: rows A(k+1) - A(k), forces likewise
    gd = torch.zeros((P + 1, P + 1), dtype=torch.float64, device="cuda")
    g.fit_pair_accumulate(NB, RC, gd, differences=True)
    torch.cuda.synchronize()
    Ad = [np.concatenate([ref_draft.design(w.species, frames[k + 1], L)
                          - ref_draft.design(w.species, frames[k], L),
                          (forces[k + 1].astype(np.float64) - forces[k]).reshape(-1, 1)], 1)
          for k in range(K - 1)]
    Gd_ref = sum(a.T @ a for a in Ad)
    Gd_ref[P, P] = 0.0
    Gd = gd.cpu().numpy()
    sd = np.max(np.abs(Gd_ref))
    # binary32 design rows lose digits in the difference: 1e-4 of the largest entry
    assert np.max(np.abs(Gd - Gd_ref)) <= 1e-4 * sd, np.max(np.abs(Gd - Gd_ref)) / sd
    g.destroy()


def _target_free_draft(w):
    return dict(kind="harmonic", k=0.0, anchor=w.positions)
