"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Bars:
  * random stream: Philox words bit-exact, uniforms bit-exact, normals 1e-13;
  * neighbour lists: exact set equality with the oracle's enumeration;
  * forces: max |F_gpu - F_oracle| <= 1e-5 max |F_oracle| per frame (binary32
    pair forces against binary64), energies 1e-5 relative;
  * log ratios: within a first-order bound propagated from the measured force
    error; decisions equal except inside the band
    |log r_oracle - log u| <= max(1e-6 max(|log u|, 1), |log r_gpu - log r_oracle|);
  * committed momenta / positions: 1e-5 relative (binary32 storage).
All inputs are seeded and binary32-representable so both sides start from the
same numbers.
"""
import sys

import numpy as np
import pytest

from paper_2606_02455_amd import workloads as W

pytestmark = pytest.mark.gpu


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


def _ora_system(ora, w, r=0):
    sl = w.replica_slice(r)
    return ora.System(sl.stop - sl.start, float(w.box[r]), w.masses()[sl], w.dt, w.gamma, w.kT,
                      w.force_unit)


def _ora_pot(ora, d):
    if d["kind"] == "lj":
        return ora.Potential.lj(d["rc"], d.get("eps", 1.0), d.get("sig", 1.0), offset=d.get("offset"))
    return ora.Potential.harmonic(d["k"], d["anchor"], offset=d.get("offset"))


def _continuous(qm, L):
    """Frames continuous with frame 0 (the window convention): undo wraps."""
    out = qm.copy()
    out[1:] -= L * np.round((out[1:] - out[0][None]) / L)
    return out


def _inject(sysg, torch, qmid, p_draft, f_draft):
    """Write caller frames (numpy [K,N,3], [K+1,N,3], [K,N,3]) into the window;
    positions are made continuous with frame 0."""
    win = sysg.window()
    K = qmid.shape[0]
    L = np.repeat(sysg.w.box, np.diff(sysg.w.atom_offsets))[None, :, None]
    qmid = _continuous(qmid, L)
    q4 = np.zeros((K, qmid.shape[1], 4), np.float32)
    q4[:, :, :3] = qmid
    win["q_mid"][:K].copy_(torch.tensor(q4))
    win["p_draft"][:K + 1].copy_(torch.tensor(np.transpose(p_draft, (0, 2, 1)).astype(np.float32)))
    win["f_draft"][:K].copy_(torch.tensor(np.transpose(f_draft, (0, 2, 1)).astype(np.float32)))
    torch.cuda.synchronize()


# ---------------------------------------------------------------------------
def test_rng_matches_oracle(torch, lsd, ora):
    _say("rng parity")
    for (seed, rep, step, n) in [(1, 0, 1, 64), (2 ** 40 + 7, 5, 2 ** 33 + 11, 1000)]:
        g = lsd.rng_normals(seed, rep, step, n).cpu().numpy()
        o = ora.normals(seed, rep, step, n)
        assert np.allclose(g, o, rtol=1e-13, atol=1e-13)
    g = lsd.rng_uniforms(9, 3, 100, 500).cpu().numpy()
    o = np.array([ora.uniform(9, 3, 100 + k + 1) for k in range(500)])
    assert np.array_equal(g, o)


def _gpu_pairs(sysg, which="target"):
    cnt, ent = sysg.neighbor_lists(which)
    cnt, ent = cnt.cpu().numpy(), ent.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    i_idx = np.concatenate([np.full(c, i) for i, c in enumerate(cnt)])
    e = np.concatenate([ent[i, :c] for i, c in enumerate(cnt)])
    j = e >> 5
    code = e & 31
    nx, ny, nz = code % 3 - 1, (code // 3) % 3 - 1, code // 9 - 1
    out = np.stack([i_idx, j, nx, ny, nz], axis=1)
    return out[np.lexsort((out[:, 4], out[:, 3], out[:, 2], out[:, 1], out[:, 0]))]


def _config(case):
    """A configuration; "<name>_bench" with the list skin of the benchmark's
    LSD run."""
    if case.endswith("_bench"):
        name = case[:-len("_bench")]
        w = W.config(name)
        w.skin = W.BENCH_SKINS[name][0]
        return w
    return W.config(case)


@pytest.mark.parametrize("case", ["c1", "box2000", "box_2rl_above", "box_2rl_below", "c2",
                                  "c2_bench", "c2_skin05", "c2_skin1"])
def test_neighbor_lists_exact(torch, lsd, ora, case):
    """Lists equal the oracle's pair sets.  A single small system takes the
    one-launch builder: nearest images when L > 2 r_list (box2000 and a box
    0.4% above 2 r_list), all 27 images otherwise (c1 and a box 0.4% below
    2 r_list, where an atom can meet two images of another); c2 takes the
    cells (c2 at its own skin and at 0.125, 0.5 and 1.0; at 1.0, about 45
    atoms per cell, a cell's 27 neighbour cells hold more candidates than
    one staging pass takes and its atoms span more than one block)."""
    _say(f"neighbour lists {case}")
    if case == "box2000":
        w = W.lj_fluid(10, rho=0.8, seed=11, K=4)
        w.positions = W.random_box_positions(w.n_atoms, float(w.box[0]), seed=12)
    elif case.startswith("box_2rl"):
        w = W.lj_fluid(6, rho=0.8, seed=13, K=4)
        L = 2.0 * (w.target["rc"] + w.skin) * (1.004 if case.endswith("above") else 0.996)
        w.box = np.array([float(W.f32(L))])
        w.positions = W.random_box_positions(w.n_atoms, float(w.box[0]), seed=14)
    elif case in ("c2_skin05", "c2_skin1"):
        w = W.config("c2")
        w.skin = 0.5 if case == "c2_skin05" else 1.0
    else:
        w = _config(case)
    sysg = lsd.LSDSystem(w, mode="lsd", k_max=1)
    K = 1
    q = w.positions[None]
    _inject(sysg, torch, q, np.zeros((2, w.n_atoms, 3)), np.zeros((1, w.n_atoms, 3)))
    sysg.mark_drafted(K)
    assert sysg.status() == 0
    L = float(w.box[0])
    skin = w.skin
    for which, rc in (("target", w.target["rc"]), ("draft", w.draft["rc"])):
        got = _gpu_pairs(sysg, which)
        method = "cells" if np.floor(L / (rc + skin)) >= 3 else "brute"
        ref = ora.pairs(w.positions, L, rc + skin, method)
        assert got.shape == ref.shape and np.array_equal(got, ref), which
    sysg.destroy()


@pytest.mark.parametrize("case,mode", [("c1", "lsd"), ("c1", "plain"), ("lj4096", "lsd"),
                                       ("c2_bench", "lsd")])
def test_pair_draft_tail_equals_per_step_launches(torch, lsd, case, mode):
    """Draft steps from first_step on in one launch (the per-step kernel's
    blocks in turn, one bounded grid barrier per step) give the trajectory
    and counters of one launch per step: one tile (c1, LSD and plain
    stepping), 64 tiles, 512 tiles over 128 blocks (c2 at the benchmark's
    skin); graph and eager windows."""
    _say(f"pair draft: one-launch chain vs per-step launches, {case} {mode}")
    w = W.lj_fluid(16, rho=0.8, seed=21, K=16) if case == "lj4096" else _config(case)
    K = w.K
    kw = dict(error_correction=2) if mode == "lsd" else {}
    ref = lsd.LSDSystem(w, mode=mode, **kw)
    ref.set_draft_tail(0)
    systems = []
    for first, graphs in ((1, True), (3, True), (3, False)):
        g = lsd.LSDSystem(w, mode=mode, **kw)
        g.set_draft_tail(first)
        g.set_graphs(graphs)
        systems.append(g)
    n = 2 if case == "c2_bench" else 4
    for rep in range(3):
        ref.run_windows(n, K)
        sr = ref.state()
        for g in systems:
            g.run_windows(n, K)
            sg = g.state()
            for k in ("q", "p", "img", "step"):
                assert np.array_equal(sr[k], sg[k]), (rep, k)
            assert np.array_equal(ref.counters(), g.counters()), rep
            assert g.status() == 0
    cn = ref.counters()[0]
    # more frames verified (LSD) or steps committed (plain) than windows: the
    # chain runs drafted steps
    assert (cn[3] if mode == "lsd" else cn[1]) > cn[0], cn
    for g in [ref] + systems:
        g.destroy()


def _perturbed_frames(w, K, seed, amp=0.02):
    rng = np.random.default_rng(seed)
    L = float(w.box[0])
    fr = []
    for k in range(K):
        x = w.positions + rng.uniform(-amp, amp, w.positions.shape)
        fr.append(W.f32(np.mod(x, L)))
    fr = np.stack(fr)
    fr[fr >= L] = 0.0
    return fr


@pytest.mark.parametrize("case", ["c1", "c2", "c2_bench"])
def test_target_forces_and_energies(torch, lsd, ora, case):
    _say(f"target forces {case}")
    w = _config(case)
    K = w.K
    sysg = lsd.LSDSystem(w, mode="lsd")
    # frames differ pairwise by at most 2 sqrt(3) amp, inside half the skin
    qm = _perturbed_frames(w, K, seed=3, amp=min(0.02, 0.1 * w.skin))
    so = _ora_system(ora, w)
    T = _ora_pot(ora, w.target)
    D = _ora_pot(ora, w.draft)
    fd = np.stack([W.f32(ora.energy_forces(D, qm[k], so.L)[1]) for k in range(K)])
    rng = np.random.default_rng(4)
    pd = W.f32(rng.normal(0, 1, (K + 1, w.n_atoms, 3)))
    _inject(sysg, torch, qm, pd, fd)
    sysg.mark_drafted(K)
    sysg.verify_window()
    sysg.accept_rollback(sync=True)
    assert sysg.status() == 0
    ft = sysg.window()["f_target"][:K].cpu().numpy().transpose(0, 2, 1)
    en = sysg.energy.cpu().numpy()[0]
    inv = sysg.window()["frame_invalid"].cpu().numpy()[0]
    assert not inv[:K].any()
    for k in range(K):
        E, F = ora.energy_forces(T, qm[k], so.L)
        err = np.max(np.abs(ft[k] - F))
        assert err <= 1e-5 * np.max(np.abs(F)), (k, err, np.max(np.abs(F)))
        assert abs(en[k] - E) <= 1e-5 * abs(E), (k, en[k], E)
    sysg.destroy()


def _oracle_window_rounded(ora, w, xi, u, q0, p0):
    """Oracle window from (q0, p0), with every stored draft array rounded to
    binary32 so that both sides can be fed the identical frames."""
    so = _ora_system(ora, w)
    T, D = _ora_pot(ora, w.target), _ora_pot(ora, w.draft)
    q, p = q0.copy(), p0.copy()
    img = np.zeros(q.shape, np.int32)
    r = ora.lsd_window(so, T, D, q, p, img, xi, u)
    r["img"] = img
    return so, T, r


def _first_midpoint_wraps(so, q0, p0):
    """Image shifts of the oracle's first half step (A of Eq. aboba) from
    (q0, p0): the wrap of q0 + dt/2 p0 / m into [0, L), as the oracle applies
    it."""
    x = q0 + (0.5 * so.dt) * p0 / so.masses[:, None]
    s = np.floor(x / so.L)
    x = x - s * so.L
    s = s + (x >= so.L) - (x < 0.0)
    return s.astype(np.int32)


@pytest.mark.parametrize("case", ["c1", "lj512", "c1_faces"])
def test_verify_and_commit_on_identical_frames(torch, lsd, ora, case):
    _say(f"verify parity {case}")
    w = W.lj_fluid(8, seed=21, K=8) if case == "lj512" else W.config("c1")
    if case == "c1_faces":
        # a layer of atoms within the jitter of every face: image counters
        # change inside the window and in the committed (reflected) step
        w.positions = _near_faces(w)
    K, N = w.K, w.n_atoms
    checked_reject = 0
    img_moves = 0
    for trial in range(6):
        xi = np.stack([ora.normals(w.seed + trial, 0, s, N) for s in range(1, K + 1)])
        u = np.array([ora.uniform(w.seed + trial, 0, s) for s in range(1, K + 1)])
        so, T, r = _oracle_window_rounded(ora, w, xi, u, w.positions, w.momenta)
        qm, pd, fd = W.f32(r["q_mid"]), W.f32(r["p_draft"]), W.f32(r["F_draft"])
        if np.any(qm >= so.L):
            qm[qm >= so.L] = 0.0
        sysg = lsd.LSDSystem(w, mode="lsd", replay=True)
        sysg.replay_u.copy_(torch.tensor(u[None, :]))
        # committed state = frame-0 momenta; positions are not read by verify
        sysg.set_state(w.positions, pd[0])
        _inject(sysg, torch, qm, pd, fd)
        sysg.mark_drafted(K)
        sysg.verify_window()
        n = int(sysg.accept_rollback(sync=True)[0])
        lr = sysg.log_ratio.cpu().numpy()[0]
        acc = sysg.accepted.cpu().numpy()[0]
        win = sysg.window()
        ft = win["f_target"][:K].cpu().numpy().transpose(0, 2, 1)
        inv = win["frame_invalid"].cpu().numpy()[0][:K]
        # frames whose atoms moved more than skin/2 from the frame-0 list
        # positions are not verified (the window ends at K_eff)
        disp = qm - qm[0][None]
        disp -= so.L * np.round(disp / so.L)
        far = np.sqrt((disp ** 2).sum(-1)).max(-1) > 0.5 * w.skin * (1 - 1e-4)
        keff = int(np.argmax(far)) if far.any() else K
        assert keff >= 1 and inv[keff:].all() and not inv[:keff].any(), (keff, inv)
        sig = so.sigma()[:, None]
        c1 = (1 + so.a) * so.dt / 2
        j_ref, ambiguous, v_ref = keff, False, None
        for k in range(keff):
            v = ora.verify_frame(so, T, qm[k], pd[k], pd[k + 1], fd[k], u[k])
            dF = np.abs(ft[k] - v["F_target"])
            assert np.max(dF) <= 1e-5 * np.max(np.abs(v["F_target"])), (trial, k)
            # first-order bound of |d log r| from the force error
            mu_t = so.a * pd[k] + c1 * v["F_target"]
            wt = (pd[k + 1] - mu_t) / sig
            bound = 2.0 * np.sum(np.abs(wt) * (c1 / sig) * dF) + 1e-9 * max(1.0, abs(v["logr"]))
            assert abs(lr[k] - v["logr"]) <= bound, (trial, k, lr[k], v["logr"], bound)
            lu = np.log(u[k])
            band = abs(v["logr"] - lu) <= max(1e-6 * max(abs(lu), 1.0), abs(lr[k] - v["logr"]))
            if band:
                if v_ref is None:
                    ambiguous = True
                continue
            assert bool(acc[k]) == v["accept"], (trial, k, acc[k], v["accept"])
            if not v["accept"] and v_ref is None and not ambiguous:
                j_ref, v_ref, dF_ref = k + 1, v, dF
        assert (acc[keff:K] == 2).all()
        if ambiguous:
            continue
        assert n == j_ref, (trial, n, j_ref)
        st = sysg.state()
        if r["n_committed"] == n:
            # image counters: the GPU counts from the wrapped first midpoint
            # (its committed counters were 0 and the injected frame-0 deltas
            # are 0), the oracle from q0 through that midpoint
            img_ref = r["img"] - _first_midpoint_wraps(so, w.positions, w.momenta)
            assert np.array_equal(st["img"], img_ref), (trial, np.argwhere(st["img"] != img_ref))
            img_moves += int(np.count_nonzero(img_ref))
        if v_ref is not None:
            checked_reject += 1
            # reflected momentum: binary32 rounding plus the first-order effect
            # of the force error on <p> and on the reflection direction delta
            k = j_ref - 1
            delta_o = c1 * (fd[k] - v_ref["F_target"]) / sig
            delta_g = c1 * (fd[k] - ft[k]) / sig
            z = (pd[k + 1] - (so.a * pd[k] + c1 * fd[k])) / sig
            coef = 2 * np.sum(delta_o * z) / np.sum(delta_o ** 2)
            dd = np.linalg.norm(delta_g - delta_o) / np.linalg.norm(delta_o)
            tol_p = (1e-5 * np.max(np.abs(v_ref["p"])) + c1 * np.max(dF_ref)
                     + 4 * sig.max() * (abs(coef) + np.linalg.norm(z)) * dd * np.abs(delta_o).max())
            assert np.max(np.abs(st["p"] - v_ref["p"])) <= tol_p, (trial, tol_p)
            dq = st["q"] - v_ref["q"]
            dq -= so.L * np.round(dq / so.L)
            assert np.max(np.abs(dq)) <= 1e-5 * so.L + so.dt * tol_p
        else:
            assert np.array_equal(st["p"], pd[j_ref])
        sysg.destroy()
    assert checked_reject >= 1
    if case == "c1_faces":
        assert img_moves >= 3, img_moves


def test_draft_steps_match_oracle(torch, lsd, ora):
    _say("draft parity c1")
    w = W.config("c1")
    K, N = w.K, w.n_atoms
    xi = np.stack([ora.normals(w.seed, 0, s, N) for s in range(1, K + 1)])
    u = np.ones(K)
    sysg = lsd.LSDSystem(w, mode="lsd", replay=True)
    sysg.replay_xi.copy_(torch.tensor(xi))
    sysg.replay_u.copy_(torch.tensor(u[None, :]))
    sysg.draft_steps(K)
    torch.cuda.synchronize()
    win = sysg.window()
    qm = win["q_mid"][:K, :, :3].cpu().numpy().astype(np.float64)
    pd = win["p_draft"][:K + 1].cpu().numpy().transpose(0, 2, 1).astype(np.float64)
    fd = win["f_draft"][:K].cpu().numpy().transpose(0, 2, 1).astype(np.float64)
    so, T, r = _oracle_window_rounded(ora, w, xi, u, w.positions, w.momenta)
    # the first midpoint is the same binary64 expression rounded to binary32
    assert np.array_equal(qm[0], W.f32(r["q_mid"][0]))
    for k in range(K):
        d = qm[k] - r["q_mid"][k]
        d -= so.L * np.round(d / so.L)
        assert np.max(np.abs(d)) < 2e-5, k
        assert np.max(np.abs(fd[k] - r["F_draft"][k])) <= 1e-4 * np.max(np.abs(r["F_draft"][k]))
        assert np.max(np.abs(pd[k + 1] - r["p_draft"][k + 1])) <= 1e-5 * np.max(np.abs(r["p_draft"][k + 1]))
    sysg.verify_window()
    sysg.accept_rollback(sync=True)
    sysg.destroy()


def test_full_size_draft_first_frame(torch, lsd, ora):
    _say("draft first frame c2")
    w = W.config("c2")
    N = w.n_atoms
    xi = ora.normals(w.seed, 0, 1, N)[None]
    sysg = lsd.LSDSystem(w, mode="lsd", replay=True, k_max=1)
    sysg.replay_xi.copy_(torch.tensor(xi))
    sysg.replay_u.fill_(1.0)
    sysg.draft_steps(1)
    torch.cuda.synchronize()
    win = sysg.window()
    qm0 = win["q_mid"][0, :, :3].cpu().numpy().astype(np.float64)
    fd0 = win["f_draft"][0].cpu().numpy().T.astype(np.float64)
    p1 = win["p_draft"][1].cpu().numpy().T.astype(np.float64)
    so = _ora_system(ora, w)
    D = _ora_pot(ora, w.draft)
    q, p = w.positions.copy(), w.momenta.copy()
    img = np.zeros((N, 3), np.int32)
    r = ora.lsd_window(so, _ora_pot(ora, w.target), D, q, p, img, xi, np.ones(1))
    assert np.array_equal(qm0, W.f32(r["q_mid"][0]))
    E, F = ora.energy_forces(D, qm0, so.L)
    assert np.max(np.abs(fd0 - F)) <= 1e-5 * np.max(np.abs(F))
    assert np.max(np.abs(p1 - r["p_draft"][1])) <= 1e-5 * np.max(np.abs(r["p_draft"][1]))
    assert sysg.status() == 0
    sysg.verify_window()
    sysg.accept_rollback(sync=True)
    sysg.destroy()


def test_draft_equals_target_is_plain_bitwise(torch, lsd):
    _say("draft == target vs plain")
    w = W.config("c1")
    same = dict(w.target)
    a = lsd.LSDSystem(w, mode="lsd", draft=same)
    b = lsd.LSDSystem(w, mode="plain")
    for win in range(25):
        a.draft_steps(8)
        a.verify_window()
        na = a.accept_rollback(sync=True)
        b.draft_steps(8)
        nb = b.accept_rollback(sync=True)
        assert na[0] == nb[0]
        assert np.all(a.accepted.cpu().numpy()[0][:na[0]] == 1)
        sa, sb = a.state(), b.state()
        assert np.array_equal(sa["q"], sb["q"]) and np.array_equal(sa["p"], sb["p"])
        assert np.array_equal(sa["img"], sb["img"]) and np.array_equal(sa["step"], sb["step"])
    assert a.state()["step"][0] >= 150
    a.destroy()
    b.destroy()


def test_run_is_deterministic(torch, lsd):
    _say("determinism")
    w = W.config("c1")
    out = []
    for rep in range(2):
        s = lsd.LSDSystem(w, mode="lsd")
        s.run_windows(40, 8)
        out.append(s.state())
        s.destroy()
    for k in ("q", "p", "img", "step"):
        assert np.array_equal(out[0][k], out[1][k])


def test_window_length_changes_only_rounding(torch, lsd):
    _say("window length")
    w = W.config("c1")
    ref = None
    for K in (1, 3, 8):
        s = lsd.LSDSystem(w, mode="lsd", k_max=8)
        while s.state()["step"][0] < 30:
            s.draft_steps(min(K, 30 - int(s.state()["step"][0])))
            s.verify_window()
            s.accept_rollback(sync=True)
        st = s.state()
        s.destroy()
        if ref is None:
            ref = st
        else:
            assert np.max(np.abs(st["p"] - ref["p"])) < 1e-3
            assert np.array_equal(st["step"], ref["step"])


def test_neighbor_overflow_is_reported(torch, lsd):
    _say("overflow status")
    w = W.config("c1")
    s = lsd.LSDSystem(w, mode="lsd", max_neighbors=(32, 32))
    s.draft_steps(2)
    s.verify_window()
    s.accept_rollback(sync=True)
    assert s.status() & lsd.STATUS_NBR_TARGET
    s.destroy()


def test_uneven_replicas_verify_per_replica(torch, lsd, ora):
    _say("replica parity")
    w = W.lj_replicas([3, 4, 5, 6], seed=300, K=6)
    K, R = w.K, w.n_replicas
    g = lsd.LSDSystem(w, mode="lsd", replay=True)
    frames_q, frames_p, frames_f, us, refs = [], [], [], [], []
    for r in range(R):
        sl = w.replica_slice(r)
        n = sl.stop - sl.start
        xi = np.stack([ora.normals(77, r, s, n) for s in range(1, K + 1)])
        u = np.array([ora.uniform(77, r, s) for s in range(1, K + 1)])
        so = _ora_system(ora, w, r)
        T, D = _ora_pot(ora, w.target), _ora_pot(ora, w.draft)
        q, p = w.positions[sl].copy(), w.momenta[sl].copy()
        res = ora.lsd_window(so, T, D, q, p, np.zeros((n, 3), np.int32), xi, u)
        qm = W.f32(res["q_mid"])
        qm[qm >= so.L] = 0.0
        frames_q.append(qm)
        frames_p.append(W.f32(res["p_draft"]))
        frames_f.append(W.f32(res["F_draft"]))
        us.append(u)
        refs.append((so, T))
    qm, pd, fd = (np.concatenate(x, axis=1) for x in (frames_q, frames_p, frames_f))
    g.replay_u.copy_(torch.tensor(np.stack(us)))
    g.set_state(w.positions, pd[0])
    _inject(g, torch, qm, pd, fd)
    g.mark_drafted(K)
    g.verify_window()
    n = g.accept_rollback(sync=True)
    lr = g.log_ratio.cpu().numpy()
    acc = g.accepted.cpu().numpy()
    ft = g.window()["f_target"][:K].cpu().numpy().transpose(0, 2, 1)
    inv = g.window()["frame_invalid"].cpu().numpy()
    for r in range(R):
        sl = w.replica_slice(r)
        so, T = refs[r]
        keff = int(np.argmax(inv[r, :K])) if inv[r, :K].any() else K
        j, decided = keff, True
        for k in range(keff):
            v = ora.verify_frame(so, T, qm[k, sl], pd[k, sl], pd[k + 1, sl], fd[k, sl], us[r][k])
            dF = np.abs(ft[k, sl] - v["F_target"])
            assert dF.max() <= 1e-5 * np.abs(v["F_target"]).max(), (r, k)
            assert abs(lr[r, k] - v["logr"]) <= 1e-4 * max(1.0, abs(v["logr"])), (r, k)
            lu = np.log(us[r][k])
            if abs(v["logr"] - lu) <= max(1e-6 * max(1.0, abs(lu)), abs(lr[r, k] - v["logr"])):
                decided = False
                break
            assert bool(acc[r, k]) == v["accept"], (r, k)
            if not v["accept"]:
                j = k + 1
                break
        if decided:
            assert n[r] == j, (r, n[r], j)
    g.destroy()


def test_graph_replays_equal_eager_launches(torch, lsd):
    _say("graph vs eager")
    for mode in ("lsd", "plain"):
        w = W.config("c1")
        a = lsd.LSDSystem(w, mode=mode)
        b = lsd.LSDSystem(w, mode=mode)
        b.set_graphs(False)
        for rep in range(6):
            a.run_windows(3, 8)
            b.run_windows(3, 8)
            sa, sb = a.state(), b.state()   # synchronises between replays
            for k in ("q", "p", "img", "step"):
                assert np.array_equal(sa[k], sb[k]), (mode, rep, k)
            assert np.array_equal(a.counters(), b.counters())
        a.destroy()
        b.destroy()


@pytest.mark.parametrize("case", ["ec_constant", "ec_linear", "obabo", "replicas_short_skin"])
def test_graph_replays_equal_eager_launches_variants(torch, lsd, case):
    # the replayed windows fuse each commit with the next window's start;
    # with error correction (constant and linear caches), the (OBABO)
    # integrator, and ragged replicas with a short skin (many list rebuilds
    # and truncated windows) they must equal the eager calls bit for bit
    _say(f"graph vs eager {case}")
    kw = {}
    if case == "replicas_short_skin":
        w = W.lj_replicas([3, 4, 5, 6], seed=310, K=8)
        kw["skin"] = 0.1
    else:
        w = W.config("c1")
    if case == "ec_constant":
        kw["error_correction"] = 1
    elif case == "ec_linear":
        kw["error_correction"] = 2
    elif case == "obabo":
        kw["integrator"] = "obabo"
    a = lsd.LSDSystem(w, mode="lsd", **kw)
    b = lsd.LSDSystem(w, mode="lsd", **kw)
    b.set_graphs(False)
    for rep in range(5):
        a.run_windows(4, 8)
        b.run_windows(4, 8)
        sa, sb = a.state(), b.state()
        for k in ("q", "p", "img", "step"):
            assert np.array_equal(sa[k], sb[k]), (case, rep, k)
        assert np.array_equal(a.counters(), b.counters()), case
    assert a.counters()[:, 1].sum() > 0
    if case == "replicas_short_skin":
        assert a.counters()[:, 4].sum() > 5      # lists rebuilt many times
    a.destroy()
    b.destroy()


def _near_faces(w):
    """The C1 lattice shifted by half a spacing: a layer of atoms sits within
    the jitter of every box face, so many cross a face within a window."""
    L = float(w.box[0])
    a = L / 4
    x = np.mod(w.positions - 0.5 * a + 0.004, L)
    x = W.f32(x)
    x[x >= L] = 0.0
    return x


def test_forces_across_box_faces_inside_a_window(torch, lsd, ora):
    _say("box-face crossings")
    w = W.config("c1")
    w.positions = _near_faces(w)
    K, N = w.K, w.n_atoms
    L = float(w.box[0])
    xi = np.stack([ora.normals(5, 0, s, N) for s in range(1, K + 1)])
    u = np.ones(K)
    so, T, r = _oracle_window_rounded(ora, w, xi, u, w.positions, w.momenta)
    qm, pd, fd = W.f32(r["q_mid"]), W.f32(r["p_draft"]), W.f32(r["F_draft"])
    qm[qm >= L] = 0.0
    # the oracle frames do wrap: count atoms that crossed a face after frame 0
    jumps = np.abs(qm[1:] - qm[0][None]) > L / 2
    assert jumps.any(axis=(0, 2)).sum() >= 3
    # identical frames, made continuous by _inject: every target force matches
    g = lsd.LSDSystem(w, mode="lsd", replay=True)
    g.replay_u.copy_(torch.tensor(u[None, :]))
    g.set_state(w.positions, pd[0])
    _inject(g, torch, qm, pd, fd)
    g.mark_drafted(K)
    g.verify_window()
    g.accept_rollback(sync=True)
    inv = g.window()["frame_invalid"].cpu().numpy()[0]
    ft = g.window()["f_target"][:K].cpu().numpy().transpose(0, 2, 1)
    keff = int(np.argmax(inv[:K])) if inv[:K].any() else K
    assert keff >= 4
    for k in range(keff):
        E, F = ora.energy_forces(T, qm[k], L)
        assert np.max(np.abs(ft[k] - F)) <= 1e-5 * np.max(np.abs(F)), k
    g.destroy()
    # the GPU's own drafting across faces: per-frame draft forces follow the
    # oracle's trajectory (a lost pair would be an O(1) error)
    h = lsd.LSDSystem(w, mode="lsd", replay=True)
    h.replay_xi.copy_(torch.tensor(xi))
    h.replay_u.fill_(1.0)
    h.draft_steps(K)
    torch.cuda.synchronize()
    fdg = h.window()["f_draft"][:K].cpu().numpy().transpose(0, 2, 1)
    invh = h.window()["frame_invalid"].cpu().numpy()[0]
    keff = int(np.argmax(invh[:K])) if invh[:K].any() else K
    for k in range(keff):
        assert np.max(np.abs(fdg[k] - r["F_draft"][k])) <= 1e-3 * np.max(np.abs(r["F_draft"][k])), k
    h.verify_window()
    h.accept_rollback(sync=True)
    h.destroy()


@pytest.mark.parametrize("case", ["c1", "lj512"])
def test_reused_lists_hold_every_pair(torch, lsd, case):
    # lists kept across windows must contain every pair within the cutoff at
    # every verified frame: forces and energies on the same frames equal
    # those from lists built afresh (GPU against GPU; the summation order and
    # the binary32 shift of frame 0 back into the box differ)
    _say(f"list reuse {case}")
    w = W.config("c1") if case == "c1" else W.lj_fluid(8, seed=23, K=8)
    K, N = w.K, w.n_atoms
    a = lsd.LSDSystem(w, mode="lsd")
    a.run_windows(10, K)
    builds_before = int(a.counters()[0, 4])
    a.draft_steps(K)
    a.verify_window()
    torch.cuda.synchronize()
    win = a.window()
    qm = win["q_mid"][:K, :, :3].double().cpu().numpy()
    pd = win["p_draft"][:K + 1].double().cpu().numpy().transpose(0, 2, 1)
    fd = win["f_draft"][:K].double().cpu().numpy().transpose(0, 2, 1)
    ft_a = win["f_target"][:K].double().cpu().numpy().transpose(0, 2, 1)
    inv_a = win["frame_invalid"].cpu().numpy()[0][:K]
    a.accept_rollback(sync=True)
    e_a = a.energy.cpu().numpy()[0][:K]
    assert int(a.counters()[0, 0]) == 11
    # the lists were kept for at least one window (else nothing is tested)
    assert builds_before < 10, builds_before
    L = float(w.box[0])
    q0 = qm[0] - L * np.floor(qm[0] / L)
    q0[q0 >= L] = 0.0
    frames = np.concatenate([q0[None], qm[1:]])
    b = lsd.LSDSystem(w, mode="lsd")
    b.set_state(w.positions, pd[0])
    _inject(b, torch, frames, pd, fd)
    b.mark_drafted(K)
    b.verify_window()
    torch.cuda.synchronize()
    winb = b.window()
    ft_b = winb["f_target"][:K].double().cpu().numpy().transpose(0, 2, 1)
    inv_b = winb["frame_invalid"].cpu().numpy()[0][:K]
    b.accept_rollback(sync=True)
    e_b = b.energy.cpu().numpy()[0][:K]
    both = (inv_a == 0) & (inv_b == 0)
    assert both[0]
    for k in np.nonzero(both)[0]:
        scale = np.max(np.abs(ft_b[k]))
        assert np.max(np.abs(ft_a[k] - ft_b[k])) <= 1e-5 * scale, k
        assert abs(e_a[k] - e_b[k]) <= 1e-5 * abs(e_b[k]), k
    a.destroy()
    b.destroy()


def test_list_reuse_changes_only_rounding(torch, lsd):
    _say("list reuse vs rebuild")
    w = W.config("c1")
    a = lsd.LSDSystem(w, mode="lsd")
    b = lsd.LSDSystem(w, mode="lsd", list_reuse=False)
    a.run_windows(40, w.K)
    b.run_windows(40, w.K)
    sa, sb = a.state(), b.state()
    ca, cb = a.counters()[0], b.counters()[0]
    assert cb[4] == cb[0] and ca[4] < ca[0]
    # same decisions, states equal up to rounding (summation order)
    assert np.array_equal(ca[:3], cb[:3]), (ca, cb)
    assert np.array_equal(sa["step"], sb["step"])
    assert np.max(np.abs(sa["p"] - sb["p"])) < 1e-3
    dq = sa["q"] - sb["q"]
    dq -= float(w.box[0]) * np.round(dq / float(w.box[0]))
    assert np.max(np.abs(dq)) < 1e-3
    a.destroy()
    b.destroy()


def test_autotuned_verification_gives_identical_results(torch, lsd):
    # every frames-per-wave variant reduces a frame's sums in the same order,
    # so the tuned choice changes only the time taken
    _say("verification autotuner")
    w = W.lj_fluid(8, seed=29, K=8)
    a = lsd.LSDSystem(w, mode="lsd")
    b = lsd.LSDSystem(w, mode="lsd")
    chosen, us = a.autotune_verify(8, repeats=3)
    assert chosen in (1, 2, 4, 8) and all(v > 0 for v in us.values())
    a.verify_window()
    a.accept_rollback()
    b.draft_steps(8)
    b.verify_window()
    b.accept_rollback()
    a.run_windows(10, 8)
    b.run_windows(10, 8)
    sa, sb = a.state(), b.state()
    for k in ("q", "p", "img", "step"):
        assert np.array_equal(sa[k], sb[k]), k
    assert np.array_equal(a.log_ratio.cpu().numpy(), b.log_ratio.cpu().numpy())
    a.destroy()
    b.destroy()


def test_every_fixed_verification_variant_gives_identical_results(torch, lsd):
    # 512 atoms (8 tiles), windows of 12 frames: frame groups of 1, 2, 4 and
    # 8 frames, the last one ragged, over windows that the skin may truncate
    _say("fixed verification variants")
    w = W.lj_fluid(8, seed=31, K=12)
    runs = []
    for fw in (1, 2, 4, 8):
        g = lsd.LSDSystem(w, mode="lsd", error_correction=1)
        g.set_verify_variant(12, fw)
        g.run_windows(12, 12)
        st = g.state()
        runs.append((st, g.log_ratio.cpu().numpy(), g.counters()))
        with pytest.raises(lsd.LSDError):
            g.set_verify_variant(12, 3)
        with pytest.raises(lsd.LSDError):
            g.set_verify_variant(13, 2)
        g.destroy()
    for st, lr, cn in runs[1:]:
        for k in ("q", "p", "img", "step"):
            assert np.array_equal(st[k], runs[0][0][k]), k
        assert np.array_equal(lr, runs[0][1])
        assert np.array_equal(cn, runs[0][2])
    assert runs[0][2][:, 1].sum() > 0


def test_timed_windows_equal_untimed_windows(torch, lsd):
    # with verification timing the windows run as graph parts around an
    # event-bracketed verification launch; the trajectory is unchanged and
    # every launch is timed
    _say("timed vs untimed windows")
    w = W.config("c1")
    a = lsd.LSDSystem(w, mode="lsd")
    b = lsd.LSDSystem(w, mode="lsd")
    b.set_verify_timing(True)
    for n in (1, 7, 50):
        a.run_windows(n, 8)
        b.run_windows(n, 8)
    sa, sb = a.state(), b.state()
    for k in ("q", "p", "img", "step"):
        assert np.array_equal(sa[k], sb[k]), k
    assert np.array_equal(a.counters(), b.counters())
    ms, n = b.verify_timing()
    assert n == 58 and 0.0 < ms / n < 5.0, (ms, n)
    a.destroy()
    b.destroy()


@pytest.mark.parametrize("every", [2, 3])
def test_sampled_timing_windows_equal_untimed_windows(torch, lsd, every):
    # every n-th window timed: timed and untimed windows interleave (whole
    # window graphs between the timed parts), with an eager window and an
    # eager verification between the calls; trajectory and counters are
    # those of the untimed run, and exactly every n-th launch is timed
    _say(f"sampled timing every {every}")
    w = W.config("c1")
    a = lsd.LSDSystem(w, mode="lsd")
    b = lsd.LSDSystem(w, mode="lsd")
    b.set_verify_timing(True, every=every)
    launches = 0
    for n in (1, 7, 50):
        for g in (a, b):
            g.run_windows(n, 8)
            g.draft_steps(8)
            g.verify_window()
            g.accept_rollback()
        launches += n + 1
    sa, sb = a.state(), b.state()
    for k in ("q", "p", "img", "step"):
        assert np.array_equal(sa[k], sb[k]), k
    assert np.array_equal(a.counters(), b.counters())
    ms, n = b.verify_timing()
    # the n-th, 2n-th, ... launches after enabling are the timed ones
    assert n == launches // every and 0.0 < ms / n < 5.0, (ms, n, launches)
    with pytest.raises(lsd.LSDError):
        b.set_verify_timing(True, every=-1)
    a.destroy()
    b.destroy()


def test_plain_lj_matches_oracle_pathwise(torch, lsd, ora):
    # plain target Langevin through graph-replayed windows (Philox stream
    # keyed by step) against the oracle's plain ABOBA steps from the same
    # binary32 start: unwrapped positions and momenta after 48 steps within
    # the binary32 error of the forces and of the stored state, grown over
    # the steps
    _say("plain LJ pathwise c1")
    w = W.config("c1")
    n_steps, K = 48, w.K
    g = lsd.LSDSystem(w, mode="plain")
    g.run_to_step(n_steps, K, check_every=2)
    st = g.state()
    assert int(st["step"][0]) == n_steps and g.status() == 0
    g.destroy()
    so = _ora_system(ora, w)
    T = _ora_pot(ora, w.target)
    q, p = w.positions.copy(), W.f32(w.momenta)
    img = np.zeros(q.shape, np.int32)
    ora.plain_run(so, T, q, p, img, w.seed, 0, 0, n_steps)
    L = float(w.box[0])
    dq = (st["q"] + st["img"] * L) - (q + img * L)
    dp = st["p"] - p
    _say(f"  max |dq| {np.abs(dq).max():.2e}, max |dp| {np.abs(dp).max():.2e}")
    # per step: binary32 forces (1e-5 of max |F|) enter p through c1, and
    # p and q are stored in binary32; 48 steps with a growth factor of 4
    c1 = (1 + so.a) * so.dt / 2
    _, F0 = ora.energy_forces(T, w.positions, L)
    per_step = c1 * 1e-5 * np.abs(F0).max() + 2 ** -23 * (1 + np.abs(p).max())
    tol_p = 4 * n_steps * per_step
    assert np.abs(dp).max() <= tol_p, (np.abs(dp).max(), tol_p)
    assert np.abs(dq).max() <= so.dt * n_steps * tol_p + 4 * n_steps * 2 ** -24 * L
