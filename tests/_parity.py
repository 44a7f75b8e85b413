"""Shared checks of GPU windows against oracle windows on identical inputs.

Decisions (Eq. reflectionVerify, accept iff log u <= log r) must agree
except inside the band |log r_oracle - log u| <= max(1e-6 max(|log u|, 1),
|log r_gpu - log r_oracle|); the log ratios and committed momenta are
bounded by first-order propagation of the measured force differences and of
binary32 rounding through the (BOB) update of Eq. bob and the reflection.
"""
import numpy as np

U32 = 2.0 ** -24   # unit roundoff of binary32


def first_decision_mismatch(acc_g, acc_o, logr_g, logr_o, u, upto):
    """Index of the first frame < upto whose decisions differ, or None.  A
    differing decision must lie inside the band; otherwise AssertionError."""
    for k in range(upto):
        if bool(acc_g[k]) != bool(acc_o[k]):
            lu = float(np.log(u[k]))
            margin = max(1e-6 * max(abs(lu), 1.0), abs(float(logr_g[k]) - float(logr_o[k])))
            assert abs(float(logr_o[k]) - lu) <= margin, (
                f"decision of frame {k} differs outside the band: log r oracle {logr_o[k]!r}, "
                f"gpu {logr_g[k]!r}, log u {lu!r}")
            return k
    return None


def draft_chain_bounds(a, c1, dFc, pd_o):
    """Bounds D[k] of |p~_k gpu - p~_k oracle| (max over components) along
    the draft chain p~_k = a p~_{k-1} + c1 F~c_k + sigma xi_k from identical
    p~_0: dFc[k] bounds the corrected draft force difference of frame k,
    and each stored momentum is rounded to binary32."""
    K = len(dFc)
    D = np.zeros(K + 1)
    for k in range(K):
        D[k + 1] = a * D[k] + c1 * np.max(dFc[k]) + 2.0 * U32 * np.abs(pd_o[k + 1]).max()
    return D


def logr_bound(xi, delta_o, sig, c1, dFt, dFc, Dk, Dk1, logr_o):
    """First-order bound of |log r_gpu - log r_oracle| for one frame: log r
    = -delta.z - |delta|^2 / 2, z = (p~_k+1 - <p~>) / sigma (the frame's
    normal draw) and delta = c1 (F~c - F) / sigma; dFt, dFc bound the target
    and corrected draft force differences, Dk, Dk1 the draft momenta."""
    d_delta = c1 * (dFt + dFc) / sig
    d_z = (Dk1 + Dk + c1 * dFc) / sig + 2.0 * U32 * (1.0 + np.abs(xi))
    w = np.abs(xi) + np.abs(delta_o)
    return (2.0 * np.sum(w * d_delta + (np.abs(delta_o) + np.abs(d_delta)) * d_z)
            + 1e-9 * max(1.0, abs(logr_o)))


def reflected_p_bound(a, c1, sig, xi, delta_o, dFt, dFc, Dk, Dk1, p_o):
    """Bound of |p_gpu - p_oracle| (max over components) for a reflected
    frame: p = <p> + sigma (z - 2 (dhat.z) dhat), dhat = delta / |delta|,
    <p> = a p~_k + c1 F.  The reflection of z moves by at most
    3 |dz| + 4 |z| |d dhat| <= 3 |dz| + 8 |z| |d delta| / |delta|."""
    nd = max(np.linalg.norm(delta_o), 1e-300)
    d_delta = np.linalg.norm(c1 * (dFt + dFc) / sig)
    d_z = np.linalg.norm((Dk1 + Dk + c1 * dFc) / sig) + 2.0 * U32 * (1.0 + np.linalg.norm(xi))
    refl = 3.0 * d_z + 8.0 * np.linalg.norm(xi) * d_delta / nd
    return (2.0 * (a * Dk + c1 * np.max(dFt) + sig.max() * refl)
            + 4.0 * U32 * (1.0 + np.abs(p_o).max()))


def run_tether_windows(torch, lsd, ora, w, k_target, k_draft, n_steps, K, ec_mode=0,
                       obabo=False, say=print):
    """Windows of K frames on one-atom tether replicas (target stiffness
    k_target, draft k_draft), GPU against oracle, each window started on both
    sides from the same binary32 state (positions, momenta and, with error
    correction, the caches).  Returns (replicas compared to the end, replicas
    whose paths parted at a band decision, rejections seen)."""
    R = w.n_replicas
    anchor = w.positions.copy()
    draft = dict(kind="harmonic", k=k_draft, anchor=anchor)
    kw = dict(error_correction=ec_mode) if ec_mode else {}
    if obabo:
        kw["integrator"] = "obabo"
    g = lsd.LSDSystem(w, mode="lsd", draft=draft, skin=8.0, **kw)
    g.set_step_limit(n_steps)
    so = [ora.System(1, float(w.box[r]), w.species_mass[0], w.dt, w.gamma, w.kT)
          for r in range(R)]
    T = [ora.Potential.harmonic(k_target, anchor[r:r + 1]) for r in range(R)]
    D = [ora.Potential.harmonic(k_draft, anchor[r:r + 1]) for r in range(R)]
    a = float(np.exp(-w.gamma * w.dt))
    c1 = (1.0 + a) * w.dt / 2.0 * w.force_unit
    sig = so[0].sigma()[:, None]
    hdt_m = 0.5 * w.dt / float(w.species_mass[0])
    f32 = lambda v: np.asarray(v, np.float32).astype(np.float64)
    q = f32(w.positions)
    p = f32(w.momenta)
    if obabo:
        # the initial OB half step (App. E): compare the GPU's start first
        qg0 = g.q.T.double().cpu().numpy()
        pg0 = g.p.T.double().cpu().numpy()
        for r in range(R):
            qr, pr, ir = q[r:r + 1].copy(), p[r:r + 1].copy(), np.zeros((1, 3), np.int32)
            ora.obabo_begin(so[r], T[r], qr, pr, ir, w.seed, r, 0)
            q[r], p[r] = qr[0], pr[0]
        assert np.max(np.abs(pg0 - p)) <= 8 * U32 * (1 + np.abs(p).max())
        assert np.max(np.abs(qg0 - q)) <= 8 * U32 * (1 + np.abs(q).max())
    ec = np.zeros((R, 3))
    ecp = np.zeros((R, 3))
    samples = np.zeros(R, np.int32)
    steps = np.zeros(R, np.int64)
    active = np.ones(R, bool)
    parted, rejections = 0, 0
    win = g.window()
    while (steps[active] < n_steps).any():
        q, p, ec, ecp = f32(q), f32(p), f32(ec), f32(ecp)
        g.set_state(q, p, img=np.zeros((R, 3), np.int32), step=steps)
        if ec_mode:
            win["error_cache"].copy_(torch.tensor(ec.T, dtype=torch.float32))
            if ec_mode == 2:
                win["error_cache_prev"].copy_(torch.tensor(ecp.T, dtype=torch.float32))
        g.draft_steps(K)
        g.verify_window()
        n_g = g.accept_rollback(sync=True)
        lr_g = g.log_ratio.cpu().numpy()
        acc_g = g.accepted.cpu().numpy()
        qg = g.q.T.double().cpu().numpy()
        pg = g.p.T.double().cpu().numpy()
        ft_g = win["f_target"][:K].double().cpu().numpy().transpose(0, 2, 1)
        fd_g = win["f_draft"][:K].double().cpu().numpy().transpose(0, 2, 1)
        ec_g = win["error_cache"].double().cpu().numpy().T if ec_mode else None
        if obabo:
            oq_g = g.obabo_q.T.double().cpu().numpy()
            op_g = g.obabo_p.T.double().cpu().numpy()
        for r in np.nonzero(active & (steps < n_steps))[0]:
            Kw = int(min(K, n_steps - steps[r]))
            xi = np.stack([ora.normals(w.seed, int(r), int(steps[r]) + k + 1, 1) for k in range(Kw)])
            u = np.array([ora.uniform(w.seed, int(r), int(steps[r]) + k + 1) for k in range(Kw)])
            qo, po, io = q[r:r + 1].copy(), p[r:r + 1].copy(), np.zeros((1, 3), np.int32)
            eco = ec[r:r + 1].copy() if ec_mode else None
            ecpo = ecp[r:r + 1].copy() if ec_mode == 2 else None
            smp = samples[r:r + 1].copy()
            ec_in, ecp_in, smp_in = (None if eco is None else eco.copy(),
                                     None if ecpo is None else ecpo.copy(), int(smp[0]))
            res = ora.lsd_window(so[r], T[r], D[r], qo, po, io, xi, u, ec=eco, ec_prev=ecpo,
                                 samples=smp if ec_mode else None)
            j = int(res["n_committed"])
            if first_decision_mismatch(acc_g[r], res["accept"], lr_g[r], res["logr"], u, j) is not None:
                active[r] = False
                parted += 1
                continue
            assert int(n_g[r]) == j, (r, int(n_g[r]), j)
            rejections += int(res["rejected"])
            # corrected draft forces of the oracle and the force differences
            dFt, dFc, dlt = [], [], []
            for k in range(j):
                corr = np.zeros((1, 3))
                if ec_mode:
                    corr = ec_in.copy()
                    if ec_mode == 2 and smp_in >= 2:
                        corr = ec_in + (k + 1) * (ec_in - ecp_in)
                Fc = res["F_draft"][k] + corr
                dFt.append(np.abs(ft_g[k, r:r + 1] - res["F_target"][k]))
                dFc.append(np.abs(fd_g[k, r:r + 1] - res["F_draft"][k])
                           + 4.0 * U32 * (k + 2) * np.abs(corr) + 2.0 * U32 * np.abs(Fc))
                dlt.append(c1 * (Fc - res["F_target"][k]) / sig)
            Db = draft_chain_bounds(a, c1, dFc, res["p_draft"])
            for k in range(j):
                bnd = logr_bound(xi[k], dlt[k], sig, c1, dFt[k], dFc[k], Db[k], Db[k + 1],
                                 res["logr"][k])
                assert abs(lr_g[r, k] - res["logr"][k]) <= bnd, (r, k, lr_g[r, k], res["logr"][k], bnd)
            if res["rejected"]:
                tol_p = reflected_p_bound(a, c1, sig, xi[j - 1], dlt[j - 1], dFt[j - 1], dFc[j - 1],
                                          Db[j - 1], Db[j], po)
            else:
                tol_p = Db[j] + 4.0 * U32 * (1.0 + np.abs(po).max())
            assert np.max(np.abs(pg[r] - po[0])) <= tol_p, (r, np.max(np.abs(pg[r] - po[0])), tol_p)
            tol_q = (2 * hdt_m * (Db[:j + 1].sum() + tol_p)
                     + 2.0 * (2 * j + 2) * U32 * np.abs(qo).max())
            dq = qg[r] - qo[0]
            assert np.max(np.abs(dq)) <= tol_q, (r, np.max(np.abs(dq)), tol_q)
            if ec_mode:
                tol_ec = dFt[j - 1].max() + np.max(dFc[j - 1]) + 4 * U32 * (1 + np.abs(eco).max())
                assert np.max(np.abs(ec_g[r] - eco[0])) <= tol_ec, (r, ec_g[r], eco[0], tol_ec)
            if obabo:
                # recovered (OBABO) state of the last committed step
                qr, pr = ora.obabo_recover(so[r], T[r], qo, po, res["p_draft"][j - 1], w.seed,
                                           int(r), int(steps[r]) + j)
                ah = float(np.exp(-0.5 * w.gamma * w.dt))
                cw = ah / (1.0 + a)
                hk = 0.5 * w.dt * w.force_unit
                tol_r = (2.0 * (ah * Db[j - 1] + (ah + cw * (1 + a)) * hk * dFt[j - 1].max()
                                + cw * (tol_p + a * Db[j - 1]))
                         + 8.0 * U32 * (1.0 + np.abs(pr).max()))
                assert np.max(np.abs(op_g[r] - pr[0])) <= tol_r, (r, op_g[r], pr[0], tol_r)
                assert np.max(np.abs(oq_g[r] - qr[0])) <= tol_q, (r, oq_g[r], qr[0])
            q[r], p[r] = qo[0], po[0]
            if ec_mode:
                ec[r] = eco[0]
                if ec_mode == 2:
                    ecp[r] = ecpo[0]
                samples[r] = smp[0]
            steps[r] += j
    g.destroy()
    compared = int(active.sum())
    say(f"  {compared} replicas compared to step {n_steps}, {parted} parted at a band decision, "
        f"{rejections} reflected windows")
    return compared, parted, rejections
