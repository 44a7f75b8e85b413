"""Oracle pins: ABOBA integrator, reflection coupling and the LSD window.

* ABOBA on a harmonic tether has the exact stationary law Var(q) = kT/k
  (the Boltzmann marginal, Sec. 2.1) and Var(p) = m kT / (1 - (omega dt/2)^2),
  Cov(q, p) = 0 (solution of the 2x2 discrete Lyapunov equation of the step).
* reflectionVerify (Eq. reflectionVerify) accepts with probability
  1 - erf(|delta| / sqrt 8) (Eq. rejection_rate), outputs target-distributed
  momenta (Eq. coupling), and is a Householder reflection of z.
* With draft == target every step is accepted and the trajectory is plain
  target Langevin (Sec. 2.2, "Probabilistic verification").
* With the step-keyed stream the committed trajectory does not depend on the
  window length K.
"""
import numpy as np
import pytest
from scipy import special, stats

from paper_2606_02455_amd import workloads as W


def _tether_system(ora, n, k, m=1.0, dt=0.1, gamma=1.0, kT=0.7, L=1000.0):
    qref = np.full((n, 3), L / 2)
    sysm = ora.System(n, L, m, dt, gamma, kT)
    return sysm, ora.Potential.harmonic(k, qref), qref


def test_aboba_harmonic_stationary_law(ora):
    n, k, m, dt, kT = 4096, 2.0, 1.3, 0.6, 0.7
    sysm, pot, qref = _tether_system(ora, n, k, m=m, dt=dt, gamma=0.8, kT=kT)
    q, p = qref.copy(), np.zeros((n, 3))
    img = np.zeros((n, 3), np.int32)
    ora.plain_run(sysm, pot, q, p, img, seed=5, replica=0, step0=0, n_steps=300)
    dq = (q - qref).ravel()
    var_p = m * kT / (1.0 - (k / m) * dt * dt / 4.0)
    assert stats.kstest(dq / np.sqrt(kT / k), "norm").pvalue > 1e-3
    assert stats.kstest(p.ravel() / np.sqrt(var_p), "norm").pvalue > 1e-3
    assert abs(np.corrcoef(dq, p.ravel())[0, 1]) < 0.03
    # the continuous-time momentum variance m kT is measurably wrong here
    assert stats.kstest(p.ravel() / np.sqrt(m * kT), "norm").pvalue < 1e-3


def test_aboba_energy_conservation_without_thermostat_noise(ora):
    # kT = 0 and tiny friction: ABOBA is velocity Verlet with friction; the
    # total energy drifts down only by friction and shows no secular heating.
    w = W.config("c1")
    sysm = ora.System(64, float(w.box[0]), 1.0, 0.002, 1e-9, 0.0)
    pot = ora.Potential.lj(2.5)
    q, p = w.positions.copy(), w.momenta.copy()
    img = np.zeros((64, 3), np.int32)
    xi = np.zeros((64, 3))
    H = []
    for t in range(500):
        ora.aboba_step(sysm, pot, q, p, img, xi)
        E, _ = ora.energy_forces(pot, q, sysm.L)
        H.append(E + 0.5 * (p ** 2).sum())
    H = np.array(H)
    assert np.max(np.abs(H - H[0])) < 2e-3 * (np.abs(H[0]) + 64)


# --- reflection coupling ---------------------------------------------------
def _gauss_pair(m, dnorm, seed):
    rng = np.random.default_rng(seed)
    sig = rng.uniform(0.5, 2.0, m)
    mu_d = rng.normal(size=m)
    direction = rng.normal(size=m)
    direction /= np.linalg.norm(direction)
    mu_t = mu_d - sig * dnorm * direction   # delta = (mu_d - mu_t)/sig = dnorm * dir
    return mu_t, mu_d, sig


@pytest.mark.parametrize("dnorm", [0.3, 1.0, 2.5])
def test_reflection_acceptance_closed_form(ora, dnorm):
    m, M = 6, 20000
    mu_t, mu_d, sig = _gauss_pair(m, dnorm, 1)
    rng = np.random.default_rng(2)
    acc = 0
    outs = np.zeros((M, m))
    for t in range(M):
        pd = mu_d + sig * rng.normal(size=m)
        a, po, lr, s1, s2 = ora.reflection_verify(mu_t, mu_d, sig, pd, rng.uniform(0, 1))
        acc += a
        outs[t] = po
        assert s2 == pytest.approx(dnorm ** 2, rel=1e-12)
    beta = special.erf(dnorm / np.sqrt(8.0))         # Eq. rejection_rate
    alpha = 1.0 - beta
    sd = np.sqrt(alpha * (1 - alpha) / M)
    assert abs(acc / M - alpha) < 4 * sd
    # coupling: the output is N(mu_t, Sigma) whatever happened
    z = (outs - mu_t) / sig
    for c in range(m):
        assert stats.kstest(z[:, c], "norm").pvalue > 1e-3
    # along delta as well
    dirn = (mu_d - mu_t) / sig
    dirn /= np.linalg.norm(dirn)
    assert stats.kstest(z @ dirn, "norm").pvalue > 1e-3


def test_reflection_is_householder(ora):
    m = 9
    mu_t, mu_d, sig = _gauss_pair(m, 3.0, 4)
    rng = np.random.default_rng(5)
    seen = 0
    for t in range(200):
        pd = mu_d + sig * rng.normal(size=m)
        a, po, lr, s1, s2 = ora.reflection_verify(mu_t, mu_d, sig, pd, 1.0)
        z = (pd - mu_d) / sig
        delta = (mu_d - mu_t) / sig
        # log ratio: the two Mahalanobis norms equal -delta.z - |delta|^2 / 2
        assert lr == pytest.approx(-s1 - 0.5 * s2, abs=1e-10)
        if a:
            assert np.array_equal(po, pd)
            continue
        seen += 1
        zr = (po - mu_t) / sig
        assert np.linalg.norm(zr) == pytest.approx(np.linalg.norm(z), rel=1e-12)
        assert delta @ zr == pytest.approx(-(delta @ z), rel=1e-10, abs=1e-10)
        # components orthogonal to delta are unchanged
        P = np.eye(m) - np.outer(delta, delta) / (delta @ delta)
        assert np.allclose(P @ zr, P @ z, atol=1e-12)
    assert seen > 50


def test_reflection_equal_means_always_accepts(ora):
    m = 5
    rng = np.random.default_rng(0)
    mu = rng.normal(size=m)
    sig = np.ones(m)
    for _ in range(100):
        pd = mu + rng.normal(size=m)
        a, po, lr, s1, s2 = ora.reflection_verify(mu, mu, sig, pd, 1.0)
        assert a and lr == 0.0 and s2 == 0.0


# --- whole windows -----------------------------------------------------------
def _c1(ora):
    w = W.config("c1")
    sysm = ora.System(64, float(w.box[0]), 1.0, w.dt, w.gamma, w.kT)
    return w, sysm, ora.Potential.lj(2.5), ora.Potential.lj(1.5)


def test_draft_equals_target_is_plain_langevin(ora):
    w, sysm, T, _ = _c1(ora)
    q1, p1, i1 = w.positions.copy(), w.momenta.copy(), np.zeros((64, 3), np.int32)
    st, tq, tp = ora.lsd_run(sysm, T, T, q1, p1, i1, seed=9, replica=0, step0=0,
                             n_steps=120, K=8, record=True)
    assert st["rejections"] == 0 and st["committed"] == 120 and st["windows"] == 15
    q2, p2, i2 = w.positions.copy(), w.momenta.copy(), np.zeros((64, 3), np.int32)
    _, pq, pp = ora.plain_run(sysm, T, q2, p2, i2, seed=9, replica=0, step0=0, n_steps=120,
                              record=True)
    assert np.array_equal(tq, pq) and np.array_equal(tp, pp)
    assert np.array_equal(i1, i2)


def test_window_length_invariance(ora):
    w, sysm, T, D = _c1(ora)
    ref = None
    for K in (1, 2, 8, 16):
        q, p, img = w.positions.copy(), w.momenta.copy(), np.zeros((64, 3), np.int32)
        st, tq, tp = ora.lsd_run(sysm, T, D, q, p, img, seed=3, replica=0, step0=0,
                                 n_steps=80, K=K, record=True)
        assert st["committed"] == 80
        if ref is None:
            ref = (tq, tp, img.copy(), st)
            assert 0 < st["rejections"] < 80
        else:
            assert np.array_equal(tq, ref[0]) and np.array_equal(tp, ref[1])
            assert np.array_equal(img, ref[2])
            assert st["rejections"] == ref[3]["rejections"]


def test_window_commits_prefix_through_first_rejection(ora):
    w, sysm, T, D = _c1(ora)
    K = 8
    xi = np.stack([ora.normals(4, 0, s, 64) for s in range(1, K + 1)])
    u = np.array([ora.uniform(4, 0, s) for s in range(1, K + 1)])
    q, p, img = w.positions.copy(), w.momenta.copy(), np.zeros((64, 3), np.int32)
    r = ora.lsd_window(sysm, T, D, q, p, img, xi, u)
    acc = r["accept"]
    j = r["n_committed"]
    if acc.all():
        assert j == K and not r["rejected"]
        assert np.array_equal(p, r["p_draft"][K])
    else:
        first = int(np.argmin(acc))
        assert j == first + 1 and r["rejected"]
        assert not np.array_equal(p, r["p_draft"][j])
    # frames are verified against the stored draft forces and momenta
    for k in range(K):
        v = ora.verify_frame(sysm, T, r["q_mid"][k], r["p_draft"][k], r["p_draft"][k + 1],
                             r["F_draft"][k], u[k])
        assert v["accept"] == bool(acc[k])
        assert v["logr"] == pytest.approx(r["logr"][k], rel=1e-12, abs=1e-12)
    # decision rule of Eq. reflectionVerify with u in (0, 1]
    assert np.array_equal(acc, u <= np.minimum(1.0, np.exp(r["logr"])))


def test_offset_draft_rejection_rate_closed_form(ora):
    # draft forces F~ = F + b: delta = c1 fu b / sigma at every state, so each
    # step is rejected with probability erf(|delta| / sqrt 8) (Eq. rejection_rate)
    n, k = 4, 1.5
    sysm, T, qref = _tether_system(ora, n, k, dt=0.05, gamma=1.0, kT=1.0)
    rng = np.random.default_rng(6)
    b = rng.normal(size=(n, 3))
    sig = sysm.sigma()[:, None]
    c1 = (1 + sysm.a) * sysm.dt / 2
    dnorm = np.linalg.norm(c1 * b / sig)
    # scale b so the rejection rate is about 0.3
    b *= 0.85 / dnorm
    dnorm = 0.85
    D = T.with_offset(b)
    q, p, img = qref.copy(), np.zeros((n, 3)), np.zeros((n, 3), np.int32)
    st, _, _ = ora.lsd_run(sysm, T, D, q, p, img, seed=12, replica=0, step0=0,
                           n_steps=20000, K=4)
    beta = special.erf(dnorm / np.sqrt(8.0))
    rate = st["rejections"] / st["committed"]
    sd = np.sqrt(beta * (1 - beta) / st["committed"])
    assert abs(rate - beta) < 4 * sd


def test_lsd_harmonic_marginals_are_target(ora):
    # target tether k_T, draft tether k_D: the committed states after many
    # steps follow the exact ABOBA law of the TARGET (Thm. 1); the draft alone
    # does not.
    kT_, kD, m, dt, kT = 2.0, 1.0, 1.0, 0.2, 1.0
    n_rep, steps = 2500, 60
    qs, ps, qd = [], [], []
    rej = com = 0
    for r in range(n_rep):
        sysm, T, qref = _tether_system(ora, 1, kT_, m=m, dt=dt, gamma=2.0, kT=kT)
        D = ora.Potential.harmonic(kD, qref)
        q, p, img = qref.copy(), np.zeros((1, 3)), np.zeros((1, 3), np.int32)
        st, _, _ = ora.lsd_run(sysm, T, D, q, p, img, seed=21, replica=r, step0=0,
                               n_steps=steps, K=4)
        rej += st["rejections"]
        com += st["committed"]
        qs.append(q[0] - qref[0])
        ps.append(p[0])
        q2, p2, i2 = qref.copy(), np.zeros((1, 3)), np.zeros((1, 3), np.int32)
        ora.plain_run(sysm, D, q2, p2, i2, seed=21, replica=r, step0=0, n_steps=steps)
        qd.append(q2[0] - qref[0])
    qs, ps, qd = np.ravel(qs), np.ravel(ps), np.ravel(qd)
    assert 0.05 < rej / com < 0.95
    var_p = m * kT / (1.0 - (kT_ / m) * dt * dt / 4.0)
    assert stats.kstest(qs / np.sqrt(kT / kT_), "norm").pvalue > 0.01
    assert stats.kstest(ps / np.sqrt(var_p), "norm").pvalue > 0.01
    assert stats.kstest(qd / np.sqrt(kT / kT_), "norm").pvalue < 1e-4


# --- speculative error correction (App. D, Alg. 3) --------------------------
def test_error_correction_cancels_a_constant_draft_error(ora):
    # draft F~ = F + b: after the first committed step the cache holds
    # dF = F - F~_bare = -b, so every later proposal has the target mean and
    # is accepted; without correction the rejection rate stays erf(|delta|/sqrt 8)
    n, k = 4, 1.5
    sysm, T, qref = _tether_system(ora, n, k, dt=0.05, gamma=1.0, kT=1.0)
    rng = np.random.default_rng(16)
    b = rng.normal(size=(n, 3))
    sig = sysm.sigma()[:, None]
    c1 = (1 + sysm.a) * sysm.dt / 2
    b *= 1.2 / np.linalg.norm(c1 * b / sig)
    D = T.with_offset(b)
    q, p, img = qref.copy(), np.zeros((n, 3)), np.zeros((n, 3), np.int32)
    ec = np.zeros((n, 3))
    st, _, _ = ora.lsd_run(sysm, T, D, q, p, img, seed=3, replica=0, step0=0, n_steps=2000, K=4,
                           ec=ec)
    assert np.allclose(ec, -b, atol=1e-12)
    # at most the windows before the first commit can reject
    assert st["rejections"] <= 1
    q2, p2, i2 = qref.copy(), np.zeros((n, 3)), np.zeros((n, 3), np.int32)
    st2, _, _ = ora.lsd_run(sysm, T, D, q2, p2, i2, seed=3, replica=0, step0=0, n_steps=2000, K=4)
    assert st2["rejections"] > 200


def test_error_correction_keeps_target_marginals(ora):
    kT_, kD, m, dt, kT = 2.0, 1.0, 1.0, 0.2, 1.0
    qs, ps = [], []
    for r in range(2000):
        sysm, T, qref = _tether_system(ora, 1, kT_, m=m, dt=dt, gamma=2.0, kT=kT)
        D = ora.Potential.harmonic(kD, qref)
        q, p, img = qref.copy(), np.zeros((1, 3)), np.zeros((1, 3), np.int32)
        ec = np.zeros((1, 3))
        ora.lsd_run(sysm, T, D, q, p, img, seed=77, replica=r, step0=0, n_steps=60, K=4, ec=ec)
        qs.append(q[0] - qref[0])
        ps.append(p[0])
    var_p = m * kT / (1.0 - (kT_ / m) * dt * dt / 4.0)
    assert stats.kstest(np.ravel(qs) / np.sqrt(kT / kT_), "norm").pvalue > 0.01
    assert stats.kstest(np.ravel(ps) / np.sqrt(var_p), "norm").pvalue > 0.01


# --- linear variant of the error correction ---------------------------------
def _mismatch_run(ora, mode, replicas=4, n_steps=1000):
    rej = com = 0
    for r in range(replicas):
        sysm, T, qref = _tether_system(ora, 4, 20.0, dt=0.05, gamma=0.1, kT=1.0)
        D = ora.Potential.harmonic(1.0, qref)
        q, p, img = qref.copy(), np.zeros((4, 3)), np.zeros((4, 3), np.int32)
        ec = np.zeros((4, 3)) if mode >= 1 else None
        ecp = np.zeros((4, 3)) if mode == 2 else None
        st, _, _ = ora.lsd_run(sysm, T, D, q, p, img, seed=5, replica=r, step0=0, n_steps=n_steps,
                               K=4, ec=ec, ec_prev=ecp)
        rej += st["rejections"]
        com += st["committed"]
    return rej / com


def test_linear_error_correction_tracks_a_smoothly_varying_error(ora):
    # stiff target, soft draft, light friction: the draft error follows the
    # smooth trajectory, so extrapolating it from the last two committed steps
    # rejects far less often than holding it constant
    r0, r1, r2 = (_mismatch_run(ora, m) for m in (0, 1, 2))
    assert r0 > 0.95
    assert r2 < 0.75 * r1, (r1, r2)


def test_linear_error_correction_cancels_a_constant_error(ora):
    n = 4
    sysm, T, qref = _tether_system(ora, n, 1.5, dt=0.05, gamma=1.0, kT=1.0)
    rng = np.random.default_rng(21)
    b = rng.normal(size=(n, 3))
    sig = sysm.sigma()[:, None]
    c1 = (1 + sysm.a) * sysm.dt / 2
    b *= 1.2 / np.linalg.norm(c1 * b / sig)
    D = T.with_offset(b)
    q, p, img = qref.copy(), np.zeros((n, 3)), np.zeros((n, 3), np.int32)
    ec, ecp = np.zeros((n, 3)), np.zeros((n, 3))
    st, _, _ = ora.lsd_run(sysm, T, D, q, p, img, seed=3, replica=0, step0=0, n_steps=2000, K=4,
                           ec=ec, ec_prev=ecp)
    assert np.allclose(ec, -b, atol=1e-12) and np.allclose(ecp, -b, atol=1e-12)
    assert st["rejections"] <= 1


def test_linear_error_correction_keeps_target_marginals(ora):
    kT_, kD, m, dt, kT = 2.0, 1.0, 1.0, 0.2, 1.0
    qs, ps = [], []
    for r in range(2000):
        sysm, T, qref = _tether_system(ora, 1, kT_, m=m, dt=dt, gamma=2.0, kT=kT)
        D = ora.Potential.harmonic(kD, qref)
        q, p, img = qref.copy(), np.zeros((1, 3)), np.zeros((1, 3), np.int32)
        ora.lsd_run(sysm, T, D, q, p, img, seed=79, replica=r, step0=0, n_steps=60, K=4,
                    ec=np.zeros((1, 3)), ec_prev=np.zeros((1, 3)))
        qs.append(q[0] - qref[0])
        ps.append(p[0])
    var_p = m * kT / (1.0 - (kT_ / m) * dt * dt / 4.0)
    assert stats.kstest(np.ravel(qs) / np.sqrt(kT / kT_), "norm").pvalue > 0.01
    assert stats.kstest(np.ravel(ps) / np.sqrt(var_p), "norm").pvalue > 0.01


# --- (OBABO) splitting (App. E) ---------------------------------------------
# For a harmonic force the (OBABO) chain samples the momenta exactly,
# Var p = m kT, and the positions with Var q = kT / (k (1 - w^2 dt^2 / 4))
# (w^2 = k / m); (ABOBA) has these two the other way round.
def _obabo_samples(ora, runner, kT_, m, dt, replicas, steps, draft_k=None):
    qs, ps = [], []
    for r in range(replicas):
        sysm, T, qref = _tether_system(ora, 1, kT_, m=m, dt=dt, gamma=1.0, kT=1.0)
        q, p, img = qref.copy(), np.zeros((1, 3)), np.zeros((1, 3), np.int32)
        if runner == "plain":
            ora.obabo_plain_run(sysm, T, q, p, img, 11, r, 0, steps)
        else:
            D = ora.Potential.harmonic(draft_k, qref)
            ora.obabo_lsd_run(sysm, T, D, q, p, img, 13, r, steps, 4)
        qs.append(q[0] - qref[0])
        ps.append(p[0])
    return np.ravel(qs), np.ravel(ps)


def test_obabo_plain_harmonic_law(ora):
    kT_, m, dt = 2.0, 1.0, 0.6
    qs, ps = _obabo_samples(ora, "plain", kT_, m, dt, 2000, 60)
    var_q = 1.0 / kT_ / (1.0 - (kT_ / m) * dt * dt / 4.0)
    assert stats.kstest(qs / np.sqrt(var_q), "norm").pvalue > 0.01
    assert stats.kstest(ps / np.sqrt(m), "norm").pvalue > 0.01
    # the (ABOBA) momentum law is rejected
    assert stats.kstest(ps / np.sqrt(m / (1.0 - (kT_ / m) * dt * dt / 4.0)), "norm").pvalue < 1e-3


def test_obabo_lsd_outputs_follow_the_obabo_law(ora):
    # staggered LSD with a softer draft plus the conditional half-step
    # recovery gives (OBABO) states with exactly the plain (OBABO) law
    kT_, m, dt = 2.0, 1.0, 0.6
    qs, ps = _obabo_samples(ora, "lsd", kT_, m, dt, 2000, 60, draft_k=1.2)
    var_q = 1.0 / kT_ / (1.0 - (kT_ / m) * dt * dt / 4.0)
    assert stats.kstest(qs / np.sqrt(var_q), "norm").pvalue > 0.01
    assert stats.kstest(ps / np.sqrt(m), "norm").pvalue > 0.01
    assert stats.kstest(ps / np.sqrt(m / (1.0 - (kT_ / m) * dt * dt / 4.0)), "norm").pvalue < 1e-3


def test_obabo_lsd_accepts_everything_when_draft_is_target(ora):
    n = 3
    sysm, T, qref = _tether_system(ora, n, 2.0, dt=0.3, gamma=1.0, kT=1.0)
    q, p, img = qref.copy(), np.zeros((n, 3)), np.zeros((n, 3), np.int32)
    st = ora.obabo_lsd_run(sysm, T, T, q, p, img, 5, 0, 200, 8)
    assert st["rejections"] == 0 and st["committed"] == 200


# --- image counters of committed states (map g after a reflection) ----------
def test_image_counters_unwrap_to_the_unbounded_trajectory(ora):
    # Forces that do not depend on the positions (a zero-stiffness tether plus
    # constant offsets; draft and target offsets differ, so windows end in
    # reflected steps) make the momenta, decisions and unwrapped positions
    # independent of the box.  Windows in a small periodic box, where atoms
    # cross faces in every half step, must therefore give q + img L equal to
    # the positions of the same windows in a box too large to wrap.  This
    # pins the counters of every committed state, including the reflected
    # step's midpoint and map g (Eq. reflectionVerify, Thm. 1).
    n, K, L, big = 200, 6, 2.0, 1024.0
    rng = np.random.default_rng(91)
    q0 = rng.uniform(0.0, L, (n, 3))
    p0 = rng.normal(size=(n, 3))
    b_t = rng.normal(size=(n, 3))
    sm = ora.System(n, L, 1.0, 0.1, 1.0, 1.0)
    sb = ora.System(n, big, 1.0, 0.1, 1.0, 1.0)
    sig = sm.sigma()[:, None]
    c1 = (1 + sm.a) * sm.dt / 2
    db = rng.normal(size=(n, 3))
    db *= 1.0 / np.linalg.norm(c1 * db / sig)   # |delta| = 1: rejection rate ~0.34
    pots = {}
    for name, s in (("small", sm), ("big", sb)):
        anc = np.zeros((n, 3))
        pots[name] = (ora.Potential.harmonic(0.0, anc, offset=b_t),
                      ora.Potential.harmonic(0.0, anc, offset=b_t + db))
    qs, ps, imgs = q0.copy(), p0.copy(), np.zeros((n, 3), np.int32)
    qb, pb, imgb = q0 + big / 2, p0.copy(), np.zeros((n, 3), np.int32)
    step, reflected, crossed = 0, 0, 0
    for _ in range(40):
        xi = np.stack([ora.normals(7, 0, step + k + 1, n) for k in range(K)])
        u = np.array([ora.uniform(7, 0, step + k + 1) for k in range(K)])
        img_before = imgs.copy()
        rs = ora.lsd_window(sm, *pots["small"], qs, ps, imgs, xi, u)
        rb = ora.lsd_window(sb, *pots["big"], qb, pb, imgb, xi, u)
        assert rs["n_committed"] == rb["n_committed"]
        assert np.array_equal(rs["accept"], rb["accept"])
        assert np.array_equal(ps, pb)
        assert not imgb.any()
        unwrapped = qs + imgs * L - q0
        assert np.max(np.abs(unwrapped - (qb - big / 2 - q0))) < 1e-9
        assert (qs >= 0).all() and (qs < L).all()
        reflected += rs["rejected"]
        if rs["rejected"]:
            crossed += int(np.count_nonzero(imgs != img_before))
        step += rs["n_committed"]
    assert reflected >= 10 and crossed >= 50, (reflected, crossed)

