"""GPU checks of speculative error correction (App. D, Alg. 3).

The draft of every frame is drawn with F~ + dF, dF being the target minus
EC-uncorrected draft force of the last committed step; target forces and the
acceptance rule are untouched, so the committed states keep the target law.
Checked against the oracle's EC runs, an exact cancellation case and exact
stationary laws.
"""
import sys

import numpy as np
import pytest
from scipy import stats

from paper_2606_02455_amd import workloads as W

import _parity

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


@pytest.mark.parametrize("mode", [1, 2])
def test_ec_windows_match_oracle_on_tethers(torch, lsd, ora, mode):
    # draft stiffness differs from the target's, so the force error changes
    # from step to step and the cache really moves.  Every window starts on
    # both sides from the same binary32 state and caches; decisions must be
    # equal outside the log-ratio band, log ratios, committed states and the
    # refreshed caches within bounds propagated from the measured force
    # differences and binary32 rounding.  mode 2: linear extrapolation of the
    # error from the last two committed steps
    _say(f"EC windows vs oracle (tethers), mode {mode}")
    R, kT_, kD, n_steps, K = 48, 2.0, 1.0, 40, 4
    w = W.tether_replicas(R, k=kT_, dt=0.2, gamma=2.0, kT=1.0, K=K, L=64.0, seed=41)
    compared, parted, rejections = _parity.run_tether_windows(
        torch, lsd, ora, w, kT_, kD, n_steps, K, ec_mode=mode, say=_say)
    assert compared >= R - 2 and compared + parted == R
    assert rejections > 0


def test_ec_cancels_a_constant_draft_error(torch, lsd):
    _say("EC constant offset (C1)")
    w = W.config("c1")
    rng = np.random.default_rng(9)
    b = rng.normal(size=(w.n_atoms, 3))
    sig = np.sqrt(1.0 * w.kT * (1 - np.exp(-2 * w.gamma * w.dt)))
    c1 = (1 + np.exp(-w.gamma * w.dt)) * w.dt / 2
    b = W.f32(b * 2.0 / np.linalg.norm(c1 * b / sig))   # |delta| = 2: erf(2/sqrt 8) = 0.68
    draft = dict(w.target)
    draft["offset"] = b
    g = lsd.LSDSystem(w, mode="lsd", draft=draft, error_correction=True)
    g.run_windows(200, w.K)
    cn = g.counters()[0]
    ec = g.window()["error_cache"].cpu().numpy().T
    # once a step is committed the cache is F - fl(F + b) = -b up to rounding
    assert int(cn[2]) <= 1, cn
    assert np.max(np.abs(ec + b)) <= 1e-5 * (1 + np.max(np.abs(b))), np.max(np.abs(ec + b))
    assert g.status() == 0
    g.destroy()
    # without correction the same draft is rejected at the closed-form rate
    g = lsd.LSDSystem(w, mode="lsd", draft=draft)
    g.run_windows(100, w.K)
    cn = g.counters()[0]
    assert cn[2] / cn[1] > 0.4
    assert g.window()["error_cache"] is None
    g.destroy()


@pytest.mark.parametrize("mode", [1, 2])
def test_ec_keeps_exact_target_law(torch, lsd, mode):
    _say(f"EC harmonic replicas KS, mode {mode}")
    kT_, kD = 2.0, 1.0
    w = W.tether_replicas(3000, k=kT_, dt=0.2, gamma=2.0, kT=1.0, K=4, seed=37)
    anchor = w.positions.copy()
    draft = dict(kind="harmonic", k=kD, anchor=anchor)
    g = lsd.LSDSystem(w, mode="lsd", draft=draft, error_correction=mode)
    g.run_to_step(60, 4, check_every=8)
    st = g.state()
    assert (st["step"] == 60).all()
    dq = (st["q"] - anchor).ravel()
    var_p = 1.0 / (1.0 - kT_ * 0.2 ** 2 / 4.0)
    assert stats.kstest(dq / np.sqrt(1.0 / kT_), "norm").pvalue > 0.01
    assert stats.kstest(st["p"].ravel() / np.sqrt(var_p), "norm").pvalue > 0.01
    g.destroy()
