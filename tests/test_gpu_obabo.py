"""GPU checks of the (OBABO) integrator (App. E): LSD runs in the staggered
frame and the (OBABO) states are recovered by the conditional half step.

Checked pathwise against the oracle's staggered LSD run (same random
streams) and against the exact harmonic laws of (OBABO): momenta m kT,
positions kT / (k (1 - w^2 dt^2 / 4)), which the (ABOBA) momentum law fails.
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


def test_obabo_windows_match_oracle_on_tethers(torch, lsd, ora):
    # the initial OB half step, then windows in the staggered frame started
    # on both sides from the same binary32 state: decisions equal outside the
    # log-ratio band, staggered states and the recovered (OBABO) outputs
    # (Eq. obabo_conditional) within bounds propagated from the measured
    # force differences and binary32 rounding
    _say("OBABO windows vs oracle (tethers)")
    R, kT_, kD, n_steps, K = 48, 2.0, 1.2, 40, 4
    w = W.tether_replicas(R, k=kT_, dt=0.6, gamma=1.0, kT=1.0, K=K, L=64.0, seed=43)
    compared, parted, rejections = _parity.run_tether_windows(
        torch, lsd, ora, w, kT_, kD, n_steps, K, obabo=True, say=_say)
    assert compared >= R - 2 and compared + parted == R
    assert rejections > 0


@pytest.mark.parametrize("mode", ["lsd", "plain"])
def test_obabo_states_follow_the_exact_law(torch, lsd, mode):
    _say(f"OBABO harmonic replicas KS ({mode})")
    kT_, m, dt = 2.0, 1.0, 0.6
    w = W.tether_replicas(3000, k=kT_, m=m, dt=dt, gamma=1.0, kT=1.0, K=4, seed=47)
    anchor = w.positions.copy()
    draft = dict(kind="harmonic", k=1.2, anchor=anchor)
    g = lsd.LSDSystem(w, mode=mode, draft=draft if mode == "lsd" else None, skin=50.0,
                      integrator="obabo")
    g.run_to_step(60, 4, check_every=8)
    st = g.state()
    assert (st["step"] == 60).all()
    dq = (st["q"] - anchor).ravel()
    var_q = 1.0 / kT_ / (1.0 - (kT_ / m) * dt * dt / 4.0)
    assert stats.kstest(dq / np.sqrt(var_q), "norm").pvalue > 0.01
    assert stats.kstest(st["p"].ravel() / np.sqrt(m), "norm").pvalue > 0.01
    # the (ABOBA) momentum law is rejected
    bad = m / (1.0 - (kT_ / m) * dt * dt / 4.0)
    assert stats.kstest(st["p"].ravel() / np.sqrt(bad), "norm").pvalue < 1e-3
    g.destroy()
