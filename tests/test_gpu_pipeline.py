"""Pipelined windows on one GPU (Alg. 2): each group of drafted frames is
verified on a second stream while drafting continues, and the drafting of a
window stops at the first rejection its verification has found.  With the
step-keyed stream, frames after the first rejection are never kept, so the
committed trajectory, the step counts and the rejections equal those of
synchronous windows bit for bit; only fewer frames are drafted and verified."""
import numpy as np
import pytest

from paper_2606_02455_amd import workloads as W

pytestmark = pytest.mark.gpu


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


def _say(msg):
    print(msg, flush=True)


def _compare(a, b, tag):
    sa, sb = a.state(), b.state()
    for k in ("q", "p", "img", "step"):
        assert np.array_equal(sa[k], sb[k]), (tag, k)
    ca, cb = a.counters(), b.counters()
    # windows, committed steps, rejections, list builds: identical; frames
    # verified: never more than the synchronous window's
    assert np.array_equal(ca[:, :3], cb[:, :3]), tag
    assert np.array_equal(ca[:, 4], cb[:, 4]), tag
    assert np.all(cb[:, 3] <= ca[:, 3]), tag
    return ca, cb


def _run_pair(lsd, w, group, rounds, windows, K, **kw):
    a = lsd.LSDSystem(w, mode="lsd", **kw)
    b = lsd.LSDSystem(w, mode="lsd", **kw)
    b.set_pipeline(group)
    for rep in range(rounds):
        a.run_windows(windows, K)
        b.run_windows(windows, K)
        ca, cb = _compare(a, b, (group, rep))
    assert a.status() == 0 and b.status() == 0
    a.destroy()
    b.destroy()
    return ca, cb


@pytest.mark.parametrize("case", ["plain_ec_off", "ec_constant", "ec_linear", "obabo"])
@pytest.mark.parametrize("group", [1, 3])
def test_pipelined_windows_equal_synchronous_ones(torch, lsd, case, group):
    _say(f"pipelined G={group} {case}")
    kw = {}
    if case == "ec_constant":
        kw["error_correction"] = 1
    elif case == "ec_linear":
        kw["error_correction"] = 2
    elif case == "obabo":
        kw["integrator"] = "obabo"
    ca, cb = _run_pair(lsd, W.config("c1"), group, 5, 4, 8, **kw)
    assert ca[:, 1].sum() > 20 and ca[:, 2].sum() > 0


def test_pipelined_ragged_replicas_short_skin(torch, lsd):
    _say("pipelined ragged replicas")
    w = W.lj_replicas([3, 4, 5, 6], seed=310, K=8)
    ca, cb = _run_pair(lsd, w, 2, 5, 4, 8, skin=0.1)
    assert ca[:, 4].sum() > 5      # lists rebuilt many times
    assert ca[:, 1].sum() > 0


def test_pipelined_drafting_stops_at_the_first_rejection(torch, lsd):
    # no error correction at C1: acceptance about two thirds, so most
    # windows reject well before K, and the frames after the rejection are
    # neither drafted to completion nor verified
    _say("pipelined: fewer frames verified")
    ca, cb = _run_pair(lsd, W.config("c1"), 1, 4, 10, 8)
    assert cb[:, 3].sum() < ca[:, 3].sum()
    # every kept frame is verified: at least the committed steps
    assert cb[:, 3].sum() >= cb[:, 1].sum()


def test_timed_pipelined_windows_equal_untimed(torch, lsd):
    _say("pipelined: timed vs untimed")
    w = W.config("c1")
    a = lsd.LSDSystem(w, mode="lsd", error_correction=1)
    b = lsd.LSDSystem(w, mode="lsd", error_correction=1)
    a.set_pipeline(2)
    b.set_pipeline(2)
    b.set_verify_timing(True, every=3)
    for rep in range(4):
        a.run_windows(6, 8)
        b.run_windows(6, 8)
        sa, sb = a.state(), b.state()
        for k in ("q", "p", "img", "step"):
            assert np.array_equal(sa[k], sb[k]), (rep, k)
        assert np.array_equal(a.counters(), b.counters())
    ms, n = b.verify_timing()
    # every third window is timed, four verification groups of two frames each
    assert n == 8 * 4 and ms > 0
    a.destroy()
    b.destroy()


def test_pipelined_network_target_with_learned_draft(torch, lsd):
    # message-passing target (forces scaled to about 0.1 eV/A RMS, so that
    # about half the steps are accepted) and a learned draft with nearly
    # zero output, ragged replicas in small boxes: the batched network
    # evaluation of each group gives the same forces as that of the whole
    # window, bit for bit
    _say("pipelined: network target, learned draft")
    w = W.triatomic_replicas(n_replicas=3, n_mol_lo=8, n_mol_hi=16, seed=41, K=8)
    target = dict(kind="mpnn", rc=5.0, weights=W.mpnn_weights(3, seed=17), n_model_species=3,
                  scale=0.1 * W.MPNN_C3_SCALE)
    P = lsd.net_param_count(3, 8)
    p = torch.zeros(P, dtype=torch.float32, device="cuda")
    draft = dict(kind="net", rc=4.0, weights=p, n_basis=8, n_model_species=3)
    for kw in ({}, {"error_correction": 2}):
        ca, cb = _run_pair(lsd, w, 2, 3, 4, 8, target=target, draft=draft, **kw)
        assert ca[:, 1].sum() > ca[:, 0].sum()      # some windows keep several steps
        assert ca[:, 2].sum() > 0
