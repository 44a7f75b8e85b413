"""Pipelined LSD (Alg. 2, App. C): the verifier-state bookkeeping under
out-of-order target returns, on the CPU.

The oracle's pipelined run (a simulated worker pool delivering results in a
random order) is pinned to the synchronous window run, which has its own
pins: with the step-keyed random streams both must commit the same states,
bit for bit.  The library's host bookkeeping (lsd_pipeline_*) replays the
same event sequences and must take the same decisions (ignored returns,
rollbacks, newly verified ids).  On random event sequences without physics
it must satisfy the end-to-end property of the paper: every verified step
was drafted from the step verified just before it."""
import numpy as np
import pytest


def _tether_system(ora, n=6, seed=3):
    rng = np.random.default_rng(seed)
    L = 40.0
    x0 = rng.uniform(5.0, 35.0, size=(n, 3))
    so = ora.System(n, L, 1.0, 0.6, 1.0, 1.0)
    T = ora.Potential.harmonic(2.0, x0)
    D = ora.Potential.harmonic(1.2, x0)
    p0 = rng.normal(size=(n, 3))
    return so, T, D, x0, p0


@pytest.mark.parametrize("workers,seed", [(1, 1), (2, 2), (4, 3), (8, 4)])
def test_pipelined_run_equals_synchronous_run(ora, workers, seed):
    from oracle import pipeline
    from paper_2606_02455_amd import lsd
    so, T, D, x0, p0 = _tether_system(ora)
    n_steps = 40
    q, p = x0.copy(), p0.copy()
    img = np.zeros((so.n, 3), np.int32)
    stats, tq, tp = ora.lsd_run(so, T, D, q, p, img, seed=11, replica=0, step0=0,
                                n_steps=n_steps, K=4, record=True)
    assert stats["rejections"] >= 5
    rng = np.random.default_rng(seed)
    V, events = pipeline.run(so, T, D, x0.copy(), p0.copy(), np.zeros((so.n, 3), np.int32),
                             11, 0, 0, n_steps, workers, rng)
    assert [v[3] for v in V] == list(range(n_steps + 1))
    for k in range(1, n_steps + 1):
        assert np.array_equal(V[k][0], tq[k - 1]) and np.array_equal(V[k][1], tp[k - 1]), k
    returns = [e for e in events if e[0] == "return"]
    if workers > 1:
        ids = [e[1] for e in returns]
        assert any(b < a for a, b in zip(ids, ids[1:]))  # out of order
        assert any(e[3] for e in returns)                # flushed steps came back
    assert any(e[4] for e in returns)                    # rollbacks
    # the library's bookkeeping takes the same decisions on the same events
    pipe = lsd.Pipeline()
    for e in events:
        if e[0] == "submit":
            assert pipe.submit() == e[1]
        else:
            assert pipe.returned(e[1], e[2]) == (e[3], e[4]), e
            assert pipe.take_verified() == e[5], e
    assert pipe.counts()[2] >= n_steps + 1


def test_bookkeeping_verifies_a_drafted_chain():
    # random submissions, returns in random order, random rejections: every
    # verified id was drafted from the id verified before it
    from paper_2606_02455_amd import lsd
    rng = np.random.default_rng(5)
    for trial in range(20):
        pipe = lsd.Pipeline()
        parent = {0: None}
        head = 0                      # the state the next draft starts from
        busy = []
        verified = [0]
        for _ in range(300):
            sid = pipe.submit()
            parent[sid] = head
            head = sid
            busy.append(sid)
            while busy and (len(busy) >= 4 or rng.random() < 0.5):
                k = busy.pop(int(rng.integers(len(busy))))
                ignored, rollback = pipe.returned(k, rng.random() > 0.3)
                if rollback:
                    head = k
                verified += pipe.take_verified()
        ep, cv, nv = pipe.counts()
        assert nv == len(verified) and len(verified) > 10
        assert verified == sorted(verified)
        for a, b in zip(verified, verified[1:]):
            assert parent[b] == a, (trial, a, b)


def test_bookkeeping_rejects_bad_ids():
    from paper_2606_02455_amd import lsd
    pipe = lsd.Pipeline()
    with pytest.raises(lsd.LSDError):
        pipe.returned(1, True)      # never submitted
    i = pipe.submit()
    assert pipe.returned(i, True) == (False, False)
    assert pipe.take_verified() == [i]
    assert pipe.returned(i, True) == (True, False)   # a second return is ignored
