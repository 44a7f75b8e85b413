"""Pipelined LSD (Alg. 2, App. C) with a simulated pool of target workers.

Test infrastructure only, like the rest of this package.  The main loop
drafts a step from the current draft state, submits it to a worker, and then
handles whichever worker results have arrived, in whatever order.  The
verifier state is the three buffers of the paper: eligible pending (EP),
conditionally verified (CV) and verified (V), keyed by the step id.

The pool is simulated on the CPU: a submitted step's target result is
computed at once by the oracle's single-step LSD map (draft_step followed by
verify_step of Alg. 2, here a window of one frame), but the result is
delivered later, in a random order chosen by `rng`: after every submission
a random subset of the busy workers finishes, and when all workers are busy
the main loop waits until a random one has finished; finished results are
handled at the next gathering, in the order they finished.  Noise and
uniforms are keyed by the simulation step a state is drafted to, so a
redraft after a rollback reuses the keys of the flushed steps, as in the
synchronous window.
"""
import numpy as np

from . import lsd_window, normals, uniform


def _draft_state(system, out, img_in):
    """The draft state y' of a one-frame window: the second position half
    step from the midpoint with the drafted momentum, wrapped (used only to
    keep drafting past a step that will turn out rejected)."""
    L = system.L
    m = np.asarray(system.masses, dtype=np.float64).reshape(-1, 1)
    q = out["q_mid"][0] + 0.5 * system.dt / m * out["p_draft"][1]
    shift = np.floor(q / L)
    return q - shift * L, out["p_draft"][1].copy(), img_in + shift.astype(np.int32)


def run(system, target, draft, q0, p0, img0, seed, replica, step0, n_steps, workers, rng,
        p_return=0.5):
    """Alg. 2 until n_steps steps are verified.  Returns (V, events): V is
    the verified sequence [(q, p, img, step)] starting with the initial
    state; events lists ('submit', id) and ('return', id, accepted,
    ignored, rollback, newly verified ids) in the order they happened."""
    n = system.n
    y = (q0.copy(), p0.copy(), img0.copy())
    ny = step0
    EP, CV = {}, {}
    V = [(q0.copy(), p0.copy(), img0.copy(), step0)]
    events = []
    next_id = 1

    def process(returns):
        nonlocal y, ny, EP, CV
        for (sid, x, acc, step) in returns:
            if sid not in EP:
                events.append(("return", sid, acc, True, False, []))
                continue
            del EP[sid]
            CV[sid] = (x, step)
            rollback = False
            if not acc:
                EP = {k: v for k, v in EP.items() if k <= sid}
                CV = {k: v for k, v in CV.items() if k <= sid}
                y = tuple(a.copy() for a in x)
                ny = step
                rollback = True
            fresh = []
            while CV and min(CV) < min(list(EP) + [np.inf]):
                k = min(CV)
                xs, st = CV.pop(k)
                V.append((xs[0].copy(), xs[1].copy(), xs[2].copy(), st))
                fresh.append(k)
            events.append(("return", sid, acc, False, rollback, fresh))

    busy = []      # workers still computing: (id, x', accepted, step)
    arrived = []   # finished results not yet gathered, in arrival order
    while len(V) < n_steps + 1:
        # draft_step from y; the worker's verify_step is computed now and
        # delivered later
        q, p, img = (a.copy() for a in y)
        xi = normals(seed, replica, ny + 1, n).reshape(1, n, 3)
        u = np.array([uniform(seed, replica, ny + 1)])
        out = lsd_window(system, target, draft, q, p, img, xi, u)
        acc = bool(out["accept"][0])
        x = (q, p, img)
        y_new = x if acc else _draft_state(system, out, y[2])
        # fetch_idle_worker: wait until some worker has finished
        while len(busy) >= workers:
            arrived.append(busy.pop(int(rng.integers(len(busy)))))
        sid = next_id
        next_id += 1
        busy.append((sid, tuple(a.copy() for a in x), acc, ny + 1))
        EP[sid] = True
        events.append(("submit", sid))
        y = tuple(a.copy() for a in y_new)
        ny += 1
        # meanwhile a random subset of the busy workers finishes
        done = [i for i in range(len(busy)) if rng.random() < p_return]
        rng.shuffle(done)
        arrived += [busy[i] for i in done]
        for i in sorted(done, reverse=True):
            busy.pop(i)
        # gather_new_returns and process them in arrival order
        process(arrived)
        arrived = []
    return V[:n_steps + 1], events
