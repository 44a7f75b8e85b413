#!/usr/bin/env python3
"""Benchmark: target-distributed MD steps/s of LSD vs plain target Langevin
on one MI355X, with the verification kernel's roofline and the FP64 oracle
timed on the host as the CPU baseline.

A timed "step" is one LSD window over the whole hot path: draft K steps
(cell + neighbour lists, K draft kernels), verify all K frames in one launch,
decide, reflect and commit.  ``value`` is committed target-distributed steps
per second.  Plain Langevin runs the same kernels with the target force
field and commits every step; it is timed over the same number of windows.

Usage: python bench.py [--gpus 1] [--steps 200] [--warmup 20] [--config c2]
Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
EC_MODES = {"off": 0, "on": 1, "linear": 2}
COPY_BYTES = 256 << 20  # calibration copy: 256 MiB read + 256 MiB written
ACCEPT_SAMPLE_WINDOWS = 400  # default untimed windows behind the reported acceptance (c1, c2)
# binary32 vector peak without packed instructions: 256 CUs x 2.4 GHz x 64
# lanes x 2 (a fused multiply-add counts two)
VALU_PEAK_TFLOPS = 256 * 2.4e9 * 64 * 2 / 1e12
LJ_PAIR_FLOPS = 31  # per directed in-cutoff pair and frame (separation, r^2, r^-6 terms, force, energy)
VERIFY_SOURCES = ["paper_2606_02455_amd/csrc/lsd_kernels.hip",
                  "paper_2606_02455_amd/csrc/lsd_device.h"]
# sources of the network-target verification (evaluation kernels and the
# transport reduction)
MPNN_SOURCES = VERIFY_SOURCES + ["paper_2606_02455_amd/csrc/mpnn.hip",
                                 "paper_2606_02455_amd/csrc/mpnn.h"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_sha(sources=VERIFY_SOURCES):
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(config_name, kernel, skin):
    """HBM bytes per verification launch from the committed rocprofv3
    counter summary, if it was taken on the current kernel source, with the
    same list skin, and holds a section for this kernel variant."""
    path = os.path.join(ROOT, "profiles", f"k_verify_{config_name}_traffic.txt")
    if not os.path.exists(path):
        return None
    head, sections, cur = {}, {}, None
    for line in open(path):
        line = line.strip()
        if line.startswith("[") and line.endswith("]"):
            cur = sections.setdefault(line[1:-1], {})
        elif "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            (cur if cur is not None else head)[k.strip()] = v.strip()
    if head.get("source_sha") != source_sha() or head.get("lsd_skin") != repr(float(skin)):
        return None
    try:
        return float(sections[kernel]["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def read_profile_avg_us(config_name, kernel, skin):
    """Average duration of the kernel in the committed rocprofv3 kernel trace
    of this configuration, if that trace was taken on the current kernel
    source and list skin."""
    path = os.path.join(ROOT, "profiles", f"k_verify_{config_name}_kernel_trace.txt")
    if not os.path.exists(path):
        return None
    head, avg = {}, None
    for line in open(path):
        t = line.strip()
        if t.startswith("#") and "=" in t:
            k, v = t[1:].split("=", 1)
            head[k.strip()] = v.strip()
        elif (t.startswith(kernel + " ") or t.startswith(f"void {kernel} ")
              or t.startswith(f"void {kernel}(")):
            parts = t.replace("void ", "", 1).replace(kernel, "", 1).split()
            try:
                avg = float(parts[1])
            except (IndexError, ValueError):
                pass
    if head.get("source_sha") != source_sha() or head.get("lsd_skin") != repr(float(skin)):
        return None
    return avg


def read_profile_keys(name, sources, skin):
    """Key = value lines (commented or not) of a committed rocprofv3 summary
    under profiles/, if it was taken on the current source of the kernels it
    covers and with the same list skin; else None."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    keys = {}
    for line in open(path):
        t = line.strip().lstrip("#").strip()
        if "=" in t and not t.startswith("cd "):
            k, v = t.split("=", 1)
            if " " not in k.strip():
                keys[k.strip()] = v.strip()
    if keys.get("source_sha") != source_sha(sources) or keys.get("lsd_skin") != repr(float(skin)):
        return None
    return keys


def in_cutoff_pairs(sysg, rc):
    """Directed pairs within rc at the current list positions (frame 0),
    counted on the GPU from the neighbour list."""
    import torch
    cnt, ent = sysg.neighbor_lists("target")
    win = sysg.window()
    x = win["q_mid"][0, :, :3].double()
    import numpy as np
    per_atom = np.repeat(np.asarray(sysg.w.box, np.float64), np.diff(sysg.w.atom_offsets))
    L = torch.tensor(per_atom, dtype=torch.float64, device=x.device)[:, None, None]
    m = ent.shape[1]
    ar = torch.arange(m, device=ent.device)[None, :]
    valid = ar < cnt[:, None].to(ar.dtype)
    e = ent.long() & 0xFFFFFFFF
    j = (e >> 5).clamp(max=sysg.N - 1)
    code = e & 31
    n = torch.stack([code % 3 - 1, (code // 3) % 3 - 1, code // 9 - 1], dim=-1).double()
    d = x[j] + n * L - x[:, None, :]
    r2 = (d * d).sum(-1)
    return int(((r2 < rc * rc) & valid).sum().item())


def cpu_baseline(w, q, p, seconds, ec_mode):
    """The FP64 oracle as it stands: LSD windows of K frames from the
    benchmark's equilibrated state until `seconds` of host time are spent
    (with the same error-correction setting as the GPU run)."""
    import numpy as np

    import oracle
    so = oracle.System(w.n_atoms, float(w.box[0]), 1.0, w.dt, w.gamma, w.kT)
    T = oracle.Potential.lj(w.target["rc"])
    D = oracle.Potential.lj(w.draft["rc"])
    q, p = q.copy(), p.copy()
    img = np.zeros(q.shape, np.int32)
    ec = np.zeros(q.shape) if ec_mode >= 1 else None
    ec_prev = np.zeros(q.shape) if ec_mode == 2 else None
    samples = np.zeros(1, np.int32)
    K, N = w.K, w.n_atoms
    committed = windows = 0
    step = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        xi = np.stack([oracle.normals(w.seed, 0, step + k + 1, N) for k in range(K)])
        u = np.array([oracle.uniform(w.seed, 0, step + k + 1) for k in range(K)])
        r = oracle.lsd_window(so, T, D, q, p, img, xi, u, ec=ec, ec_prev=ec_prev, samples=samples)
        committed += r["n_committed"]
        step += r["n_committed"]
        windows += 1
    t_lsd = time.perf_counter() - t0
    # plain target Langevin on the host for comparison
    t1 = time.perf_counter()
    n_plain = 0
    while time.perf_counter() - t1 < max(2.0, seconds / 4):
        oracle.plain_run(so, T, q, p, img, w.seed, 0, step + n_plain, 4)
        n_plain += 4
    t_plain = time.perf_counter() - t1
    return dict(value=committed / t_lsd, unit="steps/s", cores=oracle.num_threads(), kind="oracle",
                sample=(f"{windows} LSD windows (K={K}) of the {N}-atom fluid from the "
                        f"benchmark state, {committed} committed steps in {t_lsd:.1f} s"),
                plain_steps_per_s=n_plain / t_plain)


def cpu_baseline_mpnn(w, state, target, draft, ec_mode, seconds):
    """The FP64 oracle as it stands on a network-target configuration: LSD
    windows of K frames (message-passing target, the same draft with the
    same parameters, the same error-correction setting) from the benchmark's
    state, replica after replica, until `seconds` of host time are spent (at
    least one window); then plain target steps for a quarter of that."""
    import numpy as np

    import oracle
    from oracle.mpnn import MPNN
    from oracle.net import NetDraft
    from oracle.pair import PairDraft
    net = MPNN(np.asarray(target["weights"], np.float64), 3, rc=target["rc"],
               scale=target["scale"])
    if draft["kind"] == "net":
        dparams = draft["weights"].detach().cpu().numpy().astype(np.float64)
        dmodel = NetDraft(3, draft["n_basis"], draft["rc"], dparams)
    else:
        dmodel = PairDraft(3, draft["n_basis"], draft["rc"], w=np.asarray(draft["weights"]))
    K = w.K
    off = np.asarray(w.atom_offsets)
    q_all = np.asarray(state["q"], np.float64).reshape(-1, 3)
    p_all = np.asarray(state["p"], np.float64).reshape(-1, 3)
    steps = np.asarray(state["step"]).reshape(-1)
    reps = []
    for r in range(w.n_replicas):
        a, b = int(off[r]), int(off[r + 1])
        sp = w.species[a:b]
        so = oracle.System(b - a, float(w.box[r]), w.masses()[a:b], w.dt, w.gamma, w.kT,
                           w.force_unit)
        T = oracle.Potential.mpnn(net, sp)
        D = (oracle.Potential.net_draft(dmodel, sp) if draft["kind"] == "net"
             else oracle.Potential.pair_draft(dmodel, sp))
        n = b - a
        reps.append(dict(so=so, T=T, D=D, q=q_all[a:b].copy(), p=p_all[a:b].copy(),
                         img=np.zeros((n, 3), np.int32), step=int(steps[r]),
                         ec=np.zeros((n, 3)) if ec_mode >= 1 else None,
                         ec_prev=np.zeros((n, 3)) if ec_mode == 2 else None,
                         samples=np.zeros(1, np.int32), n=n))
    committed = windows = 0
    t0 = time.perf_counter()
    r = 0
    while windows == 0 or time.perf_counter() - t0 < seconds:
        R = reps[r % len(reps)]
        xi = np.stack([oracle.normals(w.seed, r % len(reps), R["step"] + k + 1, R["n"])
                       for k in range(K)])
        u = np.array([oracle.uniform(w.seed, r % len(reps), R["step"] + k + 1) for k in range(K)])
        res = oracle.lsd_window(R["so"], R["T"], R["D"], R["q"], R["p"], R["img"], xi, u,
                                ec=R["ec"], ec_prev=R["ec_prev"], samples=R["samples"])
        committed += res["n_committed"]
        R["step"] += res["n_committed"]
        windows += 1
        r += 1
    t_lsd = time.perf_counter() - t0
    t1 = time.perf_counter()
    n_plain = 0
    r = 0
    while n_plain == 0 or time.perf_counter() - t1 < max(2.0, seconds / 4):
        R = reps[r % len(reps)]
        oracle.plain_run(R["so"], R["T"], R["q"], R["p"], R["img"], w.seed, r % len(reps),
                         R["step"] + n_plain, 1)
        n_plain += 1
        r += 1
    t_plain = time.perf_counter() - t1
    return dict(value=committed / t_lsd, unit="steps/s", cores=oracle.num_threads(), kind="oracle",
                sample=(f"{windows} LSD windows (K={K}) over {min(windows, len(reps))} of "
                        f"{len(reps)} system(s) of the {w.n_atoms}-atom liquid from the benchmark "
                        f"state (FP64 message-passing target, {draft['kind']} draft), "
                        f"{committed} committed steps in {t_lsd:.1f} s"),
                plain_steps_per_s=n_plain / t_plain)


def mpnn_flops_per_frame(undirected_edges, n_atoms, H=128, R=16, T=3, RH=64):
    """Algorithmic FLOPs of one target evaluation (energy and forces) of the
    message-passing network: per undirected in-cutoff edge and layer the
    filter MLP (R -> H -> H) forward and its input-gradient backward; per atom
    and layer the node MLPs (B, C1, C2: H x H) forward and backward; the
    readout.  Multiply-add = 2 FLOPs; elementwise work is not counted."""
    per_edge = T * 2 * (2 * (R * H + H * H))
    per_atom = T * 2 * (3 * 2 * H * H) + 2 * 2 * (RH * H)
    return undirected_edges * per_edge + n_atoms * per_atom


def run_c3(args, lsd, W, torch):
    """Network-target configurations: triatomic liquid (c3: 1536 atoms, K = 8;
    c4: 256 replicas of 24-192 atoms in one system, K = 8; c5: 24 576 atoms,
    K = 32), message-passing target, pair draft fitted by force matching on
    target frames and the learned draft trained from it."""
    import numpy as np
    w = W.config(args.config)
    K, N = w.K, w.n_atoms
    nb, rc_d = args.pair_basis, float(w.draft["rc"])
    target = W.mpnn_target()
    ec_on = args.ec != "off"
    log(f"workload {w.name}: N={N} K={K} box={w.box[0]:.4f} A")
    lsd_skin, plain_skin = W.BENCH_SKINS.get(args.config, (w.skin, w.skin))
    if args.skin is not None:
        lsd_skin = args.skin
    if args.plain_skin is not None:
        plain_skin = args.plain_skin
    log(f"list skins: LSD {lsd_skin}, plain {plain_skin}")
    plain = lsd.LSDSystem(w, mode="plain", target=target, skin=plain_skin)
    eq_windows = max(1, args.equilibrate // K)
    t0 = time.perf_counter()
    plain.run_windows(eq_windows, K)
    torch.cuda.synchronize()
    log(f"equilibrated {eq_windows * K} plain steps in {time.perf_counter() - t0:.1f} s")
    # the drafts are trained on target frames of this system, or of the
    # 1536-atom liquid of the same recipe (a local model transfers)
    trainer, wt = plain, w
    if args.draft_source != args.config:
        wt = W.config(args.draft_source)
        tskin = W.BENCH_SKINS.get(args.draft_source, (wt.skin, wt.skin))[1]
        trainer = lsd.LSDSystem(wt, mode="plain", target=target, skin=tskin)
        trainer.run_windows(max(1, args.equilibrate // wt.K), wt.K)
        torch.cuda.synchronize()
        log(f"drafts trained on {wt.name} ({wt.n_atoms} atoms)")
    Kt = wt.K
    # force matching on frames of the plain target trajectory
    P = lsd.pair_params(3, nb)
    gram = torch.zeros((P + 1, P + 1), dtype=torch.float64, device="cuda")
    scratch = None
    fit_windows = max(1, (args.fit_frames + Kt - 1) // Kt)
    committed0 = int(trainer.counters()[:, 1].sum())
    t0 = time.perf_counter()
    for _ in range(fit_windows):
        trainer.draft_steps(Kt)
        # differences of consecutive frames: the draft's response to the
        # motion, which the error correction does not remove
        scratch = trainer.fit_pair_accumulate(nb, rc_d, gram, scratch=scratch, differences=True)
        trainer.accept_rollback()
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t0
    # frames actually stepped (a window ends early once an atom leaves the
    # skin), as whole-system frames
    fit_frames = (int(trainer.counters()[:, 1].sum()) - committed0) // wt.n_replicas
    G = gram.cpu().numpy()
    wts = lsd.fit_pair_solve(G, ridge=1e-8)
    log(f"fitted the pair draft on {fit_frames} target frames in {t_fit:.1f} s")
    if trainer.status():
        raise RuntimeError(f"device status {trainer.status()} during plain stepping")
    draft = dict(kind="pair", rc=rc_d, weights=wts, n_basis=nb, n_model_species=3)
    train = None
    if args.draft == "net":
        # the learned draft: starts as the fitted pair draft (edge weights 0)
        # and is trained with Adam on the force changes between consecutive
        # frames of the plain target trajectory, one step per window
        Pn = lsd.net_param_count(3, nb)
        pt = torch.tensor(lsd.net_init_params(3, nb, pair_weights=wts, seed=w.seed),
                          dtype=torch.float32, device="cuda")
        net = dict(kind="net", rc=rc_d, weights=pt, n_basis=nb, n_model_species=3,
                   precision=args.net_precision)
        grad = torch.zeros(Pn + 2, dtype=torch.float64, device="cuda")
        m1 = torch.zeros(Pn, dtype=torch.float64, device="cuda")
        m2 = torch.zeros(Pn, dtype=torch.float64, device="cuda")
        scratch_t, mse = None, []
        committed0 = int(trainer.counters()[:, 1].sum())
        t0 = time.perf_counter()
        n_train = args.net_train_windows
        for step in range(1, n_train + 1):
            trainer.draft_steps(Kt)
            scratch_t = trainer.net_train_accumulate(net, grad, scratch=scratch_t, differences=True)
            trainer.accept_rollback()
            if step == 1 or step == n_train:
                torch.cuda.synchronize()
                mse.append(grad[Pn].item() / (3.0 * max(grad[Pn + 1].item(), 1.0)))
            lr = args.net_lr * 0.5 * (1.0 + math.cos(math.pi * step / n_train))
            lsd.net_adam_step(torch, pt, m1, m2, grad, lr, step)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        train_frames = (int(trainer.counters()[:, 1].sum()) - committed0) // wt.n_replicas
        log(f"trained the learned draft ({Pn} parameters) on {train_frames} target frames in "
            f"{t_train:.1f} s; force-change MSE {mse[0]:.3g} -> {mse[-1]:.3g} (eV/A)^2")
        train = dict(windows=n_train, frames=train_frames, seconds=round(t_train, 2),
                     mse_first=mse[0], mse_last=mse[-1], parameters=Pn, system=wt.name)
        if args.net_precision == "fp8" or args.compare_precision:
            # static per-tensor activation scales: the largest |D| and |h| over
            # 16 windows of target frames of the measured system, with a 20%
            # margin
            amax = np.zeros(2)
            for _ in range(16):
                plain.draft_steps(K)
                amax = np.maximum(amax, plain.net_activation_amax(net))
                plain.accept_rollback()
            net["act_amax"] = tuple(1.2 * amax)
            train["fp8_act_amax"] = [float(a) for a in net["act_amax"]]
            log(f"FP8 activation scales from max |D| = {amax[0]:.4g}, max |h| = {amax[1]:.4g}")
        draft = net
    start = [t.clone() for t in (plain.q, plain.p, plain.img, plain.step)]

    def lsd_run(dr):
        """Autotuned, warmed-up LSD windows from the benchmark state; the
        timed windows with their verification timed by HIP events."""
        g = lsd.LSDSystem(w, mode="lsd", target=target, draft=dr,
                          error_correction=EC_MODES[args.ec], skin=lsd_skin)
        for a, b in zip((g.q, g.p, g.img, g.step), start):
            a.copy_(b)
        shape, shape_us = g.autotune_verify(K, repeats=3)
        g.verify_window()
        g.accept_rollback()
        if args.draft_tail is not None:
            g.set_draft_tail(args.draft_tail)
        if args.pipeline:
            g.set_pipeline(args.pipeline)
        # the warmup runs with the timed windows' graphs already in use, so
        # the timed region starts on warm graphs; the sums restart after it
        g.set_verify_timing(True)
        g.run_windows(args.warmup, K)
        g.reset_counters()
        g.set_verify_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.run_windows(args.steps, K)
        torch.cuda.synchronize()
        return g, time.perf_counter() - t0, shape, shape_us

    g, t_lsd, shape, shape_us = lsd_run(draft)
    ver_ms, ver_n = g.verify_timing()
    cn = g.counters()
    windows = int(cn[0, 0])
    committed, rejections, frames = (int(cn[:, c].sum()) for c in (1, 2, 3))
    log(f"LSD: {committed} steps in {t_lsd * 1e3:.1f} ms over {windows} windows; rejections "
        f"{rejections}; verify {ver_ms / max(ver_n, 1) * 1e3:.1f} us/launch; launch shape "
        f"{lsd.LSDSystem.NET_SHAPES[shape]}")
    other = None
    if args.compare_precision and args.draft == "net":
        prec = "bf16" if args.net_precision == "fp8" else "fp8"
        g2, t2, _, _ = lsd_run(dict(draft, precision=prec))
        c2 = g2.counters()
        n2, r2 = int(c2[:, 1].sum()), int(c2[:, 2].sum())
        other = dict(precision=prec, steps_per_s=round(n2 / t2, 3),
                     acceptance=round(1.0 - r2 / max(n2, 1), 5),
                     committed_per_window=round(n2 / max(int(c2[0, 0]), 1), 4))
        log(f"LSD with the {prec} node pass: {n2} steps in {t2 * 1e3:.1f} ms, rejections {r2}")
        g2.destroy()
    plain.run_windows(args.warmup, K)
    plain.reset_counters()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain.run_windows(args.steps, K)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    plain_steps = int(plain.counters()[:, 1].sum())
    log(f"plain: {plain_steps} steps in {t_plain * 1e3:.1f} ms")
    status = g.status() | plain.status()
    if status:
        raise RuntimeError(f"device status {status}: neighbour capacity overflow")
    # a plain copy of known size: the reference that scales the FETCH_SIZE /
    # WRITE_SIZE counters of rocprofv3 (profiles/)
    src = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    pairs = in_cutoff_pairs(g, float(target["rc"]))
    # replica-frames per launch (one launch per window), as whole-system
    # frames
    frames_per_launch = frames / max(windows, 1) / w.n_replicas
    flops = mpnn_flops_per_frame(pairs / 2.0, N) * frames_per_launch
    avg_s = ver_ms / max(ver_n, 1) * 1e-3
    achieved = flops / avg_s / 1e12
    peak = 157.3
    # the committed rocprofv3 summaries of this configuration: kernel time of
    # the evaluation per window, its matrix-core counters and HBM traffic
    trace = read_profile_keys(f"mpnn_{args.config}_kernel_trace.txt", MPNN_SOURCES, lsd_skin) or {}
    traffic = read_profile_keys(f"mpnn_{args.config}_traffic.txt", MPNN_SOURCES, lsd_skin) or {}
    prof_us = float(trace["verify_kernel_us_per_window"]) if "verify_kernel_us_per_window" in trace else None
    # the profiled run verifies its own number of frames per window: its
    # kernel time is compared per frame
    prof_frames = float(trace["frames_per_window"]) if "frames_per_window" in trace else None
    value, plain_rate = committed / t_lsd, plain_steps / t_plain
    dt_fs = w.dt
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host ...")
        cpu = cpu_baseline_mpnn(w, g.state(), target, draft, EC_MODES[args.ec], args.cpu_seconds)
        log(f"oracle: {cpu['value']:.4f} LSD steps/s, {cpu['plain_steps_per_s']:.4f} plain "
            f"steps/s on {cpu['cores']} threads")
    return {
        "metric": "target-distributed MD steps/s (LSD vs plain Langevin, 1 GPU); acceptance rate",
        "value": round(value, 3), "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(t_lsd / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"{w.name}: triatomic liquid, {N} atoms in {w.n_replicas} system(s), 300 K, "
                         f"dt {dt_fs} fs, gamma {w.gamma}/fs, K={K}; target: seeded "
                         f"message-passing network (3 layers, hidden 128, 16 Bessel, rc 5 A); "
                         + (f"draft: learned one-layer direct-force network (hidden 32, rc {rc_d} A, "
                            f"{nb} radial functions, {args.net_precision} node pass) initialised "
                            f"from the pair draft and trained on {train['frames'] if train else 0} "
                            f"target frames of {wt.name}; " if args.draft == "net" else "")
                         + f"pair draft: pair forces (rc {rc_d} A, {nb} basis) force-matched "
                         f"(frame-to-frame differences) on {fit_frames} target frames of "
                         f"{wt.name}; error correction {args.ec}"),
            "n_atoms": N, "K": K, "fit_frames": fit_frames,
            "draft": args.draft, "error_correction": args.ec,
            "skin": lsd_skin, "plain_skin": plain_skin},
        "acceptance": round(1.0 - rejections / max(committed, 1), 5),
        "committed_per_window": round(committed / windows, 4),
        "plain_steps_per_s": round(plain_rate, 3),
        "lsd_over_plain": round(value / plain_rate, 5),
        "ns_per_day_lsd": round(value * dt_fs * 1e-6 * 86400.0, 4),
        "ns_per_day_plain": round(plain_rate * dt_fs * 1e-6 * 86400.0, 4),
        "fit_seconds": round(t_fit, 2),
        "draft_training": train,
        "net_precision": args.net_precision if args.draft == "net" else None,
        "other_precision": other,
        "roofline": dict(bound="mfma", achieved=round(achieved, 3), peak=peak, unit="TFLOP/s",
                         frac=round(achieved / peak, 5),
                         traffic=(float(traffic["hbm_bytes_per_window"])
                                  if "hbm_bytes_per_window" in traffic else None),
                         traffic_frames_per_window=(float(traffic["frames_per_window"])
                                                    if "frames_per_window" in traffic else None),
                         kernel="message-passing target evaluation (all frames of a window)",
                         timing=("HIP events around each window's verification on its stream: "
                                 "the evaluation kernels and the transport reduction with the "
                                 "gaps between their launches"),
                         profile_avg_us=prof_us,
                         profile_frames_per_window=prof_frames,
                         frac_at_profile_us=(round(flops / frames_per_launch * prof_frames
                                                   / (prof_us * 1e-6) / 1e12 / peak, 5)
                                             if prof_us and prof_frames and frames_per_launch
                                             else None),
                         launch_shape=dict(zip(("filter_blocks", "chain_rows"),
                                               lsd.LSDSystem.NET_SHAPES[shape])),
                         autotune_us={f"{a}x{b}": round(v, 1) for (a, b), v in shape_us.items()},
                         avg_us=round(avg_s * 1e6, 2), algorithmic_flops=int(flops),
                         frames_per_launch=round(frames_per_launch, 3),
                         in_cutoff_pairs=pairs),
        "cpu_baseline": cpu,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="timed windows")
    ap.add_argument("--warmup", type=int, default=20, help="untimed windows")
    ap.add_argument("--config", default="c2", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--fit-frames", type=int, default=None,
                    help="c3/c4: target frames for force matching of the pair draft "
                         "(default 20000 for c3, 2000 whole-system frames of 256 replicas for c4)")
    ap.add_argument("--pair-basis", type=int, default=16,
                    help="c3/c4: radial functions of the pair and learned drafts")
    ap.add_argument("--draft", choices=["net", "pair"], default="net",
                    help="c3/c4: the learned draft (trained from the pair draft) or the pair draft")
    ap.add_argument("--net-precision", choices=["bf16", "fp32", "fp8"], default=None,
                    help="node pass of the learned draft (default: fp8 for c5, else bf16)")
    ap.add_argument("--net-train-windows", type=int, default=None,
                    help="c3/c4: Adam steps, one window of K target frames each "
                         "(default 2000 for c3, 500 for c4)")
    ap.add_argument("--net-lr", type=float, default=3e-3)
    ap.add_argument("--draft-source", choices=["c3", "c4", "c5"], default=None,
                    help="c3/c4/c5: system whose target frames train the drafts (default: the "
                         "measured system; drafts trained on c3 frames meet pair distances on c5 that "
                         "their fit never saw)")
    ap.add_argument("--compare-precision", action="store_true",
                    help="c3/c4/c5: also time LSD with the other node-pass precision of the "
                         "learned draft (bf16 vs fp8) and report both acceptances")
    ap.add_argument("--equilibrate", type=int, default=256, help="plain steps before timing")
    ap.add_argument("--skin", type=float, default=None,
                    help="list skin of the LSD run (default: the tuned one of the config)")
    ap.add_argument("--plain-skin", type=float, default=None,
                    help="list skin of the plain run (default: the tuned one of the config)")
    ap.add_argument("--time-every", type=int, default=8,
                    help="time every n-th verification launch with HIP events (c1, c2)")
    ap.add_argument("--verify-fw", choices=["auto", "1", "2", "4", "8"], default="auto",
                    help="frames per wave of the verification kernel (auto: autotune)")
    ap.add_argument("--draft-tail", type=int, default=None,
                    help="LSD: first draft step run in the one-launch draft chain of one system "
                         "(0: one launch per step; default: the library's)")
    ap.add_argument("--pipeline", type=int, default=0,
                    help="pipelined LSD windows: verify every group of this many drafted frames on "
                         "a second stream while drafting continues (0: synchronous windows)")
    ap.add_argument("--accept-windows", type=int, default=ACCEPT_SAMPLE_WINDOWS,
                    help="c1, c2: untimed windows behind the reported acceptance")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ec", choices=["auto", "on", "off", "linear"], default="auto",
                    help="speculative error correction of the draft (App. D); linear: "
                         "extrapolated from the last two committed errors; auto: the better "
                         "measured setting of the configuration (c1, c2: on; c3: linear)")
    args = ap.parse_args()
    if args.net_precision is None:
        args.net_precision = "fp8" if args.config == "c5" else "bf16"
    if args.draft_source is None:
        args.draft_source = args.config
    if args.net_train_windows is None:
        args.net_train_windows = 2000 if args.draft_source == "c3" else 500
    if args.fit_frames is None:
        args.fit_frames = 2000 if args.draft_source in ("c4", "c5") else 20000
    if args.ec == "auto":
        args.ec = "linear" if args.config in ("c3", "c4", "c5") else "on"
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only: the batched verification path runs the K frames "
              f"of a window on a single MI355X (asked for --gpus {args.gpus}, WORLD_SIZE {world}).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2606_02455_amd import lsd
    from paper_2606_02455_amd import workloads as W

    lsd.load()
    torch.cuda.set_device(0)
    if args.config in ("c3", "c4", "c5"):
        print(json.dumps(run_c3(args, lsd, W, torch)), flush=True)
        return
    w = W.config(args.config)
    K = w.K
    log(f"workload {w.name}: N={w.n_atoms} K={K} box={w.box[0]:.5f}")

    lsd_skin, plain_skin = W.BENCH_SKINS.get(args.config, (w.skin, w.skin))
    if args.skin is not None:
        lsd_skin = args.skin
    if args.plain_skin is not None:
        plain_skin = args.plain_skin
    log(f"list skins: LSD {lsd_skin}, plain {plain_skin}")
    plain = lsd.LSDSystem(w, mode="plain", skin=plain_skin)
    eq_windows = max(1, args.equilibrate // K)
    plain.run_windows(eq_windows, K)
    torch.cuda.synchronize()
    ec_on = args.ec != "off"
    lsds = lsd.LSDSystem(w, mode="lsd", error_correction=EC_MODES[args.ec], skin=lsd_skin)
    lsds.q.copy_(plain.q)
    lsds.p.copy_(plain.p)
    lsds.img.copy_(plain.img)
    lsds.step.copy_(plain.step)
    st0 = plain.state()
    log(f"equilibrated {int(st0['step'][0])} plain steps")

    # --- verification kernel variant, tuned on this system (one window)
    if args.verify_fw == "auto":
        chosen_fw, fw_us = lsds.autotune_verify(K, repeats=5)
        lsds.verify_window()
        lsds.accept_rollback()
        log(f"autotuned verification: {chosen_fw} frames per wave "
            f"({', '.join(f'{k}: {v:.1f} us' for k, v in fw_us.items())})")
    else:
        chosen_fw, fw_us = int(args.verify_fw), {}
        lsds.set_verify_variant(K, chosen_fw)
        log(f"verification: {chosen_fw} frames per wave (fixed)")

    # --- LSD
    if args.draft_tail is not None:
        lsds.set_draft_tail(args.draft_tail)
    if args.pipeline:
        lsds.set_pipeline(args.pipeline)
    # the warmup runs with the timed windows' graphs already in use, so the
    # timed region starts on warm graphs; the sums restart after it
    lsds.set_verify_timing(True, every=args.time_every)
    lsds.run_windows(args.warmup, K)
    lsds.reset_counters()
    lsds.set_verify_timing(True, every=args.time_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lsds.run_windows(args.steps, K)
    torch.cuda.synchronize()
    t_lsd = time.perf_counter() - t0
    ver_ms, ver_n = lsds.verify_timing()
    cn = lsds.counters()[0]
    lsds.set_verify_timing(False)
    windows, committed, rejections, frames, builds = (int(v) for v in cn)
    assert windows == args.steps
    log(f"LSD: {committed} steps in {t_lsd * 1e3:.1f} ms over {windows} windows; "
        f"rejections {rejections}; verify {ver_ms / max(ver_n, 1) * 1e3:.1f} us/launch")

    # --- acceptance over a fixed sample of windows (untimed), so that the
    # reported rate does not depend on --steps
    lsds.reset_counters()
    for done in range(0, args.accept_windows, 100):
        lsds.run_windows(min(100, args.accept_windows - done), K)
        torch.cuda.synchronize()
        log(f"acceptance sample: {min(done + 100, args.accept_windows)} windows")
    an = lsds.counters()[0]
    acc_committed, acc_rejections, acc_frames = int(an[1]), int(an[2]), int(an[3])
    log(f"acceptance sample: {args.accept_windows} windows, {acc_committed} steps, "
        f"{acc_rejections} rejections")

    # --- plain target Langevin, same kernels, same number of windows
    plain.run_windows(args.warmup, K)
    plain.reset_counters()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plain.run_windows(args.steps, K)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t1
    pc = plain.counters()[0]
    plain_steps = int(pc[1])
    log(f"plain: {plain_steps} steps in {t_plain * 1e3:.1f} ms")
    status = lsds.status() | plain.status()
    if status:
        raise RuntimeError(f"device status {status}: neighbour capacity overflow")

    # --- a plain copy of known size: the reference that scales the
    # FETCH_SIZE / WRITE_SIZE counters of rocprofv3 (profiles/)
    src = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst

    # --- roofline of the dominant kernel (one verification launch)
    frames_per_launch = frames / max(windows, 1)  # one verification launch per window
    pairs = in_cutoff_pairs(lsds, w.target["rc"])
    alg_bytes = frames_per_launch * w.n_atoms * 60.0 + pairs * 4.0
    avg_s = ver_ms / max(ver_n, 1) * 1e-3
    achieved = alg_bytes / avg_s / 1e9
    valu_flops = frames_per_launch * pairs * LJ_PAIR_FLOPS
    prof_us = read_profile_avg_us(args.config, f"k_verify<{chosen_fw}>", lsd_skin)
    roofline = dict(bound="hbm", achieved=round(achieved, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=read_traffic(args.config, f"k_verify<{chosen_fw}>", lsd_skin),
                    kernel=f"k_verify<{chosen_fw}>", avg_us=round(avg_s * 1e6, 3),
                    timing=("HIP events around each timed launch on its stream: the kernel "
                            "plus its dispatch and end-of-kernel latency"),
                    profile_avg_us=prof_us,
                    frac_at_profile_us=(round(alg_bytes / (prof_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
                                        if prof_us else None),
                    timed_launches=int(ver_n), timed_every=args.time_every,
                    autotune_us={str(k): round(v, 2) for k, v in fw_us.items()},
                    algorithmic_bytes=int(alg_bytes), frames_per_launch=round(frames_per_launch, 3),
                    in_cutoff_pairs=pairs,
                    valu=dict(achieved=round(valu_flops / avg_s / 1e12, 3),
                              peak=round(VALU_PEAK_TFLOPS, 2), unit="TFLOP/s",
                              frac=round(valu_flops / avg_s / 1e12 / VALU_PEAK_TFLOPS, 4),
                              flops_per_pair_frame=LJ_PAIR_FLOPS))

    cpu = None
    if not args.no_cpu_baseline:
        st = lsds.state()
        log("timing the FP64 oracle on the host ...")
        cpu = cpu_baseline(w, st["q"], st["p"], args.cpu_seconds, EC_MODES[args.ec])
        log(f"oracle: {cpu['value']:.3f} LSD steps/s, {cpu['plain_steps_per_s']:.3f} plain steps/s "
            f"on {cpu['cores']} threads")

    value = committed / t_lsd
    plain_rate = plain_steps / t_plain
    out = {
        "metric": "target-distributed MD steps/s (LSD vs plain Langevin, 1 GPU); acceptance rate",
        "value": round(value, 3),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_lsd / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"{w.name}: Lennard-Jones fluid, {w.n_atoms} atoms, rho*=0.8, T*=1, "
                         f"target cutoff {w.target['rc']}, draft cutoff {w.draft['rc']}, "
                         f"K={K}, dt={w.dt}, gamma={w.gamma}, seed {w.seed}, "
                         f"error correction {args.ec}"),
            "n_atoms": w.n_atoms, "K": K, "skin": lsd_skin, "plain_skin": plain_skin,
            "error_correction": args.ec,
        },
        "acceptance": round(1.0 - acc_rejections / max(acc_committed, 1), 5),
        "acceptance_sample": {"windows": args.accept_windows, "committed": acc_committed,
                              "rejections": acc_rejections,
                              "K_eff": round(acc_frames / max(args.accept_windows, 1), 3)},
        "acceptance_timed": round(1.0 - rejections / max(committed, 1), 5),
        "K": K,
        "K_eff": round(frames / max(windows, 1), 3),
        "committed_per_window": round(committed / windows, 4),
        "list_builds_per_window": round(builds / windows, 4),
        "plain_steps_per_s": round(plain_rate, 3),
        "lsd_over_plain": round(value / plain_rate, 5),
        "tau_per_day_lsd": round(value * w.dt * 86400.0, 2),
        "tau_per_day_plain": round(plain_rate * w.dt * 86400.0, 2),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
