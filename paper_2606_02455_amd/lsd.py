"""Thin ctypes binding of the LSD C ABI (include/lsd.h).

Argument marshalling only: every step of the method runs in the HIP
kernels of liblsd.so.  PyTorch supplies device memory (all state, output and
workspace buffers are torch tensors) and the stream.  There is no fallback:
if liblsd.so is missing, ``load()`` raises.
"""
import ctypes as C
import os
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblsd.so")

LSD_OK = 0
MODE_LSD, MODE_PLAIN = 0, 1
POT_LJ, POT_HARMONIC, POT_MPNN, POT_PAIR, POT_NET = 1, 2, 3, 4, 5
PREC_FP32, PREC_BF16, PREC_FP8 = 0, 1, 2
NET_HIDDEN = 32
STATUS_NBR_TARGET, STATUS_NBR_DRAFT, STATUS_CELL = 1, 2, 4

_LIB = None


class LSDError(RuntimeError):
    def __init__(self, status, where, message):
        super().__init__(f"{where} failed with status {status}: {message}")
        self.status = status


NUM_COUNTERS = 5  # LSD_NUM_COUNTERS


class Potential(C.Structure):
    _fields_ = [("kind", C.c_int32), ("cutoff", C.c_double), ("epsilon", C.c_double),
                ("sigma", C.c_double), ("k_spring", C.c_double), ("anchor", C.c_void_p),
                ("force_offset", C.c_void_p), ("weights", C.c_void_p),
                ("n_model_species", C.c_int32), ("energy_scale", C.c_double),
                ("n_basis", C.c_int32), ("precision", C.c_int32),
                ("act_amax", C.c_double * 2)]


class Config(C.Structure):
    _fields_ = [("n_atoms", C.c_int32), ("n_replicas", C.c_int32),
                ("atom_offsets", C.POINTER(C.c_int32)), ("box", C.POINTER(C.c_double)),
                ("species", C.POINTER(C.c_int32)), ("species_mass", C.POINTER(C.c_double)),
                ("n_species", C.c_int32), ("dt", C.c_double), ("gamma", C.c_double),
                ("kT", C.c_double), ("force_unit", C.c_double), ("skin", C.c_double),
                ("k_max", C.c_int32), ("mode", C.c_int32), ("seed", C.c_uint64),
                ("target", Potential), ("draft", Potential),
                ("max_neighbors_target", C.c_int32), ("max_neighbors_draft", C.c_int32),
                ("error_correction", C.c_int32), ("integrator", C.c_int32),
                ("no_list_reuse", C.c_int32)]


class Buffers(C.Structure):
    _fields_ = [("q", C.c_void_p), ("p", C.c_void_p), ("img", C.c_void_p), ("step", C.c_void_p),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("log_ratio", C.c_void_p), ("energy", C.c_void_p), ("accepted", C.c_void_p),
                ("n_committed", C.c_void_p), ("replay_u", C.c_void_p), ("replay_xi", C.c_void_p),
                ("obabo_q", C.c_void_p), ("obabo_p", C.c_void_p)]


class WindowLayout(C.Structure):
    _fields_ = [("q_mid", C.c_size_t), ("p_draft", C.c_size_t), ("f_draft", C.c_size_t),
                ("f_target", C.c_size_t), ("frame_invalid", C.c_size_t),
                ("nbr_target", C.c_size_t), ("cnt_target", C.c_size_t),
                ("nbr_draft", C.c_size_t), ("cnt_draft", C.c_size_t),
                ("error_cache", C.c_size_t), ("error_cache_prev", C.c_size_t),
                ("max_neighbors_target", C.c_int32), ("max_neighbors_draft", C.c_int32),
                ("n_atoms", C.c_int32), ("k_max", C.c_int32)]


EXPORTS = {
    "lsd_workspace_size": ([C.POINTER(Config), C.POINTER(C.c_size_t)], C.c_int),
    "lsd_init_system": ([C.POINTER(Config), C.POINTER(Buffers), C.c_void_p, C.POINTER(C.c_void_p)],
                        C.c_int),
    "lsd_draft_steps": ([C.c_void_p, C.c_int32, C.c_void_p], C.c_int),
    "lsd_mark_drafted": ([C.c_void_p, C.c_int32, C.c_void_p], C.c_int),
    "lsd_verify_window": ([C.c_void_p, C.c_void_p], C.c_int),
    "lsd_accept_rollback": ([C.c_void_p, C.POINTER(C.c_int32), C.c_void_p], C.c_int),
    "lsd_run_windows": ([C.c_void_p, C.c_int32, C.c_int32, C.c_void_p], C.c_int),
    "lsd_get_window_layout": ([C.c_void_p, C.POINTER(WindowLayout)], C.c_int),
    "lsd_get_status": ([C.c_void_p, C.POINTER(C.c_int32), C.c_void_p], C.c_int),
    "lsd_set_step_limit": ([C.c_void_p, C.c_int64], C.c_int),
    "lsd_set_graphs": ([C.c_void_p, C.c_int32], C.c_int),
    "lsd_set_pipeline": ([C.c_void_p, C.c_int32], C.c_int),
    "lsd_get_counters": ([C.c_void_p, C.POINTER(C.c_int64), C.c_void_p], C.c_int),
    "lsd_reset_counters": ([C.c_void_p, C.c_void_p], C.c_int),
    "lsd_set_verify_timing": ([C.c_void_p, C.c_int32], C.c_int),
    "lsd_set_draft_tail": ([C.c_void_p, C.c_int32], C.c_int),
    "lsd_get_verify_timing": ([C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)], C.c_int),
    "lsd_rng_normals": ([C.c_uint64, C.c_int32, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p],
                        C.c_int),
    "lsd_rng_uniforms": ([C.c_uint64, C.c_int32, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p],
                         C.c_int),
    "lsd_fit_pair_scratch_size": ([C.c_void_p, C.c_int32, C.POINTER(C.c_size_t)], C.c_int),
    "lsd_fit_pair_accumulate": ([C.c_void_p, C.c_int32, C.c_double, C.c_int32, C.c_int32,
                                 C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p], C.c_int),
    "lsd_fit_pair_solve": ([C.c_void_p, C.c_int32, C.c_double, C.c_void_p], C.c_int),
    "lsd_autotune_verify": ([C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                             C.POINTER(C.c_double), C.c_void_p], C.c_int),
    "lsd_set_verify_variant": ([C.c_void_p, C.c_int32, C.c_int32], C.c_int),
    "lsd_net_param_count": ([C.c_int32, C.c_int32], C.c_int32),
    "lsd_net_train_scratch_size": ([C.c_void_p, C.POINTER(C.c_size_t)], C.c_int),
    "lsd_net_train_accumulate": ([C.c_void_p, C.POINTER(Potential), C.c_int32, C.c_int32,
                                  C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p], C.c_int),
    "lsd_net_activation_amax": ([C.c_void_p, C.POINTER(Potential), C.c_void_p, C.c_size_t,
                                 C.c_void_p, C.c_void_p], C.c_int),
    "lsd_net_adam_step": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_double,
                           C.c_double, C.c_double, C.c_double, C.c_int64, C.c_void_p], C.c_int),
    "lsd_kinetic_energy_scratch_size": ([C.c_int32, C.c_int32, C.POINTER(C.c_size_t)], C.c_int),
    "lsd_kinetic_energy": ([C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_double), C.c_int32,
                            C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                            C.c_size_t, C.c_void_p], C.c_int),
    "lsd_kinetic_energy_noalloc": ([C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_double),
                                    C.c_int32, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                    C.c_void_p], C.c_int),
    "lsd_pipeline_create": ([C.POINTER(C.c_void_p)], C.c_int),
    "lsd_pipeline_destroy": ([C.c_void_p], C.c_int),
    "lsd_pipeline_submit": ([C.c_void_p, C.POINTER(C.c_int64)], C.c_int),
    "lsd_pipeline_return": ([C.c_void_p, C.c_int64, C.c_int32, C.POINTER(C.c_int32),
                             C.POINTER(C.c_int32)], C.c_int),
    "lsd_pipeline_take_verified": ([C.c_void_p, C.POINTER(C.c_int64), C.c_int32,
                                    C.POINTER(C.c_int32)], C.c_int),
    "lsd_pipeline_counts": ([C.c_void_p, C.POINTER(C.c_int64)], C.c_int),
    "lsd_destroy": ([C.c_void_p], C.c_int),
    "lsd_last_error": ([], C.c_char_p),
}


def load():
    """Load liblsd.so (raises ImportError if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "or python paper_2606_02455_amd/build.py")
        lib = C.CDLL(LIB_PATH)
        for name, (args, res) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _LIB = lib
    return _LIB


def _check(status, where):
    if status != LSD_OK:
        raise LSDError(status, where, load().lsd_last_error().decode())


def _stream(torch):
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def net_param_count(n_species, n_basis):
    """Length of the learned draft's parameter vector (0 if out of range)."""
    return int(load().lsd_net_param_count(int(n_species), int(n_basis)))


def net_init_params(n_species, n_basis, pair_weights=None, seed=0, gain=1.0):
    """Initial parameters of the learned draft (float32 numpy): W1 with
    N(0, gain^2 / (S B)) entries, b1 = 0, W2 = 0 and c = the pair-draft
    weights (or 0), so the draft starts as that pair draft."""
    S, B, H = int(n_species), int(n_basis), NET_HIDDEN
    P = net_param_count(S, B)
    if P == 0:
        raise ValueError("learned draft size out of range")
    rng = np.random.default_rng(seed)
    p = np.zeros(P, np.float64)
    p[:H * S * B] = rng.normal(scale=gain / np.sqrt(S * B), size=H * S * B)
    if pair_weights is not None:
        p[P - S * (S + 1) // 2 * B:] = np.asarray(pair_weights, dtype=np.float64).ravel()
    return p.astype(np.float32)


def net_adam_step(torch, params, m, v, grad, lr, t, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step of lsd_net_adam_step on CUDA tensors: params float32
    [P], m and v float64 [P], grad float64 [P+2] (cleared by the step)."""
    P = params.numel()
    assert m.numel() == P and v.numel() == P and grad.numel() >= P + 2
    _check(load().lsd_net_adam_step(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), P, float(lr),
                                    float(beta1), float(beta2), float(eps), int(t),
                                    _stream(torch)), "lsd_net_adam_step")


def pair_params(n_species, n_basis):
    """Number of pair-draft weights: S(S+1)/2 types x n_basis."""
    return n_species * (n_species + 1) // 2 * n_basis


def fit_pair_solve(gram, ridge=1e-8):
    """Weights [P] from host normal equations [P+1, P+1] (lsd_fit_pair_solve)."""
    g = np.ascontiguousarray(gram, dtype=np.float64)
    P = g.shape[0] - 1
    w = np.zeros(P)
    _check(load().lsd_fit_pair_solve(g.ctypes.data_as(C.c_void_p), P, float(ridge),
                                     w.ctypes.data_as(C.c_void_p)), "lsd_fit_pair_solve")
    return w


def kinetic_energy_scratch_size(n_replicas, max_replica_atoms):
    n = C.c_size_t()
    _check(load().lsd_kinetic_energy_scratch_size(int(n_replicas), int(max_replica_atoms),
                                                  C.byref(n)), "lsd_kinetic_energy_scratch_size")
    return n.value


def kinetic_energy(p, species, species_mass, atom_offsets, max_replica_atoms, out=None,
                   scratch=None):
    """Per-replica kinetic energy (binary64) of device momenta p [3][N]
    (float32); species: int32 device [N] or None; species_mass: host
    sequence; atom_offsets: int32 device [R+1]."""
    import torch
    R = atom_offsets.shape[0] - 1
    if out is None:
        out = torch.empty((R,), dtype=torch.float64, device=p.device)
    if scratch is None:
        scratch = torch.empty((kinetic_energy_scratch_size(R, max_replica_atoms),),
                              dtype=torch.uint8, device=p.device)
    m = (C.c_double * len(species_mass))(*[float(v) for v in species_mass])
    _check(load().lsd_kinetic_energy(_ptr(p), int(p.shape[1]), _ptr(species), m,
                                     len(species_mass), _ptr(atom_offsets), R,
                                     int(max_replica_atoms), _ptr(out), _ptr(scratch),
                                     scratch.numel(), _stream(torch)), "lsd_kinetic_energy")
    return out


def kinetic_energy_noalloc(p, species, species_mass, atom_offsets, max_replica_atoms, out):
    """kinetic_energy without caller scratch (the library's static device
    array); `out` is the caller's binary64 device tensor [R]."""
    import torch
    R = atom_offsets.shape[0] - 1
    m = (C.c_double * len(species_mass))(*[float(v) for v in species_mass])
    _check(load().lsd_kinetic_energy_noalloc(_ptr(p), int(p.shape[1]), _ptr(species), m,
                                             len(species_mass), _ptr(atom_offsets), R,
                                             int(max_replica_atoms), _ptr(out), _stream(torch)),
           "lsd_kinetic_energy_noalloc")
    return out


def rng_normals(seed, replica, step, n):
    import torch
    out = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    _check(load().lsd_rng_normals(seed, replica, step, n, _ptr(out), _stream(torch)),
           "lsd_rng_normals")
    return out


def rng_uniforms(seed, replica, step0, count):
    import torch
    out = torch.empty((count,), dtype=torch.float64, device="cuda")
    _check(load().lsd_rng_uniforms(seed, replica, step0, count, _ptr(out), _stream(torch)),
           "lsd_rng_uniforms")
    return out


class LSDSystem:
    """One or many replicas with the committed state on the GPU.

    target / draft: dicts ``{"kind": "lj", "rc": 2.5, "eps": 1, "sig": 1}`` or
    ``{"kind": "harmonic", "k": 2.0, "anchor": array[N, 3]}``, each with an
    optional ``"offset": array[N, 3]`` constant force field.
    """

    def __init__(self, workload, mode="lsd", k_max=None, target=None, draft=None, seed=None,
                 skin=None, replay=False, max_neighbors=(0, 0), error_correction=False,
                 list_reuse=True, integrator="aboba"):
        import torch
        self.torch = torch
        lib = load()
        w = workload
        self.w = w
        self.N, self.R = w.n_atoms, w.n_replicas
        self.k_max = int(k_max or w.K)
        self.mode = MODE_LSD if mode == "lsd" else MODE_PLAIN
        dev = "cuda"
        self._keep = []
        # host tables
        self._offsets = np.ascontiguousarray(w.atom_offsets, dtype=np.int32)
        self._box = np.ascontiguousarray(w.box, dtype=np.float64)
        self._species = np.ascontiguousarray(w.species, dtype=np.int32)
        self._masses = np.ascontiguousarray(w.species_mass, dtype=np.float64)
        tgt = dict(target or w.target)
        dft = dict(draft or w.draft)
        self.network_target = tgt.get("kind") == "mpnn"
        cfg = Config()
        cfg.n_atoms, cfg.n_replicas = self.N, self.R
        cfg.atom_offsets = self._offsets.ctypes.data_as(C.POINTER(C.c_int32))
        cfg.box = self._box.ctypes.data_as(C.POINTER(C.c_double))
        cfg.species = self._species.ctypes.data_as(C.POINTER(C.c_int32))
        cfg.species_mass = self._masses.ctypes.data_as(C.POINTER(C.c_double))
        cfg.n_species = len(self._masses)
        cfg.dt, cfg.gamma, cfg.kT, cfg.force_unit = w.dt, w.gamma, w.kT, w.force_unit
        cfg.skin = float(skin if skin is not None else w.skin)
        cfg.k_max = self.k_max
        cfg.mode = self.mode
        cfg.seed = int(seed if seed is not None else w.seed)
        cfg.target = self._potential(tgt)
        cfg.draft = self._potential(dft) if self.mode == MODE_LSD else Potential()
        cfg.max_neighbors_target, cfg.max_neighbors_draft = max_neighbors
        cfg.error_correction = int(error_correction)  # 0 off, 1 App. D, 2 linear
        cfg.no_list_reuse = 0 if list_reuse else 1
        if integrator not in ("aboba", "obabo"):
            raise ValueError(f"integrator {integrator!r}")
        self.obabo = integrator == "obabo"
        cfg.integrator = 1 if self.obabo else 0
        self.cfg = cfg
        nbytes = C.c_size_t()
        _check(lib.lsd_workspace_size(C.byref(cfg), C.byref(nbytes)), "lsd_workspace_size")
        t = torch
        self.q = t.tensor(w.positions.T.copy(), dtype=t.float32, device=dev).contiguous()
        self.p = t.tensor(w.momenta.T.copy(), dtype=t.float32, device=dev).contiguous()
        self.img = t.zeros((3, self.N), dtype=t.int32, device=dev)
        self.step = t.zeros((self.R,), dtype=t.int64, device=dev)
        self.workspace = t.zeros((nbytes.value,), dtype=t.uint8, device=dev)
        self.log_ratio = t.zeros((self.R, self.k_max), dtype=t.float64, device=dev)
        self.energy = t.zeros((self.R, self.k_max), dtype=t.float64, device=dev)
        self.accepted = t.zeros((self.R, self.k_max), dtype=t.uint8, device=dev)
        self.n_committed = t.zeros((self.R,), dtype=t.int32, device=dev)
        self.replay_u = t.zeros((self.R, self.k_max), dtype=t.float64, device=dev) if replay else None
        self.replay_xi = (t.zeros((self.k_max, self.N, 3), dtype=t.float64, device=dev)
                          if replay else None)
        buf = Buffers()
        buf.q, buf.p, buf.img, buf.step = _ptr(self.q), _ptr(self.p), _ptr(self.img), _ptr(self.step)
        buf.workspace, buf.workspace_bytes = _ptr(self.workspace), nbytes.value
        buf.log_ratio, buf.energy = _ptr(self.log_ratio), _ptr(self.energy)
        buf.accepted, buf.n_committed = _ptr(self.accepted), _ptr(self.n_committed)
        buf.replay_u, buf.replay_xi = _ptr(self.replay_u), _ptr(self.replay_xi)
        self.obabo_q = t.zeros((3, self.N), dtype=t.float32, device=dev) if self.obabo else None
        self.obabo_p = t.zeros((3, self.N), dtype=t.float32, device=dev) if self.obabo else None
        buf.obabo_q, buf.obabo_p = _ptr(self.obabo_q), _ptr(self.obabo_p)
        self.buf = buf
        handle = C.c_void_p()
        _check(lib.lsd_init_system(C.byref(cfg), C.byref(buf), _stream(t), C.byref(handle)),
               "lsd_init_system")
        self.h = handle
        lay = WindowLayout()
        _check(lib.lsd_get_window_layout(self.h, C.byref(lay)), "lsd_get_window_layout")
        self.layout = lay

    def _potential(self, d):
        t = self.torch
        P = Potential()
        kind = d.get("kind", "lj")
        if kind == "lj":
            P.kind, P.cutoff = POT_LJ, float(d["rc"])
            P.epsilon, P.sigma = float(d.get("eps", 1.0)), float(d.get("sig", 1.0))
        elif kind == "harmonic":
            P.kind, P.k_spring = POT_HARMONIC, float(d["k"])
            anc = t.tensor(np.asarray(d["anchor"], dtype=np.float64).reshape(-1, 3).T.copy(),
                           dtype=t.float32, device="cuda").contiguous()
            self._keep.append(anc)
            P.anchor = anc.data_ptr()
        elif kind == "mpnn":
            P.kind, P.cutoff = POT_MPNN, float(d["rc"])
            wt = t.tensor(np.asarray(d["weights"], dtype=np.float64), dtype=t.float32,
                          device="cuda").contiguous()
            self._keep.append(wt)
            P.weights = wt.data_ptr()
            P.n_model_species = int(d.get("n_model_species", len(self._masses)))
            P.energy_scale = float(d.get("scale", 1.0))
        elif kind == "pair":
            P.kind, P.cutoff = POT_PAIR, float(d["rc"])
            if d.get("weights") is None:
                raise ValueError("the pair draft needs fitted weights (fit_pair_draft)")
            wt = t.tensor(np.asarray(d["weights"], dtype=np.float64).ravel(), dtype=t.float32,
                          device="cuda").contiguous()
            self._keep.append(wt)
            P.weights = wt.data_ptr()
            P.n_model_species = int(d.get("n_model_species", len(self._masses)))
            P.n_basis = int(d["n_basis"])
        elif kind == "net":
            wt = d.get("weights")
            if wt is None:
                raise ValueError("the learned draft needs parameters (net_init_params)")
            if not (hasattr(wt, "is_cuda") and wt.is_cuda):
                wt = t.tensor(np.asarray(wt, dtype=np.float64).ravel(), dtype=t.float32,
                              device="cuda").contiguous()
            # a CUDA float32 tensor is used in place: training may update it
            self._keep.append(wt)
            self._net_fields(P, d, wt)
        else:
            raise ValueError(f"potential kind {kind!r} is not implemented by the library")
        if d.get("offset") is not None:
            off = t.tensor(np.asarray(d["offset"], dtype=np.float64).reshape(-1, 3).T.copy(),
                           dtype=t.float32, device="cuda").contiguous()
            self._keep.append(off)
            P.force_offset = off.data_ptr()
        return P

    # --- the four calls of the method -----------------------------------------
    def draft_steps(self, K):
        _check(load().lsd_draft_steps(self.h, int(K), _stream(self.torch)), "lsd_draft_steps")

    def verify_window(self):
        _check(load().lsd_verify_window(self.h, _stream(self.torch)), "lsd_verify_window")

    def accept_rollback(self, sync=False):
        if sync:
            n = (C.c_int32 * self.R)()
            _check(load().lsd_accept_rollback(self.h, n, _stream(self.torch)),
                   "lsd_accept_rollback")
            return np.array(n[:], dtype=np.int32)
        _check(load().lsd_accept_rollback(self.h, None, _stream(self.torch)), "lsd_accept_rollback")
        return None

    def run_windows(self, n_windows, K):
        _check(load().lsd_run_windows(self.h, int(n_windows), int(K), _stream(self.torch)),
               "lsd_run_windows")

    def mark_drafted(self, K):
        _check(load().lsd_mark_drafted(self.h, int(K), _stream(self.torch)), "lsd_mark_drafted")

    # --- force matching of the pair draft --------------------------------------
    def fit_pair_accumulate(self, n_basis, cutoff, gram, use_target=False, scratch=None,
                            differences=False):
        """Add the normal equations of the current window's valid frames (or
        of the differences of consecutive frames) to `gram` (float64 CUDA
        tensor [P+1, P+1]); returns the scratch tensor (reuse it)."""
        t = self.torch
        nb = C.c_size_t()
        _check(load().lsd_fit_pair_scratch_size(self.h, int(n_basis), C.byref(nb)),
               "lsd_fit_pair_scratch_size")
        if scratch is None or scratch.numel() < nb.value:
            scratch = t.empty((max(nb.value, 8),), dtype=t.uint8, device="cuda")
        _check(load().lsd_fit_pair_accumulate(self.h, int(n_basis), float(cutoff),
                                              1 if use_target else 0, 1 if differences else 0,
                                              _ptr(scratch),
                                              scratch.numel(), _ptr(gram), _stream(t)),
               "lsd_fit_pair_accumulate")
        return scratch

    def _net_fields(self, P, d, wt):
        t = self.torch
        if wt.dtype != t.float32 or not wt.is_contiguous() or not wt.is_cuda:
            raise ValueError("learned-draft parameters must be a contiguous float32 CUDA tensor")
        P.kind, P.cutoff = POT_NET, float(d["rc"])
        P.weights = wt.data_ptr()
        P.n_model_species = int(d.get("n_model_species", len(self._masses)))
        P.n_basis = int(d["n_basis"])
        P.precision = {"fp32": PREC_FP32, "bf16": PREC_BF16,
                       "fp8": PREC_FP8}[d.get("precision", "bf16")]
        if d.get("act_amax") is not None:
            P.act_amax[0], P.act_amax[1] = (float(v) for v in d["act_amax"])

    # --- training of the learned draft -------------------------------------------
    def net_train_accumulate(self, net, grad, use_target=False, scratch=None, differences=False):
        """Add the gradient of the summed squared force error of the learned
        draft `net` (a potential dict of kind "net") over the current
        window's valid frames to `grad` (float64 CUDA [P+2]: gradient,
        squared error, atom frames); net["weights"] must be the float32 CUDA
        parameter tensor.  differences: the loss of the force changes between
        consecutive frames.  Returns the scratch tensor (reuse it)."""
        t = self.torch
        nb = C.c_size_t()
        _check(load().lsd_net_train_scratch_size(self.h, C.byref(nb)),
               "lsd_net_train_scratch_size")
        if scratch is None or scratch.numel() < nb.value:
            scratch = t.empty((max(nb.value, 8),), dtype=t.uint8, device="cuda")
        P = Potential()
        self._net_fields(P, net, net["weights"])   # the caller owns the CUDA parameters
        _check(load().lsd_net_train_accumulate(self.h, C.byref(P), 1 if use_target else 0,
                                               1 if differences else 0, _ptr(scratch), scratch.numel(), _ptr(grad),
                                               _stream(t)), "lsd_net_train_accumulate")
        return scratch

    def net_activation_amax(self, net, scratch=None):
        """(max |D|, max |h|) of the learned draft on the current window's
        valid frames, the FP8 calibration (synchronises)."""
        t = self.torch
        nb = C.c_size_t()
        _check(load().lsd_net_train_scratch_size(self.h, C.byref(nb)),
               "lsd_net_train_scratch_size")
        if scratch is None or scratch.numel() < nb.value:
            scratch = t.empty((max(nb.value, 8),), dtype=t.uint8, device="cuda")
        P = Potential()
        self._net_fields(P, dict(net, precision="fp32"), net["weights"])
        out = t.zeros(2, dtype=t.float64, device="cuda")
        _check(load().lsd_net_activation_amax(self.h, C.byref(P), _ptr(scratch), scratch.numel(),
                                              _ptr(out), _stream(t)), "lsd_net_activation_amax")
        return out.cpu().numpy()

    # --- inspection -------------------------------------------------------------
    def window(self) -> Dict[str, "object"]:
        """Views into the workspace: q_mid [k_max, N, 4] (w = packed image
        deltas), p_draft [k_max+1, 3, N], f_draft / f_target [k_max, 3, N],
        frame_invalid [R, k_max]; error_cache [3, N] (None when error
        correction is off)."""
        t, L, N, K = self.torch, self.layout, self.N, self.k_max
        ws = self.workspace

        def view(off, count, dtype, shape):
            nb = count * t.empty((), dtype=dtype).element_size()
            return ws[off:off + nb].view(dtype).view(*shape)

        return dict(
            q_mid=view(L.q_mid, K * N * 4, t.float32, (K, N, 4)),
            p_draft=view(L.p_draft, (K + 1) * 3 * N, t.float32, (K + 1, 3, N)),
            f_draft=view(L.f_draft, K * 3 * N, t.float32, (K, 3, N)),
            f_target=view(L.f_target, K * 3 * N, t.float32, (K, 3, N)),
            frame_invalid=view(L.frame_invalid, self.R * K, t.int32, (self.R, K)),
            error_cache=(view(L.error_cache, 3 * N, t.float32, (3, N)) if L.error_cache else None),
            error_cache_prev=(view(L.error_cache_prev, 3 * N, t.float32, (3, N))
                              if L.error_cache_prev else None),
        )

    def neighbor_lists(self, which="target"):
        """(counts [N], entries [N, width] as int32 j << 5 | image code)."""
        t, L, N = self.torch, self.layout, self.N
        ws = self.workspace
        if which == "target":
            off, coff, m = L.nbr_target, L.cnt_target, L.max_neighbors_target
        else:
            off, coff, m = L.nbr_draft, L.cnt_draft, L.max_neighbors_draft
        cnt = ws[coff:coff + 4 * N].view(t.int32).clone()
        ent = ws[off:off + 4 * m * N].view(t.int32).view(N, m).clone()
        return cnt, ent

    def status(self):
        f = C.c_int32()
        _check(load().lsd_get_status(self.h, C.byref(f), _stream(self.torch)), "lsd_get_status")
        return int(f.value)

    NET_SHAPES = [(f, c) for f in (256, 512, 1024) for c in (16, 32, 64)]

    def autotune_verify(self, K, repeats=10):
        """Pick the fastest verification variant; drafts one window (left
        drafted).  Pair targets: frames per wave of the verification kernel
        for windows of K frames, returns (chosen, {fw: microseconds}).
        Network target: the evaluation's launch shape, returns (candidate,
        {(filter blocks, chain rows): microseconds})."""
        ch = C.c_int32()
        us = (C.c_double * 9)()
        _check(load().lsd_autotune_verify(self.h, int(K), int(repeats), C.byref(ch), us,
                                          _stream(self.torch)), "lsd_autotune_verify")
        if self.network_target:
            return int(ch.value), {self.NET_SHAPES[c]: us[c] for c in range(9)}
        return int(ch.value), {1: us[0], 2: us[1], 4: us[2], 8: us[3]}

    def set_verify_variant(self, K, frames_per_wave):
        """Fix the verification variant without timing: 1, 2, 4 or 8 frames
        per wave for windows of K frames (pair targets), or the launch-shape
        candidate 0..8 (network target)."""
        _check(load().lsd_set_verify_variant(self.h, int(K), int(frames_per_wave)),
               "lsd_set_verify_variant")

    def set_graphs(self, on=True):
        """Replay captured HIP graphs in run_windows (default) or not."""
        _check(load().lsd_set_graphs(self.h, 1 if on else 0), "lsd_set_graphs")

    def set_pipeline(self, group_frames):
        """Pipelined windows in run_windows: verify every group of
        `group_frames` drafted frames on a second stream while drafting
        continues, stopping the window's drafting at the first rejection
        (0: synchronous windows)."""
        _check(load().lsd_set_pipeline(self.h, int(group_frames)), "lsd_set_pipeline")

    def set_step_limit(self, limit):
        """Stop every replica exactly at step `limit` (None: no limit)."""
        lim = (1 << 63) - 1 if limit is None else int(limit)
        _check(load().lsd_set_step_limit(self.h, lim), "lsd_set_step_limit")

    def run_to_step(self, n_steps, K, check_every=16, max_windows=100000):
        """Windows of K frames until every replica has committed exactly
        n_steps steps."""
        self.set_step_limit(n_steps)
        done = 0
        while done < max_windows:
            self.run_windows(check_every, K)
            done += check_every
            if int(self.state()["step"].min()) >= n_steps:
                return done
        raise RuntimeError("run_to_step did not reach the step count")

    def counters(self):
        """int64 [R, 5]: windows, committed steps, rejections, frames verified,
        neighbour-list builds."""
        out = (C.c_int64 * (NUM_COUNTERS * self.R))()
        _check(load().lsd_get_counters(self.h, out, _stream(self.torch)), "lsd_get_counters")
        return np.array(out[:], dtype=np.int64).reshape(self.R, NUM_COUNTERS)

    def reset_counters(self):
        _check(load().lsd_reset_counters(self.h, _stream(self.torch)), "lsd_reset_counters")

    def set_draft_tail(self, first_step):
        """Draft steps first_step .. K-1 of a short system's window in one
        launch (0: one launch per step)."""
        _check(load().lsd_set_draft_tail(self.h, int(first_step)), "lsd_set_draft_tail")

    def set_verify_timing(self, on=True, every=1):
        """Time every `every`-th verification launch with HIP events."""
        _check(load().lsd_set_verify_timing(self.h, int(every) if on else 0),
               "lsd_set_verify_timing")

    def verify_timing(self):
        ms, n = C.c_double(), C.c_int64()
        _check(load().lsd_get_verify_timing(self.h, C.byref(ms), C.byref(n)),
               "lsd_get_verify_timing")
        return ms.value, n.value

    def kinetic_energy(self, p=None):
        """Per-replica kinetic energy (binary64, device [R]) of the committed
        momenta, or of the given device momenta [3][N]."""
        t = self.torch
        if getattr(self, "_ke_tables", None) is None:
            off = t.tensor(self._offsets, dtype=t.int32, device="cuda")
            spc = t.tensor(self._species, dtype=t.int32, device="cuda")
            nmax = int(np.diff(self._offsets).max())
            scr = t.empty((kinetic_energy_scratch_size(self.R, nmax),), dtype=t.uint8,
                          device="cuda")
            self._ke_tables = (off, spc, nmax, scr)
        off, spc, nmax, scr = self._ke_tables
        return kinetic_energy(self.p if p is None else p, spc, list(self._masses), off, nmax,
                              scratch=scr)

    def state(self):
        """Committed state; with the (OBABO) integrator q and p are the
        (OBABO) state of the last committed step (the library's own state is
        the staggered one) and img is not meaningful for them."""
        self.torch.cuda.synchronize()
        if self.obabo:
            return dict(q=self.obabo_q.T.double().cpu().numpy(),
                        p=self.obabo_p.T.double().cpu().numpy(),
                        img=self.img.T.cpu().numpy(), step=self.step.cpu().numpy())
        return dict(q=self.q.T.double().cpu().numpy(), p=self.p.T.double().cpu().numpy(),
                    img=self.img.T.cpu().numpy(), step=self.step.cpu().numpy())

    def set_state(self, q, p, img=None, step=None):
        t = self.torch
        self.q.copy_(t.tensor(np.asarray(q, dtype=np.float64).T, dtype=t.float32))
        self.p.copy_(t.tensor(np.asarray(p, dtype=np.float64).T, dtype=t.float32))
        if img is not None:
            self.img.copy_(t.tensor(np.asarray(img).T, dtype=t.int32))
        if step is not None:
            self.step.copy_(t.tensor(np.asarray(step), dtype=t.int64))

    def destroy(self):
        if getattr(self, "h", None):
            load().lsd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Pipeline:
    """Verifier state of pipelined LSD (lsd_pipeline_*): host bookkeeping of
    eligible-pending, conditionally verified and verified step ids."""

    def __init__(self):
        self.h = C.c_void_p()
        _check(load().lsd_pipeline_create(C.byref(self.h)), "lsd_pipeline_create")

    def submit(self):
        i = C.c_int64()
        _check(load().lsd_pipeline_submit(self.h, C.byref(i)), "lsd_pipeline_submit")
        return int(i.value)

    def returned(self, step_id, accepted):
        """(ignored, rollback) for a target result of step `step_id`."""
        ig, rb = C.c_int32(), C.c_int32()
        _check(load().lsd_pipeline_return(self.h, int(step_id), 1 if accepted else 0,
                                          C.byref(ig), C.byref(rb)), "lsd_pipeline_return")
        return bool(ig.value), bool(rb.value)

    def take_verified(self, cap=4096):
        ids = (C.c_int64 * cap)()
        n = C.c_int32()
        _check(load().lsd_pipeline_take_verified(self.h, ids, cap, C.byref(n)),
               "lsd_pipeline_take_verified")
        return [int(v) for v in ids[:n.value]]

    def counts(self):
        out = (C.c_int64 * 3)()
        _check(load().lsd_pipeline_counts(self.h, out), "lsd_pipeline_counts")
        return tuple(int(v) for v in out)

    def __del__(self):
        if getattr(self, "h", None) and self.h.value:
            load().lsd_pipeline_destroy(self.h)
            self.h = C.c_void_p()
