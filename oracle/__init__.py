"""FP64 CPU oracle for Langevin Speculative Dynamics -- TEST INFRASTRUCTURE.

Only tests/, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
bench.py may import this package.  It is a ctypes wrapper over the plain C
code in oracle/*.c (FP64, no FMA contraction) and shares no code with the HIP
library in paper_2606_02455_amd/.

Paper: "Speculative Sampling For Faster Molecular Dynamics" (arXiv 2606.02455).
  * Eq. aboba / Eq. bob (Sec. 2.1, Sec. 3.1): ABOBA splitting, BOB Gaussian.
  * Eq. reflectionVerify (Sec. 3.1): reflection-maximal coupling.
  * Alg. 1 (App. C): synchronous speculative window; Alg. 2 draft_step /
    verify_step per-step maps.
  * Drafts (Sec. 3, Sec. 4): pair.py, the force-matched pair draft; net.py,
    the learned one-layer direct-force draft and its training (loss
    gradient, Adam).
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

POT_NONE, POT_LJ, POT_HARMONIC, POT_EXT = 0, 1, 2, 3


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        _LIB = C.CDLL(path)
        _declare(_LIB)
    return _LIB


class _Sys(C.Structure):
    _fields_ = [("n", C.c_int), ("L", C.c_double), ("mass", C.POINTER(C.c_double)),
                ("dt", C.c_double), ("gamma", C.c_double), ("kT", C.c_double),
                ("fu", C.c_double)]


class _Pot(C.Structure):
    _fields_ = [("kind", C.c_int), ("rc", C.c_double), ("eps", C.c_double),
                ("sig", C.c_double), ("k", C.c_double),
                ("qref", C.POINTER(C.c_double)), ("offset", C.POINTER(C.c_double)),
                ("ext", C.c_void_p), ("ext_ctx", C.c_void_p)]


# contexts of the force fields of the other oracle files (kind POT_EXT)
class _MpnnCtx(C.Structure):
    _fields_ = [("m", C.c_void_p), ("species", C.c_void_p)]


class _DraftCtx(C.Structure):
    _fields_ = [("S", C.c_int), ("B", C.c_int), ("rc", C.c_double), ("w", C.c_void_p),
                ("species", C.c_void_p)]


class _WinOut(C.Structure):
    _fields_ = [("logr", C.POINTER(C.c_double)), ("S1", C.POINTER(C.c_double)),
                ("S2", C.POINTER(C.c_double)), ("E_target", C.POINTER(C.c_double)),
                ("accept", C.POINTER(C.c_int8)), ("q_mid", C.POINTER(C.c_double)),
                ("p_draft", C.POINTER(C.c_double)), ("F_draft", C.POINTER(C.c_double)),
                ("F_target", C.POINTER(C.c_double)), ("n_committed", C.c_int32),
                ("rejected", C.c_int32)]


class _Stats(C.Structure):
    _fields_ = [("windows", C.c_int64), ("rejections", C.c_int64),
                ("frames", C.c_int64), ("committed", C.c_int64)]


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


def _declare(L):
    L.ora_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                    C.POINTER(C.c_uint32)]
    L.ora_uniform.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64]
    L.ora_uniform.restype = C.c_double
    L.ora_normals.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_int, _dp]
    L.ora_pairs_brute.argtypes = [C.c_int, _dp, C.c_double, C.c_double, _ip, C.c_long]
    L.ora_pairs_brute.restype = C.c_long
    L.ora_pairs_cells.argtypes = [C.c_int, _dp, C.c_double, C.c_double, _ip, C.c_long]
    L.ora_pairs_cells.restype = C.c_long
    L.ora_energy_forces.argtypes = [C.POINTER(_Pot), C.c_int, _dp, C.c_double, _dp, C.c_int]
    L.ora_energy_forces.restype = C.c_double
    L.ora_aboba_step.argtypes = [C.POINTER(_Sys), C.POINTER(_Pot), _dp, _dp, _ip, _dp]
    L.ora_aboba_step.restype = C.c_double
    L.ora_reflection_verify.argtypes = [C.c_int, _dp, _dp, _dp, _dp, C.c_double, _dp,
                                        _dp, _dp, _dp]
    L.ora_reflection_verify.restype = C.c_int
    L.ora_verify_frame.argtypes = [C.POINTER(_Sys), C.POINTER(_Pot), _dp, _dp, _dp, _dp,
                                   C.c_double, C.c_int, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    L.ora_verify_frame.restype = C.c_int
    L.ora_lsd_window.argtypes = [C.POINTER(_Sys), C.POINTER(_Pot), C.POINTER(_Pot), _dp,
                                 _dp, _ip, C.c_int, _dp, _dp, C.POINTER(_WinOut), _dp, _dp,
                                 C.POINTER(C.c_int)]
    L.ora_lsd_window.restype = C.c_int
    L.ora_lsd_run.argtypes = [C.POINTER(_Sys), C.POINTER(_Pot), C.POINTER(_Pot), _dp, _dp,
                              _ip, C.c_uint64, C.c_uint32, C.c_uint64, C.c_int64, C.c_int,
                              _dp, _dp, C.POINTER(_Stats), _dp, _dp]
    L.ora_plain_run.argtypes = [C.POINTER(_Sys), C.POINTER(_Pot), _dp, _dp, _ip,
                                C.c_uint64, C.c_uint32, C.c_uint64, C.c_int64, _dp, _dp, _dp]
    L.ora_num_threads.restype = C.c_int
    L.ora_kinetic_energy.argtypes = [C.c_int, _dp, _dp]
    L.ora_kinetic_energy.restype = C.c_double
    L.ora_normals_tag.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint32, C.c_int, _dp]
    L.ora_obabo_step.argtypes = [C.POINTER(_Sys), C.POINTER(_Pot), _dp, _dp, _ip, _dp, _dp]
    L.ora_obabo_step.restype = C.c_double
    L.ora_obabo_plain_run.argtypes = [C.POINTER(_Sys), C.POINTER(_Pot), _dp, _dp, _ip, C.c_uint64,
                                      C.c_uint32, C.c_uint64, C.c_int64]
    L.ora_obabo_lsd_run.argtypes = [C.POINTER(_Sys), C.POINTER(_Pot), C.POINTER(_Pot), _dp, _dp,
                                    _ip, C.c_uint64, C.c_uint32, C.c_int64, C.c_int,
                                    C.POINTER(_Stats)]
    L.ora_obabo_begin.argtypes = [C.POINTER(_Sys), C.POINTER(_Pot), _dp, _dp, _ip, C.c_uint64,
                                  C.c_uint32, C.c_uint64]
    L.ora_obabo_recover.argtypes = [C.POINTER(_Sys), C.POINTER(_Pot), _dp, _dp, _dp, C.c_uint64,
                                    C.c_uint32, C.c_uint64, _dp, _dp, _ip]
    if hasattr(L, "ora_mpnn_energy_forces"):
        from . import mpnn as _m
        _m.declare(L)
    if hasattr(L, "ora_pair_forces"):
        from . import pair as _p
        _p.declare(L)
    if hasattr(L, "ora_net_forward"):
        from . import net as _n
        _n.declare(L)


def _d(a):
    """float64 C-contiguous array pointer (None -> NULL)."""
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ----------------------------------------------------------------------------
class System:
    """Cubic periodic box of edge L with per-atom masses and ABOBA parameters."""

    def __init__(self, n, L, masses, dt, gamma, kT, fu=1.0):
        self.n, self.L = int(n), float(L)
        self.masses = _f64(np.broadcast_to(np.asarray(masses, dtype=np.float64), (self.n,)))
        self.dt, self.gamma, self.kT, self.fu = float(dt), float(gamma), float(kT), float(fu)
        self._c = _Sys(self.n, self.L, _d(self.masses), self.dt, self.gamma, self.kT, self.fu)

    @property
    def a(self):
        return np.exp(-self.gamma * self.dt)

    def sigma(self):
        """sqrt of the diagonal of Sigma = M kT (1 - e^{-2 gamma dt}) per atom."""
        return np.sqrt(self.masses * self.kT * self.fu * (1.0 - np.exp(-2 * self.gamma * self.dt)))


class Potential:
    def __init__(self, kind, rc=0.0, eps=1.0, sig=1.0, k=0.0, qref=None, offset=None):
        self.kind = kind
        self.rc, self.eps, self.sig, self.k = float(rc), float(eps), float(sig), float(k)
        self.qref = None if qref is None else _f64(qref).reshape(-1, 3)
        self.offset = None if offset is None else _f64(offset).reshape(-1, 3)
        self._c = _Pot(kind, self.rc, self.eps, self.sig, self.k, _d(self.qref), _d(self.offset))

    @staticmethod
    def lj(rc, eps=1.0, sig=1.0, offset=None):
        return Potential(POT_LJ, rc=rc, eps=eps, sig=sig, offset=offset)

    @staticmethod
    def harmonic(k, qref, offset=None):
        return Potential(POT_HARMONIC, k=k, qref=qref, offset=offset)

    def with_offset(self, offset):
        if self.kind == POT_EXT:
            raise ValueError("offsets of external force fields are not supported")
        return Potential(self.kind, self.rc, self.eps, self.sig, self.k, self.qref, offset)

    @staticmethod
    def _external(fn_name, ctx, keep):
        pot = Potential(POT_EXT)
        pot._keep = keep + [ctx]
        pot._c.ext = C.cast(getattr(lib(), fn_name), C.c_void_p)
        pot._c.ext_ctx = C.cast(C.pointer(ctx), C.c_void_p)
        return pot

    @staticmethod
    def mpnn(net, species):
        """The message-passing network (oracle.mpnn.MPNN) as a force field of
        the integrator and window functions, for atoms of the given species."""
        sp = np.ascontiguousarray(species, dtype=np.int32)
        ctx = _MpnnCtx(C.cast(C.pointer(net._c), C.c_void_p), sp.ctypes.data)
        return Potential._external("ora_mpnn_ext", ctx, [net, sp])

    @staticmethod
    def net_draft(draft, species):
        """The learned draft (oracle.net.NetDraft) as a force field."""
        sp = np.ascontiguousarray(species, dtype=np.int32)
        ctx = _DraftCtx(draft.S, draft.B, draft.rc, draft.params.ctypes.data, sp.ctypes.data)
        return Potential._external("ora_net_ext", ctx, [draft, sp])

    @staticmethod
    def pair_draft(draft, species):
        """The pair draft (oracle.pair.PairDraft, weights fitted) as a force field."""
        sp = np.ascontiguousarray(species, dtype=np.int32)
        w = np.ascontiguousarray(draft.w, dtype=np.float64)
        ctx = _DraftCtx(draft.S, draft.B, draft.rc, w.ctypes.data, sp.ctypes.data)
        return Potential._external("ora_pair_ext", ctx, [draft, sp, w])


# ----------------------------------------------------------------------------
def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().ora_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def uniform(seed, replica, step):
    return lib().ora_uniform(seed, replica, step)


def normals(seed, replica, step, n):
    out = np.zeros((n, 3))
    lib().ora_normals(seed, replica, step, n, _d(out))
    return out


def pairs(x, L, rc, method="brute"):
    """All ordered (i, j, nx, ny, nz) with |x_j + n L - x_i| < rc, sorted."""
    x = _f64(x).reshape(-1, 3)
    fn = lib().ora_pairs_brute if method == "brute" else lib().ora_pairs_cells
    cnt = fn(len(x), _d(x), L, rc, None, 0)
    if cnt < 0:
        raise ValueError("cell enumeration needs floor(L/rc) >= 3")
    out = np.zeros((max(cnt, 1), 5), dtype=np.int32)
    fn(len(x), _d(x), L, rc, out.ctypes.data_as(_ip), cnt)
    out = out[:cnt]
    order = np.lexsort((out[:, 4], out[:, 3], out[:, 2], out[:, 1], out[:, 0]))
    return out[order]


def energy_forces(pot, x, L, parallel=True):
    x = _f64(x).reshape(-1, 3)
    F = np.zeros_like(x)
    E = lib().ora_energy_forces(C.byref(pot._c), len(x), _d(x), L, _d(F), int(parallel))
    return E, F


def aboba_step(system, pot, q, p, img, xi):
    """In-place plain ABOBA step; returns the potential energy at the midpoint."""
    return lib().ora_aboba_step(C.byref(system._c), C.byref(pot._c), _d(q), _d(p),
                                img.ctypes.data_as(_ip), _d(_f64(xi)))


def reflection_verify(mu_t, mu_d, sig, p_draft, u):
    mu_t, mu_d, sig, pd = (_f64(v).ravel() for v in (mu_t, mu_d, sig, p_draft))
    out = np.zeros_like(pd)
    lr, s1, s2 = C.c_double(), C.c_double(), C.c_double()
    acc = lib().ora_reflection_verify(len(pd), _d(mu_t), _d(mu_d), _d(sig), _d(pd), float(u),
                                      _d(out), C.byref(lr), C.byref(s1), C.byref(s2))
    return bool(acc), out, lr.value, s1.value, s2.value


def verify_frame(system, target, q_mid, p_prev, p_new, F_d, u):
    n = system.n
    q_mid, p_prev, p_new, F_d = (_f64(v).reshape(n, 3) for v in (q_mid, p_prev, p_new, F_d))
    Ft, po, qo = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 3))
    E, lr, s1, s2 = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    acc = lib().ora_verify_frame(C.byref(system._c), C.byref(target._c), _d(q_mid), _d(p_prev),
                                 _d(p_new), _d(F_d), float(u), 1, _d(Ft), C.byref(E),
                                 C.byref(lr), C.byref(s1), C.byref(s2), _d(po), _d(qo))
    return dict(accept=bool(acc), F_target=Ft, E_target=E.value, logr=lr.value, S1=s1.value,
                S2=s2.value, p=po, q=qo)


def lsd_window(system, target, draft, q, p, img, xi, u, ec=None, ec_prev=None, samples=None):
    """One synchronous LSD window; (q, p, img) advance in place.  ec: the
    error-correction cache [n, 3] (App. D), updated in place, or None;
    ec_prev and samples (a one-element int32 array): the linear variant."""
    n, K = system.n, len(u)
    xi = _f64(xi).reshape(K, n, 3)
    u = _f64(u)
    res = {name: np.zeros(K) for name in ("logr", "S1", "S2", "E_target")}
    acc = np.zeros(K, dtype=np.int8)
    qm, Fd, Ft = (np.zeros((K, n, 3)) for _ in range(3))
    pd = np.zeros((K + 1, n, 3))
    o = _WinOut(_d(res["logr"]), _d(res["S1"]), _d(res["S2"]), _d(res["E_target"]),
                acc.ctypes.data_as(C.POINTER(C.c_int8)), _d(qm), _d(pd), _d(Fd), _d(Ft), 0, 0)
    lib().ora_lsd_window(C.byref(system._c), C.byref(target._c), C.byref(draft._c), _d(q), _d(p),
                         img.ctypes.data_as(_ip), K, _d(xi), _d(u), C.byref(o), _d(ec),
                         _d(ec_prev),
                         None if samples is None else samples.ctypes.data_as(C.POINTER(C.c_int)))
    res.update(accept=acc.astype(bool), q_mid=qm, p_draft=pd, F_draft=Fd, F_target=Ft,
               n_committed=o.n_committed, rejected=bool(o.rejected))
    return res


def lsd_run(system, target, draft, q, p, img, seed, replica, step0, n_steps, K, record=False,
            ec=None, ec_prev=None):
    """LSD from committed step step0 until n_steps more are committed; ec
    (and ec_prev for the linear variant) are the error-correction caches."""
    n = system.n
    tq = np.zeros((n_steps, n, 3)) if record else None
    tp = np.zeros((n_steps, n, 3)) if record else None
    st = _Stats()
    lib().ora_lsd_run(C.byref(system._c), C.byref(target._c), C.byref(draft._c), _d(q), _d(p),
                      img.ctypes.data_as(_ip), seed, replica, step0, n_steps, K, _d(tq), _d(tp),
                      C.byref(st), _d(ec), _d(ec_prev))
    stats = dict(windows=st.windows, rejections=st.rejections, frames=st.frames,
                 committed=st.committed)
    return stats, tq, tp


def plain_run(system, target, q, p, img, seed, replica, step0, n_steps, record=False):
    n = system.n
    tq = np.zeros((n_steps, n, 3)) if record else None
    tp = np.zeros((n_steps, n, 3)) if record else None
    E = np.zeros(n_steps)
    lib().ora_plain_run(C.byref(system._c), C.byref(target._c), _d(q), _d(p),
                        img.ctypes.data_as(_ip), seed, replica, step0, n_steps, _d(tq), _d(tp),
                        _d(E))
    return E, tq, tp


def num_threads():
    return lib().ora_num_threads()


def kinetic_energy(p, mass):
    """K = sum_i |p_i|^2 / (2 m_i) in binary64 (p: [n, 3]; mass: scalar or
    per atom [n]); the kinetic temperature of Sec. 4.3 is 2 K / (3 n k_B)."""
    p = _f64(p).reshape(-1, 3)
    n = p.shape[0]
    m = np.ascontiguousarray(np.broadcast_to(np.asarray(mass, np.float64), (n,)))
    return lib().ora_kinetic_energy(n, _d(p), _d(m))


def kinetic_temperature(p, mass, k_B=1.0):
    """T_kin = 2 K / (3 n k_B): no constraints, no removal of the centre of
    mass motion.  The paper's formula (Sec. 4.3) lacks the 3 of the three
    axes; with it, equipartition gives <T_kin> = T."""
    p = _f64(p).reshape(-1, 3)
    return 2.0 * kinetic_energy(p, mass) / (3.0 * p.shape[0] * k_B)


# --- (OBABO) splitting (App. E) ----------------------------------------------
def normals_tag(seed, replica, step, tag, n):
    out = np.zeros((n, 3))
    lib().ora_normals_tag(seed, replica, step, tag, n, _d(out))
    return out


def obabo_step(system, pot, q, p, img, xi1, xi2):
    return lib().ora_obabo_step(C.byref(system._c), C.byref(pot._c), _d(q), _d(p),
                                img.ctypes.data_as(_ip), _d(_f64(xi1)), _d(_f64(xi2)))


def obabo_plain_run(system, pot, q, p, img, seed, replica, step0, n_steps):
    lib().ora_obabo_plain_run(C.byref(system._c), C.byref(pot._c), _d(q), _d(p),
                              img.ctypes.data_as(_ip), seed, replica, step0, n_steps)


def obabo_lsd_run(system, target, draft, q, p, img, seed, replica, n_steps, K):
    """LSD for (OBABO) in the staggered frame: (q, p) = y_0 on entry, the
    (OBABO) state at step n_steps on return."""
    st = _Stats()
    lib().ora_obabo_lsd_run(C.byref(system._c), C.byref(target._c), C.byref(draft._c), _d(q),
                            _d(p), img.ctypes.data_as(_ip), seed, replica, n_steps, K,
                            C.byref(st))
    return dict(windows=st.windows, rejections=st.rejections, frames=st.frames,
                committed=st.committed)


def obabo_begin(system, target, q, p, img, seed, replica, step=0):
    """In place: (OBABO) state y = (q, p) -> the staggered (ABOBA) state of
    LSD for (OBABO) (the OB half step with tag-3 noise at `step`)."""
    lib().ora_obabo_begin(C.byref(system._c), C.byref(target._c), _d(q), _d(p),
                          img.ctypes.data_as(_ip), seed, replica, step)


def obabo_recover(system, target, q, p, p_prev, seed, replica, step):
    """(q_n, p_n) of the (OBABO) state at committed step `step` from the
    staggered state (q, p) and the staggered momentum of the step before."""
    n = system.n
    q, p, pp = (_f64(v).reshape(n, 3) for v in (q, p, p_prev))
    qo, po = np.zeros((n, 3)), np.zeros((n, 3))
    lib().ora_obabo_recover(C.byref(system._c), C.byref(target._c), _d(q), _d(p), _d(pp), seed,
                            replica, step, _d(qo), _d(po), None)
    return qo, po
