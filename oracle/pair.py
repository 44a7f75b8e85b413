"""ctypes wrapper of the FP64 force-matched pair draft (pair_oracle.c) and
its least-squares fit.

Test infrastructure only, like the rest of this package."""
import ctypes as C

import numpy as np

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


def declare(L):
    L.ora_pair_types.argtypes = [C.c_int]
    L.ora_pair_types.restype = C.c_int
    L.ora_pair_type.argtypes = [C.c_int, C.c_int, C.c_int]
    L.ora_pair_type.restype = C.c_int
    L.ora_pair_forces.argtypes = [C.c_int, _dp, C.c_double, _ip, C.c_int, C.c_int, C.c_double,
                                  _dp, _dp]
    L.ora_pair_design.argtypes = [C.c_int, _dp, C.c_double, _ip, C.c_int, C.c_int, C.c_double,
                                  _dp]


class PairDraft:
    """Pair-force draft with S species, B basis functions and cutoff rc;
    weights w [S(S+1)/2, B] (or None until fitted)."""

    def __init__(self, n_species, n_basis=16, rc=4.0, w=None):
        from . import lib
        self.lib = lib()
        self.S, self.B, self.rc = int(n_species), int(n_basis), float(rc)
        self.T = self.lib.ora_pair_types(self.S)
        self.w = None if w is None else np.ascontiguousarray(w, dtype=np.float64).reshape(self.T, self.B)

    def type_of(self, a, b):
        return self.lib.ora_pair_type(int(a), int(b), self.S)

    def _args(self, species, x):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
        sp = np.ascontiguousarray(species, dtype=np.int32)
        return x, sp

    def forces(self, species, x, L):
        x, sp = self._args(species, x)
        F = np.zeros_like(x)
        self.lib.ora_pair_forces(len(x), x.ctypes.data_as(_dp), float(L), sp.ctypes.data_as(_ip),
                                 self.S, self.B, self.rc, self.w.ctypes.data_as(_dp),
                                 F.ctypes.data_as(_dp))
        return F

    def design(self, species, x, L):
        """A [3n, T*B] with forces.ravel() = A @ w.ravel()."""
        x, sp = self._args(species, x)
        A = np.zeros((3 * len(x), self.T * self.B))
        self.lib.ora_pair_design(len(x), x.ctypes.data_as(_dp), float(L), sp.ctypes.data_as(_ip),
                                 self.S, self.B, self.rc, A.ctypes.data_as(_dp))
        return A

    def fit(self, species, frames, forces, L, ridge=0.0):
        """Force matching: least squares over all frames (numpy lstsq on the
        stacked design, with an optional ridge term)."""
        A = np.concatenate([self.design(species, x, L) for x in frames])
        y = np.concatenate([np.asarray(f, dtype=np.float64).ravel() for f in forces])
        if ridge > 0.0:
            A = np.concatenate([A, np.sqrt(ridge) * np.eye(A.shape[1])])
            y = np.concatenate([y, np.zeros(A.shape[1])])
        w, *_ = np.linalg.lstsq(A, y, rcond=None)
        self.w = w.reshape(self.T, self.B)
        return self.w
