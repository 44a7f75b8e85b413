"""ctypes wrapper of the FP64 message-passing potential (mpnn_oracle.c).

Test infrastructure only, like the rest of this package."""
import ctypes as C

import numpy as np


class _Mpnn(C.Structure):
    _fields_ = [("n_species", C.c_int), ("H", C.c_int), ("R", C.c_int), ("T", C.c_int),
                ("RH", C.c_int), ("rc", C.c_double), ("scale", C.c_double),
                ("w", C.POINTER(C.c_double))]


def declare(L):
    L.ora_mpnn_layout.argtypes = [C.c_int] * 5
    L.ora_mpnn_layout.restype = C.c_long
    L.ora_mpnn_energy_forces.argtypes = [C.POINTER(_Mpnn), C.c_int, C.POINTER(C.c_int32),
                                         C.POINTER(C.c_double), C.c_double, C.POINTER(C.c_double)]
    L.ora_mpnn_energy_forces.restype = C.c_double


class MPNN:
    """Random-init message-passing potential with flat weights `w`."""

    def __init__(self, w, n_species, rc=5.0, scale=1.0, H=128, R=16, T=3, RH=64):
        from . import lib
        self.lib = lib()
        n = self.lib.ora_mpnn_layout(n_species, H, R, T, RH)
        w = np.ascontiguousarray(w, dtype=np.float64)
        if w.shape != (n,):
            raise ValueError(f"weights must have {n} entries, got {w.shape}")
        self.w = w
        self.n_species, self.rc, self.scale = n_species, float(rc), float(scale)
        self._c = _Mpnn(n_species, H, R, T, RH, self.rc, self.scale,
                        self.w.ctypes.data_as(C.POINTER(C.c_double)))

    def energy_forces(self, species, x, L, forces=True):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
        sp = np.ascontiguousarray(species, dtype=np.int32)
        F = np.zeros_like(x) if forces else None
        E = self.lib.ora_mpnn_energy_forces(
            C.byref(self._c), len(x), sp.ctypes.data_as(C.POINTER(C.c_int32)),
            x.ctypes.data_as(C.POINTER(C.c_double)), float(L),
            F.ctypes.data_as(C.POINTER(C.c_double)) if forces else None)
        return E, F
