"""ctypes wrapper of the FP64 learned many-body draft (net_oracle.c): forces,
the gradient of the force-matching loss, and the Adam update.

Test infrastructure only, like the rest of this package."""
import ctypes as C

import numpy as np

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
HIDDEN = 32


def declare(L):
    L.ora_net_param_count.argtypes = [C.c_int, C.c_int]
    L.ora_net_param_count.restype = C.c_int
    L.ora_net_forward.argtypes = [C.c_int, _dp, C.c_double, _ip, C.c_int, C.c_int, C.c_double,
                                  _dp, _dp, _dp, _dp, _dp]
    L.ora_net_sse_grad.argtypes = [C.c_int, _dp, C.c_double, _ip, C.c_int, C.c_int, C.c_double,
                                   _dp, _dp, _dp]
    L.ora_net_sse_grad.restype = C.c_double
    L.ora_net_backward.argtypes = [C.c_int, _dp, C.c_double, _ip, C.c_int, C.c_int, C.c_double,
                                   _dp, _dp, _dp]
    L.ora_net_adam.argtypes = [C.c_int, _dp, _dp, _dp, _dp, C.c_double, C.c_double, C.c_double,
                               C.c_double, C.c_long]


def _p(a):
    return a.ctypes.data_as(_dp)


class NetDraft:
    """One-layer direct-force draft with S species, B radial functions,
    cutoff rc and flat parameters (W1 [H][S B], b1 [S][H], W2 [B][H],
    c [S(S+1)/2][B])."""

    def __init__(self, n_species, n_basis, rc, params):
        from . import lib
        self.lib = lib()
        self.S, self.B, self.rc = int(n_species), int(n_basis), float(rc)
        self.P = self.lib.ora_net_param_count(self.S, self.B)
        self.params = np.ascontiguousarray(params, dtype=np.float64).ravel()
        assert self.params.size == self.P

    @staticmethod
    def count(S, B):
        from . import lib
        return lib().ora_net_param_count(int(S), int(B))

    def split(self, params=None):
        """(W1, b1, W2, c) views of a flat parameter vector."""
        p = self.params if params is None else params
        S, B, H = self.S, self.B, HIDDEN
        o1 = H * S * B
        o2 = o1 + S * H
        o3 = o2 + B * H
        return (p[:o1].reshape(H, S * B), p[o1:o2].reshape(S, H), p[o2:o3].reshape(B, H),
                p[o3:].reshape(-1, B))

    def _args(self, species, x):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
        sp = np.ascontiguousarray(species, dtype=np.int32)
        return x, sp

    def forward(self, species, x, L, intermediates=False):
        x, sp = self._args(species, x)
        n = len(x)
        F = np.zeros_like(x)
        D = np.zeros((n, self.S * self.B))
        z = np.zeros((n, HIDDEN))
        v = np.zeros((n, self.B))
        self.lib.ora_net_forward(n, _p(x), float(L), sp.ctypes.data_as(_ip), self.S, self.B,
                                 self.rc, _p(self.params), _p(D), _p(z), _p(v), _p(F))
        return (F, D, z, v) if intermediates else F

    def forces(self, species, x, L):
        return self.forward(species, x, L)

    def sse_grad(self, species, x, L, Y, grad=None):
        """(sum |F - Y|^2, gradient of it in the parameters); with `grad`
        given, the gradient is added to it."""
        x, sp = self._args(species, x)
        Y = np.ascontiguousarray(Y, dtype=np.float64).reshape(-1, 3)
        g = np.zeros(self.P) if grad is None else grad
        sse = self.lib.ora_net_sse_grad(len(x), _p(x), float(L), sp.ctypes.data_as(_ip), self.S,
                                        self.B, self.rc, _p(self.params), _p(Y), _p(g))
        return sse, g


    def backward(self, species, x, L, G, grad):
        """grad += sum_i G_i . dF_i/dparams (G [n, 3] = dLoss/dF)."""
        x, sp = self._args(species, x)
        G = np.ascontiguousarray(G, dtype=np.float64).reshape(-1, 3)
        self.lib.ora_net_backward(len(x), _p(x), float(L), sp.ctypes.data_as(_ip), self.S, self.B,
                                  self.rc, _p(self.params), _p(G), _p(grad))
        return grad

    def diff_sse_grad(self, species, frames, L, Ys, grad=None):
        """Squared error of the force changes between consecutive frames,
        sum_k |(F_{k+1} - F_k) - (Y_{k+1} - Y_k)|^2, and its gradient (added
        to `grad` when given)."""
        g = np.zeros(self.P) if grad is None else grad
        F = [self.forces(species, x, L) for x in frames]
        Y = [np.asarray(y, dtype=np.float64).reshape(-1, 3) for y in Ys]
        d = [(F[k + 1] - F[k]) - (Y[k + 1] - Y[k]) for k in range(len(F) - 1)]
        sse = float(sum(np.sum(dk * dk) for dk in d))
        for k, x in enumerate(frames):
            G = np.zeros_like(F[k])
            if k >= 1:
                G += 2.0 * d[k - 1]
            if k + 1 < len(F):
                G -= 2.0 * d[k]
            self.backward(species, x, L, G, g)
        return sse, g


def adam(params, m, v, g, lr, t, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step in place on float64 arrays (step count t >= 1)."""
    from . import lib
    for a in (params, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = np.ascontiguousarray(g, dtype=np.float64)
    lib().ora_net_adam(params.size, _p(params), _p(m), _p(v), _p(g), float(lr), float(beta1),
                       float(beta2), float(eps), int(t))
