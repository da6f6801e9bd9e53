"""ctypes view of the plain-C oracle (liborc.so) — TEST INFRASTRUCTURE ONLY.

Every function here marshals arguments and calls the C code; the arithmetic
lives in orc.c, each function of which cites the passage of the paper it
follows.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build()
        L = C.CDLL(path)
        p = C.c_void_p
        u8p = np.ctypeslib.ndpointer(np.uint8, flags="C")
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C")
        f32p = np.ctypeslib.ndpointer(np.float32, flags="C")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C")
        D = C.POINTER(C.c_double)
        L.orc_geometry.argtypes = [C.c_uint32, C.c_double, C.c_double, D,
                                   C.POINTER(C.c_uint32), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_uint32)]
        L.orc_geometry.restype = C.c_int
        L.orc_create.argtypes = [C.c_uint32, C.c_double, C.c_uint64, C.c_double, C.c_int,
                                 C.c_uint32, C.c_uint32]
        L.orc_create.restype = p
        L.orc_free.argtypes = [p]
        L.orc_clone.argtypes = [p]
        L.orc_clone.restype = p
        L.orc_set_positions_q.argtypes = [p, i64p, i64p]
        L.orc_set_positions_q.restype = C.c_int
        L.orc_set_step.argtypes = [p, C.c_uint32]
        L.orc_sweep.argtypes = [p, C.c_uint64, C.c_int]
        L.orc_info.argtypes = [p, D, D, D, C.POINTER(C.c_uint32), C.POINTER(C.c_int64),
                               C.POINTER(C.c_uint32), C.POINTER(C.c_uint64),
                               C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                               C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
        L.orc_get_cells.argtypes = [p, u8p, u32p, f32p, f32p]
        L.orc_get_positions_q.argtypes = [p, i64p, i64p]
        L.orc_count_overlaps.argtypes = [p]
        L.orc_count_overlaps.restype = C.c_uint64
        L.orc_hist_edges.argtypes = [C.c_uint32, C.c_double, f32p]
        L.orc_pair_hist.argtypes = [p, C.c_uint32, C.c_double, i64p]
        L.orc_pair_hist_subset.argtypes = [p, u8p, C.c_uint32, C.c_double, i64p]
        L.orc_pressure.argtypes = [i64p, C.c_uint32, C.c_double, C.c_uint32, C.c_uint64,
                                   C.c_uint32, C.c_double, D, D, D, f64p]
        L.orc_pressure.restype = C.c_int
        L.orc_psi6.argtypes = [p, C.c_void_p, f64p, f64p]
        L.orc_psi6_field.argtypes = [p, f64p, f64p, f64p, f64p]
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
        L.orc_structure_factor.argtypes = [p, i32p, C.c_uint32, f64p]
        L.orc_chi.argtypes = [p, C.c_int32, C.c_int32, f64p, f64p]
        L.orc_cq.argtypes = [p, C.c_double, C.c_double, C.c_double, C.c_uint32, f64p, i64p]
        L.orc_cq.restype = C.c_int
        L.orc_acf.argtypes = [f64p, f64p, C.c_uint32, C.c_uint32, f64p]
        L.orc_tau_fit.argtypes = [f64p, C.c_uint32, C.c_double, C.c_double]
        L.orc_tau_fit.restype = C.c_double
        L.orc_tau_int.argtypes = [f64p, C.c_uint32, C.c_double]
        L.orc_tau_int.restype = C.c_double
        L.orc_philox.argtypes = [C.c_uint32, C.c_uint32, u32p, u32p]
        L.orc_features.argtypes = [p, C.c_uint32, C.c_uint32, C.c_float, C.c_float, f32p]
        L.orc_features.restype = C.c_int
        L.orc_mlp_forward.argtypes = [f64p, f64p, f64p]
        L.orc_gmm_logpdf.argtypes = [f64p, C.c_double, C.c_double]
        L.orc_gmm_logpdf.restype = C.c_double
        L.orc_nll_grad.argtypes = [f64p, f64p, f64p, C.c_uint32, f64p]
        L.orc_nll_grad.restype = C.c_double
        L.orc_adam.argtypes = [f64p, f64p, f64p, f64p, C.c_uint32, C.c_double, C.c_uint32]
        L.orc_learned_logp.argtypes = [f64p, C.c_int64, C.c_int64, C.c_uint32, C.c_float]
        L.orc_learned_logp.restype = C.c_double
        L.orc_learned_proposals.argtypes = [f64p, C.c_uint32, C.c_float, C.c_uint64, C.c_uint32,
                                            i64p, u8p, f64p]
        L.orc_sweep_learned.argtypes = [p, f64p, C.c_float, C.c_uint64]
        L.orc_sweep_collect.argtypes = [p, C.c_uint64, f32p, f32p, C.c_uint64]
        L.orc_sweep_collect.restype = C.c_uint64
        _lib = L
    return _lib


NPARAM = 7060
Q = 2.0 ** -22


def geometry(N, eta, cell_min=2.0):
    L_, M, W, cap = C.c_double(), C.c_uint32(), C.c_int64(), C.c_uint32()
    rc = lib().orc_geometry(N, eta, cell_min, C.byref(L_), C.byref(M), C.byref(W), C.byref(cap))
    if rc != 0:
        raise ValueError("invalid geometry")
    return dict(L=L_.value, M=M.value, W=W.value, cap=cap.value, w=W.value * Q)


def philox(key, ctr):
    """Philox4x32-10 block: key = 64-bit int, ctr = 4 x uint32 -> 4 x uint32."""
    out = np.zeros(4, np.uint32)
    lib().orc_philox(key & 0xFFFFFFFF, (key >> 32) & 0xFFFFFFFF,
                     np.ascontiguousarray(ctr, dtype=np.uint32), out)
    return out


def hist_edges(K, dr):
    E = np.zeros(K + 1, np.float32)
    lib().orc_hist_edges(K, dr, E)
    return E


def pressure_fit(counts, dr, n_conf, N, L_eff, order=4):
    counts = np.ascontiguousarray(counts, dtype=np.int64)
    g, Z, P = C.c_double(), C.c_double(), C.c_double()
    coef = np.zeros(9, np.float64)
    rc = lib().orc_pressure(counts, len(counts), dr, order, n_conf, N, L_eff,
                            C.byref(g), C.byref(Z), C.byref(P), coef)
    if rc != 0:
        raise ValueError("pressure fit failed")
    return dict(g_contact=g.value, Z=Z.value, P_star=P.value, coef=coef[:order + 1])


def acf(series, maxlag):
    s = np.asarray(series, dtype=np.complex128)
    re = np.ascontiguousarray(s.real)
    im = np.ascontiguousarray(s.imag)
    out = np.zeros(maxlag + 1, np.float64)
    lib().orc_acf(re, im, len(s), maxlag, out)
    return out


def tau_fit(Cv, lo=0.05, hi=0.5):
    Cv = np.ascontiguousarray(Cv, dtype=np.float64)
    return lib().orc_tau_fit(Cv, len(Cv) - 1, lo, hi)


def tau_int(Cv, c=5.0):
    Cv = np.ascontiguousarray(Cv, dtype=np.float64)
    return lib().orc_tau_int(Cv, len(Cv) - 1, c)


def mlp_forward(params, f):
    out = np.zeros(20, np.float64)
    lib().orc_mlp_forward(np.ascontiguousarray(params, np.float64),
                          np.ascontiguousarray(f, np.float64), out)
    return out


def gmm_logpdf(out, dx, dy):
    return lib().orc_gmm_logpdf(np.ascontiguousarray(out, np.float64), dx, dy)


def nll_grad(params, F, D):
    F = np.ascontiguousarray(F, np.float64)
    D = np.ascontiguousarray(D, np.float64)
    g = np.zeros(NPARAM, np.float64)
    loss = lib().orc_nll_grad(np.ascontiguousarray(params, np.float64), F, D, F.shape[0], g)
    return loss, g


def adam(params, m, v, g, lr, t):
    lib().orc_adam(params, m, v, np.ascontiguousarray(g, np.float64), len(params), lr, t)


def learned_logp(out, Dx, Dy, step_m, eps):
    """ln P(D | out) of the learned proposal's lattice law."""
    return lib().orc_learned_logp(np.ascontiguousarray(out, np.float64), int(Dx), int(Dy),
                                  step_m, eps)


def learned_proposals(out, step_m, eps, seed, n):
    """n draws from the fixed output `out`: (D[n, 2] int64, drawn[n] bool,
    ln P(D)[n])."""
    D = np.zeros(2 * n, np.int64)
    drawn = np.zeros(n, np.uint8)
    lp = np.zeros(n, np.float64)
    lib().orc_learned_proposals(np.ascontiguousarray(out, np.float64), step_m, eps, seed, n, D,
                                drawn, lp)
    return D.reshape(n, 2), drawn.astype(bool), lp


class OracleBox:
    """One periodic box of N hard disks, advanced by the oracle's sweep."""

    def __init__(self, N, eta, seed=0, cell_min=2.0, lattice=1, step_m=26, n_trial=1,
                 _handle=None):
        if _handle is None:
            _handle = lib().orc_create(N, eta, seed, cell_min, lattice, step_m, n_trial)
            if not _handle:
                raise ValueError("invalid box parameters")
        self.h = _handle
        self.N = N
        self.eta = eta
        self.seed = seed

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_free(self.h)
            self.h = None

    def clone(self):
        return OracleBox(self.N, self.eta, self.seed, _handle=lib().orc_clone(self.h))

    def info(self):
        Le, ee, w = C.c_double(), C.c_double(), C.c_double()
        M, W, cap = C.c_uint32(), C.c_int64(), C.c_uint32()
        sw, Sx, Sy, tr, ac = C.c_uint64(), C.c_int64(), C.c_int64(), C.c_uint64(), C.c_uint64()
        lib().orc_info(self.h, C.byref(Le), C.byref(ee), C.byref(w), C.byref(M), C.byref(W),
                       C.byref(cap), C.byref(sw), C.byref(Sx), C.byref(Sy), C.byref(tr),
                       C.byref(ac))
        return dict(L_eff=Le.value, eta_eff=ee.value, w=w.value, M=M.value, W=W.value,
                    cap=cap.value, sweep=sw.value, Sx=Sx.value, Sy=Sy.value,
                    trials=tr.value, accepts=ac.value)

    def set_step(self, m):
        lib().orc_set_step(self.h, m)

    def set_positions_q(self, X, Y):
        rc = lib().orc_set_positions_q(self.h, np.ascontiguousarray(X, np.int64),
                                       np.ascontiguousarray(Y, np.int64))
        if rc != 0:
            raise ValueError("cell capacity exceeded")

    def sweep(self, k=1, cell_order=0):
        lib().orc_sweep(self.h, k, cell_order)

    def cells(self):
        i = self.info()
        nc = i["M"] ** 2
        cap = i["cap"]
        cnt = np.zeros(nc, np.uint8)
        tag = np.zeros(nc * cap, np.uint32)
        x = np.zeros(nc * cap, np.float32)
        y = np.zeros(nc * cap, np.float32)
        lib().orc_get_cells(self.h, cnt, tag, x, y)
        return cnt, tag.reshape(nc, cap), x.reshape(nc, cap), y.reshape(nc, cap)

    def positions_q(self):
        X = np.zeros(self.N, np.int64)
        Y = np.zeros(self.N, np.int64)
        lib().orc_get_positions_q(self.h, X, Y)
        return X, Y

    def positions(self):
        X, Y = self.positions_q()
        return X * Q, Y * Q

    def count_overlaps(self):
        return int(lib().orc_count_overlaps(self.h))

    def pair_hist(self, K, dr, counts=None):
        if counts is None:
            counts = np.zeros(K, np.int64)
        lib().orc_pair_hist(self.h, K, dr, counts)
        return counts

    def pair_hist_subset(self, sel, K, dr):
        counts = np.zeros(K, np.int64)
        lib().orc_pair_hist_subset(self.h, np.ascontiguousarray(sel, np.uint8), K, dr, counts)
        return counts

    def psi6(self, sel=None):
        re = np.zeros(self.N, np.float64)
        im = np.zeros(self.N, np.float64)
        if sel is None:
            lib().orc_psi6(self.h, None, re, im)
        else:
            sel = np.ascontiguousarray(sel, np.uint8)
            lib().orc_psi6(self.h, sel.ctypes.data_as(C.c_void_p), re, im)
        return re + 1j * im

    def psi6_field(self, psi):
        M = self.info()["M"]
        fre = np.zeros(M * M, np.float64)
        fim = np.zeros(M * M, np.float64)
        lib().orc_psi6_field(self.h, np.ascontiguousarray(psi.real), np.ascontiguousarray(psi.imag),
                             fre, fim)
        return fre + 1j * fim

    def structure_factor(self, hk):
        hk = np.ascontiguousarray(hk, np.int32).reshape(-1, 2)
        S = np.zeros(len(hk), np.float64)
        lib().orc_structure_factor(self.h, hk, len(hk), S)
        return S

    def chi(self, h, k):
        re = np.zeros(self.N, np.float64)
        im = np.zeros(self.N, np.float64)
        lib().orc_chi(self.h, h, k, re, im)
        return re + 1j * im

    def cq(self, qx, qy, dr, B):
        """Sums of cos(q.d) and pair counts per window r_b = b dr."""
        num = np.zeros(B, np.float64)
        cnt = np.zeros(B, np.int64)
        if lib().orc_cq(self.h, qx, qy, dr, B, num, cnt) != 0:
            raise ValueError("bins out of range")
        return num, cnt

    def sweep_learned(self, params, eps, k=1):
        lib().orc_sweep_learned(self.h, np.ascontiguousarray(params, np.float64), eps, k)

    def sweep_collect(self, k, cap):
        """k plain sweeps recording accepted moves: (F[n, 24], D[n, 2], total)."""
        F = np.zeros(cap * 24, np.float32)
        D = np.zeros(cap * 2, np.float32)
        tot = int(lib().orc_sweep_collect(self.h, k, F, D, cap))
        n = min(tot, cap)
        return F.reshape(cap, 24)[:n], D.reshape(cap, 2)[:n], tot

    def features(self, cell, self_tag, x, y):
        f = np.zeros(24, np.float32)
        n = lib().orc_features(self.h, cell, self_tag, x, y, f)
        return f, n
