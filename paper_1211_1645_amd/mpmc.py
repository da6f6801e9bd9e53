"""Python binding of the MI355X MPMC hard-disk library (libmpmc.so).

Argument marshalling only: every step of the sampler and of the observables
runs inside the HIP library.  PyTorch supplies the stream (and optionally the
caching allocator) for device work.  There is no fallback: if the library is
not built, every call raises.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpmc.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, EOVERFLOW, EIO = 0, -1, -2, -3, -4, -5, -6
LATTICE = {"square": 0, "triangular": 1, "none": 2}
SCHEDULE = {"auto": 0, "simple": 1, "fused": 2}
Q = 2.0 ** -22

_alloc_t = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_free_t = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Params(C.Structure):
    _fields_ = [("step_m", C.c_uint32), ("n_trial", C.c_uint32), ("lattice", C.c_int32),
                ("cell_min", C.c_double), ("hist_dr", C.c_double), ("hist_bins", C.c_uint32),
                ("fit_order", C.c_uint32), ("hist_block", C.c_uint32), ("schedule", C.c_uint32),
                ("tile", C.c_uint32), ("stream", C.c_void_p), ("alloc", _alloc_t),
                ("free", _free_t), ("alloc_ctx", C.c_void_p)]


class Info(C.Structure):
    _fields_ = [("N", C.c_uint32), ("M", C.c_uint32), ("cap", C.c_uint32), ("n_trial", C.c_uint32),
                ("step_m", C.c_uint32), ("tile", C.c_uint32), ("schedule", C.c_uint32),
                ("hist_bins", C.c_uint32), ("W", C.c_int64), ("L", C.c_double),
                ("L_eff", C.c_double), ("w", C.c_double), ("eta", C.c_double),
                ("eta_eff", C.c_double), ("hist_dr", C.c_double), ("sweep", C.c_uint64),
                ("Sx", C.c_int64), ("Sy", C.c_int64), ("trials", C.c_uint64),
                ("accepts", C.c_uint64), ("n_conf", C.c_uint64)]


class EosLoop(C.Structure):
    _fields_ = [(f, C.c_double) for f in ("eta_max", "p_max", "eta_min", "p_min", "p_coex",
                                          "eta_liquid", "eta_solid", "delta_f")]


class MPMCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("MPMC error %d: %s" % (code, msg))
        self.code = code


_lib = None

# name -> (restype, argtypes); every function declared in include/mpmc.h
_P = C.c_void_p
_SIGS = {
    "mpmc_default_params": [C.POINTER(Params)],
    "mpmc_init_box": [C.POINTER(C.c_void_p), C.c_uint32, C.c_double, C.c_uint64, C.POINTER(Params)],
    "mpmc_free_box": [_P],
    "mpmc_set_positions": [_P, _P, _P],
    "mpmc_set_step": [_P, C.c_uint32],
    "mpmc_sweep": [_P, C.c_uint64, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)],
    "mpmc_accumulate_contacts": [_P],
    "mpmc_reset_contacts": [_P],
    "mpmc_get_contacts": [_P, _P, C.POINTER(C.c_uint64)],
    "mpmc_measure_pressure": [_P, C.POINTER(C.c_double), C.POINTER(C.c_double),
                              C.POINTER(C.c_double), C.POINTER(C.c_double)],
    "mpmc_contact_hist_subset": [_P, _P, _P],
    "mpmc_psi6_field": [_P, _P, _P, _P, _P, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int],
    "mpmc_get_positions": [_P, _P, _P, _P, _P],
    "mpmc_measure_async": [_P, _P, C.c_int],
    "mpmc_measure_wait": [_P, C.POINTER(C.c_uint32)],
    "mpmc_structure_factor": [_P, _P, C.c_uint32, _P],
    "mpmc_structure_factor_noalloc": [_P, _P, C.c_uint32, _P],
    "mpmc_find_q0": [_P, C.c_double, C.c_double, C.c_double, C.c_double, C.POINTER(C.c_int32),
                     C.POINTER(C.c_int32), C.POINTER(C.c_double)],
    "mpmc_chi_field": [_P, C.c_int32, C.c_int32, _P, _P, _P, _P, C.c_int],
    "mpmc_cq": [_P, C.c_double, C.c_double, C.c_double, C.c_uint32, _P, _P],
    "mpmc_cq_aligned": [_P, C.c_double, C.c_double, C.c_double, C.c_double, C.c_uint32, _P, _P,
                        C.POINTER(C.c_double)],
    "mpmc_cq_bin_max": [_P, C.c_uint32, C.c_uint32, _P],
    "mpmc_eos_loop": [_P, _P, _P, C.c_uint32, C.c_uint32, C.POINTER(EosLoop)],
    "mpmc_power_law": [_P, _P, C.c_uint32, C.POINTER(C.c_double), C.POINTER(C.c_double)],
    "mpmc_get_cells": [_P, _P, _P, _P, _P],
    "mpmc_get_info": [_P, C.POINTER(Info)],
    "mpmc_validate": [_P, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)],
    "mpmc_save": [_P, C.c_char_p],
    "mpmc_load": [C.POINTER(C.c_void_p), C.c_char_p, C.POINTER(Params)],
    "mpmc_acf": [_P, _P, C.c_uint32, C.c_uint32, _P],
    "mpmc_tau": [_P, C.c_uint32, C.c_double, C.c_double, C.POINTER(C.c_double),
                 C.POINTER(C.c_double)],
    "mpmc_set_schedule": [_P, C.c_uint32, C.c_uint32, C.c_uint32],
    "mpmc_set_graphs": [_P, C.c_uint32],
    "mpmc_set_learned_cells_per_wave": [_P, C.c_uint32],
    "mpmc_profile_phases": [_P, C.c_uint32, _P],
    "mpmc_batch_create": [C.POINTER(C.c_void_p), C.c_uint32, _P, _P, _P, C.POINTER(Params)],
    "mpmc_batch_free": [_P],
    "mpmc_batch_sweep": [_P, C.c_uint64, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)],
    "mpmc_batch_box": [_P, C.c_uint32, C.POINTER(C.c_void_p)],
    "mpmc_batch_accumulate_contacts": [_P],
    "mpmc_batch_measure_pressure": [_P, _P, _P],
    "mpmc_batch_set_schedule": [_P, C.c_uint32, C.c_uint32],
    "mpmc_batch_info": [_P, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                        C.POINTER(C.c_uint32)],
    "mpmc_batch_set_graphs": [_P, C.c_uint32],
    "mpmc_learner_create": [C.POINTER(C.c_void_p), C.c_uint64, C.c_uint64, _P],
    "mpmc_learner_free": [_P],
    "mpmc_learner_set_params": [_P, _P],
    "mpmc_learner_get_params": [_P, _P],
    "mpmc_learner_collect": [_P, _P, C.c_uint64, C.POINTER(C.c_uint64)],
    "mpmc_learner_train": [_P, C.c_uint32, C.c_uint32, C.c_float, C.POINTER(C.c_double)],
    "mpmc_learner_forward": [_P, _P, C.c_uint32, _P],
    "mpmc_learner_nll_grad": [_P, _P, _P, C.c_uint32, _P, C.POINTER(C.c_double)],
    "mpmc_learner_info": [_P, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.POINTER(C.c_uint32)],
    "mpmc_learned_features": [_P, _P, C.c_uint32, _P],
    "mpmc_sweep_learned": [_P, _P, C.c_uint64, C.c_float, C.POINTER(C.c_uint64),
                           C.POINTER(C.c_uint64)],
    "mpmc_profile_learned": [_P, _P, C.c_uint32, C.c_float, _P],
    "mpmc_learned_propose": [_P, C.c_uint32, C.c_float, C.c_uint64, C.c_uint32, _P, _P, _P],
    "mpmc_learned_logp": [_P, _P, C.c_uint32, C.c_uint32, C.c_float, _P],
    "mpmc_learner_moves": [_P, C.c_uint64, C.c_uint64, _P, _P],
    "mpmc_learner_adam_step": [_P, _P, C.c_float],
}


def load():
    """Loads libmpmc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libmpmc.so is not built (run __graft_entry__.build() or "
                           "python paper_1211_1645_amd/build.py); there is no fallback")
    lib = C.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.mpmc_last_error.restype = C.c_char_p
    lib.mpmc_last_error.argtypes = []
    _lib = lib
    return lib


def _check(rc):
    if rc != OK:
        raise MPMCError(rc, _lib.mpmc_last_error().decode())


def _ptr(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


def _current_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except ImportError:
        pass
    return None


class _TorchAllocator:
    """Device memory from torch's caching allocator, through the ABI hook."""

    def __init__(self, stream):
        import torch
        self.torch = torch
        self.stream = stream
        self.a = _alloc_t(self._alloc)
        self.f = _free_t(self._free)

    def _alloc(self, nbytes, ctx):
        try:
            return self.torch.cuda.caching_allocator_alloc(int(nbytes), stream=self.stream)
        except Exception:
            return None

    def _free(self, ptr, ctx):
        self.torch.cuda.caching_allocator_delete(ptr)


class Box:
    """N hard disks in a periodic square box, sampled by MPMC on the GPU."""

    def __init__(self, N, eta, seed=0, step_m=26, n_trial=1, lattice="triangular", cell_min=2.0,
                 hist_dr=1e-3, hist_bins=100, fit_order=4, hist_block=0, schedule="auto",
                 tile=0, stream=None, torch_allocator=False, _handle=None):
        lib = load()
        self._alloc = None
        if _handle is None:
            p = self._params(step_m, n_trial, lattice, cell_min, hist_dr, hist_bins, fit_order,
                             hist_block, schedule, tile, stream, torch_allocator)
            h = C.c_void_p()
            _check(lib.mpmc_init_box(C.byref(h), N, eta, seed, C.byref(p)))
            _handle = h
        self.h = _handle
        i = self.info()
        self.N, self.M, self.cap = i["N"], i["M"], i["cap"]

    def _params(self, step_m=26, n_trial=1, lattice="triangular", cell_min=2.0, hist_dr=1e-3,
                hist_bins=100, fit_order=4, hist_block=0, schedule="auto", tile=0, stream=None,
                torch_allocator=False):
        p = Params()
        _check(load().mpmc_default_params(C.byref(p)))
        p.step_m, p.n_trial = step_m, n_trial
        p.lattice = LATTICE[lattice] if isinstance(lattice, str) else lattice
        p.cell_min, p.hist_dr, p.hist_bins, p.fit_order = cell_min, hist_dr, hist_bins, fit_order
        p.hist_block = hist_block
        p.schedule = SCHEDULE[schedule] if isinstance(schedule, str) else schedule
        p.tile = tile
        st = stream if stream is not None else _current_stream()
        p.stream = st
        if torch_allocator:
            self._alloc = _TorchAllocator(st)
            p.alloc, p.free = self._alloc.a, self._alloc.f
        return p

    @classmethod
    def load(cls, path, stream=None, schedule="auto"):
        lib = load()
        b = cls.__new__(cls)
        b._alloc = None
        p = b._params(schedule=schedule, stream=stream)
        h = C.c_void_p()
        _check(lib.mpmc_load(C.byref(h), path.encode(), C.byref(p)))
        cls.__init__(b, 0, 0.0, _handle=h)
        return b

    @classmethod
    def _borrowed(cls, handle, owner):
        b = cls.__new__(cls)
        b._alloc = None
        b._owner = owner  # keeps the batch alive while the view exists
        cls.__init__(b, 0, 0.0, _handle=handle)
        return b

    def close(self):
        if getattr(self, "_owner", None) is not None:
            self.h = None
            return
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.mpmc_free_box(self.h)
            self.h = None

    def __del__(self):
        self.close()

    # ---- sampling ---------------------------------------------------------
    def sweep(self, k=1, counts=False):
        if counts:
            t, a = C.c_uint64(), C.c_uint64()
            _check(_lib.mpmc_sweep(self.h, k, C.byref(t), C.byref(a)))
            return t.value, a.value
        _check(_lib.mpmc_sweep(self.h, k, None, None))
        return None

    def set_step(self, m):
        _check(_lib.mpmc_set_step(self.h, m))

    def set_positions_q(self, X, Y):
        X = np.ascontiguousarray(X, np.int64)
        Y = np.ascontiguousarray(Y, np.int64)
        _check(_lib.mpmc_set_positions(self.h, _ptr(X), _ptr(Y)))

    def set_schedule(self, schedule, tile=0, threads=0):
        s = SCHEDULE[schedule] if isinstance(schedule, str) else schedule
        _check(_lib.mpmc_set_schedule(self.h, s, tile, threads))

    def set_graphs(self, sweeps_per_graph):
        _check(_lib.mpmc_set_graphs(self.h, sweeps_per_graph))

    def set_learned_cells_per_wave(self, cells):
        """Active cells per wave of the learned pass (16, 32, 64; 0 = by box size)."""
        _check(_lib.mpmc_set_learned_cells_per_wave(self.h, cells))

    PHASES = ("load", "pass1", "pass2", "pass3", "pass4", "rebin_classes", "rebin_scatter",
              "tile", "entry_to_work", "launch_span", "tiles_in_flight", "last_entry")

    def profile_phases(self, sweeps=20):
        """Mean microseconds per tile of each phase of the fused sweep
        kernel, and per launch its span, mean tiles in flight and the time
        to its last workgroup's entry (the box advances by `sweeps`
        sweeps)."""
        out = np.zeros(12, np.float64)
        _check(_lib.mpmc_profile_phases(self.h, sweeps, _ptr(out)))
        return dict(zip(self.PHASES, out.tolist()))

    # ---- observables --------------------------------------------------------
    def accumulate_contacts(self):
        _check(_lib.mpmc_accumulate_contacts(self.h))

    def reset_contacts(self):
        _check(_lib.mpmc_reset_contacts(self.h))

    def contacts(self):
        K = self.info()["hist_bins"]
        c = np.zeros(K, np.int64)
        n = C.c_uint64()
        _check(_lib.mpmc_get_contacts(self.h, _ptr(c), C.byref(n)))
        return c, n.value

    def measure_pressure(self):
        P, g, Z, se = C.c_double(), C.c_double(), C.c_double(), C.c_double()
        _check(_lib.mpmc_measure_pressure(self.h, C.byref(P), C.byref(g), C.byref(Z), C.byref(se)))
        return dict(P_star=P.value, g_contact=g.value, Z=Z.value, se=se.value)

    def contact_hist_subset(self, sel):
        K = self.info()["hist_bins"]
        sel = np.ascontiguousarray(sel, np.uint8)
        c = np.zeros(K, np.int64)
        _check(_lib.mpmc_contact_hist_subset(self.h, _ptr(sel), _ptr(c)))
        return c

    def psi6_field(self, device=False):
        """Returns (psi_j by tag, field per cell, Psi_6)."""
        r, i = C.c_double(), C.c_double()
        if device:
            import torch
            re = torch.empty(self.N, dtype=torch.float32, device="cuda")
            im = torch.empty(self.N, dtype=torch.float32, device="cuda")
            fre = torch.empty(self.M * self.M, dtype=torch.float32, device="cuda")
            fim = torch.empty(self.M * self.M, dtype=torch.float32, device="cuda")
            _check(_lib.mpmc_psi6_field(self.h, C.c_void_p(re.data_ptr()), C.c_void_p(im.data_ptr()),
                                        C.c_void_p(fre.data_ptr()), C.c_void_p(fim.data_ptr()),
                                        C.byref(r), C.byref(i), 1))
            return torch.complex(re, im), torch.complex(fre, fim), complex(r.value, i.value)
        re = np.zeros(self.N, np.float32)
        im = np.zeros(self.N, np.float32)
        fre = np.zeros(self.M * self.M, np.float32)
        fim = np.zeros(self.M * self.M, np.float32)
        _check(_lib.mpmc_psi6_field(self.h, _ptr(re), _ptr(im), _ptr(fre), _ptr(fim), C.byref(r),
                                    C.byref(i), 0))
        return re + 1j * im.astype(np.complex64), fre + 1j * fim.astype(np.complex64), \
            complex(r.value, i.value)

    def psi6(self):
        """Global Psi_6 only (Sec. III)."""
        r, i = C.c_double(), C.c_double()
        _check(_lib.mpmc_psi6_field(self.h, None, None, None, None, C.byref(r), C.byref(i), 0))
        return complex(r.value, i.value)

    def measure_async(self, psi_out=None, field=False):
        """Contact histogram and psi_6 on the box's measurement stream,
        overlapping the next sweeps; psi_out: a float64 CUDA tensor of two
        elements that receives Psi_6 (re, im)."""
        ptr = None
        if psi_out is not None:
            assert psi_out.is_cuda and psi_out.dtype.is_floating_point and psi_out.numel() >= 2
            assert psi_out.element_size() == 8 and psi_out.is_contiguous()
            ptr = C.c_void_p(psi_out.data_ptr())
        _check(_lib.mpmc_measure_async(self.h, ptr, 1 if field else 0))

    def measure_wait(self):
        """Waits for the asynchronous measurements; True if a neighbour
        search among them was too short."""
        f = C.c_uint32()
        _check(_lib.mpmc_measure_wait(self.h, C.byref(f)))
        return bool(f.value)

    # ---- positional order (Sec. IV.C: S(q), q0, chi; Sec. IV.D: C_q(r)) -----
    def wave_vector(self, h, k):
        """(qx, qy) = (2 pi / L_eff)(h, k) in 1/sigma."""
        u = 2.0 * np.pi / self.info()["L_eff"]
        return u * h, u * k

    def structure_factor(self, hk):
        """S(q) at the allowed wave vectors given as integer pairs (h, k)."""
        hk = np.ascontiguousarray(np.asarray(hk, np.int32).reshape(-1, 2))
        S = np.zeros(len(hk), np.float64)
        _check(_lib.mpmc_structure_factor(self.h, _ptr(hk), len(hk), _ptr(S)))
        return S

    def structure_factor_noalloc(self, hk, S):
        """S(q) into the float64 CUDA tensor S for the int32 CUDA tensor hk
        of (h, k) pairs, with no device allocation; enqueued on the box's
        stream."""
        assert hk.is_cuda and S.is_cuda and hk.is_contiguous() and S.is_contiguous()
        assert hk.element_size() == 4 and S.element_size() == 8 and S.dtype.is_floating_point
        nq = hk.numel() // 2
        assert S.numel() >= nq
        _check(_lib.mpmc_structure_factor_noalloc(self.h, C.c_void_p(hk.data_ptr()), nq,
                                                  C.c_void_p(S.data_ptr())))

    def find_q0(self, q_lo, q_hi, theta0=0.0, dtheta=2.0 * np.pi):
        """The allowed wave vector of largest S in the window; (h, k, S)."""
        h, k, S = C.c_int32(), C.c_int32(), C.c_double()
        _check(_lib.mpmc_find_q0(self.h, q_lo, q_hi, theta0, dtheta, C.byref(h), C.byref(k),
                                 C.byref(S)))
        return h.value, k.value, S.value

    def chi_field(self, h, k):
        """chi_j = exp(i q0.x_j) by tag and its field per cell (3 x 3 mean)."""
        nc = self.M * self.M
        re, im = np.zeros(self.N, np.float32), np.zeros(self.N, np.float32)
        fre, fim = np.zeros(nc, np.float32), np.zeros(nc, np.float32)
        _check(_lib.mpmc_chi_field(self.h, h, k, _ptr(re), _ptr(im), _ptr(fre), _ptr(fim), 0))
        return re + 1j * im.astype(np.complex64), fre + 1j * fim.astype(np.complex64)

    def cq(self, qx, qy, dr, nbins, num=None, cnt=None):
        """Adds this configuration's window sums of cos(q.d) and pair counts
        into (num, cnt) (new zero arrays when None) and returns them;
        C_q(r_b) = num / cnt at r_b = b dr."""
        num = np.zeros(nbins, np.float64) if num is None else num
        cnt = np.zeros(nbins, np.int64) if cnt is None else cnt
        assert num.dtype == np.float64 and cnt.dtype == np.int64
        assert num.flags.c_contiguous and cnt.flags.c_contiguous
        assert len(num) == nbins and len(cnt) == nbins
        _check(_lib.mpmc_cq(self.h, qx, qy, dr, nbins, _ptr(num), _ptr(cnt)))
        return num, cnt

    def cq_aligned(self, qx, qy, psi_arg_ref, dr, nbins, num=None, cnt=None):
        """cq with q turned by the change of arg Psi_6 / 6 from psi_arg_ref;
        returns (num, cnt, angle)."""
        num = np.zeros(nbins, np.float64) if num is None else num
        cnt = np.zeros(nbins, np.int64) if cnt is None else cnt
        assert num.dtype == np.float64 and cnt.dtype == np.int64
        assert num.flags.c_contiguous and cnt.flags.c_contiguous
        assert len(num) == nbins and len(cnt) == nbins
        a = C.c_double()
        _check(_lib.mpmc_cq_aligned(self.h, qx, qy, psi_arg_ref, dr, nbins, _ptr(num), _ptr(cnt),
                                    C.byref(a)))
        return num, cnt, a.value

    # ---- state ------------------------------------------------------------
    def info(self):
        i = Info()
        _check(_lib.mpmc_get_info(self.h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in Info._fields_}

    def positions_q(self):
        X = np.zeros(self.N, np.int64)
        Y = np.zeros(self.N, np.int64)
        _check(_lib.mpmc_get_positions(self.h, None, None, _ptr(X), _ptr(Y)))
        return X, Y

    def positions(self):
        x = np.zeros(self.N, np.float64)
        y = np.zeros(self.N, np.float64)
        _check(_lib.mpmc_get_positions(self.h, _ptr(x), _ptr(y), None, None))
        return x, y

    def cells(self):
        nc = self.M * self.M
        cnt = np.zeros(nc, np.uint8)
        tag = np.zeros(nc * self.cap, np.uint32)
        x = np.zeros(nc * self.cap, np.float32)
        y = np.zeros(nc * self.cap, np.float32)
        _check(_lib.mpmc_get_cells(self.h, _ptr(cnt), _ptr(tag), _ptr(x), _ptr(y)))
        return cnt, tag.reshape(nc, self.cap), x.reshape(nc, self.cap), y.reshape(nc, self.cap)

    def validate(self):
        o, b = C.c_uint64(), C.c_uint64()
        _check(_lib.mpmc_validate(self.h, C.byref(o), C.byref(b)))
        return o.value, b.value

    def save(self, path):
        _check(_lib.mpmc_save(self.h, path.encode()))


class Batch:
    """Independent boxes (lists N, eta, seed) swept together, one persistent
    launch per sweep."""

    def __init__(self, N, eta, seed, step_m=26, n_trial=1, lattice="triangular", cell_min=2.0,
                 hist_dr=1e-3, hist_bins=100, fit_order=4, hist_block=0, schedule="auto", tile=0,
                 stream=None):
        lib = load()
        N = np.ascontiguousarray(N, np.uint32)
        eta = np.ascontiguousarray(eta, np.float64)
        seed = np.ascontiguousarray(seed, np.uint64)
        assert len(N) == len(eta) == len(seed)
        p = Box._params(self, step_m, n_trial, lattice, cell_min, hist_dr, hist_bins, fit_order,
                        hist_block, schedule, tile, stream, False)
        h = C.c_void_p()
        _check(lib.mpmc_batch_create(C.byref(h), len(N), _ptr(N), _ptr(eta), _ptr(seed), C.byref(p)))
        self.h = h
        self.n = len(N)

    def close(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.mpmc_batch_free(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def sweep(self, k=1, counts=False):
        if counts:
            t, a = C.c_uint64(), C.c_uint64()
            _check(_lib.mpmc_batch_sweep(self.h, k, C.byref(t), C.byref(a)))
            return t.value, a.value
        _check(_lib.mpmc_batch_sweep(self.h, k, None, None))

    def box(self, i):
        h = C.c_void_p()
        _check(_lib.mpmc_batch_box(self.h, i, C.byref(h)))
        return Box._borrowed(h, self)

    def accumulate_contacts(self):
        _check(_lib.mpmc_batch_accumulate_contacts(self.h))

    def measure_pressure(self):
        P = np.zeros(self.n, np.float64)
        se = np.zeros(self.n, np.float64)
        _check(_lib.mpmc_batch_measure_pressure(self.h, _ptr(P), _ptr(se)))
        return P, se

    def set_schedule(self, tile=0, threads=0):
        _check(_lib.mpmc_batch_set_schedule(self.h, tile, threads))

    def set_graphs(self, sweeps_per_graph):
        _check(_lib.mpmc_batch_set_graphs(self.h, sweeps_per_graph))

    def info(self):
        n, t, th, it = C.c_uint32(), C.c_uint32(), C.c_uint32(), C.c_uint32()
        _check(_lib.mpmc_batch_info(self.h, C.byref(n), C.byref(t), C.byref(th), C.byref(it)))
        return dict(nbox=n.value, tile=t.value, threads=th.value, n_items=it.value)


MLP_PARAMS = 7060


class Learner:
    """The learned proposal: network parameters, recorded moves, training."""

    def __init__(self, seed=0, capacity=1 << 20, stream=None):
        lib = load()
        h = C.c_void_p()
        st = stream if stream is not None else _current_stream()
        _check(lib.mpmc_learner_create(C.byref(h), seed, capacity, st))
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.mpmc_learner_free(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def params(self):
        p = np.zeros(MLP_PARAMS, np.float32)
        _check(_lib.mpmc_learner_get_params(self.h, _ptr(p)))
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, np.float32)
        assert p.size == MLP_PARAMS
        _check(_lib.mpmc_learner_set_params(self.h, _ptr(p)))

    def collect(self, box, sweeps):
        n = C.c_uint64()
        _check(_lib.mpmc_learner_collect(self.h, box.h, sweeps, C.byref(n)))
        return n.value

    def train(self, steps, batch=4096, lr=1e-3):
        loss = C.c_double()
        _check(_lib.mpmc_learner_train(self.h, steps, batch, lr, C.byref(loss)))
        return loss.value

    def forward(self, F):
        F = np.ascontiguousarray(F, np.float32)
        out = np.zeros((F.shape[0], 20), np.float32)
        _check(_lib.mpmc_learner_forward(self.h, _ptr(F), F.shape[0], _ptr(out)))
        return out

    def nll_grad(self, F, D):
        F = np.ascontiguousarray(F, np.float32)
        D = np.ascontiguousarray(D, np.float32)
        g = np.zeros(MLP_PARAMS, np.float32)
        loss = C.c_double()
        _check(_lib.mpmc_learner_nll_grad(self.h, _ptr(F), _ptr(D), F.shape[0], _ptr(g), C.byref(loss)))
        return loss.value, g

    def moves(self, first=0, n=None):
        """Recorded moves first..first+n-1: (F[n, 24], D[n, 2])."""
        if n is None:
            n = self.info()["n_data"] - first
        F = np.zeros((n, 24), np.float32)
        D = np.zeros((n, 2), np.float32)
        _check(_lib.mpmc_learner_moves(self.h, first, n, _ptr(F), _ptr(D)))
        return F, D

    def adam_step(self, grad, lr):
        """One Adam step with the given gradient (diagnostic)."""
        g = np.ascontiguousarray(grad, np.float32)
        assert g.size == MLP_PARAMS
        _check(_lib.mpmc_learner_adam_step(self.h, _ptr(g), lr))

    def info(self):
        n, o, s = C.c_uint64(), C.c_uint64(), C.c_uint32()
        _check(_lib.mpmc_learner_info(self.h, C.byref(n), C.byref(o), C.byref(s)))
        return dict(n_data=n.value, feature_overflow=o.value, steps=s.value)


def learned_features(box, tags):
    tags = np.ascontiguousarray(tags, np.uint32)
    F = np.zeros((len(tags), 24), np.float32)
    _check(load().mpmc_learned_features(box.h, _ptr(tags), len(tags), _ptr(F)))
    return F


def sweep_learned(box, learner, k=1, eps=0.1, counts=False):
    t, a = C.c_uint64(), C.c_uint64()
    _check(load().mpmc_sweep_learned(box.h, learner.h, k, eps, C.byref(t) if counts else None,
                                     C.byref(a) if counts else None))
    return (t.value, a.value) if counts else None


LEARN_PHASES = ("start", "features", "network", "draw", "overlap", "features_rev", "network_rev",
                "accept", "count")


def profile_learned(box, learner, sweeps=5, eps=0.1):
    """Mean microseconds per wave and colour pass of each phase of the
    learned pass (the box advances by `sweeps` learned sweeps)."""
    out = np.zeros(9, np.float64)
    _check(load().mpmc_profile_learned(box.h, learner.h, sweeps, eps, _ptr(out)))
    return dict(zip(LEARN_PHASES, out.tolist()))


def learned_propose(out, step_m, eps, seed, n):
    """n draws of the learned proposal's lattice law from one fixed network
    output: (D[n, 2] int32, drawn[n] bool, ln P(D)[n])."""
    o = np.ascontiguousarray(out, np.float32)
    assert o.size == 20
    D = np.zeros((n, 2), np.int32)
    drawn = np.zeros(n, np.uint8)
    lp = np.zeros(n, np.float64)
    _check(load().mpmc_learned_propose(_ptr(o), step_m, eps, seed, n, _ptr(D), _ptr(drawn),
                                       _ptr(lp)))
    return D, drawn.astype(bool), lp


def learned_logp(outs, D, step_m, eps):
    """ln P(D_i | out_i) of the lattice law for outs[n, 20], D[n, 2]."""
    o = np.ascontiguousarray(outs, np.float32).reshape(-1, 20)
    d = np.ascontiguousarray(D, np.int32).reshape(-1, 2)
    assert len(o) == len(d)
    lp = np.zeros(len(o), np.float64)
    _check(load().mpmc_learned_logp(_ptr(o), _ptr(d), len(o), step_m, eps, _ptr(lp)))
    return lp


def cq_bin_max(Cv, width):
    """Maxima of C over groups of `width` consecutive windows."""
    load()
    Cv = np.ascontiguousarray(Cv, np.float64)
    out = np.zeros((len(Cv) + width - 1) // width, np.float64)
    _check(_lib.mpmc_cq_bin_max(_ptr(Cv), len(Cv), width, _ptr(out)))
    return out


def eos_loop(eta, p_star, se=None, order=3):
    """Mayer-Wood loop analysis of an equation of state (Sec. IV.A): dict of
    the extrema, Maxwell pressure, coexisting densities and beta Delta f."""
    load()
    eta = np.ascontiguousarray(eta, np.float64)
    p = np.ascontiguousarray(p_star, np.float64)
    assert eta.shape == p.shape
    s = None if se is None else np.ascontiguousarray(se, np.float64)
    r = EosLoop()
    _check(_lib.mpmc_eos_loop(_ptr(eta), _ptr(p), None if s is None else _ptr(s), len(eta), order,
                              C.byref(r)))
    return {f: getattr(r, f) for f, _ in EosLoop._fields_}


def power_law(x, y):
    """(exponent, prefactor) of y = a x^b by least squares on logarithms."""
    load()
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    b, a = C.c_double(), C.c_double()
    _check(_lib.mpmc_power_law(_ptr(x), _ptr(y), len(x), C.byref(b), C.byref(a)))
    return b.value, a.value


def acf(series, maxlag):
    """C(dt) of Eq. (9) computed by the library's host analysis."""
    load()
    s = np.asarray(series, np.complex128)
    re, im = np.ascontiguousarray(s.real), np.ascontiguousarray(s.imag)
    out = np.zeros(maxlag + 1, np.float64)
    _check(_lib.mpmc_acf(_ptr(re), _ptr(im), len(s), maxlag, _ptr(out)))
    return out


def tau(Cv, lo=0.05, hi=0.5):
    """(tau from the exponential tail, integrated tau)."""
    load()
    Cv = np.ascontiguousarray(Cv, np.float64)
    t, ti = C.c_double(), C.c_double()
    _check(_lib.mpmc_tau(_ptr(Cv), len(Cv) - 1, lo, hi, C.byref(t), C.byref(ti)))
    return t.value, ti.value
