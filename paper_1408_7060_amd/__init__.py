"""MI355X ET-AIM marching library: Python binding of include/etaim.h.

Arguments are marshalled to the C ABI of libetaim.so; every step of the
method runs in the library's HIP kernels.  torch supplies device memory and
the stream.  The library must have been built (``python -m
paper_1408_7060_amd.build``); there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
from ctypes import POINTER, byref, c_double, c_int32, c_size_t, c_void_p

import numpy as np

from . import _lib
from ._lib import BLIF, CFIE, CPPIF, EFIE, FP32, FP64, EtaimError, Stats

__all__ = ["Problem", "EtaimMarch", "EtaimError", "FP32", "FP64", "EFIE", "CFIE", "CPPIF", "BLIF"]


def _torch():
    import torch
    return torch


def _dptr(t) -> int:
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return t.data_ptr()


def _stats_dict(st: Stats, iters) -> dict:
    d = {f: getattr(st, f) for f, _ in Stats._fields_ if f != "iters_per_step"}
    d["iters_per_step"] = iters
    return d


class Problem:
    """One ET-AIM problem on the current HIP device (etaim_create)."""

    def __init__(self, xyz, tri, rwg, *, fc: float, nt: int, grid, d_near: float, dt: float = 0.0,
                 beta: float = 0.0, f_bw: float = 0.0, ng: int = 0, precision: int = FP64, batch: int = 1,
                 tol: float = 1e-6, restart: int = 50, maxit: int = 1000, flags: int = 0, sync_every: int = 1,
                 alpha: float = 1.0, basis: int = 0, nsamp: int = 0, nomega: int = 0, stream=None):
        torch = _torch()
        lib = _lib.load()
        self._xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self._tri = np.ascontiguousarray(tri, dtype=np.int32)
        self._rwg = np.ascontiguousarray(rwg, dtype=np.int32)
        mesh = _lib.Mesh(len(self._xyz), self._xyz.ctypes.data_as(POINTER(c_double)), len(self._tri),
                         self._tri.ctypes.data_as(POINTER(c_int32)))
        r = _lib.Rwg(len(self._rwg), self._rwg.ctypes.data_as(POINTER(c_int32)))
        g = np.broadcast_to(np.asarray(grid, dtype=np.int32), (3,))
        p = _lib.Params(fc=fc, dt=dt, beta=beta, f_bw=f_bw, nt_steps=nt, order=3,
                        grid=(c_int32 * 3)(*[int(v) for v in g]), d_near=d_near, ng=ng, precision=precision,
                        batch=batch, tol=tol, restart=restart, maxit=maxit, flags=flags,
                        sync_every=sync_every, formulation=EFIE if alpha == 1.0 else CFIE,
                        alpha=alpha, basis=basis, nsamp=nsamp, nomega=nomega)
        if stream is None and torch.cuda.is_available():
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = c_void_p()
        _lib.check(lib.etaim_create(byref(h), byref(mesh), byref(r), byref(p),
                                    c_void_p(stream.cuda_stream if stream is not None else 0)))
        self._h = h
        self.nt, self.batch = nt, batch
        self.info = self.describe()
        self.ns = self.info["ns"]

    # -- helpers
    def _dev(self):
        return _torch().device("cuda", _torch().cuda.current_device())

    def empty(self, *shape):
        return _torch().empty(shape, dtype=_torch().complex128, device=self._dev())

    def describe(self) -> dict:
        d = _lib.Derived()
        _lib.check(_lib.load().etaim_describe(self._h, byref(d)))
        out = {}
        for f, _ in _lib.Derived._fields_:
            v = getattr(d, f)
            out[f] = list(v) if hasattr(v, "__len__") else v
        return out

    def excitation(self, khat, phat, sigma: float, td: float, out=None, noalloc: bool = False):
        """Excitation vectors V [N_t][B][ns] of the plane wave of eq. (1);
        noalloc selects etaim_excitation_planewave_noalloc (no device
        allocation inside the library; out may then be a preallocated V)."""
        kh = np.ascontiguousarray(np.atleast_2d(khat), dtype=np.float64)
        ph = np.ascontiguousarray(np.atleast_2d(phat), dtype=np.float64)
        V = out if out is not None else self.empty(self.nt, len(kh), self.ns)
        fn = _lib.load().etaim_excitation_planewave_noalloc if noalloc else _lib.load().etaim_excitation_planewave
        _lib.check(fn(self._h, len(kh), kh.ctypes.data_as(POINTER(c_double)), ph.ctypes.data_as(POINTER(c_double)),
                      sigma, td, c_void_p(_dptr(V))))
        return V

    def march(self, V, out=None, nsteps: int = 0):
        I = out if out is not None else self.empty(self.nt, self.batch, self.ns)
        it = np.zeros(self.nt, dtype=np.int32)
        st = Stats()
        st.iters_per_step = it.ctypes.data_as(POINTER(c_int32))
        _lib.check(_lib.load().etaim_march(self._h, c_void_p(_dptr(V)), c_void_p(_dptr(I)), nsteps, byref(st)))
        return I, _stats_dict(st, it)

    def march_continue(self, V, I, first: int, nsteps: int):
        """Steps first .. first + nsteps - 1 of the forward march, continuing
        the history of the last march on this problem (or a loaded state);
        I holds the earlier steps and receives these."""
        it = np.zeros(nsteps, dtype=np.int32)
        st = Stats()
        st.iters_per_step = it.ctypes.data_as(POINTER(c_int32))
        _lib.check(_lib.load().etaim_march_continue(self._h, c_void_p(_dptr(V)), c_void_p(_dptr(I)), first, nsteps,
                                                    byref(st)))
        return I, _stats_dict(st, it)

    def save_state(self) -> np.ndarray:
        """The march state (history rings, next step) as host bytes."""
        n = c_size_t(0)
        _lib.check(_lib.load().etaim_state_size(self._h, byref(n)))
        buf = np.empty(n.value, dtype=np.uint8)
        _lib.check(_lib.load().etaim_state_save(self._h, buf.ctypes.data_as(c_void_p), buf.nbytes))
        return buf

    def load_state(self, buf: np.ndarray):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _lib.check(_lib.load().etaim_state_load(self._h, buf.ctypes.data_as(c_void_p), buf.nbytes))

    def adjoint_march(self, S):
        L = self.empty(self.nt, self.batch, self.ns)
        it = np.zeros(self.nt, dtype=np.int32)
        st = Stats()
        st.iters_per_step = it.ctypes.data_as(POINTER(c_int32))
        _lib.check(_lib.load().etaim_adjoint_march(self._h, c_void_p(_dptr(S)), c_void_p(_dptr(L)), byref(st)))
        return L, _stats_dict(st, it)

    def apply_z(self, m: int, x):
        y = self.empty(*x.shape)
        _lib.check(_lib.load().etaim_apply_z(self._h, m, c_void_p(_dptr(x)), c_void_p(_dptr(y))))
        return y

    def delayed_field(self, hist):
        b = self.empty(self.batch, self.ns)
        _lib.check(_lib.load().etaim_delayed_field(self._h, c_void_p(_dptr(hist)), c_void_p(_dptr(b))))
        return b

    def farfield(self, dirs, I):
        d = np.ascontiguousarray(np.atleast_2d(dirs), dtype=np.float64)
        U = self.empty(self.nt, self.batch, len(d), 3)
        _lib.check(_lib.load().etaim_farfield(self._h, len(d), d.ctypes.data_as(POINTER(c_double)),
                                              c_void_p(_dptr(I)), c_void_p(_dptr(U))))
        return U

    def farfield_adjoint(self, dirs, U):
        d = np.ascontiguousarray(np.atleast_2d(dirs), dtype=np.float64)
        S = self.empty(self.nt, self.batch, self.ns)
        _lib.check(_lib.load().etaim_farfield_adjoint(self._h, len(d), d.ctypes.data_as(POINTER(c_double)),
                                                      c_void_p(_dptr(U)), c_void_p(_dptr(S))))
        return S

    def rcs(self, U, pol, df, pulse_sigma: float):
        """Co-polarised RCS [len(df), B, nd] (m^2, device float64) at f_c + df
        from far-field envelopes U [N_t][B][nd][3] (farfield), for the
        Gaussian pulse of width pulse_sigma; pol [nd][3] (theta-hat for
        sigma_theta-theta)."""
        torch = _torch()
        p = np.ascontiguousarray(np.atleast_2d(pol), dtype=np.float64)
        f = np.ascontiguousarray(np.atleast_1d(df), dtype=np.float64)
        out = torch.empty((len(f), self.batch, len(p)), dtype=torch.float64, device=U.device)
        _lib.check(_lib.load().etaim_rcs(self._h, len(p), p.ctypes.data_as(POINTER(c_double)), len(f),
                                         f.ctypes.data_as(POINTER(c_double)), float(pulse_sigma),
                                         c_void_p(_dptr(U)), c_void_p(out.data_ptr())))
        return out

    _EXPORT = {"lambda": (0, np.float64, lambda i: (i["ns"], 4, 64)),
               "corners": (1, np.int32, lambda i: (i["ns"], 3)),
               "rowptr": (2, np.int32, lambda i: (i["ns"] + 1,)),
               "col": (3, np.int32, lambda i: (i["nnz"],)),
               "near": (4, np.complex128, lambda i: (i["mn"] + 1, i["nnz"])),
               "diag": (5, np.complex128, lambda i: (i["ns"],)),
               "ghat": (6, np.complex128, lambda i: (i["ng"] + 1, 2, i["grid"][2] + 1, i["grid"][1] + 1,
                                                     i["grid"][0] + 1)),
               "curl_lambda": (7, np.float64, lambda i: (i["ns"], 4, 64))}

    def export(self, what: str) -> np.ndarray:
        wid, dt, shape = self._EXPORT[what]
        a = np.empty(shape(self.info), dtype=dt)
        _lib.check(_lib.load().etaim_export(self._h, wid, a.ctypes.data_as(c_void_p), a.nbytes))
        return a

    def set_profiling(self, on: bool = True, classes=None):
        """Per-class kernel tracing: all classes, or only the named ones
        (names from KERNEL_CLASSES)."""
        if classes is None:
            _lib.check(_lib.load().etaim_set_profiling(self._h, 1 if on else 0))
            return
        mask = 0
        for name in classes:
            mask |= 1 << _lib.KERNEL_CLASSES.index(name)
        _lib.check(_lib.load().etaim_set_profiling_mask(self._h, mask if on else 0))

    def set_delay_mode(self, mode: int):
        """Delayed-field algorithm: 0 the k-space temporal sum in time blocks,
        1 multilevel time blocks with temporal DFT convolutions."""
        _lib.check(_lib.load().etaim_set_delay_mode(self._h, int(mode)))

    def delay_mode(self) -> int:
        v = ctypes.c_int32()
        _lib.check(_lib.load().etaim_get_delay_mode(self._h, ctypes.byref(v)))
        return v.value

    def kernel_stats(self) -> dict:
        out = {}
        lib = _lib.load()
        for i, name in enumerate(_lib.KERNEL_CLASSES):
            ms, by, n = c_double(), c_double(), ctypes.c_int64()
            _lib.check(lib.etaim_kernel_stats(self._h, i, byref(ms), byref(by), byref(n)))
            out[name] = {"ms": ms.value, "bytes": by.value, "launches": n.value}
        return out

    @staticmethod
    def _tuning_dict(t) -> dict:
        d = {ax: [v for v in t.radix[a] if v] for a, ax in enumerate(("radix_x", "radix_y", "radix_z"))}
        for f in ("gather_rows", "lines_per_block", "interp_waves", "sync_every", "graph", "yz_engine", "x_engine",
                  "guess_order", "precond", "delay_block", "interp_engine", "apply_ms", "solve_ms"):
            d[f] = getattr(t, f)
        return d

    def autotune(self, budget_ms: int = 3000, cache: str | None = None) -> dict:
        """Time the admissible FFT plans, launch shapes and GMRES schedules on
        this problem and keep the fastest (etaim_autotune)."""
        t = _lib.Tuning()
        _lib.check(_lib.load().etaim_autotune(self._h, int(budget_ms), cache.encode() if cache else None, byref(t)))
        return self._tuning_dict(t)

    def tuning(self) -> dict:
        t = _lib.Tuning()
        _lib.check(_lib.load().etaim_get_tuning(self._h, byref(t)))
        return self._tuning_dict(t)

    def set_tuning(self, d: dict):
        t = _lib.Tuning()
        for a, ax in enumerate(("radix_x", "radix_y", "radix_z")):
            for i, v in enumerate(d[ax]):
                t.radix[a][i] = int(v)
        for f in ("gather_rows", "lines_per_block", "interp_waves", "sync_every", "graph", "yz_engine", "x_engine",
                  "guess_order", "precond", "delay_block", "interp_engine"):
            setattr(t, f, int(d.get(f, 0)))
        _lib.check(_lib.load().etaim_set_tuning(self._h, byref(t)))

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().etaim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def db_error(sigma, sigma_ref, weight, floor_db: float = 80.0) -> float:
    """Thresholded dB-error norm of eq. (2) between two RCS patterns on the
    same directions (host arrays; weight = sin(theta) on a (theta, phi) grid)."""
    a = np.ascontiguousarray(np.ravel(sigma), dtype=np.float64)
    b = np.ascontiguousarray(np.ravel(sigma_ref), dtype=np.float64)
    w = np.ascontiguousarray(np.ravel(weight), dtype=np.float64)
    if not (a.size == b.size == w.size):
        raise ValueError("sigma, sigma_ref and weight need the same size")
    err = c_double(0)
    _lib.check(_lib.load().etaim_db_error(a.size, a.ctypes.data_as(POINTER(c_double)),
                                          b.ctypes.data_as(POINTER(c_double)), w.ctypes.data_as(POINTER(c_double)),
                                          floor_db, byref(err)))
    return err.value


class EtaimMarch:
    """torch.autograd.Function: U = F(march(V)) (scattered far-field envelopes
    at the directions ``dirs``); backward runs the adjoint march:
    grad_V = Z^-H F^H grad_U."""

    @staticmethod
    def apply(V, problem: Problem, dirs):
        torch = _torch()

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, v):
                I, _ = problem.march(v.detach().contiguous())
                return problem.farfield(dirs, I)

            @staticmethod
            def backward(ctx, gU):
                S = problem.farfield_adjoint(dirs, gU.contiguous())
                lam, _ = problem.adjoint_march(S)
                return lam

        return _Fn.apply(V)
