"""ctypes binding of libwtd.so (argument marshalling only).

Every step of the Liouville apply and of the Davidson solver runs in the HIP
library; this module converts arguments, holds PyTorch tensors for device
memory and passes the current HIP stream.  It never computes any part of the
operator itself, and it raises if the library is missing: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwtd.so")

WTD_OK = 0
WTD_NOT_CONVERGED = 1
STATUS_NAMES = {0: "WTD_OK", 1: "WTD_NOT_CONVERGED", -1: "WTD_ERR_ARG", -2: "WTD_ERR_SHAPE",
                -3: "WTD_ERR_OOM", -4: "WTD_ERR_HIP", -5: "WTD_ERR_UNIMPLEMENTED",
                -6: "WTD_ERR_NONFINITE"}
FP64, FP32 = 0, 1
TERM_D, TERM_K1E, TERM_K1D, TERM_ALL = 1, 2, 4, 7
TERM_K2E, TERM_K2D, TERM_FULL = 8, 16, 31

EXPORTS = ["wtd_debug_gemm", "wtd_create", "wtd_destroy", "wtd_set_occ", "wtd_apply_liouville",
           "wtd_apply_transition", "wtd_apply_liouville_bwd", "wtd_davidson", "wtd_davidson_noalloc", "wtd_cache_pairs", "wtd_autotune", "wtd_apply_full", "wtd_solve_zvector",
           "wtd_profile_enable", "wtd_profile_read", "wtd_workspace_bytes", "wtd_set_workspace_limit",
           "wtd_set_checks", "wtd_last_error"]
CHECK_FINITE = 1


class WtdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class _System(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("cell", ctypes.c_double * 3),
        ("npw", ctypes.c_int32),
        ("mill", ctypes.c_void_p),
        ("nocc", ctypes.c_int32),
        ("ncond", ctypes.c_int32),
        ("c_occ", ctypes.c_void_p),
        ("c_cond", ctypes.c_void_p),
        ("eps_occ", ctypes.c_void_p),
        ("eps_cond", ctypes.c_void_p),
        ("fxc", ctypes.c_void_p),
        ("alpha", ctypes.c_double),
        ("k1e_scale", ctypes.c_double),
        ("v_g0", ctypes.c_double),
        ("term_mask", ctypes.c_uint32),
        ("prec", ctypes.c_int),
    ]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libwtd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2309_03513_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    lib.wtd_create.argtypes = [ctypes.POINTER(_System), i32, vp, ctypes.POINTER(vp)]
    lib.wtd_destroy.argtypes = [vp]
    lib.wtd_set_occ.argtypes = [vp, vp]
    lib.wtd_apply_liouville.argtypes = [vp, i32, vp, vp]
    lib.wtd_apply_transition.argtypes = [vp, i32, vp, vp]
    lib.wtd_apply_liouville_bwd.argtypes = [vp, i32, vp, vp, vp, vp]
    lib.wtd_davidson.argtypes = [vp, i32, i32, f64, i32, i32, vp, vp, vp, vp, vp]
    lib.wtd_davidson_noalloc.argtypes = [vp, i32, i32, f64, i32, i32, vp, vp, vp, vp, vp]
    lib.wtd_cache_pairs.argtypes = [vp, i32]
    lib.wtd_apply_full.argtypes = [vp, i32, vp, vp]
    lib.wtd_solve_zvector.argtypes = [vp, i32, vp, f64, i32, f64, vp, vp, vp, vp]
    lib.wtd_autotune.argtypes = [vp, i32, i32, vp, vp]
    lib.wtd_profile_enable.argtypes = [vp, i32]
    lib.wtd_profile_read.argtypes = [vp, i32, vp, vp, vp, vp]
    lib.wtd_workspace_bytes.argtypes = [vp, vp]
    lib.wtd_set_workspace_limit.argtypes = [ctypes.c_size_t]
    lib.wtd_set_checks.argtypes = [vp, ctypes.c_uint32]
    lib.wtd_debug_gemm.argtypes = [ctypes.c_int, i32, i32, i32, vp, i32, vp, i32, i32, vp, i32, vp]
    lib.wtd_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name != "wtd_last_error":
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status):
    if status < 0:
        raise WtdError(status, load_library().wtd_last_error().decode())
    return status


def set_workspace_limit(nbytes):
    """Cap the device memory of contexts created afterwards (0: no cap)."""
    _check(load_library().wtd_set_workspace_limit(int(nbytes)))


def _torch():
    import torch
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def as_coeff_tensor(c, dtype, device):
    """[..., npw] complex (numpy/torch) or [..., npw, 2] real -> contiguous [..., npw, 2]."""
    torch = _torch()
    if isinstance(c, np.ndarray):
        if np.iscomplexobj(c):
            c = np.stack([c.real, c.imag], axis=-1)
        return torch.from_numpy(np.ascontiguousarray(c)).to(device=device, dtype=dtype).contiguous()
    if c.is_complex():
        c = torch.view_as_real(c.resolve_conj())
    return c.to(device=device, dtype=dtype).contiguous()


class Liouville:
    """A library context for one system: apply L, its transition-space form and Davidson.

    ``system`` needs cell, n, mill, c_occ, c_cond, eps_occ, eps_cond, fxc, alpha,
    c_k and v_g0 (as produced by gen.make_system).  Arrays may be numpy or torch.
    """

    def __init__(self, system, max_nb, precision="fp64", terms=TERM_ALL, device="cuda:0",
                 stream=None):
        torch = _torch()
        lib = load_library()
        self.device = torch.device(device)
        self.prec = FP64 if precision in ("fp64", FP64) else FP32
        self.dtype = torch.float64 if self.prec == FP64 else torch.float32
        self.nocc = int(system.c_occ.shape[0])
        self.ncond = int(system.c_cond.shape[0])
        self.npw = int(np.asarray(system.mill).shape[0])
        self.max_nb = int(max_nb)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        mill = np.ascontiguousarray(np.asarray(system.mill, dtype=np.int32))
        eo = np.ascontiguousarray(np.asarray(system.eps_occ, dtype=np.float64))
        ec = np.ascontiguousarray(np.asarray(system.eps_cond, dtype=np.float64))
        with torch.cuda.device(self.device):
            c_occ = as_coeff_tensor(system.c_occ, torch.float64, self.device)
            c_cond = as_coeff_tensor(system.c_cond, torch.float64, self.device)
            fxc = None
            if system.fxc is not None:
                fxc = torch.as_tensor(np.ascontiguousarray(system.fxc, dtype=np.float64)).to(
                    self.device).contiguous()
            s = _System()
            s.n[:] = [int(v) for v in system.n]
            s.cell[:] = [float(v) for v in system.cell]
            s.npw = self.npw
            s.mill = mill.ctypes.data_as(ctypes.c_void_p)
            s.nocc, s.ncond = self.nocc, self.ncond
            s.c_occ, s.c_cond = c_occ.data_ptr(), c_cond.data_ptr()
            s.eps_occ = eo.ctypes.data_as(ctypes.c_void_p)
            s.eps_cond = ec.ctypes.data_as(ctypes.c_void_p)
            s.fxc = fxc.data_ptr() if fxc is not None else None
            s.alpha, s.k1e_scale, s.v_g0 = float(system.alpha), float(system.c_k), float(system.v_g0)
            s.term_mask = int(terms)
            s.prec = self.prec
            h = ctypes.c_void_p()
            torch.cuda.synchronize(self.device)
            _check(lib.wtd_create(ctypes.byref(s), self.max_nb,
                                  ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self._lib = lib

    # ------------------------------------------------------------------ helpers
    def _handle(self):
        if self._h is None:
            raise RuntimeError("context destroyed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            _check(self._lib.wtd_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_checks(self, finite=True):
        """Scan inputs and outputs of every apply for NaN / infinity (synchronous)."""
        _check(self._lib.wtd_set_checks(self._handle(), CHECK_FINITE if finite else 0))

    def workspace_bytes(self):
        v = ctypes.c_size_t()
        _check(self._lib.wtd_workspace_bytes(self._handle(), ctypes.byref(v)))
        return v.value

    # ------------------------------------------------------------------ operations
    def apply(self, a, out=None):
        """la = L a; a: [nb][nocc][npw][2] device tensor in the context dtype (or complex/numpy)."""
        torch = _torch()
        if not (isinstance(a, torch.Tensor) and a.dtype == self.dtype and a.is_contiguous()
                and a.device == self.device and a.dim() == 4):
            a = as_coeff_tensor(a, self.dtype, self.device)
        nb = a.shape[0]
        assert tuple(a.shape[1:]) == (self.nocc, self.npw, 2), a.shape
        if out is None:
            out = torch.empty_like(a)
        _check(self._lib.wtd_apply_liouville(self._handle(), nb, _ptr(a), _ptr(out)))
        return out

    def apply_full(self, a, out=None):
        """la = (D + K1e - K1d + K2e - K2d) a with the context's term mask."""
        torch = _torch()
        if not (isinstance(a, torch.Tensor) and a.dtype == self.dtype and a.is_contiguous()
                and a.device == self.device and a.dim() == 4):
            a = as_coeff_tensor(a, self.dtype, self.device)
        assert tuple(a.shape[1:]) == (self.nocc, self.npw, 2), a.shape
        if out is None:
            out = torch.empty_like(a)
        _check(self._lib.wtd_apply_full(self._handle(), a.shape[0], _ptr(a), _ptr(out)))
        return out

    def solve_zvector(self, U, tol=1e-8, max_iter=200, lambda_thr=0.0):
        """CG solve of the Z-vector equation; returns (Z float64 tensor, resid numpy,
        n_iter, n_exact, status)."""
        torch = _torch()
        U = as_coeff_tensor(U, torch.float64, self.device)
        Z = torch.empty_like(U)
        resid = np.zeros(U.shape[0])
        nit, nex = ctypes.c_int32(), ctypes.c_int32()
        st = _check(self._lib.wtd_solve_zvector(
            self._handle(), U.shape[0], _ptr(U), float(tol), int(max_iter), float(lambda_thr),
            _ptr(Z), resid.ctypes.data_as(ctypes.c_void_p), ctypes.byref(nit),
            ctypes.byref(nex)))
        return Z, resid, nit.value, nex.value, st

    def apply_transition(self, X, out=None):
        """T = Phi_c^T L Phi_c X; X: [nb][nocc][ncond] float64 device tensor."""
        torch = _torch()
        X = torch.as_tensor(X).to(device=self.device, dtype=torch.float64).contiguous()
        assert tuple(X.shape[1:]) == (self.nocc, self.ncond), X.shape
        if out is None:
            out = torch.empty_like(X)
        _check(self._lib.wtd_apply_transition(self._handle(), X.shape[0], _ptr(X), _ptr(out)))
        return out

    def set_occ(self, c_occ):
        c = as_coeff_tensor(c_occ, _torch().float64, self.device)
        _check(self._lib.wtd_set_occ(self._handle(), _ptr(c)))
        self._keep_occ = c  # borrowed until the stream passes the call

    def apply_bwd(self, a, g_la, want_a=True, want_occ=True):
        torch = _torch()
        a = as_coeff_tensor(a, self.dtype, self.device)
        g = as_coeff_tensor(g_la, self.dtype, self.device)
        ga = torch.empty_like(a) if want_a else None
        go = torch.empty((self.nocc, self.npw, 2), dtype=self.dtype,
                         device=self.device) if want_occ else None
        _check(self._lib.wtd_apply_liouville_bwd(self._handle(), a.shape[0], _ptr(a), _ptr(g),
                                                 _ptr(ga), _ptr(go)))
        return ga, go

    def davidson(self, nroots, nb, tol=1e-8, max_iter=100, max_sub=0, guess=None, want_x=True):
        """Returns (omega[nroots] numpy, x [nroots][nocc][npw][2] float64 tensor or None,
        resid numpy, n_iter, status)."""
        return self._davidson(self._lib.wtd_davidson, nroots, nb, tol, max_iter, max_sub, guess,
                              want_x)

    def davidson_noalloc(self, nroots, nb, tol=1e-8, max_iter=100, max_sub=0, guess=None,
                         want_x=True):
        """wtd_davidson_noalloc: the same run in the library's static device array
        (no device allocation by the library; x, if wanted, is allocated here)."""
        return self._davidson(self._lib.wtd_davidson_noalloc, nroots, nb, tol, max_iter, max_sub,
                              guess, want_x)

    def _davidson(self, fn, nroots, nb, tol, max_iter, max_sub, guess, want_x):
        torch = _torch()
        omega = np.zeros(nroots)
        resid = np.zeros(nroots)
        nit = ctypes.c_int32()
        x = torch.empty((nroots, self.nocc, self.npw, 2), dtype=torch.float64,
                        device=self.device) if want_x else None
        g = as_coeff_tensor(guess, torch.float64, self.device) if guess is not None else None
        st = _check(fn(
            self._handle(), int(nroots), int(nb), float(tol), int(max_iter), int(max_sub),
            _ptr(g), omega.ctypes.data_as(ctypes.c_void_p), _ptr(x),
            resid.ctypes.data_as(ctypes.c_void_p), ctypes.byref(nit)))
        return omega, x, resid, nit.value, st

    def cache_pairs(self, on=True):
        """Keep the pair potentials between applies until the orbitals change."""
        _check(self._lib.wtd_cache_pairs(self._handle(), 1 if on else 0))

    def autotune(self, nb=None, reps=3):
        """Pick the pair batch and density split by timing applies; returns (chunk, groups)."""
        ch, gr = ctypes.c_int32(), ctypes.c_int32()
        _check(self._lib.wtd_autotune(self._handle(), int(nb or self.max_nb), int(reps),
                                      ctypes.byref(ch), ctypes.byref(gr)))
        return ch.value, gr.value

    def profile(self, on=True):
        _check(self._lib.wtd_profile_enable(self._handle(), 1 if on else 0))

    def profile_read(self):
        n = 16
        ms = (ctypes.c_double * n)()
        calls = (ctypes.c_int64 * n)()
        names = (ctypes.c_char_p * n)()
        cnt = ctypes.c_int32()
        _check(self._lib.wtd_profile_read(self._handle(), n, ms, calls, names,
                                          ctypes.byref(cnt)))
        return {names[i].decode(): (ms[i], calls[i]) for i in range(cnt.value)}
