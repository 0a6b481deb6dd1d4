"""Thin Python binding of the C ABI in include/sn.h (libsn.so, gfx950).

Argument marshalling only: every function forwards device pointers of torch
tensors (the caller's HBM buffers) and the context's HIP stream to the
library; all arithmetic runs in the HIP kernels.  The functions carry the C
names.  If libsn.so has not been built the import of `lib()` fails loudly:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsn.so")

SN_OK, SN_ERR_INVALID, SN_ERR_UNSUPPORTED, SN_ERR_NOMEM, SN_ERR_HIP = 0, 1, 2, 3, 4
SN_ERR_NOT_CONVERGED, SN_ERR_DIVERGED, SN_ERR_CG_BREAKDOWN = 5, 6, 7
SN_FP64, SN_FP32 = 0, 1
SN_PRECOND_BLOCK_JACOBI, SN_PRECOND_MG, SN_PRECOND_DIRECT = 0, 1, 2
SN_DSA_DIAGONAL, SN_DSA_TRIANGULAR = 0, 1
SN_DIFFUSION_SIP, SN_DIFFUSION_NIP, SN_DIFFUSION_MNIP = 0, 1, 2
SN_DSA_GMRES_RESTART = 30
SN_KRYLOV_MAX_RESTART = 200

# every symbol declared in include/sn.h
EXPORTED = ("sn_context_create", "sn_context_destroy", "sn_inflow_size", "sn_thick_count", "sn_sweep",
            "sn_scalar_flux", "sn_dsa_thick_correct", "sn_source_iterate", "sn_krylov_solve", "sn_adjoint_source",
            "sn_face_response", "sn_adjoint_gradient", "sn_gradient", "sn_response", "sn_response_noalloc",
            "sn_set_kernel_timing", "sn_kernel_timing", "sn_last_error")


class SnError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sn error {code}: {msg}")
        self.code = code


class sn_mesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double), ("hz", ctypes.c_double), ("order", ctypes.c_int)]


class sn_quad(ctypes.Structure):
    _fields_ = [("ndirs", ctypes.c_int), ("omega", ctypes.POINTER(ctypes.c_double)),
                ("w", ctypes.POINTER(ctypes.c_double))]


class sn_dsa_opts(ctypes.Structure):
    _fields_ = [("cg_rtol", ctypes.c_double), ("cg_maxit", ctypes.c_int), ("mass_kind", ctypes.c_int),
                ("precond", ctypes.c_int), ("diffusion", ctypes.c_int)]


class sn_dsa_stats(ctypes.Structure):
    _fields_ = [("cg_iters", ctypes.c_int), ("cg_relres", ctypes.c_double), ("n_thick_cells", ctypes.c_int)]


class sn_iter_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_it", ctypes.c_int), ("use_dsa", ctypes.c_int),
                ("prec", ctypes.c_int), ("dsa", sn_dsa_opts), ("transpose", ctypes.c_int),
                ("phi_ckpt", ctypes.c_void_p), ("ckpt_cap", ctypes.c_int), ("fp32_refine", ctypes.c_int),
                ("dsa_form", ctypes.c_int)]


class sn_iter_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("res_hist", ctypes.POINTER(ctypes.c_double)),
                ("cg_hist", ctypes.POINTER(ctypes.c_int)), ("seconds", ctypes.c_double),
                ("fp64_checks", ctypes.c_int), ("sweeps", ctypes.c_int)]


class sn_krylov_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_it", ctypes.c_int), ("restart", ctypes.c_int),
                ("use_dsa", ctypes.c_int), ("dsa_form", ctypes.c_int), ("dsa", sn_dsa_opts),
                ("transpose", ctypes.c_int)]


_lib = None


def lib():
    """Load libsn.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2001_09196_amd.build` "
                               "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        vp, ip = ctypes.c_void_p, ctypes.c_int
        L.sn_context_create.argtypes = [ctypes.POINTER(sn_mesh), ctypes.POINTER(sn_quad), vp, vp, ctypes.c_double, vp,
                                        ctypes.POINTER(vp)]
        L.sn_context_create.restype = ip
        L.sn_context_destroy.argtypes = [vp]
        L.sn_context_destroy.restype = None
        L.sn_inflow_size.argtypes = [ctypes.POINTER(sn_mesh)]
        L.sn_inflow_size.restype = ctypes.c_long
        L.sn_thick_count.argtypes = [vp]
        L.sn_thick_count.restype = ip
        L.sn_sweep.argtypes = [vp, vp, vp, vp, ip, ip, vp]
        L.sn_sweep.restype = ip
        L.sn_scalar_flux.argtypes = [vp, vp, ip, vp]
        L.sn_scalar_flux.restype = ip
        L.sn_dsa_thick_correct.argtypes = [vp, vp, vp, vp, ctypes.POINTER(sn_dsa_opts), ctypes.POINTER(sn_dsa_stats)]
        L.sn_dsa_thick_correct.restype = ip
        L.sn_source_iterate.argtypes = [vp, vp, vp, vp, ctypes.POINTER(sn_iter_opts), ctypes.POINTER(sn_iter_stats)]
        L.sn_source_iterate.restype = ip
        L.sn_krylov_solve.argtypes = [vp, vp, vp, vp, ctypes.POINTER(sn_krylov_opts), ctypes.POINTER(sn_iter_stats)]
        L.sn_krylov_solve.restype = ip
        L.sn_adjoint_source.argtypes = [vp, vp, ip, vp, vp]
        L.sn_adjoint_source.restype = ip
        L.sn_face_response.argtypes = [vp, vp, vp, vp, ip, ctypes.POINTER(ctypes.c_double)]
        L.sn_face_response.restype = ip
        L.sn_adjoint_gradient.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.sn_adjoint_gradient.restype = ip
        L.sn_gradient.argtypes = [vp, vp, vp, ip, vp, vp, vp, vp]
        L.sn_gradient.restype = ip
        L.sn_response.argtypes = [vp, vp, vp, ip, vp, ip, ctypes.POINTER(ctypes.c_double)]
        L.sn_response.restype = ip
        L.sn_response_noalloc.argtypes = [vp, vp, vp, ip, vp, ip, ctypes.POINTER(ctypes.c_double)]
        L.sn_response_noalloc.restype = ip
        L.sn_set_kernel_timing.argtypes = [vp, ip]
        L.sn_set_kernel_timing.restype = ip
        dp = ctypes.POINTER(ctypes.c_double)
        L.sn_kernel_timing.argtypes = [vp, dp, ctypes.POINTER(ip), dp, ctypes.POINTER(ip)]
        L.sn_kernel_timing.restype = ip
        L.sn_last_error.argtypes = []
        L.sn_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int, allow=()):
    if rc != SN_OK and rc not in allow:
        raise SnError(rc, lib().sn_last_error().decode())
    return rc


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return t.data_ptr()


def _stream_handle(stream) -> Optional[int]:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream or None


class Context:
    """An sn_context: mesh, quadrature, cross sections, thick set, workspace.

    sigma_t, sigma_s: FP64 device tensors [ncells]; omega [D, 3] and w [D] are
    host arrays.  The context's stream is torch's current stream unless given.
    order: DG order (1: Q1; 2, 3: Q_p in 2D, a subset of the entry points).
    """

    def __init__(self, dim, nx, ny, nz, h, omega, w, sigma_t, sigma_s, eta=1.0, stream=None, order=1):
        import torch
        self.dim, self.nx, self.ny, self.nz = int(dim), int(nx), int(ny), int(nz)
        self.order = int(order)
        self.nn = (self.order + 1) ** self.dim
        self.ncells = self.nx * self.ny * self.nz
        self._omega = np.ascontiguousarray(omega, dtype=np.float64)
        self._w = np.ascontiguousarray(w, dtype=np.float64)
        self.ndirs = int(self._w.shape[0])
        self.mesh = sn_mesh(self.dim, self.nx, self.ny, self.nz, float(h[0]), float(h[1]),
                            float(h[2]) if len(h) > 2 else 1.0, self.order)
        quad = sn_quad(self.ndirs, self._omega.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                       self._w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        for t in (sigma_t, sigma_s):
            if t.dtype != torch.float64 or t.numel() != self.ncells:
                raise ValueError("sigma arrays must be FP64 with one value per cell")
        self.stream = torch.cuda.current_stream() if stream is None else stream
        self.device = sigma_t.device
        self._h = ctypes.c_void_p()
        _check(lib().sn_context_create(ctypes.byref(self.mesh), ctypes.byref(quad), _ptr(sigma_t), _ptr(sigma_s),
                                       float(eta), self.stream.cuda_stream or None, ctypes.byref(self._h)))
        self.nbf = int(lib().sn_inflow_size(ctypes.byref(self.mesh)))

    @property
    def handle(self):
        return self._h

    @property
    def thick_count(self) -> int:
        return int(lib().sn_thick_count(self._h))

    def close(self):
        if self._h:
            lib().sn_context_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def sn_sweep(ctx: Context, phi, q, inflow, transpose: bool, prec: int, psi):
    _check(lib().sn_sweep(ctx.handle, _ptr(phi), _ptr(q), _ptr(inflow), int(bool(transpose)), int(prec), _ptr(psi)))


def sn_scalar_flux(ctx: Context, psi, prec: int, phi_out):
    _check(lib().sn_scalar_flux(ctx.handle, _ptr(psi), int(prec), _ptr(phi_out)))


def sn_dsa_thick_correct(ctx: Context, phi_old, phi_si, phi_out, cg_rtol=1e-4, cg_maxit=1000, mass_kind=0,
                         precond=0, diffusion=SN_DIFFUSION_SIP):
    """precond: SN_PRECOND_BLOCK_JACOBI (0), SN_PRECOND_MG (1) or
    SN_PRECOND_DIRECT (2, exact band LU for small thick systems);
    diffusion: SN_DIFFUSION_SIP (CG) / _NIP / _MNIP (GMRES)."""
    o = sn_dsa_opts(float(cg_rtol), int(cg_maxit), int(mass_kind), int(precond), int(diffusion))
    st = sn_dsa_stats()
    rc = _check(lib().sn_dsa_thick_correct(ctx.handle, _ptr(phi_old), _ptr(phi_si), _ptr(phi_out), ctypes.byref(o),
                                           ctypes.byref(st)))
    return {"rc": rc, "cg_iters": st.cg_iters, "cg_relres": st.cg_relres, "n_thick_cells": st.n_thick_cells}


def _stats(max_it):
    res = np.zeros(max_it, dtype=np.float64)
    cgh = np.zeros(max_it, dtype=np.int32)
    st = sn_iter_stats(0, res.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                       cgh.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), 0.0, 0, 0)
    return st, res, cgh


def sn_source_iterate(ctx: Context, q, inflow, phi, tol=1e-8, max_it=1000, use_dsa=True, prec=SN_FP64,
                      cg_rtol=1e-4, cg_maxit=1000, mass_kind=0, transpose=False, phi_ckpt=None, precond=0,
                      fp32_refine=False, dsa_form=SN_DSA_DIAGONAL, diffusion=SN_DIFFUSION_SIP):
    """Returns dict(rc, iters, res_hist, cg_hist, seconds, fp64_checks, sweeps);
    raises on errors other than NOT_CONVERGED / DIVERGED (reported in rc).
    phi_ckpt: optional device tensor [cap, ncells, nn]; iterate it is kept in
    slot it % cap."""
    o = sn_iter_opts(float(tol), int(max_it), int(bool(use_dsa)), int(prec),
                     sn_dsa_opts(float(cg_rtol), int(cg_maxit), int(mass_kind), int(precond), int(diffusion)),
                     int(bool(transpose)), _ptr(phi_ckpt), int(phi_ckpt.shape[0]) if phi_ckpt is not None else 0, int(bool(fp32_refine)),
                     int(dsa_form))
    st, res, cgh = _stats(max_it)
    rc = _check(lib().sn_source_iterate(ctx.handle, _ptr(q), _ptr(inflow), _ptr(phi), ctypes.byref(o),
                                        ctypes.byref(st)), allow=(SN_ERR_NOT_CONVERGED, SN_ERR_DIVERGED))
    n = st.iters
    return {"rc": rc, "iters": n, "res_hist": res[:n].copy(), "cg_hist": cgh[:n].copy(), "seconds": st.seconds,
            "fp64_checks": st.fp64_checks, "sweeps": st.sweeps}


def sn_krylov_solve(ctx: Context, q, inflow, phi, tol=1e-8, max_it=1000, restart=30, use_dsa=True,
                    dsa_form=SN_DSA_DIAGONAL, cg_rtol=1e-4, cg_maxit=1000, mass_kind=0, precond=0, transpose=False,
                    diffusion=SN_DIFFUSION_SIP):
    """Flexible GMRES(restart) on the scalar-flux Schur system; returns dict
    as sn_source_iterate (raises on errors other than NOT_CONVERGED / DIVERGED)."""
    o = sn_krylov_opts(float(tol), int(max_it), int(restart), int(bool(use_dsa)), int(dsa_form),
                       sn_dsa_opts(float(cg_rtol), int(cg_maxit), int(mass_kind), int(precond), int(diffusion)),
                       int(bool(transpose)))
    st, res, cgh = _stats(max_it)
    rc = _check(lib().sn_krylov_solve(ctx.handle, _ptr(q), _ptr(inflow), _ptr(phi), ctypes.byref(o),
                                      ctypes.byref(st)), allow=(SN_ERR_NOT_CONVERGED, SN_ERR_DIVERGED))
    n = st.iters
    return {"rc": rc, "iters": n, "res_hist": res[:n].copy(), "cg_hist": cgh[:n].copy(), "seconds": st.seconds,
            "sweeps": st.sweeps}


def sn_adjoint_source(ctx: Context, r=None, face: int = -1, q_adj=None, inflow_adj=None):
    _check(lib().sn_adjoint_source(ctx.handle, _ptr(r), int(face), _ptr(q_adj), _ptr(inflow_adj)))


def sn_face_response(ctx: Context, phi, q, inflow, face: int) -> float:
    out = ctypes.c_double()
    _check(lib().sn_face_response(ctx.handle, _ptr(phi), _ptr(q), _ptr(inflow), int(face), ctypes.byref(out)))
    return out.value


def sn_adjoint_gradient(ctx: Context, phi, q, inflow, chi, q_adj, inflow_adj, g_t, g_s):
    _check(lib().sn_adjoint_gradient(ctx.handle, _ptr(phi), _ptr(q), _ptr(inflow), _ptr(chi), _ptr(q_adj),
                                     _ptr(inflow_adj), _ptr(g_t), _ptr(g_s)))


def sn_gradient(ctx: Context, psi, psi_adj, prec: int, phi, chi, g_t, g_s):
    _check(lib().sn_gradient(ctx.handle, _ptr(psi), _ptr(psi_adj), int(prec), _ptr(phi), _ptr(chi), _ptr(g_t),
                             _ptr(g_s)))


def sn_response(ctx: Context, r=None, phi=None, face: int = -1, psi=None, prec: int = SN_FP64) -> float:
    out = ctypes.c_double()
    _check(lib().sn_response(ctx.handle, _ptr(r), _ptr(phi), int(face), _ptr(psi), int(prec), ctypes.byref(out)))
    return out.value


def sn_response_noalloc(ctx: Context, r=None, phi=None, face: int = -1, psi=None, prec: int = SN_FP64) -> float:
    """sn_response without device allocation (fixed scratch, see sn.h)."""
    out = ctypes.c_double()
    _check(lib().sn_response_noalloc(ctx.handle, _ptr(r), _ptr(phi), int(face), _ptr(psi), int(prec),
                                     ctypes.byref(out)))
    return out.value


def sn_set_kernel_timing(ctx: Context, enable: bool, sweeps_only: bool = False):
    """enable: record HIP events around the sweep kernels and (unless
    sweeps_only) around each DSA solve."""
    _check(lib().sn_set_kernel_timing(ctx.handle, (2 if sweeps_only else 1) if enable else 0))


def sn_kernel_timing(ctx: Context):
    """Returns dict(sweep_ms, sweep_count, dsa_ms, dsa_count) since the last query."""
    a, c = ctypes.c_double(), ctypes.c_int()
    b, d = ctypes.c_double(), ctypes.c_int()
    _check(lib().sn_kernel_timing(ctx.handle, ctypes.byref(a), ctypes.byref(c), ctypes.byref(b), ctypes.byref(d)))
    return {"sweep_ms": a.value, "sweep_count": c.value, "dsa_ms": b.value, "dsa_count": d.value}
