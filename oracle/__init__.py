"""CPU FP64 oracle for S_N source iteration with heterogeneous DSA.

TEST INFRASTRUCTURE ONLY: the independent checker of the GPU library.  Only
the test suite, the smoke check and the benchmark's CPU-baseline leg may
import it; the product path never does.  It shares no code with the GPU
library; the two meet only through the seeded inputs of `sninputs`.

The arithmetic lives in `oracle.c` (plain C, OpenMP over directions); this
module compiles it with gcc and wraps it with ctypes.

Parity pins (tests/test_oracle_*.py) tie every function here to the paper or
to mathematics that does not depend on this code: brute-force dense solves
of the assembled system, the exact outflow factor of a pure absorber,
particle balance, symmetry, the transpose identity, infinite-medium limits,
and agreement of accelerated and unaccelerated fixed points.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (C99, -O3, OpenMP)."""
    cmd = ["gcc", "-std=c99", "-O3", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
           _SRC, "-o", _LIB + ".tmp", "-lm"]
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Mesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double), ("hz", ctypes.c_double)]


_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_lp = ctypes.POINTER(ctypes.c_long)


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            L = ctypes.CDLL(_LIB)
            mp = ctypes.POINTER(_Mesh)
            L.orc_cell_matrix.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double, _dp]
            L.orc_cell_mass.argtypes = [ctypes.c_int, _dp, _dp]
            L.orc_sweep.argtypes = [mp, ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_int, _dp]
            L.orc_sweep.restype = ctypes.c_int
            L.orc_moment.argtypes = [mp, ctypes.c_int, _dp, _dp, _dp]
            L.orc_dsa_correct.argtypes = [mp, ctypes.c_int, _dp, _dp, _dp, _dp, ctypes.c_double, ctypes.c_int,
                                          ctypes.c_int, _dp, _dp, ctypes.c_double, ctypes.c_int, _dp, _ip, _dp]
            L.orc_dsa_correct.restype = ctypes.c_int
            L.orc_dsa_dense.argtypes = [mp, ctypes.c_int, _dp, _dp, _dp, _dp, ctypes.c_double, ctypes.c_int, _dp,
                                        _lp, _ip]
            L.orc_dsa_dense.restype = ctypes.c_int
            L.orc_source_iterate.argtypes = [mp, ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_double,
                                             ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                             ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp,
                                             _ip, _ip]
            L.orc_source_iterate.restype = ctypes.c_int
            L.orc_gmres.argtypes = [mp, ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_double, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_double, ctypes.c_int, ctypes.c_int, _dp, _dp, _ip, _ip]
            L.orc_gmres.restype = ctypes.c_int
            L.orc_gradient.argtypes = [mp, ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
            L.orc_inflow_size.argtypes = [mp]
            L.orc_inflow_size.restype = ctypes.c_long
            L.orc_num_threads.restype = ctypes.c_int
            _lib = L
    return _lib


def _d(a):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _mesh(p) -> _Mesh:
    return _Mesh(p.dim, p.nx, p.ny, p.nz, float(p.h[0]), float(p.h[1]), float(p.h[2]))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def cell_matrix(dim, h, om, sigma_t):
    nn = 4 if dim == 2 else 8
    A = np.zeros(nn * nn)
    lib().orc_cell_matrix(dim, _d(_f64(h)), _d(_f64(om)), float(sigma_t), _d(A))
    return A.reshape(nn, nn)


def cell_mass(dim, h):
    nn = 4 if dim == 2 else 8
    M = np.zeros(nn * nn)
    lib().orc_cell_mass(dim, _d(_f64(h)), _d(M))
    return M.reshape(nn, nn)


def sweep(p, phi, q, inflow=None, transpose=False, sigma_t=None, sigma_s=None):
    """psi[c, d, n] = (L_d^{-1} or L_d^{-T}) (M (sigma_s phi + q)/4pi + boundary load)."""
    st = _f64(p.sigma_t if sigma_t is None else sigma_t)
    ss = _f64(p.sigma_s if sigma_s is None else sigma_s)
    phi = _f64(np.zeros(p.ncells * p.nn) if phi is None else phi).ravel()
    q = _f64(np.zeros(p.ncells) if q is None else q)
    inflow = _f64(inflow)
    psi = np.zeros(p.ncells * p.ndirs * p.nn)
    m = _mesh(p)
    rc = lib().orc_sweep(ctypes.byref(m), p.ndirs, _d(_f64(p.omega)), _d(st), _d(ss), _d(phi), _d(q),
                         _d(inflow), int(bool(transpose)), _d(psi))
    if rc:
        raise RuntimeError(f"orc_sweep failed ({rc})")
    return psi.reshape(p.ncells, p.ndirs, p.nn)


def moment(p, psi):
    phi = np.zeros(p.ncells * p.nn)
    m = _mesh(p)
    lib().orc_moment(ctypes.byref(m), p.ndirs, _d(_f64(p.w)), _d(_f64(psi).ravel()), _d(phi))
    return phi.reshape(p.ncells, p.nn)


# diffusion forms of the DSA (Sec. 3.1): eq. SIP, eq. NIP, and NIP with the
# penalty of eq. ModifiedF0
DSA_SIP, DSA_NIP, DSA_MNIP = 0, 1, 2


def dsa_correct(p, phi_old, phi_si, eta=None, mass_kind=0, cg_rtol=1e-13, cg_maxit=100000,
                sigma_t=None, sigma_s=None, dsa_op=DSA_SIP):
    st = _f64(p.sigma_t if sigma_t is None else sigma_t)
    ss = _f64(p.sigma_s if sigma_s is None else sigma_s)
    out = np.zeros(p.ncells * p.nn)
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    m = _mesh(p)
    rc = lib().orc_dsa_correct(ctypes.byref(m), p.ndirs, _d(_f64(p.omega)), _d(_f64(p.w)), _d(st), _d(ss),
                               float(p.eta if eta is None else eta), int(mass_kind), int(dsa_op),
                               _d(_f64(phi_old).ravel()), _d(_f64(phi_si).ravel()), float(cg_rtol),
                               int(cg_maxit), _d(out), ctypes.byref(it), ctypes.byref(rr))
    if rc:
        raise RuntimeError(f"orc_dsa_correct failed ({rc})")
    return out.reshape(p.ncells, p.nn), it.value, rr.value


def dsa_dense(p, eta=None, sigma_t=None, sigma_s=None, dsa_op=DSA_SIP):
    """Dense D_ff and the thick cell list (small problems only)."""
    st = _f64(p.sigma_t if sigma_t is None else sigma_t)
    ss = _f64(p.sigma_s if sigma_s is None else sigma_s)
    e = float(p.eta if eta is None else eta)
    nthick = int(np.count_nonzero(ss >= e))
    nf = nthick * p.nn
    D = np.zeros(max(nf * nf, 1))
    cells = np.zeros(max(nthick, 1), dtype=np.int64)
    nt = ctypes.c_int(0)
    m = _mesh(p)
    rc = lib().orc_dsa_dense(ctypes.byref(m), p.ndirs, _d(_f64(p.omega)), _d(_f64(p.w)), _d(st), _d(ss), e,
                             int(dsa_op), _d(D), cells.ctypes.data_as(_lp), ctypes.byref(nt))
    if rc:
        raise RuntimeError(f"orc_dsa_dense failed ({rc})")
    return D[:nf * nf].reshape(nf, nf), cells[:nt.value]


def source_iterate(p, tol=1e-8, max_it=1000, use_dsa=True, mass_kind=0, cg_rtol=1e-13, cg_maxit=100000,
                   transpose=False, phi0=None, q=None, inflow=None, eta=None, sigma_t=None, sigma_s=None,
                   dsa_form=0, dsa_op=DSA_SIP):
    """Returns dict(phi [nc, nn], iters, res_hist, cg_hist, rc).
    dsa_form: 0 diagonal heterogeneous DSA (Alg. 2), 1 triangular (Alg. 1);
    dsa_op: the diffusion form (DSA_SIP by CG, DSA_NIP / DSA_MNIP by an exact
    band LU solve; their cg_hist entries are 0)."""
    st = _f64(p.sigma_t if sigma_t is None else sigma_t)
    ss = _f64(p.sigma_s if sigma_s is None else sigma_s)
    qq = _f64(p.q if q is None else q)
    phi = np.zeros(p.ncells * p.nn) if phi0 is None else _f64(phi0).ravel().copy()
    res = np.zeros(max_it)
    cgh = np.zeros(max_it, dtype=np.int32)
    iters = ctypes.c_int(0)
    m = _mesh(p)
    rc = lib().orc_source_iterate(ctypes.byref(m), p.ndirs, _d(_f64(p.omega)), _d(_f64(p.w)), _d(st), _d(ss),
                                  _d(qq), _d(_f64(inflow)), float(p.eta if eta is None else eta),
                                  int(bool(use_dsa)), int(mass_kind), int(dsa_op), float(tol), int(max_it),
                                  float(cg_rtol),
                                  int(cg_maxit), int(bool(transpose)), int(dsa_form), _d(phi), _d(res),
                                  cgh.ctypes.data_as(_ip), ctypes.byref(iters))
    if rc not in (0, 5, 6):
        raise RuntimeError(f"orc_source_iterate failed ({rc})")
    n = iters.value
    return {"phi": phi.reshape(p.ncells, p.nn), "iters": n, "res_hist": res[:n], "cg_hist": cgh[:n], "rc": rc}


def gmres(p, tol=1e-8, max_it=1000, restart=30, use_dsa=True, dsa_form=0, mass_kind=0, cg_rtol=1e-13,
          cg_maxit=100000, transpose=False, phi0=None, q=None, inflow=None, eta=None, sigma_t=None, sigma_s=None,
          dsa_op=DSA_SIP):
    """Flexible GMRES(restart) on S phi = b, right-preconditioned by the
    heterogeneous DSA.  Returns dict(phi, iters, res_hist, cg_hist, rc);
    an iteration is one application of S (one sweep)."""
    st = _f64(p.sigma_t if sigma_t is None else sigma_t)
    ss = _f64(p.sigma_s if sigma_s is None else sigma_s)
    qq = _f64(p.q if q is None else q)
    phi = np.zeros(p.ncells * p.nn) if phi0 is None else _f64(phi0).ravel().copy()
    res = np.zeros(max_it)
    cgh = np.zeros(max_it, dtype=np.int32)
    iters = ctypes.c_int(0)
    m = _mesh(p)
    rc = lib().orc_gmres(ctypes.byref(m), p.ndirs, _d(_f64(p.omega)), _d(_f64(p.w)), _d(st), _d(ss), _d(qq),
                         _d(_f64(inflow)), float(p.eta if eta is None else eta), int(bool(use_dsa)), int(mass_kind),
                         int(dsa_op), int(dsa_form), float(tol), int(max_it), int(restart), float(cg_rtol),
                         int(cg_maxit),
                         int(bool(transpose)), _d(phi), _d(res), cgh.ctypes.data_as(_ip), ctypes.byref(iters))
    if rc not in (0, 5, 6):
        raise RuntimeError(f"orc_gmres failed ({rc})")
    n = iters.value
    return {"phi": phi.reshape(p.ncells, p.nn), "iters": n, "res_hist": res[:n], "cg_hist": cgh[:n], "rc": rc}


def gradient(p, psi, psi_adj, phi, chi, sigma_t=None, sigma_s=None):
    st = _f64(p.sigma_t if sigma_t is None else sigma_t)
    ss = _f64(p.sigma_s if sigma_s is None else sigma_s)
    gt = np.zeros(p.ncells)
    gs = np.zeros(p.ncells)
    m = _mesh(p)
    lib().orc_gradient(ctypes.byref(m), p.ndirs, _d(_f64(p.w)), _d(st), _d(ss), _d(_f64(psi).ravel()),
                       _d(_f64(psi_adj).ravel()), _d(_f64(phi).ravel()), _d(_f64(chi).ravel()), _d(gt), _d(gs))
    return gt, gs
