"""Error paths of the C ABI that the library decides on the host before any
GPU call (argument and quadrature validation), so they run without a GPU.
The codes that need device data (cross sections, NaN fluxes, iteration
limits, CG breakdown) are covered by tests/test_gpu_forms.py."""
import ctypes
import math

import numpy as np
import pytest

import sninputs
from test_library import library


def _quad(binding, om, w):
    om = np.ascontiguousarray(om, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    q = binding.sn_quad(len(w), om.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                        w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return q, (om, w)


def _create(lib, binding, mesh, quad, sig=True, eta=1.0):
    # host buffers stand in for the cross sections: every case below is
    # rejected before the library reads them
    dummy = np.ones(8)
    p = dummy.ctypes.data_as(ctypes.c_void_p) if sig else None
    out = ctypes.c_void_p(123)
    rc = binding.lib().sn_context_create(ctypes.byref(mesh), ctypes.byref(quad), p, p, float(eta), None,
                                         ctypes.byref(out))
    return rc, out, binding.lib().sn_last_error().decode()


def test_context_create_validation():
    lib, b = library()
    om, w = sninputs.level_symmetric(4, 2)
    good_mesh = b.sn_mesh(2, 4, 4, 1, 1.0, 1.0, 1.0)
    q, keep = _quad(b, om, w)
    cases = [
        ("dim 4", b.sn_mesh(4, 4, 4, 1, 1.0, 1.0, 1.0), q, True, 1.0, b.SN_ERR_INVALID),
        ("2D with nz 2", b.sn_mesh(2, 4, 4, 2, 1.0, 1.0, 1.0), q, True, 1.0, b.SN_ERR_INVALID),
        ("zero cells", b.sn_mesh(2, 0, 4, 1, 1.0, 1.0, 1.0), q, True, 1.0, b.SN_ERR_INVALID),
        ("negative width", b.sn_mesh(2, 4, 4, 1, -1.0, 1.0, 1.0), q, True, 1.0, b.SN_ERR_INVALID),
        ("NaN width", b.sn_mesh(2, 4, 4, 1, 1.0, float("nan"), 1.0), q, True, 1.0, b.SN_ERR_INVALID),
        ("NULL sigma", good_mesh, q, False, 1.0, b.SN_ERR_INVALID),
        ("NaN eta", good_mesh, q, True, float("nan"), b.SN_ERR_INVALID),
        ("order 5", b.sn_mesh(2, 4, 4, 1, 1.0, 1.0, 1.0, 5), q, True, 1.0, b.SN_ERR_INVALID),
        ("order -1", b.sn_mesh(2, 4, 4, 1, 1.0, 1.0, 1.0, -1), q, True, 1.0, b.SN_ERR_INVALID),
        ("order 2 in 3D", b.sn_mesh(3, 4, 4, 4, 1.0, 1.0, 1.0, 2), q, True, 1.0, b.SN_ERR_UNSUPPORTED),
    ]
    w_bad = w.copy()
    w_bad[0] *= 1.001                      # weights no longer sum to 4 pi
    q_sum, k1 = _quad(b, om, w_bad)
    cases.append(("weights not 4 pi", good_mesh, q_sum, True, 1.0, b.SN_ERR_INVALID))
    w_neg = w.copy()
    w_neg[0], w_neg[1] = -w_neg[0], w_neg[1] + 2 * w_neg[0]
    q_neg, k2 = _quad(b, om, w_neg)
    cases.append(("negative weight", good_mesh, q_neg, True, 1.0, b.SN_ERR_INVALID))
    om_nu = om.copy()
    om_nu[3] *= 1.01
    q_nu, k3 = _quad(b, om_nu, w)
    cases.append(("not a unit vector", good_mesh, q_nu, True, 1.0, b.SN_ERR_INVALID))
    om_zero = om.copy()
    om_zero[2] = [1.0, 0.0, 0.0]           # a direction along x: zero y component
    q_zero, k4 = _quad(b, om_zero, w)
    cases.append(("zero component", good_mesh, q_zero, True, 1.0, b.SN_ERR_UNSUPPORTED))
    q_empty = b.sn_quad(0, None, None)
    cases.append(("empty quadrature", good_mesh, q_empty, True, 1.0, b.SN_ERR_INVALID))
    for what, mesh, quad, sig, eta, code in cases:
        rc, out, msg = _create(lib, b, mesh, quad, sig, eta)
        assert rc == code, (what, rc, msg)
        assert out.value is None, what       # *out is cleared on failure
        assert msg, what


def test_null_arguments():
    lib, b = library()
    L = b.lib()
    dummy = np.zeros(8)
    p = dummy.ctypes.data_as(ctypes.c_void_p)
    st = b.sn_iter_stats()
    assert L.sn_sweep(None, None, None, None, 0, 0, p) == b.SN_ERR_INVALID
    assert L.sn_scalar_flux(None, p, 0, p) == b.SN_ERR_INVALID
    assert L.sn_dsa_thick_correct(None, p, p, p, None, None) == b.SN_ERR_INVALID
    o = b.sn_iter_opts(1e-8, 10, 1, 0, b.sn_dsa_opts(1e-4, 100, 0, 0), 0, None, 0, 0, 0)
    assert L.sn_source_iterate(None, None, None, p, ctypes.byref(o), ctypes.byref(st)) == b.SN_ERR_INVALID
    k = b.sn_krylov_opts(1e-8, 10, 30, 1, 0, b.sn_dsa_opts(1e-4, 100, 0, 0), 0)
    assert L.sn_krylov_solve(None, None, None, p, ctypes.byref(k), ctypes.byref(st)) == b.SN_ERR_INVALID
    assert L.sn_adjoint_source(None, None, -1, None, None) == b.SN_ERR_INVALID
    out = ctypes.c_double()
    assert L.sn_face_response(None, p, None, None, 1, ctypes.byref(out)) == b.SN_ERR_INVALID
    assert L.sn_adjoint_gradient(None, p, None, None, p, None, None, p, p) == b.SN_ERR_INVALID
    assert L.sn_gradient(None, p, p, 0, p, p, p, p) == b.SN_ERR_INVALID
    assert L.sn_response(None, None, None, -1, None, 0, ctypes.byref(out)) == b.SN_ERR_INVALID
    assert L.sn_set_kernel_timing(None, 1) == b.SN_ERR_INVALID
    assert L.sn_thick_count(None) == -1
    L.sn_context_destroy(None)
    bad = b.sn_mesh(3, 4, 4, 0, 1.0, 1.0, 1.0)
    assert L.sn_inflow_size(ctypes.byref(bad)) == -1
    assert L.sn_last_error().decode()
