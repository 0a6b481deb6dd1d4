"""Write oracle-derived fixtures for the full-size GPU checks.

Calls only the CPU oracle (oracle/) and the seeded input module (sninputs);
nothing here touches the GPU path.  Each fixture is small JSON: norms of the
full oracle vectors plus values at seeded sample indices, so the GPU tests
can compare sampled outputs at the full workload sizes.

  python tests/golden/make_golden.py c4adj   # C4 adjoint gradients (FD cells + sample)
  python tests/golden/make_golden.py c3      # C3 converged scalar flux (sample)
  python tests/golden/make_golden.py c5iter  # C5 after three source iterations (sample)
  python tests/golden/make_golden.py c5      # C5 converged flux and outflow adjoint (samples), hours

Converged fixtures stop at a relative residual of 1e-13 (the FP64 floor of
these problems is near 1e-14), so that a GPU solve stopped at the same
residual agrees with them to about 1e-11 and the 1e-10 bar tests the path,
not the stop.
"""
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import sninputs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def _dump(name, obj):
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(obj, f, indent=1)


def c4_adjoint():
    p = sninputs.config("c4")
    r = np.zeros(p.ncells)
    for j in range(120, 128):
        for i in range(120, 128):
            r[j * p.nx + i] = 1.0
    qadj = 4 * math.pi * r
    kw = dict(tol=6e-14, max_it=400, use_dsa=True, cg_rtol=1e-8, cg_maxit=100000)
    t0 = time.time()
    fwd = oracle.source_iterate(p, **kw)
    adj = oracle.source_iterate(p, transpose=True, q=qadj, **kw)
    psi = oracle.sweep(p, fwd["phi"], p.q)
    psia = oracle.sweep(p, adj["phi"], qadj, transpose=True)
    gt, gs = oracle.gradient(p, psi, psia, fwd["phi"], adj["phi"])
    vol = 1.0
    J = float(np.sum(r[:, None] * fwd["phi"]) * vol / 4.0)
    fd = sninputs.fd_cells(p, 20, seed=2)
    # FD cells where each gradient is large (|g| >= 1e-3 max|g|), so that the
    # finite-difference bar bites on cells that carry the response
    ok = p.sigma_t > 0
    ok &= ~p.meta["clipped"]
    big_t = np.nonzero(ok & (np.abs(gt) >= 1e-3 * np.max(np.abs(gt))))[0]
    big_s = np.nonzero(ok & (np.abs(gs) >= 1e-3 * np.max(np.abs(gs))))[0]
    fd_t = np.sort(np.random.default_rng(3).choice(big_t, 20, replace=False))
    fd_s = np.sort(np.random.default_rng(4).choice(big_s, 20, replace=False))
    sample = np.sort(np.random.default_rng(7).choice(p.ncells, 256, replace=False))
    _dump("c4_adjoint.json", {
        "what": "oracle adjoint of J = sum over cells [120,128)^2 of int phi, C4 (128^2, S8, jitter)",
        "settings": {k: v for k, v in kw.items()},
        "forward_iters": fwd["iters"], "adjoint_iters": adj["iters"],
        "forward_rc": fwd["rc"], "adjoint_rc": adj["rc"],
        "J": J,
        "fd_cells": fd.tolist(), "g_t_fd_cells": gt[fd].tolist(), "g_s_fd_cells": gs[fd].tolist(),
        "fd_cells_big_t": fd_t.tolist(), "g_t_fd_cells_big_t": gt[fd_t].tolist(),
        "fd_cells_big_s": fd_s.tolist(), "g_s_fd_cells_big_s": gs[fd_s].tolist(),
        "sample_cells": sample.tolist(), "g_t_sample": gt[sample].tolist(), "g_s_sample": gs[sample].tolist(),
        "g_t_norm": float(np.linalg.norm(gt)), "g_s_norm": float(np.linalg.norm(gs)),
        "g_t_maxabs": float(np.max(np.abs(gt))), "g_s_maxabs": float(np.max(np.abs(gs))),
        "seconds": time.time() - t0, "threads": oracle.num_threads(),
    })


def _sample(n, seed=11, count=4096):
    return np.sort(np.random.default_rng(seed).choice(n, count, replace=False))


def flux_sample(name, tol):
    p = sninputs.config(name)
    t0 = time.time()
    r = oracle.source_iterate(p, tol=tol, max_it=2000, use_dsa=True, cg_rtol=1e-8, cg_maxit=100000)
    phi = r["phi"]
    idx = _sample(p.ncells * p.nn)
    _dump(f"{name}_phi.json", {
        "what": f"oracle converged scalar flux for {name} (FP64, het-DSA, tol {tol})",
        "iters": r["iters"], "rc": r["rc"], "res_last": float(r["res_hist"][-1]),
        "norm2": float(np.linalg.norm(phi)), "maxabs": float(np.max(np.abs(phi))),
        "sample_index": idx.tolist(), "sample_value": phi.ravel()[idx].tolist(),
        "seconds": time.time() - t0, "threads": oracle.num_threads(),
    })
    print(f"{name}: {r['iters']} iterations, residual {r['res_hist'][-1]:.2e}, {time.time() - t0:.0f} s",
          flush=True)
    return p, phi


def c5_iterates(k=3):
    """C5 after k source iterations from phi = 0 with the thick-region solve
    at a CG tolerance of 1e-13 (per-iterate parity of the production path)."""
    p = sninputs.config("c5")
    t0 = time.time()
    r = oracle.source_iterate(p, tol=0.0, max_it=k, use_dsa=True, cg_rtol=1e-13, cg_maxit=100000)
    phi = r["phi"]
    idx = _sample(p.ncells * p.nn)
    _dump("c5_iter3.json", {
        "what": f"oracle scalar flux of c5 after {k} source iterations with het-DSA (CG to 1e-13)",
        "iters": r["iters"], "res_hist": r["res_hist"].tolist(), "cg_hist": r["cg_hist"].tolist(),
        "norm2": float(np.linalg.norm(phi)), "maxabs": float(np.max(np.abs(phi))),
        "sample_index": idx.tolist(), "sample_value": phi.ravel()[idx].tolist(),
        "seconds": time.time() - t0, "threads": oracle.num_threads(),
    })


def c5_adjoint(p, phi, tol):
    """Outflow partial current through the x = 128 face of c5: adjoint flux
    (transposed source iteration with unit data on that face for the
    directions leaving through it) and the gradient, computed eight
    directions at a time so that no full angular flux is held."""
    t0 = time.time()
    # transposed-sweep boundary data: 1 on the x = L face for every direction
    # with mu > 0 (it leaves through that face), in the x-face slot of the
    # inflow layout (the upwind x face of the reversed direction)
    inflow = np.zeros((p.ndirs, sninputs.inflow_size(p.dim, p.nx, p.ny, p.nz)))
    inflow[p.omega[:, 0] > 0, :p.ny * p.nz * 4] = 1.0
    adj = oracle.source_iterate(p, tol=tol, max_it=2000, use_dsa=True, cg_rtol=1e-8, cg_maxit=100000,
                                transpose=True, q=np.zeros(p.ncells), inflow=inflow)
    chi = adj["phi"]
    print(f"c5 adjoint: {adj['iters']} iterations, residual {adj['res_hist'][-1]:.2e}, {time.time() - t0:.0f} s",
          flush=True)
    gt = np.zeros(p.ncells)
    gs = None
    for d0 in range(0, p.ndirs, 8):
        sel = slice(d0, min(d0 + 8, p.ndirs))
        p1 = sninputs.Problem(p.name, p.dim, p.nx, p.ny, p.nz, p.h, p.sigma_t, p.sigma_s, p.q,
                              p.omega[sel].copy(), p.w[sel].copy())
        psi = oracle.sweep(p1, phi, p.q)
        psia = oracle.sweep(p1, chi, None, inflow=np.ascontiguousarray(inflow[sel]), transpose=True)
        a, b = oracle.gradient(p1, psi, psia, phi, chi)
        gt += a
        if gs is None:
            gs = b
        del psi, psia
    # J by reciprocity: sum_c (q_c / 4pi) int_c chi, int_c chi = (h^3 / 8) sum of the cell's nodal values
    vol = p.h[0] * p.h[1] * p.h[2]
    J = float(np.sum(p.q / (4 * math.pi) * chi.sum(axis=1)) * vol / 8.0)
    sample = np.sort(np.random.default_rng(7).choice(p.ncells, 512, replace=False))
    edge = (np.arange(p.ncells) % p.nx) >= p.nx - 8
    big = np.nonzero(edge & (np.abs(gt) >= 1e-3 * np.max(np.abs(gt))))[0]
    near = np.sort(np.random.default_rng(8).choice(big, min(256, big.size), replace=False))
    _dump("c5_adjoint.json", {
        "what": "oracle adjoint of the outflow partial current through x = 128, c5 (128^3, S12)",
        "adjoint_iters": adj["iters"], "adjoint_res_last": float(adj["res_hist"][-1]), "J": J,
        "chi_norm2": float(np.linalg.norm(chi)),
        "sample_cells": sample.tolist(), "g_t_sample": gt[sample].tolist(), "g_s_sample": gs[sample].tolist(),
        "near_cells": near.tolist(), "g_t_near": gt[near].tolist(), "g_s_near": gs[near].tolist(),
        "g_t_norm": float(np.linalg.norm(gt)), "g_s_norm": float(np.linalg.norm(gs)),
        "g_t_maxabs": float(np.max(np.abs(gt))), "g_s_maxabs": float(np.max(np.abs(gs))),
        "seconds": time.time() - t0, "threads": oracle.num_threads(),
    })


if __name__ == "__main__":
    for what in sys.argv[1:]:
        if what == "c4adj":
            c4_adjoint()
        elif what == "c3":
            flux_sample(what, 1e-13)
        elif what == "c5iter":
            c5_iterates()
        elif what == "c5":
            p, phi = flux_sample(what, 1e-13)
            c5_adjoint(p, phi, 1e-13)
        else:
            raise SystemExit(f"unknown fixture {what}")
        print("wrote", what, flush=True)
