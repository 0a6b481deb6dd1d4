"""Write oracle-derived fixtures for the full-size GPU checks.

Calls only the CPU oracle (oracle/) and the seeded input module (sninputs);
nothing here touches the GPU path.  Each fixture is small JSON: norms of the
full oracle vectors plus values at seeded sample indices, so the GPU tests
can compare sampled outputs at the full workload sizes.

  python tests/golden/make_golden.py c4adj   # C4 adjoint gradients (FD cells + sample)
  python tests/golden/make_golden.py c3      # C3 converged scalar flux (sample)
  python tests/golden/make_golden.py c5      # C5 converged scalar flux (sample), long
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
    sample = np.sort(np.random.default_rng(7).choice(p.ncells, 256, replace=False))
    _dump("c4_adjoint.json", {
        "what": "oracle adjoint of J = sum over cells [120,128)^2 of int phi, C4 (128^2, S8, jitter)",
        "settings": {k: v for k, v in kw.items()},
        "forward_iters": fwd["iters"], "adjoint_iters": adj["iters"],
        "forward_rc": fwd["rc"], "adjoint_rc": adj["rc"],
        "J": J,
        "fd_cells": fd.tolist(), "g_t_fd_cells": gt[fd].tolist(), "g_s_fd_cells": gs[fd].tolist(),
        "sample_cells": sample.tolist(), "g_t_sample": gt[sample].tolist(), "g_s_sample": gs[sample].tolist(),
        "g_t_norm": float(np.linalg.norm(gt)), "g_s_norm": float(np.linalg.norm(gs)),
        "g_t_maxabs": float(np.max(np.abs(gt))), "g_s_maxabs": float(np.max(np.abs(gs))),
        "seconds": time.time() - t0, "threads": oracle.num_threads(),
    })


def flux_sample(name, tol):
    p = sninputs.config(name)
    t0 = time.time()
    r = oracle.source_iterate(p, tol=tol, max_it=2000, use_dsa=True, cg_rtol=1e-10, cg_maxit=100000)
    phi = r["phi"]
    idx = np.sort(np.random.default_rng(11).choice(p.ncells * p.nn, 4096, replace=False))
    _dump(f"{name}_phi.json", {
        "what": f"oracle converged scalar flux for {name} (FP64, het-DSA, tol {tol})",
        "iters": r["iters"], "rc": r["rc"], "res_last": float(r["res_hist"][-1]),
        "norm2": float(np.linalg.norm(phi)), "maxabs": float(np.max(np.abs(phi))),
        "sample_index": idx.tolist(), "sample_value": phi.ravel()[idx].tolist(),
        "seconds": time.time() - t0, "threads": oracle.num_threads(),
    })


if __name__ == "__main__":
    for what in sys.argv[1:]:
        if what == "c4adj":
            c4_adjoint()
        elif what in ("c3", "c5"):
            flux_sample(what, 1e-11)
        else:
            raise SystemExit(f"unknown fixture {what}")
        print("wrote", what, flush=True)
