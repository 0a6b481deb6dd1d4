"""GPU path at the full workload sizes, in the launch configuration bench.py
times, against oracle values the CPU can produce:

* c2 (2D 256^2, S8): converged FP64 and FP32-form solutions against a full
  oracle solve (about 2-3 s on the host);
* c3 (3D 64^3, S8): converged FP64 and FP32-form solutions against sampled
  oracle values (fixture tests/golden/c3_phi.json, written by make_golden.py);
* c3 and c5 (3D 128^3, S12) single sweeps: one direction per octant, the
  whole psi field of that direction against the oracle's sweep of the same
  direction on the full grid.
"""
import json
import os

import numpy as np
import pytest

import oracle
import sninputs
from gpu_util import context, dev, rel_l2, rel_max, say
from sninputs import Problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _solve(p, prec, tol):
    from paper_2001_09196_amd import sn_source_iterate
    with context(p) as ctx:
        phi = torch.zeros((p.ncells, p.nn), dtype=torch.float64, device="cuda")
        r = sn_source_iterate(ctx, dev(p.q), None, phi, tol=tol, max_it=3000, use_dsa=True, prec=prec,
                              cg_rtol=1e-8, cg_maxit=20000)
        return phi.cpu().numpy(), r


def test_c2_converged_fp64_fp32_vs_oracle():
    p = sninputs.config("c2")
    say("c2 oracle solve")
    ref = oracle.source_iterate(p, tol=1e-12, max_it=3000, use_dsa=True, cg_rtol=1e-10)["phi"]
    say("c2 gpu fp64")
    g64, r64 = _solve(p, 0, 1e-12)
    say("c2 gpu fp32 form")
    g32, r32 = _solve(p, 1, 1e-8)
    assert r64["rc"] == 0 and r32["rc"] == 0
    e64, e32 = rel_l2(g64, ref), rel_l2(g32, ref)
    say(f"  c2: fp64 {e64:.2e} ({r64['iters']} it), fp32 form {e32:.2e} ({r32['iters']} it, "
        f"{r32['fp64_checks']} FP64 sweeps)")
    assert e64 <= 1e-10
    assert e32 <= 1e-5


def test_c3_converged_vs_oracle_sample():
    path = os.path.join(GOLD, "c3_phi.json")
    if not os.path.exists(path):
        pytest.skip("fixture c3_phi.json not generated")
    gold = json.load(open(path))
    idx = np.array(gold["sample_index"])
    ref = np.array(gold["sample_value"])
    p = sninputs.config("c3")
    say("c3 gpu fp64")
    g64, r64 = _solve(p, 0, 1e-12)
    say("c3 gpu fp32 form")
    g32, r32 = _solve(p, 1, 1e-8)
    assert r64["rc"] == 0 and r32["rc"] == 0
    for name, g, bar in (("fp64", g64, 1e-9), ("fp32", g32, 1e-5)):
        es = np.linalg.norm(g.ravel()[idx] - ref) / np.linalg.norm(ref)
        en = abs(np.linalg.norm(g) - gold["norm2"]) / gold["norm2"]
        say(f"  c3 {name}: sample rel l2 {es:.2e}, norm {en:.2e}")
        assert es <= bar and en <= bar


@pytest.mark.parametrize("name", ["c3", "c5"])
def test_fullsize_sweep_sampled_directions(name):
    """Full-grid sweep (FP64 and FP32) for one direction per octant against
    the oracle's sweep of that single direction."""
    from paper_2001_09196_amd import sn_sweep
    p = sninputs.config(name)
    rng = np.random.default_rng(3)
    phi = rng.uniform(0, 1, (p.ncells, p.nn))
    per = p.ndirs // 8
    dirs = [o * per + int(rng.integers(0, per)) for o in range(8)]
    with context(p) as ctx:
        for prec, dt, bar in ((0, torch.float64, 1e-12), (1, torch.float32, 2e-5)):
            psi = torch.empty((p.ncells, p.ndirs, p.nn), dtype=dt, device="cuda")
            say(f"{name} full sweep prec={prec}")
            sn_sweep(ctx, dev(phi), dev(p.q), None, False, prec, psi)
            torch.cuda.synchronize()
            for d in dirs:
                p1 = Problem(p.name, p.dim, p.nx, p.ny, p.nz, p.h, p.sigma_t, p.sigma_s, p.q,
                             p.omega[d:d + 1], p.w[d:d + 1])
                ref = oracle.sweep(p1, phi, p.q)[:, 0, :]
                got = psi[:, d, :].double().cpu().numpy()
                err = rel_max(got, ref)
                say(f"  dir {d}: rel max {err:.2e}")
                assert err <= bar
            del psi
            torch.cuda.empty_cache()
