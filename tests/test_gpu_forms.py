"""GPU parity of the iteration forms against the oracle, through the C ABI:

* source iteration with S12 (six direction groups per octant, the C5 layout)
  on a ragged 3D mesh, per iterate, FP64 and the plain FP32 form, forward and
  transposed;
* the triangular heterogeneous DSA (Alg. 1) per iterate and converged;
* the Krylov solve (flexible GMRES on eq. schur) against the oracle's GMRES:
  residual histories and converged fluxes, with restarts and both DSA forms;
* the per-octant adjoint contraction and face response against the full-psi
  kernels and the oracle;
* error codes that need device data (cross sections, NaN fluxes, iteration
  limits).
"""
import math

import numpy as np
import pytest

import oracle
import sninputs
from gpu_util import context, dev, random_problem, rel_l2, rel_max, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _zeros(p):
    return torch.zeros((p.ncells, p.nn), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("transpose", [False, True])
def test_si_per_iterate_s12(transpose):
    from paper_2001_09196_amd import sn_source_iterate
    p = random_problem(3, 20, 9, 7, order=12, seed=71 + int(transpose))
    assert p.ndirs == 168
    rng = np.random.default_rng(73)
    inflow = rng.uniform(0, 1, (p.ndirs, sninputs.inflow_size(p.dim, p.nx, p.ny, p.nz)))
    k = 4
    say(f"SI S12 per-iterate transpose={transpose}")
    ref = oracle.source_iterate(p, tol=0.0, max_it=k, use_dsa=True, cg_rtol=1e-13, transpose=transpose,
                                inflow=inflow)
    with context(p) as ctx:
        for prec, bar in ((0, 1e-12), (1, 2e-5)):
            phi = _zeros(p)
            r = sn_source_iterate(ctx, dev(p.q), dev(inflow), phi, tol=0.0, max_it=k, use_dsa=True, prec=prec,
                                  cg_rtol=1e-13, cg_maxit=5000, transpose=transpose)
            err = rel_l2(phi.cpu().numpy(), ref["phi"])
            say(f"  prec {prec}: {err:.2e}")
            assert r["iters"] == k and r["fp64_checks"] == 0
            assert err <= bar
            if prec == 0:
                assert np.allclose(r["res_hist"], ref["res_hist"], rtol=1e-9, atol=0)


@pytest.mark.parametrize("case", ["c1", "2d", "3d"])
def test_triangular_per_iterate(case):
    from paper_2001_09196_amd import SN_DSA_TRIANGULAR, sn_source_iterate
    if case == "c1":
        p = sninputs.config("c1")
    elif case == "2d":
        p = random_problem(2, 33, 21, 1, order=8, seed=81)
    else:
        p = random_problem(3, 13, 9, 6, order=4, seed=82)
    say(f"triangular DSA per iterate {case}")
    with context(p) as ctx:
        for k in (1, 4):
            ref = oracle.source_iterate(p, tol=0.0, max_it=k, use_dsa=True, cg_rtol=1e-13, dsa_form=1)
            phi = _zeros(p)
            r = sn_source_iterate(ctx, dev(p.q), None, phi, tol=0.0, max_it=k, use_dsa=True, cg_rtol=1e-13,
                                  cg_maxit=5000, dsa_form=SN_DSA_TRIANGULAR)
            err = rel_l2(phi.cpu().numpy(), ref["phi"])
            say(f"  k={k}: {err:.2e}, sweeps {r['sweeps']}")
            assert err <= 1e-10
            assert np.allclose(r["res_hist"], ref["res_hist"], rtol=1e-9, atol=0)
            # two sweeps per iteration (from phi = 0 the first sweep also gives b)
            assert r["sweeps"] == 2 * k


def test_triangular_converged_c1():
    from paper_2001_09196_amd import SN_DSA_TRIANGULAR, sn_source_iterate
    p = sninputs.config("c1")
    ref = oracle.source_iterate(p, tol=1e-13, max_it=3000, use_dsa=True, cg_rtol=1e-13)
    say("triangular DSA converged c1")
    with context(p) as ctx:
        phi = _zeros(p)
        r = sn_source_iterate(ctx, dev(p.q), None, phi, tol=1e-12, max_it=3000, use_dsa=True, cg_rtol=1e-13,
                              cg_maxit=5000, dsa_form=SN_DSA_TRIANGULAR)
        assert r["rc"] == 0
        assert rel_l2(phi.cpu().numpy(), ref["phi"]) <= 1e-10


@pytest.mark.parametrize("case,use_dsa,form,restart", [("c1", True, 0, 30), ("c1", False, 0, 30),
                                                        ("c1", True, 1, 30), ("2d", True, 0, 5),
                                                        ("3d", True, 0, 30), ("3d", True, 1, 8)])
def test_krylov_vs_oracle(case, use_dsa, form, restart):
    from paper_2001_09196_amd import sn_krylov_solve
    if case == "c1":
        p = sninputs.config("c1")
    elif case == "2d":
        p = random_problem(2, 27, 19, 1, order=8, seed=91)
    else:
        p = random_problem(3, 14, 10, 7, order=8, seed=92)
    say(f"Krylov {case} dsa={use_dsa} form={form} restart={restart}")
    k = 12
    ref = oracle.gmres(p, tol=0.0, max_it=k, restart=restart, use_dsa=use_dsa, dsa_form=form, cg_rtol=1e-13)
    conv = oracle.gmres(p, tol=1e-12, max_it=3000, restart=restart, use_dsa=use_dsa, dsa_form=form, cg_rtol=1e-13)
    with context(p) as ctx:
        phi = _zeros(p)
        r = sn_krylov_solve(ctx, dev(p.q), None, phi, tol=0.0, max_it=k, restart=restart, use_dsa=use_dsa,
                            dsa_form=form, cg_rtol=1e-13, cg_maxit=5000)
        assert r["iters"] == k
        err_k = rel_l2(phi.cpu().numpy(), ref["phi"])
        hist = np.max(np.abs(r["res_hist"] - ref["res_hist"]) / ref["res_hist"])
        phi = _zeros(p)
        rc = sn_krylov_solve(ctx, dev(p.q), None, phi, tol=1e-12, max_it=3000, restart=restart, use_dsa=use_dsa,
                             dsa_form=form, cg_rtol=1e-13, cg_maxit=5000)
        err_c = rel_l2(phi.cpu().numpy(), conv["phi"])
    say(f"  after {k}: {err_k:.2e}, history {hist:.2e}; converged in {rc['iters']} (oracle {conv['iters']}): "
        f"{err_c:.2e}")
    assert err_k <= 1e-9 and hist <= 1e-7
    assert rc["rc"] == 0 and conv["rc"] == 0
    assert err_c <= 1e-10
    assert abs(rc["iters"] - conv["iters"]) <= 2


@pytest.mark.parametrize("k,cdt", [(5, 1e3), (2, 1.0)])
def test_crooked_pipe_het_and_full_dsa(k, cdt):
    """The crooked-pipe stand-in of Sec. 4.1 (Table problems #5 and #2, S8,
    the paper's 0.5-unit cells): three source iterations with the
    heterogeneous DSA (eta = 1) and with full DSA (eta = 0: every cell in the
    diffusion solve, defined here since no cell is void), and twelve GMRES
    iterations with each, all with the CG at 1e-13, against the oracle."""
    import dataclasses

    from paper_2001_09196_amd import sn_krylov_solve, sn_source_iterate
    base = sninputs.crooked_pipe(k, cdt, cells_per_unit=2)
    for eta in (1.0, 0.0):
        p = dataclasses.replace(base, eta=eta)
        say(f"crooked pipe #{k} cdt={cdt} eta={eta}")
        ref = oracle.source_iterate(p, tol=0.0, max_it=3, use_dsa=True, cg_rtol=1e-13)
        refk = oracle.gmres(p, tol=0.0, max_it=12, restart=30, use_dsa=True, cg_rtol=1e-13)
        with context(p) as ctx:
            phi = _zeros(p)
            r = sn_source_iterate(ctx, dev(p.q), None, phi, tol=0.0, max_it=3, use_dsa=True, cg_rtol=1e-13,
                                  cg_maxit=100000)
            e_si = rel_l2(phi.cpu().numpy(), ref["phi"])
            phi = _zeros(p)
            rk = sn_krylov_solve(ctx, dev(p.q), None, phi, tol=0.0, max_it=12, restart=30, use_dsa=True,
                                 cg_rtol=1e-13, cg_maxit=100000)
            e_k = rel_l2(phi.cpu().numpy(), refk["phi"])
        say(f"  SI {e_si:.2e} (CG {list(r['cg_hist'])}), GMRES {e_k:.2e}")
        assert r["iters"] == 3 and rk["iters"] == 12
        assert e_si <= 1e-10 and e_k <= 1e-9


@pytest.mark.parametrize("dim,shape", [(2, (19, 13, 1)), (3, (11, 8, 6))])
def test_octant_adjoint_vs_full_psi_and_oracle(dim, shape):
    """sn_adjoint_gradient (psi regenerated one octant at a time) against the
    full-psi contraction (sn_gradient) and the oracle's gradient, for a volume
    detector plus inflow data; sn_face_response against sn_response on a full
    psi and against the oracle's sweep."""
    from paper_2001_09196_amd import (sn_adjoint_gradient, sn_adjoint_source, sn_face_response, sn_gradient,
                                      sn_response, sn_sweep)
    p = random_problem(dim, *shape, order=4, seed=101 + dim)
    rng = np.random.default_rng(102)
    phi = rng.uniform(0, 1, (p.ncells, p.nn))
    chi = rng.uniform(0, 1, (p.ncells, p.nn))
    r = np.zeros(p.ncells)
    r[rng.choice(p.ncells, 5, replace=False)] = 1.0
    nbf = sninputs.inflow_size(p.dim, p.nx, p.ny, p.nz)
    inflow = rng.uniform(0, 1, (p.ndirs, nbf))
    face = 1
    say(f"octant adjoint {p.name}")
    with context(p) as ctx:
        qa = torch.empty(p.ncells, dtype=torch.float64, device="cuda")
        ia = torch.empty((p.ndirs, nbf), dtype=torch.float64, device="cuda")
        sn_adjoint_source(ctx, dev(r), face, qa, ia)
        qa_h, ia_h = qa.cpu().numpy(), ia.cpu().numpy()
        assert np.array_equal(qa_h, 4 * math.pi * r)
        F = 2 if dim == 2 else 4
        for d in range(p.ndirs):
            expect = np.zeros(nbf)
            if p.omega[d, 0] > 0:
                expect[:p.ny * p.nz * F] = 1.0
            assert np.array_equal(ia_h[d], expect)
        gt, gs = torch.empty(p.ncells, dtype=torch.float64, device="cuda"), torch.empty(p.ncells,
                                                                                       dtype=torch.float64,
                                                                                       device="cuda")
        sn_adjoint_gradient(ctx, dev(phi), dev(p.q), dev(inflow), dev(chi), qa, ia, gt, gs)
        psi = torch.empty((p.ncells, p.ndirs, p.nn), dtype=torch.float64, device="cuda")
        psia = torch.empty_like(psi)
        sn_sweep(ctx, dev(phi), dev(p.q), dev(inflow), False, 0, psi)
        sn_sweep(ctx, dev(chi), qa, ia, True, 0, psia)
        gt2, gs2 = torch.empty_like(gt), torch.empty_like(gs)
        sn_gradient(ctx, psi, psia, 0, dev(phi), dev(chi), gt2, gs2)
        J_full = sn_response(ctx, None, None, face, psi)
        J_oct = sn_face_response(ctx, dev(phi), dev(p.q), dev(inflow), face)
        gt, gs, gt2, gs2 = (t.cpu().numpy() for t in (gt, gs, gt2, gs2))
    ref_psi = oracle.sweep(p, phi, p.q, inflow=inflow)
    ref_psia = oracle.sweep(p, chi, qa_h, inflow=ia_h, transpose=True)
    gt_o, gs_o = oracle.gradient(p, ref_psi, ref_psia, phi, chi)
    say(f"  vs full psi {rel_max(gt, gt2):.2e} / {rel_max(gs, gs2):.2e}; vs oracle {rel_max(gt, gt_o):.2e}; "
        f"face {J_oct:.12e} vs {J_full:.12e}")
    assert rel_max(gt, gt2) <= 1e-13 and np.array_equal(gs, gs2)
    assert rel_max(gt, gt_o) <= 1e-11 and rel_max(gs, gs_o) <= 1e-12
    assert abs(J_oct - J_full) <= 1e-13 * abs(J_full)


def test_error_codes_on_device():
    from paper_2001_09196_amd import Context, SnError, sn_dsa_thick_correct, sn_krylov_solve, sn_source_iterate
    from paper_2001_09196_amd.binding import (SN_ERR_CG_BREAKDOWN, SN_ERR_DIVERGED, SN_ERR_INVALID,
                                              SN_ERR_NOT_CONVERGED)
    p = sninputs.config("c1")
    say("error codes")
    ss_big = p.sigma_s.copy()
    ss_big[5] = p.sigma_t[5] * 1.5 + 1.0
    st_nan = p.sigma_t.copy()
    st_nan[7] = np.nan
    ss_neg = p.sigma_s.copy()
    ss_neg[9] = -0.1
    for what, st, ss in (("sigma_s > sigma_t", p.sigma_t, ss_big), ("NaN sigma_t", st_nan, p.sigma_s),
                         ("negative sigma_s", p.sigma_t, ss_neg)):
        with pytest.raises(SnError) as e:
            Context(p.dim, p.nx, p.ny, p.nz, p.h, p.omega, p.w, dev(st), dev(ss), eta=p.eta)
        assert e.value.code == SN_ERR_INVALID, what
    with context(p) as ctx:
        # iteration limit: phi holds the last iterate, stats are filled
        phi = _zeros(p)
        r = sn_source_iterate(ctx, dev(p.q), None, phi, tol=1e-12, max_it=1, use_dsa=True, cg_rtol=1e-13,
                              cg_maxit=5000)
        ref = oracle.source_iterate(p, tol=0.0, max_it=1, use_dsa=True, cg_rtol=1e-13)
        assert r["rc"] == SN_ERR_NOT_CONVERGED and r["iters"] == 1
        assert rel_l2(phi.cpu().numpy(), ref["phi"]) <= 1e-12
        assert r["res_hist"][0] == pytest.approx(ref["res_hist"][0], rel=1e-12)
        # a NaN initial guess: the residual is not finite (DIVERGED), and the
        # diffusion CG of its residual breaks down (p^T D p is not positive)
        nan = torch.full((p.ncells, p.nn), float("nan"), dtype=torch.float64, device="cuda")
        r = sn_source_iterate(ctx, dev(p.q), None, nan.clone(), tol=1e-8, max_it=5, use_dsa=False)
        assert r["rc"] == SN_ERR_DIVERGED
        with pytest.raises(SnError) as e:
            sn_source_iterate(ctx, dev(p.q), None, nan.clone(), tol=1e-8, max_it=5, use_dsa=True, cg_rtol=1e-8)
        assert e.value.code == SN_ERR_CG_BREAKDOWN
        with pytest.raises(SnError) as e:
            sn_dsa_thick_correct(ctx, nan, dev(np.ones((p.ncells, p.nn))), _zeros(p))
        assert e.value.code == SN_ERR_CG_BREAKDOWN
        # option checks
        for kw in ({"cg_maxit": 0}, {"mass_kind": 3}, {"dsa_form": 2}, {"tol": float("nan")}):
            with pytest.raises(SnError) as e:
                sn_source_iterate(ctx, dev(p.q), None, _zeros(p), **{"max_it": 3, **kw})
            assert e.value.code == SN_ERR_INVALID, kw
        for kw in ({"restart": 0}, {"restart": 201}):
            with pytest.raises(SnError) as e:
                sn_krylov_solve(ctx, dev(p.q), None, _zeros(p), **kw)
            assert e.value.code == SN_ERR_INVALID, kw
        r = sn_krylov_solve(ctx, dev(p.q), None, _zeros(p), tol=1e-12, max_it=2)
        assert r["rc"] == SN_ERR_NOT_CONVERGED and r["iters"] == 2
