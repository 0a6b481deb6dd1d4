"""Adjoint gradients of detector responses behind a torch.autograd.Function.

For the discrete block system (eq. system) A x = b with x = [psi_1..psi_D; phi]
and a linear response J, the adjoint (derived in the library's header) is a
source iteration with transposed sweeps:

  chi = sum_d w_d L_d^{-T} (g + Sigma_s chi),  psi~_d = L_d^{-T}(g + Sigma_s chi)

and the gradient with respect to per-cell log cross sections is

  dJ/dlog sigma_t,K = -sigma_t,K sum_d w_d psi~_d,K^T M_K psi_d,K
  dJ/dlog sigma_s,K =  sigma_s,K chi_K^T M_K phi_K / 4pi.

Two responses are supported:
  * a volume detector J = sum_c r_c int_c phi (adjoint source q = 4 pi r);
  * the partial outflow current through a domain face,
    J = sum_{d: Omega_d.n > 0} w_d (Omega_d.n) int_face psi_d (adjoint
    boundary data 1 on that face for the outgoing directions).

No angular flux of all directions is ever held.  The forward solve keeps
scalar-flux checkpoints (by default only the last, the converged phi*); the
face response and the backward contraction regenerate psi_d from phi* and
psi~_d from chi one octant at a time inside the library
(sn_face_response, sn_adjoint_gradient), and the adjoint sources come from
sn_adjoint_source.  This module only allocates the tensors and calls the C
ABI.
"""
from __future__ import annotations

import numpy as np
import torch

from .binding import (SN_FP64, Context, sn_adjoint_gradient, sn_adjoint_source, sn_face_response, sn_response,
                      sn_source_iterate)


def outgoing_face_inflow(dim, nx, ny, nz, omega, face):
    """Host copy of the transposed sweep's boundary data for the outflow
    current through `face` (2*axis + side): 1 on every node of that face for
    the directions leaving through it, laid out as the inflow of the reversed
    direction.  The library builds the same array on the device
    (sn_adjoint_source); this copy is for callers that need it on the host."""
    F = 2 if dim == 2 else 4
    sizes = [ny * nz * F, nx * nz * F] + ([nx * ny * F] if dim == 3 else [])
    offs = np.concatenate([[0], np.cumsum(sizes)])
    nbf = int(offs[-1])
    ax, side = face >> 1, face & 1
    out = np.zeros((omega.shape[0], nbf))
    for d in range(omega.shape[0]):
        on = omega[d, ax] * (1.0 if side else -1.0)
        if on > 0:
            out[d, offs[ax]:offs[ax + 1]] = 1.0
    return out


class Solver:
    """Problem description shared by forward and adjoint solves.

    ckpt_cap: scalar-flux checkpoints kept per forward solve (the last
    ckpt_cap iterates; the contraction uses the last one, phi*)."""

    def __init__(self, dim, nx, ny, nz, h, omega, w, q, eta=1.0, tol=1e-12, max_it=5000, cg_rtol=1e-12,
                 cg_maxit=10000, checkpoint=True, ckpt_cap=1):
        self.dim, self.nx, self.ny, self.nz = dim, nx, ny, nz
        self.h = tuple(h)
        self.omega = np.ascontiguousarray(omega, dtype=np.float64)
        self.w = np.ascontiguousarray(w, dtype=np.float64)
        self.q = q
        self.eta = eta
        self.tol, self.max_it, self.cg_rtol, self.cg_maxit = tol, max_it, cg_rtol, cg_maxit
        self.checkpoint = checkpoint
        self.ckpt_cap = max(1, int(ckpt_cap))
        self.nn = 4 if dim == 2 else 8
        self.ncells = nx * ny * nz
        self.memory = {}

    def context(self, sigma_t, sigma_s):
        return Context(self.dim, self.nx, self.ny, self.nz, self.h, self.omega, self.w,
                       sigma_t.contiguous(), sigma_s.contiguous(), eta=self.eta)

    def solve(self, ctx, q=None, inflow=None, transpose=False, checkpoint=False):
        dev = q.device if q is not None else torch.device("cuda")
        phi = torch.zeros((self.ncells, self.nn), dtype=torch.float64, device=dev)
        ck = None
        if checkpoint:
            ck = torch.empty((min(self.ckpt_cap, self.max_it), self.ncells, self.nn), dtype=torch.float64,
                             device=dev)
        r = sn_source_iterate(ctx, q, inflow, phi, tol=self.tol, max_it=self.max_it, use_dsa=True, prec=SN_FP64,
                              cg_rtol=self.cg_rtol, cg_maxit=self.cg_maxit, transpose=transpose, phi_ckpt=ck)
        if r["rc"] != 0:
            raise RuntimeError(f"source iteration did not converge (rc {r['rc']}, {r['iters']} iterations)")
        if ck is not None:
            # oldest first: the ring holds iterates max(0, iters - cap) .. iters - 1
            n, cap = r["iters"], ck.shape[0]
            ck = ck[:n] if n <= cap else torch.roll(ck, -(n % cap), dims=0)
        return phi, r, ck

    def memory_report(self, ck):
        """Bytes held for the gradient, next to what all of psi would take."""
        flux = self.ncells * self.nn * 8
        per_octant = -(-len(self.w) // (4 if self.dim == 2 else 8))
        return {"checkpoint_bytes": 0 if ck is None else int(ck.numel()) * 8, "phi_bytes": flux,
                "psi_all_directions_bytes": flux * len(self.w),
                "psi_octant_workspace_bytes": 2 * flux * per_octant}


class SnDetector(torch.autograd.Function):
    """J(log sigma_t, log sigma_s) for a volume detector (r) and/or an outflow
    face; backward returns grad_J * dJ/dlog sigma (adjoint, FP64)."""

    @staticmethod
    def forward(fctx, log_sigma_t, log_sigma_s, solver: Solver, r=None, face: int = -1):
        st = torch.exp(log_sigma_t.detach()).to(torch.float64).contiguous()
        ss = torch.exp(log_sigma_s.detach()).to(torch.float64).contiguous()
        ctx = solver.context(st, ss)
        phi, res, ck = solver.solve(ctx, q=solver.q, checkpoint=solver.checkpoint)
        # the converged flux is the last checkpoint; the contraction starts from it
        phi_star = ck[-1] if ck is not None else phi
        J = 0.0
        if r is not None:
            J += sn_response(ctx, r, phi_star)
        if face >= 0:
            J += sn_face_response(ctx, phi_star, solver.q, None, face)
        solver.memory = solver.memory_report(ck)
        fctx.solver, fctx.face, fctx.ctx = solver, face, ctx   # the context is freed with fctx
        fctx.forward_iters = res["iters"]
        fctx.save_for_backward(phi_star, r if r is not None else torch.empty(0, device=phi.device))
        return torch.tensor(J, dtype=torch.float64, device=phi.device)

    @staticmethod
    def backward(fctx, grad_J):
        phi, r = fctx.saved_tensors
        solver, face, ctx = fctx.solver, fctx.face, fctx.ctx
        dev = phi.device
        q_adj = torch.empty(solver.ncells, dtype=torch.float64, device=dev) if r.numel() else None
        inflow_adj = torch.empty((len(solver.w), ctx.nbf), dtype=torch.float64, device=dev) if face >= 0 else None
        sn_adjoint_source(ctx, r if r.numel() else None, face, q_adj, inflow_adj)
        chi, _, _ = solver.solve(ctx, q=q_adj, inflow=inflow_adj, transpose=True)
        gt = torch.empty(solver.ncells, dtype=torch.float64, device=dev)
        gs = torch.empty_like(gt)
        sn_adjoint_gradient(ctx, phi, solver.q, None, chi, q_adj, inflow_adj, gt, gs)
        return grad_J * gt, grad_J * gs, None, None, None


def detector_response(log_sigma_t, log_sigma_s, solver: Solver, r=None, face: int = -1):
    """J as a differentiable function of per-cell log cross sections."""
    return SnDetector.apply(log_sigma_t, log_sigma_s, solver, r, face)
