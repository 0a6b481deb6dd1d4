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

The forward solve stores the scalar flux after every source iteration
(checkpoints); the backward pass regenerates psi from the converged phi with
one sweep instead of storing psi across iterations.  Every step runs in the
library's kernels; this module only builds the adjoint inputs and calls the
C ABI.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .binding import (SN_FP64, Context, sn_gradient, sn_response, sn_source_iterate, sn_sweep)


def outgoing_face_inflow(dim, nx, ny, nz, omega, face):
    """Boundary data for the transposed sweep: 1 on every node of `face`
    (2*axis + side) for the directions leaving the domain through it, laid
    out as the inflow of the reversed direction (the face is upwind for
    -Omega_d exactly when Omega_d leaves through it)."""
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
    """Problem description shared by forward and adjoint solves."""

    def __init__(self, dim, nx, ny, nz, h, omega, w, q, eta=1.0, tol=1e-12, max_it=5000, cg_rtol=1e-12,
                 cg_maxit=10000, checkpoint=True, ckpt_bytes=8 << 30):
        self.dim, self.nx, self.ny, self.nz = dim, nx, ny, nz
        self.h = tuple(h)
        self.omega = np.ascontiguousarray(omega, dtype=np.float64)
        self.w = np.ascontiguousarray(w, dtype=np.float64)
        self.q = q
        self.eta = eta
        self.tol, self.max_it, self.cg_rtol, self.cg_maxit = tol, max_it, cg_rtol, cg_maxit
        self.checkpoint = checkpoint
        self.ckpt_bytes = int(ckpt_bytes)    # device memory for flux checkpoints (last iterates kept)
        self.nn = 4 if dim == 2 else 8
        self.ncells = nx * ny * nz

    def context(self, sigma_t, sigma_s):
        return Context(self.dim, self.nx, self.ny, self.nz, self.h, self.omega, self.w,
                       sigma_t.contiguous(), sigma_s.contiguous(), eta=self.eta)

    def solve(self, ctx, q=None, inflow=None, transpose=False, checkpoint=False):
        dev = q.device if q is not None else torch.device("cuda")
        phi = torch.zeros((self.ncells, self.nn), dtype=torch.float64, device=dev)
        ck = None
        if checkpoint:
            cap = max(1, min(self.max_it, self.ckpt_bytes // (self.ncells * self.nn * 8)))
            ck = torch.empty((cap, self.ncells, self.nn), dtype=torch.float64, device=dev)
        r = sn_source_iterate(ctx, q, inflow, phi, tol=self.tol, max_it=self.max_it, use_dsa=True, prec=SN_FP64,
                              cg_rtol=self.cg_rtol, cg_maxit=self.cg_maxit, transpose=transpose, phi_ckpt=ck)
        if r["rc"] != 0:
            raise RuntimeError(f"source iteration did not converge (rc {r['rc']}, {r['iters']} iterations)")
        if ck is not None:
            # oldest first: the ring holds iterates max(0, iters - cap) .. iters - 1
            n, cap = r["iters"], ck.shape[0]
            ck = ck[:n] if n <= cap else torch.roll(ck, -(n % cap), dims=0)
        return phi, r, ck


class SnDetector(torch.autograd.Function):
    """J(log sigma_t, log sigma_s) for a volume detector (r) and/or an outflow
    face; backward returns grad_J * dJ/dlog sigma (adjoint, FP64)."""

    @staticmethod
    def forward(fctx, log_sigma_t, log_sigma_s, solver: Solver, r=None, face: int = -1):
        st = torch.exp(log_sigma_t.detach()).to(torch.float64).contiguous()
        ss = torch.exp(log_sigma_s.detach()).to(torch.float64).contiguous()
        ctx = solver.context(st, ss)
        phi, res, ck = solver.solve(ctx, q=solver.q, checkpoint=solver.checkpoint)
        psi = None
        if face >= 0:
            psi = torch.empty((solver.ncells, len(solver.w), solver.nn), dtype=torch.float64, device=phi.device)
            sn_sweep(ctx, phi, solver.q, None, False, SN_FP64, psi)
        J = sn_response(ctx, r, phi if r is not None else None, face, psi, SN_FP64)
        del psi
        fctx.solver, fctx.face, fctx.ctx = solver, face, ctx
        fctx.forward_iters = res["iters"]
        fctx.checkpoints = ck
        fctx.save_for_backward(phi, r if r is not None else torch.empty(0, device=phi.device))
        return torch.tensor(J, dtype=torch.float64, device=phi.device)

    @staticmethod
    def backward(fctx, grad_J):
        phi, r = fctx.saved_tensors
        solver, face, ctx = fctx.solver, fctx.face, fctx.ctx
        dev = phi.device
        q_adj = (4.0 * math.pi) * r if r.numel() else None
        inflow_adj = None
        if face >= 0:
            inflow_adj = torch.tensor(outgoing_face_inflow(solver.dim, solver.nx, solver.ny, solver.nz, solver.omega,
                                                           face), dtype=torch.float64, device=dev)
        chi, _, _ = solver.solve(ctx, q=q_adj, inflow=inflow_adj, transpose=True)
        D = len(solver.w)
        psi = torch.empty((solver.ncells, D, solver.nn), dtype=torch.float64, device=dev)
        sn_sweep(ctx, phi, solver.q, None, False, SN_FP64, psi)          # regenerated from phi*
        psia = torch.empty_like(psi)
        sn_sweep(ctx, chi, q_adj, inflow_adj, True, SN_FP64, psia)
        gt = torch.empty(solver.ncells, dtype=torch.float64, device=dev)
        gs = torch.empty_like(gt)
        sn_gradient(ctx, psi, psia, SN_FP64, phi, chi, gt, gs)
        del psi, psia
        ctx.close()
        return grad_J * gt, grad_J * gs, None, None, None


def detector_response(log_sigma_t, log_sigma_s, solver: Solver, r=None, face: int = -1):
    """J as a differentiable function of per-cell log cross sections."""
    return SnDetector.apply(log_sigma_t, log_sigma_s, solver, r, face)
