"""torch.autograd bridge of the IMEX-DS adjoint.

``evolve(solver, rho0, mom0, tau, n_steps, ckpt_every)`` runs n_steps steps
of a batch from (rho0, rho u 0) with kinetic coefficient tau and returns the
end state (rho, rho u) and the interface offsets hl inside their home cells,
as tensors that torch can differentiate: the backward pass is the library's
hand-written adjoint (imexds_forward_ckpt / imexds_adjoint), so gradients
reach rho0, mom0 and tau.  ``window_objective`` is the scalar of interest
used with it: the sum of interface positions plus the mass in a window,
written with torch operations on the end state.
"""
from __future__ import annotations

import numpy as np
import torch

from . import imexds as _I


class _Evolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho0, mom0, tau, solver, n_steps, ckpt_every):
        solver.set_tau(float(tau.item()))
        solver.set_state(rho0.detach().contiguous(), mom0.detach().contiguous())
        solver.forward_ckpt(n_steps, ckpt_every)
        ctx.generation = solver.generation
        rho, mom = solver.state()
        home, hl, _ = solver.interfaces()
        ctx.solver = solver
        ctx.home = home.copy()
        ctx.tau_shape = tau.shape
        return rho, mom, torch.from_numpy(np.ascontiguousarray(hl)).to(rho.device)

    @staticmethod
    def backward(ctx, g_rho, g_mom, g_hl):
        s = ctx.solver
        if s.generation != ctx.generation:
            raise RuntimeError("evolve: the solver has run again since this forward (another "
                               "evolve, step or set_state); its adjoint would belong to that "
                               "run.  Call backward before reusing the solver, or use one "
                               "solver per graph.")
        S = s.n_slots
        dev = "cuda"
        if g_rho is None:
            g_rho = torch.zeros(S, dtype=torch.float64, device=dev)
        if g_mom is None:
            g_mom = torch.zeros(S, dtype=torch.float64, device=dev)
        g_rho0, g_mom0, _, g_tau = s.adjoint(g_rho, g_mom, g_hl)
        return g_rho0, g_mom0, g_tau.reshape(ctx.tau_shape), None, None, None


def evolve(solver, rho0, mom0, tau, n_steps, ckpt_every=50):
    """(rho, rho u, hl) after n_steps steps; differentiable in rho0, mom0 and
    tau (a 0-d or 1-element FP64 tensor).  ``solver`` is an IMEXDS context
    for the batch; its end interface homes are in solver.interfaces()."""
    return _Evolve.apply(rho0, mom0, tau, solver, int(n_steps), int(ckpt_every))


def slot_geometry(batch, home):
    """Index arrays describing each slot's interval at interface homes
    ``home``: background cell j, and the interface whose left / right piece it
    is (-1 if none)."""
    so = batch.slot_off
    S = batch.n_slots
    j = np.zeros(S, np.int64)
    kl = np.full(S, -1, np.int64)
    kr = np.full(S, -1, np.int64)
    prob = np.zeros(S, np.int64)
    for p in range(batch.n_problems):
        s0, s1 = int(so[p]), int(so[p + 1])
        prob[s0:s1] = p
        jj = np.arange(s1 - s0, dtype=np.int64)
        for kk, k in enumerate(range(int(batch.iface_off[p]), int(batch.iface_off[p + 1]))):
            sL = int(home[k]) + kk
            jj[sL + 1:] -= 1
            kl[s0 + sL] = k
            kr[s0 + sL + 1] = k
        j[s0:s1] = jj
    return j, kl, kr, prob


def window_objective(batch, home, hl, rho, cx=1.0, wa=0.4, wb=0.6):
    """Per-problem cx * sum_k x_k + sum_s rho_s |slot_s ∩ [wa, wb]| (torch,
    differentiable in hl and rho)."""
    dev = rho.device
    j, kl, kr, prob = slot_geometry(batch, home)
    h = torch.as_tensor(np.asarray(batch.h, np.float64), device=dev)
    xl = torch.as_tensor(np.asarray(batch.x_left, np.float64), device=dev)
    pt = torch.as_tensor(prob, device=dev)
    jt = torch.as_tensor(j, dtype=torch.float64, device=dev)
    hp, xp = h[pt], xl[pt]
    a = xp + jt * hp
    e = xp + (jt + 1.0) * hp
    if batch.n_iface:
        # only the two pieces of each cut cell depend on hl
        sl = torch.as_tensor(np.nonzero(kl >= 0)[0], device=dev)
        sr = torch.as_tensor(np.nonzero(kr >= 0)[0], device=dev)
        e = e.index_put((sl,), a[sl] + hl[torch.as_tensor(kl[kl >= 0], device=dev)])
        a = a.index_put((sr,), a[sr] + hl[torch.as_tensor(kr[kr >= 0], device=dev)])
    ov = (torch.minimum(e, torch.full_like(e, wb)) - torch.maximum(a, torch.full_like(a, wa)))
    ov = ov.clamp(min=0.0)
    L = torch.zeros(batch.n_problems, dtype=torch.float64, device=dev)
    L = L.index_add(0, pt, rho * ov)
    if batch.n_iface:
        ip = torch.as_tensor(np.repeat(np.arange(batch.n_problems), np.diff(batch.iface_off)),
                             device=dev)
        hk = torch.as_tensor(np.asarray(home, np.float64), device=dev)
        x = xl[ip] + hk * h[ip] + hl
        L = L.index_add(0, ip, cx * x)
    return L
