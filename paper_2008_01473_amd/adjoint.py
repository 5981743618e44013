"""Gradients of a loss of the final fields with respect to kappa, T/Tc and the
initial density, through many D2Q9 steps, with the library's hand-written
adjoint kernels and sqrt(N) checkpointing of the forward states.

    roll = Rollout(params)                  # one D2Q9 lattice, improved or standard scheme
    rho_N, u_N = rollout(rho0, kappa, T_over_Tc, roll, n_steps)   # torch.autograd.Function
    loss = ((rho_N - rho_target)**2).sum() + (u_N**2).sum()
    loss.backward()                         # rho0.grad, kappa.grad, T_over_Tc.grad

Forward: lbm_init, then n steps; the raw state is checkpointed every k = ceil(sqrt(n))
steps.  Backward: dL/df(N) from lbm_adjoint_fields, then lbm_adjoint_sweep runs the
segments in reverse (restore a checkpoint, recompute the segment's states on a
second stream while the adjoint steps of the later segment run, then the adjoint
steps back through them); finally lbm_adjoint_init gives dL/drho0.  All of this
runs in the HIP kernels and the library's runtime; this module orders the calls.
"""

import ctypes
import math

import torch

from . import _lib
from ._lib import check
from .runtime import LBM


class Rollout:
    def __init__(self, prm, device="cuda"):
        self.sim = LBM(prm, device=device)
        if self.sim.D != 2 or self.sim.count != 1:
            raise ValueError("the adjoint supports one D2Q9 lattice")
        L = _lib.lib()
        nb = L.lbm_adjoint_workspace_bytes(self.sim.h)
        if nb == 0:
            raise ValueError("no adjoint for this handle")
        self.ws = torch.empty(nb, dtype=torch.uint8, device=self.sim.device)
        self.prm = prm
        self.N = self.sim.N
        self.stats = {}

    def set_physics(self, kappa, T_over_Tc):
        check(_lib.lib().lbm_set_physics(self.sim.h, 0, float(kappa), float(T_over_Tc)), "lbm_set_physics")

    # ------------------------------------------------------------------ forward
    def forward(self, rho0, kappa, T_over_Tc, n_steps, checkpoint_every=None):
        sim = self.sim
        self.set_physics(kappa, T_over_Tc)
        self.rho0 = sim._dev64(rho0, self.N)
        sim.init(self.rho0)
        k = checkpoint_every or max(1, math.ceil(math.sqrt(max(n_steps, 1))))
        self.k, self.n = k, n_steps
        self.checkpoints = {}
        t = 0
        while t < n_steps:
            self.checkpoints[t] = sim.get_state()[0]
            m = min(k, n_steps - t)
            sim.step(m)
            t += m
        self.final_state = sim.get_state()[0]
        rho, u, _ = sim.moments()
        return rho.clone(), u.clone()

    # ----------------------------------------------------------------- backward
    def backward(self, rho_bar, u_bar):
        sim, L = self.sim, _lib.lib()
        dev = sim.device
        grad = torch.zeros(2, dtype=torch.float64, device=dev)
        lam = torch.empty(9 * self.N, dtype=torch.float64, device=dev)
        lam2 = torch.empty_like(lam)
        rb = None if rho_bar is None else rho_bar.to(dev, torch.float64).contiguous()
        ub = None if u_bar is None else u_bar.to(dev, torch.float64).contiguous()
        ws = self.ws.data_ptr()
        check(L.lbm_adjoint_fields(sim.h, self.final_state.data_ptr(), None if rb is None else rb.data_ptr(),
                                   None if ub is None else ub.data_ptr(), lam.data_ptr(), ws, grad.data_ptr()),
              "lbm_adjoint_fields")
        t0s = sorted(self.checkpoints)
        nseg = len(t0s)
        ms = [min(self.k, self.n - t) for t in t0s]
        if nseg:
            # two arenas: one segment's recomputation overlaps the next one's adjoint steps
            states = torch.empty(2 * max(ms) * sim.state_bytes, dtype=torch.uint8, device=dev)
            ck = (ctypes.c_void_p * nseg)(*[self.checkpoints[t].data_ptr() for t in t0s])
            check(L.lbm_adjoint_sweep(sim.h, ck, (ctypes.c_longlong * nseg)(*t0s), (ctypes.c_int * nseg)(*ms), nseg,
                                      states.data_ptr(), lam.data_ptr(), lam2.data_ptr(), ws, grad.data_ptr()),
                  "lbm_adjoint_sweep")
        grad_rho0 = torch.empty(self.N, dtype=torch.float64, device=dev)
        check(L.lbm_adjoint_init(sim.h, self.rho0.data_ptr(), lam.data_ptr(), grad_rho0.data_ptr(), ws,
                                 grad.data_ptr()), "lbm_adjoint_init")
        return grad_rho0, grad[0].clone(), grad[1].clone()

    def close(self):
        self.sim.close()


class _RolloutFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho0, kappa, T_over_Tc, roll, n_steps):
        rho, u = roll.forward(rho0.detach(), float(kappa), float(T_over_Tc), int(n_steps))
        ctx.roll = roll
        ctx.like = (rho0, kappa, T_over_Tc)
        return rho, u

    @staticmethod
    def backward(ctx, grad_rho, grad_u):
        g_rho0, g_k, g_t = ctx.roll.backward(grad_rho, grad_u)
        r0, k, t = ctx.like
        return (g_rho0.to(r0.device, r0.dtype).reshape(r0.shape), g_k.to(k.device, k.dtype).reshape(k.shape),
                g_t.to(t.device, t.dtype).reshape(t.shape), None, None)


def rollout(rho0, kappa, T_over_Tc, roll, n_steps):
    """Differentiable rho(N), u(N) (flattened [N] and [2, N] float64 tensors)."""
    return _RolloutFn.apply(rho0, kappa, T_over_Tc, roll, n_steps)

