"""Field-driven propagation as a differentiable torch function.

``MagnusFn`` maps the parameters theta = (A_1..A_m, w_1..w_m, phi_1..phi_m) of
the pulse E(t) = sum_k A_k sin(w_k t + phi_k) exp(-(t - t0)^2 / s^2) (the field
of eq. (VField), along one axis) to the dipole trace mu(t_0..t_N) of N
predictor-corrector Magnus-2 steps (Sec. 2.5) from fixed orbitals.

Forward: the library's magnus_step, keeping a copy of the orbitals every
``checkpoint`` steps.  Backward (the hand-written reverse mode of the step, in
the library's kernels): per checkpoint segment, latest first, the forward is run
again from its checkpoint keeping every step, then dipole_adjoint (terminal
condition) and magnus_adjoint step by step with dL/dmu(t_n) from the incoming
gradient; the per-step field sensitivities dL/dE(t_n), dL/dE(t_n + dt/2) are
contracted with dE/dtheta by the library (efe_field_vjp).  The orbitals enter as
constants (no gradient with respect to them).
"""
from __future__ import annotations

import numpy as np
import torch

from .efe import field_vjp, make_field


class MagnusFn(torch.autograd.Function):
    """mus = MagnusFn.apply(theta, Psi0, ctx, t0, s, dt, nsteps, direction, checkpoint).

    theta: float64 CPU tensor (3 m); Psi0: the context's orbital block on the
    device (not modified); returns mus, a float64 CPU tensor (nsteps + 1, 3)
    with mus[n] the dipole at t_n = n dt."""

    @staticmethod
    def forward(fctx, theta, Psi0, ctx, t0, s, dt, nsteps, direction=2, checkpoint=20):
        th = theta.detach().cpu().numpy().astype(np.float64)
        m = len(th) // 3
        if len(th) != 3 * m or m < 1:
            raise ValueError("theta holds (A, w, phi) of at least one component")
        if checkpoint < 1 or nsteps < 1:
            raise ValueError("nsteps and checkpoint must be positive")
        field, keep = make_field(direction, th[:m], th[m:2 * m], th[2 * m:], t0, s)
        Psi = Psi0.clone()
        ckpt = {}
        mus = np.zeros((nsteps + 1, 3))
        ctx.set_hamiltonian(Psi, 0.0, field)
        mus[0] = ctx.dipole(Psi)
        for n in range(nsteps):
            if n % checkpoint == 0:
                ckpt[n] = Psi.clone()
            mus[n + 1] = ctx.magnus_step(Psi, n * dt, dt, field)["mu"]
        fctx.run = dict(ctx=ctx, field=field, keep=keep, ckpt=ckpt, dt=float(dt), nsteps=int(nsteps),
                        checkpoint=int(checkpoint), m=m)
        return torch.from_numpy(mus)

    @staticmethod
    def backward(fctx, grad_mus):
        r = fctx.run
        ctx, field, dt, nsteps, K = r["ctx"], r["field"], r["dt"], r["nsteps"], r["checkpoint"]
        gmu = grad_mus.detach().cpu().numpy().astype(np.float64)
        times = np.zeros(2 * nsteps)
        dLdE = np.zeros(2 * nsteps)
        Psibar = None
        for c0 in sorted(r["ckpt"], reverse=True):
            c1 = min(c0 + K, nsteps)
            states = [r["ckpt"][c0].clone()]
            ctx.set_hamiltonian(states[0], c0 * dt, field)
            for n in range(c0, c1):
                P = states[-1].clone()
                ctx.magnus_step(P, n * dt, dt, field)
                states.append(P)
            if Psibar is None:
                Psibar = ctx.dipole_adjoint(states[-1], gmu[c1])
            for n in range(c1 - 1, c0 - 1, -1):
                gE = ctx.magnus_adjoint(states[n - c0], Psibar, n * dt, dt, field, gmu[n])
                times[2 * n], times[2 * n + 1] = n * dt, n * dt + 0.5 * dt
                dLdE[2 * n], dLdE[2 * n + 1] = gE
        grad = torch.from_numpy(field_vjp(field, times, dLdE))
        return grad, None, None, None, None, None, None, None, None


def field_gradient(ctx, Psi0, theta, t0, s, dt, nsteps, mu_target, direction=2, checkpoint=20):
    """dL/dtheta of L = sum_{n=1}^{N} (mu_d(t_n) - mu*_n)^2 through MagnusFn and
    torch.autograd.  Returns (L, grad, mus) as floats / numpy arrays."""
    th = torch.tensor(np.asarray(theta, dtype=np.float64), requires_grad=True)
    mus = MagnusFn.apply(th, Psi0, ctx, t0, s, dt, nsteps, direction, checkpoint)
    L = ((mus[1:, direction] - torch.as_tensor(np.asarray(mu_target, dtype=np.float64))) ** 2).sum()
    (g,) = torch.autograd.grad(L, th)
    return float(L.detach()), g.numpy(), mus.detach().numpy()
