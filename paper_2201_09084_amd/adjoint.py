"""Gradient of the residual interior field energy with respect to the PML profile.

theta packs the parameters of the conductivity profile sigma/eps0 = sum_k a_{d,k}
(depth/L)^k of every axis d < dim (16 coefficients each) and the damping scale s of
alpha = exp(-s Phi) (Sec. II.C), in that order.  The objective is the field energy
1/2 sum (E^2 + B^2) dV over the physical box after n steps (the energy norm of the
error in Sec. III).  The forward pass keeps checkpoints on the GPU; the backward pass
recomputes each segment and runs the transposed step: the field update and alpha damping,
and with push = 1 also the gather, Boris push and Esirkepov deposit of every particle
(with push = 0 the current does not depend on the fields or on theta).
"""
import numpy as np
import torch

from . import binding as B


def n_theta(dim: int) -> int:
    return 16 * dim + 1


def theta_of(cfg) -> np.ndarray:
    th = np.zeros(n_theta(cfg.dim))
    for d in range(cfg.dim):
        row = list(cfg.sigma_coef[d])
        th[16 * d:16 * d + len(row)] = row
    th[-1] = cfg.damping_scale
    return th


def with_theta(cfg, theta):
    th = np.asarray(theta, dtype=np.float64).reshape(-1)
    if th.size != n_theta(cfg.dim):
        raise ValueError("theta must hold 16 dim + 1 values")
    rows = [tuple(float(v) for v in th[16 * d:16 * d + 16]) for d in range(cfg.dim)]
    rows += [tuple(cfg.sigma_coef[d]) for d in range(cfg.dim, 3)]
    return cfg.replace(sigma_coef=tuple(rows), damping_scale=float(th[-1]))


def make_sim(cfg, theta, particles, n_steps: int, segment: int):
    """A GPU run prepared for forward_ckpt(n_steps) with checkpoints every `segment`."""
    ck = max(1, -(-int(n_steps) // int(segment)))
    sim = B.PmlPic(with_theta(cfg, theta), max_particles=max(1, len(particles.w)), adjoint=(segment, ck))
    if len(particles.w):
        sim.add_particles(particles.x, particles.u, particles.w)
    return sim


class InteriorEnergy(torch.autograd.Function):
    """U(theta) after n_steps; backward gives dU/dtheta from the adjoint pass."""

    @staticmethod
    def forward(ctx, theta, cfg, particles, n_steps, segment):
        sim = make_sim(cfg, theta.detach().to("cpu", torch.float64).numpy(), particles, n_steps, segment)
        U = sim.forward_ckpt(n_steps)
        ctx.sim = sim
        return torch.tensor(U, dtype=torch.float64, device=theta.device)

    @staticmethod
    def backward(ctx, gU):
        grad, _ = ctx.sim.backward()
        ctx.sim.close()
        g = torch.from_numpy(grad).to(device=gU.device) * gU
        return g.to(gU.dtype), None, None, None, None


def interior_energy(theta: torch.Tensor, cfg, particles, n_steps: int, segment: int = 50) -> torch.Tensor:
    return InteriorEnergy.apply(theta, cfg, particles, int(n_steps), int(segment))
