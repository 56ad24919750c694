"""torch.autograd Functions over libgpe.

Energy:       E(phi; V, beta, omega) with the backward kernel of gpe_energy_grad
              (grad_phi = 2 h^d H_phi phi in PyTorch's conjugate-Wirtinger convention,
              grad_V = h^d |phi|^2, dE/dbeta = 1/2 h^d sum|phi|^4, dE/domega = -Re<phi, L_z phi>).
GroundState:  phi*(V, beta, omega), the PCG ground state, whose backward solves the implicit
              adjoint A mu = Pi g on the tangent space of the sphere modulo the global phase
              (gpe_adjoint_solve) and contracts mu with (d_theta H) phi* (gpe_adjoint_param_grads).
              By the envelope property, E(phi*(theta); theta) differentiates to its partials only,
              which the composition Energy(GroundState(...)) reproduces (the adjoint right-hand
              side 2 H phi* is then normal to the tangent space).

Both compute entirely in the HIP library; the glue here only builds plans and rescales by the
quadrature weight between PyTorch's convention (sums over grid points) and the library's
quadrature-weighted inner product.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import gpe


@dataclass(frozen=True)
class Grid:
    dim: int
    n: tuple
    L: tuple

    @property
    def cell(self) -> float:
        c = 1.0
        for a in range(self.dim):
            c *= 2.0 * self.L[a] / self.n[a]
        return c


_PLANS: dict = {}


def plan_for(grid: Grid, beta: float, omega: float, dtype: str) -> gpe.Plan:
    key = (grid, float(beta), float(omega), dtype)
    p = _PLANS.get(key)
    if p is None:
        if len(_PLANS) >= 16:
            _PLANS.clear()
        p = _PLANS[key] = gpe.Plan(grid.dim, grid.n, grid.L, float(beta), float(omega), dtype)
    return p


def _dtype(phi: torch.Tensor) -> str:
    return "f64" if phi.dtype == torch.complex128 else "f32"


class Energy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi, V, beta, omega, grid: Grid):
        phi = phi.detach().contiguous()
        V = V.detach().contiguous()
        b, o = float(beta), float(omega)
        plan = plan_for(grid, b, o, _dtype(phi))
        E = plan.energy(phi, V)
        ctx.save_for_backward(phi, V)
        ctx.grid, ctx.b, ctx.o = grid, b, o
        return torch.tensor(E, dtype=V.dtype, device=V.device)

    @staticmethod
    def backward(ctx, gE):
        phi, V = ctx.saved_tensors
        plan = plan_for(ctx.grid, ctx.b, ctx.o, _dtype(phi))
        gphi, gV, db, do = plan.energy_grad(phi, V)
        g = gE.to(V.dtype)
        return (g * gphi, g * gV, g * torch.tensor(db, dtype=V.dtype, device=V.device),
                g * torch.tensor(do, dtype=V.dtype, device=V.device), None)


class GroundState(torch.autograd.Function):
    @staticmethod
    def forward(ctx, V, beta, omega, phi0, grid: Grid, solve_opts: dict, adjoint_opts: dict):
        V = V.detach().contiguous()
        b, o = float(beta), float(omega)
        plan = plan_for(grid, b, o, _dtype(phi0))
        phi = phi0.detach().clone().contiguous()
        rep = plan.pcg_solve(V, phi, **solve_opts)
        if rep["status"] != 0:
            raise RuntimeError(f"ground-state solve did not converge: {rep}")
        ctx.save_for_backward(phi, V)
        ctx.grid, ctx.b, ctx.o, ctx.aopts = grid, b, o, adjoint_opts
        ctx.report = rep
        return phi

    @staticmethod
    def backward(ctx, gphi):
        phi, V = ctx.saved_tensors
        plan = plan_for(ctx.grid, ctx.b, ctx.o, _dtype(phi))
        # PyTorch's gradient g_t gives dl = sum Re(conj(g_t) dphi) = Re<g_t / h^d, dphi>; the adjoint is
        # linear in its right-hand side, so solve with g_t and divide the contractions by h^d.
        mu, rep = plan.adjoint_solve(phi, V, gphi.contiguous(), **ctx.aopts)
        if rep["status"] != 0:
            raise RuntimeError(f"adjoint solve did not converge: {rep}")
        gV, db, do = plan.adjoint_param_grads(phi, mu)
        inv = 1.0 / ctx.grid.cell
        t = lambda x: torch.tensor(x * inv, dtype=V.dtype, device=V.device)  # noqa: E731
        return gV * inv, t(db), t(do), None, None, None, None


def energy(phi, V, beta, omega, grid: Grid):
    return Energy.apply(phi, V, beta, omega, grid)


def ground_state(V, beta, omega, phi0, grid: Grid, solve_opts: dict | None = None, adjoint_opts: dict | None = None):
    solve_opts = dict(solve_opts or {})
    solve_opts.setdefault("tol", 1e-11)
    solve_opts.setdefault("max_iter", 100000)
    adjoint_opts = dict(adjoint_opts or {})
    adjoint_opts.setdefault("tol", 1e-10)
    adjoint_opts.setdefault("max_iter", 20000)
    return GroundState.apply(V, beta, omega, phi0, grid, solve_opts, adjoint_opts)
