"""torch.autograd binding of the solve: x = A(lambda, mu, rho)^{-1} b.

Backward is the adjoint-state method: one adjoint solve A^H y = dL/dx
(ehh_solve_adjoint) and one contraction of y with the forward fields through
dA/dm (ehh_media_gradient).  The forward fields of every source are kept on the
device between forward and backward, together with the multigrid hierarchy of
the forward model, so the backward pass re-solves nothing.  Vectors are real
(nrhs, 2N) tensors in the library's layout; the gradient with respect to b is y
in that layout (dL = Re y^H db).  Argument marshalling only: every arithmetic
step runs in the library's kernels.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence, Tuple

import torch

from . import ehh


@dataclasses.dataclass
class SolveSpec:
    """Problem and solver settings of a differentiable solve.  mu_bar and
    rho_bar fix the units of the vectors (0 = means of the media given at each
    call); keep them fixed when the media change, so that b, x and the
    gradients refer to the same units."""
    dim: int
    n: Tuple[int, ...]
    h: float
    omega: float
    shift: float
    abl_cells: Tuple[int, ...]
    abl_max: float = 1.0
    atten0: float = 0.0
    mu_bar: float = 0.0
    rho_bar: float = 0.0
    tol: float = 1e-8
    maxit: int = 500
    solver: dict = dataclasses.field(default_factory=dict)   # levels, cycle, damping, precond_bits, ...


def spec_for_workload(w, mu_bar=0.0, rho_bar=0.0, tol=None, maxit=None, **solver_over) -> SolveSpec:
    kw = dict(levels=w.levels, cycle=w.cycle, cycle_level=w.cycle_level, nu1=w.nu1, nu2=w.nu2, vanka=w.vanka,
              precond_bits=w.precond_bits, restart=w.restart, dd_parts=w.dd_parts,
              dd_overlap=w.dd_overlap, dd_pad=w.dd_pad, dd_colors=w.dd_colors, damping=w.damping,
              coarse_dd_parts=w.coarse_dd_parts, coarse_dd_overlap=w.coarse_dd_overlap,
              coarse_dd_colors=w.coarse_dd_colors, damping_p=w.damping_p)
    kw.update(solver_over)
    return SolveSpec(dim=w.dim, n=tuple(w.n), h=w.h, omega=w.omega, shift=w.shift,
                     abl_cells=tuple(w.abl_cells), abl_max=w.abl_max, atten0=w.atten0,
                     mu_bar=mu_bar, rho_bar=rho_bar, tol=w.tol if tol is None else tol,
                     maxit=w.maxit if maxit is None else maxit, solver=kw)


def make_solver(spec: SolveSpec, lam, mu, rho) -> ehh.Solver:
    return ehh.Solver(spec.dim, spec.n, spec.h, spec.omega, spec.shift, spec.abl_cells,
                      lam.detach().contiguous(), mu.detach().contiguous(), rho.detach().contiguous(),
                      abl_max=spec.abl_max, atten0=spec.atten0, mu_bar=spec.mu_bar, rho_bar=spec.rho_bar,
                      **spec.solver)


class _Solve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, b, lam, mu, rho, spec: SolveSpec):
        if any(t.requires_grad for t in (lam, mu, rho)) and not (spec.mu_bar > 0 and spec.rho_bar > 0):
            raise ValueError("media gradients need fixed units: set spec.mu_bar and spec.rho_bar > 0")
        S = make_solver(spec, lam, mu, rho)
        x = torch.zeros_like(b)
        _, stats = S.solve(b.detach().contiguous(), x, tol=spec.tol, maxit=spec.maxit, raise_on_fail=True)
        ctx.solver = S
        ctx.spec = spec
        ctx.stats = stats
        ctx.media_shape = lam.shape
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        S, spec = ctx.solver, ctx.spec
        y = torch.zeros_like(x)
        _, astats = S.solve_adjoint(gx.contiguous(), y, tol=spec.tol, maxit=spec.maxit, raise_on_fail=True)
        ctx.adjoint_stats = astats
        gl = gm = gr = None
        if any(ctx.needs_input_grad[1:4]):
            opts = dict(dtype=torch.float64, device=x.device)
            gl = torch.empty(ctx.media_shape, **opts)
            gm = torch.empty(ctx.media_shape, **opts)
            gr = torch.empty(ctx.media_shape, **opts)
            S.media_gradient(y, x, gl, gm, gr)
        S.close()
        ctx.solver = None
        return (y if ctx.needs_input_grad[0] else None), gl, gm, gr, None


def elastic_helmholtz_solve(b: torch.Tensor, lam: torch.Tensor, mu: torch.Tensor, rho: torch.Tensor,
                            spec: SolveSpec) -> torch.Tensor:
    """Differentiable solve of A(lambda, mu, rho) x = b for every row of b.

    b: (nrhs, 2N) float64 device tensor in the library's layout (nondimensional
    units of `spec`); lam, mu, rho: float64 device cell arrays [Pa, Pa, kg/m^3].
    Gradients with respect to the media are per SI unit at the fixed units of
    `spec` (mu_bar, rho_bar must be set > 0 for them to be the derivatives of
    a fixed-unit problem)."""
    return _Solve.apply(b, lam, mu, rho, spec)
