"""Gradient of the deposited mass through the coupled step.

``DepositedMass.apply(c0, vs, cfg, nsteps)`` returns J = total mass deposited
on the bottom wall after ``nsteps`` coupled steps started from the fluid at
rest and the concentration field ``c0`` (the initial state of section 2.2);
its backward gives dJ/dc0 and dJ/dVs through the hand-written adjoint kernels
(``lbw_adjoint_step``).

Memory follows the square-root rule: the forward keeps the state (canonical
populations and C) every ``seg`` ~ sqrt(nsteps) steps; the backward replays
each segment from its checkpoint, keeping that segment's per-step states, and
runs the reverse steps back through it.  All arithmetic runs in the library's
kernels; this module orders calls and owns tensors.
"""
from __future__ import annotations

import math

import torch

from . import lbw


def check_supported(cfg: lbw.RunConfig) -> None:
    """The adjoint kernels cover the WENO5 transport of one particle class
    without S (so without the S-dependent settling and force either); raise
    before any step is taken otherwise."""
    if cfg.scheme_c != "weno5" or cfg.has_s or cfg.ncls > 1:
        raise ValueError("the adjoint covers WENO5 transport of one particle class without S "
                         f"(got scheme {cfg.scheme_c}, has_s {cfg.has_s}, {cfg.ncls} classes)")


def default_segment(nsteps: int) -> int:
    return max(1, int(round(math.sqrt(nsteps))))


def _solver(cfg: lbw.RunConfig, vs: float, launch=None) -> lbw.Solver:
    c = lbw.RunConfig(**{**cfg.__dict__, "vs": float(vs)})
    sol = lbw.Solver(c)
    if launch:
        sol.set_launch(**launch)
    return sol


# The per-step buffers of a replayed segment are views of one allocation per
# kind (contiguous slices), so a backward pass allocates a handful of blocks
# rather than several hundred small ones.
def _state_buffers(sol, count, populations=True):
    cfg = sol.cfgs[0]
    e = lambda *shape: torch.empty(shape, dtype=sol.dtype, device=sol.device)
    with torch.cuda.stream(sol.stream):
        f = e(count, cfg.lattice, *cfg.shape) if populations else None
        c = e(count, *cfg.shape)
        return [(f[i] if populations else None, c[i]) for i in range(count)]


def _step_buffers(sol, count, moments=True):
    """Per-step forward intermediates: node velocity and density (LBM mode),
    RK stages 1 and 2."""
    cfg = sol.cfgs[0]
    e = lambda *shape: torch.empty(shape, dtype=sol.dtype, device=sol.device)
    with torch.cuda.stream(sol.stream):
        u = e(count, cfg.dim, *cfg.shape) if moments else None
        rho = e(count, *cfg.shape) if moments else None
        a1, a2 = e(count, *cfg.shape), e(count, *cfg.shape)
        return [(u[i] if moments else None, rho[i] if moments else None, a1[i], a2[i])
                for i in range(count)]


def forward_with_checkpoints(cfg, c0: torch.Tensor, vs: float, nsteps: int, seg: int, launch=None,
                             f0=None, u=None):
    """Run nsteps from C = c0 and the fluid at rest (or the canonical
    populations f0; or, for a frozen fluid, the velocity u); return
    (J, solver, checkpoints {step: (f, c)})."""
    check_supported(cfg)
    sol = _solver(cfg, vs, launch)
    sol.set_field("c", c0)
    frozen = cfg.fluid_mode == lbw.FLUID_FROZEN
    if frozen:
        sol.set_field("u", u)
    elif f0 is not None:
        sol.set_field("f", f0)
    else:
        sol.init_equilibrium()
    starts = list(range(0, nsteps, seg))
    bufs = _state_buffers(sol, len(starts))
    ckpt = {}
    for s0, (fb, cb) in zip(starts, bufs):
        if not frozen:
            sol.export_into("f", fb)
        sol.export_into("c", cb)
        ckpt[s0] = (fb, cb)
        sol.step(min(seg, nsteps - s0))
    J = float(sol.reduce(lbw.DEPOSIT)[0])
    return J, sol, ckpt


def backward_from_checkpoints(sol: lbw.Solver, ckpt: dict, nsteps: int, seg: int, dep_bar: float):
    """(dJ/dc0, dJ/dVs) given the checkpoints of a forward run."""
    dev, dt = sol.device, sol.dtype
    cfg = sol.cfgs[0]
    with torch.cuda.stream(sol.stream):
        fbar_next = torch.zeros((cfg.lattice,) + cfg.shape, dtype=dt, device=dev)
        cbar_next = torch.zeros(cfg.shape, dtype=dt, device=dev)
        fbar = torch.empty_like(fbar_next)
        cbar = torch.empty_like(cbar_next)
        vs_bar = torch.zeros(1, dtype=torch.float64, device=dev)
    work = sol.adjoint_workspace()
    frozen = cfg.fluid_mode == lbw.FLUID_FROZEN
    # per replayed step: C before the step, and the step's own velocity,
    # density and RK stages (the populations are not needed: the reverse
    # collision uses only their moments)
    states = _state_buffers(sol, seg, populations=False)
    inter = _step_buffers(sol, seg, moments=not frozen)
    last = min(ckpt)
    for s0 in reversed(sorted(ckpt)):
        n = min(seg, nsteps - s0)
        f_s, c_s = ckpt[s0]
        if not frozen:
            sol.import_from("f", f_s)
        sol.import_from("c", c_s)
        # replay the segment in one library call: each step writes its
        # intermediates straight into that step's buffers (C is copied
        # before it)
        sol.replay([states[i][1] for i in range(n)], [inter[i][2] for i in range(n)],
                   [inter[i][3] for i in range(n)],
                   None if frozen else [inter[i][0] for i in range(n)],
                   None if frozen else [inter[i][1] for i in range(n)])
        for i in reversed(range(n)):
            c_n = states[i][1]
            u_n, rho_n, a1, a2 = inter[i]
            vs_out = vs_bar if (s0 == last and i == 0) else None
            if frozen:
                sol.adjoint_step(None, c_n, None, cbar_next, dep_bar, None, cbar, vs_out, work,
                                 a1_n=a1, a2_n=a2)
            else:
                sol.adjoint_step(None, c_n, fbar_next, cbar_next, dep_bar, fbar, cbar, vs_out, work,
                                 u_n=u_n, rho_n=rho_n, a1_n=a1, a2_n=a2)
            fbar_next, fbar = fbar, fbar_next
            cbar_next, cbar = cbar, cbar_next
    sol.stream.synchronize()
    return cbar_next.clone(), float(vs_bar.item())


class DepositedMass(torch.autograd.Function):
    """J(c0, vs) = deposited mass after nsteps; differentiable in c0 and vs."""

    @staticmethod
    def forward(ctx, c0, vs, cfg, nsteps, seg=None, launch=None, f0=None, u=None):
        seg = seg or default_segment(nsteps)
        J, sol, ckpt = forward_with_checkpoints(cfg, c0.detach(), float(vs), nsteps, seg, launch,
                                                f0, u)
        ctx.sol, ctx.ckpt, ctx.nsteps, ctx.seg = sol, ckpt, nsteps, seg
        return torch.tensor(J, dtype=torch.float64, device=c0.device)

    @staticmethod
    def backward(ctx, gJ):
        cbar, vsb = backward_from_checkpoints(ctx.sol, ctx.ckpt, ctx.nsteps, ctx.seg, float(gJ))
        ctx.sol.close()
        ctx.ckpt = None
        gc = cbar.to(torch.float64)
        gv = torch.tensor(vsb, dtype=torch.float64, device=gc.device)
        return gc, gv, None, None, None, None, None, None
