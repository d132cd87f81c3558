"""Helpers shared by the GPU parity tests: run the HIP path and the FP64
oracle on the same seeded inputs and compare field by field."""
from __future__ import annotations

import numpy as np

import oracle
from oracle import OracleConfig
from paper_2106_07694_amd import lbw


def oracle_cfg(cfg: lbw.RunConfig) -> OracleConfig:
    return OracleConfig(q=cfg.lattice, nx=cfg.nx, ny=cfg.ny, nz=cfg.nz,
                        vert_periodic=cfg.vert_periodic,
                        frozen=cfg.fluid_mode == lbw.FLUID_FROZEN,
                        scheme_c=cfg.scheme_c, has_s=cfg.has_s,
                        shifted=cfg.precision != "fp64", tau=cfg.tau,
                        body_force=tuple(cfg.body_force), u_top=tuple(cfg.u_top), vs=cfg.vs,
                        kappa_c=cfg.kappa_c, gp_c=cfg.gp_c, kappa_s=cfg.kappa_s,
                        gp_s=cfg.gp_s, weno_eps=cfg.weno_eps, n_classes=cfg.n_classes,
                        vs_class=tuple(cfg.vs_class), kappa_class=tuple(cfg.kappa_class),
                        vs_s=cfg.vs_s, phi_c=cfg.phi_c)


def as_input(x, cfg: lbw.RunConfig):
    """Round an input to the storage precision so both sides see equal values."""
    if x is None:
        return None
    if cfg.precision == "fp32_shifted":
        return np.ascontiguousarray(np.asarray(x, np.float32).astype(np.float64))
    return np.ascontiguousarray(np.asarray(x, np.float64))


def rel(a, b) -> float:
    den = float(np.max(np.abs(b))) if np.size(b) else 0.0
    num = float(np.max(np.abs(np.asarray(a, np.float64) - b))) if np.size(b) else 0.0
    return num / den if den > 0 else num


def run_gpu(cfg, c0, s0=None, u_frozen=None, f0=None, nsteps=1, launch=None):
    import torch
    sol = lbw.Solver(cfg)
    if launch:
        sol.set_launch(**launch)
    sol.set_field("c", c0)
    if s0 is not None:
        sol.set_field("s", s0)
    if cfg.fluid_mode == lbw.FLUID_FROZEN:
        sol.set_field("u", u_frozen)
    elif f0 is not None:
        sol.set_field("f", f0)
    else:
        sol.init_equilibrium()
    sol.step(nsteps)
    torch.cuda.synchronize()
    out = {k: sol.field(k).double().cpu().numpy() for k in ("c", "u", "deposit")}
    if cfg.fluid_mode == lbw.FLUID_LBM:
        out["f"] = sol.field("f").double().cpu().numpy()
    if cfg.has_s:
        out["s"] = sol.field("s").double().cpu().numpy()
    sol.close()
    return out


def run_oracle(cfg, c0, s0=None, u_frozen=None, f0=None, nsteps=1):
    ocfg = oracle_cfg(cfg)
    if cfg.fluid_mode == lbw.FLUID_LBM:
        f = oracle.equilibrium(ocfg) if f0 is None else f0
    else:
        f = None
    f, c, s, dep, u = oracle.run(ocfg, f, c0, s0, None, u_frozen, nsteps, want_u=True)
    out = {"c": c, "u": u, "deposit": dep}
    if f is not None:
        out["f"] = f
    if s is not None:
        out["s"] = s
    return out


def compare(gpu: dict, orc: dict) -> dict:
    return {k: rel(gpu[k], orc[k]) for k in orc}
