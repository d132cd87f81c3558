"""Seeded random configurations of one reverse step against the oracle's
adjoint (FP64, 1e-12 relative; dJ/dVs relative to the scale of its terms): lattice, frozen or coupled fluid, walls or
periodic vertical axis, plain or shifted FP64, grid sizes down to one column,
relaxation time, settling speed, diffusivity, buoyancy, and in 2D both the
fused and the face + gather forms of the reverse transport."""
import numpy as np
import pytest
import torch

import oracle
from paper_2106_07694_amd import lbw

from parity import oracle_cfg, rel

pytestmark = pytest.mark.gpu


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", torch.float64)


@pytest.mark.parametrize("case", range(72))
def test_random_adjoint_step(case):
    rng = np.random.default_rng(7000 + case)
    q = int(rng.choice([9, 19]))
    shape = (dict(nx=int(rng.integers(1, 40)), ny=int(rng.integers(6, 40))) if q == 9 else
             dict(nx=int(rng.integers(1, 14)), ny=int(rng.integers(1, 10)), nz=int(rng.integers(6, 20))))
    frozen = bool(rng.random() < 0.3)
    cfg = lbw.RunConfig(lattice=q, precision=str(rng.choice(["fp64", "fp64_shifted"])),
                        tau=float(rng.uniform(0.52, 1.2)), vs=float(rng.uniform(0, 0.05)),
                        kappa_c=float(rng.uniform(0, 3e-3)), gp_c=float(rng.uniform(-4e-3, 4e-3)),
                        vert_periodic=bool(rng.random() < 0.3),
                        fluid_mode=lbw.FLUID_FROZEN if frozen else lbw.FLUID_LBM, **shape)
    launch = dict(variant=int(rng.choice([0, 1])), lbm_block=int(rng.choice([64, 256, 1024])))
    ocfg = oracle_cfg(cfg)
    dim = ocfg.dim
    u0 = 0.03 * rng.standard_normal((dim,) + ocfg.shape)
    f_n = oracle.equilibrium(ocfg, 1.0 + 0.01 * rng.standard_normal(ocfg.shape), u0)
    c_n = rng.uniform(0.1, 1.0, ocfg.shape)
    fbar_next = rng.standard_normal((q,) + ocfg.shape)
    cbar_next = rng.standard_normal(ocfg.shape)
    dep_bar = float(rng.uniform(0.1, 2.0))
    fo, co, vo = oracle.adjoint_step(ocfg, None if frozen else f_n, c_n,
                                     None if frozen else fbar_next, cbar_next, dep_bar,
                                     u0 if frozen else None)
    sol = lbw.Solver(cfg)
    sol.set_launch(**launch)
    if frozen:
        sol.set_field("u", u0)
    fb = torch.zeros((q,) + ocfg.shape, dtype=torch.float64, device="cuda")
    cb = torch.zeros(ocfg.shape, dtype=torch.float64, device="cuda")
    vs = torch.zeros(1, dtype=torch.float64, device="cuda")
    work = sol.adjoint_workspace()
    torch.cuda.synchronize()
    sol.adjoint_step(None if frozen else _dev(f_n), _dev(c_n),
                     None if frozen else _dev(fbar_next), _dev(cbar_next), dep_bar,
                     None if frozen else fb, cb, vs, work)
    torch.cuda.synchronize()
    # dJ/dVs is a sum over every node of terms of both signs (adjoint times
    # concentration), so its size can be far below its terms' (cancellation)
    # while the summation order (fixed on the GPU, sequential in the oracle)
    # rounds on the terms' scale: bound it by 1e-12 of that scale
    vs_scale = float(np.sum(np.abs(cbar_next * c_n))) + dep_bar * float(np.sum(np.abs(c_n)))
    errs = {"cbar": rel(cb.cpu().numpy(), co),
            "vs_bar": abs(vs.item() - vo) / max(abs(vo), vs_scale)}
    if not frozen:
        errs["fbar"] = rel(fb.cpu().numpy(), fo)
    print(f"\ncase {case} {cfg} {launch}: {errs}")
    sol.close()
    assert max(errs.values()) < 1e-12, (errs, cfg, launch)
