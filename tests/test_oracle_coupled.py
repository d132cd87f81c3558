"""Budgets of the full coupled oracle step on the seeded two-layer workloads."""
import numpy as np
import pytest

import oracle
from oracle import OracleConfig
from paper_2106_07694_amd import workloads as W


def oracle_cfg(wl: W.Workload, shifted=None) -> OracleConfig:
    return OracleConfig(q=wl.q, nx=wl.nx, ny=wl.ny, nz=wl.nz,
                        shifted=(wl.precision != "fp64") if shifted is None else shifted,
                        tau=wl.tau, vs=wl.vs, kappa_c=wl.kappa_c, gp_c=wl.gp_c,
                        has_s=wl.has_s, kappa_s=wl.kappa_s, gp_s=wl.gp_s)


@pytest.mark.parametrize("wl", [
    W.C1.replace(nx=32, ny=64),
    W.C2.replace(nx=32, ny=64, c0=2.0),
    W.C3.replace(nx=8, ny=8, nz=24),
])
def test_coupled_budgets(wl):
    cfg = oracle_cfg(wl, shifted=False)
    c, s = W.initial_scalars(wl)
    f = oracle.equilibrium(cfg)
    s0 = oracle.sums(cfg, f, c, s)
    f2, c2, s2, dep, u = oracle.run(cfg, f, c, s, nsteps=150, want_u=True)
    s1 = oracle.sums(cfg, f2, c2, s2, dep)
    assert abs(s1[2] - s0[2]) < 1e-13 * s0[2]
    assert abs(s1[0] + s1[3] - s0[0]) < 1e-13 * s0[0]
    if wl.has_s:
        assert abs(s1[1] - s0[1]) < 1e-13 * s0[1]
    # the heavy upper layer sets the fluid in motion
    assert np.max(np.abs(u)) > 0
    # determinism: the same inputs give the same bits
    f3, c3, s3, dep3, _ = oracle.run(cfg, f, c, s, nsteps=150)
    assert np.array_equal(f3, f2) and np.array_equal(c3, c2) and np.array_equal(dep3, dep)


def test_initial_condition_recipe():
    wl = W.C1
    c, s = W.initial_scalars(wl)
    assert c.shape == (1, 128, 64) and s is None
    # upper half ~C0, lower half ~0, perturbation bounded by amp
    assert abs(c[0, -1].mean() - 1.0) < 2e-3 and abs(c[0, 0].mean()) < 2e-3
    c2, _ = W.initial_scalars(wl)
    assert np.array_equal(c, c2)
    runs = W.sweep_runs()
    assert len(runs) == 64
    assert {(r.nx, r.ny) for r in runs} <= set(W.SWEEP_GRIDS)
    assert all(0.25 <= r.c0 <= 4 and 1e-4 <= r.vs <= 2e-3 for r in runs)
