"""Seeded random configurations against the oracle (FP64) and batches against
their runs alone (bit for bit): lattice, precision form, small and odd grid
sizes, walls or periodic vertical axis, lid, body force, S, size classes,
settling set by S, buoyancy of S on the fluid fraction, scheme, transport
variant and tile shape, batches of uneven runs, graph replay.  The draws are
fixed by the seed, so every run tests the same cases.

The bar is 1e-12 of the field's maximum.  White-noise inputs can be
conditioned worse than that (the WENO weights, with eps = 1e-6, respond
steeply to near-equal neighbours): where a field misses 1e-12, the oracle is
run again with every input perturbed by a random +-1 unit in the last
place, and the field passes if it lies within four times the change that
perturbation makes to the oracle's own output.
"""
import numpy as np
import pytest

from paper_2106_07694_amd import lbw

from parity import as_input, compare, run_gpu, run_oracle

pytestmark = pytest.mark.gpu
TOL64 = 1e-12
NCASES = 200


def _draw(rng, lattice=None, precision=None, shared=None):
    """One run's configuration (shared: the options a batch must share)."""
    lattice = lattice or int(rng.choice([9, 19]))
    if lattice == 9:
        grid = dict(nx=int(rng.integers(1, 70)), ny=int(rng.integers(6, 50)))
    else:
        grid = dict(nx=int(rng.integers(1, 20)), ny=int(rng.integers(1, 14)), nz=int(rng.integers(6, 24)))
    sh = shared or dict(
        precision=precision or str(rng.choice(["fp64", "fp64_shifted"])),
        scheme_c=str(rng.choice(["weno5", "weno3", "upwind1"])),
        has_s=bool(rng.random() < 0.5),
        fluid_mode=lbw.FLUID_LBM if rng.random() < 0.85 else lbw.FLUID_FROZEN,
    )
    kw = dict(lattice=lattice, tau=float(rng.uniform(0.52, 1.2)), gp_c=float(rng.uniform(-5e-4, 5e-4)),
              vert_periodic=bool(rng.random() < 0.25), **grid, **sh)
    ncls = int(rng.choice([1, 1, 2, 3]))
    if ncls > 1:
        kw.update(n_classes=ncls, vs_class=tuple(float(v) for v in rng.uniform(0, 4e-3, ncls)),
                  kappa_class=tuple(float(v) for v in rng.uniform(0, 2e-3, ncls)))
    else:
        kw.update(vs=float(rng.uniform(0, 4e-3)), kappa_c=float(rng.uniform(0, 2e-3)))
    if rng.random() < 0.3:
        kw["u_top"] = (float(rng.uniform(-0.03, 0.03)), float(rng.uniform(-0.03, 0.03)), 0.0)
    if rng.random() < 0.3:
        kw["body_force"] = tuple(float(v) for v in rng.uniform(-1e-4, 1e-4, 3))
    if sh["has_s"]:
        kw.update(kappa_s=float(rng.uniform(0, 2e-3)), gp_s=float(rng.uniform(-3e-4, 3e-4)))
        if rng.random() < 0.5:
            kw["vs_s"] = float(rng.uniform(0, 0.8))
        if rng.random() < 0.5:
            kw["phi_c"] = float(rng.uniform(0, 0.5))
    return lbw.RunConfig(**kw)


def _launch(rng, dim):
    choice = rng.integers(0, 4)
    if choice == 0:
        return dict(variant=1)
    if dim == 3:
        tx = int(rng.choice([32, 64, 128]))
        rows = int(rng.choice([0, 8, 16])) if tx in (32, 64) else 0
        if (tx, rows) in ((32, 8), (64, 16)):
            rows = 0
        return dict(tile_x=tx, tile_rows=rows, tile_y=int(rng.integers(2, 12)),
                    lbm_block=int(rng.choice([64, 256, 1024])))
    return dict(tile_x=int(rng.choice([64, 128, 256, 512])), tile_y=int(rng.integers(2, 40)),
                lbm_block=int(rng.choice([64, 256, 1024])))


def _inputs(cfg, rng):
    c = as_input(rng.uniform(0, 1, cfg.c_shape), cfg)
    s = as_input(rng.uniform(0, 1, cfg.shape), cfg) if cfg.has_s else None
    u = (as_input(0.04 * rng.standard_normal((cfg.dim,) + cfg.shape), cfg)
         if cfg.fluid_mode == lbw.FLUID_FROZEN else None)
    return c, s, u


def _oracle_sensitivity(cfg, c0, s0, u, nsteps, o):
    """Relative change of each oracle output field when every input value is
    moved by a random +-1 unit in the last place (FP64)."""
    rng = np.random.default_rng(7)
    nudge = lambda x: None if x is None else x * (1 + np.finfo(np.float64).eps *
                                                  rng.choice([-1.0, 1.0], size=x.shape))
    o2 = run_oracle(cfg, nudge(c0), nudge(s0), nudge(u), None, nsteps)
    return compare(o2, o)


# Draws whose conditioning sits at the 1e-12 bar: a random +-1-ulp change of
# every input moves the oracle's own output by about as much.  Only these may
# use the sensitivity allowance, and only up to 1e-11.  Case 19071 (seed
# 20071: white-noise C, WENO3, frozen flow) is the one found.
SENSITIVE = {19071}
SENSITIVE_CAP = 1e-11


@pytest.mark.parametrize("case", list(range(NCASES)) + [19071])
def test_random_config_matches_oracle(case):
    rng = np.random.default_rng(1000 + case)
    cfg = _draw(rng)
    launch = _launch(rng, cfg.dim)
    nsteps = int(rng.integers(1, 12))
    c0, s0, u = _inputs(cfg, rng)
    g = run_gpu(cfg, c0, s0, u, None, nsteps, launch=launch)
    o = run_oracle(cfg, c0, s0, u, None, nsteps)
    errs = compare(g, o)
    print(f"\ncase {case}: {cfg} {launch} steps={nsteps}: {errs}")
    bad = {k: v for k, v in errs.items() if k != "u" and not v <= TOL64}
    if bad and case in SENSITIVE:
        sens = _oracle_sensitivity(cfg, c0, s0, u, nsteps, o)
        print(f"oracle sensitivity to one ulp of its input: {sens}")
        bad = {k: v for k, v in bad.items() if not (v <= 4 * sens[k] and v <= SENSITIVE_CAP)}
    assert not bad, (errs, cfg, launch)
    if "f" in o:
        du = float(np.max(np.abs(g["u"] - o["u"])))
        bound = TOL64 * float(np.max(np.abs(o["u"]))) + 64 * np.finfo(np.float64).eps * float(np.max(np.abs(o["f"])))
        assert du <= bound, (du, bound, cfg)


@pytest.mark.parametrize("case", range(12))
def test_random_batch_equals_runs_alone(case):
    """Batches share lattice, precision, fluid mode, scheme and the S option;
    everything else varies per run.  Graph replay on half of them."""
    import torch

    rng = np.random.default_rng(5000 + case)
    first = _draw(rng, precision=str(rng.choice(["fp64", "fp32_shifted"])))
    shared = dict(precision=first.precision, scheme_c=first.scheme_c, has_s=first.has_s,
                  fluid_mode=first.fluid_mode)
    cfgs = [first] + [_draw(rng, lattice=first.lattice, shared=shared)
                      for _ in range(int(rng.integers(1, 4)))]
    launch = _launch(rng, first.dim)
    launch.pop("variant", None)
    launch["graph"] = int(case % 2)
    nsteps = int(rng.integers(2, 9))
    ins = [_inputs(c, rng) for c in cfgs]
    sol = lbw.Solver(cfgs, stream=torch.cuda.Stream())
    sol.set_launch(**launch)
    for r, (c, s, u) in enumerate(ins):
        sol.set_field("c", c, run=r)
        if s is not None:
            sol.set_field("s", s, run=r)
        if u is not None:
            sol.set_field("u", u, run=r)
        else:
            sol.init_equilibrium(run=r)
    sol.step(nsteps)
    torch.cuda.synchronize()
    keys = ["c", "deposit"] + (["f"] if first.fluid_mode == lbw.FLUID_LBM else []) + (["s"] if first.has_s else [])
    got = [{k: sol.field(k, run=r).double().cpu().numpy() for k in keys} for r in range(len(cfgs))]
    sol.close()
    one = dict(launch)
    one.pop("graph")
    for r, cfg in enumerate(cfgs):
        alone = run_gpu(cfg, ins[r][0], ins[r][1], ins[r][2], None, nsteps, launch=one)
        for k in keys:
            assert np.array_equal(got[r][k], alone[k]), (case, r, k, cfgs, launch)
