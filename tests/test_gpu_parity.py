"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs, element by element.

FP64 forms must agree to 1e-12 relative (max |gpu - oracle| / max |oracle|
per field).  The velocity is a difference of populations a hundred thousand
times larger than itself early in a run, so its bound is 1e-12 relative plus
an absolute floor of 64 units in the last place of the largest population.
Cases span several blocks with ragged tails, both lattices, walls and
periodic vertical axes, a moving lid and body force, the frozen
(transport-only) mode with every scheme, the S scalar and the shifted form.
"""
import numpy as np
import pytest

from paper_2106_07694_amd import lbw, workloads as W

from parity import as_input, compare, run_gpu, run_oracle

pytestmark = pytest.mark.gpu
TOL64 = 1e-12


def _check(cfg, nsteps, c0, s0=None, u=None, f0=None, tol=TOL64, launch=None):
    c0, s0, u = as_input(c0, cfg), as_input(s0, cfg), as_input(u, cfg)
    g = run_gpu(cfg, c0, s0, u, f0, nsteps, launch=launch)
    o = run_oracle(cfg, c0, s0, u, f0, nsteps)
    errs = compare(g, o)
    print(f"\n{cfg.lattice} {cfg.precision} {cfg.nx}x{cfg.ny}x{cfg.nz} steps={nsteps}: {errs}")
    bad = {k: v for k, v in errs.items() if k != "u" and not v <= tol}
    assert not bad, errs
    if "f" in o:
        du = float(np.max(np.abs(g["u"] - o["u"])))
        fscale = float(np.max(np.abs(o["f"])))
        bound = tol * float(np.max(np.abs(o["u"]))) + 64 * np.finfo(np.float64).eps * fscale
        assert du <= bound, (du, bound, errs)
    else:
        assert errs["u"] == 0.0       # frozen: the velocity is an input
    return errs


@pytest.mark.parametrize("nsteps", [1, 10, 100, 1000])
def test_c1_full_fp64(nsteps):
    """2D D2Q9 FP64 on 64x128, the seeded two-layer workload."""
    wl = W.C1
    cfg = lbw.RunConfig.from_workload(wl)
    c0, _ = W.initial_scalars(wl)
    _check(cfg, nsteps, c0)


def _rng_fields(cfg, seed):
    rng = np.random.default_rng(seed)
    c0 = rng.uniform(0, 1, cfg.shape)
    s0 = rng.uniform(0, 1, cfg.shape) if cfg.has_s else None
    return c0, s0


@pytest.mark.parametrize("kw", [
    dict(nx=37, ny=29),                                             # ragged tail
    dict(nx=37, ny=29, vert_periodic=True),
    dict(nx=33, ny=21, u_top=(0.02, 0, 0), body_force=(1e-4, 0, 0)),
    dict(nx=1, ny=6),                                               # degenerate lateral, minimal height
    dict(nx=64, ny=40, has_s=True, kappa_s=1e-3, gp_s=-2e-4),
    dict(nx=40, ny=24, precision="fp64_shifted", has_s=True, kappa_s=1e-3, gp_s=2e-4),
    dict(nx=16, ny=12, vs=0.0, kappa_c=0.0, gp_c=0.0),             # uncoupled: no settling, diffusion, buoyancy
])
def test_d2q9_fp64_variants(kw):
    base = dict(tau=0.6, vs=2e-3, kappa_c=2e-3, gp_c=5e-4)
    base.update(kw)
    cfg = lbw.RunConfig(**base)
    c0, s0 = _rng_fields(cfg, 3)
    _check(cfg, 25, c0, s0)


@pytest.mark.parametrize("kw", [
    dict(nx=12, ny=10, nz=16),
    dict(nx=9, ny=7, nz=11, vert_periodic=True),
    dict(nx=8, ny=6, nz=12, u_top=(0.02, -0.01, 0), body_force=(1e-4, 0, 2e-5)),
    dict(nx=10, ny=6, nz=8, precision="fp64_shifted", has_s=True, kappa_s=1e-3, gp_s=1e-4),
    dict(nx=1, ny=3, nz=6),                                         # degenerate lateral axes, minimal height
    dict(nx=5, ny=1, nz=9, vert_periodic=True),
])
def test_d3q19_fp64_variants(kw):
    base = dict(lattice=19, tau=0.55, vs=2e-3, kappa_c=2e-3, gp_c=5e-4)
    base.update(kw)
    cfg = lbw.RunConfig(**base)
    c0, s0 = _rng_fields(cfg, 4)
    _check(cfg, 20, c0, s0)


@pytest.mark.parametrize("lattice", [9, 19])
@pytest.mark.parametrize("scheme", ["weno5", "weno3", "upwind1"])
@pytest.mark.parametrize("vper", [False, True])
def test_frozen_transport(lattice, scheme, vper):
    shape = dict(nx=29, ny=23) if lattice == 9 else dict(nx=11, ny=9, nz=13)
    cfg = lbw.RunConfig(lattice=lattice, fluid_mode=lbw.FLUID_FROZEN, scheme_c=scheme,
                        vert_periodic=vper, vs=0.03, kappa_c=5e-3, has_s=True, kappa_s=2e-3,
                        **shape)
    rng = np.random.default_rng(5)
    c0, s0 = _rng_fields(cfg, 6)
    u = 0.05 * rng.standard_normal((cfg.dim,) + cfg.shape)
    _check(cfg, 15, c0, s0, u)


def test_zero_steps_is_identity():
    cfg = lbw.RunConfig(nx=16, ny=12, vs=1e-3, kappa_c=1e-3, gp_c=1e-4)
    c0, _ = _rng_fields(cfg, 7)
    errs = _check(cfg, 0, c0)
    assert errs["c"] == 0.0


@pytest.mark.parametrize("lbm_block", [64, 128, 512, 1024])
def test_launch_shapes_give_identical_bits(lbm_block):
    wl = W.C1.replace(nx=48, ny=40)
    cfg = lbw.RunConfig.from_workload(wl)
    c0, _ = W.initial_scalars(wl)
    ref = run_gpu(cfg, c0, nsteps=7)
    got = run_gpu(cfg, c0, nsteps=7, launch=dict(lbm_block=lbm_block))
    for k in ref:
        assert np.array_equal(ref[k], got[k]), k


@pytest.mark.parametrize("launch", [
    dict(variant=1),
    dict(tile_x=64, tile_y=7),
    dict(tile_x=128, tile_y=5),
    dict(tile_x=256, tile_y=1000),
    dict(tile_x=512, tile_y=6),
])
def test_2d_transport_launches(launch):
    """Every transport tiling, ragged chunks included, matches the oracle."""
    cfg = lbw.RunConfig(nx=150, ny=37, tau=0.6, vs=2e-3, kappa_c=2e-3, gp_c=5e-4,
                        has_s=True, kappa_s=1e-3, gp_s=1e-4)
    c0, s0 = _rng_fields(cfg, 8)
    _check(cfg, 12, c0, s0, launch=launch)


@pytest.mark.parametrize("launch", [
    dict(variant=1),
    dict(tile_x=32, tile_y=5),
    dict(tile_x=64, tile_y=3),
    dict(tile_x=128, tile_y=64),
    dict(tile_x=32, tile_rows=16, tile_y=5),
    dict(tile_x=64, tile_rows=8, tile_y=3),
])
@pytest.mark.parametrize("vper", [False, True])
def test_3d_transport_launches(launch, vper):
    cfg = lbw.RunConfig(lattice=19, nx=45, ny=11, nz=14, tau=0.55, vs=2e-3, kappa_c=2e-3,
                        gp_c=5e-4, vert_periodic=vper)
    c0, _ = _rng_fields(cfg, 9)
    _check(cfg, 8, c0, launch=launch)


@pytest.mark.parametrize("frozen", [False, True])
def test_rebound_step_outputs_are_written_in_place(frozen):
    """Rebinding the velocity and RK-stage buffers to caller tensors: every
    step writes them there, bit for bit what the default buffers receive,
    and the state evolves identically."""
    import torch

    wl = W.C1.replace(nx=40, ny=36)
    cfg = lbw.RunConfig.from_workload(wl)
    if frozen:
        cfg = lbw.RunConfig(**{**cfg.__dict__, "fluid_mode": lbw.FLUID_FROZEN})
    c0, _ = W.initial_scalars(wl)
    u0 = np.random.default_rng(3).uniform(-0.05, 0.05, (cfg.dim,) + cfg.shape)
    sols = [lbw.Solver(cfg), lbw.Solver(cfg)]
    for s in sols:
        s.set_field("c", c0)
        if frozen:
            s.set_field("u", u0)
        else:
            s.init_equilibrium()
    names = ("stage1", "stage2") if frozen else ("u", "stage1", "stage2")
    ref, bound = sols
    for n in range(4):
        outs = {k: torch.full_like(ref.field(k), float("nan")) for k in names}
        for k in names:
            bound.rebind(k, outs[k])
        ref.step(1)
        bound.step(1)
        torch.cuda.synchronize()
        for k in names:
            assert torch.equal(outs[k], ref.field(k)), (n, k)
        for k in ("f", "c", "deposit") if not frozen else ("c", "deposit"):
            assert torch.equal(bound.field(k), ref.field(k)), (n, k)
    for k in names:
        bound.rebind(k, None)
    bound.step(1)
    ref.step(1)
    for k in names:
        assert torch.equal(bound.field(k), ref.field(k)), k
    for s in sols:
        s.close()


@pytest.mark.parametrize("kw", [dict(), dict(vert_periodic=True), dict(precision="fp64_shifted")])
def test_tall_grid_more_planes_than_one_launch_row(kw):
    """A vertical extent beyond 65,535 planes: the S update strides its
    planes over the launch's second grid dimension, and the transport's
    vertical chunks number in the tens of thousands."""
    cfg = lbw.RunConfig(nx=3, ny=70001, vs=2e-3, kappa_c=1e-3, has_s=True, kappa_s=1e-3,
                        fluid_mode=lbw.FLUID_FROZEN, **kw)
    rng = np.random.default_rng(71)
    c0, s0 = rng.uniform(0, 1, cfg.shape), rng.uniform(0, 1, cfg.shape)
    u = 0.05 * rng.standard_normal((cfg.dim,) + cfg.shape)
    _check(cfg, 3, c0, s0, u, launch=dict(tile_x=64, tile_y=2))


@pytest.mark.parametrize("kw", [dict(nx=70, ny=33), dict(nx=70, ny=33, vert_periodic=True),
                                dict(lattice=19, nx=21, ny=13, nz=17),
                                dict(lattice=19, nx=21, ny=13, nz=17, vert_periodic=True)])
@pytest.mark.parametrize("precision", ["fp64", "fp32_shifted"])
def test_s_update_fused_in_stage1_equals_separate_kernel(kw, precision):
    """The tiled transport carries the S update in its first stage; the plain
    transport runs it as a kernel of its own.  Same arithmetic and sum order:
    S agrees to a few units in the last place (frozen flow, so only the S
    update differs between the two paths)."""
    cfg = lbw.RunConfig(fluid_mode=lbw.FLUID_FROZEN, has_s=True, kappa_s=1e-3, vs=2e-3,
                        kappa_c=1e-3, precision=precision, **kw)
    rng = np.random.default_rng(73)
    c0 = as_input(rng.uniform(0, 1, cfg.shape), cfg)
    s0 = as_input(rng.uniform(0, 1, cfg.shape), cfg)
    u = as_input(0.05 * rng.standard_normal((cfg.dim,) + cfg.shape), cfg)
    fused = run_gpu(cfg, c0, s0, u, None, 9, launch=dict(tile_x=64, tile_y=5))
    plain = run_gpu(cfg, c0, s0, u, None, 9, launch=dict(variant=1))
    eps = np.finfo(np.float64 if precision == "fp64" else np.float32).eps
    d = float(np.max(np.abs(fused["s"] - plain["s"]))) / float(np.max(np.abs(plain["s"])))
    print(f"\n{precision} {kw}: S fused vs separate {d:.2e} ({int(np.count_nonzero(fused['s'] != plain['s']))} cells differ)")
    assert d <= 8 * eps, d
