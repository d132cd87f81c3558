"""GPU parity of the in-situ diagnostics (front height per column, its power
spectral density along a lateral axis, particle mass below a horizontal
plane) against the FP64 oracle on the same seeded fields.

The front height compares C with the threshold in FP64 and interpolates in
the same operation order on both sides (no products, so no fused
multiply-add can differ): it must agree bit for bit.  The mass below a plane
is the same deterministic tree reduction as the mass sums against the
oracle's sequential sum: 1e-12 relative.  The spectrum is a sum of L terms
with sines and cosines of the exact phase on both sides: bounded as stated
in _psd_close.
"""
import numpy as np
import pytest

import oracle
from paper_2106_07694_amd import lbw, workloads as W

from parity import as_input, oracle_cfg, run_oracle

pytestmark = pytest.mark.gpu
TOL64 = 1e-12


def _solver_with(cfg, c):
    sol = lbw.Solver(cfg)
    sol.set_field("c", c)
    if cfg.fluid_mode == lbw.FLUID_LBM:
        sol.init_equilibrium()
    return sol


def _layer(cfg, seed, width=3.0, amp=0.05):
    """Particle-laden fluid above clear fluid with a seeded, column-wise
    random interface displacement and cell noise."""
    rng = np.random.default_rng(seed)
    nv = cfg.ny if cfg.dim == 2 else cfg.nz
    lateral = (1, 1, cfg.nx) if cfg.dim == 2 else (1, cfg.ny, cfg.nx)
    disp = rng.uniform(-0.25, 0.25, lateral) * nv
    v = np.arange(nv, dtype=np.float64)
    v = v[None, :, None] if cfg.dim == 2 else v[:, None, None]
    c = 0.5 * (1 + np.tanh((v - 0.5 * (nv - 1) - disp) / width))
    c = c + amp * rng.uniform(-1, 1, cfg.shape)
    return as_input(c, cfg)


CASES = [
    dict(nx=37, ny=29),
    dict(nx=64, ny=128, precision="fp32_shifted"),
    dict(lattice=19, nx=9, ny=7, nz=23),
    dict(lattice=19, nx=33, ny=17, nz=40, precision="fp32_shifted"),
    dict(nx=1, ny=6),
    dict(lattice=19, nx=1, ny=1, nz=6, precision="fp32_shifted"),
    dict(nx=70, ny=700, precision="fp32_shifted"),                  # several rounds of the scan
    dict(lattice=19, nx=130, ny=128, nz=70),                        # many columns, several rounds
]


@pytest.mark.parametrize("kw", CASES)
@pytest.mark.parametrize("field", ["layer", "uniform_random"])
def test_front_height_bitwise(kw, field):
    import torch

    cfg = lbw.RunConfig(tau=0.6, vs=1e-3, kappa_c=1e-3, gp_c=1e-5, **kw)
    if field == "layer":
        c = _layer(cfg, 11)
    else:
        c = as_input(np.random.default_rng(12).uniform(0, 1, cfg.shape), cfg)
    sol = _solver_with(cfg, c)
    ocfg = oracle_cfg(cfg)
    for thr in (0.5, 0.05, 0.95, float(c.flat[c.size // 2]), -1.0, 2.0):
        got = sol.front_height(thr)
        torch.cuda.synchronize()
        want = oracle.front_height(ocfg, c, thr)
        assert got.shape == ((cfg.nx,) if cfg.dim == 2 else (cfg.ny, cfg.nx))
        assert np.array_equal(got.cpu().numpy().ravel(), want), (thr, kw)
    sol.close()


def test_front_height_degenerate_columns():
    """Bottom cell at the threshold gives 0; no cell reaching it gives nv."""
    import torch

    cfg = lbw.RunConfig(nx=4, ny=8, tau=0.6, vs=1e-3, kappa_c=1e-3, gp_c=1e-5)
    c = np.zeros(cfg.shape)
    c[0, :, 1] = 0.5                      # column 1: every cell at the threshold
    c[0, 5:, 2] = 1.0                     # column 2: step between cells 4 and 5
    sol = _solver_with(cfg, c)
    got = sol.front_height(0.5)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    assert np.array_equal(got, oracle.front_height(oracle_cfg(cfg), c, 0.5))
    assert got[0] == 8.0 and got[3] == 8.0 and got[1] == 0.0 and got[2] == 5.0
    sol.close()


@pytest.mark.parametrize("kw", CASES)
def test_mass_below_matches_oracle(kw):
    cfg = lbw.RunConfig(tau=0.6, vs=1e-3, kappa_c=1e-3, gp_c=1e-5, **kw)
    c = _layer(cfg, 13)
    sol = _solver_with(cfg, c)
    ocfg = oracle_cfg(cfg)
    nv = cfg.ny if cfg.dim == 2 else cfg.nz
    total = sol.reduce(lbw.MASS_C)[0]
    for plane in sorted({0, 1, nv // 3, nv // 2, nv - 1, nv}):
        got = sol.mass_below(plane)
        assert got.shape == (1,)
        want = oracle.mass_below(ocfg, c, plane)
        assert abs(got[0] - want) <= TOL64 * max(abs(want), 1e-300), (plane, got, want)
    assert sol.mass_below(0)[0] == 0.0
    assert sol.mass_below(nv)[0] == total        # same reduction over the same cells
    sol.close()


def test_mass_below_rejects_planes_outside_the_domain():
    cfg = lbw.RunConfig(nx=8, ny=10, tau=0.6, vs=1e-3, kappa_c=1e-3, gp_c=1e-5)
    sol = _solver_with(cfg, np.ones(cfg.shape))
    for plane in (-1, 11):
        with pytest.raises(lbw.LbwError):
            sol.mass_below(plane)
    with pytest.raises(lbw.LbwError):
        sol.front_height(float("nan"))
    sol.close()


def test_batch_diagnostics_per_run():
    """Runs of uneven height in one batch: each run's mass below a plane and
    front height equal the oracle's on that run's field."""
    import torch

    runs = [w for w in W.sweep_runs(6, grids=((16, 24), (32, 40), (24, 32)))]
    cfgs = [lbw.RunConfig.from_workload(w) for w in runs]
    sol = lbw.Solver(cfgs)
    fields = []
    for r, (w, cfg) in enumerate(zip(runs, cfgs)):
        c = as_input(W.initial_scalars(w)[0], cfg)
        fields.append(c)
        sol.set_field("c", c, run=r)
        sol.init_equilibrium(run=r)
    plane = min(c.ny for c in cfgs) // 2
    got = sol.mass_below(plane)
    for r, (cfg, c) in enumerate(zip(cfgs, fields)):
        want = oracle.mass_below(oracle_cfg(cfg), c, plane)
        assert abs(got[r] - want) <= TOL64 * abs(want), (r, got[r], want)
        thr = 0.5 * runs[r].c0
        h = sol.front_height(thr, run=r)
        torch.cuda.synchronize()
        assert np.array_equal(h.cpu().numpy(), oracle.front_height(oracle_cfg(cfg), c, thr)), r
    with pytest.raises(lbw.LbwError):
        sol.mass_below(max(c.ny for c in cfgs))   # beyond the lowest run
    sol.close()


def test_front_height_after_steps_fp64():
    """After stepping both sides from the seeded two-layer state, the front
    heights agree to the accuracy of the fields themselves."""
    import torch

    wl = W.C1.replace(nx=48, ny=64)
    cfg = lbw.RunConfig.from_workload(wl)
    c0, _ = W.initial_scalars(wl)
    sol = _solver_with(cfg, c0)
    sol.step(200)
    got = sol.front_height(0.5)
    torch.cuda.synchronize()
    o = run_oracle(cfg, c0, nsteps=200)
    want = oracle.front_height(oracle_cfg(cfg), o["c"], 0.5)
    assert np.max(np.abs(got.cpu().numpy() - want)) <= 1e-9
    ocfg = oracle_cfg(cfg)
    for plane in (10, 32):
        m = sol.mass_below(plane)[0]
        mw = oracle.mass_below(ocfg, o["c"], plane)
        assert abs(m - mw) <= TOL64 * abs(mw)
    sol.close()


def _lateral(cfg):
    return (cfg.nx,) if cfg.dim == 2 else (cfg.ny, cfg.nx)


def _psd_close(got, want, h, cfg, axis):
    """Rounding bound of the transform: each |X(k)| = |sum_j H_j e^(..)| may
    differ by delta = 1e-13 sum_j |H_j| (sum order and the sine/cosine of
    the exact phase, both within L eps), so Gamma = |X|^2 / L by at most
    (2 sqrt(L Gamma) delta + delta^2) / L, also for the mean over rows."""
    rows = np.asarray(h, np.float64).reshape(_lateral(cfg) if cfg.dim == 3 else (1, cfg.nx))
    if axis == 1:
        rows = rows.T
    length = rows.shape[1]
    delta = 1e-13 * float(np.max(np.sum(np.abs(rows), axis=1)))
    bound = (2 * np.sqrt(length * np.abs(want)) * delta + delta * delta) / length
    assert np.all(np.abs(got - want) <= bound), float(np.max(np.abs(got - want) / bound))


PSD_CASES = [
    (dict(nx=37, ny=29), 0, 0),
    (dict(nx=64, ny=128, precision="fp32_shifted"), 0, 0),
    (dict(nx=1, ny=6), 0, 0),
    (dict(nx=2, ny=6), 0, -1),
    (dict(lattice=19, nx=9, ny=7, nz=23), 0, 3),
    (dict(lattice=19, nx=9, ny=7, nz=23), 1, 8),
    (dict(lattice=19, nx=33, ny=17, nz=40, precision="fp32_shifted"), 0, -1),
    (dict(lattice=19, nx=33, ny=17, nz=40, precision="fp32_shifted"), 1, -1),
    (dict(lattice=19, nx=300, ny=2, nz=6), 0, 1),
    (dict(lattice=19, nx=3, ny=2100, nz=6), 1, -1),                 # row longer than the LDS table
    (dict(lattice=19, nx=130, ny=128, nz=70), 1, 77),
    (dict(lattice=19, nx=70, ny=30, nz=6), 1, -1),                  # one lane per row
    (dict(lattice=19, nx=20, ny=65, nz=6), 0, -1),
    (dict(lattice=19, nx=2049, ny=64, nz=6), 0, -1),                # lanes, no LDS table
]


@pytest.mark.parametrize("kw,axis,index", PSD_CASES)
def test_front_psd_matches_oracle(kw, axis, index):
    """The spectrum of the in-situ front height against the oracle's spectrum
    of the oracle's front height (the two heights are equal bit for bit),
    and repeated calls give the same bits."""
    import torch

    cfg = lbw.RunConfig(tau=0.6, vs=1e-3, kappa_c=1e-3, gp_c=1e-5, **kw)
    c = _layer(cfg, 15)
    ocfg = oracle_cfg(cfg)
    sol = _solver_with(cfg, c)
    h = sol.front_height(0.5)
    g = sol.front_psd(h, axis, index)
    g2 = sol.front_psd(h, axis, index)
    torch.cuda.synchronize()
    h_o = oracle.front_height(ocfg, c, 0.5)
    assert np.array_equal(h.cpu().numpy().ravel(), h_o)
    want = oracle.front_psd(ocfg, h_o, axis, index)
    length = cfg.nx if axis == 0 else cfg.ny
    assert g.shape == (length // 2 + 1,)
    _psd_close(g.cpu().numpy(), want, h_o, cfg, axis)
    assert torch.equal(g, g2)
    sol.close()


@pytest.mark.parametrize("nx", [1, 2, 63, 64, 1024, 2048, 2049, 5000])
def test_front_psd_of_seeded_heights(nx):
    """Seeded heights uploaded directly (not produced by the front kernel)."""
    import torch

    cfg = lbw.RunConfig(nx=nx, ny=40, tau=0.6, vs=1e-3, kappa_c=1e-3, gp_c=1e-5)
    h = np.random.default_rng(nx).uniform(0, 40, nx)
    sol = lbw.Solver(cfg)
    g = sol.front_psd(torch.tensor(h, device="cuda"))
    torch.cuda.synchronize()
    want = oracle.front_psd(oracle_cfg(cfg), h)
    _psd_close(g.cpu().numpy(), want, h, cfg, 0)
    sol.close()


def test_front_psd_rejects_bad_axes_and_rows():
    import torch

    cfg2 = lbw.RunConfig(nx=8, ny=10, tau=0.6, vs=1e-3, kappa_c=1e-3, gp_c=1e-5)
    cfg3 = lbw.RunConfig(lattice=19, nx=8, ny=5, nz=10, tau=0.6, vs=1e-3, kappa_c=1e-3, gp_c=1e-5)
    for cfg, bad in ((cfg2, [(1, 0), (0, 1), (0, -2), (2, 0)]),
                     (cfg3, [(0, 5), (1, 8), (0, -2), (2, 0), (-1, 0)])):
        sol = lbw.Solver(cfg)
        h = torch.zeros(cfg.ncol, dtype=torch.float64, device="cuda")
        out = torch.zeros(64, dtype=torch.float64, device="cuda")
        for axis, index in bad:
            with pytest.raises(lbw.LbwError):
                length = cfg.nx if axis == 0 else cfg.ny
                sol.front_psd(h, axis, index, out=out[: length // 2 + 1])
        sol.close()


def test_front_height_full_3d_size():
    """At the full 3D size (256 x 256 x 512, FP32 storage) on a seeded layer
    field: every column's front height equals the oracle's."""
    import torch

    wl = W.C3
    cfg = lbw.RunConfig.from_workload(wl)
    c = _layer(cfg, 14, width=8.0, amp=0.02)
    sol = lbw.Solver(cfg)
    sol.set_field("c", c)
    got = sol.front_height(0.5)
    torch.cuda.synchronize()
    want = oracle.front_height(oracle_cfg(cfg), c, 0.5)
    assert np.array_equal(got.cpu().numpy().ravel(), want)
    for axis in (0, 1):
        g = sol.front_psd(got, axis, -1)
        torch.cuda.synchronize()
        _psd_close(g.cpu().numpy(), oracle.front_psd(oracle_cfg(cfg), want, axis, -1), want, cfg, axis)
    m = sol.mass_below(wl.nz // 2)[0]
    mw = oracle.mass_below(oracle_cfg(cfg), c, wl.nz // 2)
    assert abs(m - mw) <= TOL64 * abs(mw)
    sol.close()


@pytest.mark.parametrize("kw", [
    dict(nx=37, ny=29, has_s=True, kappa_s=1e-3, gp_s=1e-4),
    dict(nx=37, ny=29, precision="fp32_shifted"),
    dict(lattice=19, nx=9, ny=7, nz=23, precision="fp64_shifted", has_s=True, kappa_s=1e-3,
         gp_s=1e-4),
    dict(lattice=19, nx=130, ny=128, nz=70),
])
@pytest.mark.parametrize("nsteps", [0, 3])
def test_reduction_sums_match_oracle(kw, nsteps):
    """The four FP64 sums (C, S, fluid mass, deposit) of lbw_reduce against
    the oracle's sequential sums of the oracle's state, after an even and an
    odd number of steps (the in-place populations sit in the other layout)."""
    cfg = lbw.RunConfig(tau=0.6, vs=2e-3, kappa_c=1e-3, gp_c=1e-4, **kw)
    rng = np.random.default_rng(21)
    c0 = as_input(rng.uniform(0, 1, cfg.shape), cfg)
    s0 = as_input(rng.uniform(0, 1, cfg.shape), cfg) if cfg.has_s else None
    sol = lbw.Solver(cfg)
    sol.set_field("c", c0)
    if s0 is not None:
        sol.set_field("s", s0)
    sol.init_equilibrium()
    sol.step(nsteps)
    got = {w: sol.reduce(w)[0] for w in (lbw.MASS_C, lbw.MASS_FLUID, lbw.DEPOSIT)}
    if cfg.has_s:
        got[lbw.MASS_S] = sol.reduce(lbw.MASS_S)[0]
    sol.close()
    o = run_oracle(cfg, c0, s0, nsteps=nsteps)
    want = oracle.sums(oracle_cfg(cfg), o["f"], o["c"], o.get("s"), o["deposit"])
    tol = TOL64 if cfg.precision != "fp32_shifted" else 3e-6
    for w, i in ((lbw.MASS_C, 0), (lbw.MASS_S, 1), (lbw.MASS_FLUID, 2), (lbw.DEPOSIT, 3)):
        if w in got:
            scale = max(abs(want[i]), 1e-300)
            assert abs(got[w] - want[i]) <= tol * scale, (w, got[w], want[i])
