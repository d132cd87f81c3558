"""Batched runs (one persistent launch per phase over every run's tiles) and
HIP-graph replay of steps.

A batched run must give exactly the bits of the same run done alone (same
per-node arithmetic), FP64 batches must match the oracle run by run, and
graph replays must match eager steps on every replay.
"""
import numpy as np
import pytest

from paper_2106_07694_amd import lbw, workloads as W

from parity import as_input, compare, run_oracle

pytestmark = pytest.mark.gpu


def _runs(precision, has_s=False, n=5):
    grids = [(64, 48), (128, 40), (32, 64), (96, 24), (128, 96)]
    out = []
    for i in range(n):
        nx, ny = grids[i % len(grids)]
        kw = dict(has_s=True, kappa_s=1e-3, gp_s=1e-4) if has_s else {}
        out.append(lbw.RunConfig(precision=precision, nx=nx, ny=ny, tau=0.6, vs=1e-3 * (i + 1),
                                 kappa_c=1e-3, gp_c=2e-4 * (i + 1), **kw))
    return out


def _inputs(cfg, seed):
    rng = np.random.default_rng(seed)
    c0 = as_input(rng.uniform(0, 1, cfg.shape), cfg)
    s0 = as_input(rng.uniform(0, 1, cfg.shape), cfg) if cfg.has_s else None
    return c0, s0


def _state(sol, run):
    keys = ["f", "c", "u", "deposit"] + (["s"] if sol.cfgs[run].has_s else [])
    return {k: sol.field(k, run).double().cpu().numpy() for k in keys}


def _setup(sol, cfgs):
    for i, c in enumerate(cfgs):
        c0, s0 = _inputs(c, 100 + i)
        sol.set_field("c", c0, i)
        if s0 is not None:
            sol.set_field("s", s0, i)
        sol.init_equilibrium(i)


@pytest.mark.parametrize("precision", ["fp32_shifted", "fp64"])
@pytest.mark.parametrize("has_s", [False, True])
def test_batched_equals_one_at_a_time(precision, has_s):
    import torch
    cfgs = _runs(precision, has_s)
    sol = lbw.Solver(cfgs)
    _setup(sol, cfgs)
    sol.step(9)
    torch.cuda.synchronize()
    for i, c in enumerate(cfgs):
        one = lbw.Solver(c)
        _setup_one = [c]
        c0, s0 = _inputs(c, 100 + i)
        one.set_field("c", c0)
        if s0 is not None:
            one.set_field("s", s0)
        one.init_equilibrium()
        one.step(9)
        a, b = _state(sol, i), _state(one, 0)
        for k in a:
            assert np.array_equal(a[k], b[k]), (i, k)
        one.close()
    sums = sol.reduce(lbw.MASS_C) + sol.reduce(lbw.DEPOSIT)
    for i, c in enumerate(cfgs):
        c0, _ = _inputs(c, 100 + i)
        assert abs(sums[i] - c0.sum()) < 1e-5 * c0.sum()
    sol.close()


@pytest.mark.parametrize("grids", [((24, 30), (40, 24)), ((16, 36), (8, 12), (20, 7))])
def test_batch_with_fewer_tiles_than_xcds(grids):
    """A batch whose runs hold fewer transport tiles in total than the chip has
    XCDs (here 2 and 4 tiles): every tile is still computed, so each run
    equals itself alone bit for bit."""
    import torch
    cfgs = [lbw.RunConfig(precision="fp64", nx=nx, ny=ny, tau=0.6, vs=1e-3 * (i + 1), kappa_c=1e-3,
                          gp_c=2e-4, has_s=True, kappa_s=1e-3, gp_s=1e-4)
            for i, (nx, ny) in enumerate(grids)]
    sol = lbw.Solver(cfgs)
    _setup(sol, cfgs)
    sol.step(5)
    torch.cuda.synchronize()
    for i, c in enumerate(cfgs):
        one = lbw.Solver(c)
        c0, s0 = _inputs(c, 100 + i)
        one.set_field("c", c0)
        one.set_field("s", s0)
        one.init_equilibrium()
        one.step(5)
        a, b = _state(sol, i), _state(one, 0)
        for k in a:
            assert np.array_equal(a[k], b[k]), (i, k)
        one.close()
    sol.close()


def test_batched_fp64_matches_oracle():
    import torch
    cfgs = _runs("fp64", has_s=True)
    sol = lbw.Solver(cfgs)
    _setup(sol, cfgs)
    sol.step(15)
    torch.cuda.synchronize()
    for i, c in enumerate(cfgs):
        c0, s0 = _inputs(c, 100 + i)
        o = run_oracle(c, c0, s0, nsteps=15)
        g = _state(sol, i)
        errs = compare(g, o)
        errs.pop("u")
        assert max(errs.values()) < 1e-12, (i, errs)
    sol.close()


@pytest.mark.parametrize("nbatch", [1, 4])
def test_graph_replay_matches_eager(nbatch):
    """Capture two steps, replay repeatedly (odd counts, a single step and no
    step too), interleaved with eager work and syncs; every replay must equal
    the eager reference."""
    import torch
    cfgs = _runs("fp32_shifted", has_s=True, n=nbatch)
    side = torch.cuda.Stream()
    ref = lbw.Solver(cfgs, stream=side)
    gra = lbw.Solver(cfgs, stream=side)
    _setup(ref, cfgs)
    _setup(gra, cfgs)
    gra.set_launch(graph=1)
    for rep, n in enumerate((4, 2, 0, 5, 1, 6, 3)):
        ref.step(n)
        gra.step(n)
        torch.cuda.synchronize()
        # eager work of the program between replays
        _ = (torch.ones(1000, device="cuda") * rep).sum().item()
        for i in range(nbatch):
            a, b = _state(ref, i), _state(gra, i)
            for k in a:
                assert np.array_equal(a[k], b[k]), (rep, i, k)
        assert ref.steps_done() == gra.steps_done()
    ref.close()
    gra.close()


def test_sweep_config_batched_runs():
    """The seeded 64-run sweep (uneven grids) batches and conserves particles."""
    import torch
    runs = W.sweep_runs()
    cfgs = [lbw.RunConfig.from_workload(w) for w in runs]
    sol = lbw.Solver(cfgs)
    for i, w in enumerate(runs):
        sol.setup_workload(w, run=i)
    m0 = sol.reduce(lbw.MASS_C)
    sol.step(20)
    torch.cuda.synchronize()
    m1 = sol.reduce(lbw.MASS_C) + sol.reduce(lbw.DEPOSIT)
    assert np.all(np.abs(m1 - m0) < 1e-4 * np.abs(m0))
    sol.close()
