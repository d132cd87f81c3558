"""Form (1) at the full benchmark grids, element by element against the FP64
oracle, in the launch configuration bench.py times (the tuned launch).

The 2D two-scalar workload (1024 x 2048 with S) runs 100 steps and the 3D
workload (256 x 256 x 512) 10 steps from the same seeded state on both sides
(the oracle needs about 12 s and 20 s of 16 host cores for them); every
field is compared with the FP32 bounds of tests/test_gpu_fp32.py: u 1e-4,
C 1e-5, S 1e-5, populations 1e-4 of the field's maximum.  The deposit is
compared with the oracle's own deposit (max |dD| / max |D|): it is an FP64
sum of the bottom cells' FP32 concentrations, so its relative error is that
of the bottom plane's concentration relative to itself, bounded like C's,
1e-5 (measured 2.6e-7 to 5.7e-7).

The batched sweep's 64 runs (529 MB of populations) take the non-temporal
collide-stream path, which smaller batches never reach: it must give the
same bits as the runs alone (temporal path).
"""
import numpy as np
import pytest
import torch

from paper_2106_07694_amd import autotune, lbw, workloads as W

from parity import as_input, compare, run_oracle

pytestmark = pytest.mark.gpu
TOL = {"u": 1e-4, "c": 1e-5, "s": 1e-5, "f": 1e-4}
TOL_DEPOSIT = 1e-5


def _gpu(wl, cfg, c0, s0, nsteps):
    sol = lbw.Solver(cfg)
    sol.set_launch(**(autotune.lookup(wl.name) or {}))
    sol.set_field("c", c0)
    if s0 is not None:
        sol.set_field("s", s0)
    sol.init_equilibrium()
    sol.step(nsteps)
    torch.cuda.synchronize()
    out = {k: sol.field(k).double().cpu().numpy() for k in ("c", "u", "deposit", "f")}
    if cfg.has_s:
        out["s"] = sol.field("s").double().cpu().numpy()
    sol.close()
    return out


@pytest.mark.parametrize("wl,nsteps", [(W.C2, 100), (W.C3, 10)], ids=["2d_1024x2048_s", "3d_256x256x512"])
def test_full_grid_fp32_against_oracle(wl, nsteps):
    cfg = lbw.RunConfig.from_workload(wl)
    c0, s0 = W.initial_scalars(wl)
    c0, s0 = as_input(c0, cfg), as_input(s0, cfg)
    print(f"\n[{wl.name}] GPU {nsteps} steps", flush=True)
    g = _gpu(wl, cfg, c0, s0, nsteps)
    print(f"[{wl.name}] oracle {nsteps} steps", flush=True)
    o = run_oracle(cfg, c0, s0, nsteps=nsteps)
    dep = o.pop("deposit")
    errs = compare(g, o)
    errs["deposit"] = float(np.max(np.abs(g["deposit"] - dep))) / float(np.max(np.abs(dep)))
    print(f"[{wl.name}] relative errors after {nsteps} steps: {errs}", flush=True)
    for k, v in errs.items():
        assert v <= (TOL_DEPOSIT if k == "deposit" else TOL[k]), (k, v, errs)


def test_sweep_batch_non_temporal_path_equals_runs_alone():
    runs = W.sweep_runs()
    cfgs = [lbw.RunConfig.from_workload(w) for w in runs]
    pop_bytes = sum(c.lattice * c.cells * 4 for c in cfgs)
    assert pop_bytes > 192 << 20          # beyond the size that switches to non-temporal access
    launch = autotune.lookup("sweep_64") or {}
    nsteps = 6
    sol = lbw.Solver(cfgs, stream=torch.cuda.Stream())
    sol.set_launch(**launch)
    for i, w in enumerate(runs):
        sol.setup_workload(w, run=i)
    sol.step(nsteps)
    torch.cuda.synchronize()
    big = max(range(len(runs)), key=lambda i: runs[i].cells)
    picks = sorted({0, big, len(runs) - 1})
    batched = {i: {k: sol.field(k, run=i).cpu().numpy() for k in ("f", "c", "u", "deposit")}
               for i in picks}
    sol.close()
    for i in picks:
        one = lbw.Solver(cfgs[i])
        one.set_launch(**{k: v for k, v in launch.items() if k != "graph"})
        one.setup_workload(runs[i])
        one.step(nsteps)
        torch.cuda.synchronize()
        for k in ("f", "c", "u", "deposit"):
            assert np.array_equal(one.field(k).cpu().numpy(), batched[i][k]), (i, k)
        one.close()
