"""Parity at the full benchmark sizes, in the launch configuration bench.py
times (the tuned launch).

The oracle cannot step 33.5M cells, but one coupled step at a node depends
only on data within nine cells (three RK stages of a three-cell stencil; the
populations within one).  So the GPU state after K steps is exported, one
more GPU step is taken, and for seeded sample nodes the FP64 oracle steps a
box of radius 10 around the node cut from the GPU's state at K (walls kept
where the node is near one); the node's values must agree.  The boxes are
periodic laterally and, away from walls, vertically: their edges are wrong
after one step, their centres are not.  Budgets are checked at full size.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2106_07694_amd import autotune, lbw, workloads as W

from parity import oracle_cfg

pytestmark = pytest.mark.gpu
R = 10


def _box(arr, centre, nv_axis, lo_v, hi_v, dim):
    """Cut [centre - R, centre + R] laterally (wrapped) and [lo_v, hi_v)
    vertically from a field laid out (..., z, y, x)."""
    out = arr
    if dim == 2:
        y, x = centre
        xs = np.arange(x - R, x + R + 1) % arr.shape[-1]
        out = np.take(out[..., lo_v:hi_v, :], xs, axis=-1)
    else:
        z, y, x = centre
        xs = np.arange(x - R, x + R + 1) % arr.shape[-1]
        ys = np.arange(y - R, y + R + 1) % arr.shape[-2]
        out = out[..., lo_v:hi_v, :, :]
        out = np.take(np.take(out, ys, axis=-2), xs, axis=-1)
    return np.ascontiguousarray(out, dtype=np.float64)


def _samples(wl, n, seed):
    rng = np.random.default_rng(seed)
    nv = wl.nvert
    pts = []
    for i in range(n):
        v = [0, 1, nv - 1, nv - 2][i] if i < 4 else int(rng.integers(0, nv))
        lat = [int(rng.integers(0, wl.nx))] if wl.dim == 2 else [int(rng.integers(0, wl.ny)),
                                                                 int(rng.integers(0, wl.nx))]
        pts.append(tuple([v] + lat))
    return pts


# (workload, the workload whose tuned launch bench.py times it with)
FULL = [(W.C3, W.C3), (W.C2, W.C2), (W.C6, W.C3), (W.C7, W.C2)]


@pytest.mark.parametrize("wl,tuned", FULL, ids=["3d_256x256x512", "2d_1024x2048_s",
                                                "3d_256x256x512_4classes", "2d_1024x2048_s_full_force"])
def test_full_size_one_step_samples(wl, tuned):
    K = 3
    cfg = lbw.RunConfig.from_workload(wl)
    sol = lbw.Solver(cfg)
    launch = autotune.lookup(tuned.name)
    if launch:
        sol.set_launch(**launch)
    sol.setup_workload(wl)
    m0 = sol.reduce(lbw.MASS_C)[0]
    r0 = sol.reduce(lbw.MASS_FLUID)[0]
    s0 = sol.reduce(lbw.MASS_S)[0] if wl.has_s else None
    sol.step(K)
    torch.cuda.synchronize()
    st = {k: sol.field(k).cpu().numpy() for k in ("f", "c", "deposit")}
    if wl.has_s:
        st["s"] = sol.field("s").cpu().numpy()
    sol.step(1)
    torch.cuda.synchronize()
    nx = {k: sol.field(k).cpu().numpy() for k in ("f", "c", "deposit", "u")}
    if wl.has_s:
        nx["s"] = sol.field("s").cpu().numpy()
    # budgets at full size (FP64 sums of FP32 fields)
    m1 = sol.reduce(lbw.MASS_C)[0] + sol.reduce(lbw.DEPOSIT)[0]
    r1 = sol.reduce(lbw.MASS_FLUID)[0]
    assert abs(m1 - m0) < 1e-6 * m0, (m0, m1)
    assert abs(r1 - r0) < 1e-6 * r0, (r0, r1)
    if wl.has_s:
        s1 = sol.reduce(lbw.MASS_S)[0]
        assert abs(s1 - s0) < 1e-6 * s0, (s0, s1)
    sol.close()

    nv = wl.nvert
    worst = {}
    for p in _samples(wl, 24, seed=77):
        v = p[0]
        lo_v, hi_v = max(0, v - R), min(nv, v + R + 1)
        walls_in_box = lo_v == 0 or hi_v == nv
        box_cfg = oracle_cfg(cfg)
        if wl.dim == 2:
            box_cfg.nx, box_cfg.ny, box_cfg.nz = 2 * R + 1, hi_v - lo_v, 1
        else:
            box_cfg.nx, box_cfg.ny, box_cfg.nz = 2 * R + 1, 2 * R + 1, hi_v - lo_v
        box_cfg.vert_periodic = not walls_in_box
        if walls_in_box and lo_v != 0:
            # a box touching only the top wall: its bottom edge must not
            # absorb; extend the cut down so the bottom edge is far away
            lo_v = max(0, v - 2 * R)
            if wl.dim == 2:
                box_cfg.ny = hi_v - lo_v
            else:
                box_cfg.nz = hi_v - lo_v
        lat = p[1:]
        fbox = _box(st["f"], (v,) + tuple(lat), None, lo_v, hi_v, wl.dim)
        cbox = _box(st["c"], (v,) + tuple(lat), None, lo_v, hi_v, wl.dim)
        sbox = _box(st["s"], (v,) + tuple(lat), None, lo_v, hi_v, wl.dim) if wl.has_s else None
        f1, c1, s1, dep1, u1 = oracle.run(box_cfg, fbox, cbox, sbox, None, None, 1, want_u=True)
        # node index inside the box
        iv = v - lo_v
        if wl.dim == 2:
            sl = (0, iv, R)
            gsl = (0, v, lat[0])
            col_g, col_b = lat[0], R
        else:
            sl = (iv, R, R)
            gsl = (v, lat[0], lat[1])
            col_g, col_b = lat[0] * wl.nx + lat[1], R * (2 * R + 1) + R
        cls = (slice(None),) if cfg.ncls > 1 else ()     # every size class at the node
        scale_g = np.max(np.abs(st["f"]))
        e = {
            "f": float(np.max(np.abs(nx["f"][(slice(None),) + gsl] - f1[(slice(None),) + sl]))) / scale_g,
            "c": float(np.max(np.abs(nx["c"][cls + gsl] - c1[cls + sl]))) / max(wl.c0, 1e-30),
            "u": float(np.max(np.abs(nx["u"][(slice(None),) + gsl] - u1[(slice(None),) + sl]))),
        }
        if wl.has_s:
            e["s"] = float(abs(nx["s"][gsl] - s1[sl]))
        if v == 0:
            inc_g = nx["deposit"][cls + (col_g,)] - st["deposit"][cls + (col_g,)]
            vs_max = max((wl.vs,) + tuple(wl.vs_class))
            e["deposit_step"] = float(np.max(np.abs(inc_g - dep1[cls + (col_b,)]))) / (vs_max * wl.c0)
        for k, val in e.items():
            worst[k] = max(worst.get(k, 0.0), val)
    print(f"\n{wl.name}: worst sampled one-step errors after {K} steps: {worst}")
    assert worst["f"] < 1e-5 and worst["c"] < 1e-6 and worst["u"] < 1e-7, worst
    if "s" in worst:
        assert worst["s"] < 1e-6, worst
    assert worst.get("deposit_step", 0.0) < 1e-5, worst
