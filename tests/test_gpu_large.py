"""Runs of more than 2^31 cells: the largest grids one device holds.

Cell indices, population slots (19 N values in 3D) and byte offsets then
pass 2^31, so any 32-bit index on the path would wrap.  A run whose initial
state repeats laterally with period P (3D: 64 x 64 columns, 2D: 512
columns; lateral walls are periodic) keeps that period exactly: with P a
whole number of transport tiles, every tile of the large run is computed by
the same kernel instantiation, with the same arithmetic, as the tiles of a
P-wide run of the same height.  After two steps (one even and one odd
collide-stream half, three RK stages each) every lateral copy of the large
run must equal the small run bit for bit: C, S, the velocity, the raw
population buffer, the deposit and the front height; the FP64 sums (C, fluid
mass, deposit) equal the number of copies times the small run's to rounding.
The small run itself is compared with the FP64 oracle at the FP32 bounds of
tests/test_gpu_fp32.py.

The workloads' physics and launch (the tuned launch bench.py times) on
  3D: 1024 x 1024 x 2049 = 2^31 + 2^20 cells, 215 GB of device memory;
  2D with S: 65536 x 32769 = 2^31 + 2^16 cells, 138 GB;
  2D with S: 536870400 x 6 (a plane of 2^29 - 512 cells, just under the
  limit, over the minimal height), 3.2e9 cells, 206 GB;
each from the seeded tanh-layer state (C noise of amplitude 1e-3) plus a
smooth initial velocity of amplitude 0.02 that varies along every axis.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2106_07694_amd import autotune, lbw, workloads as W

from parity import as_input, compare, oracle_cfg, run_oracle

pytestmark = pytest.mark.gpu
TOL = {"u": 1e-4, "c": 1e-5, "s": 1e-5, "f": 1e-4}
TOL_DEPOSIT = 1e-5
STEPS = 2

# (workload, large lateral sizes, small lateral sizes, vertical extent)
CASES = {
    "3d_1024x1024x2049": (W.C3, (1024, 1024), (64, 64), 2049),
    "2d_s_65536x32769": (W.C2, (65536, 1), (512, 1), 32769),
    # the widest plane a run may have (lanes address a plane with 32-bit byte
    # offsets, here up to 2^31 - 2048) over the minimal height
    "2d_s_536870400x6": (W.C2, (536870400, 1), (512, 1), 6),
}


def _cfg(wl, lateral, nv):
    if wl.dim == 3:
        return lbw.RunConfig.from_workload(wl, nx=lateral[0], ny=lateral[1], nz=nv)
    return lbw.RunConfig.from_workload(wl, nx=lateral[0], ny=nv, nz=1)


def _velocity(cfg, amp=0.02):
    """Smooth velocity, periodic over the small run's lateral sizes, varying
    along every axis (float64, shape (dim, nz, ny, nx))."""
    z = np.arange(cfg.nz, dtype=np.float64)[:, None, None]
    y = np.arange(cfg.ny, dtype=np.float64)[None, :, None]
    x = np.arange(cfg.nx, dtype=np.float64)[None, None, :]
    kx = 2 * math.pi / cfg.nx
    shape = (cfg.nz, cfg.ny, cfg.nx)
    if cfg.dim == 3:
        ky = 2 * math.pi / cfg.ny
        parts = [np.sin(ky * y + 0.011 * z), np.sin(kx * x - 0.017 * z),
                 np.cos(kx * x) * np.cos(ky * y + 0.013 * z)]
    else:
        parts = [np.sin(0.019 * y + 0.3), np.cos(kx * x + 0.007 * y)]
    u = np.stack([np.broadcast_to(p, shape) for p in parts])
    return amp * u


def _bytes(cfg):
    es = 4
    per = cfg.lattice + 3 + cfg.dim + (2 if cfg.has_s else 0)
    return cfg.cells * per * es + cfg.ncol * 8


def _tiles(t, cfg, small):
    """View of a (lead..., nz, ny, nx) tensor of the large run as lateral
    copies of the small run: (lead..., vertical, ry, sy, rx, sx)."""
    lead = t.shape[:-3]
    if cfg.dim == 3:
        return t.view(*lead, cfg.nz, cfg.ny // small.ny, small.ny, cfg.nx // small.nx, small.nx)
    return t.view(*lead, cfg.ny, 1, 1, cfg.nx // small.nx, small.nx)


def _tile(s, small):
    """The small run's (lead..., nz, ny, nx) tensor shaped to broadcast
    against _tiles: (lead..., vertical, 1, sy, 1, sx)."""
    lead = s.shape[:-3]
    if small.dim == 3:
        return s.view(*lead, small.nz, 1, small.ny, 1, small.nx)
    return s.view(*lead, small.ny, 1, 1, 1, small.nx)


def _mismatches(big, small):
    """Elements of big (the copies) that differ from small (broadcast), in
    chunks of about 2^26 elements along the vertical axis (the one after the
    leading axes)."""
    lead = big.dim() - 5
    nv = big.shape[lead]
    chunk = max(1, (1 << 26) // (big[(0,) * (lead + 1)].numel()))
    n = torch.zeros((), dtype=torch.int64, device=big.device)
    for v0 in range(0, nv, chunk):
        sl = (slice(None),) * lead + (slice(v0, v0 + chunk),)
        n += torch.ne(big[sl], small[sl]).sum()
    return int(n.item())


@pytest.mark.parametrize("name", list(CASES))
def test_run_beyond_2_31_cells_equals_its_periodic_tile(name):
    wl, lat_big, lat_small, nv = CASES[name]
    small = _cfg(wl, lat_small, nv)
    big = _cfg(wl, lat_big, nv)
    assert big.cells > 2 ** 31 and big.cells <= 2 ** 32 - 1024
    launch = autotune.lookup(wl.name) or {}
    copies = big.cells // small.cells

    need = _bytes(big)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    print(f"\n[{name}] {big.cells} cells, {need / 1e9:.1f} GB needed, {free / 1e9:.1f} of "
          f"{total / 1e9:.1f} GB free", flush=True)
    if free < need + (6 << 30):
        pytest.skip(f"needs {need / 1e9:.0f} GB of free device memory ({free / 1e9:.0f} GB free)")

    # the small run on the GPU, and against the oracle
    swl = wl.replace(name=f"{name}_tile", nx=small.nx, ny=small.ny, nz=small.nz)
    c0, s0 = W.initial_scalars(swl)
    c0, s0 = as_input(c0, small), as_input(s0, small)
    u0 = as_input(_velocity(small), small)
    print(f"[{name}] small run {small.nx}x{small.ny}x{small.nz}, {STEPS} steps", flush=True)
    ss = lbw.Solver(small)
    ss.set_launch(**launch)
    ss.set_field("c", c0)
    if s0 is not None:
        ss.set_field("s", s0)
    u0_dev = torch.from_numpy(u0).float().cuda()
    ss.init_equilibrium(u=u0_dev)
    ss.step(STEPS)
    torch.cuda.synchronize()
    st = ss.tensors[0]
    ref = {"c": st["c"].clone(), "u": st["u"].clone(), "f": st["f"].clone(),
           "deposit": st["deposit"].clone()}
    if small.has_s:
        ref["s"] = ss.field("s").clone()
    sums = {w: ss.reduce(w)[0] for w in (lbw.MASS_C, lbw.MASS_FLUID, lbw.DEPOSIT)}
    # the sums of |terms| bound the FP64 sums' rounding (a fluid node adds ~1)
    scale = {lbw.MASS_C: float(ref["c"].double().abs().sum()), lbw.MASS_FLUID: float(small.cells),
             lbw.DEPOSIT: float(ref["deposit"].abs().sum())}
    front = ss.front_height(0.5 * wl.c0).clone()
    g = {k: ss.field(k).double().cpu().numpy() for k in ("c", "u", "f", "deposit")}
    if small.has_s:
        g["s"] = ref["s"].double().cpu().numpy()
    ss.close()
    del ss, st

    print(f"[{name}] oracle {STEPS} steps", flush=True)
    f0 = oracle.equilibrium(oracle_cfg(small), None, u0)
    o = run_oracle(small, c0, s0, f0=f0, nsteps=STEPS)
    dep = o.pop("deposit")
    errs = compare(g, o)
    errs["deposit"] = float(np.max(np.abs(g["deposit"] - dep))) / float(np.max(np.abs(dep)))
    print(f"[{name}] small run against the oracle: {errs}", flush=True)
    for k, v in errs.items():
        assert v <= (TOL_DEPOSIT if k == "deposit" else TOL[k]), (k, v, errs)
    del g, o, f0

    # the large run: the small run's state tiled laterally
    print(f"[{name}] large run {big.nx}x{big.ny}x{big.nz}, {STEPS} steps", flush=True)
    sb = lbw.Solver(big)
    sb.set_launch(**launch)
    tb = sb.tensors[0]
    with torch.cuda.stream(sb.stream):
        _tiles(tb["c"], big, small).copy_(_tile(torch.from_numpy(c0).float().cuda(), small))
        if small.has_s:
            _tiles(tb["s"], big, small).copy_(_tile(torch.from_numpy(s0).float().cuda(), small))
        _tiles(tb["u"], big, small).copy_(_tile(u0_dev, small))
    sb.stream.synchronize()
    sb.init_equilibrium(u=tb["u"])     # reads the velocity, writes only f
    sb.step(STEPS)
    torch.cuda.synchronize()

    bad = {}
    cur_s = None
    if small.has_s:
        # S lives in the buffer the S update last wrote
        cur_s = tb["s"] if STEPS % 2 == 0 else tb["s_tmp"]
    pairs = {"c": (tb["c"], ref["c"]), "u": (tb["u"], ref["u"]), "f": (tb["f"], ref["f"])}
    if cur_s is not None:
        pairs["s"] = (cur_s, ref["s"])
    for k, (tbig, tsmall) in pairs.items():
        bad[k] = _mismatches(_tiles(tbig, big, small), _tile(tsmall, small))
    dep_big = tb["deposit"].view(-1, small.ncol) if big.dim == 2 else \
        tb["deposit"].view(big.ny // small.ny, small.ny, big.nx // small.nx, small.nx)
    dep_small = ref["deposit"].view(1, small.ncol) if big.dim == 2 else \
        ref["deposit"].view(1, small.ny, 1, small.nx)
    bad["deposit"] = int(torch.ne(dep_big, dep_small).sum().item())
    fb = sb.front_height(0.5 * wl.c0)
    front_big = fb.view(-1, small.nx) if big.dim == 2 else \
        fb.view(big.ny // small.ny, small.ny, big.nx // small.nx, small.nx)
    front_small = front.view(1, small.nx) if big.dim == 2 else front.view(1, small.ny, 1, small.nx)
    bad["front"] = int(torch.ne(front_big, front_small).sum().item())
    sums_big = {w: sb.reduce(w)[0] for w in sums}
    print(f"[{name}] elements differing from the tiled small run: {bad}", flush=True)
    sb.close()
    del sb, tb, pairs, cur_s
    torch.cuda.empty_cache()

    assert all(v == 0 for v in bad.values()), bad
    print(f"[{name}] sums: large {sums_big}, copies x small "
          f"{ {w: copies * v for w, v in sums.items()} }", flush=True)
    for w, v in sums.items():
        assert abs(sums_big[w] - copies * v) <= 1e-12 * copies * scale[w], (w, sums_big[w], copies * v)
