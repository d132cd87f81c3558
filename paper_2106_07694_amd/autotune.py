"""Launch-shape autotuner for liblbw.

For a workload (one run or a batch) it times candidate launch shapes with the
library's own per-phase HIP-event timing and keeps, independently, the
collide-stream block size with the least collide-stream time and the
transport tile (width, vertical chunk) with the least transport time.  The
winners are cached in ``tuned.json`` beside this file, keyed by workload
name, with the device architecture, grid and precision they were taken on.

    python -m paper_2106_07694_amd.autotune [3d|2d|adjoint|sweep|all]
"""
from __future__ import annotations

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuned.json")

LBM_BLOCKS = (128, 256, 512, 1024)
# transport tiles (columns, rows): 256 threads, and 512-thread tiles
TILES = {2: ((64, 1), (128, 1), (256, 1), (512, 1)),
         3: ((32, 8), (64, 4), (128, 2), (32, 16), (64, 8))}
CHUNKS = {2: (2, 3, 4, 6, 8, 16, 32, 64), 3: (8, 16, 32, 64, 128)}


def _time_phases(sol, steps: int) -> dict:
    import torch
    sol.step(2)
    torch.cuda.synchronize()
    sol.timing_begin()
    sol.step(steps)
    return sol.timing_end()


def tune(cfgs, setup, steps: int = 20, graph: bool = False, log=print) -> dict:
    """Best launch for the runs `cfgs`; `setup(sol)` writes initial state."""
    import torch
    from . import lbw

    stream = torch.cuda.Stream() if graph else None
    sol = lbw.Solver(cfgs, stream=stream)
    setup(sol)
    dim = cfgs[0].dim if isinstance(cfgs, list) else cfgs.dim
    best_lbm, best_lbm_ms = 256, float("inf")
    for blk in LBM_BLOCKS:
        sol.set_launch(lbm_block=blk)
        ms = _time_phases(sol, steps)["collide_stream_ms"] / steps
        log(f"  lbm_block={blk}: {ms * 1e3:.1f} us/step")
        if ms < best_lbm_ms:
            best_lbm, best_lbm_ms = blk, ms
    best_tile, best_tr_ms = None, float("inf")
    for tx, rows in TILES[dim]:
        for ch in CHUNKS[dim]:
            sol.set_launch(lbm_block=best_lbm, tile_x=tx, tile_y=ch, tile_rows=rows)
            ms = _time_phases(sol, steps)["transport_ms"] / steps
            log(f"  tile {tx}x{rows} chunk={ch}: {ms * 1e3:.1f} us/step")
            if ms < best_tr_ms:
                best_tile, best_tr_ms = (tx, rows, ch), ms
    sol.close()
    out = {"lbm_block": best_lbm, "tile_x": best_tile[0], "tile_rows": best_tile[1],
           "tile_y": best_tile[2]}
    if graph:
        out["graph"] = 1
    out["_ms"] = {"collide_stream": best_lbm_ms, "transport": best_tr_ms}
    return out


def load_cache() -> dict:
    try:
        with open(CACHE) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def lookup(name: str):
    """Launch dict for a workload (tuning metadata removed) or None."""
    e = load_cache().get(name)
    if not e:
        return None
    return {k: v for k, v in e.items() if not k.startswith("_")}


def _arch() -> str:
    import torch
    try:
        return torch.cuda.get_device_properties(0).gcnArchName
    except Exception:
        return "unknown"


def main(which: str = "all") -> int:
    from . import lbw, workloads as W

    cache = load_cache()
    jobs = []
    if which in ("3d", "all"):
        jobs.append((W.C3.name, [lbw.RunConfig.from_workload(W.C3)], [W.C3], False))
    if which in ("2d", "all"):
        jobs.append((W.C2.name, [lbw.RunConfig.from_workload(W.C2)], [W.C2], False))
    if which in ("adjoint", "all"):
        jobs.append((W.C5.name, [lbw.RunConfig.from_workload(W.C5)], [W.C5], False))
    if which in ("sweep", "all"):
        runs = W.sweep_runs()
        jobs.append(("sweep_64", [lbw.RunConfig.from_workload(w) for w in runs], runs, True))
    for name, cfgs, wls, graph in jobs:
        print(f"[autotune] {name}", flush=True)

        def setup(sol, wls=wls):
            for i, w in enumerate(wls):
                sol.setup_workload(w, run=i)

        best = tune(cfgs, setup, graph=graph, log=lambda m: print(m, flush=True))
        best["_arch"] = _arch()
        best["_grids"] = sorted({(c.nx, c.ny, c.nz) for c in cfgs})
        best["_precision"] = cfgs[0].precision
        cache[name] = best
        print(f"[autotune] {name}: {best}", flush=True)
    with open(CACHE, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1] if len(sys.argv) > 1 else "all"))
