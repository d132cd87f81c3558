"""The library driven through its C ABI alone: a plain C program
(tests/c_abi/abi_run.c, built with the library) allocates device memory with
the HIP runtime, runs 100 coupled steps of a D2Q9 FP64 run and closes the
particle and fluid budgets; the same run through the Python binding gives
the same sums bit for bit."""
import json
import os
import subprocess

import numpy as np
import pytest

from paper_2106_07694_amd import lbw

pytestmark = pytest.mark.gpu
EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "abi_run")


def test_c_program_matches_the_binding():
    import torch

    assert os.path.exists(EXE), "tests/c_abi/abi_run is built by build()"
    out = subprocess.run([EXE, "100"], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, (out.returncode, out.stdout, out.stderr)
    got = json.loads(out.stdout.strip().splitlines()[-1])
    assert got["budget_closed"] is True

    nx, ny = 64, 128
    cfg = lbw.RunConfig(nx=nx, ny=ny, tau=0.6, vs=1e-3, kappa_c=1e-3, gp_c=1e-5)
    y = np.arange(ny)[:, None]
    x = np.arange(nx)[None, :]
    c = np.where(y >= ny // 2, 1.0, 0.0) + 1e-3 * ((7 * x + 13 * y) % 17).astype(np.float64) / 17.0
    sol = lbw.Solver(cfg)
    sol.set_field("c", c[None])
    sol.init_equilibrium()
    m0, r0 = sol.reduce(lbw.MASS_C)[0], sol.reduce(lbw.MASS_FLUID)[0]
    sol.step(100)
    torch.cuda.synchronize()
    m, d, r = sol.reduce(lbw.MASS_C)[0], sol.reduce(lbw.DEPOSIT)[0], sol.reduce(lbw.MASS_FLUID)[0]
    sol.close()
    assert (got["mass0"], got["mass"], got["deposit"], got["fluid0"], got["fluid"]) == (m0, m, d, r0, r)
