"""Seeded synthetic workloads: parameters and initial scalar fields.

This module is the one piece both the product path and the test oracle use.
It holds parameters and random numbers only -- none of the method's
arithmetic (no lattice tables, no equilibria, no fluxes).  Each side builds
its own populations from these fields.

Initial state (section 2.2, eq. 16-17): a particle-laden upper layer over a
particle-free lower layer, the interface smoothed to a tanh of width two cells
and perturbed by seeded uniform noise to start the instability; a second
scalar S (sugar) in the lower layer when present; fluid at rest.  The vertical
axis is y in 2D and z in 3D.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    """One run's physics and grid, in lattice units."""
    name: str
    q: int                   # 9 (D2Q9) or 19 (D3Q19)
    nx: int
    ny: int
    nz: int
    precision: str           # "fp64" or "fp32_shifted"
    tau: float
    vs: float                # settling speed
    kappa_c: float           # particle diffusivity
    gp_c: float              # vertical force per unit C is -gp_c
    c0: float = 1.0          # upper-layer concentration
    amp: float = 1e-3        # perturbation amplitude
    width: float = 2.0       # tanh interface width (cells)
    has_s: bool = False
    kappa_s: float = 0.0
    gp_s: float = 0.0        # vertical force per unit S is -gp_s (S heavier: gp_s > 0)
    steps: int = 1000
    seed: int = 1000
    # particle size classes (eq. 11-12): with n_classes >= 2 the upper layer
    # holds c0 / n_classes of each class, class i settling at vs_class[i]
    n_classes: int = 1
    vs_class: tuple = ()
    kappa_class: tuple = ()
    # full force and settling (eq. 10, 13): Vs (1 - vs_s S), S buoyancy on
    # the fluid fraction 1 - phi_c C
    vs_s: float = 0.0
    phi_c: float = 0.0

    @property
    def dim(self) -> int:
        return 2 if self.q == 9 else 3

    @property
    def shape(self) -> tuple:
        return (self.nz, self.ny, self.nx)

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def ncol(self) -> int:
        return self.nx if self.dim == 2 else self.nx * self.ny

    @property
    def nvert(self) -> int:
        return self.ny if self.dim == 2 else self.nz

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


# The five configurations (2D FP64 small case; 2D FP32 + S; 3D FP32; batched
# sweep; adjoint).  The batched sweep's runs are drawn by ``sweep_runs``.
C1 = Workload("2d_fp64_64x128", q=9, nx=64, ny=128, nz=1, precision="fp64", tau=0.6,
              vs=1e-3, kappa_c=1e-3, gp_c=1e-5, steps=1000, seed=1000)
C2 = Workload("2d_fp32_shifted_s_1024x2048", q=9, nx=1024, ny=2048, nz=1,
              precision="fp32_shifted", tau=0.6, vs=5e-4, kappa_c=1e-3, gp_c=1e-5,
              c0=1.0, has_s=True, kappa_s=1e-4, gp_s=2e-5, steps=20000, seed=1001)
C3 = Workload("3d_d3q19_fp32_256x256x512", q=19, nx=256, ny=256, nz=512,
              precision="fp32_shifted", tau=0.55, vs=5e-4, kappa_c=5e-4, gp_c=1e-5,
              steps=2000, seed=1002)
C5 = Workload("2d_fp32_adjoint_512x1024", q=9, nx=512, ny=1024, nz=1,
              precision="fp32_shifted", tau=0.6, vs=1e-3, kappa_c=1e-3, gp_c=1e-5,
              steps=5000, seed=1004)
# The 3D workload with four particle size classes sharing the same total
# (settling speeds spread around the single-class one).
C6 = Workload("3d_d3q19_fp32_256x256x512_4classes", q=19, nx=256, ny=256, nz=512,
              precision="fp32_shifted", tau=0.55, vs=0.0, kappa_c=0.0, gp_c=1e-5,
              steps=2000, seed=1005, n_classes=4, vs_class=(2.5e-4, 5e-4, 7.5e-4, 1e-3),
              kappa_class=(5e-4, 5e-4, 5e-4, 5e-4))
# The 2D two-scalar workload with the full force and settling: particles
# settle at half speed in the sugar layer (S = 1) and phi = 1e-3 C.
C7 = C2.replace(name="2d_fp32_shifted_s_1024x2048_full_force", vs_s=0.5, phi_c=1e-3, seed=1006)
SWEEP_GRIDS = ((128, 256), (256, 512), (512, 1024))
SWEEP_RUNS = 64
SWEEP_STEPS = 5000


def sweep_runs(n: int = SWEEP_RUNS, seed: int = 1003, grids=SWEEP_GRIDS,
               steps: int = SWEEP_STEPS) -> list:
    """Batched parameter sweep: uneven 2D grids, C0 ~ U[0.25, 4],
    Vs ~ log-uniform on [1e-4, 2e-3], kappa = 1e-3, g' = 1e-5."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(n):
        nx, ny = grids[int(rng.integers(len(grids)))]
        c0 = float(rng.uniform(0.25, 4.0))
        vs = float(math.exp(rng.uniform(math.log(1e-4), math.log(2e-3))))
        out.append(Workload(f"sweep_{r:02d}_{nx}x{ny}", q=9, nx=nx, ny=ny, nz=1,
                            precision="fp32_shifted", tau=0.6, vs=vs, kappa_c=1e-3,
                            gp_c=1e-5, c0=c0, steps=steps, seed=seed * 1000 + r))
    return out


def _vertical_coordinate(wl: Workload) -> np.ndarray:
    """Vertical index broadcast to the (nz, ny, nx) field shape."""
    if wl.dim == 2:
        return np.arange(wl.ny, dtype=np.float64)[None, :, None]
    return np.arange(wl.nz, dtype=np.float64)[:, None, None]


def initial_scalars(wl: Workload, seed: int | None = None):
    """(C, S) as float64 arrays of shape (nz, ny, nx); S is None without S.

    C = C0 * (1 + tanh((v - v_i)/width))/2 + amp * U(-1, 1), v_i = (n_v - 1)/2,
    S = (1 - tanh((v - v_i)/width))/2.  With n_classes >= 2, C has shape
    (n_classes, nz, ny, nx): each class holds C0 / n_classes of the profile
    plus its own noise of amplitude amp / n_classes.
    """
    rng = np.random.default_rng(wl.seed if seed is None else seed)
    v = _vertical_coordinate(wl)
    vi = 0.5 * (wl.nvert - 1)
    profile = 0.5 * (1.0 + np.tanh((v - vi) / wl.width))
    n = max(1, wl.n_classes)
    shape = wl.shape if n == 1 else (n,) + wl.shape
    c = (wl.c0 / n) * np.broadcast_to(profile, shape).copy()
    c += (wl.amp / n) * rng.uniform(-1.0, 1.0, size=shape)
    s = None
    if wl.has_s:
        s = np.broadcast_to(1.0 - profile, wl.shape).copy()
    return np.ascontiguousarray(c), (None if s is None else np.ascontiguousarray(s))


def random_directions(n: int, shape: tuple, seed: int) -> np.ndarray:
    """n seeded standard-normal directions of the given field shape."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n,) + tuple(shape))
