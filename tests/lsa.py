"""Linear stability of a diffuse particle-laden layer (test infrastructure).

The paper's linear stability analysis (section "Linear stability analysis":
vorticity-stream function form, a base state at rest with a horizontally
uniform concentration profile, normal modes exp(i k y + sigma t), and the
generalised eigenproblem K x = sigma W x in a frame falling with the
particles) restated for the model the oracle integrates: Boussinesq
buoyancy -g' C on the vertical axis, kinematic viscosity nu, particle
diffusivity kappa, settling speed Vs, no second scalar, lattice units.

With u = (dpsi/dz, -dpsi/dy), omega = -lap(psi), M = D^2 - k^2 and the frame
moving down at Vs (where the base concentration only diffuses):

    sigma M psi = nu M^2 psi - Vs D M psi + i k g' C
    sigma C     = kappa M C + i k (dCbar/dz) psi

(the first row is the vorticity equation with omega eliminated).  Spatial
derivatives are second-order finite differences on a uniform grid; no-slip
walls (psi = dpsi/dz = 0) and C = 0 at the ends of the grid.  For a sharp
interface between C = 0 below and C = 1 above, with nu = kappa = 0, the
growth rate is sigma^2 = k g' / 2 (Rayleigh-Taylor, Boussinesq); the tests
pin the solver to that limit.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def _operators(n: int, h: float, k: float):
    """D, M = D^2 - k^2 and M^2 for psi (clamped ends) and M for C (zero ends)
    on n interior points of spacing h."""
    e = np.ones(n)
    d1 = (np.diag(e[:-1], 1) - np.diag(e[:-1], -1)) / (2 * h)
    d2 = (np.diag(e[:-1], 1) - 2 * np.diag(e) + np.diag(e[:-1], -1)) / h**2
    # fourth derivative with psi = 0 on the boundary nodes and psi' = 0 via
    # mirrored ghosts (psi_{-1} = psi_1)
    d4 = (np.diag(e[:-2], 2) - 4 * np.diag(e[:-1], 1) + 6 * np.diag(e)
          - 4 * np.diag(e[:-1], -1) + np.diag(e[:-2], -2))
    d4[0, 0] += 1.0
    d4[-1, -1] += 1.0
    d4 /= h**4
    ident = np.eye(n)
    m = d2 - k * k * ident
    m2 = d4 - 2 * k * k * d2 + k**4 * ident
    return d1, m, m2


def growth_rate(k: float, z: np.ndarray, dcbar: np.ndarray, nu: float, kappa: float,
                gp: float, vs: float = 0.0) -> complex:
    """Eigenvalue of largest real part for wavenumber k; z is the uniform
    interior grid and dcbar = dCbar/dz on it.  With C = i Ct the system is
    real:  sigma M psi = (nu M^2 - Vs D M) psi - k g' Ct,
           sigma Ct    = k dCbar psi + kappa M Ct,
    solved as a standard eigenproblem after applying M^-1 to the first row."""
    n = len(z)
    h = float(z[1] - z[0])
    d1, m, m2 = _operators(n, h, k)
    minv = np.linalg.inv(m)
    a = np.block([[minv @ (nu * m2 - vs * d1 @ m), -k * gp * minv],
                  [k * np.diag(dcbar), kappa * m]])
    w = scipy.linalg.eigvals(a)
    return complex(w[np.argmax(w.real)])


def ramp_growth_rate(k: float, d: float, gp: float, dc: float = 1.0) -> float:
    """Inviscid, non-diffusive growth rate for a linear concentration ramp of
    thickness d (dc across it) between uniform layers, in unbounded fluid.
    Inside the ramp psi'' = -m^2 psi with m^2 = k^2 (g' dc / (d sigma^2) - 1);
    outside psi ~ exp(-k |z|); the even mode matches when m tan(m d / 2) = k."""
    import scipy.optimize
    f = lambda mm: mm * np.tan(mm * d / 2) - k
    m = scipy.optimize.brentq(f, 1e-12, (np.pi - 1e-9) / d)
    return float(np.sqrt(k * k * gp * dc / (d * (m * m + k * k))))


def tanh_profile_slope(z: np.ndarray, z0: float, width: float) -> np.ndarray:
    """dCbar/dz of Cbar = (1 + tanh((z - z0) / width)) / 2."""
    return 0.5 / width / np.cosh((z - z0) / width) ** 2


def layer_setup(nx: int, ny: int, gp: float, width: float, eta: float):
    """Initial state of the growth-rate runs: C = (1 + tanh((y - y0 - eta
    cos(k x)) / width)) / 2 (particle-laden fluid above clear fluid, one
    wavelength of interface displacement across the periodic width) and the
    hydrostatic density of the mean profile (d rho / dy = -3 g' C, c_s^2 =
    1/3, mean 1), so the run starts without a box-wide acoustic transient.
    Returns (c[1, ny, nx], rho[1, ny, nx], k)."""
    k = 2 * np.pi / nx
    y = np.arange(ny, dtype=np.float64)[:, None]
    x = np.arange(nx, dtype=np.float64)[None, :]
    y0 = (ny - 1) / 2
    c = 0.5 * (1 + np.tanh((y - y0 - eta * np.cos(k * x)) / width))
    cm = c.mean(axis=1)
    rho_y = 1 - 3 * gp * np.concatenate([[0.0], np.cumsum(0.5 * (cm[1:] + cm[:-1]))])
    rho_y += 1 - rho_y.mean()
    rho = np.broadcast_to(rho_y[:, None], (ny, nx)).copy()
    return c[None].copy(), rho[None].copy(), k


def mode_amplitude(uy: np.ndarray) -> float:
    """L2 norm over rows of the first horizontal Fourier mode of the
    vertical velocity uy[ny, nx]."""
    m = np.fft.rfft(uy, axis=1)[:, 1]
    return float(np.sqrt(np.sum(np.abs(m) ** 2)))


def fitted_rate(ts, amps) -> float:
    """Least-squares slope of log(amplitude) against time."""
    return float(np.polyfit(np.asarray(ts, float), np.log(np.asarray(amps, float)), 1)[0])


def lsa_rate_for_profile(profile: np.ndarray, k: float, nu: float, kappa: float, gp: float,
                         vs: float, h: float = 0.5) -> float:
    """Growth rate of the base state given by a mean profile on the lattice
    rows (walls at -1/2 and ny - 1/2), interpolated onto a grid of spacing h."""
    ny = len(profile)
    zc = np.arange(ny, dtype=np.float64)
    dcb = np.gradient(profile, zc)
    z = np.arange(-0.5 + h, ny - 0.5 - h / 2, h)     # interior points between the walls
    return growth_rate(k, z, np.interp(z, zc, dcb), nu, kappa, gp, vs).real
