"""The early-time growth rate on the GPU path (FP64 and the FP32 shifted
production form) against linear stability analysis: the same run as the
oracle's growth-rate test (tests/test_oracle_lsa.py), stepped through the C
ABI, with the LSA eigenvalue of the run's own mean profile.

In 3D (D3Q19) the interface is displaced by an oblique mode cos(kx x + ky y)
whose wavenumber |k| = (kx^2 + ky^2)^1/2 enters the same two-dimensional
eigenproblem (the linearised equations are isotropic in the horizontal); at
that |k| the rate moves by 5% for a 10% error in the viscosity and by 2.5%
for a 5% error in |k|, so the run checks both lateral axes of the lattice and
of the transport.  It is too long for the oracle (1.3e9 cell updates), so
the LSA solver, pinned to a closed form, is the reference."""
import numpy as np
import pytest

from paper_2106_07694_amd import lbw
from lsa import fitted_rate, layer_setup, lsa_rate_for_profile, mode_amplitude

pytestmark = pytest.mark.gpu
TAU, GP, KAPPA, WIDTH, ETA = 0.6, 5e-5, 1e-4, 3.0, 0.02


@pytest.mark.parametrize("precision", ["fp64", "fp32_shifted"])
def test_gpu_growth_rate_matches_lsa(precision):
    nx, ny, nsteps, chunk, vs = 64, 160, 4000, 100, 5e-4
    cfg = lbw.RunConfig(lattice=9, nx=nx, ny=ny, precision=precision, tau=TAU, gp_c=GP,
                        kappa_c=KAPPA, vs=vs)
    c, rho, k = layer_setup(nx, ny, GP, WIDTH, ETA)
    sol = lbw.Solver(cfg)
    sol.set_field("c", c)
    sol.init_equilibrium(rho=rho)
    ts, amps, psd, profs = [], [], [], {}
    for it in range(nsteps // chunk):
        sol.step(chunk)
        t = (it + 1) * chunk
        u = sol.field("u").double().cpu().numpy()
        ts.append(t)
        amps.append(mode_amplitude(u[1, 0]))
        # in-situ: front height and its spectrum stay on the device
        psd.append(float(sol.front_psd(sol.front_height(0.5))[1]))
        profs[t] = sol.field("c").double().cpu().numpy()[0].mean(axis=1)
    sol.close()
    ts, amps = np.array(ts), np.array(amps)
    win = (ts >= 2500) & (ts <= 3500)
    sim = fitted_rate(ts[win], amps[win])
    pred = lsa_rate_for_profile(profs[3000], k, (TAU - 0.5) / 3, KAPPA, GP, vs)
    print(f"\n{precision}: growth rate {sim:.5e}, LSA {pred:.5e}, ratio {sim / pred:.4f}")
    assert amps[win][-1] > 2 * amps[win][0]
    assert abs(sim / pred - 1) < 0.01, (sim, pred)
    sim_h = 0.5 * fitted_rate(ts[win], np.array(psd)[win])     # Gamma_H ~ exp(2 sigma t)
    print(f"front-height PSD rate {sim_h:.5e}, ratio {sim_h / pred:.4f}")
    assert abs(sim_h / pred - 1) < 0.03, (sim_h, pred)


def _layer_3d(nx, ny, nz, gp, width, eta):
    """The 3D counterpart of lsa.layer_setup: C = (1 + tanh((z - z0 - eta
    cos(kx x + ky y)) / width)) / 2 with one wavelength across each lateral
    axis, and the hydrostatic density of the mean profile.  Returns (c, rho,
    |k|) with c and rho of shape (nz, ny, nx)."""
    kx, ky = 2 * np.pi / nx, 2 * np.pi / ny
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    y = np.arange(ny, dtype=np.float64)[None, :, None]
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    z0 = (nz - 1) / 2
    c = 0.5 * (1 + np.tanh((z - z0 - eta * np.cos(kx * x + ky * y)) / width))
    cm = c.mean(axis=(1, 2))
    rho_z = 1 - 3 * gp * np.concatenate([[0.0], np.cumsum(0.5 * (cm[1:] + cm[:-1]))])
    rho_z += 1 - rho_z.mean()
    rho = np.broadcast_to(rho_z[:, None, None], c.shape).copy()
    return c, rho, float(np.hypot(kx, ky))


def _oblique_amplitude(uz):
    """L2 norm over planes of the (1, 1) lateral Fourier mode of uz[nz, ny, nx]."""
    m = np.fft.fft2(uz, axes=(1, 2))[:, 1, 1]
    return float(np.sqrt(np.sum(np.abs(m) ** 2)))


@pytest.mark.parametrize("precision", ["fp64", "fp32_shifted"])
def test_gpu_growth_rate_3d_oblique_mode_matches_lsa(precision):
    nx, ny, nz, nsteps, chunk, vs = 64, 32, 160, 4000, 100, 5e-4
    cfg = lbw.RunConfig(lattice=19, nx=nx, ny=ny, nz=nz, precision=precision, tau=TAU, gp_c=GP,
                        kappa_c=KAPPA, vs=vs)
    c, rho, k = _layer_3d(nx, ny, nz, GP, WIDTH, ETA)
    sol = lbw.Solver(cfg)
    sol.set_field("c", c)
    sol.init_equilibrium(rho=rho)
    ts, amps, psd_x, psd_y, profs = [], [], [], [], {}
    for it in range(nsteps // chunk):
        sol.step(chunk)
        t = (it + 1) * chunk
        u = sol.field("u").double().cpu().numpy()
        ts.append(t)
        amps.append(_oblique_amplitude(u[2]))
        h = sol.front_height(0.5)
        psd_x.append(float(sol.front_psd(h, axis=0, index=-1)[1]))
        psd_y.append(float(sol.front_psd(h, axis=1, index=-1)[1]))
        profs[t] = sol.field("c").double().cpu().numpy().mean(axis=(1, 2))
    sol.close()
    ts, amps = np.array(ts), np.array(amps)
    win = (ts >= 2500) & (ts <= 3500)
    sim = fitted_rate(ts[win], amps[win])
    pred = lsa_rate_for_profile(profs[3000], k, (TAU - 0.5) / 3, KAPPA, GP, vs)
    print(f"\n3D {precision}: |k| {k:.4f}, growth rate {sim:.5e}, LSA {pred:.5e}, "
          f"ratio {sim / pred:.4f}")
    assert amps[win][-1] > 2 * amps[win][0]
    assert abs(sim / pred - 1) < 0.01, (sim, pred)
    for name, psd in (("x", psd_x), ("y", psd_y)):
        sim_h = 0.5 * fitted_rate(ts[win], np.array(psd)[win])
        print(f"front-height PSD rate along {name} {sim_h:.5e}, ratio {sim_h / pred:.4f}")
        assert abs(sim_h / pred - 1) < 0.03, (name, sim_h, pred)
