"""Early-time growth of the settling-driven (Rayleigh-Taylor-like) instability
against linear stability analysis (the paper's validation of its model: the
simulated early-time growth rate of the instability agrees with the LSA
prediction).

A particle-laden layer (buoyancy -g' C) lies over clear fluid with a diffuse
interface displaced by one small cosine across the periodic width; the FP64
oracle steps it from hydrostatic rest.  After the initial transient, the
horizontal Fourier mode of the vertical velocity grows as exp(sigma t); its
fitted rate must equal the LSA eigenvalue (tests/lsa.py) computed on the
run's own mean profile at the middle of the fit window.  The LSA solver is
itself pinned to a closed form (inviscid ramp profile).
"""
import numpy as np
import pytest

import oracle
from lsa import (fitted_rate, growth_rate, layer_setup, lsa_rate_for_profile, mode_amplitude,
                 ramp_growth_rate)

TAU, GP, KAPPA, WIDTH, ETA = 0.6, 5e-5, 1e-4, 3.0, 0.02


@pytest.mark.parametrize("h", [0.5, 0.25])
def test_lsa_solver_matches_ramp_closed_form(h):
    """Inviscid, non-diffusive linear ramp: sigma from m tan(m d/2) = k."""
    k, d, gp = 2 * np.pi / 64, 8.0, 5e-5
    z = np.arange(-60 + h, 60, h)
    dc = np.where(np.abs(z) < d / 2, 1 / d, 0.0)
    dc[np.isclose(np.abs(z), d / 2)] = 0.5 / d
    s = growth_rate(k, z, dc, 0.0, 0.0, gp)
    exact = ramp_growth_rate(k, d, gp)
    assert abs(s.imag) < 1e-12 and abs(s.real / exact - 1) < 5e-4, (s, exact)
    # and the sharp-interface limit sigma^2 = k g' / 2 is approached from below
    assert exact < np.sqrt(k * gp / 2) and ramp_growth_rate(k, 0.5, gp) > 0.99 * np.sqrt(k * gp / 2)


def test_lsa_solver_viscosity_and_diffusion_damp():
    k, gp = 2 * np.pi / 64, 5e-5
    z = np.arange(-60 + 0.5, 60, 0.5)
    dc = 0.5 / WIDTH / np.cosh(z / WIDTH) ** 2
    s0 = growth_rate(k, z, dc, 0.0, 0.0, gp).real
    s1 = growth_rate(k, z, dc, 1 / 30, 0.0, gp).real
    s2 = growth_rate(k, z, dc, 1 / 30, 1e-3, gp).real
    assert s0 > s1 > s2 > 0


@pytest.mark.parametrize("vs", [0.0, 5e-4])
def test_oracle_growth_rate_matches_lsa(vs):
    nx, ny, nsteps, chunk = 64, 160, 4000, 100
    cfg = oracle.OracleConfig(q=9, nx=nx, ny=ny, tau=TAU, gp_c=GP, kappa_c=KAPPA, vs=vs)
    c, rho, k = layer_setup(nx, ny, GP, WIDTH, ETA)
    f = oracle.equilibrium(cfg, rho, None)
    dep = None
    ts, amps, psd, profs = [], [], [], {}
    for it in range(nsteps // chunk):
        f, c, _, dep, u = oracle.run(cfg, f, c, None, dep, None, chunk, want_u=True)
        t = (it + 1) * chunk
        ts.append(t)
        amps.append(mode_amplitude(u[1, 0]))
        # the paper's own measure: the PSD of the front height at C0 / 2
        psd.append(oracle.front_psd(cfg, oracle.front_height(cfg, c, 0.5))[1])
        profs[t] = c[0].mean(axis=1)
    ts, amps = np.array(ts), np.array(amps)
    win = (ts >= 2500) & (ts <= 3500)
    sim = fitted_rate(ts[win], amps[win])
    pred = lsa_rate_for_profile(profs[3000], k, (TAU - 0.5) / 3, KAPPA, GP, vs)
    print(f"\nvs={vs}: growth rate oracle {sim:.5e}, LSA {pred:.5e}, ratio {sim / pred:.4f}")
    assert amps[win][-1] > 2 * amps[win][0]          # the mode grows through the window
    assert abs(sim / pred - 1) < 0.01, (sim, pred)
    # Gamma_H(k, t) = Gamma_Hi exp(2 sigma t): half the slope of log Gamma.
    # The front is interpolated between cells, and settling moves it through
    # them, which adds a jitter of about 1% to this fit.
    sim_h = 0.5 * fitted_rate(ts[win], np.array(psd)[win])
    print(f"front-height PSD rate {sim_h:.5e}, ratio {sim_h / pred:.4f}")
    assert abs(sim_h / pred - 1) < 0.03, (sim_h, pred)
