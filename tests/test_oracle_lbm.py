"""Pins of the oracle's lattice-Boltzmann part against what the method fixes.

Lattice moments (isotropy), rest state, exact mass conservation, the Guo
momentum identity (eq. 22), Poiseuille and Couette closed forms for BGK with
half-way bounce-back (section 2.3.1), and the shifted-population identity.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import OracleConfig


@pytest.mark.parametrize("q", [9, 19])
def test_lattice_isotropy(q):
    c, w, opp = oracle.lattice(q)
    dim = 2 if q == 9 else 3
    cs2 = 1.0 / 3.0
    assert abs(w.sum() - 1.0) < 1e-15
    # the velocity set is exactly {c in {-1,0,1}^dim : |c|^2 <= 2} (D3Q19)
    # or the full 3x3 neighbourhood (D2Q9), each once
    want = {v for v in itertools.product((-1, 0, 1), repeat=dim)
            if q == 9 or sum(x * x for x in v) <= 2}
    got = [tuple(int(x) for x in ci[:dim]) for ci in c]
    assert set(got) == want and len(got) == len(want)
    assert np.all(c[:, dim:] == 0)
    assert np.all(c[opp] == -c)
    d = np.eye(3)
    m1 = np.einsum("i,ia->a", w, c)
    m2 = np.einsum("i,ia,ib->ab", w, c, c)
    m3 = np.einsum("i,ia,ib,ic->abc", w, c, c, c)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    iso4 = cs2 * cs2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                        + np.einsum("ad,bc->abcd", d, d))
    sl = slice(0, dim)
    assert np.allclose(m1, 0, atol=1e-15)
    assert np.allclose(m2[sl, sl], cs2 * np.eye(dim), atol=1e-15)
    assert np.allclose(m3, 0, atol=1e-15)
    assert np.allclose(m4[sl, sl, sl, sl], iso4[sl, sl, sl, sl], atol=1e-15)


def _cfg(q, **kw):
    base = dict(q=q, nx=8, ny=12, nz=1 if q == 9 else 6, tau=0.6)
    if q == 19:
        base.update(nx=6, ny=5, nz=12)
    base.update(kw)
    return OracleConfig(**base)


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("shifted", [False, True])
def test_rest_state_is_exact(q, shifted):
    cfg = _cfg(q, shifted=shifted, vs=1e-3, kappa_c=1e-3)
    f = oracle.equilibrium(cfg)
    c = np.zeros(cfg.shape)
    f2, c2, _, dep, u = oracle.run(cfg, f, c, nsteps=7, want_u=True)
    # exact up to the rounding of sum(w) (a fixed point of the step)
    assert np.max(np.abs(f2 - f)) <= 4e-16
    assert np.max(np.abs(u)) <= 1e-16
    assert np.all(c2 == 0.0) and np.all(dep == 0.0)


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("shifted", [False, True])
def test_mass_conserved_with_walls_and_forcing(q, shifted):
    rng = np.random.default_rng(5)
    # tangential lid velocity only (a wall-normal one would inject mass)
    lid = (0.02, 0.0, 0.0) if q == 9 else (0.02, 0.01, 0.0)
    cfg = _cfg(q, shifted=shifted, gp_c=1e-3, vs=1e-3, kappa_c=1e-3,
               u_top=lid, body_force=(1e-4, 0.0, 0.0))
    u0 = 0.01 * rng.standard_normal((cfg.dim,) + cfg.shape)
    rho0 = 1.0 + 0.01 * rng.standard_normal(cfg.shape)
    f = oracle.equilibrium(cfg, rho0, u0)
    c = rng.uniform(0, 1, cfg.shape)
    s0 = oracle.sums(cfg, f, c)
    f2, c2, _, dep, _ = oracle.run(cfg, f, c, nsteps=50)
    s1 = oracle.sums(cfg, f2, c2, None, dep)
    assert abs(s1[2] - s0[2]) <= 1e-13 * s0[2]
    # particles: sum C + deposit is conserved (absorbing bottom feeds the counter)
    assert abs(s1[0] + s1[3] - s0[0]) <= 1e-13 * s0[0]
    assert s1[3] > 0.0


@pytest.mark.parametrize("q", [9, 19])
def test_guo_momentum_gain_is_exactly_the_force(q):
    """Fully periodic box: each step adds exactly sum_x F(x) to sum f c."""
    rng = np.random.default_rng(7)
    cfg = _cfg(q, vert_periodic=True, gp_c=2e-3, body_force=(3e-4, -1e-4, 2e-4))
    c_ax, _, _ = oracle.lattice(q)
    u0 = 0.01 * rng.standard_normal((cfg.dim,) + cfg.shape)
    f = oracle.equilibrium(cfg, None, u0)
    c = rng.uniform(0, 1, cfg.shape)
    for _ in range(5):
        mom0 = np.einsum("qn,qa->a", f.reshape(cfg.q, -1), c_ax.astype(float))
        fn, cn, _, _, _ = oracle.run(cfg, f, c, nsteps=1)
        mom1 = np.einsum("qn,qa->a", fn.reshape(cfg.q, -1), c_ax.astype(float))
        F = np.zeros(3)
        F[: cfg.dim] = np.array(cfg.body_force[: cfg.dim]) * cfg.nx * cfg.ny * cfg.nz
        F[cfg.dim - 1] += -cfg.gp_c * c.sum()
        assert np.allclose(mom1 - mom0, F, rtol=0, atol=1e-14 * f.size)
        f, c = fn, cn


def _poiseuille(q, tau, H, steps, force=1e-5):
    kw = dict(tau=tau, body_force=(force, 0.0, 0.0))
    if q == 9:
        cfg = OracleConfig(q=9, nx=4, ny=H, nz=1, **kw)
    else:
        cfg = OracleConfig(q=19, nx=4, ny=3, nz=H, **kw)
    f = oracle.equilibrium(cfg)
    c = np.zeros(cfg.shape)
    _, _, _, _, u = oracle.run(cfg, f, c, nsteps=steps, want_u=True)
    nu = (tau - 0.5) / 3.0
    y = np.arange(H) + 0.5            # distance from the wall at -1/2
    exact = force / (2 * nu) * y * (H - y)
    prof = u[0].mean(axis=(0, 2)) if q == 9 else u[0].mean(axis=(1, 2))
    return prof, exact


@pytest.mark.parametrize("q", [9, 19])
def test_poiseuille_exact_at_magic_tau(q):
    """Half-way bounce-back + BGK gives the exact parabola at tau = 1/2 + sqrt(3/16)."""
    tau = 0.5 + math.sqrt(3.0 / 16.0)
    prof, exact = _poiseuille(q, tau, 12, 6000)
    assert np.max(np.abs(prof - exact)) / exact.max() < 1e-10


def test_poiseuille_second_order_at_tau_06():
    errs = []
    for H in (8, 16, 32):
        nu = (0.6 - 0.5) / 3
        steps = int(12 * H * H / (math.pi ** 2 * nu))
        prof, exact = _poiseuille(9, 0.6, H, steps)
        errs.append(np.max(np.abs(prof - exact)) / exact.max())
    r1, r2 = math.log2(errs[0] / errs[1]), math.log2(errs[1] / errs[2])
    assert 1.9 < r1 < 2.1 and 1.9 < r2 < 2.1, errs


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("tau", [0.6, 1.0])
def test_couette_linear_profile(q, tau):
    H, U = 10, 0.01
    if q == 9:
        cfg = OracleConfig(q=9, nx=4, ny=H, nz=1, tau=tau, u_top=(U, 0, 0))
    else:
        cfg = OracleConfig(q=19, nx=4, ny=3, nz=H, tau=tau, u_top=(U, 0, 0))
    nu = (tau - 0.5) / 3
    steps = int(30 * H * H / (math.pi ** 2 * nu))
    f = oracle.equilibrium(cfg)
    _, _, _, _, u = oracle.run(cfg, f, np.zeros(cfg.shape), nsteps=steps, want_u=True)
    prof = u[0].mean(axis=(0, 2)) if q == 9 else u[0].mean(axis=(1, 2))
    exact = U * (np.arange(H) + 0.5) / H
    assert np.max(np.abs(prof - exact)) < 1e-12 * U * 1e3


@pytest.mark.parametrize("q", [9, 19])
def test_shifted_equals_unshifted(q):
    rng = np.random.default_rng(11)
    base = _cfg(q, gp_c=1e-3, vs=1e-3, kappa_c=1e-3, u_top=(0.01, 0, 0))
    sh = OracleConfig(**{**base.__dict__, "shifted": True})
    _, w, _ = oracle.lattice(q)
    u0 = 0.01 * rng.standard_normal((base.dim,) + base.shape)
    f = oracle.equilibrium(base, None, u0)
    g = f - w.reshape((-1, 1, 1, 1))
    c = rng.uniform(0, 1, base.shape)
    f2, c2, _, d2, u2 = oracle.run(base, f, c, nsteps=20, want_u=True)
    g2, c3, _, d3, u3 = oracle.run(sh, g, c, nsteps=20, want_u=True)
    assert np.max(np.abs(g2 + w.reshape((-1, 1, 1, 1)) - f2)) < 1e-14
    assert np.max(np.abs(c3 - c2)) < 1e-14
    assert np.max(np.abs(u3 - u2)) < 1e-15
    assert np.max(np.abs(d3 - d2)) < 1e-16
