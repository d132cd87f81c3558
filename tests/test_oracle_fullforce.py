"""Pins of the oracle's full force and settling (eq. 7, 10, 13): a settling
speed set by the local fluid density, Vs (1 - vs_s S) (the Stokes speed of
eq. 13 with rho linear in S), whose variation the conservative flux turns
into the -phi d(Vs)/dz term of eq. 7; and the buoyancy of S acting on the
fluid fraction 1 - phi, phi = phi_c C (eq. 10).

Closed forms: a uniform S gives exactly the constant-settling run at the
scaled speed; a linear S under a uniform concentration at rest gives every
interior cell the growth rate lambda = -vs vs_s dS/dz, which RK3 integrates
to the factor 1 + lambda + lambda^2/2 + lambda^3/6 (WENO is exact for the
linear flux); the momentum a step adds is the force of eq. 10.
"""
import numpy as np
import pytest

import oracle


def _cfg(q=9, **kw):
    base = dict(q=q, tau=0.6, weno_eps=1e-6, has_s=True)
    base.update(dict(nx=8, ny=40) if q == 9 else dict(nx=5, ny=4, nz=40))
    base.update(kw)
    return oracle.OracleConfig(**base)


def _vertical(cfg):
    n = cfg.ny if cfg.dim == 2 else cfg.nz
    z = np.arange(n, dtype=np.float64)
    return (z[None, :, None] if cfg.dim == 2 else z[:, None, None]) * np.ones(cfg.shape), n


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("classes", [1, 2])
def test_uniform_s_is_constant_settling_at_the_scaled_speed(q, classes):
    s0, vs_s = 0.625, 0.4
    vs = (3e-3, 1e-3)[:classes]
    kw = dict(frozen=True, kappa_s=1e-3)
    if classes > 1:
        var = _cfg(q, n_classes=2, vs_class=vs, kappa_class=(1e-3, 2e-3), vs_s=vs_s, **kw)
        const = _cfg(q, n_classes=2, vs_class=tuple(v * (1.0 - vs_s * s0) for v in vs),
                     kappa_class=(1e-3, 2e-3), **kw)
    else:
        var = _cfg(q, vs=vs[0], kappa_c=1e-3, vs_s=vs_s, **kw)
        const = _cfg(q, vs=vs[0] * (1.0 - vs_s * s0), kappa_c=1e-3, **kw)
    rng = np.random.default_rng(3)
    shape = var.shape if classes == 1 else (classes,) + var.shape
    c = rng.uniform(0, 1, shape)
    s = np.full(var.shape, s0)
    u = np.zeros((var.dim,) + var.shape)
    u[0] = 0.03                      # uniform lateral flow keeps S uniform exactly
    _, c1, s1, d1, _ = oracle.run(var, None, c, s, None, u, 10)
    _, c2, s2, d2, _ = oracle.run(const, None, c, s, None, u, 10)
    assert np.array_equal(s1, s) and np.array_equal(s2, s)
    assert np.array_equal(c1, c2) and np.array_equal(d1, d2)
    # and the speed really changed the result
    _, c3, _, _, _ = oracle.run(_cfg(q, vs=vs[0], kappa_c=1e-3, **kw), None, c if classes == 1 else c[0],
                                s, None, u, 10)
    assert not np.array_equal(c3, c1 if classes == 1 else c1[0])


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("scheme", ["weno5", "weno3", "upwind1"])
def test_settling_gradient_term_closed_form(q, scheme):
    """Fluid at rest, no diffusion, S = s_a + s_b z (unchanged: no flow), C =
    c0: the flux -Vs(z) c0 is linear in z, every reconstruction is exact for
    it, so each cell three stencils clear of the walls after all three RK
    stages grows by the RK3 factor of lambda = -vs vs_s s_b."""
    vs, vs_s, s_a, s_b, c0 = 4e-3, 0.5, 0.9, -0.02, 0.7
    cfg = _cfg(q, frozen=True, vs=vs, vs_s=vs_s, scheme_c=scheme)
    z, n = _vertical(cfg)
    s = s_a + s_b * z
    c = np.full(cfg.shape, c0)
    u = np.zeros((cfg.dim,) + cfg.shape)
    _, c1, s1, _, _ = oracle.run(cfg, None, c, s, None, u, 1)
    assert np.array_equal(s1, s)
    lam = -vs * vs_s * s_b
    want = c0 * (1 + lam + lam**2 / 2 + lam**3 / 6)
    sel = (z >= 9) & (z <= n - 10)
    assert np.max(np.abs(c1[sel] - want)) <= 1e-14, np.max(np.abs(c1[sel] - want))
    assert lam > 0 and want > c0            # slower settling below: particles gather
    # with vs_s = 0 the same cells do not change
    _, c2, _, _, _ = oracle.run(_cfg(q, frozen=True, vs=vs, scheme_c=scheme), None, c, s, None, u, 1)
    assert np.max(np.abs(c2[sel] - c0)) <= 1e-15


@pytest.mark.parametrize("q", [9, 19])
def test_momentum_gain_is_the_full_force(q):
    """Fully periodic box: a step adds sum_x F(x) to sum f c with F_vert =
    -gp_c C - gp_s S (1 - phi_c C) (eq. 10 with phi = phi_c C)."""
    rng = np.random.default_rng(8)
    gp_c, gp_s, phi_c = 2e-3, -1.5e-3, 0.3
    cfg = _cfg(q, vert_periodic=True, gp_c=gp_c, gp_s=gp_s, phi_c=phi_c, kappa_s=1e-3,
               body_force=(3e-4, -1e-4, 2e-4))
    if q == 19:
        cfg = _cfg(q, vert_periodic=True, gp_c=gp_c, gp_s=gp_s, phi_c=phi_c, kappa_s=1e-3,
                   body_force=(3e-4, -1e-4, 2e-4), nz=12)
    c_ax, _, _ = oracle.lattice(q)
    f = oracle.equilibrium(cfg, None, 0.01 * rng.standard_normal((cfg.dim,) + cfg.shape))
    c = rng.uniform(0, 1, cfg.shape)
    s = rng.uniform(0, 1, cfg.shape)
    for _ in range(4):
        mom0 = np.einsum("qn,qa->a", f.reshape(cfg.q, -1), c_ax.astype(float))
        fn, cn, sn, _, _ = oracle.run(cfg, f, c, s, nsteps=1)
        mom1 = np.einsum("qn,qa->a", fn.reshape(cfg.q, -1), c_ax.astype(float))
        F = np.zeros(3)
        F[: cfg.dim] = np.array(cfg.body_force[: cfg.dim]) * c.size
        F[cfg.dim - 1] += np.sum(-gp_c * c - gp_s * s * (1 - phi_c * c))
        assert np.allclose(mom1 - mom0, F, rtol=0, atol=1e-14 * f.size)
        # the cross term matters at this size
        F0 = F.copy()
        F0[cfg.dim - 1] += np.sum(gp_s * s * (-phi_c * c))
        assert not np.allclose(mom1 - mom0, F0, rtol=0, atol=1e-12 * f.size)
        f, c, s = fn, cn, sn


def test_zero_coefficients_change_nothing_and_need_s():
    rng = np.random.default_rng(9)
    a = _cfg(9, vs=2e-3, kappa_c=1e-3, gp_c=1e-3, gp_s=1e-3, kappa_s=1e-3)
    f = oracle.equilibrium(a)
    c, s = rng.uniform(0, 1, a.shape), rng.uniform(0, 1, a.shape)
    r1 = oracle.run(a, f, c, s, None, None, 5)
    r2 = oracle.run(_cfg(9, vs=2e-3, kappa_c=1e-3, gp_c=1e-3, gp_s=1e-3, kappa_s=1e-3, vs_s=0.0,
                         phi_c=0.0), f, c, s, None, None, 5)
    for x, y in zip(r1[:4], r2[:4]):
        assert np.array_equal(x, y)
    with pytest.raises(ValueError):
        oracle.run(_cfg(9, has_s=False, vs_s=0.1), f, c, None, None, None, 1)
