"""Pins of the oracle's scalar-transport part (supplement section 1).

WENO5 polynomial exactness (any weights up to degree 2, linear weights up to
degree 4), WENO3 likewise (degree 1 / 2), fifth-order convergence on smooth
periodic advection, the RK3 amplification factor on a diffusing Fourier mode
(S21-S23), upwind S5/S6 updates, rigid settling, the absorbing-bottom deposit
of a uniform layer and the particle budget sum C + deposit.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import OracleConfig


def _frozen(q=9, nx=4, ny=40, nz=1, **kw):
    if q == 19 and nz == 1:
        nz = ny
        ny = 3
    base = dict(q=q, nx=nx, ny=ny, nz=nz, frozen=True, tau=0.6)
    base.update(kw)
    return OracleConfig(**base)


def _vert(cfg):
    """vertical coordinate broadcast to the field shape"""
    if cfg.dim == 2:
        return np.broadcast_to(np.arange(cfg.ny, dtype=float)[None, :, None], cfg.shape)
    return np.broadcast_to(np.arange(cfg.nz, dtype=float)[:, None, None], cfg.shape)


def _interior(cfg, arr, r=3):
    nv = cfg.ny if cfg.dim == 2 else cfg.nz
    if cfg.dim == 2:
        return arr[:, r:nv - r - 1, :]
    return arr[r:nv - r - 1]


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("direction", [+1, -1])
@pytest.mark.parametrize("deg,eps", [(0, 1e-6), (1, 1e-6), (2, 1e-6), (3, 1e30), (4, 1e30)])
def test_weno5_polynomial_exactness(q, direction, deg, eps):
    """Degree <= 2 exact for any convex weights; degree <= 4 with linear weights."""
    cfg = _frozen(q, vs=0.0, kappa_c=0.0, weno_eps=eps)
    y = _vert(cfg)
    coef = [0.3, -0.7, 0.11, -0.013, 0.0021][: deg + 1]
    a = sum(cf * (y / 10.0) ** k for k, cf in enumerate(coef))
    da = sum(k * cf * (y / 10.0) ** (k - 1) / 10.0 for k, cf in enumerate(coef) if k)
    u = np.zeros((cfg.dim,) + cfg.shape)
    u[cfg.dim - 1] = 0.37 * direction     # uniform transport velocity
    L, _ = oracle.rhs_c(cfg, np.ascontiguousarray(a), u)
    exact = -0.37 * direction * da
    err = np.max(np.abs(_interior(cfg, L - exact)))
    assert err < 1e-13, err


@pytest.mark.parametrize("direction", [+1, -1])
def test_weno5_variable_velocity_quadratic_flux(direction):
    """h = w a quadratic (w and a linear) is differentiated exactly."""
    cfg = _frozen(9, vs=0.0, kappa_c=0.0)
    y = _vert(cfg)
    a = np.ascontiguousarray(0.5 + 0.03 * y)
    u = np.zeros((2,) + cfg.shape)
    u[1] = direction * (0.2 + 0.004 * y)
    L, _ = oracle.rhs_c(cfg, a, u)
    exact = -(0.004 * direction * a + u[1] * 0.03)
    assert np.max(np.abs(_interior(cfg, L - exact))) < 1e-14


@pytest.mark.parametrize("direction", [+1, -1])
@pytest.mark.parametrize("deg,eps", [(1, 1e-6), (2, 1e30)])
def test_weno3_polynomial_exactness(direction, deg, eps):
    cfg = _frozen(9, vs=0.0, kappa_c=0.0, weno_eps=eps, scheme_c="weno3")
    y = _vert(cfg)
    coef = [0.3, -0.7, 0.11][: deg + 1]
    a = sum(cf * (y / 10.0) ** k for k, cf in enumerate(coef))
    da = sum(k * cf * (y / 10.0) ** (k - 1) / 10.0 for k, cf in enumerate(coef) if k)
    u = np.zeros((2,) + cfg.shape)
    u[1] = 0.37 * direction
    L, _ = oracle.rhs_c(cfg, np.ascontiguousarray(a), u)
    assert np.max(np.abs(_interior(cfg, L + 0.37 * direction * da))) < 1e-13


def _advect_error(N, scheme, axis, eps, full_rk):
    """L1 error of periodic advection of sin(2 pi x / N) along one axis."""
    if axis == 0:
        cfg = _frozen(9, nx=N, ny=6, vert_periodic=True, scheme_c=scheme, weno_eps=eps)
        x = np.broadcast_to(np.arange(N, dtype=float)[None, None, :], cfg.shape)
    else:
        cfg = _frozen(9, nx=3, ny=N, vert_periodic=True, scheme_c=scheme, weno_eps=eps)
        x = np.broadcast_to(np.arange(N, dtype=float)[None, :, None], cfg.shape)
    k = 2 * math.pi / N
    a0 = np.ascontiguousarray(np.sin(k * x) + 0.5)
    # the full step keeps CFL ~ N^(-2/3) so RK3's error falls like N^-5 too
    U = 0.5 * (16.0 / N) ** (2.0 / 3.0) if full_rk else 0.5
    u = np.zeros((2,) + cfg.shape)
    u[axis] = U
    if not full_rk:
        L, _ = oracle.rhs_c(cfg, a0, u)
        # relative to the derivative's own amplitude U k
        return np.mean(np.abs(L + U * k * np.cos(k * x))) / (U * k)
    T = 0.25 * N / U
    n = int(round(T))
    _, c, _, _, _ = oracle.run(cfg, None, a0, u_in=u, nsteps=n)
    exact = np.sin(k * (x - U * n)) + 0.5
    return np.mean(np.abs(c - exact))


@pytest.mark.parametrize("axis", [0, 1])
def test_weno5_spatial_order(axis):
    Ns = [16, 32, 64, 128]
    errs = [_advect_error(N, "weno5", axis, 1e-6, False) for N in Ns]
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert orders[-1] >= 4.7, (errs, orders)
    lin = [_advect_error(N, "weno5", axis, 1e30, False) for N in Ns]
    lorders = [math.log2(lin[i] / lin[i + 1]) for i in range(3)]
    assert min(lorders) >= 4.9, (lin, lorders)


def test_weno5_rk3_order():
    """WENO5 in space + RK3 in time with U ~ N^(-2/3): fifth order overall."""
    Ns = [16, 32, 64]
    errs = [_advect_error(N, "weno5", 0, 1e-6, True) for N in Ns]
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(Ns) - 1)]
    assert orders[-1] >= 4.5, (errs, orders)


def test_weno3_spatial_order_linear_weights():
    Ns = [16, 32, 64, 128]
    errs = [_advect_error(N, "weno3", 0, 1e30, False) for N in Ns]
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert min(orders) >= 2.9, (errs, orders)


@pytest.mark.parametrize("q", [9, 19])
def test_rk3_amplification_of_diffusing_mode(q):
    """u = 0, vs = 0: each stage applies the central Laplacian, eigenvalue z,
    so n steps multiply a Fourier mode by (1 + z + z^2/2 + z^3/6)^n."""
    if q == 9:
        cfg = OracleConfig(q=9, nx=12, ny=10, nz=1, frozen=True, vert_periodic=True,
                           kappa_c=0.07)
        kk = (2, 3)
    else:
        cfg = OracleConfig(q=19, nx=8, ny=6, nz=10, frozen=True, vert_periodic=True,
                           kappa_c=0.05)
        kk = (1, 2, 3)
    dims = (cfg.nx, cfg.ny, cfg.nz)[: cfg.dim]
    grids = np.meshgrid(*[np.arange(n, dtype=float) for n in dims], indexing="ij")
    phase = sum(2 * math.pi * kk[i] * grids[i] / dims[i] for i in range(cfg.dim))
    a0 = np.cos(phase).transpose()[None] if cfg.dim == 2 else np.cos(phase).transpose()
    a0 = np.ascontiguousarray(a0.reshape(cfg.shape))
    z = -4 * cfg.kappa_c * sum(math.sin(math.pi * kk[i] / dims[i]) ** 2 for i in range(cfg.dim))
    G = 1 + z + z * z / 2 + z ** 3 / 6
    u = np.zeros((cfg.dim,) + cfg.shape)
    _, c, _, _, _ = oracle.run(cfg, None, a0, u_in=u, nsteps=25)
    assert np.max(np.abs(c - G ** 25 * a0)) < 1e-13


def test_upwind1_rk3_amplification():
    """First-order upwind: eigenvalue -U(1 - e^{-ik}); RK3 polynomial of it."""
    N, U, kk = 20, 0.3, 3
    cfg = OracleConfig(q=9, nx=N, ny=6, nz=1, frozen=True, vert_periodic=True,
                       scheme_c="upwind1")
    x = np.broadcast_to(np.arange(N, dtype=float)[None, None, :], cfg.shape)
    k = 2 * math.pi * kk / N
    a0 = np.ascontiguousarray(np.cos(k * x))
    u = np.zeros((2,) + cfg.shape)
    u[0] = U
    z = -U * (1 - np.exp(-1j * k))
    G = 1 + z + z * z / 2 + z ** 3 / 6
    _, c, _, _, _ = oracle.run(cfg, None, a0, u_in=u, nsteps=7)
    exact = np.real(G ** 7 * np.exp(1j * k * x))
    assert np.max(np.abs(c - exact)) < 1e-14


@pytest.mark.parametrize("U", [0.3, -0.3])
def test_s_upwind_forward_euler(U):
    """S: S^{n+1}_i = S_i - U (S_i - S_{i-1}) for U > 0 (S5), forward
    difference for U < 0 (S6), in the conservative form used here."""
    rng = np.random.default_rng(3)
    N = 16
    cfg = OracleConfig(q=9, nx=N, ny=8, nz=1, frozen=True, has_s=True, kappa_s=0.0)
    s0 = rng.uniform(0, 1, cfg.shape)
    u = np.zeros((2,) + cfg.shape)
    u[0] = U
    _, _, s1, _, _ = oracle.run(cfg, None, np.zeros(cfg.shape), s=s0, u_in=u, nsteps=1)
    if U > 0:
        exact = s0 - U * (s0 - np.roll(s0, 1, axis=2))
    else:
        exact = s0 - U * (np.roll(s0, -1, axis=2) - s0)
    assert np.max(np.abs(s1 - exact)) < 1e-15


def test_s_diffusion_and_closed_walls():
    """Forward Euler diffusion of S: a lateral mode decays by 1 + z exactly;
    walls pass no S, so sum S is conserved with any velocity."""
    N, kap = 12, 0.1
    cfg = OracleConfig(q=9, nx=N, ny=8, nz=1, frozen=True, has_s=True, kappa_s=kap)
    x = np.broadcast_to(np.arange(N, dtype=float)[None, None, :], cfg.shape)
    s0 = np.ascontiguousarray(np.cos(2 * math.pi * 2 * x / N))
    u = np.zeros((2,) + cfg.shape)
    _, _, s1, _, _ = oracle.run(cfg, None, np.zeros(cfg.shape), s=s0, u_in=u, nsteps=4)
    z = -4 * kap * math.sin(math.pi * 2 / N) ** 2
    assert np.max(np.abs(s1 - (1 + z) ** 4 * s0)) < 1e-14
    rng = np.random.default_rng(4)
    u = 0.1 * rng.standard_normal((2,) + cfg.shape)
    s0 = rng.uniform(0, 1, cfg.shape)
    _, _, s1, _, _ = oracle.run(cfg, None, np.zeros(cfg.shape), s=s0, u_in=u, nsteps=10)
    assert abs(s1.sum() - s0.sum()) < 1e-13 * s0.sum()


@pytest.mark.parametrize("q", [9, 19])
def test_uniform_layer_deposit(q):
    """Uniform C at rest: the bottom loses exactly Vs*c per column per step until
    the top wall's influence (3 cells per RK stage) reaches it."""
    c0, vs = 0.7, 0.01
    cfg = _frozen(q, nx=5, ny=64, vs=vs, kappa_c=1e-3)
    u = np.zeros((cfg.dim,) + cfg.shape)
    a = np.full(cfg.shape, c0)
    n = 5
    _, c, _, dep, _ = oracle.run(cfg, None, a, u_in=u, nsteps=n)
    ncol = cfg.ncol
    assert np.allclose(dep, n * vs * c0, rtol=1e-14, atol=0)
    assert abs(dep.sum() - n * vs * c0 * ncol) < 1e-14 * n * vs * c0 * ncol
    # the particle budget holds for any length
    _, c, _, dep, _ = oracle.run(cfg, None, a, u_in=u, nsteps=400)
    assert abs(c.sum() + dep.sum() - a.sum()) < 1e-13 * a.sum()


def test_rigid_settling_translation():
    """u = 0, kappa = 0: a smooth periodic column moves down at Vs."""
    errs = []
    for N in (32, 64):
        vs = 0.05 * (32.0 / N) ** (2.0 / 3.0)
        cfg = OracleConfig(q=9, nx=3, ny=N, nz=1, frozen=True, vert_periodic=True, vs=vs)
        y = np.broadcast_to(np.arange(N, dtype=float)[None, :, None], cfg.shape)
        k = 2 * math.pi / N
        a0 = np.ascontiguousarray(1.0 + 0.5 * np.sin(k * y))
        n = int(round(0.5 * N / vs))
        _, c, _, _, _ = oracle.run(cfg, None, a0, u_in=np.zeros((2,) + cfg.shape), nsteps=n)
        exact = 1.0 + 0.5 * np.sin(k * (y + vs * n))
        errs.append(np.mean(np.abs(c - exact)))
    assert errs[0] < 1e-4 and math.log2(errs[0] / errs[1]) > 4.5, errs


@pytest.mark.parametrize("vs,kappa,steps", [(1e-3, 1e-3, 1000), (0.2, 0.0, 150)])
def test_settling_front_overshoot(vs, kappa, steps):
    """WENO is essentially non-oscillatory: a settling front stays within
    [0, 1] up to 1e-3 (tanh front of width 2, and a sharp step at CFL 0.2)."""
    N = 96
    cfg = OracleConfig(q=9, nx=3, ny=N, nz=1, frozen=True, vs=vs, kappa_c=kappa)
    y = np.broadcast_to(np.arange(N, dtype=float)[None, :, None], cfg.shape)
    if kappa > 0:
        a0 = 0.5 * (1 + np.tanh((y - (N - 1) / 2) / 2))
    else:
        a0 = (y >= 60).astype(float)
    a0 = np.ascontiguousarray(a0)
    _, c, _, dep, _ = oracle.run(cfg, None, a0, u_in=np.zeros((2,) + cfg.shape), nsteps=steps)
    assert c.min() > -1e-3 and c.max() < 1 + 1e-3, (c.min(), c.max())
    assert abs(c.sum() + dep.sum() - a0.sum()) < 1e-12 * a0.sum()


# ---------------------------------------------------------------------------
# Wall ghosts by a mirror image (section 2.2.1, eq. 14-15).  Zero normal
# gradient of the scalar and no flow through the wall are what an even
# reflection of C and an odd reflection of the vertical fluid velocity about
# the wall produce; settling does not reverse at a wall (it is the particles'
# own motion, not the fluid's).  A walled run of height n therefore sees, in
# every stencil that reaches beyond a wall, exactly what a periodic run of
# height 2n sees when it holds the reflected run below the physical one:
# image cell n-1-m = physical cell m with C, the lateral velocities and S
# unchanged and the vertical transport velocity -u_v(m) - Vs(m), physical
# cells with u_v - Vs.  The periodic run settles at 0 (its velocity carries
# the settling), so none of the wall rules is in it: each face of the walled
# run must equal the same face of the periodic run bit for bit, except the
# two wall faces the method overrides (R10: -Vs a_0 at the bottom, 0 at the
# top).  An image built by another rule (settling reversed, C odd, fluid
# velocity even) must not agree, which shows the comparison can fail.
# ---------------------------------------------------------------------------

def _mirror_case(q, nx, nvert, scheme, vs, kappa, vs_s, seed):
    rng = np.random.default_rng(seed)
    if q == 9:
        shape, vax = (1, nvert, nx), 1
        kw = dict(q=9, nx=nx, ny=nvert, nz=1)
    else:
        shape, vax = (nvert, 3, nx), 0
        kw = dict(q=19, nx=nx, ny=3, nz=nvert)
    dim = 2 if q == 9 else 3
    a = 0.5 + rng.random(shape)
    a += 0.3 * np.sin(np.arange(nvert) / 3.0).reshape([-1 if i == vax else 1 for i in range(3)])
    u = 0.05 * (rng.random((dim,) + shape) - 0.5)
    s = rng.random(shape) if vs_s else None
    walled = OracleConfig(frozen=True, scheme_c=scheme, vs=vs, kappa_c=kappa, weno_eps=1e-6,
                          has_s=vs_s != 0.0, vs_s=vs_s, **kw)
    kw_p = dict(kw)
    if q == 9:
        kw_p["ny"] = 2 * nvert
    else:
        kw_p["nz"] = 2 * nvert
    periodic = OracleConfig(frozen=True, scheme_c=scheme, vs=0.0, kappa_c=kappa, weno_eps=1e-6,
                            vert_periodic=True, **kw_p)
    settle = vs if not vs_s else vs * (1.0 - vs_s * s)
    return walled, periodic, a, u, s, settle, vax, dim


def _image(a, u, settle, vax, dim, rule="paper"):
    """The periodic run's fields: the reflected run (image) below the run."""
    flip = lambda x: np.flip(x, axis=vax)
    uv = u[dim - 1]
    phys_w = uv - settle
    if rule == "paper":
        img_a, img_w = flip(a), flip(-uv - settle)
    elif rule == "settling_reversed":
        img_a, img_w = flip(a), flip(-(uv - settle))
    elif rule == "c_odd":
        img_a, img_w = flip(-a), flip(-uv - settle)
    elif rule == "fluid_even":
        img_a, img_w = flip(a), flip(uv - settle)
    else:
        raise ValueError(rule)
    ap = np.ascontiguousarray(np.concatenate([img_a, a], axis=vax))
    up = np.empty((dim,) + ap.shape)
    for d in range(dim - 1):
        up[d] = np.concatenate([flip(u[d]), u[d]], axis=vax)
    up[dim - 1] = np.concatenate([img_w, phys_w], axis=vax)
    return ap, up


def _upper(x, vax, n):
    """the physical half of a periodic field (the last n planes)"""
    return np.take(x, np.arange(n, 2 * n), axis=vax)


@pytest.mark.parametrize("q,nx", [(9, 7), (19, 5)])
@pytest.mark.parametrize("scheme", ["weno5", "weno3", "upwind1"])
@pytest.mark.parametrize("vs_s", [0.0, 0.4])
def test_wall_ghosts_mirror_image(q, nx, scheme, vs_s):
    n = 12
    walled, periodic, a, u, s, settle, vax, dim = _mirror_case(q, nx, n, scheme, 0.02, 3e-3,
                                                               vs_s, seed=17 + q)
    phi_w, bot_w = oracle.faces_c(walled, a, u, s)
    ap, up = _image(a, u, settle, vax, dim)
    phi_p, _ = oracle.faces_c(periodic, ap, up)
    for d in range(dim):
        pw, pp = phi_w[d], _upper(phi_p[d], vax, n)
        if d == dim - 1:
            # the top node's +face is the top wall: no flux in the walled run
            top = [slice(None)] * 3
            top[vax] = slice(n - 1, n)
            assert np.all(pw[tuple(top)] == 0.0)
            keep = [slice(None)] * 3
            keep[vax] = slice(0, n - 1)
            pw, pp = pw[tuple(keep)], pp[tuple(keep)]
        np.testing.assert_array_equal(pw, pp)
    # the bottom wall face carries the absorbed settling flux -Vs a_0
    bottom = [slice(None)] * 3
    bottom[vax] = 0
    a0 = a[tuple(bottom)]
    vs0 = settle if np.isscalar(settle) else settle[tuple(bottom)]
    np.testing.assert_array_equal(bot_w, (-vs0 * a0).ravel())
    if vs_s == 0.0:
        # the operator itself: every cell off the walls agrees bit for bit
        L_w, _ = oracle.rhs_c(walled, a, u)
        L_p, _ = oracle.rhs_c(periodic, ap, up)
        inner = [slice(None)] * 3
        inner[vax] = slice(1, n - 1)
        np.testing.assert_array_equal(L_w[tuple(inner)], _upper(L_p, vax, n)[tuple(inner)])


@pytest.mark.parametrize("q,nx", [(9, 7), (19, 5)])
@pytest.mark.parametrize("scheme", ["weno5", "weno3"])
@pytest.mark.parametrize("rule", ["settling_reversed", "c_odd", "fluid_even"])
def test_wall_ghosts_mirror_image_rejects_other_rules(q, nx, scheme, rule):
    n = 12
    walled, periodic, a, u, s, settle, vax, dim = _mirror_case(q, nx, n, scheme, 0.02, 3e-3,
                                                               0.0, seed=29 + q)
    phi_w, _ = oracle.faces_c(walled, a, u)
    ap, up = _image(a, u, settle, vax, dim, rule)
    phi_p, _ = oracle.faces_c(periodic, ap, up)
    v = dim - 1
    keep = [slice(None)] * 3
    keep[vax] = slice(0, n - 1)
    diff = np.abs(phi_w[v][tuple(keep)] - _upper(phi_p[v], vax, n)[tuple(keep)])
    assert diff.max() > 1e-6 * np.abs(phi_w[v]).max()


@pytest.mark.parametrize("q,nx", [(9, 7), (19, 5)])
@pytest.mark.parametrize("vper", [False, True])
def test_operator_is_minus_the_divergence_of_the_exposed_faces(q, nx, vper):
    """orc_faces_c exposes the fluxes orc_rhs_c differences: summing the
    per-axis differences (bottom wall face included, periodic axes wrapped)
    gives L, so the mirror-image comparison above is about the operator's own
    faces."""
    n = 12
    walled, _, a, u, _, _, vax, dim = _mirror_case(q, nx, n, "weno5", 0.02, 3e-3, 0.0, seed=41 + q)
    cfg = walled if not vper else OracleConfig(**{**walled.__dict__, "vert_periodic": True})
    phi, bottom = oracle.faces_c(cfg, a, u)
    L, _ = oracle.rhs_c(cfg, a, u)
    arr_ax = {0: 2, 1: 1, 2: 0}          # field axis of each lattice axis (z, y, x order)
    acc = np.zeros_like(a)
    for d in range(dim):
        ax = arr_ax[d] if dim == 3 else (2 if d == 0 else 1)
        left = np.roll(phi[d], 1, axis=ax)
        if d == dim - 1 and not vper:
            sl = [slice(None)] * 3
            sl[ax] = 0
            left[tuple(sl)] = bottom.reshape(left[tuple(sl)].shape)
        acc = acc + (phi[d] - left)
    np.testing.assert_allclose(L, -acc, rtol=0, atol=1e-15 * np.abs(phi).max())
    if not vper:
        top = [slice(None)] * 3
        top[vax] = n - 1
        assert np.all(phi[dim - 1][tuple(top)] == 0.0)
