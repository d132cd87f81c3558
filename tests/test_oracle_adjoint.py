"""Pins of the oracle's hand-written adjoint against central finite
differences of the (already pinned) forward oracle, in FP64.

J = total deposited mass after n steps.  Directional derivatives of J with
respect to the initial concentration, the initial populations and the
settling speed must match (J(x + e v) - J(x - e v)) / 2e.  The runs start
from a flowing state so that no face velocity sits at the upwind switch,
where the reconstructed flux is not differentiable.
"""
import numpy as np
import pytest

import oracle
from oracle import OracleConfig


def _forward_states(cfg, f0, c0, u_in, n):
    fs, cs = [], []
    f, c = f0, c0
    for _ in range(n):
        fs.append(f)
        cs.append(c)
        f, c, _, _, _ = oracle.run(cfg, f, c, None, None, u_in, 1)
    return fs, cs


def _J(cfg, f0, c0, u_in, n):
    _, _, _, dep, _ = oracle.run(cfg, f0, c0, None, None, u_in, n)
    return dep.sum()


def _gradients(cfg, f0, c0, u_in, n):
    fs, cs = _forward_states(cfg, f0, c0, u_in, n)
    cbar = np.zeros(cfg.shape)
    fbar = None if cfg.frozen else np.zeros((cfg.q,) + cfg.shape)
    vsb = 0.0
    for k in reversed(range(n)):
        fbar, cbar, v = oracle.adjoint_step(cfg, fs[k], cs[k], fbar, cbar, 1.0, u_in)
        vsb += v
    return fbar, cbar, vsb


def _flowing_state(cfg, rng):
    dim = cfg.dim
    u0 = 0.02 * rng.standard_normal((dim,) + cfg.shape) + np.array(
        [0.03, 0.02, 0.01][:dim]).reshape((dim, 1, 1, 1))
    f0 = oracle.equilibrium(cfg, 1.0 + 0.01 * rng.standard_normal(cfg.shape), u0)
    c0 = rng.uniform(0.2, 1.0, cfg.shape)
    return f0, c0, u0


def _fd(fun, x, v, e):
    return (fun(x + e * v) - fun(x - e * v)) / (2 * e)


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("shifted", [False, True])
def test_coupled_adjoint_matches_fd(q, shifted):
    rng = np.random.default_rng(21)
    if q == 9:
        cfg = OracleConfig(q=9, nx=10, ny=14, tau=0.7, vs=0.04, kappa_c=2e-3, gp_c=3e-3,
                           shifted=shifted)
    else:
        cfg = OracleConfig(q=19, nx=5, ny=4, nz=10, tau=0.7, vs=0.04, kappa_c=2e-3, gp_c=3e-3,
                           shifted=shifted)
    n = 4
    f0, c0, _ = _flowing_state(cfg, rng)    # equilibrium() already shifts
    fbar, cbar, vsb = _gradients(cfg, f0, c0, None, n)
    e = 1e-6
    for trial in range(3):
        vc = rng.standard_normal(cfg.shape)
        fd = _fd(lambda c: _J(cfg, f0, c, None, n), c0, vc, e)
        assert abs(np.sum(cbar * vc) - fd) <= 1e-6 * max(abs(fd), 1e-12), (trial, np.sum(cbar * vc), fd)
        vf = rng.standard_normal(f0.shape) * 1e-2
        fd = _fd(lambda f: _J(cfg, f, c0, None, n), f0, vf, e)
        assert abs(np.sum(fbar * vf) - fd) <= 1e-6 * max(abs(fd), 1e-12), (trial, np.sum(fbar * vf), fd)
    def Jvs(vs):
        c2 = OracleConfig(**{**cfg.__dict__, "vs": vs})
        return _J(c2, f0, c0, None, n)
    fd = (Jvs(cfg.vs + e) - Jvs(cfg.vs - e)) / (2 * e)
    assert abs(vsb - fd) <= 1e-6 * abs(fd), (vsb, fd)


@pytest.mark.parametrize("vper", [False, True])
def test_frozen_transport_adjoint_matches_fd(vper):
    rng = np.random.default_rng(22)
    cfg = OracleConfig(q=9, nx=9, ny=13, frozen=True, vert_periodic=vper, vs=0.05,
                       kappa_c=3e-3)
    u = 0.02 * rng.standard_normal((2,) + cfg.shape)
    u[0] += 0.05
    c0 = rng.uniform(0.0, 1.0, cfg.shape)
    n = 6
    _, cbar, vsb = _gradients(cfg, None, c0, u, n)
    e = 1e-6
    for trial in range(4):
        v = rng.standard_normal(cfg.shape)
        fd = _fd(lambda c: _J(cfg, None, c, u, n), c0, v, e)
        if vper:
            # no walls: nothing is ever deposited
            assert abs(fd) < 1e-14 and abs(np.sum(cbar * v)) < 1e-14
        else:
            assert abs(np.sum(cbar * v) - fd) <= 1e-7 * abs(fd), (np.sum(cbar * v), fd)
    if not vper:
        def Jvs(vs):
            return _J(OracleConfig(**{**cfg.__dict__, "vs": vs}), None, c0, u, n)
        fd = (Jvs(cfg.vs + e) - Jvs(cfg.vs - e)) / (2 * e)
        assert abs(vsb - fd) <= 1e-7 * abs(fd), (vsb, fd)


def test_adjoint_of_uniform_layer_deposit():
    """Closed form: at rest with uniform C the first steps deposit
    n Vs c per column, so dJ/dVs = n c ncol and dJ/dC0 sums to n Vs ncol
    over the cells that feed the bottom."""
    cfg = OracleConfig(q=9, nx=4, ny=60, frozen=True, vs=0.01, kappa_c=0.0)
    u = np.zeros((2,) + cfg.shape)
    c0 = np.full(cfg.shape, 0.7)
    n = 3
    _, cbar, vsb = _gradients(cfg, None, c0, u, n)
    assert abs(vsb - n * 0.7 * cfg.nx) < 1e-12
    assert abs(cbar.sum() - n * cfg.vs * cfg.nx) < 1e-12
