"""Pins of the oracle's particle size classes (eq. 11-12): N concentration
fields, each obeying the C equation with its own settling speed and
diffusivity, sharing one fluid whose buoyancy is that of the total
concentration.

Each pin reduces the N-class step to the single-class step, which the other
oracle tests pin, through a relation that holds exactly (bit for bit): an
empty class changes nothing, the class order does not matter, a frozen flow
decouples the classes, and with the linear first-order flux two halves of a
field move exactly as the field does (so the fluid sees the total).
"""
import numpy as np
import pytest

import oracle


def _cfg(q=9, **kw):
    base = dict(q=q, tau=0.6, gp_c=2e-4, weno_eps=1e-6)
    base.update(dict(nx=12, ny=16) if q == 9 else dict(nx=6, ny=5, nz=12))
    base.update(kw)
    return oracle.OracleConfig(**base)


def _fields(cfg, seed, n=1):
    rng = np.random.default_rng(seed)
    return [rng.uniform(0, 1, cfg.shape) for _ in range(n)]


def _run(cfg, cs, nsteps, u_in=None):
    c = np.stack(cs) if cfg.ncls > 1 else cs[0]
    f = None if cfg.frozen else oracle.equilibrium(cfg)
    return oracle.run(cfg, f, c, None, None, u_in, nsteps)


@pytest.mark.parametrize("q", [9, 19])
def test_an_empty_class_changes_nothing(q):
    one = _cfg(q, vs=3e-3, kappa_c=2e-3)
    two = _cfg(q, n_classes=2, vs_class=(3e-3, 1e-3), kappa_class=(2e-3, 5e-4))
    (c0,) = _fields(one, 1)
    f1, c1, _, d1, _ = _run(one, [c0], 12)
    f2, c2, _, d2, _ = _run(two, [c0, np.zeros_like(c0)], 12)
    assert np.array_equal(f1, f2)
    assert np.array_equal(c1, c2[0]) and not c2[1].any()
    assert np.array_equal(d1, d2[0]) and not d2[1].any()


@pytest.mark.parametrize("q", [9, 19])
def test_class_order_does_not_matter(q):
    ab = _cfg(q, n_classes=2, vs_class=(3e-3, 1e-3), kappa_class=(2e-3, 5e-4))
    ba = _cfg(q, n_classes=2, vs_class=(1e-3, 3e-3), kappa_class=(5e-4, 2e-3))
    ca, cb = _fields(ab, 2, 2)
    f1, c1, _, d1, _ = _run(ab, [ca, cb], 10)
    f2, c2, _, d2, _ = _run(ba, [cb, ca], 10)
    assert np.array_equal(f1, f2)                      # a + b == b + a in the force
    assert np.array_equal(c1[0], c2[1]) and np.array_equal(c1[1], c2[0])
    assert np.array_equal(d1[0], d2[1]) and np.array_equal(d1[1], d2[0])


def test_frozen_flow_decouples_the_classes():
    vs, kap = (4e-3, 1e-3, 0.0), (1e-3, 3e-3, 2e-3)
    cfg = _cfg(19, n_classes=3, frozen=True, vs_class=vs, kappa_class=kap)
    cs = _fields(cfg, 3, 3)
    u = 0.04 * np.random.default_rng(4).standard_normal((3,) + cfg.shape)
    _, c, _, d, _ = _run(cfg, cs, 8, u_in=u)
    for i in range(3):
        one = _cfg(19, frozen=True, vs=vs[i], kappa_c=kap[i])
        _, ci, _, di, _ = _run(one, [cs[i]], 8, u_in=u)
        assert np.array_equal(c[i], ci) and np.array_equal(d[i], di), i


@pytest.mark.parametrize("q", [9, 19])
def test_force_uses_the_total_concentration(q):
    """Linear first-order flux: halving is exact in binary, so two classes
    holding C/2 each with the same parameters reproduce the single-class run
    bit for bit, populations included.  A force that saw only one class, or
    each class with its own buoyancy factor, would change the populations."""
    kw = dict(scheme_c="upwind1")
    one = _cfg(q, vs=3e-3, kappa_c=2e-3, **kw)
    two = _cfg(q, n_classes=2, vs_class=(3e-3, 3e-3), kappa_class=(2e-3, 2e-3), **kw)
    (c0,) = _fields(one, 5)
    f1, c1, _, d1, _ = _run(one, [c0], 15)
    f2, c2, _, d2, _ = _run(two, [0.5 * c0, 0.5 * c0], 15)
    assert np.array_equal(f1, f2)
    for i in range(2):
        assert np.array_equal(c2[i], 0.5 * c1) and np.array_equal(d2[i], 0.5 * d1)


@pytest.mark.parametrize("q", [9, 19])
def test_each_class_keeps_its_own_budget(q):
    """Every class closes sum C_i + sum D_i on its own (walls), and the sums
    report the totals over the classes."""
    vs, kap = (5e-3, 2e-3, 1e-3), (2e-3, 1e-3, 0.0)
    cfg = _cfg(q, n_classes=3, vs_class=vs, kappa_class=kap)
    cs = _fields(cfg, 6, 3)
    f, c, _, d, _ = _run(cfg, cs, 20)
    for i in range(3):
        before = cs[i].sum()
        assert abs(c[i].sum() + d[i].sum() - before) <= 1e-12 * before, i
        assert d[i].sum() > 0
    tot = oracle.sums(cfg, f, c, None, d)
    assert abs(tot[0] - c.sum()) <= 1e-12 * c.sum() and abs(tot[3] - d.sum()) <= 1e-12 * d.sum()
    # faster classes deposit more from the same field
    assert d[0].sum() > d[1].sum() > d[2].sum()


def test_diagnostics_see_the_total():
    cfg = _cfg(9, n_classes=2, vs_class=(1e-3, 1e-3), kappa_class=(0.0, 0.0))
    one = _cfg(9)
    a, b = _fields(cfg, 7, 2)
    c = np.stack([a, b])
    assert np.array_equal(oracle.front_height(cfg, c, 0.7), oracle.front_height(one, a + b, 0.7))
    for plane in (0, 5, 16):
        assert abs(oracle.mass_below(cfg, c, plane) - oracle.mass_below(one, a + b, plane)) <= \
            1e-12 * max(1.0, (a + b).sum())


def test_invalid_class_counts_are_rejected():
    with pytest.raises(ValueError):
        _run(_cfg(9, n_classes=9, vs_class=(0.0,) * 9, kappa_class=(0.0,) * 9), _fields(_cfg(9), 1, 9), 1)
    cfg = _cfg(9, n_classes=2, vs_class=(1e-3, 1e-3), kappa_class=(0.0, 0.0))
    with pytest.raises(ValueError):
        _run(cfg, _fields(cfg, 1, 1), 1)                 # one field for two classes
