"""Pins of the oracle's in-situ diagnostics: the front of the particle field
H (lowest height where C reaches a threshold, per column; the paper's front
at phi0 / 2 used for its growth-rate analysis) and the particle mass below a
horizontal plane (whose change over a time interval is the plane's mass
flux J = dm / (A dt))."""
import numpy as np
import pytest

import oracle


def _cfg(q=9, nx=16, ny=40, nz=1):
    return oracle.OracleConfig(q=q, nx=nx, ny=ny, nz=nz)


def _column_field(cfg, prof):
    """Field with the same vertical profile in every column."""
    shape = cfg.shape
    if cfg.dim == 2:
        return np.broadcast_to(prof[None, :, None], shape).copy()
    return np.broadcast_to(prof[:, None, None], shape).copy()


@pytest.mark.parametrize("q", [9, 19])
def test_front_of_a_linear_profile_is_exact(q):
    cfg = _cfg(q, nx=6, ny=30) if q == 9 else _cfg(q, nx=4, ny=3, nz=30)
    nv = 30
    prof = np.arange(nv) / (nv - 1)            # C = v / (nv - 1) at cell centres
    c = _column_field(cfg, prof)
    for thr in (0.1, 0.5, 0.77):
        h = oracle.front_height(cfg, c, thr)
        # the crossing is where v / (nv - 1) = thr, height v + 1/2 from the wall
        assert np.allclose(h, thr * (nv - 1) + 0.5, rtol=0, atol=1e-12)


def test_front_of_a_step_is_the_interface():
    cfg = _cfg(nx=5, ny=20)
    prof = np.where(np.arange(20) >= 12, 2.0, 0.0)   # C0 = 2 from cell 12 up
    h = oracle.front_height(cfg, _column_field(cfg, prof), 1.0)
    assert np.all(h == 12.0)                          # the face between cells 11 and 12


def test_front_edge_cases():
    cfg = _cfg(nx=3, ny=10)
    assert np.all(oracle.front_height(cfg, np.zeros(cfg.shape), 0.5) == 10.0)   # no particles
    assert np.all(oracle.front_height(cfg, np.ones(cfg.shape), 0.5) == 0.0)     # reached the floor


def test_front_follows_fingers_and_its_spectrum_peaks_at_the_mode():
    """A displaced interface C0 (1 + tanh((y - y0 - eta cos(k x)) / w)) / 2:
    the front at C0 / 2 is y0 + 1/2 + eta cos(k x) up to the interpolation
    error of a tanh between cells, and its power spectral density
    |H~(k)|^2 / (k_S L_S) peaks at the displacement's wavenumber with the
    amplitude eta."""
    nx, ny, y0, eta, w = 64, 80, 39.5, 3.0, 1.5
    cfg = _cfg(nx=nx, ny=ny)
    k = 2 * np.pi / nx
    y = np.arange(ny)[:, None] + 0.0
    x = np.arange(nx)[None, :] + 0.0
    c = (0.5 * (1 + np.tanh((y - y0 - eta * np.cos(3 * k * x)) / w)))[None]
    h = oracle.front_height(cfg, c, 0.5)
    assert np.max(np.abs(h - (y0 + 0.5 + eta * np.cos(3 * k * x[0])))) < 0.05
    spec = np.abs(np.fft.rfft(h)) ** 2 / (nx * 1.0)     # k_S = 1 sample per cell, L_S = nx
    assert int(np.argmax(spec[1:])) + 1 == 3
    amp = 2 * np.abs(np.fft.rfft(h)[3]) / nx
    assert abs(amp - eta) < 0.05


@pytest.mark.parametrize("q", [9, 19])
def test_mass_below_a_plane(q):
    cfg = _cfg(q, nx=7, ny=24) if q == 9 else _cfg(q, nx=3, ny=5, nz=24)
    rng = np.random.default_rng(11)
    c = rng.uniform(0, 1, cfg.shape)
    ncol = cfg.ncol
    flat = c.reshape(-1)
    for plane in (0, 1, 9, 24):
        assert abs(oracle.mass_below(cfg, c, plane) - flat[: plane * ncol].sum()) < 1e-12
    # a closed budget: the flux through a plane is the change of the mass below it
    prof = np.where(np.arange(24) >= 10, 1.0, 0.0)
    step = _column_field(cfg, prof)
    assert oracle.mass_below(cfg, step, 10) == 0.0
    assert oracle.mass_below(cfg, step, 15) == 5.0 * ncol
    with pytest.raises(ValueError):
        oracle.mass_below(cfg, c, 25)


def test_psd_of_a_cosine_is_two_closed_form_bins():
    """H_j = B + A cos(2 pi m j / L): Gamma(0) = B^2 L, Gamma(m) = A^2 L / 4,
    every other bin zero (the transform of a single mode)."""
    nx, m, a, b = 48, 5, 2.5, 30.0
    cfg = _cfg(nx=nx, ny=40)
    h = b + a * np.cos(2 * np.pi * m * np.arange(nx) / nx)
    g = oracle.front_psd(cfg, h)
    assert g.shape == (nx // 2 + 1,)
    want = np.zeros(nx // 2 + 1)
    want[0] = b * b * nx
    want[m] = a * a * nx / 4
    assert np.max(np.abs(g - want)) < 1e-9 * want[0]


@pytest.mark.parametrize("nx", [1, 2, 31, 64])
def test_psd_parseval_and_fft(nx):
    """Parseval: sum over the full spectrum of |H~|^2 / L (the one-sided bins
    counted twice except k = 0 and, for even L, k = L/2) equals sum H_j^2; and
    every bin equals |rfft(H)|^2 / L."""
    cfg = _cfg(nx=nx, ny=40)
    h = np.random.default_rng(nx).uniform(0, 40, nx)
    g = oracle.front_psd(cfg, h)
    w = np.full(len(g), 2.0)
    w[0] = 1.0
    if nx % 2 == 0:
        w[-1] = 1.0
    assert abs(np.sum(w * g) - np.sum(h * h)) <= 1e-12 * np.sum(h * h)
    assert np.allclose(g, np.abs(np.fft.rfft(h)) ** 2 / nx, rtol=1e-11, atol=1e-11 * np.sum(h * h))


def test_psd_slices_of_a_3d_front():
    """3D: axis 0 transforms the row at y = index, axis 1 the row at x =
    index; index -1 averages over every row."""
    nx, ny = 12, 9
    cfg = _cfg(q=19, nx=nx, ny=ny, nz=8)
    h = np.random.default_rng(5).uniform(0, 8, (ny, nx))
    ref = lambda rows: np.abs(np.fft.rfft(rows, axis=-1)) ** 2 / rows.shape[-1]
    for y in (0, 4, ny - 1):
        assert np.allclose(oracle.front_psd(cfg, h, 0, y), ref(h[y]), rtol=1e-11, atol=1e-9)
    for x in (0, 7):
        assert np.allclose(oracle.front_psd(cfg, h, 1, x), ref(h[:, x]), rtol=1e-11, atol=1e-9)
    assert np.allclose(oracle.front_psd(cfg, h, 0, -1), ref(h).mean(axis=0), rtol=1e-11, atol=1e-9)
    assert np.allclose(oracle.front_psd(cfg, h, 1, -1), ref(h.T).mean(axis=0), rtol=1e-11, atol=1e-9)
    for axis, index in ((2, 0), (0, ny), (1, nx), (0, -2)):
        with pytest.raises(ValueError):
            oracle.front_psd(cfg, h, axis, index)
    with pytest.raises(ValueError):
        oracle.front_psd(_cfg(nx=8, ny=40), np.zeros(8), 1, 0)     # 2D has one lateral axis
