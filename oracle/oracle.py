"""ctypes binding of the FP64 CPU oracle (``lbw_oracle.c``).

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline timing).
Arrays are numpy float64, C-contiguous, laid out x fastest; populations are
``f[q, nz, ny, nx]`` (2D: ``f[9, 1, ny, nx]``), velocities ``u[dim, nz, ny, nx]``.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbw_oracle.c")
_LIB = os.path.join(_HERE, "liblbw_oracle.so")
_lib = None


def library_path() -> str:
    return _LIB


def build() -> str:
    """Compile the oracle with gcc: plain -O2, no FMA contraction, OpenMP."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-std=c11", "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


MAX_CLASSES = 8


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("q", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("nz", ctypes.c_int32), ("vert_periodic", ctypes.c_int32),
        ("frozen", ctypes.c_int32), ("scheme_c", ctypes.c_int32),
        ("has_s", ctypes.c_int32), ("shifted", ctypes.c_int32),
        ("n_classes", ctypes.c_int32), ("tau", ctypes.c_double),
        ("body_force", ctypes.c_double * 3), ("u_top", ctypes.c_double * 3),
        ("vs", ctypes.c_double), ("kappa_c", ctypes.c_double), ("gp_c", ctypes.c_double),
        ("kappa_s", ctypes.c_double), ("gp_s", ctypes.c_double),
        ("weno_eps", ctypes.c_double),
        ("vs_class", ctypes.c_double * MAX_CLASSES),
        ("kappa_class", ctypes.c_double * MAX_CLASSES),
        ("vs_s", ctypes.c_double), ("phi_c", ctypes.c_double),
    ]


SCHEMES = {"weno5": 0, "weno3": 1, "upwind1": 2}


@dataclasses.dataclass
class OracleConfig:
    q: int = 9
    nx: int = 64
    ny: int = 128
    nz: int = 1
    vert_periodic: bool = False
    frozen: bool = False
    scheme_c: str = "weno5"
    has_s: bool = False
    shifted: bool = False
    tau: float = 0.6
    body_force: tuple = (0.0, 0.0, 0.0)
    u_top: tuple = (0.0, 0.0, 0.0)
    vs: float = 0.0
    kappa_c: float = 0.0
    gp_c: float = 0.0
    kappa_s: float = 0.0
    gp_s: float = 0.0
    weno_eps: float = 1e-6
    # particle size classes (eq. 11-12): with n_classes >= 2 class i settles
    # at vs_class[i] and diffuses with kappa_class[i]; c is then
    # c[n_classes, nz, ny, nx] and the deposit dep[n_classes, ncol]
    n_classes: int = 1
    vs_class: tuple = ()
    kappa_class: tuple = ()
    # full force and settling (eq. 7, 10, 13; need has_s): settling speed
    # Vs (1 - vs_s S) and S buoyancy on the fluid fraction, (1 - phi_c C)
    vs_s: float = 0.0
    phi_c: float = 0.0

    @property
    def ncls(self) -> int:
        return max(1, self.n_classes)

    @property
    def dim(self) -> int:
        return 2 if self.q == 9 else 3

    @property
    def shape(self) -> tuple:
        return (self.nz, self.ny, self.nx)

    @property
    def ncol(self) -> int:
        return self.nx if self.dim == 2 else self.nx * self.ny

    def _c(self) -> _Cfg:
        c = _Cfg()
        c.q, c.nx, c.ny, c.nz = self.q, self.nx, self.ny, self.nz
        c.vert_periodic = int(self.vert_periodic)
        c.frozen = int(self.frozen)
        c.scheme_c = SCHEMES[self.scheme_c]
        c.has_s = int(self.has_s)
        c.shifted = int(self.shifted)
        c.tau = self.tau
        c.body_force = (ctypes.c_double * 3)(*self.body_force)
        c.u_top = (ctypes.c_double * 3)(*self.u_top)
        c.vs, c.kappa_c, c.gp_c = self.vs, self.kappa_c, self.gp_c
        c.kappa_s, c.gp_s, c.weno_eps = self.kappa_s, self.gp_s, self.weno_eps
        if not 0 <= self.n_classes <= MAX_CLASSES:
            raise ValueError(f"n_classes must lie in [0, {MAX_CLASSES}]")
        c.n_classes = self.n_classes if self.n_classes > 1 else 0
        c.vs_s, c.phi_c = self.vs_s, self.phi_c
        if self.n_classes > 1:
            if len(self.vs_class) != self.n_classes or len(self.kappa_class) != self.n_classes:
                raise ValueError("vs_class and kappa_class need one value per class")
            c.vs_class = (ctypes.c_double * MAX_CLASSES)(*self.vs_class)
            c.kappa_class = (ctypes.c_double * MAX_CLASSES)(*self.kappa_class)
        return c


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        cfgp = ctypes.POINTER(_Cfg)
        lib.orc_lattice.argtypes = [ctypes.c_int32, P, P, P]
        lib.orc_equilibrium.argtypes = [cfgp, P, P, P]
        lib.orc_moments.argtypes = [cfgp, P, P, P, P, P]
        lib.orc_rhs_c.argtypes = [cfgp, P, P, P, P]
        lib.orc_faces_c.argtypes = [cfgp, P, P, P, P, P]
        lib.orc_run.argtypes = [cfgp, P, P, P, P, P, P, ctypes.c_int32]
        lib.orc_sums.argtypes = [cfgp, P, P, P, P, P]
        lib.orc_adjoint_step.argtypes = [cfgp, P, P, P, P, P, ctypes.c_double, P, P, P]
        lib.orc_front_height.argtypes = [cfgp, P, ctypes.c_double, P]
        lib.orc_mass_below.argtypes = [cfgp, P, ctypes.c_int32, P]
        lib.orc_front_psd.argtypes = [cfgp, P, ctypes.c_int32, ctypes.c_int32, P]
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], "float64 C-contiguous expected"
    return a.ctypes.data


def _check(rc, name):
    if rc != 0:
        raise ValueError(f"oracle {name} rejected its arguments (rc={rc})")


def lattice(q: int):
    """(c[q,3] int, w[q] float64, opp[q] int) in the documented order."""
    lib = _load()
    c = np.zeros((q, 3), np.int32)
    w = np.zeros(q, np.float64)
    opp = np.zeros(q, np.int32)
    _check(lib.orc_lattice(q, c.ctypes.data, w.ctypes.data, opp.ctypes.data), "lattice")
    return c.astype(np.int64), w, opp.astype(np.int64)


def equilibrium(cfg: OracleConfig, rho=None, u=None) -> np.ndarray:
    lib = _load()
    f = np.zeros((cfg.q,) + cfg.shape, np.float64)
    c = cfg._c()
    _check(lib.orc_equilibrium(ctypes.byref(c), _ptr(rho), _ptr(u), _ptr(f)), "equilibrium")
    return f


def moments(cfg: OracleConfig, f, c, s=None):
    lib = _load()
    rho = np.zeros(cfg.shape, np.float64)
    u = np.zeros((cfg.dim,) + cfg.shape, np.float64)
    cc = cfg._c()
    _check(lib.orc_moments(ctypes.byref(cc), _ptr(f), _ptr(c), _ptr(s), _ptr(rho), _ptr(u)),
           "moments")
    return rho, u


def rhs_c(cfg: OracleConfig, a, u):
    """Spatial operator L(a) of the C equation and the bottom outflow per column."""
    lib = _load()
    out = np.zeros(cfg.shape, np.float64)
    outflow = np.zeros(cfg.ncol, np.float64)
    cc = cfg._c()
    _check(lib.orc_rhs_c(ctypes.byref(cc), _ptr(a), _ptr(u), _ptr(out), _ptr(outflow)), "rhs_c")
    return out, outflow


def faces_c(cfg: OracleConfig, a, u, s=None):
    """Face fluxes of the C equation: (phi[dim, nz, ny, nx] through the +axis
    face of every node, bottom[ncol] through the bottom wall)."""
    lib = _load()
    a = np.ascontiguousarray(a, np.float64)
    u = np.ascontiguousarray(u, np.float64)
    s = None if s is None else np.ascontiguousarray(s, np.float64)
    phi = np.zeros((cfg.dim,) + cfg.shape, np.float64)
    bottom = np.zeros(cfg.ncol, np.float64)
    cc = cfg._c()
    _check(lib.orc_faces_c(ctypes.byref(cc), _ptr(a), _ptr(u), _ptr(s), _ptr(phi), _ptr(bottom)),
           "faces_c")
    return phi, bottom


def run(cfg: OracleConfig, f, c, s=None, dep=None, u_in=None, nsteps=1, want_u=False):
    """Advance nsteps in place on copies; returns (f, c, s, dep, u_last)."""
    lib = _load()
    f = None if f is None else np.ascontiguousarray(f, np.float64).copy()
    c = np.ascontiguousarray(c, np.float64).copy()
    s = None if s is None else np.ascontiguousarray(s, np.float64).copy()
    dep_shape = (cfg.ncol,) if cfg.ncls == 1 else (cfg.ncls, cfg.ncol)
    dep = np.zeros(dep_shape, np.float64) if dep is None else np.ascontiguousarray(dep, np.float64).copy()
    if c.size != cfg.ncls * cfg.nx * cfg.ny * cfg.nz or dep.size != cfg.ncls * cfg.ncol:
        raise ValueError("c needs n_classes fields and dep n_classes * ncol counters")
    u_in = None if u_in is None else np.ascontiguousarray(u_in, np.float64)
    u_out = np.zeros((cfg.dim,) + cfg.shape, np.float64) if want_u else None
    if f is None:
        if not cfg.frozen:
            raise ValueError("populations required unless the fluid is frozen")
        fp = None
    else:
        fp = _ptr(f)
    cc = cfg._c()
    _check(lib.orc_run(ctypes.byref(cc), fp, _ptr(c), _ptr(s), _ptr(dep), _ptr(u_in),
                       _ptr(u_out), int(nsteps)), "run")
    return f, c, s, dep, u_out


def front_height(cfg: OracleConfig, c, thr: float) -> np.ndarray:
    """Lowest height per bottom column where C reaches thr (see the C header)."""
    lib = _load()
    c = np.ascontiguousarray(c, np.float64)
    out = np.zeros(cfg.ncol, np.float64)
    cc = cfg._c()
    _check(lib.orc_front_height(ctypes.byref(cc), _ptr(c), float(thr), _ptr(out)), "front_height")
    return out


def mass_below(cfg: OracleConfig, c, plane: int) -> float:
    """Sum of C over the cells with vertical index < plane."""
    lib = _load()
    c = np.ascontiguousarray(c, np.float64)
    out = np.zeros(1, np.float64)
    cc = cfg._c()
    _check(lib.orc_mass_below(ctypes.byref(cc), _ptr(c), int(plane), _ptr(out)), "mass_below")
    return float(out[0])


def front_psd(cfg: OracleConfig, h, axis: int = 0, index: int = 0) -> np.ndarray:
    """Power spectral density of a front height along a lateral axis (see
    the C header): Gamma(k), k = 0 .. L/2."""
    lib = _load()
    h = np.ascontiguousarray(h, np.float64).ravel()
    length = (cfg.nx if axis == 0 else cfg.ny)
    out = np.zeros(length // 2 + 1, np.float64)
    cc = cfg._c()
    _check(lib.orc_front_psd(ctypes.byref(cc), _ptr(h), int(axis), int(index), _ptr(out)),
           "front_psd")
    return out


def sums(cfg: OracleConfig, f, c, s=None, dep=None):
    lib = _load()
    out = np.zeros(4, np.float64)
    cc = cfg._c()
    _check(lib.orc_sums(ctypes.byref(cc), _ptr(f), _ptr(c), _ptr(s), _ptr(dep), _ptr(out)), "sums")
    return out


def adjoint_step(cfg: OracleConfig, f_n, c_n, fbar_next, cbar_next, dep_bar=1.0, u_in=None):
    """(fbar, cbar, vs_bar) of one step (WENO5, no S); see lbw_oracle.h."""
    lib = _load()
    cbar = np.zeros(cfg.shape, np.float64)
    fbar = None if cfg.frozen else np.zeros((cfg.q,) + cfg.shape, np.float64)
    vsb = np.zeros(1, np.float64)
    cc = cfg._c()
    _check(lib.orc_adjoint_step(ctypes.byref(cc), _ptr(None if f_n is None else np.ascontiguousarray(f_n)),
                                _ptr(np.ascontiguousarray(c_n)),
                                _ptr(None if u_in is None else np.ascontiguousarray(u_in)),
                                _ptr(None if fbar_next is None else np.ascontiguousarray(fbar_next)),
                                _ptr(np.ascontiguousarray(cbar_next)), float(dep_bar),
                                _ptr(fbar), _ptr(cbar), _ptr(vsb)), "adjoint_step")
    return fbar, cbar, float(vsb[0])
