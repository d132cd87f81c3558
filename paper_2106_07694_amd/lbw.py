"""ctypes binding of liblbw.so (include/lbw.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch provides device memory (tensors) and the HIP stream.  The
library must have been built (``paper_2106_07694_amd.build``); there is no
fallback of any kind -- a missing library or GPU raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbw.so")

D2Q9, D3Q19 = 9, 19
FP64, FP32_SHIFTED, FP64_SHIFTED = 0, 1, 2
FLUID_LBM, FLUID_FROZEN = 0, 1
WENO5, WENO3, UPWIND1 = 0, 1, 2
FIELD_F, FIELD_C, FIELD_S, FIELD_U, FIELD_DEPOSIT, FIELD_STAGE1, FIELD_STAGE2, FIELD_RHO = range(8)
MASS_C, MASS_S, MASS_FLUID, DEPOSIT = 0, 1, 2, 3
ERR_INVAL, ERR_UNSUPPORTED, ERR_HIP, ERR_NONFINITE = -1, -2, -3, -4

PRECISIONS = {"fp64": FP64, "fp32_shifted": FP32_SHIFTED, "fp64_shifted": FP64_SHIFTED}
SCHEMES = {"weno5": WENO5, "weno3": WENO3, "upwind1": UPWIND1}

EXPORTED = ("lbw_version", "lbw_last_error", "lbw_scratch_bytes", "lbw_create", "lbw_destroy",
            "lbw_set_launch", "lbw_get_launch", "lbw_init_equilibrium", "lbw_step",
            "lbw_steps_done", "lbw_export", "lbw_import", "lbw_rebind", "lbw_reduce", "lbw_timing_begin",
            "lbw_timing_end", "lbw_adjoint_work_bytes", "lbw_adjoint_step", "lbw_mass_below",
            "lbw_front_height", "lbw_front_psd", "lbw_reduce_class", "lbw_replay",
            "lbw_reduce_static")


class LbwError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbw error {code}: {msg}")
        self.code = code


MAX_CLASSES = 8


class CConfig(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("vert_periodic", ctypes.c_int32), ("fluid_mode", ctypes.c_int32),
        ("scheme_c", ctypes.c_int32), ("has_s", ctypes.c_int32), ("n_classes", ctypes.c_int32),
        ("tau", ctypes.c_double), ("body_force", ctypes.c_double * 3),
        ("u_top", ctypes.c_double * 3), ("vs", ctypes.c_double),
        ("kappa_c", ctypes.c_double), ("gp_c", ctypes.c_double),
        ("kappa_s", ctypes.c_double), ("gp_s", ctypes.c_double),
        ("weno_eps", ctypes.c_double),
        ("vs_class", ctypes.c_double * MAX_CLASSES),
        ("kappa_class", ctypes.c_double * MAX_CLASSES),
        ("vs_s", ctypes.c_double), ("phi_c", ctypes.c_double),
    ]


class CBuffers(ctypes.Structure):
    _fields_ = [
        ("f", ctypes.c_void_p), ("c", ctypes.c_void_p), ("c_s1", ctypes.c_void_p),
        ("c_s2", ctypes.c_void_p), ("s", ctypes.c_void_p), ("s_tmp", ctypes.c_void_p),
        ("u", ctypes.c_void_p), ("deposit", ctypes.c_void_p), ("scratch", ctypes.c_void_p),
        ("scratch_bytes", ctypes.c_size_t),
    ]


class CLaunch(ctypes.Structure):
    _fields_ = [("lbm_block", ctypes.c_int32), ("tile_x", ctypes.c_int32),
                ("tile_y", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("tile_rows", ctypes.c_int32)]


_lib = None


def load() -> ctypes.CDLL:
    """Load liblbw.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2106_07694_amd.build` (no fallback path exists)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32 = ctypes.c_void_p, ctypes.c_int32
    lib.lbw_version.restype = ctypes.c_int
    lib.lbw_last_error.restype = ctypes.c_char_p
    lib.lbw_scratch_bytes.argtypes = [P, I32, ctypes.POINTER(ctypes.c_size_t)]
    lib.lbw_create.argtypes = [P, P, I32, P, ctypes.POINTER(ctypes.c_void_p)]
    lib.lbw_destroy.argtypes = [P]
    lib.lbw_destroy.restype = None
    lib.lbw_set_launch.argtypes = [P, ctypes.POINTER(CLaunch)]
    lib.lbw_get_launch.argtypes = [P, ctypes.POINTER(CLaunch)]
    lib.lbw_init_equilibrium.argtypes = [P, I32, P, P]
    lib.lbw_step.argtypes = [P, I32]
    lib.lbw_steps_done.argtypes = [P, ctypes.POINTER(ctypes.c_int64)]
    lib.lbw_export.argtypes = [P, I32, I32, P]
    lib.lbw_import.argtypes = [P, I32, I32, P]
    lib.lbw_rebind.argtypes = [P, I32, I32, P]
    lib.lbw_replay.argtypes = [P, I32, I32, P, P, P, P, P]
    lib.lbw_reduce.argtypes = [P, I32, ctypes.POINTER(ctypes.c_double)]
    lib.lbw_reduce_static.argtypes = [P, I32, ctypes.POINTER(ctypes.c_double)]
    lib.lbw_mass_below.argtypes = [P, I32, ctypes.POINTER(ctypes.c_double)]
    lib.lbw_reduce_class.argtypes = [P, I32, I32, ctypes.POINTER(ctypes.c_double)]
    lib.lbw_front_height.argtypes = [P, I32, ctypes.c_double, P]
    lib.lbw_front_psd.argtypes = [P, I32, P, I32, I32, P]
    lib.lbw_adjoint_work_bytes.argtypes = [P, I32, ctypes.POINTER(ctypes.c_size_t)]
    lib.lbw_adjoint_step.argtypes = [P, I32, P, P, P, P, P, P, P, P, ctypes.c_double, P, P, P, P,
                                     ctypes.c_size_t]
    lib.lbw_timing_begin.argtypes = [P]
    lib.lbw_timing_end.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    for name in EXPORTED:
        getattr(lib, name)
    _lib = lib
    return lib


def check(rc: int) -> None:
    if rc != 0:
        raise LbwError(rc, load().lbw_last_error().decode())


@dataclasses.dataclass
class RunConfig:
    """Mirror of lbw_config with Python defaults."""
    lattice: int = D2Q9
    precision: str = "fp64"
    nx: int = 64
    ny: int = 128
    nz: int = 1
    vert_periodic: bool = False
    fluid_mode: int = FLUID_LBM
    scheme_c: str = "weno5"
    has_s: bool = False
    tau: float = 0.6
    body_force: tuple = (0.0, 0.0, 0.0)
    u_top: tuple = (0.0, 0.0, 0.0)
    vs: float = 0.0
    kappa_c: float = 0.0
    gp_c: float = 0.0
    kappa_s: float = 0.0
    gp_s: float = 0.0
    weno_eps: float = 1e-6
    # particle size classes (eq. 11-12): with n_classes >= 2, class i settles
    # at vs_class[i] and diffuses with kappa_class[i] (vs and kappa_c stay 0);
    # C is then c[n_classes, nz, ny, nx] and the deposit dep[n_classes, ncol]
    n_classes: int = 1
    vs_class: tuple = ()
    kappa_class: tuple = ()
    # the paper's full force and settling (need has_s): settling speed
    # Vs (1 - vs_s S) (eq. 13) and S buoyancy on the fluid fraction
    # -gp_s S (1 - phi_c C) (eq. 10)
    vs_s: float = 0.0
    phi_c: float = 0.0

    @property
    def ncls(self) -> int:
        return max(1, self.n_classes)

    @property
    def c_shape(self) -> tuple:
        return self.shape if self.ncls == 1 else (self.ncls,) + self.shape

    @property
    def deposit_shape(self) -> tuple:
        return (self.ncol,) if self.ncls == 1 else (self.ncls, self.ncol)

    @property
    def dim(self) -> int:
        return 2 if self.lattice == D2Q9 else 3

    @property
    def shape(self) -> tuple:
        return (self.nz, self.ny, self.nx)

    @property
    def ncol(self) -> int:
        return self.nx if self.dim == 2 else self.nx * self.ny

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    def to_c(self) -> CConfig:
        c = CConfig()
        c.lattice, c.precision = self.lattice, PRECISIONS[self.precision]
        c.nx, c.ny, c.nz = self.nx, self.ny, self.nz
        c.vert_periodic, c.fluid_mode = int(self.vert_periodic), int(self.fluid_mode)
        c.scheme_c, c.has_s = SCHEMES[self.scheme_c], int(self.has_s)
        if not 0 <= self.n_classes <= MAX_CLASSES:
            raise ValueError(f"n_classes must lie in [0, {MAX_CLASSES}]")
        c.n_classes = self.n_classes if self.n_classes > 1 else 0
        c.vs_s, c.phi_c = self.vs_s, self.phi_c
        if self.n_classes > 1:
            if len(self.vs_class) != self.n_classes or len(self.kappa_class) != self.n_classes:
                raise ValueError("vs_class and kappa_class need one value per class")
            c.vs_class = (ctypes.c_double * MAX_CLASSES)(*self.vs_class)
            c.kappa_class = (ctypes.c_double * MAX_CLASSES)(*self.kappa_class)
        c.tau = self.tau
        c.body_force = (ctypes.c_double * 3)(*self.body_force)
        c.u_top = (ctypes.c_double * 3)(*self.u_top)
        c.vs, c.kappa_c, c.gp_c = self.vs, self.kappa_c, self.gp_c
        c.kappa_s, c.gp_s, c.weno_eps = self.kappa_s, self.gp_s, self.weno_eps
        return c

    @staticmethod
    def from_workload(wl, **over) -> "RunConfig":
        kw = dict(lattice=wl.q, precision=wl.precision, nx=wl.nx, ny=wl.ny, nz=wl.nz,
                  tau=wl.tau, vs=wl.vs, kappa_c=wl.kappa_c, gp_c=wl.gp_c, has_s=wl.has_s,
                  kappa_s=wl.kappa_s, gp_s=wl.gp_s, n_classes=wl.n_classes,
                  vs_class=tuple(wl.vs_class), kappa_class=tuple(wl.kappa_class),
                  vs_s=wl.vs_s, phi_c=wl.phi_c)
        kw.update(over)
        return RunConfig(**kw)


class Solver:
    """A batch of runs bound to torch-owned device buffers and a HIP stream."""

    def __init__(self, cfgs, device="cuda", stream=None, scratch=True):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("liblbw needs a ROCm GPU; none is visible")
        lib = load()
        if isinstance(cfgs, RunConfig):
            cfgs = [cfgs]
        self.cfgs = list(cfgs)
        self.nbatch = len(self.cfgs)
        self.device = torch.device(device)
        c0 = self.cfgs[0]
        self.dtype = torch.float32 if c0.precision == "fp32_shifted" else torch.float64
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._torch = torch
        self._ccfg = (CConfig * self.nbatch)(*[c.to_c() for c in self.cfgs])
        nbytes = ctypes.c_size_t(0)
        check(lib.lbw_scratch_bytes(self._ccfg, self.nbatch, ctypes.byref(nbytes)))
        if not scratch:
            if self.nbatch > 1:
                raise ValueError("a batch needs its scratch (work lists)")
            nbytes = ctypes.c_size_t(0)
        self.tensors = []
        cbufs = []
        torch.cuda.current_stream(self.device).synchronize()
        with torch.cuda.stream(self.stream):
            self._alloc(cbufs, nbytes.value)
        self.stream.synchronize()
        self._cbuf = (CBuffers * self.nbatch)(*cbufs)
        h = ctypes.c_void_p()
        check(lib.lbw_create(self._ccfg, self._cbuf, self.nbatch,
                             ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self._lib = lib

    def _alloc(self, cbufs, scratch_bytes):
        torch = self._torch
        for i, c in enumerate(self.cfgs):
            z = lambda *shape, dt=self.dtype: torch.zeros(shape, dtype=dt, device=self.device)
            t = {
                "f": z(c.lattice, *c.shape) if c.fluid_mode == FLUID_LBM else None,
                "c": z(*c.c_shape), "c_s1": z(*c.c_shape), "c_s2": z(*c.c_shape),
                "s": z(*c.shape) if c.has_s else None,
                "s_tmp": z(*c.shape) if c.has_s else None,
                "u": z(c.dim, *c.shape),
                "deposit": z(*c.deposit_shape, dt=torch.float64),
                "scratch": (z((scratch_bytes + 7) // 8, dt=torch.float64)
                            if i == 0 and scratch_bytes else None),
            }
            self.tensors.append(t)
            b = CBuffers()
            for k in ("f", "c", "c_s1", "c_s2", "s", "s_tmp", "u", "deposit", "scratch"):
                setattr(b, k, t[k].data_ptr() if t[k] is not None else None)
            b.scratch_bytes = scratch_bytes if i == 0 else 0
            cbufs.append(b)

    # -- lifetime --------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            self._lib.lbw_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- state -----------------------------------------------------------
    def _dev(self, x, dtype=None):
        """Device copy of x made on the solver's stream (and finished)."""
        torch = self._torch
        dt = self.dtype if dtype is None else dtype
        if isinstance(x, np.ndarray):
            x = torch.from_numpy(np.ascontiguousarray(x))
        with torch.cuda.stream(self.stream):
            y = x.to(device=self.device, dtype=dt).contiguous()
        self.stream.synchronize()
        return y

    def _shape(self, name, run):
        c = self.cfgs[run]
        return {"f": (c.lattice, *c.shape), "c": c.c_shape, "s": c.shape, "u": (c.dim, *c.shape),
                "deposit": c.deposit_shape, "stage1": c.c_shape, "stage2": c.c_shape,
                "rho": c.shape}[name]

    def _checked(self, name, t, run):
        """t as a device buffer of field `name`: the library reads or writes
        exactly that field's bytes through the pointer, so a tensor of another
        size or element type, not contiguous or not on the device is refused."""
        import torch
        want = torch.float64 if name == "deposit" else self.dtype
        n = int(np.prod(self._shape(name, run)))
        if t.dtype != want:
            raise ValueError(f"{name}: element type {t.dtype}, the run stores {want}")
        if t.numel() != n:
            raise ValueError(f"{name}: {t.numel()} values, the field holds {n}")
        if not t.is_contiguous():
            raise ValueError(f"{name}: the tensor is not contiguous")
        if t.device.type != "cuda":
            raise ValueError(f"{name}: the tensor is on {t.device}, not on the device")
        return t

    def init_equilibrium(self, run=0, rho=None, u=None):
        keep = [self._checked("rho", self._dev(rho), run) if rho is not None else None,
                self._checked("u", self._dev(u), run) if u is not None else None]
        check(self._lib.lbw_init_equilibrium(
            self._h, run, keep[0].data_ptr() if keep[0] is not None else None,
            keep[1].data_ptr() if keep[1] is not None else None))
        self.stream.synchronize()

    def set_field(self, name, value, run=0):
        fid = self._FIELDS[name]
        import torch
        dt = torch.float64 if name == "deposit" else None
        src = self._checked(name, self._dev(value, dt), run)
        check(self._lib.lbw_import(self._h, run, fid, src.data_ptr()))
        self.stream.synchronize()

    def field(self, name, run=0):
        """Canonical copy of a field as a new device tensor."""
        import torch
        c = self.cfgs[run]
        shapes = {"f": (c.lattice, *c.shape), "c": c.c_shape, "s": c.shape, "u": (c.dim, *c.shape),
                  "deposit": c.deposit_shape, "stage1": c.c_shape, "stage2": c.c_shape}
        fid = self._FIELDS[name]
        dt = torch.float64 if name == "deposit" else self.dtype
        with torch.cuda.stream(self.stream):
            out = torch.empty(shapes[name], dtype=dt, device=self.device)
        check(self._lib.lbw_export(self._h, run, fid, out.data_ptr()))
        self.stream.synchronize()
        return out

    _FIELDS = {"f": FIELD_F, "c": FIELD_C, "s": FIELD_S, "u": FIELD_U, "deposit": FIELD_DEPOSIT,
               "stage1": FIELD_STAGE1, "stage2": FIELD_STAGE2, "rho": FIELD_RHO}

    def export_into(self, name, out, run=0):
        """Canonical copy of a field into an existing device tensor, ordered on
        the solver's stream (no host synchronisation)."""
        check(self._lib.lbw_export(self._h, run, self._FIELDS[name],
                                   self._checked(name, out, run).data_ptr()))

    def import_from(self, name, src, run=0):
        """Overwrite a field from a device tensor written on the solver's
        stream (no host synchronisation)."""
        check(self._lib.lbw_import(self._h, run, self._FIELDS[name],
                                   self._checked(name, src, run).data_ptr()))

    def rebind(self, name, out=None, run=0):
        """Make the next steps write the per-step field `name` ("u", "rho",
        "stage1" or "stage2") into the device tensor `out` (None: the
        solver's own buffer again; for "rho", no density is written).  The
        tensor is kept alive while bound."""
        if not hasattr(self, "_bound"):
            self._bound = {}
        check(self._lib.lbw_rebind(self._h, run, self._FIELDS[name],
                                   self._checked(name, out, run).data_ptr() if out is not None else None))
        if out is None:
            self._bound.pop((run, name), None)
        else:
            self._bound[(run, name)] = out

    def step(self, n=1):
        check(self._lib.lbw_step(self._h, int(n)))

    def replay(self, c_out, a1_out, a2_out, u_out=None, rho_out=None, run=0):
        """len(c_out) steps, keeping per step C before it and the step's
        velocity, density and first two RK stages (see lbw_replay); the lists
        hold device tensors, kept alive by the caller until the work has run."""
        n = len(c_out)
        arr = lambda ts: (ctypes.c_void_p * n)(*[t.data_ptr() for t in ts]) if ts is not None else None
        check(self._lib.lbw_replay(self._h, run, n, arr(c_out), arr(u_out), arr(rho_out), arr(a1_out),
                                   arr(a2_out)))

    def steps_done(self) -> int:
        v = ctypes.c_int64(0)
        check(self._lib.lbw_steps_done(self._h, ctypes.byref(v)))
        return v.value

    def set_launch(self, lbm_block=0, tile_x=0, tile_y=0, variant=0, graph=0, tile_rows=0):
        lc = CLaunch(lbm_block, tile_x, tile_y, variant, graph, 0, tile_rows)
        check(self._lib.lbw_set_launch(self._h, ctypes.byref(lc)))

    def get_launch(self) -> dict:
        lc = CLaunch()
        check(self._lib.lbw_get_launch(self._h, ctypes.byref(lc)))
        return {"lbm_block": lc.lbm_block, "tile_x": lc.tile_x, "tile_y": lc.tile_y,
                "variant": lc.variant, "graph": lc.graph,
                "tile_rows": lc.tile_rows}

    def reduce(self, what) -> np.ndarray:
        out = (ctypes.c_double * self.nbatch)()
        check(self._lib.lbw_reduce(self._h, int(what), out))
        return np.array(out[:], dtype=np.float64)

    def reduce_static(self, what) -> np.ndarray:
        """The sums of reduce(), computed through the library's own static
        device scratch (lbw_reduce_static: no caller scratch needed)."""
        out = (ctypes.c_double * self.nbatch)()
        check(self._lib.lbw_reduce_static(self._h, int(what), out))
        return np.array(out[:], dtype=np.float64)

    def reduce_class(self, what, cls: int) -> np.ndarray:
        """MASS_C or DEPOSIT of one particle size class, per run (FP64)."""
        out = (ctypes.c_double * self.nbatch)()
        check(self._lib.lbw_reduce_class(self._h, int(what), int(cls), out))
        return np.array(out[:], dtype=np.float64)

    def mass_below(self, plane: int) -> np.ndarray:
        """Sum of C below vertical plane index `plane`, per run (FP64)."""
        out = (ctypes.c_double * self.nbatch)()
        check(self._lib.lbw_mass_below(self._h, int(plane), out))
        return np.array(out[:], dtype=np.float64)

    def front_psd(self, height, axis: int = 0, index: int = 0, run: int = 0, out=None):
        """Power spectral density of a front height (the device tensor
        front_height returns) along a lateral axis: an FP64 device tensor of
        L/2 + 1 bins; index -1 averages over every row along that axis."""
        import torch

        cfg = self.cfgs[run]
        if height.dtype != torch.float64 or not height.is_contiguous() or height.numel() != cfg.ncol:
            raise ValueError("height must be a contiguous float64 tensor of ncol values")
        length = cfg.nx if axis == 0 else cfg.ny
        if out is None:
            with torch.cuda.stream(self.stream):
                out = torch.empty(length // 2 + 1, dtype=torch.float64, device=self.device)
        if out.dtype != torch.float64 or not out.is_contiguous() or out.numel() != length // 2 + 1:
            raise ValueError("out must be a contiguous float64 tensor of L/2 + 1 values")
        check(self._lib.lbw_front_psd(self._h, int(run), ctypes.c_void_p(height.data_ptr()),
                                      int(axis), int(index), ctypes.c_void_p(out.data_ptr())))
        return out

    def front_height(self, threshold: float, run: int = 0, out=None):
        """Front height per bottom column as an FP64 device tensor of the
        lateral shape (written on the solver's stream)."""
        import torch

        cfg = self.cfgs[run]
        lateral = (cfg.nx,) if cfg.dim == 2 else (cfg.ny, cfg.nx)
        if out is None:
            with torch.cuda.stream(self.stream):
                out = torch.empty(lateral, dtype=torch.float64, device=self.device)
        if out.dtype != torch.float64 or not out.is_contiguous() or out.numel() != int(np.prod(lateral)):
            raise ValueError("out must be a contiguous float64 tensor of the lateral shape")
        check(self._lib.lbw_front_height(self._h, int(run), float(threshold),
                                         ctypes.c_void_p(out.data_ptr())))
        return out

    def timing_begin(self):
        check(self._lib.lbw_timing_begin(self._h))

    def timing_end(self) -> dict:
        ms = (ctypes.c_double * 2)()
        n = ctypes.c_int64(0)
        check(self._lib.lbw_timing_end(self._h, ms, ctypes.byref(n)))
        return {"collide_stream_ms": ms[0], "transport_ms": ms[1], "steps": n.value}

    def adjoint_workspace(self, run=0):
        """Zero-filled device workspace tensor for adjoint_step (torch-owned)."""
        n = ctypes.c_size_t(0)
        check(self._lib.lbw_adjoint_work_bytes(self._h, run, ctypes.byref(n)))
        with self._torch.cuda.stream(self.stream):
            return self._torch.zeros((n.value + 7) // 8, dtype=self._torch.float64, device=self.device)

    def adjoint_step(self, f_n, c_n, fbar_next, cbar_next, dep_bar, fbar, cbar, vs_bar, work, run=0,
                     u_n=None, a1_n=None, a2_n=None, rho_n=None):
        """One reverse step (device tensors; see lbw_adjoint_step).  vs_bar
        (or None) receives the accumulated dJ/dVs when given."""
        ptr = lambda t: t.data_ptr() if t is not None else None
        check(self._lib.lbw_adjoint_step(self._h, run, ptr(f_n), ptr(c_n), ptr(u_n), ptr(rho_n),
                                         ptr(a1_n),
                                         ptr(a2_n), ptr(fbar_next), ptr(cbar_next), float(dep_bar),
                                         ptr(fbar), ptr(cbar), ptr(vs_bar), ptr(work),
                                         work.numel() * 8))

    def setup_workload(self, wl, run=0, seed=None):
        """Initial state of a seeded workload: two-layer scalars, fluid at rest."""
        from . import workloads
        c, s = workloads.initial_scalars(wl, seed)
        self.set_field("c", c, run)
        if s is not None:
            self.set_field("s", s, run)
        if self.cfgs[run].fluid_mode == FLUID_LBM:
            self.init_equilibrium(run)
