"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function the public header declares, and rejects invalid runs."""
import ctypes
import os
import re

import pytest

from paper_2106_07694_amd import lbw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "lbw.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\s*\*)\s*\*?\s*(lbw_\w+)\s*\(",
                                 text, re.M)))


def test_every_declared_symbol_is_exported():
    lib = lbw.load()
    names = _declared()
    assert "lbw_step" in names and "lbw_create" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(lbw.EXPORTED)


def test_version():
    assert lbw.load().lbw_version() == 3


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of lbw_config, lbw_buffers and lbw_launch have the
    header's size and field offsets (checked by a C program built from the
    header alone)."""
    import os
    import subprocess

    structs = {"lbw_config": lbw.CConfig, "lbw_buffers": lbw.CBuffers, "lbw_launch": lbw.CLaunch}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lbw.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", inc, "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def _fake_buffers(cfg: lbw.RunConfig) -> lbw.CBuffers:
    b = lbw.CBuffers()
    for i, k in enumerate(("f", "c", "c_s1", "c_s2", "s", "s_tmp", "u", "deposit", "scratch")):
        setattr(b, k, 0x10000 * (i + 1))   # never dereferenced: create only validates
    b.scratch_bytes = 1 << 20
    return b


def _create(cfgs):
    lib = lbw.load()
    arr = (lbw.CConfig * len(cfgs))(*[c.to_c() for c in cfgs])
    bufs = (lbw.CBuffers * len(cfgs))(*[_fake_buffers(c) for c in cfgs])
    h = ctypes.c_void_p()
    rc = lib.lbw_create(arr, bufs, len(cfgs), None, ctypes.byref(h))
    msg = lib.lbw_last_error().decode()
    if h:
        lib.lbw_destroy(h)
    return rc, msg


def test_valid_config_creates():
    assert _create([lbw.RunConfig()])[0] == 0
    assert _create([lbw.RunConfig(lattice=19, nx=8, ny=8, nz=16, precision="fp32_shifted")])[0] == 0


@pytest.mark.parametrize("bad,frag", [
    (dict(tau=0.5), "tau"),
    (dict(tau=0.3), "tau"),
    (dict(ny=5), "vertical"),
    (dict(nz=2), "nz"),
    (dict(lattice=27), "lattice"),
    (dict(vs=-1e-3), "vs"),
    (dict(vs=1.5), "vs"),
    (dict(kappa_c=0.3), "kappa_c"),
    (dict(kappa_c=-1.0), "kappa_c"),
    (dict(weno_eps=0.0), "weno_eps"),
    (dict(u_top=(2.0, 0, 0)), "lid"),
    (dict(nx=0), "grid"),
    (dict(lattice=19, nx=32768, ny=16384, nz=6), "horizontal plane"),
    (dict(lattice=19, nx=4096, ny=1024, nz=1025), "grid too large"),
    (dict(nx=65536, ny=65536), "grid too large"),
    (dict(n_classes=2, vs=1e-3, vs_class=(1e-3, 2e-3), kappa_class=(0.0, 0.0)), "vs_class"),
    (dict(n_classes=2, vs_class=(1e-3, 2.0), kappa_class=(0.0, 0.0)), "vs_class[1]"),
    (dict(n_classes=3, vs_class=(0.0,) * 3, kappa_class=(0.0, 0.0, 0.3)), "kappa_class[2]"),
    (dict(vs_s=0.1), "has_s"),
    (dict(phi_c=0.1), "has_s"),
    (dict(has_s=True, vs_s=float("inf")), "finite"),
])
def test_invalid_configs_rejected(bad, frag):
    rc, msg = _create([lbw.RunConfig(**bad)])
    assert rc == lbw.ERR_INVAL and frag in msg, (rc, msg)


def test_bad_precision_and_scheme_codes():
    lib = lbw.load()
    c = lbw.RunConfig().to_c()
    c.precision = 7
    b = _fake_buffers(lbw.RunConfig())
    h = ctypes.c_void_p()
    assert lib.lbw_create(ctypes.byref(c), ctypes.byref(b), 1, None, ctypes.byref(h)) == lbw.ERR_INVAL
    assert not h
    c = lbw.RunConfig().to_c()
    c.n_classes = lbw.MAX_CLASSES + 1
    assert lib.lbw_create(ctypes.byref(c), ctypes.byref(b), 1, None, ctypes.byref(h)) == lbw.ERR_INVAL
    c.n_classes = -1
    assert lib.lbw_create(ctypes.byref(c), ctypes.byref(b), 1, None, ctypes.byref(h)) == lbw.ERR_INVAL


def test_missing_buffers_rejected():
    lib = lbw.load()
    cfg = lbw.RunConfig(has_s=True)
    c = cfg.to_c()
    for field in ("f", "c", "c_s2", "u", "deposit", "s_tmp"):
        b = _fake_buffers(cfg)
        setattr(b, field, None)
        h = ctypes.c_void_p()
        assert lib.lbw_create(ctypes.byref(c), ctypes.byref(b), 1, None, ctypes.byref(h)) == lbw.ERR_INVAL
        assert not h


def test_batch_must_be_homogeneous():
    # (a valid batch is not created here: creation copies the work lists to
    # the device, which the fake pointers of these host tests cannot take)
    a = lbw.RunConfig(precision="fp32_shifted")
    rc, msg = _create([a, lbw.RunConfig(precision="fp64")])
    assert rc == lbw.ERR_INVAL and "batched" in msg
    rc, msg = _create([a, lbw.RunConfig(precision="fp32_shifted", lattice=19, nz=8)])
    assert rc == lbw.ERR_INVAL and "batched" in msg


def test_launch_shape_validation():
    lib = lbw.load()
    cfg = lbw.RunConfig()
    c, b = cfg.to_c(), _fake_buffers(cfg)
    h = ctypes.c_void_p()
    assert lib.lbw_create(ctypes.byref(c), ctypes.byref(b), 1, None, ctypes.byref(h)) == 0
    try:
        ok = lbw.CLaunch(512, 128, 16, 1, 1, 0, 0)
        assert lib.lbw_set_launch(h, ctypes.byref(ok)) == 0
        got = lbw.CLaunch()
        assert lib.lbw_get_launch(h, ctypes.byref(got)) == 0
        assert (got.lbm_block, got.tile_x, got.tile_y, got.variant, got.graph) == (512, 128, 16, 1, 1)
        # 2D: one-row tiles of 64..512 columns
        assert lib.lbw_set_launch(h, ctypes.byref(lbw.CLaunch(0, 512, 0, 0, 0, 0, 1))) == 0
        for bad in (lbw.CLaunch(100, 0, 0, 0, 0, 0), lbw.CLaunch(2048, 0, 0, 0, 0, 0),
                    lbw.CLaunch(0, 96, 0, 0, 0, 0), lbw.CLaunch(0, 32, 0, 0, 0, 0),
                    lbw.CLaunch(0, 0, 0, 3, 0, 0), lbw.CLaunch(0, 0, 0, 0, 3, 0),
                    lbw.CLaunch(0, 0, 0, 2, 0, 0), lbw.CLaunch(0, 0, 0, 0, 0, 1),
                    lbw.CLaunch(0, 256, 0, 0, 0, 0, 2)):
            assert lib.lbw_set_launch(h, ctypes.byref(bad)) == lbw.ERR_INVAL
        assert lib.lbw_step(h, -1) == lbw.ERR_INVAL
        v = ctypes.c_int64(-1)
        assert lib.lbw_steps_done(h, ctypes.byref(v)) == 0 and v.value == 0
        assert lib.lbw_export(h, 5, 1, ctypes.c_void_p(0x1000)) == lbw.ERR_INVAL
        assert lib.lbw_export(h, 0, 9, ctypes.c_void_p(0x1000)) == lbw.ERR_INVAL
        assert lib.lbw_export(h, 0, lbw.FIELD_S, ctypes.c_void_p(0x1000)) == lbw.ERR_INVAL
    finally:
        lib.lbw_destroy(h)


def test_rebind_accepts_only_per_step_outputs():
    # host-only: a single run keeps no device tables, so rebinding touches
    # no device memory
    lib = lbw.load()
    for mode, u_ok in ((lbw.FLUID_LBM, True), (lbw.FLUID_FROZEN, False)):
        cfg = lbw.RunConfig(fluid_mode=mode)
        c, b = cfg.to_c(), _fake_buffers(cfg)
        h = ctypes.c_void_p()
        assert lib.lbw_create(ctypes.byref(c), ctypes.byref(b), 1, None, ctypes.byref(h)) == 0
        try:
            p = ctypes.c_void_p(0x7000000)
            assert lib.lbw_rebind(h, 0, lbw.FIELD_STAGE1, p) == 0
            assert lib.lbw_rebind(h, 0, lbw.FIELD_STAGE2, p) == 0
            assert lib.lbw_rebind(h, 0, lbw.FIELD_STAGE1, None) == 0
            assert (lib.lbw_rebind(h, 0, lbw.FIELD_U, p) == 0) == u_ok
            assert (lib.lbw_rebind(h, 0, lbw.FIELD_RHO, p) == 0) == u_ok
            assert (lib.lbw_rebind(h, 0, lbw.FIELD_RHO, None) == 0) == u_ok
            for bad in (lbw.FIELD_F, lbw.FIELD_C, lbw.FIELD_S, lbw.FIELD_DEPOSIT, 42):
                assert lib.lbw_rebind(h, 0, bad, p) == lbw.ERR_INVAL
            assert lib.lbw_rebind(h, 3, lbw.FIELD_STAGE1, p) == lbw.ERR_INVAL
        finally:
            lib.lbw_destroy(h)


def test_tile_rows_validation_3d():
    lib = lbw.load()
    cfg = lbw.RunConfig(lattice=19, nx=8, ny=8, nz=16)
    c, b = cfg.to_c(), _fake_buffers(cfg)
    h = ctypes.c_void_p()
    assert lib.lbw_create(ctypes.byref(c), ctypes.byref(b), 1, None, ctypes.byref(h)) == 0
    try:
        for tx, rows in ((32, 0), (32, 8), (32, 16), (64, 4), (64, 8), (128, 2), (128, 0)):
            assert lib.lbw_set_launch(h, ctypes.byref(lbw.CLaunch(0, tx, 0, 0, 0, 0, rows))) == 0
            got = lbw.CLaunch()
            lib.lbw_get_launch(h, ctypes.byref(got))
            assert (got.tile_x, got.tile_rows) == (tx, rows)
        for tx, rows in ((32, 4), (64, 16), (128, 8), (32, 32), (32, 1)):
            assert lib.lbw_set_launch(h, ctypes.byref(lbw.CLaunch(0, tx, 0, 0, 0, 0, rows))) == lbw.ERR_INVAL
    finally:
        lib.lbw_destroy(h)


def test_batched_needs_scratch():
    lib = lbw.load()
    cfgs = [lbw.RunConfig(precision="fp32_shifted"), lbw.RunConfig(precision="fp32_shifted")]
    arr = (lbw.CConfig * 2)(*[c.to_c() for c in cfgs])
    bufs = (lbw.CBuffers * 2)(*[_fake_buffers(c) for c in cfgs])
    bufs[0].scratch_bytes = 64
    h = ctypes.c_void_p()
    assert lib.lbw_create(arr, bufs, 2, None, ctypes.byref(h)) == lbw.ERR_INVAL
    assert b"scratch" in lib.lbw_last_error()


def test_scratch_bytes():
    lib = lbw.load()
    arr = (lbw.CConfig * 3)(*[lbw.RunConfig().to_c()] * 3)
    n = ctypes.c_size_t()
    assert lib.lbw_scratch_bytes(arr, 3, ctypes.byref(n)) == 0
    assert n.value >= 3 * 8
    assert lib.lbw_scratch_bytes(arr, 0, ctypes.byref(n)) == lbw.ERR_INVAL


def test_adjoint_wrapper_refuses_what_the_kernels_do_not_cover():
    """The autograd wrapper checks its configuration before the forward sweep
    (host logic only)."""
    from paper_2106_07694_amd import adjoint
    adjoint.check_supported(lbw.RunConfig(vs=1e-3, kappa_c=1e-3))
    for bad in (dict(scheme_c="weno3"), dict(has_s=True),
                dict(n_classes=2, vs_class=(1e-3, 2e-3), kappa_class=(0.0, 0.0))):
        with pytest.raises(ValueError):
            adjoint.check_supported(lbw.RunConfig(**bad))


def test_binding_refuses_buffers_of_the_wrong_size_type_or_place():
    """The binding hands the library raw pointers to buffers it reads or
    writes in full, so it refuses any tensor that is not exactly the field:
    wrong element count, element type, layout or device (host logic only)."""
    import torch

    cfg = lbw.RunConfig(lattice=19, nx=8, ny=4, nz=6, precision="fp32_shifted")
    sol = lbw.Solver.__new__(lbw.Solver)      # no device needed for the checks
    sol.cfgs, sol.dtype = [cfg], torch.float32
    n = cfg.cells
    cases = [("c", torch.zeros(n + 1), "values"), ("f", torch.zeros(19 * n - 1), "values"),
             ("c", torch.zeros(n, dtype=torch.float64), "element type"),
             ("deposit", torch.zeros(cfg.ncol, dtype=torch.float32), "element type"),
             ("rho", torch.zeros(n, dtype=torch.float64), "element type"),
             ("u", torch.zeros(2, 3 * n)[0, :].view(3, n)[:, :].t().contiguous().t(), "contiguous"),
             ("c", torch.zeros(n), "not on the device"),
             ("deposit", torch.zeros(cfg.ncol, dtype=torch.float64), "not on the device")]
    for name, t, reason in cases:
        with pytest.raises(ValueError, match=reason):
            sol._checked(name, t, 0)


def test_tiled_launch_larger_than_one_dispatch_is_refused():
    """A single run's tiled transport launches one block per tile and chunk;
    a launch shape whose work-items would reach 2^32 (a huge run with
    one-plane chunks and tiles that fit its lateral sizes badly) is refused
    instead of dispatched."""
    lib = lbw.load()
    cfg = lbw.RunConfig(lattice=19, nx=33, ny=9, nz=14_000_000, precision="fp32_shifted")
    c, b = cfg.to_c(), _fake_buffers(cfg)
    h = ctypes.c_void_p()
    assert lib.lbw_create(ctypes.byref(c), ctypes.byref(b), 1, None, ctypes.byref(h)) == 0
    try:
        assert lib.lbw_set_launch(h, ctypes.byref(lbw.CLaunch(0, 0, 1, 0, 0, 0, 0))) == lbw.ERR_INVAL
        assert "work-items" in lib.lbw_last_error().decode()
        # the plain transport (one thread per node) and longer chunks still fit
        assert lib.lbw_set_launch(h, ctypes.byref(lbw.CLaunch(0, 0, 1, 1, 0, 0, 0))) == 0
        assert lib.lbw_set_launch(h, ctypes.byref(lbw.CLaunch(0, 0, 64, 0, 0, 0, 0))) == 0
    finally:
        lib.lbw_destroy(h)
