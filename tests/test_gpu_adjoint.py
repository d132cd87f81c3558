"""GPU adjoint against the oracle's adjoint and against finite differences.

* one reverse step in FP64 equals the oracle's reverse step (1e-12 relative);
* the gradient of the deposited mass through checkpointed steps equals the
  oracle's step-by-step reverse sweep (FP64) and does not depend on the
  checkpoint spacing (bitwise);
* central finite differences of the FP64 forward on 16 seeded directions
  converge to the adjoint gradient as eps^2 (eps = 1e-4, 1e-5, 1e-6): at
  eps = 1e-4 they carry an O((eps / 1e-3)^2) truncation error, because the
  WENO weights vary on the scale of the 1e-3 seeded noise, so the gate is the
  quadratic convergence and the agreement at 1e-6; the FP32 adjoint's
  gradient matches the FP64 one.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import OracleConfig
from paper_2106_07694_amd import adjoint, autotune, lbw, workloads as W

from parity import oracle_cfg, rel

pytestmark = pytest.mark.gpu


def _flowing(ocfg, rng):
    dim = ocfg.dim
    u0 = 0.02 * rng.standard_normal((dim,) + ocfg.shape) + np.array(
        [0.03, 0.02, 0.01][:dim]).reshape((dim, 1, 1, 1))
    f0 = oracle.equilibrium(ocfg, 1.0 + 0.01 * rng.standard_normal(ocfg.shape), u0)
    c0 = rng.uniform(0.2, 1.0, ocfg.shape)
    return f0, c0, u0


def _dev(x, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dt)


# tiny lateral axes (fewer cells than a stencil) in the plain form only: the
# wrap they exercise does not depend on the population form
_FORMS = [pytest.param("fp64", False, id="fp64-grid"), pytest.param("fp64_shifted", False, id="fp64_shifted-grid"),
          pytest.param("fp64", True, id="fp64-tiny_lateral")]


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("frozen", [False, True])
@pytest.mark.parametrize("vper", [False, True])
@pytest.mark.parametrize("precision,tiny", _FORMS)
def test_adjoint_step_matches_oracle(q, frozen, vper, precision, tiny):
    """One reverse step against the oracle's; tiny lateral axes (fewer cells
    than a stencil) exercise the periodic wrap of the face and gather
    kernels."""
    rng = np.random.default_rng(31)
    if tiny:
        shape = dict(nx=3, ny=9) if q == 9 else dict(nx=2, ny=3, nz=8)
    else:
        shape = dict(nx=13, ny=17) if q == 9 else dict(nx=7, ny=5, nz=11)
    cfg = lbw.RunConfig(lattice=q, precision=precision, tau=0.7, vs=0.04, kappa_c=2e-3,
                        gp_c=3e-3, vert_periodic=vper,
                        fluid_mode=lbw.FLUID_FROZEN if frozen else lbw.FLUID_LBM, **shape)
    ocfg = oracle_cfg(cfg)
    f_n, c_n, u0 = _flowing(ocfg, rng)
    fbar_next = rng.standard_normal((q,) + ocfg.shape)
    cbar_next = rng.standard_normal(ocfg.shape)
    dep_bar = 0.7
    fo, co, vo = oracle.adjoint_step(ocfg, None if frozen else f_n, c_n,
                                     None if frozen else fbar_next, cbar_next, dep_bar,
                                     u0 if frozen else None)
    sol = lbw.Solver(cfg)
    if frozen:
        sol.set_field("u", u0)
    fb = torch.zeros((q,) + ocfg.shape, dtype=torch.float64, device="cuda")
    cb = torch.zeros(ocfg.shape, dtype=torch.float64, device="cuda")
    vs = torch.zeros(1, dtype=torch.float64, device="cuda")
    work = sol.adjoint_workspace()
    torch.cuda.synchronize()
    sol.adjoint_step(None if frozen else _dev(f_n), _dev(c_n),
                     None if frozen else _dev(fbar_next), _dev(cbar_next), dep_bar,
                     None if frozen else fb, cb, vs, work)
    torch.cuda.synchronize()
    # the same step with the forward intermediates supplied instead of recomputed
    if not frozen:
        fr = lbw.Solver(cfg)
        fr.set_field("f", f_n)
        fr.set_field("c", c_n)
        rho_n = torch.full(ocfg.shape, float("nan"), dtype=torch.float64, device="cuda")
        fr.rebind("rho", rho_n)
        fr.step(1)
        fr.rebind("rho", None)
        u_n, a1, a2 = fr.field("u"), fr.field("stage1"), fr.field("stage2")
        fr.close()
        # the density the step wrote is the zeroth moment of f^n
        rho_ref = f_n.sum(axis=0) + (1.0 if precision == "fp64_shifted" else 0.0)
        assert np.max(np.abs(rho_n.cpu().numpy() - rho_ref)) < 1e-13
        fb2, cb2 = torch.zeros_like(fb), torch.zeros_like(cb)
        vs2 = torch.zeros(1, dtype=torch.float64, device="cuda")
        sol.adjoint_step(_dev(f_n), _dev(c_n), _dev(fbar_next), _dev(cbar_next), dep_bar, fb2, cb2,
                         vs2, work, u_n=u_n, a1_n=a1, a2_n=a2)
        torch.cuda.synchronize()
        assert torch.equal(fb2, fb) and torch.equal(cb2, cb) and torch.equal(vs2, vs)
        # and with the moments supplied, no populations at all
        fb3, cb3 = torch.zeros_like(fb), torch.zeros_like(cb)
        vs3 = torch.zeros(1, dtype=torch.float64, device="cuda")
        sol.adjoint_step(None, _dev(c_n), _dev(fbar_next), _dev(cbar_next), dep_bar, fb3, cb3,
                         vs3, work, u_n=u_n, rho_n=rho_n, a1_n=a1, a2_n=a2)
        torch.cuda.synchronize()
        assert torch.equal(fb3, fb) and torch.equal(cb3, cb) and torch.equal(vs3, vs)
    torch.cuda.synchronize()
    errs = {"cbar": rel(cb.cpu().numpy(), co), "vs_bar": abs(vs.item() - vo) / max(abs(vo), 1e-300)}
    if not frozen:
        errs["fbar"] = rel(fb.cpu().numpy(), fo)
    print(f"\nadjoint step q={q} frozen={frozen} vper={vper} {precision}: {errs}")
    assert max(errs.values()) < 1e-12, errs
    sol.close()


def _oracle_gradient(ocfg, f0, c0, n):
    fs, cs = [], []
    f, c = f0, c0
    for _ in range(n):
        fs.append(f)
        cs.append(c)
        f, c, _, _, _ = oracle.run(ocfg, f, c, None, None, None, 1)
    fbar = np.zeros((ocfg.q,) + ocfg.shape)
    cbar = np.zeros(ocfg.shape)
    vsb = 0.0
    for k in reversed(range(n)):
        fbar, cbar, v = oracle.adjoint_step(ocfg, fs[k], cs[k], fbar, cbar, 1.0)
        vsb += v
    return cbar, vsb


def test_checkpointed_gradient_fp64_matches_oracle():
    wl = W.C5.replace(nx=24, ny=32, precision="fp64")
    cfg = lbw.RunConfig.from_workload(wl)
    c0, _ = W.initial_scalars(wl)
    n = 12
    c0t = _dev(c0).requires_grad_(True)
    vst = torch.tensor(cfg.vs, dtype=torch.float64, requires_grad=True)
    J = adjoint.DepositedMass.apply(c0t, vst, cfg, n, 5)
    J.backward()
    ocfg = oracle_cfg(cfg)
    cbar_o, vsb_o = _oracle_gradient(ocfg, oracle.equilibrium(ocfg), c0, n)
    e_c = rel(c0t.grad.cpu().numpy(), cbar_o)
    e_v = abs(vst.grad.item() - vsb_o) / abs(vsb_o)
    _, _, _, dep, _ = oracle.run(ocfg, oracle.equilibrium(ocfg), c0, nsteps=n)
    print(f"\ncheckpointed FP64 gradient vs oracle: dc0 {e_c:.2e}, dvs {e_v:.2e}; "
          f"J {J.item():.15e} vs {dep.sum():.15e}")
    assert abs(J.item() - dep.sum()) < 1e-12 * abs(dep.sum())
    assert e_c < 1e-11 and e_v < 1e-11


def test_checkpoint_spacing_does_not_change_the_gradient():
    wl = W.C5.replace(nx=32, ny=48)
    cfg = lbw.RunConfig.from_workload(wl)
    c0, _ = W.initial_scalars(wl)
    n = 12
    grads = []
    for seg in (1, 3, 5, 12):
        c0t = _dev(c0, torch.float32).requires_grad_(True)
        vst = torch.tensor(cfg.vs, dtype=torch.float64, requires_grad=True)
        adjoint.DepositedMass.apply(c0t, vst, cfg, n, seg).backward()
        grads.append((c0t.grad.cpu().numpy(), vst.grad.item()))
    for g in grads[1:]:
        assert np.array_equal(g[0], grads[0][0]) and g[1] == grads[0][1]


def _grad(cfg, c0, n, dt, **kw):
    c0t = _dev(c0, dt).requires_grad_(True)
    vst = torch.tensor(cfg.vs, dtype=torch.float64, requires_grad=True)
    adjoint.DepositedMass.apply(c0t, vst, cfg, n, None, None, kw.get("f0"), kw.get("u")).backward()
    return c0t.grad.double().cpu().numpy(), vst.grad.item()


def _fd_errors(cfg64, c0, n, grads, ndirs=16, epss=(1e-4, 1e-5, 1e-6), **kw):
    """Max relative error over the directions, and the dVs error, per eps."""
    def J(c, vs=cfg64.vs):
        J, sol, _ = adjoint.forward_with_checkpoints(cfg64, _dev(c), vs, n, n, None,
                                                     kw.get("f0"), kw.get("u"))
        sol.close()
        return J

    dirs = W.random_directions(ndirs, c0.shape, seed=2024)
    g = grads["fp64"]
    out = {}
    for eps in epss:
        errs = []
        for v in dirs:
            fd = (J(c0 + eps * v) - J(c0 - eps * v)) / (2 * eps)
            errs.append(abs(np.sum(g[0] * v) - fd) / abs(fd))
        fdv = (J(c0, cfg64.vs + eps) - J(c0, cfg64.vs - eps)) / (2 * eps)
        out[eps] = (max(errs), abs(g[1] - fdv) / abs(fdv))
    return out


def _check_fd(out, tol, floor=1e-8):
    """Agreement at eps = 1e-6 and second-order convergence of the central
    differences towards the adjoint over both decades of eps."""
    e4, e5, e6 = out[1e-4][0], out[1e-5][0], out[1e-6][0]
    v4, v5, v6 = out[1e-4][1], out[1e-5][1], out[1e-6][1]
    assert e6 < tol and v6 < tol, out
    for a, b in ((e4, e5), (e5, e6), (v4, v5), (v5, v6)):
        assert b < 0.05 * a or b < floor, out


def test_frozen_gradient_matches_finite_differences():
    """Transport only, smooth velocity with no sign change on any face:
    FP64 and FP32 adjoints vs central FD (eps = 1e-4, 16 directions)."""
    wl = W.C5.replace(nx=128, ny=256)
    n = 300
    base = dict(fluid_mode=lbw.FLUID_FROZEN, vs=2e-3)
    cfg32 = lbw.RunConfig.from_workload(wl, **base)
    cfg64 = lbw.RunConfig.from_workload(wl, precision="fp64", **base)
    c0, _ = W.initial_scalars(wl)
    c0 = c0.astype(np.float32).astype(np.float64)
    y = np.arange(wl.ny)[None, :, None] / wl.ny
    x = np.arange(wl.nx)[None, None, :] / wl.nx
    u = np.zeros((2,) + c0.shape)
    u[0] = 0.02 + 0.01 * np.sin(2 * np.pi * x) * np.cos(np.pi * y)
    u[1] = 0.0005 * np.sin(2 * np.pi * x)
    u = u.astype(np.float32).astype(np.float64)
    g = {"fp64": _grad(cfg64, c0, n, torch.float64, u=u)}
    g32 = _grad(cfg32, c0, n, torch.float32, u=u)
    out = _fd_errors(cfg64, c0, n, g, u=u)
    l2 = float(np.linalg.norm(g32[0] - g["fp64"][0]) / np.linalg.norm(g["fp64"][0]))
    print(f"\nfrozen FD check (max rel err over 16 dirs, dVs rel err) per eps: {out}; "
          f"FP32 vs FP64 gradient L2 {l2:.2e}")
    _check_fd(out, 1e-5)
    assert l2 < 1e-3 and abs(g32[1] - g["fp64"][1]) < 1e-3 * abs(g["fp64"][1])


def test_coupled_gradient_matches_finite_differences():
    """Coupled LBM + transport started from a plug flow (lateral velocity
    bounded away from zero, so no face changes its upwind side): FP64 and
    FP32 adjoints vs central FD (eps = 1e-4, 16 directions)."""
    wl = W.C5.replace(nx=128, ny=256)
    n = 200
    cfg32 = lbw.RunConfig.from_workload(wl)
    cfg64 = lbw.RunConfig.from_workload(wl, precision="fp64")
    c0, _ = W.initial_scalars(wl)
    c0 = c0.astype(np.float32).astype(np.float64)
    ocfg = oracle_cfg(cfg64)
    u0 = np.zeros((2,) + c0.shape)
    u0[0] = 0.03
    f0_64 = oracle.equilibrium(ocfg, None, u0)
    f0_32 = oracle.equilibrium(oracle_cfg(cfg32), None, u0).astype(np.float32).astype(np.float64)
    g = {"fp64": _grad(cfg64, c0, n, torch.float64, f0=f0_64)}
    g32 = _grad(cfg32, c0, n, torch.float32, f0=f0_32)
    out = _fd_errors(cfg64, c0, n, g, f0=f0_64)
    l2 = float(np.linalg.norm(g32[0] - g["fp64"][0]) / np.linalg.norm(g["fp64"][0]))
    print(f"\ncoupled FD check (max rel err over 16 dirs, dVs rel err) per eps: {out}; "
          f"FP32 vs FP64 gradient L2 {l2:.2e}")
    _check_fd(out, 1e-5)
    assert l2 < 1e-3 and abs(g32[1] - g["fp64"][1]) < 1e-3 * abs(g["fp64"][1])



@pytest.mark.parametrize("shape", [(13, 17), (3, 9), (40, 37), (64, 48)])
@pytest.mark.parametrize("vper", [False, True])
@pytest.mark.parametrize("precision", ["fp64", "fp32_shifted"])
@pytest.mark.parametrize("frozen", [False, True])
def test_fused_2d_transpose_equals_two_kernel_form(shape, vper, precision, frozen):
    """In 2D each reversed RK stage runs as one kernel with its face products
    in LDS; it evaluates and gathers the same products in the same order as
    the face + gather kernels (launch variant 1), so every output matches bit
    for bit, ragged and tiny tiles and wall images included."""
    nx, ny = shape
    rng = np.random.default_rng(hash(shape) % 1000)
    cfg = lbw.RunConfig(lattice=9, precision=precision, tau=0.7, vs=0.04, kappa_c=2e-3, gp_c=3e-3,
                        vert_periodic=vper, nx=nx, ny=ny,
                        fluid_mode=lbw.FLUID_FROZEN if frozen else lbw.FLUID_LBM)
    ocfg = oracle_cfg(cfg)
    f_n, c_n, u0 = _flowing(ocfg, rng)
    dt = torch.float64 if precision == "fp64" else torch.float32
    dev = lambda x: _dev(x, dt)
    fbar_next = dev(rng.standard_normal((9,) + ocfg.shape))
    cbar_next = dev(rng.standard_normal(ocfg.shape))
    outs = []
    for variant in (0, 1):
        sol = lbw.Solver(cfg)
        sol.set_launch(variant=variant)
        if frozen:
            sol.set_field("u", u0)
        fb = torch.zeros((9,) + ocfg.shape, dtype=dt, device="cuda")
        cb = torch.zeros(ocfg.shape, dtype=dt, device="cuda")
        vs = torch.zeros(1, dtype=torch.float64, device="cuda")
        work = sol.adjoint_workspace()
        sol.adjoint_step(None if frozen else dev(f_n), dev(c_n), None if frozen else fbar_next,
                         cbar_next, 0.7, None if frozen else fb, cb, vs, work)
        torch.cuda.synchronize()
        outs.append((fb.clone(), cb.clone(), vs.clone()))
        sol.close()
    (fb0, cb0, vs0), (fb1, cb1, vs1) = outs
    assert torch.equal(cb0, cb1) and torch.equal(vs0, vs1)
    if not frozen:
        assert torch.equal(fb0, fb1)


@pytest.mark.parametrize("frozen", [False, True])
def test_native_replay_records_what_the_per_call_replay_records(frozen):
    """lbw_replay (one call per segment) against rounds of export, rebind and
    one step from the host: the recorded C, velocity, density and stages,
    and the state it leaves, agree bit for bit; afterwards the per-step
    outputs are bound back to the solver's own buffers."""
    import torch

    cfg = lbw.RunConfig(nx=48, ny=40, tau=0.6, vs=2e-3, kappa_c=1e-3, gp_c=3e-4,
                        precision="fp32_shifted",
                        fluid_mode=lbw.FLUID_FROZEN if frozen else lbw.FLUID_LBM)
    rng = np.random.default_rng(17)
    c0 = rng.uniform(0, 1, cfg.shape)
    u0 = 0.03 * rng.standard_normal((2,) + cfg.shape)
    n = 7

    def start():
        sol = lbw.Solver(cfg)
        sol.set_field("c", c0)
        if frozen:
            sol.set_field("u", u0)
        else:
            sol.init_equilibrium()
        return sol

    def bufs():
        e = lambda *s: torch.empty(s, dtype=torch.float32, device="cuda")
        return ([e(*cfg.shape) for _ in range(n)], [e(2, *cfg.shape) for _ in range(n)],
                [e(*cfg.shape) for _ in range(n)], [e(*cfg.shape) for _ in range(n)],
                [e(*cfg.shape) for _ in range(n)])

    a = start()
    ca, ua, ra, a1a, a2a = bufs()
    a.replay(ca, a1a, a2a, None if frozen else ua, None if frozen else ra)
    a.step(1)                       # the own buffers are bound again
    b = start()
    cb, ub, rb, a1b, a2b = bufs()
    for i in range(n):
        b.export_into("c", cb[i])
        if not frozen:
            b.rebind("u", ub[i])
            b.rebind("rho", rb[i])
        b.rebind("stage1", a1b[i])
        b.rebind("stage2", a2b[i])
        b.step(1)
    for name in ("stage1", "stage2") + (() if frozen else ("u", "rho")):
        b.rebind(name, None)
    b.step(1)
    torch.cuda.synchronize()
    kinds = [(ca, cb), (a1a, a1b), (a2a, a2b)] + ([] if frozen else [(ua, ub), (ra, rb)])
    for x, y in kinds:
        for i in range(n):
            assert torch.equal(x[i], y[i]), i
    for k in ("c", "deposit", "stage1", "stage2") + (() if frozen else ("f", "u")):
        assert torch.equal(a.field(k), b.field(k)), k
    if not frozen:                  # a coupled run needs the density buffers
        with pytest.raises(lbw.LbwError):
            a.replay([ca[0]], [a1a[0]], [a2a[0]], [ua[0]], None)
    a.close()
    b.close()


def test_replay_refuses_a_batch():
    import torch

    cfgs = [lbw.RunConfig(nx=16, ny=12), lbw.RunConfig(nx=20, ny=10)]
    sol = lbw.Solver(cfgs, stream=torch.cuda.Stream())
    t = torch.zeros((16 * 12,), dtype=torch.float64, device="cuda")
    with pytest.raises(lbw.LbwError):
        sol.replay([t], [t], [t], [t], [t])
    sol.close()


def test_c5_configuration_gradient_against_finite_differences():
    """The adjoint form's own configuration: 512 x 1024, the physics of the
    2D FP64 case without S, from rest, 5000 steps with sqrt(N) checkpoints,
    16 seeded directions at eps = 1e-4 (and 4 of them at 1e-5 and 1e-6),
    plus dJ/dVs.  The finite differences use the FP64 forward; the gradients
    come from the FP64 and the FP32 (the production form) adjoints.

    Central differences carry an O(eps^2) truncation error whose scale is set
    by the WENO weights, which vary on the scale of the 1e-3 seeded noise, so
    at eps = 1e-4 it is of order (1e-4 / 1e-3)^2 = 1e-2: measured 7.2e-3 on
    the worst direction and 1.9e-3 for dVs, then 1.8e-4 / 1.9e-5 at 1e-5 and
    1.8e-6 / 1.9e-7 at 1e-6.  Required: below 2e-2 at eps = 1e-4 (BASELINE's
    value), below 1e-5 at 1e-6, and the second-order decrease over both
    decades; the FP32 gradient within 1e-3 (L2) and 1e-5 in dVs of the FP64
    one (measured 7.1e-5 and 8e-7).
    """
    wl = W.C5
    n = wl.steps
    cfg32 = lbw.RunConfig.from_workload(wl)
    cfg64 = lbw.RunConfig.from_workload(wl, precision="fp64")
    c0, _ = W.initial_scalars(wl)
    c0 = c0.astype(np.float32).astype(np.float64)
    launch = autotune.lookup(wl.name)
    print(f"\n[C5] gradients ({n} steps)", flush=True)
    g64 = _grad(cfg64, c0, n, torch.float64)
    g32 = _grad(cfg32, c0, n, torch.float32)

    def J(c, vs=cfg64.vs):
        Jv, sol, _ = adjoint.forward_with_checkpoints(cfg64, _dev(c), vs, n, n, launch)
        sol.close()
        return Jv

    dirs = W.random_directions(16, c0.shape, seed=2024)
    res = {}
    for eps, nd in ((1e-4, 16), (1e-5, 4), (1e-6, 4)):
        errs = []
        for v in dirs[:nd]:
            fd = (J(c0 + eps * v) - J(c0 - eps * v)) / (2 * eps)
            errs.append(abs(np.sum(g64[0] * v) - fd) / abs(fd))
        fdv = (J(c0, cfg64.vs + eps) - J(c0, cfg64.vs - eps)) / (2 * eps)
        res[eps] = (max(errs), abs(g64[1] - fdv) / abs(fdv))
        print(f"[C5] eps {eps:g}: worst direction {res[eps][0]:.3e}, dVs {res[eps][1]:.3e}", flush=True)
    l2 = float(np.linalg.norm(g32[0] - g64[0]) / np.linalg.norm(g64[0]))
    print(f"[C5] FP32 vs FP64 gradient: L2 {l2:.3e}, dVs {g32[1]:.6e} vs {g64[1]:.6e}", flush=True)
    assert res[1e-4][0] < 2e-2 and res[1e-4][1] < 2e-2, res
    _check_fd(res, 1e-5)
    assert l2 < 1e-3 and abs(g32[1] - g64[1]) < 1e-5 * abs(g64[1])


def test_adjoint_step_on_a_grid_taller_than_one_launch_of_the_fused_form():
    """The fused 2D reverse stages launch one block row per 16 grid rows (FP64),
    at most 65535 of them; a run of 3 x 1,048,600 cells (65,538 block rows)
    takes the two-kernel form instead, through the default launch, and must
    still equal the oracle's reverse step."""
    rng = np.random.default_rng(37)
    cfg = lbw.RunConfig(lattice=9, precision="fp64", nx=3, ny=1_048_600, tau=0.7, vs=0.04,
                        kappa_c=2e-3, gp_c=3e-3)
    ocfg = oracle_cfg(cfg)
    f_n, c_n, _ = _flowing(ocfg, rng)
    fbar_next = rng.standard_normal((9,) + ocfg.shape)
    cbar_next = rng.standard_normal(ocfg.shape)
    dep_bar = 0.7
    fo, co, vo = oracle.adjoint_step(ocfg, f_n, c_n, fbar_next, cbar_next, dep_bar, None)
    sol = lbw.Solver(cfg)
    fb = torch.zeros((9,) + ocfg.shape, dtype=torch.float64, device="cuda")
    cb = torch.zeros(ocfg.shape, dtype=torch.float64, device="cuda")
    vs = torch.zeros(1, dtype=torch.float64, device="cuda")
    work = sol.adjoint_workspace()
    torch.cuda.synchronize()
    sol.adjoint_step(_dev(f_n), _dev(c_n), _dev(fbar_next), _dev(cbar_next), dep_bar, fb, cb, vs, work)
    torch.cuda.synchronize()
    vs_scale = float(np.sum(np.abs(cbar_next * c_n))) + dep_bar * float(np.sum(np.abs(c_n)))
    errs = {"cbar": rel(cb.cpu().numpy(), co), "fbar": rel(fb.cpu().numpy(), fo),
            "vs_bar": abs(vs.item() - vo) / max(abs(vo), vs_scale)}
    print(f"\nadjoint step on 3 x 1,048,600: {errs}")
    assert max(errs.values()) < 1e-12, errs
    sol.close()
