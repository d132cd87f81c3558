"""The no-allocation reduction (lbw_reduce_static) against lbw_reduce.

lbw_reduce_static is lbw_reduce with its partial sums in the library's own
static device array instead of the caller's scratch, so both must give the
same bits on the same state.  Two calls in a row, the second on a smaller
input, show that what the first call leaves in the shared array does not
reach the second; a handle created without any scratch can still reduce
through it; batches beyond the array's 128 runs are refused.
"""
import numpy as np
import pytest

from paper_2106_07694_amd import lbw, workloads as W

pytestmark = pytest.mark.gpu

WHATS = (lbw.MASS_C, lbw.MASS_FLUID, lbw.DEPOSIT)


def _solver(cfgs, wls, scratch=True, steps=7):
    sol = lbw.Solver(cfgs, scratch=scratch)
    for i, w in enumerate(wls):
        sol.setup_workload(w, run=i)
    sol.step(steps)
    return sol


def _same(sol, what):
    a = sol.reduce(what)
    b = sol.reduce_static(what)
    np.testing.assert_array_equal(a, b)
    assert np.all(np.isfinite(b))
    return b


def test_static_reduce_equals_reduce_larger_then_smaller():
    # first call: a batch of three uneven 2D runs (48 x 256 partials + sums)
    big = [W.C1.replace(nx=96, ny=160, precision="fp32_shifted"),
           W.C1.replace(nx=64, ny=128, precision="fp32_shifted", c0=2.0),
           W.C1.replace(nx=32, ny=64, precision="fp32_shifted", vs=2e-3)]
    sol = _solver([lbw.RunConfig.from_workload(w) for w in big], big)
    first = {w: _same(sol, w) for w in WHATS}
    sol.close()
    # second call: one smaller 3D run; the array still holds the batch's values
    small = W.C3.replace(nx=16, ny=8, nz=24)
    sol = _solver(lbw.RunConfig.from_workload(small), [small])
    second = {w: _same(sol, w) for w in WHATS}
    sol.close()
    assert first[lbw.MASS_C].shape == (3,) and second[lbw.MASS_C].shape == (1,)
    assert second[lbw.MASS_C][0] != first[lbw.MASS_C][0]


def test_static_reduce_without_caller_scratch():
    wl = W.C1.replace(nx=40, ny=72)
    cfg = lbw.RunConfig.from_workload(wl)
    ref = _solver(cfg, [wl])
    expect = {w: ref.reduce(w) for w in WHATS}
    ref.close()
    sol = _solver(cfg, [wl], scratch=False)
    with pytest.raises(lbw.LbwError):
        sol.reduce(lbw.MASS_C)          # the plain call needs the caller's scratch
    for w in WHATS:
        np.testing.assert_array_equal(sol.reduce_static(w), expect[w])
    sol.close()


def test_static_reduce_refuses_more_than_128_runs():
    wl = W.C1.replace(nx=2, ny=6, precision="fp32_shifted")
    cfgs = [lbw.RunConfig.from_workload(wl)] * 129
    sol = lbw.Solver(cfgs)
    with pytest.raises(lbw.LbwError) as e:
        sol.reduce_static(lbw.MASS_C)
    assert e.value.code == lbw.ERR_INVAL
    assert sol.reduce(lbw.MASS_C).shape == (129,)
    sol.close()
