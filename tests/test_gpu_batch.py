"""Batched stepping on the GPU: many solves of uneven size advanced by one
persistent launch per step must give each solve bitwise the result it gets
alone, for any mix of sizes, boundary kinds and step counts."""
import numpy as np
import pytest

from paper_1010_4135_amd import inputs

pytestmark = pytest.mark.gpu


def _lib():
    from paper_1010_4135_amd import lbm3d
    return lbm3d


def _mix(precision):
    return [
        inputs.riemann_3d(1, grid=(32, 32, 32), precision=precision),
        inputs.shock_bubble(2, grid=(48, 32, 32), precision=precision, mach=3.0, ratio=0.3),
        inputs.riemann_3d(3, grid=(70, 19, 13), precision=precision),
        inputs.shock_bubble(4, grid=(65, 21, 17), precision=precision, mach=6.0, ratio=4.0),
        inputs.smooth_periodic(5, grid=(20, 12, 9), precision=precision),
        inputs.shock_bubble(6, grid=(128, 24, 16), precision=precision, mach=2.5, ratio=0.5),
        inputs.riemann_3d(7, grid=(64, 19, 11), precision=precision),
    ]


def _alone(case, steps):
    s = _lib().Solver(dict(case.params))
    s.init(*case.fields)
    s.step(steps)
    f = s.get_f()
    s.close()
    return f


@pytest.mark.parametrize("precision", ["fp32_t64", "fp64", "fp32"])
def test_batch_equals_alone_bitwise(precision):
    lbm3d = _lib()
    cases = _mix(precision)
    steps = [40, 23, 40, 1, 17, 30, 12]
    solvers = []
    for c in cases:
        s = lbm3d.Solver(dict(c.params))
        s.init(*c.fields)
        solvers.append(s)
    # a first batched run, then a second one with a different membership
    lbm3d.lbm3d_batch_step([s.h for s in solvers], [k // 2 for k in steps])
    lbm3d.lbm3d_batch_step([s.h for s in solvers], [k - k // 2 for k in steps])
    for c, s, k in zip(cases, solvers, steps):
        _, done = s.status()
        assert done == k
        assert np.array_equal(s.get_f(), _alone(c, k)), c.name
        s.close()


def test_batch_rejects_bad_arguments():
    lbm3d = _lib()
    a = lbm3d.Solver(inputs.smooth_periodic(1, grid=(16, 8, 8), precision="fp32").params)
    b = lbm3d.Solver(inputs.smooth_periodic(1, grid=(16, 8, 8), precision="fp64").params)
    c = inputs.smooth_periodic(1, grid=(16, 8, 8), precision="fp32")
    a.init(*c.fields)
    b.init(*c.fields)
    with pytest.raises(lbm3d.LbmError) as ei:
        lbm3d.lbm3d_batch_step([a.h, b.h], [1, 1])
    assert ei.value.code == lbm3d.E_INVAL
    with pytest.raises(lbm3d.LbmError) as ei:
        lbm3d.lbm3d_batch_step([a.h, a.h], [1, 1])
    assert ei.value.code == lbm3d.E_INVAL
    d = lbm3d.Solver(c.params)
    with pytest.raises(lbm3d.LbmError) as ei:
        lbm3d.lbm3d_batch_step([a.h, d.h], [1, 1])
    assert ei.value.code == lbm3d.E_STATE
    lbm3d.lbm3d_batch_step([a.h], [0])
    assert a.status()[1] == 0


def test_batch_autotuner_keeps_states():
    lbm3d = _lib()
    cases = _mix("fp32_t64")
    solvers = []
    for c in cases:
        s = lbm3d.Solver(dict(c.params))
        s.init(*c.fields)
        s.step(3)
        solvers.append(s)
    before = [s.get_f() for s in solvers]
    tz = lbm3d.lbm3d_batch_tune([s.h for s in solvers], 3)
    assert tz in (8, 16, 32)
    for s, f in zip(solvers, before):
        assert np.array_equal(s.get_f(), f) and s.status()[1] == 3
    lbm3d.lbm3d_batch_step([s.h for s in solvers], [9] * len(solvers))
    for c, s in zip(cases, solvers):
        assert np.array_equal(s.get_f(), _alone(c, 12)), c.name
        s.close()
