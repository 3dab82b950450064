"""The allocation-free batched step (lbm3d_batch_step_noalloc, tables in a
static device array) against lbm3d_batch_step through the C ABI: bitwise the
same distributions on two calls in a row, the second with a smaller batch,
and the size limit is refused with E_NOMEM."""
import numpy as np
import pytest

from paper_1010_4135_amd import inputs

pytestmark = pytest.mark.gpu


def _lib():
    from paper_1010_4135_amd import lbm3d
    return lbm3d


def _solvers(cases):
    lbm3d = _lib()
    out = []
    for c in cases:
        s = lbm3d.Solver(dict(c.params))
        s.init(*c.fields)
        out.append(s)
    return out


def _compare(cases, steps):
    lbm3d = _lib()
    a = _solvers(cases)
    b = _solvers(cases)
    lbm3d.lbm3d_batch_step([s.h for s in a], steps)
    lbm3d.lbm3d_batch_step_noalloc([s.h for s in b], steps)
    for c, x, y, k in zip(cases, a, b, steps):
        assert x.status()[1] == y.status()[1] == k
        assert np.array_equal(x.get_f(), y.get_f()), c.name
        assert not (y.status()[0] & lbm3d.HEALTH_NONFINITE)
    for s in a + b:
        s.close()


@pytest.mark.parametrize("precision", ["fp32_t64", "fp64"])
def test_noalloc_batch_equals_batch_on_two_calls(precision):
    first = [
        inputs.riemann_3d(1, grid=(32, 32, 32), precision=precision),
        inputs.shock_bubble(2, grid=(128, 40, 24), precision=precision, mach=3.0, ratio=0.3),
        inputs.riemann_3d(3, grid=(70, 19, 13), precision=precision),
        inputs.smooth_periodic(4, grid=(20, 12, 9), precision=precision),
        inputs.shock_bubble(5, grid=(65, 21, 17), precision=precision, mach=6.0, ratio=4.0),
    ]
    print(f"[noalloc {precision}] first call: {len(first)} solves", flush=True)
    _compare(first, [37, 20, 37, 5, 12])
    second = [inputs.riemann_3d(6, grid=(40, 16, 8), precision=precision),
              inputs.shock_bubble(7, grid=(48, 16, 16), precision=precision, mach=2.0, ratio=2.0)]
    print(f"[noalloc {precision}] second call: {len(second)} smaller solves", flush=True)
    _compare(second, [9, 14])


def test_noalloc_rejects_tables_beyond_its_scratch():
    """Tables beyond the 4 MiB array are refused (E_NOMEM) before any device
    work: at tile depth 1, four 64 x 1 x 65535 grids make 262140 tiles of
    20 B (5.2 MB); lbm3d_batch_step takes the same batch."""
    lbm3d = _lib()
    c = inputs.make_params((64, 1, 65535), (0,) * 6, precision="fp32")
    nx, ny, nz = c["grid"]
    one = np.ones((nz, ny, nx))
    zero = np.zeros((nz, ny, nx))
    solvers = []
    for _ in range(4):
        s = lbm3d.Solver(c)
        s.init(one, zero, zero, zero, one)
        solvers.append(s)
    lbm3d.lbm3d_batch_set_depth("fp32", 1)
    try:
        with pytest.raises(lbm3d.LbmError) as ei:
            lbm3d.lbm3d_batch_step_noalloc([s.h for s in solvers], [1] * 4)
        assert ei.value.code == lbm3d.E_NOMEM
        assert all(s.status()[1] == 0 for s in solvers)
        lbm3d.lbm3d_batch_step([s.h for s in solvers], [1] * 4)
        assert all(s.status()[1] == 1 for s in solvers)
    finally:
        lbm3d.lbm3d_batch_set_depth("fp32", 0)
    for s in solvers:
        s.close()
