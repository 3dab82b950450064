"""The two plane orders of a level give bitwise the same results.

Levels below 2 GiB are stored plane-major by default (the 15 velocity planes
of one z side by side); LBM3D_VELOCITY_MAJOR forces the velocity-major order
that larger levels always use.  Only addresses differ, never the arithmetic,
so the distributions after any number of steps must be bitwise equal:
- on the tiled step with dense rows, ragged rows (lanes past the face store
  into the sink region) and a one-column x tail (whose layers stay in
  memory);
- on the untiled step, whose dense-row x layers live in the x-layer block;
- on the second-order upwind variant;
- on the batched step, with members of both orders in one batch;
- after a checkpoint is restored into a solve of the other order.
"""
import numpy as np
import pytest

from paper_1010_4135_amd import inputs

pytestmark = pytest.mark.gpu

VELOCITY_MAJOR = 8


def _lib():
    from paper_1010_4135_amd import lbm3d
    return lbm3d


def _cases(p):
    return [
        ("shockbubble_dense_128x40x24", inputs.shock_bubble(3, grid=(128, 40, 24), precision=p, mach=3.0, ratio=0.4),
         25, False),
        ("riemann_ragged_70x19x13", inputs.riemann_3d(3, grid=(70, 19, 13), precision=p), 25, False),
        ("shockbubble_ragged_66x20x12", inputs.shock_bubble(5, grid=(66, 20, 12), precision=p, mach=4.0, ratio=0.3),
         25, False),
        ("shockbubble_tail1_65x9x7", inputs.shock_bubble(7, grid=(65, 9, 7), precision=p, mach=2.0, ratio=2.0),
         25, False),
        ("shockbubble_dense_untiled_128x16x12",
         inputs.shock_bubble(9, grid=(128, 16, 12), precision=p, mach=2.5, ratio=0.5), 20, True),
    ]


def _run(params, fields, steps, untiled=False, vm=False):
    prm = dict(params)
    if vm:
        prm["flags"] = int(prm.get("flags", 0)) | VELOCITY_MAJOR
    s = _lib().Solver(prm)
    s.init(*fields)
    if untiled:
        s.set_tile(0, 1)
    if steps:
        s.step(steps)
    return s


@pytest.mark.parametrize("precision", ["fp64", "fp32_t64", "fp32"])
def test_plane_orders_are_bitwise_equal(precision):
    for name, c, steps, untiled in _cases(precision):
        print(f"[layout {precision} {name}] {steps} steps, untiled={untiled}", flush=True)
        a = _run(c.params, c.fields, steps, untiled)
        b = _run(c.params, c.fields, steps, untiled, vm=True)
        fa, fb = a.get_f(), b.get_f()
        assert np.array_equal(fa, fb), name
        assert a.status() == b.status(), name
        assert np.array_equal(a.conserved(), b.conserved()), name
        a.close()
        b.close()


def test_upwind_variant_plane_orders_are_bitwise_equal():
    c = inputs.shock_bubble(11, grid=(64, 12, 10), precision="fp64", mach=2.0, ratio=0.5)
    c.params = dict(c.params, flags=2)
    a = _run(c.params, c.fields, 15)
    b = _run(c.params, c.fields, 15, vm=True)
    assert np.array_equal(a.get_f(), b.get_f())
    a.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp32_t64", "fp64"])
def test_batch_mixes_plane_orders(precision):
    """A batch holding the same solves in both orders (and other members)
    leaves each pair bitwise equal, and equal to the solve stepped alone."""
    lbm3d = _lib()
    base = [
        inputs.shock_bubble(2, grid=(48, 32, 32), precision=precision, mach=3.0, ratio=0.3),
        inputs.riemann_3d(3, grid=(70, 19, 13), precision=precision),
        inputs.shock_bubble(6, grid=(128, 24, 16), precision=precision, mach=2.5, ratio=0.5),
    ]
    steps = [23, 40, 30]
    solvers = []
    for c in base:
        for vm in (False, True):
            prm = dict(c.params)
            if vm:
                prm["flags"] = int(prm.get("flags", 0)) | VELOCITY_MAJOR
            s = lbm3d.Solver(prm)
            s.init(*c.fields)
            solvers.append(s)
    lbm3d.lbm3d_batch_step([s.h for s in solvers], [k for k in steps for _ in range(2)])
    for j, (c, k) in enumerate(zip(base, steps)):
        pm, vm = solvers[2 * j], solvers[2 * j + 1]
        alone = _run(c.params, c.fields, k)
        fp = pm.get_f()
        assert np.array_equal(fp, vm.get_f()), c.name
        assert np.array_equal(fp, alone.get_f()), c.name
        alone.close()
    for s in solvers:
        s.close()


def test_checkpoint_moves_between_plane_orders():
    """A checkpoint (interior distributions in a fixed layout) taken from one
    order and restored into the other continues bitwise alike."""
    c = inputs.shock_bubble(4, grid=(66, 20, 12), precision="fp32_t64", mach=4.0, ratio=0.3)
    a = _run(c.params, c.fields, 10)
    b = _run(c.params, c.fields, 0, vm=True)
    b.set_f(a.get_f())
    a.step(12)
    b.step(12)
    assert np.array_equal(a.get_f(), b.get_f())
    a.close()
    b.close()


def test_level_above_2gib_stays_velocity_major_and_matches_oracle():
    """An FP64 level of 256x256x282 nodes would take 2.33 GB plane-major,
    beyond the 32-bit byte offsets the tiled kernels reach from a velocity's
    base, so it is stored velocity-major (155 MB per velocity block) and
    still runs tiled: 3 steps against the FP64 oracle at the FP64 bar."""
    import os

    import oracle
    from paper_1010_4135_amd import metrics

    case = inputs.riemann_3d(12, grid=(256, 256, 282), precision="fp64")
    print("[layout] 256x256x282 fp64, 3 steps", flush=True)
    s = _run(case.params, case.fields, 3)
    by, tz = s.get_tile()
    assert by > 0, "the velocity-major level runs tiled"
    mg = s.moments()
    s.close()
    oracle.set_threads(len(os.sched_getaffinity(0)))
    o = oracle.Oracle(case.params)
    o.init(*case.fields)
    o.step(3)
    err = metrics.rel_l1(mg, o.moments())
    print("[layout] 256x256x282 fp64 vs oracle " + " ".join(f"{k}={v:.3e}" for k, v in err.items()), flush=True)
    assert max(err.values()) <= 1e-12, err
