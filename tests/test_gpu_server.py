"""Continuous-batching server on the GPU.

- Every served result equals the same solve run alone through the library
  (bitwise: same precision, same per-node arithmetic) and matches the FP64
  oracle: FP64 solves to the FP64 bar (relative L1 <= 1e-12 per field),
  FP32 solves within FP32_SHORT_TOL.
- Solves submitted while others run are admitted without waiting for them
  to finish; admission respects the device-memory budget; cancel works.
- A solve that goes non-finite is stopped at the next tick (E_NONFINITE,
  fewer steps than asked) and the solves beside it are bitwise unaffected.
- One waiter per ticket; solves refused by the stability admission come
  back E_UNSTABLE.
"""
import threading
import time

import numpy as np
import pytest

import oracle
from paper_1010_4135_amd import inputs, metrics

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_SHORT_TOL = 2e-5  # FP32 modes against the FP64 oracle after at most 90 steps


def _lib():
    from paper_1010_4135_amd import lbm3d
    return lbm3d


def _alone(case, steps):
    s = _lib().Solver(dict(case.params))
    s.init(*case.fields)
    s.step(steps)
    m = s.moments()
    s.close()
    return m


def _oracle(case, steps):
    o = oracle.Oracle(dict(case.params))
    o.init(*case.fields)
    o.step(steps)
    return o.moments()


def _shape(case):
    nx, ny, nz = case.grid
    return (nz, ny, nx)


def test_served_results_equal_solo_runs_and_match_the_oracle():
    lbm3d = _lib()
    cases = [
        (inputs.riemann_3d(1, grid=(32, 32, 32), precision="fp32_t64"), 70),
        (inputs.shock_bubble(2, grid=(48, 32, 32), precision="fp32_t64", mach=4.0, ratio=0.2), 45),
        (inputs.riemann_3d(3, grid=(40, 24, 20), precision="fp64"), 33),
        (inputs.shock_bubble(4, grid=(64, 24, 16), precision="fp32", mach=2.0, ratio=5.0), 90),
        (inputs.riemann_3d(5, grid=(33, 17, 9), precision="fp32_t64"), 1),
        (inputs.riemann_3d(6, grid=(16, 16, 16), precision="fp32_t64"), 0),
        (inputs.shock_bubble(7, grid=(70, 20, 12), precision="fp64", mach=5.0, ratio=3.0), 50),
    ]
    with lbm3d.Server(8 << 30, 4, tick_steps=16) as srv:
        tickets = []
        for c, n in cases:
            tickets.append(srv.submit(c.params, c.fields, n))
            time.sleep(0.002)
        for (c, n), t in zip(cases, tickets):
            rc, got, tm = srv.wait(t, _shape(c))
            assert rc == lbm3d.OK
            assert tm["steps"] == n and tm["t_submit"] <= tm["t_admit"] <= tm["t_done"]
            ref = _alone(c, n)
            for a, b in zip(got, ref):
                assert np.array_equal(a, b), (c.name, n)
            err = metrics.rel_l1(got, _oracle(c, n))
            prec = c.params["precision"]
            print(f"[served {prec} {c.name} {c.grid} {n} steps] " +
                  " ".join(f"{k}={v:.2e}" for k, v in err.items()), flush=True)
            assert max(err.values()) <= (FP64_TOL if prec == "fp64" else FP32_SHORT_TOL), (c.name, err)
        st = srv.stats()
    assert st["admitted"] == len(cases) and st["completed"] == len(cases) and st["evicted"] == 0
    assert st["ticks"] >= 1 and 0.0 < st["busy_s"] <= st["wall_s"]


def test_continuous_admission_overlaps_running_solves():
    """A long solve is running when a short one arrives: the short one is
    admitted and finishes before the long one."""
    lbm3d = _lib()
    long_case = inputs.riemann_3d(7, grid=(96, 64, 64), precision="fp32_t64")
    short_case = inputs.riemann_3d(8, grid=(32, 32, 32), precision="fp32_t64")
    with lbm3d.Server(8 << 30, 8, tick_steps=8) as srv:
        # (about 0.4 s of ticks: far longer than the short
        # solve's admission and its three ticks)
        t_long = srv.submit(long_case.params, long_case.fields, 6000)
        time.sleep(0.05)
        t_short = srv.submit(short_case.params, short_case.fields, 20)
        rc_s, _, tm_s = srv.wait(t_short, _shape(short_case))
        rc_l, _, tm_l = srv.wait(t_long, _shape(long_case))
    print(f"[admission] short admitted {tm_s['t_admit']:.3f} s, done {tm_s['t_done']:.3f} s; "
          f"long admitted {tm_l['t_admit']:.3f} s, done {tm_l['t_done']:.3f} s", flush=True)
    assert rc_s == lbm3d.OK and rc_l == lbm3d.OK
    assert tm_s["t_admit"] < tm_l["t_done"]
    assert tm_s["t_done"] < tm_l["t_done"]


def test_budget_admission_and_refusal():
    lbm3d = _lib()
    c = inputs.riemann_3d(9, grid=(32, 32, 32), precision="fp32")
    fp = lbm3d.lbm3d_footprint(c.params)
    # budget for exactly one solve: the others wait in arrival order
    with lbm3d.Server(fp + 1024, 8, tick_steps=4) as srv:
        ts = [srv.submit(c.params, c.fields, 12) for _ in range(3)]
        tms = [srv.wait(t, _shape(c))[2] for t in ts]
        for a, b in zip(tms, tms[1:]):
            assert b["t_admit"] >= a["t_done"]
        big = inputs.riemann_3d(9, grid=(64, 64, 64), precision="fp32")
        with pytest.raises(lbm3d.LbmError) as ei:
            srv.submit(big.params, big.fields, 1)
        assert ei.value.code == lbm3d.E_NOMEM


def test_cancel_queued_ticket():
    lbm3d = _lib()
    c = inputs.riemann_3d(10, grid=(64, 64, 64), precision="fp32_t64")
    fp = lbm3d.lbm3d_footprint(c.params)
    with lbm3d.Server(fp + 1024, 1, tick_steps=8) as srv:
        t1 = srv.submit(c.params, c.fields, 400)
        t2 = srv.submit(c.params, c.fields, 400)
        srv.cancel(t2)
        rc2, _, _ = srv.wait(t2, _shape(c))
        rc1, _, _ = srv.wait(t1, _shape(c))
    assert rc2 == lbm3d.E_CANCELLED and rc1 == lbm3d.OK
    with pytest.raises(lbm3d.LbmError):
        srv2 = lbm3d.Server(1 << 30, 1)
        try:
            srv2.poll(12345)
        finally:
            srv2.close()


def test_cancel_running_ticket_and_close_with_work_in_flight():
    """A running solve cancelled between ticks stops with E_CANCELLED after
    some of its steps, and the solve beside it is bitwise its solo run;
    closing the server with solves running and queued cancels them and
    returns (the helper thread that admits and reads back drains first)."""
    lbm3d = _lib()
    long = inputs.riemann_3d(13, grid=(64, 64, 64), precision="fp32_t64")
    short = inputs.riemann_3d(14, grid=(32, 32, 32), precision="fp32_t64")
    with lbm3d.Server(8 << 30, 4, tick_steps=8) as srv:
        t1 = srv.submit(long.params, long.fields, 1000000)
        t2 = srv.submit(short.params, short.fields, 50)
        rc2, f2, tm2 = srv.wait(t2, _shape(short))
        srv.cancel(t1)
        rc1, _, tm1 = srv.wait(t1, _shape(long))
        assert rc2 == lbm3d.OK and tm2["steps"] == 50
        assert rc1 == lbm3d.E_CANCELLED and 0 < tm1["steps"] < 1000000
        for a, b in zip(f2, _alone(short, 50)):
            assert np.array_equal(a, b)
        for _ in range(3):
            srv.submit(long.params, long.fields, 1000000)
        st = srv.stats()
        assert st["admitted"] >= 2
    # (the with-block closed the server with those three in flight)


def _unstable_case(precision="fp32", flags=0):
    """(c1, c2, eta0) = (2, 6, 2) at the post-shock state of a Mach-8 shock,
    slightly perturbed: admitted by the Courant and diffusion numbers but
    linearly unstable (the von Neumann factor is about 1.06); the oracle's
    FP64 run of it is non-finite within 300 steps."""
    rho2, u2, p2, _ = inputs.rankine_hugoniot(8.0)
    g = (16, 8, 8)
    prm = inputs.make_params(g, (0,) * 6, precision=precision, c1=2.0, c2=6.0, eta0=2.0, flags=flags)
    rng = np.random.default_rng(0)
    nx, ny, nz = g
    f = [np.full((nz, ny, nx), v) for v in (rho2, u2, 0.0, 0.0, p2)]
    f[0] = f[0] * (1 + 1e-3 * rng.standard_normal(f[0].shape))
    return inputs.Case("unstable", 0, prm, tuple(f), 3000)


def test_nonfinite_solve_is_evicted_early_and_others_are_unaffected():
    lbm3d = _lib()
    bad = _unstable_case()
    good = [(inputs.riemann_3d(11, grid=(32, 32, 32), precision="fp32"), 600),
            (inputs.shock_bubble(12, grid=(64, 16, 16), precision="fp32", mach=3.0, ratio=0.5), 900)]
    with lbm3d.Server(8 << 30, 8, tick_steps=32) as srv:
        tb = srv.submit(bad.params, bad.fields, bad.steps)
        tg = [srv.submit(c.params, c.fields, n) for c, n in good]
        rc, _, tm = srv.wait(tb, _shape(bad))
        assert rc == lbm3d.E_NONFINITE
        assert tm["health"] & lbm3d.HEALTH_NONFINITE
        assert tm["steps"] < bad.steps
        print(f"[eviction] non-finite solve stopped after {tm['steps']} of {bad.steps} steps", flush=True)
        for (c, n), t in zip(good, tg):
            rc, got, tmg = srv.wait(t, _shape(c))
            assert rc == lbm3d.OK and tmg["steps"] == n
            for a, b in zip(got, _alone(c, n)):
                assert np.array_equal(a, b), c.name
        st = srv.stats()
    assert st["evicted"] == 1


def test_stability_admission_flag_refuses_the_unstable_solve():
    lbm3d = _lib()
    bad = _unstable_case(flags=lbm3d.CHECK_STABILITY)
    ok = inputs.riemann_3d(13, grid=(16, 16, 16), precision="fp32")
    ok.params = dict(ok.params, flags=lbm3d.CHECK_STABILITY)
    with lbm3d.Server(4 << 30, 4, tick_steps=8) as srv:
        tb = srv.submit(bad.params, bad.fields, 100)
        to = srv.submit(ok.params, ok.fields, 20)
        rc, _, tm = srv.wait(tb, _shape(bad))
        assert rc == lbm3d.E_UNSTABLE and tm["steps"] == 0
        rc, got, _ = srv.wait(to, _shape(ok))
        assert rc == lbm3d.OK
    # the same check on a solver handle
    s = lbm3d.Solver(bad.params)
    with pytest.raises(lbm3d.LbmError) as ei:
        s.init(*bad.fields)
    assert ei.value.code == lbm3d.E_UNSTABLE
    s.close()


def test_one_waiter_per_ticket():
    """Two threads wait on one ticket: one collects it, the other is told
    the ticket is taken (E_STATE) or already gone (E_NOTFOUND)."""
    lbm3d = _lib()
    c = inputs.riemann_3d(14, grid=(64, 64, 32), precision="fp32")
    out = [None, None]
    with lbm3d.Server(4 << 30, 2, tick_steps=8) as srv:
        t = srv.submit(c.params, c.fields, 300)

        def waiter(k):
            try:
                out[k] = srv.wait(t, _shape(c))[0]
            except lbm3d.LbmError as e:
                out[k] = e.code

        th = [threading.Thread(target=waiter, args=(k,)) for k in range(2)]
        for x in th:
            x.start()
        for x in th:
            x.join(timeout=60)
    assert sorted(out, key=lambda v: v != lbm3d.OK)[0] == lbm3d.OK
    assert sum(v == lbm3d.OK for v in out) == 1
    assert all(v in (lbm3d.OK, lbm3d.E_STATE, lbm3d.E_NOTFOUND) for v in out), out
