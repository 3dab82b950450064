"""Seeded synthetic workloads for the 3D FD-LB solver.

This module only draws initial macroscopic fields and run parameters; it holds
none of the lattice Boltzmann arithmetic (no velocity set, equilibrium, flux
or moments).  Both the GPU library and the FP64 oracle are fed from it.

Model constants common to every workload: gamma = 1.4 (b = 5), the paper's
high-Mach velocity-model triple (c1, c2, eta0) = (8, 24, 8) (Sec. 4 (1b)),
dt = tau = 1e-5 as in every run of the paper, dx = 1/256.

The shock problems use the Rankine-Hugoniot jump conditions of an ideal gas
for the post-shock state; for a Mach-2 shock into (rho, p) = (1, 1) they give
the paper's post-shock state of Sec. 4 (2): rho = 2.66667, |u| = 1.47902,
T = 1.6875 (p = 4.5), front speed D = 2.36643.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

PERIODIC, OUTFLOW, INFLOW, REFLECT = 0, 1, 2, 3
FP64, FP32, FP32_T64 = "fp64", "fp32", "fp32_t64"

MODEL = dict(c1=8.0, c2=24.0, eta0=8.0, gamma=1.4, tau=1e-5, dt=1e-5, dx=1.0 / 256.0)

BATCH_GRIDS = [(32, 32, 32), (48, 32, 32), (64, 64, 64), (96, 64, 64), (128, 128, 128)]
SERVE_GRIDS = BATCH_GRIDS + [(192, 128, 128)]


@dataclasses.dataclass
class Case:
    """One solve: run parameters, initial (rho, ux, uy, uz, p) on the
    interior nodes (arrays of shape (nz, ny, nx), x fastest) and a step count."""
    name: str
    seed: int
    params: dict
    fields: tuple
    steps: int
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def grid(self):
        return tuple(self.params["grid"])

    @property
    def sites(self) -> int:
        nx, ny, nz = self.grid
        return nx * ny * nz


def make_params(grid, bc, inflow=None, precision=FP64, flags=0, **model) -> dict:
    m = dict(MODEL)
    m.update(model)
    infl = [[0.0] * 5 for _ in range(6)]
    if inflow is not None:
        for k, st in inflow.items():
            infl[k] = [float(v) for v in st]
    return dict(grid=tuple(int(g) for g in grid), bc=tuple(int(b) for b in bc),
                inflow=infl, precision=precision, flags=int(flags), **m)


def rankine_hugoniot(mach: float, rho1: float = 1.0, p1: float = 1.0, gamma: float = 1.4):
    """Post-shock (rho2, u2, p2) and front speed D of a shock of Mach number
    `mach` running into gas at rest (rho1, p1); u2 and D point the same way."""
    g = gamma
    m2 = mach * mach
    a1 = math.sqrt(g * p1 / rho1)
    D = mach * a1
    rho2 = rho1 * (g + 1.0) * m2 / ((g - 1.0) * m2 + 2.0)
    p2 = p1 * (1.0 + 2.0 * g / (g + 1.0) * (m2 - 1.0))
    u2 = D * (1.0 - rho1 / rho2)
    return rho2, u2, p2, D


def node_coords(grid, dx):
    """Node-centre coordinates x_i = (i + 1/2) dx along each axis."""
    nx, ny, nz = grid
    return ((np.arange(nx) + 0.5) * dx, (np.arange(ny) + 0.5) * dx, (np.arange(nz) + 0.5) * dx)


def _blank(grid):
    nx, ny, nz = grid
    return [np.zeros((nz, ny, nx)) for _ in range(5)]


def _draw_state(rng, log_p=False):
    rho = rng.uniform(0.1, 2.0)
    u = rng.uniform(-1.0, 1.0)
    p = math.exp(rng.uniform(math.log(0.1), math.log(10.0))) if log_p else rng.uniform(0.1, 10.0)
    return rho, u, p


def riemann_1d(seed: int, grid=(256, 4, 4), steps: int = 500, precision=FP64, **model) -> Case:
    """Quasi-1D Riemann problem: discontinuity at x = 0.5 of [0, 1], outflow
    (linear extrapolation) at both x ends, periodic in y and z, u_y = u_z = 0.
    rho ~ U[0.1, 2], u_x ~ U[-1, 1], p ~ U[0.1, 10] on each side."""
    rng = np.random.default_rng(seed)
    left = _draw_state(rng)
    right = _draw_state(rng)
    m = dict(MODEL)
    m.update(model)
    m["dx"] = model.get("dx", 1.0 / grid[0])
    prm = make_params(grid, (OUTFLOW, OUTFLOW, PERIODIC, PERIODIC, PERIODIC, PERIODIC),
                      precision=precision, **{k: m[k] for k in MODEL})
    rho, ux, uy, uz, p = _blank(grid)
    xs = node_coords(grid, prm["dx"])[0]
    L = xs < 0.5
    for arr, k in ((rho, 0), (ux, 1), (p, 2)):
        arr[...] = np.where(L[None, None, :], left[k], right[k])
    return Case("riemann_1d", seed, prm, (rho, ux, uy, uz, p), steps,
                dict(left=left, right=right, x0=0.5))


def riemann_3d(seed: int, grid=(128, 128, 128), steps: int = 1000, precision=FP64, **model) -> Case:
    """3D Riemann problem on a periodic box: two states split by the plane
    n.(x - x_c) = 0 through the box centre, with n uniform on the sphere
    (the periodic wrap makes a second interface).  Each side moves along n
    with u_n ~ U[-1, 1]; rho ~ U[0.1, 2]; p log-uniform on [0.1, 10], so
    pressure ratios reach 100."""
    rng = np.random.default_rng(seed)
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    left = _draw_state(rng, log_p=True)
    right = _draw_state(rng, log_p=True)
    prm = make_params(grid, (PERIODIC,) * 6, precision=precision, **model)
    nx, ny, nz = grid
    zz, yy, xx = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5,
                             indexing="ij")
    side = (n[0] * (xx - nx / 2) + n[1] * (yy - ny / 2) + n[2] * (zz - nz / 2)) < 0.0
    rho = np.where(side, left[0], right[0])
    p = np.where(side, left[2], right[2])
    un = np.where(side, left[1], right[1])
    ux, uy, uz = un * n[0], un * n[1], un * n[2]
    return Case("riemann_3d", seed, prm, (rho, ux, uy, uz, p), steps,
                dict(left=left, right=right, normal=n.tolist()))


def shock_bubble(seed: int, grid=(256, 128, 128), steps: int = 2000, precision=FP32_T64,
                 mach=None, ratio=None, **model) -> Case:
    """Planar shock travelling in +x into quiescent gas (rho, p) = (1, 1),
    hitting a sphere of equal pressure and density ratio `ratio` (a light
    bubble or a heavy droplet) whose surface is smoothed over one cell.
    Geometry scales with the grid: at 256x128x128 the shock starts at x = 60
    and the sphere (radius 20 cells) sits at (96, 64, 64).  Mach ~ U[1.5, 8]; ratio log-uniform on [0.1, 10].
    x: fixed post-shock inflow at -x, extrapolation outflow at +x; y and z
    reflecting walls (the paper's set-up, mirrored in x)."""
    rng = np.random.default_rng(seed)
    if mach is None:
        mach = rng.uniform(1.5, 8.0)
    if ratio is None:
        ratio = math.exp(rng.uniform(math.log(0.1), math.log(10.0)))
    nx, ny, nz = grid
    gamma = model.get("gamma", MODEL["gamma"])
    rho2, u2, p2, D = rankine_hugoniot(mach, 1.0, 1.0, gamma)
    post = (rho2, u2, 0.0, 0.0, p2)
    prm = make_params(grid, (INFLOW, OUTFLOW, REFLECT, REFLECT, REFLECT, REFLECT),
                      inflow={0: post}, precision=precision, **model)
    xs = 60.0 * nx / 256.0
    cx, cy, cz = 0.375 * nx, 0.5 * ny, 0.5 * nz
    r = 20.0 * ny / 128.0
    zz, yy, xx = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                             np.arange(nx, dtype=np.float64), indexing="ij")
    rho = np.ones((nz, ny, nx))
    ux = np.zeros((nz, ny, nx))
    uy = np.zeros((nz, ny, nx))
    uz = np.zeros((nz, ny, nx))
    p = np.ones((nz, ny, nx))
    # density 1 outside and `ratio` inside the sphere, blended over about one
    # cell with a tanh profile so the stair-stepped surface has no one-node
    # protrusions
    dist = np.sqrt((xx - cx) ** 2 + (yy - cy) ** 2 + (zz - cz) ** 2)
    rho[...] = 1.0 + (ratio - 1.0) * 0.5 * (1.0 - np.tanh((dist - r) / 1.0))
    shocked = xx < xs
    rho[shocked] = rho2
    ux[shocked] = u2
    p[shocked] = p2
    return Case("shock_bubble", seed, prm, (rho, ux, uy, uz, p), steps,
                dict(mach=mach, ratio=ratio, post=post, D=D, shock_x=xs, centre=(cx, cy, cz),
                     radius=r))


# The paper's own shock-bubble and shock-droplet runs (Sec. 4 (2), Eqs.
# (light) and (heavy)).
PAPER_BUBBLE_MODEL = dict(c1=2.0, c2=6.0, eta0=4.0, gamma=1.4, tau=1e-5, dt=1e-5, dx=0.001)
PAPER_POST_SHOCK = (2.66667, -1.47902, 0.0, 0.0, 4.5)  # p = 4.5 (the printed 3.94406 is rho |u|)
PAPER_SPHERE_DENSITY = {"bubble": 0.1358, "droplet": 4.1538}


def paper_shock_bubble(kind: str = "bubble", precision=FP64, radius: float = 20.0, shock_x: float = 230.0,
                       smooth: float = 1.0, steps: int = 10000) -> Case:
    """The paper's planar Mach-2 shock running right to left into a light
    bubble (rho = 0.1358) or a heavy droplet (rho = 4.1538) at rest with
    p = 1, in quiescent gas (1, 0, 0, 0, 1).  The paper's node indices run
    over (0:301, 0:81, 0:81) and include the two boundary-node layers of
    every face, so the interior is 298 x 78 x 78 and the sphere's centre,
    node (200, 40, 40), is interior node (198, 38, 38).  Faces: the post-shock
    state fixed at +x, extrapolation at -x, reflecting walls in y and z.
    (c1, c2, eta0) = (2, 6, 4), gamma = 1.4, dx = 0.001, dt = tau = 1e-5;
    t = 0.1 is 10000 steps.  Not stated by the paper and chosen here: the
    sphere's radius (20 nodes, half the tube's width across), the shock's
    start (paper node x = 230, 10 nodes to the right of the sphere) and a
    density jump blended over `smooth` cells (0: a sharp, stair-stepped
    surface)."""
    if kind not in PAPER_SPHERE_DENSITY:
        raise ValueError(f"kind must be one of {sorted(PAPER_SPHERE_DENSITY)}")
    grid = (298, 78, 78)
    nx, ny, nz = grid
    prm = make_params(grid, (OUTFLOW, INFLOW, REFLECT, REFLECT, REFLECT, REFLECT),
                      inflow={1: PAPER_POST_SHOCK}, precision=precision, **PAPER_BUBBLE_MODEL)
    # interior node i is the paper's node i + 2
    cx, cy, cz = 200.0 - 2, 40.0 - 2, 40.0 - 2
    xs = shock_x - 2
    zz, yy, xx = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                             np.arange(nx, dtype=np.float64), indexing="ij")
    dist = np.sqrt((xx - cx) ** 2 + (yy - cy) ** 2 + (zz - cz) ** 2)
    inside = PAPER_SPHERE_DENSITY[kind]
    if smooth > 0:
        rho = 1.0 + (inside - 1.0) * 0.5 * (1.0 - np.tanh((dist - radius) / smooth))
    else:
        rho = np.where(dist <= radius, inside, 1.0)
    ux = np.zeros_like(rho)
    p = np.ones_like(rho)
    post = xx > xs
    rho[post] = PAPER_POST_SHOCK[0]
    ux[post] = PAPER_POST_SHOCK[1]
    p[post] = PAPER_POST_SHOCK[4]
    z = np.zeros_like(rho)
    return Case(f"paper_shock_{kind}", 0, prm, (rho, ux, z, z.copy(), p), steps,
                dict(kind=kind, radius=radius, shock_x=shock_x, centre=(cx, cy, cz), smooth=smooth))


def batch_cases(seed: int, count: int = 64, steps: int = 500, precision=FP32_T64,
                grids=BATCH_GRIDS) -> list:
    """Independent solves of uneven size: grid drawn from `grids`, a 3D
    Riemann problem or a shock-bubble problem with probability 1/2 each."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        g = grids[int(rng.integers(len(grids)))]
        sub = int(rng.integers(2 ** 31 - 1))
        if rng.random() < 0.5:
            out.append(riemann_3d(sub, grid=g, steps=steps, precision=precision))
        else:
            out.append(shock_bubble(sub, grid=g, steps=steps, precision=precision))
    return out


def serve_trace(seed: int, count: int = 64, rate: float = 10.0, grids=SERVE_GRIDS,
                steps_range=(200, 3000), precision=FP32_T64) -> list:
    """Open arrival stream: (arrival time in s, Case) pairs with Poisson
    arrivals of the given rate; grid, problem kind and step count drawn per
    request (steps ~ U{200..3000}, shock Mach ~ U[1.5, 8])."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(count):
        t += rng.exponential(1.0 / rate)
        g = grids[int(rng.integers(len(grids)))]
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        sub = int(rng.integers(2 ** 31 - 1))
        if rng.random() < 0.5:
            c = riemann_3d(sub, grid=g, steps=steps, precision=precision)
        else:
            c = shock_bubble(sub, grid=g, steps=steps, precision=precision)
        out.append((t, c))
    return out


def fixed_states():
    """A fixed (rho, ux, uy, uz, p) per face (-x, +x, -y, +y, -z, +z): subsonic
    states near smooth_periodic's mean, each flowing into or along its face,
    for cases that hold fixed-state faces on any axis."""
    return [[1.2, 0.3, 0.0, 0.05, 1.1],
            [0.9, -0.25, 0.05, 0.0, 0.95],
            [1.1, 0.0, 0.2, -0.05, 1.0],
            [0.95, 0.05, -0.15, 0.0, 1.05],
            [1.05, -0.05, 0.0, 0.25, 0.9],
            [1.0, 0.0, 0.05, -0.2, 1.1]]


def smooth_periodic(seed: int, grid=(24, 20, 16), amp: float = 0.2, precision=FP64, **model) -> Case:
    """Smooth random periodic state (a few low Fourier modes per field);
    used for conservation and symmetry checks."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = grid
    zz, yy, xx = np.meshgrid(np.arange(nz) / nz, np.arange(ny) / ny, np.arange(nx) / nx,
                             indexing="ij")

    def field():
        out = np.zeros((nz, ny, nx))
        for _ in range(3):
            k = rng.integers(-2, 3, size=3)
            ph = rng.uniform(0, 2 * math.pi)
            out += rng.uniform(-1, 1) * np.cos(2 * math.pi * (k[0] * xx + k[1] * yy + k[2] * zz) + ph)
        return out / 3.0

    rho = 1.0 + amp * field()
    p = 1.0 + amp * field()
    ux, uy, uz = (amp * 2.0 * field() for _ in range(3))
    prm = make_params(grid, (PERIODIC,) * 6, precision=precision, **model)
    return Case("smooth_periodic", seed, prm, (rho, ux, uy, uz, p), 20)
