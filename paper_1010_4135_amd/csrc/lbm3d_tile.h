// The fused FD-LB time step on one tile of 64 x BY nodes marching along z.
//
// Data flow per tile (a workgroup of BY wavefronts, one x-row of 64 nodes
// per wavefront):
//   - every thread keeps, per velocity, a short queue of its column's values
//     along z (f at z-1 .. z+2 as the upwind side needs) in registers, plus
//     the NND face value g_{z-1/2} of the previous z step, so the z
//     direction costs one new face per velocity and step and one global
//     load per velocity (the plane two or three ahead, prefetched);
//   - the current z plane of all 15 velocities is staged in LDS with the
//     face halo the x and y stencils need (two nodes on the upwind side, one
//     on the other; one on each side for the dissipation of the rest and
//     axis velocities).  Halo rows are read by whole wavefronts (64
//     consecutive x); the halo columns of a row are gathered into one
//     register per wavefront.  The halo of the next plane is loaded while
//     the current one is computed, so the LDS barriers are the only waits on
//     the critical path;
//   - moments, equilibrium, NND convection in x, y, z, dissipation and the
//     BGK forward-Euler update are evaluated in registers and each new f is
//     written once;
//   - nodes next to a periodic or reflecting face (and to an x outflow face)
//     also write the boundary layers of the new level, so no second kernel
//     is needed for them.
// Per node, the arithmetic is the same sequence of operations as a direct
// evaluation of the stencil, so results do not depend on the tile shape.
#pragma once

#include "lbm3d_model.h"

namespace lbm3d {

constexpr int TILE_X = 64;

// Build-time tuning knobs of the sweep (defaults are the tuned choice):
// LBM3D_HALO_PREFETCH loads the next plane's halo during the current
// plane's compute (1) or right before staging it (0).
#ifndef LBM3D_HALO_PREFETCH
#define LBM3D_HALO_PREFETCH 1
#endif

// Workgroup barrier that orders LDS accesses only: global loads in flight
// (the prefetch of the planes ahead) and global stores are not drained.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int BY, typename S>
struct TilePlane {
    S v[NV][BY + 4][TILE_X + 4];
};

// Halo rows of velocity i for a tile of height BY: y offsets relative to the
// tile origin.  v_y > 0: -2, -1, BY; v_y < 0: -1, BY, BY+1; v_y = 0 (rest and
// x/z axis velocities, which carry dissipation): -1, BY.
__host__ __device__ constexpr int halo_rows(int i) { return vsign(i, 1) == 0 ? 2 : 3; }
__host__ __device__ constexpr int halo_row(int i, int k, int by)
{
    return vsign(i, 1) > 0 ? (k == 0 ? -2 : (k == 1 ? -1 : by))
         : vsign(i, 1) < 0 ? (k == 0 ? -1 : (k == 1 ? by : by + 1))
                           : (k == 0 ? -1 : by);
}
__host__ __device__ constexpr int halo_jobs()
{
    int n = 0;
    for (int i = 0; i < NV; i++) n += halo_rows(i);
    return n;
}

// Job table of the halo rows: entry j = (velocity << 2) | code, code 0..3
// for row offsets -2, -1, BY, BY+1.  Wavefront w of a tile stages jobs
// w, w+BY, w+2BY, ... (a uniform index, so decoding is scalar work).
struct HaloJobs {
    uint8_t e[64];
};
__host__ __device__ constexpr HaloJobs make_halo_jobs()
{
    HaloJobs t{};
    int n = 0;
    for (int i = 0; i < NV; i++)
        for (int k = 0; k < halo_rows(i); k++) {
            const int r = halo_row(i, k, 1000);
            const int code = r == -2 ? 0 : (r == -1 ? 1 : (r == 1000 ? 2 : 3));
            t.e[n++] = (uint8_t)((i << 2) | code);
        }
    return t;
}
__constant__ const HaloJobs kHaloJobs = make_halo_jobs();

// Everything a tile needs about its solve.
template <int MODE>
struct StepArgs {
    using S = typename Types<MODE>::S;
    Grid g;
    FaceBC bc;
    uint32_t fused;  // faces whose boundary layers the step kernel writes itself
    const S* f;
    S* fn;
    uint32_t* health;
};

// Extrapolated boundary states of Sec. 4 (2): layer 1 = 2 q(i0) - q(i1),
// layer 2 = 2 (layer 1) - q(i0).
template <typename M>
__device__ __forceinline__ void extrapolate(const Macro<M>& a, const Macro<M>& b, Macro<M>& l1, Macro<M>& l2)
{
    l1.rho = M(2) * a.rho - b.rho;
    l1.ux = M(2) * a.ux - b.ux;
    l1.uy = M(2) * a.uy - b.uy;
    l1.uz = M(2) * a.uz - b.uz;
    l1.T = M(2) * a.T - b.T;
    l2.rho = M(2) * l1.rho - a.rho;
    l2.ux = M(2) * l1.ux - a.ux;
    l2.uy = M(2) * l1.uy - a.uy;
    l2.uz = M(2) * l1.uz - a.uz;
    l2.T = M(2) * l1.T - a.T;
}

// Reflecting wall (Sec. 4 (2)): wall layer = q with zero normal velocity,
// mirror layer = q with the normal velocity negated.
template <typename M>
__device__ __forceinline__ void reflect(const Macro<M>& a, int axis, Macro<M>& wall, Macro<M>& mirror)
{
    wall = a;
    mirror = a;
    if (axis == 0) {
        wall.ux = M(0);
        mirror.ux = -a.ux;
    } else if (axis == 1) {
        wall.uy = M(0);
        mirror.uy = -a.uy;
    } else {
        wall.uz = M(0);
        mirror.uz = -a.uz;
    }
}

template <typename S, typename C>
__device__ __forceinline__ void store_node(S* __restrict__ fn, int64_t sv, uint32_t off, const C (&v)[NV])
{
#pragma unroll
    for (int i = 0; i < NV; i++) (fn + i * sv)[off] = static_cast<S>(v[i]);
}

template <typename M>
__device__ __forceinline__ Macro<M> shfl_macro(const Macro<M>& q, int src_lane)
{
    Macro<M> r;
    r.rho = __shfl(q.rho, src_lane);
    r.ux = __shfl(q.ux, src_lane);
    r.uy = __shfl(q.uy, src_lane);
    r.uz = __shfl(q.uz, src_lane);
    r.T = __shfl(q.T, src_lane);
    return r;
}

// Periodic copies: bit k set if boundary-layer slot k (-2, -1, n, n+1) of an
// axis of n nodes is a copy of node c.
__device__ __forceinline__ int wrap_mask(int c, int n)
{
    int m = 0;
    if (((-2 % n) + n) % n == c) m |= 1;
    if (((-1 % n) + n) % n == c) m |= 2;
    if (n % n == c) m |= 4;
    if ((n + 1) % n == c) m |= 8;
    return m;
}
__device__ __forceinline__ int wrap_slot(int k, int n) { return k == 0 ? -2 : k == 1 ? -1 : k == 2 ? n : n + 1; }

template <int MODE, int BY>
__device__ __forceinline__ void step_tile(const StepArgs<MODE>& A, const Model<double>& md,
                                          const Model<float>& mf, int x0, int y0, int z0, int z1,
                                          TilePlane<BY, typename Types<MODE>::S>& P)
{
    using S = typename Types<MODE>::S;
    using C = typename Types<MODE>::C;
    using M = typename Types<MODE>::M;
    const Model<C>& mc = pick<C>(md, mf);
    const Model<M>& mm = pick<M>(md, mf);
    const Grid& g = A.g;
    const S* __restrict__ f = A.f;
    S* __restrict__ fn = A.fn;

    const int tx = threadIdx.x & (TILE_X - 1);
    const int ty = threadIdx.x / TILE_X;
    const int wave = __builtin_amdgcn_readfirstlane(ty);
    const int x = x0 + tx, y = y0 + ty;
    const bool act = (x < g.nx) && (y < g.ny);
    // every load is clamped into the padded array: nodes beyond the last
    // boundary layer are never read by an active node's stencil.  Velocity
    // planes are addressed as a uniform base pointer plus one 32-bit
    // per-thread offset (a velocity plane holds < 2^31 elements).
    const int xl = min(x, g.nx + 1), yl = min(y, g.ny + 1);
    const int64_t sv = g.sv;
    const uint32_t sy = (uint32_t)g.sy, sz = (uint32_t)g.sz;
    const uint32_t col = (uint32_t)(g.org + (int64_t)yl * g.sy + xl);
    const uint32_t rowoff = (uint32_t)(g.org + xl);

    C q[NV][4];  // f at z-1, z, z+1, z+2 along this thread's column
    C gp[NV];    // NND face value g_{z-1/2} of the z-advected velocities
#pragma unroll
    for (int i = 0; i < NV; i++) {
        const S* fi = f + i * sv;
        q[i][0] = static_cast<C>(fi[col + (uint32_t)(z0 - 1) * sz]);
        q[i][1] = static_cast<C>(fi[col + (uint32_t)z0 * sz]);
        q[i][2] = static_cast<C>(fi[col + (uint32_t)(z0 + 1) * sz]);
        q[i][3] = C(0);
        gp[i] = C(0);
        if (vsign(i, 2) < 0) {
            q[i][3] = static_cast<C>(fi[col + (uint32_t)(z0 + 2) * sz]);
            gp[i] = face_neg(q[i][0], q[i][1], q[i][2]);
        } else if (vsign(i, 2) > 0) {
            const C fm2 = static_cast<C>(fi[col + (uint32_t)(z0 - 2) * sz]);
            gp[i] = face_pos(fm2, q[i][0], q[i][1]);
        }
    }

    // x halo of this wavefront's row, gathered into one register: lane
    // 4v + p holds velocity v at x0-2, x0-1, x0+64, x0+65 for p = 0..3
    const int hv = min(tx >> 2, NV - 1), hp = tx & 3;
    const int hx = min(hp == 0 ? x0 - 2 : hp == 1 ? x0 - 1 : hp == 2 ? x0 + TILE_X : x0 + TILE_X + 1, g.nx + 1);
    const S* hptr = f + hv * sv + (g.org + (int64_t)yl * g.sy + hx);
    const int hcol = hp < 2 ? hp : hp + TILE_X;
    const bool hlane = tx < 4 * NV;
    // halo rows of this wavefront: jobs wave, wave + BY, ...
    constexpr int NJ = halo_jobs();
    static_assert(NJ % BY == 0, "every wavefront stages the same number of halo rows");
    constexpr int NK = NJ / BY;
    S hrow[NK];
    S hcolv = S(0);
#pragma unroll
    for (int k = 0; k < NK; k++) hrow[k] = S(0);
    auto load_halo = [&](int zz) {
        const uint32_t zo = (uint32_t)zz * sz;
        hcolv = hptr[zo];
#pragma unroll
        for (int k = 0; k < NK; k++) {
            const int e = kHaloJobs.e[wave + k * BY];
            const int i = e >> 2, code = e & 3;
            const int r = code < 2 ? code - 2 : BY + code - 2;
            const uint32_t yh = (uint32_t)min(y0 + r, g.ny + 1);
            hrow[k] = (f + i * sv)[rowoff + yh * sy + zo];
        }
    };
    auto store_halo = [&]() {
        if (hlane) P.v[hv][ty + 2][hcol] = hcolv;
#pragma unroll
        for (int k = 0; k < NK; k++) {
            const int e = kHaloJobs.e[wave + k * BY];
            const int i = e >> 2, code = e & 3;
            const int r = code < 2 ? code - 2 : BY + code - 2;
            P.v[i][r + 2][tx + 2] = hrow[k];
        }
    };
    load_halo(z0);

    // Every memory operation of the sweep is unconditional, so the
    // compiler's wait counts stay exact (on this architecture loads and
    // stores share one in-order counter): lanes outside the grid compute on
    // clamped data and store to a sink element past the end of each velocity
    // plane that is never read; the prefetch past the last plane is clamped.
    const uint32_t sink = (uint32_t)g.sink;
    uint32_t hacc = 0;
    // plane z0 is staged before the sweep; plane z+1 at the end of step z
#pragma unroll
    for (int i = 0; i < NV; i++) P.v[i][ty + 2][tx + 2] = static_cast<S>(q[i][1]);
    store_halo();
    for (int z = z0; z < z1; z++) {
        const uint32_t zo = (uint32_t)z * sz;
        // start the loads of the next plane's halo and of the planes ahead
        C nxt[NV];
        {
            if (LBM3D_HALO_PREFETCH) load_halo(min(z + 1, g.nz));
            const uint32_t o2 = col + (uint32_t)min(z + 2, g.nz + 1) * sz;
            const uint32_t o3 = col + (uint32_t)min(z + 3, g.nz + 1) * sz;
#pragma unroll
            for (int i = 0; i < NV; i++) {
                const S* fi = f + i * sv;
                nxt[i] = static_cast<C>(fi[vsign(i, 2) < 0 ? o3 : o2]);
            }
        }
        lds_barrier();
        {
            C fc[NV];
#pragma unroll
            for (int i = 0; i < NV; i++) fc[i] = q[i][1];
            const Macro<M> mac = moments<M, C>(fc, mm);
            hacc |= health_bits(mac);
            C feq[NV];
            equilibrium<C, M>(mac, mm, mc, feq);
            const uint32_t out = act ? col + zo : sink;
#pragma unroll
            for (int i = 0; i < NV; i++) {
                const int sx = vsign(i, 0), syy = vsign(i, 1), szz = vsign(i, 2), grp = vgroup(i);
                const C vm = (grp == 1) ? mc.c1 : mc.k;
                const C f0 = q[i][1];
                const S* row = &P.v[i][ty + 2][tx + 2];
                C xm1 = C(0), xp1 = C(0), ym1 = C(0), yp1 = C(0);
                C conv = C(0);
                if (sx != 0 || grp <= 1) {
                    xm1 = static_cast<C>(row[-1]);
                    xp1 = static_cast<C>(row[1]);
                }
                if (syy != 0 || grp <= 1) {
                    ym1 = static_cast<C>(row[-(TILE_X + 4)]);
                    yp1 = static_cast<C>(row[TILE_X + 4]);
                }
                if (sx > 0) conv += vm * nnd_diff<1, C>(static_cast<C>(row[-2]), xm1, f0, xp1, C(0));
                if (sx < 0) conv -= vm * nnd_diff<-1, C>(C(0), xm1, f0, xp1, static_cast<C>(row[2]));
                if (syy > 0)
                    conv += vm * nnd_diff<1, C>(static_cast<C>(row[-2 * (TILE_X + 4)]), ym1, f0, yp1, C(0));
                if (syy < 0)
                    conv -= vm * nnd_diff<-1, C>(C(0), ym1, f0, yp1, static_cast<C>(row[2 * (TILE_X + 4)]));
                if (szz > 0) {
                    const C gz = face_pos(q[i][0], q[i][1], q[i][2]);
                    conv += vm * (gz - gp[i]);
                    gp[i] = gz;
                }
                if (szz < 0) {
                    const C gz = face_neg(q[i][1], q[i][2], q[i][3]);
                    conv -= vm * (gz - gp[i]);
                    gp[i] = gz;
                }
                C ov = f0 - mc.k_adv * conv - mc.k_bgk * (f0 - feq[i]);
                if (grp <= 1) {
                    const C lap = ((xm1 + xp1) + (ym1 + yp1)) + (q[i][0] + q[i][2]) - C(6) * f0;
                    ov += (grp == 0 ? mc.k_lap0 : mc.k_lap1) * lap;
                }
                (fn + i * sv)[out] = static_cast<S>(ov);
            }

        }
        lds_barrier();
#pragma unroll
        for (int i = 0; i < NV; i++) {
            q[i][0] = q[i][1];
            q[i][1] = q[i][2];
            if (vsign(i, 2) < 0) {
                q[i][2] = q[i][3];
                q[i][3] = nxt[i];
            } else {
                q[i][2] = nxt[i];
            }
        }
        // stage plane z+1: own values and its halo
#pragma unroll
        for (int i = 0; i < NV; i++) P.v[i][ty + 2][tx + 2] = static_cast<S>(q[i][1]);
        if (!LBM3D_HALO_PREFETCH) load_halo(min(z + 1, g.nz));
        store_halo();
    }
    if (act && hacc) atomicOr(A.health, hacc);

    // ---- boundary layers of the new level (Sec. 4 (2)).  The node next to
    // each periodic, reflecting or (x) outflow face writes them after the
    // sweep, from its new values read back (this thread stored them, so the
    // reads see them); keeping this out of the sweep keeps its register
    // footprint small.  Edges and corners of the layers are never read.
    // ---- which boundary layers of the new level this node writes
    const int nxg = g.nx, nyg = g.ny, nzg = g.nz;
    auto kind_fused = [&](int face, int kind) { return ((A.fused >> face) & 1) && A.bc.kind[face] == kind; };
    const int pxm = (act && kind_fused(0, BC_PERIODIC)) ? wrap_mask(x, nxg) : 0;
    const int pym = (act && kind_fused(2, BC_PERIODIC)) ? wrap_mask(y, nyg) : 0;
    const bool pz = kind_fused(4, BC_PERIODIC);
    const bool rx_lo = act && x == 0 && kind_fused(0, BC_REFLECT);
    const bool rx_hi = act && x == nxg - 1 && kind_fused(1, BC_REFLECT);
    const bool ry_lo = act && y == 0 && kind_fused(2, BC_REFLECT);
    const bool ry_hi = act && y == nyg - 1 && kind_fused(3, BC_REFLECT);
    // outflow along x: the node next to the face pairs with its x neighbour,
    // which sits in the adjacent lane (the host fuses this face only then)
    const bool ox_lo_t = x0 == 0 && kind_fused(0, BC_OUTFLOW);  // tile-uniform
    const bool ox_hi_t = x0 <= nxg - 1 && nxg - 1 < x0 + TILE_X && kind_fused(1, BC_OUTFLOW);
    const bool ox_lo = act && x == 0 && ox_lo_t, ox_hi = act && x == nxg - 1 && ox_hi_t;
    const bool ox_src = act && ((x == 1 && ox_lo_t) || (x == nxg - 2 && ox_hi_t));
    const bool xy_bnd = (pxm | pym) || rx_lo || rx_hi || ry_lo || ry_hi || ox_lo || ox_hi || ox_src;
    const bool ox_t = ox_lo_t || ox_hi_t;

    const bool zlo_t = z0 == 0 && (kind_fused(4, BC_PERIODIC) || kind_fused(4, BC_REFLECT));
    const bool zhi_t = z1 >= nzg - 1 && (pz || kind_fused(5, BC_REFLECT));
    if (!(xy_bnd || zlo_t || zhi_t || (pz && z0 < 2)) ) return;
    for (int z = z0; z < z1; z++) {
        const int pzm = (pz && (z < 2 || z >= nzg - 2)) ? wrap_mask(z, nzg) : 0;
        const bool rz_lo = z == 0 && kind_fused(4, BC_REFLECT);
        const bool rz_hi = z == nzg - 1 && kind_fused(5, BC_REFLECT);
        if (!(act && (xy_bnd || pzm || rz_lo || rz_hi))) continue;
        const uint32_t out = col + (uint32_t)z * sz;
        C o[NV];
#pragma unroll
        for (int i = 0; i < NV; i++) o[i] = static_cast<C>((fn + i * sv)[out]);
#pragma unroll
        for (int k = 0; k < 4; k++) {
            if ((pxm >> k) & 1) store_node(fn, sv, out + (uint32_t)(wrap_slot(k, nxg) - x), o);
            if ((pym >> k) & 1) store_node(fn, sv, out + (uint32_t)(wrap_slot(k, nyg) - y) * sy, o);
            if ((pzm >> k) & 1) store_node(fn, sv, out + (uint32_t)(wrap_slot(k, nzg) - z) * sz, o);
        }
        if (rx_lo || rx_hi || ry_lo || ry_hi || rz_lo || rz_hi || ox_lo || ox_hi || ox_src) {
            const Macro<M> qn = moments<M, C>(o, mm);
            Macro<M> l1, l2;
            C e[NV];
            auto emit = [&](uint32_t off1, uint32_t off2) {
                equilibrium<C, M>(l1, mm, mc, e);
                store_node(fn, sv, off1, e);
                equilibrium<C, M>(l2, mm, mc, e);
                store_node(fn, sv, off2, e);
            };
            if (rx_lo) { reflect(qn, 0, l1, l2); emit(out - 1u, out - 2u); }
            if (rx_hi) { reflect(qn, 0, l1, l2); emit(out + 1u, out + 2u); }
            if (ry_lo) { reflect(qn, 1, l1, l2); emit(out - sy, out - 2u * sy); }
            if (ry_hi) { reflect(qn, 1, l1, l2); emit(out + sy, out + 2u * sy); }
            if (rz_lo) { reflect(qn, 2, l1, l2); emit(out - sz, out - 2u * sz); }
            if (rz_hi) { reflect(qn, 2, l1, l2); emit(out + sz, out + 2u * sz); }
            if (ox_t) {
                // the outflow pair: the x neighbour's new state from the adjacent lane
                const Macro<M> qr = shfl_macro(qn, min(tx + 1, TILE_X - 1));
                const Macro<M> ql = shfl_macro(qn, max(tx - 1, 0));
                if (ox_lo) { extrapolate(qn, qr, l1, l2); emit(out - 1u, out - 2u); }
                if (ox_hi) { extrapolate(qn, ql, l1, l2); emit(out + 1u, out + 2u); }
            }
        }
    }
}

// Tile order: tiles are numbered with y fastest, then x, then the z chunk,
// and consecutive numbers are given to workgroups that land on the same
// XCD (dispatch assigns workgroup b to XCD b mod 8), so that tiles sharing
// halo rows share an L2.
__device__ __forceinline__ int xcd_tile(int b, int nblocks)
{
    const int per = nblocks >> 3, rem = nblocks & 7;
    const int xcd = b & 7, slot = b >> 3;
    return xcd * per + min(xcd, rem) + slot;
}

}  // namespace lbm3d
