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
//   - the boundary layers of the new level are written by a separate,
//     light launch (one thread per boundary line); a build option moves
//     the periodic and reflecting ones into the tiles next to the face.
// Per node, the arithmetic is the same sequence of operations as a direct
// evaluation of the stencil, so results do not depend on the tile shape.
#pragma once

#include "lbm3d_model.h"

namespace lbm3d {

// Build-time tuning knobs of the sweep (defaults are the tuned choice):
// LBM3D_HALO_PREFETCH loads the next plane's halo during the current
// plane's compute (1) or right before staging it (0).
#ifndef LBM3D_HALO_PREFETCH
#define LBM3D_HALO_PREFETCH 1
#endif
// LBM3D_FUSE_LAYERS: 1 = the tiled step writes the boundary layers whose
// source nodes a tile owns (after its sweep); 0 = a separate launch of the
// boundary-layer kernel writes all of them.
#ifndef LBM3D_FUSE_LAYERS
#define LBM3D_FUSE_LAYERS 0
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

// Does a tile owning nodes [lo, hi) along an axis of n nodes write layer
// nodes of this face?  Periodic: a layer node copies node (slot mod n), and
// the owner of that node writes it.  Reflecting / extrapolating: the owner
// of the node next to the face (the host fuses an extrapolating face only if
// the second node in lies in the same tile).
__device__ __forceinline__ bool layer_owner(int kind, int side, int n, int lo, int hi)
{
    if (kind == BC_INFLOW) return false;
    if (kind == BC_PERIODIC) {
        const int s1 = side ? (n % n) : (((-1 % n) + n) % n);
        const int s2 = side ? ((n + 1) % n) : (((-2 % n) + n) % n);
        return (s1 >= lo && s1 < hi) || (s2 >= lo && s2 < hi);
    }
    const int i0 = side ? n - 1 : 0;
    return i0 >= lo && i0 < hi;
}

// Layer nodes of one face on the line through `line` (offset of the line's
// node 0 along the axis, node stride st), for a tile owning [lo, hi).
template <int MODE>
__device__ __forceinline__ void layer_line(const StepArgs<MODE>& A, const Model<typename Types<MODE>::M>& mm,
                                           const Model<typename Types<MODE>::C>& mc, int face, uint32_t line,
                                           uint32_t st, int n, int lo, int hi)
{
    using S = typename Types<MODE>::S;
    using C = typename Types<MODE>::C;
    using M = typename Types<MODE>::M;
    const int64_t sv = A.g.sv;
    S* __restrict__ fn = A.fn;
    const int side = face & 1, kind = A.bc.kind[face], axis = face >> 1;
    const int g1 = side ? n : -1, g2 = side ? n + 1 : -2;  // wall / first layer, second layer
    auto at = [&](int c) { return line + (uint32_t)c * st; };
    C a[NV];
    if (kind == BC_PERIODIC) {
        const int gs[2] = {g1, g2};
#pragma unroll
        for (int k = 0; k < 2; k++) {
            const int src = ((gs[k] % n) + n) % n;
            if (src < lo || src >= hi) continue;
#pragma unroll
            for (int i = 0; i < NV; i++) a[i] = static_cast<C>((fn + i * sv)[at(src)]);
            store_node(fn, sv, at(gs[k]), a);
        }
        return;
    }
    const int i0 = side ? n - 1 : 0, i1 = side ? n - 2 : 1;
#pragma unroll
    for (int i = 0; i < NV; i++) a[i] = static_cast<C>((fn + i * sv)[at(i0)]);
    const Macro<M> q0 = moments<M, C>(a, mm);
    Macro<M> l1, l2;
    if (kind == BC_REFLECT) {
        reflect(q0, axis, l1, l2);
    } else {  // BC_OUTFLOW
#pragma unroll
        for (int i = 0; i < NV; i++) a[i] = static_cast<C>((fn + i * sv)[at(i1)]);
        const Macro<M> q1 = moments<M, C>(a, mm);
        extrapolate(q0, q1, l1, l2);
    }
    equilibrium<C, M>(l1, mm, mc, a);
    store_node(fn, sv, at(g1), a);
    equilibrium<C, M>(l2, mm, mc, a);
    store_node(fn, sv, at(g2), a);
}

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

    // ---- boundary layers of the new level (Sec. 4 (2)).  After the sweep,
    // the tile writes the layers whose source nodes it owns, as dense "line
    // jobs" spread over all its threads: one job is one line of nodes
    // perpendicular to a face; it reads back the one or two new nodes next
    // to the face (written above by this workgroup; the barrier makes them
    // visible) and writes the two layer nodes.  Edges and corners of the
    // layers are never read.
#if !LBM3D_FUSE_LAYERS
    if (act && hacc) atomicOr(A.health, hacc);
    return;
#else
    const int zc = z1 - z0;
    const int xe = min(x0 + TILE_X, g.nx), ye = min(y0 + BY, g.ny);
    bool work[6];
#pragma unroll
    for (int face = 0; face < 6; face++) {
        const int axis = face >> 1;
        const int lo = axis == 0 ? x0 : axis == 1 ? y0 : z0;
        const int hi = axis == 0 ? xe : axis == 1 ? ye : z1;  // tile owns nodes [lo, hi) along axis
        const int n = axis == 0 ? g.nx : axis == 1 ? g.ny : g.nz;
        work[face] = ((A.fused >> face) & 1) && layer_owner(A.bc.kind[face], face & 1, n, lo, hi);
    }
    if (!(work[0] || work[1] || work[2] || work[3] || work[4] || work[5])) {
        if (act && hacc) atomicOr(A.health, hacc);
        return;
    }
    if (act && hacc) atomicOr(A.health, hacc);
    __syncthreads();
    const int nthr = TILE_X * BY;
#pragma unroll
    for (int face = 0; face < 6; face++) {
        if (!work[face]) continue;
        const int axis = face >> 1;
        // lines of this face inside the tile: the two other coordinates
        const int cnt = axis == 0 ? (ye - y0) * zc : axis == 1 ? (xe - x0) * zc : (xe - x0) * (ye - y0);
        for (int j = threadIdx.x; j < cnt; j += nthr) {
            int cx = 0, cy = 0, cz = 0;
            if (axis == 0) { cy = y0 + j % (ye - y0); cz = z0 + j / (ye - y0); }
            else if (axis == 1) { cx = x0 + j % (xe - x0); cz = z0 + j / (xe - x0); }
            else { cx = x0 + j % (xe - x0); cy = y0 + j / (xe - x0); }
            const uint32_t line = (uint32_t)(g.org + (int64_t)cz * g.sz + (int64_t)cy * g.sy + cx);
            const uint32_t st = axis == 0 ? 1u : axis == 1 ? sy : sz;
            const int n = axis == 0 ? g.nx : axis == 1 ? g.ny : g.nz;
            const int lo = axis == 0 ? x0 : axis == 1 ? y0 : z0;
            const int hi = axis == 0 ? xe : axis == 1 ? ye : z1;
            layer_line<MODE>(A, mm, mc, face, line, st, n, lo, hi);
        }
    }
#endif
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
