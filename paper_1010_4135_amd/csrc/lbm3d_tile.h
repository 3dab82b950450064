// The fused FD-LB time step on one tile of 64 x BY nodes marching along z,
// and the boundary-layer rules of Sec. 4 (2).
//
// Data flow per tile (a workgroup of BY wavefronts, one x-row of 64 nodes
// per wavefront):
//   - along z every thread keeps, per velocity, a ring of four of its
//     column's values (z-1 .. z+2, or z .. z+3 for v_z < 0) and the minmod
//     of the previous z face, so z costs one global load, one new difference
//     and one minmod per velocity and plane; the z loop is unrolled over the
//     ring's four phases so that no value is ever moved, and each plane's
//     load goes straight into the ring slot it will be read from a plane
//     later;
//   - the current z plane of all 15 velocities is staged in LDS with the
//     halo the x and y stencils need (two nodes on the upwind side, one on
//     the other; one on each side for the dissipation of the rest and axis
//     velocities).  Two LDS planes alternate, so one barrier per plane
//     separates staging from reading.  Halo rows are read by whole
//     wavefronts (64 consecutive x) through a uniform job table; the halo
//     columns of a row are gathered into one register per wavefront; a
//     plane's halo is loaded two planes ahead, with the ring loads of the
//     same plane;
//   - global memory is addressed as a uniform (scalar) base per velocity
//     and plane plus one 32-bit per-lane byte offset;
//   - moments, equilibrium, NND convection in x, y, z, dissipation and the
//     BGK forward-Euler update are evaluated in registers and each new f is
//     written once.
// Per node the arithmetic is node_update() and the NND helpers, shared with
// the one-node-per-thread kernel, so results do not depend on the launch
// shape.
#pragma once

#include "lbm3d_model.h"

namespace lbm3d {


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
    const S* f;
    S* fn;
    uint32_t* health;
    double xin[2][5];  // fixed states of the x faces (rho, ux, uy, uz, T)
};

// State of boundary layer j (1: the layer next to the face, 2: the one
// beyond it) from the moments of the node next to the face (a) and of the
// node after that (b), Sec. 4 (2):
//  - extrapolating face: (rho, u, T) extrapolated linearly through b and
//    a, i.e. a + j (a - b);
//  - reflecting face: a with the normal velocity set to zero (layer 1, the
//    wall) or negated (layer 2, the mirror image).
// Both are one formula, q = a + c (a - b) with the normal velocity then
// scaled by m: (c, m) = (j, 1) when extrapolating, (0, 0) or (0, -1) when
// reflecting (c = 0 gives q = a exactly, whatever b).  A per-lane (c, m)
// then forms any layer without selecting between the two rules.
template <typename M>
__device__ __forceinline__ void layer_coefs(int kind, int j, M& c, M& m)
{
    const bool refl = kind == BC_REFLECT;
    const int ci = refl ? 0 : j;
    const int mi = refl ? 1 - j : 1;
    c = static_cast<M>(ci);
    m = static_cast<M>(mi);
}

template <typename M>
__device__ __forceinline__ Macro<M> layer_state(const Macro<M>& a, const Macro<M>& b, M c, M m, int axis)
{
    const M drho = a.rho - b.rho;
    const M dux = a.ux - b.ux;
    const M duy = a.uy - b.uy;
    const M duz = a.uz - b.uz;
    const M dT = a.T - b.T;
    Macro<M> q;
    q.rho = fmac(c, drho, a.rho);
    q.ux = fmac(c, dux, a.ux);
    q.uy = fmac(c, duy, a.uy);
    q.uz = fmac(c, duz, a.uz);
    q.T = fmac(c, dT, a.T);
    if (axis == 0) q.ux = m * q.ux;
    if (axis == 1) q.uy = m * q.uy;
    if (axis == 2) q.uz = m * q.uz;
    return q;
}

// A pointer into the distribution array as a global-space pointer: where
// the array's address comes from a table in memory rather than a kernel
// argument the compiler cannot tell it is global and would emit flat
// accesses, which every LDS wait then also waits for.
template <typename S>
__device__ __forceinline__ __attribute__((address_space(1))) S* gptr(S* p)
{
    return reinterpret_cast<__attribute__((address_space(1))) S*>(reinterpret_cast<uint64_t>(p));
}

template <typename P, typename C>
__device__ __forceinline__ void store_node(P fn, int64_t sv, uint32_t off, const C (&v)[NV])
{
    using S = typename std::remove_reference<decltype(*fn)>::type;
#pragma unroll
    for (int i = 0; i < NV; i++) (fn + i * sv)[off] = static_cast<S>(v[i]);
}

// Layer node of a face: the first layer is read by every velocity's
// stencil, the second only by the velocities advected into the grid through
// that face (sign `in` along the axis), whose NND flux reaches two nodes
// upwind.  Only those values are written.
template <typename P, typename C>
__device__ __forceinline__ void store_layer(P fn, int64_t sv, uint32_t off, const C (&v)[NV],
                                            bool second, int axis, int in)
{
#pragma unroll
    for (int i = 0; i < NV; i++)
        if (!second || vsign(i, axis) == in) (fn + i * sv)[off] = v[i];
}

// Boundary layers of one face on the line of nodes through `line` (offset
// of the line's node 0, node stride st along the face normal, n nodes; the
// layer nodes next to the face and beyond it at offsets l1 and l2):
// periodic copy, reflecting wall or linear extrapolation, the layer f being
// the equilibrium of the layer state.
template <int MODE>
__device__ __forceinline__ void layer_line(const StepArgs<MODE>& A, const Model<typename Types<MODE>::M>& mm,
                                           const Model<typename Types<MODE>::C>& mc, int face, uint32_t line,
                                           uint32_t st, int n, uint32_t l1, uint32_t l2)
{
    using C = typename Types<MODE>::C;
    using M = typename Types<MODE>::M;
    const int64_t sv = A.g.sv;
    const auto fn = gptr(A.fn);
    const int side = face & 1, kind = A.bc.kind[face], axis = face >> 1;
    const int g1 = side ? n : -1, g2 = side ? n + 1 : -2;  // wall / first layer, second layer
    const int in = side ? -1 : 1;
    auto at = [&](int c) { return line + (uint32_t)c * st; };
    C a[NV];
    if (kind == BC_PERIODIC) {
        const int gs[2] = {g1, g2};
        const uint32_t ls[2] = {l1, l2};
#pragma unroll
        for (int k = 0; k < 2; k++) {
            const int src = ((gs[k] % n) + n) % n;
#pragma unroll
            for (int i = 0; i < NV; i++)
                if (k == 0 || vsign(i, axis) == in) a[i] = static_cast<C>((fn + i * sv)[at(src)]);
            store_layer(fn, sv, ls[k], a, k == 1, axis, in);
        }
        return;
    }
    const int i0 = side ? n - 1 : 0, i1 = side ? n - 2 : 1;
#pragma unroll
    for (int i = 0; i < NV; i++) a[i] = static_cast<C>((fn + i * sv)[at(i0)]);
    const Macro<M> q0 = moments<M, C>(a, mm);
    Macro<M> q1 = q0;  // (unused by a reflecting face)
    if (kind == BC_OUTFLOW) {
#pragma unroll
        for (int i = 0; i < NV; i++) a[i] = static_cast<C>((fn + i * sv)[at(i1)]);
        q1 = moments<M, C>(a, mm);
    }
    M c1, m1, c2, m2;
    layer_coefs(kind, 1, c1, m1);
    layer_coefs(kind, 2, c2, m2);
    const Macro<M> q1s = layer_state(q0, q1, c1, m1, axis);
    const Macro<M> q2s = layer_state(q0, q1, c2, m2, axis);
    equilibrium<C, M>(q1s, mm, mc, a);
    store_layer(fn, sv, l1, a, false, axis, in);
    equilibrium<C, M>(q2s, mm, mc, a);
    store_layer(fn, sv, l2, a, true, axis, in);
}

// Ring slot of plane z + j of velocity I's column at unroll phase K: the
// ring holds planes z-1 .. z+2 (v_z >= 0) or z .. z+3 (v_z < 0).
template <int I>
__host__ __device__ constexpr int ring_slot(int j, int K)
{
    return vsign(I, 2) < 0 ? ((K + j) & 3) : ((K + j + 1) & 3);
}

// A uniform pointer made opaque to the optimiser: it stays in scalar
// registers and per-lane offsets are not re-associated into it, so each
// access is one scalar base plus one 32-bit lane offset (the base of the
// next velocity plane is one scalar add away).
template <typename T>
__device__ __forceinline__ T* sreg(T* p)
{
    uint64_t v = reinterpret_cast<uint64_t>(p);
    asm("" : "+s"(v));
    return reinterpret_cast<T*>(v);
}

// Global access through a uniform base pointer and a 32-bit byte offset
// (global address space, so the scalar-base form of the instruction applies).
// The offset is passed through an empty asm so that its zero extension is
// formed at the access (and matched there) rather than hoisted as a 64-bit
// value.
template <typename S>
__device__ __forceinline__ S ld_at(const S* base, uint32_t off)
{
    using GP = const __attribute__((address_space(1))) S*;
    asm("" : "+v"(off));
    return *reinterpret_cast<GP>(reinterpret_cast<uint64_t>(base) + (uint64_t)off);
}
// Stores of the new level.  NT: streaming (non-temporal): they are not read
// again in this step, and keeping them out of the L2 leaves it to the
// planes that neighbouring tiles read as their halos.  Otherwise plain,
// for solves whose two levels fit the memory-side cache, from which the
// next step then reads them (see STREAM_MIN_BYTES).
template <bool NT, typename S>
__device__ __forceinline__ void st_at(S* base, uint32_t off, S v)
{
    using GP = __attribute__((address_space(1))) S*;
    asm("" : "+v"(off));
    GP p = reinterpret_cast<GP>(reinterpret_cast<uint64_t>(base) + (uint64_t)off);
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Index v in [-2, n + 9] wrapped into [0, n) (periodic faces).
__device__ __forceinline__ int wrap_idx(int v, int n)
{
    if (n >= 10) return v < 0 ? v + n : (v >= n ? v - n : v);
    return ((v % n) + n) % n;
}

// Value held by lane l (per lane) of this wavefront.
__device__ __forceinline__ float lane_get(float v, int l)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(l << 2, __builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double lane_get(double v, int l)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(l << 2, (int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(l << 2, (int)(uint32_t)(u >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
template <typename M>
__device__ __forceinline__ Macro<M> shfl_macro(const Macro<M>& q, int l)
{
    Macro<M> r;
    r.rho = lane_get(q.rho, l);
    r.ux = lane_get(q.ux, l);
    r.uy = lane_get(q.uy, l);
    r.uz = lane_get(q.uz, l);
    r.T = lane_get(q.T, l);
    return r;
}

// XF: this tile forms extrapolating or reflecting x layers itself (see
// x_forms(); the caller selects the instantiation per tile).  VK: the FP64
// model constants may be held in vector registers (see below).  NT: the new
// level is stored non-temporally (see st_at).
template <int MODE, int BY, bool XF, bool VK, bool NT>
__device__ __forceinline__ void step_tile_x(const StepArgs<MODE>& A, const Model<double>& md,
                                            const Model<float>& mf, int x0, int y0, int z0, int z1,
                                            TilePlane<BY, typename Types<MODE>::S> (&P)[2])
{
    using S = typename Types<MODE>::S;
    using C = typename Types<MODE>::C;
    using M = typename Types<MODE>::M;
    constexpr uint32_t ES = sizeof(S);
    const Model<C>& mc = pick<C>(md, mf);
    Model<M> mm = pick<M>(md, mf);
    if constexpr (VK && MODE == MODE_FP32_T64 && BY >= 8) {
        // Uniform FP64 constants held in vector registers.  The scalar
        // file cannot hold them beside the pointers and loop state, and the
        // compiler would spill them into vector lanes and read them back
        // (one VALU instruction per dword) in every plane.  The 8-row
        // tiles have the vector registers to spare at two wavefronts per
        // SIMD; the smaller tiles do not, and FP32 constants fit the
        // scalar file.
        auto vk = [](M& v) { asm volatile("" : "+v"(v)); };
        vk(mm.r_aT);
        vk(mm.x_a0); vk(mm.x_aT); vk(mm.x_au); vk(mm.x_b0); vk(mm.x_bT); vk(mm.x_bu);
        vk(mm.d_a0); vk(mm.d_aT); vk(mm.d_au); vk(mm.d_b0); vk(mm.d_bT); vk(mm.d_bu);
        vk(mm.c1); vk(mm.k); vk(mm.e0sq); vk(mm.c1sq); vk(mm.c2sq); vk(mm.inv_b); vk(mm.x_d); vk(mm.d_d);
    }
    const Grid& g = A.g;
    const S* __restrict__ f = A.f;
    S* __restrict__ fn = A.fn;

    const int tx = threadIdx.x & (TILE_X - 1);
    const int ty = threadIdx.x / TILE_X;
    const int wave = __builtin_amdgcn_readfirstlane(ty);
    const int x = x0 + tx, y = y0 + ty;
    const bool act = (x < g.nx) && (y < g.ny);
    const int64_t sv = g.sv, sy = g.sy, sz = g.sz;
    const int zmax = g.nz + 1;
    // Faces handled inside the tile, so their layers need not be in memory:
    //  - the -x face (first tile): fixed-state halo columns are written into
    //    both LDS planes once; extrapolated and reflecting columns are
    //    formed per plane from the moments of the nodes next to the face
    //    (Sec. 4 (2)), by the wavefront that owns the row;
    //  - the +x face (last tile): the same, into the halo columns when
    //    64-wide tiles cover x exactly, else into the row's own LDS columns
    //    just past the face (those of lanes xr, xr + 1, which are outside
    //    the grid); with a one-column tail (xr = 1) the layers stay in
    //    memory, as do fixed-state layers past a ragged edge (the lanes
    //    there load them from memory with their own column);
    //  - periodic faces: columns, rows and planes wrap (any nx).
    // Other layers are read from memory.  Every load is clamped into the
    // padded array: nodes beyond the last layer are never read by an
    // active node's stencil.
    const bool xin_tile = (g.nx % TILE_X) == 0;
    const int xr = g.nx - x0;  // interior columns from x0 to the +x face
    const bool lf = x0 == 0;
    const bool rf = xr <= TILE_X && xr >= 2;  // this tile forms the +x layers
    const bool redge = xin_tile && xr == TILE_X;  // ... in its halo columns
    const int kL = A.bc.kind[0], kR = A.bc.kind[1];
    const bool xwrap = kL == BC_PERIODIC;
    const bool ywrap = A.bc.kind[2] == BC_PERIODIC;
    const bool zwrap = A.bc.kind[4] == BC_PERIODIC;
    // x wrapped into [0, nx) for the columns a stencil can read (-2 .. nx+1);
    // columns further right only feed lanes outside the grid
    auto xw = [&](int v) {
        return v < 0 ? ((v % g.nx) + g.nx) % g.nx : (v < g.nx ? v : (v < g.nx + 2 ? (v - g.nx) % g.nx : 0));
    };
    auto zsel = [&](int zz) { return zwrap ? wrap_idx(zz, g.nz) : min(zz, zmax); };
    // the plane after zz (wrapped or clamped like zsel), without a division
    auto znext = [&](int zz) { return zwrap ? (zz + 1 == g.nz ? 0 : zz + 1) : min(zz + 1, zmax); };
    const int xl = xwrap ? xw(x) : min(x, g.nx + 1);
    const int yl = ywrap ? wrap_idx(min(y, g.ny + 9), g.ny) : min(y, g.ny + 1);
    // uniform base of velocity i at plane zz (node (0, 0, zz))
    auto base = [&](const S* p, int i, int zz) { return p + ((int64_t)i * sv + g.org + (int64_t)zz * sz); };
    auto wbase = [&](S* p, int i, int zz) { return p + ((int64_t)i * sv + g.org + (int64_t)zz * sz); };
    const uint32_t colb = (uint32_t)((int64_t)yl * sy + xl) * ES;  // this thread's node within a plane
    const uint32_t xlb = (uint32_t)xl * ES;
    // lanes outside the grid store into the sink region past the end of each
    // velocity plane, which is never read, so every store is unconditional;
    // each lane has its own element there (row y mod SINK_ROWS, which is
    // uniform per wavefront, and its lane)
    const int64_t sinkrel = g.sink - g.org + (int64_t)((y0 + wave) & (SINK_ROWS - 1)) * TILE_X;

    // ---- z ring and carried minmods
    C q[NV][4];
    C mz[NV];
    C ez6 = C(0);  // f_z - f_{z-1} of the -z axis velocity (its dissipation)
    static_for<NV>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        constexpr int SZ = vsign(I, 2);
        auto at = [&](int zz) { return static_cast<C>(ld_at(base(f, I, zz), colb)); };
        q[I][3] = C(0);
        mz[I] = C(0);
        if constexpr (SZ < 0) {
            q[I][0] = at(z0);
            q[I][1] = at(zsel(z0 + 1));
            q[I][2] = at(zsel(z0 + 2));
            const C e0 = q[I][0] - at(zsel(z0 - 1));
            mz[I] = minmod(e0, q[I][1] - q[I][0]);
            if constexpr (I == 6) ez6 = e0;
        } else {
            q[I][0] = at(zsel(z0 - 1));
            q[I][1] = at(z0);
            q[I][2] = at(zsel(z0 + 1));
            if constexpr (SZ > 0) mz[I] = minmod(q[I][1] - q[I][0], q[I][0] - at(zsel(z0 - 2)));
        }
    });

    // ---- halo of a plane: x columns gathered into one register (lane 4v+p
    // holds velocity v at x0-2, x0-1, x0+64, x0+65 for p = 0..3) and the
    // halo rows of this wavefront's jobs wave, wave + BY, ...
    const int hv = min(tx >> 2, NV - 1), hp = tx & 3;
    int hx = hp == 0 ? x0 - 2 : hp == 1 ? x0 - 1 : hp == 2 ? x0 + TILE_X : x0 + TILE_X + 1;
    bool hlane = tx < 4 * NV;  // this lane's gathered value is staged
    if (xwrap) {
        hx = xw(hx);
    } else {
        // columns formed in the tile: load a cached column instead
        if (lf && hp < 2) { hx = 0; hlane = false; }
        if (rf && hp >= 2) { hx = g.nx - 1; hlane = false; }
        hx = min(hx, g.nx + 1);
    }
    const S* hptr = f + ((int64_t)hv * sv + g.org + (int64_t)yl * sy + hx);
    const int hcol = hp < 2 ? hp : hp + TILE_X;
    constexpr int NJ = halo_jobs();
    static_assert(NJ % BY == 0, "every wavefront stages the same number of halo rows");
    constexpr int NK = NJ / BY;
    int yhk[NK];  // rows of this wavefront's halo jobs (uniform)
#pragma unroll
    for (int k = 0; k < NK; k++) {
        const int e = kHaloJobs.e[wave + k * BY];
        const int code = e & 3;
        const int r = code < 2 ? code - 2 : BY + code - 2;
        yhk[k] = ywrap ? wrap_idx(y0 + r, g.ny) : min(y0 + r, g.ny + 1);
    }
    // two register sets of halo values: the set of plane z+2 is loaded
    // while the set of plane z+1 waits to be staged, so a tile reads its
    // halo rows at the same time as the neighbouring tiles load them as
    // their own planes (the L2 then serves one of the two)
    S hrow[2][NK];
    S hcolv[2] = {S(0), S(0)};
    auto load_halo = [&](int set, int zz) {
        // (through a global-space pointer: a generic one, as the batched
        // step's table-loaded f would give, becomes a flat load, which the
        // LDS waits would then wait for as well)
        using GP = const __attribute__((address_space(1))) S*;
        hcolv[set] = reinterpret_cast<GP>(reinterpret_cast<uint64_t>(hptr))[(int64_t)zz * sz];
#pragma unroll
        for (int k = 0; k < NK; k++) {
            const int i = kHaloJobs.e[wave + k * BY] >> 2;
            hrow[set][k] = ld_at(sreg(base(f, i, zz) + (int64_t)yhk[k] * sy), xlb);
        }
    };
    auto store_halo = [&](int set, TilePlane<BY, S>& T) {
        if (hlane) T.v[hv][ty + 2][hcol] = hcolv[set];
#pragma unroll
        for (int k = 0; k < NK; k++) {
            const int e = kHaloJobs.e[wave + k * BY];
            const int i = e >> 2, code = e & 3;
            const int r = code < 2 ? code - 2 : BY + code - 2;
            T.v[i][r + 2][tx + 2] = hrow[set][k];
        }
    };

    // fixed-state x columns: the equilibrium of the face state, written
    // into both planes once (lanes 0, 1: columns of layers -1, -2; lanes
    // 2, 3: layers nx, nx+1)
    {
        const bool lfix = lf && kL == BC_INFLOW, rfix = redge && kR == BC_INFLOW;
        if (lfix || rfix) {
            const int side = tx >= 2 ? 1 : 0;
            Macro<M> qf;
            // (selects, not an index by `side`: a per-lane index would put
            // the kernel argument in private memory)
            qf.rho = static_cast<M>(side ? A.xin[1][0] : A.xin[0][0]);
            qf.ux = static_cast<M>(side ? A.xin[1][1] : A.xin[0][1]);
            qf.uy = static_cast<M>(side ? A.xin[1][2] : A.xin[0][2]);
            qf.uz = static_cast<M>(side ? A.xin[1][3] : A.xin[0][3]);
            qf.T = static_cast<M>(side ? A.xin[1][4] : A.xin[0][4]);
            C e[NV];
            equilibrium<C, M>(qf, mm, mc, e);
            if (tx < 4 && (side ? rfix : lfix)) {
                const int colw = tx == 0 ? 1 : tx == 1 ? 0 : tx + TILE_X;
#pragma unroll
                for (int i = 0; i < NV; i++) {
                    P[0].v[i][ty + 2][colw] = static_cast<S>(e[i]);
                    P[1].v[i][ty + 2][colw] = static_cast<S>(e[i]);
                }
            }
        }
    }
    // layers of an extrapolating or reflecting x face of one plane from the
    // moments of this row's two nodes next to the face, one value per lane:
    // lane 32 s + 15 j + i (i < 15, j < 2) forms velocity i of layer j+1 of
    // face s (0: -x, 1: +x) and writes it into the plane's LDS column of
    // that layer node (a halo column, or past a ragged +x face a column of
    // the row itself, overwriting what the lane there staged), which only
    // this wavefront reads (so no barrier orders it)
    auto form_x = [&](const Macro<M>& mq, TilePlane<BY, S>& T) {
        const int side = tx >> 5, ll = tx & 31;
        const int j = ll >= NV ? 1 : 0, iv = min(ll - NV * j, NV - 1);
        const int kind = side ? kR : kL;
        const bool on = ll < 2 * NV && (side ? rf : lf) && (kind == BC_OUTFLOW || kind == BC_REFLECT);
        // (source lanes clamped into the wavefront: a tile that forms only
        // the -x layers computes unused +x values)
        const int xs = min(xr, TILE_X);
        const Macro<M> q0 = shfl_macro(mq, side ? xs - 1 : 0);
        const Macro<M> q1 = shfl_macro(mq, side ? max(xs - 2, 0) : 1);
        M c, m;
        layer_coefs(kind, j + 1, c, m);
        const Macro<M> qs = layer_state(q0, q1, c, m, 0);
        const C val = static_cast<C>(feq_vel<M>(iv, eq_coef<M, M>(qs, mm), mm));
        if (on) T.v[iv][ty + 2][side ? xr + 2 + j : 1 - j] = static_cast<S>(val);
    };

    // stage plane z0 in P[0]; the halo of plane z0+1 waits in set 1
    load_halo(0, z0);
    static_for<NV>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        P[0].v[I][ty + 2][tx + 2] = static_cast<S>(q[I][ring_slot<I>(0, 0)]);
    });
    store_halo(0, P[0]);
    load_halo(1, zsel(z0 + 1));

    uint32_t hacc = 0;
    int za = zsel(z0 + 2), zb = zsel(z0 + 3);  // planes z+2 and z+3 of the current step
    // one plane at unroll phase K: prefetch, barrier, compute from P[K & 1],
    // stage plane z+1 in P[(K + 1) & 1]
    auto plane = [&](auto kc, int z) {
        constexpr int K = decltype(kc)::value;
        TilePlane<BY, S>& cur = P[K & 1];
        TilePlane<BY, S>& nxt = P[(K + 1) & 1];
        // planes z+2 (v_z >= 0) and z+3 (v_z < 0), walked velocity by velocity;
        // the slot they fill is not read in this plane
        const S* pa = base(f, 0, za);
        const int64_t db = (int64_t)(zb - za) * sz;
        auto ring_load = [&](auto ic) {
            constexpr int I = decltype(ic)::value;
            pa = sreg(pa);
            const S* p = vsign(I, 2) < 0 ? sreg(pa + db) : pa;
            q[I][(K + 3) & 3] = static_cast<C>(ld_at(p, colb));
            pa += sv;
        };
        load_halo(K & 1, za);
        za = znext(za);
        zb = znext(zb);
        lds_barrier();

        C fc[NV];
        static_for<NV>([&](auto ic) {
            constexpr int I = decltype(ic)::value;
            fc[I] = q[I][ring_slot<I>(0, K)];
        });
        const Macro<M> mac = moments<M, C>(fc, mm);
        hacc |= health_bits(mac);
        // on tiles that form x layers (their own copy of the sweep, so no
        // branch keeps the scheduler from interleaving it with the node's
        // equilibrium) the layers of this plane come first
        if constexpr (XF) form_x(mac, cur);
        C feq[NV];
        equilibrium<C, M>(mac, mm, mc, feq);
        const uint32_t outb = act ? colb : (uint32_t)((sinkrel - (int64_t)z * sz) * ES) + (uint32_t)tx * ES;
        S* po = wbase(fn, 0, z);
        static_for<NV>([&](auto ic) {
            constexpr int I = decltype(ic)::value;
            constexpr int SX = vsign(I, 0), SY = vsign(I, 1), SZ = vsign(I, 2), G = vgroup(I);
            constexpr int RW = TILE_X + 4;
            const C f0 = fc[I];
            const S* row = &cur.v[I][ty + 2][tx + 2];
            C Dx = C(0), Dy = C(0), Dz = C(0), lx = C(0), ly = C(0), lz = C(0);
            if constexpr (SX > 0) {
                const C m2 = row[-2], m1 = row[-1], p1 = row[1];
                const C e0 = f0 - m1, e1 = p1 - f0;
                Dx = nnd_pos(m1 - m2, e0, e1);
                lx = e1 - e0;
            } else if constexpr (SX < 0) {
                const C m1 = row[-1], p1 = row[1], p2 = row[2];
                const C e0 = f0 - m1, e1 = p1 - f0;
                Dx = nnd_neg(e0, e1, p2 - p1);
                lx = e1 - e0;
            } else if constexpr (G <= 1) {
                lx = static_cast<C>(row[-1]) + static_cast<C>(row[1]);
            }
            if constexpr (SY > 0) {
                const C m2 = row[-2 * RW], m1 = row[-RW], p1 = row[RW];
                const C e0 = f0 - m1, e1 = p1 - f0;
                Dy = nnd_pos(m1 - m2, e0, e1);
                ly = e1 - e0;
            } else if constexpr (SY < 0) {
                const C m1 = row[-RW], p1 = row[RW], p2 = row[2 * RW];
                const C e0 = f0 - m1, e1 = p1 - f0;
                Dy = nnd_neg(e0, e1, p2 - p1);
                ly = e1 - e0;
            } else if constexpr (G <= 1) {
                ly = static_cast<C>(row[-RW]) + static_cast<C>(row[RW]);
            }
            if constexpr (SZ > 0) {
                const C e0 = f0 - q[I][ring_slot<I>(-1, K)], e1 = q[I][ring_slot<I>(1, K)] - f0;
                Dz = nnd_pos_c(e0, e1, mz[I]);
                lz = e1 - e0;
            } else if constexpr (SZ < 0) {
                const C p1 = q[I][ring_slot<I>(1, K)];
                const C e1 = p1 - f0;
                Dz = nnd_neg_c(e1, q[I][ring_slot<I>(2, K)] - p1, mz[I]);
                if constexpr (G == 1) {
                    lz = e1 - ez6;
                    ez6 = e1;
                }
            } else if constexpr (G <= 1) {
                lz = q[I][ring_slot<I>(-1, K)] + q[I][ring_slot<I>(1, K)];
            }
            const C out = node_update<I, C>(f0, feq[I], Dx, Dy, Dz, lx, ly, lz, mc);
            po = sreg(po);
            st_at<NT>(po, outb, static_cast<S>(out));
            po += sv;
            ring_load(ic);
        });

        // stage plane z+1: own values and its halo
        static_for<NV>([&](auto ic) {
            constexpr int I = decltype(ic)::value;
            nxt.v[I][ty + 2][tx + 2] = static_cast<S>(q[I][ring_slot<I>(1, K)]);
        });
        store_halo((K + 1) & 1, nxt);
    };

    for (int z = z0;;) {
        plane(std::integral_constant<int, 0>{}, z);
        if (++z >= z1) break;
        plane(std::integral_constant<int, 1>{}, z);
        if (++z >= z1) break;
        plane(std::integral_constant<int, 2>{}, z);
        if (++z >= z1) break;
        plane(std::integral_constant<int, 3>{}, z);
        if (++z >= z1) break;
    }
    report_health(A.health, act ? hacc : 0u);
}

// Does the tile at x0 form extrapolating or reflecting x layers itself?
// (The first tile forms the -x layers, the last the +x layers unless its
// tail is a single column; ghost_faces() leaves the same faces out.)
template <int MODE>
__device__ __forceinline__ bool x_forms(const StepArgs<MODE>& A, int x0)
{
    auto formed = [](int k) { return k == BC_OUTFLOW || k == BC_REFLECT; };
    const int xr = A.g.nx - x0;
    return (x0 == 0 && formed(A.bc.kind[0])) || (xr <= TILE_X && xr >= 2 && formed(A.bc.kind[1]));
}

template <int MODE, int BY, bool VK, bool NT>
__device__ __forceinline__ void step_tile(const StepArgs<MODE>& A, const Model<double>& md,
                                          const Model<float>& mf, int x0, int y0, int z0, int z1,
                                          TilePlane<BY, typename Types<MODE>::S> (&P)[2])
{
    if (x_forms(A, x0))
        step_tile_x<MODE, BY, true, VK, NT>(A, md, mf, x0, y0, z0, z1, P);
    else
        step_tile_x<MODE, BY, false, VK, NT>(A, md, mf, x0, y0, z0, z1, P);
}

// Tile order: tiles are numbered with x (or y) fastest, then the other
// axis, then the z chunk, and consecutive numbers are given to workgroups
// that land on the same XCD (dispatch assigns workgroup b to XCD b mod 8),
// so that tiles sharing halo rows and columns share an L2.
__device__ __forceinline__ int xcd_tile(int b, int nblocks)
{
    const int per = nblocks >> 3, rem = nblocks & 7;
    const int xcd = b & 7, slot = b >> 3;
    return xcd * per + min(xcd, rem) + slot;
}

}  // namespace lbm3d
