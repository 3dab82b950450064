// Device kernels of the lbm3d library for gfx950: initial state, the fused
// time step, boundary layers, moments, FP64 conservation totals and the
// checkpoint pack/unpack.
#include "lbm3d_tile.h"

#include <cmath>

namespace lbm3d {

// --------------------------------------------------------- the fused step --
// One explicit step of Eq. (lp) with NND convection at every interior node:
//   f_i^{n+1} = f_i - dt/dx sum_a v_ia (g_{I+1/2} - g_{I-1/2})
//               - dt/tau (f_i - f_i^eq) + lambda_i dt/dx^2 sum_a (f_{I+1} - 2 f_I + f_{I-1})
// reading every term at level n (forward Euler, Eq. (fi1)).  The boundary
// layers of f^n hold valid values, so every neighbour load is in bounds.
template <int I, typename S, typename C>
__device__ __forceinline__ void update_one(const S* __restrict__ fi, S* __restrict__ fo,
                                           int64_t sy, int64_t sz, C f0, C feq,
                                           const Model<C>& m)
{
    constexpr int SX = vsign(I, 0), SY = vsign(I, 1), SZ = vsign(I, 2), G = vgroup(I);
    const C vm = (G == 1) ? m.c1 : m.k;
    C conv = C(0);
    const int64_t st[3] = {1, sy, sz};
    constexpr int SG[3] = {SX, SY, SZ};
#pragma unroll
    for (int a = 0; a < 3; a++) {
        if (SG[a] == 0) continue;
        const int64_t s = st[a];
        const C fm1 = static_cast<C>(fi[-s]);
        const C fp1 = static_cast<C>(fi[s]);
        C d;
        if (SG[a] > 0) {
            const C fm2 = static_cast<C>(fi[-2 * s]);
            d = nnd_diff<1, C>(fm2, fm1, f0, fp1, C(0));
            conv += vm * d;
        } else {
            const C fp2 = static_cast<C>(fi[2 * s]);
            d = nnd_diff<-1, C>(C(0), fm1, f0, fp1, fp2);
            conv -= vm * d;
        }
    }
    C out = f0 - m.k_adv * conv - m.k_bgk * (f0 - feq);
    if constexpr (G <= 1) {
        const C lap = ((static_cast<C>(fi[-1]) + static_cast<C>(fi[1])) +
                       (static_cast<C>(fi[-sy]) + static_cast<C>(fi[sy]))) +
                      (static_cast<C>(fi[-sz]) + static_cast<C>(fi[sz])) - C(6) * f0;
        out += (G == 0 ? m.k_lap0 : m.k_lap1) * lap;
    }
    *fo = static_cast<S>(out);
}

template <typename S, typename C, int I = 0>
__device__ __forceinline__ void update_all(const S* __restrict__ f, S* __restrict__ fn, int64_t site,
                                           int64_t sv, int64_t sy, int64_t sz, const C (&fc)[NV],
                                           const C (&feq)[NV], const Model<C>& m)
{
    if constexpr (I < NV) {
        update_one<I, S, C>(f + I * sv + site, fn + I * sv + site, sy, sz, fc[I], feq[I], m);
        update_all<S, C, I + 1>(f, fn, site, sv, sy, sz, fc, feq, m);
    }
}

template <int MODE>
__global__ void __launch_bounds__(TX * TY)
k_step(Grid g, Model<double> md, Model<float> mf, const typename Types<MODE>::S* __restrict__ f,
       typename Types<MODE>::S* __restrict__ fn, uint32_t* __restrict__ health)
{
    using S = typename Types<MODE>::S;
    using C = typename Types<MODE>::C;
    using M = typename Types<MODE>::M;
    const int x = blockIdx.x * TX + threadIdx.x;
    const int y = blockIdx.y * TY + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    const Model<C>& mc = pick<C>(md, mf);
    const Model<M>& mm = pick<M>(md, mf);
    const int64_t site = g.org + (int64_t)z * g.sz + (int64_t)y * g.sy + x;
    C fc[NV];
#pragma unroll
    for (int i = 0; i < NV; i++) fc[i] = static_cast<C>(f[i * g.sv + site]);
    const Macro<M> q = moments<M, C>(fc, mm);
    const uint32_t hb = health_bits(q);
    if (hb) atomicOr(health, hb);
    C feq[NV];
    equilibrium<C, M>(q, mm, mc, feq);
    update_all<S, C>(f, fn, site, g.sv, g.sy, g.sz, fc, feq, mc);
}

// Tiled fused step: one workgroup per 64 x BY x TZ tile (see lbm3d_tile.h).
// LBM3D_WAVES_PER_EU (build-time tuning knob): register budget of the tiled
// kernel as wavefronts per SIMD (0 = compiler's choice).
#ifndef LBM3D_WAVES_PER_EU
#define LBM3D_WAVES_PER_EU 0
#endif
#if LBM3D_WAVES_PER_EU > 0
#define LBM3D_TILED_ATTR __attribute__((amdgpu_waves_per_eu(LBM3D_WAVES_PER_EU)))
#else
#define LBM3D_TILED_ATTR
#endif

template <int MODE, int BY>
__global__ void __launch_bounds__(TILE_X * BY) LBM3D_TILED_ATTR
k_step_tiled(StepArgs<MODE> A, Model<double> md, Model<float> mf, int ntx, int nty, int tz)
{
    __shared__ TilePlane<BY, typename Types<MODE>::S> P;
    const int t = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    const int tyi = t % nty;
    const int r = t / nty;
    const int txi = r % ntx;
    const int tzi = r / ntx;
    const int z0 = tzi * tz;
    const int z1 = min(z0 + tz, A.g.nz);
    step_tile<MODE, BY>(A, md, mf, txi * TILE_X, tyi * BY, z0, z1, P);
}

// ------------------------------------------------------- initial state ----
template <int MODE>
__global__ void k_init(Grid g, Model<double> md, Model<float> mf, const double* __restrict__ q5,
                       typename Types<MODE>::S* __restrict__ f)
{
    using S = typename Types<MODE>::S;
    using C = typename Types<MODE>::C;
    using M = typename Types<MODE>::M;
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int x = (int)(k % g.nx);
    const int y = (int)((k / g.nx) % g.ny);
    const int z = (int)(k / ((int64_t)g.nx * g.ny));
    Macro<M> q;
    q.rho = static_cast<M>(q5[k]);
    q.ux = static_cast<M>(q5[n + k]);
    q.uy = static_cast<M>(q5[2 * n + k]);
    q.uz = static_cast<M>(q5[3 * n + k]);
    q.T = static_cast<M>(q5[4 * n + k] / q5[k]);
    C feq[NV];
    equilibrium<C, M>(q, pick<M>(md, mf), pick<C>(md, mf), feq);
    const int64_t site = g.org + (int64_t)z * g.sz + (int64_t)y * g.sy + x;
#pragma unroll
    for (int i = 0; i < NV; i++) f[i * g.sv + site] = static_cast<S>(feq[i]);
}

// ----------------------------------------------------- boundary layers ----
// Layers -1, -2 (low face) or n, n+1 (high face) along one axis, Sec. 4 (2):
// fixed state; linear extrapolation of (rho, u, T) from the two nodes next
// to the face; reflection (wall layer: the node next to the face with zero
// normal velocity; mirror layer: its normal velocity negated); distributions
// are f^eq of those values.  Periodic faces copy f from the other side.
// Only face layers are written: the stencils never read edges or corners.
template <int MODE>
__global__ void k_ghosts(Grid g, FaceBC bc, Model<double> md, Model<float> mf, double4 fixed_q,
                         double fixed_T, int face_mask, typename Types<MODE>::S* __restrict__ f)
{
    using S = typename Types<MODE>::S;
    using C = typename Types<MODE>::C;
    using M = typename Types<MODE>::M;
    const int face = blockIdx.z;
    if (!((face_mask >> face) & 1)) return;
    const int axis = face >> 1, side = face & 1;
    const int n[3] = {g.nx, g.ny, g.nz};
    // tangential axes, x first where possible so that a wavefront writes
    // consecutive addresses
    const int t1 = axis == 0 ? 1 : 0, t2 = axis == 2 ? 1 : 2;
    const int64_t cnt = (int64_t)n[t1] * n[t2];
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= cnt) return;
    const int64_t st[3] = {1, g.sy, g.sz};
    const int b1 = (int)(k % n[t1]), b2 = (int)(k / n[t1]);
    const int64_t base = g.org + b1 * st[t1] + (int64_t)b2 * st[t2];
    const int64_t sa = st[axis];
    const int na = n[axis];
    // ghost coordinates along the axis and the interior nodes next to the face
    const int g1 = side ? na : -1, g2 = side ? na + 1 : -2;
    const int i0 = side ? na - 1 : 0, i1 = side ? na - 2 : 1;
    const int kind = bc.kind[face];
    if (kind == BC_PERIODIC) {
        const int w1 = ((g1 % na) + na) % na, w2 = ((g2 % na) + na) % na;
#pragma unroll
        for (int i = 0; i < NV; i++) {
            S* fi = f + i * g.sv + base;
            fi[g1 * sa] = fi[w1 * sa];
            fi[g2 * sa] = fi[w2 * sa];
        }
        return;
    }
    const Model<C>& mc = pick<C>(md, mf);
    const Model<M>& mm = pick<M>(md, mf);
    Macro<M> q1, q2;
    if (kind == BC_INFLOW) {
        // fixed state of the face being filled: (rho, ux, uy, uz) and T
        q1.rho = static_cast<M>(fixed_q.x);
        q1.ux = static_cast<M>(fixed_q.y);
        q1.uy = static_cast<M>(fixed_q.z);
        q1.uz = static_cast<M>(fixed_q.w);
        q1.T = static_cast<M>(fixed_T);
        q2 = q1;
    } else {
        C fa[NV];
#pragma unroll
        for (int i = 0; i < NV; i++) fa[i] = static_cast<C>(f[i * g.sv + base + i0 * sa]);
        const Macro<M> qa = moments<M, C>(fa, mm);
        if (kind == BC_OUTFLOW) {
            C fb[NV];
#pragma unroll
            for (int i = 0; i < NV; i++) fb[i] = static_cast<C>(f[i * g.sv + base + i1 * sa]);
            const Macro<M> qb = moments<M, C>(fb, mm);
            q1.rho = M(2) * qa.rho - qb.rho;
            q1.ux = M(2) * qa.ux - qb.ux;
            q1.uy = M(2) * qa.uy - qb.uy;
            q1.uz = M(2) * qa.uz - qb.uz;
            q1.T = M(2) * qa.T - qb.T;
            q2.rho = M(2) * q1.rho - qa.rho;
            q2.ux = M(2) * q1.ux - qa.ux;
            q2.uy = M(2) * q1.uy - qa.uy;
            q2.uz = M(2) * q1.uz - qa.uz;
            q2.T = M(2) * q1.T - qa.T;
        } else {  // BC_REFLECT
            q1 = qa;
            q2 = qa;
            M* n1 = axis == 0 ? &q1.ux : (axis == 1 ? &q1.uy : &q1.uz);
            M* n2 = axis == 0 ? &q2.ux : (axis == 1 ? &q2.uy : &q2.uz);
            *n1 = M(0);
            *n2 = -*n2;
        }
    }
    C e1[NV], e2[NV];
    equilibrium<C, M>(q1, mm, mc, e1);
    equilibrium<C, M>(q2, mm, mc, e2);
#pragma unroll
    for (int i = 0; i < NV; i++) {
        S* fi = f + i * g.sv + base;
        fi[g1 * sa] = static_cast<S>(e1[i]);
        fi[g2 * sa] = static_cast<S>(e2[i]);
    }
}

// -------------------------------------------------------------- moments --
template <int MODE>
__global__ void k_moments(Grid g, Model<double> md, Model<float> mf,
                          const typename Types<MODE>::S* __restrict__ f, double* __restrict__ q5)
{
    using C = typename Types<MODE>::C;
    using M = typename Types<MODE>::M;
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int x = (int)(k % g.nx);
    const int y = (int)((k / g.nx) % g.ny);
    const int z = (int)(k / ((int64_t)g.nx * g.ny));
    const int64_t site = g.org + (int64_t)z * g.sz + (int64_t)y * g.sy + x;
    C fc[NV];
#pragma unroll
    for (int i = 0; i < NV; i++) fc[i] = static_cast<C>(f[i * g.sv + site]);
    const Macro<M> q = moments<M, C>(fc, pick<M>(md, mf));
    q5[k] = (double)q.rho;
    q5[n + k] = (double)q.ux;
    q5[2 * n + k] = (double)q.uy;
    q5[3 * n + k] = (double)q.uz;
    q5[4 * n + k] = (double)q.rho * (double)q.T;
}

// ------------------------------------------------- conservation totals ----
// Per block: FP64 sums over its nodes of (rho, rho u, energy) reduced by a
// fixed LDS tree; then one block adds the per-block partials in a fixed
// tree.  No floating atomics, so the totals are bitwise reproducible.
constexpr int RB = 256;

template <int MODE>
__global__ void __launch_bounds__(RB)
k_conserved_partial(Grid g, Model<double> md, const typename Types<MODE>::S* __restrict__ f,
                    double* __restrict__ partial)
{
    __shared__ double sh[5][RB];
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    double acc[5] = {0, 0, 0, 0, 0};
    for (int64_t k = (int64_t)blockIdx.x * RB + threadIdx.x; k < n; k += (int64_t)gridDim.x * RB) {
        const int x = (int)(k % g.nx);
        const int y = (int)((k / g.nx) % g.ny);
        const int z = (int)(k / ((int64_t)g.nx * g.ny));
        const int64_t site = g.org + (int64_t)z * g.sz + (int64_t)y * g.sy + x;
        double v[NV];
#pragma unroll
        for (int i = 0; i < NV; i++) v[i] = (double)f[i * g.sv + site];
        const double sa = ((v[1] + v[2]) + (v[3] + v[4])) + (v[5] + v[6]);
        const double sd = ((v[7] + v[8]) + (v[9] + v[10])) + ((v[11] + v[12]) + (v[13] + v[14]));
        const double dxs = ((v[7] - v[8]) + (v[9] - v[10])) + ((v[11] - v[12]) + (v[13] - v[14]));
        const double dys = ((v[7] + v[8]) - (v[9] + v[10])) + ((v[11] + v[12]) - (v[13] + v[14]));
        const double dzs = ((v[7] + v[8]) + (v[9] + v[10])) - ((v[11] + v[12]) + (v[13] + v[14]));
        acc[0] += v[0] + sa + sd;
        acc[1] += md.c1 * (v[1] - v[2]) + md.k * dxs;
        acc[2] += md.c1 * (v[3] - v[4]) + md.k * dys;
        acc[3] += md.c1 * (v[5] - v[6]) + md.k * dzs;
        acc[4] += 0.5 * (md.e0sq * v[0] + md.c1sq * sa + md.c2sq * sd);
    }
#pragma unroll
    for (int c = 0; c < 5; c++) sh[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int w = RB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int c = 0; c < 5; c++) sh[c][threadIdx.x] += sh[c][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < 5) partial[(int64_t)blockIdx.x * 5 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void __launch_bounds__(RB) k_conserved_final(const double* __restrict__ partial, int nb,
                                                       double* __restrict__ out)
{
    __shared__ double sh[5][RB];
    double acc[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nb; b += RB)
#pragma unroll
        for (int c = 0; c < 5; c++) acc[c] += partial[(int64_t)b * 5 + c];
#pragma unroll
    for (int c = 0; c < 5; c++) sh[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int w = RB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int c = 0; c < 5; c++) sh[c][threadIdx.x] += sh[c][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < 5) out[threadIdx.x] = sh[threadIdx.x][0];
}

// ------------------------------------------------- checkpoint pack ------
template <typename S>
__global__ void k_pack(Grid g, S* __restrict__ f, S* __restrict__ dense, int to_dense)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n * NV) return;
    const int i = (int)(k / n);
    const int64_t r = k - (int64_t)i * n;
    const int x = (int)(r % g.nx);
    const int y = (int)((r / g.nx) % g.ny);
    const int z = (int)(r / ((int64_t)g.nx * g.ny));
    const int64_t site = (int64_t)i * g.sv + g.org + (int64_t)z * g.sz + (int64_t)y * g.sy + x;
    if (to_dense)
        dense[k] = f[site];
    else
        f[site] = dense[k];
}

// ------------------------------------------------------------- launches --
static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

#define LBM3D_DISPATCH(mode, ...)                                          \
    switch (mode) {                                                        \
    case MODE_FP64: { constexpr int MD = MODE_FP64; __VA_ARGS__; } break;  \
    case MODE_FP32: { constexpr int MD = MODE_FP32; __VA_ARGS__; } break;  \
    default: { constexpr int MD = MODE_FP32_T64; __VA_ARGS__; } break;     \
    }

static Model<float> to_float(const Model<double>& d)
{
    Model<float> f;
    const double* src = reinterpret_cast<const double*>(&d);
    float* dst = reinterpret_cast<float*>(&f);
    static_assert(sizeof(Model<double>) == 2 * sizeof(Model<float>), "model layout");
    for (size_t i = 0; i < sizeof(Model<float>) / sizeof(float); i++) dst[i] = (float)src[i];
    return f;
}

hipError_t launch_init(int mode, const Grid& g, const Model<double>& md, const double* q5, void* f,
                       hipStream_t s)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const Model<float> mf = to_float(md);
    LBM3D_DISPATCH(mode, k_init<MD><<<dim3(blocks_for(n, 256)), dim3(256), 0, s>>>(g, md, mf, q5, (typename Types<MD>::S*)f));
    return hipGetLastError();
}

TileCfg default_tile(int mode, const Grid& g)
{
    TileCfg t;
    t.by = mode == MODE_FP64 ? 4 : 8;
    t.tz = mode == MODE_FP64 ? 32 : 16;
    if (g.nz < 2 * t.tz) t.tz = std::max(1, g.nz / 4);
    return t;
}

bool tile_supported(int mode, const TileCfg& t)
{
    if (t.tz < 1) return false;
    if (t.by == 0) return true;
    if (t.by == 2 || t.by == 4) return true;
    return t.by == 8 && mode != MODE_FP64;
}

// LBM3D_FUSE_LAYERS (build-time tuning knob): 1 = the tiled step writes the
// boundary layers it can, 0 = all layers are left to k_ghosts.
#ifndef LBM3D_FUSE_LAYERS
#define LBM3D_FUSE_LAYERS 1
#endif

uint32_t fused_faces(const Grid& g, const FaceBC& bc, const TileCfg& tc)
{
    if (tc.by == 0 || !LBM3D_FUSE_LAYERS) return 0u;  // the untiled kernel leaves all layers to k_ghosts
    uint32_t m = 0;
    for (int face = 0; face < 6; face++) {
        const int k = bc.kind[face];
        if (k == BC_PERIODIC || k == BC_REFLECT) m |= 1u << face;
        // outflow along x pairs lanes of one wavefront: node n-1 and n-2 must
        // share a 64-wide tile row
        if (k == BC_OUTFLOW && face == 0) m |= 1u;
        if (k == BC_OUTFLOW && face == 1 && (g.nx % TILE_X) != 1) m |= 2u;
    }
    return m;
}

uint32_t ghost_faces(const FaceBC& bc, uint32_t fused)
{
    uint32_t m = 0;
    for (int face = 0; face < 6; face++)
        if (bc.kind[face] != BC_INFLOW && !((fused >> face) & 1)) m |= 1u << face;
    return m;
}

template <int MODE, int BY>
static void launch_tiled(const Grid& g, const FaceBC& bc, uint32_t fused, int tz, const Model<double>& md,
                         const Model<float>& mf, const void* f, void* fn, uint32_t* health, hipStream_t s)
{
    using S = typename Types<MODE>::S;
    const int ntx = (g.nx + TILE_X - 1) / TILE_X;
    const int nty = (g.ny + BY - 1) / BY;
    const int ntz = (g.nz + tz - 1) / tz;
    const int nb = ntx * nty * ntz;
    StepArgs<MODE> A;
    A.g = g;
    A.bc = bc;
    A.fused = fused;
    A.f = (const S*)f;
    A.fn = (S*)fn;
    A.health = health;
    k_step_tiled<MODE, BY><<<dim3(nb), dim3(TILE_X * BY), 0, s>>>(A, md, mf, ntx, nty, tz);
}

hipError_t launch_step(int mode, const Grid& g, const FaceBC& bc, const TileCfg& tc, const Model<double>& md,
                       const Model<float>& mf, const void* f, void* fn, uint32_t* health,
                       hipStream_t s)
{
    if (tc.by != 0) {
        const uint32_t fu = fused_faces(g, bc, tc);
        switch (tc.by) {
        case 2: LBM3D_DISPATCH(mode, launch_tiled<MD, 2>(g, bc, fu, tc.tz, md, mf, f, fn, health, s)); break;
        case 8:
            if (mode == MODE_FP64) return hipErrorInvalidValue;
            if (mode == MODE_FP32) launch_tiled<MODE_FP32, 8>(g, bc, fu, tc.tz, md, mf, f, fn, health, s);
            else launch_tiled<MODE_FP32_T64, 8>(g, bc, fu, tc.tz, md, mf, f, fn, health, s);
            break;
        default: LBM3D_DISPATCH(mode, launch_tiled<MD, 4>(g, bc, fu, tc.tz, md, mf, f, fn, health, s)); break;
        }
        return hipGetLastError();
    }
    dim3 grid((g.nx + TX - 1) / TX, (g.ny + TY - 1) / TY, g.nz);
    LBM3D_DISPATCH(mode, k_step<MD><<<grid, dim3(TX, TY), 0, s>>>(g, md, mf, (const typename Types<MD>::S*)f, (typename Types<MD>::S*)fn, health));
    return hipGetLastError();
}

hipError_t launch_ghosts(int mode, const Grid& g, const FaceBC& bc, const Model<double>& md,
                         const double (*inflow)[5], bool include_fixed, void* f, hipStream_t s,
                         uint32_t face_mask)
{
    const Model<float> mf = to_float(md);
    const int n[3] = {g.nx, g.ny, g.nz};
    // fixed-state faces are filled one launch each (their state travels as
    // kernel arguments); the faces in face_mask in one launch
    int mask = 0;
    for (int face = 0; face < 6; face++)
        if (bc.kind[face] != BC_INFLOW && ((face_mask >> face) & 1)) mask |= 1 << face;
    int64_t maxcnt = 1;
    for (int a = 0; a < 3; a++) maxcnt = std::max<int64_t>(maxcnt, (int64_t)n[(a + 1) % 3] * n[(a + 2) % 3]);
    const unsigned nb = blocks_for(maxcnt, 256);
    if (mask) {
        LBM3D_DISPATCH(mode, k_ghosts<MD><<<dim3(nb, 1, 6), dim3(256), 0, s>>>(g, bc, md, mf, double4{0, 0, 0, 0}, 0.0, mask, (typename Types<MD>::S*)f));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (include_fixed) {
        for (int face = 0; face < 6; face++) {
            if (bc.kind[face] != BC_INFLOW) continue;
            const double* st = inflow[face];
            const double4 q{st[0], st[1], st[2], st[3]};
            const double T = st[4] / st[0];
            LBM3D_DISPATCH(mode, k_ghosts<MD><<<dim3(nb, 1, 6), dim3(256), 0, s>>>(g, bc, md, mf, q, T, 1 << face, (typename Types<MD>::S*)f));
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

hipError_t launch_moments(int mode, const Grid& g, const Model<double>& md, const void* f, double* q5,
                          hipStream_t s)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const Model<float> mf = to_float(md);
    LBM3D_DISPATCH(mode, k_moments<MD><<<dim3(blocks_for(n, 256)), dim3(256), 0, s>>>(g, md, mf, (const typename Types<MD>::S*)f, q5));
    return hipGetLastError();
}

int conserved_blocks(const Grid& g)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    return (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + RB - 1) / RB));
}

hipError_t launch_conserved(int mode, const Grid& g, const Model<double>& md, const void* f,
                            double* partial, int nblocks, double* out5, hipStream_t s)
{
    LBM3D_DISPATCH(mode, k_conserved_partial<MD><<<dim3(nblocks), dim3(RB), 0, s>>>(g, md, (const typename Types<MD>::S*)f, partial));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_conserved_final, dim3(1), dim3(RB), 0, s, (const double*)partial, nblocks, out5);
    return hipGetLastError();
}

hipError_t launch_pack(int mode, const Grid& g, const void* f, void* dense, bool to_dense, hipStream_t s)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz * NV;
    if (mode == MODE_FP64)
        hipLaunchKernelGGL(k_pack<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, g, (double*)f,
                           (double*)dense, to_dense ? 1 : 0);
    else
        hipLaunchKernelGGL(k_pack<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, g, (float*)f,
                           (float*)dense, to_dense ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_batch_step(int, const SolveDesc*, const Tile*, int, int, hipStream_t)
{
    return hipErrorNotSupported;
}

hipError_t launch_batch_ghosts(int, const SolveDesc*, int, int, hipStream_t)
{
    return hipErrorNotSupported;
}

}  // namespace lbm3d
