// Device kernels of the lbm3d library for gfx950: initial state, the fused
// time step, boundary layers, moments, FP64 conservation totals and the
// checkpoint pack/unpack.
#include "lbm3d_tile.h"

#include <hip/hip_ext.h>

#include <cmath>

namespace lbm3d {

// --------------------------------------------------------- the fused step --
// One explicit step of Eq. (lp) with NND convection at every interior node:
//   f_i^{n+1} = f_i - dt/dx sum_a v_ia (g_{I+1/2} - g_{I-1/2})
//               - dt/tau (f_i - f_i^eq) + lambda_i dt/dx^2 sum_a (f_{I+1} - 2 f_I + f_{I-1})
// reading every term at level n (forward Euler, Eq. (fi1)).  The boundary
// layers of f^n hold valid values, so every neighbour load is in bounds.
// This one-node-per-thread kernel and the tiled one evaluate the same
// operations per node (node_update and the NND helpers), so they agree
// bitwise.
template <int I, bool U2, typename S, typename C>
__device__ __forceinline__ void update_one(const S* __restrict__ fi, S* __restrict__ fo, int64_t site,
                                           const int64_t (&xo)[4], int64_t sy, int64_t sz, C f0, C feq,
                                           const Model<C>& m)
{
    constexpr int SG[3] = {vsign(I, 0), vsign(I, 1), vsign(I, 2)};
    constexpr int G = vgroup(I);
    // neighbour at distance d (-2, -1, 1, 2) along axis a: x neighbours
    // through the per-thread offsets xo (which reach the x layers), y and z
    // neighbours by stride
    auto nb = [&](int a, int d) {
        const int64_t o = a == 0 ? xo[d < 0 ? d + 2 : d + 1] : site + d * (a == 1 ? sy : sz);
        return static_cast<C>(fi[o]);
    };
    C D[3] = {C(0), C(0), C(0)}, L[3] = {C(0), C(0), C(0)};
#pragma unroll
    for (int a = 0; a < 3; a++) {
        if (SG[a] > 0) {
            const C fm2 = nb(a, -2), fm1 = nb(a, -1), fp1 = nb(a, 1);
            const C e0 = f0 - fm1, e1 = fp1 - f0;
            D[a] = U2 ? up2_pos(fm1 - fm2, e0) : nnd_pos(fm1 - fm2, e0, e1);
            L[a] = e1 - e0;
        } else if (SG[a] < 0) {
            const C fm1 = nb(a, -1), fp1 = nb(a, 1), fp2 = nb(a, 2);
            const C e0 = f0 - fm1, e1 = fp1 - f0;
            D[a] = U2 ? up2_neg(e1, fp2 - fp1) : nnd_neg(e0, e1, fp2 - fp1);
            L[a] = e1 - e0;
        } else if (G <= 1) {
            L[a] = nb(a, -1) + nb(a, 1);
        }
    }
    fo[site] = static_cast<S>(node_update<I, C>(f0, feq, D[0], D[1], D[2], L[0], L[1], L[2], m));
}

template <bool U2, typename S, typename C, int I = 0>
__device__ __forceinline__ void update_all(const S* __restrict__ f, S* __restrict__ fn, int64_t site,
                                           const int64_t (&xo)[4], int64_t sv, int64_t sy, int64_t sz,
                                           const C (&fc)[NV], const C (&feq)[NV], const Model<C>& m)
{
    if constexpr (I < NV) {
        update_one<I, U2, S, C>(f + I * sv, fn + I * sv, site, xo, sy, sz, fc[I], feq[I], m);
        update_all<U2, S, C, I + 1>(f, fn, site, xo, sv, sy, sz, fc, feq, m);
    }
}

// Offsets (within a velocity plane) of the x neighbours at distance -2, -1,
// +1, +2 of node (x, y, z) at `site`: along the row, or in the x-layer block
// for those beyond a face when rows are dense.
__device__ __forceinline__ void x_offsets(const Grid& g, int x, int y, int z, int64_t site, int64_t (&xo)[4])
{
    const int d[4] = {-2, -1, 1, 2};
    const int64_t row = g.xg + (int64_t)(z + NG) * g.xgz + (int64_t)(y + NG) * 4;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int xx = x + d[k];
        const bool out = g.xg != 0 && (xx < 0 || xx >= g.nx);
        const int64_t layer = xx < 0 ? xx + 2 : 2 + (xx - g.nx);  // 0: -2, 1: -1, 2: nx, 3: nx+1
        xo[k] = out ? row + layer : site + d[k];
    }
}

// U2: the second-order upwind variant in place of NND (untiled only).
template <int MODE, bool U2>
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
    report_health(health, health_bits(q));
    C feq[NV];
    equilibrium<C, M>(q, mm, mc, feq);
    int64_t xo[4];
    x_offsets(g, x, y, z, site, xo);
    update_all<U2, S, C>(f, fn, site, xo, g.sv, g.sy, g.sz, fc, feq, mc);
}

// Tiled fused step: one workgroup per 64 x BY x TZ tile (see lbm3d_tile.h).

template <int MODE, int BY, bool NT>
__global__ void __launch_bounds__(TILE_X * BY)
k_step_tiled(StepArgs<MODE> A, Model<double> md, Model<float> mf, int ntx, int nty, int tz)
{
    __shared__ TilePlane<BY, typename Types<MODE>::S> P[2];
    const int t = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    // tiles numbered x fastest, then y, then the z chunk
    const int txi = t % ntx;
    const int r = t / ntx;
    const int tyi = r % nty;
    const int tzi = r / nty;
    const int z0 = tzi * tz;
    const int z1 = min(z0 + tz, A.g.nz);
    step_tile<MODE, BY, true, NT>(A, md, mf, txi * TILE_X, tyi * BY, z0, z1, P);
}

// Batched fused step: persistent workgroups walk a packed list of tiles from
// many solves (any sizes, one precision), each tile advanced by the same
// step_tile body as a single solve, so every solve's result is bitwise the
// same alone or in any batch.
// A uniform value the optimiser may not re-derive: it stays in a scalar
// register (or a spill slot) rather than being loaded again from the
// read-only table it came from.
template <typename T>
__device__ __forceinline__ void keep(T& v)
{
    asm volatile("" : "+s"(v));
}
template <typename T>
__device__ __forceinline__ void keep_model(Model<T>& m)
{
    keep(m.c1); keep(m.k); keep(m.c1sq); keep(m.c2sq); keep(m.e0sq); keep(m.inv_b); keep(m.r_aT);
    keep(m.x_a0); keep(m.x_aT); keep(m.x_au); keep(m.x_b0); keep(m.x_bT); keep(m.x_bu); keep(m.x_d);
    keep(m.d_a0); keep(m.d_aT); keep(m.d_au); keep(m.d_b0); keep(m.d_bT); keep(m.d_bu); keep(m.d_d);
    keep(m.k_adv); keep(m.k_bgk); keep(m.k_lap0); keep(m.k_lap1); keep(m.a1); keep(m.ad);
}

template <int MODE, int BY, bool NT>
__global__ void __launch_bounds__(TILE_X * BY)
k_batch_step(const BatchSolve* __restrict__ solves, const BatchTile* __restrict__ tiles, BatchQueue* queue,
             int nlists, int parity, const BatchCount* __restrict__ counts)
{
    using S = typename Types<MODE>::S;
    __shared__ TilePlane<BY, S> P[2];
    __shared__ int s_k;
    // workgroup b works on list b mod nlists (dispatch places workgroup b on
    // XCD b mod 8, so a list's tiles share one L2); the `per` workgroups of a
    // list take its tiles in order from the list's counter
    const int list = (int)blockIdx.x % nlists;
    const int per = (int)gridDim.x / nlists;
    const int first = queue->first[list];
    const int cnt = queue->first[list + 1] - first;
    for (;;) {
        if (threadIdx.x == 0) {
            const int k = (int)atomicAdd(&queue->next[list], 1u);
            // every workgroup makes exactly one grab past the end, so the
            // one that draws cnt + per - 1 is the last to touch the counter:
            // it leaves it at zero for the next launch
            if (k == cnt + per - 1) atomicExch(&queue->next[list], 0u);
            s_k = k;
        }
        __syncthreads();
        const int k = s_k;
        if (k >= cnt) break;
        const BatchTile tile = tiles[first + k];
        const BatchSolve& d = solves[tile.solve];
        // the member's parity: given (timing trials), or from its own step
        // count, which also says whether it still steps in this run (the
        // same for the whole workgroup, so the barriers stay uniform)
        int par = parity;
        bool run = true;
        if (parity < 0) {
            const BatchCount c = counts[tile.solve];
            par = c.done & 1;
            run = c.done < c.target;
        }
        if (run) {
            StepArgs<MODE> A;
            A.g = d.g;
            A.bc = d.bc;
            const int cur = d.cur0 ^ par;
            A.f = (const S*)d.f[cur];
            A.fn = (S*)d.f[cur ^ 1];
            A.health = d.health;
#pragma unroll
            for (int j = 0; j < 10; j++) A.xin[j / 5][j % 5] = d.xin[j / 5][j % 5];
            Model<double> md = d.md;
            Model<float> mf = d.mf;
            // the tile's solve is read once per tile: without this the
            // compiler re-loads its constants and strides from the table in
            // every plane, each a scalar-memory round trip the plane then
            // waits for
            keep(A.g.sy); keep(A.g.sz); keep(A.g.sv); keep(A.g.org); keep(A.g.sink); keep(A.g.xg);
            keep(A.f); keep(A.fn);
            keep_model(mf);
            step_tile<MODE, BY, true, NT>(A, md, mf, tile.txi * TILE_X, tile.tyi * BY, tile.z0, tile.z1, P);
        }
        lds_barrier();  // the plane buffers (and s_k) are reused by the next tile
    }
}

// Step counts of the batch members after a step: done += 1 while below the
// target.
__global__ void __launch_bounds__(64) k_batch_count(BatchCount* __restrict__ counts, int n)
{
    const int m = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (m < n && counts[m].done < counts[m].target) counts[m].done += 1;
}

// Health words of the members of a batch, gathered into one array.
__global__ void __launch_bounds__(64)
k_gather_health(const BatchSolve* __restrict__ solves, int n, uint32_t* __restrict__ out)
{
    const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k < n) out[k] = *solves[k].health;
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
// are f^eq of those values.  Periodic faces copy f from the other side.  One
// thread per line of nodes perpendicular to a face (x fastest on the y and z
// faces), all requested faces in one launch; the per-line work is the same
// layer_line routine the tiled step uses for the layers it writes itself,
// so both paths produce identical layers.  Only face layers are written:
// the stencils never read edges or corners.
struct FixedStates {
    double q[6][5];  // (rho, ux, uy, uz, T) per fixed-state face
};

// Line j (over the selected faces in order) of one solve's boundary layers.
// Line counts and indices are 32-bit (32-bit division is a short native
// sequence, 64-bit division a long emulated one): the host accepts only
// grids whose velocity plane holds fewer than 2e9 elements, so the lines of
// all six faces, 2 (nx ny + ny nz + nz nx), stay below 4.01e9 < 2^32.
template <int MODE>
__device__ __forceinline__ void layer_job(const StepArgs<MODE>& A, const Model<double>& md, const Model<float>& mf,
                                          const FixedStates* fx, uint32_t faces, uint32_t j)
{
    using C = typename Types<MODE>::C;
    using M = typename Types<MODE>::M;
    const Grid& g = A.g;
    const uint32_t nx = (uint32_t)g.nx, ny = (uint32_t)g.ny, nz = (uint32_t)g.nz;
#pragma unroll
    for (int face = 0; face < 6; face++) {
        if (!((faces >> face) & 1)) continue;
        const int axis = face >> 1;
        const uint32_t cnt = axis == 0 ? ny * nz : axis == 1 ? nx * nz : nx * ny;
        if (j >= cnt) {
            j -= cnt;
            continue;
        }
        int cx = 0, cy = 0, cz = 0;
        if (axis == 0) { cy = (int)(j % ny); cz = (int)(j / ny); }
        else if (axis == 1) { cx = (int)(j % nx); cz = (int)(j / nx); }
        else { cx = (int)(j % nx); cy = (int)(j / nx); }
        const uint32_t line = (uint32_t)(g.org + (int64_t)cz * g.sz + (int64_t)cy * g.sy + cx);
        const uint32_t st = axis == 0 ? 1u : axis == 1 ? (uint32_t)g.sy : (uint32_t)g.sz;
        const int n = axis == 0 ? g.nx : axis == 1 ? g.ny : g.nz;
        const int side = face & 1;
        // the two layer nodes of the line: beyond its ends, or in the
        // x-layer block of a dense-row array
        uint32_t l1 = line + (uint32_t)(side ? n : -1) * st;
        uint32_t l2 = line + (uint32_t)(side ? n + 1 : -2) * st;
        if (axis == 0 && g.xg != 0) {
            const uint32_t row = (uint32_t)(g.xg + (int64_t)(cz + NG) * g.xgz + (int64_t)(cy + NG) * 4);
            l1 = row + (side ? 2u : 1u);
            l2 = row + (side ? 3u : 0u);
        }
        if (A.bc.kind[face] == BC_INFLOW) {
            if (!fx) return;
            Macro<M> q;
            q.rho = static_cast<M>(fx->q[face][0]);
            q.ux = static_cast<M>(fx->q[face][1]);
            q.uy = static_cast<M>(fx->q[face][2]);
            q.uz = static_cast<M>(fx->q[face][3]);
            q.T = static_cast<M>(fx->q[face][4]);
            C e[NV];
            equilibrium<C, M>(q, pick<M>(md, mf), pick<C>(md, mf), e);
            store_node(gptr(A.fn), g.sv, l1, e);
            store_node(gptr(A.fn), g.sv, l2, e);
        } else {
            layer_line<MODE>(A, pick<M>(md, mf), pick<C>(md, mf), face, line, st, n, l1, l2);
        }
        return;
    }
}

template <int MODE>
__global__ void __launch_bounds__(64)
k_layers(StepArgs<MODE> A, Model<double> md, Model<float> mf, FixedStates fx, uint32_t faces)
{
    layer_job<MODE>(A, md, mf, &fx, faces, blockIdx.x * blockDim.x + threadIdx.x);
}

// Boundary layers of many solves in one launch: job k covers workgroups
// [first[k], first[k+1]) of solve jobs[k].solve (faces jobs[k].faces);
// block_job[b] names the job of workgroup b.
template <int MODE>
__global__ void __launch_bounds__(64)
k_layers_batch(const BatchSolve* __restrict__ solves, const BatchLayerJob* __restrict__ jobs,
               const int32_t* __restrict__ block_job, int parity, const BatchCount* __restrict__ counts)
{
    using S = typename Types<MODE>::S;
    const int b = (int)blockIdx.x;
    const BatchLayerJob jb = jobs[block_job[b]];
    const BatchSolve& d = solves[jb.solve];
    int par = parity;
    if (parity < 0) {
        // (read before this step's count; members past their target did
        // not step)
        const BatchCount c = counts[jb.solve];
        if (c.done >= c.target) return;
        par = c.done & 1;
    }
    StepArgs<MODE> A;
    A.g = d.g;
    A.bc = d.bc;
    const int cur = d.cur0 ^ par;
    A.f = nullptr;
    A.fn = (S*)d.f[cur ^ 1];
    A.health = nullptr;
    layer_job<MODE>(A, d.md, d.mf, nullptr, jb.faces, (uint32_t)(b - jb.first) * 64u + threadIdx.x);
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

template <int MODE, int BY>
static void launch_tiled(const Grid& g, const FaceBC& bc, int tz, bool stream, const Model<double>& md,
                         const Model<float>& mf, const double (*inflow)[5], const void* f, void* fn,
                         uint32_t* health, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    using S = typename Types<MODE>::S;
    const int ntx = (g.nx + TILE_X - 1) / TILE_X;
    const int nty = (g.ny + BY - 1) / BY;
    const int ntz = (g.nz + tz - 1) / tz;
    const int nb = ntx * nty * ntz;
    StepArgs<MODE> A;
    A.g = g;
    A.bc = bc;
    A.f = (const S*)f;
    A.fn = (S*)fn;
    A.health = health;
    x_fixed_states(inflow, A.xin);
    const dim3 grid(nb), block(TILE_X * BY);
    if (e0 || e1) {
        if (stream)
            hipExtLaunchKernelGGL(k_step_tiled<MODE, BY, true>, grid, block, 0, s, e0, e1, 0, A, md, mf, ntx, nty, tz);
        else
            hipExtLaunchKernelGGL(k_step_tiled<MODE, BY, false>, grid, block, 0, s, e0, e1, 0, A, md, mf, ntx, nty,
                                  tz);
    } else if (stream) {
        k_step_tiled<MODE, BY, true><<<grid, block, 0, s>>>(A, md, mf, ntx, nty, tz);
    } else {
        k_step_tiled<MODE, BY, false><<<grid, block, 0, s>>>(A, md, mf, ntx, nty, tz);
    }
}

template <int MODE>
static void launch_untiled(dim3 grid, dim3 block, bool upwind2, const Grid& g, const Model<double>& md,
                           const Model<float>& mf, const void* f, void* fn, uint32_t* health, hipStream_t s,
                           hipEvent_t e0, hipEvent_t e1)
{
    using S = typename Types<MODE>::S;
    const S* fi = (const S*)f;
    S* fo = (S*)fn;
    if (e0 || e1) {
        if (upwind2)
            hipExtLaunchKernelGGL(k_step<MODE, true>, grid, block, 0, s, e0, e1, 0, g, md, mf, fi, fo, health);
        else
            hipExtLaunchKernelGGL(k_step<MODE, false>, grid, block, 0, s, e0, e1, 0, g, md, mf, fi, fo, health);
    } else if (upwind2) {
        k_step<MODE, true><<<grid, block, 0, s>>>(g, md, mf, fi, fo, health);
    } else {
        k_step<MODE, false><<<grid, block, 0, s>>>(g, md, mf, fi, fo, health);
    }
}

hipError_t launch_step(int mode, const Grid& g, const FaceBC& bc, const TileCfg& tc, const Model<double>& md,
                       const Model<float>& mf, const double (*inflow)[5], const void* f, void* fn,
                       uint32_t* health, hipStream_t s, bool upwind2, hipEvent_t e0, hipEvent_t e1)
{
    if (upwind2 && tc.by != 0) return hipErrorInvalidValue;
    if (tc.by != 0) {
        switch (tc.by) {
        case 2:
            LBM3D_DISPATCH(mode, launch_tiled<MD, 2>(g, bc, tc.tz, tc.stream, md, mf, inflow, f, fn, health, s, e0, e1));
            break;
        case 8:
            if (mode == MODE_FP64) return hipErrorInvalidValue;
            if (mode == MODE_FP32)
                launch_tiled<MODE_FP32, 8>(g, bc, tc.tz, tc.stream, md, mf, inflow, f, fn, health, s, e0, e1);
            else
                launch_tiled<MODE_FP32_T64, 8>(g, bc, tc.tz, tc.stream, md, mf, inflow, f, fn, health, s, e0, e1);
            break;
        default:
            LBM3D_DISPATCH(mode, launch_tiled<MD, 4>(g, bc, tc.tz, tc.stream, md, mf, inflow, f, fn, health, s, e0, e1));
            break;
        }
        return hipGetLastError();
    }
    const dim3 grid((g.nx + TX - 1) / TX, (g.ny + TY - 1) / TY, g.nz), block(TX, TY);
    LBM3D_DISPATCH(mode, launch_untiled<MD>(grid, block, upwind2, g, md, mf, f, fn, health, s, e0, e1));
    return hipGetLastError();
}

hipError_t launch_ghosts(int mode, const Grid& g, const FaceBC& bc, const Model<double>& md,
                         const double (*inflow)[5], bool include_fixed, void* f, hipStream_t s,
                         uint32_t face_mask)
{
    const Model<float> mf = to_float(md);
    uint32_t faces = 0;
    int64_t lines = 0;
    FixedStates fx{};
    for (int face = 0; face < 6; face++) {
        const bool fixed = bc.kind[face] == BC_INFLOW;
        if (fixed ? !include_fixed : !((face_mask >> face) & 1)) continue;
        faces |= 1u << face;
        const int axis = face >> 1;
        lines += axis == 0 ? (int64_t)g.ny * g.nz : axis == 1 ? (int64_t)g.nx * g.nz : (int64_t)g.nx * g.ny;
        if (fixed) {
            const double* st = inflow[face];
            fx.q[face][0] = st[0];
            fx.q[face][1] = st[1];
            fx.q[face][2] = st[2];
            fx.q[face][3] = st[3];
            fx.q[face][4] = st[4] / st[0];  // T = p / rho
        }
    }
    if (!faces) return hipSuccess;
    // one wavefront per block: the x-face lines (scattered rows) then spread
    // over every CU instead of crowding the first few
    const unsigned nb = blocks_for(lines, 64);
    LBM3D_DISPATCH(mode, {
        StepArgs<MD> A{};
        A.g = g;
        A.bc = bc;
        A.f = nullptr;
        A.fn = (typename Types<MD>::S*)f;
        A.health = nullptr;
        k_layers<MD><<<dim3(nb), dim3(64), 0, s>>>(A, md, mf, fx, faces);
    });
    return hipGetLastError();
}

hipError_t launch_moments(int mode, const Grid& g, const Model<double>& md, const void* f, double* q5,
                          hipStream_t s)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const Model<float> mf = to_float(md);
    LBM3D_DISPATCH(mode, k_moments<MD><<<dim3(blocks_for(n, 256)), dim3(256), 0, s>>>(g, md, mf, (const typename Types<MD>::S*)f, q5));
    return hipGetLastError();
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

hipError_t launch_gather_health(const BatchSolve* solves, int n, uint32_t* out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_gather_health<<<dim3(blocks_for(n, 64)), dim3(64), 0, s>>>(solves, n, out);
    return hipGetLastError();
}

hipError_t launch_batch_layers(int mode, const BatchSolve* solves, const BatchLayerJob* jobs, const int32_t* block_job,
                               int nblocks, int parity, const BatchCount* counts, hipStream_t s)
{
    if (nblocks <= 0) return hipSuccess;
    if (parity < 0 && !counts) return hipErrorInvalidValue;
    LBM3D_DISPATCH(mode,
                   k_layers_batch<MD><<<dim3(nblocks), dim3(64), 0, s>>>(solves, jobs, block_job, parity, counts));
    return hipGetLastError();
}

hipError_t launch_batch_count(BatchCount* counts, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_batch_count<<<dim3(blocks_for(n, 64)), dim3(64), 0, s>>>(counts, n);
    return hipGetLastError();
}

template <int MODE, int BY>
static void launch_batch(unsigned nblocks, bool stream, const BatchSolve* solves, const BatchTile* tiles,
                         BatchQueue* queue, int nlists, int parity, const BatchCount* counts, hipStream_t s)
{
    if (stream)
        k_batch_step<MODE, BY, true>
            <<<dim3(nblocks), dim3(TILE_X * BY), 0, s>>>(solves, tiles, queue, nlists, parity, counts);
    else
        k_batch_step<MODE, BY, false>
            <<<dim3(nblocks), dim3(TILE_X * BY), 0, s>>>(solves, tiles, queue, nlists, parity, counts);
}

hipError_t launch_batch_step(int mode, int by, bool stream, const BatchSolve* solves, const BatchTile* tiles,
                             BatchQueue* queue, int nlists, int nblocks, int parity, const BatchCount* counts,
                             hipStream_t s)
{
    if (nblocks <= 0 || nlists <= 0 || nlists > BATCH_MAX_LISTS || nblocks % nlists) return hipErrorInvalidValue;
    if (parity < 0 && !counts) return hipErrorInvalidValue;
    // the batch's tile heights: 4 rows in FP64, 8 in the FP32 modes
    if (by != (mode == MODE_FP64 ? 4 : 8)) return hipErrorInvalidValue;
    const unsigned nb = (unsigned)nblocks;
    if (mode == MODE_FP64) launch_batch<MODE_FP64, 4>(nb, stream, solves, tiles, queue, nlists, parity, counts, s);
    else if (mode == MODE_FP32)
        launch_batch<MODE_FP32, 8>(nb, stream, solves, tiles, queue, nlists, parity, counts, s);
    else launch_batch<MODE_FP32_T64, 8>(nb, stream, solves, tiles, queue, nlists, parity, counts, s);
    return hipGetLastError();
}

}  // namespace lbm3d
