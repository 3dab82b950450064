// Device-side model of the 15-velocity FD-LB scheme: velocity signs,
// moment recovery, equilibrium, minmod and the per-node update.
#pragma once

#include <type_traits>

#include "lbm3d_internal.h"

namespace lbm3d {

// Velocity order: 0 rest; 1..6 = c1 (+x, -x, +y, -y, +z, -z); 7..14 =
// (c2/sqrt3)(sx, sy, sz) with bit a of (i-7) giving the sign of axis a
// (clear = +).  Sec. 2, Eq. (vv).
__host__ __device__ constexpr int vsign(int i, int a)
{
    return i == 0 ? 0
         : (i <= 6 ? (((i - 1) >> 1) == a ? (((i - 1) & 1) ? -1 : 1) : 0)
                   : ((((i - 7) >> a) & 1) ? -1 : 1));
}
__host__ __device__ constexpr int vgroup(int i) { return i == 0 ? 0 : (i <= 6 ? 1 : 2); }

// minmod(X, Y) of Sec. 3 is the median of (X, Y, 0): same signs give the
// argument of smaller magnitude, otherwise 0.
__device__ __forceinline__ float minmod(float a, float b) { return __builtin_amdgcn_fmed3f(a, b, 0.0f); }
__device__ __forceinline__ double minmod(double a, double b)
{
    return fmax(fmin(a, b), fmin(fmax(a, b), 0.0));
}

// Macroscopic state of one node.
template <typename M>
struct Macro {
    M rho, ux, uy, uz, T;
};

// Moments of the 15 distributions, Eqs. (e1)-(e3) applied to f:
// rho = sum f, rho u = sum f v, rho (b T + u^2) = sum f (v^2 + eta^2).
template <typename M, typename C>
__device__ __forceinline__ Macro<M> moments(const C (&f)[NV], const Model<M>& m)
{
    M g[NV];
#pragma unroll
    for (int i = 0; i < NV; i++) g[i] = static_cast<M>(f[i]);
    const M sa = ((g[1] + g[2]) + (g[3] + g[4])) + (g[5] + g[6]);
    // Walsh sums of the diagonal group: total and one signed sum per axis
    const M p01 = g[7] + g[8], m01 = g[7] - g[8];
    const M p23 = g[9] + g[10], m23 = g[9] - g[10];
    const M p45 = g[11] + g[12], m45 = g[11] - g[12];
    const M p67 = g[13] + g[14], m67 = g[13] - g[14];
    const M sd = (p01 + p23) + (p45 + p67);
    const M dx = (m01 + m23) + (m45 + m67);
    const M dy = (p01 - p23) + (p45 - p67);
    const M dz = (p01 + p23) - (p45 + p67);
    Macro<M> q;
    q.rho = g[0] + sa + sd;
    const M jx = m.c1 * (g[1] - g[2]) + m.k * dx;
    const M jy = m.c1 * (g[3] - g[4]) + m.k * dy;
    const M jz = m.c1 * (g[5] - g[6]) + m.k * dz;
    const M E = m.e0sq * g[0] + m.c1sq * sa + m.c2sq * sd;
    const M ir = M(1) / q.rho;
    q.ux = jx * ir;
    q.uy = jy * ir;
    q.uz = jz * ir;
    const M usq = q.ux * q.ux + q.uy * q.uy + q.uz * q.uz;
    q.T = (E * ir - usq) * m.inv_b;
    return q;
}

// Group coefficients of Eqs. (eq)/(e18) for one macroscopic state: A and B
// of each group depend on T and u^2 and are formed in the moment type M,
// then everything is taken to the bulk type C.
template <typename C>
struct EqCoef {
    C rho, ar, ax, bx, ad, bd, ux, uy, uz;
};

template <typename C, typename M>
__device__ __forceinline__ EqCoef<C> eq_coef(const Macro<M>& q, const Model<M>& mm)
{
    const M usq = q.ux * q.ux + q.uy * q.uy + q.uz * q.uz;
    EqCoef<C> c;
    c.rho = static_cast<C>(q.rho);
    c.ar = static_cast<C>(mm.r_aT * q.T);
    c.ax = static_cast<C>(mm.x_a0 + mm.x_aT * q.T + mm.x_au * usq);
    c.bx = static_cast<C>(mm.x_b0 + mm.x_bT * q.T + mm.x_bu * usq);
    c.ad = static_cast<C>(mm.d_a0 + mm.d_aT * q.T + mm.d_au * usq);
    c.bd = static_cast<C>(mm.d_b0 + mm.d_bT * q.T + mm.d_bu * usq);
    c.ux = static_cast<C>(q.ux);
    c.uy = static_cast<C>(q.uy);
    c.uz = static_cast<C>(q.uz);
    return c;
}

// f_i^eq = rho (A + B s + D s^2), s = v_i.u, for velocity i.  The same
// operations for a compile-time i (folded) and a per-lane i (selected), so
// both agree bitwise.  Each value is its own statement: with expression-
// local contraction the rounding then does not depend on the caller.
template <typename C>
__device__ __forceinline__ C feq_vel(int i, const EqCoef<C> c, const Model<C>& mc)
{
    if (i == 0) return c.rho * c.ar;
    if (i <= 6) {
        // (selects on values: an index into the struct would send it to
        // private memory)
        const int a = (i - 1) >> 1;
        const C ux = c.ux, uy = c.uy, uz = c.uz;
        const C uyz = a == 1 ? uy : uz;
        const C u = a == 0 ? ux : uyz;
        const C s = mc.c1 * u;
        const C t = mc.x_d * s;
        const C w = t * s + c.ax;
        const C even = c.rho * w;
        const C bs = c.bx * s;
        const C odd = c.rho * bs;
        return ((i - 1) & 1) ? even - odd : even + odd;
    }
    // diagonal d = i - 7, signs (bit0: x, bit1: y, bit2: z); normalised so
    // that the x sign is +, s is +/- k ((ux +/- uy) +/- uz)
    const int d = i - 7;
    const bool fy = ((d >> 1) ^ d) & 1, fz = ((d >> 2) ^ d) & 1;  // y, z sign differs from x
    const C b = fy ? c.ux - c.uy : c.ux + c.uy;
    const C t = fz ? b - c.uz : b + c.uz;
    const C sv = mc.k * t;
    const C s = (d & 1) ? -sv : sv;
    const C h = mc.d_d * s + c.bd;
    const C w = s * h + c.ad;
    return c.rho * w;
}

// f^eq of Eqs. (eq)/(e18) for all 15 velocities, evaluated in the moment
// type M and rounded once to the bulk type C.  (In the FP32_T64 mode the
// polynomial A + B s + D s^2 cancels strongly at high Mach number -- by a
// factor 8 for the upwind axis velocity at Mach 10 -- so it is evaluated in
// double like the temperature it depends on.)
template <typename C, typename M>
__device__ __forceinline__ void equilibrium(const Macro<M>& q, const Model<M>& mm,
                                            const Model<C>& mc, C (&feq)[NV])
{
    (void)mc;
    const EqCoef<M> c = eq_coef<M, M>(q, mm);
#pragma unroll
    for (int i = 0; i < NV; i++) feq[i] = static_cast<C>(feq_vel<M>(i, c, mm));
}

enum { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_INFLOW = 2, BC_REFLECT = 3 };
enum { H_NONFINITE = 1u, H_RHO = 2u, H_T = 4u };

// ----------------------------------------------------------------- types --
template <int MODE> struct Types;
template <> struct Types<MODE_FP64>     { using S = double; using C = double; using M = double; };
template <> struct Types<MODE_FP32>     { using S = float;  using C = float;  using M = float;  };
template <> struct Types<MODE_FP32_T64> { using S = float;  using C = float;  using M = double; };

template <typename T> __device__ __forceinline__ const Model<T>& pick(const Model<double>& d, const Model<float>& f);
template <> __device__ __forceinline__ const Model<double>& pick<double>(const Model<double>& d, const Model<float>&) { return d; }
template <> __device__ __forceinline__ const Model<float>& pick<float>(const Model<double>&, const Model<float>& f) { return f; }

template <typename M>
__device__ __forceinline__ uint32_t health_bits(const Macro<M>& q)
{
    uint32_t h = 0;
    if (!(q.rho > M(0))) h |= H_RHO;
    if (!(q.T > M(0))) h |= H_T;
    if (!isfinite(q.rho) || !isfinite(q.T) || !isfinite(q.ux) || !isfinite(q.uy) || !isfinite(q.uz))
        h |= H_NONFINITE;
    return h;
}

// Add health bits to a solve's health word, one atomic per wavefront: the
// bits are OR-ed over the wavefront's live lanes first.  A per-lane atomic
// would put every unhealthy node of a tile on the same address (a solve with
// T <= 0 along a whole interface plane then queues thousands of atomics on
// one L2 channel at each tile end).
__device__ __forceinline__ void report_health(uint32_t* health, uint32_t h)
{
    uint32_t w = 0;
    if (__ballot(h & H_NONFINITE)) w |= H_NONFINITE;
    if (__ballot(h & H_RHO)) w |= H_RHO;
    if (__ballot(h & H_T)) w |= H_T;
    const unsigned first = (unsigned)__ffsll((long long)__ballot(1)) - 1u;
    if (w && __lane_id() == first) atomicOr(health, w);
}

// ------------------------------------------------------- per-node update --
// Explicit fused multiply-add, so that every kernel rounds the update the
// same way whatever the compiler's contraction choices in its context.
__device__ __forceinline__ float fmac(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmac(double a, double b, double c) { return __builtin_fma(a, b, c); }

// NND flux difference along one axis (Sec. 3, Eq. (nnd)).  With h = v g and
// e_k = f_{I+k} - f_{I+k-1} the differences of consecutive nodes:
//   v > 0:  g_{I+1/2} = f_I + mm(e_1, e_0)/2, so
//           g_{I+1/2} - g_{I-1/2} = e_0 + (mm(e_1, e_0) - mm(e_0, e_-1)) / 2;
//   v < 0:  g_{I+1/2} = f_{I+1} - mm(e_1, e_2)/2, so
//           g_{I+1/2} - g_{I-1/2} = e_1 - (mm(e_1, e_2) - mm(e_0, e_1)) / 2
// (the f^+ / f^- split of the paper, minmod being odd and positively
// homogeneous).  The _c forms take the second minmod from the node before
// along the axis and return the first one for the node after: a sweep along
// the axis then evaluates one minmod per node, with bitwise the same result.
template <typename C>
__device__ __forceinline__ C nnd_pos(C em1, C e0, C e1)
{
    return fmac(C(0.5), minmod(e1, e0) - minmod(e0, em1), e0);
}
template <typename C>
__device__ __forceinline__ C nnd_neg(C e0, C e1, C e2)
{
    return fmac(C(-0.5), minmod(e1, e2) - minmod(e0, e1), e1);
}
template <typename C>
__device__ __forceinline__ C nnd_pos_c(C e0, C e1, C& mprev)
{
    const C m = minmod(e1, e0);
    const C d = fmac(C(0.5), m - mprev, e0);
    mprev = m;
    return d;
}
template <typename C>
__device__ __forceinline__ C nnd_neg_c(C e1, C e2, C& mprev)
{
    const C m = minmod(e1, e2);
    const C d = fmac(C(-0.5), m - mprev, e1);
    mprev = m;
    return d;
}

// The comparison variant of Sec. 3 (the original Kataoka-Tsutahara scheme):
// the second-order upwind difference, g_{I+1/2} = f_I + e_0 / 2 for v > 0 and
// f_{I+1} - e_2 / 2 for v < 0, i.e. the NND forms with the limited slope
// replaced by the upwind one:
//   v > 0:  (3 f_I - 4 f_{I-1} + f_{I-2}) / 2 = e_0 + (e_0 - e_-1) / 2,
//   v < 0:  (-3 f_I + 4 f_{I+1} - f_{I+2}) / 2 = e_1 - (e_2 - e_1) / 2.
template <typename C>
__device__ __forceinline__ C up2_pos(C em1, C e0)
{
    return fmac(C(0.5), e0 - em1, e0);
}
template <typename C>
__device__ __forceinline__ C up2_neg(C e1, C e2)
{
    return fmac(C(-0.5), e2 - e1, e1);
}

// Laplacian of Eq. (lp) from one part per axis: along an axis the velocity
// is advected on, the part is e_1 - e_0 = f_{I+1} - 2 f_I + f_{I-1}; along
// the other axes it is f_{I+1} + f_{I-1}, whose -2 f_I terms are added once.
template <int I, typename C>
__device__ __forceinline__ C lap_sum(C lx, C ly, C lz, C f0)
{
    constexpr int G = vgroup(I);
    if constexpr (G == 0) {
        return fmac(C(-6), f0, (lx + ly) + lz);
    } else {
        constexpr int ax = (I - 1) >> 1;
        const C own = ax == 0 ? lx : (ax == 1 ? ly : lz);
        const C pb = ax == 0 ? ly : lx;
        const C pc = ax == 2 ? ly : lz;
        return own + fmac(C(-4), f0, pb + pc);
    }
}

// f_i^{n+1} of Eq. (fi1) for velocity I from its flux differences along x,
// y, z (those with v_ia = 0 are ignored) and Laplacian parts (used for the
// rest and axis velocities):
//   f + dt/tau (f^eq - f) - dt/dx sum_a v_ia D_a + lambda_i dt/dx^2 Lap f.
template <int I, typename C>
__device__ __forceinline__ C node_update(C f0, C feq, C dx_, C dy_, C dz_, C lx, C ly, C lz, const Model<C>& m)
{
    constexpr int SX = vsign(I, 0), SY = vsign(I, 1), SZ = vsign(I, 2), G = vgroup(I);
    const C a = (G == 1) ? m.a1 : m.ad;  // dt/dx |v_ia|
    C acc = fmac(m.k_bgk, feq - f0, f0);
    if constexpr (SX != 0) acc = fmac(SX > 0 ? -a : a, dx_, acc);
    if constexpr (SY != 0) acc = fmac(SY > 0 ? -a : a, dy_, acc);
    if constexpr (SZ != 0) acc = fmac(SZ > 0 ? -a : a, dz_, acc);
    if constexpr (G <= 1) acc = fmac(G == 0 ? m.k_lap0 : m.k_lap1, lap_sum<I, C>(lx, ly, lz, f0), acc);
    return acc;
}

// Compile-time loop.
template <int N, int I = 0, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<N, I + 1>(f);
    }
}

}  // namespace lbm3d
