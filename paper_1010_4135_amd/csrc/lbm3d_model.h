// Device-side model of the 15-velocity FD-LB scheme: velocity signs,
// moment recovery, equilibrium, minmod and the per-node update.
#pragma once

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

// f^eq = rho (A + B s + D s^2) of Eqs. (eq)/(e18) for all 15 velocities.
// The group coefficients A, B depend on T and u^2 and are formed in the
// moment type M; the 15 values are then evaluated in the bulk type C.
template <typename C, typename M>
__device__ __forceinline__ void equilibrium(const Macro<M>& q, const Model<M>& mm,
                                            const Model<C>& mc, C (&feq)[NV])
{
    const M usq = q.ux * q.ux + q.uy * q.uy + q.uz * q.uz;
    const C rho = static_cast<C>(q.rho);
    const C ar = static_cast<C>(mm.r_aT * q.T);
    const C ax = static_cast<C>(mm.x_a0 + mm.x_aT * q.T + mm.x_au * usq);
    const C bx = static_cast<C>(mm.x_b0 + mm.x_bT * q.T + mm.x_bu * usq);
    const C ad = static_cast<C>(mm.d_a0 + mm.d_aT * q.T + mm.d_au * usq);
    const C bd = static_cast<C>(mm.d_b0 + mm.d_bT * q.T + mm.d_bu * usq);
    const C ux = static_cast<C>(q.ux), uy = static_cast<C>(q.uy), uz = static_cast<C>(q.uz);
    feq[0] = rho * ar;
    const C u3[3] = {ux, uy, uz};
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const C s = mc.c1 * u3[a];
        const C even = rho * (ax + mc.x_d * s * s);
        const C odd = rho * (bx * s);
        feq[1 + 2 * a] = even + odd;
        feq[2 + 2 * a] = even - odd;
    }
    // four |s| classes of the diagonal group: s and -s share A + D s^2
    const C sxy = ux + uy, dxy = ux - uy;
    const C sv[4] = {mc.k * (sxy + uz), mc.k * (dxy + uz), mc.k * (sxy - uz), mc.k * (dxy - uz)};
    // diagonal d has signs (bit0: x, bit1: y, bit2: z); its s equals
    // +sv[c] or -sv[c] for the class c below
#pragma unroll
    for (int d = 0; d < 8; d++) {
        const int sx = (d & 1) ? -1 : 1, sy = (d & 2) ? -1 : 1, sz = (d & 4) ? -1 : 1;
        // normalise so the x sign is +: classes (+,+,+), (+,-,+), (+,+,-), (+,-,-)
        const int ny = sy * sx, nz = sz * sx;
        const int c = (ny < 0 ? 1 : 0) + (nz < 0 ? 2 : 0);
        const C s = sx > 0 ? sv[c] : -sv[c];
        feq[7 + d] = rho * (ad + s * (bd + mc.d_d * s));
    }
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

// ---------------------------------------------------- NND flux, one axis --
// Face values of the NND reconstruction along one axis for a velocity
// component of sign SG (Sec. 3, Eq. (nnd)): with h = v g,
//   v > 0:  g_{I+1/2} = f_I + mm(f_{I+1}-f_I, f_I-f_{I-1}) / 2
//   v < 0:  g_{I+1/2} = f_{I+1} - mm(f_{I+1}-f_I, f_{I+2}-f_{I+1}) / 2
// (the f^+ / f^- split with minmod odd and positively homogeneous).
// Returns g_{I+1/2} - g_{I-1/2}; fm2..fp2 are f at I-2..I+2 (the two values
// on the downwind far side are not used).
// Face value g_{I+1/2} for v > 0 from f_{I-1}, f_I, f_{I+1}.
template <typename C>
__device__ __forceinline__ C face_pos(C fm1, C f0, C fp1)
{
    return f0 + C(0.5) * minmod(fp1 - f0, f0 - fm1);
}
// Face value g_{I+1/2} for v < 0 from f_I, f_{I+1}, f_{I+2}.
template <typename C>
__device__ __forceinline__ C face_neg(C f0, C fp1, C fp2)
{
    return fp1 - C(0.5) * minmod(fp1 - f0, fp2 - fp1);
}
template <int SG, typename C>
__device__ __forceinline__ C nnd_diff(C fm2, C fm1, C f0, C fp1, C fp2)
{
    if constexpr (SG > 0)
        return face_pos(fm1, f0, fp1) - face_pos(fm2, fm1, f0);
    else
        return face_neg(f0, fp1, fp2) - face_neg(fm1, f0, fp1);
}

}  // namespace lbm3d
