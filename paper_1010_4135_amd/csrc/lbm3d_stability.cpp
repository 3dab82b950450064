// Von Neumann stability analysis of the linearised scheme (Sec. 3): a small
// perturbation F exp(i k.x) of a uniform equilibrium grows per step by the
// amplification matrix
//   G_ij = (1 - dt/tau - sum_a (v_ia dt/dx) phi_ia) delta_ij
//          + (dt/tau) d f_i^eq / d f_j
//          + lambda_i dt sum_a (exp(i k_a dx) - 2 + exp(-i k_a dx)) / dx^2 delta_ij,
// with the NND symbol phi = (1 - at)(1 - exp(-i k_a dx)) for v_ia >= 0 and
// (1 - at)(exp(i k_a dx) - 1) for v_ia < 0 (at: the linearisation parameter
// of the limiter, |at| < 1/2).  The scheme is stable for max |omega| <= 1
// over the eigenvalues omega of G.  Host code only: no device call.
#include "lbm3d_api_impl.h"

#include <array>
#include <cmath>
#include <complex>
#include <vector>

namespace lbm3d {
namespace {

using cd = std::complex<double>;

struct Velocities {
    double v[NV][3];
    double e[NV];  // |v|^2 + eta^2
};

Velocities velocities(const Model<double>& m)
{
    Velocities s{};
    for (int i = 0; i < NV; i++) {
        if (i == 0) {
            s.e[i] = m.e0sq;
        } else if (i <= 6) {
            const int a = (i - 1) >> 1;
            s.v[i][a] = ((i - 1) & 1) ? -m.c1 : m.c1;
            s.e[i] = m.c1sq;
        } else {
            for (int a = 0; a < 3; a++) s.v[i][a] = (((i - 7) >> a) & 1) ? -m.k : m.k;
            s.e[i] = m.c2sq;
        }
    }
    return s;
}

// Jacobian d f_i^eq / d f_j at the state (rho, u, T), through the moments:
// d rho / d f_j = 1, d u_a / d f_j = (v_ja - u_a) / rho and
// d T / d f_j = ((e_j - E/rho) - 2 u.(v_j - u)) / (rho b), E/rho = b T + u^2.
void eq_jacobian(const Model<double>& m, const Velocities& s, const double q[5], double (&J)[NV][NV])
{
    const double rho = q[0], u[3] = {q[1], q[2], q[3]}, T = q[4];
    const double b = 1.0 / m.inv_b;
    const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const double er = b * T + usq;
    for (int i = 0; i < NV; i++) {
        const double si = s.v[i][0] * u[0] + s.v[i][1] * u[1] + s.v[i][2] * u[2];
        // group polynomials A = a0 + aT T + au u^2, B = b0 + bT T + bu u^2, D
        double a0 = 0, aT = m.r_aT, au = 0, b0 = 0, bT = 0, bu = 0, d = 0;
        if (i >= 1 && i <= 6) {
            a0 = m.x_a0; aT = m.x_aT; au = m.x_au; b0 = m.x_b0; bT = m.x_bT; bu = m.x_bu; d = m.x_d;
        } else if (i >= 7) {
            a0 = m.d_a0; aT = m.d_aT; au = m.d_au; b0 = m.d_b0; bT = m.d_bT; bu = m.d_bu; d = m.d_d;
        }
        const double A = a0 + aT * T + au * usq, B = b0 + bT * T + bu * usq;
        const double f_rho = A + B * si + d * si * si;        // d f^eq / d rho
        const double f_T = rho * (aT + bT * si);               // d f^eq / d T
        double f_u[3];                                         // d f^eq / d u_a
        for (int a = 0; a < 3; a++)
            f_u[a] = rho * (2.0 * u[a] * (au + bu * si) + (B + 2.0 * d * si) * s.v[i][a]);
        for (int j = 0; j < NV; j++) {
            double du[3], udv = 0.0;
            for (int a = 0; a < 3; a++) {
                du[a] = (s.v[j][a] - u[a]) / rho;
                udv += u[a] * (s.v[j][a] - u[a]);
            }
            const double dT = ((s.e[j] - er) - 2.0 * udv) / (rho * b);
            J[i][j] = f_rho + f_T * dT + f_u[0] * du[0] + f_u[1] * du[1] + f_u[2] * du[2];
        }
    }
}

// Spectral radius of G from the growth of its powers: with N = 2^20,
// |G^N|^(1/N) -> max |omega| (the excess over it is at most c^(1/N) for a
// condition constant c of the eigenvectors, below 2e-5 for c < 1e9).
// Squarings are rescaled to stay finite; logarithms carry the scale.
double spectral_radius(cd (&G)[NV][NV])
{
    constexpr int SQ = 20;
    cd M[NV][NV], P[NV][NV];
    for (int i = 0; i < NV; i++)
        for (int j = 0; j < NV; j++) M[i][j] = G[i][j];
    double logscale = 0.0;  // log of the factor divided out of M so far (of G^(2^t))
    for (int t = 0; t < SQ; t++) {
        double mx = 0.0;
        for (int i = 0; i < NV; i++)
            for (int j = 0; j < NV; j++) {
                cd acc = 0.0;
                for (int k = 0; k < NV; k++) acc += M[i][k] * M[k][j];
                P[i][j] = acc;
                mx = std::fmax(mx, std::abs(acc));
            }
        if (!(mx > 0.0) || !std::isfinite(mx)) return mx > 0.0 ? INFINITY : 0.0;
        for (int i = 0; i < NV; i++)
            for (int j = 0; j < NV; j++) M[i][j] = P[i][j] / mx;
        logscale = 2.0 * logscale + std::log(mx);
    }
    double fro = 0.0;
    for (int i = 0; i < NV; i++)
        for (int j = 0; j < NV; j++) fro += std::norm(M[i][j]);
    const double N = std::ldexp(1.0, SQ);
    return std::exp((logscale + 0.5 * std::log(fro)) / N);
}

}  // namespace

// max |omega| over k dx in [0, pi] (nk points) along `axis` for state q.
static double scan(const lbm3d_params* p, const double q[5], int axis, int nk, double* kdx_at)
{
    double om = 0.0, k = 0.0;
    if (lbm3d_stability(p, q, axis, 0.0, 3.14159265358979323846, nk, 0.0, &om, &k) != LBM3D_OK) return INFINITY;
    if (kdx_at) *kdx_at = k;
    return om;
}

int32_t admission(const lbm3d_params* p, const double* rho, const double* ux, const double* uy, const double* uz,
                  const double* pr, double* worst)
{
    const int64_t n = (int64_t)p->nx * p->ny * p->nz;
    if (n < 1) return LBM3D_E_INVAL;
    // the states at which the linearised scheme is least stable lie at the
    // extremes of the initial fields: the fastest node, the coldest and the
    // hottest; fixed inflow states are added
    int64_t kmax_u = 0, kmin_t = 0, kmax_t = 0;
    double best_u = -1.0, best_lo = INFINITY, best_hi = -INFINITY;
    for (int64_t k = 0; k < n; k++) {
        if (!(rho[k] > 0.0) || !(pr[k] > 0.0)) return LBM3D_E_INVAL;
        const double u2 = ux[k] * ux[k] + uy[k] * uy[k] + uz[k] * uz[k];
        const double T = pr[k] / rho[k];
        if (u2 > best_u) { best_u = u2; kmax_u = k; }
        if (T < best_lo) { best_lo = T; kmin_t = k; }
        if (T > best_hi) { best_hi = T; kmax_t = k; }
    }
    std::vector<std::array<double, 5>> states;
    for (int64_t k : {kmax_u, kmin_t, kmax_t})
        states.push_back({rho[k], ux[k], uy[k], uz[k], pr[k] / rho[k]});
    for (int face = 0; face < 6; face++)
        if (p->bc[face] == LBM3D_INFLOW) {
            const double* st = p->inflow[face];
            states.push_back({st[0], st[1], st[2], st[3], st[4] / st[0]});
        }
    double w = 0.0;
    for (const auto& q : states)
        for (int axis = 0; axis < 4; axis++) w = std::fmax(w, scan(p, q.data(), axis, 33, nullptr));
    if (worst) *worst = w;
    return w > 1.0 + STABILITY_TOL ? LBM3D_E_UNSTABLE : LBM3D_OK;
}

}  // namespace lbm3d

using namespace lbm3d;

extern "C" int32_t lbm3d_admit(const lbm3d_params* p, const double* rho, const double* ux, const double* uy,
                               const double* uz, const double* pr, double* max_omega)
{
    if (!p || !rho || !ux || !uy || !uz || !pr) return LBM3D_E_INVAL;
    const int32_t v = validate(p);
    if (v != LBM3D_OK) return v;
    return admission(p, rho, ux, uy, uz, pr, max_omega);
}

extern "C" int32_t lbm3d_stability(const lbm3d_params* p, const double* q, int32_t axis, double kdx_lo,
                                   double kdx_hi, int32_t nk, double alpha_t, double* max_omega,
                                   double* kdx_at_max)
{
    if (!p || !q || !max_omega || nk < 1 || axis < 0 || axis > 3) return LBM3D_E_INVAL;
    const int32_t v = validate(p);
    if (v != LBM3D_OK && v != LBM3D_E_UNSTABLE) return v;  // an unadmitted step may still be analysed
    if (!(q[0] > 0.0) || !(q[4] > 0.0) || !std::isfinite(q[0]) || !std::isfinite(q[4])) return LBM3D_E_INVAL;
    for (int a = 1; a <= 3; a++)
        if (!std::isfinite(q[a])) return LBM3D_E_INVAL;
    if (!std::isfinite(kdx_lo) || !std::isfinite(kdx_hi) || !std::isfinite(alpha_t) || !(std::fabs(alpha_t) < 0.5))
        return LBM3D_E_INVAL;
    const Model<double> m = make_model(p);
    const Velocities s = velocities(m);
    double J[NV][NV];
    eq_jacobian(m, s, q, J);
    const double lam[3] = {m.k_lap0, m.k_lap1, 0.0};  // lambda_i dt / dx^2 per group
    double best = -1.0, best_k = kdx_lo;
    for (int n = 0; n < nk; n++) {
        const double th = nk == 1 ? kdx_lo : kdx_lo + (kdx_hi - kdx_lo) * n / (nk - 1);
        double thv[3] = {0.0, 0.0, 0.0};  // k_a dx per axis
        for (int a = 0; a < 3; a++)
            if (axis == 3 || axis == a) thv[a] = th;
        cd G[NV][NV];
        for (int i = 0; i < NV; i++) {
            const int grp = i == 0 ? 0 : (i <= 6 ? 1 : 2);
            cd diag = 1.0 - m.k_bgk;
            for (int a = 0; a < 3; a++) {
                if (thv[a] == 0.0) continue;
                const cd e = std::polar(1.0, thv[a]);
                const double va = s.v[i][a];
                if (va != 0.0) {
                    // NND, linearised; or the second-order upwind difference
                    // (3 - 4 e^{-ik} + e^{-2ik}) / 2, mirrored for v < 0
                    cd phi;
                    if (p->flags & LBM3D_UPWIND2)
                        phi = va > 0.0 ? 0.5 * (3.0 - 4.0 * std::conj(e) + std::conj(e * e))
                                       : 0.5 * (-3.0 + 4.0 * e - e * e);
                    else
                        phi = va > 0.0 ? (1.0 - alpha_t) * (1.0 - std::conj(e)) : (1.0 - alpha_t) * (e - 1.0);
                    diag -= m.k_adv * va * phi;
                }
                diag += lam[grp] * (2.0 * std::cos(thv[a]) - 2.0);
            }
            for (int j = 0; j < NV; j++) G[i][j] = m.k_bgk * J[i][j];
            G[i][i] += diag;
        }
        const double r = spectral_radius(G);
        if (r > best) {
            best = r;
            best_k = th;
        }
    }
    *max_omega = best;
    if (kdx_at_max) *kdx_at_max = best_k;
    return LBM3D_OK;
}
