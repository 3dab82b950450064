/*
 * lbm3d_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of the three-dimensional
 * finite-difference lattice Boltzmann (FD-LB) model of Chen, Xu, Zhang and
 * Li, "Three-Dimensional Lattice Boltzmann Model for High-Speed Compressible
 * Flows" (arXiv:1010.4135).  It exists to check the HIP implementation and is
 * only ever loaded by the test suite, the package smoke check and the CPU
 * baseline leg of the benchmark.  It shares no code, header, table or helper
 * with the GPU library: its parameter struct, velocity table, equilibrium,
 * flux and boundary code are written here, once, from the paper.
 *
 * Every step follows the paper literally, in its own order and notation:
 *   - discrete velocities v_i and eta_i ............ Sec. 2, Eq. (vv)
 *   - moment recovery (rho, u, T) from f ........... Sec. 2, Eqs. (e1)-(e3)
 *     (the paper states them for f^eq; applied to f, the usual LB reading)
 *   - equilibrium f^eq = rho(A + B v.u + D (v.u)^2)  Sec. 2, Eqs. (eq), (e18)
 *   - NND flux with f^+ / f^- splitting, minmod .... Sec. 3, Eq. (nnd) ff.
 *   - artificial dissipation lambda_i Lap f ......... Sec. 3, Eq. (lp)
 *   - explicit forward-Euler time advance ........... Sec. 3, Eq. (fi1)
 *   - (variant) the second-order upwind difference of the original
 *     Kataoka-Tsutahara scheme in place of NND ...... Sec. 3, opening
 *     paragraph; Sec. 4 (1a), Fig. 6
 *   - boundary nodes (fixed state, linear extrapolation, reflection)
 *                                                    Sec. 4 (2), shock-bubble
 * Readings where the paper is silent are listed at each place they are used.
 *
 * Storage: f[15][nz+4][ny+4][nx+4] (two boundary layers per face), x fastest.
 * Velocity order: i=0 rest; i=1..6 = c1(+x,-x,+y,-y,+z,-z); i=7..14 =
 * (c2/sqrt3)(sx,sy,sz), where bit0/1/2 of (i-7) set the sign of x/y/z
 * (bit clear -> +).  (The paper numbers them 1..15; the order inside a group
 * is not fixed by the paper and results do not depend on it.)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NV 15
#define NG 2

enum { ORC_PERIODIC = 0, ORC_OUTFLOW = 1, ORC_INFLOW = 2, ORC_REFLECT = 3 };
enum { ORC_NO_DISSIPATION = 1u, ORC_UPWIND2 = 2u };

typedef struct {
    int32_t nx, ny, nz;
    double c1, c2, eta0;
    double gamma;
    double tau, dt, dx;
    int32_t bc[6];          /* faces -x,+x,-y,+y,-z,+z */
    double inflow[6][5];    /* (rho, ux, uy, uz, p) for fixed-state faces */
    uint32_t flags;
} orc_params;

typedef struct {
    orc_params p;
    double v[NV][3];   /* discrete velocities, Eq. (vv) */
    double eta[NV];    /* eta_i, Eq. (vv) */
    double lam[NV];    /* lambda_i, Eq. (lp) */
    double b;          /* b = 2/(gamma-1), Sec. 2 */
    int64_t mx, my, mz;
    double *f, *fn;
    int64_t steps;
    /* node-steps, since init, whose state at level n had rho <= 0 and
     * T <= 0 (NaN counts in both): a diagnostic, not part of the scheme */
    int64_t nonpos_rho, nonpos_T;
} orc_state;

/* ---------------------------------------------------------------- model -- */

/* Discrete velocity set of Kataoka and Tsutahara, Sec. 2, Eq. (vv). */
static void velocity_set(double c1, double c2, double v[NV][3], double eta[NV], double eta0)
{
    memset(v, 0, sizeof(double) * NV * 3);
    for (int i = 0; i < NV; i++) eta[i] = 0.0;
    eta[0] = eta0;                       /* rest particle carries eta_0 */
    for (int a = 0; a < 3; a++) {        /* c1 (+-1,0,0), c1 (0,+-1,0), c1 (0,0,+-1) */
        v[1 + 2 * a][a] = c1;
        v[2 + 2 * a][a] = -c1;
    }
    double k = c2 / sqrt(3.0);           /* (c2/sqrt3)(+-1,+-1,+-1) */
    for (int d = 0; d < 8; d++)
        for (int a = 0; a < 3; a++)
            v[7 + d][a] = ((d >> a) & 1) ? -k : k;
}

/* f_i^eq = rho (A_i + B_i v_ia u_a + D_i (v_ia u_a)^2), Sec. 2, Eqs. (eq) and
 * (e18), with the gas constant R = 1 (so P = rho T). */
static void equilibrium(const double v[NV][3], double c1, double c2, double eta0, double b,
                        double rho, double ux, double uy, double uz, double T, double feq[NV])
{
    double c1s = c1 * c1, c2s = c2 * c2, e0s = eta0 * eta0;
    double usq = ux * ux + uy * uy + uz * uz;
    for (int i = 0; i < NV; i++) {
        double A, B, D;
        if (i == 0) {
            A = (b - 3.0) / e0s * T;
            B = 0.0;
            D = 0.0;
        } else if (i <= 6) {
            A = 1.0 / (6.0 * (c1s - c2s)) *
                (-c2s + ((b - 3.0) * c2s / e0s + 3.0) * T + c2s / c1s * usq);
            B = (-c2s + (b + 2.0) * T + usq) / (2.0 * c1s * (c1s - c2s));
            D = 1.0 / (2.0 * c1s * c1s);
        } else {
            A = 1.0 / (8.0 * (c2s - c1s)) *
                (-c1s + ((b - 3.0) * c1s / e0s + 3.0) * T + (3.0 * c1s - c2s) / (2.0 * c2s) * usq);
            B = 3.0 * (-c1s + (b + 2.0) * T + usq) / (8.0 * c2s * (c2s - c1s));
            D = 9.0 / (16.0 * c2s * c2s);
        }
        double s = v[i][0] * ux + v[i][1] * uy + v[i][2] * uz;
        feq[i] = rho * (A + B * s + D * s * s);
    }
}

/* Macroscopic variables from f: Eqs. (e1)-(e3) applied to f (the paper gives
 * them as constraints on f^eq; the scheme conserves exactly these sums).
 * q = (rho, ux, uy, uz, T) with rho (b T + u^2) = sum f (v^2 + eta^2). */
static void moments(const double v[NV][3], const double eta[NV], double b,
                    const double f[NV], double q[5])
{
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0}, E = 0.0;
    for (int i = 0; i < NV; i++) {
        rho += f[i];
        for (int a = 0; a < 3; a++) j[a] += f[i] * v[i][a];
        E += f[i] * (v[i][0] * v[i][0] + v[i][1] * v[i][1] + v[i][2] * v[i][2] + eta[i] * eta[i]);
    }
    double ux = j[0] / rho, uy = j[1] / rho, uz = j[2] / rho;
    q[0] = rho;
    q[1] = ux;
    q[2] = uy;
    q[3] = uz;
    q[4] = (E / rho - (ux * ux + uy * uy + uz * uz)) / b;
}

/* minmod(X, Y) = 1/2 min(|X|,|Y|) [Sign X + Sign Y], Sec. 3. */
static double sgn(double x) { return (x > 0.0) ? 1.0 : ((x < 0.0) ? -1.0 : 0.0); }
static double minmod(double X, double Y)
{
    return 0.5 * fmin(fabs(X), fabs(Y)) * (sgn(X) + sgn(Y));
}

/* --------------------------------------------------------------- layout -- */

static inline int64_t idx(const orc_state* s, int i, int64_t x, int64_t y, int64_t z)
{
    return (((int64_t)i * s->mz + (z + NG)) * s->my + (y + NG)) * s->mx + (x + NG);
}

static void site_f(const orc_state* s, const double* f, int64_t x, int64_t y, int64_t z, double out[NV])
{
    for (int i = 0; i < NV; i++) out[i] = f[idx(s, i, x, y, z)];
}

static void set_site_feq(orc_state* s, double* f, int64_t x, int64_t y, int64_t z, const double q[5])
{
    double feq[NV];
    equilibrium((const double(*)[3])s->v, s->p.c1, s->p.c2, s->p.eta0, s->b,
                q[0], q[1], q[2], q[3], q[4], feq);
    for (int i = 0; i < NV; i++) f[idx(s, i, x, y, z)] = feq[i];
}

/* ------------------------------------------------------- boundary nodes -- */

/* Boundary layers for one face.  Sec. 4 (2) gives the rules for the
 * macroscopic variables (rho, u, T) on the two boundary-node layers:
 *   fixed state (the right side of the shock-bubble run): both layers take
 *     the prescribed state;
 *   extrapolation (the left side): q(1) = 2 q(2) - q(3), q(0) = 2 q(1) - q(2)
 *     in the paper's numbering, i.e. layers -1 and -2 here from interior
 *     nodes 0 and 1;
 *   reflection (the other four faces): the first layer is the wall node, a
 *     copy of the last interior node with zero normal velocity; the second
 *     layer mirrors the last interior node with the normal velocity negated.
 * Reading: the paper gives only macroscopic values for the boundary nodes;
 * their distributions are taken as f^eq of those values.  Periodic faces
 * (not used in the paper; needed for the conservation checks) copy f from
 * the opposite side.  Only face layers are filled: the stencils are
 * axis-aligned, so edge and corner layers are never read. */
static void fill_face(orc_state* s, double* f, int axis, int side)
{
    const int64_t n[3] = {s->p.nx, s->p.ny, s->p.nz};
    int face = 2 * axis + side;
    int bc = s->p.bc[face];
    int t1 = (axis + 1) % 3, t2 = (axis + 2) % 3;
    for (int64_t b2 = 0; b2 < n[t2]; b2++) {
        for (int64_t b1 = 0; b1 < n[t1]; b1++) {
            for (int layer = 1; layer <= NG; layer++) {
                /* ghost coordinate along the axis, and interior nodes i0 (the
                 * one adjacent to the face) and i1 (the next one in) */
                int64_t g = side ? (n[axis] - 1 + layer) : (-layer);
                int64_t i0 = side ? (n[axis] - 1) : 0;
                int64_t i1 = side ? (n[axis] - 2) : 1;
                int64_t c[3], c0[3], c1x[3];
                c[t1] = c0[t1] = c1x[t1] = b1;
                c[t2] = c0[t2] = c1x[t2] = b2;
                c[axis] = g;
                c0[axis] = i0;
                c1x[axis] = i1;
                if (bc == ORC_PERIODIC) {
                    int64_t w = ((g % n[axis]) + n[axis]) % n[axis];
                    int64_t cw[3] = {c[0], c[1], c[2]};
                    cw[axis] = w;
                    for (int i = 0; i < NV; i++)
                        f[idx(s, i, c[0], c[1], c[2])] = f[idx(s, i, cw[0], cw[1], cw[2])];
                    continue;
                }
                double q[5];
                if (bc == ORC_INFLOW) {
                    const double* st = s->p.inflow[face];
                    q[0] = st[0];
                    q[1] = st[1];
                    q[2] = st[2];
                    q[3] = st[3];
                    q[4] = st[4] / st[0];  /* T = p / rho (R = 1) */
                } else if (bc == ORC_OUTFLOW) {
                    double fa[NV], fb[NV], qa[5], qb[5];
                    site_f(s, f, c0[0], c0[1], c0[2], fa);
                    site_f(s, f, c1x[0], c1x[1], c1x[2], fb);
                    moments((const double(*)[3])s->v, s->eta, s->b, fa, qa);
                    moments((const double(*)[3])s->v, s->eta, s->b, fb, qb);
                    /* layer 1: 2 q(i0) - q(i1); layer 2: 2 q(layer1) - q(i0) */
                    double q1[5];
                    for (int k = 0; k < 5; k++) q1[k] = 2.0 * qa[k] - qb[k];
                    if (layer == 1) {
                        for (int k = 0; k < 5; k++) q[k] = q1[k];
                    } else {
                        for (int k = 0; k < 5; k++) q[k] = 2.0 * q1[k] - qa[k];
                    }
                } else { /* ORC_REFLECT */
                    double fa[NV];
                    site_f(s, f, c0[0], c0[1], c0[2], fa);
                    moments((const double(*)[3])s->v, s->eta, s->b, fa, q);
                    if (layer == 1)
                        q[1 + axis] = 0.0;          /* wall node */
                    else
                        q[1 + axis] = -q[1 + axis]; /* mirror node */
                }
                set_site_feq(s, f, c[0], c[1], c[2], q);
            }
        }
    }
}

static void fill_boundaries(orc_state* s, double* f)
{
    for (int axis = 0; axis < 3; axis++)
        for (int side = 0; side < 2; side++) fill_face(s, f, axis, side);
}

/* ------------------------------------------------------------ the step -- */

/* One explicit time step of Eq. (lp) with the NND convection term:
 *   f_i^{n+1} = f_i^n + dt [ - sum_a (h_{I+1/2} - h_{I-1/2}) / dx
 *                            - (f_i^n - f_i^eq) / tau
 *                            + lambda_i sum_a (f_{I+1} - 2 f_I + f_{I-1}) / dx^2 ]
 * Forward difference in time as in Eq. (fi1) (reading: every term at level
 * n).  The NND flux is evaluated literally with the f^+ / f^- split along
 * each of x, y and z (the paper writes "x or y"; the model is 3D and the sum
 * over alpha runs over all three axes). */
static void step_once(orc_state* s)
{
    const orc_params* p = &s->p;
    const double dx = p->dx, dt = p->dt, tau = p->tau;
    const int64_t stride[3] = {1, s->mx, s->mx * s->my};
    const double* f = s->f;
    double* fn = s->fn;
    int64_t bad_rho = 0, bad_T = 0;
#pragma omp parallel for collapse(3) schedule(static) reduction(+ : bad_rho, bad_T)
    for (int64_t z = 0; z < p->nz; z++) {
        for (int64_t y = 0; y < p->ny; y++) {
            for (int64_t x = 0; x < p->nx; x++) {
                double fs[NV], q[5], feq[NV];
                site_f(s, f, x, y, z, fs);
                moments((const double(*)[3])s->v, s->eta, s->b, fs, q);
                if (!(q[0] > 0.0)) bad_rho++;
                if (!(q[4] > 0.0)) bad_T++;
                equilibrium((const double(*)[3])s->v, p->c1, p->c2, p->eta0, s->b,
                            q[0], q[1], q[2], q[3], q[4], feq);
                for (int i = 0; i < NV; i++) {
                    const int64_t I = idx(s, i, x, y, z);
                    const double fI = f[I];
                    double conv = 0.0;
                    double lap = 0.0;
                    for (int a = 0; a < 3; a++) {
                        const double va = s->v[i][a];
                        const double wp = 0.5 * (va + fabs(va)); /* f^+ = wp f */
                        const double wm = 0.5 * (va - fabs(va)); /* f^- = wm f */
                        double fp[5], fm[5];  /* nodes I-2 .. I+2 along axis a */
                        for (int k = -2; k <= 2; k++) {
                            double val = f[I + k * stride[a]];
                            fp[k + 2] = wp * val;
                            fm[k + 2] = wm * val;
                        }
                        /* h_{I+1/2} = f^L_{I+1/2} + f^R_{I+1/2} */
                        double fL_p = fp[2] + 0.5 * minmod(fp[3] - fp[2], fp[2] - fp[1]);
                        double fR_p = fm[3] - 0.5 * minmod(fm[3] - fm[2], fm[4] - fm[3]);
                        /* h_{I-1/2} = f^L_{I-1/2} + f^R_{I-1/2} */
                        double fL_m = fp[1] + 0.5 * minmod(fp[2] - fp[1], fp[1] - fp[0]);
                        double fR_m = fm[2] - 0.5 * minmod(fm[2] - fm[1], fm[3] - fm[2]);
                        double h_p = fL_p + fR_p;
                        double h_m = fL_m + fR_m;
                        if (p->flags & ORC_UPWIND2) {
                            /* second-order upwind difference of the original
                             * scheme: v (3 f_I - 4 f_{I-1} + f_{I-2}) / (2 dx)
                             * for v > 0, v (-3 f_I + 4 f_{I+1} - f_{I+2}) /
                             * (2 dx) for v < 0 */
                            double fI2[5];
                            for (int k = -2; k <= 2; k++) fI2[k + 2] = f[I + k * stride[a]];
                            if (va > 0.0)
                                conv += va * (3.0 * fI2[2] - 4.0 * fI2[1] + fI2[0]) / (2.0 * dx);
                            else if (va < 0.0)
                                conv += va * (-3.0 * fI2[2] + 4.0 * fI2[3] - fI2[4]) / (2.0 * dx);
                        } else {
                            conv += (h_p - h_m) / dx;
                        }
                        lap += (f[I + stride[a]] - 2.0 * fI + f[I - stride[a]]) / (dx * dx);
                    }
                    double lam = (p->flags & ORC_NO_DISSIPATION) ? 0.0 : s->lam[i];
                    fn[I] = fI + dt * (-conv - (fI - feq[i]) / tau + lam * lap);
                }
            }
        }
    }
    double* t = s->f;
    s->f = s->fn;
    s->fn = t;
    fill_boundaries(s, s->f);
    s->steps++;
    s->nonpos_rho += bad_rho;
    s->nonpos_T += bad_T;
}

/* ------------------------------------------------------------- exports -- */

orc_state* orc_create(const orc_params* p)
{
    if (!p || p->nx < 1 || p->ny < 1 || p->nz < 1) return NULL;
    orc_state* s = (orc_state*)calloc(1, sizeof(orc_state));
    if (!s) return NULL;
    s->p = *p;
    s->b = 2.0 / (p->gamma - 1.0);
    velocity_set(p->c1, p->c2, s->v, s->eta, p->eta0);
    /* lambda_i of Eq. (lp): c1 dx for the rest particle, c1 dx / 10 for the
     * six axis velocities, 0 for the eight diagonal ones */
    s->lam[0] = p->c1 * p->dx;
    for (int i = 1; i <= 6; i++) s->lam[i] = p->c1 * p->dx / 10.0;
    for (int i = 7; i < NV; i++) s->lam[i] = 0.0;
    s->mx = p->nx + 2 * NG;
    s->my = p->ny + 2 * NG;
    s->mz = p->nz + 2 * NG;
    size_t n = (size_t)NV * s->mx * s->my * s->mz;
    s->f = (double*)calloc(n, sizeof(double));
    s->fn = (double*)calloc(n, sizeof(double));
    if (!s->f || !s->fn) {
        free(s->f);
        free(s->fn);
        free(s);
        return NULL;
    }
    return s;
}

void orc_destroy(orc_state* s)
{
    if (!s) return;
    free(s->f);
    free(s->fn);
    free(s);
}

/* Initial distributions: f_i = f_i^eq(rho, u, T = p / rho) on every interior
 * node (reading: the paper states initial macroscopic fields only). */
void orc_init(orc_state* s, const double* rho, const double* ux, const double* uy,
              const double* uz, const double* pr)
{
    const orc_params* p = &s->p;
    for (int64_t z = 0; z < p->nz; z++)
        for (int64_t y = 0; y < p->ny; y++)
            for (int64_t x = 0; x < p->nx; x++) {
                int64_t k = (z * p->ny + y) * p->nx + x;
                double q[5] = {rho[k], ux[k], uy[k], uz[k], pr[k] / rho[k]};
                set_site_feq(s, s->f, x, y, z, q);
            }
    fill_boundaries(s, s->f);
    s->steps = 0;
    s->nonpos_rho = 0;
    s->nonpos_T = 0;
}

void orc_step(orc_state* s, int64_t nsteps)
{
    for (int64_t n = 0; n < nsteps; n++) step_once(s);
}

/* (rho, u, p = rho T) on every interior node. */
void orc_moments(const orc_state* s, double* rho, double* ux, double* uy, double* uz, double* pr)
{
    const orc_params* p = &s->p;
    for (int64_t z = 0; z < p->nz; z++)
        for (int64_t y = 0; y < p->ny; y++)
            for (int64_t x = 0; x < p->nx; x++) {
                double fs[NV], q[5];
                site_f(s, s->f, x, y, z, fs);
                moments((const double(*)[3])s->v, s->eta, s->b, fs, q);
                int64_t k = (z * p->ny + y) * p->nx + x;
                rho[k] = q[0];
                ux[k] = q[1];
                uy[k] = q[2];
                uz[k] = q[3];
                pr[k] = q[0] * q[4];
            }
}

/* Domain totals over interior nodes: mass, momentum (x, y, z) and total
 * energy, the last being 1/2 sum_i f_i (v_i^2 + eta_i^2) = rho (b T + u^2)/2
 * per node (the conserved density of the energy equation, Eq. (e2)). */
void orc_conserved(const orc_state* s, double out[5])
{
    const orc_params* p = &s->p;
    for (int k = 0; k < 5; k++) out[k] = 0.0;
    for (int64_t z = 0; z < p->nz; z++)
        for (int64_t y = 0; y < p->ny; y++)
            for (int64_t x = 0; x < p->nx; x++)
                for (int i = 0; i < NV; i++) {
                    double fi = s->f[idx(s, i, x, y, z)];
                    const double* v = s->v[i];
                    out[0] += fi;
                    out[1] += fi * v[0];
                    out[2] += fi * v[1];
                    out[3] += fi * v[2];
                    out[4] += 0.5 * fi * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2] + s->eta[i] * s->eta[i]);
                }
}

/* Interior distributions as [15][nz][ny][nx], x fastest. */
void orc_get_f(const orc_state* s, double* out)
{
    const orc_params* p = &s->p;
    for (int i = 0; i < NV; i++)
        for (int64_t z = 0; z < p->nz; z++)
            for (int64_t y = 0; y < p->ny; y++)
                for (int64_t x = 0; x < p->nx; x++)
                    out[(((int64_t)i * p->nz + z) * p->ny + y) * p->nx + x] = s->f[idx(s, i, x, y, z)];
}

void orc_set_f(orc_state* s, const double* in)
{
    const orc_params* p = &s->p;
    for (int i = 0; i < NV; i++)
        for (int64_t z = 0; z < p->nz; z++)
            for (int64_t y = 0; y < p->ny; y++)
                for (int64_t x = 0; x < p->nx; x++)
                    s->f[idx(s, i, x, y, z)] = in[(((int64_t)i * p->nz + z) * p->ny + y) * p->nx + x];
    fill_boundaries(s, s->f);
}

/* Distributions including the boundary layers: [15][nz+4][ny+4][nx+4]. */
void orc_get_f_padded(const orc_state* s, double* out)
{
    memcpy(out, s->f, sizeof(double) * (size_t)NV * s->mx * s->my * s->mz);
}

int64_t orc_steps_done(const orc_state* s) { return s->steps; }

/* Node-steps since init that started from a state with rho <= 0 (out[0])
 * and with T <= 0 (out[1]), counted on the interior nodes at the moments
 * each step recovers from f^n. */
void orc_nonphysical(const orc_state* s, int64_t out[2])
{
    out[0] = s->nonpos_rho;
    out[1] = s->nonpos_T;
}

/* Stand-alone model functions, exposed for the checks. */
void orc_velocities(double c1, double c2, double eta0, double v[NV][3], double eta[NV])
{
    velocity_set(c1, c2, v, eta, eta0);
}

void orc_equilibrium(double c1, double c2, double eta0, double gamma, double rho, double ux,
                     double uy, double uz, double T, double feq[NV])
{
    double v[NV][3], eta[NV];
    velocity_set(c1, c2, v, eta, eta0);
    equilibrium((const double(*)[3])v, c1, c2, eta0, 2.0 / (gamma - 1.0), rho, ux, uy, uz, T, feq);
}

void orc_moments_of(double c1, double c2, double eta0, double gamma, const double f[NV], double q[5])
{
    double v[NV][3], eta[NV];
    velocity_set(c1, c2, v, eta, eta0);
    moments((const double(*)[3])v, eta, 2.0 / (gamma - 1.0), f, q);
}

double orc_minmod(double X, double Y) { return minmod(X, Y); }

int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
