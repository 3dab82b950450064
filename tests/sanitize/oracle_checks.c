/* The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer:
 * steps of small solves with every boundary kind and flag combination. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t nx, ny, nz;
    double c1, c2, eta0;
    double gamma;
    double tau, dt, dx;
    int32_t bc[6];
    double inflow[6][5];
    uint32_t flags;
} orc_params;
typedef struct orc_state orc_state;
orc_state* orc_create(const orc_params* p);
void orc_destroy(orc_state* s);
void orc_init(orc_state* s, const double* rho, const double* ux, const double* uy, const double* uz, const double* pr);
void orc_step(orc_state* s, int64_t nsteps);
void orc_moments(const orc_state* s, double* rho, double* ux, double* uy, double* uz, double* pr);
void orc_conserved(const orc_state* s, double out[5]);

int main(void)
{
    const int bcs[4][6] = {{0, 0, 0, 0, 0, 0}, {1, 1, 3, 3, 0, 0}, {2, 1, 3, 3, 3, 3}, {3, 3, 1, 1, 3, 1}};
    int bad = 0;
    for (int b = 0; b < 4; b++)
        for (uint32_t flags = 0; flags < 4; flags++) {
            orc_params p;
            memset(&p, 0, sizeof p);
            p.nx = 7 + b;
            p.ny = 5;
            p.nz = 4;
            p.c1 = 8;
            p.c2 = 24;
            p.eta0 = 8;
            p.gamma = 1.4;
            p.tau = 1e-5;
            p.dt = 1e-5;
            p.dx = 1.0 / 256;
            memcpy(p.bc, bcs[b], sizeof p.bc);
            for (int c = 0; c < 5; c++) p.inflow[0][c] = c == 0 || c == 4 ? 1.2 : 0.1;
            p.flags = flags;
            const int n = p.nx * p.ny * p.nz;
            double* f = calloc((size_t)5 * n, sizeof(double));
            for (int k = 0; k < n; k++) {
                f[k] = 1.0 + 0.1 * sin(k);
                f[n + k] = 0.2 * cos(k);
                f[4 * n + k] = 1.0 + 0.05 * k / n;
            }
            orc_state* s = orc_create(&p);
            orc_init(s, f, f + n, f + 2 * n, f + 3 * n, f + 4 * n);
            orc_step(s, 5);
            orc_moments(s, f, f + n, f + 2 * n, f + 3 * n, f + 4 * n);
            for (int k = 0; k < 5 * n; k++)
                if (!isfinite(f[k])) bad++;
            double tot[5];
            orc_conserved(s, tot);
            orc_destroy(s);
            free(f);
        }
    if (bad) {
        fprintf(stderr, "%d non-finite values\n", bad);
        return 1;
    }
    printf("oracle checks passed\n");
    return 0;
}
