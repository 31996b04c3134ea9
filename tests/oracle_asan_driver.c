/*
 * Drives every entry point of the C oracle (oracle/wave2d_oracle.c) on small
 * grids, for building with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitized.py).  Grids are allocated to their exact
 * size, so any read or write outside them is reported.  Exit code 0 and
 * no sanitizer report means every access stayed in bounds.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int orc_brackets(int scheme, double lam, double a[3], double b[3], int* has_b);
double orc_lambda_max(int scheme);
int orc_set_scheme(int id, int nclass, int deg, const double* a, const double* b);
int orc_class_brackets(int scheme, double lam, double a[9], double b[9], int* has_b);
int orc_first_step(int nx, int ny, double h, double tau, double c, int scheme, unsigned flags, const double* u0,
                   const double* v0, double* u1);
int orc_step(int nx, int ny, double h, double tau, double c, int scheme, unsigned flags, const double* um1,
             const double* u, double* up1);
int orc_steps(int nx, int ny, double h, double tau, double c, int scheme, unsigned flags, long steps, double* um1,
              double* u);
int orc_run(int nx, int ny, double h, double tau, double c, int scheme, unsigned flags, long steps, const double* u0,
            const double* v0, double* u_prev_out, double* u_out);
void orc_norms(long n, const double* a, const double* b, double out[4]);

static double* grid(int nx, int ny, unsigned seed)
{
    double* p = (double*)malloc((size_t)nx * ny * sizeof(double));
    for (int k = 0; k < nx * ny; ++k) {
        seed = seed * 1103515245u + 12345u;
        p[k] = (double)(seed >> 8) / 16777216.0 - 0.5;
    }
    return p;
}

int main(void)
{
    /* a registered scheme: the cross set's weights (A and B / tau per class) */
    double a[3 * 13] = {0}, b[3 * 13] = {0};
    a[0 * 13 + 2] = 2.0 / 3.0; a[0 * 13 + 4] = -1.0 / 6.0;
    a[2 * 13 + 2] = -1.0 / 24.0; a[2 * 13 + 4] = 1.0 / 24.0;
    b[0 * 13 + 2] = 2.0 / 9.0; b[0 * 13 + 4] = -1.0 / 30.0;
    b[2 * 13 + 2] = -1.0 / 72.0; b[2 * 13 + 4] = 1.0 / 120.0;
    if (orc_set_scheme(1000, 3, 12, a, b)) return 10;
    /* a radius-3 scheme: the complete degree-6 set's weights, classes
     * (1,0), (1,1), (2,0), (2,1), (3,0) (nodes up to three lines out) */
    double a6[9 * 13] = {0}, b6[9 * 13] = {0};
    a6[0 * 13 + 2] = 3.0 / 4; a6[0 * 13 + 4] = -77.0 / 144; a6[0 * 13 + 6] = 19.0 / 240;
    a6[1 * 13 + 4] = 5.0 / 36; a6[1 * 13 + 6] = -1.0 / 30;
    a6[2 * 13 + 2] = -3.0 / 40; a6[2 * 13 + 4] = 7.0 / 72; a6[2 * 13 + 6] = -1.0 / 60;
    a6[3 * 13 + 4] = -1.0 / 144; a6[3 * 13 + 6] = 1.0 / 240;
    a6[5 * 13 + 2] = 1.0 / 180; a6[5 * 13 + 4] = -1.0 / 144; a6[5 * 13 + 6] = 1.0 / 720;
    b6[0 * 13 + 2] = 1.0 / 4; b6[0 * 13 + 4] = -77.0 / 720; b6[0 * 13 + 6] = 19.0 / 1680;
    b6[1 * 13 + 4] = 1.0 / 36; b6[1 * 13 + 6] = -1.0 / 210;
    b6[2 * 13 + 2] = -1.0 / 40; b6[2 * 13 + 4] = 7.0 / 360; b6[2 * 13 + 6] = -1.0 / 420;
    b6[3 * 13 + 4] = -1.0 / 720; b6[3 * 13 + 6] = 1.0 / 1680;
    b6[5 * 13 + 2] = 1.0 / 540; b6[5 * 13 + 4] = -1.0 / 720; b6[5 * 13 + 6] = 1.0 / 5040;
    if (orc_set_scheme(1001, 9, 12, a6, b6)) return 10;
    const int schemes[] = {5, 9, 13, 109, 1000, 1001};
    const int shapes[][2] = {{3, 3}, {5, 5}, {4, 7}, {19, 5}, {6, 40}, {7, 7}, {8, 3}};
    const unsigned flagsets[] = {0u, 1u, 4u, 5u};
    int runs = 0;
    for (int si = 0; si < 6; ++si) {
        double ba[3], bb[3], ca[9], cb[9];
        int hb;
        if ((orc_brackets(schemes[si], 0.5, ba, bb, &hb) == 0) != (schemes[si] != 1001)) return 11;
        if (orc_class_brackets(schemes[si], 0.5, ca, cb, &hb)) return 11;
        (void)orc_lambda_max(schemes[si]);
        for (int sh = 0; sh < 7; ++sh)
            for (int fi = 0; fi < 4; ++fi) {
                const int nx = shapes[sh][0], ny = shapes[sh][1];
                const unsigned f = flagsets[fi];
                const int r = schemes[si] == 1001 ? 3 : (schemes[si] == 13 || schemes[si] == 1000) ? 2 : 1;
                const int ok = !((f & 4u) && (nx < 2 * r + 1 || ny < 2 * r + 1));
                double* u0 = grid(nx, ny, 1u + (unsigned)sh);
                double* v0 = grid(nx, ny, 7u + (unsigned)fi);
                double* up = grid(nx, ny, 3u);
                double* uc = grid(nx, ny, 5u);
                double* w = grid(nx, ny, 9u);
                const double h = 1.0 / (nx > ny ? nx : ny), tau = 0.3 * h;
                int rc = orc_run(nx, ny, h, tau, 1.0, schemes[si], f, 6, u0, v0, up, uc);
                if ((rc == 0) != ok) return 12;
                if (ok) {
                    if (orc_first_step(nx, ny, h, tau, 1.0, schemes[si], f, u0, v0, w)) return 13;
                    if (orc_step(nx, ny, h, tau, 1.0, schemes[si], f, up, uc, w)) return 14;
                    if (orc_steps(nx, ny, h, tau, 1.0, schemes[si], f, 3, up, uc)) return 15;
                    double nr[4];
                    orc_norms((long)nx * ny, uc, w, nr);
                    if (!(nr[1] >= 0.0)) return 16;
                    ++runs;
                }
                free(u0); free(v0); free(up); free(uc); free(w);
            }
    }
    printf("oracle entry points exercised: %d runs\n", runs);
    return 0;
}
