/* Host-only driver that runs the oracle's entry points (triangulation,
 * geometry, forces, observables, noise, whole steps) on small seeded inputs,
 * built with -fsanitize=address,undefined by test_sanitizers.py.  Inputs
 * come from a local 64-bit LCG (a sanitizer run, not a parity case).
 * Exit status 0 when every call returned OK and every output is finite. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "../oracle/spv_oracle.c"

static uint64_t lcg = 0x2017020912345ULL;
static double uni(void)
{
    lcg = lcg * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(lcg >> 11) * 0x1.0p-53;
}

static int finite_all(const double* v, int64_t n)
{
    for (int64_t i = 0; i < n; i++)
        if (!isfinite(v[i])) return 0;
    return 1;
}

static int one_system(int64_t n, double L, int nsteps)
{
    double* x = malloc(sizeof(double) * n);
    double* y = malloc(sizeof(double) * n);
    double* th = malloc(sizeof(double) * n);
    double* A0 = malloc(sizeof(double) * n);
    double* P0 = malloc(sizeof(double) * n);
    double* A = malloc(sizeof(double) * n);
    double* P = malloc(sizeof(double) * n);
    double* fx = malloc(sizeof(double) * n);
    double* fy = malloc(sizeof(double) * n);
    int32_t* off = malloc(sizeof(int32_t) * (n + 1));
    int64_t cap = 32 * n + 64;
    int32_t* ring = malloc(sizeof(int32_t) * cap);
    double* E = malloc(sizeof(double) * (nsteps + 1));
    double* Q = malloc(sizeof(double) * (nsteps + 1));
    int rc = 1;
    for (int64_t i = 0; i < n; i++) {
        x[i] = uni() * L;
        y[i] = uni() * L;
        A0[i] = 1.0;
        P0[i] = 3.8;
    }
    int q = orc_grid_q(L);
    double Lx, Ly;
    orc_quantize(n, x, L, q, &Lx);
    orc_quantize(n, y, L, q, &Ly);
    for (int64_t i = 0; i < n; i++) th[i] = orc_theta0(7, (uint64_t)i);
    int64_t ntri = 0;
    double mcr = 0.0;
    if (orc_triangulate(n, x, y, Lx, Ly, q, off, ring, cap, &ntri, &mcr) != ORC_OK) goto done;
    if (ntri != 2 * n || off[n] != 6 * n) goto done;
    if (orc_geometry(n, x, y, Lx, Ly, off, ring, A, P) != ORC_OK) goto done;
    if (orc_forces(n, x, y, Lx, Ly, off, ring, A0, P0, 1.0, 1.0, fx, fy) != ORC_OK) goto done;
    double e, qb, sa;
    orc_observables(n, A, P, A0, P0, 1.0, 1.0, &e, &qb, &sa);
    if (!isfinite(e) || !isfinite(qb) || fabs(sa - Lx * Ly) > 1e-9 * Lx * Ly) goto done;
    orc_params prm = {1.0, 1.0, 1.0, 0.1, 1.0, 0.01, 11};
    if (orc_run(n, x, y, th, Lx, Ly, q, A0, P0, &prm, 0, nsteps, E, Q, fx, fy, off, ring, cap) != ORC_OK) goto done;
    if (!finite_all(x, n) || !finite_all(y, n) || !finite_all(fx, n) || !finite_all(E, nsteps + 1)) goto done;
    rc = 0;
done:
    free(x); free(y); free(th); free(A0); free(P0); free(A); free(P); free(fx); free(fy);
    free(off); free(ring); free(E); free(Q);
    return rc;
}

int main(void)
{
    int64_t a[3] = {0, 0, 0}, b[3] = {5, 0, 0}, c[3] = {0, 5, 0}, d[3] = {5, 5, 0}, r[5] = {0, 1, 2, 3, 0};
    (void)orc_incircle_sos(a, b, c, d, r);
    uint64_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    orc_philox4x64(ctr, key, out);
    if (one_system(64, 8.0, 5) || one_system(500, sqrt(500.0), 3) || one_system(3000, sqrt(3000.0), 2)) {
        fprintf(stderr, "oracle call failed\n");
        return 1;
    }
    printf("sanitized oracle ok\n");
    return 0;
}
