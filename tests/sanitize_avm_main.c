/* Host-only driver that runs the oracle's vertex-model entry points
 * (geometry, forces, a run of steps with T1 transitions) on a jittered
 * periodic honeycomb, built with -fsanitize=address,undefined by
 * test_sanitizers.py and linked with both oracle sources.  Inputs come from a
 * local 64-bit LCG (a sanitizer run, not a parity case).  Exit status 0 when
 * every call returned OK, every output is finite, the network stays a valid
 * trivalent tiling and at least one T1 transition ran. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    double KA, KP, mu, v0, Dr, dt;
    uint64_t seed;
    double l_t1, l_new;
} avm_params;

int orc_grid_q(double Lmax);
void orc_quantize(int64_t n, double* v, double L, int q, double* Lq);
double orc_theta0(uint64_t seed, uint64_t tag);
int orc_avm_geometry(int64_t nc, const double* vx, const double* vy, double Lx, double Ly, const int32_t* off,
                     const int32_t* cv, double* A, double* P);
int orc_avm_forces(int64_t nc, int64_t nv, const double* vx, const double* vy, double Lx, double Ly,
                   const int32_t* off, const int32_t* cv, const double* A0, const double* P0, double KA, double KP,
                   double* fx, double* fy);
int orc_avm_run(int64_t nc, int64_t nv, double* vx, double* vy, double* theta, double Lx, double Ly, int q,
                int32_t* off, int32_t* cv, int64_t cap, const double* A0, const double* P0, const avm_params* p,
                uint64_t step0, int64_t nsteps, double* E, double* qbar, int64_t* counters);

static uint64_t lcg = 0x1702029390210ULL;
static double uni(void)
{
    lcg = lcg * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(lcg >> 11) * 0x1.0p-53;
}

static double wrap(double v, double L)
{
    v = fmod(v, L);
    return v < 0 ? v + L : v;
}

static double mimg(double d, double L) { return d - L * round(d / L); }

static int finite_all(const double* v, int64_t n)
{
    for (int64_t i = 0; i < n; i++)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* every vertex in exactly three cells, every cell at least three vertices */
static int valid_network(int64_t nc, int64_t nv, const int32_t* off, const int32_t* cv)
{
    if (off[0] != 0 || off[nc] != 3 * nv) return 0;
    int* cnt = calloc((size_t)nv, sizeof(int));
    int ok = 1;
    for (int64_t c = 0; c < nc && ok; c++) {
        if (off[c + 1] - off[c] < 3) ok = 0;
        for (int32_t m = off[c]; m < off[c + 1] && ok; m++) {
            if (cv[m] < 0 || cv[m] >= nv) ok = 0;
            else cnt[cv[m]]++;
        }
    }
    for (int64_t v = 0; v < nv && ok; v++)
        if (cnt[v] != 3) ok = 0;
    free(cnt);
    return ok;
}

/* honeycomb of nx by ny hexagons (ny even), unit centre spacing, vertices
 * shared by position, each list counter-clockwise; jittered and put on the
 * grid 2^-q of the quantised box */
static int one_network(int nx, int ny, double jitter, int nsteps)
{
    const int64_t nc = (int64_t)nx * ny, nv = 2 * nc, cap = 3 * nv + 512;
    const double h = sqrt(3.0) / 2.0, R = 1.0 / sqrt(3.0), Lx0 = nx, Ly0 = ny * h;
    double* vx = malloc(sizeof(double) * nv);
    double* vy = malloc(sizeof(double) * nv);
    double* th = malloc(sizeof(double) * nc);
    double* A0 = malloc(sizeof(double) * nc);
    double* P0 = malloc(sizeof(double) * nc);
    double* A = malloc(sizeof(double) * nc);
    double* P = malloc(sizeof(double) * nc);
    double* fx = malloc(sizeof(double) * nv);
    double* fy = malloc(sizeof(double) * nv);
    double* E = malloc(sizeof(double) * (nsteps + 1));
    double* Q = malloc(sizeof(double) * (nsteps + 1));
    int32_t* off = malloc(sizeof(int32_t) * (nc + 1));
    int32_t* cv = malloc(sizeof(int32_t) * cap);
    int64_t cnt[2] = {0, 0};
    int rc = 1;
    int64_t used = 0;
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            const int64_t c = (int64_t)j * nx + i;
            const double cx = i + 0.5 * (j & 1), cy = j * h;
            off[c] = (int32_t)(6 * c);
            for (int k = 0; k < 6; k++) {
                const double a = (30.0 + 60.0 * k) * (4.0 * atan(1.0)) / 180.0;
                const double px = wrap(cx + R * cos(a), Lx0), py = wrap(cy + R * sin(a), Ly0);
                int64_t v = 0;
                while (v < used && !(fabs(mimg(vx[v] - px, Lx0)) < 1e-6 && fabs(mimg(vy[v] - py, Ly0)) < 1e-6)) v++;
                if (v == used) {
                    if (used == nv) goto done;
                    vx[used] = px;
                    vy[used] = py;
                    used++;
                }
                cv[6 * c + k] = (int32_t)v;
            }
        }
    off[nc] = (int32_t)(6 * nc);
    if (used != nv || !valid_network(nc, nv, off, cv)) goto done;
    const int q = orc_grid_q(Lx0 > Ly0 ? Lx0 : Ly0);
    double Lx, Ly;
    orc_quantize(0, NULL, Lx0, q, &Lx);
    orc_quantize(0, NULL, Ly0, q, &Ly);
    const double s = ldexp(1.0, q);
    for (int64_t v = 0; v < nv; v++) {
        const double x = wrap(vx[v] * (Lx / Lx0) + jitter * (2 * uni() - 1), Lx);
        const double y = wrap(vy[v] * (Ly / Ly0) + jitter * (2 * uni() - 1), Ly);
        vx[v] = wrap(round(x * s) / s, Lx);
        vy[v] = wrap(round(y * s) / s, Ly);
    }
    for (int64_t c = 0; c < nc; c++) {
        A0[c] = 0.8 + 0.4 * uni();
        P0[c] = 3.6 + 0.3 * uni();
        th[c] = orc_theta0(9, (uint64_t)c);
    }
    if (orc_avm_geometry(nc, vx, vy, Lx, Ly, off, cv, A, P) != 0) goto done;
    double sa = 0;
    for (int64_t c = 0; c < nc; c++) sa += A[c];
    if (!finite_all(P, nc) || fabs(sa - Lx * Ly) > 1e-9 * Lx * Ly) goto done;
    if (orc_avm_forces(nc, nv, vx, vy, Lx, Ly, off, cv, A0, P0, 1.0, 1.0, fx, fy) != 0) goto done;
    if (!finite_all(fx, nv) || !finite_all(fy, nv)) goto done;
    avm_params prm = {1.0, 1.0, 1.0, 0.3, 1.0, 0.01, 13, 0.3, 0.35};
    if (orc_avm_run(nc, nv, vx, vy, th, Lx, Ly, q, off, cv, cap, A0, P0, &prm, 0, nsteps, E, Q, cnt) != 0) goto done;
    if (!finite_all(vx, nv) || !finite_all(vy, nv) || !finite_all(E, nsteps + 1) || !finite_all(Q, nsteps + 1))
        goto done;
    if (cnt[0] <= 0 || !valid_network(nc, nv, off, cv)) goto done;
    if (orc_avm_geometry(nc, vx, vy, Lx, Ly, off, cv, A, P) != 0) goto done;
    sa = 0;
    for (int64_t c = 0; c < nc; c++) sa += A[c];
    if (fabs(sa - Lx * Ly) > 1e-9 * Lx * Ly) goto done;
    /* a cell list with fewer than three vertices is rejected, not read past */
    off[1] = off[0] + 2;
    if (orc_avm_geometry(nc, vx, vy, Lx, Ly, off, cv, A, P) == 0) goto done;
    printf("network %dx%d: %lld T1 in %lld rounds\n", nx, ny, (long long)cnt[0], (long long)cnt[1]);
    rc = 0;
done:
    free(vx); free(vy); free(th); free(A0); free(P0); free(A); free(P); free(fx); free(fy);
    free(E); free(Q); free(off); free(cv);
    return rc;
}

int main(void)
{
    if (one_network(6, 6, 0.15, 60) || one_network(12, 10, 0.15, 40)) {
        fprintf(stderr, "avm oracle call failed\n");
        return 1;
    }
    printf("sanitized avm oracle ok\n");
    return 0;
}
