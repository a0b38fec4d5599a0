/*
 * avm_oracle.c -- plain CPU oracle of the active vertex model (AVM).
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test-suite and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP library.
 *
 * What it computes (Sussman, "cellGPU", arXiv:1702.02939):
 *   - the degrees of freedom are the vertices h_v of a trivalent polygonal
 *     tiling of the flat torus; cell c is the polygon of its vertex list,
 *     counter-clockwise (Sec. II.A, Fig. 1);
 *   - the energy of Eq. (1) over the cells' areas and perimeters, and the
 *     vertex forces F_v = -dE/dh_v (App. A) by forward-mode dual numbers on
 *     each cell's energy (topology held fixed);
 *   - the equation of motion Eq. (4): dh_v/dt = mu F_v + (v0 / n) sum of the
 *     directors of the n = 3 cells at v, Euler-Maruyama, the cell directors
 *     rotating with the white noise of Sec. II.A;
 *   - T1 transitions (Sec. II.D, Fig. 1 right): an edge shorter than a
 *     threshold is turned into the perpendicular edge through its midpoint
 *     and the two cells at its ends become neighbours; at most one transition
 *     per cell in a round, rounds repeated until no edge qualifies.
 *
 * Readings where the paper is silent:
 *   - vertices live on the dyadic grid 2^-q like the cell positions of the
 *     Voronoi model, re-quantised after every move, so that edge lengths are
 *     differences of exact doubles; the T1 test is dx*dx + dy*dy < l_T1^2
 *     evaluated in double without fused operations;
 *   - the new edge of a T1 has length l_new, the vertex that stays with the
 *     cell on the left of the old edge (the cell keeping it) on that side;
 *   - an edge qualifies only if both cells sharing it have more than three
 *     vertices and the two cells at its ends share no vertex yet; in a round
 *     an edge flips when its key (smaller vertex tag, larger vertex tag) is
 *     the smallest key among qualifying edges touching any of its four cells;
 *   - noise and update order as the Voronoi model: Philox4x64-10, counter
 *     (step, cell tag); vertices move with the directors of the step start,
 *     then the directors rotate.
 *
 * Build: compiled into liboracle.so with spv_oracle.c (gcc -ffp-contract=off).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define AVM_OK 0
#define AVM_EINVAL -1
#define AVM_ENOMEM -2
#define AVM_ECAP -5
#define AVM_EFAIL -8

double orc_normal(uint64_t seed, uint64_t step, uint64_t tag); /* spv_oracle.c (the oracle's own Philox) */

typedef struct {
    double KA, KP, mu, v0, Dr, dt;
    uint64_t seed;
    double l_t1, l_new;
} avm_params;

static double mimg(double d, double L)
{
    if (d > 0.5 * L) return d - L;
    if (d < -0.5 * L) return d + L;
    return d;
}

static double wrap_q(double v, double L, int q)
{
    const double s = ldexp(1.0, q);
    double X = nearbyint(v * s);
    const double LX = nearbyint(L * s);
    X = fmod(X, LX);
    if (X < 0) X += LX;
    if (X >= LX) X -= LX;
    return X / s;
}

/* ------------------------------------------------------------------ */
/* geometry and energy                                                 */
/* ------------------------------------------------------------------ */
typedef struct { double v, gx, gy; } dn;
static dn dn_c(double v) { dn r = {v, 0, 0}; return r; }
static dn dn_add(dn a, dn b) { dn r = {a.v + b.v, a.gx + b.gx, a.gy + b.gy}; return r; }
static dn dn_sub(dn a, dn b) { dn r = {a.v - b.v, a.gx - b.gx, a.gy - b.gy}; return r; }
static dn dn_mul(dn a, dn b) { dn r = {a.v * b.v, a.gx * b.v + a.v * b.gx, a.gy * b.v + a.v * b.gy}; return r; }
static dn dn_scale(dn a, double s) { dn r = {a.v * s, a.gx * s, a.gy * s}; return r; }
static dn dn_sqrt(dn a)
{
    const double s = sqrt(a.v);
    dn r = {s, 0, 0};
    if (s > 0) {
        r.gx = a.gx / (2 * s);
        r.gy = a.gy / (2 * s);
    }
    return r;
}

/* energy of a polygon with vertex displacements (px, py) from its first
 * vertex: K_A (A - A0)^2 + K_P (P - P0)^2, A by the shoelace formula */
static dn poly_energy(int k, const dn* px, const dn* py, double A0, double P0, double KA, double KP, double* Aout,
                      double* Pout)
{
    dn a2 = dn_c(0), per = dn_c(0);
    for (int m = 0; m < k; m++) {
        const int n = (m + 1) % k;
        a2 = dn_add(a2, dn_sub(dn_mul(px[m], py[n]), dn_mul(py[m], px[n])));
        const dn ex = dn_sub(px[n], px[m]), ey = dn_sub(py[n], py[m]);
        per = dn_add(per, dn_sqrt(dn_add(dn_mul(ex, ex), dn_mul(ey, ey))));
    }
    const dn A = dn_scale(a2, 0.5);
    if (Aout) *Aout = A.v;
    if (Pout) *Pout = per.v;
    const dn da = dn_sub(A, dn_c(A0)), dp = dn_sub(per, dn_c(P0));
    return dn_add(dn_scale(dn_mul(da, da), KA), dn_scale(dn_mul(dp, dp), KP));
}

/* displacements of cell c's vertices from its first vertex (minimum image
 * of each edge, accumulated around the polygon) */
static void cell_disp(const int32_t* off, const int32_t* cv, int c, const double* vx, const double* vy, double Lx,
                      double Ly, double* dx, double* dy)
{
    const int k = off[c + 1] - off[c];
    const int32_t* v = cv + off[c];
    dx[0] = dy[0] = 0;
    for (int m = 1; m < k; m++) {
        dx[m] = dx[m - 1] + mimg(vx[v[m]] - vx[v[m - 1]], Lx);
        dy[m] = dy[m - 1] + mimg(vy[v[m]] - vy[v[m - 1]], Ly);
    }
}

#define KV_MAX 64

int orc_avm_geometry(int64_t nc, const double* vx, const double* vy, double Lx, double Ly, const int32_t* off,
                     const int32_t* cv, double* A, double* P)
{
    double dx[KV_MAX], dy[KV_MAX];
    dn px[KV_MAX], py[KV_MAX];
    for (int64_t c = 0; c < nc; c++) {
        const int k = off[c + 1] - off[c];
        if (k < 3 || k > KV_MAX) return AVM_EINVAL;
        cell_disp(off, cv, (int)c, vx, vy, Lx, Ly, dx, dy);
        for (int m = 0; m < k; m++) {
            px[m] = dn_c(dx[m]);
            py[m] = dn_c(dy[m]);
        }
        poly_energy(k, px, py, 0, 0, 0, 0, &A[c], &P[c]);
    }
    return AVM_OK;
}

/* F_v = -sum over the cells at v of dE_c/dh_v, each derivative by two
 * tangent passes (seed dx or dy on vertex v's displacement) */
int orc_avm_forces(int64_t nc, int64_t nv, const double* vx, const double* vy, double Lx, double Ly,
                   const int32_t* off, const int32_t* cv, const double* A0, const double* P0, double KA, double KP,
                   double* fx, double* fy)
{
    double dx[KV_MAX], dy[KV_MAX];
    dn px[KV_MAX], py[KV_MAX];
    for (int64_t v = 0; v < nv; v++) fx[v] = fy[v] = 0;
    for (int64_t c = 0; c < nc; c++) {
        const int k = off[c + 1] - off[c];
        if (k < 3 || k > KV_MAX) return AVM_EINVAL;
        cell_disp(off, cv, (int)c, vx, vy, Lx, Ly, dx, dy);
        for (int s = 0; s < k; s++) {
            for (int m = 0; m < k; m++) {
                px[m] = dn_c(dx[m]);
                py[m] = dn_c(dy[m]);
            }
            px[s].gx = 1.0;
            py[s].gy = 1.0;
            const dn e = poly_energy(k, px, py, A0[c], P0[c], KA, KP, NULL, NULL);
            const int v = cv[off[c] + s];
            fx[v] -= e.gx;
            fy[v] -= e.gy;
        }
    }
    return AVM_OK;
}

/* ------------------------------------------------------------------ */
/* T1 transitions on the cell lists                                    */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t nc, nv, cap;
    int32_t* off;  /* nc + 1 */
    int32_t* cv;   /* cap entries */
} net;

static int pos_in(const net* N, int c, int v)
{
    for (int m = N->off[c]; m < N->off[c + 1]; m++)
        if (N->cv[m] == v) return m - N->off[c];
    return -1;
}

static int cell_len(const net* N, int c) { return N->off[c + 1] - N->off[c]; }
static int cell_at(const net* N, int c, int m)
{
    const int k = cell_len(N, c);
    return N->cv[N->off[c] + ((m % k) + k) % k];
}

/* the three cells of every vertex (vertex -> cells table, rebuilt per round) */
static void vertex_cells(const net* N, int32_t* vcell)
{
    for (int64_t v = 0; v < N->nv; v++) vcell[3 * v] = vcell[3 * v + 1] = vcell[3 * v + 2] = -1;
    for (int64_t c = 0; c < N->nc; c++)
        for (int m = N->off[c]; m < N->off[c + 1]; m++) {
            int32_t* s = vcell + 3 * N->cv[m];
            if (s[0] < 0) s[0] = (int32_t)c;
            else if (s[1] < 0) s[1] = (int32_t)c;
            else s[2] = (int32_t)c;
        }
}

typedef struct { int v1, v2, X, Y, C1, D1; int64_t key; } t1edge;

static int third_cell(const int32_t* vcell, int v, int a, int b)
{
    for (int k = 0; k < 3; k++)
        if (vcell[3 * v + k] != a && vcell[3 * v + k] != b) return vcell[3 * v + k];
    return -1;
}

static int share_vertex(const net* N, int a, int b)
{
    for (int m = N->off[a]; m < N->off[a + 1]; m++)
        for (int n = N->off[b]; n < N->off[b + 1]; n++)
            if (N->cv[m] == N->cv[n]) return 1;
    return 0;
}

/* replace cell c's list by the k entries of list */
static int set_cell(net* N, int c, const int32_t* list, int k)
{
    const int old = cell_len(N, c), d = k - old;
    if (d != 0) {
        if (N->off[N->nc] + d > N->cap) return AVM_ECAP;
        memmove(N->cv + N->off[c + 1] + d, N->cv + N->off[c + 1],
                sizeof(int32_t) * (size_t)(N->off[N->nc] - N->off[c + 1]));
        for (int64_t e = c + 1; e <= N->nc; e++) N->off[e] += d;
    }
    memcpy(N->cv + N->off[c], list, sizeof(int32_t) * (size_t)k);
    return AVM_OK;
}

/* remove vertex v from cell c's list */
static int cell_remove(net* N, int c, int v)
{
    int32_t tmp[KV_MAX];
    int k = 0;
    for (int m = N->off[c]; m < N->off[c + 1]; m++)
        if (N->cv[m] != v) tmp[k++] = N->cv[m];
    return set_cell(N, c, tmp, k);
}

/* insert vertex w into cell c's list just before vertex v */
static int cell_insert_before(net* N, int c, int v, int w)
{
    int32_t tmp[KV_MAX];
    int k = 0;
    if (cell_len(N, c) + 1 > KV_MAX) return AVM_ECAP;
    for (int m = N->off[c]; m < N->off[c + 1]; m++) {
        if (N->cv[m] == v) tmp[k++] = w;
        tmp[k++] = N->cv[m];
    }
    return set_cell(N, c, tmp, k);
}

/* One round: every qualifying edge whose key is the smallest among the
 * qualifying edges touching its four cells flips.  Returns the number of
 * flips (>= 0) or an error. */
static int t1_round(net* N, double* vx, double* vy, double Lx, double Ly, int q, double lt1, double lnew,
                    int32_t* vcell, int64_t* cmin, t1edge* E)
{
    vertex_cells(N, vcell);
    int ne = 0;
    const double l2 = lt1 * lt1;
    for (int64_t c = 0; c < N->nc; c++) {
        const int k = cell_len(N, (int)c);
        for (int m = 0; m < k; m++) {
            /* each edge once: in the cell that holds it as v1 -> v2 with v1 < v2 */
            const int v1 = cell_at(N, (int)c, m), v2 = cell_at(N, (int)c, m + 1);
            if (v1 > v2) continue;
            const double dx = mimg(vx[v2] - vx[v1], Lx), dy = mimg(vy[v2] - vy[v1], Ly);
            const double xx = dx * dx, yy = dy * dy;
            if (!(xx + yy < l2)) continue;
            const int X = (int)c;
            /* Y: the other cell holding both v1 and v2 */
            int Yc = -1, C1 = -1, D1 = -1;
            for (int s = 0; s < 3; s++) {
                const int cc = vcell[3 * v1 + s];
                if (cc != X && pos_in(N, cc, v2) >= 0) Yc = cc;
            }
            if (Yc < 0) return AVM_EFAIL;
            C1 = third_cell(vcell, v1, X, Yc);
            D1 = third_cell(vcell, v2, X, Yc);
            if (C1 < 0 || D1 < 0) return AVM_EFAIL;
            if (cell_len(N, X) <= 3 || cell_len(N, Yc) <= 3) continue;
            if (C1 == D1 || share_vertex(N, C1, D1)) continue;
            t1edge e = {v1, v2, X, Yc, C1, D1, ((int64_t)v1 << 32) | (int64_t)v2};
            E[ne++] = e;
        }
    }
    if (ne == 0) return 0;
    for (int64_t c = 0; c < N->nc; c++) cmin[c] = INT64_MAX;
    for (int i = 0; i < ne; i++) {
        const int cs[4] = {E[i].X, E[i].Y, E[i].C1, E[i].D1};
        for (int k = 0; k < 4; k++)
            if (E[i].key < cmin[cs[k]]) cmin[cs[k]] = E[i].key;
    }
    int flips = 0;
    for (int i = 0; i < ne; i++) {
        const t1edge e = E[i];
        if (cmin[e.X] != e.key || cmin[e.Y] != e.key || cmin[e.C1] != e.key || cmin[e.D1] != e.key) continue;
        /* geometry: the perpendicular of the edge through its midpoint, v1
         * on the side of X (left of v1 -> v2) */
        const double ex = mimg(vx[e.v2] - vx[e.v1], Lx), ey = mimg(vy[e.v2] - vy[e.v1], Ly);
        const double mx = vx[e.v1] + 0.5 * ex, my = vy[e.v1] + 0.5 * ey;
        const double len = sqrt(ex * ex + ey * ey);
        if (!(len > 0)) return AVM_EFAIL;
        const double rx = -ey / len, ry = ex / len;
        vx[e.v1] = wrap_q(mx + 0.5 * lnew * rx, Lx, q);
        vy[e.v1] = wrap_q(my + 0.5 * lnew * ry, Ly, q);
        vx[e.v2] = wrap_q(mx - 0.5 * lnew * rx, Lx, q);
        vy[e.v2] = wrap_q(my - 0.5 * lnew * ry, Ly, q);
        /* topology: X and Y lose a vertex, the end cells gain one */
        int st;
        if ((st = cell_remove(N, e.X, e.v2)) || (st = cell_remove(N, e.Y, e.v1)) ||
            (st = cell_insert_before(N, e.C1, e.v1, e.v2)) || (st = cell_insert_before(N, e.D1, e.v2, e.v1)))
            return st;
        flips++;
    }
    return flips;
}

/* ------------------------------------------------------------------ */
/* a run of steps                                                      */
/* ------------------------------------------------------------------ */
/* n steps from the state (vx, vy, theta, cell lists off/cv with room for
 * cap entries); all arrays updated in place.  step0: noise counter of the
 * first step.  counters[0] = T1 transitions, counters[1] = T1 rounds.  E and
 * qbar (nsteps + 1 entries, may be NULL): energy and mean shape index at the
 * start of every step and at the end. */
int orc_avm_run(int64_t nc, int64_t nv, double* vx, double* vy, double* theta, double Lx, double Ly, int q,
                int32_t* off, int32_t* cv, int64_t cap, const double* A0, const double* P0, const avm_params* p,
                uint64_t step0, int64_t nsteps, double* E, double* qbar, int64_t* counters)
{
    double* fx = malloc(sizeof(double) * (size_t)nv);
    double* fy = malloc(sizeof(double) * (size_t)nv);
    double* A = malloc(sizeof(double) * (size_t)nc);
    double* P = malloc(sizeof(double) * (size_t)nc);
    int32_t* vcell = malloc(sizeof(int32_t) * 3 * (size_t)nv);
    int64_t* cmin = malloc(sizeof(int64_t) * (size_t)nc);
    t1edge* edges = malloc(sizeof(t1edge) * 3 * (size_t)nv);
    int st = AVM_OK;
    if (!fx || !fy || !A || !P || !vcell || !cmin || !edges) {
        st = AVM_ENOMEM;
        goto done;
    }
    net N = {nc, nv, cap, off, cv};
    const double amp = sqrt(2.0 * p->Dr * p->dt);
    if (counters) counters[0] = counters[1] = 0;
    for (int64_t t = 0; t <= nsteps; t++) {
        if ((st = orc_avm_geometry(nc, vx, vy, Lx, Ly, off, cv, A, P))) goto done;
        if (E || qbar) {
            double e = 0, qs = 0;
            for (int64_t c = 0; c < nc; c++) {
                e += p->KA * (A[c] - A0[c]) * (A[c] - A0[c]) + p->KP * (P[c] - P0[c]) * (P[c] - P0[c]);
                qs += P[c] / sqrt(A[c]);
            }
            if (E) E[t] = e;
            if (qbar) qbar[t] = qs / (double)nc;
        }
        if (t == nsteps) break;
        if ((st = orc_avm_forces(nc, nv, vx, vy, Lx, Ly, off, cv, A0, P0, p->KA, p->KP, fx, fy))) goto done;
        /* Eq. (4): each vertex moves with the mean director of its cells */
        vertex_cells(&N, vcell);
        for (int64_t v = 0; v < nv; v++) {
            double sx = 0, sy = 0;
            for (int k = 0; k < 3; k++) {
                sx += cos(theta[vcell[3 * v + k]]);
                sy += sin(theta[vcell[3 * v + k]]);
            }
            const double nx = vx[v] + p->dt * (p->mu * fx[v] + p->v0 * sx / 3.0);
            const double ny = vy[v] + p->dt * (p->mu * fy[v] + p->v0 * sy / 3.0);
            vx[v] = wrap_q(nx, Lx, q);
            vy[v] = wrap_q(ny, Ly, q);
        }
        for (int64_t c = 0; c < nc; c++) theta[c] += amp * orc_normal(p->seed, step0 + (uint64_t)t, (uint64_t)c);
        /* T1 rounds until no edge qualifies */
        for (int r = 0;; r++) {
            if (r >= 1000) {
                st = AVM_EFAIL;
                goto done;
            }
            const int f = t1_round(&N, vx, vy, Lx, Ly, q, p->l_t1, p->l_new, vcell, cmin, edges);
            if (f < 0) {
                st = f;
                goto done;
            }
            if (f == 0) break;
            if (counters) {
                counters[0] += f;
                counters[1] += 1;
            }
        }
    }
done:
    free(fx);
    free(fy);
    free(A);
    free(P);
    free(vcell);
    free(cmin);
    free(edges);
    return st;
}
