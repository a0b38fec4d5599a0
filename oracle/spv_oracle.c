/*
 * spv_oracle.c -- plain CPU oracle of one self-propelled Voronoi (SPV) step.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test-suite, the smoke
 * check and the benchmark's CPU-baseline leg may load this library.  It
 * shares no code, header, table or helper with the HIP library.
 *
 * What it computes (Sussman, "cellGPU", arXiv:1702.02939):
 *   - the Delaunay triangulation of the cell centres on the flat torus,
 *     defined by the empty-circumcircle property (Sec. II.C.3), rebuilt
 *     from scratch every step by Bowyer-Watson insertion of the box points
 *     plus a band of periodic images;
 *   - Voronoi areas A_i and perimeters P_i, the Voronoi vertices being the
 *     circumcentres of the Delaunay triangles (Sec. II.C.1);
 *   - the energy of Eq. (1) and the forces F_i = -dE/dr_i (the sign of
 *     App. B, Eq. B1) by forward-mode dual numbers applied to the energy of
 *     the cells whose shape depends on r_i (topology held fixed);
 *   - the equation of motion Eq. (3) integrated by Euler-Maruyama with the
 *     rotational white noise of Sec. II.A.
 *
 * Readings where the paper is silent:
 *   - positions live on the dyadic grid 2^-q, q = 51 - ceil(log2 max(Lx,Ly)),
 *     so that every minimum-image displacement is an exact double and the
 *     orientation / in-circle signs are exact;
 *   - four or more cocircular points are resolved by symbolic perturbation
 *     of the lifted coordinate |p|^2, the point of highest rank (rank = tag)
 *     carrying the dominant perturbation;
 *   - noise: Philox4x64-10 (Salmon et al., SC'11) with key (seed, 0) and
 *     counter (step, tag, 0, 0); Box-Muller cos branch on 53-bit uniforms
 *     (r >> 11) * 2^-53 + 2^-54;
 *   - update order: positions move with the director of the step start,
 *     then the director rotates by sqrt(2 Dr dt) * xi.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_TWO_PI 6.283185307179586476925286766559

typedef __int128 i128;
typedef unsigned __int128 u128;

/* ------------------------------------------------------------------ */
/* grid quantisation                                                   */
/* ------------------------------------------------------------------ */

/* q such that the larger box side is at most 2^(51-q). */
int orc_grid_q(double Lmax)
{
    int e;
    double f = frexp(Lmax, &e);          /* Lmax = f 2^e, f in [0.5,1) */
    int c = (f == 0.5) ? e - 1 : e;      /* ceil(log2 Lmax) */
    return 51 - c;
}

static int64_t to_grid(double v, int q) { return (int64_t)llrint(ldexp(v, q)); }

static int64_t wrap_grid(int64_t X, int64_t LX)
{
    X %= LX;
    if (X < 0) X += LX;
    return X;
}

/* Quantise n values onto the grid of box side L (returned rounded too). */
void orc_quantize(int64_t n, double* v, double L, int q, double* Lq)
{
    int64_t LX = to_grid(L, q);
    for (int64_t k = 0; k < n; k++) v[k] = ldexp((double)wrap_grid(to_grid(v[k], q), LX), -q);
    *Lq = ldexp((double)LX, -q);
}

/* ------------------------------------------------------------------ */
/* exact arithmetic: sign-magnitude integers with 32-bit limbs          */
/* ------------------------------------------------------------------ */
#define NLIMB 10
typedef struct { int sgn; uint32_t w[NLIMB]; } big;

static big big_from(i128 v)
{
    big r;
    memset(&r, 0, sizeof r);
    if (v == 0) return r;
    r.sgn = v < 0 ? -1 : 1;
    u128 m = v < 0 ? (u128)0 - (u128)v : (u128)v;
    for (int k = 0; k < 4; k++) { r.w[k] = (uint32_t)m; m >>= 32; }
    return r;
}

static big big_mul(const big* a, const big* b)
{
    big r;
    memset(&r, 0, sizeof r);
    if (!a->sgn || !b->sgn) return r;
    for (int i = 0; i < NLIMB; i++) {
        uint64_t carry = 0;
        for (int j = 0; i + j < NLIMB; j++) {
            uint64_t t = (uint64_t)a->w[i] * b->w[j] + r.w[i + j] + carry;
            r.w[i + j] = (uint32_t)t;
            carry = t >> 32;
        }
    }
    r.sgn = a->sgn * b->sgn;
    return r;
}

static int big_cmpmag(const big* a, const big* b)
{
    for (int k = NLIMB - 1; k >= 0; k--)
        if (a->w[k] != b->w[k]) return a->w[k] > b->w[k] ? 1 : -1;
    return 0;
}

static big big_add(const big* a, const big* b)
{
    if (!a->sgn) return *b;
    if (!b->sgn) return *a;
    big r;
    memset(&r, 0, sizeof r);
    if (a->sgn == b->sgn) {
        uint64_t c = 0;
        for (int k = 0; k < NLIMB; k++) {
            uint64_t t = (uint64_t)a->w[k] + b->w[k] + c;
            r.w[k] = (uint32_t)t;
            c = t >> 32;
        }
        r.sgn = a->sgn;
        return r;
    }
    int cm = big_cmpmag(a, b);
    if (cm == 0) return r;
    const big* hi = cm > 0 ? a : b;
    const big* lo = cm > 0 ? b : a;
    int64_t br = 0;
    for (int k = 0; k < NLIMB; k++) {
        int64_t t = (int64_t)hi->w[k] - lo->w[k] - br;
        br = t < 0;
        if (t < 0) t += ((int64_t)1 << 32);
        r.w[k] = (uint32_t)t;
    }
    r.sgn = hi->sgn;
    return r;
}

/* ------------------------------------------------------------------ */
/* predicates on integer grid coordinates                               */
/* ------------------------------------------------------------------ */

/* > 0 iff a, b, c are in counter-clockwise order. Exact (|coords| < 2^61). */
static int orient_xy(int64_t ax, int64_t ay, int64_t bx, int64_t by, int64_t cx, int64_t cy)
{
    i128 det = (i128)(ax - cx) * (by - cy) - (i128)(ay - cy) * (bx - cx);
    return (det > 0) - (det < 0);
}

static int64_t orc_exact_incircle_calls = 0;

/* > 0 iff d lies strictly inside the circle through a, b, c (a, b, c CCW);
 * this is the 4x4 determinant of rows (x, y, x^2+y^2, 1) of a, b, c, d. */
static int incircle_xy(int64_t ax, int64_t ay, int64_t bx, int64_t by,
                       int64_t cx, int64_t cy, int64_t dx, int64_t dy)
{
    int64_t adx = ax - dx, ady = ay - dy, bdx = bx - dx, bdy = by - dy, cdx = cx - dx, cdy = cy - dy;
    const int64_t lim = (int64_t)1 << 53;
    if (llabs(adx) < lim && llabs(ady) < lim && llabs(bdx) < lim && llabs(bdy) < lim &&
        llabs(cdx) < lim && llabs(cdy) < lim) {
        /* floating-point filter; every input below is an exact double, so the
         * rounding error of the expression is at most ~1.1e-15 * permanent */
        double fadx = (double)adx, fady = (double)ady, fbdx = (double)bdx, fbdy = (double)bdy;
        double fcdx = (double)cdx, fcdy = (double)cdy;
        double al = fadx * fadx + fady * fady, bl = fbdx * fbdx + fbdy * fbdy, cl = fcdx * fcdx + fcdy * fcdy;
        double t1 = fbdx * fcdy - fbdy * fcdx, t2 = fcdx * fady - fcdy * fadx, t3 = fadx * fbdy - fady * fbdx;
        double det = al * t1 + bl * t2 + cl * t3;
        double perm = (fabs(fbdx * fcdy) + fabs(fbdy * fcdx)) * al + (fabs(fcdx * fady) + fabs(fcdy * fadx)) * bl +
                      (fabs(fadx * fbdy) + fabs(fady * fbdx)) * cl;
        double bound = 4.0e-15 * perm;
        if (det > bound) return 1;
        if (-det > bound) return -1;
    }
    orc_exact_incircle_calls++;
    big al = big_from((i128)adx * adx + (i128)ady * ady);
    big bl = big_from((i128)bdx * bdx + (i128)bdy * bdy);
    big cl = big_from((i128)cdx * cdx + (i128)cdy * cdy);
    big t1 = big_from((i128)bdx * cdy - (i128)bdy * cdx);
    big t2 = big_from((i128)cdx * ady - (i128)cdy * adx);
    big t3 = big_from((i128)adx * bdy - (i128)ady * bdx);
    big p1 = big_mul(&al, &t1), p2 = big_mul(&bl, &t2), p3 = big_mul(&cl, &t3);
    big s = big_add(&p1, &p2);
    s = big_add(&s, &p3);
    return s.sgn;
}

/* In-circle with the symbolic tie-break: lifted coordinate of point p is
 * |p|^2 + eps^(f(rank p)), f decreasing in rank.  When the exact determinant
 * is zero its sign is that of the cofactor of the highest-rank row. */
static int incircle_sos(const int64_t* P, const int64_t* rank, int a, int b, int c, int d)
{
    int s = incircle_xy(P[2 * a], P[2 * a + 1], P[2 * b], P[2 * b + 1], P[2 * c], P[2 * c + 1], P[2 * d], P[2 * d + 1]);
    if (s) return s;
    int id[4] = {a, b, c, d};
    int top = 0;
    for (int k = 1; k < 4; k++) if (rank[id[k]] > rank[id[top]]) top = k;
#define OR3(u, v, w) orient_xy(P[2 * (u)], P[2 * (u) + 1], P[2 * (v)], P[2 * (v) + 1], P[2 * (w)], P[2 * (w) + 1])
    switch (top) {
    case 0: return OR3(b, c, d);
    case 1: return -OR3(a, c, d);
    case 2: return OR3(a, b, d);
    default: return -OR3(a, b, c);
    }
#undef OR3
}

/* exported for the test-suite: same predicates on raw integer input */
int orc_orient(const int64_t* a, const int64_t* b, const int64_t* c)
{
    return orient_xy(a[0], a[1], b[0], b[1], c[0], c[1]);
}
int orc_incircle(const int64_t* a, const int64_t* b, const int64_t* c, const int64_t* d)
{
    return incircle_xy(a[0], a[1], b[0], b[1], c[0], c[1], d[0], d[1]);
}
int orc_incircle_sos(const int64_t* a, const int64_t* b, const int64_t* c, const int64_t* d, const int64_t* ranks)
{
    int64_t P[8] = {a[0], a[1], b[0], b[1], c[0], c[1], d[0], d[1]};
    return incircle_sos(P, ranks, 0, 1, 2, 3);
}
int64_t orc_exact_calls(void) { return orc_exact_incircle_calls; }

/* ------------------------------------------------------------------ */
/* Bowyer-Watson triangulation                                          */
/* ------------------------------------------------------------------ */
typedef struct { int v[3]; int n[3]; } tri;   /* CCW vertices; n[k] across the edge opposite v[k] */

typedef struct {
    int64_t* P;      /* 2 * np grid coordinates */
    int64_t* rank;
    int np;
    tri* t;
    int nt, cap;
    int* freel;
    int nfree, freecap;
    int* vtri;       /* one live triangle per vertex */
    int* mark;       /* per triangle: stamp of the last cavity search that tested it */
    int* incav;      /* per triangle: stamp if in the current cavity */
    int stamp;
} bw;

static int bw_newtri(bw* T)
{
    if (T->nfree > 0) return T->freel[--T->nfree];
    if (T->nt == T->cap) {
        T->cap = T->cap ? 2 * T->cap : 1024;
        T->t = realloc(T->t, sizeof(tri) * T->cap);
        T->mark = realloc(T->mark, sizeof(int) * T->cap);
        T->incav = realloc(T->incav, sizeof(int) * T->cap);
    }
    T->mark[T->nt] = 0;
    T->incav[T->nt] = 0;
    return T->nt++;
}

static void bw_free(bw* T, int k)
{
    if (T->nfree == T->freecap) {
        T->freecap = T->freecap ? 2 * T->freecap : 1024;
        T->freel = realloc(T->freel, sizeof(int) * T->freecap);
    }
    T->t[k].v[0] = -1;
    T->freel[T->nfree++] = k;
}

static int orient_ids(const bw* T, int a, int b, int c)
{
    const int64_t* P = T->P;
    return orient_xy(P[2 * a], P[2 * a + 1], P[2 * b], P[2 * b + 1], P[2 * c], P[2 * c + 1]);
}

/* Walk from triangle `start` to a triangle containing point p (inside or on
 * its boundary).  Returns -1 if the walk leaves the hull. */
static int bw_locate(const bw* T, int start, int p, uint32_t* rng)
{
    int t = start;
    for (long guard = 0; guard < 100000000L; guard++) {
        *rng = *rng * 1664525u + 1013904223u;
        int k0 = (int)((*rng >> 16) % 3u);
        int moved = 0;
        for (int e = 0; e < 3; e++) {
            int k = (k0 + e) % 3;
            int a = T->t[t].v[(k + 1) % 3], b = T->t[t].v[(k + 2) % 3];
            if (orient_ids(T, a, b, p) < 0) {
                t = T->t[t].n[k];
                if (t < 0) return -1;
                moved = 1;
                break;
            }
        }
        if (!moved) return t;
    }
    return -1;
}

typedef struct { int a, b, out; } bedge;

/* insert point p; returns 0 on success */
static int bw_insert(bw* T, int p, int* last, uint32_t* rng, int** stack, int* stcap,
                     bedge** be, int* becap, int** cav, int* cavcap, int* start_of, int* end_of)
{
    int t0 = bw_locate(T, *last, p, rng);
    if (t0 < 0) return -1;
    T->stamp++;
    int st = T->stamp;
    int ns = 0, nbe = 0, ncav = 0;
#define PUSH(arr, n, cap, val) do { if ((n) == (cap)) { (cap) = (cap) ? 2 * (cap) : 256; (arr) = realloc((arr), sizeof(*(arr)) * (cap)); } (arr)[(n)++] = (val); } while (0)
    T->incav[t0] = st;
    T->mark[t0] = st;
    PUSH(*stack, ns, *stcap, t0);
    PUSH(*cav, ncav, *cavcap, t0);
    while (ns > 0) {
        int c = (*stack)[--ns];
        for (int k = 0; k < 3; k++) {
            int nb = T->t[c].n[k];
            if (nb >= 0 && T->incav[nb] == st) continue;
            int take = 0;
            if (nb >= 0) {
                if (T->mark[nb] != st) {
                    T->mark[nb] = st;
                    const tri* tn = &T->t[nb];
                    if (incircle_sos(T->P, T->rank, tn->v[0], tn->v[1], tn->v[2], p) > 0) take = 1;
                } else {
                    take = 0;   /* tested before and rejected */
                }
            }
            if (take) {
                T->incav[nb] = st;
                PUSH(*stack, ns, *stcap, nb);
                PUSH(*cav, ncav, *cavcap, nb);
            } else {
                bedge e = {T->t[c].v[(k + 1) % 3], T->t[c].v[(k + 2) % 3], nb};
                PUSH(*be, nbe, *becap, e);
            }
        }
    }
    /* a rejected neighbour can be reached twice; the boundary list may then
     * hold an edge whose outside triangle joined the cavity later: drop it */
    int m = 0;
    for (int k = 0; k < nbe; k++) {
        bedge e = (*be)[k];
        if (e.out >= 0 && T->incav[e.out] == st) continue;
        (*be)[m++] = e;
    }
    nbe = m;
    for (int k = 0; k < ncav; k++) bw_free(T, (*cav)[k]);
    int* newt = *stack;   /* reuse: stack is empty now */
    if (*stcap < nbe) { *stcap = nbe; *stack = realloc(*stack, sizeof(int) * nbe); newt = *stack; }
    for (int k = 0; k < nbe; k++) {
        bedge e = (*be)[k];
        int nt = bw_newtri(T);
        tri* t = &T->t[nt];
        t->v[0] = e.a; t->v[1] = e.b; t->v[2] = p;
        t->n[2] = e.out;
        t->n[0] = t->n[1] = -1;
        if (e.out >= 0) {
            tri* o = &T->t[e.out];
            for (int j = 0; j < 3; j++) {
                int oa = o->v[(j + 1) % 3], ob = o->v[(j + 2) % 3];
                if (oa == e.b && ob == e.a) { o->n[j] = nt; break; }
            }
        }
        start_of[e.a] = nt;
        end_of[e.b] = nt;
        newt[k] = nt;
        T->vtri[e.a] = nt; T->vtri[e.b] = nt; T->vtri[p] = nt;
    }
    for (int k = 0; k < nbe; k++) {
        tri* t = &T->t[newt[k]];
        t->n[0] = start_of[t->v[1]];   /* edge (b, p) */
        t->n[1] = end_of[t->v[0]];     /* edge (p, a) */
    }
    *last = newt[0];
#undef PUSH
    return 0;
}

/* ------------------------------------------------------------------ */
/* periodic triangulation                                              */
/* ------------------------------------------------------------------ */
enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_EPRECOND = -4, ORC_ECAPACITY = -5, ORC_EFAIL = -8 };

static int cmp_i64pair(const void* a, const void* b)
{
    const int64_t* x = a; const int64_t* y = b;
    if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
    if (x[1] != y[1]) return x[1] < y[1] ? -1 : 1;
    return 0;
}

/*
 * Periodic Delaunay triangulation of n points (grid coordinates X, Y in
 * [0,LX) x [0,LY)).  Output: for every point (tag order) its neighbours in
 * counter-clockwise order starting at the smallest tag (ring_off[n+1],
 * ring[...]).  ntri_out = number of triangles on the torus.  Returns
 * ORC_EPRECOND if some triangle's circumradius reaches min(Lx,Ly)/4 or if
 * the image band cannot certify the result.
 */
static int triangulate_grid(int64_t n, const int64_t* X, const int64_t* Y, int64_t LX, int64_t LY,
                            int32_t* ring_off, int32_t* ring, int64_t cap, int64_t* ntri_out,
                            double* maxcr_out)
{
    if (n < 3) return ORC_EINVAL;
    double spacing = sqrt((double)LX * (double)LY / (double)n);
    int64_t Lmin = LX < LY ? LX : LY;
    double w = 3.0 * spacing;
    for (int attempt = 0; attempt < 8; attempt++) {
        int64_t W = (int64_t)ceil(w);
        if (W > Lmin) W = Lmin;
        /* box points first (ids 0..n-1), then images inside the band */
        int64_t maxp = 9 * n + 4;
        int64_t* P = malloc(sizeof(int64_t) * 2 * maxp);
        int64_t* rank = malloc(sizeof(int64_t) * maxp);
        int* tagof = malloc(sizeof(int) * maxp);
        if (!P || !rank || !tagof) { free(P); free(rank); free(tagof); return ORC_ENOMEM; }
        int np = 0;
        for (int64_t i = 0; i < n; i++) {
            P[2 * np] = X[i]; P[2 * np + 1] = Y[i];
            rank[np] = (int64_t)i * 16 + 4; tagof[np] = (int)i; np++;
        }
        for (int sy = -1; sy <= 1; sy++)
            for (int sx = -1; sx <= 1; sx++) {
                if (!sx && !sy) continue;
                int img = (sy + 1) * 3 + (sx + 1);
                for (int64_t i = 0; i < n; i++) {
                    int64_t px = X[i] + sx * LX, py = Y[i] + sy * LY;
                    if (px < -W || px >= LX + W || py < -W || py >= LY + W) continue;
                    P[2 * np] = px; P[2 * np + 1] = py;
                    rank[np] = (int64_t)i * 16 + img; tagof[np] = (int)i; np++;
                }
            }
        /* frame: four corners strictly outside the extended region */
        int64_t F = W + (int64_t)ceil(spacing) + 1;
        int64_t fx[4] = {-F, LX + F, LX + F, -F}, fy[4] = {-F, -F, LY + F, LY + F};
        int f0 = np;
        for (int k = 0; k < 4; k++) {
            P[2 * np] = fx[k]; P[2 * np + 1] = fy[k];
            rank[np] = INT64_MAX - 4 + k; tagof[np] = -1; np++;
        }
        /* insertion order: bins of side ~2 spacings, rows in serpentine order */
        double bs = 2.0 * spacing;
        int64_t ex0 = -W, ey0 = -W;
        int64_t nbx = (int64_t)((double)(LX + 2 * W) / bs) + 1, nby = (int64_t)((double)(LY + 2 * W) / bs) + 1;
        int64_t* key = malloc(sizeof(int64_t) * 2 * f0);
        for (int k = 0; k < f0; k++) {
            int64_t bx = (int64_t)((double)(P[2 * k] - ex0) / bs), by = (int64_t)((double)(P[2 * k + 1] - ey0) / bs);
            if (bx >= nbx) bx = nbx - 1;
            if (by >= nby) by = nby - 1;
            if (by & 1) bx = nbx - 1 - bx;
            key[2 * k] = by * nbx + bx;
            key[2 * k + 1] = k;
        }
        qsort(key, f0, 2 * sizeof(int64_t), cmp_i64pair);

        bw T;
        memset(&T, 0, sizeof T);
        T.P = P; T.rank = rank; T.np = np;
        T.vtri = malloc(sizeof(int) * np);
        for (int k = 0; k < np; k++) T.vtri[k] = -1;
        int ta = bw_newtri(&T), tb = bw_newtri(&T);
        /* corners 0..3 CCW: (f0, f0+1, f0+2) and (f0, f0+2, f0+3) */
        T.t[ta].v[0] = f0; T.t[ta].v[1] = f0 + 1; T.t[ta].v[2] = f0 + 2;
        T.t[ta].n[0] = -1; T.t[ta].n[1] = tb; T.t[ta].n[2] = -1;
        T.t[tb].v[0] = f0; T.t[tb].v[1] = f0 + 2; T.t[tb].v[2] = f0 + 3;
        T.t[tb].n[0] = -1; T.t[tb].n[1] = -1; T.t[tb].n[2] = ta;
        for (int k = 0; k < 4; k++) T.vtri[f0 + k] = (k == 1) ? ta : tb;
        int last = ta;
        uint32_t rng = 12345u;
        int *stack = NULL, *cav = NULL;
        bedge* be = NULL;
        int stcap = 0, becap = 0, cavcap = 0;
        int* start_of = malloc(sizeof(int) * np);
        int* end_of = malloc(sizeof(int) * np);
        int rc = ORC_OK;
        for (int k = 0; k < f0; k++) {
            int p = (int)key[2 * k + 1];
            if (bw_insert(&T, p, &last, &rng, &stack, &stcap, &be, &becap, &cav, &cavcap, start_of, end_of)) {
                rc = ORC_EFAIL;
                break;
            }
        }
        free(stack); free(cav); free(be); free(start_of); free(end_of); free(key);

        /* stars of the box points; certify every incident triangle */
        int retry = 0;
        int64_t total = 0, ntri3 = 0;
        double maxcr = 0.0;
        double ext_lo_x = (double)-W, ext_hi_x = (double)(LX + W), ext_lo_y = (double)-W, ext_hi_y = (double)(LY + W);
        double Lm = (double)Lmin;
        for (int64_t i = 0; rc == ORC_OK && i < n; i++) {
            int v = (int)i;
            int t = T.vtri[v];
            if (t < 0) { rc = ORC_EFAIL; break; }
            int k = 0;
            while (T.t[t].v[k] != v) k++;
            int t_start = t;
            int deg = 0;
            int64_t base = total;
            int nbuf[64];
            do {
                int a = T.t[t].v[(k + 1) % 3], b = T.t[t].v[(k + 2) % 3];
                if (a >= f0 || b >= f0) { retry = 1; break; }
                /* circumcircle of (v, a, b) relative to v, in grid units */
                double bx = (double)(P[2 * a] - P[2 * v]), by = (double)(P[2 * a + 1] - P[2 * v + 1]);
                double cx = (double)(P[2 * b] - P[2 * v]), cy = (double)(P[2 * b + 1] - P[2 * v + 1]);
                double den = 2.0 * (bx * cy - by * cx);
                double b2 = bx * bx + by * by, c2 = cx * cx + cy * cy;
                double ux = (cy * b2 - by * c2) / den, uy = (bx * c2 - cx * b2) / den;
                double r = sqrt(ux * ux + uy * uy) * (1.0 + 1e-9) + 1.0;
                double ccx = (double)P[2 * v] + ux, ccy = (double)P[2 * v + 1] + uy;
                if (ccx - r <= ext_lo_x || ccx + r >= ext_hi_x || ccy - r <= ext_lo_y || ccy + r >= ext_hi_y) {
                    retry = 1;
                    break;
                }
                if (r > maxcr) maxcr = r;
                if (deg >= 64) { rc = ORC_ECAPACITY; break; }
                nbuf[deg++] = a;
                int tn = T.t[t].n[(k + 1) % 3];   /* across edge (v, b) */
                if (tn < 0) { retry = 1; break; }
                t = tn;
                k = 0;
                while (T.t[t].v[k] != v) k++;
            } while (t != t_start);
            if (retry || rc != ORC_OK) break;
            /* minimum-image consistency and canonical rotation */
            int smin = 0;
            for (int m = 0; m < deg; m++) {
                int a = nbuf[m];
                int64_t dx = P[2 * a] - P[2 * v], dy = P[2 * a + 1] - P[2 * v + 1];
                if (2 * llabs(dx) >= LX || 2 * llabs(dy) >= LY) { rc = ORC_EPRECOND; break; }
                if (tagof[a] < tagof[nbuf[smin]]) smin = m;
            }
            if (rc != ORC_OK) break;
            if (base + deg > cap) { rc = ORC_ECAPACITY; break; }
            ring_off[i] = (int32_t)base;
            for (int m = 0; m < deg; m++) ring[base + m] = tagof[nbuf[(smin + m) % deg]];
            total += deg;
            ntri3 += deg;
        }
        if (rc == ORC_OK && !retry) ring_off[n] = (int32_t)total;
        free(T.t); free(T.mark); free(T.incav); free(T.freel); free(T.vtri);
        free(P); free(rank); free(tagof);
        if (rc != ORC_OK) return rc;
        if (!retry) {
            if (maxcr >= Lm / 4.0) return ORC_EPRECOND;
            if (ntri_out) *ntri_out = ntri3 / 3;
            if (maxcr_out) *maxcr_out = maxcr;
            return ORC_OK;
        }
        if (W >= Lmin) return ORC_EPRECOND;
        w *= 2.0;
    }
    return ORC_EPRECOND;
}

int orc_triangulate(int64_t n, const double* x, const double* y, double Lx, double Ly, int q,
                    int32_t* ring_off, int32_t* ring, int64_t cap, int64_t* ntri_out, double* maxcr_out)
{
    int64_t* X = malloc(sizeof(int64_t) * n);
    int64_t* Y = malloc(sizeof(int64_t) * n);
    if (!X || !Y) { free(X); free(Y); return ORC_ENOMEM; }
    int64_t LX = to_grid(Lx, q), LY = to_grid(Ly, q);
    for (int64_t i = 0; i < n; i++) {
        X[i] = to_grid(x[i], q);
        Y[i] = to_grid(y[i], q);
        if (X[i] < 0 || X[i] >= LX || Y[i] < 0 || Y[i] >= LY || ldexp((double)X[i], -q) != x[i] ||
            ldexp((double)Y[i], -q) != y[i]) {
            free(X); free(Y);
            return ORC_EINVAL;
        }
    }
    /* distinct positions are required */
    int64_t* srt = malloc(sizeof(int64_t) * 2 * n);
    for (int64_t i = 0; i < n; i++) { srt[2 * i] = X[i]; srt[2 * i + 1] = Y[i]; }
    qsort(srt, n, 2 * sizeof(int64_t), cmp_i64pair);
    for (int64_t i = 1; i < n; i++)
        if (srt[2 * i] == srt[2 * i - 2] && srt[2 * i + 1] == srt[2 * i - 1]) { free(srt); free(X); free(Y); return ORC_EINVAL; }
    free(srt);
    double mcr = 0.0;
    int rc = triangulate_grid(n, X, Y, LX, LY, ring_off, ring, cap, ntri_out, &mcr);
    if (maxcr_out) *maxcr_out = ldexp(mcr, -q);
    free(X); free(Y);
    return rc;
}

/* ------------------------------------------------------------------ */
/* geometry and energy (plain double)                                   */
/* ------------------------------------------------------------------ */

static double min_image(double d, double L)
{
    if (d > 0.5 * L) d -= L;
    else if (d < -0.5 * L) d += L;
    return d;
}

/* circumcentre of (0, b, c) */
static void circumcentre(double bx, double by, double cx, double cy, double* ux, double* uy)
{
    double b2 = bx * bx + by * by, c2 = cx * cx + cy * cy;
    double den = 2.0 * (bx * cy - by * cx);
    *ux = (cy * b2 - by * c2) / den;
    *uy = (bx * c2 - cx * b2) / den;
}

/* Area and perimeter of every Voronoi cell (Sec. II.C.1): the polygon of
 * cell i is the sequence of circumcentres of (i, j_m, j_{m+1}). */
int orc_geometry(int64_t n, const double* x, const double* y, double Lx, double Ly,
                 const int32_t* ring_off, const int32_t* ring, double* A, double* P)
{
    for (int64_t i = 0; i < n; i++) {
        int k = ring_off[i + 1] - ring_off[i];
        const int32_t* r = ring + ring_off[i];
        double a2 = 0.0, per = 0.0, u0x = 0, u0y = 0, upx = 0, upy = 0;
        for (int m = 0; m < k; m++) {
            int j = r[m], jn = r[(m + 1) % k];
            double bx = min_image(x[j] - x[i], Lx), by = min_image(y[j] - y[i], Ly);
            double cx = min_image(x[jn] - x[i], Lx), cy = min_image(y[jn] - y[i], Ly);
            double ux, uy;
            circumcentre(bx, by, cx, cy, &ux, &uy);
            if (m == 0) { u0x = ux; u0y = uy; }
            else {
                a2 += upx * uy - upy * ux;
                per += hypot(ux - upx, uy - upy);
            }
            upx = ux; upy = uy;
        }
        a2 += upx * u0y - upy * u0x;
        per += hypot(u0x - upx, u0y - upy);
        A[i] = 0.5 * a2;
        P[i] = per;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* forces: forward-mode dual numbers, two tangent directions            */
/* ------------------------------------------------------------------ */
typedef struct { double v, gx, gy; } dual;

static dual dc(double v) { dual r = {v, 0.0, 0.0}; return r; }
static dual dadd(dual a, dual b) { dual r = {a.v + b.v, a.gx + b.gx, a.gy + b.gy}; return r; }
static dual dsub(dual a, dual b) { dual r = {a.v - b.v, a.gx - b.gx, a.gy - b.gy}; return r; }
static dual dmul(dual a, dual b) { dual r = {a.v * b.v, a.gx * b.v + a.v * b.gx, a.gy * b.v + a.v * b.gy}; return r; }
static dual ddiv(dual a, dual b)
{
    double q = a.v / b.v;
    dual r = {q, (a.gx - q * b.gx) / b.v, (a.gy - q * b.gy) / b.v};
    return r;
}
/* sqrt; at 0 (a zero-length Voronoi edge, exactly at a T1 configuration)
 * the one-sided derivative is undefined and the tangent is taken as 0 */
static dual dsqrt(dual a)
{
    double s = sqrt(a.v);
    if (s == 0.0) { dual z = {0.0, 0.0, 0.0}; return z; }
    dual r = {s, a.gx / (2.0 * s), a.gy / (2.0 * s)};
    return r;
}

/* energy of one cell; its centre is r_c, neighbour displacements (d[m]) are
 * duals carrying the derivative with respect to the moving cell */
static dual cell_energy(int k, const dual* dx, const dual* dy, double A0, double P0, double KA, double KP)
{
    dual a2 = dc(0.0), per = dc(0.0), u0x = dc(0), u0y = dc(0), upx = dc(0), upy = dc(0);
    for (int m = 0; m < k; m++) {
        int mn = (m + 1) % k;
        dual b2 = dadd(dmul(dx[m], dx[m]), dmul(dy[m], dy[m]));
        dual c2 = dadd(dmul(dx[mn], dx[mn]), dmul(dy[mn], dy[mn]));
        dual den = dmul(dc(2.0), dsub(dmul(dx[m], dy[mn]), dmul(dy[m], dx[mn])));
        dual ux = ddiv(dsub(dmul(dy[mn], b2), dmul(dy[m], c2)), den);
        dual uy = ddiv(dsub(dmul(dx[m], c2), dmul(dx[mn], b2)), den);
        if (m == 0) { u0x = ux; u0y = uy; }
        else {
            a2 = dadd(a2, dsub(dmul(upx, uy), dmul(upy, ux)));
            dual ex = dsub(ux, upx), ey = dsub(uy, upy);
            per = dadd(per, dsqrt(dadd(dmul(ex, ex), dmul(ey, ey))));
        }
        upx = ux; upy = uy;
    }
    a2 = dadd(a2, dsub(dmul(upx, u0y), dmul(upy, u0x)));
    dual ex = dsub(u0x, upx), ey = dsub(u0y, upy);
    per = dadd(per, dsqrt(dadd(dmul(ex, ex), dmul(ey, ey))));
    dual A = dmul(dc(0.5), a2);
    dual dA = dsub(A, dc(A0)), dP = dsub(per, dc(P0));
    return dadd(dmul(dc(KA), dmul(dA, dA)), dmul(dc(KP), dmul(dP, dP)));
}

/* F_i = -d/dr_i sum_{c in {i} + ring(i)} E_c  (topology held fixed) */
int orc_forces(int64_t n, const double* x, const double* y, double Lx, double Ly,
               const int32_t* ring_off, const int32_t* ring, const double* A0, const double* P0,
               double KA, double KP, double* fx, double* fy)
{
    dual dx[64], dy[64];
    for (int64_t i = 0; i < n; i++) {
        int ki = ring_off[i + 1] - ring_off[i];
        const int32_t* ri = ring + ring_off[i];
        dual Etot = dc(0.0);
        for (int s = -1; s < ki; s++) {
            int64_t c = s < 0 ? i : ri[s];
            int kc = ring_off[c + 1] - ring_off[c];
            const int32_t* rc = ring + ring_off[c];
            if (kc > 64) return ORC_ECAPACITY;
            for (int m = 0; m < kc; m++) {
                int j = rc[m];
                dx[m] = dc(min_image(x[j] - x[c], Lx));
                dy[m] = dc(min_image(y[j] - y[c], Ly));
                if (c == i) { dx[m].gx = -1.0; dy[m].gy = -1.0; }
                else if (j == i) { dx[m].gx = 1.0; dy[m].gy = 1.0; }
            }
            Etot = dadd(Etot, cell_energy(kc, dx, dy, A0[c], P0[c], KA, KP));
        }
        fx[i] = -Etot.gx;
        fy[i] = -Etot.gy;
    }
    return ORC_OK;
}

/* E, mean shape index q = P/sqrt(A), total area */
void orc_observables(int64_t n, const double* A, const double* P, const double* A0, const double* P0,
                     double KA, double KP, double* E, double* qbar, double* sumA)
{
    double e = 0.0, qs = 0.0, sa = 0.0;
    for (int64_t i = 0; i < n; i++) {
        e += KA * (A[i] - A0[i]) * (A[i] - A0[i]) + KP * (P[i] - P0[i]) * (P[i] - P0[i]);
        qs += P[i] / sqrt(A[i]);
        sa += A[i];
    }
    *E = e;
    *qbar = qs / (double)n;
    *sumA = sa;
}

/* ------------------------------------------------------------------ */
/* Philox4x64-10 and the rotational noise                               */
/* ------------------------------------------------------------------ */
void orc_philox4x64(const uint64_t* ctr, const uint64_t* key, uint64_t* out)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3], k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; r++) {
        u128 p0 = (u128)M0 * c0, p1 = (u128)M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static double u01(uint64_t r) { return ldexp((double)(r >> 11), -53) + ldexp(1.0, -54); }

/* standard normal for (seed, step, tag) */
double orc_normal(uint64_t seed, uint64_t step, uint64_t tag)
{
    uint64_t ctr[4] = {step, tag, 0, 0}, key[2] = {seed, 0}, r[4];
    orc_philox4x64(ctr, key, r);
    double u1 = u01(r[0]), u2 = u01(r[1]);
    return sqrt(-2.0 * log(u1)) * cos(ORC_TWO_PI * u2);
}

/* initial director for (seed, tag) */
double orc_theta0(uint64_t seed, uint64_t tag)
{
    uint64_t ctr[4] = {UINT64_MAX, tag, 0, 0}, key[2] = {seed, 0}, r[4];
    orc_philox4x64(ctr, key, r);
    return ORC_TWO_PI * u01(r[0]);
}

/* ------------------------------------------------------------------ */
/* the whole step                                                       */
/* ------------------------------------------------------------------ */
typedef struct {
    double KA, KP, mu, v0, Dr, dt;
    uint64_t seed;
} orc_params;

/*
 * Run nsteps SPV steps from (x, y, theta) on the grid of exponent q.
 * Step s (0-based, global index step0 + s): triangulate, geometry, forces,
 * then r += dt (mu F + v0 n), quantise and wrap; theta += sqrt(2 Dr dt) xi.
 * E_traj/q_traj (nsteps+1 entries each, optional) receive E and qbar of the
 * state at the start of every step and of the final state.
 * ring_off/ring (optional) receive the topology of the final state.
 */
int orc_run(int64_t n, double* x, double* y, double* theta, double Lx, double Ly, int q,
            const double* A0, const double* P0, const orc_params* prm, uint64_t step0, int64_t nsteps,
            double* E_traj, double* q_traj, double* fx_out, double* fy_out,
            int32_t* ring_off_out, int32_t* ring_out, int64_t ring_cap)
{
    int64_t cap = 16 * n + 64;
    int32_t* off = malloc(sizeof(int32_t) * (n + 1));
    int32_t* rg = malloc(sizeof(int32_t) * cap);
    double* A = malloc(sizeof(double) * n);
    double* P = malloc(sizeof(double) * n);
    double* fx = malloc(sizeof(double) * n);
    double* fy = malloc(sizeof(double) * n);
    if (!off || !rg || !A || !P || !fx || !fy) { free(off); free(rg); free(A); free(P); free(fx); free(fy); return ORC_ENOMEM; }
    int64_t LX = to_grid(Lx, q), LY = to_grid(Ly, q);
    double noise = sqrt(2.0 * prm->Dr * prm->dt);
    int rc = ORC_OK;
    for (int64_t s = 0; s <= nsteps; s++) {
        int64_t ntri;
        double mcr;
        rc = orc_triangulate(n, x, y, Lx, Ly, q, off, rg, cap, &ntri, &mcr);
        if (rc != ORC_OK) break;
        orc_geometry(n, x, y, Lx, Ly, off, rg, A, P);
        if (E_traj || q_traj) {
            double E, qb, sa;
            orc_observables(n, A, P, A0, P0, prm->KA, prm->KP, &E, &qb, &sa);
            if (E_traj) E_traj[s] = E;
            if (q_traj) q_traj[s] = qb;
        }
        if (s == nsteps) break;
        orc_forces(n, x, y, Lx, Ly, off, rg, A0, P0, prm->KA, prm->KP, fx, fy);
        uint64_t step = step0 + (uint64_t)s;
        for (int64_t i = 0; i < n; i++) {
            double th = theta[i];
            double nx = x[i] + prm->dt * (prm->mu * fx[i] + prm->v0 * cos(th));
            double ny = y[i] + prm->dt * (prm->mu * fy[i] + prm->v0 * sin(th));
            x[i] = ldexp((double)wrap_grid(to_grid(nx, q), LX), -q);
            y[i] = ldexp((double)wrap_grid(to_grid(ny, q), LY), -q);
            theta[i] = th + noise * orc_normal(prm->seed, step, (uint64_t)i);
        }
    }
    if (rc == ORC_OK) {
        if (fx_out && fy_out) {
            orc_forces(n, x, y, Lx, Ly, off, rg, A0, P0, prm->KA, prm->KP, fx_out, fy_out);
        }
        if (ring_off_out && ring_out) {
            if (off[n] > ring_cap) rc = ORC_ECAPACITY;
            else {
                memcpy(ring_off_out, off, sizeof(int32_t) * (n + 1));
                memcpy(ring_out, rg, sizeof(int32_t) * off[n]);
            }
        }
    }
    free(off); free(rg); free(A); free(P); free(fx); free(fy);
    return rc;
}
