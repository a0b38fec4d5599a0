// avm_kernels.hpp -- the active vertex model (AVM) step on gfx950.
//
// Degrees of freedom are the vertices h_v of a trivalent polygonal tiling of
// the periodic box (Sussman 2017, Sec. II.A and Fig. 1).  Topology, kept
// flat for coalesced access:
//   vv[v][k]  the three neighbour vertices of v, counter-clockwise;
//   vc[v][k]  the cell between vv[v][k] and vv[v][k+1] (k+1 mod 3);
//   cv[c][m]  the vertices of cell c counter-clockwise (cdeg[c] of them).
// Cell vc[v][k] holds the directed edge v -> vv[v][k] (the cell lies on its
// left), so in that cell v's successor is vv[v][k] and its predecessor is
// vv[v][k+1]: a vertex's force needs only its three neighbours and the
// energy coefficients of its three cells (App. A).
//
// One step: cell geometry (area, perimeter, a = 2 K_A (A - A0),
// b = 2 K_P (P - P0)); vertex forces and the Eq. 4 move (the mean director
// of the three cells); then T1 rounds (Sec. II.D), the first one also
// rotating the directors: an edge shorter than l_T1 is replaced by its
// perpendicular of length l_new through the same midpoint and the cells at
// its ends become neighbours, at most one transition per cell in a round (an
// edge flips when its key is the smallest key of the qualifying edges at
// each of its four cells), rounds repeated until none qualifies.  Vertices
// live on the dyadic grid 2^-q (re-quantised after every move), so edge
// lengths are exact differences and the T1 test dx*dx + dy*dy < l_T1^2 (no
// fused operations) decides the same way on any implementation that
// follows it.
//
// Memory order is free: vertices and cells carry the labels they were
// created with (vtag, ctag), and everything a result depends on -- which
// end of an edge owns it, the T1 keys, the noise counters -- is taken from
// the labels, never from the slots, so a spatial re-sort (Sec. II.B) moves
// data without changing any result.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spv_common.hpp"

namespace spv {

constexpr int AVM_KV = 16;           // most vertices of a cell
constexpr int AVM_DEV_ROUNDS = 3;    // most T1 rounds per step on the device (then a marking pass that halts if needed)
constexpr int AVM_MAX_ROUNDS = 64;   // T1 rounds per step in all

struct AvmParam {
    double Lx, Ly, hLx, hLy;
    double scale, inv_scale, LXu, LYu;  // grid 2^-q, box in grid units
    double mu, v0, dt, amp;             // Eq. 4, noise amplitude sqrt(2 Dr dt)
    double KA, KP;
    double lt1sq, lnew;                 // T1 threshold squared, new edge length
    uint64_t seed;
};

struct AvmState {
    unsigned long long step;            // noise counter of the next step
    unsigned long long t1, rounds;      // statistics
    unsigned err;
    int halt;                           // a step needs more rounds than the device runs: later kernels wait
    int any[AVM_MAX_ROUNDS + 1];        // round r found a qualifying edge
};

struct AvmArrays {
    double *x, *y;                      // current vertex positions
    double *xo, *yo;                    // the other buffer (the move writes it)
    int* vv;
    int* vc;
    int* cv;
    uint8_t* cdeg;
    double *th, *A0, *P0, *A, *P, *ca, *cb;
    double *fx, *fy;
    long long* lock[2];
    uint8_t* cand;                      // a vertex's candidate edges of the current round (bit k: edge to vv[v][k])
    uint8_t* dirty;                     // round in which a vertex is examined next (rounds >= 1)
    int* lcell;                         // the four cells each candidate edge locked (4 per edge, 3 edges per vertex)
    int* vtag;                          // creation label of each vertex slot
    int* ctag;                          // creation label of each cell slot
    int nv, nc;
};

__device__ __forceinline__ double avm_wrap(double v, double LU)
{
    // v in grid units (an integer-valued double): reduce into [0, LU)
    double X = v - LU * floor(v / LU);
    if (X >= LU) X -= LU;
    if (X < 0.0) X += LU;
    return X;
}

// cell geometry; block 0 also clears the step's round flags.  The first
// eight list entries are read as two 16-byte words and their position
// gathers issued together (entries past the degree re-read the first
// vertex); sums in list order, closing at the first vertex.
__global__ __launch_bounds__(256) void k_avm_geom(AvmArrays a, const AvmParam* __restrict__ pp, AvmState* st)
{
#pragma clang fp contract(off)
    if (st->halt) return;
    const AvmParam& P = *pp;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.x == 0)
        for (int r = threadIdx.x; r <= AVM_MAX_ROUNDS; r += blockDim.x) st->any[r] = 0;
    if (c >= a.nc) return;
    const int k = a.cdeg[c];
    const int* row = a.cv + (size_t)c * AVM_KV;
    const int4 w0 = reinterpret_cast<const int4*>(row)[0], w1 = reinterpret_cast<const int4*>(row)[1];
    const int id[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
    double xs[8], ys[8];
#pragma unroll
    for (int m = 0; m < 8; m++) {
        const int j = m < k ? id[m] : id[0];
        xs[m] = a.x[j];
        ys[m] = a.y[j];
    }
    double px = 0.0, py = 0.0, a2 = 0.0, per = 0.0;
#pragma unroll
    for (int m = 1; m < 8; m++) {
        if (m <= k) {
            double qx = 0.0, qy = 0.0;
            if (m < k) {
                qx = mimg(xs[m] - xs[0], P.Lx, P.hLx);
                qy = mimg(ys[m] - ys[0], P.Ly, P.hLy);
            }
            a2 += px * qy - py * qx;
            const double ex = qx - px, ey = qy - py;
            per += sqrt(ex * ex + ey * ey);
            px = qx;
            py = qy;
        }
    }
    for (int m = 8; m <= k; m++) {  // cells with eight vertices or more
        double qx = 0.0, qy = 0.0;
        if (m < k) {
            const int j = row[m];
            qx = mimg(a.x[j] - xs[0], P.Lx, P.hLx);
            qy = mimg(a.y[j] - ys[0], P.Ly, P.hLy);
        }
        a2 += px * qy - py * qx;
        const double ex = qx - px, ey = qy - py;
        per += sqrt(ex * ex + ey * ey);
        px = qx;
        py = qy;
    }
    const double A = 0.5 * a2;
    a.A[c] = A;
    a.P[c] = per;
    a.ca[c] = 2.0 * P.KA * (A - a.A0[c]);
    a.cb[c] = 2.0 * P.KP * (per - a.P0[c]);
}

// Vertex forces F_v = -sum over v's cells of (a dA/dh + b dP/dh) (App. A:
// dA/dh = (h+_y - h-_y, h-_x - h+_x) / 2, dP/dh = t_in - t_out with unit edge
// vectors, a zero-length edge contributing 0): stored (!MOVE), or the Eq. 4
// move into the other buffer, re-quantised and wrapped (MOVE)
template <bool MOVE>
__global__ __launch_bounds__(256) void k_avm_force(AvmArrays a, const AvmParam* __restrict__ pp, AvmState* st)
{
#pragma clang fp contract(off)
    if (st->halt) return;
    const AvmParam& P = *pp;
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= a.nv) return;
    const double hx = a.x[v], hy = a.y[v];
    int n[3], c[3];
    double dx[3], dy[3], il[3];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        n[k] = a.vv[3 * v + k];
        c[k] = a.vc[3 * v + k];
    }
#pragma unroll
    for (int k = 0; k < 3; k++) {
        dx[k] = mimg(a.x[n[k]] - hx, P.Lx, P.hLx);
        dy[k] = mimg(a.y[n[k]] - hy, P.Ly, P.hLy);
        const double l2 = dx[k] * dx[k] + dy[k] * dy[k];
        il[k] = l2 > 0.0 ? 1.0 / sqrt(l2) : 0.0;
    }
    double fx = 0.0, fy = 0.0, sx = 0.0, sy = 0.0;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const int s = k, p = (k + 1) % 3;  // successor and predecessor of v in cell c[k]
        const double dAx = 0.5 * (dy[s] - dy[p]), dAy = 0.5 * (dx[p] - dx[s]);
        const double dPx = -dx[p] * il[p] - dx[s] * il[s], dPy = -dy[p] * il[p] - dy[s] * il[s];
        const double ca = a.ca[c[k]], cb = a.cb[c[k]];
        fx -= ca * dAx + cb * dPx;
        fy -= ca * dAy + cb * dPy;
        if (MOVE) {
            double sn, cs;
            sincos(a.th[c[k]], &sn, &cs);
            sx += cs;
            sy += sn;
        }
    }
    if (!MOVE) {
        a.fx[v] = fx;
        a.fy[v] = fy;
        return;
    }
    const double nx = hx + P.dt * (P.mu * fx + P.v0 * sx / 3.0);
    const double ny = hy + P.dt * (P.mu * fy + P.v0 * sy / 3.0);
    double X = avm_wrap(rint(nx * P.scale), P.LXu), Y = avm_wrap(rint(ny * P.scale), P.LYu);
    if (!(X >= 0.0 && X < P.LXu && Y >= 0.0 && Y < P.LYu)) {
        atomicOr(&st->err, ERR_NONFINITE);
        X = rint(hx * P.scale);
        Y = rint(hy * P.scale);
    }
    a.xo[v] = X * P.inv_scale;
    a.yo[v] = Y * P.inv_scale;
}

// T1 round r, first pass, for vertex v: its qualifying edges (each handled
// by its smaller-label end) and, per cell, the smallest key among them.  A
// vertex with a short edge (qualifying or not) is examined again in round
// r + 1, and so are the six vertices of every flip (apply), so that rounds
// >= 1 visit only those: no other edge can qualify there, since positions
// move only at flips and every other change of eligibility (a cell's vertex
// count, the end cells' shared vertices) touches edges that were already
// short.  The locks this vertex's candidate edges took in round r - 1 are
// released here (in the set round r + 1 uses).
__device__ __forceinline__ bool avm_mark_vertex(const AvmArrays& a, const AvmParam& P, AvmState* st, int r, int v,
                                                long long* lock, long long* prev)
{
#pragma clang fp contract(off)
    if (r > 0) {
        const unsigned old = a.cand[v];
        for (int k = 0; k < 3; k++)
            if (old & (1u << k))
                for (int j = 0; j < 4; j++) prev[a.lcell[12 * v + 4 * k + j]] = 0x7fffffffffffffffll;
    }
    unsigned mask = 0;
    bool shortedge = false;
    const double xv = a.x[v], yv = a.y[v];
    int tv = -1;
    for (int k = 0; k < 3; k++) {
        const int u = a.vv[3 * v + k];
        const double ex = mimg(a.x[u] - xv, P.Lx, P.hLx), ey = mimg(a.y[u] - yv, P.Ly, P.hLy);
        const double xx = ex * ex, yy = ey * ey;
        if (!(xx + yy < P.lt1sq)) continue;
        shortedge = true;
        if (tv < 0) tv = a.vtag[v];
        const int tu = a.vtag[u];
        if (tu < tv) continue;  // the other end handles it
        const int X = a.vc[3 * v + k], C1 = a.vc[3 * v + (k + 1) % 3], Y = a.vc[3 * v + (k + 2) % 3];
        int q = 0;
        while (q < 3 && a.vv[3 * u + q] != v) q++;
        if (q == 3) {
            atomicOr(&st->err, ERR_REPAIR);
            continue;
        }
        const int D1 = a.vc[3 * u + (q + 1) % 3];
        if (a.cdeg[X] <= 3 || a.cdeg[Y] <= 3 || C1 == D1) continue;
        bool share = false;
        const int* l1 = a.cv + (size_t)C1 * AVM_KV;
        const int* l2 = a.cv + (size_t)D1 * AVM_KV;
        for (int i = 0; i < a.cdeg[C1] && !share; i++)
            for (int j = 0; j < a.cdeg[D1]; j++)
                if (l1[i] == l2[j]) share = true;
        if (share) continue;
        const long long key = ((long long)tv << 32) | (long long)tu;
        atomicMin(&lock[X], key);
        atomicMin(&lock[Y], key);
        atomicMin(&lock[C1], key);
        atomicMin(&lock[D1], key);
        int* lc = a.lcell + 12 * v + 4 * k;
        lc[0] = X;
        lc[1] = Y;
        lc[2] = C1;
        lc[3] = D1;
        mask |= 1u << k;
    }
    a.cand[v] = (uint8_t)mask;
    a.dirty[v] = shortedge ? (uint8_t)(r + 1) : (uint8_t)0;  // examined: no stale flag stays behind
    return mask != 0;
}

// Round 0 visits every vertex (one per thread) and rotates the directors
// (after the move, with the step's counter).  Rounds >= 1 visit the
// vertices flagged for them (eight flags per thread).  CHECK: the pass after
// the device's rounds, which halts the batch when it still finds an edge.
// HOST: a round run from the host for a halted step.
__global__ __launch_bounds__(256) void k_avm_t1_mark(AvmArrays a, const AvmParam* __restrict__ pp, AvmState* st,
                                                     int r, int host, int check)
{
    if (!host && st->halt) return;
    const AvmParam& P = *pp;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    long long* lock = a.lock[r & 1];
    long long* prev = a.lock[(r + 1) & 1];
    bool found = false;
    if (r == 0) {
        if (t < a.nc) a.th[t] += P.amp * normal_for(P.seed, st->step, (uint64_t)a.ctag[t]);
        if (t < a.nv) found = avm_mark_vertex(a, P, st, 0, t, lock, prev);
    } else {
        if (!st->any[r - 1]) return;  // nothing flipped in the last round: nothing new qualifies
        // vertices t, t + S, ..., t + 7 S: flagged vertices sit together in
        // memory (neighbours of the same flips), so that consecutive ones go
        // to different threads; the eight flags are read before any work
        const int S = (a.nv + 7) >> 3;
        if (t >= S) return;
        uint8_t f[8];
#pragma unroll
        for (int j = 0; j < 8; j++) f[j] = t + j * S < a.nv ? a.dirty[t + j * S] : (uint8_t)0;
#pragma unroll
        for (int j = 0; j < 8; j++)
            if (f[j] == r) found |= avm_mark_vertex(a, P, st, r, t + j * S, lock, prev);
    }
    if (found) {
        st->any[r] = 1;
        if (check) st->halt = 1;
    }
}

__device__ __forceinline__ void cell_remove(int* l, uint8_t* deg, int w)
{
    const int k = *deg;
    int j = 0;
    for (int i = 0; i < k; i++)
        if (l[i] != w) l[j++] = l[i];
    *deg = (uint8_t)j;
}

// insert w just before v in the list (false when the list is full)
__device__ __forceinline__ bool cell_insert_before(int* l, uint8_t* deg, int v, int w)
{
    const int k = *deg;
    if (k >= AVM_KV) return false;
    int i = 0;
    while (i < k && l[i] != v) i++;
    for (int j = k; j > i; j--) l[j] = l[j - 1];
    l[i] = w;
    *deg = (uint8_t)(k + 1);
    return true;
}

// The same two edits on a list held in registers (all indices constant after
// unrolling): loaded and stored as four 16-byte words, so that a flip's four
// cell lists cost one round trip instead of a dependent walk each.
__device__ __forceinline__ void row_load(const int* p, int (&r)[AVM_KV])
{
    const int4* q = reinterpret_cast<const int4*>(p);
#pragma unroll
    for (int v = 0; v < AVM_KV / 4; v++) {
        const int4 w = q[v];
        r[4 * v] = w.x;
        r[4 * v + 1] = w.y;
        r[4 * v + 2] = w.z;
        r[4 * v + 3] = w.w;
    }
}

__device__ __forceinline__ void row_store(int* p, const int (&r)[AVM_KV])
{
    int4* q = reinterpret_cast<int4*>(p);
#pragma unroll
    for (int v = 0; v < AVM_KV / 4; v++) q[v] = make_int4(r[4 * v], r[4 * v + 1], r[4 * v + 2], r[4 * v + 3]);
}

// remove the one entry w among the first k; returns the new length
__device__ __forceinline__ int row_remove(int (&r)[AVM_KV], int k, int w)
{
    int pos = AVM_KV;
#pragma unroll
    for (int i = AVM_KV - 1; i >= 0; i--)
        if (i < k && r[i] == w) pos = i;
#pragma unroll
    for (int i = 0; i + 1 < AVM_KV; i++)
        if (i >= pos) r[i] = r[i + 1];
    return pos < k ? k - 1 : k;
}

// insert w just before v (at the end when v is absent); k < AVM_KV
__device__ __forceinline__ void row_insert_before(int (&r)[AVM_KV], int k, int v, int w)
{
    int pos = k;
#pragma unroll
    for (int i = AVM_KV - 1; i >= 0; i--)
        if (i < k && r[i] == v) pos = i;
#pragma unroll
    for (int i = AVM_KV - 1; i > 0; i--)
        if (i > pos) r[i] = r[i - 1];
#pragma unroll
    for (int i = 0; i < AVM_KV; i++)
        if (i == pos) r[i] = w;
}

// T1 round r, second pass for vertex v: an edge whose key holds all four of
// its cells flips (such edges share no cell and no vertex)
__device__ __forceinline__ void avm_apply_vertex(const AvmArrays& a, const AvmParam& P, AvmState* st, int r, int v,
                                                 unsigned mask)
{
#pragma clang fp contract(off)
    const long long* lock = a.lock[r & 1];
    for (int k = 0; k < 3; k++) {
        if (!(mask & (1u << k))) continue;
        const int u = a.vv[3 * v + k];
        const long long key = ((long long)a.vtag[v] << 32) | (long long)a.vtag[u];
        const int X = a.vc[3 * v + k], C1 = a.vc[3 * v + (k + 1) % 3], Y = a.vc[3 * v + (k + 2) % 3];
        int q = 0;
        while (q < 3 && a.vv[3 * u + q] != v) q++;
        const int D1 = a.vc[3 * u + (q + 1) % 3];
        if (lock[X] != key || lock[Y] != key || lock[C1] != key || lock[D1] != key) continue;
        // neighbours: around v (v2 = u, a_, b_), around u (v, c_, d_)
        const int an = a.vv[3 * v + (k + 1) % 3], bn = a.vv[3 * v + (k + 2) % 3];
        const int cn = a.vv[3 * u + (q + 1) % 3], dn = a.vv[3 * u + (q + 2) % 3];
        // geometry: the perpendicular through the midpoint, v (the smaller
        // label) on X's side
        const double ex = mimg(a.x[u] - a.x[v], P.Lx, P.hLx), ey = mimg(a.y[u] - a.y[v], P.Ly, P.hLy);
        const double mx = a.x[v] + 0.5 * ex, my = a.y[v] + 0.5 * ey;
        const double len = sqrt(ex * ex + ey * ey);
        const double rx = -ey / len, ry = ex / len;
        const double h = 0.5 * P.lnew;
        a.x[v] = avm_wrap(rint((mx + h * rx) * P.scale), P.LXu) * P.inv_scale;
        a.y[v] = avm_wrap(rint((my + h * ry) * P.scale), P.LYu) * P.inv_scale;
        a.x[u] = avm_wrap(rint((mx - h * rx) * P.scale), P.LXu) * P.inv_scale;
        a.y[u] = avm_wrap(rint((my - h * ry) * P.scale), P.LYu) * P.inv_scale;
        // topology: v keeps a_ and takes d_, u keeps c_ and takes b_
        a.vv[3 * v + 0] = dn;
        a.vv[3 * v + 1] = an;
        a.vv[3 * v + 2] = u;
        a.vc[3 * v + 0] = X;
        a.vc[3 * v + 1] = C1;
        a.vc[3 * v + 2] = D1;
        a.vv[3 * u + 0] = bn;
        a.vv[3 * u + 1] = cn;
        a.vv[3 * u + 2] = v;
        a.vc[3 * u + 0] = Y;
        a.vc[3 * u + 1] = D1;
        a.vc[3 * u + 2] = C1;
        for (int j = 0; j < 3; j++) {
            if (a.vv[3 * bn + j] == v) a.vv[3 * bn + j] = u;
            if (a.vv[3 * dn + j] == u) a.vv[3 * dn + j] = v;
        }
        if (X != Y && X != C1 && X != D1 && Y != C1 && Y != D1) {
            // four distinct lists (always, unless a cell meets itself):
            // all loaded together, edited in registers, stored
            int lX[AVM_KV], lY[AVM_KV], lC[AVM_KV], lD[AVM_KV];
            row_load(a.cv + (size_t)X * AVM_KV, lX);
            row_load(a.cv + (size_t)Y * AVM_KV, lY);
            row_load(a.cv + (size_t)C1 * AVM_KV, lC);
            row_load(a.cv + (size_t)D1 * AVM_KV, lD);
            const int kX = a.cdeg[X], kY = a.cdeg[Y], kC = a.cdeg[C1], kD = a.cdeg[D1];
            a.cdeg[X] = (uint8_t)row_remove(lX, kX, u);
            a.cdeg[Y] = (uint8_t)row_remove(lY, kY, v);
            row_store(a.cv + (size_t)X * AVM_KV, lX);
            row_store(a.cv + (size_t)Y * AVM_KV, lY);
            if (kC < AVM_KV && kD < AVM_KV) {
                row_insert_before(lC, kC, v, u);
                row_insert_before(lD, kD, u, v);
                a.cdeg[C1] = (uint8_t)(kC + 1);
                a.cdeg[D1] = (uint8_t)(kD + 1);
                row_store(a.cv + (size_t)C1 * AVM_KV, lC);
                row_store(a.cv + (size_t)D1 * AVM_KV, lD);
            } else {
                atomicOr(&st->err, ERR_CAPACITY);
            }
        } else {
            cell_remove(a.cv + (size_t)X * AVM_KV, a.cdeg + X, u);
            cell_remove(a.cv + (size_t)Y * AVM_KV, a.cdeg + Y, v);
            const bool ok1 = cell_insert_before(a.cv + (size_t)C1 * AVM_KV, a.cdeg + C1, v, u);
            const bool ok2 = cell_insert_before(a.cv + (size_t)D1 * AVM_KV, a.cdeg + D1, u, v);
            if (!ok1 || !ok2) atomicOr(&st->err, ERR_CAPACITY);
        }
        // every edge at the moved vertices changed: examine them next round
        const uint8_t nr = (uint8_t)(r + 1);
        a.dirty[v] = a.dirty[u] = a.dirty[an] = a.dirty[bn] = a.dirty[cn] = a.dirty[dn] = nr;
        atomicAdd(&st->t1, 1ull);
        break;
    }
}

// T1 round r, second pass: eight candidate masks per thread; round 0 counts
// the step
__global__ __launch_bounds__(256) void k_avm_t1_apply(AvmArrays a, const AvmParam* __restrict__ pp, AvmState* st,
                                                      int r, int host)
{
    if (!host && st->halt) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (r == 0 && t == 0) st->step += 1ull;  // the step's noise is drawn
    if (!st->any[r]) return;
    if (t == 0) atomicAdd(&st->rounds, 1ull);
    // vertices t, t + S, ..., t + 7 S (conflicting candidates sit together
    // in memory: spread over threads), the eight masks read first
    const int S = (a.nv + 7) >> 3;
    if (t >= S) return;
    uint8_t m8[8];
    unsigned any = 0;
#pragma unroll
    for (int j = 0; j < 8; j++) {
        m8[j] = t + j * S < a.nv ? a.cand[t + j * S] : (uint8_t)0;
        any |= m8[j];
    }
    if (!any) return;
    const AvmParam& P = *pp;
#pragma unroll 1
    for (int j = 0; j < 8; j++)
        if (m8[j]) avm_apply_vertex(a, P, st, r, t + j * S, m8[j]);
}

// ---------------------------------------------------------------- spatial re-sort
// Vertices by their position's bin, cells by their first vertex's bin, the
// bins ranked along a Hilbert curve (or row by row): a counting sort (keys
// and counts, a scan of the counts, a scatter, then each bin's few entries
// ordered by label so the order is deterministic), then every array
// gathered into its new slot with vertex and cell indices renamed.
struct AvmBins {
    double bsx, bsy;                    // bin sides
    int nbx, nby, nb;
    const int* rank;                    // rank of bin (by * nbx + bx) along the curve
};

__device__ __forceinline__ int avm_bin_rank(const AvmBins& b, double x, double y)
{
    const int bx = min((int)(x / b.bsx), b.nbx - 1), by = min((int)(y / b.bsy), b.nby - 1);
    return b.rank[by * b.nbx + bx];
}

__global__ __launch_bounds__(256) void k_avm_keys(AvmArrays a, AvmBins b, int* vkey, int* vcount, int* ckey,
                                                  int* ccount)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < a.nv) {
        const int k = avm_bin_rank(b, a.x[t], a.y[t]);
        vkey[t] = k;
        atomicAdd(&vcount[k], 1);
    }
    if (t < a.nc) {
        const int v0 = a.cv[(size_t)t * AVM_KV];
        const int k = avm_bin_rank(b, a.x[v0], a.y[v0]);
        ckey[t] = k;
        atomicAdd(&ccount[k], 1);
    }
}

// slot of every entry within its bin's range (start: exclusive scan of the
// counts; fill: zeroed counts)
__global__ __launch_bounds__(256) void k_avm_scatter(const int* vkey, const int* vstart, int* vfill, int* vperm,
                                                     const int* ckey, const int* cstart, int* cfill, int* cperm,
                                                     int nv, int nc)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nv) {
        const int k = vkey[t];
        vperm[vstart[k] + atomicAdd(&vfill[k], 1)] = t;
    }
    if (t < nc) {
        const int k = ckey[t];
        cperm[cstart[k] + atomicAdd(&cfill[k], 1)] = t;
    }
}

// each bin's entries by label, their inverse permutation, and the bin's fill
// counter back to zero for the next sort
__global__ __launch_bounds__(256) void k_avm_bin_order(const int* start, int* fill, int* perm, int* inv,
                                                       const int* tag, int nb)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int s = start[b], e = start[b + 1];
    for (int i = s + 1; i < e; i++) {
        const int x = perm[i], tx = tag[x];
        int j = i - 1;
        while (j >= s && tag[perm[j]] > tx) {
            perm[j + 1] = perm[j];
            j--;
        }
        perm[j + 1] = x;
    }
    for (int i = s; i < e; i++) inv[perm[i]] = i;
    fill[b] = 0;
}

// new slot t holds old vertex vperm[t] / old cell cperm[t]
__global__ __launch_bounds__(256) void k_avm_gather(AvmArrays src, AvmArrays dst, const int* __restrict__ vperm,
                                                   const int* __restrict__ vinv, const int* __restrict__ cperm,
                                                   const int* __restrict__ cinv)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < src.nv) {
        const int i = vperm[t];
        dst.x[t] = src.x[i];
        dst.y[t] = src.y[i];
        dst.vtag[t] = src.vtag[i];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            dst.vv[3 * t + k] = vinv[src.vv[3 * i + k]];
            dst.vc[3 * t + k] = cinv[src.vc[3 * i + k]];
        }
    }
    if (t < src.nc) {
        const int c = cperm[t];
        const int k = src.cdeg[c];
        dst.cdeg[t] = (uint8_t)k;
        for (int m = 0; m < k; m++) dst.cv[(size_t)t * AVM_KV + m] = vinv[src.cv[(size_t)c * AVM_KV + m]];
        dst.th[t] = src.th[c];
        dst.A0[t] = src.A0[c];
        dst.P0[t] = src.P0[c];
        dst.ctag[t] = src.ctag[c];
    }
}

// per-slot values into label order
__global__ void k_avm_by_label(const double* __restrict__ in, const int* __restrict__ tag, double* __restrict__ out,
                               int n)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[tag[t]] = in[t];
}

__global__ void k_avm_iota(int* a, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = i;
}

// host rounds finished: the next step may run
__global__ void k_avm_resume(AvmState* st)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) st->halt = 0;
}

// initial directors: 2 pi u, u from Philox counter (2^64 - 1, cell label);
// at creation slots and labels coincide
__global__ void k_avm_theta0(double* th, uint64_t seed, int n)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    uint64_t r[4];
    philox4x64(~0ull, (uint64_t)c, 0, 0, seed, 0, r);
    th[c] = 2.0 * 3.14159265358979323846 * u01(r[0]);
}

__global__ void k_avm_fill_lock(long long* a, long long* b, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = b[i] = 0x7fffffffffffffffll;
}

}  // namespace spv
