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
// of the three cells); director rotation; then T1 rounds (Sec. II.D): an
// edge shorter than l_T1 is replaced by its perpendicular of length l_new
// through the same midpoint and the cells at its ends become neighbours, at
// most one transition per cell in a round (an edge flips when its key is the
// smallest key of the qualifying edges at each of its four cells), rounds
// repeated until none qualifies.  Vertices live on the dyadic grid 2^-q
// (re-quantised after every move), so edge lengths are exact differences
// and the T1 test dx*dx + dy*dy < l_T1^2 (no fused operations) decides the
// same way on any implementation that follows it.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spv_common.hpp"

namespace spv {

constexpr int AVM_KV = 16;           // most vertices of a cell
constexpr int AVM_DEV_ROUNDS = 2;    // T1 rounds per step on the device
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
    int halt;                           // a step's last device round still flipped: later kernels wait
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
    uint8_t* cand;
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

// cell geometry; block 0 also clears the step's round flags
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
    const int* v = a.cv + (size_t)c * AVM_KV;
    const double x0 = a.x[v[0]], y0 = a.y[v[0]];
    double px = 0.0, py = 0.0, a2 = 0.0, per = 0.0;
    for (int m = 1; m <= k; m++) {
        double qx = 0.0, qy = 0.0;
        if (m < k) {
            qx = mimg(a.x[v[m]] - x0, P.Lx, P.hLx);
            qy = mimg(a.y[v[m]] - y0, P.Ly, P.hLy);
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
// vectors, a zero-length edge contributing 0); MOVE: then Eq. 4 into the
// other buffer, re-quantised and wrapped
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
    a.fx[v] = fx;
    a.fy[v] = fy;
    if (!MOVE) return;
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

// directors rotate (after the move; the step is counted by the next kernel)
__global__ __launch_bounds__(256) void k_avm_theta(AvmArrays a, const AvmParam* __restrict__ pp, AvmState* st)
{
    if (st->halt) return;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < a.nc) a.th[c] += pp->amp * normal_for(pp->seed, st->step, (uint64_t)c);
}

// T1 round r, first pass: the qualifying edges (owned by their smaller
// vertex) and, per cell, the smallest key among them
__global__ __launch_bounds__(256) void k_avm_t1_mark(AvmArrays a, const AvmParam* __restrict__ pp, AvmState* st,
                                                     int r)
{
#pragma clang fp contract(off)
    if (st->halt && r < AVM_DEV_ROUNDS) return;
    if (r == 0 && blockIdx.x == 0 && threadIdx.x == 0) st->step += 1ull;  // the step's noise is drawn
    if (r > 0 && !st->any[r - 1]) return;  // nothing flipped in the last round: nothing new qualifies
    const AvmParam& P = *pp;
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= a.nv) return;
    unsigned mask = 0;
    long long* lock = a.lock[r & 1];
    for (int k = 0; k < 3; k++) {
        const int u = a.vv[3 * v + k];
        if (u <= v) continue;
        const double ex = mimg(a.x[u] - a.x[v], P.Lx, P.hLx), ey = mimg(a.y[u] - a.y[v], P.Ly, P.hLy);
        const double xx = ex * ex, yy = ey * ey;
        if (!(xx + yy < P.lt1sq)) continue;
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
        const long long key = ((long long)v << 32) | (long long)u;
        atomicMin(&lock[X], key);
        atomicMin(&lock[Y], key);
        atomicMin(&lock[C1], key);
        atomicMin(&lock[D1], key);
        mask |= 1u << k;
    }
    a.cand[v] = (uint8_t)mask;
    if (mask) st->any[r] = 1;
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

// T1 round r, second pass: an edge whose key holds all four of its cells
// flips (such edges share no cell and no vertex); every thread also clears
// the next round's locks in its range
__global__ __launch_bounds__(256) void k_avm_t1_apply(AvmArrays a, const AvmParam* __restrict__ pp, AvmState* st,
                                                      int r, int last)
{
#pragma clang fp contract(off)
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < a.nc) a.lock[(r + 1) & 1][t] = 0x7fffffffffffffffll;
    if (st->halt && r < AVM_DEV_ROUNDS) return;
    if (!st->any[r]) return;
    if (t == 0) {
        atomicAdd(&st->rounds, 1ull);
        // the step's last device round flipped: later rounds may be needed
        // before the next step (the host runs them)
        if (last) st->halt = 1;
    }
    if (t >= a.nv) return;
    const int v = t;
    const unsigned mask = a.cand[v];
    if (!mask) return;
    const AvmParam& P = *pp;
    const long long* lock = a.lock[r & 1];
    for (int k = 0; k < 3; k++) {
        if (!(mask & (1u << k))) continue;
        const int u = a.vv[3 * v + k];
        const long long key = ((long long)v << 32) | (long long)u;
        const int X = a.vc[3 * v + k], C1 = a.vc[3 * v + (k + 1) % 3], Y = a.vc[3 * v + (k + 2) % 3];
        int q = 0;
        while (q < 3 && a.vv[3 * u + q] != v) q++;
        const int D1 = a.vc[3 * u + (q + 1) % 3];
        if (lock[X] != key || lock[Y] != key || lock[C1] != key || lock[D1] != key) continue;
        // neighbours: around v (v2 = u, a_, b_), around u (v, c_, d_)
        const int an = a.vv[3 * v + (k + 1) % 3], bn = a.vv[3 * v + (k + 2) % 3];
        const int cn = a.vv[3 * u + (q + 1) % 3], dn = a.vv[3 * u + (q + 2) % 3];
        // geometry: the perpendicular through the midpoint, v on X's side
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
        cell_remove(a.cv + (size_t)X * AVM_KV, a.cdeg + X, u);
        cell_remove(a.cv + (size_t)Y * AVM_KV, a.cdeg + Y, v);
        const bool ok1 = cell_insert_before(a.cv + (size_t)C1 * AVM_KV, a.cdeg + C1, v, u);
        const bool ok2 = cell_insert_before(a.cv + (size_t)D1 * AVM_KV, a.cdeg + D1, u, v);
        if (!ok1 || !ok2) atomicOr(&st->err, ERR_CAPACITY);
        atomicAdd(&st->t1, 1ull);
        break;
    }
}

// host rounds finished: the next step may run
__global__ void k_avm_resume(AvmState* st)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) st->halt = 0;
}

// initial directors: 2 pi u, u from Philox counter (2^64 - 1, cell)
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
