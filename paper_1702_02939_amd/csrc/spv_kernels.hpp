// spv_kernels.hpp -- HIP kernels of the SPV step on gfx950.
//
// One step (Sussman 2017, Sec. II.C) is
//   force+update   F_i = -dE/dr_i by the App. B chain rule through the Voronoi
//                  vertices, then r_i += dt (mu F_i + v0 n_i) (Eq. 3) and the
//                  director turns by sqrt(2 Dr dt) xi (Sec. II.A);
//   geometry+test  Voronoi area / perimeter of every cell (Sec. II.C.1) fused
//                  with the empty-circumcircle test of its ring (Sec. II.C.3);
//   repair rounds  flagged rings rebuilt on the device from the candidate
//                  neighbours inside a search disk (locality lemma, Sec.
//                  II.C.4) by exact gift-wrapping, then the touched cells get
//                  their opposite vertices rebuilt and are re-tested; repeated
//                  until no flag is raised (cf. the repeat-until-no-change rule
//                  of Sec. II.D).
// Streaming passes use GL = 8 lanes per cell: lane l handles ring slots
// l, l + 8, ...; per-slot values (displacements, Voronoi vertices, unit edge
// vectors, neighbour coefficients) are staged in LDS so that a slot can read
// its ring neighbours m +- 1 for any ring length.  Rings are cell-major
// [N][KC]; a cell's 8 lanes read one contiguous 32-byte row segment.
// Every kernel first checks the device halt flag, so that a step whose
// repair did not converge turns the rest of a captured graph into no-ops.
#pragma once
#include "spv_common.hpp"
#include "spv_exact.hpp"

namespace spv {

constexpr int GL = 8;          // lanes per cell in the streaming kernels
constexpr int CPB = 256 / GL;  // cells per 256-thread block
constexpr int RP_CAP = 1024;   // max candidate neighbours of one repaired cell

// ---------------------------------------------------------------- helpers

template <typename R>
__device__ __forceinline__ void circumcentre(R bx, R by, R cx, R cy, R& ux, R& uy)
{
    const R nb = bx * bx + by * by, nc = cx * cx + cy * cy;
    const R inv = R(0.5) / (bx * cy - by * cx);
    ux = (cy * nb - by * nc) * inv;
    uy = (bx * nc - cx * nb) * inv;
}

template <typename R>
__device__ __forceinline__ void unit(R ex, R ey, R& tx, R& ty)
{
    const R l2 = ex * ex + ey * ey;
    if (l2 > R(0)) {
        const R r = R(1) / sqrt(l2);
        tx = ex * r;
        ty = ey * r;
    } else {  // zero-length Voronoi edge (exact T1 configuration)
        tx = ty = R(0);
    }
}

// In-circle with lazily loaded tags (the tie-break almost never runs).
__device__ __forceinline__ int incircle_tags(double bx, double by, double cx, double cy, double px, double py,
                                             const int* tag, int gi, int gb, int gc, int gp, double scale,
                                             int* exact_count)
{
    const double nb = bx * bx + by * by, nc = cx * cx + cy * cy, np = px * px + py * py;
    const double t1 = cx * py, t2 = cy * px, t3 = px * by, t4 = py * bx, t5 = bx * cy, t6 = by * cx;
    const double det = nb * (t1 - t2) + nc * (t3 - t4) + np * (t5 - t6);
    const double perm = nb * (fabs(t1) + fabs(t2)) + nc * (fabs(t3) + fabs(t4)) + np * (fabs(t5) + fabs(t6));
    const double bound = 2.0e-15 * perm;
    if (det > bound) return -1;
    if (det < -bound) return 1;
    return incircle_sos(bx, by, cx, cy, px, py, tag[gi], tag[gb], tag[gc], tag[gp], scale, exact_count);
}

// append c to the repair worklist of round r (once per round)
__device__ __forceinline__ void push_flag(const Work& w, DevState* st, int r, int c)
{
    const unsigned bit = 1u << (c & 31);
    if (!(atomicOr(&w.flagbits[c >> 5], bit) & bit)) {
        const int slot = atomicAdd(&st->wl_count[r], 1);
        w.wl[r & 1][slot] = c;
    }
}

// append c to the touched list of round r (once per round)
__device__ __forceinline__ void push_touch(const Work& w, DevState* st, int r, int c)
{
    const unsigned bit = 1u << (c & 31);
    if (!(atomicOr(&w.touchbits[c >> 5], bit) & bit)) {
        const int slot = atomicAdd(&st->tl_count[r], 1);
        w.tl[r & 1][slot] = c;
    }
}

// XCD-aware block order: the 8 XCDs receive consecutive workgroups in turn;
// remap so that each XCD works on one contiguous range of cells (neighbour
// gathers then hit that XCD's L2).  The grid is padded to a multiple of 8.
__device__ __forceinline__ int xcd_block(int b, int grid)
{
    const int per = grid >> 3;
    return (b & 7) * per + (b >> 3);
}

// ---------------------------------------------------------------- force (+ update)
// Vertex h_m (circumcentre of i, j_m, j_{m+1}, frame of i) is shared by cells
// i, j_m, j_{m+1}; its neighbours in those polygons are h_{m-1}, h_{m+1} and
// h'_m = circumcentre(j_m, opp_m, j_{m+1}).  With unit edge vectors
//   t1 = (h_m - h_{m-1})/|.|, t2 = (h_{m+1} - h_m)/|.|, t3 = (h'_m - h_m)/|.|
// the vertex gradient of E (App. A; perimeter term incoming minus outgoing) is
//   g_m = a_i dA_i + b_i (t1 - t2) + a_jm dA_jm + b_jm (t1 - t3)
//       + a_jn dA_jn + b_jn (-t2 - t3),
// dA_c = 1/2 (h+_y - h-_y, h-_x - h+_x) for the CCW neighbours (h-, h+) of h_m
// in cell c, and F_i = -sum_m J_m^T g_m with the circumcentre Jacobian of
// App. B (Eq. B4), read with s = b x c in the denominator and its gradient.
template <typename R, bool MULTI, int KC, bool UPDATE>
__global__ __launch_bounds__(256) void k_force(Cells<R> c, double* __restrict__ xo, double* __restrict__ yo,
                                               double* __restrict__ tho, double* __restrict__ fxo,
                                               double* __restrict__ fyo, const SysParam* __restrict__ sp,
                                               DevState* st, int N)
{
    constexpr int NS = KC / GL;
    __shared__ R sD[CPB][KC][2];  // displacement of ring cell m
    __shared__ R sH[CPB][KC][2];  // Voronoi vertex m
    __shared__ R sE[CPB][KC][2];  // unit edge vector h_m -> h_{m+1}
    __shared__ R sC[CPB][KC][2];  // (a, b) of ring cell m
    if (st->halt) return;
    const int g = threadIdx.x / GL, l = threadIdx.x % GL;
    const int i = xcd_block(blockIdx.x, gridDim.x) * CPB + g;
    const bool valid = i < N;
    const int ii = valid ? i : 0;
    const SysParam& P = sp[MULTI ? c.sys[ii] : 0];
    int k = valid ? c.deg[ii] : 0;
    if (k < 3 || k > KC) k = 0;  // reported by the validity test
    const double xi = c.x[ii], yi = c.y[ii];
    const R* __restrict__ ca = c.ca;
    const R* __restrict__ cb = c.cb;

    double dmx[NS], dmy[NS], odx[NS], ody[NS];
    bool hasopp[NS];
#pragma unroll
    for (int s = 0; s < NS; s++) {
        const int m = l + s * GL;
        dmx[s] = dmy[s] = odx[s] = ody[s] = 0.0;
        hasopp[s] = false;
        if (m < k) {
            const int j = c.ring[ii * KC + m];
            dmx[s] = mimg(c.x[j] - xi, P.Lx, P.hLx);
            dmy[s] = mimg(c.y[j] - yi, P.Ly, P.hLy);
            sD[g][m][0] = (R)dmx[s];
            sD[g][m][1] = (R)dmy[s];
            sC[g][m][0] = ca[j];
            sC[g][m][1] = cb[j];
            const int o = c.opp[ii * KC + m];
            if (o >= 0) {
                hasopp[s] = true;
                odx[s] = mimg(c.x[o] - xi, P.Lx, P.hLx);
                ody[s] = mimg(c.y[o] - yi, P.Ly, P.hLy);
            }
        }
    }
    __syncthreads();
    R hqx[NS], hqy[NS];
#pragma unroll
    for (int s = 0; s < NS; s++) {
        const int m = l + s * GL;
        hqx[s] = hqy[s] = R(0);
        if (m < k) {
            const int mn = (m + 1 == k) ? 0 : m + 1;
            const R bx = sD[g][m][0], by = sD[g][m][1], cx = sD[g][mn][0], cy = sD[g][mn][1];
            R hx, hy;
            circumcentre(bx, by, cx, cy, hx, hy);
            sH[g][m][0] = hx;
            sH[g][m][1] = hy;
            hqx[s] = hx;
            hqy[s] = hy;
            if (hasopp[s]) {
                // third vertex of edge (j_m, j_{m+1}): circumcentre of (j_m, opp_m, j_{m+1})
                const R ex = (R)(odx[s] - dmx[s]), ey = (R)(ody[s] - dmy[s]);
                R qx, qy;
                circumcentre(ex, ey, cx - bx, cy - by, qx, qy);
                hqx[s] = qx + bx;
                hqy[s] = qy + by;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < NS; s++) {
        const int m = l + s * GL;
        if (m < k) {
            const int mn = (m + 1 == k) ? 0 : m + 1;
            R tx, ty;
            unit(sH[g][mn][0] - sH[g][m][0], sH[g][mn][1] - sH[g][m][1], tx, ty);
            sE[g][m][0] = tx;
            sE[g][m][1] = ty;
        }
    }
    __syncthreads();
    R fx = R(0), fy = R(0);
    const R ai = valid ? ca[ii] : R(0), bi = valid ? cb[ii] : R(0);
#pragma unroll
    for (int s = 0; s < NS; s++) {
        const int m = l + s * GL;
        if (m < k) {
            const int mn = (m + 1 == k) ? 0 : m + 1, mp = (m == 0) ? k - 1 : m - 1;
            const R hpx = sH[g][mp][0], hpy = sH[g][mp][1];
            const R hcx = sH[g][m][0], hcy = sH[g][m][1];
            const R hnx = sH[g][mn][0], hny = sH[g][mn][1];
            const R t1x = sE[g][mp][0], t1y = sE[g][mp][1];
            const R t2x = sE[g][m][0], t2y = sE[g][m][1];
            R t3x, t3y;
            unit(hqx[s] - hcx, hqy[s] - hcy, t3x, t3y);
            const R am = sC[g][m][0], bm = sC[g][m][1], an = sC[g][mn][0], bn = sC[g][mn][1];
            const R qx = hqx[s], qy = hqy[s];
            R gx = ai * R(0.5) * (hny - hpy) + bi * (t1x - t2x);
            R gy = ai * R(0.5) * (hpx - hnx) + bi * (t1y - t2y);
            gx += am * R(0.5) * (hpy - qy) + bm * (t1x - t3x);
            gy += am * R(0.5) * (qx - hpx) + bm * (t1y - t3y);
            gx += an * R(0.5) * (qy - hny) + bn * (-t2x - t3x);
            gy += an * R(0.5) * (hnx - qx) + bn * (-t2y - t3y);
            // J_m^T g, b = d_m, c = d_{m+1}, e = c - b
            const R Bx = sD[g][m][0], By = sD[g][m][1], Cx = sD[g][mn][0], Cy = sD[g][mn][1];
            const R ex = Cx - Bx, ey = Cy - By;
            const R sc = Bx * Cy - By * Cx;
            const R be = Bx * ex + By * ey, ce = Cx * ex + Cy * ey;
            const R nb = Bx * Bx + By * By, nc = Cx * Cx + Cy * Cy;
            const R betaD = -nc * be, gammaD = nb * ce;
            const R zx = betaD * Bx + gammaD * Cx, zy = betaD * By + gammaD * Cy;
            const R gbx = R(2) * be * Cx + nc * ex, gby = R(2) * be * Cy + nc * ey;    // grad(beta D)
            const R ggx = R(-2) * ce * Bx - nb * ex, ggy = R(-2) * ce * By - nb * ey;  // grad(gamma D)
            const R is = R(1) / sc;
            const R gdx = R(2) * is * (-ey), gdy = R(2) * is * ex;                     // grad(D) / D
            const R invD = R(0.5) * is * is;                                           // 1 / (2 s^2)
            const R gB = gx * Bx + gy * By, gC = gx * Cx + gy * Cy, gZ = gx * zx + gy * zy;
            fx -= gx + invD * (gB * gbx + gC * ggx - (betaD + gammaD) * gx - gZ * gdx);
            fy -= gy + invD * (gB * gby + gC * ggy - (betaD + gammaD) * gy - gZ * gdy);
        }
    }
#pragma unroll
    for (int off = GL / 2; off > 0; off >>= 1) {
        fx += __shfl_xor(fx, off);
        fy += __shfl_xor(fy, off);
    }
    if (!UPDATE) {
        if (valid && l == 0) {
            fxo[i] = (double)fx;
            fyo[i] = (double)fy;
        }
        return;
    }
    double disp = 0.0;
    if (valid && l == 0) {
        const double th = c.th[i];
        double sn, cs;
        sincos(th, &sn, &cs);
        const double xn = xi + P.dt * (P.mu * (double)fx + P.v0 * cs);
        const double yn = yi + P.dt * (P.mu * (double)fy + P.v0 * sn);
        double X = rint(xn * P.scale), Y = rint(yn * P.scale);
        if (X < 0.0) X += P.LXu;
        else if (X >= P.LXu) X -= P.LXu;
        if (Y < 0.0) Y += P.LYu;
        else if (Y >= P.LYu) Y -= P.LYu;
        if (!(X >= 0.0 && X < P.LXu && Y >= 0.0 && Y < P.LYu)) {
            atomicOr(&st->err, ERR_NONFINITE);
            X = rint(xi * P.scale);  // keep the stored state finite and inside the box
            Y = rint(yi * P.scale);
        }
        const double xq = X * P.inv_scale, yq = Y * P.inv_scale;
        xo[i] = xq;
        yo[i] = yq;
        tho[i] = th + P.amp * normal_for(P.seed, st->step, (uint64_t)c.tag[i]);
        const double ddx = mimg(xq - xi, P.Lx, P.hLx), ddy = mimg(yq - yi, P.Ly, P.hLy);
        disp = sqrt(ddx * ddx + ddy * ddy);
    }
    unsigned long long b = __double_as_longlong(disp);
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(b, off);
        b = o > b ? o : b;
    }
    if ((threadIdx.x & 63) == 0 && b) atomicMax(&st->disp_bits, b);
}

// ---------------------------------------------------------------- geometry + validity test
// For cell i with CCW ring (j_0 .. j_{k-1}) and exact displacements d_m:
//   u_m = circumcentre(0, d_m, d_{m+1})      (Voronoi vertex, frame of i)
//   A_i = 1/2 sum u_m x u_{m+1},  P_i = sum |u_{m+1} - u_m|
// and the ring is valid when every (i, j_m, j_{m+1}) is counter-clockwise and
// the cell opp_m across edge (j_m, j_{m+1}) is not strictly inside its
// circumcircle (local Delaunay property of every edge).  The predicates use
// the exact FP64 displacements whatever R is.
// LIST: process the touched list of round `round` (clearing its bits) and
// push failures to round + 1; otherwise all cells, failures to round 0.
// OPP: rebuild opp first -- in the CCW ring of j_m the pattern
// ..., opp_m, j_{m+1}, i, ... must appear; otherwise the rings disagree and
// the cells are flagged.
template <typename R, bool MULTI, int KC, bool LIST, bool OPP>
__global__ __launch_bounds__(256) void k_geom(Cells<R> c, Work w, const SysParam* __restrict__ sp, DevState* st,
                                              int N, int round)
{
    constexpr int NS = KC / GL;
    __shared__ double sD[CPB][KC][2];
    __shared__ R sU[CPB][KC][2];
    __shared__ int sJ[CPB][KC];
    if (st->halt) return;
    const int g = threadIdx.x / GL, l = threadIdx.x % GL;
    const int n = LIST ? st->tl_count[round] : N;
    const int rnext = LIST ? round + 1 : 0;
    const int* __restrict__ list = w.tl[round & 1];
    const int bstart = LIST ? (int)blockIdx.x : xcd_block(blockIdx.x, gridDim.x);
    int exact = 0;
    for (int base = bstart * CPB; base < n; base += gridDim.x * CPB) {
        const int t = base + g;
        const bool valid = t < n;
        const int i = valid ? (LIST ? list[t] : t) : 0;
        if (LIST && valid && l == 0) atomicAnd(&w.touchbits[i >> 5], ~(1u << (i & 31)));
        const SysParam& P = sp[MULTI ? c.sys[i] : 0];
        int k = valid ? c.deg[i] : 0;
        if (valid && (k < 3 || k > KC)) {
            if (l == 0) atomicOr(&st->err, ERR_DEGREE);
            k = 0;
        }
        const double xi = c.x[i], yi = c.y[i];
#pragma unroll
        for (int s = 0; s < NS; s++) {
            const int m = l + s * GL;
            if (m < k) {
                const int j = c.ring[i * KC + m];
                sJ[g][m] = j;
                sD[g][m][0] = mimg(c.x[j] - xi, P.Lx, P.hLx);
                sD[g][m][1] = mimg(c.y[j] - yi, P.Ly, P.hLy);
            }
        }
        __syncthreads();
        const double rlim2 = 0.0625 * fmin(P.Lx, P.Ly) * fmin(P.Lx, P.Ly);
#pragma unroll
        for (int s = 0; s < NS; s++) {
            const int m = l + s * GL;
            if (m < k) {
                const int mn = (m + 1 == k) ? 0 : m + 1;
                const int jm = sJ[g][m], jn = sJ[g][mn];
                int o;
                if (OPP) {
                    o = -1;
                    const int kj = min((int)c.deg[jm], KC);
                    for (int p = 0; p < kj; p++) {
                        if (c.ring[jm * KC + p] == i) {
                            const int pm1 = (p == 0) ? kj - 1 : p - 1;
                            const int pm2 = (pm1 == 0) ? kj - 1 : pm1 - 1;
                            if (c.ring[jm * KC + pm1] == jn) o = c.ring[jm * KC + pm2];
                            break;
                        }
                    }
                    c.opp[i * KC + m] = o;
                } else {
                    o = c.opp[i * KC + m];
                }
                const double bx = sD[g][m][0], by = sD[g][m][1], cx = sD[g][mn][0], cy = sD[g][mn][1];
                bool fail = cross_sign(bx, by, cx, cy, bx * cy - by * cx, P.scale) <= 0;
                R ux, uy;
                circumcentre((R)bx, (R)by, (R)cx, (R)cy, ux, uy);
                if (!fail) {
                    if (o < 0) {
                        fail = true;
                    } else {
                        const double px = mimg(c.x[o] - xi, P.Lx, P.hLx), py = mimg(c.y[o] - yi, P.Ly, P.hLy);
                        fail = incircle_tags(bx, by, cx, cy, px, py, c.tag, i, jm, jn, o, P.scale, &exact) > 0;
                    }
                    // a circumradius >= min(L)/4 is either a non-Delaunay triangle
                    // or a true violation of the box precondition; the repair
                    // tells them apart (it cannot certify a disk wider than L/2)
                    if (!fail && (double)(ux * ux + uy * uy) >= rlim2) fail = true;
                }
                if (fail) {
                    push_flag(w, st, rnext, i);
                    push_flag(w, st, rnext, jm);
                    push_flag(w, st, rnext, jn);
                    if (o >= 0) push_flag(w, st, rnext, o);
                }
                sU[g][m][0] = ux;
                sU[g][m][1] = uy;
            }
        }
        __syncthreads();
        R a2 = R(0), per = R(0);
#pragma unroll
        for (int s = 0; s < NS; s++) {
            const int m = l + s * GL;
            if (m < k) {
                const int mn = (m + 1 == k) ? 0 : m + 1;
                const R ux = sU[g][m][0], uy = sU[g][m][1], vx = sU[g][mn][0], vy = sU[g][mn][1];
                a2 += ux * vy - uy * vx;
                per += sqrt((vx - ux) * (vx - ux) + (vy - uy) * (vy - uy));
            }
        }
#pragma unroll
        for (int off = GL / 2; off > 0; off >>= 1) {
            a2 += __shfl_xor(a2, off);
            per += __shfl_xor(per, off);
        }
        if (valid && l == 0 && k >= 3) {
            const R A = R(0.5) * a2;
            c.A[i] = A;
            c.P[i] = per;
            c.ca[i] = (R)(2.0 * P.KA * ((double)A - c.A0[i]));
            c.cb[i] = (R)(2.0 * P.KP * ((double)per - c.P0[i]));
        }
        __syncthreads();  // LDS is reused by the next group of cells
    }
    if (exact) atomicAdd(&st->exact_calls, (unsigned long long)exact);
}

// ---------------------------------------------------------------- repair
// One 64-lane wavefront rebuilds the Delaunay ring of one flagged cell i.
// Candidates: every cell of i's system within distance R, gathered from the
// bins of the last re-sort (searched with R + drift, drift bounding the
// motion since then).  The ring is traced counter-clockwise by gift-wrapping:
// from the nearest candidate (always a Delaunay neighbour) the next neighbour
// after c is the left-side candidate p whose circle through (i, c, p)
// contains no other left-side candidate -- an arg-min under the exact
// in-circle order, per lane and then across the wave.  The ring is certified
// when every new circumdisk lies inside the search disk (2 |u_m| <= R), which
// makes each new triangle empty with respect to all cells; otherwise R doubles.
template <typename R, bool MULTI, int KC>
__global__ __launch_bounds__(64) void k_repair(Cells<R> c, Work w, const SysParam* __restrict__ sp, DevState* st,
                                               int round)
{
    constexpr int KMAX = 64;
    __shared__ double sx[RP_CAP], sy[RP_CAP];
    __shared__ int sid[RP_CAP];
    __shared__ int s_n;
    __shared__ int s_ring[KMAX + 1];
    if (st->halt) return;
    const int lane = threadIdx.x;
    const int nw = st->wl_count[round];
    const int* __restrict__ wl = w.wl[round & 1];
    const double drift = st->drift;
    int exact = 0;
    for (int wi = blockIdx.x; wi < nw; wi += gridDim.x) {
        const int i = wl[wi];
        if (lane == 0) atomicAnd(&w.flagbits[i >> 5], ~(1u << (i & 31)));
        const SysParam& P = sp[MULTI ? c.sys[i] : 0];
        const double xi = c.x[i], yi = c.y[i];
        const int kold = min((int)c.deg[i], KC);
        const double Rmax = 0.5 * fmin(P.Lx, P.Ly) * (1.0 - 1e-9);
        double Rs = fmin(P.R0, Rmax);
        int k = 0;
        bool ok = false, at_max = false;
        int last_n = 0, last_closed = 0, attempts = 0;
        double last_umax = 0.0;
        for (int attempt = 0; attempt < 16 && !ok; attempt++) {
            attempts = attempt + 1;
            if (lane == 0) s_n = 0;
            __syncthreads();
            const double Rw = Rs + drift;
            int rbx = (int)ceil(Rw / P.bsx), rby = (int)ceil(Rw / P.bsy);
            int wx = 2 * rbx + 1, wy = 2 * rby + 1;
            const int cbx = min((int)(xi / P.bsx), P.nbx - 1), cby = min((int)(yi / P.bsy), P.nby - 1);
            int bx0 = cbx - rbx, by0 = cby - rby;
            if (wx >= P.nbx) {
                wx = P.nbx;
                bx0 = 0;
            }
            if (wy >= P.nby) {
                wy = P.nby;
                by0 = 0;
            }
            const double R2 = Rs * Rs * (1.0 + 1e-12);
            const int lo = P.cell_off, hi = P.cell_off + P.n;
            for (int b = lane; b < wx * wy; b += 64) {
                int bx = bx0 + b % wx, by = by0 + b / wx;
                bx = ((bx % P.nbx) + P.nbx) % P.nbx;
                by = ((by % P.nby) + P.nby) % P.nby;
                const int key = w.bin_key[P.bin_off + by * P.nbx + bx];
                const int c1 = min(w.bin_start[key + 1], hi);
                for (int q = max(w.bin_start[key], lo); q < c1; q++) {
                    if (q == i) continue;
                    const double dx = mimg(c.x[q] - xi, P.Lx, P.hLx), dy = mimg(c.y[q] - yi, P.Ly, P.hLy);
                    if (dx * dx + dy * dy <= R2) {
                        const int slot = atomicAdd(&s_n, 1);
                        if (slot < RP_CAP) {
                            sx[slot] = dx;
                            sy[slot] = dy;
                            sid[slot] = q;
                        }
                    }
                }
            }
            __syncthreads();
            const int n = s_n;
            last_n = n;
            if (n > RP_CAP) {
                if (lane == 0) atomicOr(&st->err, ERR_CAPACITY);
                break;
            }
            // nearest candidate: exact squared distance in grid units, ties by tag
            unsigned long long bh = ~0ull, bl = ~0ull;
            int best = -1;
            for (int q = lane; q < n; q += 64) {
                const __int128 X = to_units(sx[q], P.scale), Y = to_units(sy[q], P.scale);
                const unsigned __int128 d2 = (unsigned __int128)(X * X + Y * Y);
                const unsigned long long h = (unsigned long long)(d2 >> 64), lw = (unsigned long long)d2;
                if (best < 0 || h < bh || (h == bh && (lw < bl || (lw == bl && c.tag[sid[q]] < c.tag[sid[best]])))) {
                    bh = h;
                    bl = lw;
                    best = q;
                }
            }
            for (int off = 32; off >= 1; off >>= 1) {
                const unsigned long long oh = __shfl_xor(bh, off), ol = __shfl_xor(bl, off);
                const int ob = __shfl_xor(best, off);
                if (ob >= 0 && (best < 0 || oh < bh ||
                                (oh == bh && (ol < bl || (ol == bl && c.tag[sid[ob]] < c.tag[sid[best]]))))) {
                    bh = oh;
                    bl = ol;
                    best = ob;
                }
            }
            if (best < 0) {  // no candidate at all
                if (at_max) break;
                Rs = fmin(2.0 * Rs, Rmax);
                at_max = (Rs >= Rmax);
                continue;
            }
            const int start = best;
            if (lane == 0) s_ring[0] = start;
            k = 1;
            int cur = start;
            bool closed = false;
            while (k <= KMAX) {
                const double cx = sx[cur], cy = sy[cur];
                const int gc = sid[cur];
                int nb = -1;
                for (int q = lane; q < n; q += 64) {
                    if (q == cur) continue;
                    const double px = sx[q], py = sy[q];
                    if (cross_sign(cx, cy, px, py, cx * py - cy * px, P.scale) <= 0) continue;
                    if (nb < 0 || incircle_tags(cx, cy, sx[nb], sy[nb], px, py, c.tag, i, gc, sid[nb], sid[q],
                                                P.scale, &exact) > 0)
                        nb = q;
                }
                for (int off = 32; off >= 1; off >>= 1) {
                    const int ob = __shfl_xor(nb, off);
                    if (ob >= 0 && ob != nb &&
                        (nb < 0 || incircle_tags(cx, cy, sx[nb], sy[nb], sx[ob], sy[ob], c.tag, i, gc, sid[nb],
                                                 sid[ob], P.scale, &exact) > 0))
                        nb = ob;
                }
                if (nb < 0) break;  // star open: search disk too small
                if (nb == start) {
                    closed = true;
                    break;
                }
                if (lane == 0) s_ring[k] = nb;
                k++;
                cur = nb;
            }
            __syncthreads();
            double umax = 0.0;
            if (closed && k >= 3) {
                for (int m = lane; m < k; m += 64) {
                    const int p = s_ring[m], q = s_ring[(m + 1 == k) ? 0 : m + 1];
                    double ux, uy;
                    circumcentre(sx[p], sy[p], sx[q], sy[q], ux, uy);
                    umax = fmax(umax, sqrt(ux * ux + uy * uy));
                }
                for (int off = 32; off >= 1; off >>= 1) umax = fmax(umax, __shfl_xor(umax, off));
                if (2.0 * umax * (1.0 + 1e-9) <= Rs) ok = true;
            }
            last_closed = closed ? 1 : 0;
            last_umax = umax;
            if (!ok) {
                if (at_max) break;
                // an uncertified star may be wrong (outer triangles clipped by
                // the search disk), so its circumradii say nothing: double R
                Rs = fmin(2.0 * Rs, Rmax);
                at_max = (Rs >= Rmax);
                if (lane == 0) atomicAdd(&st->retries, 1ull);
            }
        }
        if (!ok || k > KC) {
            if (lane == 0) {
                atomicOr(&st->err, !ok ? (at_max ? ERR_PRECOND : ERR_REPAIR) : ERR_CAPACITY);
                if (atomicCAS(&st->fail_set, 0, 1) == 0) {
                    st->fail_cell = c.tag[i];
                    st->fail_n = last_n;
                    st->fail_k = k;
                    st->fail_closed = last_closed;
                    st->fail_attempts = attempts;
                    st->fail_R = Rs;
                    st->fail_umax = last_umax;
                }
            }
            __syncthreads();
            continue;
        }
        // canonical rotation: start at the smallest tag
        int mt = 0x7fffffff, mi = 0;
        for (int m = lane; m < k; m += 64) {
            const int t = c.tag[sid[s_ring[m]]];
            if (t < mt) {
                mt = t;
                mi = m;
            }
        }
        for (int off = 32; off >= 1; off >>= 1) {
            const int ot = __shfl_xor(mt, off), oi = __shfl_xor(mi, off);
            if (ot < mt) {
                mt = ot;
                mi = oi;
            }
        }
        // touch the old neighbourhood before overwriting it
        for (int m = lane; m < kold; m += 64) push_touch(w, st, round, c.ring[i * KC + m]);
        __syncthreads();
        for (int m = lane; m < k; m += 64) {
            const int q = sid[s_ring[(mi + m) % k]];
            c.ring[i * KC + m] = q;
            push_touch(w, st, round, q);
        }
        if (lane == 0) {
            c.deg[i] = (uint8_t)k;
            push_touch(w, st, round, i);
            atomicAdd(&st->repaired, 1ull);
            atomicMax(&st->max_deg, k);
        }
        __syncthreads();
    }
    if (exact) atomicAdd(&st->exact_calls, (unsigned long long)exact);
}

// ---------------------------------------------------------------- step bookkeeping
// After the last device repair round: count the step, accumulate the drift,
// halt if rounds remain (the host finishes them) or an error was raised, and
// clear the per-step counters otherwise.
__global__ void k_finalize(DevState* st, int rounds)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (st->halt) return;
    st->step += 1ull;
    st->drift += __longlong_as_double((long long)st->disp_bits);
    st->disp_bits = 0ull;
    int used = 0;
    for (int r = 0; r < rounds; r++) used += st->wl_count[r] > 0;
    st->rounds += (unsigned long long)used;
    if (st->err || st->wl_count[rounds] > 0) {
        st->halt = 1;
        st->halt_round = rounds;
        return;
    }
    for (int r = 0; r <= rounds; r++) st->wl_count[r] = 0;
    for (int r = 0; r < rounds; r++) st->tl_count[r] = 0;
}

// host recovery finished: clear the per-step counters and resume
__global__ void k_resume(DevState* st)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int r = 0; r <= MAX_ROUNDS; r++) st->wl_count[r] = 0;
    for (int r = 0; r < MAX_ROUNDS; r++) st->tl_count[r] = 0;
    st->halt = 0;
}

__global__ void k_set_halt(DevState* st, int v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) st->halt = v;
}

// worklist of round 0 = every cell (initial triangulation)
__global__ void k_all_to_worklist(Work w, DevState* st, int N)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) {
        w.wl[0][i] = i;
        atomicOr(&w.flagbits[i >> 5], 1u << (i & 31));
    }
    if (i == 0) st->wl_count[0] = N;
}

// ---------------------------------------------------------------- spatial re-sort
__global__ void k_fill_i32(int* a, int n, int val)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = val;
}

template <typename R, bool MULTI>
__global__ void k_bin_keys(Cells<R> c, Work w, const SysParam* __restrict__ sp, const DevState* st, int N,
                           int* key, int* hist)
{
    if (st->halt) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const SysParam& P = sp[MULTI ? c.sys[i] : 0];
    const int bx = min((int)(c.x[i] / P.bsx), P.nbx - 1), by = min((int)(c.y[i] / P.bsy), P.nby - 1);
    const int kk = w.bin_key[P.bin_off + by * P.nbx + bx];
    key[i] = kk;
    atomicAdd(&hist[kk], 1);
}

// exclusive scan of n ints by one 1024-thread block (16 items per thread per
// pass); out has n + 1 entries
__global__ __launch_bounds__(1024) void k_scan(const int* __restrict__ in, int* __restrict__ out, int n,
                                               const DevState* st)
{
    constexpr int IPT = 16, CH = 1024 * IPT;
    __shared__ int part[16];
    __shared__ int carry;
    if (st->halt) return;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < n; base += CH) {
        const int i0 = base + tid * IPT;
        int v[IPT];
        int sum = 0;
#pragma unroll
        for (int k = 0; k < IPT; k++) {
            v[k] = (i0 + k < n) ? in[i0 + k] : 0;
            sum += v[k];
        }
        int inc = sum;
        for (int off = 1; off < 64; off <<= 1) {
            const int o = __shfl_up(inc, off);
            if (lane >= off) inc += o;
        }
        if (lane == 63) part[wid] = inc;
        __syncthreads();
        if (wid == 0) {
            int p = lane < 16 ? part[lane] : 0;
            for (int off = 1; off < 16; off <<= 1) {
                const int o = __shfl_up(p, off);
                if (lane >= off) p += o;
            }
            if (lane < 16) part[lane] = p;
        }
        __syncthreads();
        int run = carry + (wid ? part[wid - 1] : 0) + inc - sum;
#pragma unroll
        for (int k = 0; k < IPT; k++) {
            if (i0 + k < n) out[i0 + k] = run;
            run += v[k];
        }
        __syncthreads();
        if (tid == 1023) carry = run;
        __syncthreads();
    }
    if (tid == 0) out[n] = carry;
}

__global__ void k_bin_scatter(const int* key, const int* start, int* fill, int* perm, int n, const DevState* st)
{
    if (st->halt) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int r = key[i];
    perm[start[r] + atomicAdd(&fill[r], 1)] = i;
}

// order the few cells of each bin by tag so the permutation is deterministic
__global__ void k_bin_sort(const int* start, int* perm, const int* tag, int nb, const DevState* st)
{
    if (st->halt) return;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nb) return;
    const int s = start[r], e = start[r + 1];
    for (int a = s + 1; a < e; a++) {
        const int cc = perm[a];
        const int tc = tag[cc];
        int b = a - 1;
        while (b >= s && tag[perm[b]] > tc) {
            perm[b + 1] = perm[b];
            b--;
        }
        perm[b + 1] = cc;
    }
}

__global__ void k_inv_perm(const int* perm, int* inv, int n, const DevState* st)
{
    if (st->halt) return;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) inv[perm[p]] = p;
}

// new slot p holds old cell perm[p]; neighbour indices go through inv
template <typename R, int KC>
__global__ void k_gather(Cells<R> src, Cells<R> dst, const int* perm, const int* inv, int N, DevState* st)
{
    if (st->halt) return;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0) st->drift = 0.0;
    if (p >= N) return;
    const int i = perm[p];
    dst.x[p] = src.x[i];
    dst.y[p] = src.y[i];
    dst.th[p] = src.th[i];
    dst.tag[p] = src.tag[i];
    dst.sys[p] = src.sys[i];
    dst.A0[p] = src.A0[i];
    dst.P0[p] = src.P0[i];
    dst.A[p] = src.A[i];
    dst.P[p] = src.P[i];
    dst.ca[p] = src.ca[i];
    dst.cb[p] = src.cb[i];
    const int k = min((int)src.deg[i], KC);
    dst.deg[p] = (uint8_t)k;
    for (int m = 0; m < k; m++) {
        dst.ring[p * KC + m] = inv[src.ring[i * KC + m]];
        const int o = src.opp[i * KC + m];
        dst.opp[p * KC + m] = o >= 0 ? inv[o] : -1;
    }
}

// ---------------------------------------------------------------- outputs and observables
// out[cell_off(sys) + tag] = in[i]
template <typename T>
__global__ void k_to_tag_order(const T* in, const int* tag, const int* sys, const SysParam* sp, double* out, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[sp[sys[i]].cell_off + tag[i]] = (double)in[i];
}

// one block per system; fixed in-block tree (deterministic)
template <typename R>
__global__ __launch_bounds__(256) void k_observables(const R* A, const R* P, const double* A0, const double* P0,
                                                     const SysParam* sp, double* out)
{
    __shared__ double s[3][256];
    const SysParam& S = sp[blockIdx.x];
    double e = 0.0, q = 0.0, a = 0.0;
    for (int i = S.cell_off + threadIdx.x; i < S.cell_off + S.n; i += 256) {
        const double Ai = (double)A[i], Pi = (double)P[i];
        const double dA = Ai - A0[i], dP = Pi - P0[i];
        e += S.KA * dA * dA + S.KP * dP * dP;
        q += Pi / sqrt(Ai);
        a += Ai;
    }
    s[0][threadIdx.x] = e;
    s[1][threadIdx.x] = q;
    s[2][threadIdx.x] = a;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h)
            for (int k = 0; k < 3; k++) s[k][threadIdx.x] += s[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; k++) out[3 * blockIdx.x + k] = s[k][0];
}

__global__ void k_theta0(double* th, const int* tag, const int* sys, const SysParam* sp, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t r[4];
    philox4x64(~0ull, (uint64_t)tag[i], 0, 0, sp[sys[i]].seed, 0, r);
    th[i] = 2.0 * 3.14159265358979323846 * u01(r[0]);
}

}  // namespace spv
