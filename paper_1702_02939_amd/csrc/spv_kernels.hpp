// spv_kernels.hpp -- HIP kernels of the SPV step on gfx950.
//
// One step (Sussman 2017, Sec. II.C) is
//   force+update   F_i = -dE/dr_i by the App. B chain rule through the Voronoi
//                  vertices, then r_i += dt (mu F_i + v0 n_i) (Eq. 3) and the
//                  director turns by sqrt(2 Dr dt) xi (Sec. II.A);
//   geometry+test  Voronoi area / perimeter of every cell (Sec. II.C.1) fused
//                  with the empty-circumcircle test of its ring (Sec. II.C.3);
//   repair         flagged rings rebuilt on the device from the candidate
//                  neighbours inside a search disk (locality lemma, Sec.
//                  II.C.4), by exact gift-wrapping around the cell.
// Layout: structure of arrays, one thread per cell for the streaming passes,
// one 64-lane wavefront per cell for the repair; neighbour rings are
// slot-major int32 [kcap][N] so that slot m of 64 consecutive cells is one
// coalesced load.
#pragma once
#include "spv_common.hpp"
#include "spv_exact.hpp"

namespace spv {

constexpr int RP_CAP = 1024;  // max candidate neighbours of one repaired cell
constexpr int RP_KMAX = 64;   // max ring length during the gift wrap

struct StepParams {
    double mu, v0, dt, amp;  // amp = sqrt(2 Dr dt)
    double KA, KP;
    uint64_t seed, step;
};

// ---------------------------------------------------------------- small helpers

__device__ __forceinline__ void circumcentre(double bx, double by, double cx, double cy, double s, double& ux,
                                             double& uy)
{
    double nb = bx * bx + by * by, nc = cx * cx + cy * cy;
    double inv = 0.5 / s;
    ux = (cy * nb - by * nc) * inv;
    uy = (bx * nc - cx * nb) * inv;
}

// In-circle with lazily loaded tags (the tie-break almost never runs).
__device__ __forceinline__ int incircle_tags(double bx, double by, double cx, double cy, double px, double py,
                                             const int* tag, int gi, int gb, int gc, int gp, double scale,
                                             int* exact_count)
{
    double nb = bx * bx + by * by, nc = cx * cx + cy * cy, np = px * px + py * py;
    double t1 = cx * py, t2 = cy * px, t3 = px * by, t4 = py * bx, t5 = bx * cy, t6 = by * cx;
    double det = nb * (t1 - t2) + nc * (t3 - t4) + np * (t5 - t6);
    double perm = nb * (fabs(t1) + fabs(t2)) + nc * (fabs(t3) + fabs(t4)) + np * (fabs(t5) + fabs(t6));
    double bound = 2.0e-15 * perm;
    if (det > bound) return -1;
    if (det < -bound) return 1;
    return incircle_sos(bx, by, cx, cy, px, py, tag[gi], tag[gb], tag[gc], tag[gp], scale, exact_count);
}

__device__ __forceinline__ void flag_cell(const View& v, int c) { v.flag[c] = 1; }

// ---------------------------------------------------------------- initial directors
__global__ void k_theta0(double* th, const int* tag, int n, uint64_t seed)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t r[4];
    philox4x64(~0ull, (uint64_t)tag[i], 0, 0, seed, 0, r);
    th[i] = 2.0 * 3.14159265358979323846 * u01(r[0]);
}

__global__ void k_iota(int* a, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = i;
}

__global__ void k_fill_u8(uint8_t* a, int n, uint8_t val)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = val;
}

__global__ void k_fill_i32(int* a, int n, int val)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = val;
}

// counters: mode 0 = step start, 1 = repair round start, 2 = worklist preset to n
__global__ void k_reset(DevCounters* c, int mode, int n)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    c->fail_count = 0;
    if (mode == 0) c->disp_bits = 0ull;
    if (mode >= 1) {
        c->wl_count = (mode == 2) ? n : 0;
        c->touched_count = 0;
    }
}

// ---------------------------------------------------------------- geometry + validity test
// For cell i with CCW ring (j_0 .. j_{k-1}) and exact displacements d_m:
//   u_m = circumcentre(0, d_m, d_{m+1})      (Voronoi vertex, frame of i)
//   A_i = 1/2 sum u_m x u_{m+1},  P_i = sum |u_{m+1} - u_m|
// and the ring is valid when every (i, j_m, j_{m+1}) is counter-clockwise and
// the cell opp_m across edge (j_m, j_{m+1}) is not strictly inside its
// circumcircle (local Delaunay property of every edge).
__device__ __forceinline__ void geom_test_cell(const View& v, int i, double KA, double KP, int* exact)
{
    const int N = v.N;
    const double xi = v.x[i], yi = v.y[i];
    const int k = v.deg[i];
    if (k < 3) {
        atomicOr(&v.cnt->err, ERR_DEGREE);
        return;
    }
    const int j0 = v.ring[i];
    const double b0x = mimg(v.x[j0] - xi, v.Lx, v.hLx), b0y = mimg(v.y[j0] - yi, v.Ly, v.hLy);
    int jm = j0;
    double bx = b0x, by = b0y;
    double a2 = 0.0, per = 0.0, u0x = 0.0, u0y = 0.0, upx = 0.0, upy = 0.0;
    const double rlim2 = 0.0625 * fmin(v.Lx, v.Ly) * fmin(v.Lx, v.Ly);
    bool any_fail = false;
    for (int m = 0; m < k; m++) {
        int jn;
        double cx, cy;
        if (m + 1 < k) {
            jn = v.ring[(m + 1) * N + i];
            cx = mimg(v.x[jn] - xi, v.Lx, v.hLx);
            cy = mimg(v.y[jn] - yi, v.Ly, v.hLy);
        } else {
            jn = j0;
            cx = b0x;
            cy = b0y;
        }
        const double s = bx * cy - by * cx;
        double ux, uy;
        circumcentre(bx, by, cx, cy, s, ux, uy);
        const int o = v.opp[m * N + i];
        bool fail = cross_sign(bx, by, cx, cy, s, v.scale) <= 0;
        if (!fail) {
            if (o < 0) {
                fail = true;
            } else {
                double px = mimg(v.x[o] - xi, v.Lx, v.hLx), py = mimg(v.y[o] - yi, v.Ly, v.hLy);
                fail = incircle_tags(bx, by, cx, cy, px, py, v.tag, i, jm, jn, o, v.scale, exact) > 0;
            }
            // a circumradius >= min(L)/4 is either a non-Delaunay triangle that
            // another cell's test will catch, or a true violation of the box
            // precondition; the repair tells them apart (it cannot certify a
            // disk wider than L/2 and then reports the precondition)
            if (!fail && ux * ux + uy * uy >= rlim2) fail = true;
        }
        if (fail) {
            any_fail = true;
            flag_cell(v, i);
            flag_cell(v, jm);
            flag_cell(v, jn);
            if (o >= 0) flag_cell(v, o);
        }
        if (m == 0) {
            u0x = ux;
            u0y = uy;
        } else {
            a2 += upx * uy - upy * ux;
            per += sqrt((ux - upx) * (ux - upx) + (uy - upy) * (uy - upy));
        }
        upx = ux;
        upy = uy;
        jm = jn;
        bx = cx;
        by = cy;
    }
    a2 += upx * u0y - upy * u0x;
    per += sqrt((u0x - upx) * (u0x - upx) + (u0y - upy) * (u0y - upy));
    const double A = 0.5 * a2;
    v.A[i] = A;
    v.P[i] = per;
    v.ca[i] = 2.0 * KA * (A - v.A0[i]);
    v.cb[i] = 2.0 * KP * (per - v.P0[i]);
    if (any_fail) atomicAdd(&v.cnt->fail_count, 1);
}

template <bool LIST>
__global__ __launch_bounds__(256) void k_geom_test(View v, double KA, double KP)
{
    const int n = LIST ? v.cnt->touched_count : v.N;
    int exact = 0;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        const int i = LIST ? v.list2[t] : t;
        geom_test_cell(v, i, KA, KP, &exact);
    }
    if (exact) atomicAdd(&v.cnt->exact_calls, exact);
}

// ---------------------------------------------------------------- force (+ update)
// Vertex h_m = r_i + u(d_m, d_{m+1}) is shared by cells i, j_m, j_{m+1}; its
// neighbours in the three polygons are h_{m-1}, h_{m+1} and h'_m, the
// circumcentre of (j_m, opp_m, j_{m+1}).  With unit edge vectors
//   t1 = (h_m - h_{m-1})/|.|, t2 = (h_{m+1} - h_m)/|.|, t3 = (h'_m - h_m)/|.|
// the vertex gradient of E (App. A, perimeter term with the incoming-minus-
// outgoing sign) is
//   g_m = a_i dA_i + b_i (t1 - t2) + a_jm dA_jm + b_jm (t1 - t3)
//       + a_jn dA_jn + b_jn (-t2 - t3),
// dA_c = 1/2 (h+_y - h-_y, h-_x - h+_x) for the CCW neighbours (h-, h+) of h_m
// in cell c, and F_i = -sum_m J_m^T g_m with the circumcentre Jacobian of
// App. B (Eq. B4).
__device__ __forceinline__ void unit(double ex, double ey, double& tx, double& ty)
{
    double l2 = ex * ex + ey * ey;
    if (l2 > 0.0) {
        double r = 1.0 / sqrt(l2);
        tx = ex * r;
        ty = ey * r;
    } else {
        tx = ty = 0.0;
    }
}

__device__ __forceinline__ void force_cell(const View& v, int i, double& Fx, double& Fy)
{
    const int N = v.N;
    const double xi = v.x[i], yi = v.y[i];
    const int k = v.deg[i];
    Fx = Fy = 0.0;
    if (k < 3) return;  // reported by the validity test
    const int jl = v.ring[(k - 1) * N + i];
    const int j0 = v.ring[i];
    const int j1 = v.ring[N + i];
    const double dlx = mimg(v.x[jl] - xi, v.Lx, v.hLx), dly = mimg(v.y[jl] - yi, v.Ly, v.hLy);
    const double d0x = mimg(v.x[j0] - xi, v.Lx, v.hLx), d0y = mimg(v.y[j0] - yi, v.Ly, v.hLy);
    const double d1x = mimg(v.x[j1] - xi, v.Lx, v.hLx), d1y = mimg(v.y[j1] - yi, v.Ly, v.hLy);
    double hlx, hly, h0x, h0y;
    circumcentre(dlx, dly, d0x, d0y, dlx * d0y - dly * d0x, hlx, hly);
    circumcentre(d0x, d0y, d1x, d1y, d0x * d1y - d0y * d1x, h0x, h0y);
    const double ai = v.ca[i], bi = v.cb[i];
    const double a0 = v.ca[j0], b0 = v.cb[j0];
    const double a1 = v.ca[j1], b1 = v.cb[j1];

    double hpx = hlx, hpy = hly;   // h_{m-1}
    double hcx = h0x, hcy = h0y;   // h_m
    double dmx = d0x, dmy = d0y;   // d_m
    double dnx = d1x, dny = d1y;   // d_{m+1}
    double am = a0, bm = b0, an = a1, bn = b1;
    double t1x, t1y;
    unit(hcx - hpx, hcy - hpy, t1x, t1y);
    double fx = 0.0, fy = 0.0;
    for (int m = 0; m < k; m++) {
        double hnx, hny, dnnx = 0.0, dnny = 0.0, ann = 0.0, bnn = 0.0;
        if (m == k - 1) {
            hnx = h0x;
            hny = h0y;
        } else if (m == k - 2) {
            hnx = hlx;
            hny = hly;
            dnnx = d0x;
            dnny = d0y;
            ann = a0;
            bnn = b0;
        } else {
            const int jnn = v.ring[(m + 2) * N + i];
            dnnx = mimg(v.x[jnn] - xi, v.Lx, v.hLx);
            dnny = mimg(v.y[jnn] - yi, v.Ly, v.hLy);
            ann = v.ca[jnn];
            bnn = v.cb[jnn];
            circumcentre(dnx, dny, dnnx, dnny, dnx * dnny - dny * dnnx, hnx, hny);
        }
        // third vertex h'_m of edge (j_m, j_{m+1}): circumcentre of (j_m, opp_m, j_{m+1})
        const int o = v.opp[m * N + i];
        double qx = hcx, qy = hcy;  // a missing opp (inconsistent ring) is reported by the test
        if (o >= 0) {
            const double dox = mimg(v.x[o] - xi, v.Lx, v.hLx), doy = mimg(v.y[o] - yi, v.Ly, v.hLy);
            const double ex = dox - dmx, ey = doy - dmy, fx2 = dnx - dmx, fy2 = dny - dmy;
            circumcentre(ex, ey, fx2, fy2, ex * fy2 - ey * fx2, qx, qy);
            qx += dmx;
            qy += dmy;
        }
        double t2x, t2y, t3x, t3y;
        unit(hnx - hcx, hny - hcy, t2x, t2y);
        unit(qx - hcx, qy - hcy, t3x, t3y);
        double gx = ai * 0.5 * (hny - hpy) + bi * (t1x - t2x);
        double gy = ai * 0.5 * (hpx - hnx) + bi * (t1y - t2y);
        gx += am * 0.5 * (hpy - qy) + bm * (t1x - t3x);
        gy += am * 0.5 * (qx - hpx) + bm * (t1y - t3y);
        gx += an * 0.5 * (qy - hny) + bn * (-t2x - t3x);
        gy += an * 0.5 * (hnx - qx) + bn * (-t2y - t3y);

        // J_m^T g with b = d_m, c = d_{m+1}, e = c - b (App. B, with the
        // cross product s = b x c in both the denominator and its gradient)
        {
            const double Bx = dmx, By = dmy, Cx = dnx, Cy = dny;
            const double ex = Cx - Bx, ey = Cy - By;
            const double s = Bx * Cy - By * Cx;
            const double D = 2.0 * s * s;
            const double be = Bx * ex + By * ey, ce = Cx * ex + Cy * ey;
            const double nb = Bx * Bx + By * By, nc = Cx * Cx + Cy * Cy;
            const double betaD = -nc * be, gammaD = nb * ce;
            const double zx = betaD * Bx + gammaD * Cx, zy = betaD * By + gammaD * Cy;
            const double gbx = 2.0 * be * Cx + nc * ex, gby = 2.0 * be * Cy + nc * ey;        // grad(beta D)
            const double ggx = -2.0 * ce * Bx - nb * ex, ggy = -2.0 * ce * By - nb * ey;      // grad(gamma D)
            const double gdx = (2.0 / s) * (-ey), gdy = (2.0 / s) * ex;                      // grad(D)/D
            const double invD = 1.0 / D;
            const double gB = gx * Bx + gy * By, gC = gx * Cx + gy * Cy, gZ = gx * zx + gy * zy;
            const double jx = gx + invD * (gB * gbx + gC * ggx - (betaD + gammaD) * gx - gZ * gdx);
            const double jy = gy + invD * (gB * gby + gC * ggy - (betaD + gammaD) * gy - gZ * gdy);
            fx -= jx;
            fy -= jy;
        }
        // advance the window
        hpx = hcx; hpy = hcy;
        hcx = hnx; hcy = hny;
        t1x = t2x; t1y = t2y;
        dmx = dnx; dmy = dny;
        dnx = dnnx; dny = dnny;
        am = an; bm = bn;
        an = ann; bn = bnn;
    }
    Fx = fx;
    Fy = fy;
}

// UPDATE: r += dt (mu F + v0 n), re-quantised and wrapped; theta += amp xi.
// Writes the new state into (xo, yo, tho); the old buffers stay untouched so
// that neighbours read step-start positions.  Without UPDATE only the force
// is written (tag order is handled by the caller).
template <bool UPDATE>
__global__ __launch_bounds__(256) void k_force(View v, double* xo, double* yo, double* tho, double* fxo,
                                               double* fyo, StepParams sp)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double disp = 0.0;
    if (i < v.N) {
        double Fx, Fy;
        force_cell(v, i, Fx, Fy);
        if (!UPDATE) {
            fxo[i] = Fx;
            fyo[i] = Fy;
        } else {
            const double xi = v.x[i], yi = v.y[i], th = v.th[i];
            double sn, cs;
            sincos(th, &sn, &cs);
            const double xn = xi + sp.dt * (sp.mu * Fx + sp.v0 * cs);
            const double yn = yi + sp.dt * (sp.mu * Fy + sp.v0 * sn);
            double X = rint(xn * v.scale), Y = rint(yn * v.scale);
            if (X < 0.0) X += v.LXu;
            else if (X >= v.LXu) X -= v.LXu;
            if (Y < 0.0) Y += v.LYu;
            else if (Y >= v.LYu) Y -= v.LYu;
            const double xq = X * v.inv_scale, yq = Y * v.inv_scale;
            if (!(X >= 0.0 && X < v.LXu && Y >= 0.0 && Y < v.LYu)) atomicOr(&v.cnt->err, ERR_NONFINITE);
            xo[i] = xq;
            yo[i] = yq;
            tho[i] = th + sp.amp * normal_for(sp.seed, sp.step, (uint64_t)v.tag[i]);
            const double ddx = mimg(xq - xi, v.Lx, v.hLx), ddy = mimg(yq - yi, v.Ly, v.hLy);
            disp = sqrt(ddx * ddx + ddy * ddy);
        }
    }
    if (UPDATE) {
        // wave max of a non-negative double through its bit pattern
        unsigned long long b = __double_as_longlong(disp);
        for (int off = 32; off >= 1; off >>= 1) {
            unsigned long long o = __shfl_xor(b, off);
            b = o > b ? o : b;
        }
        if ((threadIdx.x & 63) == 0 && b) atomicMax(&v.cnt->disp_bits, b);
    }
}

// ---------------------------------------------------------------- compaction
// Wave-aggregated stream compaction: out <- { i : a[i] != 0 }, a[i] cleared.
__global__ __launch_bounds__(256) void k_compact(uint8_t* a, int n, int* out, int* count)
{
    const int lane = threadIdx.x & 63;
    const int stride = gridDim.x * blockDim.x;
    for (int base = blockIdx.x * blockDim.x; base < n; base += stride) {
        const int i = base + threadIdx.x;
        bool f = false;
        if (i < n) {
            f = a[i] != 0;
            if (f) a[i] = 0;
        }
        const unsigned long long mask = __ballot(f);
        const int cnt = __popcll(mask);
        int slot = 0;
        if (lane == 0 && cnt) slot = atomicAdd(count, cnt);
        slot = __shfl(slot, 0);
        if (f) out[slot + __popcll(mask & ((1ull << lane) - 1ull))] = i;
    }
}

// ---------------------------------------------------------------- opp rebuild
// opp_m(i) is the third vertex of the triangle across edge (j_m, j_{m+1}):
// in the CCW ring of j_m the sequence ..., opp_m, j_{m+1}, i, ... appears.  A
// ring that does not contain that pattern is inconsistent: flag the cells.
template <bool LIST>
__global__ __launch_bounds__(256) void k_opp(View v)
{
    const int N = v.N;
    const int n = LIST ? v.cnt->touched_count : N;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        const int i = LIST ? v.list2[t] : t;
        const int k = v.deg[i];
        bool bad = false;
        for (int m = 0; m < k; m++) {
            const int j = v.ring[m * N + i];
            const int jn = v.ring[((m + 1 == k) ? 0 : m + 1) * N + i];
            const int kj = v.deg[j];
            int o = -1;
            for (int p = 0; p < kj; p++) {
                if (v.ring[p * N + j] == i) {
                    const int pm1 = (p + kj - 1) % kj, pm2 = (p + kj - 2) % kj;
                    if (v.ring[pm1 * N + j] == jn) o = v.ring[pm2 * N + j];
                    break;
                }
            }
            if (o < 0) {
                bad = true;
                flag_cell(v, j);
                flag_cell(v, jn);
            }
            v.opp[m * N + i] = o;
        }
        if (bad) {
            flag_cell(v, i);
            atomicAdd(&v.cnt->fail_count, 1);
        }
    }
}

// ---------------------------------------------------------------- repair
// One 64-lane wavefront rebuilds the Delaunay ring of one flagged cell i.
// Candidates: every cell within distance R of i, gathered from the bins of
// the last re-sort (searched with R + drift, drift bounding the motion since
// then).  The ring is traced counter-clockwise by gift-wrapping: from the
// nearest candidate (always a Delaunay neighbour), the next neighbour after
// c is the left-side candidate p whose circle through (i, c, p) contains no
// other left-side candidate -- an arg-min under the exact in-circle order,
// taken per lane and then across the wave.  The result is certified when
// every new circumdisk lies inside the search disk (2 |u_m| <= R), which
// makes each new triangle empty with respect to all cells; otherwise R grows.
__global__ __launch_bounds__(64) void k_repair(View v, double R0, double drift)
{
    __shared__ double sx[RP_CAP], sy[RP_CAP];
    __shared__ int sid[RP_CAP];
    __shared__ int s_n;
    __shared__ int s_ring[RP_KMAX + 1];
    const int lane = threadIdx.x;
    const int N = v.N;
    const int nw = v.cnt->wl_count;
    const double Rmax = 0.5 * fmin(v.Lx, v.Ly) * (1.0 - 1e-9);
    int exact = 0;
    for (int w = blockIdx.x; w < nw; w += gridDim.x) {
        const int i = v.worklist[w];
        const double xi = v.x[i], yi = v.y[i];
        const int kold = v.deg[i];
        double R = fmin(R0, Rmax);
        int k = 0;
        bool ok = false;
        bool at_max = false;
        int last_n = 0, last_closed = 0, attempts = 0;
        double last_umax = 0.0;
        for (int attempt = 0; attempt < 16 && !ok; attempt++) {
            attempts = attempt + 1;
            if (lane == 0) s_n = 0;
            __syncthreads();
            const double Rs = R + drift;
            int rbx = (int)ceil(Rs / v.bsx), rby = (int)ceil(Rs / v.bsy);
            int wx = 2 * rbx + 1, wy = 2 * rby + 1;
            int cbx = min((int)(xi / v.bsx), v.nbx - 1), cby = min((int)(yi / v.bsy), v.nby - 1);
            int bx0 = cbx - rbx, by0 = cby - rby;
            if (wx >= v.nbx) { wx = v.nbx; bx0 = 0; }
            if (wy >= v.nby) { wy = v.nby; by0 = 0; }
            const double R2 = R * R * (1.0 + 1e-12);
            for (int b = lane; b < wx * wy; b += 64) {
                int bx = bx0 + b % wx, by = by0 + b / wx;
                bx = ((bx % v.nbx) + v.nbx) % v.nbx;
                by = ((by % v.nby) + v.nby) % v.nby;
                const int r = v.bin_rank[by * v.nbx + bx];
                const int c1 = min(v.bin_start[r + 1], N);
                for (int c = max(v.bin_start[r], 0); c < c1; c++) {
                    if (c == i) continue;
                    const double dx = mimg(v.x[c] - xi, v.Lx, v.hLx), dy = mimg(v.y[c] - yi, v.Ly, v.hLy);
                    if (dx * dx + dy * dy <= R2) {
                        const int slot = atomicAdd(&s_n, 1);
                        if (slot < RP_CAP) {
                            sx[slot] = dx;
                            sy[slot] = dy;
                            sid[slot] = c;
                        }
                    }
                }
            }
            __syncthreads();
            const int n = s_n;
            last_n = n;
            if (n > RP_CAP) {
                if (lane == 0) atomicOr(&v.cnt->err, ERR_CAPACITY);
                break;
            }
            // nearest candidate: exact squared distance in grid units, ties by tag
            unsigned long long bh = ~0ull, bl = ~0ull;
            int best = -1;
            for (int q = lane; q < n; q += 64) {
                const __int128 X = to_units(sx[q], v.scale), Y = to_units(sy[q], v.scale);
                const unsigned __int128 d2 = (unsigned __int128)(X * X + Y * Y);
                const unsigned long long h = (unsigned long long)(d2 >> 64), l = (unsigned long long)d2;
                if (best < 0 || h < bh || (h == bh && (l < bl || (l == bl && v.tag[sid[q]] < v.tag[sid[best]])))) {
                    bh = h;
                    bl = l;
                    best = q;
                }
            }
            for (int off = 32; off >= 1; off >>= 1) {
                const unsigned long long oh = __shfl_xor(bh, off), ol = __shfl_xor(bl, off);
                const int ob = __shfl_xor(best, off);
                if (ob >= 0 && (best < 0 || oh < bh ||
                                (oh == bh && (ol < bl || (ol == bl && v.tag[sid[ob]] < v.tag[sid[best]]))))) {
                    bh = oh;
                    bl = ol;
                    best = ob;
                }
            }
            if (best < 0) {  // no candidate at all
                if (at_max) break;
                R = fmin(2.0 * R, Rmax);
                at_max = (R >= Rmax);
                continue;
            }
            const int start = best;
            if (lane == 0) s_ring[0] = start;
            k = 1;
            int cur = start;
            bool closed = false;
            while (k <= RP_KMAX) {
                const double cx = sx[cur], cy = sy[cur];
                const int gc = sid[cur];
                int nb = -1;
                for (int q = lane; q < n; q += 64) {
                    if (q == cur) continue;
                    const double px = sx[q], py = sy[q];
                    if (cross_sign(cx, cy, px, py, cx * py - cy * px, v.scale) <= 0) continue;
                    if (nb < 0 || incircle_tags(cx, cy, sx[nb], sy[nb], px, py, v.tag, i, gc, sid[nb], sid[q],
                                                v.scale, &exact) > 0)
                        nb = q;
                }
                for (int off = 32; off >= 1; off >>= 1) {
                    const int ob = __shfl_xor(nb, off);
                    if (ob >= 0 && ob != nb &&
                        (nb < 0 || incircle_tags(cx, cy, sx[nb], sy[nb], sx[ob], sy[ob], v.tag, i, gc, sid[nb],
                                                 sid[ob], v.scale, &exact) > 0))
                        nb = ob;
                }
                if (nb < 0) break;               // star open: search disk too small
                if (nb == start) { closed = true; break; }
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
                    circumcentre(sx[p], sy[p], sx[q], sy[q], sx[p] * sy[q] - sy[p] * sx[q], ux, uy);
                    umax = fmax(umax, sqrt(ux * ux + uy * uy));
                }
                for (int off = 32; off >= 1; off >>= 1) umax = fmax(umax, __shfl_xor(umax, off));
                if (2.0 * umax * (1.0 + 1e-9) <= R) ok = true;
            }
            last_closed = closed ? 1 : 0;
            last_umax = umax;
            if (!ok) {
                if (at_max) break;
                // an uncertified star may be wrong (outer triangles clipped by
                // the search disk), so its circumradii say nothing: double R
                R = fmin(2.0 * R, Rmax);
                at_max = (R >= Rmax);
                if (lane == 0) atomicAdd(&v.cnt->retries, 1);
            }
        }
        if (!ok) {
            if (lane == 0) {
                atomicOr(&v.cnt->err, at_max ? ERR_PRECOND : ERR_REPAIR);
                if (atomicCAS(&v.cnt->fail_set, 0, 1) == 0) {
                    v.cnt->fail_cell = v.tag[i];
                    v.cnt->fail_n = last_n;
                    v.cnt->fail_k = k;
                    v.cnt->fail_closed = last_closed;
                    v.cnt->fail_attempts = attempts;
                    v.cnt->fail_R = R;
                    v.cnt->fail_umax = last_umax;
                }
            }
            __syncthreads();
            continue;
        }
        if (k > v.kcap) {
            if (lane == 0) atomicOr(&v.cnt->err, ERR_CAPACITY);
            __syncthreads();
            continue;
        }
        // canonical rotation: start at the smallest tag
        int mt = 0x7fffffff, mi = 0;
        for (int m = lane; m < k; m += 64) {
            const int t = v.tag[sid[s_ring[m]]];
            if (t < mt) { mt = t; mi = m; }
        }
        for (int off = 32; off >= 1; off >>= 1) {
            const int ot = __shfl_xor(mt, off), oi = __shfl_xor(mi, off);
            if (ot < mt) { mt = ot; mi = oi; }
        }
        // touch the old neighbourhood before overwriting it
        for (int m = lane; m < kold; m += 64) v.touched[v.ring[m * N + i]] = 1;
        __syncthreads();
        for (int m = lane; m < k; m += 64) {
            const int c = sid[s_ring[(mi + m) % k]];
            v.ring[m * N + i] = c;
            v.touched[c] = 1;
        }
        if (lane == 0) {
            v.deg[i] = (uint8_t)k;
            v.touched[i] = 1;
            atomicAdd(&v.cnt->repaired, 1);
            atomicMax(&v.cnt->max_deg, k);
        }
        __syncthreads();
    }
    if (exact) atomicAdd(&v.cnt->exact_calls, exact);
}

// ---------------------------------------------------------------- spatial re-sort
__global__ void k_bin_keys(View v, int* key, int* hist)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= v.N) return;
    const int bx = min((int)(v.x[i] / v.bsx), v.nbx - 1), by = min((int)(v.y[i] / v.bsy), v.nby - 1);
    const int r = v.bin_rank[by * v.nbx + bx];
    key[i] = r;
    atomicAdd(&hist[r], 1);
}

// exclusive scan of n ints by one 1024-thread block; out has n + 1 entries
__global__ __launch_bounds__(1024) void k_scan(const int* in, int* out, int n)
{
    __shared__ int part[1024 / 64];
    __shared__ int carry;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < n; base += 1024) {
        const int i = base + tid;
        const int val = i < n ? in[i] : 0;
        int inc = val;
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
        const int wbase = wid ? part[wid - 1] : 0;
        if (i < n) out[i] = carry + wbase + inc - val;
        __syncthreads();
        if (tid == 1023) carry += wbase + inc;
        __syncthreads();
    }
    if (tid == 0) out[n] = carry;
}

__global__ void k_bin_scatter(const int* key, const int* start, int* fill, int* perm, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int r = key[i];
    perm[start[r] + atomicAdd(&fill[r], 1)] = i;
}

// order the few cells of each bin by tag so the permutation is deterministic
__global__ void k_bin_sort(const int* start, int* perm, const int* tag, int nb)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nb) return;
    const int s = start[r], e = start[r + 1];
    for (int a = s + 1; a < e; a++) {
        const int c = perm[a];
        const int tc = tag[c];
        int b = a - 1;
        while (b >= s && tag[perm[b]] > tc) {
            perm[b + 1] = perm[b];
            b--;
        }
        perm[b + 1] = c;
    }
}

__global__ void k_inv_perm(const int* perm, int* inv, int n)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) inv[perm[p]] = p;
}

// new slot p holds old cell perm[p]; neighbour indices go through inv
__global__ void k_gather(View src, View dst, const int* perm, const int* inv)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= src.N) return;
    const int N = src.N;
    const int i = perm[p];
    dst.x[p] = src.x[i];
    dst.y[p] = src.y[i];
    dst.th[p] = src.th[i];
    dst.tag[p] = src.tag[i];
    dst.A0[p] = src.A0[i];
    dst.P0[p] = src.P0[i];
    dst.A[p] = src.A[i];
    dst.P[p] = src.P[i];
    dst.ca[p] = src.ca[i];
    dst.cb[p] = src.cb[i];
    const int k = src.deg[i];
    dst.deg[p] = (uint8_t)k;
    for (int m = 0; m < k; m++) {
        dst.ring[m * N + p] = inv[src.ring[m * N + i]];
        const int o = src.opp[m * N + i];
        dst.opp[m * N + p] = o >= 0 ? inv[o] : -1;
    }
}

// ---------------------------------------------------------------- observables
// Deterministic two-level reduction: fixed grid, fixed in-block tree.
__global__ __launch_bounds__(256) void k_obs_partial(View v, double KA, double KP, double* part)
{
    __shared__ double s[3][256];
    double e = 0.0, q = 0.0, a = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < v.N; i += gridDim.x * blockDim.x) {
        const double A = v.A[i], P = v.P[i];
        const double dA = A - v.A0[i], dP = P - v.P0[i];
        e += KA * dA * dA + KP * dP * dP;
        q += P / sqrt(A);
        a += A;
    }
    s[0][threadIdx.x] = e;
    s[1][threadIdx.x] = q;
    s[2][threadIdx.x] = a;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h)
            for (int c = 0; c < 3; c++) s[c][threadIdx.x] += s[c][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; c++) part[c * gridDim.x + blockIdx.x] = s[c][0];
}

__global__ __launch_bounds__(256) void k_obs_final(const double* part, int nb, double* out)
{
    __shared__ double s[3][256];
    for (int c = 0; c < 3; c++) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < nb; b += 256) acc += part[c * nb + b];
        s[c][threadIdx.x] = acc;
    }
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h)
            for (int c = 0; c < 3; c++) s[c][threadIdx.x] += s[c][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; c++) out[c] = s[c][0];
}

// out[tag[i]] = in[i]
__global__ void k_to_tag_order(const double* in, const int* tag, double* out, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[tag[i]] = in[i];
}

}  // namespace spv
