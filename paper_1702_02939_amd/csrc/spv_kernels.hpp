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
// Streaming passes use a group of lanes per cell (8 in the geometry / test
// passes, KC / 4 in the force pass): lane l handles ring slots l, l + GL,
// ...; per-slot values (displacements, Voronoi vertices, unit edge vectors,
// neighbour coefficients) are staged in LDS so that a slot can read its ring
// neighbours m +- 1 for any ring length.  Rings are cell-major [N][KC]; a
// cell's lanes read one contiguous row segment.
// Every kernel first checks the device halt flag, so that a step whose
// repair did not converge turns the rest of a captured graph into no-ops.
#pragma once
#include "spv_common.hpp"
#include "spv_exact.hpp"

namespace spv {

constexpr int GL = 8;          // lanes per cell in the geometry / test kernels
constexpr int CPB = 256 / GL;  // cells per 256-thread block
// the force kernels: kcap/4 lanes per cell (four ring slots each), so a
// 256-thread block holds 1024/kcap cells and at most 1024 (cell, slot) items
constexpr int force_lanes(int kc) { return kc / 4; }
constexpr int force_cells_per_block(int kc) { return 256 / force_lanes(kc); }
// the item kernel: cells per 256-thread block (at most 64: the first
// wavefront owns them); about 6 items per cell
constexpr int items_cells_per_block(int kc) { return 1024 / kc; }
constexpr int RP_CAP = 1024;   // max candidate neighbours of one repaired cell

// ---------------------------------------------------------------- helpers

// The geometry and force arithmetic below fixes its own fused multiply-adds
// (explicit fma, no automatic contraction): its rounding then does not depend
// on the code it is inlined into, and the two force kernels agree bitwise.

// FP64 reciprocal and reciprocal square root: the hardware estimate refined
// by two Newton steps (about 1 ulp; only non-degenerate arguments are
// meaningful: a zero denominator belongs to a triangle already flagged)
__device__ __forceinline__ double fast_rcp(double d)
{
#pragma clang fp contract(off)
    double r = __builtin_amdgcn_rcp(d);
    r = r * fma(-d, r, 2.0);
    r = r * fma(-d, r, 2.0);
    return r;
}
__device__ __forceinline__ float fast_rcp(float d) { return 1.0f / d; }
__device__ __forceinline__ double fast_rsqrt(double x)
{
#pragma clang fp contract(off)
    const double hx = 0.5 * x;
    double y = __builtin_amdgcn_rsq(x);
    y = y * fma(-hx, y * y, 1.5);
    y = y * fma(-hx, y * y, 1.5);
    return y;
}
__device__ __forceinline__ float fast_rsqrt(float x) { return 1.0f / sqrtf(x); }

template <typename R>
__device__ __forceinline__ void circumcentre(R bx, R by, R cx, R cy, R& ux, R& uy)
{
#pragma clang fp contract(off)
    const R nb = fma(bx, bx, by * by), nc = fma(cx, cx, cy * cy);
    const R inv = R(0.5) * fast_rcp(fma(bx, cy, -(by * cx)));
    ux = fma(cy, nb, -(by * nc)) * inv;
    uy = fma(bx, nc, -(cx * nb)) * inv;
}

template <typename R>
__device__ __forceinline__ void unit(R ex, R ey, R& tx, R& ty)
{
#pragma clang fp contract(off)
    const R l2 = fma(ex, ex, ey * ey);
    if (l2 > R(0)) {
        const R r = fast_rsqrt(l2);
        tx = ex * r;
        ty = ey * r;
    } else {  // zero-length Voronoi edge (exact T1 configuration)
        tx = ty = R(0);
    }
}

// Unit vector of a Voronoi edge from its dual Delaunay edge: the edge runs
// along the perpendicular (px, py) of the Delaunay edge, so its direction is
// taken from the exact displacements rather than from the difference (dx, dy)
// of two nearly equal rounded vertices (which loses all relative accuracy on
// short edges); a zero-length edge (exact T1 configuration) keeps a zero
// vector, as the difference-based form gives.
template <typename R>
__device__ __forceinline__ void edge_unit(R dx, R dy, R px, R py, R& tx, R& ty)
{
#pragma clang fp contract(off)
    if (dx == R(0) && dy == R(0)) {
        tx = ty = R(0);
        return;
    }
    const R r = fast_rsqrt(fma(px, px, py * py));
    tx = px * r;
    ty = py * r;
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
    (*exact_count)++;
    return incircle_exact_sos(bx, by, cx, cy, px, py, tag[gi], tag[gb], tag[gc], tag[gp], scale);
}

// Filter only: 1 when p is certainly strictly inside the circle through
// (0, b, c) (b, c counter-clockwise), -1 when certainly outside, 0 when the
// double evaluation cannot tell.
__device__ __forceinline__ int incircle_filter(double bx, double by, double cx, double cy, double px, double py)
{
    const double nb = bx * bx + by * by, nc = cx * cx + cy * cy, np = px * px + py * py;
    const double t1 = cx * py, t2 = cy * px, t3 = px * by, t4 = py * bx, t5 = bx * cy, t6 = by * cx;
    const double det = nb * (t1 - t2) + nc * (t3 - t4) + np * (t5 - t6);
    const double perm = nb * (fabs(t1) + fabs(t2)) + nc * (fabs(t3) + fabs(t4)) + np * (fabs(t5) + fabs(t6));
    const double bound = 2.0e-15 * perm;
    if (det > bound) return -1;
    if (det < -bound) return 1;
    return 0;
}

// Wave-aggregated append: the active lanes with `want` write c to list, one
// counter atomic per wave (same-address atomics from many waves serialise at
// the device coherence point across the XCDs).
__device__ __forceinline__ void wave_append(int* list, int* count, int c, bool want)
{
    const unsigned long long mask = __ballot(want);
    if (!mask) return;
    const int lane = __lane_id();
    const int leader = __ffsll((unsigned long long)mask) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(count, __popcll(mask));
    base = __shfl(base, leader);
    if (want) list[base + __popcll(mask & ((1ull << lane) - 1ull))] = c;
}

// append the cells of a failed triangle and its opposite cell (entries < 0
// skipped) to the repair worklist of round r, each once per round: the four
// bitmap atomics are in flight together and the wave appends every new entry
// with one counter atomic (two round trips instead of eight)
__device__ __forceinline__ void push_flags4(const Work& w, DevState* st, int r, int c0, int c1, int c2, int c3)
{
    const int cs[4] = {c0, c1, c2, c3};
    unsigned old[4];
#pragma unroll
    for (int v = 0; v < 4; v++)
        old[v] = cs[v] >= 0 ? atomicOr(&w.flagbits[cs[v] >> 5], 1u << (cs[v] & 31)) : ~0u;
    bool want[4];
    unsigned long long m[4];
    int total = 0;
#pragma unroll
    for (int v = 0; v < 4; v++) {
        want[v] = cs[v] >= 0 && !(old[v] & (1u << (cs[v] & 31)));
        m[v] = __ballot(want[v]);
        total += __popcll(m[v]);
    }
    if (!total) return;
    const int lane = __lane_id();
    const int leader = __ffsll((unsigned long long)__ballot(1)) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(&st->wl_count[r], total);
    base = __shfl(base, leader);
    const unsigned long long below = (1ull << lane) - 1ull;
    int* list = w.wl[r & 1];
#pragma unroll
    for (int v = 0; v < 4; v++) {
        if (want[v]) list[base + __popcll(m[v] & below)] = cs[v];
        base += __popcll(m[v]);
    }
}

// Where a validity pass sends the cells of a failed triangle (c0 .. c2 >= 0;
// c3, the opposite cell, may be -1): the worklist of round r (BYTES false),
// or the flag bytes of dense round r (plain stores of 1, no counter: every
// writer stores the same value, and the round's repair kernel runs after
// this kernel has ended)
template <bool BYTES>
__device__ __forceinline__ void flag_cells(const Work& w, DevState* st, int r, int c0, int c1, int c2, int c3)
{
    if (BYTES) {
        w.flag8[c0] = 1;
        w.flag8[c1] = 1;
        w.flag8[c2] = 1;
        if (c3 >= 0) w.flag8[c3] = 1;
        st->dany[r] = 1;
    } else {
        push_flags4(w, st, r, c0, c1, c2, c3);
    }
}

// append c (if >= 0) to the touched list of round r, once per round
__device__ __forceinline__ void push_touch(const Work& w, DevState* st, int r, int c)
{
    bool want = false;
    if (c >= 0) {
        const unsigned bit = 1u << (c & 31);
        want = !(atomicOr(&w.touchbits[c >> 5], bit) & bit);
    }
    wave_append(w.tl[r & 1], &st->tl_count[r], c, want);
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
//
// Two kernels compute it, with bitwise the same result: k_force_cells gives
// each cell kcap/4 lanes (four ring slots each), k_force_items gives each
// thread whole (cell, slot) items from a prefix sum of the ring lengths, so
// that no lane idles on slots a short ring lacks.  Both evaluate slot m with
// slot_term and sum a cell's slots in the same order: lane l of the cell
// subtracts slots l, l + GL, l + 2 GL, ... from zero, and the GL partial sums
// are added pairwise as a butterfly over the lanes (offsets GL/2 .. 1).
// ACC (with UPDATE = false): subtract the force from fxo / fyo instead of
// storing it (adds the gradient of the energy-like functional to them).

// J_m^T g_m of slot m from b = d_m, c = d_{m+1}, the vertices h_{m-1}, h_m,
// h_{m+1}, h'_m and the coefficients of i, j_m, j_{m+1}
template <typename R>
__device__ __forceinline__ void slot_term(R Bx, R By, R Cx, R Cy, R hpx, R hpy, R hcx, R hcy, R hnx, R hny, R qx,
                                          R qy, R ai, R bi, R am, R bm, R an, R bn, R& vx, R& vy)
{
#pragma clang fp contract(off)
    R t1x, t1y, t2x, t2y, t3x, t3y;
    if constexpr (sizeof(R) == 4) {
        // FP32: directions from the dual Delaunay edges d_m, d_{m+1}
        // (counter-clockwise perpendiculars) and d_{m+1} - d_m
        // (clockwise perpendicular: away from the cell)
        edge_unit(hcx - hpx, hcy - hpy, -By, Bx, t1x, t1y);
        edge_unit(hnx - hcx, hny - hcy, -Cy, Cx, t2x, t2y);
        edge_unit(qx - hcx, qy - hcy, Cy - By, Bx - Cx, t3x, t3y);
    } else {
        unit(hcx - hpx, hcy - hpy, t1x, t1y);
        unit(hnx - hcx, hny - hcy, t2x, t2y);
        unit(qx - hcx, qy - hcy, t3x, t3y);
    }
    const R ai2 = ai * R(0.5), am2 = am * R(0.5), an2 = an * R(0.5);
    R gx = fma(bi, t1x - t2x, ai2 * (hny - hpy));
    R gy = fma(bi, t1y - t2y, ai2 * (hpx - hnx));
    gx = gx + fma(bm, t1x - t3x, am2 * (hpy - qy));
    gy = gy + fma(bm, t1y - t3y, am2 * (qx - hpx));
    gx = gx + fma(bn, -t2x - t3x, an2 * (qy - hny));
    gy = gy + fma(bn, -t2y - t3y, an2 * (hnx - qx));
    // J_m^T g, b = d_m, c = d_{m+1}, e = c - b
    const R ex = Cx - Bx, ey = Cy - By;
    const R sc = fma(Bx, Cy, -(By * Cx));
    const R be = fma(Bx, ex, By * ey), ce = fma(Cx, ex, Cy * ey);
    const R nb = fma(Bx, Bx, By * By), nc = fma(Cx, Cx, Cy * Cy);
    const R betaD = -nc * be, gammaD = nb * ce;
    const R zx = fma(betaD, Bx, gammaD * Cx), zy = fma(betaD, By, gammaD * Cy);
    const R be2 = R(2) * be, ce2 = R(-2) * ce;
    const R gbx = fma(be2, Cx, nc * ex), gby = fma(be2, Cy, nc * ey);        // grad(beta D)
    const R ggx = fma(ce2, Bx, -(nb * ex)), ggy = fma(ce2, By, -(nb * ey));  // grad(gamma D)
    const R is = fast_rcp(sc);
    const R is2 = R(2) * is;
    const R gdx = is2 * (-ey), gdy = is2 * ex;  // grad(D) / D
    const R invD = (R(0.5) * is) * is;          // 1 / (2 s^2)
    const R gB = fma(gx, Bx, gy * By), gC = fma(gx, Cx, gy * Cy), gZ = fma(gx, zx, gy * zy);
    const R bg = betaD + gammaD;
    R X = fma(gB, gbx, gC * ggx), Y = fma(gB, gby, gC * ggy);
    X = fma(-bg, gx, X);
    Y = fma(-bg, gy, Y);
    X = fma(-gZ, gdx, X);
    Y = fma(-gZ, gdy, Y);
    vx = fma(invD, X, gx);
    vy = fma(invD, Y, gy);
}

// h'_m (frame of the cell): circumcentre of (j_m, opp_m, j_{m+1}), or h_m
// itself when the edge has no opposite cell recorded
template <typename R>
__device__ __forceinline__ void opp_vertex(const Cells<R>& c, const SysParam& P, int o, double xi, double yi,
                                           double dmx, double dmy, double dnx, double dny, R hcx, R hcy, R& qx,
                                           R& qy)
{
    qx = hcx;
    qy = hcy;
    if (o >= 0) {
        const double dox = mimg_near(at(c.x, o) - xi, P.Lx, P.iLx), doy = mimg_near(at(c.y, o) - yi, P.Ly, P.iLy);
        R ux, uy;
        circumcentre((R)(dox - dmx), (R)(doy - dmy), (R)(dnx - dmx), (R)(dny - dmy), ux, uy);
        qx = ux + (R)dmx;
        qy = uy + (R)dmy;
    }
}

// X mod LU in grid units for an integral X of any size (the wrap of Eq. 3
// onto the periodic box): one correction in the common case, an exact
// integer remainder when a step moved a cell by more than a box length (a
// stiff random start can); NaN for a non-finite X or one beyond int64 units
__device__ __forceinline__ double wrap_units(double X, double LU)
{
    if (X >= 0.0 && X < LU) return X;
    if (X < 0.0 && X >= -LU) return X + LU;
    if (X >= LU && X < 2.0 * LU) return X - LU;
    if (!(fabs(X) < 4.0e18)) return NAN;
    const long long L = (long long)LU;
    long long r = (long long)X % L;
    if (r < 0) r += L;
    return (double)r;
}

// Eq. 3 for one cell from its force and the values parked at kernel start
// (x, y, theta, noise, sin, cos): the quantised, wrapped position, the
// rotated director, and the displacement length returned
__device__ __forceinline__ double update_cell(const SysParam& Q, const double* u0, double Fx, double Fy, int iu,
                                              double* __restrict__ xo, double* __restrict__ yo,
                                              double* __restrict__ tho, DevState* st, const CellCount& cc)
{
    const double xu = u0[0], yu = u0[1], thu = u0[2], nzu = u0[3], sn = u0[4], cs = u0[5];
    const double xn = xu + Q.dt * (Q.mu * Fx + Q.v0 * cs);
    const double yn = yu + Q.dt * (Q.mu * Fy + Q.v0 * sn);
    double X = wrap_units(rint(xn * Q.scale), Q.LXu), Y = wrap_units(rint(yn * Q.scale), Q.LYu);
    if (!(X >= 0.0 && X < Q.LXu && Y >= 0.0 && Y < Q.LYu)) {
        atomicOr(&st->err, ERR_NONFINITE);
        X = rint(xu * Q.scale);  // keep the stored state finite and inside the box
        Y = rint(yu * Q.scale);
    }
    const double xq = X * Q.inv_scale, yq = Y * Q.inv_scale;
    xo[iu] = xq;
    yo[iu] = yq;
    tho[iu] = thu + Q.amp * nzu;
    if (cc.count) {
        // this step's cell list: the cell's bin and its slot there
        const int bx = min((int)(xq / Q.bsx), Q.nbx - 1), by = min((int)(yq / Q.bsy), Q.nby - 1);
        const int b = Q.bin_off + by * Q.nbx + bx;
        cc.bin[iu] = b;
        cc.slot[iu] = atomicAdd(&cc.count[b], 1);
    }
    // the unwrapped move (a jump across the box counts in full: it bounds the
    // drift from the binned position) plus a grid unit for the quantisation
    const double ddx = xn - xu, ddy = yn - yu;
    return sqrt(ddx * ddx + ddy * ddy) + Q.inv_scale;
}

// x, y, theta, noise, sin, cos of the update of cell iu
template <typename R, bool MULTI>
__device__ __forceinline__ void park_update(const Cells<R>& c, const SysParam* __restrict__ sp, const DevState* st,
                                            int iu, double* u0)
{
    const SysParam& Q = sp[MULTI ? c.sys[iu] : 0];
    const double th0 = c.th[iu];
    double sn0, cs0;
    sincos(th0, &sn0, &cs0);
    u0[0] = c.x[iu];
    u0[1] = c.y[iu];
    u0[2] = th0;
    u0[3] = normal_for(Q.seed, st->step, (uint64_t)c.tag[iu]);
    u0[4] = sn0;
    u0[5] = cs0;
}

template <typename R, bool MULTI, int KC, bool UPDATE, bool ACC = false>
__global__ __launch_bounds__(256) void k_force_cells(Cells<R> c, double* __restrict__ xo, double* __restrict__ yo,
                                                     double* __restrict__ tho, double* __restrict__ fxo,
                                                     double* __restrict__ fyo, const SysParam* __restrict__ sp,
                                                     DevState* st, int N, double* __restrict__ blockmax, CellCount cc)
{
    constexpr int GL = force_lanes(KC), CPB = force_cells_per_block(KC);
    constexpr int NS = KC / GL;
    __shared__ R sH[CPB][KC][2];  // Voronoi vertex m (frame of the cell)
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
    // the update of cell iu (first CPB threads): its state, director
    // trigonometry and noise are computed up front, under the latency of the
    // neighbour gathers below (parked in LDS, not registers: the body keeps
    // its occupancy)
    const int iu = xcd_block(blockIdx.x, gridDim.x) * CPB + (int)threadIdx.x;
    const bool upd = UPDATE && threadIdx.x < CPB && iu < N;
    __shared__ double sU0[UPDATE ? CPB : 1][6];
    if (upd) park_update<R, MULTI>(c, sp, st, iu, sU0[threadIdx.x]);

    // slot m of this lane: displacements d_m, d_{m+1} (the next slot's ring
    // entry is read again from the same cache line rather than through LDS),
    // coefficients of j_m and j_{m+1}, and the opposite vertex of edge m
    R bxs[NS], bys[NS], cxs[NS], cys[NS], ams[NS], bms[NS], ans[NS], bns[NS], qxs[NS], qys[NS];
#pragma unroll
    for (int s = 0; s < NS; s++) {
        const int m = l + s * GL;
        bxs[s] = bys[s] = cxs[s] = cys[s] = ams[s] = bms[s] = ans[s] = bns[s] = qxs[s] = qys[s] = R(0);
        if (m < k) {
            const int mn = (m + 1 == k) ? 0 : m + 1;
            const int jm = at(c.ring, rslot<KC>(c.rhi, ii, m)), jn = at(c.ring, rslot<KC>(c.rhi, ii, mn)),
                      o = at(c.opp, rslot<KC>(c.rhi, ii, m));
            const double dmx = mimg_near(at(c.x, jm) - xi, P.Lx, P.iLx), dmy = mimg_near(at(c.y, jm) - yi, P.Ly, P.iLy);
            const double dnx = mimg_near(at(c.x, jn) - xi, P.Lx, P.iLx), dny = mimg_near(at(c.y, jn) - yi, P.Ly, P.iLy);
            ams[s] = at(ca, jm);
            bms[s] = at(cb, jm);
            ans[s] = at(ca, jn);
            bns[s] = at(cb, jn);
            bxs[s] = (R)dmx;
            bys[s] = (R)dmy;
            cxs[s] = (R)dnx;
            cys[s] = (R)dny;
            R hx, hy;
            circumcentre(bxs[s], bys[s], cxs[s], cys[s], hx, hy);
            sH[g][m][0] = hx;
            sH[g][m][1] = hy;
            opp_vertex(c, P, o, xi, yi, dmx, dmy, dnx, dny, hx, hy, qxs[s], qys[s]);
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
            R vx, vy;
            slot_term(bxs[s], bys[s], cxs[s], cys[s], sH[g][mp][0], sH[g][mp][1], sH[g][m][0], sH[g][m][1],
                      sH[g][mn][0], sH[g][mn][1], qxs[s], qys[s], ai, bi, ams[s], bms[s], ans[s], bns[s], vx, vy);
            fx -= vx;
            fy -= vy;
        }
    }
#pragma unroll
    for (int off = GL / 2; off > 0; off >>= 1) {
        fx += __shfl_xor(fx, off);
        fy += __shfl_xor(fy, off);
    }
    if (!UPDATE) {
        if (valid && l == 0) {
            if (ACC) {
                fxo[i] -= (double)fx;
                fyo[i] -= (double)fy;
            } else {
                fxo[i] = (double)fx;
                fyo[i] = (double)fy;
            }
        }
        return;
    }
    // the update runs on the first CPB threads (at most one wavefront) --
    // one thread per cell instead of one lane per lane group
    __shared__ double sF[CPB][2];
    if (l == 0) {
        sF[g][0] = (double)fx;
        sF[g][1] = (double)fy;
    }
    __syncthreads();
    if (threadIdx.x >= 64) return;
    double disp = 0.0;
    if (upd)
        disp = update_cell(sp[MULTI ? c.sys[iu] : 0], sU0[threadIdx.x], sF[threadIdx.x][0], sF[threadIdx.x][1], iu,
                           xo, yo, tho, st, cc);
    // block max of the displacement -> blockmax[block] (reduced by the all-cells geometry pass)
    for (int off = 32; off >= 1; off >>= 1) disp = fmax(disp, __shfl_xor(disp, off));
    if (threadIdx.x == 0) blockmax[blockIdx.x] = disp;
}

template <typename R, bool MULTI, int KC, bool UPDATE, bool ACC = false>
__global__ __launch_bounds__(256) void k_force_items(Cells<R> c, double* __restrict__ xo, double* __restrict__ yo,
                                                     double* __restrict__ tho, double* __restrict__ fxo,
                                                     double* __restrict__ fyo, const SysParam* __restrict__ sp,
                                                     DevState* st, int N, double* __restrict__ blockmax, CellCount cc)
{
    constexpr int GL = force_lanes(KC), CPB = items_cells_per_block(KC);
    constexpr int ITEMS = CPB * KC;  // most items a block can hold
    static_assert(CPB <= 64, "the first wavefront owns the cells of a block");
    __shared__ uint16_t sMap[ITEMS];    // item -> cell | slot << 8
    __shared__ R sF[ITEMS][2];          // the item's term of its cell's force
    __shared__ int sOff[CPB], sK[CPB];  // first item and ring length of each cell
    __shared__ int sItems;
    __shared__ double sU0[UPDATE ? CPB : 1][6];
    if (st->halt) return;
    const int base = xcd_block(blockIdx.x, gridDim.x) * CPB;
    const int t = threadIdx.x;
    if (t < 64) {
        // first wavefront: ring lengths, their prefix sum and the item map
        const int i = base + t;
        int k = (t < CPB && i < N) ? (int)c.deg[i] : 0;
        if (k < 3 || k > KC) k = 0;  // reported by the validity test
        int incl = k;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int v = __shfl_up(incl, off);
            if (t >= off) incl += v;
        }
        if (t < CPB) {
            sOff[t] = incl - k;
            sK[t] = k;
            for (int m = 0; m < k; m++) sMap[incl - k + m] = (uint16_t)(t | m << 8);
        }
        if (t == 63) sItems = incl;
    } else if (UPDATE && t >= 256 - CPB) {
        // last wavefront (the fewest items): the update values of each cell,
        // computed while the others gather
        const int u = t - (256 - CPB);
        if (base + u < N) park_update<R, MULTI>(c, sp, st, base + u, sU0[u]);
    }
    __syncthreads();
    const int S = sItems;
    const R* __restrict__ ca = c.ca;
    const R* __restrict__ cb = c.cb;
    // item (cell, slot m): the three Voronoi vertices around edge m are
    // computed here from d_{m-1} .. d_{m+2} (no exchange between items)
    for (int s = t; s < S; s += 256) {
        const int e = sMap[s];
        const int g = e & 0xff, m = e >> 8, k = sK[g];
        const int i = base + g;
        const SysParam& P = sp[MULTI ? c.sys[i] : 0];
        const int mp = (m == 0) ? k - 1 : m - 1, mn = (m + 1 == k) ? 0 : m + 1, mnn = (mn + 1 == k) ? 0 : mn + 1;
        const int jp = at(c.ring, rslot<KC>(c.rhi, i, mp)), jm = at(c.ring, rslot<KC>(c.rhi, i, m)),
                  jn = at(c.ring, rslot<KC>(c.rhi, i, mn)), jq = at(c.ring, rslot<KC>(c.rhi, i, mnn));
        const int o = at(c.opp, rslot<KC>(c.rhi, i, m));
        const double xi = at(c.x, i), yi = at(c.y, i);
        const double dpx = mimg_near(at(c.x, jp) - xi, P.Lx, P.iLx), dpy = mimg_near(at(c.y, jp) - yi, P.Ly, P.iLy);
        const double dmx = mimg_near(at(c.x, jm) - xi, P.Lx, P.iLx), dmy = mimg_near(at(c.y, jm) - yi, P.Ly, P.iLy);
        const double dnx = mimg_near(at(c.x, jn) - xi, P.Lx, P.iLx), dny = mimg_near(at(c.y, jn) - yi, P.Ly, P.iLy);
        const double dqx = mimg_near(at(c.x, jq) - xi, P.Lx, P.iLx), dqy = mimg_near(at(c.y, jq) - yi, P.Ly, P.iLy);
        const R Bx = (R)dmx, By = (R)dmy, Cx = (R)dnx, Cy = (R)dny;
        R hpx, hpy, hcx, hcy, hnx, hny, qx, qy;
        circumcentre((R)dpx, (R)dpy, Bx, By, hpx, hpy);
        circumcentre(Bx, By, Cx, Cy, hcx, hcy);
        circumcentre(Cx, Cy, (R)dqx, (R)dqy, hnx, hny);
        opp_vertex(c, P, o, xi, yi, dmx, dmy, dnx, dny, hcx, hcy, qx, qy);
        slot_term(Bx, By, Cx, Cy, hpx, hpy, hcx, hcy, hnx, hny, qx, qy, at(ca, i), at(cb, i), at(ca, jm), at(cb, jm),
                  at(ca, jn), at(cb, jn), sF[s][0], sF[s][1]);
    }
    __syncthreads();
    if (t >= 64) return;
    // first wavefront: each cell's force in the order of k_force_cells
    const int iu = base + t;
    const bool own = t < CPB && iu < N;
    R fx = R(0), fy = R(0);
    if (own) {
        const int o0 = sOff[t], k = sK[t];
        R px[GL], py[GL];
#pragma unroll
        for (int l = 0; l < GL; l++) {
            px[l] = R(0);
            py[l] = R(0);
            for (int m = l; m < k; m += GL) {
                px[l] -= sF[o0 + m][0];
                py[l] -= sF[o0 + m][1];
            }
        }
#pragma unroll
        for (int off = GL / 2; off > 0; off >>= 1)
#pragma unroll
            for (int l = 0; l < off; l++) {
                px[l] += px[l + off];
                py[l] += py[l + off];
            }
        fx = px[0];
        fy = py[0];
    }
    if (!UPDATE) {
        if (own) {
            if (ACC) {
                fxo[iu] -= (double)fx;
                fyo[iu] -= (double)fy;
            } else {
                fxo[iu] = (double)fx;
                fyo[iu] = (double)fy;
            }
        }
        return;
    }
    double disp = 0.0;
    if (own) disp = update_cell(sp[MULTI ? c.sys[iu] : 0], sU0[t], (double)fx, (double)fy, iu, xo, yo, tho, st, cc);
    for (int off = 32; off >= 1; off >>= 1) disp = fmax(disp, __shfl_xor(disp, off));
    if (t == 0) blockmax[blockIdx.x] = disp;
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
template <typename R, int KC>
struct GeomLds {
    double (*sD)[KC][2];  // displacements of ring slot m (cell group g)
    R (*sU)[KC][2];       // Voronoi vertices
    int (*sJ)[KC];        // ring members
};

// Terms of Voronoi edge (u_m, u_{m+1}) in A_i = 1/2 sum u_m x u_{m+1} and
// P_i = sum |u_{m+1} - u_m| (explicit fused multiply-adds: both geometry
// kernels round them alike)
template <typename R>
__device__ __forceinline__ void edge_terms(R ux, R uy, R vx, R vy, R& a2, R& per)
{
#pragma clang fp contract(off)
    const R dx = vx - ux, dy = vy - uy;
    a2 = fma(ux, vy, -(uy * vx));
    per = sqrt(fma(dx, dx, dy * dy));
}

// the step's largest displacement (block maxima of the force kernel) added
// to the drift bound, and the step counted (block 0 of the all-cells pass)
__device__ __forceinline__ void close_drift(DevState* st, const double* __restrict__ blockmax, int nblk)
{
    __shared__ double swm[256 / 64];
    double m = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) m = fmax(m, blockmax[b]);
    for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) swm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 1; v < (int)(blockDim.x >> 6); v++) m = fmax(m, swm[v]);
        st->step += 1ull;
        st->drift += m;
        st->disp_bits = __double_as_longlong(m);
    }
}

// One pass over cells t = base + g (g = threadIdx.x / GL) of a list (LIST)
// or of all cells; every thread of the block takes part (block barriers).
// EXACT = false (the all-cells pass): a predicate that the double filter
// cannot decide flags the cell instead of being evaluated exactly; the
// repair and the exact re-test of the touched cells then settle it.
// DM_TBYTES: the list holds cells whose touched byte the caller cleared (no
// touched bit to clear); DM_FBYTES: failures go to the flag bytes of dense
// round rnext instead of its worklist.
enum : int { DM_TBYTES = 1, DM_FBYTES = 2 };
template <typename R, bool MULTI, int KC, bool LIST, bool OPP, bool EXACT = true, int DM = 0>
__device__ __forceinline__ void geom_pass(const Cells<R>& c, const Work& w, const SysParam* __restrict__ sp,
                                          DevState* st, int base, int n, const int* __restrict__ list, int rnext,
                                          const GeomLds<R, KC>& S, int& exact)
{
    constexpr int NS = KC / GL;
    const int g = threadIdx.x / GL, l = threadIdx.x % GL;
    double (*sD)[KC][2] = S.sD;
    R (*sU)[KC][2] = S.sU;
    int (*sJ)[KC] = S.sJ;
    const int t = base + g;
    const bool valid = t < n;
    const int i = valid ? (LIST ? list[t] : t) : 0;
    if (LIST && !(DM & DM_TBYTES) && valid && l == 0) atomicAnd(&w.touchbits[i >> 5], ~(1u << (i & 31)));
    if (!LIST && w.cplace && valid && l == 0) w.cplace[w.cur_start[w.cbin[i]] + w.cslot[i]] = i;
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
            const int j = c.ring[rslot<KC>(c.rhi, i, m)];
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
                // jm's ring row in one go (16-byte loads of its first part,
                // and of its second part only when jm has more than RLO
                // neighbours), searched in registers for i and the two
                // entries before it
                o = -1;
                const int kj = min((int)c.deg[jm], KC);
                int row[KC];
                const int4* __restrict__ rv = reinterpret_cast<const int4*>(c.ring + (size_t)jm * RLO);
#pragma unroll
                for (int v = 0; v < RLO / 4; v++) {
                    const int4 t4 = rv[v];
                    row[4 * v] = t4.x;
                    row[4 * v + 1] = t4.y;
                    row[4 * v + 2] = t4.z;
                    row[4 * v + 3] = t4.w;
                }
#pragma unroll
                for (int q = RLO; q < KC; q++) row[q] = -1;
                if (kj > RLO) {
                    const int4* __restrict__ hv =
                        reinterpret_cast<const int4*>(c.ring + c.rhi + (size_t)jm * (KC - RLO));
#pragma unroll
                    for (int v = 0; v < (KC - RLO) / 4; v++) {
                        const int4 t4 = hv[v];
                        row[RLO + 4 * v] = t4.x;
                        row[RLO + 4 * v + 1] = t4.y;
                        row[RLO + 4 * v + 2] = t4.z;
                        row[RLO + 4 * v + 3] = t4.w;
                    }
                }
                int p = -1;
#pragma unroll
                for (int q = KC - 1; q >= 0; q--)
                    if (q < kj && row[q] == i) p = q;
                if (p >= 0) {
                    const int pm1 = (p == 0) ? kj - 1 : p - 1;
                    const int pm2 = (pm1 == 0) ? kj - 1 : pm1 - 1;
                    int v1 = -1, v2 = -1;
#pragma unroll
                    for (int q = 0; q < KC; q++) {
                        if (q == pm1) v1 = row[q];
                        if (q == pm2) v2 = row[q];
                    }
                    if (v1 == jn) o = v2;
                }
                c.opp[rslot<KC>(c.rhi, i, m)] = o;
            } else {
                o = c.opp[rslot<KC>(c.rhi, i, m)];
            }
            const double bx = sD[g][m][0], by = sD[g][m][1], cx = sD[g][mn][0], cy = sD[g][mn][1];
            bool fail;
            if (EXACT) {
                fail = cross_sign(bx, by, cx, cy, bx * cy - by * cx, P.scale) <= 0;
            } else {
                const double cr = bx * cy - by * cx;
                fail = !(cr > 1.5e-15 * (fabs(bx * cy) + fabs(by * cx)));
            }
            R ux, uy;
            circumcentre((R)bx, (R)by, (R)cx, (R)cy, ux, uy);
            if (!fail) {
                if (o < 0) {
                    fail = true;
                } else {
                    const double px = mimg(c.x[o] - xi, P.Lx, P.hLx), py = mimg(c.y[o] - yi, P.Ly, P.hLy);
                    if (EXACT)
                        fail = incircle_tags(bx, by, cx, cy, px, py, c.tag, i, jm, jn, o, P.scale, &exact) > 0;
                    else
                        fail = incircle_filter(bx, by, cx, cy, px, py) >= 0;
                }
                // a circumradius >= min(L)/4 is either a non-Delaunay triangle
                // or a true violation of the box precondition; the repair
                // tells them apart (it cannot certify a disk wider than L/2)
                if (!fail && (double)(ux * ux + uy * uy) >= rlim2) fail = true;
            }
            if (fail) flag_cells<(DM & DM_FBYTES) != 0>(w, st, rnext, i, jm, jn, o);
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
            R ta, tp;
            edge_terms(sU[g][m][0], sU[g][m][1], sU[g][mn][0], sU[g][mn][1], ta, tp);
            a2 += ta;
            per += tp;
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
    __syncthreads();  // LDS is reused by the next pass
}

// Geometry + test kernel.  LIST: the touched list of round `round` (its bits
// cleared), failures to round + 1; otherwise all cells, failures to round 0.
// STEP (all-cells pass of a step): block 0 also counts the step and adds the
// step's largest displacement (block maxima of the force kernel) to the drift
// bound that the repair rounds of this step search with.  The all-cells pass
// of one system with kcap 16 asks for 7 wavefronts per SIMD: it fits in 72
// registers without spilling, and its blocks then need fewer rounds (the
// batched variant would spill; the exact list passes keep their larger
// register budget).
template <typename R, bool MULTI, int KC, bool LIST, bool OPP, bool STEP = false, bool DENSE = false>
__global__ __launch_bounds__(256, (STEP && !MULTI && KC == 16) ? 7 : 1) void k_geom(Cells<R> c, Work w, const SysParam* __restrict__ sp, DevState* st,
                                              int N, int round, const double* __restrict__ blockmax = nullptr,
                                              int nblk = 0)
{
    __shared__ double sD[CPB][KC][2];
    __shared__ R sU[CPB][KC][2];
    __shared__ int sJ[CPB][KC];
    if (st->halt) return;
    const int n = LIST ? st->tl_count[round] : N;
    const int rnext = LIST ? round + 1 : 0;
    const int* __restrict__ list = w.tl[round & 1];
    const int bstart = LIST ? (int)blockIdx.x : xcd_block(blockIdx.x, gridDim.x);
    const GeomLds<R, KC> S{sD, sU, sJ};
    int exact = 0;
    for (int base = bstart * CPB; base < n; base += gridDim.x * CPB)
        geom_pass<R, MULTI, KC, LIST, OPP, !STEP, DENSE ? DM_FBYTES : 0>(c, w, sp, st, base, n, list, rnext, S,
                                                                         exact);
    if (exact) atomicAdd(&st->exact_calls, (unsigned long long)exact);
    if (STEP && blockIdx.x == 0) close_drift(st, blockmax, nblk);
}

// The all-cells geometry + validity pass of a step with one thread per (cell,
// ring slot) item (the layout of k_force_items; same results as k_geom with
// STEP: the same filters, and the area and perimeter summed in its order).
// An item computes u_m and u_{m+1} itself, tests triangle (i, j_m, j_{m+1})
// against opp_m and writes its edge's area and perimeter terms.
template <typename R, bool MULTI, int KC, bool DENSE = false>
__global__ __launch_bounds__(256) void k_geom_items(Cells<R> c, Work w, const SysParam* __restrict__ sp,
                                                    DevState* st, int N, const double* __restrict__ blockmax, int nblk)
{
    constexpr int CPB_I = items_cells_per_block(KC);
    constexpr int ITEMS = CPB_I * KC;
    static_assert(CPB_I <= 64, "the first wavefront owns the cells of a block");
    __shared__ uint16_t sMap[ITEMS];      // item -> cell | slot << 8
    __shared__ R sT[ITEMS][2];            // the item's area and perimeter terms
    __shared__ int sOff[CPB_I], sK[CPB_I];  // first item and ring length of each cell
    __shared__ int sItems;
    if (st->halt) return;
    const int base = xcd_block(blockIdx.x, gridDim.x) * CPB_I;
    const int t = threadIdx.x;
    if (t < 64) {
        const int i = base + t;
        const bool valid = t < CPB_I && i < N;
        if (w.cplace && valid) w.cplace[w.cur_start[w.cbin[i]] + w.cslot[i]] = i;
        int k = valid ? (int)c.deg[i] : 0;
        if (valid && (k < 3 || k > KC)) {
            atomicOr(&st->err, ERR_DEGREE);
            k = 0;
        }
        int incl = k;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int v = __shfl_up(incl, off);
            if (t >= off) incl += v;
        }
        if (t < CPB_I) {
            sOff[t] = incl - k;
            sK[t] = k;
            for (int m = 0; m < k; m++) sMap[incl - k + m] = (uint16_t)(t | m << 8);
        }
        if (t == 63) sItems = incl;
    }
    __syncthreads();
    const int S = sItems;
    for (int s = t; s < S; s += 256) {
        const int e = sMap[s];
        const int g = e & 0xff, m = e >> 8, k = sK[g];
        const int i = base + g;
        const SysParam& P = sp[MULTI ? c.sys[i] : 0];
        const int mn = (m + 1 == k) ? 0 : m + 1, mnn = (mn + 1 == k) ? 0 : mn + 1;
        const int jm = at(c.ring, rslot<KC>(c.rhi, i, m)), jn = at(c.ring, rslot<KC>(c.rhi, i, mn)),
                  jq = at(c.ring, rslot<KC>(c.rhi, i, mnn));
        const int o = at(c.opp, rslot<KC>(c.rhi, i, m));
        const double xi = at(c.x, i), yi = at(c.y, i);
        const double bx = mimg(at(c.x, jm) - xi, P.Lx, P.hLx), by = mimg(at(c.y, jm) - yi, P.Ly, P.hLy);
        const double cx = mimg(at(c.x, jn) - xi, P.Lx, P.hLx), cy = mimg(at(c.y, jn) - yi, P.Ly, P.hLy);
        const double qx = mimg(at(c.x, jq) - xi, P.Lx, P.hLx), qy = mimg(at(c.y, jq) - yi, P.Ly, P.hLy);
        const double cr = bx * cy - by * cx;
        bool fail = !(cr > 1.5e-15 * (fabs(bx * cy) + fabs(by * cx)));
        R ux, uy, vx, vy;
        circumcentre((R)bx, (R)by, (R)cx, (R)cy, ux, uy);
        circumcentre((R)cx, (R)cy, (R)qx, (R)qy, vx, vy);
        if (!fail) {
            if (o < 0) {
                fail = true;
            } else {
                const double px = mimg(at(c.x, o) - xi, P.Lx, P.hLx), py = mimg(at(c.y, o) - yi, P.Ly, P.hLy);
                fail = incircle_filter(bx, by, cx, cy, px, py) >= 0;
            }
            const double rlim2 = 0.0625 * fmin(P.Lx, P.Ly) * fmin(P.Lx, P.Ly);
            if (!fail && (double)(ux * ux + uy * uy) >= rlim2) fail = true;
        }
        if (fail) flag_cells<DENSE>(w, st, 0, i, jm, jn, o);
        edge_terms(ux, uy, vx, vy, sT[s][0], sT[s][1]);
    }
    __syncthreads();
    if (t < CPB_I && base + t < N && sK[t] >= 3) {
        // the order of k_geom: lane l of GL sums slots l, l + GL, ..., then
        // the lane butterfly
        const int i = base + t, o0 = sOff[t], k = sK[t];
        const SysParam& P = sp[MULTI ? c.sys[i] : 0];
        R pa[GL], pp[GL];
#pragma unroll
        for (int l = 0; l < GL; l++) {
            pa[l] = R(0);
            pp[l] = R(0);
            for (int m = l; m < k; m += GL) {
                pa[l] += sT[o0 + m][0];
                pp[l] += sT[o0 + m][1];
            }
        }
#pragma unroll
        for (int off = GL / 2; off > 0; off >>= 1)
#pragma unroll
            for (int l = 0; l < off; l++) {
                pa[l] += pa[l + off];
                pp[l] += pp[l + off];
            }
        const R A = R(0.5) * pa[0];
        c.A[i] = A;
        c.P[i] = pp[0];
        c.ca[i] = (R)(2.0 * P.KA * ((double)A - c.A0[i]));
        c.cb[i] = (R)(2.0 * P.KP * ((double)pp[0] - c.P0[i]));
    }
    if (blockIdx.x == 0) close_drift(st, blockmax, nblk);
}

// ---------------------------------------------------------------- repair
// One 64-lane wavefront rebuilds the Delaunay ring of one flagged cell i.
// Candidates: every cell of i's system within distance R, gathered from the
// bins of the last re-sort (searched with R + drift, drift bounding the
// motion since then), or from this step's cell list when one was built (no
// drift).  The ring is traced counter-clockwise by gift-wrapping:
// from the nearest candidate (always a Delaunay neighbour) the next neighbour
// after c is the left-side candidate p whose circle through (i, c, p)
// contains no other left-side candidate -- an arg-min under the exact
// in-circle order, per lane and then across the wave.  The ring is certified
// when every new circumdisk lies inside the search disk (2 |u_m| <= R), which
// makes each new triangle empty with respect to all cells; otherwise R doubles.

// LDS of one repairing wavefront
struct RepairLds {
    double* sx;   // candidate displacements
    double* sy;
    int* sid;     // candidate cell
    int* stg;     // candidate tag
    int* s_n;     // candidate count
    int* s_ring;  // ring under construction (candidate slots), KMAX + 1 entries
    int* s_tmp;   // KMAX + 1 entries of scratch
    int cap;      // capacity of sx .. stg
};

constexpr int KMAX = 64;      // longest ring a repair may trace
constexpr int STAR_MAX = 48;  // most candidates the parallel star takes

// Wave-level barrier: the lanes of one wavefront exchange LDS data with no
// workgroup barrier (several wavefronts of a block repair different cells).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// v of lane l (l uniform across the wavefront)
__device__ __forceinline__ double readlane_d(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Delaunay neighbours of the cell at the origin among the n candidates
// (sx, sy), decided all at once, one candidate p per lane.  The circles
// through 0 and p have centres p/2 + t perp(p); a candidate q left of the
// line 0 -> p lies outside the circle iff t <= t_q, one on the right iff
// t >= t_q, with t_q = (|q|^2 - p.q) / (2 p x q), and a candidate strictly
// inside the segment (0, p) lies inside every such circle.  So (0, p) has an
// empty circle iff max over right-side t_q < min over left-side t_q.  Each
// key carries a rounding bound; the members are then ordered
// counter-clockwise by exact angle comparisons into s_ring.  Returns the
// number of members with closed = (at least 3 and every consecutive pair
// turns counter-clockwise), or -1 when some decision is within rounding
// (near-ties such as cocircular cells, near-collinear candidates): the
// caller then uses the exact sequential construction.
__device__ int star_parallel(const double* __restrict__ sx, const double* __restrict__ sy, int n, int* s_ring,
                             int* s_tmp, double scale, bool& closed)
{
    const int lane = threadIdx.x & 63;
    // G lanes per candidate split the loop over the other candidates (three
    // for 17 to 21 candidates: 51 to 63 lanes busy instead of 34 to 42)
    const int G = n <= 16 ? 4 : (n <= 21 ? 3 : (n <= 32 ? 2 : 1));
    const int per_pass = G == 3 ? 21 : 64 / G;
    // lane / G and lane % G without a division (lane * 21846 >> 16 is
    // lane / 3 for lane < 64)
    const int gl = G == 3 ? (lane * 21846) >> 16 : lane >> (G == 4 ? 2 : G == 2 ? 1 : 0);
    const int r = lane - gl * G;
    int unsure = 0, k = 0;
    for (int base = 0; base < n; base += per_pass) {
        // (lane 63 idles when G = 3: its candidate index is past the end)
        const int pi = gl < per_pass ? base + gl : n;
        bool mem = false, blocked = false;
        double ulo = INFINITY, uhi = INFINITY, llo = -INFINITY, lhi = -INFINITY;
        if (pi < n) {
            const double px = sx[pi], py = sy[pi];
#pragma unroll 4
            for (int q = r; q < n; q += G) {
                if (q == pi) continue;
                const double qx = sx[q], qy = sy[q];
                const double a = px * qy, b = py * qx;
                const double cr = a - b;
                const double ecr = 1e-15 * (fabs(a) + fabs(b));
                if (!(fabs(cr) > 4.0 * ecr)) {
                    if (cross_sign_exact(px, py, qx, qy, scale) != 0) {
                        unsure = 1;  // nearly collinear: t_q is ill-conditioned
                    } else {
                        // exactly collinear: q = lambda p excludes p iff 0 < lambda < 1
                        const __int128 PX = to_units(px, scale), PY = to_units(py, scale);
                        const __int128 QX = to_units(qx, scale), QY = to_units(qy, scale);
                        if (PX * QX + PY * QY > 0 && QX * QX + QY * QY < PX * PX + PY * PY) blocked = true;
                    }
                    continue;
                }
                // one reciprocal: ir = 1 / (2 p x q) (hardware estimate and
                // two Newton steps, within about an ulp); the bound is that
                // of num / (2 cr) with |num error| <= 4e-15 (|q|^2 + |p.q|
                // terms), |cr error| <= ecr <= |cr| / 4, and a relative
                // margin of 4e-15 (some 18 ulps) for ir and the product
                const double pq = fabs(px * qx) + fabs(py * qy);
                const double num = qx * qx + qy * qy - (px * qx + py * qy);
                const double ir = fast_rcp(2.0 * cr);
                const double t = num * ir;
                const double air = fabs(ir);
                const double e = air * (4e-15 * (qx * qx + qy * qy + pq)) + fabs(t) * (4.0 * ecr * air + 4e-15);
                if (cr > 0.0) {
                    ulo = fmin(ulo, t - e);
                    uhi = fmin(uhi, t + e);
                } else {
                    llo = fmax(llo, t - e);
                    lhi = fmax(lhi, t + e);
                }
            }
        }
        // combine the G lanes of each candidate (aligned groups)
        if (G == 3) {
            // only the group's first lane (r = 0) uses the result: it reads
            // lanes + 1 and + 2, the rest of its group
            ulo = fmin(ulo, fmin(__shfl_down(ulo, 1), __shfl_down(ulo, 2)));
            uhi = fmin(uhi, fmin(__shfl_down(uhi, 1), __shfl_down(uhi, 2)));
            llo = fmax(llo, fmax(__shfl_down(llo, 1), __shfl_down(llo, 2)));
            lhi = fmax(lhi, fmax(__shfl_down(lhi, 1), __shfl_down(lhi, 2)));
            const int bl = blocked ? 1 : 0;
            blocked = (bl | __shfl_down(bl, 1) | __shfl_down(bl, 2)) != 0;
        } else {
            for (int off = 1; off < G; off <<= 1) {
                ulo = fmin(ulo, __shfl_xor(ulo, off));
                uhi = fmin(uhi, __shfl_xor(uhi, off));
                llo = fmax(llo, __shfl_xor(llo, off));
                lhi = fmax(lhi, __shfl_xor(lhi, off));
                blocked = __shfl_xor((int)blocked, off) != 0 || blocked;
            }
        }
        if (pi < n && r == 0 && !blocked) {
            if (ulo > lhi) mem = true;           // certainly a non-empty interval
            else if (!(llo > uhi)) unsure = 1;  // and not certainly empty either
        }
        const unsigned long long m = __ballot(mem);
        if (mem) {
            const int pos = k + __popcll(m & ((1ull << lane) - 1ull));
            if (pos <= KMAX) s_tmp[pos] = pi;
        }
        k += __popcll(m);
    }
    closed = false;
    if (__ballot(unsure)) return -1;
    if (k > KMAX) return k;
    wave_sync();
    // counter-clockwise order from the direction (1, 0): half-plane, then
    // the exact sign of the cross product (no two members share a ray).
    // Member j's coordinates come from lane j's registers (the loop index is
    // uniform), not through LDS.
    int rank = 0, my = -1;
    double ax = 0.0, ay = 0.0;
    if (lane < k) {
        my = s_tmp[lane];
        ax = sx[my];
        ay = sy[my];
    }
    const int ha = (ay < 0.0 || (ay == 0.0 && ax < 0.0)) ? 1 : 0;
    for (int j = 0; j < k; j++) {
        const double bx = readlane_d(ax, j), by = readlane_d(ay, j);
        if (lane < k && j != lane) {
            const int hb = (by < 0.0 || (by == 0.0 && bx < 0.0)) ? 1 : 0;
            if (hb != ha) rank += hb < ha;
            else rank += cross_sign(bx, by, ax, ay, bx * ay - by * ax, scale) > 0;
        }
    }
    wave_sync();
    if (lane < k) s_ring[rank] = my;
    wave_sync();
    bool ccw = true;
    for (int m = lane; m < k; m += 64) {
        const int p = s_ring[m], q = s_ring[(m + 1 == k) ? 0 : m + 1];
        const double ax = sx[p], ay = sy[p], bx = sx[q], by = sy[q];
        ccw = ccw && cross_sign(ax, ay, bx, by, ax * by - ay * bx, scale) > 0;
    }
    closed = k >= 3 && !__ballot(!ccw);
    return k;
}

// Rebuild the ring of cell i (all 64 lanes of the calling wavefront).
// defer_on_cap: more candidates than L.cap leave the cell untouched and
// return false (the caller hands the round to a larger kernel); otherwise
// that is a capacity error.  Returns true when the ring was rewritten.
// DENSE: the cell's flag byte was cleared by the caller, and the touched
// cells are marked in the touched bytes of dense round `round`.
template <typename R, bool MULTI, int KC, bool DENSE = false>
__device__ bool repair_one(const Cells<R>& c, const Work& w, const SysParam* __restrict__ sp, DevState* st, int round,
                           int i, double drift, const RepairLds& L, bool defer_on_cap, bool& deferred, int& exact,
                           int& cand)
{
    const int lane = threadIdx.x & 63;
    double* __restrict__ sx = L.sx;
    double* __restrict__ sy = L.sy;
    int* __restrict__ sid = L.sid;
    int* __restrict__ stg = L.stg;
    int* __restrict__ s_ring = L.s_ring;
    if (!DENSE && lane == 0) atomicAnd(&w.flagbits[i >> 5], ~(1u << (i & 31)));
    const SysParam& P = sp[MULTI ? c.sys[i] : 0];
    const double xi = c.x[i], yi = c.y[i];
    const int kold = min((int)c.deg[i], KC);
    // the old ring row (touched at the end), read while the search runs
    const int qrow = lane < KC ? c.ring[rslot<KC>(c.rhi, i, lane)] : -1;
    const double Rmax = 0.5 * fmin(P.Lx, P.Ly) * (1.0 - 1e-9);
    // first radius R0 (2.5 mean spacings: a Delaunay star rarely reaches
    // further than half of it); doubled while the star is not certified
    double Rs = fmin(P.R0, Rmax);
    // bins: this step's cell list when there is one (then drift is 0), else
    // the memory order of the last re-sort
    const bool cur = w.cur_cells != nullptr;
    int k = 0;
    bool ok = false, at_max = false;
    int last_n = 0, last_closed = 0, attempts = 0;
    double last_umax = 0.0;
    for (int attempt = 0; attempt < 16 && !ok; attempt++) {
        attempts = attempt + 1;
        if (lane == 0) *L.s_n = 0;
        wave_sync();
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
        // the window's bins 64 at a time: each lane reads one bin's range,
        // a prefix sum over the wave numbers the cells of the group, and the
        // lanes then take one cell each (the owning bin found by a binary
        // search over the lanes' offsets): three dependent loads per cell
        // instead of a walk through each bin
        const int nbins = wx * wy;
        for (int b0 = 0; b0 < nbins; b0 += 64) {
            const int b = b0 + lane;
            int s0 = 0, cnt = 0;
            if (b < nbins) {
                int bx = bx0 + b % wx, by = by0 + b / wx;
                bx = ((bx % P.nbx) + P.nbx) % P.nbx;
                by = ((by % P.nby) + P.nby) % P.nby;
                const int bi = P.bin_off + by * P.nbx + bx;
                const int2 br = cur ? make_int2(w.cur_start[bi], w.cur_start[bi + 1]) : w.bin_range[bi];
                s0 = max(br.x, lo);
                cnt = max(min(br.y, hi) - s0, 0);
            }
            int inc = cnt;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int v = __shfl_up(inc, off);
                if (lane >= off) inc += v;
            }
            const int exc = inc - cnt;
            const int tot = __shfl(inc, 63);
            for (int base = 0; base < tot; base += 64) {
                const int idx = base + lane;
                // the last lane whose offset is <= idx owns cell idx
                int own = 0;
#pragma unroll
                for (int step = 32; step >= 1; step >>= 1) {
                    const int cl = min(own + step, 63);
                    if (__shfl(exc, cl) <= idx) own = cl;
                }
                const int so = __shfl(s0, own), eo = __shfl(exc, own);
                if (idx < tot) {
                    const int e = so + (idx - eo);
                    const int q = cur ? w.cur_cells[e] : e;
                    if (q != i) {
                        const double dx = mimg(c.x[q] - xi, P.Lx, P.hLx), dy = mimg(c.y[q] - yi, P.Ly, P.hLy);
                        if (dx * dx + dy * dy <= R2) {
                            const int slot = atomicAdd(L.s_n, 1);
                            if (slot < L.cap) {
                                sx[slot] = dx;
                                sy[slot] = dy;
                                sid[slot] = q;
                                stg[slot] = c.tag[q];
                            }
                        }
                    }
                }
            }
        }
        wave_sync();
        const int n = *L.s_n;
        last_n = n;
        cand += n;
        if (n > L.cap) {
            if (defer_on_cap) {
                deferred = true;
                return false;
            }
            if (lane == 0) atomicOr(&st->err, ERR_CAPACITY);
            break;
        }
        bool closed = false;
        // the parallel star costs n^2 / 64 key evaluations per lane, the
        // sequential wrap about 7 n / 64 plus a wave reduction per member:
        // past STAR_MAX candidates the wrap is cheaper
        k = n <= STAR_MAX ? star_parallel(sx, sy, n, s_ring, L.s_tmp, P.scale, closed) : -1;
        if (k < 0) {
            // exact sequential construction: from the nearest candidate (exact
            // squared distance in grid units, ties by tag), gift-wrapping
            k = 0;
            unsigned long long bh = ~0ull, bl = ~0ull;
            int best = -1;
            for (int q = lane; q < n; q += 64) {
                const __int128 X = to_units(sx[q], P.scale), Y = to_units(sy[q], P.scale);
                const unsigned __int128 d2 = (unsigned __int128)(X * X + Y * Y);
                const unsigned long long h = (unsigned long long)(d2 >> 64), lw = (unsigned long long)d2;
                if (best < 0 || h < bh || (h == bh && (lw < bl || (lw == bl && stg[q] < stg[best])))) {
                    bh = h;
                    bl = lw;
                    best = q;
                }
            }
            for (int off = 32; off >= 1; off >>= 1) {
                const unsigned long long oh = __shfl_xor(bh, off), ol = __shfl_xor(bl, off);
                const int ob = __shfl_xor(best, off);
                if (ob >= 0 && (best < 0 || oh < bh || (oh == bh && (ol < bl || (ol == bl && stg[ob] < stg[best]))))) {
                    bh = oh;
                    bl = ol;
                    best = ob;
                }
            }
            if (best >= 0) {
                const int start = best;
                if (lane == 0) s_ring[0] = start;
                k = 1;
                int cur = start;
                while (k <= KMAX) {
                    const double cx = sx[cur], cy = sy[cur];
                    const int gc = sid[cur];
                    // Next neighbour after c: the left-side candidate whose circle
                    // through (i, c, p) is first met when the circle centre
                    // c/2 + t perp(c) moves left; t_p = (|p|^2 - c.p) / (2 c x p).
                    // p strictly inside circle(i, c, q)  <=>  t_p < t_q.  The keys
                    // are double estimates with a per-key error bound; the exact
                    // in-circle order decides whenever the two best keys overlap.
                    double t1 = INFINITY, e1 = 0.0, t2 = INFINITY, e2 = 0.0;
                    int nb = -1;
                    for (int q = lane; q < n; q += 64) {
                        if (q == cur) continue;
                        const double px = sx[q], py = sy[q];
                        const double cr = cx * py - cy * px;
                        if (cross_sign(cx, cy, px, py, cr, P.scale) <= 0) continue;
                        const double num = px * px + py * py - (cx * px + cy * py);
                        const double t = num / (2.0 * cr);
                        // rounding bounds: |d num| <= 4e-15 (|p|^2 + |c.p|), |d cr| <= ecr
                        const double ecr = 1e-15 * (fabs(cx * py) + fabs(cy * px));
                        const double bnd = (ecr > 0.25 * fabs(cr))
                                               ? INFINITY
                                               : 4e-15 * (px * px + py * py + fabs(cx * px) + fabs(cy * py)) /
                                                         (2.0 * fabs(cr)) +
                                                     fabs(t) * (2.0 * ecr / fabs(cr) + 4e-15);
                        if (t < t1) {
                            t2 = t1;
                            e2 = e1;
                            t1 = t;
                            e1 = bnd;
                            nb = q;
                        } else if (t < t2) {
                            t2 = t;
                            e2 = bnd;
                        }
                    }
                    // wave arg-min of (t1, nb) keeping the runner-up key
                    for (int off = 32; off >= 1; off >>= 1) {
                        const double ot1 = __shfl_xor(t1, off), oe1 = __shfl_xor(e1, off);
                        const double ot2 = __shfl_xor(t2, off), oe2 = __shfl_xor(e2, off);
                        const int onb = __shfl_xor(nb, off);
                        if (ot1 < t1 || (ot1 == t1 && onb >= 0 && (nb < 0 || onb < nb))) {
                            // other side wins: my best becomes a runner-up candidate
                            if (t1 < ot2) {
                                t2 = t1;
                                e2 = e1;
                            } else {
                                t2 = ot2;
                                e2 = oe2;
                            }
                            t1 = ot1;
                            e1 = oe1;
                            nb = onb;
                        } else {
                            if (ot1 < t2) {
                                t2 = ot1;
                                e2 = oe1;
                            }
                        }
                    }
                    if (nb >= 0 && t2 - e2 <= t1 + e1) {
                        // the keys cannot separate the best from the runner-up:
                        // exact arg-min under the in-circle order (rare)
                        nb = -1;
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
            }
        }
        wave_sync();
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
            // a closed star that is not certified is usually right with a
            // circumdisk reaching just past the search disk: the next radius
            // is the one that would certify it, between 1.25 R and 2 R.  An
            // uncertified star may also be wrong (outer triangles clipped by
            // the disk; its circumradii then say little, and may be huge): R
            // never more than doubles, and from the fourth attempt on, or for
            // an open star, it doubles.
            Rs = fmin((closed && attempt < 3) ? fmin(fmax(2.02 * umax, 1.25 * Rs), 2.0 * Rs) : 2.0 * Rs, Rmax);
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
        wave_sync();
        return false;
    }
    // canonical rotation: start at the smallest tag
    int mt = 0x7fffffff, mi = 0;
    for (int m = lane; m < k; m += 64) {
        const int t = stg[s_ring[m]];
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
    // touch the old neighbourhood (lanes 0..31), the new one (lanes 32..63)
    // and the cell itself in one wave-wide append (k, kold <= 32); the old
    // ring is consumed by the append (a data dependence) before the new one
    // is stored over it
    const int qnew = (lane >= 32 && lane - 32 < k) ? sid[s_ring[(mi + lane - 32) % k]] : -1;
    const int qold = lane < kold ? qrow : -1;
    int t = lane < 32 ? qold : qnew;
    const bool self_lane = (lane == 31 && kold < 32) || (lane == 63 && k < 32);
    if (self_lane && t < 0) t = i;
    if (DENSE) {
        if (t >= 0) w.touch8[t] = 1;
        if (kold >= 32 && k >= 32 && lane == 0) w.touch8[i] = 1;
        if (lane == 0) st->tany[round] = 1;
    } else {
        push_touch(w, st, round, t);
        if (kold >= 32 && k >= 32) push_touch(w, st, round, lane == 0 ? i : -1);
    }
    wave_sync();
    if (qnew >= 0) c.ring[rslot<KC>(c.rhi, i, lane - 32)] = qnew;
    if (lane == 0) c.deg[i] = (uint8_t)k;
    wave_sync();
    return true;
}

// Repair round `round`: one wavefront per flagged cell of the worklist.
template <typename R, bool MULTI, int KC>
__global__ __launch_bounds__(64) void k_repair(Cells<R> c, Work w, const SysParam* __restrict__ sp, DevState* st,
                                               int round)
{
    __shared__ double sx[RP_CAP], sy[RP_CAP];
    __shared__ int sid[RP_CAP], stg[RP_CAP];
    __shared__ int s_n;
    __shared__ int s_ring[KMAX + 1], s_tmp[KMAX + 1];
    if (st->halt) return;
    const int nw = st->wl_count[round];
    const int* __restrict__ wl = w.wl[round & 1];
    const double drift = w.cur_cells ? 0.0 : st->drift;
    const RepairLds L{sx, sy, sid, stg, &s_n, s_ring, s_tmp, RP_CAP};
    int exact = 0, nrep = 0, cand = 0;
    bool deferred = false;
    for (int wi = blockIdx.x; wi < nw; wi += gridDim.x)
        nrep += repair_one<R, MULTI, KC>(c, w, sp, st, round, wl[wi], drift, L, false, deferred, exact, cand) ? 1 : 0;
    if (threadIdx.x == 0 && nrep) {
        atomicAdd(&st->repaired, (unsigned long long)nrep);
        atomicAdd(&st->candidates, (unsigned long long)cand);
    }
    if (exact) atomicAdd(&st->exact_calls, (unsigned long long)exact);
}

// ---------------------------------------------------------------- dense rounds
// While many cells fail per step (the transient after a random start: about
// a fifth of all cells in the first steps), appending each flagged or
// touched cell to a list through one counter serialises the grid on that
// counter.  A dense step instead marks cells in one byte per cell (plain
// stores, no counter).  Round r then compacts the flag bytes into a list
// (one counter atomic per block of 1024 cells), repairs the list with a
// fixed grid of wavefronts, one cell at a time each (balanced to within one
// cell per wavefront), and re-tests the touched cells, each block compacting
// its 64 cells' touched bytes in LDS.  A repair wavefront keeps RP_DENSE
// candidates in LDS (a small footprint, so that many wavefronts share a
// compute unit); a cell with more candidates is handed to the worklist of
// round nd (the number of dense rounds), which the tail and the host rounds
// take with their larger capacities.  The last dense re-test also sends its
// failures to that worklist; the tail then runs the later rounds.  Dense
// round r lists its cells in tl[r & 1] (count dcount[r]); the worklists wl
// and the touched counters are left to the rounds from nd on.
constexpr int RP_DENSE = 160;      // candidates a dense repair holds
constexpr int DENSE_TCHUNK = 64;   // cells scanned per re-test block
constexpr int COMPACT_CELLS = 1024;  // flag bytes per compaction block (4 per thread)

// append cell i to the worklist of round r, once per round (rare: a dense
// repair with more than RP_DENSE candidates)
__device__ __forceinline__ void push_one(const Work& w, DevState* st, int r, int i)
{
    const unsigned bit = 1u << (i & 31);
    if (!(atomicOr(&w.flagbits[i >> 5], bit) & bit)) w.wl[r & 1][atomicAdd(&st->wl_count[r], 1)] = i;
}

// flag bytes of dense round r -> list tl[r & 1] (count dcount[r]); the bytes
// are cleared.  flag8 is padded with zeros to a multiple of COMPACT_CELLS.
__global__ __launch_bounds__(256) void k_compact_flags(Work w, DevState* st, int r)
{
    __shared__ int s_sum[4];
    __shared__ int s_base;
    if (st->halt || !st->dany[r]) return;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int c0 = blockIdx.x * COMPACT_CELLS + 4 * t;
    unsigned v = *reinterpret_cast<const unsigned*>(w.flag8 + c0);
    const int cnt = ((v & 0xffu) != 0) + ((v & 0xff00u) != 0) + ((v & 0xff0000u) != 0) + ((v >> 24) != 0);
    int incl = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(incl, off);
        if (lane >= off) incl += u;
    }
    if (lane == 63) s_sum[wv] = incl;
    __syncthreads();
    int before = 0, total = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        before += k < wv ? s_sum[k] : 0;
        total += s_sum[k];
    }
    if (total == 0) return;
    if (t == 0) s_base = atomicAdd(&st->dcount[r], total);
    __syncthreads();
    if (cnt) {
        int* __restrict__ list = w.tl[r & 1];
        int pos = s_base + before + incl - cnt;
#pragma unroll
        for (int k = 0; k < 4; k++)
            if ((v >> (8 * k)) & 0xffu) list[pos++] = c0 + k;
        *reinterpret_cast<unsigned*>(w.flag8 + c0) = 0u;
    }
}

// the repair of dense round r: wavefront g takes list entries g, g + grid, ...
template <typename R, bool MULTI, int KC>
__global__ __launch_bounds__(64, 4) void k_repair_dense(Cells<R> c, Work w, const SysParam* __restrict__ sp,
                                                        DevState* st, int round, int nd)
{
    __shared__ double sx[RP_DENSE], sy[RP_DENSE];
    __shared__ int sid[RP_DENSE], stg[RP_DENSE];
    __shared__ int s_n;
    __shared__ int s_ring[KMAX + 1], s_tmp[KMAX + 1];
    if (st->halt || !st->dany[round]) return;
    const int nw = st->dcount[round];
    if ((int)blockIdx.x >= nw) return;
    const int* __restrict__ list = w.tl[round & 1];
    const double drift = w.cur_cells ? 0.0 : st->drift;
    const RepairLds L{sx, sy, sid, stg, &s_n, s_ring, s_tmp, RP_DENSE};
    int exact = 0, nrep = 0, cand = 0;
    for (int wi = blockIdx.x; wi < nw; wi += gridDim.x) {
        const int i = list[wi];
        bool deferred = false;
        nrep += repair_one<R, MULTI, KC, true>(c, w, sp, st, round, i, drift, L, true, deferred, exact, cand) ? 1 : 0;
        if (deferred && threadIdx.x == 0) push_one(w, st, nd, i);
    }
    if (threadIdx.x == 0 && nrep) {
        atomicAdd(&st->repaired, (unsigned long long)nrep);
        atomicAdd(&st->candidates, (unsigned long long)cand);
    }
    if (exact) atomicAdd(&st->exact_calls, (unsigned long long)exact);
}

// LAST: the re-test of the last dense round (failures to the worklist of
// round round + 1 = nd)
template <typename R, bool MULTI, int KC, bool LAST>
__global__ __launch_bounds__(256) void k_retest_dense(Cells<R> c, Work w, const SysParam* __restrict__ sp,
                                                      DevState* st, int N, int round)
{
    __shared__ double sD[CPB][KC][2];
    __shared__ R sU[CPB][KC][2];
    __shared__ int sJ[CPB][KC];
    __shared__ int s_list[DENSE_TCHUNK];
    __shared__ int s_n;
    static_assert(DENSE_TCHUNK == 64, "one wavefront scans the block's cells");
    if (st->halt || !st->tany[round]) return;
    if (threadIdx.x < 64) {
        const int cell = xcd_block(blockIdx.x, gridDim.x) * DENSE_TCHUNK + threadIdx.x;
        const bool t = cell < N && w.touch8[cell] != 0;
        if (t) w.touch8[cell] = 0;
        const unsigned long long m = __ballot(t);
        if (t) s_list[__popcll(m & ((1ull << threadIdx.x) - 1ull))] = cell;
        if (threadIdx.x == 0) s_n = __popcll(m);
    }
    __syncthreads();
    const int n = s_n;
    if (n == 0) return;
    const GeomLds<R, KC> S{sD, sU, sJ};
    int exact = 0;
    for (int b = 0; b < n; b += CPB)
        geom_pass<R, MULTI, KC, true, true, true, LAST ? DM_TBYTES : (DM_TBYTES | DM_FBYTES)>(
            c, w, sp, st, b, n, s_list, round + 1, S, exact);
    if (exact) atomicAdd(&st->exact_calls, (unsigned long long)exact);
}

// ---------------------------------------------------------------- step tail
// After the full-grid repair of round 0: every block of the tail grid
// re-tests a share of the cells that round touched (rebuilding their
// opposite vertices); the last block to finish then runs rounds
// 1 .. rounds-1 and closes the step alone.  After round 0 a step usually has
// no or a handful of flagged cells, which a few wavefronts repair (one cell
// each) and a block-wide geometry pass re-tests, with block barriers between
// the phases instead of kernel boundaries.  A round with more than max_items
// cells, a cell with more than RP_TAIL candidates, rounds left at the end or
// an error halt the step; the host then finishes it with full-grid rounds.
// Otherwise the per-step counters are cleared for the next step.  No block
// ever waits for another (the hand-over is a counter, not a barrier).
constexpr int TAIL_WAVES = 8;
constexpr int TAIL_BLOCKS = 32;  // the smallest tail grid
constexpr int TAIL_THREADS = 64 * TAIL_WAVES;
constexpr int TAIL_CPB = TAIL_THREADS / GL;
constexpr int RP_TAIL = 512;
constexpr int MAX_FULL_ROUNDS = 4;  // repair rounds over the whole grid before the tail
static_assert(MAX_FULL_ROUNDS < MAX_ROUNDS, "the tail reads wl_count[0 .. MAX_FULL_ROUNDS]");

// counters written by atomics of other wavefronts of this block: read at
// device scope (past the compute unit's L1)
__device__ __forceinline__ int load_count(const int* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// f: rounds 0 .. f-1 ran over the whole grid; the tail re-tests round f-1's
// touched cells and runs rounds f .. rounds-1.
template <typename R, bool MULTI, int KC>
__global__ __launch_bounds__(TAIL_THREADS) void k_tail(Cells<R> c, Work w, const SysParam* __restrict__ sp,
                                                       DevState* st, int rounds, int max_items, int f)
{
    constexpr size_t kRepBytes =
        (size_t)TAIL_WAVES * (RP_TAIL * (2 * sizeof(double) + 2 * sizeof(int)) + 2 * (KMAX + 1) * sizeof(int));
    constexpr size_t kGeoBytes = (size_t)TAIL_CPB * KC * (2 * sizeof(double) + 2 * sizeof(R) + sizeof(int));
    __shared__ __align__(16) unsigned char raw[kRepBytes > kGeoBytes ? kRepBytes : kGeoBytes];
    __shared__ int s_n[TAIL_WAVES];
    __shared__ int s_defer;
    if (st->halt) return;
    const int wave = threadIdx.x >> 6;
    // repair views (one slice per wavefront)
    unsigned char* q = raw;
    double* sx = reinterpret_cast<double*>(q) + wave * RP_TAIL;
    q += (size_t)TAIL_WAVES * RP_TAIL * sizeof(double);
    double* sy = reinterpret_cast<double*>(q) + wave * RP_TAIL;
    q += (size_t)TAIL_WAVES * RP_TAIL * sizeof(double);
    int* sid = reinterpret_cast<int*>(q) + wave * RP_TAIL;
    q += (size_t)TAIL_WAVES * RP_TAIL * sizeof(int);
    int* stg = reinterpret_cast<int*>(q) + wave * RP_TAIL;
    q += (size_t)TAIL_WAVES * RP_TAIL * sizeof(int);
    int* sring = reinterpret_cast<int*>(q) + wave * (KMAX + 1);
    q += (size_t)TAIL_WAVES * (KMAX + 1) * sizeof(int);
    int* stmp = reinterpret_cast<int*>(q) + wave * (KMAX + 1);
    const RepairLds L{sx, sy, sid, stg, &s_n[wave], sring, stmp, RP_TAIL};
    // geometry views (the same memory, used between block barriers)
    unsigned char* g = raw;
    const GeomLds<R, KC> S{reinterpret_cast<double(*)[KC][2]>(g),
                           reinterpret_cast<R(*)[KC][2]>(g + (size_t)TAIL_CPB * KC * 2 * sizeof(double)),
                           reinterpret_cast<int(*)[KC]>(g + (size_t)TAIL_CPB * KC * 2 * (sizeof(double) + sizeof(R)))};

    int exact = 0, nrep = 0, cand = 0;
    {
        // re-test of round f-1, shared by the grid; failures go to round f
        const int nt = st->tl_count[f - 1];
        const int* __restrict__ tl = w.tl[(f - 1) & 1];
        for (int base = blockIdx.x * TAIL_CPB; base < nt; base += gridDim.x * TAIL_CPB)
            geom_pass<R, MULTI, KC, true, true>(c, w, sp, st, base, nt, tl, f, S, exact);
    }
    __shared__ int s_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        // release: this block's writes before its count (no acquire needed here)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        s_last = atomicAdd(&st->done, 1) == (int)gridDim.x - 1;
    }
    __syncthreads();
    if (!s_last) {
        if (exact) atomicAdd(&st->exact_calls, (unsigned long long)exact);
        return;
    }
    // the step's counters and error word: device-scope atomic loads (they
    // read past the L2, where the other blocks' atomics were performed before
    // their counts), issued together into registers, one round trip
    __shared__ int s_w0, s_w1, s_err;
    if (threadIdx.x == 0) {
        int cnt[MAX_FULL_ROUNDS + 1];
#pragma unroll
        for (int v = 0; v <= MAX_FULL_ROUNDS; v++) cnt[v] = load_count(&st->wl_count[v]);
        const unsigned e = __hip_atomic_load(&st->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        st->done = 0;
        int u = 0, w1 = 0;
#pragma unroll
        for (int v = 0; v <= MAX_FULL_ROUNDS; v++) {
            // a round before f had work: its worklist, or its flag bytes (dense)
            if (v < f) u += (cnt[v] > 0 || (v < DENSE_ROUNDS && st->dany[v])) ? 1 : 0;
            if (v == f) w1 = cnt[v];
        }
        s_w0 = u;  // full-grid rounds that had work
        s_w1 = w1;
        s_err = (int)e;
    }
    __syncthreads();
    // later rounds read worklist entries that other blocks stored: acquire
    // (invalidates this XCD's L2) only when there are any
    if (s_w1 > 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    int used = s_w0;
    int r = f, halt_at = -1;
    double drift = 0.0;
    for (; r < rounds; r++) {
        const int nw = r == f ? s_w1 : load_count(&st->wl_count[r]);
        if (nw == 0) break;
        if (r == f) drift = w.cur_cells ? 0.0 : st->drift;
        if (nw > max_items) {
            halt_at = r;
            break;
        }
        used++;
        if (threadIdx.x == 0) s_defer = 0;
        __syncthreads();
        const int* __restrict__ wl = w.wl[r & 1];
        for (int wi = wave; wi < nw; wi += TAIL_WAVES) {
            bool deferred = false;
            nrep += repair_one<R, MULTI, KC>(c, w, sp, st, r, wl[wi], drift, L, true, deferred, exact, cand) ? 1 : 0;
            if (deferred && (threadIdx.x & 63) == 0) s_defer = 1;
        }
        __syncthreads();
        if (s_defer) {
            halt_at = r;
            break;
        }
        const int nt = load_count(&st->tl_count[r]);
        const int* __restrict__ tl = w.tl[r & 1];
        for (int base = 0; base < nt; base += TAIL_CPB)
            geom_pass<R, MULTI, KC, true, true>(c, w, sp, st, base, nt, tl, r + 1, S, exact);
        __syncthreads();
    }
    if (halt_at < 0 && r == rounds && (rounds == f ? s_w1 : load_count(&st->wl_count[rounds])) > 0)
        halt_at = rounds;
    if ((threadIdx.x & 63) == 0 && nrep) {
        atomicAdd(&st->repaired, (unsigned long long)nrep);
        atomicAdd(&st->candidates, (unsigned long long)cand);
    }
    if (exact) atomicAdd(&st->exact_calls, (unsigned long long)exact);
    __syncthreads();
    if (threadIdx.x != 0) return;
    atomicAdd(&st->rounds, (unsigned long long)used);  // statistics: no read-back
    const bool tail_ran = used > s_w0;
    if (halt_at >= 0 || s_err ||
        (tail_ran && __hip_atomic_load(&st->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
        st->halt = 1;
        st->halt_round = halt_at >= 0 ? halt_at : rounds;
        return;
    }
    for (int v = 0; v <= rounds; v++) st->wl_count[v] = 0;
    for (int v = 0; v < rounds; v++) st->tl_count[v] = 0;
    for (int v = 0; v <= DENSE_ROUNDS; v++) st->dany[v] = 0;
    for (int v = 0; v < DENSE_ROUNDS; v++) {
        st->tany[v] = 0;
        st->dcount[v] = 0;
    }
}

// host recovery finished: clear the per-step counters and resume
__global__ void k_resume(DevState* st)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int r = 0; r <= MAX_ROUNDS; r++) st->wl_count[r] = 0;
    for (int r = 0; r < MAX_ROUNDS; r++) st->tl_count[r] = 0;
    for (int r = 0; r <= DENSE_ROUNDS; r++) st->dany[r] = 0;
    for (int r = 0; r < DENSE_ROUNDS; r++) {
        st->tany[r] = 0;
        st->dcount[r] = 0;
    }
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

// exclusive scan of n ints into out[0..n] (out[n] = total) in two launches:
// per-chunk sums with their scan (last block), chunk scans with offsets
constexpr int SCAN_CHUNK = 4096;  // elements per 256-thread block (16 per thread)

__device__ __forceinline__ int block_inclusive_scan256(int v, int* part)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(v, off);
        if (lane >= off) v += o;
    }
    if (lane == 63) part[wid] = v;
    __syncthreads();
    int add = 0;
    for (int k = 0; k < wid; k++) add += part[k];
    __syncthreads();
    return v + add;
}

// The chunk sums and, in the last block to finish (a counter, no wait), their
// exclusive scan in place (sums[nchunk] = total): the first two passes in
// one launch.
__global__ __launch_bounds__(256) void k_scan_sums_last(const int* __restrict__ in, int n, int* sums, DevState* st)
{
    __shared__ int part[4];
    __shared__ int s_last;
    if (st->halt) return;
    const int base = blockIdx.x * SCAN_CHUNK + threadIdx.x * 16;
    int v = 0;
#pragma unroll
    for (int k = 0; k < 16; k++) v += (base + k < n) ? in[base + k] : 0;
    const int tot = block_inclusive_scan256(v, part);
    if (threadIdx.x == 255) {
        sums[blockIdx.x] = tot;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        s_last = atomicAdd(&st->scan_done, 1) == (int)gridDim.x - 1;
    }
    __syncthreads();
    if (!s_last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __shared__ int carry;
    if (threadIdx.x == 0) {
        carry = 0;
        st->scan_done = 0;
    }
    __syncthreads();
    const int nb = gridDim.x;
    for (int b0 = 0; b0 < nb; b0 += 256) {
        const int b = b0 + threadIdx.x;
        const int x = b < nb ? __hip_atomic_load(&sums[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
        const int inc = block_inclusive_scan256(x, part);
        const int c0 = carry;
        if (b < nb) sums[b] = c0 + inc - x;
        __syncthreads();
        if (threadIdx.x == 255) carry = c0 + inc;
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[nb] = carry;
}

// ZERO: the input counts are cleared after they are read (the cell list's
// counts start the next step at zero without a fill launch)
template <bool ZERO = false>
__global__ __launch_bounds__(256) void k_scan_apply(int* __restrict__ in, int* __restrict__ out, int n,
                                                    const int* __restrict__ offs, const DevState* st)
{
    __shared__ int part[4];
    if (st->halt) return;
    const int base = blockIdx.x * SCAN_CHUNK + threadIdx.x * 16;
    int v[16];
    int sum = 0;
#pragma unroll
    for (int k = 0; k < 16; k++) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        sum += v[k];
    }
    if (ZERO) {
#pragma unroll
        for (int k = 0; k < 16; k++)
            if (base + k < n && v[k]) in[base + k] = 0;
    }
    int run = offs[blockIdx.x] + block_inclusive_scan256(sum, part) - sum;
#pragma unroll
    for (int k = 0; k < 16; k++) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = offs[gridDim.x];  // total
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
// order the cells of each bin by tag (deterministic memory order) and record
// the bin's cell range under its spatial index (one load for the repair)
__global__ void k_bin_sort(const int* start, const int* bin_key, int2* range, int* perm, const int* tag, int nb,
                           const DevState* st)
{
    if (st->halt) return;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int r = bin_key[b];
    const int s = start[r], e = start[r + 1];
    range[b] = make_int2(s, e);
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
    if (p == 0) {
        st->last_drift = st->drift;
        st->drift = 0.0;
    }
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
        dst.ring[rslot<KC>(dst.rhi, p, m)] = inv[src.ring[rslot<KC>(src.rhi, i, m)]];
        const int o = src.opp[rslot<KC>(src.rhi, i, m)];
        dst.opp[rslot<KC>(dst.rhi, p, m)] = o >= 0 ? inv[o] : -1;
    }
}

// ---------------------------------------------------------------- cell list of a step
// While cells move fast, the repairs of a step search a cell list of the
// step's own positions (cells of each spatial bin listed together, in no
// particular order inside a bin) instead of the last re-sort's memory order
// widened by the drift: the force kernel's update counts every cell into its
// bin (CellCount), the re-sort's scan kernels turn the counts into starts,
// and the all-cells geometry pass places the cells (Work::cplace).

// ---------------------------------------------------------------- hybrid comparison mode
// The rows (ring length, then kc entries, -1 past the length) of the listed
// cells, for the host repair.
template <int KC>
__global__ void k_pack_rows(const int* __restrict__ list, int n, const uint8_t* __restrict__ deg,
                            const int* __restrict__ ring, int rhi, int* __restrict__ out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int i = list[t];
    const int k = min((int)deg[i], KC);
    int* o = out + (size_t)t * (KC + 1);
    o[0] = k;
    for (int m = 0; m < KC; m++) o[1 + m] = m < k ? ring[rslot<KC>(rhi, i, m)] : -1;
}

// The host's new rows (cell, length, kc entries) into the ring arrays; the
// cells leave the pending worklist (their flag bits cleared).
template <int KC>
__global__ void k_unpack_rows(const int* __restrict__ in, int n, uint8_t* __restrict__ deg, int* __restrict__ ring,
                              int rhi, unsigned* flagbits)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int* r = in + (size_t)t * (KC + 2);
    const int i = r[0], k = r[1];
    deg[i] = (uint8_t)k;
    for (int m = 0; m < k; m++) ring[rslot<KC>(rhi, i, m)] = r[2 + m];
    atomicAnd(&flagbits[i >> 5], ~(1u << (i & 31)));
}

// ---------------------------------------------------------------- outputs and observables
// out[cell_off(sys) + tag] = in[i]
// one system: out[i] = in[tag[i]] (tag order -> memory order)
__global__ void k_from_tag_order(const double* __restrict__ in, const int* __restrict__ tag, double* __restrict__ out,
                                 int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[tag[i]];
}

template <typename T>
__global__ void k_to_tag_order(const T* in, const int* tag, const int* sys, const SysParam* sp, double* out, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[sp[sys[i]].cell_off + tag[i]] = (double)in[i];
}

// Observables (Eq. 1 energy, sum of P/sqrt(A), sum of A) in two fixed-order
// stages: block (s, chunk) sums cells [chunk * OBS_CHUNK, ...) of system s,
// then one block per system adds its chunks in order (deterministic).
constexpr int OBS_CHUNK = 8192;

template <typename R>
__global__ __launch_bounds__(256) void k_observables(const R* A, const R* P, const double* A0, const double* P0,
                                                     const SysParam* sp, int chunks, double* part)
{
    __shared__ double s[3][256];
    const int sys = blockIdx.x / chunks, ch = blockIdx.x % chunks;
    const SysParam& S = sp[sys];
    double e = 0.0, q = 0.0, a = 0.0;
    const int first = S.cell_off + ch * OBS_CHUNK, last = S.cell_off + min(S.n, (ch + 1) * OBS_CHUNK);
    for (int i = first + threadIdx.x; i < last; i += 256) {
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
        for (int k = 0; k < 3; k++) part[3 * blockIdx.x + k] = s[k][0];
}

__global__ void k_observables_sum(const double* part, int chunks, double* out)
{
    if (threadIdx.x >= 3) return;
    double v = 0.0;
    for (int ch = 0; ch < chunks; ch++) v += part[3 * (blockIdx.x * chunks + ch) + threadIdx.x];
    out[3 * blockIdx.x + threadIdx.x] = v;
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
