// spv_adjoint.hpp -- tangent-mode kernels for the trajectory adjoint.
//
// With the topology held as recorded in the forward pass, one step is the
// smooth map r -> r + dt mu F(r; P0) + const (Eq. 3; the noise and the
// director do not depend on r).  Its transposed Jacobian applied to an
// adjoint vector lambda is lambda + dt mu dF[lambda], because dF/dr = -H is
// symmetric (H the Hessian of Eq. 1), and its P0 derivative is
// dt mu 2 K_P dP[lambda] (dF_j/dP0_i = 2 K_P dP_i/dr_j).  dF[lambda] (the
// Hessian-vector product, sign included) and dA, dP (directional derivatives
// of every cell's area and perimeter along lambda) are computed here by
// forward-mode dual arithmetic over the same formulas as the force kernel:
// circumcentres, polygon derivatives of App. A and the circumcentre Jacobian
// of App. B.  One thread per cell; positions and lambda in FP64.
#pragma once
#include "spv_common.hpp"
#include "spv_kernels.hpp"

namespace spv {

struct Dual {
    double v, d;  // value and directional derivative
};

__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator-(Dual a) { return {-a.v, -a.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Dual operator*(double s, Dual a) { return {s * a.v, s * a.d}; }
__device__ __forceinline__ Dual operator/(Dual a, Dual b)
{
    const double q = a.v / b.v;
    return {q, (a.d - q * b.d) / b.v};
}
__device__ __forceinline__ Dual dsqrt(Dual a)
{
    const double r = sqrt(a.v);
    return {r, r > 0.0 ? a.d / (2.0 * r) : 0.0};
}

__device__ __forceinline__ void dual_cc(Dual bx, Dual by, Dual cx, Dual cy, Dual& ux, Dual& uy)
{
    const Dual nb = bx * bx + by * by, nc = cx * cx + cy * cy;
    const Dual den = 2.0 * (bx * cy - by * cx);
    ux = (cy * nb - by * nc) / den;
    uy = (bx * nc - cx * nb) / den;
}

__device__ __forceinline__ void dual_unit(Dual ex, Dual ey, Dual& tx, Dual& ty)
{
    const Dual l = dsqrt(ex * ex + ey * ey);
    if (l.v > 0.0) {
        tx = ex / l;
        ty = ey / l;
    } else {
        tx = {0.0, 0.0};
        ty = {0.0, 0.0};
    }
}

// displacement of cell j from cell i with its tangent lambda_j - lambda_i
__device__ __forceinline__ void dual_disp(const double* x, const double* y, const double* lx, const double* ly,
                                          const SysParam& P, int i, int j, Dual& dx, Dual& dy)
{
    dx = {mimg(x[j] - x[i], P.Lx, P.hLx), lx[j] - lx[i]};
    dy = {mimg(y[j] - y[i], P.Ly, P.hLy), ly[j] - ly[i]};
}

// Both tangent kernels use GL lanes per cell (lane l takes ring slots l,
// l + GL, ...) and sum the lanes' parts with shuffles; grid: N * GL threads.

// directional derivatives of A_i and P_i along lambda (topology fixed);
// with aq != nullptr also the coefficients of w qbar = (w/N) sum P_c / sqrt(A_c)
// at this state: aq = d/dA, bq = d/dP (used by the next backward step)
template <int KC>
__global__ __launch_bounds__(256) void k_tangent_geom(Cells<double> c, const double* __restrict__ lx,
                                                      const double* __restrict__ ly, const SysParam* __restrict__ sp,
                                                      int N, double* __restrict__ dA, double* __restrict__ dP,
                                                      double w, double* __restrict__ aq, double* __restrict__ bq)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = gid / GL, l = gid % GL;
    const bool valid = i < N;
    const int ii = valid ? i : 0;
    if (aq && valid && l == 0) {
        const double sa = sqrt(c.A[i]);
        aq[i] = -w * c.P[i] / (2.0 * N * c.A[i] * sa);
        bq[i] = w / (N * sa);
    }
    const SysParam& P = sp[c.sys[ii]];
    const int k = valid ? min((int)c.deg[ii], KC) : 0;
    double a2 = 0.0, per = 0.0;  // tangents of 2A and P, this lane's slots
    if (k >= 3) {
        for (int m = l; m < k; m += GL) {
            // u_m = cc(d_m, d_{m+1}), u_{m+1} = cc(d_{m+1}, d_{m+2})
            Dual bx, by, cx, cy, ex, ey;
            dual_disp(c.x, c.y, lx, ly, P, ii, c.ring[rslot<KC>(c.rhi, ii, m)], bx, by);
            dual_disp(c.x, c.y, lx, ly, P, ii, c.ring[rslot<KC>(c.rhi, ii, (m + 1) % k)], cx, cy);
            dual_disp(c.x, c.y, lx, ly, P, ii, c.ring[rslot<KC>(c.rhi, ii, (m + 2) % k)], ex, ey);
            Dual ux, uy, vx, vy;
            dual_cc(bx, by, cx, cy, ux, uy);
            dual_cc(cx, cy, ex, ey, vx, vy);
            a2 += (ux * vy - uy * vx).d;
            per += dsqrt((vx - ux) * (vx - ux) + (vy - uy) * (vy - uy)).d;
        }
    }
#pragma unroll
    for (int off = GL / 2; off > 0; off >>= 1) {
        a2 += __shfl_xor(a2, off);
        per += __shfl_xor(per, off);
    }
    if (valid && l == 0) {
        dA[i] = k >= 3 ? 0.5 * a2 : 0.0;
        dP[i] = k >= 3 ? per : 0.0;
    }
}

// dF_i[lambda]: tangent of F_i = -sum_m J_m^T g_m (see k_force), with the
// area / perimeter coefficients a_c = 2 K_A (A_c - A0_c), b_c = 2 K_P (P_c - P0_c)
// carrying tangents 2 K_A dA_c and 2 K_P dP_c.
// STEP: instead of dF, write the adjoint of one step into the other lambda
// buffer, lo = lambda + dt mu dF[lambda], and add dt mu 2 K_P dP_i to g_i.
template <int KC, bool STEP = false>
__global__ __launch_bounds__(256) void k_tangent_force(Cells<double> c, const double* __restrict__ lx,
                                                       const double* __restrict__ ly,
                                                       const double* __restrict__ dA, const double* __restrict__ dP,
                                                       const SysParam* __restrict__ sp, int N,
                                                       double* __restrict__ fdx, double* __restrict__ fdy,
                                                       double* __restrict__ g = nullptr)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = gid / GL, l = gid % GL;
    const bool valid = i < N;
    const int ii = valid ? i : 0;
    const SysParam& P = sp[c.sys[ii]];
    const int k = valid ? min((int)c.deg[ii], KC) : 0;
    auto coef = [&](int j, Dual& a, Dual& b) {
        a = {c.ca[j], 2.0 * P.KA * dA[j]};
        b = {c.cb[j], 2.0 * P.KP * dP[j]};
    };
    auto vertex = [&](int m, Dual& hx, Dual& hy) {  // h_m in the frame of i
        Dual bx, by, cx, cy;
        dual_disp(c.x, c.y, lx, ly, P, ii, c.ring[rslot<KC>(c.rhi, ii, m)], bx, by);
        dual_disp(c.x, c.y, lx, ly, P, ii, c.ring[rslot<KC>(c.rhi, ii, (m + 1) % k)], cx, cy);
        dual_cc(bx, by, cx, cy, hx, hy);
    };
    double fxd = 0.0, fyd = 0.0;
    if (k >= 3) {
        Dual ai, bi;
        coef(ii, ai, bi);
        for (int m = l; m < k; m += GL) {
            const int mn = (m + 1) % k, mp = (m + k - 1) % k;
            const int jm = c.ring[rslot<KC>(c.rhi, ii, m)], jn = c.ring[rslot<KC>(c.rhi, ii, mn)];
            Dual Bx, By, Cx, Cy;
            dual_disp(c.x, c.y, lx, ly, P, ii, jm, Bx, By);
            dual_disp(c.x, c.y, lx, ly, P, ii, jn, Cx, Cy);
            Dual hpx, hpy, hcx, hcy, hnx, hny;
            vertex(mp, hpx, hpy);
            dual_cc(Bx, By, Cx, Cy, hcx, hcy);
            vertex(mn, hnx, hny);
            Dual qx = hcx, qy = hcy;
            const int o = c.opp[rslot<KC>(c.rhi, ii, m)];
            if (o >= 0) {
                Dual ox, oy;
                dual_disp(c.x, c.y, lx, ly, P, ii, o, ox, oy);
                Dual ex = ox - Bx, ey = oy - By, gx2 = Cx - Bx, gy2 = Cy - By, tx, ty;
                dual_cc(ex, ey, gx2, gy2, tx, ty);
                qx = tx + Bx;
                qy = ty + By;
            }
            Dual t1x, t1y, t2x, t2y, t3x, t3y;
            dual_unit(hcx - hpx, hcy - hpy, t1x, t1y);
            dual_unit(hnx - hcx, hny - hcy, t2x, t2y);
            dual_unit(qx - hcx, qy - hcy, t3x, t3y);
            Dual am, bm, an, bn;
            coef(jm, am, bm);
            coef(jn, an, bn);
            Dual gx = ai * (0.5 * (hny - hpy)) + bi * (t1x - t2x);
            Dual gy = ai * (0.5 * (hpx - hnx)) + bi * (t1y - t2y);
            gx = gx + am * (0.5 * (hpy - qy)) + bm * (t1x - t3x);
            gy = gy + am * (0.5 * (qx - hpx)) + bm * (t1y - t3y);
            gx = gx + an * (0.5 * (qy - hny)) + bn * (-t2x - t3x);
            gy = gy + an * (0.5 * (hnx - qx)) + bn * (-t2y - t3y);
            const Dual ex = Cx - Bx, ey = Cy - By;
            const Dual s = Bx * Cy - By * Cx;
            const Dual be = Bx * ex + By * ey, ce = Cx * ex + Cy * ey;
            const Dual nb = Bx * Bx + By * By, nc = Cx * Cx + Cy * Cy;
            const Dual betaD = -(nc * be), gammaD = nb * ce;
            const Dual zx = betaD * Bx + gammaD * Cx, zy = betaD * By + gammaD * Cy;
            const Dual gbx = 2.0 * (be * Cx) + nc * ex, gby = 2.0 * (be * Cy) + nc * ey;
            const Dual ggx = -(2.0 * (ce * Bx)) - nb * ex, ggy = -(2.0 * (ce * By)) - nb * ey;
            const Dual one = {1.0, 0.0};
            const Dual is = one / s;
            const Dual gdx = 2.0 * (is * (-ey)), gdy = 2.0 * (is * ex);
            const Dual invD = 0.5 * (is * is);
            const Dual gB = gx * Bx + gy * By, gC = gx * Cx + gy * Cy, gZ = gx * zx + gy * zy;
            fxd -= (gx + invD * (gB * gbx + gC * ggx - (betaD + gammaD) * gx - gZ * gdx)).d;
            fyd -= (gy + invD * (gB * gby + gC * ggy - (betaD + gammaD) * gy - gZ * gdy)).d;
        }
    }
#pragma unroll
    for (int off = GL / 2; off > 0; off >>= 1) {
        fxd += __shfl_xor(fxd, off);
        fyd += __shfl_xor(fyd, off);
    }
    if (!valid || l != 0) return;
    if (STEP) {
        const double h = P.dt * P.mu;
        fdx[i] = lx[i] + h * fxd;
        fdy[i] = ly[i] + h * fyd;
        g[i] += h * 2.0 * P.KP * dP[i];
    } else {
        fdx[i] = fxd;
        fdy[i] = fyd;
    }
}

// coefficients of w * qbar = w/N sum P_c / sqrt(A_c): d/dA and d/dP
__global__ void k_qbar_coef(const double* __restrict__ A, const double* __restrict__ P, int N, double w,
                            double* __restrict__ aq, double* __restrict__ bq)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double sa = sqrt(A[i]);
    aq[i] = -w * P[i] / (2.0 * N * A[i] * sa);
    bq[i] = w / (N * sa);
}

// lambda <- lambda - fq   (fq = -grad(w qbar) from the force kernel with q coefficients)
__global__ void k_adj_add_grad(double* lx, double* ly, const double* fqx, const double* fqy, int N)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    lx[i] -= fqx[i];
    ly[i] -= fqy[i];
}

// g_i += dt mu 2 K_P dP_i;  lambda <- lambda + dt mu dF[lambda]
__global__ void k_adj_step(double* lx, double* ly, const double* fdx, const double* fdy, const double* dP,
                           double* g, const SysParam* sp, const int* sys, int N)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const SysParam& P = sp[sys[i]];
    const double h = P.dt * P.mu;
    g[i] += h * 2.0 * P.KP * dP[i];
    lx[i] += h * fdx[i];
    ly[i] += h * fdy[i];
}

// deterministic single-block sum of w * qbar (observable accumulation); a
// halted step (host repair pending) adds nothing
__global__ __launch_bounds__(256) void k_qbar_accum(const double* A, const double* P, int N, double w, double* acc,
                                                    const DevState* st)
{
    __shared__ double s[256];
    if (st->halt) return;
    double q = 0.0;
    for (int i = threadIdx.x; i < N; i += 256) q += P[i] / sqrt(A[i]);
    s[threadIdx.x] = q;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *acc += w * s[0] / N;
}

// Every per-cell array of a state in one launch (snapshots of the trajectory).
struct StatePtrs {
    double *x, *y, *th;
    uint8_t* deg;
    int *ring, *opp;
    double *A, *P, *ca, *cb;
};

__global__ void k_state_copy(StatePtrs dst, StatePtrs src, int N, int K)
{
    const size_t nk = (size_t)N * K;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < nk; e += (size_t)gridDim.x * blockDim.x) {
        dst.ring[e] = src.ring[e];
        dst.opp[e] = src.opp[e];
        if (e < (size_t)N) {
            dst.x[e] = src.x[e];
            dst.y[e] = src.y[e];
            dst.th[e] = src.th[e];
            dst.deg[e] = src.deg[e];
            dst.A[e] = src.A[e];
            dst.P[e] = src.P[e];
            dst.ca[e] = src.ca[e];
            dst.cb[e] = src.cb[e];
        }
    }
}

}  // namespace spv
