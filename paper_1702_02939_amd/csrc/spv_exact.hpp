// spv_exact.hpp -- exact geometric predicates for the SPV topology test and
// repair on gfx950.
//
// Inputs are minimum-image displacements from the cell at the origin.  Cell
// positions live on the dyadic grid 2^-q (q = 51 - ceil(log2 max(Lx, Ly))),
// so each displacement is an exact double with |d| 2^q < 2^51.  Every sign
// below is therefore exact: a double-precision filter decides the clear cases
// and the rest fall back to integer arithmetic on grid units (int128 for
// orientation, a 256-bit two's-complement accumulator for the in-circle
// determinant, whose magnitude stays below 2^208).
//
// The predicates compile for the host too (the hybrid mode's host repair).
//
// The Delaunay validity of a triangle is the empty-circumcircle property
// (Sussman 2017, Sec. II.C.3).  Four or more cocircular cells are resolved by
// symbolic perturbation of the lifted coordinate |p|^2, the highest-tag point
// carrying the dominant perturbation; the resulting sign is the cofactor of
// that point's row in the 4x4 lifted determinant.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spv {

struct I256 {
    uint64_t w[4];  // little-endian words, two's complement
};

__host__ __device__ __forceinline__ I256 i256_zero() { I256 r; r.w[0] = r.w[1] = r.w[2] = r.w[3] = 0; return r; }

__host__ __device__ __forceinline__ I256 i256_add(const I256& a, const I256& b)
{
    I256 r;
    uint64_t c = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        uint64_t s = a.w[k] + c;
        uint64_t c1 = s < c;
        uint64_t t = s + b.w[k];
        uint64_t c2 = t < s;
        r.w[k] = t;
        c = c1 | c2;
    }
    return r;
}

__host__ __device__ __forceinline__ I256 i256_neg(const I256& a)
{
    I256 r;
    uint64_t c = 1;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        uint64_t t = ~a.w[k] + c;
        c = (c && t == 0) ? 1 : 0;
        r.w[k] = t;
    }
    return r;
}

__host__ __device__ __forceinline__ int i256_sign(const I256& a)
{
    if ((int64_t)a.w[3] < 0) return -1;
    return (a.w[0] | a.w[1] | a.w[2] | a.w[3]) ? 1 : 0;
}

// unsigned 128 x unsigned 128 -> 256
__host__ __device__ __forceinline__ I256 u128_mul(unsigned __int128 a, unsigned __int128 b)
{
    uint64_t a0 = (uint64_t)a, a1 = (uint64_t)(a >> 64), b0 = (uint64_t)b, b1 = (uint64_t)(b >> 64);
    unsigned __int128 p00 = (unsigned __int128)a0 * b0;
    unsigned __int128 p01 = (unsigned __int128)a0 * b1;
    unsigned __int128 p10 = (unsigned __int128)a1 * b0;
    unsigned __int128 p11 = (unsigned __int128)a1 * b1;
    // column sums in 128-bit accumulators
    unsigned __int128 c1 = (p00 >> 64) + (uint64_t)p01 + (uint64_t)p10;
    unsigned __int128 c2 = (c1 >> 64) + (p01 >> 64) + (p10 >> 64) + (uint64_t)p11;
    unsigned __int128 c3 = (c2 >> 64) + (p11 >> 64);
    I256 r;
    r.w[0] = (uint64_t)p00;
    r.w[1] = (uint64_t)c1;
    r.w[2] = (uint64_t)c2;
    r.w[3] = (uint64_t)c3;
    return r;
}

// non-negative 128 x signed 128 -> signed 256
__host__ __device__ __forceinline__ I256 mul_u_s(unsigned __int128 a, __int128 b)
{
    if (b < 0) return i256_neg(u128_mul(a, (unsigned __int128)(-b)));
    return u128_mul(a, (unsigned __int128)b);
}

__host__ __device__ __forceinline__ int64_t to_units(double d, double scale) { return (int64_t)(d * scale); }

__host__ __device__ __forceinline__ int sgn128(__int128 v) { return (v > 0) - (v < 0); }

// sign of b x c (orientation of (0, b, c)); exact
__host__ __device__ __forceinline__ int cross_sign_exact(double bx, double by, double cx, double cy, double scale)
{
    int64_t X1 = to_units(bx, scale), Y1 = to_units(by, scale), X2 = to_units(cx, scale), Y2 = to_units(cy, scale);
    return sgn128((__int128)X1 * Y2 - (__int128)Y1 * X2);
}

// filtered sign of b x c; s must be the double evaluation bx*cy - by*cx
__host__ __device__ __forceinline__ int cross_sign(double bx, double by, double cx, double cy, double s, double scale)
{
    double bound = 1.5e-15 * (fabs(bx * cy) + fabs(by * cx));
    if (s > bound) return 1;
    if (s < -bound) return -1;
    return cross_sign_exact(bx, by, cx, cy, scale);
}

// orientation of (b, c, p): sign of (c - b) x (p - b); exact in units
__host__ __device__ __forceinline__ int orient3_exact(double bx, double by, double cx, double cy, double px, double py,
                                             double scale)
{
    int64_t Bx = to_units(bx, scale), By = to_units(by, scale);
    int64_t Cx = to_units(cx, scale) - Bx, Cy = to_units(cy, scale) - By;
    int64_t Px = to_units(px, scale) - Bx, Py = to_units(py, scale) - By;
    return sgn128((__int128)Cx * Py - (__int128)Cy * Px);
}

// exact value sign of  -( |b|^2 (c x p) + |c|^2 (p x b) + |p|^2 (b x c) )
__host__ __device__ __noinline__ int incircle_exact(double bx, double by, double cx, double cy, double px, double py,
                                           double scale)
{
    int64_t Bx = to_units(bx, scale), By = to_units(by, scale);
    int64_t Cx = to_units(cx, scale), Cy = to_units(cy, scale);
    int64_t Px = to_units(px, scale), Py = to_units(py, scale);
    unsigned __int128 nb = (unsigned __int128)((__int128)Bx * Bx + (__int128)By * By);
    unsigned __int128 nc = (unsigned __int128)((__int128)Cx * Cx + (__int128)Cy * Cy);
    unsigned __int128 np = (unsigned __int128)((__int128)Px * Px + (__int128)Py * Py);
    __int128 cxp = (__int128)Cx * Py - (__int128)Cy * Px;
    __int128 pxb = (__int128)Px * By - (__int128)Py * Bx;
    __int128 bxc = (__int128)Bx * Cy - (__int128)By * Cx;
    I256 s = i256_add(i256_add(mul_u_s(nb, cxp), mul_u_s(nc, pxb)), mul_u_s(np, bxc));
    return -i256_sign(s);
}

// Exact in-circle sign for the cell i at the origin and displacements b, c,
// p, when the double filter could not decide: > 0 iff p lies strictly inside
// the circle through (0, b, c) for (0, b, c) counter-clockwise (the 4x4
// lifted determinant with rows (i, b, c, p)); ties broken by the tags
// (ti, tb, tc, tp).
__host__ __device__ __forceinline__ int incircle_exact_sos(double bx, double by, double cx, double cy, double px, double py,
                                               int ti, int tb, int tc, int tp, double scale)
{
    int s = incircle_exact(bx, by, cx, cy, px, py, scale);
    if (s) return s;
    // cofactor of the highest-tag row of the lifted determinant
    int top = ti, which = 0;
    if (tb > top) { top = tb; which = 1; }
    if (tc > top) { top = tc; which = 2; }
    if (tp > top) { top = tp; which = 3; }
    switch (which) {
    case 0: return orient3_exact(bx, by, cx, cy, px, py, scale);
    case 1: return -cross_sign_exact(cx, cy, px, py, scale);
    case 2: return cross_sign_exact(bx, by, px, py, scale);
    default: return -cross_sign_exact(bx, by, cx, cy, scale);
    }
}

}  // namespace spv
