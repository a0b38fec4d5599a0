// spv_common.hpp -- device state view, small device helpers, Philox noise.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spv {

// error-word bits (device -> host)
enum : unsigned {
    ERR_PRECOND = 1u,    // a Delaunay circumradius reached min(Lx, Ly)/4, or search radius >= L/2
    ERR_CAPACITY = 2u,   // ring degree above kcap or too many repair candidates
    ERR_NONFINITE = 4u,  // non-finite force or position
    ERR_REPAIR = 8u,     // a ring could not be rebuilt
    ERR_DEGREE = 16u,    // ring with fewer than 3 members
};

// counters read back by the host once per repair round
struct DevCounters {
    int fail_count;          // cells flagged by the validity test
    int wl_count;            // repair worklist size
    int touched_count;       // cells whose neighbourhood changed
    unsigned err;            // error word
    unsigned long long disp_bits;  // max |displacement| of the last update (bits of a non-negative double)
    int exact_calls;         // exact-arithmetic fallbacks of the in-circle filter
    int max_deg;             // largest ring written by the repair
    int repaired;            // cells rebuilt
    int retries;             // repair radius enlargements
    // first repair failure (diagnostics for the error message)
    int fail_cell, fail_n, fail_k, fail_closed, fail_attempts, fail_set;
    double fail_R, fail_umax;
};

// Everything a kernel needs about one system; passed by value.
struct View {
    int N;
    int kcap;
    double Lx, Ly, hLx, hLy;  // box and half box
    double scale, inv_scale;  // 2^q and 2^-q
    double LXu, LYu;          // box in grid units (exact doubles)
    // per-cell state, current buffers
    double* x;
    double* y;
    double* th;
    int* tag;
    double* A0;
    double* P0;
    uint8_t* deg;
    int* ring;  // [kcap][N]
    int* opp;   // [kcap][N]
    double* A;
    double* P;
    double* ca;  // 2 K_A (A - A0)
    double* cb;  // 2 K_P (P - P0)
    // scratch
    uint8_t* flag;
    uint8_t* touched;
    int* worklist;
    int* list2;
    DevCounters* cnt;
    // bins (cells are stored in bin order of the last re-sort)
    int nbx, nby;
    double bsx, bsy;          // bin sides
    const int* bin_rank;      // spatial bin -> position along the Hilbert curve
    const int* bin_start;     // [nbins + 1], indexed by Hilbert position
};

__device__ __forceinline__ double mimg(double d, double L, double hL)
{
    return d > hL ? d - L : (d < -hL ? d + L : d);
}

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of
// (c0, c1, c2, c3) -> (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)),
// key bumped by the Weyl constants between rounds.
__device__ __forceinline__ void philox4x64(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                           uint64_t k1, uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; r++) {
        uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
        uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// 53-bit uniform in the open interval (0, 1)
__device__ __forceinline__ double u01(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53 + 0x1.0p-54; }

// one standard normal for (seed, step, tag): Box-Muller, cosine branch
__device__ __forceinline__ double normal_for(uint64_t seed, uint64_t step, uint64_t tag)
{
    uint64_t r[4];
    philox4x64(step, tag, 0, 0, seed, 0, r);
    double u1 = u01(r[0]), u2 = u01(r[1]);
    return sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
}

}  // namespace spv
