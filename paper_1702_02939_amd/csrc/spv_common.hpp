// spv_common.hpp -- device data structures, small helpers, Philox noise.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spv {

// error-word bits (device -> host)
enum : unsigned {
    ERR_PRECOND = 1u,    // a Delaunay circumradius reached min(Lx, Ly)/4 (search disk would exceed L/2)
    ERR_CAPACITY = 2u,   // ring longer than kcap or too many repair candidates
    ERR_NONFINITE = 4u,  // non-finite force or position
    ERR_REPAIR = 8u,     // a ring could not be rebuilt
    ERR_DEGREE = 16u,    // ring with fewer than 3 members
};

constexpr int MAX_ROUNDS = 32;  // repair rounds per step (device rounds + host recovery rounds)
constexpr int DENSE_ROUNDS = 2; // rounds of a dense step (flag bytes scanned by the whole grid)

// Per-system constants (a batch holds several independent systems laid out
// one after the other; a single system is a batch of one).
struct SysParam {
    double Lx, Ly, hLx, hLy;  // box (on the grid) and half box
    double iLx, iLy;          // 1 / Lx, 1 / Ly
    double scale, inv_scale;  // 2^q and 2^-q
    double LXu, LYu;          // box in grid units (exact doubles)
    double bsx, bsy;          // bin sides
    double R0;                // first repair search radius
    double mu, v0, dt, amp;   // Eq. 3 and the noise amplitude sqrt(2 Dr dt)
    double KA, KP;            // Eq. 1 moduli
    uint64_t seed;            // Philox key
    int nbx, nby;             // bins per side
    int bin_off;              // first global bin of this system
    int cell_off, n;          // cells [cell_off, cell_off + n)
    int pad;
};

// Device-side control block of one batch.
struct DevState {
    int wl_count[MAX_ROUNDS + 1];  // size of the repair worklist of round r (list r & 1)
    int tl_count[MAX_ROUNDS];      // size of the touched list of round r (list r & 1)
    unsigned err;                  // error word
    int halt;                      // a step did not converge on the device: later kernels do nothing
    int halt_round;                // first round whose worklist is still pending
    int done;                      // tail blocks finished with their share of the step
    unsigned long long disp_bits;  // max |displacement| of the current step (bits of a non-negative double)
    double drift;                  // sum of per-step max displacements since the last re-sort
    double last_drift;             // drift when the last re-sort started
    unsigned long long step;       // completed steps (noise counter of the next step)
    // statistics
    unsigned long long repaired, exact_calls, retries, rounds;
    unsigned long long candidates;  // candidates gathered by the repairs (all attempts)
    int max_deg;
    // first repair failure (diagnostics for the error message)
    int fail_set, fail_cell, fail_n, fail_k, fail_closed, fail_attempts;
    double fail_R, fail_umax;
    // dense rounds: some cell was flagged for round r / touched in round r
    // (plain stores of 1; read by later kernels; cleared when the step closes)
    int dany[DENSE_ROUNDS + 1];
    int tany[DENSE_ROUNDS];
    int dcount[DENSE_ROUNDS];  // cells listed for dense round r
    int scan_done;             // blocks of a scan's first pass finished (reset by the last)
};

// Per-cell arrays of one configuration (the library keeps two and swaps them
// at every re-sort; x, y, theta additionally alternate at every step).
template <typename R>
struct Cells {
    double* x;
    double* y;
    double* th;
    int* tag;    // index of the cell inside its system
    int* sys;    // system of the cell
    double* A0;
    double* P0;
    uint8_t* deg;
    int* ring;   // kcap slots per cell (split rows, rslot), counter-clockwise, starting at the smallest tag
    int* opp;    // the same layout: third vertex across edge (ring[m], ring[m+1])
    int rhi;     // first index of the rows' second parts (RLO x cells of the array set)
    R* A;
    R* P;
    R* ca;       // 2 K_A (A - A0)
    R* cb;       // 2 K_P (P - P0)
};

// Ring and opposite-vertex rows are stored in two parts, so that a cell with
// at most RLO neighbours (nearly all of them) is read as one 32-byte row:
// slot m < RLO of cell i at [i RLO + m], slot m >= RLO at
// [rhi + i (kcap - RLO) + m - RLO], rhi = RLO x the cells of the array set.
constexpr int RLO = 8;

template <int KC>
__host__ __device__ __forceinline__ int rslot(int rhi, int i, int m)
{
    return m < RLO ? i * RLO + m : rhi + i * (KC - RLO) + (m - RLO);
}

__host__ __forceinline__ size_t rslot_host(int rhi, int kc, int i, int m)
{
    return m < RLO ? (size_t)i * RLO + m : (size_t)rhi + (size_t)i * (kc - RLO) + (m - RLO);
}

// Work lists and bitmaps shared by both configurations.
struct Work {
    unsigned* flagbits;   // cell is in the pending repair worklist
    unsigned* touchbits;  // cell is in the pending touched list
    int* wl[2];
    int* tl[2];
    // dense rounds: one byte per cell instead of lists (no append counters)
    uint8_t* flag8;   // flagged for the current dense round
    uint8_t* touch8;  // touched by the current dense round's repairs
    // bins (cells are stored in the order of their global bin at the last re-sort)
    const int* bin_key;     // [sum of bins] spatial bin of a system -> global key
    const int* bin_start;   // [total bins + 1], by key
    const int2* bin_range;  // [sum of bins] cells [x, y) of a spatial bin
    // this step's cell list (null when the repairs use the re-sort's bins):
    // cells cur_cells[cur_start[b] .. cur_start[b + 1]) lie in spatial bin b
    const int* cur_start;   // [sum of bins + 1]
    const int* cur_cells;   // [N]
    // the list's placement, done by the step's all-cells pass (null: none):
    // cell i goes to cplace[cur_start[cbin[i]] + cslot[i]]
    const int* cbin;
    const int* cslot;
    int* cplace;
};

// Bin and slot of every cell in this step's cell list, counted by the force
// kernel's update from the new positions (null count: no list this step).
struct CellCount {
    int* bin;
    int* slot;
    int* count;
};

__host__ __device__ __forceinline__ double mimg(double d, double L, double hL)
{
    return d > hL ? d - L : (d < -hL ? d + L : d);
}

// The same minimum image in three instructions, d - L rint(d / L), for a
// displacement that is known to be short (a Delaunay neighbour: shorter than
// L/2 by the periodic-validity precondition) or near +-L.  The product may
// round, but only within an ulp of +-L/2 could that change the image; the
// result d - kL (k in {-1, 0, 1}) is exact on the position grid.
__device__ __forceinline__ double mimg_near(double d, double L, double iL)
{
    return fma(-L, rint(d * iL), d);
}

// p[j] through a 32-bit byte offset (j >= 0, j * sizeof(T) < 2^32): the
// load then adds the offset to the array's scalar base itself, and arrays
// indexed by the same cell share one offset computation
template <typename T>
__device__ __forceinline__ T at(const T* p, int j)
{
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + (uint32_t)j * (uint32_t)sizeof(T));
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
