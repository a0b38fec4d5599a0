// spv_api.hip -- host runtime and C-ABI of the SPV step library (gfx950).
//
// The host side allocates, orders launches on the handle's stream, captures
// whole re-sort periods (resort_every steps + the re-sort) as HIP graphs and
// reads back one small control block per period; every arithmetic step of
// the model runs in the kernels of spv_kernels.hpp.
//
// State: two full sets of per-cell arrays.  In configuration `cfg` set[cfg]
// is current and set[cfg ^ 1] is scratch; x, y, theta additionally alternate
// between the two sets at every step (the update writes the other set, so
// neighbours read step-start positions).  A period has an even number of
// steps, so positions are back in set[cfg] when the re-sort gathers
// everything into set[cfg ^ 1] and the configuration flips.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/spv.h"
#include "spv_adjoint.hpp"
#include "spv_host_repair.hpp"
#include "spv_kernels.hpp"
#include "spv_tune.hpp"

using namespace spv;

// Scratch of spv_force_tangent_static (see static_scratch below).
constexpr int kStaticCells = 65536;
static __device__ __align__(256) double scratch[6 * kStaticCells];

namespace {

thread_local std::string g_err;

spv_status fail(spv_status st, const std::string& msg)
{
    g_err = msg;
    return st;
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(SPV_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));              \
    } while (0)

#define ST_TRY(expr)                   \
    do {                               \
        spv_status st_ = (expr);       \
        if (st_ != SPV_OK) return st_; \
    } while (0)

// ceil(log2 L) exactly, from the binary exponent
int grid_exponent(double Lmax)
{
    int e = 0;
    double f = std::frexp(Lmax, &e);  // Lmax = f 2^e, f in [0.5, 1)
    int c = (f == 0.5) ? e - 1 : e;
    return 51 - c;
}

// position along a Hilbert curve of side n (power of two) of cell (x, y):
// descend the quadrant tree, at each level adding the quadrant's rank in the
// curve's visiting order and reflecting / swapping the coordinates so that
// the sub-square is traversed in the canonical orientation.
int64_t hilbert_index(int64_t n, int64_t x, int64_t y)
{
    int64_t d = 0;
    for (int64_t h = n / 2; h > 0; h /= 2) {
        const int64_t rx = (x & h) ? 1 : 0, ry = (y & h) ? 1 : 0;
        d += h * h * ((3 * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) {
                x = n - 1 - x;
                y = n - 1 - y;
            }
            std::swap(x, y);
        }
    }
    return d;
}

// kernel classes timed by spv_kernel_time
enum { T_FORCE, T_GEOM, T_REPAIR, T_RETEST, T_TAIL, T_LIST, T_COMPACT, T_RESORT, T_HOST, T_COUNT };

// Scratch of spv_force_tangent_static (the entry point that allocates
// nothing): v in memory order (2 N), the tangents of A and P (2 N) and the
// result in memory order (2 N) for at most kStaticCells cells -- 6 x 65536
// doubles = 3 MiB, which every device the library runs on holds until the
// process ends.  Host code never passes the array's name to a kernel (on the
// host it is only a stand-in for the symbol): it uses the device address
// taken once per device by static_scratch().
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
double* g_scratch_ptr[kMaxDevices] = {};

// the current device's address of `scratch` (looked up on first use)
spv_status static_scratch(double** out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SPV_EINVAL, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SPV_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return SPV_OK;
}

struct ArraySet {
    double *x = nullptr, *y = nullptr, *th = nullptr;
    int *tag = nullptr, *sys = nullptr;
    double *A0 = nullptr, *P0 = nullptr;
    uint8_t* deg = nullptr;
    int *ring = nullptr, *opp = nullptr;
    void *A = nullptr, *P = nullptr, *ca = nullptr, *cb = nullptr;  // R-typed
};

struct EvPair {
    hipEvent_t a = nullptr, b = nullptr;
};

// Device copy of the dynamic state of a single-system handle (positions,
// directors, topology, geometry and energy coefficients), FP64.
struct Snapshot {
    double *x = nullptr, *y = nullptr, *th = nullptr;
    uint8_t* deg = nullptr;
    int *ring = nullptr, *opp = nullptr;
    double *A = nullptr, *P = nullptr, *ca = nullptr, *cb = nullptr;
};

struct TrajCheckpoint {
    Snapshot snap;
    double* acc = nullptr;  // accumulated observable at the checkpoint (device)
    int pos = 0;
    uint64_t step = 0;
};

}  // namespace

struct spv_sys {
    int S = 1, N = 0, KC = 16;
    double* scratch = nullptr;  // this device's address of the static scratch array
    int dev_rounds = 2, max_rounds = 16, unit = 16;
    int repair_cells = 64;  // repair grid = N / this (clamped to [256, 4096] blocks)
    int tail_items = 64;    // largest later round the one-block tail takes
    int full_rounds = 1;    // repair rounds over the whole grid before the tail
    int force_mode = 0;     // force kernel: 1 lanes per cell, 2 per (cell, slot) item, 0 by size
    int dense = 0;          // dense first rounds: 0 while hot, 1 never, 2 always
    int repair_mode = 0;    // 0 device repair, 1 hybrid (device test, host repair)
    bool never_resort = false;  // no spatial re-sort: repairs always search the step's cell list
    // dense first rounds after the hot phase too, while the measured repairs
    // per step stay above N / 64 (on) / N / 256 (off again)
    bool dense_busy = false;
    // adaptive re-sort: while cells move fast (the drift of a period exceeds
    // drift_limit, one bin side) steps run eagerly and re-sort as soon as
    // the drift passes the limit; a full quiet period returns to graphs
    bool hot = true;
    int quiet = 0;
    double drift_limit = 1.0;
    double drift_rate = INFINITY;  // drift added per step over the last eager batch (unknown: one step)
    double bin_factor = 1.0;
    int tune_source = 0;
    double tune_ms = 0.0;
    bool mixed = false, multi = false, use_graphs = true;
    spv_params prm{};
    hipStream_t stream = nullptr;      // caller's stream (all work is ordered on it)
    hipStream_t cap_stream = nullptr;  // private stream used only to capture graphs
    std::vector<SysParam> hsp;
    std::vector<int> cell_off;
    SysParam* d_sp = nullptr;
    ArraySet set[2];
    int cfg = 0, pos = 0;              // configuration and steps done in the current period
    Work work{};
    int total_bins = 0;
    int *d_bin_key = nullptr, *d_bin_start = nullptr, *d_key = nullptr, *d_hist = nullptr, *d_fill = nullptr;
    int *d_perm = nullptr, *d_inv = nullptr, *d_chunk = nullptr;
    int2* d_bin_range = nullptr;
    // cell list of a step (while hot)
    int *d_cbin = nullptr, *d_cslot = nullptr, *d_ccount = nullptr, *d_cstart = nullptr, *d_ccells = nullptr;
    int* d_cchunk = nullptr;
    DevState* d_st = nullptr;
    DevState* h_st = nullptr;  // pinned copy
    double *d_stage = nullptr, *d_fx = nullptr, *d_fy = nullptr, *d_obs = nullptr, *d_blockmax = nullptr;
    double* d_obs_part = nullptr;  // [S][obs_chunks][3]
    int obs_chunks = 1;
    std::vector<void*> allocs;
    // graphs of one period starting in configuration 0 / 1
    // graphs of one period starting in configuration 0 / 1, by period length
    std::map<std::pair<int, int>, hipGraphExec_t> graphs;
    std::map<std::vector<int64_t>, hipGraphExec_t> tgraphs;  // trajectory segments (adjoint), by shape

    // bookkeeping
    uint64_t step = 0;
    int64_t resorts = 0;
    int64_t graph_periods = 0;  // re-sort periods replayed as a captured graph
    int64_t dense_steps = 0;    // steps whose first repair rounds ran dense
    int64_t host_rounds = 0;    // repair rounds run by host recovery
    int64_t recoveries = 0;     // steps finished by host recovery
    // hybrid mode: host repair, pinned staging and the device row buffers
    HostRepair hr;
    int64_t hyb_repaired = 0, hyb_rounds = 0;
    double *h_x = nullptr, *h_y = nullptr;
    int *h_tag = nullptr, *h_sys = nullptr, *h_list = nullptr, *h_rows = nullptr, *h_new = nullptr,
        *h_touch = nullptr;
    int *d_rows = nullptr, *d_new = nullptr;
    std::vector<uint8_t> h_mark;
    spv_status sticky = SPV_OK;
    std::string sticky_msg;
    // timing
    bool timing = false;
    double t_ms[T_COUNT] = {};
    int64_t t_n[T_COUNT] = {};
    std::vector<std::pair<int, EvPair>> pending;  // eager launches
    std::vector<EvPair> pool;
    // trajectory adjoint
    bool no_resort = false;       // keep the memory order fixed during a recorded trajectory
    int64_t traj_T = 0, traj_k = 0;
    bool traj_valid = false;
    std::vector<TrajCheckpoint> ckpt;  // state at steps 0, k, 2k, ... and at T (last)
    std::vector<Snapshot> seg;         // per-step states of the segment being differentiated
    double *d_lx = nullptr, *d_ly = nullptr, *d_g = nullptr, *d_dA = nullptr, *d_dP = nullptr;
    double *d_fdx = nullptr, *d_fdy = nullptr, *d_aq = nullptr, *d_bq = nullptr, *d_acc = nullptr;
    double *d_lx2 = nullptr, *d_ly2 = nullptr;  // the adjoint's second buffer
};

namespace {

template <class T>
spv_status dalloc(spv_sys* s, T** p, size_t count)
{
    void* q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        return fail(SPV_ENOMEM, "hipMalloc failed");
    }
    s->allocs.push_back(q);
    *p = static_cast<T*>(q);
    return SPV_OK;
}

spv_status alloc_set(spv_sys* s, ArraySet& a)
{
    const size_t N = s->N, K = s->KC, rs = s->mixed ? sizeof(float) : sizeof(double);
    ST_TRY(dalloc(s, &a.x, N));
    ST_TRY(dalloc(s, &a.y, N));
    ST_TRY(dalloc(s, &a.th, N));
    ST_TRY(dalloc(s, &a.tag, N));
    ST_TRY(dalloc(s, &a.sys, N));
    ST_TRY(dalloc(s, &a.A0, N));
    ST_TRY(dalloc(s, &a.P0, N));
    ST_TRY(dalloc(s, &a.deg, N));
    ST_TRY(dalloc(s, &a.ring, N * K));
    ST_TRY(dalloc(s, &a.opp, N * K));
    uint8_t* raw = nullptr;
    ST_TRY(dalloc(s, &raw, 4 * N * rs));
    a.A = raw;
    a.P = raw + N * rs;
    a.ca = raw + 2 * N * rs;
    a.cb = raw + 3 * N * rs;
    HIP_TRY(hipMemsetAsync(a.deg, 0, N, s->stream));
    HIP_TRY(hipMemsetAsync(a.ring, 0, N * K * sizeof(int), s->stream));
    HIP_TRY(hipMemsetAsync(a.opp, 0xff, N * K * sizeof(int), s->stream));
    HIP_TRY(hipMemsetAsync(raw, 0, 4 * N * rs, s->stream));
    return SPV_OK;
}

template <typename R>
Cells<R> cells(const spv_sys* s, int cfg, int parity)
{
    const ArraySet& P = s->set[cfg];
    const ArraySet& Q = s->set[cfg ^ 1];
    Cells<R> c;
    c.x = parity ? Q.x : P.x;
    c.y = parity ? Q.y : P.y;
    c.th = parity ? Q.th : P.th;
    c.tag = P.tag;
    c.sys = P.sys;
    c.A0 = P.A0;
    c.P0 = P.P0;
    c.deg = P.deg;
    c.ring = P.ring;
    c.opp = P.opp;
    c.rhi = RLO * s->N;
    c.A = static_cast<R*>(P.A);
    c.P = static_cast<R*>(P.P);
    c.ca = static_cast<R*>(P.ca);
    c.cb = static_cast<R*>(P.cb);
    return c;
}

// run f.template operator()<R, MULTI, KC>() for the handle's instantiation
template <class F>
void dispatch(const spv_sys* s, F&& f)
{
    if (s->mixed) {
        if (s->multi) {
            if (s->KC == 16) f.template operator()<float, true, 16>();
            else f.template operator()<float, true, 32>();
        } else {
            if (s->KC == 16) f.template operator()<float, false, 16>();
            else f.template operator()<float, false, 32>();
        }
    } else {
        if (s->multi) {
            if (s->KC == 16) f.template operator()<double, true, 16>();
            else f.template operator()<double, true, 32>();
        } else {
            if (s->KC == 16) f.template operator()<double, false, 16>();
            else f.template operator()<double, false, 32>();
        }
    }
}

inline unsigned grid_for(int n, int block) { return (unsigned)std::max(1, (n + block - 1) / block); }

// all-cell grid of the 8-lanes-per-cell kernels, padded to a multiple of 8 XCDs
inline unsigned cell_grid(const spv_sys* s) { return (grid_for(s->N, CPB) + 7u) & ~7u; }
// the force kernel's grid (its own cells per block), also padded
inline bool items_kernel(const spv_sys* s);
inline unsigned force_grid(const spv_sys* s)
{
    const int cpb = items_kernel(s) ? items_cells_per_block(s->KC) : force_cells_per_block(s->KC);
    return (grid_for(s->N, cpb) + 7u) & ~7u;
}
// the force kernel of the handle (both give bitwise the same forces)
constexpr int kItemsFromCells = 1 << 18;
inline bool items_kernel(const spv_sys* s)
{
    return s->force_mode == 2 || (s->force_mode == 0 && s->N >= kItemsFromCells);
}
template <typename R, bool MULTI, int KC, bool UPDATE, bool ACC = false>
auto force_kernel(const spv_sys* s)
{
    return items_kernel(s) ? k_force_items<R, MULTI, KC, UPDATE, ACC> : k_force_cells<R, MULTI, KC, UPDATE, ACC>;
}
// the tail grid shares the re-test of the last full-grid round: 32 blocks
// from up to 2^18 cells, then one per 8192 cells, at most 128 (N = 1e6:
// step 239.5 -> 233.6 us; more blocks at N = 1e5 only add to the hand-over)
inline unsigned tail_grid(const spv_sys* s)
{
    return (unsigned)std::min(std::max(s->N / 8192, TAIL_BLOCKS), 128);
}
inline unsigned repair_grid(const spv_sys* s)
{
    return (unsigned)std::min(std::max(s->N / s->repair_cells, 256), 4096);
}

// ---------------------------------------------------------------- timing
EvPair take_events(spv_sys* s)
{
    EvPair e;
    if (!s->pool.empty()) {
        e = s->pool.back();
        s->pool.pop_back();
    } else {
        (void)hipEventCreate(&e.a);
        (void)hipEventCreate(&e.b);
    }
    return e;
}

void collect_eager_timing(spv_sys* s)
{
    for (auto& t : s->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, t.second.a, t.second.b) == hipSuccess) {
            s->t_ms[t.first] += ms;
            s->t_n[t.first] += 1;
        }
        s->pool.push_back(t.second);
    }
    s->pending.clear();
}

// ---------------------------------------------------------------- launch sequences
// Launch on `st`; with an event pair (timing), the events are attached to the
// dispatch itself (start and end of the kernel's execution).
template <typename K, typename... Args>
void launch(EvPair ev, K kernel, dim3 grid, dim3 block, hipStream_t st, Args... args)
{
    if (ev.a)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, st, ev.a, ev.b, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
}

// the event pair of the next launch of kernel class `cat` while timing
// (none otherwise; timing never coincides with graph capture)
EvPair tev(spv_sys* s, int cat)
{
    if (!s->timing) return EvPair{};
    EvPair e = take_events(s);
    s->pending.push_back({cat, e});
    return e;
}

inline bool dense_step(const spv_sys* s, bool hot)
{
    return s->dense == 2 || (s->dense == 0 && (hot || s->dense_busy));
}

// after `done` steps that repaired `rep` cells: dense rounds while repairs
// are many (a large share of the cells failing, as in the fluid regime)
void note_repairs(spv_sys* s, uint64_t rep, uint64_t done)
{
    if (!done) return;
    const double per = (double)rep / (double)done;
    if (per > s->N / 64.0) s->dense_busy = true;
    else if (per < s->N / 256.0) s->dense_busy = false;
}

// the work lists, with this step's cell list for the repairs when cur
// place: the step's all-cells pass also places the cells of this step's list
Work work_for(const spv_sys* s, bool cur, bool place = false)
{
    Work w = s->work;
    w.cur_start = cur ? s->d_cstart : nullptr;
    w.cur_cells = cur ? s->d_ccells : nullptr;
    w.cbin = (cur && place) ? s->d_cbin : nullptr;
    w.cslot = (cur && place) ? s->d_cslot : nullptr;
    w.cplace = (cur && place) ? s->d_ccells : nullptr;
    return w;
}

// the counting half of this step's cell list (done by the force kernel's
// update; the counts are zero here: cleared at creation and by every list's
// scan)
CellCount cell_count_for(const spv_sys* s, bool cur)
{
    return cur ? CellCount{s->d_cbin, s->d_cslot, s->d_ccount} : CellCount{nullptr, nullptr, nullptr};
}

// the counts of this step's cell list into bin starts
void enqueue_cell_scan(spv_sys* s, hipStream_t st)
{
    const int nb = s->total_bins;
    const unsigned nchunk = grid_for(nb, SCAN_CHUNK);
    launch(tev(s, T_LIST), k_scan_sums_last, dim3(nchunk), dim3(256), st, (const int*)s->d_ccount, nb, s->d_cchunk,
           s->d_st);
    launch(tev(s, T_LIST), k_scan_apply<true>, dim3(nchunk), dim3(256), st, s->d_ccount, s->d_cstart, nb,
           (const int*)s->d_cchunk, (const DevState*)s->d_st);
}

// wavefronts of a dense repair round: about one per four cells, at most
// what the chip holds at once (256 CUs x 4 SIMDs x 4 wavefronts of
// k_repair_dense's register budget)
inline unsigned dense_repair_grid(const spv_sys* s) { return (unsigned)std::min(std::max(s->N / 4, 64), 4096); }

// The repair rounds of a dense step: rounds 0 .. nd-1 scan flag and touched
// bytes over the whole grid, the tail takes the rest from the worklist of
// round nd.
template <typename R, bool MULTI, int KC>
void enqueue_dense_rounds(spv_sys* s, hipStream_t st, const Cells<R>& nxt, const Work& wk)
{
    const int nd = std::min(DENSE_ROUNDS, s->dev_rounds);
    const unsigned tg = (grid_for(s->N, DENSE_TCHUNK) + 7u) & ~7u;
    const SysParam* sp = s->d_sp;
    for (int r = 0; r < nd; r++) {
        launch(tev(s, T_COMPACT), k_compact_flags, dim3(grid_for(s->N, COMPACT_CELLS)), dim3(256), st, wk, s->d_st,
               r);
        launch(tev(s, T_REPAIR), k_repair_dense<R, MULTI, KC>, dim3(dense_repair_grid(s)), dim3(64), st, nxt, wk, sp,
               s->d_st, r, nd);
        if (r + 1 < nd)
            launch(tev(s, T_RETEST), k_retest_dense<R, MULTI, KC, false>, dim3(tg), dim3(256), st, nxt, wk, sp,
                   s->d_st, s->N, r);
        else
            launch(tev(s, T_RETEST), k_retest_dense<R, MULTI, KC, true>, dim3(tg), dim3(256), st, nxt, wk, sp,
                   s->d_st, s->N, r);
    }
    launch(tev(s, T_TAIL), k_tail<R, MULTI, KC>, dim3(tail_grid(s)), dim3(TAIL_THREADS), st, nxt, wk, sp, s->d_st,
           s->dev_rounds, s->tail_items, nd);
}

// One step on stream `st` from (cfg, parity).  hot: the step of the
// fast-moving phase (its repairs search a cell list of the step's positions;
// dense first rounds unless switched off).
template <typename R, bool MULTI, int KC>
void enqueue_step(spv_sys* s, hipStream_t st, int cfg, int parity, bool hot)
{
    Cells<R> cur = cells<R>(s, cfg, parity), nxt = cells<R>(s, cfg, parity ^ 1);
    const unsigned cg = cell_grid(s), rg = repair_grid(s);
    const SysParam* sp = s->d_sp;
    // the repairs search this step's cell list while cells move fast, and
    // always when the memory order is never re-sorted
    const bool curl = hot || s->never_resort;
    launch(tev(s, T_FORCE), force_kernel<R, MULTI, KC, true>(s), dim3(force_grid(s)), dim3(256), st, cur, nxt.x,
           nxt.y, nxt.th, (double*)nullptr, (double*)nullptr, sp, s->d_st, s->N, s->d_blockmax, cell_count_for(s, curl));
    if (curl) enqueue_cell_scan(s, st);
    const Work wk = work_for(s, curl), wplace = work_for(s, curl, true);
    const bool dense = dense_step(s, hot);
    const double* bmax = s->d_blockmax;
    if (items_kernel(s)) {
        const dim3 g((grid_for(s->N, items_cells_per_block(KC)) + 7u) & ~7u);
        if (dense)
            launch(tev(s, T_GEOM), k_geom_items<R, MULTI, KC, true>, g, dim3(256), st, nxt, wplace, sp, s->d_st,
                   s->N, bmax, (int)force_grid(s));
        else
            launch(tev(s, T_GEOM), k_geom_items<R, MULTI, KC>, g, dim3(256), st, nxt, wplace, sp, s->d_st, s->N, bmax,
                   (int)force_grid(s));
    } else {
        if (dense)
            launch(tev(s, T_GEOM), k_geom<R, MULTI, KC, false, false, true, true>, dim3(cg), dim3(256), st, nxt,
                   wplace, sp, s->d_st, s->N, 0, bmax, (int)force_grid(s));
        else
            launch(tev(s, T_GEOM), k_geom<R, MULTI, KC, false, false, true>, dim3(cg), dim3(256), st, nxt, wplace, sp,
                   s->d_st, s->N, 0, bmax, (int)force_grid(s));
    }
    if (dense) {
        enqueue_dense_rounds<R, MULTI, KC>(s, st, nxt, wk);
        return;
    }
    // rounds 0 .. f-1 over the whole grid; the last one's re-test, later
    // rounds and the step's close in the tail
    // while cells move fast (hot), rounds 1 .. 3 are big too: all of them over
    // the whole grid, so that a step rarely stops for host rounds
    const int f = std::min(hot ? MAX_FULL_ROUNDS : s->full_rounds, s->dev_rounds);
    launch(tev(s, T_REPAIR), k_repair<R, MULTI, KC>, dim3(rg), dim3(64), st, nxt, wk, sp, s->d_st, 0);
    for (int r = 1; r < f; r++) {
        launch(tev(s, T_RETEST), k_geom<R, MULTI, KC, true, true>, dim3(std::min(grid_for(s->N, CPB), 512u)),
               dim3(256), st, nxt, wk, sp, s->d_st, s->N, r - 1, (const double*)nullptr, 0);
        launch(tev(s, T_REPAIR), k_repair<R, MULTI, KC>, dim3(rg), dim3(64), st, nxt, wk, sp, s->d_st, r);
    }
    launch(tev(s, T_TAIL), k_tail<R, MULTI, KC>, dim3(tail_grid(s)), dim3(TAIL_THREADS), st, nxt, wk, sp, s->d_st,
           s->dev_rounds, s->tail_items, f);
}

// Re-sort from (cfg, parity 0) into set[cfg ^ 1] (the caller flips cfg).
template <typename R, bool MULTI, int KC>
void enqueue_resort(spv_sys* s, hipStream_t st, int cfg)
{
    Cells<R> src = cells<R>(s, cfg, 0), dst = cells<R>(s, cfg ^ 1, 0);
    const int N = s->N, nb = s->total_bins;
    const unsigned nchunk = grid_for(nb, SCAN_CHUNK);
    launch(tev(s, T_RESORT), k_fill_i32, dim3(grid_for(nb, 256)), dim3(256), st, s->d_hist, nb, 0);
    launch(tev(s, T_RESORT), k_fill_i32, dim3(grid_for(nb, 256)), dim3(256), st, s->d_fill, nb, 0);
    launch(tev(s, T_RESORT), k_bin_keys<R, MULTI>, dim3(grid_for(N, 256)), dim3(256), st, src, s->work,
           (const SysParam*)s->d_sp, (const DevState*)s->d_st, N, s->d_key, s->d_hist);
    launch(tev(s, T_RESORT), k_scan_sums_last, dim3(nchunk), dim3(256), st, (const int*)s->d_hist, nb, s->d_chunk,
           s->d_st);
    launch(tev(s, T_RESORT), k_scan_apply<false>, dim3(nchunk), dim3(256), st, s->d_hist, s->d_bin_start, nb,
           (const int*)s->d_chunk, (const DevState*)s->d_st);
    launch(tev(s, T_RESORT), k_bin_scatter, dim3(grid_for(N, 256)), dim3(256), st, (const int*)s->d_key,
           (const int*)s->d_bin_start, s->d_fill, s->d_perm, N, (const DevState*)s->d_st);
    launch(tev(s, T_RESORT), k_bin_sort, dim3(grid_for(nb, 256)), dim3(256), st, (const int*)s->d_bin_start,
           (const int*)s->d_bin_key, s->d_bin_range, s->d_perm, (const int*)src.tag, nb, (const DevState*)s->d_st);
    launch(tev(s, T_RESORT), k_inv_perm, dim3(grid_for(N, 256)), dim3(256), st, (const int*)s->d_perm, s->d_inv, N,
           (const DevState*)s->d_st);
    launch(tev(s, T_RESORT), k_gather<R, KC>, dim3(grid_for(N, 256)), dim3(256), st, src, dst, (const int*)s->d_perm,
           (const int*)s->d_inv, N, s->d_st);
}

// one host-driven repair round (creation and recovery); cur: the halted
// step built a cell list of the current positions
template <typename R, bool MULTI, int KC>
void enqueue_round(spv_sys* s, hipStream_t st, int round, unsigned rgrid, bool curlist)
{
    Cells<R> cur = cells<R>(s, s->cfg, s->pos & 1);
    const SysParam* sp = s->d_sp;
    launch(tev(s, T_HOST), k_repair<R, MULTI, KC>, dim3(rgrid), dim3(64), st, cur, work_for(s, curlist), sp, s->d_st,
           round);
    launch(tev(s, T_HOST), k_geom<R, MULTI, KC, true, true>, dim3(std::min(grid_for(s->N, CPB), 4096u)), dim3(256), st,
           cur, s->work, sp, s->d_st, s->N, round, (const double*)nullptr, 0);
}

// ---------------------------------------------------------------- control block
spv_status read_state(spv_sys* s)
{
    HIP_TRY(hipMemcpyAsync(s->h_st, s->d_st, sizeof(DevState), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    HIP_TRY(hipGetLastError());
    collect_eager_timing(s);
    return SPV_OK;
}

spv_status error_from_word(spv_sys* s)
{
    const DevState& d = *s->h_st;
    const unsigned e = d.err;
    char buf[400];
    std::snprintf(buf, sizeof buf,
                  "device error word 0x%x at step %llu (first repair failure: tag %d, %d candidates, ring %d, "
                  "closed %d, %d attempts, R %.4g, max circumradius %.4g)",
                  e, (unsigned long long)d.step, d.fail_set ? d.fail_cell : -1, d.fail_n, d.fail_k, d.fail_closed,
                  d.fail_attempts, d.fail_R, d.fail_umax);
    spv_status st = SPV_EREPAIR;
    std::string what = ": ring could not be rebuilt";
    if (e & ERR_NONFINITE) {
        st = SPV_ENONFINITE;
        what = ": non-finite force or position";
    } else if (e & ERR_PRECOND) {
        st = SPV_EPRECOND;
        what = ": a Delaunay circumradius reached min(Lx,Ly)/4";
    } else if (e & ERR_CAPACITY) {
        st = SPV_ECAPACITY;
        what = ": ring longer than kcap or too many repair candidates";
    } else if (e & ERR_DEGREE) {
        what = ": ring with fewer than 3 cells";
    }
    s->sticky = st;
    s->sticky_msg = std::string(buf) + what;
    return fail(st, s->sticky_msg);
}

// Finish the repair of the halted step on the host side: more rounds, each
// read back, until no flag is left.
spv_status recover(spv_sys* s, bool curlist)
{
    if (s->h_st->err) return error_from_word(s);
    int r = s->h_st->halt_round;
    s->recoveries++;
    hipLaunchKernelGGL(k_set_halt, dim3(1), dim3(64), 0, s->stream, s->d_st, 0);
    while (true) {
        if (r >= s->max_rounds || r >= MAX_ROUNDS) {
            s->sticky = SPV_EREPAIR;
            s->sticky_msg = "topology repair did not converge within repair_rounds";
            return fail(SPV_EREPAIR, s->sticky_msg);
        }
        const unsigned rg = (unsigned)std::min(std::max(s->h_st->wl_count[r], 1), 65535);
        dispatch(s, [&]<typename R, bool MULTI, int KC>() {
            enqueue_round<R, MULTI, KC>(s, s->stream, r, rg, curlist);
        });
        HIP_TRY(hipGetLastError());
        ST_TRY(read_state(s));
        s->host_rounds++;
        if (s->h_st->err) return error_from_word(s);
        if (s->h_st->wl_count[r + 1] == 0) break;
        r++;
    }
    hipLaunchKernelGGL(k_resume, dim3(1), dim3(64), 0, s->stream, s->d_st);
    HIP_TRY(hipGetLastError());
    return SPV_OK;
}

// The graph of a period of gu steps (then the re-sort) from configuration g,
// captured on first use.
spv_status period_graph(spv_sys* s, int g, int gu, hipGraphExec_t* out)
{
    const int key = 2 * gu + (dense_step(s, false) ? 1 : 0);  // the dense flavour is captured too
    auto it = s->graphs.find({g, key});
    if (it != s->graphs.end()) {
        *out = it->second;
        return SPV_OK;
    }
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeRelaxed));
    for (int k = 0; k < gu; k++)
        dispatch(s, [&]<typename R, bool MULTI, int KC>() {
            enqueue_step<R, MULTI, KC>(s, s->cap_stream, g, k & 1, false);
        });
    if (!s->never_resort)
        dispatch(s, [&]<typename R, bool MULTI, int KC>() { enqueue_resort<R, MULTI, KC>(s, s->cap_stream, g); });
    hipError_t e0 = hipGetLastError();
    hipError_t e1 = hipStreamEndCapture(s->cap_stream, &graph);
    if (e1 == hipSuccess && e0 != hipSuccess) e1 = e0;
    if (e1 != hipSuccess) return fail(SPV_EHIP, std::string("graph capture: ") + hipGetErrorString(e1));
    hipGraphExec_t ex = nullptr;
    hipError_t e2 = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) return fail(SPV_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e2));
    s->graphs[{g, key}] = ex;
    *out = ex;
    return SPV_OK;
}

// Steps per captured period: the re-sort period, or else the longest multiple
// of 8 steps below it over which the drift bound stays within the limit at
// the measured drift rate (so that the repair searches stay about as wide as
// the bins); 0 when not even 8 steps do (the steps then run eagerly, with
// re-sorts as soon as the drift passes the limit).
int graph_unit(const spv_sys* s)
{
    const double r = s->drift_rate;
    if (!(r * s->unit > s->drift_limit)) return s->unit;
    for (int u = (s->unit - 1) / 8 * 8; u >= 8; u -= 8)
        if (r * u <= s->drift_limit) return u;
    return 0;
}

spv_status do_resort_eager(spv_sys* s)
{
    dispatch(s, [&]<typename R, bool MULTI, int KC>() { enqueue_resort<R, MULTI, KC>(s, s->stream, s->cfg); });
    HIP_TRY(hipGetLastError());
    // the host mirror follows what k_gather does on the device, so that the
    // next batch is sized from a zero drift
    s->h_st->last_drift = s->h_st->drift;
    s->h_st->drift = 0.0;
    s->cfg ^= 1;
    s->pos = 0;
    s->resorts++;
    return SPV_OK;
}

// ---------------------------------------------------------------- hybrid comparison mode
// A step: forces and update, then the validity test of every ring (failures
// to the worklist of round 0), on the device.
template <typename R, bool MULTI, int KC>
void enqueue_test(spv_sys* s, hipStream_t st, int cfg, int parity)
{
    Cells<R> cur = cells<R>(s, cfg, parity), nxt = cells<R>(s, cfg, parity ^ 1);
    const SysParam* sp = s->d_sp;
    const double* bmax = s->d_blockmax;
    launch(tev(s, T_FORCE), force_kernel<R, MULTI, KC, true>(s), dim3(force_grid(s)), dim3(256), st, cur, nxt.x,
           nxt.y, nxt.th, (double*)nullptr, (double*)nullptr, sp, s->d_st, s->N, s->d_blockmax, CellCount{});
    if (items_kernel(s))
        launch(tev(s, T_GEOM), k_geom_items<R, MULTI, KC>,
               dim3((grid_for(s->N, items_cells_per_block(KC)) + 7u) & ~7u), dim3(256), st, nxt, s->work, sp,
               s->d_st, s->N, bmax, (int)force_grid(s));
    else
        launch(tev(s, T_GEOM), k_geom<R, MULTI, KC, false, false, true>, dim3(cell_grid(s)), dim3(256), st, nxt,
               s->work, sp, s->d_st, s->N, 0, bmax, (int)force_grid(s));
}

// Round r of a hybrid step: the worklist, the listed cells' old rows and (in
// the first round) the positions, tags and systems go to the host; the host
// rebuilds the rings; the new rows and the touched cells come back, and the
// device re-tests the touched cells (failures to the worklist of round r + 1).
template <typename R, bool MULTI, int KC>
spv_status hybrid_round(spv_sys* s, int r, bool first)
{
    const int n = s->h_st->wl_count[r], N = s->N;
    hipStream_t st = s->stream;
    Cells<R> c = cells<R>(s, s->cfg, s->pos & 1);
    const int* wl = s->work.wl[r & 1];
    HIP_TRY(hipMemcpyAsync(s->h_list, wl, (size_t)n * sizeof(int), hipMemcpyDeviceToHost, st));
    launch(tev(s, T_HOST), k_pack_rows<KC>, dim3(grid_for(n, 256)), dim3(256), st, wl, n, (const uint8_t*)c.deg,
           (const int*)c.ring, c.rhi, s->d_rows);
    HIP_TRY(hipMemcpyAsync(s->h_rows, s->d_rows, (size_t)n * (KC + 1) * sizeof(int), hipMemcpyDeviceToHost, st));
    if (first) {
        HIP_TRY(hipMemcpyAsync(s->h_x, c.x, (size_t)N * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(s->h_y, c.y, (size_t)N * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(s->h_tag, c.tag, (size_t)N * sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(s->h_sys, c.sys, (size_t)N * sizeof(int), hipMemcpyDeviceToHost, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    if (first) s->hr.build(s->h_x, s->h_y, s->h_sys, N, s->hsp, s->total_bins);
    int nt = 0;
    auto touch = [&](int q) {
        if (q >= 0 && !s->h_mark[q]) {
            s->h_mark[q] = 1;
            s->h_touch[nt++] = q;
        }
    };
    for (int t = 0; t < n; t++) {
        const int i = s->h_list[t];
        const unsigned e = s->hr.repair(i, s->h_x, s->h_y, s->h_tag, s->h_sys, s->hsp, KC);
        if (e) {
            for (int q = 0; q < nt; q++) s->h_mark[s->h_touch[q]] = 0;
            s->sticky = (e & ERR_PRECOND) ? SPV_EPRECOND : (e & ERR_CAPACITY) ? SPV_ECAPACITY : SPV_EREPAIR;
            s->sticky_msg = "host repair (hybrid mode) failed at step " + std::to_string(s->step) + " for tag " +
                            std::to_string(s->h_tag[i]);
            return fail(s->sticky, s->sticky_msg);
        }
        const int* old = s->h_rows + (size_t)t * (KC + 1);
        for (int m = 0; m < old[0]; m++) touch(old[1 + m]);
        int* row = s->h_new + (size_t)t * (KC + 2);
        const int k = (int)s->hr.ring.size();
        row[0] = i;
        row[1] = k;
        for (int m = 0; m < k; m++) {
            row[2 + m] = s->hr.ring[m];
            touch(s->hr.ring[m]);
        }
        touch(i);
    }
    for (int q = 0; q < nt; q++) s->h_mark[s->h_touch[q]] = 0;
    HIP_TRY(hipMemcpyAsync(s->d_new, s->h_new, (size_t)n * (KC + 2) * sizeof(int), hipMemcpyHostToDevice, st));
    launch(tev(s, T_HOST), k_unpack_rows<KC>, dim3(grid_for(n, 256)), dim3(256), st, (const int*)s->d_new, n, c.deg,
           c.ring, c.rhi, s->work.flagbits);
    HIP_TRY(hipMemcpyAsync(s->work.tl[r & 1], s->h_touch, (size_t)nt * sizeof(int), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(reinterpret_cast<char*>(s->d_st) + offsetof(DevState, tl_count) + r * sizeof(int), &nt,
                           sizeof(int), hipMemcpyHostToDevice, st));
    launch(tev(s, T_HOST), k_geom<R, MULTI, KC, true, true>, dim3(std::min(grid_for(N, CPB), 4096u)), dim3(256), st,
           c, s->work, (const SysParam*)s->d_sp, s->d_st, N, r, (const double*)nullptr, 0);
    s->hyb_repaired += n;
    s->hyb_rounds++;
    return read_state(s);
}

spv_status run_steps_hybrid(spv_sys* s, int64_t n)
{
    for (; n > 0; n--) {
        if (!(s->pos & 1) && s->pos > 0 && s->pos >= s->unit && !s->never_resort) ST_TRY(do_resort_eager(s));
        const int cfg = s->cfg, par = s->pos & 1;
        dispatch(s, [&]<typename R, bool MULTI, int KC>() { enqueue_test<R, MULTI, KC>(s, s->stream, cfg, par); });
        HIP_TRY(hipGetLastError());
        ST_TRY(read_state(s));  // the worklist size: the per-step device-to-host round trip
        if (s->h_st->err) return error_from_word(s);
        s->step += 1;
        s->pos += 1;
        for (int r = 0; s->h_st->wl_count[r] > 0; r++) {
            if (r >= s->max_rounds || r + 1 >= MAX_ROUNDS) {
                s->sticky = SPV_EREPAIR;
                s->sticky_msg = "topology repair did not converge within repair_rounds";
                return fail(SPV_EREPAIR, s->sticky_msg);
            }
            spv_status st = SPV_OK;
            dispatch(s, [&]<typename R, bool MULTI, int KC>() { st = hybrid_round<R, MULTI, KC>(s, r, r == 0); });
            ST_TRY(st);
            if (s->h_st->err) return error_from_word(s);
        }
        hipLaunchKernelGGL(k_resume, dim3(1), dim3(64), 0, s->stream, s->d_st);
        HIP_TRY(hipGetLastError());
    }
    return read_state(s);
}

spv_status run_steps(spv_sys* s, int64_t n)
{
    if (s->sticky != SPV_OK) return fail(s->sticky, s->sticky_msg);
    if (s->repair_mode == 1) return run_steps_hybrid(s, n);
    while (n > 0) {
        if (!(s->pos & 1) && !s->no_resort && !s->never_resort && s->pos > 0) {
            // re-sort at the period's end; once quiet, also as soon as the
            // drift bound (which widens the repair searches) passes the limit,
            // and when a period of the graph length is complete, so that the
            // graphs start from a fresh re-sort.  While hot, the repairs search
            // each step's own cell list and the drift does not matter.
            const int gq = s->hot ? 0 : graph_unit(s);
            if (s->pos >= s->unit || (!s->hot && s->h_st->drift > s->drift_limit) || (gq > 0 && s->pos >= gq))
                ST_TRY(do_resort_eager(s));
        }
        // (never re-sorting: periods of the re-sort period's length, from any
        // even position, without the re-sort)
        const int gu = s->hot ? 0 : s->never_resort ? s->unit : graph_unit(s);
        const bool at_start = s->never_resort ? !(s->pos & 1) : s->pos == 0;
        if (at_start && gu > 0 && n >= gu && s->use_graphs && !s->timing && !s->no_resort) {
            hipGraphExec_t ex = nullptr;
            ST_TRY(period_graph(s, s->cfg, gu, &ex));
            const uint64_t before = s->step, rep0 = s->h_st->repaired;
            const double drift0 = s->h_st->drift;
            const bool dense = dense_step(s, false);
            HIP_TRY(hipGraphLaunch(ex, s->stream));
            ST_TRY(read_state(s));
            s->graph_periods++;
            const uint64_t done = s->h_st->step - before;
            if (dense) s->dense_steps += (int64_t)done;
            note_repairs(s, s->h_st->repaired - rep0, done);
            if (s->h_st->halt) {
                // the period stopped after `done` steps (the last one unfinished);
                // later kernels, including its re-sort, did nothing
                s->step += done;
                n -= (int64_t)done;
                s->pos += (int)done;
                ST_TRY(recover(s, s->never_resort));
                continue;
            }
            s->step += done;
            n -= (int64_t)done;
            if (!s->never_resort) {
                s->cfg ^= 1;
                s->resorts++;
            }
            // the drift rate of the period sets the next period's length; too
            // fast for 8 steps: back to the fast-moving mode
            s->drift_rate = ((s->never_resort ? s->h_st->drift : s->h_st->last_drift) - drift0) / (double)done;
            if (graph_unit(s) == 0) {
                s->hot = true;
                s->quiet = 0;
            }
        } else {
            // eager: a batch of steps (up to kEagerBatch, not past the next
            // re-sort point), one read-back
            constexpr int64_t kEagerBatch = 8;
            int64_t b = std::min<int64_t>(n, kEagerBatch);
            if (!s->no_resort && !s->never_resort) b = std::min<int64_t>(b, std::max(1, s->unit - s->pos));
            // never re-sorting, graphs start at even positions: one step to get there
            if (s->never_resort && !s->hot && (s->pos & 1)) b = 1;
            const uint64_t before = s->step, rep0 = s->h_st->repaired;
            const double drift0 = s->h_st->drift;
            const bool hot = s->hot, dense = dense_step(s, hot);
            for (int64_t j = 0; j < b; j++) {
                const int cfg = s->cfg, par = (int)((s->pos + j) & 1);
                dispatch(s, [&]<typename R, bool MULTI, int KC>() {
                    enqueue_step<R, MULTI, KC>(s, s->stream, cfg, par, hot);
                });
            }
            HIP_TRY(hipGetLastError());
            ST_TRY(read_state(s));
            // steps after a halted one did nothing (as in a graph period)
            const uint64_t done = s->h_st->step - before;
            s->step += done;
            s->pos += (int)done;
            n -= (int64_t)done;
            if (dense) s->dense_steps += (int64_t)done;
            note_repairs(s, s->h_st->repaired - rep0, done);
            if (s->h_st->halt) ST_TRY(recover(s, hot || s->never_resort));
            if (hot) {
                // quiet once the measured drift rate has allowed graph periods
                // (at least 8 steps within the drift limit) for a whole period
                if (done > 0 && !s->h_st->halt) s->drift_rate = (s->h_st->drift - drift0) / (double)done;
                const int g = graph_unit(s);
                if (g == 0) {
                    s->quiet = 0;
                } else {
                    s->quiet += (int)done;
                    if (s->quiet >= g) s->hot = false;
                }
            }
        }
    }
    return SPV_OK;
}

spv_status copy_in(const double* src, std::vector<double>& dst, size_t n)
{
    dst.resize(n);
    HIP_TRY(hipMemcpy(dst.data(), src, n * sizeof(double), hipMemcpyDefault));
    return SPV_OK;
}

void destroy_all(spv_sys* s)
{
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (auto& kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto& kv : s->tgraphs) (void)hipGraphExecDestroy(kv.second);
    for (auto& e : s->pool) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    for (auto& t : s->pending) {
        (void)hipEventDestroy(t.second.a);
        (void)hipEventDestroy(t.second.b);
    }
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    for (void* p : s->allocs) (void)hipFree(p);
    if (s->h_st) (void)hipHostFree(s->h_st);
    for (void* p : {(void*)s->h_x, (void*)s->h_y, (void*)s->h_tag, (void*)s->h_sys, (void*)s->h_list,
                    (void*)s->h_touch, (void*)s->h_rows, (void*)s->h_new})
        if (p) (void)hipHostFree(p);
    delete s;
}

struct SysInput {
    int64_t n;
    double Lx, Ly;
    double v0;
    uint64_t seed;
};

spv_status seat_cells(spv_sys* s, const std::vector<double>& hx, const std::vector<double>& hy,
                      const std::vector<double>& hA0, const std::vector<double>& hP0, const std::vector<double>& hth,
                      const std::vector<int>& htag, const std::vector<int>& hsys, uint64_t step0);

// Shared creation: hx, hy, hA0, hP0 are host arrays concatenated by system;
// hth empty means default directors.
spv_status create_impl(spv_sys* s, const std::vector<SysInput>& in, std::vector<double>& hx,
                       std::vector<double>& hy, const std::vector<double>& hA0, const std::vector<double>& hP0,
                       const std::vector<double>& hth)
{
    ST_TRY(static_scratch(&s->scratch));
    const int S = (int)in.size();
    s->S = S;
    s->multi = S > 1;
    int64_t Ntot = 0;
    for (auto& v : in) Ntot += v.n;
    if (Ntot > (int64_t)1 << 30) return fail(SPV_EINVAL, "too many cells");
    s->N = (int)Ntot;
    const int N = s->N;
    std::vector<int> htag(N), hsys(N);
    std::vector<int> hbinkey;
    s->hsp.resize(S);
    s->cell_off.resize(S + 1);
    int off = 0, boff = 0;
    for (int k = 0; k < S; k++) {
        const SysInput& v = in[k];
        SysParam& P = s->hsp[k];
        std::memset(&P, 0, sizeof P);
        const int q = grid_exponent(std::max(v.Lx, v.Ly));
        P.scale = std::ldexp(1.0, q);
        P.inv_scale = 1.0 / P.scale;
        P.LXu = std::rint(v.Lx * P.scale);
        P.LYu = std::rint(v.Ly * P.scale);
        P.Lx = P.LXu / P.scale;
        P.Ly = P.LYu / P.scale;
        P.hLx = 0.5 * P.Lx;
        P.hLy = 0.5 * P.Ly;
        P.iLx = 1.0 / P.Lx;
        P.iLy = 1.0 / P.Ly;
        P.mu = s->prm.mu;
        P.v0 = v.v0;
        P.dt = s->prm.dt;
        P.amp = std::sqrt(2.0 * s->prm.Dr * s->prm.dt);
        P.KA = s->prm.KA;
        P.KP = s->prm.KP;
        P.seed = v.seed;
        P.cell_off = off;
        P.n = (int)v.n;
        const double spacing = std::sqrt(P.Lx * P.Ly / (double)v.n);
        P.R0 = 2.5 * spacing;
        P.nbx = std::max(1, (int)std::floor(P.Lx / (s->bin_factor * spacing)));
        P.nby = std::max(1, (int)std::floor(P.Ly / (s->bin_factor * spacing)));
        P.bsx = P.Lx / P.nbx;
        P.bsy = P.Ly / P.nby;
        P.bin_off = boff;
        // quantise, validate, reject duplicates
        std::vector<std::pair<double, double>> pts((size_t)v.n);
        for (int64_t t = 0; t < v.n; t++) {
            double& x = hx[off + t];
            double& y = hy[off + t];
            if (!std::isfinite(x) || !std::isfinite(y) || x < 0.0 || x >= v.Lx || y < 0.0 || y >= v.Ly)
                return fail(SPV_EINVAL, "positions must be finite and inside [0,Lx) x [0,Ly)");
            double X = std::rint(x * P.scale), Y = std::rint(y * P.scale);
            if (X >= P.LXu) X -= P.LXu;
            if (Y >= P.LYu) Y -= P.LYu;
            x = X / P.scale;
            y = Y / P.scale;
            pts[t] = {x, y};
            htag[off + t] = (int)t;
            hsys[off + t] = k;
        }
        std::sort(pts.begin(), pts.end());
        for (size_t t = 1; t < pts.size(); t++)
            if (pts[t] == pts[t - 1]) return fail(SPV_EINVAL, "two cells share a position on the grid");
        // bins of this system ranked along a Hilbert curve
        const int nb = P.nbx * P.nby;
        int64_t n2 = 1;
        while (n2 < std::max(P.nbx, P.nby)) n2 *= 2;
        std::vector<std::pair<int64_t, int>> key(nb);
        for (int by = 0; by < P.nby; by++)
            for (int bx = 0; bx < P.nbx; bx++)
                key[by * P.nbx + bx] = {s->prm.bin_order == 1 ? (int64_t)(by * P.nbx + bx) : hilbert_index(n2, bx, by),
                                        by * P.nbx + bx};
        std::sort(key.begin(), key.end());
        hbinkey.resize(boff + nb);
        for (int r = 0; r < nb; r++) hbinkey[boff + key[r].second] = boff + r;
        off += (int)v.n;
        boff += nb;
    }
    s->cell_off[S] = off;
    for (int k = 0; k < S; k++) s->cell_off[k] = s->hsp[k].cell_off;
    s->drift_limit = INFINITY;
    for (int k = 0; k < S; k++) s->drift_limit = std::min({s->drift_limit, s->hsp[k].bsx, s->hsp[k].bsy});
    s->total_bins = boff;

    // device state
    ST_TRY(alloc_set(s, s->set[0]));
    ST_TRY(alloc_set(s, s->set[1]));
    const size_t nwords = (N + 31) / 32;
    ST_TRY(dalloc(s, &s->work.flagbits, nwords));
    ST_TRY(dalloc(s, &s->work.touchbits, nwords));
    {
        // flag bytes padded to whole compaction blocks (the padding stays 0)
        const size_t nf = (size_t)grid_for(N, COMPACT_CELLS) * COMPACT_CELLS;
        ST_TRY(dalloc(s, &s->work.flag8, nf));
        HIP_TRY(hipMemsetAsync(s->work.flag8, 0, nf, s->stream));
    }
    ST_TRY(dalloc(s, &s->work.touch8, N));
    for (int k = 0; k < 2; k++) {
        ST_TRY(dalloc(s, &s->work.wl[k], N));
        ST_TRY(dalloc(s, &s->work.tl[k], N));
    }
    ST_TRY(dalloc(s, &s->d_bin_key, s->total_bins));
    ST_TRY(dalloc(s, &s->d_bin_start, s->total_bins + 1));
    ST_TRY(dalloc(s, &s->d_bin_range, s->total_bins));
    s->work.bin_key = s->d_bin_key;
    s->work.bin_start = s->d_bin_start;
    s->work.bin_range = s->d_bin_range;
    ST_TRY(dalloc(s, &s->d_key, N));
    ST_TRY(dalloc(s, &s->d_hist, s->total_bins));
    ST_TRY(dalloc(s, &s->d_fill, s->total_bins));
    ST_TRY(dalloc(s, &s->d_perm, N));
    ST_TRY(dalloc(s, &s->d_chunk, grid_for(s->total_bins, SCAN_CHUNK) + 1));
    ST_TRY(dalloc(s, &s->d_inv, N));
    ST_TRY(dalloc(s, &s->d_cbin, N));
    ST_TRY(dalloc(s, &s->d_cslot, N));
    ST_TRY(dalloc(s, &s->d_ccells, N));
    ST_TRY(dalloc(s, &s->d_ccount, s->total_bins));
    HIP_TRY(hipMemsetAsync(s->d_ccount, 0, (size_t)s->total_bins * sizeof(int), s->stream));
    ST_TRY(dalloc(s, &s->d_cstart, s->total_bins + 1));
    ST_TRY(dalloc(s, &s->d_cchunk, grid_for(s->total_bins, SCAN_CHUNK) + 1));
    ST_TRY(dalloc(s, &s->d_st, 1));
    ST_TRY(dalloc(s, &s->d_sp, S));
    ST_TRY(dalloc(s, &s->d_stage, N));
    ST_TRY(dalloc(s, &s->d_fx, N));
    ST_TRY(dalloc(s, &s->d_fy, N));
    ST_TRY(dalloc(s, &s->d_obs, 3 * S));
    int64_t nmax = 1;
    for (const auto& v : in) nmax = std::max<int64_t>(nmax, v.n);
    s->obs_chunks = (int)((nmax + OBS_CHUNK - 1) / OBS_CHUNK);
    ST_TRY(dalloc(s, &s->d_obs_part, (size_t)3 * S * s->obs_chunks));
    ST_TRY(dalloc(s, &s->d_blockmax, cell_grid(s)));
    HIP_TRY(hipHostMalloc((void**)&s->h_st, sizeof(DevState), hipHostMallocDefault));
    if (s->repair_mode == 1) {
        const size_t K = (size_t)s->KC;
        HIP_TRY(hipHostMalloc((void**)&s->h_x, N * sizeof(double), hipHostMallocDefault));
        HIP_TRY(hipHostMalloc((void**)&s->h_y, N * sizeof(double), hipHostMallocDefault));
        HIP_TRY(hipHostMalloc((void**)&s->h_tag, N * sizeof(int), hipHostMallocDefault));
        HIP_TRY(hipHostMalloc((void**)&s->h_sys, N * sizeof(int), hipHostMallocDefault));
        HIP_TRY(hipHostMalloc((void**)&s->h_list, N * sizeof(int), hipHostMallocDefault));
        HIP_TRY(hipHostMalloc((void**)&s->h_touch, N * sizeof(int), hipHostMallocDefault));
        HIP_TRY(hipHostMalloc((void**)&s->h_rows, N * (K + 1) * sizeof(int), hipHostMallocDefault));
        HIP_TRY(hipHostMalloc((void**)&s->h_new, N * (K + 2) * sizeof(int), hipHostMallocDefault));
        ST_TRY(dalloc(s, &s->d_rows, N * (K + 1)));
        ST_TRY(dalloc(s, &s->d_new, N * (K + 2)));
        s->h_mark.assign(N, 0);
    }
    HIP_TRY(hipMemcpyAsync(s->d_sp, s->hsp.data(), S * sizeof(SysParam), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(s->d_bin_key, hbinkey.data(), s->total_bins * sizeof(int), hipMemcpyHostToDevice,
                           s->stream));
    HIP_TRY(hipStreamCreate(&s->cap_stream));
    return seat_cells(s, hx, hy, hA0, hP0, hth, htag, hsys, 0);
}

// Put cells (tag order per system, grid-exact positions) into configuration
// 0 and build their triangulation from scratch: the state after creation or
// after loading a checkpoint.  Statistics restart; the step index is step0.
spv_status seat_cells(spv_sys* s, const std::vector<double>& hx, const std::vector<double>& hy,
                      const std::vector<double>& hA0, const std::vector<double>& hP0, const std::vector<double>& hth,
                      const std::vector<int>& htag, const std::vector<int>& hsys, uint64_t step0)
{
    const int N = s->N;
    const size_t nwords = (N + 31) / 32;
    HIP_TRY(hipStreamSynchronize(s->stream));
    for (int k = 0; k < 2; k++) HIP_TRY(hipMemsetAsync(s->set[k].deg, 0, N, s->stream));
    HIP_TRY(hipMemsetAsync(s->d_st, 0, sizeof(DevState), s->stream));
    HIP_TRY(hipMemcpyAsync(reinterpret_cast<char*>(s->d_st) + offsetof(DevState, step), &step0, sizeof step0,
                           hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemsetAsync(s->work.flagbits, 0, nwords * sizeof(unsigned), s->stream));
    HIP_TRY(hipMemsetAsync(s->work.touchbits, 0, nwords * sizeof(unsigned), s->stream));
    HIP_TRY(hipMemsetAsync(s->work.flag8, 0, N, s->stream));
    HIP_TRY(hipMemsetAsync(s->work.touch8, 0, N, s->stream));
    ArraySet& A = s->set[0];
    HIP_TRY(hipMemcpyAsync(A.x, hx.data(), N * sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(A.y, hy.data(), N * sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(A.A0, hA0.data(), N * sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(A.P0, hP0.data(), N * sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(A.tag, htag.data(), N * sizeof(int), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(A.sys, hsys.data(), N * sizeof(int), hipMemcpyHostToDevice, s->stream));
    if (!hth.empty())
        HIP_TRY(hipMemcpyAsync(A.th, hth.data(), N * sizeof(double), hipMemcpyHostToDevice, s->stream));
    else
        hipLaunchKernelGGL(k_theta0, dim3(grid_for(N, 256)), dim3(256), 0, s->stream, A.th, A.tag, A.sys, s->d_sp, N);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s->stream));  // the host vectors may die after return

    // spatial order, then the triangulation from scratch: every cell repaired
    s->cfg = 0;
    s->pos = 0;
    s->step = step0;
    s->hot = true;
    s->quiet = 0;
    s->drift_rate = INFINITY;
    s->dense_busy = false;
    ST_TRY(do_resort_eager(s));
    s->resorts = 0;
    s->graph_periods = s->dense_steps = s->host_rounds = s->recoveries = 0;
    s->hyb_repaired = s->hyb_rounds = 0;
    s->hr.candidates = 0;
    hipLaunchKernelGGL(k_all_to_worklist, dim3(grid_for(N, 256)), dim3(256), 0, s->stream, s->work, s->d_st, N);
    int r = 0;
    while (true) {
        if (r >= MAX_ROUNDS) return fail(SPV_EREPAIR, "initial triangulation did not converge");
        const unsigned rg = (r == 0) ? (unsigned)std::min(N, 65535) : 4096u;
        dispatch(s, [&]<typename R, bool MULTI, int KC>() { enqueue_round<R, MULTI, KC>(s, s->stream, r, rg, false); });
        HIP_TRY(hipGetLastError());
        ST_TRY(read_state(s));
        if (s->h_st->err) {
            spv_status st = error_from_word(s);
            return st;
        }
        if (s->h_st->wl_count[r + 1] == 0) break;
        r++;
    }
    hipLaunchKernelGGL(k_resume, dim3(1), dim3(64), 0, s->stream, s->d_st);
    HIP_TRY(hipGetLastError());
    ST_TRY(read_state(s));
    return SPV_OK;
}

spv_status setup_params(spv_sys* s, const spv_params* params, void* stream)
{
    const spv_params& p = *params;
    if (p.precision != SPV_FP64 && p.precision != SPV_MIXED) return fail(SPV_EINVAL, "precision must be FP64 or MIXED");
    if (!(p.dt > 0.0) || !(p.Dr >= 0.0) || !std::isfinite(p.dt) || !std::isfinite(p.Dr) || !std::isfinite(p.mu) ||
        !std::isfinite(p.v0) || !std::isfinite(p.KA) || !std::isfinite(p.KP))
        return fail(SPV_EINVAL, "invalid model parameters");
    s->prm = p;
    s->mixed = p.precision == SPV_MIXED;
    s->KC = p.kcap > 0 ? p.kcap : 16;
    if (s->KC != 16 && s->KC != 32) return fail(SPV_EINVAL, "kcap must be 16 or 32");
    s->max_rounds = p.repair_rounds > 0 ? std::min(p.repair_rounds, MAX_ROUNDS) : 16;
    s->dev_rounds = p.device_rounds > 0 ? std::min(p.device_rounds, s->max_rounds) : std::min(8, s->max_rounds);
    if (s->dev_rounds > s->max_rounds) return fail(SPV_EINVAL, "device_rounds exceeds repair_rounds");
    s->unit = p.resort_every > 0 ? p.resort_every : 32;
    s->never_resort = p.resort_every == -1;
    if (s->unit & 1) s->unit += 1;
    s->use_graphs = p.no_graphs == 0;
    if (p.repair_cells < 0 || p.resort_every < -1 || p.device_rounds < 0)
        return fail(SPV_EINVAL, "negative scheduling knob");
    s->repair_cells = p.repair_cells > 0 ? p.repair_cells : 64;
    if (p.tail_items < 0 || p.full_rounds < 0) return fail(SPV_EINVAL, "negative scheduling knob");
    s->tail_items = p.tail_items > 0 ? p.tail_items : 64;
    s->full_rounds = p.full_rounds > 0 ? p.full_rounds : 1;
    if (s->full_rounds > MAX_FULL_ROUNDS) return fail(SPV_EINVAL, "full_rounds must be at most 4");
    s->bin_factor = p.bin_factor != 0.0 ? p.bin_factor : 1.0;
    if (!(s->bin_factor >= 0.5 && s->bin_factor <= 8.0)) return fail(SPV_EINVAL, "bin_factor must be in [0.5, 8]");
    if (p.autotune < 0 || p.autotune > 2) return fail(SPV_EINVAL, "autotune must be 0, 1 or 2");
    if (p.bin_order < 0 || p.bin_order > 1) return fail(SPV_EINVAL, "bin_order must be 0 or 1");
    if (p.force_mode < 0 || p.force_mode > 2) return fail(SPV_EINVAL, "force_mode must be 0, 1 or 2");
    s->force_mode = p.force_mode;
    if (p.dense < 0 || p.dense > 2) return fail(SPV_EINVAL, "dense must be 0, 1 or 2");
    s->dense = p.dense;
    if (p.repair_mode < 0 || p.repair_mode > 1) return fail(SPV_EINVAL, "repair_mode must be 0 or 1");
    s->repair_mode = p.repair_mode;
    s->stream = (hipStream_t)stream;
    return SPV_OK;
}

// The kernels address ring and opposite-vertex rows (int32, N x kcap) with
// 32-bit byte offsets and form row indices i * kcap + m in int: both need
// N * kcap < 2^30 (N < 2^26 cells at kcap 16, 2^25 at kcap 32).  Checked on
// the host before any copy or allocation.
constexpr int64_t kMaxRingEntries = (int64_t)1 << 30;
spv_status check_ring_extent(int64_t N, int kcap)
{
    if (N * (int64_t)kcap >= kMaxRingEntries)
        return fail(SPV_EINVAL, "N * kcap must be below 2^30 (ring rows are addressed with 32-bit offsets)");
    return SPV_OK;
}

spv_status finish_create(spv_sys* s, spv_status st, spv_sys** out)
{
    if (st != SPV_OK) {
        std::string keep = g_err;
        destroy_all(s);
        g_err = keep;
        return st;
    }
    *out = s;
    return SPV_OK;
}

template <typename F>
spv_status with_tag_order(spv_sys* s, F&& launch_into_stage, double* dst)
{
    launch_into_stage(s->d_stage);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(dst, s->d_stage, (size_t)s->N * sizeof(double), hipMemcpyDefault, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return SPV_OK;
}

template <typename T>
spv_status out_tag_order(spv_sys* s, const T* src, double* dst)
{
    const ArraySet& P = s->set[s->cfg];
    return with_tag_order(
        s,
        [&](double* stage) {
            hipLaunchKernelGGL(k_to_tag_order<T>, dim3(grid_for(s->N, 256)), dim3(256), 0, s->stream, src, P.tag,
                               P.sys, s->d_sp, stage, s->N);
        },
        dst);
}

// ---------------------------------------------------------------- checkpoints
// Layout (little-endian, 8-byte fields): header, one record per system, then
// x, y, theta, A0, P0 as double[N] each, tag order.
struct StateHeader {
    char magic[8];  // "SPVSTAT" + version byte 1
    int32_t S, precision;
    int64_t N;
    uint64_t step;
};
struct StateSystem {
    int64_t n;
    double Lx, Ly, v0;
    uint64_t seed;
};
constexpr char kStateMagic[8] = {'S', 'P', 'V', 'S', 'T', 'A', 'T', 1};

int64_t state_bytes(const spv_sys* s)
{
    return (int64_t)sizeof(StateHeader) + (int64_t)s->S * (int64_t)sizeof(StateSystem) + 5 * (int64_t)s->N * 8;
}

spv_status save_state(spv_sys* s, void* buf, int64_t cap, int64_t* needed)
{
    const int64_t bytes = state_bytes(s);
    if (needed) *needed = bytes;
    if (!buf || cap < bytes) return fail(SPV_ECAPACITY, "state buffer too small (see *needed)");
    if (s->sticky != SPV_OK) return fail(s->sticky, s->sticky_msg);
    const size_t N = s->N;
    std::vector<char> out((size_t)bytes);
    StateHeader h{};
    std::memcpy(h.magic, kStateMagic, 8);
    h.S = s->S;
    h.precision = s->mixed ? SPV_MIXED : SPV_FP64;
    h.N = s->N;
    h.step = s->step;
    std::memcpy(out.data(), &h, sizeof h);
    char* p = out.data() + sizeof h;
    for (int k = 0; k < s->S; k++) {
        const SysParam& P = s->hsp[k];
        StateSystem r{P.n, P.Lx, P.Ly, P.v0, P.seed};
        std::memcpy(p, &r, sizeof r);
        p += sizeof r;
    }
    double* arr = reinterpret_cast<double*>(p);
    const int par = s->pos & 1;
    const ArraySet& live = s->set[par ? s->cfg ^ 1 : s->cfg];
    const ArraySet& fixed = s->set[s->cfg];
    ST_TRY(out_tag_order(s, live.x, arr));
    ST_TRY(out_tag_order(s, live.y, arr + N));
    ST_TRY(out_tag_order(s, live.th, arr + 2 * N));
    ST_TRY(out_tag_order(s, fixed.A0, arr + 3 * N));
    ST_TRY(out_tag_order(s, fixed.P0, arr + 4 * N));
    HIP_TRY(hipMemcpy(buf, out.data(), (size_t)bytes, hipMemcpyDefault));
    return SPV_OK;
}

spv_status load_state(spv_sys* s, const void* buf, int64_t len)
{
    const int64_t bytes = state_bytes(s);
    if (!buf || len != bytes) return fail(SPV_EINVAL, "state size does not match this handle's layout");
    std::vector<char> in((size_t)bytes);
    HIP_TRY(hipMemcpy(in.data(), buf, (size_t)bytes, hipMemcpyDefault));
    StateHeader h;
    std::memcpy(&h, in.data(), sizeof h);
    if (std::memcmp(h.magic, kStateMagic, 8) != 0) return fail(SPV_EINVAL, "not an SPV state (bad magic/version)");
    if (h.S != s->S || h.N != s->N || h.precision != (s->mixed ? SPV_MIXED : SPV_FP64))
        return fail(SPV_EINVAL, "state has another number of systems, cells or precision");
    const char* p = in.data() + sizeof h;
    for (int k = 0; k < s->S; k++) {
        StateSystem r;
        std::memcpy(&r, p, sizeof r);
        p += sizeof r;
        const SysParam& P = s->hsp[k];
        if (r.n != P.n || r.Lx != P.Lx || r.Ly != P.Ly)
            return fail(SPV_EINVAL, "state system " + std::to_string(k) + " has another size or box");
    }
    const size_t N = s->N;
    const double* arr = reinterpret_cast<const double*>(p);
    std::vector<double> hx(arr, arr + N), hy(arr + N, arr + 2 * N), hth(arr + 2 * N, arr + 3 * N),
        hA0(arr + 3 * N, arr + 4 * N), hP0(arr + 4 * N, arr + 5 * N);
    std::vector<int> htag(N), hsys(N);
    for (int k = 0; k < s->S; k++) {
        const SysParam& P = s->hsp[k];
        for (int t = 0; t < P.n; t++) {
            const size_t i = (size_t)P.cell_off + t;
            htag[i] = t;
            hsys[i] = k;
            const double X = hx[i] * P.scale, Y = hy[i] * P.scale;
            if (!(X >= 0.0 && X < P.LXu && Y >= 0.0 && Y < P.LYu) || X != std::rint(X) || Y != std::rint(Y))
                return fail(SPV_EINVAL, "state positions are not on this handle's grid");
            if (!std::isfinite(hth[i]) || !(hA0[i] > 0.0) || !std::isfinite(hA0[i]) || !std::isfinite(hP0[i]))
                return fail(SPV_EINVAL, "state holds non-finite directors or targets");
        }
    }
    // every check passed: replace the state (a failure from here on leaves
    // the handle unusable until the next successful load)
    s->traj_valid = false;
    s->sticky = SPV_OK;
    spv_status st = seat_cells(s, hx, hy, hA0, hP0, hth, htag, hsys, h.step);
    if (st != SPV_OK && s->sticky == SPV_OK) {
        s->sticky = st;
        s->sticky_msg = "loading the state failed: " + g_err;
    }
    return st;
}

// ---------------------------------------------------------------- autotuner
// Everything creation needs, kept so the tuner can build clones.
struct CreateArgs {
    std::vector<SysInput> in;
    std::vector<double> x, y, A0, P0, th;
    spv_params prm{};
    void* stream = nullptr;
};

spv_status build_handle(const CreateArgs& a, const spv_params& p, spv_sys** out)
{
    *out = nullptr;
    spv_sys* s = new spv_sys();
    spv_status st = setup_params(s, &p, a.stream);
    if (st != SPV_OK) return finish_create(s, st, out);
    std::vector<double> hx = a.x, hy = a.y;  // quantised in place
    return finish_create(s, create_impl(s, a.in, hx, hy, a.A0, a.P0, a.th), out);
}

Knobs knobs_of(const spv_sys* s)
{
    return {s->unit, s->dev_rounds, s->repair_cells, s->tail_items, s->full_rounds, s->force_mode, s->bin_factor};
}

spv_params with_knobs(spv_params p, const Knobs& k)
{
    p.resort_every = k.resort_every;
    p.device_rounds = k.device_rounds;
    p.repair_cells = k.repair_cells;
    p.tail_items = k.tail_items;
    p.full_rounds = k.full_rounds;
    p.force_mode = k.force_mode;
    p.bin_factor = k.bin_factor;
    p.autotune = 0;
    return p;
}

// Start a period, run one (captures and replays its graph), then time
// `steps` steps; steps is a multiple of every candidate period.
spv_status trial_ms(spv_sys* s, int steps, double* ms)
{
    if (s->pos & 1) ST_TRY(run_steps(s, 1));
    if (s->pos != 0) ST_TRY(do_resort_eager(s));
    ST_TRY(run_steps(s, s->unit));
    HIP_TRY(hipStreamSynchronize(s->stream));
    const auto t0 = std::chrono::steady_clock::now();
    ST_TRY(run_steps(s, steps));
    HIP_TRY(hipStreamSynchronize(s->stream));
    const auto t1 = std::chrono::steady_clock::now();
    *ms = std::chrono::duration<double, std::milli>(t1 - t0).count() / steps;
    return SPV_OK;
}

std::mutex g_tune_mu;
std::map<std::string, TuneEntry> g_tune_mem;  // this process's cache (file entries merged in)

spv_status tune_key_for(const CreateArgs& a, std::string& key)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    std::string arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    int64_t N = 0;
    for (const auto& v : a.in) N += v.n;
    key = tune_key(arch, prop.multiProcessorCount, a.prm.precision == SPV_MIXED, a.prm.kcap > 0 ? a.prm.kcap : 16, N,
                   (int)a.in.size());
    return SPV_OK;
}

// The search: warm a clone for 256 steps from the input; from that state,
// time the bin side, then the repair grid, the tail's largest round, the
// full-grid rounds, the device repair budget and the re-sort period, one
// knob at a time, each candidate on a fresh clone of the warmed state; a
// candidate replaces the current choice only when 3% faster.
spv_status run_trials(const CreateArgs& a, Knobs& best, double& best_ms)
{
    constexpr int kWarm = 256, kTrial = 128;  // kTrial: a multiple of every candidate period
    const double kMargin = 0.97;
    spv_sys* w = nullptr;
    ST_TRY(build_handle(a, with_knobs(a.prm, best), &w));
    CreateArgs b = a;
    b.prm = with_knobs(a.prm, best);
    spv_status st = run_steps(w, kWarm);
    const ArraySet& live = w->set[(w->pos & 1) ? w->cfg ^ 1 : w->cfg];
    b.th.resize(b.x.size());
    if (st == SPV_OK) st = out_tag_order(w, live.x, b.x.data());
    if (st == SPV_OK) st = out_tag_order(w, live.y, b.y.data());
    if (st == SPV_OK) st = out_tag_order(w, live.th, b.th.data());
    destroy_all(w);
    ST_TRY(st);

    // every candidate is timed on a fresh clone of the same warmed state (the
    // same dynamics, the same repairs): only the knobs differ between trials
    const int maxr = a.prm.repair_rounds > 0 ? std::min(a.prm.repair_rounds, MAX_ROUNDS) : 16;
    auto time_knobs = [&](const Knobs& k, double* ms) {
        *ms = INFINITY;
        spv_sys* c = nullptr;
        if (build_handle(b, with_knobs(b.prm, k), &c) != SPV_OK) return false;
        const bool ok = trial_ms(c, kTrial, ms) == SPV_OK;
        destroy_all(c);
        return ok;
    };
    bool any = false;
    best_ms = INFINITY;
    for (double f : {1.0, 1.5, 2.0}) {
        Knobs k = best;
        k.bin_factor = f;
        double ms;
        if (time_knobs(k, &ms) && (!any || ms < kMargin * best_ms)) {
            best = k;
            best_ms = ms;
            any = true;
        }
    }
    if (!any) return fail(SPV_EHIP, "autotune: no trial ran");

    struct Axis {
        int Knobs::*field;
        int cand[3];
    };
    const Axis axes[] = {{&Knobs::repair_cells, {16, 64, 256}},
                         {&Knobs::tail_items, {16, 64, 256}},
                         {&Knobs::full_rounds, {1, 2, 1}},
                         {&Knobs::force_mode, {1, 2, 1}},
                         {&Knobs::device_rounds, {2, 4, 8}},
                         {&Knobs::resort_every, {16, 32, 64}}};
    for (const Axis& ax : axes) {
        Knobs choice = best;
        double choice_ms = best_ms;
        for (int v : ax.cand) {
            if (v == best.*ax.field) continue;
            Knobs k = best;
            k.*ax.field = v;
            if (k.device_rounds > maxr || k.full_rounds > k.device_rounds) continue;
            double ms;
            if (time_knobs(k, &ms) && ms < kMargin * best_ms && ms < choice_ms) {
                choice = k;
                choice_ms = ms;
            }
        }
        best = choice;
        best_ms = choice_ms;
    }
    return SPV_OK;
}

// Creation with the knobs of a.prm, or tuned ones when a.prm.autotune is set.
spv_status create_tuned(const CreateArgs& a, spv_sys** out)
{
    *out = nullptr;
    spv_params p = a.prm;
    // the hybrid mode's cost is the host round trip, and the re-sort period is
    // a knob of the trials: no trials for either
    if (p.autotune == 0 || p.repair_mode == 1 || p.resort_every == -1) {
        p.autotune = 0;
        return build_handle(a, p, out);
    }
    // validate the parameters (and fill in the defaults) before any trial
    spv_sys* probe = new spv_sys();
    spv_status st = setup_params(probe, &p, a.stream);
    Knobs k = knobs_of(probe);
    delete probe;
    ST_TRY(st);
    std::string key;
    ST_TRY(tune_key_for(a, key));
    const char* path = std::getenv("SPV_TUNE_CACHE");
    int source = 0;
    double ms = 0.0;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        if (path && *path) {
            std::map<std::string, TuneEntry> file;
            if (cache_load(path, file) == 0)
                for (auto& kv : file) g_tune_mem[kv.first] = kv.second;
        }
        auto it = g_tune_mem.find(key);
        if (p.autotune == 1 && it != g_tune_mem.end()) {
            k = it->second.k;
            ms = it->second.ms_per_step;
            source = 1;
        }
    }
    if (source == 0) {
        Knobs t = k;
        double tms = 0.0;
        const std::string keep = g_err;
        if (run_trials(a, t, tms) == SPV_OK) {
            k = t;
            ms = tms;
            source = 2;
            std::lock_guard<std::mutex> lock(g_tune_mu);
            g_tune_mem[key] = {k, ms};
            if (path && *path) {
                std::map<std::string, TuneEntry> file;
                if (cache_load(path, file) == 0) {  // never replace a file we cannot read
                    file[key] = {k, ms};
                    (void)cache_store(path, file);
                }
            }
        }
        g_err = keep;
    }
    ST_TRY(build_handle(a, with_knobs(p, k), out));
    (*out)->tune_source = source;
    (*out)->tune_ms = ms;
    return SPV_OK;
}

// ---------------------------------------------------------------- trajectory adjoint
spv_status snap_alloc(spv_sys* s, Snapshot& z)
{
    if (z.x) return SPV_OK;
    const size_t N = s->N, K = s->KC;
    ST_TRY(dalloc(s, &z.x, N));
    ST_TRY(dalloc(s, &z.y, N));
    ST_TRY(dalloc(s, &z.th, N));
    ST_TRY(dalloc(s, &z.deg, N));
    ST_TRY(dalloc(s, &z.ring, N * K));
    ST_TRY(dalloc(s, &z.opp, N * K));
    ST_TRY(dalloc(s, &z.A, N));
    ST_TRY(dalloc(s, &z.P, N));
    ST_TRY(dalloc(s, &z.ca, N));
    ST_TRY(dalloc(s, &z.cb, N));
    return SPV_OK;
}

// copy between the live state (current configuration and parity) and z
spv_status snap_copy(spv_sys* s, Snapshot& z, bool take, hipStream_t stream = nullptr)
{
    const int N = s->N, K = s->KC;
    const ArraySet& cur = s->set[s->cfg];
    const ArraySet& par = s->set[(s->pos & 1) ? s->cfg ^ 1 : s->cfg];
    const StatePtrs live{par.x,  par.y,  par.th, cur.deg, cur.ring, cur.opp, static_cast<double*>(cur.A),
                         static_cast<double*>(cur.P), static_cast<double*>(cur.ca), static_cast<double*>(cur.cb)};
    const StatePtrs snap{z.x, z.y, z.th, z.deg, z.ring, z.opp, z.A, z.P, z.ca, z.cb};
    const unsigned grid = std::min(grid_for(N * K, 256), 2048u);
    hipLaunchKernelGGL(k_state_copy, dim3(grid), dim3(256), 0, stream ? stream : s->stream, take ? snap : live,
                       take ? live : snap, N, K);
    HIP_TRY(hipGetLastError());
    return SPV_OK;
}

Cells<double> snap_cells(const spv_sys* s, const Snapshot& z)
{
    Cells<double> c = cells<double>(s, s->cfg, 0);
    c.x = z.x;
    c.y = z.y;
    c.th = z.th;
    c.deg = z.deg;
    c.ring = z.ring;
    c.opp = z.opp;
    c.A = z.A;
    c.P = z.P;
    c.ca = z.ca;
    c.cb = z.cb;
    return c;
}

spv_status traj_buffers(spv_sys* s)
{
    if (s->d_lx) return SPV_OK;
    const size_t N = s->N;
    for (double** p : {&s->d_lx, &s->d_ly, &s->d_lx2, &s->d_ly2, &s->d_g, &s->d_dA, &s->d_dP, &s->d_fdx, &s->d_fdy,
                       &s->d_aq, &s->d_bq})
        ST_TRY(dalloc(s, p, N));
    ST_TRY(dalloc(s, &s->d_acc, 1));
    return SPV_OK;
}

// the state (and the observable accumulated so far) at a segment start
spv_status take_checkpoint(spv_sys* s, TrajCheckpoint& c)
{
    ST_TRY(snap_alloc(s, c.snap));
    if (!c.acc) ST_TRY(dalloc(s, &c.acc, 1));
    ST_TRY(snap_copy(s, c.snap, true));
    HIP_TRY(hipMemcpyAsync(c.acc, s->d_acc, sizeof(double), hipMemcpyDeviceToDevice, s->stream));
    c.pos = s->pos;
    c.step = s->step;
    return SPV_OK;
}

// restore a checkpoint, including the device noise counter; clears a
// halted step's device state (the segment is then redone)
spv_status restore_checkpoint(spv_sys* s, const TrajCheckpoint& c, bool with_acc)
{
    s->pos = c.pos;
    s->step = c.step;
    ST_TRY(snap_copy(s, const_cast<Snapshot&>(c.snap), false));
    if (with_acc) HIP_TRY(hipMemcpyAsync(s->d_acc, c.acc, sizeof(double), hipMemcpyDeviceToDevice, s->stream));
    // a halted step leaves flagged / touched cells behind: forget them with
    // their counters (the restored state is a completed step's)
    const size_t nwords = ((size_t)s->N + 31) / 32;
    HIP_TRY(hipMemsetAsync(s->work.flagbits, 0, nwords * sizeof(unsigned), s->stream));
    HIP_TRY(hipMemsetAsync(s->work.touchbits, 0, nwords * sizeof(unsigned), s->stream));
    HIP_TRY(hipMemsetAsync(s->work.flag8, 0, (size_t)s->N, s->stream));
    HIP_TRY(hipMemsetAsync(s->work.touch8, 0, (size_t)s->N, s->stream));
    hipLaunchKernelGGL(k_resume, dim3(1), dim3(64), 0, s->stream, s->d_st);
    HIP_TRY(hipGetLastError());
    ST_TRY(read_state(s));
    s->h_st->step = c.step;
    HIP_TRY(hipMemcpyAsync(reinterpret_cast<char*>(s->d_st) + offsetof(DevState, step), &s->h_st->step,
                           sizeof(unsigned long long), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return SPV_OK;
}

// m steps of a recorded segment, enqueued back to back (no re-sort), each
// followed by after(j); one read-back.  *ok = false when a step needed host
// repair rounds (the later kernels did nothing; the caller redoes the
// segment one step at a time from its checkpoint).
// The launches enq(stream) makes, captured on first use as a graph under key
// (a trajectory segment of a given shape: the same buffers every time) and
// replayed on the handle's stream.
template <typename F>
spv_status traj_graph(spv_sys* s, const std::vector<int64_t>& key, F&& enq)
{
    auto it = s->tgraphs.find(key);
    if (it == s->tgraphs.end()) {
        hipGraph_t graph = nullptr;
        HIP_TRY(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeRelaxed));
        enq(s->cap_stream);
        hipError_t e0 = hipGetLastError();
        hipError_t e1 = hipStreamEndCapture(s->cap_stream, &graph);
        if (e1 == hipSuccess && e0 != hipSuccess) e1 = e0;
        if (e1 != hipSuccess) return fail(SPV_EHIP, std::string("graph capture: ") + hipGetErrorString(e1));
        hipGraphExec_t ex = nullptr;
        hipError_t e2 = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e2 != hipSuccess) return fail(SPV_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e2));
        it = s->tgraphs.emplace(key, ex).first;
    }
    HIP_TRY(hipGraphLaunch(it->second, s->stream));
    return SPV_OK;
}

// m steps of a trajectory segment with after(j, stream) after step j, then
// one read-back; *ok when every step finished on the device.  kind >= 0:
// the segment's launches replay a graph captured for its shape (kind, m,
// parity, configuration, step flavour, extra) -- what the events of the
// timing mode cannot be part of.
template <typename After>
spv_status segment_fast(spv_sys* s, int64_t m, After&& after, bool* ok, int64_t kind = -1, int64_t extra = 0)
{
    const uint64_t before = s->step;
    const int pos0 = s->pos, cfg = s->cfg;
    const bool hot = s->hot;
    auto enq = [&](hipStream_t stream) {
        for (int64_t j = 0; j < m; j++) {
            const int par = (int)((pos0 + j) & 1);
            dispatch(s, [&]<typename R, bool MULTI, int KC>() {
                enqueue_step<R, MULTI, KC>(s, stream, cfg, par, hot);
            });
            s->pos = pos0 + (int)j + 1;  // after() sees the state after step j + 1
            after(j + 1, stream);
        }
    };
    if (kind >= 0 && s->use_graphs && !s->timing)
        ST_TRY(traj_graph(s, {kind, m, pos0 & 1, cfg, hot ? 1 : 0, dense_step(s, hot) ? 1 : 0, extra}, enq));
    else
        enq(s->stream);
    s->pos = pos0 + (int)m;  // a replayed graph did not run enq's bookkeeping
    HIP_TRY(hipGetLastError());
    ST_TRY(read_state(s));
    if (s->h_st->err) return error_from_word(s);
    *ok = !s->h_st->halt && s->h_st->step - before == (uint64_t)m;
    if (*ok) s->step += m;
    else s->pos = pos0;  // the caller restores the segment's checkpoint
    return SPV_OK;
}

spv_status traj_forward(spv_sys* s, int64_t T, int64_t k, double* Q)
{
    if (s->S != 1 || s->mixed) return fail(SPV_EINVAL, "the trajectory adjoint needs a single FP64 system");
    if (T < 1 || k < 1) return fail(SPV_EINVAL, "T and ckpt_every must be positive");
    if (s->sticky != SPV_OK) return fail(s->sticky, s->sticky_msg);
    ST_TRY(traj_buffers(s));
    const int64_t nck = (T + k - 1) / k;
    s->ckpt.resize(nck + 1);
    s->traj_valid = false;
    s->no_resort = true;
    HIP_TRY(hipMemsetAsync(s->d_acc, 0, sizeof(double), s->stream));
    const double w = 1.0 / (double)T;
    auto accum = [&](int64_t, hipStream_t stream) {
        const ArraySet& cur = s->set[s->cfg];
        hipLaunchKernelGGL(k_qbar_accum, dim3(1), dim3(256), 0, stream, (const double*)cur.A, (const double*)cur.P,
                           s->N, w, s->d_acc, (const DevState*)s->d_st);
    };
    spv_status st = SPV_OK;
    for (int64_t c = 0; c < nck && st == SPV_OK; c++) {
        const int64_t m = std::min<int64_t>(k, T - c * k);
        st = take_checkpoint(s, s->ckpt[c]);
        bool ok = false;
        if (st == SPV_OK) st = segment_fast(s, m, accum, &ok, 1, T);
        if (st == SPV_OK && !ok) {
            st = restore_checkpoint(s, s->ckpt[c], true);
            for (int64_t j = 0; j < m && st == SPV_OK; j++) {
                st = run_steps(s, 1);
                if (st == SPV_OK) accum(j + 1, s->stream);
            }
        }
    }
    if (st == SPV_OK) st = take_checkpoint(s, s->ckpt[nck]);
    s->no_resort = false;
    if (st != SPV_OK) return st;
    double q = 0.0;
    HIP_TRY(hipMemcpyAsync(&q, s->d_acc, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (Q) *Q = q;
    s->traj_T = T;
    s->traj_k = k;
    s->traj_valid = true;
    return SPV_OK;
}

// One backward step over r_{t-1} -> r_t with the adjoint lambda in buffer
// li:  lambda += d(w qbar)/dr at r_t (the force kernel with the qbar
// coefficients aq, bq of r_t, which the previous backward step computed),
// then  lambda' = lambda + dt mu dF(r_{t-1})[lambda]  into buffer li ^ 1 and
// g += dt mu 2 K_P dP(r_{t-1})[lambda];  the tangent-geometry pass at r_{t-1}
// also leaves the qbar coefficients of r_{t-1} for the next backward step.
template <int KC>
void enqueue_adjoint_step(spv_sys* s, const Snapshot& at_t, const Snapshot& at_prev, int li, hipStream_t stream)
{
    const int N = s->N;
    const double w = 1.0 / (double)s->traj_T;
    double* lx = li ? s->d_lx2 : s->d_lx;
    double* ly = li ? s->d_ly2 : s->d_ly;
    double* lxo = li ? s->d_lx : s->d_lx2;
    double* lyo = li ? s->d_ly : s->d_ly2;
    Cells<double> ct = snap_cells(s, at_t);
    ct.ca = s->d_aq;
    ct.cb = s->d_bq;
    hipLaunchKernelGGL((force_kernel<double, false, KC, false, true>(s)), dim3(force_grid(s)), dim3(256), 0, stream, ct,
                       (double*)nullptr, (double*)nullptr, (double*)nullptr, lx, ly, (const SysParam*)s->d_sp,
                       s->d_st, N, s->d_blockmax, CellCount{});
    Cells<double> cp = snap_cells(s, at_prev);
    hipLaunchKernelGGL((k_tangent_geom<KC>), dim3(grid_for(N * GL, 256)), dim3(256), 0, stream, cp, (const double*)lx,
                       (const double*)ly, (const SysParam*)s->d_sp, N, s->d_dA, s->d_dP, w, s->d_aq, s->d_bq);
    hipLaunchKernelGGL((k_tangent_force<KC, true>), dim3(grid_for(N * GL, 256)), dim3(256), 0, stream, cp, (const double*)lx,
                       (const double*)ly, (const double*)s->d_dA, (const double*)s->d_dP, (const SysParam*)s->d_sp, N,
                       lxo, lyo, s->d_g);
}

__global__ void k_adj_out(const double* g, const double* A0, const int* tag, double scale, double* out, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[tag[i]] = scale * g[i] * sqrt(A0[i]);
}

spv_status traj_backward(spv_sys* s, double dQ, double* dQ_dp0)
{
    if (!s->traj_valid) return fail(SPV_EINVAL, "spv_traj_forward must precede spv_traj_backward");
    const int64_t T = s->traj_T, k = s->traj_k, nck = (T + k - 1) / k;
    const size_t N = s->N;
    s->seg.resize(k + 1);
    for (auto& z : s->seg) ST_TRY(snap_alloc(s, z));
    HIP_TRY(hipMemsetAsync(s->d_lx, 0, N * 8, s->stream));
    HIP_TRY(hipMemsetAsync(s->d_ly, 0, N * 8, s->stream));
    HIP_TRY(hipMemsetAsync(s->d_g, 0, N * 8, s->stream));
    s->no_resort = true;
    int li = 0;
    const double w = 1.0 / (double)T;
    spv_status st = SPV_OK;
    for (int64_t c = nck - 1; c >= 0 && st == SPV_OK; c--) {
        // recompute the segment from its checkpoint, recording every state
        const int64_t m = std::min<int64_t>(k, T - c * k);
        st = restore_checkpoint(s, s->ckpt[c], false);
        if (st == SPV_OK) st = snap_copy(s, s->seg[0], true);
        bool ok = false;
        if (st == SPV_OK)
            st = segment_fast(
                s, m, [&](int64_t j, hipStream_t stream) { (void)snap_copy(s, s->seg[j], true, stream); }, &ok, 2);
        if (st == SPV_OK && !ok) {
            st = restore_checkpoint(s, s->ckpt[c], false);
            for (int64_t j = 1; j <= m && st == SPV_OK; j++) {
                st = run_steps(s, 1);
                if (st == SPV_OK) st = snap_copy(s, s->seg[j], true);
            }
        }
        if (st != SPV_OK) break;
        // qbar coefficients of the segment's last state, then the steps
        // backwards (a graph per segment shape)
        auto adj = [&](hipStream_t stream) {
            hipLaunchKernelGGL(k_qbar_coef, dim3(grid_for(N, 256)), dim3(256), 0, stream, (const double*)s->seg[m].A,
                               (const double*)s->seg[m].P, (int)N, w, s->d_aq, s->d_bq);
            int l = li;
            for (int64_t j = m; j >= 1; j--) {
                if (s->KC == 16) enqueue_adjoint_step<16>(s, s->seg[j], s->seg[j - 1], l, stream);
                else enqueue_adjoint_step<32>(s, s->seg[j], s->seg[j - 1], l, stream);
                l ^= 1;
            }
        };
        if (s->use_graphs && !s->timing) st = traj_graph(s, {3, m, li, s->cfg, T}, adj);
        else adj(s->stream);
        li ^= (int)(m & 1);
        if (st == SPV_OK && hipGetLastError() != hipSuccess) st = fail(SPV_EHIP, "adjoint kernel launch failed");
    }
    // back to the state reached by the forward pass
    if (st == SPV_OK) st = restore_checkpoint(s, s->ckpt[nck], false);
    s->no_resort = false;
    if (st != SPV_OK) return st;
    const ArraySet& cur = s->set[s->cfg];
    return with_tag_order(
        s,
        [&](double* stage) {
            hipLaunchKernelGGL(k_adj_out, dim3(grid_for(s->N, 256)), dim3(256), 0, s->stream, (const double*)s->d_g,
                               (const double*)cur.A0, (const int*)cur.tag, dQ, stage, s->N);
        },
        dQ_dp0);
}

// H v for tests: dF[v] at the current state (v and the result in tag order)
template <int KC>
spv_status hvp_impl(spv_sys* s, const double* vx, const double* vy, double* hx, double* hy)
{
    const int N = s->N;
    ST_TRY(traj_buffers(s));
    const ArraySet& cur = s->set[s->cfg];
    std::vector<double> hvx, hvy;
    ST_TRY(copy_in(vx, hvx, N));
    ST_TRY(copy_in(vy, hvy, N));
    std::vector<int> tag(N);
    HIP_TRY(hipMemcpy(tag.data(), cur.tag, N * sizeof(int), hipMemcpyDeviceToHost));
    std::vector<double> mx(N), my(N);
    for (int i = 0; i < N; i++) {
        mx[i] = hvx[tag[i]];
        my[i] = hvy[tag[i]];
    }
    HIP_TRY(hipMemcpyAsync(s->d_lx, mx.data(), N * 8, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(s->d_ly, my.data(), N * 8, hipMemcpyHostToDevice, s->stream));
    Cells<double> c = cells<double>(s, s->cfg, s->pos & 1);
    hipLaunchKernelGGL((k_tangent_geom<KC>), dim3(grid_for(N * GL, 256)), dim3(256), 0, s->stream, c, (const double*)s->d_lx,
                       (const double*)s->d_ly, (const SysParam*)s->d_sp, N, s->d_dA, s->d_dP, 0.0, (double*)nullptr,
                       (double*)nullptr);
    hipLaunchKernelGGL((k_tangent_force<KC, false>), dim3(grid_for(N * GL, 256)), dim3(256), 0, s->stream, c, (const double*)s->d_lx,
                       (const double*)s->d_ly, (const double*)s->d_dA, (const double*)s->d_dP,
                       (const SysParam*)s->d_sp, N, s->d_fdx, s->d_fdy, (double*)nullptr);
    HIP_TRY(hipGetLastError());
    ST_TRY(out_tag_order(s, s->d_fdx, hx));
    return out_tag_order(s, s->d_fdy, hy);
}

}  // namespace

namespace {
bool device_pointer(const void* p)
{
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();  // clear the error of an unregistered host pointer
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

template <int KC>
spv_status hvp_static(spv_sys* s, const double* vx, const double* vy, double* fx, double* fy)
{
    const int N = s->N;
    const ArraySet& cur = s->set[s->cfg];
    double* lx = s->scratch;
    double *ly = lx + N, *dA = ly + N, *dP = dA + N, *ox = dP + N, *oy = ox + N;
    const unsigned g = grid_for(N, 256);
    hipLaunchKernelGGL(k_from_tag_order, dim3(g), dim3(256), 0, s->stream, vx, (const int*)cur.tag, lx, N);
    hipLaunchKernelGGL(k_from_tag_order, dim3(g), dim3(256), 0, s->stream, vy, (const int*)cur.tag, ly, N);
    Cells<double> c = cells<double>(s, s->cfg, s->pos & 1);
    hipLaunchKernelGGL((k_tangent_geom<KC>), dim3(grid_for(N * GL, 256)), dim3(256), 0, s->stream, c,
                       (const double*)lx, (const double*)ly, (const SysParam*)s->d_sp, N, dA, dP, 0.0,
                       (double*)nullptr, (double*)nullptr);
    hipLaunchKernelGGL((k_tangent_force<KC, false>), dim3(grid_for(N * GL, 256)), dim3(256), 0, s->stream, c,
                       (const double*)lx, (const double*)ly, (const double*)dA, (const double*)dP,
                       (const SysParam*)s->d_sp, N, ox, oy, (double*)nullptr);
    hipLaunchKernelGGL(k_to_tag_order<double>, dim3(g), dim3(256), 0, s->stream, (const double*)ox,
                       (const int*)cur.tag, (const int*)cur.sys, (const SysParam*)s->d_sp, fx, N);
    hipLaunchKernelGGL(k_to_tag_order<double>, dim3(g), dim3(256), 0, s->stream, (const double*)oy,
                       (const int*)cur.tag, (const int*)cur.sys, (const SysParam*)s->d_sp, fy, N);
    HIP_TRY(hipGetLastError());
    return SPV_OK;
}
}  // namespace

// ====================================================================== active vertex model
#include "avm_kernels.hpp"
#include "avm_api.hpp"

// ====================================================================== C-ABI
extern "C" {

const char* spv_last_error(void) { return g_err.c_str(); }

// kcap 0: rings of up to 16 entries, or 32 when the starting triangulation
// has a longer ring (the creation is repeated once with 32; a ring that
// outgrows the capacity later in the run is an error, as with kcap given)
spv_status create_regrow(CreateArgs& a, int64_t Ntot, spv_sys** out)
{
    const bool auto_cap = a.prm.kcap == 0;
    spv_status st = create_tuned(a, out);
    if (st != SPV_ECAPACITY || !auto_cap) return st;
    ST_TRY(check_ring_extent(Ntot, 32));
    a.prm.kcap = 32;
    return create_tuned(a, out);
}

spv_status spv_create(spv_sys** out, int64_t N, const double* x, const double* y, double Lx, double Ly,
                      const double* A0, const double* P0, double p0, const double* theta0,
                      const spv_params* params, void* stream)
{
    if (!out) return fail(SPV_EINVAL, "out is NULL");
    *out = nullptr;
    if (N < 3 || N > (int64_t)1 << 30) return fail(SPV_EINVAL, "N must be in [3, 2^30]");
    if (!x || !y || !params) return fail(SPV_EINVAL, "x, y and params are required");
    if (!(Lx > 0.0) || !(Ly > 0.0) || !std::isfinite(Lx) || !std::isfinite(Ly))
        return fail(SPV_EINVAL, "box sides must be positive and finite");
    if (!A0 && !P0 && !std::isfinite(p0)) return fail(SPV_EINVAL, "p0 must be finite");
    {
        spv_sys probe;  // parameters are checked before any copy
        ST_TRY(setup_params(&probe, params, stream));
        ST_TRY(check_ring_extent(N, probe.KC));
    }
    CreateArgs a;
    a.prm = *params;
    a.stream = stream;
    ST_TRY(copy_in(x, a.x, N));
    ST_TRY(copy_in(y, a.y, N));
    if (A0) {
        ST_TRY(copy_in(A0, a.A0, N));
    } else {
        a.A0.assign(N, 1.0);
    }
    if (P0) {
        ST_TRY(copy_in(P0, a.P0, N));
    } else {
        a.P0.resize(N);
        for (int64_t i = 0; i < N; i++) a.P0[i] = p0 * std::sqrt(a.A0[i]);
    }
    for (int64_t i = 0; i < N; i++)
        if (!std::isfinite(a.A0[i]) || !std::isfinite(a.P0[i]) || a.A0[i] <= 0.0)
            return fail(SPV_EINVAL, "A0 must be positive and finite, P0 finite");
    if (theta0) {
        ST_TRY(copy_in(theta0, a.th, N));
        for (int64_t i = 0; i < N; i++)
            if (!std::isfinite(a.th[i])) return fail(SPV_EINVAL, "theta0 must be finite");
    }
    a.in = {{N, Lx, Ly, params->v0, params->seed}};
    return create_regrow(a, N, out);
}

spv_status spv_batch_create(spv_sys** out, int32_t S, const int64_t* N_s, const double* Lx_s, const double* Ly_s,
                            const double* x, const double* y, const double* P0, const double* p0_s,
                            const double* v0_s, const uint64_t* seed_s, const spv_params* params, void* stream)
{
    if (!out) return fail(SPV_EINVAL, "out is NULL");
    *out = nullptr;
    if (S < 1 || !N_s || !Lx_s || !Ly_s || !x || !y || !params || (!P0 && !p0_s))
        return fail(SPV_EINVAL, "bad batch arguments");
    std::vector<SysInput> in(S);
    int64_t Ntot = 0;
    for (int k = 0; k < S; k++) {
        if (N_s[k] < 3 || !(Lx_s[k] > 0.0) || !(Ly_s[k] > 0.0) || !std::isfinite(Lx_s[k]) || !std::isfinite(Ly_s[k]))
            return fail(SPV_EINVAL, "every system needs N >= 3 and a positive finite box");
        in[k] = {N_s[k], Lx_s[k], Ly_s[k], v0_s ? v0_s[k] : params->v0, seed_s ? seed_s[k] : params->seed};
        if (!std::isfinite(in[k].v0)) return fail(SPV_EINVAL, "v0 must be finite");
        Ntot += N_s[k];
        if (Ntot > (int64_t)1 << 30) return fail(SPV_EINVAL, "too many cells");
    }
    {
        spv_sys probe;
        ST_TRY(setup_params(&probe, params, stream));
        ST_TRY(check_ring_extent(Ntot, probe.KC));
    }
    CreateArgs a;
    a.prm = *params;
    a.stream = stream;
    a.in = in;
    a.A0.assign(Ntot, 1.0);
    ST_TRY(copy_in(x, a.x, Ntot));
    ST_TRY(copy_in(y, a.y, Ntot));
    if (P0) {
        ST_TRY(copy_in(P0, a.P0, Ntot));
    } else {
        a.P0.resize(Ntot);
        int64_t o = 0;
        for (int k = 0; k < S; k++)
            for (int64_t t = 0; t < N_s[k]; t++) a.P0[o++] = p0_s[k];
    }
    for (int64_t i = 0; i < Ntot; i++)
        if (!std::isfinite(a.P0[i])) return fail(SPV_EINVAL, "P0 must be finite");
    return create_regrow(a, Ntot, out);
}

// kcap 0: a ring that outgrows 16 entries during a run.  The step that
// failed has moved the cells but not finished its topology; the state is
// saved as it is (the sticky error set aside), a handle with kcap 32 and the
// same knobs is built from it, and the state is loaded there, which rebuilds
// the topology of those positions from scratch -- the finished step.  The
// new handle's contents then replace this one's (the caller's pointer stays
// valid; statistics restart as after spv_load_state).
spv_status regrow_capacity(spv_sys* s)
{
    std::vector<char> buf((size_t)state_bytes(s));
    const spv_status sticky = s->sticky;
    const std::string sticky_msg = s->sticky_msg;
    s->sticky = SPV_OK;
    spv_status st = save_state(s, buf.data(), (int64_t)buf.size(), nullptr);
    s->sticky = sticky;
    s->sticky_msg = sticky_msg;
    ST_TRY(st);
    StateHeader h;
    std::memcpy(&h, buf.data(), sizeof h);
    CreateArgs a;
    a.stream = s->stream;
    const char* p = buf.data() + sizeof h;
    for (int k = 0; k < h.S; k++) {
        StateSystem r;
        std::memcpy(&r, p, sizeof r);
        p += sizeof r;
        a.in.push_back({r.n, r.Lx, r.Ly, r.v0, r.seed});
    }
    const size_t N = (size_t)h.N;
    const double* arr = reinterpret_cast<const double*>(p);
    a.x.assign(arr, arr + N);
    a.y.assign(arr + N, arr + 2 * N);
    a.th.assign(arr + 2 * N, arr + 3 * N);
    a.A0.assign(arr + 3 * N, arr + 4 * N);
    a.P0.assign(arr + 4 * N, arr + 5 * N);
    spv_params prm = with_knobs(s->prm, knobs_of(s));
    prm.kcap = 32;
    ST_TRY(check_ring_extent((int64_t)N, 32));
    spv_sys* t = nullptr;
    ST_TRY(build_handle(a, prm, &t));
    st = load_state(t, buf.data(), (int64_t)buf.size());
    if (st != SPV_OK) {
        destroy_all(t);
        return st;
    }
    t->prm.kcap = 0;  // still the caller's setting
    t->tune_source = s->tune_source;
    t->tune_ms = s->tune_ms;
    const bool timing = s->timing;
    std::swap(*s, *t);
    destroy_all(t);  // the old arrays, graphs and streams
    if (timing) ST_TRY(spv_set_timing(s, 1));
    return SPV_OK;
}

spv_status spv_step(spv_sys* s, int64_t nsteps)
{
    if (!s || nsteps < 0) return fail(SPV_EINVAL, "bad handle or nsteps");
    s->traj_valid = false;  // the recorded trajectory no longer ends at the current state
    const uint64_t target = s->step + (uint64_t)nsteps;
    spv_status st = run_steps(s, nsteps);
    if (st == SPV_ECAPACITY && s->prm.kcap == 0 && s->KC == 16 && (s->h_st->err & ERR_CAPACITY)) {
        ST_TRY(regrow_capacity(s));
        st = run_steps(s, (int64_t)(target - s->step));
    }
    return st;
}

spv_status spv_save_state(spv_sys* s, void* buf, int64_t cap, int64_t* needed)
{
    if (!s || cap < 0) return fail(SPV_EINVAL, "bad handle or capacity");
    return save_state(s, buf, cap, needed);
}

spv_status spv_load_state(spv_sys* s, const void* buf, int64_t len)
{
    if (!s) return fail(SPV_EINVAL, "bad handle");
    return load_state(s, buf, len);
}

spv_status spv_get_tuning(spv_sys* s, spv_tuning* out)
{
    if (!s || !out) return fail(SPV_EINVAL, "bad argument");
    out->resort_every = s->unit;
    out->device_rounds = s->dev_rounds;
    out->repair_cells = s->repair_cells;
    out->tail_items = s->tail_items;
    out->full_rounds = s->full_rounds;
    out->force_mode = items_kernel(s) ? 2 : 1;
    out->source = s->tune_source;
    out->bin_factor = s->bin_factor;
    out->ms_per_step = s->tune_ms;
    return SPV_OK;
}

spv_status spv_get_kcap(spv_sys* s, int32_t* kcap)
{
    if (!s || !kcap) return fail(SPV_EINVAL, "bad argument");
    *kcap = s->KC;
    return SPV_OK;
}

spv_status spv_get_size(spv_sys* s, int32_t* S, int64_t* N)
{
    if (!s) return fail(SPV_EINVAL, "bad handle");
    if (S) *S = s->S;
    if (N) *N = s->N;
    return SPV_OK;
}

spv_status spv_get_system_range(spv_sys* s, int32_t sys, int64_t* first, int64_t* n)
{
    if (!s || sys < 0 || sys >= s->S) return fail(SPV_EINVAL, "bad handle or system index");
    if (first) *first = s->hsp[sys].cell_off;
    if (n) *n = s->hsp[sys].n;
    return SPV_OK;
}

spv_status spv_get_system_box(spv_sys* s, int32_t sys, double* Lx, double* Ly, int32_t* q)
{
    if (!s || sys < 0 || sys >= s->S) return fail(SPV_EINVAL, "bad handle or system index");
    if (Lx) *Lx = s->hsp[sys].Lx;
    if (Ly) *Ly = s->hsp[sys].Ly;
    if (q) *q = grid_exponent(std::max(s->hsp[sys].Lx, s->hsp[sys].Ly));
    return SPV_OK;
}

spv_status spv_get_box(spv_sys* s, double* Lx, double* Ly, int32_t* q) { return spv_get_system_box(s, 0, Lx, Ly, q); }

spv_status spv_get_positions(spv_sys* s, double* x, double* y)
{
    if (!s || !x || !y) return fail(SPV_EINVAL, "bad argument");
    const int par = s->pos & 1;
    const ArraySet& cur = s->set[par ? s->cfg ^ 1 : s->cfg];
    ST_TRY(out_tag_order(s, cur.x, x));
    return out_tag_order(s, cur.y, y);
}

spv_status spv_get_directors(spv_sys* s, double* theta)
{
    if (!s || !theta) return fail(SPV_EINVAL, "bad argument");
    const int par = s->pos & 1;
    const ArraySet& cur = s->set[par ? s->cfg ^ 1 : s->cfg];
    return out_tag_order(s, cur.th, theta);
}

spv_status spv_get_forces(spv_sys* s, double* fx, double* fy)
{
    if (!s || !fx || !fy) return fail(SPV_EINVAL, "bad argument");
    dispatch(s, [&]<typename R, bool MULTI, int KC>() {
        Cells<R> c = cells<R>(s, s->cfg, s->pos & 1);
        hipLaunchKernelGGL((force_kernel<R, MULTI, KC, false>(s)), dim3(force_grid(s)), dim3(256), 0, s->stream, c,
                           (double*)nullptr, (double*)nullptr, (double*)nullptr, s->d_fx, s->d_fy, s->d_sp, s->d_st,
                           s->N, s->d_blockmax, CellCount{});
    });
    HIP_TRY(hipGetLastError());
    ST_TRY(out_tag_order(s, s->d_fx, fx));
    return out_tag_order(s, s->d_fy, fy);
}

spv_status spv_get_geometry(spv_sys* s, double* A, double* P)
{
    if (!s || !A || !P) return fail(SPV_EINVAL, "bad argument");
    const ArraySet& cur = s->set[s->cfg];
    if (s->mixed) {
        ST_TRY(out_tag_order(s, static_cast<const float*>(cur.A), A));
        return out_tag_order(s, static_cast<const float*>(cur.P), P);
    }
    ST_TRY(out_tag_order(s, static_cast<const double*>(cur.A), A));
    return out_tag_order(s, static_cast<const double*>(cur.P), P);
}

spv_status spv_get_neighbors(spv_sys* s, int32_t* offsets, int32_t* nbr, int64_t cap, int64_t* needed)
{
    if (!s || !offsets) return fail(SPV_EINVAL, "bad argument");
    const int N = s->N, K = s->KC;
    const ArraySet& cur = s->set[s->cfg];
    std::vector<uint8_t> deg(N);
    std::vector<int> ring((size_t)N * K), tag(N), sys(N);
    HIP_TRY(hipMemcpyAsync(deg.data(), cur.deg, N, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(ring.data(), cur.ring, (size_t)N * K * sizeof(int), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(tag.data(), cur.tag, N * sizeof(int), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(sys.data(), cur.sys, N * sizeof(int), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    std::vector<int> gid(N), slot_of(N);
    for (int i = 0; i < N; i++) {
        gid[i] = s->hsp[sys[i]].cell_off + tag[i];
        slot_of[gid[i]] = i;
    }
    int64_t tot = 0;
    for (int t = 0; t < N; t++) {
        offsets[t] = (int32_t)tot;
        tot += deg[slot_of[t]];
    }
    offsets[N] = (int32_t)tot;
    if (needed) *needed = tot;
    if (!nbr || cap < tot) return fail(SPV_ECAPACITY, "nbr buffer too small");
    for (int t = 0; t < N; t++) {
        const int i = slot_of[t];
        for (int m = 0; m < deg[i]; m++) nbr[offsets[t] + m] = gid[ring[rslot_host(RLO * N, K, i, m)]];
    }
    return SPV_OK;
}

spv_status spv_debug_set_ring(spv_sys* s, int64_t cell, int32_t k, const int32_t* nbr)
{
    if (!s || !nbr) return fail(SPV_EINVAL, "bad argument");
    const int N = s->N, K = s->KC;
    if (cell < 0 || cell >= N) return fail(SPV_EINVAL, "cell index out of range");
    if (k < 3 || k > K) return fail(SPV_EINVAL, "ring length outside [3, kcap]");
    int sysk = 0;
    while (sysk + 1 < s->S && s->hsp[sysk + 1].cell_off <= cell) sysk++;
    const int64_t lo = s->hsp[sysk].cell_off, hi = lo + s->hsp[sysk].n;
    for (int m = 0; m < k; m++) {
        if (nbr[m] < lo || nbr[m] >= hi || nbr[m] == cell)
            return fail(SPV_EINVAL, "ring member outside the cell's system or the cell itself");
        for (int q = 0; q < m; q++)
            if (nbr[q] == nbr[m]) return fail(SPV_EINVAL, "repeated ring member");
    }
    const ArraySet& cur = s->set[s->cfg];
    std::vector<int> tag(N), sys(N);
    HIP_TRY(hipMemcpyAsync(tag.data(), cur.tag, N * sizeof(int), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(sys.data(), cur.sys, N * sizeof(int), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    std::vector<int> slot_of(N);
    for (int i = 0; i < N; i++) slot_of[s->hsp[sys[i]].cell_off + tag[i]] = i;
    // the row in its two parts (first RLO slots, then the overflow part),
    // every slot past k cleared; no opposite cell recorded for any edge
    const int i = slot_of[cell];
    std::vector<int> row(K, -1), opp(K, -1);
    for (int m = 0; m < k; m++) row[m] = slot_of[nbr[m]];
    const uint8_t d = (uint8_t)k;
    const size_t lo_off = (size_t)i * RLO, hi_off = (size_t)RLO * N + (size_t)i * (K - RLO);
    HIP_TRY(hipMemcpyAsync(cur.ring + lo_off, row.data(), RLO * sizeof(int), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(cur.ring + hi_off, row.data() + RLO, (K - RLO) * sizeof(int), hipMemcpyHostToDevice,
                           s->stream));
    HIP_TRY(hipMemcpyAsync(cur.opp + lo_off, opp.data(), RLO * sizeof(int), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(cur.opp + hi_off, opp.data() + RLO, (K - RLO) * sizeof(int), hipMemcpyHostToDevice,
                           s->stream));
    HIP_TRY(hipMemcpyAsync(cur.deg + i, &d, 1, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->traj_valid = false;
    return SPV_OK;
}

static spv_status observables_all(spv_sys* s, std::vector<double>& h)
{
    const ArraySet& cur = s->set[s->cfg];
    const int ch = s->obs_chunks;
    if (s->mixed)
        hipLaunchKernelGGL(k_observables<float>, dim3(s->S * ch), dim3(256), 0, s->stream, (const float*)cur.A,
                           (const float*)cur.P, cur.A0, cur.P0, s->d_sp, ch, s->d_obs_part);
    else
        hipLaunchKernelGGL(k_observables<double>, dim3(s->S * ch), dim3(256), 0, s->stream, (const double*)cur.A,
                           (const double*)cur.P, cur.A0, cur.P0, s->d_sp, ch, s->d_obs_part);
    hipLaunchKernelGGL(k_observables_sum, dim3(s->S), dim3(64), 0, s->stream, (const double*)s->d_obs_part, ch,
                       s->d_obs);
    HIP_TRY(hipGetLastError());
    h.resize(3 * s->S);
    HIP_TRY(hipMemcpyAsync(h.data(), s->d_obs, 3 * s->S * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    return read_state(s);
}

spv_status spv_get_observables(spv_sys* s, double* E, double* qbar, double* sumA, int64_t* counters)
{
    if (!s) return fail(SPV_EINVAL, "bad handle");
    std::vector<double> h;
    ST_TRY(observables_all(s, h));
    double e = 0, q = 0, a = 0;
    for (int k = 0; k < s->S; k++) {
        e += h[3 * k];
        q += h[3 * k + 1];
        a += h[3 * k + 2];
    }
    if (E) *E = e;
    if (qbar) *qbar = q / s->N;
    if (sumA) *sumA = a;
    if (counters) {
        const DevState& d = *s->h_st;
        counters[0] = (int64_t)s->step;
        counters[1] = (int64_t)d.repaired + s->hyb_repaired;
        counters[2] = (int64_t)d.rounds + s->hyb_rounds;
        counters[3] = (int64_t)d.exact_calls;
        {
            std::vector<uint8_t> deg(s->N);
            HIP_TRY(hipMemcpy(deg.data(), s->set[s->cfg].deg, s->N, hipMemcpyDeviceToHost));
            counters[4] = *std::max_element(deg.begin(), deg.end());
        }
        counters[5] = s->resorts;
        counters[6] = (int64_t)d.retries;
        counters[7] = (int64_t)d.err;
        counters[8] = s->graph_periods;
        counters[9] = s->dense_steps;
        counters[10] = s->host_rounds;
        counters[11] = s->recoveries;
        counters[12] = (int64_t)d.candidates + s->hr.candidates;
    }
    return SPV_OK;
}

spv_status spv_get_system_observables(spv_sys* s, int32_t sys, double* E, double* qbar, double* sumA)
{
    if (!s || sys < 0 || sys >= s->S) return fail(SPV_EINVAL, "bad handle or system index");
    std::vector<double> h;
    ST_TRY(observables_all(s, h));
    if (E) *E = h[3 * sys];
    if (qbar) *qbar = h[3 * sys + 1] / s->hsp[sys].n;
    if (sumA) *sumA = h[3 * sys + 2];
    return SPV_OK;
}

spv_status spv_set_timing(spv_sys* s, int32_t enable)
{
    if (!s) return fail(SPV_EINVAL, "bad handle");
    HIP_TRY(hipStreamSynchronize(s->stream));
    collect_eager_timing(s);
    s->timing = enable != 0;
    for (int k = 0; k < T_COUNT; k++) {
        s->t_ms[k] = 0.0;
        s->t_n[k] = 0;
    }
    return SPV_OK;
}

spv_status spv_kernel_time(spv_sys* s, int32_t which, double* total_ms, int64_t* launches)
{
    if (!s || which < 0 || which >= T_COUNT) return fail(SPV_EINVAL, "bad argument");
    HIP_TRY(hipStreamSynchronize(s->stream));
    collect_eager_timing(s);
    if (total_ms) *total_ms = s->t_ms[which];
    if (launches) *launches = s->t_n[which];
    return SPV_OK;
}

spv_status spv_traj_forward(spv_sys* s, int64_t T, int64_t ckpt_every, double* Q)
{
    if (!s) return fail(SPV_EINVAL, "bad handle");
    return traj_forward(s, T, ckpt_every, Q);
}

spv_status spv_traj_backward(spv_sys* s, double dQ, double* dQ_dp0)
{
    if (!s || !dQ_dp0) return fail(SPV_EINVAL, "bad argument");
    return traj_backward(s, dQ, dQ_dp0);
}

spv_status spv_force_tangent(spv_sys* s, const double* vx, const double* vy, double* fx, double* fy)
{
    if (!s || !vx || !vy || !fx || !fy) return fail(SPV_EINVAL, "bad argument");
    if (s->mixed || s->S != 1) return fail(SPV_EINVAL, "the force tangent needs a single FP64 system");
    return s->KC == 16 ? hvp_impl<16>(s, vx, vy, fx, fy) : hvp_impl<32>(s, vx, vy, fx, fy);
}


spv_status spv_force_tangent_static(spv_sys* s, const double* vx, const double* vy, double* fx, double* fy)
{
    if (!s || !vx || !vy || !fx || !fy) return fail(SPV_EINVAL, "bad argument");
    if (s->mixed || s->S != 1) return fail(SPV_EINVAL, "the force tangent needs a single FP64 system");
    if (s->N > kStaticCells)
        return fail(SPV_EINVAL, "spv_force_tangent_static takes at most 65536 cells (its static scratch)");
    if (!device_pointer(vx) || !device_pointer(vy) || !device_pointer(fx) || !device_pointer(fy))
        return fail(SPV_EINVAL, "spv_force_tangent_static needs device pointers");
    if (!s->scratch) return fail(SPV_EHIP, "no static scratch on this handle's device");
    if (s->sticky != SPV_OK) return fail(s->sticky, s->sticky_msg);
    return s->KC == 16 ? hvp_static<16>(s, vx, vy, fx, fy) : hvp_static<32>(s, vx, vy, fx, fy);
}

spv_status spv_destroy(spv_sys* s)
{
    if (!s) return fail(SPV_EINVAL, "bad handle");
    destroy_all(s);
    return SPV_OK;
}

// ---------------------------------------------------------------- active vertex model
spv_status spv_avm_create(spv_avm** out, int64_t Nc, int64_t Nv, const double* vx, const double* vy,
                          const int32_t* cell_off, const int32_t* cell_vtx, double Lx, double Ly, const double* A0,
                          const double* P0, double p0, const double* theta0, const spv_avm_params* params,
                          void* stream)
{
    if (!out) return fail(SPV_EINVAL, "out is NULL");
    *out = nullptr;
    if (!vx || !vy || !cell_off || !cell_vtx || !params) return fail(SPV_EINVAL, "missing argument");
    if (Nc < 3 || Nc > (1 << 28) || Nv != 2 * Nc)
        return fail(SPV_EINVAL, "a trivalent tiling of the torus has Nv = 2 Nc vertices (Nc >= 3)");
    if (!(Lx > 0.0) || !(Ly > 0.0) || !std::isfinite(Lx) || !std::isfinite(Ly))
        return fail(SPV_EINVAL, "box sides must be positive and finite");
    const spv_avm_params& pr = *params;
    if (!(pr.dt > 0.0) || !(pr.Dr >= 0.0) || !std::isfinite(pr.mu) || !std::isfinite(pr.v0) ||
        !std::isfinite(pr.KA) || !std::isfinite(pr.KP) || !std::isfinite(pr.dt) || !std::isfinite(pr.Dr))
        return fail(SPV_EINVAL, "invalid model parameters");
    if (!(pr.t1_length > 0.0) || !std::isfinite(pr.t1_length) || pr.t1_new_length < 0.0 ||
        !std::isfinite(pr.t1_new_length))
        return fail(SPV_EINVAL, "t1_length must be positive, t1_new_length non-negative");
    const double lnew = pr.t1_new_length > 0.0 ? pr.t1_new_length : 1.5 * pr.t1_length;
    if (!(lnew > pr.t1_length)) return fail(SPV_EINVAL, "t1_new_length must exceed t1_length");
    if (pr.resort_every < -1) return fail(SPV_EINVAL, "resort_every must be -1, 0 or positive");
    if (pr.bin_order != 0 && pr.bin_order != 1) return fail(SPV_EINVAL, "bin_order must be 0 or 1");
    const int nc = (int)Nc, nv = (int)Nv;
    std::vector<int32_t> off(nc + 1);
    HIP_TRY(hipMemcpy(off.data(), cell_off, (nc + 1) * sizeof(int32_t), hipMemcpyDefault));
    if (off[nc] != 3 * nv) return fail(SPV_EINVAL, "the cells must list 3 Nv vertex entries in all");
    std::vector<int32_t> cv(off[nc]);
    HIP_TRY(hipMemcpy(cv.data(), cell_vtx, cv.size() * sizeof(int32_t), hipMemcpyDefault));
    std::vector<double> hx, hy, ha0(nc, 1.0), hp0(nc), hth;
    ST_TRY(copy_in(vx, hx, nv));
    ST_TRY(copy_in(vy, hy, nv));
    if (A0) ST_TRY(copy_in(A0, ha0, nc));
    if (P0) {
        ST_TRY(copy_in(P0, hp0, nc));
    } else {
        if (!std::isfinite(p0)) return fail(SPV_EINVAL, "p0 must be finite");
        for (int c = 0; c < nc; c++) hp0[c] = p0 * std::sqrt(ha0[c]);
    }
    for (int c = 0; c < nc; c++)
        if (!(ha0[c] > 0.0) || !std::isfinite(ha0[c]) || !std::isfinite(hp0[c]))
            return fail(SPV_EINVAL, "A0 must be positive and finite, P0 finite");
    if (theta0) ST_TRY(copy_in(theta0, hth, nc));
    std::vector<int> vv, vc, cvf;
    std::vector<uint8_t> deg;
    ST_TRY(avm_topology(nc, nv, off, cv, vv, vc, cvf, deg));
    spv_avm* h = new spv_avm();
    h->nc = nc;
    h->nv = nv;
    h->stream = (hipStream_t)stream;
    h->resort_every = pr.resort_every == 0 ? AVM_DEFAULT_RESORT : pr.resort_every;
    AvmParam& P = h->hp;
    const int q = grid_exponent(std::max(Lx, Ly));
    P.scale = std::ldexp(1.0, q);
    P.inv_scale = 1.0 / P.scale;
    P.LXu = std::rint(Lx * P.scale);
    P.LYu = std::rint(Ly * P.scale);
    P.Lx = P.LXu / P.scale;
    P.Ly = P.LYu / P.scale;
    P.hLx = 0.5 * P.Lx;
    P.hLy = 0.5 * P.Ly;
    P.mu = pr.mu;
    P.v0 = pr.v0;
    P.dt = pr.dt;
    P.amp = std::sqrt(2.0 * pr.Dr * pr.dt);
    P.KA = pr.KA;
    P.KP = pr.KP;
    P.lt1sq = pr.t1_length * pr.t1_length;
    P.lnew = lnew;
    P.seed = pr.seed;
    for (int v = 0; v < nv; v++) {
        if (!std::isfinite(hx[v]) || !std::isfinite(hy[v]) || hx[v] < 0.0 || hx[v] >= Lx || hy[v] < 0.0 ||
            hy[v] >= Ly) {
            avm_free(h);
            return fail(SPV_EINVAL, "vertex positions must be finite and inside [0,Lx) x [0,Ly)");
        }
        double X = std::rint(hx[v] * P.scale), Y = std::rint(hy[v] * P.scale);
        if (X >= P.LXu) X -= P.LXu;
        if (Y >= P.LYu) Y -= P.LYu;
        hx[v] = X / P.scale;
        hy[v] = Y / P.scale;
    }
    spv_status st = SPV_OK;
    auto T = [&](spv_status x) {
        if (st == SPV_OK) st = x;
    };
    AvmDev& d = h->d;
    const std::vector<int> rank = avm_bin_ranks(h->bins, P.Lx, P.Ly, nc, pr.bin_order);
    const int nb = h->bins.nb;
    const bool sorting = h->resort_every > 0;
    for (int b = 0; b < 2; b++) {
        T(avm_alloc(h, &d.x[b], nv));
        T(avm_alloc(h, &d.y[b], nv));
        if (b == 1 && !sorting) break;  // one array set without re-sorts
        T(avm_alloc(h, &d.vv[b], 3 * (size_t)nv));
        T(avm_alloc(h, &d.vc[b], 3 * (size_t)nv));
        T(avm_alloc(h, &d.cv[b], (size_t)nc * AVM_KV));
        T(avm_alloc(h, &d.vtag[b], nv));
        T(avm_alloc(h, &d.ctag[b], nc));
        T(avm_alloc(h, &d.cdeg[b], nc));
        for (double** p : {&d.th[b], &d.A0[b], &d.P0[b]}) T(avm_alloc(h, p, nc));
    }
    const size_t nv8 = ((size_t)nv + 7) / 8 * 8;
    T(avm_alloc(h, &d.cand, nv8));
    T(avm_alloc(h, &d.dirty, nv8));
    T(avm_alloc(h, &d.lcell, 12 * (size_t)nv));
    for (double** p : {&d.A, &d.P, &d.ca, &d.cb}) T(avm_alloc(h, p, nc));
    T(avm_alloc(h, &d.fx, nv));
    T(avm_alloc(h, &d.fy, nv));
    T(avm_alloc(h, &d.out, nv));
    T(avm_alloc(h, &d.lock[0], nc));
    T(avm_alloc(h, &d.lock[1], nc));
    if (sorting) {
        for (int** p : {&d.vkey, &d.vperm, &d.vinv}) T(avm_alloc(h, p, nv));
        for (int** p : {&d.ckey, &d.cperm, &d.cinv}) T(avm_alloc(h, p, nc));
        for (int** p : {&d.vcount, &d.ccount, &d.rank}) T(avm_alloc(h, p, nb));
        for (int** p : {&d.vstart, &d.cstart}) T(avm_alloc(h, p, (size_t)nb + 1));
        for (int** p : {&d.vchunk, &d.cchunk}) T(avm_alloc(h, p, (size_t)grid_for(nb, SCAN_CHUNK) + 1));
        T(avm_alloc(h, &h->d_scan, 1));
    }
    h->bins.rank = d.rank;
    T(avm_alloc(h, &h->d_p, 1));
    T(avm_alloc(h, &h->d_st, 1));
    T(avm_alloc(h, &h->d_sp, 1));
    h->obs_chunks = (nc + OBS_CHUNK - 1) / OBS_CHUNK;
    T(avm_alloc(h, &h->d_obs, 3));
    T(avm_alloc(h, &h->d_obs_part, 3 * (size_t)h->obs_chunks));
    if (st != SPV_OK) {
        std::string keep = spv_last_error();
        avm_free(h);
        return fail(st, keep);
    }
    if (hipHostMalloc((void**)&h->h_st, sizeof(AvmState), hipHostMallocDefault) != hipSuccess) {
        avm_free(h);
        return fail(SPV_ENOMEM, "hipHostMalloc failed");
    }
    std::memset(h->h_st, 0, sizeof(AvmState));
    SysParam sp{};
    sp.KA = pr.KA;
    sp.KP = pr.KP;
    sp.n = nc;
    hipStream_t s = h->stream;
    auto up = [&](void* dst, const void* src, size_t bytes) {
        if (st == SPV_OK && hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) != hipSuccess)
            st = fail(SPV_EHIP, "upload failed");
    };
    up(d.x[0], hx.data(), nv * sizeof(double));
    up(d.y[0], hy.data(), nv * sizeof(double));
    up(d.vv[0], vv.data(), vv.size() * sizeof(int));
    up(d.vc[0], vc.data(), vc.size() * sizeof(int));
    up(d.cv[0], cvf.data(), cvf.size() * sizeof(int));
    up(d.cdeg[0], deg.data(), nc);
    up(d.A0[0], ha0.data(), nc * sizeof(double));
    up(d.P0[0], hp0.data(), nc * sizeof(double));
    if (!hth.empty()) up(d.th[0], hth.data(), nc * sizeof(double));
    if (sorting) up(d.rank, rank.data(), nb * sizeof(int));
    up(h->d_p, &h->hp, sizeof(AvmParam));
    up(h->d_st, h->h_st, sizeof(AvmState));
    up(h->d_sp, &sp, sizeof(SysParam));
    if (st == SPV_OK) {
        if (hth.empty())
            hipLaunchKernelGGL(k_avm_theta0, dim3(avm_grid(nc)), dim3(256), 0, s, d.th[0], (uint64_t)pr.seed, nc);
        hipLaunchKernelGGL(k_avm_fill_lock, dim3(avm_grid(nc)), dim3(256), 0, s, d.lock[0], d.lock[1], nc);
        HIP_TRY(hipMemsetAsync(d.cand, 0, nv8, s));
        HIP_TRY(hipMemsetAsync(d.dirty, 0, nv8, s));
        hipLaunchKernelGGL(k_avm_iota, dim3(avm_grid(nv)), dim3(256), 0, s, d.vtag[0], nv);
        hipLaunchKernelGGL(k_avm_iota, dim3(avm_grid(nc)), dim3(256), 0, s, d.ctag[0], nc);
        if (sorting) {
            hipLaunchKernelGGL(k_fill_i32, dim3(avm_grid(nb)), dim3(256), 0, s, d.vcount, nb, 0);
            hipLaunchKernelGGL(k_fill_i32, dim3(avm_grid(nb)), dim3(256), 0, s, d.ccount, nb, 0);
            HIP_TRY(hipMemsetAsync(h->d_scan, 0, sizeof(DevState), s));
        }
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
            st = fail(SPV_EHIP, "initialisation kernels failed");
    }
    if (st == SPV_OK && sorting) st = avm_resort(h);
    if (st != SPV_OK) {
        std::string keep = spv_last_error();
        avm_free(h);
        return fail(st, keep);
    }
    *out = h;
    return SPV_OK;
}

spv_status spv_avm_step(spv_avm* h, int64_t nsteps)
{
    if (!h || nsteps < 0) return fail(SPV_EINVAL, "bad argument");
    return avm_steps(h, nsteps);
}

// a per-slot array into label order, then to the caller's memory (host or
// device)
static spv_status avm_out(spv_avm* h, const double* src, bool vertices, double* dst)
{
    const int n = vertices ? h->nv : h->nc;
    const int* tag = vertices ? h->d.vtag[h->set] : h->d.ctag[h->set];
    hipLaunchKernelGGL(k_avm_by_label, dim3(avm_grid(n)), dim3(256), 0, h->stream, src, tag, h->d.out, n);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(dst, h->d.out, n * sizeof(double), hipMemcpyDefault, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return SPV_OK;
}

spv_status spv_avm_get_vertices(spv_avm* h, double* vx, double* vy)
{
    if (!h || !vx || !vy) return fail(SPV_EINVAL, "bad argument");
    ST_TRY(avm_out(h, h->d.x[h->cur], true, vx));
    return avm_out(h, h->d.y[h->cur], true, vy);
}

spv_status spv_avm_get_directors(spv_avm* h, double* theta)
{
    if (!h || !theta) return fail(SPV_EINVAL, "bad argument");
    return avm_out(h, h->d.th[h->set], false, theta);
}

// geometry and forces at the current state (the step's own kernels without
// the move)
static spv_status avm_eval(spv_avm* h)
{
    if (h->sticky != SPV_OK) return fail(h->sticky, h->sticky_msg);
    const AvmArrays a = avm_arrays(h, h->cur);
    hipLaunchKernelGGL(k_avm_geom, dim3(avm_grid(h->nc)), dim3(256), 0, h->stream, a, (const AvmParam*)h->d_p,
                       h->d_st);
    hipLaunchKernelGGL(k_avm_force<false>, dim3(avm_grid(h->nv)), dim3(256), 0, h->stream, a,
                       (const AvmParam*)h->d_p, h->d_st);
    HIP_TRY(hipGetLastError());
    return SPV_OK;
}

spv_status spv_avm_get_forces(spv_avm* h, double* fx, double* fy)
{
    if (!h || !fx || !fy) return fail(SPV_EINVAL, "bad argument");
    ST_TRY(avm_eval(h));
    ST_TRY(avm_out(h, h->d.fx, true, fx));
    return avm_out(h, h->d.fy, true, fy);
}

spv_status spv_avm_get_geometry(spv_avm* h, double* A, double* P)
{
    if (!h || !A || !P) return fail(SPV_EINVAL, "bad argument");
    ST_TRY(avm_eval(h));
    ST_TRY(avm_out(h, h->d.A, false, A));
    return avm_out(h, h->d.P, false, P);
}

spv_status spv_avm_get_cells(spv_avm* h, int32_t* cell_off, int32_t* cell_vtx, int64_t cap, int64_t* needed)
{
    if (!h || !cell_off) return fail(SPV_EINVAL, "bad argument");
    const int nc = h->nc, nv = h->nv, s = h->set;
    std::vector<int> cvf((size_t)nc * AVM_KV), vtag(nv), ctag(nc);
    std::vector<uint8_t> deg(nc);
    HIP_TRY(hipMemcpyAsync(cvf.data(), h->d.cv[s], cvf.size() * sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpyAsync(deg.data(), h->d.cdeg[s], nc, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpyAsync(vtag.data(), h->d.vtag[s], nv * sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpyAsync(ctag.data(), h->d.ctag[s], nc * sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    std::vector<int> slot(nc);  // slot of each cell label
    for (int c = 0; c < nc; c++) slot[ctag[c]] = c;
    int64_t tot = 0;
    for (int t = 0; t < nc; t++) {
        cell_off[t] = (int32_t)tot;
        tot += deg[slot[t]];
    }
    cell_off[nc] = (int32_t)tot;
    if (needed) *needed = tot;
    if (!cell_vtx || cap < tot) return fail(SPV_ECAPACITY, "cell_vtx too small");
    for (int t = 0; t < nc; t++) {
        const int c = slot[t];
        for (int m = 0; m < deg[c]; m++) cell_vtx[cell_off[t] + m] = vtag[cvf[(size_t)c * AVM_KV + m]];
    }
    return SPV_OK;
}

spv_status spv_avm_get_observables(spv_avm* h, double* E, double* qbar, int64_t* counters)
{
    if (!h) return fail(SPV_EINVAL, "bad handle");
    ST_TRY(avm_eval(h));
    hipLaunchKernelGGL(k_observables<double>, dim3(h->obs_chunks), dim3(256), 0, h->stream, (const double*)h->d.A,
                       (const double*)h->d.P, (const double*)h->d.A0[h->set], (const double*)h->d.P0[h->set],
                       (const SysParam*)h->d_sp, h->obs_chunks, h->d_obs_part);
    hipLaunchKernelGGL(k_observables_sum, dim3(1), dim3(64), 0, h->stream, (const double*)h->d_obs_part,
                       h->obs_chunks, h->d_obs);
    double o[3];
    HIP_TRY(hipMemcpyAsync(o, h->d_obs, sizeof o, hipMemcpyDeviceToHost, h->stream));
    ST_TRY(avm_read(h));
    if (E) *E = o[0];
    if (qbar) *qbar = o[1] / h->nc;
    if (counters) {
        counters[0] = (int64_t)h->h_st->step;
        counters[1] = (int64_t)h->h_st->t1;
        counters[2] = (int64_t)h->h_st->rounds;
        counters[3] = h->host_rounds;
        counters[4] = h->graph_batches;
        counters[5] = h->resorts;
    }
    return SPV_OK;
}

spv_status spv_avm_destroy(spv_avm* h)
{
    if (!h) return fail(SPV_EINVAL, "bad handle");
    avm_free(h);
    return SPV_OK;
}

spv_status spv_voronoi_network(spv_sys* s, double* vx, double* vy, int32_t* cell_off, int32_t* cell_vtx)
{
    if (!s || !vx || !vy || !cell_off || !cell_vtx) return fail(SPV_EINVAL, "bad argument");
    if (s->S != 1) return fail(SPV_EINVAL, "single systems only");
    const int N = s->N;
    std::vector<double> x(N), y(N);
    ST_TRY(spv_get_positions(s, x.data(), y.data()));
    std::vector<int32_t> off(N + 1), nbr(6 * (size_t)N);
    int64_t need = 0;
    ST_TRY(spv_get_neighbors(s, off.data(), nbr.data(), (int64_t)nbr.size(), &need));
    if (need != 6 * (int64_t)N) return fail(SPV_EHIP, "unexpected neighbour count");
    const SysParam& P = s->hsp[0];
    std::map<std::array<int, 3>, int> ids;
    int nv = 0;
    for (int i = 0; i < N; i++) {
        const int k = off[i + 1] - off[i];
        for (int m = 0; m < k; m++) {
            const int a = nbr[off[i] + m], b = nbr[off[i] + (m + 1) % k];
            std::array<int, 3> t{i, a, b};
            const int r = (int)(std::min_element(t.begin(), t.end()) - t.begin());
            std::rotate(t.begin(), t.begin() + r, t.end());
            auto it = ids.find(t);
            int id;
            if (it == ids.end()) {
                // the circumcentre in i's frame (i is the triangle's smallest tag)
                const double bx = mimg(x[a] - x[i], P.Lx, P.hLx), by = mimg(y[a] - y[i], P.Ly, P.hLy);
                const double cx = mimg(x[b] - x[i], P.Lx, P.hLx), cy = mimg(y[b] - y[i], P.Ly, P.hLy);
                const double nb = bx * bx + by * by, nc = cx * cx + cy * cy, d = 2.0 * (bx * cy - by * cx);
                const double ux = (cy * nb - by * nc) / d, uy = (bx * nc - cx * nb) / d;
                double X = std::fmod(std::rint((x[i] + ux) * P.scale), P.LXu);
                double Y = std::fmod(std::rint((y[i] + uy) * P.scale), P.LYu);
                if (X < 0) X += P.LXu;
                if (Y < 0) Y += P.LYu;
                id = nv++;
                if (id >= 2 * N) return fail(SPV_EHIP, "more Voronoi vertices than 2N");
                ids.emplace(t, id);
                vx[id] = X / P.scale;
                vy[id] = Y / P.scale;
            } else {
                id = it->second;
            }
            cell_vtx[off[i] + m] = id;
        }
        cell_off[i] = off[i];
    }
    cell_off[N] = off[N];
    if (nv != 2 * N) return fail(SPV_EHIP, "the tessellation does not have 2N vertices");
    return SPV_OK;
}

}  // extern "C"
