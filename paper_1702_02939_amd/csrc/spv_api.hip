// spv_api.hip -- host runtime and C-ABI of the SPV step library (gfx950).
//
// The host side only allocates, orders launches on the handle's stream and
// reads back one small counter block per repair round; every arithmetic step
// of the model runs in the kernels of spv_kernels.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "../../include/spv.h"
#include "spv_kernels.hpp"

using namespace spv;

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

enum { T_FORCE = 0, T_GEOM = 1, T_REPAIR = 2, T_COUNT = 3 };

struct TimedLaunch {
    int which;
    hipEvent_t a, b;
};

}  // namespace

struct spv_sys {
    int N = 0;
    int kcap = 16;
    int repair_rounds = 16;
    int resort_every = 64;
    double Lx = 0, Ly = 0;
    int q = 0;
    spv_params prm{};
    hipStream_t stream = nullptr;
    View v{};   // current buffers
    View a{};   // alternate buffers (update target, re-sort target)
    // bins
    int nbins = 0;
    double spacing = 1.0;
    int* d_bin_rank = nullptr;
    int* d_bin_start = nullptr;
    int* d_key = nullptr;
    int* d_hist = nullptr;
    int* d_fill = nullptr;
    int* d_perm = nullptr;
    int* d_inv = nullptr;
    // scratch
    DevCounters* d_cnt = nullptr;
    DevCounters* h_cnt = nullptr;  // pinned
    double* d_stage = nullptr;     // N doubles
    double* d_fx = nullptr;
    double* d_fy = nullptr;
    double* d_part = nullptr;
    double* d_obs = nullptr;
    std::vector<void*> allocs;
    // bookkeeping
    uint64_t step = 0;
    int64_t steps_since_resort = 0;
    double drift = 0.0;
    int64_t repaired = 0, rounds = 0, exact_calls = 0, resorts = 0, retries = 0;
    int max_deg = 0;
    unsigned err_word = 0;
    // timing
    bool timing = false;
    double t_ms[T_COUNT] = {0, 0, 0};
    int64_t t_n[T_COUNT] = {0, 0, 0};
    std::vector<TimedLaunch> pending;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> event_pool;
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

#define ST_TRY(expr)                          \
    do {                                      \
        spv_status st_ = (expr);              \
        if (st_ != SPV_OK) return st_;        \
    } while (0)

spv_status alloc_view(spv_sys* s, View& w)
{
    const size_t N = s->N, K = s->kcap;
    ST_TRY(dalloc(s, &w.x, N));
    ST_TRY(dalloc(s, &w.y, N));
    ST_TRY(dalloc(s, &w.th, N));
    ST_TRY(dalloc(s, &w.tag, N));
    ST_TRY(dalloc(s, &w.A0, N));
    ST_TRY(dalloc(s, &w.P0, N));
    ST_TRY(dalloc(s, &w.deg, N));
    ST_TRY(dalloc(s, &w.ring, N * K));
    ST_TRY(dalloc(s, &w.opp, N * K));
    ST_TRY(dalloc(s, &w.A, N));
    ST_TRY(dalloc(s, &w.P, N));
    ST_TRY(dalloc(s, &w.ca, N));
    ST_TRY(dalloc(s, &w.cb, N));
    HIP_TRY(hipMemsetAsync(w.deg, 0, N, s->stream));
    HIP_TRY(hipMemsetAsync(w.ring, 0, N * K * sizeof(int), s->stream));
    HIP_TRY(hipMemsetAsync(w.opp, 0xff, N * K * sizeof(int), s->stream));
    HIP_TRY(hipMemsetAsync(w.ca, 0, N * sizeof(double), s->stream));
    HIP_TRY(hipMemsetAsync(w.cb, 0, N * sizeof(double), s->stream));
    HIP_TRY(hipMemsetAsync(w.A, 0, N * sizeof(double), s->stream));
    HIP_TRY(hipMemsetAsync(w.P, 0, N * sizeof(double), s->stream));
    return SPV_OK;
}

inline unsigned grid_for(int n, int block) { return (unsigned)std::max(1, (n + block - 1) / block); }

// ---------------------------------------------------------------- timing
void begin_timed(spv_sys* s, int which, hipEvent_t* stop)
{
    *stop = nullptr;
    if (!s->timing) return;
    std::pair<hipEvent_t, hipEvent_t> ev;
    if (!s->event_pool.empty()) {
        ev = s->event_pool.back();
        s->event_pool.pop_back();
    } else {
        (void)hipEventCreate(&ev.first);
        (void)hipEventCreate(&ev.second);
    }
    (void)hipEventRecord(ev.first, s->stream);
    s->pending.push_back({which, ev.first, ev.second});
    *stop = ev.second;
}

void end_timed(spv_sys* s, hipEvent_t stop)
{
    if (stop) (void)hipEventRecord(stop, s->stream);
}

void collect_timing(spv_sys* s)
{
    for (auto& t : s->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
            s->t_ms[t.which] += ms;
            s->t_n[t.which] += 1;
        }
        s->event_pool.push_back({t.a, t.b});
    }
    s->pending.clear();
}

// ---------------------------------------------------------------- counters
spv_status read_counters(spv_sys* s)
{
    HIP_TRY(hipMemcpyAsync(s->h_cnt, s->d_cnt, sizeof(DevCounters), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    HIP_TRY(hipGetLastError());
    collect_timing(s);
    return SPV_OK;
}

spv_status check_err(spv_sys* s)
{
    const unsigned e = s->h_cnt->err;
    if (!e) return SPV_OK;
    s->err_word |= e;
    char buf[400];
    const DevCounters& c = *s->h_cnt;
    std::snprintf(buf, sizeof buf,
                  "device error word 0x%x at step %llu (first repair failure: tag %d, %d candidates, ring %d, "
                  "closed %d, %d attempts, R %.4g, max circumradius %.4g)",
                  e, (unsigned long long)s->step, c.fail_set ? c.fail_cell : -1, c.fail_n, c.fail_k, c.fail_closed,
                  c.fail_attempts, c.fail_R, c.fail_umax);
    if (e & ERR_NONFINITE) return fail(SPV_ENONFINITE, std::string(buf) + ": non-finite force or position");
    if (e & ERR_PRECOND)
        return fail(SPV_EPRECOND, std::string(buf) + ": a Delaunay circumradius reached min(Lx,Ly)/4");
    if (e & ERR_CAPACITY) return fail(SPV_ECAPACITY, std::string(buf) + ": ring longer than kcap");
    if (e & ERR_DEGREE) return fail(SPV_EREPAIR, std::string(buf) + ": ring with fewer than 3 cells");
    return fail(SPV_EREPAIR, std::string(buf) + ": ring could not be rebuilt");
}

// ---------------------------------------------------------------- re-sort
// Permute cells into the Hilbert order of their bins; afterwards bin_start
// indexes the cells of every bin (stored contiguously).
spv_status resort(spv_sys* s)
{
    const int N = s->N, nb = s->nbins;
    HIP_TRY(hipMemsetAsync(s->d_hist, 0, nb * sizeof(int), s->stream));
    HIP_TRY(hipMemsetAsync(s->d_fill, 0, nb * sizeof(int), s->stream));
    View v = s->v;
    hipLaunchKernelGGL(k_bin_keys, dim3(grid_for(N, 256)), dim3(256), 0, s->stream, v, s->d_key, s->d_hist);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s->stream, s->d_hist, s->d_bin_start, nb);
    hipLaunchKernelGGL(k_bin_scatter, dim3(grid_for(N, 256)), dim3(256), 0, s->stream, s->d_key, s->d_bin_start,
                       s->d_fill, s->d_perm, N);
    hipLaunchKernelGGL(k_bin_sort, dim3(grid_for(nb, 256)), dim3(256), 0, s->stream, s->d_bin_start, s->d_perm,
                       v.tag, nb);
    hipLaunchKernelGGL(k_inv_perm, dim3(grid_for(N, 256)), dim3(256), 0, s->stream, s->d_perm, s->d_inv, N);
    hipLaunchKernelGGL(k_gather, dim3(grid_for(N, 256)), dim3(256), 0, s->stream, s->v, s->a, s->d_perm,
                       s->d_inv);
    HIP_TRY(hipGetLastError());
    std::swap(s->v.x, s->a.x);
    std::swap(s->v.y, s->a.y);
    std::swap(s->v.th, s->a.th);
    std::swap(s->v.tag, s->a.tag);
    std::swap(s->v.A0, s->a.A0);
    std::swap(s->v.P0, s->a.P0);
    std::swap(s->v.deg, s->a.deg);
    std::swap(s->v.ring, s->a.ring);
    std::swap(s->v.opp, s->a.opp);
    std::swap(s->v.A, s->a.A);
    std::swap(s->v.P, s->a.P);
    std::swap(s->v.ca, s->a.ca);
    std::swap(s->v.cb, s->a.cb);
    s->drift = 0.0;
    s->steps_since_resort = 0;
    s->resorts++;
    return SPV_OK;
}

// ---------------------------------------------------------------- repair rounds
// Loop until the validity test raises no flag: compact the flags into a
// worklist, rebuild those rings, rebuild opp and re-test every cell whose
// neighbourhood changed.  `fail_count` is the number of failing cells of the
// last test (already read back).
spv_status repair_loop(spv_sys* s, int fail_count, double R0)
{
    int rounds = 0;
    const int N = s->N;
    while (fail_count > 0) {
        if (++rounds > s->repair_rounds)
            return fail(SPV_EREPAIR, "topology repair did not converge within repair_rounds");
        View v = s->v;
        hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s->stream, s->d_cnt, 1, 0);
        const unsigned cg = std::min(grid_for(N, 256), 2048u);
        hipLaunchKernelGGL(k_compact, dim3(cg), dim3(256), 0, s->stream, v.flag, N, v.worklist, &s->d_cnt->wl_count);
        const unsigned rg = (unsigned)std::min(std::max(4 * fail_count + 64, 64), std::max(N, 64));
        hipEvent_t stop;
        begin_timed(s, T_REPAIR, &stop);
        hipLaunchKernelGGL(k_repair, dim3(std::min(rg, 65535u)), dim3(64), 0, s->stream, v, R0, s->drift);
        end_timed(s, stop);
        hipLaunchKernelGGL(k_compact, dim3(cg), dim3(256), 0, s->stream, v.touched, N, v.list2,
                           &s->d_cnt->touched_count);
        const unsigned lg = std::min(grid_for(N, 256), 1024u);
        hipLaunchKernelGGL(k_opp<true>, dim3(lg), dim3(256), 0, s->stream, v);
        hipLaunchKernelGGL(k_geom_test<true>, dim3(lg), dim3(256), 0, s->stream, v, s->prm.KA, s->prm.KP);
        HIP_TRY(hipGetLastError());
        ST_TRY(read_counters(s));
        s->rounds++;
        ST_TRY(check_err(s));
        fail_count = s->h_cnt->fail_count;
    }
    return SPV_OK;
}

double default_radius(const spv_sys* s) { return 2.5 * s->spacing; }

spv_status one_step(spv_sys* s)
{
    const int N = s->N;
    const double min_bs = std::min(s->v.bsx, s->v.bsy);
    if (s->steps_since_resort >= s->resort_every || s->drift > 0.5 * min_bs) ST_TRY(resort(s));
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s->stream, s->d_cnt, 0, 0);
    StepParams sp;
    sp.mu = s->prm.mu;
    sp.v0 = s->prm.v0;
    sp.dt = s->prm.dt;
    sp.amp = std::sqrt(2.0 * s->prm.Dr * s->prm.dt);
    sp.KA = s->prm.KA;
    sp.KP = s->prm.KP;
    sp.seed = s->prm.seed;
    sp.step = s->step;
    hipEvent_t stop;
    begin_timed(s, T_FORCE, &stop);
    hipLaunchKernelGGL(k_force<true>, dim3(grid_for(N, 256)), dim3(256), 0, s->stream, s->v, s->a.x, s->a.y, s->a.th,
                       (double*)nullptr, (double*)nullptr, sp);
    end_timed(s, stop);
    std::swap(s->v.x, s->a.x);
    std::swap(s->v.y, s->a.y);
    std::swap(s->v.th, s->a.th);
    begin_timed(s, T_GEOM, &stop);
    hipLaunchKernelGGL(k_geom_test<false>, dim3(grid_for(N, 256)), dim3(256), 0, s->stream, s->v, s->prm.KA,
                       s->prm.KP);
    end_timed(s, stop);
    HIP_TRY(hipGetLastError());
    ST_TRY(read_counters(s));
    s->step++;
    s->steps_since_resort++;
    s->drift += __builtin_bit_cast(double, s->h_cnt->disp_bits);
    ST_TRY(check_err(s));
    return repair_loop(s, s->h_cnt->fail_count, default_radius(s));
}

spv_status copy_out_tag_order(spv_sys* s, const double* dsrc, double* dst)
{
    hipLaunchKernelGGL(k_to_tag_order, dim3(grid_for(s->N, 256)), dim3(256), 0, s->stream, dsrc, s->v.tag,
                       s->d_stage, s->N);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(dst, s->d_stage, s->N * sizeof(double), hipMemcpyDefault, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
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
    for (void* p : s->allocs) (void)hipFree(p);
    if (s->h_cnt) (void)hipHostFree(s->h_cnt);
    for (auto& e : s->event_pool) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    for (auto& t : s->pending) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    delete s;
}

spv_status create_impl(spv_sys* s, int64_t N64, const double* x, const double* y, double Lx, double Ly,
                       const double* A0, const double* P0, double p0, const double* theta0)
{
    const int N = (int)N64;
    s->N = N;
    // grid and box
    s->q = grid_exponent(std::max(Lx, Ly));
    const double scale = std::ldexp(1.0, s->q);
    const double LXu = std::rint(Lx * scale), LYu = std::rint(Ly * scale);
    s->Lx = LXu / scale;
    s->Ly = LYu / scale;
    // host copies of the inputs (host or device pointers)
    std::vector<double> hx, hy, hA0, hP0, hth;
    ST_TRY(copy_in(x, hx, N));
    ST_TRY(copy_in(y, hy, N));
    for (int i = 0; i < N; i++) {
        if (!std::isfinite(hx[i]) || !std::isfinite(hy[i]) || hx[i] < 0.0 || hx[i] >= Lx || hy[i] < 0.0 ||
            hy[i] >= Ly)
            return fail(SPV_EINVAL, "positions must be finite and inside [0,Lx) x [0,Ly)");
        double X = std::rint(hx[i] * scale), Y = std::rint(hy[i] * scale);
        if (X >= LXu) X -= LXu;
        if (Y >= LYu) Y -= LYu;
        hx[i] = X / scale;
        hy[i] = Y / scale;
    }
    {
        std::vector<std::pair<double, double>> pts(N);
        for (int i = 0; i < N; i++) pts[i] = {hx[i], hy[i]};
        std::sort(pts.begin(), pts.end());
        for (int i = 1; i < N; i++)
            if (pts[i] == pts[i - 1]) return fail(SPV_EINVAL, "two cells share a position on the grid");
    }
    if (A0) ST_TRY(copy_in(A0, hA0, N));
    else hA0.assign(N, 1.0);
    if (P0) ST_TRY(copy_in(P0, hP0, N));
    else {
        hP0.resize(N);
        for (int i = 0; i < N; i++) hP0[i] = p0 * std::sqrt(hA0[i]);
    }
    for (int i = 0; i < N; i++)
        if (!std::isfinite(hA0[i]) || !std::isfinite(hP0[i]) || hA0[i] <= 0.0)
            return fail(SPV_EINVAL, "A0 must be positive and finite, P0 finite");
    if (theta0) {
        ST_TRY(copy_in(theta0, hth, N));
        for (int i = 0; i < N; i++)
            if (!std::isfinite(hth[i])) return fail(SPV_EINVAL, "theta0 must be finite");
    }

    // bins of side >= mean spacing, ordered along a Hilbert curve
    s->spacing = std::sqrt(s->Lx * s->Ly / N);
    const int nbx = std::max(1, (int)std::floor(s->Lx / s->spacing));
    const int nby = std::max(1, (int)std::floor(s->Ly / s->spacing));
    s->nbins = nbx * nby;
    std::vector<int> rank(s->nbins);
    {
        int64_t n2 = 1;
        while (n2 < std::max(nbx, nby)) n2 *= 2;
        std::vector<std::pair<int64_t, int>> key(s->nbins);
        for (int by = 0; by < nby; by++)
            for (int bx = 0; bx < nbx; bx++) key[by * nbx + bx] = {hilbert_index(n2, bx, by), by * nbx + bx};
        std::sort(key.begin(), key.end());
        for (int r = 0; r < s->nbins; r++) rank[key[r].second] = r;
    }

    // device state
    ST_TRY(alloc_view(s, s->v));
    ST_TRY(alloc_view(s, s->a));
    ST_TRY(dalloc(s, &s->v.flag, N));
    ST_TRY(dalloc(s, &s->v.touched, N));
    ST_TRY(dalloc(s, &s->v.worklist, N));
    ST_TRY(dalloc(s, &s->v.list2, N));
    ST_TRY(dalloc(s, &s->d_cnt, 1));
    ST_TRY(dalloc(s, &s->d_bin_rank, s->nbins));
    ST_TRY(dalloc(s, &s->d_bin_start, s->nbins + 1));
    ST_TRY(dalloc(s, &s->d_key, N));
    ST_TRY(dalloc(s, &s->d_hist, s->nbins));
    ST_TRY(dalloc(s, &s->d_fill, s->nbins));
    ST_TRY(dalloc(s, &s->d_perm, N));
    ST_TRY(dalloc(s, &s->d_inv, N));
    ST_TRY(dalloc(s, &s->d_stage, N));
    ST_TRY(dalloc(s, &s->d_fx, N));
    ST_TRY(dalloc(s, &s->d_fy, N));
    ST_TRY(dalloc(s, &s->d_part, 3 * 1024));
    ST_TRY(dalloc(s, &s->d_obs, 3));
    HIP_TRY(hipHostMalloc((void**)&s->h_cnt, sizeof(DevCounters), hipHostMallocDefault));
    HIP_TRY(hipMemsetAsync(s->d_cnt, 0, sizeof(DevCounters), s->stream));
    HIP_TRY(hipMemsetAsync(s->v.flag, 0, N, s->stream));
    HIP_TRY(hipMemsetAsync(s->v.touched, 0, N, s->stream));
    for (View* w : {&s->v, &s->a}) {
        View& vv = *w;
        vv.N = N;
        vv.kcap = s->kcap;
        vv.Lx = s->Lx;
        vv.Ly = s->Ly;
        vv.hLx = 0.5 * s->Lx;
        vv.hLy = 0.5 * s->Ly;
        vv.scale = scale;
        vv.inv_scale = 1.0 / scale;
        vv.LXu = LXu;
        vv.LYu = LYu;
        vv.flag = s->v.flag;
        vv.touched = s->v.touched;
        vv.worklist = s->v.worklist;
        vv.list2 = s->v.list2;
        vv.cnt = s->d_cnt;
        vv.nbx = nbx;
        vv.nby = nby;
        vv.bsx = s->Lx / nbx;
        vv.bsy = s->Ly / nby;
        vv.bin_rank = s->d_bin_rank;
        vv.bin_start = s->d_bin_start;
    }
    HIP_TRY(hipMemcpyAsync(s->v.x, hx.data(), N * sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(s->v.y, hy.data(), N * sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(s->v.A0, hA0.data(), N * sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(s->v.P0, hP0.data(), N * sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(s->d_bin_rank, rank.data(), s->nbins * sizeof(int), hipMemcpyHostToDevice, s->stream));
    hipLaunchKernelGGL(k_iota, dim3(grid_for(N, 256)), dim3(256), 0, s->stream, s->v.tag, N);
    if (theta0)
        HIP_TRY(hipMemcpyAsync(s->v.th, hth.data(), N * sizeof(double), hipMemcpyHostToDevice, s->stream));
    else
        hipLaunchKernelGGL(k_theta0, dim3(grid_for(N, 256)), dim3(256), 0, s->stream, s->v.th, s->v.tag, N,
                           (uint64_t)s->prm.seed);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s->stream));  // host vectors die at return

    // spatial order, then the triangulation from scratch: every cell repaired
    ST_TRY(resort(s));
    View v = s->v;
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s->stream, s->d_cnt, 2, N);
    hipLaunchKernelGGL(k_iota, dim3(grid_for(N, 256)), dim3(256), 0, s->stream, v.worklist, N);
    hipLaunchKernelGGL(k_repair, dim3(std::min(N, 65535)), dim3(64), 0, s->stream, v, default_radius(s), 0.0);
    hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(N, 256)), dim3(256), 0, s->stream, v.touched, N, (uint8_t)0);
    hipLaunchKernelGGL(k_opp<false>, dim3(grid_for(N, 256)), dim3(256), 0, s->stream, v);
    hipLaunchKernelGGL(k_geom_test<false>, dim3(grid_for(N, 256)), dim3(256), 0, s->stream, v, s->prm.KA,
                       s->prm.KP);
    HIP_TRY(hipGetLastError());
    ST_TRY(read_counters(s));
    ST_TRY(check_err(s));
    ST_TRY(repair_loop(s, s->h_cnt->fail_count, default_radius(s)));
    return SPV_OK;
}

}  // namespace

// ====================================================================== C-ABI
extern "C" {

const char* spv_last_error(void) { return g_err.c_str(); }

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
    const spv_params& p = *params;
    if (p.precision != SPV_FP64) return fail(SPV_EINVAL, "precision must be SPV_FP64");
    if (!(p.dt > 0.0) || !(p.Dr >= 0.0) || !std::isfinite(p.mu) || !std::isfinite(p.v0) || !std::isfinite(p.KA) ||
        !std::isfinite(p.KP))
        return fail(SPV_EINVAL, "invalid model parameters");
    if (!A0 && !P0 && !std::isfinite(p0)) return fail(SPV_EINVAL, "p0 must be finite");
    spv_sys* s = new spv_sys();
    s->prm = p;
    s->kcap = p.kcap > 0 ? p.kcap : 16;
    if (s->kcap < 3 || s->kcap > RP_KMAX) {
        delete s;
        return fail(SPV_EINVAL, "kcap must be in [3, 64]");
    }
    s->repair_rounds = p.repair_rounds > 0 ? p.repair_rounds : 16;
    s->resort_every = p.resort_every > 0 ? p.resort_every : 64;
    s->stream = (hipStream_t)stream;
    spv_status st = create_impl(s, N, x, y, Lx, Ly, A0, P0, p0, theta0);
    if (st != SPV_OK) {
        std::string keep = g_err;
        destroy_all(s);
        g_err = keep;
        return st;
    }
    *out = s;
    return SPV_OK;
}

spv_status spv_step(spv_sys* s, int64_t nsteps)
{
    if (!s || nsteps < 0) return fail(SPV_EINVAL, "bad handle or nsteps");
    for (int64_t k = 0; k < nsteps; k++) ST_TRY(one_step(s));
    return SPV_OK;
}

spv_status spv_get_box(spv_sys* s, double* Lx, double* Ly, int32_t* q)
{
    if (!s) return fail(SPV_EINVAL, "bad handle");
    if (Lx) *Lx = s->Lx;
    if (Ly) *Ly = s->Ly;
    if (q) *q = s->q;
    return SPV_OK;
}

spv_status spv_get_positions(spv_sys* s, double* x, double* y)
{
    if (!s || !x || !y) return fail(SPV_EINVAL, "bad argument");
    ST_TRY(copy_out_tag_order(s, s->v.x, x));
    return copy_out_tag_order(s, s->v.y, y);
}

spv_status spv_get_directors(spv_sys* s, double* theta)
{
    if (!s || !theta) return fail(SPV_EINVAL, "bad argument");
    return copy_out_tag_order(s, s->v.th, theta);
}

spv_status spv_get_forces(spv_sys* s, double* fx, double* fy)
{
    if (!s || !fx || !fy) return fail(SPV_EINVAL, "bad argument");
    StepParams sp{};
    hipLaunchKernelGGL(k_force<false>, dim3(grid_for(s->N, 256)), dim3(256), 0, s->stream, s->v, (double*)nullptr,
                       (double*)nullptr, (double*)nullptr, s->d_fx, s->d_fy, sp);
    HIP_TRY(hipGetLastError());
    ST_TRY(copy_out_tag_order(s, s->d_fx, fx));
    return copy_out_tag_order(s, s->d_fy, fy);
}

spv_status spv_get_geometry(spv_sys* s, double* A, double* P)
{
    if (!s || !A || !P) return fail(SPV_EINVAL, "bad argument");
    ST_TRY(copy_out_tag_order(s, s->v.A, A));
    return copy_out_tag_order(s, s->v.P, P);
}

spv_status spv_get_neighbors(spv_sys* s, int32_t* offsets, int32_t* nbr, int64_t cap, int64_t* needed)
{
    if (!s || !offsets) return fail(SPV_EINVAL, "bad argument");
    const int N = s->N, K = s->kcap;
    std::vector<uint8_t> deg(N);
    std::vector<int> ring((size_t)N * K), tag(N);
    HIP_TRY(hipMemcpyAsync(deg.data(), s->v.deg, N, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(ring.data(), s->v.ring, (size_t)N * K * sizeof(int), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(tag.data(), s->v.tag, N * sizeof(int), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    std::vector<int> slot_of_tag(N);
    for (int i = 0; i < N; i++) slot_of_tag[tag[i]] = i;
    int64_t tot = 0;
    for (int t = 0; t < N; t++) {
        offsets[t] = (int32_t)tot;
        tot += deg[slot_of_tag[t]];
    }
    offsets[N] = (int32_t)tot;
    if (needed) *needed = tot;
    if (!nbr || cap < tot) return fail(SPV_ECAPACITY, "nbr buffer too small");
    for (int t = 0; t < N; t++) {
        const int i = slot_of_tag[t];
        for (int m = 0; m < deg[i]; m++) nbr[offsets[t] + m] = tag[ring[(size_t)m * N + i]];
    }
    return SPV_OK;
}

spv_status spv_get_observables(spv_sys* s, double* E, double* qbar, double* sumA, int64_t* counters)
{
    if (!s) return fail(SPV_EINVAL, "bad handle");
    const int nb = 1024;
    hipLaunchKernelGGL(k_obs_partial, dim3(nb), dim3(256), 0, s->stream, s->v, s->prm.KA, s->prm.KP, s->d_part);
    hipLaunchKernelGGL(k_obs_final, dim3(1), dim3(256), 0, s->stream, s->d_part, nb, s->d_obs);
    HIP_TRY(hipGetLastError());
    double h[3];
    HIP_TRY(hipMemcpyAsync(h, s->d_obs, sizeof h, hipMemcpyDeviceToHost, s->stream));
    ST_TRY(read_counters(s));
    if (E) *E = h[0];
    if (qbar) *qbar = h[1] / s->N;
    if (sumA) *sumA = h[2];
    if (counters) {
        const DevCounters& c = *s->h_cnt;
        counters[0] = (int64_t)s->step;
        counters[1] = c.repaired;
        counters[2] = s->rounds;
        counters[3] = c.exact_calls;
        counters[4] = c.max_deg;
        counters[5] = s->resorts;
        counters[6] = c.retries;
        counters[7] = (int64_t)(c.err | s->err_word);
    }
    return SPV_OK;
}

spv_status spv_set_timing(spv_sys* s, int32_t enable)
{
    if (!s) return fail(SPV_EINVAL, "bad handle");
    HIP_TRY(hipStreamSynchronize(s->stream));
    collect_timing(s);
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
    collect_timing(s);
    if (total_ms) *total_ms = s->t_ms[which];
    if (launches) *launches = s->t_n[which];
    return SPV_OK;
}

spv_status spv_destroy(spv_sys* s)
{
    if (!s) return fail(SPV_EINVAL, "bad handle");
    destroy_all(s);
    return SPV_OK;
}

}  // extern "C"
