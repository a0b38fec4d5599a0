// avm_api.hpp -- host runtime of the active vertex model (included by
// spv_api.hip after the Voronoi model's runtime; shares its error handling,
// scan and observables kernels and the Hilbert ranking).
//
// A handle owns the vertex positions (two buffers: the move writes the
// other), the flat topology (vv, vc, cv), the cell directors, targets and
// geometry, the creation labels of vertices and cells, the T1 locks and a
// control block.  A step is geometry, force + move, one to three T1 rounds
// of two passes each (the first marking pass visits every vertex and also
// rotates the directors; later passes only the vertices the round before
// flagged), and a last marking pass that halts the later kernels of the
// batch when one more round is needed; the host then runs more rounds (one
// read-back each) until none qualifies.  The number of device rounds follows
// the rounds the last batch needed per step: one while flips seldom
// conflict (five launches a step), up to three when they often do.  Batches of eight steps are
// captured once as HIP graphs and replayed.  A spatial re-sort (vertices
// and cells along a Hilbert curve of bins) runs at creation and every
// resort_every steps; results do not depend on it.

namespace {

constexpr int AVM_BATCH = 8;             // steps between read-backs (one graph)
constexpr int AVM_DEFAULT_RESORT = 1000; // steps between re-sorts when resort_every is 0

struct AvmDev {
    double *x[2] = {nullptr, nullptr}, *y[2] = {nullptr, nullptr};
    // slot-indexed arrays in two sets: a re-sort gathers from one into the other
    int *vv[2] = {nullptr, nullptr}, *vc[2] = {nullptr, nullptr}, *cv[2] = {nullptr, nullptr};
    int *vtag[2] = {nullptr, nullptr}, *ctag[2] = {nullptr, nullptr};
    uint8_t* cdeg[2] = {nullptr, nullptr};
    double *th[2] = {nullptr, nullptr}, *A0[2] = {nullptr, nullptr}, *P0[2] = {nullptr, nullptr};
    uint8_t *cand = nullptr, *dirty = nullptr;  // padded to a multiple of 8 vertices
    int* lcell = nullptr;
    double *A = nullptr, *P = nullptr, *ca = nullptr, *cb = nullptr;
    double *fx = nullptr, *fy = nullptr;
    double* out = nullptr;  // label-order staging of one read-out (Nv)
    long long* lock[2] = {nullptr, nullptr};
    // re-sort scratch
    int *vkey = nullptr, *ckey = nullptr, *vcount = nullptr, *ccount = nullptr;
    int *vstart = nullptr, *cstart = nullptr, *vchunk = nullptr, *cchunk = nullptr;
    int *vperm = nullptr, *cperm = nullptr, *vinv = nullptr, *cinv = nullptr, *rank = nullptr;
};

}  // namespace

struct spv_avm {
    int nc = 0, nv = 0, cur = 0, set = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;  // private stream used only to capture graphs
    AvmDev d;
    AvmParam hp{};
    AvmBins bins{};
    AvmParam* d_p = nullptr;
    AvmState* d_st = nullptr;
    AvmState* h_st = nullptr;
    DevState* d_scan = nullptr;        // control block of the shared scan kernels (never halted)
    SysParam* d_sp = nullptr;          // for the shared observables kernels
    double *d_obs = nullptr, *d_obs_part = nullptr;
    int obs_chunks = 1;
    int resort_every = AVM_DEFAULT_RESORT;  // -1: never
    int64_t since_sort = 0;
    int dev_rounds = AVM_DEV_ROUNDS;  // T1 rounds of a step on the device (1 .. AVM_DEV_ROUNDS)
    std::map<std::array<int, 3>, hipGraphExec_t> graphs;  // (position buffer, array set, rounds) -> batch graph
    std::vector<void*> allocs;
    int64_t host_rounds = 0, graph_batches = 0, resorts = 0;
    spv_status sticky = SPV_OK;
    std::string sticky_msg;
};

namespace {

template <class T>
spv_status avm_alloc(spv_avm* h, T** p, size_t n)
{
    void* q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return fail(SPV_ENOMEM, "hipMalloc failed");
    h->allocs.push_back(q);
    *p = static_cast<T*>(q);
    return SPV_OK;
}

void avm_free(spv_avm* h)
{
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (auto& g : h->graphs) (void)hipGraphExecDestroy(g.second);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    for (void* p : h->allocs) (void)hipFree(p);
    if (h->h_st) (void)hipHostFree(h->h_st);
    delete h;
}

// the kernels' view: positions of buffer b (and the other as the move's
// output), slot arrays of set s
AvmArrays avm_arrays(const spv_avm* h, int b, int s)
{
    AvmArrays a;
    a.x = h->d.x[b];
    a.y = h->d.y[b];
    a.xo = h->d.x[b ^ 1];
    a.yo = h->d.y[b ^ 1];
    a.vv = h->d.vv[s];
    a.vc = h->d.vc[s];
    a.cv = h->d.cv[s];
    a.cdeg = h->d.cdeg[s];
    a.th = h->d.th[s];
    a.A0 = h->d.A0[s];
    a.P0 = h->d.P0[s];
    a.vtag = h->d.vtag[s];
    a.ctag = h->d.ctag[s];
    a.A = h->d.A;
    a.P = h->d.P;
    a.ca = h->d.ca;
    a.cb = h->d.cb;
    a.fx = h->d.fx;
    a.fy = h->d.fy;
    a.lock[0] = h->d.lock[0];
    a.lock[1] = h->d.lock[1];
    a.cand = h->d.cand;
    a.dirty = h->d.dirty;
    a.lcell = h->d.lcell;
    a.nv = h->nv;
    a.nc = h->nc;
    return a;
}

AvmArrays avm_arrays(const spv_avm* h, int b) { return avm_arrays(h, b, h->set); }

unsigned avm_grid(int n) { return grid_for(n, 256); }
unsigned avm_grid8(int n) { return grid_for((n + 7) / 8, 256); }  // eight vertices per thread

spv_status avm_read(spv_avm* h)
{
    HIP_TRY(hipMemcpyAsync(h->h_st, h->d_st, sizeof(AvmState), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return SPV_OK;
}

spv_status avm_error(spv_avm* h)
{
    const unsigned e = h->h_st->err;
    h->sticky = (e & ERR_NONFINITE) ? SPV_ENONFINITE : (e & ERR_CAPACITY) ? SPV_ECAPACITY : SPV_EREPAIR;
    h->sticky_msg = (e & ERR_NONFINITE)   ? "non-finite vertex position"
                    : (e & ERR_CAPACITY) ? "a T1 would give a cell more than 16 vertices"
                                         : "inconsistent vertex topology";
    return fail(h->sticky, h->sticky_msg);
}

// one step from position buffer b on stream s (h->dev_rounds rounds)
void enqueue_avm_step(spv_avm* h, hipStream_t s, int b)
{
    const int nr = h->dev_rounds;
    const unsigned gv = avm_grid(h->nv), gc = avm_grid(h->nc), g8 = avm_grid8(h->nv);
    const AvmArrays a = avm_arrays(h, b), n = avm_arrays(h, b ^ 1);
    const AvmParam* p = h->d_p;
    hipLaunchKernelGGL(k_avm_geom, dim3(gc), dim3(256), 0, s, a, p, h->d_st);
    hipLaunchKernelGGL(k_avm_force<true>, dim3(gv), dim3(256), 0, s, a, p, h->d_st);
    for (int r = 0; r < nr; r++) {
        hipLaunchKernelGGL(k_avm_t1_mark, dim3(r == 0 ? gv : g8), dim3(256), 0, s, n, p, h->d_st, r, 0, 0);
        hipLaunchKernelGGL(k_avm_t1_apply, dim3(g8), dim3(256), 0, s, n, p, h->d_st, r, 0);
    }
    hipLaunchKernelGGL(k_avm_t1_mark, dim3(g8), dim3(256), 0, s, n, p, h->d_st, nr, 0, 1);
}

// The graph of a batch of AVM_BATCH steps from position buffer b with the
// current array set and round count, captured on first use.
spv_status avm_batch_graph(spv_avm* h, int b, hipGraphExec_t* out)
{
    const std::array<int, 3> key{b, h->set, h->dev_rounds};
    auto it = h->graphs.find(key);
    if (it != h->graphs.end()) {
        *out = it->second;
        return SPV_OK;
    }
    if (!h->cap_stream) HIP_TRY(hipStreamCreate(&h->cap_stream));
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeRelaxed));
    for (int j = 0; j < AVM_BATCH; j++) enqueue_avm_step(h, h->cap_stream, b ^ (j & 1));
    hipError_t e0 = hipGetLastError();
    hipError_t e1 = hipStreamEndCapture(h->cap_stream, &graph);
    if (e1 == hipSuccess && e0 != hipSuccess) e1 = e0;
    if (e1 != hipSuccess) return fail(SPV_EHIP, std::string("graph capture: ") + hipGetErrorString(e1));
    hipGraphExec_t ex = nullptr;
    hipError_t e2 = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) return fail(SPV_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e2));
    h->graphs[key] = ex;
    *out = ex;
    return SPV_OK;
}

// more T1 rounds for the halted step (its positions are current; the
// marking pass after its `first` device rounds found edges), one read-back
// each, until one finds none
spv_status avm_finish_rounds(spv_avm* h, int first)
{
    const unsigned g8 = avm_grid8(h->nv);
    const AvmArrays a = avm_arrays(h, h->cur);
    for (int r = first;; r++) {
        if (r + 1 > AVM_MAX_ROUNDS) {
            h->sticky = SPV_EREPAIR;
            h->sticky_msg = "T1 transitions did not settle within 64 rounds";
            return fail(SPV_EREPAIR, h->sticky_msg);
        }
        hipLaunchKernelGGL(k_avm_t1_apply, dim3(g8), dim3(256), 0, h->stream, a, (const AvmParam*)h->d_p, h->d_st,
                           r, 1);
        hipLaunchKernelGGL(k_avm_t1_mark, dim3(g8), dim3(256), 0, h->stream, a, (const AvmParam*)h->d_p, h->d_st,
                           r + 1, 1, 0);
        HIP_TRY(hipGetLastError());
        ST_TRY(avm_read(h));
        h->host_rounds++;
        if (h->h_st->err) return avm_error(h);
        if (!h->h_st->any[r + 1]) break;
    }
    // both lock sets are clean again: the last marking pass found nothing
    // and cleared the other set
    hipLaunchKernelGGL(k_avm_resume, dim3(1), dim3(64), 0, h->stream, h->d_st);
    HIP_TRY(hipGetLastError());
    return SPV_OK;
}

// Re-sort between steps: the positions move to the other buffer, the slot
// arrays to the other set (the locks are all clear between steps and the
// geometry, force and candidate arrays are rebuilt before they are read).
spv_status avm_resort(spv_avm* h)
{
    hipStream_t s = h->stream;
    const int nv = h->nv, nc = h->nc, nb = h->bins.nb;
    const unsigned nchunk = grid_for(nb, SCAN_CHUNK);
    const AvmArrays src = avm_arrays(h, h->cur, h->set);
    AvmArrays dst = avm_arrays(h, h->cur ^ 1, h->set ^ 1);
    AvmDev& d = h->d;
    hipLaunchKernelGGL(k_avm_keys, dim3(avm_grid(nv)), dim3(256), 0, s, src, h->bins, d.vkey, d.vcount, d.ckey,
                       d.ccount);
    hipLaunchKernelGGL(k_scan_sums_last, dim3(nchunk), dim3(256), 0, s, (const int*)d.vcount, nb, d.vchunk, h->d_scan);
    hipLaunchKernelGGL(k_scan_apply<true>, dim3(nchunk), dim3(256), 0, s, d.vcount, d.vstart, nb,
                       (const int*)d.vchunk, (const DevState*)h->d_scan);
    hipLaunchKernelGGL(k_scan_sums_last, dim3(nchunk), dim3(256), 0, s, (const int*)d.ccount, nb, d.cchunk, h->d_scan);
    hipLaunchKernelGGL(k_scan_apply<true>, dim3(nchunk), dim3(256), 0, s, d.ccount, d.cstart, nb,
                       (const int*)d.cchunk, (const DevState*)h->d_scan);
    hipLaunchKernelGGL(k_avm_scatter, dim3(avm_grid(nv)), dim3(256), 0, s, (const int*)d.vkey, (const int*)d.vstart,
                       d.vcount, d.vperm, (const int*)d.ckey, (const int*)d.cstart, d.ccount, d.cperm, nv, nc);
    hipLaunchKernelGGL(k_avm_bin_order, dim3(avm_grid(nb)), dim3(256), 0, s, (const int*)d.vstart, d.vcount, d.vperm,
                       d.vinv, (const int*)src.vtag, nb);
    hipLaunchKernelGGL(k_avm_bin_order, dim3(avm_grid(nb)), dim3(256), 0, s, (const int*)d.cstart, d.ccount, d.cperm,
                       d.cinv, (const int*)src.ctag, nb);
    dst.x = d.x[h->cur ^ 1];
    dst.y = d.y[h->cur ^ 1];
    hipLaunchKernelGGL(k_avm_gather, dim3(avm_grid(nv)), dim3(256), 0, s, src, dst, (const int*)d.vperm,
                       (const int*)d.vinv, (const int*)d.cperm, (const int*)d.cinv);
    HIP_TRY(hipGetLastError());
    h->cur ^= 1;
    h->set ^= 1;
    h->since_sort = 0;
    h->resorts++;
    return SPV_OK;
}

spv_status avm_steps(spv_avm* h, int64_t n)
{
    if (h->sticky != SPV_OK) return fail(h->sticky, h->sticky_msg);
    while (n > 0) {
        if (h->resort_every > 0 && h->since_sort >= h->resort_every) ST_TRY(avm_resort(h));
        int64_t b = std::min<int64_t>(n, AVM_BATCH);
        if (h->resort_every > 0) b = std::min<int64_t>(b, h->resort_every - h->since_sort);
        const unsigned long long before = h->h_st->step, rounds0 = h->h_st->rounds;
        const int cur0 = h->cur, nr = h->dev_rounds;
        if (b == AVM_BATCH) {
            hipGraphExec_t ex = nullptr;
            ST_TRY(avm_batch_graph(h, cur0, &ex));
            HIP_TRY(hipGraphLaunch(ex, h->stream));
            h->graph_batches++;
        } else {
            for (int64_t j = 0; j < b; j++) enqueue_avm_step(h, h->stream, cur0 ^ (int)(j & 1));
        }
        HIP_TRY(hipGetLastError());
        ST_TRY(avm_read(h));
        if (h->h_st->err) return avm_error(h);
        const int64_t done = (int64_t)(h->h_st->step - before);
        // steps after a halted one did nothing: the current buffer is the
        // one the last completed step wrote
        h->cur = (int)((cur0 + done) & 1);
        n -= done;
        h->since_sort += done;
        const bool halted = h->h_st->halt != 0;
        if (halted) ST_TRY(avm_finish_rounds(h, nr));
        // rounds with flips per step over this batch (a halted step's host
        // rounds included; the control block was just read) -> the next
        // batch's device rounds
        if (done > 0) {
            const double rate = (double)(h->h_st->rounds - rounds0) / (double)done;
            h->dev_rounds = rate <= 1.15 ? 1 : (rate <= 1.6 ? 2 : AVM_DEV_ROUNDS);
        }
    }
    return SPV_OK;
}

// Check a trivalent periodic polygon network and derive each vertex's
// neighbours and cells in counter-clockwise order: in cell c (vertices
// counter-clockwise) vertex v with successor s and predecessor p contributes
// the sector from s to p, so around v the triples (s, c, p) chain with
// p_k = s_{k+1}.
spv_status avm_topology(int nc, int nv, const std::vector<int32_t>& off, const std::vector<int32_t>& cv,
                        std::vector<int>& vv, std::vector<int>& vc, std::vector<int>& cvf, std::vector<uint8_t>& deg)
{
    if (off.size() != (size_t)nc + 1 || off[0] != 0) return fail(SPV_EINVAL, "cell_off must start at 0");
    std::vector<int> cnt(nv, 0);
    std::vector<std::array<int, 9>> tri(nv);  // (s, c, p) x 3 per vertex
    cvf.assign((size_t)nc * AVM_KV, -1);
    deg.assign(nc, 0);
    for (int c = 0; c < nc; c++) {
        const int k = off[c + 1] - off[c];
        if (k < 3 || k > AVM_KV) return fail(SPV_EINVAL, "every cell needs 3 to 16 vertices");
        deg[c] = (uint8_t)k;
        for (int m = 0; m < k; m++) {
            const int v = cv[off[c] + m], s = cv[off[c] + (m + 1) % k], p = cv[off[c] + (m + k - 1) % k];
            if (v < 0 || v >= nv) return fail(SPV_EINVAL, "vertex index out of range");
            if (cnt[v] >= 3) return fail(SPV_EINVAL, "a vertex in more than three cells (the network must be trivalent)");
            tri[v][3 * cnt[v]] = s;
            tri[v][3 * cnt[v] + 1] = c;
            tri[v][3 * cnt[v] + 2] = p;
            cnt[v]++;
            cvf[(size_t)c * AVM_KV + m] = v;
        }
    }
    vv.assign((size_t)3 * nv, -1);
    vc.assign((size_t)3 * nv, -1);
    for (int v = 0; v < nv; v++) {
        if (cnt[v] != 3) return fail(SPV_EINVAL, "every vertex must be in exactly three cells");
        int k0 = 0;
        for (int k = 0; k < 3; k++) {
            vv[3 * v + k] = tri[v][3 * k0];
            vc[3 * v + k] = tri[v][3 * k0 + 1];
            const int p = tri[v][3 * k0 + 2];
            int next = -1;
            for (int j = 0; j < 3; j++)
                if (tri[v][3 * j] == p) next = j;
            if (next < 0) return fail(SPV_EINVAL, "cells around a vertex are not consistently counter-clockwise");
            k0 = next;
        }
        if (k0 != 0) return fail(SPV_EINVAL, "cells around a vertex are not consistently counter-clockwise");
    }
    return SPV_OK;
}

// bins of about one cell each, ranked along a Hilbert curve (order 0) or
// row by row (order 1)
std::vector<int> avm_bin_ranks(AvmBins& b, double Lx, double Ly, int nc, int order)
{
    const double side = std::sqrt(Lx * Ly / nc);
    b.nbx = std::max(1, (int)std::floor(Lx / side));
    b.nby = std::max(1, (int)std::floor(Ly / side));
    b.nb = b.nbx * b.nby;
    b.bsx = Lx / b.nbx;
    b.bsy = Ly / b.nby;
    int64_t n2 = 1;
    while (n2 < std::max(b.nbx, b.nby)) n2 *= 2;
    std::vector<std::pair<int64_t, int>> key(b.nb);
    for (int by = 0; by < b.nby; by++)
        for (int bx = 0; bx < b.nbx; bx++)
            key[by * b.nbx + bx] = {order == 1 ? (int64_t)(by * b.nbx + bx) : hilbert_index(n2, bx, by),
                                    by * b.nbx + bx};
    std::sort(key.begin(), key.end());
    std::vector<int> rank(b.nb);
    for (int r = 0; r < b.nb; r++) rank[key[r].second] = r;
    return rank;
}

}  // namespace
