// avm_api.hpp -- host runtime of the active vertex model (included by
// spv_api.hip after the Voronoi model's runtime; shares its error handling
// and observables kernels).
//
// A handle owns the vertex positions (two buffers: the move writes the
// other), the flat topology (vv, vc, cv), the cell directors, targets and
// geometry, the T1 locks and a control block.  A step is seven launches:
// geometry, force + move, director rotation, two T1 rounds of two passes
// each; a step whose
// second round still flipped halts the later kernels of its batch and the
// host runs more rounds (one read-back each) until none qualifies.

namespace {

struct AvmDev {
    double *x[2] = {nullptr, nullptr}, *y[2] = {nullptr, nullptr};
    int *vv = nullptr, *vc = nullptr, *cv = nullptr;
    uint8_t *cdeg = nullptr, *cand = nullptr;
    double *th = nullptr, *A0 = nullptr, *P0 = nullptr, *A = nullptr, *P = nullptr, *ca = nullptr, *cb = nullptr;
    double *fx = nullptr, *fy = nullptr;
    long long* lock[2] = {nullptr, nullptr};
};

}  // namespace

struct spv_avm {
    int nc = 0, nv = 0, cur = 0;
    hipStream_t stream = nullptr;
    AvmDev d;
    AvmParam hp{};
    AvmParam* d_p = nullptr;
    AvmState* d_st = nullptr;
    AvmState* h_st = nullptr;
    SysParam* d_sp = nullptr;  // for the shared observables kernels
    double *d_obs = nullptr, *d_obs_part = nullptr;
    int obs_chunks = 1;
    std::vector<void*> allocs;
    int64_t host_rounds = 0;
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
    for (void* p : h->allocs) (void)hipFree(p);
    if (h->h_st) (void)hipHostFree(h->h_st);
    delete h;
}

// the kernels' view; positions of buffer b (and the other as the move's output)
AvmArrays avm_arrays(const spv_avm* h, int b)
{
    AvmArrays a;
    a.x = h->d.x[b];
    a.y = h->d.y[b];
    a.xo = h->d.x[b ^ 1];
    a.yo = h->d.y[b ^ 1];
    a.vv = h->d.vv;
    a.vc = h->d.vc;
    a.cv = h->d.cv;
    a.cdeg = h->d.cdeg;
    a.th = h->d.th;
    a.A0 = h->d.A0;
    a.P0 = h->d.P0;
    a.A = h->d.A;
    a.P = h->d.P;
    a.ca = h->d.ca;
    a.cb = h->d.cb;
    a.fx = h->d.fx;
    a.fy = h->d.fy;
    a.lock[0] = h->d.lock[0];
    a.lock[1] = h->d.lock[1];
    a.cand = h->d.cand;
    a.nv = h->nv;
    a.nc = h->nc;
    return a;
}

unsigned avm_grid(int n) { return grid_for(n, 256); }

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

void enqueue_avm_step(spv_avm* h)
{
    const unsigned gv = avm_grid(h->nv), gc = avm_grid(h->nc), gt = avm_grid(std::max(h->nv, h->nc));
    const AvmArrays a = avm_arrays(h, h->cur), b = avm_arrays(h, h->cur ^ 1);
    hipLaunchKernelGGL(k_avm_geom, dim3(gc), dim3(256), 0, h->stream, a, (const AvmParam*)h->d_p, h->d_st);
    hipLaunchKernelGGL(k_avm_force<true>, dim3(gv), dim3(256), 0, h->stream, a, (const AvmParam*)h->d_p, h->d_st);
    hipLaunchKernelGGL(k_avm_theta, dim3(gc), dim3(256), 0, h->stream, a, (const AvmParam*)h->d_p, h->d_st);
    for (int r = 0; r < AVM_DEV_ROUNDS; r++) {
        hipLaunchKernelGGL(k_avm_t1_mark, dim3(gv), dim3(256), 0, h->stream, b, (const AvmParam*)h->d_p, h->d_st, r);
        hipLaunchKernelGGL(k_avm_t1_apply, dim3(gt), dim3(256), 0, h->stream, b, (const AvmParam*)h->d_p, h->d_st,
                           r, r == AVM_DEV_ROUNDS - 1 ? 1 : 0);
    }
    h->cur ^= 1;
}

// more T1 rounds for the halted step (its positions are current), one
// read-back each, until one finds no qualifying edge
spv_status avm_finish_rounds(spv_avm* h)
{
    const unsigned gv = avm_grid(h->nv), gt = avm_grid(std::max(h->nv, h->nc));
    const AvmArrays a = avm_arrays(h, h->cur);
    for (int r = AVM_DEV_ROUNDS;; r++) {
        if (r >= AVM_MAX_ROUNDS) {
            h->sticky = SPV_EREPAIR;
            h->sticky_msg = "T1 transitions did not settle within 64 rounds";
            return fail(SPV_EREPAIR, h->sticky_msg);
        }
        hipLaunchKernelGGL(k_avm_t1_mark, dim3(gv), dim3(256), 0, h->stream, a, (const AvmParam*)h->d_p, h->d_st, r);
        hipLaunchKernelGGL(k_avm_t1_apply, dim3(gt), dim3(256), 0, h->stream, a, (const AvmParam*)h->d_p, h->d_st, r,
                           0);
        HIP_TRY(hipGetLastError());
        ST_TRY(avm_read(h));
        h->host_rounds++;
        if (h->h_st->err) return avm_error(h);
        if (!h->h_st->any[r]) break;
    }
    // both lock sets are clean again: the last round marked nothing, and its
    // apply cleared the other set
    hipLaunchKernelGGL(k_avm_resume, dim3(1), dim3(64), 0, h->stream, h->d_st);
    HIP_TRY(hipGetLastError());
    return SPV_OK;
}

spv_status avm_steps(spv_avm* h, int64_t n)
{
    if (h->sticky != SPV_OK) return fail(h->sticky, h->sticky_msg);
    while (n > 0) {
        const int64_t b = std::min<int64_t>(n, 8);
        const unsigned long long before = h->h_st->step;
        const int cur0 = h->cur;
        for (int64_t j = 0; j < b; j++) enqueue_avm_step(h);
        HIP_TRY(hipGetLastError());
        ST_TRY(avm_read(h));
        if (h->h_st->err) return avm_error(h);
        const int64_t done = (int64_t)(h->h_st->step - before);
        // steps after a halted one did nothing: the current buffer is the
        // one the last completed step wrote
        h->cur = (int)((cur0 + done) & 1);
        n -= done;
        if (h->h_st->halt) ST_TRY(avm_finish_rounds(h));
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

}  // namespace
