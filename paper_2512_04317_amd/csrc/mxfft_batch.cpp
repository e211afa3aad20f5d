// mxfft_batch.cpp -- uneven batches: a work list of slice groups of different
// sizes anywhere in one pool, transformed by one HIP graph launch.  Groups of
// the same size share one branch (one plan, one stream, one launch sequence
// over all their slices, addressed through a per-slice offset table); the
// branches of different sizes run side by side.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>
#include <vector>

#include "mxfft.h"
#include "mxfft_internal.hpp"

struct mxfft_batch_s {
    struct Group {
        mxfft_group g{};
        int32_t kbase = 0;            // first k_out index of the group
        int branch = 0;
    };
    struct Branch {
        int n = 0, count = 0;
        mxfft_plan_t plan = nullptr;
        hipStream_t stream = nullptr;  // branch stream (captured, never launched on directly)
        hipEvent_t done = nullptr;
        mxfft_tuning tuning{};
        unsigned long long* d_off = nullptr;  // element offset of each slice in the pools
        int32_t* d_kidx = nullptr;            // k_out index of each slice
        int32_t* d_k = nullptr;               // k of each slice in branch order
    };
    struct Graph {
        bool valid = false;
        const void* in = nullptr;
        void* out = nullptr;
        int32_t* k = nullptr;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<Group> groups;
    std::vector<Branch> branches;
    hipStream_t capture = nullptr;
    hipEvent_t fork = nullptr;
    Graph graphs[3];                   // forward, inverse, round trip
    int last_op = -1;
};

namespace {

void drop_graph(mxfft_batch_s::Graph& gr)
{
    if (gr.exec) (void)hipGraphExecDestroy(gr.exec);
    if (gr.graph) (void)hipGraphDestroy(gr.graph);
    gr = mxfft_batch_s::Graph{};
}

void release(mxfft_batch_s* b)
{
    (void)hipDeviceSynchronize();
    for (auto& gr : b->graphs) drop_graph(gr);
    for (auto& br : b->branches) {
        if (br.plan) mxfft_plan_destroy(br.plan);
        if (br.done) (void)hipEventDestroy(br.done);
        if (br.stream) (void)hipStreamDestroy(br.stream);
        (void)hipFree(br.d_off);
        (void)hipFree(br.d_kidx);
        (void)hipFree(br.d_k);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    delete b;
}

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// One branch: the plan's launch sequence over every slice of that size, the
// slices addressed in the pools through the offset table; k to the branch's
// own array, then scattered to the callers' slice order.
mxfft_status run_branch(const mxfft_batch_s::Branch& br, int op, const void* in, void* out, int32_t* k)
{
    mxk::Workspace w = mxk::plan_workspace(br.plan);
    w.slice_off = br.d_off;
    int32_t* kb = k ? br.d_k : nullptr;
    mxfft_status st;
    switch (op) {
    case 0: st = mxk::plan_forward_ws(br.plan, w, in, out, br.count, kb, br.stream); break;
    case 1: st = mxk::plan_inverse_ws(br.plan, w, in, out, br.count, nullptr, br.stream); break;
    default: st = mxk::plan_roundtrip_ws(br.plan, w, in, out, br.count, kb, br.stream); break;
    }
    if (st != MXFFT_OK || !kb) return st;
    return mxk::launch_scatter_k(kb, br.d_kidx, k, br.count, br.stream) == hipSuccess ? MXFFT_OK : MXFFT_EHIP;
}

// Capture op over every group into gr: fork from the capture stream, one
// branch per group, join back.
mxfft_status capture(mxfft_batch_s* b, int op, const void* in, void* out, int32_t* k, mxfft_batch_s::Graph& gr)
{
    drop_graph(gr);
    if (hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal) != hipSuccess) return MXFFT_EHIP;
    mxfft_status st = MXFFT_OK;
    bool ok = hipEventRecord(b->fork, b->capture) == hipSuccess;
    for (auto& br : b->branches) {
        if (!ok || st != MXFFT_OK) break;
        ok = hipStreamWaitEvent(br.stream, b->fork, 0) == hipSuccess;
        if (ok) st = run_branch(br, op, in, out, k);
        ok = ok && hipEventRecord(br.done, br.stream) == hipSuccess;
        ok = ok && hipStreamWaitEvent(b->capture, br.done, 0) == hipSuccess;
    }
    hipGraph_t graph = nullptr;
    const bool ended = hipStreamEndCapture(b->capture, &graph) == hipSuccess;
    if (!ok || !ended || st != MXFFT_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st != MXFFT_OK ? st : MXFFT_EHIP;
    }
    hipGraphExec_t exec = nullptr;
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return MXFFT_EHIP;
    }
    gr.valid = true;
    gr.in = in;
    gr.out = out;
    gr.k = k;
    gr.graph = graph;
    gr.exec = exec;
    return MXFFT_OK;
}

}  // namespace

extern "C" {

mxfft_status mxfft_batch_create(mxfft_batch_t* out, const mxfft_group* groups, int32_t ngroups,
                                const mxfft_params* p, const char* tune_cache, void* stream)
{
    if (!out || !groups || !p || ngroups < 1 || ngroups > 4096) return MXFFT_EINVAL;
    *out = nullptr;
    // groups: valid sizes, no overlap of their [offset, offset + count n^2) ranges
    std::vector<std::pair<uint64_t, uint64_t>> span;
    long total = 0;
    for (int i = 0; i < ngroups; i++) {
        const mxfft_group& g = groups[i];
        if (!pow2(g.n) || g.n < 2 || g.n > 4096 || g.count < 1 || g.count > 65535) return MXFFT_EINVAL;
        span.emplace_back(g.offset, g.offset + (uint64_t)g.count * g.n * g.n);
        total += g.count;
    }
    if (total > INT32_MAX) return MXFFT_EINVAL;
    std::sort(span.begin(), span.end());
    for (size_t i = 1; i < span.size(); i++)
        if (span[i].first < span[i - 1].second) return MXFFT_EINVAL;

    mxfft_batch_s* b = new mxfft_batch_s();
    mxfft_status st = MXFFT_OK;
    bool ok = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess;
    // the work list: groups in the caller's order, merged into one branch per
    // distinct n (branches in order of first appearance)
    std::vector<std::vector<unsigned long long>> offs;
    std::vector<std::vector<int32_t>> kidx;
    int32_t kbase = 0;
    for (int i = 0; i < ngroups; i++) {
        mxfft_batch_s::Group g;
        g.g = groups[i];
        g.kbase = kbase;
        kbase += g.g.count;
        auto it = std::find_if(b->branches.begin(), b->branches.end(), [&](const auto& br) { return br.n == g.g.n; });
        if (it == b->branches.end()) {
            b->branches.emplace_back();
            b->branches.back().n = g.g.n;
            offs.emplace_back();
            kidx.emplace_back();
            it = b->branches.end() - 1;
        }
        g.branch = (int)(it - b->branches.begin());
        for (int j = 0; j < g.g.count; j++) {
            offs[g.branch].push_back(g.g.offset + (unsigned long long)j * g.g.n * g.g.n);
            kidx[g.branch].push_back(g.kbase + j);
        }
        it->count += g.g.count;
        b->groups.push_back(g);
    }
    for (size_t r = 0; r < b->branches.size() && ok && st == MXFFT_OK; r++) {
        auto& br = b->branches[r];
        st = mxfft_plan(&br.plan, br.n, br.count, p, stream);
        if (st != MXFFT_OK) break;
        ok = hipStreamCreateWithFlags(&br.stream, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&br.done, hipEventDisableTiming) == hipSuccess;
        ok = ok && hipMalloc((void**)&br.d_off, offs[r].size() * sizeof(unsigned long long)) == hipSuccess;
        ok = ok && hipMalloc((void**)&br.d_kidx, kidx[r].size() * sizeof(int32_t)) == hipSuccess;
        ok = ok && hipMalloc((void**)&br.d_k, kidx[r].size() * sizeof(int32_t)) == hipSuccess;
        ok = ok && hipMemcpy(br.d_off, offs[r].data(), offs[r].size() * sizeof(unsigned long long),
                             hipMemcpyHostToDevice) == hipSuccess;
        ok = ok && hipMemcpy(br.d_kidx, kidx[r].data(), kidx[r].size() * sizeof(int32_t), hipMemcpyHostToDevice) ==
                       hipSuccess;
        if (!ok) break;
        // the line kernels are tuned on up to 1024 slices of that size; the
        // register-resident passes keep their defaults here: the choices that
        // win for one size alone (a separate statistics read) were measured
        // slower with the other sizes' branches beside them
        st = mxfft_plan_get_tuning(br.plan, &br.tuning);
        if (st != MXFFT_OK || br.tuning.fast) continue;
        st = mxfft_tune(br.n, p, std::min(br.count, 1024), tune_cache, 0, &br.tuning, stream);
        if (st != MXFFT_OK) break;
        st = mxfft_plan_set_tuning(br.plan, &br.tuning);
    }
    ok = ok && hipStreamSynchronize((hipStream_t)stream) == hipSuccess;
    if (!ok || st != MXFFT_OK) {
        release(b);
        return st != MXFFT_OK ? st : MXFFT_EHIP;
    }
    *out = b;
    return MXFFT_OK;
}

mxfft_status mxfft_batch_execute(mxfft_batch_t b, int32_t op, const void* in, void* out, int32_t* k_out,
                                 void* stream)
{
    if (!b || !in || !out || op < 0 || op > 2) return MXFFT_EINVAL;
    mxfft_batch_s::Graph& gr = b->graphs[op];
    if (!gr.valid || gr.in != in || gr.out != out || gr.k != k_out) {
        const mxfft_status st = capture(b, op, in, out, k_out, gr);
        if (st != MXFFT_OK) return st;
    }
    if (hipGraphLaunch(gr.exec, (hipStream_t)stream) != hipSuccess) return MXFFT_EHIP;
    b->last_op = op;
    return MXFFT_OK;
}

mxfft_status mxfft_batch_last_status(mxfft_batch_t b, void* stream)
{
    if (!b) return MXFFT_EINVAL;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return MXFFT_EHIP;
    for (auto& br : b->branches) {
        const mxfft_status st = mxfft_plan_last_status(br.plan, br.stream);
        if (st != MXFFT_OK) return st;
    }
    return MXFFT_OK;
}

mxfft_status mxfft_batch_group_tuning(mxfft_batch_t b, int32_t g, mxfft_tuning* out)
{
    if (!b || !out || g < 0 || g >= (int32_t)b->groups.size()) return MXFFT_EINVAL;
    *out = b->branches[b->groups[g].branch].tuning;
    return MXFFT_OK;
}

mxfft_status mxfft_batch_destroy(mxfft_batch_t b)
{
    if (!b) return MXFFT_OK;
    release(b);
    return MXFFT_OK;
}

}  // extern "C"
