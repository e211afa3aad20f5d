// mxfft_batch.cpp -- uneven batches: groups of slices of different sizes,
// transformed by one HIP graph launch with one independent branch per group.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>
#include <vector>

#include "mxfft.h"

struct mxfft_batch_s {
    struct Group {
        mxfft_group g{};
        int32_t kbase = 0;            // first k_out index of the group
        mxfft_plan_t plan = nullptr;
        hipStream_t stream = nullptr;  // branch stream (captured, never launched on directly)
        hipEvent_t done = nullptr;
        mxfft_tuning tuning{};
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
    for (auto& g : b->groups) {
        if (g.plan) mxfft_plan_destroy(g.plan);
        if (g.done) (void)hipEventDestroy(g.done);
        if (g.stream) (void)hipStreamDestroy(g.stream);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    delete b;
}

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

mxfft_status run_group(const mxfft_batch_s::Group& g, int op, const void* in, void* out, int32_t* k)
{
    const size_t off = (size_t)g.g.offset * 8;
    const void* src = (const char*)in + off;
    void* dst = (char*)out + off;
    int32_t* kg = k ? k + g.kbase : nullptr;
    switch (op) {
    case 0: return mxfft_forward(g.plan, src, dst, g.g.count, kg, g.stream);
    case 1: return mxfft_inverse(g.plan, src, dst, g.g.count, nullptr, g.stream);
    default: return mxfft_roundtrip(g.plan, src, dst, g.g.count, kg, g.stream);
    }
}

// Capture op over every group into gr: fork from the capture stream, one
// branch per group, join back.
mxfft_status capture(mxfft_batch_s* b, int op, const void* in, void* out, int32_t* k, mxfft_batch_s::Graph& gr)
{
    drop_graph(gr);
    if (hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal) != hipSuccess) return MXFFT_EHIP;
    mxfft_status st = MXFFT_OK;
    bool ok = hipEventRecord(b->fork, b->capture) == hipSuccess;
    for (auto& g : b->groups) {
        if (!ok || st != MXFFT_OK) break;
        ok = hipStreamWaitEvent(g.stream, b->fork, 0) == hipSuccess;
        if (ok) st = run_group(g, op, in, out, k);
        ok = ok && hipEventRecord(g.done, g.stream) == hipSuccess;
        ok = ok && hipStreamWaitEvent(b->capture, g.done, 0) == hipSuccess;
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
    // one tuning per distinct n (sample: up to 64 slices of that size)
    std::vector<std::pair<int, mxfft_tuning>> tuned;
    int32_t kbase = 0;
    for (int i = 0; i < ngroups && ok && st == MXFFT_OK; i++) {
        mxfft_batch_s::Group g;
        g.g = groups[i];
        g.kbase = kbase;
        kbase += g.g.count;
        b->groups.push_back(g);
        auto& G = b->groups.back();
        st = mxfft_plan(&G.plan, G.g.n, G.g.count, p, stream);
        if (st != MXFFT_OK) break;
        ok = hipStreamCreateWithFlags(&G.stream, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&G.done, hipEventDisableTiming) == hipSuccess;
        auto it = std::find_if(tuned.begin(), tuned.end(), [&](const auto& t) { return t.first == G.g.n; });
        if (it == tuned.end()) {
            int sample = 0;
            for (int j = 0; j < ngroups; j++)
                if (groups[j].n == G.g.n) sample += groups[j].count;
            mxfft_tuning t{};
            st = mxfft_tune(G.g.n, p, std::min(sample, 64), tune_cache, 0, &t, stream);
            if (st != MXFFT_OK) break;
            tuned.emplace_back(G.g.n, t);
            it = tuned.end() - 1;
        }
        G.tuning = it->second;
        if (!G.tuning.fast) st = mxfft_plan_set_tuning(G.plan, &G.tuning);
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
    for (auto& g : b->groups) {
        const mxfft_status st = mxfft_plan_last_status(g.plan, g.stream);
        if (st != MXFFT_OK) return st;
    }
    return MXFFT_OK;
}

mxfft_status mxfft_batch_group_tuning(mxfft_batch_t b, int32_t g, mxfft_tuning* out)
{
    if (!b || !out || g < 0 || g >= (int32_t)b->groups.size()) return MXFFT_EINVAL;
    *out = b->groups[g].tuning;
    return MXFFT_OK;
}

mxfft_status mxfft_batch_destroy(mxfft_batch_t b)
{
    if (!b) return MXFFT_OK;
    release(b);
    return MXFFT_OK;
}

}  // extern "C"
