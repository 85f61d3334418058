// Graph form of a batched call: the pass launches of a fixed block array
// captured once into a HIP graph that owns its job table and workspace,
// then replayed with a single launch.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/pa.h"
#include "pa_kernels.h"
#include "pa_runtime.h"

using namespace pa::rt;

struct pa_graph_s {
    int device = 0;
    void *buf = nullptr;           // job table + A/S workspace of every block
    hipStream_t capture = nullptr;  // private stream the launches were captured on
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint32_t count = 0;
    bool modified = false;
    BatchForm form = kFormLanes;  // launch form captured
    // group layouts the launches were captured for (length, plain-path
    // blocks, blocks per shared seed)
    std::vector<std::vector<uint64_t>> groups;
};

namespace {

void destroy_graph(pa_graph_s *g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->capture) {
        release_stream_state(g->capture);
        (void)hipStreamDestroy(g->capture);
    }
    if (g->buf) (void)hipFree(g->buf);
    delete g;
}

struct CaptureFlag {
    CaptureFlag() : old(set_capturing(true)) {}
    ~CaptureFlag() { set_capturing(old); }
    bool old;
};

}  // namespace

extern "C" {

pa_status pa_graph_create(const pa_block *blocks, uint32_t count, int modified, pa_graph_t *graph) {
    if (!graph) return fail(PA_ERR_INVALID_ARG, "null graph out-pointer");
    *graph = nullptr;
    if (count == 0) return fail(PA_ERR_INVALID_ARG, "empty block array");
    BatchPrep bp;
    PA_TRY(prepare_batch(blocks, count, modified != 0, &bp, batch_form(kFormLanes)));
    pa_graph_s *g = new (std::nothrow) pa_graph_s();
    if (!g) return fail(PA_ERR_OUT_OF_MEMORY, "host allocation");
    g->count = count;
    g->modified = modified != 0;
    g->form = bp.form;
    for (const auto &gr : bp.groups) g->groups.push_back(gr.layout());
    auto bail = [&](pa_status st) {
        destroy_graph(g);
        return st;
    };
    hipError_t e = hipGetDevice(&g->device);
    if (e == hipSuccess) e = hipMalloc(&g->buf, bp.total_bytes);
    if (e != hipSuccess) return bail(from_hip(e, "graph workspace"));
    build_table(bp, g->buf);
    e = hipMemcpy(g->buf, bp.blob.data(), bp.blob.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&g->capture, hipStreamNonBlocking);
    if (e != hipSuccess) return bail(from_hip(e, "graph setup"));
    // everything created lazily on the launch path exists before capture:
    // per-device kernel attributes and the capture stream's side lanes
    for (const auto &gr : bp.groups) {
        e = pa::warm_launch_state(*gr.plan.host);
        if (e != hipSuccess) return bail(from_hip(e, "kernel setup"));
    }
    {
        const int lanes = (int)std::min<size_t>(bp.groups.size(), (size_t)kMaxLanes);
        hipStream_t lane_s[kMaxLanes];
        pa_status ls = fork_lanes(g->capture, lanes, lane_s);
        if (ls == PA_OK) ls = join_lanes(g->capture, lanes);
        if (ls != PA_OK) return bail(ls);
        e = hipStreamSynchronize(g->capture);
        if (e != hipSuccess) return bail(from_hip(e, "lane setup"));
    }
    e = hipStreamBeginCapture(g->capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bail(from_hip(e, "hipStreamBeginCapture"));
    pa_status st;
    {
        CaptureFlag cf;
        st = launch_batch(bp, g->buf, g->capture);
    }
    hipGraph_t captured = nullptr;
    e = hipStreamEndCapture(g->capture, &captured);
    g->graph = captured;
    if (st != PA_OK) return bail(st);
    if (e != hipSuccess) return bail(from_hip(e, "hipStreamEndCapture"));
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return bail(from_hip(e, "hipGraphInstantiate"));
    *graph = g;
    return PA_OK;
}

pa_status pa_graph_launch(pa_graph_t graph, void *stream) {
    if (!graph) return fail(PA_ERR_INVALID_ARG, "null graph");
    int dev = 0;
    PA_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (dev != graph->device) return fail(PA_ERR_INVALID_ARG, "graph belongs to another device");
    PA_HIP(hipGraphLaunch(graph->exec, (hipStream_t)stream), "hipGraphLaunch");
    return PA_OK;
}

pa_status pa_graph_update(pa_graph_t graph, const pa_block *blocks, uint32_t count, void *stream) {
    if (!graph) return fail(PA_ERR_INVALID_ARG, "null graph");
    int dev = 0;
    PA_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (dev != graph->device) return fail(PA_ERR_INVALID_ARG, "graph belongs to another device");
    if (count != graph->count) return fail(PA_ERR_INVALID_ARG, "block count differs from the graph's");
    BatchPrep bp;
    PA_TRY(prepare_batch(blocks, count, graph->modified, &bp, graph->form));
    bool same = bp.groups.size() == graph->groups.size();
    for (size_t i = 0; same && i < bp.groups.size(); ++i) same = bp.groups[i].layout() == graph->groups[i];
    if (!same)
        return fail(PA_ERR_INVALID_ARG,
                    "blocks need other transform lengths, or share seeds otherwise, than the graph was built for");
    // Same group layouts give the same table layout (descriptors, residues
    // and spectra in group order); the captured launches keep their plans.
    build_table(bp, graph->buf);
    return stage_upload((hipStream_t)stream, graph->buf, bp.blob.data(), bp.blob.size());
}

uint32_t pa_graph_block_count(pa_graph_t graph) { return graph ? graph->count : 0; }

pa_status pa_graph_destroy(pa_graph_t graph) {
    if (!graph) return PA_OK;
    destroy_graph(graph);
    return PA_OK;
}

}  // extern "C"
