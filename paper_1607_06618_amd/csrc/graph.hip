// Whole-path replay: the batched path recorded into one HIP graph by stream
// capture, replayed with one launch per batch.
#include <new>
#include <vector>

#include "gerbil.h"

#include "common.h"
#include "internal.h"

struct gerbil_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint32_t n_nodes = 0;
    uint32_t n_kernel = 0;
};

namespace {

void release(gerbil_graph* g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

int32_t enqueue_path(const gerbil_pipeline* pl, const gerbil_params* p, gerbil_encoded* enc, gerbil_bins* bins,
                     gerbil_counted* state, hipStream_t stream) {
    int32_t st = gerbil_encode(pl->ascii, pl->offsets, pl->n_reads, pl->n_bytes, p->k, pl->ws_encode,
                               pl->ws_encode_bytes, enc, stream);
    if (st == GERBIL_OK) st = gerbil_bin(enc, p, pl->ws_bin, pl->ws_bin_bytes, bins, stream);
    if (st == GERBIL_OK)
        st = gerbil_count(bins, p, pl->ws_count, pl->ws_count_bytes, pl->keys, pl->counts, pl->cap, state, stream);
    if (st == GERBIL_OK) st = gerbil_histogram(state, pl->hist, pl->hist_len, stream);
    return st;
}

}  // namespace

extern "C" {

int32_t gerbil_graph_capture(const gerbil_pipeline* pl, const gerbil_params* p, gerbil_encoded* enc,
                             gerbil_bins* bins, gerbil_counted* state, hipStream_t stream, gerbil_graph** out) {
    if (!pl || !p || !enc || !bins || !state || !out || !stream) return GERBIL_EINVAL;
    *out = nullptr;
    if (p->mode != GERBIL_BATCHED) return GERBIL_EUNSUPPORTED;
    hipStreamCaptureStatus cs;
    if (hipStreamIsCapturing(stream, &cs) != hipSuccess) return GERBIL_EDEVICE;
    if (cs != hipStreamCaptureStatusNone) return GERBIL_EINVAL;
    gerbil_params q = *p;
    q.timing_events = nullptr;   // event nodes are not part of the replayed path

    gerbil_graph* g = new (std::nothrow) gerbil_graph();
    if (!g) return GERBIL_EDEVICE;
    // Relaxed: the launchers may query device attributes while recording.
    if (hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
        release(g);
        return GERBIL_EDEVICE;
    }
    const int32_t st = enqueue_path(pl, &q, enc, bins, state, stream);
    const hipError_t ec = hipStreamEndCapture(stream, &g->graph);
    if (st != GERBIL_OK || ec != hipSuccess || !g->graph) {
        release(g);
        return st != GERBIL_OK ? st : GERBIL_EDEVICE;
    }
    size_t n = 0;
    if (hipGraphGetNodes(g->graph, nullptr, &n) != hipSuccess) {
        release(g);
        return GERBIL_EDEVICE;
    }
    std::vector<hipGraphNode_t> nodes(n);
    if (n && hipGraphGetNodes(g->graph, nodes.data(), &n) != hipSuccess) {
        release(g);
        return GERBIL_EDEVICE;
    }
    g->n_nodes = (uint32_t)n;
    for (size_t i = 0; i < n; i++) {
        hipGraphNodeType t;
        if (hipGraphNodeGetType(nodes[i], &t) != hipSuccess) {
            release(g);
            return GERBIL_EDEVICE;
        }
        if (t != hipGraphNodeTypeKernel) {
            release(g);
            return GERBIL_EUNSUPPORTED;
        }
        g->n_kernel++;
    }
    if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) {
        release(g);
        return GERBIL_EDEVICE;
    }
    *out = g;
    return GERBIL_OK;
}

int32_t gerbil_graph_launch(const gerbil_graph* g, hipStream_t stream) {
    if (!g || !g->exec) return GERBIL_EINVAL;
    return hipGraphLaunch(g->exec, stream) == hipSuccess ? GERBIL_OK : GERBIL_EDEVICE;
}

int32_t gerbil_graph_info(const gerbil_graph* g, uint32_t* n_nodes, uint32_t* n_kernel_nodes) {
    if (!g) return GERBIL_EINVAL;
    if (n_nodes) *n_nodes = g->n_nodes;
    if (n_kernel_nodes) *n_kernel_nodes = g->n_kernel;
    return GERBIL_OK;
}

int32_t gerbil_graph_destroy(gerbil_graph* g) {
    release(g);
    return GERBIL_OK;
}

}  // extern "C"
