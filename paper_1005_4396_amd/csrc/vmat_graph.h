// Replay of captured kernel sequences (HIP graphs) for the iteration loops.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>
#include <string>

#include "vmat_internal.h"

namespace vmat {

// Kinds of captured sequences kept per handle.
enum GraphKind { G_MASTER_D = 0, G_MASTER_AP = 1, G_BATCH_DIR = 2, G_BATCH_STEP = 3 };

// Everything a captured sequence takes by value: the pointers and scalars it
// was captured with.  A different key captures again.
typedef uint64_t GraphKey[GRAPH_KEY_LEN];

// VMAT_NO_GRAPH: launch the iteration kernels one by one instead of replaying
// a captured graph (the same kernels and arguments, so the same bits).
inline bool graphs_off() { return getenv("VMAT_NO_GRAPH") != nullptr; }

// Captures `body` into the handle's graph of this kind (replacing any earlier
// one) and records its key.  Graphs hold kernels only.
template <class F>
vmat_status capture_graph(vmat_ctx* h, int kind, const GraphKey key, F body) {
    hipGraphExec_t& exec = h->iter_graph[kind];
    if (exec) {
        (void)hipGraphExecDestroy(exec);
        exec = nullptr;
    }
    if (!h->cap_stream) VMAT_HIP(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    VMAT_HIP(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    vmat_status rc = body(h->cap_stream);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(h->cap_stream, &graph);
    if (rc != VMAT_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(VMAT_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
        exec = nullptr;
        return fail(VMAT_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
    }
    for (int i = 0; i < GRAPH_KEY_LEN; ++i) h->iter_key[kind][i] = key[i];
    return VMAT_OK;
}

// Enqueues `body` on st: replayed from a graph captured once per key, or
// launched directly when graphs are off.
template <class F>
vmat_status run_iteration(vmat_ctx* h, int kind, const GraphKey key, F body, hipStream_t st) {
    if (graphs_off()) return body(st);
    bool same = h->iter_graph[kind] != nullptr;
    for (int i = 0; i < GRAPH_KEY_LEN; ++i) same = same && h->iter_key[kind][i] == key[i];
    if (!same) {
        const vmat_status rc = capture_graph(h, kind, key, body);
        if (rc != VMAT_OK) return rc;
    }
    VMAT_HIP(hipGraphLaunch(h->iter_graph[kind], st));
    return VMAT_OK;
}

}  // namespace vmat
