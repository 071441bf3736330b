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

// gamma enters the captured control kernels by value: part of the key
inline uint64_t gamma_bits(const vmat_ctx* h) {
    uint64_t b;
    std::memcpy(&b, &h->gamma, sizeof(b));
    return b;
}

// Enqueues `body` on st: replayed from a graph captured once per key, or
// launched directly when VMAT_NO_GRAPH is set.  Graphs hold kernels only.
template <class F>
vmat_status run_iteration(vmat_ctx* h, int kind, const GraphKey key, F body, hipStream_t st) {
    if (getenv("VMAT_NO_GRAPH")) return body(st);
    hipGraphExec_t& exec = h->iter_graph[kind];
    bool same = exec != nullptr;
    for (int i = 0; i < GRAPH_KEY_LEN; ++i) same = same && h->iter_key[kind][i] == key[i];
    if (!same) {
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
    }
    VMAT_HIP(hipGraphLaunch(exec, st));
    return VMAT_OK;
}

}  // namespace vmat
