// hipGraph capture of library calls: everything the caller enqueues on a
// stream between af_graph_begin and af_graph_end becomes one replayable graph.
#include <hip/hip_runtime.h>

#include <new>

#include "common.h"

using namespace afm;

struct af_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" af_status af_graph_begin(af_stream stream) {
    clear_error();
    AF_CHECK_ARG(stream, "capture needs a non-default stream");
    AF_HIP(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal));
    return AF_OK;
}

extern "C" af_status af_graph_end(af_stream stream, af_graph** out) {
    clear_error();
    AF_CHECK_ARG(stream && out, "stream and out must be non-null");
    af_graph* g = new (std::nothrow) af_graph();
    if (!g) { set_error("out of host memory"); return AF_ENOMEM; }
    hipError_t e = hipStreamEndCapture((hipStream_t)stream, &g->graph);
    if (e != hipSuccess) {
        delete g;
        set_error("hipStreamEndCapture failed: %s", hipGetErrorString(e));
        return AF_EHIP;
    }
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g->graph);
        delete g;
        set_error("hipGraphInstantiate failed: %s", hipGetErrorString(e));
        return AF_EHIP;
    }
    *out = g;
    return AF_OK;
}

extern "C" af_status af_graph_launch(af_graph* g, af_stream stream) {
    clear_error();
    AF_CHECK_ARG(g && g->exec, "graph must be non-null");
    AF_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return AF_OK;
}

extern "C" void af_graph_destroy(af_graph* g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}
