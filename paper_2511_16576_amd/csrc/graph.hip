// HIP graph capture of a caller's sequence of libpolymh calls on a stream
// (the batched query pipeline is captured once and replayed per batch, so
// the dozens of small launches cost one graph launch).  Streams that wait
// on an event recorded on the capturing stream join the capture, so a
// caller can fork work onto several streams and join it back: their
// branches run concurrently when the graph is replayed.
#include "internal.hpp"

#include <new>

struct polymh_graph_t {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

polymh_status polymh_graph_begin(void *stream)
{
    if (!stream) return polymh::set_error(POLYMH_EINVAL, "graph_begin: capture needs a non-null stream");
    hipError_t e = hipStreamBeginCapture(reinterpret_cast<hipStream_t>(stream), hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return polymh::set_error(POLYMH_EDEVICE, "graph_begin: %s", hipGetErrorString(e));
    return POLYMH_OK;
}

polymh_status polymh_graph_end(void *stream, polymh_graph *out)
{
    if (!stream || !out) return polymh::set_error(POLYMH_EINVAL, "graph_end: NULL argument");
    *out = nullptr;
    polymh_graph_t *g = new (std::nothrow) polymh_graph_t;
    if (!g) return polymh::set_error(POLYMH_EDEVICE, "graph_end: out of host memory");
    hipError_t e = hipStreamEndCapture(reinterpret_cast<hipStream_t>(stream), &g->graph);
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        if (g->graph) (void)hipGraphDestroy(g->graph);   // the capture's error is the one reported
        delete g;
        return polymh::set_error(POLYMH_EDEVICE, "graph_end: %s", hipGetErrorString(e));
    }
    *out = g;
    return POLYMH_OK;
}

polymh_status polymh_graph_launch(polymh_graph g, void *stream)
{
    if (!g || !g->exec) return polymh::set_error(POLYMH_EINVAL, "graph_launch: no graph");
    hipError_t e = hipGraphLaunch(g->exec, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return polymh::set_error(POLYMH_EDEVICE, "graph_launch: %s", hipGetErrorString(e));
    return POLYMH_OK;
}

void polymh_graph_destroy(polymh_graph g)
{
    if (!g) return;
    // a destroy call has no caller to report to
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

}  // extern "C"
