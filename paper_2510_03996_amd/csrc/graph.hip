// Graph capture of library calls: a layer schedule, a bootstrap or any other
// sequence of calls issued on one stream is recorded once into a hipGraph
// (helper streams the calls fork join back inside the capture) and replayed
// as one launch.
#include "internal.h"

struct he_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

using namespace he;

extern "C" {

int he_capture_begin(he_ctx* h, he_stream stream) {
  if (!h) return set_error(HE_EINVAL, "null context");
  hipStream_t s = (hipStream_t)stream;
  if (!s) return set_error(HE_EINVAL, "graph capture needs a non-default stream");
  if (h->c.prof_on) return set_error(HE_EINVAL, "profiling is on: its event waits cannot be captured");
  if (stream_capturing(s)) return set_error(HE_EINVAL, "the stream is already capturing");
  HE_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
  return HE_OK;
}

int he_capture_end(he_ctx* h, he_stream stream, he_graph** out) {
  if (!h || !out) return set_error(HE_EINVAL, "null argument");
  *out = nullptr;
  hipStream_t s = (hipStream_t)stream;
  if (!stream_capturing(s)) return set_error(HE_EINVAL, "the stream is not capturing");
  hipGraph_t g = nullptr;
  HE_HIP(hipStreamEndCapture(s, &g));
  hipGraphExec_t x = nullptr;
  hipError_t e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    hipGraphDestroy(g);
    return hip_error(e, "graph instantiation");
  }
  he_graph* r = new (std::nothrow) he_graph;
  if (!r) {
    hipGraphExecDestroy(x);
    hipGraphDestroy(g);
    return set_error(HE_ENOMEM, "host allocation failed");
  }
  r->graph = g;
  r->exec = x;
  *out = r;
  return HE_OK;
}

int he_graph_launch(he_graph* g, he_stream stream) {
  if (!g || !g->exec) return set_error(HE_EINVAL, "null graph");
  HE_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
  return HE_OK;
}

int he_graph_destroy(he_graph* g) {
  if (!g) return HE_OK;
  if (g->exec) hipGraphExecDestroy(g->exec);
  if (g->graph) hipGraphDestroy(g->graph);
  delete g;
  return HE_OK;
}

}  // extern "C"
