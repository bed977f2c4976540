// HIP-graph capture and replay of whole relaxation iterations.
//
// One iteration is build_cells (A -> B) + relax_step + project on B; the next
// is build_cells (B -> A) + ... on A. An even number of iterations therefore
// returns the state to buffer set A, so the captured sequence can be replayed
// any number of times. Every node is a kernel: the hot calls use no memset or
// copy, which keeps replays equal to eager runs.
#include <new>

#include "internal.h"

struct fppg_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int32_t iters = 0;
};

using namespace fppg;

extern "C" fppg_status fppg_graph_create(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, float* pos_a,
                                         int32_t* id_a, int32_t* owner_a, float* pos_b, int32_t* id_b,
                                         int32_t* owner_b, int32_t* cell_start, int32_t* feat_seg, double* feat_u,
                                         int32_t n_feat, uint32_t move_mask, float* amax, float* disp,
                                         int64_t* counters, void* ws, size_t ws_bytes, int32_t iters,
                                         void* stream, fppg_graph** out) {
  if (!ctx || !geom || !out) return fail(ctx, FPPG_E_ARG, "null ctx/geom/out");
  *out = nullptr;
  if (iters < 2 || (iters & 1)) return fail(ctx, FPPG_E_ARG, "iters must be even and >= 2");
  if (ctx->profiling) return fail(ctx, FPPG_E_ARG, "disable profiling before capturing a graph");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (s == nullptr) return fail(ctx, FPPG_E_ARG, "capture needs a non-default stream");
  FPPG_HIP(ctx, hipSetDevice(ctx->device));
  FPPG_HIP(ctx, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  fppg_status st = FPPG_OK;
  for (int32_t it = 0; it < iters && st == FPPG_OK; ++it) {
    float* pi = (it & 1) ? pos_b : pos_a;
    int32_t* ii = (it & 1) ? id_b : id_a;
    int32_t* oi = (it & 1) ? owner_b : owner_a;
    float* po = (it & 1) ? pos_a : pos_b;
    int32_t* io = (it & 1) ? id_a : id_b;
    int32_t* oo = (it & 1) ? owner_a : owner_b;
    st = fppg_build_cells(ctx, geom, n, pi, ii, oi, po, io, oo, cell_start, ws, ws_bytes, stream);
    if (st == FPPG_OK)
      st = fppg_relax_step(ctx, geom, n, po, oo, cell_start, feat_seg, n_feat, move_mask, 0u, nullptr, amax, disp,
                           nullptr, 0, ws, ws_bytes, stream);
    if (st == FPPG_OK)
      st = fppg_project(ctx, geom, n, po, oo, disp, feat_seg, feat_u, n_feat, move_mask, counters, nullptr, 0, ws,
                        ws_bytes, stream);
  }
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(s, &graph);
  if (st != FPPG_OK) {
    if (graph) hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    hipGraphDestroy(graph);
    return hip_fail(ctx, e, "hipGraphInstantiate");
  }
  fppg_graph* g = new (std::nothrow) fppg_graph();
  if (!g) {
    hipGraphExecDestroy(exec);
    hipGraphDestroy(graph);
    return fail(ctx, FPPG_E_CAPACITY, "out of host memory");
  }
  g->graph = graph;
  g->exec = exec;
  g->iters = iters;
  *out = g;
  return FPPG_OK;
}

extern "C" fppg_status fppg_graph_launch(fppg_ctx* ctx, fppg_graph* g, int32_t repeats, void* stream) {
  if (!ctx || !g || repeats < 0) return fail(ctx, FPPG_E_ARG, "null ctx/graph or negative repeats");
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int32_t r = 0; r < repeats; ++r) FPPG_HIP(ctx, hipGraphLaunch(g->exec, s));
  return FPPG_OK;
}

extern "C" void fppg_graph_destroy(fppg_graph* g) {
  if (!g) return;
  if (g->exec) hipGraphExecDestroy(g->exec);
  if (g->graph) hipGraphDestroy(g->graph);
  delete g;
}
