// Batched queries.  A batch is one plan whose tables come from many queries.
// Its factor build and summary are recorded as one launch per stage and tree
// level, each covering every query (every kernel walks a (table, tile) work
// list): gj_batch_launch (and gj_batch_launch_kernels) replay that graph,
// gj_batch_launch_eager issues the same launches unrecorded.  The persistent
// kernel of batch_persist.hip (every stage of every query in one launch, from
// a device task queue) is planned but switched off: gj_batch_launch_persistent.
// Workspaces are sized by row counts only (an entry count never exceeds its
// table's row count), so nothing inside either graph allocates or waits for
// the host.
#include <vector>

#include "kernels.h"
#include "persist.h"
#include "plan.h"

using namespace gjh;

struct gj_batch {
  gj_ctx* ctx = nullptr;
  gj_factors* f = nullptr;
  gj_summary* s = nullptr;  // one set of summary arrays for all queries
  std::vector<gj_summary*> views;
  hipGraph_t graph = nullptr;  // one launch per stage
  hipGraphExec_t exec = nullptr;
  gjk::PArgs pargs{};  // shape of the persistent kernel's plan (not launched)
  int pgrid = 0;
  hipStream_t cap = nullptr;
  hipEvent_t done = nullptr;  // end of a launch on a stream other than the context's
  std::vector<int64_t> cnt_host;
  bool counters_valid = false;
};

static void batch_destroy(gj_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->done) (void)hipEventDestroy(b->done);
  for (gj_summary* v : b->views) delete v;
  if (b->s) {
    b->s->borrowed = false;
    gj_free_summary(b->s);
  }
  if (b->f) gj_free_factors(b->f);
  delete b;
}

extern "C" {

gj_status gj_batch_create(gj_ctx* ctx, int32_t n_queries, const int32_t* q_off, const gj_table* tables,
                          const gj_join_graph* graphs, const gj_tune* tune, gj_batch** out) {
  GJ_SCOPE(ctx);
  if (!ctx || n_queries < 1 || !q_off || !tables || !graphs || !out) {
    set_error("gj_batch_create: bad argument");
    return GJ_E_INVALID;
  }
  gj_tune saved = ctx->tune;
  if (tune) {
    gj_status st = gj_ctx_set_tune(ctx, tune);
    if (st) return st;
  }
  gj_batch* b = new gj_batch();
  b->ctx = ctx;
  b->f = new gj_factors(ctx);
  b->f->plan.ctx = ctx;
  std::vector<int> qoff(q_off, q_off + n_queries + 1);
  gj_status st = plan_tables(b->f->plan, n_queries, qoff.data(), tables, graphs);
  if (!st) st = plan_device(b->f->plan, b->f->arena, b->f->F);
  ctx->tune = saved;
  if (st) {
    batch_destroy(b);
    return st;
  }
  b->s = new gj_summary(ctx);
  b->s->f = b->f;
  b->f->refs++;
  b->s->borrowed = true;
  if ((st = alloc_summary(b->f->plan, b->s->arena, b->s->S))) {
    batch_destroy(b);
    return st;
  }
  // the persistent kernel's plan (stage instances, dependencies, tasks) is
  // built so that its shape can be inspected; the kernel itself is not
  // recorded or launched (see gj_batch_launch_persistent)
  const Plan& P = b->f->plan;
  std::vector<gjk::PStage> stages;
  std::vector<int32_t> deps;
  std::vector<gjk::PTask> tasks;
  gjk::build_persistent_plan(P, (tune ? *tune : ctx->tune).batch_task_rows, stages, deps, tasks);
  b->pargs.ntasks = (int32_t)tasks.size();
  b->pargs.nstages = (int32_t)stages.size();
  b->pargs.nq = P.nq;
  // record factor build + summary of every query as one launch per stage
  if ((st = check(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking), "capture stream")) ||
      (st = check(hipStreamSynchronize(ctx->stream), "capture")) ||
      (st = check(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal), "begin capture"))) {
    batch_destroy(b);
    return st;
  }
  launch_factors(b->f->plan, b->f->F, b->cap);
  launch_summary(b->f->plan, b->f->F, b->s->S, b->cap);
  hipError_t e1 = hipGetLastError();
  hipError_t e2 = hipStreamEndCapture(b->cap, &b->graph);
  if ((st = check(e1, "batch kernels")) || (st = check(e2, "end capture")) ||
      (st = check(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "graph instantiate"))) {
    batch_destroy(b);
    return st;
  }
  *out = b;
  return GJ_OK;
}

// Work launched on a stream other than the context's: the context's stream
// (on which results, views and downloads are read) waits for its end.
static gj_status join_context_stream(gj_batch* b, hipStream_t s) {
  if (s == b->ctx->stream) return GJ_OK;
  gj_status st;
  if (!b->done && (st = check(hipEventCreateWithFlags(&b->done, hipEventDisableTiming), "event"))) return st;
  if ((st = check(hipEventRecord(b->done, s), "event record"))) return st;
  return check(hipStreamWaitEvent(b->ctx->stream, b->done, 0), "stream wait");
}

gj_status gj_batch_launch(gj_batch* b, void* hip_stream) {
  GJ_SCOPE(b ? b->ctx : nullptr);
  if (!b) {
    set_error("gj_batch_launch: null batch");
    return GJ_E_INVALID;
  }
  b->counters_valid = false;
  hipStream_t s = hip_stream ? (hipStream_t)hip_stream : b->ctx->stream;
  gj_status st = check(hipGraphLaunch(b->exec, s), "graph launch");
  if (st) return st;
  return join_context_stream(b, s);
}

gj_status gj_batch_launch_kernels(gj_batch* b, void* hip_stream) { return gj_batch_launch(b, hip_stream); }

gj_status gj_batch_launch_persistent(gj_batch* b, void* hip_stream) {
  GJ_SCOPE(b ? b->ctx : nullptr);
  (void)hip_stream;
  set_error("gj_batch_launch_persistent: the persistent batch kernel is switched off (its first launch on the "
            "device did not finish within the run's limit and the cause has not been shown); use gj_batch_launch");
  return GJ_E_INVALID;
}

gj_status gj_batch_info(const gj_batch* b, int32_t* n_tasks, int32_t* n_stages, int32_t* grid) {
  if (!b) return GJ_E_INVALID;
  if (n_tasks) *n_tasks = b->pargs.ntasks;
  if (n_stages) *n_stages = b->pargs.nstages;
  if (grid) *grid = b->pgrid;
  return GJ_OK;
}

gj_status gj_batch_launch_eager(gj_batch* b, void* hip_stream) {
  GJ_SCOPE(b ? b->ctx : nullptr);
  if (!b) {
    set_error("gj_batch_launch_eager: null batch");
    return GJ_E_INVALID;
  }
  b->counters_valid = false;
  hipStream_t s = hip_stream ? (hipStream_t)hip_stream : b->ctx->stream;
  launch_factors(b->f->plan, b->f->F, s);
  launch_summary(b->f->plan, b->f->F, b->s->S, s);
  gj_status st = check(hipGetLastError(), "batch kernels");
  if (st) return st;
  return join_context_stream(b, s);
}

const int64_t* gj_batch_join_sizes(const gj_batch* b) { return b ? b->s->S.qsize : nullptr; }
const int32_t* gj_batch_status(const gj_batch* b) { return b ? b->s->S.qstatus : nullptr; }

gj_status gj_batch_summary(gj_batch* b, int32_t q, const gj_summary** out) {
  GJ_SCOPE(b ? b->ctx : nullptr);
  if (!b || !out || q < 0 || q >= b->f->plan.nq) {
    set_error("gj_batch_summary: bad argument");
    return GJ_E_INVALID;
  }
  hipStream_t s = b->ctx->stream;
  gj_status st;
  if (!b->counters_valid) {
    b->cnt_host.assign((size_t)b->f->plan.nt * CNT_STRIDE, 0);
    if ((st = check(hipMemcpyAsync(b->cnt_host.data(), b->f->F.cnt, b->cnt_host.size() * 8, hipMemcpyDeviceToHost,
                                   s),
                    "counters")) ||
        (st = check(hipStreamSynchronize(s), "counters")))
      return st;
    b->counters_valid = true;
  }
  int64_t js = 0;
  int32_t qs = 0;
  if ((st = check(hipMemcpyAsync(&js, b->s->S.qsize + q, 8, hipMemcpyDeviceToHost, s), "join size")) ||
      (st = check(hipMemcpyAsync(&qs, b->s->S.qstatus + q, 4, hipMemcpyDeviceToHost, s), "status")) ||
      (st = check(hipStreamSynchronize(s), "join size")))
    return st;
  if (qs == GJ_E_OVERFLOW) {
    set_error("query %d: join size does not fit below 2^63-1", q);
    return GJ_E_OVERFLOW;
  }
  gj_summary* v = new gj_summary(b->ctx);
  v->f = b->f;
  v->S = b->s->S;
  v->query = q;
  v->borrowed = true;
  v->cnt_host = b->cnt_host;
  v->join_size = js;
  b->views.push_back(v);
  *out = v;
  return GJ_OK;
}

void gj_free_batch(gj_batch* b) { batch_destroy(b); }

}  // extern "C"
