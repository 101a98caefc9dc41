// Batched filter over independent problems of uneven size, captured once
// into a HIP graph (the k-point / small-cell batching pattern of the band
// energy sum, FE governing equations section).
//
// Schedule: jobs sorted by estimated cost, assigned to nstreams streams by
// longest-processing-time-first; the capture forks the streams from the
// first one with an event and joins them back, so independent small filters
// overlap on the chip.  Each job is exactly one pawfe_cheb_filter call with
// its own workspace; the filter path enqueues kernel launches only (no
// memset, copy or allocation), which is what makes it capturable.
//
// Autotuner: per job, the column block size among {64, 128, 256} (and
// nvec when smaller) by timing a degree-3 filter of the job itself; per
// batch, the number of streams among {1, 2, 4} by timing the whole schedule
// eagerly.  A job with a fixed block size still runs one timed degree-2
// filter (its cost estimate, and the eager first launch of its kernels).
// Tuning runs write into temporary outputs, never into the jobs' Xout
// (which may alias Xin).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>
#include <string>
#include <vector>

#include "internal.h"

#define CHECK(x)                            \
  do {                                      \
    const pawfe_status st_ = (x);           \
    if (st_ != PAWFE_OK) return st_;        \
  } while (0)

struct pawfe_batch {
  std::vector<pawfe_filter_job> jobs;
  std::vector<int32_t> block, stream_of;
  std::vector<void*> ws;
  std::vector<size_t> ws_bytes;
  int32_t prec = PAWFE_FP64;
  int32_t nstreams = 1;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;   // [0] fork, [1..] joins
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

using pawfe::fail;

void release(pawfe_batch* b) {
  if (!b) return;
  if (!b->streams.empty()) (void)hipStreamSynchronize(b->streams[0]);
  (void)hipDeviceSynchronize();
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (hipEvent_t e : b->events) (void)hipEventDestroy(e);
  for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
  for (void* p : b->ws)
    if (p) (void)hipFree(p);
  delete b;
}

pawfe_status check_job(const pawfe_filter_job& j, int idx) {
  const std::string at = "job " + std::to_string(idx) + ": ";
  if (!j.op) return fail(PAWFE_EINVAL, at + "op is NULL");
  if (!j.Xin || !j.Xout || !j.lambda_in) return fail(PAWFE_EINVAL, at + "NULL buffer");
  if (j.nvec < 1 || j.ldx < j.nvec || j.ldo < j.nvec) return fail(PAWFE_EINVAL, at + "bad nvec / leading dimension");
  if (j.degree < 2) return fail(PAWFE_EINVAL, at + "Chebyshev degree must be >= 2");
  if (!(j.b0 < j.bW && j.bW < j.bU)) return fail(PAWFE_EINVAL, at + "bounds must satisfy b0 < bW < bU");
  return PAWFE_OK;
}

// time (ms) of one filter of job j with the given block into `out`, degree m
pawfe_status time_filter(const pawfe_filter_job& j, int32_t block, int32_t m, int32_t prec, void* ws,
                         size_t wsb, void* out, hipStream_t s, float* ms) {
  hipEvent_t e0, e1;
  PAWFE_HIP(hipEventCreate(&e0));
  PAWFE_HIP(hipEventCreate(&e1));
  pawfe_status st = PAWFE_OK;
  for (int rep = 0; rep < 2 && st == PAWFE_OK; ++rep) {   // first run warms caches and lazy set-up
    if (rep == 1) (void)hipEventRecord(e0, s);
    st = pawfe_cheb_filter(j.op, j.Xin, j.ldx, out, j.nvec, j.nvec, block, j.lambda_in, m, j.b0, j.bW, j.bU,
                           prec, ws, wsb, s);
  }
  (void)hipEventRecord(e1, s);
  if (hipEventSynchronize(e1) != hipSuccess && st == PAWFE_OK) st = fail(PAWFE_EHIP, "tuning run failed");
  if (st == PAWFE_OK) (void)hipEventElapsedTime(ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

// longest-processing-time-first assignment of jobs (by cost) to ns streams
std::vector<int32_t> lpt(const std::vector<double>& cost, int ns, std::vector<int>& order) {
  order.resize(cost.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<double> load(ns, 0.0);
  std::vector<int32_t> of(cost.size(), 0);
  for (int j : order) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    of[j] = k;
    load[k] += cost[j];
  }
  return of;
}

// enqueue the multi-stream schedule: fork from streams[0], jobs, join back
pawfe_status enqueue(pawfe_batch* b, const std::vector<int>& order, const std::vector<void*>& outs) {
  const int ns = b->nstreams;
  if (ns > 1) {
    PAWFE_HIP(hipEventRecord(b->events[0], b->streams[0]));
    for (int k = 1; k < ns; ++k) PAWFE_HIP(hipStreamWaitEvent(b->streams[k], b->events[0], 0));
  }
  for (int j : order) {
    const pawfe_filter_job& J = b->jobs[j];
    void* out = outs.empty() ? J.Xout : outs[j];
    const int64_t ldo = outs.empty() ? J.ldo : J.nvec;
    const pawfe_status st = pawfe_cheb_filter(J.op, J.Xin, J.ldx, out, ldo, J.nvec, b->block[j], J.lambda_in,
                                              J.degree, J.b0, J.bW, J.bU, b->prec, b->ws[j], b->ws_bytes[j],
                                              b->streams[b->stream_of[j]]);
    if (st != PAWFE_OK) return st;
  }
  if (ns > 1) {
    for (int k = 1; k < ns; ++k) {
      PAWFE_HIP(hipEventRecord(b->events[k], b->streams[k]));
      PAWFE_HIP(hipStreamWaitEvent(b->streams[0], b->events[k], 0));
    }
  }
  return PAWFE_OK;
}

pawfe_status make_streams(pawfe_batch* b, int ns) {
  while ((int)b->streams.size() < ns) {
    hipStream_t s;
    PAWFE_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));   // default priority
    b->streams.push_back(s);
  }
  while ((int)b->events.size() < ns) {
    hipEvent_t e;
    PAWFE_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    b->events.push_back(e);
  }
  return PAWFE_OK;
}

pawfe_status build(pawfe_batch* b, const pawfe_filter_job* jobs, int32_t njobs, int32_t nstreams, hipStream_t s) {
  const int n = njobs;
  b->jobs.assign(jobs, jobs + n);
  b->block.assign(n, 0);
  b->ws.assign(n, nullptr);
  b->ws_bytes.assign(n, 0);
  std::vector<double> cost(n, 0.0);
  // temporary outputs for the tuning runs (never the jobs' own Xout)
  std::vector<void*> tmp(n, nullptr);
  struct TmpGuard {
    std::vector<void*>& t;
    ~TmpGuard() {
      (void)hipDeviceSynchronize();
      for (void* p : t)
        if (p) (void)hipFree(p);
    }
  } guard{tmp};
  // every job runs eagerly at least once before the capture (a degree-2
  // filter into a temporary output), so all lazily initialized launch
  // parameters exist before capturing
  const bool tune_any = true;
  for (int j = 0; j < n; ++j) {
    const pawfe_filter_job& J = b->jobs[j];
    int64_t ndof = 0;
    if (pawfe_query(J.op, &ndof, nullptr, nullptr, nullptr, nullptr, nullptr) != PAWFE_OK)
      return fail(PAWFE_EINVAL, "job " + std::to_string(j) + ": bad operator");
    const size_t esz = J.op->cplx ? 16 : 8;   // complex (k-point) operators: complex128 columns
    if (tune_any && hipMalloc(&tmp[j], (size_t)ndof * J.nvec * esz) != hipSuccess)
      return fail(PAWFE_ENOMEM, "tuning output allocation failed");
    std::vector<int32_t> cand;
    if (J.block > 0) {
      cand.push_back(J.block);
    } else {
      for (int32_t c : {64, 128, 256})
        if (c <= J.nvec) cand.push_back(c);
      if (J.nvec < 256 && (cand.empty() || cand.back() != J.nvec)) cand.push_back((int32_t)J.nvec);
    }
    size_t wmax = 0;
    for (int32_t c : cand) {
      size_t w = 0;
      // one block state: the batch's own streams provide the overlap, the
      // filter then keeps every block of a job on the job's stream
      CHECK(pawfe_cheb_filter_workspace(J.op, std::min<int64_t>(J.nvec, c), c, b->prec, &w));
      wmax = std::max(wmax, w);
    }
    if (hipMalloc(&b->ws[j], wmax) != hipSuccess) return fail(PAWFE_ENOMEM, "batch workspace allocation failed");
    b->ws_bytes[j] = wmax;
    if (cand.size() == 1) {
      b->block[j] = cand[0];
      float ms = 0.f;
      CHECK(time_filter(J, cand[0], 2, b->prec, b->ws[j], wmax, tmp[j], s, &ms));
      cost[j] = (double)ms * (J.degree + 1) / 3.0;
      continue;
    }
    float best = 0.f;
    for (int32_t c : cand) {
      float ms = 0.f;
      CHECK(time_filter(J, c, 3, b->prec, b->ws[j], wmax, tmp[j], s, &ms));
      if (b->block[j] == 0 || ms < best) {
        best = ms;
        b->block[j] = c;
      }
    }
    // degree-3 time -> degree-m estimate (two applies at set-up, one per theta)
    cost[j] = (double)best * (J.degree + 1) / 4.0;
  }
  // number of streams: given, or the fastest of 1, 2, 4 for the whole batch
  std::vector<int> order;
  if (nstreams > 0) {
    b->nstreams = std::min(nstreams, 16);
    b->stream_of = lpt(cost, b->nstreams, order);
    CHECK(make_streams(b, b->nstreams));
  } else {
    CHECK(make_streams(b, 4));
    float best = 0.f;
    int best_ns = 1;
    hipEvent_t e0, e1;
    PAWFE_HIP(hipEventCreate(&e0));
    PAWFE_HIP(hipEventCreate(&e1));
    for (int ns : {1, 2, 4}) {
      b->nstreams = ns;
      b->stream_of = lpt(cost, ns, order);
      PAWFE_HIP(hipStreamSynchronize(b->streams[0]));
      PAWFE_HIP(hipEventRecord(e0, b->streams[0]));
      CHECK(enqueue(b, order, tmp));
      PAWFE_HIP(hipEventRecord(e1, b->streams[0]));
      PAWFE_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      PAWFE_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (ns == 1 || ms < best) {
        best = ms;
        best_ns = ns;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->nstreams = best_ns;
    b->stream_of = lpt(cost, best_ns, order);
  }
  PAWFE_HIP(hipDeviceSynchronize());
  // capture the schedule once
  PAWFE_HIP(hipStreamBeginCapture(b->streams[0], hipStreamCaptureModeRelaxed));
  const pawfe_status st = enqueue(b, order, {});
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(b->streams[0], &g);
  if (st != PAWFE_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (ec != hipSuccess || !g) return fail(PAWFE_EHIP, std::string("graph capture failed: ") + hipGetErrorString(ec));
  b->graph = g;
  PAWFE_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  return PAWFE_OK;
}

}  // namespace

extern "C" {

pawfe_status pawfe_batch_create(const pawfe_filter_job* jobs, int32_t njobs, int32_t prec, int32_t nstreams,
                                void* stream, pawfe_batch** out) {
  if (!out) return fail(PAWFE_EINVAL, "out is NULL");
  *out = nullptr;
  if (!jobs || njobs < 1) return fail(PAWFE_EINVAL, "no jobs");
  if (prec != PAWFE_FP64 && prec != PAWFE_FP32) return fail(PAWFE_EUNSUPPORTED, "batch precision must be FP64 or FP32");
  for (int j = 0; j < njobs; ++j) CHECK(check_job(jobs[j], j));
  pawfe_batch* b = new (std::nothrow) pawfe_batch;
  if (!b) return fail(PAWFE_ENOMEM, "host allocation failed");
  b->prec = prec;
  const pawfe_status st = build(b, jobs, njobs, nstreams, reinterpret_cast<hipStream_t>(stream));
  if (st != PAWFE_OK) {
    release(b);
    return st;
  }
  *out = b;
  return PAWFE_OK;
}

pawfe_status pawfe_batch_run(pawfe_batch* b, void* stream) {
  if (!b || !b->exec) return fail(PAWFE_EINVAL, "batch is NULL");
  PAWFE_HIP(hipGraphLaunch(b->exec, reinterpret_cast<hipStream_t>(stream)));
  return PAWFE_OK;
}

pawfe_status pawfe_batch_query(const pawfe_batch* b, int32_t* nstreams, int32_t* blocks, int32_t* stream_of_job) {
  if (!b) return fail(PAWFE_EINVAL, "batch is NULL");
  if (nstreams) *nstreams = b->nstreams;
  for (size_t j = 0; j < b->jobs.size(); ++j) {
    if (blocks) blocks[j] = b->block[j];
    if (stream_of_job) stream_of_job[j] = b->stream_of[j];
  }
  return PAWFE_OK;
}

void pawfe_batch_destroy(pawfe_batch* b) { release(b); }

}  // extern "C"
