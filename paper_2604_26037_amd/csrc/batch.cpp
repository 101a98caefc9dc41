// Batched filter over independent problems of uneven size, captured once
// into a HIP graph (the k-point / small-cell batching pattern of the band
// energy sum, FE governing equations section).
//
// Schedule: jobs sorted by estimated cost and cut, in that order, into
// consecutive groups of at most a budget of kernel launches; each group is
// one captured graph, its jobs spread over nstreams streams by
// longest-processing-time-first (the capture forks the streams from the
// first one with an event and joins them back, so independent small filters
// overlap on the chip).  A replay launches the groups' graphs one after
// another.  The budget bounds the size and the longest dependency chain of
// every graph (a single graph of every filter of a large batch runs to
// 10^5 launches).  Each job is exactly one pawfe_cheb_filter call with its
// own workspace; the filter path enqueues kernel launches only (no memset,
// copy or allocation), which is what makes it capturable.
//
// Autotuner: per job, the column block size among {64, 128, 256} (and
// nvec when smaller) by timing a degree-3 filter of the job itself; per
// batch, the number of streams among {1, 2, 4} by timing the whole schedule
// eagerly.  A job with a fixed block size still runs one timed degree-2
// filter (its cost estimate, and the eager first launch of its kernels).
// Tuning runs write into temporary outputs, never into the jobs' Xout
// (which may alias Xin).
//
// Tuning cache: the decisions (block size and cost estimate per job, stream
// count per batch) are kept in a process-wide table keyed by what they
// depend on -- the GPU architecture, the operator's shape (cells, degree,
// Gauss rule, atoms and projectors, real or complex, graded / GGA), the
// column count and the precision -- and can be saved to and loaded from a
// text file (pawfe_tune_cache_save / _load).  A job found in the table is
// not timed again; it still runs one eager degree-2 filter before the
// capture, as a job with a fixed block size does.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <fstream>
#include <map>
#include <mutex>
#include <numeric>
#include <sstream>
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
  std::vector<std::vector<int>> groups;   // job indices of each graph, in launch order
  std::vector<hipGraph_t> graphs;
  std::vector<hipGraphExec_t> execs;
  int32_t ntimed = 0;   // timed filter runs (and stream-count trials) spent on tuning
};

namespace {

using pawfe::fail;

// launches per captured graph unless the caller sets another budget
constexpr int64_t kDefaultGraphLaunches = 16384;

// ---- tuning cache ---------------------------------------------------------------

struct TuneEntry {
  int32_t block = 0;   // job entries: chosen block size; batch entries: stream count
  double cost = 0.0;   // job entries: estimated ms of the job's filter
};

std::mutex g_cache_mu;
std::map<std::string, TuneEntry> g_cache;

std::string arch_name() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a(prop.gcnArchName);
  return a.substr(0, a.find(':'));
}

// what the tuning of one job depends on (no spaces: one token of the file)
std::string job_key(const pawfe_filter_job& J, int32_t prec, const std::string& arch) {
  const pawfe_op* op = J.op;
  std::ostringstream k;
  k << "job/" << arch << "/n" << op->n[0] << "x" << op->n[1] << "x" << op->n[2] << "/p" << op->p << "/q" << op->nq
    << "/a" << op->natoms << "/j" << op->npj_total << "/c" << (op->cplx ? 1 : 0) << "/g" << (op->graded ? 1 : 0)
    << "/v" << (op->gga ? 1 : 0) << "/s" << op->nsrow << "/N" << J.nvec << "/m" << J.degree << "/P" << prec;
  return k.str();
}

void release(pawfe_batch* b) {
  if (!b) return;
  if (!b->streams.empty()) (void)hipStreamSynchronize(b->streams[0]);
  (void)hipDeviceSynchronize();
  for (hipGraphExec_t e : b->execs) (void)hipGraphExecDestroy(e);
  for (hipGraph_t g : b->graphs) (void)hipGraphDestroy(g);
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

// kernel launches of one filter of job j with the given block (an upper
// bound: the step sequence of pawfe_cheb_filter, one launch per non-empty
// cell colour and atom colour; complex operators add the imaginary-term cell
// launches and the lambda duplication)
int64_t est_launches(const pawfe_filter_job& J, int32_t block) {
  const pawfe_op* op = J.op;
  int64_t nC = 0, nA = 0;
  for (int c = 0; c < op->ncolour; ++c) nC += op->colour_off[c + 1] > op->colour_off[c];
  for (int c = 0; c < op->natom_colours; ++c) nA += op->fix_colour_off[c + 1] > op->fix_colour_off[c];
  const int64_t cx = op->cplx ? 1 : 0, cell = nC * (1 + cx);
  const int64_t residual = 4 + nA + cell, step = 6 + nA + cell, final = 4 + nA;
  const int64_t per_block = residual + cx + 1 + (int64_t)(J.degree - 1) * step + final;
  return per_block * ((J.nvec + block - 1) / block);
}

// cut the jobs (by decreasing cost) into graphs of at most `budget`
// estimated launches (at least one job each) and spread each graph's jobs
// over ns streams, longest-processing-time-first
void plan(pawfe_batch* b, int ns, const std::vector<double>& cost, const std::vector<int64_t>& est,
          int64_t budget) {
  std::vector<int> order(cost.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  b->groups.clear();
  int64_t acc = 0;
  for (int j : order) {
    if (b->groups.empty() || acc + est[j] > budget) {
      b->groups.emplace_back();
      acc = 0;
    }
    b->groups.back().push_back(j);
    acc += est[j];
  }
  b->nstreams = ns;
  b->stream_of.assign(cost.size(), 0);
  for (const std::vector<int>& grp : b->groups) {
    std::vector<double> load(ns, 0.0);
    for (int j : grp) {
      const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      b->stream_of[j] = k;
      load[k] += cost[j];
    }
  }
}

// enqueue one group: fork from streams[0], its jobs, join back
pawfe_status enqueue_group(pawfe_batch* b, const std::vector<int>& grp, const std::vector<void*>& outs) {
  const int ns = b->nstreams;
  if (ns > 1) {
    PAWFE_HIP(hipEventRecord(b->events[0], b->streams[0]));
    for (int k = 1; k < ns; ++k) PAWFE_HIP(hipStreamWaitEvent(b->streams[k], b->events[0], 0));
  }
  for (int j : grp) {
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

pawfe_status build(pawfe_batch* b, const pawfe_filter_job* jobs, int32_t njobs, int32_t nstreams, int64_t budget,
                   hipStream_t s) {
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
  const std::string arch = arch_name();
  std::vector<std::string> keys(n);
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
    // One block state per job: the batch's own streams provide the overlap,
    // so every filter of a job keeps all its blocks on the job's stream.
    // Each filter call (timed candidates and the captured one) is handed
    // exactly the bytes of one state of its own block size, which is below
    // two states of that size, so the filter never forks blocks onto the
    // operator's internal streams inside a batch.  The allocation holds the
    // largest candidate's state.
    std::vector<size_t> wc(cand.size(), 0);
    size_t wmax = 0;
    for (size_t i = 0; i < cand.size(); ++i) {
      CHECK(pawfe_cheb_filter_workspace(J.op, std::min<int64_t>(J.nvec, cand[i]), cand[i], b->prec, &wc[i]));
      wmax = std::max(wmax, wc[i]);
    }
    if (hipMalloc(&b->ws[j], wmax) != hipSuccess) return fail(PAWFE_ENOMEM, "batch workspace allocation failed");
    keys[j] = job_key(J, b->prec, arch);
    TuneEntry hit;
    bool cached = false;
    if (cand.size() > 1) {
      std::lock_guard<std::mutex> lk(g_cache_mu);
      auto it = g_cache.find(keys[j]);
      if (it != g_cache.end() && std::find(cand.begin(), cand.end(), it->second.block) != cand.end()) {
        hit = it->second;
        cached = true;
      }
    }
    if (cached) {   // a tuned decision: one eager degree-2 filter of the chosen block
      const size_t i = std::find(cand.begin(), cand.end(), hit.block) - cand.begin();
      b->block[j] = hit.block;
      b->ws_bytes[j] = wc[i];
      float ms = 0.f;
      CHECK(time_filter(J, hit.block, 2, b->prec, b->ws[j], wc[i], tmp[j], s, &ms));
      cost[j] = hit.cost;
      continue;
    }
    if (cand.size() == 1) {
      b->block[j] = cand[0];
      b->ws_bytes[j] = wc[0];
      float ms = 0.f;
      CHECK(time_filter(J, cand[0], 2, b->prec, b->ws[j], wc[0], tmp[j], s, &ms));
      cost[j] = (double)ms * (J.degree + 1) / 3.0;
      continue;
    }
    float best = 0.f;
    for (size_t i = 0; i < cand.size(); ++i) {
      float ms = 0.f;
      CHECK(time_filter(J, cand[i], 3, b->prec, b->ws[j], wc[i], tmp[j], s, &ms));
      ++b->ntimed;
      if (b->block[j] == 0 || ms < best) {
        best = ms;
        b->block[j] = cand[i];
        b->ws_bytes[j] = wc[i];
      }
    }
    // degree-3 time -> degree-m estimate (two applies at set-up, one per theta)
    cost[j] = (double)best * (J.degree + 1) / 4.0;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cache[keys[j]] = TuneEntry{b->block[j], cost[j]};
  }
  std::vector<int64_t> est(n);
  for (int j = 0; j < n; ++j) est[j] = est_launches(b->jobs[j], b->block[j]);
  // number of streams: given, cached under the sorted job keys and the
  // launch budget, or the fastest of 1, 2, 4 for the whole batch
  std::string bkey = "batch/" + std::to_string(budget);
  {
    std::vector<std::string> sk(keys);
    std::sort(sk.begin(), sk.end());
    for (const std::string& k : sk) bkey += "+" + k;
  }
  if (nstreams > 0) {
    plan(b, std::min(nstreams, 16), cost, est, budget);
    CHECK(make_streams(b, b->nstreams));
  } else {
    CHECK(make_streams(b, 4));
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cache.find(bkey);
    if (it != g_cache.end() && (it->second.block == 1 || it->second.block == 2 || it->second.block == 4)) {
      plan(b, it->second.block, cost, est, budget);
      nstreams = it->second.block;
    }
  }
  if (nstreams <= 0) {
    float best = 0.f;
    int best_ns = 1;
    hipEvent_t e0, e1;
    PAWFE_HIP(hipEventCreate(&e0));
    PAWFE_HIP(hipEventCreate(&e1));
    for (int ns : {1, 2, 4}) {
      plan(b, ns, cost, est, budget);
      PAWFE_HIP(hipStreamSynchronize(b->streams[0]));
      PAWFE_HIP(hipEventRecord(e0, b->streams[0]));
      for (const std::vector<int>& grp : b->groups) CHECK(enqueue_group(b, grp, tmp));
      PAWFE_HIP(hipEventRecord(e1, b->streams[0]));
      PAWFE_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      PAWFE_HIP(hipEventElapsedTime(&ms, e0, e1));
      ++b->ntimed;
      if (ns == 1 || ms < best) {
        best = ms;
        best_ns = ns;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    plan(b, best_ns, cost, est, budget);
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cache[bkey] = TuneEntry{best_ns, 0.0};
  }
  PAWFE_HIP(hipDeviceSynchronize());
  // capture each group once
  for (const std::vector<int>& grp : b->groups) {
    PAWFE_HIP(hipStreamBeginCapture(b->streams[0], hipStreamCaptureModeRelaxed));
    const pawfe_status st = enqueue_group(b, grp, {});
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(b->streams[0], &g);
    if (st != PAWFE_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (ec != hipSuccess || !g)
      return fail(PAWFE_EHIP, std::string("graph capture failed: ") + hipGetErrorString(ec));
    b->graphs.push_back(g);
    hipGraphExec_t ex = nullptr;
    PAWFE_HIP(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
    b->execs.push_back(ex);
  }
  return PAWFE_OK;
}

}  // namespace

extern "C" {

pawfe_status pawfe_batch_create(const pawfe_filter_job* jobs, int32_t njobs, int32_t prec, int32_t nstreams,
                                int32_t max_graph_launches, void* stream, pawfe_batch** out) {
  if (!out) return fail(PAWFE_EINVAL, "out is NULL");
  *out = nullptr;
  if (!jobs || njobs < 1) return fail(PAWFE_EINVAL, "no jobs");
  if (prec != PAWFE_FP64 && prec != PAWFE_FP32) return fail(PAWFE_EUNSUPPORTED, "batch precision must be FP64 or FP32");
  for (int j = 0; j < njobs; ++j) CHECK(check_job(jobs[j], j));
  pawfe_batch* b = new (std::nothrow) pawfe_batch;
  if (!b) return fail(PAWFE_ENOMEM, "host allocation failed");
  b->prec = prec;
  const int64_t budget = max_graph_launches > 0 ? max_graph_launches : kDefaultGraphLaunches;
  const pawfe_status st = build(b, jobs, njobs, nstreams, budget, reinterpret_cast<hipStream_t>(stream));
  if (st != PAWFE_OK) {
    release(b);
    return st;
  }
  *out = b;
  return PAWFE_OK;
}

pawfe_status pawfe_batch_run(pawfe_batch* b, void* stream) {
  if (!b || b->execs.empty()) return fail(PAWFE_EINVAL, "batch is NULL");
  for (hipGraphExec_t e : b->execs) PAWFE_HIP(hipGraphLaunch(e, reinterpret_cast<hipStream_t>(stream)));
  return PAWFE_OK;
}

pawfe_status pawfe_batch_query(const pawfe_batch* b, int32_t* nstreams, int32_t* blocks, int32_t* stream_of_job,
                               int32_t* ngraphs) {
  if (!b) return fail(PAWFE_EINVAL, "batch is NULL");
  if (nstreams) *nstreams = b->nstreams;
  if (ngraphs) *ngraphs = (int32_t)b->execs.size();
  for (size_t j = 0; j < b->jobs.size(); ++j) {
    if (blocks) blocks[j] = b->block[j];
    if (stream_of_job) stream_of_job[j] = b->stream_of[j];
  }
  return PAWFE_OK;
}

void pawfe_batch_destroy(pawfe_batch* b) { release(b); }

pawfe_status pawfe_batch_tuning_runs(const pawfe_batch* b, int32_t* ntimed) {
  if (!b || !ntimed) return fail(PAWFE_EINVAL, "batch or ntimed is NULL");
  *ntimed = b->ntimed;
  return PAWFE_OK;
}

pawfe_status pawfe_tune_cache_clear(void) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  g_cache.clear();
  return PAWFE_OK;
}

pawfe_status pawfe_tune_cache_size(int64_t* nentries) {
  if (!nentries) return fail(PAWFE_EINVAL, "nentries is NULL");
  std::lock_guard<std::mutex> lk(g_cache_mu);
  *nentries = (int64_t)g_cache.size();
  return PAWFE_OK;
}

// File format: a first line "pawfe-tune-cache 1", then one entry per line:
// "<key> <block or stream count> <cost in ms>".  Entries read from the file
// replace those of the same key; lines that do not parse are an error.
pawfe_status pawfe_tune_cache_load(const char* path) {
  if (!path) return fail(PAWFE_EINVAL, "path is NULL");
  std::ifstream in(path);
  if (!in) return fail(PAWFE_EINVAL, std::string("cannot open ") + path);
  std::string line;
  if (!std::getline(in, line) || line != "pawfe-tune-cache 1") return fail(PAWFE_EINVAL, "not a pawfe tuning cache");
  std::map<std::string, TuneEntry> rd;
  while (std::getline(in, line)) {
    if (line.empty()) continue;
    std::istringstream ls(line);
    std::string key;
    TuneEntry e;
    std::string rest;
    if (!(ls >> key >> e.block >> e.cost) || (ls >> rest) || e.block < 1 || !(e.cost >= 0.0))
      return fail(PAWFE_EINVAL, "malformed tuning-cache line: " + line);
    rd[key] = e;
  }
  std::lock_guard<std::mutex> lk(g_cache_mu);
  for (auto& kv : rd) g_cache[kv.first] = kv.second;
  return PAWFE_OK;
}

pawfe_status pawfe_tune_cache_save(const char* path) {
  if (!path) return fail(PAWFE_EINVAL, "path is NULL");
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream out(tmp, std::ios::trunc);
    if (!out) return fail(PAWFE_EINVAL, std::string("cannot write ") + tmp);
    out << "pawfe-tune-cache 1\n";
    std::lock_guard<std::mutex> lk(g_cache_mu);
    out.precision(17);
    for (const auto& kv : g_cache) out << kv.first << " " << kv.second.block << " " << kv.second.cost << "\n";
    if (!out) return fail(PAWFE_EINVAL, std::string("write failed: ") + tmp);
  }
  if (std::rename(tmp.c_str(), path) != 0) return fail(PAWFE_EINVAL, std::string("cannot rename to ") + path);
  return PAWFE_OK;
}

}  // extern "C"
