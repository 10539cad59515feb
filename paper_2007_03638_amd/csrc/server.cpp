// Continuous-batching job server: a FIFO queue, admission by device-memory footprint and free slots, one
// host worker per slot with its own HIP stream and workspace, so the device work of concurrently running
// jobs overlaps. Contraction programs of concurrent jobs meet in a batcher: calls of the same program at the
// same extents are run as one sequence of grouped MFMA launches, and a sequence seen before with the same
// buffers is replayed from a captured HIP graph. Each job's operands go through exactly the kernels, tiles and
// reduction order they would alone, so its result is independent of the mix.
#include <algorithm>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

#include "common.h"
#include "mera_eval.h"
#include "network.h"
#include "optim.h"

namespace mera {

int ctx_device_of(const mera_ctx* ctx);  // capi.cpp

size_t job_footprint(const mera_shape& s, Prec prec, int krylov_dim = 0) {
  auto dims = layer_dims(s);
  const double eb = (double)elem_bytes(prec);
  double bytes = 0;
  for (const LayerDim& L : dims) {
    const double a = L.a, b = L.b;
    double layer;
    if (L.ternary) {
      // ternary derivative programs: about ten a^6 / a^4 b^2 intermediates, operators b^4
      layer = eb * (10 * a * a * a * a * a * a + 10 * a * a * a * a * b * b + 4 * b * b * b * b);
    } else {
      // largest intermediates of one layer's derivative program: two a^6 b, three a^6, operators b^6
      layer = eb * (2 * a * a * a * a * a * a * b + 3 * a * a * a * a * a * a + 4 * b * b * b * b * b * b);
      // split-K partial sums of the a^4 b environment reductions (up to 64 splits)
      layer += eb * 64.0 * a * a * a * a * b;
    }
    bytes = std::max(bytes, layer);
  }
  const double chi6 = (double)dims.back().opsize(s.chi);
  // Krylov basis (dimension + 1 vectors, residual), fixed point, h~, sigma, scratch, hs/rho levels, FP64 warm starts
  // of the last two evaluations (extrapolated starts)
  const int kdim = krylov_dim > 0 ? krylov_dim : default_krylov_dim((size_t)(eb * chi6));
  bytes += eb * chi6 * ((kdim + 2) + 6 + 2 * (s.T + 1)) + 32.0 * chi6;
  // forward activations of the transition layers, kept within the default intermediate limit
  const double act = (double)activation_cache_bytes(dims, elem_bytes(prec));
  if (act <= (double)((size_t)32 << 30)) bytes += act;
  // tensors, gradients, history, per-factor retraction scratch (FP64)
  double params = 0;
  for (const LayerDim& L : dims) params += (double)L.a * L.a * L.a * L.a + (double)L.wrows() * L.b;
  bytes += 8.0 * params * (16 + 2 * 8);
  return (size_t)(bytes * 1.1) + ((size_t)64 << 20);
}


// Groups run_program calls of concurrently running jobs. A call opens a batch keyed by (program, extents,
// precision, chunk) or joins the open batch of that key; the opener (leader) waits until every other worker
// running a job of the same shape is itself waiting in the batcher (or the batch is full, or the wait bound has
// passed), then runs the group on its own stream. By default the wait bound is a tenth of the program's estimated
// run time (its multiply-adds at kMacRate plus kLaunchSeconds per kernel launch), at most kMaxAdaptiveWait: jobs of
// one shape are usually at different points of their iterations, so most waits are lost, and a wait bounded by the
// program's own cost keeps that loss small (a fixed 2 ms wait would dominate the sub-millisecond programs of small
// chi). A configured max_wait >= 0 replaces it with a fixed bound. Stream order: the leader's stream waits for each member's
// "ready" event (recorded on the member's stream at the call), and each member's stream waits for the
// leader's "done" event afterwards, so a member continues exactly as if it had launched the work itself.
struct GroupBatcher : Batcher {
  bool grouping = true;
  bool graphs = true;
  double max_wait = -1.0;  // fixed bound (seconds) of a leader's wait for members; < 0: bound by the program's cost
  static constexpr double kWaitFraction = 0.1;
  static constexpr double kMaxAdaptiveWait = 2e-3;
  static constexpr double kMacRate = 50e12;       // multiply-adds per second of a large FP32 contraction
  static constexpr double kLaunchSeconds = 10e-6;  // host and dispatch cost of one kernel launch

  struct WorkerState {
    std::string shape;  // shape of the job being run ("" while idle)
    bool waiting = false;
    hipEvent_t ready = nullptr, done = nullptr;
  };
  struct Request {
    Ctx* ctx = nullptr;
    const std::vector<void*>* ext = nullptr;
    bool done = false;
    int status = 0;
    std::string err;
  };
  struct Batch {
    std::vector<Request*> reqs;
  };
  struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    int seen = 0;
  };

  std::mutex mu;
  std::condition_variable cv;
  std::map<const Ctx*, WorkerState> states;
  std::map<std::string, Batch*> open;
  std::map<std::string, double> est_cache;  // batch key -> estimated run time (seconds)
  std::mutex gmu;
  std::map<std::string, GraphEntry> graph_cache;
  static constexpr size_t kMaxGraphs = 4096;
  mera_server_stats stats{};

  ~GroupBatcher() override {
    (void)hipDeviceSynchronize();
    for (auto& kv : graph_cache)
      if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    for (auto& kv : states) {
      if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
      if (kv.second.done) (void)hipEventDestroy(kv.second.done);
    }
  }

  void attach(Ctx& ctx) {
    std::lock_guard<std::mutex> lk(mu);
    WorkerState& w = states[&ctx];
    MERA_HIP(hipEventCreateWithFlags(&w.ready, hipEventDisableTiming));
    MERA_HIP(hipEventCreateWithFlags(&w.done, hipEventDisableTiming));
  }
  void set_shape(const Ctx& ctx, const std::string& shape) {
    {
      std::lock_guard<std::mutex> lk(mu);
      states[&ctx].shape = shape;
    }
    cv.notify_all();
  }

  static std::string batch_key(const Program& prog, const LegDims& dims, Prec prec, int64_t chunk) {
    std::string k = prog.name + "|" + std::to_string((int)prec) + "|" + std::to_string(chunk);
    for (size_t c = 0; c < dims.size(); ++c)
      if (dims[c]) k += "," + std::to_string(c) + ":" + std::to_string(dims[c]);
    return k;
  }

  // Estimated run time of one program run: every step's multiply-adds (the product of the extents of the legs of
  // its two operands; a sliced loop covers the whole leg) at kMacRate, plus kLaunchSeconds per launch.
  static double estimate_seconds(const Program& prog, const LegDims& dims, int64_t chunk) {
    double macs = 0.0;
    for (const StepDef& s : prog.steps) {
      std::string legs = s.la + s.lb;
      std::sort(legs.begin(), legs.end());
      legs.erase(std::unique(legs.begin(), legs.end()), legs.end());
      double m = 1.0;
      for (char c : legs) m *= (double)std::max<int64_t>(1, dims[(unsigned char)c]);
      macs += m;
    }
    int64_t launches = (int64_t)prog.steps.size();
    const unsigned char L = (unsigned char)prog.slice_leg;
    if (prog.slice_leg && chunk > 0 && chunk < dims[L] && prog.loop_begin >= 0)
      launches += (int64_t)(prog.loop_end - prog.loop_begin) * (dims[L] / chunk - 1);
    return macs / kMacRate + (double)launches * kLaunchSeconds;
  }

  // true while some other worker running a job of the same shape is neither waiting nor in the batch
  bool others_coming(const Ctx* me, const Batch& b) const {
    const std::string& shape = states.at(me).shape;
    for (const auto& kv : states) {
      if (kv.first == me || kv.second.waiting || kv.second.shape.empty() || kv.second.shape != shape) continue;
      bool member = false;
      for (const Request* r : b.reqs) member = member || r->ctx == kv.first;
      if (!member) return true;
    }
    return false;
  }

  void run(Ctx& ctx, const Program& prog, const LegDims& dims, const std::vector<void*>& ext, Prec prec,
           int64_t chunk) override {
    if ((!grouping && !graphs) || !prog.batch) {
      run_group(ctx, prog, dims, {Binding{&ctx, ext}}, prec, chunk, false, nullptr);
      return;
    }
    const std::string key = batch_key(prog, dims, prec, chunk);
    Request req;
    req.ctx = &ctx;
    req.ext = &ext;
    std::unique_lock<std::mutex> lk(mu);
    WorkerState& me = states.at(&ctx);
    MERA_HIP(hipEventRecord(me.ready, ctx.stream));
    if (grouping) {
      auto it = open.find(key);
      if (it != open.end() && (int)it->second->reqs.size() < kGettMaxGroup) {
        it->second->reqs.push_back(&req);
        me.waiting = true;
        cv.notify_all();
        cv.wait(lk, [&] { return req.done; });
        me.waiting = false;
        if (req.status) throw Error((mera_status)req.status, req.err);
        return;
      }
    }
    Batch b;
    b.reqs.push_back(&req);
    const bool opened = grouping && !open.count(key);
    if (opened) open[key] = &b;
    me.waiting = true;
    cv.notify_all();
    if (opened) {
      double wait = max_wait;
      if (wait < 0) {
        auto est = est_cache.find(key);
        if (est == est_cache.end()) est = est_cache.emplace(key, estimate_seconds(prog, dims, chunk)).first;
        wait = std::min(kMaxAdaptiveWait, kWaitFraction * est->second);
      }
      const auto deadline = std::chrono::steady_clock::now() + std::chrono::duration<double>(wait);
      cv.wait_until(lk, deadline,
                    [&] { return (int)b.reqs.size() >= kGettMaxGroup || !others_coming(&ctx, b); });
      open.erase(key);
    }
    stats.batches += 1;
    stats.bindings += (int64_t)b.reqs.size();
    if (b.reqs.size() > 1) stats.grouped_batches += 1;
    lk.unlock();

    int status = 0;
    std::string err;
    try {
      execute(ctx, prog, dims, b.reqs, prec, chunk, key);
    } catch (const Error& e) {
      status = e.status;
      err = e.what();
    } catch (const std::exception& e) {
      status = MERA_EINVAL;
      err = e.what();
    } catch (...) {
      status = MERA_EINVAL;
      err = "unknown error in grouped run";
    }
    lk.lock();
    for (Request* r : b.reqs)
      if (r != &req) {
        r->status = status;
        r->err = err;
        r->done = true;
      }
    me.waiting = false;
    lk.unlock();
    cv.notify_all();
    if (status) throw Error((mera_status)status, err);
  }

  void execute(Ctx& lead, const Program& prog, const LegDims& dims, const std::vector<Request*>& reqs, Prec prec,
               int64_t chunk, const std::string& key) {
    std::vector<Binding> group;
    for (Request* r : reqs) group.push_back(Binding{r->ctx, *r->ext});
    for (Request* r : reqs)
      if (r->ctx != &lead) MERA_HIP(hipStreamWaitEvent(lead.stream, states_at(r->ctx).ready, 0));
    if (graphs && !lead.profiling) {
      std::vector<const void*> touched;
      const double macs = run_group(lead, prog, dims, group, prec, chunk, true, &touched);
      std::string gk = key;
      char hex[24];
      for (const void* p : touched) {
        std::snprintf(hex, sizeof hex, "|%llx", (unsigned long long)(uintptr_t)p);
        gk += hex;
      }
      GraphEntry* ge = nullptr;
      {
        std::lock_guard<std::mutex> g(gmu);
        auto it = graph_cache.find(gk);
        if (it != graph_cache.end()) ge = &it->second;
        else if (graph_cache.size() < kMaxGraphs) ge = &graph_cache[gk];
      }
      if (ge && ge->exec) {
        MERA_HIP(hipGraphLaunch(ge->exec, lead.stream));
        for (const Binding& b : group) b.ctx->macs += macs;
        stats_add(&mera_server_stats::graph_launches);
      } else if (ge && ge->seen >= 1) {
        // second sight of the same program on the same buffers: capture it once, replay it from now on
        hipGraph_t graph = nullptr;
        MERA_HIP(hipStreamBeginCapture(lead.stream, hipStreamCaptureModeThreadLocal));
        try {
          run_group(lead, prog, dims, group, prec, chunk, false, nullptr);
        } catch (...) {
          (void)hipStreamEndCapture(lead.stream, &graph);
          if (graph) (void)hipGraphDestroy(graph);
          throw;
        }
        MERA_HIP(hipStreamEndCapture(lead.stream, &graph));
        hipGraphExec_t exec = nullptr;
        const hipError_t ie = hipGraphInstantiateWithFlags(&exec, graph, 0);
        (void)hipGraphDestroy(graph);
        MERA_HIP(ie);
        ge->exec = exec;
        MERA_HIP(hipGraphLaunch(exec, lead.stream));
        stats_add(&mera_server_stats::graph_captures);
      } else {
        if (ge) ge->seen += 1;
        run_group(lead, prog, dims, group, prec, chunk, false, nullptr);
        stats_add(&mera_server_stats::eager_runs);
      }
    } else {
      run_group(lead, prog, dims, group, prec, chunk, false, nullptr);
      stats_add(&mera_server_stats::eager_runs);
    }
    const hipEvent_t done = states_at(&lead).done;
    MERA_HIP(hipEventRecord(done, lead.stream));
    for (Request* r : reqs)
      if (r->ctx != &lead) MERA_HIP(hipStreamWaitEvent(r->ctx->stream, done, 0));
  }

  WorkerState& states_at(const Ctx* c) {
    std::lock_guard<std::mutex> lk(mu);
    return states.at(c);
  }
  void stats_add(int64_t mera_server_stats::*field) {
    std::lock_guard<std::mutex> lk(mu);
    stats.*field += 1;
  }
};

struct Server {
  int device = 0;
  size_t budget = 0;
  int max_slots = 1;
  std::mutex mu;
  std::condition_variable cv;
  struct Entry {
    JobSpec spec;
    size_t footprint = 0;
    bool finished = false;
    int error = 0;
    mera_result res{};
    std::chrono::steady_clock::time_point submitted;
  };
  std::map<uint64_t, Entry> jobs;
  std::deque<uint64_t> queue;
  size_t in_use = 0;
  uint64_t next_id = 1;
  bool stop = false;
  bool started = false;  // a job has been submitted (configuration is frozen)
  GroupBatcher batcher;
  std::shared_ptr<PlanCache> plans = std::make_shared<PlanCache>();
  std::vector<std::thread> workers;

  void worker() {
    Ctx ctx;
    ctx.device = device;
    (void)hipSetDevice(device);
    hipStream_t st = nullptr;
    // non-blocking: no implicit ordering with the legacy null stream, so stream capture on one worker cannot be
    // invalidated by another thread's null-stream work
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
    ctx.stream = st;
    ctx.plans = plans;
    ctx.batcher = &batcher;
    batcher.attach(ctx);
    for (;;) {
      uint64_t id = 0;
      JobSpec spec;
      size_t fp = 0;
      std::chrono::steady_clock::time_point sub;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] {
          return stop || (!queue.empty() && in_use + jobs[queue.front()].footprint <= budget);
        });
        if (stop) break;
        id = queue.front();
        queue.pop_front();
        Entry& e = jobs[id];
        fp = e.footprint;
        in_use += fp;
        spec = e.spec;
        sub = e.submitted;
      }
      mera_result res{};
      int err = 0;
      const auto t0 = std::chrono::steady_clock::now();
      batcher.set_shape(ctx, std::to_string(spec.shape.T) + "/" + std::to_string(spec.shape.d) + "/" +
                                 std::to_string(spec.shape.chi) + "/" + std::to_string((int)spec.prec));
      try {
        OptResult r = optimize(ctx, spec, nullptr, 0);
        res.energy = r.energy;
        res.gnorm = r.gnorm;
        res.iterations = r.iterations;
        res.evaluations = r.evaluations;
        res.status = r.status;
        res.polish_iter = r.polish_iter;
        res.macs = r.macs;
        res.krylov_applications = r.krylov_apps;
      } catch (const Error& e) {
        err = e.status;
        res.status = e.status;
      } catch (...) {
        err = MERA_EINVAL;
        res.status = MERA_EINVAL;
      }
      const auto t1 = std::chrono::steady_clock::now();
      res.seconds = std::chrono::duration<double>(t1 - t0).count();
      res.queued_seconds = std::chrono::duration<double>(t0 - sub).count();
      // release this job's workspace so the next job's footprint accounting holds
      try {
        ctx.sync();
      } catch (...) {
      }
      batcher.set_shape(ctx, "");
      ctx.scratch.clear();
      {
        std::lock_guard<std::mutex> lk(mu);
        Entry& e = jobs[id];
        e.finished = true;
        e.error = err;
        e.res = res;
        in_use -= fp;
      }
      cv.notify_all();
    }
    if (st) (void)hipStreamDestroy(st);
  }
};

}  // namespace mera

struct mera_server {
  mera::Server s;
};

using namespace mera;

extern "C" {

size_t mera_job_footprint(const mera_shape* shape, mera_prec prec) {
  if (!shape) return 0;
  try {
    return job_footprint(*shape, prec == MERA_FP64 ? Prec::F64 : Prec::F32);
  } catch (...) {
    return 0;
  }
}

mera_status mera_server_create(mera_ctx* ctx, size_t hbm_budget, int max_slots, mera_server** out) {
  if (!ctx || !out || max_slots < 1 || hbm_budget == 0) return MERA_EINVAL;
  *out = nullptr;
  try {
    auto* srv = new mera_server;
    srv->s.device = ctx_device_of(ctx);
    srv->s.budget = hbm_budget;
    srv->s.max_slots = max_slots;
    for (int i = 0; i < max_slots; ++i) srv->s.workers.emplace_back([srv] { srv->s.worker(); });
    *out = srv;
    return MERA_OK;
  } catch (...) {
    return MERA_EINVAL;
  }
}

mera_status mera_server_configure(mera_server* srv, int group_launches, int graph_capture, double max_wait_us) {
  if (!srv || std::isnan(max_wait_us)) return MERA_EINVAL;
  std::lock_guard<std::mutex> lk(srv->s.mu);
  if (srv->s.started) return MERA_EBUSY;
  srv->s.batcher.grouping = group_launches != 0;
  srv->s.batcher.graphs = graph_capture != 0;
  srv->s.batcher.max_wait = max_wait_us < 0 ? -1.0 : max_wait_us * 1e-6;
  return MERA_OK;
}

mera_status mera_server_get_stats(mera_server* srv, mera_server_stats* out) {
  if (!srv || !out) return MERA_EINVAL;
  std::lock_guard<std::mutex> lk(srv->s.batcher.mu);
  *out = srv->s.batcher.stats;
  return MERA_OK;
}

mera_status mera_server_submit(mera_server* srv, const mera_job* job, uint64_t* job_id) {
  if (!srv || !job || !job_id) return MERA_EINVAL;
  try {
    JobSpec spec = JobSpec::from_c(*job);
    // a job that may switch to FP64 polishing holds FP64 buffers from then on: admit it at that size
    const Prec peak = spec.polish_tol > 0 ? Prec::F64 : spec.prec;
    const size_t fp = job_footprint(spec.shape, peak, spec.krylov.dim);
    if (fp > srv->s.budget) return MERA_ENOMEM;
    {
      std::lock_guard<std::mutex> lk(srv->s.mu);
      srv->s.started = true;
      const uint64_t id = srv->s.next_id++;
      auto& e = srv->s.jobs[id];
      e.spec = std::move(spec);
      e.footprint = fp;
      e.submitted = std::chrono::steady_clock::now();
      srv->s.queue.push_back(id);
      *job_id = id;
    }
    srv->s.cv.notify_all();
    return MERA_OK;
  } catch (const Error& e) {
    return e.status;
  } catch (...) {
    return MERA_EINVAL;
  }
}

mera_status mera_server_poll(mera_server* srv, uint64_t job_id, mera_result* out) {
  if (!srv || !out) return MERA_EINVAL;
  std::lock_guard<std::mutex> lk(srv->s.mu);
  auto it = srv->s.jobs.find(job_id);
  if (it == srv->s.jobs.end()) return MERA_EINVAL;
  if (!it->second.finished) return MERA_EBUSY;
  *out = it->second.res;
  return it->second.error ? (mera_status)it->second.error : MERA_OK;
}

void mera_server_destroy(mera_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->s.mu);
    srv->s.stop = true;
  }
  srv->s.cv.notify_all();
  for (auto& t : srv->s.workers)
    if (t.joinable()) t.join();
  delete srv;
}

}  // extern "C"
