// Continuous-batching job server: a FIFO queue, admission by device-memory footprint and free slots, one
// host worker per slot with its own HIP stream and workspace, so the device work of concurrently running
// jobs overlaps. Each job runs exactly the kernels and reduction order it would run alone, so its result is
// independent of the mix.
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

size_t job_footprint(const mera_shape& s, Prec prec) {
  auto dims = layer_dims(s);
  const double eb = (double)elem_bytes(prec);
  double bytes = 0;
  for (const LayerDim& L : dims) {
    const double a = L.a, b = L.b;
    // largest intermediates of one layer's derivative program: two a^6 b, three a^6, operators b^6
    double layer = eb * (2 * a * a * a * a * a * a * b + 3 * a * a * a * a * a * a + 4 * b * b * b * b * b * b);
    // split-K partial sums of the a^4 b environment reductions (up to 64 splits)
    layer += eb * 64.0 * a * a * a * a * b;
    bytes = std::max(bytes, layer);
  }
  const double chi = s.chi, chi6 = chi * chi * chi * chi * chi * chi;
  // Krylov basis (dim 4 + residual), fixed point, h~, sigma, scratch, hs/rho levels, FP64 warm starts
  bytes += eb * chi6 * (6 + 6 + 2 * (s.T + 1)) + 16.0 * chi6;
  // tensors, gradients, history (FP64)
  double params = 0;
  for (const LayerDim& L : dims) params += (double)L.a * L.a * (L.a * L.a + L.b);
  bytes += 8.0 * params * (9 + 2 * 8);
  return (size_t)(bytes * 1.1) + ((size_t)64 << 20);
}

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
  std::vector<std::thread> workers;

  void worker() {
    Ctx ctx;
    ctx.device = device;
    (void)hipSetDevice(device);
    hipStream_t st = nullptr;
    if (hipStreamCreate(&st) != hipSuccess) st = nullptr;
    ctx.stream = st;
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
      ctx.scratch.clear();
      ctx.plans->map.clear();
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

mera_status mera_server_submit(mera_server* srv, const mera_job* job, uint64_t* job_id) {
  if (!srv || !job || !job_id) return MERA_EINVAL;
  try {
    JobSpec spec = JobSpec::from_c(*job);
    const size_t fp = job_footprint(spec.shape, spec.prec);
    if (fp > srv->s.budget) return MERA_ENOMEM;
    {
      std::lock_guard<std::mutex> lk(srv->s.mu);
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
