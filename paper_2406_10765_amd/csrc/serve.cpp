// Request loop: eigen-solves of different cells admitted by slot and device footprint, run
// concurrently on per-slot streams, each advanced step by step to its tolerance.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pw.h"
#include "slots.hpp"

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Request {
  unsigned long long ticket = 0;
  pw_request r{};
  std::vector<double> tau, mode_amp, mode_phase;
  std::vector<int> mode_miller;
  double t_arrive = NAN, t_admit = NAN, t_done = NAN;
  pw_status status = PW_PENDING;
  bool done = false;
  int steps = 0, nbands = 0;
  std::vector<double> eig, resid;
  size_t plan_bytes = 0, block_bytes = 0, need = 0;
  size_t off = 0;
  long ld = 0;
  int bypassed = 0;     // times a later request was admitted ahead of this one
  std::string message;  // pw_last_error text of the failing call, or of a step the solve retried
  int retried = 0;      // steps the solve took again after a failed Cholesky test
};

// First-fit allocator over [0, size) with coalescing.
class Range {
 public:
  explicit Range(size_t size) : total_(size) { free_[0] = size; }
  bool alloc(size_t n, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n, o = it->first + n;
        free_.erase(it);
        if (rest) free_[o] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t total() const { return total_; }

 private:
  size_t total_;
  std::map<size_t, size_t> free_;
};

}  // namespace

struct pw_server_s {
  pw_server_cfg cfg{};
  int device = 0;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> queue;
  std::map<unsigned long long, std::unique_ptr<Request>> reqs;
  std::unique_ptr<Range> mem;
  std::vector<std::thread> workers;
  unsigned long long next_ticket = 1;
  bool stop = false;
  hipEvent_t start_ev = nullptr;  // recorded on the caller's stream at creation

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  void worker(int slot);
  void run(Request* q, hipStream_t stream, const pw::SlotResources* res);
  Request* admit_locked();
};

// Admission (called with the lock held): the first queued request, in arrival order, whose
// footprint fits the free arena (first-fit placement).  A request that does not fit may be passed
// by later, smaller ones, but only kMaxBypass times; after that nothing behind it is admitted until
// it fits, so a large request is delayed by a bounded amount of work and never starved.
Request* pw_server_s::admit_locked() {
  constexpr int kMaxBypass = 16;
  for (auto it = queue.begin(); it != queue.end(); ++it) {
    Request* c = *it;
    size_t off = 0;
    if (mem->alloc(c->need, &off)) {
      c->off = off;
      for (auto jt = queue.begin(); jt != it; ++jt) ++(*jt)->bypassed;
      queue.erase(it);
      return c;
    }
    if (c->bypassed >= kMaxBypass) return nullptr;
  }
  return nullptr;
}

void pw_server_s::run(Request* q, hipStream_t stream, const pw::SlotResources* res) {
  pw_request& r = q->r;
  const int nb = r.cell.nbands;
  q->eig.assign(nb, NAN);
  q->resid.assign(nb, NAN);
  q->nbands = nb;
  if (cfg.flags & PW_SERVER_DRY_RUN) {
    const int steps = r.max_steps < 3 ? r.max_steps : 3;
    std::this_thread::sleep_for(std::chrono::milliseconds(2 * steps));
    q->steps = steps;
    for (int i = 0; i < nb; ++i) {
      q->eig[i] = i;
      q->resid[i] = 0.0;
    }
    q->status = PW_OK;
    return;
  }
  unsigned char* base = static_cast<unsigned char*>(cfg.arena_dev) + q->off;
  pw_handle* h = nullptr;
  pw_status s = pw::setup_handle(&r.cell, base, q->plan_bytes, stream, res, &h);
  if (s != PW_OK) {
    q->status = s;
    q->message = std::string("pw_setup: ") + pw_last_error(nullptr);
    return;
  }
  void* X = base + q->plan_bytes;
  s = pw_random_block(h, X, nb, (int)q->ld, r.seed);
  if (s != PW_OK) {
    q->status = s;
    q->message = std::string("pw_random_block: ") + pw_last_error(h);
    pw_destroy(h);
    return;
  }
  double b = 0.0;
  s = pw_spectrum_bound(h, 20, r.seed + 1, &b);
  if (s != PW_OK) {
    q->status = s;
    q->message = std::string("pw_spectrum_bound: ") + pw_last_error(h);
    pw_destroy(h);
    return;
  }
  int steps = 0;
  const int nconv = (r.nconv > 0 && r.nconv <= nb) ? r.nconv : nb;
  s = pw_solve(h, X, nb, (int)q->ld, nconv, r.tol, r.degree, r.max_steps, b, q->eig.data(), q->resid.data(),
               &steps);
  q->steps = steps;
  q->status = s;
  const char* rmsg = nullptr;
  q->retried = pw_solve_retries(h, &rmsg);
  if (s != PW_OK)
    q->message = std::string("pw_solve: ") + pw_last_error(h);
  else if (q->retried > 0 && rmsg)
    q->message = std::string("pw_solve retried ") + rmsg;
  pw_destroy(h);
}

void pw_server_s::worker(int slot) {
  (void)hipSetDevice(device);
  hipStream_t stream = nullptr;
  pw::SlotResources res;
  bool have_res = false;
  if (!(cfg.flags & PW_SERVER_DRY_RUN)) {
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) stream = nullptr;
    if (start_ev) (void)hipStreamWaitEvent(stream, start_ev, 0);
    // one rocBLAS handle, second stream and event pair per slot, lent to each request's handle
    have_res = pw::slot_resources_create(stream, &res) == PW_OK;
  }
  for (;;) {
    Request* q = nullptr;
    {
      std::unique_lock<std::mutex> lk(mu);
      for (;;) {
        if (stop) break;
        q = admit_locked();
        if (q) break;
        cv.wait(lk);
      }
      if (!q) break;
      q->t_admit = now();
    }
    run(q, stream, have_res ? &res : nullptr);
    {
      std::lock_guard<std::mutex> lk(mu);
      mem->release(q->off, q->need);
      q->t_done = now();
      q->done = true;
    }
    cv.notify_all();
  }
  if (have_res) pw::slot_resources_destroy(&res);
  if (stream) hipStreamDestroy(stream);
}

extern "C" {

pw_status pw_server_create(const pw_server_cfg* cfg, pw_server** out) {
  if (!cfg || !out) return PW_EINVAL;
  *out = nullptr;
  if (cfg->max_slots < 1 || cfg->max_slots > 64 || !cfg->arena_dev || cfg->arena_bytes < kAlign ||
      (reinterpret_cast<uintptr_t>(cfg->arena_dev) % kAlign) || (cfg->flags & ~PW_SERVER_DRY_RUN))
    return PW_EINVAL;
  pw_server_s* s = nullptr;
  try {
    s = new pw_server_s();
    s->cfg = *cfg;
    s->t0 = std::chrono::steady_clock::now();
    s->mem.reset(new Range(cfg->arena_bytes / kAlign * kAlign));
    if (!(cfg->flags & PW_SERVER_DRY_RUN)) {
      if (hipGetDevice(&s->device) != hipSuccess ||
          hipEventCreateWithFlags(&s->start_ev, hipEventDisableTiming) != hipSuccess ||
          hipEventRecord(s->start_ev, static_cast<hipStream_t>(cfg->hip_stream)) != hipSuccess) {
        if (s->start_ev) hipEventDestroy(s->start_ev);
        delete s;
        return PW_EDEVICE;
      }
    }
    for (int i = 0; i < cfg->max_slots; ++i) s->workers.emplace_back(&pw_server_s::worker, s, i);
  } catch (...) {
    if (s) {
      {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
      }
      s->cv.notify_all();
      for (auto& t : s->workers) t.join();
      delete s;
    }
    return PW_ENOMEM;
  }
  *out = s;
  return PW_OK;
}

double pw_server_clock(const pw_server* s) { return s ? s->now() : NAN; }

pw_status pw_submit(pw_server* s, const pw_request* r, double t_arrive, unsigned long long* ticket) {
  if (!s || !r || !ticket) return PW_EINVAL;
  if (r->max_steps < 1 || r->degree < 1 || r->degree > 1000 || !(r->tol > 0.0) || r->nconv < 0) return PW_EINVAL;
  pw_info info;
  pw_status st = pw_plan(&r->cell, &info);
  if (st != PW_OK) return st;
  std::unique_ptr<Request> q;
  try {
    q.reset(new Request());
  } catch (const std::bad_alloc&) {
    return PW_ENOMEM;
  }
  q->r = *r;
  const pw_cell_desc& c = r->cell;
  q->tau.assign(c.tau, c.tau + 3 * c.natoms);
  if (c.nmodes > 0) {
    q->mode_miller.assign(c.mode_miller, c.mode_miller + 3 * c.nmodes);
    q->mode_amp.assign(c.mode_amp, c.mode_amp + c.nmodes);
    q->mode_phase.assign(c.mode_phase, c.mode_phase + c.nmodes);
  }
  q->r.cell.tau = q->tau.empty() ? nullptr : q->tau.data();
  q->r.cell.mode_miller = q->mode_miller.empty() ? nullptr : q->mode_miller.data();
  q->r.cell.mode_amp = q->mode_amp.empty() ? nullptr : q->mode_amp.data();
  q->r.cell.mode_phase = q->mode_phase.empty() ? nullptr : q->mode_phase.data();
  q->ld = (long)((info.npw + 15) / 16 * 16);
  q->plan_bytes = align_up(info.footprint_bytes);
  q->block_bytes = align_up((size_t)c.nbands * q->ld * (c.prec == PW_FP64 ? 16 : 8));
  q->need = q->plan_bytes + q->block_bytes;
  if (q->need > s->mem->total()) return PW_ENOMEM;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return PW_EINVAL;
  q->ticket = s->next_ticket++;
  q->t_arrive = std::isfinite(t_arrive) ? t_arrive : s->now();
  *ticket = q->ticket;
  s->queue.push_back(q.get());
  s->reqs[q->ticket] = std::move(q);
  s->cv.notify_all();
  return PW_OK;
}

pw_status pw_poll(pw_server* s, unsigned long long ticket, pw_result* out) {
  if (!s || !out) return PW_EINVAL;
  std::unique_ptr<Request> q;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return PW_EINVAL;
    if (!it->second->done) return PW_PENDING;
    q = std::move(it->second);
    s->reqs.erase(it);
  }
  out->status = q->status;
  out->nbands = q->nbands;
  out->steps = q->steps;
  if (out->eig && !q->eig.empty()) std::memcpy(out->eig, q->eig.data(), sizeof(double) * q->eig.size());
  if (out->resid && !q->resid.empty()) std::memcpy(out->resid, q->resid.data(), sizeof(double) * q->resid.size());
  out->t_arrive = q->t_arrive;
  out->t_admit = q->t_admit;
  out->t_done = q->t_done;
  std::snprintf(out->message, sizeof(out->message), "%s", q->message.c_str());
  out->retried = q->retried;
  return PW_OK;
}

pw_status pw_server_destroy(pw_server* s) {
  if (!s) return PW_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->queue.clear();
  }
  s->cv.notify_all();
  for (auto& t : s->workers) t.join();
  if (s->start_ev) hipEventDestroy(s->start_ev);
  delete s;
  return PW_OK;
}

}  // extern "C"
