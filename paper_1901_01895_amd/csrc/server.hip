// Serving: continuous batching of RK4IP propagation requests on one device.
//
// A worker thread owns every device resource.  Each round it
//   1. admits queued requests in arrival order while the admitted footprint
//      stays within the budget and fewer than max_active are resident
//      (creating the request's plan, uploading its field, taking the FP64
//      input power);
//   2. advances every resident request by up to steps_per_tick RK4IP steps,
//      the requests spread round-robin over n_streams streams so that their
//      kernels run concurrently on the device;
//   3. retires requests that have taken all L/h steps: FP64 output power,
//      copy back, plan freed, latency stamped, waiters woken.
// Requests keep their own plan and work fields, and the step schedule
// carries h N(A) across rounds (run_steps start/finish), so every result is
// bit-identical to a lone mmnlse_propagate of the same request.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.h"

using mmnlse::Plan;
using clk = std::chrono::steady_clock;

namespace {

struct SReq {
  uint64_t ticket = 0;
  mmnlse_config cfg{};
  std::vector<double> beta, alpha;
  std::vector<float> S, kappa;
  std::vector<unsigned char> in, out;
  int32_t dtype = MMNLSE_C64;
  size_t bytes = 0;
  int state = 0;  // 0 queued, 1 resident, 2 done
  mmnlse_status status = MMNLSE_OK;
  std::string err;
  mmnlse_t plan = nullptr;
  double2 *stage = nullptr;
  int64_t n_steps = 0, done_steps = 0;
  double p_in = 0, p_out = 0;
  clk::time_point t_submit, t_start, t_done;
};

size_t field_bytes(const SReq &r) { return (size_t)r.cfg.M * r.cfg.T * (r.dtype == MMNLSE_C128 ? 16 : 8); }

}  // namespace

struct mmnlse_server {
  int device = 0;
  size_t budget = 0;
  int max_active = 32, n_streams = 4, steps_per_tick = 8;
  std::vector<hipStream_t> streams;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<SReq *> queue;
  std::unordered_map<uint64_t, SReq *> all;
  std::vector<SReq *> active;  // worker thread only
  uint64_t next_ticket = 1;
  bool stop = false;
  size_t used = 0, peak = 0;
  int64_t submitted = 0, completed = 0, failed = 0, rounds = 0;
  std::thread worker;
};

namespace {

void req_error(SReq *r, mmnlse_status st, const std::string &msg) {
  if (r->status == MMNLSE_OK) {
    r->status = st;
    r->err = msg;
  }
}

void release(SReq *r) {
  if (r->plan) mmnlse_destroy(r->plan);
  r->plan = nullptr;
  if (r->stage) hipFree(r->stage);
  r->stage = nullptr;
}

// Create the plan, upload the field (into the plan's third work field) and
// take the input power.
void activate(SReq *r, hipStream_t st) {
  r->t_start = clk::now();
  mmnlse_status e = mmnlse_create(&r->cfg, st, &r->plan);
  if (e != MMNLSE_OK) {
    req_error(r, e, mmnlse_last_error());
    return;
  }
  Plan &pl = *r->plan->pl;
  const size_t MT = (size_t)pl.M * pl.T;
  float2 *field = pl.buf[2];
  hipError_t he;
  if (r->dtype == MMNLSE_C64) {
    he = hipMemcpyAsync(field, r->in.data(), MT * sizeof(float2), hipMemcpyHostToDevice, st);
  } else {
    he = hipMalloc(&r->stage, MT * sizeof(double2));
    if (he == hipSuccess) he = hipMemcpyAsync(r->stage, r->in.data(), MT * sizeof(double2), hipMemcpyHostToDevice, st);
    if (he == hipSuccess) he = mmnlse::launch_convert_c128_to_c64(pl, r->stage, field, MT);
  }
  if (he == hipSuccess) he = mmnlse::reduce_norms(pl, field, nullptr, MT, &r->p_in, nullptr);
  if (he != hipSuccess) {
    req_error(r, he == hipErrorOutOfMemory ? MMNLSE_E_NOMEM : MMNLSE_E_DEVICE,
              std::string("admission: ") + hipGetErrorString(he));
    return;
  }
  r->in.clear();
  r->in.shrink_to_fit();
  r->p_in *= pl.dt;
  if (!std::isfinite(r->p_in)) req_error(r, MMNLSE_E_NONFINITE, "input field is not finite");
  r->n_steps = pl.n_steps;
  r->done_steps = 0;
}

// Output power, copy back, free.
void retire(SReq *r) {
  Plan &pl = *r->plan->pl;
  const size_t MT = (size_t)pl.M * pl.T;
  float2 *field = pl.buf[2];
  hipError_t he = mmnlse::reduce_norms(pl, field, nullptr, MT, &r->p_out, nullptr);
  r->out.resize(field_bytes(*r));
  if (he == hipSuccess) {
    if (r->dtype == MMNLSE_C64) {
      he = hipMemcpyAsync(r->out.data(), field, MT * sizeof(float2), hipMemcpyDeviceToHost, pl.stream);
    } else {
      he = mmnlse::launch_convert_c64_to_c128(pl, field, r->stage, MT);
      if (he == hipSuccess)
        he = hipMemcpyAsync(r->out.data(), r->stage, MT * sizeof(double2), hipMemcpyDeviceToHost, pl.stream);
    }
  }
  if (he == hipSuccess) he = hipStreamSynchronize(pl.stream);
  if (he != hipSuccess) {
    req_error(r, MMNLSE_E_DEVICE, std::string("retire: ") + hipGetErrorString(he));
    return;
  }
  r->p_out *= pl.dt;
  if (!std::isfinite(r->p_out)) req_error(r, MMNLSE_E_NONFINITE, "result is not finite");
}

void finish(mmnlse_server *s, SReq *r) {
  release(r);
  r->t_done = clk::now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->used -= r->bytes;
    r->state = 2;
    if (r->status == MMNLSE_OK) ++s->completed;
    else ++s->failed;
  }
  s->cv_done.notify_all();
}

void worker_main(mmnlse_server *s) {
  hipSetDevice(s->device);
  size_t rr = 0;
  for (;;) {
    std::vector<SReq *> admit;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty() || !s->active.empty(); });
      if (s->stop && s->active.empty()) break;
      while (!s->stop && !s->queue.empty() && (int)(s->active.size() + admit.size()) < s->max_active &&
             s->used + s->queue.front()->bytes <= s->budget) {
        SReq *r = s->queue.front();
        s->queue.pop_front();
        s->used += r->bytes;
        s->peak = std::max(s->peak, s->used);
        r->state = 1;
        admit.push_back(r);
      }
    }
    for (SReq *r : admit) {
      activate(r, s->streams[rr++ % s->streams.size()]);
      if (r->status != MMNLSE_OK) finish(s, r);
      else s->active.push_back(r);
    }
    if (s->active.empty()) continue;
    // one scheduling round: every resident request advances, streams in parallel
    for (SReq *r : s->active) {
      Plan &pl = *r->plan->pl;
      // a round stops at a span end: the amplifier acts there and the next
      // step starts afresh, as in mmnlse_propagate
      const int64_t d = r->done_steps, sp = pl.span_steps;
      int64_t n = std::min<int64_t>(s->steps_per_tick, r->n_steps - d);
      if (sp > 0) n = std::min<int64_t>(n, sp - d % sp);
      const bool first = d == 0 || (sp > 0 && d % sp == 0);
      const bool span_end = sp > 0 && (d + n) % sp == 0;
      const bool last = d + n == r->n_steps || span_end;
      hipError_t e = mmnlse::run_steps(pl, pl.buf[2], n, pl.h, pl.E, pl.buf, nullptr, first, last);
      if (e == hipSuccess && span_end) e = mmnlse::launch_amplify(pl, pl.buf[2]);
      if (e != hipSuccess) req_error(r, MMNLSE_E_DEVICE, std::string("steps: ") + hipGetErrorString(e));
      r->done_steps += n;
    }
    for (hipStream_t st : s->streams) {
      hipError_t e = hipStreamSynchronize(st);
      if (e != hipSuccess)
        for (SReq *r : s->active)
          if (r->plan->pl->stream == st) req_error(r, MMNLSE_E_DEVICE, std::string("round: ") + hipGetErrorString(e));
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      ++s->rounds;
    }
    std::vector<SReq *> still;
    for (SReq *r : s->active) {
      if (r->status != MMNLSE_OK || r->done_steps >= r->n_steps) {
        if (r->status == MMNLSE_OK) retire(r);
        finish(s, r);
      } else {
        still.push_back(r);
      }
    }
    s->active.swap(still);
  }
}

mmnlse_status copy_config(SReq *r, const mmnlse_config *cfg) {
  r->cfg = *cfg;
  const size_t M = cfg->M;
  r->beta.assign(cfg->beta, cfg->beta + M * cfg->n_beta);
  if (cfg->alpha) r->alpha.assign(cfg->alpha, cfg->alpha + M);
  if (cfg->S) r->S.assign(cfg->S, cfg->S + M * M * M * M);
  const bool manakov = (cfg->flags & MMNLSE_KERR_MANAKOV) != 0;
  if (manakov) r->kappa.assign(cfg->kappa, cfg->kappa + M * M);
  r->cfg.beta = r->beta.empty() ? nullptr : r->beta.data();
  r->cfg.alpha = cfg->alpha ? r->alpha.data() : nullptr;
  r->cfg.S = cfg->S ? r->S.data() : nullptr;
  r->cfg.kappa = manakov ? r->kappa.data() : nullptr;
  return MMNLSE_OK;
}

mmnlse_status poll_impl(mmnlse_server *s, uint64_t ticket, void *A_out, mmnlse_stats *st, double *lat,
                        bool block) {
  SReq *r = nullptr;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) {
      mmnlse::set_last_error("unknown ticket");
      return MMNLSE_E_INVALID;
    }
    r = it->second;
    if (block) s->cv_done.wait(lk, [&] { return r->state == 2; });
    if (r->state != 2) {
      mmnlse::set_last_error("request not finished");
      return MMNLSE_E_BUSY;
    }
    s->all.erase(it);
  }
  const mmnlse_status status = r->status;
  if (status == MMNLSE_OK && A_out) std::memcpy(A_out, r->out.data(), r->out.size());
  if (st) {
    *st = mmnlse_stats{};
    st->power_in = r->p_in;
    st->power_out = r->p_out;
    st->seconds = std::chrono::duration<double>(r->t_done - r->t_start).count();
    st->steps = r->done_steps;
  }
  if (lat) *lat = std::chrono::duration<double>(r->t_done - r->t_submit).count();
  mmnlse::set_last_error(status == MMNLSE_OK ? std::string() : r->err);
  delete r;
  return status;
}

}  // namespace

extern "C" {

mmnlse_status mmnlse_server_create(const mmnlse_server_config *cfg, mmnlse_server_t *out) {
  mmnlse::set_last_error("");
  if (!cfg || !out) {
    mmnlse::set_last_error("null argument");
    return MMNLSE_E_INVALID;
  }
  *out = nullptr;
  if (cfg->max_active < 0 || cfg->n_streams < 0 || cfg->n_streams > 64 || cfg->steps_per_tick < 0) {
    mmnlse::set_last_error("negative or too large server parameter");
    return MMNLSE_E_INVALID;
  }
  mmnlse_server *s = new (std::nothrow) mmnlse_server();
  if (!s) return MMNLSE_E_NOMEM;
  hipGetDevice(&s->device);
  s->max_active = cfg->max_active ? cfg->max_active : 32;
  s->n_streams = cfg->n_streams ? cfg->n_streams : 4;
  s->steps_per_tick = cfg->steps_per_tick ? cfg->steps_per_tick : 8;
  s->budget = cfg->mem_budget_bytes;
  if (!s->budget) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      delete s;
      mmnlse::set_last_error("hipMemGetInfo failed");
      return MMNLSE_E_DEVICE;
    }
    s->budget = fr / 10 * 8;
  }
  for (int i = 0; i < s->n_streams; ++i) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (auto x : s->streams) hipStreamDestroy(x);
      delete s;
      mmnlse::set_last_error("stream creation failed");
      return MMNLSE_E_DEVICE;
    }
    s->streams.push_back(st);
  }
  s->worker = std::thread(worker_main, s);
  *out = s;
  return MMNLSE_OK;
}

mmnlse_status mmnlse_server_submit(mmnlse_server_t s, const mmnlse_config *cfg, const void *A_in, int32_t dtype,
                                   uint64_t *ticket) {
  mmnlse::set_last_error("");
  if (!s || !cfg || !A_in || !ticket) {
    mmnlse::set_last_error("null argument");
    return MMNLSE_E_INVALID;
  }
  if (dtype != MMNLSE_C64 && dtype != MMNLSE_C128) {
    mmnlse::set_last_error("unknown dtype");
    return MMNLSE_E_INVALID;
  }
  std::string why;
  const mmnlse_status v = mmnlse::validate_config(*cfg, why);
  if (v != MMNLSE_OK) {
    mmnlse::set_last_error(why);
    return v;
  }
  SReq *r = new (std::nothrow) SReq();
  if (!r) return MMNLSE_E_NOMEM;
  copy_config(r, cfg);
  r->dtype = dtype;
  const size_t fb = field_bytes(*r);
  r->in.assign((const unsigned char *)A_in, (const unsigned char *)A_in + fb);
  r->bytes = mmnlse::estimate_plan_bytes(r->cfg) + (dtype == MMNLSE_C128 ? (size_t)cfg->M * cfg->T * 16 : 0);
  r->t_submit = clk::now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (r->bytes > s->budget) {
      delete r;
      mmnlse::set_last_error("request footprint exceeds the server's memory budget");
      return MMNLSE_E_NOMEM;
    }
    r->ticket = s->next_ticket++;
    s->all[r->ticket] = r;
    s->queue.push_back(r);
    ++s->submitted;
    *ticket = r->ticket;
  }
  s->cv_work.notify_one();
  return MMNLSE_OK;
}

mmnlse_status mmnlse_server_poll(mmnlse_server_t s, uint64_t ticket, void *A_out, mmnlse_stats *st,
                                 double *latency_s) {
  if (!s) return MMNLSE_E_INVALID;
  return poll_impl(s, ticket, A_out, st, latency_s, false);
}

mmnlse_status mmnlse_server_wait(mmnlse_server_t s, uint64_t ticket, void *A_out, mmnlse_stats *st,
                                 double *latency_s) {
  if (!s) return MMNLSE_E_INVALID;
  return poll_impl(s, ticket, A_out, st, latency_s, true);
}

mmnlse_status mmnlse_server_stats(mmnlse_server_t s, mmnlse_server_counters *out) {
  if (!s || !out) return MMNLSE_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->failed = s->failed;
  out->queued = (int32_t)s->queue.size();
  int32_t resident = 0;
  for (auto &kv : s->all)
    if (kv.second->state == 1) ++resident;
  out->active = resident;
  out->admitted_bytes = s->used;
  out->peak_admitted_bytes = s->peak;
  out->rounds = s->rounds;
  return MMNLSE_OK;
}

mmnlse_status mmnlse_server_destroy(mmnlse_server_t s) {
  if (!s) return MMNLSE_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto &kv : s->all) {
    release(kv.second);
    delete kv.second;
  }
  for (auto st : s->streams) hipStreamDestroy(st);
  delete s;
  return MMNLSE_OK;
}

}  // extern "C"
