// Serving: continuous batching of RK4IP propagation requests on one device.
//
// Two host threads own the device work.
//   * The planner admits queued requests in arrival order while the admitted
//     footprint stays within the budget and fewer than max_active are
//     resident, and for each one creates its plan, uploads its field and
//     takes the FP64 input power, all on a stream of its own, so that plan
//     set-up never holds up the requests already running.
//   * The worker keeps every resident request moving: it launches up to
//     steps_per_tick RK4IP steps of a request on one of n_streams serving
//     streams and records an event after them; whenever a request's event has
//     completed it launches the request's next tick, or retires it once all
//     L/h steps are done (FP64 output power and copy back on a stream of the
//     worker's own that waits only on that request's event).  A request
//     never waits for the others' ticks, so short and long requests share the
//     device without a common round.
// Requests keep their own plan and work fields, and the step schedule
// carries h N(A) across ticks (run_steps start/finish), so every result is
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
  hipStream_t stream = nullptr;  // serving stream of its ticks
  hipEvent_t ev = nullptr;       // recorded after the tick in flight
  bool inflight = false;
  int64_t tick_steps = 0;        // steps of the tick in flight
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
  std::vector<hipStream_t> streams;    // serving streams (ticks)
  hipStream_t plan_stream = nullptr;   // planner: plan set-up, upload, input power
  hipStream_t retire_stream = nullptr; // worker: output power and copy back
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_plan;
  std::deque<SReq *> queue;            // submitted, not yet admitted
  std::deque<SReq *> ready;            // planned by the planner, not yet taken by the worker
  std::unordered_map<uint64_t, SReq *> all;
  std::vector<SReq *> active;          // worker thread only
  uint64_t next_ticket = 1;
  bool stop = false, planner_done = false;
  int resident = 0;                    // admitted and not finished
  size_t used = 0, peak = 0;
  int64_t submitted = 0, completed = 0, failed = 0, rounds = 0;
  size_t rr = 0;                       // planner: next serving stream
  std::thread planner, worker;
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
  if (r->ev) hipEventDestroy(r->ev);
  r->ev = nullptr;
}

// Create the plan, upload the field (into the plan's third work field) and
// take the input power, on stream st (synchronised before returning).
void activate(SReq *r, hipStream_t st) {
  r->t_start = clk::now();
  if (hipEventCreateWithFlags(&r->ev, hipEventDisableTiming) != hipSuccess) {
    req_error(r, MMNLSE_E_DEVICE, "event creation failed");
    return;
  }
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

// Output power and copy back on stream st, after the request's last tick
// (its event); synchronises st.
void retire(SReq *r, hipStream_t st) {
  Plan &pl = *r->plan->pl;
  pl.stream = st;
  if (hipStreamWaitEvent(st, r->ev, 0) != hipSuccess) {
    req_error(r, MMNLSE_E_DEVICE, "retire: stream wait failed");
    return;
  }
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
    --s->resident;
    r->state = 2;
    if (r->status == MMNLSE_OK) ++s->completed;
    else ++s->failed;
  }
  s->cv_done.notify_all();
  s->cv_plan.notify_one();
}

void planner_main(mmnlse_server *s) {
  hipSetDevice(s->device);
  for (;;) {
    SReq *r = nullptr;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_plan.wait(lk, [&] {
        return s->stop || (!s->queue.empty() && s->resident < s->max_active &&
                           s->used + s->queue.front()->bytes <= s->budget);
      });
      if (s->stop) {
        s->planner_done = true;
        break;
      }
      r = s->queue.front();
      s->queue.pop_front();
      s->used += r->bytes;
      s->peak = std::max(s->peak, s->used);
      ++s->resident;
      r->state = 1;
      r->stream = s->streams[s->rr++ % s->streams.size()];
    }
    activate(r, s->plan_stream);
    if (r->plan) r->plan->pl->stream = r->stream;  // its ticks run on the serving stream
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->ready.push_back(r);
    }
    s->cv_work.notify_one();
  }
  s->cv_work.notify_one();
}

// Launch the next tick of r on its stream (up to steps_per_tick steps, cut at
// a span end, where the amplifier acts and the next step starts afresh, as
// in mmnlse_propagate) and record its event.
void launch_tick(mmnlse_server *s, SReq *r) {
  Plan &pl = *r->plan->pl;
  const int64_t d = r->done_steps, sp = pl.span_steps;
  int64_t n = std::min<int64_t>(s->steps_per_tick, r->n_steps - d);
  if (sp > 0) n = std::min<int64_t>(n, sp - d % sp);
  const bool first = d == 0 || (sp > 0 && d % sp == 0);
  const bool span_end = sp > 0 && (d + n) % sp == 0;
  const bool last = d + n == r->n_steps || span_end;
  hipError_t e = mmnlse::run_steps(pl, pl.buf[2], n, pl.h, pl.E, pl.buf, nullptr, first, last);
  if (e == hipSuccess && span_end) e = mmnlse::launch_amplify(pl, pl.buf[2]);
  if (e == hipSuccess) e = hipEventRecord(r->ev, pl.stream);
  if (e != hipSuccess) {
    req_error(r, MMNLSE_E_DEVICE, std::string("steps: ") + hipGetErrorString(e));
    return;
  }
  r->tick_steps = n;
  r->inflight = true;
}

void worker_main(mmnlse_server *s) {
  hipSetDevice(s->device);
  for (;;) {
    std::vector<SReq *> fresh;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->active.empty())
        s->cv_work.wait(lk, [&] { return !s->ready.empty() || (s->stop && s->planner_done); });
      if (s->active.empty() && s->ready.empty() && s->stop && s->planner_done) break;
      fresh.assign(s->ready.begin(), s->ready.end());
      s->ready.clear();
    }
    for (SReq *r : fresh) {
      if (r->status != MMNLSE_OK) finish(s, r);
      else s->active.push_back(r);
    }
    bool progressed = !fresh.empty();
    int64_t ticks = 0;
    std::vector<SReq *> still;
    for (SReq *r : s->active) {
      if (r->inflight) {
        const hipError_t q = hipEventQuery(r->ev);
        if (q == hipErrorNotReady) {
          still.push_back(r);
          continue;
        }
        r->inflight = false;
        progressed = true;
        if (q != hipSuccess) req_error(r, MMNLSE_E_DEVICE, std::string("tick: ") + hipGetErrorString(q));
        else r->done_steps += r->tick_steps;
      }
      if (r->status != MMNLSE_OK || r->done_steps >= r->n_steps) {
        if (r->status == MMNLSE_OK) retire(r, s->retire_stream);
        finish(s, r);
        continue;
      }
      launch_tick(s, r);
      ++ticks;
      still.push_back(r);
    }
    s->active.swap(still);
    if (ticks) {
      std::lock_guard<std::mutex> lk(s->mu);
      s->rounds += ticks;
    }
    // nothing finished: give the device a moment before polling again
    if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
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
  for (int i = 0; i < s->n_streams + 2; ++i) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (auto x : s->streams) hipStreamDestroy(x);
      delete s;
      mmnlse::set_last_error("stream creation failed");
      return MMNLSE_E_DEVICE;
    }
    s->streams.push_back(st);
  }
  s->retire_stream = s->streams.back();
  s->streams.pop_back();
  s->plan_stream = s->streams.back();
  s->streams.pop_back();
  s->worker = std::thread(worker_main, s);
  s->planner = std::thread(planner_main, s);
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
  s->cv_plan.notify_one();
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
  // the planner stops admitting; the worker runs what is resident to the end
  s->cv_plan.notify_all();
  if (s->planner.joinable()) s->planner.join();
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto &kv : s->all) {
    release(kv.second);
    delete kv.second;
  }
  for (auto st : s->streams) hipStreamDestroy(st);
  hipStreamDestroy(s->plan_stream);
  hipStreamDestroy(s->retire_stream);
  delete s;
  return MMNLSE_OK;
}

}  // extern "C"
