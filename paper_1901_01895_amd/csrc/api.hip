// C-ABI of libmmnlse: plan creation, the RK4IP step schedule and the
// propagate / advance / component entry points declared in mmnlse.h.

#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "common.h"

namespace mmnlse {

static thread_local std::string g_err;

static mmnlse_status fail(mmnlse_status s, const std::string &msg) {
  g_err = msg;
  return s;
}

static mmnlse_status hipfail(hipError_t e, const char *what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return MMNLSE_E_DEVICE;
}

#define HIPCHK(expr, what)                          \
  do {                                              \
    hipError_t e_ = (expr);                         \
    if (e_ != hipSuccess) return hipfail(e_, what); \
  } while (0)

static int ilog2i(int64_t x) {
  int r = 0;
  while ((int64_t(1) << r) < x) ++r;
  return r;
}

// Split an FP64 complex value into FP32 hi + lo.
static inline float4 split_hilo(double re, double im) {
  const float hr = (float)re, hi = (float)im;
  return make_float4(hr, hi, (float)(re - (double)hr), (float)(im - (double)hi));
}

// Tabulate E_p(f) = exp(h/2 * L_p(w_f)) / T in the FFT's storage order;
// L_p(w) = -alpha_p/2 + i sum_n beta_{n,p} (-w)^n / n! (Eq. 1 in the
// frequency domain with the exp(-i w t) forward kernel), w_f = 2 pi fftfreq.
// device fields are accessed two samples (16 bytes) at a time
static bool misaligned(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) != 0; }
static const char *kAlign = "device field pointers must be 16-byte aligned";

static hipError_t dev_alloc(Plan &pl, void **p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes);
  if (e == hipSuccess) pl.bytes += bytes;
  return e;
}

static void free_plan(Plan *pl) {
  if (!pl) return;
  hipFree(pl->tw);
  hipFree(pl->twc);
  hipFree(pl->E);
  hipFree(pl->E2);
  hipFree(pl->Ea);
  hipFree(pl->Eb);
  hipFree(pl->beta_d);
  hipFree(pl->alpha_d);
  hipFree(pl->Sg);
  hipFree(pl->kappa);
  hipFree(pl->gain);
  hipFree(pl->Sp);
  hipFree(pl->Sph);
  hipFree(pl->Spl);
  hipFree(pl->pairs);
  hipFree(pl->tile_both);
  hipFree(pl->koff);
  hipFree(pl->passes);
  hipFree(pl->klist);
  hipFree(pl->gtiles);
  hipFree(pl->glist);
  hipFree(pl->grange);
  hipFree(pl->gkoff);
  for (auto &b : pl->buf) hipFree(b);
  for (auto &b : pl->sd) hipFree(b);
  hipFree(pl->red);
  if (pl->graph) hipGraphExecDestroy(pl->graph);
  if (pl->cap_stream) hipStreamDestroy(pl->cap_stream);
  delete pl;
}

// The RK4IP step of Eq. (6a-f) as four fused launches (eight when the FFT is
// four-step; five / nine for Kerr kernels without the fused K_23), over the
// state A and two work fields:
//   (pre)  W0 = h N(A)                                   k1 before dispersion
//   F_a    A <- D A (=A_I),  W0 <- D W0 (=k1)            Eq. 6a, 6b
//   K_23   k2 = h N(A_I + k1/2)                          Eq. 6c
//          k3 = h N(A_I + k2/2); W0 <- A_I + k3;
//          W1 <- A_I + k1/6 + k2/3 + k3/3                Eq. 6d and the 6f sum
//   F_b    W0 <- D W0,  W1 <- D W1                       Eq. 6e, 6f
//   K_4    k4 = h N(W0); A <- W1 + k4/6                  Eq. 6e, 6f
//          and, unless last, W0 = h N(A) for the next step.
// k2 and k3 only need the same sample of every mode, so both evaluations fit
// one launch; so do k4 and the next step's k1.
// passes of the iterated trapezoidal nonlinear step (SSFM-Agrawal): the first
// takes the end-point phase at z, the second from the field it reached
constexpr int kAgrawalPasses = 2;

hipError_t run_steps(Plan &pl, float2 *A, int64_t n_steps, double h, const float4 *E,
                     float2 *const *work, Prof *prof, bool start, bool finish) {
  if (n_steps <= 0) return hipSuccess;
  float2 *W0 = work[0], *W1 = work[1];
  hipError_t e;
  auto kerr = [&](const KerrLaunch &k) -> hipError_t {
    if (prof && (e = prof->record(prof->kerr, pl.stream)) != hipSuccess) return e;
    if ((e = launch_kerr(pl, h, k)) != hipSuccess) return e;
    if (prof) {
      prof->kerr_evals += ((k.stage == STAGE_K4 && k.next) || k.stage == STAGE_K23) ? 2 : 1;
      return prof->record(prof->kerr, pl.stream);
    }
    return hipSuccess;
  };
  auto linear = [&](float2 *a, float2 *b) -> hipError_t {
    if (prof && (e = prof->record(prof->lin, pl.stream)) != hipSuccess) return e;
    if ((e = launch_linear(pl, E, a, a, b, b)) != hipSuccess) return e;
    return prof ? prof->record(prof->lin, pl.stream) : hipSuccess;
  };
  KerrLaunch k{};
  // k2 and k3 from X (A_I, or the state for the split-step) and k1 in W0:
  // one fused launch where the Kerr kernel supports it, else two.
  auto stages23 = [&](float2 *X) -> hipError_t {
    k = KerrLaunch{};
    k.src0 = X;
    k.src1 = W0;
    if (kerr_fuses_k23(pl.kerr_path)) {
      k.stage = STAGE_K23;
      k.out0 = W0;
      k.out1 = W1;
      return kerr(k);
    }
    k.stage = STAGE_K2;
    k.out0 = W1;
    if ((e = kerr(k)) != hipSuccess) return e;
    k = KerrLaunch{};
    k.stage = STAGE_K3;
    k.src0 = X;
    k.src1 = W0;
    k.src2 = W1;
    k.out0 = W0;
    k.out1 = W1;
    return kerr(k);
  };
  if (pl.method == MMNLSE_SSFM_AGRAWAL) {
    // Eq. (4) with the nonlinear integral by the trapezoidal rule, the end
    // point's phase recomputed from the field reached (kAgrawalPasses passes):
    // W0 = D A(z); W1 = D[W0 exp(i g h Phi(A))]; A = D[W0 exp(i g h/2 (Phi(A) + Phi(W1)))]
    auto lin1 = [&](const float2 *in, float2 *out) -> hipError_t {
      if (prof && (e = prof->record(prof->lin, pl.stream)) != hipSuccess) return e;
      if ((e = launch_linear(pl, E, in, out, nullptr, nullptr)) != hipSuccess) return e;
      return prof ? prof->record(prof->lin, pl.stream) : hipSuccess;
    };
    auto phase = [&](const float2 *Aend, float2 *out) -> hipError_t {
      if (prof && (e = prof->record(prof->kerr, pl.stream)) != hipSuccess) return e;
      if ((e = launch_manakov_phase(pl, h, A, Aend, W0, out)) != hipSuccess) return e;
      if (prof) {
        prof->kerr_evals += 1;
        return prof->record(prof->kerr, pl.stream);
      }
      return hipSuccess;
    };
    // the last half step of a step and the first of the next one share one
    // forward transform: A(z+h) = D Y and the next W0 = D D Y (four-step plans)
    auto lin2 = [&](float2 *Y) -> hipError_t {
      if (prof && (e = prof->record(prof->lin, pl.stream)) != hipSuccess) return e;
      if ((e = launch_linear_twice(pl, E, Y, Y, W0)) != hipSuccess) return e;
      return prof ? prof->record(prof->lin, pl.stream) : hipSuccess;
    };
    // W0 = D A is carried between calls like h N(A) on the RK4IP path: a call
    // without `start` finds it left by the previous call without `finish`
    bool have_w0 = !start && pl.four_step;
    for (int64_t s = 0; s < n_steps; ++s) {
      if (!have_w0 && (e = lin1(A, W0)) != hipSuccess) return e;
      const float2 *Aend = A;  // first pass: the end-point phase taken at z
      for (int it = 0; it < kAgrawalPasses; ++it) {
        const bool last = it + 1 == kAgrawalPasses;
        float2 *out = last ? A : W1;
        if ((e = phase(Aend, out)) != hipSuccess) return e;
        have_w0 = last && pl.four_step && (s + 1 < n_steps || !finish);
        if ((e = have_w0 ? lin2(out) : lin1(out, out)) != hipSuccess) return e;
        Aend = W1;
      }
    }
    return hipSuccess;
  }
  if (pl.method == MMNLSE_SSFM_RK4) {
    // Eq. (4): D_half, RK4 over h on A' = N(A), D_half; the two half steps
    // between consecutive steps are one full step exp(h L) (table E2).
    auto one = [&](const float4 *tab) -> hipError_t {
      if (prof && (e = prof->record(prof->lin, pl.stream)) != hipSuccess) return e;
      if ((e = launch_linear(pl, tab, A, A, nullptr, nullptr)) != hipSuccess) return e;
      return prof ? prof->record(prof->lin, pl.stream) : hipSuccess;
    };
    if (start && (e = one(E)) != hipSuccess) return e;
    for (int64_t s = 0; s < n_steps; ++s) {
      k = KerrLaunch{};
      k.stage = STAGE_PLAIN;  // k1
      k.src0 = A;
      k.out0 = W0;
      if ((e = kerr(k)) != hipSuccess) return e;
      // k2 = h N(A + k1/2), k3; W0 <- A + k3, W1 <- A + k1/6 + k2/3 + k3/3
      if ((e = stages23(A)) != hipSuccess) return e;
      k = KerrLaunch{};
      k.stage = STAGE_K4;  // A <- W1 + h N(W0)/6
      k.src0 = W0;
      k.src1 = W1;
      k.out0 = A;
      k.next = 0;
      if ((e = kerr(k)) != hipSuccess) return e;
      const bool last = s + 1 == n_steps && finish;
      if ((e = one(last ? E : pl.E2)) != hipSuccess) return e;
    }
    return hipSuccess;
  }
  if (pl.solo) {  // whole steps in one launch; timed as Kerr-class work
    if (prof && (e = prof->record(prof->kerr, pl.stream)) != hipSuccess) return e;
    if ((e = launch_rk4ip_solo(pl, A, W0, n_steps, h, E, start, finish)) != hipSuccess) return e;
    if (prof) {
      prof->kerr_evals += 4 * n_steps + (start ? 1 : 0) - (finish ? 1 : 0);
      return prof->record(prof->kerr, pl.stream);
    }
    return hipSuccess;
  }
  if (start) {
    k.stage = STAGE_PLAIN;
    k.src0 = A;
    k.out0 = W0;
    if ((e = kerr(k)) != hipSuccess) return e;
  }
  for (int64_t s = 0; s < n_steps; ++s) {
    if ((e = linear(A, W0)) != hipSuccess) return e;
    if ((e = stages23(A)) != hipSuccess) return e;
    if ((e = linear(W0, W1)) != hipSuccess) return e;
    k = KerrLaunch{};
    k.stage = STAGE_K4;
    k.src0 = W0;
    k.src1 = W1;
    k.out0 = A;
    k.out1 = W0;
    k.next = (s + 1 < n_steps || !finish) ? 1 : 0;
    if ((e = kerr(k)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Launch-bound plans (a field of at most 2^20 samples: a step is 4 to 8 short
// kernels) replay their middle steps as a HIP graph of kGraphSteps steps,
// captured once per field pointer, so the host pays one launch per chunk.
// The graph holds exactly the kernels run_steps issues (no memset nodes), in
// the same order with the same arguments, so results are bit-identical to
// the eager schedule.  MMNLSE_GRAPH=0 turns it off.
constexpr int kGraphSteps = 16;

static bool graph_eligible(const Plan &pl) {
  const char *env = std::getenv("MMNLSE_GRAPH");
  if (env && env[0] == '0') return false;
  return pl.method == MMNLSE_RK4IP && !pl.solo && (size_t)pl.M * pl.T <= ((size_t)1 << 20);
}

static hipError_t capture_graph(Plan &pl, float2 *A) {
  hipError_t e;
  if (pl.graph) {
    if ((e = hipGraphExecDestroy(pl.graph)) != hipSuccess) return e;
    pl.graph = nullptr;
    pl.graph_A = nullptr;
  }
  if (!pl.cap_stream && (e = hipStreamCreateWithFlags(&pl.cap_stream, hipStreamNonBlocking)) != hipSuccess)
    return e;
  hipStream_t user = pl.stream;
  pl.stream = pl.cap_stream;  // the launch wrappers issue on pl.stream
  hipGraph_t g = nullptr;
  e = hipStreamBeginCapture(pl.cap_stream, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) {
    const hipError_t er = run_steps(pl, A, kGraphSteps, pl.h, pl.E, pl.buf, nullptr, false, false);
    e = hipStreamEndCapture(pl.cap_stream, &g);
    if (er != hipSuccess) e = er;
  }
  pl.stream = user;
  if (e == hipSuccess) e = hipGraphInstantiate(&pl.graph, g, nullptr, nullptr, 0);
  if (g) hipGraphDestroy(g);
  if (e != hipSuccess) {
    pl.graph = nullptr;
    return e;
  }
  pl.graph_A = A;
  pl.graph_steps = kGraphSteps;
  return hipSuccess;
}

// n_steps of the fixed-step schedule on A: eager, or first step, graph
// replays of the middle steps, and the remaining steps (the last one
// without the look-ahead evaluation), which is the same launch sequence.
// The graph for a field pointer is captured on the first call that passes
// it, also a short one, so that a later long call on it only replays.
static hipError_t advance_steps(Plan &pl, float2 *A, int64_t n_steps) {
  if (n_steps > 0 && graph_eligible(pl) && !pl.graph_failed && pl.graph_A != A &&
      capture_graph(pl, A) != hipSuccess) {
    (void)hipGetLastError();
    pl.graph_failed = true;
  }
  if (pl.graph_failed || pl.graph_A != A || !graph_eligible(pl) || n_steps < 2 + kGraphSteps)
    return run_steps(pl, A, n_steps, pl.h, pl.E, pl.buf);
  hipError_t e;
  const int64_t k = (n_steps - 2) / kGraphSteps, tail = n_steps - 1 - k * kGraphSteps;
  if ((e = run_steps(pl, A, 1, pl.h, pl.E, pl.buf, nullptr, true, false)) != hipSuccess) return e;
  for (int64_t i = 0; i < k; ++i)
    if ((e = hipGraphLaunch(pl.graph, pl.stream)) != hipSuccess) return e;
  return run_steps(pl, A, tail, pl.h, pl.E, pl.buf, nullptr, false, true);
}

static bool check_symmetric(const float *S, int M, double tol, std::string &why) {
  double smax = 0.0;
  const size_t n4 = (size_t)M * M * M * M;
  for (size_t i = 0; i < n4; ++i) smax = std::max(smax, (double)std::fabs(S[i]));
  const double lim = tol * (smax > 0 ? smax : 1.0);
  auto at = [&](int p, int l, int m, int n) { return (double)S[(((size_t)p * M + l) * M + m) * M + n]; };
  for (int p = 0; p < M; ++p)
    for (int l = 0; l < M; ++l)
      for (int m = 0; m < M; ++m)
        for (int n = 0; n < M; ++n) {
          const double v = at(p, l, m, n);
          if (std::fabs(v - at(p, m, l, n)) > lim) {
            why = "S is not symmetric in (l,m)";
            return false;
          }
          if (std::fabs(v - at(n, l, m, p)) > lim) {
            why = "S is not symmetric in (p,n)";
            return false;
          }
        }
  return true;
}

hipError_t setup_mfma(Plan &pl, const float *S);  // kerr_mfma.hip

// Argument checks shared by mmnlse_create and mmnlse_server_submit.
mmnlse_status validate_config(const mmnlse_config &c, std::string &why) {
  auto bad = [&](const char *m) {
    why = m;
    return MMNLSE_E_INVALID;
  };
  const int M = c.M, T = c.T;
  if (M < 1 || M > 256) return bad("M must be in [1, 256]");
  if (T < 64 || T > (1 << 20) || (T & (T - 1))) return bad("T must be a power of two in [64, 2^20]");
  if (!(c.dt_ps > 0) || !std::isfinite(c.dt_ps)) return bad("dt must be positive");
  if (c.n_beta < 0 || c.n_beta > 8) return bad("n_beta must be in [0, 8]");
  if (c.n_beta > 0 && !c.beta) return bad("beta is NULL");
  const bool manakov = (c.flags & MMNLSE_KERR_MANAKOV) != 0;
  if (manakov && !c.kappa) return bad("kappa is NULL but MMNLSE_KERR_MANAKOV is set");
  if (manakov && c.precision != MMNLSE_FP32) return bad("the Manakov form runs in FP32 only");
  if (manakov) {
    for (size_t i = 0; i < (size_t)M * M; ++i)
      if (!std::isfinite(c.kappa[i])) return bad("kappa is not finite");
  }
  if (!c.S && !manakov) return bad("S is NULL");
  if (!std::isfinite(c.gamma)) return bad("gamma must be finite");
  if (!(c.h_km > 0) || !std::isfinite(c.h_km)) return bad("h must be positive");
  if (!(c.L_km >= 0) || !std::isfinite(c.L_km)) return bad("L must be >= 0");
  const double ratio = c.L_km / c.h_km;
  if (std::fabs(ratio - std::round(ratio)) > 1e-9 * std::max(1.0, ratio)) return bad("L/h is not an integer");
  if (c.precision != MMNLSE_FP32 && c.precision != MMNLSE_SPLIT_BF16 && c.precision != MMNLSE_SPLIT_BF16_S)
    return bad("unknown precision");
  if (c.method != MMNLSE_RK4IP && c.method != MMNLSE_SSFM_RK4 && c.method != MMNLSE_SSFM_AGRAWAL)
    return bad("unknown method");
  if (c.method == MMNLSE_SSFM_AGRAWAL && !(c.flags & MMNLSE_KERR_MANAKOV))
    return bad("SSFM_AGRAWAL needs the Manakov operator (MMNLSE_KERR_MANAKOV)");
  if (c.diag_every < 0) return bad("diag_every < 0");
  if (!(c.span_km >= 0) || !std::isfinite(c.span_km)) return bad("span must be >= 0");
  if (c.span_km > 0) {
    const double per = c.span_km / c.h_km, spans = c.L_km / c.span_km;
    if (std::round(per) < 1 || std::fabs(per - std::round(per)) > 1e-9 * std::max(1.0, per))
      return bad("span/h is not a positive integer");
    if (std::fabs(spans - std::round(spans)) > 1e-9 * std::max(1.0, spans))
      return bad("L/span is not an integer");
  }
  for (int i = 0; i < M * c.n_beta; ++i)
    if (!std::isfinite(c.beta[i])) return bad("beta is not finite");
  if (c.alpha)
    for (int i = 0; i < M; ++i)
      if (!std::isfinite(c.alpha[i])) return bad("alpha is not finite");
  if (manakov) return MMNLSE_OK;
  const size_t n4 = (size_t)M * M * M * M;
  for (size_t i = 0; i < n4; ++i)
    if (!std::isfinite(c.S[i])) return bad("S is not finite");
  const bool sym = (c.flags & MMNLSE_S_SYMMETRIC) != 0;
  if (sym && !check_symmetric(c.S, M, 1e-6, why)) {
    why += " but MMNLSE_S_SYMMETRIC is set";
    return MMNLSE_E_INVALID;
  }
  if (c.precision != MMNLSE_FP32 && !sym) return bad("split-bf16 precision needs MMNLSE_S_SYMMETRIC");
  return MMNLSE_OK;
}

void set_last_error(const std::string &msg) { g_err = msg; }


size_t estimate_plan_bytes(const mmnlse_config &cfg) {
  const size_t M = (size_t)cfg.M, T = (size_t)cfg.T, MT = M * T;
  size_t b = 3 * MT * sizeof(float2) + MT * sizeof(float4) + 2 * T * sizeof(float4) + 1024 * sizeof(double2);
  if (cfg.method == MMNLSE_SSFM_RK4) b += MT * sizeof(float4);
  b += M * (size_t)std::max(0, cfg.n_beta) * sizeof(double) + (cfg.alpha ? M * sizeof(double) : 0);
  if (cfg.span_km > 0) b += M * sizeof(float);
  if (cfg.flags & MMNLSE_KERR_MANAKOV) return b + M * M * sizeof(float);
  const bool sym = (cfg.flags & MMNLSE_S_SYMMETRIC) != 0;
  const bool mfma = cfg.precision != MMNLSE_FP32 ||
                    (!(cfg.flags & MMNLSE_KERR_GENERIC) && cfg.M >= 3 && sym);
  if (mfma) {
    const size_t P = M * (M + 1) / 2, Ppad = (P + 63) / 64 * 64;
    // FP32, or bf16 hi + lo: 4 bytes per entry either way, rows padded by up to a quarter;
    // pair and offset tables
    b += (Ppad + Ppad / 4) * Ppad * 4 + Ppad * 16;
  } else {
    b += M * M * M * M * sizeof(float);
  }
  return b;
}

}  // namespace mmnlse

using namespace mmnlse;

static mmnlse_status step_doubling_delta(Plan &pl, const void *X, double *delta);

extern "C" {

const char *mmnlse_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// Host bytes the plan set-up builds in temporary tables at most: the
// twiddles, and the generic tensor copy or the packed tensor with its plan.
static size_t estimate_host_bytes(const mmnlse_config &cfg) {
  const size_t M = (size_t)cfg.M, P = M * (M + 1) / 2;
  return 2 * (size_t)cfg.T * sizeof(float4) + std::max(M * M * M * M * sizeof(float), 5 * P * P + 64 * P);
}

static mmnlse_status create_impl(const mmnlse_config *cfg, void *stream, mmnlse_t *out, Plan *&pl_out) {
  {
    std::string why;
    const mmnlse_status v = validate_config(*cfg, why);
    if (v != MMNLSE_OK) return fail(v, why);
  }
  // optional cap on the host memory of the set-up (checked before any device call)
  if (const char *lim = std::getenv("MMNLSE_HOST_BYTES_LIMIT")) {
    const double cap = std::atof(lim);
    if (cap > 0 && (double)estimate_host_bytes(*cfg) > cap)
      return fail(MMNLSE_E_NOMEM, "plan set-up needs more host memory than MMNLSE_HOST_BYTES_LIMIT allows");
  }
  const int M = cfg->M, T = cfg->T;
  const double nst = std::round(cfg->L_km / cfg->h_km);
  const size_t n4 = (size_t)M * M * M * M;
  const bool sym = (cfg->flags & MMNLSE_S_SYMMETRIC) != 0;
  Plan *pl = new (std::nothrow) Plan();
  if (!pl) return fail(MMNLSE_E_NOMEM, "host allocation");
  pl_out = pl;
  pl->M = M;
  pl->T = T;
  pl->logT = ilog2i(T);
  pl->dt = cfg->dt_ps;
  pl->h = cfg->h_km;
  pl->L = cfg->L_km;
  pl->gamma = cfg->gamma;
  pl->n_steps = (int64_t)nst;
  pl->n_beta = cfg->n_beta;
  pl->precision = cfg->precision;
  pl->method = cfg->method;
  pl->diag_every = cfg->diag_every;
  if (cfg->span_km > 0) {
    pl->span = cfg->span_km;
    pl->span_steps = (int64_t)std::round(cfg->span_km / cfg->h_km);
  }
  pl->flags = cfg->flags;
  pl->stream = (hipStream_t)stream;
  hipGetDevice(&pl->device);
  // One LDS pass per row when the row fits and there are enough rows to fill
  // the chip; otherwise the four-step FFT, whose passes spread each row over
  // many workgroups (2 * M single-pass workgroups would leave most CUs idle).
  const char *force4 = std::getenv("MMNLSE_FORCE_FOUR_STEP");
  pl->four_step = T > 16384 || (T >= 4096 && 2 * M < 128) || (force4 && force4[0] == '1' && T >= 1024);
  if (force4 && force4[0] == '0' && T <= 16384) pl->four_step = false;
  if (pl->four_step) {
    pl->N1 = 1 << (pl->logT / 2);
    pl->N2 = T / pl->N1;
  }

  // Kerr path
  const bool force_generic = (cfg->flags & MMNLSE_KERR_GENERIC) != 0;
  const char *fpath = std::getenv("MMNLSE_KERR_PATH");
  const bool manakov = (cfg->flags & MMNLSE_KERR_MANAKOV) != 0;
  if (manakov) pl->kerr_path = KERR_MANAKOV;
  else if (cfg->precision != MMNLSE_FP32) pl->kerr_path = KERR_MFMA;
  else if (force_generic) pl->kerr_path = KERR_GENERIC;
  else if (sym && M >= 3) pl->kerr_path = KERR_MFMA;
  else if (M <= 8) pl->kerr_path = KERR_SMALL;
  else pl->kerr_path = KERR_GENERIC;
  if (fpath && !force_generic && !manakov && cfg->precision == MMNLSE_FP32) {
    const int v = std::atoi(fpath);
    if (v == KERR_SMALL && M <= 8) pl->kerr_path = KERR_SMALL;
    if (v == KERR_GENERIC) pl->kerr_path = KERR_GENERIC;
    if (v == KERR_MFMA && sym) pl->kerr_path = KERR_MFMA;
  }
  // A one-mode RK4IP field of at most 2048 samples runs whole steps in one
  // workgroup (its Kerr term is pointwise): one launch per call instead of
  // four to eight per step.  Its transform is the single-pass one, so the
  // tables are built in natural bin order.  Measured per step, one
  // workgroup against the launched schedule: T = 256 5.3 vs 13.6 us, 1024
  // 10.2 vs 17.7, 2048 17.9 vs 25.8, 4096 34.7 vs 26.5 (there the eight
  // transforms per step on one CU are bound by its LDS bandwidth).
  // MMNLSE_SOLO=1 also takes T = 4096, MMNLSE_SOLO=0 turns it off.
  const char *fsolo = std::getenv("MMNLSE_SOLO");
  const int solo_max = fsolo && fsolo[0] == '1' ? 4096 : 2048;
  pl->solo = M == 1 && T >= 64 && T <= solo_max && pl->kerr_path == KERR_SMALL && pl->method == MMNLSE_RK4IP &&
             !(fsolo && fsolo[0] == '0') && !(force4 && force4[0] == '1');
  if (pl->solo) {
    pl->four_step = false;
    pl->N1 = pl->N2 = 0;
  }
  if (pl->kerr_path == KERR_GENERIC && M > 128) {
    free_plan(pl);
    return fail(MMNLSE_E_UNSUPPORTED, "generic Kerr kernel supports M <= 128 (use a symmetric S)");
  }

  hipError_t e;
  const size_t MT = (size_t)M * T;
  // twiddles
  {
    std::vector<float4> tw(T);
    for (int j = 0; j < T; ++j) {
      const double ang = -2.0 * M_PI * (double)j / (double)T;
      tw[j] = split_hilo(std::cos(ang), std::sin(ang));
    }
    if ((e = dev_alloc(*pl, (void **)&pl->tw, sizeof(float4) * T)) != hipSuccess) goto nomem;
    if ((e = hipMemcpy(pl->tw, tw.data(), sizeof(float4) * T, hipMemcpyHostToDevice)) != hipSuccess) goto dev;
    if (pl->four_step) {  // the column passes' twiddles W_T^(n2 k1), permuted into their access order
      const int N1 = pl->N1, N2 = pl->N2;
      std::vector<float4> twc(T);
      for (int cb = 0; cb < N2 / kFftCols; ++cb)
        for (int n1 = 0; n1 < N1; ++n1)
          for (int c = 0; c < kFftCols; ++c)
            twc[((size_t)cb * N1 + n1) * kFftCols + c] = tw[((size_t)(cb * kFftCols + c) * n1) & (T - 1)];
      if ((e = dev_alloc(*pl, (void **)&pl->twc, sizeof(float4) * T)) != hipSuccess) goto nomem;
      if ((e = hipMemcpy(pl->twc, twc.data(), sizeof(float4) * T, hipMemcpyHostToDevice)) != hipSuccess) goto dev;
    }
  }
  // coefficients, then the propagator tables built from them on the device
  if (cfg->n_beta) {
    const size_t nb = sizeof(double) * M * cfg->n_beta;
    if ((e = dev_alloc(*pl, (void **)&pl->beta_d, nb)) != hipSuccess) goto nomem;
    if ((e = hipMemcpy(pl->beta_d, cfg->beta, nb, hipMemcpyHostToDevice)) != hipSuccess) goto dev;
  }
  if (cfg->alpha) {
    if ((e = dev_alloc(*pl, (void **)&pl->alpha_d, sizeof(double) * M)) != hipSuccess) goto nomem;
    if ((e = hipMemcpy(pl->alpha_d, cfg->alpha, sizeof(double) * M, hipMemcpyHostToDevice)) != hipSuccess)
      goto dev;
  }
  if (pl->span_steps > 0) {  // field gain of the span-end amplifier, FP64 then rounded once
    std::vector<float> g(M);
    for (int p = 0; p < M; ++p) g[p] = (float)std::exp(0.5 * (cfg->alpha ? cfg->alpha[p] : 0.0) * pl->span);
    if ((e = dev_alloc(*pl, (void **)&pl->gain, sizeof(float) * M)) != hipSuccess) goto nomem;
    if ((e = hipMemcpy(pl->gain, g.data(), sizeof(float) * M, hipMemcpyHostToDevice)) != hipSuccess) goto dev;
  }
  if ((e = dev_alloc(*pl, (void **)&pl->E, sizeof(float4) * MT)) != hipSuccess) goto nomem;
  if ((e = launch_tabulate_E(*pl, pl->h, pl->E)) != hipSuccess) goto dev;
  if (pl->method == MMNLSE_SSFM_RK4) {
    if ((e = dev_alloc(*pl, (void **)&pl->E2, sizeof(float4) * MT)) != hipSuccess) goto nomem;
    if ((e = launch_tabulate_E(*pl, 2.0 * pl->h, pl->E2)) != hipSuccess) goto dev;
  }
  if (pl->kerr_path == KERR_MANAKOV) {
    if ((e = dev_alloc(*pl, (void **)&pl->kappa, sizeof(float) * M * M)) != hipSuccess) goto nomem;
    if ((e = hipMemcpy(pl->kappa, cfg->kappa, sizeof(float) * M * M, hipMemcpyHostToDevice)) != hipSuccess) goto dev;
  } else if (pl->kerr_path != KERR_MFMA) {
    std::vector<float> Sg(n4);
    for (int p = 0; p < M; ++p)
      for (int l = 0; l < M; ++l)
        for (int m = 0; m < M; ++m)
          for (int n = 0; n < M; ++n)
            Sg[(((size_t)p * M + n) * M + m) * M + l] = cfg->S[(((size_t)p * M + l) * M + m) * M + n];
    if ((e = dev_alloc(*pl, (void **)&pl->Sg, sizeof(float) * n4)) != hipSuccess) goto nomem;
    if ((e = hipMemcpy(pl->Sg, Sg.data(), sizeof(float) * n4, hipMemcpyHostToDevice)) != hipSuccess) goto dev;
  } else {
    if ((e = setup_mfma(*pl, cfg->S)) != hipSuccess) {
      if (e == hipErrorOutOfMemory) goto nomem;
      if (e == hipErrorNotSupported) {
        free_plan(pl);
        return fail(MMNLSE_E_UNSUPPORTED, "matrix-core Kerr path not available in this library");
      }
      goto dev;
    }
  }
  for (auto &b : pl->buf)
    if ((e = dev_alloc(*pl, (void **)&b, sizeof(float2) * MT)) != hipSuccess) goto nomem;
  pl->red_n = reduction_blocks(MT);
  if ((e = dev_alloc(*pl, (void **)&pl->red, sizeof(double2) * 1024)) != hipSuccess) goto nomem;
  if ((e = hipStreamSynchronize(pl->stream)) != hipSuccess) goto dev;  // tables ready, errors surfaced
  {
    mmnlse_ctx *c = new (std::nothrow) mmnlse_ctx{pl};
    if (!c) {
      free_plan(pl);
      return fail(MMNLSE_E_NOMEM, "host allocation");
    }
    *out = c;
  }
  return MMNLSE_OK;
nomem:
  free_plan(pl);
  (void)hipGetLastError();
  return fail(MMNLSE_E_NOMEM, "device allocation failed");
dev:
  free_plan(pl);
  return hipfail(e, "create");
}

extern "C" mmnlse_status mmnlse_create(const mmnlse_config *cfg, void *stream, mmnlse_t *out) {
  g_err.clear();
  if (!cfg || !out) return fail(MMNLSE_E_INVALID, "null argument");
  *out = nullptr;
  Plan *pl = nullptr;
  try {
    return create_impl(cfg, stream, out, pl);
  } catch (const std::bad_alloc &) {
    // host tables (twiddles, tensor copies, the contraction plan) did not fit
    if (pl && !*out) free_plan(pl);
    (void)hipGetLastError();
    return fail(MMNLSE_E_NOMEM, "host memory exhausted while building the plan's tables");
  }
}

extern "C" {

mmnlse_status mmnlse_destroy(mmnlse_t h) {
  if (!h) return MMNLSE_OK;
  if (h->pl && h->pl->stream) hipStreamSynchronize(h->pl->stream);
  else hipDeviceSynchronize();
  free_plan(h->pl);
  delete h;
  return MMNLSE_OK;
}

mmnlse_status mmnlse_advance(mmnlse_t h, void *A, int64_t n_steps) {
  g_err.clear();
  if (!h || !A) return fail(MMNLSE_E_INVALID, "null argument");
  if (n_steps < 0) return fail(MMNLSE_E_INVALID, "n_steps < 0");
  if (misaligned(A)) return fail(MMNLSE_E_INVALID, kAlign);
  Plan &pl = *h->pl;
  hipError_t e = advance_steps(pl, (float2 *)A, n_steps);
  if (e != hipSuccess) return hipfail(e, "advance");
  return MMNLSE_OK;
}

mmnlse_status mmnlse_amplify(mmnlse_t h, void *A) {
  g_err.clear();
  if (!h || !A) return fail(MMNLSE_E_INVALID, "null argument");
  Plan &pl = *h->pl;
  if (pl.span_steps <= 0) return fail(MMNLSE_E_INVALID, "the plan has no spans (span_km == 0)");
  const hipError_t e = launch_amplify(pl, (float2 *)A);
  if (e != hipSuccess) return hipfail(e, "amplify");
  return MMNLSE_OK;
}

mmnlse_status mmnlse_propagate(mmnlse_t h, const void *A_in, void *A_out, int32_t dtype, int32_t on_device,
                               mmnlse_stats *st) {
  g_err.clear();
  if (!h || !A_in || !A_out) return fail(MMNLSE_E_INVALID, "null argument");
  if (dtype != MMNLSE_C64 && dtype != MMNLSE_C128) return fail(MMNLSE_E_INVALID, "unknown dtype");
  if (on_device && (misaligned(A_in) || misaligned(A_out))) return fail(MMNLSE_E_INVALID, kAlign);
  Plan &pl = *h->pl;
  const size_t MT = (size_t)pl.M * pl.T;
  float2 *state = pl.buf[2];
  double2 *stage128 = nullptr;
  struct Guard {
    double2 *&p;
    ~Guard() { if (p) hipFree(p); }
  } guard{stage128};
  if (dtype == MMNLSE_C128 && !on_device)
    HIPCHK(hipMalloc(&stage128, sizeof(double2) * MT), "staging alloc");
  if (dtype == MMNLSE_C64) {
    if (on_device) {
      // run in place on A_out
      if (A_out != A_in)
        HIPCHK(hipMemcpyAsync(A_out, A_in, sizeof(float2) * MT, hipMemcpyDeviceToDevice, pl.stream), "copy");
      state = (float2 *)A_out;
    } else {
      HIPCHK(hipMemcpyAsync(state, A_in, sizeof(float2) * MT, hipMemcpyHostToDevice, pl.stream), "upload");
    }
  } else {
    const double2 *src = (const double2 *)A_in;
    if (!on_device) {
      HIPCHK(hipMemcpyAsync(stage128, A_in, sizeof(double2) * MT, hipMemcpyHostToDevice, pl.stream), "upload");
      src = stage128;
    }
    HIPCHK(launch_convert_c128_to_c64(pl, src, state, MT), "convert");
  }
  double p_in = 0, p_out = 0;
  HIPCHK(reduce_norms(pl, state, nullptr, MT, &p_in, nullptr), "power");
  if (!std::isfinite(p_in)) return fail(MMNLSE_E_NONFINITE, "input field is not finite");
  const auto t0 = std::chrono::steady_clock::now();
  double drift_max = 0, err_max = 0;
  int64_t points = 0;
  hipError_t e = hipSuccess;
  if (pl.diag_every > 0 || pl.span_steps > 0) {
    // chunks end at every diagnostic point (multiples of diag_every, and the
    // end) and every span end; the amplifier acts before the diagnostics
    for (int64_t done = 0; done < pl.n_steps && e == hipSuccess;) {
      int64_t c = pl.n_steps - done;
      if (pl.diag_every > 0) c = std::min<int64_t>(c, pl.diag_every - done % pl.diag_every);
      if (pl.span_steps > 0) c = std::min<int64_t>(c, pl.span_steps - done % pl.span_steps);
      if (pl.method == MMNLSE_SSFM_AGRAWAL) {
        // carry the split step's shared transform across diagnostic points
        // (not across a span end, where the amplifier changes the field)
        const bool first = done == 0 || (pl.span_steps > 0 && done % pl.span_steps == 0);
        const bool last = done + c == pl.n_steps || (pl.span_steps > 0 && (done + c) % pl.span_steps == 0);
        e = run_steps(pl, state, c, pl.h, pl.E, pl.buf, nullptr, first, last);
      } else {
        e = advance_steps(pl, state, c);
      }
      if (e != hipSuccess) break;
      done += c;
      if (pl.span_steps > 0 && done % pl.span_steps == 0 && (e = launch_amplify(pl, state)) != hipSuccess)
        break;
      if (pl.diag_every == 0 || (done % pl.diag_every != 0 && done != pl.n_steps)) continue;
      double p = 0;
      if ((e = reduce_norms(pl, state, nullptr, MT, &p, nullptr)) != hipSuccess) break;
      drift_max = std::max(drift_max, std::fabs(p / p_in - 1.0));
      if (pl.method == MMNLSE_RK4IP) {
        double d = 0;
        const mmnlse_status s2 = step_doubling_delta(pl, state, &d);
        if (s2 != MMNLSE_OK) return s2;
        err_max = std::max(err_max, d / 15.0);
      }
      ++points;
    }
  } else {
    e = advance_steps(pl, state, pl.n_steps);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(pl.stream);
  const auto t1 = std::chrono::steady_clock::now();
  if (e != hipSuccess) return hipfail(e, "steps");
  HIPCHK(reduce_norms(pl, state, nullptr, MT, &p_out, nullptr), "power");
  if (dtype == MMNLSE_C64) {
    if (!on_device)
      HIPCHK(hipMemcpyAsync(A_out, state, sizeof(float2) * MT, hipMemcpyDeviceToHost, pl.stream), "download");
  } else {
    double2 *dst = on_device ? (double2 *)A_out : stage128;
    HIPCHK(launch_convert_c64_to_c128(pl, state, dst, MT), "convert");
    if (!on_device)
      HIPCHK(hipMemcpyAsync(A_out, stage128, sizeof(double2) * MT, hipMemcpyDeviceToHost, pl.stream), "download");
  }
  HIPCHK(hipStreamSynchronize(pl.stream), "download");
  p_in *= pl.dt;
  p_out *= pl.dt;
  if (st) {
    st->power_in = p_in;
    st->power_out = p_out;
    st->seconds = std::chrono::duration<double>(t1 - t0).count();
    st->steps = pl.n_steps;
    st->power_drift_max = drift_max;
    st->local_err_max = err_max;
    st->diag_points = points;
  }
  if (!std::isfinite(p_out)) return fail(MMNLSE_E_NONFINITE, "result is not finite");
  return MMNLSE_OK;
}

mmnlse_status mmnlse_linear_half_step(mmnlse_t h, const void *X, void *Y) {
  g_err.clear();
  if (!h || !X || !Y) return fail(MMNLSE_E_INVALID, "null argument");
  if (misaligned(X) || misaligned(Y)) return fail(MMNLSE_E_INVALID, kAlign);
  Plan &pl = *h->pl;
  hipError_t e = launch_linear(pl, pl.E, (const float2 *)X, (float2 *)Y, nullptr, nullptr);
  if (e != hipSuccess) return hipfail(e, "linear");
  return MMNLSE_OK;
}

mmnlse_status mmnlse_kerr(mmnlse_t h, const void *X, void *Y) {
  g_err.clear();
  if (!h || !X || !Y) return fail(MMNLSE_E_INVALID, "null argument");
  if (X == Y) return fail(MMNLSE_E_INVALID, "Y must not alias X");
  Plan &pl = *h->pl;
  KerrLaunch k{};
  k.stage = STAGE_PLAIN;
  k.src0 = (const float2 *)X;
  k.out0 = (float2 *)Y;
  hipError_t e = launch_kerr(pl, pl.h, k);
  if (e != hipSuccess) return hipfail(e, "kerr");
  return MMNLSE_OK;
}

mmnlse_status mmnlse_power(mmnlse_t h, const void *X, double *out) {
  g_err.clear();
  if (!h || !X || !out) return fail(MMNLSE_E_INVALID, "null argument");
  Plan &pl = *h->pl;
  double s = 0;
  hipError_t e = reduce_norms(pl, (const float2 *)X, nullptr, (size_t)pl.M * pl.T, &s, nullptr);
  if (e != hipSuccess) return hipfail(e, "power");
  *out = s * pl.dt;
  return MMNLSE_OK;
}

static mmnlse_status step_doubling_delta(Plan &pl, const void *X, double *delta) {
  if (pl.method != MMNLSE_RK4IP) return fail(MMNLSE_E_UNSUPPORTED, "step doubling is implemented for RK4IP plans");
  const size_t MT = (size_t)pl.M * pl.T;
  hipError_t e;
  if (!pl.E2) {
    if ((e = dev_alloc(pl, (void **)&pl.E2, sizeof(float4) * MT)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(MMNLSE_E_NOMEM, "device allocation failed");
    }
    HIPCHK(launch_tabulate_E(pl, 2.0 * pl.h, pl.E2), "tabulate");
  }
  for (auto &b : pl.sd)
    if (!b && (e = dev_alloc(pl, (void **)&b, sizeof(float2) * MT)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(MMNLSE_E_NOMEM, "device allocation failed");
    }
  float2 *fine = pl.sd[0], *coarse = pl.sd[1];
  HIPCHK(hipMemcpyAsync(fine, X, sizeof(float2) * MT, hipMemcpyDeviceToDevice, pl.stream), "copy");
  HIPCHK(hipMemcpyAsync(coarse, X, sizeof(float2) * MT, hipMemcpyDeviceToDevice, pl.stream), "copy");
  float2 *work[2] = {pl.buf[0], pl.buf[1]};
  HIPCHK(run_steps(pl, fine, 2, pl.h, pl.E, work), "fine steps");
  HIPCHK(run_steps(pl, coarse, 1, 2.0 * pl.h, pl.E2, work), "coarse step");
  double sf = 0, sd = 0;
  HIPCHK(reduce_norms(pl, fine, coarse, MT, &sf, &sd), "norms");
  *delta = sf > 0 ? std::sqrt(sd / sf) : 0.0;
  return MMNLSE_OK;
}

mmnlse_status mmnlse_step_doubling(mmnlse_t h, const void *X, double *delta) {
  g_err.clear();
  if (!h || !X || !delta) return fail(MMNLSE_E_INVALID, "null argument");
  if (misaligned(X)) return fail(MMNLSE_E_INVALID, kAlign);
  return step_doubling_delta(*h->pl, X, delta);
}

// Step-doubling control (the paper steps with a fixed h; the exponent 1/5 is
// the fifth-order local error of RK4IP, Section 3.2): a trial of size h from z
// runs one step of h (tables for h) and two of h/2 (tables for h/2) from the
// same state, delta = ||fine - coarse|| / ||fine|| in FP64; the fine result is
// kept when delta <= tol.  The next trial is h * clamp(0.9 (tol/delta)^(1/5),
// 0.5, 2) (2 for delta == 0, 0.5 for a non-finite delta), at most h_max, cut
// to the distance left.
static double adaptive_factor(double delta, double tol) {
  if (!std::isfinite(delta)) return 0.5;
  if (delta == 0.0) return 2.0;
  return std::min(2.0, std::max(0.5, 0.9 * std::pow(tol / delta, 0.2)));
}

mmnlse_status mmnlse_propagate_adaptive(mmnlse_t h, void *A, const mmnlse_adaptive_config *ac,
                                        mmnlse_trial *log, int64_t log_cap, mmnlse_adaptive_result *res) {
  g_err.clear();
  if (!h || !A || !ac || !res) return fail(MMNLSE_E_INVALID, "null argument");
  if (log_cap < 0 || (log_cap > 0 && !log)) return fail(MMNLSE_E_INVALID, "log_cap > 0 needs a log array");
  if (misaligned(A)) return fail(MMNLSE_E_INVALID, kAlign);
  Plan &pl = *h->pl;
  if (pl.method != MMNLSE_RK4IP) return fail(MMNLSE_E_UNSUPPORTED, "adaptive stepping is implemented for RK4IP plans");
  const double L = ac->length_km, tol = ac->tol, hmin = ac->h_min_km;
  const double hmax = ac->h_max_km > 0 ? ac->h_max_km : HUGE_VAL;
  if (!(L > 0) || !std::isfinite(L)) return fail(MMNLSE_E_INVALID, "length_km must be finite and > 0");
  if (!(tol > 0) || !std::isfinite(tol)) return fail(MMNLSE_E_INVALID, "tol must be finite and > 0");
  if (!(ac->h_init_km > 0) || !std::isfinite(ac->h_init_km)) return fail(MMNLSE_E_INVALID, "h_init_km must be > 0");
  if (!(hmin >= 0) || !(ac->h_max_km >= 0)) return fail(MMNLSE_E_INVALID, "h_min_km and h_max_km must be >= 0");
  if (ac->max_trials <= 0) return fail(MMNLSE_E_INVALID, "max_trials must be > 0");
  const size_t MT = (size_t)pl.M * pl.T;
  hipError_t e;
  auto alloc = [&](void **p, size_t bytes) -> bool {
    if (*p) return true;
    if (dev_alloc(pl, p, bytes) == hipSuccess) return true;
    (void)hipGetLastError();
    return false;
  };
  if (!alloc((void **)&pl.Ea, sizeof(float4) * MT) || !alloc((void **)&pl.Eb, sizeof(float4) * MT) ||
      !alloc((void **)&pl.sd[0], sizeof(float2) * MT) || !alloc((void **)&pl.sd[1], sizeof(float2) * MT))
    return fail(MMNLSE_E_NOMEM, "device allocation failed");
  float2 *X = (float2 *)A, *fine = pl.sd[0], *coarse = pl.sd[1];
  float2 *work[2] = {pl.buf[0], pl.buf[1]};
  *res = mmnlse_adaptive_result{};
  const auto t0 = std::chrono::steady_clock::now();
  double z = 0.0, step = std::min(ac->h_init_km, hmax);
  int64_t trials = 0;
  mmnlse_status st = MMNLSE_OK;
  while (L - z > 1e-12 * L) {
    if (!(step > 0) || step < hmin) {
      st = fail(MMNLSE_E_STEP, "step size fell below h_min");
      break;
    }
    if (trials >= ac->max_trials) {
      st = fail(MMNLSE_E_STEP, "max_trials reached before the end of the fiber");
      break;
    }
    step = std::min(step, L - z);
    if (pl.Ea_h != step) {
      pl.Ea_h = 0;
      HIPCHK(launch_tabulate_E(pl, step, pl.Ea), "tabulate");
      HIPCHK(launch_tabulate_E(pl, 0.5 * step, pl.Eb), "tabulate");
      pl.Ea_h = step;
    }
    HIPCHK(hipMemcpyAsync(fine, X, sizeof(float2) * MT, hipMemcpyDeviceToDevice, pl.stream), "copy");
    HIPCHK(hipMemcpyAsync(coarse, X, sizeof(float2) * MT, hipMemcpyDeviceToDevice, pl.stream), "copy");
    HIPCHK(run_steps(pl, fine, 2, 0.5 * step, pl.Eb, work), "fine steps");
    HIPCHK(run_steps(pl, coarse, 1, step, pl.Ea, work), "coarse step");
    double sf = 0, sd = 0;
    HIPCHK(reduce_norms(pl, fine, coarse, MT, &sf, &sd), "norms");
    const double delta = sf > 0 ? std::sqrt(sd / sf) : (sd == 0 ? 0.0 : NAN);
    const bool ok = delta <= tol;
    if (trials < log_cap) log[trials] = mmnlse_trial{z, step, delta, ok ? 1 : 0, 0};
    ++trials;
    if (ok) {
      HIPCHK(hipMemcpyAsync(X, fine, sizeof(float2) * MT, hipMemcpyDeviceToDevice, pl.stream), "copy");
      z += step;
      ++res->accepted;
    } else {
      ++res->rejected;
    }
    step = std::min(hmax, step * adaptive_factor(delta, tol));
  }
  HIPCHK(hipStreamSynchronize(pl.stream), "synchronize");
  res->z_km = z;
  res->h_next_km = step;
  res->trials = trials;
  res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return st;
}

mmnlse_status mmnlse_profile(mmnlse_t h, void *A, int64_t n_steps, double *ms, int64_t *counts) {
  g_err.clear();
  if (!h || !A || !ms || !counts) return fail(MMNLSE_E_INVALID, "null argument");
  if (n_steps < 0) return fail(MMNLSE_E_INVALID, "n_steps < 0");
  if (misaligned(A)) return fail(MMNLSE_E_INVALID, kAlign);
  Plan &pl = *h->pl;
  Prof prof;
  hipError_t e = run_steps(pl, (float2 *)A, n_steps, pl.h, pl.E, pl.buf, &prof);
  if (e == hipSuccess) e = hipStreamSynchronize(pl.stream);
  double tk = 0, tl = 0;
  for (size_t i = 0; e == hipSuccess && i + 1 < prof.kerr.size(); i += 2) {
    float t = 0;
    e = hipEventElapsedTime(&t, prof.kerr[i], prof.kerr[i + 1]);
    tk += t;
  }
  for (size_t i = 0; e == hipSuccess && i + 1 < prof.lin.size(); i += 2) {
    float t = 0;
    e = hipEventElapsedTime(&t, prof.lin[i], prof.lin[i + 1]);
    tl += t;
  }
  for (auto ev : prof.kerr) hipEventDestroy(ev);
  for (auto ev : prof.lin) hipEventDestroy(ev);
  if (e != hipSuccess) return hipfail(e, "profile");
  ms[0] = tk;
  ms[1] = tl;
  counts[0] = (int64_t)prof.kerr.size() / 2;
  counts[1] = (int64_t)prof.lin.size() / 2;
  counts[2] = prof.kerr_evals;
  return MMNLSE_OK;
}

mmnlse_status mmnlse_synchronize(mmnlse_t h) {
  g_err.clear();
  if (!h) return fail(MMNLSE_E_INVALID, "null argument");
  HIPCHK(hipStreamSynchronize(h->pl->stream), "synchronize");
  return MMNLSE_OK;
}

mmnlse_status mmnlse_footprint(const mmnlse_t h, size_t *bytes) {
  if (!h || !bytes) return fail(MMNLSE_E_INVALID, "null argument");
  *bytes = h->pl->bytes;
  return MMNLSE_OK;
}

mmnlse_status mmnlse_kerr_plan(const float *S, int32_t M, int32_t precision, int32_t *counts, int32_t *perm,
                               int32_t *rows, int32_t *passes, int32_t *klist, double *entries) {
  g_err.clear();
  if (!S || !counts) return fail(MMNLSE_E_INVALID, "null argument");
  if (M < 1 || M > 256) return fail(MMNLSE_E_INVALID, "M must be in 1..256");
  if (precision != MMNLSE_FP32 && precision != MMNLSE_SPLIT_BF16 && precision != MMNLSE_SPLIT_BF16_S)
    return fail(MMNLSE_E_INVALID, "unknown precision");
  KerrPlan kp;
  try {
    plan_kerr(S, M, precision != MMNLSE_FP32, kp);
  } catch (const std::bad_alloc &) {
    return fail(MMNLSE_E_NOMEM, "host allocation");
  }
  counts[0] = kp.P;
  counts[1] = kp.Ppad;
  counts[2] = (int32_t)kp.passes.size();
  counts[3] = (int32_t)kp.klist.size();
  counts[4] = kp.kw;
  counts[5] = kp.rtm;
  counts[6] = kp.nrt;
  if (perm) std::copy(kp.cols.begin(), kp.cols.end(), perm);
  if (rows) std::copy(kp.rows.begin(), kp.rows.end(), rows);
  for (size_t i = 0; passes && i < kp.passes.size(); ++i) {
    passes[4 * i] = kp.passes[i].x;
    passes[4 * i + 1] = kp.passes[i].y;
    passes[4 * i + 2] = kp.passes[i].z;
    passes[4 * i + 3] = kp.passes[i].w;
  }
  if (klist) std::copy(kp.klist.begin(), kp.klist.end(), klist);
  if (entries)
    for (int i = 0; i < 3; ++i) entries[i] = kp.entries[i];
  return MMNLSE_OK;
}

mmnlse_status mmnlse_kerr_work(const mmnlse_t h, double *entries) {
  g_err.clear();
  if (!h || !entries) return fail(MMNLSE_E_INVALID, "null argument");
  const Plan &pl = *h->pl;
  if (pl.kerr_path != KERR_MFMA) return fail(MMNLSE_E_UNSUPPORTED, "work counts exist for the matrix-core path");
  for (int i = 0; i < 3; ++i) entries[i] = pl.kerr_entries[i];
  return MMNLSE_OK;
}

mmnlse_status mmnlse_kerr_path(const mmnlse_t h, int32_t *path) {
  if (!h || !path) return fail(MMNLSE_E_INVALID, "null argument");
  *path = h->pl->kerr_path;
  return MMNLSE_OK;
}

}  // extern "C"
