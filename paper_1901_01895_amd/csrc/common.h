// Internal declarations shared by the HIP sources of libmmnlse.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "mmnlse.h"

namespace mmnlse {

// columns per workgroup in the strided (column) passes of the four-step FFT
constexpr int kFftCols = 16;

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------

// a * (w_hi + w_lo) with w = (hi.re, hi.im, lo.re, lo.im): the small lo
// product is folded in before the hi product is rounded, so the twiddle or
// propagator factor acts as if it were exact and rounding stays unbiased.
__device__ __forceinline__ float2 cmul_hilo(float2 a, float4 w) {
  float cre = a.x * w.z - a.y * w.w;
  float cim = a.x * w.w + a.y * w.z;
  float re = fmaf(a.x, w.x, fmaf(-a.y, w.y, cre));
  float im = fmaf(a.x, w.y, fmaf(a.y, w.x, cim));
  return make_float2(re, im);
}

__device__ __forceinline__ float4 conj_hilo(float4 w) { return make_float4(w.x, -w.y, w.z, -w.w); }

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// a + s*b
__device__ __forceinline__ float2 caxpy(float2 a, float s, float2 b) {
  return make_float2(fmaf(s, b.x, a.x), fmaf(s, b.y, a.y));
}
// acc + a*b (complex)
__device__ __forceinline__ float2 cfma(float2 acc, float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, acc.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, acc.y)));
}
// acc + a*conj(b)
__device__ __forceinline__ float2 cfma_conj(float2 acc, float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, fmaf(a.y, b.y, acc.x)), fmaf(a.y, b.x, fmaf(-a.x, b.y, acc.y)));
}

// ---------------------------------------------------------------------------
// host-side plan
// ---------------------------------------------------------------------------

enum KerrPath : int32_t { KERR_SMALL = 0, KERR_GENERIC = 1, KERR_MFMA = 2, KERR_MANAKOV = 3 };

// Which fields a Kerr launch reads and writes (the RK4 combinations of Eq. 6
// fused into the kernel's prologue and epilogue).
enum KerrStage : int32_t {
  // out0 = h N(src0)
  STAGE_PLAIN = 0,
  // X = src0 + src2/2 (A_I + k2/2); k3 = h N(X);
  // out0 = src0 + k3 (A_I + k3), out1 = src0 + src1/6 + src2/3 + k3/3
  STAGE_K3 = 1,
  // k4 = h N(src0) (src0 = D(A_I + k3)); A = src1 + k4/6 -> out0;
  // if `next`, out1 = h N(A) (k1 input of the following step)
  STAGE_K4 = 2,
  // X = src0 + src1/2 (A_I + k1/2); out0 = h N(X)
  STAGE_K2 = 3,
  // STAGE_K2 then STAGE_K3 in one launch (both are pointwise in t):
  // k2 = h N(src0 + src1/2), kept in out1; k3 = h N(src0 + k2/2);
  // out0 = src0 + k3, out1 = src0 + src1/6 + k2/3 + k3/3 (out0 may be src1)
  STAGE_K23 = 4,
};

// Kerr paths whose kernels implement STAGE_K23
inline bool kerr_fuses_k23(KerrPath p) { return p == KERR_MFMA || p == KERR_SMALL || p == KERR_MANAKOV; }

struct KerrLaunch {
  KerrStage stage;
  const float2 *src0, *src1, *src2;
  float2 *out0, *out1;
  int next;  // STAGE_K4: also evaluate h N(A)
};

struct Plan {
  // problem
  int M = 0, T = 0, logT = 0;
  double dt = 0, h = 0, gamma = 0, L = 0;
  int64_t n_steps = 0;
  int n_beta = 0;
  int precision = MMNLSE_FP32;
  int method = MMNLSE_RK4IP;
  int diag_every = 0;  // propagate: diagnostics every this many steps (0 = end only)
  int64_t span_steps = 0;  // steps per amplified span (0 = no amplifiers)
  double span = 0;         // span length in km
  uint32_t flags = 0;
  KerrPath kerr_path = KERR_GENERIC;
  // FFT decomposition: single pass in LDS when !four_step, else T = N1 * N2
  bool four_step = false;
  // one mode, 64 <= T <= 2048 (4096 on request), RK4IP: whole steps in one
  // workgroup (rk4ip_solo)
  bool solo = false;
  int N1 = 0, N2 = 0;
  hipStream_t stream = nullptr;
  int device = 0;

  // coefficients: host copies and the device copies the tables are built from
  double *beta_h = nullptr;   // [M][n_beta]
  double *alpha_h = nullptr;  // [M]
  double *beta_d = nullptr;   // [M][n_beta] (null when n_beta == 0)
  double *alpha_d = nullptr;  // [M] or null for no attenuation

  // device tables
  float4 *tw = nullptr;   // [T] exp(-2 pi i j / T) as FP32 hi + lo
  float4 *twc = nullptr;  // four-step: the column passes' twiddles W_T^(n2 k1) in their access
                          // order, [N2 / kFftCols][N1][kFftCols] (the same values as tw)
  float4 *E = nullptr;    // [M][T] exp(h/2 L)/T as hi + lo, in the FFT's storage order
  float4 *E2 = nullptr;   // same for step 2h, i.e. exp(h L)/T: the split-step's full
                          // linear step and the step-doubling coarse step
  // adaptive stepping (lazy): exp(h/2 L)/T for the trial step h and for h/2
  float4 *Ea = nullptr, *Eb = nullptr;
  double Ea_h = 0;        // trial step the two tables hold (0 = none)
  float *Sg = nullptr;    // generic tensor layout [p][n][m][l]
  float *kappa = nullptr; // Manakov coupling matrix [a][b]
  float *gain = nullptr;  // [M] span-end field gain exp(alpha_p span / 2) (span_steps > 0)
  // packed symmetric tensor (matrix-core path): rows r = (p<=n), cols q = (l<=m)
  int P = 0, Ppad = 0;
  int mfma_rows = 0;            // row slots of the contraction (row tiles x 32, padding included)
  float *Sp = nullptr;          // [mfma_rows][Ppad] FP32, weight 2 for l<m folded in
  uint16_t *Sph = nullptr;      // bf16 hi of Sp
  uint16_t *Spl = nullptr;      // bf16 lo of Sp - hi
  int32_t *pairs = nullptr;     // [mfma_rows] packed (a | b << 16) of each row slot, -1 = padding
  uint8_t *tile_both = nullptr; // [row tiles] 1: both lane halves scatter at once (KerrPlan::both)
  int32_t *koff = nullptr;      // [Ppad][2] LDS byte offsets of (X_a, X_b) per q, kernel lane order
  int koff_tt = 0;              // tile width (samples) the offsets were built for
  int4 *passes = nullptr;       // [npass] (first row tile, tiles, k-list offset, k-list length)
  int32_t *klist = nullptr;     // nonzero k-steps of each pass
  int npass = 0, mfma_rtm = 2;
  // matrix-core kernel with B formed once per workgroup (kerr_group.hip)
  int ngroups = 0;              // 0: that kernel is not set up for this plan
  int g_tt = 0;                 // its samples per workgroup
  int32_t *gtiles = nullptr;    // [ngroups][4][rw] row tiles of each wave
  int2 *glist = nullptr;        // k-list entries (k-step, per-wave slot masks)
  int2 *grange = nullptr;       // [ngroups] (offset, length) into glist
  int32_t *gkoff = nullptr;     // [Ppad/2] column modes (a, b), 8 bits each, two columns per word,
                                // in the order the lane halves form them
  double kerr_entries[3] = {0, 0, 0};  // packed P*P, multiplied (listed blocks), nonzero

  // replayed step graph for launch-bound plans: `graph_steps` middle RK4IP
  // steps on the field at `graph_A`, captured on `cap_stream`
  hipGraphExec_t graph = nullptr;
  float2 *graph_A = nullptr;
  int graph_steps = 0;
  hipStream_t cap_stream = nullptr;
  bool graph_failed = false;  // capture did not work here: stay eager

  // workspace
  float2 *buf[3] = {nullptr, nullptr, nullptr};
  float2 *sd[3] = {nullptr, nullptr, nullptr};  // step-doubling workspace (lazy)
  double *red = nullptr;   // reduction partials
  int red_n = 0;
  size_t bytes = 0;
};

// Host-side plan of the packed matrix-core contraction (kerr_plan.hip).
struct KerrPlan {
  int P = 0, Ppad = 0, kw = 8, nk = 0, nrt = 0, rtm = 2;
  std::vector<int> perm;             // [P] sorted pair order (rows and columns are cut from it)
  std::vector<int> cols;             // [Ppad] natural pair index at each column position, -1 = padding
  std::vector<int> a, b;             // [Ppad] column pair (a <= b) at each position, padding (0, 0)
  std::vector<int> rows;             // [nrt*32] natural pair index in each row slot, -1 = padding
  std::vector<int> ra, rb;           // [nrt*32] row pair of each slot, padding (0, 0)
  std::vector<int4> passes;          // (first row tile, tiles, k-list offset, k-list length)
  std::vector<int32_t> klist;        // k-steps of each pass that hold a nonzero
  std::vector<uint8_t> occ;          // [nrt][nk] 1 where the (row tile, k-step) block holds a nonzero
  // [nrt] 1 where the tile's rows are placed so that the two lane halves can
  // scatter at once: the rows in slots 8g + j and 8g + 4 + j (j < 4), which
  // the halves take together, differ in both modes (p and n) unless one is
  // padding
  std::vector<uint8_t> both;
  double entries[3] = {0, 0, 0};     // packed P*P, multiplied, nonzero
};
void plan_kerr(const float *S, int M, bool split, KerrPlan &kp);

// Row groups of the matrix-core kernel that forms B once per workgroup
// (kerr_group.hip): the row tiles are cut into groups of at most nw x rw
// consecutive tiles, each wave of a workgroup owns up to rw tiles of a group,
// and the group's k-list names every k-step where one of its tiles holds a
// nonzero block, with a byte per wave marking which of that wave's tile
// slots do.  Tiles are dealt to the waves to even out the blocks each wave
// multiplies per chunk of kc listed k-steps (one barrier per chunk).
struct KerrGroups {
  int nw = 0, rw = 0, kc = 0, ngroups = 0;
  std::vector<int32_t> tiles;  // [ngroups][nw][rw] row tile, -1 = empty slot
  std::vector<int2> list;      // (k-step, masks): bit j of byte w = slot j of wave w is nonzero
  std::vector<int2> range;     // [ngroups] (offset, length) into list
  double blocks = 0;           // (tile, k-step) blocks multiplied
  double chunk_max = 0;        // sum over chunks of the busiest wave's blocks
};
void plan_groups(const KerrPlan &kp, int nw, int rw, int kc, KerrGroups &g);
float packed_entry(const float *S, int M, int ar, int br, int aq, int bq);
// samples per workgroup of the matrix-core kernel for M modes and T samples
int mfma_tile_width(int M, int T);

// Host-side launch check before a kernel with a large block or dynamic LDS:
// `threads` within the kernel's compiled limit (launch bounds, registers) and
// its static LDS plus `dyn_lds` within a CU's 160 KiB.  An oversized
// configuration returns hipErrorInvalidConfiguration instead of launching.
hipError_t check_launch(const void *kern, unsigned threads, size_t dyn_lds);

// kernels (launch wrappers); all asynchronous on plan.stream
hipError_t launch_linear(const Plan &pl, const float4 *E, const float2 *in0, float2 *out0,
                         const float2 *in1, float2 *out1);
hipError_t launch_kerr(const Plan &pl, double h, const KerrLaunch &k);
// out1 = D in, out2 = D D in (D = exp(h/2 L) from table E); in may be out1.  One
// forward transform for both when the transform is four-step.
hipError_t launch_linear_twice(const Plan &pl, const float4 *E, const float2 *in, float2 *out1,
                               float2 *out2);
// out = DA * exp(i (h gamma / 2) kappa (|Az|^2 + |Aend|^2)) (Manakov form, SSFM-Agrawal)
hipError_t launch_manakov_phase(const Plan &pl, double h, const float2 *Az, const float2 *Aend,
                                const float2 *DA, float2 *out);
// n_steps RK4IP steps of a one-mode plan (pl.solo) in one launch of one
// workgroup, with run_steps' start / finish contract for N1 = h N(A)
hipError_t launch_rk4ip_solo(const Plan &pl, float2 *A, float2 *N1, int64_t n_steps, double h, const float4 *E,
                             bool start, bool finish);
// E[p][pos] = exp(h/2 L_p)/T (hi + lo) in the FFT's storage order, from beta_d / alpha_d
hipError_t launch_tabulate_E(const Plan &pl, double h, float4 *E);
// A[p][:] *= gain[p] in place (the amplifier after a span; needs pl.gain)
hipError_t launch_amplify(const Plan &pl, float2 *A);
hipError_t launch_convert_c128_to_c64(const Plan &pl, const double2 *in, float2 *out, size_t n);
hipError_t launch_convert_c64_to_c128(const Plan &pl, const float2 *in, double2 *out, size_t n);
// blocks (and FP64 partial pairs) of the norm reduction over n values: n/4096 in 1..1024
int reduction_blocks(size_t n);
// FP64 sum of |x|^2 (and of |x - y|^2 when y != nullptr) -> host values (synchronises)
hipError_t reduce_norms(const Plan &pl, const float2 *x, const float2 *y, size_t n, double *sx,
                        double *sxy);

// optional per-launch event pairs (measurement only)
struct Prof {
  std::vector<hipEvent_t> kerr, lin;  // start/stop pairs, in launch order
  int64_t kerr_evals = 0;
  hipError_t record(std::vector<hipEvent_t> &v, hipStream_t s) {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    v.push_back(e);
    return hipEventRecord(e, s);
  }
};

// The RK4IP step schedule.  work[0] carries h N(A) between steps: `start`
// computes it from A first, `finish` leaves it out after the last step.  A
// propagation split into chunks (first chunk start, last chunk finish, the
// work buffers kept between chunks) does exactly the arithmetic of one call.
// The split-step schemes keep the same contract (SSFM-Agrawal carries the
// first half step D A of the next step in work[0] on four-step plans).
hipError_t run_steps(Plan &pl, float2 *A, int64_t n_steps, double h, const float4 *E,
                     float2 *const *work, Prof *prof = nullptr, bool start = true,
                     bool finish = true);

// Argument checks shared by mmnlse_create and the server (E_INVALID + reason).
mmnlse_status validate_config(const mmnlse_config &cfg, std::string &why);
void set_last_error(const std::string &msg);

// Device bytes a plan for `cfg` will hold (fields, tables, tensor), without
// allocating; used for admission control.
size_t estimate_plan_bytes(const mmnlse_config &cfg);

}  // namespace mmnlse

struct mmnlse_ctx {
  mmnlse::Plan *pl;
};
