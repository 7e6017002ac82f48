// Device helpers shared by the two matrix-core Kerr kernels (kerr_mfma.hip,
// kerr_group.hip): operand conversions, forming B_q = X_l X_m from the LDS
// field tile, and the mode-space scatter of 32x32 accumulator tiles.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.h"

namespace mmnlse {
namespace mfma {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatv2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Two floats to bf16 (round to nearest even), packed in element order.
__device__ __forceinline__ uint32_t to_bf16x2(float x0, float x1) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((floatv2){x0, x1}, bf16x2));
}

// Two floats to bf16 hi (round to nearest even) and bf16 lo = bf16(x - hi),
// each pair packed in one register in element order.
__device__ __forceinline__ void split2(float x0, float x1, uint32_t &hi, uint32_t &lo) {
  const uint32_t hb = __builtin_bit_cast(uint32_t, __builtin_convertvector((floatv2){x0, x1}, bf16x2));
  const float r0 = x0 - __builtin_bit_cast(float, hb << 16);
  const float r1 = x1 - __builtin_bit_cast(float, hb & 0xffff0000u);
  hi = hb;
  lo = __builtin_bit_cast(uint32_t, __builtin_convertvector((floatv2){r0, r1}, bf16x2));
}

// B_q = X_a X_b at the lane's sample, X_a and X_b read at byte offsets oa, ob of
// the lane's column base xb in the LDS field tile.
__device__ __forceinline__ float2 form_b(const char *xb, int oa, int ob) {
  const float2 xa = *(const float2 *)(xb + oa);
  const float2 xc = *(const float2 *)(xb + ob);
  return make_float2(fmaf(xa.x, xc.x, -xa.y * xc.y), fmaf(xa.x, xc.y, xa.y * xc.x));
}

// Output row of accumulator register v for lane-half `half` of a 32x32 tile.
__device__ __forceinline__ int acc_row(int v, int half) { return 8 * (v >> 2) + 4 * half + (v & 3); }

// Orders the LDS accesses made before it by some lanes of the wave against
// those made after it by other lanes.  A wave's LDS operations complete in
// issue order, so this only has to stop the compiler from moving, merging or
// sinking per-lane code across it (it emits no instruction).
__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace mfma
}  // namespace mmnlse

namespace mmnlse {
namespace mfma {

// Exchanges the upper 32 lanes of a with the lower 32 lanes of b
// (v_permlane32_swap): afterwards lanes 0..31 hold (a, b) = (own a, old a of
// lane + 32) and lanes 32..63 hold (a, b) = (old b of lane - 32, own b).
__device__ __forceinline__ void swap_halves(float &a, float &b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, a), __builtin_bit_cast(unsigned, b),
                                                  false, false);
  a = __builtin_bit_cast(float, (unsigned)r[0]);
  b = __builtin_bit_cast(float, (unsigned)r[1]);
}

// Mode-space epilogue of one 32-row tile rt of C over 64 samples, given as
// the accumulators of its two 32-sample column tiles (re0, im0: samples
// 0..31, re1, im1: samples 32..63).  Swapping lane halves first gives every
// lane l all 32 rows of sample l, so the lanes touch 64 distinct samples and
// can update the LDS tiles (width 64) without ordering between them; the
// rows are then walked in order, row (p, n) adding C conj(X_n) to Os[p] and,
// for p != n, C conj(X_p) to Os[n].  Consecutive rows with the same p sum
// into a register first.  pairs[slot] = p | n << 16, -1 = padding row.
__device__ __forceinline__ void scatter_tile64(const int *pairs, floatx16 re0, floatx16 im0, floatx16 re1,
                                               floatx16 im1, int rt, const float2 *__restrict__ Xs,
                                               float2 *__restrict__ Os, int lane) {
  constexpr int TT = 64;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    float a = re0[v], b = re1[v];
    swap_halves(a, b);
    re0[v] = a;
    re1[v] = b;
    a = im0[v];
    b = im1[v];
    swap_halves(a, b);
    im0[v] = a;
    im1[v] = b;
  }
  // row acc_row(v, 0) of the lane's sample is in (re0[v], im0[v]), row acc_row(v, 1) in (re1[v], im1[v])
  const int4 *pt = (const int4 *)(pairs + rt * 32);
  int pr[32];  // the tile's 32 pairs, wave-uniform
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int4 q = pt[i];
    pr[4 * i] = __builtin_amdgcn_readfirstlane(q.x);
    pr[4 * i + 1] = __builtin_amdgcn_readfirstlane(q.y);
    pr[4 * i + 2] = __builtin_amdgcn_readfirstlane(q.z);
    pr[4 * i + 3] = __builtin_amdgcn_readfirstlane(q.w);
  }
  int cur = -1;
  float2 acc = make_float2(0.f, 0.f), xp = make_float2(0.f, 0.f);
#pragma unroll
  for (int r = 0; r < 32; ++r) {
    const int v = (r >> 3) * 4 + (r & 3);
    const bool upper = (r >> 2) & 1;
    const float2 C = upper ? make_float2(re1[v], im1[v]) : make_float2(re0[v], im0[v]);
    const int ab = pr[r];
    if (ab >= 0) {
      const int p = ab & 0xffff, n = ab >> 16;
      if (p != cur) {
        if (cur >= 0) Os[cur * TT + lane] = cadd(Os[cur * TT + lane], acc);
        cur = p;
        acc = make_float2(0.f, 0.f);
        xp = Xs[p * TT + lane];
      }
      acc = cfma_conj(acc, C, Xs[n * TT + lane]);
      if (p != n) Os[n * TT + lane] = cfma_conj(Os[n * TT + lane], C, xp);
    }
  }
  if (cur >= 0) Os[cur * TT + lane] = cadd(Os[cur * TT + lane], acc);
}

}  // namespace mfma
}  // namespace mmnlse

namespace mmnlse {
namespace mfma {

// Mode-space epilogue of one 32-row tile rt of C for the wave's 32 samples
// (column `col` of LDS tiles of width TT): the accumulator layout gives lane
// half h the rows acc_row(v, h), v = 0..15.  The halves take turns (their
// lanes share the samples); within a half every lane owns one sample, so its
// rows are walked in order without ordering between lanes: row (p, n) adds
// C conj(X_n) to Os[p] and, for p != n, C conj(X_p) to Os[n], consecutive
// rows with the same p summed in a register first.  pairs[slot] = p | n << 16,
// -1 = padding row.
template <int TT>
__device__ __forceinline__ void scatter_tile32(const int *pairs, const floatx16 &cre, const floatx16 &cim, int rt,
                                               const float2 *__restrict__ Xs, float2 *__restrict__ Os, int lane,
                                               int col) {
  const int half = lane >> 5;
  // the tile's 32 pairs, wave-uniform, read before the lane halves diverge
  const int4 *pt = (const int4 *)(pairs + rt * 32);
  int pr[32];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int4 q = pt[i];
    pr[4 * i] = __builtin_amdgcn_readfirstlane(q.x);
    pr[4 * i + 1] = __builtin_amdgcn_readfirstlane(q.y);
    pr[4 * i + 2] = __builtin_amdgcn_readfirstlane(q.z);
    pr[4 * i + 3] = __builtin_amdgcn_readfirstlane(q.w);
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (half == h) {
      int cur = -1;
      float2 acc = make_float2(0.f, 0.f), xp = make_float2(0.f, 0.f);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int ab = pr[acc_row(v, h)];
        if (ab >= 0) {
          const int p = ab & 0xffff, n = ab >> 16;
          const float2 C = make_float2(cre[v], cim[v]);
          if (p != cur) {
            if (cur >= 0) Os[cur * TT + col] = cadd(Os[cur * TT + col], acc);
            cur = p;
            acc = make_float2(0.f, 0.f);
            xp = Xs[p * TT + col];
          }
          acc = cfma_conj(acc, C, Xs[n * TT + col]);
          if (p != n) Os[n * TT + col] = cfma_conj(Os[n * TT + col], C, xp);
        }
      }
      if (cur >= 0) Os[cur * TT + col] = cadd(Os[cur * TT + col], acc);
    }
    wave_lds_order();
  }
}

// Scatter of one 32-row tile by both lane halves at once, for tiles whose
// rows the plan has placed so that the rows the halves take at the same step
// (slots 8g + j and 8g + 4 + j) differ in p and in n: the read-modify-writes
// of one instruction then never meet, and each half walks only its own 16
// rows.  Rows are not merged by p here (the halves' runs differ).
template <int TT>
__device__ __forceinline__ void scatter_tile32_both(const int *pairs, const floatx16 &cre, const floatx16 &cim,
                                                    int rt, const float2 *__restrict__ Xs,
                                                    float2 *__restrict__ Os, int lane, int col) {
  const int half = lane >> 5;
  // this half's slots 8g + 4 half + j: int4 number 2g + half of the tile
  const int4 *pt = (const int4 *)(pairs + rt * 32) + half;
  int pr[16];
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int4 q = pt[2 * g];
    pr[4 * g] = q.x;
    pr[4 * g + 1] = q.y;
    pr[4 * g + 2] = q.z;
    pr[4 * g + 3] = q.w;
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int ab = pr[v];
    if (ab >= 0) {
      const int p = ab & 0xffff, n = ab >> 16;
      const float2 C = make_float2(cre[v], cim[v]);
      Os[p * TT + col] = cfma_conj(Os[p * TT + col], C, Xs[n * TT + col]);
      if (p != n) Os[n * TT + col] = cfma_conj(Os[n * TT + col], C, Xs[p * TT + col]);
    }
  }
}

}  // namespace mfma
}  // namespace mmnlse
