// Packed Kerr contraction on matrix cores for a tensor symmetric in (l,m)
// and in (p,n) (every fully symmetric tensor).
//
// With pairs q = (l <= m) and r = (p <= n), P = M(M+1)/2 of each,
//   B_q(t)  = X_l(t) X_m(t)                              (formed on the fly)
//   C_r(t)  = sum_q Sp[r][q] B_q(t),  Sp[r][q] = w_q S[p,l,m,n], w_q = 2 for l<m
//   N_p(t)  = i gamma ( sum_{r=(p,n)} C_r conj(X_n) + sum_{r=(n,p), n<p} C_r conj(X_n) ),
// i.e. one real GEMM Sp[P x P] * [Re B | Im B][P x 2T] per evaluation plus a
// cheap scatter; this is the dense part of the Kerr term and it runs on MFMA.
//
// Workgroup = W waves; wave w owns 32 samples (64 real GEMM columns: the real
// and imaginary parts of B), so a workgroup covers 32W samples of every mode.
// Every wave walks all row tiles of Sp (32 rows each, RT at a time so that
// one B fragment feeds RT tiles); Sp is pre-swizzled so that each lane loads
// its MFMA A-operand with one coalesced 16-byte load.  The mode-space
// epilogue accumulates into the wave's own columns of an LDS tile, so no
// atomics are needed and the result is deterministic.
//
// FP32 path: v_mfma_f32_32x32x2_f32.  Split path: Sp and B are split into
// bf16 hi + lo (lo = bf16(x - hi)); hi*hi + hi*lo + lo*hi on
// v_mfma_f32_32x32x16_bf16, accumulated in FP32 (the lo*lo term, 2^-16 of
// the product, is dropped).

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <utility>
#include <vector>

#include "common.h"
#include "mfma_util.h"

namespace mmnlse {
namespace {

using namespace mfma;

struct MArgs {
  const float2 *src0, *src1, *src2;
  float2 *out0, *out1;
  const float4 *A32;     // FP32 swizzle: [row tiles][Ppad/8][64] float4
  const uint4 *Ah, *Al;  // bf16 swizzle: [row tiles][Ppad/16][64] 8 x bf16
  const int *pairs;      // [P] per row slot a | b << 16, -1 for a padding row (zero weights)
  const uint8_t *tboth;  // [row tiles] 1: the lane halves scatter the tile at once
  const int4 *koff;      // B operand: byte offsets of X_a, X_b rows in the LDS tile, lane order
  const int4 *passes;    // [npass] (first row tile, tiles, k-list offset, k-list length)
  const int *klist;      // k-steps of each pass that hold a nonzero entry of its rows
  float hg;
  int M, T, P, Ppad, next, koff_tt, npass, rtm;  // P: row slots (row tiles x 32)
};

// A pass's k-list read through registers: lane i of `cur` holds entry
// base + i, of `nxt` entry base + 64 + i (loaded 64 entries before it is
// needed).  Entries come out with v_readlane, so the k-loop issues no scalar
// memory loads (their counter is shared with LDS and would force full waits
// on the B-operand reads).
struct KList {
  const int *kl;
  int len, base, cur, nxt;
  // clamped, so that the load is unconditional (entries past the end are
  // never used)
  __device__ __forceinline__ int load(int c, int lane) const { return kl[min(64 * c + lane, len - 1)]; }
  __device__ __forceinline__ void init(const int *k, int n, int lane) {
    kl = k;
    len = n;
    base = 0;
    cur = load(0, lane);
    nxt = load(1, lane);
  }
  // entry i, base <= i < base + 128
  __device__ __forceinline__ int at(int i) const {
    const int o = i - base;
    return o < 64 ? __builtin_amdgcn_readlane(cur, o) : __builtin_amdgcn_readlane(nxt, o - 64);
  }
  // the walk has left entries base .. base + 63 behind
  __device__ __forceinline__ void slide(int lane) {
    cur = nxt;
    base += 64;
    nxt = load(base / 64 + 1, lane);
  }
};

// One pass over RT consecutive row tiles (rows 32*rt0 .. 32*(rt0+RT)-1) for
// the wave's 32 samples: accumulate C over the listed k-steps, then scatter
// into Os.  The k-loop is unrolled by two over two register sets for the A
// operand and the B offsets: the operands of k-step i + 2 are loaded into
// the set that k-step i has just used, so every load has a whole k-step to
// arrive and no registers are copied.  The loads are issued unconditionally
// (indices clamped into the list), so the compiler counts them instead of
// waiting for all.
template <int W, int RT, int SPLIT>
__device__ __forceinline__ void contract_pass(const MArgs &a, const float2 *Xs, float2 *Os, int lane, int col,
                                              int rt0, const int *kl, int len) {
  constexpr int TT = 32 * W;
  const int half = lane >> 5;
  const char *xb = (const char *)(Xs + col);
  floatx16 cre[RT], cim[RT];
#pragma unroll
  for (int j = 0; j < RT; ++j) {
    cre[j] = floatx16{0};
    cim[j] = floatx16{0};
  }
  len = __builtin_amdgcn_readfirstlane(len);
  const int last = len - 1;
  // The k-loop, for the k-steps kat(0..len-1).  A dense pass walks every
  // k-step in order (kat is the identity, so addresses advance by a stride);
  // a pass with zero blocks reads its list through registers.
  if (!SPLIT) {
    const int nk = a.Ppad / 8;  // 4 k-steps of 2 per iteration (a group of 8 columns)
    const float4 *Ab = a.A32 + (size_t)rt0 * nk * 64 + lane;
    // this lane half's (oa, ob) for the 4 k-steps of a group
    const int4 *ko = a.koff + 2 * half;
    auto kloop = [&](auto kat, auto slide) {
      float4 av[2][RT];
      int4 o0[2], o1[2];
      float2 xa[2][4], xc[2][4];  // the X_a, X_b of a set's k-step, read one k-step ahead
      auto load = [&](int set, int kq) {
#pragma unroll
        for (int j = 0; j < RT; ++j) av[set][j] = Ab[((size_t)j * nk + kq) * 64];
        o0[set] = ko[4 * kq];
        o1[set] = ko[4 * kq + 1];
      };
      auto readx = [&](int set) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int oa = s == 0 ? o0[set].x : s == 1 ? o0[set].z : s == 2 ? o1[set].x : o1[set].z;
          const int ob = s == 0 ? o0[set].y : s == 1 ? o0[set].w : s == 2 ? o1[set].y : o1[set].w;
          xa[set][s] = *(const float2 *)(xb + oa);
          xc[set][s] = *(const float2 *)(xb + ob);
        }
      };
      // products of the set's k-step, then the X reads of the other set's
      // k-step (the next one), which run while these products execute
      auto body = [&](int set) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const float2 x = xa[set][s], y = xc[set][s];
          const float2 b = make_float2(fmaf(x.x, y.x, -x.y * y.y), fmaf(x.x, y.y, x.y * y.x));
#pragma unroll
          for (int j = 0; j < RT; ++j) {
            const float4 v = av[set][j];
            const float av_s = s == 0 ? v.x : s == 1 ? v.y : s == 2 ? v.z : v.w;
            cre[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av_s, b.x, cre[j], 0, 0, 0);
            cim[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av_s, b.y, cim[j], 0, 0, 0);
          }
        }
        readx(1 - set);
      };
      load(0, kat(0));
      load(1, kat(min(1, last)));
      readx(0);
      // pairs of k-steps, in chunks of 64 list entries (the list window
      // slides between chunks); an odd last k-step after the loop.  The
      // operands are loaded a whole k-step ahead of their use and the X
      // values one k-step ahead (scheduling barriers keep them there; FP32
      // only: on the split paths the scheduler's interleaving of one
      // k-step's B formation with the other's products is worth more).
      for (int c0 = 0; c0 < last; c0 += 64) {
        const int cend = min(c0 + 64, last);
        for (int it = c0; it < cend; it += 2) {
          body(0);
          load(0, kat(min(it + 2, last)));
          __builtin_amdgcn_sched_barrier(0);
          body(1);
          load(1, kat(min(it + 3, last)));
          __builtin_amdgcn_sched_barrier(0);
        }
        slide();
      }
      if (len & 1) body(0);
    };
    if (len == nk) {
      kloop([](int i) { return i; }, [] {});
    } else {
      KList L;
      L.init(kl, len, lane);
      kloop([&](int i) { return L.at(i); }, [&] { L.slide(lane); });
    }
  } else {
    const int nk = a.Ppad / 16;  // k-steps of 16
    const uint4 *Hb = a.Ah + (size_t)rt0 * nk * 64 + lane;
    const uint4 *Lb = a.Al + (size_t)rt0 * nk * 64 + lane;
    // this lane half's (oa, ob) for the 8 pairs of a k-step
    const int4 *ko = a.koff + 4 * half;
    auto kloop = [&](auto kat, auto slide) {
      uint4 ah[2][RT], al[2][RT];
      int4 o[2][4];
      auto load = [&](int set, int ks) {
#pragma unroll
        for (int j = 0; j < RT; ++j) {
          ah[set][j] = Hb[((size_t)j * nk + ks) * 64];
          al[set][j] = Lb[((size_t)j * nk + ks) * 64];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) o[set][i] = ko[8 * ks + i];
      };
      float2 xr[4][4];  // X_a, X_b of the next k-step's elements 2i, 2i+1, read ahead
      auto readx = [&](int set) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          xr[i][0] = *(const float2 *)(xb + o[set][i].x);
          xr[i][1] = *(const float2 *)(xb + o[set][i].y);
          xr[i][2] = *(const float2 *)(xb + o[set][i].z);
          xr[i][3] = *(const float2 *)(xb + o[set][i].w);
        }
      };
      auto cmulx = [](float2 x, float2 y) {
        return make_float2(fmaf(x.x, y.x, -x.y * y.y), fmaf(x.x, y.y, x.y * y.x));
      };
      // B of the set's k-step from the X values read ahead, then the reads of
      // the next k-step (the other set's offsets), then the products
      auto body = [&](int set) {
        uint32_t urh[4], url[4], uih[4], uil[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {  // elements 2i and 2i+1
          const float2 b0 = cmulx(xr[i][0], xr[i][1]);
          const float2 b1 = cmulx(xr[i][2], xr[i][3]);
          if (SPLIT == 1) {
            split2(b0.x, b1.x, urh[i], url[i]);
            split2(b0.y, b1.y, uih[i], uil[i]);
          } else {  // B rounded to bf16 only
            urh[i] = to_bf16x2(b0.x, b1.x);
            uih[i] = to_bf16x2(b0.y, b1.y);
            url[i] = uil[i] = 0;
          }
        }
        const bf16x8 rh = __builtin_bit_cast(bf16x8, make_uint4(urh[0], urh[1], urh[2], urh[3]));
        const bf16x8 rl = __builtin_bit_cast(bf16x8, make_uint4(url[0], url[1], url[2], url[3]));
        const bf16x8 ih = __builtin_bit_cast(bf16x8, make_uint4(uih[0], uih[1], uih[2], uih[3]));
        const bf16x8 il = __builtin_bit_cast(bf16x8, make_uint4(uil[0], uil[1], uil[2], uil[3]));
        readx(1 - set);
#pragma unroll
        for (int j = 0; j < RT; ++j) {
          const bf16x8 sh = __builtin_bit_cast(bf16x8, ah[set][j]);
          const bf16x8 sl = __builtin_bit_cast(bf16x8, al[set][j]);
          cre[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sl, rh, cre[j], 0, 0, 0);
          if (SPLIT == 1) cre[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sh, rl, cre[j], 0, 0, 0);
          cre[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sh, rh, cre[j], 0, 0, 0);
          cim[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sl, ih, cim[j], 0, 0, 0);
          if (SPLIT == 1) cim[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sh, il, cim[j], 0, 0, 0);
          cim[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sh, ih, cim[j], 0, 0, 0);
        }
      };
      load(0, kat(0));
      load(1, kat(min(1, last)));
      readx(0);
      // pairs of k-steps, in chunks of 64 list entries (the list window
      // slides between chunks); an odd last k-step after the loop
      for (int c0 = 0; c0 < last; c0 += 64) {
        const int cend = min(c0 + 64, last);
        for (int it = c0; it < cend; it += 2) {
          body(0);
          load(0, kat(min(it + 2, last)));
          // the operand loads stay a k-step ahead; every other kind of
          // instruction may still be interleaved across the two k-steps
          __builtin_amdgcn_sched_barrier(0x038F);
          body(1);
          load(1, kat(min(it + 3, last)));
          __builtin_amdgcn_sched_barrier(0x038F);
        }
        slide();
      }
      if (len & 1) body(0);
    };
    if (len == nk) {
      kloop([](int i) { return i; }, [] {});
    } else {
      KList L;
      L.init(kl, len, lane);
      kloop([&](int i) { return L.at(i); }, [&] { L.slide(lane); });
    }
  }
#pragma unroll
  for (int j = 0; j < RT; ++j) {
    if (__builtin_amdgcn_readfirstlane((int)a.tboth[rt0 + j]))
      scatter_tile32_both<TT>(a.pairs, cre[j], cim[j], rt0 + j, Xs, Os, lane, col);
    else
      scatter_tile32<TT>(a.pairs, cre[j], cim[j], rt0 + j, Xs, Os, lane, col);
  }
}

// Full contraction for one wave: the passes of the plan's pass table (runs of
// 1, 2 or RTM row tiles chosen at setup; rows are padded to a multiple of 32
// only) are dealt to the row groups, pass u to row group u % R.
// A pass multiplies only the k-steps of its list (where its rows hold a
// nonzero entry); a pass with an empty list contributes nothing.
template <int W, int R, int SPLIT, int RTM>
__device__ __forceinline__ void contract(const MArgs &a, const float2 *Xs, float2 *Os, int lane, int col,
                                         int rg) {
  for (int u = rg; u < a.npass; u += R) {
    const int4 ps = a.passes[u];
    if (ps.w == 0) continue;
    const int *kl = a.klist + ps.z;
    if (RTM == 4 && ps.y == 4) contract_pass<W, (RTM == 4 ? 4 : 1), SPLIT>(a, Xs, Os, lane, col, ps.x, kl, ps.w);
    else if (ps.y == 2) contract_pass<W, 2, SPLIT>(a, Xs, Os, lane, col, ps.x, kl, ps.w);
    else contract_pass<W, 1, SPLIT>(a, Xs, Os, lane, col, ps.x, kl, ps.w);
  }
}

// Workgroup = W column groups x R row groups of waves.  Wave w owns the 32
// samples of column group w % W and the passes of row group w / W, and
// scatters into that row group's partial tile; the R partials are summed in
// a fixed order, so the result does not depend on timing.
template <int W, int R, int SPLIT, int RTM, int STAGE>
__global__ __launch_bounds__(64 * W * R) void kerr_mfma(MArgs a) {
  constexpr int TT = 32 * W;
  constexpr int NT = 64 * W * R;
  extern __shared__ float2 sh[];
  const int MT = a.M * TT;
  float2 *Xs = sh;
  float2 *Os = sh + MT;  // R partial tiles
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int cg = w % W, rg = w / W;
  const int col = 32 * cg + (lane & 31);
  const int t0 = blockIdx.x * TT;
  for (int idx = threadIdx.x; idx < MT; idx += NT) {
    const size_t g = (size_t)(idx / TT) * a.T + t0 + (idx % TT);
    float2 v = a.src0[g];
    if (STAGE == STAGE_K2 || STAGE == STAGE_K23) v = caxpy(v, 0.5f, a.src1[g]);
    if (STAGE == STAGE_K3) v = caxpy(v, 0.5f, a.src2[g]);
    Xs[idx] = v;
  }
  for (int idx = threadIdx.x; idx < R * MT; idx += NT) Os[idx] = make_float2(0.f, 0.f);
  __syncthreads();
  contract<W, R, SPLIT, RTM>(a, Xs, Os + rg * MT, lane, col, rg);
  __syncthreads();
  for (int idx = threadIdx.x; idx < MT; idx += NT) {
    const size_t g = (size_t)(idx / TT) * a.T + t0 + (idx % TT);
    float2 o = Os[idx];
#pragma unroll
    for (int r = 1; r < R; ++r) o = cadd(o, Os[r * MT + idx]);
    const float2 k = make_float2(-a.hg * o.y, a.hg * o.x);  // i h gamma sum
    if (STAGE == STAGE_PLAIN || STAGE == STAGE_K2) {
      a.out0[g] = k;
    } else if (STAGE == STAGE_K23) {  // k2 -> out1 (read back below), next argument A_I + k2/2
      a.out1[g] = k;
      Xs[idx] = caxpy(a.src0[g], 0.5f, k);
    } else if (STAGE == STAGE_K3) {
      const float2 ai = a.src0[g], k1 = a.src1[g], k2 = a.src2[g];
      a.out0[g] = cadd(ai, k);
      float2 z = caxpy(ai, 1.f / 6.f, k1);
      z = caxpy(z, 1.f / 3.f, k2);
      a.out1[g] = caxpy(z, 1.f / 3.f, k);
    } else {
      const float2 An = caxpy(a.src1[g], 1.f / 6.f, k);
      a.out0[g] = An;
      Xs[idx] = An;
    }
  }
  if ((STAGE == STAGE_K4 && a.next) || STAGE == STAGE_K23) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < R * MT; idx += NT) Os[idx] = make_float2(0.f, 0.f);
    __syncthreads();
    contract<W, R, SPLIT, RTM>(a, Xs, Os + rg * MT, lane, col, rg);
    __syncthreads();
    for (int idx = threadIdx.x; idx < MT; idx += NT) {
      const size_t g = (size_t)(idx / TT) * a.T + t0 + (idx % TT);
      float2 o = Os[idx];
#pragma unroll
      for (int r = 1; r < R; ++r) o = cadd(o, Os[r * MT + idx]);
      const float2 k = make_float2(-a.hg * o.y, a.hg * o.x);
      if (STAGE == STAGE_K23) {  // same thread wrote out1[g] (k2) above
        const float2 ai = a.src0[g], k1 = a.src1[g], k2 = a.out1[g];
        a.out0[g] = cadd(ai, k);
        float2 z = caxpy(ai, 1.f / 6.f, k1);
        z = caxpy(z, 1.f / 3.f, k2);
        a.out1[g] = caxpy(z, 1.f / 3.f, k);
      } else {
        a.out1[g] = k;
      }
    }
  }
}

template <int W, int R, int SPLIT, int RTM>
hipError_t go(const MArgs &a, KerrStage st, hipStream_t s) {
  constexpr int TT = 32 * W;
  if (a.koff_tt != TT) return hipErrorInvalidValue;  // offsets built for another tile width
  const dim3 grid(a.T / TT), block(64 * W * R);
  const size_t shm = (size_t)(1 + R) * a.M * TT * sizeof(float2);
  auto launch = [&](auto kern) -> hipError_t {
    hipError_t e = check_launch((const void *)kern, block.x, shm);
    if (e != hipSuccess) return e;
    if (shm > 65536) {
      e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, grid, block, shm, s, a);
    return hipGetLastError();
  };
  switch (st) {
    case STAGE_PLAIN: return launch(kerr_mfma<W, R, SPLIT, RTM, STAGE_PLAIN>);
    case STAGE_K2: return launch(kerr_mfma<W, R, SPLIT, RTM, STAGE_K2>);
    case STAGE_K3: return launch(kerr_mfma<W, R, SPLIT, RTM, STAGE_K3>);
    case STAGE_K4: return launch(kerr_mfma<W, R, SPLIT, RTM, STAGE_K4>);
    case STAGE_K23: return launch(kerr_mfma<W, R, SPLIT, RTM, STAGE_K23>);
  }
  return hipErrorInvalidValue;
}

// Workgroup shape by mode count (LDS holds the field tile and R partials,
// (1 + R) * M * 32W * 8 bytes <= 160 KiB):
//   M <= 64: 4 column groups (128 samples), 1 row group
//   M <= 125: 1 column group (32 samples), 4 row groups
//   M <= 208: 1 x 2;   M <= 256: 1 x 1
template <int SPLIT, int RTM>
hipError_t go_shape(const MArgs &a, KerrStage st, hipStream_t s) {
  if (mfma_tile_width(a.M, a.T) == 128) return go<4, 1, SPLIT, RTM>(a, st, s);
  if (a.M <= 125) return go<1, 4, SPLIT, RTM>(a, st, s);
  if (a.M <= 208) return go<1, 2, SPLIT, RTM>(a, st, s);
  return go<1, 1, SPLIT, RTM>(a, st, s);
}

template <int SPLIT>
hipError_t go_w(const MArgs &a, KerrStage st, hipStream_t s) {
  // row tiles per pass (fixed when the pass table was built)
  if (a.rtm == 4) return go_shape<SPLIT, 4>(a, st, s);
  return go_shape<SPLIT, 2>(a, st, s);
}

uint16_t bf16_bits(float x) {  // round to nearest even
  uint32_t u;
  std::memcpy(&u, &x, 4);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}

float bf16_value(uint16_t b) {
  uint32_t u = (uint32_t)b << 16;
  float x;
  std::memcpy(&x, &u, 4);
  return x;
}

}  // namespace

hipError_t setup_groups(Plan &pl, const KerrPlan &kp);  // kerr_group.hip
hipError_t launch_kerr_group(const Plan &pl, double h, const KerrLaunch &k);

hipError_t launch_kerr_mfma(const Plan &pl, double h, const KerrLaunch &k) {
  if (pl.ngroups > 0) return launch_kerr_group(pl, h, k);
  MArgs a;
  a.src0 = k.src0;
  a.src1 = k.src1;
  a.src2 = k.src2;
  a.out0 = k.out0;
  a.out1 = k.out1;
  a.A32 = (const float4 *)pl.Sp;
  a.Ah = (const uint4 *)pl.Sph;
  a.Al = (const uint4 *)pl.Spl;
  a.pairs = pl.pairs;
  a.tboth = pl.tile_both;
  a.koff = (const int4 *)pl.koff;
  a.koff_tt = pl.koff_tt;
  a.passes = (const int4 *)pl.passes;
  a.klist = pl.klist;
  a.npass = pl.npass;
  a.rtm = pl.mfma_rtm;
  a.hg = (float)(h * pl.gamma);
  a.M = pl.M;
  a.T = pl.T;
  a.P = pl.mfma_rows;
  a.Ppad = pl.Ppad;
  a.next = k.next;
  if (pl.precision == MMNLSE_SPLIT_BF16) return go_w<1>(a, k.stage, pl.stream);
  if (pl.precision == MMNLSE_SPLIT_BF16_S) return go_w<2>(a, k.stage, pl.stream);
  return go_w<0>(a, k.stage, pl.stream);
}

// Build the device tables of the contraction from its host plan: the pair
// table, the B-operand offsets, the swizzled A operand, the passes and
// their k-lists.
hipError_t setup_mfma(Plan &pl, const float *S) {
  const int M = pl.M;
  const bool split = pl.precision != MMNLSE_FP32;  // both bf16 modes share the tables
  KerrPlan kp;
  plan_kerr(S, M, split, kp);
  const int P = kp.P, Ppad = kp.Ppad, nrt = kp.nrt, nk = kp.nk, R = nrt * 32;
  pl.P = P;
  pl.Ppad = Ppad;
  pl.mfma_rows = R;
  const int *a = kp.a.data(), *b = kp.b.data();  // columns
  const int *rows = kp.rows.data(), *ra = kp.ra.data(), *rb = kp.rb.data();
  const int *cols = kp.cols.data();
  std::vector<int32_t> pairs(R, -1);
  for (int i = 0; i < R; ++i)
    if (rows[i] >= 0) pairs[i] = ra[i] | (rb[i] << 16);
  // row slot r, column position q
  auto Sp = [&](int r, int q) -> float {
    return rows[r] >= 0 && cols[q] >= 0 ? packed_entry(S, M, ra[r], rb[r], a[q], b[q]) : 0.f;
  };
  hipError_t e;
  auto alloc_copy = [&](void **dst, const void *src, size_t bytes) -> hipError_t {
    hipError_t r = hipMalloc(dst, bytes);
    if (r != hipSuccess) return r;
    pl.bytes += bytes;
    return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
  };
  if ((e = alloc_copy((void **)&pl.pairs, pairs.data(), sizeof(int32_t) * R)) != hipSuccess) return e;
  if ((e = alloc_copy((void **)&pl.tile_both, kp.both.data(), sizeof(uint8_t) * nrt)) != hipSuccess) return e;
  // B-operand offsets (bytes into the LDS field tile [M][TT] float2) of X_a and
  // X_b for column q, in the order a lane reads them: split path q = 16 ks +
  // 8 half + e (natural order); FP32 path q = 8 kq + 2 s + half stored at
  // ((kq * 2 + half) * 4 + s).
  const int TT = mfma_tile_width(M, pl.T);
  std::vector<int32_t> koff(2 * (size_t)Ppad);
  for (int q = 0; q < Ppad; ++q) {
    size_t slot = q;
    if (!split) {
      const int kq = q / 8, s = (q % 8) / 2, hf = q % 2;
      slot = ((size_t)kq * 2 + hf) * 4 + s;
    }
    koff[2 * slot] = a[q] * TT * 8;
    koff[2 * slot + 1] = b[q] * TT * 8;
  }
  if ((e = alloc_copy((void **)&pl.koff, koff.data(), sizeof(int32_t) * koff.size())) != hipSuccess) return e;
  pl.koff_tt = TT;
  // swizzled A operand: each lane's MFMA A fragment of a (row tile, k-step) in one 16-byte load
  if (!split) {
    std::vector<float> sw((size_t)R * Ppad);
    for (int rt = 0; rt < nrt; ++rt)
      for (int kq = 0; kq < nk; ++kq)
        for (int lane = 0; lane < 64; ++lane)
          for (int s = 0; s < 4; ++s)
            sw[(((size_t)rt * nk + kq) * 64 + lane) * 4 + s] = Sp(rt * 32 + (lane & 31), 8 * kq + 2 * s + (lane >> 5));
    if ((e = alloc_copy((void **)&pl.Sp, sw.data(), sizeof(float) * sw.size())) != hipSuccess) return e;
  } else {
    std::vector<uint16_t> hi((size_t)R * Ppad), lo((size_t)R * Ppad);
    for (int rt = 0; rt < nrt; ++rt)
      for (int ks = 0; ks < nk; ++ks)
        for (int lane = 0; lane < 64; ++lane)
          for (int e8 = 0; e8 < 8; ++e8) {
            const float v = Sp(rt * 32 + (lane & 31), 16 * ks + 8 * (lane >> 5) + e8);
            const uint16_t hb = bf16_bits(v);
            const size_t idx = (((size_t)rt * nk + ks) * 64 + lane) * 8 + e8;
            hi[idx] = hb;
            lo[idx] = bf16_bits(v - bf16_value(hb));
          }
    if ((e = alloc_copy((void **)&pl.Sph, hi.data(), sizeof(uint16_t) * hi.size())) != hipSuccess) return e;
    if ((e = alloc_copy((void **)&pl.Spl, lo.data(), sizeof(uint16_t) * lo.size())) != hipSuccess) return e;
  }
  std::vector<int32_t> klist = kp.klist;
  if (klist.empty()) klist.push_back(0);
  if ((e = alloc_copy((void **)&pl.passes, kp.passes.data(), sizeof(int4) * kp.passes.size())) != hipSuccess)
    return e;
  if ((e = alloc_copy((void **)&pl.klist, klist.data(), sizeof(int32_t) * klist.size())) != hipSuccess) return e;
  pl.npass = (int)kp.passes.size();
  pl.mfma_rtm = kp.rtm;
  for (int i = 0; i < 3; ++i) pl.kerr_entries[i] = kp.entries[i];
  // the kernel that forms B once per workgroup (kerr_group.hip) where it
  // applies; MMNLSE_GROUP_KERNEL=0 keeps the per-pass kernel above
  return setup_groups(pl, kp);
}

}  // namespace mmnlse
