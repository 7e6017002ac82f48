// Packed Kerr contraction on matrix cores with the B operand formed once per
// workgroup and k-step, shared by the workgroup's four waves.
//
// Same packed form as kerr_mfma.hip (Kerr term of Eq. 1 for a tensor
// symmetric in (l,m) and in (p,n)):
//   B_q(t) = X_l(t) X_m(t),  C_r(t) = sum_q Sp[r][q] B_q(t),
//   N_p(t) = i gamma ( sum_{r=(p,n)} C_r conj(X_n) + sum_{r=(n,p), n<p} C_r conj(X_n) ).
// SPLIT = 0: FP32 on v_mfma_f32_32x32x2_f32 (k-steps of 8 columns, four
// products of depth 2).  SPLIT = 1: Sp and B split into bf16 hi + lo (lo =
// bf16(x - hi)), multiplied as hi*lo + lo*hi + hi*hi on
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation (k-steps of 16 columns);
// SPLIT = 2: B rounded to bf16 once (S hi*B + S lo*B).
//
// Workgroup = 4 waves (one per SIMD) x 64 samples, two 32-sample column tiles,
// so every A fragment loaded feeds both column tiles.  The row tiles of Sp
// (32 rows each) are cut into groups of up to 4 x RW tiles; each wave owns up
// to RW tiles of a group and keeps their accumulators in registers for the
// whole k-loop.  The k-loop walks the group's listed k-steps (those where
// some tile of the group holds a nonzero) in chunks of KC.  For every chunk
// the four waves form B = X_l X_m once for its columns and the workgroup's
// samples, in the MFMA B-operand layout (split into bf16 hi and lo on the
// split paths), into a double-buffered LDS area (one barrier per chunk), and
// each wave multiplies those of its tiles whose block at the k-step holds a
// nonzero (bit masks of the plan).  Forming B costs one pass over the
// columns per group instead of one per pass of one to four row tiles (the
// vector-instruction load of kerr_mfma.hip's split path), and the A operand
// is read once per 64 samples instead of once per 32.
//
// After a group's k-loop each wave scatters its tiles into a partial output
// tile in LDS: its own when four fit (NPART = 4), else the waves sharing a
// partial (NPART = 2 or 1) take turns.  The scatter swaps accumulator lane
// halves so that each lane walks all 32 rows of one sample (scatter_tile64).
// The partials are summed in a fixed order, so the result does not depend
// on timing.  The RK4 stage prologue and epilogue are those of
// kerr_mfma.hip.
//
// setup_groups enables the kernel only for tensors whose group blocks are
// nearly all nonzero (dense tensors); strongly masked ones stay on the
// per-pass kernel, which skips their zero blocks at less cost.

#include <algorithm>
#include <cstdlib>
#include <vector>

#include "common.h"
#include "mfma_util.h"


namespace mmnlse {
namespace {

using namespace mfma;

constexpr int NW = 4;  // waves per workgroup

struct GArgs {
  const float2 *src0, *src1, *src2;
  float2 *out0, *out1;
  const uint4 *Ah, *Al;  // split: swizzled A operand [row tiles][nk][64 lanes] 8 x bf16 (hi, lo)
  const float4 *A32;     // FP32: swizzled A operand [row tiles][nk][64 lanes] 4 x float
  const int *pairs;      // [row slots] p | n << 16, -1 = padding row
  const int *kmodes;     // [nk][2 lane halves][NE / 2]: modes (a, b) of the NE columns a lane half
                         // forms per k-step, 8 bits each, two columns per word (a, b, a', b')
  const int *gtiles;     // [ngroups][NW][RW] row tile of each wave slot, -1 = empty
  const int2 *glist;     // listed k-steps: (k-step, slot masks, byte w for wave w)
  const int2 *grange;    // [ngroups] (offset, length) into glist
  float hg;
  int M, T, P, nk, ngroups, next;
};

// A group's k-list read through registers: lane i of (ck, cm) holds entry
// base + i, of (xk, xm) entry base + 64 + i; entries come out with
// v_readlane, so the k-loop issues no scalar memory loads (their counter is
// shared with LDS and would force waits on the B-operand reads).
struct GList {
  const int2 *p;
  int len, base;
  int ck, cm, xk, xm;
  __device__ __forceinline__ void load(int c, int lane, int &k, int &m) const {
    const int i = 64 * c + lane;
    const int2 v = i < len ? p[i] : make_int2(0, 0);
    k = v.x;
    m = v.y;
  }
  __device__ __forceinline__ void init(const int2 *q, int n, int lane) {
    p = q;
    len = n;
    base = 0;
    load(0, lane, ck, cm);
    load(1, lane, xk, xm);
  }
  // entry i, base <= i < base + 128
  __device__ __forceinline__ int2 at(int i) const {
    const int o = i - base;
    return o < 64 ? make_int2(__builtin_amdgcn_readlane(ck, o), __builtin_amdgcn_readlane(cm, o))
                  : make_int2(__builtin_amdgcn_readlane(xk, o - 64), __builtin_amdgcn_readlane(xm, o - 64));
  }
  // no entry below i is read again: slide the window when i leaves its first half
  __device__ __forceinline__ void retire(int i, int lane) {
    if (i >= base + 64) {
      ck = xk;
      cm = xm;
      base += 64;
      load(base / 64 + 1, lane, xk, xm);
    }
  }
};

template <int TT, int RW, int NPART, int KC, int SPLIT>
__device__ __forceinline__ void contract(const GArgs &a, const float2 *Xs, float2 *Os, uint4 *Bs, int w,
                                         int lane) {
  constexpr int CT = TT / 32;                // 32-sample column tiles
  // B operands per (k-step, column tile), 16 bytes per lane each: split rh, ih
  // (, rl, il) of 8 bf16; FP32 re, im of 4 floats (one per 32x32x2 product)
  constexpr int NOP = SPLIT == 1 ? 4 : 2;
  constexpr int NE = SPLIT ? 8 : 4;          // columns a lane half forms per k-step (k-step: 2 NE columns)
  constexpr int UPW = KC * CT / NW;          // (k-step, column tile) units each wave forms per chunk
  static_assert(UPW >= 1 && UPW * NW == KC * CT, "the chunk's units are shared evenly by the waves");
  static_assert(KC % 2 == 0, "the A-operand registers alternate between two sets");
  const int half = lane >> 5;
  const int MT = a.M * TT;
  for (int g = 0; g < a.ngroups; ++g) {
    const int2 rg = a.grange[g];
    const int len = rg.y, nch = (len + KC - 1) / KC;
    int tile[RW];
#pragma unroll
    for (int j = 0; j < RW; ++j) tile[j] = __builtin_amdgcn_readfirstlane(a.gtiles[(g * NW + w) * RW + j]);
    floatx16 cre[RW][CT], cim[RW][CT];
#pragma unroll
    for (int j = 0; j < RW; ++j)
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        cre[j][c] = floatx16{0};
        cim[j][c] = floatx16{0};
      }
    GList L;
    L.init(a.glist + rg.x, len, lane);

    // B of unit u = w + NW i of chunk c (listed entry c*KC + u / CT, column
    // tile u % CT) into buffer `buf`, from the column modes o (loaded one
    // chunk ahead)
    auto form = [&](int c, int buf, const int4 (&o)[UPW]) {
#pragma unroll
      for (int i = 0; i < UPW; ++i) {
        const int u = w + NW * i, ukk = u / CT, uct = u % CT;
        if (c * KC + ukk < len) {
          const char *xb = (const char *)(Xs + 32 * uct + (lane & 31));
          constexpr int sh = 3 + (TT == 64 ? 6 : 5);  // byte offset of mode row r in the tile: r * TT * 8
          const int ow[4] = {o[i].x, o[i].y, o[i].z, o[i].w};
          uint4 *dst = Bs + ((buf * KC + ukk) * CT + uct) * NOP * 64 + lane;
          // elements 2k and 2k+1 of the lane's NE from word k, converted as they are formed
          if (SPLIT == 0) {
            float re[4], im[4];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
              const int q = ow[k];
              const float2 b0 = form_b(xb, (q & 0xff) << sh, ((q >> 8) & 0xff) << sh);
              const float2 b1 = form_b(xb, ((q >> 16) & 0xff) << sh, ((unsigned)q >> 24) << sh);
              re[2 * k] = b0.x;
              im[2 * k] = b0.y;
              re[2 * k + 1] = b1.x;
              im[2 * k + 1] = b1.y;
            }
            dst[0] = __builtin_bit_cast(uint4, make_float4(re[0], re[1], re[2], re[3]));
            dst[64] = __builtin_bit_cast(uint4, make_float4(im[0], im[1], im[2], im[3]));
          } else {
            uint32_t urh[4], url[4], uih[4], uil[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const int q = ow[k];
              const float2 b0 = form_b(xb, (q & 0xff) << sh, ((q >> 8) & 0xff) << sh);
              const float2 b1 = form_b(xb, ((q >> 16) & 0xff) << sh, ((unsigned)q >> 24) << sh);
              if (SPLIT == 1) {
                split2(b0.x, b1.x, urh[k], url[k]);
                split2(b0.y, b1.y, uih[k], uil[k]);
              } else {
                urh[k] = to_bf16x2(b0.x, b1.x);
                uih[k] = to_bf16x2(b0.y, b1.y);
              }
            }
            dst[0] = make_uint4(urh[0], urh[1], urh[2], urh[3]);
            dst[64] = make_uint4(uih[0], uih[1], uih[2], uih[3]);
            if (SPLIT == 1) {
              dst[128] = make_uint4(url[0], url[1], url[2], url[3]);
              dst[192] = make_uint4(uil[0], uil[1], uil[2], uil[3]);
            }
          }
        }
      }
    };
    // column modes of the entries this wave forms in chunk c (entries
    // clamped into the list, so the loads are issued unconditionally and
    // the compiler can count them)
    auto load_koff = [&](int c, int4 (&o)[UPW]) {
#pragma unroll
      for (int i = 0; i < UPW; ++i) {
        const int e = min(c * KC + (w + NW * i) / CT, len - 1);
        const int *km = a.kmodes + (2 * L.at(e).x + half) * (NE / 2);
        if (NE == 8) {
          o[i] = *(const int4 *)km;
        } else {
          const int2 v = *(const int2 *)km;
          o[i] = make_int4(v.x, v.y, 0, 0);
        }
      }
    };
    // A operand of entry e (clamped) for every slot of the wave, in register
    // set `set`; unconditional for the same reason (an empty slot reads tile 0)
    uint4 ah[2][RW], al[2][RW];   // split: hi, lo
    float4 af[2][RW];             // FP32
    auto load_a = [&](int e, int set) {
      const int ks = L.at(min(e, len - 1)).x;
#pragma unroll
      for (int j = 0; j < RW; ++j) {
        const size_t off = ((size_t)max(tile[j], 0) * a.nk + ks) * 64 + lane;
        if (SPLIT) {
          ah[set][j] = a.Ah[off];
          al[set][j] = a.Al[off];
        } else {
          af[set][j] = a.A32[off];
        }
      }
    };

    int4 ko_cur[UPW], ko_nxt[UPW];
    if (len > 0) {
      load_koff(0, ko_cur);
      load_a(0, 0);
      form(0, 0, ko_cur);
      load_koff(1, ko_cur);
    }
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
      L.retire(c * KC, lane);
      load_koff(c + 2, ko_nxt);
      form(c + 1, (c + 1) & 1, ko_cur);
#pragma unroll
      for (int kk = 0; kk < KC; ++kk) {
        const int e = c * KC + kk;
        load_a(e + 1, (kk + 1) & 1);
        if (e < len) {
          const int m = (L.at(e).y >> (8 * w)) & 0xff;
          const uint4 *src = Bs + ((c & 1) * KC + kk) * CT * NOP * 64 + lane;
          if (SPLIT == 0) {
            float4 br[CT], bi[CT];
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
              br[ct] = __builtin_bit_cast(float4, src[(ct * NOP + 0) * 64]);
              bi[ct] = __builtin_bit_cast(float4, src[(ct * NOP + 1) * 64]);
            }
            // the wave's tiles whose block at this k-step holds a nonzero;
            // the k-step's 8 columns are 4 products of depth 2 (element s of
            // the lane's A and B float4: columns 2s + lane half)
#pragma unroll
            for (int j = 0; j < RW; ++j)
              if ((m >> j) & 1) {
                const float4 av = af[kk & 1][j];
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) {
                  const float as = s4 == 0 ? av.x : s4 == 1 ? av.y : s4 == 2 ? av.z : av.w;
#pragma unroll
                  for (int ct = 0; ct < CT; ++ct) {
                    const float brs = s4 == 0 ? br[ct].x : s4 == 1 ? br[ct].y : s4 == 2 ? br[ct].z : br[ct].w;
                    const float bis = s4 == 0 ? bi[ct].x : s4 == 1 ? bi[ct].y : s4 == 2 ? bi[ct].z : bi[ct].w;
                    cre[j][ct] = __builtin_amdgcn_mfma_f32_32x32x2f32(as, brs, cre[j][ct], 0, 0, 0);
                    cim[j][ct] = __builtin_amdgcn_mfma_f32_32x32x2f32(as, bis, cim[j][ct], 0, 0, 0);
                  }
                }
              }
          } else {
            bf16x8 rh[CT], ih[CT], rl[CT], il[CT];
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
              rh[ct] = __builtin_bit_cast(bf16x8, src[(ct * NOP + 0) * 64]);
              ih[ct] = __builtin_bit_cast(bf16x8, src[(ct * NOP + 1) * 64]);
              if (SPLIT == 1) {
                rl[ct] = __builtin_bit_cast(bf16x8, src[(ct * NOP + 2) * 64]);
                il[ct] = __builtin_bit_cast(bf16x8, src[(ct * NOP + 3) * 64]);
              }
            }
            // the wave's tiles whose block at this k-step holds a nonzero
#pragma unroll
            for (int j = 0; j < RW; ++j)
              if ((m >> j) & 1) {
                const bf16x8 sh = __builtin_bit_cast(bf16x8, ah[kk & 1][j]);
                const bf16x8 sl = __builtin_bit_cast(bf16x8, al[kk & 1][j]);
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) {
                  cre[j][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sl, rh[ct], cre[j][ct], 0, 0, 0);
                  cim[j][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sl, ih[ct], cim[j][ct], 0, 0, 0);
                  if (SPLIT == 1) {
                    cre[j][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sh, rl[ct], cre[j][ct], 0, 0, 0);
                    cim[j][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sh, il[ct], cim[j][ct], 0, 0, 0);
                  }
                  cre[j][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sh, rh[ct], cre[j][ct], 0, 0, 0);
                  cim[j][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sh, ih[ct], cim[j][ct], 0, 0, 0);
                }
              }
          }
        }
      }
#pragma unroll
      for (int i = 0; i < UPW; ++i) ko_cur[i] = ko_nxt[i];
      __syncthreads();
    }

    // mode-space scatter of the group's tiles
    static_assert(CT == 2, "the scatter takes the two column tiles of 64 samples");
    auto scatter = [&](float2 *O) {
#pragma unroll
      for (int j = 0; j < RW; ++j)
        if (tile[j] >= 0) scatter_tile64(a.pairs, cre[j][0], cim[j][0], cre[j][1], cim[j][1], tile[j], Xs, O, lane);
    };
    // wave w scatters into partial w % NPART in turn w / NPART; the waves
    // sharing a partial take turns, separated by barriers
    constexpr int turns = NW / NPART;
    const int part = w % NPART, turn = w / NPART;
#pragma unroll 1
    for (int s = 0; s < turns; ++s) {
      if (turn == s) scatter(Os + part * MT);
      if (turns > 1) __syncthreads();
    }
  }
}

template <int TT, int RW, int NPART, int KC, int SPLIT, int STAGE>
__global__ __launch_bounds__(64 * NW) void kerr_group(GArgs a) {
  constexpr int NT = 64 * NW;
  extern __shared__ float2 sh[];
  const int MT = a.M * TT;
  float2 *Xs = sh;
  float2 *Os = sh + MT;                        // NPART partial tiles
  uint4 *Bs = (uint4 *)(Os + NPART * MT);      // [2][KC][TT/32][NOP][64] B operands
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int t0 = blockIdx.x * TT;
  for (int idx = threadIdx.x; idx < MT; idx += NT) {
    const size_t g = (size_t)(idx / TT) * a.T + t0 + (idx % TT);
    float2 v = a.src0[g];
    if (STAGE == STAGE_K2 || STAGE == STAGE_K23) v = caxpy(v, 0.5f, a.src1[g]);
    if (STAGE == STAGE_K3) v = caxpy(v, 0.5f, a.src2[g]);
    Xs[idx] = v;
  }
  for (int idx = threadIdx.x; idx < NPART * MT; idx += NT) Os[idx] = make_float2(0.f, 0.f);
  __syncthreads();
  contract<TT, RW, NPART, KC, SPLIT>(a, Xs, Os, Bs, w, lane);
  __syncthreads();
  for (int idx = threadIdx.x; idx < MT; idx += NT) {
    const size_t g = (size_t)(idx / TT) * a.T + t0 + (idx % TT);
    float2 o = Os[idx];
#pragma unroll
    for (int r = 1; r < NPART; ++r) o = cadd(o, Os[r * MT + idx]);
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
    for (int idx = threadIdx.x; idx < NPART * MT; idx += NT) Os[idx] = make_float2(0.f, 0.f);
    __syncthreads();
    contract<TT, RW, NPART, KC, SPLIT>(a, Xs, Os, Bs, w, lane);
    __syncthreads();
    for (int idx = threadIdx.x; idx < MT; idx += NT) {
      const size_t g = (size_t)(idx / TT) * a.T + t0 + (idx % TT);
      float2 o = Os[idx];
#pragma unroll
      for (int r = 1; r < NPART; ++r) o = cadd(o, Os[r * MT + idx]);
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

// Workgroup shape: 64 samples, k-chunks of 2 listed k-steps, and as many
// partial output tiles as LDS holds: (1 + NPART) M 64 8 + 32768 bytes <= 160
// KiB, i.e. four partials up to 51 modes, two up to 85, one up to 128.
// Tiles per wave: 4 (256 accumulator registers) with a partial tile per wave;
// 3 when waves share partials (the turn-taking scatter needs the registers).
constexpr int kTT = 64, kKC = 2;

constexpr size_t kLdsMax = 160 * 1024;

// LDS of a workgroup: field tile, NPART partial output tiles, two B buffers
// (sized for the three-product split, the largest)
size_t lds_bytes(int M, int npart) {
  return (size_t)(1 + npart) * M * kTT * sizeof(float2) + (size_t)2 * kKC * (kTT / 32) * 4 * 64 * sizeof(uint4);
}

// partial output tiles: as many as LDS holds (4, 2 or 1; 0 = does not fit)
int group_partials(int M) {
  for (int n : {4, 2, 1})
    if (lds_bytes(M, n) <= kLdsMax) return n;
  return 0;
}
int group_tiles_per_wave(int M) { return group_partials(M) == 4 ? 4 : 3; }

template <int TT, int RW, int NPART, int KC, int SPLIT>
hipError_t go(const GArgs &a, KerrStage st, hipStream_t s) {
  const dim3 grid(a.T / TT), block(64 * NW);
  const size_t shm = lds_bytes(a.M, NPART);
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
    case STAGE_PLAIN: return launch(kerr_group<TT, RW, NPART, KC, SPLIT, STAGE_PLAIN>);
    case STAGE_K2: return launch(kerr_group<TT, RW, NPART, KC, SPLIT, STAGE_K2>);
    case STAGE_K3: return launch(kerr_group<TT, RW, NPART, KC, SPLIT, STAGE_K3>);
    case STAGE_K4: return launch(kerr_group<TT, RW, NPART, KC, SPLIT, STAGE_K4>);
    case STAGE_K23: return launch(kerr_group<TT, RW, NPART, KC, SPLIT, STAGE_K23>);
  }
  return hipErrorInvalidValue;
}

template <int SPLIT>
hipError_t go_shape(const GArgs &a, KerrStage st, hipStream_t s) {
  switch (group_partials(a.M)) {
    case 4: return go<kTT, 4, 4, kKC, SPLIT>(a, st, s);
    case 2: return go<kTT, 3, 2, kKC, SPLIT>(a, st, s);
    default: return go<kTT, 3, 1, kKC, SPLIT>(a, st, s);
  }
}

}  // namespace

// Build the group tables of the kernel for plan pl from the contraction plan
// kp (FP32 or split, as kp was built); the A operand and pair tables of
// setup_mfma are shared.  Leaves pl.ngroups == 0 when the kernel does not
// apply: it needs 64 samples per workgroup, LDS for M modes, and a tensor
// whose group blocks are nearly all nonzero.
hipError_t setup_groups(Plan &pl, const KerrPlan &kp) {
  const bool split = pl.precision != MMNLSE_FP32;
  if (group_partials(pl.M) == 0 || pl.T % kTT != 0 || kp.nrt == 0) return hipSuccess;
  bool force = false;
  if (const char *env = std::getenv("MMNLSE_GROUP_KERNEL")) {
    if (env[0] == '0') return hipSuccess;
    force = env[0] == '1';
  }
  KerrGroups g;
  plan_groups(kp, NW, group_tiles_per_wave(pl.M), kKC, g);
  // The kernel keeps the four waves of a workgroup in step (one barrier per
  // chunk) and skips zero blocks only per wave and k-step, so on a strongly
  // masked tensor the waves idle at the barriers behind the busiest one and
  // on the branches around skipped blocks; there the per-pass kernel of
  // kerr_mfma.hip is faster (measured on the 70 %-masked 36-mode tensor,
  // whose group blocks are 61 % nonzero: split 2.04 vs 1.72 ms per step,
  // FP32 3.53 vs 2.84).  The group kernel is used when at least 90 % of the
  // blocks of the groups' listed k-steps are nonzero (dense 120-mode tensor:
  // split 449 -> 297 ms per step, FP32 935 -> 893).  MMNLSE_GROUP_KERNEL=1
  // uses it for every tensor, =0 for none.
  double listed_blocks = 0;
  for (int gi = 0; gi < g.ngroups; ++gi) {
    int n = 0;
    for (int j = 0; j < NW * g.rw; ++j) n += g.tiles[(size_t)gi * NW * g.rw + j] >= 0;
    listed_blocks += (double)g.range[gi].y * n;
  }
  if (!force && g.blocks < 0.9 * listed_blocks) return hipSuccess;
  // column modes, 8 bits each, in the order a lane half forms them: k-step ks
  // of kw columns, half h, element e: column kw ks + (split ? 8 h + e : 2 e + h);
  // two columns per word (a, b, a', b')
  const int kw = kp.kw, ne = kw / 2;
  std::vector<uint32_t> modes((size_t)kp.Ppad / 2, 0u);
  for (int ks = 0; ks < kp.nk; ++ks)
    for (int h = 0; h < 2; ++h)
      for (int e = 0; e < ne; ++e) {
        const int q = kw * ks + (split ? 8 * h + e : 2 * e + h);
        const size_t word = ((size_t)ks * 2 + h) * (ne / 2) + e / 2;
        modes[word] |= ((uint32_t)kp.a[q] | (uint32_t)kp.b[q] << 8) << (16 * (e % 2));
      }
  std::vector<int2> list = g.list;
  if (list.empty()) list.push_back(make_int2(0, 0));
  hipError_t e;
  auto alloc_copy = [&](void **dst, const void *src, size_t bytes) -> hipError_t {
    hipError_t r = hipMalloc(dst, bytes);
    if (r != hipSuccess) return r;
    pl.bytes += bytes;
    return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
  };
  if ((e = alloc_copy((void **)&pl.gtiles, g.tiles.data(), sizeof(int32_t) * g.tiles.size())) != hipSuccess) return e;
  if ((e = alloc_copy((void **)&pl.glist, list.data(), sizeof(int2) * list.size())) != hipSuccess) return e;
  if ((e = alloc_copy((void **)&pl.grange, g.range.data(), sizeof(int2) * g.range.size())) != hipSuccess) return e;
  if ((e = alloc_copy((void **)&pl.gkoff, modes.data(), sizeof(uint32_t) * modes.size())) != hipSuccess) return e;
  pl.ngroups = g.ngroups;
  pl.g_tt = kTT;
  pl.kerr_entries[1] = g.blocks * 32.0 * kw;
  return hipSuccess;
}

hipError_t launch_kerr_group(const Plan &pl, double h, const KerrLaunch &k) {
  GArgs a;
  a.src0 = k.src0;
  a.src1 = k.src1;
  a.src2 = k.src2;
  a.out0 = k.out0;
  a.out1 = k.out1;
  a.Ah = (const uint4 *)pl.Sph;
  a.Al = (const uint4 *)pl.Spl;
  a.A32 = (const float4 *)pl.Sp;
  a.pairs = pl.pairs;
  a.kmodes = pl.gkoff;
  a.gtiles = pl.gtiles;
  a.glist = pl.glist;
  a.grange = pl.grange;
  a.hg = (float)(h * pl.gamma);
  a.M = pl.M;
  a.T = pl.T;
  a.P = pl.mfma_rows;
  a.nk = pl.Ppad / (pl.precision == MMNLSE_FP32 ? 8 : 16);
  a.ngroups = pl.ngroups;
  a.next = k.next;
  if (pl.T % pl.g_tt != 0) return hipErrorInvalidValue;
  if (pl.precision == MMNLSE_SPLIT_BF16_S) return go_shape<2>(a, k.stage, pl.stream);
  if (pl.precision == MMNLSE_SPLIT_BF16) return go_shape<1>(a, k.stage, pl.stream);
  return go_shape<0>(a, k.stage, pl.stream);
}

}  // namespace mmnlse
