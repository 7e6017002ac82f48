// Kerr increment h N(X), N_p = i gamma sum_{l,m,n} S_plmn X_l X_m conj(X_n)
// (the bracketed nonlinear terms of Eq. 6b-6e), evaluated pointwise in time:
// every sample t couples all modes, which is the column access the paper's
// nonlinear kernels stage through shared memory (Section 4.4).
//
// The RK4 stage combinations of Eq. 6c-6f are fused into the prologue (the
// argument A_I + k/2) and the epilogue (A_I + k3, A_I + k1/6 + k2/3 + k3/3,
// A = D(..) + k4/6) so they cost no extra pass over the fields.
//
// Two kernels here, both for any real S:
//   kerr_small<M>  M <= 8: one thread per sample, all modes in registers,
//                  S read through the scalar cache (wave-uniform indices).
//   kerr_tiled     any M <= 128: a workgroup stages 64 samples of all modes
//                  in LDS; each wave computes whole modes p.
// The packed matrix-core contraction for symmetric S is in kerr_mfma.hip.

#include "common.h"

namespace mmnlse {
namespace {

struct KArgs {
  const float2 *src0, *src1, *src2;
  float2 *out0, *out1;
  const float *Sg;     // [p][n][m][l]
  const float *kappa;  // [a][b] (Manakov form)
  float hg;         // h * gamma
  int M, T, next;
};

// ---------------------------------------------------------------------------
// small M
// ---------------------------------------------------------------------------
template <int M>
__device__ __forceinline__ void eval_small(const float *__restrict__ Sg, float hg, const float2 (&x)[M],
                                           float2 (&k)[M]) {
#pragma unroll
  for (int p = 0; p < M; ++p) {
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int n = 0; n < M; ++n) {
      float2 an = make_float2(0.f, 0.f);
#pragma unroll
      for (int m = 0; m < M; ++m) {
        const float *s = Sg + ((p * M + n) * M + m) * M;
        float2 am = make_float2(0.f, 0.f);
#pragma unroll
        for (int l = 0; l < M; ++l) {
          am.x = fmaf(s[l], x[l].x, am.x);
          am.y = fmaf(s[l], x[l].y, am.y);
        }
        an = cfma(an, am, x[m]);
      }
      acc = cfma_conj(acc, an, x[n]);
    }
    k[p] = make_float2(-hg * acc.y, hg * acc.x);  // i * h * gamma * acc
  }
}

template <int M, int STAGE>
__global__ __launch_bounds__(256) void kerr_small(KArgs a) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= a.T) return;
  float2 x[M], k[M];
#pragma unroll
  for (int p = 0; p < M; ++p) {
    const size_t g = (size_t)p * a.T + t;
    float2 v = a.src0[g];
    if (STAGE == STAGE_K2 || STAGE == STAGE_K23) v = caxpy(v, 0.5f, a.src1[g]);
    if (STAGE == STAGE_K3) v = caxpy(v, 0.5f, a.src2[g]);
    x[p] = v;
  }
  eval_small<M>(a.Sg, a.hg, x, k);
  if (STAGE == STAGE_K23) {  // k3 from A_I + k2/2; k2 stays in registers
    float2 k2[M];
#pragma unroll
    for (int p = 0; p < M; ++p) {
      k2[p] = k[p];
      x[p] = caxpy(a.src0[(size_t)p * a.T + t], 0.5f, k2[p]);
    }
    eval_small<M>(a.Sg, a.hg, x, k);
#pragma unroll
    for (int p = 0; p < M; ++p) {
      const size_t g = (size_t)p * a.T + t;
      const float2 ai = a.src0[g], k1 = a.src1[g];
      a.out0[g] = cadd(ai, k[p]);
      float2 z = caxpy(ai, 1.f / 6.f, k1);
      z = caxpy(z, 1.f / 3.f, k2[p]);
      a.out1[g] = caxpy(z, 1.f / 3.f, k[p]);
    }
    return;
  }
#pragma unroll
  for (int p = 0; p < M; ++p) {
    const size_t g = (size_t)p * a.T + t;
    if (STAGE == STAGE_PLAIN || STAGE == STAGE_K2) {
      a.out0[g] = k[p];
    } else if (STAGE == STAGE_K3) {
      const float2 ai = a.src0[g], k1 = a.src1[g], k2 = a.src2[g];
      a.out0[g] = cadd(ai, k[p]);
      float2 z = caxpy(ai, 1.f / 6.f, k1);
      z = caxpy(z, 1.f / 3.f, k2);
      a.out1[g] = caxpy(z, 1.f / 3.f, k[p]);
    } else {  // STAGE_K4
      x[p] = caxpy(a.src1[g], 1.f / 6.f, k[p]);
      a.out0[g] = x[p];
    }
  }
  if (STAGE == STAGE_K4 && a.next) {
    eval_small<M>(a.Sg, a.hg, x, k);
#pragma unroll
    for (int p = 0; p < M; ++p) a.out1[(size_t)p * a.T + t] = k[p];
  }
}

// ---------------------------------------------------------------------------
// LDS-tiled, any M
// ---------------------------------------------------------------------------
constexpr int TT = 64;   // samples per workgroup
constexpr int GW = 4;    // waves per workgroup

__device__ __forceinline__ void eval_tiled(const KArgs &a, const float2 *Xs, float2 *Ks, int w,
                                           int lane) {
  const int M = a.M;
  for (int p0 = w; p0 < M; p0 += GW) {
    const int p = __builtin_amdgcn_readfirstlane(p0);
    float2 acc = make_float2(0.f, 0.f);
    for (int n = 0; n < M; ++n) {
      float2 an = make_float2(0.f, 0.f);
      for (int m = 0; m < M; ++m) {
        const float *__restrict__ s = a.Sg + ((size_t)(p * M + n) * M + m) * M;
        float2 am = make_float2(0.f, 0.f);
        for (int l = 0; l < M; ++l) {
          const float2 xl = Xs[l * TT + lane];
          const float sv = s[l];
          am.x = fmaf(sv, xl.x, am.x);
          am.y = fmaf(sv, xl.y, am.y);
        }
        an = cfma(an, am, Xs[m * TT + lane]);
      }
      acc = cfma_conj(acc, an, Xs[n * TT + lane]);
    }
    Ks[p * TT + lane] = make_float2(-a.hg * acc.y, a.hg * acc.x);
  }
}

template <int STAGE>
__global__ __launch_bounds__(TT * GW) void kerr_tiled(KArgs a) {
  extern __shared__ float2 sh[];
  float2 *Xs = sh;
  float2 *Ks = sh + a.M * TT;
  const int t0 = blockIdx.x * TT;
  const int lane = threadIdx.x & (TT - 1);
  const int w = threadIdx.x / TT;
  for (int idx = threadIdx.x; idx < a.M * TT; idx += TT * GW) {
    const size_t g = (size_t)(idx / TT) * a.T + t0 + (idx % TT);
    float2 v = a.src0[g];
    if (STAGE == STAGE_K2) v = caxpy(v, 0.5f, a.src1[g]);
    if (STAGE == STAGE_K3) v = caxpy(v, 0.5f, a.src2[g]);
    Xs[idx] = v;
  }
  __syncthreads();
  eval_tiled(a, Xs, Ks, w, lane);
  __syncthreads();
  for (int p = w; p < a.M; p += GW) {
    const size_t g = (size_t)p * a.T + t0 + lane;
    const float2 k = Ks[p * TT + lane];
    if (STAGE == STAGE_PLAIN || STAGE == STAGE_K2) {
      a.out0[g] = k;
    } else if (STAGE == STAGE_K3) {
      const float2 ai = a.src0[g], k1 = a.src1[g], k2 = a.src2[g];
      a.out0[g] = cadd(ai, k);
      float2 z = caxpy(ai, 1.f / 6.f, k1);
      z = caxpy(z, 1.f / 3.f, k2);
      a.out1[g] = caxpy(z, 1.f / 3.f, k);
    } else {
      const float2 An = caxpy(a.src1[g], 1.f / 6.f, k);
      a.out0[g] = An;
      Xs[p * TT + lane] = An;
    }
  }
  if (STAGE == STAGE_K4 && a.next) {
    __syncthreads();
    eval_tiled(a, Xs, Ks, w, lane);
    __syncthreads();
    for (int p = w; p < a.M; p += GW) a.out1[(size_t)p * a.T + t0 + lane] = Ks[p * TT + lane];
  }
}

// ---------------------------------------------------------------------------
// Manakov / XPM form of Eq. (1): k_a = i h gamma (sum_b kappa_ab |X_b|^2) X_a.
// A workgroup stages the intensities |X_b|^2 of 64 samples of all modes in
// LDS; each wave takes whole modes a (wave-uniform row of kappa through the
// scalar cache).  Up to 256 modes (two 64 KiB intensity tiles).
// ---------------------------------------------------------------------------
template <int STAGE>
__device__ __forceinline__ float2 stage_arg(const KArgs &a, size_t g) {
  float2 v = a.src0[g];
  if (STAGE == STAGE_K2) v = caxpy(v, 0.5f, a.src1[g]);
  if (STAGE == STAGE_K3) v = caxpy(v, 0.5f, a.src2[g]);
  return v;
}

__device__ __forceinline__ float xpm_phase(const KArgs &a, const float *Is, int p, int lane) {
  const float *__restrict__ k = a.kappa + (size_t)p * a.M;
  float phi = 0.f;
  for (int b = 0; b < a.M; ++b) phi = fmaf(k[b], Is[b * TT + lane], phi);
  return phi;
}

template <int STAGE>
__global__ __launch_bounds__(TT * GW) void kerr_manakov(KArgs a) {
  extern __shared__ float shf[];
  float *Is = shf;                // |X_b|^2 of the stage argument
  float *Is2 = shf + a.M * TT;    // K4: |A(z+h)|^2 for the next step's k1; K23: |A_I + k2/2|^2
  const int t0 = blockIdx.x * TT;
  const int lane = threadIdx.x & (TT - 1);
  const int w = threadIdx.x / TT;
  for (int idx = threadIdx.x; idx < a.M * TT; idx += TT * GW) {
    const float2 v = stage_arg<STAGE == STAGE_K23 ? STAGE_K2 : STAGE>(a, (size_t)(idx / TT) * a.T + t0 + (idx % TT));
    Is[idx] = fmaf(v.x, v.x, v.y * v.y);
  }
  __syncthreads();
  if (STAGE == STAGE_K23) {
    // k2 = h N(A_I + k1/2) for every mode of the tile (kept in out1), then
    // k3 = h N(A_I + k2/2) from the intensities of that second argument;
    // the same arithmetic as a K2 launch followed by a K3 launch.  out0 is
    // src1 (k1): each element's k1 is read before its out0 is written, and
    // the staging above read every mode's k1 before the barrier.
    for (int p0 = w; p0 < a.M; p0 += GW) {
      const int p = __builtin_amdgcn_readfirstlane(p0);
      const float hphi = a.hg * xpm_phase(a, Is, p, lane);
      const size_t g = (size_t)p * a.T + t0 + lane;
      const float2 ai = a.src0[g];
      const float2 x = caxpy(ai, 0.5f, a.src1[g]);
      const float2 k2 = make_float2(-hphi * x.y, hphi * x.x);
      a.out1[g] = k2;
      const float2 x3 = caxpy(ai, 0.5f, k2);
      Is2[p * TT + lane] = fmaf(x3.x, x3.x, x3.y * x3.y);
    }
    __syncthreads();
    for (int p0 = w; p0 < a.M; p0 += GW) {
      const int p = __builtin_amdgcn_readfirstlane(p0);
      const float hphi = a.hg * xpm_phase(a, Is2, p, lane);
      const size_t g = (size_t)p * a.T + t0 + lane;
      const float2 ai = a.src0[g], k1 = a.src1[g], k2 = a.out1[g];  // k2: this thread's own write
      const float2 x3 = caxpy(ai, 0.5f, k2);
      const float2 k3 = make_float2(-hphi * x3.y, hphi * x3.x);
      a.out0[g] = cadd(ai, k3);
      float2 z = caxpy(ai, 1.f / 6.f, k1);
      z = caxpy(z, 1.f / 3.f, k2);
      a.out1[g] = caxpy(z, 1.f / 3.f, k3);
    }
    return;
  }
  for (int p0 = w; p0 < a.M; p0 += GW) {
    const int p = __builtin_amdgcn_readfirstlane(p0);
    const float hphi = a.hg * xpm_phase(a, Is, p, lane);
    const size_t g = (size_t)p * a.T + t0 + lane;
    const float2 x = stage_arg<STAGE>(a, g);
    const float2 k = make_float2(-hphi * x.y, hphi * x.x);
    if (STAGE == STAGE_PLAIN || STAGE == STAGE_K2) {
      a.out0[g] = k;
    } else if (STAGE == STAGE_K3) {
      const float2 ai = a.src0[g], k1 = a.src1[g], k2 = a.src2[g];
      a.out0[g] = cadd(ai, k);
      float2 z = caxpy(ai, 1.f / 6.f, k1);
      z = caxpy(z, 1.f / 3.f, k2);
      a.out1[g] = caxpy(z, 1.f / 3.f, k);
    } else {
      const float2 An = caxpy(a.src1[g], 1.f / 6.f, k);
      a.out0[g] = An;
      Is2[p * TT + lane] = fmaf(An.x, An.x, An.y * An.y);
    }
  }
  if (STAGE == STAGE_K4 && a.next) {
    __syncthreads();
    for (int p0 = w; p0 < a.M; p0 += GW) {
      const int p = __builtin_amdgcn_readfirstlane(p0);
      const float hphi = a.hg * xpm_phase(a, Is2, p, lane);
      const size_t g = (size_t)p * a.T + t0 + lane;
      const float2 An = a.out0[g];  // written by this thread above
      a.out1[g] = make_float2(-hphi * An.y, hphi * An.x);
    }
  }
}

// Nonlinear step of the split-step with the iterated trapezoidal rule for
// the Manakov form (Eq. 4 with Eq. 1's operator): the exponential of the
// integrated operator is a phase rotation per mode,
//   out0 = src1 * exp(i (h gamma / 2) sum_b kappa_ab (|src0_b|^2 + |src2_b|^2)),
// src0 = A(z), src2 = the current estimate of A(z+h), src1 = D A(z).  A
// workgroup owns 64 samples of every mode and stages the intensities in LDS
// before writing, so out0 may be src0 or src2.
__global__ __launch_bounds__(TT * GW) void manakov_phase(KArgs a) {
  extern __shared__ float shf[];
  float *Is = shf;  // |A(z)|^2 + |A_end|^2
  const int t0 = blockIdx.x * TT;
  const int lane = threadIdx.x & (TT - 1);
  const int w = threadIdx.x / TT;
  for (int idx = threadIdx.x; idx < a.M * TT; idx += TT * GW) {
    const size_t g = (size_t)(idx / TT) * a.T + t0 + (idx % TT);
    const float2 u = a.src0[g], v = a.src2[g];
    Is[idx] = fmaf(u.x, u.x, u.y * u.y) + fmaf(v.x, v.x, v.y * v.y);
  }
  __syncthreads();
  for (int p0 = w; p0 < a.M; p0 += GW) {
    const int p = __builtin_amdgcn_readfirstlane(p0);
    const float ang = 0.5f * a.hg * xpm_phase(a, Is, p, lane);
    float sn, cs;
    sincosf(ang, &sn, &cs);
    const size_t g = (size_t)p * a.T + t0 + lane;
    const float2 x = a.src1[g];
    a.out0[g] = make_float2(x.x * cs - x.y * sn, x.x * sn + x.y * cs);
  }
}

hipError_t go_manakov(const KArgs &a, KerrStage st, hipStream_t s) {
  dim3 grid(a.T / TT);
  const size_t shm = (size_t)(st == STAGE_K4 || st == STAGE_K23 ? 2 : 1) * a.M * TT * sizeof(float);
  auto launch = [&](auto kern) -> hipError_t {
    hipError_t e = check_launch((const void *)kern, TT * GW, shm);
    if (e != hipSuccess) return e;
    if (shm > 65536) {
      e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, grid, dim3(TT * GW), shm, s, a);
    return hipGetLastError();
  };
  switch (st) {
    case STAGE_PLAIN: return launch(kerr_manakov<STAGE_PLAIN>);
    case STAGE_K2: return launch(kerr_manakov<STAGE_K2>);
    case STAGE_K3: return launch(kerr_manakov<STAGE_K3>);
    case STAGE_K4: return launch(kerr_manakov<STAGE_K4>);
    case STAGE_K23: return launch(kerr_manakov<STAGE_K23>);
  }
  return hipErrorInvalidValue;
}

template <int M>
hipError_t go_small(const KArgs &a, KerrStage st, hipStream_t s) {
  dim3 grid((a.T + 255) / 256);
  switch (st) {
    case STAGE_PLAIN: hipLaunchKernelGGL((kerr_small<M, STAGE_PLAIN>), grid, dim3(256), 0, s, a); break;
    case STAGE_K2: hipLaunchKernelGGL((kerr_small<M, STAGE_K2>), grid, dim3(256), 0, s, a); break;
    case STAGE_K3: hipLaunchKernelGGL((kerr_small<M, STAGE_K3>), grid, dim3(256), 0, s, a); break;
    case STAGE_K4: hipLaunchKernelGGL((kerr_small<M, STAGE_K4>), grid, dim3(256), 0, s, a); break;
    case STAGE_K23: hipLaunchKernelGGL((kerr_small<M, STAGE_K23>), grid, dim3(256), 0, s, a); break;
  }
  return hipGetLastError();
}

hipError_t go_tiled(const KArgs &a, KerrStage st, hipStream_t s) {
  dim3 grid(a.T / TT);
  const size_t shm = (size_t)2 * a.M * TT * sizeof(float2);
  auto launch = [&](auto kern) -> hipError_t {
    hipError_t e = check_launch((const void *)kern, TT * GW, shm);
    if (e != hipSuccess) return e;
    if (shm > 65536) {
      e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, grid, dim3(TT * GW), shm, s, a);
    return hipGetLastError();
  };
  switch (st) {
    case STAGE_PLAIN: return launch(kerr_tiled<STAGE_PLAIN>);
    case STAGE_K2: return launch(kerr_tiled<STAGE_K2>);
    case STAGE_K3: return launch(kerr_tiled<STAGE_K3>);
    case STAGE_K4: return launch(kerr_tiled<STAGE_K4>);
    default: break;
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_kerr_mfma(const Plan &pl, double h, const KerrLaunch &k);

hipError_t launch_manakov_phase(const Plan &pl, double h, const float2 *Az, const float2 *Aend,
                                const float2 *DA, float2 *out) {
  KArgs a{};
  a.src0 = Az;
  a.src1 = DA;
  a.src2 = Aend;
  a.out0 = out;
  a.kappa = pl.kappa;
  a.hg = (float)(h * pl.gamma);
  a.M = pl.M;
  a.T = pl.T;
  const size_t shm = (size_t)a.M * TT * sizeof(float);
  hipError_t e = check_launch((const void *)manakov_phase, TT * GW, shm);
  if (e != hipSuccess) return e;
  if (shm > 65536) {
    e = hipFuncSetAttribute((const void *)manakov_phase, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(manakov_phase, dim3(a.T / TT), dim3(TT * GW), shm, pl.stream, a);
  return hipGetLastError();
}

hipError_t launch_kerr(const Plan &pl, double h, const KerrLaunch &k) {
  if (pl.kerr_path == KERR_MFMA) return launch_kerr_mfma(pl, h, k);
  KArgs a;
  a.src0 = k.src0;
  a.src1 = k.src1;
  a.src2 = k.src2;
  a.out0 = k.out0;
  a.out1 = k.out1;
  a.Sg = pl.Sg;
  a.kappa = pl.kappa;
  a.hg = (float)(h * pl.gamma);
  a.M = pl.M;
  a.T = pl.T;
  a.next = k.next;
  if (pl.kerr_path == KERR_MANAKOV) return go_manakov(a, k.stage, pl.stream);
  if (pl.kerr_path == KERR_SMALL) {
    switch (pl.M) {
      case 1: return go_small<1>(a, k.stage, pl.stream);
      case 2: return go_small<2>(a, k.stage, pl.stream);
      case 3: return go_small<3>(a, k.stage, pl.stream);
      case 4: return go_small<4>(a, k.stage, pl.stream);
      case 5: return go_small<5>(a, k.stage, pl.stream);
      case 6: return go_small<6>(a, k.stage, pl.stream);
      case 7: return go_small<7>(a, k.stage, pl.stream);
      case 8: return go_small<8>(a, k.stage, pl.stream);
    }
    return hipErrorInvalidValue;
  }
  return go_tiled(a, k.stage, pl.stream);
}

}  // namespace mmnlse
