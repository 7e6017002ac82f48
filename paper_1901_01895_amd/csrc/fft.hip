// Half-step linear propagator D = exp(h/2 L) applied per mode in the
// frequency domain (Eq. 6a, 6b, 6e, 6f; Section 3.1 of the paper):
// forward FFT -> multiply by E = exp(h/2 L)/T -> inverse FFT.
//
// FFTs are Stockham radix-4 (plus one radix-2 stage for odd log2 sizes) on
// data staged in LDS, FP32 arithmetic.  Every twiddle and every propagator
// factor is an FP32 hi + lo pair tabulated in FP64, multiplied with
// cmul_hilo, so no factor carries a fixed rounding bias from one step to the
// next (a biased twiddle turns into a gain error that grows linearly with the
// number of round trips).
//
// T <= 2^14: one workgroup transforms whole rows in LDS, multiplies and
// transforms back (one HBM read + one write per field).
// T >= 2^15 (or when forced): four-step with T = N1*N2, time index
// n = N2*n1 + n2, frequency f = k1 + N1*k2:
//   pass A: per column n2, FFT over n1 (stride N2), times W_T^(n2*k1)
//   pass B: per row k1, FFT over n2 (contiguous), times E (tabulated in this
//           transposed bin order), inverse FFT over k2
//   pass C: times W_T^(-n2*k1), inverse FFT over k1 per column
// All passes work in place, each workgroup owning disjoint elements.
// launch_linear_twice applies D twice from one forward transform (pass A,
// pass B writing the spectrum times E and times E twice, pass C on both).
// The twiddles of an L-point transform in the four-step passes are the
// entries W_L^j = W_T^(j T/L) of the table; a workgroup copies those L
// entries to LDS first (at most 16 KB) so that its butterflies read them
// there instead of through the vector memory path.

#include "common.h"

namespace mmnlse {
namespace {

constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x >> 1); }

template <bool INV>
__device__ __forceinline__ void dft4(float2 &a0, float2 &a1, float2 &a2, float2 &a3) {
  float2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = csub(a1, a3);
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  // forward: W4 = -i, so y1 = t1 - i t3, y3 = t1 + i t3; inverse swaps them
  float2 mi_t3 = make_float2(t3.y, -t3.x);
  if (!INV) {
    a1 = cadd(t1, mi_t3);
    a3 = csub(t1, mi_t3);
  } else {
    a1 = csub(t1, mi_t3);
    a3 = cadd(t1, mi_t3);
  }
}

// One Stockham stage of radix R on NB sequences of length L in LDS.
// Element i of sequence b lives at buf[b*BS + i*ES].  Ns = size of the
// sub-transforms already done; twiddle W_{Ns*R}^(r*k) = W_T^((r*k) << sh)
// with sh = logT - log2(Ns*R).
template <int R, int L, int NB, int ES, int BS, int NT, bool INV>
__device__ __forceinline__ void stockham_stage(float2 *buf, int Ns, int sh,
                                               const float4 *__restrict__ tw) {
  constexpr int U = NB * (L / R);
  constexpr int PER = (U + NT - 1) / NT;
  float2 v[PER][R];
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int u = tid + q * NT;
    if (PER * NT == U || u < U) {
      int j, b;
      if (ES == 1) { j = u % (L / R); b = u / (L / R); }
      else { b = u % NB; j = u / NB; }
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = buf[b * BS + (j + r * (L / R)) * ES];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int u = tid + q * NT;
    if (PER * NT == U || u < U) {
      int j, b;
      if (ES == 1) { j = u % (L / R); b = u / (L / R); }
      else { b = u % NB; j = u / NB; }
      const int k = j & (Ns - 1);
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float4 w = tw[(r * k) << sh];
          if (INV) w = conj_hilo(w);
          v[q][r] = cmul_hilo(v[q][r], w);
        }
      }
      if (R == 4) {
        dft4<INV>(v[q][0], v[q][1], v[q][2], v[q][3]);
      } else {
        float2 a = v[q][0], c = v[q][1];
        v[q][0] = cadd(a, c);
        v[q][1] = csub(a, c);
      }
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[b * BS + (base + r * Ns) * ES] = v[q][r];
    }
  }
  __syncthreads();
}

// Full FFT (unnormalised) of NB sequences of length L in LDS.
template <int L, int NB, int ES, int BS, int NT, bool INV>
__device__ __forceinline__ void lds_fft(float2 *buf, const float4 *__restrict__ tw, int logT) {
  constexpr int LOG = ilog2c(L);
  int Ns = 1, logNs = 0;
#pragma unroll
  for (int s = 0; s < LOG / 2; ++s) {
    stockham_stage<4, L, NB, ES, BS, NT, INV>(buf, Ns, logT - (logNs + 2), tw);
    Ns <<= 2;
    logNs += 2;
  }
  if (LOG & 1) stockham_stage<2, L, NB, ES, BS, NT, INV>(buf, Ns, logT - (logNs + 1), tw);
}

// twl[j] = tw[j << (logT - logL)] = W_L^j for j < L, copied to LDS; the
// stages index it with logL in place of logT and read the same values
template <int L, int NT>
__device__ __forceinline__ void load_twiddles(float4 *twl, const float4 *__restrict__ tw, int logT) {
  constexpr int LOG = ilog2c(L);
  for (int j = threadIdx.x; j < L; j += NT) twl[j] = tw[(size_t)j << (logT - LOG)];
}

// two consecutive complex samples as one 16-byte access (fields are
// 16-byte aligned, every pair starts at an even sample index)
__device__ __forceinline__ float4 ld2(const float2 *p) { return *reinterpret_cast<const float4 *>(p); }
__device__ __forceinline__ void st2(float2 *p, float4 v) { *reinterpret_cast<float4 *>(p) = v; }

struct LinArgs {
  const float2 *in[2];
  float2 *out[2];
  const float4 *E;
  const float4 *tw;
  const float4 *twc;  // four-step column-pass twiddles in access order
  int M, T, logT;
  int N1, N2;
};

// ---------------------------------------------------------------------------
// single pass: NB whole rows of length L per workgroup
// ---------------------------------------------------------------------------
template <int L, int NB, int NT>
__global__ __launch_bounds__(NT) void linear_single(LinArgs a) {
  __shared__ __align__(16) float2 buf[L * NB];
  const int job = blockIdx.y;
  const float2 *__restrict__ in = a.in[job];
  float2 *__restrict__ out = a.out[job];
  const int row0 = blockIdx.x * NB;
  // two samples (16 bytes) per access; L is even, so a pair never straddles rows
  for (int idx = 2 * threadIdx.x; idx < L * NB; idx += 2 * NT) {
    const int row = row0 + idx / L;
    const float4 v = row < a.M ? ld2(in + (size_t)row * L + (idx % L)) : make_float4(0.f, 0.f, 0.f, 0.f);
    st2(buf + idx, v);
  }
  __syncthreads();
  lds_fft<L, NB, 1, L, NT, false>(buf, a.tw, a.logT);
  for (int idx = threadIdx.x; idx < L * NB; idx += NT) {
    const int row = row0 + idx / L;
    if (row < a.M) buf[idx] = cmul_hilo(buf[idx], a.E[(size_t)row * L + (idx % L)]);
  }
  __syncthreads();
  lds_fft<L, NB, 1, L, NT, true>(buf, a.tw, a.logT);
  for (int idx = 2 * threadIdx.x; idx < L * NB; idx += 2 * NT) {
    const int row = row0 + idx / L;
    if (row < a.M) st2(out + (size_t)row * L + (idx % L), ld2(buf + idx));
  }
}

// ---------------------------------------------------------------------------
// four-step passes
// ---------------------------------------------------------------------------
constexpr int COLS = kFftCols;  // columns per workgroup in the strided passes

// pass A (INV=false) and pass C (INV=true): C columns of one row
template <int N1, int NT, bool INV>
__global__ __launch_bounds__(NT) void linear_cols(LinArgs a) {
  __shared__ __align__(16) float2 buf[N1 * COLS];
  __shared__ float4 twl[N1];
  load_twiddles<N1, NT>(twl, a.tw, a.logT);
  const int job = blockIdx.y;
  const int cblocks = a.N2 / COLS;
  const int row = blockIdx.x / cblocks;
  const int c0 = (blockIdx.x % cblocks) * COLS;
  const float2 *__restrict__ in = INV ? a.out[job] : a.in[job];
  float2 *__restrict__ out = a.out[job];
  const size_t rbase = (size_t)row * a.T + c0;
  // twc[idx] = W_T^((c0 + c) n1) for idx = n1 COLS + c: read in the order of
  // the samples, 32 contiguous bytes per thread
  const float4 *__restrict__ twc = a.twc + (size_t)(c0 / COLS) * N1 * COLS;
  for (int idx = 2 * threadIdx.x; idx < N1 * COLS; idx += 2 * NT) {
    const int n1 = idx / COLS, c = idx % COLS;  // c even: columns c, c+1
    const float4 v = ld2(in + rbase + (size_t)n1 * a.N2 + c);
    float2 x0 = make_float2(v.x, v.y), x1 = make_float2(v.z, v.w);
    if (INV) {
      x0 = cmul_hilo(x0, conj_hilo(twc[idx]));
      x1 = cmul_hilo(x1, conj_hilo(twc[idx + 1]));
    }
    st2(buf + idx, make_float4(x0.x, x0.y, x1.x, x1.y));
  }
  __syncthreads();
  lds_fft<N1, COLS, COLS, 1, NT, INV>(buf, twl, ilog2c(N1));
  for (int idx = 2 * threadIdx.x; idx < N1 * COLS; idx += 2 * NT) {
    const int k1 = idx / COLS, c = idx % COLS;
    const float4 v = ld2(buf + idx);
    float2 x0 = make_float2(v.x, v.y), x1 = make_float2(v.z, v.w);
    if (!INV) {  // k1 in place of n1: twc[k1 COLS + c] = W_T^((c0 + c) k1)
      x0 = cmul_hilo(x0, twc[idx]);
      x1 = cmul_hilo(x1, twc[idx + 1]);
    }
    st2(out + rbase + (size_t)k1 * a.N2 + c, make_float4(x0.x, x0.y, x1.x, x1.y));
  }
}

// pass B: NB rows k1 of length N2: FFT, times E, inverse FFT.  DUAL (one
// field, out[0]): also the spectrum times E a second time into out[1], i.e.
// the propagator applied twice (E holds 1/T once, so the second factor is
// E * T, exact for T = 2^k)
template <int N2, int NB, int NT, bool DUAL>
__global__ __launch_bounds__(NT) void linear_rows(LinArgs a) {
  __shared__ __align__(16) float2 buf[N2 * NB];
  __shared__ __align__(16) float2 buf2[DUAL ? N2 * NB : 2];
  __shared__ float4 twl[N2];
  load_twiddles<N2, NT>(twl, a.tw, a.logT);
  const int job = blockIdx.y;
  float2 *__restrict__ io = a.out[job];
  const int rows_per_mode = a.N1 / NB;
  const int mode = blockIdx.x / rows_per_mode;
  const size_t base = (size_t)mode * a.T + (size_t)(blockIdx.x % rows_per_mode) * NB * N2;
  for (int idx = 2 * threadIdx.x; idx < N2 * NB; idx += 2 * NT) st2(buf + idx, ld2(io + base + idx));
  __syncthreads();
  lds_fft<N2, NB, 1, N2, NT, false>(buf, twl, ilog2c(N2));
  const float Tf = (float)a.T;
  for (int idx = threadIdx.x; idx < N2 * NB; idx += NT) {
    const float4 e = a.E[base + idx];
    const float2 y = cmul_hilo(buf[idx], e);
    buf[idx] = y;
    if (DUAL) buf2[idx] = cmul_hilo(y, make_float4(e.x * Tf, e.y * Tf, e.z * Tf, e.w * Tf));
  }
  __syncthreads();
  lds_fft<N2, NB, 1, N2, NT, true>(buf, twl, ilog2c(N2));
  if (DUAL) lds_fft<N2, NB, 1, N2, NT, true>(buf2, twl, ilog2c(N2));
  for (int idx = 2 * threadIdx.x; idx < N2 * NB; idx += 2 * NT) st2(io + base + idx, ld2(buf + idx));
  if (DUAL)
    for (int idx = 2 * threadIdx.x; idx < N2 * NB; idx += 2 * NT) st2(a.out[1] + base + idx, ld2(buf2 + idx));
}

// pass B on both fields of a two-field application in one workgroup: each
// propagator factor is read once and applied to the same bin of both (the
// 2 NB rows are transformed as one batch of sequences; per row the
// arithmetic is that of linear_rows)
template <int N2, int NB, int NT>
__global__ __launch_bounds__(NT) void linear_rows_pair(LinArgs a) {
  __shared__ __align__(16) float2 buf[2 * N2 * NB];
  __shared__ float4 twl[N2];
  load_twiddles<N2, NT>(twl, a.tw, a.logT);
  float2 *__restrict__ io0 = a.out[0];
  float2 *__restrict__ io1 = a.out[1];
  const int rows_per_mode = a.N1 / NB;
  const int mode = blockIdx.x / rows_per_mode;
  const size_t base = (size_t)mode * a.T + (size_t)(blockIdx.x % rows_per_mode) * NB * N2;
  for (int idx = 2 * threadIdx.x; idx < N2 * NB; idx += 2 * NT) {
    st2(buf + idx, ld2(io0 + base + idx));
    st2(buf + N2 * NB + idx, ld2(io1 + base + idx));
  }
  __syncthreads();
  lds_fft<N2, 2 * NB, 1, N2, NT, false>(buf, twl, ilog2c(N2));
  for (int idx = threadIdx.x; idx < N2 * NB; idx += NT) {
    const float4 e = a.E[base + idx];
    buf[idx] = cmul_hilo(buf[idx], e);
    buf[N2 * NB + idx] = cmul_hilo(buf[N2 * NB + idx], e);
  }
  __syncthreads();
  lds_fft<N2, 2 * NB, 1, N2, NT, true>(buf, twl, ilog2c(N2));
  for (int idx = 2 * threadIdx.x; idx < N2 * NB; idx += 2 * NT) {
    st2(io0 + base + idx, ld2(buf + idx));
    st2(io1 + base + idx, ld2(buf + N2 * NB + idx));
  }
}

template <int L, int NB, int NT>
hipError_t go_single(const LinArgs &a, int njobs, hipStream_t s) {
  dim3 grid((a.M + NB - 1) / NB, njobs);
  hipLaunchKernelGGL((linear_single<L, NB, NT>), grid, dim3(NT), 0, s, a);
  return hipGetLastError();
}

template <int N1, int NT>
hipError_t go_cols(const LinArgs &a, int njobs, hipStream_t s, bool inv) {
  dim3 grid(a.M * (a.N2 / COLS), njobs);
  if (inv) hipLaunchKernelGGL((linear_cols<N1, NT, true>), grid, dim3(NT), 0, s, a);
  else hipLaunchKernelGGL((linear_cols<N1, NT, false>), grid, dim3(NT), 0, s, a);
  return hipGetLastError();
}

template <int N2, int NB, int NT>
hipError_t go_rows(const LinArgs &a, int njobs, hipStream_t s) {
  // njobs == 0: the DUAL form on out[0] (outputs out[0] and out[1])
  // njobs == 2: both fields in one workgroup (linear_rows_pair)
  const dim3 grid(a.M * (a.N1 / NB));
  if (njobs == 2) hipLaunchKernelGGL((linear_rows_pair<N2, NB, NT>), grid, dim3(NT), 0, s, a);
  else if (njobs == 1) hipLaunchKernelGGL((linear_rows<N2, NB, NT, false>), grid, dim3(NT), 0, s, a);
  else hipLaunchKernelGGL((linear_rows<N2, NB, NT, true>), grid, dim3(NT), 0, s, a);
  return hipGetLastError();
}

hipError_t cols_dispatch(const LinArgs &a, int njobs, hipStream_t s, bool inv) {
  switch (a.N1) {
    case 32: return go_cols<32, 128>(a, njobs, s, inv);
    case 64: return go_cols<64, 256>(a, njobs, s, inv);
    case 128: return go_cols<128, 256>(a, njobs, s, inv);
    case 256: return go_cols<256, 256>(a, njobs, s, inv);
    case 512: return go_cols<512, 512>(a, njobs, s, inv);
    case 1024: return go_cols<1024, 1024>(a, njobs, s, inv);
  }
  return hipErrorInvalidValue;
}

hipError_t rows_dispatch(const LinArgs &a, int njobs, hipStream_t s) {
  // NB rows per workgroup; N1 (rows per mode) is a multiple of NB for every
  // decomposition the plan chooses (N1 >= 32)
  switch (a.N2) {
    case 32: return go_rows<32, 32, 256>(a, njobs, s);
    case 64: return go_rows<64, 16, 256>(a, njobs, s);
    case 128: return go_rows<128, 8, 256>(a, njobs, s);
    case 256: return go_rows<256, 8, 256>(a, njobs, s);
    case 512: return go_rows<512, 4, 256>(a, njobs, s);
    case 1024: return go_rows<1024, 2, 256>(a, njobs, s);
  }
  return hipErrorInvalidValue;
}

hipError_t single_dispatch(const LinArgs &a, int njobs, hipStream_t s) {
  switch (a.T) {
    case 64: return go_single<64, 16, 256>(a, njobs, s);
    case 128: return go_single<128, 8, 256>(a, njobs, s);
    case 256: return go_single<256, 4, 256>(a, njobs, s);
    case 512: return go_single<512, 2, 256>(a, njobs, s);
    case 1024: return go_single<1024, 1, 256>(a, njobs, s);
    case 2048: return go_single<2048, 1, 256>(a, njobs, s);
    case 4096: return go_single<4096, 1, 256>(a, njobs, s);
    case 8192: return go_single<8192, 1, 512>(a, njobs, s);
    case 16384: return go_single<16384, 1, 1024>(a, njobs, s);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// whole RK4IP steps of a one-mode field in one workgroup (64 <= T <= 4096)
//
// With one mode the Kerr term is pointwise, so a step needs nothing from
// other workgroups.  Thread tid owns samples tid + NT j of the field, of the
// carried h N(A) and of the RK4 stages, all in registers; the two transforms
// of each linear half step (A and h N(A), then A_I + k3 and the stage sum)
// run in LDS as two sequences of one Stockham FFT; the T twiddles are copied
// to LDS once per launch and each thread keeps the propagator factors of its
// own bins in registers.  The arithmetic is that of the single-pass linear
// kernel and kerr_small<1> in the same order (Eq. 6a-f), so one launch for
// any number of steps gives the same field as the four-launch schedule on
// the single-pass transform.

struct SoloArgs {
  float2 *A;         // [T] field, in and out
  float2 *N1;        // [T] h N(A) carried between calls (read unless start, written unless finish)
  const float4 *E;   // [T] exp(h/2 L)/T hi + lo, natural bin order
  const float4 *tw;  // [T] W_T^j hi + lo
  const float *S;    // S_0000
  float hg;          // h gamma
  int n_steps, start, finish;
};

template <int L>
constexpr int solo_threads() { return L / 4 < 64 ? 64 : (L / 4 > 1024 ? 1024 : L / 4); }

template <int L, int NT>
__global__ __launch_bounds__(NT) void rk4ip_solo(SoloArgs a) {
  constexpr int PT = L / NT;  // samples per thread
  constexpr int LOG = ilog2c(L);
  extern __shared__ float4 smem[];
  float4 *twl = smem;                                  // [L]
  float2 *buf = reinterpret_cast<float2 *>(smem + L);  // [2][L]
  const int tid = threadIdx.x;
  for (int j = tid; j < L; j += NT) twl[j] = a.tw[j];
  const float s0 = a.S[0];
  const float hg = a.hg;
  // i h gamma S |x|^2 x, as eval_small for one mode
  auto hN = [&](float2 x) -> float2 {
    float2 am = make_float2(0.f, 0.f);
    am.x = fmaf(s0, x.x, am.x);
    am.y = fmaf(s0, x.y, am.y);
    const float2 an = cfma(make_float2(0.f, 0.f), am, x);
    const float2 acc = cfma_conj(make_float2(0.f, 0.f), an, x);
    return make_float2(-hg * acc.y, hg * acc.x);
  };
  float4 e[PT];
  float2 A[PT], N1[PT];
#pragma unroll
  for (int j = 0; j < PT; ++j) {
    const int t = tid + NT * j;
    e[j] = a.E[t];
    A[j] = a.A[t];
    N1[j] = a.start ? hN(A[j]) : a.N1[t];
  }
  __syncthreads();
  // x0 <- D x0, x1 <- D x1
  auto lin2 = [&](float2 (&x0)[PT], float2 (&x1)[PT]) {
#pragma unroll
    for (int j = 0; j < PT; ++j) {
      buf[tid + NT * j] = x0[j];
      buf[L + tid + NT * j] = x1[j];
    }
    __syncthreads();
    lds_fft<L, 2, 1, L, NT, false>(buf, twl, LOG);
#pragma unroll
    for (int j = 0; j < PT; ++j) {
      const int f = tid + NT * j;
      buf[f] = cmul_hilo(buf[f], e[j]);
      buf[L + f] = cmul_hilo(buf[L + f], e[j]);
    }
    __syncthreads();
    lds_fft<L, 2, 1, L, NT, true>(buf, twl, LOG);
    // each thread reads back, and next writes, only its own samples: the
    // next transform's first read of other samples follows a barrier
#pragma unroll
    for (int j = 0; j < PT; ++j) {
      x0[j] = buf[tid + NT * j];
      x1[j] = buf[L + tid + NT * j];
    }
  };
  for (int s = 0; s < a.n_steps; ++s) {
    float2 X[PT], K1[PT];
#pragma unroll
    for (int j = 0; j < PT; ++j) {
      X[j] = A[j];
      K1[j] = N1[j];
    }
    lin2(X, K1);  // A_I = D A, k1 = D h N(A)
    float2 Y[PT], Z[PT];
#pragma unroll
    for (int j = 0; j < PT; ++j) {
      const float2 ai = X[j], k1 = K1[j];
      const float2 k2 = hN(caxpy(ai, 0.5f, k1));
      const float2 k3 = hN(caxpy(ai, 0.5f, k2));
      Y[j] = cadd(ai, k3);
      float2 z = caxpy(ai, 1.f / 6.f, k1);
      z = caxpy(z, 1.f / 3.f, k2);
      Z[j] = caxpy(z, 1.f / 3.f, k3);
    }
    lin2(Y, Z);  // D (A_I + k3), D (A_I + k1/6 + k2/3 + k3/3)
    const bool more = s + 1 < a.n_steps || !a.finish;
#pragma unroll
    for (int j = 0; j < PT; ++j) {
      A[j] = caxpy(Z[j], 1.f / 6.f, hN(Y[j]));
      if (more) N1[j] = hN(A[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < PT; ++j) {
    const int t = tid + NT * j;
    a.A[t] = A[j];
    if (!a.finish) a.N1[t] = N1[j];
  }
}

template <int L>
hipError_t go_solo(const SoloArgs &a, hipStream_t s) {
  constexpr int NT = solo_threads<L>();
  const size_t shm = (size_t)L * (sizeof(float4) + 2 * sizeof(float2));
  hipError_t e = check_launch((const void *)rk4ip_solo<L, NT>, NT, shm);
  if (e != hipSuccess) return e;
  if (shm > 65536) {
    e = hipFuncSetAttribute((const void *)rk4ip_solo<L, NT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((rk4ip_solo<L, NT>), dim3(1), dim3(NT), shm, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_linear(const Plan &pl, const float4 *E, const float2 *in0, float2 *out0,
                         const float2 *in1, float2 *out1) {
  LinArgs a;
  a.in[0] = in0;
  a.out[0] = out0;
  a.in[1] = in1;
  a.out[1] = out1;
  a.E = E;
  a.tw = pl.tw;
  a.twc = pl.twc;
  a.M = pl.M;
  a.T = pl.T;
  a.logT = pl.logT;
  a.N1 = pl.N1;
  a.N2 = pl.N2;
  const int njobs = in1 ? 2 : 1;
  for (const void *p : {(const void *)in0, (const void *)out0, (const void *)in1, (const void *)out1})
    if (reinterpret_cast<uintptr_t>(p) & 15) return hipErrorInvalidValue;  // entry points check first
  if (!pl.four_step) return single_dispatch(a, njobs, pl.stream);
  hipError_t e = cols_dispatch(a, njobs, pl.stream, false);
  if (e != hipSuccess) return e;
  e = rows_dispatch(a, njobs, pl.stream);
  if (e != hipSuccess) return e;
  return cols_dispatch(a, njobs, pl.stream, true);
}

hipError_t launch_linear_twice(const Plan &pl, const float4 *E, const float2 *in, float2 *out1,
                               float2 *out2) {
  if (!pl.four_step) {  // one LDS pass per application: two applications
    hipError_t e = launch_linear(pl, E, in, out1, nullptr, nullptr);
    if (e != hipSuccess) return e;
    return launch_linear(pl, E, out1, out2, nullptr, nullptr);
  }
  for (const void *p : {(const void *)in, (const void *)out1, (const void *)out2})
    if (reinterpret_cast<uintptr_t>(p) & 15) return hipErrorInvalidValue;  // entry points check first
  LinArgs a;
  a.in[0] = in;
  a.out[0] = out1;
  a.in[1] = out1;
  a.out[1] = out2;
  a.E = E;
  a.tw = pl.tw;
  a.twc = pl.twc;
  a.M = pl.M;
  a.T = pl.T;
  a.logT = pl.logT;
  a.N1 = pl.N1;
  a.N2 = pl.N2;
  hipError_t e = cols_dispatch(a, 1, pl.stream, false);  // in -> out1
  if (e != hipSuccess) return e;
  e = rows_dispatch(a, 0, pl.stream);                    // out1 -> out1 (E) and out2 (E twice)
  if (e != hipSuccess) return e;
  return cols_dispatch(a, 2, pl.stream, true);           // both, in place
}

hipError_t launch_rk4ip_solo(const Plan &pl, float2 *A, float2 *N1, int64_t n_steps, double h, const float4 *E,
                             bool start, bool finish) {
  if (!pl.solo || pl.M != 1 || n_steps > INT32_MAX) return hipErrorInvalidValue;
  SoloArgs a;
  a.A = A;
  a.N1 = N1;
  a.E = E;
  a.tw = pl.tw;
  a.S = pl.Sg;
  a.hg = (float)(h * pl.gamma);
  a.n_steps = (int)n_steps;
  a.start = start ? 1 : 0;
  a.finish = finish ? 1 : 0;
  switch (pl.T) {
    case 64: return go_solo<64>(a, pl.stream);
    case 128: return go_solo<128>(a, pl.stream);
    case 256: return go_solo<256>(a, pl.stream);
    case 512: return go_solo<512>(a, pl.stream);
    case 1024: return go_solo<1024>(a, pl.stream);
    case 2048: return go_solo<2048>(a, pl.stream);
    case 4096: return go_solo<4096>(a, pl.stream);
  }
  return hipErrorInvalidValue;
}

}  // namespace mmnlse
