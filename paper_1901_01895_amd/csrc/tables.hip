// Device tabulation of the linear propagator exp(h/2 L) / T (Eq. 6a and the
// operator L of Eq. 1), per mode and frequency bin, in the storage order of
// the FFT that applies it.
//
// L_p(w) = -alpha_p/2 + i sum_n beta_{n,p} (-w)^n / n!  (forward transform
// kernel exp(-i w t), w = 2 pi fftfreq(T, dt) with the Nyquist bin negative).
// Phase and magnitude are evaluated in FP64 and stored as an FP32 hi + lo pair
// per component, so the factor carries no fixed FP32 rounding bias.  1/T of
// the inverse transform is folded in.  Evaluated on the device, so a new step
// size (the adaptive controller changes it every trial) costs one launch.

#include "common.h"

namespace mmnlse {
namespace {

struct TabArgs {
  const double *beta;   // [M][n_beta]
  const double *alpha;  // [M] or null
  float4 *E;            // [M][T]
  double h, dt;
  int M, T, n_beta, four_step, N1, N2;
};

__global__ __launch_bounds__(256) void tabulate_E(TabArgs a) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)a.M * a.T) return;
  const int p = (int)(idx / a.T), pos = (int)(idx % a.T);
  int f = pos;
  if (a.four_step) {  // position N2*k1 + k2 holds bin k1 + N1*k2
    const int k1 = pos / a.N2, k2 = pos % a.N2;
    f = k1 + a.N1 * k2;
  }
  const double freq = (double)(f < a.T / 2 ? f : f - a.T) / ((double)a.T * a.dt);
  const double w = 2.0 * M_PI * freq;
  const double *b = a.beta + (size_t)p * a.n_beta;
  double phase = 0.0, pw = 1.0, fact = 1.0;
  for (int n = 0; n < a.n_beta; ++n) {
    if (n > 0) fact *= n;
    phase += b[n] * pw / fact;
    pw *= -w;
  }
  const double att = a.alpha ? a.alpha[p] : 0.0;
  const double mag = exp(-0.25 * a.h * att) / (double)a.T;
  double s, c;
  sincos(0.5 * a.h * phase, &s, &c);
  const double re = mag * c, im = mag * s;
  const float rh = (float)re, ih = (float)im;
  a.E[idx] = make_float4(rh, ih, (float)(re - (double)rh), (float)(im - (double)ih));
}

}  // namespace

hipError_t launch_tabulate_E(const Plan &pl, double h, float4 *E) {
  TabArgs a;
  a.beta = pl.beta_d;
  a.alpha = pl.alpha_d;
  a.E = E;
  a.h = h;
  a.dt = pl.dt;
  a.M = pl.M;
  a.T = pl.T;
  a.n_beta = pl.n_beta;
  a.four_step = pl.four_step ? 1 : 0;
  a.N1 = pl.N1;
  a.N2 = pl.N2;
  const int64_t n = (int64_t)pl.M * pl.T;
  hipLaunchKernelGGL(tabulate_E, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, pl.stream, a);
  return hipGetLastError();
}

}  // namespace mmnlse
