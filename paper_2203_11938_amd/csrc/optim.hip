// optim.hip -- the device arithmetic of phi-SfT's outer optimisation loop (Sec. 3.3,
// "Adaptive Optimisation Scheme"; Sec. 3.4: Adam, learning rate 1e-3), on gfx950:
//   k_frame_loss  per loss frame and sheet, the energy E_t = sum_i |x_t,i - target_t,i|^2
//                 (the 3D stand-in for the per-frame reconstruction energy) in FP64 with a
//                 fixed summation order, and its gradient 2 (x - target);
//   k_adam        one Adam step (Kingma and Ba) over a parameter array, optionally in log
//                 space (material parameters) or on a per-vertex scale (forces as loads on
//                 each vertex's area share).
// The window logic that decides which frames are active runs on the host.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/phisft_sim.h"
#include "kernels.h"

namespace phisft {

constexpr int kOptThreads = 256;

__device__ __forceinline__ double opt_wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) {
    int2 t = *reinterpret_cast<int2*>(&v);
    t.x = __shfl_xor(t.x, o);
    t.y = __shfl_xor(t.y, o);
    v += *reinterpret_cast<double*>(&t);
  }
  return v;
}

// One workgroup per (frame, sheet): blockIdx.x = frame * ninst + sheet.
template <typename T>
__global__ void __launch_bounds__(kOptThreads) k_frame_loss(const T* __restrict__ x,
                                                            const T* __restrict__ tgt, int nv,
                                                            const int* __restrict__ voff,
                                                            const int* __restrict__ vcount,
                                                            int ninst, double* __restrict__ energy,
                                                            T* __restrict__ dl) {
  __shared__ double s_w[kOptThreads / 64];
  const int f = blockIdx.x / ninst, b = blockIdx.x - f * ninst;
  const int v0 = voff[b], n = vcount[b];
  const size_t base = (size_t)f * 3 * nv;
  double acc = 0.0;
  for (int k = threadIdx.x; k < 3 * n; k += kOptThreads) {
    const int c = k / n, i = v0 + (k - c * n);
    const size_t e = base + (size_t)c * nv + i;
    const double d = (double)x[e] - (double)tgt[e];
    acc += d * d;
    if (dl) dl[e] = (T)(2.0 * d);
  }
  acc = opt_wave_sum(acc);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kOptThreads / 64; ++w) t += s_w[w];
    energy[blockIdx.x] = t;
  }
}

// theta <- theta - lr mhat / (sqrt(vhat) + eps) with the bias-corrected moments of step t.
// The parameter p is theta itself, exp(theta) (log_space), or scale[e % period] * theta;
// the gradient is taken to theta by the chain rule.
template <typename T>
__global__ void __launch_bounds__(kOptThreads) k_adam(T* __restrict__ p, const T* __restrict__ g,
                                                      double* __restrict__ m1,
                                                      double* __restrict__ m2, long n,
                                                      const double* __restrict__ scale, int period,
                                                      int log_space, double lr, double b1, double b2,
                                                      double eps, double c1, double c2) {
  const long e = (long)blockIdx.x * kOptThreads + threadIdx.x;
  if (e >= n) return;
  const double pv = (double)p[e];
  double gt = (double)g[e], th = pv;
  double s = 1.0;
  if (log_space) {
    th = log(pv);
    gt *= pv;
  } else if (scale) {
    s = scale[e % period];
    th = pv / s;
    gt *= s;
  }
  const double a = b1 * m1[e] + (1.0 - b1) * gt;
  const double v = b2 * m2[e] + (1.0 - b2) * gt * gt;
  m1[e] = a;
  m2[e] = v;
  th -= lr * (a / c1) / (sqrt(v / c2) + eps);
  p[e] = (T)(log_space ? exp(th) : s * th);
}

template <typename T>
void launch_frame_loss(const T* x, const T* tgt, int nv, const int* voff, const int* vcount,
                       int ninst, int nframes, double* energy, T* dl, hipStream_t st) {
  if (nframes > 0)
    hipLaunchKernelGGL((k_frame_loss<T>), dim3(nframes * ninst), dim3(kOptThreads), 0, st, x, tgt,
                       nv, voff, vcount, ninst, energy, dl);
}
template void launch_frame_loss<float>(const float*, const float*, int, const int*, const int*, int,
                                       int, double*, float*, hipStream_t);
template void launch_frame_loss<double>(const double*, const double*, int, const int*, const int*,
                                        int, int, double*, double*, hipStream_t);

}  // namespace phisft

using namespace phisft;

extern "C" {

sim_status sim_adam_step(void* param, int32_t precision, const void* grad, double* m1, double* m2,
                         int64_t n, const double* scale, int32_t period, int32_t log_space,
                         double lr, double beta1, double beta2, double eps, int32_t t,
                         void* stream) {
  if (n < 0 || t < 1 || (n > 0 && (!param || !grad || !m1 || !m2)) ||
      (precision != SIM_FP32 && precision != SIM_FP64) || (scale && period < 1) ||
      (scale && log_space) || !(lr >= 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) ||
      !(beta2 >= 0.0 && beta2 < 1.0) || !(eps >= 0.0))
    return SIM_E_INVALID;
  if (n == 0) return SIM_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const double c1 = 1.0 - std::pow(beta1, t), c2 = 1.0 - std::pow(beta2, t);
  const dim3 grid((unsigned)((n + kOptThreads - 1) / kOptThreads));
  if (precision == SIM_FP64)
    hipLaunchKernelGGL(k_adam<double>, grid, dim3(kOptThreads), 0, st, static_cast<double*>(param),
                       static_cast<const double*>(grad), m1, m2, (long)n, scale, period, log_space,
                       lr, beta1, beta2, eps, c1, c2);
  else
    hipLaunchKernelGGL(k_adam<float>, grid, dim3(kOptThreads), 0, st, static_cast<float*>(param),
                       static_cast<const float*>(grad), m1, m2, (long)n, scale, period, log_space,
                       lr, beta1, beta2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? SIM_OK : SIM_E_HIP;
}

}  // extern "C"
