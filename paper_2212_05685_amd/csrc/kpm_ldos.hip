// Local density of states by KPM for unit probes: the damped Chebyshev series
// of each probe's moments evaluated at a set of energies (kpm_ldos).
#include <hip/hip_runtime.h>

#include "kpm_internal.h"

namespace kpm {

// For unit probes e_I: A_I(E) = sum_m w_m mu_{I,m} T_m(x) / sqrt(1 - x^2),
// x = (E - b)/a, w_m = (2 - delta_m0) g_m / (pi a), g_m the Jackson kernel.
// First the reduced moments are scaled in place by w_m ...
__global__ __launch_bounds__(kBlock) void k_ldos_weights(const InstDev* __restrict__ insts, int M) {
  const InstDev& I = insts[blockIdx.y];
  const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (long long)I.R * M) return;
  const int m = (int)(t % M);
  const double q = 1.0 / (double)(M + 1);
  const double g = ((double)(M - m + 1) * cospi(m * q) + sinpi(m * q) * cospi(q) / sinpi(q)) * q;
  I.musum[t] *= (m == 0 ? 1.0 : 2.0) * g / (M_PI * I.ab[0]);
}

// ... then one thread per (energy, probe) sums the series with the Chebyshev
// recurrence T_{m+1} = 2x T_m - T_{m-1}, the scaled moments of its probe
// staged through LDS in chunks.  Energies outside the rescaled band give 0.
__global__ __launch_bounds__(kBlock) void k_ldos_eval(const InstDev* __restrict__ insts, int M,
                                                      const double* __restrict__ energies, int ne,
                                                      double* __restrict__ out) {
  const InstDev& I = insts[0];
  const int p = blockIdx.y;
  const int e = blockIdx.x * kBlock + threadIdx.x;
  __shared__ double w[kBlock];
  const double x = e < ne ? (energies[e] - I.ab[1]) / I.ab[0] : 0.0;
  const bool inside = fabs(x) < 1.0;
  const double* row = I.musum + (long long)p * M;
  double t0 = 1.0, t1 = x, acc = 0.0;
  for (int m0 = 0; m0 < M; m0 += kBlock) {
    __syncthreads();
    if (m0 + (int)threadIdx.x < M) w[threadIdx.x] = row[m0 + threadIdx.x];
    __syncthreads();
    const int mmax = min(kBlock, M - m0);
    for (int k = 0; k < mmax; ++k) {
      acc = fma(w[k], t0, acc);
      const double t2 = fma(2.0 * x, t1, -t0);
      t0 = t1;
      t1 = t2;
    }
  }
  if (e < ne) out[(long long)p * ne + e] = inside ? acc / sqrt((1.0 - x) * (1.0 + x)) : 0.0;
}

hipError_t launch_ldos(const InstDev* insts, int R, int M, const double* energies, int ne,
                       double* out, hipStream_t s) {
  dim3 g1(((long long)R * M + kBlock - 1) / kBlock, 1);
  hipLaunchKernelGGL(k_ldos_weights, g1, dim3(kBlock), 0, s, insts, M);
  dim3 g2((ne + kBlock - 1) / kBlock, R);
  hipLaunchKernelGGL(k_ldos_eval, g2, dim3(kBlock), 0, s, insts, M, energies, ne, out);
  return hipGetLastError();
}

}  // namespace kpm
