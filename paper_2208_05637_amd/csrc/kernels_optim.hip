// Adam update of the network parameters (Kingma and Ba, ICLR 2015; the
// paper's optimiser, Sec. 6).  One lane per parameter, grid-stride; the
// moments are FP64, the update is formed in FP64 in a fixed operation order
// (no contraction into fused multiply-adds) and the parameter is rounded to
// the nearest FP32 value.  Memory-bound: 4 + 8 + 8 + 8 bytes read and
// 4 + 8 + 8 written per parameter.
#include "nqs_internal.h"

#pragma clang fp contract(off)

namespace nqs {

__global__ __launch_bounds__(256) void adam_kernel(long long n, float* __restrict__ p, const double* __restrict__ g,
                                                   double* __restrict__ m, double* __restrict__ v, AdamCoef k) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double gi = g[i];
    const double mi = k.b1 * m[i] + k.one_m_b1 * gi;
    const double vi = k.b2 * v[i] + k.one_m_b2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const double mhat = mi / k.bc1;
    const double vhat = vi / k.bc2;
    const double upd = k.lr * mhat / (sqrt(vhat) + k.eps);
    p[i] = (float)((double)p[i] - upd);
  }
}

void launch_adam(long long n, float* p, const double* g, double* m, double* v, const AdamCoef& k, int cu_count,
                 hipStream_t s) {
  if (n <= 0) return;
  const long long want = (n + 255) / 256;
  const long long cap = 8LL * (cu_count > 0 ? cu_count : 256);
  const unsigned blocks = (unsigned)(want < cap ? want : cap);
  hipLaunchKernelGGL(adam_kernel, dim3(blocks), dim3(256), 0, s, n, p, g, m, v, k);
}

}  // namespace nqs
