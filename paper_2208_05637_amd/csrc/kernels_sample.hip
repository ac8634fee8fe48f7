// Unique-sample autoregressive sampler (Sec. 4, Sampling).
//
// A buffer of distinct configurations with occurrence counts starts as one
// configuration (all qubits 0) carrying every draw.  At sampling position t
// (qubit q = order[t]) each entry is doubled into children with x_q = 0 and
// x_q = 1, its draws are split between them by a binomial draw with the
// network's conditional P(x_q = 1 | earlier positions) (forced to 0 or 1 by
// the Hamming-weight modifier), empty children are dropped and, beyond the
// buffer capacity, the children with the fewest draws are eliminated (ties
// broken by buffer order).  The buffer order is kept sorted by the bits in
// sampling order: children with x_q = 0 come first, each group in parent
// order.
//
// Random numbers: Philox4x64 with 10 rounds (Salmon et al., SC 2011),
// counter (parent configuration's low word, t, its high word, j) for blocks
// j = 0, 1, ..., key (seed, 0), so a draw does not depend on the entry's place
// in the buffer.  Binomial Bin(c, p), exact: with q = min(p, 1 - p),
// inversion of the distribution function summed from k = 0 when c q < 32,
// else Hormann's BTRS rejection method; reflected when p > 1/2.  The arithmetic is written in
// a fixed operation order without contraction into fused multiply-adds, so a
// host implementation of the same definition draws the same counts.
#include "nqs_internal.h"

#pragma clang fp contract(off)

namespace nqs {

__device__ __forceinline__ void philox4x64_10(uint64_t (&c)[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__device__ __forceinline__ double uniform53(uint64_t w) {
  return (double)(w >> 11) * (1.0 / 9007199254740992.0);
}

// The uniforms of one draw: the four words of Philox block j = 0, 1, ... of
// the counter (c0, c1, c2, j), in order.
struct Uniforms {
  uint64_t c0, c1, c2, key, j;
  uint64_t w[4];
  int used;
  __device__ Uniforms(uint64_t a, uint64_t b, uint64_t c, uint64_t k) : c0(a), c1(b), c2(c), key(k), j(0), used(4) {}
  __device__ double next() {
    if (used == 4) {
      uint64_t blk[4] = {c0, c1, c2, j};
      philox4x64_10(blk, key, 0ull);
#pragma unroll
      for (int i = 0; i < 4; ++i) w[i] = blk[i];
      used = 0;
      ++j;
    }
    const int i = used++;
    return uniform53(i == 0 ? w[0] : (i == 1 ? w[1] : (i == 2 ? w[2] : w[3])));
  }
};

// fc(k) = log(k!) - [(k + 1/2) log(k + 1) - (k + 1) + log(2 pi) / 2] for integer-valued k >= 0.
__device__ double stirling_corr(double k) {
  if (k < 16.0) return lgamma(k + 1.0) - ((k + 0.5) * log(k + 1.0) - (k + 1.0) + 0.5 * log(2.0 * 3.141592653589793));
  const double x = k + 1.0;
  const double x2 = x * x;
  return (1.0 / 12.0 - (1.0 / 360.0 - (1.0 / 1260.0 - (1.0 / 1680.0) / x2) / x2) / x2) / x;
}

// log(a! / b!) for a >= b >= 0, as d log(b+1) + (a + 1/2) log1p(d/(b+1)) - d + fc(a) - fc(b), d = a - b:
// its rounding stays at the size of the result next to 10^12.
__device__ double log_fact_ratio(long long a, long long b) {
  const long long d = a - b;
  if (d == 0) return 0.0;
  const double dd = (double)d, ad = (double)a, bd = (double)b;
  return dd * log(bd + 1.0) + (ad + 0.5) * log1p(dd / (bd + 1.0)) - dd + stirling_corr(ad) - stirling_corr(bd);
}

constexpr int kMaxAttempts = 4096;

// Bin(n, p), p <= 1/2, n p >= 32: Hormann's BTRS (transformed rejection with
// squeeze; J. Statist. Comput. Simul. 46, 1993), each attempt on the next two
// uniforms; the acceptance test compares log V with log f(k)/f(m) at the mode
// m.  Attempts are capped (each accepts with probability above 0.75); at the
// cap the draw is the mode.
__device__ long long binomial_btrs(long long n, double p, Uniforms& uni) {
  const double nd = (double)n;
  const double q = 1.0 - p;
  const double spq = sqrt(nd * p * q);
  const double b = 1.15 + 2.53 * spq;
  const double a = -0.0873 + 0.0248 * b + 0.01 * p;
  const double c = nd * p + 0.5;
  const double vr = 0.92 - 4.2 / b;
  const double alpha = (2.83 + 5.1 / b) * spq;
  const double lpq = log(p / q);
  const long long m = (long long)floor((nd + 1.0) * p);
  for (int it = 0; it < kMaxAttempts; ++it) {
    const double u = uni.next() - 0.5;
    double v = uni.next();
    const double us = 0.5 - fabs(u);
    const double kf = floor(us > 0.0 ? (2.0 * a / us + b) * u + c : -1.0);   // us = 0 only at u = -1/2
    if (us >= 0.07 && v <= vr) return (long long)kf;
    if (kf < 0.0 || kf > nd) continue;
    const long long k = (long long)kf;
    v = v * alpha / (a / (us * us) + b);
    // log f(k)/f(m) = log(m!/k!) + log((n-m)!/(n-k)!) + (k - m) log(p/q)
    const double lr = k >= m ? -log_fact_ratio(k, m) + log_fact_ratio(n - m, n - k)
                             : log_fact_ratio(m, k) - log_fact_ratio(n - k, n - m);
    if (v == 0.0 || log(v) <= lr + (double)(k - m) * lpq) return k;
  }
  return m;
}

__device__ long long binomial_draw(long long c, double p, Uniforms& uni) {
  if (c == 0 || !(p > 0.0)) return 0;
  if (!(p < 1.0)) return c;
  const bool flip = p > 0.5;
  const double q = flip ? 1.0 - p : p;
  const double cd = (double)c;
  long long k;
  if (cd * q < 32.0) {
    const double u1 = uni.next();
    const double r = q / (1.0 - q);
    double pk = exp(cd * log1p(-q));
    double F = pk;
    k = 0;
    // terms past the underflowing tail are 0: stopping there bounds the
    // search even when u1 lies above the rounded total of the distribution
    while (u1 > F && k < c && pk > 0.0) {
      pk *= r * (double)(c - k) / (double)(k + 1);
      k += 1;
      F += pk;
    }
  } else {
    k = binomial_btrs(c, q, uni);
  }
  return flip ? c - k : k;
}

__global__ void sample_init_kernel(uint64_t* x, int words, long long* cnt, long long n_draws, long long* d_u) {
  for (int w = 0; w < words; ++w) x[w] = 0;
  cnt[0] = n_draws;
  *d_u = 1;
}

// Children of entry i: (x, c - k) at i and (x | 1 << q, k) at U + i.  The
// counter of the draw is (x's low word, t, x's high word, 0).
template <int W>
__global__ void sample_split_kernel(const uint64_t* __restrict__ x, const long long* __restrict__ cnt,
                                    const double2* __restrict__ cond, const long long* __restrict__ d_u,
                                    long long umax, int t, int q, uint64_t seed, uint64_t* __restrict__ kx,
                                    long long* __restrict__ kc, long long* __restrict__ d_nk) {
  const long long U = *d_u;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *d_nk = 2 * U;
  if (i >= U || i >= umax) return;
  const double2 cd = cond[i];
  const int code = (int)cd.y;
  const double p1 = code == 1 ? 0.0 : (code == 2 ? 1.0 : 1.0 / (1.0 + exp(-cd.x)));
  uint64_t xi[W];
#pragma unroll
  for (int k = 0; k < W; ++k) xi[k] = x[i * W + k];
  Uniforms uni(xi[0], (uint64_t)t, W == 2 ? xi[W - 1] : 0ull, seed);
  const long long c = cnt[i];
  const long long k1 = binomial_draw(c, p1, uni);
#pragma unroll
  for (int k = 0; k < W; ++k) {
    kx[i * W + k] = xi[k];
    kx[(U + i) * W + k] = xi[k] | ((q >> 6) == k ? (1ull << (q & 63)) : 0ull);
  }
  kc[i] = c - k1;
  kc[U + i] = k1;
}

constexpr int kSelThreads = 1024;

__device__ long long block_count_ge(const long long* kc, long long nk, long long v, long long* sh) {
  long long n = 0;
  for (long long i = threadIdx.x; i < nk; i += kSelThreads) n += kc[i] >= v ? 1 : 0;
  for (int o = 32; o >= 1; o >>= 1) n += __shfl_xor(n, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = n;
  __syncthreads();
  long long tot = 0;
  for (int k = 0; k < kSelThreads / 64; ++k) tot += sh[k];
  __syncthreads();
  return tot;
}

// Threshold of the elimination: sel[0] = tau, sel[1] = quota.  Children with
// more than tau draws are kept, and the first `quota` (in buffer order) with
// exactly tau; tau = 0 keeps every non-empty child.
__global__ __launch_bounds__(kSelThreads) void sample_select_kernel(const long long* __restrict__ kc,
                                                                   const long long* __restrict__ d_nk,
                                                                   long long umax, long long* __restrict__ sel) {
  __shared__ long long sh[kSelThreads / 64];
  const long long nk = *d_nk;
  long long tau = 0, quota = 0;
  if (block_count_ge(kc, nk, 1, sh) > umax) {
    long long mx = 0;
    for (long long i = threadIdx.x; i < nk; i += kSelThreads) mx = kc[i] > mx ? kc[i] : mx;
    for (int o = 32; o >= 1; o >>= 1) {
      const long long v = __shfl_xor(mx, o);
      mx = v > mx ? v : mx;
    }
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
    __syncthreads();
    mx = 0;
    for (int k = 0; k < kSelThreads / 64; ++k) mx = sh[k] > mx ? sh[k] : mx;
    __syncthreads();
    // largest tau with at least umax children of >= tau draws
    long long lo = 1, hi = mx + 1;
    while (hi - lo > 1) {
      const long long mid = lo + (hi - lo) / 2;
      if (block_count_ge(kc, nk, mid, sh) >= umax) lo = mid;
      else hi = mid;
    }
    tau = lo;
    quota = umax - block_count_ge(kc, nk, tau + 1, sh);
  }
  if (threadIdx.x == 0) {
    sel[0] = tau;
    sel[1] = quota;
  }
}

__global__ void sample_tie_flags(const long long* __restrict__ kc, const long long* __restrict__ d_nk,
                                 const long long* __restrict__ sel, long long n2, int* __restrict__ eq) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n2) return;
  const long long tau = sel[0];
  eq[i] = (i < *d_nk && tau > 0 && kc[i] == tau) ? 1 : 0;
}

__global__ void sample_keep_flags(const long long* __restrict__ kc, const long long* __restrict__ d_nk,
                                  const long long* __restrict__ sel, const long long* __restrict__ eqoff,
                                  long long n2, int* __restrict__ keep) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n2) return;
  const long long tau = sel[0], quota = sel[1];
  bool k = false;
  if (i < *d_nk) {
    const long long c = kc[i];
    k = c > tau || (tau > 0 && c == tau && eqoff[i] < quota);
  }
  keep[i] = k ? 1 : 0;
}

template <int W>
__global__ void sample_compact_kernel(const uint64_t* __restrict__ kx, const long long* __restrict__ kc,
                                      const int* __restrict__ keep, const long long* __restrict__ koff,
                                      long long n2, uint64_t* __restrict__ x, long long* __restrict__ cnt,
                                      long long* __restrict__ d_u) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *d_u = koff[n2];
  if (i >= n2 || !keep[i]) return;
  const long long d = koff[i];
#pragma unroll
  for (int k = 0; k < W; ++k) x[d * W + k] = kx[i * W + k];
  cnt[d] = kc[i];
}

template <int W>
__global__ void sample_finish_kernel(const uint64_t* __restrict__ x, const long long* __restrict__ cnt,
                                     const long long* __restrict__ d_u, long long umax, uint64_t* __restrict__ ox,
                                     double* __restrict__ ow, long long* __restrict__ on) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long U = *d_u;
  if (i == 0) *on = U;
  if (i >= U || i >= umax) return;
#pragma unroll
  for (int k = 0; k < W; ++k) ox[i * W + k] = x[i * W + k];
  ow[i] = (double)cnt[i];
}

static unsigned blocks_for(long long n, int t) { return (unsigned)((n + t - 1) / t); }

void launch_sample_init(uint64_t* x, int words, long long* cnt, long long n_draws, long long* d_u, hipStream_t s) {
  hipLaunchKernelGGL(sample_init_kernel, dim3(1), dim3(1), 0, s, x, words, cnt, n_draws, d_u);
}

void launch_sample_step(const SampleBufs& b, long long umax, int t, int q, uint64_t seed, hipStream_t s) {
  const long long n2 = 2 * umax;
  auto split = b.words == 2 ? sample_split_kernel<2> : sample_split_kernel<1>;
  hipLaunchKernelGGL(split, dim3(blocks_for(umax, 256)), dim3(256), 0, s, b.x, b.cnt,
                     (const double2*)b.cond, b.d_u, umax, t, q, seed, b.kx, b.kc, b.d_nk);
  hipLaunchKernelGGL(sample_select_kernel, dim3(1), dim3(kSelThreads), 0, s, b.kc, b.d_nk, umax, b.sel);
  hipLaunchKernelGGL(sample_tie_flags, dim3(blocks_for(n2, 256)), dim3(256), 0, s, b.kc, b.d_nk, b.sel, n2, b.eq);
  launch_scan(b.eq, n2, b.eqoff, b.stmp, s);
  hipLaunchKernelGGL(sample_keep_flags, dim3(blocks_for(n2, 256)), dim3(256), 0, s, b.kc, b.d_nk, b.sel,
                     b.eqoff, n2, b.keep);
  launch_scan(b.keep, n2, b.koff, b.stmp, s);
  auto compact = b.words == 2 ? sample_compact_kernel<2> : sample_compact_kernel<1>;
  hipLaunchKernelGGL(compact, dim3(blocks_for(n2, 256)), dim3(256), 0, s, b.kx, b.kc, b.keep,
                     b.koff, n2, b.x, b.cnt, b.d_u);
}

void launch_sample_finish(const SampleBufs& b, long long umax, uint64_t* ox, double* ow, long long* on,
                          hipStream_t s) {
  auto finish = b.words == 2 ? sample_finish_kernel<2> : sample_finish_kernel<1>;
  hipLaunchKernelGGL(finish, dim3(blocks_for(umax, 256)), dim3(256), 0, s, b.x, b.cnt, b.d_u,
                     umax, ox, ow, on);
}

}  // namespace nqs
