// Hamiltonian-side kernels: enumeration of connected configurations with
// their matrix elements (Sec. 5.1, Eq. mtx_element, Alg. 1), deduplication of
// connected configurations per chunk (Sec. 5.2), the ratio-and-reduce of
// Eq. local_energy_auto and the weighted energy of Eq. total_energy_sum.
#include "nqs_internal.h"

namespace nqs {

constexpr uint64_t kUp = 0x5555555555555555ull;
constexpr uint64_t kDn = 0xAAAAAAAAAAAAAAAAull;

__global__ void fill_u32_kernel(unsigned* p, unsigned v, long long count) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = v;
}
__global__ void fill_u64_kernel(unsigned long long* p, unsigned long long v, long long count) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = v;
}
void launch_fill_u32(void* p, unsigned v, long long count, hipStream_t s) {
  if (count <= 0) return;
  long long blocks = (count + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (unsigned*)p, v, count);
}
void launch_fill_u64(void* p, unsigned long long v, long long count, hipStream_t s) {
  if (count <= 0) return;
  long long blocks = (count + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     (unsigned long long*)p, v, count);
}

// A bit string of W 64-bit words (word w = qubits 64w .. 64w+63).
template <int W>
struct Bits {
  uint64_t w[W];
};
template <int W>
__device__ __forceinline__ Bits<W> load_bits(const uint64_t* __restrict__ p, long long i) {
  Bits<W> b;
#pragma unroll
  for (int k = 0; k < W; ++k) b.w[k] = p[i * W + k];
  return b;
}
template <int W>
__device__ __forceinline__ int popc_and(const Bits<W>& a, const uint64_t* __restrict__ m, long long i) {
  int c = 0;
#pragma unroll
  for (int k = 0; k < W; ++k) c += __popcll(a.w[k] & m[i * W + k]);
  return c;
}

// h_g(x) = sum_{k in g} ct_k (-1)^{popcount(x & z_k)}, sequential in canonical
// order; the sign is applied by flipping the sign bit (exact).
template <bool IMAG, int W>
__device__ __forceinline__ void group_h(const HamDev& H, const Bits<W>& x, long long k0, long long k1,
                                        double& re, double& im) {
  double a = 0.0, b = 0.0;
  for (long long k = k0; k < k1; ++k) {
    const unsigned long long par = (unsigned long long)(popc_and<W>(x, H.tz, k) & 1) << 63;
    a += __longlong_as_double(__double_as_longlong(H.tre[k]) ^ par);
    if constexpr (IMAG) b += __longlong_as_double(__double_as_longlong(H.tim[k]) ^ par);
  }
  re = a;
  im = b;
}

// h_g(x) from the structured tables: sum over the group's sub-groups s of
// (-1)^{popcount(x & u_s)} T_s[bits of x at the flip's qubits], sub-groups in
// order; the same sum as group_h in another order.
template <bool IMAG, int W>
__device__ __forceinline__ void group_h_tables(const HamDev& H, const Bits<W>& x, int g, double& re, double& im) {
  int idx = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int p = H.fpos[4 * g + j];
    if (p >= 0) {
      const uint64_t word = W == 1 ? x.w[0] : x.w[(p >> 6) & (W - 1)];
      idx |= (int)((word >> (p & 63)) & 1ull) << j;
    }
  }
  double a = 0.0, b = 0.0;
  for (long long s = H.soff[g]; s < H.soff[g + 1]; ++s) {
    const unsigned long long par = (unsigned long long)(popc_and<W>(x, H.su, s) & 1) << 63;
    const long long e = H.stab[s] + idx;
    a += __longlong_as_double(__double_as_longlong(H.tabre[e]) ^ par);
    if constexpr (IMAG) b += __longlong_as_double(__double_as_longlong(H.tabim[e]) ^ par);
  }
  re = a;
  im = b;
}

// h_g(x) of group g, from the term list or from the tables
template <bool IMAG, int W>
__device__ __forceinline__ void group_value(const HamDev& H, const Bits<W>& x, int g, double& re, double& im) {
  if (H.tables) group_h_tables<IMAG, W>(H, x, g, re, im);
  else group_h<IMAG, W>(H, x, H.goff[g], H.goff[g + 1], re, im);
}

// the flip f keeps the number of up (even qubits) and down (odd qubits) electrons
template <int W>
__device__ __forceinline__ bool sector_ok(const Bits<W>& x, const Bits<W>& f) {
  int xu = 0, fu = 0, xd = 0, fd = 0;
#pragma unroll
  for (int k = 0; k < W; ++k) {
    xu += __popcll(x.w[k] & f.w[k] & kUp);
    fu += __popcll(f.w[k] & kUp);
    xd += __popcll(x.w[k] & f.w[k] & kDn);
    fd += __popcll(f.w[k] & kDn);
  }
  return 2 * xu == fu && 2 * xd == fd;
}

template <bool IMAG, int W>
__global__ void diag_kernel(HamDev H, const uint64_t* __restrict__ xs, long long S,
                            double* __restrict__ diag) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S) return;
  double re = 0.0, im = 0.0;
  if (H.gfirst) group_value<IMAG, W>(H, load_bits<W>(xs, i), 0, re, im);
  diag[2 * i] = re;
  diag[2 * i + 1] = im;
}

void launch_diag(const HamDev& H, const uint64_t* x, long long S, double* diag, hipStream_t s) {
  if (S <= 0) return;
  unsigned blocks = (unsigned)((S + 255) / 256);
  if (H.words == 2) {
    if (H.tim) hipLaunchKernelGGL((diag_kernel<true, 2>), dim3(blocks), dim3(256), 0, s, H, x, S, diag);
    else hipLaunchKernelGGL((diag_kernel<false, 2>), dim3(blocks), dim3(256), 0, s, H, x, S, diag);
    return;
  }
  if (H.tim) hipLaunchKernelGGL((diag_kernel<true, 1>), dim3(blocks), dim3(256), 0, s, H, x, S, diag);
  else hipLaunchKernelGGL((diag_kernel<false, 1>), dim3(blocks), dim3(256), 0, s, H, x, S, diag);
}

// One thread per sample, one block row per range of gper groups (excluding
// the empty flip).  Counts the valid (sample, group) pairs.
template <bool IMAG, int W>
__global__ void count_kernel(HamDev H, const uint64_t* __restrict__ xs, long long S, int R, int gper,
                             int* __restrict__ cnt) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  const int g0 = H.gfirst + r * gper;
  const int g1 = min(H.G, g0 + gper);
  const Bits<W> x = load_bits<W>(xs, i < S ? i : 0);
  int c = 0;
  for (int g = g0; g < g1; ++g) {
    const Bits<W> f = load_bits<W>(H.gx, g);
    bool ok;
    if (H.filter) {
      ok = sector_ok<W>(x, f);
    } else {
      double re, im;
      group_value<IMAG, W>(H, x, g, re, im);
      ok = (re != 0.0) || (im != 0.0);
    }
    c += ok ? 1 : 0;
  }
  if (i < S) cnt[i * R + r] = c;
}

void launch_count(const HamDev& H, const uint64_t* x, long long S, int R, int gper, int* cnt,
                  hipStream_t s) {
  if (S <= 0) return;
  dim3 grid((unsigned)((S + 255) / 256), (unsigned)R);
  if (H.words == 2) {
    if (H.tim) hipLaunchKernelGGL((count_kernel<true, 2>), grid, dim3(256), 0, s, H, x, S, R, gper, cnt);
    else hipLaunchKernelGGL((count_kernel<false, 2>), grid, dim3(256), 0, s, H, x, S, R, gper, cnt);
    return;
  }
  if (H.tim) hipLaunchKernelGGL((count_kernel<true, 1>), grid, dim3(256), 0, s, H, x, S, R, gper, cnt);
  else hipLaunchKernelGGL((count_kernel<false, 1>), grid, dim3(256), 0, s, H, x, S, R, gper, cnt);
}

// Exclusive scan of n counts into off[0..n] (off[n] = total) in three
// passes over tiles of kScanTile counts: tile sums, an exclusive scan of the
// tile sums (one workgroup), then each tile's local scan plus its offset.
// Loads and stores are coalesced; tmp holds scan_tiles(n) + 1 values.
constexpr int kScanThreads = 1024, kScanItems = 4, kScanTile = kScanThreads * kScanItems;

long long scan_tiles(long long n) { return (n + kScanTile - 1) / kScanTile; }

__device__ __forceinline__ long long block_sum_1024(long long v, long long* sh) {
  // sum over the 1024 threads of the block, result in every thread
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  if (lane == 0) sh[w] = v;
  __syncthreads();
  long long tot = 0;
  for (int k = 0; k < kScanThreads / 64; ++k) tot += sh[k];
  __syncthreads();
  return tot;
}

__global__ __launch_bounds__(kScanThreads) void scan_tile_sums(const int* __restrict__ cnt, long long n,
                                                               long long* __restrict__ tmp) {
  __shared__ long long sh[kScanThreads / 64];
  const long long base = (long long)blockIdx.x * kScanTile;
  long long v = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const long long i = base + k * kScanThreads + threadIdx.x;
    if (i < n) v += cnt[i];
  }
  const long long tot = block_sum_1024(v, sh);
  if (threadIdx.x == 0) tmp[blockIdx.x] = tot;
}

// Exclusive scan of m tile sums in place (tmp[m] = total), one workgroup.
__global__ __launch_bounds__(kScanThreads) void scan_tile_offsets(long long* __restrict__ tmp, long long m) {
  __shared__ long long part[kScanThreads];
  const int t = threadIdx.x;
  long long carry = 0;
  for (long long c0 = 0; c0 < m; c0 += kScanThreads) {
    const long long i = c0 + t;
    const long long v = i < m ? tmp[i] : 0;
    part[t] = v;
    __syncthreads();
    for (int d = 1; d < kScanThreads; d <<= 1) {
      const long long u = t >= d ? part[t - d] : 0;
      __syncthreads();
      part[t] += u;
      __syncthreads();
    }
    if (i < m) tmp[i] = carry + part[t] - v;
    carry += part[kScanThreads - 1];
    __syncthreads();
  }
  if (t == 0) tmp[m] = carry;
}

__global__ __launch_bounds__(kScanThreads) void scan_tile_apply(const int* __restrict__ cnt, long long n,
                                                                const long long* __restrict__ tmp,
                                                                long long* __restrict__ off) {
  __shared__ int vals[kScanTile];
  __shared__ long long part[kScanThreads];
  const int t = threadIdx.x;
  const long long base = (long long)blockIdx.x * kScanTile;
  // coalesced load of the tile, then each thread scans kScanItems consecutive counts
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const long long i = base + k * kScanThreads + t;
    vals[k * kScanThreads + t] = i < n ? cnt[i] : 0;
  }
  __syncthreads();
  long long loc[kScanItems];
  long long run = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    loc[k] = run;
    run += vals[t * kScanItems + k];
  }
  part[t] = run;
  __syncthreads();
  for (int d = 1; d < kScanThreads; d <<= 1) {
    const long long u = t >= d ? part[t - d] : 0;
    __syncthreads();
    part[t] += u;
    __syncthreads();
  }
  const long long pre = tmp[blockIdx.x] + part[t] - run;
  __syncthreads();
  // back through LDS so the stores are coalesced too
  long long* outv = (long long*)vals;   // kScanTile ints reused as kScanTile / 2 longs: two halves
#pragma unroll
  for (int half = 0; half < 2; ++half) {
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const int j = t * kScanItems + k;
      if ((j >> 11) == half) outv[j & 2047] = pre + loc[k];
    }
    __syncthreads();
    for (int j = t; j < 2048; j += kScanThreads) {
      const long long i = base + half * 2048 + j;
      if (i < n) off[i] = outv[j];
    }
    __syncthreads();
  }
  if (blockIdx.x == gridDim.x - 1 && t == 0) off[n] = tmp[gridDim.x];
}

void launch_scan(const int* cnt, long long n, long long* off, long long* tmp, hipStream_t s) {
  const long long m = scan_tiles(n);
  if (m == 0) {
    launch_fill_u64(off, 0ull, 1, s);
    return;
  }
  hipLaunchKernelGGL(scan_tile_sums, dim3((unsigned)m), dim3(kScanThreads), 0, s, cnt, n, tmp);
  hipLaunchKernelGGL(scan_tile_offsets, dim3(1), dim3(kScanThreads), 0, s, tmp, m);
  hipLaunchKernelGGL(scan_tile_apply, dim3((unsigned)m), dim3(kScanThreads), 0, s, cnt, n,
                     (const long long*)tmp, off);
}

template <bool IMAG, int W>
__global__ void write_kernel(HamDev H, const uint64_t* __restrict__ xs, long long S, int R, int gper,
                             const long long* __restrict__ off, long long cap,
                             uint64_t* __restrict__ xe, double* __restrict__ he,
                             int* __restrict__ esample, int hstride, unsigned* err) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  const int g0 = H.gfirst + r * gper;
  const int g1 = min(H.G, g0 + gper);
  const bool live = i < S;
  const Bits<W> x = load_bits<W>(xs, live ? i : 0);
  long long pos = live ? off[i * R + r] : 0;
  bool over = false;
  for (int g = g0; g < g1; ++g) {
    const Bits<W> f = load_bits<W>(H.gx, g);
    double re, im;
    group_value<IMAG, W>(H, x, g, re, im);
    const bool ok = H.filter ? sector_ok<W>(x, f) : ((re != 0.0) || (im != 0.0));
    if (live && ok) {
      if (pos < cap) {
#pragma unroll
        for (int k = 0; k < W; ++k) xe[pos * W + k] = x.w[k] ^ f.w[k];
        he[pos * hstride] = re;
        if (hstride == 2) he[pos * 2 + 1] = im;
        if (esample) esample[pos] = (int)i;
      } else {
        over = true;
      }
      ++pos;
    }
  }
  if (over) atomicOr(err, kErrEntryOverflow);
}

// The same entries from the term list, with the work turned around: a
// workgroup takes kWsSamples samples and one group range, stages the range's
// groups and terms in LDS in batches (coalesced loads, shared by its samples),
// and each wave walks its samples one at a time with its lanes on 64
// consecutive groups.  A ballot over the kept groups and a prefix count give
// every kept group its place in the sample's segment, so each store
// instruction writes consecutive entries.  h_g(x) is the same sequential sum
// over the group's terms as group_h.
constexpr int kWsSamples = 64;              // samples per workgroup
constexpr int kWsWaves = 4;                 // waves per workgroup
constexpr int kWsGroups = 448;              // groups per staged batch (four workgroups per CU in LDS)
constexpr int kWsTerms = 2048;              // terms per staged batch (and the largest group it takes)

template <bool IMAG, int W>
__global__ __launch_bounds__(64 * kWsWaves) void write_staged_kernel(
    HamDev H, const uint64_t* __restrict__ xs, long long S, int R, int gper, const long long* __restrict__ off,
    long long cap, uint64_t* __restrict__ xe, double* __restrict__ he, int* __restrict__ esample, int hstride,
    unsigned* err) {
  __shared__ uint64_t lgx[kWsGroups * W];
  __shared__ int loff[kWsGroups + 1];
  __shared__ uint64_t ltz[kWsTerms * W];
  __shared__ double lre[kWsTerms];
  __shared__ double lim[IMAG ? kWsTerms : 1];
  __shared__ int lkept[kWsWaves][128];   // per wave: kept groups awaiting evaluation
  __shared__ int lge;
  constexpr int SPW = kWsSamples / kWsWaves;   // samples per wave
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r = blockIdx.y;
  const int g0 = H.gfirst + r * gper;
  const int g1 = min(H.G, g0 + gper);
  // lane j < SPW holds sample j of this wave: its bits and its write position
  const long long i_l = (long long)blockIdx.x * kWsSamples + wv * SPW + (lane < SPW ? lane : 0);
  const bool live_l = lane < SPW && i_l < S;
  Bits<W> x_l = load_bits<W>(xs, live_l ? i_l : 0);
  long long pos_l = live_l ? off[i_l * R + r] : 0;
  bool over = false;
  for (int gb = g0; gb < g1;) {
    // the batch: groups [gb, ge) whose terms fit (a group alone always fits: the host checks)
    __syncthreads();
    if (threadIdx.x == 0) {
      const long long kb = H.goff[gb];
      int lo = gb + 1, hi = min(g1, gb + kWsGroups);   // largest ge in [lo, hi] with goff[ge] - kb <= kWsTerms
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (H.goff[mid] - kb <= kWsTerms) lo = mid;
        else hi = mid - 1;
      }
      lge = lo;
    }
    __syncthreads();
    const int ge = lge, ng = ge - gb;
    const long long kb = H.goff[gb];
    const int nt = (int)(H.goff[ge] - kb);
    for (int t = threadIdx.x; t < ng * W; t += blockDim.x) lgx[t] = H.gx[(long long)gb * W + t];
    for (int t = threadIdx.x; t <= ng; t += blockDim.x) loff[t] = (int)(H.goff[gb + t] - kb);
    for (int t = threadIdx.x; t < nt * W; t += blockDim.x) ltz[t] = H.tz[kb * W + t];
    for (int t = threadIdx.x; t < nt; t += blockDim.x) {
      lre[t] = H.tre[kb + t];
      if constexpr (IMAG) lim[t] = H.tim[kb + t];
    }
    __syncthreads();
    for (int j = 0; j < SPW; ++j) {
      const long long i = (long long)blockIdx.x * kWsSamples + wv * SPW + j;
      if (i >= S) break;
      Bits<W> x;
#pragma unroll
      for (int k = 0; k < W; ++k) {
        const unsigned lo32 = __builtin_amdgcn_readlane((unsigned)x_l.w[k], j);
        const unsigned hi32 = __builtin_amdgcn_readlane((unsigned)(x_l.w[k] >> 32), j);
        x.w[k] = ((uint64_t)hi32 << 32) | lo32;
      }
      long long pos;
      {
        const unsigned lo32 = __builtin_amdgcn_readlane((unsigned)pos_l, j);
        const unsigned hi32 = __builtin_amdgcn_readlane((unsigned)((unsigned long long)pos_l >> 32), j);
        pos = (long long)(((unsigned long long)hi32 << 32) | lo32);
      }
      // h_g(x) of the group at batch index q, summed over its terms in order
      auto group_sum = [&](int q, double& a, double& b) {
        a = 0.0;
        b = 0.0;
        const int k1 = loff[q + 1];
        for (int kk = loff[q]; kk < k1; ++kk) {
          int c = 0;
#pragma unroll
          for (int k = 0; k < W; ++k) c += __popcll(x.w[k] & ltz[kk * W + k]);
          const unsigned long long par = (unsigned long long)(c & 1) << 63;
          a += __longlong_as_double(__double_as_longlong(lre[kk]) ^ par);
          if constexpr (IMAG) b += __longlong_as_double(__double_as_longlong(lim[kk]) ^ par);
        }
      };
      auto store = [&](long long p, const Bits<W>& f, double a, double b) {
        if (p < cap) {
#pragma unroll
          for (int k = 0; k < W; ++k) xe[p * W + k] = x.w[k] ^ f.w[k];
          he[p * hstride] = a;
          if (hstride == 2) he[p * 2 + 1] = b;
          if (esample) esample[p] = (int)i;
        } else {
          over = true;
        }
      };
      if (H.filter) {
        // the sector test decides which groups the sample keeps; they are listed
        // in order and evaluated 64 at a time, one per lane, so no lane idles on
        // a group the sample does not keep
        int* kept = lkept[wv];
        int nk = 0;
        auto evaluate = [&](int cnt) {
          if (lane < cnt) {
            const int q = kept[lane];
            Bits<W> f;
#pragma unroll
            for (int k = 0; k < W; ++k) f.w[k] = lgx[q * W + k];
            double a, b;
            group_sum(q, a, b);
            store(pos + lane, f, a, b);
          }
          pos += cnt;
        };
        for (int q0 = 0; q0 < ng; q0 += 64) {
          const int q = q0 + lane;
          const bool act = q < ng;
          Bits<W> f;
#pragma unroll
          for (int k = 0; k < W; ++k) f.w[k] = act ? lgx[q * W + k] : 0;
          const bool ok = act && sector_ok<W>(x, f);
          const unsigned long long bal = __ballot(ok);
          if (ok) kept[nk + __popcll(bal & ((1ull << lane) - 1))] = q;
          nk += __popcll(bal);
          __builtin_amdgcn_wave_barrier();
          if (nk >= 64) {
            evaluate(64);
            __builtin_amdgcn_wave_barrier();
            if (lane < nk - 64) kept[lane] = kept[64 + lane];
            __builtin_amdgcn_wave_barrier();
            nk -= 64;
          }
        }
        if (nk > 0) evaluate(nk);
        __builtin_amdgcn_wave_barrier();
      } else {
        // without the sector test a group is kept where h != 0: every group is evaluated
        for (int q0 = 0; q0 < ng; q0 += 64) {
          const int q = q0 + lane;
          const bool act = q < ng;
          Bits<W> f;
#pragma unroll
          for (int k = 0; k < W; ++k) f.w[k] = act ? lgx[q * W + k] : 0;
          double a = 0.0, b = 0.0;
          if (act) group_sum(q, a, b);
          const bool ok = act && ((a != 0.0) || (b != 0.0));
          const unsigned long long bal = __ballot(ok);
          if (ok) store(pos + __popcll(bal & ((1ull << lane) - 1)), f, a, b);
          pos += __popcll(bal);
        }
      }
      if (lane == j) pos_l = pos;
    }
    gb = ge;
  }
  if (over) atomicOr(err, kErrEntryOverflow);
}

template <int W>
static void launch_write_w(const HamDev& H, const uint64_t* x, long long S, int R, int gper,
                           const long long* off, long long cap, uint64_t* xe, double* he, int* esample,
                           int hstride, unsigned* err, hipStream_t s) {
  dim3 grid((unsigned)((S + 255) / 256), (unsigned)R);
  if (H.tim)
    hipLaunchKernelGGL((write_kernel<true, W>), grid, dim3(256), 0, s, H, x, S, R, gper, off, cap, xe, he,
                       esample, hstride, err);
  else
    hipLaunchKernelGGL((write_kernel<false, W>), grid, dim3(256), 0, s, H, x, S, R, gper, off, cap, xe,
                       he, esample, hstride, err);
}

void launch_write(const HamDev& H, const uint64_t* x, long long S, int R, int gper,
                  const long long* off, long long cap, uint64_t* xe, double* he, int* esample,
                  int hstride, unsigned* err, hipStream_t s) {
  if (S <= 0) return;
  if (!H.tables && H.max_gterms <= kWsTerms) {
    const dim3 grid((unsigned)((S + kWsSamples - 1) / kWsSamples), (unsigned)R), block(64 * kWsWaves);
    if (H.words == 2) {
      if (H.tim) hipLaunchKernelGGL((write_staged_kernel<true, 2>), grid, block, 0, s, H, x, S, R, gper, off, cap, xe,
                                    he, esample, hstride, err);
      else hipLaunchKernelGGL((write_staged_kernel<false, 2>), grid, block, 0, s, H, x, S, R, gper, off, cap, xe,
                              he, esample, hstride, err);
    } else {
      if (H.tim) hipLaunchKernelGGL((write_staged_kernel<true, 1>), grid, block, 0, s, H, x, S, R, gper, off, cap, xe,
                                    he, esample, hstride, err);
      else hipLaunchKernelGGL((write_staged_kernel<false, 1>), grid, block, 0, s, H, x, S, R, gper, off, cap, xe,
                              he, esample, hstride, err);
    }
    return;
  }
  if (H.words == 2) launch_write_w<2>(H, x, S, R, gper, off, cap, xe, he, esample, hstride, err, s);
  else launch_write_w<1>(H, x, S, R, gper, off, cap, xe, he, esample, hstride, err, s);
}

__global__ void copy_i64_kernel(const long long* src, long long* dst) { *dst = *src; }
void launch_copy_i64(const long long* src, long long* dst, hipStream_t s) {
  hipLaunchKernelGGL(copy_i64_kernel, dim3(1), dim3(1), 0, s, src, dst);
}

// off[i] = first entry whose sample index is >= i (entries sample-major), i in [0, B].
__global__ void seg_offsets_kernel(const int* __restrict__ es, long long n, long long B,
                                   long long* __restrict__ off) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > B) return;
  long long lo = 0, hi = n;
  while (lo < hi) {
    const long long mid = (lo + hi) >> 1;
    if (es[mid] < i) lo = mid + 1;
    else hi = mid;
  }
  off[i] = lo;
}
void launch_seg_offsets(const int* esample, long long n_entries, long long B, long long* off, hipStream_t s) {
  hipLaunchKernelGGL(seg_offsets_kernel, dim3((unsigned)((B + 1 + 255) / 256)), dim3(256), 0, s, esample,
                     n_entries, B, off);
}

// ------------------------------------------------------------------ dedup
// Open addressing with linear probing over a table of 16-byte records (a key
// word and an int: the owner or rank of the key), so that a probe and the
// update of its slot touch one cache line.  Keys are x' values; the all-ones
// word marks an empty slot, which below 64 qubits is no configuration.  At
// exactly 64 qubits, and for two-word keys, a key word is a slot word instead:
// (hash tag << 32) | the entry that inserted the key (entries < 2^30, so a
// slot word is never the all-ones marker), and a probe whose tag matches
// compares the full key with that entry's words.
//
// Two orders of the distinct configurations:
//  - first-entry order (the connected-set call, whose output lists them): each
//    slot records the smallest entry holding its key, then a scan over the
//    first holders ranks them, sample-major as the entries are, independent
//    of the hash layout and of scheduling;
//  - insertion order (the local-energy chunks): the entry whose insert filled
//    a slot ranks it, each workgroup taking a block of ranks for its inserts
//    in entry order.  One pass and one table line per entry; the ranks follow
//    the entries' order up to the interleaving of workgroups.  Every row's log
//    psi depends on that row alone, so the order changes no value.
constexpr unsigned long long kEmpty = ~0ull;
constexpr int kDedupTile = 2048;
constexpr int kDedupLds = 4096;
constexpr int kNoEntry = 0x7FFFFFFF;

struct __align__(16) HRec {
  unsigned long long key;
  int rank;   // the owner (smallest entry) while inserting in first-entry order, then the rank
  int pad;
};
static_assert(sizeof(HRec) == kHashRecBytes, "hash record size");

__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z ^= z >> 30; z *= 0xbf58476d1ce4e5b9ull;
  z ^= z >> 27; z *= 0x94d049bb133111ebull;
  z ^= z >> 31;
  return z;
}

__global__ void fill_rec_kernel(HRec* __restrict__ t, long long count) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  HRec e;
  e.key = kEmpty;
  e.rank = kNoEntry;
  e.pad = 0;
  for (; i < count; i += stride) t[i] = e;
}

// First-entry order, one-word keys below 64 qubits: each workgroup collapses
// its tile of entries in an LDS table first, then inserts the tile-unique keys.
// eu[e] <- global slot of entry e's key; rank field <- smallest entry holding it.
__global__ __launch_bounds__(512) void dedup_insert_kernel(const uint64_t* __restrict__ xe,
                                                           const long long* __restrict__ d_count,
                                                           long long cap, HRec* __restrict__ tab,
                                                           long long HT, int* __restrict__ eu,
                                                           unsigned* err) {
  __shared__ unsigned long long lkeys[kDedupLds];
  __shared__ int lglob[kDedupLds];
  __shared__ int lmin[kDedupLds];
  long long count = *d_count;
  if (count > cap) count = cap;
  const long long e0 = (long long)blockIdx.x * kDedupTile;
  if (e0 >= count) return;
  for (int s = threadIdx.x; s < kDedupLds; s += blockDim.x) {
    lkeys[s] = kEmpty;
    lglob[s] = -1;
    lmin[s] = kNoEntry;
  }
  __syncthreads();
  int lslot[kDedupTile / 512];
#pragma unroll
  for (int q = 0; q < kDedupTile / 512; ++q) {
    const long long e = e0 + q * 512 + threadIdx.x;
    lslot[q] = -1;
    if (e < count) {
      const unsigned long long key = xe[e];
      unsigned s = (unsigned)mix64(key) & (kDedupLds - 1);
      for (int probe = 0; probe < kDedupLds; ++probe) {
        unsigned long long prev = atomicCAS(&lkeys[s], kEmpty, key);
        if (prev == kEmpty || prev == key) { lslot[q] = (int)s; break; }
        s = (s + 1) & (kDedupLds - 1);
      }
      if (lslot[q] >= 0) atomicMin(&lmin[lslot[q]], (int)e);
    }
  }
  __syncthreads();
  const unsigned long long hmask = (unsigned long long)HT - 1;
  for (int s = threadIdx.x; s < kDedupLds; s += blockDim.x) {
    const unsigned long long key = lkeys[s];
    if (key == kEmpty) continue;
    unsigned long long gs = mix64(key) & hmask;
    int found = -1;
    for (long long probe = 0; probe < HT; ++probe) {
      unsigned long long prev = atomicCAS(&tab[gs].key, kEmpty, key);
      if (prev == kEmpty || prev == key) { found = (int)gs; break; }
      gs = (gs + 1) & hmask;
    }
    if (found < 0) atomicOr(err, kErrHashOverflow);
    else atomicMin(&tab[found].rank, lmin[s]);
    lglob[s] = found;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kDedupTile / 512; ++q) {
    const long long e = e0 + q * 512 + threadIdx.x;
    if (e < count) eu[e] = lslot[q] >= 0 ? lglob[lslot[q]] : -1;
  }
}

// Probe for entry e's key (W words, key: its words, hsh: its hash); inserts it
// when absent.  Returns the slot (or -1 when the table is full) and sets won
// when this call filled the slot; where the key was already there, rank is
// its slot's rank field, read right away (kNoEntry until its inserter writes
// it; written once, so any other value is final).
template <int W, bool SLOT>
__device__ __forceinline__ int dedup_probe_insert(const uint64_t* __restrict__ xe, long long e,
                                                  const uint64_t (&key)[W], unsigned long long hsh,
                                                  HRec* __restrict__ tab, long long HT, bool& won, int& rank) {
  const unsigned long long mine = SLOT ? ((hsh & 0xFFFFFFFF00000000ull) | (unsigned long long)e) : key[0];
  const unsigned long long hmask = (unsigned long long)HT - 1;
  unsigned long long gs = hsh & hmask;
  won = false;
  for (long long probe = 0; probe < HT; ++probe) {
    // a plain read first: a slot, once filled in this chunk, keeps its key word, so
    // a key read here is final and needs no atomic; an empty read (possibly stale)
    // goes to the CAS, which decides
    unsigned long long prev = __builtin_nontemporal_load(&tab[gs].key);
    if (prev == kEmpty) {
      prev = atomicCAS(&tab[gs].key, kEmpty, mine);
      if (prev == kEmpty) { won = true; return (int)gs; }
    }
    if constexpr (SLOT) {
      if ((prev >> 32) == (mine >> 32)) {
        const long long pe = (long long)(prev & 0xFFFFFFFFull);
        bool same = true;
#pragma unroll
        for (int k = 0; k < W; ++k) same = same && xe[W * pe + k] == key[k];
        if (same) {
          rank = __builtin_nontemporal_load(&tab[gs].rank);
          return (int)gs;
        }
      }
    } else {
      if (prev == mine) {
        rank = __builtin_nontemporal_load(&tab[gs].rank);
        return (int)gs;
      }
    }
    gs = (gs + 1) & hmask;
  }
  return -1;
}

template <int W>
__device__ __forceinline__ unsigned long long key_hash(const uint64_t (&key)[W]) {
  return W == 2 ? mix64(key[0] ^ mix64(key[W - 1])) : mix64(key[0]);
}

// First-entry order, slot words: one lane per entry, straight into the table.
// eu[e] <- global slot of entry e's key; rank field <- smallest entry holding it.
template <int W>
__global__ __launch_bounds__(256) void dedup_insert_slot_kernel(const uint64_t* __restrict__ xe,
                                                                const long long* __restrict__ d_count,
                                                                long long cap, HRec* __restrict__ tab,
                                                                long long HT, int* __restrict__ eu,
                                                                unsigned* err) {
  long long count = *d_count;
  if (count > cap) count = cap;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  uint64_t key[W];
#pragma unroll
  for (int k = 0; k < W; ++k) key[k] = xe[W * e + k];
  bool won;
  int rank_seen;
  const int found = dedup_probe_insert<W, true>(xe, e, key, key_hash<W>(key), tab, HT, won, rank_seen);
  if (found < 0) atomicOr(err, kErrHashOverflow);
  else atomicMin(&tab[found].rank, (int)e);
  eu[e] = found;
}

// Insertion order: one lane per entry.  The lane that fills a slot writes the
// key's rank into it and the key into xu[rank]; *d_nu counts the distinct
// keys (it starts at zero).  eu[e] <- the rank of entry e's key where it is
// known when the lane finishes (its own insert, or a rank already written by
// the key's inserter), else -1 - slot for dedup_remap_pending_kernel, and
// kRankOverflow where the table was full.
constexpr int kRankedThreads = 1024;
constexpr int kRankOverflow = 1 << 30;   // above every rank (entries < 2^30)
template <int W, bool SLOT>
__global__ __launch_bounds__(kRankedThreads) void dedup_insert_ranked_kernel(const uint64_t* __restrict__ xe,
                                                                  const long long* __restrict__ d_count,
                                                                  long long cap, HRec* __restrict__ tab,
                                                                  long long HT, int* __restrict__ eu,
                                                                  uint64_t* __restrict__ xu,
                                                                  long long* __restrict__ d_nu, unsigned* err) {
  constexpr int NWV = kRankedThreads / 64;
  __shared__ int wsum[NWV];
  __shared__ long long base;
  long long count = *d_count;
  if (count > cap) count = cap;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t key[W];
  bool won = false;
  int found = -1, rank_seen = kNoEntry;
  if (e < count) {
#pragma unroll
    for (int k = 0; k < W; ++k) key[k] = xe[W * e + k];
    found = dedup_probe_insert<W, SLOT>(xe, e, key, key_hash<W>(key), tab, HT, won, rank_seen);
    if (found < 0) {
      atomicOr(err, kErrHashOverflow);
      eu[e] = kRankOverflow;
    }
  }
  // one block of ranks per workgroup, in entry order inside it
  const unsigned long long bal = __ballot(won);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) wsum[wv] = __popcll(bal);
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int w = 0; w < NWV; ++w) tot += wsum[w];
    base = tot ? (long long)atomicAdd((unsigned long long*)d_nu, (unsigned long long)tot) : 0;
  }
  __syncthreads();
  if (won) {
    int before = 0;
    for (int w = 0; w < wv; ++w) before += wsum[w];
    const long long r = base + before + __popcll(bal & ((1ull << lane) - 1));
    tab[found].rank = (int)r;
#pragma unroll
    for (int k = 0; k < W; ++k) xu[r * W + k] = key[k];
    eu[e] = (int)r;
  } else if (found >= 0) {
    eu[e] = rank_seen != kNoEntry ? rank_seen : -1 - found;
  }
}

// eu[e] <- the rank of its key for the entries the insert left pending
// (eu[e] = -1 - slot); -1 for kRankOverflow.
__global__ void dedup_remap_pending_kernel(const long long* __restrict__ d_count, long long cap,
                                           const HRec* __restrict__ tab, int* __restrict__ eu) {
  long long count = *d_count;
  if (count > cap) count = cap;
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (; e < count; e += stride) {
    const int v = eu[e];
    if (v >= 0 && v < kRankOverflow) continue;
    const int r = v < 0 ? tab[-1 - (long long)v].rank : kNoEntry;
    eu[e] = r != kNoEntry ? r : -1;
  }
}

// first[e] = 1 where entry e is the first holder of its key (0 beyond the count).
__global__ void dedup_first_kernel(const long long* __restrict__ d_count, long long cap,
                                   const int* __restrict__ eu, const HRec* __restrict__ tab,
                                   int* __restrict__ first) {
  long long count = *d_count;
  if (count > cap) count = cap;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < cap; e += stride) {
    int f = 0;
    if (e < count) {
      const int g = eu[e];
      f = (g >= 0 && tab[g].rank == (int)e) ? 1 : 0;
    }
    first[e] = f;
  }
}

// The first holders, in entry order: xu[rank] = key, the slot's rank field = rank.
template <int W>
__global__ void dedup_place_kernel(const long long* __restrict__ d_count, long long cap,
                                   const int* __restrict__ first, const long long* __restrict__ rank,
                                   const uint64_t* __restrict__ xe, const int* __restrict__ eu,
                                   HRec* __restrict__ tab, uint64_t* __restrict__ xu,
                                   long long* __restrict__ d_nu) {
  long long count = *d_count;
  if (count > cap) count = cap;
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long i0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i0 == 0) *d_nu = rank[cap];
  for (long long e = i0; e < count; e += stride) {
    if (!first[e]) continue;
    const long long id = rank[e];
#pragma unroll
    for (int k = 0; k < W; ++k) xu[id * W + k] = xe[e * W + k];
    tab[eu[e]].rank = (int)id;
  }
}

// eu[e] <- the rank of its slot's key.
__global__ void dedup_remap_kernel(const long long* __restrict__ d_count, long long cap,
                                   const HRec* __restrict__ tab, int* __restrict__ eu) {
  long long count = *d_count;
  if (count > cap) count = cap;
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (; e < count; e += stride) {
    const int s = eu[e];
    eu[e] = s >= 0 ? tab[s].rank : -1;
  }
}

long long dedup_rank_tmp_elems(long long cap) { return scan_tiles(cap) + 1; }

// Look-back to the previous chunk (one-word keys below 64 qubits, whose
// table holds the keys themselves): the previous chunk's table maps a key to
// its rank among that chunk's distinct configurations, so a distinct
// configuration of this chunk that the previous chunk already evaluated takes
// that value instead of a forward row.  src[u] = the previous rank or -1;
// isnew[u] = 1 where src[u] < 0 (0 past the count, for the scan).
__global__ void lookback_probe_kernel(const uint64_t* __restrict__ xu, const long long* __restrict__ d_nu,
                                      long long cap, const HRec* __restrict__ ptab, long long HT,
                                      int* __restrict__ src, int* __restrict__ isnew) {
  const long long nu = *d_nu < cap ? *d_nu : cap;
  const unsigned long long hmask = (unsigned long long)HT - 1;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x; u < cap; u += stride) {
    if (u >= nu) {
      isnew[u] = 0;
      continue;
    }
    const unsigned long long key = xu[u];
    unsigned long long gs = mix64(key) & hmask;
    int r = -1;
    for (long long probe = 0; probe < HT; ++probe) {
      const unsigned long long k = ptab[gs].key;
      if (k == key) { r = ptab[gs].rank; break; }
      if (k == kEmpty) break;
      gs = (gs + 1) & hmask;
    }
    src[u] = r;
    isnew[u] = r < 0 ? 1 : 0;
  }
}

// The new configurations in order: xnew[rank[u]] = xu[u] (rank: the exclusive
// scan of isnew); *d_nnew = their number.
__global__ void lookback_compact_kernel(const uint64_t* __restrict__ xu, const long long* __restrict__ d_nu,
                                        long long cap, const int* __restrict__ isnew,
                                        const long long* __restrict__ rank, uint64_t* __restrict__ xnew,
                                        long long* __restrict__ d_nnew) {
  const long long nu = *d_nu < cap ? *d_nu : cap;
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long i0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i0 == 0) *d_nnew = rank[cap];
  for (long long u = i0; u < nu; u += stride)
    if (isnew[u]) xnew[rank[u]] = xu[u];
}

// lp[u] = lp_prev[src[u]] for a configuration the previous chunk evaluated,
// lp_new[rank[u]] for a new one (pairs of doubles).
__global__ void lookback_gather_kernel(const long long* __restrict__ d_nu, long long cap, const int* __restrict__ src,
                                       const long long* __restrict__ rank, const double2* __restrict__ lp_prev,
                                       const double2* __restrict__ lp_new, double2* __restrict__ lp) {
  const long long nu = *d_nu < cap ? *d_nu : cap;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x; u < nu; u += stride) {
    const int r = src[u];
    lp[u] = r >= 0 ? lp_prev[r] : lp_new[rank[u]];
  }
}

static long long lookback_blocks(long long cap) {
  long long blocks = (cap + 255) / 256;
  return blocks > 16384 ? 16384 : (blocks < 1 ? 1 : blocks);
}

void launch_lookback(const uint64_t* xu, const long long* d_nu, long long cap, const void* ptable, long long HT,
                     int* src, int* isnew, long long* rank, long long* rank_tmp, uint64_t* xnew, long long* d_nnew,
                     hipStream_t s) {
  const long long blocks = lookback_blocks(cap);
  hipLaunchKernelGGL(lookback_probe_kernel, dim3((unsigned)blocks), dim3(256), 0, s, xu, d_nu, cap,
                     (const HRec*)ptable, HT, src, isnew);
  launch_scan(isnew, cap, rank, rank_tmp, s);
  hipLaunchKernelGGL(lookback_compact_kernel, dim3((unsigned)blocks), dim3(256), 0, s, xu, d_nu, cap, isnew, rank,
                     xnew, d_nnew);
}

void launch_lookback_gather(const long long* d_nu, long long cap, const int* src, const long long* rank,
                            const double* lp_prev, const double* lp_new, double* lp, hipStream_t s) {
  hipLaunchKernelGGL(lookback_gather_kernel, dim3((unsigned)lookback_blocks(cap)), dim3(256), 0, s, d_nu, cap, src,
                     rank, (const double2*)lp_prev, (const double2*)lp_new, (double2*)lp);
}

void launch_dedup(const uint64_t* xe, int words, bool all_ones_key, const long long* d_count, long long cap,
                  void* table, long long HT, bool first_order, int* eu, uint64_t* xu, long long* d_nu, int* first,
                  long long* rank, long long* rank_tmp, unsigned* err, hipStream_t s) {
  HRec* tab = (HRec*)table;
  {
    long long blocks = (HT + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(fill_rec_kernel, dim3((unsigned)blocks), dim3(256), 0, s, tab, HT);
  }
  launch_fill_u64(d_nu, 0ull, 1, s);
  if (cap <= 0) return;
  long long blocks = (cap + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  const bool slot = words == 2 || all_ones_key;
  const unsigned lane_blocks = (unsigned)((cap + 255) / 256);
  if (!first_order) {
    const dim3 g((unsigned)((cap + kRankedThreads - 1) / kRankedThreads)), b(kRankedThreads);
    if (words == 2)
      hipLaunchKernelGGL((dedup_insert_ranked_kernel<2, true>), g, b, 0, s, xe, d_count, cap, tab, HT, eu, xu, d_nu,
                         err);
    else if (slot)
      hipLaunchKernelGGL((dedup_insert_ranked_kernel<1, true>), g, b, 0, s, xe, d_count, cap, tab, HT, eu, xu, d_nu,
                         err);
    else
      hipLaunchKernelGGL((dedup_insert_ranked_kernel<1, false>), g, b, 0, s, xe, d_count, cap, tab, HT, eu, xu, d_nu,
                         err);
    hipLaunchKernelGGL(dedup_remap_pending_kernel, dim3((unsigned)blocks), dim3(256), 0, s, d_count, cap,
                       (const HRec*)tab, eu);
    return;
  }
  if (words == 2)
    hipLaunchKernelGGL(dedup_insert_slot_kernel<2>, dim3(lane_blocks), dim3(256), 0, s, xe, d_count, cap, tab, HT,
                       eu, err);
  else if (slot)
    hipLaunchKernelGGL(dedup_insert_slot_kernel<1>, dim3(lane_blocks), dim3(256), 0, s, xe, d_count, cap, tab, HT,
                       eu, err);
  else
    hipLaunchKernelGGL(dedup_insert_kernel, dim3((unsigned)((cap + kDedupTile - 1) / kDedupTile)), dim3(512), 0, s,
                       xe, d_count, cap, tab, HT, eu, err);
  hipLaunchKernelGGL(dedup_first_kernel, dim3((unsigned)blocks), dim3(256), 0, s, d_count, cap, eu,
                     (const HRec*)tab, first);
  launch_scan(first, cap, rank, rank_tmp, s);
  auto place = words == 2 ? dedup_place_kernel<2> : dedup_place_kernel<1>;
  hipLaunchKernelGGL(place, dim3((unsigned)blocks), dim3(256), 0, s, d_count, cap, first, rank, xe, eu, tab, xu,
                     d_nu);
  hipLaunchKernelGGL(dedup_remap_kernel, dim3((unsigned)blocks), dim3(256), 0, s, d_count, cap,
                     (const HRec*)tab, eu);
}

// ------------------------------------------------------- ratio-and-reduce
// Neumaier-compensated accumulation, then a fixed-shape tree: the result
// does not depend on scheduling.
struct Comp {
  double s, c;
  __device__ void add(double v) {
    double t = s + v;
    if (fabs(s) >= fabs(v)) c += (s - t) + v;
    else c += (v - t) + s;
    s = t;
  }
  __device__ void merge(const Comp& o) {
    add(o.s);
    c += o.c;
  }
  __device__ double value() const { return s + c; }
};

// E_loc(x_i) = diag_i + sum_e h_e exp(lp(x'_e) - lp(x_i)).  Each sample's
// entries are cut into kReduceSlices equal slices, one workgroup each
// (enough workgroups to keep every CU streaming); a slice is summed with
// per-thread compensation and a fixed tree, and the slices are then added to
// the diagonal in slice order.  The cut depends only on the sample's own
// entry range, so the result does not depend on scheduling or chunking.
constexpr int kReduceSlices = 8;

__global__ __launch_bounds__(256) void reduce_part_kernel(long long S, int R, const long long* __restrict__ off,
                                                          long long cap, const double* __restrict__ he,
                                                          int hstride, const int* __restrict__ eu,
                                                          const double2* __restrict__ lpe,
                                                          const double2* __restrict__ lps,
                                                          double* __restrict__ partials) {
  __shared__ double red[4][256];
  const long long i = blockIdx.x / kReduceSlices;
  const int part = (int)(blockIdx.x % kReduceSlices);
  if (i >= S) return;
  long long a = off[i * R];
  long long b = off[(i + 1) * R];
  if (a > cap) a = cap;
  if (b > cap) b = cap;
  const long long per = (b - a + kReduceSlices - 1) / kReduceSlices;
  const long long pa = a + part * per;
  const long long pb = pa + per < b ? pa + per : b;
  const double2 ls = lps[i];
  Comp cr{0.0, 0.0}, ci{0.0, 0.0};
  for (long long e = pa + threadIdx.x; e < pb; e += 256) {
    const int u = eu ? eu[e] : (int)0;
    const double2 lp = eu ? (u >= 0 ? lpe[u] : make_double2(-INFINITY, 0.0)) : lpe[e];
    if (lp.x == -INFINITY) continue;
    const double hr = he[e * hstride];
    const double hi = hstride == 2 ? he[e * 2 + 1] : 0.0;
    const double mag = exp(lp.x - ls.x);
    double sn, cs;
    sincos(lp.y - ls.y, &sn, &cs);
    cr.add(mag * (hr * cs - hi * sn));
    ci.add(mag * (hr * sn + hi * cs));
  }
  red[0][threadIdx.x] = cr.s;
  red[1][threadIdx.x] = cr.c;
  red[2][threadIdx.x] = ci.s;
  red[3][threadIdx.x] = ci.c;
  __syncthreads();
  for (int d = 128; d >= 1; d >>= 1) {
    if ((int)threadIdx.x < d) {
      Comp x{red[0][threadIdx.x], red[1][threadIdx.x]}, y{red[0][threadIdx.x + d], red[1][threadIdx.x + d]};
      x.merge(y);
      red[0][threadIdx.x] = x.s;
      red[1][threadIdx.x] = x.c;
      Comp p{red[2][threadIdx.x], red[3][threadIdx.x]}, q{red[2][threadIdx.x + d], red[3][threadIdx.x + d]};
      p.merge(q);
      red[2][threadIdx.x] = p.s;
      red[3][threadIdx.x] = p.c;
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) partials[(i * kReduceSlices + part) * 4 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void reduce_combine_kernel(long long S, const double* __restrict__ diag,
                                      const double2* __restrict__ lps, const double* __restrict__ partials,
                                      double* __restrict__ eloc, unsigned* err) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S) return;
  Comp tr{diag[2 * i], 0.0}, ti{diag[2 * i + 1], 0.0};
  for (int k = 0; k < kReduceSlices; ++k) {
    const double* q = partials + (i * kReduceSlices + k) * 4;
    tr.merge(Comp{q[0], q[1]});
    ti.merge(Comp{q[2], q[3]});
  }
  if (lps[i].x == -INFINITY) {
    atomicOr(err, kErrZeroAmp);
    eloc[2 * i] = NAN;
    eloc[2 * i + 1] = NAN;
  } else {
    eloc[2 * i] = tr.value();
    eloc[2 * i + 1] = ti.value();
  }
}

long long reduce_partials_elems(long long S) { return S * kReduceSlices * 4; }

void launch_reduce(long long S, int R, const long long* off, long long cap, const double* diag,
                   const double* he, int hstride, const int* eu, const double* lpe,
                   const double* lps, double* eloc, double* partials, unsigned* err, hipStream_t s) {
  if (S <= 0) return;
  hipLaunchKernelGGL(reduce_part_kernel, dim3((unsigned)(S * kReduceSlices)), dim3(256), 0, s, S, R, off, cap,
                     he, hstride, eu, (const double2*)lpe, (const double2*)lps, partials);
  hipLaunchKernelGGL(reduce_combine_kernel, dim3((unsigned)((S + 255) / 256)), dim3(256), 0, s, S, diag,
                     (const double2*)lps, (const double*)partials, eloc, err);
}

// Weighted energy: W = sum w, E = sum w Re(l) / W, I = sum w Im(l) / W.
__global__ __launch_bounds__(1024) void energy_kernel(const double* __restrict__ eloc,
                                                      const double* __restrict__ w, long long B,
                                                      double* __restrict__ energy, unsigned* err) {
  __shared__ double red[6][1024];
  const int t = threadIdx.x;
  Comp sw{0, 0}, sr{0, 0}, si{0, 0};
  for (long long i = t; i < B; i += 1024) {
    const double wi = w ? w[i] : 1.0;
    sw.add(wi);
    sr.add(wi * eloc[2 * i]);
    si.add(wi * eloc[2 * i + 1]);
  }
  red[0][t] = sw.s; red[1][t] = sw.c; red[2][t] = sr.s; red[3][t] = sr.c; red[4][t] = si.s; red[5][t] = si.c;
  __syncthreads();
  for (int d = 512; d >= 1; d >>= 1) {
    if (t < d) {
      for (int k = 0; k < 3; ++k) {
        Comp a{red[2 * k][t], red[2 * k + 1][t]}, b{red[2 * k][t + d], red[2 * k + 1][t + d]};
        a.merge(b);
        red[2 * k][t] = a.s;
        red[2 * k + 1][t] = a.c;
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    const double W = red[0][0] + red[1][0];
    energy[0] = (red[2][0] + red[3][0]) / W;
    energy[1] = (red[4][0] + red[5][0]) / W;
    energy[2] = W;
    if (!(W > 0.0)) atomicOr(err, kErrZeroAmp);
  }
}

void launch_energy(const double* eloc, const double* w, long long B, double* energy, unsigned* err,
                   hipStream_t s) {
  hipLaunchKernelGGL(energy_kernel, dim3(1), dim3(1024), 0, s, eloc, w, B, energy, err);
}

}  // namespace nqs
