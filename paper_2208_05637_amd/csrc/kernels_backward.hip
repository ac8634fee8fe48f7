// Parameter packing, and the hand-written backward pass of the VMC gradient
// (Sec. 3, Eq. grad): the sample forward is recomputed per chunk of samples
// (activations of connected configurations are never stored), the output
// seeds are built from the local energies, and masked GEMMs propagate them to
// every weight and bias.
#include "nqs_internal.h"

namespace nqs {

// ------------------------------------------------------------------ masks
// In original (unpacked) indexing; degrees: qubit j -> 1 + pos[j], hidden
// unit k -> 1 + k mod (n-1).
enum MaskKind { MK_NONE = 0, MK_L1 = 1, MK_HID = 2, MK_HEAD_O = 3, MK_HEAD_P = 4 };

__device__ __forceinline__ bool mask_at(const Geom& g, int kind, int row, int col) {
  const int nm1 = g.n - 1;
  switch (kind) {
    case MK_L1: return (row % nm1) + 1 >= g.pos[col] + 1;
    case MK_HID: return (row % nm1) >= (col % nm1);
    case MK_HEAD_O: return g.pos[row] + 1 > (col % nm1) + 1;
    case MK_HEAD_P: return (col % nm1) + 1 <= g.n - 2;
  }
  return true;
}

// Which tensor of the flat layout holds parameter p: returns kind and
// (row, col) for weights, or -1 kind for a bias.  The layers of a separate
// phase network and its head are dense (MK_NONE).
__device__ __forceinline__ void locate(const Geom& g, long long p, int& tensor, int& kind, int& row,
                                       int& col, int& in) {
  const int L = g.L;
  const int ntens = g.phase_mode ? 4 * L + 4 : 2 * L + 4;
  int t = 0;
  while (t + 1 < ntens && p >= g.poff[t + 1]) ++t;
  tensor = t;
  const long long local = p - g.poff[t];
  if (g.phase_mode && t >= 2 * L + 2 && t < 4 * L + 2) {
    const int l = (t - 2 * L - 2) / 2 + 1;
    in = l == 1 ? g.n - 2 : g.h;
    if ((t - 2 * L - 2) % 2 == 0) {
      kind = MK_NONE;
      row = (int)(local / in);
      col = (int)(local % in);
    } else {
      kind = -1;
      row = (int)local;
      col = 0;
    }
    return;
  }
  if (g.phase_mode && t >= 4 * L + 2) t -= 2 * L;   // the phase head, as a head below
  if (t < 2 * L) {
    const int l = t / 2;
    in = l == 0 ? g.n : g.h;
    if (t % 2 == 0) {
      kind = l == 0 ? MK_L1 : MK_HID;
      row = (int)(local / in);
      col = (int)(local % in);
    } else {
      kind = -1;
      row = (int)local;
      col = 0;
    }
  } else {
    const int k = t - 2 * L;   // 0 W_o, 1 b_o, 2 W_p, 3 b_p
    in = g.h;
    if (k == 0 || k == 2) {
      kind = k == 0 ? MK_HEAD_O : (g.phase_mode ? MK_NONE : MK_HEAD_P);
      row = (int)(local / g.h);
      col = (int)(local % g.h);
    } else {
      kind = -1;
      row = (int)local;
      col = 0;
    }
  }
}

__device__ __forceinline__ unsigned short rne_bf16(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// With BF16 weights (P_BF16W) the network's weights are the parameters
// rounded to BF16; the backward differentiates that network.
template <typename T>
__global__ void pack_masked_kernel(Geom g, const float* __restrict__ params, T* __restrict__ wm) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.n_params) return;
  int tensor, kind, row, col, in;
  locate(g, p, tensor, kind, row, col, in);
  float v = params[p];
  if (kind >= 0 && g.prec == P_BF16W) v = __uint_as_float(((unsigned)rne_bf16(v)) << 16);
  wm[p] = (kind < 0 || mask_at(g, kind, row, col)) ? (T)v : (T)0;
}

void launch_pack_masked(const Geom& g, const float* params, void* wm, hipStream_t s) {
  const unsigned blocks = (unsigned)((g.n_params + 255) / 256);
  if (g.prec == P_F64)
    hipLaunchKernelGGL(pack_masked_kernel<double>, dim3(blocks), dim3(256), 0, s, g, params, (double*)wm);
  else
    hipLaunchKernelGGL(pack_masked_kernel<float>, dim3(blocks), dim3(256), 0, s, g, params, (float*)wm);
}

// ---------------------------------------------------- fused-kernel packing
// Value of the packed operand of fragment part (layer 1 / hidden / head) at
// sorted row `row` and packed column `k`, zero where masked or out of range.
__device__ float packed_value(const Geom& g, const float* params, int part, int layer, int row, int k) {
  const int n = g.n, h = g.h;
  if (g.net_kind == 2) {         // separate phase network: dense, units in their own order
    if (part == 0) {             // columns: the first n-2 positions
      if (row >= h || k >= n - 2) return 0.f;
      return params[g.poff[poff_phase_layer(g, 1)] + (long long)row * (n - 2) + k];
    }
    if (part == 1) {
      if (row >= h || k >= h) return 0.f;
      return params[g.poff[poff_phase_layer(g, layer)] + (long long)row * h + k];
    }
    if (row >= 4 || k >= h) return 0.f;
    return params[g.poff[poff_phase_head(g)] + (long long)row * h + k];
  }
  if (part == 0) {               // layer 1: rows sorted units, cols positions
    if (row >= h || k >= n) return 0.f;
    const int deg = class_of_sorted(g, row) + 1;
    if (!(k < deg)) return 0.f;
    return params[g.poff[0] + (long long)orig_of_sorted(g, row) * n + g.order[k]];
  }
  if (part == 1) {               // hidden layer `layer` (2..L)
    if (row >= h || k >= h) return 0.f;
    const int lim = prefix_of_class(g, class_of_sorted(g, row) + 1);
    if (!(k < lim)) return 0.f;
    return params[g.poff[2 * (layer - 1)] + (long long)orig_of_sorted(g, row) * h + orig_of_sorted(g, k)];
  }
  // head: rows positions 0..n-1 then 4 phase rows
  if (k >= h || row >= n + 4) return 0.f;
  if (row < n) {
    if (!(k < prefix_of_class(g, row))) return 0.f;
    return params[g.poff[2 * g.L] + (long long)g.order[row] * h + orig_of_sorted(g, k)];
  }
  if (g.net_kind == 1 || !(k < prefix_of_class(g, n - 2))) return 0.f;
  return params[g.poff[poff_phase_head(g)] + (long long)(row - n) * h + orig_of_sorted(g, k)];
}

__global__ void pack_fused_kernel(Geom g, const float* __restrict__ params, uint4* __restrict__ out) {
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long f = tid >> 6;
  const int lane = (int)(tid & 63);
  if (f >= g.nfrag) return;
  int part, layer = 1, blk, ks;
  long long local;
  if (f < g.frag_h) {
    part = 0;
    local = f;
    blk = 0;
    while (blk + 1 <= g.NB && local >= g.off1[blk + 1]) ++blk;
    ks = (int)(local - g.off1[blk]);
  } else if (f < g.frag_head) {
    part = 1;
    const long long per = g.offh[g.NB];
    layer = 2 + (int)((f - g.frag_h) / per);
    local = (f - g.frag_h) % per;
    blk = 0;
    while (blk + 1 <= g.NB && local >= g.offh[blk + 1]) ++blk;
    ks = (int)(local - g.offh[blk]);
  } else {
    part = 2;
    local = f - g.frag_head;
    blk = 0;
    while (blk + 1 <= g.NHB && local >= g.offo[blk + 1]) ++blk;
    ks = (int)(local - g.offo[blk]);
  }
  uint4 hi = make_uint4(0, 0, 0, 0), lo = make_uint4(0, 0, 0, 0);
  if (g.prec == P_BF16 || g.prec == P_BF16X3 || g.prec == P_BF16W) {
    const int row = 32 * blk + (lane & 31);
    const int k0 = 16 * ks + 8 * (lane >> 5);
    unsigned short vh[8], vl[8];
    for (int j = 0; j < 8; ++j) {
      const float v = packed_value(g, params, part, layer, row, k0 + j);
      vh[j] = rne_bf16(v);
      vl[j] = rne_bf16(v - __uint_as_float(((unsigned)vh[j]) << 16));
    }
    hi = make_uint4(vh[0] | (vh[1] << 16), vh[2] | (vh[3] << 16), vh[4] | (vh[5] << 16), vh[6] | (vh[7] << 16));
    lo = make_uint4(vl[0] | (vl[1] << 16), vl[2] | (vl[3] << 16), vl[4] | (vl[5] << 16), vl[6] | (vl[7] << 16));
  } else if (g.prec == P_F32) {
    const int row = 32 * blk + (lane & 31);
    const int k0 = 8 * ks + 4 * (lane >> 5);
    float v[4];
    for (int j = 0; j < 4; ++j) v[j] = packed_value(g, params, part, layer, row, k0 + j);
    hi = __builtin_bit_cast(uint4, make_float4(v[0], v[1], v[2], v[3]));
  } else {
    const int row = 16 * blk + (lane & 15);
    const int k0 = 8 * ks + 2 * (lane >> 4);
    double v[2];
    for (int j = 0; j < 2; ++j) v[j] = (double)packed_value(g, params, part, layer, row, k0 + j);
    hi = __builtin_bit_cast(uint4, make_double2(v[0], v[1]));
  }
  out[f * 64 + lane] = hi;
  if (g.planes == 2) out[(g.nfrag + f) * 64 + lane] = lo;
}

template <typename S>
__global__ void pack_bias_kernel(Geom g, const float* __restrict__ params, S* __restrict__ b) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nh = (long long)g.L * g.h;
  const long long total = nh + (long long)g.NHB * g.TB;
  if (i >= total) return;
  S v = 0;
  if (g.net_kind == 2) {
    if (i < nh) {
      const int l = (int)(i / g.h), u = (int)(i % g.h);
      v = (S)params[g.poff[poff_phase_layer(g, l + 1) + 1] + u];
    } else {
      const int t = (int)(i - nh);
      if (t < 4) v = (S)params[g.poff[poff_phase_head(g) + 1] + t];
    }
  } else if (i < nh) {
    const int l = (int)(i / g.h), u = (int)(i % g.h);
    v = (S)params[g.poff[2 * l + 1] + orig_of_sorted(g, u)];
  } else {
    const int t = (int)(i - nh);
    if (t < g.n) v = (S)params[g.poff[2 * g.L + 1] + g.order[t]];
    else if (t < g.n + 4 && g.net_kind == 0) v = (S)params[g.poff[poff_phase_head(g) + 1] + (t - g.n)];
  }
  b[i] = v;
}

void launch_pack_fused(const Geom& g, const float* params, void* packed, hipStream_t s) {
  const long long threads = g.nfrag * 64;
  hipLaunchKernelGGL(pack_fused_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, g,
                     params, (uint4*)packed);
  const long long nb = (long long)g.L * g.h + (long long)g.NHB * g.TB;
  void* bias = (char*)packed + g.bias_byte;
  if (g.prec == P_F64)
    hipLaunchKernelGGL(pack_bias_kernel<double>, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, g,
                       params, (double*)bias);
  else
    hipLaunchKernelGGL(pack_bias_kernel<float>, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, g,
                       params, (float*)bias);
}

// ------------------------------------------------------------ small GEMM
// C(i,j) = sum_k A(i,k) B(k,j) with A(i,k) = A[i*sa0 + k*sa1],
// B(k,j) = B[k*sb0 + j*sb1]; 64x64 tiles, 256 threads, 4x4 per thread.
enum Epi { E_FWD = 0, E_FWD_LIN = 1, E_STORE = 2, E_ADD = 3, E_GRAD = 4 };

struct GemmArgs {
  int Mr, Nc, K;
  const void* A; long long sa0, sa1;
  const void* B; long long sb0, sb1;
  void* C; long long ldc;
  const void* bias;        // E_FWD / E_FWD_LIN
  double* grad; long long grad_off; int mask_kind; long long grad_ld;   // E_GRAD
};

template <typename T, int EPI>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs a, Geom g) {
  __shared__ T As[16][65];
  __shared__ T Bs[16][65];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const T* A = (const T*)a.A;
  const T* B = (const T*)a.B;
  T acc[4][4] = {};
  for (int k0 = 0; k0 < a.K; k0 += 16) {
    for (int e = threadIdx.x; e < 1024; e += 256) {
      const int r = e >> 4, kk = e & 15;        // A tile: 64 rows x 16 k
      const int gi = i0 + r, gk = k0 + kk;
      As[kk][r] = (gi < a.Mr && gk < a.K) ? A[gi * a.sa0 + gk * a.sa1] : (T)0;
      const int kb = e >> 6, c = e & 63;        // B tile: 16 k x 64 cols
      const int gkb = k0 + kb, gj = j0 + c;
      Bs[kb][c] = (gkb < a.K && gj < a.Nc) ? B[gkb * a.sb0 + gj * a.sb1] : (T)0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      T av[4], bv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) { av[q] = As[kk][ty + 16 * q]; bv[q] = Bs[kk][tx + 16 * q]; }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] += av[p] * bv[q];
    }
    __syncthreads();
  }
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int i = i0 + ty + 16 * p;
    if (i >= a.Mr) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = j0 + tx + 16 * q;
      if (j >= a.Nc) continue;
      T v = acc[p][q];
      if constexpr (EPI == E_FWD || EPI == E_FWD_LIN) {
        v += ((const T*)a.bias)[j];
        if (EPI == E_FWD) v = v > (T)0 ? v : (T)0;
        ((T*)a.C)[i * a.ldc + j] = v;
      } else if constexpr (EPI == E_STORE) {
        ((T*)a.C)[i * a.ldc + j] = v;
      } else if constexpr (EPI == E_ADD) {
        ((T*)a.C)[i * a.ldc + j] += v;
      } else {
        if (mask_at(g, a.mask_kind, i, j)) a.grad[a.grad_off + (long long)i * a.grad_ld + j] += (double)v;
      }
    }
  }
}

// The FP32 form on the matrix cores: the same 64x64 tiles and 16-deep k
// steps through LDS; each of the four waves owns a 32x32 quarter of the tile
// and accumulates it with v_mfma_f32_32x32x2f32 (lane l supplies A row l % 32
// and B column l % 32 at k = l / 32; accumulator r of lane l holds row
// 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32 of the quarter).
typedef __attribute__((ext_vector_type(16))) float gemm_f32x16;
template <int EPI>
__global__ __launch_bounds__(256) void gemm_mfma_kernel(GemmArgs a, Geom g) {
  __shared__ float As[16][65];
  __shared__ float Bs[16][65];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wy = wave >> 1, wx = wave & 1;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const float* A = (const float*)a.A;
  const float* B = (const float*)a.B;
  gemm_f32x16 acc = {};
  const int li = lane & 31, lk = lane >> 5;
  for (int k0 = 0; k0 < a.K; k0 += 16) {
    for (int e = threadIdx.x; e < 1024; e += 256) {
      const int r = e >> 4, kk = e & 15;        // A tile: 64 rows x 16 k
      const int gi = i0 + r, gk = k0 + kk;
      As[kk][r] = (gi < a.Mr && gk < a.K) ? A[gi * a.sa0 + gk * a.sa1] : 0.f;
      const int kb = e >> 6, c = e & 63;        // B tile: 16 k x 64 cols
      const int gkb = k0 + kb, gj = j0 + c;
      Bs[kb][c] = (gkb < a.K && gj < a.Nc) ? B[gkb * a.sb0 + gj * a.sb1] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; kk += 2)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(As[kk + lk][wy * 32 + li], Bs[kk + lk][wx * 32 + li], acc, 0, 0, 0);
    __syncthreads();
  }
  const int j = j0 + wx * 32 + li;
  if (j >= a.Nc) return;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = i0 + wy * 32 + 8 * (r >> 2) + 4 * lk + (r & 3);
    if (i >= a.Mr) continue;
    float v = acc[r];
    if constexpr (EPI == E_FWD || EPI == E_FWD_LIN) {
      v += ((const float*)a.bias)[j];
      if (EPI == E_FWD) v = v > 0.f ? v : 0.f;
      ((float*)a.C)[i * a.ldc + j] = v;
    } else if constexpr (EPI == E_STORE) {
      ((float*)a.C)[i * a.ldc + j] = v;
    } else if constexpr (EPI == E_ADD) {
      ((float*)a.C)[i * a.ldc + j] += v;
    } else {
      if (mask_at(g, a.mask_kind, i, j)) a.grad[a.grad_off + (long long)i * a.grad_ld + j] += (double)v;
    }
  }
}

template <typename T, int EPI>
static void gemm(const GemmArgs& a, const Geom& g, hipStream_t s) {
  if (a.Mr <= 0 || a.Nc <= 0) return;
  dim3 grid((unsigned)((a.Nc + 63) / 64), (unsigned)((a.Mr + 63) / 64));
  if constexpr (sizeof(T) == 4) hipLaunchKernelGGL((gemm_mfma_kernel<EPI>), grid, dim3(256), 0, s, a, g);
  else hipLaunchKernelGGL((gemm_kernel<T, EPI>), grid, dim3(256), 0, s, a, g);
}

// Bit of qubit j of sample i (g.words 64-bit words per sample).
__device__ __forceinline__ int qubit_bit(const Geom& g, const uint64_t* __restrict__ x, long long i, int j) {
  return (int)((x[i * g.words + (j >> 6)] >> (j & 63)) & 1ull);
}

template <typename T>
__global__ void bits_kernel(Geom g, const uint64_t* __restrict__ x, long long S, T* __restrict__ s) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= S * g.n) return;
  const long long i = e / g.n;
  const int j = (int)(e % g.n);
  s[e] = qubit_bit(g, x, i, j) ? (T)1 : (T)-1;
}

template <typename T>
__global__ void relu_mask_kernel(const T* __restrict__ act, T* __restrict__ d, long long count) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count && !(act[e] > (T)0)) d[e] = (T)0;
}

// grad[off + j] += sum_i D[i * ld + j] in a fixed order (deterministic): a
// workgroup takes 64 columns; each of its 16 row segments is summed in order
// in FP64, then the 16 segment sums in order.
constexpr int kColsumCols = 64, kColsumSegs = 16;
template <typename T>
__global__ __launch_bounds__(kColsumCols * kColsumSegs) void colsum_kernel(const T* __restrict__ D, long long S,
                                                                           int cols, long long ld,
                                                                           double* __restrict__ grad, long long off) {
  __shared__ double part[kColsumSegs][kColsumCols];
  const int c = threadIdx.x % kColsumCols, sg = threadIdx.x / kColsumCols;
  const int j = blockIdx.x * kColsumCols + c;
  const long long per = (S + kColsumSegs - 1) / kColsumSegs;
  const long long i0 = sg * per, i1 = i0 + per < S ? i0 + per : S;
  double acc = 0.0;
  if (j < cols)
    for (long long i = i0; i < i1; ++i) acc += (double)D[i * ld + j];
  part[sg][c] = acc;
  __syncthreads();
  if (sg == 0 && j < cols) {
    double t = 0.0;
    for (int q = 0; q < kColsumSegs; ++q) t += part[q][c];
    grad[off + j] += t;
  }
}
template <typename T>
static void colsum(const T* D, long long S, int cols, long long ld, double* grad, long long off, hipStream_t s) {
  if (cols <= 0) return;
  hipLaunchKernelGGL(colsum_kernel<T>, dim3((unsigned)((cols + kColsumCols - 1) / kColsumCols)),
                     dim3(kColsumCols * kColsumSegs), 0, s, D, S, cols, ld, grad, off);
}

// Output seeds for sample i with g_la = 2 (w/W)(Re l - E), g_phi = 2 (w/W) Im l:
// d o_j = g_la * 1/2 * free_j * (x_j - sigmoid(o_j)); d p_c = g_phi [c == sel].
template <typename T>
__global__ void seed_kernel(Geom g, const uint64_t* __restrict__ x, long long S,
                            const double* __restrict__ eloc, const double* __restrict__ w,
                            const double* __restrict__ energy, const T* __restrict__ hout,
                            T* __restrict__ dh) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S) return;
  const int n = g.n, ld = n + 4;
  const double W = energy[2], E = energy[0];
  const double wi = w ? w[i] : 1.0;
  const double gla = 2.0 * (wi / W) * (eloc[2 * i] - E);
  const double gph = 2.0 * (wi / W) * eloc[2 * i + 1];
  const bool constrained = g.n_up >= 0 && g.n_dn >= 0;
  int placed[2] = {0, 0};
  int remaining[2] = {(int)__popcll(g.spin_pos[0]) + (int)__popcll(g.spin_pos_hi[0]),
                      (int)__popcll(g.spin_pos[1]) + (int)__popcll(g.spin_pos_hi[1])};
  for (int t = 0; t < n; ++t) {
    const int j = g.order[t];
    const int sp = j & 1;
    remaining[sp] -= 1;
    const int bit = qubit_bit(g, x, i, j);
    bool fr = true;
    if (constrained) {
      const int ns = sp ? g.n_dn : g.n_up;
      fr = !(placed[sp] >= ns || placed[sp] + remaining[sp] < ns);
    }
    placed[sp] += bit;
    const double o = (double)hout[i * ld + j];
    const double sig = 1.0 / (1.0 + exp(-o));
    dh[i * ld + j] = fr ? (T)(gla * 0.5 * ((double)bit - sig)) : (T)0;
  }
  const int sel = 2 * qubit_bit(g, x, i, g.order[n - 2]) + qubit_bit(g, x, i, g.order[n - 1]);
  for (int c = 0; c < 4; ++c) dh[i * ld + n + c] = c == sel ? (T)gph : (T)0;
}

// Input of a separate phase network: the first n-2 entries in sampling order.
template <typename T>
__global__ void phase_input_kernel(Geom g, const T* __restrict__ s, long long S, T* __restrict__ v) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int np = g.n - 2;
  if (e >= S * np) return;
  const long long i = e / np;
  const int t = (int)(e % np);
  v[e] = s[i * g.n + g.order[t]];
}

// Forward of L ReLU layers over S rows: acts[l] = relu(in_l W_l^T + b_l), the
// weight and bias of layer l at poff[wi(l)], poff[wi(l) + 1].
template <typename T, class WIdx>
static void mlp_forward(const Geom& g, const T* wm, const T* in0, int k0, long long S, T* acts, WIdx wi,
                        hipStream_t s) {
  const int h = g.h;
  for (int l = 1; l <= g.L; ++l) {
    const int K = l == 1 ? k0 : h;
    GemmArgs a{};
    a.Mr = (int)S; a.Nc = h; a.K = K;
    a.A = l == 1 ? (const void*)in0 : (const void*)(acts + (long long)(l - 2) * S * h);
    a.sa0 = K; a.sa1 = 1;
    a.B = wm + g.poff[wi(l)]; a.sb0 = 1; a.sb1 = K;
    a.C = acts + (long long)(l - 1) * S * h; a.ldc = h;
    a.bias = wm + g.poff[wi(l) + 1];
    gemm<T, E_FWD>(a, g, s);
  }
}

// Reverse pass through those layers from d(acts[L]) in da: gradients of the
// weights (masked by mask_of(l)) and biases; da and dz are S x h scratch.
template <typename T, class WIdx, class MIdx>
static void mlp_backward(const Geom& g, const T* wm, const T* in0, int k0, long long S, const T* acts, T* da,
                         T* dz, double* grad, WIdx wi, MIdx mask_of, hipStream_t s) {
  const int h = g.h;
  for (int l = g.L; l >= 1; --l) {
    const int K = l == 1 ? k0 : h;
    const T* act = acts + (long long)(l - 1) * S * h;
    const T* prev = l == 1 ? in0 : acts + (long long)(l - 2) * S * h;
    const long long cnt = S * h;
    hipLaunchKernelGGL(relu_mask_kernel<T>, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, act, da, cnt);
    GemmArgs a{};
    a.Mr = h; a.Nc = K; a.K = (int)S;
    a.A = da; a.sa0 = 1; a.sa1 = h;
    a.B = prev; a.sb0 = K; a.sb1 = 1;
    a.grad = grad; a.grad_off = g.poff[wi(l)]; a.grad_ld = K;
    a.mask_kind = mask_of(l);
    gemm<T, E_GRAD>(a, g, s);
    colsum<T>(da, S, h, (long long)h, grad, g.poff[wi(l) + 1], s);
    if (l > 1) {
      GemmArgs b{};
      b.Mr = (int)S; b.Nc = K; b.K = h;
      b.A = da; b.sa0 = h; b.sa1 = 1;
      b.B = wm + g.poff[wi(l)]; b.sb0 = K; b.sb1 = 1;
      b.C = dz; b.ldc = K;
      gemm<T, E_STORE>(b, g, s);
      T* t = da; da = dz; dz = t;
    }
  }
}

template <typename T>
static void backward_t(const Geom& g, const T* wm, const uint64_t* x, long long S, const double* eloc,
                       const double* w, const double* energy, T* scratch, double* grad, hipStream_t s) {
  const int n = g.n, h = g.h, L = g.L, ld = n + 4;
  const bool two = g.phase_mode == 1;
  T* sb = scratch;
  T* acts = sb + S * n;
  T* hout = acts + (long long)L * S * h;
  T* dh = hout + S * ld;
  T* da = dh + S * ld;
  T* dz = da + S * h;
  T* pin = dz + S * h;                     // separate phase network: input and activations
  T* pacts = pin + S * (n - 2);
  const unsigned eb = (unsigned)((S * n + 255) / 256);
  hipLaunchKernelGGL(bits_kernel<T>, dim3(eb), dim3(256), 0, s, g, x, S, sb);
  // forward recompute
  auto trunk_w = [&](int l) { return 2 * (l - 1); };
  auto phase_w = [&](int l) { return poff_phase_layer(g, l); };
  mlp_forward<T>(g, wm, sb, n, S, acts, trunk_w, s);
  const T* aL = acts + (long long)(L - 1) * S * h;
  const T* phin = aL;                      // what the phase head reads
  if (two) {
    const long long ne = S * (n - 2);
    hipLaunchKernelGGL(phase_input_kernel<T>, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, g,
                       (const T*)sb, S, pin);
    mlp_forward<T>(g, wm, pin, n - 2, S, pacts, phase_w, s);
    phin = pacts + (long long)(L - 1) * S * h;
  }
  const int hw[2] = {2 * L, poff_phase_head(g)};
  for (int part = 0; part < 2; ++part) {
    GemmArgs a{};
    a.Mr = (int)S; a.Nc = part == 0 ? n : 4; a.K = h;
    a.A = part == 0 ? aL : phin; a.sa0 = h; a.sa1 = 1;
    a.B = wm + g.poff[hw[part]]; a.sb0 = 1; a.sb1 = h;
    a.C = hout + (part == 0 ? 0 : n); a.ldc = ld;
    a.bias = wm + g.poff[hw[part] + 1];
    gemm<T, E_FWD_LIN>(a, g, s);
  }
  hipLaunchKernelGGL(seed_kernel<T>, dim3((unsigned)((S + 255) / 256)), dim3(256), 0, s, g, x, S, eloc, w,
                     energy, hout, dh);
  // head gradients
  for (int part = 0; part < 2; ++part) {
    GemmArgs a{};
    a.Mr = part == 0 ? n : 4; a.Nc = h; a.K = (int)S;
    a.A = dh + (part == 0 ? 0 : n); a.sa0 = 1; a.sa1 = ld;
    a.B = part == 0 ? aL : phin; a.sb0 = h; a.sb1 = 1;
    a.grad = grad; a.grad_off = g.poff[hw[part]]; a.grad_ld = h;
    a.mask_kind = part == 0 ? MK_HEAD_O : (two ? MK_NONE : MK_HEAD_P);
    gemm<T, E_GRAD>(a, g, s);
    colsum<T>(dh + (part == 0 ? 0 : n), S, a.Mr, (long long)ld, grad, g.poff[hw[part] + 1], s);
  }
  // d a_L = d o (M_o W_o) [+ d p (M_p W_p) with the shared trunk]
  {
    GemmArgs a{};
    a.Mr = (int)S; a.Nc = h; a.K = n;
    a.A = dh; a.sa0 = ld; a.sa1 = 1;
    a.B = wm + g.poff[2 * L]; a.sb0 = h; a.sb1 = 1;
    a.C = da; a.ldc = h;
    gemm<T, E_STORE>(a, g, s);
    if (!two) {
      a.K = 4;
      a.A = dh + n;
      a.B = wm + g.poff[hw[1]];
      gemm<T, E_ADD>(a, g, s);
    }
  }
  mlp_backward<T>(g, wm, sb, n, S, acts, da, dz, grad, trunk_w,
                  [&](int l) { return l == 1 ? (int)MK_L1 : (int)MK_HID; }, s);
  if (two) {
    // d c_L = d p W_p, then through the phase network's dense layers
    GemmArgs a{};
    a.Mr = (int)S; a.Nc = h; a.K = 4;
    a.A = dh + n; a.sa0 = ld; a.sa1 = 1;
    a.B = wm + g.poff[hw[1]]; a.sb0 = h; a.sb1 = 1;
    a.C = da; a.ldc = h;
    gemm<T, E_STORE>(a, g, s);
    mlp_backward<T>(g, wm, pin, n - 2, S, pacts, da, dz, grad, phase_w, [&](int) { return (int)MK_NONE; }, s);
  }
}

long long backward_scratch_elems(const Geom& g, long long S) {
  long long e = S * (long long)(g.n + (long long)g.L * g.h + 2 * (g.n + 4) + 2 * g.h);
  if (g.phase_mode == 1) e += S * (long long)((g.n - 2) + (long long)g.L * g.h);
  return e;
}

void launch_backward(const Geom& g, const void* wm, const uint64_t* x, long long S,
                     const double* eloc, const double* w, const double* energy, void* scratch,
                     double* grad, hipStream_t s) {
  if (S <= 0) return;
  if (g.prec == P_F64)
    backward_t<double>(g, (const double*)wm, x, S, eloc, w, energy, (double*)scratch, grad, s);
  else
    backward_t<float>(g, (const float*)wm, x, S, eloc, w, energy, (float*)scratch, grad, s);
}

}  // namespace nqs
