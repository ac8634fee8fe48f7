// Fused masked-MLP forward on MFMA: x (uint64 bit string) -> (log|psi|, phi).
//
// One workgroup (8 or 16 waves) owns a tile of M configurations and carries them
// through every layer of the network of Sec. 4 without leaving the CU:
//   * prologue: the configuration bits are permuted into sampling order and
//     the +-1 input fragments of the first layer are generated in registers
//     (no input matrix in memory);
//   * each layer computes C^T = W A^T with MFMA, W streamed from L2 in a
//     pre-packed fragment layout (1 KB per (unit block, k step), coalesced),
//     A read from LDS, where the activations of the tile live in MFMA operand
//     order; bias + ReLU + conversion are applied on the accumulators and
//     written back in place;
//   * hidden units are sorted by MADE degree, so every mask is a prefix and
//     fully masked (block, k step) pairs are neither stored nor multiplied;
//   * the head produces the n conditional logits and the 4 phases; the
//     per-row epilogue applies the Hamming-weight modifier (Eq. modifier),
//     sums the log-sigmoids of free positions in FP64 and selects the phase.
// A model with a separate phase network runs the same kernel twice over the
// same rows: the modulus network (writes log|psi|) and the phase network
// (dense layers over the first n-2 positions, a 4-row head; writes phi).
// Arithmetic kinds: FP64 and FP32 MFMA; plain BF16; split BF16 (weights and
// activations as hi + lo BF16 planes, three products); BF16 weights with
// hi + lo activations (two products).  With two activation planes a tile
// holds half the rows of plain BF16, so every weight byte streamed from L2
// serves half as many rows: the BF16-weight kind streams one weight plane,
// split BF16 two.
#include <algorithm>
#include <atomic>

#include "net.h"

namespace nqs {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(4))) double f64x4;

template <int P> struct Tr;
// PL: planes of the activation operand, PLW: planes of the weight operand.
template <> struct Tr<P_BF16> {
  static constexpr int TB = 32, KSTEP = 16, PL = 1, PLW = 1, MH = 65536;
  using Acc = f32x16; using S = float;
  static constexpr int NACC = 16;
};
template <> struct Tr<P_BF16X3> {
  static constexpr int TB = 32, KSTEP = 16, PL = 2, PLW = 2, MH = 32768;
  using Acc = f32x16; using S = float;
  static constexpr int NACC = 16;
};
template <> struct Tr<P_BF16W> {
  static constexpr int TB = 32, KSTEP = 16, PL = 2, PLW = 1, MH = 32768;
  using Acc = f32x16; using S = float;
  static constexpr int NACC = 16;
};
template <> struct Tr<P_F32> {
  static constexpr int TB = 32, KSTEP = 8, PL = 1, PLW = 1, MH = 32768;
  using Acc = f32x16; using S = float;
  static constexpr int NACC = 16;
};
template <> struct Tr<P_F64> {
  static constexpr int TB = 16, KSTEP = 8, PL = 1, PLW = 1, MH = 16384;
  using Acc = f64x4; using S = double;
  static constexpr int NACC = 4;
};

// Configurations per workgroup: the activations of the tile fill 128 KB of
// LDS (the narrow FP64 nets use half of it so the head staging fits); MD = 2
// halves the tile (the autotuner's second tile shape: half the LDS, so two
// workgroups share a CU, at half the reuse of each weight fragment).
template <int P, int H, int MD = 1>
constexpr int rows_per_block() {
  return ((P == P_F64 && H < 256) ? 8192 / H : Tr<P>::MH / H) / MD;
}
// The half tile exists where it keeps at least one MFMA block of rows.
template <int P, int H>
constexpr bool has_half_tile() {
  return P != P_F64 && rows_per_block<P, H>() >= 2 * Tr<P>::TB;
}

// Waves per workgroup of variant 0: 16 (four per SIMD) for the wide BF16
// nets, so that every SIMD keeps two or more waves in flight until the end of
// each layer; 8 elsewhere.  Variant 1 (BF16, split BF16, FP32) takes the other
// count; the autotuner chooses between them.
template <int P, int H>
constexpr int default_waves() {
  return ((P == P_BF16 || P == P_BF16X3 || P == P_BF16W) && H >= 512) ? 16 : 8;
}
// Variant v: waves from its low bit (0: the default count, 1: the other),
// tile from its second bit (0: the full tile, 1: the half tile).
template <int P, int H, int V>
constexpr int variant_waves() {
  return (V & 1) == 0 ? default_waves<P, H>() : (default_waves<P, H>() == 16 ? 8 : 16);
}
template <int V>
constexpr int variant_md() { return (V & 2) ? 2 : 1; }

// Head k slices (one LDS staging plane each) when the head has fewer
// (block, m-block) tiles than waves: a power of two, at most 8, and no more
// than the planes that fit in 128 KB.
constexpr int pow2_floor(int v) { return v >= 8 ? 8 : v >= 4 ? 4 : v >= 2 ? 2 : 1; }
// Head outputs of the widest network a bit string of W words allows: n + 4
// with n = 64 W.
template <int W>
constexpr int head_rows_max() { return 64 * W + 4; }
template <int P, int H, int NW, int W, int MD = 1>
constexpr int head_ksplit_max() {
  constexpr int M = rows_per_block<P, H, MD>();
  constexpr int MB = M / Tr<P>::TB;
  constexpr int SP = ((head_rows_max<W>() + Tr<P>::TB - 1) / Tr<P>::TB) * Tr<P>::TB + 1;
  constexpr int fit = pow2_floor(131072 / (M * SP * (int)sizeof(typename Tr<P>::S)));
  constexpr int want = MB >= NW ? 1 : pow2_floor(NW / MB);
  return want < fit ? want : fit;
}

typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
typedef __attribute__((ext_vector_type(2))) float f32x2;

// Two FP32 values to BF16, rounded to nearest even (one v_cvt_pk_bf16_f32 on
// gfx950), packed with a in the low half.
__device__ __forceinline__ unsigned bf16x2_rne(float a, float b) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){a, b}, bf16x2));
}

// AX: the activation operand is exact in BF16 (its low plane is zero), so the
// split products need only wl*ah + wh*ah (split BF16) or wh*ah (BF16 weights).
template <int P, bool AX = false>
__device__ __forceinline__ void mma(typename Tr<P>::Acc& acc, const uint4* w, const uint4* a) {
  if constexpr (P == P_BF16) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, w[0]),
                                                  __builtin_bit_cast(bf16x8, a[0]), acc, 0, 0, 0);
  } else if constexpr (P == P_BF16X3) {
    bf16x8 wh = __builtin_bit_cast(bf16x8, w[0]), wl = __builtin_bit_cast(bf16x8, w[1]);
    bf16x8 ah = __builtin_bit_cast(bf16x8, a[0]), al = __builtin_bit_cast(bf16x8, a[1]);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wl, ah, acc, 0, 0, 0);
    if constexpr (!AX) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wh, al, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wh, ah, acc, 0, 0, 0);
  } else if constexpr (P == P_BF16W) {
    // BF16 weights times a two-term BF16 activation
    bf16x8 wh = __builtin_bit_cast(bf16x8, w[0]);
    bf16x8 ah = __builtin_bit_cast(bf16x8, a[0]), al = __builtin_bit_cast(bf16x8, a[1]);
    if constexpr (!AX) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wh, al, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wh, ah, acc, 0, 0, 0);
  } else if constexpr (P == P_F32) {
    float4 wf = __builtin_bit_cast(float4, w[0]);
    float4 af = __builtin_bit_cast(float4, a[0]);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(wf.x, af.x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(wf.y, af.y, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(wf.z, af.z, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(wf.w, af.w, acc, 0, 0, 0);
  } else {
    double2 wd = __builtin_bit_cast(double2, w[0]);
    double2 ad = __builtin_bit_cast(double2, a[0]);
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(wd.x, ad.x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(wd.y, ad.y, acc, 0, 0, 0);
  }
}

// Word of a tile row's bit string (sampling order) that holds positions
// k0 .. k0 + 7, and the position of its bit 0.  A fragment's positions never
// straddle two words (k0 is a multiple of 2, 4 or 8 and the group is as long).
template <int W>
__device__ __forceinline__ uint64_t y_word(const uint64_t* ylds, int row, int k0, int& base) {
  if constexpr (W == 1) {
    base = 0;
    return ylds[row];
  } else {
    base = k0 & ~63;
    return ylds[row * W + (k0 >> 6)];
  }
}

// +-1 input fragment of the first layer for m-block mb, k step ks.
// Element (row m, k) is +1/-1 for occupied/empty position k < n, 0 beyond.
template <int P, int W>
__device__ __forceinline__ void input_frag(const uint64_t* ylds, int mb, int ks, int lane, int n,
                                           uint4* out) {
  using T = Tr<P>;
  int base;
  if constexpr (P == P_BF16 || P == P_BF16X3 || P == P_BF16W) {
    int k0 = ks * 16 + 8 * (lane >> 5);
    uint64_t y = y_word<W>(ylds, mb * 32 + (lane & 31), k0, base);
    unsigned short v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      int k = k0 + j;
      v[j] = k < n ? (((y >> (k - base)) & 1ull) ? (unsigned short)0x3F80 : (unsigned short)0xBF80)
                   : (unsigned short)0;
    }
    out[0] = make_uint4(v[0] | (v[1] << 16), v[2] | (v[3] << 16), v[4] | (v[5] << 16),
                        v[6] | (v[7] << 16));
    if constexpr (T::PL == 2) out[1] = make_uint4(0, 0, 0, 0);
  } else if constexpr (P == P_F32) {
    int k0 = ks * 8 + 4 * (lane >> 5);
    uint64_t y = y_word<W>(ylds, mb * 32 + (lane & 31), k0, base);
    float v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int k = k0 + j;
      v[j] = k < n ? (((y >> (k - base)) & 1ull) ? 1.f : -1.f) : 0.f;
    }
    out[0] = __builtin_bit_cast(uint4, make_float4(v[0], v[1], v[2], v[3]));
  } else {
    int k0 = ks * 8 + 2 * (lane >> 4);
    uint64_t y = y_word<W>(ylds, mb * 16 + (lane & 15), k0, base);
    double v[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      int k = k0 + j;
      v[j] = k < n ? (((y >> (k - base)) & 1ull) ? 1.0 : -1.0) : 0.0;
    }
    out[0] = __builtin_bit_cast(uint4, make_double2(v[0], v[1]));
  }
}

// Write relu(acc + bias) of tile (nb, mb) into the LDS activations, in the
// operand order of the next layer.
template <int P, int MB>
__device__ __forceinline__ void store_act(char* act, const typename Tr<P>::Acc& acc,
                                          const typename Tr<P>::S* bias, int nb, int mb, int lane,
                                          int KSH) {
  using T = Tr<P>;
  if constexpr (P == P_F64) {
    // 16x16x4 f64 accumulator: lane l, register rr holds row (l/16) + 4 rr, column l%16.
    const int m = lane & 15, g = lane >> 4;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int nl = g + 4 * rr;                 // unit inside the 16-block
      double t = acc[rr] + bias[16 * nb + nl];
      t = t > 0.0 ? t : 0.0;
      const int ks = 2 * nb + (nl >> 3);
      const int kk = nl & 7;                     // k inside the 8-wide step
      const int lp = m + 16 * (kk >> 1);
      *(double*)(act + ((long)(ks * MB + mb) * 64 + lp) * 16 + 8 * (kk & 1)) = t;
    }
  } else {
    const int m = lane & 31, hf = lane >> 5;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int n0 = 32 * nb + 8 * q + 4 * hf;
      const float4 b4 = *(const float4*)(bias + n0);
      float v0 = acc[4 * q + 0] + b4.x, v1 = acc[4 * q + 1] + b4.y;
      float v2 = acc[4 * q + 2] + b4.z, v3 = acc[4 * q + 3] + b4.w;
      v0 = v0 > 0.f ? v0 : 0.f; v1 = v1 > 0.f ? v1 : 0.f;
      v2 = v2 > 0.f ? v2 : 0.f; v3 = v3 > 0.f ? v3 : 0.f;
      if constexpr (P == P_F32) {
        const int ks = 4 * nb + q;
        const int lp = m + 32 * hf;
        *(float4*)(act + ((long)(ks * MB + mb) * 64 + lp) * 16) = make_float4(v0, v1, v2, v3);
      } else {
        const int ks = 2 * nb + (q >> 1);
        const int lp = m + 32 * (q & 1);
        const unsigned h01 = bf16x2_rne(v0, v1), h23 = bf16x2_rne(v2, v3);
        char* dst = act + ((long)(ks * MB + mb) * 64 + lp) * 16 + 8 * hf;
        *(uint2*)dst = make_uint2(h01, h23);
        if constexpr (T::PL == 2) {
          // low term: the exact residual v - hi (Sterbenz), rounded to BF16
          const float r0 = v0 - __uint_as_float(h01 << 16), r1 = v1 - __uint_as_float(h01 & 0xFFFF0000u);
          const float r2 = v2 - __uint_as_float(h23 << 16), r3 = v3 - __uint_as_float(h23 & 0xFFFF0000u);
          char* dlo = dst + (long)KSH * MB * 64 * 16;
          *(uint2*)dlo = make_uint2(bf16x2_rne(r0, r1), bf16x2_rne(r2, r3));
        }
      }
    }
  }
}

// K loop of one layer for the wave's NBW n-blocks and MBW m-blocks.  Weight
// fragments are double-buffered in registers and requested two k steps
// before use; blocks whose (masked) k range has ended are skipped.
// act(j, ks, frag) supplies the activation fragment of m-block j.
// Loads are unconditional (the k index is clamped into the block's range, a
// cache hit) so the compiler can count outstanding loads exactly; only the
// MFMAs of finished blocks are skipped, on a wave-uniform scalar branch.
//
// Every block's k extent is even and the extents ascend with the block index
// inside a wave, so the loop runs in phases with a compile-time set of active
// blocks {I0..NBW-1}: no branches in the steady state, static register
// double-buffering, and exact load accounting by the compiler.
//
// Weight fragments are read with raw buffer loads: a scalar byte offset per
// (block, k step), one VGPR for the lane offset, and hardware range checking
// against the packed buffer.  Scheduling fences keep the compiler from
// pulling the next loads' consumers up next to them.
struct WBuf {
  __amdgpu_buffer_rsrc_t rsrc;
  int plane_bytes;   // offset of the second (low) bf16 plane
  int voff;          // lane * 16
};

__device__ __forceinline__ uint4 wload(const WBuf& b, int soff) {
  return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(b.rsrc, b.voff, soff, 0));
}

// With PF, activation fragments are double-buffered too: the fragments of
// step k+1 are requested before the MFMAs of step k, so the LDS latency is
// covered by those MFMAs; afa holds step ks on entry (and on exit).  Without
// PF (shapes whose registers would not hold the second buffer) each step
// reads its fragments right before its MFMAs.
template <int P, int NBW, int MBW, int I0, bool AX, bool PF, class ActFn>
__device__ __forceinline__ void kphase(typename Tr<P>::Acc (&acc)[NBW][MBW], const WBuf& wb_,
                                       const int (&wbase)[NBW], const int (&kend)[NBW], int ks,
                                       uint4 (&wa)[NBW][Tr<P>::PLW], uint4 (&wb)[NBW][Tr<P>::PLW],
                                       uint4 (&afa)[MBW][Tr<P>::PL], uint4 (&afb)[MBW][Tr<P>::PL],
                                       ActFn& act) {
  constexpr int PL = Tr<P>::PL, PLW = Tr<P>::PLW;
  auto loadw = [&](uint4 (&w)[NBW][PLW], int k) {
#pragma unroll
    for (int i = I0; i < NBW; ++i) {
      const int kc = max(0, k < kend[i] ? k : kend[i] - 1);   // clamped into the block
      const int so = wbase[i] + kc * 1024;
      w[i][0] = wload(wb_, so);
      if constexpr (PLW == 2) w[i][1] = wload(wb_, so + wb_.plane_bytes);
    }
  };
  // the last block's extent bounds every k this wave reads
  const int klast = kend[NBW - 1] - 1;
  auto rd = [&](uint4 (&af)[MBW][PL], int k) {
    const int kc = k < klast ? k : klast;
#pragma unroll
    for (int j = 0; j < MBW; ++j) act(j, kc, af[j]);
  };
  auto mm = [&](uint4 (&w)[NBW][PLW], uint4 (&af)[MBW][PL]) {
#pragma unroll
    for (int i = I0; i < NBW; ++i)
#pragma unroll
      for (int j = 0; j < MBW; ++j) mma<P, AX>(acc[i][j], w[i], af[j]);
  };
  const int stop = kend[I0];
  auto body = [&]() {
    if constexpr (PF) rd(afb, ks + 1);
    else rd(afa, ks);
    mm(wa, afa);
    __builtin_amdgcn_sched_barrier(0);
    loadw(wa, ks + 2);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (PF) {
      rd(afa, ks + 2);
      mm(wb, afb);
    } else {
      rd(afa, ks + 1);
      mm(wb, afa);
    }
    __builtin_amdgcn_sched_barrier(0);
    loadw(wb, ks + 3);
    __builtin_amdgcn_sched_barrier(0);
    ks += 2;
  };
  if constexpr (I0 == 0) {
    // the caller guarantees ks < kend[0]: a do-while keeps the preloads of
    // every block in front of the loop instead of sunk behind an entry test
    do { body(); } while (ks < stop);
  } else {
    while (ks < stop) body();
  }
  if constexpr (I0 + 1 < NBW) kphase<P, NBW, MBW, I0 + 1, AX, PF>(acc, wb_, wbase, kend, ks, wa, wb, afa, afb, act);
}

// Whether the second activation buffer fits the register budget of a wave
// (128 VGPRs at 16 waves per workgroup, 256 at 8): accumulators, two weight
// buffers, two activation buffers and addressing.
template <int P, int NBW, int MBW, int NW>
constexpr bool act_prefetch() {
  constexpr int acc = P == P_F64 ? 8 : 16;
  constexpr int PL = Tr<P>::PL, PLW = Tr<P>::PLW;
  return acc * NBW * MBW + 8 * PLW * NBW + 8 * PL * MBW + 40 + 4 * MBW <= 2048 / NW;
}

// The first two k steps' weight fragments of a layer, requested ahead of
// the k loop (before the barrier that precedes the layer, so their L2
// latency overlaps the barrier wait).  Loads are clamped into each block's
// range (a block without fragments reads a neighbour's, never used).
template <int P, int NBW>
struct WPre {
  uint4 wa[NBW][Tr<P>::PLW], wb[NBW][Tr<P>::PLW];
  int kend[NBW], wbase[NBW];
};

template <int P, int NBW>
__device__ __forceinline__ void kloop_pre(WPre<P, NBW>& pre, const WBuf& wbuf, const int (&fragi)[NBW],
                                          const int (&ksi)[NBW]) {
  constexpr int PLW = Tr<P>::PLW;
#pragma unroll
  for (int i = 0; i < NBW; ++i) {
    pre.kend[i] = __builtin_amdgcn_readfirstlane(ksi[i]);
    pre.wbase[i] = __builtin_amdgcn_readfirstlane(fragi[i] * 1024);
  }
  // same issue order as the loop body (all of wa, then all of wb) so the
  // outstanding-load state is identical on loop entry and on the back edge
#pragma unroll
  for (int i = 0; i < NBW; ++i) {
    const int k0 = max(0, 0 < pre.kend[i] ? 0 : pre.kend[i] - 1);
    pre.wa[i][0] = wload(wbuf, pre.wbase[i] + k0 * 1024);
    if constexpr (PLW == 2) pre.wa[i][1] = wload(wbuf, pre.wbase[i] + k0 * 1024 + wbuf.plane_bytes);
  }
#pragma unroll
  for (int i = 0; i < NBW; ++i) {
    const int k1 = max(0, 1 < pre.kend[i] ? 1 : pre.kend[i] - 1);
    pre.wb[i][0] = wload(wbuf, pre.wbase[i] + k1 * 1024);
    if constexpr (PLW == 2) pre.wb[i][1] = wload(wbuf, pre.wbase[i] + k1 * 1024 + wbuf.plane_bytes);
  }
}

// K loop of one layer from k step 0, its first fragments already requested
// by kloop_pre.
template <int P, int NBW, int MBW, int NW, bool AX, class ActFn>
__device__ __forceinline__ void kloop(typename Tr<P>::Acc (&acc)[NBW][MBW], const WBuf& wbuf,
                                      WPre<P, NBW>& pre, ActFn act) {
  constexpr int PL = Tr<P>::PL;
  // every block has at least two k steps and the extents ascend, so after
  // this test phase 0 (all blocks active) is non-empty
  if (pre.kend[NBW - 1] <= 0 || pre.kend[0] <= 0) return;
  constexpr bool PF = act_prefetch<P, NBW, MBW, NW>();
  uint4 afa[MBW][PL], afb[MBW][PL];
  if constexpr (PF) {
#pragma unroll
    for (int j = 0; j < MBW; ++j) act(j, 0, afa[j]);
  }
  __builtin_amdgcn_sched_barrier(0);
  kphase<P, NBW, MBW, 0, AX, PF>(acc, wbuf, pre.wbase, pre.kend, 0, pre.wa, pre.wb, afa, afb, act);
}

// Head k loop for one (block, m-block) tile over [k0, k1) (multiples of 8):
// eight weight fragments are requested back to back, then consumed in order,
// so the load latency is paid once per eight MFMA steps.
template <int P, class ActFn>
__device__ __forceinline__ void head_loop(typename Tr<P>::Acc& acc, const WBuf& wbuf, int frag0,
                                          int k0, int k1, ActFn act) {
  constexpr int PL = Tr<P>::PL, PLW = Tr<P>::PLW;
  constexpr int D = 8;
  const int base = __builtin_amdgcn_readfirstlane(frag0 * 1024);
  k0 = __builtin_amdgcn_readfirstlane(k0);
  k1 = __builtin_amdgcn_readfirstlane(k1);
  for (int k = k0; k < k1; k += D) {
    uint4 w[D][PLW];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      w[d][0] = wload(wbuf, base + (k + d) * 1024);
      if constexpr (PLW == 2) w[d][1] = wload(wbuf, base + (k + d) * 1024 + wbuf.plane_bytes);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int d = 0; d < D; ++d) {
      uint4 af[PL];
      act(k + d, af);
      mma<P>(acc, w[d], af);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <typename S>
__device__ __forceinline__ S softplus(S z) {
  S a = z > S(0) ? z : -z;
  S m = z > S(0) ? z : S(0);
  if constexpr (sizeof(S) == 4) return m + log1pf(expf(-a));
  else return m + log1p(exp(-a));
}

// Shape constants of one (precision, width, waves, tile) instance of the kernel.
template <int P, int H, int NW_, int W = 1, int MD = 1>
struct Shape {
  using T = Tr<P>;
  using S = typename T::S;
  static constexpr int NW = NW_, NT = 64 * NW;
  static constexpr int TB = T::TB, PL = T::PL;
  static constexpr int M = rows_per_block<P, H, MD>();
  static constexpr int NB = H / TB, MB = M / TB;
  static constexpr int WN = NB < NW ? NB : NW, WM = NW / WN;
  static constexpr int NBW = NB / WN, MBW = MB / WM;
  static constexpr int KSH = H / T::KSTEP;
  static constexpr int NHBMAX = (head_rows_max<W>() + TB - 1) / TB;
  static constexpr int HP = (NHBMAX * MB + NW - 1) / NW;
  static constexpr int SP = NHBMAX * TB + 1;
  static constexpr int KSPLIT_MAX = head_ksplit_max<P, H, NW, W, MD>();
  static constexpr long ACT_BYTES = (long)PL * KSH * MB * 1024;
  static constexpr long STAGE_BYTES = (long)M * SP * sizeof(S) * KSPLIT_MAX;
  static constexpr long REGION = ACT_BYTES > STAGE_BYTES ? ACT_BYTES : STAGE_BYTES;
  // LDS: activations / head staging, then the tile's bit strings (W words
  // each, in sampling order), then the bias being applied
  static constexpr long Y_OFF = REGION;
  static constexpr long B_OFF = Y_OFF + (long)M * 8 * W;
  static constexpr long LDS = B_OFF + (long)(H + NHBMAX * TB) * sizeof(S);
  static constexpr bool FITS = LDS <= 160 * 1024;
  static_assert(MB % WM == 0 && NB % WN == 0 && MB >= 1, "tile shape");
  // one-word shapes always fit; a two-word shape whose head staging does
  // not fit (256-row tiles) is reported unsupported instead
  static_assert(W == 2 || FITS, "LDS budget");
};

// Ones among positions p < t (popc_below2) and p > t (popc_above2) of a
// two-word string (a0: positions 0..63, a1: positions 64..127), 0 <= t < 128.
__device__ __forceinline__ int popc_below2(uint64_t a0, uint64_t a1, int t) {
  if (t <= 64) return t == 0 ? 0 : __popcll(a0 & (~0ull >> (64 - t)));
  return __popcll(a0) + __popcll(a1 & (~0ull >> (128 - t)));
}
__device__ __forceinline__ int popc_above2(uint64_t a0, uint64_t a1, int t) {
  if (t >= 64) return t >= 127 ? 0 : __popcll(a1 & (~0ull << (t - 63)));
  return (t >= 63 ? 0 : __popcll(a0 & (~0ull << (t + 1)))) + __popcll(a1);
}

// Rows [row0, row0 + M) of one batch through the whole network; rows at or
// beyond count are computed on a copy of row0 and not written.
template <int P, int H, int NW, int W, int MD>
__device__ __forceinline__ void fwd_tile(const Geom& g, const uint4* __restrict__ wpk,
                                         const uint64_t* __restrict__ xs, long long row0, long long count,
                                         double2* __restrict__ out, char* act, int cond) {
  using Sh = Shape<P, H, NW, W, MD>;
  using T = Tr<P>;
  using Acc = typename T::Acc;
  using S = typename T::S;
  constexpr int TB = Sh::TB, PL = Sh::PL, NT = Sh::NT, M = Sh::M;
  constexpr int NB = Sh::NB, MB = Sh::MB, WN = Sh::WN, WM = Sh::WM, NBW = Sh::NBW, MBW = Sh::MBW;
  constexpr int KSH = Sh::KSH, HP = Sh::HP, SP = Sh::SP, KSPLIT_MAX = Sh::KSPLIT_MAX;
  uint64_t* ylds = (uint64_t*)(act + Sh::Y_OFF);
  // bias of the layer being finished (H entries), then of the head
  S* blds = (S*)(act + Sh::B_OFF);
  S* stage = (S*)act;
  constexpr int BPT = (H + NT - 1) / NT;   // bias entries staged per thread

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform
  const int wn = wave % WN, wm = wave / WN;

  const S* biases = (const S*)((const char*)wpk + g.bias_byte);
  WBuf wbuf;
  wbuf.rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)wpk, (short)0, (int)g.bias_byte, 0x00020000);
  wbuf.plane_bytes = (int)(g.nfrag * 1024);
  wbuf.voff = lane * 16;

  static_assert(M <= NT, "one configuration per thread");
  // n-blocks of this wave.  The masked k extent grows with the block index,
  // so blocks are dealt in mirrored pairs (p, NB-1-p): every wave then runs
  // the same number of k steps and all waves of a SIMD stay busy until the
  // end of the layer.  Inside a wave the blocks are listed in ascending
  // order, the order in which the k loop retires them.  With one block per
  // wave, the blocks are dealt over the SIMDs in a snake instead (waves s,
  // s+4, s+8, s+12 share SIMD s), which balances the SIMDs.
  int nbl[NBW], mbl[MBW];
  if constexpr (NBW % 2 == 0) {
#pragma unroll
    for (int r = 0; r < NBW / 2; ++r) {
      const int p = wn + WN * r;
      nbl[r] = p;
      nbl[NBW - 1 - r] = NB - 1 - p;
    }
  } else {
    const int grp = (WN == NW) ? (((wave >> 2) & 1) ? (wave & ~3) + 3 - (wave & 3) : wave) : wn;
#pragma unroll
    for (int i = 0; i < NBW; ++i) nbl[i] = grp * NBW + i;
  }
#pragma unroll
  for (int j = 0; j < MBW; ++j) mbl[j] = j * WM + wm;

  // fragments of a layer's first k steps: 1 = layer 1, 2..L = hidden layers.
  // They are requested before the barrier that ends the previous layer,
  // except where four accumulator tiles per wave leave no registers for them
  // during the epilogue.
  constexpr bool EARLY = !(P == P_BF16 && MBW >= 4);
  WPre<P, NBW> pre;
  auto preload = [&](int l) {
    int ksi[NBW], fragi[NBW];
    const int lbase = l == 1 ? 0 : (int)(g.frag_h + (long long)(l - 2) * g.offh[NB]);
#pragma unroll
    for (int i = 0; i < NBW; ++i) {
      ksi[i] = l == 1 ? g.ks1[nbl[i]] : g.ksh[nbl[i]];
      fragi[i] = l == 1 ? g.off1[nbl[i]] : lbase + g.offh[nbl[i]];
    }
    kloop_pre<P, NBW>(pre, wbuf, fragi, ksi);
  };

  if constexpr (W == 1) {
    uint64_t x = 0;
    if (tid < M) {
      const long long row = row0 + tid;
      x = xs[row < count ? row : row0];
    }
    if (EARLY) preload(1);   // overlaps the configuration load
    if (tid < M) {
      // bits into sampling order: y bit p = x bit order[p]
      uint64_t y;
      if (g.order_kind == 2) {
        y = __builtin_bitreverse64(x) >> (64 - g.n);
      } else if (g.order_kind == 1) {
        y = x;
      } else {
        // unrolled with constant indices, so the order bytes are scalar loads
        y = 0;
#pragma unroll
        for (int p = 0; p < 64; ++p)
          if (p < g.n) y |= ((x >> g.order[p]) & 1ull) << p;
      }
      ylds[tid] = y;
    }
  } else {
    // two words: word w holds qubits (positions) 64w .. 64w+63
    uint64_t x0 = 0, x1 = 0;
    if (tid < M) {
      const long long row = row0 + tid;
      const long long r = row < count ? row : row0;
      x0 = xs[2 * r];
      x1 = xs[2 * r + 1];
    }
    if (EARLY) preload(1);
    if (tid < M) {
      uint64_t y0, y1;
      if (g.order_kind == 2) {
        // reverse the 128-bit string, then drop the 128 - n empty positions
        const uint64_t r0 = __builtin_bitreverse64(x1), r1 = __builtin_bitreverse64(x0);
        const int sh = 128 - g.n;   // 0 .. 63
        y0 = sh == 0 ? r0 : ((r0 >> sh) | (r1 << (64 - sh)));
        y1 = r1 >> sh;
      } else if (g.order_kind == 1) {
        y0 = x0;
        y1 = x1;
      } else {
        y0 = 0;
        y1 = 0;
#pragma unroll
        for (int p = 0; p < 2 * 64; ++p)
          if (p < g.n) {
            const int q = g.order[p];
            const uint64_t b = ((q < 64 ? x0 : x1) >> (q & 63)) & 1ull;
            if (p < 64) y0 |= b << p;
            else y1 |= b << (p - 64);
          }
      }
      ylds[2 * tid] = y0;
      ylds[2 * tid + 1] = y1;
    }
  }
  for (int t = tid; t < H; t += NT) blds[t] = biases[t];
  __syncthreads();
  if (!EARLY) preload(1);

  Acc acc[NBW][MBW];
  auto lds_act = [&](int j, int ks, uint4 (&f)[PL]) {
    const uint4* a = (const uint4*)act + ((long)(ks * MB + mbl[j])) * 64 + lane;
    f[0] = a[0];
    if constexpr (PL == 2) f[1] = a[(long)KSH * MB * 64];
  };

  // ---------------------------------------------------------------- layer 1
  {
#pragma unroll
    for (int i = 0; i < NBW; ++i)
#pragma unroll
      for (int j = 0; j < MBW; ++j) acc[i][j] = Acc{};
    // the +-1 inputs are exact in BF16
    kloop<P, NBW, MBW, Sh::NW, true>(acc, wbuf, pre,
                                     [&](int j, int ks, uint4 (&f)[PL]) { input_frag<P, W>(ylds, mbl[j], ks, lane, g.n, f); });
#pragma unroll
    for (int i = 0; i < NBW; ++i)
#pragma unroll
      for (int j = 0; j < MBW; ++j) store_act<P, MB>(act, acc[i][j], blds, nbl[i], mbl[j], lane, KSH);
    if (EARLY && g.L >= 2) preload(2);
    __syncthreads();
    if (!EARLY && g.L >= 2) preload(2);
  }

  // ----------------------------------------------------------- hidden layers
  for (int l = 2; l <= g.L; ++l) {
#pragma unroll
    for (int i = 0; i < NBW; ++i)
#pragma unroll
      for (int j = 0; j < MBW; ++j) acc[i][j] = Acc{};
    // this layer's bias is requested before the k loop and parked in LDS
    // after it, so the epilogue reads it without waiting on L2
    S breg[BPT];
    const S* bsrc = biases + (long)(l - 1) * H;
#pragma unroll
    for (int e = 0; e < BPT; ++e) breg[e] = (tid + e * NT < H) ? bsrc[tid + e * NT] : S(0);
    kloop<P, NBW, MBW, Sh::NW, false>(acc, wbuf, pre, lds_act);
#pragma unroll
    for (int e = 0; e < BPT; ++e)
      if (tid + e * NT < H) blds[tid + e * NT] = breg[e];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NBW; ++i)
#pragma unroll
      for (int j = 0; j < MBW; ++j) store_act<P, MB>(act, acc[i][j], blds, nbl[i], mbl[j], lane, KSH);
    if (EARLY && l < g.L) preload(l + 1);
    __syncthreads();
    if (!EARLY && l < g.L) preload(l + 1);
  }

  // -------------------------------------------------------------------- head
  // Work items (head n-block, m-block, k slice) are spread over all waves;
  // k slices of one tile are summed from their staging planes in the epilogue.
  Acc hacc[HP];
  const int nho = g.net_kind == 2 ? 4 : g.n + 4;   // head outputs: n conditionals, 4 phases
  S hbreg = tid < nho ? biases[(long)g.L * H + tid] : S(0);
  const int npairs = g.NHB * MB;
  const int ksplit = npairs >= NW ? 1 : min(KSPLIT_MAX, NW / npairs);
  const int nitems = npairs * ksplit;
#pragma unroll
  for (int hp = 0; hp < HP; ++hp) {
    hacc[hp] = Acc{};
    const int item = wave + NW * hp;
    if (item < nitems) {
      const int pr = item / ksplit, part = item % ksplit;
      const int nb = pr / MB, mb = pr % MB;
      const int kso = g.kso[nb];
      const int chunk = (((kso + ksplit - 1) / ksplit) + 7) & ~7;   // head extents are multiples of 8
      const int k0 = part * chunk, k1 = min(kso, k0 + chunk);
      head_loop<P>(hacc[hp], wbuf, (int)(g.frag_head + g.offo[nb]), k0, k1, [&](int ks, uint4 (&f)[PL]) {
        const uint4* a = (const uint4*)act + ((long)(ks * MB + mb)) * 64 + lane;
        f[0] = a[0];
        if constexpr (PL == 2) f[1] = a[(long)KSH * MB * 64];
      });
    }
  }
  if (tid < nho) blds[tid] = hbreg;
  __syncthreads();
  // each k slice writes its own staging plane; the epilogue adds the planes
  // in a fixed order, so the result does not depend on wave scheduling
#pragma unroll
  for (int hp = 0; hp < HP; ++hp) {
    const int item = wave + NW * hp;
    if (item < nitems) {
      const int pr = item / ksplit, part = item % ksplit;
      const int nb = pr / MB, mb = pr % MB;
      S* plane = stage + (long)part * M * SP;
      if constexpr (P == P_F64) {
        const int m = mb * 16 + (lane & 15), gq = lane >> 4;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) plane[m * SP + nb * 16 + gq + 4 * rr] = hacc[hp][rr];
      } else {
        const int m = mb * 32 + (lane & 31), hf = lane >> 5;
#pragma unroll
        for (int r = 0; r < 16; ++r) plane[m * SP + nb * 32 + 8 * (r >> 2) + 4 * hf + (r & 3)] = hacc[hp][r];
      }
    }
  }
  __syncthreads();

  // ------------------------------------------------------------ row epilogue
  constexpr int TPR = NT / M >= 1 ? NT / M : 1;
  const int row = tid / TPR, sub = tid % TPR;
  if (row < M) {
    const S* hb = blds;
    const uint64_t y = ylds[row * W];
    const uint64_t yh = W == 2 ? ylds[row * W + 1] : 0ull;   // positions 64..127
    const bool constrained = g.n_up >= 0 && g.n_dn >= 0;
    auto head_out = [&](int col) {
      S v = stage[row * SP + col];
      for (int p = 1; p < ksplit; ++p) v += stage[((long)p * M + row) * SP + col];
      return v + hb[col];
    };
    double sum = 0.0;
    int bad = 0;
    const uint64_t sp0 = g.spin_pos[0], sp1 = g.spin_pos[1];
    const uint64_t sp0h = W == 2 ? g.spin_pos_hi[0] : 0ull, sp1h = W == 2 ? g.spin_pos_hi[1] : 0ull;
    // bit of position t, and the spin of the qubit there
    auto ybit = [&](int t) -> int {
      if constexpr (W == 1) return (int)((y >> t) & 1ull);
      else return (int)(((t < 64 ? y : yh) >> (t & 63)) & 1ull);
    };
    auto spin = [&](int t) -> int {
      if constexpr (W == 1) return (int)((sp1 >> t) & 1ull);
      else return (int)(((t < 64 ? sp1 : sp1h) >> (t & 63)) & 1ull);
    };
    // c = ones among the earlier positions of spin sp, rem = later positions of spin sp
    auto spin_counts = [&](int t, int sp, int& c, int& rem) {
      const uint64_t spm = sp ? sp1 : sp0;
      if constexpr (W == 1) {
        const uint64_t low = t == 0 ? 0ull : (~0ull >> (64 - t));
        const uint64_t high = t >= 63 ? 0ull : (~0ull << (t + 1));
        c = __popcll(y & spm & low);
        rem = __popcll(spm & high);
      } else {
        const uint64_t spmh = sp ? sp1h : sp0h;
        c = popc_below2(y & spm, yh & spmh, t);
        rem = popc_above2(spm, spmh, t);
      }
    };
    const long long grow = row0 + row;
    if (g.net_kind == 2) {
      // separate phase network: the phase of the completion of the last two positions
      if (sub == 0 && grow < count) {
        const int sel = 2 * ybit(g.n - 2) + ybit(g.n - 1);
        ((double*)out)[2 * grow + 1] = (double)head_out(sel);
      }
      return;
    }
    if (cond >= 0) {
      // sampler: the conditional logit at position cond and its forcing,
      // from the bits before it (later bits do not enter)
      if (sub == 0 && grow < count) {
        const int t = cond;
        int code = 0;
        if (constrained) {
          const int sp = spin(t);
          int c, rem;
          spin_counts(t, sp, c, rem);
          const int ns = sp ? g.n_dn : g.n_up;
          code = (c + rem < ns) ? 2 : (c >= ns ? 1 : 0);
        }
        out[grow] = make_double2((double)head_out(t), (double)code);
      }
      return;
    }
    for (int t = sub; t < g.n; t += TPR) {
      const S o = head_out(t);
      const int sp = spin(t);   // spin of the qubit at position t
      const int bit = ybit(t);
      bool fr = true;
      if (constrained) {
        int c, rem;
        spin_counts(t, sp, c, rem);
        const int ns = sp ? g.n_dn : g.n_up;
        const bool f0 = c >= ns, f1 = c + rem < ns;
        bad |= (f0 && bit) || (f1 && !bit);
        fr = !(f0 || f1);
      }
      if (fr) sum -= (double)softplus<S>(bit ? -o : o);
    }
#pragma unroll
    for (int off = TPR / 2; off >= 1; off >>= 1) {
      sum += __shfl_xor(sum, off);
      bad |= __shfl_xor(bad, off);
    }
    if (sub == 0 && grow < count) {
      const double la = bad ? -INFINITY : 0.5 * sum;
      if (g.net_kind == 1) {
        // modulus network of a two-network model: the phase network writes phi
        ((double*)out)[2 * grow] = la;
      } else {
        const int sel = 2 * ybit(g.n - 2) + ybit(g.n - 1);
        out[grow] = make_double2(la, (double)head_out(g.n + sel));
      }
    }
  }
}

template <typename Seg>
__device__ __forceinline__ long long seg_rows(const Seg& sg) {
  long long rows = sg.rows_bound;
  if (sg.d_count) {
    const long long c = *sg.d_count;
    rows = c < rows ? c : rows;
  }
  return rows;
}

// Tiles of M rows.  Workgroup b takes tiles tile_base + b, then + tile_stride,
// ... below ntiles: one tile each when the grid covers every tile
// (tile_stride = ntiles), several when only a resident grid is launched.
// Tiles past a segment's device-side row count are skipped (a single segment
// ends its loop there).  Consecutive tiles of one workgroup are separated by
// a barrier: the previous tile's epilogue reads the LDS the next prologue
// writes.
// MULTI = false: one segment, geometry in the kernel arguments.
// MULTI = true: up to kMaxSeg segments (a work list of tiles from several
// networks); a tile's segment is found from the tile index and its geometry
// read from the segment's device copy.
// W: 64-bit words per bit string (2 only with MULTI = false).
template <int P, int H, int NW, bool MULTI, int W, int MD>
__global__ __launch_bounds__(64 * NW) void fused_forward(Geom g0, FwdLaunch la) {
  using Sh = Shape<P, H, NW, W, MD>;
  constexpr int M = Sh::M;
  extern __shared__ uint4 smem[];
  char* act = (char*)smem;
  bool again = false;
  for (long long t = la.tile_base + blockIdx.x; t < la.ntiles; t += la.tile_stride) {
    if constexpr (!MULTI) {
      const FwdSeg& sg = la.seg[0];
      const long long rows = seg_rows(sg);
      if (t * M >= rows) break;
      if (again) __syncthreads();
      fwd_tile<P, H, NW, W, MD>(g0, (const uint4*)sg.packed, sg.x, t * M, rows, (double2*)sg.out, act, la.cond_pos);
      again = true;
    } else {
      static_assert(W == 1, "multi-segment launches take one-word bit strings");
      int k = 0;
      for (int j = 1; j < la.nseg; ++j)
        if (t >= la.seg[j].tile0) k = j;
      const FwdSeg& sg = la.seg[k];
      const long long rows = seg_rows(sg);
      const long long row0 = (t - sg.tile0) * M;
      // the geometry is read in place: nothing in this kernel writes global
      // memory before the tile's outputs, so its loads stay scalar
      if (row0 < rows) {
        if (again) __syncthreads();
        fwd_tile<P, H, NW, W, MD>(*sg.geom, (const uint4*)sg.packed, sg.x, row0, rows, (double2*)sg.out, act,
                              la.cond_pos);
        again = true;
      }
    }
  }
  if (blockIdx.x == 0 && la.tile_base == 0 && threadIdx.x == 0) {
    for (int k = 0; k < la.nseg; ++k)
      if (la.seg[k].prof_slot) *la.seg[k].prof_slot = seg_rows(la.seg[k]);
  }
}

__global__ void store_geom_kernel(Geom g, Geom* dst) {
  const int* src = (const int*)&g;
  for (int i = threadIdx.x; i < (int)(sizeof(Geom) / 4); i += blockDim.x) ((int*)dst)[i] = src[i];
}

void launch_store_geom(const Geom& g, Geom* dst, hipStream_t s) {
  static_assert(sizeof(Geom) % 4 == 0, "Geom is copied in 32-bit words");
  hipLaunchKernelGGL(store_geom_kernel, dim3(1), dim3(256), 0, s, g, dst);
}

template <int P, int H, int V, bool MULTI, int W>
static void launch_one(const Geom& g, FwdLaunch& la, bool resident, int cu_count, hipStream_t s) {
  constexpr int NW = variant_waves<P, H, V>();
  constexpr int MD = variant_md<V>();
  using Sh = Shape<P, H, NW, W, MD>;
  if constexpr (!Sh::FITS) {
    return;   // forward_supported() rejects this shape before any launch
  } else {
  constexpr size_t LDS = Sh::LDS;
  auto kern = fused_forward<P, H, NW, MULTI, W, MD>;
  // the LDS opt-in, once per device (one bit per device ordinal), safe across threads
  static std::atomic<unsigned long long> attr_done{0};
  int dev = 0;
  (void)hipGetDevice(&dev);
  const unsigned long long bit = 1ull << (dev & 63);
  if (!(attr_done.load(std::memory_order_acquire) & bit)) {
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS);
    attr_done.fetch_or(bit, std::memory_order_release);
  }
  long long tiles = 0;
  for (int k = 0; k < la.nseg; ++k) {
    la.seg[k].tile0 = tiles;
    tiles += (la.seg[k].rows_bound + Sh::M - 1) / Sh::M;
  }
  la.ntiles = tiles;
  if (tiles <= 0) return;
  if (resident) {
    // workgroups that fit on the device at once (per device ordinal, queried once)
    static std::atomic<int> per_cu[64];
    int occ = per_cu[dev & 63].load(std::memory_order_acquire);
    if (occ <= 0) {
      int n = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void*)kern, 64 * NW, LDS) != hipSuccess || n < 1)
        n = 1;
      occ = n;
      per_cu[dev & 63].store(occ, std::memory_order_release);
    }
    const long long grid = std::min<long long>(tiles, (long long)std::max(cu_count, 1) * occ);
    la.tile_base = 0;
    la.tile_stride = grid;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(64 * NW), LDS, s, g, la);
    return;
  }
  // a dispatch counts its work-items in 32 bits: larger launches are split
  la.tile_stride = tiles;
  const long long max_tiles = 0xFFFFFFFFLL / (64 * NW);
  for (long long t0 = 0; t0 < tiles; t0 += max_tiles) {
    la.tile_base = t0;
    const long long nb = std::min(max_tiles, tiles - t0);
    hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(64 * NW), LDS, s, g, la);
  }
  }
}

int forward_rows_per_block(int prec, int h) {
  switch (prec) {
    case P_BF16: return 65536 / h;
    case P_BF16X3: case P_BF16W: return 32768 / h;
    case P_F32: return 32768 / h;
    default: return h < 256 ? 8192 / h : 16384 / h;
  }
}

template <int P, int H>
static constexpr bool fits_two_words() {
  return Shape<P, H, variant_waves<P, H, 0>(), 2>::FITS &&
         (P == P_F64 || Shape<P, H, variant_waves<P, H, 1>(), 2>::FITS);
}

bool forward_supported(int prec, int h, int words) {
  if (words == 2) {
    // tiles of 256 rows leave no LDS for the head staging of 132 outputs
    static_assert(!fits_two_words<P_BF16, 256>() && !fits_two_words<P_F32, 128>(), "two-word shapes");
    static_assert(fits_two_words<P_BF16, 512>() && fits_two_words<P_F32, 256>() && fits_two_words<P_F64, 64>() &&
                      fits_two_words<P_BF16W, 256>() && fits_two_words<P_BF16X3, 256>(),
                  "two-word shapes");
    if ((prec == P_BF16 && h == 256) || (prec == P_F32 && h == 128)) return false;
  } else if (words != 1) {
    return false;
  }
  switch (prec) {
    case P_BF16: case P_BF16X3: case P_BF16W: return h == 256 || h == 512 || h == 1024;
    case P_F32: return h == 128 || h == 256 || h == 512 || h == 1024;
    case P_F64: return h == 64 || h == 128 || h == 256 || h == 512 || h == 1024;
  }
  return false;
}

int forward_variants(int prec, int h) {
  if (prec == P_F64) return 1;
  return forward_rows_per_block(prec, h) >= 64 ? 4 : 2;   // the half tile keeps 32 rows or more
}

int forward_variant_waves(int prec, int h, int v) {
  const int d = ((prec == P_BF16 || prec == P_BF16X3 || prec == P_BF16W) && h >= 512) ? 16 : 8;
  return (v & 1) == 0 ? d : (d == 16 ? 8 : 16);
}

int forward_variant_rows(int prec, int h, int v) {
  return forward_rows_per_block(prec, h) / ((v & 2) ? 2 : 1);
}

template <bool MULTI, int W>
static void dispatch(const Geom& g, int prec, int h, int v, bool res, int cus, FwdLaunch& la, hipStream_t s) {
#define NQS_CASE(P, H)                                                              \
  if (prec == P && h == H) {                                                        \
    if constexpr (P != P_F64) {                                                     \
      if (v == 1) { launch_one<P, H, 1, MULTI, W>(g, la, res, cus, s); return; }    \
    }                                                                               \
    if constexpr (has_half_tile<P, H>()) {                                          \
      if (v == 2) { launch_one<P, H, 2, MULTI, W>(g, la, res, cus, s); return; }    \
      if (v == 3) { launch_one<P, H, 3, MULTI, W>(g, la, res, cus, s); return; }    \
    }                                                                               \
    launch_one<P, H, 0, MULTI, W>(g, la, res, cus, s);                              \
    return;                                                                         \
  }
  NQS_CASE(P_BF16, 256) NQS_CASE(P_BF16, 512) NQS_CASE(P_BF16, 1024)
  NQS_CASE(P_BF16X3, 256) NQS_CASE(P_BF16X3, 512) NQS_CASE(P_BF16X3, 1024)
  NQS_CASE(P_BF16W, 256) NQS_CASE(P_BF16W, 512) NQS_CASE(P_BF16W, 1024)
  NQS_CASE(P_F32, 128) NQS_CASE(P_F32, 256) NQS_CASE(P_F32, 512) NQS_CASE(P_F32, 1024)
  NQS_CASE(P_F64, 64) NQS_CASE(P_F64, 128) NQS_CASE(P_F64, 256) NQS_CASE(P_F64, 512)
  NQS_CASE(P_F64, 1024)
#undef NQS_CASE
}

void launch_forward(const Geom& g, int variant, bool resident, int cu_count, const void* packed,
                    const uint64_t* x, long long rows_bound, const long long* d_count, double* out,
                    long long* prof_slot, hipStream_t s) {
  FwdLaunch la{};
  la.nseg = 1;
  la.cond_pos = -1;
  la.seg[0] = FwdSeg{nullptr, packed, x, d_count, out, rows_bound, 0, prof_slot};
  if (g.words == 2) dispatch<false, 2>(g, g.prec, g.h, variant, resident, cu_count, la, s);
  else dispatch<false, 1>(g, g.prec, g.h, variant, resident, cu_count, la, s);
}

void launch_forward_cond(const Geom& g, int variant, bool resident, int cu_count, const void* packed,
                         const uint64_t* x, long long rows_bound, const long long* d_count, double* out, int t,
                         hipStream_t s) {
  FwdLaunch la{};
  la.nseg = 1;
  la.cond_pos = t;
  la.seg[0] = FwdSeg{nullptr, packed, x, d_count, out, rows_bound, 0, nullptr};
  if (g.words == 2) dispatch<false, 2>(g, g.prec, g.h, variant, resident, cu_count, la, s);
  else dispatch<false, 1>(g, g.prec, g.h, variant, resident, cu_count, la, s);
}

void launch_forward_multi(int prec, int h, int variant, bool resident, int cu_count, FwdLaunch la,
                          hipStream_t s) {
  if (la.nseg < 1 || la.nseg > kMaxSeg) return;
  la.cond_pos = -1;
  Geom unused{};
  dispatch<true, 1>(unused, prec, h, variant, resident, cu_count, la, s);
}

}  // namespace nqs
