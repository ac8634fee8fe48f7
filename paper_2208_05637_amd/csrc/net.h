// The network's geometry and the fused forward's launch interface, shared by
// the forward kernel, the other kernels and the host side.  Nothing here is
// part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace nqs {

constexpr int kMaxLayers = 16;
constexpr int kMaxQubits = 128;   // bit strings of up to two 64-bit words
constexpr int kMaxNB = 64;        // n-blocks of the fused kernel (h / TB)
constexpr int kMaxNHB = 9;        // head n-blocks ((n + 4) / TB rounded up)
constexpr int kMaxSeg = 8;        // segments of one multi-segment forward launch

enum Prec { P_F64 = 0, P_F32 = 1, P_BF16 = 2, P_BF16X3 = 3, P_BF16W = 4 };

// Device error-word bits (mirrors NQS_DEV_* in nqs.h).
constexpr unsigned kErrZeroAmp = 1u, kErrEntryOverflow = 2u, kErrHashOverflow = 4u;

// Network geometry, passed by value to kernels.  "Sorted units": hidden
// units reordered by degree m_k = 1 + (k mod (n-1)), ascending, so every
// mask becomes a prefix in that order.  "Positions": inputs and head rows
// reordered into sampling order.
struct Geom {
  int n, L, h, prec;
  int n_up, n_dn;           // -1 = unconstrained
  int TB, KSTEP, NB, NHB;   // MFMA block rows, k per fragment, hidden/head n-blocks
  int nhead;                // n + 4
  int q, r;                 // h = q (n-1) + r units per degree class (see class_of)
  int planes;               // 2 for split bf16 (hi, lo), else 1
  int acc_bytes;            // 8 for the FP64 path, else 4
  int order_kind;           // 1: order is the identity, 2: the reverse (n-1, ..., 0), 0: other
  int phase_mode;           // 0: phase head on the shared trunk; 1: separate phase network
  int net_kind;             // what this geometry evaluates: 0 the shared-trunk network (log|psi|
                            // and phi), 1 the modulus network of phase_mode 1 (log|psi| only),
                            // 2 the phase network of phase_mode 1 (phi only; dense layers, units
                            // in their own order, inputs = the first n-2 positions)
  int words;                // 64-bit words per bit string: 1 (n <= 64) or 2
  uint64_t spin_pos[2];     // positions 0..63 whose qubit has spin 0 (even) / 1 (odd)
  uint64_t spin_pos_hi[2];  // the same for positions 64..127
  int8_t order[kMaxQubits]; // position -> qubit
  int8_t pos[kMaxQubits];   // qubit -> position
  int ks1[kMaxNB];  int off1[kMaxNB + 1];
  int ksh[kMaxNB];  int offh[kMaxNB + 1];
  int kso[kMaxNHB]; int offo[kMaxNHB + 1];
  long long frag_h;         // first fragment of hidden layer 2
  long long frag_head;      // first fragment of the head
  long long nfrag;          // fragments per plane
  long long bias_byte;      // byte offset of the biases inside the packed buffer
  long long head_bias_off;  // element offset of the head bias inside the bias array
  long long poff[4 * kMaxLayers + 4];  // offsets of W_1, b_1, ..., W_L, b_L, W_o, b_o, then
                                       // (phase_mode 1) V_1, e_1, ..., V_L, e_L, then W_p, b_p
  long long n_params;
};

// Index into poff of the phase network's layer-l weight (l = 1..L; its bias
// follows) and of the phase head's weight (its bias follows).
__host__ __device__ inline int poff_phase_layer(const Geom& g, int l) { return 2 * g.L + 2 + 2 * (l - 1); }
__host__ __device__ inline int poff_phase_head(const Geom& g) { return g.phase_mode ? 4 * g.L + 2 : 2 * g.L + 2; }

// Unit-class helpers on the sorted hidden units.
__host__ __device__ inline int prefix_of_class(const Geom& g, int c) {
  if (c <= 0) return 0;
  int nm1 = g.n - 1;
  if (c > nm1) c = nm1;
  int v = c * g.q + (c < g.r ? c : g.r);
  return v < g.h ? v : g.h;
}
__host__ __device__ inline int class_of_sorted(const Geom& g, int u) {
  if (g.q == 0) return u;
  int big = g.r * (g.q + 1);
  return u < big ? u / (g.q + 1) : g.r + (u - big) / g.q;
}
__host__ __device__ inline int orig_of_sorted(const Geom& g, int u) {
  int c = class_of_sorted(g, u);
  return c + (u - prefix_of_class(g, c)) * (g.n - 1);
}

void launch_pack_fused(const Geom& g, const float* params, void* packed, hipStream_t s);
void launch_pack_masked(const Geom& g, const float* params, void* wm, hipStream_t s);

// One batch of configurations of one network inside a forward launch:
// rows [0, min(*d_count, rows_bound)) of x -> out[row] = (log|psi|, phi).
struct FwdSeg {
  const Geom* geom;          // device copy of the geometry (multi-segment launches)
  const void* packed;        // packed weights (launch_pack_fused)
  const uint64_t* x;
  const long long* d_count;  // nullable: then rows = rows_bound
  double* out;               // [rows][2]
  long long rows_bound;
  long long tile0;           // first tile of the segment inside the launch
  long long* prof_slot;      // nullable: receives the row count
};
struct FwdLaunch {
  int nseg;
  int cond_pos;   // -1: (log|psi|, phi); >= 0: (logit at that sampling position, forcing code)
  long long ntiles;
  long long tile_base;     // tile of workgroup 0 (a launch too large for one dispatch is split)
  long long tile_stride;   // tiles between a workgroup's successive tiles
  FwdSeg seg[kMaxSeg];
};

// Fused forward over tiles of rows.  variant selects the workgroup shape:
// its waves (forward_variant_waves) and its tile (forward_variant_rows: the
// full tile of forward_rows_per_block rows, or half of it; forward_variants
// says how many variants a (precision, width) has).  resident:
// false = one workgroup per tile (the grid covers the row bound); true = as
// many workgroups as fit on the device's cu_count CUs at once, each looping
// over tiles with a stride of the grid size.  The rows and their arithmetic
// are the same either way.
void launch_forward(const Geom& g, int variant, bool resident, int cu_count, const void* packed,
                    const uint64_t* x, long long rows_bound, const long long* d_count, double* out,
                    long long* prof_slot, hipStream_t s);
// Several segments of networks with equal (precision, width); each segment's
// geometry is read from seg.geom, a device copy written by launch_store_geom.
// la.seg[*].tile0 and la.ntiles are filled in here.
void launch_forward_multi(int prec, int h, int variant, bool resident, int cu_count, FwdLaunch la,
                          hipStream_t s);
// Conditional form for the sampler: out[row] = (o_t, code) with o_t the
// conditional logit at sampling position t and code 0 (free), 1 (forced to
// 0) or 2 (forced to 1) by the Hamming-weight modifier.
void launch_forward_cond(const Geom& g, int variant, bool resident, int cu_count, const void* packed,
                         const uint64_t* x, long long rows_bound, const long long* d_count, double* out, int t,
                         hipStream_t s);
void launch_store_geom(const Geom& g, Geom* dst, hipStream_t s);
int forward_variants(int prec, int h);
int forward_variant_waves(int prec, int h, int variant);
int forward_variant_rows(int prec, int h, int variant);   // configurations per workgroup tile

int forward_rows_per_block(int prec, int h);
// (prec, width) has a fused forward for bit strings of `words` 64-bit words
bool forward_supported(int prec, int h, int words);

}  // namespace nqs
