// Internal declarations shared by the host side (nqs_capi.cpp) and the HIP
// kernels.  Nothing here is part of the C ABI.
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

// Tensor of the Hamiltonian on the device.  Masks and bit strings take
// `words` 64-bit words each (word w = qubits 64w .. 64w+63).
struct HamDev {
  const uint64_t* gx;
  const long long* goff;
  const uint64_t* tz;
  const double* tre;
  const double* tim;   // nullptr when every folded coefficient is real
  int G;
  int gfirst;          // 1 if group 0 is the empty flip
  int filter;          // spin-sector filter on
  int words;           // 1 or 2
  // structured matrix elements (tables != 0): sub-groups soff[g] .. soff[g+1],
  // off-flip masks su[s][words], table of sub-group s at stab[s], 2^m entries
  // indexed by the bits of x at fpos[4g .. 4g+3] (-1 unused)
  int tables;
  const long long* soff;
  const uint64_t* su;
  const long long* stab;
  const double* tabre;
  const double* tabim;   // nullptr when every folded coefficient is real
  const int8_t* fpos;
};

// ---- launchers (kernels_*.hip) -------------------------------------------
void launch_fill_u32(void* p, unsigned v, long long count, hipStream_t s);
void launch_fill_u64(void* p, unsigned long long v, long long count, hipStream_t s);

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

// Fused forward over tiles of forward_rows_per_block rows.  variant selects
// the workgroup shape (forward_variants / forward_variant_waves).  resident:
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

void launch_diag(const HamDev& H, const uint64_t* x, long long S, double* diag, hipStream_t s);
void launch_count(const HamDev& H, const uint64_t* x, long long S, int R, int gper, int* cnt,
                  hipStream_t s);
// exclusive scan; tmp holds scan_tiles(n) + 1 values
long long scan_tiles(long long n);
void launch_scan(const int* cnt, long long n, long long* off, long long* tmp, hipStream_t s);
void launch_write(const HamDev& H, const uint64_t* x, long long S, int R, int gper,
                  const long long* off, long long cap, uint64_t* xe, double* he, int* esample,
                  int hstride, unsigned* err, hipStream_t s);

// Distinct keys of xe[0 .. min(*d_count, cap)) (`words` 64-bit words each)
// into xu, eu[e] = index of entry e's key in xu, *d_nu = their number, through
// `table`: HT records of kHashRecBytes (HT a power of two above the count).
// first_order: xu in the order of the keys' first entries (first: int[cap],
// rank: i64[cap + 1], rank_tmp: dedup_rank_tmp_elems(cap)); otherwise in the
// order their inserts filled the table (first, rank, rank_tmp unused).
// all_ones_key: one-word keys may be the all-ones word (64 qubits), so the
// table takes slot words instead of keys.  After the call the table maps each
// key (one-word keys below 64 qubits) to its index in xu.
constexpr size_t kHashRecBytes = 16;
long long dedup_rank_tmp_elems(long long cap);
void launch_dedup(const uint64_t* xe, int words, bool all_ones_key, const long long* d_count, long long cap,
                  void* table, long long HT, bool first_order, int* eu, uint64_t* xu, long long* d_nu, int* first,
                  long long* rank, long long* rank_tmp, unsigned* err, hipStream_t s);
// Look-back of a chunk's distinct configurations xu[0 .. *d_nu) into the
// previous chunk's one-word table (ptable, after that chunk's launch_dedup):
// src[u] = the previous index or -1; the new ones compacted in order into
// xnew, *d_nnew = their number, rank[u] = the position of a new one.
// isnew: int[cap], rank: i64[cap + 1], rank_tmp: dedup_rank_tmp_elems(cap).
void launch_lookback(const uint64_t* xu, const long long* d_nu, long long cap, const void* ptable, long long HT,
                     int* src, int* isnew, long long* rank, long long* rank_tmp, uint64_t* xnew, long long* d_nnew,
                     hipStream_t s);
// lp[u] = lp_prev[src[u]] where src[u] >= 0, else lp_new[rank[u]] (pairs of
// doubles), u < *d_nu.
void launch_lookback_gather(const long long* d_nu, long long cap, const int* src, const long long* rank,
                            const double* lp_prev, const double* lp_new, double* lp, hipStream_t s);

// partials holds reduce_partials_elems(S) doubles
long long reduce_partials_elems(long long S);
void launch_reduce(long long S, int R, const long long* off, long long cap, const double* diag,
                   const double* he, int hstride, const int* eu, const double* lpe,
                   const double* lps, double* eloc, double* partials, unsigned* err, hipStream_t s);
void launch_energy(const double* eloc, const double* w, long long B, double* energy,
                   unsigned* err, hipStream_t s);

// backward: recompute the sample forward on S samples and accumulate the
// gradient into grad (f64, flat parameter layout).  scratch holds
// backward_scratch_elems(g, S) elements of the path's backward type
// (double for the FP64 path, float otherwise).
long long backward_scratch_elems(const Geom& g, long long S);
void launch_backward(const Geom& g, const void* wm, const uint64_t* x, long long S,
                     const double* eloc, const double* w, const double* energy, void* scratch,
                     double* grad, hipStream_t s);

// Sampler buffers (kernels_sample.hip); capacity umax entries, children 2 umax.
struct SampleBufs {
  uint64_t* x;       // [umax] configurations, in buffer order
  long long* cnt;    // [umax] draws
  double* cond;      // [umax][2] conditional logit and forcing code
  uint64_t* kx;      // [2 umax] children
  long long* kc;     // [2 umax]
  int* eq;           // [2 umax] tie flags
  int* keep;         // [2 umax]
  long long* eqoff;  // [2 umax + 1]
  long long* koff;   // [2 umax + 1]
  long long* stmp;   // scan_tiles(2 umax) + 1
  long long* sel;    // [2] threshold, quota
  long long* d_u;    // entries in the buffer
  long long* d_nk;   // children
  int words;         // 64-bit words per configuration (x and kx hold `words` words each)
};
void launch_sample_init(uint64_t* x, int words, long long* cnt, long long n_draws, long long* d_u, hipStream_t s);
void launch_sample_step(const SampleBufs& b, long long umax, int t, int q, uint64_t seed, hipStream_t s);
void launch_sample_finish(const SampleBufs& b, long long umax, uint64_t* ox, double* ow, long long* on,
                          hipStream_t s);

// Adam coefficients, formed on the host: bc1 = 1 - b1^t, bc2 = 1 - b2^t.
struct AdamCoef {
  double lr, b1, b2, one_m_b1, one_m_b2, bc1, bc2, eps;
};
void launch_adam(long long n, float* p, const double* g, double* m, double* v, const AdamCoef& k, int cu_count,
                 hipStream_t s);

int forward_rows_per_block(int prec, int h);
// (prec, width) has a fused forward for bit strings of `words` 64-bit words
bool forward_supported(int prec, int h, int words);

}  // namespace nqs
