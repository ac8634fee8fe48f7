// Internal declarations shared by the host side (nqs_capi.cpp) and the HIP
// kernels.  Nothing here is part of the C ABI.
#pragma once
#include "net.h"

namespace nqs {

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
  long long max_gterms;  // terms of the largest group past the empty flip
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

}  // namespace nqs
