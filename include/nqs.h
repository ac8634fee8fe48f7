/*
 * nqs.h -- C ABI of the MI355X (gfx950) local-energy / VMC-gradient library.
 *
 * The library evaluates, for a batch of bit-string samples x_i and a masked
 * autoregressive amplitude/phase network psi_theta, the quantities of
 * Zhao, Stokes & Veerapaneni, "Scalable neural quantum states architecture
 * for quantum chemistry" (arXiv 2208.05637):
 *
 *   local energy   E_loc(x) = sum_k alpha_k <x|P_k|x^k> psi(x^k)/psi(x)
 *                  (Sec. 5.1, Eq. local_energy_auto; matrix element by
 *                  Eq. mtx_element; Alg. 1),
 *   energy         E = sum_i w_i Re E_loc(x_i) / sum_i w_i
 *                  (Sec. 5.2, Eq. total_energy_sum, with sample weights),
 *   gradient       g = 2 Re sum_i (w_i/W) (E_loc(x_i) - E) conj(d log psi(x_i))
 *                  (Sec. 3, Eq. grad, with baseline b = E; this is the
 *                  gradient of <H>, i.e. twice the gradient of the paper's
 *                  L = <H>/2).
 *
 * Conventions shared by every call
 *   - A bit string (a sample, a configuration, a mask) of n qubits is W =
 *     ceil(n / 64) uint64 words, W = 1 for n <= 64 and W = 2 for
 *     64 < n <= 128 (the paper's largest system has 76 qubits, Sec. 6):
 *     qubit j is bit (j mod 64) of word j / 64 (qubit j is the paper's
 *     x_{j+1}).  Arrays of bit strings are word-major per string: string i
 *     occupies words [i*W, i*W + W).
 *   - A Pauli string is (x_mask, z_mask): factor on qubit j is I, X, Z, Y for
 *     (x_j, z_j) = (0,0), (1,0), (0,1), (1,1) (Sec. 3, Eq. 1).
 *   - Even qubits carry spin up, odd qubits spin down (Sec. 4, Constraints).
 *   - Status codes are returned, never exceptions; nqs_last_error() gives a
 *     thread-local text for the last failing call on the calling thread.
 *   - Argument errors are detected on the host before anything is enqueued.
 *     Errors found on the device (zero amplitude of a sample, entry-buffer
 *     overflow, hash-table overflow) set bits of a device error word kept in
 *     the first bytes of the workspace; nqs_device_status() reads it.
 *   - Device pointers ("d_") are caller-owned device memory; the library
 *     never allocates or frees device memory.  Host pointers are read during
 *     the call only.  Handles (ctx, ham, plan) are host objects owned by the
 *     library and released with the matching *_destroy.
 *   - Every device call is stream-ordered on the context's stream, performs
 *     no host synchronisation and no allocation (so it can be captured into a
 *     HIP graph), unless stated otherwise.
 */
#ifndef NQS_H
#define NQS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NQS_OK = 0,
  NQS_ERR_INVALID_ARGUMENT = 1,
  NQS_ERR_UNSUPPORTED = 2,          /* n_qubits > 128, width, device not gfx950 */
  NQS_ERR_NOT_HERMITIAN = 3,        /* nonzero imaginary Pauli coefficient    */
  NQS_ERR_WORKSPACE_TOO_SMALL = 4,
  NQS_ERR_HIP = 5,                  /* a HIP runtime call failed              */
  NQS_ERR_DEVICE = 6                /* device error word is nonzero           */
} nqs_status;

/* Device error-word bits (nqs_device_status). */
#define NQS_DEV_ZERO_AMPLITUDE   1u  /* a sample has psi = 0 (outside the sector) */
#define NQS_DEV_ENTRY_OVERFLOW   2u  /* more connected entries than planned      */
#define NQS_DEV_HASH_OVERFLOW    4u  /* dedup hash table full                    */

/* Text for a status code (static storage). */
const char* nqs_status_str(int status);
/* Copies the calling thread's last error text into buf (NUL-terminated,
   truncated to len); returns the full length of the text. */
size_t nqs_last_error(char* buf, size_t len);
/* Library version, major*10000 + minor*100 + patch. */
int nqs_version(void);
/* SHA-256 (hex, static storage) of the sources the library was built from,
   as computed by the package's build script; "unknown" for a build that did
   not define it.  The Python binding refuses a library whose hash differs
   from that of the sources beside it (a stale build). */
const char* nqs_source_hash(void);

/* ------------------------------------------------------------------ context */
typedef struct nqs_ctx nqs_ctx;
/* Binds a HIP device and stream (a hipStream_t passed as void*; NULL = the
   default stream).  Fails with NQS_ERR_UNSUPPORTED unless the device is gfx950.
   No device memory is allocated. */
nqs_status nqs_ctx_create(int device, void* stream, nqs_ctx** out);
nqs_status nqs_ctx_set_stream(nqs_ctx* ctx, void* stream);
void       nqs_ctx_destroy(nqs_ctx* ctx);

/* -------------------------------------------------------------- Hamiltonian
 * Sec. 3 (Eq. hamiltonpauli) and Sec. 5.1: H = sum_k alpha_k P_k, parsed once
 * into a tensor of unique flips.  nqs_ham_create works on the host only:
 *   1. identical (x_mask, z_mask) are merged by sequential FP64 addition in
 *      input order;
 *   2. merged terms with |alpha| < drop_tol are removed;
 *   3. alpha must be real (a Hermitian H has real Pauli coefficients): any
 *      nonzero coeff_imag[k] gives NQS_ERR_NOT_HERMITIAN;
 *   4. the factor (-i)^{popcount(x&z)} of Eq. mtx_element is folded into the
 *      coefficient: ct_k = alpha_k (-i)^{r_k}, stored as (re, im) planes;
 *   5. terms are sorted by (x_mask, z_mask) ascending and grouped by x_mask
 *      (one group per distinct flip; group 0 is the empty flip if present).
 * Masks are ordered as unsigned integers of n bits (the last word most
 * significant).  Device layout (structure of arrays, written by
 * nqs_ham_upload into caller storage of nqs_ham_info's `bytes`): gx[G][W]
 * u64 flips, goff[G+1] i64 term offsets, tz[K][W] u64 z masks, tc_re[K] f64,
 * tc_im[K] f64 (only if has_imag).
 */
typedef struct {
  int            n_qubits;     /* 1..128 */
  int64_t        n_terms;      /* input terms, >= 0 */
  const uint64_t* x_mask;      /* host [n_terms][W] */
  const uint64_t* z_mask;      /* host [n_terms][W] */
  const double*   coeff;       /* host [n_terms], real part */
  const double*   coeff_imag;  /* host [n_terms] or NULL; must be all zero */
  double          drop_tol;    /* merged |alpha| < drop_tol removed (e.g. 1e-10) */
  uint32_t        flags;       /* NQS_H_* */
} nqs_pauli_terms;

/* The Hamiltonian conserves the number of up and of down electrons, so a
   flip group can be skipped for a sample when it changes either count
   (an integer test).  Without the flag a group is skipped only when its
   matrix element is exactly 0.0. */
#define NQS_H_CONSERVES_SPIN_SECTORS 1u
/* Structured matrix elements (the Jordan-Wigner structure of a molecular
   Hamiltonian, Sec. 5.1).  Inside group g with flip f every term's z mask is
   split as z = u xor (z & f), u = z & ~f.  The terms with equal u form a
   sub-group s (in order of first appearance in the canonical order); its
   table T_s has 2^m entries, m = popcount(f) <= 4, T_s[b] = sum over its
   terms of ct_k (-1)^{popcount(z_k & f & spread(b))} in canonical order,
   spread(b) placing bit j of b on the j-th lowest qubit of f.  The
   enumeration then evaluates
       h_g(x) = sum_s (-1)^{popcount(x & u_s)} T_s[bits of x at f]
   which is Eq. mtx_element summed over the group, in another order: a
   double excitation is one sub-group with a 16-entry table, a single
   excitation a few 4-entry tables (a linear form in the occupations), the
   diagonal one entry per term.  A group whose flip has more than 4 qubits
   gives NQS_ERR_UNSUPPORTED at nqs_ham_create. */
#define NQS_H_TABLES 2u

typedef struct nqs_ham nqs_ham;
nqs_status nqs_ham_create(const nqs_pauli_terms* terms, nqs_ham** out);
/* K merged terms, G groups, device bytes, has_imag (any odd-Y string). */
nqs_status nqs_ham_info(const nqs_ham* ham, int64_t* K, int64_t* G, size_t* bytes,
                        int* has_imag, int* n_qubits);
/* Copies the tensor into d_storage (>= bytes, 256-byte aligned) on the
   context's stream and records the pointer; the storage must outlive every
   plan built on this Hamiltonian.  This call synchronises the stream. */
nqs_status nqs_ham_upload(nqs_ham* ham, nqs_ctx* ctx, void* d_storage, size_t bytes);
/* Host copy of the canonical tensor (any pointer may be NULL to skip):
   gx [G][W], goff [G+1], tz [K][W], tc_re [K], tc_im [K]. */
nqs_status nqs_ham_export(const nqs_ham* ham, uint64_t* gx, int64_t* goff, uint64_t* tz,
                          double* tc_re, double* tc_im);
/* Sizes and host copy of the tables of an NQS_H_TABLES Hamiltonian (zero
   sizes otherwise; any pointer may be NULL to skip): S sub-groups, E table
   entries; soff [G+1] first sub-group of each group, su [S][W] off-flip z
   masks, stab [S] first table entry of each sub-group, tab_re [E],
   tab_im [E] (zero unless has_imag), fpos [G][4] the flip's qubits in
   ascending order, -1 past its popcount. */
nqs_status nqs_ham_table_info(const nqs_ham* ham, int64_t* S, int64_t* E);
nqs_status nqs_ham_export_tables(const nqs_ham* ham, int64_t* soff, uint64_t* su, int64_t* stab,
                                 double* tab_re, double* tab_im, int8_t* fpos);
void       nqs_ham_destroy(nqs_ham* ham);

/* ------------------------------------------------------------------ network
 * Sec. 4 (Architecture, Constraints): masked autoregressive network with a
 * shared trunk of n_layers masked ReLU layers of `width` units, a
 * conditional head (n logits, pi_j = sigmoid) and a 4-way phase head.
 *   s = 2x - 1;  a_l = ReLU((M_l*W_l) a_{l-1} + b_l);
 *   o = (M_o*W_o) a_L + b_o;  p = (M_p*W_p) a_L + b_p;
 *   log|psi| = 1/2 sum_{free j} log pi_j(x_j);  phi = p[2 x_{o[n-2]} + x_{o[n-1]}]
 * with qubit degrees d(j) = 1 + position of j in `order`, hidden degrees
 * m_k = 1 + (k mod (n-1)), masks [m_k >= d(j)], [m_k >= m_k'], [d(j) > m_k],
 * [m_k <= n-2], and the Hamming-weight modifier of Eq. modifier (a position
 * is forced to 0 once n_s spin-s electrons are placed, to 1 when the
 * remaining spin-s positions are all needed; forced positions contribute 0,
 * a contradicted forced value gives psi = 0).
 * Parameters: one flat FP32 buffer W_1, b_1, ..., W_L, b_L, W_o, b_o,
 * [V_1, e_1, ..., V_L, e_L with NQS_PHASE_SEPARATE,] W_p, b_p, weights
 * row-major [out][in] (in_1 = n).  Gradients use the same
 * layout in FP64; masked-out weights receive 0.
 */
/* Arithmetic of the network on the connected configurations:
 *   NQS_FP64   FP64 MFMA;  NQS_FP32  FP32 MFMA;
 *   NQS_BF16   BF16 weights and activations, FP32 accumulation;
 *   NQS_BF16X3 FP32 weights and activations each split into two BF16 terms
 *              (hi + lo), three BF16 products per multiply-add (lo*lo
 *              dropped), FP32 accumulation;
 *   NQS_BF16W  a BF16 network: every weight is the parameter rounded to the
 *              nearest BF16 (ties to even) when packed, for the forward and
 *              the backward alike, so the gradient is that network's;
 *              biases stay FP32; activations are split into two BF16 terms
 *              (two BF16 products per multiply-add), FP32 accumulation.
 *              With BF16-valued parameters the rounding is the identity. */
enum { NQS_FP64 = 0, NQS_FP32 = 1, NQS_BF16 = 2, NQS_BF16X3 = 3, NQS_BF16W = 4 };

/* The phase network (Sec. 4, Architecture: modulus and phase sub-models).
 *   NQS_PHASE_SHARED    the phase head W_p [4][h] reads the last hidden layer
 *                       of the masked trunk, restricted to units of degree
 *                       <= n-2;
 *   NQS_PHASE_SEPARATE  the paper's separate phase sub-model: a plain MLP of
 *                       the same depth L and width h whose input is the first
 *                       n-2 entries in sampling order (2x-1), c_1 =
 *                       ReLU(V_1 v + e_1), c_l = ReLU(V_l c_{l-1} + e_l), then
 *                       W_p [4][h]; no masks (its input already excludes the
 *                       last two positions).  Its layers V_1 [h][n-2], e_1,
 *                       ..., V_L [h][h], e_L sit in the parameter layout
 *                       between b_o and W_p.  n_qubits >= 3.
 * In both, phi = p[2 x_{order[n-2]} + x_{order[n-1]}]. */
enum { NQS_PHASE_SHARED = 0, NQS_PHASE_SEPARATE = 1 };

typedef struct {
  int            n_qubits;   /* 2..128 */
  int            n_layers;   /* >= 1 */
  int            width;      /* 64, 128, 256, 512 or 1024 (precision dependent; above
                                64 qubits not FP32 at 128 nor BF16 at 256) */
  const int32_t* order;      /* host [n_qubits] sampling order, NULL = n-1, ..., 0 */
  int            n_up, n_dn; /* electrons per spin; both -1 = unconstrained */
  int            precision;  /* NQS_FP64 | NQS_FP32 | NQS_BF16 | NQS_BF16X3 | NQS_BF16W
                                (above); Hamiltonian sums, ratios and reductions
                                are FP64 in every case */
  int            phase_mode; /* NQS_PHASE_SHARED or NQS_PHASE_SEPARATE (below) */
} nqs_net_desc;

nqs_status nqs_net_param_count(const nqs_net_desc* net, int64_t* n_params);

/* --------------------------------------------------------------------- plan */
/* Dedup applies at every width (Sec. 5.2, local removal of replicated
   configurations).  Below 64 qubits (one-word strings whose table holds the
   strings themselves) it also looks back one chunk: a chunk's distinct
   configurations that the previous chunk of the same call evaluated take that
   chunk's log psi instead of a forward row (the same values; the workspace
   then holds two hash tables and two log psi sets). */
#define NQS_PLAN_DEDUP_ON   1u   /* deduplicate connected configurations per chunk */
#define NQS_PLAN_DEDUP_OFF  2u   /* never deduplicate (default when no flag is set) */
#define NQS_PLAN_DEDUP_AUTO 4u   /* size the workspace for dedup, start with it on and
                                    let nqs_plan_autotune decide */

typedef struct nqs_plan nqs_plan;
/* Fixes the chunking (chunk_samples samples per chunk; <= 0 picks a default
   from the per-sample entry bound) and the kernel variants for batches of
   up to max_batch samples.  Host only. */
nqs_status nqs_plan_create(nqs_ctx* ctx, const nqs_ham* ham, const nqs_net_desc* net,
                           int64_t max_batch, uint32_t flags, int64_t chunk_samples,
                           nqs_plan** out);
nqs_status nqs_plan_workspace_size(const nqs_plan* plan, int64_t batch, size_t* bytes);
/* Plan facts: per-sample entry bound, chunk size, dedup on/off, number of
   parameters. */
nqs_status nqs_plan_info(const nqs_plan* plan, int64_t* entries_per_sample,
                         int64_t* chunk_samples, int* dedup, int64_t* n_params);
void       nqs_plan_destroy(nqs_plan* plan);

/* Sets what the autotuner chooses: the forward's workgroup shape, as waves
   per workgroup and configurations per workgroup tile (a pair that
   nqs_plan_autotune reports; each <= 0 keeps the current value), dedup (1 on,
   0 off, < 0 keep; on needs a plan created with DEDUP_ON or
   DEDUP_AUTO), the chunk (between half the created chunk and the created
   chunk; <= 0 keeps) and the forward's grid (resident: 1 = as many
   workgroups as the device holds at once, each looping over tiles of rows;
   0 = one workgroup per tile; < 0 keep).  Host only. */
nqs_status nqs_plan_configure(nqs_plan* plan, int waves_per_block, int rows_per_block, int dedup,
                              int64_t chunk_samples, int resident);

/* Workgroup shape of the plan's connected-configuration forward: waves per
   workgroup, configurations per workgroup, whether the plan was tuned, and
   whether the forward runs a resident grid (each output may be NULL). */
nqs_status nqs_plan_kernel_info(const nqs_plan* plan, int* waves_per_block, int* rows_per_block,
                                int* tuned, int* resident);

/* Autotuner for the chunked local-energy path (the paper's mini-batches,
   Sec. 5.2 and Sec. 6): times the local-energy phase on the first
   min(B, 2 * chunk) samples of d_samples for every candidate
     forward workgroup shape (waves per workgroup x tile: the full tile,
     and half of it where that keeps 32 rows or more) x dedup on/off (only with
     NQS_PLAN_DEDUP_AUTO) x chunk in {plan chunk, plan chunk / 2}
     x forward grid (one workgroup per tile, or resident workgroups
     looping over tiles)
   and keeps the fastest in the plan.  The choice is cached per process,
   keyed by the network shape, the Hamiltonian's term and group counts and
   the plan's chunk; a later call with the same key applies it without timing
   (NQS_TUNE_FORCE re-times; NQS_TUNE_CACHE_ONLY applies a cached choice if
   there is one and otherwise returns NQS_OK with n_candidates = 0 and the
   plan unchanged, without timing or touching the device).  Every candidate
   computes the same local energies up to the forward's rounding (dedup,
   chunking and the grid change nothing; the two workgroup shapes split the
   head's k sum differently).  Synchronises the
   context's stream; not for use under graph capture.  d_ws must hold
   nqs_plan_workspace_size(plan, B) bytes.  report may be NULL.  With the
   environment variable NQS_TUNE_LOG set, each timed candidate is also
   reported as one line on stderr. */
#define NQS_TUNE_FORCE 1u
#define NQS_TUNE_CACHE_ONLY 2u
#define NQS_TUNE_MAX_CANDIDATES 32
typedef struct {
  int     waves_per_block;
  int     rows_per_block;  /* configurations per workgroup tile */
  int     dedup;
  int64_t chunk_samples;
  int     resident;        /* 1: resident grid looping over tiles */
  double  ms;              /* one local-energy pass over the probe samples */
} nqs_tune_candidate;
typedef struct {
  int     n_candidates;
  int     chosen;          /* index into cand */
  int     from_cache;      /* 1: applied from the cache, cand[0] is the cached choice */
  int64_t probe_samples;
  nqs_tune_candidate cand[NQS_TUNE_MAX_CANDIDATES];
} nqs_tune_report;
nqs_status nqs_plan_autotune(nqs_plan* plan, const float* d_params, const uint64_t* d_samples, int64_t B,
                             void* d_ws, size_t ws_bytes, uint32_t flags, nqs_tune_report* report);

/* The tuner's cached choices as a text file, so that a later process applies
   them without timing (a tuning database, as kept for the chunk size of the
   paper's mini-batches, Sec. 5.2).  nqs_tune_db_save writes every entry of
   this process's cache to path (through a temporary file renamed over it);
   nqs_tune_db_load adds the entries of path to the cache, replacing equal
   keys, and sets *n_loaded (may be NULL).  A key holds the network shape and
   precision, the Hamiltonian's term and group counts, the per-sample entry
   bound, the created chunk, the dedup mode and the device index; an entry is
   applied by nqs_plan_autotune (without NQS_TUNE_FORCE) only to a plan with
   the same key whose workspace has room for it.  Errors: NULL path or an
   unreadable/unwritable file (NQS_ERR_INVALID_ARGUMENT); a malformed line
   stops the load with NQS_ERR_INVALID_ARGUMENT, keeping the lines before
   it.  Host only. */
nqs_status nqs_tune_db_save(const char* path);
nqs_status nqs_tune_db_load(const char* path, int* n_loaded);

/* ---------------------------------------------------------------- hot path
 * All pointers are device pointers; d_ws is a workspace of at least
 * nqs_plan_workspace_size(plan, B) bytes, 256-byte aligned.  Samples are
 * read as uint64 [B][W]; weights f64 [B] (NULL = all 1).
 */

/* log psi for n configurations: d_out[2*i] = log|psi|, d_out[2*i+1] = phi,
   computed by the connected-configuration forward kernel of the plan's
   precision (-inf for psi = 0).  Sec. 4, the complex logarithm of f. */
nqs_status nqs_log_psi(nqs_plan* plan, const float* d_params, const uint64_t* d_x, int64_t n,
                       double* d_out, void* d_ws, size_t ws_bytes);

/* Local energies d_eloc[2*i] + i d_eloc[2*i+1] (Eq. local_energy_auto). */
nqs_status nqs_local_energy(nqs_plan* plan, const float* d_params, const uint64_t* d_samples,
                            int64_t B, double* d_eloc, void* d_ws, size_t ws_bytes);

/* Local energies (d_eloc may be NULL), the energy d_energy[3] = {E, mean of
   Im E_loc, W = sum w} (Eq. total_energy_sum) and the gradient d_grad
   [n_params] f64 (Eq. grad, see the top of this file).  The backward pass
   recomputes the sample forward instead of storing activations of the
   connected configurations, chunk by chunk (gradient accumulation). */
nqs_status nqs_energy_grad(nqs_plan* plan, const float* d_params, const uint64_t* d_samples,
                           const double* d_weights, int64_t B, double* d_eloc,
                           double* d_energy, double* d_grad, void* d_ws, size_t ws_bytes);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc):
   nqs_energy_grad with the library's own workspace, a static device array of
   NQS_NOALLOC_SCRATCH_BYTES per GPU, held from the first context created on
   that GPU until the process ends.  Calls no allocating routine.  Arguments
   and results as nqs_energy_grad; d_flags (device uint32, may be NULL)
   receives the call's device error word (NQS_DEV_* bits), which the call
   clears at its start.  Fails with NQS_ERR_WORKSPACE_TOO_SMALL, before
   anything is enqueued, when nqs_plan_workspace_size(plan, B) exceeds the
   array (create the plan with a smaller max_batch or chunk).  Every call on
   one GPU uses the same array: calls that overlap on that GPU (several
   streams or threads) race, so the caller orders them.  Not profiled. */
#define NQS_NOALLOC_SCRATCH_BYTES (256u << 20)
nqs_status nqs_energy_grad_noalloc(nqs_plan* plan, const float* d_params, const uint64_t* d_samples,
                                   const double* d_weights, int64_t B, double* d_eloc,
                                   double* d_energy, double* d_grad, uint32_t* d_flags);

/* Several independent (Hamiltonian, network, samples) instances in one call
   (the paper's independent units of work, Sec. 5.2).  Each instance uses
   its own plan (all plans on the same context) and its own part of d_ws,
   which must hold nqs_multi_workspace_size bytes.  The sample forwards of
   all instances are one work list, and so are the connected-configuration
   forwards of each chunk round (round r holds chunk r of every instance that
   has one): one forward launch per round and per group of at most 8
   instances with equal precision, width and forward variant.  Enumeration,
   ratio-and-reduce, energy and gradient run per instance.  Each instance's
   results equal those of nqs_energy_grad on it alone. */
typedef struct {
  nqs_plan*       plan;
  const float*    d_params;
  const uint64_t* d_samples;
  const double*   d_weights;
  int64_t         B;
  double*         d_eloc;    /* may be NULL */
  double*         d_energy;  /* [3] */
  double*         d_grad;    /* [n_params] */
} nqs_instance;
/* Instances of more than 64 qubits, and instances whose forward variant
   takes the half tile (nqs_plan_configure), run their forwards as launches
   of their own inside the same call: the shared work lists take one-word
   strings in full tiles. */
nqs_status nqs_multi_workspace_size(int n_inst, const nqs_instance* inst, size_t* bytes);
nqs_status nqs_energy_grad_multi(int n_inst, const nqs_instance* inst, void* d_ws, size_t ws_bytes);

/* ---------------------------------------------------------------- sampler
 * Unique-sample autoregressive sampling of the plan's network (Sec. 4,
 * Sampling; Eq. modifier for the Hamming-weight constraint).  A buffer of
 * distinct configurations with draw counts starts as the all-zero
 * configuration holding n_draws draws; at each sampling position t (qubit
 * order[t]) every entry is doubled into x = 0 / x = 1 children, its draws
 * are split by a binomial draw with the network's conditional probability
 * (0 or 1 where the modifier forces the value), empty children are dropped,
 * and beyond max_unique entries those with the fewest draws are eliminated
 * (ties: earlier buffer entries kept; the buffer is ordered by the bits in
 * sampling order).  Random numbers: Philox4x64-10, counter (the parent's
 * word 0, t, its word 1 (0 up to 64 qubits), j) for blocks j = 0, 1, ...,
 * key (seed, 0); Bin(c, p), exact: by inversion from 0 when
 * c min(p, 1-p) < 32 (first uniform of block 0), else Hormann's BTRS
 * rejection method (1993; two uniforms per attempt, in block order),
 * reflected for p > 1/2.
 * Outputs (device): d_x[u] configurations (W uint64 words each), d_w[u]
 * their draw counts as f64 weights, d_n_unique[0] = U <= max_unique, for
 * u < U in buffer order.  d_x and d_w hold max_unique entries.  The network
 * arithmetic is the plan's precision.  d_ws: nqs_sample_workspace_size
 * bytes, 256-byte aligned.  Stream-ordered, no host synchronisation. */
nqs_status nqs_sample_workspace_size(const nqs_plan* plan, int64_t max_unique, size_t* bytes);
nqs_status nqs_sample(nqs_plan* plan, const float* d_params, int64_t n_draws, uint64_t seed,
                      int64_t max_unique, uint64_t* d_x, double* d_w, int64_t* d_n_unique,
                      void* d_ws, size_t ws_bytes);

/* -------------------------------------------------------------- optimizer
 * One Adam step (Kingma and Ba, ICLR 2015; the paper trains with Adam, Sec. 6,
 * learning rate 1e-3, betas (0.9, 0.99)) on the FP32 parameters with the FP64
 * gradient of nqs_energy_grad, for every i < n:
 *   m_i <- b1 m_i + (1 - b1) g_i
 *   v_i <- b2 v_i + (1 - b2) g_i g_i
 *   p_i <- p_i - lr (m_i / (1 - b1^t)) / (sqrt(v_i / (1 - b2^t)) + eps)
 * with t = step >= 1, the number of this step.  d_m and d_v are FP64 [n],
 * caller-owned, zero before step 1.  The update is FP64, evaluated in the
 * order written (no fused multiply-adds), and the parameter is rounded to the
 * nearest FP32.  Errors: NULL pointers with n > 0, step < 1, lr < 0,
 * betas outside [0, 1) or eps < 0 give NQS_ERR_INVALID_ARGUMENT, nothing is
 * enqueued.  Stream-ordered on the context's stream, capture-safe. */
nqs_status nqs_adam_step(nqs_ctx* ctx, int64_t n, float* d_params, const double* d_grad, double* d_m,
                         double* d_v, int64_t step, double lr, double beta1, double beta2, double eps);

/* ------------------------------------------------------ test / table path
 * nqs_connected enumerates, for samples [0, B), the diagonal element
 * d_diag[2*i..] (group with empty flip) and the compacted connected entries
 * in sample-major, group-ascending order: d_entry_sample[e] (i32),
 * d_entry_x[e] = x_i ^ f_g (W u64 words), d_entry_h[2*e..] = sum over the group's
 * terms of ct_k (-1)^{popcount(x_i & z_k)} summed sequentially in canonical
 * order (FP64).  Entry buffers must hold `capacity` entries; the count is
 * written to d_n_entries[0] (if it exceeds capacity only the first
 * `capacity` are written and NQS_DEV_ENTRY_OVERFLOW is raised).  With dedup
 * (plan flag) d_unique[u] receives the distinct x' (W words each, in the order of their first entries), d_n_unique[0]
 * their number and d_entry_unique[e] the index of entry e's x' in d_unique;
 * without dedup these outputs may be NULL.
 */
nqs_status nqs_connected(nqs_plan* plan, const uint64_t* d_samples, int64_t B, int64_t capacity,
                         double* d_diag, int32_t* d_entry_sample, uint64_t* d_entry_x,
                         double* d_entry_h, int64_t* d_n_entries, uint64_t* d_unique,
                         int32_t* d_entry_unique, int64_t* d_n_unique, void* d_ws, size_t ws_bytes);

/* Ratio-and-reduce with caller-supplied log amplitudes (for example an exact
   eigenvector): d_eloc[i] = diag[i] + sum_{e: sample(e)=i} h_e
   exp(logpsi_entry[e] - logpsi_sample[i]) (complex logs as (log|psi|, phi)
   pairs).  Entries must be sample-major as produced by nqs_connected.  Sum in
   FP64 with compensation, deterministic order. */
nqs_status nqs_reduce_table(nqs_plan* plan, int64_t B, const double* d_logpsi_samples,
                            const double* d_logpsi_entries, const double* d_diag,
                            const int32_t* d_entry_sample, const double* d_entry_h,
                            int64_t n_entries, double* d_eloc, void* d_ws, size_t ws_bytes);

/* ------------------------------------------------------------- profiling
 * While enabled, nqs_local_energy / nqs_energy_grad record HIP events on the
 * context's stream around each call, around its local-energy phase and
 * around every connected-configuration forward launch, and the forward
 * kernel stores the number of rows it processed into a slot of the
 * workspace.  nqs_plan_profile_read synchronises the stream, returns the
 * totals accumulated since the last read (or enable) and resets them.
 * Enabling profiling adds event records to the stream; do not enable it for
 * graph capture.
 */
typedef struct {
  int64_t calls;            /* profiled hot-path calls                        */
  int64_t forward_launches; /* connected-configuration forward launches       */
  double  call_ms;          /* sum of call durations                          */
  double  eloc_ms;          /* sum of local-energy phase durations            */
  double  forward_ms;       /* sum of forward kernel durations                */
  double  forward_rows;     /* configurations evaluated by those launches     */
  double  forward_flops;    /* forward_rows * 2 * (unmasked weights per row)  */
  double  forward_flops_executed;  /* forward_rows * MFMA flops issued per row
                                      (masked tiles skipped, padding included;
                                      NQS_BF16X3 counts each of its BF16 MFMAs) */
} nqs_profile;
nqs_status nqs_plan_profile(nqs_plan* plan, int enable);
nqs_status nqs_plan_profile_read(nqs_plan* plan, void* d_ws, nqs_profile* out);

/* Synchronises the context's stream, reads the device error word of the
   workspace d_ws into *flags (NQS_DEV_* bits) and clears it.  Not for use
   inside graph capture. */
nqs_status nqs_device_status(nqs_ctx* ctx, void* d_ws, uint32_t* flags);
/* The same for a multi-instance call's workspace d_ws: reads and clears the
   error word of every instance of inst (the list given to
   nqs_energy_grad_multi) and sets *flags to their bitwise or. */
nqs_status nqs_multi_device_status(int n_inst, const nqs_instance* inst, void* d_ws, uint32_t* flags);

#ifdef __cplusplus
}
#endif
#endif /* NQS_H */
