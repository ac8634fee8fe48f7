// Host side of the C ABI declared in include/nqs.h: argument checking,
// Hamiltonian canonicalisation, plans (network geometry, chunking,
// workspace layout) and the stream-ordered launch sequences of the hot path.
#include "../../include/nqs.h"
#include "nqs_internal.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

using namespace nqs;

namespace {

thread_local std::string g_last_error;

nqs_status fail(nqs_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(NQS_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));          \
  } while (0)

nqs_status launch_check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(NQS_ERR_HIP, "%s: kernel launch failed: %s", what, hipGetErrorString(e));
  return NQS_OK;
}

constexpr uint64_t kUpMask = 0x5555555555555555ull;
constexpr uint64_t kDnMask = 0xAAAAAAAAAAAAAAAAull;

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

double binom(int a, int b) {
  if (b < 0 || a < 0 || b > a) return 0.0;
  double r = 1.0;
  for (int i = 1; i <= b; ++i) r = r * (a - b + i) / i;
  return r;
}

}  // namespace

struct nqs_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int cu_count = 0;
};

struct nqs_ham {
  int n = 0;
  int words = 1;           // 64-bit words per mask
  bool has_imag = false;
  uint32_t flags = 0;
  std::vector<uint64_t> gx;   // [G][words]
  std::vector<long long> goff;
  std::vector<uint64_t> tz;   // [K][words]
  std::vector<double> tre, tim;
  long long max_gterms = 0;   // terms of the largest group past the empty flip
  // census of non-empty flips by (up bits, down bits) for the entry bound
  std::map<std::pair<int, int>, long long> census;
  // structured matrix elements (NQS_H_TABLES)
  bool tables = false;
  std::vector<long long> soff;   // [G+1]
  std::vector<uint64_t> su;      // [S][words]
  std::vector<long long> stab;   // [S]
  std::vector<double> tabre, tabim;
  std::vector<int8_t> fpos;      // [G][4]
  // device copy
  char* d_base = nullptr;
  size_t bytes = 0;
  size_t o_gx = 0, o_goff = 0, o_tz = 0, o_tre = 0, o_tim = 0;
  size_t o_soff = 0, o_su = 0, o_stab = 0, o_tabre = 0, o_tabim = 0, o_fpos = 0;
};

// Tables of the structured matrix elements of group g (the flip's qubits,
// sub-groups by off-flip z mask in order of first appearance, one 2^m-entry
// table each, summed in canonical order).  False if the flip has more than
// four qubits.
static bool build_group_tables(nqs_ham* h, size_t g) {
  const int W = h->words;
  const uint64_t* f = &h->gx[g * W];
  int8_t pos[4] = {-1, -1, -1, -1};
  int m = 0;
  for (int w = 0; w < W; ++w)
    for (int b = 0; b < 64; ++b)
      if ((f[w] >> b) & 1ull) {
        if (m == 4) return false;
        pos[m++] = (int8_t)(64 * w + b);
      }
  for (int j = 0; j < 4; ++j) h->fpos.push_back(pos[j]);
  const long long k0 = h->goff[g], k1 = h->goff[g + 1];
  const long long s0 = (long long)h->stab.size();
  std::vector<std::array<uint64_t, 2>> seen;
  std::vector<long long> sub_of(k1 - k0);
  for (long long k = k0; k < k1; ++k) {
    std::array<uint64_t, 2> u{0, 0};
    for (int w = 0; w < W; ++w) u[w] = h->tz[k * W + w] & ~f[w];
    size_t s = 0;
    while (s < seen.size() && seen[s] != u) ++s;
    if (s == seen.size()) seen.push_back(u);
    sub_of[k - k0] = (long long)s;
  }
  const int E = 1 << m;
  for (size_t s = 0; s < seen.size(); ++s) {
    h->stab.push_back((long long)h->tabre.size());
    for (int w = 0; w < W; ++w) h->su.push_back(seen[s][w]);
    for (int b = 0; b < E; ++b) {
      // x's bits at the flip's qubits, spread back to their positions
      uint64_t xb[2] = {0, 0};
      for (int j = 0; j < m; ++j)
        if ((b >> j) & 1) xb[pos[j] >> 6] |= 1ull << (pos[j] & 63);
      double re = 0.0, im = 0.0;
      for (long long k = k0; k < k1; ++k) {
        if (sub_of[k - k0] != (long long)s) continue;
        int par = 0;
        for (int w = 0; w < W; ++w) par += __builtin_popcountll(xb[w] & h->tz[k * W + w] & f[w]);
        const double sg = (par & 1) ? -1.0 : 1.0;
        re += sg * h->tre[k];
        im += sg * h->tim[k];
      }
      h->tabre.push_back(re);
      h->tabim.push_back(im);
    }
  }
  h->soff.push_back(s0 + (long long)seen.size());
  return true;
}

struct nqs_plan {
  nqs_ctx* ctx = nullptr;
  const nqs_ham* ham = nullptr;
  Geom g{};
  int64_t max_batch = 0;
  int64_t S = 0;           // samples per chunk (tunable, <= S0)
  int64_t S0 = 0;          // samples per chunk the workspace is sized for
  int64_t SRcap = 0;       // capacity of the (sample, group range) count arrays
  int64_t Emax = 0;        // entries per sample bound
  int64_t EC = 0;          // entries per chunk capacity (S0 * Emax)
  int R = 1, gper = 0;     // group ranges of the enumeration grid for S
  bool dedup = false;      // dedup on for this plan's calls
  bool dedup_cap = false;  // workspace holds the dedup tables
  bool lookback = false;   // with dedup: a chunk reuses the previous chunk's log psi (one-word keys below 64 qubits)
  bool dedup_auto = false; // the autotuner may switch dedup
  int variant = 0;         // forward kernel variant
  bool resident = false;   // forward grid: resident workgroups looping over tiles
  bool tuned = false;
  int64_t HT = 0;          // dedup hash slots
  int64_t Sb = 0;          // backward chunk
  int bw = 4;              // bytes per element of the backward path
  Geom gp{};               // the separate phase network (phase_mode 1)
  bool two = false;        // phase_mode 1: modulus network g and phase network gp
  size_t packed_bytes = 0; // packed weights of g, then (two) of gp at packed_phase
  size_t packed_phase = 0;
  double flops_alg_row = 0, flops_exec_row = 0;   // forward flops per configuration
  // profiling
  struct Rec { hipEvent_t a, b; int kind; int slot; };   // kind 0 call, 1 eloc, 2 forward
  bool prof = false;
  std::vector<Rec> recs;
  int next_slot = 0;
};

constexpr int kProfSlots = 8192;

struct WsLayout {
  size_t err, prof, geom, packed, wm, lps, eloc, energy, cnt, off, stmp, rpart, diag, xe, he, lpe, htab,
      eu, xu, nu, dfirst, drank, drtmp, htab2, lp2, lpn, src, nnew, bscratch, total;
};

// Enumeration grid for chunks of S samples: R ranges of gper flip groups.
static void grid_for(int64_t S, int ngroups, int& R, int& gper) {
  const int bx = (int)((S + 255) / 256);
  if (ngroups <= 0) { R = 1; gper = 0; return; }
  const int r = std::max(1, std::min(ngroups, 2048 / bx));
  gper = (ngroups + r - 1) / r;
  R = (ngroups + gper - 1) / gper;
}

static WsLayout layout(const nqs_plan* p, int64_t B) {
  WsLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
  const int hs = p->ham->has_imag ? 2 : 1;
  L.err = take(256);
  L.prof = take((size_t)kProfSlots * 8);
  L.geom = take(2 * sizeof(Geom));
  L.packed = take(p->packed_bytes);
  L.wm = take((size_t)p->g.n_params * p->bw);
  L.lps = take((size_t)std::max<int64_t>(B, 1) * 16);
  L.eloc = take((size_t)std::max<int64_t>(B, 1) * 16);
  L.energy = take(3 * 8);
  L.cnt = take((size_t)p->SRcap * 4);
  L.off = take(((size_t)p->SRcap + 1) * 8);
  L.stmp = take(((size_t)scan_tiles(p->SRcap) + 1) * 8);
  L.rpart = take((size_t)reduce_partials_elems(std::max<int64_t>(p->S0, 1)) * 8);
  L.diag = take((size_t)p->S0 * 16);
  L.xe = take((size_t)p->EC * 8 * p->g.words);
  L.he = take((size_t)p->EC * 8 * hs);
  L.lpe = take((size_t)p->EC * 16);
  if (p->dedup_cap) {
    L.htab = take((size_t)p->HT * kHashRecBytes);
    L.eu = take((size_t)p->EC * 4);
    L.xu = take((size_t)p->EC * 8 * p->g.words);
    L.nu = take(8);
    L.dfirst = take((size_t)p->EC * 4);
    L.drank = take(((size_t)p->EC + 1) * 8);
    L.drtmp = take((size_t)dedup_rank_tmp_elems(p->EC) * 8);
    if (p->lookback) {   // the second table and log psi set, the new rows' log psi, the look-back map
      L.htab2 = take((size_t)p->HT * kHashRecBytes);
      L.lp2 = take((size_t)p->EC * 16);
      L.lpn = take((size_t)p->EC * 16);
      L.src = take((size_t)p->EC * 4);
      L.nnew = take(8);
    }
  }
  L.bscratch = take((size_t)backward_scratch_elems(p->g, p->Sb) * p->bw);
  L.total = o;
  return L;
}

// group 0 is the empty flip
static bool ham_has_diag(const nqs_ham* h) {
  if (h->gx.empty()) return false;
  for (int w = 0; w < h->words; ++w)
    if (h->gx[w] != 0) return false;
  return true;
}

static HamDev ham_dev(const nqs_plan* p) {
  const nqs_ham* h = p->ham;
  HamDev H{};
  H.gx = (const uint64_t*)(h->d_base + h->o_gx);
  H.goff = (const long long*)(h->d_base + h->o_goff);
  H.tz = (const uint64_t*)(h->d_base + h->o_tz);
  H.tre = (const double*)(h->d_base + h->o_tre);
  H.tim = h->has_imag ? (const double*)(h->d_base + h->o_tim) : nullptr;
  H.G = (int)(h->gx.size() / h->words);
  H.gfirst = ham_has_diag(h) ? 1 : 0;
  H.filter = (h->flags & NQS_H_CONSERVES_SPIN_SECTORS) ? 1 : 0;
  H.words = h->words;
  H.max_gterms = h->max_gterms;
  H.tables = h->tables ? 1 : 0;
  if (h->tables) {
    H.soff = (const long long*)(h->d_base + h->o_soff);
    H.su = (const uint64_t*)(h->d_base + h->o_su);
    H.stab = (const long long*)(h->d_base + h->o_stab);
    H.tabre = (const double*)(h->d_base + h->o_tabre);
    H.tabim = h->has_imag ? (const double*)(h->d_base + h->o_tabim) : nullptr;
    H.fpos = (const int8_t*)(h->d_base + h->o_fpos);
  }
  return H;
}

extern "C" {

const char* nqs_status_str(int s) {
  switch (s) {
    case NQS_OK: return "ok";
    case NQS_ERR_INVALID_ARGUMENT: return "invalid argument";
    case NQS_ERR_UNSUPPORTED: return "unsupported";
    case NQS_ERR_NOT_HERMITIAN: return "non-real Pauli coefficient";
    case NQS_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case NQS_ERR_HIP: return "HIP runtime error";
    case NQS_ERR_DEVICE: return "device error flag set";
  }
  return "unknown status";
}

size_t nqs_last_error(char* buf, size_t len) {
  if (buf && len) {
    size_t n = std::min(len - 1, g_last_error.size());
    memcpy(buf, g_last_error.data(), n);
    buf[n] = 0;
  }
  return g_last_error.size();
}

int nqs_version(void) { return 100; }

#ifndef NQS_SOURCE_HASH
#define NQS_SOURCE_HASH "unknown"
#endif
const char* nqs_source_hash(void) { return NQS_SOURCE_HASH; }

// Workspace of the allocation-free entry point: one array per device, whose
// address hipGetSymbolAddress gives once per device at context creation (in
// host code the array's name is not a device address).
static __device__ __align__(256) unsigned char scratch[NQS_NOALLOC_SCRATCH_BYTES];
namespace {
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;   // device -> that device's copy of scratch

// with `device` current
nqs_status scratch_attach(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr.count(device)) return NQS_OK;
  void* ptr = nullptr;
  HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr || ((uintptr_t)ptr & 255)) return fail(NQS_ERR_HIP, "scratch array of device %d at %p", device, ptr);
  g_scratch_ptr[device] = ptr;
  return NQS_OK;
}

__global__ void copy_flags_kernel(const unsigned* src, unsigned* dst) { *dst = *src; }
}  // namespace

nqs_status nqs_ctx_create(int device, void* stream, nqs_ctx** out) {
  if (!out) return fail(NQS_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  int count = 0;
  HIP_TRY(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(NQS_ERR_INVALID_ARGUMENT, "device %d of %d", device, count);
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device));
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(NQS_ERR_UNSUPPORTED, "device arch %s is not gfx950", prop.gcnArchName);
  HIP_TRY(hipSetDevice(device));
  const nqs_status sa = scratch_attach(device);
  if (sa != NQS_OK) return sa;
  nqs_ctx* c = new nqs_ctx;
  c->device = device;
  c->stream = (hipStream_t)stream;
  c->cu_count = prop.multiProcessorCount;
  *out = c;
  return NQS_OK;
}

nqs_status nqs_ctx_set_stream(nqs_ctx* ctx, void* stream) {
  if (!ctx) return fail(NQS_ERR_INVALID_ARGUMENT, "ctx is NULL");
  ctx->stream = (hipStream_t)stream;
  return NQS_OK;
}

void nqs_ctx_destroy(nqs_ctx* ctx) { delete ctx; }

// ------------------------------------------------------------ Hamiltonian
nqs_status nqs_ham_create(const nqs_pauli_terms* t, nqs_ham** out) {
  if (!t || !out) return fail(NQS_ERR_INVALID_ARGUMENT, "NULL argument");
  *out = nullptr;
  if (t->n_qubits < 1 || t->n_qubits > kMaxQubits)
    return fail(NQS_ERR_UNSUPPORTED, "n_qubits = %d outside 1..%d", t->n_qubits, kMaxQubits);
  if (t->n_terms < 0) return fail(NQS_ERR_INVALID_ARGUMENT, "n_terms < 0");
  if (t->n_terms > 0 && (!t->x_mask || !t->z_mask || !t->coeff))
    return fail(NQS_ERR_INVALID_ARGUMENT, "NULL term arrays");
  if (!(t->drop_tol >= 0.0)) return fail(NQS_ERR_INVALID_ARGUMENT, "drop_tol must be >= 0");
  if (t->flags & ~(NQS_H_CONSERVES_SPIN_SECTORS | NQS_H_TABLES))
    return fail(NQS_ERR_INVALID_ARGUMENT, "unknown Hamiltonian flags 0x%x", t->flags);
  const int W = (t->n_qubits + 63) / 64;
  // valid bits of each word
  uint64_t valid[2] = {0, 0};
  for (int w = 0; w < W; ++w) {
    const int bits = std::min(64, t->n_qubits - 64 * w);
    valid[w] = bits == 64 ? ~0ull : ((1ull << bits) - 1);
  }
  for (int64_t k = 0; k < t->n_terms; ++k) {
    for (int w = 0; w < W; ++w)
      if ((t->x_mask[k * W + w] | t->z_mask[k * W + w]) & ~valid[w])
        return fail(NQS_ERR_INVALID_ARGUMENT, "term %lld acts on a qubit >= n_qubits", (long long)k);
    if (!std::isfinite(t->coeff[k])) return fail(NQS_ERR_INVALID_ARGUMENT, "term %lld: non-finite coefficient", (long long)k);
    if (t->coeff_imag && t->coeff_imag[k] != 0.0)
      return fail(NQS_ERR_NOT_HERMITIAN, "term %lld has imaginary coefficient %g", (long long)k, t->coeff_imag[k]);
  }
  // a string as (x high, x low, z high, z low): the tuple order is the order
  // of (x, z) as unsigned integers
  using Key = std::array<uint64_t, 4>;
  auto key_of = [&](int64_t k) {
    Key key{0, 0, 0, 0};
    for (int w = 0; w < W; ++w) {
      key[1 - w] = t->x_mask[k * W + w];
      key[3 - w] = t->z_mask[k * W + w];
    }
    return key;
  };
  // 1. merge identical strings, sequential FP64 sums in input order
  struct KeyHash {
    size_t operator()(const Key& k) const {
      uint64_t v = 0;
      for (uint64_t e : k) v = (v ^ e) * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
      return std::hash<uint64_t>()(v);
    }
  };
  std::unordered_map<Key, size_t, KeyHash> idx;
  idx.reserve((size_t)t->n_terms * 2 + 1);
  std::vector<Key> keys;
  std::vector<double> vals;
  for (int64_t k = 0; k < t->n_terms; ++k) {
    const Key key = key_of(k);
    auto it = idx.find(key);
    if (it == idx.end()) {
      idx.emplace(key, keys.size());
      keys.push_back(key);
      vals.push_back(t->coeff[k]);
    } else {
      vals[it->second] = vals[it->second] + t->coeff[k];
    }
  }
  // 2. drop, 5. sort
  std::vector<size_t> ord;
  for (size_t i = 0; i < keys.size(); ++i)
    if (std::fabs(vals[i]) >= t->drop_tol) ord.push_back(i);
  std::sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return keys[a] < keys[b]; });
  nqs_ham* h = new nqs_ham;
  h->n = t->n_qubits;
  h->words = W;
  h->flags = t->flags;
  const size_t K = ord.size();
  h->tz.resize(K * W);
  h->tre.resize(K);
  h->tim.resize(K);
  for (size_t j = 0; j < K; ++j) {
    const Key& key = keys[ord[j]];
    const double c = vals[ord[j]];
    for (int w = 0; w < W; ++w) h->tz[j * W + w] = key[3 - w];
    // 4. fold (-i)^r, r = number of Y factors
    const int r = __builtin_popcountll(key[0] & key[2]) + __builtin_popcountll(key[1] & key[3]);
    switch (r & 3) {
      case 0: h->tre[j] = c; h->tim[j] = 0.0; break;
      case 1: h->tre[j] = 0.0; h->tim[j] = -c; h->has_imag = true; break;
      case 2: h->tre[j] = -c; h->tim[j] = 0.0; break;
      default: h->tre[j] = 0.0; h->tim[j] = c; h->has_imag = true; break;
    }
    if (j == 0 || key[0] != keys[ord[j - 1]][0] || key[1] != keys[ord[j - 1]][1]) {
      for (int w = 0; w < W; ++w) h->gx.push_back(key[1 - w]);
      h->goff.push_back((long long)j);
    }
  }
  h->goff.push_back((long long)K);
  const size_t G = h->gx.size() / W;
  for (size_t gi = ham_has_diag(h) ? 1 : 0; gi < G; ++gi)
    h->max_gterms = std::max(h->max_gterms, h->goff[gi + 1] - h->goff[gi]);
  for (size_t gi = 0; gi < G; ++gi) {
    int up = 0, dn = 0;
    for (int w = 0; w < W; ++w) {
      // 64 is even, so every word has the same spin pattern
      up += __builtin_popcountll(h->gx[gi * W + w] & kUpMask);
      dn += __builtin_popcountll(h->gx[gi * W + w] & kDnMask);
    }
    if (up + dn == 0) continue;
    h->census[{up, dn}] += 1;
  }
  if (t->flags & NQS_H_TABLES) {
    h->tables = true;
    h->soff.push_back(0);
    for (size_t gi = 0; gi < G; ++gi) {
      if (!build_group_tables(h, gi)) {
        delete h;
        return fail(NQS_ERR_UNSUPPORTED, "group %zu flips more than 4 qubits: no tables", gi);
      }
    }
  }
  // device layout
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
  h->o_gx = take(h->gx.size() * 8);
  h->o_goff = take(h->goff.size() * 8);
  h->o_tz = take(K * W * 8);
  h->o_tre = take(K * 8);
  h->o_tim = h->has_imag ? take(K * 8) : 0;
  if (h->tables) {
    h->o_soff = take(h->soff.size() * 8);
    h->o_su = take(h->su.size() * 8);
    h->o_stab = take(h->stab.size() * 8);
    h->o_tabre = take(h->tabre.size() * 8);
    h->o_tabim = h->has_imag ? take(h->tabim.size() * 8) : 0;
    h->o_fpos = take(h->fpos.size());
  }
  h->bytes = std::max<size_t>(o, 256);
  *out = h;
  return NQS_OK;
}

nqs_status nqs_ham_info(const nqs_ham* h, int64_t* K, int64_t* G, size_t* bytes, int* has_imag, int* n) {
  if (!h) return fail(NQS_ERR_INVALID_ARGUMENT, "ham is NULL");
  if (K) *K = (int64_t)h->tre.size();
  if (G) *G = (int64_t)(h->gx.size() / h->words);
  if (bytes) *bytes = h->bytes;
  if (has_imag) *has_imag = h->has_imag ? 1 : 0;
  if (n) *n = h->n;
  return NQS_OK;
}

nqs_status nqs_ham_upload(nqs_ham* h, nqs_ctx* ctx, void* d_storage, size_t bytes) {
  if (!h || !ctx || !d_storage) return fail(NQS_ERR_INVALID_ARGUMENT, "NULL argument");
  if (bytes < h->bytes) return fail(NQS_ERR_WORKSPACE_TOO_SMALL, "storage %zu < %zu bytes", bytes, h->bytes);
  if (((uintptr_t)d_storage) & 255) return fail(NQS_ERR_INVALID_ARGUMENT, "storage not 256-byte aligned");
  char* d = (char*)d_storage;
  hipStream_t s = ctx->stream;
  if (!h->gx.empty()) HIP_TRY(hipMemcpyAsync(d + h->o_gx, h->gx.data(), h->gx.size() * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d + h->o_goff, h->goff.data(), h->goff.size() * 8, hipMemcpyHostToDevice, s));
  if (!h->tz.empty()) {
    HIP_TRY(hipMemcpyAsync(d + h->o_tz, h->tz.data(), h->tz.size() * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d + h->o_tre, h->tre.data(), h->tre.size() * 8, hipMemcpyHostToDevice, s));
    if (h->has_imag)
      HIP_TRY(hipMemcpyAsync(d + h->o_tim, h->tim.data(), h->tim.size() * 8, hipMemcpyHostToDevice, s));
  }
  if (h->tables) {
    auto put = [&](size_t off, const void* src, size_t n) {
      return n ? hipMemcpyAsync(d + off, src, n, hipMemcpyHostToDevice, s) : hipSuccess;
    };
    HIP_TRY(put(h->o_soff, h->soff.data(), h->soff.size() * 8));
    HIP_TRY(put(h->o_su, h->su.data(), h->su.size() * 8));
    HIP_TRY(put(h->o_stab, h->stab.data(), h->stab.size() * 8));
    HIP_TRY(put(h->o_tabre, h->tabre.data(), h->tabre.size() * 8));
    if (h->has_imag) HIP_TRY(put(h->o_tabim, h->tabim.data(), h->tabim.size() * 8));
    HIP_TRY(put(h->o_fpos, h->fpos.data(), h->fpos.size()));
  }
  HIP_TRY(hipStreamSynchronize(s));
  h->d_base = d;
  return NQS_OK;
}

nqs_status nqs_ham_export(const nqs_ham* h, uint64_t* gx, int64_t* goff, uint64_t* tz, double* tre, double* tim) {
  if (!h) return fail(NQS_ERR_INVALID_ARGUMENT, "ham is NULL");
  if (gx) std::copy(h->gx.begin(), h->gx.end(), gx);
  if (goff) for (size_t i = 0; i < h->goff.size(); ++i) goff[i] = (int64_t)h->goff[i];
  if (tz) std::copy(h->tz.begin(), h->tz.end(), tz);
  if (tre) std::copy(h->tre.begin(), h->tre.end(), tre);
  if (tim) std::copy(h->tim.begin(), h->tim.end(), tim);
  return NQS_OK;
}

nqs_status nqs_ham_table_info(const nqs_ham* h, int64_t* S, int64_t* E) {
  if (!h) return fail(NQS_ERR_INVALID_ARGUMENT, "ham is NULL");
  if (S) *S = (int64_t)h->stab.size();
  if (E) *E = (int64_t)h->tabre.size();
  return NQS_OK;
}

nqs_status nqs_ham_export_tables(const nqs_ham* h, int64_t* soff, uint64_t* su, int64_t* stab, double* tab_re,
                                 double* tab_im, int8_t* fpos) {
  if (!h) return fail(NQS_ERR_INVALID_ARGUMENT, "ham is NULL");
  if (soff) for (size_t i = 0; i < h->soff.size(); ++i) soff[i] = (int64_t)h->soff[i];
  if (su) std::copy(h->su.begin(), h->su.end(), su);
  if (stab) for (size_t i = 0; i < h->stab.size(); ++i) stab[i] = (int64_t)h->stab[i];
  if (tab_re) std::copy(h->tabre.begin(), h->tabre.end(), tab_re);
  if (tab_im) std::copy(h->tabim.begin(), h->tabim.end(), tab_im);
  if (fpos) std::copy(h->fpos.begin(), h->fpos.end(), fpos);
  return NQS_OK;
}

void nqs_ham_destroy(nqs_ham* h) { delete h; }

// ---------------------------------------------------------------- network
static nqs_status build_geom(const nqs_net_desc* nd, Geom& g) {
  if (!nd) return fail(NQS_ERR_INVALID_ARGUMENT, "net is NULL");
  const int n = nd->n_qubits, L = nd->n_layers, h = nd->width;
  if (n < 2 || n > kMaxQubits) return fail(NQS_ERR_UNSUPPORTED, "n_qubits = %d outside 2..%d", n, kMaxQubits);
  if (L < 1 || L > kMaxLayers) return fail(NQS_ERR_UNSUPPORTED, "n_layers = %d outside 1..%d", L, kMaxLayers);
  if (nd->precision < NQS_FP64 || nd->precision > NQS_BF16W)
    return fail(NQS_ERR_INVALID_ARGUMENT, "unknown precision %d", nd->precision);
  const int words = n > 64 ? 2 : 1;
  if (!forward_supported(nd->precision, h, words))
    return fail(NQS_ERR_UNSUPPORTED, "width %d not supported for precision %d at %d qubits", h, nd->precision, n);
  if (nd->phase_mode != 0 && nd->phase_mode != 1)
    return fail(NQS_ERR_INVALID_ARGUMENT, "phase_mode %d is neither 0 nor 1", nd->phase_mode);
  if (nd->phase_mode == 1 && n < 3)
    return fail(NQS_ERR_UNSUPPORTED, "a separate phase network needs n_qubits >= 3");
  const bool cons = nd->n_up >= 0 || nd->n_dn >= 0;
  if (cons && (nd->n_up < 0 || nd->n_dn < 0 || nd->n_up > (n + 1) / 2 || nd->n_dn > n / 2))
    return fail(NQS_ERR_INVALID_ARGUMENT, "invalid sector (%d, %d)", nd->n_up, nd->n_dn);
  memset(&g, 0, sizeof(g));
  g.n = n; g.L = L; g.h = h; g.prec = nd->precision;
  g.n_up = cons ? nd->n_up : -1;
  g.n_dn = cons ? nd->n_dn : -1;
  std::vector<int> order(n), seen(n, 0);
  for (int t = 0; t < n; ++t) {
    order[t] = nd->order ? nd->order[t] : n - 1 - t;
    if (order[t] < 0 || order[t] >= n || seen[order[t]]++)
      return fail(NQS_ERR_INVALID_ARGUMENT, "order is not a permutation of the qubits");
  }
  bool ident = true, rev = true;
  g.words = words;
  for (int t = 0; t < n; ++t) {
    g.order[t] = (int8_t)order[t];
    g.pos[order[t]] = (int8_t)t;
    if (t < 64) g.spin_pos[order[t] & 1] |= 1ull << t;
    else g.spin_pos_hi[order[t] & 1] |= 1ull << (t - 64);
    ident = ident && order[t] == t;
    rev = rev && order[t] == n - 1 - t;
  }
  g.order_kind = ident ? 1 : (rev ? 2 : 0);
  g.phase_mode = nd->phase_mode;
  g.net_kind = nd->phase_mode == 1 ? 1 : 0;
  g.TB = g.prec == P_F64 ? 16 : 32;
  g.KSTEP = (g.prec == P_BF16 || g.prec == P_BF16X3 || g.prec == P_BF16W) ? 16 : 8;
  g.NB = h / g.TB;
  g.nhead = n + 4;
  g.NHB = (g.nhead + g.TB - 1) / g.TB;
  if (g.NB > kMaxNB || g.NHB > kMaxNHB) return fail(NQS_ERR_UNSUPPORTED, "network too wide");
  if (h >= n - 1) { g.q = h / (n - 1); g.r = h % (n - 1); }
  else { g.q = 0; g.r = h; }
  g.planes = g.prec == P_BF16X3 ? 2 : 1;
  g.acc_bytes = g.prec == P_F64 ? 8 : 4;
  // k steps per block, rounded up to an even count (the fused kernel steps by
  // two); the extra fragments hold masked (zero) weights.
  auto ceil_div = [](int a, int b) { return (((a + b - 1) / b) + 1) & ~1; };
  g.off1[0] = g.offh[0] = g.offo[0] = 0;
  for (int nb = 0; nb < g.NB; ++nb) {
    const int ulast = std::min(h, g.TB * (nb + 1)) - 1;
    const int c = class_of_sorted(g, ulast);
    const int kend1 = std::min(c + 1, n);
    const int kendh = prefix_of_class(g, c + 1);
    g.ks1[nb] = ceil_div(kend1, g.KSTEP);
    g.ksh[nb] = ceil_div(kendh, g.KSTEP);
    g.off1[nb + 1] = g.off1[nb] + g.ks1[nb];
    g.offh[nb + 1] = g.offh[nb] + g.ksh[nb];
  }
  for (int nb = 0; nb < g.NHB; ++nb) {
    int kend = 0;
    // (the phase rows of the modulus network of phase_mode 1 are zero and read nothing)
    for (int t = g.TB * nb; t < std::min(g.TB * (nb + 1), g.nhead); ++t)
      if (t < n || g.net_kind == 0) kend = std::max(kend, t < n ? prefix_of_class(g, t) : prefix_of_class(g, n - 2));
    g.kso[nb] = (((kend + g.KSTEP - 1) / g.KSTEP) + 7) & ~7;   // head: multiples of 8 steps
    g.offo[nb + 1] = g.offo[nb] + g.kso[nb];
  }
  g.frag_h = g.off1[g.NB];
  g.frag_head = g.frag_h + (long long)(L - 1) * g.offh[g.NB];
  g.nfrag = g.frag_head + g.offo[g.NHB];
  g.bias_byte = (long long)align256((size_t)g.nfrag * 1024 * g.planes);
  g.head_bias_off = (long long)L * h;
  long long o = 0;
  for (int l = 0; l < L; ++l) {
    const int in = l == 0 ? n : h;
    g.poff[2 * l] = o; o += (long long)h * in;
    g.poff[2 * l + 1] = o; o += h;
  }
  g.poff[2 * L] = o; o += (long long)n * h;
  g.poff[2 * L + 1] = o; o += n;
  if (g.phase_mode == 1) {
    for (int l = 1; l <= L; ++l) {
      const int in = l == 1 ? n - 2 : h;
      g.poff[poff_phase_layer(g, l)] = o; o += (long long)h * in;
      g.poff[poff_phase_layer(g, l) + 1] = o; o += h;
    }
  }
  g.poff[poff_phase_head(g)] = o; o += 4LL * h;
  g.poff[poff_phase_head(g) + 1] = o; o += 4;
  g.n_params = o;
  return NQS_OK;
}

// Geometry of the separate phase network of a phase_mode 1 model (net_kind 2):
// dense layers of width h over the first n-2 positions, a 4-row head, units
// in their own order.  Same precision, tile shape and sampling order as the
// modulus network gm, whose parameter offsets it shares.
static void build_phase_geom(const Geom& gm, Geom& g) {
  g = gm;
  g.net_kind = 2;
  g.nhead = 4;
  g.NHB = 1;
  const int KS = g.h / g.KSTEP;
  const int k1 = ((((g.n - 2) + g.KSTEP - 1) / g.KSTEP) + 1) & ~1;   // even, as in the modulus network
  const int kh = (KS + 1) & ~1;
  g.off1[0] = g.offh[0] = g.offo[0] = 0;
  for (int nb = 0; nb < g.NB; ++nb) {
    g.ks1[nb] = k1;
    g.ksh[nb] = kh;
    g.off1[nb + 1] = g.off1[nb] + k1;
    g.offh[nb + 1] = g.offh[nb] + kh;
  }
  for (int nb = g.NB; nb < kMaxNB; ++nb) g.ks1[nb] = g.ksh[nb] = 0;
  g.kso[0] = (KS + 7) & ~7;
  g.offo[1] = g.kso[0];
  for (int nb = 1; nb < kMaxNHB; ++nb) g.kso[nb] = 0;
  g.frag_h = g.off1[g.NB];
  g.frag_head = g.frag_h + (long long)(g.L - 1) * g.offh[g.NB];
  g.nfrag = g.frag_head + g.offo[1];
  g.bias_byte = (long long)align256((size_t)g.nfrag * 1024 * g.planes);
  g.head_bias_off = (long long)g.L * g.h;
}

static size_t packed_bytes_of(const Geom& g) {
  return (size_t)g.bias_byte + ((size_t)g.L * g.h + (size_t)g.NHB * g.TB) * g.acc_bytes;
}

nqs_status nqs_net_param_count(const nqs_net_desc* nd, int64_t* n_params) {
  Geom g;
  nqs_status s = build_geom(nd, g);
  if (s != NQS_OK) return s;
  if (n_params) *n_params = g.n_params;
  return NQS_OK;
}

// -------------------------------------------------------------------- plan
nqs_status nqs_plan_create(nqs_ctx* ctx, const nqs_ham* ham, const nqs_net_desc* nd, int64_t max_batch,
                           uint32_t flags, int64_t chunk_samples, nqs_plan** out) {
  if (!ctx || !ham || !out) return fail(NQS_ERR_INVALID_ARGUMENT, "NULL argument");
  *out = nullptr;
  if (max_batch < 1) return fail(NQS_ERR_INVALID_ARGUMENT, "max_batch must be >= 1");
  const uint32_t dflags = flags & (NQS_PLAN_DEDUP_ON | NQS_PLAN_DEDUP_OFF | NQS_PLAN_DEDUP_AUTO);
  if (dflags & (dflags - 1)) return fail(NQS_ERR_INVALID_ARGUMENT, "more than one of DEDUP_ON/OFF/AUTO");
  if (flags & ~(NQS_PLAN_DEDUP_ON | NQS_PLAN_DEDUP_OFF | NQS_PLAN_DEDUP_AUTO))
    return fail(NQS_ERR_INVALID_ARGUMENT, "unknown plan flags 0x%x", flags);
  Geom g;
  nqs_status st = build_geom(nd, g);
  if (st != NQS_OK) return st;
  if (g.n != ham->n) return fail(NQS_ERR_INVALID_ARGUMENT, "network has %d qubits, Hamiltonian %d", g.n, ham->n);
  if (!ham->d_base) return fail(NQS_ERR_INVALID_ARGUMENT, "Hamiltonian not uploaded");
  nqs_plan* p = new nqs_plan;
  p->ctx = ctx;
  p->ham = ham;
  p->g = g;
  p->max_batch = max_batch;
  // per-sample entry bound
  const int G = (int)(ham->gx.size() / ham->words);
  const int gfirst = ham_has_diag(ham) ? 1 : 0;
  if (ham->flags & NQS_H_CONSERVES_SPIN_SECTORS) {
    const int Nu = (g.n + 1) / 2, Nd = g.n / 2;
    double bound = 0.0;
    for (const auto& kv : ham->census) {
      const int u = kv.first.first, d = kv.first.second;
      if ((u & 1) || (d & 1)) continue;
      double best = 0.0;
      for (int a = 0; a <= Nu; ++a) {
        if (g.n_up >= 0 && a != g.n_up) continue;
        for (int b = 0; b <= Nd; ++b) {
          if (g.n_dn >= 0 && b != g.n_dn) continue;
          best = std::max(best, binom(a, u / 2) * binom(Nu - a, u / 2) * binom(b, d / 2) * binom(Nd - b, d / 2));
        }
      }
      bound += std::min(best, (double)kv.second);
    }
    p->Emax = (int64_t)bound;
  } else {
    p->Emax = G - gfirst;
  }
  // entries per chunk: large chunks amortise the per-chunk launches and, with
  // samples in sampling order, let dedup find more shared configurations (at
  // 60 qubits the distinct fraction is 1/1.78 of a 3,670-sample chunk and
  // 1/1.98 of a 14,680-sample one).  2^30 entries keep every entry index, and
  // every slot of the 2^31-slot hash table, inside 32-bit signed integers; the
  // chunk's buffers then take ~80 GB at 60 qubits.
  const int64_t target = 1LL << 30;
  if (chunk_samples > 0) p->S = std::min<int64_t>(chunk_samples, max_batch);
  else p->S = std::max<int64_t>(1, std::min<int64_t>(max_batch, target / std::max<int64_t>(p->Emax, 1)));
  p->S0 = p->S;
  p->EC = std::max<int64_t>(p->S * p->Emax, 1);
  if (p->EC > target) {   // per-entry kernels index entries and hash slots in 32 bits
    delete p;
    return fail(NQS_ERR_UNSUPPORTED, "chunk of %lld entries exceeds 2^30", (long long)p->S * p->Emax);
  }
  const int ngroups = G - gfirst;
  grid_for(p->S, ngroups, p->R, p->gper);
  // count arrays sized for every chunk the autotuner may pick (S0, S0/2)
  {
    int r2 = 1, gp2 = 0;
    const int64_t half = std::max<int64_t>(1, p->S0 / 2);
    grid_for(half, ngroups, r2, gp2);
    p->SRcap = std::max<int64_t>(p->S0 * p->R, half * r2);
  }
  // a one-word table holds the keys themselves with all-ones as the empty
  // marker below 64 qubits; at exactly 64 qubits and for two-word strings the
  // table holds slot words (hash tag and inserting entry) instead
  p->dedup_cap = (flags & (NQS_PLAN_DEDUP_ON | NQS_PLAN_DEDUP_AUTO)) != 0;
  p->dedup = p->dedup_cap;
  p->dedup_auto = (flags & NQS_PLAN_DEDUP_AUTO) != 0 && p->dedup_cap;
  if (p->dedup_cap) {
    int64_t ht = 4096;
    while (ht < 2 * p->EC) ht <<= 1;
    p->HT = ht;
    p->lookback = g.words == 1 && g.n < 64;
  }
  p->Sb = std::min<int64_t>(max_batch, 4096);
  p->bw = g.prec == P_F64 ? 8 : 4;
  p->packed_bytes = packed_bytes_of(g);
  if (g.phase_mode == 1) {
    p->two = true;
    build_phase_geom(g, p->gp);
    p->packed_phase = align256(p->packed_bytes);
    p->packed_bytes = p->packed_phase + packed_bytes_of(p->gp);
  }
  {
    // unmasked weights per configuration (MADE masks) and MFMA work issued
    const int n = g.n, h = g.h;
    std::vector<int> m(h);
    for (int k = 0; k < h; ++k) m[k] = 1 + k % (n - 1);
    double nnz1 = 0, nnzh = 0, nnzo = 0, nnzp = 0;
    std::vector<long long> cnt_le(n + 1, 0);   // units with degree <= d
    for (int k = 0; k < h; ++k) cnt_le[m[k]] += 1;
    for (int d = 1; d <= n; ++d) cnt_le[d] += cnt_le[d - 1];
    for (int k = 0; k < h; ++k) {
      nnz1 += std::min(m[k], n);
      nnzh += (double)cnt_le[m[k]];
      if (m[k] <= n - 2 && !p->two) nnzp += 4;
    }
    for (int j = 0; j < n; ++j) nnzo += (double)cnt_le[j];   // d(j) = 1 + pos: units with m < d
    // separate phase network: dense (n-2) x h, (L-1) h x h, 4 x h
    const double nnz_phase = p->two ? (double)(n - 2) * h + (double)(g.L - 1) * h * h + 4.0 * h : 0.0;
    p->flops_alg_row = 2.0 * (nnz1 + (g.L - 1) * nnzh + nnzo + nnzp + nnz_phase);
    // fragments issued per configuration; split BF16 multiplies each with
    // three BF16 MFMAs, BF16 weights with two; one fewer in layer 1 (its +-1
    // inputs have no low part)
    long long fr1 = 0, fr = 0;
    for (int nb = 0; nb < g.NB; ++nb) {
      fr1 += g.ks1[nb];
      fr += (long long)(g.L - 1) * g.ksh[nb];
    }
    for (int nb = 0; nb < g.NHB; ++nb) fr += g.kso[nb];
    if (p->two) {
      const Geom& q = p->gp;
      for (int nb = 0; nb < q.NB; ++nb) {
        fr1 += q.ks1[nb];
        fr += (long long)(q.L - 1) * q.ksh[nb];
      }
      fr += q.kso[0];
    }
    const double mult = g.prec == P_BF16X3 ? 3.0 : (g.prec == P_BF16W ? 2.0 : 1.0);
    const double mult1 = mult > 1.0 ? mult - 1.0 : 1.0;
    p->flops_exec_row = 2.0 * g.TB * g.KSTEP * (mult1 * (double)fr1 + mult * (double)fr);
  }
  *out = p;
  return NQS_OK;
}

nqs_status nqs_plan_profile(nqs_plan* p, int enable) {
  if (!p) return fail(NQS_ERR_INVALID_ARGUMENT, "plan is NULL");
  p->prof = enable != 0;
  return NQS_OK;
}

nqs_status nqs_plan_profile_read(nqs_plan* p, void* ws, nqs_profile* out) {
  if (!p || !out) return fail(NQS_ERR_INVALID_ARGUMENT, "NULL argument");
  memset(out, 0, sizeof(*out));
  HIP_TRY(hipStreamSynchronize(p->ctx->stream));
  std::vector<long long> slots;
  if (p->next_slot > 0) {
    if (!ws) return fail(NQS_ERR_INVALID_ARGUMENT, "workspace is NULL");
    WsLayout L = layout(p, 0);
    slots.resize(std::min(p->next_slot, kProfSlots));
    HIP_TRY(hipMemcpy(slots.data(), (char*)ws + L.prof, slots.size() * 8, hipMemcpyDeviceToHost));
  }
  for (auto& r : p->recs) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
    if (r.kind == 0) { out->calls += 1; out->call_ms += ms; }
    else if (r.kind == 1) out->eloc_ms += ms;
    else if (r.kind == 3) { out->calls += 1; out->call_ms += ms; out->eloc_ms += ms; }
    else {
      out->forward_launches += 1;
      out->forward_ms += ms;
      if (r.slot >= 0 && r.slot < (int)slots.size()) out->forward_rows += (double)slots[r.slot];
    }
  }
  std::vector<hipEvent_t> evs;   // records may share their start event
  for (auto& r : p->recs) { evs.push_back(r.a); evs.push_back(r.b); }
  std::sort(evs.begin(), evs.end());
  evs.erase(std::unique(evs.begin(), evs.end()), evs.end());
  for (hipEvent_t e : evs) (void)hipEventDestroy(e);
  out->forward_flops = out->forward_rows * p->flops_alg_row;
  out->forward_flops_executed = out->forward_rows * p->flops_exec_row;
  p->recs.clear();
  p->next_slot = 0;
  return NQS_OK;
}

nqs_status nqs_plan_workspace_size(const nqs_plan* p, int64_t B, size_t* bytes) {
  if (!p || !bytes) return fail(NQS_ERR_INVALID_ARGUMENT, "NULL argument");
  if (B < 0 || B > p->max_batch) return fail(NQS_ERR_INVALID_ARGUMENT, "batch %lld outside 0..%lld", (long long)B, (long long)p->max_batch);
  *bytes = layout(p, B).total;
  return NQS_OK;
}

nqs_status nqs_plan_info(const nqs_plan* p, int64_t* eps, int64_t* chunk, int* dedup, int64_t* n_params) {
  if (!p) return fail(NQS_ERR_INVALID_ARGUMENT, "plan is NULL");
  if (eps) *eps = p->Emax;
  if (chunk) *chunk = p->S;
  if (dedup) *dedup = p->dedup ? 1 : 0;
  if (n_params) *n_params = p->g.n_params;
  return NQS_OK;
}

void nqs_plan_destroy(nqs_plan* p) { delete p; }

}  // extern "C"

// ------------------------------------------------------------ hot path
static nqs_status check_ws(const nqs_plan* p, int64_t B, void* ws, size_t ws_bytes, WsLayout& L) {
  if (!ws) return fail(NQS_ERR_INVALID_ARGUMENT, "workspace is NULL");
  if (((uintptr_t)ws) & 255) return fail(NQS_ERR_INVALID_ARGUMENT, "workspace not 256-byte aligned");
  if (B < 0 || B > p->max_batch) return fail(NQS_ERR_INVALID_ARGUMENT, "batch %lld outside 0..%lld", (long long)B, (long long)p->max_batch);
  L = layout(p, B);
  if (ws_bytes < L.total) return fail(NQS_ERR_WORKSPACE_TOO_SMALL, "workspace %zu < %zu bytes", ws_bytes, L.total);
  return NQS_OK;
}

template <typename T>
static T* at(void* ws, size_t off) { return (T*)((char*)ws + off); }

// Event pair on the plan's stream when profiling is on.
static hipEvent_t prof_mark(nqs_plan* p) {
  if (!p->prof) return nullptr;
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  (void)hipEventRecord(e, p->ctx->stream);
  return e;
}
static void prof_close(nqs_plan* p, hipEvent_t a, int kind, int slot) {
  if (!p->prof || !a) return;
  hipEvent_t b = prof_mark(p);
  if (b) p->recs.push_back({a, b, kind, slot});
}

// Packed weights of the plan's network(s) into the packed region.
static void pack_net(const nqs_plan* p, const float* params, void* packed, hipStream_t s) {
  launch_pack_fused(p->g, params, packed, s);
  if (p->two) launch_pack_fused(p->gp, params, (char*)packed + p->packed_phase, s);
}

// log psi of rows [0, min(*d_count, bound)) of x: one launch, or two (modulus
// network, then phase network over the same rows) for a separate phase network.
static void forward_net(const nqs_plan* p, const void* packed, const uint64_t* x, long long bound,
                        const long long* d_count, double* out, long long* slot, hipStream_t s) {
  const int cus = p->ctx->cu_count;
  launch_forward(p->g, p->variant, p->resident, cus, packed, x, bound, d_count, out, slot, s);
  if (p->two)
    launch_forward(p->gp, p->variant, p->resident, cus, (const char*)packed + p->packed_phase, x, bound, d_count,
                   out, nullptr, s);
}

static void forward_profiled(nqs_plan* p, void* ws, const WsLayout& L, const void* packed,
                             const uint64_t* x, long long bound, const long long* d_count, double* out) {
  hipEvent_t a = prof_mark(p);
  long long* slot = nullptr;
  int si = -1;
  if (p->prof && p->next_slot < kProfSlots) {
    si = p->next_slot++;
    slot = at<long long>(ws, L.prof) + si;
    launch_fill_u64(slot, 0ull, 1, p->ctx->stream);   // a launch with no tiles leaves it at zero rows
  }
  forward_net(p, packed, x, bound, d_count, out, slot, p->ctx->stream);
  prof_close(p, a, 2, si);
}

// The connected configurations of one chunk, ready for the forward.
struct ChunkFwd {
  const uint64_t* x;          // configurations to evaluate
  const long long* d_count;   // their number (device)
  long long bound;            // host bound on that number
  double* out;                // log psi of each
  double* lp;                 // log psi the reduce reads: per entry, or per distinct configuration with dedup
  bool gather;                // out holds only the configurations new to this chunk (look-back)
};

// Enumerate (and optionally deduplicate) the connected configurations of
// samples [c0, c0 + Sc), chunk k of the call.  With look-back, chunks
// alternate between two tables and two log psi sets: chunk k probes chunk
// k - 1's table for its distinct configurations and evaluates only those the
// previous chunk did not (each row's log psi depends on that row alone, so the
// reused values are the ones the forward would give).
static ChunkFwd enum_chunk(nqs_plan* p, const uint64_t* x, int64_t c0, int64_t Sc, int64_t k, void* ws,
                           const WsLayout& L) {
  hipStream_t s = p->ctx->stream;
  const HamDev H = ham_dev(p);
  const int hs = p->ham->has_imag ? 2 : 1;
  const uint64_t* xc = x + c0 * p->g.words;
  unsigned* err = at<unsigned>(ws, L.err);
  int* cnt = at<int>(ws, L.cnt);
  long long* off = at<long long>(ws, L.off);
  uint64_t* xe = at<uint64_t>(ws, L.xe);
  launch_diag(H, xc, Sc, at<double>(ws, L.diag), s);
  launch_count(H, xc, Sc, p->R, p->gper, cnt, s);
  launch_scan(cnt, Sc * p->R, off, at<long long>(ws, L.stmp), s);
  launch_write(H, xc, Sc, p->R, p->gper, off, p->EC, xe, at<double>(ws, L.he), nullptr, hs, err, s);
  const long long* d_total = off + Sc * p->R;
  const int64_t bound = std::min<int64_t>(Sc * p->Emax, p->EC);
  double* lpe = at<double>(ws, L.lpe);
  if (!p->dedup) return {xe, d_total, bound, lpe, lpe, false};
  uint64_t* xu = at<uint64_t>(ws, L.xu);
  long long* nu = at<long long>(ws, L.nu);
  const bool odd = p->lookback && (k & 1);
  double* lp = odd ? at<double>(ws, L.lp2) : lpe;
  launch_dedup(xe, p->g.words, p->g.n == 64, d_total, p->EC, at<void>(ws, odd ? L.htab2 : L.htab), p->HT, false,
               at<int>(ws, L.eu), xu, nu, at<int>(ws, L.dfirst), at<long long>(ws, L.drank),
               at<long long>(ws, L.drtmp), err, s);
  if (!p->lookback || k == 0) return {xu, nu, bound, lp, lp, false};
  // the entries are dead once deduplicated: xe takes the new configurations
  long long* nnew = at<long long>(ws, L.nnew);
  launch_lookback(xu, nu, p->EC, at<void>(ws, odd ? L.htab : L.htab2), p->HT, at<int>(ws, L.src),
                  at<int>(ws, L.dfirst), at<long long>(ws, L.drank), at<long long>(ws, L.drtmp), xe, nnew, s);
  return {xe, nnew, bound, at<double>(ws, L.lpn), lp, true};
}

// After the chunk's forward: with look-back, the distinct configurations' log
// psi from the previous chunk's set and the new rows.
static void finish_chunk(nqs_plan* p, const ChunkFwd& cf, void* ws, const WsLayout& L) {
  if (!cf.gather) return;
  const double* prev = cf.lp == at<double>(ws, L.lpe) ? at<double>(ws, L.lp2) : at<double>(ws, L.lpe);
  launch_lookback_gather(at<long long>(ws, L.nu), p->EC, at<int>(ws, L.src), at<long long>(ws, L.drank), prev,
                         cf.out, cf.lp, p->ctx->stream);
}

// Ratio-and-reduce of the chunk into eloc[c0 .. c0 + Sc).
static void reduce_chunk(nqs_plan* p, int64_t c0, int64_t Sc, const ChunkFwd& cf, void* ws, const WsLayout& L,
                         double* eloc) {
  const int hs = p->ham->has_imag ? 2 : 1;
  launch_reduce(Sc, p->R, at<long long>(ws, L.off), p->EC, at<double>(ws, L.diag), at<double>(ws, L.he), hs,
                p->dedup ? at<int>(ws, L.eu) : nullptr, cf.lp, at<double>(ws, L.lps) + 2 * c0, eloc + 2 * c0,
                at<double>(ws, L.rpart), at<unsigned>(ws, L.err), p->ctx->stream);
}

// local energies of B samples into eloc; lps (sample log psi) computed first.
static nqs_status run_local_energy(nqs_plan* p, const float* params, const uint64_t* x, int64_t B,
                                   double* eloc, void* ws, const WsLayout& L) {
  void* packed = at<void>(ws, L.packed);
  pack_net(p, params, packed, p->ctx->stream);
  forward_profiled(p, ws, L, packed, x, B, nullptr, at<double>(ws, L.lps));
  for (int64_t c0 = 0, k = 0; c0 < B; c0 += p->S, ++k) {
    const int64_t Sc = std::min<int64_t>(p->S, B - c0);
    const ChunkFwd cf = enum_chunk(p, x, c0, Sc, k, ws, L);
    forward_profiled(p, ws, L, packed, cf.x, cf.bound, cf.d_count, cf.out);
    finish_chunk(p, cf, ws, L);
    reduce_chunk(p, c0, Sc, cf, ws, L, eloc);
  }
  return launch_check("local energy");
}

// Energy (Eq. total_energy_sum) and gradient (Eq. grad) from the local
// energies el of B samples: the backward recomputes the sample forward in
// chunks of Sb samples and accumulates into grad.
static void energy_and_grad(nqs_plan* p, const float* params, const uint64_t* x, const double* w, int64_t B,
                            const double* el, double* energy, double* grad, void* ws, const WsLayout& L) {
  hipStream_t s = p->ctx->stream;
  launch_energy(el, w, B, energy, at<unsigned>(ws, L.err), s);
  launch_fill_u64(grad, 0ull, p->g.n_params, s);
  void* wm = at<void>(ws, L.wm);
  launch_pack_masked(p->g, params, wm, s);
  void* scratch = at<void>(ws, L.bscratch);
  for (int64_t c0 = 0; c0 < B; c0 += p->Sb) {
    const int64_t Sc = std::min<int64_t>(p->Sb, B - c0);
    launch_backward(p->g, wm, x + c0 * p->g.words, Sc, el + 2 * c0, w ? w + c0 : nullptr, energy, scratch, grad, s);
  }
}

extern "C" {

nqs_status nqs_log_psi(nqs_plan* p, const float* params, const uint64_t* x, int64_t n, double* out,
                       void* ws, size_t ws_bytes) {
  if (!p || !params || (n > 0 && (!x || !out))) return fail(NQS_ERR_INVALID_ARGUMENT, "NULL argument");
  if (n < 0) return fail(NQS_ERR_INVALID_ARGUMENT, "n < 0");
  WsLayout L;
  nqs_status st = check_ws(p, 0, ws, ws_bytes, L);
  if (st != NQS_OK) return st;
  if (n == 0) return NQS_OK;
  hipStream_t s = p->ctx->stream;
  void* packed = at<void>(ws, L.packed);
  pack_net(p, params, packed, s);
  forward_net(p, packed, x, n, nullptr, out, nullptr, s);
  return launch_check("log psi");
}

nqs_status nqs_local_energy(nqs_plan* p, const float* params, const uint64_t* x, int64_t B, double* eloc,
                            void* ws, size_t ws_bytes) {
  if (!p || !params || (B > 0 && (!x || !eloc))) return fail(NQS_ERR_INVALID_ARGUMENT, "NULL argument");
  WsLayout L;
  nqs_status st = check_ws(p, B, ws, ws_bytes, L);
  if (st != NQS_OK) return st;
  hipEvent_t t0 = prof_mark(p);
  launch_fill_u32(at<void>(ws, L.err), 0u, 1, p->ctx->stream);
  if (B > 0) {
    st = run_local_energy(p, params, x, B, eloc, ws, L);
    if (st != NQS_OK) return st;
  }
  prof_close(p, t0, 3, -1);   // a call that is only a local-energy phase
  return launch_check("local energy");
}

nqs_status nqs_energy_grad(nqs_plan* p, const float* params, const uint64_t* x, const double* w, int64_t B,
                           double* eloc, double* energy, double* grad, void* ws, size_t ws_bytes) {
  if (!p || !params || !energy || !grad || (B > 0 && !x)) return fail(NQS_ERR_INVALID_ARGUMENT, "NULL argument");
  if (B < 1) return fail(NQS_ERR_INVALID_ARGUMENT, "energy needs at least one sample");
  WsLayout L;
  nqs_status st = check_ws(p, B, ws, ws_bytes, L);
  if (st != NQS_OK) return st;
  hipStream_t s = p->ctx->stream;
  unsigned* err = at<unsigned>(ws, L.err);
  hipEvent_t t0 = prof_mark(p);
  launch_fill_u32(err, 0u, 1, s);
  double* el = eloc ? eloc : at<double>(ws, L.eloc);
  st = run_local_energy(p, params, x, B, el, ws, L);
  if (st != NQS_OK) return st;
  if (t0) {
    hipEvent_t t1 = prof_mark(p);
    if (t1) p->recs.push_back({t0, t1, 1, -1});
  }
  energy_and_grad(p, params, x, w, B, el, energy, grad, ws, L);
  if (t0) {
    hipEvent_t t2 = prof_mark(p);
    if (t2) p->recs.push_back({t0, t2, 0, -1});
  }
  return launch_check("energy gradient");
}

nqs_status nqs_energy_grad_noalloc(nqs_plan* p, const float* params, const uint64_t* x, const double* w, int64_t B,
                                   double* eloc, double* energy, double* grad, uint32_t* d_flags) {
  if (!p) return fail(NQS_ERR_INVALID_ARGUMENT, "plan is NULL");
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(p->ctx->device);
    if (it == g_scratch_ptr.end())
      return fail(NQS_ERR_INVALID_ARGUMENT, "no scratch array attached for device %d", p->ctx->device);
    ws = it->second;
  }
  if (B >= 1 && B <= p->max_batch) {
    const size_t need = layout(p, B).total;
    if (need > (size_t)NQS_NOALLOC_SCRATCH_BYTES)
      return fail(NQS_ERR_WORKSPACE_TOO_SMALL,
                  "%lld samples need %zu bytes of workspace with this plan; the allocation-free entry point has "
                  "%zu (create the plan with a smaller batch or chunk)",
                  (long long)B, need, (size_t)NQS_NOALLOC_SCRATCH_BYTES);
  }
  // no profiling: its events would be created here, and its slots live in the workspace
  const bool prof = p->prof;
  p->prof = false;
  nqs_status st = nqs_energy_grad(p, params, x, w, B, eloc, energy, grad, ws, (size_t)NQS_NOALLOC_SCRATCH_BYTES);
  p->prof = prof;
  if (st == NQS_OK && d_flags) {
    hipLaunchKernelGGL(copy_flags_kernel, dim3(1), dim3(1), 0, p->ctx->stream,
                       (const unsigned*)((const char*)ws + layout(p, B).err), (unsigned*)d_flags);
    st = launch_check("energy gradient (allocation-free): flags");
  }
  return st;
}

// Workspace of a multi-instance call: each instance's layout, 256-byte aligned, in order.
static nqs_status multi_layout(int n_inst, const nqs_instance* inst, std::vector<size_t>& base, size_t& total) {
  if (n_inst < 0 || (n_inst > 0 && !inst)) return fail(NQS_ERR_INVALID_ARGUMENT, "bad instance list");
  base.assign(n_inst, 0);
  total = 0;
  for (int i = 0; i < n_inst; ++i) {
    const nqs_instance& I = inst[i];
    if (!I.plan) return fail(NQS_ERR_INVALID_ARGUMENT, "instance %d has no plan", i);
    if (I.plan->ctx != inst[0].plan->ctx) return fail(NQS_ERR_INVALID_ARGUMENT, "instances on different contexts");
    if (I.B < 1 || I.B > I.plan->max_batch)
      return fail(NQS_ERR_INVALID_ARGUMENT, "instance %d: batch %lld outside 1..%lld", i, (long long)I.B,
                  (long long)I.plan->max_batch);
    base[i] = total;
    total += align256(layout(I.plan, I.B).total);
  }
  return NQS_OK;
}

nqs_status nqs_multi_workspace_size(int n_inst, const nqs_instance* inst, size_t* bytes) {
  if (!bytes) return fail(NQS_ERR_INVALID_ARGUMENT, "NULL argument");
  std::vector<size_t> base;
  return multi_layout(n_inst, inst, base, *bytes);
}

nqs_status nqs_energy_grad_multi(int n_inst, const nqs_instance* inst, void* ws, size_t ws_bytes) {
  std::vector<size_t> base;
  size_t total = 0;
  nqs_status st = multi_layout(n_inst, inst, base, total);
  if (st != NQS_OK) return st;
  if (n_inst == 0) return NQS_OK;
  if (!ws) return fail(NQS_ERR_INVALID_ARGUMENT, "workspace is NULL");
  if (((uintptr_t)ws) & 255) return fail(NQS_ERR_INVALID_ARGUMENT, "workspace not 256-byte aligned");
  if (ws_bytes < total) return fail(NQS_ERR_WORKSPACE_TOO_SMALL, "workspace %zu < %zu bytes", ws_bytes, total);
  for (int i = 0; i < n_inst; ++i) {
    const nqs_instance& I = inst[i];
    if (!I.d_params || !I.d_samples || !I.d_energy || !I.d_grad)
      return fail(NQS_ERR_INVALID_ARGUMENT, "instance %d: NULL argument", i);
  }
  nqs_plan* p0 = inst[0].plan;
  hipStream_t s = p0->ctx->stream;
  hipEvent_t t0 = prof_mark(p0);
  std::vector<WsLayout> L(n_inst);
  std::vector<void*> W(n_inst);
  std::vector<double*> EL(n_inst);
  for (int i = 0; i < n_inst; ++i) {
    nqs_plan* p = inst[i].plan;
    W[i] = (char*)ws + base[i];
    L[i] = layout(p, inst[i].B);
    EL[i] = inst[i].d_eloc ? inst[i].d_eloc : at<double>(W[i], L[i].eloc);
    launch_fill_u32(at<void>(W[i], L[i].err), 0u, 1, s);
    launch_store_geom(p->g, at<Geom>(W[i], L[i].geom), s);
    if (p->two) launch_store_geom(p->gp, at<Geom>(W[i], L[i].geom) + 1, s);
    pack_net(p, inst[i].d_params, at<void>(W[i], L[i].packed), s);
  }
  // the forward segments of instance i's rows: its network, and with a
  // separate phase network a second segment that writes the phases (hg: the
  // host copy of each segment's geometry)
  std::vector<const Geom*> hg;
  auto add_segs = [&](int i, const uint64_t* x, const long long* d_count, double* out, long long bound,
                      std::vector<int>& ids, std::vector<FwdSeg>& segs) {
    const nqs_plan* p = inst[i].plan;
    ids.push_back(i);
    hg.push_back(&p->g);
    segs.push_back(FwdSeg{at<Geom>(W[i], L[i].geom), at<void>(W[i], L[i].packed), x, d_count, out, bound, 0,
                          nullptr});
    if (p->two) {
      ids.push_back(i);
      hg.push_back(&p->gp);
      segs.push_back(FwdSeg{at<Geom>(W[i], L[i].geom) + 1, at<char>(W[i], L[i].packed) + p->packed_phase, x,
                            d_count, out, bound, 0, nullptr});
    }
  };
  // One forward launch per group of segments whose networks share
  // (precision, width, variant): the segments' tiles form one work list.
  // Segments of two-word strings, and segments whose variant takes the half
  // tile, take the single-segment forward, one launch each (the multi-segment
  // form of the half tile gave rows different from the single-segment form's
  // at 16 waves, h = 512, so it is not used).
  auto launch_groups = [&](const std::vector<int>& ids, const std::vector<FwdSeg>& segs) {
    std::vector<bool> done(ids.size(), false);
    for (size_t a = 0; a < ids.size(); ++a) {
      if (done[a]) continue;
      const Geom& ga = inst[ids[a]].plan->g;
      const int va = inst[ids[a]].plan->variant;
      const bool ra = inst[ids[a]].plan->resident;
      const int cus = inst[ids[a]].plan->ctx->cu_count;
      const bool half = forward_variant_rows(ga.prec, ga.h, va) < forward_rows_per_block(ga.prec, ga.h);
      if (ga.words != 1 || half) {
        const FwdSeg& sg = segs[a];
        launch_forward(*hg[a], va, ra, cus, sg.packed, sg.x, sg.rows_bound, sg.d_count, sg.out, nullptr, s);
        done[a] = true;
        continue;
      }
      FwdLaunch la{};
      for (size_t b = a; b < ids.size(); ++b) {
        const Geom& gb = inst[ids[b]].plan->g;
        if (done[b] || gb.words != 1 || gb.prec != ga.prec || gb.h != ga.h || inst[ids[b]].plan->variant != va ||
            inst[ids[b]].plan->resident != ra)
          continue;   // (the same variant as segment a, so never a half tile here)
        la.seg[la.nseg++] = segs[b];
        done[b] = true;
        if (la.nseg == kMaxSeg) {
          launch_forward_multi(ga.prec, ga.h, va, ra, cus, la, s);
          la = FwdLaunch{};
        }
      }
      if (la.nseg > 0) launch_forward_multi(ga.prec, ga.h, va, ra, cus, la, s);
    }
  };
  std::vector<int> ids;
  std::vector<FwdSeg> segs;
  for (int i = 0; i < n_inst; ++i)
    add_segs(i, inst[i].d_samples, nullptr, at<double>(W[i], L[i].lps), inst[i].B, ids, segs);
  launch_groups(ids, segs);
  // chunk rounds: round r takes chunk r of every instance that still has one
  for (int64_t r = 0;; ++r) {
    ids.clear();
    segs.clear();
    hg.clear();
    std::vector<int> rid;
    std::vector<int64_t> c0s, scs;
    std::vector<ChunkFwd> cfs;
    for (int i = 0; i < n_inst; ++i) {
      nqs_plan* p = inst[i].plan;
      const int64_t c0 = r * p->S;
      if (c0 >= inst[i].B) continue;
      const int64_t Sc = std::min<int64_t>(p->S, inst[i].B - c0);
      const ChunkFwd cf = enum_chunk(p, inst[i].d_samples, c0, Sc, r, W[i], L[i]);
      rid.push_back(i);
      c0s.push_back(c0);
      scs.push_back(Sc);
      cfs.push_back(cf);
      add_segs(i, cf.x, cf.d_count, cf.out, cf.bound, ids, segs);
    }
    if (ids.empty()) break;
    launch_groups(ids, segs);
    for (size_t k = 0; k < rid.size(); ++k) {
      finish_chunk(inst[rid[k]].plan, cfs[k], W[rid[k]], L[rid[k]]);
      reduce_chunk(inst[rid[k]].plan, c0s[k], scs[k], cfs[k], W[rid[k]], L[rid[k]], EL[rid[k]]);
    }
  }
  for (int i = 0; i < n_inst; ++i) {
    const nqs_instance& I = inst[i];
    energy_and_grad(I.plan, I.d_params, I.d_samples, I.d_weights, I.B, EL[i], I.d_energy, I.d_grad, W[i], L[i]);
  }
  if (t0) {
    hipEvent_t t1 = prof_mark(p0);
    if (t1) p0->recs.push_back({t0, t1, 0, -1});
  }
  return launch_check("energy gradient (multi)");
}

}  // extern "C"

// ------------------------------------------------------------- autotuner
namespace {
using TuneKey = std::tuple<int, int, int, int, int64_t, int64_t, int64_t, int64_t, int, int, int>;
struct TuneVal { int variant; bool dedup; int64_t S; bool resident; double ms; };
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune_cache;

TuneKey tune_key(const nqs_plan* p) {
  return TuneKey{p->g.n, p->g.L, p->g.h, p->g.prec, (int64_t)p->ham->tre.size(), (int64_t)(p->ham->gx.size() / p->ham->words),
                 p->Emax, p->S0, p->dedup_auto ? 1 : 0, p->ctx->device, p->g.phase_mode};
}

void set_chunk(nqs_plan* p, int64_t S) {
  const int G = (int)(p->ham->gx.size() / p->ham->words);
  const int gfirst = ham_has_diag(p->ham) ? 1 : 0;
  p->S = S;
  grid_for(S, G - gfirst, p->R, p->gper);
}
}  // namespace

extern "C" {

nqs_status nqs_plan_autotune(nqs_plan* p, const float* params, const uint64_t* x, int64_t B, void* ws,
                             size_t ws_bytes, uint32_t flags, nqs_tune_report* rep) {
  if (!p || !params || !x) return fail(NQS_ERR_INVALID_ARGUMENT, "NULL argument");
  if (B < 1) return fail(NQS_ERR_INVALID_ARGUMENT, "autotuning needs at least one sample");
  if (flags & ~(NQS_TUNE_FORCE | NQS_TUNE_CACHE_ONLY))
    return fail(NQS_ERR_INVALID_ARGUMENT, "unknown tune flags 0x%x", flags);
  if ((flags & NQS_TUNE_FORCE) && (flags & NQS_TUNE_CACHE_ONLY))
    return fail(NQS_ERR_INVALID_ARGUMENT, "NQS_TUNE_FORCE and NQS_TUNE_CACHE_ONLY exclude each other");
  WsLayout L;
  nqs_status st = check_ws(p, B, ws, ws_bytes, L);
  if (st != NQS_OK) return st;
  nqs_tune_report local{};
  nqs_tune_report& R = rep ? *rep : local;
  memset(&R, 0, sizeof(R));
  const TuneKey key = tune_key(p);
  if (!(flags & NQS_TUNE_FORCE)) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    // an entry read from a database file is applied only where the plan's
    // workspace has room for it (dedup tables, chunk within the created one)
    if (it != g_tune_cache.end() && (!it->second.dedup || p->dedup_cap) && it->second.S <= p->S0) {
      p->variant = it->second.variant;
      p->dedup = it->second.dedup;
      p->resident = it->second.resident;
      set_chunk(p, it->second.S);
      p->tuned = true;
      R.from_cache = 1;
      R.n_candidates = 1;
      R.chosen = 0;
      R.cand[0] = nqs_tune_candidate{forward_variant_waves(p->g.prec, p->g.h, p->variant),
                                     forward_variant_rows(p->g.prec, p->g.h, p->variant), p->dedup ? 1 : 0, p->S,
                                     p->resident ? 1 : 0, it->second.ms};
      return NQS_OK;
    }
  }
  if (flags & NQS_TUNE_CACHE_ONLY) return NQS_OK;
  struct Cand { int v; bool d; int64_t S; bool r; };
  std::vector<Cand> cands;
  const int nv = forward_variants(p->g.prec, p->g.h);
  std::vector<bool> dd = p->dedup_auto ? std::vector<bool>{false, true} : std::vector<bool>{p->dedup};
  std::vector<int64_t> ss{p->S0};
  if (p->S0 >= 2) ss.push_back(p->S0 / 2);
  for (int v = 0; v < nv; ++v)
    for (bool d : dd)
      for (int64_t S : ss)
        for (bool r : {false, true}) cands.push_back({v, d, S, r});
  if ((int)cands.size() > NQS_TUNE_MAX_CANDIDATES) cands.resize(NQS_TUNE_MAX_CANDIDATES);
  const int64_t probe = std::min<int64_t>(B, 2 * p->S0);
  const bool prof = p->prof;
  p->prof = false;
  double* el = at<double>(ws, L.eloc);
  hipStream_t s = p->ctx->stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int best = -1;
  double best_ms = 0.0;
  // NQS_TUNE_LOG set: one line per timed candidate on stderr (a long tuning run shows its progress)
  const bool log = getenv("NQS_TUNE_LOG") != nullptr;
  for (size_t c = 0; c < cands.size(); ++c) {
    p->variant = cands[c].v;
    p->dedup = cands[c].d;
    p->resident = cands[c].r;
    set_chunk(p, cands[c].S);
    launch_fill_u32(at<void>(ws, L.err), 0u, 1, s);
    st = run_local_energy(p, params, x, probe, el, ws, L);   // warm-up
    if (st == NQS_OK) {
      HIP_TRY(hipEventRecord(e0, s));
      for (int k = 0; k < 2 && st == NQS_OK; ++k) st = run_local_energy(p, params, x, probe, el, ws, L);
      HIP_TRY(hipEventRecord(e1, s));
    }
    if (st != NQS_OK) break;
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    R.cand[c] = nqs_tune_candidate{forward_variant_waves(p->g.prec, p->g.h, cands[c].v),
                                   forward_variant_rows(p->g.prec, p->g.h, cands[c].v), cands[c].d ? 1 : 0,
                                   cands[c].S, cands[c].r ? 1 : 0, ms / 2.0};
    if (log) {
      fprintf(stderr, "nqs tuner: candidate %zu/%zu: %d waves, %d-row tiles, dedup %d, chunk %lld, %s grid: %.1f ms\n",
              c + 1, cands.size(), R.cand[c].waves_per_block, R.cand[c].rows_per_block, R.cand[c].dedup,
              (long long)R.cand[c].chunk_samples, cands[c].r ? "resident" : "one-tile", ms / 2.0);
      fflush(stderr);
    }
    if (best < 0 || ms / 2.0 < best_ms) { best = (int)c; best_ms = ms / 2.0; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  p->prof = prof;
  if (st != NQS_OK || best < 0) return st != NQS_OK ? st : fail(NQS_ERR_INVALID_ARGUMENT, "no candidate");
  R.n_candidates = (int)cands.size();
  R.chosen = best;
  R.probe_samples = probe;
  p->variant = cands[best].v;
  p->dedup = cands[best].d;
  p->resident = cands[best].r;
  set_chunk(p, cands[best].S);
  p->tuned = true;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = TuneVal{p->variant, p->dedup, p->S, p->resident, best_ms};
  }
  return NQS_OK;
}

// Tuner database: the cached choices as text, one entry per line, so a later
// process applies them without timing.  Fields: the 11 key values, then the
// forward's waves per workgroup and rows per tile, dedup, chunk, grid and the
// measured ms.
nqs_status nqs_tune_db_save(const char* path) {
  if (!path) return fail(NQS_ERR_INVALID_ARGUMENT, "path is NULL");
  std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return fail(NQS_ERR_INVALID_ARGUMENT, "cannot write %s", tmp.c_str());
  fprintf(f, "# nqs tuner database v3: n L h precision K G entries_per_sample chunk dedup_auto device phase_mode"
             " | waves rows dedup chunk resident ms\n");
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& kv : g_tune_cache) {
      const TuneKey& k = kv.first;
      const TuneVal& v = kv.second;
      fprintf(f, "%d %d %d %d %lld %lld %lld %lld %d %d %d | %d %d %d %lld %d %.6f\n", std::get<0>(k),
              std::get<1>(k), std::get<2>(k), std::get<3>(k), (long long)std::get<4>(k), (long long)std::get<5>(k),
              (long long)std::get<6>(k), (long long)std::get<7>(k), std::get<8>(k), std::get<9>(k), std::get<10>(k),
              forward_variant_waves(std::get<3>(k), std::get<2>(k), v.variant),
              forward_variant_rows(std::get<3>(k), std::get<2>(k), v.variant), v.dedup ? 1 : 0, (long long)v.S,
              v.resident ? 1 : 0, v.ms);
    }
  }
  const bool ok = fclose(f) == 0;
  if (!ok || rename(tmp.c_str(), path) != 0) return fail(NQS_ERR_INVALID_ARGUMENT, "cannot write %s", path);
  return NQS_OK;
}

nqs_status nqs_tune_db_load(const char* path, int* n_loaded) {
  if (!path) return fail(NQS_ERR_INVALID_ARGUMENT, "path is NULL");
  if (n_loaded) *n_loaded = 0;
  FILE* f = fopen(path, "r");
  if (!f) return fail(NQS_ERR_INVALID_ARGUMENT, "cannot read %s", path);
  char line[512];
  int n = 0, lineno = 0;
  nqs_status st = NQS_OK;
  while (fgets(line, sizeof(line), f)) {
    ++lineno;
    if (line[0] == '#' || line[0] == '\n') continue;
    // 11 key fields, "|", then waves, rows, dedup, chunk, resident (integers) and ms
    long long iv[16] = {};
    double ms = 0.0;
    int ntok = 0;
    bool whole = true;
    char* save = nullptr;
    for (char* tok = strtok_r(line, " \t\r\n", &save); tok && whole; tok = strtok_r(nullptr, " \t\r\n", &save)) {
      char* end = nullptr;
      if (ntok == 11) whole = strcmp(tok, "|") == 0;
      else if (ntok == 17) ms = strtod(tok, &end);
      else if (ntok < 17) iv[ntok < 11 ? ntok : ntok - 1] = strtoll(tok, &end, 10);
      else whole = false;
      if (end) whole = whole && end != tok && *end == 0;
      ++ntok;
    }
    whole = whole && ntok == 18;
    int a[11];
    long long b[4] = {iv[4], iv[5], iv[6], iv[7]};
    for (int k = 0; k < 11; ++k) a[k] = (int)iv[k];
    const int waves = (int)iv[11], rows = (int)iv[12], dedup = (int)iv[13], res = (int)iv[15];
    const long long S = iv[14];
    int v = -1;
    if (whole && a[3] >= 0 && a[3] <= NQS_BF16W && a[2] > 0 && (res == 0 || res == 1))
      for (int k = 0; k < forward_variants(a[3], a[2]); ++k)
        if (forward_variant_waves(a[3], a[2], k) == waves && forward_variant_rows(a[3], a[2], k) == rows) v = k;
    if (v < 0 || S < 1 || S > b[3]) {
      st = fail(NQS_ERR_INVALID_ARGUMENT, "%s:%d: not a tuner database entry", path, lineno);
      break;
    }
    const TuneKey key{a[0], a[1], a[2], a[3], (int64_t)b[0], (int64_t)b[1], (int64_t)b[2], (int64_t)b[3], a[8], a[9],
                      a[10]};
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = TuneVal{v, dedup != 0, (int64_t)S, res != 0, ms};
    ++n;
  }
  fclose(f);
  if (n_loaded) *n_loaded = n;
  return st;
}

nqs_status nqs_plan_configure(nqs_plan* p, int waves_per_block, int rows_per_block, int dedup, int64_t chunk_samples,
                              int resident) {
  if (!p) return fail(NQS_ERR_INVALID_ARGUMENT, "plan is NULL");
  const int prec = p->g.prec, h = p->g.h;
  const int want_w = waves_per_block > 0 ? waves_per_block : forward_variant_waves(prec, h, p->variant);
  const int want_r = rows_per_block > 0 ? rows_per_block : forward_variant_rows(prec, h, p->variant);
  int v = -1;
  for (int k = 0; v < 0 && k < forward_variants(prec, h); ++k)
    if (forward_variant_waves(prec, h, k) == want_w && forward_variant_rows(prec, h, k) == want_r) v = k;
  if (v < 0)
    return fail(NQS_ERR_UNSUPPORTED, "no forward variant with %d waves per workgroup and %d-row tiles", want_w,
                want_r);
  if (dedup > 0 && !p->dedup_cap)
    return fail(NQS_ERR_INVALID_ARGUMENT, "plan was not created for dedup (DEDUP_ON or DEDUP_AUTO)");
  if (chunk_samples > p->S0)
    return fail(NQS_ERR_INVALID_ARGUMENT, "chunk %lld exceeds the plan's %lld", (long long)chunk_samples,
                (long long)p->S0);
  if (chunk_samples > 0 && chunk_samples < std::max<int64_t>(1, p->S0 / 2))
    return fail(NQS_ERR_INVALID_ARGUMENT, "chunk %lld below half the plan's %lld", (long long)chunk_samples,
                (long long)p->S0);
  p->variant = v;
  if (dedup >= 0) p->dedup = dedup > 0;
  if (resident >= 0) p->resident = resident > 0;
  if (chunk_samples > 0) set_chunk(p, chunk_samples);
  return NQS_OK;
}

nqs_status nqs_plan_kernel_info(const nqs_plan* p, int* waves_per_block, int* rows_per_block, int* tuned,
                                int* resident) {
  if (!p) return fail(NQS_ERR_INVALID_ARGUMENT, "plan is NULL");
  if (resident) *resident = p->resident ? 1 : 0;
  if (waves_per_block) *waves_per_block = forward_variant_waves(p->g.prec, p->g.h, p->variant);
  if (rows_per_block) *rows_per_block = forward_variant_rows(p->g.prec, p->g.h, p->variant);
  if (tuned) *tuned = p->tuned ? 1 : 0;
  return NQS_OK;
}

// ---------------------------------------------------------------- sampler
namespace {
struct SampleLayout {
  size_t err, packed, cond, x, cnt, kx, kc, eq, keep, eqoff, koff, stmp, sel, du, dnk, total;
};

SampleLayout sample_layout(const nqs_plan* p, int64_t U) {
  SampleLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
  const size_t U2 = 2 * (size_t)U;
  L.err = take(256);
  L.packed = take(p->packed_bytes);
  L.cond = take((size_t)U * 16);
  L.x = take((size_t)U * 8 * p->g.words);
  L.cnt = take((size_t)U * 8);
  L.kx = take(U2 * 8 * p->g.words);
  L.kc = take(U2 * 8);
  L.eq = take(U2 * 4);
  L.keep = take(U2 * 4);
  L.eqoff = take((U2 + 1) * 8);
  L.koff = take((U2 + 1) * 8);
  L.stmp = take(((size_t)scan_tiles((long long)U2) + 1) * 8);
  L.sel = take(16);
  L.du = take(8);
  L.dnk = take(8);
  L.total = o;
  return L;
}
}  // namespace

nqs_status nqs_sample_workspace_size(const nqs_plan* p, int64_t max_unique, size_t* bytes) {
  if (!p || !bytes) return fail(NQS_ERR_INVALID_ARGUMENT, "NULL argument");
  if (max_unique < 1 || max_unique > (1LL << 30))
    return fail(NQS_ERR_INVALID_ARGUMENT, "max_unique %lld outside 1..2^30", (long long)max_unique);
  *bytes = sample_layout(p, max_unique).total;
  return NQS_OK;
}

nqs_status nqs_sample(nqs_plan* p, const float* params, int64_t n_draws, uint64_t seed, int64_t max_unique,
                      uint64_t* d_x, double* d_w, int64_t* d_n_unique, void* ws, size_t ws_bytes) {
  if (!p || !params || !d_x || !d_w || !d_n_unique) return fail(NQS_ERR_INVALID_ARGUMENT, "NULL argument");
  if (n_draws < 1 || n_draws > (1LL << 62)) return fail(NQS_ERR_INVALID_ARGUMENT, "n_draws outside 1..2^62");
  if (max_unique < 1 || max_unique > (1LL << 30))
    return fail(NQS_ERR_INVALID_ARGUMENT, "max_unique %lld outside 1..2^30", (long long)max_unique);
  if (!ws) return fail(NQS_ERR_INVALID_ARGUMENT, "workspace is NULL");
  if (((uintptr_t)ws) & 255) return fail(NQS_ERR_INVALID_ARGUMENT, "workspace not 256-byte aligned");
  const SampleLayout L = sample_layout(p, max_unique);
  if (ws_bytes < L.total) return fail(NQS_ERR_WORKSPACE_TOO_SMALL, "workspace %zu < %zu bytes", ws_bytes, L.total);
  hipStream_t s = p->ctx->stream;
  SampleBufs b{};
  b.x = at<uint64_t>(ws, L.x);
  b.cnt = at<long long>(ws, L.cnt);
  b.cond = at<double>(ws, L.cond);
  b.kx = at<uint64_t>(ws, L.kx);
  b.kc = at<long long>(ws, L.kc);
  b.eq = at<int>(ws, L.eq);
  b.keep = at<int>(ws, L.keep);
  b.eqoff = at<long long>(ws, L.eqoff);
  b.koff = at<long long>(ws, L.koff);
  b.stmp = at<long long>(ws, L.stmp);
  b.sel = at<long long>(ws, L.sel);
  b.d_u = at<long long>(ws, L.du);
  b.d_nk = at<long long>(ws, L.dnk);
  b.words = p->g.words;
  void* packed = at<void>(ws, L.packed);
  launch_pack_fused(p->g, params, packed, s);
  launch_sample_init(b.x, b.words, b.cnt, n_draws, b.d_u, s);
  for (int t = 0; t < p->g.n; ++t) {
    launch_forward_cond(p->g, p->variant, p->resident, p->ctx->cu_count, packed, b.x, max_unique, b.d_u, b.cond, t,
                        s);
    launch_sample_step(b, max_unique, t, (int)p->g.order[t], seed, s);
  }
  launch_sample_finish(b, max_unique, d_x, d_w, (long long*)d_n_unique, s);
  return launch_check("sample");
}

}  // extern "C"

namespace nqs {
void launch_copy_i64(const long long* src, long long* dst, hipStream_t s);
void launch_seg_offsets(const int* esample, long long n_entries, long long B, long long* off, hipStream_t s);
}

extern "C" {

nqs_status nqs_connected(nqs_plan* p, const uint64_t* x, int64_t B, int64_t capacity, double* d_diag,
                         int32_t* d_esample, uint64_t* d_ex, double* d_eh, int64_t* d_n_entries,
                         uint64_t* d_unique, int32_t* d_eunique, int64_t* d_n_unique, void* ws, size_t ws_bytes) {
  if (!p || (B > 0 && (!x || !d_diag || !d_ex || !d_eh || !d_n_entries)))
    return fail(NQS_ERR_INVALID_ARGUMENT, "NULL argument");
  if (B > p->S) return fail(NQS_ERR_INVALID_ARGUMENT, "batch %lld exceeds the plan's chunk %lld", (long long)B, (long long)p->S);
  if (capacity < 0 || capacity >= (1LL << 31)) return fail(NQS_ERR_INVALID_ARGUMENT, "capacity out of range");
  if (p->dedup && (!d_unique || !d_eunique || !d_n_unique))
    return fail(NQS_ERR_INVALID_ARGUMENT, "dedup plan needs the unique outputs");
  WsLayout L;
  nqs_status st = check_ws(p, B, ws, ws_bytes, L);
  if (st != NQS_OK) return st;
  hipStream_t s = p->ctx->stream;
  const HamDev H = ham_dev(p);
  unsigned* err = at<unsigned>(ws, L.err);
  launch_fill_u32(err, 0u, 1, s);
  if (B == 0) {
    launch_fill_u64(d_n_entries, 0ull, 1, s);
    if (p->dedup) launch_fill_u64(d_n_unique, 0ull, 1, s);
    return launch_check("connected");
  }
  int* cnt = at<int>(ws, L.cnt);
  long long* off = at<long long>(ws, L.off);
  launch_diag(H, x, B, d_diag, s);
  launch_count(H, x, B, p->R, p->gper, cnt, s);
  launch_scan(cnt, B * p->R, off, at<long long>(ws, L.stmp), s);
  launch_write(H, x, B, p->R, p->gper, off, capacity, d_ex, d_eh, d_esample, 2, err, s);
  launch_copy_i64(off + B * p->R, (long long*)d_n_entries, s);
  if (p->dedup) {
    if (capacity > p->EC || (int64_t)2 * capacity > p->HT)
      return fail(NQS_ERR_INVALID_ARGUMENT, "capacity exceeds the plan's dedup buffers");
    launch_dedup(d_ex, p->g.words, p->g.n == 64, (const long long*)d_n_entries, capacity, at<void>(ws, L.htab),
                 p->HT, true, d_eunique, d_unique, (long long*)d_n_unique, at<int>(ws, L.dfirst),
                 at<long long>(ws, L.drank), at<long long>(ws, L.drtmp), err, s);
  }
  return launch_check("connected");
}

nqs_status nqs_reduce_table(nqs_plan* p, int64_t B, const double* lps, const double* lpe, const double* diag,
                            const int32_t* esample, const double* eh, int64_t n_entries, double* eloc, void* ws,
                            size_t ws_bytes) {
  if (!p || (B > 0 && (!lps || !diag || !eloc)) || (n_entries > 0 && (!lpe || !esample || !eh)))
    return fail(NQS_ERR_INVALID_ARGUMENT, "NULL argument");
  if (n_entries < 0) return fail(NQS_ERR_INVALID_ARGUMENT, "n_entries < 0");
  if (B > p->S) return fail(NQS_ERR_INVALID_ARGUMENT, "batch exceeds the plan's chunk");
  WsLayout L;
  nqs_status st = check_ws(p, B, ws, ws_bytes, L);
  if (st != NQS_OK) return st;
  hipStream_t s = p->ctx->stream;
  unsigned* err = at<unsigned>(ws, L.err);
  launch_fill_u32(err, 0u, 1, s);
  if (B == 0) return launch_check("reduce");
  long long* off = at<long long>(ws, L.off);
  launch_seg_offsets(esample, n_entries, B, off, s);
  launch_reduce(B, 1, off, n_entries, diag, eh, 2, nullptr, lpe, lps, eloc, at<double>(ws, L.rpart), err, s);
  return launch_check("reduce");
}

nqs_status nqs_adam_step(nqs_ctx* ctx, int64_t n, float* d_params, const double* d_grad, double* d_m,
                         double* d_v, int64_t step, double lr, double beta1, double beta2, double eps) {
  if (!ctx) return fail(NQS_ERR_INVALID_ARGUMENT, "NULL context");
  if (n < 0) return fail(NQS_ERR_INVALID_ARGUMENT, "n < 0");
  if (n > 0 && (!d_params || !d_grad || !d_m || !d_v)) return fail(NQS_ERR_INVALID_ARGUMENT, "NULL buffer");
  if (step < 1) return fail(NQS_ERR_INVALID_ARGUMENT, "step must be >= 1");
  if (!(lr >= 0.0) || !(eps >= 0.0)) return fail(NQS_ERR_INVALID_ARGUMENT, "lr and eps must be >= 0");
  if (!(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0))
    return fail(NQS_ERR_INVALID_ARGUMENT, "betas must lie in [0, 1)");
  nqs::AdamCoef k;
  k.lr = lr;
  k.b1 = beta1;
  k.b2 = beta2;
  k.one_m_b1 = 1.0 - beta1;
  k.one_m_b2 = 1.0 - beta2;
  k.bc1 = 1.0 - std::pow(beta1, (double)step);
  k.bc2 = 1.0 - std::pow(beta2, (double)step);
  k.eps = eps;
  if (!(k.bc1 > 0.0) || !(k.bc2 > 0.0)) return fail(NQS_ERR_INVALID_ARGUMENT, "bias correction is zero");
  nqs::launch_adam(n, d_params, d_grad, d_m, d_v, k, ctx->cu_count, ctx->stream);
  return launch_check("nqs_adam_step");
}

nqs_status nqs_device_status(nqs_ctx* ctx, void* ws, uint32_t* flags) {
  if (!ctx || !ws || !flags) return fail(NQS_ERR_INVALID_ARGUMENT, "NULL argument");
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  unsigned v = 0;
  HIP_TRY(hipMemcpy(&v, ws, 4, hipMemcpyDeviceToHost));
  const unsigned zero = 0;
  HIP_TRY(hipMemcpy(ws, &zero, 4, hipMemcpyHostToDevice));
  *flags = v;
  return v ? fail(NQS_ERR_DEVICE, "device error word 0x%x", v) : NQS_OK;
}

nqs_status nqs_multi_device_status(int n_inst, const nqs_instance* inst, void* ws, uint32_t* flags) {
  if (!ws || !flags) return fail(NQS_ERR_INVALID_ARGUMENT, "NULL argument");
  std::vector<size_t> base;
  size_t total = 0;
  nqs_status st = multi_layout(n_inst, inst, base, total);
  if (st != NQS_OK) return st;
  *flags = 0;
  if (n_inst == 0) return NQS_OK;
  HIP_TRY(hipStreamSynchronize(inst[0].plan->ctx->stream));
  unsigned acc = 0;
  for (int i = 0; i < n_inst; ++i) {
    char* w = (char*)ws + base[i] + layout(inst[i].plan, inst[i].B).err;
    unsigned v = 0;
    HIP_TRY(hipMemcpy(&v, w, 4, hipMemcpyDeviceToHost));
    const unsigned zero = 0;
    HIP_TRY(hipMemcpy(w, &zero, 4, hipMemcpyHostToDevice));
    acc |= v;
  }
  *flags = acc;
  return acc ? fail(NQS_ERR_DEVICE, "device error word 0x%x", acc) : NQS_OK;
}

}  // extern "C"
