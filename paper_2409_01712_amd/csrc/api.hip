// C ABI of the KRR library: handles, argument validation and the host-side
// orchestration of the Build / Associate / Predict phases of the paper's KRR
// driver (arXiv 2409.01712, Algorithm 1).  Every arithmetic step runs in the
// HIP kernels of build.hip, factor.hip and solve.hip.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.h"

using namespace krr;

struct TimerRec {
  int stage;
  hipEvent_t a, b;
};

struct krr_context_s {
  int device = 0;
  hipStream_t stream = nullptr;
  krr_options opts{};
  int64_t allocated = 0;  // bytes of the blocks handed out
  // device memory cache: freed blocks by size, and the size of every live block
  std::multimap<size_t, void *> cache;
  size_t cached = 0;
  std::unordered_map<void *, size_t> live_sizes;
  // stage timers
  uint32_t timing = 0;  // bit s: stage s is timed
  std::vector<TimerRec> recs;
  std::vector<hipEvent_t> pool;
  double total_ms[KRR_STAGE_COUNT] = {};
  int64_t intervals[KRR_STAGE_COUNT] = {};
  // live kernel/factor handles; krr_destroy defers the free until they are released
  int64_t live = 0;
  bool destroy_pending = false;
  // schedule choices (krr_set_tuning / krr_autotune); 0 / -1 fields: the defaults
  krr_tuning tune{};
  // instantiated graphs of the batched calls' launch sequences, by launch shape
  std::map<std::string, hipGraphExec_t> graphs;
  int64_t graph_replays = 0;
  // device job tables of the batched factorization and solve, kept at stable
  // addresses so that their graphs can be replayed (grown, never shrunk)
  void *jobtab[2] = {nullptr, nullptr};
  size_t jobtab_bytes[2] = {0, 0};
  // second stream and events for the factorization's lookahead
  hipStream_t aux = nullptr, side = nullptr, fmain = nullptr;
  hipStream_t cap = nullptr;  // graph capture
  int aux_e = 8;              // eighths of the CUs the aux stream uses
  hipStream_t aux_by_e[9] = {};  // the aux streams made so far, by eighths (kept)
  std::vector<hipEvent_t> sched_ev;  // ordering events of the factorization schedule
  // second stream and events of the split quad sweeps
  hipStream_t sw2 = nullptr;
  std::vector<hipEvent_t> sweep_ev;
};

struct krr_kernel_s {
  krr_context ctx = nullptr;
  const int8_t *G = nullptr;
  int64_t n = 0, m = 0, ldg = 0;
  double gamma = 0, lambda = 0;
  int kind = KRR_KERNEL_GAUSSIAN;
  // IBS: the thermometer-encoded genotypes (n x ldh, mh = ldh columns), owned
  int8_t *H = nullptr;
  int64_t ldh = 0;
  // confounders: their FP64 copy (n x q) and the factors exp(-gamma dc) (packed tiles)
  double *Cc = nullptr;
  double *Ec = nullptr;
  int64_t q = 0;
  // what the Gram reads: G, or H for the IBS kernel
  const int8_t *gram_src() const { return H ? H : G; }
  int64_t gram_m() const { return H ? ldh : m; }
  int64_t gram_ld() const { return H ? ldh : ldg; }
  int vmode() const {
    return kind == KRR_KERNEL_IBS ? VAL_TABLE : kind == KRR_KERNEL_LINEAR ? VAL_LINEAR : VAL_EXP;
  }
  TileLayout L;
  int8_t *Gs = nullptr;  // the Gram's genotypes slab-major, or null
  int64_t gs_bytes = 0;
  int32_t *D = nullptr;  // exact distances, packed lower tiles
  float *A = nullptr;    // K + lambda I, FP32, packed lower tiles (null once consumed)
  int32_t *nrm = nullptr;
  double *etab = nullptr;
  int64_t etab_len = 0;
  double *tnorm = nullptr;      // per-tile Frobenius norms
  double *tnorm_part = nullptr;
  std::vector<double> tnorm_host;
  double norm_a = -1.0;
};

struct krr_factor_s {
  krr_context ctx = nullptr;
  krr_kernel K = nullptr;  // must outlive the factor (its distances feed the residual)
  TileLayout L;
  float *Lst = nullptr;   // FP32 factor, packed lower tiles
  float *Linv = nullptr;  // inverses of the diagonal tiles, nt x nb x nb
  float *Cpair = nullptr; // coupling tiles of the paired sweeps, nt / 2 (first solve)
  float *Cquad = nullptr; // coupling tiles of the quad sweeps, 4 (nt / 4) (first solve)
  krr_factor_info info{};
  std::vector<uint8_t> pmap;
};

namespace {

#define HIPCHK(x)                                  \
  do {                                             \
    hipError_t _e = (x);                           \
    if (_e != hipSuccess) {                        \
      if (getenv("KRR_DEBUG"))                     \
        fprintf(stderr, "krr: %s failed: %s\n", #x, \
                hipGetErrorString(_e));            \
      return KRR_ERROR_HIP;                        \
    }                                              \
  } while (0)

#define CHK(x)                    \
  do {                            \
    krr_status _s = (x);          \
    if (_s != KRR_SUCCESS) return _s; \
  } while (0)

// Device memory goes through a per-context cache: a freed block is kept and
// handed to a later request of about its size instead of going back to the
// runtime (whose free synchronizes the device and whose large allocations map
// pages, milliseconds per call).  Every free in this library happens after the
// work that used the block has completed (the calls synchronize their stream
// before releasing memory), so any later call may reuse a cached block.
constexpr size_t KRR_CACHE_MAX = (size_t)64 << 30;  // larger caches return blocks to the runtime

// Device memory from the caller's allocator when the context has one.
void raw_free(krr_context ctx, void *p, size_t size) {
  if (ctx->opts.device_free) ctx->opts.device_free(p, size, ctx->opts.alloc_user);
  else (void)hipFree(p);
}

hipError_t raw_alloc(krr_context ctx, void **p, size_t bytes) {
  if (!ctx->opts.device_alloc) return hipMalloc(p, bytes);
  *p = ctx->opts.device_alloc(bytes, ctx->opts.alloc_user);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}

void cache_flush(krr_context ctx) {
  for (auto &kv : ctx->cache) raw_free(ctx, kv.second, kv.first);
  ctx->cache.clear();
  ctx->cached = 0;
}

krr_status dalloc(krr_context ctx, void **p, size_t bytes) {
  *p = nullptr;
  bytes = (std::max<size_t>(bytes, 16) + 255) & ~(size_t)255;
  if (ctx->opts.workspace_limit > 0 && ctx->allocated + (int64_t)bytes > ctx->opts.workspace_limit)
    return KRR_ERROR_OUT_OF_MEMORY;
  size_t size = bytes;
  // the smallest cached block that fits, if it wastes at most a quarter
  auto it = ctx->cache.lower_bound(bytes);
  if (it != ctx->cache.end() && it->first <= bytes + bytes / 4) {
    size = it->first;
    *p = it->second;
    ctx->cached -= size;
    ctx->cache.erase(it);
  } else {
    hipError_t e = raw_alloc(ctx, p, bytes);
    if (e == hipErrorOutOfMemory && !ctx->cache.empty()) {
      (void)hipGetLastError();
      cache_flush(ctx);
      e = raw_alloc(ctx, p, bytes);
    }
    if (e != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      return e == hipErrorOutOfMemory ? KRR_ERROR_OUT_OF_MEMORY : KRR_ERROR_HIP;
    }
  }
  ctx->live_sizes[*p] = size;
  ctx->allocated += (int64_t)size;
  return KRR_SUCCESS;
}

template <typename T>
krr_status dalloc_t(krr_context ctx, T **p, int64_t count) {
  return dalloc(ctx, (void **)p, (size_t)count * sizeof(T));
}

void dfree(krr_context ctx, void *p, size_t /*bytes*/) {
  if (!p) return;
  auto it = ctx->live_sizes.find(p);
  if (it == ctx->live_sizes.end()) return;  // not from dalloc: not ours to free
  const size_t size = it->second;
  ctx->live_sizes.erase(it);
  ctx->allocated -= (int64_t)size;
  if (ctx->cached + size <= KRR_CACHE_MAX) {
    ctx->cache.emplace(size, p);
    ctx->cached += size;
  } else {
    raw_free(ctx, p, size);
  }
}

krr_status launch_ok() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    if (getenv("KRR_DEBUG")) fprintf(stderr, "krr: launch failed: %s\n", hipGetErrorString(e));
    return KRR_ERROR_HIP;
  }
  return KRR_SUCCESS;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

TileLayout make_layout(int64_t n, int nb) {
  TileLayout L;
  L.nb = nb;
  L.n = n;
  L.nt = (int)((n + nb - 1) / nb);
  L.np = (int64_t)L.nt * nb;
  return L;
}

struct Scoped {  // frees device buffers on scope exit unless released
  krr_context ctx;
  std::vector<std::pair<void *, size_t>> bufs;
  explicit Scoped(krr_context c) : ctx(c) {}
  template <typename T>
  krr_status alloc(T **p, int64_t count) {
    CHK(dalloc_t(ctx, p, count));
    bufs.push_back({(void *)*p, (size_t)count * sizeof(T)});
    return KRR_SUCCESS;
  }
  void release() { bufs.clear(); }
  ~Scoped() {
    // an early return may leave work in flight; the blocks go back to the cache
    if (!bufs.empty()) (void)hipDeviceSynchronize();
    for (auto &b : bufs) dfree(ctx, b.first, b.second);
  }
};

hipEvent_t take_event(krr_context c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

// Brackets the launches of one stage with events when timing is enabled.
struct Stage {
  krr_context c;
  hipStream_t st;
  int64_t idx = -1;
  Stage(krr_context ctx, int stage, hipStream_t stream = nullptr) : c(ctx) {
    st = stream ? stream : c->stream;
    if (!((c->timing >> stage) & 1u)) return;
    TimerRec r{stage, take_event(c), take_event(c)};
    if (!r.a || !r.b) return;
    if (hipEventRecord(r.a, st) != hipSuccess) return;
    c->recs.push_back(r);
    idx = (int64_t)c->recs.size() - 1;
  }
  ~Stage() {
    if (idx >= 0) (void)hipEventRecord(c->recs[idx].b, st);
  }
};

void timers_drain(krr_context c) {
  if (c->recs.empty()) return;
  (void)hipEventSynchronize(c->recs.back().b);
  for (auto &r : c->recs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      c->total_ms[r.stage] += ms;
      c->intervals[r.stage] += 1;
    } else {
      (void)hipGetLastError();
    }
    c->pool.push_back(r.a);
    c->pool.push_back(r.b);
  }
  c->recs.clear();
}

}  // namespace

extern "C" {

const char *krr_stage_name(int32_t stage) {
  static const char *names[KRR_STAGE_COUNT] = {
      "row_norms", "gram", "potrf", "trsm", "convert", "update",
      "fwd_sweep", "bwd_sweep", "residual", "cross_gram", "predict_apply"};
  if (stage < 0 || stage >= KRR_STAGE_COUNT) return "unknown";
  return names[stage];
}

krr_status krr_timers_enable(krr_context ctx, int32_t enable) {
  return krr_timers_enable_stages(ctx, enable ? (1u << KRR_STAGE_COUNT) - 1u : 0u);
}

krr_status krr_timers_enable_stages(krr_context ctx, uint32_t stage_mask) {
  if (!ctx) return KRR_ERROR_INVALID_VALUE;
  HIPCHK(hipSetDevice(ctx->device));
  timers_drain(ctx);
  for (int i = 0; i < KRR_STAGE_COUNT; ++i) {
    ctx->total_ms[i] = 0;
    ctx->intervals[i] = 0;
  }
  ctx->timing = stage_mask & ((1u << KRR_STAGE_COUNT) - 1u);
  return KRR_SUCCESS;
}

krr_status krr_timers_read(krr_context ctx, double *total_ms, int64_t *intervals, int32_t count) {
  if (!ctx || count < 0) return KRR_ERROR_INVALID_VALUE;
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  timers_drain(ctx);
  for (int i = 0; i < count && i < KRR_STAGE_COUNT; ++i) {
    if (total_ms) total_ms[i] = ctx->total_ms[i];
    if (intervals) intervals[i] = ctx->intervals[i];
  }
  return KRR_SUCCESS;
}

const char *krr_status_string(krr_status s) {
  switch (s) {
    case KRR_SUCCESS: return "success";
    case KRR_ERROR_INVALID_VALUE: return "invalid value";
    case KRR_ERROR_BAD_GENOTYPE: return "genotype value outside {0,1,2}";
    case KRR_ERROR_OUT_OF_MEMORY: return "out of device memory or workspace limit";
    case KRR_ERROR_NOT_POSITIVE_DEFINITE: return "matrix not positive definite (Cholesky breakdown)";
    case KRR_ERROR_NOT_CONVERGED: return "refinement did not converge";
    case KRR_ERROR_HIP: return "HIP runtime error";
    case KRR_ERROR_NOT_SUPPORTED: return "not supported";
    case KRR_ERROR_SCRATCH_TOO_SMALL:
      return "input needs more than the fixed scratch of the no-allocation entry point";
  }
  return "unknown status";
}

// Fixed device scratch of the no-allocation entry point (krr_predict_noalloc).
// Each device the library runs on holds its own copy of this array until the
// process ends.  In host code its name is a host-side stand-in: kernels and
// copies get the device address taken once per device (scratch_init, called by
// krr_create with that device current), never the name itself.
static __device__ __align__(256) uint8_t scratch[KRR_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int KRR_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[KRR_MAX_DEVICES] = {};

// The calling thread's current device must be `device`.
krr_status scratch_init(int device) {
  if (device < 0 || device >= KRR_MAX_DEVICES) return KRR_ERROR_NOT_SUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return KRR_SUCCESS;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return KRR_ERROR_HIP;
  }
  g_scratch_ptr[device] = p;
  return KRR_SUCCESS;
}

void *scratch_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return (device >= 0 && device < KRR_MAX_DEVICES) ? g_scratch_ptr[device] : nullptr;
}
}  // namespace

krr_status krr_create(krr_context *out, int device, void *stream, const krr_options *opts) {
  if (!out) return KRR_ERROR_INVALID_VALUE;
  *out = nullptr;
  krr_options o{};
  if (opts) o = *opts;
  if (o.tile == 0) o.tile = 512;
  if (o.tile != 256 && o.tile != 512) return KRR_ERROR_INVALID_VALUE;
  if (o.workspace_limit < 0) return KRR_ERROR_INVALID_VALUE;
  if (!o.device_alloc != !o.device_free) return KRR_ERROR_INVALID_VALUE;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess) {
    (void)hipGetLastError();
    return KRR_ERROR_HIP;
  }
  if (device < 0 || device >= count) return KRR_ERROR_INVALID_VALUE;
  HIPCHK(hipSetDevice(device));
  CHK(scratch_init(device));
  build_kernel_attrs();
  factor_kernel_attrs();
  solve_kernel_attrs();
  krr_context c = new krr_context_s();
  c->device = device;
  c->stream = (hipStream_t)stream;
  c->opts = o;
  c->tune = krr_tuning{o.tile, 0, 0, -1, -1, 0};
  *out = c;
  return KRR_SUCCESS;
}

static void graphs_clear(krr_context ctx) {
  for (auto &kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
  ctx->graphs.clear();
}

static void context_free(krr_context ctx) {
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  graphs_clear(ctx);
  for (int q = 0; q < 2; ++q) dfree(ctx, ctx->jobtab[q], ctx->jobtab_bytes[q]);
  timers_drain(ctx);
  for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
  cache_flush(ctx);
  for (hipStream_t x : {ctx->side, ctx->fmain, ctx->cap, ctx->sw2}) {
    if (x) {
      (void)hipStreamSynchronize(x);
      (void)hipStreamDestroy(x);
    }
  }
  for (hipStream_t x : ctx->aux_by_e) {
    if (x) {
      (void)hipStreamSynchronize(x);
      (void)hipStreamDestroy(x);
    }
  }
  for (hipEvent_t e : ctx->sched_ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : ctx->sweep_ev) (void)hipEventDestroy(e);
  delete ctx;
}

// The factorization's three streams (default priority): its own main stream
// (the critical path), a side stream and an aux stream.
// The aux stream (the wide trailing updates, off the critical path) may be
// limited to q eighths of the compute units, so that the main and side
// streams find free ones: CU i is enabled when (i / 8) % 8 < q.  Measured at
// n = 32768, seven eighths took the adaptive path from 81.9-82.4 to
// 80.8-81.3 ms per step (its diagonal chain no longer starves while the wide
// update fills the chip at a group start) and the plain FP32 path, whose wide
// updates are most of its work, from 138 to 207 ms; but a masked stream is a
// hardware queue of its own, and with masked streams in one context a second
// context's factorization in the same process ran 17% slower (161 against
// 137 ms).  So no mask by default (tuning 0); each mask's stream is made once
// per context and kept.  KRR_AUX_CU_EIGHTHS overrides the tuning.
static krr_status context_aux(krr_context ctx, bool low_precision) {
  (void)low_precision;
  for (hipStream_t *x : {&ctx->fmain, &ctx->side})
    if (!*x) HIPCHK(hipStreamCreateWithFlags(x, hipStreamNonBlocking));
  const char *e = getenv("KRR_AUX_CU_EIGHTHS");
  int q = e ? atoi(e) : ctx->tune.aux_cu_eighths;
  if (q == 0) q = 8;
  if (q < 0 || q > 8) q = 8;
  if (!ctx->aux_by_e[q]) {
    int ncu = 0;
    HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device));
    hipStream_t st = nullptr;
    if (q < 8 && ncu > 0) {
      std::vector<uint32_t> mask((ncu + 31) / 32, 0u);
      for (int i = 0; i < ncu; ++i)
        if (((i >> 3) & 7) < q) mask[i / 32] |= 1u << (i % 32);
      if (hipExtStreamCreateWithCUMask(&st, (uint32_t)mask.size(), mask.data()) != hipSuccess) {
        (void)hipGetLastError();
        st = nullptr;
      }
    }
    if (!st) HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    ctx->aux_by_e[q] = st;
  }
  ctx->aux = ctx->aux_by_e[q];
  ctx->aux_e = q;
  return KRR_SUCCESS;
}

// A handle was released: free the context if it was destroyed while handles lived.
static void context_unref(krr_context ctx) {
  if (--ctx->live == 0 && ctx->destroy_pending) context_free(ctx);
}

krr_status krr_destroy(krr_context ctx) {
  if (!ctx || ctx->destroy_pending) return KRR_ERROR_INVALID_VALUE;
  if (ctx->live > 0) {
    ctx->destroy_pending = true;  // freed when the last kernel/factor is released
    return KRR_SUCCESS;
  }
  context_free(ctx);
  return KRR_SUCCESS;
}

krr_status krr_set_stream(krr_context ctx, void *stream) {
  if (!ctx) return KRR_ERROR_INVALID_VALUE;
  ctx->stream = (hipStream_t)stream;
  return KRR_SUCCESS;
}

static void kernel_free(krr_kernel K) {
  krr_context c = K->ctx;
  const TileLayout &L = K->L;
  dfree(c, K->D, (size_t)L.elems() * 4);
  dfree(c, K->A, (size_t)L.elems() * 4);
  dfree(c, K->nrm, (size_t)L.np * 4);
  dfree(c, K->etab, (size_t)K->etab_len * 8);
  dfree(c, K->H, (size_t)K->n * K->ldh);
  dfree(c, K->Cc, (size_t)K->n * K->q * 8);
  dfree(c, K->Ec, (size_t)L.elems() * 8);
  dfree(c, K->tnorm, (size_t)L.ntiles() * 8);
  dfree(c, K->Gs, (size_t)K->gs_bytes);
  const int sb = L.nb / 256;
  dfree(c, K->tnorm_part, (size_t)L.ntiles() * sb * sb * 8);
}

static krr_status build_args(const int8_t *G, int64_t n, int64_t m, int64_t ldg, double gamma,
                             double lambda) {
  if (!G || n <= 0 || m <= 0 || ldg < m || (ldg % 16) != 0 || !aligned16(G))
    return KRR_ERROR_INVALID_VALUE;
  if (!(gamma > 0) || !isfinite(gamma) || !(lambda >= 0) || !isfinite(lambda))
    return KRR_ERROR_INVALID_VALUE;
  if (m > (1LL << 28) || n > (1LL << 30)) return KRR_ERROR_NOT_SUPPORTED;
  return KRR_SUCCESS;
}

// A kernel handle with its device buffers allocated (contents not yet built).
static krr_status kernel_new(krr_context ctx, const int8_t *G, int64_t n, int64_t m, int64_t ldg,
                             double gamma, double lambda, krr_kernel *out) {
  krr_kernel K = new krr_kernel_s();
  K->ctx = ctx;
  K->G = G;
  K->n = n;
  K->m = m;
  K->ldg = ldg;
  K->gamma = gamma;
  K->lambda = lambda;
  K->L = make_layout(n, ctx->opts.tile);
  const TileLayout &L = K->L;
  K->etab_len = 4 * m + 1;
  const int sb = L.nb / 256;
  krr_status st = KRR_SUCCESS;
  do {
    if ((st = dalloc_t(ctx, &K->D, L.elems())) != KRR_SUCCESS) break;
    if ((st = dalloc_t(ctx, &K->A, L.elems())) != KRR_SUCCESS) break;
    if ((st = dalloc_t(ctx, &K->nrm, L.np)) != KRR_SUCCESS) break;
    if ((st = dalloc_t(ctx, &K->etab, K->etab_len)) != KRR_SUCCESS) break;
    if ((st = dalloc_t(ctx, &K->tnorm, L.ntiles())) != KRR_SUCCESS) break;
    if ((st = dalloc_t(ctx, &K->tnorm_part, L.ntiles() * sb * sb)) != KRR_SUCCESS) break;
  } while (0);
  if (st != KRR_SUCCESS) {
    kernel_free(K);
    delete K;
    K = nullptr;
  }
  *out = K;
  return st;
}

krr_status krr_build_kernel(krr_context ctx, const int8_t *G, int64_t n, int64_t m, int64_t ldg,
                            double gamma, double lambda, krr_kernel *out) {
  return krr_build_kernel_ex(ctx, G, n, m, ldg, gamma, lambda, nullptr, out);
}

krr_status krr_build_kernel_ex(krr_context ctx, const int8_t *G, int64_t n, int64_t m, int64_t ldg,
                               double gamma, double lambda, const krr_kernel_desc *desc,
                               krr_kernel *out) {
  if (!out) return KRR_ERROR_INVALID_VALUE;
  *out = nullptr;
  if (!ctx || ctx->destroy_pending) return KRR_ERROR_INVALID_VALUE;
  CHK(build_args(G, n, m, ldg, gamma, lambda));
  krr_kernel_desc dsc{};
  if (desc) dsc = *desc;
  if (dsc.kind != KRR_KERNEL_GAUSSIAN && dsc.kind != KRR_KERNEL_IBS &&
      dsc.kind != KRR_KERNEL_LINEAR)
    return KRR_ERROR_INVALID_VALUE;
  if (dsc.C) {
    if (dsc.kind != KRR_KERNEL_GAUSSIAN || dsc.q <= 0 || dsc.ldc < dsc.q) return KRR_ERROR_INVALID_VALUE;
    if (dsc.q > KRR_CONF_QMAX) return KRR_ERROR_NOT_SUPPORTED;
  }
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  krr_kernel K = nullptr;
  CHK(kernel_new(ctx, G, n, m, ldg, gamma, lambda, &K));
  K->kind = dsc.kind;
  const TileLayout &L = K->L;
  const int sb = L.nb / 256;
  krr_status st = KRR_SUCCESS;
  int32_t *flag = nullptr;
  do {
    if ((st = dalloc_t(ctx, &flag, 1)) != KRR_SUCCESS) break;
    if (K->kind == KRR_KERNEL_IBS) {
      // encoded rows: [g >= 1] then [g >= 2], each half padded to 16 bytes; the
      // squared distance of two encoded rows is sum_k |g_ik - g_jk| <= 2m
      K->ldh = 2 * ((m + 15) / 16 * 16);
      if ((st = dalloc_t(ctx, &K->H, n * K->ldh)) != KRR_SUCCESS) break;
      dfree(ctx, K->etab, (size_t)K->etab_len * 8);
      K->etab = nullptr;
      K->etab_len = 2 * m + 1;
      if ((st = dalloc_t(ctx, &K->etab, K->etab_len)) != KRR_SUCCESS) break;
    }
    if (dsc.C) {
      K->q = dsc.q;
      if ((st = dalloc_t(ctx, &K->Cc, n * dsc.q)) != KRR_SUCCESS) break;
      if ((st = dalloc_t(ctx, &K->Ec, L.elems())) != KRR_SUCCESS) break;
      if (hipMemcpy2DAsync(K->Cc, dsc.q * 8, dsc.C, dsc.ldc * 8, dsc.q * 8, n,
                           hipMemcpyDeviceToDevice, s) != hipSuccess) {
        st = KRR_ERROR_HIP;
        break;
      }
    }
    launch_fill_i32(flag, 1, 0, s);
    // the genotypes slab-major for the Gram (kept with the kernel until its
    // release); KRR_GRAM_SLAB=0 streams the row-major matrix instead
    static const bool slab = [] {
      const char *e = getenv("KRR_GRAM_SLAB");
      return !e || atoi(e) != 0;
    }();
    if (slab) {
      K->gs_bytes = L.np * ((K->gram_m() + 63) / 64) * 64;
      if ((st = dalloc_t(ctx, &K->Gs, K->gs_bytes)) != KRR_SUCCESS) break;
    }
    {
      Stage t(ctx, KRR_STAGE_ROW_NORMS);  // the genotypes' preparation
      if (K->Gs && !K->H) {  // the slab-major copy, the row norms and the check in one pass
        launch_slab_major_norms(G, n, L.np, m, ldg, K->Gs, K->nrm, flag, s);
      } else {
        launch_row_norms(G, n, L.np, m, ldg, K->nrm, flag, s);  // and the genotype check
        if (K->H) {
          launch_ibs_encode(G, n, m, ldg, K->H, K->ldh, s);
          launch_row_norms(K->H, n, L.np, K->ldh, K->ldh, K->nrm, flag, s);
        }
        if (K->Gs)
          launch_slab_major(K->gram_src(), n, L.np, K->gram_m(), K->gram_ld(), K->Gs, s);
      }
    }
    int32_t hflag = 0;
    if (hipMemcpyAsync(&hflag, flag, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      st = KRR_ERROR_HIP;
      break;
    }
    if ((st = launch_ok()) != KRR_SUCCESS) break;
    if (hflag) {
      st = KRR_ERROR_BAD_GENOTYPE;
      break;
    }
    if (K->kind == KRR_KERNEL_IBS) launch_ibs_table(K->etab, K->etab_len, m, s);
    else if (K->kind == KRR_KERNEL_GAUSSIAN) launch_exp_table(K->etab, K->etab_len, gamma, s);
    if (K->Ec) launch_conf_factor(K->Cc, n, K->q, K->q, gamma, L, K->Ec, s);
    {
      Stage t(ctx, KRR_STAGE_GRAM);
      launch_gram_tiles(K->gram_src(), K->gram_m(), K->gram_ld(), K->nrm, K->etab, K->etab_len,
                        lambda, L, K->D, K->A, K->tnorm_part, K->vmode(), K->Ec, K->Gs, s);
    }
    launch_tile_norms(K->tnorm_part, sb * sb, L.ntiles(), K->tnorm, s);
    st = launch_ok();
  } while (0);
  if (flag) dfree(ctx, flag, 4);
  if (st != KRR_SUCCESS) {
    kernel_free(K);
    delete K;
    return st;
  }
  ctx->live++;
  *out = K;
  return KRR_SUCCESS;
}

static void norm_from_tiles(krr_kernel K) {
  const TileLayout &L = K->L;
  double s = 0.0;
  for (int I = 0; I < L.nt; ++I)
    for (int J = 0; J <= I; ++J) {
      const double v = K->tnorm_host[TileLayout::tri(I, J)];
      s += (I == J ? 1.0 : 2.0) * v * v;
    }
  // padding rows contribute identity entries (1 each) to the stored tiles
  s -= (double)(L.np - L.n);
  K->norm_a = sqrt(s > 0 ? s : 0.0);
}

krr_status krr_build_kernel_batched(krr_context ctx, int32_t batch, const int8_t *const *G,
                                    const int64_t *n, int64_t m, const int64_t *ldg,
                                    const double *gamma, const double *lambda, krr_kernel *out) {
  if (!out || batch <= 0) return KRR_ERROR_INVALID_VALUE;
  for (int b = 0; b < batch; ++b) out[b] = nullptr;
  if (!ctx || ctx->destroy_pending || !G || !n || !ldg || !gamma || !lambda)
    return KRR_ERROR_INVALID_VALUE;
  for (int b = 0; b < batch; ++b) CHK(build_args(G[b], n[b], m, ldg[b], gamma[b], lambda[b]));
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  // largest instances first, so that the small ones fill the tail of each launch
  std::vector<int> order(batch);
  for (int b = 0; b < batch; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return n[a] > n[b]; });
  std::vector<krr_kernel> Ks(batch, nullptr);
  std::vector<BuildJob> jobs(batch);
  std::vector<int32_t> hflags(batch, 0);
  BuildJob *djobs = nullptr;
  int32_t *flags = nullptr;
  krr_status st = KRR_SUCCESS;
  do {
    int64_t rows = 0, blocks = 0, max_len = 0, max_tiles = 0;
    for (int q = 0; q < batch && st == KRR_SUCCESS; ++q) {
      const int b = order[q];
      st = kernel_new(ctx, G[b], n[b], m, ldg[b], gamma[b], lambda[b], &Ks[b]);
      if (st != KRR_SUCCESS) break;
      krr_kernel K = Ks[b];
      BuildJob &j = jobs[q];
      j.G = G[b];
      j.n = n[b];
      j.np = K->L.np;
      j.ldg = ldg[b];
      j.nrm = K->nrm;
      j.flag = nullptr;  // set below
      j.etab = K->etab;
      j.etab_len = K->etab_len;
      j.gamma = gamma[b];
      j.lambda = lambda[b];
      j.D = K->D;
      j.A = K->A;
      j.part = K->tnorm_part;
      j.tnorm = K->tnorm;
      j.ntiles = K->L.ntiles();
      j.row0 = rows;
      j.block0 = blocks;
      rows += K->L.np;
      blocks += gram_blocks(K->L);
      max_len = std::max(max_len, K->etab_len);
      max_tiles = std::max(max_tiles, K->L.ntiles());
    }
    if (st != KRR_SUCCESS) break;
    if ((st = dalloc_t(ctx, &djobs, batch)) != KRR_SUCCESS) break;
    if ((st = dalloc_t(ctx, &flags, batch)) != KRR_SUCCESS) break;
    for (int q = 0; q < batch; ++q) jobs[q].flag = flags + q;
    if (hipMemcpy(djobs, jobs.data(), sizeof(BuildJob) * batch, hipMemcpyHostToDevice) !=
        hipSuccess) {
      st = KRR_ERROR_HIP;
      break;
    }
    launch_fill_i32(flags, batch, 0, s);
    {
      Stage t(ctx, KRR_STAGE_ROW_NORMS);
      launch_row_norms_batched(djobs, batch, rows, m, s);
    }
    if (hipMemcpyAsync(hflags.data(), flags, 4 * batch, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      st = KRR_ERROR_HIP;
      break;
    }
    if ((st = launch_ok()) != KRR_SUCCESS) break;
    for (int q = 0; q < batch; ++q)
      if (hflags[q]) st = KRR_ERROR_BAD_GENOTYPE;
    if (st != KRR_SUCCESS) break;
    launch_exp_tables_batched(djobs, batch, max_len, s);
    {
      Stage t(ctx, KRR_STAGE_GRAM);
      launch_gram_tiles_batched(djobs, batch, blocks, m, ctx->opts.tile, s);
    }
    launch_tile_norms_batched(djobs, batch, max_tiles, ctx->opts.tile, s);
    if ((st = launch_ok()) != KRR_SUCCESS) break;
    // the Frobenius norms the precision rule needs, all in one synchronization
    for (int b = 0; b < batch && st == KRR_SUCCESS; ++b) {
      krr_kernel K = Ks[b];
      K->tnorm_host.resize(K->L.ntiles());
      if (hipMemcpyAsync(K->tnorm_host.data(), K->tnorm, K->L.ntiles() * 8,
                         hipMemcpyDeviceToHost, s) != hipSuccess)
        st = KRR_ERROR_HIP;
    }
    if (st == KRR_SUCCESS && hipStreamSynchronize(s) != hipSuccess) st = KRR_ERROR_HIP;
  } while (0);
  if (djobs) dfree(ctx, djobs, sizeof(BuildJob) * batch);
  if (flags) dfree(ctx, flags, 4 * batch);
  if (st != KRR_SUCCESS) {
    for (krr_kernel K : Ks)
      if (K) {
        kernel_free(K);
        delete K;
      }
    return st;
  }
  for (int b = 0; b < batch; ++b) {
    norm_from_tiles(Ks[b]);
    out[b] = Ks[b];
    ctx->live++;
  }
  return KRR_SUCCESS;
}

krr_status krr_kernel_release(krr_kernel K) {
  if (!K) return KRR_ERROR_INVALID_VALUE;
  krr_context c = K->ctx;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  kernel_free(K);
  delete K;
  context_unref(c);
  return KRR_SUCCESS;
}

static krr_status kernel_norm(krr_kernel K) {
  if (K->norm_a >= 0) return KRR_SUCCESS;
  const TileLayout &L = K->L;
  K->tnorm_host.resize(L.ntiles());
  HIPCHK(hipMemcpyAsync(K->tnorm_host.data(), K->tnorm, L.ntiles() * 8, hipMemcpyDeviceToHost,
                        K->ctx->stream));
  HIPCHK(hipStreamSynchronize(K->ctx->stream));
  norm_from_tiles(K);
  return KRR_SUCCESS;
}

krr_status krr_kernel_tile_norms(krr_kernel K, double *host_dst, int64_t count) {
  if (!K || !host_dst || count < K->L.ntiles()) return KRR_ERROR_INVALID_VALUE;
  HIPCHK(hipSetDevice(K->ctx->device));
  CHK(kernel_norm(K));
  memcpy(host_dst, K->tnorm_host.data(), K->L.ntiles() * 8);
  return KRR_SUCCESS;
}

// Slots of the split-K diagonal-tile load: up to KRR_MAX_GROUP chunks of
// every 64 x 64 block of the lower half of a tile.
static size_t load_part_bytes(const TileLayout &L) {
  const int NB = L.nb / 64;
  return (size_t)KRR_MAX_GROUP * (NB * (NB + 1) / 2) * 64 * 64 * 4;
}

static void factor_work_free(krr_context c, FactorWork &w, const TileLayout &L) {
  const int64_t te = L.tile_elems(), pt = std::max(L.nt - 1, 1);
  const int parts = std::max((L.nb / 64) * (L.nb / 64), L.nb / 16);
  const int64_t chunk = std::min(w.inv_chunk, L.nt);
  dfree(c, w.W64, te * 8);
  dfree(c, w.WL64, L.nt * te * 8);
  dfree(c, w.Dinv64, (int64_t)L.nt * L.nb * 64 * 8);
  dfree(c, w.Winv64, chunk * te * 8);
  dfree(c, w.Tmp64, chunk * te / 2 * 8);
  for (PanelBuf &pb : w.pb) {  // unallocated slots hold null pointers
    dfree(c, pb.P32, pt * te * 4);
    dfree(c, pb.P16, pt * te * 2);
    dfree(c, pb.P8, pt * te);
    dfree(c, pb.pnorm, (pt + 2) * 4);
    dfree(c, pb.pexp8, pt * 4);
  }
  dfree(c, w.pnorm_part, pt * parts * 8);
  dfree(c, w.pmax_part, pt * parts * 4);
  dfree(c, w.flag, 4);
  dfree(c, w.counts, 3 * 8);
  dfree(c, w.lpart, load_part_bytes(L));
  dfree(c, w.WX64, te * 8);
  w = FactorWork();
}

static krr_status factor_work_alloc(krr_context c, FactorWork &w, const TileLayout &L,
                                    bool need16, bool need8, int slots, bool split_load = true) {
  const int64_t te = L.tile_elems(), pt = std::max(L.nt - 1, 1);
  const int parts = std::max((L.nb / 64) * (L.nb / 64), L.nb / 16);
  const int64_t chunk = std::min(w.inv_chunk, L.nt);
  krr_status st;
#define WA(ptr, cnt)                                                        \
  if ((st = dalloc(c, (void **)&(ptr), (size_t)(cnt))) != KRR_SUCCESS) { \
    factor_work_free(c, w, L);                                            \
    return st;                                                            \
  }
  WA(w.W64, te * 8);
  WA(w.WL64, L.nt * te * 8);
  WA(w.Dinv64, (int64_t)L.nt * L.nb * 64 * 8);
  WA(w.Winv64, chunk * te * 8);
  WA(w.Tmp64, chunk * te / 2 * 8);
  for (int q = 0; q < slots; ++q) {
    PanelBuf &pb = w.pb[q];
    WA(pb.P32, pt * te * 4);
    WA(pb.P16, need16 ? pt * te * 2 : 16);
    WA(pb.P8, need8 ? pt * te : 16);
    WA(pb.pnorm, (pt + 2) * 4);  // + the norms' extremes
    WA(pb.pexp8, pt * 4);
  }
  WA(w.pnorm_part, pt * parts * 8);
  WA(w.pmax_part, pt * parts * 4);
  WA(w.flag, 4);
  WA(w.counts, 3 * 8);
  if (split_load) {  // single instance: split-K tile loads, the next row's panel in the steps
    WA(w.lpart, load_part_bytes(L));
    WA(w.WX64, te * 8);
  }
#undef WA
  return KRR_SUCCESS;
}

// Precisions in force for one factorization attempt.
struct FactorPlan {
  int mode;
  int allow16, allow8;
  bool diag64;
};

static krr_status resolve_policy(const krr_precision_policy *policy, krr_precision_policy &p,
                                 FactorPlan &fp) {
  p = krr_precision_policy{};
  if (policy) {
    p = *policy;
  } else {
    p.mode = KRR_POLICY_ADAPTIVE;
    p.allowed = (1 << KRR_PREC_FP16) | (1 << KRR_PREC_FP8);
    p.eps = 1.0;
    p.high_panels = 1;
    p.allow_promotion = 1;
    p.diag_fp64 = 1;
  }
  if (p.mode < KRR_POLICY_FP32 || p.mode > KRR_POLICY_FIXED_MAP) return KRR_ERROR_INVALID_VALUE;
  if (p.mode == KRR_POLICY_ADAPTIVE && !(p.eps > 0)) return KRR_ERROR_INVALID_VALUE;
  if (p.mode == KRR_POLICY_ADAPTIVE && (p.rule < KRR_RULE_OPERAND || p.rule > KRR_RULE_BOTH))
    return KRR_ERROR_INVALID_VALUE;
  if (p.mode == KRR_POLICY_FIXED && p.fixed_prec != KRR_PREC_FP16 && p.fixed_prec != KRR_PREC_FP8)
    return KRR_ERROR_INVALID_VALUE;
  if (p.mode == KRR_POLICY_FIXED_MAP && (!p.fixed_map || p.fixed_map_count <= 0))
    return KRR_ERROR_INVALID_VALUE;
  if (p.high_panels < 0) return KRR_ERROR_INVALID_VALUE;
  fp.allow16 = fp.allow8 = 0;
  if (p.mode == KRR_POLICY_ADAPTIVE) {
    fp.allow16 = (p.allowed >> KRR_PREC_FP16) & 1;
    fp.allow8 = (p.allowed >> KRR_PREC_FP8) & 1;
  } else if (p.mode == KRR_POLICY_FIXED) {
    fp.allow16 = p.fixed_prec == KRR_PREC_FP16;
    fp.allow8 = p.fixed_prec == KRR_PREC_FP8;
  } else if (p.mode == KRR_POLICY_FIXED_MAP) {
    for (int64_t e = 0; e < p.fixed_map_count; ++e) {
      fp.allow16 |= p.fixed_map[e] == KRR_PREC_FP16;
      fp.allow8 |= p.fixed_map[e] == KRR_PREC_FP8;
    }
  }
  fp.mode = p.mode;
  fp.diag64 = p.diag_fp64 != 0;
  return KRR_SUCCESS;
}

// After a breakdown in tile row `brow`: every panel before it may use one
// precision level less than before (cap: the lowest precision a panel may
// use); when all of them are FP32 already, FP64 pivots.  False when nothing
// is left to promote.
static bool promote_panels(std::vector<uint8_t> &cap, int brow, FactorPlan &fp) {
  bool changed = false;
  for (int k = 0; k < brow && k < (int)cap.size(); ++k)
    if (cap[k] > KRR_PREC_FP32) {
      cap[k]--;
      changed = true;
    }
  if (changed) return true;
  if (!fp.diag64) {
    fp.diag64 = true;
    return true;
  }
  return false;
}

// Panels per grouped trailing update (KRR_GROUP overrides): 8 when updates
// may run in FP16/FP8 -- cheap updates, so deeper products and fewer
// launches pay -- and 4 for FP32 updates, whose groups are long enough
// already and whose updates overlap the factorization better in smaller
// pieces (measured at n = 32768: FP8 88.3 ms with 8 against 89.5 with 4,
// FP32 142 ms with 4 against 148 with 8; 48 instances in lockstep: FP8
// 215 ms with 8 against 218 with 4, FP32 272 ms with 4 against 279 with 8).
static int panel_group(const FactorPlan &fp) { return (fp.allow8 || fp.allow16) ? 8 : 4; }

// The group size in force: KRR_GROUP (debugging), else the context's tuning,
// else the default above.
static int group_size(krr_context ctx, const FactorPlan &fp) {
  const char *g_env = getenv("KRR_GROUP");
  const int g = g_env ? atoi(g_env)
                      : (ctx->tune.panel_group > 0 ? ctx->tune.panel_group : panel_group(fp));
  return std::max(1, std::min(KRR_MAX_GROUP, g));
}

// Enqueue one factorization attempt of F (its matrix already in F->Lst):
// clears the breakdown flag, the counters and the precision map, runs the
// tile Cholesky on s (one stream) or on the context's three streams joined
// back into s (lookahead), and counts the updates per precision.  Nothing
// here waits for the device.
// The lookahead schedule's events (4 NT + 2 groups + 5), created ahead of use
// (and of any capture of the schedule).
static bool sched_events(krr_context ctx, int NT, int g) {
  std::vector<hipEvent_t> &E = ctx->sched_ev;
  const size_t need = (size_t)4 * NT + 2 * ((NT + g - 1) / g) + 5;
  while (E.size() < need) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return false;
    E.push_back(e);
  }
  return true;
}

static krr_status factor_enqueue(krr_context ctx, krr_kernel K, krr_factorization F,
                                 const krr_precision_policy &p, const FactorPlan &fp,
                                 FactorWork &w, uint8_t *dmap, int64_t mapsz,
                                 const uint8_t *fmap, const uint8_t *pcap, bool lookahead,
                                 int g, hipStream_t s) {
  const TileLayout &L = F->L;
  launch_fill_i32(w.flag, 1, 0, s);
  launch_fill_i32((int32_t *)w.counts, 6, 0, s);
  launch_fill_u8(dmap, mapsz, 255, s);
  UpdatePolicy up;
  up.mode = fp.mode;
  up.allow16 = fp.allow16;
  up.allow8 = fp.allow8;
  up.high_panels = p.high_panels;
  up.fixed_prec = p.fixed_prec;
  up.rule = p.rule;
  up.thr = p.eps * K->norm_a / L.nt;
  up.fmap = fmap;
  up.pcap = pcap;
  up.tnorm = K->tnorm;
  // FP16 operands: chosen by the rule, or FP8 ones promoted a level after a breakdown
  up.have16 = fp.allow16 || (fp.allow8 && p.allow_promotion);
  const bool need16 = up.have16 != 0, need8 = fp.allow8 != 0;
  const bool scale8 = p.no_fp8_scale == 0;
  const int64_t te = L.tile_elems();
  // Panels are produced in groups of g block columns.  Inside a group
  // each panel updates the group's later columns right away; everything
  // to the right of the group gets one update by the whole group (K = g nb).
  auto slot = [&](int k) -> PanelBuf & { return w.pb[((k / g) & 1) * g + (k % g)]; };
  auto panels = [&](int G0, int npan, const PanelBuf **ps) {
    for (int q = 0; q < npan; ++q) ps[q] = &slot(G0 + q);
  };
  // POTRF(k); the updates of tile (k, k) by panels q0 .. q0+nq-1 are folded in;
  // with row.A, the panel's row tile k+1 formed in the same steps
  auto potrf = [&](int k, int q0, int nq, hipStream_t st, const RowPanel &row = RowPanel{}) {
    DiagUpdate du{};
    du.npan = nq;
    du.pmap = dmap;
    for (int q = 0; q < nq; ++q) {
      du.P[q] = slot(q0 + q).P32 + (int64_t)(k - (q0 + q) - 1) * te;
      du.pmap_at[q] = (int64_t)(q0 + q) * L.ntiles() + TileLayout::tri(k, k);
    }
    Stage t(ctx, KRR_STAGE_POTRF, st);
    // with the lookahead schedule the steps also form the FP32 factor tile and
    // the tile inverse but for its last block row (off the side stream)
    launch_potrf_tile(F->Lst + TileLayout::tri(k, k) * te, k, L, fp.diag64, w, du,
                      lookahead ? F->Linv + (int64_t)k * te : nullptr, st, row);
  };
  // TRSM of panel k, tiles k+1+t_lo .. : by substitution (no inverse) or
  // as a product with inv(L_kk) after forming it
  auto trsm_subst = [&](int k, int t_lo, int t_hi, hipStream_t st) {
    Stage t(ctx, KRR_STAGE_TRSM, st);
    launch_trsm_subst(F->Lst, k, L, fp.diag64, w, slot(k), t_lo, t_hi, st);
  };
  auto trsm_gemm = [&](int k, int t_lo, int t_hi, hipStream_t st) {
    {
      Stage t(ctx, KRR_STAGE_POTRF, st);
      launch_tile_inverse_last_row(F->Linv + (int64_t)k * te, k, L, fp.diag64, w, st);
    }
    Stage t(ctx, KRR_STAGE_TRSM, st);
    launch_trsm_gemm(F->Lst, F->Linv + (int64_t)k * te, k, L, w, slot(k), t_lo, t_hi, st);
  };
  auto convert = [&](int k, hipStream_t st) {
    Stage t(ctx, KRR_STAGE_CONVERT, st);
    launch_convert_panel(F->Lst, k, L, w, scale8, slot(k), need16, need8, &up, st);
  };
  // panels G0 .. G0+npan-1 onto the tiles of columns jlo .. jhi (which: UPD_*)
  auto update = [&](int G0, int npan, int jlo, int jhi, int which, hipStream_t st) {
    if (jlo > jhi || jlo >= L.nt) return;
    const PanelBuf *ps[KRR_MAX_GROUP];
    panels(G0, npan, ps);
    Stage t(ctx, KRR_STAGE_UPDATE, st);
    launch_update(F->Lst, G0, npan, jlo, jhi, L, up, w, ps, dmap, which, st);
  };
  const int NT = L.nt;
  if (!lookahead) {
    // One stream, in program order, with few launches per tile (this path
    // serves many small instances at once): the panel by substitution, and
    // the tile inverses (needed only by the solves) at the end, a chunk of
    // tiles per launch sequence.
    for (int G0 = 0; G0 < NT; G0 += g) {
      const int gend = std::min(G0 + g, NT);
      for (int k = G0; k < gend; ++k) {
        potrf(k, 0, 0, s);
        if (k + 1 < NT) {
          trsm_subst(k, 0, NT - 1 - k, s);
          convert(k, s);
        }
        // panel k onto the group's later diagonal tiles; column k+1 below the
        // diagonal gets the group's panels G0 .. k in one product
        update(k, 1, k + 1, gend - 1, UPD_DIAG, s);
        if (k + 1 < gend) update(G0, k - G0 + 1, k + 1, k + 1, UPD_OFFDIAG, s);
      }
      update(G0, gend - G0, gend, NT - 1, UPD_ALL, s);
    }
    Stage t(ctx, KRR_STAGE_POTRF, s);
    launch_tile_inverses(F->Lst, F->Linv, 0, NT, L, fp.diag64, w, s);
  } else {
    // Three streams.  Main, the critical path: POTRF(k) (with the tile's
    // last updates folded into its load) and the TRSM of row k+1 alone.
    // Side: the rest of each panel's TRSM, its operand copies, its updates
    // of the group's later columns, and the group's update of the next
    // group's columns.  Aux: each group's update of every column beyond the
    // next group, started after the update of the next group's columns.
    // Events order all updates of any one tile, so the factor does not
    // depend on the schedule.
    hipStream_t sm = ctx->fmain, sd = ctx->side, sx = ctx->aux;
    const int ngroups = (NT + g - 1) / g;
    // KRR_ROW_IN_STEPS=1: row tile k+1 of panel k formed inside POTRF(k)'s
    // steps, in place of the substitution TRSM launch after them.  Measured
    // slower (72.4 against 66.7 ms a benchmark step at tile 256): the steps
    // then wait for column k's updates on the side stream, which the later
    // TRSM launch waits for only after the tile's factorization.
    const char *ris = getenv("KRR_ROW_IN_STEPS");
    const bool row_in_steps = w.WX64 && ris && atoi(ris) != 0;
    std::vector<hipEvent_t> &E = ctx->sched_ev;
    bool ok = sched_events(ctx, NT, g);
    hipEvent_t *e_t1 = E.data(), *e_conv = e_t1 + NT, *e_uin = e_conv + NT,
               *e_udiag = e_uin + NT, *e_aux = e_udiag + NT, *e_narrow = e_aux + ngroups,
               *e_join = e_narrow + ngroups, e_early = e_join[4];
    // Panel 0 (FP32 under the adaptive policies, so its updates are the
    // costliest) goes to every column beyond the first group as soon as it
    // exists, on aux while the first group is factored; the first group's
    // boundary updates then carry panels 1 .. g-1 only.
    const bool early0 = NT > g && g > 1;
    auto rec = [&](hipEvent_t e, hipStream_t st) {
      ok = ok && hipEventRecord(e, st) == hipSuccess;
    };
    auto wait = [&](hipStream_t st, hipEvent_t e) {
      ok = ok && hipStreamWaitEvent(st, e, 0) == hipSuccess;
    };
    // all three start after the work already on the caller's stream
    rec(e_join[0], s);
    wait(sm, e_join[0]);
    wait(sd, e_join[0]);
    wait(sx, e_join[0]);
    for (int G0 = 0; G0 < NT && ok; G0 += g) {
      const int gi = G0 / g, gend = std::min(G0 + g, NT), nend = std::min(gend + g, NT);
      for (int k = G0; k < gend; ++k) {
        // tile (k, k) still lacks panel k-1 (inside the group) or the
        // whole previous group (at its start); the earlier panels of the
        // group reached it through the side stream's diagonal updates
        if (k >= G0 + 2) wait(sm, e_udiag[k - 2]);
        // row tile k+1 of the panel waits for column k's updates: the
        // in-group ones (side), or the previous group's update of this
        // group's columns (side)
        hipEvent_t col_ready = k > G0 ? e_uin[k - 1] : (gi > 0 ? e_narrow[gi - 1] : nullptr);
        RowPanel row;
        if (row_in_steps && k + 1 < NT) {
          row.A = F->Lst + TileLayout::tri(k + 1, k) * te;
          row.P32 = slot(k).P32;
          row.pnorm_part = w.pnorm_part;
          row.pmax_part = w.pmax_part;
          row.parts = trsm_parts(L.nb);
          row.wait = col_ready;
        }
        if (k > G0) {
          potrf(k, k - 1, 1, sm, row);
        } else if (early0 && gi == 1) {  // panel 0 reached it through aux
          wait(sm, e_early);
          potrf(k, 1, g - 1, sm, row);
        } else {
          potrf(k, std::max(G0 - g, 0), G0 > 0 ? g : 0, sm, row);
        }
        if (k + 1 >= NT) break;
        if (!row_in_steps) {
          if (col_ready) wait(sm, col_ready);
          trsm_subst(k, 0, 1, sm);
        }
        rec(e_t1[k], sm);
        wait(sd, e_t1[k]);
        trsm_gemm(k, 1, NT, sd);
        convert(k, sd);
        rec(e_conv[k], sd);
        if (early0 && k == 0) {
          wait(sx, e_conv[0]);
          update(0, 1, gend, NT - 1, UPD_ALL, sx);
          rec(e_early, sx);
        }
        // column k+1 below the diagonal gets every panel of the group so far
        // in one product (the later columns wait for their turn), which is
        // all the next TRSM needs; then the diagonal tiles further right
        if (k + 1 < gend) update(G0, k - G0 + 1, k + 1, k + 1, UPD_OFFDIAG, sd);
        rec(e_uin[k], sd);
        update(k, 1, k + 2, gend - 1, UPD_DIAG, sd);
        rec(e_udiag[k], sd);
      }
      if (gend >= NT) break;
      const int p0 = (early0 && gi == 0) ? 1 : 0;  // panel 0 already applied beyond
      const int q0 = G0 + p0, npan = gend - q0;
      // the next group's columns, after the previous group's aux update
      // reached them; its first diagonal tile on the main stream
      if (gi > 0) {
        wait(sm, e_aux[gi - 1]);
        wait(sd, e_aux[gi - 1]);
      }
      if (p0) wait(sd, e_early);
      update(q0, npan, gend, nend - 1, UPD_OFFDIAG, sd);
      update(q0, npan, gend + 1, nend - 1, UPD_DIAG, sd);
      rec(e_narrow[gi], sd);
      // aux: everything right of the next group, once the next group's
      // columns are done, so that the update the main stream waits for does
      // not share the chip with this much larger one
      if (nend < NT) {
        wait(sx, e_narrow[gi]);
        update(q0, npan, nend, NT - 1, UPD_ALL, sx);
      }
      rec(e_aux[gi], sx);
    }
    // join on the caller's stream
    rec(e_join[1], sd);
    rec(e_join[2], sx);
    rec(e_join[3], sm);
    wait(s, e_join[1]);
    wait(s, e_join[2]);
    wait(s, e_join[3]);
    if (!ok) return KRR_ERROR_HIP;
  }
  if (lookahead) {  // the last tile has no panel below it
    Stage t(ctx, KRR_STAGE_POTRF, s);
    launch_tile_inverse_last_row(F->Linv + (int64_t)(NT - 1) * te, NT - 1, L, fp.diag64, w, s);
  }
  launch_count_pmap(dmap, mapsz, w.counts, s);
  return KRR_SUCCESS;
}

static krr_status factor_run(krr_context ctx, krr_kernel K, krr_factorization F,
                             const krr_precision_policy &p, const FactorPlan &fp, FactorWork &w,
                             uint8_t *dmap, int64_t mapsz, const uint8_t *fmap,
                             const uint8_t *pcap, bool lookahead, int g, hipStream_t s);

krr_status krr_factor(krr_context ctx, krr_kernel K, const krr_precision_policy *policy,
                      krr_factorization *out) {
  if (!out) return KRR_ERROR_INVALID_VALUE;
  *out = nullptr;
  if (!ctx || !K || K->ctx != ctx) return KRR_ERROR_INVALID_VALUE;
  krr_precision_policy p;
  FactorPlan fp;
  CHK(resolve_policy(policy, p, fp));
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  const TileLayout &L = K->L;
  CHK(kernel_norm(K));
  const char *la_env = getenv("KRR_NO_LOOKAHEAD");
  const bool lookahead = la_env ? atoi(la_env) == 0 : ctx->tune.lookahead != 0;
  const int g = group_size(ctx, fp);
  if (lookahead) CHK(context_aux(ctx, fp.allow8 || fp.allow16));

  krr_factorization F = new krr_factor_s();
  F->ctx = ctx;
  F->K = K;
  F->L = L;
  F->info.nt = L.nt;
  F->info.tile = L.nb;
  F->info.norm_a = K->norm_a;
  F->info.breakdown_col = -1;
  FactorWork w;
  krr_status st = KRR_SUCCESS;
  uint8_t *dmap = nullptr, *fmap = nullptr, *pcap = nullptr;
  // precision of every (panel, tile) update; copied to the host for the
  // diagnostics accessor (NT^2 (NT+1) / 2 bytes: 30 MB at NT = 391)
  const int64_t mapsz = (int64_t)L.nt * L.ntiles();
  if (p.mode == KRR_POLICY_FIXED_MAP && p.fixed_map_count != mapsz) {
    delete F;
    return KRR_ERROR_INVALID_VALUE;
  }
  // lowest precision each panel may use; lowered panel by panel on breakdown
  std::vector<uint8_t> cap(L.nt, (uint8_t)KRR_PREC_FP8);
  do {
    if (K->A) {  // consume the build's matrix in place
      F->Lst = K->A;
      K->A = nullptr;
    } else {
      if ((st = dalloc_t(ctx, &F->Lst, L.elems())) != KRR_SUCCESS) break;
      launch_expand_tiles(K->D, K->etab, K->etab_len, K->lambda, K->vmode(), K->Ec, L,
                          F->Lst, s);
    }
    if ((st = dalloc_t(ctx, &F->Linv, (int64_t)L.nt * L.tile_elems())) != KRR_SUCCESS) break;
    if ((st = factor_work_alloc(ctx, w, L, fp.allow16 || p.allow_promotion, fp.allow8,
                                std::min(2 * g, 2 * KRR_MAX_GROUP))) != KRR_SUCCESS)
      break;
    if ((st = dalloc_t(ctx, &dmap, mapsz)) != KRR_SUCCESS) break;
    if ((st = dalloc_t(ctx, &pcap, L.nt)) != KRR_SUCCESS) break;
    if (p.mode == KRR_POLICY_FIXED_MAP) {
      if ((st = dalloc_t(ctx, &fmap, mapsz)) != KRR_SUCCESS) break;
      if (hipMemcpyAsync(fmap, p.fixed_map, mapsz, hipMemcpyHostToDevice, s) != hipSuccess) {
        st = KRR_ERROR_HIP;
        break;
      }
    }
    for (int attempt = 0;; ++attempt) {
      if (attempt > 0) launch_expand_tiles(K->D, K->etab, K->etab_len, K->lambda, K->vmode(), K->Ec, L,
                          F->Lst, s);
      // the caps (host memory, pageable): the copy completes before the call returns
      if (hipMemcpyAsync(pcap, cap.data(), L.nt, hipMemcpyHostToDevice, s) != hipSuccess) {
        st = KRR_ERROR_HIP;
        break;
      }
      if ((st = factor_run(ctx, K, F, p, fp, w, dmap, mapsz, fmap, pcap, lookahead, g, s)) !=
          KRR_SUCCESS)
        break;
      if ((st = launch_ok()) != KRR_SUCCESS) break;
      int32_t hflag = 0;
      unsigned long long hc[3] = {0, 0, 0};
      if (hipMemcpyAsync(&hflag, w.flag, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipMemcpyAsync(hc, w.counts, 24, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) {
        st = KRR_ERROR_HIP;
        break;
      }
      for (int q = 0; q < 3; ++q) F->info.updates[q] = (int64_t)hc[q];
      if (hflag == 0) break;
      F->info.breakdown_col = hflag - 1;
      if (!p.allow_promotion) {
        st = KRR_ERROR_NOT_POSITIVE_DEFINITE;
        break;
      }
      if (!promote_panels(cap, (int)((hflag - 1) / L.nb), fp)) {
        st = KRR_ERROR_NOT_POSITIVE_DEFINITE;
        break;
      }
      F->info.promotions++;
    }
    if (st == KRR_SUCCESS) {
      F->pmap.resize(mapsz);
      if (hipMemcpy(F->pmap.data(), dmap, mapsz, hipMemcpyDeviceToHost) != hipSuccess)
        st = KRR_ERROR_HIP;
    }
  } while (0);
  // on an error, work may still be in flight on the factorization's streams:
  // let it finish before its memory goes back to the cache
  if (st != KRR_SUCCESS) (void)hipDeviceSynchronize();
  if (dmap) dfree(ctx, dmap, mapsz);
  if (fmap) dfree(ctx, fmap, mapsz);
  if (pcap) dfree(ctx, pcap, L.nt);
  factor_work_free(ctx, w, L);
  if (st != KRR_SUCCESS) {
    dfree(ctx, F->Lst, L.elems() * 4);
    dfree(ctx, F->Linv, (size_t)L.nt * L.tile_elems() * 4);
    delete F;
    return st;
  }
  if (ctx->opts.verbose)
    fprintf(stderr, "krr_factor: n=%lld nt=%d updates fp32=%lld fp16=%lld fp8=%lld promotions=%d\n",
            (long long)L.n, L.nt, (long long)F->info.updates[0], (long long)F->info.updates[1],
            (long long)F->info.updates[2], F->info.promotions);
  ctx->live++;
  *out = F;
  return KRR_SUCCESS;
}

static void factor_free(krr_factorization F) {
  krr_context c = F->ctx;
  dfree(c, F->Lst, F->L.elems() * 4);
  dfree(c, F->Linv, (size_t)F->L.nt * F->L.tile_elems() * 4);
  if (F->Cpair) dfree(c, F->Cpair, (size_t)(F->L.nt / 2) * F->L.tile_elems() * 4);
  if (F->Cquad) dfree(c, F->Cquad, (size_t)4 * (F->L.nt / 4) * F->L.tile_elems() * 4);
  delete F;
}

// Run a fixed launch sequence through a HIP graph: captured from `enqueue`
// on the first call with a given key (the launch shape, including the device
// addresses the kernels are given), instantiated, kept in the context and
// replayed on later calls.  The sequence must hold kernel launches only.
// KRR_NO_GRAPH=1 enqueues directly.
constexpr size_t KRR_GRAPH_CACHE_MAX = 64;

// Job table `which` (0 factorization, 1 solve) of at least `bytes`, at the
// same address from call to call while it is large enough.  Only used on the
// context stream by calls that synchronize before returning.
static krr_status job_table(krr_context ctx, int which, size_t bytes, void **out) {
  if (ctx->jobtab_bytes[which] < bytes) {
    if (ctx->jobtab[which]) {
      HIPCHK(hipStreamSynchronize(ctx->stream));
      dfree(ctx, ctx->jobtab[which], ctx->jobtab_bytes[which]);
      ctx->jobtab[which] = nullptr;
      ctx->jobtab_bytes[which] = 0;
    }
    const size_t cap = std::max<size_t>(bytes, 4096);
    CHK(dalloc(ctx, &ctx->jobtab[which], cap));
    ctx->jobtab_bytes[which] = cap;
  }
  *out = ctx->jobtab[which];
  return KRR_SUCCESS;
}

static krr_status graph_run(krr_context ctx, const std::string &key, hipStream_t s,
                            const std::function<void(hipStream_t)> &enqueue) {
  const char *e = getenv("KRR_NO_GRAPH");
  if (e && atoi(e) != 0) {
    enqueue(s);
    return launch_ok();
  }
  auto it = ctx->graphs.find(key);
  if (it == ctx->graphs.end()) {
    if (ctx->graphs.size() >= KRR_GRAPH_CACHE_MAX) {
      HIPCHK(hipStreamSynchronize(s));  // no replay of an evicted graph is in flight
      graphs_clear(ctx);
    }
    // captured on a stream of the context's own (the caller's stream may be
    // the null stream, which cannot be captured); nothing runs while capturing
    if (!ctx->cap) HIPCHK(hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal));
    enqueue(ctx->cap);
    const hipError_t ce = hipStreamEndCapture(ctx->cap, &g);
    if (ce != hipSuccess || !g) {
      (void)hipGetLastError();
      if (g) (void)hipGraphDestroy(g);
      return KRR_ERROR_HIP;
    }
    hipGraphExec_t x = nullptr;
    const hipError_t ie = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
      (void)hipGetLastError();
      return KRR_ERROR_HIP;
    }
    it = ctx->graphs.emplace(key, x).first;
  }
  HIPCHK(hipGraphLaunch(it->second, s));
  ctx->graph_replays++;
  return launch_ok();
}

// One factorization attempt of a single instance, its launches enqueued
// directly.  (A HIP-graph form of the three-stream schedule -- captured once
// per key of every address and value its launches take, then replayed, to
// take the host's enqueue time off the critical path -- ended the process
// with a host segmentation fault in this call on its first GPU runs, also
// with the kernel attributes and the schedule's events set up before the
// capture; the cause is not known, so it is switched off: KRR_FACTOR_GRAPH=1
// returns KRR_ERROR_NOT_SUPPORTED.)
static krr_status factor_run(krr_context ctx, krr_kernel K, krr_factorization F,
                             const krr_precision_policy &p, const FactorPlan &fp, FactorWork &w,
                             uint8_t *dmap, int64_t mapsz, const uint8_t *fmap,
                             const uint8_t *pcap, bool lookahead, int g, hipStream_t s) {
  const char *e = getenv("KRR_FACTOR_GRAPH");
  if (e && atoi(e) != 0) return KRR_ERROR_NOT_SUPPORTED;
  return factor_enqueue(ctx, K, F, p, fp, w, dmap, mapsz, fmap, pcap, lookahead, g, s);
}

krr_status krr_context_graphs(krr_context ctx, int64_t *cached, int64_t *launches) {
  if (!ctx) return KRR_ERROR_INVALID_VALUE;
  if (cached) *cached = (int64_t)ctx->graphs.size();
  if (launches) *launches = ctx->graph_replays;
  return KRR_SUCCESS;
}

krr_status krr_factor_batched(krr_context ctx, int32_t batch, const krr_kernel *K,
                              const krr_precision_policy *policy, krr_factorization *out) {
  if (!out || batch <= 0) return KRR_ERROR_INVALID_VALUE;
  for (int b = 0; b < batch; ++b) out[b] = nullptr;
  if (!ctx || !K) return KRR_ERROR_INVALID_VALUE;
  for (int b = 0; b < batch; ++b) {
    if (!K[b] || K[b]->ctx != ctx) return KRR_ERROR_INVALID_VALUE;
    for (int c = 0; c < b; ++c)
      if (K[c] == K[b]) return KRR_ERROR_INVALID_VALUE;  // one factorization per kernel
  }
  krr_precision_policy p;
  FactorPlan fp;
  CHK(resolve_policy(policy, p, fp));
  if (p.mode == KRR_POLICY_FIXED_MAP) return KRR_ERROR_NOT_SUPPORTED;  // one map per instance
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  {  // Frobenius norms of kernels not built by the batched build, in one synchronization
    bool any = false;
    for (int b = 0; b < batch; ++b) {
      krr_kernel k = K[b];
      if (k->norm_a >= 0) continue;
      k->tnorm_host.resize(k->L.ntiles());
      HIPCHK(hipMemcpyAsync(k->tnorm_host.data(), k->tnorm, k->L.ntiles() * 8,
                            hipMemcpyDeviceToHost, s));
      any = true;
    }
    if (any) {
      HIPCHK(hipStreamSynchronize(s));
      for (int b = 0; b < batch; ++b)
        if (K[b]->norm_a < 0) norm_from_tiles(K[b]);
    }
  }
  const int g = group_size(ctx, fp);
  const bool need16 = fp.allow16 || p.allow_promotion;
  std::vector<FactorWork> W(batch);
  std::vector<krr_factorization> Fs(batch, nullptr);
  std::vector<uint8_t *> dmap(batch, nullptr);
  std::vector<int64_t> mapsz(batch, 0);
  std::vector<int> nts(batch);
  std::vector<FactorJob> jobs(batch);
  FactorJob *djobs = nullptr;
  std::vector<int32_t> hflag(batch, 0);
  std::vector<unsigned long long> hc(3 * (size_t)batch, 0);
  krr_status st = KRR_SUCCESS;
  do {
    // memory: each instance its own factor storage, workspace and map
    for (int b = 0; b < batch && st == KRR_SUCCESS; ++b) {
      const TileLayout &L = K[b]->L;
      krr_factorization F = Fs[b] = new krr_factor_s();
      F->ctx = ctx;
      F->K = K[b];
      F->L = L;
      F->info.nt = L.nt;
      F->info.tile = L.nb;
      F->info.norm_a = K[b]->norm_a;
      F->info.breakdown_col = -1;
      if (K[b]->A) {  // consume the build's matrix in place
        F->Lst = K[b]->A;
        K[b]->A = nullptr;
      } else {
        if ((st = dalloc_t(ctx, &F->Lst, L.elems())) != KRR_SUCCESS) break;
        launch_expand_tiles(K[b]->D, K[b]->etab, K[b]->etab_len, K[b]->lambda, K[b]->vmode(),
                            K[b]->Ec, L, F->Lst, s);
      }
      if ((st = dalloc_t(ctx, &F->Linv, (int64_t)L.nt * L.tile_elems())) != KRR_SUCCESS) break;
      mapsz[b] = (int64_t)L.nt * L.ntiles();
      if ((st = dalloc_t(ctx, &dmap[b], mapsz[b])) != KRR_SUCCESS) break;
      if ((st = factor_work_alloc(ctx, W[b], L, need16, fp.allow8,
                                  std::min(2 * g, KRR_SLOTS), false)) != KRR_SUCCESS)
        break;
      nts[b] = L.nt;
      launch_fill_i32(W[b].flag, 1, 0, s);
      launch_fill_i32((int32_t *)W[b].counts, 6, 0, s);
      launch_fill_u8(dmap[b], mapsz[b], 255, s);
      FactorJob &j = jobs[b];
      j = FactorJob{};
      j.Lst = F->Lst;
      j.Linv = F->Linv;
      j.W = W[b].W64;
      j.WL = W[b].WL64;
      j.Dinv = W[b].Dinv64;
      j.Winv = W[b].Winv64;
      j.Tmp = W[b].Tmp64;
      for (int q = 0; q < KRR_SLOTS; ++q) {
        j.P32[q] = W[b].pb[q].P32;
        j.P16[q] = W[b].pb[q].P16;
        j.P8[q] = W[b].pb[q].P8;
        j.pnorm[q] = W[b].pb[q].pnorm;
        j.pexp8[q] = W[b].pb[q].pexp8;
      }
      j.pnorm_part = W[b].pnorm_part;
      j.pmax_part = W[b].pmax_part;
      j.flag = W[b].flag;
      j.pmap = dmap[b];
      j.ntiles = L.ntiles();
      j.thr = p.eps * K[b]->norm_a / L.nt;
      j.tnorm = K[b]->tnorm;
      j.nt = L.nt;
    }
    if (st != KRR_SUCCESS) break;
    if ((st = job_table(ctx, 0, sizeof(FactorJob) * batch, (void **)&djobs)) != KRR_SUCCESS)
      break;
    if (hipMemcpyAsync(djobs, jobs.data(), sizeof(FactorJob) * batch, hipMemcpyHostToDevice, s) !=
        hipSuccess) {
      st = KRR_ERROR_HIP;
      break;
    }
    UpdatePolicy up;
    up.mode = fp.mode;
    up.allow16 = fp.allow16;
    up.allow8 = fp.allow8;
    up.high_panels = p.high_panels;
    up.fixed_prec = p.fixed_prec;
    up.rule = p.rule;
    up.have16 = fp.allow16;  // no promotion caps in the lockstep: FP16 only if the rule has it
    up.thr = 0;  // per instance, from the table (with the tile norms)
    {
      // every lockstep launch of the factorization in one graph, replayed for
      // batches of the same shape (the instances' pointers come from the table)
      char kb[256];
      snprintf(kb, sizeof kb, "factor|%p|%d|%d|%d|%d|%d|%d|%d|%d|%d|%d|%d|%d", (void *)djobs,
               batch, ctx->opts.tile, g, fp.diag64 ? 1 : 0, fp.allow16, fp.allow8,
               p.no_fp8_scale, up.mode, up.high_panels, up.fixed_prec, up.rule,
               (int)sizeof(FactorJob));
      std::string key = kb;
      for (int b = 0; b < batch; ++b) key += "|" + std::to_string(nts[b]);
      Stage t(ctx, KRR_STAGE_POTRF, s);
      st = graph_run(ctx, key, s, [&](hipStream_t cs) {
        launch_factor_lockstep(djobs, nts.data(), batch, ctx->opts.tile, g, up, fp.diag64,
                               fp.allow16 != 0, fp.allow8 != 0, p.no_fp8_scale == 0, cs);
      });
      if (st != KRR_SUCCESS) break;
    }
    for (int b = 0; b < batch; ++b) {
      launch_count_pmap(dmap[b], mapsz[b], W[b].counts, s);
      if (hipMemcpyAsync(&hflag[b], W[b].flag, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipMemcpyAsync(&hc[3 * b], W[b].counts, 24, hipMemcpyDeviceToHost, s) != hipSuccess)
        st = KRR_ERROR_HIP;
    }
    if (st == KRR_SUCCESS) st = launch_ok();
    if (st != KRR_SUCCESS) break;
    if (hipStreamSynchronize(s) != hipSuccess) {
      st = KRR_ERROR_HIP;
      break;
    }
    for (int b = 0; b < batch; ++b) {
      for (int q = 0; q < 3; ++q) Fs[b]->info.updates[q] = (int64_t)hc[3 * b + q];
      if (hflag[b] == 0) {
        Fs[b]->pmap.resize(mapsz[b]);
        if (hipMemcpy(Fs[b]->pmap.data(), dmap[b], mapsz[b], hipMemcpyDeviceToHost) != hipSuccess)
          st = KRR_ERROR_HIP;
      }
    }
  } while (0);
  if (st != KRR_SUCCESS) (void)hipDeviceSynchronize();  // nothing left in flight
  for (int b = 0; b < batch; ++b) {
    factor_work_free(ctx, W[b], K[b]->L);
    if (dmap[b]) dfree(ctx, dmap[b], mapsz[b]);
  }

  // an instance that broke down is factored again on its own, with promotion
  for (int b = 0; b < batch && st == KRR_SUCCESS; ++b) {
    if (hflag[b] == 0) continue;
    if (!p.allow_promotion) {
      st = KRR_ERROR_NOT_POSITIVE_DEFINITE;
      break;
    }
    factor_free(Fs[b]);
    Fs[b] = nullptr;
    krr_factorization F = nullptr;
    st = krr_factor(ctx, K[b], policy, &F);
    if (st == KRR_SUCCESS) {
      ctx->live--;  // counted once, below, with the others
      Fs[b] = F;
    }
  }
  if (st != KRR_SUCCESS) {
    for (krr_factorization F : Fs)
      if (F) factor_free(F);
    return st;
  }
  for (int b = 0; b < batch; ++b) {
    out[b] = Fs[b];
    ctx->live++;
  }
  return KRR_SUCCESS;
}

krr_status krr_factor_release(krr_factorization F) {
  if (!F) return KRR_ERROR_INVALID_VALUE;
  krr_context c = F->ctx;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  factor_free(F);  // the factor, the tile inverses and the sweeps' coupling tiles
  context_unref(c);
  return KRR_SUCCESS;
}

krr_status krr_factor_get_info(krr_factorization F, krr_factor_info *info) {
  if (!F || !info) return KRR_ERROR_INVALID_VALUE;
  *info = F->info;
  return KRR_SUCCESS;
}

krr_status krr_factor_precision_map(krr_factorization F, uint8_t *host_dst, int64_t count) {
  if (!F || !host_dst) return KRR_ERROR_INVALID_VALUE;
  if (F->pmap.empty()) return KRR_ERROR_NOT_SUPPORTED;
  if (count < (int64_t)F->pmap.size()) return KRR_ERROR_INVALID_VALUE;
  memcpy(host_dst, F->pmap.data(), F->pmap.size());
  return KRR_SUCCESS;
}

// pcg_ok: the call implements KRR_REFINE_PCG (krr_solve); elsewhere it is
// NOT_SUPPORTED and AUTO means IR.
static krr_status refine_args(const krr_refine_opts *opts, bool pcg_ok, krr_refine_opts &o) {
  o = krr_refine_opts{};
  if (opts) {
    o = *opts;
  } else {
    o.method = KRR_REFINE_IR;
    o.max_iters = 30;
    o.tol = 1e-6;
  }
  if (o.method < KRR_REFINE_NONE || o.method > KRR_REFINE_AUTO || o.max_iters < 0 || !(o.tol >= 0))
    return KRR_ERROR_INVALID_VALUE;
  if (o.method == KRR_REFINE_PCG && !pcg_ok) return KRR_ERROR_NOT_SUPPORTED;
  if (o.method == KRR_REFINE_AUTO && !pcg_ok) o.method = KRR_REFINE_IR;
  return KRR_SUCCESS;
}

// Device buffers of one solve; right-hand sides row-major np x r.
struct SolveBufs {
  double *Yr = nullptr, *Xr = nullptr, *Rr = nullptr, *cn = nullptr, *Pr = nullptr;
  float *Bf = nullptr, *Zf = nullptr, *Xf = nullptr;
  const float *C = nullptr;  // coupling tiles of the paired sweeps, or null
  const float *Q = nullptr;  // coupling tiles of the quad sweeps, or null
  double *cw = nullptr;      // workspace of the column reductions
  int z = 1;                 // column ranges of the residual (Pr holds z np r)
  bool once = false;         // residual with each stored tile read once (z = NT slots)
};

// The coupling tiles of the paired sweeps, formed on the first solve with a
// factor and kept with it; KRR_SWEEP_PAIRS=0 sweeps one tile per step.  At
// tile 256 with the wide panel launches the tiles go four a step, with the
// quads' coupling tiles formed the same way (KRR_SWEEP_QUADS=0: pairs).
static krr_status sweep_coupling(krr_context ctx, krr_factorization F, Scoped &sc, SolveBufs &b,
                                 hipStream_t s) {
  b.C = nullptr;
  b.Q = nullptr;
  const char *e = getenv("KRR_SWEEP_PAIRS");
  const TileLayout &L = F->L;
  const int64_t npair = L.nt / 2;
  // KRR_SWEEP_PAIRS=2 (one persistent launch per sweep) is switched off: its
  // first runs hung and the cause is not known
  if (e && atoi(e) == 2) return KRR_ERROR_NOT_SUPPORTED;
  const bool pairs = e ? atoi(e) != 0 : ctx->tune.sweep_pairs != 0;
  if (!pairs || npair == 0) return KRR_SUCCESS;
  if (!F->Cpair) {
    float *tmp = nullptr;
    CHK(sc.alloc(&tmp, npair * L.tile_elems()));
    CHK(dalloc_t(ctx, &F->Cpair, npair * L.tile_elems()));
    launch_sweep_coupling(F->Lst, F->Linv, L, tmp, F->Cpair, s);
  }
  b.C = F->Cpair;
  const char *eq = getenv("KRR_SWEEP_QUADS");
  const int64_t nquad = L.nt / 4;
  if ((eq && atoi(eq) == 0) || nquad == 0 || !sweep_quads_supported(L.nb)) return KRR_SUCCESS;
  if (!F->Cquad) {
    float *tmp = nullptr;
    CHK(sc.alloc(&tmp, 4 * nquad * L.tile_elems()));
    CHK(dalloc_t(ctx, &F->Cquad, 4 * nquad * L.tile_elems()));
    launch_quad_coupling(F->Lst, F->Linv, F->Cpair, L, tmp, F->Cquad, s);
  }
  b.Q = F->Cquad;
  return KRR_SUCCESS;
}

// z: column ranges of the residual with each stored tile read twice (0:
// min(8, NT)); z = -1: each stored tile read once (one slot per partner
// tile) when its slots take at most 1 GiB, else the default.
static krr_status solve_alloc(Scoped &sc, const TileLayout &L, int r, SolveBufs &b, int z) {
  const int64_t cnt = L.np * r;
  b.once = z == -1 && residual_once_bytes(L, r) <= ((int64_t)1 << 30);
  if (z <= 0 && !b.once) z = residual_split(L);
  b.z = b.once ? L.nt : std::max(1, std::min(z, L.nt));
  CHK(sc.alloc(&b.Pr, cnt * b.z));
  CHK(sc.alloc(&b.Yr, cnt));
  CHK(sc.alloc(&b.Xr, cnt));
  CHK(sc.alloc(&b.Rr, cnt));
  CHK(sc.alloc(&b.cn, 2 * r));
  CHK(sc.alloc(&b.cw, col_dots_workspace(r)));
  CHK(sc.alloc(&b.Bf, cnt));
  CHK(sc.alloc(&b.Zf, cnt));
  CHK(sc.alloc(&b.Xf, cnt));
  return KRR_SUCCESS;
}

// The split quad sweeps' second stream and events (two per quad step), made
// once per context and grown with the tile count; null when the sweeps do
// not go by quads or KRR_SWEEP_SPLIT=0.
static const SweepSplit *sweep_split(krr_context ctx, const TileLayout &L, const SolveBufs &b,
                                     SweepSplit &sp) {
  const char *e = getenv("KRR_SWEEP_SPLIT");
  if ((e ? atoi(e) : 0) == 0 || !b.C || !b.Q || L.nt < 12) return nullptr;
  if (!ctx->sw2 && hipStreamCreateWithFlags(&ctx->sw2, hipStreamNonBlocking) != hipSuccess) {
    ctx->sw2 = nullptr;
    return nullptr;
  }
  const size_t need = (size_t)2 * (L.nt / 4);
  while (ctx->sweep_ev.size() < need) {
    hipEvent_t ev;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return nullptr;
    ctx->sweep_ev.push_back(ev);
  }
  sp = SweepSplit{ctx->sw2, ctx->sweep_ev.data(), (int)need};
  return &sp;
}

// dst += L^-T L^-1 src with FP32 sweeps (src, dst: FP64, row-major np x r;
// the sweeps work on column-major FP32 copies).
static void solve_sweeps(krr_context ctx, krr_factorization F, int r, SolveBufs &b,
                         const double *src, double *dst, hipStream_t s) {
  const TileLayout &L = F->L;
  SweepSplit spb;
  const SweepSplit *sp = sweep_split(ctx, L, b, spb);
  launch_rows_f64_to_cols_f32(src, L.np, r, b.Bf, s);
  {
    Stage t(ctx, KRR_STAGE_FWD, s);
    launch_fwd_sweep(F->Lst, F->Linv, b.C, b.Q, L, r, b.Bf, b.Zf, s, sp);
  }
  {
    Stage t(ctx, KRR_STAGE_BWD, s);
    launch_bwd_sweep(F->Lst, F->Linv, b.C, b.Q, L, r, b.Zf, b.Xf, s, sp);
  }
  launch_cols_f32_axpy_rows_f64(b.Xf, L.np, r, 1.0, dst, s);
}

// R = Y - (K + lambda I) X in FP64, then the squared column norms of R and X
// into cn[0 .. r) and cn[r .. 2r).
static void residual_norms(krr_context ctx, krr_factorization F, int r, SolveBufs &b,
                           hipStream_t s) {
  krr_kernel K = F->K;
  const TileLayout &L = F->L;
  {
    Stage t(ctx, KRR_STAGE_RESIDUAL, s);
    if (b.once)
      launch_residual_once(K->D, K->etab, K->etab_len, K->gamma, K->vmode(), K->Ec, K->lambda, L,
                           r, b.Xr, b.Yr, b.Rr, b.Pr, s);
    else
      launch_residual(K->D, K->etab, K->etab_len, K->gamma, K->vmode(), K->Ec, K->lambda, L, r,
                      b.Xr, b.Yr, b.Rr, b.Pr, b.z, s);
  }
  launch_col_norms(b.Rr, L.np, r, b.cn, b.cw, s);
  launch_col_norms(b.Xr, L.np, r, b.cn + r, b.cw, s);
}

// The refinement's stop quantities from the squared norms: the forward-error
// bound max_j ||r_j|| / (lambda ||x_j||) and the backward error.
static void refine_bounds(const double *hn, const double *yn, int r, double lambda, double norm_a,
                          double &bound, double &berr) {
  const double lam = lambda > 0 ? lambda : 1e-300;
  bound = 0;
  berr = 0;
  for (int c = 0; c < r; ++c) {
    const double rn = sqrt(hn[c]), xn = sqrt(hn[r + c]), ynn = sqrt(yn[c]);
    const double b = xn > 0 ? rn / (lam * xn) : (rn > 0 ? INFINITY : 0.0);
    bound = std::max(bound, b);
    const double den = norm_a * xn + ynn;
    berr = std::max(berr, den > 0 ? rn / den : 0.0);
  }
}

// Conjugate-gradient state: z (preconditioned residual), p (direction),
// nq = -A p, a zero right-hand side for the residual kernel, and per-column
// scalars p . nq, rho and the next rho.
struct PcgBufs {
  double *Z = nullptr, *P = nullptr, *Nq = nullptr, *Y0 = nullptr, *dots = nullptr;
};

static krr_status pcg_alloc(Scoped &sc, const TileLayout &L, int r, PcgBufs &pb) {
  const int64_t cnt = L.np * r;
  CHK(sc.alloc(&pb.Z, cnt));
  CHK(sc.alloc(&pb.P, cnt));
  CHK(sc.alloc(&pb.Nq, cnt));
  CHK(sc.alloc(&pb.Y0, cnt));
  CHK(sc.alloc(&pb.dots, 3 * r));
  launch_fill_f64(pb.Y0, cnt, 0.0, sc.ctx->stream);
  return KRR_SUCCESS;
}

// Conjugate gradients on (K + lambda I) X = Y, column by column, preconditioned
// by the factor (z = L^-T L^-1 r with the FP32 sweeps), from the current X and
// its true residual in b.Rr.  A p comes from the FP64 residual kernel with a
// zero right-hand side.  Runs until the updated residual meets the stop rule
// or `it` reaches the budget; the caller then recomputes the true residual,
// which alone decides convergence, and restarts from it if it falls short.
static krr_status pcg_run(krr_context ctx, krr_factorization F, int r, SolveBufs &b, PcgBufs &pb,
                          const std::vector<double> &yn, const krr_refine_opts &o, int &it,
                          hipStream_t s) {
  krr_kernel K = F->K;
  const TileLayout &L = F->L;
  const int64_t cnt = L.np * r;
  double *pnq = pb.dots, *rho = pb.dots + r, *rho_next = pb.dots + 2 * r;
  launch_fill_f64(pb.Z, cnt, 0.0, s);
  solve_sweeps(ctx, F, r, b, b.Rr, pb.Z, s);
  launch_pcg_dir(pb.P, pb.Z, nullptr, nullptr, cnt, r, s);
  launch_col_dots(b.Rr, pb.Z, L.np, r, rho, b.cw, s);
  std::vector<double> hn(2 * r);
  while (it < o.max_iters) {
    {
      Stage t(ctx, KRR_STAGE_RESIDUAL, s);
      if (b.once)
        launch_residual_once(K->D, K->etab, K->etab_len, K->gamma, K->vmode(), K->Ec, K->lambda,
                             L, r, pb.P, pb.Y0, pb.Nq, b.Pr, s);
      else
        launch_residual(K->D, K->etab, K->etab_len, K->gamma, K->vmode(), K->Ec, K->lambda, L,
                        r, pb.P, pb.Y0, pb.Nq, b.Pr, b.z, s);
    }
    launch_col_dots(pb.P, pb.Nq, L.np, r, pnq, b.cw, s);
    launch_pcg_step(b.Xr, b.Rr, pb.P, pb.Nq, rho, pnq, cnt, r, s);
    ++it;
    launch_col_norms(b.Rr, L.np, r, b.cn, b.cw, s);
    launch_col_norms(b.Xr, L.np, r, b.cn + r, b.cw, s);
    CHK(launch_ok());
    HIPCHK(hipMemcpyAsync(hn.data(), b.cn, 2 * r * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double bound, berr;
    refine_bounds(hn.data(), yn.data(), r, K->lambda, K->norm_a, bound, berr);
    if (ctx->opts.verbose) fprintf(stderr, "krr_solve: pcg it=%d updated bound=%.3e\n", it, bound);
    if (bound <= o.tol) break;
    launch_fill_f64(pb.Z, cnt, 0.0, s);
    solve_sweeps(ctx, F, r, b, b.Rr, pb.Z, s);
    launch_col_dots(b.Rr, pb.Z, L.np, r, rho_next, b.cw, s);
    launch_pcg_dir(pb.P, pb.Z, rho_next, rho, cnt, r, s);
    std::swap(rho, rho_next);
  }
  return KRR_SUCCESS;
}

krr_status krr_solve(krr_context ctx, krr_factorization F, const double *Y, int64_t nrhs, int64_t ldy,
                     double *X, int64_t ldx, const krr_refine_opts *opts, krr_solve_info *info) {
  if (!ctx || !F || !Y || !X || nrhs <= 0 || nrhs > 4096) return KRR_ERROR_INVALID_VALUE;
  krr_kernel K = F->K;
  if (K->ctx != ctx) return KRR_ERROR_INVALID_VALUE;
  const TileLayout &L = F->L;
  if (ldy < L.n || ldx < L.n) return KRR_ERROR_INVALID_VALUE;
  krr_refine_opts o;
  CHK(refine_args(opts, true, o));
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  const int r = (int)nrhs;
  const int64_t cnt = L.np * r;
  Scoped sc(ctx);
  SolveBufs b;
  CHK(solve_alloc(sc, L, r, b,
                  ctx->tune.residual_split));
  CHK(sweep_coupling(ctx, F, sc, b, s));
  launch_colmajor_to_rows(Y, L.n, ldy, r, L.np, b.Yr, s);
  launch_fill_f64(b.Xr, cnt, 0.0, s);
  solve_sweeps(ctx, F, r, b, b.Yr, b.Xr, s);  // the unrefined FP32 solve
  CHK(launch_ok());
  krr_solve_info inf{};
  inf.first_bound = -1;
  krr_status st = KRR_SUCCESS;
  if (o.method != KRR_REFINE_NONE) {
    std::vector<double> hn(2 * r), yn(r);
    launch_col_norms(b.Yr, L.np, r, b.cn, b.cw, s);
    HIPCHK(hipMemcpyAsync(yn.data(), b.cn, r * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    PcgBufs pb;
    if (o.method == KRR_REFINE_PCG || o.method == KRR_REFINE_AUTO) CHK(pcg_alloc(sc, L, r, pb));
    bool pcg = o.method == KRR_REFINE_PCG;
    double prev = 0;
    int it = 0;
    for (;;) {
      residual_norms(ctx, F, r, b, s);  // the true residual of the current X
      CHK(launch_ok());
      HIPCHK(hipMemcpyAsync(hn.data(), b.cn, 2 * r * 8, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      double bound, berr;
      refine_bounds(hn.data(), yn.data(), r, K->lambda, K->norm_a, bound, berr);
      if (it == 0) inf.first_bound = bound;
      inf.fwd_err_bound = bound;
      inf.backward_err = berr;
      if (bound <= o.tol) {
        inf.converged = 1;
        break;
      }
      if (it >= o.max_iters) break;
      // AUTO: refinement while each iteration at least halves the bound, then CG
      if (o.method == KRR_REFINE_AUTO && it > 0 && bound > 0.5 * prev) pcg = true;
      prev = bound;
      if (pcg) {
        CHK(pcg_run(ctx, F, r, b, pb, yn, o, it, s));
      } else {
        solve_sweeps(ctx, F, r, b, b.Rr, b.Xr, s);
        ++it;
      }
    }
    inf.iters = it;
    if (!inf.converged) st = KRR_ERROR_NOT_CONVERGED;
  }
  launch_rows_to_colmajor(b.Xr, L.n, r, X, ldx, s);
  CHK(launch_ok());
  HIPCHK(hipStreamSynchronize(s));
  if (info) *info = inf;
  if (ctx->opts.verbose)
    fprintf(stderr, "krr_solve: iters=%d bound=%.3e first=%.3e\n", inf.iters, inf.fwd_err_bound,
            inf.first_bound);
  return st;
}

krr_status krr_solve_batched(krr_context ctx, int32_t batch, const krr_factorization *F,
                             const double *const *Y, int64_t nrhs, const int64_t *ldy,
                             double *const *X, const int64_t *ldx, const krr_refine_opts *opts,
                             krr_solve_info *info) {
  if (!ctx || batch <= 0 || !F || !Y || !X || !ldy || !ldx || nrhs <= 0 || nrhs > 4096)
    return KRR_ERROR_INVALID_VALUE;
  for (int b = 0; b < batch; ++b) {
    if (!F[b] || !Y[b] || !X[b] || F[b]->K->ctx != ctx) return KRR_ERROR_INVALID_VALUE;
    if (ldy[b] < F[b]->L.n || ldx[b] < F[b]->L.n) return KRR_ERROR_INVALID_VALUE;
    // the lockstep residual has no confounders and no linear kernel
    if (F[b]->K->Ec || F[b]->K->kind == KRR_KERNEL_LINEAR) return KRR_ERROR_NOT_SUPPORTED;
  }
  krr_refine_opts o;
  CHK(refine_args(opts, false, o));
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  const int r = (int)nrhs, nb = ctx->opts.tile;
  Scoped sc(ctx);
  std::vector<SolveBufs> B(batch);
  for (int b = 0; b < batch; ++b)
    CHK(solve_alloc(sc, F[b]->L, r, B[b], residual_split_batched(F[b]->L)));
  SolveJob *djobs = nullptr;
  CHK(job_table(ctx, 1, sizeof(SolveJob) * batch, (void **)&djobs));
  // The table of the instances a batched launch covers; every instance's
  // steps run in lockstep in one launch per step (sweeps) or per pass
  // (residual), all on the context stream.
  std::vector<SolveJob> all(batch);
  std::vector<std::vector<SolveJob>> tables;  // every uploaded table lives until the return
  for (int b = 0; b < batch; ++b) {
    krr_kernel K = F[b]->K;
    SolveJob &j = all[b];
    j.Lst = F[b]->Lst;
    j.Linv = F[b]->Linv;
    j.B = B[b].Bf;
    j.Z = B[b].Zf;
    j.X = B[b].Xf;
    j.nt = F[b]->L.nt;
    j.D = K->D;
    j.etab = K->etab;
    j.etab_len = K->etab_len;
    j.gamma = K->gamma;
    j.wshift = K->vmode() != VAL_EXP ? -1 : residual_exp_shift(K->gamma, K->etab_len);
    j.np = F[b]->L.np;
    j.Xd = B[b].Xr;
    j.part = B[b].Pr;
    j.rb0 = 0;
  }
  // upload the table of the instances in `ids` (rb0 prefix over them); its
  // host copy is kept until the call returns, past any asynchronous copy
  auto upload = [&](const std::vector<int> &ids, int &ntmax, int64_t &rblocks,
                    bool &fact) -> krr_status {
    tables.emplace_back();
    std::vector<SolveJob> &act = tables.back();
    ntmax = 0;
    rblocks = 0;
    fact = true;
    for (int b : ids) {
      SolveJob j = all[b];
      j.rb0 = rblocks;
      rblocks += j.np / 64;
      ntmax = std::max(ntmax, j.nt);
      fact = fact && j.wshift >= 0;
      act.push_back(j);
    }
    HIPCHK(hipMemcpyAsync(djobs, act.data(), sizeof(SolveJob) * act.size(), hipMemcpyHostToDevice,
                          s));
    return KRR_SUCCESS;
  };
  auto sweeps = [&](const std::vector<int> &ids, bool from_residual) -> krr_status {
    for (int b : ids) {
      const int64_t cnt = F[b]->L.np * r;
      launch_f64_to_f32(from_residual ? B[b].Rr : B[b].Yr, cnt, B[b].Bf, s);
    }
    int ntmax;
    int64_t rblocks;
    bool fact;
    CHK(upload(ids, ntmax, rblocks, fact));
    {
      char kb[128];
      snprintf(kb, sizeof kb, "sweeps|%p|%d|%d|%d|%d", (void *)djobs, (int)ids.size(), ntmax, nb,
               r);
      Stage t(ctx, KRR_STAGE_FWD, s);
      CHK(graph_run(ctx, kb, s, [&](hipStream_t cs) {
        launch_sweeps_batched(djobs, (int)ids.size(), ntmax, nb, r, cs);
      }));
    }
    for (int b : ids) launch_axpy_f32_to_f64(B[b].Xf, F[b]->L.np * r, 1.0, B[b].Xr, s);
    return launch_ok();
  };
  std::vector<int> ids(batch);
  for (int b = 0; b < batch; ++b) ids[b] = b;
  for (int b = 0; b < batch; ++b) {
    const TileLayout &L = F[b]->L;
    launch_colmajor_to_rows(Y[b], L.n, ldy[b], r, L.np, B[b].Yr, s);
    launch_fill_f64(B[b].Xr, L.np * r, 0.0, s);
  }
  CHK(sweeps(ids, false));  // the unrefined FP32 solves
  std::vector<krr_solve_info> inf(batch);
  for (auto &x : inf) x.first_bound = -1;
  std::vector<double> hn(2 * (size_t)r * batch), yn((size_t)r * batch);
  if (o.method != KRR_REFINE_NONE) {
    for (int b = 0; b < batch; ++b) {
      launch_col_norms(B[b].Yr, F[b]->L.np, r, B[b].cn, B[b].cw, s);
      HIPCHK(hipMemcpyAsync(yn.data() + (size_t)r * b, B[b].cn, r * 8, hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    for (int it = 0; !ids.empty(); ++it) {
      int ntmax;
      int64_t rblocks;
      bool fact;
      CHK(upload(ids, ntmax, rblocks, fact));
      {
        Stage t(ctx, KRR_STAGE_RESIDUAL, s);
        launch_residual_batched(djobs, (int)ids.size(), rblocks, fact, nb, r, s);
      }
      for (int b : ids) {
        const TileLayout &L = F[b]->L;
        launch_residual_sum(B[b].Pr, residual_split_batched(L), L, r, F[b]->K->lambda, B[b].Xr,
                            B[b].Yr, B[b].Rr, s);
        launch_col_norms(B[b].Rr, L.np, r, B[b].cn, B[b].cw, s);
        launch_col_norms(B[b].Xr, L.np, r, B[b].cn + r, B[b].cw, s);
        HIPCHK(hipMemcpyAsync(hn.data() + 2 * (size_t)r * b, B[b].cn, 2 * r * 8,
                              hipMemcpyDeviceToHost, s));
      }
      CHK(launch_ok());
      HIPCHK(hipStreamSynchronize(s));
      std::vector<int> next;
      for (int b : ids) {
        double bound, berr;
        refine_bounds(hn.data() + 2 * (size_t)r * b, yn.data() + (size_t)r * b, r,
                      F[b]->K->lambda, F[b]->K->norm_a, bound, berr);
        if (it == 0) inf[b].first_bound = bound;
        inf[b].fwd_err_bound = bound;
        inf[b].backward_err = berr;
        inf[b].iters = it;
        if (bound <= o.tol) inf[b].converged = 1;
        else if (it < o.max_iters) next.push_back(b);
      }
      ids.swap(next);
      if (!ids.empty()) CHK(sweeps(ids, true));
    }
  }
  for (int b = 0; b < batch; ++b)
    launch_rows_to_colmajor(B[b].Xr, F[b]->L.n, r, X[b], ldx[b], s);
  CHK(launch_ok());
  HIPCHK(hipStreamSynchronize(s));
  krr_status st = KRR_SUCCESS;
  for (int b = 0; b < batch; ++b) {
    if (o.method != KRR_REFINE_NONE && !inf[b].converged) st = KRR_ERROR_NOT_CONVERGED;
    if (info) info[b] = inf[b];
  }
  return st;
}

static krr_status predict_args(krr_context ctx, krr_kernel K, const int8_t *T, int64_t n_test,
                               int64_t ldt, const double *X, int64_t nrhs, int64_t ldx,
                               const double *P, int64_t ldp) {
  if (!ctx || !K || !T || !X || !P || n_test <= 0 || nrhs <= 0 || nrhs > 4096)
    return KRR_ERROR_INVALID_VALUE;
  if (K->ctx != ctx) return KRR_ERROR_INVALID_VALUE;
  if (ldt < K->m || (ldt % 16) != 0 || !aligned16(T) || ldx < K->n || ldp < n_test)
    return KRR_ERROR_INVALID_VALUE;
  return KRR_SUCCESS;
}

// Working buffers of one Predict: nrm_t (n_test), flag (1), Dt (chunk x np
// int32), Xr (np x r FP64); for the IBS kernel Tenc (n_test x ldh, the
// encoded test rows); with confounders Et (chunk x np FP64).
struct PredictBufs {
  int32_t *nrm_t = nullptr, *flag = nullptr, *Dt = nullptr;
  double *Xr = nullptr, *Et = nullptr;
  int8_t *Tenc = nullptr;
  int64_t chunk = 0;
};

// Test rows per pass, so the cross-distance block (and the confounder
// factors) stay within ~2 GiB.
static int64_t predict_chunk(krr_kernel K, int64_t n_test) {
  const int64_t per = K->L.np * (K->Ec ? 12 : 4);
  int64_t chunk = std::max<int64_t>(256, ((int64_t)1 << 31) / per / 256 * 256);
  return std::min<int64_t>(chunk, (n_test + 255) / 256 * 256);
}

static krr_status predict_alloc(Scoped &sc, krr_kernel K, int64_t n_test, int r, PredictBufs &b) {
  const TileLayout &L = K->L;
  b.chunk = predict_chunk(K, n_test);
  CHK(sc.alloc(&b.nrm_t, (n_test + 255) / 256 * 256));
  CHK(sc.alloc(&b.flag, 1));
  CHK(sc.alloc(&b.Dt, b.chunk * L.np));
  CHK(sc.alloc(&b.Xr, L.np * r));
  if (K->H) CHK(sc.alloc(&b.Tenc, n_test * K->ldh));
  if (K->Ec) CHK(sc.alloc(&b.Et, b.chunk * L.np));
  return KRR_SUCCESS;
}

// Checks T's genotypes (one wait), then runs the cross Gram and the FP64
// product chunk by chunk of test rows.  Ct: the test rows' confounders when
// the kernel has them (n_test x q, ldct).
static krr_status predict_run(krr_context ctx, krr_kernel K, const int8_t *T, int64_t n_test,
                              int64_t ldt, const double *Ct, int64_t ldct, const double *X, int r,
                              int64_t ldx, double *P, int64_t ldp, const PredictBufs &b) {
  hipStream_t s = ctx->stream;
  const TileLayout &L = K->L;
  launch_fill_i32(b.flag, 1, 0, s);
  launch_row_norms(T, n_test, n_test, K->m, ldt, b.nrm_t, b.flag, s);
  int32_t hflag = 0;
  HIPCHK(hipMemcpyAsync(&hflag, b.flag, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  CHK(launch_ok());
  if (hflag) return KRR_ERROR_BAD_GENOTYPE;
  const int8_t *Tsrc = T;
  int64_t ldsrc = ldt;
  if (K->H) {  // the IBS kernel compares encoded rows
    launch_ibs_encode(T, n_test, K->m, ldt, b.Tenc, K->ldh, s);
    launch_row_norms(b.Tenc, n_test, n_test, K->ldh, K->ldh, b.nrm_t, b.flag, s);
    Tsrc = b.Tenc;
    ldsrc = K->ldh;
  }
  launch_colmajor_to_rows(X, K->n, ldx, r, L.np, b.Xr, s);
  for (int64_t r0 = 0; r0 < n_test; r0 += b.chunk) {
    const int64_t rows = std::min(b.chunk, n_test - r0);
    {
      Stage t(ctx, KRR_STAGE_CROSS_GRAM);
      launch_cross_gram(Tsrc + r0 * ldsrc, rows, b.nrm_t + r0, K->gram_src(), K->n, K->gram_m(),
                        ldsrc, K->gram_ld(), K->nrm, L.np, b.Dt, L.np,
                        K->vmode() == VAL_LINEAR, s);
      if (K->Ec)
        launch_conf_factor_cross(Ct + r0 * ldct, rows, ldct, K->Cc, K->n, K->q, K->q, K->gamma,
                                 L.np, b.Et, L.np, s);
    }
    Stage t(ctx, KRR_STAGE_PREDICT);
    launch_predict_apply(b.Dt, rows, L.np, L.np, K->etab, K->etab_len, b.Xr, r, P + r0, ldp,
                         K->Ec ? b.Et : nullptr, K->vmode() == VAL_LINEAR, s);
  }
  CHK(launch_ok());
  HIPCHK(hipStreamSynchronize(s));
  return KRR_SUCCESS;
}

krr_status krr_predict_ex(krr_context ctx, krr_kernel K, const int8_t *T, int64_t n_test,
                          int64_t ldt, const double *Ct, int64_t ldct, const double *X,
                          int64_t nrhs, int64_t ldx, double *P, int64_t ldp) {
  CHK(predict_args(ctx, K, T, n_test, ldt, X, nrhs, ldx, P, ldp));
  if (K->Ec && (!Ct || ldct < K->q)) return KRR_ERROR_INVALID_VALUE;
  HIPCHK(hipSetDevice(ctx->device));
  Scoped sc(ctx);
  PredictBufs b;
  CHK(predict_alloc(sc, K, n_test, (int)nrhs, b));
  return predict_run(ctx, K, T, n_test, ldt, Ct, ldct, X, (int)nrhs, ldx, P, ldp, b);
}

krr_status krr_predict(krr_context ctx, krr_kernel K, const int8_t *T, int64_t n_test, int64_t ldt,
                       const double *X, int64_t nrhs, int64_t ldx, double *P, int64_t ldp) {
  if (K && K->Ec) return KRR_ERROR_INVALID_VALUE;  // needs the test rows' confounders
  return krr_predict_ex(ctx, K, T, n_test, ldt, nullptr, 0, X, nrhs, ldx, P, ldp);
}

krr_status krr_predict_batched(krr_context ctx, int32_t batch, const krr_kernel *K,
                               const int8_t *const *T, const int64_t *n_test, const int64_t *ldt,
                               const double *const *X, int64_t nrhs, const int64_t *ldx,
                               double *const *P, const int64_t *ldp) {
  if (!ctx || batch <= 0 || !K || !T || !n_test || !ldt || !X || !ldx || !P || !ldp)
    return KRR_ERROR_INVALID_VALUE;
  for (int b = 0; b < batch; ++b) {
    CHK(predict_args(ctx, K[b], T[b], n_test[b], ldt[b], X[b], nrhs, ldx[b], P[b], ldp[b]));
    if (K[b]->kind != KRR_KERNEL_GAUSSIAN || K[b]->Ec)
      return KRR_ERROR_NOT_SUPPORTED;  // krr_predict_ex per instance
  }
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  const int r = (int)nrhs;
  // one cross-distance and one X buffer, sized for the largest instance
  int64_t dt_elems = 0, x_elems = 0, nrm_elems = 0;
  std::vector<int64_t> chunk(batch), nrm_off(batch);
  for (int b = 0; b < batch; ++b) {
    const int64_t np = K[b]->L.np;
    chunk[b] = std::max<int64_t>(256, ((int64_t)1 << 29) / np / 256 * 256);
    chunk[b] = std::min<int64_t>(chunk[b], (n_test[b] + 255) / 256 * 256);
    dt_elems = std::max(dt_elems, chunk[b] * np);
    x_elems = std::max(x_elems, np * r);
    nrm_off[b] = nrm_elems;
    nrm_elems += (n_test[b] + 255) / 256 * 256;
  }
  Scoped sc(ctx);
  int32_t *nrm_t, *flag, *Dt;
  double *Xr;
  CHK(sc.alloc(&nrm_t, nrm_elems));
  CHK(sc.alloc(&flag, batch));
  CHK(sc.alloc(&Dt, dt_elems));
  CHK(sc.alloc(&Xr, x_elems));
  // every instance's genotype check, then one wait
  launch_fill_i32(flag, batch, 0, s);
  for (int b = 0; b < batch; ++b)
    launch_row_norms(T[b], n_test[b], n_test[b], K[b]->m, ldt[b], nrm_t + nrm_off[b], flag + b, s);
  std::vector<int32_t> hflag(batch, 0);
  HIPCHK(hipMemcpyAsync(hflag.data(), flag, 4 * (size_t)batch, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  CHK(launch_ok());
  for (int b = 0; b < batch; ++b)
    if (hflag[b]) return KRR_ERROR_BAD_GENOTYPE;
  for (int b = 0; b < batch; ++b) {
    const krr_kernel k = K[b];
    const TileLayout &L = k->L;
    launch_colmajor_to_rows(X[b], k->n, ldx[b], r, L.np, Xr, s);
    for (int64_t r0 = 0; r0 < n_test[b]; r0 += chunk[b]) {
      const int64_t rows = std::min(chunk[b], n_test[b] - r0);
      {
        Stage t(ctx, KRR_STAGE_CROSS_GRAM);
        launch_cross_gram(T[b] + r0 * ldt[b], rows, nrm_t + nrm_off[b] + r0, k->G, k->n, k->m,
                          ldt[b], k->ldg, k->nrm, L.np, Dt, L.np, false, s);
      }
      Stage t(ctx, KRR_STAGE_PREDICT);
      launch_predict_apply(Dt, rows, L.np, L.np, k->etab, k->etab_len, Xr, r, P[b] + r0, ldp[b],
                           nullptr, false, s);
    }
  }
  CHK(launch_ok());
  HIPCHK(hipStreamSynchronize(s));
  return KRR_SUCCESS;
}

// Layout of the fixed scratch for one no-allocation Predict: flag, test-row
// norms, the row-major copy of X, then the cross distances of `chunk` test
// rows.  Returns false when even a 64-row chunk does not fit.
static bool noalloc_layout(int64_t n_test, int64_t np, int r, int64_t *off_nrm, int64_t *off_x,
                           int64_t *off_dt, int64_t *chunk) {
  auto up = [](int64_t b) { return (b + 255) / 256 * 256; };
  *off_nrm = 256;
  *off_x = *off_nrm + up(n_test * 4);
  *off_dt = *off_x + up(np * (int64_t)r * 8);
  const int64_t room = (int64_t)KRR_NOALLOC_SCRATCH_BYTES - *off_dt;
  if (room <= 0) return false;
  int64_t c = room / (np * 4) / 64 * 64;  // rows of cross distances that fit
  c = std::min<int64_t>(c, (n_test + 63) / 64 * 64);
  if (c < 64) return false;
  *chunk = c;
  return true;
}

krr_status krr_predict_noalloc(krr_context ctx, krr_kernel K, const int8_t *T, int64_t n_test,
                               int64_t ldt, const double *X, int64_t nrhs, int64_t ldx, double *P,
                               int64_t ldp) {
  CHK(predict_args(ctx, K, T, n_test, ldt, X, nrhs, ldx, P, ldp));
  if (K->kind != KRR_KERNEL_GAUSSIAN || K->Ec)
    return KRR_ERROR_NOT_SUPPORTED;  // the Gaussian kernel without confounders
  const int r = (int)nrhs;
  int64_t off_nrm, off_x, off_dt, chunk;
  if (!noalloc_layout(n_test, K->L.np, r, &off_nrm, &off_x, &off_dt, &chunk))
    return KRR_ERROR_SCRATCH_TOO_SMALL;
  HIPCHK(hipSetDevice(ctx->device));
  uint8_t *base = (uint8_t *)scratch_ptr(ctx->device);  // set up by krr_create
  if (!base) return KRR_ERROR_HIP;
  PredictBufs b;
  b.flag = (int32_t *)base;
  b.nrm_t = (int32_t *)(base + off_nrm);
  b.Xr = (double *)(base + off_x);
  b.Dt = (int32_t *)(base + off_dt);
  b.chunk = chunk;
  return predict_run(ctx, K, T, n_test, ldt, nullptr, 0, X, r, ldx, P, ldp, b);
}

krr_status krr_noalloc_limits(int64_t n, int64_t n_test, int64_t nrhs, int32_t tile,
                              int64_t *scratch_bytes, int32_t *fits) {
  if (!scratch_bytes || !fits || n <= 0 || n_test <= 0 || nrhs <= 0) return KRR_ERROR_INVALID_VALUE;
  if (tile == 0) tile = 512;
  if (tile != 256 && tile != 512) return KRR_ERROR_INVALID_VALUE;
  *scratch_bytes = (int64_t)KRR_NOALLOC_SCRATCH_BYTES;
  int64_t a, b, c, d;
  *fits = (nrhs <= 4096 && noalloc_layout(n_test, make_layout(n, tile).np, (int)nrhs, &a, &b, &c, &d))
              ? 1
              : 0;
  return KRR_SUCCESS;
}

krr_status krr_context_memory(krr_context ctx, int64_t *allocated, int64_t *cached) {
  if (!ctx) return KRR_ERROR_INVALID_VALUE;
  if (allocated) *allocated = ctx->allocated;
  if (cached) *cached = (int64_t)ctx->cached;
  return KRR_SUCCESS;
}

krr_status krr_debug_encode_fp8(krr_context ctx, const float *x, int64_t n, uint8_t *out) {
  if (!ctx || !x || !out || n <= 0) return KRR_ERROR_INVALID_VALUE;
  HIPCHK(hipSetDevice(ctx->device));
  launch_encode_fp8(x, n, out, ctx->stream);
  CHK(launch_ok());
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return KRR_SUCCESS;
}

krr_status krr_kernel_copy_distances(krr_kernel K, int64_t i0, int64_t j0, int64_t rows,
                                     int64_t cols, int32_t *dst, int64_t ld) {
  if (!K || !dst || rows <= 0 || cols <= 0 || ld < cols || i0 < 0 || j0 < 0 ||
      i0 + rows > K->n || j0 + cols > K->n)
    return KRR_ERROR_INVALID_VALUE;
  HIPCHK(hipSetDevice(K->ctx->device));
  launch_copy_tiles_i32(K->D, K->L, i0, j0, rows, cols, dst, ld, K->ctx->stream);
  CHK(launch_ok());
  HIPCHK(hipStreamSynchronize(K->ctx->stream));
  return KRR_SUCCESS;
}

krr_status krr_kernel_copy_matrix(krr_kernel K, int64_t i0, int64_t j0, int64_t rows,
                                  int64_t cols, float *dst, int64_t ld) {
  if (!K || !dst || rows <= 0 || cols <= 0 || ld < cols || i0 < 0 || j0 < 0 ||
      i0 + rows > K->n || j0 + cols > K->n || !K->A)
    return KRR_ERROR_INVALID_VALUE;
  HIPCHK(hipSetDevice(K->ctx->device));
  launch_copy_tiles_f32(K->A, K->L, i0, j0, rows, cols, false, dst, ld, K->ctx->stream);
  CHK(launch_ok());
  HIPCHK(hipStreamSynchronize(K->ctx->stream));
  return KRR_SUCCESS;
}

krr_status krr_factor_copy_l(krr_factorization F, int64_t i0, int64_t j0, int64_t rows, int64_t cols,
                             float *dst, int64_t ld) {
  if (!F || !dst || rows <= 0 || cols <= 0 || ld < cols || i0 < 0 || j0 < 0 ||
      i0 + rows > F->L.n || j0 + cols > F->L.n)
    return KRR_ERROR_INVALID_VALUE;
  krr_context c = F->ctx;
  HIPCHK(hipSetDevice(c->device));
  launch_copy_tiles_f32(F->Lst, F->L, i0, j0, rows, cols, true, dst, ld, c->stream);
  CHK(launch_ok());
  HIPCHK(hipStreamSynchronize(c->stream));
  return KRR_SUCCESS;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Schedule tuning and the autotuner.

static bool tuning_valid(const krr_tuning &t) {
  return (t.tile == 256 || t.tile == 512) && t.panel_group >= 0 && t.panel_group <= KRR_MAX_GROUP &&
         t.residual_split >= -1 && t.residual_split <= 16 && t.sweep_pairs >= -1 &&
         t.sweep_pairs <= 1 && t.lookahead >= -1 && t.lookahead <= 1 && t.aux_cu_eighths >= 0 &&
         t.aux_cu_eighths <= 8;
}

krr_status krr_set_tuning(krr_context ctx, const krr_tuning *t) {
  if (!ctx || !t || !tuning_valid(*t)) return KRR_ERROR_INVALID_VALUE;
  if (t->tile != ctx->opts.tile && ctx->live > 0) return KRR_ERROR_INVALID_VALUE;
  ctx->tune = *t;
  ctx->opts.tile = t->tile;
  return KRR_SUCCESS;
}

krr_status krr_get_tuning(krr_context ctx, krr_tuning *t) {
  if (!ctx || !t) return KRR_ERROR_INVALID_VALUE;
  *t = ctx->tune;
  t->tile = ctx->opts.tile;
  return KRR_SUCCESS;
}

krr_status krr_tuning_key(int device, int64_t n, int64_t m, int64_t nrhs,
                          const krr_precision_policy *policy, const krr_refine_opts *refine,
                          char *key, int32_t cap) {
  if (!key || cap <= 0 || n <= 0 || m <= 0 || nrhs <= 0) return KRR_ERROR_INVALID_VALUE;
  krr_precision_policy p;
  FactorPlan fp;
  CHK(resolve_policy(policy, p, fp));
  const int method = refine ? refine->method : KRR_REFINE_IR;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    (void)hipGetLastError();
    return KRR_ERROR_HIP;
  }
  char arch[sizeof(prop.gcnArchName) + 1];
  memcpy(arch, prop.gcnArchName, sizeof(prop.gcnArchName));
  arch[sizeof(prop.gcnArchName)] = 0;
  for (char *c = arch; *c; ++c)
    if (*c == '"' || *c == '\\' || *c == ' ') *c = '_';
  const int w = snprintf(key, (size_t)cap, "%s|cu%d|n%lld|m%lld|r%lld|mode%d|d64%d|ref%d", arch,
                         prop.multiProcessorCount, (long long)n, (long long)m, (long long)nrhs,
                         p.mode, p.diag_fp64 ? 1 : 0, method);
  return (w > 0 && w < cap) ? KRR_SUCCESS : KRR_ERROR_INVALID_VALUE;
}

// One line of the cache file: "key": {fields}
static bool cache_parse_line(const char *line, std::string &key, krr_tuning &t, double &ms,
                             bool &well_formed) {
  const char *q0 = strchr(line, '"');
  if (!q0) return false;
  const char *q1 = strchr(q0 + 1, '"');
  if (!q1) return false;
  key.assign(q0 + 1, q1 - q0 - 1);
  int tile, g, z, pr, la, aq;
  well_formed = sscanf(q1 + 1,
                       " : {\"tile\": %d, \"panel_group\": %d, \"residual_split\": %d, "
                       "\"sweep_pairs\": %d, \"lookahead\": %d, \"aux_cu_eighths\": %d, "
                       "\"ms\": %lf}",
                       &tile, &g, &z, &pr, &la, &aq, &ms) == 7;
  if (well_formed) {
    t = krr_tuning{tile, g, z, pr, la, aq};
    well_formed = tuning_valid(t);
  }
  return true;
}

static std::map<std::string, std::string> cache_read(const char *path) {
  std::map<std::string, std::string> lines;
  FILE *f = fopen(path, "r");
  if (!f) return lines;
  char buf[1024];
  while (fgets(buf, sizeof buf, f)) {
    std::string key;
    krr_tuning t;
    double ms;
    bool ok;
    size_t len = strlen(buf);
    while (len && (buf[len - 1] == '\n' || buf[len - 1] == '\r' || buf[len - 1] == ',')) buf[--len] = 0;
    if (cache_parse_line(buf, key, t, ms, ok)) lines[key] = buf;
  }
  fclose(f);
  return lines;
}

krr_status krr_tuning_cache_load(const char *path, const char *key, krr_tuning *t, double *ms,
                                 int32_t *found) {
  if (!path || !key || !t || !found) return KRR_ERROR_INVALID_VALUE;
  *found = 0;
  auto lines = cache_read(path);
  auto it = lines.find(key);
  if (it == lines.end()) return KRR_SUCCESS;
  std::string k;
  krr_tuning v;
  double m = 0;
  bool ok = false;
  cache_parse_line(it->second.c_str(), k, v, m, ok);
  if (!ok) return KRR_ERROR_INVALID_VALUE;
  *t = v;
  if (ms) *ms = m;
  *found = 1;
  return KRR_SUCCESS;
}

krr_status krr_tuning_cache_store(const char *path, const char *key, const krr_tuning *t,
                                  double ms) {
  if (!path || !key || !t || !tuning_valid(*t) || strchr(key, '"') || strchr(key, '\n'))
    return KRR_ERROR_INVALID_VALUE;
  auto lines = cache_read(path);
  char buf[1024];
  snprintf(buf, sizeof buf,
           "\"%s\": {\"tile\": %d, \"panel_group\": %d, \"residual_split\": %d, "
           "\"sweep_pairs\": %d, \"lookahead\": %d, \"aux_cu_eighths\": %d, \"ms\": %.6f}",
           key, t->tile, t->panel_group, t->residual_split, t->sweep_pairs, t->lookahead,
           t->aux_cu_eighths, ms);
  lines[key] = buf;
  std::string tmp = std::string(path) + ".tmp";
  FILE *f = fopen(tmp.c_str(), "w");
  if (!f) return KRR_ERROR_INVALID_VALUE;
  fprintf(f, "{\n");
  size_t i = 0;
  for (auto &kv : lines) fprintf(f, "%s%s\n", kv.second.c_str(), ++i < lines.size() ? "," : "");
  fprintf(f, "}\n");
  const bool ok = fclose(f) == 0 && rename(tmp.c_str(), path) == 0;
  return ok ? KRR_SUCCESS : KRR_ERROR_INVALID_VALUE;
}

krr_status krr_autotune(krr_context ctx, const int8_t *G, int64_t n, int64_t m, int64_t ldg,
                        double gamma, double lambda, const double *Y, int64_t nrhs, int64_t ldy,
                        const krr_precision_policy *policy, const krr_refine_opts *refine,
                        const char *cache_path, krr_tuning *out, double *best_ms) {
  if (!ctx || !out || !Y || nrhs <= 0 || ldy < n || ctx->destroy_pending)
    return KRR_ERROR_INVALID_VALUE;
  CHK(build_args(G, n, m, ldg, gamma, lambda));
  if (ctx->live > 0) return KRR_ERROR_INVALID_VALUE;
  char key[512];
  CHK(krr_tuning_key(ctx->device, n, m, nrhs, policy, refine, key, sizeof key));
  if (cache_path) {
    krr_tuning t;
    double ms = 0;
    int32_t found = 0;
    if (krr_tuning_cache_load(cache_path, key, &t, &ms, &found) == KRR_SUCCESS && found) {
      CHK(krr_set_tuning(ctx, &t));
      *out = t;
      if (best_ms) *best_ms = ms;
      return KRR_SUCCESS;
    }
  }
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  double *X = nullptr;
  CHK(dalloc_t(ctx, &X, n * nrhs));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    dfree(ctx, X, (size_t)n * nrhs * 8);
    return KRR_ERROR_HIP;
  }
  const krr_tuning saved = ctx->tune;
  const int saved_tile = ctx->opts.tile;
  // one whole step under tuning t; its time in ms, or a negative value on failure
  auto run = [&](const krr_tuning &t) -> double {
    ctx->tune = t;
    ctx->opts.tile = t.tile;
    if (hipEventRecord(e0, s) != hipSuccess) return -1;
    krr_kernel K = nullptr;
    krr_factorization F = nullptr;
    krr_status st = krr_build_kernel(ctx, G, n, m, ldg, gamma, lambda, &K);
    if (st == KRR_SUCCESS) st = krr_factor(ctx, K, policy, &F);
    if (st == KRR_SUCCESS) st = krr_solve(ctx, F, Y, nrhs, ldy, X, n, refine, nullptr);
    if (F) krr_factor_release(F);
    if (K) krr_kernel_release(K);
    float ms = -1;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      return -1;
    return st == KRR_SUCCESS ? (double)ms : -1;
  };
  krr_tuning best{saved_tile, 0, 0, -1, -1, 0};
  double best_t = -1;
  auto consider = [&](const krr_tuning &t, bool warm) {
    if (warm) run(t);
    const double ms = run(t);
    if (ms >= 0 && (best_t < 0 || ms < best_t)) {
      best_t = ms;
      best = t;
    }
  };
  for (int tile : {512, 256}) {
    krr_tuning t{tile, 0, 0, -1, -1, 0};
    consider(t, true);
  }
  if (best_t >= 0) {
    const krr_tuning b0 = best;
    for (int g : {4, 6, 8}) {
      krr_tuning t = b0;
      t.panel_group = g;
      consider(t, false);
    }
    const krr_tuning b1 = best;
    for (int z : {-1, 4, 16}) {
      krr_tuning t = b1;
      t.residual_split = z;
      consider(t, false);
    }
    const krr_tuning b2 = best;
    for (int pr : {1, 0}) {
      krr_tuning t = b2;
      t.sweep_pairs = pr;
      consider(t, false);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  dfree(ctx, X, (size_t)n * nrhs * 8);
  if (best_t < 0) {
    ctx->tune = saved;
    ctx->opts.tile = saved_tile;
    return KRR_ERROR_NOT_CONVERGED;
  }
  ctx->tune = best;
  ctx->opts.tile = best.tile;
  *out = best;
  if (best_ms) *best_ms = best_t;
  if (cache_path) (void)krr_tuning_cache_store(cache_path, key, &best, best_t);
  return KRR_SUCCESS;
}

// ---------------------------------------------------------------------------
// Ridge Regression (the RR subsection, Eq. 1-2): beta = (X^T X + lambda I)^-1
// X^T Y.  X^T X is the linear kernel of the SNP columns (the rows of X^T),
// through the same INT8 Gram with exact int32 accumulation; the factorization,
// solves and FP64 refinement are the KRR ones.

krr_status krr_rr_fit(krr_context ctx, const int8_t *G, int64_t n, int64_t m, int64_t ldg,
                      const double *Y, int64_t nrhs, int64_t ldy, double lambda,
                      const krr_precision_policy *policy, const krr_refine_opts *refine,
                      double *beta, int64_t ldb, krr_solve_info *info) {
  if (!ctx || !Y || !beta || nrhs <= 0 || nrhs > 4096 || ldy < n || ldb < m)
    return KRR_ERROR_INVALID_VALUE;
  CHK(build_args(G, n, m, ldg, 1.0, lambda));
  if (n > (1LL << 22)) return KRR_ERROR_NOT_SUPPORTED;  // X^T X entries <= 4n stay exact in FP32
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  const int64_t ldgt = (n + 15) / 16 * 16;
  Scoped sc(ctx);
  int8_t *Gt = nullptr;
  double *B = nullptr;
  CHK(sc.alloc(&Gt, m * ldgt));
  CHK(sc.alloc(&B, m * nrhs));
  launch_transpose_i8(G, n, m, ldg, Gt, ldgt, s);                      // X^T: SNPs as rows
  launch_int8_t_times_f64(G, n, m, ldg, Y, (int)nrhs, ldy, B, m, s);   // X^T Y
  CHK(launch_ok());
  krr_kernel_desc d{};
  d.kind = KRR_KERNEL_LINEAR;
  krr_kernel K = nullptr;
  krr_factorization F = nullptr;
  krr_status st = krr_build_kernel_ex(ctx, Gt, m, n, ldgt, 1.0, lambda, &d, &K);
  if (st == KRR_SUCCESS) st = krr_factor(ctx, K, policy, &F);
  if (st == KRR_SUCCESS) st = krr_solve(ctx, F, B, nrhs, m, beta, ldb, refine, info);
  if (F) krr_factor_release(F);
  if (K) krr_kernel_release(K);
  return st;
}

krr_status krr_rr_predict(krr_context ctx, const int8_t *T, int64_t n_test, int64_t m,
                          int64_t ldt, const double *beta, int64_t nrhs, int64_t ldb, double *P,
                          int64_t ldp) {
  if (!ctx || !T || !beta || !P || n_test <= 0 || m <= 0 || nrhs <= 0 || ldt < m ||
      ldb < m || ldp < n_test)
    return KRR_ERROR_INVALID_VALUE;
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  const int64_t ldtt = (n_test + 15) / 16 * 16;
  Scoped sc(ctx);
  int8_t *Tt = nullptr;
  CHK(sc.alloc(&Tt, m * ldtt));
  launch_transpose_i8(T, n_test, m, ldt, Tt, ldtt, s);
  // P = T beta = (T^T)^T beta, the same int8-transposed product as X^T Y
  launch_int8_t_times_f64(Tt, m, n_test, ldtt, beta, (int)nrhs, ldb, P, ldp, s);
  CHK(launch_ok());
  HIPCHK(hipStreamSynchronize(s));
  return KRR_SUCCESS;
}
