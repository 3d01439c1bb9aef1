// C-ABI of libwf: context, batched MAP solve driver, simulations, band powers,
// operator-level calls and instrumentation.  The declarations and the contract of
// every entry point are in include/wf.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <sys/stat.h>
#include <tuple>
#include <vector>

#include "wf.h"
#include "wf_launch.hpp"
#include "wf_rfft.hpp"

using namespace wf;

// Device scratch of the allocation-free entry point (wf_hvp_noalloc), one copy per GPU that
// the library runs on, held until the process ends.  In host code this name is not a device
// address: each device's address is taken once, with that device current, by
// hipGetSymbolAddress in noalloc_setup (called from wf_create) and only that address is used.
static __device__ __align__(256) unsigned char scratch[WF_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t kAlign = 256;
constexpr int kNdot = 5 * MMAX + 1;
constexpr double kSimBudgetBytes = 48.0 * 1024 * 1024 * 1024;   // workspace cap of a sim chunk
constexpr int kMaxChunk = 256;
// the band-power estimates of several maps: one uneven batch of up to this many solves and bytes
// (classes of equal shape then run independently, so no solve waits for a slower map's)
constexpr double kMultiBudgetBytes = 96.0 * 1024 * 1024 * 1024;
constexpr int kMaxChunkMulti = 8192;
// Vectors of one instance are laid out back to back with this many extra bytes between
// them (an odd multiple of 256 B), so the 2m + 3 streams of a pass do not start at the same
// offset modulo a large power of two.
constexpr size_t kVecPadBytes = 4096 + 256;
constexpr int kMaxStreams = 4;   // the context stream plus up to 3 more for the classes of an uneven batch

const char* kKindNames[KK_COUNT] = {"colinv", "row", "colfwd", "passA", "passB", "post", "coef", "misc", "cg_dir",
                                     "simulate", "catalog"};

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
  int gen = 0;
};

}  // namespace

struct wf_ctx {
  int dev = 0;
  std::string err;
  hipStream_t cs = nullptr;
  hipEvent_t evIn = nullptr, evOut = nullptr;
  std::map<std::pair<int, int>, void*> tw;   // (n, dtype) -> twiddles
  std::map<std::tuple<int, int, int>, bool> prepared;
  Arena solveA, simA, opA, accA, refA;
  int* hstat = nullptr;
  size_t hstatCap = 0;
  // instrumentation
  bool prof = false;
  int64_t launches[KK_COUNT] = {};
  double ms[KK_COUNT] = {};
  double bytes[KK_COUNT] = {};
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pendingEv;
  std::vector<hipEvent_t> evPool;
  // graph cache: one captured graph per class of the current batch (key: arena, shapes, options)
  std::map<std::string, hipGraphExec_t> gexecs;
  // streams beside cs that run classes of an uneven batch concurrently, with their fork/join events
  std::vector<hipStream_t> xs;
  std::vector<hipEvent_t> xev;
  hipEvent_t evFork = nullptr;
  // chain tile choices: fixed by the caller (rbv > 0) or tuned per shape and batch size
  ChainCfg fixedCfg;
  bool fixedSet = false;
  std::map<std::tuple<int, int, int, int>, ChainCfg> tuned;
  // host copies of the twiddle tables (the allocation-free entry point stages them into the
  // device scratch) and this device's scratch address
  std::map<std::pair<int, int>, std::vector<char>> htw;
  void* scratch = nullptr;
  // on-disk cache of tuned tiles (empty path: none) and the device it is keyed by
  std::string tunePath, tuneDev;
  // catalog response: deconvolution tables 1 / phi^(k / 2n) per n
  std::map<int, std::vector<double>> catDk;
};

namespace {

int fail(wf_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(call)                                                                              \
  do {                                                                                            \
    hipError_t _e = (call);                                                                       \
    if (_e != hipSuccess)                                                                         \
      return fail(ctx, WF_EHIP, std::string(#call) + ": " + hipGetErrorString(_e));               \
  } while (0)

int esize_of(int dtype) { return dtype == WF_F64 ? 16 : 8; }
int rsize_of(int dtype) { return dtype == WF_F64 ? 8 : 4; }

int arena_reserve(wf_ctx* ctx, Arena& a, size_t bytes) {
  if (bytes <= a.cap) {
    a.used = 0;
    return WF_OK;
  }
  if (a.base) {
    // work of an earlier call (on any of the context's streams) may still use the old block
    HIPCHK(hipStreamSynchronize(ctx->cs));
    for (auto x : ctx->xs) HIPCHK(hipStreamSynchronize(x));
    HIPCHK(hipFree(a.base));
    a.base = nullptr;
    a.cap = 0;
  }
  size_t want = bytes + bytes / 8;
  if (hipMalloc((void**)&a.base, want) != hipSuccess) {
    (void)hipGetLastError();
    a.base = nullptr;
    if (hipMalloc((void**)&a.base, bytes) != hipSuccess) {
      (void)hipGetLastError();
      a.base = nullptr;
      return fail(ctx, WF_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    want = bytes;
  }
  a.cap = want;
  a.used = 0;
  a.gen++;
  if (&a == &ctx->solveA) {
    for (auto& kv : ctx->gexecs) (void)hipGraphExecDestroy(kv.second);
    ctx->gexecs.clear();
  }
  return WF_OK;
}

char* arena_take(Arena& a, size_t bytes) {
  char* p = a.base + a.used;
  a.used += align_up(bytes);
  return p;
}

int host_status(wf_ctx* ctx, size_t n) {
  if (n <= ctx->hstatCap) return WF_OK;
  if (ctx->hstat) (void)hipHostFree(ctx->hstat);
  ctx->hstat = nullptr;
  HIPCHK(hipHostMalloc((void**)&ctx->hstat, n * sizeof(int), hipHostMallocDefault));
  ctx->hstatCap = n;
  return WF_OK;
}

// Twiddles, generated in float64: exp(-2 pi i k / n) for k in [0, n); for power-of-two n
// also the stage tables of the register-staged transforms (column schedules of length n
// and row schedules of length n / 2, at tw_col_off / tw_row_off).
static void stage_table(std::vector<double>& h, int64_t at, int len, int E, bool rev) {
  const int S = rs_nst(len, E), R0 = rs_radix(len, E, rev, 0);
  for (int s = 1; s < S; ++s) {
    const int R = rs_radix(len, E, rev, s), NS = rs_ns(len, E, rev, s);
    const int64_t off = at + (NS - R0);
    for (int r = 1; r < R; ++r)
      for (int k = 0; k < NS; ++k) {
        const int64_t M = (int64_t)NS * R;
        const double a = 2.0 * M_PI * (double)(((int64_t)r * k) % M) / (double)M;
        const int64_t e = off + (int64_t)(r - 1) * NS + k;
        h[2 * e] = std::cos(a);
        h[2 * e + 1] = -std::sin(a);
      }
  }
}

// the twiddle table of (n, dtype) as device-ready bytes
void twiddle_bytes(int n, int dtype, std::vector<char>& out) {
  const bool pow2 = (n & (n - 1)) == 0 && n >= 8;
  const int64_t entries = pow2 ? tw_ext_entries(n) : n;
  std::vector<double> h(2 * (size_t)entries, 0.0);
  for (int k = 0; k < n; ++k) {
    const double a = 2.0 * M_PI * (double)k / (double)n;
    h[2 * k] = std::cos(a);
    h[2 * k + 1] = -std::sin(a);
  }
  if (pow2) {
    for (int E = 2; E <= 32; E *= 2) stage_table(h, tw_col_off(n, E), n, E, false);
    for (int E = 8; E <= 32; E *= 2) {
      stage_table(h, tw_row_off(n, E, false), n / 2, E, false);
      stage_table(h, tw_row_off(n, E, true), n / 2, E, true);
    }
  }
  const size_t bytes = (size_t)entries * esize_of(dtype);
  out.resize(bytes);
  if (dtype == WF_F64) {
    std::memcpy(out.data(), h.data(), bytes);
  } else {
    std::vector<float> f(h.begin(), h.end());
    std::memcpy(out.data(), f.data(), bytes);
  }
}

int twiddles(wf_ctx* ctx, int n, int dtype, const void** out) {
  auto key = std::make_pair(n, dtype);
  auto it = ctx->tw.find(key);
  if (it != ctx->tw.end()) {
    *out = it->second;
    return WF_OK;
  }
  std::vector<char> h;
  twiddle_bytes(n, dtype, h);
  void* d = nullptr;
  HIPCHK(hipMalloc(&d, h.size()));
  HIPCHK(hipMemcpy(d, h.data(), h.size(), hipMemcpyHostToDevice));
  ctx->tw[key] = d;
  *out = d;
  return WF_OK;
}

// Per-device address of `scratch`, taken once per device with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

int noalloc_setup(wf_ctx* ctx) {
  if (ctx->dev < 0 || ctx->dev >= kMaxDevices) return fail(ctx, WF_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[ctx->dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(ctx, WF_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch[ctx->dev] = p;
  }
  ctx->scratch = g_scratch[ctx->dev];
  return WF_OK;
}

int prepare(wf_ctx* ctx, int n, int c, int dtype) {
  auto key = std::make_tuple(n, c, dtype);
  if (ctx->prepared.count(key)) return WF_OK;
  HIPCHK(chain_prepare(dtype, n, c));
  ctx->prepared[key] = true;
  return WF_OK;
}

// ---------------------------------------------------------------------------- launch helpers
hipEvent_t ev_get(wf_ctx* ctx) {
  if (!ctx->evPool.empty()) {
    hipEvent_t e = ctx->evPool.back();
    ctx->evPool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

struct Timed {
  wf_ctx* ctx;
  int kind;
  hipEvent_t a = nullptr, b = nullptr;
  Timed(wf_ctx* c, int k) : ctx(c), kind(k) {
    ctx->launches[k]++;
    if (ctx->prof) {
      a = ev_get(ctx);
      b = ev_get(ctx);
      (void)hipEventRecord(a, ctx->cs);
    }
  }
  ~Timed() {
    if (ctx->prof) {
      (void)hipEventRecord(b, ctx->cs);
      ctx->pendingEv.push_back({kind, {a, b}});
    }
  }
};

int drain_events(wf_ctx* ctx) {
  if (ctx->pendingEv.empty()) return WF_OK;
  HIPCHK(hipStreamSynchronize(ctx->cs));
  for (auto& pe : ctx->pendingEv) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, pe.second.first, pe.second.second) == hipSuccess) ctx->ms[pe.first] += t;
    ctx->evPool.push_back(pe.second.first);
    ctx->evPool.push_back(pe.second.second);
  }
  ctx->pendingEv.clear();
  return WF_OK;
}

// tiles of operator-level calls: the fixed choice if one is set and supported, else the default
// operator calls run every mode through the three passes (the single pass is for solvers)
ChainCfg op_cfg(const wf_ctx* ctx, int dtype, int n, int c) {
  return ctx->fixedSet && ctx->fixedCfg.reg != 8 && chain_cfg_supported(dtype, n, c, ctx->fixedCfg) ? ctx->fixedCfg
                                                                                                     : ChainCfg();
}

hipError_t chain(wf_ctx* ctx, int dtype, int n, int c, int which, const Job* jobs, int batch, const void* tw,
                 const ChainCfg* cfgp = nullptr) {
  Timed t(ctx, (cfgp && cfgp->sim) ? KK_SIM : (which == CH_COLINV ? KK_COLINV : (which == CH_ROW ? KK_ROW : KK_COLFWD)));
  const ChainCfg cfg = cfgp ? *cfgp : op_cfg(ctx, dtype, n, c);
  return chain_launch(dtype, n, c, which, cfg, jobs, batch, tw, ctx->cs);
}

// ---------------------------------------------------------------------------- validation
int check_problem(wf_ctx* ctx, const wf_problem* p, bool need_data) {
  if (!p) return fail(ctx, WF_EINVAL, "null problem");
  if (!chain_supported(p->n))
    return fail(ctx, WF_EINVAL, "unsupported n=" + std::to_string(p->n) +
                                    " (need n % 8 == 0, 8 <= n <= 1024, n = 2^a or 3*2^a)");
  if (p->ncomp != 1 && p->ncomp != 2) return fail(ctx, WF_EINVAL, "ncomp must be 1 or 2");
  if (p->dtype != WF_F32 && p->dtype != WF_F64) return fail(ctx, WF_EINVAL, "dtype must be WF_F32 or WF_F64");
  if (p->nbands < 0 || p->nbands > 4096) return fail(ctx, WF_EINVAL, "nbands out of range");
  if (!p->w || !p->pshape || !p->band) return fail(ctx, WF_EINVAL, "null w / pshape / band");
  if (p->nbands > 0 && !p->theta) return fail(ctx, WF_EINVAL, "null theta");
  if (need_data && !p->d) return fail(ctx, WF_EINVAL, "null d");
  if (p->theta)
    for (int b = 0; b < p->nbands; ++b)
      if (!std::isfinite(p->theta[b])) return fail(ctx, WF_ENONFINITE, "non-finite theta");
  return WF_OK;
}

void fill_opts(const wf_lbfgs_opts* o, wf_lbfgs_opts& r) {
  wf_lbfgs_default(&r);
  if (o) r = *o;
  if (r.m <= 0) r.m = 10;
  if (r.max_iter <= 0) r.max_iter = 20000;
  if (!(r.rel_grad_tol > 0)) r.rel_grad_tol = 1e-6;
  if (r.precond != 0) r.precond = 1;
  if (r.method != WF_METHOD_CG) r.method = WF_METHOD_LBFGS;
  if (r.method == WF_METHOD_CG) r.m = 1;   // CG keeps w, g, p and Dp: one pair of the vector block
  if (r.refine < 0) r.refine = 0;
  if (r.refine > 16) r.refine = 16;
  if (!(r.refine_tol > 0)) r.refine_tol = 1e-10;
}

// ---------------------------------------------------------------------------- prior tables
struct PriorTab {
  void* sq = nullptr;         // [c][n][h] real
  int32_t* bandI = nullptr;   // [c][n][h]
  double* theta = nullptr;    // [nbands]
  void* a = nullptr;          // preconditioned solves: P = 1 / (1 + S <W>)
  void* ainv = nullptr;       // and 1 / P
};

size_t prior_bytes(const wf_problem* p, bool precond = false) {
  const size_t L = (size_t)p->ncomp * p->n * (p->n / 2);
  return align_up(L * rsize_of(p->dtype)) + align_up(L * 4) + align_up(sizeof(double) * (std::max(1, p->nbands) + 1)) +
         (precond ? 2 * align_up(L * rsize_of(p->dtype)) : 0);
}

int build_prior(wf_ctx* ctx, Arena& a, const wf_problem* p, const double* theta, PriorTab& t, bool precond = false) {
  const size_t L = (size_t)p->ncomp * p->n * (p->n / 2);
  t.sq = arena_take(a, L * rsize_of(p->dtype));
  t.bandI = (int32_t*)arena_take(a, L * 4);
  t.theta = (double*)arena_take(a, sizeof(double) * (std::max(1, p->nbands) + 1));
  double* meanW = t.theta + std::max(1, p->nbands);
  t.a = t.ainv = nullptr;
  if (precond) {
    t.a = arena_take(a, L * rsize_of(p->dtype));
    t.ainv = arena_take(a, L * rsize_of(p->dtype));
  }
  if (p->nbands > 0)
    HIPCHK(hipMemcpyAsync(t.theta, theta, sizeof(double) * p->nbands, hipMemcpyHostToDevice, ctx->cs));
  HIPCHK(prior_table_launch(p->dtype, p->n, p->ncomp, p->pshape, p->band, t.theta, p->nbands,
                            precond ? p->w : nullptr, meanW, t.sq, t.bandI, t.a, t.ainv, ctx->cs));
  return WF_OK;
}

struct StreamScope {
  wf_ctx* ctx;
  hipStream_t us;
  StreamScope(wf_ctx* c, void* s) : ctx(c), us((hipStream_t)s) {
    (void)hipSetDevice(ctx->dev);
    (void)hipEventRecord(ctx->evIn, us);
    (void)hipStreamWaitEvent(ctx->cs, ctx->evIn, 0);
  }
  ~StreamScope() {
    (void)hipEventRecord(ctx->evOut, ctx->cs);
    (void)hipStreamWaitEvent(us, ctx->evOut, 0);
  }
};

// ---------------------------------------------------------------------------- catalogs
// The catalog-level response (sec. 3.4) as a non-uniform FFT on the fine grid of N = 2n
// points per side.  Set-up on the device, once per call and catalog: each galaxy's fine cell
// (rho = 2 r wrapped into [0, N)), a stable radix sort of the galaxies by cell (a cell keeps
// the input order, so every sum over galaxies has the same order on every call), and in the
// sorted order each galaxy's cell and kernel weights and the first galaxy of every cell.
struct CatPlan {
  int n = 0, N = 0, c = 0, ngal = 0, tiles = 0;
  const wf_catalog* src = nullptr;
  uint32_t* perm = nullptr;   // device: sorted position -> input index (after cat_fill)
};

constexpr int kCatMaxGal = 1 << 27;

int check_catalog(wf_ctx* ctx, const wf_problem* p, const wf_catalog* cat, bool solve) {
  if (!p || !cat) return fail(ctx, WF_EINVAL, "null problem / catalog");
  if (!chain_supported(p->n) || !chain_supported(2 * p->n))
    return fail(ctx, WF_EINVAL, "unsupported n=" + std::to_string(p->n) +
                                    " for a catalog (need n % 8 == 0, 8 <= n <= 512, n = 2^a or 3*2^a)");
  if (p->ncomp != 1 && p->ncomp != 2) return fail(ctx, WF_EINVAL, "ncomp must be 1 or 2");
  if (p->dtype != WF_F32) return fail(ctx, WF_EINVAL, "catalogs are float32 only");
  if (cat->ngal < 1 || cat->ngal > kCatMaxGal) return fail(ctx, WF_EINVAL, "ngal out of range");
  if (!cat->pos) return fail(ctx, WF_EINVAL, "null catalog positions");
  if (!solve) return WF_OK;
  if (!cat->e || !cat->wgt) return fail(ctx, WF_EINVAL, "null catalog e / wgt");
  if (p->nbands < 0 || p->nbands > 4096) return fail(ctx, WF_EINVAL, "nbands out of range");
  if (!p->pshape || !p->band) return fail(ctx, WF_EINVAL, "null pshape / band");
  if (p->nbands > 0 && !p->theta) return fail(ctx, WF_EINVAL, "null theta");
  for (int b = 0; b < p->nbands; ++b)
    if (!std::isfinite(p->theta[b])) return fail(ctx, WF_ENONFINITE, "non-finite theta");
  return WF_OK;
}

void cat_plan(const wf_catalog* cat, int n, int c, CatPlan& h) {
  h.n = n;
  h.N = 2 * n;
  h.c = c;
  h.ngal = cat->ngal;
  h.tiles = h.N / CAT_TS;
  h.src = cat;
}

int cat_key_bits(int N) {
  int b = 1;
  while ((1ull << b) < (unsigned long long)N * N) ++b;
  return b;
}

// 1 / phi^(k / N) for k = 0 .. n/2, phi the spreading kernel exp(beta (sqrt(1 - (2z/W)^2) - 1))
// on |z| <= W/2 (the device's beta, W): phi^(xi) = int phi(z) cos(2 pi xi z) dz
// = W int_0^{pi/2} exp(beta (cos t - 1)) cos(pi xi W sin t) cos t dt  (z = W/2 sin t), whose
// integrand is smooth (analytic in t), by composite Simpson in float64 on 1024 intervals (the
// k-independent factors tabulated once); kept per context and n.
const std::vector<double>& cat_deconv(wf_ctx* ctx, int n, int N) {
  auto it = ctx->catDk.find(n);
  if (it != ctx->catDk.end()) return it->second;
  constexpr int M = 1024;
  const double W = CAT_W, beta = (double)CAT_BETA, hq = 0.5 * M_PI / M;
  std::vector<double> amp(M + 1), arg(M + 1);
  for (int q = 0; q <= M; ++q) {
    const double t = q * hq;
    amp[q] = std::exp(beta * (std::cos(t) - 1.0)) * std::cos(t) * ((q == 0 || q == M) ? 1.0 : (q % 2 ? 4.0 : 2.0));
    arg[q] = M_PI * W * std::sin(t);
  }
  std::vector<double> dk(n / 2 + 1, 0.0);
  for (int k = 0; k <= n / 2; ++k) {
    const double xi = (double)k / N;
    double s = 0.0;
    for (int q = 0; q <= M; ++q) s += amp[q] * std::cos(xi * arg[q]);
    dk[k] = 1.0 / (W * s * hq / 3.0);
  }
  return ctx->catDk[n] = std::move(dk);
}

int cat_sort_bytes(wf_ctx* ctx, int N, int ngal, size_t& bytes) {
  bytes = 0;
  HIPCHK(cat_sort_launch(nullptr, &bytes, nullptr, nullptr, nullptr, nullptr, ngal, cat_key_bits(N), ctx->cs));
  return WF_OK;
}

size_t cat_bytes(int n, int c, int ngal, size_t sortBytes) {
  const size_t N = 2 * (size_t)n, g = (size_t)ngal, C = (size_t)c;
  return 4 * align_up(4 * g) + align_up(sortBytes) + align_up(sizeof(int)) + align_up(8 * g) +
         align_up(4 * CAT_REC * g) + align_up(4 * (N * N + 1)) + 2 * align_up(4 * C * g) + align_up(4 * g) +
         align_up(4 * C * n * (n / 2)) + align_up(8 * ((g + NT - 1) / NT)) + align_up(8 * ((size_t)n / 2 + 1)) +
         2 * align_up(8 * C * N * (N / 2)) + align_up(4 * C * N * N);
}

// Device set-up of one catalog: keys, sort, windows and cell table; the descriptor (host copy
// cd; jfwd / jadj are set by the caller), its fine-grid forward and adjoint jobs (host copies
// jf, ja, switched off), the table T from the scale table sq (nullptr: the unscaled operator)
// and, for solves, the measurements and weights gathered into the sorted order.
int cat_fill(wf_ctx* ctx, Arena& A, CatPlan& h, size_t sortBytes, const void* sq, bool solve, CatDesc& cd, Job& jf,
             Job& ja) {
  const int n = h.n, N = h.N, c = h.c, g = h.ngal;
  uint32_t* kin = (uint32_t*)arena_take(A, 4 * (size_t)g);
  uint32_t* kout = (uint32_t*)arena_take(A, 4 * (size_t)g);
  uint32_t* vin = (uint32_t*)arena_take(A, 4 * (size_t)g);
  uint32_t* perm = (uint32_t*)arena_take(A, 4 * (size_t)g);
  void* temp = arena_take(A, sortBytes);
  int* bad = (int*)arena_take(A, sizeof(int));
  int2* cell = (int2*)arena_take(A, 8 * (size_t)g);
  float4* rec = (float4*)arena_take(A, 4 * CAT_REC * (size_t)g);
  int* cellStart = (int*)arena_take(A, 4 * ((size_t)N * N + 1));
  float* de = (float*)arena_take(A, 4 * (size_t)c * g);
  float* dr = (float*)arena_take(A, 4 * (size_t)c * g);
  float* dw = (float*)arena_take(A, 4 * (size_t)g);
  float* dT = (float*)arena_take(A, 4 * (size_t)c * n * (n / 2));
  double* dpart = (double*)arena_take(A, 8 * (size_t)((g + NT - 1) / NT));
  double* ddk = (double*)arena_take(A, 8 * (size_t)(n / 2 + 1));
  void* y2 = arena_take(A, 8 * (size_t)c * N * (N / 2));
  void* yN = arena_take(A, 8 * (size_t)c * N * (N / 2));
  float* map = (float*)arena_take(A, 4 * (size_t)c * N * N);
  if (A.used > A.cap) return fail(ctx, WF_ENOMEM, "internal: catalog workspace overflow");
  const std::vector<double>& dk = cat_deconv(ctx, n, N);
  int hbad = 0;
  HIPCHK(hipMemcpyAsync(bad, &hbad, sizeof(int), hipMemcpyHostToDevice, ctx->cs));
  HIPCHK(hipMemcpyAsync(ddk, dk.data(), 8 * dk.size(), hipMemcpyHostToDevice, ctx->cs));
  HIPCHK(cat_keys_launch(h.src->pos, g, N, kin, vin, bad, ctx->cs));
  size_t tb = sortBytes;
  HIPCHK(cat_sort_launch(temp, &tb, kin, kout, vin, perm, g, cat_key_bits(N), ctx->cs));
  HIPCHK(cat_prep_launch(h.src->pos, kout, perm, g, N, cell, rec, cellStart, ctx->cs));
  HIPCHK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->cs));
  HIPCHK(hipStreamSynchronize(ctx->cs));   // hbad is local
  if (hbad) return fail(ctx, WF_ENONFINITE, "non-finite galaxy position");
  HIPCHK(cat_table_launch(n, N, c, (const float*)sq, ddk, dT, ctx->cs));
  if (solve) {
    HIPCHK(cat_permute_launch(h.src->e, (const int*)perm, de, g, c, 1, 0, ctx->cs));
    HIPCHK(cat_permute_launch(h.src->wgt, (const int*)perm, dw, g, 1, 1, 0, ctx->cs));
  }
  h.perm = perm;
  std::memset(&cd, 0, sizeof cd);
  cd.n = n;
  cd.N = N;
  cd.c = c;
  cd.ngal = g;
  cd.tiles = h.tiles;
  cd.nrowPart = c * n / RB_MIN;
  cd.cell = cell;
  cd.rec = rec;
  cd.cellStart = cellStart;
  cd.e = de;
  cd.wgt = dw;
  cd.T = dT;
  cd.aTab = nullptr;
  cd.y2 = y2;
  cd.u = map;
  cd.v = map;
  cd.r = dr;
  cd.partI = dpart;
  std::memset(&jf, 0, sizeof jf);
  std::memset(&ja, 0, sizeof ja);
  jf.mode = ja.mode = CM_NONE;
  jf.boost_band = ja.boost_band = -1;
  jf.vin = y2;
  jf.y = yN;
  jf.xout = map;
  ja.d = map;
  ja.y = yN;
  ja.vout = y2;
  return WF_OK;
}

hipError_t cat_step(wf_ctx* ctx, int which, int c, int blocks, const Job* jobs, CatDesc* cats, int count) {
  Timed t(ctx, KK_CAT);
  return cat_launch(which, c, blocks, jobs, cats, count, ctx->cs);
}

// ---------------------------------------------------------------------------- solve core
struct Klass {
  int n, c, dtype;
  std::vector<int> members;   // user indices
  int first = 0;              // position in the class-ordered arrays
  int64_t L = 0;
  int nchunk = 0, pstride = 0;
  int pu = PASS_U_FEW;   // vector loads per thread per stream of the class's vector passes
  ChainCfg cfg;    // tile choice of the transform chain
  const void* tw = nullptr;
  // catalog classes (sec. 3.4): fine grid N = 2n, its tiles per side, interpolation blocks of
  // the largest catalog, and the class's descriptors and fine-grid forward / adjoint jobs
  bool cat = false;
  int N = 0, tiles = 0, nblkI = 0;
  ChainCfg cfgN;
  const void* twN = nullptr;
  CatDesc* dcats = nullptr;
  Job* fjobs = nullptr;
  Job* ajobs = nullptr;
};

struct SolveOut {
  std::vector<void*> w;         // per user index: whitened solution
  std::vector<void*> y;         // per user index: intermediate buffer
  std::vector<PriorTab> prior;  // per user index
  std::vector<StateStat> st;    // per user index
  std::vector<int> order;       // class-ordered position of each user index
};

// On-disk cache of the tuned tiles: one line per (device, n, ncomp, dtype, batch-size bucket)
// with the choice, "<version> <device> <n> <c> <dtype> <bucket> <rbv> <cpb> <group> <reg>",
// where device is the architecture name and compute-unit count.  The path is WF_TUNE_CACHE
// if set (empty: no cache), else $XDG_CACHE_HOME/libwf/tiles.txt or ~/.cache/libwf/tiles.txt.
// Lines of another version or device, and choices the shape does not support, are ignored;
// every choice computes the same result, so a stale line costs speed at most.
constexpr int kTuneVersion = 1;

void tune_cache_open(wf_ctx* ctx) {
  const char* env = std::getenv("WF_TUNE_CACHE");
  std::string path;
  if (env) {
    path = env;
  } else if (const char* x = std::getenv("XDG_CACHE_HOME"); x && *x) {
    path = std::string(x) + "/libwf/tiles.txt";
  } else if (const char* h = std::getenv("HOME"); h && *h) {
    path = std::string(h) + "/.cache/libwf/tiles.txt";
  }
  hipDeviceProp_t prop;
  if (path.empty() || hipGetDeviceProperties(&prop, ctx->dev) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  std::string arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  ctx->tunePath = path;
  ctx->tuneDev = arch + "/" + std::to_string(prop.multiProcessorCount);
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return;
  char dev[128];
  int v, n, c, dt, bucket;
  ChainCfg cfg;
  while (std::fscanf(f, "%d %127s %d %d %d %d %d %d %d %d", &v, dev, &n, &c, &dt, &bucket, &cfg.rbv, &cfg.cpb, &cfg.group,
                     &cfg.reg) == 10) {
    if (v == kTuneVersion && ctx->tuneDev == dev && chain_supported(n) && (c == 1 || c == 2) &&
        (dt == WF_F32 || dt == WF_F64) && cfg.group >= 0 && chain_cfg_supported(dt, n, c, cfg))
      ctx->tuned[std::make_tuple(n, c, dt, bucket)] = cfg;
  }
  std::fclose(f);
}

void tune_cache_add(wf_ctx* ctx, const std::tuple<int, int, int, int>& key, const ChainCfg& cfg) {
  if (ctx->tunePath.empty()) return;
  const size_t slash = ctx->tunePath.rfind('/');
  if (slash != std::string::npos && slash > 0) {   // create the directories
    for (size_t i = 1; i <= slash; ++i)
      if (ctx->tunePath[i] == '/' || i == slash) (void)mkdir(ctx->tunePath.substr(0, i).c_str(), 0755);
  }
  FILE* f = std::fopen(ctx->tunePath.c_str(), "a");
  if (!f) return;
  std::fprintf(f, "%d %s %d %d %d %d %d %d %d %d\n", kTuneVersion, ctx->tuneDev.c_str(), std::get<0>(key),
               std::get<1>(key), std::get<2>(key), std::get<3>(key), cfg.rbv, cfg.cpb, cfg.group, cfg.reg);
  std::fclose(f);
}

// Autotuner of the transform chain's tiles: times the curvature product of this class's own
// instances as the solver runs it (zero direction, real W and prior tables, the extra dots
// with g and m - 1 kept Dp_j) for every supported tile choice, best of 5, and keeps the
// fastest per (n, ncomp, dtype, batch-size bucket).  Runs once per key and
// context, outside graph capture; the buffers it touches are initialised afterwards.
int tune_chain(wf_ctx* ctx, Klass& k, const std::vector<InstDesc>& hd, Job* djobs, int m) {
  const int cnt = (int)k.members.size();
  const int bucket = cnt >= 64 ? 64 : (cnt >= 16 ? 16 : (cnt >= 4 ? 4 : 1));
  if (ctx->fixedSet) {
    k.cfg = chain_cfg_supported(k.dtype, k.n, k.c, ctx->fixedCfg) ? ctx->fixedCfg : ChainCfg();
    return WF_OK;
  }
  const auto key = std::make_tuple(k.n, k.c, k.dtype, bucket);
  auto it = ctx->tuned.find(key);
  if (it != ctx->tuned.end()) {
    k.cfg = it->second;
    return WF_OK;
  }
  k.cfg = ChainCfg();
  if (k.dtype != WF_F32 || cnt < 4 || ctx->prof) {
    ctx->tuned[key] = k.cfg;
    return WF_OK;
  }
  std::vector<Job> hj(cnt);
  for (int j = 0; j < cnt; ++j) {
    const InstDesc& D = hd[k.first + j];
    Job& jb = hj[j];
    std::memset(&jb, 0, sizeof jb);
    const size_t vb = (size_t)D.vstride * D.esize;
    jb.mode = CM_HV;
    jb.boost_band = -1;
    jb.vin = (char*)D.X + 2 * vb;
    jb.vadd = jb.vin;
    jb.vout = (char*)D.X + (2 + (size_t)m) * vb;
    jb.y = D.y;
    jb.W = D.W;
    jb.sIn = D.sq;
    jb.sOut = D.sq;
    jb.aTab = D.aTab;
    jb.part = D.partChain;
    jb.pstride = D.pstride;
    // the solver's curvature products also read g and the m - 1 other kept Dp_j
    jb.gvec = (char*)D.X + vb;
    jb.dpBase = (char*)D.X + (2 + (size_t)m) * vb;
    jb.dpStride = D.vstride;
    jb.dpMask = m > 1 ? ((1u << m) - 2u) : 0u;
    for (int v = 1; v < 2 + 2 * m; ++v)
      if (v == 1 || v == 2 || v >= 3 + m) HIPCHK(hipMemsetAsync((char*)D.X + v * vb, 0, (size_t)D.L * D.esize, ctx->cs));
  }
  Job* dj = djobs + k.first;
  HIPCHK(hipMemcpyAsync(dj, hj.data(), sizeof(Job) * cnt, hipMemcpyHostToDevice, ctx->cs));
  std::vector<ChainCfg> cands;
  for (int reg = 0; reg < 8; ++reg)
    for (int rbv : {2, 4, 8}) {
      if ((reg & 1) && rbv != 4) continue;   // the register-staged row pass has its own tile
      for (int cpb : {1, 2, 4})
        for (int grp : {0, 32}) {
          if (grp > 0 && cnt <= grp) continue;
          ChainCfg c;
          c.rbv = rbv;
          c.cpb = cpb;
          c.group = grp;
          c.reg = reg;
          if (chain_cfg_supported(k.dtype, k.n, k.c, c)) cands.push_back(c);
        }
    }
  {   // the single pass for maps that fit one work-group's LDS
    ChainCfg c;
    c.reg = 8;
    if (chain_cfg_supported(k.dtype, k.n, k.c, c)) cands.push_back(c);
  }
  hipEvent_t e0 = ev_get(ctx), e1 = ev_get(ctx);
  std::vector<float> times;
  for (const ChainCfg& c : cands) {
    auto run = [&]() -> hipError_t {
      const int G = c.group > 0 ? std::min(c.group, cnt) : cnt;
      for (int g0 = 0; g0 < cnt; g0 += G)
        for (int w = 0; w < 3; ++w) {
          hipError_t e = chain_launch(k.dtype, k.n, k.c, w, c, dj + g0, std::min(G, cnt - g0), k.tw, ctx->cs);
          if (e != hipSuccess) return e;
        }
      return hipSuccess;
    };
    HIPCHK(run());   // warm-up
    float tmin = 1e30f;
    for (int r = 0; r < 5; ++r) {
      HIPCHK(hipEventRecord(e0, ctx->cs));
      HIPCHK(run());
      HIPCHK(hipEventRecord(e1, ctx->cs));
      HIPCHK(hipEventSynchronize(e1));
      float t = 0.f;
      HIPCHK(hipEventElapsedTime(&t, e0, e1));
      tmin = std::min(tmin, t);
    }
    times.push_back(tmin);
  }
  // fastest candidate; one that launches each pass once for the whole class wins unless a
  // grouped one is more than 3 % faster (the timing noise is about 1-2 %, and grouping
  // multiplies the launches)
  size_t bi = 0, bu = cands.size();
  for (size_t i = 0; i < cands.size(); ++i) {
    if (times[i] < times[bi]) bi = i;
    if (cands[i].group == 0 && (bu == cands.size() || times[i] < times[bu])) bu = i;
  }
  if (!cands.empty()) k.cfg = (bu < cands.size() && times[bu] <= 1.03f * times[bi]) ? cands[bu] : cands[bi];
  ctx->evPool.push_back(e0);
  ctx->evPool.push_back(e1);
  ctx->tuned[key] = k.cfg;
  tune_cache_add(ctx, key, k.cfg);
  return WF_OK;
}

// Float64 residual refinement of float32 solves (option refine > 0).  The stop test of the
// float32 solve measures the whitened gradient, which the stiff (high signal-to-noise) modes
// dominate; on very red spectra (the CMB workload) a solve stopped at 1e-6 can still be 1e-2
// off in the map, and float32 cannot evaluate the gradient much below 1e-7 of its start.
// Each round evaluates the exact gradient g of every instance of the float32 classes in
// float64 (float64 copies of d, W, the prior tables and the solution v; the same rounded
// tables as the float32 solve, so both solve the same problem), and for the instances
// whose float64 relative gradient |g|_w / |g(0)|_w still exceeds refine_tol runs a float32
// correction solve of D delta = -g (the same batched solver on zero data, with -g as an
// explicit right-hand side, to a relative gradient of max(0.3 refine_tol / current, 1e-3)),
// then v += delta in float64.  At most `refine` correction rounds; the last evaluation gives
// the reported chi^2 and relative gradient.  Instances whose first solve did not converge are
// left as they are.
// The float32 evaluation of a correction's own gradient is limited by the stiff part of D
// acting on a residual that sits mostly in soft modes: its relative-gradient stop ends between
// ~1e-5 and ~1e-3 of its start on the CMB maps (against ~2e-8 for a full solve), so a round
// asks for at most a 1e-3 reduction (which gives more in the float64 gradient) and is capped
// at six times the iterations of the first solve (at least kRefineMinIter; each round starts a
// new history, and on the 1024^2 CMB map a round needs several times the first solve's
// iterations); a round that hits its cap still improves the field and is kept.
#ifndef WF_REFINE_TOL_MIN
#define WF_REFINE_TOL_MIN 1e-3
#endif
#ifndef WF_REFINE_ITER_FACTOR
#define WF_REFINE_ITER_FACTOR 6
#endif
constexpr double kRefineTolMin = WF_REFINE_TOL_MIN;
constexpr int kRefineIterFactor = WF_REFINE_ITER_FACTOR;
constexpr int kRefineMinIter = 200;

template <typename InitF, typename RunF>
int refine_f64(wf_ctx* ctx, const wf_lbfgs_opts& o, const std::vector<Klass>& ks, std::vector<InstDesc>& hd,
               InstDesc* ddesc, LbState* dst, StateStat* dss, std::vector<StateStat>& hs, InitF& init_class,
               RunF& run_loop) {
  const double T = o.refine_tol;
  std::vector<int> fk;
  for (size_t c = 0; c < ks.size(); ++c)
    if (ks[c].dtype == WF_F32 && !ks[c].cat) fk.push_back((int)c);
  if (fk.empty()) return WF_OK;
  const int B = (int)hd.size();
  struct Ref {
    void *v64 = nullptr, *g64 = nullptr, *y64 = nullptr, *d64 = nullptr, *W64 = nullptr, *sq64 = nullptr,
         *a64 = nullptr, *ainv64 = nullptr;
    float* rhs = nullptr;
    double *part64 = nullptr, *rpart = nullptr;
  };
  std::vector<Ref> rf(B);
  auto nblk_of = [](int64_t L) { return (int)std::min<int64_t>(256, (L + 255) / 256); };
  size_t total = 0;
  for (int c : fk) {
    const Klass& k = ks[c];
    const size_t L = (size_t)k.L, npix = (size_t)k.c * k.n * k.n, cnt = k.members.size();
    const size_t per = 3 * align_up(L * 16) + align_up(npix * 8) + align_up((size_t)k.n * k.n * 8) + 3 * align_up(L * 8) +
                       align_up(L * 8) + align_up(sizeof(double) * PK_COUNT * k.pstride) +
                       align_up(sizeof(double) * nblk_of(k.L));
    total += per * cnt + align_up(npix * 4) + align_up(sizeof(Job) * cnt) + align_up(sizeof(RhsJob) * cnt) +
             2 * align_up(sizeof(CvtJob) * 6 * cnt);
  }
  int rc = arena_reserve(ctx, ctx->refA, total);
  if (rc) return rc;
  Arena& A = ctx->refA;
  struct KRef {
    void* zero = nullptr;
    Job* jobs = nullptr;
    RhsJob* rj = nullptr;
    CvtJob* cv = nullptr;   // promotions, then the accumulation / demotion jobs
    CvtJob* cv2 = nullptr;
    const void* tw = nullptr;
  };
  std::vector<KRef> kr(ks.size());
  ChainCfg cfg64;
  for (int c : fk) {
    const Klass& k = ks[c];
    const size_t L = (size_t)k.L, npix = (size_t)k.c * k.n * k.n, cnt = k.members.size();
    KRef& K = kr[c];
    K.zero = arena_take(A, npix * 4);
    K.jobs = (Job*)arena_take(A, sizeof(Job) * cnt);
    K.rj = (RhsJob*)arena_take(A, sizeof(RhsJob) * cnt);
    K.cv = (CvtJob*)arena_take(A, sizeof(CvtJob) * 6 * cnt);
    K.cv2 = (CvtJob*)arena_take(A, sizeof(CvtJob) * 6 * cnt);
    HIPCHK(hipMemsetAsync(K.zero, 0, npix * 4, ctx->cs));
    rc = twiddles(ctx, k.n, WF_F64, &K.tw);
    if (rc) return rc;
    rc = prepare(ctx, k.n, k.c, WF_F64);
    if (rc) return rc;
    std::vector<Job> hj(cnt);
    std::vector<RhsJob> hr(cnt);
    std::vector<CvtJob> hc;
    for (size_t j = 0; j < cnt; ++j) {
      const int gi = k.first + (int)j;
      const InstDesc& D = hd[gi];
      Ref& r = rf[gi];
      r.v64 = arena_take(A, L * 16);
      r.g64 = arena_take(A, L * 16);
      r.y64 = arena_take(A, L * 16);
      r.d64 = arena_take(A, npix * 8);
      r.W64 = arena_take(A, (size_t)k.n * k.n * 8);
      r.sq64 = arena_take(A, L * 8);
      r.a64 = arena_take(A, L * 8);
      r.ainv64 = arena_take(A, L * 8);
      r.rhs = (float*)arena_take(A, L * 8);
      r.part64 = (double*)arena_take(A, sizeof(double) * PK_COUNT * k.pstride);
      r.rpart = (double*)arena_take(A, sizeof(double) * nblk_of(k.L));
      hc.push_back(CvtJob{D.d, r.d64, (int64_t)npix, CVT_F32_F64, 0});
      hc.push_back(CvtJob{D.W, r.W64, (int64_t)k.n * k.n, CVT_F32_F64, 0});
      hc.push_back(CvtJob{D.sq, r.sq64, (int64_t)L, CVT_F32_F64, 0});
      hc.push_back(CvtJob{D.X, r.v64, (int64_t)(2 * L), CVT_F32_F64, 0});
      if (D.aTab) {
        hc.push_back(CvtJob{D.aTab, r.a64, (int64_t)L, CVT_F32_F64, 0});
        hc.push_back(CvtJob{D.ainv, r.ainv64, (int64_t)L, CVT_F32_F64, 0});
      }
      Job& jb = hj[j];
      std::memset(&jb, 0, sizeof jb);
      jb.mode = CM_GRAD;
      jb.boost_band = -1;
      jb.vin = r.v64;
      jb.vadd = r.v64;
      jb.vout = r.g64;
      jb.y = r.y64;
      jb.d = r.d64;
      jb.W = r.W64;
      jb.sIn = r.sq64;
      jb.sOut = r.sq64;
      jb.aTab = D.aTab ? r.a64 : nullptr;
      jb.part = r.part64;
      jb.pstride = k.pstride;
      hr[j] = RhsJob{(const double*)r.g64, D.aTab ? (const double*)r.ainv64 : nullptr, r.rhs, r.rpart, (int64_t)L};
    }
    HIPCHK(hipMemcpyAsync(K.jobs, hj.data(), sizeof(Job) * cnt, hipMemcpyHostToDevice, ctx->cs));
    HIPCHK(hipMemcpyAsync(K.rj, hr.data(), sizeof(RhsJob) * cnt, hipMemcpyHostToDevice, ctx->cs));
    HIPCHK(hipMemcpyAsync(K.cv, hc.data(), sizeof(CvtJob) * hc.size(), hipMemcpyHostToDevice, ctx->cs));
    {
      Timed t(ctx, KK_MISC);
      HIPCHK(convert_launch(K.cv, (int)hc.size(), (int64_t)std::max(npix, 2 * L), ctx->cs));
    }
  }
  std::vector<double> rho(B, 0.0), prev(B, 0.0), chi(B, 0.0);
  std::vector<int> conv0(B, 0), live(B, 0), addIt(B, 0), addGrad(B, 0);
  for (int c : fk)
    for (size_t j = 0; j < ks[c].members.size(); ++j) {
      const int gi = ks[c].first + (int)j;
      conv0[gi] = hs[gi].status == WF_SOLVE_CONVERGED;
      live[gi] = conv0[gi];
    }
  for (int round = 0;; ++round) {
    // float64 exact gradient, right-hand side and norms of every instance of the float32 classes
    for (int c : fk) {
      const Klass& k = ks[c];
      const int cnt = (int)k.members.size();
      for (int w = 0; w < 3; ++w) HIPCHK(chain(ctx, WF_F64, k.n, k.c, w, kr[c].jobs, cnt, kr[c].tw, &cfg64));
      Timed t(ctx, KK_MISC);
      HIPCHK(refine_rhs_launch(kr[c].rj, cnt, nblk_of(k.L), ctx->cs));
    }
    std::vector<std::vector<double>> hp(B), hq(B);
    for (int c : fk)
      for (size_t j = 0; j < ks[c].members.size(); ++j) {
        const int gi = ks[c].first + (int)j;
        hp[gi].resize((size_t)PK_COUNT * ks[c].pstride);
        hq[gi].resize(nblk_of(ks[c].L));
        HIPCHK(hipMemcpyAsync(hp[gi].data(), rf[gi].part64, sizeof(double) * hp[gi].size(), hipMemcpyDeviceToHost,
                              ctx->cs));
        HIPCHK(hipMemcpyAsync(hq[gi].data(), rf[gi].rpart, sizeof(double) * hq[gi].size(), hipMemcpyDeviceToHost,
                              ctx->cs));
      }
    HIPCHK(hipStreamSynchronize(ctx->cs));
    bool any = false;
    for (int c : fk) {
      const Klass& k = ks[c];
      const int ncol = (k.n / 2) / TB, nrow = k.c * k.n / RB_MIN;
      for (size_t j = 0; j < k.members.size(); ++j) {
        const int gi = k.first + (int)j;
        double gw = 0.0, pr = 0.0, res = 0.0;
        for (double v : hq[gi]) gw += v;
        for (int b = 0; b < ncol; ++b) pr += hp[gi][(size_t)PK_PRIOR * k.pstride + b];
        for (int b = 0; b < nrow; ++b) res += hp[gi][(size_t)PK_RES * k.pstride + b];
        const double g0 = hs[gi].g0norm;
        prev[gi] = rho[gi];
        rho[gi] = g0 > 0.0 ? std::sqrt(gw) / g0 : 0.0;
        chi[gi] = 2.0 * pr + res;
        if (conv0[gi]) addGrad[gi] += 1;
        // stop refining an instance that is done, that stopped improving (a round must at
        // least halve its gradient) or whose values are not finite
        if (live[gi] && (!(rho[gi] > T) || !std::isfinite(rho[gi]) || (round > 0 && !(rho[gi] < 0.5 * prev[gi]))))
          live[gi] = 0;
        any = any || live[gi];
      }
    }
    if (!any || round >= o.refine) break;
    // float32 correction solves of the instances still refined; the other members of their
    // classes stop at once (infinite tolerance); their v64 keeps their solution
    std::vector<int64_t> nrun(ks.size(), 0);
    for (int c : fk) {
      const Klass& k = ks[c];
      bool cls = false;
      for (size_t j = 0; j < k.members.size(); ++j) cls = cls || live[k.first + (int)j];
      if (!cls) continue;
      std::vector<InstDesc> dd(hd.begin() + k.first, hd.begin() + k.first + k.members.size());
      for (size_t j = 0; j < k.members.size(); ++j) {
        const int gi = k.first + (int)j;
        dd[j].d = kr[c].zero;
        dd[j].rhs = rf[gi].rhs;
        dd[j].dchi2Tol = 0.0;
        dd[j].tol = live[gi] ? std::max(0.3 * T / rho[gi], kRefineTolMin) : 1e300;
        dd[j].maxIter = std::min(o.max_iter, std::max(kRefineMinIter, kRefineIterFactor * hs[gi].iter));
      }
      HIPCHK(hipMemcpyAsync(ddesc + k.first, dd.data(), sizeof(InstDesc) * dd.size(), hipMemcpyHostToDevice, ctx->cs));
      rc = init_class(k);
      if (rc) return rc;
      nrun[c] = (int64_t)k.members.size();
    }
    rc = run_loop(nrun);
    if (rc) return rc;
    std::vector<StateStat> cs(B);
    HIPCHK(state_stats_launch(dst, dss, B, ctx->cs));
    HIPCHK(hipMemcpyAsync(cs.data(), dss, sizeof(StateStat) * B, hipMemcpyDeviceToHost, ctx->cs));
    HIPCHK(hipStreamSynchronize(ctx->cs));
    for (int c : fk) {
      if (nrun[c] == 0) continue;
      const Klass& k = ks[c];
      std::vector<CvtJob> hc;
      for (size_t j = 0; j < k.members.size(); ++j) {
        const int gi = k.first + (int)j;
        for (int q = 0; q < KK_COUNT; ++q) ctx->bytes[q] += cs[gi].bytes[q];
        if (!live[gi]) continue;
        addIt[gi] += cs[gi].iter;
        addGrad[gi] += cs[gi].ngrad;
        if (cs[gi].status == WF_SOLVE_NONFINITE) {   // keep the last good solution
          live[gi] = 0;
          continue;
        }
        hc.push_back(CvtJob{hd[gi].X, rf[gi].v64, 2 * k.L, CVT_ADD_F32_F64, 0});
      }
      if (!hc.empty()) {
        HIPCHK(hipMemcpyAsync(kr[c].cv2, hc.data(), sizeof(CvtJob) * hc.size(), hipMemcpyHostToDevice, ctx->cs));
        Timed t(ctx, KK_MISC);
        HIPCHK(convert_launch(kr[c].cv2, (int)hc.size(), 2 * k.L, ctx->cs));
      }
    }
  }
  // the refined solutions back into the solver's float32 vectors (the packing, maps and band
  // statistics read them there)
  for (int c : fk) {
    const Klass& k = ks[c];
    std::vector<CvtJob> hc;
    for (size_t j = 0; j < k.members.size(); ++j) {
      const int gi = k.first + (int)j;
      hc.push_back(CvtJob{rf[gi].v64, hd[gi].X, 2 * k.L, CVT_F64_F32, 0});
      if (!conv0[gi]) continue;
      StateStat& S = hs[gi];
      S.status = rho[gi] <= T ? WF_SOLVE_CONVERGED : WF_SOLVE_MAXITER;
      S.iter += addIt[gi];
      S.ngrad += addGrad[gi];
      S.chi2 = chi[gi];
      S.gg = (rho[gi] * S.g0norm) * (rho[gi] * S.g0norm);
    }
    HIPCHK(hipMemcpyAsync(kr[c].cv2, hc.data(), sizeof(CvtJob) * hc.size(), hipMemcpyHostToDevice, ctx->cs));
    Timed t(ctx, KK_MISC);
    HIPCHK(convert_launch(kr[c].cv2, (int)hc.size(), 2 * k.L, ctx->cs));
  }
  HIPCHK(hipStreamSynchronize(ctx->cs));
  return WF_OK;
}

// tols: nullable per-instance relative-gradient tolerances (user index), else o's
// cats (nullable): catalogs [B] in place of the problems' pixel data (every instance then
// uses the catalog response; no preconditioner, no refinement)
int solve_core(wf_ctx* ctx, const wf_problem* probs, int B, const wf_lbfgs_opts& o, SolveOut& out,
               const double* tols = nullptr, const wf_catalog* cats = nullptr) {
  const int m = o.m;
  if (m < 1 || m > MMAX) return fail(ctx, WF_EINVAL, "m must be in [1, 16]");
  if (cats && (o.precond || o.refine > 0)) return fail(ctx, WF_EINVAL, "catalog solves take no precond / refine");
  // group into classes of equal (n, ncomp, dtype) and response
  const bool isCat = cats != nullptr;
  std::vector<Klass> ks;
  for (int i = 0; i < B; ++i) {
    const wf_problem* p = &probs[i];
    int rc = isCat ? check_catalog(ctx, p, &cats[i], true) : check_problem(ctx, p, true);
    if (rc) return rc;
    bool found = false;
    for (auto& k : ks)
      if (k.n == p->n && k.c == p->ncomp && k.dtype == p->dtype && k.cat == isCat) {
        k.members.push_back(i);
        found = true;
        break;
      }
    if (!found) {
      Klass k;
      k.n = p->n;
      k.c = p->ncomp;
      k.dtype = p->dtype;
      k.cat = isCat;
      k.members.push_back(i);
      ks.push_back(k);
    }
  }
  // catalogs: shapes and the sorts' workspaces
  std::vector<CatPlan> ch(isCat ? B : 0);
  std::vector<size_t> sortB(ch.size(), 0);
  for (int i = 0; i < (int)ch.size(); ++i) {
    cat_plan(&cats[i], probs[i].n, probs[i].ncomp, ch[i]);
    int rc = cat_sort_bytes(ctx, ch[i].N, ch[i].ngal, sortB[i]);
    if (rc) return rc;
  }
  // distinct priors within the call
  std::map<std::tuple<const void*, const void*, int, int, int, std::vector<double>>, int> pmap;
  std::vector<int> pidx(B);
  std::vector<int> prepIdx;
  for (int i = 0; i < B; ++i) {
    const wf_problem* p = &probs[i];
    std::vector<double> th(p->theta, p->theta + p->nbands);
    // a preconditioned table also depends on W
    th.push_back(o.precond ? (double)(uintptr_t)p->w : 0.0);
    auto key = std::make_tuple((const void*)p->pshape, (const void*)p->band, p->n, p->ncomp, p->dtype, th);
    auto it = pmap.find(key);
    if (it == pmap.end()) {
      const int id = (int)prepIdx.size();
      pmap[key] = id;
      prepIdx.push_back(i);
      pidx[i] = id;
    } else {
      pidx[i] = it->second;
    }
  }
  // sizes
  size_t total = 0;
  for (int id : prepIdx) total += prior_bytes(&probs[id], o.precond != 0);
  int pos = 0;
  for (auto& k : ks) {
    k.first = pos;
    pos += (int)k.members.size();
    k.L = (int64_t)k.c * k.n * (k.n / 2);
    const size_t eb = esize_of(k.dtype);
    const int64_t nvec = k.L * 2 / (k.dtype == WF_F64 ? 2 : 4);
    const int64_t many = (nvec + NT * PASS_U_MANY - 1) / (NT * PASS_U_MANY);
    k.pu = many * (int64_t)k.members.size() >= PASS_MANY_MIN_GROUPS ? PASS_U_MANY : PASS_U_FEW;
    k.nchunk = (int)((nvec + NT * k.pu - 1) / (NT * k.pu));
    k.pstride = k.c * k.n / RB_MIN;   // row partials per component and RB_MIN rows
    const size_t vsb = (size_t)k.L * eb + kVecPadBytes;
    const size_t per = align_up((size_t)(2 + 2 * m) * vsb) + align_up(vsb) +
                       align_up(sizeof(double) * PK_COUNT * k.pstride) + align_up(sizeof(double) * kNdot * k.nchunk);
    total += per * k.members.size();
    int rc = twiddles(ctx, k.n, k.dtype, &k.tw);
    if (rc) return rc;
    rc = prepare(ctx, k.n, k.c, k.dtype);
    if (rc) return rc;
    if (k.cat) {
      k.N = 2 * k.n;
      k.tiles = k.N / CAT_TS;
      k.nblkI = 1;
      for (int ui : k.members) {
        k.nblkI = std::max(k.nblkI, (ch[ui].ngal + NT - 1) / NT);
        total += cat_bytes(k.n, k.c, ch[ui].ngal, sortB[ui]);
      }
      total += 2 * align_up(sizeof(Job) * k.members.size()) + align_up(sizeof(CatDesc) * k.members.size());
      k.cfgN = op_cfg(ctx, WF_F32, k.N, k.c);
      rc = twiddles(ctx, k.N, WF_F32, &k.twN);
      if (rc) return rc;
      rc = prepare(ctx, k.N, k.c, WF_F32);
      if (rc) return rc;
    }
  }
  total += align_up(sizeof(InstDesc) * B) + align_up(sizeof(LbState) * B) + align_up(sizeof(Job) * B) +
           align_up(sizeof(int) * B) + align_up(sizeof(StateStat) * B);
  int rc = arena_reserve(ctx, ctx->solveA, total);
  if (rc) return rc;
  Arena& A = ctx->solveA;
  InstDesc* ddesc = (InstDesc*)arena_take(A, sizeof(InstDesc) * B);
  LbState* dst = (LbState*)arena_take(A, sizeof(LbState) * B);
  Job* djobs = (Job*)arena_take(A, sizeof(Job) * B);
  int* dstat = (int*)arena_take(A, sizeof(int) * B);
  StateStat* dss = (StateStat*)arena_take(A, sizeof(StateStat) * B);
  // the catalog classes' descriptor and job arrays next, at offsets fixed by the batch shape
  // (captured graphs take them as kernel arguments)
  for (auto& k : ks) {
    if (!k.cat) continue;
    k.dcats = (CatDesc*)arena_take(A, sizeof(CatDesc) * k.members.size());
    k.fjobs = (Job*)arena_take(A, sizeof(Job) * k.members.size());
    k.ajobs = (Job*)arena_take(A, sizeof(Job) * k.members.size());
  }
  std::vector<PriorTab> ptabs(prepIdx.size());
  for (size_t id = 0; id < prepIdx.size(); ++id) {
    rc = build_prior(ctx, A, &probs[prepIdx[id]], probs[prepIdx[id]].theta, ptabs[id], o.precond != 0);
    if (rc) return rc;
  }
  std::vector<InstDesc> hd(B);
  out.w.assign(B, nullptr);
  out.y.assign(B, nullptr);
  out.prior.assign(B, PriorTab());
  out.order.assign(B, 0);
  for (auto& k : ks) {
    const size_t eb = esize_of(k.dtype);
    std::vector<CatDesc> hcd(k.cat ? k.members.size() : 0);
    std::vector<Job> hjf(hcd.size()), hja(hcd.size());
    for (size_t j = 0; j < k.members.size(); ++j) {
      const int ui = k.members[j];
      const int gi = k.first + (int)j;
      const wf_problem* p = &probs[ui];
      InstDesc& D = hd[gi];
      const size_t vsb = (size_t)k.L * eb + kVecPadBytes;
      D.X = arena_take(A, (size_t)(2 + 2 * m) * vsb);
      D.y = arena_take(A, vsb);
      D.vstride = (int64_t)(vsb / eb);
      D.NV = 2 + 2 * m;
      D.nchunk = k.nchunk;
      D.d = k.cat ? nullptr : p->d;
      D.W = k.cat ? nullptr : p->w;
      D.sq = ptabs[pidx[ui]].sq;
      D.aTab = ptabs[pidx[ui]].a;
      D.ainv = ptabs[pidx[ui]].ainv;
      D.partChain = (double*)arena_take(A, sizeof(double) * PK_COUNT * k.pstride);
      D.partA = (double*)arena_take(A, sizeof(double) * kNdot * k.nchunk);
      D.statusOut = dstat + gi;
      D.n = k.n;
      D.c = k.c;
      D.L = k.L;
      D.pstride = k.pstride;
      D.m = m;
      D.esize = (int)eb;
      D.maxIter = o.max_iter;
      D.refreshEvery = o.refresh_every;
      D.tol = tols ? tols[ui] : o.rel_grad_tol;
      D.dchi2Tol = o.dchi2_tol;
      D.vbytes = (double)k.L * eb;
      out.w[ui] = D.X;
      out.y[ui] = D.y;
      out.prior[ui] = ptabs[pidx[ui]];
      out.order[ui] = gi;
      if (k.cat) {
        rc = cat_fill(ctx, A, ch[ui], sortB[ui], D.sq, true, hcd[j], hjf[j], hja[j]);
        if (rc) return rc;
        hcd[j].jfwd = k.fjobs + j;
        hcd[j].jadj = k.ajobs + j;
      }
    }
    if (k.cat) {
      HIPCHK(hipMemcpyAsync(k.dcats, hcd.data(), sizeof(CatDesc) * hcd.size(), hipMemcpyHostToDevice, ctx->cs));
      HIPCHK(hipMemcpyAsync(k.fjobs, hjf.data(), sizeof(Job) * hjf.size(), hipMemcpyHostToDevice, ctx->cs));
      HIPCHK(hipMemcpyAsync(k.ajobs, hja.data(), sizeof(Job) * hja.size(), hipMemcpyHostToDevice, ctx->cs));
      HIPCHK(hipStreamSynchronize(ctx->cs));   // host copies are local
    }
  }
  HIPCHK(hipMemcpyAsync(ddesc, hd.data(), sizeof(InstDesc) * B, hipMemcpyHostToDevice, ctx->cs));
  for (auto& k : ks) {
    if (k.cat) continue;   // the coarse chain does not run for catalogs
    rc = tune_chain(ctx, k, hd, djobs, m);
    if (rc) return rc;
  }
  // start of a solve of every instance of a class: w = 0, state reset, exact gradient first
  auto init_class = [&](const Klass& k) -> int {
    const int cnt = (int)k.members.size();
    {
      Timed t(ctx, KK_MISC);
      const int64_t nvec = k.L * 2 / (k.dtype == WF_F64 ? 2 : 4);
      const unsigned bx = (unsigned)std::min<int64_t>((nvec + 255) / 256, 1024);
      HIPCHK(lbfgs_launch(k.dtype == WF_F64, m, k.pu, LB_ZERO, dim3(bx, cnt), ddesc + k.first, dst + k.first,
                          djobs + k.first, cnt, ctx->cs));
    }
    {
      Timed t(ctx, KK_MISC);
      HIPCHK(lbfgs_launch(k.dtype == WF_F64, m, k.pu, LB_INIT, dim3(1), ddesc + k.first, dst + k.first, djobs + k.first, cnt,
                          ctx->cs));
    }
    return WF_OK;
  };
  for (auto& k : ks) {
    rc = init_class(k);
    if (rc) return rc;
  }
  // one iteration of one class (classes share no buffers, so their iterations are independent)
  const bool cg = o.method == WF_METHOD_CG;
  auto body = [&](const Klass& k) -> int {
    const int cnt = (int)k.members.size();
    const int dt = k.dtype == WF_F64;
    if (k.cat) {
      // the catalog response in place of the coarse chain: pad to the fine grid, forward
      // transform, interpolation at the galaxies, spreading, adjoint transform, unpad
      Job* jc = djobs + k.first;
      HIPCHK(cat_step(ctx, CAT_PAD, k.c, k.N / 4, jc, k.dcats, cnt));
      HIPCHK(chain(ctx, WF_F32, k.N, k.c, CH_COLINV, k.fjobs, cnt, k.twN, &k.cfgN));
      HIPCHK(chain(ctx, WF_F32, k.N, k.c, CH_ROW, k.fjobs, cnt, k.twN, &k.cfgN));
      HIPCHK(cat_step(ctx, CAT_INTERP, k.c, k.nblkI, jc, k.dcats, cnt));
      HIPCHK(cat_step(ctx, CAT_SPREAD, k.c, k.tiles * k.tiles, jc, k.dcats, cnt));
      HIPCHK(chain(ctx, WF_F32, k.N, k.c, CH_ROW, k.ajobs, cnt, k.twN, &k.cfgN));
      HIPCHK(chain(ctx, WF_F32, k.N, k.c, CH_COLFWD, k.ajobs, cnt, k.twN, &k.cfgN));
      HIPCHK(cat_step(ctx, CAT_UNPAD, k.c, k.n / 4, jc, k.dcats, cnt));
    } else {
      const int G = k.cfg.group > 0 ? std::min(k.cfg.group, cnt) : cnt;
      for (int g0 = 0; g0 < cnt; g0 += G) {
        const int gc = std::min(G, cnt - g0);
        for (int w = 0; w < 3; ++w) HIPCHK(chain(ctx, k.dtype, k.n, k.c, w, djobs + k.first + g0, gc, k.tw, &k.cfg));
      }
    }
    auto launch = [&](int kk, int which, dim3 grid) -> int {
      Timed t(ctx, kk);
      HIPCHK(lbfgs_launch(dt, m, k.pu, which, grid, ddesc + k.first, dst + k.first, djobs + k.first, cnt, ctx->cs));
      return WF_OK;
    };
    int rc;
    if (cg) {
      if ((rc = launch(KK_COEF, LB_CGSTEP, dim3(cnt)))) return rc;
      if ((rc = launch(KK_PASSB, LB_CGPASS, dim3(k.nchunk, cnt)))) return rc;
      if ((rc = launch(KK_POST, LB_CGPOST, dim3(cnt)))) return rc;
      if ((rc = launch(KK_DIR, LB_CGDIR, dim3(k.nchunk, cnt)))) return rc;
    } else {
      if ((rc = launch(KK_PASSA, LB_PASSA, dim3(k.nchunk, cnt)))) return rc;
      if ((rc = launch(KK_COEF, LB_COEF, dim3(cnt)))) return rc;
      if ((rc = launch(KK_PASSB, LB_PASSB, dim3(k.nchunk, cnt)))) return rc;
      if ((rc = launch(KK_POST, LB_POSTB, dim3(cnt)))) return rc;
    }
    return WF_OK;
  };
  rc = host_status(ctx, B);
  if (rc) return rc;
  int K = o.iters_per_poll > 0 ? o.iters_per_poll : 8;   // iterations an instance may run past its stop are no-ops
  const bool graph = o.use_graph != 0 && !ctx->prof && K > 0;
  const int nk = (int)ks.size();
  std::vector<hipGraphExec_t> gx(nk, nullptr);
  if (graph) {
    // K iterations of each class captured once per (arena, batch shape, options); graphs of
    // earlier batch shapes are dropped
    std::vector<std::string> keys(nk);
    for (int c = 0; c < nk; ++c) {
      const Klass& k = ks[c];
      char buf[160];
      snprintf(buf, sizeof buf, "%p/%d/%d/%d/%d/%d|%d,%d,%d,%d,%zu,%d,%d,%d,%d|%d,%d", (void*)A.base, A.gen, B, m, K,
               o.method, k.first, k.n, k.c, k.dtype, k.members.size(), k.cfg.rbv, k.cfg.cpb, k.cfg.group, k.cfg.reg,
               (int)k.cat, k.nblkI);
      keys[c] = buf;
    }
    for (auto it = ctx->gexecs.begin(); it != ctx->gexecs.end();) {
      if (std::find(keys.begin(), keys.end(), it->first) == keys.end()) {
        (void)hipGraphExecDestroy(it->second);
        it = ctx->gexecs.erase(it);
      } else {
        ++it;
      }
    }
    for (int c = 0; c < nk; ++c) {
      auto it = ctx->gexecs.find(keys[c]);
      if (it != ctx->gexecs.end()) {
        gx[c] = it->second;
        continue;
      }
      hipGraph_t g = nullptr;
      HIPCHK(hipStreamBeginCapture(ctx->cs, hipStreamCaptureModeRelaxed));
      int brc = WF_OK;
      int64_t saved[KK_COUNT];
      std::memcpy(saved, ctx->launches, sizeof saved);
      for (int r = 0; r < K && brc == WF_OK; ++r) brc = body(ks[c]);
      std::memcpy(ctx->launches, saved, sizeof saved);
      hipError_t e = hipStreamEndCapture(ctx->cs, &g);
      if (brc) return brc;
      if (e != hipSuccess) return fail(ctx, WF_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
      e = hipGraphInstantiate(&gx[c], g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return fail(ctx, WF_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
      ctx->gexecs[keys[c]] = gx[c];
    }
    // concurrent streams for the classes of an uneven batch (default priority)
    const int nx = std::min(nk, kMaxStreams) - 1;
    if (!ctx->evFork && nx > 0) HIPCHK(hipEventCreateWithFlags(&ctx->evFork, hipEventDisableTiming));
    while ((int)ctx->xs.size() < nx) {
      hipStream_t x = nullptr;
      hipEvent_t ev = nullptr;
      HIPCHK(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
      ctx->xs.push_back(x);
      HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      ctx->xev.push_back(ev);
    }
  }
  // Host-polled iterations until every instance of the classes with nrun[c] > 0 has stopped.
  // One iteration takes at most four bodies (curvature product, flush of w, exact gradient,
  // dots after a failed confirmation), so the device's own max_iter test, which flushes w
  // before it stops, always comes first.
  auto run_loop = [&](std::vector<int64_t> nrun) -> int {
    const int64_t maxBodies = 4LL * o.max_iter + 64;
    int64_t bodies = 0;
    while (true) {
      if (graph) {
        // classes with running instances, heaviest first (running instances x vector length),
        // each onto the stream with the least load so far: the long classes of an uneven batch
        // get streams of their own
        std::vector<int> act;
        for (int c = 0; c < nk; ++c)
          if (nrun[c] > 0) act.push_back(c);
        std::stable_sort(act.begin(), act.end(),
                         [&](int x, int y) { return nrun[x] * ks[x].L > nrun[y] * ks[y].L; });
        const int ns = std::min((int)act.size(), kMaxStreams);
        std::vector<int64_t> sload(ns, 0);
        if (ns > 1) HIPCHK(hipEventRecord(ctx->evFork, ctx->cs));
        for (int s = 1; s < ns; ++s) HIPCHK(hipStreamWaitEvent(ctx->xs[s - 1], ctx->evFork, 0));
        for (size_t a = 0; a < act.size(); ++a) {
          const int s = (int)(std::min_element(sload.begin(), sload.end()) - sload.begin());
          sload[s] += nrun[act[a]] * ks[act[a]].L;
          HIPCHK(hipGraphLaunch(gx[act[a]], s == 0 ? ctx->cs : ctx->xs[s - 1]));
          // count launches as if enqueued one by one
          ctx->launches[KK_COLINV] += K;
          ctx->launches[KK_ROW] += ks[act[a]].cat ? 2 * K : K;
          ctx->launches[KK_COLFWD] += K;
          if (ks[act[a]].cat) ctx->launches[KK_CAT] += 4 * K;
          ctx->launches[KK_POST] += K;
          if (!cg) ctx->launches[KK_PASSA] += K;
          ctx->launches[KK_COEF] += K;
          ctx->launches[KK_PASSB] += K;
          if (cg) ctx->launches[KK_DIR] += K;
        }
        for (int s = 1; s < ns; ++s) {
          HIPCHK(hipEventRecord(ctx->xev[s - 1], ctx->xs[s - 1]));
          HIPCHK(hipStreamWaitEvent(ctx->cs, ctx->xev[s - 1], 0));
        }
      } else {
        for (int r = 0; r < K; ++r)
          for (int c = 0; c < nk; ++c) {
            if (nrun[c] == 0) continue;
            int brc = body(ks[c]);
            if (brc) return brc;
          }
      }
      bodies += K;
      HIPCHK(hipMemcpyAsync(ctx->hstat, dstat, sizeof(int) * B, hipMemcpyDeviceToHost, ctx->cs));
      HIPCHK(hipStreamSynchronize(ctx->cs));
      int drc = drain_events(ctx);
      if (drc) return drc;
      int64_t running = 0;
      for (int c = 0; c < nk; ++c) {
        if (nrun[c] == 0) continue;
        int64_t r = 0;
        for (size_t j = 0; j < ks[c].members.size(); ++j) r += (ctx->hstat[ks[c].first + (int)j] == ST_RUNNING);
        nrun[c] = r;
        running += r;
      }
      if (running == 0 || bodies >= maxBodies) break;
    }
    return WF_OK;
  };
  {
    std::vector<int64_t> nrun(nk);
    for (int c = 0; c < nk; ++c) nrun[c] = (int64_t)ks[c].members.size();
    rc = run_loop(nrun);
    if (rc) return rc;
  }
  std::vector<StateStat> hs(B);
  HIPCHK(state_stats_launch(dst, dss, B, ctx->cs));
  HIPCHK(hipMemcpyAsync(hs.data(), dss, sizeof(StateStat) * B, hipMemcpyDeviceToHost, ctx->cs));
  HIPCHK(hipStreamSynchronize(ctx->cs));
  for (int gi = 0; gi < B; ++gi) {
    if (hs[gi].status == ST_RUNNING) hs[gi].status = WF_SOLVE_MAXITER;
    for (int k = 0; k < KK_COUNT; ++k) ctx->bytes[k] += hs[gi].bytes[k];
  }
  if (o.refine > 0) {
    rc = refine_f64(ctx, o, ks, hd, ddesc, dst, dss, hs, init_class, run_loop);
    if (rc) return rc;
  }
  out.st.resize(B);
  for (int ui = 0; ui < B; ++ui) out.st[ui] = hs[out.order[ui]];
  return WF_OK;
}

void fill_stats(const SolveOut& so, int B, wf_solve_stats* stats) {
  if (!stats) return;
  for (int i = 0; i < B; ++i) {
    const StateStat& S = so.st[i];
    stats[i].iters = S.iter;
    stats[i].status = S.status;
    stats[i].ngrad = S.ngrad;
    stats[i].reserved = 0;
    stats[i].chi2 = S.chi2;
    stats[i].rel_grad = S.g0norm > 0 ? std::sqrt(S.gg) / S.g0norm : 0.0;
  }
}

// forward map of solved fields into caller buffers (mode CM_FWD on the whitened w)
// s = sqrt(S) w with partners filled, into the caller's buffers: one launch per class of
// equal (n, ncomp, dtype), from a device table of per-instance pointers
int pack_solutions(wf_ctx* ctx, const wf_problem* probs, int B, const SolveOut& so, void* const* s_out) {
  std::map<std::tuple<int, int, int>, std::vector<int>> cls;
  for (int i = 0; i < B; ++i) cls[std::make_tuple(probs[i].n, probs[i].ncomp, probs[i].dtype)].push_back(i);
  std::vector<PackEntry> tab;
  tab.reserve(B);
  for (auto& kv : cls)
    for (int i : kv.second) tab.push_back(PackEntry{so.w[i], so.prior[i].sq, s_out[i]});
  int rc = arena_reserve(ctx, ctx->opA, align_up(sizeof(PackEntry) * tab.size()));
  if (rc) return rc;
  PackEntry* dt = (PackEntry*)arena_take(ctx->opA, sizeof(PackEntry) * tab.size());
  HIPCHK(hipMemcpyAsync(dt, tab.data(), sizeof(PackEntry) * tab.size(), hipMemcpyHostToDevice, ctx->cs));
  size_t off = 0;
  for (auto& kv : cls) {
    const int cnt = (int)kv.second.size();
    HIPCHK(pack_tab_launch(std::get<2>(kv.first), std::get<0>(kv.first), std::get<1>(kv.first), cnt, dt + off,
                           ctx->cs));
    off += (size_t)cnt;
  }
  // the table is reused by the next call on this arena
  HIPCHK(hipStreamSynchronize(ctx->cs));
  return WF_OK;
}

int maps_from_solution(wf_ctx* ctx, const wf_problem* probs, int B, const SolveOut& so, void* const* map_out) {
  if (!map_out) return WF_OK;
  std::map<std::tuple<int, int, int>, std::vector<int>> cls;
  for (int i = 0; i < B; ++i)
    if (map_out[i]) cls[std::make_tuple(probs[i].n, probs[i].ncomp, probs[i].dtype)].push_back(i);
  for (auto& kv : cls) {
    const int n = std::get<0>(kv.first), c = std::get<1>(kv.first), dt = std::get<2>(kv.first);
    const auto& mem = kv.second;
    std::vector<Job> hj(mem.size());
    for (size_t j = 0; j < mem.size(); ++j) {
      Job& jb = hj[j];
      std::memset(&jb, 0, sizeof jb);
      jb.mode = CM_FWD;
      jb.boost_band = -1;
      jb.vin = so.w[mem[j]];
      jb.y = so.y[mem[j]];
      jb.sIn = so.prior[mem[j]].sq;
      jb.xout = map_out[mem[j]];
    }
    int rc = arena_reserve(ctx, ctx->opA, align_up(sizeof(Job) * mem.size()));
    if (rc) return rc;
    Job* dj = (Job*)arena_take(ctx->opA, sizeof(Job) * mem.size());
    HIPCHK(hipMemcpyAsync(dj, hj.data(), sizeof(Job) * mem.size(), hipMemcpyHostToDevice, ctx->cs));
    const void* tw = nullptr;
    rc = twiddles(ctx, n, dt, &tw);
    if (rc) return rc;
    HIPCHK(chain(ctx, dt, n, c, CH_COLINV, dj, (int)mem.size(), tw));
    HIPCHK(chain(ctx, dt, n, c, CH_ROW, dj, (int)mem.size(), tw));
    HIPCHK(hipStreamSynchronize(ctx->cs));   // the job array is reused by the next group
  }
  return WF_OK;
}

// ---------------------------------------------------------------------------- small dense solve
// Gaussian elimination with partial pivoting, float64 (A is n x n row-major, overwritten).
bool dense_solve(std::vector<double> A, std::vector<double>& x, int n) {
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int r = k + 1; r < n; ++r)
      if (std::fabs(A[(size_t)r * n + k]) > std::fabs(A[(size_t)piv * n + k])) piv = r;
    if (!(std::fabs(A[(size_t)piv * n + k]) > 0)) return false;
    if (piv != k) {
      for (int cc = 0; cc < n; ++cc) std::swap(A[(size_t)k * n + cc], A[(size_t)piv * n + cc]);
      std::swap(x[k], x[piv]);
    }
    for (int r = k + 1; r < n; ++r) {
      const double f = A[(size_t)r * n + k] / A[(size_t)k * n + k];
      for (int cc = k; cc < n; ++cc) A[(size_t)r * n + cc] -= f * A[(size_t)k * n + cc];
      x[r] -= f * x[k];
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    double s = x[k];
    for (int cc = k + 1; cc < n; ++cc) s -= A[(size_t)k * n + cc] * x[cc];
    x[k] = s / A[(size_t)k * n + k];
  }
  return true;
}

// ---------------------------------------------------------------------------- band powers
// E of the solved (whitened) fields, HOST [B][nbands]
int band_E_solved(wf_ctx* ctx, const wf_problem* probs, int B, const SolveOut& so, std::vector<double>& E) {
  const int nb = probs[0].nbands;
  E.assign((size_t)B * nb, 0.0);
  if (nb == 0 || B == 0) return WF_OK;
  const int64_t L = (int64_t)probs[0].ncomp * probs[0].n * (probs[0].n / 2);
  const int nblk = band_nblk(L);
  const size_t need = align_up(sizeof(BandJob) * B) + align_up(sizeof(double) * (size_t)B * nblk * nb) +
                      align_up(sizeof(double) * (size_t)B * nb);
  int rc = arena_reserve(ctx, ctx->opA, need);
  if (rc) return rc;
  BandJob* dj = (BandJob*)arena_take(ctx->opA, sizeof(BandJob) * B);
  double* part = (double*)arena_take(ctx->opA, sizeof(double) * (size_t)B * nblk * nb);
  double* dE = (double*)arena_take(ctx->opA, sizeof(double) * (size_t)B * nb);
  std::vector<BandJob> hj(B);
  for (int i = 0; i < B; ++i) {
    hj[i].f = so.w[i];
    hj[i].sq = so.prior[i].sq;
    hj[i].aw = so.prior[i].a;
    hj[i].bandI = so.prior[i].bandI;
    hj[i].theta = so.prior[i].theta;
    hj[i].part = part + (size_t)i * nblk * nb;
    hj[i].E = dE + (size_t)i * nb;
    hj[i].L = L;
    hj[i].nbands = nb;
    hj[i].raw = 0;
  }
  HIPCHK(hipMemcpyAsync(dj, hj.data(), sizeof(BandJob) * B, hipMemcpyHostToDevice, ctx->cs));
  {
    Timed t(ctx, KK_MISC);
    HIPCHK(band_launch(probs[0].dtype, dj, B, L, ctx->cs));
  }
  HIPCHK(hipMemcpyAsync(E.data(), dE, sizeof(double) * (size_t)B * nb, hipMemcpyDeviceToHost, ctx->cs));
  HIPCHK(hipStreamSynchronize(ctx->cs));
  return WF_OK;
}

struct SimEntry {
  int kind;   // 0 data, 1 fiducial simulation, 2 boosted simulation
  int sim;
  int band;
  int col;    // boosted simulations: index of `band` in the list of simulated columns
};

// Simulate the data of a list of simulation entries into dbuf (d of entry j at dbuf + j * c n^2).
// `draws` (nullable) holds the normals of simulation simBase at its start.
int simulate_entries(wf_ctx* ctx, const wf_problem* p, const std::vector<SimEntry>& ents, uint64_t seed,
                     const void* draws, int simBase, const PriorTab& ptrue, void* dbuf, void* ybuf,
                     double boost_factor) {
  const int n = p->n, c = p->ncomp, dt = p->dtype;
  const size_t rs = rsize_of(dt), eb = esize_of(dt);
  const int64_t L = (int64_t)c * n * (n / 2);
  const int64_t npix = (int64_t)c * n * n;
  std::vector<Job> hj;
  std::vector<int> slot;
  for (size_t j = 0; j < ents.size(); ++j) {
    if (ents[j].kind == 0) continue;
    Job jb;
    std::memset(&jb, 0, sizeof jb);
    jb.mode = CM_SIM;
    jb.boost_band = ents[j].kind == 2 ? ents[j].band : -1;
    jb.boost_factor = std::sqrt(boost_factor);
    jb.sim = ents[j].sim;
    jb.seed = seed;
    jb.y = (char*)ybuf + (size_t)hj.size() * L * eb;
    jb.W = p->w;
    jb.sIn = ptrue.sq;
    jb.band = ptrue.bandI;
    jb.draws = draws ? (const char*)draws + (size_t)(ents[j].sim - simBase) * 2 * npix * rs : nullptr;
    jb.xout = (char*)dbuf + j * npix * rs;
    hj.push_back(jb);
  }
  if (hj.empty()) return WF_OK;
  Job* dj = (Job*)arena_take(ctx->simA, sizeof(Job) * hj.size());
  HIPCHK(hipMemcpyAsync(dj, hj.data(), sizeof(Job) * hj.size(), hipMemcpyHostToDevice, ctx->cs));
  const void* tw = nullptr;
  int rc = twiddles(ctx, n, dt, &tw);
  if (rc) return rc;
  rc = prepare(ctx, n, c, dt);
  if (rc) return rc;
  ChainCfg scfg;
  scfg.sim = 1;
  HIPCHK(chain(ctx, dt, n, c, CH_COLINV, dj, (int)hj.size(), tw, &scfg));
  HIPCHK(chain(ctx, dt, n, c, CH_ROW, dj, (int)hj.size(), tw, &scfg));
  return WF_OK;
}

// The quadratic estimator's solves (sec. 2.3-2.4): optional data map, nsim fiducial
// simulations and nsim * nbands boosted ones, in chunks of one batched solve each.
// The solves of one band-power estimate: the data map (with_data), nsim fiducial
// simulations and, per simulation, one with each band of `cols` boosted.  E0 [nsim][nb],
// E2 [nsim][cols.size()][nb].
// theta_sim: nullable amplitudes the simulations are drawn with (the solves always use
// p->theta)
int run_qe(wf_ctx* ctx, const wf_problem* p, bool with_data, int nsim, uint64_t seed, const void* draws,
           const wf_lbfgs_opts& o, const std::vector<int>& cols, std::vector<double>& Edata, std::vector<double>& E0,
           std::vector<double>& E2, int& notConverged, const double* theta_sim = nullptr) {
  const int nb = p->nbands;
  const int nc = (int)cols.size();
  const int n = p->n, c = p->ncomp, dt = p->dtype;
  std::vector<SimEntry> all;
  if (with_data) all.push_back({0, 0, -1, -1});
  for (int i = 0; i < nsim; ++i) {
    all.push_back({1, i, -1, -1});
    for (int j = 0; j < nc; ++j) all.push_back({2, i, cols[j], j});
  }
  Edata.assign(nb, 0.0);
  E0.assign((size_t)nsim * nb, 0.0);
  E2.assign((size_t)nsim * nc * nb, 0.0);
  notConverged = 0;
  const size_t rs = rsize_of(dt), eb = esize_of(dt);
  const int64_t L = (int64_t)c * n * (n / 2);
  const int64_t npix = (int64_t)c * n * n;
  const double perInst = (double)(3 + 2 * o.m) * L * eb + (double)npix * rs + (double)L * eb;
  int chunk = (int)std::max(1.0, std::min((double)kMaxChunk, kSimBudgetBytes / perInst));
  for (size_t off = 0; off < all.size(); off += chunk) {
    const size_t cnt = std::min(all.size() - off, (size_t)chunk);
    std::vector<SimEntry> ents(all.begin() + off, all.begin() + off + cnt);
    const size_t need = prior_bytes(p) + align_up(sizeof(Job) * cnt) + align_up((size_t)npix * rs * cnt) +
                        align_up((size_t)L * eb * cnt);
    int rc = arena_reserve(ctx, ctx->simA, need);
    if (rc) return rc;
    PriorTab ptrue;
    rc = build_prior(ctx, ctx->simA, p, theta_sim ? theta_sim : p->theta, ptrue);
    if (rc) return rc;
    void* dbuf = arena_take(ctx->simA, (size_t)npix * rs * cnt);
    void* ybuf = arena_take(ctx->simA, (size_t)L * eb * cnt);
    rc = simulate_entries(ctx, p, ents, seed, draws, 0, ptrue, dbuf, ybuf, 2.0);
    if (rc) return rc;
    std::vector<wf_problem> probs(cnt, *p);
    for (size_t j = 0; j < cnt; ++j)
      if (ents[j].kind != 0) probs[j].d = (const char*)dbuf + j * npix * rs;
    SolveOut so;
    rc = solve_core(ctx, probs.data(), (int)cnt, o, so);
    if (rc) return rc;
    for (size_t j = 0; j < cnt; ++j) notConverged += so.st[j].status != WF_SOLVE_CONVERGED;
    std::vector<double> E;
    rc = band_E_solved(ctx, probs.data(), (int)cnt, so, E);
    if (rc) return rc;
    for (size_t j = 0; j < cnt; ++j) {
      const double* e = &E[j * nb];
      if (ents[j].kind == 0)
        std::copy(e, e + nb, Edata.begin());
      else if (ents[j].kind == 1)
        std::copy(e, e + nb, E0.begin() + (size_t)ents[j].sim * nb);
      else
        for (int l = 0; l < nb; ++l) E2[((size_t)ents[j].sim * nc + ents[j].col) * nb + l] = e[l];
    }
  }
  return WF_OK;
}

// The solves of the band-power estimates of several maps (all Fisher columns simulated),
// shared among batched solves: per map the data map, nsim fiducial simulations and nsim *
// nbands boosted ones, the maps ordered by size (largest first), cut into chunks of at most
// kMaxChunkMulti solves and kMultiBudgetBytes of workspace; each chunk is one batched
// (uneven) solve whose classes of equal shape run independently.  Map i's simulations use
// the Philox key seed + i.  Edata[i] [nb_i], E0[i] [nsim][nb_i],
// E2[i] [nsim][nb_i][nb_i]; notConverged counts solves that did not converge.
int run_qe_multi(wf_ctx* ctx, const wf_problem* probs, int np, int nsim, uint64_t seed, const wf_lbfgs_opts& o,
                 std::vector<std::vector<double>>& Edata, std::vector<std::vector<double>>& E0,
                 std::vector<std::vector<double>>& E2, int& notConverged) {
  struct MEnt {
    int prob;
    SimEntry e;
  };
  std::vector<MEnt> all;
  Edata.assign(np, {});
  E0.assign(np, {});
  E2.assign(np, {});
  std::vector<int> order(np);
  for (int i = 0; i < np; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return (int64_t)probs[a].ncomp * probs[a].n * probs[a].n > (int64_t)probs[b].ncomp * probs[b].n * probs[b].n;
  });
  for (int i : order) {
    const int nb = probs[i].nbands;
    Edata[i].assign(nb, 0.0);
    E0[i].assign((size_t)nsim * nb, 0.0);
    E2[i].assign((size_t)nsim * nb * nb, 0.0);
    all.push_back({i, {0, 0, -1, -1}});
    for (int s = 0; s < nsim; ++s) {
      all.push_back({i, {1, s, -1, -1}});
      for (int l = 0; l < nb; ++l) all.push_back({i, {2, s, l, l}});
    }
  }
  notConverged = 0;
  auto shape = [&](int i, int64_t& L, int64_t& npix, size_t& rs, size_t& eb) {
    const wf_problem& p = probs[i];
    L = (int64_t)p.ncomp * p.n * (p.n / 2);
    npix = (int64_t)p.ncomp * p.n * p.n;
    rs = rsize_of(p.dtype);
    eb = esize_of(p.dtype);
  };
  size_t off = 0;
  while (off < all.size()) {
    // the chunk: as many entries as the instance and workspace caps allow
    size_t cnt = 0;
    double bytes = 0.0;
    while (off + cnt < all.size() && cnt < (size_t)kMaxChunkMulti) {
      int64_t L, npix;
      size_t rs, eb;
      shape(all[off + cnt].prob, L, npix, rs, eb);
      const double per = (double)(3 + 2 * o.m) * L * eb + (double)npix * rs + (double)L * eb;
      if (cnt > 0 && bytes + per > kMultiBudgetBytes) break;
      bytes += per;
      ++cnt;
    }
    // workspace of the simulations: prior tables of each map in the chunk, jobs, data, intermediates
    size_t need = 0;
    for (size_t j = 0; j < cnt;) {
      const int pi = all[off + j].prob;
      size_t e = j;
      while (e < cnt && all[off + e].prob == pi) ++e;
      int64_t L, npix;
      size_t rs, eb;
      shape(pi, L, npix, rs, eb);
      need += prior_bytes(&probs[pi]) + align_up(sizeof(Job) * (e - j)) + align_up((size_t)npix * rs * (e - j)) +
              align_up((size_t)L * eb * (e - j));
      j = e;
    }
    int rc = arena_reserve(ctx, ctx->simA, need);
    if (rc) return rc;
    std::vector<wf_problem> cp(cnt);
    for (size_t j = 0; j < cnt;) {
      const int pi = all[off + j].prob;
      size_t e = j;
      while (e < cnt && all[off + e].prob == pi) ++e;
      int64_t L, npix;
      size_t rs, eb;
      shape(pi, L, npix, rs, eb);
      PriorTab ptrue;
      rc = build_prior(ctx, ctx->simA, &probs[pi], probs[pi].theta, ptrue);
      if (rc) return rc;
      void* dbuf = arena_take(ctx->simA, (size_t)npix * rs * (e - j));
      void* ybuf = arena_take(ctx->simA, (size_t)L * eb * (e - j));
      std::vector<SimEntry> ents;
      for (size_t q = j; q < e; ++q) ents.push_back(all[off + q].e);
      rc = simulate_entries(ctx, &probs[pi], ents, seed + (uint64_t)pi, nullptr, 0, ptrue, dbuf, ybuf, 2.0);
      if (rc) return rc;
      for (size_t q = j; q < e; ++q) {
        cp[q] = probs[pi];
        if (all[off + q].e.kind != 0) cp[q].d = (const char*)dbuf + (q - j) * npix * rs;
      }
      j = e;
    }
    SolveOut so;
    rc = solve_core(ctx, cp.data(), (int)cnt, o, so);
    if (rc) return rc;
    for (size_t j = 0; j < cnt; ++j) notConverged += so.st[j].status != WF_SOLVE_CONVERGED;
    // band statistics map by map (band_E_solved takes one shape)
    for (size_t j = 0; j < cnt;) {
      const int pi = all[off + j].prob;
      size_t e = j;
      while (e < cnt && all[off + e].prob == pi) ++e;
      SolveOut sub;
      sub.w.assign(so.w.begin() + j, so.w.begin() + e);
      sub.prior.assign(so.prior.begin() + j, so.prior.begin() + e);
      std::vector<double> E;
      rc = band_E_solved(ctx, cp.data() + j, (int)(e - j), sub, E);
      if (rc) return rc;
      const int nb = probs[pi].nbands;
      for (size_t q = j; q < e; ++q) {
        const double* v = &E[(q - j) * nb];
        const SimEntry& en = all[off + q].e;
        if (en.kind == 0)
          std::copy(v, v + nb, Edata[pi].begin());
        else if (en.kind == 1)
          std::copy(v, v + nb, E0[pi].begin() + (size_t)en.sim * nb);
        else
          std::copy(v, v + nb, E2[pi].begin() + ((size_t)en.sim * nb + en.col) * nb);
      }
      j = e;
    }
    off += cnt;
  }
  return WF_OK;
}

// Bias b_l = <E0_l> and the symmetrised Fisher matrix from the simulated columns `cols`
// (F_ll' from the boosted minus fiducial E of column l', eq. fisher with Delta_l' =
// theta_l').  The other columns are interpolated in units of D_l, the variance of E0_l
// over the simulations (an estimate of F_ll for the optimal quadratic estimator): the
// normalised response Fr_ll' / sqrt(D_l D_l') is taken along the diagonals from the
// nearest simulated columns of the same band group (bands with equal consecutive ids in
// grp), the row shift kept inside the row's group; linear in the band index when both
// neighbours' rows exist, else the one that does, and beyond a group's last (first)
// simulated column the one neighbour with the row clamped into the group.
void bias_fisher(const double* theta, int nsim, int nb, const std::vector<int>& cols, const std::vector<int>& grp,
                 const std::vector<double>& E0, const std::vector<double>& E2, double* b, double* F) {
  const int nc = (int)cols.size();
  for (int l = 0; l < nb; ++l) {
    double s = 0.0;
    for (int i = 0; i < nsim; ++i) s += E0[(size_t)i * nb + l];
    b[l] = nsim > 0 ? s / nsim : 0.0;
  }
  std::vector<double> Fr((size_t)nb * nb, 0.0);   // Fr[l][l2]: response of E_l to band l2
  std::vector<char> have(nb, 0);
  for (int j = 0; j < nc; ++j) {
    const int l2 = cols[j];
    have[l2] = 1;
    for (int l = 0; l < nb; ++l) {
      double s = 0.0;
      for (int i = 0; i < nsim; ++i) s += E2[((size_t)i * nc + j) * nb + l] - E0[(size_t)i * nb + l];
      Fr[(size_t)l * nb + l2] = nsim > 0 ? s / nsim / theta[l2] : 0.0;
    }
  }
  // per-band scale: sample variance of E0 (1 if not positive or a single simulation)
  std::vector<double> sq(nb, 1.0);
  if (nsim > 1)
    for (int l = 0; l < nb; ++l) {
      const double m = b[l];
      double v = 0.0;
      for (int i = 0; i < nsim; ++i) {
        const double e = E0[(size_t)i * nb + l] - m;
        v += e * e;
      }
      v /= (nsim - 1);
      sq[l] = v > 0 ? std::sqrt(v) : 1.0;
    }
  auto rn = [&](int l, int l2) { return Fr[(size_t)l * nb + l2] / (sq[l] * sq[l2]); };
  // group extents [lo, hi) of every band
  std::vector<int> lo(nb), hi(nb);
  for (int l = 0; l < nb;) {
    int e = l + 1;
    while (e < nb && grp[e] == grp[l]) ++e;
    for (int k = l; k < e; ++k) {
      lo[k] = l;
      hi[k] = e;
    }
    l = e;
  }
  for (int l2 = 0; l2 < nb; ++l2) {
    if (have[l2]) continue;
    int a = -1, bb = -1;
    for (int k = lo[l2]; k < l2; ++k)
      if (have[k]) a = k;
    for (int k = hi[l2] - 1; k > l2; --k)
      if (have[k]) bb = k;
    for (int l = 0; l < nb; ++l) {
      const int ra = l + (a - l2), rb = l + (bb - l2);
      const bool okA = a >= 0 && ra >= lo[l] && ra < hi[l];
      const bool okB = bb >= 0 && rb >= lo[l] && rb < hi[l];
      double v;
      if (okA && okB) {
        const double va = rn(ra, a), vb = rn(rb, bb);
        v = va + (vb - va) * (double)(l2 - a) / (double)(bb - a);
      } else if (okA) {
        v = rn(ra, a);
      } else if (okB) {
        v = rn(rb, bb);
      } else {
        const int sc = a >= 0 ? a : bb;
        v = rn(std::min(std::max(l + (sc - l2), lo[l]), hi[l] - 1), sc);
      }
      Fr[(size_t)l * nb + l2] = sq[l] * sq[l2] * v;
    }
  }
  for (int l = 0; l < nb; ++l)
    for (int l2 = 0; l2 < nb; ++l2) F[(size_t)l * nb + l2] = 0.5 * (Fr[(size_t)l * nb + l2] + Fr[(size_t)l2 * nb + l]);
}

// Monte Carlo variance of the Fisher estimate with every column simulated: per entry, the
// sample variance over the simulations of each one's symmetrised estimate
// (Fr_i,ll' + Fr_i,l'l) / 2 with Fr_i,ll' = (E2_i,l(l') - E0_i,l) / theta_l', divided by nsim
// (the variance of the mean; 0 with one simulation).
void fisher_variance(const double* theta, int nsim, int nb, const std::vector<double>& E0,
                     const std::vector<double>& E2, double* Fv) {
  for (int l = 0; l < nb; ++l)
    for (int l2 = 0; l2 < nb; ++l2) {
      if (nsim < 2) {
        Fv[(size_t)l * nb + l2] = 0.0;
        continue;
      }
      auto est = [&](int i) {
        const double a = (E2[((size_t)i * nb + l2) * nb + l] - E0[(size_t)i * nb + l]) / theta[l2];
        const double c = (E2[((size_t)i * nb + l) * nb + l2] - E0[(size_t)i * nb + l2]) / theta[l];
        return 0.5 * (a + c);
      };
      double m = 0.0;
      for (int i = 0; i < nsim; ++i) m += est(i);
      m /= nsim;
      double v = 0.0;
      for (int i = 0; i < nsim; ++i) {
        const double e = est(i) - m;
        v += e * e;
      }
      Fv[(size_t)l * nb + l2] = v / (nsim - 1) / nsim;
    }
}

// Newton step Theta_hat = Theta_fid + F^-1 (E - b) (eq. eq:wfmv) on the bands that carry
// information: a band whose Fisher diagonal is not positive or is below kFisherFloor of the
// largest (its E does not respond to its amplitude above the rounding of E, e.g. bands beyond
// a spectrum's cut-off, whose modes have no signal) keeps its fiducial amplitude, and the step
// is solved on the others.  Returns false if that system is singular.
constexpr double kFisherFloor = 1e-9;
bool newton_step(const double* theta, const std::vector<double>& F, const std::vector<double>& E,
                 const std::vector<double>& b, int nb, double* out) {
  double fmax = 0.0;
  for (int l = 0; l < nb; ++l) fmax = std::max(fmax, F[(size_t)l * nb + l]);
  std::vector<int> use;
  for (int l = 0; l < nb; ++l)
    if (F[(size_t)l * nb + l] > kFisherFloor * fmax) use.push_back(l);
  for (int l = 0; l < nb; ++l) out[l] = theta[l];
  const int k = (int)use.size();
  if (k == 0) return nb == 0;
  std::vector<double> A((size_t)k * k), x(k);
  for (int i = 0; i < k; ++i) {
    x[i] = E[use[i]] - b[use[i]];
    for (int j = 0; j < k; ++j) A[(size_t)i * k + j] = F[(size_t)use[i] * nb + use[j]];
  }
  if (!dense_solve(A, x, k)) return false;
  for (int i = 0; i < k; ++i) out[use[i]] = theta[use[i]] + x[i];
  return true;
}

// Simulated columns and band groups of a sampled-Fisher call: rows strictly increasing in
// [0, nb), groups nullable (one group) or [nb] ids, every group with a simulated column.
int parse_rows(wf_ctx* ctx, int nb, const int32_t* rows, int32_t nrows, const int32_t* groups, std::vector<int>& cols,
               std::vector<int>& grp) {
  cols.clear();
  grp.assign(nb, 0);
  if (!rows) {
    for (int l = 0; l < nb; ++l) cols.push_back(l);
  } else {
    if (nrows < 1 || nrows > nb) return fail(ctx, WF_EINVAL, "need 1 <= nrows <= nbands");
    for (int j = 0; j < nrows; ++j) {
      if (rows[j] < 0 || rows[j] >= nb || (j > 0 && rows[j] <= rows[j - 1]))
        return fail(ctx, WF_EINVAL, "rows must be strictly increasing band indices");
      cols.push_back(rows[j]);
    }
  }
  if (groups)
    for (int l = 0; l < nb; ++l) grp[l] = groups[l];
  for (int l = 0; l < nb;) {
    int e = l + 1;
    while (e < nb && grp[e] == grp[l]) ++e;
    bool any = false;
    for (int c : cols) any = any || (c >= l && c < e);
    if (!any) return fail(ctx, WF_EINVAL, "every band group needs a simulated row");
    l = e;
  }
  return WF_OK;
}

// One quadratic band-power estimate around p->theta (MAP of the data, E, b, F, Newton step);
// with_data = false: b and F only.
int qe_estimate(wf_ctx* ctx, const wf_problem* p, bool with_data, int nsim, uint64_t seed, const void* draws,
                const wf_lbfgs_opts& o, const std::vector<int>& cols, const std::vector<int>& grp, double* theta_hat,
                std::vector<double>& E, std::vector<double>& hb, std::vector<double>& hF, std::vector<double>& E0,
                int& nc) {
  const int nb = p->nbands;
  std::vector<double> E2;
  int rc = run_qe(ctx, p, with_data, nsim, seed, draws, o, cols, E, E0, E2, nc);
  if (rc) return rc;
  hb.assign(nb, 0.0);
  hF.assign((size_t)nb * nb, 0.0);
  bias_fisher(p->theta, nsim, nb, cols, grp, E0, E2, hb.data(), hF.data());
  if (!with_data) return WF_OK;
  if (!newton_step(p->theta, hF, E, hb, nb, theta_hat)) return fail(ctx, WF_ENONFINITE, "singular Fisher matrix");
  return WF_OK;
}

// ---------------------------------------------------------------------------- operator jobs
int op_setup(wf_ctx* ctx, const wf_problem* p, int batch, size_t extra, PriorTab* pt, void** vin, void** vy,
             void** vout, Job** dj, double** part, const void** tw) {
  const int n = p->n, c = p->ncomp, dt = p->dtype;
  const int64_t L = (int64_t)c * n * (n / 2);
  const size_t eb = esize_of(dt);
  const int pstride = c * n / RB_MIN;
  const size_t need = prior_bytes(p) + 3 * align_up((size_t)L * eb * batch) + align_up(sizeof(Job) * batch) +
                      align_up(sizeof(double) * PK_COUNT * pstride * batch) + extra;
  int rc = arena_reserve(ctx, ctx->opA, need);
  if (rc) return rc;
  if (pt) {
    rc = build_prior(ctx, ctx->opA, p, p->theta, *pt);
    if (rc) return rc;
  } else {
    arena_take(ctx->opA, prior_bytes(p));
  }
  *vin = arena_take(ctx->opA, (size_t)L * eb * batch);
  *vy = arena_take(ctx->opA, (size_t)L * eb * batch);
  *vout = arena_take(ctx->opA, (size_t)L * eb * batch);
  *dj = (Job*)arena_take(ctx->opA, sizeof(Job) * batch);
  *part = (double*)arena_take(ctx->opA, sizeof(double) * PK_COUNT * pstride * batch);
  rc = twiddles(ctx, n, dt, tw);
  if (rc) return rc;
  return prepare(ctx, n, c, dt);
}

int check_op(wf_ctx* ctx, const wf_problem* p, int batch, const void* a, const void* b) {
  if (!ctx) return WF_EINVAL;
  if (!p) return fail(ctx, WF_EINVAL, "null problem");
  if (!chain_supported(p->n)) return fail(ctx, WF_EINVAL, "unsupported n=" + std::to_string(p->n));
  if (p->ncomp != 1 && p->ncomp != 2) return fail(ctx, WF_EINVAL, "ncomp must be 1 or 2");
  if (p->dtype != WF_F32 && p->dtype != WF_F64) return fail(ctx, WF_EINVAL, "bad dtype");
  if (batch < 0 || batch > 65535) return fail(ctx, WF_EINVAL, "batch out of range");
  if (batch > 0 && (!a || !b)) return fail(ctx, WF_EINVAL, "null array");
  return WF_OK;
}

// One catalog's response operator: forward (s -> values at the galaxies, CM_FWD) or adjoint
// (residuals -> field, CM_ADJ / CM_ADJ_GRAD), unscaled, on the fine grid.
int cat_operator(wf_ctx* ctx, const wf_problem* p, const wf_catalog* cat, const void* in, void* out, int mode,
                 void* stream) {
  if (!ctx) return WF_EINVAL;
  int rc = check_catalog(ctx, p, cat, false);
  if (rc) return rc;
  if (!in || !out) return fail(ctx, WF_EINVAL, "null array");
  StreamScope ss(ctx, stream);
  const int n = p->n, c = p->ncomp, N = 2 * n;
  CatPlan h;
  cat_plan(cat, n, c, h);
  size_t sortBytes = 0;
  rc = cat_sort_bytes(ctx, N, h.ngal, sortBytes);
  if (rc) return rc;
  const int64_t L = (int64_t)c * n * (n / 2);
  rc = arena_reserve(ctx, ctx->opA, cat_bytes(n, c, h.ngal, sortBytes) + align_up((size_t)L * 8) +
                                        align_up(3 * sizeof(Job)) + align_up(sizeof(CatDesc)));
  if (rc) return rc;
  Job* dj = (Job*)arena_take(ctx->opA, 3 * sizeof(Job));   // coarse job, fine forward, fine adjoint
  CatDesc* dc = (CatDesc*)arena_take(ctx->opA, sizeof(CatDesc));
  void* vc = arena_take(ctx->opA, (size_t)L * 8);
  const void* twN = nullptr;
  rc = twiddles(ctx, N, WF_F32, &twN);
  if (rc) return rc;
  rc = prepare(ctx, N, c, WF_F32);
  if (rc) return rc;
  CatDesc hc;
  Job hj[3];
  rc = cat_fill(ctx, ctx->opA, h, sortBytes, nullptr, false, hc, hj[1], hj[2]);
  if (rc) return rc;
  hc.jfwd = dj + 1;
  hc.jadj = dj + 2;
  std::memset(&hj[0], 0, sizeof(Job));
  hj[0].mode = mode;
  hj[0].boost_band = -1;
  if (mode == CM_FWD) {
    HIPCHK(unpack_launch(WF_F32, n, c, 1, in, vc, ctx->cs));
    hj[0].vin = vc;
    hj[1].mode = CM_FWD;
  } else {
    HIPCHK(cat_permute_launch((const float*)in, (const int*)h.perm, hc.r, h.ngal, c, 1, 1, ctx->cs));
    hj[0].vout = vc;
    hj[2].mode = CM_ADJ;
  }
  HIPCHK(hipMemcpyAsync(dc, &hc, sizeof hc, hipMemcpyHostToDevice, ctx->cs));
  HIPCHK(hipMemcpyAsync(dj, hj, sizeof hj, hipMemcpyHostToDevice, ctx->cs));
  const ChainCfg cfg = op_cfg(ctx, WF_F32, N, c);
  if (mode == CM_FWD) {
    HIPCHK(cat_step(ctx, CAT_PAD, c, N / 4, dj, dc, 1));
    HIPCHK(chain(ctx, WF_F32, N, c, CH_COLINV, dj + 1, 1, twN, &cfg));
    HIPCHK(chain(ctx, WF_F32, N, c, CH_ROW, dj + 1, 1, twN, &cfg));
    HIPCHK(cat_step(ctx, CAT_INTERP, c, (h.ngal + NT - 1) / NT, dj, dc, 1));
    HIPCHK(cat_permute_launch(hc.r, (const int*)h.perm, (float*)out, h.ngal, c, 0, 1, ctx->cs));
  } else {
    HIPCHK(cat_step(ctx, CAT_SPREAD, c, h.tiles * h.tiles, dj, dc, 1));
    HIPCHK(chain(ctx, WF_F32, N, c, CH_ROW, dj + 2, 1, twN, &cfg));
    HIPCHK(chain(ctx, WF_F32, N, c, CH_COLFWD, dj + 2, 1, twN, &cfg));
    HIPCHK(cat_step(ctx, CAT_UNPAD, c, n / 4, dj, dc, 1));
    HIPCHK(pack_launch(WF_F32, n, c, 1, vc, L, nullptr, 0, nullptr, out, ctx->cs));
  }
  HIPCHK(hipStreamSynchronize(ctx->cs));
  return WF_OK;
}

}  // namespace

// ============================================================================ C-ABI
extern "C" {

void wf_lbfgs_default(wf_lbfgs_opts* o) {
  if (!o) return;
  o->m = 10;
  o->max_iter = 20000;
  o->rel_grad_tol = 1e-6;
  o->dchi2_tol = 0.0;
  o->refresh_every = 0;
  o->iters_per_poll = 0;
  o->use_graph = 1;
  o->precond = 0;
  o->method = WF_METHOD_LBFGS;
  o->refine = 0;
  o->refine_tol = 1e-10;
}

int wf_create(wf_ctx** out, int hip_device) {
  if (!out) return WF_EINVAL;
  *out = nullptr;
  wf_ctx* c = new (std::nothrow) wf_ctx();
  if (!c) return WF_ENOMEM;
  c->dev = hip_device;
  if (hipSetDevice(hip_device) != hipSuccess || hipStreamCreateWithFlags(&c->cs, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->evIn, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->evOut, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return WF_EHIP;
  }
  tune_cache_open(c);
  if (noalloc_setup(c) != WF_OK) {
    (void)hipEventDestroy(c->evIn);
    (void)hipEventDestroy(c->evOut);
    (void)hipStreamDestroy(c->cs);
    delete c;
    return WF_EHIP;
  }
  *out = c;
  return WF_OK;
}

void wf_destroy(wf_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->dev);
  if (c->cs) (void)hipStreamSynchronize(c->cs);
  for (auto& kv : c->gexecs) (void)hipGraphExecDestroy(kv.second);
  for (auto x : c->xs) {
    (void)hipStreamSynchronize(x);
    (void)hipStreamDestroy(x);
  }
  for (auto e : c->xev) (void)hipEventDestroy(e);
  if (c->evFork) (void)hipEventDestroy(c->evFork);
  for (auto& kv : c->tw) (void)hipFree(kv.second);
  for (Arena* a : {&c->solveA, &c->simA, &c->opA, &c->accA, &c->refA})
    if (a->base) (void)hipFree(a->base);
  if (c->hstat) (void)hipHostFree(c->hstat);
  for (auto& pe : c->pendingEv) {
    (void)hipEventDestroy(pe.second.first);
    (void)hipEventDestroy(pe.second.second);
  }
  for (auto e : c->evPool) (void)hipEventDestroy(e);
  if (c->evIn) (void)hipEventDestroy(c->evIn);
  if (c->evOut) (void)hipEventDestroy(c->evOut);
  if (c->cs) (void)hipStreamDestroy(c->cs);
  delete c;
}

const char* wf_last_error(const wf_ctx* c) { return c ? c->err.c_str() : "null context"; }

int map_wf_solve(wf_ctx* ctx, const wf_problem* probs, int32_t batch, const wf_lbfgs_opts* opts, void* const* s_out,
                 void* const* map_out, wf_solve_stats* stats, void* stream) {
  if (!ctx) return WF_EINVAL;
  if (batch < 0 || batch > 65535 || (batch > 0 && (!probs || !s_out)))
    return fail(ctx, WF_EINVAL, "bad batch / null arrays");
  if (batch == 0) return WF_OK;
  for (int i = 0; i < batch; ++i)
    if (!s_out[i]) return fail(ctx, WF_EINVAL, "null s_out entry");
  wf_lbfgs_opts o;
  fill_opts(opts, o);
  StreamScope ss(ctx, stream);
  SolveOut so;
  int rc = solve_core(ctx, probs, batch, o, so);
  if (rc) return rc;
  rc = pack_solutions(ctx, probs, batch, so, s_out);
  if (rc) return rc;
  rc = maps_from_solution(ctx, probs, batch, so, map_out);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(ctx->cs));
  fill_stats(so, batch, stats);
  for (int i = 0; i < batch; ++i)
    if (so.st[i].status != WF_SOLVE_CONVERGED) return WF_NOT_CONVERGED;
  return WF_OK;
}

int map_wf_solve_catalog(wf_ctx* ctx, const wf_problem* probs, const wf_catalog* cats, int32_t batch,
                         const wf_lbfgs_opts* opts, void* const* s_out, wf_solve_stats* stats, void* stream) {
  if (!ctx) return WF_EINVAL;
  if (batch < 0 || batch > 65535 || (batch > 0 && (!probs || !cats || !s_out)))
    return fail(ctx, WF_EINVAL, "bad batch / null arrays");
  if (batch == 0) return WF_OK;
  for (int i = 0; i < batch; ++i)
    if (!s_out[i]) return fail(ctx, WF_EINVAL, "null s_out entry");
  wf_lbfgs_opts o;
  fill_opts(opts, o);
  StreamScope ss(ctx, stream);
  SolveOut so;
  int rc = solve_core(ctx, probs, batch, o, so, nullptr, cats);
  if (rc) return rc;
  rc = pack_solutions(ctx, probs, batch, so, s_out);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(ctx->cs));
  fill_stats(so, batch, stats);
  for (int i = 0; i < batch; ++i)
    if (so.st[i].status != WF_SOLVE_CONVERGED) return WF_NOT_CONVERGED;
  return WF_OK;
}

int wf_catalog_forward(wf_ctx* ctx, const wf_problem* prob, const wf_catalog* cat, const void* s, float* gamma,
                       void* stream) {
  return cat_operator(ctx, prob, cat, s, gamma, CM_FWD, stream);
}

int wf_catalog_adjoint(wf_ctx* ctx, const wf_problem* prob, const wf_catalog* cat, const float* r, void* s,
                       int32_t flags, void* stream) {
  if (!ctx) return WF_EINVAL;
  if (flags & ~WF_ADJ_GRAD) return fail(ctx, WF_EINVAL, "bad flags");
  return cat_operator(ctx, prob, cat, r, s, (flags & WF_ADJ_GRAD) ? CM_ADJ_GRAD : CM_ADJ, stream);
}

int wf_simulate(wf_ctx* ctx, const wf_problem* p, int32_t nsim, uint64_t seed, int32_t sim0, const void* draws,
                const double* theta_true, int32_t boost_band, double boost_factor, void* d_out, void* stream) {
  if (!ctx) return WF_EINVAL;
  int rc = check_problem(ctx, p, false);
  if (rc) return rc;
  if (nsim < 0 || nsim > 65535 || (nsim > 0 && !d_out)) return fail(ctx, WF_EINVAL, "bad nsim / null d_out");
  if (!(boost_factor > 0)) return fail(ctx, WF_EINVAL, "boost_factor must be > 0");
  if (nsim == 0) return WF_OK;
  StreamScope ss(ctx, stream);
  const int n = p->n, c = p->ncomp, dt = p->dtype;
  const int64_t L = (int64_t)c * n * (n / 2);
  const size_t eb = esize_of(dt), rs = rsize_of(dt);
  const size_t need = prior_bytes(p) + align_up(sizeof(Job) * nsim) + align_up((size_t)L * eb * nsim);
  rc = arena_reserve(ctx, ctx->simA, need);
  if (rc) return rc;
  PriorTab pt;
  rc = build_prior(ctx, ctx->simA, p, theta_true ? theta_true : p->theta, pt);
  if (rc) return rc;
  void* ybuf = arena_take(ctx->simA, (size_t)L * eb * nsim);
  std::vector<SimEntry> ents;
  for (int i = 0; i < nsim; ++i) ents.push_back({boost_band >= 0 ? 2 : 1, sim0 + i, boost_band});
  rc = simulate_entries(ctx, p, ents, seed, draws, sim0, pt, d_out, ybuf, boost_factor);
  if (rc) return rc;
  return WF_OK;
}

int sim_fisher_rows(wf_ctx* ctx, const wf_problem* p, int32_t nsim, uint64_t seed, const void* draws,
                    const wf_lbfgs_opts* opts, const int32_t* rows, int32_t nrows, const int32_t* groups, double* F,
                    double* b, double* E_sims, void* stream) {
  if (!ctx) return WF_EINVAL;
  int rc = check_problem(ctx, p, false);
  if (rc) return rc;
  if (nsim < 1 || !F || !b) return fail(ctx, WF_EINVAL, "need nsim >= 1 and F, b");
  for (int l = 0; l < p->nbands; ++l)
    if (!(p->theta[l] > 0)) return fail(ctx, WF_EINVAL, "fiducial band amplitudes must be > 0");
  std::vector<int> cols, grp;
  rc = parse_rows(ctx, p->nbands, rows, nrows, groups, cols, grp);
  if (rc) return rc;
  wf_lbfgs_opts o;
  fill_opts(opts, o);
  StreamScope ss(ctx, stream);
  std::vector<double> E, hb, hF, E0;
  int nc = 0;
  rc = qe_estimate(ctx, p, false, nsim, seed, draws, o, cols, grp, nullptr, E, hb, hF, E0, nc);
  if (rc) return rc;
  std::copy(hb.begin(), hb.end(), b);
  std::copy(hF.begin(), hF.end(), F);
  if (E_sims) std::copy(E0.begin(), E0.end(), E_sims);
  return nc ? WF_NOT_CONVERGED : WF_OK;
}

int sim_fisher(wf_ctx* ctx, const wf_problem* p, int32_t nsim, uint64_t seed, const void* draws,
               const wf_lbfgs_opts* opts, double* F, double* b, double* F_var, double* E_sims, void* stream) {
  if (!ctx) return WF_EINVAL;
  int rc = check_problem(ctx, p, false);
  if (rc) return rc;
  if (nsim < 1 || !F || !b) return fail(ctx, WF_EINVAL, "need nsim >= 1 and F, b");
  const int nb = p->nbands;
  for (int l = 0; l < nb; ++l)
    if (!(p->theta[l] > 0)) return fail(ctx, WF_EINVAL, "fiducial band amplitudes must be > 0");
  std::vector<int> cols, grp;
  rc = parse_rows(ctx, nb, nullptr, 0, nullptr, cols, grp);
  if (rc) return rc;
  wf_lbfgs_opts o;
  fill_opts(opts, o);
  StreamScope ss(ctx, stream);
  std::vector<double> Ed, E0, E2;
  int nc = 0;
  rc = run_qe(ctx, p, false, nsim, seed, draws, o, cols, Ed, E0, E2, nc);
  if (rc) return rc;
  bias_fisher(p->theta, nsim, nb, cols, grp, E0, E2, b, F);
  if (F_var) fisher_variance(p->theta, nsim, nb, E0, E2, F_var);
  if (E_sims) std::copy(E0.begin(), E0.end(), E_sims);
  return nc ? WF_NOT_CONVERGED : WF_OK;
}

int bandpower_iterate(wf_ctx* ctx, const wf_problem* p, int32_t nsim, uint64_t seed, const void* draws,
                      const wf_lbfgs_opts* opts, const int32_t* rows, int32_t nrows, const int32_t* groups,
                      int32_t max_iter, double rel_tol, double floor_frac, double* theta_hat, double* theta_hist,
                      int32_t* n_iter, double* E, double* b, double* F, void* stream) {
  if (!ctx) return WF_EINVAL;
  int rc = check_problem(ctx, p, true);
  if (rc) return rc;
  if (nsim < 1 || !theta_hat) return fail(ctx, WF_EINVAL, "need nsim >= 1 and theta_hat");
  if (max_iter < 1 || !(rel_tol >= 0) || !(floor_frac > 0 && floor_frac <= 1))
    return fail(ctx, WF_EINVAL, "need max_iter >= 1, rel_tol >= 0 and 0 < floor_frac <= 1");
  const int nb = p->nbands;
  for (int l = 0; l < nb; ++l)
    if (!(p->theta[l] > 0)) return fail(ctx, WF_EINVAL, "fiducial band amplitudes must be > 0");
  std::vector<int> cols, grp;
  rc = parse_rows(ctx, nb, rows, nrows, groups, cols, grp);
  if (rc) return rc;
  wf_lbfgs_opts o;
  fill_opts(opts, o);
  StreamScope ss(ctx, stream);
  std::vector<double> fid(p->theta, p->theta + nb), th(nb), hE, hb, hF, E0;
  if (theta_hist) std::copy(fid.begin(), fid.end(), theta_hist);
  int done = 0, ncTot = 0;
  while (done < max_iter) {
    wf_problem q = *p;
    q.theta = fid.data();
    int nc = 0;
    rc = qe_estimate(ctx, &q, true, nsim, seed, draws, o, cols, grp, th.data(), hE, hb, hF, E0, nc);
    if (rc) return rc;
    ncTot += nc;
    ++done;
    double rel = 0.0;
    for (int l = 0; l < nb; ++l) {
      const double nx = std::max(th[l], floor_frac * fid[l]);
      rel = std::max(rel, std::fabs(nx - fid[l]) / fid[l]);
      fid[l] = nx;
    }
    if (theta_hist) std::copy(fid.begin(), fid.end(), theta_hist + (size_t)done * nb);
    if (rel <= rel_tol) break;
  }
  std::copy(th.begin(), th.end(), theta_hat);
  if (n_iter) *n_iter = done;
  if (E) std::copy(hE.begin(), hE.end(), E);
  if (b) std::copy(hb.begin(), hb.end(), b);
  if (F) std::copy(hF.begin(), hF.end(), F);
  return ncTot ? WF_NOT_CONVERGED : WF_OK;
}

int bmode_leakage_qe(wf_ctx* ctx, const wf_problem* p, int32_t nsim, uint64_t seed, const void* draws,
                     const wf_lbfgs_opts* opts, const int32_t* b_bands, int32_t nbb, double* theta_b, double* E_b,
                     double* bias_b, double* F_bb, void* stream) {
  if (!ctx) return WF_EINVAL;
  int rc = check_problem(ctx, p, true);
  if (rc) return rc;
  const int nb = p->nbands;
  if (nsim < 1 || !theta_b || !b_bands || nbb < 1 || nbb > nb)
    return fail(ctx, WF_EINVAL, "need nsim >= 1, theta_b and 1 <= nbb <= nbands B bands");
  for (int j = 0; j < nbb; ++j)
    if (b_bands[j] < 0 || b_bands[j] >= nb || (j > 0 && b_bands[j] <= b_bands[j - 1]))
      return fail(ctx, WF_EINVAL, "b_bands must be strictly increasing band indices");
  for (int l = 0; l < nb; ++l)
    if (!(p->theta[l] > 0)) return fail(ctx, WF_EINVAL, "fiducial band amplitudes must be > 0");
  wf_lbfgs_opts o;
  fill_opts(opts, o);
  StreamScope ss(ctx, stream);
  const std::vector<int> cols(b_bands, b_bands + nbb);
  // the data and simulations without B power (noise plus E->B leakage)
  std::vector<double> thl(p->theta, p->theta + nb);
  for (int l : cols) thl[l] = 0.0;
  std::vector<double> Ed, El, E2u, Ed2, E0, E2;
  int nc1 = 0, nc2 = 0;
  rc = run_qe(ctx, p, true, nsim, seed, draws, o, std::vector<int>(), Ed, El, E2u, nc1, thl.data());
  if (rc) return rc;
  // fiducial simulations and boosted B bands: the B block of the Fisher matrix
  rc = run_qe(ctx, p, false, nsim, seed, draws, o, cols, Ed2, E0, E2, nc2);
  if (rc) return rc;
  std::vector<double> Fbb((size_t)nbb * nbb), Fr((size_t)nbb * nbb), bb(nbb), x(nbb);
  for (int j = 0; j < nbb; ++j) {
    double s = 0.0;
    for (int i = 0; i < nsim; ++i) s += El[(size_t)i * nb + cols[j]];
    bb[j] = s / nsim;
    for (int j2 = 0; j2 < nbb; ++j2) {   // row: band cols[j]; column: boosted band cols[j2]
      double t = 0.0;
      for (int i = 0; i < nsim; ++i) t += E2[((size_t)i * nbb + j2) * nb + cols[j]] - E0[(size_t)i * nb + cols[j]];
      Fr[(size_t)j * nbb + j2] = t / nsim / p->theta[cols[j2]];
    }
  }
  for (int j = 0; j < nbb; ++j)
    for (int j2 = 0; j2 < nbb; ++j2)
      Fbb[(size_t)j * nbb + j2] = 0.5 * (Fr[(size_t)j * nbb + j2] + Fr[(size_t)j2 * nbb + j]);
  for (int j = 0; j < nbb; ++j) x[j] = Ed[cols[j]] - bb[j];
  if (!dense_solve(Fbb, x, nbb)) return fail(ctx, WF_ENONFINITE, "singular B-band Fisher block");
  std::copy(x.begin(), x.end(), theta_b);
  if (E_b)
    for (int j = 0; j < nbb; ++j) E_b[j] = Ed[cols[j]];
  if (bias_b) std::copy(bb.begin(), bb.end(), bias_b);
  if (F_bb) std::copy(Fbb.begin(), Fbb.end(), F_bb);
  return (nc1 || nc2) ? WF_NOT_CONVERGED : WF_OK;
}

int bandpower_qe(wf_ctx* ctx, const wf_problem* p, int32_t nsim, uint64_t seed, const void* draws,
                 const wf_lbfgs_opts* opts, double* theta_hat, double* E, double* b, double* F, void* stream) {
  if (!ctx) return WF_EINVAL;
  int rc = check_problem(ctx, p, true);
  if (rc) return rc;
  if (nsim < 1 || !theta_hat) return fail(ctx, WF_EINVAL, "need nsim >= 1 and theta_hat");
  for (int l = 0; l < p->nbands; ++l)
    if (!(p->theta[l] > 0)) return fail(ctx, WF_EINVAL, "fiducial band amplitudes must be > 0");
  std::vector<int> cols, grp;
  rc = parse_rows(ctx, p->nbands, nullptr, 0, nullptr, cols, grp);
  if (rc) return rc;
  wf_lbfgs_opts o;
  fill_opts(opts, o);
  StreamScope ss(ctx, stream);
  std::vector<double> hE, hb, hF, E0;
  int nc = 0;
  rc = qe_estimate(ctx, p, true, nsim, seed, draws, o, cols, grp, theta_hat, hE, hb, hF, E0, nc);
  if (rc) return rc;
  if (E) std::copy(hE.begin(), hE.end(), E);
  if (b) std::copy(hb.begin(), hb.end(), b);
  if (F) std::copy(hF.begin(), hF.end(), F);
  return nc ? WF_NOT_CONVERGED : WF_OK;
}

int bandpower_qe_batch(wf_ctx* ctx, const wf_problem* probs, int32_t nprob, int32_t nsim, uint64_t seed,
                       const wf_lbfgs_opts* opts, double* const* theta_hat, double* const* E, double* const* b,
                       double* const* F, void* stream) {
  if (!ctx) return WF_EINVAL;
  if (nprob < 0 || nprob > 4096 || (nprob > 0 && (!probs || !theta_hat)))
    return fail(ctx, WF_EINVAL, "bad nprob / null arrays");
  if (nsim < 1) return fail(ctx, WF_EINVAL, "need nsim >= 1");
  for (int i = 0; i < nprob; ++i) {
    int rc = check_problem(ctx, &probs[i], true);
    if (rc) return rc;
    if (!theta_hat[i]) return fail(ctx, WF_EINVAL, "null theta_hat entry");
    for (int l = 0; l < probs[i].nbands; ++l)
      if (!(probs[i].theta[l] > 0)) return fail(ctx, WF_EINVAL, "fiducial band amplitudes must be > 0");
  }
  if (nprob == 0) return WF_OK;
  wf_lbfgs_opts o;
  fill_opts(opts, o);
  StreamScope ss(ctx, stream);
  std::vector<std::vector<double>> Ed, E0, E2;
  int nc = 0;
  int rc = run_qe_multi(ctx, probs, nprob, nsim, seed, o, Ed, E0, E2, nc);
  if (rc) return rc;
  for (int i = 0; i < nprob; ++i) {
    const int nb = probs[i].nbands;
    std::vector<int> cols(nb), grp(nb, 0);
    for (int l = 0; l < nb; ++l) cols[l] = l;
    std::vector<double> hb(nb), hF((size_t)nb * nb);
    bias_fisher(probs[i].theta, nsim, nb, cols, grp, E0[i], E2[i], hb.data(), hF.data());
    if (!newton_step(probs[i].theta, hF, Ed[i], hb, nb, theta_hat[i]))
      return fail(ctx, WF_ENONFINITE, "singular Fisher matrix of map " + std::to_string(i));
    if (E && E[i]) std::copy(Ed[i].begin(), Ed[i].end(), E[i]);
    if (b && b[i]) std::copy(hb.begin(), hb.end(), b[i]);
    if (F && F[i]) std::copy(hF.begin(), hF.end(), F[i]);
  }
  return nc ? WF_NOT_CONVERGED : WF_OK;
}

int wf_copy_bandwidth(wf_ctx* ctx, const void* src, void* dst, uint64_t bytes, int32_t reps, double* gbps) {
  if (!ctx) return WF_EINVAL;
  if (!src || !dst || !gbps || bytes == 0 || bytes % 16 != 0 || reps < 1)
    return fail(ctx, WF_EINVAL, "need src, dst, gbps, bytes a positive multiple of 16 and reps >= 1");
  (void)hipSetDevice(ctx->dev);
  hipEvent_t e0 = ev_get(ctx), e1 = ev_get(ctx);
  HIPCHK(stream_copy_launch(src, dst, bytes, ctx->cs));   // warm-up
  HIPCHK(hipEventRecord(e0, ctx->cs));
  for (int r = 0; r < reps; ++r) HIPCHK(stream_copy_launch(src, dst, bytes, ctx->cs));
  HIPCHK(hipEventRecord(e1, ctx->cs));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  ctx->evPool.push_back(e0);
  ctx->evPool.push_back(e1);
  *gbps = ms > 0.f ? 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9 : 0.0;
  return WF_OK;
}

int wf_forward(wf_ctx* ctx, const wf_problem* p, int32_t batch, const void* s, void* x, int32_t flags,
               void* stream) {
  int rc = check_op(ctx, p, batch, s, x);
  if (rc || batch == 0) return rc;
  if (flags & ~WF_MASK) return fail(ctx, WF_EINVAL, "bad flags");
  if ((flags & WF_MASK) && !p->w) return fail(ctx, WF_EINVAL, "WF_MASK needs w");
  StreamScope ss(ctx, stream);
  void *vin, *vy, *vout;
  Job* dj;
  double* part;
  const void* tw;
  rc = op_setup(ctx, p, batch, 0, nullptr, &vin, &vy, &vout, &dj, &part, &tw);
  if (rc) return rc;
  const int n = p->n, c = p->ncomp, dt = p->dtype;
  const int64_t L = (int64_t)c * n * (n / 2);
  const size_t eb = esize_of(dt), rs = rsize_of(dt);
  HIPCHK(unpack_launch(dt, n, c, batch, s, vin, ctx->cs));
  std::vector<Job> hj(batch);
  for (int i = 0; i < batch; ++i) {
    std::memset(&hj[i], 0, sizeof(Job));
    hj[i].mode = CM_FWD;
    hj[i].boost_band = -1;
    hj[i].W = (flags & WF_MASK) ? p->w : nullptr;
    hj[i].vin = (char*)vin + (size_t)i * L * eb;
    hj[i].y = (char*)vy + (size_t)i * L * eb;
    hj[i].xout = (char*)x + (size_t)i * c * n * n * rs;
  }
  HIPCHK(hipMemcpyAsync(dj, hj.data(), sizeof(Job) * batch, hipMemcpyHostToDevice, ctx->cs));
  HIPCHK(chain(ctx, dt, n, c, CH_COLINV, dj, batch, tw));
  HIPCHK(chain(ctx, dt, n, c, CH_ROW, dj, batch, tw));
  HIPCHK(hipStreamSynchronize(ctx->cs));
  return WF_OK;
}

int wf_adjoint(wf_ctx* ctx, const wf_problem* p, int32_t batch, const void* x, void* s, int32_t flags, void* stream) {
  int rc = check_op(ctx, p, batch, x, s);
  if (rc || batch == 0) return rc;
  if (flags & ~(WF_ADJ_GRAD | WF_MASK)) return fail(ctx, WF_EINVAL, "bad flags");
  if ((flags & WF_MASK) && !p->w) return fail(ctx, WF_EINVAL, "WF_MASK needs w");
  StreamScope ss(ctx, stream);
  void *vin, *vy, *vout;
  Job* dj;
  double* part;
  const void* tw;
  rc = op_setup(ctx, p, batch, 0, nullptr, &vin, &vy, &vout, &dj, &part, &tw);
  if (rc) return rc;
  const int n = p->n, c = p->ncomp, dt = p->dtype;
  const int64_t L = (int64_t)c * n * (n / 2);
  const size_t eb = esize_of(dt), rs = rsize_of(dt);
  std::vector<Job> hj(batch);
  for (int i = 0; i < batch; ++i) {
    std::memset(&hj[i], 0, sizeof(Job));
    hj[i].mode = (flags & WF_ADJ_GRAD) ? CM_ADJ_GRAD : CM_ADJ;
    hj[i].boost_band = -1;
    hj[i].W = (flags & WF_MASK) ? p->w : nullptr;
    hj[i].d = (const char*)x + (size_t)i * c * n * n * rs;
    hj[i].y = (char*)vy + (size_t)i * L * eb;
    hj[i].vout = (char*)vout + (size_t)i * L * eb;
  }
  HIPCHK(hipMemcpyAsync(dj, hj.data(), sizeof(Job) * batch, hipMemcpyHostToDevice, ctx->cs));
  HIPCHK(chain(ctx, dt, n, c, CH_ROW, dj, batch, tw));
  HIPCHK(chain(ctx, dt, n, c, CH_COLFWD, dj, batch, tw));
  HIPCHK(pack_launch(dt, n, c, batch, vout, L, nullptr, 0, nullptr, s, ctx->cs));
  HIPCHK(hipStreamSynchronize(ctx->cs));
  return WF_OK;
}

static int raw_chain(wf_ctx* ctx, const wf_problem* p, int batch, const void* s, double* chi2, void* out, int mode,
                     void* stream) {
  StreamScope ss(ctx, stream);
  void *vin, *vy, *vout;
  Job* dj;
  double* part;
  const void* tw;
  PriorTab pt;
  int rc = op_setup(ctx, p, batch, 0, &pt, &vin, &vy, &vout, &dj, &part, &tw);
  if (rc) return rc;
  const int n = p->n, c = p->ncomp, dt = p->dtype;
  const int64_t L = (int64_t)c * n * (n / 2);
  const size_t eb = esize_of(dt);
  const int pstride = c * n / RB_MIN;
  HIPCHK(unpack_launch(dt, n, c, batch, s, vin, ctx->cs));
  std::vector<Job> hj(batch);
  for (int i = 0; i < batch; ++i) {
    std::memset(&hj[i], 0, sizeof(Job));
    hj[i].mode = mode;
    hj[i].boost_band = -1;
    hj[i].vin = (char*)vin + (size_t)i * L * eb;
    hj[i].vadd = hj[i].vin;
    hj[i].y = (char*)vy + (size_t)i * L * eb;
    hj[i].vout = (char*)vout + (size_t)i * L * eb;
    hj[i].d = p->d;
    hj[i].W = p->w;
    hj[i].sOut = pt.sq;
    hj[i].part = part + (size_t)i * PK_COUNT * pstride;
    hj[i].pstride = pstride;
  }
  HIPCHK(hipMemcpyAsync(dj, hj.data(), sizeof(Job) * batch, hipMemcpyHostToDevice, ctx->cs));
  for (int w = 0; w < 3; ++w) HIPCHK(chain(ctx, dt, n, c, w, dj, batch, tw));
  if (out) HIPCHK(pack_launch(dt, n, c, batch, vout, L, nullptr, 0, nullptr, out, ctx->cs));
  if (chi2) {
    std::vector<double> hp((size_t)PK_COUNT * pstride * batch);
    HIPCHK(hipMemcpyAsync(hp.data(), part, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, ctx->cs));
    HIPCHK(hipStreamSynchronize(ctx->cs));
    const int ncol = (n / 2) / TB, nrow = c * n / RB_MIN;
    for (int i = 0; i < batch; ++i) {
      const double* q = &hp[(size_t)i * PK_COUNT * pstride];
      double pr = 0.0, rs = 0.0;
      for (int b = 0; b < ncol; ++b) pr += q[PK_PRIOR * pstride + b];
      for (int b = 0; b < nrow; ++b) rs += q[PK_RES * pstride + b];
      chi2[i] = 2.0 * pr + rs;
    }
  }
  HIPCHK(hipStreamSynchronize(ctx->cs));
  return WF_OK;
}

int wf_chi2_grad(wf_ctx* ctx, const wf_problem* p, int32_t batch, const void* s, double* chi2, void* grad_s,
                 void* stream) {
  int rc = check_op(ctx, p, batch, s, chi2);
  if (rc || batch == 0) return rc;
  rc = check_problem(ctx, p, true);
  if (rc) return rc;
  return raw_chain(ctx, p, batch, s, chi2, grad_s, CM_RAW_GRAD, stream);
}

int posterior_error(wf_ctx* ctx, const wf_problem* p, int32_t nsim, uint64_t seed, const void* draws,
                    const wf_lbfgs_opts* opts, void* var_modes, void* var_pix, void* stream) {
  if (!ctx) return WF_EINVAL;
  int rc = check_problem(ctx, p, false);
  if (rc) return rc;
  if (nsim < 1 || (!var_modes && !var_pix)) return fail(ctx, WF_EINVAL, "need nsim >= 1 and an output");
  wf_lbfgs_opts o;
  fill_opts(opts, o);
  StreamScope ss(ctx, stream);
  const int n = p->n, c = p->ncomp, dt = p->dtype;
  const size_t rs = rsize_of(dt), eb = esize_of(dt);
  const int64_t L = (int64_t)c * n * (n / 2), npix = (int64_t)c * n * n, next = (int64_t)c * n * (n / 2 + 1);
  // float64 sums over all simulations, kept across the chunks
  rc = arena_reserve(ctx, ctx->accA, align_up(sizeof(double) * next) + align_up(sizeof(double) * npix));
  if (rc) return rc;
  double* accM = (double*)arena_take(ctx->accA, sizeof(double) * next);
  double* accP = (double*)arena_take(ctx->accA, sizeof(double) * npix);
  HIPCHK(hipMemsetAsync(accM, 0, sizeof(double) * next, ctx->cs));
  HIPCHK(hipMemsetAsync(accP, 0, sizeof(double) * npix, ctx->cs));
  const double perInst = (double)(3 + 2 * o.m) * L * eb + 2.0 * npix * rs + 2.0 * next * eb;
  const int chunk = (int)std::max(1.0, std::min((double)kMaxChunk, kSimBudgetBytes / perInst));
  int notConv = 0;
  for (int off = 0; off < nsim; off += chunk) {
    const int cnt = std::min(nsim - off, chunk);
    std::vector<SimEntry> ents;
    for (int j = 0; j < cnt; ++j) ents.push_back({1, off + j, -1, -1});
    const size_t need = prior_bytes(p) + align_up(sizeof(Job) * cnt) + align_up((size_t)npix * rs * cnt) +
                        align_up((size_t)L * eb * cnt) + 2 * align_up((size_t)next * eb * cnt);
    rc = arena_reserve(ctx, ctx->simA, need);
    if (rc) return rc;
    PriorTab pt;
    rc = build_prior(ctx, ctx->simA, p, p->theta, pt);
    if (rc) return rc;
    void* dbuf = arena_take(ctx->simA, (size_t)npix * rs * cnt);
    void* ybuf = arena_take(ctx->simA, (size_t)L * eb * cnt);   // L eb = npix rs: also a pixel batch
    void* sbuf = arena_take(ctx->simA, (size_t)next * eb * cnt);
    void* shbuf = arena_take(ctx->simA, (size_t)next * eb * cnt);
    // data, MAP, signal coefficients of the simulations (same normals)
    rc = simulate_entries(ctx, p, ents, seed, draws, 0, pt, dbuf, ybuf, 2.0);
    if (rc) return rc;
    std::vector<wf_problem> probs(cnt, *p);
    for (int j = 0; j < cnt; ++j) probs[j].d = (const char*)dbuf + (size_t)j * npix * rs;
    SolveOut so;
    rc = solve_core(ctx, probs.data(), cnt, o, so);
    if (rc) return rc;
    for (int j = 0; j < cnt; ++j) {
      notConv += so.st[j].status != WF_SOLVE_CONVERGED;
      HIPCHK(pack_launch(dt, n, c, 1, so.w[j], 0, so.prior[j].sq, 1, nullptr, (char*)shbuf + (size_t)j * next * eb,
                         ctx->cs));
    }
    HIPCHK(sim_coeffs_launch(dt, n, c, cnt, off, seed, draws ? (const char*)draws + (size_t)off * 2 * npix * rs : nullptr,
                             pt.sq, sbuf, ctx->cs));
    if (var_modes) HIPCHK(sqdiff_acc_launch(dt, next, 2, cnt, sbuf, shbuf, accM, ctx->cs));
    if (var_pix) {   // R s - R s_hat = R (s - s_hat)
      rc = wf_forward(ctx, p, cnt, sbuf, dbuf, 0, ctx->cs);
      if (rc) return rc;
      rc = wf_forward(ctx, p, cnt, shbuf, ybuf, 0, ctx->cs);
      if (rc) return rc;
      HIPCHK(sqdiff_acc_launch(dt, npix, 1, cnt, dbuf, ybuf, accP, ctx->cs));
    }
  }
  if (var_modes) HIPCHK(acc_out_launch(dt, next, accM, 1.0 / nsim, var_modes, ctx->cs));
  if (var_pix) HIPCHK(acc_out_launch(dt, npix, accP, 1.0 / nsim, var_pix, ctx->cs));
  return notConv ? WF_NOT_CONVERGED : WF_OK;
}

int convergence_by_band(wf_ctx* ctx, const wf_problem* p, int32_t ntol, const double* tols, const wf_lbfgs_opts* opts,
                        double* power, double* err_power, double* cv, int32_t* iters, void* const* s_out,
                        void* stream) {
  if (!ctx) return WF_EINVAL;
  int rc = check_problem(ctx, p, true);
  if (rc) return rc;
  if (ntol < 1 || ntol > 64 || !tols || !power) return fail(ctx, WF_EINVAL, "need 1 <= ntol <= 64, tols and power");
  for (int t = 0; t < ntol; ++t)
    if (!(tols[t] > 0)) return fail(ctx, WF_EINVAL, "tolerances must be > 0");
  wf_lbfgs_opts o;
  fill_opts(opts, o);
  StreamScope ss(ctx, stream);
  const int B = ntol + 1, nb = p->nbands, n = p->n, c = p->ncomp, dt = p->dtype;
  // one batched solve: the reference (opts->rel_grad_tol) and one copy per tolerance
  std::vector<wf_problem> probs(B, *p);
  std::vector<double> tv(B);
  tv[0] = o.rel_grad_tol;
  for (int t = 0; t < ntol; ++t) tv[t + 1] = tols[t];
  SolveOut so;
  rc = solve_core(ctx, probs.data(), B, o, so, tv.data());
  if (rc) return rc;
  const int64_t L = (int64_t)c * n * (n / 2);
  if (nb > 0) {
    const int nj = 2 * B - 1, nblk = band_nblk(L);
    const size_t need = align_up(sizeof(BandJob) * nj) + align_up(sizeof(double) * (size_t)nj * nblk * nb) +
                        align_up(sizeof(double) * (size_t)nj * nb);
    rc = arena_reserve(ctx, ctx->opA, need);
    if (rc) return rc;
    BandJob* dj = (BandJob*)arena_take(ctx->opA, sizeof(BandJob) * nj);
    double* part = (double*)arena_take(ctx->opA, sizeof(double) * (size_t)nj * nblk * nb);
    double* dE = (double*)arena_take(ctx->opA, sizeof(double) * (size_t)nj * nb);
    std::vector<BandJob> hj(nj);
    for (int j = 0; j < nj; ++j) {
      const int i = j < B ? j : j - B + 1;   // jobs B.. are the differences to the reference
      hj[j].f = so.w[i];
      hj[j].f2 = j < B ? nullptr : so.w[0];
      hj[j].sq = so.prior[i].sq;
      hj[j].aw = so.prior[i].a;
      hj[j].bandI = so.prior[i].bandI;
      hj[j].theta = so.prior[i].theta;
      hj[j].part = part + (size_t)j * nblk * nb;
      hj[j].E = dE + (size_t)j * nb;
      hj[j].L = L;
      hj[j].nbands = nb;
      hj[j].raw = 2;
    }
    HIPCHK(hipMemcpyAsync(dj, hj.data(), sizeof(BandJob) * nj, hipMemcpyHostToDevice, ctx->cs));
    HIPCHK(band_launch(dt, dj, nj, L, ctx->cs));
    std::vector<double> hE((size_t)nj * nb);
    HIPCHK(hipMemcpyAsync(hE.data(), dE, sizeof(double) * hE.size(), hipMemcpyDeviceToHost, ctx->cs));
    std::vector<int32_t> bI(L);
    HIPCHK(hipMemcpyAsync(bI.data(), so.prior[0].bandI, sizeof(int32_t) * L, hipMemcpyDeviceToHost, ctx->cs));
    HIPCHK(hipStreamSynchronize(ctx->cs));
    std::copy(hE.begin(), hE.begin() + (size_t)B * nb, power);
    if (err_power) std::copy(hE.begin() + (size_t)B * nb, hE.end(), err_power);
    if (cv) {   // sqrt(2 / N_l), N_l = full-plane modes of band l (two per free entry)
      std::vector<int64_t> cnt(nb, 0);
      for (int64_t e = 0; e < L; ++e)
        if (bI[e] >= 0 && bI[e] < nb) ++cnt[bI[e]];
      for (int l = 0; l < nb; ++l) cv[l] = cnt[l] > 0 ? std::sqrt(2.0 / (2.0 * cnt[l])) : 0.0;
    }
  }
  if (iters)
    for (int i = 0; i < B; ++i) iters[i] = so.st[i].iter;
  if (s_out)
    for (int i = 0; i < B; ++i)
      if (s_out[i])
        HIPCHK(pack_launch(dt, n, c, 1, so.w[i], 0, so.prior[i].sq, 1, nullptr, s_out[i], ctx->cs));
  return so.st[0].status == WF_SOLVE_CONVERGED ? WF_OK : WF_NOT_CONVERGED;
}

int wf_hvp(wf_ctx* ctx, const wf_problem* p, int32_t batch, const void* pv, void* Dp, void* stream) {
  int rc = check_op(ctx, p, batch, pv, Dp);
  if (rc || batch == 0) return rc;
  rc = check_problem(ctx, p, false);
  if (rc) return rc;
  return raw_chain(ctx, p, batch, pv, nullptr, Dp, CM_RAW_HV, stream);
}

}  // extern "C"

namespace {
// E_l (eq. el) of `batch` external fields with p's prior, into E HOST [batch][nbands]; the
// caller has checked the arguments and entered the stream scope.
int band_E_ext(wf_ctx* ctx, const wf_problem* p, int batch, const void* s, double* E) {
  const int nb = p->nbands;
  const int n = p->n, c = p->ncomp, dt = p->dtype;
  const int64_t L = (int64_t)c * n * (n / 2);
  const size_t eb = esize_of(dt);
  const int nblk = band_nblk(L);
  const size_t extra = align_up(sizeof(BandJob) * batch) + align_up(sizeof(double) * (size_t)batch * nblk * nb) +
                       align_up(sizeof(double) * (size_t)batch * nb);
  void *vin, *vy, *vout;
  Job* dj;
  double* part;
  const void* tw;
  PriorTab pt;
  int rc = op_setup(ctx, p, batch, extra, &pt, &vin, &vy, &vout, &dj, &part, &tw);
  if (rc) return rc;
  HIPCHK(unpack_launch(dt, n, c, batch, s, vin, ctx->cs));
  BandJob* bj = (BandJob*)arena_take(ctx->opA, sizeof(BandJob) * batch);
  double* bpart = (double*)arena_take(ctx->opA, sizeof(double) * (size_t)batch * nblk * nb);
  double* dE = (double*)arena_take(ctx->opA, sizeof(double) * (size_t)batch * nb);
  std::vector<BandJob> hj(batch);
  for (int i = 0; i < batch; ++i) {
    hj[i].f = (char*)vin + (size_t)i * L * eb;
    hj[i].f2 = nullptr;
    hj[i].sq = pt.sq;
    hj[i].aw = nullptr;
    hj[i].bandI = pt.bandI;
    hj[i].theta = pt.theta;
    hj[i].part = bpart + (size_t)i * nblk * nb;
    hj[i].E = dE + (size_t)i * nb;
    hj[i].L = L;
    hj[i].nbands = nb;
    hj[i].raw = 1;
  }
  HIPCHK(hipMemcpyAsync(bj, hj.data(), sizeof(BandJob) * batch, hipMemcpyHostToDevice, ctx->cs));
  HIPCHK(band_launch(dt, bj, batch, L, ctx->cs));
  HIPCHK(hipMemcpyAsync(E, dE, sizeof(double) * (size_t)batch * nb, hipMemcpyDeviceToHost, ctx->cs));
  HIPCHK(hipStreamSynchronize(ctx->cs));
  return WF_OK;
}
}  // namespace

extern "C" {

int wf_hvp_noalloc(wf_ctx* ctx, const wf_problem* p, int32_t batch, const void* pv, void* Dp, void* stream) {
  int rc = check_op(ctx, p, batch, pv, Dp);
  if (rc || batch == 0) return rc;
  rc = check_problem(ctx, p, false);
  if (rc) return rc;
  if (!ctx->scratch) return fail(ctx, WF_EHIP, "no device scratch on this context's device");
  const int n = p->n, c = p->ncomp, dt = p->dtype, nb = p->nbands;
  const int64_t L = (int64_t)c * n * (n / 2);
  const size_t eb = esize_of(dt), rs = rsize_of(dt);
  const int pstride = c * n / RB_MIN;
  auto key = std::make_pair(n, dt);
  if (!ctx->htw.count(key)) twiddle_bytes(n, dt, ctx->htw[key]);
  const std::vector<char>& htw = ctx->htw[key];
  // scratch layout: twiddles, prior tables (sqrt S, band, theta and one spare double),
  // field / intermediate / output vectors, jobs, chain partials
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  const size_t oTw = take(htw.size());
  const size_t oSq = take((size_t)L * rs);
  const size_t oBand = take((size_t)L * 4);
  const size_t oTheta = take(sizeof(double) * (std::max(1, nb) + 1));
  const size_t oIn = take((size_t)L * eb * batch);
  const size_t oY = take((size_t)L * eb * batch);
  const size_t oOut = take((size_t)L * eb * batch);
  const size_t oJobs = take(sizeof(Job) * batch);
  const size_t oPart = take(sizeof(double) * PK_COUNT * pstride * batch);
  if (off > (size_t)WF_NOALLOC_SCRATCH_BYTES)
    return fail(ctx, WF_EINVAL, "wf_hvp_noalloc needs " + std::to_string(off) + " bytes of scratch for this batch; the limit is " +
                                    std::to_string((size_t)WF_NOALLOC_SCRATCH_BYTES) + " bytes");
  rc = prepare(ctx, n, c, dt);   // kernel attributes only
  if (rc) return rc;
  StreamScope ss(ctx, stream);
  char* S = (char*)ctx->scratch;
  double* theta = (double*)(S + oTheta);
  HIPCHK(hipMemcpyAsync(S + oTw, htw.data(), htw.size(), hipMemcpyHostToDevice, ctx->cs));
  if (nb > 0) HIPCHK(hipMemcpyAsync(theta, p->theta, sizeof(double) * nb, hipMemcpyHostToDevice, ctx->cs));
  HIPCHK(prior_table_launch(dt, n, c, p->pshape, p->band, theta, nb, nullptr, theta + std::max(1, nb), S + oSq,
                            (int32_t*)(S + oBand), nullptr, nullptr, ctx->cs));
  HIPCHK(unpack_launch(dt, n, c, batch, pv, S + oIn, ctx->cs));
  std::vector<Job> hj(batch);
  for (int i = 0; i < batch; ++i) {
    std::memset(&hj[i], 0, sizeof(Job));
    hj[i].mode = CM_RAW_HV;
    hj[i].boost_band = -1;
    hj[i].vin = S + oIn + (size_t)i * L * eb;
    hj[i].vadd = hj[i].vin;
    hj[i].y = S + oY + (size_t)i * L * eb;
    hj[i].vout = S + oOut + (size_t)i * L * eb;
    hj[i].d = p->d;
    hj[i].W = p->w;
    hj[i].sOut = S + oSq;
    hj[i].part = (double*)(S + oPart) + (size_t)i * PK_COUNT * pstride;
    hj[i].pstride = pstride;
  }
  Job* dj = (Job*)(S + oJobs);
  HIPCHK(hipMemcpyAsync(dj, hj.data(), sizeof(Job) * batch, hipMemcpyHostToDevice, ctx->cs));
  for (int w = 0; w < 3; ++w) HIPCHK(chain(ctx, dt, n, c, w, dj, batch, S + oTw));
  HIPCHK(pack_launch(dt, n, c, batch, S + oOut, L, nullptr, 0, nullptr, Dp, ctx->cs));
  return WF_OK;
}

int wf_band_E(wf_ctx* ctx, const wf_problem* p, int32_t batch, const void* s, double* E, void* stream) {
  int rc = check_op(ctx, p, batch, s, E);
  if (rc || batch == 0) return rc;
  rc = check_problem(ctx, p, false);
  if (rc) return rc;
  if (p->nbands == 0) return WF_OK;
  StreamScope ss(ctx, stream);
  return band_E_ext(ctx, p, batch, s, E);
}

int wf_chi2_dtheta(wf_ctx* ctx, const wf_problem* p, int32_t batch, const void* s, const double* gout,
                   double* dtheta, void* stream) {
  int rc = check_op(ctx, p, batch, s, dtheta);
  if (rc) return rc;
  rc = check_problem(ctx, p, false);
  if (rc) return rc;
  const int nb = p->nbands;
  if (nb == 0) return WF_OK;
  if (!dtheta) return fail(ctx, WF_EINVAL, "null dtheta");
  for (int b = 0; b < nb; ++b) dtheta[b] = 0.0;
  if (batch == 0) return WF_OK;
  if (gout)
    for (int i = 0; i < batch; ++i)
      if (!std::isfinite(gout[i])) return fail(ctx, WF_ENONFINITE, "non-finite gout");
  StreamScope ss(ctx, stream);
  std::vector<double> E((size_t)batch * nb);
  rc = band_E_ext(ctx, p, batch, s, E.data());
  if (rc) return rc;
  // d chi^2 / d theta_b = -sum_{k in b, full plane} |s_k|^2 / (theta_b^2 P_k) = -2 E_b
  for (int b = 0; b < nb; ++b) {
    double a = 0.0;
    for (int i = 0; i < batch; ++i) a += (gout ? gout[i] : 1.0) * E[(size_t)i * nb + b];
    dtheta[b] = -2.0 * a;
  }
  return WF_OK;
}

int wf_set_chain_tiles(wf_ctx* ctx, int32_t rbv, int32_t cpb, int32_t group, int32_t reg) {
  if (!ctx) return WF_EINVAL;
  if (rbv == 0) {
    ctx->fixedSet = false;
    return WF_OK;
  }
  if (!(rbv == 2 || rbv == 4 || rbv == 8) || !(cpb == 1 || cpb == 2 || cpb == 4) || group < 0 || reg < 0 || reg > 8)
    return fail(ctx, WF_EINVAL, "tiles: rbv in {2,4,8}, cpb in {1,2,4}, group >= 0, reg in [0, 8]");
  ctx->fixedCfg.rbv = rbv;
  ctx->fixedCfg.cpb = cpb;
  ctx->fixedCfg.group = group;
  ctx->fixedCfg.reg = reg;
  ctx->fixedSet = true;
  return WF_OK;
}

int wf_get_chain_tiles(wf_ctx* ctx, int32_t n, int32_t ncomp, int32_t dtype, int32_t batch, int32_t* rbv, int32_t* cpb,
                       int32_t* group, int32_t* reg) {
  if (!ctx || !rbv || !cpb || !group || !reg) return WF_EINVAL;
  const int bucket = batch >= 64 ? 64 : (batch >= 16 ? 16 : (batch >= 4 ? 4 : 1));
  auto it = ctx->tuned.find(std::make_tuple((int)n, (int)ncomp, (int)dtype, bucket));
  ChainCfg c = it != ctx->tuned.end() ? it->second : ChainCfg();
  if (ctx->fixedSet) c = chain_cfg_supported(dtype, n, ncomp, ctx->fixedCfg) ? ctx->fixedCfg : ChainCfg();
  *rbv = c.rbv;
  *cpb = c.cpb;
  *group = c.group;
  *reg = c.reg;
  return it != ctx->tuned.end() || ctx->fixedSet ? WF_OK : WF_NOT_CONVERGED;
}

int wf_set_profiling(wf_ctx* ctx, int32_t on) {
  if (!ctx) return WF_EINVAL;
  ctx->prof = on != 0;
  return WF_OK;
}

int wf_kernel_kinds(void) { return KK_COUNT; }

const char* wf_kernel_kind_name(int32_t k) { return (k >= 0 && k < KK_COUNT) ? kKindNames[k] : ""; }

int wf_get_kernel_stats(wf_ctx* ctx, int64_t* launches, double* ms, double* bytes) {
  if (!ctx) return WF_EINVAL;
  int rc = drain_events(ctx);
  if (rc) return rc;
  for (int k = 0; k < KK_COUNT; ++k) {
    if (launches) launches[k] = ctx->launches[k];
    if (ms) ms[k] = ctx->ms[k];
    if (bytes) bytes[k] = ctx->bytes[k];
  }
  return WF_OK;
}

int wf_reset_kernel_stats(wf_ctx* ctx) {
  if (!ctx) return WF_EINVAL;
  int rc = drain_events(ctx);
  if (rc) return rc;
  for (int k = 0; k < KK_COUNT; ++k) {
    ctx->launches[k] = 0;
    ctx->ms[k] = 0.0;
    ctx->bytes[k] = 0.0;
  }
  return WF_OK;
}

}  // extern "C"
