// Shared device/host definitions of libwf (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wf {

// ------------------------------------------------------------------------ complex
template <typename T>
struct cpx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> mk(T a, T b) {
  cpx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T>
__device__ __forceinline__ cpx<T> add(cpx<T> a, cpx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cpx<T> sub(cpx<T> a, cpx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cpx<T> mul(cpx<T> a, cpx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cpx<T> mulc(cpx<T> a, cpx<T> b) {
  return mk(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename T>
__device__ __forceinline__ cpx<T> conj(cpx<T> a) { return mk(a.x, -a.y); }
template <typename T>
__device__ __forceinline__ cpx<T> scale(cpx<T> a, T s) { return mk(a.x * s, a.y * s); }

// ------------------------------------------------------------------------ global accesses
// Device pointers taken from job descriptors are generic pointers, which compile to flat
// accesses with 64-bit per-lane addresses.  gld / gst address global memory explicitly from
// a work-group-uniform base with a 32-bit byte offset (the base stays in scalar registers,
// the offset takes one vector register); i * sizeof(T) must stay below 4 GiB.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
typedef float gf32x2 __attribute__((ext_vector_type(2)));
typedef float gf32x4 __attribute__((ext_vector_type(4)));
typedef double gf64x2 __attribute__((ext_vector_type(2)));
// the builtin type a T moves as (class types cannot be copied out of a qualified address space)
template <typename T>
struct GStore {
  using type = T;
};
template <>
struct GStore<cpx<float>> {
  using type = gf32x2;
};
template <>
struct GStore<cpx<double>> {
  using type = gf64x2;
};
template <>
struct GStore<float2> {
  using type = gf32x2;
};
template <>
struct GStore<float4> {
  using type = gf32x4;
};
template <>
struct GStore<double2> {
  using type = gf64x2;
};
template <typename T>
__device__ __forceinline__ T gld(const T* base, uint32_t i) {
  using S = typename GStore<T>::type;
  const S v = *(gptr<const S>)((gptr<const char>)(const char*)base + i * (uint32_t)sizeof(T));
  T r;
  __builtin_memcpy(&r, &v, sizeof(T));
  return r;
}
// the same load with the non-temporal hint, for streams that a pass reads once and that no
// cache can hold until they are read again (the solver's history vectors)
template <typename T>
__device__ __forceinline__ T gldnt(const T* base, uint32_t i) {
  using S = typename GStore<T>::type;
  const S v = __builtin_nontemporal_load((gptr<const S>)((gptr<const char>)(const char*)base + i * (uint32_t)sizeof(T)));
  T r;
  __builtin_memcpy(&r, &v, sizeof(T));
  return r;
}
template <typename T>
__device__ __forceinline__ void gst(T* base, uint32_t i, const T& x) {
  using S = typename GStore<T>::type;
  S v;
  __builtin_memcpy(&v, &x, sizeof(T));
  *(gptr<S>)((gptr<char>)(char*)base + i * (uint32_t)sizeof(T)) = v;
}

// ------------------------------------------------------------------------ layout
// Internal storage of a harmonic field: column blocks of TB columns, each block a
// contiguous [n][TB] array, so a column pass reads contiguous memory and a row pass
// over R consecutive rows reads contiguous R*TB runs.  The Nyquist column kx = n/2
// (always dead) is not stored.
constexpr int TB = 2;
constexpr int RB_MIN = 2;  // granularity of the row pass's partial sums (rows)
constexpr int NT = 256;    // threads per work-group of the transform and vector passes
// vector loads per thread per stream in a vector pass (a template parameter of the passes): 8
// (longer runs per stream) for a class with enough work-groups to fill the GPU, else 4 (twice the
// work-groups, for the few-instance classes of an uneven batch and their tails)
constexpr int PASS_U_FEW = 4, PASS_U_MANY = 8;
constexpr int64_t PASS_MANY_MIN_GROUPS = 4096;   // work-groups per pass launch needed for PASS_U_MANY

__host__ __device__ __forceinline__ int64_t fidx(int n, int c, int ky, int kx) {
  const int h = n >> 1;
  return ((int64_t)(c * (h / TB) + kx / TB) * n + ky) * TB + (kx % TB);
}

// live = not DC, not on a Nyquist line; free = live and not a kx = 0 conjugate partner
__host__ __device__ __forceinline__ bool is_live(int n, int ky, int kx) {
  return !((ky == 0 && kx == 0) || ky == (n >> 1) || kx == (n >> 1));
}
__host__ __device__ __forceinline__ bool is_partner(int n, int ky, int kx) {
  return kx == 0 && ky > (n >> 1);
}
__host__ __device__ __forceinline__ bool is_free(int n, int ky, int kx) {
  return is_live(n, ky, kx) && !is_partner(n, ky, kx);
}

// ------------------------------------------------------------------------ chain jobs
// One instance's work for one pass of the transform chain (column inverse, row,
// column forward).  The solver kernels write these on the device every iteration;
// operator-level calls fill them on the host.
enum ChainMode : int {
  CM_NONE = 0,
  CM_HV = 1,        // out = v + sOut . R^T W R (sIn . v)             (whitened curvature)
  CM_GRAD = 2,      // out = v + sOut . R^T W (R (sIn . v) - d)       (whitened gradient)
  CM_FWD = 3,       // x = R (sIn . v)  (sIn may be null)             (forward only)
  CM_ADJ = 4,       // out = R^T x                                     (metric adjoint)
  CM_ADJ_GRAD = 5,  // out = 2 R^T x on free entries
  CM_RAW_GRAD = 6,  // out = 4 (S^-1 v + R^T W (R v - d)), chi^2 partials (raw field)
  CM_RAW_HV = 7,    // out = 4 (S^-1 v + R^T W R v)
  CM_SIM = 8,       // x = M (R (sIn . boost . z / sqrt 2) + noise)     (simulation)
  CM_FLUSH = 9,     // solver only: no transform this iteration, pass B brings w up to date
  CM_DOTS = 10      // solver only: no transform, pass A takes the dots of the exact gradient that
                    // a failed stop confirmation left out
};

// partial-sum kinds written per block
enum { PK_PRIOR = 0, PK_RES = 1, PK_VO = 2, PK_OO = 3, PK_DG = 4, PK_DD = 5 };   // PK_DD + j, j < MMAX
constexpr int MMAX = 16;
constexpr int PK_COUNT = PK_DD + MMAX;

struct Job {
  int mode;
  int boost_band;       // CM_SIM
  int sim;              // CM_SIM: simulation index (Philox counter word 1)
  int pad0;
  double boost_factor;  // CM_SIM
  uint64_t seed;        // CM_SIM (Philox key), used when draws == nullptr
  const void* vin;      // column-inverse input (internal layout)
  void* y;              // intermediate (internal layout)
  void* vout;           // column-forward output (internal layout)
  const void* vadd;     // added term in the column-forward epilogue
  const void* d;        // data [c][n][n] (CM_GRAD, CM_RAW_GRAD) or pixel input (CM_ADJ*)
  const void* W;        // [n][n]
  const void* sIn;      // scale table for the column inverse (sqrt S), nullable
  const void* sOut;     // scale / liveness table for the column forward (sqrt S)
  const void* aTab;     // prior weight of the solver variable (preconditioned solves), nullable -> 1
  const int32_t* band;  // internal-layout band table (CM_SIM boost)
  const void* draws;    // [2][c][n][n] normals (CM_SIM), nullable -> Philox
  void* xout;           // pixel output (CM_FWD, CM_SIM)
  double* part;         // [PK_COUNT][pstride] partial sums
  int pstride;
  int pad1;
  // curvature mode inside the solver: also accumulate out . g (gvec) and out . Dp_j for the
  // history slots j set in dpMask (Dp_j at dpBase + j * dpStride)
  const void* gvec;
  const void* dpBase;
  int64_t dpStride;
  uint32_t dpMask;
  int pad2;
};

// ------------------------------------------------------------------------ solver state

enum { ST_RUNNING = -1 };   // otherwise WF_SOLVE_* values

// kernel kinds for instrumentation
enum {
  KK_COLINV = 0, KK_ROW = 1, KK_COLFWD = 2, KK_PASSA = 3, KK_PASSB = 4, KK_POST = 5, KK_COEF = 6,
  KK_MISC = 7, KK_DIR = 8, KK_SIM = 9, KK_CAT = 10, KK_COUNT = 11
};

struct LbState {
  int status;
  int iter;
  int nhist;         // kept pairs: slots head, head-1, ..., head-nhist+1 (mod m)
  int head;
  int pending;       // the newest pair's step is not yet applied to g
  int npend;         // the newest npend pairs' steps are not yet applied to w:
                     // the iterate is w + sum alpha_i p_i over them
  int npendB;        // npend when pass B ran (for post B)
  int flushB;        // pass B applies the pending steps to w
  int dirB;          // pass B forms a direction
  int after;         // decision waiting for a flush of w: 0 none, 1 exact-gradient refresh,
                     // 2 + status: stop with that status
  int chainMode;     // mode of the chain enqueued in this iteration
  int lastWasGrad;   // g currently holds an exact gradient
  int ngrad;
  int lastGradIter;
  int newslot;       // slot of the direction being formed
  int m;
  int doB;           // pass B runs in this iteration
  double g0norm;
  double gg;
  double chi2;
  double dchi2;
  double gdotp;      // g . p of the current direction (measured)
  double pDp;
  double alpha[MMAX];
  double PD[MMAX][MMAX];   // p_i . Dp_j
  double DD[MMAX][MMAX];   // Dp_i . Dp_j
  double gP[MMAX];         // g . p_i of the current gradient
  double gD[MMAX];         // g . Dp_i
  double pkD[MMAX];        // p . Dp_j of the current direction (from the Gram entries)
  double coef[2 * MMAX + 1];   // direction on (p_0..p_{m-1}, Dp_0..Dp_{m-1}, g)
  double bytes[KK_COUNT];      // algorithmic bytes moved for this instance
  // conjugate gradients: rho = g.g of the current gradient, beta of the next direction
  double rho;
  double beta;
  int doDir;                   // the direction pass runs in this iteration
  int confirm;                 // the pending exact gradient confirms a stop: pass A takes g.g only
};

// What the host reads back of an instance's state at the end of a solve (the full state is
// ~4.7 KB per instance; this is what the statistics, the refinement and the byte counts use).
struct StateStat {
  int status;
  int iter;
  int ngrad;
  int pad;
  double chi2;
  double gg;
  double g0norm;
  double bytes[KK_COUNT];
};

// One instance of a batched pack (internal whitened field -> caller's external field).
struct PackEntry {
  const void* in;   // internal field
  const void* sq;   // sqrt S table (internal layout), nullable
  void* out;        // [C][n][n/2+1] external field
};

// Elementwise conversion job of the float64 refinement (counts in real elements).
struct CvtJob {
  const void* src;
  void* dst;
  int64_t n;
  int op;   // CVT_*
  int pad;
};
enum { CVT_F32_F64 = 0, CVT_F64_F32 = 1, CVT_ADD_F32_F64 = 2 };

// Right-hand side of a float32 correction solve from a float64 gradient g (L complex
// elements, internal layout): rhs = -g rounded to float32, and per block the partial sums of
// |g|^2 in the solver's whitened metric (1 / P_k per element when ainv is given).
struct RhsJob {
  const double* g;
  const double* ainv;
  float* rhs;
  double* part;   // [gridDim.x]
  int64_t L;
};

// ------------------------------------------------------------------------ catalog response
// A galaxy of a catalog in fine-grid coordinates rho = 2 r (the fine grid has N = 2n points per
// side): integer cell and fraction, so that kernel offsets keep full float32 precision.
constexpr int CAT_W = 8;      // interpolation kernel width in fine-grid points
constexpr int CAT_H = CAT_W / 2;
constexpr int CAT_D = CAT_W + 1;   // fine points per axis around a galaxy's cell: cell - H .. cell + H
constexpr int CAT_REC = 12;   // floats of a galaxy record: CAT_D weights along y, the x fraction, 0, 0
constexpr int CAT_TS = 16;    // fine-grid tile side of the spreading pass
constexpr float CAT_BETA = 2.30f * CAT_W;   // exponential-of-semicircle shape for oversampling 2

// One catalog instance: galaxies sorted by fine-grid cell, their windows, tables and the
// buffers of its fine-grid passes.
struct CatDesc {
  int n, N, c, ngal;
  int tiles;              // fine-grid tiles per side (N / CAT_TS)
  int nrowPart;           // row-partial slots of the coarse grid (c n / RB_MIN)
  const int2* cell;       // [ngal] fine-grid cell (y, x) of each galaxy
  const float4* rec;      // [ngal][CAT_REC / 4]: phi at the fine rows cell - H .. cell + H, and the
                          // fraction fx of rho_x (the x weights are phi(fx + H - t))
  const int* cellStart;   // [N * N + 1] first sorted galaxy of each fine cell (row-major)
  const float* e;         // [c][ngal] measurements (sorted), solver gradients only
  const float* wgt;       // [ngal] inverse noise variance (sorted)
  const float* T;         // [c][n][n/2] coarse internal layout: prior (or 1) x (N/n) / deconvolution
  const float* aTab;      // prior weight of the solver variable, nullable -> 1
  void* y2;               // fine-grid half-plane field, internal layout (complex float)
  float* u;               // [c][N][N] fine-grid map
  float* v;               // [c][N][N] spread residuals (may be u: interpolation is done first)
  float* r;               // [ngal][c] residuals or field values (sorted, components interleaved)
  double* partI;          // [ceil(ngal / NT)] chi^2 partials of the interpolation
  Job* jfwd;              // this instance's fine-grid forward and adjoint jobs
  Job* jadj;
};

// One field's band-statistic job.
struct BandJob {
  const void* f;          // field, internal layout
  const void* f2;         // nullable: the statistic is taken of f - f2
  const void* sq;         // sqrt S table (raw fields)
  const void* aw;         // solver-variable weight P_k (preconditioned solution), nullable
  const int32_t* bandI;   // internal band table (-1 = none / not free)
  const double* theta;    // [nbands] (device)
  double* part;           // [nblk][nbands]
  double* E;              // [nbands] output (device)
  int64_t L;
  int nbands;
  int raw;                // 0: whitened field, E_l; 1: raw field, E_l; 2: whitened field, band power sum S |w|^2
};

// Static per-instance description of a solve.
// The 2m + 2 vectors of an instance (w, g, p_0..p_{m-1}, Dp_0..Dp_{m-1}) are stored one
// after the other, vstride complex elements apart (each vector padded by an odd multiple of
// 256 B so the streams of a pass do not share offsets modulo a large power of two).
struct InstDesc {
  void* X;          // vector v at X + v * vstride
  void* y;          // transform intermediate
  const void* d;
  const void* W;
  const void* sq;   // scale table (internal layout, real): sqrt S, or sqrt(S P) when preconditioned
  const void* aTab; // preconditioned solves: P_k = 1 / (1 + S_k <W>); else null
  const void* ainv; // preconditioned solves: 1 / P_k (whitened gradient norm); else null
  const void* rhs;  // correction solves of a float64 refinement: the gradient is D v - rhs
                    // (the chain runs on zero data and pass A subtracts rhs); else null
  double* partChain;   // [PK_COUNT][pstride]
  double* partA;       // [nblkA][NDOT]
  int* statusOut;      // compact per-instance status for host polling
  int n, c;
  int64_t L;           // complex elements per vector
  int64_t vstride;     // complex elements between vectors
  int NV;              // vectors per instance (2m + 2)
  int nchunk;          // work-groups of a vector pass
  int pstride;
  int m;
  int esize;           // bytes of one complex element
  int maxIter;
  int refreshEvery;
  double tol;
  double dchi2Tol;
  double vbytes;       // bytes of one vector
};

}  // namespace wf
