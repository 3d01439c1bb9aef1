// Device-resident batched L-BFGS (sec. 2.2) and the small kernels around it.
//
// One iteration of an instance (every kernel skips instances that have stopped):
//   chain    curvature product Dp = D p of the new direction, or the exact gradient
//            (transform passes, wf_chain.hpp); in curvature mode it also returns the dots
//            of Dp with the stored g and with the kept Dp_j;
//   passA    only after an exact-gradient evaluation: dots of the new g with the kept
//            pairs (otherwise these come from the previous pass B and a one-step update);
//            g.g alone when the gradient confirms a stop, the dots following in a
//            transform-free iteration if the confirmation fails;
//   coef     step length alpha = -g.p / p.Dp of the exact line search of a quadratic
//            (eq. eq_chib), Gram entries of the new pair, stop test after an exact gradient,
//            and the two-loop recursion run on coefficients: the direction is a combination
//            of the kept p_i, Dp_i and g (s_i = alpha_i p_i, y_i = alpha_i Dp_i);
//   passB    applies the pending step to g (g += alpha Dp), forms the direction in the next
//            history slot and measures g.g, g.p and the dots of g with the pairs; when told
//            to, brings w up to date;
//   postB    stop test on the measured g, choice of the next chain (curvature product,
//            exact-gradient refresh, a flush-only iteration, or none) and the remaining Gram
//            entries.
// The iterate is updated lazily: w is stored at the last flush and the current iterate is
// w + sum alpha_i p_i over the pending pairs, whose vectors are the newest kept ones.  Pass B
// flushes when the direction it writes would overwrite a pending pair (every m iterations)
// and before an exact-gradient refresh or a stop.  (g is not deferred: forming the direction
// from a stale g plus pending Dp terms that cancel it would lose the direction's accuracy in
// float32.)  Per iteration the vector traffic is about 3m + 11 field vectors (m kept pairs),
// plus 2 at a flush.
#pragma once
#include "wf_chain.hpp"

namespace wf {

template <typename T> struct VecT;
template <> struct VecT<float> { using type = float4; static constexpr int W = 4; };
template <> struct VecT<double> { using type = double2; static constexpr int W = 2; };

template <typename V> __device__ __forceinline__ double vdot(const V& a, const V& b);
template <> __device__ __forceinline__ double vdot<float4>(const float4& a, const float4& b) {
  return (double)a.x * b.x + (double)a.y * b.y + (double)a.z * b.z + (double)a.w * b.w;
}
template <> __device__ __forceinline__ double vdot<double2>(const double2& a, const double2& b) {
  return a.x * b.x + a.y * b.y;
}
__device__ __forceinline__ float4 vaxpy(float a, const float4& x, const float4& y) {
  return make_float4(y.x + a * x.x, y.y + a * x.y, y.z + a * x.z, y.w + a * x.w);
}
__device__ __forceinline__ double2 vaxpy(double a, const double2& x, const double2& y) {
  return make_double2(y.x + a * x.x, y.y + a * x.y);
}
__device__ __forceinline__ float4 vscale(float a, const float4& x) { return make_float4(a * x.x, a * x.y, a * x.z, a * x.w); }
// |g|^2 in the whitened norm of a preconditioned solve: sum over the complex elements of the
// vector element e of |g_k|^2 / P_k (ainv = 1 / P)
__device__ __forceinline__ double wnorm2(const float4& g, const float* ainv, uint32_t e) {
  const float2 a = gld(reinterpret_cast<const float2*>(ainv), e);
  return (double)a.x * ((double)g.x * g.x + (double)g.y * g.y) + (double)a.y * ((double)g.z * g.z + (double)g.w * g.w);
}
__device__ __forceinline__ double wnorm2(const double2& g, const double* ainv, uint32_t e) {
  return gld(ainv, e) * (g.x * g.x + g.y * g.y);
}
__device__ __forceinline__ double2 vscale(double a, const double2& x) { return make_double2(a * x.x, a * x.y); }
template <typename V> __device__ __forceinline__ V vzero();
template <> __device__ __forceinline__ float4 vzero<float4>() { return make_float4(0.f, 0.f, 0.f, 0.f); }
template <> __device__ __forceinline__ double2 vzero<double2>() { return make_double2(0.0, 0.0); }

constexpr int NDOT = 5 * MMAX + 1;          // partials per block of k_passA


// keeps the compiler from moving the loads of the next stream above this point, so a
// work-group streams one vector at a time (measurably better HBM efficiency than issuing
// the loads of every stream element by element)
__device__ __forceinline__ void stream_fence() { asm volatile("" ::: "memory"); }

// ------------------------------------------------------------------------ init
template <typename T>
__global__ void k_zero(InstDesc* desc, int batch) {
  const int i = blockIdx.y;
  if (i >= batch) return;
  using V = typename VecT<T>::type;
  constexpr int VW = VecT<T>::W;
  const InstDesc& D = desc[i];
  V* X = reinterpret_cast<V*>(D.X);   // vector 0 is w
  const int64_t nv = D.L * 2 / VW;
  V z;
  if constexpr (VW == 4) z = make_float4(0.f, 0.f, 0.f, 0.f); else z = make_double2(0.0, 0.0);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nv; e += (int64_t)gridDim.x * blockDim.x)
    X[e] = z;
}

__device__ __forceinline__ char* vec_ptr(const InstDesc& D, int v) {
  return reinterpret_cast<char*>(D.X) + (size_t)v * D.vstride * D.esize;
}

// slots of the kept pairs, newest first
__device__ __forceinline__ int slot_of(int head, int j, int m) { return (head - j + 2 * m) % m; }

__device__ __forceinline__ void make_job(Job& jb, const InstDesc& D, int mode, int slot, uint32_t dpMask) {
  jb.mode = mode;
  jb.boost_band = -1;
  jb.sim = 0;
  jb.boost_factor = 1.0;
  jb.seed = 0;
  jb.y = D.y;
  jb.d = D.d;
  jb.W = D.W;
  jb.sIn = D.sq;
  jb.sOut = D.sq;
  jb.aTab = D.aTab;
  jb.band = nullptr;
  jb.draws = nullptr;
  jb.xout = nullptr;
  jb.part = D.partChain;
  jb.pstride = D.pstride;
  jb.gvec = nullptr;
  jb.dpBase = nullptr;
  jb.dpStride = D.vstride;
  jb.dpMask = 0;
  if (mode == CM_HV) {
    char* p = vec_ptr(D, 2 + slot);
    jb.vin = p;
    jb.vadd = p;
    jb.vout = vec_ptr(D, 2 + D.m + slot);
    jb.gvec = vec_ptr(D, 1);
    jb.dpBase = vec_ptr(D, 2 + D.m);
    jb.dpMask = dpMask;
  } else {
    jb.vin = vec_ptr(D, 0);    // w
    jb.vadd = vec_ptr(D, 0);
    jb.vout = vec_ptr(D, 1);   // g
  }
}

__device__ __forceinline__ void add_chain_bytes(LbState& S, const InstDesc& D, int mode, int extra) {
  const double V = D.vbytes;
  S.bytes[KK_COLINV] += 2.0 * V;                              // read field, write intermediate
  S.bytes[KK_ROW] += 2.0 * V + (mode == CM_GRAD ? V : 0.0);    // intermediate in/out (+ data)
  S.bytes[KK_COLFWD] += (3.0 + extra) * V;                    // intermediate, added term, output (+ dots)
}

__global__ void k_init(InstDesc* desc, LbState* st, Job* jobs, int batch) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch) return;
  LbState& S = st[i];
  const InstDesc& D = desc[i];
  S.status = ST_RUNNING;
  S.iter = 0;
  S.nhist = 0;
  S.m = D.m;
  S.head = D.m - 1;
  S.newslot = 0;
  S.pending = 0;
  S.npend = 0;
  S.npendB = 0;
  S.flushB = 0;
  S.dirB = 0;
  S.after = 0;
  S.chainMode = CM_GRAD;
  S.lastWasGrad = 0;
  S.ngrad = 0;
  S.lastGradIter = 0;
  S.doB = 0;
  S.g0norm = -1.0;
  S.gg = 0.0;
  S.chi2 = 0.0;
  S.dchi2 = 0.0;
  S.gdotp = 0.0;
  S.pDp = 0.0;
  S.rho = 0.0;
  S.beta = 0.0;
  S.doDir = 0;
  S.confirm = 0;
  for (int k = 0; k < KK_COUNT; ++k) S.bytes[k] = 0.0;
  S.bytes[KK_MISC] += D.vbytes;   // zeroing w
  add_chain_bytes(S, D, CM_GRAD, 0);
  make_job(jobs[i], D, CM_GRAD, 0, 0u);
  D.statusOut[0] = ST_RUNNING;
}

// ------------------------------------------------------------------------ pass A (dots only)
// After an exact gradient: g.g, g.p_j, g.Dp_j for the kept pairs, one slot at a time.  An
// exact gradient that confirms a stop needs g.g only; the dots follow in a CM_DOTS
// iteration if the confirmation fails.
template <typename T, int M, int PASS_U>
__global__ __launch_bounds__(NT) void k_passA(const InstDesc* __restrict__ desc, const LbState* __restrict__ st) {
  const int i = rev_instance();
  const LbState& S = st[i];
  if (S.status != ST_RUNNING || !(S.chainMode == CM_GRAD || S.chainMode == CM_DOTS)) return;
  const InstDesc& D = desc[i];
  using V = typename VecT<T>::type;
  constexpr int VW = VecT<T>::W;
  __shared__ double red[NT / 64][NDOT];
  const int nh = (S.chainMode == CM_GRAD && S.confirm) ? 0 : S.nhist, head = S.head;
  // element offsets (units of V) from the instance's vector block, 32-bit
  const uint32_t nvec = (uint32_t)(D.L * 2 / VW);
  const uint32_t vs = (uint32_t)(D.vstride * 2 / VW);
  const uint32_t e0 = blockIdx.x * (uint32_t)(NT * PASS_U) + threadIdx.x;
  const V* X = reinterpret_cast<const V*>(D.X);
  const uint32_t og = vs, oP = 2 * vs, oD = (2 + M) * vs;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  bool ok[PASS_U];
  V gv[PASS_U];
  double gg = 0.0;
  const T* ainv = reinterpret_cast<const T*>(D.ainv);
  // a correction solve's exact gradient is D v - rhs: the chain ran on zero data
  const V* R = (S.chainMode == CM_GRAD) ? reinterpret_cast<const V*>(D.rhs) : nullptr;
#pragma unroll
  for (int u = 0; u < PASS_U; ++u) {
    const uint32_t e = e0 + (uint32_t)u * NT;
    ok[u] = e < nvec;
    if (ok[u]) {
      gv[u] = gld(X, og + e);
      if (R) {
        gv[u] = vaxpy(T(-1), gld(R, e), gv[u]);
        gst(reinterpret_cast<V*>(D.X), og + e, gv[u]);
      }
      gg += ainv ? wnorm2(gv[u], ainv, e) : vdot(gv[u], gv[u]);
    }
  }
  {
    const double a = wave_sum(gg);
    if (lane == 0) red[wv][2 * M] = a;
  }
#pragma unroll
  for (int j = 0; j < M; ++j) {
    stream_fence();
    double a0 = 0.0, a1 = 0.0;
    if (j < nh) {
      const uint32_t sp = (uint32_t)slot_of(head, j, M) * vs;
      V pv[PASS_U], dv[PASS_U];
#pragma unroll
      for (int u = 0; u < PASS_U; ++u)
        if (ok[u]) pv[u] = gld(X, oP + sp + e0 + (uint32_t)u * NT);
#pragma unroll
      for (int u = 0; u < PASS_U; ++u)
        if (ok[u]) dv[u] = gld(X, oD + sp + e0 + (uint32_t)u * NT);
#pragma unroll
      for (int u = 0; u < PASS_U; ++u) {
        if (ok[u]) {
          a0 += vdot(gv[u], pv[u]);
          a1 += vdot(gv[u], dv[u]);
        }
      }
    }
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    if (lane == 0) {
      red[wv][j] = a0;
      red[wv][M + j] = a1;
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * M + 1) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) t += red[k][threadIdx.x];
    D.partA[(int64_t)blockIdx.x * NDOT + threadIdx.x] = t;
  }
}

// sum of `cnt` partial rows (stride `stride`) of column t, 4 threads per column
__device__ __forceinline__ void reduce_columns(const double* part, int nblk, int stride, int ncol, double* sums,
                                               double (*part4)[NDOT]) {
  const int t = threadIdx.x & 63, q = threadIdx.x >> 6;
  if (t < ncol) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int b = q;
    for (; b + 12 < nblk; b += 16) {
      a0 += part[(int64_t)b * stride + t];
      a1 += part[(int64_t)(b + 4) * stride + t];
      a2 += part[(int64_t)(b + 8) * stride + t];
      a3 += part[(int64_t)(b + 12) * stride + t];
    }
    for (; b < nblk; b += 4) a0 += part[(int64_t)b * stride + t];
    part4[q][t] = (a0 + a1) + (a2 + a3);
  }
  __syncthreads();
  if (threadIdx.x < ncol) sums[threadIdx.x] = (part4[0][threadIdx.x] + part4[1][threadIdx.x]) +
                                              (part4[2][threadIdx.x] + part4[3][threadIdx.x]);
  __syncthreads();
}

// whole-state copy between global memory and LDS by every thread of the work-group
__device__ __forceinline__ void copy_state(LbState* dst, const LbState* src) {
  static_assert(sizeof(LbState) % 8 == 0, "state size");
  const uint64_t* s = reinterpret_cast<const uint64_t*>(src);
  uint64_t* d = reinterpret_cast<uint64_t*>(dst);
  for (int k = threadIdx.x; k < (int)(sizeof(LbState) / 8); k += blockDim.x) d[k] = s[k];
}

// ------------------------------------------------------------------------ coefficients
// 256 threads per instance.  Thread 0 folds the new pair into the Gram blocks (or takes the
// exact-gradient dots) and runs the stop test; all threads then copy the Gram blocks in
// history order (position 0 = newest pair) into LDS, and thread 0 runs the two-loop recursion
// on those with every index known at compile time, so its coefficient arrays stay in registers.
template <int M>
__device__ __forceinline__ int coef_update(const InstDesc& D, LbState& S, Job& job, int mode, const double* chs,
                                           const double* sums);
template <int M>
__device__ __forceinline__ void coef_twoloop(const InstDesc& D, LbState& S, const double (*qPD)[M],
                                             const double (*qDD)[M], const double* qgP, const double* qgD,
                                             const double* qal);

template <int M>
__global__ __launch_bounds__(256) void k_coef(const InstDesc* __restrict__ desc, LbState* st, Job* jobs) {
  const int i = blockIdx.x;
  LbState& Sg = st[i];
  if (Sg.status != ST_RUNNING) return;
  const InstDesc& D = desc[i];
  const int mode = Sg.chainMode;
  if (mode == CM_FLUSH) {   // no transform this iteration: pass B only brings w up to date
    if (threadIdx.x == 0) {
      Sg.doB = 1;
      Sg.dirB = 0;
      Sg.flushB = 1;
      Sg.npendB = Sg.npend;
      Sg.bytes[KK_PASSB] += D.vbytes * (2.0 * Sg.nhist + 1.0 + 2.0);
    }
    return;
  }
  __shared__ __align__(16) LbState S;
  copy_state(&S, &Sg);
  __shared__ double sums[NDOT];
  __shared__ double part4[4][NDOT];
  __shared__ double chs[3 + MMAX + 2];
  __shared__ double qPD[M][M], qDD[M][M], qgP[M], qgD[M], qal[M];
  __shared__ int run;
  const int ncol = (D.n / 2) / TB, nrow = D.c * D.n / RB_MIN;
  if (mode == CM_GRAD || mode == CM_DOTS) reduce_columns(D.partA, D.nchunk, NDOT, 2 * M + 1, sums, part4);
  // chain partial sums: one wave per kind, fixed-order lane sums and a fixed shuffle tree
  {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int t = wv; t < 3 + M + 2; t += (int)(blockDim.x >> 6)) {
      int kind = -1, nb = 0;
      if (t < 3 + M) {
        if (mode == CM_HV) {
          kind = PK_VO + t;
          nb = ncol;
        }
      } else if (mode == CM_GRAD) {
        kind = (t == 3 + M) ? PK_PRIOR : PK_RES;
        nb = (t == 3 + M) ? ncol : nrow;
      }
      double a = 0.0;
      if (kind >= 0)
        for (int b = lane; b < nb; b += 64) a += D.partChain[kind * D.pstride + b];
      a = wave_sum(a);
      if (lane == 0) chs[t] = a;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) run = coef_update<M>(D, S, jobs[i], mode, chs, sums);
  __syncthreads();
  if (run) {   // (uniform: read from LDS after the barrier)
    const int nh = S.nhist, head = S.head;
    for (int t = threadIdx.x; t < M * M; t += blockDim.x) {
      const int j = t / M, u = t % M;
      const bool in = j < nh && u < nh;
      const int sj = slot_of(head, j, M), su = slot_of(head, u, M);
      qPD[j][u] = in ? S.PD[sj][su] : 0.0;
      qDD[j][u] = in ? S.DD[sj][su] : 0.0;
    }
    for (int t = threadIdx.x; t < M; t += blockDim.x) {
      const bool in = t < nh;
      const int sj = slot_of(head, t, M);
      qgP[t] = in ? S.gP[sj] : 0.0;
      qgD[t] = in ? S.gD[sj] : 0.0;
      qal[t] = in ? S.alpha[sj] : 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) coef_twoloop<M>(D, S, qPD, qDD, qgP, qgD, qal);
  }
  __syncthreads();
  copy_state(&Sg, &S);
}

// Folds the last curvature product into the state (CM_HV) or takes the exact gradient's
// dots (CM_GRAD); returns 1 when a new direction is to be formed.
template <int M>
__device__ __forceinline__ int coef_update(const InstDesc& D, LbState& S, Job& job, int mode, const double* chs,
                                           const double* sums) {
  int status = ST_RUNNING;
  if (mode == CM_HV) {
    const double pDp = chs[0], DpDp = chs[1], DpG = chs[2];
    if (!(pDp > 0.0) || !isfinite(pDp) || !isfinite(DpDp)) {
      S.status = 2;
      D.statusOut[0] = 2;
      job.mode = CM_NONE;
      S.chainMode = CM_NONE;
      S.doB = 0;
      return 0;
    }
    const int nh = S.nhist, head = S.head, ns = S.newslot;
    const double alpha = -S.gdotp / pDp;
    // Gram entries of the new pair (p_k, Dp_k) in slot ns against the kept pairs: p_k . Dp_j
    // from the previous pass B, p_j . Dp_k = p_k . Dp_j (D is symmetric), Dp_k . Dp_j
    // measured by the chain
    for (int j = 0; j < nh; ++j) {
      const int sj = slot_of(head, j, M);
      if (sj == ns) continue;
      const double pd = S.pkD[sj], dd = chs[3 + sj];
      S.PD[ns][sj] = pd;
      S.PD[sj][ns] = pd;
      S.DD[ns][sj] = dd;
      S.DD[sj][ns] = dd;
      // one-step update of the dots of g_{k+1} = g_k + alpha Dp_k with the kept pairs
      S.gP[sj] += alpha * pd;
      S.gD[sj] += alpha * dd;
    }
    S.PD[ns][ns] = pDp;
    S.DD[ns][ns] = DpDp;
    S.gP[ns] = S.gdotp + alpha * pDp;
    S.gD[ns] = DpG + alpha * DpDp;
    S.alpha[ns] = alpha;
    S.head = ns;
    S.nhist = nh + 1 < M ? nh + 1 : M;
    S.pending = 1;
    S.npend += 1;
    S.pDp = pDp;
    S.dchi2 = 4.0 * (alpha * S.gdotp + 0.5 * alpha * alpha * pDp);
    S.chi2 += S.dchi2;
    S.iter += 1;
    S.lastWasGrad = 0;
  } else if (mode == CM_GRAD || mode == CM_DOTS) {
    const int nh = S.nhist, head = S.head;
    const bool dots = mode == CM_DOTS || !S.confirm;   // pass A took the dots with the kept pairs
    if (mode == CM_GRAD) {
      S.chi2 = 2.0 * chs[3 + M] + chs[4 + M];
      S.ngrad += 1;
      S.lastGradIter = S.iter;
      S.pending = 0;
      S.npend = 0;   // an exact gradient is only taken at a flushed iterate
      S.lastWasGrad = 1;
    }
    S.bytes[KK_PASSA] += D.vbytes * (1.0 + (dots ? 2.0 * nh : 0.0) + (mode == CM_GRAD && D.rhs ? 2.0 : 0.0));
    if (dots) {
      for (int j = 0; j < nh; ++j) {
        const int sj = slot_of(head, j, M);
        S.gP[sj] = sums[j];
        S.gD[sj] = sums[M + j];
      }
    }
    const double gg = sums[2 * M];
    S.gg = gg;
    if (mode == CM_GRAD) {
      if (S.g0norm < 0.0) S.g0norm = sqrt(gg);
      const double g0 = S.g0norm;
      const double rel = g0 > 0.0 ? sqrt(gg) / g0 : 0.0;
      if (!isfinite(gg) || !isfinite(S.chi2)) status = 2;
      else if (g0 == 0.0 || rel <= D.tol) status = 0;
      else if (S.iter >= D.maxIter) status = 1;
      if (status == ST_RUNNING && !dots) {   // the confirmation failed: take the dots first
        S.confirm = 0;
        S.chainMode = CM_DOTS;
        job.mode = CM_NONE;
        S.doB = 0;
        return 0;
      }
    }
    S.confirm = 0;
  }
  if (status != ST_RUNNING) {
    S.status = status;
    D.statusOut[0] = status;
    job.mode = CM_NONE;
    S.chainMode = CM_NONE;
    S.doB = 0;
    return 0;
  }
  return 1;
}

// Two-loop recursion in the coefficients of (p_0..p_{M-1}, Dp_0..Dp_{M-1}, g) by history
// position; entries at positions >= nhist are zero in the LDS copies.
template <int M>
__device__ __forceinline__ void coef_twoloop(const InstDesc& D, LbState& S, const double (*qPD)[M],
                                             const double (*qDD)[M], const double* qgP, const double* qgD,
                                             const double* qal) {
  const int nh = S.nhist, head = S.head;
  double cP[M], cD[M], a[M], rho[M];
  double cg = 1.0;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    cP[j] = 0.0;
    cD[j] = 0.0;
    a[j] = 0.0;
    rho[j] = 0.0;
  }
#pragma unroll
  for (int j = 0; j < M; ++j) {   // newest to oldest
    if (j < nh) {
      const double al = qal[j];
      rho[j] = 1.0 / (al * al * qPD[j][j]);
      double sq = cg * qgP[j];
#pragma unroll
      for (int t = 0; t < j; ++t) sq += cD[t] * qPD[j][t];
      a[j] = rho[j] * al * sq;
      cD[j] -= a[j] * al;
    }
  }
  if (nh > 0) {
    const double gam = qPD[0][0] / qDD[0][0];
    cg *= gam;
#pragma unroll
    for (int t = 0; t < M; ++t) cD[t] *= gam;
  }
#pragma unroll
  for (int j = M - 1; j >= 0; --j) {   // oldest to newest
    if (j < nh) {
      const double al = qal[j];
      double yr = cg * qgD[j];
#pragma unroll
      for (int t = 0; t < M; ++t) yr += cD[t] * qDD[j][t] + cP[t] * qPD[t][j];
      const double beta = rho[j] * al * yr;
      cP[j] += al * (a[j] - beta);
    }
  }
#pragma unroll
  for (int j = 0; j < M; ++j) {   // every slot: the kept pairs' coefficients, zero for the others
    const int sj = slot_of(head, j, M);
    S.coef[sj] = j < nh ? -cP[j] : 0.0;
    S.coef[MMAX + sj] = j < nh ? -cD[j] : 0.0;
  }
  S.coef[2 * MMAX] = -cg;
  S.newslot = (head + 1) % M;
  S.doB = 1;
  S.dirB = 1;
  // bring w up to date in this pass B when the direction would overwrite a pending pair
  S.flushB = (nh == M && S.npend == M) ? 1 : 0;
  S.npendB = S.npend;
  S.bytes[KK_PASSB] += D.vbytes * (2.0 * nh + 2.0 + (S.pending ? 1.0 : 0.0) + (S.flushB ? 2.0 : 0.0));
}

// ------------------------------------------------------------------------ pass B
// One kernel for the streaming pass and, when the history wraps or before a refresh or a stop,
// the flush of the pending steps into w (a run-time branch: a second launch per iteration for
// the flushing instances cost more than the extra registers, 136 instead of 110 VGPRs).
template <typename T, int M, int PASS_U>
__global__ __launch_bounds__(NT) void k_passB(const InstDesc* __restrict__ desc, const LbState* __restrict__ st) {
  const int i = rev_instance();
  const LbState& S = st[i];
  if (S.status != ST_RUNNING || !S.doB) return;
  const bool flush = S.flushB != 0;
  const InstDesc& D = desc[i];
  using V = typename VecT<T>::type;
  constexpr int VW = VecT<T>::W;
  __shared__ double red[NT / 64][NDOT];
  const int nh = S.nhist, head = S.head, ns = S.newslot, pend = S.pending, np = S.npendB, dir = S.dirB;
  const T alh = pend ? T(S.alpha[head]) : T(0);
  T cP[M], cD[M], al[M];
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const int sj = slot_of(head, j, M);
    al[j] = j < np ? T(S.alpha[sj]) : T(0);
    cP[j] = dir ? T(S.coef[sj]) : T(0);
    cD[j] = dir ? T(S.coef[MMAX + sj]) : T(0);
  }
  const T cg = dir ? T(S.coef[2 * MMAX]) : T(0);
  // element offsets (units of V) from the instance's vector block, 32-bit
  const uint32_t nvec = (uint32_t)(D.L * 2 / VW);
  const uint32_t vs = (uint32_t)(D.vstride * 2 / VW);
  const uint32_t e0 = blockIdx.x * (uint32_t)(NT * PASS_U) + threadIdx.x;
  V* X = reinterpret_cast<V*>(D.X);
  const uint32_t ow = 0, og = vs, oP = 2 * vs, oD = (2 + M) * vs;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  bool ok[PASS_U];
  V gv[PASS_U], acc[PASS_U];
  V wa[PASS_U];
#pragma unroll
  for (int u = 0; u < PASS_U; ++u) {
    const uint32_t e = e0 + (uint32_t)u * NT;
    ok[u] = e < nvec;
    if (ok[u]) gv[u] = gld(X, og + e);
    wa[u] = vzero<V>();
  }
  if (pend) {   // the step of the newest pair on g: g += alpha Dp
    const uint32_t sh = (uint32_t)head * vs;
#pragma unroll
    for (int u = 0; u < PASS_U; ++u) {
      const uint32_t e = e0 + (uint32_t)u * NT;
      if (ok[u]) {
        gv[u] = vaxpy(alh, gld(X, oD + sh + e), gv[u]);
        gst(X, og + e, gv[u]);
      }
    }
  }
  double gg = 0.0;
  const T* ainv = reinterpret_cast<const T*>(D.ainv);
#pragma unroll
  for (int u = 0; u < PASS_U; ++u) {
    if (ok[u]) {
      gg += ainv ? wnorm2(gv[u], ainv, e0 + (uint32_t)u * NT) : vdot(gv[u], gv[u]);
      acc[u] = vscale(cg, gv[u]);
    }
  }
  {
    const double a = wave_sum(gg);
    if (lane == 0) red[wv][2 * M] = a;
  }
  // one kept pair at a time: accumulate the direction (and the pending steps of w), dots of
  // g with the pair.  The pairs are read with the non-temporal hint: a batch's history is
  // far larger than any cache, and streaming it past the caches took pass B from 5.14 to
  // 5.5 TB/s on the 127-map 512^2 shear batch.
#pragma unroll
  for (int j = 0; j < M; ++j) {
    stream_fence();
    double a0 = 0.0, a1 = 0.0;
    if (j < nh) {
      const uint32_t sp = (uint32_t)slot_of(head, j, M) * vs;
      V pv[PASS_U], dv[PASS_U];
#pragma unroll
      for (int u = 0; u < PASS_U; ++u)
        if (ok[u]) pv[u] = gldnt(X, oP + sp + e0 + (uint32_t)u * NT);
#pragma unroll
      for (int u = 0; u < PASS_U; ++u)
        if (ok[u]) dv[u] = gldnt(X, oD + sp + e0 + (uint32_t)u * NT);
#pragma unroll
      for (int u = 0; u < PASS_U; ++u) {
        if (ok[u]) {
          a0 += vdot(gv[u], pv[u]);
          a1 += vdot(gv[u], dv[u]);
          acc[u] = vaxpy(cP[j], pv[u], acc[u]);
          acc[u] = vaxpy(cD[j], dv[u], acc[u]);
          if (flush && j < np) wa[u] = vaxpy(al[j], pv[u], wa[u]);
        }
      }
    }
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    if (lane == 0) {
      red[wv][j] = a0;
      red[wv][M + j] = a1;
    }
  }
  stream_fence();
  if (flush) {   // w += sum alpha p over the pending pairs
#pragma unroll
    for (int u = 0; u < PASS_U; ++u) {
      const uint32_t e = e0 + (uint32_t)u * NT;
      if (ok[u]) gst(X, ow + e, vaxpy(T(1), wa[u], gld(X, ow + e)));
    }
  }
  double gp = 0.0;
  if (dir) {
#pragma unroll
    for (int u = 0; u < PASS_U; ++u) {
      if (ok[u]) {
        gst(X, oP + (uint32_t)ns * vs + e0 + (uint32_t)u * NT, acc[u]);
        gp += vdot(gv[u], acc[u]);
      }
    }
  }
  {
    const double a = wave_sum(gp);
    if (lane == 0) red[wv][2 * M + 1] = a;
  }
  __syncthreads();
  if (threadIdx.x < 2 * M + 2) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) t += red[k][threadIdx.x];
    D.partA[(int64_t)blockIdx.x * NDOT + threadIdx.x] = t;
  }
}

// ------------------------------------------------------------------------ post B
template <int M>
__device__ __forceinline__ int postB_scalar(const InstDesc& D, LbState& S, Job& job, const double* sums);

template <int M>
__global__ __launch_bounds__(256) void k_postB(const InstDesc* __restrict__ desc, LbState* st, Job* jobs) {
  const int i = blockIdx.x;
  LbState& Sg = st[i];
  if (Sg.status != ST_RUNNING || !Sg.doB) return;
  const InstDesc& D = desc[i];
  // the scalar part runs in one thread on an LDS copy of the state
  __shared__ __align__(16) LbState S;
  copy_state(&S, &Sg);
  __shared__ double sums[NDOT];
  __shared__ double part4[4][NDOT];
  __shared__ int next;
  reduce_columns(D.partA, D.nchunk, NDOT, 2 * M + 2, sums, part4);   // (synchronises)
  if (threadIdx.x == 0) next = postB_scalar<M>(D, S, jobs[i], sums);
  __syncthreads();
  if (next == CM_HV) {   // (uniform) p . Dp_j of the new direction, one kept pair per thread
    const int nh = S.nhist, head = S.head;
    if ((int)threadIdx.x < nh) {
      const int sj = slot_of(head, threadIdx.x, M);
      // from its coefficients: p = sum c b, b in {p_i, Dp_i, g}
      double v = S.coef[2 * MMAX] * S.gD[sj];
      for (int t = 0; t < nh; ++t) {
        const int st2 = slot_of(head, t, M);
        v += S.coef[st2] * S.PD[st2][sj] + S.coef[MMAX + st2] * S.DD[st2][sj];
      }
      S.pkD[sj] = v;
    }
  }
  __syncthreads();
  copy_state(&Sg, &S);
}

// Stop test and next chain mode; returns that mode (CM_NONE once stopped).  For CM_HV the
// caller fills pkD with the new direction's dots with the kept Dp.
template <int M>
__device__ __forceinline__ int postB_scalar(const InstDesc& D, LbState& S, Job& job, const double* sums) {
  const int nh = S.nhist, head = S.head, ns = S.newslot, dir = S.dirB;
  S.doB = 0;
  S.pending = 0;
  if (S.flushB) S.npend = 0;
  int sl[M];
  for (int j = 0; j < M; ++j) sl[j] = slot_of(head, j, M);
  // the measured dots of the current gradient replace the one-step updates
  for (int j = 0; j < nh; ++j) {
    S.gP[sl[j]] = sums[j];
    S.gD[sl[j]] = sums[M + j];
  }
  const double gg = sums[2 * M], gp = dir ? sums[2 * M + 1] : 0.0;
  S.gg = gg;
  if (dir) S.gdotp = gp;
  const double g0 = S.g0norm;
  const double rel = g0 > 0.0 ? sqrt(gg) / g0 : 0.0;
  int next = CM_HV, status = ST_RUNNING;
  if (S.after != 0) {   // a flush-only iteration carrying an earlier decision
    if (S.after == 1) next = CM_GRAD;
    else status = S.after - 2;
    S.after = 0;
  } else {
    S.confirm = 0;
    if (!isfinite(gg) || !isfinite(gp)) {
      status = 2;
    } else if (rel <= D.tol) {
      next = CM_GRAD;                 // confirm with the exact gradient
      S.confirm = 1;
    } else if (S.iter >= D.maxIter) {
      status = 1;
    } else if (D.dchi2Tol > 0.0 && S.iter > 0 && fabs(S.dchi2) < D.dchi2Tol) {
      status = 0;
    } else if (!(gp < 0.0)) {
      next = CM_GRAD;                 // not a descent direction (round-off): refresh
    } else if (D.refreshEvery > 0 && S.iter - S.lastGradIter >= D.refreshEvery) {
      next = CM_GRAD;
    }
    // a refresh or a stop needs the current iterate in w: apply the pending steps first
    if (S.npend > 0 && (next == CM_GRAD || status == 0 || status == 1)) {
      S.after = next == CM_GRAD ? 1 : 2 + status;
      next = CM_FLUSH;
      status = ST_RUNNING;
    }
  }
  if (status != ST_RUNNING) {
    S.status = status;
    D.statusOut[0] = status;
    job.mode = CM_NONE;
    S.chainMode = CM_NONE;
    return CM_NONE;
  }
  if (next == CM_HV) {
    uint32_t mask = 0u;
    for (int j = 0; j < nh; ++j)
      if (sl[j] != ns) mask |= 1u << sl[j];
    add_chain_bytes(S, D, CM_HV, 1 + __popc(mask));
    make_job(job, D, CM_HV, ns, mask);
  } else {
    // a direction just formed overwrote slot ns: if that slot held the oldest pair, drop it
    if (dir && nh == M) S.nhist = M - 1;
    if (next == CM_GRAD) {
      add_chain_bytes(S, D, CM_GRAD, 0);
      make_job(job, D, CM_GRAD, ns, 0u);
    } else {
      job.mode = CM_NONE;   // flush-only iteration: no transform
    }
  }
  S.chainMode = next;
  D.statusOut[0] = ST_RUNNING;
  return next;
}

// ======================================================================== conjugate gradients
// CG on the same quadratic, operator and variable as the L-BFGS solve (the whitened
// variable, or the split-preconditioned one: the chain applies P^1/2 D P^1/2), an
// alternative optimiser in the same batched engine (sec. 4 lists CG among the standard
// choices for this problem).  Per iteration: the curvature product Dp (chain, no extra
// dots), alpha = rho / p.Dp, w += alpha p, g += alpha Dp, rho' = g.g, beta = rho' / rho,
// p = -g + beta p.  The exact gradient is taken at the start, to confirm the stop (the
// same relative whitened-gradient test as L-BFGS) and every refreshEvery iterations;
// after it the recursion restarts (beta = 0).  Vectors: w, g, p = slot 0 of the p block,
// Dp = slot 0 of the Dp block.

__device__ __forceinline__ void cg_job(Job& jb, const InstDesc& D, int mode) {
  make_job(jb, D, mode, 0, 0u);
  jb.gvec = nullptr;
  jb.dpBase = nullptr;   // no solver dots in the curvature product
}

__device__ __forceinline__ void cg_stop(const InstDesc& D, LbState& S, Job& job, int status) {
  S.status = status;
  D.statusOut[0] = status;
  S.chainMode = CM_NONE;
  S.doB = 0;
  S.doDir = 0;
  job.mode = CM_NONE;
}

// after the chain: alpha (curvature product) or the chi^2 of an exact gradient
__global__ __launch_bounds__(256) void k_cg_step(const InstDesc* __restrict__ desc, LbState* st, Job* jobs) {
  const int i = blockIdx.x;
  LbState& S = st[i];
  if (S.status != ST_RUNNING) return;
  const InstDesc& D = desc[i];
  const int mode = S.chainMode;
  const int ncol = (D.n / 2) / TB, nrow = D.c * D.n / RB_MIN;
  __shared__ double chs[2];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (wv < 2) {   // one wave per partial kind, fixed-order sums
    int kind = -1, nb = 0;
    if (mode == CM_HV) {
      if (wv == 0) {
        kind = PK_VO;   // p . Dp
        nb = ncol;
      }
    } else {
      kind = wv == 0 ? PK_PRIOR : PK_RES;
      nb = wv == 0 ? ncol : nrow;
    }
    double a = 0.0;
    if (kind >= 0)
      for (int b = lane; b < nb; b += 64) a += D.partChain[kind * D.pstride + b];
    a = wave_sum(a);
    if (lane == 0) chs[wv] = a;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  if (mode == CM_HV) {
    const double pDp = chs[0];
    if (!(pDp > 0.0) || !isfinite(pDp)) {
      cg_stop(D, S, jobs[i], 2);
      return;
    }
    const double alpha = S.rho / pDp;
    S.alpha[0] = alpha;
    S.pDp = pDp;
    S.dchi2 = 4.0 * (alpha * S.gdotp + 0.5 * alpha * alpha * pDp);
    S.chi2 += S.dchi2;
    S.iter += 1;
    S.lastWasGrad = 0;
    S.doB = 1;
    S.bytes[KK_PASSB] += 6.0 * D.vbytes;   // w, p, g, Dp read; w, g written
  } else {
    S.chi2 = 2.0 * chs[0] + chs[1];
    S.ngrad += 1;
    S.lastGradIter = S.iter;
    S.lastWasGrad = 1;
    S.doB = 2;
    S.bytes[KK_PASSB] += D.vbytes * (D.rhs ? 3.0 : 1.0);   // g read (and rhs read, g written)
  }
}

// vector pass: w += alpha p, g += alpha Dp (after a curvature product); partial sums of g.g
// and of the whitened |g|^2 (kinds 0 and 1 of partA)
template <typename T, int PASS_U>
__global__ __launch_bounds__(NT) void k_cg_pass(const InstDesc* __restrict__ desc, const LbState* __restrict__ st) {
  const int i = rev_instance();
  const LbState& S = st[i];
  if (S.status != ST_RUNNING || !S.doB) return;
  const InstDesc& D = desc[i];
  using V = typename VecT<T>::type;
  constexpr int VW = VecT<T>::W;
  __shared__ double red[NT / 64][2];
  const uint32_t nvec = (uint32_t)(D.L * 2 / VW);
  const uint32_t vs = (uint32_t)(D.vstride * 2 / VW);
  const uint32_t e0 = blockIdx.x * (uint32_t)(NT * PASS_U) + threadIdx.x;
  V* X = reinterpret_cast<V*>(D.X);
  const uint32_t ow = 0, og = vs, op = 2 * vs, od = (uint32_t)(2 + D.m) * vs;
  const bool upd = S.doB == 1;
  const T al = T(S.alpha[0]);
  const T* ainv = reinterpret_cast<const T*>(D.ainv);
  double gg = 0.0, gw = 0.0;
#pragma unroll
  for (int u = 0; u < PASS_U; ++u) {
    const uint32_t e = e0 + (uint32_t)u * NT;
    if (e < nvec) {
      V g = gld(X, og + e);
      if (upd) {
        const V p = gld(X, op + e), dp = gld(X, od + e), w = gld(X, ow + e);
        g = vaxpy(al, dp, g);
        gst(X, og + e, g);
        gst(X, ow + e, vaxpy(al, p, w));
      } else if (D.rhs) {   // a correction solve's exact gradient is D v - rhs
        g = vaxpy(T(-1), gld(reinterpret_cast<const V*>(D.rhs), e), g);
        gst(X, og + e, g);
      }
      const double t = vdot(g, g);
      gg += t;
      gw += ainv ? wnorm2(g, ainv, e) : t;
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  gg = wave_sum(gg);
  gw = wave_sum(gw);
  if (lane == 0) {
    red[wv][0] = gg;
    red[wv][1] = gw;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) t += red[k][threadIdx.x];
    D.partA[(int64_t)blockIdx.x * NDOT + threadIdx.x] = t;
  }
}

// after the pass: stop test, beta and the next chain
__global__ __launch_bounds__(256) void k_cg_post(const InstDesc* __restrict__ desc, LbState* st, Job* jobs) {
  const int i = blockIdx.x;
  LbState& S = st[i];
  if (S.status != ST_RUNNING || !S.doB) return;
  const InstDesc& D = desc[i];
  __shared__ double sums[NDOT];
  __shared__ double part4[4][NDOT];
  reduce_columns(D.partA, D.nchunk, NDOT, 2, sums, part4);   // (synchronises)
  if (threadIdx.x != 0) return;
  const double rho = sums[0], gw = sums[1];
  const bool exact = S.doB == 2;
  S.doB = 0;
  S.gg = gw;
  if (exact && S.g0norm < 0.0) S.g0norm = sqrt(gw);
  const double g0 = S.g0norm;
  const double rel = g0 > 0.0 ? sqrt(gw) / g0 : 0.0;
  int status = ST_RUNNING, next = CM_HV;
  bool restart = exact;
  if (!isfinite(rho) || !isfinite(gw) || !isfinite(S.chi2)) {
    status = 2;
  } else if (rel <= D.tol || g0 == 0.0) {
    if (exact) status = 0;
    else next = CM_GRAD;              // confirm with the exact gradient
  } else if (S.iter >= D.maxIter) {
    status = 1;
  } else if (!exact && D.dchi2Tol > 0.0 && S.iter > 0 && fabs(S.dchi2) < D.dchi2Tol) {
    status = 0;
  } else if (!exact && D.refreshEvery > 0 && S.iter - S.lastGradIter >= D.refreshEvery) {
    next = CM_GRAD;
  }
  if (status != ST_RUNNING) {
    cg_stop(D, S, jobs[i], status);
    return;
  }
  if (next == CM_GRAD) {
    S.doDir = 0;
    S.chainMode = CM_GRAD;
    cg_job(jobs[i], D, CM_GRAD);
    add_chain_bytes(S, D, CM_GRAD, 0);
    return;
  }
  S.beta = restart ? 0.0 : rho / S.rho;
  S.rho = rho;
  S.gdotp = -rho;   // g . p of the new direction: g is orthogonal to the previous one
  S.doDir = 1;
  S.bytes[KK_DIR] += (restart ? 2.0 : 3.0) * D.vbytes;
  S.chainMode = CM_HV;
  cg_job(jobs[i], D, CM_HV);
  add_chain_bytes(S, D, CM_HV, 0);
}

// direction pass: p = -g + beta p (p = -g after an exact gradient)
template <typename T, int PASS_U>
__global__ __launch_bounds__(NT) void k_cg_dir(const InstDesc* __restrict__ desc, const LbState* __restrict__ st) {
  const int i = blockIdx.y;
  const LbState& S = st[i];
  if (S.status != ST_RUNNING || !S.doDir) return;
  const InstDesc& D = desc[i];
  using V = typename VecT<T>::type;
  constexpr int VW = VecT<T>::W;
  const uint32_t nvec = (uint32_t)(D.L * 2 / VW);
  const uint32_t vs = (uint32_t)(D.vstride * 2 / VW);
  const uint32_t e0 = blockIdx.x * (uint32_t)(NT * PASS_U) + threadIdx.x;
  V* X = reinterpret_cast<V*>(D.X);
  const uint32_t og = vs, op = 2 * vs;
  const T be = T(S.beta);
#pragma unroll
  for (int u = 0; u < PASS_U; ++u) {
    const uint32_t e = e0 + (uint32_t)u * NT;
    if (e < nvec) {
      const V g = gld(X, og + e);
      gst(X, op + e, be != T(0) ? vaxpy(T(-1), g, vscale(be, gld(X, op + e))) : vscale(T(-1), g));
    }
  }
}

// ------------------------------------------------------------------------ tables and packing
// sqrt S on the internal layout (0 on dead modes and conjugate partners), computed in
// float64 from P_k and theta; internal band table (-1 off the free modes).  With meanW
// (preconditioned solves) the scale becomes sqrt(S P) with P = 1 / (1 + S <W>), and a = P,
// ainv = 1 / P are written as well.
template <typename T>
__global__ void k_prior_table(int n, int C, const double* __restrict__ pshape, const int32_t* __restrict__ band,
                              const double* __restrict__ theta, int nbands, const double* __restrict__ meanW,
                              T* __restrict__ sq, int32_t* __restrict__ bandI, T* __restrict__ aT,
                              T* __restrict__ ainvT) {
  const int h = n / 2;
  const int64_t tot = (int64_t)C * n * h;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e / ((int64_t)n * h));
    const int r = (int)(e % ((int64_t)n * h));
    const int ky = r / h, kx = r % h;
    const int64_t src = ((int64_t)c * n + ky) * (h + 1) + kx;
    double S = 0.0;
    int b = -1;
    if (is_free(n, ky, kx)) {
      b = band[src];
      const double amp = (b >= 0 && b < nbands) ? theta[b] : 1.0;
      S = amp * pshape[src];
      if (!(S > 0.0)) S = 0.0;
      if (!(b >= 0 && b < nbands)) b = -1;
    }
    const int64_t o = fidx(n, c, ky, kx);
    double P = 1.0;
    if (meanW) P = 1.0 / (1.0 + S * meanW[0]);
    sq[o] = T(sqrt(S * P));
    bandI[o] = (S > 0.0) ? b : -1;
    if (aT) aT[o] = T(P);
    if (ainvT) ainvT[o] = T(1.0 / P);
  }
}

// pixel mean of W in float64 (one work-group)
template <typename T>
__global__ __launch_bounds__(1024) void k_mean_w(const T* __restrict__ W, int64_t npix, double* __restrict__ out) {
  __shared__ double red[1024 / 64];
  double a = 0.0;
  for (int64_t e = threadIdx.x; e < npix; e += 1024) a += (double)W[e];
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < 1024 / 64; ++i) t += red[i];
    out[0] = t / (double)npix;
  }
}

// external [C][n][n/2+1] -> internal (the Nyquist column is dropped)
template <typename T>
__global__ void k_unpack(int n, int C, int batch, const cpx<T>* __restrict__ ext, cpx<T>* __restrict__ in) {
  const int h = n / 2;
  const int64_t per = (int64_t)C * n * h;
  const int64_t tot = per * batch;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / per, r0 = e % per;
    const int c = (int)(r0 / ((int64_t)n * h));
    const int r = (int)(r0 % ((int64_t)n * h));
    const int ky = r / h, kx = r % h;
    in[i * per + fidx(n, c, ky, kx)] = ext[i * (int64_t)C * n * (h + 1) + ((int64_t)c * n + ky) * (h + 1) + kx];
  }
}

// internal -> external.  fill = 1: free entries scaled by sq (if given), partners as the
// conjugates of their free entries, dead entries 0.  fill = 0: copy every stored entry
// (live ones; dead entries 0).
template <typename T>
__global__ void k_pack(int n, int C, int batch, const cpx<T>* __restrict__ in, int64_t inStride,
                       const T* __restrict__ sq, int fill, cpx<T>* const* __restrict__ outs,
                       cpx<T>* __restrict__ out0) {
  const int h = n / 2;
  const int64_t per = (int64_t)C * n * (h + 1);
  const int64_t tot = per * batch;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / per, r0 = e % per;
    const int c = (int)(r0 / ((int64_t)n * (h + 1)));
    const int r = (int)(r0 % ((int64_t)n * (h + 1)));
    const int ky = r / (h + 1), kx = r % (h + 1);
    cpx<T> v = mk(T(0), T(0));
    if (kx < h && is_live(n, ky, kx)) {
      const bool part = is_partner(n, ky, kx);
      const int kyr = (fill && part) ? n - ky : ky;
      const int64_t src = fidx(n, c, kyr, kx);
      v = in[i * inStride + src];
      if (sq) v = scale(v, sq[src]);
      if (fill && part) v = conj(v);
    }
    cpx<T>* o = outs ? outs[i] : out0 + i * per;
    if (o) o[r0] = v;
  }
}

// k_pack with fill = 1 over a batch whose inputs, prior tables and outputs are given per
// instance (one launch for a class of solved fields that need not share a prior).
template <typename T>
__global__ void k_pack_tab(int n, int C, int batch, const PackEntry* __restrict__ tab) {
  const int h = n / 2;
  const int64_t per = (int64_t)C * n * (h + 1);
  const int64_t tot = per * batch;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / per, r0 = e % per;
    const PackEntry pe = tab[i];
    const int c = (int)(r0 / ((int64_t)n * (h + 1)));
    const int r = (int)(r0 % ((int64_t)n * (h + 1)));
    const int ky = r / (h + 1), kx = r % (h + 1);
    cpx<T> v = mk(T(0), T(0));
    if (kx < h && is_live(n, ky, kx)) {
      const bool part = is_partner(n, ky, kx);
      const int64_t src = fidx(n, c, part ? n - ky : ky, kx);
      v = reinterpret_cast<const cpx<T>*>(pe.in)[src];
      if (pe.sq) v = scale(v, reinterpret_cast<const T*>(pe.sq)[src]);
      if (part) v = conj(v);
    }
    reinterpret_cast<cpx<T>*>(pe.out)[r0] = v;
  }
}

// Signal coefficients of simulations sim0 .. sim0 + nsim - 1 (sec. 2.4) in the external
// layout [nsim][C][n][n/2+1]: s = sqrt S (z_re, z_im) / sqrt 2 on the free entries with the
// simulation pass's normals and rounding (draws, or the Philox stream when draws is null),
// kx = 0 partners the conjugates of their free entries, dead entries 0.  sq: internal
// sqrt S table.
template <typename T>
__global__ void k_sim_coeffs(int n, int C, int nsim, int sim0, uint64_t seed, const T* __restrict__ draws,
                             const T* __restrict__ sq, cpx<T>* __restrict__ out) {
  const int h = n / 2;
  const int64_t plane = (int64_t)n * (h + 1), per = (int64_t)C * plane, tot = per * nsim;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / per);
    const int64_t r0 = e % per;
    const int c = (int)(r0 / plane);
    const int r = (int)(r0 % plane);
    const int ky = r / (h + 1), kx = r % (h + 1);
    cpx<T> v = mk(T(0), T(0));
    if (kx < h && is_live(n, ky, kx)) {
      const bool part = is_partner(n, ky, kx);
      const int kyr = part ? n - ky : ky;
      const int64_t qn = ((int64_t)c * n + kyr) * n + 2 * kx;
      cpx<T> z;
      if (draws) {
        const T* dr = draws + (int64_t)i * 2 * C * n * n;
        z = mk(dr[qn], dr[qn + 1]);
      } else {   // the same normals as the simulation pass draws for this field type
        T z0, z1;
        philox_normal_pair<T>(seed, sim0 + i, qn, z0, z1);
        z = mk(z0, z1);
      }
      const T sc = sq[fidx(n, c, kyr, kx)] * T(0.70710678118654752440084436210485);
      v = scale(z, sc);
      if (part) v = conj(v);
    }
    out[e] = v;
  }
}

// acc[e] += sum_i sum_{p < P} (a[i][e P + p] - b[i][e P + p])^2 over the count arrays of
// len * P reals (b nullable: 0), in float64; one thread per e, fixed order in i.
template <typename T>
__global__ void k_sqdiff_acc(int64_t len, int P, int count, const T* __restrict__ a, const T* __restrict__ b,
                             double* __restrict__ acc) {
  const int64_t stride = len * P;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (int64_t)gridDim.x * blockDim.x) {
    double s = acc[e];
    for (int i = 0; i < count; ++i)
      for (int p = 0; p < P; ++p) {
        const int64_t o = (int64_t)i * stride + e * P + p;
        const double d = (double)a[o] - (b ? (double)b[o] : 0.0);
        s += d * d;
      }
    acc[e] = s;
  }
}

// out[e] = T(acc[e] * scale)
template <typename T>
__global__ void k_acc_out(int64_t len, const double* __restrict__ acc, double scale, T* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (int64_t)gridDim.x * blockDim.x)
    out[e] = T(acc[e] * scale);
}

// Band statistic E_l = Theta_l^-1 sum_{free k in l} |w_k|^2 for a whitened field, or
// sum |s_k|^2 / (Theta_l S_k) for a raw one (sec. 2.3, eq. el; the free half-plane sum
// is half the full-plane sum); or the band power sum_{free k in l} |s_k|^2 of a whitened
// field (raw == 2).  With f2 the field is f - f2.  Deterministic two-stage reduction: per-block partials
// for every band, then a fixed-order sum over blocks.
constexpr int BAND_EPT = 16;

template <typename T>
__global__ __launch_bounds__(NT) void k_band_part(const BandJob* __restrict__ jobs) {
  const BandJob& jb = jobs[blockIdx.y];
  __shared__ double red[NT / 64];
  const cpx<T>* f = reinterpret_cast<const cpx<T>*>(jb.f);
  const T* sq = reinterpret_cast<const T*>(jb.sq);
  int bl[BAND_EPT];
  double v[BAND_EPT];
  const int64_t base = (int64_t)blockIdx.x * NT * BAND_EPT;
#pragma unroll
  for (int k = 0; k < BAND_EPT; ++k) {
    const int64_t e = base + (int64_t)k * NT + threadIdx.x;
    bl[k] = -1;
    v[k] = 0.0;
    if (e < jb.L) {
      bl[k] = jb.bandI[e];
      if (bl[k] >= 0) {
        cpx<T> a = f[e];
        if (jb.f2) a = sub(a, reinterpret_cast<const cpx<T>*>(jb.f2)[e]);
        double t = (double)a.x * a.x + (double)a.y * a.y;
        if (jb.aw) t *= (double)reinterpret_cast<const T*>(jb.aw)[e];
        if (jb.raw == 1) {
          const double s = (double)sq[e];
          t /= s * s;
        } else if (jb.raw == 2) {
          const double s = (double)sq[e];
          t *= s * s;
        }
        v[k] = t;
      }
    }
  }
  for (int l = 0; l < jb.nbands; ++l) {
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < BAND_EPT; ++k) acc += (bl[k] == l) ? v[k] : 0.0;
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) jb.part[(int64_t)blockIdx.x * jb.nbands + l] = t;
  }
}

__global__ void k_band_final(const BandJob* __restrict__ jobs, int nblk) {
  const BandJob& jb = jobs[blockIdx.x];
  for (int l = threadIdx.x; l < jb.nbands; l += blockDim.x) {
    double a = 0.0;
    for (int b = 0; b < nblk; ++b) a += jb.part[(int64_t)b * jb.nbands + l];
    jb.E[l] = jb.raw == 2 ? a : a / jb.theta[l];
  }
}

// ------------------------------------------------------------------------ float64 refinement
// compact copy of the states' scalars the host reads at the end of a solve
__global__ void k_state_stats(const LbState* __restrict__ st, StateStat* __restrict__ out, int batch) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch) return;
  const LbState& S = st[i];
  StateStat r;
  r.status = S.status;
  r.iter = S.iter;
  r.ngrad = S.ngrad;
  r.pad = 0;
  r.chi2 = S.chi2;
  r.gg = S.gg;
  r.g0norm = S.g0norm;
  for (int k = 0; k < KK_COUNT; ++k) r.bytes[k] = S.bytes[k];
  out[i] = r;
}

__global__ void k_convert(const CvtJob* __restrict__ jobs) {
  const CvtJob J = jobs[blockIdx.y];
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < J.n; e += step) {
    if (J.op == CVT_F32_F64)
      reinterpret_cast<double*>(J.dst)[e] = (double)reinterpret_cast<const float*>(J.src)[e];
    else if (J.op == CVT_F64_F32)
      reinterpret_cast<float*>(J.dst)[e] = (float)reinterpret_cast<const double*>(J.src)[e];
    else
      reinterpret_cast<double*>(J.dst)[e] += (double)reinterpret_cast<const float*>(J.src)[e];
  }
}

__global__ __launch_bounds__(256) void k_refine_rhs(const RhsJob* __restrict__ jobs) {
  const RhsJob J = jobs[blockIdx.y];
  __shared__ double red[4];
  double a = 0.0;
  const int64_t step = (int64_t)gridDim.x * 256;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < J.L; e += step) {
    const double gr = J.g[2 * e], gi = J.g[2 * e + 1];
    J.rhs[2 * e] = (float)(-gr);
    J.rhs[2 * e + 1] = (float)(-gi);
    const double t = gr * gr + gi * gi;
    a += J.ainv ? J.ainv[e] * t : t;
  }
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) J.part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// ------------------------------------------------------------------------ copy ceiling
// Streaming copy for the bandwidth reference: 16-byte non-temporal loads and stores (the data
// is not reused, so it bypasses the caches), each thread issues the COPY_U loads of its tile
// before any of its stores; one tile of 256 * COPY_U vectors per work-group.  (Of the
// variants measured, 4 loads per thread and non-temporal accesses stream fastest.)
constexpr int COPY_U = 4;
typedef float f32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_stream_copy(const float4* __restrict__ src0, float4* __restrict__ dst0,
                                                      uint64_t n) {
  const f32x4* src = reinterpret_cast<const f32x4*>(src0);
  f32x4* dst = reinterpret_cast<f32x4*>(dst0);
  const uint64_t base = (uint64_t)blockIdx.x * (256 * COPY_U) + threadIdx.x;
  f32x4 v[COPY_U];
#pragma unroll
  for (int u = 0; u < COPY_U; ++u) {
    const uint64_t e = base + (uint64_t)u * 256;
    if (e < n) v[u] = __builtin_nontemporal_load(src + e);
  }
#pragma unroll
  for (int u = 0; u < COPY_U; ++u) {
    const uint64_t e = base + (uint64_t)u * 256;
    if (e < n) __builtin_nontemporal_store(v[u], dst + e);
  }
}

}  // namespace wf
