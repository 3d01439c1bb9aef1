// Device-resident batched L-BFGS (sec. 2.2) and the small kernels around it.
//
// Per iteration and instance the sequence is
//   chain (gradient or curvature product)  ->  k_post  ->  k_passA  ->  k_coef  ->  k_passB
// k_post   takes the exact step of the quadratic, alpha = -g.p / p.Dp (eq. eq_chib), or
//          records an exact gradient evaluation;
// k_passA  applies the step to w and g (w += alpha p, g += alpha Dp) and computes the
//          dot products of the new g and of the newest pair with the kept pairs;
// k_coef   updates the Gram entries, tests convergence and runs the two-loop recursion
//          on coefficients: the direction is a combination of the kept p_i, Dp_i and g
//          (s_i = alpha_i p_i, y_i = alpha_i Dp_i), so only scalars are touched;
// k_passB  forms the direction p = sum coef_j b_j in the next history slot.
// Instances that have stopped skip every kernel (per-instance convergence masks).
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
__device__ __forceinline__ double2 vscale(double a, const double2& x) { return make_double2(a * x.x, a * x.y); }

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

__device__ __forceinline__ void make_job(Job& jb, const InstDesc& D, int mode, int slot) {
  const size_t eb = (size_t)D.esize;
  char* X = reinterpret_cast<char*>(D.X);
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
  jb.band = nullptr;
  jb.draws = nullptr;
  jb.xout = nullptr;
  jb.part = D.partChain;
  jb.pstride = D.pstride;
  jb.vcs = D.L;
  jb.vcstr = D.L;
  const size_t vb = (size_t)D.vstride * eb;
  if (mode == CM_HV) {
    char* p = X + (size_t)(2 + slot) * vb;
    char* dp = X + (size_t)(2 + D.m + slot) * vb;
    jb.vin = p;
    jb.vadd = p;
    jb.vout = dp;
  } else {
    jb.vin = X;         // w
    jb.vadd = X;
    jb.vout = X + vb;   // g
  }
}

__device__ __forceinline__ void add_chain_bytes(LbState& S, const InstDesc& D, int mode) {
  const double V = D.vbytes;
  S.bytes[KK_COLINV] += 2.0 * V;                              // read field, write intermediate
  S.bytes[KK_ROW] += 2.0 * V + (mode == CM_GRAD ? V : 0.0);    // intermediate in/out (+ data)
  S.bytes[KK_COLFWD] += 3.0 * V;                              // intermediate, added term, output
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
  S.chainMode = CM_GRAD;
  S.lastWasGrad = 0;
  S.ngrad = 0;
  S.lastGradIter = 0;
  S.g0norm = -1.0;
  S.gg = 0.0;
  S.chi2 = 0.0;
  S.dchi2 = 0.0;
  S.gdotp = 0.0;
  S.pDp = 0.0;
  for (int k = 0; k < KK_COUNT; ++k) S.bytes[k] = 0.0;
  S.bytes[KK_MISC] += D.vbytes;   // zeroing w
  add_chain_bytes(S, D, CM_GRAD);
  make_job(jobs[i], D, CM_GRAD, 0);
}

// ------------------------------------------------------------------------ post-chain
__device__ __forceinline__ double wave_block_sum(const double* p, int nb) {
  double a = 0.0;
  for (int b = threadIdx.x; b < nb; b += 64) a += p[b];
  return wave_sum(a);
}

__global__ __launch_bounds__(64) void k_post(const InstDesc* __restrict__ desc, LbState* st, Job* jobs) {
  const int i = blockIdx.x;
  LbState& S = st[i];
  if (S.status != ST_RUNNING) return;
  const InstDesc& D = desc[i];
  const int mode = S.chainMode;
  const int ncol = (D.n / 2) / TB, nrow = D.n / RB;
  const double* part = D.partChain;
  if (mode == CM_HV) {
    const double pDp = wave_block_sum(part + PK_VO * D.pstride, ncol);
    if (threadIdx.x != 0) return;
    if (!(pDp > 0.0) || !isfinite(pDp)) {
      S.status = 2;
      D.statusOut[0] = 2;
      jobs[i].mode = CM_NONE;
      return;
    }
    const double alpha = -S.gdotp / pDp;
    const int ns = S.newslot;
    S.alpha[ns] = alpha;
    S.head = ns;
    S.nhist = S.nhist + 1 < S.m ? S.nhist + 1 : S.m;
    S.pending = 1;
    S.pDp = pDp;
    S.dchi2 = 4.0 * (alpha * S.gdotp + 0.5 * alpha * alpha * pDp);
    S.chi2 += S.dchi2;
    S.iter += 1;
  } else if (mode == CM_GRAD) {
    const double wsq = wave_block_sum(part + PK_PRIOR * D.pstride, ncol);
    const double rsq = wave_block_sum(part + PK_RES * D.pstride, nrow);
    if (threadIdx.x != 0) return;
    S.chi2 = 2.0 * wsq + rsq;
    S.ngrad += 1;
    S.lastGradIter = S.iter;
    S.pending = 0;
    if (!isfinite(S.chi2)) {
      S.status = 2;
      D.statusOut[0] = 2;
      jobs[i].mode = CM_NONE;
    }
  }
}

// ------------------------------------------------------------------------ pass A
template <typename T, int M>
__global__ __launch_bounds__(NT) void k_passA(const InstDesc* __restrict__ desc, const LbState* __restrict__ st) {
  const int i = blockIdx.y;
  const LbState& S = st[i];
  if (S.status != ST_RUNNING) return;
  const InstDesc& D = desc[i];
  using V = typename VecT<T>::type;
  constexpr int VW = VecT<T>::W;
  __shared__ double red[NT / 64][NDOT];
  const int nh = S.nhist, head = S.head, pend = S.pending;
  const T al = pend ? T(S.alpha[head]) : T(0);
  const int64_t nvec = D.L * 2 / VW;
  const int64_t vs = D.vstride * 2 / VW;                  // vector elements between vectors
  const int64_t e0 = (int64_t)blockIdx.x * PASS_CV + threadIdx.x;
  V* X = reinterpret_cast<V*>(D.X);
  V* w = X;
  V* g = X + vs;
  const V* P = X + 2 * vs;
  const V* Dp = X + (2 + M) * vs;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  bool ok[PASS_U];
#pragma unroll
  for (int u = 0; u < PASS_U; ++u) ok[u] = e0 + (int64_t)u * NT < nvec;

  // the new gradient (after the pending step) and the newest pair
  V gv[PASS_U], ph[PASS_U], dh[PASS_U];
#pragma unroll
  for (int u = 0; u < PASS_U; ++u) {
    const int64_t e = e0 + (int64_t)u * NT;
    if (ok[u]) {
      gv[u] = g[e];
      if (pend) {
        ph[u] = P[(int64_t)head * vs + e];
        dh[u] = Dp[(int64_t)head * vs + e];
      }
    }
  }
  double gg = 0.0;
  if (pend) {
#pragma unroll
    for (int u = 0; u < PASS_U; ++u) {
      const int64_t e = e0 + (int64_t)u * NT;
      if (ok[u]) {
        const V wv0 = w[e];
        w[e] = vaxpy(al, ph[u], wv0);
        gv[u] = vaxpy(al, dh[u], gv[u]);
        g[e] = gv[u];
      }
    }
  }
#pragma unroll
  for (int u = 0; u < PASS_U; ++u)
    if (ok[u]) gg += vdot(gv[u], gv[u]);
  {
    const double a = wave_sum(gg);
    if (lane == 0) red[wv][5 * M] = a;
  }
  // one history slot at a time: dots with the new gradient and with the newest pair
#pragma unroll
  for (int j = 0; j < M; ++j) {
    stream_fence();
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0, a4 = 0.0;
    if (j < nh) {
      const int64_t sp = (int64_t)((head - j + 2 * M) % M) * vs;
      V pv[PASS_U], dv[PASS_U];
#pragma unroll
      for (int u = 0; u < PASS_U; ++u)
        if (ok[u]) pv[u] = P[sp + e0 + (int64_t)u * NT];
#pragma unroll
      for (int u = 0; u < PASS_U; ++u)
        if (ok[u]) dv[u] = Dp[sp + e0 + (int64_t)u * NT];
#pragma unroll
      for (int u = 0; u < PASS_U; ++u) {
        if (ok[u]) {
          a0 += vdot(gv[u], pv[u]);
          a1 += vdot(gv[u], dv[u]);
          if (pend) {
            a2 += vdot(ph[u], dv[u]);
            a3 += vdot(pv[u], dh[u]);
            a4 += vdot(dh[u], dv[u]);
          }
        }
      }
    }
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    a2 = wave_sum(a2);
    a3 = wave_sum(a3);
    a4 = wave_sum(a4);
    if (lane == 0) {
      red[wv][j] = a0;
      red[wv][M + j] = a1;
      red[wv][2 * M + j] = a2;
      red[wv][3 * M + j] = a3;
      red[wv][4 * M + j] = a4;
    }
  }
  __syncthreads();
  if (threadIdx.x < 5 * M + 1) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) t += red[k][threadIdx.x];
    D.partA[(int64_t)blockIdx.x * NDOT + threadIdx.x] = t;
  }
}

// ------------------------------------------------------------------------ coefficients
// One work-group per instance: the partial sums and the small Gram state are staged in
// LDS by all threads, then thread 0 runs the scalar recursion out of LDS.
template <int M>
__global__ __launch_bounds__(256) void k_coef(const InstDesc* __restrict__ desc, LbState* st, Job* jobs) {
  const int i = blockIdx.x;
  LbState& S = st[i];
  if (S.status != ST_RUNNING) return;
  const InstDesc& D = desc[i];
  __shared__ double sums[NDOT];
  __shared__ double sPD[M][M], sDD[M][M], sal[M], sgP[M], sgD[M];
  const int nblk = D.nchunk;
  {
    // 4 threads per sum, each over every 4th block with 4 independent loads in flight;
    // the four parts are combined in a fixed order
    __shared__ double part4[4][NDOT];
    const int t = threadIdx.x & 63, q = threadIdx.x >> 6;
    if (t < 5 * M + 1) {
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int b = q;
      for (; b + 12 < nblk; b += 16) {
        a0 += D.partA[(int64_t)b * NDOT + t];
        a1 += D.partA[(int64_t)(b + 4) * NDOT + t];
        a2 += D.partA[(int64_t)(b + 8) * NDOT + t];
        a3 += D.partA[(int64_t)(b + 12) * NDOT + t];
      }
      for (; b < nblk; b += 4) a0 += D.partA[(int64_t)b * NDOT + t];
      part4[q][t] = (a0 + a1) + (a2 + a3);
    }
    __syncthreads();
    if (threadIdx.x < 5 * M + 1)
      sums[threadIdx.x] = (part4[0][threadIdx.x] + part4[1][threadIdx.x]) +
                          (part4[2][threadIdx.x] + part4[3][threadIdx.x]);
  }
  for (int t = threadIdx.x; t < M * M; t += blockDim.x) {
    sPD[t / M][t % M] = S.PD[t / M][t % M];
    sDD[t / M][t % M] = S.DD[t / M][t % M];
  }
  for (int t = threadIdx.x; t < M; t += blockDim.x) sal[t] = S.alpha[t];
  __syncthreads();
  if (threadIdx.x != 0) return;

  const int nh = S.nhist, head = S.head;
  const int pend = S.pending;
  int sl[M];
  for (int j = 0; j < M; ++j) sl[j] = (head - j + 2 * M) % M;
  // bytes of the pass just finished
  S.bytes[KK_PASSA] += D.vbytes * (1.0 + 2.0 * nh + (pend ? 3.0 : 0.0));
  for (int j = 0; j < nh; ++j) {
    const int s = sl[j];
    sgP[s] = sums[j];
    sgD[s] = sums[M + j];
    S.gP[s] = sums[j];
    S.gD[s] = sums[M + j];
    if (pend) {
      sPD[head][s] = sums[2 * M + j];
      sPD[s][head] = sums[3 * M + j];
      sDD[head][s] = sums[4 * M + j];
      sDD[s][head] = sums[4 * M + j];
      S.PD[head][s] = sums[2 * M + j];
      S.PD[s][head] = sums[3 * M + j];
      S.DD[head][s] = sums[4 * M + j];
      S.DD[s][head] = sums[4 * M + j];
    }
  }
  const double gg = sums[5 * M];
  S.gg = gg;
  S.pending = 0;
  double g0 = S.g0norm;
  if (g0 < 0.0) {
    g0 = sqrt(gg);
    S.g0norm = g0;
  }
  const double rel = g0 > 0.0 ? sqrt(gg) / g0 : 0.0;
  const int lastWasGrad = S.lastWasGrad;
  const int iter = S.iter;

  int next = CM_HV;
  int status = ST_RUNNING;
  if (!isfinite(gg)) {
    status = 2;
    next = CM_NONE;
  } else if (g0 == 0.0) {
    status = 0;
    next = CM_NONE;
  } else if (rel <= D.tol) {
    if (lastWasGrad) {
      status = 0;
      next = CM_NONE;
    } else {
      next = CM_GRAD;
    }
  } else if (iter >= D.maxIter) {
    status = 1;
    next = CM_NONE;
  } else if (D.dchi2Tol > 0.0 && pend && fabs(S.dchi2) < D.dchi2Tol) {
    status = 0;
    next = CM_NONE;
  } else if (D.refreshEvery > 0 && iter - S.lastGradIter >= D.refreshEvery && !lastWasGrad) {
    next = CM_GRAD;
  }

  if (next == CM_HV) {
    // two-loop recursion in the coefficients of (p_0..p_{M-1}, Dp_0..Dp_{M-1}, g)
    double c[2 * M + 1];
    for (int k = 0; k < 2 * M + 1; ++k) c[k] = 0.0;
    c[2 * M] = 1.0;
    double a[M], rho[M];
    for (int j = 0; j < nh; ++j) {           // newest to oldest
      const int s = sl[j];
      const double al = sal[s];
      rho[j] = 1.0 / (al * al * sPD[s][s]);
      double sq = c[2 * M] * sgP[s];
      for (int t = 0; t < nh; ++t) sq += c[M + sl[t]] * sPD[s][sl[t]];
      a[j] = rho[j] * al * sq;
      c[M + s] -= a[j] * al;
    }
    if (nh > 0) {
      const double gam = sPD[head][head] / sDD[head][head];
      for (int k = 0; k < 2 * M + 1; ++k) c[k] *= gam;
    }
    for (int j = nh - 1; j >= 0; --j) {      // oldest to newest
      const int s = sl[j];
      const double al = sal[s];
      double yr = c[2 * M] * sgD[s];
      for (int t = 0; t < nh; ++t) yr += c[M + sl[t]] * sDD[s][sl[t]] + c[sl[t]] * sPD[sl[t]][s];
      const double beta = rho[j] * al * yr;
      c[s] += al * (a[j] - beta);
    }
    double gdp = -c[2 * M] * gg;
    for (int t = 0; t < nh; ++t) gdp -= c[sl[t]] * sgP[sl[t]] + c[M + sl[t]] * sgD[sl[t]];
    for (int k = 0; k < M; ++k) {
      S.coef[k] = -c[k];
      S.coef[MMAX + k] = -c[M + k];
    }
    S.coef[2 * MMAX] = -c[2 * M];
    S.gdotp = gdp;
    S.newslot = (head + 1) % M;
    if (!(gdp < 0.0) || !isfinite(gdp)) {
      // not a descent direction (round-off at the end of a solve): fall back to an
      // exact-gradient refresh, which resets the scalar bookkeeping
      next = lastWasGrad ? CM_NONE : CM_GRAD;
      if (next == CM_NONE) status = (rel <= 10.0 * D.tol) ? 0 : 2;
    }
  }
  if (next == CM_HV) {
    S.bytes[KK_PASSB] += D.vbytes * (2.0 * nh + 2.0);
    add_chain_bytes(S, D, CM_HV);
    make_job(jobs[i], D, CM_HV, S.newslot);
  } else if (next == CM_GRAD) {
    add_chain_bytes(S, D, CM_GRAD);
    make_job(jobs[i], D, CM_GRAD, 0);
  } else {
    jobs[i].mode = CM_NONE;
  }
  S.status = status;
  S.chainMode = next;
  S.lastWasGrad = (next == CM_GRAD) ? 1 : (next == CM_HV ? 0 : lastWasGrad);
  D.statusOut[0] = status;
}

// ------------------------------------------------------------------------ pass B
template <typename T, int M>
__global__ __launch_bounds__(NT) void k_passB(const InstDesc* __restrict__ desc, const LbState* __restrict__ st) {
  const int i = blockIdx.y;
  const LbState& S = st[i];
  if (S.status != ST_RUNNING || S.chainMode != CM_HV) return;
  const InstDesc& D = desc[i];
  using V = typename VecT<T>::type;
  constexpr int VW = VecT<T>::W;
  const int nh = S.nhist, head = S.head, ns = S.newslot;
  int sl[M];
  T cP[M], cD[M];
#pragma unroll
  for (int j = 0; j < M; ++j) {
    sl[j] = (head - j + 2 * M) % M;
    cP[j] = T(S.coef[sl[j]]);
    cD[j] = T(S.coef[MMAX + sl[j]]);
  }
  const T cg = T(S.coef[2 * MMAX]);
  const int64_t nvec = D.L * 2 / VW;
  const int64_t vs = D.vstride * 2 / VW;
  const int64_t e0 = (int64_t)blockIdx.x * PASS_CV + threadIdx.x;
  V* X = reinterpret_cast<V*>(D.X);
  const V* g = X + vs;
  V* P = X + 2 * vs;
  const V* Dp = X + (2 + M) * vs;
  bool ok[PASS_U];
  V acc[PASS_U];
#pragma unroll
  for (int u = 0; u < PASS_U; ++u) {
    ok[u] = e0 + (int64_t)u * NT < nvec;
    if (ok[u]) acc[u] = vscale(cg, g[e0 + (int64_t)u * NT]);
  }
#pragma unroll
  for (int j = 0; j < M; ++j) {
    stream_fence();
    if (j < nh) {
      const int64_t sp = (int64_t)sl[j] * vs;
#pragma unroll
      for (int u = 0; u < PASS_U; ++u)
        if (ok[u]) acc[u] = vaxpy(cP[j], P[sp + e0 + (int64_t)u * NT], acc[u]);
#pragma unroll
      for (int u = 0; u < PASS_U; ++u)
        if (ok[u]) acc[u] = vaxpy(cD[j], Dp[sp + e0 + (int64_t)u * NT], acc[u]);
    }
  }
  stream_fence();
#pragma unroll
  for (int u = 0; u < PASS_U; ++u)
    if (ok[u]) P[(int64_t)ns * vs + e0 + (int64_t)u * NT] = acc[u];
}

// ------------------------------------------------------------------------ tables and packing
// sqrt S on the internal layout (0 on dead modes and conjugate partners), computed in
// float64 from P_k and theta; internal band table (-1 off the free modes).
template <typename T>
__global__ void k_prior_table(int n, int C, const double* __restrict__ pshape, const int32_t* __restrict__ band,
                              const double* __restrict__ theta, int nbands, T* __restrict__ sq,
                              int32_t* __restrict__ bandI) {
  const int h = n / 2;
  const int64_t tot = (int64_t)C * n * h;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e / ((int64_t)n * h));
    const int r = (int)(e % ((int64_t)n * h));
    const int ky = r / h, kx = r % h;
    const int64_t src = ((int64_t)c * n + ky) * (h + 1) + kx;
    double s = 0.0;
    int b = -1;
    if (is_free(n, ky, kx)) {
      b = band[src];
      const double amp = (b >= 0 && b < nbands) ? theta[b] : 1.0;
      const double S = amp * pshape[src];
      s = S > 0.0 ? sqrt(S) : 0.0;
      if (!(b >= 0 && b < nbands)) b = -1;
    }
    const int64_t o = fidx(n, c, ky, kx);
    sq[o] = T(s);
    bandI[o] = (s > 0.0) ? b : -1;
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
__global__ void k_pack(int n, int C, int batch, const cpx<T>* __restrict__ in, int64_t inStride, int64_t vcs,
                       int64_t vcstr, const T* __restrict__ sq, int fill, cpx<T>* const* __restrict__ outs,
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
      v = in[i * inStride + vview(src, vcs, vcstr)];
      if (sq) v = scale(v, sq[src]);
      if (fill && part) v = conj(v);
    }
    cpx<T>* o = outs ? outs[i] : out0 + i * per;
    if (o) o[r0] = v;
  }
}

// Band statistic E_l = Theta_l^-1 sum_{free k in l} |w_k|^2 for a whitened field, or
// sum |s_k|^2 / (Theta_l S_k) for a raw one (sec. 2.3, eq. el; the free half-plane sum
// is half the full-plane sum).  Deterministic two-stage reduction: per-block partials
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
        const cpx<T> a = f[vview(e, jb.vcs, jb.vcstr)];
        double t = (double)a.x * a.x + (double)a.y * a.y;
        if (jb.raw) {
          const double s = (double)sq[e];
          t /= s * s;
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
    jb.E[l] = a / jb.theta[l];
  }
}

}  // namespace wf
