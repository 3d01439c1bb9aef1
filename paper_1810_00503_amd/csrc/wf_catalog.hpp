// Catalog-level response (sec. 3.4): the field of the harmonic coefficients evaluated at each
// galaxy's own position instead of binned pixels, gamma(r_g) = n^-1 sum_k gamma~_k
// exp(2 pi i k.r_g / n), and its adjoint, as a non-uniform FFT on a fine grid of N = 2n
// points per side:
//
//   pad      coarse field -> fine half-plane spectrum, each band mode scaled by T_k
//            = (prior scale) (N/n) / (phi^(ky/N) phi^(kx/N)) (deconvolution of the kernel);
//   forward  the transform passes of the chain at size N (column inverse, row) -> fine map u;
//   interp   per galaxy, sum of u over the (CAT_W + 1)^2 fine points around its cell (the
//            kernel phi is 0 beyond W/2, so these hold every point it reaches) with the
//            separable exponential-of-semicircle weights -> gamma(r_g), and the weighted
//            residual (solver) or the value (forward operator);
//   spread   the adjoint of interp with the same weights, per fine-grid tile in two passes:
//            along x per galaxy cell row, then the CAT_W + 1 rows per point, each sum in a
//            fixed order;
//   adjoint  the transform passes at size N (row, column forward) -> fine spectrum;
//   unpad    band modes back to the coarse layout, times T_k, plus the solver's prior term
//            and the dot partials of the chain's column-forward pass.
//
// Inside the batched solver these replace the three coarse passes of a curvature product or
// exact gradient; the jobs the solver writes each iteration drive them as they drive the
// chain.  Set-up, once per call: each galaxy's fine cell (key), a stable radix sort of the
// galaxies by cell, and in the sorted order the cells, a 48-byte record per galaxy (its CAT_W + 1
// weights along y and the fraction of its x coordinate, from which a pass computes the x weight
// it needs: fewer bytes per galaxy than a stored x row, which the spreading pass is bound by)
// and the first galaxy of every cell.  The kernel: phi(z) = exp(beta (sqrt(1 - (2z/W)^2) - 1)) on |z| <= W/2, beta = 2.3 W for
// oversampling 2 (Barnett, Magland & af Klinteberg, SIAM J. Sci. Comput. 41, 2019); its
// Fourier transform is tabulated on the host in float64.
#pragma once
#include "wf_chain.hpp"   // wave_sum, the layout helpers

namespace wf {

__device__ __forceinline__ float es_kernel(float z) {
  const float t = z * (2.0f / (float)CAT_W);
  const float q = 1.0f - t * t;
  return q >= 0.0f ? expf(CAT_BETA * (sqrtf(q) - 1.0f)) : 0.0f;
}

// j in [-N, 2N) -> j mod N
__device__ __forceinline__ int cat_wrap(int j, int N) {
  j += j < 0 ? N : 0;
  return j >= N ? j - N : j;
}

// XCD-aware work order: the dispatcher hands work-groups to the 8 XCDs in turn, so one XCD runs
// every 8th; logical block of work-group b (of nblk) such that each XCD takes one contiguous
// range of logical blocks (neighbouring tiles, which read the same galaxies, share its L2)
__device__ __forceinline__ int xcd_order(int b, int nblk) {
  const int x = b & 7, q = nblk >> 3, rem = nblk & 7;
  return x * q + min(x, rem) + (b >> 3);
}

__device__ __forceinline__ bool cat_solver_mode(int mode) { return mode == CM_HV || mode == CM_GRAD; }

// ------------------------------------------------------------------------ pad
// grid (N / 4 fine column blocks, instances).  In solver modes it also switches the instance's
// fine-grid jobs on (or off when the instance does no transform this iteration) and writes the
// prior partials of an exact gradient (one slot per coarse column block).
template <int C>
__global__ __launch_bounds__(NT) void k_cat_pad(const Job* __restrict__ jobs, CatDesc* __restrict__ cats) {
  const int i = blockIdx.y;
  const Job& jb = jobs[i];
  CatDesc& cd = cats[i];
  const int mode = jb.mode;
  const bool solver = cat_solver_mode(mode);
  if (blockIdx.x == 0 && threadIdx.x == 0 && mode != CM_FWD) {
    cd.jfwd->mode = solver ? CM_FWD : CM_NONE;
    cd.jadj->mode = solver ? CM_ADJ : CM_NONE;
  }
  if (!(solver || mode == CM_FWD)) return;
  __shared__ double red[NT / 64];
  const int n = cd.n, N = cd.N, h = n / 2;
  const int b = blockIdx.x;
  const bool band = 2 * b < h;
  const cpx<float>* vin = reinterpret_cast<const cpx<float>*>(jb.vin);
  cpx<float>* y2 = reinterpret_cast<cpx<float>*>(cd.y2);
  double acc = 0.0;
  for (int e = threadIdx.x; e < C * N * TB; e += NT) {
    const int cc = e / (N * TB), r = e % (N * TB), KY = r / TB, kx = 2 * b + r % TB;
    cpx<float> val = mk(0.0f, 0.0f);
    if (band && (KY < h || KY > N - h)) {
      const int ky = KY < h ? KY : KY - N + n;
      const uint32_t o = (uint32_t)fidx(n, cc, ky, kx);
      const float t = cd.T[o];
      if (t != 0.0f) {
        const cpx<float> v = vin[o];
        val = mk(t * v.x, t * v.y);
        if (mode == CM_GRAD) {
          const double wa = cd.aTab ? (double)cd.aTab[o] : 1.0;
          acc += wa * ((double)v.x * v.x + (double)v.y * v.y);
        }
      }
    }
    y2[fidx(N, cc, KY, kx)] = val;
  }
  if (mode == CM_GRAD) {
    const double a = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0 && band) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < NT / 64; ++k) t += red[k];
      jb.part[PK_PRIOR * jb.pstride + b] = t;
    }
  }
}

// ------------------------------------------------------------------------ interpolation
// grid (blocks of NT galaxies, instances): gamma_a(r_g) from the fine map; the residual
// wgt (gamma - e) and its chi^2 partial (exact gradient), wgt gamma (curvature), or gamma
// (forward operator), into cd.r in the sorted order.
template <int C>
__global__ __launch_bounds__(NT) void k_cat_interp(const Job* __restrict__ jobs, const CatDesc* __restrict__ cats) {
  const int i = blockIdx.y;
  const Job& jb = jobs[i];
  const int mode = jb.mode;
  if (!(cat_solver_mode(mode) || mode == CM_FWD)) return;
  const CatDesc& cd = cats[i];
  const int lb = xcd_order(blockIdx.x, gridDim.x);
  if (lb * NT >= cd.ngal) return;   // the grid covers the class's largest catalog
  __shared__ double red[NT / 64];
  const int g = lb * NT + threadIdx.x;
  double acc = 0.0;
  if (g < cd.ngal) {
    const int N = cd.N;
    const int2 c0 = cd.cell[g];
    float w[2 * CAT_D];
    {
      const float4 a0 = cd.rec[3 * (size_t)g], a1 = cd.rec[3 * (size_t)g + 1], a2 = cd.rec[3 * (size_t)g + 2];
      const float rw[CAT_REC] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w, a2.x, a2.y, a2.z, a2.w};
#pragma unroll
      for (int t = 0; t < CAT_D; ++t) {
        w[t] = rw[t];
        w[CAT_D + t] = es_kernel(rw[CAT_D] + (float)(CAT_H - t));
      }
    }
    int jx[CAT_D];
#pragma unroll
    for (int t = 0; t < CAT_D; ++t) jx[t] = cat_wrap(c0.y - CAT_H + t, N);
    float gam[C];
#pragma unroll
    for (int cc = 0; cc < C; ++cc) gam[cc] = 0.0f;
#pragma unroll 3
    for (int ty = 0; ty < CAT_D; ++ty) {
      const int jy = cat_wrap(c0.x - CAT_H + ty, N);
#pragma unroll
      for (int cc = 0; cc < C; ++cc) {
        const float* row = cd.u + ((size_t)cc * N + jy) * N;
        float a = 0.0f;
#pragma unroll
        for (int tx = 0; tx < CAT_D; ++tx) a += w[CAT_D + tx] * row[jx[tx]];
        gam[cc] += w[ty] * a;
      }
    }
    const float wg = mode == CM_FWD ? 1.0f : cd.wgt[g];
#pragma unroll
    for (int cc = 0; cc < C; ++cc) {
      float r;
      if (mode == CM_GRAD) {
        const float d = gam[cc] - cd.e[(size_t)cc * cd.ngal + g];
        r = wg * d;
        acc += (double)r * d;
      } else if (mode == CM_HV) {
        r = wg * gam[cc];
      } else {
        r = gam[cc];
      }
      cd.r[(size_t)g * C + cc] = r;
    }
  }
  if (mode == CM_GRAD) {
    const double a = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < NT / 64; ++k) t += red[k];
      cd.partI[lb] = t;
    }
  }
}

// ------------------------------------------------------------------------ spreading
// grid (tiles * tiles, instances), CAT_SPREAD_NT threads: the adjoint of interp on a CAT_TS x
// CAT_TS tile of fine points, v(jy, jx) = sum_g wy_g[jy - cy_g + H] wx_g[jx - cx_g + H] r_g.
// A galaxy reaches the tile only from the cell rows of the tile widened by H on each side
// (CAT_ROWS rows).  Pass 1, one thread per (widened row R, tile column jx): the galaxies of the
// cells jx - H .. jx + H of row R, consecutive in sorted order (two runs where the row wraps),
// t_d = sum wy_g[d] wx_g[e] r_g for d = 0 .. 2H, e = jx + H - (cell of g), in registers, CAT_U
// galaxies at a time so that their loads are in flight together.
// Pass 2, one thread per point: v(jy, jx) = sum_d t_d of row R = jy + H - d, in order of d.
// Every pair it forms contributes, and each point's sum has the same order on every call.
// Block 0 of an exact gradient also reduces the interpolation's chi^2 partials (one per NT
// galaxies, in a fixed order) into the residual slots the solver reads.
constexpr int CAT_ROWS = CAT_TS + 2 * CAT_H;
constexpr int CAT_SPREAD_NT = CAT_ROWS * CAT_TS;
constexpr int CAT_U = 2;   // galaxies per step of a pass-1 thread
template <int C>
__global__ __launch_bounds__(CAT_SPREAD_NT) void k_cat_spread(const Job* __restrict__ jobs,
                                                                const CatDesc* __restrict__ cats) {
  const int i = blockIdx.y;
  const Job& jb = jobs[i];
  const int mode = jb.mode;
  if (!(cat_solver_mode(mode) || mode == CM_ADJ || mode == CM_ADJ_GRAD)) return;
  const CatDesc& cd = cats[i];
  const int tiles = cd.tiles, N = cd.N, ngal = cd.ngal;
  __shared__ float tsh[CAT_D][C][CAT_ROWS][CAT_TS];   // [d][c][widened row][column]
  __shared__ double red[CAT_SPREAD_NT / 64];
  if (mode == CM_GRAD && blockIdx.x == 0) {
    // strided per-thread sums, then the waves' fixed-order shuffle trees, then wave order
    const int nb = (ngal + NT - 1) / NT;
    double a = 0.0;
    for (int k = threadIdx.x; k < nb; k += CAT_SPREAD_NT) a += cd.partI[k];
    a = wave_sum(a);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
      for (int w = 0; w < CAT_SPREAD_NT / 64; ++w) t += red[w];
    for (int k = threadIdx.x; k < cd.nrowPart; k += CAT_SPREAD_NT)
      jb.part[PK_RES * jb.pstride + k] = k == 0 ? t : 0.0;
  }
  if ((int)blockIdx.x >= tiles * tiles) return;
  const int tb = xcd_order(blockIdx.x, tiles * tiles);
  const int ty = tb / tiles, tx = tb % tiles;
  {
    const int r = (int)threadIdx.x / CAT_TS, col = (int)threadIdx.x % CAT_TS;
    const int jx = tx * CAT_TS + col;
    const int* cs = cd.cellStart + (size_t)cat_wrap(ty * CAT_TS - CAT_H + r, N) * N;
    const float4* __restrict__ rec = cd.rec;
    const float* __restrict__ rr = cd.r;
    float t[CAT_D][C];
#pragma unroll
    for (int d = 0; d < CAT_D; ++d)
#pragma unroll
      for (int cc = 0; cc < C; ++cc) t[d][cc] = 0.0f;
    // first galaxy of each of the thread's cells jx - H + m, m = 0 .. 2H, and the end of the last
    int beg[CAT_D + 1];
#pragma unroll
    for (int m = 0; m < CAT_D; ++m) beg[m] = cs[cat_wrap(jx - CAT_H + m, N)];
    beg[CAT_D] = cs[cat_wrap(jx + CAT_H, N) + 1];
    // the row wraps between cells m = mw - 1 and mw (mw = CAT_D: no wrap)
    const int mw = jx - CAT_H < 0 ? CAT_H - jx : (jx + CAT_H >= N ? N - (jx - CAT_H) : CAT_D);
    // beg[mw] by selects (a register array indexed at run time would live in scratch)
    int begW = beg[CAT_D];
#pragma unroll
    for (int k = 0; k < CAT_D; ++k) begW = k == mw ? beg[k] : begW;
    for (int run = 0; run < 2; ++run) {
      const int m0 = run == 0 ? 0 : mw, m1 = run == 0 ? mw : CAT_D;   // cells [m0, m1)
      if (m1 <= m0) continue;
      const int ga = run == 0 ? beg[0] : begW;
      const int gb = m1 == CAT_D ? beg[CAT_D] : cs[N];   // a wrapping run ends with the row
      for (int g0 = ga; g0 < gb; g0 += CAT_U) {
#pragma unroll
        for (int j = 0; j < CAT_U; ++j) {
          const bool ok = g0 + j < gb;
          const int g = ok ? g0 + j : gb - 1;
          int m = m0;   // cell of g: the last m in [m0, m1) with beg[m] <= g
#pragma unroll
          for (int k = 1; k < CAT_D; ++k) m += (k > m0 && k < m1 && beg[k] <= g) ? 1 : 0;
          const int e = 2 * CAT_H - m;
          const float4 a0 = rec[3 * (size_t)g], a1 = rec[3 * (size_t)g + 1], a2 = rec[3 * (size_t)g + 2];
          const float w[CAT_REC] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w, a2.x, a2.y, a2.z, a2.w};
          const float wx = ok ? es_kernel(w[CAT_D] + (float)(CAT_H - e)) : 0.0f;
          float rv[C];
          if constexpr (C == 2) {
            const float2 q = reinterpret_cast<const float2*>(rr)[g];
            rv[0] = q.x;
            rv[1] = q.y;
          } else {
            rv[0] = rr[g];
          }
#pragma unroll
          for (int cc = 0; cc < C; ++cc) {
            const float a = wx * rv[cc];
#pragma unroll
            for (int d = 0; d < CAT_D; ++d) t[d][cc] += w[d] * a;
          }
        }
      }
    }
#pragma unroll
    for (int d = 0; d < CAT_D; ++d)
#pragma unroll
      for (int cc = 0; cc < C; ++cc) tsh[d][cc][r][col] = t[d][cc];
  }
  __syncthreads();
  if ((int)threadIdx.x < CAT_TS * CAT_TS) {
    const int py = (int)threadIdx.x / CAT_TS, px = (int)threadIdx.x % CAT_TS;
    const int jy = ty * CAT_TS + py, jx = tx * CAT_TS + px;
    float acc[C];
#pragma unroll
    for (int cc = 0; cc < C; ++cc) acc[cc] = 0.0f;
    // galaxy row R = jy + H - d is widened row py + 2H - d
#pragma unroll
    for (int d = 0; d < CAT_D; ++d)
#pragma unroll
      for (int cc = 0; cc < C; ++cc) acc[cc] += tsh[d][cc][py + 2 * CAT_H - d][px];
#pragma unroll
    for (int cc = 0; cc < C; ++cc) cd.v[((size_t)cc * N + jy) * N + jx] = acc[cc];
  }
}

// ------------------------------------------------------------------------ unpad
// grid (n / 4 coarse column blocks, instances), CAT_UNPAD_NT threads: the fine spectrum t of
// the band modes back on the coarse layout; solver modes: out = wa v + T t on the free modes
// with the dot partials [VO, OO, DG, DD_j] of the column-forward pass (one slot per column
// block); operator modes: out = T t on the live modes (metric adjoint) or 2 T t on the free ones
// (gradient form).  A thread's elements (CAT_UNPAD_K at most) have all their loads issued before
// the arithmetic, and the loads of each kept Dp_j together.
constexpr int CAT_UNPAD_NT = 1024;
constexpr int CAT_UNPAD_K = 4;
template <int C>
__global__ __launch_bounds__(CAT_UNPAD_NT) void k_cat_unpad(const Job* __restrict__ jobs,
                                                              const CatDesc* __restrict__ cats) {
  const int i = blockIdx.y;
  const Job& jb = jobs[i];
  const int mode = jb.mode;
  if (!(cat_solver_mode(mode) || mode == CM_ADJ || mode == CM_ADJ_GRAD)) return;
  const CatDesc& cd = cats[i];
  constexpr int NW = CAT_UNPAD_NT / 64;
  __shared__ double red2[NW][3 + MMAX];
  const int n = cd.n, N = cd.N, h = n / 2;
  const int b = blockIdx.x;
  const cpx<float>* y2 = reinterpret_cast<const cpx<float>*>(cd.y2);
  cpx<float>* vout = reinterpret_cast<cpx<float>*>(jb.vout);
  const bool solver = cat_solver_mode(mode);
  const bool extras = mode == CM_HV && jb.dpBase != nullptr;
  const uint32_t mask = extras ? jb.dpMask : 0u;
  double avo = 0.0, aoo = 0.0, adg = 0.0, add[MMAX];
#pragma unroll
  for (int j = 0; j < MMAX; ++j) add[j] = 0.0;
  const int NEL = C * n * TB;
  for (int e0 = threadIdx.x; e0 < NEL; e0 += CAT_UNPAD_NT * CAT_UNPAD_K) {
    uint32_t o[CAT_UNPAD_K];
    bool ok[CAT_UNPAD_K], keep[CAT_UNPAD_K];
    float Tv[CAT_UNPAD_K];
    cpx<float> t[CAT_UNPAD_K], a[CAT_UNPAD_K], out[CAT_UNPAD_K];
#pragma unroll
    for (int k = 0; k < CAT_UNPAD_K; ++k) {
      const int e = e0 + k * CAT_UNPAD_NT;
      ok[k] = e < NEL;
      const int ee = ok[k] ? e : NEL - 1;   // past the end: any valid element, not stored
      const int cc = ee / (n * TB), r = ee % (n * TB), ky = r / TB, kx = 2 * b + r % TB;
      o[k] = (uint32_t)fidx(n, cc, ky, kx);
      const int KY = ky < h ? ky : ky - n + N;
      Tv[k] = cd.T[o[k]];
      t[k] = y2[fidx(N, cc, KY, kx)];
      a[k] = solver ? reinterpret_cast<const cpx<float>*>(jb.vadd)[o[k]] : mk(0.0f, 0.0f);
      keep[k] = ok[k] && (solver || mode == CM_ADJ_GRAD ? is_free(n, ky, kx) : is_live(n, ky, kx));
    }
#pragma unroll
    for (int k = 0; k < CAT_UNPAD_K; ++k) {
      cpx<float> v = mk(0.0f, 0.0f);
      if (solver) {
        if (keep[k] && Tv[k] != 0.0f) {
          const float wa = cd.aTab ? cd.aTab[o[k]] : 1.0f;
          v = mk(wa * a[k].x + Tv[k] * t[k].x, wa * a[k].y + Tv[k] * t[k].y);
          avo += (double)a[k].x * v.x + (double)a[k].y * v.y;
        }
        if (ok[k]) aoo += (double)v.x * v.x + (double)v.y * v.y;
      } else if (keep[k]) {
        const float f = mode == CM_ADJ ? Tv[k] : 2.0f * Tv[k];
        v = mk(f * t[k].x, f * t[k].y);
      }
      out[k] = v;
      if (ok[k]) vout[o[k]] = v;
    }
    if (extras) {
      const cpx<float>* gvec = reinterpret_cast<const cpx<float>*>(jb.gvec);
      cpx<float> gv[CAT_UNPAD_K];
#pragma unroll
      for (int k = 0; k < CAT_UNPAD_K; ++k) gv[k] = gvec[o[k]];
#pragma unroll
      for (int k = 0; k < CAT_UNPAD_K; ++k)
        if (ok[k]) adg += (double)gv[k].x * out[k].x + (double)gv[k].y * out[k].y;
      const cpx<float>* dpb = reinterpret_cast<const cpx<float>*>(jb.dpBase);
#pragma unroll
      for (int j = 0; j < MMAX; ++j) {
        if ((mask >> j) & 1u) {
          cpx<float> dj[CAT_UNPAD_K];
#pragma unroll
          for (int k = 0; k < CAT_UNPAD_K; ++k) dj[k] = gldnt(dpb, (uint32_t)((int64_t)j * jb.dpStride + o[k]));
#pragma unroll
          for (int k = 0; k < CAT_UNPAD_K; ++k)
            if (ok[k]) add[j] += (double)dj[k].x * out[k].x + (double)dj[k].y * out[k].y;
        }
      }
    }
  }
  if (!solver) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  {
    const double a0 = wave_sum(avo), a1 = wave_sum(aoo);
    if (lane == 0) {
      red2[wv][0] = a0;
      red2[wv][1] = a1;
    }
  }
  if (extras) {
    const double a2 = wave_sum(adg);
    if (lane == 0) red2[wv][2] = a2;
#pragma unroll
    for (int j = 0; j < MMAX; ++j) {
      if ((mask >> j) & 1u) {
        const double aj = wave_sum(add[j]);
        if (lane == 0) red2[wv][3 + j] = aj;
      }
    }
  }
  __syncthreads();
  const int nv = extras ? 3 + MMAX : 2;
  const int tid = threadIdx.x;
  if (tid < nv && (tid < 3 || ((mask >> (tid - 3)) & 1u))) {
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < NW; ++k) sum += red2[k][tid];
    jb.part[(PK_VO + tid) * jb.pstride + b] = sum;
  }
}

// ------------------------------------------------------------------------ tables, permutations
// T on the coarse internal layout: (sq, or 1 on the live modes when sq is null) (N/n) dk[|ky|]
// dk[kx], dk = 1 / phi^(k/N); 0 where sq is 0 or the mode is dead
__global__ void k_cat_table(int n, int N, int C, const float* __restrict__ sq, const double* __restrict__ dk,
                            float* __restrict__ T) {
  const int h = n / 2;
  const int64_t tot = (int64_t)C * n * h;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e / ((int64_t)n * h));
    const int r = (int)(e % ((int64_t)n * h));
    const int ky = r / h, kx = r % h;
    const int64_t o = fidx(n, c, ky, kx);
    const int ks = ky < h ? ky : n - ky;
    float v = 0.0f;
    if (is_live(n, ky, kx)) {
      const double f = (double)N / (double)n * dk[ks] * dk[kx];
      v = sq ? (float)((double)sq[o] * f) : (float)f;
    }
    T[o] = v;
  }
}

// ------------------------------------------------------------------------ set-up
// fine-grid cell and fraction of coordinate x (pixel units): rho = 2 x wrapped into [0, N)
__device__ __forceinline__ void cat_cell(double x, int N, int& cell, float& frac) {
  double r = fmod(2.0 * x, (double)N);
  if (r < 0.0) r += (double)N;
  const double fl = floor(r);
  int ci = (int)fl;
  float fr = (float)(r - fl);
  if (fr >= 1.0f) {   // rounded up to the next cell
    fr = 0.0f;
    ++ci;
  }
  if (ci >= N) ci -= N;   // r == N after the wrap of a tiny negative value
  cell = ci;
  frac = fr;
}

// key[g] = fine cell (row-major) of galaxy g, idx[g] = g; *bad = 1 if a position is not finite
__global__ void k_cat_keys(const double* __restrict__ pos, int ngal, int N, uint32_t* __restrict__ key,
                           uint32_t* __restrict__ idx, int* __restrict__ bad) {
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < ngal; g += gridDim.x * blockDim.x) {
    const double y = pos[2 * (size_t)g], x = pos[2 * (size_t)g + 1];
    uint32_t k = 0;
    if (isfinite(y) && isfinite(x)) {
      int cy, cx;
      float fy, fx;
      cat_cell(y, N, cy, fy);
      cat_cell(x, N, cx, fx);
      k = (uint32_t)cy * (uint32_t)N + (uint32_t)cx;
    } else {
      *bad = 1;
    }
    key[g] = k;
    idx[g] = (uint32_t)g;
  }
}

// In the sorted order (skey, perm from the stable sort): cells, records (the weights
// phi(rho_y - j) at j = cell - H .. cell + H and the fraction of rho_x) and the first galaxy of
// every cell (cells before the first galaxy start at 0, after the last at ngal)
__global__ void k_cat_prep(const double* __restrict__ pos, const uint32_t* __restrict__ skey,
                           const uint32_t* __restrict__ perm, int ngal, int N, int2* __restrict__ cell,
                           float4* __restrict__ rec, int* __restrict__ cellStart) {
  const uint32_t ncell = (uint32_t)N * (uint32_t)N;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < ngal; q += gridDim.x * blockDim.x) {
    const uint32_t g = perm[q];
    const double y = pos[2 * (size_t)g], x = pos[2 * (size_t)g + 1];
    int cy = 0, cx = 0;
    float fy = 0.0f, fx = 0.0f;
    if (isfinite(y) && isfinite(x)) {
      cat_cell(y, N, cy, fy);
      cat_cell(x, N, cx, fx);
    }
    cell[q] = make_int2(cy, cx);
    float w[CAT_REC];
#pragma unroll
    for (int t = 0; t < CAT_D; ++t) w[t] = es_kernel(fy + (float)(CAT_H - t));
    w[CAT_D] = fx;
#pragma unroll
    for (int t = CAT_D + 1; t < CAT_REC; ++t) w[t] = 0.0f;
#pragma unroll
    for (int k = 0; k < CAT_REC / 4; ++k)
      rec[(size_t)q * (CAT_REC / 4) + k] = make_float4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
    const uint32_t k = skey[q];
    const uint32_t kp = q == 0 ? 0u : skey[q - 1] + 1u;
    for (uint32_t c = kp; c <= k; ++c) cellStart[c] = q;
    if (q == ngal - 1)
      for (uint32_t c = k + 1; c <= ncell; ++c) cellStart[c] = ngal;
  }
}

// To the sorted order, dst = src[c][perm[g]] at [c][g] (planar) or [g][c] (interleaved), or back,
// dst[c][perm[g]] = src at [c][g] or [g][c]
__global__ void k_cat_permute(const float* __restrict__ src, const int* __restrict__ perm, float* __restrict__ dst,
                              int ngal, int C, int gather, int inter) {
  const int64_t tot = (int64_t)C * ngal;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e / ngal), g = (int)(e % ngal);
    const int64_t s = inter ? (int64_t)g * C + c : e;   // sorted side
    if (gather)
      dst[s] = src[(int64_t)c * ngal + perm[g]];
    else
      dst[(int64_t)c * ngal + perm[g]] = src[s];
  }
}

}  // namespace wf
