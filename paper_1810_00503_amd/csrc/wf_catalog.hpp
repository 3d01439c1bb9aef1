// Catalog-level response (sec. 3.4): the field of the harmonic coefficients evaluated at each
// galaxy's own position instead of binned pixels, gamma(r_g) = n^-1 sum_k gamma~_k
// exp(2 pi i k.r_g / n), and its adjoint, as a non-uniform FFT on a fine grid of N = 2n
// points per side:
//
//   pad      coarse field -> fine half-plane spectrum, each band mode scaled by T_k
//            = (prior scale) (N/n) / (phi^(ky/N) phi^(kx/N)) (deconvolution of the kernel);
//   forward  the transform passes of the chain at size N (column inverse, row) -> fine map u;
//   interp   per galaxy, sum of u over the CAT_W x CAT_W fine points around rho = 2 r with
//            the separable exponential-of-semicircle kernel phi -> gamma(r_g), and the
//            weighted residual (solver) or the value (forward operator);
//   spread   the adjoint of interp: per fine-grid tile, each point gathers phi-weighted
//            residuals of the galaxies whose window covers it (deterministic order);
//   adjoint  the transform passes at size N (row, column forward) -> fine spectrum;
//   unpad    band modes back to the coarse layout, times T_k, plus the solver's prior term
//            and the dot partials of the chain's column-forward pass.
//
// Inside the batched solver these replace the three coarse passes of a curvature product or
// exact gradient; the jobs the solver writes each iteration drive them as they drive the
// chain.  The kernel: phi(z) = exp(beta (sqrt(1 - (2z/W)^2) - 1)) on |z| <= W/2, beta = 2.3 W for
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

// first fine point of a galaxy's window, ceil(rho - W/2), and the CAT_W weights phi(rho - j)
__device__ __forceinline__ int es_window(int cell, float frac, float (&w)[CAT_W]) {
  const int off = frac > 0.0f ? -(CAT_W / 2 - 1) : -(CAT_W / 2);
#pragma unroll
  for (int t = 0; t < CAT_W; ++t) w[t] = es_kernel(frac - (float)(off + t));
  return cell + off;
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
  if ((int)blockIdx.x * NT >= cd.ngal) return;   // the grid covers the class's largest catalog
  __shared__ double red[NT / 64];
  const int g = blockIdx.x * NT + threadIdx.x;
  double acc = 0.0;
  if (g < cd.ngal) {
    const int N = cd.N;
    const GalPos gp = cd.pos[g];
    float wy[CAT_W], wx[CAT_W];
    const int jy0 = es_window(gp.cy, gp.fy, wy), jx0 = es_window(gp.cx, gp.fx, wx);
    int jx[CAT_W];
#pragma unroll
    for (int t = 0; t < CAT_W; ++t) jx[t] = (jx0 + t + N) % N;
    float gam[C];
#pragma unroll
    for (int cc = 0; cc < C; ++cc) gam[cc] = 0.0f;
#pragma unroll
    for (int ty = 0; ty < CAT_W; ++ty) {
      const int jy = (jy0 + ty + N) % N;
#pragma unroll
      for (int cc = 0; cc < C; ++cc) {
        const float* row = cd.u + ((size_t)cc * N + jy) * N;
        float a = 0.0f;
#pragma unroll
        for (int tx = 0; tx < CAT_W; ++tx) a += wx[tx] * row[jx[tx]];
        gam[cc] += wy[ty] * a;
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
      cd.r[(size_t)cc * cd.ngal + g] = r;
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
      cd.partI[blockIdx.x] = t;
    }
  }
}

// ------------------------------------------------------------------------ spreading
// grid (tiles * tiles, instances), NT = CAT_TS^2 threads, one fine point each: v(j) = sum over
// the galaxies of the tile and its neighbours (whose windows can reach it) of phi phi r, the
// galaxies staged through LDS in chunks of NT and summed in their sorted order.  Block 0 of an
// exact gradient also reduces the interpolation's chi^2 partials (one per NT galaxies) into
// the residual slots the solver reads.
template <int C>
__global__ __launch_bounds__(NT) void k_cat_spread(const Job* __restrict__ jobs, const CatDesc* __restrict__ cats) {
  const int i = blockIdx.y;
  const Job& jb = jobs[i];
  const int mode = jb.mode;
  if (!(cat_solver_mode(mode) || mode == CM_ADJ || mode == CM_ADJ_GRAD)) return;
  const CatDesc& cd = cats[i];
  const int tiles = cd.tiles, N = cd.N;
  if (mode == CM_GRAD && blockIdx.x == 0) {
    double t = 0.0;
    if (threadIdx.x == 0)
      for (int k = 0; k < (cd.ngal + NT - 1) / NT; ++k) t += cd.partI[k];
    for (int k = threadIdx.x; k < cd.nrowPart; k += NT) jb.part[PK_RES * jb.pstride + k] = k == 0 ? t : 0.0;
  }
  if ((int)blockIdx.x >= tiles * tiles) return;
  __shared__ int sjy[NT], sjx[NT];
  __shared__ float swy[NT][CAT_W + 1], swx[NT][CAT_W + 1];
  __shared__ float sr[C][NT];
  const int ty = blockIdx.x / tiles, tx = blockIdx.x % tiles;
  const int jy = ty * CAT_TS + (int)threadIdx.x / CAT_TS, jx = tx * CAT_TS + (int)threadIdx.x % CAT_TS;
  float acc[C];
#pragma unroll
  for (int cc = 0; cc < C; ++cc) acc[cc] = 0.0f;
  // distinct neighbour tiles: all three offsets, or every tile of a grid of fewer than three
  const int nd = tiles >= 3 ? 3 : tiles;
  for (int ay = 0; ay < nd; ++ay) {
    for (int ax = 0; ax < nd; ++ax) {
      const int ny = (ty + (nd == 3 ? ay - 1 : ay) + tiles) % tiles;
      const int nx = (tx + (nd == 3 ? ax - 1 : ax) + tiles) % tiles;
      const int nt = ny * tiles + nx;
      const int g0 = cd.tileStart[nt], g1 = cd.tileStart[nt + 1];
      for (int base = g0; base < g1; base += NT) {
        const int cnt = min(NT, g1 - base);
        __syncthreads();
        if ((int)threadIdx.x < cnt) {
          const int g = base + threadIdx.x;
          const GalPos gp = cd.pos[g];
          float wy[CAT_W], wx[CAT_W];
          sjy[threadIdx.x] = es_window(gp.cy, gp.fy, wy);
          sjx[threadIdx.x] = es_window(gp.cx, gp.fx, wx);
#pragma unroll
          for (int t = 0; t < CAT_W; ++t) {
            swy[threadIdx.x][t] = wy[t];
            swx[threadIdx.x][t] = wx[t];
          }
#pragma unroll
          for (int cc = 0; cc < C; ++cc) sr[cc][threadIdx.x] = cd.r[(size_t)cc * cd.ngal + g];
        }
        __syncthreads();
        for (int q = 0; q < cnt; ++q) {
          const int oy = (jy - sjy[q] + 2 * N) % N;
          const int ox = (jx - sjx[q] + 2 * N) % N;
          if (oy < CAT_W && ox < CAT_W) {
            const float w = swy[q][oy] * swx[q][ox];
#pragma unroll
            for (int cc = 0; cc < C; ++cc) acc[cc] += w * sr[cc][q];
          }
        }
      }
    }
  }
#pragma unroll
  for (int cc = 0; cc < C; ++cc) cd.v[((size_t)cc * N + jy) * N + jx] = acc[cc];
}

// ------------------------------------------------------------------------ unpad
// grid (n / 4 coarse column blocks, instances): the fine spectrum t of the band modes back on
// the coarse layout; solver modes: out = wa v + T t on the free modes with the dot partials
// [VO, OO, DG, DD_j] of the column-forward pass (one slot per column block); operator modes:
// out = T t on the live modes (metric adjoint) or 2 T t on the free ones (gradient form).
template <int C>
__global__ __launch_bounds__(NT) void k_cat_unpad(const Job* __restrict__ jobs, const CatDesc* __restrict__ cats) {
  const int i = blockIdx.y;
  const Job& jb = jobs[i];
  const int mode = jb.mode;
  if (!(cat_solver_mode(mode) || mode == CM_ADJ || mode == CM_ADJ_GRAD)) return;
  const CatDesc& cd = cats[i];
  __shared__ double red2[NT / 64][3 + MMAX];
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
  for (int e = threadIdx.x; e < C * n * TB; e += NT) {
    const int cc = e / (n * TB), r = e % (n * TB), ky = r / TB, kx = 2 * b + r % TB;
    const uint32_t o = (uint32_t)fidx(n, cc, ky, kx);
    const int KY = ky < h ? ky : ky - n + N;
    const float T = cd.T[o];
    cpx<float> out = mk(0.0f, 0.0f);
    if (solver) {
      if (T != 0.0f && is_free(n, ky, kx)) {
        const cpx<float> t = y2[fidx(N, cc, KY, kx)];
        const cpx<float> a = reinterpret_cast<const cpx<float>*>(jb.vadd)[o];
        const float wa = cd.aTab ? cd.aTab[o] : 1.0f;
        out = mk(wa * a.x + T * t.x, wa * a.y + T * t.y);
        avo += (double)a.x * out.x + (double)a.y * out.y;
      }
      aoo += (double)out.x * out.x + (double)out.y * out.y;
      if (extras) {
        const cpx<float> gv = reinterpret_cast<const cpx<float>*>(jb.gvec)[o];
        adg += (double)gv.x * out.x + (double)gv.y * out.y;
        const cpx<float>* dpb = reinterpret_cast<const cpx<float>*>(jb.dpBase);
#pragma unroll
        for (int j = 0; j < MMAX; ++j) {
          if ((mask >> j) & 1u) {
            const cpx<float> dj = dpb[(int64_t)j * jb.dpStride + o];
            add[j] += (double)dj.x * out.x + (double)dj.y * out.y;
          }
        }
      }
    } else if (mode == CM_ADJ) {
      if (is_live(n, ky, kx)) {
        const cpx<float> t = y2[fidx(N, cc, KY, kx)];
        out = mk(T * t.x, T * t.y);
      }
    } else if (is_free(n, ky, kx)) {
      const cpx<float> t = y2[fidx(N, cc, KY, kx)];
      out = mk(2.0f * T * t.x, 2.0f * T * t.y);
    }
    vout[o] = out;
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
    for (int k = 0; k < NT / 64; ++k) sum += red2[k][tid];
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

// dst[c][g] = src[c][perm[g]] (to the sorted order) or dst[c][perm[g]] = src[c][g] (back)
__global__ void k_cat_permute(const float* __restrict__ src, const int* __restrict__ perm, float* __restrict__ dst,
                              int ngal, int C, int gather) {
  const int64_t tot = (int64_t)C * ngal;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e / ngal), g = (int)(e % ngal);
    if (gather)
      dst[e] = src[(int64_t)c * ngal + perm[g]];
    else
      dst[(int64_t)c * ngal + perm[g]] = src[e];
  }
}

}  // namespace wf
