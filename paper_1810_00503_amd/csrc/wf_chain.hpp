// Transform chain of one evaluation of the objective's gradient or curvature product:
//
//   column pass (inverse):  rotate (spin-2) and scale the half-plane field, complete the
//                           kx = 0 column by Hermitian symmetry, inverse FFT along ky;
//   row pass:               per image row, complex-to-real inverse FFT along kx, the pixel
//                           operation (W x, W (x - d), simulation noise), chi^2 partials,
//                           real-to-complex forward FFT;
//   column pass (forward):  forward FFT along ky, inverse rotation, prior scale and the
//                           added term, dot-product partials.
//
// Every pass stages its tile in LDS and transforms it with the Stockham FFT of
// wf_fft.hpp.  A work-group of the column passes owns CPB column blocks of TB columns
// (both components; each block contiguous in memory); a work-group of the row pass owns
// RBV rows.  CPB and RBV are tile choices made per problem shape by the autotuner.
#pragma once
#include "wf_fft.hpp"

namespace wf {

// ------------------------------------------------------------------------ Philox4x32-10
// Salmon, Moraes, Dror & Shaw (SC'11): ten rounds of two 32x32 -> 64-bit products with
// multipliers 0xD2511F53 / 0xCD9E8D57, Weyl key increments 0x9E3779B9 / 0xBB67AE85.
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                              uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Normals q and q + 1 (q even) of simulation `sim`: Box-Muller of the Philox pair that
// holds them, in float64.
__device__ __forceinline__ void philox_normal_pair(uint64_t seed, int sim, int64_t q, double& z0, double& z1) {
  uint32_t c0 = (uint32_t)(q >> 2), c1 = (uint32_t)sim, c2 = 0u, c3 = 0u;
  philox4x32_10(c0, c1, c2, c3, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
  const bool hi = (q & 2) != 0;
  const uint32_t xa = hi ? c2 : c0, xb = hi ? c3 : c1;
  const double u0 = ((double)xa + 0.5) * 2.3283064365386963e-10;
  const double u1 = ((double)xb + 0.5) * 2.3283064365386963e-10;
  const double r = sqrt(-2.0 * log(u0));
  const double ang = 6.283185307179586 * u1;
  z0 = r * cos(ang);
  z1 = r * sin(ang);
}

// ------------------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the work-group (NT threads); result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) t += red[i];
  }
  return t;
}

// spin-2 rotation coefficients cos 2a, sin 2a at integer (kx, ky) (exact rationals)
template <typename T>
__device__ __forceinline__ void rot2(int kx, int kys, T& c2, T& s2) {
  const T fx = T(kx), fy = T(kys);
  const T k2 = fx * fx + fy * fy;
  if (k2 > T(0)) {
    const T inv = T(1) / k2;
    c2 = (fx * fx - fy * fy) * inv;
    s2 = T(2) * fx * fy * inv;
  } else {
    c2 = T(1);
    s2 = T(0);
  }
}

template <typename T>
__device__ __forceinline__ size_t chain_lds_col(int N, int C) { return (size_t)(N + N * C * TB) * sizeof(cpx<T>); }

// ------------------------------------------------------------------------ column inverse
template <typename T, int N, int C, int CPB>
__global__ __launch_bounds__(NT) void k_colinv(const Job* __restrict__ jobs, const cpx<T>* __restrict__ twg) {
  const Job& jb = jobs[blockIdx.y];
  const int mode = jb.mode;
  if (mode == CM_NONE || mode == CM_ADJ || mode == CM_ADJ_GRAD) return;
  constexpr int NB = CPB * C * TB;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* buf = tw + N;
  __shared__ double red[NT / 64];
  const int tid = threadIdx.x, q = blockIdx.x;
  for (int i = tid; i < N; i += NT) tw[i] = twg[i];

  const cpx<T>* vin = reinterpret_cast<const cpx<T>*>(jb.vin);
  const T* sIn = reinterpret_cast<const T*>(jb.sIn);
  const T* sOut = reinterpret_cast<const T*>(jb.sOut);
  const bool raw = (mode == CM_RAW_GRAD || mode == CM_RAW_HV);
  const bool sim = (mode == CM_SIM);
  const T* draws = reinterpret_cast<const T*>(jb.draws);
  const T bamp = T(jb.boost_factor);
  double acc = 0.0;
  for (int ee = tid; ee < CPB * N * TB; ee += NT) {
    const int cb = ee / (N * TB), e = ee % (N * TB);
    const int qb = q * CPB + cb;                     // column block
    const int ky = e / TB, col = e % TB, kx = qb * TB + col;
    // offset of this column block in the (chunk-interleaved) input view
    int64_t dv[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int64_t bs = fidx(N, c, 0, qb * TB);
      dv[c] = jb.vcs > 0 ? vview(bs, jb.vcs, jb.vcstr) - bs : 0;
    }
    cpx<T> a[C];
#pragma unroll
    for (int c = 0; c < C; ++c) a[c] = mk(T(0), T(0));
    if (is_live(N, ky, kx)) {
      const bool part = is_partner(N, ky, kx);
      const int kyr = part ? N - ky : ky;   // stored (free) entry of the pair
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int64_t src = fidx(N, c, kyr, kx);
        cpx<T> v;
        T sc = T(1);
        if (sim) {
          const int64_t qn = ((int64_t)c * N + kyr) * N + 2 * kx;
          if (draws) {
            v = mk(draws[qn], draws[qn + 1]);
          } else {
            double z0, z1;
            philox_normal_pair(jb.seed, jb.sim, qn, z0, z1);
            v = mk(T(z0), T(z1));
          }
          sc = sIn[src] * T(0.70710678118654752440084436210485);
          if (jb.band && jb.boost_band >= 0 && jb.band[src] == jb.boost_band) sc *= bamp;
        } else {
          v = vin[src + dv[c]];
          if (sIn) sc = sIn[src];
          if (raw) {
            const T sq = sOut[src];
            if (sq == T(0)) {
              v = mk(T(0), T(0));
            } else if (!part && mode == CM_RAW_GRAD) {
              acc += ((double)v.x * v.x + (double)v.y * v.y) / ((double)sq * sq);
            }
          } else if (mode == CM_GRAD && !part) {
            const double wa = jb.aTab ? (double)reinterpret_cast<const T*>(jb.aTab)[src] : 1.0;
            acc += wa * ((double)v.x * v.x + (double)v.y * v.y);
          }
        }
        a[c] = scale(v, sc);
      }
      if constexpr (C == 2) {
        T c2, s2;
        rot2<T>(kx, kyr < N / 2 ? kyr : kyr - N, c2, s2);
        const cpx<T> e0 = a[0], b0 = a[1];
        a[0] = mk(c2 * e0.x - s2 * b0.x, c2 * e0.y - s2 * b0.y);
        a[1] = mk(s2 * e0.x + c2 * b0.x, s2 * e0.y + c2 * b0.y);
      }
      if (part) {
#pragma unroll
        for (int c = 0; c < C; ++c) a[c] = conj(a[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) buf[ky * NB + (cb * C + c) * TB + col] = a[c];
  }
  __syncthreads();
  lds_fft<T, N, NB, 1, NB, 1, false, true>(buf, tw);

  cpx<T>* y = reinterpret_cast<cpx<T>*>(jb.y);
  for (int ee = tid; ee < CPB * N * TB; ee += NT) {
    const int cb = ee / (N * TB), e = ee % (N * TB);
    const int ky = e / TB, col = e % TB;
#pragma unroll
    for (int c = 0; c < C; ++c) y[fidx(N, c, 0, (q * CPB + cb) * TB) + e] = buf[ky * NB + (cb * C + c) * TB + col];
  }
  if (mode == CM_GRAD || mode == CM_RAW_GRAD) {
    const double t = block_sum(acc, red);
    if (tid < CPB) jb.part[PK_PRIOR * jb.pstride + q * CPB + tid] = tid == 0 ? t : 0.0;
  }
}

// ------------------------------------------------------------------------ row pass
template <typename T, int N, int C, int RBV>
__global__ __launch_bounds__(NT) void k_row(const Job* __restrict__ jobs, const cpx<T>* __restrict__ twg) {
  const Job& jb = jobs[blockIdx.y];
  const int mode = jb.mode;
  if (mode == CM_NONE) return;
  constexpr int RB = RBV;
  constexpr int H = N / 2, NBR = C * RB, SBR = H;
  constexpr int NE = NBR * H;
  constexpr int KP = (NE + NT - 1) / NT;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* buf = tw + N;
  __shared__ double red[NT / 64];
  const int tid = threadIdx.x, y0 = blockIdx.x * RB;
  for (int i = tid; i < N; i += NT) tw[i] = twg[i];

  const bool adjIn = (mode == CM_ADJ || mode == CM_ADJ_GRAD);
  cpx<T>* Y = reinterpret_cast<cpx<T>*>(jb.y);

  if (!adjIn) {
    for (int e = tid; e < NE; e += NT) {
      const int c = e / (RB * H), r2 = e % (RB * H);
      const int qq = r2 / (RB * TB), w2 = r2 % (RB * TB);
      const int yl = w2 / TB, col = w2 % TB;
      buf[(c * RB + yl) * SBR + qq * TB + col] = Y[fidx(N, c, y0, qq * TB) + w2];
    }
    __syncthreads();
    // complex-to-real pre-processing (X_{n/2} = 0, X_0 taken real):
    //   Z_k = (X_k + conj X_{H-k}) + i w^-k (X_k - conj X_{H-k}),  w = exp(-2 pi i / N)
    cpx<T> z[KP];
#pragma unroll
    for (int kk = 0; kk < KP; ++kk) {
      const int u = tid + kk * NT;
      if ((NE % NT == 0) || u < NE) {
        const int b = u / H, k = u % H;
        const cpx<T> X = buf[b * SBR + k];
        if (k == 0) {
          z[kk] = mk(X.x, X.x);
        } else {
          const cpx<T> Xm = conj(buf[b * SBR + H - k]);
          const cpx<T> t = mulc(sub(X, Xm), tw[k]);   // w^-k (X - Xm)
          const cpx<T> s = add(X, Xm);
          z[kk] = mk(s.x - t.y, s.y + t.x);           // s + i t
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KP; ++kk) {
      const int u = tid + kk * NT;
      if ((NE % NT == 0) || u < NE) buf[(u / H) * SBR + (u % H)] = z[kk];
    }
    __syncthreads();
    lds_fft<T, H, NBR, SBR, 1, 2, true, true>(buf, tw);
  }

  // pixel operation: element j of row b holds pixels (2j, 2j+1)
  const T invn = T(1) / T(N);
  const T* W = reinterpret_cast<const T*>(jb.W);
  const T* dd = reinterpret_cast<const T*>(jb.d);
  T* xout = reinterpret_cast<T*>(jb.xout);
  const T* draws = reinterpret_cast<const T*>(jb.draws);
  double acc = 0.0;
  for (int e = tid; e < NE; e += NT) {
    const int b = e / H, j = e % H;
    const int c = b / RB, yl = b % RB;
    const int64_t pix = (int64_t)(y0 + yl) * N + 2 * j;
    const int64_t cp = (int64_t)c * N * N + pix;
    cpx<T> zf;
    if (adjIn) {
      T x0 = dd[cp], x1 = dd[cp + 1];
      if (W) {   // masked adjoint: R^T M x
        if (!(W[pix] > T(0))) x0 = T(0);
        if (!(W[pix + 1] > T(0))) x1 = T(0);
      }
      zf = mk(x0 * invn, x1 * invn);
    } else {
      const cpx<T> zz = buf[b * SBR + j];
      const T x0 = zz.x * invn, x1 = zz.y * invn;
      if (mode == CM_FWD) {   // masked forward M R s when W is given
        xout[cp] = (W && !(W[pix] > T(0))) ? T(0) : x0;
        xout[cp + 1] = (W && !(W[pix + 1] > T(0))) ? T(0) : x1;
        continue;
      }
      const T W0 = W[pix], W1 = W[pix + 1];
      if (mode == CM_SIM) {
        T n0, n1;
        const int64_t qn = (int64_t)C * N * N + cp;
        if (draws) {
          n0 = draws[qn];
          n1 = draws[qn + 1];
        } else {
          double z0, z1;
          philox_normal_pair(jb.seed, jb.sim, qn, z0, z1);
          n0 = T(z0);
          n1 = T(z1);
        }
        xout[cp] = W0 > T(0) ? x0 + n0 / sqrt(W0) : T(0);
        xout[cp + 1] = W1 > T(0) ? x1 + n1 / sqrt(W1) : T(0);
        continue;
      }
      T r0, r1;
      if (mode == CM_HV || mode == CM_RAW_HV) {
        r0 = W0 * x0;
        r1 = W1 * x1;
      } else {  // CM_GRAD, CM_RAW_GRAD: r = W (x - d); masked pixels contribute nothing
        r0 = T(0);
        r1 = T(0);
        if (W0 > T(0)) {
          const T e0 = x0 - dd[cp];
          r0 = W0 * e0;
          acc += (double)r0 * e0;
        }
        if (W1 > T(0)) {
          const T e1 = x1 - dd[cp + 1];
          r1 = W1 * e1;
          acc += (double)r1 * e1;
        }
      }
      zf = mk(r0 * invn, r1 * invn);
    }
    buf[b * SBR + j] = zf;
  }
  if (mode == CM_FWD || mode == CM_SIM) return;
  __syncthreads();
  lds_fft<T, H, NBR, SBR, 1, 2, true, false>(buf, tw);
  // real-to-complex post-processing:
  //   X_k = 1/2 (Z_k + conj Z_{H-k}) - i/2 w^k (Z_k - conj Z_{H-k}),  Z_H = Z_0
  cpx<T> xr[KP];
#pragma unroll
  for (int kk = 0; kk < KP; ++kk) {
    const int u = tid + kk * NT;
    if ((NE % NT == 0) || u < NE) {
      const int b = u / H, k = u % H;
      const cpx<T> Zk = buf[b * SBR + k];
      const cpx<T> Zm = conj(buf[b * SBR + (k == 0 ? 0 : H - k)]);
      const cpx<T> A = add(Zk, Zm);
      const cpx<T> t = mul(tw[k], sub(Zk, Zm));
      xr[kk] = mk(T(0.5) * (A.x + t.y), T(0.5) * (A.y - t.x));
    }
  }
  __syncthreads();
#pragma unroll
  for (int kk = 0; kk < KP; ++kk) {
    const int u = tid + kk * NT;
    if ((NE % NT == 0) || u < NE) buf[(u / H) * SBR + (u % H)] = xr[kk];
  }
  __syncthreads();
  for (int e = tid; e < NE; e += NT) {
    const int c = e / (RB * H), r2 = e % (RB * H);
    const int qq = r2 / (RB * TB), w2 = r2 % (RB * TB);
    const int yl = w2 / TB, col = w2 % TB;
    Y[fidx(N, c, y0, qq * TB) + w2] = buf[(c * RB + yl) * SBR + qq * TB + col];
  }
  if (mode == CM_GRAD || mode == CM_RAW_GRAD) {
    // partials are kept per RB_MIN rows so the reduction does not depend on RBV
    const double t = block_sum(acc, red);
    if (tid < RB / RB_MIN) jb.part[PK_RES * jb.pstride + blockIdx.x * (RB / RB_MIN) + tid] = tid == 0 ? t : 0.0;
  }
}

// ------------------------------------------------------------------------ column forward
template <typename T, int N, int C, int CPB>
__global__ __launch_bounds__(NT) void k_colfwd(const Job* __restrict__ jobs, const cpx<T>* __restrict__ twg) {
  const Job& jb = jobs[blockIdx.y];
  const int mode = jb.mode;
  if (mode == CM_NONE || mode == CM_FWD || mode == CM_SIM) return;
  constexpr int NB = CPB * C * TB;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* buf = tw + N;
  __shared__ double red[NT / 64];
  const int tid = threadIdx.x, q = blockIdx.x;
  for (int i = tid; i < N; i += NT) tw[i] = twg[i];
  const cpx<T>* Y = reinterpret_cast<const cpx<T>*>(jb.y);
  for (int ee = tid; ee < CPB * N * TB; ee += NT) {
    const int cb = ee / (N * TB), e = ee % (N * TB);
    const int ky = e / TB, col = e % TB;
#pragma unroll
    for (int c = 0; c < C; ++c) buf[ky * NB + (cb * C + c) * TB + col] = Y[fidx(N, c, 0, (q * CPB + cb) * TB) + e];
  }
  __syncthreads();
  lds_fft<T, N, NB, 1, NB, 1, false, false>(buf, tw);

  const cpx<T>* vadd = reinterpret_cast<const cpx<T>*>(jb.vadd);
  const T* sOut = reinterpret_cast<const T*>(jb.sOut);
  cpx<T>* vout = reinterpret_cast<cpx<T>*>(jb.vout);
  double avo = 0.0, aoo = 0.0, adg = 0.0;
  double add[MMAX];
#pragma unroll
  for (int j = 0; j < MMAX; ++j) add[j] = 0.0;
  // curvature products inside the solver also dot the new Dp with g and the kept Dp_j
  const bool extras = (mode == CM_HV) && jb.dpBase != nullptr;
  const cpx<T>* gvec = reinterpret_cast<const cpx<T>*>(jb.gvec);
  const cpx<T>* dpb = reinterpret_cast<const cpx<T>*>(jb.dpBase);
  for (int ee = tid; ee < CPB * N * TB; ee += NT) {
    const int cb = ee / (N * TB), e = ee % (N * TB);
    const int qb = q * CPB + cb;
    const int ky = e / TB, col = e % TB, kx = qb * TB + col;
    int64_t dv[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int64_t bs = fidx(N, c, 0, qb * TB);
      dv[c] = jb.vcs > 0 ? vview(bs, jb.vcs, jb.vcstr) - bs : 0;
    }
    cpx<T> t[C];
#pragma unroll
    for (int c = 0; c < C; ++c) t[c] = buf[ky * NB + (cb * C + c) * TB + col];
    if constexpr (C == 2) {
      T c2, s2;
      rot2<T>(kx, ky < N / 2 ? ky : ky - N, c2, s2);
      const cpx<T> g1 = t[0], g2 = t[1];
      t[0] = mk(c2 * g1.x + s2 * g2.x, c2 * g1.y + s2 * g2.y);
      t[1] = mk(-s2 * g1.x + c2 * g2.x, -s2 * g1.y + c2 * g2.y);
    }
    const bool fr = is_free(N, ky, kx);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int64_t o = fidx(N, c, ky, kx);
      cpx<T> out = mk(T(0), T(0));
      if (mode == CM_HV || mode == CM_GRAD) {
        const T sq = sOut[o];
        if (fr && sq != T(0)) {
          const cpx<T> v = vadd[o + dv[c]];
          const T wa = jb.aTab ? reinterpret_cast<const T*>(jb.aTab)[o] : T(1);
          out = mk(wa * v.x + sq * t[c].x, wa * v.y + sq * t[c].y);
          avo += (double)v.x * out.x + (double)v.y * out.y;
        }
        aoo += (double)out.x * out.x + (double)out.y * out.y;
        if (extras) {
          const cpx<T> gv = gvec[o + dv[c]];
          adg += (double)gv.x * out.x + (double)gv.y * out.y;
#pragma unroll
          for (int j = 0; j < MMAX; ++j) {
            if ((jb.dpMask >> j) & 1u) {
              const cpx<T> dj = dpb[(int64_t)j * jb.dpStride + o + dv[c]];
              add[j] += (double)dj.x * out.x + (double)dj.y * out.y;
            }
          }
        }
      } else if (mode == CM_RAW_GRAD || mode == CM_RAW_HV) {
        const T sq = sOut[o];
        if (fr && sq != T(0)) {
          const cpx<T> v = vadd[o + dv[c]];
          const T is = T(1) / (sq * sq);
          out = mk(T(4) * (v.x * is + t[c].x), T(4) * (v.y * is + t[c].y));
        }
      } else if (mode == CM_ADJ) {
        if (is_live(N, ky, kx)) out = t[c];
      } else {  // CM_ADJ_GRAD
        if (fr) out = scale(t[c], T(2));
      }
      vout[o + dv[c]] = out;
    }
  }
  if (mode == CM_HV || mode == CM_GRAD) {
    // one combined reduction: [VO, OO, DG, DD_0 .. DD_{MMAX-1}] -> kinds PK_VO + idx
    __shared__ double red2[NT / 64][3 + MMAX];
    const int lane = tid & 63, wv = tid >> 6;
    const int nv = extras ? 3 + MMAX : 2;
    const uint32_t mask = jb.dpMask;
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
    if (tid < nv && (tid < 3 || ((mask >> (tid - 3)) & 1u))) {
      double sum = 0.0;
#pragma unroll
      for (int k = 0; k < NT / 64; ++k) sum += red2[k][tid];
      jb.part[(PK_VO + tid) * jb.pstride + q * CPB] = sum;
#pragma unroll
      for (int cb = 1; cb < CPB; ++cb) jb.part[(PK_VO + tid) * jb.pstride + q * CPB + cb] = 0.0;
    }
  }
}

}  // namespace wf
