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
// wf_fft.hpp; for power-of-two grids in float32 a register-staged variant of each pass
// (wf_rfft.hpp, end of this file) keeps the transform in registers between LDS exchanges.  A work-group of the column passes owns CPB column blocks of TB columns
// (both components; each block contiguous in memory); a work-group of the row pass owns
// RBV rows.  CPB and RBV are tile choices made per problem shape by the autotuner.
#pragma once
#include "wf_rfft.hpp"

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
// holds them, u = (x + 1/2) 2^-32.  R = double for float64 fields; float32 fields take the
// transform in float32 (the hardware log, square root and sine/cosine), whose few-ulp
// differences from the float64 transform are below the fields' own rounding.
template <typename R>
__device__ __forceinline__ void philox_normal_pair(uint64_t seed, int sim, int64_t q, R& z0, R& z1) {
  uint32_t c0 = (uint32_t)(q >> 2), c1 = (uint32_t)sim, c2 = 0u, c3 = 0u;
  philox4x32_10(c0, c1, c2, c3, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
  const bool hi = (q & 2) != 0;
  const uint32_t xa = hi ? c2 : c0, xb = hi ? c3 : c1;
  if constexpr (sizeof(R) == 8) {
    const double u0 = ((double)xa + 0.5) * 2.3283064365386963e-10;
    const double u1 = ((double)xb + 0.5) * 2.3283064365386963e-10;
    const double r = sqrt(-2.0 * log(u0));
    const double ang = 6.283185307179586 * u1;
    z0 = r * cos(ang);
    z1 = r * sin(ang);
  } else {
    const float u0 = ((float)xa + 0.5f) * 2.3283064365386963e-10f;
    const float u1 = ((float)xb + 0.5f) * 2.3283064365386963e-10f;
    const float r = sqrtf(-2.0f * logf(u0));
    float sn, cs;
    sincosf(6.2831853071795865f * u1, &sn, &cs);
    z0 = r * cs;
    z1 = r * sn;
  }
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

// ------------------------------------------------------------------------ traversal order
// Consecutive passes over a batch walk the instances in opposite orders (column passes and
// the solver's direction pass forward, the row pass and the passes after the column-forward
// one in reverse), so each pass starts on the instances whose vectors the previous pass
// wrote last, which a batch the size of the memory-side cache still holds there.
__device__ __forceinline__ int rev_instance() { return (int)(gridDim.y - 1 - blockIdx.y); }

// ------------------------------------------------------------------------ per-element steps
// Column-inverse input of component c at (ky, kx): scale (sqrt S, simulation amplitude),
// liveness, prior partial (gradient modes).  Returns the value before the spin-2 rotation;
// part/kyr tell whether (ky, kx) is a kx = 0 conjugate partner and which stored row holds its
// free entry.  SIMK: the simulation mode
// (normals from draws or Philox) is compiled in; it costs registers, so only the
// kernels that simulation launches use it.
template <typename T, int N, bool SIMK>
__device__ __forceinline__ cpx<T> colinv_in(const Job& jb, int mode, int c, int ky, int kx, bool& part,
                                            int& kyr, double& acc) {
  cpx<T> a = mk(T(0), T(0));
  part = false;
  kyr = ky;
  if (!is_live(N, ky, kx)) return a;
  part = is_partner(N, ky, kx);
  kyr = part ? N - ky : ky;
  const uint32_t src = (uint32_t)fidx(N, c, kyr, kx);
  const T* sIn = reinterpret_cast<const T*>(jb.sIn);
  cpx<T> v;
  T sc = T(1);
  if (SIMK && mode == CM_SIM) {
    const T* draws = reinterpret_cast<const T*>(jb.draws);
    const int64_t qn = ((int64_t)c * N + kyr) * N + 2 * kx;
    if (draws) {
      v = mk(draws[qn], draws[qn + 1]);
    } else {
      T z0, z1;
      philox_normal_pair<T>(jb.seed, jb.sim, qn, z0, z1);
      v = mk(z0, z1);
    }
    sc = gld(sIn, src) * T(0.70710678118654752440084436210485);
    if (jb.band && jb.boost_band >= 0 && gld(jb.band, src) == jb.boost_band) sc *= T(jb.boost_factor);
  } else {
    v = gld(reinterpret_cast<const cpx<T>*>(jb.vin), src);
    if (sIn) sc = gld(sIn, src);
    if (mode == CM_RAW_GRAD || mode == CM_RAW_HV) {
      const T sq = gld(reinterpret_cast<const T*>(jb.sOut), src);
      if (sq == T(0)) {
        v = mk(T(0), T(0));
      } else if (!part && mode == CM_RAW_GRAD) {
        acc += ((double)v.x * v.x + (double)v.y * v.y) / ((double)sq * sq);
      }
    } else if (mode == CM_GRAD && !part) {
      const double wa = jb.aTab ? (double)gld(reinterpret_cast<const T*>(jb.aTab), src) : 1.0;
      acc += wa * ((double)v.x * v.x + (double)v.y * v.y);
    }
  }
  return scale(v, sc);
}

// The same for the curvature and gradient modes, whitened or raw (CM_HV, CM_GRAD,
// CM_RAW_HV, CM_RAW_GRAD), split in two so that a thread issues the global loads of all its
// elements (colinv_ld) before the arithmetic of the first (colinv_fin): a load behind a
// data-dependent branch waits for the loads before it, so the one-call form costs a memory
// round trip per element.  wa is the solver weight (whitened) or the sqrt S of sOut (raw).
__device__ __forceinline__ bool colinv_hot(int mode) {
  return mode == CM_HV || mode == CM_GRAD || mode == CM_RAW_HV || mode == CM_RAW_GRAD;
}
template <typename T, int N>
__device__ __forceinline__ void colinv_ld(const Job& jb, bool grad, bool raw, int c, int ky, int kx, cpx<T>& v,
                                          T& sc, T& wa) {
  const uint32_t src = (uint32_t)fidx(N, c, is_partner(N, ky, kx) ? N - ky : ky, kx);
  v = gld(reinterpret_cast<const cpx<T>*>(jb.vin), src);
  sc = jb.sIn ? gld(reinterpret_cast<const T*>(jb.sIn), src) : T(1);
  if (raw) wa = gld(reinterpret_cast<const T*>(jb.sOut), src);
  else wa = (grad && jb.aTab) ? gld(reinterpret_cast<const T*>(jb.aTab), src) : T(1);
}
template <typename T, int N>
__device__ __forceinline__ cpx<T> colinv_fin(bool grad, bool raw, int ky, int kx, cpx<T> v, T sc, T wa, bool& part,
                                             int& kyr, double& acc) {
  part = false;
  kyr = ky;
  if (!is_live(N, ky, kx)) return mk(T(0), T(0));
  part = is_partner(N, ky, kx);
  kyr = part ? N - ky : ky;
  if (raw) {
    if (wa == T(0)) v = mk(T(0), T(0));
    else if (grad && !part) acc += ((double)v.x * v.x + (double)v.y * v.y) / ((double)wa * wa);
  } else if (grad && !part) {
    acc += (double)wa * ((double)v.x * v.x + (double)v.y * v.y);
  }
  return scale(v, sc);
}

// Pixel step of the row pass for complex element j of image row y of component c (pixels
// 2j, 2j + 1).  Adjoint modes read the pixels into z; otherwise z holds the unnormalised
// inverse transform and becomes the input of the forward transform (or is written to xout
// and the pass ends there: CM_FWD, CM_SIM).
template <typename T, int N, int C, bool SIMK>
__device__ __forceinline__ void row_pixel(const Job& jb, int mode, bool adjIn, int c, int y, int j, cpx<T>& z,
                                          double& acc) {
  const T invn = T(1) / T(N);
  const T* W = reinterpret_cast<const T*>(jb.W);
  const T* dd = reinterpret_cast<const T*>(jb.d);
  const uint32_t pix = (uint32_t)y * N + 2 * j;
  const uint32_t cp = (uint32_t)c * N * N + pix;
  if (adjIn) {
    T x0 = gld(dd, cp), x1 = gld(dd, cp + 1);
    if (W) {   // masked adjoint: R^T M x
      if (!(gld(W, pix) > T(0))) x0 = T(0);
      if (!(gld(W, pix + 1) > T(0))) x1 = T(0);
    }
    z = mk(x0 * invn, x1 * invn);
    return;
  }
  const T x0 = z.x * invn, x1 = z.y * invn;
  T* xout = reinterpret_cast<T*>(jb.xout);
  if (mode == CM_FWD) {   // masked forward M R s when W is given
    gst(xout, cp, (W && !(gld(W, pix) > T(0))) ? T(0) : x0);
    gst(xout, cp + 1, (W && !(gld(W, pix + 1) > T(0))) ? T(0) : x1);
    return;
  }
  const T W0 = gld(W, pix), W1 = gld(W, pix + 1);
  if (SIMK && mode == CM_SIM) {
    const T* draws = reinterpret_cast<const T*>(jb.draws);
    T n0, n1;
    const int64_t qn = (int64_t)C * N * N + cp;
    if (draws) {
      n0 = draws[qn];
      n1 = draws[qn + 1];
    } else {
      philox_normal_pair<T>(jb.seed, jb.sim, qn, n0, n1);
    }
    xout[cp] = W0 > T(0) ? x0 + n0 / sqrt(W0) : T(0);
    xout[cp + 1] = W1 > T(0) ? x1 + n1 / sqrt(W1) : T(0);
    return;
  }
  T r0, r1;
  if (mode == CM_HV || mode == CM_RAW_HV) {
    r0 = W0 * x0;
    r1 = W1 * x1;
  } else {  // CM_GRAD, CM_RAW_GRAD: r = W (x - d); masked pixels contribute nothing
    r0 = T(0);
    r1 = T(0);
    if (W0 > T(0)) {
      const T e0 = x0 - gld(dd, cp);
      r0 = W0 * e0;
      acc += (double)r0 * e0;
    }
    if (W1 > T(0)) {
      const T e1 = x1 - gld(dd, cp + 1);
      r1 = W1 * e1;
      acc += (double)r1 * e1;
    }
  }
  z = mk(r0 * invn, r1 * invn);
}

// row_pixel's curvature and gradient branches (whitened or raw) on a preloaded pixel pair of
// W (and of d), so that a thread can issue the loads of all its elements first
template <typename T, int N, typename T2>
__device__ __forceinline__ void row_pixel_hot(bool grad, T2 w, T2 d, cpx<T>& z, double& acc) {
  const T invn = T(1) / T(N);
  const T x0 = z.x * invn, x1 = z.y * invn;
  T r0, r1;
  if (!grad) {
    r0 = w.x * x0;
    r1 = w.y * x1;
  } else {   // masked pixels contribute nothing
    const T e0 = x0 - d.x, e1 = x1 - d.y;
    const bool m0 = w.x > T(0), m1 = w.y > T(0);
    r0 = m0 ? w.x * e0 : T(0);
    r1 = m1 ? w.y * e1 : T(0);
    acc += m0 ? (double)r0 * e0 : 0.0;
    acc += m1 ? (double)r1 * e1 : 0.0;
  }
  z = mk(r0 * invn, r1 * invn);
}

// Column-forward output of component c at (ky, kx) = internal index o (t: forward
// transform after the inverse rotation): prior scale, added term, the v.out and out.out
// partials; writes and returns the output.
template <typename T, int N>
__device__ __forceinline__ cpx<T> colfwd_val(const Job& jb, int mode, int ky, int kx, int64_t o,
                                             cpx<T> t, double& avo, double& aoo) {
  const bool fr = is_free(N, ky, kx);
  const uint32_t oi = (uint32_t)o;
  cpx<T> out = mk(T(0), T(0));
  if (mode == CM_HV || mode == CM_GRAD) {
    const T sq = gld(reinterpret_cast<const T*>(jb.sOut), oi);
    if (fr && sq != T(0)) {
      const cpx<T> v = gld(reinterpret_cast<const cpx<T>*>(jb.vadd), oi);
      const T wa = jb.aTab ? gld(reinterpret_cast<const T*>(jb.aTab), oi) : T(1);
      out = mk(wa * v.x + sq * t.x, wa * v.y + sq * t.y);
      avo += (double)v.x * out.x + (double)v.y * out.y;
    }
    aoo += (double)out.x * out.x + (double)out.y * out.y;
  } else if (mode == CM_RAW_GRAD || mode == CM_RAW_HV) {
    const T sq = gld(reinterpret_cast<const T*>(jb.sOut), oi);
    if (fr && sq != T(0)) {
      const cpx<T> v = gld(reinterpret_cast<const cpx<T>*>(jb.vadd), oi);
      const T is = T(1) / (sq * sq);
      out = mk(T(4) * (v.x * is + t.x), T(4) * (v.y * is + t.y));
    }
  } else if (mode == CM_ADJ) {
    if (is_live(N, ky, kx)) out = t;
  } else {  // CM_ADJ_GRAD
    if (fr) out = scale(t, T(2));
  }
  gst(reinterpret_cast<cpx<T>*>(jb.vout), oi, out);
  return out;
}

// colfwd_val's curvature and gradient branches (CM_HV, CM_GRAD; raw: CM_RAW_HV,
// CM_RAW_GRAD) split like colinv_ld / colinv_fin: the loads of all of a thread's elements
// first, then the arithmetic; the caller stores the returned output.
template <typename T>
__device__ __forceinline__ void colfwd_ld(const Job& jb, uint32_t o, T& sq, cpx<T>& a, T& wa) {
  sq = gld(reinterpret_cast<const T*>(jb.sOut), o);
  a = gld(reinterpret_cast<const cpx<T>*>(jb.vadd), o);
  wa = jb.aTab ? gld(reinterpret_cast<const T*>(jb.aTab), o) : T(1);
}
template <typename T, int N>
__device__ __forceinline__ cpx<T> colfwd_fin(bool raw, int ky, int kx, cpx<T> t, T sq, cpx<T> a, T wa, double& avo,
                                             double& aoo) {
  const bool keep = is_free(N, ky, kx) && sq != T(0);
  if (raw) {
    const T is = keep ? T(1) / (sq * sq) : T(0);
    return keep ? mk(T(4) * (a.x * is + t.x), T(4) * (a.y * is + t.y)) : mk(T(0), T(0));
  }
  const cpx<T> out = keep ? mk(wa * a.x + sq * t.x, wa * a.y + sq * t.y) : mk(T(0), T(0));
  const double dvo = (double)a.x * out.x + (double)a.y * out.y;
  avo += keep ? dvo : 0.0;
  aoo += (double)out.x * out.x + (double)out.y * out.y;
  return out;
}

// For curvature products inside the solver (extras): the dots of the output at o with g and
// with the kept Dp_j (read with the non-temporal hint, like the history in pass B: the batch's
// vectors do not fit any cache; 15.9 -> 15.1 ms of column-forward per 127-map shear solve).
template <typename T>
__device__ __forceinline__ void colfwd_extras(const Job& jb, int64_t o, cpx<T> out, double& adg, double (&add)[MMAX]) {
  const cpx<T> gv = reinterpret_cast<const cpx<T>*>(jb.gvec)[o];
  adg += (double)gv.x * out.x + (double)gv.y * out.y;
  const cpx<T>* dpb = reinterpret_cast<const cpx<T>*>(jb.dpBase);
#pragma unroll
  for (int j = 0; j < MMAX; ++j) {
    if ((jb.dpMask >> j) & 1u) {
      const cpx<T> dj = gldnt(dpb, (uint32_t)((int64_t)j * jb.dpStride + o));
      add[j] += (double)dj.x * out.x + (double)dj.y * out.y;
    }
  }
}

// The same plus, for curvature products inside the solver (extras), the dots of the output
// with g and with the kept Dp_j.
template <typename T, int N>
__device__ __forceinline__ void colfwd_out(const Job& jb, int mode, bool extras, int ky, int kx, int64_t o,
                                           cpx<T> t, double& avo, double& aoo, double& adg,
                                           double (&add)[MMAX]) {
  const cpx<T> out = colfwd_val<T, N>(jb, mode, ky, kx, o, t, avo, aoo);
  if (extras) {
    const cpx<T> gv = reinterpret_cast<const cpx<T>*>(jb.gvec)[o];
    adg += (double)gv.x * out.x + (double)gv.y * out.y;
    const cpx<T>* dpb = reinterpret_cast<const cpx<T>*>(jb.dpBase);
#pragma unroll
    for (int j = 0; j < MMAX; ++j) {
      if ((jb.dpMask >> j) & 1u) {
        const cpx<T> dj = gldnt(dpb, (uint32_t)((int64_t)j * jb.dpStride + o));
        add[j] += (double)dj.x * out.x + (double)dj.y * out.y;
      }
    }
  }
}

// Work-group reduction of the column-forward partials: [VO, OO, DG, DD_0 .. DD_{MMAX-1}] ->
// kinds PK_VO + idx, one value per column block (the first block of the work-group holds the
// sum, the others 0).  Every thread must call it.
__device__ __forceinline__ void colfwd_reduce(const Job& jb, int mode, bool extras, double avo, double aoo, double adg,
                                              const double (&add)[MMAX], int q, int cpb) {
  if (!(mode == CM_HV || mode == CM_GRAD)) return;
  __shared__ double red2[NT / 64][3 + MMAX];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
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
    jb.part[(PK_VO + tid) * jb.pstride + q * cpb] = sum;
    for (int cb = 1; cb < cpb; ++cb) jb.part[(PK_VO + tid) * jb.pstride + q * cpb + cb] = 0.0;
  }
}

// ------------------------------------------------------------------------ column inverse
// SIMK: the variant launched for simulation jobs (CM_SIM); the others skip such jobs.
template <typename T, int N, int C, int CPB, bool SIMK>
__global__ __launch_bounds__(NT) void k_colinv(const Job* __restrict__ jobs, const cpx<T>* __restrict__ twg) {
  const Job& jb = jobs[blockIdx.y];
  const int mode = jb.mode;
  if (mode == CM_NONE || mode == CM_ADJ || mode == CM_ADJ_GRAD || (!SIMK && mode == CM_SIM)) return;
  constexpr int NB = CPB * C * TB;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* buf = tw + N;
  __shared__ double red[NT / 64];
  const int tid = threadIdx.x, q = blockIdx.x;
  for (int i = tid; i < N; i += NT) tw[i] = twg[i];

  double acc = 0.0;
  // elements ee = tid + k NT, in chunks of KCH whose loads are all issued first (hot modes)
  constexpr int NEL = CPB * N * TB, KI = (NEL + NT - 1) / NT, KCH = KI < 4 ? KI : 4;
  const bool hot = colinv_hot(mode), grad = (mode == CM_GRAD || mode == CM_RAW_GRAD);
  const bool raw = (mode == CM_RAW_HV || mode == CM_RAW_GRAD);
  for (int k0 = 0; k0 < KI; k0 += KCH) {
    cpx<T> av[KCH][C];
    T sc[KCH][C], wa[KCH][C];
    if (hot) {
#pragma unroll
      for (int k = 0; k < KCH; ++k) {
        const int ee = min(tid + (k0 + k) * NT, NEL - 1);   // past the end: any valid entry
        const int e = ee % (N * TB), kx = (q * CPB + ee / (N * TB)) * TB + e % TB;
#pragma unroll
        for (int c = 0; c < C; ++c) colinv_ld<T, N>(jb, grad, raw, c, e / TB, kx, av[k][c], sc[k][c], wa[k][c]);
      }
    }
#pragma unroll
    for (int k = 0; k < KCH; ++k) {
      const int ee = tid + (k0 + k) * NT;
      if (k0 + k >= KI || ee >= NEL) break;
      const int cb = ee / (N * TB), e = ee % (N * TB);
      const int qb = q * CPB + cb;                     // column block
      const int ky = e / TB, col = e % TB, kx = qb * TB + col;
      cpx<T> a[C];
      bool part = false;
      int kyr = ky;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        a[c] = hot ? colinv_fin<T, N>(grad, raw, ky, kx, av[k][c], sc[k][c], wa[k][c], part, kyr, acc)
                   : colinv_in<T, N, SIMK>(jb, mode, c, ky, kx, part, kyr, acc);
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
#pragma unroll
      for (int c = 0; c < C; ++c) buf[ky * NB + (cb * C + c) * TB + col] = a[c];
    }
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
template <typename T, int N, int C, int RBV, bool SIMK>
__global__ __launch_bounds__(NT) void k_row(const Job* __restrict__ jobs, const cpx<T>* __restrict__ twg) {
  const Job& jb = jobs[rev_instance()];
  const int mode = jb.mode;
  if (mode == CM_NONE || (!SIMK && mode == CM_SIM)) return;
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
  double acc = 0.0;
  if (colinv_hot(mode)) {
    // W (and d) pixel pairs of a chunk of elements loaded first, then row_pixel_hot
    using T2 = typename std::conditional<std::is_same<T, float>::value, float2, double2>::type;
    const bool grad = (mode == CM_GRAD || mode == CM_RAW_GRAD);
    const T2* W2 = reinterpret_cast<const T2*>(jb.W);
    const T2* D2 = grad ? reinterpret_cast<const T2*>(jb.d) : nullptr;
    constexpr int KCH = KP < 8 ? KP : 8;
    for (int k0 = 0; k0 < KP; k0 += KCH) {
      T2 wv[KCH], dv[KCH];
#pragma unroll
      for (int k = 0; k < KCH; ++k) {
        const int e = min(tid + (k0 + k) * NT, NE - 1);   // past the end: any valid element
        const int b = e / H;
        const uint32_t p2 = (uint32_t)(y0 + b % RB) * (N / 2) + e % H;
        wv[k] = gld(W2, p2);
        if (grad) dv[k] = gld(D2, (uint32_t)(b / RB) * (N * N / 2) + p2);
        else dv[k] = T2{T(0), T(0)};
      }
#pragma unroll
      for (int k = 0; k < KCH; ++k) {
        const int e = tid + (k0 + k) * NT;
        if (k0 + k >= KP || e >= NE) break;
        const int b = e / H, j = e % H;
        cpx<T> zf = buf[b * SBR + j];
        row_pixel_hot<T, N>(grad, wv[k], dv[k], zf, acc);
        buf[b * SBR + j] = zf;
      }
    }
  } else {
    for (int e = tid; e < NE; e += NT) {
      const int b = e / H, j = e % H;
      cpx<T> zf = buf[b * SBR + j];
      row_pixel<T, N, C, SIMK>(jb, mode, adjIn, b / RB, y0 + b % RB, j, zf, acc);
      if (mode != CM_FWD && mode != CM_SIM) buf[b * SBR + j] = zf;
    }
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
    // partials are kept per component and RB_MIN rows (slot c * N / RB_MIN + row / RB_MIN), so
    // the reduction does not depend on the row tile; this tile's sum goes to its first slot
    const double t = block_sum(acc, red);
    constexpr int PR = RB / RB_MIN;
    if (tid < C * PR)
      jb.part[PK_RES * jb.pstride + (tid / PR) * (N / RB_MIN) + blockIdx.x * PR + tid % PR] = tid == 0 ? t : 0.0;
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

  double avo = 0.0, aoo = 0.0, adg = 0.0;
  double add[MMAX];
#pragma unroll
  for (int j = 0; j < MMAX; ++j) add[j] = 0.0;
  // curvature products inside the solver also dot the new Dp with g and the kept Dp_j
  const bool extras = (mode == CM_HV) && jb.dpBase != nullptr;
  // elements ee = tid + k NT, in chunks of KCH whose epilogue loads are all issued first
  // (curvature and gradient modes)
  constexpr int NEL = CPB * N * TB, KI = (NEL + NT - 1) / NT, KCH = KI < 4 ? KI : 4;
  const bool hot = colinv_hot(mode), raw = (mode == CM_RAW_HV || mode == CM_RAW_GRAD);
  cpx<T>* vo = reinterpret_cast<cpx<T>*>(jb.vout);
  for (int k0 = 0; k0 < KI; k0 += KCH) {
    T sqv[KCH][C], wav[KCH][C];
    cpx<T> vav[KCH][C];
    if (hot) {
#pragma unroll
      for (int k = 0; k < KCH; ++k) {
        const int ee = min(tid + (k0 + k) * NT, NEL - 1);   // past the end: any valid entry
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const uint32_t o = (uint32_t)(fidx(N, c, 0, (q * CPB + ee / (N * TB)) * TB) + ee % (N * TB));
          colfwd_ld<T>(jb, o, sqv[k][c], vav[k][c], wav[k][c]);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < KCH; ++k) {
      const int ee = tid + (k0 + k) * NT;
      if (k0 + k >= KI || ee >= NEL) break;
      const int cb = ee / (N * TB), e = ee % (N * TB);
      const int qb = q * CPB + cb;
      const int ky = e / TB, col = e % TB, kx = qb * TB + col;
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
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int64_t o = fidx(N, c, 0, qb * TB) + e;
        if (hot) {
          const cpx<T> out = colfwd_fin<T, N>(raw, ky, kx, t[c], sqv[k][c], vav[k][c], wav[k][c], avo, aoo);
          gst(vo, (uint32_t)o, out);
          if (extras) colfwd_extras<T>(jb, o, out, adg, add);
        } else {
          colfwd_out<T, N>(jb, mode, extras, ky, kx, o, t[c], avo, aoo, adg, add);
        }
      }
    }
  }
  colfwd_reduce(jb, mode, extras, avo, aoo, adg, add, q, CPB);
}

// ======================================================================== single pass
// Small maps (the whole field fits one work-group's LDS): the three passes of a solver's
// curvature product or exact gradient (CM_HV, CM_GRAD) in one kernel, one work-group per
// instance.  The field is read once and Dp written once, against 7 vectors of traffic for the
// three passes; the intermediate never leaves LDS.  LDS layout [c][y][k] (k < N/2 complex): the
// column transforms run per component over the H columns (stride H), the row transforms over
// the C N rows.  The complex-to-real and real-to-complex untangle steps pair k with H - k in
// one thread, so they run in place without a barrier between reads and writes.  Partial sums
// go to the same slots the three passes fill (the first slot of each kind, the others 0).
// Other modes return: operator calls use the three passes.
template <typename T, int N, int C>
constexpr size_t lds_chain1() { return (size_t)(N + C * N * (N / 2)) * sizeof(cpx<T>); }
constexpr int CHAIN1_NT = 1024;   // threads per work-group: one work-group fills a CU (LDS-bound)

template <typename T, int N, int C>
__global__ __launch_bounds__(CHAIN1_NT) void k_chain1(const Job* __restrict__ jobs, const cpx<T>* __restrict__ twg) {
  const Job& jb = jobs[blockIdx.x];
  const int mode = jb.mode;
  if (!(mode == CM_HV || mode == CM_GRAD)) return;
  constexpr int H = N / 2, NE = C * N * H;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* buf = tw + N;
  constexpr int TP = CHAIN1_NT, NW = TP / 64;
  const int tid = threadIdx.x;
  const bool grad = mode == CM_GRAD;
  for (int i = tid; i < N; i += TP) tw[i] = twg[i];
  // ---- column-inverse prologue: scale, Hermitian completion, rotation, prior partial
  double accP = 0.0;
  for (int e = tid; e < N * H; e += TP) {
    const int ky = e / H, kx = e % H;
    cpx<T> a[C];
    bool part = false;
    int kyr = ky;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      cpx<T> v;
      T sc, wa;
      colinv_ld<T, N>(jb, grad, false, c, ky, kx, v, sc, wa);
      a[c] = colinv_fin<T, N>(grad, false, ky, kx, v, sc, wa, part, kyr, accP);
    }
    if constexpr (C == 2) {
      T c2, s2;
      rot2<T>(kx, kyr < H ? kyr : kyr - N, c2, s2);
      const cpx<T> e0 = a[0], b0 = a[1];
      a[0] = mk(c2 * e0.x - s2 * b0.x, c2 * e0.y - s2 * b0.y);
      a[1] = mk(s2 * e0.x + c2 * b0.x, s2 * e0.y + c2 * b0.y);
    }
    if (part) {
#pragma unroll
      for (int c = 0; c < C; ++c) a[c] = conj(a[c]);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) buf[(c * N + ky) * H + kx] = a[c];
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < C; ++c) lds_fft<T, N, H, 1, H, 1, false, true, TP>(buf + c * N * H, tw);
  // ---- complex-to-real untangle, per row b and pair (k, H - k):
  //   Z_k = (X_k + conj X_{H-k}) + i w^-k (X_k - conj X_{H-k}),  X_0 real part only
  for (int e = tid; e < C * N * (H / 2 + 1); e += TP) {
    const int b = e / (H / 2 + 1), k = e % (H / 2 + 1);
    cpx<T>* row = buf + b * H;
    if (k == 0) {
      const cpx<T> X = row[0];
      row[0] = mk(X.x, X.x);
    } else {
      const cpx<T> X = row[k], Y = row[H - k];
      const cpx<T> Xm = conj(Y), Ym = conj(X);
      const cpx<T> t1 = mulc(sub(X, Xm), tw[k]), s1 = add(X, Xm);
      const cpx<T> t2 = mulc(sub(Y, Ym), tw[H - k]), s2 = add(Y, Ym);
      row[k] = mk(s1.x - t1.y, s1.y + t1.x);
      if (k != H - k) row[H - k] = mk(s2.x - t2.y, s2.y + t2.x);
    }
  }
  __syncthreads();
  lds_fft<T, H, C * N, H, 1, 2, true, true, TP>(buf, tw);
  // ---- pixel step: element j of row (c, y) holds pixels (2j, 2j + 1)
  double accR = 0.0;
  {
    using T2 = typename std::conditional<std::is_same<T, float>::value, float2, double2>::type;
    const T2* W2 = reinterpret_cast<const T2*>(jb.W);
    const T2* D2 = grad ? reinterpret_cast<const T2*>(jb.d) : nullptr;
    for (int e = tid; e < NE; e += TP) {
      const int b = e / H, j = e % H;
      const int c = b / N, y = b % N;
      const uint32_t p2 = (uint32_t)y * H + j;
      const T2 w = gld(W2, p2);
      const T2 d = grad ? gld(D2, (uint32_t)c * (N * H) + p2) : T2{T(0), T(0)};
      cpx<T> z = buf[e];
      row_pixel_hot<T, N>(grad, w, d, z, accR);
      buf[e] = z;
    }
  }
  __syncthreads();
  lds_fft<T, H, C * N, H, 1, 2, true, false, TP>(buf, tw);
  // ---- real-to-complex untangle, pair (k, H - k), Z_H = Z_0:
  //   X_k = 1/2 (Z_k + conj Z_{H-k}) - i/2 w^k (Z_k - conj Z_{H-k})
  for (int e = tid; e < C * N * (H / 2 + 1); e += TP) {
    const int b = e / (H / 2 + 1), k = e % (H / 2 + 1);
    cpx<T>* row = buf + b * H;
    const int km = k == 0 ? 0 : H - k;
    const cpx<T> Zk = row[k], Zm = row[km];
    auto untangle = [&](cpx<T> A0, cpx<T> B0, int kk) {
      const cpx<T> Bc = conj(B0);
      const cpx<T> A = add(A0, Bc);
      const cpx<T> t = mul(tw[kk], sub(A0, Bc));
      return mk(T(0.5) * (A.x + t.y), T(0.5) * (A.y - t.x));
    };
    const cpx<T> xk = untangle(Zk, Zm, k);
    if (k != 0 && k != km) {
      const cpx<T> xm = untangle(Zm, Zk, km);
      row[km] = xm;
    }
    row[k] = xk;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < C; ++c) lds_fft<T, N, H, 1, H, 1, false, false, TP>(buf + c * N * H, tw);
  // ---- column-forward epilogue: inverse rotation, x S^1/2, + added term, solver dots
  double avo = 0.0, aoo = 0.0, adg = 0.0;
  double add[MMAX];
#pragma unroll
  for (int j = 0; j < MMAX; ++j) add[j] = 0.0;
  const bool extras = (mode == CM_HV) && jb.dpBase != nullptr;
  cpx<T>* vo = reinterpret_cast<cpx<T>*>(jb.vout);
  for (int e = tid; e < N * H; e += TP) {
    const int ky = e / H, kx = e % H;
    cpx<T> t[C];
#pragma unroll
    for (int c = 0; c < C; ++c) t[c] = buf[(c * N + ky) * H + kx];
    if constexpr (C == 2) {
      T c2, s2;
      rot2<T>(kx, ky < H ? ky : ky - N, c2, s2);
      const cpx<T> g1 = t[0], g2 = t[1];
      t[0] = mk(c2 * g1.x + s2 * g2.x, c2 * g1.y + s2 * g2.y);
      t[1] = mk(-s2 * g1.x + c2 * g2.x, -s2 * g1.y + c2 * g2.y);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int64_t o = fidx(N, c, ky, kx);
      T sq, wa;
      cpx<T> va;
      colfwd_ld<T>(jb, (uint32_t)o, sq, va, wa);
      const cpx<T> out = colfwd_fin<T, N>(false, ky, kx, t[c], sq, va, wa, avo, aoo);
      gst(vo, (uint32_t)o, out);
      if (extras) colfwd_extras<T>(jb, o, out, adg, add);
    }
  }
  // work-group sums of the partials (wave shuffle trees, then the waves in order), each kind
  // into its first slot and 0 into the others the solver reduces
  const int lane = tid & 63, wv = tid >> 6;
  constexpr int NV = 3 + MMAX + 2;   // VO, OO, DG, DD_0..DD_{MMAX-1}, prior, residual
  double vals[NV];
  vals[0] = avo;
  vals[1] = aoo;
  vals[2] = adg;
#pragma unroll
  for (int j = 0; j < MMAX; ++j) vals[3 + j] = add[j];
  vals[3 + MMAX] = accP;
  vals[4 + MMAX] = accR;
  __shared__ double redv[NW][NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double x = wave_sum(vals[v]);
    if (lane == 0) redv[wv][v] = x;
  }
  __syncthreads();
  constexpr int NCOL = N / 2 / TB, NROW = C * N / RB_MIN;
  const uint32_t mask = extras ? jb.dpMask : 0u;
  if (tid < NV) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) t += redv[w][tid];
    if (tid < 2 || (extras && tid < 3) || (tid >= 3 && tid < 3 + MMAX && ((mask >> (tid - 3)) & 1u)))
      jb.part[(PK_VO + tid) * jb.pstride] = t;
    else if (grad && tid == 3 + MMAX)
      jb.part[PK_PRIOR * jb.pstride] = t;
    else if (grad && tid == 4 + MMAX)
      jb.part[PK_RES * jb.pstride] = t;
  }
  for (int k = tid; k < (NCOL - 1) * (3 + MMAX); k += TP) {
    const int kind = k / (NCOL - 1), slot = 1 + k % (NCOL - 1);
    if (kind < 3 || ((mask >> (kind - 3)) & 1u)) jb.part[(PK_VO + kind) * jb.pstride + slot] = 0.0;
  }
  if (grad) {
    for (int k = tid; k < NCOL - 1; k += TP) jb.part[PK_PRIOR * jb.pstride + 1 + k] = 0.0;
    for (int k = tid; k < NROW - 1; k += TP) jb.part[PK_RES * jb.pstride + 1 + k] = 0.0;
  }
}

// ======================================================================== register-staged
// Power-of-two n >= 128, float32: the same passes with the register-staged FFT of
// wf_rfft.hpp (simulation jobs run on the LDS-staged variants).  First-stage inputs are read from global memory (column passes) or from the
// LDS staging tile (row pass) straight into registers; last-stage outputs go from registers
// to global memory; the row pass chains its inverse and forward transforms in registers
// around the pixel step.  The spin-2 rotation exchanges the partner component between lanes.

// Register-staged row pass: a work-group owns RB rows of one component, E elements per
// thread.  LDS row strides of the staging tile and of the exchange layouts (index
// i + i / R_0 in a row) were chosen for at most 2-way bank conflicts of every access pattern.
__host__ __device__ constexpr int rowr_e(int n) { return n <= 256 ? 8 : 16; }
__host__ __device__ constexpr int rowr_rb(int n) { return rowr_e(n) * NT / (n / 2); }
__host__ __device__ constexpr int rowr_io_stride(int H) { return H + (H == 64 ? 6 : (H == 512 ? 4 : 2)); }
// exchange layouts: row b at b * rowr_x_stride, index i at i + i / rowr_xpad
__host__ __device__ constexpr int rowr_xpad(int H) { return H <= 128 ? 8 : 16; }
__host__ __device__ constexpr int rowr_x_stride(int H, int E, bool rev) { return H + H / rowr_xpad(H); }
__host__ __device__ constexpr int rowr_data_stride(int H, int E) {
  const int a = rowr_io_stride(H), b = rowr_x_stride(H, E, false), c = rowr_x_stride(H, E, true);
  return a > b ? (a > c ? a : c) : (b > c ? b : c);
}
template <int N>
constexpr size_t lds_rowr() {
  return ((size_t)rowr_rb(N) * rowr_data_stride(N / 2, rowr_e(N)) + (size_t)N) * sizeof(cpx<float>);
}
template <int N, int C, int CPB>
constexpr size_t lds_colr() {
  constexpr int NB = CPB * C * TB, E = NB * N / NT;
  return ((size_t)(N + N / rs_radix(N, E, false, 0)) * NB + (size_t)N) * sizeof(cpx<float>);
}

template <int N, int C, int CPB>
__global__ __launch_bounds__(NT) void k_colinvr(const Job* __restrict__ jobs, const cpx<float>* __restrict__ twg) {
  using T = float;
  const Job& jb = jobs[blockIdx.y];
  const int mode = jb.mode;
  if (mode == CM_NONE || mode == CM_ADJ || mode == CM_ADJ_GRAD || mode == CM_SIM) return;
  constexpr int NB = CPB * C * TB, E = NB * N / NT;
  constexpr int PQ = rs_radix(N, E, false, 0), NST = rs_nst(N, E);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* data = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* st = data + (N + N / PQ) * NB;
  __shared__ double red[NT / 64];
  const int tid = threadIdx.x, q = blockIdx.x;
  {
    const cpx<T>* g = twg + tw_col_off(N, E);
    for (int i = tid; i < N; i += NT) st[i] = g[i];
  }
  auto lx = [](uint32_t b, uint32_t i) { return (i + i / PQ) * NB + b; };
  // this thread's transform (the same in every stage: NT is a multiple of NB)
  const uint32_t b = (uint32_t)tid % NB;
  const int col = b % TB, c = (b / TB) % C, cb = b / (TB * C);
  const int qb = q * CPB + cb, kx = qb * TB + col;
  const int64_t bs = fidx(N, c, 0, qb * TB);
  double acc = 0.0;
  cpx<T> v[E];
  {
    constexpr int R0 = PQ, NQ0 = N / R0, K0 = E / R0;
    const bool hot = colinv_hot(mode), grad = (mode == CM_GRAD || mode == CM_RAW_GRAD);
    const bool raw = (mode == CM_RAW_HV || mode == CM_RAW_GRAD);
    T sc[E], wa[E];
    if (hot) {
      sfor<0, E>([&](auto I) {
        constexpr int i = decltype(I)::value;
        const int ky = (int)(((uint32_t)tid + (i / R0) * NT) / NB) + (i % R0) * NQ0;
        colinv_ld<T, N>(jb, grad, raw, c, ky, kx, v[i], sc[i], wa[i]);
      });
    }
    sfor<0, K0>([&](auto KK) {
      constexpr int kk = decltype(KK)::value;
      const int j = ((uint32_t)tid + kk * NT) / NB;
      sfor<0, R0>([&](auto RR) {
        constexpr int r = decltype(RR)::value;
        const int ky = j + r * NQ0;
        bool part;
        int kyr;
        cpx<T> a = hot ? colinv_fin<T, N>(grad, raw, ky, kx, v[kk * R0 + r], sc[kk * R0 + r], wa[kk * R0 + r], part,
                                          kyr, acc)
                       : colinv_in<T, N, false>(jb, mode, c, ky, kx, part, kyr, acc);
        if constexpr (C == 2) {
          const T ox = lane_xor2(a.x), oy = lane_xor2(a.y);   // the other component
          T c2, s2;
          rot2<T>(kx, kyr < N / 2 ? kyr : kyr - N, c2, s2);
          a = (c == 0) ? mk(c2 * a.x - s2 * ox, c2 * a.y - s2 * oy) : mk(s2 * ox + c2 * a.x, s2 * oy + c2 * a.y);
        }
        v[kk * R0 + r] = part ? conj(a) : a;
      });
    });
  }
  rs_fft<T, N, NB, E, false, true, false>(v, data, st, lx, tid);
  {
    constexpr int RL = rs_radix(N, E, false, NST - 1), NQL = N / RL, KL = E / RL;
    cpx<T>* y = reinterpret_cast<cpx<T>*>(jb.y);
    sfor<0, KL>([&](auto KK) {
      constexpr int kk = decltype(KK)::value;
      const uint32_t j = ((uint32_t)tid + kk * NT) / NB;
      sfor<0, RL>([&](auto RR) {
        constexpr int r = decltype(RR)::value;
        gst(y, (uint32_t)bs + (j + r * NQL) * TB + col, v[kk * RL + r]);
      });
    });
  }
  if (mode == CM_GRAD || mode == CM_RAW_GRAD) {
    const double t = block_sum(acc, red);
    if (tid < CPB) jb.part[PK_PRIOR * jb.pstride + q * CPB + tid] = tid == 0 ? t : 0.0;
  }
}

// One tile (RB rows of one component) per work-group: blockIdx.x = component * (N / RB) + row
// tile, blockIdx.y = instance (in reverse order, see rev_instance).
template <int N, int C>
__global__ __launch_bounds__(NT) void k_rowr(const Job* __restrict__ jobs, const cpx<float>* __restrict__ twg) {
  using T = float;
  const Job& jb = jobs[rev_instance()];
  const int mode = jb.mode;
  if (mode == CM_NONE || mode == CM_SIM) return;
  constexpr int H = N / 2, E = rowr_e(N), RB = rowr_rb(N), NE = RB * H, KS = NE / NT;
  static_assert(RB % RB_MIN == 0 && N % RB == 0 && NE % NT == 0, "row tile");
  constexpr int TPC = N / RB;   // tiles per component
  constexpr int NST = rs_nst(H, E);
  constexpr int PQI = rs_radix(H, E, false, 0);
  constexpr int SBIO = rowr_io_stride(H), SBXI = rowr_x_stride(H, E, false), SBXF = rowr_x_stride(H, E, true);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* data = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* stI = data + RB * rowr_data_stride(H, E);
  cpx<T>* stF = stI + H;
  __shared__ double red[NT / 64];
  const uint32_t tid = threadIdx.x;
  const int c = blockIdx.x / TPC, tile = blockIdx.x % TPC, y0 = tile * RB;
  auto lio = [](uint32_t b, uint32_t i) { return b * SBIO + i; };
  constexpr int XP = rowr_xpad(H);
  auto lxi = [](uint32_t b, uint32_t i) { return b * SBXI + i + i / XP; };
  auto lxf = [](uint32_t b, uint32_t i) { return b * SBXF + i + i / XP; };
  const bool adjIn = (mode == CM_ADJ || mode == CM_ADJ_GRAD);
  cpx<T>* Y = reinterpret_cast<cpx<T>*>(jb.y) + fidx(N, c, y0, 0);   // column block 0 of this tile
  cpx<T> v[E];
  double acc = 0.0;
  // the tile's RB x TB runs of every column block, coalesced, and the twiddles w^k of the
  // complex-to-real pre-processing, issued before the (L2-resident) stage twiddles are staged
  constexpr int R0 = PQI, NQ0 = H / R0, K0 = E / R0;
  cpx<T> pf[KS], wpre[E];
  if (!adjIn) {
    sfor<0, KS>([&](auto K) {
      constexpr int k = decltype(K)::value;
      const uint32_t e = tid + k * NT;
      pf[k] = gld(Y, (e / (RB * TB)) * N * TB + e % (RB * TB));
    });
    sfor<0, E>([&](auto I) {
      constexpr int i = decltype(I)::value;
      wpre[i] = gld(twg, (tid + (i / R0) * NT) % NQ0 + (i % R0) * NQ0);
    });
  }
  {
    const cpx<T>* gI = twg + tw_row_off(N, E, false);
    const cpx<T>* gF = twg + tw_row_off(N, E, true);
    for (uint32_t i = tid; i < H; i += NT) {
      stI[i] = gld(gI, i);
      stF[i] = gld(gF, i);
    }
  }
  if (!adjIn) {
    sfor<0, KS>([&](auto K) {
      constexpr int k = decltype(K)::value;
      const uint32_t e = tid + k * NT, w2 = e % (RB * TB);
      data[lio(w2 / TB, (e / (RB * TB)) * TB + w2 % TB)] = pf[k];
    });
    __syncthreads();
    // complex-to-real pre-processing into the first stage's registers (see k_row)
    sfor<0, K0>([&](auto KK) {
      constexpr int kk = decltype(KK)::value;
      const uint32_t u = tid + kk * NT, b = u / NQ0, j = u % NQ0;
      sfor<0, R0>([&](auto RR) {
        constexpr int r = decltype(RR)::value;
        const uint32_t k = j + r * NQ0;
        const cpx<T> X = data[lio(b, k)];
        cpx<T> z;
        if (k == 0) {
          z = mk(X.x, X.x);
        } else {
          const cpx<T> Xm = conj(data[lio(b, H - k)]);
          const cpx<T> tw = mulc(sub(X, Xm), wpre[kk * R0 + r]);
          const cpx<T> sm = add(X, Xm);
          z = mk(sm.x - tw.y, sm.y + tw.x);
        }
        v[kk * R0 + r] = z;
      });
    });
    rs_fft<T, H, RB, E, true, true, false>(v, data, stI, lxi, tid);
  }
  {
    // pixel step in the inverse's last-stage layout, which is the forward's first-stage one
    constexpr int RL = rs_radix(H, E, false, NST - 1), NQL = H / RL, KL = E / RL;
    if (colinv_hot(mode)) {
      // row_pixel's curvature and gradient branches with the W (and d) pixel pairs of all E
      // elements loaded first
      const bool grad = (mode == CM_GRAD || mode == CM_RAW_GRAD);
      const float2* W2 = reinterpret_cast<const float2*>(jb.W);
      const float2* D2 = grad ? reinterpret_cast<const float2*>(jb.d) + (uint32_t)c * (N * N / 2) : nullptr;
      float2 wv[E], dv[E];
      sfor<0, E>([&](auto I) {
        constexpr int i = decltype(I)::value;
        const uint32_t u = tid + (i / RL) * NT;
        const uint32_t p2 = (uint32_t)(y0 + u / NQL) * (N / 2) + u % NQL + (i % RL) * NQL;
        wv[i] = gld(W2, p2);
        dv[i] = grad ? gld(D2, p2) : make_float2(0.f, 0.f);
      });
      sfor<0, E>([&](auto I) { row_pixel_hot<T, N>(grad, wv[decltype(I)::value], dv[decltype(I)::value], v[decltype(I)::value], acc); });
    } else {
      sfor<0, KL>([&](auto KK) {
        constexpr int kk = decltype(KK)::value;
        const uint32_t u = tid + kk * NT, b = u / NQL, j = u % NQL;
        sfor<0, RL>([&](auto RR) {
          constexpr int r = decltype(RR)::value;
          row_pixel<T, N, C, false>(jb, mode, adjIn, c, y0 + b, j + r * NQL, v[kk * RL + r], acc);
        });
      });
    }
  }
  if (mode == CM_FWD) return;
  rs_fft<T, H, RB, E, true, false, true>(v, data, stF, lxf, tid);
  cpx<T> wpost[KS];
  {
    // outputs are in the inverse's first-stage layout: to LDS in natural order for the
    // real-to-complex untangle, which pairs k with H - k; its twiddles are loaded first
    sfor<0, KS>([&](auto K) {
      constexpr int kq = decltype(K)::value;
      const uint32_t e = tid + kq * NT;
      wpost[kq] = gld(twg, (e / (RB * TB)) * TB + e % TB);
    });
    __syncthreads();
    sfor<0, K0>([&](auto KK) {
      constexpr int kk = decltype(KK)::value;
      const uint32_t u = tid + kk * NT, b = u / NQ0, j = u % NQ0;
      sfor<0, R0>([&](auto RR) {
        constexpr int r = decltype(RR)::value;
        data[lio(b, j + r * NQ0)] = v[kk * R0 + r];
      });
    });
    __syncthreads();
  }
  sfor<0, KS>([&](auto K) {
    constexpr int kq = decltype(K)::value;
    const uint32_t e = tid + kq * NT, qq = e / (RB * TB), w2 = e % (RB * TB);
    const uint32_t b = w2 / TB, k = qq * TB + w2 % TB;
    const cpx<T> Zk = data[lio(b, k)];
    const cpx<T> Zm = conj(data[lio(b, k == 0 ? 0 : H - k)]);
    const cpx<T> A = add(Zk, Zm);
    const cpx<T> tw = mul(wpost[kq], sub(Zk, Zm));
    gst(Y, qq * N * TB + w2, mk(T(0.5) * (A.x + tw.y), T(0.5) * (A.y - tw.x)));
  });
  if (mode == CM_GRAD || mode == CM_RAW_GRAD) {
    const double tsum = block_sum(acc, red);
    constexpr int PR = RB / RB_MIN;
    if (tid < PR) jb.part[PK_RES * jb.pstride + c * (N / RB_MIN) + tile * PR + tid] = tid == 0 ? tsum : 0.0;
  }
}

template <int N, int C, int CPB>
__global__ __launch_bounds__(NT) void k_colfwdr(const Job* __restrict__ jobs, const cpx<float>* __restrict__ twg) {
  using T = float;
  const Job& jb = jobs[blockIdx.y];
  const int mode = jb.mode;
  if (mode == CM_NONE || mode == CM_FWD || mode == CM_SIM) return;
  constexpr int NB = CPB * C * TB, E = NB * N / NT;
  constexpr int PQ = rs_radix(N, E, false, 0), NST = rs_nst(N, E);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* data = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* st = data + (N + N / PQ) * NB;
  const int tid = threadIdx.x, q = blockIdx.x;
  {
    const cpx<T>* g = twg + tw_col_off(N, E);
    for (int i = tid; i < N; i += NT) st[i] = g[i];
  }
  auto lx = [](uint32_t b, uint32_t i) { return (i + i / PQ) * NB + b; };
  const uint32_t b = (uint32_t)tid % NB;
  const int col = b % TB, c = (b / TB) % C, cb = b / (TB * C);
  const int qb = q * CPB + cb, kx = qb * TB + col;
  const int64_t bs = fidx(N, c, 0, qb * TB);
  const cpx<T>* Y = reinterpret_cast<const cpx<T>*>(jb.y);
  cpx<T> v[E];
  {
    constexpr int R0 = PQ, NQ0 = N / R0, K0 = E / R0;
    sfor<0, K0>([&](auto KK) {
      constexpr int kk = decltype(KK)::value;
      const uint32_t j = ((uint32_t)tid + kk * NT) / NB;
      sfor<0, R0>([&](auto RR) {
        constexpr int r = decltype(RR)::value;
        v[kk * R0 + r] = gld(Y, (uint32_t)bs + (j + r * NQ0) * TB + col);
      });
    });
  }
  rs_fft<T, N, NB, E, false, false, false>(v, data, st, lx, tid);
  constexpr int RL = rs_radix(N, E, false, NST - 1), NQL = N / RL, KL = E / RL;
  double avo = 0.0, aoo = 0.0;
  // curvature and gradient modes: the epilogue's loads (prior scale, added term, solver
  // weight) of all E elements are issued before the first use
  const bool hot = colinv_hot(mode), raw = (mode == CM_RAW_HV || mode == CM_RAW_GRAD);
  T sqv[E], wav[E];
  cpx<T> vav[E];
  if (hot) {
    sfor<0, E>([&](auto I) {
      constexpr int i = decltype(I)::value;
      const uint32_t o = (uint32_t)bs + (((uint32_t)tid + (i / RL) * NT) / NB + (i % RL) * NQL) * TB + col;
      colfwd_ld<T>(jb, o, sqv[i], vav[i], wav[i]);
    });
  }
  cpx<T>* vo = reinterpret_cast<cpx<T>*>(jb.vout);
  sfor<0, KL>([&](auto KK) {
    constexpr int kk = decltype(KK)::value;
    const uint32_t j = ((uint32_t)tid + kk * NT) / NB;
    sfor<0, RL>([&](auto RR) {
      constexpr int r = decltype(RR)::value;
      constexpr int i = kk * RL + r;
      const int ky = j + r * NQL;
      cpx<T> t = v[i];
      if constexpr (C == 2) {
        const T ox = lane_xor2(t.x), oy = lane_xor2(t.y);   // the other component
        T c2, s2;
        rot2<T>(kx, ky < N / 2 ? ky : ky - N, c2, s2);
        t = (c == 0) ? mk(c2 * t.x + s2 * ox, c2 * t.y + s2 * oy) : mk(-s2 * ox + c2 * t.x, -s2 * oy + c2 * t.y);
      }
      const uint32_t o = (uint32_t)bs + ky * TB + col;
      if (hot) {
        const cpx<T> out = colfwd_fin<T, N>(raw, ky, kx, t, sqv[i], vav[i], wav[i], avo, aoo);
        gst(vo, o, out);
        v[i] = out;
      } else {
        v[i] = colfwd_val<T, N>(jb, mode, ky, kx, o, t, avo, aoo);
      }
    });
  });
  if (!(mode == CM_HV || mode == CM_GRAD)) return;
  // partials [VO, OO, DG, DD_0 .. DD_{MMAX-1}] -> kinds PK_VO + idx.  The dots with g and the
  // kept Dp_j (curvature products inside the solver) run one vector at a time, so only one
  // FP64 accumulator is live.
  __shared__ double red2[NT / 64][3 + MMAX];
  const int lane = tid & 63, wv = tid >> 6;
  const bool extras = (mode == CM_HV) && jb.dpBase != nullptr;
  const uint32_t mask = extras ? jb.dpMask : 0u;
  {
    const double a0 = wave_sum(avo), a1 = wave_sum(aoo);
    if (lane == 0) {
      red2[wv][0] = a0;
      red2[wv][1] = a1;
    }
  }
  auto dot_with = [&](const cpx<T>* u) {
    double a = 0.0;
    sfor<0, KL>([&](auto KK) {
      constexpr int kk = decltype(KK)::value;
      const uint32_t j = ((uint32_t)tid + kk * NT) / NB;
      sfor<0, RL>([&](auto RR) {
        constexpr int r = decltype(RR)::value;
        const cpx<T> w = gldnt(u, (uint32_t)bs + (j + r * NQL) * TB + col);
        a += (double)w.x * v[kk * RL + r].x + (double)w.y * v[kk * RL + r].y;
      });
    });
    return wave_sum(a);
  };
  if (extras) {
    const double ag = dot_with(reinterpret_cast<const cpx<T>*>(jb.gvec));
    if (lane == 0) red2[wv][2] = ag;
    const cpx<T>* dpb = reinterpret_cast<const cpx<T>*>(jb.dpBase);
    for (int jj = 0; jj < MMAX; ++jj) {
      if ((mask >> jj) & 1u) {
        const double aj = dot_with(dpb + (int64_t)jj * jb.dpStride);
        if (lane == 0) red2[wv][3 + jj] = aj;
      }
    }
  }
  __syncthreads();
  const int nv = extras ? 3 + MMAX : 2;
  if (tid < nv && (tid < 3 || ((mask >> (tid - 3)) & 1u))) {
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) sum += red2[k][tid];
    jb.part[(PK_VO + tid) * jb.pstride + q * CPB] = sum;
    for (int cb = 1; cb < CPB; ++cb) jb.part[(PK_VO + tid) * jb.pstride + q * CPB + cb] = 0.0;
  }
}

}  // namespace wf
