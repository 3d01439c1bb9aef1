// Self-sorting (Stockham) mixed-radix FFT on data staged in LDS.
//
// NB independent transforms of length N; element j of transform b lives at
// lds[b * SB + j * SJ].  Stage s with radix R and sub-transform length NS (product of
// the radices before it) maps butterfly j in [0, N/R):
//   inputs   a[j + r N/R]                         r = 0..R-1
//   twiddle  a_r *= w_{NS R}^{r (j mod NS)}       (w_M = exp(-2 pi i / M); conjugated
//                                                  for the inverse transform)
//   outputs  a'[(j div NS) NS R + (j mod NS) + r NS] = DFT_R(a)_r
// The radices are 8s with a 4/4, 4 or 2 remainder, preceded by one radix-3 stage
// when 3 divides N.  Twiddles come from a table tw[k] = exp(-2 pi i k / (N * TS))
// generated in float64 on the host; TS = 2 lets a length-n table serve an n/2 FFT.
// Transforms are unnormalised in both directions.
#pragma once
#include "wf_common.hpp"

namespace wf {

__host__ __device__ constexpr int fft_num_stages(int N) {
  int st = 0;
  if (N % 3 == 0) { st++; N /= 3; }
  int L = 0;
  while ((1 << L) < N) L++;
  const int a = L / 3, r = L % 3;
  if (r == 0) return st + a;
  if (r == 1) return st + (a >= 1 ? a + 1 : 1);
  return st + a + 1;
}

__host__ __device__ constexpr int fft_stage_radix(int N, int s) {
  if (N % 3 == 0) {
    if (s == 0) return 3;
    s -= 1;
    N /= 3;
  }
  int L = 0;
  while ((1 << L) < N) L++;
  const int a = L / 3, r = L % 3;
  if (r == 0) return 8;
  if (r == 1) {
    if (a == 0) return 2;
    return (s < a - 1) ? 8 : 4;
  }
  return (s < a) ? 8 : 4;
}

// ------------------------------------------------------------------------ small DFTs
template <typename T, bool INV>
__device__ __forceinline__ cpx<T> mul_mi(cpx<T> a) {   // a * (-i) forward, a * (+i) inverse
  return INV ? mk(-a.y, a.x) : mk(a.y, -a.x);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft2(cpx<T>& a0, cpx<T>& a1) {
  cpx<T> t = a0;
  a0 = add(t, a1);
  a1 = sub(t, a1);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(cpx<T>& a0, cpx<T>& a1, cpx<T>& a2, cpx<T>& a3) {
  cpx<T> t0 = add(a0, a2), t1 = sub(a0, a2), t2 = add(a1, a3), t3 = mul_mi<T, INV>(sub(a1, a3));
  a0 = add(t0, t2);
  a2 = sub(t0, t2);
  a1 = add(t1, t3);
  a3 = sub(t1, t3);
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dft(cpx<T>* v) {
  if constexpr (R == 2) {
    dft2<T, INV>(v[0], v[1]);
  } else if constexpr (R == 3) {
    // w = exp(-+2 pi i / 3) = -1/2 -+ i sqrt(3)/2
    const T h = T(0.5), s3 = T(0.86602540378443864676372317075294);
    cpx<T> t = add(v[1], v[2]);
    cpx<T> u = sub(v[1], v[2]);
    cpx<T> a = mk(v[0].x - h * t.x, v[0].y - h * t.y);
    // b = (-+ i s3) u
    cpx<T> b = INV ? mk(-s3 * u.y, s3 * u.x) : mk(s3 * u.y, -s3 * u.x);
    v[0] = add(v[0], t);
    v[1] = add(a, b);
    v[2] = sub(a, b);
  } else if constexpr (R == 4) {
    dft4<T, INV>(v[0], v[1], v[2], v[3]);
  } else {  // R == 8: two DFT4 of the even and odd samples, then twiddles w8^k
    cpx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    cpx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<T, INV>(e0, e1, e2, e3);
    dft4<T, INV>(o0, o1, o2, o3);
    const T r2 = T(0.70710678118654752440084436210485);
    // w8^1 = (1 -+ i)/sqrt2, w8^2 = -+ i, w8^3 = (-1 -+ i)/sqrt2
    cpx<T> w1 = INV ? mk(r2 * (o1.x - o1.y), r2 * (o1.y + o1.x)) : mk(r2 * (o1.x + o1.y), r2 * (o1.y - o1.x));
    cpx<T> w2 = mul_mi<T, INV>(o2);
    cpx<T> w3 = INV ? mk(r2 * (-o3.x - o3.y), r2 * (o3.x - o3.y)) : mk(r2 * (o3.y - o3.x), r2 * (-o3.x - o3.y));
    v[0] = add(e0, o0);
    v[4] = sub(e0, o0);
    v[1] = add(e1, w1);
    v[5] = sub(e1, w1);
    v[2] = add(e2, w2);
    v[6] = sub(e2, w2);
    v[3] = add(e3, w3);
    v[7] = sub(e3, w3);
  }
}

// ------------------------------------------------------------------------ LDS stages
// JFAST: consecutive threads take consecutive j (row layout, SJ = 1); otherwise
// consecutive b (column layout, SB = 1).  TPB threads per work-group.
template <typename T, int N, int NB, int SB, int SJ, int TS, bool JFAST, int R, int NS, bool INV, int TPB = NT>
__device__ __forceinline__ void fft_stage(cpx<T>* __restrict__ a, const cpx<T>* __restrict__ tw) {
  constexpr int NQ = N / R;
  constexpr int NBF = NB * NQ;
  constexpr int K = (NBF + TPB - 1) / TPB;
  const int tid = threadIdx.x;
  cpx<T> v[K][R];
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int u = tid + kk * TPB;
    if ((NBF % TPB == 0) || u < NBF) {
      const int b = JFAST ? u / NQ : u % NB;
      const int j = JFAST ? u % NQ : u / NB;
#pragma unroll
      for (int r = 0; r < R; ++r) v[kk][r] = a[b * SB + (j + r * NQ) * SJ];
    }
  }
  __syncthreads();
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int u = tid + kk * TPB;
    if ((NBF % TPB == 0) || u < NBF) {
      const int b = JFAST ? u / NQ : u % NB;
      const int j = JFAST ? u % NQ : u / NB;
      const int k = j % NS;
      if constexpr (NS > 1) {
        constexpr int STEP = N / (NS * R);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const cpx<T> w = tw[(r * k * STEP) * TS];
          v[kk][r] = INV ? mulc(v[kk][r], w) : mul(v[kk][r], w);
        }
      }
      dft<T, R, INV>(v[kk]);
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) a[b * SB + (base + r * NS) * SJ] = v[kk][r];
    }
  }
  __syncthreads();
}

template <typename T, int N, int NB, int SB, int SJ, int TS, bool JFAST, bool INV, int S, int NS, int TPB>
__device__ __forceinline__ void fft_stages(cpx<T>* a, const cpx<T>* tw) {
  if constexpr (S < fft_num_stages(N)) {
    constexpr int R = fft_stage_radix(N, S);
    fft_stage<T, N, NB, SB, SJ, TS, JFAST, R, NS, INV, TPB>(a, tw);
    fft_stages<T, N, NB, SB, SJ, TS, JFAST, INV, S + 1, NS * R, TPB>(a, tw);
  }
}

// Entry: caller has synchronised after filling `a`; returns synchronised.
template <typename T, int N, int NB, int SB, int SJ, int TS, bool JFAST, bool INV, int TPB = NT>
__device__ __forceinline__ void lds_fft(cpx<T>* a, const cpx<T>* tw) {
  fft_stages<T, N, NB, SB, SJ, TS, JFAST, INV, 0, 1, TPB>(a, tw);
}

}  // namespace wf
