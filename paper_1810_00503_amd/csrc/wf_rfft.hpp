// Register-staged Stockham FFT for power-of-two lengths.
//
// Each thread keeps E elements of the work-group's NB transforms (length N, E * NT = NB * N)
// in registers.  A stage of radix R runs E / R register DFTs per thread; only between stages
// does data pass through LDS (one write and one read per element), so a transform with S
// stages costs S - 1 LDS round trips, and the first stage's inputs and the last stage's
// outputs never touch LDS: callers load them from and store them to global memory, or chain
// two transforms in registers (the last stage of one and the first stage of the next use the
// same radix and the same thread mapping).
//
// Stage s (radix R, NS = product of the radices before it, NQ = N / R) maps butterfly j of
// transform b:
//   inputs   element j + r NQ                               r = 0..R-1
//   twiddle  input r times w_{NS R}^{r (j mod NS)}          (conjugate for the inverse)
//   outputs  element (j div NS) NS R + (j mod NS) + r NS
// which is the self-sorting Stockham recursion; after the last stage (NS R = N) output r of
// butterfly j is element j + r NQ.  Butterfly u = tid + kk NT of a thread (kk < E / R) is
// (b, j) = (u / NQ, u % NQ) with JFAST (rows: consecutive threads take consecutive j) and
// (u % NB, u / NB) otherwise (columns: consecutive threads take consecutive transforms).
//
// Radix schedule: N = 2^L in S = ceil(L / log2 min(E, 32)) stages of nearly equal radix,
// larger radices first (REV reverses the order).  Register DFTs of radix 16 and 32 are
// split 4 x 4 and 8 x 4 with compile-time twiddles.
//
// Stage twiddles come from a table generated in float64 on the host: for stage s >= 1 the
// entries (r - 1) NS + k = w_{NS R}^{r k} (r in [1, R), k in [0, NS)) at offset NS - R_0, in
// all fewer than N entries per schedule.  The host keeps one table per (length, E, order)
// after the grid-side table w_n^k of the LDS Stockham kernels; tw_col_off / tw_row_off give
// their positions.
#pragma once
#include <type_traits>
#include "wf_fft.hpp"

namespace wf {

// compile-time loop: f(std::integral_constant<int, i>) for i in [B, E)
template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    sfor<B + 1, E>(f);
  }
}

__host__ __device__ constexpr int ilog2c(int x) {
  int l = 0;
  while ((1 << l) < x) ++l;
  return l;
}

__host__ __device__ constexpr int rs_nst(int N, int E) {
  const int L = ilog2c(N), b = ilog2c(E < 32 ? E : 32);
  return (L + b - 1) / b;
}
__host__ __device__ constexpr int rs_radix(int N, int E, bool rev, int s) {
  const int S = rs_nst(N, E), L = ilog2c(N);
  const int t = rev ? S - 1 - s : s;
  const int base = L / S, extra = L % S;
  return 1 << (base + (t < extra ? 1 : 0));
}
__host__ __device__ constexpr int rs_ns(int N, int E, bool rev, int s) {
  int p = 1;
  for (int t = 0; t < s; ++t) p *= rs_radix(N, E, rev, t);
  return p;
}

// positions (complex entries) of the stage-twiddle tables inside a grid side's twiddle
// array: [0, n) w_n^k; column schedules (length n) for E = 2..32 at n log2 E; row schedules
// (length n / 2) for E = 8, 16, 32 at n (3 + log2 E), forward order then reversed.
__host__ __device__ constexpr int64_t tw_col_off(int n, int E) { return (int64_t)n * ilog2c(E); }
__host__ __device__ constexpr int64_t tw_row_off(int n, int E, bool rev) {
  return (int64_t)n * (3 + ilog2c(E)) + (rev ? n / 2 : 0);
}
constexpr int64_t tw_ext_entries(int n) { return (int64_t)9 * n; }

// ------------------------------------------------------------------------ constant twiddles
// cos(pi m / 16) for any integer m
__host__ __device__ constexpr double cos_pi16(int m) {
  const double t[9] = {1.0,
                       0.98078528040323044912618224,
                       0.92387953251128675612818319,
                       0.83146961230254523707878838,
                       0.70710678118654752440084436,
                       0.55557023301960222474283081,
                       0.38268343236508977172845998,
                       0.19509032201612826784828487,
                       0.0};
  m = ((m % 32) + 32) % 32;
  return m <= 8 ? t[m] : (m <= 16 ? -t[16 - m] : (m <= 24 ? -t[m - 16] : t[32 - m]));
}

// a * w_R^X with w_R = exp(-2 pi i / R) (conjugated for INV); R divides 32
template <typename T, int R, int X, bool INV>
__device__ __forceinline__ cpx<T> cmul_w(cpx<T> a) {
  constexpr int m = (((X * (32 / R)) % 32) + 32) % 32;
  if constexpr (m == 0) {
    return a;
  } else if constexpr (m == 16) {
    return mk(-a.x, -a.y);
  } else if constexpr (m == 8) {
    return mul_mi<T, INV>(a);
  } else if constexpr (m == 24) {
    return mul_mi<T, !INV>(a);
  } else {
    constexpr double c = cos_pi16(m);
    constexpr double s = INV ? cos_pi16(8 - m) : -cos_pi16(8 - m);
    return mk(T(c) * a.x - T(s) * a.y, T(c) * a.y + T(s) * a.x);
  }
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void rdft(cpx<T>* v);

// DFT of length R1 R2 in registers: x[j1 + R1 j2] -> X[k2 + R2 k1]
template <typename T, int R1, int R2, bool INV>
__device__ __forceinline__ void rdft_split(cpx<T>* v) {
  constexpr int R = R1 * R2;
  cpx<T> y[R];
  sfor<0, R1>([&](auto J1) {
    constexpr int j1 = decltype(J1)::value;
    cpx<T> t[R2];
    sfor<0, R2>([&](auto J2) { t[decltype(J2)::value] = v[j1 + R1 * decltype(J2)::value]; });
    rdft<T, R2, INV>(t);
    sfor<0, R2>([&](auto K2) {
      constexpr int k2 = decltype(K2)::value;
      y[j1 * R2 + k2] = cmul_w<T, R, j1 * k2, INV>(t[k2]);
    });
  });
  sfor<0, R2>([&](auto K2) {
    constexpr int k2 = decltype(K2)::value;
    cpx<T> u[R1];
    sfor<0, R1>([&](auto J1) { u[decltype(J1)::value] = y[decltype(J1)::value * R2 + k2]; });
    rdft<T, R1, INV>(u);
    sfor<0, R1>([&](auto K1) { v[k2 + R2 * decltype(K1)::value] = u[decltype(K1)::value]; });
  });
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void rdft(cpx<T>* v) {
  if constexpr (R == 1) {
  } else if constexpr (R == 16) {
    rdft_split<T, 4, 4, INV>(v);
  } else if constexpr (R == 32) {
    rdft_split<T, 8, 4, INV>(v);
  } else {
    dft<T, R, INV>(v);
  }
}

// ------------------------------------------------------------------------ transform
// v: on entry stage 0's inputs, on exit the last stage's outputs (see above).  lds: exchange
// buffer addressed by lid(b, i); stw: this schedule's stage-twiddle table (LDS or global);
// tid: the thread's index in the work-group.
// Starts every exchange with a barrier, so the caller may still have LDS reads in flight
// from the previous use of the buffer; returns without a trailing barrier.
template <typename T, int N, int NB, int E, bool JFAST, bool INV, bool REV, typename LID>
__device__ __forceinline__ void rs_fft(cpx<T> (&v)[E], cpx<T>* __restrict__ lds, const cpx<T>* __restrict__ stw,
                                       LID lid, uint32_t tid) {
  static_assert(NB * N == E * NT, "E elements per thread");
  constexpr int NST = rs_nst(N, E);
  constexpr int R0 = rs_radix(N, E, REV, 0);
  sfor<0, NST>([&](auto S_) {
    constexpr int s = decltype(S_)::value;
    constexpr int R = rs_radix(N, E, REV, s), NS = rs_ns(N, E, REV, s), NQ = N / R, K = E / R;
    if constexpr (s > 0) {
      constexpr int off = NS - R0;
      sfor<0, K>([&](auto KK) {
        constexpr int kk = decltype(KK)::value;
        const uint32_t u = tid + kk * NT;
        const uint32_t j = JFAST ? u % NQ : u / NB;
        const uint32_t k = j % NS;
        sfor<1, R>([&](auto RR) {
          constexpr int r = decltype(RR)::value;
          const cpx<T> w = stw[off + (r - 1) * NS + k];
          v[kk * R + r] = INV ? mulc(v[kk * R + r], w) : mul(v[kk * R + r], w);
        });
      });
    }
    sfor<0, K>([&](auto KK) { rdft<T, R, INV>(&v[decltype(KK)::value * R]); });
    if constexpr (s + 1 < NST) {
      __syncthreads();
      sfor<0, K>([&](auto KK) {
        constexpr int kk = decltype(KK)::value;
        const uint32_t u = tid + kk * NT;
        const uint32_t b = JFAST ? u / NQ : u % NB, j = JFAST ? u % NQ : u / NB;
        const uint32_t base = (j / NS) * NS * R + (j % NS);
        sfor<0, R>([&](auto RR) {
          constexpr int r = decltype(RR)::value;
          lds[lid(b, base + r * NS)] = v[kk * R + r];
        });
      });
      __syncthreads();
      constexpr int R2 = rs_radix(N, E, REV, s + 1), NQ2 = N / R2, K2 = E / R2;
      sfor<0, K2>([&](auto KK) {
        constexpr int kk = decltype(KK)::value;
        const uint32_t u = tid + kk * NT;
        const uint32_t b = JFAST ? u / NQ2 : u % NB, j = JFAST ? u % NQ2 : u / NB;
        sfor<0, R2>([&](auto RR) {
          constexpr int r = decltype(RR)::value;
          v[kk * R2 + r] = lds[lid(b, j + r * NQ2)];
        });
      });
    }
  });
}

// value of the lane whose index differs in bit 1 (partner component of a column pair);
// every lane of the wave must be active
__device__ __forceinline__ float lane_xor2(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4E, 0xF, 0xF, false));
}

}  // namespace wf
