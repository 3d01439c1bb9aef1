// Instantiation of the transform-chain kernels for one element type and a list of grid
// sides.  Included by the wf_chain_*.hip units with WF_T, WF_SIZES, WF_VARIANTS and the
// entry-point names defined.
#include <algorithm>
#include <type_traits>
#include "wf_chain.hpp"
#include "wf_launch.hpp"

namespace wf {

template <typename T, int N, int C, int CPB>
static size_t lds_colpass() { return (size_t)(N + N * CPB * C * TB) * sizeof(cpx<T>); }
template <typename T, int N, int C, int RBV>
static size_t lds_rowpass() { return (size_t)(N + C * RBV * (N / 2)) * sizeof(cpx<T>); }

template <typename T, int N, int C, int CPB, bool SIMK = false>
static hipError_t prep_col() {
  if ((N / 2 / TB) % CPB != 0) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void*)k_colinv<T, N, C, CPB, SIMK>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_colpass<T, N, C, CPB>());
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_colfwd<T, N, C, CPB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds_colpass<T, N, C, CPB>());
}
template <typename T, int N, int C, int RBV, bool SIMK = false>
static hipError_t prep_row() {
  return hipFuncSetAttribute((const void*)k_row<T, N, C, RBV, SIMK>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds_rowpass<T, N, C, RBV>());
}

// register-staged passes: float32, power-of-two n >= 128
template <typename T, int N>
constexpr bool reg_ok() {
  return std::is_same<T, float>::value && N >= 128 && (N & (N - 1)) == 0;
}
template <int N, int C, int CPB>
constexpr bool regcol_ok() {
  return (N / 2 / TB) % CPB == 0 && CPB * C * TB * N / NT >= 4 && CPB * C * TB * N / NT <= 32;
}
template <int N, int C, int CPB>
static hipError_t prep_colr() {
  if constexpr (regcol_ok<N, C, CPB>()) {
    hipError_t e = hipFuncSetAttribute((const void*)k_colinvr<N, C, CPB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds_colr<N, C, CPB>());
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_colfwdr<N, C, CPB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds_colr<N, C, CPB>());
  }
  return hipSuccess;
}

// single-pass kernel: the field and the twiddles in at most 150 KB of LDS
template <typename T, int N, int C>
constexpr bool chain1_ok() {
  return N <= 128 && lds_chain1<T, N, C>() <= (size_t)150 * 1024;
}

template <typename T, int N, int C>
static hipError_t prep_t() {
  hipError_t e = hipSuccess;
  if constexpr (chain1_ok<T, N, C>())
    e = hipFuncSetAttribute((const void*)k_chain1<T, N, C>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds_chain1<T, N, C>());
  if (e == hipSuccess) e = prep_col<T, N, C, 1>();
  if (e == hipSuccess) e = prep_row<T, N, C, 4>();
  if (e == hipSuccess) e = prep_col<T, N, C, 1, true>();
  if (e == hipSuccess) e = prep_row<T, N, C, 4, true>();
#if WF_VARIANTS
  if (e == hipSuccess) e = prep_col<T, N, C, 2>();
  if (e == hipSuccess) e = prep_col<T, N, C, 4>();
  if (e == hipSuccess) e = prep_row<T, N, C, 2>();
  if (e == hipSuccess) e = prep_row<T, N, C, 8>();
  if constexpr (reg_ok<T, N>()) {
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)k_rowr<N, C>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds_rowr<N>());
    if (e == hipSuccess) e = prep_colr<N, C, 1>();
    if (e == hipSuccess) e = prep_colr<N, C, 2>();
    if (e == hipSuccess) e = prep_colr<N, C, 4>();
  }
#endif
  return e;
}

template <int N, int C, int CPB>
static hipError_t launch_colr(int which, const Job* jobs, int batch, const cpx<float>* t, hipStream_t st) {
  if constexpr (regcol_ok<N, C, CPB>()) {
    const dim3 grid(N / 2 / TB / CPB, batch);
    if (which == CH_COLINV)
      k_colinvr<N, C, CPB><<<grid, dim3(NT), lds_colr<N, C, CPB>(), st>>>(jobs, t);
    else
      k_colfwdr<N, C, CPB><<<grid, dim3(NT), lds_colr<N, C, CPB>(), st>>>(jobs, t);
    return hipSuccess;
  }
  return hipErrorInvalidValue;
}

template <typename T, int N, int C, int CPB, bool SIMK = false>
static void launch_col(int which, const Job* jobs, int batch, const cpx<T>* t, hipStream_t st) {
  const size_t lc = lds_colpass<T, N, C, CPB>();
  const dim3 grid(N / 2 / TB / CPB, batch);
  if (which == CH_COLINV)
    k_colinv<T, N, C, CPB, SIMK><<<grid, dim3(NT), lc, st>>>(jobs, t);
  else
    k_colfwd<T, N, C, CPB><<<grid, dim3(NT), lc, st>>>(jobs, t);
}

template <typename T, int N, int C, int RBV, bool SIMK = false>
static void launch_row(const Job* jobs, int batch, const cpx<T>* t, hipStream_t st) {
  k_row<T, N, C, RBV, SIMK><<<dim3(N / RBV, batch), dim3(NT), lds_rowpass<T, N, C, RBV>(), st>>>(jobs, t);
}

template <typename T, int N, int C>
static hipError_t launch_t(int which, const ChainCfg& cfg, const Job* jobs, int batch, const void* tw,
                           hipStream_t st) {
  const cpx<T>* t = reinterpret_cast<const cpx<T>*>(tw);
  if (cfg.reg == 8 && !cfg.sim) {   // single pass: launched by the column-inverse call
    if constexpr (chain1_ok<T, N, C>()) {
      if (which == CH_COLINV) k_chain1<T, N, C><<<dim3(batch), dim3(CHAIN1_NT), lds_chain1<T, N, C>(), st>>>(jobs, t);
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  if (cfg.sim) {   // simulation jobs: the LDS-staged passes with the simulation mode compiled in
    if (which == CH_ROW)
      launch_row<T, N, C, 4, true>(jobs, batch, t, st);
    else
      launch_col<T, N, C, 1, true>(which, jobs, batch, t, st);
    return hipGetLastError();
  }
#if WF_VARIANTS
  if constexpr (reg_ok<T, N>()) {
    const cpx<float>* tf = reinterpret_cast<const cpx<float>*>(tw);
    if (which == CH_ROW && (cfg.reg & 1)) {
      k_rowr<N, C><<<dim3(C * (N / rowr_rb(N)), batch), dim3(NT), lds_rowr<N>(), st>>>(jobs, tf);
      return hipGetLastError();
    }
    if ((which == CH_COLINV && (cfg.reg & 2)) || (which == CH_COLFWD && (cfg.reg & 4))) {
      hipError_t e = hipErrorInvalidValue;
      switch (cfg.cpb) {
        case 1: e = launch_colr<N, C, 1>(which, jobs, batch, tf, st); break;
        case 2: e = launch_colr<N, C, 2>(which, jobs, batch, tf, st); break;
        case 4: e = launch_colr<N, C, 4>(which, jobs, batch, tf, st); break;
        default: break;
      }
      return e != hipSuccess ? e : hipGetLastError();
    }
  }
#endif
  if ((which == CH_ROW && (cfg.reg & 1)) || (which == CH_COLINV && (cfg.reg & 2)) ||
      (which == CH_COLFWD && (cfg.reg & 4)))
    return hipErrorInvalidValue;
  if (which == CH_ROW) {
    switch (cfg.rbv) {
      case 4: launch_row<T, N, C, 4>(jobs, batch, t, st); break;
#if WF_VARIANTS
      case 2: launch_row<T, N, C, 2>(jobs, batch, t, st); break;
      case 8: launch_row<T, N, C, 8>(jobs, batch, t, st); break;
#endif
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (cfg.cpb) {
      case 1: launch_col<T, N, C, 1>(which, jobs, batch, t, st); break;
#if WF_VARIANTS
      case 2:
        if ((N / 2 / TB) % 2 != 0) return hipErrorInvalidValue;
        launch_col<T, N, C, 2>(which, jobs, batch, t, st);
        break;
      case 4:
        if ((N / 2 / TB) % 4 != 0) return hipErrorInvalidValue;
        launch_col<T, N, C, 4>(which, jobs, batch, t, st);
        break;
#endif
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

#define WF_CASE_L(N) \
  case N: return c == 1 ? launch_t<WF_T, N, 1>(which, cfg, jobs, batch, tw, st) : launch_t<WF_T, N, 2>(which, cfg, jobs, batch, tw, st);
#define WF_CASE_P(N) \
  case N: return c == 1 ? prep_t<WF_T, N, 1>() : prep_t<WF_T, N, 2>();

hipError_t WF_LAUNCH_NAME(int n, int c, int which, const ChainCfg& cfg, const Job* jobs, int batch, const void* tw,
                          hipStream_t st) {
  if (c != 1 && c != 2) return hipErrorInvalidValue;
  switch (n) {
    WF_SIZES(WF_CASE_L)
    default: return hipErrorInvalidValue;
  }
}

hipError_t WF_PREP_NAME(int n, int c) {
  if (c != 1 && c != 2) return hipErrorInvalidValue;
  switch (n) {
    WF_SIZES(WF_CASE_P)
    default: return hipErrorInvalidValue;
  }
}

}  // namespace wf
