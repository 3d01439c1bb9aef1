// Instantiation of the transform-chain kernels for one element type and a list of grid
// sides.  Included by the wf_chain_*.hip units with WF_T, WF_SIZES, WF_VARIANTS and the
// entry-point names defined.
#include "wf_chain.hpp"
#include "wf_launch.hpp"

namespace wf {

template <typename T, int N, int C, int CPB>
static size_t lds_colpass() { return (size_t)(N + N * CPB * C * TB) * sizeof(cpx<T>); }
template <typename T, int N, int C, int RBV>
static size_t lds_rowpass() { return (size_t)(N + C * RBV * (N / 2)) * sizeof(cpx<T>); }

template <typename T, int N, int C, int CPB>
static hipError_t prep_col() {
  if ((N / 2 / TB) % CPB != 0) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void*)k_colinv<T, N, C, CPB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds_colpass<T, N, C, CPB>());
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_colfwd<T, N, C, CPB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds_colpass<T, N, C, CPB>());
}
template <typename T, int N, int C, int RBV>
static hipError_t prep_row() {
  return hipFuncSetAttribute((const void*)k_row<T, N, C, RBV>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds_rowpass<T, N, C, RBV>());
}

template <typename T, int N, int C>
static hipError_t prep_t() {
  hipError_t e = prep_col<T, N, C, 1>();
  if (e == hipSuccess) e = prep_row<T, N, C, 4>();
#if WF_VARIANTS
  if (e == hipSuccess) e = prep_col<T, N, C, 2>();
  if (e == hipSuccess) e = prep_col<T, N, C, 4>();
  if (e == hipSuccess) e = prep_row<T, N, C, 2>();
  if (e == hipSuccess) e = prep_row<T, N, C, 8>();
#endif
  return e;
}

template <typename T, int N, int C, int CPB>
static void launch_col(int which, const Job* jobs, int batch, const cpx<T>* t, hipStream_t st) {
  const size_t lc = lds_colpass<T, N, C, CPB>();
  const dim3 grid(N / 2 / TB / CPB, batch);
  if (which == CH_COLINV)
    k_colinv<T, N, C, CPB><<<grid, dim3(NT), lc, st>>>(jobs, t);
  else
    k_colfwd<T, N, C, CPB><<<grid, dim3(NT), lc, st>>>(jobs, t);
}

template <typename T, int N, int C, int RBV>
static void launch_row(const Job* jobs, int batch, const cpx<T>* t, hipStream_t st) {
  k_row<T, N, C, RBV><<<dim3(N / RBV, batch), dim3(NT), lds_rowpass<T, N, C, RBV>(), st>>>(jobs, t);
}

template <typename T, int N, int C>
static hipError_t launch_t(int which, const ChainCfg& cfg, const Job* jobs, int batch, const void* tw,
                           hipStream_t st) {
  const cpx<T>* t = reinterpret_cast<const cpx<T>*>(tw);
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
