// Instantiation of the transform-chain kernels for one element type.  Included once
// per type by wf_chain_f32.hip / wf_chain_f64.hip with WF_T defined.
#include "wf_chain.hpp"
#include "wf_launch.hpp"

namespace wf {

template <typename T, int N, int C>
static size_t lds_colpass() { return (size_t)(N + N * C * TB) * sizeof(cpx<T>); }
template <typename T, int N, int C>
static size_t lds_rowpass() { return (size_t)(N + C * RB * (N / 2)) * sizeof(cpx<T>); }

template <typename T, int N, int C>
static hipError_t prep_t() {
  hipError_t e;
  e = hipFuncSetAttribute((const void*)k_colinv<T, N, C>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds_colpass<T, N, C>());
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_colfwd<T, N, C>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds_colpass<T, N, C>());
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_row<T, N, C>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds_rowpass<T, N, C>());
}

template <typename T, int N, int C>
static hipError_t launch_t(int which, const Job* jobs, int batch, const void* tw, hipStream_t st) {
  const cpx<T>* t = reinterpret_cast<const cpx<T>*>(tw);
  const size_t lc = lds_colpass<T, N, C>(), lr = lds_rowpass<T, N, C>();
  if (which == CH_COLINV) {
    k_colinv<T, N, C><<<dim3(N / 2 / TB, batch), dim3(NT), lc, st>>>(jobs, t);
  } else if (which == CH_ROW) {
    k_row<T, N, C><<<dim3(N / RB, batch), dim3(NT), lr, st>>>(jobs, t);
  } else {
    k_colfwd<T, N, C><<<dim3(N / 2 / TB, batch), dim3(NT), lc, st>>>(jobs, t);
  }
  return hipGetLastError();
}

#define WF_SIZES(X) X(8) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)

#define WF_CASE_L(N) \
  case N: return c == 1 ? launch_t<WF_T, N, 1>(which, jobs, batch, tw, st) : launch_t<WF_T, N, 2>(which, jobs, batch, tw, st);
#define WF_CASE_P(N) \
  case N: return c == 1 ? prep_t<WF_T, N, 1>() : prep_t<WF_T, N, 2>();

hipError_t WF_LAUNCH_NAME(int n, int c, int which, const Job* jobs, int batch, const void* tw, hipStream_t st) {
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
