// Instantiations and host launchers of the solver, table, packing and band kernels.
#include "wf_solver.hpp"
#include "wf_launch.hpp"

namespace wf {

bool chain_supported(int n) {
  if (n < 8 || n > 1024 || (n % 8) != 0) return false;
  int m = n;
  if (m % 3 == 0) m /= 3;
  return (m & (m - 1)) == 0;
}

template <typename T, int M>
static hipError_t lb_t(int which, int pu, dim3 grid, InstDesc* desc, LbState* st, Job* jobs, int count, hipStream_t s) {
  const bool many = pu == PASS_U_MANY;
  switch (which) {
    case LB_ZERO: k_zero<T><<<grid, dim3(256), 0, s>>>(desc, count); break;
    case LB_INIT: k_init<<<dim3((count + 63) / 64), dim3(64), 0, s>>>(desc, st, jobs, count); break;
    case LB_POSTB: k_postB<M><<<dim3(count), dim3(256), 0, s>>>(desc, st, jobs); break;
    case LB_PASSA:
      if (many) k_passA<T, M, PASS_U_MANY><<<grid, dim3(NT), 0, s>>>(desc, st);
      else k_passA<T, M, PASS_U_FEW><<<grid, dim3(NT), 0, s>>>(desc, st);
      break;
    case LB_COEF: k_coef<M><<<dim3(count), dim3(256), 0, s>>>(desc, st, jobs); break;
    case LB_PASSB:
      if (many) k_passB<T, M, PASS_U_MANY><<<grid, dim3(NT), 0, s>>>(desc, st);
      else k_passB<T, M, PASS_U_FEW><<<grid, dim3(NT), 0, s>>>(desc, st);
      break;
    case LB_CGSTEP: k_cg_step<<<dim3(count), dim3(256), 0, s>>>(desc, st, jobs); break;
    case LB_CGPASS:
      if (many) k_cg_pass<T, PASS_U_MANY><<<grid, dim3(NT), 0, s>>>(desc, st);
      else k_cg_pass<T, PASS_U_FEW><<<grid, dim3(NT), 0, s>>>(desc, st);
      break;
    case LB_CGPOST: k_cg_post<<<dim3(count), dim3(256), 0, s>>>(desc, st, jobs); break;
    case LB_CGDIR:
      if (many) k_cg_dir<T, PASS_U_MANY><<<grid, dim3(NT), 0, s>>>(desc, st);
      else k_cg_dir<T, PASS_U_FEW><<<grid, dim3(NT), 0, s>>>(desc, st);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t lb_m(int m, int which, int pu, dim3 grid, InstDesc* desc, LbState* st, Job* jobs, int count,
                       hipStream_t s) {
  switch (m) {
#define WF_M(M) case M: return lb_t<T, M>(which, pu, grid, desc, st, jobs, count, s);
    WF_M(1) WF_M(2) WF_M(3) WF_M(4) WF_M(5) WF_M(6) WF_M(7) WF_M(8)
    WF_M(9) WF_M(10) WF_M(11) WF_M(12) WF_M(13) WF_M(14) WF_M(15) WF_M(16)
#undef WF_M
    default: return hipErrorInvalidValue;
  }
}

hipError_t lbfgs_launch(int dtype, int m, int pu, int which, dim3 grid, InstDesc* desc, LbState* st, Job* jobs,
                        int count, hipStream_t s) {
  if (pu != PASS_U_FEW && pu != PASS_U_MANY) return hipErrorInvalidValue;
  return dtype == 0 ? lb_m<float>(m, which, pu, grid, desc, st, jobs, count, s)
                    : lb_m<double>(m, which, pu, grid, desc, st, jobs, count, s);
}

static dim3 flat_grid(int64_t tot) {
  int64_t b = (tot + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}

hipError_t prior_table_launch(int dtype, int n, int c, const double* pshape, const int32_t* band, const double* theta,
                              int nbands, const void* W, double* meanW, void* sq, int32_t* bandI, void* aT, void* ainvT,
                              hipStream_t s) {
  const dim3 g = flat_grid((int64_t)c * n * (n / 2));
  if (W) {
    if (dtype == 0)
      k_mean_w<float><<<1, 1024, 0, s>>>((const float*)W, (int64_t)n * n, meanW);
    else
      k_mean_w<double><<<1, 1024, 0, s>>>((const double*)W, (int64_t)n * n, meanW);
  }
  const double* mw = W ? meanW : nullptr;
  if (dtype == 0)
    k_prior_table<float><<<g, 256, 0, s>>>(n, c, pshape, band, theta, nbands, mw, (float*)sq, bandI, (float*)aT,
                                          (float*)ainvT);
  else
    k_prior_table<double><<<g, 256, 0, s>>>(n, c, pshape, band, theta, nbands, mw, (double*)sq, bandI, (double*)aT,
                                           (double*)ainvT);
  return hipGetLastError();
}

hipError_t unpack_launch(int dtype, int n, int c, int batch, const void* ext, void* in, hipStream_t s) {
  const dim3 g = flat_grid((int64_t)batch * c * n * (n / 2));
  if (dtype == 0)
    k_unpack<float><<<g, 256, 0, s>>>(n, c, batch, (const cpx<float>*)ext, (cpx<float>*)in);
  else
    k_unpack<double><<<g, 256, 0, s>>>(n, c, batch, (const cpx<double>*)ext, (cpx<double>*)in);
  return hipGetLastError();
}

hipError_t pack_launch(int dtype, int n, int c, int batch, const void* in, int64_t inStride,
                       const void* sq, int fill, void* const* outs, void* out0, hipStream_t s) {
  const dim3 g = flat_grid((int64_t)batch * c * n * (n / 2 + 1));
  if (dtype == 0)
    k_pack<float><<<g, 256, 0, s>>>(n, c, batch, (const cpx<float>*)in, inStride, (const float*)sq, fill,
                                    (cpx<float>* const*)outs, (cpx<float>*)out0);
  else
    k_pack<double><<<g, 256, 0, s>>>(n, c, batch, (const cpx<double>*)in, inStride, (const double*)sq, fill,
                                     (cpx<double>* const*)outs, (cpx<double>*)out0);
  return hipGetLastError();
}

hipError_t pack_tab_launch(int dtype, int n, int c, int batch, const PackEntry* tab, hipStream_t s) {
  const dim3 g = flat_grid((int64_t)batch * c * n * (n / 2 + 1));
  if (dtype == 0)
    k_pack_tab<float><<<g, 256, 0, s>>>(n, c, batch, tab);
  else
    k_pack_tab<double><<<g, 256, 0, s>>>(n, c, batch, tab);
  return hipGetLastError();
}

hipError_t sim_coeffs_launch(int dtype, int n, int c, int nsim, int sim0, uint64_t seed, const void* draws,
                             const void* sq, void* out, hipStream_t s) {
  const dim3 g = flat_grid((int64_t)nsim * c * n * (n / 2 + 1));
  if (dtype == 0)
    k_sim_coeffs<float><<<g, 256, 0, s>>>(n, c, nsim, sim0, seed, (const float*)draws, (const float*)sq,
                                          (cpx<float>*)out);
  else
    k_sim_coeffs<double><<<g, 256, 0, s>>>(n, c, nsim, sim0, seed, (const double*)draws, (const double*)sq,
                                           (cpx<double>*)out);
  return hipGetLastError();
}

hipError_t sqdiff_acc_launch(int dtype, int64_t len, int P, int count, const void* a, const void* b, double* acc,
                             hipStream_t s) {
  const dim3 g = flat_grid(len);
  if (dtype == 0)
    k_sqdiff_acc<float><<<g, 256, 0, s>>>(len, P, count, (const float*)a, (const float*)b, acc);
  else
    k_sqdiff_acc<double><<<g, 256, 0, s>>>(len, P, count, (const double*)a, (const double*)b, acc);
  return hipGetLastError();
}

hipError_t acc_out_launch(int dtype, int64_t len, const double* acc, double scale, void* out, hipStream_t s) {
  const dim3 g = flat_grid(len);
  if (dtype == 0)
    k_acc_out<float><<<g, 256, 0, s>>>(len, acc, scale, (float*)out);
  else
    k_acc_out<double><<<g, 256, 0, s>>>(len, acc, scale, (double*)out);
  return hipGetLastError();
}

int band_nblk(int64_t L) { return (int)((L + (int64_t)NT * BAND_EPT - 1) / ((int64_t)NT * BAND_EPT)); }

hipError_t band_launch(int dtype, const BandJob* jobs, int count, int64_t L, hipStream_t s) {
  const int nb = band_nblk(L);
  if (dtype == 0)
    k_band_part<float><<<dim3(nb, count), NT, 0, s>>>(jobs);
  else
    k_band_part<double><<<dim3(nb, count), NT, 0, s>>>(jobs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_band_final<<<dim3(count), dim3(64), 0, s>>>(jobs, nb);
  return hipGetLastError();
}

hipError_t convert_launch(const CvtJob* jobs, int count, int64_t maxn, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t b = (maxn + 255) / 256;
  b = b < 1 ? 1 : (b > 1024 ? 1024 : b);
  k_convert<<<dim3((unsigned)b, count), 256, 0, s>>>(jobs);
  return hipGetLastError();
}

hipError_t refine_rhs_launch(const RhsJob* jobs, int count, int nblk, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  k_refine_rhs<<<dim3(nblk, count), 256, 0, s>>>(jobs);
  return hipGetLastError();
}

hipError_t state_stats_launch(const LbState* st, StateStat* out, int batch, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  k_state_stats<<<dim3((unsigned)((batch + 255) / 256)), 256, 0, s>>>(st, out, batch);
  return hipGetLastError();
}

hipError_t stream_copy_launch(const void* src, void* dst, uint64_t bytes, hipStream_t s) {
  const uint64_t n = bytes / 16;
  const uint64_t blocks = (n + 256 * COPY_U - 1) / (256 * COPY_U);
  if (blocks == 0 || blocks > 0x7fffffffull) return hipErrorInvalidValue;
  k_stream_copy<<<dim3((unsigned)blocks), 256, 0, s>>>((const float4*)src, (float4*)dst, n);
  return hipGetLastError();
}

}  // namespace wf
