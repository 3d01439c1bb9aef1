// Host-side launchers of the templated kernels (defined in the per-type units).
#pragma once
#include "wf_common.hpp"

namespace wf {

enum { CH_COLINV = 0, CH_ROW = 1, CH_COLFWD = 2 };

// supported grid sides: n % 8 == 0, n = 2^a or 3 * 2^a, 8 <= n <= 1024
bool chain_supported(int n);

// Launch one pass of the transform chain for `batch` jobs.  Returns hipSuccess or the
// launch error; hipErrorInvalidValue if (n, c) has no instantiation.
hipError_t chain_launch_f32(int n, int c, int which, const Job* jobs, int batch, const void* tw, hipStream_t st);
hipError_t chain_launch_f64(int n, int c, int which, const Job* jobs, int batch, const void* tw, hipStream_t st);
// one-time per-kernel set-up (LDS limits); must run outside stream capture
hipError_t chain_prepare_f32(int n, int c);
hipError_t chain_prepare_f64(int n, int c);

enum { LB_ZERO = 0, LB_INIT = 1, LB_POSTB = 2, LB_PASSA = 3, LB_COEF = 4, LB_PASSB = 5 };
hipError_t lbfgs_launch(int dtype, int m, int which, dim3 grid, InstDesc* desc, LbState* st, Job* jobs, int count,
                        hipStream_t s);

hipError_t prior_table_launch(int dtype, int n, int c, const double* pshape, const int32_t* band, const double* theta,
                              int nbands, void* sq, int32_t* bandI, hipStream_t s);
hipError_t unpack_launch(int dtype, int n, int c, int batch, const void* ext, void* in, hipStream_t s);
hipError_t pack_launch(int dtype, int n, int c, int batch, const void* in, int64_t inStride, int64_t vcs,
                       int64_t vcstr, const void* sq, int fill, void* const* outs, void* out0, hipStream_t s);
hipError_t band_launch(int dtype, const BandJob* jobs, int count, int64_t L, hipStream_t s);
int band_nblk(int64_t L);

}  // namespace wf
