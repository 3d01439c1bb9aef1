// Host-side launchers of the templated kernels (defined in the per-type units).
#pragma once
#include "wf_common.hpp"

namespace wf {

enum { CH_COLINV = 0, CH_ROW = 1, CH_COLFWD = 2 };

// supported grid sides: n % 8 == 0, n = 2^a or 3 * 2^a, 8 <= n <= 1024
bool chain_supported(int n);

// Tile choice of the transform chain: rows per work-group of the row pass (2, 4, 8),
// column blocks per work-group of the column passes (1, 2, 4), instances per launch
// (0 = all) and which passes use the register-staged FFT (bit 0: row pass, whose tile is
// then fixed by n; bit 1: column inverse; bit 2: column forward).  float32 supports every
// choice (register-staged passes for power-of-two n >= 128), float64 the defaults (4, 1,
// LDS-staged).  reg = 8 alone: the single-pass kernel (k_chain1) for maps whose field fits
// one work-group's LDS; the column-inverse call then runs all three passes of a solver's
// curvature product or gradient and the other two calls launch nothing.
struct ChainCfg {
  int rbv = 4;
  int cpb = 1;
  int group = 0;
  int reg = 0;
  int sim = 0;   // simulation passes (CM_SIM jobs): fixed LDS-staged variants, the other fields ignored
};

// Launch one pass of the transform chain for `batch` jobs.  Returns hipSuccess or the
// launch error; hipErrorInvalidValue if (n, c, cfg) has no instantiation.
hipError_t chain_launch_f32_s(int n, int c, int which, const ChainCfg& cfg, const Job* jobs, int batch,
                              const void* tw, hipStream_t st);
hipError_t chain_launch_f32_l(int n, int c, int which, const ChainCfg& cfg, const Job* jobs, int batch,
                              const void* tw, hipStream_t st);
hipError_t chain_launch_f64(int n, int c, int which, const ChainCfg& cfg, const Job* jobs, int batch,
                            const void* tw, hipStream_t st);
// one-time per-kernel set-up (LDS limits); must run outside stream capture
hipError_t chain_prepare_f32_s(int n, int c);
hipError_t chain_prepare_f32_l(int n, int c);
hipError_t chain_prepare_f64(int n, int c);

inline hipError_t chain_launch(int dtype, int n, int c, int which, const ChainCfg& cfg, const Job* jobs, int batch,
                               const void* tw, hipStream_t st) {
  if (dtype != 0) return chain_launch_f64(n, c, which, cfg, jobs, batch, tw, st);
  return n <= 96 ? chain_launch_f32_s(n, c, which, cfg, jobs, batch, tw, st)
                 : chain_launch_f32_l(n, c, which, cfg, jobs, batch, tw, st);
}
inline hipError_t chain_prepare(int dtype, int n, int c) {
  if (dtype != 0) return chain_prepare_f64(n, c);
  return n <= 96 ? chain_prepare_f32_s(n, c) : chain_prepare_f32_l(n, c);
}
inline bool chain_reg_supported(int dtype, int n) { return dtype == 0 && n >= 128 && (n & (n - 1)) == 0; }
// register-staged column passes: elements per thread cpb * c * TB * n / NT in [4, 32]
inline bool chain_regcol_supported(int n, int c, int cpb) {
  const int e = cpb * c * TB * n / NT;
  return e >= 4 && e <= 32;
}
// single pass: the field and the twiddles in at most 150 KB of LDS (n <= 128)
inline bool chain1_supported(int dtype, int n, int c) {
  return n <= 128 && (size_t)(n + c * n * (n / 2)) * (dtype != 0 ? 16 : 8) <= (size_t)150 * 1024;
}
inline bool chain_cfg_supported(int dtype, int n, int c, const ChainCfg& cfg) {
  if (cfg.reg == 8) return cfg.group == 0 && chain1_supported(dtype, n, c);
  if (dtype != 0) return cfg.rbv == 4 && cfg.cpb == 1 && cfg.reg == 0;
  const int ncb = n / 2 / TB;   // column blocks
  if (cfg.reg < 0 || cfg.reg > 7) return false;
  if (cfg.reg != 0 && !chain_reg_supported(dtype, n)) return false;
  if ((cfg.reg & 6) && !chain_regcol_supported(n, c, cfg.cpb)) return false;
  return (cfg.rbv == 2 || cfg.rbv == 4 || cfg.rbv == 8) && (cfg.cpb == 1 || cfg.cpb == 2 || cfg.cpb == 4) &&
         ncb % cfg.cpb == 0;
}

enum { LB_ZERO = 0, LB_INIT = 1, LB_POSTB = 2, LB_PASSA = 3, LB_COEF = 4, LB_PASSB = 5,
       LB_CGSTEP = 7, LB_CGPASS = 8, LB_CGPOST = 9, LB_CGDIR = 10 };
// pu: vector loads per thread per stream of the vector passes (PASS_U_FEW or PASS_U_MANY); the
// grid of a vector pass is (ceil(vector elements / (NT pu)), instances)
hipError_t lbfgs_launch(int dtype, int m, int pu, int which, dim3 grid, InstDesc* desc, LbState* st, Job* jobs,
                        int count, hipStream_t s);

// prior tables; with W non-null also the preconditioner (mean of W into meanW, a, ainv)
hipError_t prior_table_launch(int dtype, int n, int c, const double* pshape, const int32_t* band, const double* theta,
                              int nbands, const void* W, double* meanW, void* sq, int32_t* bandI, void* aT, void* ainvT,
                              hipStream_t s);
hipError_t unpack_launch(int dtype, int n, int c, int batch, const void* ext, void* in, hipStream_t s);
// tab: device [batch] of per-instance (internal field, sqrt S table, external output)
hipError_t pack_tab_launch(int dtype, int n, int c, int batch, const PackEntry* tab, hipStream_t s);
hipError_t pack_launch(int dtype, int n, int c, int batch, const void* in, int64_t inStride,
                       const void* sq, int fill, void* const* outs, void* out0, hipStream_t s);
hipError_t band_launch(int dtype, const BandJob* jobs, int count, int64_t L, hipStream_t s);
// simulation signal coefficients (external layout), squared-difference accumulation, output
hipError_t sim_coeffs_launch(int dtype, int n, int c, int nsim, int sim0, uint64_t seed, const void* draws,
                             const void* sq, void* out, hipStream_t s);
hipError_t sqdiff_acc_launch(int dtype, int64_t len, int P, int count, const void* a, const void* b, double* acc,
                             hipStream_t s);
hipError_t acc_out_launch(int dtype, int64_t len, const double* acc, double scale, void* out, hipStream_t s);
int band_nblk(int64_t L);
// float64 refinement: elementwise conversions (CvtJob, maxn = largest count) and the float32
// right-hand side with per-block norm partials of a float64 gradient (nblk blocks per job)
hipError_t convert_launch(const CvtJob* jobs, int count, int64_t maxn, hipStream_t s);
hipError_t refine_rhs_launch(const RhsJob* jobs, int count, int nblk, hipStream_t s);
// catalog response (wf_catalog.hpp): pad (blocks = N / 4), interpolation (blocks of NT
// galaxies of the largest catalog), spreading (blocks = tiles^2), unpad (blocks = n / 4);
// one launch for `count` instances of equal (n, c)
enum { CAT_PAD = 0, CAT_INTERP = 1, CAT_SPREAD = 2, CAT_UNPAD = 3 };
hipError_t cat_launch(int which, int c, int blocks, const Job* jobs, CatDesc* cats, int count, hipStream_t s);
hipError_t cat_table_launch(int n, int N, int c, const float* sq, const double* dk, float* T, hipStream_t s);
// catalog set-up: cell keys of the positions (pos [ngal][2] float64), the stable sort of
// (key, index) pairs on the low endBit bits (temp == nullptr: *tempBytes gets the workspace
// size and nothing runs), then the cells, weights and cell table in the sorted order
hipError_t cat_keys_launch(const double* pos, int ngal, int N, uint32_t* key, uint32_t* idx, int* bad, hipStream_t s);
hipError_t cat_sort_launch(void* temp, size_t* tempBytes, const uint32_t* kin, uint32_t* kout, const uint32_t* vin,
                           uint32_t* vout, int ngal, int endBit, hipStream_t s);
hipError_t cat_prep_launch(const double* pos, const uint32_t* skey, const uint32_t* perm, int ngal, int N,
                           int2* cell, float4* rec, int* cellStart, hipStream_t s);
// inter: the sorted side is [ngal][c] (interleaved) instead of [c][ngal]
hipError_t cat_permute_launch(const float* src, const int* perm, float* dst, int ngal, int c, int gather, int inter,
                              hipStream_t s);
// the states' scalars the host reads at the end of a solve, [batch] StateStat
hipError_t state_stats_launch(const LbState* st, StateStat* out, int batch, hipStream_t s);
// streaming copy of `bytes` (a multiple of 16) for the bandwidth reference
hipError_t stream_copy_launch(const void* src, void* dst, uint64_t bytes, hipStream_t s);

}  // namespace wf
