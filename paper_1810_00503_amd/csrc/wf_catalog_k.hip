// Host launchers of the catalog-response kernels (wf_catalog.hpp).
#include <rocprim/device/device_radix_sort.hpp>

#include "wf_catalog.hpp"
#include "wf_launch.hpp"

namespace wf {

hipError_t cat_launch(int which, int c, int blocks, const Job* jobs, CatDesc* cats, int count, hipStream_t s) {
  if (count <= 0 || blocks <= 0) return hipSuccess;
  const dim3 g(blocks, count);
  if (c != 1 && c != 2) return hipErrorInvalidValue;
  switch (which) {
    case CAT_PAD:
      if (c == 1) k_cat_pad<1><<<g, NT, 0, s>>>(jobs, cats); else k_cat_pad<2><<<g, NT, 0, s>>>(jobs, cats);
      break;
    case CAT_INTERP:
      if (c == 1) k_cat_interp<1><<<g, NT, 0, s>>>(jobs, cats); else k_cat_interp<2><<<g, NT, 0, s>>>(jobs, cats);
      break;
    case CAT_SPREAD:
      if (c == 1) k_cat_spread<1><<<g, CAT_SPREAD_NT, 0, s>>>(jobs, cats);
      else k_cat_spread<2><<<g, CAT_SPREAD_NT, 0, s>>>(jobs, cats);
      break;
    case CAT_UNPAD:
      if (c == 1) k_cat_unpad<1><<<g, CAT_UNPAD_NT, 0, s>>>(jobs, cats);
      else k_cat_unpad<2><<<g, CAT_UNPAD_NT, 0, s>>>(jobs, cats);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t cat_table_launch(int n, int N, int c, const float* sq, const double* dk, float* T, hipStream_t s) {
  const int64_t tot = (int64_t)c * n * (n / 2);
  const unsigned b = (unsigned)std::min<int64_t>((tot + 255) / 256, 4096);
  k_cat_table<<<b, 256, 0, s>>>(n, N, c, sq, dk, T);
  return hipGetLastError();
}

hipError_t cat_keys_launch(const double* pos, int ngal, int N, uint32_t* key, uint32_t* idx, int* bad, hipStream_t s) {
  if (ngal <= 0) return hipSuccess;
  const unsigned b = (unsigned)std::min<int64_t>(((int64_t)ngal + 255) / 256, 4096);
  k_cat_keys<<<b, 256, 0, s>>>(pos, ngal, N, key, idx, bad);
  return hipGetLastError();
}

hipError_t cat_sort_launch(void* temp, size_t* tempBytes, const uint32_t* kin, uint32_t* kout, const uint32_t* vin,
                           uint32_t* vout, int ngal, int endBit, hipStream_t s) {
  // LSD radix sort: stable, so galaxies of one cell keep their input order
  return rocprim::radix_sort_pairs(temp, *tempBytes, kin, kout, vin, vout, (size_t)ngal, 0u, (unsigned)endBit, s);
}

hipError_t cat_prep_launch(const double* pos, const uint32_t* skey, const uint32_t* perm, int ngal, int N,
                           int2* cell, float4* rec, int* cellStart, hipStream_t s) {
  if (ngal <= 0) return hipSuccess;
  const unsigned b = (unsigned)std::min<int64_t>(((int64_t)ngal + 255) / 256, 4096);
  k_cat_prep<<<b, 256, 0, s>>>(pos, skey, perm, ngal, N, cell, rec, cellStart);
  return hipGetLastError();
}

hipError_t cat_permute_launch(const float* src, const int* perm, float* dst, int ngal, int c, int gather, int inter,
                              hipStream_t s) {
  const int64_t tot = (int64_t)c * ngal;
  if (tot <= 0) return hipSuccess;
  const unsigned b = (unsigned)std::min<int64_t>((tot + 255) / 256, 4096);
  k_cat_permute<<<b, 256, 0, s>>>(src, perm, dst, ngal, c, gather, inter);
  return hipGetLastError();
}

}  // namespace wf
