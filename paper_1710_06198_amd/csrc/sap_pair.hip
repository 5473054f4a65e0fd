// The fine SAP with two right-hand sides per workgroup (lane pairs share
// every link and clover load); the block solve itself is in fine_site.h.
#include "fine_site.h"

template <typename T, bool CPL>
__global__ void __launch_bounds__(512, 1) k_sap_fine_pair(FineOp<T> op, const cplx<T>* __restrict__ eta, cplx<T>* z,
                                                         const double* __restrict__ mu_dev,
                                                         const int* __restrict__ blist, int nblk, int nrhs,
                                                         int mr_steps, T epsbar) {
  sap_block_solve<T, 1, true, CPL>(op, eta, z, mu_dev, blist, nblk, nrhs, mr_steps, epsbar);
}

void launch_sap_fine_pair(const FineOp<float>& op, const cplx<float>* eta, cplx<float>* z, int nrhs,
                          const double* mu_dev, const int* block_list, int nblk, int mr_steps, size_t lds_bytes,
                          unsigned n8, hipStream_t st, double epsbar) {
  const dim3 grid(n8 * ((nrhs + 1) / 2)), block(2 * op.g.bvol);
  if (epsbar != 0.0)
    hipLaunchKernelGGL((k_sap_fine_pair<float, true>), grid, block, lds_bytes, st, op, eta, z, mu_dev, block_list,
                       nblk, nrhs, mr_steps, (float)epsbar);
  else
    hipLaunchKernelGGL((k_sap_fine_pair<float, false>), grid, block, lds_bytes, st, op, eta, z, mu_dev, block_list,
                       nblk, nrhs, mr_steps, 0.0f);
}
