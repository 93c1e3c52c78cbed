// The greedy's orthonormal basis as a ROM stack (the certified decomposition of Algorithm 1):
// t^s = nu_s sum_j beta_j^s zeta_j + nu_s Delta^s, so with full-rule snapshots the cell tangent is
// sum_j (nu_s beta_j^s) zeta_j up to the greedy's tolerance.  With this stack the coefficients of the
// ROM apply are bounded by the snapshot norms, so the reduced-precision combination (the walk
// kernels of lat_apply.hip) meets no cancellation; with the principal tangents and alpha it is the
// same operator.
#include "lat_internal.h"

namespace {

// basis stack [a][e][cap] from Z [cap][nsnap]; coefficients c_ik = nu_i beta_ik
__global__ void k_basis_stack(int64_t nsnap, int cap, int n_r, const double *__restrict__ Z,
                              double *__restrict__ stack)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nsnap) return;
    for (int k = 0; k < cap; ++k) stack[j * cap + k] = k < n_r ? Z[(int64_t)k * nsnap + j] : 0.0;
}

__global__ void k_basis_coef(int64_t ncells, int cap, int n_r, const double *__restrict__ nu,
                             const double *__restrict__ beta, double *__restrict__ coef)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncells * cap) return;
    const int k = (int)(t % cap);
    const int64_t c = t / cap;
    coef[t] = k < n_r ? nu[c] * beta[t] : 0.0;
}

}  // namespace

extern "C" lat_status lat_basis_stack(const lat_plan *P, const double *Z, const double *nu, const double *beta,
                                      int32_t n_r, double *stack, double *coef, hipStream_t stream)
{
    if (!P || !Z || !nu || !beta || !stack || !coef) return LAT_E_ARG;
    if (n_r < 0 || n_r > P->cap) return LAT_E_SHAPE;
    hipLaunchKernelGGL(k_basis_stack, dim3((unsigned)lat_cdiv(P->nsnap, 256)), dim3(256), 0, stream, P->nsnap, P->cap,
                       n_r, Z, stack);
    hipLaunchKernelGGL(k_basis_coef, dim3((unsigned)lat_cdiv(P->ncells * P->cap, 256)), dim3(256), 0, stream,
                       P->ncells, P->cap, n_r, nu, beta, coef);
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}
