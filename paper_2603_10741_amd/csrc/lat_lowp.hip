// Reduced-precision ROM apply: Y_i = M_i (sum_k c_ik B_k) M_i X_i with the stack B and the
// coefficients c held in low precision.
//
//   LAT_F32   stack and coefficients rounded to FP32; combination and apply on the FP32 VALU.
//   LAT_BF16  the combination sum_k c_ik B_k -- the dense (entries x principals) x (principals x
//             cells) contraction -- runs on the bf16 matrix cores with FP32 accumulation.  Each
//             FP64 operand is split into bf16 slices x = x0 + x1 + x2 (x1 = bf16(x - x0), ...,
//             remainders formed in FP64) and the slice products are grouped by level
//             p + q = 0, 1, 2; each level accumulates in its own FP32 register and the levels are
//             summed in FP64 (smallest first).  The number of levels follows refine_tol
//             (2^-8, 2^-16, 2^-24 per level).  The combined block goes through LDS (row = cell)
//             so that each lane then applies its own cell's block to its right-hand sides in FP32.
//
// Used with the greedy's orthonormal basis (stack = zeta_j, c_ij = nu_i beta_ij; see
// lat_basis_stack) the coefficients are bounded by the snapshot norm and the combination has no
// cancellation; with the principal tangents and alpha it computes the same operator.
#include "lat_internal.h"

namespace {

using bf16x8 = lat_bf16x8;
using f32x4 = lat_f32x4;

template <int DIM>
struct Geo {
    static constexpr int NO = DIM == 2 ? 9 : 27;
    static constexpr int E = NO * DIM * DIM;
    static constexpr int NPL = DIM == 2 ? 1 : 3;           // stencil planes (offset z = -1, 0, 1 in 3D)
    static constexpr int OPP = NO / NPL;                  // offsets per plane
    static constexpr int EPL = OPP * DIM * DIM;           // entries per plane (36 / 81)
    static constexpr int EPP = (EPL + 15) / 16 * 16;      // padded to the 16-row matrix tiles (48 / 96)
};

__device__ __forceinline__ void slice3(double x, uint16_t s[3]) { lat_slice3(x, s); }

// stack [a][e][cap] (FP64) -> slices [lev][a][NPL*EPP][64]; row plane*EPP + t holds entry plane*EPL + t
__global__ void k_slice_stack(int64_t nloc, int E, int EPL, int EPP, int EP, int cap, int n_r,
                              const double *__restrict__ K, uint16_t *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // over nloc*EP*64
    const int64_t tot = nloc * EP * 64;
    if (t >= tot) return;
    const int k = (int)(t % 64);
    const int64_t rest = t / 64;
    const int row = (int)(rest % EP);
    const int64_t a = rest / EP;
    const int plane = row / EPP, tt = row % EPP;
    uint16_t s[3] = {0, 0, 0};
    if (k < n_r && tt < EPL) slice3(K[(a * E + plane * EPL + tt) * cap + k], s);
#pragma unroll
    for (int lev = 0; lev < 3; ++lev) out[lev * tot + t] = s[lev];
}

// coefficients [N_s][cap] canonical -> slices [lev][ld][64] (plan order)
__global__ void k_slice_coef(int64_t ld, int cap, int n_r, const int32_t *__restrict__ perm,
                             const double *__restrict__ c, uint16_t *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // over ld*64
    if (t >= ld * 64) return;
    const int k = (int)(t % 64);
    const int64_t p = t / 64;
    const int cell = perm[p];
    uint16_t s[3] = {0, 0, 0};
    if (cell >= 0 && k < n_r) slice3(c[(int64_t)cell * cap + k], s);
#pragma unroll
    for (int lev = 0; lev < 3; ++lev) out[lev * ld * 64 + t] = s[lev];
}

__global__ void k_to_f32_stack(int64_t n, const double *__restrict__ K, float *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[t] = (float)K[t];
}

__global__ void k_to_f32_coef(int64_t ld, int cap, int n_r, const int32_t *__restrict__ perm,
                              const double *__restrict__ c, float *__restrict__ out)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (p >= ld) return;
    const int cell = perm[p];
    out[(int64_t)k * ld + p] = (cell >= 0 && k < n_r) ? (float)c[(int64_t)cell * cap + k] : 0.0f;
}

__global__ void k_fill0(int64_t n, double *__restrict__ y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = 0.0;
}

struct LowpArgs {
    int nn, m, cap, n_r, nch, chunks_per_group, ngroups;
    int64_t ld, nloc;
    const int32_t *goff, *unode, *unbr;
    const uint64_t *umask;
    const uint16_t *kslice, *cslice;   // bf16
    const float *kf32, *cf32;          // f32
    const double *X;
    double *Y;
};

// bf16 matrix-core path.  One wave (64 lanes = 64 cells of a group) per block; the stencil is
// combined and applied one plane of offsets at a time to bound the LDS footprint.
template <int DIM, int NKB, int NLEV, int MC>
__global__ __launch_bounds__(64) void k_apply_bf16(LowpArgs A)
{
    using G = Geo<DIM>;
    constexpr int EPL = G::EPL, EPP = G::EPP, NMB = EPP / 16, LDW = EPP + 1, NPL = G::NPL, OPP = G::OPP;
    constexpr int EP = NPL * EPP;
    __shared__ float kt_s[64 * LDW];
    const int wave = lat_xcd_block(blockIdx.x, gridDim.x), l = threadIdx.x;
    const int g = wave / A.chunks_per_group, ch = wave % A.chunks_per_group;
    if (g >= A.ngroups) return;
    const int q0 = A.goff[g] + ch * A.nch;
    const int q1 = min(A.goff[g + 1], q0 + A.nch);
    if (q0 >= q1) return;
    const int m = A.m;
    const int lr = l & 15, lk = (l >> 4) * 8;
    const int64_t slice_c = A.ld * 64, slice_k = A.nloc * EP * 64;
    // coefficient operands (B: k x cells): lane holds cell nb*16 + lr, k = kb*32 + lk .. +7
    bf16x8 cb[NLEV][4][NKB];
#pragma unroll
    for (int lev = 0; lev < NLEV; ++lev)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
            for (int kb = 0; kb < NKB; ++kb)
                cb[lev][nb][kb] = *reinterpret_cast<const bf16x8 *>(
                    A.cslice + lev * slice_c + ((int64_t)g * 64 + nb * 16 + lr) * 64 + kb * 32 + lk);
    for (int q = q0; q < q1; ++q) {
        const int a = A.unode[q];
        const bool own = (A.umask[q] >> l) & 1;
        float acc_y[DIM][MC];
#pragma unroll
        for (int i = 0; i < DIM; ++i)
#pragma unroll
            for (int c = 0; c < MC; ++c) acc_y[i][c] = 0.f;
        for (int pl = 0; pl < NPL; ++pl) {
            // ---- combination on the matrix cores: Ktilde[entry][cell] for this plane
#pragma unroll
            for (int mb = 0; mb < NMB; ++mb) {
                bf16x8 ka[NLEV][NKB];
#pragma unroll
                for (int lev = 0; lev < NLEV; ++lev)
#pragma unroll
                    for (int kb = 0; kb < NKB; ++kb)
                        ka[lev][kb] = *reinterpret_cast<const bf16x8 *>(
                            A.kslice + lev * slice_k + ((int64_t)a * EP + pl * EPP + mb * 16 + lr) * 64 + kb * 32 + lk);
#pragma unroll
                for (int nb = 0; nb < 4; ++nb) {
                    f32x4 acc[NLEV];
#pragma unroll
                    for (int lev = 0; lev < NLEV; ++lev) acc[lev] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
                        for (int lev = 0; lev < NLEV; ++lev)
#pragma unroll
                            for (int pc = 0; pc <= lev; ++pc)
                                acc[lev] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ka[lev - pc][kb], cb[pc][nb][kb],
                                                                                  acc[lev], 0, 0, 0);
                    // D[i][j]: this lane holds column j = lr (cell nb*16 + lr), rows i = 4 (l >> 4) + r
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        double v = 0.0;
#pragma unroll
                        for (int lev = NLEV - 1; lev >= 0; --lev) v += (double)acc[lev][r];
                        kt_s[(nb * 16 + lr) * LDW + mb * 16 + 4 * (l >> 4) + r] = (float)v;
                    }
                }
            }
            __syncthreads();
            // ---- apply this plane's offsets: lane = cell
            for (int oo = 0; oo < OPP; ++oo) {
                const int o = pl * OPP + oo;
                const int nb = A.unbr[(int64_t)q * G::NO + o];
                if (nb < 0) continue;
                const bool nb_own = (A.umask[nb] >> l) & 1;
                float kt[DIM][DIM];
#pragma unroll
                for (int i = 0; i < DIM; ++i)
#pragma unroll
                    for (int j = 0; j < DIM; ++j) kt[i][j] = kt_s[l * LDW + (oo * DIM + i) * DIM + j];
#pragma unroll
                for (int j = 0; j < DIM; ++j)
#pragma unroll
                    for (int c = 0; c < MC; ++c) {
                        const float x = nb_own ? (float)A.X[(((int64_t)nb * DIM + j) * m + c) * 64 + l] : 0.f;
#pragma unroll
                        for (int i = 0; i < DIM; ++i) acc_y[i][c] = fmaf(kt[i][j], x, acc_y[i][c]);
                    }
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < DIM; ++i)
#pragma unroll
            for (int c = 0; c < MC; ++c)
                A.Y[(((int64_t)q * DIM + i) * m + c) * 64 + l] = own ? (double)acc_y[i][c] : 0.0;
    }
}

// FP32 VALU path: same structure as the FP64 apply with FP32 operands.
template <int DIM, int MC, int NR>
__global__ __launch_bounds__(256) void k_apply_f32(LowpArgs A)
{
    using G = Geo<DIM>;
    constexpr int E = G::E;
    const int wave = __builtin_amdgcn_readfirstlane(lat_xcd_block(blockIdx.x, gridDim.x) * 4 + (int)(threadIdx.x >> 6));
    const int l = threadIdx.x & 63;
    const int g = wave / A.chunks_per_group, ch = wave % A.chunks_per_group;
    if (g >= A.ngroups) return;
    const int q0 = A.goff[g] + ch * A.nch;
    const int q1 = min(A.goff[g + 1], q0 + A.nch);
    if (q0 >= q1) return;
    const int64_t p = (int64_t)g * 64 + l;
    const int m = A.m;
    float cf[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) cf[k] = k < A.n_r ? A.cf32[(int64_t)k * A.ld + p] : 0.f;
    for (int q = q0; q < q1; ++q) {
        const int a = A.unode[q];
        const bool own = (A.umask[q] >> l) & 1;
        for (int c0 = 0; c0 < m; c0 += MC) {
            float acc[DIM][MC];
#pragma unroll
            for (int i = 0; i < DIM; ++i)
#pragma unroll
                for (int c = 0; c < MC; ++c) acc[i][c] = 0.f;
            for (int o = 0; o < G::NO; ++o) {
                const int nb = A.unbr[(int64_t)q * G::NO + o];
                if (nb < 0) continue;
                const bool nb_own = (A.umask[nb] >> l) & 1;
                float kt[DIM][DIM];
#pragma unroll
                for (int i = 0; i < DIM; ++i)
#pragma unroll
                    for (int j = 0; j < DIM; ++j) {
                        const float *kp = A.kf32 + ((int64_t)a * E + (o * DIM + i) * DIM + j) * A.cap;
                        float s = 0.f;
#pragma unroll
                        for (int k = 0; k < NR; ++k)
                            if (k < A.n_r) s = fmaf(cf[k], kp[k], s);
                        kt[i][j] = s;
                    }
#pragma unroll
                for (int j = 0; j < DIM; ++j)
#pragma unroll
                    for (int c = 0; c < MC; ++c) {
                        const float x = nb_own ? (float)A.X[(((int64_t)nb * DIM + j) * m + c0 + c) * 64 + l] : 0.f;
#pragma unroll
                        for (int i = 0; i < DIM; ++i) acc[i][c] = fmaf(kt[i][j], x, acc[i][c]);
                    }
            }
#pragma unroll
            for (int i = 0; i < DIM; ++i)
#pragma unroll
                for (int c = 0; c < MC; ++c)
                    A.Y[(((int64_t)q * DIM + i) * m + c0 + c) * 64 + l] = own ? (double)acc[i][c] : 0.0;
        }
    }
}

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

LowpArgs base(const lat_plan *P, int m, int nch)
{
    LowpArgs A{};
    A.nn = P->nn; A.m = m; A.cap = P->cap; A.ld = P->ld; A.nloc = P->nloc; A.nch = nch;
    A.ngroups = P->ngroups;
    A.chunks_per_group = (int)lat_cdiv(std::max(P->maxunion, 1), nch);
    A.goff = P->goff; A.unode = P->unode; A.unbr = P->unbr; A.umask = P->umask;
    return A;
}

template <int DIM, int NKB, int NLEV>
lat_status launch_bf16_m(const LowpArgs &A, int nwaves, hipStream_t s)
{
    dim3 grid((unsigned)nwaves), block(64);
    switch (A.m) {   // one pass over the right-hand sides (m <= 16)
    case 16: hipLaunchKernelGGL((k_apply_bf16<DIM, NKB, NLEV, 16>), grid, block, 0, s, A); break;
    case 8: hipLaunchKernelGGL((k_apply_bf16<DIM, NKB, NLEV, 8>), grid, block, 0, s, A); break;
    case 4: hipLaunchKernelGGL((k_apply_bf16<DIM, NKB, NLEV, 4>), grid, block, 0, s, A); break;
    case 2: hipLaunchKernelGGL((k_apply_bf16<DIM, NKB, NLEV, 2>), grid, block, 0, s, A); break;
    case 1: hipLaunchKernelGGL((k_apply_bf16<DIM, NKB, NLEV, 1>), grid, block, 0, s, A); break;
    default: return LAT_E_ARG;
    }
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

template <int DIM>
lat_status launch_bf16(const LowpArgs &A, int nkb, int nlev, int nwaves, hipStream_t s)
{
    if (nkb == 1) {
        if (nlev == 1) return launch_bf16_m<DIM, 1, 1>(A, nwaves, s);
        if (nlev == 2) return launch_bf16_m<DIM, 1, 2>(A, nwaves, s);
        return launch_bf16_m<DIM, 1, 3>(A, nwaves, s);
    }
    if (nlev == 1) return launch_bf16_m<DIM, 2, 1>(A, nwaves, s);
    if (nlev == 2) return launch_bf16_m<DIM, 2, 2>(A, nwaves, s);
    return launch_bf16_m<DIM, 2, 3>(A, nwaves, s);
}

template <int DIM, int MC>
lat_status launch_f32_nr(const LowpArgs &A, int nwaves, hipStream_t s)
{
    dim3 grid((unsigned)lat_cdiv(nwaves, 4)), block(256);
    if (A.n_r <= 8) hipLaunchKernelGGL((k_apply_f32<DIM, MC, 8>), grid, block, 0, s, A);
    else if (A.n_r <= 16) hipLaunchKernelGGL((k_apply_f32<DIM, MC, 16>), grid, block, 0, s, A);
    else if (A.n_r <= 32) hipLaunchKernelGGL((k_apply_f32<DIM, MC, 32>), grid, block, 0, s, A);
    else hipLaunchKernelGGL((k_apply_f32<DIM, MC, 64>), grid, block, 0, s, A);
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

template <int DIM>
lat_status launch_f32(const LowpArgs &A, int nwaves, hipStream_t s)
{
    const int m = A.m;
    if (m % 16 == 0) return launch_f32_nr<DIM, 16>(A, nwaves, s);
    if (m % 8 == 0) return launch_f32_nr<DIM, 8>(A, nwaves, s);
    if (m % 4 == 0) return launch_f32_nr<DIM, 4>(A, nwaves, s);
    if (m % 2 == 0) return launch_f32_nr<DIM, 2>(A, nwaves, s);
    return launch_f32_nr<DIM, 1>(A, nwaves, s);
}

}  // namespace

// Internal entry used by lat_apply_combo for prec != LAT_F64.
lat_status lat_apply_lowp(const lat_plan *P, const double *K, int n_r, const double *coef, const double *X, double *Y,
                          int m, int prec, double refine_tol, hipStream_t s)
{
    if (n_r < 1) {                                   // empty basis: Y = 0 on every owned DOF
        const int64_t ny = P->npacked * P->dim * (int64_t)m * 64;
        hipLaunchKernelGGL(k_fill0, dim3((unsigned)lat_cdiv(ny, 256)), dim3(256), 0, s, ny, Y);
        LAT_LAUNCH_CHECK();
        return LAT_OK;
    }
    const int nch = 4;
    LowpArgs A = base(P, m, nch);
    A.n_r = n_r; A.X = X; A.Y = Y;
    const int nwaves = P->ngroups * A.chunks_per_group;
    if (prec == LAT_BF16) {
        if (m != 1 && m != 2 && m != 4 && m != 8 && m != 16) return LAT_E_ARG;
        const int nlev0 = refine_tol >= 0x1p-8 ? 1 : (refine_tol >= 0x1p-16 ? 2 : 3);
        if ((P->dim == 2 && (m == 8 || m == 16) && P->nn >= 3) || (P->dim == 3 && m <= 16))
            return lat_apply_lowp_walk(P, K, n_r, coef, X, Y, m, nlev0, s);
        const int64_t tot = P->nloc * (int64_t)P->EP * 64;
        const int EPL = P->dim == 2 ? Geo<2>::EPL : Geo<3>::EPL, EPP = P->dim == 2 ? Geo<2>::EPP : Geo<3>::EPP;
        hipLaunchKernelGGL(k_slice_stack, dim3((unsigned)lat_cdiv(tot, 256)), dim3(256), 0, s, (int64_t)P->nloc, P->E,
                           EPL, EPP, P->EP, P->cap, n_r, K, P->lp_kslice);
        hipLaunchKernelGGL(k_slice_coef, dim3((unsigned)lat_cdiv(P->ld * 64, 256)), dim3(256), 0, s, P->ld, P->cap,
                           n_r, P->perm, coef, P->lp_cslice);
        LAT_LAUNCH_CHECK();
        A.kslice = P->lp_kslice; A.cslice = P->lp_cslice;
        const int nlev = refine_tol >= 0x1p-8 ? 1 : (refine_tol >= 0x1p-16 ? 2 : 3);
        const int nkb = n_r <= 32 ? 1 : 2;
        return P->dim == 2 ? launch_bf16<2>(A, nkb, nlev, nwaves, s) : launch_bf16<3>(A, nkb, nlev, nwaves, s);
    }
    if ((P->dim == 2 && (m == 8 || m == 16) && P->nn >= 3) || (P->dim == 3 && m <= 16))
        return lat_apply_lowp_walk(P, K, n_r, coef, X, Y, m, 4, s);
    const int64_t nst = P->nloc * (int64_t)P->E * P->cap;
    hipLaunchKernelGGL(k_to_f32_stack, dim3((unsigned)lat_cdiv(nst, 256)), dim3(256), 0, s, nst, K, P->lp_kf32);
    hipLaunchKernelGGL(k_to_f32_coef, dim3((unsigned)lat_cdiv(P->ld, 256), (unsigned)P->cap), dim3(256), 0, s, P->ld,
                       P->cap, n_r, P->perm, coef, P->lp_cf32);
    LAT_LAUNCH_CHECK();
    A.kf32 = P->lp_kf32; A.cf32 = P->lp_cf32;
    return P->dim == 2 ? launch_f32<2>(A, nwaves, s) : launch_f32<3>(A, nwaves, s);
}

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
