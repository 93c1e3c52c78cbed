// Operator applies on the packed, cell-interleaved layout.
//
//   ROM apply (eq. romstiffnessmatrix):  Y_i = M_i (sum_k alpha_ik K_k) M_i X_i
//   plain per-cell apply:                Y_i = M_i K_i M_i X_i
//   adjoint forms:                       G_ik = <Ybar_i, K_k X_i>
//
// One wave = one group of 64 cells (lanes) walking a run of packed nodes.  For a node a and a
// stencil offset o the combination Ktilde_i[a,o] = sum_k alpha_ik K_k[a,o] reads the principal
// stack at a wave-uniform address (scalar loads, shared by the 64 cells) and the lane's own
// alpha_i from registers; the d x d block is then applied to the lane's m right-hand sides.
// X / Y rows are 64 consecutive doubles (one per cell): every vector access is a coalesced
// 512-byte transaction.  Nothing is accumulated across threads: results are reproducible.
#include "lat_internal.h"

namespace {

template <int DIM>
struct Geo {
    static constexpr int NO = DIM == 2 ? 9 : 27;
    static constexpr int E = NO * DIM * DIM;
};

struct ApplyArgs {
    int nn, m, cap, n_r, nch, chunks_per_group;
    int64_t ld;
    const int32_t *goff, *unode, *unbr;
    const uint64_t *umask;
    const double *K;          // principal stack [(a*E+e)*cap + k]  or plain ops [(q*E+e)*64 + l]
    const double *alpha_il;   // [cap][ld]
    const double *X;
    const double *Ybar;       // forms only
    double *Y;                // apply output, or form partials [chunk][ld*cap]
};

__device__ __forceinline__ int offset_node(int a, int o, int nn, int dim)
{
    int ix = a % nn + o % 3 - 1, iy = (a / nn) % nn + (o / 3) % 3 - 1;
    int iz = dim == 3 ? a / (nn * nn) + o / 9 - 1 : 0;
    return ix + nn * (iy + nn * iz);
}

// MODE 0: ROM apply, 1: ROM apply transposed, 2: plain apply
template <int DIM, int MC, int NR, int MODE>
__global__ __launch_bounds__(256) void k_apply(ApplyArgs A)
{
    using G = Geo<DIM>;
    constexpr int E = G::E;
    const int wave = (int)(blockIdx.x * 4 + (threadIdx.x >> 6));
    const int l = threadIdx.x & 63;
    const int g = wave / A.chunks_per_group, ch = wave % A.chunks_per_group;
    if (g >= (int)(A.ld / LAT_WAVE)) return;
    const int q0 = A.goff[g] + ch * A.nch;
    const int q1 = min(A.goff[g + 1], q0 + A.nch);
    if (q0 >= q1) return;
    const int64_t p = (int64_t)g * LAT_WAVE + l;
    const int m = A.m;
    double alpha[MODE == 2 ? 1 : NR];
    if (MODE != 2) {
#pragma unroll
        for (int k = 0; k < NR; ++k) alpha[k] = k < A.n_r ? A.alpha_il[(int64_t)k * A.ld + p] : 0.0;
    }
    for (int q = q0; q < q1; ++q) {
        const int a = A.unode[q];
        const uint64_t msk = A.umask[q];
        for (int c0 = 0; c0 < m; c0 += MC) {
            double acc[DIM][MC];
#pragma unroll
            for (int i = 0; i < DIM; ++i)
#pragma unroll
                for (int c = 0; c < MC; ++c) acc[i][c] = 0.0;
            for (int o = 0; o < G::NO; ++o) {
                const int nb = A.unbr[(int64_t)q * G::NO + o];
                if (nb < 0) continue;
                const bool nb_own = (A.umask[nb] >> l) & 1;    // inputs at DOFs a cell does not own are ignored
                double kt[DIM][DIM];
                if (MODE == 2) {
#pragma unroll
                    for (int i = 0; i < DIM; ++i)
#pragma unroll
                        for (int j = 0; j < DIM; ++j)
                            kt[i][j] = A.K[((int64_t)q * E + (o * DIM + i) * DIM + j) * LAT_WAVE + l];
                } else {
                    const int arow = MODE == 0 ? a : offset_node(a, o, A.nn, DIM);
                    const int orow = MODE == 0 ? o : G::NO - 1 - o;
#pragma unroll
                    for (int i = 0; i < DIM; ++i)
#pragma unroll
                        for (int j = 0; j < DIM; ++j) {
                            // MODE 1 reads the transposed block K[(a+o, j), (a, i)]
                            const int ent = MODE == 0 ? (orow * DIM + i) * DIM + j : (orow * DIM + j) * DIM + i;
                            const double *kp = A.K + ((int64_t)arow * E + ent) * A.cap;
                            double s = 0.0;
#pragma unroll
                            for (int k = 0; k < NR; ++k)
                                if (k < A.n_r) s = fma(alpha[k], kp[k], s);
                            kt[i][j] = s;
                        }
                }
#pragma unroll
                for (int j = 0; j < DIM; ++j)
#pragma unroll
                    for (int c = 0; c < MC; ++c) {
                        const double x = nb_own ? A.X[(((int64_t)nb * DIM + j) * m + c0 + c) * LAT_WAVE + l] : 0.0;
#pragma unroll
                        for (int i = 0; i < DIM; ++i) acc[i][c] = fma(kt[i][j], x, acc[i][c]);
                    }
            }
            const bool own = (msk >> l) & 1;
#pragma unroll
            for (int i = 0; i < DIM; ++i)
#pragma unroll
                for (int c = 0; c < MC; ++c)
                    A.Y[(((int64_t)q * DIM + i) * m + c0 + c) * LAT_WAVE + l] = own ? acc[i][c] : 0.0;
        }
    }
}

// Adjoint forms: partial sums over a run of nodes of G_ik = sum_{a,o,i,j} K_k[a,o,i,j] W_i[a,o,i,j],
// W_i[a,o,i,j] = sum_r Ybar_i[a,i,r] X_i[a+o,j,r].  Output [chunk][lane][cap].
template <int DIM, int NR>
__global__ __launch_bounds__(256) void k_forms(ApplyArgs A)
{
    using G = Geo<DIM>;
    constexpr int E = G::E;
    const int wave = (int)(blockIdx.x * 4 + (threadIdx.x >> 6));
    const int l = threadIdx.x & 63;
    const int g = wave / A.chunks_per_group, ch = wave % A.chunks_per_group;
    if (g >= (int)(A.ld / LAT_WAVE)) return;
    const int q0 = A.goff[g] + ch * A.nch;
    const int q1 = min(A.goff[g + 1], q0 + A.nch);
    const int64_t p = (int64_t)g * LAT_WAVE + l;
    const int m = A.m;
    double gk[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) gk[k] = 0.0;
    for (int q = q0; q < q1; ++q) {
        const int a = A.unode[q];
        if (!((A.umask[q] >> l) & 1)) continue;          // Ybar only counts at owned DOFs
        for (int o = 0; o < G::NO; ++o) {
            const int nb = A.unbr[(int64_t)q * G::NO + o];
            if (nb < 0 || !((A.umask[nb] >> l) & 1)) continue;
#pragma unroll
            for (int i = 0; i < DIM; ++i)
#pragma unroll
                for (int j = 0; j < DIM; ++j) {
                    double w = 0.0;
                    for (int r = 0; r < m; ++r)
                        w = fma(A.Ybar[(((int64_t)q * DIM + i) * m + r) * LAT_WAVE + l],
                                A.X[(((int64_t)nb * DIM + j) * m + r) * LAT_WAVE + l], w);
                    const double *kp = A.K + ((int64_t)a * E + (o * DIM + i) * DIM + j) * A.cap;
#pragma unroll
                    for (int k = 0; k < NR; ++k)
                        if (k < A.n_r) gk[k] = fma(w, kp[k], gk[k]);
                }
        }
    }
#pragma unroll
    for (int k = 0; k < NR; ++k)
        if (k < A.cap) A.Y[((int64_t)ch * A.ld + p) * A.cap + k] = gk[k];
    for (int k = NR; k < A.cap; ++k) A.Y[((int64_t)ch * A.ld + p) * A.cap + k] = 0.0;
}

__global__ void k_alpha_il(int64_t ld, int cap, int n_r, const int32_t *__restrict__ perm,
                           const double *__restrict__ alpha, double *__restrict__ alpha_il)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (p >= ld) return;
    const int c = perm[p];
    alpha_il[(int64_t)k * ld + p] = (c >= 0 && k < n_r) ? alpha[(int64_t)c * cap + k] : 0.0;
}

// forms [ld][cap] (plan order) -> canonical [N_s][cap]
__global__ void k_forms_scatter(int64_t ld, int cap, const int32_t *__restrict__ perm,
                                const double *__restrict__ f, double *__restrict__ out)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ld) return;
    const int c = perm[p];
    if (c < 0) return;
    for (int k = 0; k < cap; ++k) out[(int64_t)c * cap + k] = f[p * cap + k];
}

// direct Lame part: bar_{s_k} = sum_i alpha_ik G_ik (ascending canonical i), zero elsewhere
__global__ void k_direct_lame(int64_t ncells, int cap, int n_r, const int32_t *__restrict__ S,
                              const int32_t *__restrict__ lane, const double *__restrict__ alpha,
                              const double *__restrict__ f, double *__restrict__ bar)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    double v = 0.0;
    for (int k = 0; k < n_r; ++k) {
        if (S[k] != c) continue;
        double s = 0.0;
        for (int64_t i = 0; i < ncells; ++i) s = fma(alpha[i * cap + k], f[(int64_t)lane[i] * cap + k], s);
        v += s;
    }
    bar[c] = v;
}

template <int DIM, int MC, int MODE>
lat_status launch_apply_nr(const ApplyArgs &A, int nwaves, hipStream_t s)
{
    dim3 grid((unsigned)lat_cdiv(nwaves, 4)), block(256);
    const int nr = A.n_r;
    if (MODE == 2 || nr <= 8) hipLaunchKernelGGL((k_apply<DIM, MC, 8, MODE>), grid, block, 0, s, A);
    else if (nr <= 16) hipLaunchKernelGGL((k_apply<DIM, MC, 16, MODE>), grid, block, 0, s, A);
    else if (nr <= 32) hipLaunchKernelGGL((k_apply<DIM, MC, 32, MODE>), grid, block, 0, s, A);
    else hipLaunchKernelGGL((k_apply<DIM, MC, 64, MODE>), grid, block, 0, s, A);
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

template <int DIM, int MODE>
lat_status launch_apply(const ApplyArgs &A, int nwaves, hipStream_t s)
{
    const int m = A.m;
    if (m % 16 == 0) return launch_apply_nr<DIM, 16, MODE>(A, nwaves, s);
    if (m % 8 == 0) return launch_apply_nr<DIM, 8, MODE>(A, nwaves, s);
    if (m % 4 == 0) return launch_apply_nr<DIM, 4, MODE>(A, nwaves, s);
    if (m % 2 == 0) return launch_apply_nr<DIM, 2, MODE>(A, nwaves, s);
    return launch_apply_nr<DIM, 1, MODE>(A, nwaves, s);
}

ApplyArgs base_args(const lat_plan *P, int m, int nch)
{
    ApplyArgs A{};
    A.nn = P->nn; A.m = m; A.cap = P->cap; A.ld = P->ld; A.nch = nch;
    A.chunks_per_group = (int)lat_cdiv(std::max(P->maxunion, 1), nch);
    A.goff = P->goff; A.unode = P->unode; A.unbr = P->unbr; A.umask = P->umask;
    return A;
}

constexpr int APPLY_NODES_PER_WAVE = 4;
constexpr int FORM_NODES_PER_WAVE = 64;

lat_status run_apply(const lat_plan *P, int mode, const double *K, int n_r, const double *alpha, const double *X,
                     double *Y, int m, hipStream_t s)
{
    ApplyArgs A = base_args(P, m, APPLY_NODES_PER_WAVE);
    A.K = K; A.X = X; A.Y = Y; A.n_r = n_r;
    if (mode != 2) {
        hipLaunchKernelGGL(k_alpha_il, dim3((unsigned)lat_cdiv(P->ld, 256), (unsigned)P->cap), dim3(256), 0, s, P->ld,
                           P->cap, n_r, P->perm, alpha, P->alpha_il);
        LAT_LAUNCH_CHECK();
        A.alpha_il = P->alpha_il;
    }
    const int nwaves = P->ngroups * A.chunks_per_group;
    if (P->dim == 2) {
        if (mode == 0) return launch_apply<2, 0>(A, nwaves, s);
        if (mode == 1) return launch_apply<2, 1>(A, nwaves, s);
        return launch_apply<2, 2>(A, nwaves, s);
    }
    if (mode == 0) return launch_apply<3, 0>(A, nwaves, s);
    if (mode == 1) return launch_apply<3, 1>(A, nwaves, s);
    return launch_apply<3, 2>(A, nwaves, s);
}

// G [ld][cap] (plan order) of <Ybar_i, K_k X_i> for a principal stack K.
lat_status run_forms(const lat_plan *P, const double *K, int n_r, const double *X, const double *Ybar, int m,
                     double *out_pl, hipStream_t s)
{
    ApplyArgs A = base_args(P, m, FORM_NODES_PER_WAVE);
    A.K = K; A.X = X; A.Ybar = Ybar; A.Y = P->form_part; A.n_r = n_r;
    if (A.chunks_per_group > P->napc) return LAT_E_SHAPE;
    const int nwaves = P->ngroups * A.chunks_per_group;
    dim3 grid((unsigned)lat_cdiv(nwaves, 4)), block(256);
#define FORMS(D)                                                                                   \
    do {                                                                                           \
        if (n_r <= 8) hipLaunchKernelGGL((k_forms<D, 8>), grid, block, 0, s, A);                   \
        else if (n_r <= 16) hipLaunchKernelGGL((k_forms<D, 16>), grid, block, 0, s, A);            \
        else if (n_r <= 32) hipLaunchKernelGGL((k_forms<D, 32>), grid, block, 0, s, A);            \
        else hipLaunchKernelGGL((k_forms<D, 64>), grid, block, 0, s, A);                           \
    } while (0)
    if (P->dim == 2) FORMS(2);
    else FORMS(3);
#undef FORMS
    LAT_LAUNCH_CHECK();
    return lat_tree_reduce(P->form_part, A.chunks_per_group, P->ld * P->cap, 0, out_pl, P->g_t1, P->g_t2, s);
}

}  // namespace

extern "C" {

lat_status lat_apply_combo(const lat_plan *P, const double *K, int32_t n_r, const double *alpha, const double *X,
                           double *Y, int32_t m, lat_prec prec, int32_t transpose, hipStream_t stream)
{
    if (!P || !K || !alpha || !X || !Y || m < 1) return LAT_E_ARG;
    if (n_r < 0 || n_r > P->cap) return LAT_E_SHAPE;
    if (prec != LAT_F64) return LAT_E_ARG;
    return run_apply(P, transpose ? 1 : 0, K, n_r, alpha, X, Y, m, stream);
}

lat_status lat_apply_plain(const lat_plan *P, const double *plain_ops, const double *X, double *Y, int32_t m,
                           hipStream_t stream)
{
    if (!P || !plain_ops || !X || !Y || m < 1) return LAT_E_ARG;
    return run_apply(P, 2, plain_ops, 0, nullptr, X, Y, m, stream);
}

lat_status lat_apply_combo_adjoint(const lat_plan *P, const double *K, const double *K_mu, const double *K_lam,
                                   const int32_t *S, int32_t n_r, const double *alpha, const double *X,
                                   const double *Ybar, int32_t m, double *Xbar, double *alpha_bar, double *mu_bar,
                                   double *lam_bar, hipStream_t stream)
{
    if (!P || !K || !alpha || !X || !Ybar || m < 1) return LAT_E_ARG;
    if (n_r < 0 || n_r > P->cap) return LAT_E_SHAPE;
    if ((mu_bar && !K_mu) || (lam_bar && !K_lam) || ((mu_bar || lam_bar) && !S)) return LAT_E_ARG;
    lat_status st;
    if (Xbar && (st = run_apply(P, 1, K, n_r, alpha, Ybar, Xbar, m, stream)) != LAT_OK) return st;
    const dim3 lg((unsigned)lat_cdiv(P->ld, 256));
    if (alpha_bar) {
        if ((st = run_forms(P, K, n_r, X, Ybar, m, P->form_out, stream)) != LAT_OK) return st;
        hipLaunchKernelGGL(k_forms_scatter, lg, dim3(256), 0, stream, P->ld, P->cap, P->perm, P->form_out, alpha_bar);
        LAT_LAUNCH_CHECK();
    }
    const double *parts[2] = {K_mu, K_lam};
    double *bars[2] = {mu_bar, lam_bar};
    for (int t = 0; t < 2; ++t) {
        if (!bars[t]) continue;
        if ((st = run_forms(P, parts[t], n_r, X, Ybar, m, P->form_out, stream)) != LAT_OK) return st;
        hipLaunchKernelGGL(k_direct_lame, dim3((unsigned)lat_cdiv(P->ncells, 256)), dim3(256), 0, stream, P->ncells,
                           P->cap, n_r, S, P->lane, alpha, P->form_out, bars[t]);
        LAT_LAUNCH_CHECK();
    }
    return LAT_OK;
}

}  // extern "C"
