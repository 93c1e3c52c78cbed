// Reverse mode of the RB coefficients (least-squares formula of Sec. 3.2.2) with the principal
// set frozen, chained to the per-cell Lame parameters through the snapshots
// t_s = mu_s t^mu_s + lam_s t^lam_s (the tangent is linear in (mu, lam) at fixed u).
//
// With T_S = Z R (the greedy's certified decomposition, Algorithm 1), alpha_i = R^{-1} nu_i beta_i
// and the least-squares residual rho_i = t_i - T_S alpha_i = nu_i Delta_i:
//   q_i = R^{-T} abar_i,   v_i = R^{-1} q_i
//   tbar_i  = T_S v_i = Z q_i                          (cotangent of t_i as data)
//   TbarS   = sum_i ( nu_i Delta_i v_i^T - Z q_i alpha_i^T )  (cotangent of the basis columns)
//   mubar_i += <tbar_i, t^mu_i> = q_i . (Z^T t^mu_i)
//   mubar_{s_k} += sum_i nu_i v_ik <Delta_i, t^mu_{s_k}> - alpha_ik q_i . (Z^T t^mu_{s_k})
// The contractions over the snapshot rows (Z^T T^mu, Delta^T T^mu_S, ...) stream the per-lane
// matrix once with a wave-uniform second operand held as [row][cap].
#include "lat_internal.h"

namespace {

// q_i, v_i per lane (plan order), written to qv[0][p][cap], qv[1][p][cap]
// NR = the plan's cap: every index below is a compile-time constant, so q stays in registers; v
// overwrites q in place (entry k of the backward pass reads only entries above k, already final).
template <int NR>
__global__ __launch_bounds__(256) void k_aa_solve(int64_t ld, int n_r, const int32_t *__restrict__ perm,
                                                  const double *__restrict__ R, const double *__restrict__ abar,
                                                  double *__restrict__ qv)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ld) return;
    const int c = perm[p];
    double q[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) q[k] = 0.0;
    if (c >= 0) {
#pragma unroll
        for (int k = 0; k < NR; ++k) {                  // R^T q = abar (forward)
            if (k < n_r) {
                double acc = abar[(int64_t)c * NR + k];
#pragma unroll
                for (int l = 0; l < k; ++l) acc = fma(-R[l * NR + k], q[l], acc);
                q[k] = acc / R[k * NR + k];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) qv[p * NR + k] = q[k];
    if (c >= 0) {
#pragma unroll
        for (int k = NR - 1; k >= 0; --k) {             // R v = q (backward)
            if (k < n_r) {
                double acc = q[k];
#pragma unroll
                for (int l = k + 1; l < NR; ++l)
                    if (l < n_r) acc = fma(-R[k * NR + l], q[l], acc);
                q[k] = acc / R[k * NR + k];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) qv[(ld + p) * NR + k] = q[k];
}

// U[j][k] = Z[k][j] (k < n_r), 0 beyond
__global__ void k_aa_zt(int64_t nsnap, int cap, int n_r, const double *__restrict__ Z, double *__restrict__ U)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nsnap) return;
    for (int k = 0; k < cap; ++k) U[j * cap + k] = k < n_r ? Z[(int64_t)k * nsnap + j] : 0.0;
}

// U[j][k] = V[j][lane(S[k])] (k < n_r), 0 beyond
__global__ void k_aa_cols(int64_t nsnap, int64_t ld, int cap, int n_r, const int32_t *__restrict__ S,
                          const int32_t *__restrict__ lane, const double *__restrict__ V, double *__restrict__ U)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nsnap) return;
    for (int k = 0; k < cap; ++k) U[j * cap + k] = k < n_r ? V[j * ld + lane[S[k]]] : 0.0;
}

// part[chunk][p][k] = sum_{j in chunk} V[j][p] U[j][k]   (V FP64 or FP32; FP64 arithmetic)
template <int NR, class VT>
__global__ __launch_bounds__(256) void k_aa_contract(int64_t nsnap, int64_t ld, int cap, int rows_per_chunk,
                                                     const VT *__restrict__ V, const double *__restrict__ U,
                                                     double *__restrict__ part)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t b = blockIdx.y;
    if (p >= ld) return;
    const int64_t j0 = b * rows_per_chunk, j1 = j0 + rows_per_chunk < nsnap ? j0 + rows_per_chunk : nsnap;
    double acc[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) acc[k] = 0.0;
    for (int64_t j = j0; j < j1; ++j) {
        const double x = (double)V[j * ld + p];
        const double *u = U + j * cap;
#pragma unroll
        for (int k = 0; k < NR; ++k) acc[k] = fma(x, u[k], acc[k]);
    }
#pragma unroll
    for (int k = 0; k < NR; ++k)
        if (k < cap) part[(b * ld + p) * cap + k] = acc[k];
    for (int k = NR; k < cap; ++k) part[(b * ld + p) * cap + k] = 0.0;
}

// The same contraction on the matrix cores: part[chunk] = V_chunk^T U_chunk, a
// (lanes x rows) x (rows x principals) product, with v_mfma_f64_16x16x4 tiles of 16 lanes x 16
// principals.  A workgroup of 4 waves takes 256 lanes and one chunk of rows; wave w owns lanes
// 64 w .. 64 w + 63 (4 lane tiles) and every principal tile, so V is read once and U once per
// 256 lanes.  Rows go 4 at a time (one MFMA k-step); the sum over a chunk is in row order per
// MFMA, and chunks are combined by the fixed tree.
typedef double aa_v4d __attribute__((ext_vector_type(4)));

template <int NR, class VT>
__global__ __launch_bounds__(256) void k_aa_contract_mfma(int64_t nsnap, int64_t ld, int cap, int rows_per_chunk,
                                                          const VT *__restrict__ V, const double *__restrict__ U,
                                                          double *__restrict__ part)
{
    constexpr int NKT = NR / 16;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int l = threadIdx.x & 63;
    const int64_t pw = (int64_t)blockIdx.x * 256 + 64 * w;           // this wave's first lane
    if (pw >= ld) return;                                             // wave-uniform (ld % 64 == 0)
    const int64_t b = blockIdx.y;
    const int64_t j0 = b * rows_per_chunk, j1 = j0 + rows_per_chunk < nsnap ? j0 + rows_per_chunk : nsnap;
    aa_v4d acc[4][NKT];
#pragma unroll
    for (int pt = 0; pt < 4; ++pt)
#pragma unroll
        for (int kt = 0; kt < NKT; ++kt) acc[pt][kt] = aa_v4d{0.0, 0.0, 0.0, 0.0};
    for (int64_t j = j0; j < j1; j += 4) {
        const int64_t jr = j + (l >> 4);                              // this lane's row of the k-step
        const bool live = jr < j1;
        const int64_t jc = live ? jr : j0;
        double a[4], bv[NKT];
#pragma unroll
        for (int pt = 0; pt < 4; ++pt) {
            const double v = (double)V[jc * ld + pw + 16 * pt + (l & 15)];
            a[pt] = live ? v : 0.0;
        }
#pragma unroll
        for (int kt = 0; kt < NKT; ++kt) {
            const double u = U[jc * cap + 16 * kt + (l & 15)];
            bv[kt] = live ? u : 0.0;
        }
#pragma unroll
        for (int pt = 0; pt < 4; ++pt)
#pragma unroll
            for (int kt = 0; kt < NKT; ++kt) acc[pt][kt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[pt], bv[kt], acc[pt][kt], 0, 0, 0);
    }
    // lane l, reg r -> lane row (l / 16) + 4 r of the tile, principal column l % 16
#pragma unroll
    for (int pt = 0; pt < 4; ++pt)
#pragma unroll
        for (int kt = 0; kt < NKT; ++kt)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                part[(b * ld + pw + 16 * pt + (l >> 4) + 4 * r) * cap + 16 * kt + (l & 15)] = acc[pt][kt][r];
    for (int k = NR; k < cap; ++k)
        part[(b * ld + pw + l) * cap + k] = 0.0;
}

// The same row contraction against NS stacks at once: every V tile is loaded once and feeds the
// NS accumulators (out_t[p][k] = sum_j V[j][p] U_t[j][k]); chunk partials part_t as above.
template <int NR, int NS, class VT>
__global__ __launch_bounds__(256) void k_aa_contract_ns_mfma(int64_t nsnap, int64_t ld, int cap, int rows_per_chunk,
                                                             const VT *__restrict__ V,
                                                             const double *__restrict__ U0,
                                                             const double *__restrict__ U1,
                                                             const double *__restrict__ U2, double *__restrict__ part0,
                                                             double *__restrict__ part1, double *__restrict__ part2)
{
    constexpr int NKT = NR / 16;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int l = threadIdx.x & 63;
    const int64_t pw = (int64_t)blockIdx.x * 256 + 64 * w;
    if (pw >= ld) return;                                             // wave-uniform (ld % 64 == 0)
    const int64_t b = blockIdx.y;
    const int64_t j0 = b * rows_per_chunk, j1 = j0 + rows_per_chunk < nsnap ? j0 + rows_per_chunk : nsnap;
    const double *Us[3] = {U0, U1, U2};
    aa_v4d acc[NS][4][NKT];
#pragma unroll
    for (int t = 0; t < NS; ++t)
#pragma unroll
        for (int pt = 0; pt < 4; ++pt)
#pragma unroll
            for (int kt = 0; kt < NKT; ++kt) acc[t][pt][kt] = aa_v4d{0.0, 0.0, 0.0, 0.0};
    for (int64_t j = j0; j < j1; j += 4) {
        const int64_t jr = j + (l >> 4);
        const bool live = jr < j1;
        const int64_t jc = live ? jr : j0;
        double a[4];
#pragma unroll
        for (int pt = 0; pt < 4; ++pt) {
            const double v = (double)V[jc * ld + pw + 16 * pt + (l & 15)];
            a[pt] = live ? v : 0.0;
        }
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            double bv[NKT];
#pragma unroll
            for (int kt = 0; kt < NKT; ++kt) {
                const double u = Us[t][jc * cap + 16 * kt + (l & 15)];
                bv[kt] = live ? u : 0.0;
            }
#pragma unroll
            for (int pt = 0; pt < 4; ++pt)
#pragma unroll
                for (int kt = 0; kt < NKT; ++kt)
                    acc[t][pt][kt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[pt], bv[kt], acc[t][pt][kt], 0, 0, 0);
        }
    }
    double *parts[3] = {part0, part1, part2};
#pragma unroll
    for (int t = 0; t < NS; ++t) {
#pragma unroll
        for (int pt = 0; pt < 4; ++pt)
#pragma unroll
            for (int kt = 0; kt < NKT; ++kt)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    parts[t][(b * ld + pw + 16 * pt + (l >> 4) + 4 * r) * cap + 16 * kt + (l & 15)] = acc[t][pt][kt][r];
        for (int k = NR; k < cap; ++k) parts[t][(b * ld + pw + l) * cap + k] = 0.0;
    }
}

// per-cell term: bar_c += q_c . A[p_c]   (A = Z^T t^x, plan order [ld][cap])
__global__ void k_aa_cellterm(int64_t ld, int cap, int n_r, const int32_t *__restrict__ perm,
                              const double *__restrict__ qv, const double *__restrict__ Am,
                              const double *__restrict__ Al, double *__restrict__ mbar, double *__restrict__ lbar)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ld) return;
    const int c = perm[p];
    if (c < 0) return;
    double sm = 0.0, sl = 0.0;
    for (int k = 0; k < n_r; ++k) {
        sm = fma(qv[p * cap + k], Am[p * cap + k], sm);
        sl = fma(qv[p * cap + k], Al[p * cap + k], sl);
    }
    if (mbar) mbar[c] += sm;
    if (lbar) lbar[c] += sl;
}

// principal term for slot k: one workgroup per slot, strided over the cells (canonical order),
// fixed-shape tree in LDS (deterministic)
__global__ __launch_bounds__(256) void k_aa_principal(int64_t ncells, int64_t ld, int cap, int n_r,
                                                      const int32_t *__restrict__ S,
                                                      const int32_t *__restrict__ lane, const double *__restrict__ nu,
                                                      const double *__restrict__ alpha, const double *__restrict__ qv,
                                                      const double *__restrict__ Am, const double *__restrict__ Al,
                                                      const double *__restrict__ Bm, const double *__restrict__ Bl,
                                                      double *__restrict__ mbar, double *__restrict__ lbar)
{
    __shared__ double shm[256], shl[256];
    const int k = blockIdx.x;
    const int sk = S[k];
    const int64_t pk = lane[sk];
    double sm = 0.0, sl = 0.0;
    for (int64_t i = threadIdx.x; i < ncells; i += 256) {
        const int64_t pi = lane[i];
        const double vik = qv[(ld + pi) * cap + k];
        double qAm = 0.0, qAl = 0.0;
        for (int l = 0; l < n_r; ++l) {
            qAm = fma(qv[pi * cap + l], Am[pk * cap + l], qAm);
            qAl = fma(qv[pi * cap + l], Al[pk * cap + l], qAl);
        }
        const double aik = alpha[i * cap + k];
        sm += nu[i] * vik * Bm[pi * cap + k] - aik * qAm;
        sl += nu[i] * vik * Bl[pi * cap + k] - aik * qAl;
    }
    shm[threadIdx.x] = sm; shl[threadIdx.x] = sl;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) { shm[threadIdx.x] += shm[threadIdx.x + w]; shl[threadIdx.x] += shl[threadIdx.x + w]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (mbar) mbar[sk] += shm[0];
        if (lbar) lbar[sk] += shl[0];
    }
}

template <class VT>
lat_status contract_t(const lat_plan *P, int n_r, const VT *V, const double *U, double *out, hipStream_t s)
{
    const int rows = P->aa_rows;
    dim3 grid((unsigned)lat_cdiv(P->ld, 256), (unsigned)P->aa_nchunk);
#define CM(NRV) hipLaunchKernelGGL((k_aa_contract_mfma<NRV, VT>), grid, dim3(256), 0, s, P->nsnap, P->ld, P->cap, rows, V, \
                                   U, P->aa_part)
#define CV(NRV) hipLaunchKernelGGL((k_aa_contract<NRV, VT>), grid, dim3(256), 0, s, P->nsnap, P->ld, P->cap, rows, V, U, \
                                   P->aa_part)
    if (n_r > 8 && P->cap >= 16) {
        if (n_r <= 16) CM(16);
        else if (n_r <= 32) CM(32);
        else CM(64);
    } else if (n_r <= 8) CV(8);
    else if (n_r <= 16) CV(16);
    else if (n_r <= 32) CV(32);
    else CV(64);
#undef CM
#undef CV
    LAT_LAUNCH_CHECK();
    return lat_tree_reduce(P->aa_part, P->aa_nchunk, P->ld * P->cap, 0, out, P->g_t1, P->g_t2, s);
}

lat_status contract(const lat_plan *P, int n_r, const double *V, const double *U, double *out, hipStream_t s)
{
    return contract_t<double>(P, n_r, V, U, out, s);
}

template <class VT>
lat_status contract_multi_t(const lat_plan *P, int n_r, const VT *V, const double *const *U, int ns,
                            double *const *part, hipStream_t s)
{
    dim3 grid((unsigned)lat_cdiv(P->ld, 256), (unsigned)P->aa_nchunk);
    const double *u1 = ns > 1 ? U[1] : U[0], *u2 = ns > 2 ? U[2] : U[0];
    double *p1 = ns > 1 ? part[1] : part[0], *p2 = ns > 2 ? part[2] : part[0];
#define CN(NRV, NSV) hipLaunchKernelGGL((k_aa_contract_ns_mfma<NRV, NSV, VT>), grid, dim3(256), 0, s, P->nsnap, P->ld, \
                                        P->cap, P->aa_rows, V, U[0], u1, u2, part[0], p1, p2)
    if (n_r <= 16) {
        if (ns == 1) CN(16, 1); else if (ns == 2) CN(16, 2); else CN(16, 3);
    } else {
        if (ns == 1) CN(32, 1); else if (ns == 2) CN(32, 2); else CN(32, 3);
    }
#undef CN
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

}  // namespace

lat_status lat_contract_rows(const lat_plan *P, int n_r, const double *V, const float *V32, const double *U,
                             double *out, hipStream_t s)
{
    if ((V == nullptr) == (V32 == nullptr)) return LAT_E_ARG;
    return V ? contract_t<double>(P, n_r, V, U, out, s) : contract_t<float>(P, n_r, V32, U, out, s);
}

lat_status lat_contract_rows_multi(const lat_plan *P, int n_r, const double *V, const float *V32,
                                   const double *const *U, int ns, double *const *part, hipStream_t s)
{
    if (ns < 1 || ns > 3 || n_r > 32 || P->cap < 16 || (V == nullptr) == (V32 == nullptr)) return LAT_E_ARG;
    return V ? contract_multi_t<double>(P, n_r, V, U, ns, part, s) : contract_multi_t<float>(P, n_r, V32, U, ns, part, s);
}

extern "C" lat_status lat_alpha_adjoint(const lat_plan *Pp, const double *delta, const double *Z, const double *R,
                                        const double *nu, const int32_t *S, int32_t n_r, const double *alpha,
                                        const double *alpha_bar, const double *snap_mu, const double *snap_lam,
                                        double *mu_bar, double *lam_bar, void *work, size_t work_bytes,
                                        hipStream_t stream)
{
    if (!Pp || !delta || !Z || !R || !nu || !S || !alpha || !alpha_bar || !snap_mu || !snap_lam) return LAT_E_ARG;
    if (n_r < 0 || n_r > Pp->cap) return LAT_E_SHAPE;
    lat_plan Vw;
    lat_status st0 = lat_ws_bind(Pp, LAT_CALL_ALPHA_ADJOINT, work, work_bytes, &Vw);
    if (st0 != LAT_OK) return st0;
    const lat_plan *P = &Vw;
    if (n_r == 0) return LAT_OK;
    const int64_t ld = P->ld, cap = P->cap;
    const dim3 lg((unsigned)lat_cdiv(ld, 256)), sg((unsigned)lat_cdiv(P->nsnap, 256));
    double *Am = P->aa_A, *Al = P->aa_A + ld * cap, *Bm = P->aa_B, *Bl = P->aa_B + ld * cap;
#define SOLVE(NRV) hipLaunchKernelGGL(k_aa_solve<NRV>, lg, dim3(256), 0, stream, ld, n_r, P->perm, R, alpha_bar, P->aa_q)
    switch (cap) {
    case 8: SOLVE(8); break;
    case 16: SOLVE(16); break;
    case 32: SOLVE(32); break;
    case 64: SOLVE(64); break;
    default: return LAT_E_SHAPE;
    }
#undef SOLVE
    LAT_LAUNCH_CHECK();
    lat_status st;
    // A = Z^T T^mu, Z^T T^lam
    hipLaunchKernelGGL(k_aa_zt, sg, dim3(256), 0, stream, P->nsnap, (int)cap, n_r, Z, P->aa_gath);
    LAT_LAUNCH_CHECK();
    if ((st = contract(P, n_r, snap_mu, P->aa_gath, Am, stream)) != LAT_OK) return st;
    if ((st = contract(P, n_r, snap_lam, P->aa_gath, Al, stream)) != LAT_OK) return st;
    // B = Delta^T T^mu_S, Delta^T T^lam_S
    hipLaunchKernelGGL(k_aa_cols, sg, dim3(256), 0, stream, P->nsnap, ld, (int)cap, n_r, S, P->lane, snap_mu, P->aa_gath);
    LAT_LAUNCH_CHECK();
    if (n_r <= 32 && cap >= 16 && P->aa_gath2 && P->wf_part) {
        // one pass over Delta for both (the caller's workspace holds the second gathered set)
        double *gath2 = P->aa_gath2;
        hipLaunchKernelGGL(k_aa_cols, sg, dim3(256), 0, stream, P->nsnap, ld, (int)cap, n_r, S, P->lane, snap_lam,
                           gath2);
        LAT_LAUNCH_CHECK();
        const int64_t ldc = ld * cap;
        const double *U2[2] = {P->aa_gath, gath2};
        double *parts[2] = {P->wf_part, P->wf_part + P->aa_nchunk * ldc};
        if ((st = lat_contract_rows_multi(P, n_r, delta, nullptr, U2, 2, parts, stream)) != LAT_OK) return st;
        if ((st = lat_tree_reduce(parts[0], P->aa_nchunk, ldc, 0, Bm, P->g_t1, P->g_t2, stream)) != LAT_OK) return st;
        if ((st = lat_tree_reduce(parts[1], P->aa_nchunk, ldc, 0, Bl, P->g_t1, P->g_t2, stream)) != LAT_OK) return st;
    } else {
        if ((st = contract(P, n_r, delta, P->aa_gath, Bm, stream)) != LAT_OK) return st;
        hipLaunchKernelGGL(k_aa_cols, sg, dim3(256), 0, stream, P->nsnap, ld, (int)cap, n_r, S, P->lane, snap_lam,
                           P->aa_gath);
        LAT_LAUNCH_CHECK();
        if ((st = contract(P, n_r, delta, P->aa_gath, Bl, stream)) != LAT_OK) return st;
    }
    hipLaunchKernelGGL(k_aa_cellterm, lg, dim3(256), 0, stream, ld, (int)cap, n_r, P->perm, P->aa_q, Am, Al, mu_bar,
                       lam_bar);
    hipLaunchKernelGGL(k_aa_principal, dim3((unsigned)n_r), dim3(256), 0, stream, P->ncells, ld, (int)cap, n_r, S, P->lane,
                       nu, alpha, P->aa_q, Am, Al, Bm, Bl, mu_bar, lam_bar);
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}
