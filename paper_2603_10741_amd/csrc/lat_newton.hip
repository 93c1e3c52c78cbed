// Load-stepped Newton-Raphson on the ROM tangent (Sec. 2.2.5) and the matrix-free tangent solve
// K~ du = -r (eq. linsys with the operator of eq. romstiffnessmatrix) by preconditioned MINRES.
//
// K~ is symmetric (every principal tangent is the Hessian of a stored energy) but need not be
// definite: the tangent of a pre-stressed lattice loses definiteness near buckling, and the
// Newton step is still defined there.  MINRES (Lanczos on K~ with an SPD preconditioner M, the
// tridiagonal factor reduced by Givens rotations) minimises ||b - K~ x||_{M^-1} over the Krylov
// space for any symmetric non-singular K~, so the step equals that of a direct solve up to the
// tolerance.  M^-1 is D^-1 (D = |diag K~|) or D^-1 + P K0^-1 P^T with a coarse space of the
// cell-corner nodes (two levels).
//
// A product K~ z is one per-cell apply with a single right-hand side on the packed layout (the
// combined stencils formed once, or the ROM apply forming them), followed by an owner-ordered
// assembly onto the global nodes that also forms the partial sums of z.K~z.  The Lanczos and
// rotation scalars live in a small device control block and are finalised by single-workgroup
// kernels, so the host only reads the control block every `check` iterations.  Every reduction
// has a fixed order (per-block LDS trees or shuffle trees, then the block partials in index
// order): a solve is reproducible bit for bit on a given plan.
#include <chrono>
#include <cmath>
#include <mutex>

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "lat_internal.h"

namespace {

constexpr int NB = 256;   // threads per workgroup of the vector kernels

struct NGrid {
    int dim, nel, nn, nloc;
    int ncell[3];
    int64_t gs[3];
};

NGrid make_ngrid(const lat_plan *P)
{
    NGrid g;
    g.dim = P->dim; g.nel = P->nel; g.nn = P->nn; g.nloc = P->nloc;
    for (int ax = 0; ax < 3; ++ax) {
        g.ncell[ax] = P->ncell[ax];
        g.gs[ax] = ax < P->dim ? (int64_t)P->ncell[ax] * P->nel + 1 : 1;
    }
    return g;
}

// Tables of the packed layout, for locating a cell's local node in a packed vector.
struct PackMap {
    const int32_t *lane;   // [N_s] canonical cell -> plan lane
    const int32_t *uidx;   // [ngroups][nloc] packed index within the group, or -1
    const int32_t *goff;   // [ngroups+1] packed-node offset of each group
};

// Calls f(cell, a) for every cell owning global node G (background id bg), in ascending
// canonical cell id: the order in which the library's assembly sums.
template <class F>
__device__ __forceinline__ void for_owners(const NGrid &g, int64_t bg, const int32_t *__restrict__ l2g, F &&f)
{
    int gc[3] = {0, 0, 0};
    for (int ax = 0; ax < g.dim; ++ax) { gc[ax] = (int)(bg % g.gs[ax]); bg /= g.gs[ax]; }
    for (int kz = (g.dim == 3 ? 1 : 0); kz >= 0; --kz)
        for (int ky = 1; ky >= 0; --ky)
            for (int kx = 1; kx >= 0; --kx) {
                const int kk[3] = {kx, ky, kz};
                int cc[3] = {0, 0, 0}, ia[3] = {0, 0, 0};
                bool ok = true;
                for (int ax = 0; ax < g.dim; ++ax) {
                    const int base = gc[ax] / g.nel;
                    const int c = kk[ax] ? base - 1 : base;
                    const int loc = gc[ax] - c * g.nel;
                    ok = ok && c >= 0 && c < g.ncell[ax] && loc >= 0 && loc <= g.nel;
                    cc[ax] = c; ia[ax] = loc;
                }
                if (!ok) continue;
                const int64_t cell = cc[0] + (int64_t)g.ncell[0] * (cc[1] + (int64_t)g.ncell[1] * cc[2]);
                const int a = ia[0] + g.nn * (ia[1] + g.nn * ia[2]);
                if (l2g[cell * g.nloc + a] < 0) continue;
                f(cell, a);
            }
}

// Packed index of component 0 of (cell, local node a) with one right-hand side; component i is
// at + i * 64.  -1 if the node is not in the union of the cell's group (never for an owned node).
__device__ __forceinline__ int64_t packed_slot(const PackMap &pm, int nloc, int dim, int64_t cell, int a)
{
    const int p = pm.lane[cell];
    const int g = p / LAT_WAVE, l = p % LAT_WAVE;
    const int qi = pm.uidx[(int64_t)g * nloc + a];
    if (qi < 0) return -1;
    const int64_t q = (int64_t)pm.goff[g] + qi;
    return q * dim * LAT_WAVE + l;
}

// Packed node q and lane l of (cell, local node a); false if the node is not in the union of the
// cell's group (never for an owned node).
__device__ __forceinline__ bool packed_ql(const PackMap &pm, int nloc, int64_t cell, int a, int64_t *q, int *l)
{
    const int p = pm.lane[cell];
    const int g = p / LAT_WAVE;
    const int qi = pm.uidx[(int64_t)g * nloc + a];
    *q = (int64_t)pm.goff[g] + qi;
    *l = p % LAT_WAVE;
    return qi >= 0;
}

constexpr int MAXOWN = 8;   // cells owning a node: at most 2^d

// Packed slots (component 0) of the owners of every global node in ascending cell id, -1 padded:
// own[G * 2^d + k].  Built once per solve so that the per-iteration assembly and scatter read
// 4 or 8 indices instead of re-deriving the owners from the node's background coordinates.
__global__ void __launch_bounds__(NB) k_owner_table(NGrid g, PackMap pm, int64_t nglobal,
                                                    const int64_t *__restrict__ g2bg, const int32_t *__restrict__ l2g,
                                                    int32_t *__restrict__ own)
{
    const int64_t G = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (G >= nglobal) return;
    const int no = 1 << g.dim;
    int k = 0;
    for_owners(g, g2bg[G], l2g, [&](int64_t cell, int a) {
        const int64_t s0 = packed_slot(pm, g.nloc, g.dim, cell, a);
        if (s0 >= 0 && k < no) own[G * no + k++] = (int32_t)s0;
    });
    for (; k < no; ++k) own[G * no + k] = -1;
}

__device__ __forceinline__ double block_sum(double v, double *sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = NB / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// sum of part[0..n) in a fixed order by one workgroup
__device__ __forceinline__ double sum_parts(const double *__restrict__ part, int n, double *sh)
{
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += NB) acc += part[i];
    return block_sum(acc, sh);
}

// Scalars of the MINRES recurrence (ESW-style indexing: step j uses gamma_j, gamma_{j-1},
// c_j, c_{j-1}, s_j, s_{j-1}; eta tracks +-||r_j||_{D^-1}).
struct MrCtl {
    double gam, gam_prev, c, c_prev, s, s_prev, eta, eta0, tol_eta;
    double cv1, cv2;                 // Lanczos coefficients delta_j / gamma_j, gamma_j / gamma_{j-1}
    double a1, a2, a3, cx, inv_gam;  // step coefficients for the direction and solution updates
    int32_t done, last, status, iters;
};

// |diag K~| on the free components, inverted (0 on prescribed ones, 1 where the diagonal vanishes)
__global__ void __launch_bounds__(NB) k_jacobi(NGrid g, int64_t nglobal, const int64_t *__restrict__ g2bg,
                                               const int32_t *__restrict__ l2g, const double *__restrict__ K,
                                               const double *__restrict__ alpha, int cap, int n_r, int E,
                                               const uint8_t *__restrict__ fixed, double *__restrict__ dinv)
{
    const int64_t G = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (G >= nglobal) return;
    const int d = g.dim;
    const int oc = d == 2 ? 4 : 13;   // offset index of (0, 0[, 0])
    double dg[3] = {0.0, 0.0, 0.0};
    for_owners(g, g2bg[G], l2g, [&](int64_t cell, int a) {
        for (int i = 0; i < d; ++i) {
            const double *kr = K + ((int64_t)a * E + (oc * d + i) * d + i) * cap;
            const double *ar = alpha + cell * cap;
            double s = 0.0;
            for (int k = 0; k < n_r; ++k) s = fma(ar[k], kr[k], s);
            dg[i] += s;
        }
    });
    for (int i = 0; i < d; ++i) {
        const int64_t j = G * d + i;
        const double a = fabs(dg[i]);
        dinv[j] = fixed[j] ? 0.0 : (a > 0.0 ? 1.0 / a : 1.0);
    }
}

// The same from per-cell stencils in the packed layout of lat_apply_plain
__global__ void __launch_bounds__(NB) k_jacobi_ops(NGrid g, PackMap pm, int64_t nglobal,
                                                   const int64_t *__restrict__ g2bg,
                                                   const int32_t *__restrict__ l2g, const double *__restrict__ ops,
                                                   int E, const uint8_t *__restrict__ fixed, double *__restrict__ dinv)
{
    const int64_t G = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (G >= nglobal) return;
    const int d = g.dim;
    const int oc = d == 2 ? 4 : 13;
    double dg[3] = {0.0, 0.0, 0.0};
    for_owners(g, g2bg[G], l2g, [&](int64_t cell, int a) {
        int64_t q;
        int l;
        if (!packed_ql(pm, g.nloc, cell, a, &q, &l)) return;
        for (int i = 0; i < d; ++i) dg[i] += ops[(q * E + (oc * d + i) * d + i) * LAT_WAVE + l];
    });
    for (int i = 0; i < d; ++i) {
        const int64_t j = G * d + i;
        const double a = fabs(dg[i]);
        dinv[j] = fixed[j] ? 0.0 : (a > 0.0 ? 1.0 / a : 1.0);
    }
}

// v1 = b (free), z1 = D^-1 v1; x = w0 = w1 = v0 = 0; partial <z1, v1>
__global__ void __launch_bounds__(NB) k_mr_init(int64_t n, const uint8_t *__restrict__ fixed,
                                                const double *__restrict__ dinv, const double *__restrict__ b,
                                                double *__restrict__ x, double *__restrict__ v0,
                                                double *__restrict__ v1, double *__restrict__ z1,
                                                double *__restrict__ w0, double *__restrict__ w1,
                                                double *__restrict__ part)
{
    __shared__ double sh[NB];
    double zv = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * NB + threadIdx.x; j < n; j += (int64_t)gridDim.x * NB) {
        const double bj = fixed[j] ? 0.0 : b[j];
        const double zj = dinv[j] * bj;
        x[j] = 0.0; v0[j] = 0.0; w0[j] = 0.0; w1[j] = 0.0;
        v1[j] = bj; z1[j] = zj;
        zv = fma(zj, bj, zv);
    }
    zv = block_sum(zv, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = zv;
}

__global__ void k_ctl_clear(MrCtl *ctl)
{
    ctl->done = 0;
    ctl->last = 0;
}

__global__ void __launch_bounds__(NB) k_mr_init_fin(int nb, const double *__restrict__ part, double tol, MrCtl *ctl)
{
    __shared__ double sh[NB];
    const double zv = sum_parts(part, nb, sh);
    if (threadIdx.x == 0) {
        const double g1 = sqrt(fmax(zv, 0.0));
        ctl->gam = g1; ctl->gam_prev = 1.0;
        ctl->c = 1.0; ctl->c_prev = 1.0; ctl->s = 0.0; ctl->s_prev = 0.0;
        ctl->eta = g1; ctl->eta0 = g1; ctl->tol_eta = tol * g1;
        ctl->inv_gam = g1 > 0.0 ? 1.0 / g1 : 0.0;
        ctl->iters = 0; ctl->status = LAT_OK; ctl->last = 0;
        ctl->done = !(g1 > 0.0);   // b = 0 on the free components: x = 0
    }
}

// z <- z / gamma (the first normalised Lanczos vector), scattered into the packed apply input
template <int D>
__global__ void __launch_bounds__(NB) k_mr_scale(int64_t nglobal, const int32_t *__restrict__ own,
                                                 double *__restrict__ z, double *__restrict__ ppk,
                                                 const MrCtl *__restrict__ ctl)
{
    if (ctl->done) return;
    const int64_t G = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (G >= nglobal) return;
    const double ig = ctl->inv_gam;
    double zv[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        zv[i] = z[G * D + i] * ig;
        z[G * D + i] = zv[i];
    }
#pragma unroll
    for (int k = 0; k < (1 << D); ++k) {
        const int32_t s0 = own[G * (1 << D) + k];
        if (s0 >= 0)
#pragma unroll
            for (int i = 0; i < D; ++i) ppk[s0 + i * LAT_WAVE] = zv[i];
    }
}

// y = assembled, masked K~ z from the packed apply output (owners summed in ascending cell id);
// partial <y, z>
template <int D>
__global__ void __launch_bounds__(NB) k_mr_ap(int64_t nglobal, const int32_t *__restrict__ own,
                                              const uint8_t *__restrict__ fixed, const double *__restrict__ ypk,
                                              const double *__restrict__ z, double *__restrict__ y,
                                              double *__restrict__ part, const MrCtl *__restrict__ ctl)
{
    __shared__ double sh[NB];
    if (ctl->done) return;
    const int64_t G = (int64_t)blockIdx.x * NB + threadIdx.x;
    double dot = 0.0;
    if (G < nglobal) {
        double acc[D];
#pragma unroll
        for (int i = 0; i < D; ++i) acc[i] = 0.0;
#pragma unroll
        for (int k = 0; k < (1 << D); ++k) {
            const int32_t s0 = own[G * (1 << D) + k];
            if (s0 >= 0)
#pragma unroll
                for (int i = 0; i < D; ++i) acc[i] += ypk[s0 + i * LAT_WAVE];
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const int64_t j = G * D + i;
            const double v = fixed[j] ? 0.0 : acc[i];
            y[j] = v;
            dot = fma(z[j], v, dot);
        }
    }
    dot = block_sum(dot, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = dot;
}

// delta_j = <K~ z_j, z_j> and the Lanczos coefficients; ends the solve one step after the
// rotation kernel has flagged convergence (the solution update of that step has been applied)
__global__ void __launch_bounds__(NB) k_mr_delta(int nb, const double *__restrict__ part, MrCtl *ctl)
{
    __shared__ double sh[NB];
    if (ctl->done) return;
    if (ctl->last) {
        if (threadIdx.x == 0) ctl->done = 1;
        return;
    }
    const double delta = sum_parts(part, nb, sh);
    if (threadIdx.x == 0) {
        ctl->a1 = delta;   // kept until the rotation kernel of this step
        ctl->cv1 = delta / ctl->gam;
        ctl->cv2 = ctl->gam / ctl->gam_prev;
    }
}

// v_{j+1} = y - cv1 v_j - cv2 v_{j-1} (written over v_{j-1}); z_{j+1} = D^-1 v_{j+1};
// partial <z_{j+1}, v_{j+1}>
__global__ void __launch_bounds__(NB) k_mr_v(int64_t n, const double *__restrict__ y, const double *__restrict__ vj,
                                             double *__restrict__ vprev_next, const double *__restrict__ dinv,
                                             double *__restrict__ znext, double *__restrict__ part,
                                             const MrCtl *__restrict__ ctl)
{
    __shared__ double sh[NB];
    if (ctl->done) return;
    const double c1 = ctl->cv1, c2 = ctl->cv2;
    double zv = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * NB + threadIdx.x; j < n; j += (int64_t)gridDim.x * NB) {
        const double v = fma(-c2, vprev_next[j], fma(-c1, vj[j], y[j]));
        const double z = dinv[j] * v;
        vprev_next[j] = v;
        znext[j] = z;
        zv = fma(z, v, zv);
    }
    zv = block_sum(zv, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = zv;
}

// gamma_{j+1}, the Givens rotation of step j, the step coefficients and the residual estimate
__global__ void __launch_bounds__(NB) k_mr_rot(int nb, const double *__restrict__ part, int it, MrCtl *ctl)
{
    __shared__ double sh[NB];
    if (ctl->done) return;
    const double zv = sum_parts(part, nb, sh);
    if (threadIdx.x == 0) {
        const double delta = ctl->a1;
        const double gn = sqrt(fmax(zv, 0.0));
        const double g = ctl->gam;
        const double a0 = ctl->c * delta - ctl->c_prev * ctl->s * g;
        const double a1 = sqrt(a0 * a0 + gn * gn);
        const double a2 = ctl->s * delta + ctl->c_prev * ctl->c * g;
        const double a3 = ctl->s_prev * g;
        if (!(a1 > 0.0) || !isfinite(a1)) {   // K~ singular on the Krylov space (or non-finite)
            ctl->status = LAT_E_SINGULAR;
            ctl->done = 1;
        } else {
            const double cn = a0 / a1, sn = gn / a1;
            ctl->a1 = a1; ctl->a2 = a2; ctl->a3 = a3;
            ctl->cx = cn * ctl->eta;
            ctl->inv_gam = gn > 0.0 ? 1.0 / gn : 0.0;
            ctl->eta = -sn * ctl->eta;
            ctl->c_prev = ctl->c; ctl->c = cn;
            ctl->s_prev = ctl->s; ctl->s = sn;
            ctl->gam_prev = g; ctl->gam = gn;
            ctl->iters = it + 1;
            if (fabs(ctl->eta) <= ctl->tol_eta || !(gn > 0.0)) ctl->last = 1;
        }
    }
}

// End of step j, per node: w_{j+1} = (z_j - a3 w_{j-1} - a2 w_j) / a1 (written over w_{j-1}),
// x += cx w_{j+1}; then the next Lanczos vector z_{j+1} <- z_{j+1} / gamma_{j+1}, scattered into
// the packed input of the next product.
template <int D>
__global__ void __launch_bounds__(NB) k_mr_x(int64_t nglobal, const int32_t *__restrict__ own,
                                             const double *__restrict__ zj, const double *__restrict__ wj,
                                             double *__restrict__ wprev_next, double *__restrict__ x,
                                             double *__restrict__ znext, double *__restrict__ ppk,
                                             const MrCtl *__restrict__ ctl)
{
    if (ctl->done) return;
    const int64_t G = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (G >= nglobal) return;
    const double ia1 = 1.0 / ctl->a1, a2 = ctl->a2, a3 = ctl->a3, cx = ctl->cx, ig = ctl->inv_gam;
    double zv[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const int64_t j = G * D + i;
        const double w = (zj[j] - a3 * wprev_next[j] - a2 * wj[j]) * ia1;
        wprev_next[j] = w;
        x[j] = fma(cx, w, x[j]);
        zv[i] = znext[j] * ig;
        znext[j] = zv[i];
    }
#pragma unroll
    for (int k = 0; k < (1 << D); ++k) {
        const int32_t s0 = own[G * (1 << D) + k];
        if (s0 >= 0)
#pragma unroll
            for (int i = 0; i < D; ++i) ppk[s0 + i * LAT_WAVE] = zv[i];
    }
}

// ---------------------------------------------------------------------- two-level preconditioner
// Coarse space: the cell-corner nodes of the lattice (the primal corners of the FETI-DP coarse
// problem, Sec. 3.3) with Q1 interpolation on the grid of corners, P.  The preconditioner is
// M^-1 = D^-1 + P K0^-1 P^T with the Galerkin coarse operator K0 = P^T K~ P (prescribed
// components removed from P's rows), factorised once per tangent solve.  Coarse node
// C = cx + (C_x+1)(cy + (C_y+1) cz); coarse DOF C d + i.

// Per fine node: the enclosing coarse cell's low corner and the local grid coordinates.
__global__ void __launch_bounds__(NB) k_coarse_tables(NGrid g, int64_t nglobal, const int64_t *__restrict__ g2bg,
                                                      int32_t *__restrict__ cbase, uint32_t *__restrict__ cloc)
{
    const int64_t G = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (G >= nglobal) return;
    int64_t bg = g2bg[G];
    int32_t base = 0, stride = 1;
    uint32_t loc = 0;
    for (int ax = 0; ax < g.dim; ++ax) {
        const int gc = (int)(bg % g.gs[ax]);
        bg /= g.gs[ax];
        const int b = min(gc / g.nel, g.ncell[ax] - 1);
        base += b * stride;
        stride *= g.ncell[ax] + 1;
        loc |= (uint32_t)(gc - b * g.nel) << (10 * ax);
    }
    cbase[G] = base;
    cloc[G] = loc;
}

// prim[c][a] = 1 when cell c is the lowest-id owner of its active local node a (each fine node
// enters the restriction once)
__global__ void __launch_bounds__(NB) k_coarse_prim(NGrid g, int64_t ncells, const int64_t *__restrict__ g2bg,
                                                    const int32_t *__restrict__ l2g, uint8_t *__restrict__ prim)
{
    const int64_t t = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (t >= ncells * g.nloc) return;
    const int64_t c = t / g.nloc;
    const int32_t G = l2g[t];
    uint8_t v = 0;
    if (G >= 0) {
        int64_t first = -1;
        for_owners(g, g2bg[G], l2g, [&](int64_t cell, int) {
            if (first < 0) first = cell;
        });
        v = first == c;
    }
    prim[t] = v;
}

// Q1 corner function k of a cell at its local node with grid coordinates (ix, iy, iz)
__device__ __forceinline__ double corner_phi(int k, int dim, int nel, const int (&ic)[3])
{
    const double h = 1.0 / nel;
    double f = 1.0;
    for (int ax = 0; ax < dim; ++ax) {
        const double t = ic[ax] * h;
        f *= ((k >> ax) & 1) ? t : 1.0 - t;
    }
    return f;
}

// All 2^D corner functions at once from the per-axis coordinates t = ic / n
template <int D>
__device__ __forceinline__ void corner_phis(double h, const int (&ic)[3], double (&phi)[1 << D])
{
    double t[3], u[3];
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
        t[ax] = ic[ax] * h;
        u[ax] = 1.0 - t[ax];
    }
#pragma unroll
    for (int k = 0; k < (1 << D); ++k) {
        double f = (k & 1) ? t[0] : u[0];
#pragma unroll
        for (int ax = 1; ax < D; ++ax) f *= ((k >> ax) & 1) ? t[ax] : u[ax];
        phi[k] = f;
    }
}

// The cells' corner functions on the packed layout, m = 2^d d right-hand sides (r = k d + i:
// corner k, component i), zero on prescribed components and on DOFs a cell does not own.
__global__ void __launch_bounds__(NB) k_coarse_X(NGrid g, int64_t npk, const int32_t *__restrict__ qgroup,
                                                 const int32_t *__restrict__ unode, const int32_t *__restrict__ perm,
                                                 const int32_t *__restrict__ l2g, const uint8_t *__restrict__ fixed,
                                                 double *__restrict__ X)
{
    const int64_t t = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (t >= npk * LAT_WAVE) return;
    const int d = g.dim, m = (1 << d) * d;
    const int l = (int)(t % LAT_WAVE);
    const int64_t q = t / LAT_WAVE;
    const int cell = perm[(int64_t)qgroup[q] * LAT_WAVE + l];
    const int a = unode[q];
    const int32_t G = cell >= 0 ? l2g[(int64_t)cell * g.nloc + a] : -1;
    const int ic[3] = {a % g.nn, (a / g.nn) % g.nn, a / (g.nn * g.nn)};
    for (int j = 0; j < d; ++j) {
        const bool free_j = G >= 0 && !fixed[(int64_t)G * d + j];
        for (int r = 0; r < m; ++r) {
            const double v = (free_j && r % d == j) ? corner_phi(r / d, d, g.nel, ic) : 0.0;
            X[((q * d + j) * m + r) * LAT_WAVE + l] = v;
        }
    }
}

// Per-cell coarse matrices K0s[c][r1][r2] = sum over the cell's DOFs of X[., r1] (K~ X)[., r2]
template <int MM>
__global__ void __launch_bounds__(LAT_WAVE) k_coarse_cellmat(int dim, const int32_t *__restrict__ goff,
                                                             const int32_t *__restrict__ perm,
                                                             const double *__restrict__ X,
                                                             const double *__restrict__ Y, double *__restrict__ K0s)
{
    const int g = blockIdx.x, r1 = blockIdx.y, l = threadIdx.x;
    const int cell = perm[(int64_t)g * LAT_WAVE + l];
    double acc[MM];
#pragma unroll
    for (int r = 0; r < MM; ++r) acc[r] = 0.0;
    for (int64_t q = goff[g]; q < goff[g + 1]; ++q)
        for (int j = 0; j < dim; ++j) {
            const int64_t row = (q * dim + j) * MM;
            const double x1 = X[(row + r1) * LAT_WAVE + l];
            if (x1 != 0.0)
#pragma unroll
                for (int r = 0; r < MM; ++r) acc[r] = fma(x1, Y[(row + r) * LAT_WAVE + l], acc[r]);
        }
    if (cell >= 0)
#pragma unroll
        for (int r = 0; r < MM; ++r) K0s[((int64_t)cell * MM + r1) * MM + r] = acc[r];
}

// Dense K0 (row-major, pre-zeroed), one thread per coarse row: the cells around the row's corner
// in ascending id; a row with no free fine support gets a unit diagonal.
__global__ void __launch_bounds__(NB) k_coarse_assemble(NGrid g, int ncd, const double *__restrict__ K0s,
                                                        double *__restrict__ K0)
{
    const int R = blockIdx.x * NB + threadIdx.x;
    if (R >= ncd) return;
    const int d = g.dim, nco = 1 << d, m = nco * d;
    const int C1 = R / d, i1 = R % d;
    const int cs0 = g.ncell[0] + 1, cs1 = g.ncell[1] + 1;
    const int c1[3] = {C1 % cs0, (C1 / cs0) % cs1, C1 / (cs0 * cs1)};
    double *row = K0 + (int64_t)R * ncd;
    for (int kz = (d == 3 ? 1 : 0); kz >= 0; --kz)
        for (int ky = 1; ky >= 0; --ky)
            for (int kx = 1; kx >= 0; --kx) {
                const int kk[3] = {kx, ky, kz};
                int cc[3] = {0, 0, 0}, bits = 0;
                bool ok = true;
                for (int ax = 0; ax < d; ++ax) {
                    cc[ax] = c1[ax] - kk[ax];
                    ok = ok && cc[ax] >= 0 && cc[ax] < g.ncell[ax];
                    bits |= kk[ax] << ax;
                }
                if (!ok) continue;
                const int64_t cell = cc[0] + (int64_t)g.ncell[0] * (cc[1] + (int64_t)g.ncell[1] * cc[2]);
                const double *ks = K0s + ((int64_t)cell * m + bits * d + i1) * m;
                for (int k2 = 0; k2 < nco; ++k2) {
                    const int C2 = (cc[0] + (k2 & 1)) +
                                   cs0 * ((cc[1] + ((k2 >> 1) & 1)) + cs1 * (cc[2] + ((k2 >> 2) & 1)));
                    for (int i2 = 0; i2 < d; ++i2) row[C2 * d + i2] += ks[k2 * d + i2];
                }
            }
    if (row[R] == 0.0) row[R] = 1.0;
}

// Copy the lower triangle (column-major, as factorised) of a symmetric matrix into the upper one.
__global__ void __launch_bounds__(NB) k_symmetrize(int64_t n, double *__restrict__ A)
{
    const int64_t t = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (t >= n * n) return;
    const int64_t i = t / n, j = t % n;
    if (i > j) A[j + i * n] = A[i + j * n];
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, LAT_WAVE);
    return v;
}

// Restriction, one workgroup per cell: cpart[c][k][i] = sum over the cell's primary nodes of
// phi_k v_i (per-thread sums, wave sums by a fixed shuffle tree, then the 4 waves in order)
template <int D>
__global__ void __launch_bounds__(NB) k_cr_restrict(int nel, int nn, int64_t ncells, const int32_t *__restrict__ l2g,
                                                    const uint8_t *__restrict__ prim, const double *__restrict__ v,
                                                    double *__restrict__ cpart, const MrCtl *__restrict__ ctl)
{
    constexpr int NCO = 1 << D, NA = NCO * D, NWV = NB / LAT_WAVE;
    __shared__ double sh[NWV][NA];
    if (ctl->done) return;
    const int64_t c = blockIdx.x;
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nloc = D == 2 ? nn * nn : nn * nn * nn;
    const double h = 1.0 / nel;
    double acc[NCO][D];
#pragma unroll
    for (int k = 0; k < NCO; ++k)
#pragma unroll
        for (int i = 0; i < D; ++i) acc[k][i] = 0.0;
    for (int a = threadIdx.x; a < nloc; a += NB) {
        if (!prim[c * nloc + a]) continue;
        const int64_t G = l2g[c * nloc + a];
        const int ic[3] = {a % nn, (a / nn) % nn, a / (nn * nn)};
        double phi[NCO];
        corner_phis<D>(h, ic, phi);
        double vi[D];
#pragma unroll
        for (int i = 0; i < D; ++i) vi[i] = v[G * D + i];
#pragma unroll
        for (int k = 0; k < NCO; ++k)
#pragma unroll
            for (int i = 0; i < D; ++i) acc[k][i] = fma(phi[k], vi[i], acc[k][i]);
    }
#pragma unroll
    for (int k = 0; k < NCO; ++k)
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const double s = wave_sum(acc[k][i]);
            if (l == 0) sh[wv][k * D + i] = s;
        }
    __syncthreads();
    if (threadIdx.x < NA) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NWV; ++w) s += sh[w][threadIdx.x];
        cpart[c * NA + threadIdx.x] = s;
    }
}

// rc[C d + i] = sum over the cells around corner C (ascending id) of their partials
__global__ void __launch_bounds__(NB) k_cr_sum(NGrid g, int ncd, const double *__restrict__ cpart,
                                               double *__restrict__ rc, const MrCtl *__restrict__ ctl)
{
    if (ctl->done) return;
    const int R = blockIdx.x * NB + threadIdx.x;
    if (R >= ncd) return;
    const int d = g.dim, nco = 1 << d;
    const int C = R / d, i = R % d;
    const int cs0 = g.ncell[0] + 1, cs1 = g.ncell[1] + 1;
    const int c1[3] = {C % cs0, (C / cs0) % cs1, C / (cs0 * cs1)};
    double acc = 0.0;
    for (int kz = (d == 3 ? 1 : 0); kz >= 0; --kz)
        for (int ky = 1; ky >= 0; --ky)
            for (int kx = 1; kx >= 0; --kx) {
                const int kk[3] = {kx, ky, kz};
                int cc[3] = {0, 0, 0}, bits = 0;
                bool ok = true;
                for (int ax = 0; ax < d; ++ax) {
                    cc[ax] = c1[ax] - kk[ax];
                    ok = ok && cc[ax] >= 0 && cc[ax] < g.ncell[ax];
                    bits |= kk[ax] << ax;
                }
                if (!ok) continue;
                const int64_t cell = cc[0] + (int64_t)g.ncell[0] * (cc[1] + (int64_t)g.ncell[1] * cc[2]);
                acc += cpart[(cell * nco + bits) * d + i];
            }
    rc[R] = acc;
}

// ec = K0^-1 rc, one workgroup per row (four independent partial sums per thread, wave sums by a
// fixed shuffle tree, the waves combined in order)
__global__ void __launch_bounds__(NB) k_cr_gemv(int ncd, const double *__restrict__ A, const double *__restrict__ x,
                                                double *__restrict__ y, const MrCtl *__restrict__ ctl)
{
    constexpr int NWV = NB / LAT_WAVE;
    __shared__ double sh[NWV];
    if (ctl->done) return;
    const int64_t R = blockIdx.x;
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const double *row = A + R * ncd;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int c = threadIdx.x;
    for (; c + 3 * NB < ncd; c += 4 * NB) {
        a0 = fma(row[c], x[c], a0);
        a1 = fma(row[c + NB], x[c + NB], a1);
        a2 = fma(row[c + 2 * NB], x[c + 2 * NB], a2);
        a3 = fma(row[c + 3 * NB], x[c + 3 * NB], a3);
    }
    for (; c < ncd; c += NB) a0 = fma(row[c], x[c], a0);
    const double s = wave_sum((a0 + a1) + (a2 + a3));
    if (l == 0) sh[wv] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < NWV; ++w) t += sh[w];
        y[R] = t;
    }
}

// z += P ec on the free components; partial <z, v>
template <int D>
__global__ void __launch_bounds__(NB) k_cr_prolong(int nel, int cs0, int cs1, int64_t nglobal,
                                                   const int32_t *__restrict__ cbase, const uint32_t *__restrict__ cloc,
                                                   const uint8_t *__restrict__ fixed, const double *__restrict__ ec,
                                                   const double *__restrict__ v, double *__restrict__ z,
                                                   double *__restrict__ part, const MrCtl *__restrict__ ctl)
{
    __shared__ double sh[NB];
    if (ctl->done) return;
    const int64_t G = (int64_t)blockIdx.x * NB + threadIdx.x;
    double dot = 0.0;
    if (G < nglobal) {
        const int32_t base = cbase[G];
        const uint32_t lc = cloc[G];
        const int ic[3] = {(int)(lc & 1023u), (int)((lc >> 10) & 1023u), (int)((lc >> 20) & 1023u)};
        double add[D], phi[1 << D];
        corner_phis<D>(1.0 / nel, ic, phi);
#pragma unroll
        for (int i = 0; i < D; ++i) add[i] = 0.0;
#pragma unroll
        for (int k = 0; k < (1 << D); ++k) {
            const double f = phi[k];
            const int C = base + (k & 1) + cs0 * (((k >> 1) & 1) + cs1 * ((k >> 2) & 1));
#pragma unroll
            for (int i = 0; i < D; ++i) add[i] = fma(f, ec[(int64_t)C * D + i], add[i]);
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const int64_t j = G * D + i;
            const double zj = fixed[j] ? z[j] : z[j] + add[i];
            z[j] = zj;
            dot = fma(zj, v[j], dot);
        }
    }
    dot = block_sum(dot, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = dot;
}

// Combined stencil of every cell, K~_s = sum_k alpha_sk K_k (eq. romstiffnessmatrix), in the
// packed per-cell operator layout of lat_apply_plain: ops[(q E + e) 64 + l] for packed node q of
// group g and lane l (cell perm[64 g + l]; padding lanes get 0).  One thread per (q, l) keeps its
// cell's coefficients in registers and walks the E stencil entries of node unode[q]; the
// principal entries it reads are the same for the 64 lanes of a wave.
template <int NR>
__global__ void __launch_bounds__(NB) k_combine_ops(int64_t npk, int E, int cap, int n_r,
                                                    const int32_t *__restrict__ qgroup,
                                                    const int32_t *__restrict__ unode, const int32_t *__restrict__ perm,
                                                    const double *__restrict__ K, const double *__restrict__ alpha,
                                                    double *__restrict__ ops)
{
    const int64_t t = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (t >= npk * LAT_WAVE) return;
    const int l = (int)(t % LAT_WAVE);
    const int64_t q = t / LAT_WAVE;
    const int cell = perm[(int64_t)qgroup[q] * LAT_WAVE + l];
    double al[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) al[k] = (cell >= 0 && k < n_r) ? alpha[(int64_t)cell * cap + k] : 0.0;
    const double *kq = K + (int64_t)unode[q] * E * cap;
    double *oq = ops + q * E * LAT_WAVE + l;
    for (int e = 0; e < E; ++e) {
        const double *kr = kq + (int64_t)e * cap;
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < NR; ++k)
            if (k < n_r) s = fma(al[k], kr[k], s);
        oq[(int64_t)e * LAT_WAVE] = s;
    }
}

lat_status combine_ops(const lat_plan *P, const double *K, int n_r, const double *alpha, double *ops, hipStream_t s)
{
    if (P->npacked == 0) return LAT_OK;
    const int64_t nt = P->npacked * LAT_WAVE;
    const dim3 grid((unsigned)lat_cdiv(nt, NB));
    const int32_t *qgroup = P->goff + P->ngroups + 1;
#define CO(NRV) hipLaunchKernelGGL((k_combine_ops<NRV>), grid, dim3(NB), 0, s, (int64_t)P->npacked, P->E, P->cap, n_r, \
                                   qgroup, P->unode, P->perm, K, alpha, ops)
    if (n_r <= 8) CO(8);
    else if (n_r <= 16) CO(16);
    else if (n_r <= 32) CO(32);
    else CO(64);
#undef CO
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

__global__ void __launch_bounds__(NB) k_fill(int64_t n, double v, double *__restrict__ y)
{
    for (int64_t j = (int64_t)blockIdx.x * NB + threadIdx.x; j < n; j += (int64_t)gridDim.x * NB) y[j] = v;
}

// y = a + s b
__global__ void __launch_bounds__(NB) k_axpy(int64_t n, const double *__restrict__ a, double s,
                                             const double *__restrict__ b, double *__restrict__ y)
{
    for (int64_t j = (int64_t)blockIdx.x * NB + threadIdx.x; j < n; j += (int64_t)gridDim.x * NB)
        y[j] = fma(s, b[j], a[j]);
}

// r = (assembled f_int - lf f_ext) on free components, 0 on prescribed ones; partial r.r
__global__ void __launch_bounds__(NB) k_residual(int64_t n, const double *__restrict__ fasm,
                                                 const double *__restrict__ fext, double lf,
                                                 const uint8_t *__restrict__ fixed, double *__restrict__ r,
                                                 double *__restrict__ part)
{
    __shared__ double sh[NB];
    double rr = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * NB + threadIdx.x; j < n; j += (int64_t)gridDim.x * NB) {
        double v = fasm[j];
        if (fext) v = fma(-lf, fext[j], v);
        if (fixed[j]) v = 0.0;
        r[j] = v;
        rr = fma(v, v, rr);
    }
    rr = block_sum(rr, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = rr;
}

__global__ void __launch_bounds__(NB) k_sum_fin(int nb, const double *__restrict__ part, double *__restrict__ out)
{
    __shared__ double sh[NB];
    const double s = sum_parts(part, nb, sh);
    if (threadIdx.x == 0) out[0] = s;
}

// x = -y
__global__ void __launch_bounds__(NB) k_neg(int64_t n, const double *__restrict__ y, double *__restrict__ x)
{
    for (int64_t j = (int64_t)blockIdx.x * NB + threadIdx.x; j < n; j += (int64_t)gridDim.x * NB) x[j] = -y[j];
}

unsigned vec_blocks(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(lat_cdiv(n, NB), 2048)); }

// Device buffers of one call, released on every return path.
struct Arena {
    std::vector<void *> ptrs;
    std::vector<hipEvent_t> evs;
    ~Arena()
    {
        for (hipEvent_t e : evs) (void)hipEventDestroy(e);
        for (void *p : ptrs) (void)hipFree(p);
    }
    lat_status event(hipEvent_t *e)
    {
        if (hipEventCreate(e) != hipSuccess) return LAT_E_DEVICE;
        evs.push_back(*e);
        return LAT_OK;
    }
    template <class T>
    lat_status get(T **p, int64_t n)
    {
        if (hipMalloc((void **)p, (size_t)std::max<int64_t>(n, 1) * sizeof(T)) != hipSuccess) {
            *p = nullptr;
            return LAT_E_NOMEM;
        }
        ptrs.push_back((void *)*p);
        return LAT_OK;
    }
};

#define NCHK(expr) do { lat_status st_ = (expr); if (st_ != LAT_OK) return st_; } while (0)

struct MrWork {
    double *v[2] = {nullptr, nullptr}, *z[2] = {nullptr, nullptr}, *w[2] = {nullptr, nullptr};
    double *y = nullptr, *dinv = nullptr, *ppk = nullptr, *ypk = nullptr, *part = nullptr;
    double *ops = nullptr;       // combined per-cell stencils (packed), when materialised
    int32_t *own = nullptr;      // [n_global][2^d] packed slots of each node's owners
    MrCtl *ctl = nullptr;
    static constexpr int NT = 64;            // products timed per solve (the first NT)
    hipEvent_t tev[2 * NT] = {};
    unsigned nbn = 1, nbv = 1;   // blocks over nodes, over components
    // two-level preconditioner (coarse space of cell corners)
    bool coarse = false;         // requested and within the size limit
    bool coarse_on = false;      // the current solve's coarse operator factorised
    int ncd = 0, mc = 0;         // coarse DOFs, corner functions per cell
    int32_t *cbase = nullptr;
    uint32_t *cloc = nullptr;
    uint8_t *prim = nullptr;
    double *Xc = nullptr, *Yc = nullptr, *K0s = nullptr, *K0 = nullptr, *cpart = nullptr, *rc = nullptr, *ec = nullptr;
    int32_t *info = nullptr;
};

constexpr int COARSE_MAX = 16384;   // coarse DOFs held as a dense factor

// One rocBLAS handle per device for the coarse factorisation (created on first use, kept).
rocblas_handle solver_handle()
{
    static std::mutex mu;
    static rocblas_handle h[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(mu);
    if (!h[dev] && rocblas_create_handle(&h[dev]) != rocblas_status_success) h[dev] = nullptr;
    return h[dev];
}

lat_status mr_alloc(const lat_plan *P, Arena &ar, MrWork &w, bool materialize, hipStream_t s, bool coarse = false,
                    const uint8_t *fixed = nullptr)
{
    const int64_t n = P->nglobal * P->dim;
    const int64_t npk = std::max<int64_t>(P->npacked, 1) * P->dim * LAT_WAVE;
    w.nbn = (unsigned)std::max<int64_t>(1, lat_cdiv(P->nglobal, NB));
    w.nbv = vec_blocks(n);
    for (auto &p : w.v) NCHK(ar.get(&p, n));
    for (auto &p : w.z) NCHK(ar.get(&p, n));
    for (auto &p : w.w) NCHK(ar.get(&p, n));
    NCHK(ar.get(&w.y, n)); NCHK(ar.get(&w.dinv, n));
    NCHK(ar.get(&w.ppk, npk)); NCHK(ar.get(&w.ypk, npk));
    NCHK(ar.get(&w.part, (int64_t)std::max(w.nbn, w.nbv))); NCHK(ar.get(&w.ctl, 1));
    for (auto &e : w.tev) NCHK(ar.event(&e));
    if (npk >= INT32_MAX) return LAT_E_SHAPE;   // packed slots are held as int32
    NCHK(ar.get(&w.own, P->nglobal << P->dim));
    hipLaunchKernelGGL(k_owner_table, dim3(w.nbn), dim3(NB), 0, s, make_ngrid(P), PackMap{P->lane, P->uidx, P->goff},
                       P->nglobal, P->g2bg, P->l2g, w.own);
    LAT_LAUNCH_CHECK();
    if (materialize) NCHK(ar.get(&w.ops, std::max<int64_t>(P->npacked, 1) * P->E * LAT_WAVE));
    int64_t nc = 1;
    for (int ax = 0; ax < P->dim; ++ax) nc *= P->ncell[ax] + 1;
    w.ncd = (int)std::min<int64_t>(nc * P->dim, INT32_MAX);
    w.mc = (1 << P->dim) * P->dim;
    w.coarse = coarse && fixed && nc * P->dim <= COARSE_MAX && P->npacked > 0;
    if (w.coarse) {
        const NGrid g = make_ngrid(P);
        const int64_t npm = P->npacked * P->dim * w.mc * LAT_WAVE;
        NCHK(ar.get(&w.cbase, P->nglobal)); NCHK(ar.get(&w.cloc, P->nglobal));
        NCHK(ar.get(&w.prim, P->ncells * P->nloc));
        NCHK(ar.get(&w.Xc, npm)); NCHK(ar.get(&w.Yc, npm));
        NCHK(ar.get(&w.K0s, P->ncells * w.mc * w.mc));
        NCHK(ar.get(&w.K0, (int64_t)w.ncd * w.ncd));
        NCHK(ar.get(&w.cpart, P->ncells * (1 << P->dim) * P->dim));
        NCHK(ar.get(&w.rc, w.ncd)); NCHK(ar.get(&w.ec, w.ncd)); NCHK(ar.get(&w.info, 1));
        hipLaunchKernelGGL(k_coarse_tables, dim3(w.nbn), dim3(NB), 0, s, g, P->nglobal, P->g2bg, w.cbase, w.cloc);
        hipLaunchKernelGGL(k_coarse_prim, dim3((unsigned)lat_cdiv(P->ncells * P->nloc, NB)), dim3(NB), 0, s, g,
                           P->ncells, P->g2bg, P->l2g, w.prim);
        hipLaunchKernelGGL(k_coarse_X, dim3((unsigned)lat_cdiv(P->npacked * LAT_WAVE, NB)), dim3(NB), 0, s, g,
                           (int64_t)P->npacked, P->goff + P->ngroups + 1, P->unode, P->perm, P->l2g, fixed, w.Xc);
        LAT_LAUNCH_CHECK();
    }
    return LAT_OK;
}

// K0 = P^T K~ P (dense, row-major) of the operator given by `ops` or (K, alpha): one apply of the
// cells' corner functions, per-cell m x m products, owner-ordered assembly.
lat_status coarse_operator(const lat_plan *P, MrWork &w, const double *K, int n_r, const double *alpha,
                           const double *ops, hipStream_t s)
{
    if (ops) NCHK(lat_apply_plain(P, ops, w.Xc, w.Yc, w.mc, s));
    else NCHK(lat_apply_combo(P, K, n_r, alpha, w.Xc, w.Yc, w.mc, LAT_F64, 0.0, 0, nullptr, nullptr, 0, s));
    const dim3 cg((unsigned)P->ngroups, (unsigned)w.mc);
    if (w.mc == 8)
        hipLaunchKernelGGL(k_coarse_cellmat<8>, cg, dim3(LAT_WAVE), 0, s, P->dim, P->goff, P->perm, w.Xc, w.Yc, w.K0s);
    else
        hipLaunchKernelGGL(k_coarse_cellmat<24>, cg, dim3(LAT_WAVE), 0, s, P->dim, P->goff, P->perm, w.Xc, w.Yc,
                           w.K0s);
    const int64_t nn2 = (int64_t)w.ncd * w.ncd;
    hipLaunchKernelGGL(k_fill, dim3(vec_blocks(nn2)), dim3(NB), 0, s, nn2, 0.0, w.K0);
    hipLaunchKernelGGL(k_coarse_assemble, dim3((unsigned)lat_cdiv(w.ncd, NB)), dim3(NB), 0, s, make_ngrid(P), w.ncd,
                       w.K0s, w.K0);
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

// Form and invert K0 for this solve; a coarse operator that is not positive definite (an
// indefinite tangent) leaves the solve with the diagonal preconditioner alone.
lat_status coarse_setup(const lat_plan *P, MrWork &w, const double *K, int n_r, const double *alpha,
                        const double *ops, hipStream_t s)
{
    w.coarse_on = false;
    if (!w.coarse) return LAT_OK;
    NCHK(coarse_operator(P, w, K, n_r, alpha, ops, s));
    rocblas_handle h = solver_handle();
    if (!h || rocblas_set_stream(h, s) != rocblas_status_success) return LAT_E_DEVICE;
    int32_t info = 0;
    if (rocsolver_dpotrf(h, rocblas_fill_lower, w.ncd, w.K0, w.ncd, w.info) != rocblas_status_success)
        return LAT_E_DEVICE;
    LAT_HIP(hipMemcpyAsync(&info, w.info, sizeof(info), hipMemcpyDeviceToHost, s));
    LAT_HIP(hipStreamSynchronize(s));
    if (info != 0) return LAT_OK;
    if (rocsolver_dpotri(h, rocblas_fill_lower, w.ncd, w.K0, w.ncd, w.info) != rocblas_status_success)
        return LAT_E_DEVICE;
    LAT_HIP(hipMemcpyAsync(&info, w.info, sizeof(info), hipMemcpyDeviceToHost, s));
    LAT_HIP(hipStreamSynchronize(s));
    if (info != 0) return LAT_OK;
    const int64_t nn2 = (int64_t)w.ncd * w.ncd;
    hipLaunchKernelGGL(k_symmetrize, dim3((unsigned)lat_cdiv(nn2, NB)), dim3(NB), 0, s, (int64_t)w.ncd, w.K0);
    LAT_LAUNCH_CHECK();
    w.coarse_on = true;
    return LAT_OK;
}

// z += P K0^-1 P^T v; partial <z, v> over the node blocks into w.part
lat_status coarse_apply(const lat_plan *P, MrWork &w, const uint8_t *fixed, const double *v, double *z, hipStream_t s)
{
    const NGrid g = make_ngrid(P);
    const unsigned nbc = (unsigned)P->ncells;
    const unsigned nbr = (unsigned)lat_cdiv(w.ncd, NB);
    const unsigned nbg = (unsigned)w.ncd;
    const int cs0 = P->ncell[0] + 1, cs1 = P->ncell[1] + 1;
    if (P->dim == 2)
        hipLaunchKernelGGL(k_cr_restrict<2>, dim3(nbc), dim3(NB), 0, s, P->nel, P->nn, P->ncells, P->l2g, w.prim, v,
                           w.cpart, w.ctl);
    else
        hipLaunchKernelGGL(k_cr_restrict<3>, dim3(nbc), dim3(NB), 0, s, P->nel, P->nn, P->ncells, P->l2g, w.prim, v,
                           w.cpart, w.ctl);
    hipLaunchKernelGGL(k_cr_sum, dim3(nbr), dim3(NB), 0, s, g, w.ncd, w.cpart, w.rc, w.ctl);
    hipLaunchKernelGGL(k_cr_gemv, dim3(nbg), dim3(NB), 0, s, w.ncd, w.K0, w.rc, w.ec, w.ctl);
    if (P->dim == 2)
        hipLaunchKernelGGL(k_cr_prolong<2>, dim3(w.nbn), dim3(NB), 0, s, P->nel, cs0, cs1, P->nglobal, w.cbase, w.cloc,
                           fixed, w.ec, v, z, w.part, w.ctl);
    else
        hipLaunchKernelGGL(k_cr_prolong<3>, dim3(w.nbn), dim3(NB), 0, s, P->nel, cs0, cs1, P->nglobal, w.cbase, w.cloc,
                           fixed, w.ec, v, z, w.part, w.ctl);
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

// Preconditioned MINRES from x = 0 on the operator given by per-cell stencils `ops` (packed
// layout of lat_apply_plain), or, when ops is null, by the principal stack K and coefficients
// alpha (every product a ROM apply).  Synchronises the stream.  *relres = ||r||_{D^-1} /
// ||b||_{D^-1} as tracked by the rotations.
lat_status mr_run(const lat_plan *P, MrWork &w, const double *K, int n_r, const double *alpha, const double *ops,
                  const uint8_t *fixed, const double *b, double *x, double tol, int maxit, int check, int *iters,
                  double *relres, hipStream_t s, double *t_product_us = nullptr)
{
    const NGrid g = make_ngrid(P);
    const PackMap pm{P->lane, P->uidx, P->goff};
    const int64_t n = P->nglobal * P->dim;
    const int64_t npk = std::max<int64_t>(P->npacked, 1) * P->dim * LAT_WAVE;
    hipLaunchKernelGGL(k_fill, dim3(vec_blocks(npk)), dim3(NB), 0, s, npk, 0.0, w.ppk);
    if (ops)
        hipLaunchKernelGGL(k_jacobi_ops, dim3(w.nbn), dim3(NB), 0, s, g, pm, P->nglobal, P->g2bg, P->l2g, ops, P->E,
                           fixed, w.dinv);
    else
        hipLaunchKernelGGL(k_jacobi, dim3(w.nbn), dim3(NB), 0, s, g, P->nglobal, P->g2bg, P->l2g, K, alpha, P->cap,
                           n_r, P->E, fixed, w.dinv);
    NCHK(coarse_setup(P, w, K, n_r, alpha, ops, s));
    const bool two = w.coarse_on;
    const int nbz = two ? (int)w.nbn : (int)w.nbv;   // partial sums of <z, v>: node or component blocks
    // v_0 = v[0], v_1 = v[1], z_1 = z[1], w_0 = w[0], w_1 = w[1]
    hipLaunchKernelGGL(k_mr_init, dim3(w.nbv), dim3(NB), 0, s, n, fixed, w.dinv, b, x, w.v[0], w.v[1], w.z[1], w.w[0],
                       w.w[1], w.part);
    if (two) {
        // the control block is not yet initialised: clear its stop flag for the coarse kernels
        hipLaunchKernelGGL(k_ctl_clear, dim3(1), dim3(1), 0, s, w.ctl);
        NCHK(coarse_apply(P, w, fixed, w.v[1], w.z[1], s));
    }
    hipLaunchKernelGGL(k_mr_init_fin, dim3(1), dim3(NB), 0, s, nbz, w.part, tol, w.ctl);
    // z_1 / gamma_1 into the packed input of the first product
    if (P->dim == 2)
        hipLaunchKernelGGL(k_mr_scale<2>, dim3(w.nbn), dim3(NB), 0, s, P->nglobal, w.own, w.z[1], w.ppk, w.ctl);
    else
        hipLaunchKernelGGL(k_mr_scale<3>, dim3(w.nbn), dim3(NB), 0, s, P->nglobal, w.own, w.z[1], w.ppk, w.ctl);
    LAT_LAUNCH_CHECK();
    MrCtl h{};
    int it = 0, ntimed = 0;
    // products timed: from the 9th of a batch on (the host has run ahead by then, so the events
    // bracket the kernel and not a launch gap), at most NT per solve
    const int tskip = std::min(8, check - 1);
    for (;;) {
        LAT_HIP(hipMemcpyAsync(&h, w.ctl, sizeof(MrCtl), hipMemcpyDeviceToHost, s));
        LAT_HIP(hipStreamSynchronize(s));
        if (h.done || h.last || it >= maxit) break;
        const int nb = std::min(check, maxit - it);
        for (int k = 0; k < nb; ++k, ++it) {
            const int j = it + 1;                      // Lanczos step
            double *vj = w.v[j % 2], *vjm1 = w.v[(j + 1) % 2];   // v_{j+1} is written over v_{j-1}
            double *zj = w.z[j % 2], *zj1 = w.z[(j + 1) % 2];
            double *wj = w.w[j % 2], *wjm1 = w.w[(j + 1) % 2];   // w_{j+1} is written over w_{j-1}
            const bool timed = t_product_us && k >= tskip && ntimed < MrWork::NT;
            if (timed) LAT_HIP(hipEventRecord(w.tev[2 * ntimed], s));
            if (ops) NCHK(lat_apply_plain(P, ops, w.ppk, w.ypk, 1, s));
            else NCHK(lat_apply_combo(P, K, n_r, alpha, w.ppk, w.ypk, 1, LAT_F64, 0.0, 0, nullptr, nullptr, 0, s));
            if (timed) LAT_HIP(hipEventRecord(w.tev[2 * ntimed++ + 1], s));
            if (P->dim == 2)
                hipLaunchKernelGGL(k_mr_ap<2>, dim3(w.nbn), dim3(NB), 0, s, P->nglobal, w.own, fixed, w.ypk, zj, w.y,
                                   w.part, w.ctl);
            else
                hipLaunchKernelGGL(k_mr_ap<3>, dim3(w.nbn), dim3(NB), 0, s, P->nglobal, w.own, fixed, w.ypk, zj, w.y,
                                   w.part, w.ctl);
            hipLaunchKernelGGL(k_mr_delta, dim3(1), dim3(NB), 0, s, (int)w.nbn, w.part, w.ctl);
            hipLaunchKernelGGL(k_mr_v, dim3(w.nbv), dim3(NB), 0, s, n, w.y, vj, vjm1, w.dinv, zj1, w.part, w.ctl);
            if (two) NCHK(coarse_apply(P, w, fixed, vjm1, zj1, s));   // v_{j+1} now lives in vjm1
            hipLaunchKernelGGL(k_mr_rot, dim3(1), dim3(NB), 0, s, nbz, w.part, it, w.ctl);
            if (P->dim == 2)
                hipLaunchKernelGGL(k_mr_x<2>, dim3(w.nbn), dim3(NB), 0, s, P->nglobal, w.own, zj, wj, wjm1, x, zj1,
                                   w.ppk, w.ctl);
            else
                hipLaunchKernelGGL(k_mr_x<3>, dim3(w.nbn), dim3(NB), 0, s, P->nglobal, w.own, zj, wj, wjm1, x, zj1,
                                   w.ppk, w.ctl);
            LAT_LAUNCH_CHECK();
        }
    }
    if (t_product_us) {   // mean duration of the timed products (events on the launch stream)
        const int nt = ntimed;
        double tot = 0.0;
        for (int k = 0; k < nt; ++k) {
            float ms = 0.0f;
            LAT_HIP(hipEventElapsedTime(&ms, w.tev[2 * k], w.tev[2 * k + 1]));
            tot += ms;
        }
        *t_product_us = nt > 0 ? 1e3 * tot / nt : 0.0;
    }
    if (iters) *iters = h.iters;
    if (relres) *relres = h.eta0 > 0.0 ? std::fabs(h.eta) / h.eta0 : 0.0;
    if (h.status == LAT_E_SINGULAR) return LAT_E_SINGULAR;
    return (h.done || h.last) ? LAT_OK : LAT_E_NOCONV;
}

double ms_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

lat_status lat_combine_ops(const lat_plan *P, const double *K, int n_r, const double *alpha, double *ops, hipStream_t s)
{
    return combine_ops(P, K, n_r, alpha, ops, s);
}

extern "C" {

lat_status lat_rom_solve(const lat_plan *P, const double *K, int32_t n_r, const double *alpha, const uint8_t *fixed,
                         const double *b, double *x, double tol, int32_t maxit, int32_t check, int32_t materialize,
                         int32_t precond, int32_t *iters, double *relres, int32_t *coarse_used, hipStream_t stream)
{
    if (coarse_used) *coarse_used = 0;
    if (!P || !K || !alpha || !fixed || !b || !x) return LAT_E_ARG;
    if (n_r < 0 || n_r > P->cap || !(tol > 0.0) || maxit < 0 || check < 1 || (precond != 0 && precond != 1))
        return LAT_E_ARG;
    if (P->nglobal == 0) {
        if (iters) *iters = 0;
        if (relres) *relres = 0.0;
        return LAT_OK;
    }
    Arena ar;
    MrWork w;
    NCHK(mr_alloc(P, ar, w, materialize != 0, stream, precond == 1, fixed));
    int it = 0;
    double rr = 0.0;
    if (w.ops) NCHK(combine_ops(P, K, n_r, alpha, w.ops, stream));
    const lat_status st = mr_run(P, w, K, n_r, alpha, w.ops, fixed, b, x, tol, maxit, check, &it, &rr, stream);
    if (iters) *iters = it;
    if (relres) *relres = rr;
    if (coarse_used) *coarse_used = w.coarse_on;
    LAT_HIP(hipStreamSynchronize(stream));
    return st;
}

lat_status lat_coarse_operator(const lat_plan *P, const double *K, int32_t n_r, const double *alpha,
                               const uint8_t *fixed, int32_t materialize, double *K0, hipStream_t stream)
{
    if (!P || !K || !alpha || !fixed || !K0) return LAT_E_ARG;
    if (n_r < 0 || n_r > P->cap) return LAT_E_ARG;
    if (P->nglobal == 0 || P->npacked == 0) return LAT_E_SHAPE;
    Arena ar;
    MrWork w;
    NCHK(mr_alloc(P, ar, w, materialize != 0, stream, true, fixed));
    if (!w.coarse) return LAT_E_SHAPE;
    if (w.ops) NCHK(combine_ops(P, K, n_r, alpha, w.ops, stream));
    NCHK(coarse_operator(P, w, K, n_r, alpha, w.ops, stream));
    LAT_HIP(hipMemcpyAsync(K0, w.K0, (size_t)w.ncd * w.ncd * sizeof(double), hipMemcpyDeviceToDevice, stream));
    LAT_HIP(hipStreamSynchronize(stream));
    return LAT_OK;
}

lat_status lat_newton_solve(const lat_plan *P, const double *mu, const double *lam, const uint8_t *fixed,
                            const double *ubar, const double *f_ext, const lat_newton_opts *o, double *u,
                            lat_newton_record *records, int32_t max_records, int32_t *n_records, hipStream_t s)
{
    if (n_records) *n_records = 0;
    if (!P || !mu || !lam || !fixed || !ubar || !o || !u) return LAT_E_ARG;
    if (o->n_inc < 1 || o->max_newton < 1 || o->max_backtrack < 0 || o->cap < 1 || o->cap > P->cap ||
        o->cg_maxit < 1 || o->cg_check < 1 || (o->matvec != 0 && o->matvec != 1) ||
        (o->tangent != 0 && o->tangent != 1) || o->precond < 0 || o->precond > 2 ||
        (o->precond == 2 && o->tangent == 1) || o->feti_n_delta < 0 ||
        (o->snap_rule != LAT_RULE_FULL && o->snap_rule != LAT_RULE_REDUCED && o->snap_rule != LAT_RULE_MATERIAL &&
         o->snap_rule != LAT_RULE_SAMPLED) ||
        !(o->rb_tol > 0.0) || !(o->newton_tol > 0.0) || !(o->armijo_beta > 0.0 && o->armijo_beta < 1.0) ||
        !(o->armijo_c >= 0.0 && o->armijo_c < 1.0) || !(o->cg_tol > 0.0) || max_records < 0 ||
        (max_records > 0 && !records))
        return LAT_E_ARG;
    if (P->nglobal == 0) return LAT_OK;
    const int d = P->dim;
    const int64_t n = P->nglobal * d;
    Arena ar;
    MrWork w;
    const bool full = o->tangent == 1;   // each cell's own tangent (the standard method)
    NCHK(mr_alloc(P, ar, w, full || o->matvec == 0, s, o->precond >= 1, fixed));
    const bool feti = o->precond == 2;
    double *u_try, *du, *rhs, *r, *r_try, *fasm, *f_cil, *snap, *K, *alpha, *R, *scal, *beta = nullptr, *nu = nullptr;
    int32_t *S, *nr_d, *st_d, *gst_d;
    NCHK(ar.get(&u_try, n)); NCHK(ar.get(&du, n)); NCHK(ar.get(&rhs, n)); NCHK(ar.get(&r, n));
    NCHK(ar.get(&r_try, n)); NCHK(ar.get(&fasm, n));
    NCHK(ar.get(&f_cil, (int64_t)P->nloc * d * P->ld));
    NCHK(ar.get(&snap, P->nsnap * P->ld));
    NCHK(ar.get(&K, (int64_t)P->nloc * P->E * P->cap));
    NCHK(ar.get(&alpha, P->ncells * P->cap));
    NCHK(ar.get(&R, (int64_t)P->cap * P->cap));
    NCHK(ar.get(&scal, 2));
    if (feti) { NCHK(ar.get(&beta, P->ncells * P->cap)); NCHK(ar.get(&nu, P->ncells)); }
    NCHK(ar.get(&S, P->cap)); NCHK(ar.get(&nr_d, 1)); NCHK(ar.get(&st_d, 2)); NCHK(ar.get(&gst_d, 2));
    const unsigned nbv = w.nbv;
    const lat_rule rule = (lat_rule)o->snap_rule;

    // residual (and snapshots) at `at` into `res`; returns the HOST norm (inf if not admissible)
    auto evaluate = [&](const double *at, double lf, double *res, double *norm, int32_t *code) -> lat_status {
        NCHK(lat_status_reset(st_d, s));
        NCHK(lat_residual_tangent(P, at, mu, lam, rule, f_cil, nullptr, full ? nullptr : snap, full ? w.ops : nullptr,
                                  st_d, nullptr, 0, s));
        NCHK(lat_assemble(P, f_cil, d, fasm, s));
        hipLaunchKernelGGL(k_residual, dim3(nbv), dim3(NB), 0, s, n, fasm, f_ext, lf, fixed, res, w.part);
        hipLaunchKernelGGL(k_sum_fin, dim3(1), dim3(NB), 0, s, (int)nbv, w.part, scal);
        LAT_LAUNCH_CHECK();
        double rr = 0.0;
        int32_t hst[2] = {0, 0};
        LAT_HIP(hipMemcpyAsync(&rr, scal, sizeof(double), hipMemcpyDeviceToHost, s));
        LAT_HIP(hipMemcpyAsync(hst, st_d, sizeof(hst), hipMemcpyDeviceToHost, s));
        LAT_HIP(hipStreamSynchronize(s));
        *code = hst[0];
        *norm = (hst[0] == LAT_OK && std::isfinite(rr)) ? std::sqrt(rr) : INFINITY;
        return LAT_OK;
    };

    int nrec = 0;
    lat_status result = LAT_OK;
    for (int t = 1; t <= o->n_inc && result == LAT_OK; ++t) {
        const double lf = (double)t / o->n_inc;
        auto t0 = std::chrono::steady_clock::now();
        hipLaunchKernelGGL(k_axpy, dim3(nbv), dim3(NB), 0, s, n, u, 1.0 / o->n_inc, ubar, u);
        LAT_LAUNCH_CHECK();
        double rn = 0.0;
        int32_t code = 0;
        NCHK(evaluate(u, lf, r, &rn, &code));
        if (code != LAT_OK) return (lat_status)code;
        double t_eval = ms_since(t0);
        const double r0 = rn;
        if (r0 == 0.0) continue;
        bool conv = false;
        for (int it = 0; it < o->max_newton; ++it) {
            lat_newton_record rec{};
            rec.increment = t; rec.iteration = it; rec.res_before = rn; rec.res0 = r0;
            // reduced basis at u and the principal tangents (the standard method uses the cells' own
            // tangents, already formed with the residual)
            t0 = std::chrono::steady_clock::now();
            int32_t hnr = 0;
            if (!full) {
                NCHK(lat_status_reset(gst_d, s));
                // the greedy reads only the rows the snapshot rule fills
                const int64_t rows = lat_snapshot_rows(P, rule);
                NCHK(lat_select_principal_rows(P, snap, rows, o->rb_tol, o->cap, S, nr_d, alpha, beta, nu, R, nullptr,
                                               scal + 1, gst_d, nullptr, 0, s));
                int32_t hg[2] = {0, 0};
                double ach = 0.0;
                LAT_HIP(hipMemcpyAsync(&hnr, nr_d, sizeof(int32_t), hipMemcpyDeviceToHost, s));
                LAT_HIP(hipMemcpyAsync(hg, gst_d, sizeof(hg), hipMemcpyDeviceToHost, s));
                LAT_HIP(hipMemcpyAsync(&ach, scal + 1, sizeof(double), hipMemcpyDeviceToHost, s));
                LAT_HIP(hipStreamSynchronize(s));
                NCHK(lat_status_reset(st_d, s));
                NCHK(lat_principal_ops(P, u, mu, lam, S, hnr, K, nullptr, nullptr, st_d, nullptr, 0, s));
                if (w.ops) NCHK(combine_ops(P, K, hnr, alpha, w.ops, s));
                LAT_HIP(hipStreamSynchronize(s));
                rec.rb_achieved = ach; rec.greedy_status = hg[0];
            }
            rec.n_r = hnr;
            rec.t_init_ms = ms_since(t0);
            // tangent solve K~ du = -r
            t0 = std::chrono::steady_clock::now();
            hipLaunchKernelGGL(k_neg, dim3(nbv), dim3(NB), 0, s, n, r, rhs);
            LAT_LAUNCH_CHECK();
            int cgit = 0;
            double cgrel = 0.0;
            lat_status cst = LAT_E_NOCONV;
            bool need_mr = true;
            if (feti && hnr > 0) {
                // inexact FETI-DP (Sec. 3.3); a solve that stops short (an indefinite tangent) hands
                // the step to MINRES
                lat_feti_opts fo{};
                fo.n_delta = o->feti_n_delta; fo.enrich = 0; fo.max_enrich = 3; fo.inner_it = 32; fo.inner_tol = 1e-2; fo.restart = 60;
                fo.maxit = std::min(o->cg_maxit, 600); fo.materialize = w.ops != nullptr; fo.indefinite = 0;
                fo.coords = 1;
                fo.tol = o->cg_tol;
                lat_feti_info fi{};
                const lat_status fst = lat_feti_solve(P, K, hnr, alpha, S, R, nu, beta, fixed, rhs, du, &fo, &fi, s);
                if (fst != LAT_OK && fst != LAT_E_NOCONV && fst != LAT_E_SINGULAR) return fst;
                rec.solver = 1; rec.feti_iters = fi.iters; rec.feti_relres = fi.relres;
                rec.feti_enrich = fi.enrich; rec.t_feti_setup_ms = fi.t_setup_ms;
                if (fst == LAT_OK) {
                    need_mr = false;
                    cst = LAT_OK; cgit = fi.iters; cgrel = fi.relres;
                } else {
                    rec.solver = 2;
                }
            }
            if (need_mr) {
                cst = mr_run(P, w, K, hnr, alpha, w.ops, fixed, rhs, du, o->cg_tol, o->cg_maxit, o->cg_check, &cgit,
                             &cgrel, s, &rec.t_product_us);
                if (cst != LAT_OK && cst != LAT_E_NOCONV && cst != LAT_E_SINGULAR) return cst;
            }
            rec.cg_iters = cgit; rec.cg_relres = cgrel; rec.cg_status = cst; rec.coarse = need_mr && w.coarse_on;
            rec.t_solve_ms = ms_since(t0);
            // Armijo backtracking on ||r||
            t0 = std::chrono::steady_clock::now();
            int m = 0;
            double step = 1.0, rt = INFINITY;
            bool ok = false;
            for (; m <= o->max_backtrack; ++m, step *= o->armijo_beta) {
                hipLaunchKernelGGL(k_axpy, dim3(nbv), dim3(NB), 0, s, n, u, step, du, u_try);
                LAT_LAUNCH_CHECK();
                NCHK(evaluate(u_try, lf, r_try, &rt, &code));
                if (std::isfinite(rt) && rt <= (1.0 - o->armijo_c * step) * rn) { ok = true; break; }
            }
            rec.t_eval_ms = t_eval + ms_since(t0);
            t_eval = 0.0;
            rec.backtracks = m; rec.step = ok ? step : 0.0; rec.res_after = ok ? rt : rn;
            if (records && nrec < max_records) records[nrec] = rec;
            ++nrec;
            if (o->verbose) {
                std::fprintf(stderr, "newton inc %d it %d: n_r %d, solve %d its (status %d, coarse %d, solver %d, "
                             "feti %d its), m %d, |r|/|r0| %.3e, ms init %.1f solve %.1f eval %.1f\n", t, it, rec.n_r,
                             rec.cg_iters, rec.cg_status, rec.coarse, rec.solver, rec.feti_iters, rec.backtracks,
                             (ok ? rt : rn) / r0, rec.t_init_ms, rec.t_solve_ms, rec.t_eval_ms);
                std::fflush(stderr);
            }
            if (!ok) { result = LAT_E_NOCONV; break; }
            LAT_HIP(hipMemcpyAsync(u, u_try, n * sizeof(double), hipMemcpyDeviceToDevice, s));
            std::swap(r_try, r);   // the snapshots in `snap` belong to the accepted state already
            rn = rt;
            if (rn <= o->newton_tol * r0) { conv = true; break; }
        }
        if (!conv && result == LAT_OK) result = LAT_E_NOCONV;
    }
    LAT_HIP(hipStreamSynchronize(s));
    if (n_records) *n_records = nrec;
    return result;
}

}  // extern "C"
