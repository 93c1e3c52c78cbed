// Greedy selection of principal cells (Algorithm 1, Sec. 3.2.2), RB coefficients (the
// least-squares formula of Sec. 3.2.2, solved through the greedy's certified decomposition),
// and the reverse mode of those coefficients.
//
// The snapshot matrix T is cell-interleaved: row = snapshot entry, column = cell lane, so a
// wave streams 64 cells' entries with unit stride.  All decisions use FP64 in a fixed order:
//   - dot products / squared norms: chunks of 256 consecutive rows, each thread accumulating
//     its lane by s = fma(x, y, s) from 0; chunk sums combined by a pairwise tree (neighbours
//     (2k, 2k+1) per level, odd last element carried), done 256 rows per launch in LDS;
//   - inf-norms: max of |x| (exact, order-free);
//   - arg-max: largest inf-norm, ties to the lowest canonical cell id.
// The loop is device-driven: every iteration's kernels read a device 'done' flag and return
// at once when it is set, so the host enqueues `cap` iterations without synchronising.
#include "lat_internal.h"

namespace {

enum { C_DONE = 0, C_SEL = 1, C_NR = 2, C_CELL = 3 };
enum { D_RHO = 0, D_ACH = 1 };

// ---------------------------------------------------------------------------- tree reduction
// in [nrows][ld] -> out [ceil(nrows/256)][ld]; blockDim = 256 = TLX lanes x TRY row slots (few
// lanes per block: the greedy reduces ~150 rows of only ~1000 lanes, which needs many blocks).
// A second array (in2 -> out2, operation op2) may be reduced in the same launch.  When the
// launch produces the final value (one block of rows) it is written at out[p * ostride + ooff].
constexpr int TLX = 4, TRY = 256 / TLX;

struct TreeIO {
    const double *in;
    double *out;
    int op;
};

__device__ __forceinline__ void tree_block(double (*sh)[TLX + 1], const TreeIO &io, int64_t nrows, int64_t ld, int64_t p,
                                           int lx, int ry, int64_t ostride, int64_t ooff, bool final_level)
{
    const int64_t r0 = (int64_t)blockIdx.y * LAT_TREE;
    const int n0 = (int)((nrows - r0) < LAT_TREE ? (nrows - r0) : LAT_TREE);
    for (int t = ry; t < LAT_TREE; t += TRY) {
        double v = 0.0;
        if (t < n0 && p < ld) v = io.in[(r0 + t) * ld + p];
        sh[t][lx] = v;
    }
    __syncthreads();
    int n = n0;
    while (n > 1) {
        const int half = n >> 1;
        constexpr int PPT = (LAT_TREE / 2 + TRY - 1) / TRY;   // pairs per thread and level
        double vals[PPT];
#pragma unroll
        for (int t = 0; t < PPT; ++t) {
            const int k = ry + TRY * t;
            if (k < half) {
                const double x = sh[2 * k][lx], y = sh[2 * k + 1][lx];
                vals[t] = io.op == 0 ? x + y : fmax(x, y);
            }
        }
        const double tail = (n & 1) ? sh[n - 1][lx] : 0.0;
        __syncthreads();
#pragma unroll
        for (int t = 0; t < PPT; ++t) {
            const int k = ry + TRY * t;
            if (k < half) sh[k][lx] = vals[t];
        }
        if ((n & 1) && ry == 0) sh[half][lx] = tail;
        __syncthreads();
        n = half + (n & 1);
    }
    if (ry == 0 && p < ld) {
        if (final_level) io.out[p * ostride + ooff] = sh[0][lx];
        else io.out[(int64_t)blockIdx.y * ld + p] = sh[0][lx];
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_tree(TreeIO a, TreeIO b, int two, int64_t nrows, int64_t ld, int64_t ostride,
                                              int64_t ooff, int final_level, const int32_t *__restrict__ skip)
{
    __shared__ double sh[LAT_TREE][TLX + 1];
    if (skip && skip[0]) return;
    const int lx = threadIdx.x % TLX, ry = threadIdx.x / TLX;
    const int64_t p = (int64_t)blockIdx.x * TLX + lx;
    tree_block(sh, a, nrows, ld, p, lx, ry, ostride, ooff, final_level);
    if (two) tree_block(sh, b, nrows, ld, p, lx, ry, 1, 0, final_level);
}

// ---------------------------------------------------------------------------- greedy passes
// grid: x = lane blocks of 256, y = chunk (z for chunks beyond 65535)
__device__ __forceinline__ int64_t chunk_id() { return (int64_t)blockIdx.y + (int64_t)blockIdx.z * 65535; }

// squared norms of the raw snapshots
__global__ __launch_bounds__(256) void k_sq(const double *__restrict__ T, int64_t nsnap, int64_t ld, int64_t nchunk,
                                            double *__restrict__ psq)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t b = chunk_id();
    if (p >= ld || b >= nchunk) return;
    const int64_t j0 = b * LAT_CHUNK, j1 = j0 + LAT_CHUNK < nsnap ? j0 + LAT_CHUNK : nsnap;
    double s = 0.0;
    #pragma unroll 16
    for (int64_t j = j0; j < j1; ++j) { const double x = T[j * ld + p]; s = fma(x, x, s); }
    psq[b * ld + p] = s;
}

// Delta_0 = t / ||t||_2 (IEEE division; zero snapshot -> 0) with sq / inf partials of Delta_0.
// The chunk is read in register batches before it is written back (the same column is both
// read and written, so batching is what lets the loads run ahead of the stores).
constexpr int GB = 16;
__global__ __launch_bounds__(256) void k_normalize(double *__restrict__ T, int64_t nsnap, int64_t ld, int64_t nchunk,
                                                   const double *__restrict__ nu, double *__restrict__ psq,
                                                   double *__restrict__ pinf)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t b = chunk_id();
    if (p >= ld || b >= nchunk) return;
    const int64_t j0 = b * LAT_CHUNK, j1 = j0 + LAT_CHUNK < nsnap ? j0 + LAT_CHUNK : nsnap;
    const double n = nu[p];
    double s = 0.0, m = 0.0;
    for (int64_t jb = j0; jb < j1; jb += GB) {
        double v[GB];
#pragma unroll
        for (int t = 0; t < GB; ++t) v[t] = jb + t < j1 ? T[(jb + t) * ld + p] : 0.0;
#pragma unroll
        for (int t = 0; t < GB; ++t) {
            if (jb + t < j1) {
                const double x = n > 0.0 ? v[t] / n : 0.0;
                T[(jb + t) * ld + p] = x;
                s = fma(x, x, s);
                m = fmax(m, fabs(x));
            }
        }
    }
    psq[b * ld + p] = s;
    pinf[b * ld + p] = m;
}

__global__ void k_sqrt(int64_t ld, const double *__restrict__ sq, double *__restrict__ nu)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < ld) nu[p] = sqrt(sq[p]);
}

// Lagged residuals.  Iteration it works on Delta^(it) = Delta^(f) - sum_{k=f}^{it-1} beta_k zeta_k^T,
// f = it - it % LAT_GREEDY_LAG: T holds Delta^(f) and the NP = it - f pending updates are replayed
// on load, x = fma(-beta_k, zeta_k[j], x) for k = f, f+1, ..., exactly the operations the
// eager update would have applied one pass at a time, so every value is the eager one bit for
// bit.  Only the update that completes a multiple of LAT_GREEDY_LAG writes Delta back: a pass
// reads T once and writes it one iteration in LAT_GREEDY_LAG.
template <int NP>
struct Lag {
    double nb[NP > 0 ? NP : 1];
    const double *z[NP > 0 ? NP : 1];
    __device__ __forceinline__ Lag(const double *__restrict__ zring, int64_t nsnap, int f,
                                   const double *__restrict__ beta_pl, int64_t bstride, int64_t p)
    {
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            nb[k] = -beta_pl[p * bstride + f + k];
            z[k] = zring + (int64_t)((f + k) % LAT_GREEDY_LAG) * nsnap;
        }
    }
    __device__ __forceinline__ double replay(double x, int64_t j) const
    {
#pragma unroll
        for (int k = 0; k < NP; ++k) x = fma(nb[k], z[k][j], x);
        return x;
    }
};

// beta partials: Delta^(it) . zeta_it, it = f + NP
template <int NP>
__global__ __launch_bounds__(256) void k_dot(const double *__restrict__ T, int64_t nsnap, int64_t ld, int64_t nchunk,
                                             const double *__restrict__ zring, int f,
                                             const double *__restrict__ beta_pl, int64_t bstride,
                                             const int32_t *__restrict__ ictl, double *__restrict__ pdot)
{
    if (ictl[C_DONE]) return;
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t b = chunk_id();
    if (p >= ld || b >= nchunk) return;
    const int64_t j0 = b * LAT_CHUNK, j1 = j0 + LAT_CHUNK < nsnap ? j0 + LAT_CHUNK : nsnap;
    const Lag<NP> lag(zring, nsnap, f, beta_pl, bstride, p);
    const double *__restrict__ zeta = zring + (int64_t)((f + NP) % LAT_GREEDY_LAG) * nsnap;
    double s = 0.0;
    #pragma unroll 16
    for (int64_t j = j0; j < j1; ++j) s = fma(lag.replay(T[j * ld + p], j), zeta[j], s);
    pdot[b * ld + p] = s;
}

// Delta^(it+1) = Delta^(it) - beta_it zeta_it (it = f + NP) with its sq / inf partials; WB: written
// back (it + 1 a multiple of LAT_GREEDY_LAG; batched like k_normalize), else only measured
template <int NP, bool WB>
__global__ __launch_bounds__(256) void k_update(double *__restrict__ T, int64_t nsnap, int64_t ld, int64_t nchunk,
                                                const double *__restrict__ zring, int f,
                                                const double *__restrict__ beta_pl, int64_t bstride,
                                                const int32_t *__restrict__ ictl, double *__restrict__ psq,
                                                double *__restrict__ pinf)
{
    if (ictl[C_DONE]) return;
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t b = chunk_id();
    if (p >= ld || b >= nchunk) return;
    const int64_t j0 = b * LAT_CHUNK, j1 = j0 + LAT_CHUNK < nsnap ? j0 + LAT_CHUNK : nsnap;
    const Lag<NP> lag(zring, nsnap, f, beta_pl, bstride, p);
    const double *__restrict__ zeta = zring + (int64_t)((f + NP) % LAT_GREEDY_LAG) * nsnap;
    const double nb = -beta_pl[p * bstride + f + NP];
    double s = 0.0, m = 0.0;
    if (WB) {
        for (int64_t jb = j0; jb < j1; jb += GB) {
            double v[GB];
#pragma unroll
            for (int t = 0; t < GB; ++t) v[t] = jb + t < j1 ? T[(jb + t) * ld + p] : 0.0;
#pragma unroll
            for (int t = 0; t < GB; ++t) {
                if (jb + t < j1) {
                    const double x = fma(nb, zeta[jb + t], lag.replay(v[t], jb + t));
                    T[(jb + t) * ld + p] = x;
                    s = fma(x, x, s);
                    m = fmax(m, fabs(x));
                }
            }
        }
    } else {
        #pragma unroll 16
        for (int64_t j = j0; j < j1; ++j) {
            const double x = fma(nb, zeta[j], lag.replay(T[j * ld + p], j));
            s = fma(x, x, s);
            m = fmax(m, fabs(x));
        }
    }
    psq[b * ld + p] = s;
    pinf[b * ld + p] = m;
}

// After the loop: the updates still pending at exit (n_r - f of them, f = n_r - n_r % LAT_GREEDY_LAG)
// go into T, so that T holds Delta^(n_r) as the eager loop leaves it
template <int NP>
__device__ __forceinline__ void flush_rows(double *__restrict__ T, int64_t nsnap, int64_t ld, int64_t j0, int64_t j1,
                                           int64_t p, const double *__restrict__ zring, int f,
                                           const double *__restrict__ beta_pl, int64_t bstride)
{
    const Lag<NP> lag(zring, nsnap, f, beta_pl, bstride, p);
    for (int64_t jb = j0; jb < j1; jb += GB) {
        double v[GB];
#pragma unroll
        for (int t = 0; t < GB; ++t) v[t] = jb + t < j1 ? T[(jb + t) * ld + p] : 0.0;
#pragma unroll
        for (int t = 0; t < GB; ++t)
            if (jb + t < j1) T[(jb + t) * ld + p] = lag.replay(v[t], jb + t);
    }
}

__global__ __launch_bounds__(256) void k_flush(double *__restrict__ T, int64_t nsnap, int64_t ld, int64_t nchunk,
                                               const double *__restrict__ zring, const double *__restrict__ beta_pl,
                                               int64_t bstride, const int32_t *__restrict__ ictl)
{
    static_assert(LAT_GREEDY_LAG == 8, "the cases below cover 1..7 pending updates");
    const int nr = ictl[C_NR];
    const int f = nr - nr % LAT_GREEDY_LAG, np = nr - f;
    if (np == 0) return;
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t b = chunk_id();
    if (p >= ld || b >= nchunk) return;
    const int64_t j0 = b * LAT_CHUNK, j1 = j0 + LAT_CHUNK < nsnap ? j0 + LAT_CHUNK : nsnap;
    switch (np) {
    case 1: flush_rows<1>(T, nsnap, ld, j0, j1, p, zring, f, beta_pl, bstride); break;
    case 2: flush_rows<2>(T, nsnap, ld, j0, j1, p, zring, f, beta_pl, bstride); break;
    case 3: flush_rows<3>(T, nsnap, ld, j0, j1, p, zring, f, beta_pl, bstride); break;
    case 4: flush_rows<4>(T, nsnap, ld, j0, j1, p, zring, f, beta_pl, bstride); break;
    case 5: flush_rows<5>(T, nsnap, ld, j0, j1, p, zring, f, beta_pl, bstride); break;
    case 6: flush_rows<6>(T, nsnap, ld, j0, j1, p, zring, f, beta_pl, bstride); break;
    default: flush_rows<7>(T, nsnap, ld, j0, j1, p, zring, f, beta_pl, bstride); break;
    }
}

// Arg-max of the inf-norms over the lanes (ties -> lowest canonical cell), stop test, and the
// bookkeeping of iteration `it`.  One workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_select(int64_t ld, const int32_t *__restrict__ perm,
                                                 const double *__restrict__ inf, const double *__restrict__ sq,
                                                 double tol, int it, int cap, int32_t *__restrict__ ictl,
                                                 double *__restrict__ dctl, int32_t *__restrict__ S,
                                                 int32_t *__restrict__ n_r, int32_t *st)
{
    __shared__ double bv[1024];
    __shared__ int bc[1024];
    __shared__ int bl[1024];
    if (ictl[C_DONE]) return;
    double v = -1.0;
    int c = 0x7fffffff, l = -1;
    for (int64_t p = threadIdx.x; p < ld; p += 1024) {
        const int cell = perm[p];
        if (cell < 0) continue;
        const double x = inf[p];
        if (x > v || (x == v && cell < c)) { v = x; c = cell; l = (int)p; }
    }
    bv[threadIdx.x] = v; bc[threadIdx.x] = c; bl[threadIdx.x] = l;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double x = bv[threadIdx.x + w];
            const int cc = bc[threadIdx.x + w];
            if (x > bv[threadIdx.x] || (x == bv[threadIdx.x] && cc < bc[threadIdx.x])) {
                bv[threadIdx.x] = x; bc[threadIdx.x] = cc; bl[threadIdx.x] = bl[threadIdx.x + w];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double top = bv[0];
        dctl[D_ACH] = top > 0.0 ? top : 0.0;
        if (!(top > tol)) {                 // converged
            ictl[C_DONE] = 1;
            *n_r = it;
            ictl[C_NR] = it;
        } else if (it >= cap) {             // cap reached above the tolerance
            ictl[C_DONE] = 1;
            *n_r = it;
            ictl[C_NR] = it;
            lat_flag(st, LAT_W_CAP, 0x7fffffff);
        } else {
            ictl[C_SEL] = bl[0];
            ictl[C_CELL] = bc[0];
            S[it] = bc[0];
            dctl[D_RHO] = sqrt(sq[bl[0]]);
            *n_r = it + 1;
            ictl[C_NR] = it + 1;
        }
    }
}

// zeta_it = Delta^(it)[:, s_it] / ||Delta^(it)[:, s_it]||_2 (it = f + NP; the column replays the
// pending updates like the passes) into its ring slot, and the basis row Z[it]
template <int NP>
__global__ void k_zeta(const double *__restrict__ T, int64_t nsnap, int64_t ld, const int32_t *__restrict__ ictl,
                       const double *__restrict__ dctl, double *__restrict__ zring, int f,
                       const double *__restrict__ beta_pl, int64_t bstride, double *__restrict__ Zrow)
{
    if (ictl[C_DONE]) return;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nsnap) return;
    const int64_t sel = ictl[C_SEL];
    const Lag<NP> lag(zring, nsnap, f, beta_pl, bstride, sel);
    const double z = lag.replay(T[j * ld + sel], j) / dctl[D_RHO];
    zring[(int64_t)((f + NP) % LAT_GREEDY_LAG) * nsnap + j] = z;
    if (Zrow) Zrow[j] = z;
}

__global__ void k_store_beta(int64_t ld, int it, int cap, const int32_t *__restrict__ ictl,
                             const double *__restrict__ beta, double *__restrict__ beta_pl)
{
    if (ictl[C_DONE]) return;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < ld) beta_pl[p * cap + it] = beta[p];
}

__global__ void k_init_ctl(int32_t *ictl, double *dctl, int32_t *S, int cap, int32_t *n_r)
{
    const int t = threadIdx.x;
    if (t < 16) ictl[t] = 0;
    if (t < 16) dctl[t] = 0.0;
    if (t < cap) S[t] = -1;
    if (t == 0) *n_r = 0;
}

__global__ void k_zero(int64_t n, double *__restrict__ x)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.0;
}

// R[j][k] = nu_{s_k} beta_j^{s_k}, j <= k < n_r   (R has stride cap, beta_pl stride pcap)
__global__ void k_build_R(int cap, int pcap, const int32_t *__restrict__ ictl, const int32_t *__restrict__ S,
                          const int32_t *__restrict__ lane, const double *__restrict__ nu_pl,
                          const double *__restrict__ beta_pl, double *__restrict__ R)
{
    const int j = threadIdx.x, k = blockIdx.x;
    if (j >= cap || k >= cap) return;
    const int nr = ictl[C_NR];
    double v = 0.0;
    if (k < nr && j <= k) {
        const int pk = lane[S[k]];
        v = nu_pl[pk] * beta_pl[(int64_t)pk * pcap + j];
    }
    R[j * cap + k] = v;
}

// alpha^s: R alpha = nu_s beta^s by back-substitution from the last row (fma order
// acc = fma(-R[k][l], alpha_l, acc) for l = k+1 .. n_r-1); outputs in canonical order.
// NR = the plan's cap: every index is a compile-time constant, so alpha stays in registers.
template <int NR>
__global__ __launch_bounds__(256) void k_alpha(int64_t ld, int pcap, const int32_t *__restrict__ ictl,
                                               const int32_t *__restrict__ perm, const double *__restrict__ R,
                                               const double *__restrict__ nu_pl, const double *__restrict__ beta_pl,
                                               double *__restrict__ alpha, double *__restrict__ beta,
                                               double *__restrict__ nu)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ld) return;
    const int c = perm[p];
    if (c < 0) return;
    const int nr = ictl[C_NR];
    const double n = nu_pl[p];
    double a[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) a[k] = 0.0;
#pragma unroll
    for (int k = NR - 1; k >= 0; --k) {
        if (k < nr) {
            double acc = n * beta_pl[p * pcap + k];
#pragma unroll
            for (int l = k + 1; l < NR; ++l)
                if (l < nr) acc = fma(-R[k * NR + l], a[l], acc);
            a[k] = acc / R[k * NR + k];
        }
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        alpha[(int64_t)c * NR + k] = a[k];
        if (beta) beta[(int64_t)c * NR + k] = k < nr ? beta_pl[p * pcap + k] : 0.0;
    }
    if (nu) nu[c] = n;
}

__global__ void k_achieved(const double *__restrict__ dctl, double *__restrict__ achieved)
{
    if (threadIdx.x == 0) *achieved = dctl[D_ACH];
}

dim3 chunk_grid(int64_t ld, int64_t nchunk)
{
    return dim3((unsigned)lat_cdiv(ld, 256), (unsigned)(nchunk < 65535 ? nchunk : 65535), (unsigned)lat_cdiv(nchunk, 65535));
}

}  // namespace

// Pairwise-tree reduction of one or two [nrows][ld] arrays; final values to out[p * ostride + ooff]
// (second array: out2[p]).  `skip` (device flag, may be NULL) makes every launch return at once.
static lat_status tree2(const double *in, int op, double *out, int64_t ostride, int64_t ooff, const double *in2, int op2,
                        double *out2, int64_t nrows, int64_t ld, double *t1, double *t2, double *t3, double *t4,
                        const int32_t *skip, hipStream_t s)
{
    const double *src = in, *src2 = in2;
    int64_t n = nrows;
    double *bufs[2] = {t1, t2}, *bufs2[2] = {t3, t4};
    int which = 0;
    while (true) {
        const int64_t nb = lat_cdiv(n, LAT_TREE);
        const bool fin = nb == 1;
        TreeIO a{src, fin ? out : bufs[which], op};
        TreeIO b{src2, fin ? out2 : bufs2[which], op2};
        hipLaunchKernelGGL(k_tree, dim3((unsigned)lat_cdiv(ld, TLX), (unsigned)nb), dim3(256), 0, s, a, b, in2 ? 1 : 0, n,
                           ld, fin ? ostride : (int64_t)1, fin ? ooff : (int64_t)0, fin ? 1 : 0, skip);
        LAT_LAUNCH_CHECK();
        if (fin) break;
        src = bufs[which];
        src2 = bufs2[which];
        n = nb;
        which ^= 1;
    }
    return LAT_OK;
}

lat_status lat_tree_reduce(const double *in, int64_t nrows, int64_t ld, int op, double *out, double *t1, double *t2,
                           hipStream_t s)
{
    return tree2(in, op, out, 1, 0, nullptr, 0, nullptr, nrows, ld, t1, t2, nullptr, nullptr, nullptr, s);
}

extern "C" lat_status lat_select_principal(const lat_plan *P, double *snap, double tol, int32_t cap, int32_t *S,
                                           int32_t *n_r, double *alpha, double *beta, double *nu, double *R, double *Z,
                                           double *achieved, int32_t *dev_status, void *work, size_t work_bytes,
                                           hipStream_t stream)
{
    if (!P) return LAT_E_ARG;
    return lat_select_principal_rows(P, snap, P->nsnap, tol, cap, S, n_r, alpha, beta, nu, R, Z, achieved,
                                     dev_status, work, work_bytes, stream);
}

// The greedy on the first `rows` snapshot rows: the chunk sums and pairwise trees take a zero
// chunk without rounding, so when the rows past `rows` are zero the result is the full sweep's,
// bit for bit, at the cost of the data rows only.
extern "C" lat_status lat_select_principal_rows(const lat_plan *Pp, double *snap, int64_t rows, double tol, int32_t cap,
                                                int32_t *S, int32_t *n_r, double *alpha, double *beta, double *nu,
                                                double *R, double *Z, double *achieved, int32_t *dev_status,
                                                void *work, size_t work_bytes, hipStream_t stream)
{
    if (!Pp || !snap || !S || !n_r || !alpha || !R || !achieved) return LAT_E_ARG;
    if (!(tol > 0.0) || cap < 1) return LAT_E_ARG;
    if (cap > Pp->cap || rows < 1 || rows > Pp->nsnap) return LAT_E_SHAPE;
    lat_plan V;
    lat_status st0 = lat_ws_bind(Pp, LAT_CALL_SELECT_PRINCIPAL, work, work_bytes, &V);
    if (st0 != LAT_OK) return st0;
    const lat_plan *P = &V;
    const int64_t ld = P->ld, ns = rows, nc = lat_cdiv(rows, LAT_CHUNK);
    const dim3 cg = chunk_grid(ld, nc);
    const dim3 lg((unsigned)lat_cdiv(ld, 256));
    lat_status st;
    hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(64), 0, stream, P->ictl, P->dctl, S, P->cap, n_r);
    hipLaunchKernelGGL(k_zero, dim3((unsigned)lat_cdiv(ld * P->cap, 256)), dim3(256), 0, stream, ld * P->cap, P->beta_pl);
    if (Z) hipLaunchKernelGGL(k_zero, dim3((unsigned)lat_cdiv((int64_t)P->cap * P->nsnap, 256)), dim3(256), 0, stream,
                              (int64_t)P->cap * P->nsnap, Z);
    LAT_LAUNCH_CHECK();
    // nu_s = ||t^s||_2 and the normalisation Delta_0 = t / nu
    hipLaunchKernelGGL(k_sq, cg, dim3(256), 0, stream, snap, ns, ld, nc, P->g_sq);
    LAT_LAUNCH_CHECK();
    if ((st = lat_tree_reduce(P->g_sq, nc, ld, 0, P->v_sq, P->g_t1, P->g_t2, stream)) != LAT_OK) return st;
    hipLaunchKernelGGL(k_sqrt, lg, dim3(256), 0, stream, ld, P->v_sq, P->v_nu);
    hipLaunchKernelGGL(k_normalize, cg, dim3(256), 0, stream, snap, ns, ld, nc, P->v_nu, P->g_sq, P->g_inf);
    LAT_LAUNCH_CHECK();
    if ((st = tree2(P->g_sq, 0, P->v_sq, 1, 0, P->g_inf, 1, P->v_inf, nc, ld, P->g_t1, P->g_t2, P->g_t3, P->g_t4,
                    nullptr, stream)) != LAT_OK) return st;
    for (int it = 0; it <= cap; ++it) {
        hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, stream, ld, P->perm, P->v_inf, P->v_sq, tol, it, cap,
                           P->ictl, P->dctl, S, n_r, dev_status);
        LAT_LAUNCH_CHECK();
        if (it == cap) break;
        static_assert(LAT_GREEDY_LAG == 8, "the pass dispatch below covers 0..7 pending updates");
        const int np = it % LAT_GREEDY_LAG, f = it - np;
        const bool wb = np == LAT_GREEDY_LAG - 1;
        double *zrow = Z ? Z + (int64_t)it * P->nsnap : nullptr;
#define LAGGED(NPV)                                                                                                    \
    case NPV:                                                                                                          \
        hipLaunchKernelGGL(k_zeta<NPV>, dim3((unsigned)lat_cdiv(ns, 256)), dim3(256), 0, stream, snap, ns, ld, P->ictl, \
                           P->dctl, P->zeta, f, P->beta_pl, P->cap, zrow);                                             \
        hipLaunchKernelGGL(k_dot<NPV>, cg, dim3(256), 0, stream, snap, ns, ld, nc, P->zeta, f, P->beta_pl, P->cap,    \
                           P->ictl, P->g_dot);                                                                          \
        break;
        switch (np) { LAGGED(0) LAGGED(1) LAGGED(2) LAGGED(3) LAGGED(4) LAGGED(5) LAGGED(6) LAGGED(7) }
#undef LAGGED
        LAT_LAUNCH_CHECK();
        // beta_i lands directly in its column of the plan-order coordinate matrix
        if ((st = tree2(P->g_dot, 0, P->beta_pl, P->cap, it, nullptr, 0, nullptr, nc, ld, P->g_t1, P->g_t2, nullptr,
                        nullptr, P->ictl + C_DONE, stream)) != LAT_OK) return st;
#define LAGGED(NPV)                                                                                                    \
    case NPV:                                                                                                          \
        if (wb) hipLaunchKernelGGL((k_update<NPV, true>), cg, dim3(256), 0, stream, snap, ns, ld, nc, P->zeta, f,     \
                                   P->beta_pl, P->cap, P->ictl, P->g_sq, P->g_inf);                                    \
        else hipLaunchKernelGGL((k_update<NPV, false>), cg, dim3(256), 0, stream, snap, ns, ld, nc, P->zeta, f,       \
                                P->beta_pl, P->cap, P->ictl, P->g_sq, P->g_inf);                                       \
        break;
        switch (np) { LAGGED(0) LAGGED(1) LAGGED(2) LAGGED(3) LAGGED(4) LAGGED(5) LAGGED(6) LAGGED(7) }
#undef LAGGED
        LAT_LAUNCH_CHECK();
        if ((st = tree2(P->g_sq, 0, P->v_sq, 1, 0, P->g_inf, 1, P->v_inf, nc, ld, P->g_t1, P->g_t2, P->g_t3, P->g_t4,
                        P->ictl + C_DONE, stream)) != LAT_OK) return st;
    }
    hipLaunchKernelGGL(k_flush, cg, dim3(256), 0, stream, snap, ns, ld, nc, P->zeta, P->beta_pl, P->cap, P->ictl);
    LAT_LAUNCH_CHECK();
    // R, alpha (canonical order), beta, nu, achieved
    hipLaunchKernelGGL(k_build_R, dim3((unsigned)P->cap), dim3(64), 0, stream, P->cap, P->cap, P->ictl, S, P->lane,
                       P->v_nu, P->beta_pl, R);
#define ALPHA(NRV) hipLaunchKernelGGL(k_alpha<NRV>, lg, dim3(256), 0, stream, ld, P->cap, P->ictl, P->perm, R, P->v_nu, \
                                    P->beta_pl, alpha, beta, nu)
    switch (P->cap) {
    case 8: ALPHA(8); break;
    case 16: ALPHA(16); break;
    case 32: ALPHA(32); break;
    case 64: ALPHA(64); break;
    default: return LAT_E_SHAPE;
    }
#undef ALPHA
    hipLaunchKernelGGL(k_achieved, dim3(1), dim3(64), 0, stream, P->dctl, achieved);
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}
