// Plan creation, DOF maps (eq. residualvector: the Boolean assembly operators A^s as index
// maps), lane grouping, packed layouts, layout conversions and deterministic assembly.
#include <algorithm>
#include <cstring>
#include <numeric>

#include "lat_internal.h"

namespace {

// --------------------------------------------------------------------------- DOF-map kernels
// A local node is active in a cell when one of its (up to 2^d) elements is kept.
__global__ void k_active(int dim, int nel, int64_t ncells, const uint8_t *__restrict__ keep,
                         uint8_t *__restrict__ act)
{
    const int nn = nel + 1;
    const int nloc = dim == 2 ? nn * nn : nn * nn * nn;
    const int nelem = dim == 2 ? nel * nel : nel * nel * nel;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncells * nloc) return;
    int64_t c = t / nloc;
    int a = (int)(t % nloc);
    int ia[3] = {a % nn, (a / nn) % nn, dim == 3 ? a / (nn * nn) : 0};
    uint8_t on = 0;
    for (int k = 0; k < (1 << dim); ++k) {
        int ie[3] = {0, 0, 0};
        bool ok = true;
        for (int ax = 0; ax < dim; ++ax) {
            ie[ax] = ia[ax] - ((k >> ax) & 1);
            ok = ok && ie[ax] >= 0 && ie[ax] < nel;
        }
        if (!ok) continue;
        int e = ie[0] + nel * (ie[1] + nel * ie[2]);
        on |= keep[c * nelem + e];
    }
    act[t] = on ? 1 : 0;
}

// Counts active nodes per cell: one workgroup per cell.
__global__ void k_count(int nloc, const uint8_t *__restrict__ act, int32_t *__restrict__ nact)
{
    __shared__ int sh[256];
    int64_t c = blockIdx.x;
    int s = 0;
    for (int a = threadIdx.x; a < nloc; a += blockDim.x) s += act[c * nloc + a];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) nact[c] = sh[0];
}

struct Grid {
    int dim, nel, nn;
    int ncell[3];
    int64_t gs[3];
};

// Flags background nodes that are active in at least one cell containing them.
__global__ void k_global_flags(Grid g, int64_t nbg, const uint8_t *__restrict__ act, int32_t *__restrict__ flag)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nbg) return;
    int64_t r = t;
    int gc[3] = {0, 0, 0};
    for (int ax = 0; ax < g.dim; ++ax) { gc[ax] = (int)(r % g.gs[ax]); r /= g.gs[ax]; }
    const int nloc = g.dim == 2 ? g.nn * g.nn : g.nn * g.nn * g.nn;
    int on = 0;
    // the cells containing this node: per axis, the cell below and/or above the node
    for (int k = 0; k < (1 << g.dim) && !on; ++k) {
        int cc[3] = {0, 0, 0}, ia[3] = {0, 0, 0};
        bool ok = true;
        for (int ax = 0; ax < g.dim; ++ax) {
            int base = gc[ax] / g.nel;            // cell whose low face is at or below the node
            int c = ((k >> ax) & 1) ? base - 1 : base;
            int loc = gc[ax] - c * g.nel;
            ok = ok && c >= 0 && c < g.ncell[ax] && loc >= 0 && loc <= g.nel;
            cc[ax] = c; ia[ax] = loc;
        }
        if (!ok) continue;
        int64_t cell = cc[0] + (int64_t)g.ncell[0] * (cc[1] + (int64_t)g.ncell[1] * cc[2]);
        int a = ia[0] + g.nn * (ia[1] + g.nn * ia[2]);
        on |= act[cell * nloc + a];
    }
    flag[t] = on ? 1 : 0;
}

// Exclusive scan of int32 flags in blocks of 1024 (three phases).
__global__ void k_scan_blocks(int64_t n, const int32_t *__restrict__ in, int32_t *__restrict__ out,
                              int32_t *__restrict__ bsum)
{
    __shared__ int32_t sh[1024];
    int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    int32_t v = i < n ? in[i] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = 1; w < 1024; w <<= 1) {
        int32_t x = (int)threadIdx.x >= w ? sh[threadIdx.x - w] : 0;
        __syncthreads();
        sh[threadIdx.x] += x;
        __syncthreads();
    }
    if (i < n) out[i] = sh[threadIdx.x] - v;
    if (threadIdx.x == 1023) bsum[blockIdx.x] = sh[1023];
}

__global__ void k_scan_sums(int64_t nb, int32_t *__restrict__ bsum, int32_t *__restrict__ total)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int32_t run = 0;
        for (int64_t b = 0; b < nb; ++b) { int32_t v = bsum[b]; bsum[b] = run; run += v; }
        *total = run;
    }
}

__global__ void k_scan_add(int64_t n, const int32_t *__restrict__ flag, int32_t *__restrict__ out,
                           const int32_t *__restrict__ bsum, int64_t *__restrict__ g2bg)
{
    int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    if (i >= n) return;
    int32_t id = out[i] + bsum[blockIdx.x];
    if (flag[i]) { out[i] = id; if (g2bg) g2bg[id] = i; }
    else out[i] = -1;
}

__global__ void k_l2g(Grid g, int64_t ncells, const uint8_t *__restrict__ act, const int32_t *__restrict__ gid,
                      int32_t *__restrict__ l2g)
{
    const int nloc = g.dim == 2 ? g.nn * g.nn : g.nn * g.nn * g.nn;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncells * nloc) return;
    int64_t c = t / nloc;
    int a = (int)(t % nloc);
    int64_t r = c;
    int64_t gidx = 0, st = 1;
    int ia[3] = {a % g.nn, (a / g.nn) % g.nn, g.dim == 3 ? a / (g.nn * g.nn) : 0};
    for (int ax = 0; ax < g.dim; ++ax) {
        int cc = (int)(r % g.ncell[ax]); r /= g.ncell[ax];
        gidx += ((int64_t)cc * g.nel + ia[ax]) * st;
        st *= g.gs[ax];
    }
    l2g[t] = act[t] ? gid[gidx] : -1;
}

// --------------------------------------------------------------------------- layout kernels
__global__ void k_interleave_u8(int64_t rows, int64_t ld, int64_t ncells, const int32_t *__restrict__ perm,
                                const uint8_t *__restrict__ src, uint8_t *__restrict__ dst)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t r = blockIdx.y;
    if (p >= ld) return;
    int c = perm[p];
    dst[r * ld + p] = c >= 0 ? src[(int64_t)c * rows + r] : 0;
}

__global__ void k_interleave_i32(int64_t rows, int64_t ld, const int32_t *__restrict__ perm,
                                 const int32_t *__restrict__ src, int32_t *__restrict__ dst)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t r = blockIdx.y;
    if (p >= ld) return;
    int c = perm[p];
    dst[r * ld + p] = c >= 0 ? src[(int64_t)c * rows + r] : -1;
}

// canonical [N_s][nloc][k] -> CIL(k) [nloc][k][ld] and back
__global__ void k_canon_to_cil(int64_t nloc, int64_t k, int64_t ld, const int32_t *__restrict__ perm,
                               const double *__restrict__ canon, double *__restrict__ cil)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t row = (int64_t)blockIdx.y + (int64_t)blockIdx.z * 65535;
    if (p >= ld || row >= nloc * k) return;
    int c = perm[p];
    cil[row * ld + p] = c >= 0 ? canon[(int64_t)c * nloc * k + row] : 0.0;
}

__global__ void k_cil_to_canon(int64_t nloc, int64_t k, int64_t ld, const int32_t *__restrict__ perm,
                               const double *__restrict__ cil, double *__restrict__ canon)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t row = (int64_t)blockIdx.y + (int64_t)blockIdx.z * 65535;
    if (p >= ld || row >= nloc * k) return;
    int c = perm[p];
    if (c >= 0) canon[(int64_t)c * nloc * k + row] = cil[row * ld + p];
}

// packed [(q*d+i)*m+r][64] <-> canonical [N_s][nloc][d][m]
__global__ void k_pack(int dim, int m, int64_t nloc, int64_t npk, const int32_t *__restrict__ perm,
                       const int32_t *__restrict__ goff_q, const int32_t *__restrict__ unode,
                       const int32_t *__restrict__ l2g, const double *__restrict__ canon, double *__restrict__ packed)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // over npk*d*m*64
    int64_t tot = npk * dim * m * LAT_WAVE;
    if (t >= tot) return;
    int l = (int)(t % LAT_WAVE);
    int64_t rest = t / LAT_WAVE;
    int r = (int)(rest % m); rest /= m;
    int i = (int)(rest % dim);
    int64_t q = rest / dim;
    int g = goff_q[q];
    int c = perm[(int64_t)g * LAT_WAVE + l];
    double v = 0.0;
    if (c >= 0) {
        int a = unode[q];
        if (l2g[(int64_t)c * nloc + a] >= 0) v = canon[(((int64_t)c * nloc + a) * dim + i) * m + r];
    }
    packed[t] = v;
}

__global__ void k_unpack(int dim, int m, int64_t nloc, int64_t ncells, const int32_t *__restrict__ lane,
                         const int32_t *__restrict__ uidx, const int32_t *__restrict__ goff,
                         const int32_t *__restrict__ l2g, const double *__restrict__ packed,
                         double *__restrict__ canon)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // over ncells*nloc*d*m
    int64_t tot = ncells * nloc * dim * m;
    if (t >= tot) return;
    int r = (int)(t % m);
    int64_t rest = t / m;
    int i = (int)(rest % dim); rest /= dim;
    int a = (int)(rest % nloc);
    int64_t c = rest / nloc;
    int p = lane[c];
    int g = p / LAT_WAVE, l = p % LAT_WAVE;
    int qi = uidx[(int64_t)g * nloc + a];
    double v = 0.0;
    if (qi >= 0 && l2g[c * nloc + a] >= 0) {
        int64_t q = goff[g] + qi;
        v = packed[((q * dim + i) * m + r) * LAT_WAVE + l];
    }
    canon[t] = v;
}

__global__ void k_plain_to_canon(int E, int64_t nloc, int64_t ncells, const int32_t *__restrict__ lane,
                                 const int32_t *__restrict__ uidx, const int32_t *__restrict__ goff,
                                 const double *__restrict__ ops, double *__restrict__ canon)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t tot = ncells * nloc * E;
    if (t >= tot) return;
    int e = (int)(t % E);
    int64_t rest = t / E;
    int a = (int)(rest % nloc);
    int64_t c = rest / nloc;
    int p = lane[c];
    int g = p / LAT_WAVE, l = p % LAT_WAVE;
    int qi = uidx[(int64_t)g * nloc + a];
    canon[t] = qi >= 0 ? ops[(((int64_t)goff[g] + qi) * E + e) * LAT_WAVE + l] : 0.0;
}

// Deterministic assembly: every global node sums the cells that own it in ascending order.
__global__ void k_assemble(Grid g, int64_t nglobal, int k, int64_t ld, const int64_t *__restrict__ g2bg,
                           const int32_t *__restrict__ l2g, const int32_t *__restrict__ lane,
                           const double *__restrict__ local, double *__restrict__ out)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nglobal) return;
    int64_t r = g2bg[t];
    int gc[3] = {0, 0, 0};
    for (int ax = 0; ax < g.dim; ++ax) { gc[ax] = (int)(r % g.gs[ax]); r /= g.gs[ax]; }
    const int nloc = g.dim == 2 ? g.nn * g.nn : g.nn * g.nn * g.nn;
    double acc[3] = {0.0, 0.0, 0.0};
    // enumerate containing cells in ascending canonical id: z outer, then y, then x (low first)
    for (int kz = (g.dim == 3 ? 1 : 0); kz >= 0; --kz)
        for (int ky = 1; ky >= 0; --ky)
            for (int kx = 1; kx >= 0; --kx) {
                int kk[3] = {kx, ky, kz};
                int cc[3] = {0, 0, 0}, ia[3] = {0, 0, 0};
                bool ok = true;
                for (int ax = 0; ax < g.dim; ++ax) {
                    int base = gc[ax] / g.nel;
                    int c = kk[ax] ? base - 1 : base;
                    int loc = gc[ax] - c * g.nel;
                    ok = ok && c >= 0 && c < g.ncell[ax] && loc >= 0 && loc <= g.nel;
                    cc[ax] = c; ia[ax] = loc;
                }
                if (!ok) continue;
                int64_t cell = cc[0] + (int64_t)g.ncell[0] * (cc[1] + (int64_t)g.ncell[1] * cc[2]);
                int a = ia[0] + g.nn * (ia[1] + g.nn * ia[2]);
                if (l2g[cell * nloc + a] < 0) continue;
                int p = lane[cell];
                for (int i = 0; i < k; ++i) acc[i] += local[((int64_t)a * k + i) * ld + p];
            }
    for (int i = 0; i < k; ++i) out[t * k + i] = acc[i];
}

// w^s = A^{sT} w: global [n_global][k] -> CIL(k), zero at nodes a cell does not own
__global__ void k_gather(int k, int64_t ld, const int32_t *__restrict__ l2g_il, const double *__restrict__ glob,
                         double *__restrict__ cil)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int a = blockIdx.y;
    if (p >= ld) return;
    const int g = l2g_il[(int64_t)a * ld + p];
    for (int i = 0; i < k; ++i) cil[((int64_t)a * k + i) * ld + p] = g >= 0 ? glob[(int64_t)g * k + i] : 0.0;
}

__global__ void k_status_reset(int32_t *st)
{
    if (threadIdx.x == 0) { st[0] = LAT_OK; st[1] = 0x7fffffff; }
}

Grid make_grid(const lat_plan *P)
{
    Grid g;
    g.dim = P->dim; g.nel = P->nel; g.nn = P->nn;
    for (int ax = 0; ax < 3; ++ax) {
        g.ncell[ax] = P->ncell[ax];
        g.gs[ax] = ax < P->dim ? (int64_t)P->ncell[ax] * P->nel + 1 : 1;
    }
    return g;
}

template <class T>
lat_status dalloc(T **p, size_t n)
{
    if (n == 0) n = 1;
    if (hipMalloc((void **)p, n * sizeof(T)) != hipSuccess) { *p = nullptr; return LAT_E_NOMEM; }
    return LAT_OK;
}

// DOF-map kernels into caller-provided (or plan) buffers.  act: [N_s][nloc] scratch.
lat_status run_dofmap(const lat_plan *P, uint8_t *act, int32_t *flag, int32_t *gid, int32_t *bsum,
                      int32_t *d_total, int32_t *l2g, int32_t *nact, int64_t *g2bg, hipStream_t s)
{
    Grid g = make_grid(P);
    int64_t nt = P->ncells * P->nloc;
    hipLaunchKernelGGL(k_active, dim3((unsigned)lat_cdiv(nt, 256)), dim3(256), 0, s, P->dim, P->nel, P->ncells,
                       P->keep, act);
    LAT_LAUNCH_CHECK();
    if (nact) {
        hipLaunchKernelGGL(k_count, dim3((unsigned)P->ncells), dim3(256), 0, s, P->nloc, act, nact);
        LAT_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_global_flags, dim3((unsigned)lat_cdiv(P->nbg, 256)), dim3(256), 0, s, g, P->nbg, act, flag);
    LAT_LAUNCH_CHECK();
    int64_t nb = lat_cdiv(P->nbg, 1024);
    hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(1024), 0, s, P->nbg, flag, gid, bsum);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(64), 0, s, nb, bsum, d_total);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(1024), 0, s, P->nbg, flag, gid, bsum, g2bg);
    LAT_LAUNCH_CHECK();
    if (l2g) {
        hipLaunchKernelGGL(k_l2g, dim3((unsigned)lat_cdiv(nt, 256)), dim3(256), 0, s, g, P->ncells, act, gid, l2g);
        LAT_LAUNCH_CHECK();
    }
    return LAT_OK;
}

// ---- caller workspaces
struct WsItem {
    void **ptr;          // field of the plan copy
    size_t bytes;
    int fast;            // 0: always; 1: only with the "fast" size; 2: the same region as the item before
};

// The scratch of each call, in carving order (every item starts on a 256-byte boundary).
int ws_items(const lat_plan *P, lat_plan *V, int call, WsItem *it)
{
    int n = 0;
    auto add = [&](void *field, int64_t elems, size_t esz, int fast) {
        it[n].ptr = (void **)field;          // NULL: a size only (carved by the call itself)
        it[n].bytes = (size_t)std::max<int64_t>(elems, 1) * esz;
        it[n].fast = fast;
        ++n;
    };
    const int64_t ld = P->ld, cap = P->cap, nloc = P->nloc, tr = P->tree_elems;
    switch (call) {
    case LAT_CALL_RESIDUAL_TANGENT:
    case LAT_CALL_RESIDUAL_ADJOINT:
        add(&V->u_cil, nloc * P->dim * ld, 8, 0);
        add(&V->w_part, nloc * ld, 8, 0);
        add(&V->w_part2, nloc * ld, 8, 0);
        add(&V->v_sq, ld, 8, 0);
        add(&V->v_inf, ld, 8, 0);
        add(&V->g_t1, tr, 8, 0);
        add(&V->g_t2, tr, 8, 0);
        break;
    case LAT_CALL_PRINCIPAL_OPS:
        add(&V->u_cil, nloc * P->dim * ld, 8, 0);
        break;
    case LAT_CALL_SELECT_PRINCIPAL:
        add(&V->g_sq, P->nchunk * ld, 8, 0);
        add(&V->g_inf, P->nchunk * ld, 8, 0);
        add(&V->g_dot, P->nchunk * ld, 8, 0);
        add(&V->g_t1, tr, 8, 0);
        add(&V->g_t2, tr, 8, 0);
        add(&V->g_t3, tr, 8, 0);
        add(&V->g_t4, tr, 8, 0);
        add(&V->v_sq, ld, 8, 0);
        add(&V->v_inf, ld, 8, 0);
        add(&V->v_beta, ld, 8, 0);
        add(&V->v_nu, ld, 8, 0);
        add(&V->beta_pl, ld * cap, 8, 0);
        add(&V->zeta, LAT_GREEDY_LAG * P->nsnap, 8, 0);
        add(&V->ictl, 64, 4, 0);
        add(&V->dctl, 64, 8, 0);
        break;
    case LAT_CALL_APPLY_COMBO:
        add(&V->alpha_il, cap * ld, 8, 0);
        add(&V->lp_err, 2 * (int64_t)P->nblk_lp, 8, 0);
        add(&V->lp_gate, 8, 4, 0);
        break;
    case LAT_CALL_APPLY_COMBO_ADJOINT:
        add(&V->alpha_il, cap * ld, 8, 0);
        add(&V->lp_err, 2 * (int64_t)P->nblk_lp, 8, 0);
        add(&V->lp_gate, 8, 4, 0);
        add(&V->form_part, (int64_t)P->napc * ld * cap, 8, 0);
        add(&V->form_out, ld * cap, 8, 0);
        add(&V->form_out3, 3 * ld * cap, 8, 0);
        add(&V->g_t1, tr, 8, 0);
        add(&V->g_t2, tr, 8, 0);
        add(&V->aa_part, P->aa_nchunk * ld * cap, 8, 0);
        // fast: the cells' W (FP64) for every lane and its contraction partials of three stacks; the
        // call carves them from the rest of the workspace, in lane batches when less is given
        add(nullptr, lat_forms_batch_bytes(P, ld), 1, 1);
        break;
    case LAT_CALL_ALPHA_ADJOINT:
        add(&V->aa_A, 2 * cap * ld, 8, 0);
        add(&V->aa_B, 2 * ld * cap, 8, 0);
        add(&V->aa_q, 2 * cap * ld, 8, 0);
        add(&V->aa_gath, P->nsnap * cap, 8, 0);
        add(&V->aa_part, P->aa_nchunk * ld * cap, 8, 0);
        add(&V->g_t1, tr, 8, 0);
        add(&V->g_t2, tr, 8, 0);
        add(&V->wf_part, 2 * P->aa_nchunk * ld * cap, 8, 1);
        add(&V->aa_gath2, P->nsnap * cap, 8, 1);
        break;
    default: break;
    }
    return n;
}

size_t ws_align(size_t b) { return (b + 255) & ~(size_t)255; }

void free_plan(lat_plan *P)
{
    if (!P) return;
    void *ptrs[] = {P->keep, P->keep_il, P->perm, P->lane, P->l2g, P->l2g_il, P->nact, P->g2bg, P->dm_act, P->dm_flag,
                    P->dm_gid, P->dm_bsum, P->goff,
                    P->unode, P->unbr, P->umask, P->uidx, P->u_cil, P->w_part, P->w_part2, P->g_sq, P->g_inf,
                    P->g_dot, P->g_t1, P->g_t2, P->g_t3, P->g_t4, P->v_sq, P->v_inf, P->v_beta, P->v_nu, P->beta_pl, P->zeta,
                    P->ictl, P->dctl, P->form_part, P->form_out, P->form_out3, P->alpha_il, P->aa_A, P->aa_B, P->aa_q, P->aa_gath, P->aa_part,
                    P->lp_err, P->lp_gate};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete P;
}

}  // namespace

extern "C" {

const char *lat_status_string(lat_status s)
{
    switch (s) {
    case LAT_OK: return "ok";
    case LAT_E_ARG: return "invalid argument";
    case LAT_E_SHAPE: return "shape mismatch";
    case LAT_E_DEVICE: return "HIP runtime error";
    case LAT_E_NOMEM: return "out of device memory";
    case LAT_E_INVERTED: return "inverted element (J <= 0)";
    case LAT_E_NONFINITE: return "non-finite value";
    case LAT_W_CAP: return "principal-cell cap reached above tolerance";
    case LAT_E_NOCONV: return "iteration limit reached before convergence";
    case LAT_E_SINGULAR: return "singular operator in the tangent solve";
    }
    return "unknown status";
}

lat_status lat_status_reset(int32_t *dev_status, hipStream_t stream)
{
    if (!dev_status) return LAT_E_ARG;
    hipLaunchKernelGGL(k_status_reset, dim3(1), dim3(64), 0, stream, dev_status);
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

lat_status lat_plan_create(int32_t dim, const int32_t ncell[3], int32_t nel, const uint8_t *keep_host,
                           int32_t cap, hipStream_t stream, lat_plan **out)
{
    if (!out) return LAT_E_ARG;
    *out = nullptr;
    if ((dim != 2 && dim != 3) || !ncell || !keep_host || nel < 1 || nel > 64 || cap < 1 || cap > LAT_MAX_CAP)
        return LAT_E_ARG;
    for (int ax = 0; ax < dim; ++ax)
        if (ncell[ax] < 1) return LAT_E_ARG;
    lat_plan *P = new lat_plan();
    P->dim = dim; P->nel = nel; P->nn = nel + 1;
    P->nloc = lat_ipow(nel + 1, dim); P->nelem = lat_ipow(nel, dim);
    P->no = lat_ipow(3, dim); P->E = P->no * dim * dim; P->nc = 1 << dim;
    P->ncells = 1; P->nbg = 1;
    for (int ax = 0; ax < 3; ++ax) {
        P->ncell[ax] = ax < dim ? ncell[ax] : 1;
        P->ncells *= P->ncell[ax];
        P->nbg *= ax < dim ? (int64_t)ncell[ax] * nel + 1 : 1;
    }
    if (P->nbg >= (int64_t)INT32_MAX || P->ncells >= (int64_t)INT32_MAX / 64) { delete P; return LAT_E_ARG; }
    P->nsnap = (int64_t)P->nloc * P->E;
    P->cap = 8;                                     // stride of every [..][cap] array: a power of two >= cap
    while (P->cap < cap) P->cap *= 2;
    cap = P->cap;
    LAT_HIP(hipGetDevice(&P->device));
    lat_status st;
#define ALLOC(ptr, n) do { if ((st = dalloc(&(ptr), (size_t)(n))) != LAT_OK) { free_plan(P); return st; } } while (0)
#define HCHK(call) do { hipError_t e_ = (call); if (e_ != hipSuccess) { \
        std::fprintf(stderr, "liblat: %s failed: %s\n", #call, hipGetErrorString(e_)); free_plan(P); return LAT_E_DEVICE; } } while (0)
    const int64_t Ns = P->ncells, nloc = P->nloc;
    ALLOC(P->keep, Ns * P->nelem);
    HCHK(hipMemcpyAsync(P->keep, keep_host, (size_t)(Ns * P->nelem), hipMemcpyHostToDevice, stream));
    // ---- DOF maps on the device
    ALLOC(P->dm_act, Ns * nloc);
    ALLOC(P->dm_flag, P->nbg);
    ALLOC(P->dm_gid, P->nbg);
    ALLOC(P->dm_bsum, lat_cdiv(P->nbg, 1024) + 1);
    ALLOC(P->l2g, Ns * nloc);
    ALLOC(P->nact, Ns);
    ALLOC(P->g2bg, P->nbg);      // only the first nglobal entries are used
    uint8_t *act = P->dm_act;
    int32_t *tot = P->dm_bsum + lat_cdiv(P->nbg, 1024);
    if ((st = run_dofmap(P, act, P->dm_flag, P->dm_gid, P->dm_bsum, tot, P->l2g, P->nact, P->g2bg, stream)) != LAT_OK) {
        free_plan(P); return st;
    }
    std::vector<uint8_t> h_act((size_t)(Ns * nloc));
    std::vector<int32_t> h_nact((size_t)Ns);
    int32_t h_tot = 0;
    HCHK(hipMemcpyAsync(h_act.data(), act, h_act.size(), hipMemcpyDeviceToHost, stream));
    HCHK(hipMemcpyAsync(h_nact.data(), P->nact, h_nact.size() * 4, hipMemcpyDeviceToHost, stream));
    HCHK(hipMemcpyAsync(&h_tot, tot, 4, hipMemcpyDeviceToHost, stream));
    HCHK(hipStreamSynchronize(stream));
    P->nglobal = h_tot;

    // ---- lane grouping (host): sort cells by a coarse mask signature, then by active count,
    // so that each group of 64 lanes holds cells with similar active-node sets.
    const int nn = P->nn;
    std::vector<uint64_t> sig((size_t)Ns, 0);
    {
        int probes_per_axis = dim == 2 ? 8 : 4;     // 64 probe nodes in both cases
        for (int64_t c = 0; c < Ns; ++c) {
            uint64_t s = 0; int bit = 0;
            for (int pz = 0; pz < (dim == 3 ? probes_per_axis : 1); ++pz)
                for (int py = 0; py < probes_per_axis; ++py)
                    for (int px = 0; px < probes_per_axis; ++px) {
                        int ix = (int)((px + 0.5) * nn / probes_per_axis);
                        int iy = (int)((py + 0.5) * nn / probes_per_axis);
                        int iz = dim == 3 ? (int)((pz + 0.5) * nn / probes_per_axis) : 0;
                        int a = ix + nn * (iy + nn * iz);
                        if (h_act[(size_t)(c * nloc + a)]) s |= (uint64_t)1 << bit;
                        ++bit;
                    }
            sig[(size_t)c] = s;
        }
    }
    std::vector<int32_t> order((size_t)Ns);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        if (sig[x] != sig[y]) return sig[x] < sig[y];
        return h_nact[x] < h_nact[y];
    });
    P->ngroups = (int)lat_cdiv(Ns, LAT_WAVE);
    P->ld = (int64_t)P->ngroups * LAT_WAVE;
    const int64_t ld = P->ld;
    std::vector<int32_t> h_perm((size_t)ld, -1), h_lane((size_t)Ns);
    for (int64_t t = 0; t < Ns; ++t) { h_perm[(size_t)t] = order[(size_t)t]; h_lane[(size_t)order[(size_t)t]] = (int32_t)t; }
    // ---- packed layout: per group, the union of its cells' active nodes
    std::vector<int32_t> h_goff((size_t)P->ngroups + 1, 0), h_uidx((size_t)P->ngroups * nloc, -1), h_unode;
    std::vector<uint64_t> h_umask;
    P->maxunion = 0;
    for (int g = 0; g < P->ngroups; ++g) {
        int cnt = 0;
        for (int a = 0; a < nloc; ++a) {
            uint64_t msk = 0;
            for (int l = 0; l < LAT_WAVE; ++l) {
                int c = h_perm[(size_t)g * LAT_WAVE + l];
                if (c >= 0 && h_act[(size_t)((int64_t)c * nloc + a)]) msk |= (uint64_t)1 << l;
            }
            if (msk) {
                h_uidx[(size_t)g * nloc + a] = cnt++;
                h_unode.push_back(a);
                h_umask.push_back(msk);
            }
        }
        h_goff[(size_t)g + 1] = h_goff[(size_t)g] + cnt;
        P->maxunion = std::max(P->maxunion, cnt);
    }
    P->npacked = h_goff[(size_t)P->ngroups];
    std::vector<int32_t> h_unbr((size_t)std::max<int64_t>(P->npacked, 1) * P->no, -1);
    for (int g = 0; g < P->ngroups; ++g)
        for (int q = h_goff[(size_t)g]; q < h_goff[(size_t)g + 1]; ++q) {
            int a = h_unode[(size_t)q];
            int ia[3] = {a % nn, (a / nn) % nn, dim == 3 ? a / (nn * nn) : 0};
            for (int o = 0; o < P->no; ++o) {
                int ib[3] = {ia[0] + o % 3 - 1, ia[1] + (o / 3) % 3 - 1, dim == 3 ? ia[2] + o / 9 - 1 : 0};
                bool ok = true;
                for (int ax = 0; ax < dim; ++ax) ok = ok && ib[ax] >= 0 && ib[ax] < nn;
                if (!ok) continue;
                int b = ib[0] + nn * (ib[1] + nn * ib[2]);
                int qi = h_uidx[(size_t)g * nloc + b];
                h_unbr[(size_t)q * P->no + o] = qi >= 0 ? h_goff[(size_t)g] + qi : -1;
            }
        }
    // group index of each packed node is needed by the pack kernel: store it in a q-indexed table
    std::vector<int32_t> h_qgroup((size_t)std::max<int64_t>(P->npacked, 1), 0);
    for (int g = 0; g < P->ngroups; ++g)
        for (int q = h_goff[(size_t)g]; q < h_goff[(size_t)g + 1]; ++q) h_qgroup[(size_t)q] = g;

    ALLOC(P->perm, ld);
    ALLOC(P->lane, Ns);
    ALLOC(P->goff, P->ngroups + 1 + std::max<int64_t>(P->npacked, 1));   // goff then q -> group
    ALLOC(P->unode, P->npacked);
    ALLOC(P->unbr, P->npacked * P->no);
    ALLOC(P->umask, P->npacked);
    ALLOC(P->uidx, (int64_t)P->ngroups * nloc);
    HCHK(hipMemcpyAsync(P->perm, h_perm.data(), h_perm.size() * 4, hipMemcpyHostToDevice, stream));
    HCHK(hipMemcpyAsync(P->lane, h_lane.data(), h_lane.size() * 4, hipMemcpyHostToDevice, stream));
    HCHK(hipMemcpyAsync(P->goff, h_goff.data(), h_goff.size() * 4, hipMemcpyHostToDevice, stream));
    HCHK(hipMemcpyAsync(P->goff + P->ngroups + 1, h_qgroup.data(), h_qgroup.size() * 4, hipMemcpyHostToDevice, stream));
    if (P->npacked > 0) {
        HCHK(hipMemcpyAsync(P->unode, h_unode.data(), h_unode.size() * 4, hipMemcpyHostToDevice, stream));
        HCHK(hipMemcpyAsync(P->unbr, h_unbr.data(), (size_t)P->npacked * P->no * 4, hipMemcpyHostToDevice, stream));
        HCHK(hipMemcpyAsync(P->umask, h_umask.data(), h_umask.size() * 8, hipMemcpyHostToDevice, stream));
    }
    HCHK(hipMemcpyAsync(P->uidx, h_uidx.data(), h_uidx.size() * 4, hipMemcpyHostToDevice, stream));
    // interleaved copies of the element masks and the local-to-global map
    ALLOC(P->keep_il, (int64_t)P->nelem * ld);
    ALLOC(P->l2g_il, nloc * ld);
    hipLaunchKernelGGL(k_interleave_u8, dim3((unsigned)lat_cdiv(ld, 256), (unsigned)P->nelem), dim3(256), 0, stream,
                       (int64_t)P->nelem, ld, Ns, P->perm, P->keep, P->keep_il);
    hipLaunchKernelGGL(k_interleave_i32, dim3((unsigned)lat_cdiv(ld, 256), (unsigned)nloc), dim3(256), 0, stream,
                       nloc, ld, P->perm, P->l2g, P->l2g_il);
    HCHK(hipGetLastError());
    // ---- workspace
    P->nchunk = lat_cdiv(P->nsnap, LAT_CHUNK);
    P->napc = (int)lat_cdiv(std::max(P->maxunion, 1), 8);           // 8 packed nodes per adjoint chunk
    int64_t tree_rows = std::max<int64_t>(lat_cdiv(std::max<int64_t>(P->nchunk, nloc), LAT_TREE), 1);
    // rows per chunk of the alpha-adjoint contractions: enough workgroups to fill the chip
    P->aa_rows = 128;
    while (P->aa_rows < 4096 && lat_cdiv(P->nsnap, P->aa_rows * 2) * lat_cdiv(ld, 256) >= 4096) P->aa_rows *= 2;
    P->aa_nchunk = lat_cdiv(P->nsnap, P->aa_rows);
    int64_t tree_elems = std::max<int64_t>(tree_rows * ld, lat_cdiv(P->napc, LAT_TREE) * ld * cap);
    tree_elems = std::max<int64_t>(tree_elems, lat_cdiv(P->aa_nchunk, LAT_TREE) * ld * cap);
    P->tree_elems = tree_elems;
    // largest walk grid: the 2D row walk (group x row x at most two segments), the 3D runs of 16 nodes
    P->nblk_lp = (int)std::max<int64_t>(std::max<int64_t>((int64_t)P->ngroups * P->nn * 2, lat_cdiv(P->npacked, 16)), 1);
    ALLOC(P->u_cil, nloc * dim * ld);
    ALLOC(P->w_part, nloc * ld);
    ALLOC(P->w_part2, nloc * ld);
    ALLOC(P->g_sq, P->nchunk * ld);
    ALLOC(P->g_inf, P->nchunk * ld);
    ALLOC(P->g_dot, P->nchunk * ld);
    ALLOC(P->g_t1, tree_elems);
    ALLOC(P->g_t2, tree_elems);
    ALLOC(P->g_t3, tree_elems);
    ALLOC(P->g_t4, tree_elems);
    ALLOC(P->v_sq, ld); ALLOC(P->v_inf, ld); ALLOC(P->v_beta, ld); ALLOC(P->v_nu, ld);
    ALLOC(P->beta_pl, ld * cap);
    ALLOC(P->zeta, LAT_GREEDY_LAG * P->nsnap);
    ALLOC(P->ictl, 64);
    ALLOC(P->dctl, 64);
    ALLOC(P->form_part, (int64_t)P->napc * ld * cap);
    ALLOC(P->form_out, ld * cap);
    ALLOC(P->form_out3, 3 * ld * cap);
    ALLOC(P->alpha_il, (int64_t)cap * ld);
    ALLOC(P->aa_A, (int64_t)cap * ld * 2);         // Z^T T_mu, Z^T T_lam   [2][ld][cap]
    ALLOC(P->aa_B, ld * cap * 2);                   // Delta^T T_S parts     [2][ld][cap]
    ALLOC(P->aa_q, (int64_t)cap * ld * 2);          // q, v                  [2][ld][cap]
    ALLOC(P->aa_gath, P->nsnap * cap);              // uniform operand       [nsnap][cap]
    ALLOC(P->aa_part, P->aa_nchunk * ld * cap);
    ALLOC(P->lp_err, 2 * (int64_t)P->nblk_lp);
    ALLOC(P->lp_gate, 8);
    HCHK(hipStreamSynchronize(stream));
#undef ALLOC
#undef HCHK
    *out = P;
    return LAT_OK;
}

lat_status lat_plan_destroy(lat_plan *plan)
{
    if (!plan) return LAT_E_ARG;
    (void)hipDeviceSynchronize();
    free_plan(plan);
    return LAT_OK;
}

lat_status lat_plan_query(const lat_plan *P, size_t *min_bytes, size_t *fast_bytes)
{
    if (!P || (!min_bytes && !fast_bytes)) return LAT_E_ARG;
    for (int c = 0; c < LAT_CALL_N; ++c) {
        size_t mn = 0, fs = 0;
        lat_ws_sizes(P, c, &mn, &fs);
        if (min_bytes) min_bytes[c] = mn;
        if (fast_bytes) fast_bytes[c] = fs;
    }
    return LAT_OK;
}

lat_status lat_plan_info(const lat_plan *P, int64_t *info)
{
    if (!P || !info) return LAT_E_ARG;
    info[LAT_INFO_DIM] = P->dim; info[LAT_INFO_NEL] = P->nel; info[LAT_INFO_NCELLS] = P->ncells;
    info[LAT_INFO_NLOC] = P->nloc; info[LAT_INFO_NELEM] = P->nelem; info[LAT_INFO_E] = P->E;
    info[LAT_INFO_NSNAP] = P->nsnap; info[LAT_INFO_LD] = P->ld; info[LAT_INFO_NGROUPS] = P->ngroups;
    info[LAT_INFO_NPACKED] = P->npacked; info[LAT_INFO_NGLOBAL] = P->nglobal; info[LAT_INFO_CAP] = P->cap;
    return LAT_OK;
}

lat_status lat_dofmap(const lat_plan *P, int32_t *l2g, int32_t *n_active, int64_t *g2bg, int32_t *perm,
                      hipStream_t stream)
{
    if (!P) return LAT_E_ARG;
    if (l2g || n_active || g2bg) {
        lat_status st = run_dofmap(P, P->dm_act, P->dm_flag, P->dm_gid, P->dm_bsum,
                                   P->dm_bsum + lat_cdiv(P->nbg, 1024), l2g, n_active, g2bg, stream);
        if (st != LAT_OK) return st;
    }
    if (perm) LAT_HIP(hipMemcpyAsync(perm, P->perm, (size_t)P->ld * 4, hipMemcpyDeviceToDevice, stream));
    return LAT_OK;
}

lat_status lat_pack(const lat_plan *P, const double *canon, double *packed, int32_t m, hipStream_t stream)
{
    if (!P || !canon || !packed || m < 1) return LAT_E_ARG;
    int64_t tot = P->npacked * P->dim * m * LAT_WAVE;
    if (tot == 0) return LAT_OK;
    hipLaunchKernelGGL(k_pack, dim3((unsigned)lat_cdiv(tot, 256)), dim3(256), 0, stream, P->dim, m, (int64_t)P->nloc,
                       P->npacked, P->perm, P->goff + P->ngroups + 1, P->unode, P->l2g, canon, packed);
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

lat_status lat_unpack(const lat_plan *P, const double *packed, double *canon, int32_t m, hipStream_t stream)
{
    if (!P || !canon || !packed || m < 1) return LAT_E_ARG;
    int64_t tot = P->ncells * P->nloc * P->dim * m;
    hipLaunchKernelGGL(k_unpack, dim3((unsigned)lat_cdiv(tot, 256)), dim3(256), 0, stream, P->dim, m, (int64_t)P->nloc,
                       P->ncells, P->lane, P->uidx, P->goff, P->l2g, packed, canon);
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

static dim3 rows_grid(int64_t ld, int64_t rows)
{
    return dim3((unsigned)lat_cdiv(ld, 256), (unsigned)std::min<int64_t>(rows, 65535), (unsigned)lat_cdiv(rows, 65535));
}

lat_status lat_cil_to_canon(const lat_plan *P, const double *cil, int64_t k, double *canon, hipStream_t stream)
{
    if (!P || !cil || !canon || k < 1) return LAT_E_ARG;
    hipLaunchKernelGGL(k_cil_to_canon, rows_grid(P->ld, P->nloc * k), dim3(256), 0, stream, (int64_t)P->nloc, k, P->ld,
                       P->perm, cil, canon);
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

lat_status lat_canon_to_cil(const lat_plan *P, const double *canon, int64_t k, double *cil, hipStream_t stream)
{
    if (!P || !cil || !canon || k < 1) return LAT_E_ARG;
    hipLaunchKernelGGL(k_canon_to_cil, rows_grid(P->ld, P->nloc * k), dim3(256), 0, stream, (int64_t)P->nloc, k, P->ld,
                       P->perm, canon, cil);
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

lat_status lat_plain_ops_to_canon(const lat_plan *P, const double *ops, double *canon, hipStream_t stream)
{
    if (!P || !ops || !canon) return LAT_E_ARG;
    int64_t tot = P->ncells * P->nloc * P->E;
    hipLaunchKernelGGL(k_plain_to_canon, dim3((unsigned)lat_cdiv(tot, 256)), dim3(256), 0, stream, P->E,
                       (int64_t)P->nloc, P->ncells, P->lane, P->uidx, P->goff, ops, canon);
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

lat_status lat_assemble(const lat_plan *P, const double *local, int32_t k, double *out, hipStream_t stream)
{
    if (!P || !local || !out || k < 1 || k > 3) return LAT_E_ARG;
    Grid g = make_grid(P);
    hipLaunchKernelGGL(k_assemble, dim3((unsigned)lat_cdiv(P->nglobal, 256)), dim3(256), 0, stream, g, P->nglobal, k,
                       P->ld, P->g2bg, P->l2g, P->lane, local, out);
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

lat_status lat_gather(const lat_plan *P, const double *global, int32_t k, double *local, hipStream_t stream)
{
    if (!P || !global || !local || k < 1) return LAT_E_ARG;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)lat_cdiv(P->ld, 256), (unsigned)P->nloc), dim3(256), 0, stream, k, P->ld,
                       P->l2g_il, global, local);
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

}  // extern "C"

void lat_ws_sizes(const lat_plan *P, int call, size_t *min_bytes, size_t *fast_bytes)
{
    lat_plan V = *P;
    WsItem it[32];
    const int n = ws_items(P, &V, call, it);
    size_t mn = 0, fs = 0, last = 0;
    for (int t = 0; t < n; ++t) {
        const size_t b = ws_align(it[t].bytes);
        if (it[t].fast == 0) { mn += b; fs += b; }
        else if (it[t].fast == 1) { fs += b; last = b; }
        else if (b > last) { fs += b - last; last = b; }
    }
    *min_bytes = mn;
    *fast_bytes = fs;
}

size_t lat_forms_batch_bytes(const lat_plan *P, int64_t lanes)
{
    return ((size_t)P->nsnap * lanes * 8 + 255) / 256 * 256 +
           ((size_t)3 * P->aa_nchunk * lanes * P->cap * 8 + 255) / 256 * 256;
}

lat_status lat_ws_bind(const lat_plan *P, int call, void *work, size_t work_bytes, lat_plan *V)
{
    *V = *P;
    WsItem it[32];
    const int n = ws_items(P, V, call, it);
    V->ws_rest = nullptr;
    V->ws_rest_bytes = 0;
    if (!work) {
        // the plan's own scratch; it holds none of the buffers that only a fast workspace brings
        for (int t = 0; t < n; ++t)
            if (it[t].fast && it[t].ptr) *it[t].ptr = nullptr;
        return LAT_OK;
    }
    if (((uintptr_t)work & 255) != 0) return LAT_E_ARG;
    size_t mn = 0, fs = 0;
    lat_ws_sizes(P, call, &mn, &fs);
    if (work_bytes < mn) return LAT_E_SHAPE;
    const bool fast = work_bytes >= fs;
    char *base = (char *)work;
    size_t off = 0, last_off = 0;
    for (int t = 0; t < n; ++t) {
        if (!it[t].ptr) continue;                      // carved by the call from the rest
        if (it[t].fast && !fast) { *it[t].ptr = nullptr; continue; }
        if (it[t].fast == 2) { *it[t].ptr = base + last_off; continue; }
        *it[t].ptr = base + off;
        last_off = off;
        off += ws_align(it[t].bytes);
    }
    if (work_bytes > off) {
        V->ws_rest = base + off;
        V->ws_rest_bytes = work_bytes - off;
    }
    return LAT_OK;
}

