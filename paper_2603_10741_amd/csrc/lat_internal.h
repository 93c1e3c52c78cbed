// Internal definitions shared by the liblat HIP sources (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <vector>

#include "lat.h"

#define LAT_WAVE 64
#define LAT_CHUNK 256          // rows per fixed-order dot-product chunk
#define LAT_TREE 256           // rows reduced per tree-kernel launch
#define LAT_MAX_CAP 64

// The greedy writes its residuals back every LAT_GREEDY_LAG iterations; the passes in between
// replay the pending updates on load (the basis rows they need are kept in a ring of this length).
constexpr int LAT_GREEDY_LAG = 8;

struct lat_plan {
    int dim, nel, nn, nloc, nelem, no, E, nc;
    int ncell[3];
    int64_t ncells, nglobal, nsnap, ld, npacked, nbg;
    int ngroups, cap, device;
    int64_t nchunk;            // greedy dot-product chunks over the snapshot rows
    int maxunion;              // largest union of active nodes in a group
    int napc;                  // node chunks per group for the adjoint forms
    // device tables (immutable after creation)
    uint8_t *keep = nullptr;       // [N_s][nelem] canonical
    uint8_t *keep_il = nullptr;    // [nelem][ld]
    int32_t *perm = nullptr;       // [ld] lane -> canonical cell / -1
    int32_t *lane = nullptr;       // [N_s] canonical cell -> lane
    int32_t *l2g = nullptr;        // [N_s][nloc]
    int32_t *l2g_il = nullptr;     // [nloc][ld]
    int32_t *nact = nullptr;       // [N_s]
    int64_t *g2bg = nullptr;       // [nglobal]
    uint8_t *dm_act = nullptr;     // DOF-map scratch: [N_s][nloc] active flags
    int32_t *dm_flag = nullptr;    // [nbg] background flags
    int32_t *dm_gid = nullptr;     // [nbg] scan output
    int32_t *dm_bsum = nullptr;    // [nbg/1024 + 1] block sums + total
    int32_t *goff = nullptr;       // [ngroups+1] packed-node offsets of the groups
    int32_t *unode = nullptr;      // [npacked] local node of each packed node
    int32_t *unbr = nullptr;       // [npacked][no] packed neighbour (a+o) or -1
    uint64_t *umask = nullptr;     // [npacked] lanes owning the node
    int32_t *uidx = nullptr;       // [ngroups][nloc] packed index within the group or -1
    // workspace (device)
    double *u_cil = nullptr;       // [nloc][dim][ld]
    double *w_part = nullptr;      // [nloc][ld] per-node partials (energy, adjoint dots)
    double *w_part2 = nullptr;     // [nloc][ld]
    double *g_sq = nullptr;        // [nchunk][ld]
    double *g_inf = nullptr;       // [nchunk][ld]
    double *g_dot = nullptr;       // [nchunk][ld]
    double *g_t1 = nullptr;        // [ceil(max(nchunk,nloc)/256)][ld] tree scratch
    double *g_t2 = nullptr;
    double *g_t3 = nullptr, *g_t4 = nullptr;   // second-array tree scratch
    double *v_sq = nullptr, *v_inf = nullptr, *v_beta = nullptr, *v_nu = nullptr;   // [ld]
    double *beta_pl = nullptr;     // [ld][cap] plan-order coordinates
    double *zeta = nullptr;        // [LAT_GREEDY_LAG][nsnap] ring of the latest basis rows
    int32_t *ictl = nullptr;       // small control block: done, sel lane, n_r, ...
    double *dctl = nullptr;        // rho, achieved, ...
    double *form_part = nullptr;   // [napc][ld][cap] adjoint form partials
    double *form_out = nullptr;    // [ld][cap]
    double *form_out3 = nullptr;   // [3][ld][cap] forms of up to three stacks (ROM adjoint)
    double *alpha_il = nullptr;    // [cap][ld] interleaved RB coefficients
    double *aa_A = nullptr;        // [cap][ld] alpha-adjoint products
    double *aa_B = nullptr;        // [ld][cap]
    double *aa_q = nullptr;        // [2][ld][cap] q = R^{-T} alpha_bar, v = R^{-1} q
    double *aa_gath = nullptr;     // [nsnap][cap] uniform operand (Z^T or principal columns)
    double *aa_part = nullptr;     // partials for the alpha adjoint
    int64_t aa_nchunk = 0;
    int aa_rows = 4096;            // snapshot rows per alpha-adjoint chunk
    int64_t tree_elems = 0;        // size of each tree scratch array (g_t1 .. g_t4)
    int nblk_lp = 0;               // largest grid of a walk kernel (per-block error partials)
    // reduced-precision ROM apply: the FP64-measured error estimate and the refinement gates
    double *lp_err = nullptr;      // [nblk_lp][2] per-block (sum |K~ - K~64|^2, sum |K~64|^2)
    int32_t *lp_gate = nullptr;    // [8] refinement gates (1 = the next, more precise pass runs)
    // adjoint forms: W[(a, e)][lane] = sum_r Ybar X (FP64, or FP32 in w_forms32), and the alpha
    // adjoint's second uniform operand; only in a caller workspace of the "fast" size
    double *wf_part = nullptr;     // alpha adjoint: [2][aa_nchunk][ld][cap] contraction partials
    double *aa_gath2 = nullptr;    // [nsnap][cap]
    // the part of a caller workspace past the call's minimum (the ROM adjoint carves its W batches
    // and their contraction partials from it)
    char *ws_rest = nullptr;
    size_t ws_rest_bytes = 0;
};

// ---- bf16 slices (reduced-precision combination on the bf16 matrix cores)
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 lat_bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(short)))) short lat_s16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float lat_f32x4;

// round-to-nearest-even bf16 of a float (bit pattern)
__device__ __forceinline__ uint16_t lat_to_bf16(float x)
{
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ double lat_from_bf16(uint16_t b) { return (double)__uint_as_float((uint32_t)b << 16); }

// three bf16 slices of x with FP64 remainders: x ~ s0 + s1 + s2
__device__ __forceinline__ void lat_slice3(double x, uint16_t s[3])
{
    double r = x;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        s[t] = lat_to_bf16((float)r);
        r -= lat_from_bf16(s[t]);
    }
}

#define LAT_HIP(call)                                                        \
    do {                                                                     \
        hipError_t e_ = (call);                                              \
        if (e_ != hipSuccess) {                                              \
            std::fprintf(stderr, "liblat: %s failed: %s (%s:%d)\n", #call,   \
                         hipGetErrorString(e_), __FILE__, __LINE__);         \
            return LAT_E_DEVICE;                                             \
        }                                                                    \
    } while (0)

#define LAT_LAUNCH_CHECK() LAT_HIP(hipGetLastError())

static inline int lat_ipow(int b, int e) { int r = 1; while (e-- > 0) r *= b; return r; }
static inline int64_t lat_cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).  This maps the
// hardware block index to a logical one so that every XCD receives a contiguous range of logical
// blocks: neighbouring node chunks, whose stencils read the same vector entries, share an L2.
// A bijection on [0, n).
__device__ __forceinline__ int lat_xcd_block(int b, int n)
{
    const int q = n >> 3, r = n & 7, x = b & 7, s = b >> 3;
    return x * q + (x < r ? x : r) + s;
}

// Device status word helpers.  The code word keeps the most severe code raised so far: OK below the
// cap warning below every error (among errors, the larger code), so a warning raised after an
// error never hides it.  The cell word keeps the lowest canonical id of a cell that raised an
// error (warnings carry no cell).
__device__ __forceinline__ int lat_severity(int code)
{
    return code == LAT_OK ? 0 : (code == LAT_W_CAP ? 1 : 2 + code);
}
__device__ inline void lat_flag(int32_t *st, int code, int cell)
{
    if (!st) return;
    int old = __hip_atomic_load(&st[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (lat_severity(code) > lat_severity(old)) {
        const int prev = atomicCAS(&st[0], old, code);
        if (prev == old) break;
        old = prev;
    }
    if (code != LAT_W_CAP) atomicMin(&st[1], cell);
}

// Caller workspaces (defined in lat_plan.hip).  A call's scratch is carved from `work` into a copy
// of the plan (*V = *P with its scratch pointers moved into work); the kernels read the copy.
// work == NULL: V keeps the plan's own scratch (no "fast"-only buffers).  LAT_E_SHAPE when
// work_bytes is below the call's minimum, LAT_E_ARG when work is not 256-byte aligned.
lat_status lat_ws_bind(const lat_plan *P, int call, void *work, size_t work_bytes, lat_plan *V);
void lat_ws_sizes(const lat_plan *P, int call, size_t *min_bytes, size_t *fast_bytes);
// bytes of the ROM adjoint's W (FP64) and three-stack contraction partials for `lanes` plan lanes
size_t lat_forms_batch_bytes(const lat_plan *P, int64_t lanes);

// Shared internal launches (defined in lat_greedy.hip).
// Pairwise-tree reduction over rows of in [nrows][ld] (row-major, lanes fastest), applying
// sum (op 0) or max (op 1); result [ld] in out.  Uses t1/t2 as scratch ([ceil(nrows/256)][ld]).
lat_status lat_tree_reduce(const double *in, int64_t nrows, int64_t ld, int op, double *out, double *t1,
                           double *t2, hipStream_t s);

// Row contraction out[p][k] = sum_j V[j][p] U[j][k] over the n_snap snapshot rows, V [nsnap][ld]
// (FP64 in V, or FP32 in V32: exactly one of them is non-NULL; the products and sums are FP64),
// U [nsnap][cap] (a principal stack), out [ld][cap] in plan order; fixed-order chunk partials and
// tree (defined in lat_adjoint.hip).
lat_status lat_contract_rows(const lat_plan *P, int n_r, const double *V, const float *V32, const double *U,
                             double *out, hipStream_t s);
// The same for ns (1..3) stacks in one pass over V (n_r <= 32, cap >= 16): chunk partials
// part[t] [aa_nchunk][ld][cap], to be reduced by lat_tree_reduce.
lat_status lat_contract_rows_multi(const lat_plan *P, int n_r, const double *V, const float *V32,
                                   const double *const *U, int ns, double *const *part, hipStream_t s);

// Combined stencils of every cell, sum_k alpha_sk K_k, in lat_apply_plain's packed operator layout
// (defined in lat_newton.hip).
lat_status lat_combine_ops(const lat_plan *P, const double *K, int n_r, const double *alpha, double *ops, hipStream_t s);
