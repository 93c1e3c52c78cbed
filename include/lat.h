/*
 * lat.h -- C ABI of the MI355X principal-cell lattice library (liblat.so, gfx950).
 *
 * The library implements, on one GPU, the data-parallel hot path of the reduced-order
 * lattice solver of "Efficient Fine-Scale Simulation of Nonlinear Hyperelastic Lattice
 * Structures" (Sec. 3.1-3.2):
 *   - local-to-global DOF maps of voxelised unit cells           (eq. residualvector)
 *   - per-cell neo-Hookean residual, energy and tangent          (eq. internalloadvec,
 *     Sec. 3.1.4, eq. fullquadraturerule, eq. snapshots)
 *   - greedy selection of principal cells and RB coefficients    (Algorithm 1, Sec. 3.2.2)
 *   - the ROM operator apply Y_i = sum_k alpha_ik K_k X_i         (eq. romstiffnessmatrix)
 *   - the plain per-cell apply Y_i = K_i X_i (the standard operator, Sec. 3.1.4)
 *   - reverse-mode (adjoint) forms of the residual and of the ROM apply
 *   - the load-stepped Newton-Raphson solve on the ROM tangent with Armijo backtracking and its
 *     matrix-free preconditioned MINRES tangent solves                 (Sec. 2.2.5, eq. linsys).
 *
 * General conventions
 *   - Every array argument is a DEVICE pointer owned by the caller, unless its comment says
 *     HOST.  The library never frees or keeps caller memory.
 *   - Every call is enqueued on the given HIP stream and returns without waiting, unless
 *     stated otherwise.  Argument and shape errors are detected on the host and returned
 *     synchronously; nothing is enqueued then.
 *   - Data-dependent failures (an inverted element, a non-finite value) and the greedy's cap
 *     warning are written to a caller-provided device status word `dev_status` int32[2] =
 *     {code, first bad cell} (initialise it with lat_status_reset); the caller reads it after
 *     synchronising.  The code word keeps the most severe code raised since the reset: LAT_OK,
 *     then LAT_W_CAP, then any error (LAT_E_INVERTED < LAT_E_NONFINITE), so a later warning never
 *     hides an error; the cell word keeps the lowest canonical id of a cell that raised an error
 *     (INT32_MAX when none did).
 *   - Scratch.  A plan owns immutable tables and a default scratch workspace.  Every stream-ordered
 *     call that needs scratch takes `work` / `work_bytes`: a caller device buffer (256-byte
 *     aligned) of at least the call's minimum size from lat_plan_query, or NULL for the plan's
 *     default workspace.  Calls with NULL work on one plan must not overlap in time (one stream
 *     per plan, or synchronise); calls with distinct caller workspaces may run concurrently on
 *     different streams.  The library keeps no pointer to `work` after the call's kernels end.
 *     A workspace of the "fast" size enables the faster variants named at each call.
 *   - Principal-cell arrays: every array documented below as [..][cap] or [cap] uses the PLAN's
 *     cap as its stride, i.e. LAT_INFO_CAP from lat_plan_info (the cap given to lat_plan_create
 *     rounded up to a power of two >= 8), whatever cap a later call passes.
 *   - Indices are 0-based.  Geometry: cell edge 1, n Q1 elements per cell axis, h = 1/n;
 *     element e = ex + n(ey + n ez); local node a = ix + (n+1)(iy + (n+1) iz); element
 *     corners x-fastest; cells numbered x-fastest over the lattice ("canonical" order).
 *   - Stencil entry index e = ((o * d) + i) * d + j with offset index
 *     o = (ox+1) + 3(oy+1) + 9(oz+1); entry (a, o, i, j) = K[(a,i),(a+o,j)].  E = 3^d d^2.
 *
 * Layouts defined by a plan (query the sizes with lat_plan_info):
 *   plan lanes   cells are sorted by a mask-similarity key and grouped 64 at a time;
 *                plan lane p = 64 g + l (group g, lane l); ld = 64 * n_groups; the map
 *                lane -> canonical cell (or -1 for padding) is returned by lat_dofmap.
 *   CIL(k)       cell-interleaved local field: element (a, c) of cell s at
 *                [(a * k + c) * ld + lane(s)], a < (n+1)^d, c < k.  The snapshot matrix T is
 *                CIL(E): row index (a, e) = the canonical snapshot index, column = lane.
 *   packed       operator-apply vectors: for group g the union of its cells' active nodes
 *                (n_packed nodes in total); element (node q, i, r, l) at
 *                [((q * d + i) * m + r) * 64 + l].  Entries at DOFs a cell does not own are
 *                ignored on input and written as 0 on output.
 *   plain ops    per-cell stencils in packed form: [(q * E + e) * 64 + l].
 *   principal    stack of principal stencils: [(a * E + e) * cap + k], a over all (n+1)^d
 *                local nodes, k < cap principal slots (slots >= n_r hold zeros).
 */
#ifndef LAT_H
#define LAT_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LAT_OK = 0,
    LAT_E_ARG = 1,        /* bad argument (null pointer, out-of-range value) */
    LAT_E_SHAPE = 2,      /* sizes inconsistent with the plan */
    LAT_E_DEVICE = 3,     /* a HIP runtime call failed */
    LAT_E_NOMEM = 4,      /* device allocation failed */
    LAT_E_INVERTED = 5,   /* (device status) J <= 0 at a Gauss point */
    LAT_E_NONFINITE = 6,  /* (device status) non-finite displacement or Jacobian */
    LAT_W_CAP = 7,        /* (device status) greedy stopped at the cap above the tolerance */
    LAT_E_NOCONV = 8,     /* an iterative solve stopped at its iteration limit */
    LAT_E_SINGULAR = 9    /* the tangent solve met an operator singular on its Krylov space */
} lat_status;

/* snapshot data: the assembled cell tangent with 2^d Gauss points / with 1 point per element, the
 * material tangent dP/dF at the centre of every kept element, or the full-rule tangent's entries at
 * a sub-grid of local nodes (see lat_residual_tangent) */
typedef enum { LAT_RULE_FULL = 0, LAT_RULE_REDUCED = 1, LAT_RULE_MATERIAL = 2, LAT_RULE_SAMPLED = 3 } lat_rule;
/* node stride of LAT_RULE_SAMPLED: the local nodes whose every coordinate is a multiple of it */
#define LAT_SAMPLE_STRIDE 2
typedef enum { LAT_F64 = 0, LAT_F32 = 1, LAT_BF16 = 2 } lat_prec;

typedef struct lat_plan lat_plan;

/* The calls that take a caller workspace (index of lat_plan_query's arrays). */
typedef enum {
    LAT_CALL_RESIDUAL_TANGENT = 0,   /* lat_residual_tangent */
    LAT_CALL_PRINCIPAL_OPS = 1,      /* lat_principal_ops */
    LAT_CALL_SELECT_PRINCIPAL = 2,   /* lat_select_principal, lat_select_principal_rows */
    LAT_CALL_APPLY_COMBO = 3,        /* lat_apply_combo */
    LAT_CALL_APPLY_COMBO_ADJOINT = 4,/* lat_apply_combo_adjoint */
    LAT_CALL_ALPHA_ADJOINT = 5,      /* lat_alpha_adjoint */
    LAT_CALL_RESIDUAL_ADJOINT = 6,   /* lat_residual_adjoint */
    LAT_CALL_N = 7
} lat_call;

enum {
    LAT_INFO_DIM = 0, LAT_INFO_NEL, LAT_INFO_NCELLS, LAT_INFO_NLOC, LAT_INFO_NELEM, LAT_INFO_E,
    LAT_INFO_NSNAP, LAT_INFO_LD, LAT_INFO_NGROUPS, LAT_INFO_NPACKED, LAT_INFO_NGLOBAL, LAT_INFO_CAP,
    LAT_INFO_N
};

/* Human-readable text of a status code (static storage). */
const char *lat_status_string(lat_status s);

/* Builds a plan for a lattice of ncell[0] x ncell[1] (x ncell[2]) congruent cells of
 * nel^dim Q1 elements.  keep_host: HOST uint8 [N_s][nel^dim], 1 = element kept.
 * cap: maximum number of principal cells any later call will use (1..64); the plan rounds it up
 * to a power of two >= 8 (LAT_INFO_CAP), the stride of every principal-cell array.
 * Runs the DOF-map kernels (active nodes, global numbering, local-to-global maps;
 * eq. residualvector) on `stream`, then derives the plan's lane grouping and packed
 * layout on the host.  Synchronises `stream`.  Allocates device memory.
 * On error *out is NULL. */
lat_status lat_plan_create(int32_t dim, const int32_t ncell[3], int32_t nel, const uint8_t *keep_host,
                           int32_t cap, hipStream_t stream, lat_plan **out);
lat_status lat_plan_destroy(lat_plan *plan);
/* info: HOST int64[LAT_INFO_N], filled with the sizes above. */
lat_status lat_plan_info(const lat_plan *plan, int64_t *info);

/* Workspace sizes in bytes of every call that takes one (HOST size_t[LAT_CALL_N] each, either may
 * be NULL): min_bytes[c] is the least `work_bytes` call c accepts (below it the call returns
 * LAT_E_SHAPE), fast_bytes[c] >= min_bytes[c] the size from which the call's faster variant runs.
 * The sizes depend on the plan only. */
lat_status lat_plan_query(const lat_plan *plan, size_t *min_bytes, size_t *fast_bytes);

/* Writes {LAT_OK, INT32_MAX} to the device status word. */
lat_status lat_status_reset(int32_t *dev_status, hipStream_t stream);

/* DOF maps (eq. residualvector; A^s is the Boolean matrix of l2g).  Recomputes them from the
 * plan's element masks with the DOF-map kernels.  Outputs (any may be NULL):
 *   l2g      int32 [N_s][(n+1)^d]  global active-node id of local node a of cell s, or -1
 *   n_active int32 [N_s]           number of active local nodes per cell
 *   g2bg     int64 [n_global]      background-grid id of each global node (lexicographic over
 *                                  the lattice's (C_x n+1) x ... node grid, x fastest)
 *   perm     int32 [ld]            canonical cell of each plan lane, -1 for padding lanes */
lat_status lat_dofmap(const lat_plan *plan, int32_t *l2g, int32_t *n_active, int64_t *g2bg, int32_t *perm,
                      hipStream_t stream);

/* Residual, energy and tangent of every cell at the global displacement
 * u_global [n_global][d] (u^s = A^{sT} u), per-cell Lame parameters mu, lam [N_s] (canonical).
 * Material-form neo-Hookean law W = mu/2 (I1-3) - mu ln J + lam/2 (ln J)^2 (plane strain in 2D).
 * Outputs (any may be NULL):
 *   f_int     CIL(d)   internal force f^{int,s} (eq. internalloadvec), cell-local, full rule
 *   energy    [N_s]    stored energy per cell (canonical order), full rule
 *   snap      CIL(E)   snapshot matrix T: the assembled cell tangent in stencil layout
 *                      (eq. snapshots), quadrature `snap_rule` (FULL or REDUCED); or, with
 *                      LAT_RULE_MATERIAL, the material tangent A = dP/dF at the centre of every
 *                      kept element (the Remark on snapshots of Sec. 3.2.2), A_iJkL of element e in
 *                      row (e d^2 + i d + J) d^2 + k d + L, zeros for elements not kept and for the
 *                      rows past n^d d^4; or, with LAT_RULE_SAMPLED, a limited set of entries of the
 *                      full-rule tangent (the some_data(K) choice of the same Remark): the complete
 *                      stencil rows (3^d d^2 entries) of the nodes of the sub-grid of stride
 *                      LAT_SAMPLE_STRIDE, node j (lexicographic, x fastest) in rows j 3^d d^2 ...,
 *                      zeros past them; those rows equal the FULL snapshot's rows of the same node
 *                      bit for bit
 *   plain_ops packed   every cell's full-rule tangent in stencil form (for lat_apply_plain)
 * Errors J <= 0 (LAT_E_INVERTED) / a non-finite displacement or Jacobian (LAT_E_NONFINITE) go to
 * dev_status with the cell; the outputs of such a cell are then undefined.
 * work: LAT_CALL_RESIDUAL_TANGENT workspace or NULL (see the conventions). */
lat_status lat_residual_tangent(const lat_plan *plan, const double *u_global, const double *mu, const double *lam,
                                lat_rule snap_rule, double *f_int, double *energy, double *snap, double *plain_ops,
                                int32_t *dev_status, void *work, size_t work_bytes, hipStream_t stream);

/* Number of leading snapshot rows that `rule` can make nonzero (the rest of the n_snap rows are
 * zero): n_snap for FULL / REDUCED, n^d d^4 for MATERIAL, ((n / LAT_SAMPLE_STRIDE) + 1)^d 3^d d^2 for
 * SAMPLED; the `rows` argument of lat_select_principal_rows.  -1 for a NULL plan or unknown rule. */
int64_t lat_snapshot_rows(const lat_plan *plan, lat_rule rule);

/* Principal operators K^r = K^{s_r}(u^{s_r}) (eq. reducedbasis), full rule, in the principal
 * stack layout, for the cells S[0..n_r) (device int32 [cap], canonical ids; n_r <= cap is a
 * HOST value).  K = mu K_mu + lam K_lam at fixed u; K_mu / K_lam (may be NULL) receive those
 * parts, for the adjoint.  Slots k >= n_r are zeroed.  LAT_E_SHAPE when n_r > LAT_INFO_CAP.
 * work: LAT_CALL_PRINCIPAL_OPS workspace or NULL. */
lat_status lat_principal_ops(const lat_plan *plan, const double *u_global, const double *mu, const double *lam,
                             const int32_t *S, int32_t n_r, double *K, double *K_mu, double *K_lam,
                             int32_t *dev_status, void *work, size_t work_bytes, hipStream_t stream);

/* Greedy selection of principal cells (Algorithm 1) on the snapshot matrix `snap` (CIL(E),
 * overwritten by the residuals Delta), tolerance tol > 0, at most cap <= plan cap selections.
 * Ties of the arg-max go to the lowest canonical cell id; a zero snapshot is never selected.
 * Dot products use a fixed order: chunks of 256 consecutive snapshot entries accumulated by
 * fma from 0, chunk sums combined by a pairwise tree; so results are reproducible bit for bit.
 * Outputs (device):
 *   S        int32 [cap]      principal cells (canonical ids), -1 past n_r
 *   n_r      int32 [1]        number selected
 *   alpha    f64 [N_s][cap]   RB coefficients (least-squares coordinates, via R alpha = nu beta)
 *   beta     f64 [N_s][cap]   greedy coordinates beta_i^s              (may be NULL)
 *   nu       f64 [N_s]        snapshot 2-norms                           (may be NULL)
 *   R        f64 [cap][cap]   R[j][k] = nu_{s_k} beta_j^{s_k}, j <= k
 *   Z        f64 [cap][n_snap] orthonormal basis zeta_i                   (may be NULL)
 *   achieved f64 [1]          max_s ||Delta^s||_inf at exit
 * LAT_W_CAP goes to dev_status when the cap stops the loop above tol.  The arrays' cap dimension is
 * the plan's LAT_INFO_CAP; the argument cap (1..LAT_INFO_CAP, else LAT_E_SHAPE) only limits the
 * number of selections.  work: LAT_CALL_SELECT_PRINCIPAL workspace or NULL. */
lat_status lat_select_principal(const lat_plan *plan, double *snap, double tol, int32_t cap, int32_t *S,
                                int32_t *n_r, double *alpha, double *beta, double *nu, double *R, double *Z,
                                double *achieved, int32_t *dev_status, void *work, size_t work_bytes,
                                hipStream_t stream);

/* lat_select_principal on the first `rows` snapshot rows only (1 <= rows <= n_snap): for snapshots
 * whose rows past `rows` are zero (lat_snapshot_rows of their rule) the outputs equal those
 * of lat_select_principal bit for bit (the chunk sums and pairwise trees take a zero chunk
 * exactly), at the cost of the rows read.  Rows past `rows` are neither read nor written; Z keeps
 * its [cap][n_snap] layout with zeros there. */
lat_status lat_select_principal_rows(const lat_plan *plan, double *snap, int64_t rows, double tol, int32_t cap,
                                     int32_t *S, int32_t *n_r, double *alpha, double *beta, double *nu, double *R,
                                     double *Z, double *achieved, int32_t *dev_status, void *work,
                                     size_t work_bytes, hipStream_t stream);

/* ROM apply (eq. romstiffnessmatrix): Y_i = M_i (sum_k alpha_ik K_k) M_i X_i for every cell at
 * once, M_i the active-DOF mask of cell i.  K: a stack of n_r stencils in the principal stack
 * layout (cap slots) -- the principal tangents from lat_principal_ops with alpha the RB
 * coefficients, or the greedy's orthonormal basis with its coefficients (lat_basis_stack), which
 * is the same operator when the snapshots use the full rule.  n_r is a HOST value
 * (0..LAT_INFO_CAP, else LAT_E_SHAPE), alpha [N_s][cap] canonical, X and Y packed with m >= 1
 * right-hand sides; transpose != 0 applies the transposed operator.  X and Y are FP64 for every
 * prec, and so is the apply of the combined stencil to X; prec selects the precision of the
 * combination sum_k alpha_ik K_k (the dense contraction over the principal cells):
 *   LAT_F64   FP64 (FP64 matrix cores);
 *   LAT_F32   operands rounded to FP32 on the FP32 matrix cores;
 *   LAT_BF16  operands split into bf16 slices x = x0 + x1 + x2 (remainders formed in FP64), slice
 *             products grouped in levels p + q (each level about 2^-8 below the one before) on the
 *             bf16 matrix cores with FP32 accumulation per level and FP64 sums of the levels;
 *             1, 2 or 3 levels to start with, as refine_tol >= 2^-8, >= 2^-16 or less.
 * FP64-measured refinement (F32 / BF16): every pass forms the combination of one node (2D) or
 * one stencil slice (3D) per workgroup a second time in FP64 and measures the relative
 * Frobenius difference over all of them; when it exceeds refine_tol (>= 0, else LAT_E_ARG) the
 * apply runs again with one more bf16 level, and after the third level (or after FP32) with the
 * FP64 combination.  The decisions are taken on the device (no host synchronisation).
 * err_est (device double, may be NULL) receives the estimate of the pass that stood: the relative
 * error of the combined operator against its FP64 value at the sampled nodes, 0 for LAT_F64 and
 * when the FP64 combination ran.
 * work: LAT_CALL_APPLY_COMBO workspace or NULL. */
lat_status lat_apply_combo(const lat_plan *plan, const double *K, int32_t n_r, const double *alpha,
                           const double *X, double *Y, int32_t m, lat_prec prec, double refine_tol,
                           int32_t transpose, double *err_est, void *work, size_t work_bytes, hipStream_t stream);

/* lat_apply_combo for callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the same operation, arguments and results, with
 * the call's scratch in a fixed device array of LAT_NOALLOC_SCRATCH_BYTES that the library holds
 * on every GPU it runs on until the process ends (no allocation, no workspace argument).  The
 * current device must be the plan's (else LAT_E_ARG).  LAT_E_SHAPE when the call's scratch
 * (lat_plan_query's minimum for LAT_CALL_APPLY_COMBO: 8 cap ld bytes of coefficients plus the
 * refinement's per-block partials) exceeds the array.  Every call on one GPU shares that GPU's
 * array: calls that overlap in time on one GPU (other streams, other threads) race and must not
 * be issued. */
#define LAT_NOALLOC_SCRATCH_BYTES (16u << 20)
lat_status lat_apply_combo_noalloc(const lat_plan *plan, const double *K, int32_t n_r, const double *alpha,
                                   const double *X, double *Y, int32_t m, lat_prec prec, double refine_tol,
                                   int32_t transpose, double *err_est, hipStream_t stream);

/* The greedy's orthonormal basis as a ROM stack: stack[(a E + e) cap + k] = Z[k][(a, e)] and
 * coefficients coef[s][k] = nu_s beta_k^s (the certified decomposition of Algorithm 1), k < n_r
 * (HOST value), zero beyond.  Z [cap][n_snap], nu [N_s], beta [N_s][cap] from
 * lat_select_principal; stack [(n+1)^d][E][cap], coef [N_s][cap]. */
lat_status lat_basis_stack(const lat_plan *plan, const double *Z, const double *nu, const double *beta,
                           int32_t n_r, double *stack, double *coef, hipStream_t stream);

/* Plain per-cell apply Y_i = M_i K_i M_i X_i with every cell's own full-rule tangent
 * (plain_ops from lat_residual_tangent).  X, Y packed. */
lat_status lat_apply_plain(const lat_plan *plan, const double *plain_ops, const double *X, double *Y, int32_t m,
                           hipStream_t stream);

/* Adjoint of the ROM apply for a cotangent Ybar (packed), with S frozen:
 *   Xbar      packed            Xbar_i = M_i Ktilde_i^T M_i Ybar_i               (may be NULL)
 *   alpha_bar f64 [N_s][cap]    alpha_bar_ik = <M_i Ybar_i, K_k M_i X_i>          (may be NULL)
 *   mu_bar, lam_bar f64 [N_s]   the part through the principal tangents:
 *                               lam/mu_bar_{s_k} = sum_i alpha_ik <Ybar_i, K_{mu/lam,k} X_i>
 *                               (written, not accumulated; zero for non-principal cells).
 *                               Requires K_mu / K_lam from lat_principal_ops and S.
 * prec / refine_tol / err_est: the precision of Xbar's combination, as for lat_apply_combo (its
 * transposed apply).  The forms <Ybar_i, K_k X_i> are sums of products of FP64 data; with room in
 * the workspace past its minimum they are taken from the cells' W[(a, e)] = sum_r Ybar X, held in
 * FP64 (LAT_F64) or FP32 (LAT_F32 / LAT_BF16), by one contraction per stack on the FP64 matrix
 * cores, in batches of as many 64-lane groups as that room holds (the fast size holds every lane at
 * once; below one group's worth, a fused per-node kernel in FP64 serves).
 * work: LAT_CALL_APPLY_COMBO_ADJOINT workspace or NULL (the fused kernel then). */
lat_status lat_apply_combo_adjoint(const lat_plan *plan, const double *K, const double *K_mu, const double *K_lam,
                                   const int32_t *S, int32_t n_r, const double *alpha, const double *X,
                                   const double *Ybar, int32_t m, double *Xbar, double *alpha_bar, double *mu_bar,
                                   double *lam_bar, lat_prec prec, double refine_tol, double *err_est, void *work,
                                   size_t work_bytes, hipStream_t stream);

/* Reverse mode of the RB coefficients alpha = (T_S^T T_S)^{-1} T_S^T t (least squares, S frozen),
 * chained to the per-cell Lame parameters through the snapshots t_s = mu_s t^mu_s + lam_s t^lam_s.
 * Uses the greedy's outputs: Delta (= snap after lat_select_principal), Z, R, nu, and the snapshot
 * parts snap_mu, snap_lam (CIL(E), from lat_residual_tangent with mu = 1, lam = 0 and mu = 0,
 * lam = 1).  alpha_bar [N_s][cap].  ACCUMULATES into mu_bar, lam_bar [N_s].
 * work: LAT_CALL_ALPHA_ADJOINT workspace or NULL (with the fast size, n_r <= 32: one pass over
 * Delta for both Lame parts). */
lat_status lat_alpha_adjoint(const lat_plan *plan, const double *delta, const double *Z, const double *R,
                             const double *nu, const int32_t *S, int32_t n_r, const double *alpha,
                             const double *alpha_bar, const double *snap_mu, const double *snap_lam,
                             double *mu_bar, double *lam_bar, void *work, size_t work_bytes, hipStream_t stream);

/* Reverse mode of the residual r = sum_s A^s f^{int,s}(u^s) for a cell-local cotangent
 * w (CIL(d)):  ubar_local = K_s^T w_s (CIL(d), may be NULL), ubar_global = sum_s A^s ubar_local
 * ([n_global][d], may be NULL), mu_bar_s = <w_s, f^mu_s>, lam_bar_s = <w_s, f^lam_s> ([N_s],
 * written; may be NULL), with f = mu f^mu + lam f^lam at fixed u.
 * work: LAT_CALL_RESIDUAL_ADJOINT workspace or NULL. */
lat_status lat_residual_adjoint(const lat_plan *plan, const double *u_global, const double *mu, const double *lam,
                                const double *w, double *ubar_local, double *ubar_global, double *mu_bar,
                                double *lam_bar, int32_t *dev_status, void *work, size_t work_bytes,
                                hipStream_t stream);

/* Assembly r = sum_s A^s v_s of a cell-local field v (CIL(k)) into out [n_global][k], summing the
 * cells that share a node in ascending canonical order (deterministic). */
lat_status lat_assemble(const lat_plan *plan, const double *local, int32_t k, double *out, hipStream_t stream);

/* Gather w^s = A^{sT} w of a global field global [n_global][k] into CIL(k) (zero at nodes a cell
 * does not own). */
lat_status lat_gather(const lat_plan *plan, const double *global, int32_t k, double *local, hipStream_t stream);

/* Layout conversions.  canon: [N_s][(n+1)^d][d][m] (cell-major); packed as above. */
lat_status lat_pack(const lat_plan *plan, const double *canon, double *packed, int32_t m, hipStream_t stream);
lat_status lat_unpack(const lat_plan *plan, const double *packed, double *canon, int32_t m, hipStream_t stream);
/* CIL(k) <-> canonical [N_s][(n+1)^d][k]. */
lat_status lat_cil_to_canon(const lat_plan *plan, const double *cil, int64_t k, double *canon, hipStream_t stream);
lat_status lat_canon_to_cil(const lat_plan *plan, const double *canon, int64_t k, double *cil, hipStream_t stream);
/* Packed plain-ops -> canonical stencils [N_s][n_snap] (zero outside each group's union). */
lat_status lat_plain_ops_to_canon(const lat_plan *plan, const double *ops, double *canon, hipStream_t stream);

/* ---------------------------------------------------------------------------------------------
 * Nonlinear solve on the ROM tangent (Sec. 2.2.5, Newton-Raphson method; the reduced basis is
 * rebuilt at every iteration, Sec. 3.2.3).  Global vectors are [n_global][d], node-major, in the
 * plan's global numbering; `fixed` is a device uint8 [n_global][d] (1 = prescribed component).
 * These calls synchronise `stream`, allocate their device workspace for the duration of the call
 * and free it before returning; the hot-path calls inside them use the plan's default workspace
 * (so they must not overlap other NULL-workspace calls on the plan).
 * ------------------------------------------------------------------------------------------- */

/* Tangent solve K~ x = b on the free components (eq. linsys with the ROM operator of
 * eq. romstiffnessmatrix, K~ = sum_s A^s M_s (sum_k alpha_sk K_k) M_s A^{sT}) by MINRES
 * preconditioned with D = |diag K~|: K~ is symmetric but may be indefinite (a pre-stressed lattice
 * near buckling), and MINRES minimises ||b - K~ x||_{D^-1} over the Krylov space for any
 * symmetric non-singular K~.  Every product is a per-cell apply (one right-hand side) followed by an
 * owner-ordered assembly.  materialize != 0: the combined stencils sum_k alpha_sk K_k of all cells
 * are formed once (device memory n_packed E 64 doubles, the lat_apply_plain layout) and every
 * product reads them; materialize == 0: every product is a ROM apply that forms them on the fly
 * (no per-cell storage).  precond = 0: D = |diag K~|; precond = 1: two levels,
 * M^-1 = D^-1 + P K0^-1 P^T with the coarse operator of lat_coarse_operator, factorised per call
 * (rocSOLVER Cholesky and inverse, FP64); a K0 that is not positive definite or larger than the
 * limit leaves D alone, and *coarse_used (HOST, may be NULL) says which ran.  The stop test then
 * uses ||.||_{M^-1} in place of ||.||_{D^-1}.  K, n_r (HOST), alpha as for lat_apply_combo.
 * b [n_global][d] (prescribed components ignored), x [n_global][d] out (prescribed components 0;
 * x starts from 0).  Stops when the residual estimate of the rotations satisfies
 * ||r||_{D^-1} <= tol ||b||_{D^-1} (tol > 0), after at most maxit iterations, checking on the host
 * every `check` iterations (>= 1).  HOST outputs: iters, relres = ||r||_{D^-1} / ||b||_{D^-1}
 * (0 when b = 0).  Returns LAT_OK when converged, LAT_E_NOCONV at maxit (x holds the last
 * iterate), LAT_E_SINGULAR when K~ is singular on the Krylov space (x holds the last iterate). */
lat_status lat_rom_solve(const lat_plan *plan, const double *K, int32_t n_r, const double *alpha,
                         const uint8_t *fixed, const double *b, double *x, double tol, int32_t maxit,
                         int32_t check, int32_t materialize, int32_t precond, int32_t *iters, double *relres,
                         int32_t *coarse_used, hipStream_t stream);

/* The coarse operator of the two-level preconditioner: K0 = P^T K~ P, P the Q1 interpolation from
 * the cell-corner nodes (coarse node C = cx + (C_x+1)(cy + (C_y+1) cz), coarse DOF C d + i, the
 * corners being the primal nodes of the coarse problem of Sec. 3.3) to the global nodes with
 * the prescribed components' rows removed.  Formed with one ROM apply of the cells' 2^d d corner
 * functions (materialize as in lat_rom_solve), per-cell products and an owner-ordered assembly;
 * a coarse DOF with no free fine support gets a unit diagonal.  K0: device [n_c d][n_c d],
 * row-major, n_c = prod (C_x+1).  LAT_E_SHAPE when n_c d > 16384 (the dense factor's limit). */
lat_status lat_coarse_operator(const lat_plan *plan, const double *K, int32_t n_r, const double *alpha,
                               const uint8_t *fixed, int32_t materialize, double *K0, hipStream_t stream);

/* ---- Inexact FETI-DP solve of the ROM tangent system (Sec. 3.3, eq. ifetidp_precond) ----
 * Each cell is a subdomain.  Local nodes are primal (cell corners, plus `level` nodes per cell edge
 * at the edge coordinates round(k n / (level + 1)), k = 1..level, halves rounded up), dual (the
 * other cell-boundary nodes) or interior; the classes are those of the union of the cells' active
 * nodes.  Primal nodes are assembled globally (ascending global id); a dual node shared by k >= 2
 * cells (where active) carries k - 1 Lagrange multipliers chaining those cells in ascending id. */

/* The partition at enrichment `level` (>= 0), for tests and tools: HOST outputs.
 * counts [4]: primal global nodes, node-level multipliers, remaining (dual + interior) local
 * nodes, dual local nodes.  node_class [(n+1)^d] (may be NULL): 0 interior, 1 dual, 2 primal, -1
 * active in no cell.  primal_nodes [counts[0]] (may be NULL): their global ids, ascending.
 * mult [counts[1]][4] (may be NULL): (cell_1, node_1, cell_2, node_2) per multiplier, by global
 * node then chain position, cell_1 < cell_2 canonical ids.  Synchronises `stream`. */
lat_status lat_feti_partition(const lat_plan *plan, int32_t level, int32_t *node_class, int64_t *counts,
                              int64_t *primal_nodes, int32_t *mult, hipStream_t stream);

/* Options of lat_feti_solve (HOST struct). */
typedef struct {
    int32_t n_delta;      /* principal cells in the local reduced models: 0 = all n_r, else min(n_delta, n_r) */
    int32_t enrich;       /* enrichment level to start from (0 = corner primal nodes only) */
    int32_t max_enrich;   /* highest enrichment level tried (>= enrich) */
    int32_t inner_it;     /* PCG steps of the interface sub-solve F~^-pcg (0 = its Dirichlet preconditioner) */
    int32_t restart;      /* FGMRES restart length, 1..512 */
    int32_t maxit;        /* FGMRES iterations in total, >= 1 */
    int32_t materialize;  /* products K~ u from the combined stencils (1) or from ROM applies (0) */
    int32_t indefinite;   /* principal remaining blocks left indefinite after enrichment: 0 = shifted
                             to definiteness; 1 = inverted by pivoted LU, the interface block by its
                             Dirichlet preconditioner alone (see lat_feti_solve) */
    int32_t coords;       /* the cells' coordinates delta^s in the local models: 1 = one-hot on the
                             nearest of the first n_delta principal cells in snapshot space (needs R,
                             nu, beta; lanes are then grouped by principal cell and each group's
                             products are one GEMM); 0 = least squares over them (see lat_feti_solve) */
    int32_t prec;         /* precision of the local solves' blocks G_r in the preconditioner: LAT_F64, or
                             LAT_F32 (coords = 1; halves their bytes; the operator, the residual and
                             everything else stay FP64) */
    double tol;           /* stop at ||res|| <= tol ||rhs|| (2-norms of the saddle-point system), > 0 */
    double inner_tol;     /* > 0: the interface sub-solve also stops once its preconditioned residual
                             r.z has fallen below inner_tol^2 times its start (a relative reduction of
                             inner_tol), inner_it steps being the cap (one 4-byte host read per step);
                             0: always inner_it steps.  FGMRES accepts the varying inner solve. */
} lat_feti_opts;

/* What a solve did (HOST struct). */
typedef struct {
    int32_t iters;        /* FGMRES iterations */
    int32_t restarts;
    int32_t enrich;       /* enrichment level used */
    int32_t n_delta;      /* principal cells in the local reduced models */
    int32_t n_shift;      /* principal remaining blocks not positive definite after enrichment */
    int32_t reserved;
    int64_t n_primal;     /* assembled primal DOFs */
    int64_t n_mult;       /* multiplier rows: interface DOFs, then prescribed dual components */
    int64_t n_rdofs;      /* remaining DOFs per cell (union layout) */
    int64_t n_ddofs;      /* dual DOFs per cell */
    double relres;        /* true relative residual of the saddle-point system at exit */
    double max_shift;     /* largest diagonal shift s of those blocks (0 when none) */
    double t_setup_ms;    /* partition, principal factorisations, coarse problem */
    double t_solve_ms;    /* FGMRES */
} lat_feti_info;

/* Solve K~ x = b on the free components (eq. linsys with the ROM operator of eq.
 * romstiffnessmatrix, as lat_rom_solve) by iterating on the FETI-DP saddle-point system
 *     [K~  B^T] [u]   [f]      K~ the partially assembled ROM tangent, B the interface jumps,
 *     [B   0  ] [l] = [0]      f = b split over the cells sharing a node (primal rows: b)
 * with restarted FGMRES, right-preconditioned by the block factorisation of eq. ifetidp_precond.
 * Its local operators are reduced models over the first n_delta principal cells r (Algorithm 1's
 * order): the inverse remaining block G_r = (K_RR^r)^-1 (a Cholesky factor and inverse per
 * principal cell, FP64), the primal harmonic extension -G_r K_RP^r, the local primal Schur
 * complement and the local dual Schur complement F_dd^r = (G_r)_dd with its inverse; cell s uses
 * sum_r delta_r^s (.)_r.  delta^s (opts->coords): one-hot on the principal cell r < n_delta whose
 * snapshot is nearest to the cell's, ||t_s - t_{s_r}||^2 = nu_s^2 + nu_{s_r}^2 - 2 nu_s
 * sum_j beta_j^s R[j][r] (exact from the greedy's outputs, ties to the lowest r); or the
 * least-squares coordinates of its snapshot in the first n_delta principal snapshots
 * (R[:nd,:nd] delta = nu_s beta^s[:nd]; alpha when nd = n_r or R is NULL), whose combinations of
 * inverses extrapolate and converge far worse in practice.  The assembled coarse problem is inverted in FP64 (LU); the interface block F^-1 is
 * `inner_it` PCG steps (fewer when `inner_tol` is met) on B K~rom^-1 B^T with the Dirichlet preconditioner
 * B_D (sum_r delta_r (F_dd^r)^-1) B_D^T, B_D = (B B^T)^-1 B node by node.  A principal remaining
 * block that is not positive definite (Cholesky failure or a pivot <= 1e-12 of its diagonal entry)
 * raises the enrichment level and the setup restarts (Sec. 3.3.2), while the next level adds an
 * active primal node and does not pass max_enrich; past that, a block that is not positive
 * definite but nonsingular (pivoted LU, pivots > 1e-13 of the largest diagonal entry; info->n_shift
 * counts them) enters the local models as (K_RR^r + s diag K_RR^r)^-1, s the smallest of 1e-6,
 * 1e-5, ..., 1 that makes it positive definite (opts->indefinite = 0, info->max_shift), or is
 * inverted by that LU with the interface block then its Dirichlet preconditioner alone
 * (opts->indefinite = 1).  FGMRES iterates on the exact operator either way.  A ROM tangent that is
 * itself indefinite (a lattice past buckling) is out of this preconditioner's reach: expect
 * LAT_E_NOCONV (lat_rom_solve's MINRES handles it).
 * K, n_r (HOST, 1..cap), alpha as for lat_apply_combo; S [cap] the principal cells
 * (lat_select_principal); R [cap][cap], nu [N_s], beta [N_s][cap] from the greedy, or all NULL.
 * fixed [n_global][d] (1 = prescribed): a prescribed component of a dual node is imposed by one more
 * multiplier row (on its lowest-id owner), so boundary cells keep the local operators of free
 * cells; prescribed primal components leave the coarse problem; those of interior nodes are
 * removed.  b [n_global][d] (prescribed components ignored),
 * x [n_global][d] out: primal nodes from u_P, others the mean of the owning cells' u_R, prescribed
 * components 0; x starts from 0.  Device workspace is allocated for the call and freed before it
 * returns; synchronises `stream`.  info (HOST, may be NULL) receives the statistics.  Returns LAT_OK
 * when ||res|| <= tol ||rhs||, LAT_E_NOCONV at maxit (x holds the last iterate), LAT_E_SINGULAR
 * when a principal remaining block, a dual block or the coarse matrix is singular, or the Krylov
 * space breaks down, LAT_E_SHAPE when the coarse problem exceeds 40000 DOFs. */
lat_status lat_feti_solve(const lat_plan *plan, const double *K, int32_t n_r, const double *alpha, const int32_t *S,
                          const double *R, const double *nu, const double *beta, const uint8_t *fixed, const double *b,
                          double *x, const lat_feti_opts *opts, lat_feti_info *info, hipStream_t stream);

/* Options of lat_newton_solve (HOST struct). */
typedef struct {
    int32_t n_inc;          /* load increments, >= 1 */
    int32_t max_newton;     /* Newton iterations per increment, >= 1 */
    int32_t max_backtrack;  /* Armijo reductions per iteration, >= 0 */
    int32_t cap;            /* principal-cell cap per iteration, 1..plan cap */
    int32_t cg_maxit;       /* MINRES iterations per tangent solve, >= 1 */
    int32_t cg_check;       /* iterations between host convergence reads, >= 1 */
    int32_t snap_rule;      /* lat_rule of the snapshots fed to the greedy */
    int32_t verbose;        /* nonzero: one progress line per Newton iteration on stderr */
    int32_t matvec;         /* ROM tangent products: 0 = combined stencils formed once per iteration,
                               1 = ROM apply forming them on the fly (see lat_rom_solve) */
    int32_t tangent;        /* 0 = ROM tangent (the method), 1 = every cell's own full-rule tangent
                               (the standard method, for comparison; no greedy) */
    int32_t precond;        /* tangent solve: 0 / 1 = lat_rom_solve's MINRES with its precond 0 / 1;
                               2 = the inexact FETI-DP solve (lat_feti_solve, ROM tangent only; interface
                               sub-solve to a relative reduction of 1e-2, at most 32 PCG steps), with
                               MINRES (two levels) taking over a step it does not converge on */
    int32_t feti_n_delta;   /* precond 2: lat_feti_opts.n_delta (0 = every principal cell) */
    double rb_tol;          /* greedy tolerance (Algorithm 1), > 0 */
    double newton_tol;      /* stop an increment at ||r|| / ||r(u_0)|| <= newton_tol, > 0 */
    double armijo_beta;     /* step reduction factor, in (0, 1) */
    double armijo_c;        /* sufficient-decrease constant, in [0, 1) */
    double cg_tol;          /* relative residual ||r||_{D^-1} of each tangent solve, > 0 */
} lat_newton_opts;

/* One Newton iteration (HOST struct). */
typedef struct {
    int32_t increment;      /* 1..n_inc */
    int32_t iteration;      /* 0-based within the increment */
    int32_t n_r;            /* principal cells of this iteration's reduced basis (0: standard method) */
    int32_t backtracks;     /* Armijo exponent m of the accepted step beta^m */
    int32_t cg_iters;       /* MINRES iterations of the tangent solve */
    int32_t greedy_status;  /* LAT_OK or LAT_W_CAP */
    int32_t cg_status;      /* LAT_OK, LAT_E_NOCONV or LAT_E_SINGULAR */
    int32_t coarse;         /* 1 if the two-level preconditioner's coarse correction ran */
    double step;            /* beta^m */
    double res_before;      /* ||r(u_k)||_2 */
    double res_after;       /* ||r(u_k + beta^m du)||_2 */
    double res0;            /* ||r(u_0)||_2 of the increment */
    double rb_achieved;     /* the greedy's max_s ||Delta^s||_inf at exit */
    double cg_relres;       /* ||r||_{D^-1} / ||rhs||_{D^-1} at the end of the tangent solve */
    double t_init_ms;       /* greedy + principal tangents + preconditioner */
    double t_solve_ms;      /* tangent solve */
    double t_eval_ms;       /* residual + snapshot evaluations (predictor and line-search trials) */
    double t_product_us;    /* mean duration of one tangent product (the per-cell or ROM apply),
                               HIP events around up to 64 products of the solve, taken from the
                               9th product of each host batch on (0 when none was timed) */
    int32_t solver;         /* 0 MINRES, 1 FETI-DP, 2 FETI-DP stopped short and MINRES solved */
    int32_t feti_iters;     /* FETI-DP FGMRES iterations (solver 1, 2) */
    int32_t feti_enrich;    /* FETI-DP enrichment level used */
    int32_t reserved;
    double feti_relres;     /* FETI-DP saddle-point relative residual at its exit */
    double t_feti_setup_ms; /* FETI-DP setup (partition, principal factorisations, coarse problem) */
} lat_newton_record;

/* Load-stepped Newton-Raphson with Armijo backtracking (Sec. 2.2.5) on the ROM tangent.
 * mu, lam [N_s] (device, canonical); fixed [n_global][d]; ubar [n_global][d]: the displacement
 * added to every node over the whole load (increment t adds ubar / n_inc to u at its start, which
 * carries the prescribed components to t / n_inc of their final value and is the increment's
 * first iterate); f_ext [n_global][d] external nodal forces of the whole load, scaled by t / n_inc
 * (may be NULL).  u [n_global][d] device, in: the initial state, out: the final state.
 * Residual r(u) = sum_s A^s f^{int,s} - (t/n_inc) f_ext, zero on prescribed components.
 * Each iteration: snapshots at u (opts->snap_rule) -> greedy (rb_tol, cap) -> principal tangents
 * -> tangent solve K~ du = -r (lat_rom_solve's MINRES, or lat_feti_solve by opts->precond; its
 * status goes to the record and a solve stopped early still provides the direction) -> the smallest m <= max_backtrack with
 * ||r(u + beta^m du)|| <= (1 - c beta^m) ||r(u)|| (a trial with J <= 0 anywhere fails) ->
 * u += beta^m du; the increment ends when ||r|| <= newton_tol ||r(u_0)||.
 * records: HOST array of max_records entries (may be NULL), one per Newton iteration in order;
 * *n_records (HOST, may be NULL) receives the number of iterations run (which may exceed
 * max_records).  Returns LAT_OK, LAT_E_NOCONV (iteration or backtracking limit; u holds the last
 * accepted state), LAT_E_INVERTED / LAT_E_NONFINITE (an increment's first iterate is not
 * admissible), or an argument/device error. */
lat_status lat_newton_solve(const lat_plan *plan, const double *mu, const double *lam, const uint8_t *fixed,
                            const double *ubar, const double *f_ext, const lat_newton_opts *opts, double *u,
                            lat_newton_record *records, int32_t max_records, int32_t *n_records,
                            hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* LAT_H */
