// Inexact FETI-DP solve of the ROM tangent system (Sec. 3.3, eq. ifetidp_precond).
//
// Every cell is a subdomain.  Its local nodes are primal (cell corners, plus the edge nodes of the
// enrichment level), dual (the other cell-boundary nodes) or interior; remaining = dual + interior.
// The unknowns of the saddle-point system are the cells' remaining DOFs u_R (not assembled), the
// assembled primal DOFs u_P and one Lagrange multiplier per continuity equation of a dual DOF
// (a node shared by k cells: k - 1 equations chaining the cells in ascending id):
//     [ K~   B^T ] [u]   [f]        K~ = partially assembled ROM tangent (primal rows summed),
//     [ B    0   ] [l] = [0]        B  = jumps of u_R across the interfaces.
// FGMRES (right preconditioned, restarted) iterates on it with the block preconditioner
//     A^-1 ~ [I  -K^-1 B^T] [K^-1        ] [I        ]
//            [0   I       ] [     -F^-1  ] [-B K^-1 I]
// where every local operator of K~^-1 comes from a reduced model over the principal cells: for the
// first n_delta principal cells r the remaining block K_RR^r is factorised and inverted once
// (G_r), with the primal harmonic extension Phi_r = -G_r K_RP^r, the local primal Schur complement
// S_r = K_PP^r + K_PR^r Phi_r and the dual blocks F_dd^r = (G_r)_dd (the local dual Schur
// complement) and its inverse; a cell's operator is sum_r delta_r^s (.)_r with delta^s the
// reduced-basis coordinates of its snapshot (the greedy's R system cut to n_delta principal
// cells, which is alpha itself when n_delta = n_r).  The coarse problem sum_s A_P^s S^s A_P^sT is
// assembled and inverted in FP64.  F^-1 is a few PCG steps on the interface operator
// F~ = B K~rom^-1 B^T (formed from the dual blocks only) with the Dirichlet preconditioner
// B_D (sum_r delta_r (F_dd^r)^-1) B_D^T, B_D = (B B^T)^-1 B per shared node.  When a principal
// remaining block is not positive definite the partition is enriched (one more primal node on
// every cell edge, for all cells) and the setup restarts (Sec. 3.3.2); when no further level adds
// an active primal node (voxel struts leave most cell edges void) a block that stays indefinite
// but is nonsingular enters the local models as (K_RR^r + s diag K_RR^r)^-1 with the smallest s of a
// decade ladder that makes it definite (the default), or is inverted exactly by pivoted LU with
// the interface block then taken by its Dirichlet preconditioner alone (PCG needs a definite
// operator); FGMRES iterates on the exact operator either way.
//
// Data layout (lanes = the plan's cell lanes, fastest):
//   u_R    [n_R rows][ld]   row = remaining node index * d + component (the union of the cells'
//                           active remaining nodes, lexicographic); padding / inactive entries 0
//   u_P    [n_Pg * d]       the global primal nodes in ascending global id
//   lambda [n_mult * d]
// so the local products are plain GEMMs (rocBLAS, FP64): [ld x n_R] x [n_R x n_delta n_R].
// Prescribed components of dual nodes are imposed by one more multiplier row each (u = 0 on the
// first owning cell; the interface rows carry it to the others), so that the local remaining
// blocks stay those of free cells and the reduced models apply to boundary cells unchanged;
// prescribed primal components are removed from the coarse problem.  Degrees of freedom that do
// not exist (a node inactive in a cell, a prescribed component of an interior node) are identity
// rows of the saddle-point operator and of the preconditioner.
#include <chrono>
#include <cmath>
#include <memory>
#include <mutex>

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "lat_internal.h"

namespace {

constexpr int NB = 256;

#define FCHK(expr) do { lat_status st_ = (expr); if (st_ != LAT_OK) return st_; } while (0)
#define RBCHK(expr) do { if ((expr) != rocblas_status_success) return LAT_E_DEVICE; } while (0)

struct FArena {
    std::vector<void *> ptrs;
    ~FArena()
    {
        for (void *p : ptrs) (void)hipFree(p);
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
    template <class T>
    lat_status put(T **p, const std::vector<T> &h, hipStream_t s)
    {
        FCHK(get(p, (int64_t)h.size()));
        if (!h.empty()) LAT_HIP(hipMemcpyAsync(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
        return LAT_OK;
    }
};

// One rocBLAS handle per device (created on first use, kept), with atomics off so that every
// product is reproducible.
rocblas_handle feti_handle()
{
    static std::mutex mu;
    static rocblas_handle h[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(mu);
    if (!h[dev]) {
        if (rocblas_create_handle(&h[dev]) != rocblas_status_success) return h[dev] = nullptr;
        (void)rocblas_set_atomics_mode(h[dev], rocblas_atomics_not_allowed);
    }
    return h[dev];
}

// thread-per-element grids (the grid-stride kernels accept any grid)
unsigned blocks(int64_t n) { return (unsigned)std::max<int64_t>(1, lat_cdiv(n, NB)); }

// ------------------------------------------------------------------------------------------
// Partition (host)
// ------------------------------------------------------------------------------------------
struct Part {
    int level = 0, d = 0, nloc = 0;
    int nRn = 0, nPn = 0, nDn = 0;         // remaining / primal / dual local nodes (union over cells)
    int64_t nPg = 0, nsets = 0, nmult = 0;  // global primal nodes, shared dual nodes, multipliers
    std::vector<int32_t> cls;               // [nloc] 0 interior, 1 dual, 2 primal, -1 never active
    std::vector<int32_t> fnode;             // [nloc] remaining index, nRn + primal index, or -1
    std::vector<int32_t> rnode, pnode;      // local node of each remaining / primal index
    std::vector<int32_t> dual_rn;           // [nDn] remaining index of each dual node
    std::vector<int32_t> dpos;              // [nRn] dual position of each remaining node or -1
    // prescribed components of dual nodes: one multiplier row each (after the interface rows)
    int64_t ndir = 0;
    std::vector<int32_t> dir_lane, dir_rn, dir_dn, dir_i;
    std::vector<int64_t> pglob;             // [nPg] global node of each global primal node
    std::vector<int32_t> prim_g;            // [nPn][ld] global primal index of (primal node, lane) or -1
    std::vector<int32_t> pg_off, pg_lane, pg_p;        // global primal -> owners (lane, primal index)
    std::vector<int32_t> set_off, set_m0;              // shared dual node -> members, first multiplier
    std::vector<int64_t> set_g;                        // global node of each set
    std::vector<int32_t> mem_lane, mem_rn, mem_dn, mem_cell, mem_a;
    std::vector<int32_t> gn_off, gn_lane, gn_fn;       // global node -> owners (lane, FETI node)
    std::vector<int32_t> gp_of_g;                      // [n_global] global primal index or -1
};

std::vector<int> edge_positions(int nel, int level)
{
    std::vector<char> on((size_t)nel + 1, 0);
    for (int k = 1; k <= level; ++k) {
        int t = (2 * k * nel + level + 1) / (2 * (level + 1));
        t = std::min(std::max(t, 1), nel - 1);
        on[(size_t)t] = 1;
    }
    std::vector<int> p;
    for (int t = 1; t < nel; ++t)
        if (on[(size_t)t]) p.push_back(t);
    return p;
}

void build_part(const lat_plan *P, int level, const std::vector<int32_t> &l2g, const std::vector<int32_t> &lane_of,
                Part &pt)
{
    const int d = P->dim, n = P->nel, nn = P->nn, nloc = P->nloc;
    const int64_t Ns = P->ncells, ld = P->ld;
    pt = Part{};
    pt.level = level; pt.d = d; pt.nloc = nloc;
    std::vector<char> tpos((size_t)nn, 0);
    for (int t : edge_positions(n, level)) tpos[(size_t)t] = 1;
    std::vector<char> uact((size_t)nloc, 0);
    for (int64_t s = 0; s < Ns; ++s)
        for (int a = 0; a < nloc; ++a)
            if (l2g[(size_t)(s * nloc + a)] >= 0) uact[(size_t)a] = 1;
    pt.cls.assign((size_t)nloc, -1);
    for (int a = 0; a < nloc; ++a) {
        if (!uact[(size_t)a]) continue;
        const int c[3] = {a % nn, (a / nn) % nn, d == 3 ? a / (nn * nn) : 0};
        int nb = 0, fre = -1;
        for (int ax = 0; ax < d; ++ax) {
            if (c[ax] == 0 || c[ax] == n) ++nb;
            else fre = c[ax];
        }
        int k = 0;
        if (nb == d) k = 2;
        else if (nb == d - 1) k = tpos[(size_t)fre] ? 2 : 1;
        else if (nb >= 1) k = 1;
        pt.cls[(size_t)a] = k;
    }
    pt.fnode.assign((size_t)nloc, -1);
    for (int a = 0; a < nloc; ++a)
        if (pt.cls[(size_t)a] == 0 || pt.cls[(size_t)a] == 1) {
            pt.fnode[(size_t)a] = (int32_t)pt.rnode.size();
            pt.rnode.push_back(a);
        }
    pt.nRn = (int)pt.rnode.size();
    for (int a = 0; a < nloc; ++a)
        if (pt.cls[(size_t)a] == 2) {
            pt.fnode[(size_t)a] = pt.nRn + (int32_t)pt.pnode.size();
            pt.pnode.push_back(a);
        }
    pt.nPn = (int)pt.pnode.size();
    for (int rn = 0; rn < pt.nRn; ++rn)
        if (pt.cls[(size_t)pt.rnode[(size_t)rn]] == 1) pt.dual_rn.push_back(rn);
    pt.nDn = (int)pt.dual_rn.size();
    pt.dpos.assign((size_t)pt.nRn, -1);
    std::vector<int32_t> &dpos = pt.dpos;
    for (int k = 0; k < pt.nDn; ++k) dpos[(size_t)pt.dual_rn[(size_t)k]] = k;
    // owners of every global node, ascending cell id
    const int64_t ng = P->nglobal;
    pt.gn_off.assign((size_t)ng + 1, 0);
    for (int64_t s = 0; s < Ns; ++s)
        for (int a = 0; a < nloc; ++a) {
            const int32_t g = l2g[(size_t)(s * nloc + a)];
            if (g >= 0) ++pt.gn_off[(size_t)g + 1];
        }
    for (int64_t g = 0; g < ng; ++g) pt.gn_off[(size_t)g + 1] += pt.gn_off[(size_t)g];
    pt.gn_lane.assign((size_t)pt.gn_off[(size_t)ng], 0);
    pt.gn_fn.assign((size_t)pt.gn_off[(size_t)ng], 0);
    std::vector<int32_t> gcell((size_t)pt.gn_off[(size_t)ng], 0), ga((size_t)pt.gn_off[(size_t)ng], 0);
    {
        std::vector<int32_t> fill(pt.gn_off.begin(), pt.gn_off.end() - 1);
        for (int64_t s = 0; s < Ns; ++s)
            for (int a = 0; a < nloc; ++a) {
                const int32_t g = l2g[(size_t)(s * nloc + a)];
                if (g < 0) continue;
                const int32_t k = fill[(size_t)g]++;
                pt.gn_lane[(size_t)k] = lane_of[(size_t)s];
                pt.gn_fn[(size_t)k] = pt.fnode[(size_t)a];
                gcell[(size_t)k] = (int32_t)s;
                ga[(size_t)k] = a;
            }
    }
    // global primal nodes
    pt.gp_of_g.assign((size_t)ng, -1);
    for (int64_t g = 0; g < ng; ++g) {
        const int32_t k0 = pt.gn_off[(size_t)g];
        if (pt.gn_off[(size_t)g + 1] > k0 && pt.cls[(size_t)ga[(size_t)k0]] == 2) {
            pt.gp_of_g[(size_t)g] = (int32_t)pt.pglob.size();
            pt.pglob.push_back(g);
        }
    }
    pt.nPg = (int64_t)pt.pglob.size();
    pt.prim_g.assign((size_t)pt.nPn * ld, -1);
    pt.pg_off.assign((size_t)pt.nPg + 1, 0);
    for (int64_t G = 0; G < pt.nPg; ++G) {
        const int64_t g = pt.pglob[(size_t)G];
        pt.pg_off[(size_t)G + 1] = pt.pg_off[(size_t)G];
        for (int32_t k = pt.gn_off[(size_t)g]; k < pt.gn_off[(size_t)g + 1]; ++k) {
            const int p = pt.gn_fn[(size_t)k] - pt.nRn;
            pt.pg_lane.push_back(pt.gn_lane[(size_t)k]);
            pt.pg_p.push_back(p);
            pt.prim_g[(size_t)p * ld + pt.gn_lane[(size_t)k]] = (int32_t)G;
            ++pt.pg_off[(size_t)G + 1];
        }
    }
    // shared dual nodes and their multiplier chains
    pt.set_off.push_back(0);
    for (int64_t g = 0; g < ng; ++g) {
        const int32_t k0 = pt.gn_off[(size_t)g], k1 = pt.gn_off[(size_t)g + 1];
        if (k1 - k0 < 2 || pt.cls[(size_t)ga[(size_t)k0]] != 1) continue;
        pt.set_m0.push_back((int32_t)pt.nmult);
        pt.set_g.push_back(g);
        for (int32_t k = k0; k < k1; ++k) {
            const int rn = pt.gn_fn[(size_t)k];
            pt.mem_lane.push_back(pt.gn_lane[(size_t)k]);
            pt.mem_rn.push_back(rn);
            pt.mem_dn.push_back(dpos[(size_t)rn]);
            pt.mem_cell.push_back(gcell[(size_t)k]);
            pt.mem_a.push_back(ga[(size_t)k]);
        }
        pt.set_off.push_back((int32_t)pt.mem_lane.size());
        pt.nmult += k1 - k0 - 1;
    }
    pt.nsets = (int64_t)pt.set_m0.size();
}

// Multiplier rows of the prescribed components of dual nodes (first owner, ascending global node
// and component); `fixed` [n_global][d] on the host.
void build_dirichlet(const lat_plan *P, const std::vector<uint8_t> &fixed, Part &pt)
{
    const int d = P->dim;
    pt.ndir = 0;
    pt.dir_lane.clear(); pt.dir_rn.clear(); pt.dir_dn.clear(); pt.dir_i.clear();
    for (int64_t g = 0; g < P->nglobal; ++g) {
        const int32_t k0 = pt.gn_off[(size_t)g];
        if (pt.gn_off[(size_t)g + 1] == k0 || pt.gp_of_g[(size_t)g] >= 0) continue;
        const int rn = pt.gn_fn[(size_t)k0];
        if (pt.dpos[(size_t)rn] < 0) continue;
        for (int i = 0; i < d; ++i)
            if (fixed[(size_t)(g * d + i)]) {
                pt.dir_lane.push_back(pt.gn_lane[(size_t)k0]);
                pt.dir_rn.push_back(rn);
                pt.dir_dn.push_back(pt.dpos[(size_t)rn]);
                pt.dir_i.push_back(i);
                ++pt.ndir;
            }
    }
}

// B_D = (B B^T)^-1 B for the chain jump operator of a node shared by k cells (rows e_t - e_{t+1}),
// k = 2..8: table bd[k][t][u] (t < k - 1, u < k).
std::vector<double> chain_scaling()
{
    std::vector<double> bd(9 * 8 * 8, 0.0);
    for (int k = 2; k <= 8; ++k) {
        const int m = k - 1;
        // M = B B^T is tridiagonal (2 on the diagonal, -1 beside it); invert it by Gauss-Jordan
        std::vector<double> M((size_t)m * 2 * m, 0.0);
        for (int i = 0; i < m; ++i) {
            M[(size_t)i * 2 * m + i] = 2.0;
            if (i > 0) M[(size_t)i * 2 * m + i - 1] = -1.0;
            if (i + 1 < m) M[(size_t)i * 2 * m + i + 1] = -1.0;
            M[(size_t)i * 2 * m + m + i] = 1.0;
        }
        for (int c = 0; c < m; ++c) {
            const double pv = M[(size_t)c * 2 * m + c];
            for (int j = 0; j < 2 * m; ++j) M[(size_t)c * 2 * m + j] /= pv;
            for (int r = 0; r < m; ++r) {
                if (r == c) continue;
                const double f = M[(size_t)r * 2 * m + c];
                for (int j = 0; j < 2 * m; ++j) M[(size_t)r * 2 * m + j] -= f * M[(size_t)c * 2 * m + j];
            }
        }
        for (int t = 0; t < m; ++t)
            for (int u = 0; u < k; ++u) {
                double v = 0.0;   // sum_j Minv[t][j] B[j][u], B[j][u] = [u == j] - [u == j + 1]
                for (int j = 0; j < m; ++j) {
                    const double b = (u == j ? 1.0 : 0.0) - (u == j + 1 ? 1.0 : 0.0);
                    v += M[(size_t)t * 2 * m + m + j] * b;
                }
                bd[((size_t)k * 8 + t) * 8 + u] = v;
            }
    }
    return bd;
}

// Device copies of the partition tables.
struct PartDev {
    int32_t *fnode, *rnode, *pnode, *dual_rn, *prim_g, *pg_off, *pg_lane, *pg_p;
    int32_t *set_off, *set_m0, *mem_lane, *mem_rn, *mem_dn, *gn_off, *gn_lane, *gn_fn, *gp_of_g;
    int64_t *pglob, *set_g;
    double *bd;
    int32_t *dpos, *dir_lane, *dir_rn, *dir_dn, *dir_i;
};

lat_status upload_part(const Part &pt, FArena &ar, PartDev &pd, hipStream_t s)
{
    FCHK(ar.put(&pd.fnode, pt.fnode, s)); FCHK(ar.put(&pd.rnode, pt.rnode, s)); FCHK(ar.put(&pd.pnode, pt.pnode, s));
    FCHK(ar.put(&pd.dual_rn, pt.dual_rn, s)); FCHK(ar.put(&pd.prim_g, pt.prim_g, s));
    FCHK(ar.put(&pd.pg_off, pt.pg_off, s)); FCHK(ar.put(&pd.pg_lane, pt.pg_lane, s)); FCHK(ar.put(&pd.pg_p, pt.pg_p, s));
    FCHK(ar.put(&pd.set_off, pt.set_off, s)); FCHK(ar.put(&pd.set_m0, pt.set_m0, s));
    FCHK(ar.put(&pd.mem_lane, pt.mem_lane, s)); FCHK(ar.put(&pd.mem_rn, pt.mem_rn, s)); FCHK(ar.put(&pd.mem_dn, pt.mem_dn, s));
    FCHK(ar.put(&pd.gn_off, pt.gn_off, s)); FCHK(ar.put(&pd.gn_lane, pt.gn_lane, s)); FCHK(ar.put(&pd.gn_fn, pt.gn_fn, s));
    FCHK(ar.put(&pd.gp_of_g, pt.gp_of_g, s)); FCHK(ar.put(&pd.pglob, pt.pglob, s)); FCHK(ar.put(&pd.set_g, pt.set_g, s));
    FCHK(ar.put(&pd.dpos, pt.dpos, s));
    FCHK(ar.put(&pd.dir_lane, pt.dir_lane, s)); FCHK(ar.put(&pd.dir_rn, pt.dir_rn, s));
    FCHK(ar.put(&pd.dir_dn, pt.dir_dn, s)); FCHK(ar.put(&pd.dir_i, pt.dir_i, s));
    const std::vector<double> bd = chain_scaling();
    FCHK(ar.put(&pd.bd, bd, s));
    LAT_HIP(hipStreamSynchronize(s));     // the host tables are pageable: finish before they go
    return LAT_OK;
}

// ------------------------------------------------------------------------------------------
// Kernels
// ------------------------------------------------------------------------------------------
__global__ void k_ffill(int64_t n, double v, double *__restrict__ y)
{
    for (int64_t j = (int64_t)blockIdx.x * NB + threadIdx.x; j < n; j += (int64_t)gridDim.x * NB) y[j] = v;
}

// live masks: remaining rows, primal DOFs, multipliers, dual rows
// (a prescribed component of a dual node stays live: its multiplier row imposes it)
__global__ void k_live_R(int d, int nloc, int nRn, int64_t ld, const int32_t *__restrict__ rnode,
                         const int32_t *__restrict__ dpos, const int32_t *__restrict__ perm,
                         const int32_t *__restrict__ l2g, const uint8_t *__restrict__ fixed, uint8_t *__restrict__ live)
{
    const int64_t t = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (t >= (int64_t)nRn * ld) return;
    const int64_t lane = t % ld;
    const int rn = (int)(t / ld);
    const int cell = perm[lane];
    const int32_t g = cell >= 0 ? l2g[(int64_t)cell * nloc + rnode[rn]] : -1;
    for (int i = 0; i < d; ++i)
        live[((int64_t)rn * d + i) * ld + lane] = g >= 0 && (dpos[rn] >= 0 || !fixed[(int64_t)g * d + i]);
}

__global__ void k_live_P(int d, int64_t nPg, const int64_t *__restrict__ pglob, const uint8_t *__restrict__ fixed,
                         uint8_t *__restrict__ live)
{
    const int64_t G = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (G >= nPg) return;
    for (int i = 0; i < d; ++i) live[G * d + i] = !fixed[pglob[G] * d + i];
}

__global__ void k_fill_u8(int64_t n, uint8_t v, uint8_t *__restrict__ y)
{
    for (int64_t j = (int64_t)blockIdx.x * NB + threadIdx.x; j < n; j += (int64_t)gridDim.x * NB) y[j] = v;
}

__global__ void k_live_D(int d, int nDn, int64_t ld, const int32_t *__restrict__ dual_rn,
                         const uint8_t *__restrict__ liveR, uint8_t *__restrict__ liveD)
{
    const int64_t t = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (t >= (int64_t)nDn * d * ld) return;
    const int64_t lane = t % ld;
    const int64_t row = t / ld;
    const int dn = (int)(row / d), i = (int)(row % d);
    liveD[t] = liveR[((int64_t)dual_rn[dn] * d + i) * ld + lane];
}

// The operator's input on the plan's packed layout (one right-hand side): remaining rows from u_R,
// primal nodes from u_P, zero where the DOF does not exist.
__global__ void k_to_packed(int d, int64_t npk, int nloc, int nRn, int64_t ld, const int32_t *__restrict__ qgroup,
                            const int32_t *__restrict__ unode, const uint64_t *__restrict__ umask,
                            const int32_t *__restrict__ fnode, const int32_t *__restrict__ prim_g,
                            const uint8_t *__restrict__ liveR, const uint8_t *__restrict__ liveP,
                            const double *__restrict__ uR, const double *__restrict__ uP, double *__restrict__ X)
{
    const int64_t t = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (t >= npk * LAT_WAVE) return;
    const int l = (int)(t % LAT_WAVE);
    const int64_t q = t / LAT_WAVE;
    const int64_t lane = (int64_t)qgroup[q] * LAT_WAVE + l;
    const bool own = (umask[q] >> l) & 1ull;
    const int fa = fnode[unode[q]];
    for (int i = 0; i < d; ++i) {
        double v = 0.0;
        if (own && fa >= 0) {
            if (fa < nRn) {
                const int64_t r = ((int64_t)fa * d + i) * ld + lane;
                v = liveR[r] ? uR[r] : 0.0;
            } else {
                const int32_t G = prim_g[(int64_t)(fa - nRn) * ld + lane];
                v = (G >= 0 && liveP[(int64_t)G * d + i]) ? uP[(int64_t)G * d + i] : 0.0;
            }
        }
        X[(q * d + i) * LAT_WAVE + l] = v;
    }
}

// remaining rows of the product (identity rows where the DOF does not exist)
__global__ void k_from_packed_R(int d, int nloc, int nRn, int64_t ld, const int32_t *__restrict__ rnode,
                                const int32_t *__restrict__ uidx, const int32_t *__restrict__ goff,
                                const uint8_t *__restrict__ liveR, const double *__restrict__ Y,
                                const double *__restrict__ uR, double *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (t >= (int64_t)nRn * ld) return;
    const int64_t lane = t % ld;
    const int rn = (int)(t / ld);
    const int64_t g = lane / LAT_WAVE;
    const int l = (int)(lane % LAT_WAVE);
    const int qi = uidx[g * nloc + rnode[rn]];
    for (int i = 0; i < d; ++i) {
        const int64_t r = ((int64_t)rn * d + i) * ld + lane;
        out[r] = liveR[r] ? (qi >= 0 ? Y[(((int64_t)goff[g] + qi) * d + i) * LAT_WAVE + l] : 0.0) : uR[r];
    }
}

// primal rows: sum over the owners in ascending cell id
__global__ void k_from_packed_P(int d, int nloc, int64_t nPg, const int32_t *__restrict__ pg_off,
                                const int32_t *__restrict__ pg_lane, const int32_t *__restrict__ pg_p,
                                const int32_t *__restrict__ pnode, const int32_t *__restrict__ uidx,
                                const int32_t *__restrict__ goff, const uint8_t *__restrict__ liveP,
                                const double *__restrict__ Y, const double *__restrict__ uP, double *__restrict__ out)
{
    const int64_t G = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (G >= nPg) return;
    for (int i = 0; i < d; ++i) {
        if (!liveP[G * d + i]) { out[G * d + i] = uP[G * d + i]; continue; }
        double acc = 0.0;
        for (int k = pg_off[G]; k < pg_off[G + 1]; ++k) {
            const int64_t lane = pg_lane[k];
            const int64_t g = lane / LAT_WAVE;
            const int qi = uidx[g * nloc + pnode[pg_p[k]]];
            if (qi >= 0) acc += Y[(((int64_t)goff[g] + qi) * d + i) * LAT_WAVE + lane % LAT_WAVE];
        }
        out[G * d + i] = acc;
    }
}

// out_R += B^T lambda on the members of every shared dual node (each member row belongs to one set)
__global__ void k_bt_add(int d, int64_t nsets, int64_t ld, const int32_t *__restrict__ set_off,
                         const int32_t *__restrict__ set_m0, const int32_t *__restrict__ mem_lane,
                         const int32_t *__restrict__ mem_rn, const uint8_t *__restrict__ liveL,
                         const double *__restrict__ lam, double *__restrict__ outR)
{
    const int64_t s = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (s >= nsets) return;
    const int k0 = set_off[s], k = set_off[s + 1] - k0;
    const int64_t m0 = set_m0[s];
    for (int i = 0; i < d; ++i) {
        if (!liveL[m0 * d + i]) continue;
        for (int t = 0; t < k; ++t) {
            const double v = (t < k - 1 ? lam[(m0 + t) * d + i] : 0.0) - (t > 0 ? lam[(m0 + t - 1) * d + i] : 0.0);
            outR[((int64_t)mem_rn[k0 + t] * d + i) * ld + mem_lane[k0 + t]] += v;
        }
    }
}

// out_L = B u_R (identity rows on multipliers of prescribed components)
__global__ void k_b(int d, int64_t nsets, int64_t ld, const int32_t *__restrict__ set_off,
                    const int32_t *__restrict__ set_m0, const int32_t *__restrict__ mem_lane,
                    const int32_t *__restrict__ mem_rn, const uint8_t *__restrict__ liveL,
                    const double *__restrict__ uR, const double *__restrict__ lam_in, double *__restrict__ outL)
{
    const int64_t s = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (s >= nsets) return;
    const int k0 = set_off[s], k = set_off[s + 1] - k0;
    const int64_t m0 = set_m0[s];
    for (int t = 0; t < k - 1; ++t)
        for (int i = 0; i < d; ++i) {
            const int64_t m = (m0 + t) * d + i;
            outL[m] = liveL[m] ? uR[((int64_t)mem_rn[k0 + t] * d + i) * ld + mem_lane[k0 + t]] -
                                     uR[((int64_t)mem_rn[k0 + t + 1] * d + i) * ld + mem_lane[k0 + t + 1]]
                               : lam_in[m];
        }
}

// the multiplier rows of prescribed dual components (rows Lint + j): B^T adds, B reads
__global__ void k_dir_bt(int d, int64_t ndir, int64_t ld, int64_t Lint, const int32_t *__restrict__ dir_lane,
                         const int32_t *__restrict__ dir_row, const int32_t *__restrict__ dir_i,
                         const double *__restrict__ lam, double *__restrict__ out)
{
    const int64_t j = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (j >= ndir) return;
    out[((int64_t)dir_row[j] * d + dir_i[j]) * ld + dir_lane[j]] += lam[Lint + j];
}

__global__ void k_dir_b(int d, int64_t ndir, int64_t ld, int64_t Lint, const int32_t *__restrict__ dir_lane,
                        const int32_t *__restrict__ dir_row, const int32_t *__restrict__ dir_i,
                        const double *__restrict__ u, double *__restrict__ outL)
{
    const int64_t j = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (j >= ndir) return;
    outL[Lint + j] = u[((int64_t)dir_row[j] * d + dir_i[j]) * ld + dir_lane[j]];
}

// the same two on the dual rows [nDn d][ld] (the interface operator's local vectors);
// qd must be zero outside the members
__global__ void k_bt_dual(int d, int64_t nsets, int64_t ld, const int32_t *__restrict__ set_off,
                          const int32_t *__restrict__ set_m0, const int32_t *__restrict__ mem_lane,
                          const int32_t *__restrict__ mem_dn, const uint8_t *__restrict__ liveL,
                          const double *__restrict__ bd, int scaled, const double *__restrict__ lam,
                          double *__restrict__ qd)
{
    const int64_t s = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (s >= nsets) return;
    const int k0 = set_off[s], k = set_off[s + 1] - k0;
    const int64_t m0 = set_m0[s];
    for (int i = 0; i < d; ++i) {
        const bool lv = liveL[m0 * d + i];
        for (int u = 0; u < k; ++u) {
            double v = 0.0;
            if (lv) {
                if (scaled) {
                    for (int t = 0; t < k - 1; ++t) v += bd[((int64_t)k * 8 + t) * 8 + u] * lam[(m0 + t) * d + i];
                } else {
                    v = (u < k - 1 ? lam[(m0 + u) * d + i] : 0.0) - (u > 0 ? lam[(m0 + u - 1) * d + i] : 0.0);
                }
            }
            qd[((int64_t)mem_dn[k0 + u] * d + i) * ld + mem_lane[k0 + u]] = v;
        }
    }
}

__global__ void k_b_dual(int d, int64_t nsets, int64_t ld, const int32_t *__restrict__ set_off,
                         const int32_t *__restrict__ set_m0, const int32_t *__restrict__ mem_lane,
                         const int32_t *__restrict__ mem_dn, const uint8_t *__restrict__ liveL,
                         const double *__restrict__ bd, int scaled, const double *__restrict__ vd,
                         const double *__restrict__ lam_in, double *__restrict__ outL)
{
    const int64_t s = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (s >= nsets) return;
    const int k0 = set_off[s], k = set_off[s + 1] - k0;
    const int64_t m0 = set_m0[s];
    for (int t = 0; t < k - 1; ++t)
        for (int i = 0; i < d; ++i) {
            const int64_t m = (m0 + t) * d + i;
            if (!liveL[m]) { outL[m] = lam_in[m]; continue; }
            double v = 0.0;
            if (scaled) {
                for (int u = 0; u < k; ++u)
                    v += bd[((int64_t)k * 8 + t) * 8 + u] * vd[((int64_t)mem_dn[k0 + u] * d + i) * ld + mem_lane[k0 + u]];
            } else {
                v = vd[((int64_t)mem_dn[k0 + t] * d + i) * ld + mem_lane[k0 + t]] -
                    vd[((int64_t)mem_dn[k0 + t + 1] * d + i) * ld + mem_lane[k0 + t + 1]];
            }
            outL[m] = v;
        }
}

// Scaled stack of a local block vector x [rows][ld]: S[(r rows + j) ld + lane] = delta[lane][r] x,
// and xm = the masked x (both as column-major [ld x ...] matrices).
__global__ void k_scale_stack(int64_t rows, int64_t ld, int nd, const double *__restrict__ delta,
                              const uint8_t *__restrict__ live, const double *__restrict__ x,
                              double *__restrict__ xm, double *__restrict__ S)
{
    const int64_t t = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (t >= rows * ld) return;
    const int64_t lane = t % ld;
    const double v = (!live || live[t]) ? x[t] : 0.0;
    if (xm) xm[t] = v;
    for (int r = 0; r < nd; ++r) S[(int64_t)r * rows * ld + t] = delta[lane * nd + r] * v;
}

// h[p][lane] = sum_r delta[lane][r] T[(r np + p) ld + lane]
__global__ void k_combine_delta(int64_t np, int64_t ld, int nd, const double *__restrict__ delta,
                                const double *__restrict__ T, double *__restrict__ h)
{
    const int64_t t = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (t >= np * ld) return;
    const int64_t lane = t % ld;
    double acc = 0.0;
    for (int r = 0; r < nd; ++r) acc = fma(delta[lane * nd + r], T[(int64_t)r * np * ld + t], acc);
    h[t] = acc;
}

// primal assembly of the local h [nPn d][ld]: out[G d + i] = base + sum over owners (live), base (dead)
__global__ void k_assemble_P(int d, int64_t ld, int64_t nPg, const int32_t *__restrict__ pg_off,
                             const int32_t *__restrict__ pg_lane, const int32_t *__restrict__ pg_p,
                             const uint8_t *__restrict__ liveP, const double *__restrict__ h,
                             const double *__restrict__ base, double *__restrict__ out)
{
    const int64_t G = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (G >= nPg) return;
    for (int i = 0; i < d; ++i) {
        const double b = base ? base[G * d + i] : 0.0;
        if (!liveP[G * d + i]) { out[G * d + i] = b; continue; }
        double acc = b;
        for (int k = pg_off[G]; k < pg_off[G + 1]; ++k) acc += h[((int64_t)pg_p[k] * d + i) * ld + pg_lane[k]];
        out[G * d + i] = acc;
    }
}

// e[(p d + i) ld + lane] = u_P of the cell's primal node (0 where absent or prescribed)
__global__ void k_gather_P(int d, int nPn, int64_t ld, const int32_t *__restrict__ prim_g,
                           const uint8_t *__restrict__ liveP, const double *__restrict__ uP, double *__restrict__ e)
{
    const int64_t t = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (t >= (int64_t)nPn * ld) return;
    const int64_t lane = t % ld;
    const int p = (int)(t / ld);
    const int32_t G = prim_g[t];
    for (int i = 0; i < d; ++i)
        e[((int64_t)p * d + i) * ld + lane] = (G >= 0 && liveP[(int64_t)G * d + i]) ? uP[(int64_t)G * d + i] : 0.0;
}

// z = live ? z : g
__global__ void k_identity_rows(int64_t n, const uint8_t *__restrict__ live, const double *__restrict__ g,
                                double *__restrict__ z)
{
    for (int64_t j = (int64_t)blockIdx.x * NB + threadIdx.x; j < n; j += (int64_t)gridDim.x * NB)
        if (!live[j]) z[j] = g[j];
}

// the principal cells' local matrices in FETI order (remaining DOFs first), column-major
__global__ void k_kloc(int d, int nn, int nloc, int E, int cap, int nF, int nFn, int nRn,
                       const int32_t *__restrict__ fnode, const int32_t *__restrict__ rnode,
                       const int32_t *__restrict__ pnode, const int32_t *__restrict__ S,
                       const int32_t *__restrict__ l2g, const double *__restrict__ K, double *__restrict__ Kl)
{
    const int64_t t = (int64_t)blockIdx.x * NB + threadIdx.x;
    const int r = blockIdx.y;
    if (t >= nFn) return;
    const int fa = (int)t;
    const int a = fa < nRn ? rnode[fa] : pnode[fa - nRn];
    const int64_t cell = S[r];
    double *M = Kl + (int64_t)r * nF * nF;
    if (l2g[cell * nloc + a] < 0) {
        for (int i = 0; i < d; ++i) M[((int64_t)fa * d + i) * nF + fa * d + i] = 1.0;
        return;
    }
    const int no = d == 3 ? 27 : 9;
    const int c[3] = {a % nn, (a / nn) % nn, d == 3 ? a / (nn * nn) : 0};
    for (int o = 0; o < no; ++o) {
        const int off[3] = {o % 3 - 1, (o / 3) % 3 - 1, o / 9 - 1};
        int b = 0, st = 1;
        bool in = true;
        for (int ax = 0; ax < d; ++ax) {
            const int cb = c[ax] + off[ax];
            in = in && cb >= 0 && cb < nn;
            b += cb * st;
            st *= nn;
        }
        if (!in) continue;
        const int fb = fnode[b];
        if (fb < 0 || l2g[cell * nloc + b] < 0) continue;
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j)
                M[((int64_t)fb * d + j) * nF + fa * d + i] = K[((int64_t)a * E + (o * d + i) * d + j) * cap + r];
    }
}

// dst[b][c ldd + r] = src[b strideS + (c0 + c) lds + r0 + r]
__global__ void k_copy_sub(int64_t rows, int64_t cols, int nb, const double *__restrict__ src, int64_t lds,
                           int64_t strideS, int64_t r0, int64_t c0, double *__restrict__ dst, int64_t ldd,
                           int64_t strideD, double scale)
{
    const int64_t t = (int64_t)blockIdx.x * NB + threadIdx.x;
    const int b = blockIdx.y;
    if (t >= rows * cols || b >= nb) return;
    const int64_t r = t % rows, c = t / rows;
    dst[b * strideD + c * ldd + r] = scale * src[b * strideS + (c0 + c) * lds + r0 + r];
}

// gather of index rows (and columns): dst[b][c ldd + r] = src[b strideS + idxc[c] lds + idxr[r]]
__global__ void k_gather_sub(int64_t rows, int64_t cols, int nb, int d, const int32_t *__restrict__ idxr_node,
                             const int32_t *__restrict__ idxc_node, const double *__restrict__ src, int64_t lds,
                             int64_t strideS, double *__restrict__ dst, int64_t ldd, int64_t strideD)
{
    const int64_t t = (int64_t)blockIdx.x * NB + threadIdx.x;
    const int b = blockIdx.y;
    if (t >= rows * cols || b >= nb) return;
    const int64_t r = t % rows, c = t / rows;
    const int64_t sr = (int64_t)idxr_node[r / d] * d + r % d;
    const int64_t sc = idxc_node ? (int64_t)idxc_node[c / d] * d + c % d : c;
    dst[b * strideD + c * ldd + r] = src[b * strideS + sc * lds + sr];
}

// non-definiteness check after a Cholesky factorisation: pivot L_ii^2 <= eps K_ii, or LAPACK info
__global__ void k_pivots(int64_t n, int nb, const double *__restrict__ L, int64_t strideL,
                         const double *__restrict__ Kdiag, const int32_t *__restrict__ info, int32_t *__restrict__ bad)
{
    const int b = blockIdx.x;
    if (b >= nb) return;
    __shared__ int flag;
    if (threadIdx.x == 0) flag = info[b] != 0;
    __syncthreads();
    for (int64_t i = threadIdx.x; i < n; i += NB) {
        const double l = L[b * strideL + i * n + i];
        if (!(l * l > 1e-12 * fabs(Kdiag[b * n + i]))) flag = 1;
    }
    __syncthreads();
    if (threadIdx.x == 0) bad[b] = flag;
}

// numerically singular LU factor: a pivot |U_ii| <= 1e-13 max_j |A_jj| (or not finite)
__global__ void k_lu_check(int64_t n, const double *__restrict__ U, const double *__restrict__ dg,
                           int32_t *__restrict__ sing)
{
    __shared__ double sh[NB];
    __shared__ int flag;
    double mx = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += NB) mx = fmax(mx, fabs(dg[i]));
    sh[threadIdx.x] = mx;
    if (threadIdx.x == 0) flag = 0;
    __syncthreads();
    for (int s = NB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    const double scale = sh[0];
    for (int64_t i = threadIdx.x; i < n; i += NB) {
        const double u = U[i * n + i];
        if (!(fabs(u) > 1e-13 * scale)) flag = 1;
    }
    __syncthreads();
    if (threadIdx.x == 0) *sing = flag;
}

__global__ void k_diag(int64_t n, int nb, const double *__restrict__ A, int64_t strideA, double *__restrict__ dg)
{
    const int64_t t = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (t >= n * nb) return;
    const int64_t b = t / n, i = t % n;
    dg[t] = A[b * strideA + i * n + i];
}

// copy the lower triangle to the upper one (column-major, batched)
__global__ void k_symm(int64_t n, int nb, double *__restrict__ A, int64_t strideA)
{
    const int64_t t = (int64_t)blockIdx.x * NB + threadIdx.x;
    const int b = blockIdx.y;
    if (t >= n * n || b >= nb) return;
    const int64_t i = t % n, j = t / n;
    if (i < j) A[b * strideA + j * n + i] = A[b * strideA + i * n + j];
}

// per-lane reduced-basis coordinates over the first nd principal cells:
// R[:nd,:nd] delta = nu beta[:nd] (back substitution); alpha itself when nd == n_r or R is absent
__global__ void k_delta(int64_t ld, int nd, int n_r, int cap, const int32_t *__restrict__ perm,
                        const double *__restrict__ alpha, const double *__restrict__ R, const double *__restrict__ nu,
                        const double *__restrict__ beta, double *__restrict__ delta)
{
    const int64_t lane = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (lane >= ld) return;
    const int cell = perm[lane];
    double *dl = delta + lane * nd;
    if (cell < 0) {
        for (int r = 0; r < nd; ++r) dl[r] = 0.0;
        return;
    }
    if (nd == n_r || !R) {
        for (int r = 0; r < nd; ++r) dl[r] = alpha[(int64_t)cell * cap + r];
        return;
    }
    for (int j = nd - 1; j >= 0; --j) {
        double v = nu[cell] * beta[(int64_t)cell * cap + j];
        for (int k = j + 1; k < nd; ++k) v -= R[(int64_t)j * cap + k] * dl[k];
        dl[j] = R[(int64_t)j * cap + j] != 0.0 ? v / R[(int64_t)j * cap + j] : 0.0;
    }
}

// one-hot coordinates: delta^s = e_r for the principal cell r < nd nearest to cell s in snapshot
// space, ||t_s - t_{s_r}||^2 = nu_s^2 + nu_{s_r}^2 - 2 nu_s sum_{j <= r} beta_j^s R[j][r] (the greedy's
// final residual of s is orthogonal to every basis vector); ties go to the lowest r
__global__ void k_delta_nearest(int64_t ld, int nd, int cap, const int32_t *__restrict__ perm,
                                const int32_t *__restrict__ S, const double *__restrict__ R,
                                const double *__restrict__ nu, const double *__restrict__ beta,
                                double *__restrict__ delta)
{
    const int64_t lane = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (lane >= ld) return;
    const int cell = perm[lane];
    double *dl = delta + lane * nd;
    for (int r = 0; r < nd; ++r) dl[r] = 0.0;
    if (cell < 0) return;
    const double ns = nu[cell];
    int best = 0;
    double bd = INFINITY;
    for (int r = 0; r < nd; ++r) {
        double dot = 0.0;
        for (int j = 0; j <= r; ++j) dot = fma(beta[(int64_t)cell * cap + j], R[(int64_t)j * cap + r], dot);
        const double nr = nu[S[r]];
        const double d2 = ns * ns + nr * nr - 2.0 * ns * dot;
        if (d2 < bd) { bd = d2; best = r; }
    }
    dl[best] = 1.0;
}

// lane gather / scatter of a local block vector [rows][ld] into the principal-cell order:
// xg[j ld + k] = live ? x[j ld + order[k]] : 0 (k < nv), 0 past nv; x[j ld + order[k]] = xg[j ld + k]
__global__ void k_gather_lanes(int64_t rows, int64_t ld, int64_t nv, const int32_t *__restrict__ order,
                               const uint8_t *__restrict__ live, const double *__restrict__ x, double *__restrict__ xg)
{
    const int64_t t = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (t >= rows * ld) return;
    const int64_t k = t % ld, j = t / ld;
    double v = 0.0;
    if (k < nv) {
        const int64_t src = j * ld + order[k];
        v = (!live || live[src]) ? x[src] : 0.0;
    }
    xg[t] = v;
}

__global__ void k_scatter_lanes(int64_t rows, int64_t ld, int64_t nv, const int32_t *__restrict__ order,
                                const double *__restrict__ xg, double *__restrict__ x)
{
    const int64_t t = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (t >= rows * ld) return;
    const int64_t k = t % ld, j = t / ld;
    if (k < nv) x[j * ld + order[k]] = xg[t];
}

// Grouped product for the one-hot models, one launch for every principal cell (groups of 512+
// lanes, where a matrix-core library GEMM per group pays, go to rocBLAS):
//   C[k, n] = beta C[k, n] + sum_j X[k, j] op(M_r)[j, n]   for the lanes k of group r,
// X, C column-major [ld x ...] in group order, op(M_r) = M_r (K x N, ldm) or M_r^T (M_r N x K).
// A workgroup of 4 waves computes a 64-lane x 64-column tile of one group (tiles listed in `tiles`
// as (group, first lane, end lane)); K is staged through LDS 32 at a time and contracted on the FP64
// matrix cores: wave w owns lanes 16w..16w+15, four 16 x 16 output tiles, one v_mfma_f64_16x16x4
// per tile and k-step (A = the lanes' X from LDS, B = the block's columns).  The principal block
// is read once per 64 lanes of its group; FP32 blocks are widened on the way into LDS.
constexpr int GT = 64, GK = 32;
constexpr int64_t GBIG = 512;   // groups this large go to rocBLAS (FP64 blocks only)
typedef double feti_v4d __attribute__((ext_vector_type(4)));
template <bool TRANS, class MT>
__global__ __launch_bounds__(256) void k_grouped_gemm(int64_t ld, int64_t N, int64_t K, int64_t Kc,
                                                      const int32_t *__restrict__ tiles, const double *__restrict__ X,
                                                      const MT *__restrict__ M, int64_t ldm, int64_t strideM,
                                                      double beta, double *__restrict__ C, double *__restrict__ part)
{
    __shared__ double xs[GK][GT + 1];
    __shared__ double ms[GK][GT + 1];
    const int r = tiles[3 * blockIdx.y], k0 = tiles[3 * blockIdx.y + 1], k1 = tiles[3 * blockIdx.y + 2];
    const int64_t n0 = (int64_t)blockIdx.x * GT;
    const int64_t jb = (int64_t)blockIdx.z * Kc, je = min(K, jb + Kc);   // this split's share of K
    const MT *Mr = M + (int64_t)r * strideM;
    const int t = threadIdx.x;
    const int w = t >> 6, l = t & 63;
    constexpr int PT = GK * GT / 256;                    // staged values per thread and operand
    double xr[PT], mr[PT];
    // the next k-stage's operands into registers (issued before the current stage's products)
    auto gload = [&](int64_t j0) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < PT; ++q) {
            const int e = t + 256 * q;
            {
                const int kk = e / GT, row = e % GT;
                const int64_t j = j0 + kk, k = k0 + row;
                xr[q] = (j < je && k < k1) ? X[j * ld + k] : 0.0;
            }
            int kk, c;
            if (TRANS) { kk = e / GT; c = e % GT; }      // M[(j) ldm + n]: n fastest
            else { c = e / GK; kk = e % GK; }             // M[(n) ldm + j]: j fastest
            const int64_t j = j0 + kk, n = n0 + c;
            mr[q] = (j < je && n < N) ? (double)(TRANS ? Mr[j * ldm + n] : Mr[n * ldm + j]) : 0.0;
        }
    };
    feti_v4d acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = feti_v4d{0.0, 0.0, 0.0, 0.0};
    if (jb < je) gload(jb);
    for (int64_t j0 = jb; j0 < je; j0 += GK) {
#pragma unroll
        for (int q = 0; q < PT; ++q) {
            const int e = t + 256 * q;
            xs[e / GT][e % GT] = xr[q];
            if (TRANS) ms[e / GT][e % GT] = mr[q];
            else ms[e % GK][e / GK] = mr[q];
        }
        __syncthreads();
        if (j0 + GK < je) gload(j0 + GK);
#pragma unroll
        for (int kk = 0; kk < GK; kk += 4) {
            const double a = xs[kk + (l >> 4)][16 * w + (l & 15)];
#pragma unroll
            for (int c = 0; c < 4; ++c)
                acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, ms[kk + (l >> 4)][16 * c + (l & 15)], acc[c], 0, 0, 0);
        }
        __syncthreads();
    }
    // output element (row (l / 16) + 4 q, column l % 16) of each 16 x 16 tile; a split writes its
    // partial sums, reduced in split order by k_split_sum
    double *out = gridDim.z > 1 ? part + (int64_t)blockIdx.z * N * ld : C;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int64_t n = n0 + 16 * c + (l & 15);
        if (n >= N) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t k = k0 + 16 * w + (l >> 4) + 4 * q;
            if (k >= k1) continue;
            const int64_t idx = n * ld + k;
            out[idx] = (gridDim.z > 1 || beta == 0.0) ? acc[c][q] : fma(beta, C[idx], acc[c][q]);
        }
    }
}

// C = beta C + sum_z part[z] over the lanes in group order (z ascending), rows < nv
__global__ void k_split_sum(int64_t ld, int64_t N, int64_t nv, int nz, const double *__restrict__ part, double beta,
                            double *__restrict__ C)
{
    const int64_t t = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (t >= N * ld) return;
    if (t % ld >= nv) return;
    double acc = 0.0;
    for (int z = 0; z < nz; ++z) acc += part[(int64_t)z * N * ld + t];
    C[t] = beta == 0.0 ? acc : fma(beta, C[t], acc);
}

// local coarse matrices of the one-hot models: C[lane] = S_{sel[lane]} (zero for padding lanes)
__global__ void k_select_spp(int64_t np2, int64_t ld, const int32_t *__restrict__ sel, const double *__restrict__ Spp,
                             double *__restrict__ C)
{
    const int64_t t = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (t >= np2 * ld) return;
    const int64_t lane = t / np2, e = t % np2;
    const int r = sel[lane];
    C[t] = r >= 0 ? Spp[(int64_t)r * np2 + e] : 0.0;
}

// principal cell of each lane under one-hot coordinates (-1 for padding lanes)
__global__ void k_to_f32(int64_t n, const double *__restrict__ x, float *__restrict__ y)
{
    for (int64_t j = (int64_t)blockIdx.x * NB + threadIdx.x; j < n; j += (int64_t)gridDim.x * NB) y[j] = (float)x[j];
}

__global__ void k_onehot_sel(int64_t ld, int nd, const double *__restrict__ delta, int32_t *__restrict__ sel)
{
    const int64_t lane = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (lane >= ld) return;
    int r = -1;
    for (int k = 0; k < nd; ++k)
        if (delta[lane * nd + k] != 0.0) r = k;
    sel[lane] = r;
}

// assembled coarse matrix (column-major, n = nPg d): row thread (G, i) sums its owners' local
// matrices C[lane][(p2 d + j) nP + p1 d + i] in ascending cell id; identity on prescribed rows
__global__ void k_coarse_asm(int d, int nPn, int64_t ld, int64_t nPg, const int32_t *__restrict__ pg_off,
                             const int32_t *__restrict__ pg_lane, const int32_t *__restrict__ pg_p,
                             const int32_t *__restrict__ prim_g, const uint8_t *__restrict__ liveP,
                             const double *__restrict__ C, double *__restrict__ S)
{
    const int64_t row = (int64_t)blockIdx.x * NB + threadIdx.x;
    const int64_t n = nPg * d;
    if (row >= n) return;
    const int64_t G = row / d;
    const int i = (int)(row % d);
    const int64_t nP = (int64_t)nPn * d;
    if (!liveP[row]) {
        S[row * n + row] = 1.0;
        return;
    }
    for (int k = pg_off[G]; k < pg_off[G + 1]; ++k) {
        const int64_t lane = pg_lane[k];
        const int p1 = pg_p[k];
        const double *Cl = C + lane * nP * nP;
        for (int p2 = 0; p2 < nPn; ++p2) {
            const int32_t G2 = prim_g[(int64_t)p2 * ld + lane];
            if (G2 < 0) continue;
            for (int j = 0; j < d; ++j) {
                const int64_t col = (int64_t)G2 * d + j;
                if (!liveP[col]) continue;
                S[col * n + row] += Cl[((int64_t)p2 * d + j) * nP + (int64_t)p1 * d + i];
            }
        }
    }
}

// right-hand side split: b_R = b / (owners) on the remaining rows, b_P = b on the primal nodes
__global__ void k_rhs(int d, int nloc, int nRn, int64_t ld, const int32_t *__restrict__ rnode,
                      const int32_t *__restrict__ perm, const int32_t *__restrict__ l2g,
                      const int32_t *__restrict__ gn_off, const uint8_t *__restrict__ liveR,
                      const uint8_t *__restrict__ fixed, const double *__restrict__ b, double *__restrict__ bR)
{
    const int64_t t = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (t >= (int64_t)nRn * ld) return;
    const int64_t lane = t % ld;
    const int rn = (int)(t / ld);
    const int cell = perm[lane];
    const int32_t g = cell >= 0 ? l2g[(int64_t)cell * nloc + rnode[rn]] : -1;
    for (int i = 0; i < d; ++i) {
        const int64_t r = ((int64_t)rn * d + i) * ld + lane;
        bR[r] = (liveR[r] && !fixed[(int64_t)g * d + i]) ? b[(int64_t)g * d + i] / (double)(gn_off[g + 1] - gn_off[g])
                                                        : 0.0;
    }
}

__global__ void k_rhs_P(int d, int64_t nPg, const int64_t *__restrict__ pglob, const uint8_t *__restrict__ liveP,
                        const double *__restrict__ b, double *__restrict__ bP)
{
    const int64_t G = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (G >= nPg) return;
    for (int i = 0; i < d; ++i) bP[G * d + i] = liveP[G * d + i] ? b[pglob[G] * d + i] : 0.0;
}

// global solution: u_P on primal nodes, the owners' mean of u_R elsewhere, 0 on prescribed ones
__global__ void k_solution(int d, int64_t nglobal, int nRn, int64_t ld, const int32_t *__restrict__ gn_off,
                           const int32_t *__restrict__ gn_lane, const int32_t *__restrict__ gn_fn,
                           const int32_t *__restrict__ gp_of_g, const uint8_t *__restrict__ fixed,
                           const double *__restrict__ uR, const double *__restrict__ uP, double *__restrict__ x)
{
    const int64_t g = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (g >= nglobal) return;
    const int32_t G = gp_of_g[g];
    for (int i = 0; i < d; ++i) {
        double v = 0.0;
        if (!fixed[g * d + i]) {
            if (G >= 0) {
                v = uP[(int64_t)G * d + i];
            } else {
                const int k0 = gn_off[g], k1 = gn_off[g + 1];
                for (int k = k0; k < k1; ++k) v += uR[((int64_t)gn_fn[k] * d + i) * ld + gn_lane[k]];
                v = k1 > k0 ? v / (double)(k1 - k0) : 0.0;
            }
        }
        x[g * d + i] = v;
    }
}

// fixed-order dot products: per-block partials, summed on the host or by k_pcg_* in index order
__global__ void k_dot_part(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                           double *__restrict__ part)
{
    __shared__ double sh[NB];
    double acc = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * NB + threadIdx.x; j < n; j += (int64_t)gridDim.x * NB)
        acc = fma(x[j], y[j], acc);
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = NB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__device__ double sum_part(int nb, const double *__restrict__ part)
{
    __shared__ double sh[NB];
    double acc = 0.0;
    for (int j = threadIdx.x; j < nb; j += NB) acc += part[j];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = NB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// PCG scalars of the interface sub-solve
struct PcgCtl {
    double rz, alpha, beta, rz0;
    int32_t stop;     // breakdown (r.z or p.q not positive and finite): no further updates
    int32_t conv;     // r.z has fallen below tol2 rz0 (the relative inner tolerance)
};

__global__ void k_pcg_init(int nb, const double *__restrict__ part, PcgCtl *c)
{
    const double rz = sum_part(nb, part);
    if (threadIdx.x == 0) {
        c->rz = rz;
        c->rz0 = rz;
        c->stop = !(rz > 0.0) || !isfinite(rz);
        c->conv = 0;
        c->alpha = c->beta = 0.0;
    }
}

__global__ void k_pcg_alpha(int nb, const double *__restrict__ part, PcgCtl *c)
{
    const double pq = sum_part(nb, part);
    if (threadIdx.x == 0 && !c->stop) {
        if (!(pq > 0.0) || !isfinite(pq)) { c->stop = 1; c->alpha = 0.0; }
        else c->alpha = c->rz / pq;
    }
}

__global__ void k_pcg_beta(int nb, const double *__restrict__ part, double tol2, PcgCtl *c)
{
    const double rz = sum_part(nb, part);
    if (threadIdx.x == 0 && !c->stop) {
        if (!(rz > 0.0) || !isfinite(rz)) { c->stop = 1; c->beta = 0.0; }
        else { c->beta = rz / c->rz; c->rz = rz; }
        if (tol2 > 0.0 && !(rz > tol2 * c->rz0)) c->conv = 1;
    }
}

// x += alpha p; r -= alpha q
__global__ void k_pcg_xr(int64_t n, const PcgCtl *c, const double *__restrict__ p, const double *__restrict__ q,
                         double *__restrict__ x, double *__restrict__ r)
{
    if (c->stop) return;
    const double a = c->alpha;
    for (int64_t j = (int64_t)blockIdx.x * NB + threadIdx.x; j < n; j += (int64_t)gridDim.x * NB) {
        x[j] = fma(a, p[j], x[j]);
        r[j] = fma(-a, q[j], r[j]);
    }
}

// p = z + beta p
__global__ void k_pcg_p(int64_t n, const PcgCtl *c, const double *__restrict__ z, double *__restrict__ p)
{
    if (c->stop) return;
    const double b = c->beta;
    for (int64_t j = (int64_t)blockIdx.x * NB + threadIdx.x; j < n; j += (int64_t)gridDim.x * NB) p[j] = fma(b, p[j], z[j]);
}

__global__ void k_axpby(int64_t n, double a, const double *__restrict__ x, double b, double *__restrict__ y)
{
    for (int64_t j = (int64_t)blockIdx.x * NB + threadIdx.x; j < n; j += (int64_t)gridDim.x * NB) y[j] = a * x[j] + b * y[j];
}

__global__ void k_copy(int64_t n, const double *__restrict__ x, double *__restrict__ y)
{
    for (int64_t j = (int64_t)blockIdx.x * NB + threadIdx.x; j < n; j += (int64_t)gridDim.x * NB) y[j] = x[j];
}

// ------------------------------------------------------------------------------------------
// Solver state
// ------------------------------------------------------------------------------------------
constexpr int DOT_BLOCKS = 1024;

struct Feti {
    const lat_plan *P = nullptr;
    hipStream_t s = nullptr;
    rocblas_handle h = nullptr;
    Part pt;
    PartDev pd{};
    int d = 0, nd = 0, n_r = 0;
    int64_t ld = 0, nRr = 0, nPr = 0, nDr = 0, nPgd = 0, L = 0, Lint = 0, nF = 0, Nv = 0;
    // operator
    const double *K = nullptr, *alpha = nullptr, *ops = nullptr;
    double *Xpk = nullptr, *Ypk = nullptr;
    uint8_t *liveR = nullptr, *liveP = nullptr, *liveL = nullptr, *liveD = nullptr;
    // reduced models over the principal cells
    float *G32 = nullptr;            // FP32 copy of the G_r (reduced-precision local solves)
    double *split = nullptr;         // split-K partial sums of the grouped products
    int64_t split_rows = 0;          // their capacity, in output columns x splits
    bool g32 = false;
    double *G = nullptr, *Phi = nullptr, *Spp = nullptr, *Fdd = nullptr, *Sdd = nullptr, *Phid = nullptr;
    double *delta = nullptr, *Sc = nullptr;   // [ld][nd], coarse inverse [nPgd]^2
    double *cmv = nullptr;                    // chunk partials of the coarse product [nPgd / CMV_W][nPgd]
    // scratch
    double *As = nullptr, *xm = nullptr, *T1 = nullptr, *hl = nullptr, *hP = nullptr, *uP = nullptr, *el = nullptr;
    double *qd = nullptr, *vd = nullptr;
    double *part = nullptr, *hpart = nullptr;
    PcgCtl *pc = nullptr;
    double *px = nullptr, *pr = nullptr, *pz = nullptr, *pp = nullptr, *pq = nullptr;
    double *w1 = nullptr, *w2 = nullptr, *w3 = nullptr;   // full-length work vectors
    int inner_it = 0;
    double inner_tol2 = 0.0;        // squared relative tolerance of the interface sub-solve (0: fixed steps)
    int n_shift = 0;        // principal remaining blocks that are not positive definite
    double max_shift = 0.0; // largest diagonal shift (indef_mode 0)
    int indef_mode = 0;     // 0: shift to definiteness; 1: pivoted-LU inverses, interface by its Dirichlet preconditioner
    int coords = 0;         // 0: least-squares coordinates; 1: nearest principal cell
    // one-hot coordinates: lanes grouped by principal cell (order[off[r] .. off[r+1]) use r)
    bool onehot = false;
    int32_t *order = nullptr;
    int32_t *tiles = nullptr;       // (group, first lane, end lane) per 64-lane tile of the small groups
    int64_t ntiles = 0;
    std::vector<int> big;           // groups of at least GBIG lanes: one rocBLAS GEMM each
    std::vector<int64_t> off;
    int64_t nv = 0;          // lanes with a principal cell (padding lanes excluded)
    double *Xg = nullptr, *Yg = nullptr;
};

// GEMM wrapper (column-major, FP64)
lat_status gemm(const Feti &f, rocblas_operation ta, rocblas_operation tb, int64_t m, int64_t n, int64_t k,
                double alpha, const double *A, int64_t lda, const double *B, int64_t ldb, double beta, double *C,
                int64_t ldc)
{
    if (m == 0 || n == 0) return LAT_OK;
    if (k == 0) {                   // an empty sum (every call here has ldc == m)
        if (beta == 0.0) {
            hipLaunchKernelGGL(k_ffill, dim3(blocks(m * n)), dim3(NB), 0, f.s, m * n, 0.0, C);
            LAT_LAUNCH_CHECK();
        }
        return LAT_OK;
    }
    if (m > INT32_MAX || n > INT32_MAX || k > INT32_MAX || lda > INT32_MAX || ldb > INT32_MAX || ldc > INT32_MAX)
        return LAT_E_SHAPE;
    RBCHK(rocblas_dgemm(f.h, ta, tb, (rocblas_int)m, (rocblas_int)n, (rocblas_int)k, &alpha, A, (rocblas_int)lda, B,
                        (rocblas_int)ldb, &beta, C, (rocblas_int)ldc));
    return LAT_OK;
}

// x (n) dot y -> host value, fixed order
lat_status dot_host(Feti &f, int64_t n, const double *x, const double *y, double *out)
{
    hipLaunchKernelGGL(k_dot_part, dim3(DOT_BLOCKS), dim3(NB), 0, f.s, n, x, y, f.part);
    LAT_LAUNCH_CHECK();
    std::vector<double> h(DOT_BLOCKS);
    LAT_HIP(hipMemcpyAsync(h.data(), f.part, DOT_BLOCKS * sizeof(double), hipMemcpyDeviceToHost, f.s));
    LAT_HIP(hipStreamSynchronize(f.s));
    double acc = 0.0;
    for (double v : h) acc += v;
    *out = acc;
    return LAT_OK;
}

// the saddle-point operator: out = A w
lat_status op_apply(Feti &f, const double *w, double *out)
{
    const lat_plan *P = f.P;
    const double *wR = w, *wP = w + f.nRr * f.ld, *wL = wP + f.nPgd;
    double *oR = out, *oP = out + f.nRr * f.ld, *oL = oP + f.nPgd;
    const int32_t *qgroup = P->goff + P->ngroups + 1;
    hipLaunchKernelGGL(k_to_packed, dim3(blocks(P->npacked * LAT_WAVE)), dim3(NB), 0, f.s, f.d, (int64_t)P->npacked,
                       P->nloc, f.pt.nRn, f.ld, qgroup, P->unode, P->umask, f.pd.fnode, f.pd.prim_g, f.liveR, f.liveP,
                       wR, wP, f.Xpk);
    LAT_LAUNCH_CHECK();
    if (f.ops) FCHK(lat_apply_plain(P, f.ops, f.Xpk, f.Ypk, 1, f.s));
    else FCHK(lat_apply_combo(P, f.K, f.n_r, f.alpha, f.Xpk, f.Ypk, 1, LAT_F64, 0.0, 0, nullptr, nullptr, 0, f.s));
    hipLaunchKernelGGL(k_from_packed_R, dim3(blocks((int64_t)f.pt.nRn * f.ld)), dim3(NB), 0, f.s, f.d, P->nloc,
                       f.pt.nRn, f.ld, f.pd.rnode, P->uidx, P->goff, f.liveR, f.Ypk, wR, oR);
    hipLaunchKernelGGL(k_from_packed_P, dim3(blocks(f.pt.nPg)), dim3(NB), 0, f.s, f.d, P->nloc, f.pt.nPg, f.pd.pg_off,
                       f.pd.pg_lane, f.pd.pg_p, f.pd.pnode, P->uidx, P->goff, f.liveP, f.Ypk, wP, oP);
    hipLaunchKernelGGL(k_bt_add, dim3(blocks(f.pt.nsets)), dim3(NB), 0, f.s, f.d, f.pt.nsets, f.ld, f.pd.set_off,
                       f.pd.set_m0, f.pd.mem_lane, f.pd.mem_rn, f.liveL, wL, oR);
    hipLaunchKernelGGL(k_b, dim3(blocks(f.pt.nsets)), dim3(NB), 0, f.s, f.d, f.pt.nsets, f.ld, f.pd.set_off, f.pd.set_m0,
                       f.pd.mem_lane, f.pd.mem_rn, f.liveL, wR, wL, oL);
    hipLaunchKernelGGL(k_dir_bt, dim3(blocks(f.pt.ndir)), dim3(NB), 0, f.s, f.d, f.pt.ndir, f.ld, f.Lint, f.pd.dir_lane,
                       f.pd.dir_rn, f.pd.dir_i, wL, oR);
    hipLaunchKernelGGL(k_dir_b, dim3(blocks(f.pt.ndir)), dim3(NB), 0, f.s, f.d, f.pt.ndir, f.ld, f.Lint, f.pd.dir_lane,
                       f.pd.dir_rn, f.pd.dir_i, wR, oL);
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

// y = A x for the coarse inverse A (n x n, column-major): workgroups of 256 rows x one chunk of CMV_W
// columns (about a thousand of them for the coarse sizes here, where a library matrix-vector
// product launches a few dozen and streams the matrix at a tenth of the chip's bandwidth), each
// thread summing its row over the chunk in column order; k_cmv_sum adds the chunks in order.
constexpr int CMV_W = 64;
__global__ __launch_bounds__(256) void k_cmv_part(int64_t n, const double *__restrict__ A, const double *__restrict__ x,
                                                  double *__restrict__ part)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.y * CMV_W, j1 = j0 + CMV_W < n ? j0 + CMV_W : n;
    if (i >= n) return;
    double s = 0.0;
    for (int64_t j = j0; j < j1; ++j) s = fma(A[j * n + i], x[j], s);
    part[(int64_t)blockIdx.y * n + i] = s;
}

__global__ void k_cmv_sum(int64_t n, int nc, const double *__restrict__ part, double *__restrict__ y)
{
    const int64_t i = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int c = 0; c < nc; ++c) s += part[(int64_t)c * n + i];
    y[i] = s;
}

// coarse part shared by K~rom^-1 and F~: given t = sum_r delta_r Phi_r^T g (per cell, [nP][ld])
// in f.T1 layout, h_P = base + assembled, u_P = Sc^-1 h_P, el = gathered u_P
lat_status coarse_part(Feti &f, const double *base)
{
    if (f.onehot)   // the per-group products were scattered back into lane order already
        hipLaunchKernelGGL(k_scatter_lanes, dim3(blocks(f.nPr * f.ld)), dim3(NB), 0, f.s, f.nPr, f.ld, f.nv, f.order,
                           (const double *)f.T1, f.hl);
    else
        hipLaunchKernelGGL(k_combine_delta, dim3(blocks(f.nPr * f.ld)), dim3(NB), 0, f.s, f.nPr, f.ld, f.nd, f.delta,
                           f.T1, f.hl);
    hipLaunchKernelGGL(k_assemble_P, dim3(blocks(f.pt.nPg)), dim3(NB), 0, f.s, f.d, f.ld, f.pt.nPg, f.pd.pg_off,
                       f.pd.pg_lane, f.pd.pg_p, f.liveP, f.hl, base, f.hP);
    LAT_LAUNCH_CHECK();
    if (f.nPgd > 0) {
        const int64_t nc = lat_cdiv(f.nPgd, CMV_W);
        hipLaunchKernelGGL(k_cmv_part, dim3((unsigned)lat_cdiv(f.nPgd, 256), (unsigned)nc), dim3(256), 0, f.s, f.nPgd,
                           (const double *)f.Sc, (const double *)f.hP, f.cmv);
        hipLaunchKernelGGL(k_cmv_sum, dim3(blocks(f.nPgd)), dim3(NB), 0, f.s, f.nPgd, (int)nc, (const double *)f.cmv,
                           f.uP);
        LAT_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_gather_P, dim3(blocks((int64_t)f.pt.nPn * f.ld)), dim3(NB), 0, f.s, f.d, f.pt.nPn, f.ld,
                       f.pd.prim_g, f.liveP, f.uP, f.el);
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

// one-hot models: C_g[off_r .., :] (op) = X_g[off_r .., :] M_r (op(M_r)) for every principal cell r,
// lanes in group order (column-major [ld x k] blocks, M_r [k x n] or its transpose)
template <class MT>
lat_status grouped_launch(Feti &f, rocblas_operation tm, int64_t n, int64_t k, const double *Xg, const MT *M,
                          int64_t ldm, int64_t strideM, double beta, double *Cg)
{
    // split K when the output tiles alone would leave the chip idle (narrow products)
    const int64_t ct = lat_cdiv(n, GT);
    int64_t nz = 1;
    // (only without rocBLAS-served groups: the partial sums cover every lane of the small groups)
    while (f.big.empty() && nz < 64 && ct * f.ntiles * nz < 1024 && lat_cdiv(k, GK) >= 4 * nz &&
           (nz * 2) * n <= f.split_rows)
        nz *= 2;
    const int64_t Kc = lat_cdiv(lat_cdiv(k, nz), GK) * GK;
    const dim3 grid((unsigned)ct, (unsigned)f.ntiles, (unsigned)nz);
    if (tm == rocblas_operation_none)
        hipLaunchKernelGGL((k_grouped_gemm<false, MT>), grid, dim3(256), 0, f.s, f.ld, n, k, Kc, (const int32_t *)f.tiles,
                           Xg, M, ldm, strideM, beta, Cg, f.split);
    else
        hipLaunchKernelGGL((k_grouped_gemm<true, MT>), grid, dim3(256), 0, f.s, f.ld, n, k, Kc, (const int32_t *)f.tiles,
                           Xg, M, ldm, strideM, beta, Cg, f.split);
    if (nz > 1)
        hipLaunchKernelGGL(k_split_sum, dim3(blocks(n * f.ld)), dim3(NB), 0, f.s, f.ld, n, f.nv, (int)nz,
                           (const double *)f.split, beta, Cg);
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

lat_status grouped(Feti &f, rocblas_operation tm, int64_t n, int64_t k, const double *Xg, const double *M,
                   int64_t ldm, int64_t strideM, double beta, double *Cg)
{
    if (n == 0) return LAT_OK;
    for (int r : f.big) {
        const int64_t m = f.off[(size_t)r + 1] - f.off[(size_t)r];
        FCHK(gemm(f, rocblas_operation_none, tm, m, n, k, 1.0, Xg + f.off[(size_t)r], f.ld, M + (int64_t)r * strideM, ldm,
                  beta, Cg + f.off[(size_t)r], f.ld));
    }
    if (f.ntiles == 0) return LAT_OK;
    return grouped_launch<double>(f, tm, n, k, Xg, M, ldm, strideM, beta, Cg);
}

// the local solves' blocks G_r, in FP32 when the reduced-precision inner apply is on (every group
// then goes through the grouped kernel)
lat_status grouped_G(Feti &f, int64_t nR, const double *Xg, double beta, double *Cg)
{
    if (f.g32) return f.ntiles ? grouped_launch<float>(f, rocblas_operation_none, nR, nR, Xg, f.G32, nR, nR * nR, beta, Cg)
                               : LAT_OK;
    return grouped(f, rocblas_operation_none, nR, nR, Xg, f.G, nR, nR * nR, beta, Cg);
}

// K~rom^-1 with one-hot models: every cell's local operators are its principal cell's
lat_status krom_onehot(Feti &f, const double *gR, const double *gP, double *zR, double *zP)
{
    const int64_t nR = f.nRr, ld = f.ld, nP = f.nPr;
    hipLaunchKernelGGL(k_gather_lanes, dim3(blocks(nR * ld)), dim3(NB), 0, f.s, nR, ld, f.nv, f.order, f.liveR, gR, f.Xg);
    LAT_LAUNCH_CHECK();
    FCHK(grouped_G(f, nR, f.Xg, 0.0, f.Yg));
    FCHK(grouped(f, rocblas_operation_none, nP, nR, f.Xg, f.Phi, nR, nR * nP, 0.0, f.T1));
    FCHK(coarse_part(f, gP));
    hipLaunchKernelGGL(k_gather_lanes, dim3(blocks(nP * ld)), dim3(NB), 0, f.s, nP, ld, f.nv, f.order,
                       (const uint8_t *)nullptr, (const double *)f.el, f.As);
    LAT_LAUNCH_CHECK();
    FCHK(grouped(f, rocblas_operation_transpose, nR, nP, f.As, f.Phi, nR, nR * nP, 1.0, f.Yg));
    hipLaunchKernelGGL(k_ffill, dim3(blocks(nR * ld)), dim3(NB), 0, f.s, nR * ld, 0.0, zR);
    hipLaunchKernelGGL(k_scatter_lanes, dim3(blocks(nR * ld)), dim3(NB), 0, f.s, nR, ld, f.nv, f.order,
                       (const double *)f.Yg, zR);
    hipLaunchKernelGGL(k_identity_rows, dim3(blocks(nR * ld)), dim3(NB), 0, f.s, nR * ld, f.liveR, gR, zR);
    if (zP != f.uP)
        hipLaunchKernelGGL(k_copy, dim3(blocks(f.nPgd)), dim3(NB), 0, f.s, f.nPgd, (const double *)f.uP, zP);
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

// (zR, zP) = K~rom^-1 (gR, gP); identity on rows that do not exist
lat_status krom(Feti &f, const double *gR, const double *gP, double *zR, double *zP)
{
    if (f.onehot) return krom_onehot(f, gR, gP, zR, zP);
    const int64_t nR = f.nRr, ld = f.ld, nd = f.nd, nP = f.nPr;
    hipLaunchKernelGGL(k_scale_stack, dim3(blocks(nR * ld)), dim3(NB), 0, f.s, nR, ld, f.nd, f.delta, f.liveR, gR,
                       f.xm, f.As);
    LAT_LAUNCH_CHECK();
    // local solves: zR = sum_r diag(delta_r) g G_r
    FCHK(gemm(f, rocblas_operation_none, rocblas_operation_transpose, ld, nR, nd * nR, 1.0, f.As, ld, f.G, nR, 0.0,
              zR, ld));
    // coarse: t = g Phi_r per principal cell, combined per lane
    FCHK(gemm(f, rocblas_operation_none, rocblas_operation_none, ld, nd * nP, nR, 1.0, f.xm, ld, f.Phi, nR, 0.0, f.T1,
              ld));
    FCHK(coarse_part(f, gP));
    // zR += sum_r diag(delta_r) e Phi_r^T
    hipLaunchKernelGGL(k_scale_stack, dim3(blocks(nP * ld)), dim3(NB), 0, f.s, nP, ld, f.nd, f.delta,
                       (const uint8_t *)nullptr, f.el, (double *)nullptr, f.As);
    LAT_LAUNCH_CHECK();
    FCHK(gemm(f, rocblas_operation_none, rocblas_operation_transpose, ld, nR, nd * nP, 1.0, f.As, ld, f.Phi, nR, 1.0,
              zR, ld));
    hipLaunchKernelGGL(k_identity_rows, dim3(blocks(nR * ld)), dim3(NB), 0, f.s, nR * ld, f.liveR, gR, zR);
    if (zP != f.uP)
        hipLaunchKernelGGL(k_copy, dim3(blocks(f.nPgd)), dim3(NB), 0, f.s, f.nPgd, (const double *)f.uP, zP);
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

// out = F~ lam = B K~rom^-1 B^T lam, from the dual blocks
lat_status fdual(Feti &f, const double *lam, double *out)
{
    const int64_t nD = f.nDr, ld = f.ld, nd = f.nd, nP = f.nPr;
    hipLaunchKernelGGL(k_ffill, dim3(blocks(nD * ld)), dim3(NB), 0, f.s, nD * ld, 0.0, f.qd);
    hipLaunchKernelGGL(k_bt_dual, dim3(blocks(f.pt.nsets)), dim3(NB), 0, f.s, f.d, f.pt.nsets, ld, f.pd.set_off,
                       f.pd.set_m0, f.pd.mem_lane, f.pd.mem_dn, f.liveL, f.pd.bd, 0, lam, f.qd);
    hipLaunchKernelGGL(k_dir_bt, dim3(blocks(f.pt.ndir)), dim3(NB), 0, f.s, f.d, f.pt.ndir, ld, f.Lint, f.pd.dir_lane,
                       f.pd.dir_dn, f.pd.dir_i, lam, f.qd);
    if (f.onehot) {
        hipLaunchKernelGGL(k_gather_lanes, dim3(blocks(nD * ld)), dim3(NB), 0, f.s, nD, ld, f.nv, f.order, f.liveD,
                           (const double *)f.qd, f.Xg);
        LAT_LAUNCH_CHECK();
        FCHK(grouped(f, rocblas_operation_none, nD, nD, f.Xg, f.Fdd, nD, nD * nD, 0.0, f.Yg));
        FCHK(grouped(f, rocblas_operation_none, nP, nD, f.Xg, f.Phid, nD, nD * nP, 0.0, f.T1));
        FCHK(coarse_part(f, nullptr));
        hipLaunchKernelGGL(k_gather_lanes, dim3(blocks(nP * ld)), dim3(NB), 0, f.s, nP, ld, f.nv, f.order,
                           (const uint8_t *)nullptr, (const double *)f.el, f.As);
        LAT_LAUNCH_CHECK();
        FCHK(grouped(f, rocblas_operation_transpose, nD, nP, f.As, f.Phid, nD, nD * nP, 1.0, f.Yg));
        hipLaunchKernelGGL(k_ffill, dim3(blocks(nD * ld)), dim3(NB), 0, f.s, nD * ld, 0.0, f.vd);
        hipLaunchKernelGGL(k_scatter_lanes, dim3(blocks(nD * ld)), dim3(NB), 0, f.s, nD, ld, f.nv, f.order,
                           (const double *)f.Yg, f.vd);
        hipLaunchKernelGGL(k_b_dual, dim3(blocks(f.pt.nsets)), dim3(NB), 0, f.s, f.d, f.pt.nsets, ld, f.pd.set_off,
                           f.pd.set_m0, f.pd.mem_lane, f.pd.mem_dn, f.liveL, f.pd.bd, 0, (const double *)f.vd, lam, out);
        hipLaunchKernelGGL(k_dir_b, dim3(blocks(f.pt.ndir)), dim3(NB), 0, f.s, f.d, f.pt.ndir, ld, f.Lint, f.pd.dir_lane,
                           f.pd.dir_dn, f.pd.dir_i, (const double *)f.vd, out);
        LAT_LAUNCH_CHECK();
        return LAT_OK;
    }
    hipLaunchKernelGGL(k_scale_stack, dim3(blocks(nD * ld)), dim3(NB), 0, f.s, nD, ld, f.nd, f.delta, f.liveD, f.qd,
                       f.xm, f.As);
    LAT_LAUNCH_CHECK();
    FCHK(gemm(f, rocblas_operation_none, rocblas_operation_transpose, ld, nD, nd * nD, 1.0, f.As, ld, f.Fdd, nD, 0.0,
              f.vd, ld));
    FCHK(gemm(f, rocblas_operation_none, rocblas_operation_none, ld, nd * nP, nD, 1.0, f.xm, ld, f.Phid, nD, 0.0, f.T1,
              ld));
    FCHK(coarse_part(f, nullptr));
    hipLaunchKernelGGL(k_scale_stack, dim3(blocks(nP * ld)), dim3(NB), 0, f.s, nP, ld, f.nd, f.delta,
                       (const uint8_t *)nullptr, f.el, (double *)nullptr, f.As);
    LAT_LAUNCH_CHECK();
    FCHK(gemm(f, rocblas_operation_none, rocblas_operation_transpose, ld, nD, nd * nP, 1.0, f.As, ld, f.Phid, nD, 1.0,
              f.vd, ld));
    hipLaunchKernelGGL(k_b_dual, dim3(blocks(f.pt.nsets)), dim3(NB), 0, f.s, f.d, f.pt.nsets, ld, f.pd.set_off,
                       f.pd.set_m0, f.pd.mem_lane, f.pd.mem_dn, f.liveL, f.pd.bd, 0, (const double *)f.vd, lam, out);
    hipLaunchKernelGGL(k_dir_b, dim3(blocks(f.pt.ndir)), dim3(NB), 0, f.s, f.d, f.pt.ndir, ld, f.Lint, f.pd.dir_lane,
                       f.pd.dir_dn, f.pd.dir_i, (const double *)f.vd, out);
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

// out = B_D (sum_r delta_r S_dd^r) B_D^T r  (Dirichlet preconditioner of the interface problem)
lat_status dirichlet(Feti &f, const double *r, double *out)
{
    const int64_t nD = f.nDr, ld = f.ld, nd = f.nd;
    hipLaunchKernelGGL(k_ffill, dim3(blocks(nD * ld)), dim3(NB), 0, f.s, nD * ld, 0.0, f.qd);
    hipLaunchKernelGGL(k_bt_dual, dim3(blocks(f.pt.nsets)), dim3(NB), 0, f.s, f.d, f.pt.nsets, ld, f.pd.set_off,
                       f.pd.set_m0, f.pd.mem_lane, f.pd.mem_dn, f.liveL, f.pd.bd, 1, r, f.qd);
    hipLaunchKernelGGL(k_dir_bt, dim3(blocks(f.pt.ndir)), dim3(NB), 0, f.s, f.d, f.pt.ndir, ld, f.Lint, f.pd.dir_lane,
                       f.pd.dir_dn, f.pd.dir_i, r, f.qd);
    if (f.onehot) {
        hipLaunchKernelGGL(k_gather_lanes, dim3(blocks(nD * ld)), dim3(NB), 0, f.s, nD, ld, f.nv, f.order, f.liveD,
                           (const double *)f.qd, f.Xg);
        LAT_LAUNCH_CHECK();
        FCHK(grouped(f, rocblas_operation_none, nD, nD, f.Xg, f.Sdd, nD, nD * nD, 0.0, f.Yg));
        hipLaunchKernelGGL(k_ffill, dim3(blocks(nD * ld)), dim3(NB), 0, f.s, nD * ld, 0.0, f.vd);
        hipLaunchKernelGGL(k_scatter_lanes, dim3(blocks(nD * ld)), dim3(NB), 0, f.s, nD, ld, f.nv, f.order,
                           (const double *)f.Yg, f.vd);
        LAT_LAUNCH_CHECK();
    } else {
        hipLaunchKernelGGL(k_scale_stack, dim3(blocks(nD * ld)), dim3(NB), 0, f.s, nD, ld, f.nd, f.delta, f.liveD, f.qd,
                           (double *)nullptr, f.As);
        LAT_LAUNCH_CHECK();
        FCHK(gemm(f, rocblas_operation_none, rocblas_operation_transpose, ld, nD, nd * nD, 1.0, f.As, ld, f.Sdd, nD, 0.0,
                  f.vd, ld));
    }
    hipLaunchKernelGGL(k_b_dual, dim3(blocks(f.pt.nsets)), dim3(NB), 0, f.s, f.d, f.pt.nsets, ld, f.pd.set_off,
                       f.pd.set_m0, f.pd.mem_lane, f.pd.mem_dn, f.liveL, f.pd.bd, 1, (const double *)f.vd, r, out);
    hipLaunchKernelGGL(k_dir_b, dim3(blocks(f.pt.ndir)), dim3(NB), 0, f.s, f.d, f.pt.ndir, ld, f.Lint, f.pd.dir_lane,
                       f.pd.dir_dn, f.pd.dir_i, (const double *)f.vd, out);
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

// x ~ F~^-1 g: inner_it PCG steps from 0 (the Dirichlet preconditioner alone when inner_it = 0)
lat_status fpcg(Feti &f, const double *g, double *x)
{
    const int64_t n = f.L;
    if (n == 0) return LAT_OK;
    if (f.inner_it <= 0) return dirichlet(f, g, x);
    const unsigned bl = blocks(n);
    hipLaunchKernelGGL(k_ffill, dim3(bl), dim3(NB), 0, f.s, n, 0.0, x);
    hipLaunchKernelGGL(k_copy, dim3(bl), dim3(NB), 0, f.s, n, g, f.pr);
    LAT_LAUNCH_CHECK();
    FCHK(dirichlet(f, f.pr, f.pz));
    hipLaunchKernelGGL(k_copy, dim3(bl), dim3(NB), 0, f.s, n, (const double *)f.pz, f.pp);
    hipLaunchKernelGGL(k_dot_part, dim3(DOT_BLOCKS), dim3(NB), 0, f.s, n, (const double *)f.pr, (const double *)f.pz,
                       f.part);
    hipLaunchKernelGGL(k_pcg_init, dim3(1), dim3(NB), 0, f.s, DOT_BLOCKS, (const double *)f.part, f.pc);
    LAT_LAUNCH_CHECK();
    for (int it = 0; it < f.inner_it; ++it) {
        FCHK(fdual(f, f.pp, f.pq));
        hipLaunchKernelGGL(k_dot_part, dim3(DOT_BLOCKS), dim3(NB), 0, f.s, n, (const double *)f.pp,
                           (const double *)f.pq, f.part);
        hipLaunchKernelGGL(k_pcg_alpha, dim3(1), dim3(NB), 0, f.s, DOT_BLOCKS, (const double *)f.part, f.pc);
        hipLaunchKernelGGL(k_pcg_xr, dim3(bl), dim3(NB), 0, f.s, n, (const PcgCtl *)f.pc, (const double *)f.pp,
                           (const double *)f.pq, x, f.pr);
        LAT_LAUNCH_CHECK();
        if (it + 1 == f.inner_it) break;
        FCHK(dirichlet(f, f.pr, f.pz));
        hipLaunchKernelGGL(k_dot_part, dim3(DOT_BLOCKS), dim3(NB), 0, f.s, n, (const double *)f.pr,
                           (const double *)f.pz, f.part);
        hipLaunchKernelGGL(k_pcg_beta, dim3(1), dim3(NB), 0, f.s, DOT_BLOCKS, (const double *)f.part, f.inner_tol2,
                           f.pc);
        LAT_LAUNCH_CHECK();
        if (f.inner_tol2 > 0.0) {
            // relative inner tolerance: stop launching once the sub-solve has converged or broken down
            int32_t flags[2];
            LAT_HIP(hipMemcpyAsync(flags, &f.pc->stop, sizeof(flags), hipMemcpyDeviceToHost, f.s));
            LAT_HIP(hipStreamSynchronize(f.s));
            if (flags[0] || flags[1]) break;
        }
        hipLaunchKernelGGL(k_pcg_p, dim3(bl), dim3(NB), 0, f.s, n, (const PcgCtl *)f.pc, (const double *)f.pz, f.pp);
        LAT_LAUNCH_CHECK();
    }
    // rows of prescribed multipliers: identity
    hipLaunchKernelGGL(k_identity_rows, dim3(bl), dim3(NB), 0, f.s, n, f.liveL, g, x);
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

// z = M^-1 v, the block preconditioner of eq. ifetidp_precond
lat_status precond(Feti &f, const double *v, double *z)
{
    const int64_t nR = f.nRr * f.ld;
    const double *vR = v, *vP = v + nR, *vL = vP + f.nPgd;
    double *zR = z, *zP = z + nR, *zL = zP + f.nPgd;
    FCHK(krom(f, vR, vP, zR, zP));                          // w = K^-1 v_u
    double *t = f.w3 + nR + f.nPgd;                          // t = B w_R - v_L
    hipLaunchKernelGGL(k_b, dim3(blocks(f.pt.nsets)), dim3(NB), 0, f.s, f.d, f.pt.nsets, f.ld, f.pd.set_off,
                       f.pd.set_m0, f.pd.mem_lane, f.pd.mem_rn, f.liveL, (const double *)zR, vL, t);
    hipLaunchKernelGGL(k_dir_b, dim3(blocks(f.pt.ndir)), dim3(NB), 0, f.s, f.d, f.pt.ndir, f.ld, f.Lint, f.pd.dir_lane,
                       f.pd.dir_rn, f.pd.dir_i, (const double *)zR, t);
    LAT_LAUNCH_CHECK();
    if (f.L > 0) {
        hipLaunchKernelGGL(k_axpby, dim3(blocks(f.L)), dim3(NB), 0, f.s, f.L, -1.0, vL, 1.0, t);
        // the identity rows of t must stay v_L (k_b wrote v_L there; the axpby made them 0)
        hipLaunchKernelGGL(k_identity_rows, dim3(blocks(f.L)), dim3(NB), 0, f.s, f.L, f.liveL, vL, t);
        LAT_LAUNCH_CHECK();
    }
    FCHK(fpcg(f, t, zL));                                    // z_L = F^-1 (B w_R - v_L)
    // z_u -= K^-1 (B^T z_L, 0)
    double *bR = f.w3, *bP = f.w3 + nR;
    hipLaunchKernelGGL(k_ffill, dim3(blocks(nR + f.nPgd)), dim3(NB), 0, f.s, nR + f.nPgd, 0.0, bR);
    hipLaunchKernelGGL(k_bt_add, dim3(blocks(f.pt.nsets)), dim3(NB), 0, f.s, f.d, f.pt.nsets, f.ld, f.pd.set_off,
                       f.pd.set_m0, f.pd.mem_lane, f.pd.mem_rn, f.liveL, (const double *)zL, bR);
    hipLaunchKernelGGL(k_dir_bt, dim3(blocks(f.pt.ndir)), dim3(NB), 0, f.s, f.d, f.pt.ndir, f.ld, f.Lint, f.pd.dir_lane,
                       f.pd.dir_rn, f.pd.dir_i, (const double *)zL, bR);
    LAT_LAUNCH_CHECK();
    double *yR = f.w2, *yP = f.w2 + nR;
    FCHK(krom(f, bR, bP, yR, yP));
    hipLaunchKernelGGL(k_axpby, dim3(blocks(nR + f.nPgd)), dim3(NB), 0, f.s, nR + f.nPgd, -1.0, (const double *)yR, 1.0,
                       zR);
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

// A += shift diag(A) (the diagonal saved in dg), one matrix
__global__ void k_shift_diag(int64_t n, double shift, const double *__restrict__ dg, double *__restrict__ A)
{
    const int64_t i = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (i < n) A[i * n + i] += shift * fabs(dg[i]);
}

// Invert a batch of symmetric matrices in place.  Cholesky first; bad[b] = 1 when matrix b is not
// positive definite (a failed factorisation or a pivot <= 1e-12 of its diagonal entry).
//   fallback 0: nothing is inverted when one is bad;
//   fallback 1: the bad ones are inverted by pivoted LU (*singular when one is numerically singular);
//   fallback 2: a bad one that LU finds nonsingular is replaced by A + s diag(A) with the smallest s
//               of 1e-6, 1e-5, ..., 1 that makes it positive definite, and that is inverted
//               (*singular when LU finds it singular or no s works); shift[b] receives s.
lat_status sym_inverse(Feti &f, FArena &ar, int64_t n, int nb, double *A, int fallback, std::vector<int32_t> &bad,
                       std::vector<double> &shift, bool *singular)
{
    bad.assign((size_t)nb, 0);
    shift.assign((size_t)nb, 0.0);
    *singular = false;
    if (n == 0 || nb == 0) return LAT_OK;
    if (n > INT32_MAX) return LAT_E_SHAPE;
    int32_t *info = nullptr, *dbad = nullptr;
    double *dg = nullptr, *copy = nullptr;
    FCHK(ar.get(&info, nb)); FCHK(ar.get(&dbad, nb)); FCHK(ar.get(&dg, n * nb));
    if (fallback) {
        FCHK(ar.get(&copy, n * n * nb));
        hipLaunchKernelGGL(k_copy, dim3(blocks(n * n * nb)), dim3(NB), 0, f.s, n * n * nb, (const double *)A, copy);
    }
    hipLaunchKernelGGL(k_diag, dim3(blocks(n * nb)), dim3(NB), 0, f.s, n, nb, (const double *)A, n * n, dg);
    LAT_LAUNCH_CHECK();
    RBCHK(rocsolver_dpotrf_strided_batched(f.h, rocblas_fill_lower, (rocblas_int)n, A, (rocblas_int)n, n * n, info, nb));
    hipLaunchKernelGGL(k_pivots, dim3(nb), dim3(NB), 0, f.s, n, nb, (const double *)A, n * n, (const double *)dg,
                       (const int32_t *)info, dbad);
    LAT_LAUNCH_CHECK();
    LAT_HIP(hipMemcpyAsync(bad.data(), dbad, (size_t)nb * 4, hipMemcpyDeviceToHost, f.s));
    LAT_HIP(hipStreamSynchronize(f.s));
    int nbad = 0;
    for (int b = 0; b < nb; ++b) nbad += bad[(size_t)b] != 0;
    if (nbad && !fallback) return LAT_OK;
    // Cholesky inverses of the definite ones (the others are overwritten below)
    RBCHK(rocsolver_dpotri_strided_batched(f.h, rocblas_fill_lower, (rocblas_int)n, A, (rocblas_int)n, n * n, info, nb));
    hipLaunchKernelGGL(k_symm, dim3(blocks(n * n), (unsigned)nb), dim3(NB), 0, f.s, n, nb, A, n * n);
    LAT_LAUNCH_CHECK();
    if (!nbad) return LAT_OK;
    int32_t *ipiv = nullptr;
    FCHK(ar.get(&ipiv, n));
    for (int b = 0; b < nb; ++b) {
        if (!bad[(size_t)b]) continue;
        double *Ab = A + (int64_t)b * n * n;
        const double *Cb = copy + (int64_t)b * n * n, *dgb = dg + (int64_t)b * n;
        // is it singular?  (pivoted LU, pivots against the largest diagonal entry)
        hipLaunchKernelGGL(k_copy, dim3(blocks(n * n)), dim3(NB), 0, f.s, n * n, Cb, Ab);
        LAT_LAUNCH_CHECK();
        RBCHK(rocsolver_dgetrf(f.h, (rocblas_int)n, (rocblas_int)n, Ab, (rocblas_int)n, ipiv, info));
        hipLaunchKernelGGL(k_lu_check, dim3(1), dim3(NB), 0, f.s, n, (const double *)Ab, dgb, dbad + b);
        LAT_LAUNCH_CHECK();
        int32_t hinfo[2] = {0, 0};
        LAT_HIP(hipMemcpyAsync(&hinfo[0], info, 4, hipMemcpyDeviceToHost, f.s));
        LAT_HIP(hipMemcpyAsync(&hinfo[1], dbad + b, 4, hipMemcpyDeviceToHost, f.s));
        LAT_HIP(hipStreamSynchronize(f.s));
        if (hinfo[0] != 0 || hinfo[1] != 0) { *singular = true; return LAT_OK; }
        if (fallback == 1) {
            RBCHK(rocsolver_dgetri(f.h, (rocblas_int)n, Ab, (rocblas_int)n, ipiv, info));
            continue;
        }
        bool ok = false;
        for (double sft = 1e-6; sft <= 1.0 + 1e-12 && !ok; sft *= 10.0) {
            hipLaunchKernelGGL(k_copy, dim3(blocks(n * n)), dim3(NB), 0, f.s, n * n, Cb, Ab);
            hipLaunchKernelGGL(k_shift_diag, dim3(blocks(n)), dim3(NB), 0, f.s, n, sft, dgb, Ab);
            LAT_LAUNCH_CHECK();
            RBCHK(rocsolver_dpotrf(f.h, rocblas_fill_lower, (rocblas_int)n, Ab, (rocblas_int)n, info));
            hipLaunchKernelGGL(k_pivots, dim3(1), dim3(NB), 0, f.s, n, 1, (const double *)Ab, n * n, dgb,
                               (const int32_t *)info, dbad + b);
            LAT_LAUNCH_CHECK();
            int32_t hb = 1;
            LAT_HIP(hipMemcpyAsync(&hb, dbad + b, 4, hipMemcpyDeviceToHost, f.s));
            LAT_HIP(hipStreamSynchronize(f.s));
            if (!hb) {
                ok = true;
                shift[(size_t)b] = sft;
                RBCHK(rocsolver_dpotri(f.h, rocblas_fill_lower, (rocblas_int)n, Ab, (rocblas_int)n, info));
                hipLaunchKernelGGL(k_symm, dim3(blocks(n * n), 1u), dim3(NB), 0, f.s, n, 1, Ab, n * n);
                LAT_LAUNCH_CHECK();
            }
        }
        if (!ok) { *singular = true; return LAT_OK; }
    }
    return LAT_OK;
}

double ms_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

constexpr int64_t COARSE_LIMIT = 40000;   // assembled primal DOFs held as a dense inverse

// Setup at one enrichment level.  *definite = false when a principal remaining block is not
// positive definite (nothing else is formed then).
lat_status setup_level(Feti &f, FArena &ar, const std::vector<int32_t> &h_l2g, const std::vector<int32_t> &h_lane,
                       const std::vector<uint8_t> &h_fixed, const int32_t *S, const double *R, const double *nu,
                       const double *beta, const uint8_t *fixed, int level, bool last, bool *definite)
{
    const lat_plan *P = f.P;
    build_part(P, level, h_l2g, h_lane, f.pt);
    build_dirichlet(P, h_fixed, f.pt);
    const Part &pt = f.pt;
    const int d = f.d;
    f.ld = P->ld;
    f.nRr = (int64_t)pt.nRn * d; f.nPr = (int64_t)pt.nPn * d; f.nDr = (int64_t)pt.nDn * d;
    f.nPgd = pt.nPg * d; f.Lint = pt.nmult * d; f.L = f.Lint + pt.ndir; f.nF = f.nRr + f.nPr;
    f.Nv = f.nRr * f.ld + f.nPgd + f.L;
    if (f.nPgd > COARSE_LIMIT) return LAT_E_SHAPE;
    FCHK(upload_part(pt, ar, f.pd, f.s));
    const int nd = f.nd;
    // principal local matrices -> remaining blocks
    double *Kl = nullptr;
    FCHK(ar.get(&Kl, f.nF * f.nF * nd));
    hipLaunchKernelGGL(k_ffill, dim3(blocks(f.nF * f.nF * nd)), dim3(NB), 0, f.s, f.nF * f.nF * nd, 0.0, Kl);
    hipLaunchKernelGGL(k_kloc, dim3((unsigned)lat_cdiv(pt.nRn + pt.nPn, NB), (unsigned)nd), dim3(NB), 0, f.s, d, P->nn,
                       P->nloc, P->E, P->cap, (int)f.nF, pt.nRn + pt.nPn, pt.nRn, f.pd.fnode, f.pd.rnode, f.pd.pnode, S,
                       P->l2g, f.K, Kl);
    LAT_LAUNCH_CHECK();
    FCHK(ar.get(&f.G, f.nRr * f.nRr * nd));
    hipLaunchKernelGGL(k_copy_sub, dim3(blocks(f.nRr * f.nRr), (unsigned)nd), dim3(NB), 0, f.s, f.nRr, f.nRr, nd,
                       (const double *)Kl, f.nF, f.nF * f.nF, (int64_t)0, (int64_t)0, f.G, f.nRr, f.nRr * f.nRr, 1.0);
    LAT_LAUNCH_CHECK();
    std::vector<int32_t> bad;
    std::vector<double> shift;
    bool singular = false;
    FCHK(sym_inverse(f, ar, f.nRr, nd, f.G, last ? (f.indef_mode == 0 ? 2 : 1) : 0, bad, shift, &singular));
    if (singular) return LAT_E_SINGULAR;
    f.n_shift = 0;
    f.max_shift = 0.0;
    for (int b = 0; b < nd; ++b) {
        f.n_shift += bad[(size_t)b] != 0;
        f.max_shift = std::max(f.max_shift, shift[(size_t)b]);
    }
    *definite = f.n_shift == 0;
    if (!*definite && !last) return LAT_OK;
    // Phi_r = -G_r K_RP^r; S_r = K_PP^r + K_RP^rT Phi_r
    FCHK(ar.get(&f.Phi, f.nRr * f.nPr * nd));
    FCHK(ar.get(&f.Spp, f.nPr * f.nPr * nd));
    if (f.nPr > 0 && f.nRr > 0) {
        const double mone = -1.0, zero = 0.0, one = 1.0;
        RBCHK(rocblas_dgemm_strided_batched(f.h, rocblas_operation_none, rocblas_operation_none, (rocblas_int)f.nRr,
                                            (rocblas_int)f.nPr, (rocblas_int)f.nRr, &mone, f.G, (rocblas_int)f.nRr,
                                            f.nRr * f.nRr, Kl + f.nRr * f.nF, (rocblas_int)f.nF, f.nF * f.nF, &zero,
                                            f.Phi, (rocblas_int)f.nRr, f.nRr * f.nPr, nd));
        hipLaunchKernelGGL(k_copy_sub, dim3(blocks(f.nPr * f.nPr), (unsigned)nd), dim3(NB), 0, f.s, f.nPr, f.nPr, nd,
                           (const double *)Kl, f.nF, f.nF * f.nF, f.nRr, f.nRr, f.Spp, f.nPr, f.nPr * f.nPr, 1.0);
        LAT_LAUNCH_CHECK();
        RBCHK(rocblas_dgemm_strided_batched(f.h, rocblas_operation_transpose, rocblas_operation_none, (rocblas_int)f.nPr,
                                            (rocblas_int)f.nPr, (rocblas_int)f.nRr, &one, Kl + f.nRr * f.nF,
                                            (rocblas_int)f.nF, f.nF * f.nF, f.Phi, (rocblas_int)f.nRr, f.nRr * f.nPr,
                                            &one, f.Spp, (rocblas_int)f.nPr, f.nPr * f.nPr, nd));
    } else if (f.nPr > 0) {
        hipLaunchKernelGGL(k_copy_sub, dim3(blocks(f.nPr * f.nPr), (unsigned)nd), dim3(NB), 0, f.s, f.nPr, f.nPr, nd,
                           (const double *)Kl, f.nF, f.nF * f.nF, f.nRr, f.nRr, f.Spp, f.nPr, f.nPr * f.nPr, 1.0);
        LAT_LAUNCH_CHECK();
    }
    // dual blocks: F_dd^r = (G_r)_dd, its inverse, Phi_d^r = dual rows of Phi_r
    FCHK(ar.get(&f.Fdd, f.nDr * f.nDr * nd));
    FCHK(ar.get(&f.Sdd, f.nDr * f.nDr * nd));
    FCHK(ar.get(&f.Phid, f.nDr * f.nPr * nd));
    if (f.nDr > 0) {
        hipLaunchKernelGGL(k_gather_sub, dim3(blocks(f.nDr * f.nDr), (unsigned)nd), dim3(NB), 0, f.s, f.nDr, f.nDr, nd,
                           d, f.pd.dual_rn, f.pd.dual_rn, (const double *)f.G, f.nRr, f.nRr * f.nRr, f.Fdd, f.nDr,
                           f.nDr * f.nDr);
        hipLaunchKernelGGL(k_copy_sub, dim3(blocks(f.nDr * f.nDr), (unsigned)nd), dim3(NB), 0, f.s, f.nDr, f.nDr, nd,
                           (const double *)f.Fdd, f.nDr, f.nDr * f.nDr, (int64_t)0, (int64_t)0, f.Sdd, f.nDr,
                           f.nDr * f.nDr, 1.0);
        if (f.nPr > 0)
            hipLaunchKernelGGL(k_gather_sub, dim3(blocks(f.nDr * f.nPr), (unsigned)nd), dim3(NB), 0, f.s, f.nDr, f.nPr,
                               nd, d, f.pd.dual_rn, (const int32_t *)nullptr, (const double *)f.Phi, f.nRr,
                               f.nRr * f.nPr, f.Phid, f.nDr, f.nDr * f.nPr);
        LAT_LAUNCH_CHECK();
        std::vector<int32_t> bad2;
        std::vector<double> sh2;
        bool sing2 = false;
        FCHK(sym_inverse(f, ar, f.nDr, nd, f.Sdd, 1, bad2, sh2, &sing2));
        if (sing2) return LAT_E_SINGULAR;
    }
    // coordinates of every cell
    FCHK(ar.get(&f.delta, f.ld * nd));
    if (f.coords == 1)
        hipLaunchKernelGGL(k_delta_nearest, dim3(blocks(f.ld)), dim3(NB), 0, f.s, f.ld, nd, P->cap, P->perm, S, R, nu,
                           beta, f.delta);
    else
        hipLaunchKernelGGL(k_delta, dim3(blocks(f.ld)), dim3(NB), 0, f.s, f.ld, nd, f.n_r, P->cap, P->perm, f.alpha, R,
                           nu, beta, f.delta);
    LAT_LAUNCH_CHECK();
    int32_t *sel = nullptr;
    FCHK(ar.get(&sel, f.ld));
    f.onehot = f.coords == 1;
    if (f.onehot) {
        // lanes grouped by their principal cell (ascending lane within a group)
        hipLaunchKernelGGL(k_onehot_sel, dim3(blocks(f.ld)), dim3(NB), 0, f.s, f.ld, nd, (const double *)f.delta, sel);
        LAT_LAUNCH_CHECK();
        std::vector<int32_t> hsel((size_t)f.ld);
        LAT_HIP(hipMemcpyAsync(hsel.data(), sel, (size_t)f.ld * 4, hipMemcpyDeviceToHost, f.s));
        LAT_HIP(hipStreamSynchronize(f.s));
        f.off.assign((size_t)nd + 1, 0);
        for (int32_t r : hsel)
            if (r >= 0) ++f.off[(size_t)r + 1];
        for (int r = 0; r < nd; ++r) f.off[(size_t)r + 1] += f.off[(size_t)r];
        f.nv = f.off[(size_t)nd];
        std::vector<int32_t> ord((size_t)std::max<int64_t>(f.nv, 1), 0);
        std::vector<int64_t> fill(f.off.begin(), f.off.end() - 1);
        for (int64_t l = 0; l < f.ld; ++l)
            if (hsel[(size_t)l] >= 0) ord[(size_t)fill[(size_t)hsel[(size_t)l]]++] = (int32_t)l;
        FCHK(ar.put(&f.order, ord, f.s));
        std::vector<int32_t> tl;
        f.big.clear();
        for (int r = 0; r < nd; ++r) {
            if (!f.g32 && f.off[(size_t)r + 1] - f.off[(size_t)r] >= GBIG) { f.big.push_back(r); continue; }
            for (int64_t k0 = f.off[(size_t)r]; k0 < f.off[(size_t)r + 1]; k0 += GT) {
                tl.push_back(r);
                tl.push_back((int32_t)k0);
                tl.push_back((int32_t)std::min<int64_t>(k0 + GT, f.off[(size_t)r + 1]));
            }
        }
        f.ntiles = (int64_t)tl.size() / 3;
        FCHK(ar.put(&f.tiles, tl, f.s));
        LAT_HIP(hipStreamSynchronize(f.s));
    }
    // masks
    FCHK(ar.get(&f.liveR, f.nRr * f.ld)); FCHK(ar.get(&f.liveP, f.nPgd)); FCHK(ar.get(&f.liveL, f.L));
    FCHK(ar.get(&f.liveD, f.nDr * f.ld));
    hipLaunchKernelGGL(k_live_R, dim3(blocks((int64_t)pt.nRn * f.ld)), dim3(NB), 0, f.s, d, P->nloc, pt.nRn, f.ld,
                       f.pd.rnode, f.pd.dpos, P->perm, P->l2g, fixed, f.liveR);
    hipLaunchKernelGGL(k_live_P, dim3(blocks(pt.nPg)), dim3(NB), 0, f.s, d, pt.nPg, f.pd.pglob, fixed, f.liveP);
    hipLaunchKernelGGL(k_fill_u8, dim3(blocks(f.L)), dim3(NB), 0, f.s, f.L, (uint8_t)1, f.liveL);
    hipLaunchKernelGGL(k_live_D, dim3(blocks(f.nDr * f.ld)), dim3(NB), 0, f.s, d, pt.nDn, f.ld, f.pd.dual_rn,
                       (const uint8_t *)f.liveR, f.liveD);
    LAT_LAUNCH_CHECK();
    // coarse problem: local C = sum_r delta_r S_r per lane, assembled, inverted (LU, FP64)
    FCHK(ar.get(&f.Sc, std::max<int64_t>(f.nPgd * f.nPgd, 1)));
    if (f.nPgd > 0) {
        double *C = nullptr;
        FCHK(ar.get(&C, f.nPr * f.nPr * f.ld));
        if (f.onehot) {
            hipLaunchKernelGGL(k_select_spp, dim3(blocks(f.nPr * f.nPr * f.ld)), dim3(NB), 0, f.s, f.nPr * f.nPr, f.ld,
                               (const int32_t *)sel, (const double *)f.Spp, C);
            LAT_LAUNCH_CHECK();
        } else {
            FCHK(gemm(f, rocblas_operation_none, rocblas_operation_none, f.nPr * f.nPr, f.ld, nd, 1.0, f.Spp,
                      f.nPr * f.nPr, f.delta, nd, 0.0, C, f.nPr * f.nPr));
        }
        hipLaunchKernelGGL(k_ffill, dim3(blocks(f.nPgd * f.nPgd)), dim3(NB), 0, f.s, f.nPgd * f.nPgd, 0.0, f.Sc);
        hipLaunchKernelGGL(k_coarse_asm, dim3(blocks(f.nPgd)), dim3(NB), 0, f.s, d, pt.nPn, f.ld, pt.nPg, f.pd.pg_off,
                           f.pd.pg_lane, f.pd.pg_p, f.pd.prim_g, (const uint8_t *)f.liveP, (const double *)C, f.Sc);
        LAT_LAUNCH_CHECK();
        int32_t *ipiv = nullptr, *info = nullptr;
        FCHK(ar.get(&ipiv, f.nPgd)); FCHK(ar.get(&info, 1));
        RBCHK(rocsolver_dgetrf(f.h, (rocblas_int)f.nPgd, (rocblas_int)f.nPgd, f.Sc, (rocblas_int)f.nPgd, ipiv, info));
        int32_t hinfo = 0;
        LAT_HIP(hipMemcpyAsync(&hinfo, info, 4, hipMemcpyDeviceToHost, f.s));
        LAT_HIP(hipStreamSynchronize(f.s));
        if (hinfo != 0) return LAT_E_SINGULAR;
        RBCHK(rocsolver_dgetri(f.h, (rocblas_int)f.nPgd, f.Sc, (rocblas_int)f.nPgd, ipiv, info));
    }
    // scratch of the applies
    const int64_t stack_rows = std::max<int64_t>({f.nRr, f.nDr, f.nPr, 1});
    FCHK(ar.get(&f.As, stack_rows * f.ld * (f.onehot ? 1 : nd)));
    if (f.onehot) {
        FCHK(ar.get(&f.Xg, stack_rows * f.ld)); FCHK(ar.get(&f.Yg, stack_rows * f.ld));
        f.split_rows = 2 * stack_rows;
        FCHK(ar.get(&f.split, f.split_rows * f.ld));
    }
    if (f.g32) {
        FCHK(ar.get(&f.G32, f.nRr * f.nRr * nd));
        hipLaunchKernelGGL(k_to_f32, dim3(blocks(std::min<int64_t>(f.nRr * f.nRr * nd, (int64_t)1 << 26))), dim3(NB), 0,
                           f.s, f.nRr * f.nRr * nd, (const double *)f.G, f.G32);
        LAT_LAUNCH_CHECK();
    }

    FCHK(ar.get(&f.xm, stack_rows * f.ld));
    FCHK(ar.get(&f.T1, f.nPr * nd * f.ld));
    FCHK(ar.get(&f.hl, f.nPr * f.ld)); FCHK(ar.get(&f.el, f.nPr * f.ld));
    FCHK(ar.get(&f.hP, f.nPgd)); FCHK(ar.get(&f.uP, f.nPgd));
    FCHK(ar.get(&f.cmv, std::max<int64_t>(lat_cdiv(f.nPgd, CMV_W) * f.nPgd, 1)));
    FCHK(ar.get(&f.qd, f.nDr * f.ld)); FCHK(ar.get(&f.vd, f.nDr * f.ld));
    FCHK(ar.get(&f.pc, 1));
    FCHK(ar.get(&f.px, f.L)); FCHK(ar.get(&f.pr, f.L)); FCHK(ar.get(&f.pz, f.L)); FCHK(ar.get(&f.pp, f.L));
    FCHK(ar.get(&f.pq, f.L));
    FCHK(ar.get(&f.w1, f.Nv)); FCHK(ar.get(&f.w2, f.Nv)); FCHK(ar.get(&f.w3, f.Nv));
    return LAT_OK;
}

}  // namespace

extern "C" {

lat_status lat_feti_partition(const lat_plan *P, int32_t level, int32_t *node_class, int64_t *counts,
                              int64_t *primal_nodes, int32_t *mult, hipStream_t stream)
{
    if (!P || !counts || level < 0) return LAT_E_ARG;
    std::vector<int32_t> h_l2g((size_t)(P->ncells * P->nloc)), h_lane((size_t)P->ncells);
    LAT_HIP(hipMemcpyAsync(h_l2g.data(), P->l2g, h_l2g.size() * 4, hipMemcpyDeviceToHost, stream));
    LAT_HIP(hipMemcpyAsync(h_lane.data(), P->lane, h_lane.size() * 4, hipMemcpyDeviceToHost, stream));
    LAT_HIP(hipStreamSynchronize(stream));
    Part pt;
    build_part(P, level, h_l2g, h_lane, pt);
    counts[0] = pt.nPg; counts[1] = pt.nmult; counts[2] = pt.nRn; counts[3] = pt.nDn;
    if (node_class) std::copy(pt.cls.begin(), pt.cls.end(), node_class);
    if (primal_nodes) std::copy(pt.pglob.begin(), pt.pglob.end(), primal_nodes);
    if (mult) {
        int64_t r = 0;
        for (int64_t s = 0; s < pt.nsets; ++s)
            for (int32_t k = pt.set_off[(size_t)s]; k + 1 < pt.set_off[(size_t)s + 1]; ++k, ++r) {
                mult[r * 4 + 0] = pt.mem_cell[(size_t)k]; mult[r * 4 + 1] = pt.mem_a[(size_t)k];
                mult[r * 4 + 2] = pt.mem_cell[(size_t)k + 1]; mult[r * 4 + 3] = pt.mem_a[(size_t)k + 1];
            }
    }
    return LAT_OK;
}

lat_status lat_feti_solve(const lat_plan *P, const double *K, int32_t n_r, const double *alpha, const int32_t *S,
                          const double *R, const double *nu, const double *beta, const uint8_t *fixed, const double *b,
                          double *x, const lat_feti_opts *opts, lat_feti_info *info, hipStream_t stream)
{
    if (info) *info = lat_feti_info{};
    if (!P || !K || !alpha || !S || !fixed || !b || !x || !opts) return LAT_E_ARG;
    if ((R || nu || beta) && !(R && nu && beta)) return LAT_E_ARG;
    if (n_r < 1 || n_r > P->cap) return LAT_E_SHAPE;
    if (opts->enrich < 0 || opts->max_enrich < opts->enrich || opts->inner_it < 0 || opts->restart < 1 ||
        opts->restart > 512 || opts->maxit < 1 || !(opts->tol > 0.0) || opts->n_delta < 0 || opts->indefinite < 0 ||
        !(opts->inner_tol >= 0.0) || !std::isfinite(opts->inner_tol) ||
        opts->indefinite > 1 || opts->coords < 0 || opts->coords > 1 || (opts->coords == 1 && !R) ||
        (opts->prec != LAT_F64 && opts->prec != LAT_F32) || (opts->prec == LAT_F32 && opts->coords != 1))
        return LAT_E_ARG;
    const auto t0 = std::chrono::steady_clock::now();
    Feti f;
    f.P = P; f.s = stream; f.d = P->dim; f.n_r = n_r; f.K = K; f.alpha = alpha;
    f.nd = opts->n_delta == 0 ? n_r : std::min<int>(opts->n_delta, n_r);
    f.inner_it = opts->inner_it;
    f.inner_tol2 = opts->inner_tol * opts->inner_tol;
    f.indef_mode = opts->indefinite;
    f.coords = opts->coords;
    f.g32 = opts->prec == LAT_F32;
    f.h = feti_handle();
    if (!f.h || rocblas_set_stream(f.h, stream) != rocblas_status_success) return LAT_E_DEVICE;
    FArena ar;
    const int64_t npk = std::max<int64_t>(P->npacked, 1) * P->dim * LAT_WAVE;
    FCHK(ar.get(&f.Xpk, npk)); FCHK(ar.get(&f.Ypk, npk)); FCHK(ar.get(&f.part, DOT_BLOCKS));
    if (opts->materialize) {
        double *ops = nullptr;
        FCHK(ar.get(&ops, std::max<int64_t>(P->npacked, 1) * P->E * LAT_WAVE));
        FCHK(lat_combine_ops(P, K, n_r, alpha, ops, stream));
        f.ops = ops;
    }
    std::vector<int32_t> h_l2g((size_t)(P->ncells * P->nloc)), h_lane((size_t)P->ncells);
    LAT_HIP(hipMemcpyAsync(h_l2g.data(), P->l2g, h_l2g.size() * 4, hipMemcpyDeviceToHost, stream));
    LAT_HIP(hipMemcpyAsync(h_lane.data(), P->lane, h_lane.size() * 4, hipMemcpyDeviceToHost, stream));
    std::vector<uint8_t> h_fixed((size_t)(P->nglobal * P->dim));
    if (!h_fixed.empty())
        LAT_HIP(hipMemcpyAsync(h_fixed.data(), fixed, h_fixed.size(), hipMemcpyDeviceToHost, stream));
    LAT_HIP(hipStreamSynchronize(stream));
    // enrichment loop (Sec. 3.3.2): while a principal remaining block is not positive definite, restart
    // the setup with one more primal node per cell edge, as long as that adds an active primal node
    // and max_enrich allows; past that point a block that is not definite but nonsingular is shifted
    // (A + s diag A, the smallest s of a ladder that makes it definite) and inverted
    int level = opts->enrich;
    for (;;) {
        std::unique_ptr<FArena> lev(new FArena());
        bool definite = false;
        bool more = level < opts->max_enrich && level < P->nel - 1;
        if (more) {   // would the next level add an active primal node?
            Part nx;
            build_part(P, level + 1, h_l2g, h_lane, nx);
            Part cur;
            build_part(P, level, h_l2g, h_lane, cur);
            more = nx.nPn > cur.nPn;
        }
        lat_status st = setup_level(f, *lev, h_l2g, h_lane, h_fixed, S, R, nu, beta, fixed, level, !more, &definite);
        if (st != LAT_OK) {
            if (info) { info->enrich = level; info->t_setup_ms = ms_since(t0); }
            return st;
        }
        if (definite || !more) {
            ar.ptrs.insert(ar.ptrs.end(), lev->ptrs.begin(), lev->ptrs.end());
            lev->ptrs.clear();
            break;
        }
        ++level;
    }
    // PCG needs a positive definite interface operator: with indefinite local inverses the interface
    // block is its Dirichlet preconditioner alone
    if (f.n_shift > 0 && f.indef_mode == 1) f.inner_it = 0;
    const double t_setup = ms_since(t0);
    const auto t1 = std::chrono::steady_clock::now();
    if (info) {
        info->enrich = level; info->n_delta = f.nd; info->n_shift = f.n_shift; info->max_shift = f.max_shift;
        info->n_primal = f.nPgd; info->n_mult = f.L;
        info->n_rdofs = f.nRr; info->n_ddofs = f.nDr; info->t_setup_ms = t_setup;
    }
    // right-hand side of the saddle-point system
    const int64_t N = f.Nv, nR = f.nRr * f.ld;
    const int m = opts->restart;
    double *V = nullptr, *Z = nullptr, *bv = nullptr, *xv = nullptr, *hcol = nullptr;
    FCHK(ar.get(&V, N * (int64_t)(m + 1))); FCHK(ar.get(&Z, N * (int64_t)m));
    FCHK(ar.get(&bv, N)); FCHK(ar.get(&xv, N)); FCHK(ar.get(&hcol, m + 1));
    hipLaunchKernelGGL(k_ffill, dim3(blocks(N)), dim3(NB), 0, stream, N, 0.0, bv);
    hipLaunchKernelGGL(k_ffill, dim3(blocks(N)), dim3(NB), 0, stream, N, 0.0, xv);
    hipLaunchKernelGGL(k_rhs, dim3(blocks((int64_t)f.pt.nRn * f.ld)), dim3(NB), 0, stream, f.d, P->nloc, f.pt.nRn, f.ld,
                       f.pd.rnode, P->perm, P->l2g, f.pd.gn_off, (const uint8_t *)f.liveR, fixed, b, bv);
    hipLaunchKernelGGL(k_rhs_P, dim3(blocks(f.pt.nPg)), dim3(NB), 0, stream, f.d, f.pt.nPg, f.pd.pglob,
                       (const uint8_t *)f.liveP, b, bv + nR);
    LAT_LAUNCH_CHECK();
    double bnorm2 = 0.0;
    FCHK(dot_host(f, N, bv, bv, &bnorm2));
    const double bnorm = std::sqrt(bnorm2);
    int iters = 0, restarts = 0;
    double relres = 0.0;
    lat_status result = LAT_OK;
    if (bnorm > 0.0) {
        // restarted FGMRES (right preconditioning, classical Gram-Schmidt twice)
        double *r = f.w1;
        hipLaunchKernelGGL(k_copy, dim3(blocks(N)), dim3(NB), 0, stream, N, (const double *)bv, r);
        LAT_LAUNCH_CHECK();
        double beta_r = bnorm;
        std::vector<double> H((size_t)(m + 1) * m, 0.0), cs((size_t)m), sn((size_t)m), gv((size_t)m + 1), hh((size_t)m + 1);
        for (;;) {
            hipLaunchKernelGGL(k_axpby, dim3(blocks(N)), dim3(NB), 0, stream, N, 1.0 / beta_r, (const double *)r, 0.0, V);
            LAT_LAUNCH_CHECK();
            std::fill(H.begin(), H.end(), 0.0);
            std::fill(gv.begin(), gv.end(), 0.0);
            gv[0] = beta_r;
            int k = 0;                   // usable columns of this cycle
            bool breakdown = false;
            for (int j = 0; j < m && iters < opts->maxit; ++j) {
                double *vj = V + (int64_t)j * N, *zj = Z + (int64_t)j * N, *w = V + (int64_t)(j + 1) * N;
                FCHK(precond(f, vj, zj));
                FCHK(op_apply(f, zj, w));
                const double one = 1.0, zero = 0.0, mone = -1.0;
                // classical Gram-Schmidt; a second pass only when the first one cancelled most of w
                // (its norm fell below 0.7 of the norm before: the Kahan-Parlett criterion)
                double wb2 = 0.0, wn2 = 0.0;
                FCHK(dot_host(f, N, w, w, &wb2));
                for (int pass = 0; pass < 2; ++pass) {
                    RBCHK(rocblas_dgemv(f.h, rocblas_operation_transpose, (rocblas_int)N, j + 1, &one, V, (rocblas_int)N,
                                        w, 1, &zero, hcol, 1));
                    RBCHK(rocblas_dgemv(f.h, rocblas_operation_none, (rocblas_int)N, j + 1, &mone, V, (rocblas_int)N,
                                        hcol, 1, &one, w, 1));
                    LAT_HIP(hipMemcpyAsync(hh.data(), hcol, (size_t)(j + 1) * 8, hipMemcpyDeviceToHost, stream));
                    FCHK(dot_host(f, N, w, w, &wn2));
                    for (int i = 0; i <= j; ++i) H[(size_t)j * (m + 1) + i] += hh[(size_t)i];
                    if (wn2 >= 0.49 * wb2) break;
                    wb2 = wn2;
                }
                const double wn = std::sqrt(wn2);
                H[(size_t)j * (m + 1) + j + 1] = wn;
                ++iters;
                if (wn > 0.0) {
                    hipLaunchKernelGGL(k_axpby, dim3(blocks(N)), dim3(NB), 0, stream, N, 1.0 / wn, (const double *)w,
                                       0.0, w);
                    LAT_LAUNCH_CHECK();
                }
                // Givens rotations of the new column
                double *hc = &H[(size_t)j * (m + 1)];
                for (int i = 0; i < j; ++i) {
                    const double t = cs[(size_t)i] * hc[i] + sn[(size_t)i] * hc[i + 1];
                    hc[i + 1] = -sn[(size_t)i] * hc[i] + cs[(size_t)i] * hc[i + 1];
                    hc[i] = t;
                }
                const double rr = std::hypot(hc[j], hc[j + 1]);
                if (!(rr > 0.0) || !std::isfinite(rr)) { breakdown = true; break; }   // column j unusable
                cs[(size_t)j] = hc[j] / rr;
                sn[(size_t)j] = hc[j + 1] / rr;
                hc[j] = rr;
                hc[j + 1] = 0.0;
                gv[(size_t)j + 1] = -sn[(size_t)j] * gv[(size_t)j];
                gv[(size_t)j] = cs[(size_t)j] * gv[(size_t)j];
                k = j + 1;
                if (!(std::fabs(gv[(size_t)j + 1]) > opts->tol * bnorm) || !(wn > 0.0)) break;
            }
            if (breakdown && k == 0) { result = LAT_E_SINGULAR; break; }
            // y = H^-1 g (upper triangular k x k), x += Z y
            std::vector<double> y((size_t)k, 0.0);
            for (int i = k - 1; i >= 0; --i) {
                double v = gv[(size_t)i];
                for (int c = i + 1; c < k; ++c) v -= H[(size_t)c * (m + 1) + i] * y[(size_t)c];
                y[(size_t)i] = v / H[(size_t)i * (m + 1) + i];
            }
            if (k > 0) {
                LAT_HIP(hipMemcpyAsync(hcol, y.data(), (size_t)k * 8, hipMemcpyHostToDevice, stream));
                LAT_HIP(hipStreamSynchronize(stream));
                const double one = 1.0;
                RBCHK(rocblas_dgemv(f.h, rocblas_operation_none, (rocblas_int)N, k, &one, Z, (rocblas_int)N, hcol, 1, &one,
                                    xv, 1));
            }
            // true residual of the saddle-point system
            FCHK(op_apply(f, xv, f.w2));
            hipLaunchKernelGGL(k_copy, dim3(blocks(N)), dim3(NB), 0, stream, N, (const double *)bv, r);
            hipLaunchKernelGGL(k_axpby, dim3(blocks(N)), dim3(NB), 0, stream, N, -1.0, (const double *)f.w2, 1.0, r);
            LAT_LAUNCH_CHECK();
            double r2 = 0.0;
            FCHK(dot_host(f, N, r, r, &r2));
            beta_r = std::sqrt(r2);
            relres = beta_r / bnorm;
            if (!(beta_r > opts->tol * bnorm)) break;
            if (breakdown) { result = LAT_E_SINGULAR; break; }
            if (iters >= opts->maxit) { result = LAT_E_NOCONV; break; }
            ++restarts;
        }
    }
    hipLaunchKernelGGL(k_solution, dim3(blocks(P->nglobal)), dim3(NB), 0, stream, f.d, P->nglobal, f.pt.nRn, f.ld,
                       f.pd.gn_off, f.pd.gn_lane, f.pd.gn_fn, f.pd.gp_of_g, fixed, (const double *)xv,
                       (const double *)(xv + nR), x);
    LAT_LAUNCH_CHECK();
    LAT_HIP(hipStreamSynchronize(stream));
    if (info) {
        info->iters = iters; info->restarts = restarts; info->relres = relres; info->t_solve_ms = ms_since(t1);
    }
    if (result == LAT_OK && relres > opts->tol) result = LAT_E_NOCONV;
    return result;
}

}  // extern "C"
