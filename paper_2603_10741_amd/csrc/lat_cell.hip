// Cell operators of the compressible neo-Hookean law on voxelised Q1 cells:
// internal force (eq. internalloadvec), stored energy, tangent (Sec. 3.1.4 and
// eq. fullquadraturerule) in stencil layout, snapshots (eq. snapshots), principal
// operators (eq. reducedbasis) and the reverse mode of the residual.
//
// Work decomposition: one thread per (cell lane, local node a[, tangent row i in 3D]).
// Lanes are cells (cell-interleaved layouts), so every wave works on the same node of 64
// cells: element masks, displacements and outputs are read/written with unit stride.
// The thread visits the (up to) 2^d elements around its node and, at each Gauss point,
// builds F, J, ln J and p_c = F^{-T} g_c for the element's corners; the tangent row of
// node a then follows from the identity (material form of the paper's D tensor)
//   K[(a,i),(c,j)] += w [ mu d_ij (g_a . g_c) + (mu - lam ln J) (p_a)_j (p_c)_i + lam (p_a)_i (p_c)_j ].
// Every output entry is written by exactly one thread: no atomics, bitwise reproducible.
#include "lat_internal.h"

#include <type_traits>

namespace {

template <int DIM>
struct Geo {
    static constexpr int NC = 1 << DIM;          // element corners
    static constexpr int NO = DIM == 2 ? 9 : 27; // stencil offsets
    static constexpr int E = NO * DIM * DIM;     // stencil entries per node
};

// Quadrature point coordinates on the element reference square/cube [0,1]^d.
template <int RULE>
__device__ __forceinline__ double gauss_x(int k)
{
    if (RULE == LAT_RULE_REDUCED) return 0.5;
    return k == 0 ? 0.5 - 0.5 / sqrt(3.0) : 0.5 + 0.5 / sqrt(3.0);
}

// d N_c / d xi_J at quadrature point q (tensor index), times 1/h.
template <int DIM, int RULE>
__device__ __forceinline__ double shape_grad(int q, int c, int J, double invh)
{
    constexpr int NP = RULE == LAT_RULE_REDUCED ? 1 : 2;
    double v = invh;
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
        int kq = (ax == 0 ? q : (ax == 1 ? q / NP : q / (NP * NP))) % NP;
        double x = gauss_x<RULE>(kq);
        int bit = (c >> ax) & 1;
        if (ax == J) v *= bit ? 1.0 : -1.0;
        else v *= bit ? x : 1.0 - x;
    }
    return v;
}

struct CellArgs {
    int nel, nloc;
    int64_t ld;
    const double *u_cil;        // [nloc][d][ld]
    const uint8_t *keep_il;     // [nelem][ld]
    const int32_t *perm;        // [ld]
    const int32_t *lane;        // [N_s]
    const double *mu, *lam;     // [N_s] canonical (material mode 0)
    int matmode;                // 0: arrays, 1: (1,0), 2: (0,1)
    // all-cells outputs
    double *f;                  // CIL(d)
    double *epart;              // [nloc][ld]
    double *T;                  // CIL(E)
    double *ops;                // packed plain ops
    const int32_t *uidx, *goff;
    // principal mode
    const int32_t *S;
    int n_r, cap;
    double *Kst;                // [(a*E+e)*cap + k]
    int32_t *st;
    int nsa;                    // sampled rule: sub-grid nodes per axis
};

template <int DIM, int RULE, bool PRINCIPAL>
__global__ __launch_bounds__(256) void k_cell(CellArgs A)
{
    using G = Geo<DIM>;
    constexpr int NQ = RULE == LAT_RULE_REDUCED ? 1 : (1 << DIM);
    constexpr int NROW = DIM == 2 ? 2 : 1;       // tangent rows per thread
    const int nel = A.nel, nn = nel + 1;
    const int64_t ld = A.ld;
    // sampled rule: full-rule rows of the sub-grid node arow (every coordinate a multiple of the
    // stride), written to snapshot row arow; otherwise arow is the node itself
    const int arow = blockIdx.y;
    int a = arow;
    if (RULE == LAT_RULE_SAMPLED) {
        const int nsa = A.nsa;
        a = LAT_SAMPLE_STRIDE * ((arow % nsa) + nn * ((arow / nsa) % nsa) + (DIM == 3 ? nn * nn * (arow / (nsa * nsa)) : 0));
    }
    // 3D: blockIdx.z = row i (3) x offset plane (3); a thread accumulates the 9 offsets of its
    // plane, which keeps the accumulators in registers (all 27 would spill)
    const int row0 = DIM == 2 ? 0 : (int)blockIdx.z / 3;
    const int pz = DIM == 2 ? 1 : (int)blockIdx.z % 3;
    int64_t p;
    int cell, slot = 0;
    if (PRINCIPAL) {
        slot = threadIdx.x;
        if (slot >= A.cap) return;
        cell = slot < A.n_r ? A.S[slot] : -1;
        p = cell >= 0 ? A.lane[cell] : 0;
    } else {
        p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        if (p >= ld) return;
        cell = A.perm[p];
    }
    const double h = 1.0 / nel, invh = (double)nel;
    double hd = h;
#pragma unroll
    for (int ax = 1; ax < DIM; ++ax) hd *= h;
    const double wq = (RULE == LAT_RULE_REDUCED ? 1.0 : (DIM == 2 ? 0.25 : 0.125)) * hd;
    double mu = 0.0, lam = 0.0;
    if (cell >= 0) {
        mu = A.matmode == 0 ? A.mu[cell] : (A.matmode == 1 ? 1.0 : 0.0);
        lam = A.matmode == 0 ? A.lam[cell] : (A.matmode == 2 ? 1.0 : 0.0);
    }
    const int ia[3] = {a % nn, (a / nn) % nn, DIM == 3 ? a / (nn * nn) : 0};

    constexpr int NOP = 9;                       // offsets per plane (all of them in 2D)
    double acc[NOP][NROW][DIM];
    double facc[NROW];
    double en = 0.0;
#pragma unroll
    for (int o = 0; o < NOP; ++o)
#pragma unroll
        for (int r = 0; r < NROW; ++r)
#pragma unroll
            for (int j = 0; j < DIM; ++j) acc[o][r][j] = 0.0;
#pragma unroll
    for (int r = 0; r < NROW; ++r) facc[r] = 0.0;

    // one element around node a per call; k (node a is corner k of the element) is a compile-time
    // constant so that every accumulator index below is static
    auto element = [&](auto kc) __attribute__((always_inline)) {
        constexpr int k = decltype(kc)::value;
            int ie[3] = {0, 0, 0};
            bool ok = true;
#pragma unroll
            for (int ax = 0; ax < DIM; ++ax) {
                ie[ax] = ia[ax] - ((k >> ax) & 1);
                ok = ok && ie[ax] >= 0 && ie[ax] < nel;
            }
            if (!ok) return;
            // 3D: element k touches plane pz only from below (pz = 0: k above node a's layer) or
            // above (pz = 2); plane 1 takes every element (and carries the force and energy)
            if (DIM == 3 && ((pz == 0 && !((k >> 2) & 1)) || (pz == 2 && ((k >> 2) & 1)))) return;
            const int e = ie[0] + nel * (ie[1] + nel * ie[2]);
            if (!A.keep_il[(int64_t)e * ld + p]) return;
            double ue[G::NC][DIM];
#pragma unroll
            for (int c = 0; c < G::NC; ++c) {
                int b = (ie[0] + (c & 1)) + nn * ((ie[1] + ((c >> 1) & 1)) + nn * (DIM == 3 ? ie[2] + ((c >> 2) & 1) : 0));
#pragma unroll
                for (int i = 0; i < DIM; ++i) ue[c][i] = A.u_cil[((int64_t)b * DIM + i) * ld + p];
            }
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                double F[DIM][DIM];
#pragma unroll
                for (int i = 0; i < DIM; ++i)
#pragma unroll
                    for (int J = 0; J < DIM; ++J) F[i][J] = (i == J) ? 1.0 : 0.0;
#pragma unroll
                for (int c = 0; c < G::NC; ++c)
#pragma unroll
                    for (int J = 0; J < DIM; ++J) {
                        const double g = shape_grad<DIM, RULE>(q, c, J, invh);
#pragma unroll
                        for (int i = 0; i < DIM; ++i) F[i][J] += ue[c][i] * g;
                    }
                double Jd, H[DIM][DIM];                // H = F^{-T}
                if (DIM == 2) {
                    Jd = F[0][0] * F[1][1] - F[0][1] * F[1][0];
                    const double r = 1.0 / Jd;
                    H[0][0] = F[1][1] * r; H[0][1] = -F[1][0] * r;
                    H[1][0] = -F[0][1] * r; H[1][1] = F[0][0] * r;
                } else {
                    double C[3][3];                     // cofactors
                    C[0][0] = F[1][1] * F[2][2] - F[1][2] * F[2][1];
                    C[0][1] = F[1][2] * F[2][0] - F[1][0] * F[2][2];
                    C[0][2] = F[1][0] * F[2][1] - F[1][1] * F[2][0];
                    C[1][0] = F[0][2] * F[2][1] - F[0][1] * F[2][2];
                    C[1][1] = F[0][0] * F[2][2] - F[0][2] * F[2][0];
                    C[1][2] = F[0][1] * F[2][0] - F[0][0] * F[2][1];
                    C[2][0] = F[0][1] * F[1][2] - F[0][2] * F[1][1];
                    C[2][1] = F[0][2] * F[1][0] - F[0][0] * F[1][2];
                    C[2][2] = F[0][0] * F[1][1] - F[0][1] * F[1][0];
                    Jd = F[0][0] * C[0][0] + F[0][1] * C[0][1] + F[0][2] * C[0][2];
                    const double r = 1.0 / Jd;
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int J = 0; J < 3; ++J) H[i][J] = C[i][J] * r;
                }
                double lnJ = 0.0;
                if (Jd > 0.0 && isfinite(Jd)) {
                    lnJ = log(Jd);
                } else {
                    lat_flag(A.st, isfinite(Jd) ? LAT_E_INVERTED : LAT_E_NONFINITE, cell);
                }
                double gk[DIM], pk[DIM];
#pragma unroll
                for (int J = 0; J < DIM; ++J) gk[J] = shape_grad<DIM, RULE>(q, k, J, invh);
#pragma unroll
                for (int i = 0; i < DIM; ++i) {
                    double s = 0.0;
#pragma unroll
                    for (int J = 0; J < DIM; ++J) s += H[i][J] * gk[J];
                    pk[i] = s;
                }
                // internal force row(s): P g_a = mu (F g_a - p_a) + lam ln J p_a
#pragma unroll
                for (int r = 0; r < NROW; ++r) {
                    const int i = DIM == 2 ? r : row0;
                    double Fg = 0.0;
#pragma unroll
                    for (int J = 0; J < DIM; ++J) Fg += F[i][J] * gk[J];
                    if (pz == 1) facc[r] += wq * (mu * (Fg - pk[i]) + lam * lnJ * pk[i]);
                }
                if (k == 0 && pz == 1) {                // element energy, owned by its corner 0
                    double I1 = DIM == 2 ? 1.0 : 0.0;
#pragma unroll
                    for (int i = 0; i < DIM; ++i)
#pragma unroll
                        for (int J = 0; J < DIM; ++J) I1 += F[i][J] * F[i][J];
                    en += wq * (0.5 * mu * (I1 - 3.0) - mu * lnJ + 0.5 * lam * lnJ * lnJ);
                }
                const double c2 = mu - lam * lnJ;
#pragma unroll
                for (int c = 0; c < G::NC; ++c) {
                    int oi = 0, sc = 1;                 // in-plane offset index (x fastest)
#pragma unroll
                    for (int ax = 0; ax < 2; ++ax) { oi += (((c >> ax) & 1) - ((k >> ax) & 1) + 1) * sc; sc *= 3; }
                    if (DIM == 3 && (((c >> 2) & 1) - ((k >> 2) & 1) + 1) != pz) continue;
                    double gc[DIM], pc[DIM], gkgc = 0.0;
#pragma unroll
                    for (int J = 0; J < DIM; ++J) { gc[J] = shape_grad<DIM, RULE>(q, c, J, invh); gkgc += gk[J] * gc[J]; }
#pragma unroll
                    for (int i = 0; i < DIM; ++i) {
                        double s = 0.0;
#pragma unroll
                        for (int J = 0; J < DIM; ++J) s += H[i][J] * gc[J];
                        pc[i] = s;
                    }
#pragma unroll
                    for (int r = 0; r < NROW; ++r) {
                        const int i = DIM == 2 ? r : row0;
#pragma unroll
                        for (int j = 0; j < DIM; ++j) {
                            double v = c2 * pk[j] * pc[i] + lam * pk[i] * pc[j];
                            if (i == j) v += mu * gkgc;
                            acc[oi][r][j] += wq * v;
                        }
                    }
                }
            }
    };
    if (cell >= 0) {
        element(std::integral_constant<int, 0>{});
        element(std::integral_constant<int, 1>{});
        element(std::integral_constant<int, 2>{});
        element(std::integral_constant<int, 3>{});
        if (DIM == 3) {
            element(std::integral_constant<int, 4>{});
            element(std::integral_constant<int, 5>{});
            element(std::integral_constant<int, 6>{});
            element(std::integral_constant<int, 7>{});
        }
    }
    // ---- outputs
    constexpr int E = G::E;
    const int obase = DIM == 3 ? 9 * pz : 0;
    if (PRINCIPAL) {
#pragma unroll
        for (int o = 0; o < NOP; ++o)
#pragma unroll
            for (int r = 0; r < NROW; ++r)
#pragma unroll
                for (int j = 0; j < DIM; ++j) {
                    const int i = DIM == 2 ? r : row0;
                    const int ent = ((obase + o) * DIM + i) * DIM + j;
                    A.Kst[((int64_t)a * E + ent) * A.cap + slot] = acc[o][r][j];
                }
        return;
    }
    if (A.f && pz == 1) {
#pragma unroll
        for (int r = 0; r < NROW; ++r) {
            const int i = DIM == 2 ? r : row0;
            A.f[((int64_t)a * DIM + i) * ld + p] = facc[r];
        }
    }
    if (A.epart && row0 == 0 && pz == 1) A.epart[(int64_t)a * ld + p] = en;
    // stencil rows and packed operators: written once, larger than L2 (non-temporal stores)
    if (A.T) {
#pragma unroll
        for (int o = 0; o < NOP; ++o)
#pragma unroll
            for (int r = 0; r < NROW; ++r)
#pragma unroll
                for (int j = 0; j < DIM; ++j) {
                    const int i = DIM == 2 ? r : row0;
                    const int ent = ((obase + o) * DIM + i) * DIM + j;
                    __builtin_nontemporal_store(acc[o][r][j], &A.T[((int64_t)arow * E + ent) * ld + p]);
                }
    }
    if (A.ops) {
        const int g = (int)(p / LAT_WAVE), l = (int)(p % LAT_WAVE);
        const int qi = A.uidx[(int64_t)g * A.nloc + a];
        if (qi >= 0) {
            const int64_t q = A.goff[g] + qi;
#pragma unroll
            for (int o = 0; o < NOP; ++o)
#pragma unroll
                for (int r = 0; r < NROW; ++r)
#pragma unroll
                    for (int j = 0; j < DIM; ++j) {
                        const int i = DIM == 2 ? r : row0;
                        const int ent = ((obase + o) * DIM + i) * DIM + j;
                        __builtin_nontemporal_store(acc[o][r][j], &A.ops[(q * E + ent) * LAT_WAVE + l]);
                    }
        }
    }
}

// 3D residual, energy and tangent with the quadrature-point data computed once per element and
// node.  One workgroup of 9 waves per (group of 64 lanes, node a); wave w owns tangent row
// i = w / 3 and offset plane pz = w % 3 of node a's stencil (27 entries).  For each of the up to 8
// elements around a (a is the element's corner k), waves 0..NQ-1 take one quadrature point each:
// F, H = F^{-T}, c2 = mu - lam ln J, the force row P g_a and, when a is the element's corner 0, the
// energy (kept in registers); (H, c2, w) go to LDS, w the point's weight for lanes that keep the
// element and 0 otherwise.  After a barrier every wave whose plane the element touches accumulates
//   K[(a,i),(c,j)] += w [ mu d_ij (g_a . g_c) + c2 (p_a)_j (p_c)_i + lam (p_a)_i (p_c)_j ],  p = H g,
// over the points and the element's four corners c in that plane.  Elements that no lane keeps
// are skipped (a workgroup-uniform decision: every wave sees the same 64 lanes).  The force rows and
// energies of the point-waves are summed in point order at the end.
constexpr int CELL3_GPV = 11;        // per quadrature point: H (9), c2, w

template <int RULE, bool PRINCIPAL>
__global__ __launch_bounds__(576) void k_cell3(CellArgs A)
{
    using G = Geo<3>;
    constexpr int NQ = RULE == LAT_RULE_REDUCED ? 1 : 8;
    __shared__ double gp[NQ * CELL3_GPV * 64];
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int l = threadIdx.x & 63;
    const int row = w / 3, pz = w % 3;
    const int nel = A.nel, nn = nel + 1;
    const int64_t ld = A.ld;
    const int arow = blockIdx.y;
    int a = arow;
    if (RULE == LAT_RULE_SAMPLED) {
        const int nsa = A.nsa;
        a = LAT_SAMPLE_STRIDE * ((arow % nsa) + nn * ((arow / nsa) % nsa) + nn * nn * (arow / (nsa * nsa)));
    }
    int64_t p;
    int cell, slot = 0;
    if (PRINCIPAL) {
        slot = l;
        cell = slot < A.n_r ? A.S[slot] : -1;
        p = cell >= 0 ? A.lane[cell] : 0;
    } else {
        p = (int64_t)blockIdx.x * LAT_WAVE + l;
        cell = A.perm[p];
    }
    const double h = 1.0 / nel, invh = (double)nel;
    const double wq = (RULE == LAT_RULE_REDUCED ? 1.0 : 0.125) * h * h * h;
    double mu = 0.0, lam = 0.0;
    if (cell >= 0) {
        mu = A.matmode == 0 ? A.mu[cell] : (A.matmode == 1 ? 1.0 : 0.0);
        lam = A.matmode == 0 ? A.lam[cell] : (A.matmode == 2 ? 1.0 : 0.0);
    }
    const int ia[3] = {a % nn, (a / nn) % nn, a / (nn * nn)};
    double acc[9][3];
#pragma unroll
    for (int o = 0; o < 9; ++o)
#pragma unroll
        for (int j = 0; j < 3; ++j) acc[o][j] = 0.0;
    double facc[3] = {0.0, 0.0, 0.0}, en = 0.0;

    auto element = [&](auto kc) __attribute__((always_inline)) {
        constexpr int k = decltype(kc)::value;
        int ie[3];
        bool ok = true;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            ie[ax] = ia[ax] - ((k >> ax) & 1);
            ok = ok && ie[ax] >= 0 && ie[ax] < nel;
        }
        if (!ok) return;                                        // the same for the whole workgroup
        const int e = ie[0] + nel * (ie[1] + nel * ie[2]);
        const bool kept = cell >= 0 && A.keep_il[(int64_t)e * ld + p];
        if (__builtin_amdgcn_ballot_w64(kept) == 0) return;     // no lane keeps it (uniform)
        // ---- quadrature-point phase: wave w < NQ takes point q = w
        if (w < NQ) {
            const int q = w;
            double Hs[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            double c2 = 0.0, wgt = 0.0;
            if (kept) {
                double ue[8][3];
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const int b = (ie[0] + (c & 1)) + nn * ((ie[1] + ((c >> 1) & 1)) + nn * (ie[2] + ((c >> 2) & 1)));
#pragma unroll
                    for (int i = 0; i < 3; ++i) ue[c][i] = A.u_cil[((int64_t)b * 3 + i) * ld + p];
                }
                double F[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
#pragma unroll
                for (int c = 0; c < 8; ++c)
#pragma unroll
                    for (int J = 0; J < 3; ++J) {
                        const double g = shape_grad<3, RULE>(q, c, J, invh);
#pragma unroll
                        for (int i = 0; i < 3; ++i) F[i][J] += ue[c][i] * g;
                    }
                double C[3][3];                                     // cofactors
                C[0][0] = F[1][1] * F[2][2] - F[1][2] * F[2][1];
                C[0][1] = F[1][2] * F[2][0] - F[1][0] * F[2][2];
                C[0][2] = F[1][0] * F[2][1] - F[1][1] * F[2][0];
                C[1][0] = F[0][2] * F[2][1] - F[0][1] * F[2][2];
                C[1][1] = F[0][0] * F[2][2] - F[0][2] * F[2][0];
                C[1][2] = F[0][1] * F[2][0] - F[0][0] * F[2][1];
                C[2][0] = F[0][1] * F[1][2] - F[0][2] * F[1][1];
                C[2][1] = F[0][2] * F[1][0] - F[0][0] * F[1][2];
                C[2][2] = F[0][0] * F[1][1] - F[0][1] * F[1][0];
                const double Jd = F[0][0] * C[0][0] + F[0][1] * C[0][1] + F[0][2] * C[0][2];
                const double r = 1.0 / Jd;
                double lnJ = 0.0;
                if (Jd > 0.0 && isfinite(Jd)) lnJ = log(Jd);
                else lat_flag(A.st, isfinite(Jd) ? LAT_E_INVERTED : LAT_E_NONFINITE, cell);
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int J = 0; J < 3; ++J) Hs[3 * i + J] = C[i][J] * r;
                c2 = mu - lam * lnJ;
                wgt = wq;
                // force rows at node a (corner k): P g_a = mu (F g_a - p_a) + lam ln J p_a
                double gk[3];
#pragma unroll
                for (int J = 0; J < 3; ++J) gk[J] = shape_grad<3, RULE>(q, k, J, invh);
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    double pk = 0.0, Fg = 0.0;
#pragma unroll
                    for (int J = 0; J < 3; ++J) {
                        pk += Hs[3 * i + J] * gk[J];
                        Fg += F[i][J] * gk[J];
                    }
                    facc[i] += wq * (mu * (Fg - pk) + lam * lnJ * pk);
                }
                if (k == 0) {                                       // element energy, owned by corner 0
                    double I1 = 0.0;
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int J = 0; J < 3; ++J) I1 += F[i][J] * F[i][J];
                    en += wq * (0.5 * mu * (I1 - 3.0) - mu * lnJ + 0.5 * lam * lnJ * lnJ);
                }
            }
#pragma unroll
            for (int t = 0; t < 9; ++t) gp[(q * CELL3_GPV + t) * 64 + l] = Hs[t];
            gp[(q * CELL3_GPV + 9) * 64 + l] = c2;
            gp[(q * CELL3_GPV + 10) * 64 + l] = wgt;
        }
        __syncthreads();
        // ---- accumulation phase: the element touches planes pz = 1 - k_z + {0, 1}
        const int kz = (k >> 2) & 1;
        if (pz == 1 || pz == 2 - 2 * kz) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                double Hq[9];
#pragma unroll
                for (int t = 0; t < 9; ++t) Hq[t] = gp[(q * CELL3_GPV + t) * 64 + l];
                const double c2 = gp[(q * CELL3_GPV + 9) * 64 + l];
                const double wgt = gp[(q * CELL3_GPV + 10) * 64 + l];
                double gk[3], pk[3];
#pragma unroll
                for (int J = 0; J < 3; ++J) gk[J] = shape_grad<3, RULE>(q, k, J, invh);
#pragma unroll
                for (int i = 0; i < 3; ++i) pk[i] = Hq[3 * i] * gk[0] + Hq[3 * i + 1] * gk[1] + Hq[3 * i + 2] * gk[2];
                const double pk_row = row == 0 ? pk[0] : (row == 1 ? pk[1] : pk[2]);
                double wc2pk[3];
#pragma unroll
                for (int j = 0; j < 3; ++j) wc2pk[j] = wgt * c2 * pk[j];
                const double wlpk = wgt * lam * pk_row, wmu = wgt * mu;
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    if ((((c >> 2) & 1) - kz + 1) != pz) continue;      // uniform per wave
                    int oi = 0, sc = 1;                                 // in-plane offset index (x fastest)
#pragma unroll
                    for (int ax = 0; ax < 2; ++ax) { oi += (((c >> ax) & 1) - ((k >> ax) & 1) + 1) * sc; sc *= 3; }
                    double gc[3], gkgc = 0.0;
#pragma unroll
                    for (int J = 0; J < 3; ++J) { gc[J] = shape_grad<3, RULE>(q, c, J, invh); gkgc += gk[J] * gc[J]; }
                    double pc[3];
#pragma unroll
                    for (int i = 0; i < 3; ++i) pc[i] = Hq[3 * i] * gc[0] + Hq[3 * i + 1] * gc[1] + Hq[3 * i + 2] * gc[2];
                    const double pc_row = row == 0 ? pc[0] : (row == 1 ? pc[1] : pc[2]);
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        double v = fma(wc2pk[j], pc_row, acc[oi][j]);
                        v = fma(wlpk, pc[j], v);
                        acc[oi][j] = (j == row) ? fma(wmu, gkgc, v) : v;
                    }
                }
            }
        }
        __syncthreads();                                        // gp is rewritten by the next element
    };
    element(std::integral_constant<int, 0>{});
    element(std::integral_constant<int, 1>{});
    element(std::integral_constant<int, 2>{});
    element(std::integral_constant<int, 3>{});
    element(std::integral_constant<int, 4>{});
    element(std::integral_constant<int, 5>{});
    element(std::integral_constant<int, 6>{});
    element(std::integral_constant<int, 7>{});

    // ---- outputs
    constexpr int E = G::E;
    const int obase = 9 * pz;
    if (PRINCIPAL) {
        if (slot < A.cap) {
#pragma unroll
            for (int o = 0; o < 9; ++o)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    A.Kst[((int64_t)a * E + ((obase + o) * 3 + row) * 3 + j) * A.cap + slot] = acc[o][j];
        }
        return;
    }
    if (A.f || A.epart) {
        // force rows and energy: the point-waves' partials through LDS, summed in point order
        double *fr = gp;                                        // [NQ][4][64], gp is free now
        if (w < NQ) {
#pragma unroll
            for (int i = 0; i < 3; ++i) fr[(w * 4 + i) * 64 + l] = facc[i];
            fr[(w * 4 + 3) * 64 + l] = en;
        }
        __syncthreads();
        if (w == 0) {
            double fs[3] = {0.0, 0.0, 0.0}, es = 0.0;
            for (int q = 0; q < NQ; ++q) {
#pragma unroll
                for (int i = 0; i < 3; ++i) fs[i] += fr[(q * 4 + i) * 64 + l];
                es += fr[(q * 4 + 3) * 64 + l];
            }
            if (A.f)
#pragma unroll
                for (int i = 0; i < 3; ++i) A.f[((int64_t)a * 3 + i) * ld + p] = fs[i];
            if (A.epart) A.epart[(int64_t)a * ld + p] = es;
        }
    }
    if (A.T) {
#pragma unroll
        for (int o = 0; o < 9; ++o)
#pragma unroll
            for (int j = 0; j < 3; ++j) A.T[((int64_t)arow * E + ((obase + o) * 3 + row) * 3 + j) * ld + p] = acc[o][j];
    }
    if (A.ops) {
        const int g = (int)(p / LAT_WAVE);
        const int qi = A.uidx[(int64_t)g * A.nloc + a];
        if (qi >= 0) {
            const int64_t q = A.goff[g] + qi;
#pragma unroll
            for (int o = 0; o < 9; ++o)
#pragma unroll
                for (int j = 0; j < 3; ++j) A.ops[(q * E + ((obase + o) * 3 + row) * 3 + j) * LAT_WAVE + l] = acc[o][j];
        }
    }
}

// Trilinear shape-function gradients at the 2 x 2 x 2 Gauss points of the unit cube (before the 1/h
// scaling): g[q][c][J], q = qx + 2 qy + 4 qz, c = cx + 2 cy + 4 cz; and L[m] = sum_q g_a(q) . g_b(q)
// for corners with a ^ b = m (the sum depends on which axes the corners differ in only: reflecting
// the cube in an axis maps the Gauss points onto themselves).  The node-line kernel reads L; it forms
// the gradients themselves from the 1D coordinates (the same products, so the same values), which
// keeps them out of the scalar registers.
struct G3Table {
    double g[8][8][3];
    double L[8];
};
constexpr G3Table make_g3()
{
    G3Table t{};
    const double x[2] = {0.21132486540518711775, 0.78867513459481288225};   // 1/2 -+ 1/(2 sqrt 3)
    for (int q = 0; q < 8; ++q)
        for (int c = 0; c < 8; ++c)
            for (int J = 0; J < 3; ++J) {
                double v = 1.0;
                for (int ax = 0; ax < 3; ++ax) {
                    const int kq = (q >> ax) & 1, bit = (c >> ax) & 1;
                    if (ax == J) v *= bit ? 1.0 : -1.0;
                    else v *= bit ? x[kq] : 1.0 - x[kq];
                }
                t.g[q][c][J] = v;
            }
    for (int m = 0; m < 8; ++m) {
        double s = 0.0;
        for (int q = 0; q < 8; ++q)
            for (int J = 0; J < 3; ++J) s += t.g[q][0][J] * t.g[q][m][J];
        t.L[m] = s;
    }
    return t;
}
__constant__ G3Table c_g3 = make_g3();

// Full-rule 3D residual and tangent by node lines.  A workgroup owns the node line (y0, z0) of 64 cell
// lanes and sweeps it in x: at step ex the (up to) four elements (ex, y0 - 1 + dy, z0 - 1 + dz) touch
// the line's nodes x = ex (their corner with x-bit 0) and x = ex + 1 (x-bit 1).  Each kept element's
// eight Gauss points are formed once per line, four at a time: the corner vectors p_c = F^{-T} g_c of
// all eight corners, w (mu - lam ln J), the points' force terms w P g_a of the two line nodes and
// the point's energy go to LDS.  The node rows follow from
//   K[(a,i),(b,j)] += w [ (mu - lam ln J) (p_a)_j (p_b)_i + lam (p_a)_i (p_b)_j ]
// summed over the points, plus mu d_ij sum_q w g_a . g_b = mu d_ij (h/8) L[a ^ b] once per element.
//
// Two roles of four waves each.  The point waves form one chunk (four points of one element) into
// one of two LDS buffers and meet the barrier; the accumulation waves meet the same barrier and then
// sum that chunk while the point waves form the next one into the other buffer.  Accumulation wave
// (s, t) holds the 81 entries (oy, oz, i, j) of one x-offset block of one node row: when ex + s is
// even its node is x = ex, else x = ex + 1; t = 0 takes the corners b at the node's own x (offset 0,
// summed over the two steps that touch the node, then written), t = 1 those at the other x (offset
// +1 or -1, complete after one step).  Every entry of every node row is written once, by one wave:
// no atomics.  Wave (0, 0) also sums the force rows and element energies (owned by the element's
// corner 0) in point order.  Lanes that do not keep an element form F = I at its points and give it
// zero weight.  The roles are separate branches, so the accumulators are not live where the points
// are formed and two waves fit on a SIMD.
constexpr int LAT_TAN3_MAX_NEL = 16;     // element slots of a line fit one 64-bit mask (k_cell3 above)

template <bool PRINCIPAL, bool SAMPLED>
__global__ __launch_bounds__(512) void k_tan3(CellArgs A)
{
    constexpr int E = Geo<3>::E;
    // per point: p_c [cx][cy + 2 cz][i] (24), w (mu - lam ln J), w P g of x = ex (3) and x = ex + 1 (3),
    // w W (energy)
    constexpr int PV = 32;
    __shared__ double pd[8 * PV * 64];           // the eight points of one element
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int l = threadIdx.x & 63;
    const int nel = A.nel, nn = nel + 1;
    const int64_t ld = A.ld;
    // sampled entries: the lines through the sub-grid nodes, whose rows are stored alone, in sub-grid
    // order (the same arithmetic as the full sweep, so the same bits)
    constexpr int SS = LAT_SAMPLE_STRIDE;
    const int nsa = A.nsa;
    const int y0 = SAMPLED ? SS * ((int)blockIdx.y % nsa) : (int)blockIdx.y % nn;
    const int z0 = SAMPLED ? SS * ((int)blockIdx.y / nsa) : (int)blockIdx.y / nn;
    const int line = nn * (y0 + nn * z0);         // node index of x = 0 on the line
    int64_t p;
    int cell, slot = 0;
    if (PRINCIPAL) {
        slot = l;
        cell = slot < A.n_r ? A.S[slot] : -1;
        p = cell >= 0 ? A.lane[cell] : 0;
    } else {
        p = (int64_t)blockIdx.x * LAT_WAVE + l;
        cell = A.perm[p];
    }
    const double h = 1.0 / nel, invh = (double)nel;
    const double wq = 0.125 * h * h * h;
    double mu = 0.0, lam = 0.0;
    if (cell >= 0) {
        mu = A.matmode == 0 ? A.mu[cell] : (A.matmode == 1 ? 1.0 : 0.0);
        lam = A.matmode == 0 ? A.lam[cell] : (A.matmode == 2 ? 1.0 : 0.0);
    }
    const bool forces = !PRINCIPAL && !SAMPLED && (A.f || A.epart);
    const uint32_t poff0 = (uint32_t)p * 8u;
    // the line's element slots 4 ex + dy + 2 dz (ex < nel <= 16): bit set in `pmask` when the element
    // (ex, y0 - 1 + dy, z0 - 1 + dz) exists and some lane keeps it (uniform over the workgroup: every
    // wave holds the same 64 lanes), in `kmask` when this lane keeps it
    uint64_t pmask = 0, kmask = 0;
    for (int sl = 0; sl < 4 * nel; ++sl) {
        const int ex = sl >> 2, ey = y0 - 1 + (sl & 1), ez = z0 - 1 + ((sl >> 1) & 1);
        bool kept = false;
        if (ey >= 0 && ey < nel && ez >= 0 && ez < nel && cell >= 0)
            kept = *((const uint8_t *)(A.keep_il + (int64_t)(ex + nel * (ey + nel * ez)) * ld) + (poff0 >> 3));
        if (kept) kmask |= 1ull << sl;
        if (__builtin_amdgcn_ballot_w64(kept) != 0) pmask |= 1ull << sl;
    }

    if (w >= 4) {
        // ================= point role =================
        // Points gw and gw + 4 of each kept element (in slot order), formed together in registers while
        // the accumulation waves read the previous element from LDS; between two barriers they are
        // written to LDS.  The next element's corner displacements are loaded before that.
        const int gw = w - 4;
        // 1D Gauss coordinates (1/2 -+ 1/(2 sqrt 3)) of this wave's points in x and y, and the
        // products phi_x phi_y of the gradients' z components (the same for both points)
        constexpr double GX0 = 0.21132486540518711775, GX1 = 0.78867513459481288225;
        const double px1 = (gw & 1) ? GX1 : GX0, px0 = 1.0 - px1;
        const double py1 = (gw >> 1) ? GX1 : GX0, py0 = 1.0 - py1;
        double Cxy[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) Cxy[t] = ((t & 1) ? px1 : px0) * ((t >> 1) ? py1 : py0);
        uint64_t m = pmask;
        double u[8][3];
        auto load_u = [&](int sl) __attribute__((always_inline)) {
            const int ex = sl >> 2, ey = y0 - 1 + (sl & 1), ez = z0 - 1 + ((sl >> 1) & 1);
            const int nb0 = ex + nn * (ey + nn * ez);
            const bool kept = (kmask >> sl) & 1;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int b = nb0 + (c & 1) + nn * (((c >> 1) & 1) + nn * ((c >> 2) & 1));
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    u[c][i] = kept ? *(const double *)((const char *)(A.u_cil + ((int64_t)b * 3 + i) * ld) + poff0) : 0.0;
            }
        };
        int sl = m ? __builtin_ctzll(m) : -1;
        if (sl >= 0) load_u(sl);
        while (sl >= 0) {
            m &= m - 1;
            const int dy = sl & 1, dz = (sl >> 1) & 1;
            const int kA = 2 * (1 - dy) + 4 * (1 - dz);          // corner of node x = ex (x = ex + 1: kA + 1)
            const double wk = ((kmask >> sl) & 1) ? wq : 0.0;
            // corner differences along each axis, shared by the two points: dX[y + 2z] = u(1,y,z) - u(0,y,z), ...
            double dX[4][3], dY[4][3], dZ[4][3];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int t0 = t & 1, t1 = t >> 1;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    dX[t][i] = u[1 + 2 * t0 + 4 * t1][i] - u[2 * t0 + 4 * t1][i];
                    dY[t][i] = u[t0 + 2 + 4 * t1][i] - u[t0 + 4 * t1][i];
                    dZ[t][i] = u[t0 + 2 * t1 + 4][i] - u[t0 + 2 * t1][i];
                }
            }
            const int ay = 1 - dy, az = 1 - dz;                  // the line's corner bits in the element
            double out[2][PV];
#pragma unroll
            for (int h2 = 0; h2 < 2; ++h2) {
                // gradients at point (qx, qy, qz) = (gw & 1, gw >> 1, h2): for corner c = x + 2y + 4z,
                // ghat_c = (s(x) Ayz[y + 2z], s(y) B[x + 2z], s(z) Cxy[x + 2y]), s(b) = b ? 1 : -1,
                // Ayz = phi_y phi_z, Bxz = phi_x phi_z, Cxy = phi_x phi_y (the products in the table's order)
                const double pz1 = h2 ? GX1 : GX0, pz0 = 1.0 - pz1;
                double Ayz[4], Bxz[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    Ayz[t] = ((t & 1) ? py1 : py0) * ((t >> 1) ? pz1 : pz0);
                    Bxz[t] = ((t & 1) ? px1 : px0) * ((t >> 1) ? pz1 : pz0);
                }
                double F[3][3];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    double g0 = 0.0, g1 = 0.0, g2 = 0.0;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        g0 = fma(Ayz[t], dX[t][i], g0);
                        g1 = fma(Bxz[t], dY[t][i], g1);
                        g2 = fma(Cxy[t], dZ[t][i], g2);
                    }
                    F[i][0] = i == 0 ? fma(invh, g0, 1.0) : invh * g0;
                    F[i][1] = i == 1 ? fma(invh, g1, 1.0) : invh * g1;
                    F[i][2] = i == 2 ? fma(invh, g2, 1.0) : invh * g2;
                }
                // cofactors and J with every product-sum fused explicitly: the full and the sampled sweeps
                // then round identically whatever else the compiler sees around them
                double C[3][3];
                C[0][0] = fma(F[1][1], F[2][2], -(F[1][2] * F[2][1]));
                C[0][1] = fma(F[1][2], F[2][0], -(F[1][0] * F[2][2]));
                C[0][2] = fma(F[1][0], F[2][1], -(F[1][1] * F[2][0]));
                C[1][0] = fma(F[0][2], F[2][1], -(F[0][1] * F[2][2]));
                C[1][1] = fma(F[0][0], F[2][2], -(F[0][2] * F[2][0]));
                C[1][2] = fma(F[0][1], F[2][0], -(F[0][0] * F[2][1]));
                C[2][0] = fma(F[0][1], F[1][2], -(F[0][2] * F[1][1]));
                C[2][1] = fma(F[0][2], F[1][0], -(F[0][0] * F[1][2]));
                C[2][2] = fma(F[0][0], F[1][1], -(F[0][1] * F[1][0]));
                const double Jd = fma(F[0][0], C[0][0], fma(F[0][1], C[0][1], F[0][2] * C[0][2]));
                double lnJ = 0.0;
                if (Jd > 0.0 && isfinite(Jd)) lnJ = log(Jd);
                else if (wk != 0.0) lat_flag(A.st, isfinite(Jd) ? LAT_E_INVERTED : LAT_E_NONFINITE, cell);
                const double rh = invh / Jd;                            // p_c = (C / J)(ghat_c / h)
                double Ch[3][3];
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int J = 0; J < 3; ++J) Ch[i][J] = C[i][J] * rh;
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const int cx = c & 1, cy = (c >> 1) & 1, cz = c >> 2;
                    const double g0 = cx ? Ayz[cy + 2 * cz] : -Ayz[cy + 2 * cz];
                    const double g1 = cy ? Bxz[cx + 2 * cz] : -Bxz[cx + 2 * cz];
                    const double g2 = cz ? Cxy[cx + 2 * cy] : -Cxy[cx + 2 * cy];
#pragma unroll
                    for (int i = 0; i < 3; ++i)
                        out[h2][cx * 12 + (c >> 1) * 3 + i] = fma(Ch[i][0], g0, fma(Ch[i][1], g1, Ch[i][2] * g2));
                }
                out[h2][24] = wk * fma(-lam, lnJ, mu);
                if (forces) {
                    // force terms of the two line nodes (corners x + 2 ay + 4 az, x = 0, 1):
                    // w P g_a = w (mu (F g_a - p_a) + lam ln J p_a)
                    const double Aa = az ? (ay ? Ayz[3] : Ayz[2]) : (ay ? Ayz[1] : Ayz[0]);
#pragma unroll
                    for (int x = 0; x < 2; ++x) {
                        const double Ba = az ? Bxz[x + 2] : Bxz[x];
                        const double Ca = ay ? Cxy[x + 2] : Cxy[x];
                        const double g0 = x ? Aa : -Aa, g1 = ay ? Ba : -Ba, g2 = az ? Ca : -Ca;
#pragma unroll
                        for (int i = 0; i < 3; ++i) {
                            const double pa = fma(Ch[i][0], g0, fma(Ch[i][1], g1, Ch[i][2] * g2));
                            const double Fg = invh * fma(F[i][0], g0, fma(F[i][1], g1, F[i][2] * g2));
                            out[h2][25 + 3 * x + i] = wk * fma(mu, Fg - pa, lam * lnJ * pa);
                        }
                    }
                    double I1 = 0.0;
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int J = 0; J < 3; ++J) I1 += F[i][J] * F[i][J];
                    out[h2][31] = wk * (0.5 * mu * (I1 - 3.0) - mu * lnJ + 0.5 * lam * lnJ * lnJ);
                } else {
#pragma unroll
                    for (int v = 25; v < PV; ++v) out[h2][v] = 0.0;
                }
            }
            sl = m ? __builtin_ctzll(m) : -1;
            if (sl >= 0) load_u(sl);                             // the next element, during the write phase
            __syncthreads();                                     // the previous element has been read
#pragma unroll
            for (int h2 = 0; h2 < 2; ++h2)
#pragma unroll
                for (int v = 0; v < PV; ++v) pd[((gw + 4 * h2) * PV + v) * 64 + l] = out[h2][v];
            __syncthreads();                                     // this element is in LDS
        }
        return;
    }

    // ================= accumulation role =================
    const int s = w & 1, t = w >> 1;
    const bool fwave = forces && w == 0;
    const double muL = mu * 0.125 * h;            // mu sum_q w g_a . g_b = mu (h/8) L
    const double lw0 = wq * lam;
    double acc[9][9];
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
        for (int e = 0; e < 9; ++e) acc[k][e] = 0.0;
    double fc[3] = {0.0, 0.0, 0.0}, fn[3] = {0.0, 0.0, 0.0}, en = 0.0;
    // entries k9 = 3 (oz + 1) + oy + 1 in `mask` (a constant) of block ox of node x:
    // rows 9 (ox + 1) + 27 k9 + 3 i + j.  The stencil rows and packed operators are written once and
    // are far larger than L2: non-temporal stores (BCC 10^3 tangent 1.43 -> 1.17 ms).
    auto store = [&](auto maskc, int x, int ox, uint32_t poff) __attribute__((always_inline)) {
        constexpr int mask = decltype(maskc)::value;
        const int node = line + x;
        const uint32_t loff = (uint32_t)l * 8u;
        if (PRINCIPAL) {
            if (slot < A.cap) {
                const int64_t cap = A.cap;
                char *base = (char *)(A.Kst + ((int64_t)node * E + 9 * (ox + 1)) * cap);
#pragma unroll
                for (int k = 0; k < 9; ++k)
                    if ((mask >> k) & 1)
#pragma unroll
                        for (int e = 0; e < 9; ++e) *(double *)(base + (int64_t)(27 * k + e) * cap * 8 + loff) = acc[k][e];
            }
            return;
        }
        if (A.T) {
            int64_t orow = node;
            if (SAMPLED) {
                if (x % SS != 0 || x / SS >= nsa) return;
                orow = x / SS + nsa * (y0 / SS + nsa * (z0 / SS));
            }
            char *base = (char *)(A.T + (orow * E + 9 * (ox + 1)) * ld);
#pragma unroll
            for (int k = 0; k < 9; ++k)
                if ((mask >> k) & 1)
#pragma unroll
                    for (int e = 0; e < 9; ++e)
                        __builtin_nontemporal_store(acc[k][e], (double *)(base + (int64_t)(27 * k + e) * ld * 8 + poff));
        }
        if (A.ops) {
            const int g = (int)blockIdx.x;
            const int qi = A.uidx[(int64_t)g * A.nloc + node];
            if (qi >= 0) {
                const int64_t q = (int64_t)A.goff[g] + qi;         // packed node (64-bit: beyond 2^31 / (E 64))
                char *base = (char *)(A.ops + (q * E + 9 * (ox + 1)) * LAT_WAVE);
#pragma unroll
                for (int k = 0; k < 9; ++k)
                    if ((mask >> k) & 1)
#pragma unroll
                        for (int e = 0; e < 9; ++e)
                            __builtin_nontemporal_store(acc[k][e], (double *)(base + (int64_t)(27 * k + e) * LAT_WAVE * 8 + loff));
            }
        }
    };
    for (int ex = -1; ex <= nel; ++ex) {
        // the lane offset is made opaque at every step, so that no per-lane address is formed once
        // outside the sweep and kept live across it
        uint32_t poff = poff0;
        asm volatile("" : "+v"(poff));
        const int r = (ex + s) & 1;                            // my node: x = ex + r
        const int bx = r ^ t;                                  // x-bit of my block's corners b
        auto element = [&](auto dyc, auto dzc) __attribute__((always_inline)) {
            constexpr int dy = decltype(dyc)::value, dz = decltype(dzc)::value;
            constexpr int ay = 1 - dy, az = 1 - dz;            // the line's corner bits in the element
            const int sl = 4 * ex + dy + 2 * dz;
            if (ex >= 0 && ex < nel && ((pmask >> sl) & 1)) {
            const bool kept = (kmask >> sl) & 1;
            const double lw = kept ? lw0 : 0.0;
            {
                __syncthreads();                               // the point waves start writing
                __syncthreads();                               // the element's eight points are in LDS
                const double *buf = pd + l;
                const double *pa_base = buf + (r * 12 + (ay + 2 * az) * 3) * 64;
                const double *pb_base = buf + bx * 12 * 64;
#pragma unroll 1
                for (int qq = 0; qq < 8; ++qq) {
                    double c2pa[3], lpa[3];
                    const double c2w = buf[(qq * PV + 24) * 64];
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        const double pa = pa_base[(qq * PV + i) * 64];
                        c2pa[i] = c2w * pa;
                        lpa[i] = lw * pa;
                    }
#pragma unroll
                    for (int bz = 0; bz < 2; ++bz)
#pragma unroll
                        for (int by = 0; by < 2; ++by) {
                            const int k9 = (by - ay + 1) + 3 * (bz - az + 1);
                            double pb[3];
#pragma unroll
                            for (int j = 0; j < 3; ++j) pb[j] = pb_base[(qq * PV + (by + 2 * bz) * 3 + j) * 64];
#pragma unroll
                            for (int i = 0; i < 3; ++i)
#pragma unroll
                                for (int j = 0; j < 3; ++j)
                                    acc[k9][3 * i + j] = fma(c2pa[j], pb[i], fma(lpa[i], pb[j], acc[k9][3 * i + j]));
                        }
                }
                if (fwave) {
                    for (int qq = 0; qq < 8; ++qq) {
#pragma unroll
                        for (int i = 0; i < 3; ++i) {
                            fc[i] += buf[(qq * PV + 25 + i) * 64];
                            fn[i] += buf[(qq * PV + 28 + i) * 64];
                        }
                        if (dy == 1 && dz == 1) en += buf[(qq * PV + 31) * 64];
                    }
                }
            }
            // mu d_ij (h/8) L[a ^ b], once per element; a ^ b = t + 2 (ay ^ by) + 4 (az ^ bz)
            const double mk = kept ? muL : 0.0;
#pragma unroll
            for (int bz = 0; bz < 2; ++bz)
#pragma unroll
                for (int by = 0; by < 2; ++by) {
                    const int k9 = (by - ay + 1) + 3 * (bz - az + 1);
                    const double L = c_g3.L[t + 2 * (ay ^ by) + 4 * (az ^ bz)];
                    acc[k9][0] = fma(mk, L, acc[k9][0]);
                    acc[k9][4] = fma(mk, L, acc[k9][4]);
                    acc[k9][8] = fma(mk, L, acc[k9][8]);
                }
            }
            // Blocks that are complete after this step (t = 1 always: offset +1 of x = ex or -1 of
            // x = ex + 1; t = 0 when its node is x = ex: offset 0; steps -1 and nel write the line's zero
            // end blocks) are written in four parts, each as soon as no later element of the step
            // touches it: after element (0, 0) the entries (oy, oz) = (-1, -1), after (1, 0) the rest
            // of oz = -1, after (0, 1) the rest of oy = -1, after (1, 1) the others.  The stores are
            // spread over the step instead of queueing at its end.
            constexpr int gmask = dy == 0 && dz == 0 ? 0x001 : dz == 0 ? 0x006 : dy == 0 ? 0x048 : 0x1b0;
            const int x = ex + (t == 1 ? r : 0);
            if ((t == 1 || r == 0) && x >= 0 && x <= nel) {
                store(std::integral_constant<int, gmask>{}, x, t == 0 ? 0 : (r ? -1 : 1), poff);
#pragma unroll
                for (int k = 0; k < 9; ++k)
                    if ((gmask >> k) & 1)
#pragma unroll
                        for (int e = 0; e < 9; ++e) acc[k][e] = 0.0;
            }
        };
        element(std::integral_constant<int, 0>{}, std::integral_constant<int, 0>{});
        element(std::integral_constant<int, 1>{}, std::integral_constant<int, 0>{});
        element(std::integral_constant<int, 0>{}, std::integral_constant<int, 1>{});
        element(std::integral_constant<int, 1>{}, std::integral_constant<int, 1>{});
        // node x = ex is complete: its force row and energy; the next node's partials move up
        if (fwave && ex >= 0) {
            const int node = line + ex;
            if (A.f)
#pragma unroll
                for (int i = 0; i < 3; ++i) *(double *)((char *)(A.f + ((int64_t)node * 3 + i) * ld) + poff) = fc[i];
            if (A.epart) *(double *)((char *)(A.epart + (int64_t)node * ld) + poff) = en;
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) { fc[i] = fn[i]; fn[i] = 0.0; }
        en = 0.0;
    }
}

// Internal force and energy without the tangent (a residual evaluation, e.g. a line-search trial).
// One thread per (lane, element) of one parity colour: the elements whose index along every axis
// has the colour's parity share no node, so each thread adds its corner forces f_c = sum_q w P g_c
// to f without atomics; the colours run in a fixed order (deterministic).  The element energy
// goes to epart row e (every element is in exactly one colour).
template <int DIM>
__global__ __launch_bounds__(256) void k_force_color(int nel, int64_t ld, int color, const double *__restrict__ u_cil,
                                                     const uint8_t *__restrict__ keep_il,
                                                     const int32_t *__restrict__ perm, const double *__restrict__ mu_a,
                                                     const double *__restrict__ lam_a, double *__restrict__ f,
                                                     double *__restrict__ epart, int32_t *st)
{
    using G = Geo<DIM>;
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= ld) return;
    const int nn = nel + 1;
    int cnt[3] = {1, 1, 1}, ie[3] = {0, 0, 0};
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) cnt[ax] = (nel - ((color >> ax) & 1) + 1) / 2;
    int rest = blockIdx.y;
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
        ie[ax] = 2 * (rest % cnt[ax]) + ((color >> ax) & 1);
        rest /= cnt[ax];
    }
    if (rest > 0) return;                                       // past this colour's elements
    const int e = ie[0] + nel * (ie[1] + nel * ie[2]);
    const int cell = perm[p];
    double en = 0.0;
    if (cell >= 0 && keep_il[(int64_t)e * ld + p]) {
        const double mu = mu_a[cell], lam = lam_a[cell];
        const double h = 1.0 / nel, invh = (double)nel;
        double hd = h;
#pragma unroll
        for (int ax = 1; ax < DIM; ++ax) hd *= h;
        const double wq = (DIM == 2 ? 0.25 : 0.125) * hd;
        int node[G::NC];
        double ue[G::NC][DIM], fe[G::NC][DIM];
#pragma unroll
        for (int c = 0; c < G::NC; ++c) {
            node[c] = (ie[0] + (c & 1)) + nn * ((ie[1] + ((c >> 1) & 1)) + nn * (DIM == 3 ? ie[2] + ((c >> 2) & 1) : 0));
#pragma unroll
            for (int i = 0; i < DIM; ++i) {
                ue[c][i] = u_cil[((int64_t)node[c] * DIM + i) * ld + p];
                fe[c][i] = 0.0;
            }
        }
#pragma unroll
        for (int q = 0; q < (1 << DIM); ++q) {
            double F[DIM][DIM];
#pragma unroll
            for (int i = 0; i < DIM; ++i)
#pragma unroll
                for (int J = 0; J < DIM; ++J) F[i][J] = (i == J) ? 1.0 : 0.0;
#pragma unroll
            for (int c = 0; c < G::NC; ++c)
#pragma unroll
                for (int J = 0; J < DIM; ++J) {
                    const double g = shape_grad<DIM, LAT_RULE_FULL>(q, c, J, invh);
#pragma unroll
                    for (int i = 0; i < DIM; ++i) F[i][J] += ue[c][i] * g;
                }
            double Jd, H[DIM][DIM];
            if (DIM == 2) {
                Jd = F[0][0] * F[1][1] - F[0][1] * F[1][0];
                const double r = 1.0 / Jd;
                H[0][0] = F[1][1] * r; H[0][1] = -F[1][0] * r;
                H[1][0] = -F[0][1] * r; H[1][1] = F[0][0] * r;
            } else {
                double C[3][3];
                C[0][0] = F[1][1] * F[2][2] - F[1][2] * F[2][1];
                C[0][1] = F[1][2] * F[2][0] - F[1][0] * F[2][2];
                C[0][2] = F[1][0] * F[2][1] - F[1][1] * F[2][0];
                C[1][0] = F[0][2] * F[2][1] - F[0][1] * F[2][2];
                C[1][1] = F[0][0] * F[2][2] - F[0][2] * F[2][0];
                C[1][2] = F[0][1] * F[2][0] - F[0][0] * F[2][1];
                C[2][0] = F[0][1] * F[1][2] - F[0][2] * F[1][1];
                C[2][1] = F[0][2] * F[1][0] - F[0][0] * F[1][2];
                C[2][2] = F[0][0] * F[1][1] - F[0][1] * F[1][0];
                Jd = F[0][0] * C[0][0] + F[0][1] * C[0][1] + F[0][2] * C[0][2];
                const double r = 1.0 / Jd;
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int J = 0; J < 3; ++J) H[i][J] = C[i][J] * r;
            }
            double lnJ = 0.0;
            if (Jd > 0.0 && isfinite(Jd)) lnJ = log(Jd);
            else lat_flag(st, isfinite(Jd) ? LAT_E_INVERTED : LAT_E_NONFINITE, cell);
            // P = mu (F - H) + lam ln J H
            double Pm[DIM][DIM], I1 = DIM == 2 ? 1.0 : 0.0;
#pragma unroll
            for (int i = 0; i < DIM; ++i)
#pragma unroll
                for (int J = 0; J < DIM; ++J) {
                    Pm[i][J] = mu * (F[i][J] - H[i][J]) + lam * lnJ * H[i][J];
                    I1 += F[i][J] * F[i][J];
                }
            en += wq * (0.5 * mu * (I1 - 3.0) - mu * lnJ + 0.5 * lam * lnJ * lnJ);
#pragma unroll
            for (int c = 0; c < G::NC; ++c)
#pragma unroll
                for (int i = 0; i < DIM; ++i) {
                    double s = 0.0;
#pragma unroll
                    for (int J = 0; J < DIM; ++J) s += Pm[i][J] * shape_grad<DIM, LAT_RULE_FULL>(q, c, J, invh);
                    fe[c][i] += wq * s;
                }
        }
        if (f)
#pragma unroll
            for (int c = 0; c < G::NC; ++c)
#pragma unroll
                for (int i = 0; i < DIM; ++i) f[((int64_t)node[c] * DIM + i) * ld + p] += fe[c][i];
    }
    if (epart) epart[(int64_t)e * ld + p] = en;
}

// u^s = A^{sT} u gathered into the cell-interleaved layout (zero at nodes a cell does not own).
__global__ void k_gather_u(int dim, int nloc, int64_t ld, const int32_t *__restrict__ l2g_il,
                           const int32_t *__restrict__ perm, const double *__restrict__ ug,
                           double *__restrict__ u_cil, int32_t *st)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int a = blockIdx.y;
    if (p >= ld) return;
    int g = l2g_il[(int64_t)a * ld + p];
    for (int i = 0; i < dim; ++i) {
        double v = g >= 0 ? ug[(int64_t)g * dim + i] : 0.0;
        if (!isfinite(v)) { lat_flag(st, LAT_E_NONFINITE, perm[p]); v = 0.0; }
        u_cil[((int64_t)a * dim + i) * ld + p] = v;
    }
}

__global__ void k_scatter_lanes(int64_t ld, const int32_t *__restrict__ perm, const double *__restrict__ v,
                                double *__restrict__ out)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ld) return;
    int c = perm[p];
    if (c >= 0) out[c] = v[p];
}

// Reverse mode of the residual at one node: (K^T w)_a = sum_e sum_q w_q dP(Gw) g_a with
// dP(G) = mu G + (mu - lam ln J) H G^T H + lam tr(G F^{-1}) H  (A's major symmetry), and the
// Lame-parameter parts <w_a, f^mu_a>, <w_a, f^lam_a>.
template <int DIM>
__global__ __launch_bounds__(256) void k_residual_adjoint(int nel, int64_t ld, const double *__restrict__ u_cil,
                                                          const double *__restrict__ w_cil,
                                                          const uint8_t *__restrict__ keep_il,
                                                          const int32_t *__restrict__ perm,
                                                          const double *__restrict__ mu_a,
                                                          const double *__restrict__ lam_a,
                                                          double *__restrict__ ubar, double *__restrict__ pmu,
                                                          double *__restrict__ plam, int32_t *st)
{
    using G = Geo<DIM>;
    constexpr int NQ = 1 << DIM;
    const int nn = nel + 1;
    const int a = blockIdx.y;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ld) return;
    const int cell = perm[p];
    const double h = 1.0 / nel, invh = (double)nel;
    double hd = h;
#pragma unroll
    for (int ax = 1; ax < DIM; ++ax) hd *= h;
    const double wq = (DIM == 2 ? 0.25 : 0.125) * hd;
    const int ia[3] = {a % nn, (a / nn) % nn, DIM == 3 ? a / (nn * nn) : 0};
    double ub[DIM], fm[DIM], fl[DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i) { ub[i] = 0.0; fm[i] = 0.0; fl[i] = 0.0; }
    double mu = 0.0, lam = 0.0;
    if (cell >= 0) { mu = mu_a[cell]; lam = lam_a[cell]; }
    if (cell >= 0) {
#pragma unroll
        for (int k = 0; k < G::NC; ++k) {
            int ie[3] = {0, 0, 0};
            bool ok = true;
#pragma unroll
            for (int ax = 0; ax < DIM; ++ax) {
                ie[ax] = ia[ax] - ((k >> ax) & 1);
                ok = ok && ie[ax] >= 0 && ie[ax] < nel;
            }
            if (!ok) continue;
            const int e = ie[0] + nel * (ie[1] + nel * ie[2]);
            if (!keep_il[(int64_t)e * ld + p]) continue;
            double ue[G::NC][DIM], we[G::NC][DIM];
#pragma unroll
            for (int c = 0; c < G::NC; ++c) {
                int b = (ie[0] + (c & 1)) + nn * ((ie[1] + ((c >> 1) & 1)) + nn * (DIM == 3 ? ie[2] + ((c >> 2) & 1) : 0));
#pragma unroll
                for (int i = 0; i < DIM; ++i) {
                    ue[c][i] = u_cil[((int64_t)b * DIM + i) * ld + p];
                    we[c][i] = w_cil[((int64_t)b * DIM + i) * ld + p];
                }
            }
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                double F[DIM][DIM], Gw[DIM][DIM];
#pragma unroll
                for (int i = 0; i < DIM; ++i)
#pragma unroll
                    for (int J = 0; J < DIM; ++J) { F[i][J] = (i == J) ? 1.0 : 0.0; Gw[i][J] = 0.0; }
#pragma unroll
                for (int c = 0; c < G::NC; ++c)
#pragma unroll
                    for (int J = 0; J < DIM; ++J) {
                        const double g = shape_grad<DIM, LAT_RULE_FULL>(q, c, J, invh);
#pragma unroll
                        for (int i = 0; i < DIM; ++i) { F[i][J] += ue[c][i] * g; Gw[i][J] += we[c][i] * g; }
                    }
                double Jd, H[DIM][DIM];
                if (DIM == 2) {
                    Jd = F[0][0] * F[1][1] - F[0][1] * F[1][0];
                    const double r = 1.0 / Jd;
                    H[0][0] = F[1][1] * r; H[0][1] = -F[1][0] * r;
                    H[1][0] = -F[0][1] * r; H[1][1] = F[0][0] * r;
                } else {
                    double C[3][3];
                    C[0][0] = F[1][1] * F[2][2] - F[1][2] * F[2][1];
                    C[0][1] = F[1][2] * F[2][0] - F[1][0] * F[2][2];
                    C[0][2] = F[1][0] * F[2][1] - F[1][1] * F[2][0];
                    C[1][0] = F[0][2] * F[2][1] - F[0][1] * F[2][2];
                    C[1][1] = F[0][0] * F[2][2] - F[0][2] * F[2][0];
                    C[1][2] = F[0][1] * F[2][0] - F[0][0] * F[2][1];
                    C[2][0] = F[0][1] * F[1][2] - F[0][2] * F[1][1];
                    C[2][1] = F[0][2] * F[1][0] - F[0][0] * F[1][2];
                    C[2][2] = F[0][0] * F[1][1] - F[0][1] * F[1][0];
                    Jd = F[0][0] * C[0][0] + F[0][1] * C[0][1] + F[0][2] * C[0][2];
                    const double r = 1.0 / Jd;
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int J = 0; J < 3; ++J) H[i][J] = C[i][J] * r;
                }
                double lnJ = 0.0;
                if (Jd > 0.0 && isfinite(Jd)) lnJ = log(Jd);
                else lat_flag(st, isfinite(Jd) ? LAT_E_INVERTED : LAT_E_NONFINITE, cell);
                // tr(Gw F^{-1}) = sum_iJ Gw_iJ Finv_Ji = sum_iJ Gw_iJ H_iJ
                double tr = 0.0;
#pragma unroll
                for (int i = 0; i < DIM; ++i)
#pragma unroll
                    for (int J = 0; J < DIM; ++J) tr += Gw[i][J] * H[i][J];
                // M = H Gw^T H
                double M[DIM][DIM];
#pragma unroll
                for (int j = 0; j < DIM; ++j)
#pragma unroll
                    for (int L = 0; L < DIM; ++L) {
                        double s = 0.0;
#pragma unroll
                        for (int x = 0; x < DIM; ++x)
#pragma unroll
                            for (int y = 0; y < DIM; ++y) s += H[j][x] * Gw[y][x] * H[y][L];
                        M[j][L] = s;
                    }
                double gk[DIM];
#pragma unroll
                for (int J = 0; J < DIM; ++J) gk[J] = shape_grad<DIM, LAT_RULE_FULL>(q, k, J, invh);
                const double c2 = mu - lam * lnJ;
#pragma unroll
                for (int j = 0; j < DIM; ++j) {
                    double s = 0.0, sfm = 0.0, sfl = 0.0;
#pragma unroll
                    for (int L = 0; L < DIM; ++L) {
                        s += (mu * Gw[j][L] + c2 * M[j][L] + lam * tr * H[j][L]) * gk[L];
                        sfm += (F[j][L] - H[j][L]) * gk[L];
                        sfl += lnJ * H[j][L] * gk[L];
                    }
                    ub[j] += wq * s;
                    fm[j] += wq * sfm;
                    fl[j] += wq * sfl;
                }
            }
        }
    }
    double dm = 0.0, dl = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        const double wa = cell >= 0 ? w_cil[((int64_t)a * DIM + i) * ld + p] : 0.0;
        dm += wa * fm[i];
        dl += wa * fl[i];
        if (ubar) ubar[((int64_t)a * DIM + i) * ld + p] = ub[i];
    }
    pmu[(int64_t)a * ld + p] = dm;
    plam[(int64_t)a * ld + p] = dl;
}

template <int DIM, int RULE, bool PRINCIPAL>
lat_status launch_cell(const lat_plan *P, CellArgs &A, hipStream_t s)
{
    if (DIM == 3 && RULE == LAT_RULE_FULL && P->nel <= LAT_TAN3_MAX_NEL) {
        const int nn = P->nel + 1;
        dim3 grid(PRINCIPAL ? 1u : (unsigned)(P->ld / LAT_WAVE), (unsigned)(nn * nn));
        hipLaunchKernelGGL((k_tan3<PRINCIPAL, false>), grid, dim3(512), 0, s, A);
        LAT_LAUNCH_CHECK();
        return LAT_OK;
    }
    if (DIM == 3) {
        dim3 grid(PRINCIPAL ? 1u : (unsigned)(P->ld / LAT_WAVE), (unsigned)P->nloc);
        hipLaunchKernelGGL((k_cell3<RULE, PRINCIPAL>), grid, dim3(576), 0, s, A);
        LAT_LAUNCH_CHECK();
        return LAT_OK;
    }
    if (PRINCIPAL) {
        dim3 grid(1, (unsigned)P->nloc, DIM == 3 ? 9 : 1);
        hipLaunchKernelGGL((k_cell<DIM, RULE, true>), grid, dim3(64), 0, s, A);
    } else {
        dim3 grid((unsigned)lat_cdiv(P->ld, 256), (unsigned)P->nloc, DIM == 3 ? 9 : 1);
        hipLaunchKernelGGL((k_cell<DIM, RULE, false>), grid, dim3(256), 0, s, A);
    }
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

template <bool PRINCIPAL>
lat_status dispatch_cell(const lat_plan *P, int rule, CellArgs &A, hipStream_t s)
{
    if (P->dim == 2)
        return rule == LAT_RULE_FULL ? launch_cell<2, LAT_RULE_FULL, PRINCIPAL>(P, A, s)
                                     : launch_cell<2, LAT_RULE_REDUCED, PRINCIPAL>(P, A, s);
    return rule == LAT_RULE_FULL ? launch_cell<3, LAT_RULE_FULL, PRINCIPAL>(P, A, s)
                                 : launch_cell<3, LAT_RULE_REDUCED, PRINCIPAL>(P, A, s);
}

CellArgs base_args(const lat_plan *P)
{
    CellArgs A{};
    A.nel = P->nel; A.nloc = P->nloc; A.ld = P->ld;
    A.u_cil = P->u_cil; A.keep_il = P->keep_il; A.perm = P->perm; A.lane = P->lane;
    A.uidx = P->uidx; A.goff = P->goff; A.cap = P->cap;
    return A;
}

// Material-tangent snapshots (the Remark on snapshots of Sec. 3.2.2: the cell-to-cell differences
// of the tangent sit in the pulled-back constitutive tensor): A = dP/dF at the centre of every kept
// element, A_iJkL = mu d_ik d_JL + (mu - lam ln J) F^-1_Li F^-1_Jk + lam F^-1_Ji F^-1_Lk (plane strain
// in 2D), in rows (e d^2 + i d + J) d^2 + k d + L of CIL(E); elements that are not kept give zeros.
template <int DIM>
__global__ __launch_bounds__(256) void k_material_snap(int nel, int64_t ld, const uint8_t *__restrict__ keep_il,
                                                       const int32_t *__restrict__ perm,
                                                       const double *__restrict__ u_cil, const double *__restrict__ mu,
                                                       const double *__restrict__ lam, double *__restrict__ T,
                                                       int32_t *st)
{
    constexpr int D4 = DIM * DIM * DIM * DIM;
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int e = blockIdx.y;
    if (p >= ld) return;
    const int c = perm[p];
    double out[D4];
#pragma unroll
    for (int t = 0; t < D4; ++t) out[t] = 0.0;
    if (c >= 0 && keep_il[(int64_t)e * ld + p]) {
        const int nn = nel + 1;
        const int ec[3] = {e % nel, (e / nel) % nel, e / (nel * nel)};
        const double g0 = nel * (DIM == 2 ? 0.5 : 0.25);   // |dN/dX| of a corner function at the centre
        double F[DIM][DIM];
#pragma unroll
        for (int i = 0; i < DIM; ++i)
#pragma unroll
            for (int J = 0; J < DIM; ++J) F[i][J] = i == J ? 1.0 : 0.0;
#pragma unroll
        for (int cb = 0; cb < (1 << DIM); ++cb) {
            int a = 0, str = 1;
#pragma unroll
            for (int ax = 0; ax < DIM; ++ax) {
                a += (ec[ax] + ((cb >> ax) & 1)) * str;
                str *= nn;
            }
#pragma unroll
            for (int i = 0; i < DIM; ++i) {
                const double ua = u_cil[((int64_t)a * DIM + i) * ld + p];
#pragma unroll
                for (int J = 0; J < DIM; ++J) F[i][J] = fma(ua, ((cb >> J) & 1) ? g0 : -g0, F[i][J]);
            }
        }
        double Fi[DIM][DIM], det;
        if (DIM == 2) {
            det = F[0][0] * F[1][1] - F[0][1] * F[1][0];
            Fi[0][0] = F[1][1] / det; Fi[0][1] = -F[0][1] / det;
            Fi[1][0] = -F[1][0] / det; Fi[1][1] = F[0][0] / det;
        } else {
            const double c00 = F[1][1] * F[2][2] - F[1][2] * F[2][1];
            const double c01 = F[1][2] * F[2][0] - F[1][0] * F[2][2];
            const double c02 = F[1][0] * F[2][1] - F[1][1] * F[2][0];
            det = F[0][0] * c00 + F[0][1] * c01 + F[0][2] * c02;
            const double id = 1.0 / det;
            Fi[0][0] = c00 * id; Fi[1][0] = c01 * id; Fi[2][0] = c02 * id;
            Fi[0][1] = (F[0][2] * F[2][1] - F[0][1] * F[2][2]) * id;
            Fi[1][1] = (F[0][0] * F[2][2] - F[0][2] * F[2][0]) * id;
            Fi[2][1] = (F[0][1] * F[2][0] - F[0][0] * F[2][1]) * id;
            Fi[0][2] = (F[0][1] * F[1][2] - F[0][2] * F[1][1]) * id;
            Fi[1][2] = (F[0][2] * F[1][0] - F[0][0] * F[1][2]) * id;
            Fi[2][2] = (F[0][0] * F[1][1] - F[0][1] * F[1][0]) * id;
        }
        if (!(det > 0.0) || !isfinite(det)) {
            lat_flag(st, isfinite(det) ? LAT_E_INVERTED : LAT_E_NONFINITE, c);
        } else {
            const double m = mu[c], l = lam[c], ml = m - l * log(det);
#pragma unroll
            for (int i = 0; i < DIM; ++i)
#pragma unroll
                for (int J = 0; J < DIM; ++J)
#pragma unroll
                    for (int k = 0; k < DIM; ++k)
#pragma unroll
                        for (int L = 0; L < DIM; ++L)
                            out[((i * DIM + J) * DIM + k) * DIM + L] = (i == k && J == L ? m : 0.0) +
                                                                       ml * Fi[L][i] * Fi[J][k] +
                                                                       l * Fi[J][i] * Fi[L][k];
        }
    }
#pragma unroll
    for (int t = 0; t < D4; ++t) T[((int64_t)e * D4 + t) * ld + p] = out[t];
}

__global__ void k_zero_rows(int64_t n, double *__restrict__ y)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        y[j] = 0.0;
}

// zeros in the snapshot rows past `rows` (the greedy over all n_snap rows then sees the same data)
lat_status zero_rows_past(const lat_plan *P, int64_t rows, double *snap, hipStream_t s)
{
    const int64_t rest = (P->nsnap - rows) * P->ld;
    if (rest > 0) {
        hipLaunchKernelGGL(k_zero_rows, dim3((unsigned)std::min<int64_t>(lat_cdiv(rest, 256), 4096)), dim3(256), 0, s,
                           rest, snap + rows * P->ld);
        LAT_LAUNCH_CHECK();
    }
    return LAT_OK;
}

lat_status gather_u(const lat_plan *P, const double *u_global, int32_t *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather_u, dim3((unsigned)lat_cdiv(P->ld, 256), (unsigned)P->nloc), dim3(256), 0, s, P->dim,
                       P->nloc, P->ld, P->l2g_il, P->perm, u_global, P->u_cil, st);
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

}  // namespace

extern "C" {

int64_t lat_snapshot_rows(const lat_plan *P, lat_rule rule)
{
    if (!P) return -1;
    const int64_t d2 = (int64_t)P->dim * P->dim;
    switch (rule) {
    case LAT_RULE_FULL:
    case LAT_RULE_REDUCED: return P->nsnap;
    case LAT_RULE_MATERIAL: return P->nelem * d2 * d2;
    case LAT_RULE_SAMPLED: return (int64_t)lat_ipow(P->nel / LAT_SAMPLE_STRIDE + 1, P->dim) * P->E;
    default: return -1;
    }
}

lat_status lat_residual_tangent(const lat_plan *Pp, const double *u_global, const double *mu, const double *lam,
                                lat_rule snap_rule, double *f_int, double *energy, double *snap, double *plain_ops,
                                int32_t *dev_status, void *work, size_t work_bytes, hipStream_t stream)
{
    if (!Pp || !u_global || !mu || !lam) return LAT_E_ARG;
    if (snap_rule != LAT_RULE_FULL && snap_rule != LAT_RULE_REDUCED && snap_rule != LAT_RULE_MATERIAL &&
        snap_rule != LAT_RULE_SAMPLED)
        return LAT_E_ARG;
    lat_plan V;
    lat_status st = lat_ws_bind(Pp, LAT_CALL_RESIDUAL_TANGENT, work, work_bytes, &V);
    if (st != LAT_OK) return st;
    const lat_plan *P = &V;
    st = gather_u(P, u_global, dev_status, stream);
    if (st != LAT_OK) return st;
    CellArgs A = base_args(P);
    A.mu = mu; A.lam = lam; A.matmode = 0; A.st = dev_status;
    const bool full_snap = snap && snap_rule == LAT_RULE_FULL;
    int64_t energy_rows = P->nloc;                   // rows of w_part holding energy partials
    if (plain_ops || full_snap) {
        A.f = f_int;
        A.epart = energy ? P->w_part : nullptr;
        A.T = full_snap ? snap : nullptr;
        A.ops = plain_ops;
        if ((st = dispatch_cell<false>(P, LAT_RULE_FULL, A, stream)) != LAT_OK) return st;
    } else if (f_int || energy) {
        // residual and energy only: element-centric, colour by colour
        if (f_int) {
            const int64_t nf = (int64_t)P->nloc * P->dim * P->ld;
            hipLaunchKernelGGL(k_zero_rows, dim3((unsigned)std::min<int64_t>(lat_cdiv(nf, 256), 8192)), dim3(256), 0,
                               stream, nf, f_int);
            LAT_LAUNCH_CHECK();
        }
        const int half = (P->nel + 1) / 2;
        const unsigned ecol = (unsigned)lat_ipow(half, P->dim);
        for (int color = 0; color < (1 << P->dim); ++color) {
            const dim3 grid((unsigned)lat_cdiv(P->ld, 256), ecol);
            if (P->dim == 2)
                hipLaunchKernelGGL(k_force_color<2>, grid, dim3(256), 0, stream, P->nel, P->ld, color, P->u_cil,
                                   P->keep_il, P->perm, mu, lam, f_int, energy ? P->w_part : nullptr, dev_status);
            else
                hipLaunchKernelGGL(k_force_color<3>, grid, dim3(256), 0, stream, P->nel, P->ld, color, P->u_cil,
                                   P->keep_il, P->perm, mu, lam, f_int, energy ? P->w_part : nullptr, dev_status);
            LAT_LAUNCH_CHECK();
        }
        energy_rows = P->nelem;
    }
    if (snap && snap_rule == LAT_RULE_REDUCED) {
        CellArgs B = base_args(P);
        B.mu = mu; B.lam = lam; B.matmode = 0; B.st = dev_status; B.T = snap;
        if ((st = dispatch_cell<false>(P, LAT_RULE_REDUCED, B, stream)) != LAT_OK) return st;
    }
    if (snap && snap_rule == LAT_RULE_MATERIAL) {
        const int d4 = P->dim * P->dim * P->dim * P->dim;
        const int64_t rows = (int64_t)P->nelem * d4;
        const dim3 grid((unsigned)lat_cdiv(P->ld, 256), (unsigned)P->nelem);
        if (P->dim == 2)
            hipLaunchKernelGGL(k_material_snap<2>, grid, dim3(256), 0, stream, P->nel, P->ld, P->keep_il, P->perm,
                               P->u_cil, mu, lam, snap, dev_status);
        else
            hipLaunchKernelGGL(k_material_snap<3>, grid, dim3(256), 0, stream, P->nel, P->ld, P->keep_il, P->perm,
                               P->u_cil, mu, lam, snap, dev_status);
        if ((st = zero_rows_past(P, rows, snap, stream)) != LAT_OK) return st;
    }
    if (snap && snap_rule == LAT_RULE_SAMPLED) {
        CellArgs B = base_args(P);
        B.mu = mu; B.lam = lam; B.matmode = 0; B.st = dev_status; B.T = snap;
        B.nsa = P->nel / LAT_SAMPLE_STRIDE + 1;
        const int64_t nsamp = lat_snapshot_rows(P, LAT_RULE_SAMPLED) / P->E;
        if (P->dim == 2)
            hipLaunchKernelGGL((k_cell<2, LAT_RULE_SAMPLED, false>), dim3((unsigned)lat_cdiv(P->ld, 256), (unsigned)nsamp),
                               dim3(256), 0, stream, B);
        else
            if (P->nel <= LAT_TAN3_MAX_NEL)
                hipLaunchKernelGGL((k_tan3<false, true>), dim3((unsigned)(P->ld / LAT_WAVE), (unsigned)(B.nsa * B.nsa)),
                                   dim3(512), 0, stream, B);
            else
                hipLaunchKernelGGL((k_cell3<LAT_RULE_SAMPLED, false>), dim3((unsigned)(P->ld / LAT_WAVE), (unsigned)nsamp),
                                   dim3(576), 0, stream, B);
        LAT_LAUNCH_CHECK();
        if ((st = zero_rows_past(P, nsamp * P->E, snap, stream)) != LAT_OK) return st;
    }
    if (energy) {
        if ((st = lat_tree_reduce(P->w_part, energy_rows, P->ld, 0, P->v_sq, P->g_t1, P->g_t2, stream)) != LAT_OK) return st;
        hipLaunchKernelGGL(k_scatter_lanes, dim3((unsigned)lat_cdiv(P->ld, 256)), dim3(256), 0, stream, P->ld, P->perm,
                           P->v_sq, energy);
        LAT_LAUNCH_CHECK();
    }
    return LAT_OK;
}

lat_status lat_principal_ops(const lat_plan *Pp, const double *u_global, const double *mu, const double *lam,
                             const int32_t *S, int32_t n_r, double *K, double *K_mu, double *K_lam,
                             int32_t *dev_status, void *work, size_t work_bytes, hipStream_t stream)
{
    if (!Pp || !u_global || !mu || !lam || !S || !K) return LAT_E_ARG;
    if (n_r < 0 || n_r > Pp->cap) return LAT_E_SHAPE;
    lat_plan V;
    lat_status st = lat_ws_bind(Pp, LAT_CALL_PRINCIPAL_OPS, work, work_bytes, &V);
    if (st != LAT_OK) return st;
    const lat_plan *P = &V;
    st = gather_u(P, u_global, dev_status, stream);
    if (st != LAT_OK) return st;
    double *outs[3] = {K, K_mu, K_lam};
    for (int mode = 0; mode < 3; ++mode) {
        if (!outs[mode]) continue;
        CellArgs A = base_args(P);
        A.mu = mu; A.lam = lam; A.matmode = mode; A.st = dev_status;
        A.S = S; A.n_r = n_r; A.Kst = outs[mode];
        if ((st = dispatch_cell<true>(P, LAT_RULE_FULL, A, stream)) != LAT_OK) return st;
    }
    return LAT_OK;
}

lat_status lat_residual_adjoint(const lat_plan *Pp, const double *u_global, const double *mu, const double *lam,
                                const double *w, double *ubar_local, double *ubar_global, double *mu_bar,
                                double *lam_bar, int32_t *dev_status, void *work, size_t work_bytes,
                                hipStream_t stream)
{
    if (!Pp || !u_global || !mu || !lam || !w) return LAT_E_ARG;
    if (ubar_global && !ubar_local) return LAT_E_ARG;     // assembly reads the local result
    lat_plan V;
    lat_status st = lat_ws_bind(Pp, LAT_CALL_RESIDUAL_ADJOINT, work, work_bytes, &V);
    if (st != LAT_OK) return st;
    const lat_plan *P = &V;
    st = gather_u(P, u_global, dev_status, stream);
    if (st != LAT_OK) return st;
    dim3 grid((unsigned)lat_cdiv(P->ld, 256), (unsigned)P->nloc);
    if (P->dim == 2)
        hipLaunchKernelGGL(k_residual_adjoint<2>, grid, dim3(256), 0, stream, P->nel, P->ld, P->u_cil, w, P->keep_il,
                           P->perm, mu, lam, ubar_local, P->w_part, P->w_part2, dev_status);
    else
        hipLaunchKernelGGL(k_residual_adjoint<3>, grid, dim3(256), 0, stream, P->nel, P->ld, P->u_cil, w, P->keep_il,
                           P->perm, mu, lam, ubar_local, P->w_part, P->w_part2, dev_status);
    LAT_LAUNCH_CHECK();
    if (mu_bar) {
        if ((st = lat_tree_reduce(P->w_part, P->nloc, P->ld, 0, P->v_sq, P->g_t1, P->g_t2, stream)) != LAT_OK) return st;
        hipLaunchKernelGGL(k_scatter_lanes, dim3((unsigned)lat_cdiv(P->ld, 256)), dim3(256), 0, stream, P->ld, P->perm,
                           P->v_sq, mu_bar);
        LAT_LAUNCH_CHECK();
    }
    if (lam_bar) {
        if ((st = lat_tree_reduce(P->w_part2, P->nloc, P->ld, 0, P->v_inf, P->g_t1, P->g_t2, stream)) != LAT_OK) return st;
        hipLaunchKernelGGL(k_scatter_lanes, dim3((unsigned)lat_cdiv(P->ld, 256)), dim3(256), 0, stream, P->ld, P->perm,
                           P->v_inf, lam_bar);
        LAT_LAUNCH_CHECK();
    }
    if (ubar_global) return lat_assemble(P, ubar_local, P->dim, ubar_global, stream);
    return LAT_OK;
}

}  // extern "C"
