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

typedef double v4d __attribute__((ext_vector_type(4)));

struct ApplyArgs {
    int nn, m, cap, n_r, nch, chunks_per_group, nseg;
    int rb, mc;               // walks: right-hand sides rb .. rb + mc - 1 of the m columns
    int64_t ld;
    const int32_t *gate;      // walks: run only when *gate != 0 (NULL: always)
    double *errp;             // reduced-precision walks: per-block error partials [2 * grid] (or NULL)
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

// Sum of (a, b) over the 512 threads of a walk workgroup (fixed order: wave butterflies, then the
// waves in order); thread 0 writes the pair to out[0..1].
__device__ __forceinline__ void block_sum2_512(double a, double b, double *red, double *out)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off);
        b += __shfl_xor(b, off);
    }
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) { red[2 * w] = a; red[2 * w + 1] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0.0, sb = 0.0;
        for (int t = 0; t < 8; ++t) { sa += red[2 * t]; sb += red[2 * t + 1]; }
        out[0] = sa;
        out[1] = sb;
    }
}

// MODE 0: ROM apply, 1: ROM apply transposed, 2: plain apply.
// Pointers are separate __restrict__ arguments: read-only, non-aliased memory lets wave-uniform
// reads (node tables, principal stack) go through the scalar cache.
template <int DIM, int MC, int NR, int MODE>
__global__ __launch_bounds__(256) void k_apply(ApplyArgs A, const int32_t *__restrict__ goff,
                                               const int32_t *__restrict__ unode, const int32_t *__restrict__ unbr,
                                               const uint64_t *__restrict__ umask, const double *__restrict__ K,
                                               const double *__restrict__ alpha_il, const double *__restrict__ X,
                                               double *__restrict__ Y)
{
    using G = Geo<DIM>;
    constexpr int E = G::E;
    // the wave index is uniform across the wave; say so, so that everything derived from it
    // (node ids, principal-stack addresses) is read with scalar loads
    const int wave = __builtin_amdgcn_readfirstlane(lat_xcd_block(blockIdx.x, gridDim.x) * 4 + (int)(threadIdx.x >> 6));
    const int l = threadIdx.x & 63;
    const int g = wave / A.chunks_per_group, ch = wave % A.chunks_per_group;
    if (g >= (int)(A.ld / LAT_WAVE)) return;
    // wave ch of the group takes nodes ch, ch + cpg, ch + 2 cpg, ...: at any moment the waves of
    // a group work on one compact band of nodes, whose stencil neighbourhoods overlap in L2
    const int cpg = A.chunks_per_group;
    const int q0 = goff[g] + ch;
    const int q1 = goff[g + 1];
    if (q0 >= q1) return;
    const int64_t p = (int64_t)g * LAT_WAVE + l;
    const int m = A.m;
    const int cap = A.cap;
    double alpha[MODE == 2 ? 1 : NR];
    if (MODE != 2) {
#pragma unroll
        for (int k = 0; k < NR; ++k) alpha[k] = alpha_il[(int64_t)k * A.ld + p];   // zero beyond n_r
    }
    for (int q = q0; q < q1; q += cpg) {
        const int a = unode[q];
        const uint64_t msk = umask[q];
        for (int c0 = 0; c0 < m; c0 += MC) {
            double acc[DIM][MC];
#pragma unroll
            for (int i = 0; i < DIM; ++i)
#pragma unroll
                for (int c = 0; c < MC; ++c) acc[i][c] = 0.0;
            for (int o = 0; o < G::NO; ++o) {
                const int nb = unbr[(int64_t)q * G::NO + o];
                if (nb < 0) continue;
                const bool nb_own = (umask[nb] >> l) & 1;    // inputs at DOFs a cell does not own are ignored
                double kt[DIM][DIM];
                if (MODE == 2) {
#pragma unroll
                    for (int i = 0; i < DIM; ++i)
#pragma unroll
                        for (int j = 0; j < DIM; ++j)
                            kt[i][j] = K[((int64_t)q * E + (o * DIM + i) * DIM + j) * LAT_WAVE + l];
                } else {
                    const int arow = MODE == 0 ? a : offset_node(a, o, A.nn, DIM);
                    const int orow = MODE == 0 ? o : G::NO - 1 - o;
#pragma unroll
                    for (int i = 0; i < DIM; ++i)
#pragma unroll
                        for (int j = 0; j < DIM; ++j) {
                            // MODE 1 reads the transposed block K[(a+o, j), (a, i)]
                            const int ent = MODE == 0 ? (orow * DIM + i) * DIM + j : (orow * DIM + j) * DIM + i;
                            const double *kp = K + ((int64_t)arow * E + ent) * cap;
                            double s = 0.0;
#pragma unroll
                            for (int k = 0; k < NR; ++k) s = fma(alpha[k], kp[k], s);
                            kt[i][j] = s;
                        }
                }
#pragma unroll
                for (int j = 0; j < DIM; ++j)
#pragma unroll
                    for (int c = 0; c < MC; ++c) {
                        const double x = nb_own ? X[(((int64_t)nb * DIM + j) * m + c0 + c) * LAT_WAVE + l] : 0.0;
#pragma unroll
                        for (int i = 0; i < DIM; ++i) acc[i][c] = fma(kt[i][j], x, acc[i][c]);
                    }
            }
            const bool own = (msk >> l) & 1;
#pragma unroll
            for (int i = 0; i < DIM; ++i)
#pragma unroll
                for (int c = 0; c < MC; ++c)
                    Y[(((int64_t)q * DIM + i) * m + c0 + c) * LAT_WAVE + l] = own ? acc[i][c] : 0.0;
        }
    }
}

// 2D row walk, software pipelined.  One workgroup = one group of 64 cells (lanes) and one node
// row y; its NW = 8 waves split the right-hand sides (wave w owns MW = m / 8 of them) and walk
// x = 0..n in step.  Per step (node x):
//   - the node's combined stencil Ktilde[e][cell] = sum_k K_k[e] alpha[k][cell] (36 entries x 64
//     cells, a dense contraction over the principal cells) is formed on the matrix cores with
//     v_mfma_f64_16x16x4 from the principal block staged in LDS one step earlier; the 12 tiles of
//     16 entries x 16 cells go to the 8 waves (cell tile w & 3; entry tiles {0, 2} or {1},
//     alternating with the node's parity so every wave does 3 tiles per 2 nodes).  For the plain
//     apply each wave copies its share of the cell's own stencil instead.  Result -> LDS;
//   - it stages the next node's principal block and issues the loads of X column x+2 into a
//     4-slot register window (columns x-1 .. x+2 of rows y-1, y, y+1);
//   - one barrier; then each wave applies the node's 2x2 blocks to its right-hand sides.
// Every X entry is fetched once per row walk and all loads are issued a step ahead of use.
template <int MW, int NR, int MODE, int LP, bool IDLE = false>
__global__ __launch_bounds__(512) void k_apply2d_rw(ApplyArgs A, const int32_t *__restrict__ goff,
                                                    const int32_t *__restrict__ uidx,
                                                    const uint64_t *__restrict__ umask, const double *__restrict__ K,
                                                    const double *__restrict__ alpha_il, const double *__restrict__ X,
                                                    double *__restrict__ Y)
{
    constexpr int E = 36, NW = 8;
    constexpr bool BFS = LP >= 1 && LP <= 3;            // bf16 slice products (LP levels)
    constexpr bool F32M = LP == 4;                       // FP32 operands on the FP32 matrix cores
    constexpr int NLV = BFS ? LP : 1;
    constexpr int KB = MODE == 2 ? 1 : E * NR;          // principal block of one node (doubles)
    constexpr int KPT = (KB + NW * 64 - 1) / (NW * 64);  // staged per thread
    __shared__ double kt_s[2][E][64];
    constexpr int KSTR = NR + 1;                        // row stride of a staged block (doubles)
    __shared__ double kb_s[2][MODE == 2 || BFS ? 1 : E * KSTR];
    // BFS: the staged block as bf16 slices [buf][slice][48 rows][KSR], sliced once per node
    constexpr int KSR = 32 * (NR <= 32 ? 1 : NR / 32) + 8;
    __shared__ __align__(16) uint16_t ks_s[2][NLV][BFS ? 48 * KSR : 1];
    // reduced precision: the combination of one node per workgroup (the segment's middle node) is
    // formed again in FP64 from an FP64 copy of its block, and the squared differences are summed
    constexpr bool SAMPLE = LP >= 1;
    __shared__ double kb64[SAMPLE ? E * KSTR : 1];
    __shared__ double kts[SAMPLE ? E * 64 : 1];          // the sampled node's reduced-precision stencils
    __shared__ double red[16];
    if (A.gate && *A.gate == 0) return;                  // a refinement pass that is not needed
    const int nn = A.nn, nloc = nn * nn, m = A.m, cap = A.cap;
    const int lb = lat_xcd_block(blockIdx.x, gridDim.x);
    const int nseg = A.nseg;                             // each row is walked in nseg x-segments
    const int g = lb / (nn * nseg), y = (lb / nseg) % nn, seg = lb % nseg;
    const int xs0 = (seg * nn) / nseg, xs1 = ((seg + 1) * nn) / nseg;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int l = threadIdx.x & 63, tid = threadIdx.x;
    const int64_t p = (int64_t)g * LAT_WAVE + l;
    const int r0 = A.rb + w * MW;
    const bool act = !IDLE || w * MW < A.mc;             // IDLE (chunks < 8): the waves past it only form
    const int xsamp = SAMPLE && A.errp ? (xs0 + xs1) / 2 : -1;
    const int e0 = (w * E) / NW, e1 = ((w + 1) * E) / NW;   // this wave's share of the entries
    const int32_t *ui = uidx + (int64_t)g * nloc;
    const int gq = goff[g];
    // alpha as the B operand of v_mfma_f64_16x16x4: wave w combines for cells ct*16 .. ct*16+15
    // (ct = w & 3); lane l holds alpha[k = 4 s + l / 16][cell = ct*16 + l % 16] in aB[s]
    const int ct = w & 3;
    double aB[MODE == 2 || BFS ? 1 : NR / 4];
    if (MODE != 2 && !BFS) {
#pragma unroll
        for (int s = 0; s < NR / 4; ++s)
            aB[s] = alpha_il[(int64_t)(4 * s + (l >> 4)) * A.ld + (int64_t)g * LAT_WAVE + ct * 16 + (l & 15)];
    }
    // BFS: the coefficients as bf16 slices, B operand of v_mfma_f32_16x16x32_bf16: lane l holds
    // c[k = 32 kb + 8 (l / 16) .. + 7][cell = ct*16 + l % 16] in cB[slice][kb]
    constexpr int NKB = NR <= 32 ? 1 : NR / 32;
    lat_bf16x8 cB[NLV][NKB];
    if (BFS) {
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb) {
            lat_s16x8 sl[NLV];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int k = 32 * kb + 8 * (l >> 4) + t;
                const double c = k < NR ? alpha_il[(int64_t)k * A.ld + (int64_t)g * LAT_WAVE + ct * 16 + (l & 15)] : 0.0;
                uint16_t b3[3];
                lat_slice3(c, b3);
#pragma unroll
                for (int v = 0; v < NLV; ++v) sl[v][t] = (short)b3[v];
            }
#pragma unroll
            for (int v = 0; v < NLV; ++v) cB[v][kb] = __builtin_bit_cast(lat_bf16x8, sl[v]);
        }
    }
    // principal-block staging (ROM modes): block[e * NR + k] = K_k[row(e)][ent(e)]
    double kpre[KPT];
    auto fetch_block = [&](int x) {
        if (MODE == 2) return;
        const bool inx = x < nn;
#pragma unroll
        for (int t = 0; t < KPT; ++t) {
            const int idx = tid + t * NW * 64;
            double v = 0.0;
            if (inx && idx < KB) {
                const int e = idx / NR, k = idx % NR;
                const int o = e >> 2, i = (e >> 1) & 1, j = e & 1;
                int arow = x + nn * y, ent = e;
                bool valid = true;
                if (MODE == 1) {       // transposed block K[(a+o, j), (a, i)]
                    const int xb = x + (o % 3) - 1, yb = y + (o / 3) - 1;
                    valid = xb >= 0 && xb < nn && yb >= 0 && yb < nn;
                    arow = valid ? xb + nn * yb : 0;
                    ent = ((8 - o) * 2 + j) * 2 + i;
                }
                if (valid) v = K[((int64_t)arow * E + ent) * cap + k];
            }
            kpre[t] = v;
        }
    };
    auto store_block = [&](int buf, int xnode) {
        if (MODE == 2) return;
#pragma unroll
        for (int t = 0; t < KPT; ++t) {
            const int idx = tid + t * NW * 64;
            if (idx < KB) {
                if (SAMPLE && xnode == xsamp) kb64[(idx / NR) * KSTR + idx % NR] = kpre[t];
                if (BFS) {
                    uint16_t b3[3];
                    lat_slice3(kpre[t], b3);
#pragma unroll
                    for (int v = 0; v < NLV; ++v) ks_s[buf][v][(idx / NR) * KSR + idx % NR] = b3[v];
                } else {
                    kb_s[buf][(idx / NR) * KSTR + idx % NR] = kpre[t];
                }
            }
        }
    };
    // plain mode: this wave's share of the cell's own stencil, one step ahead
    double ppre[(E + NW - 1) / NW];
    auto fetch_plain = [&](int x) {
        if (MODE != 2) return;
        int qi = -1;
        if (x < nn) qi = ui[x + nn * y];
        const int64_t q = qi >= 0 ? gq + qi : 0;
#pragma unroll
        for (int t = 0; t < (E + NW - 1) / NW; ++t) {
            const int e = e0 + t;
            const double v = (e < e1) ? K[(q * E + (e < E ? e : 0)) * LAT_WAVE + l] : 0.0;
            ppre[t] = qi >= 0 ? v : 0.0;
        }
    };
    double xw[4][3][2][MW];            // [slot][row y-1..y+1][dof][rhs]; column c lives in slot (c+1) % 4
    auto load_col = [&](double (&col)[3][2][MW], int xc) {
        if (!act) return;
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            const int yy = y + dy - 1;
            int qi = -1;
            if (xc >= 0 && xc < nn && yy >= 0 && yy < nn) qi = ui[xc + nn * yy];
            const int64_t q = qi >= 0 ? gq + qi : 0;        // always a valid packed node index
            const bool own = qi >= 0 && ((umask[q] >> l) & 1);
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int c = 0; c < MW; ++c) {
                    const double v = X[((q * 2 + j) * m + r0 + c) * LAT_WAVE + l];
                    col[dy][j][c] = own ? v : 0.0;
                }
        }
    };
    auto step = [&](int x, int sp, int sc, int sn, int sf) {
        const int a = x + nn * y;
        const int qi = ui[a];
        const int buf = x & 1;
        // (1) this wave's entries of the node's blocks -> LDS
        if (qi >= 0) {
            if (MODE == 2) {
#pragma unroll
                for (int t = 0; t < (E + NW - 1) / NW; ++t)
                    if (e0 + t < e1) kt_s[buf][e0 + t][l] = ppre[t];
            } else {
                // Ktilde[e][cell] = sum_k K[e][k] alpha[k][cell] as 16 x 16 tiles (entries x cells):
                // 3 entry tiles (the last holds entries 32..35) x 4 cell tiles; wave w takes cell tile
                // w & 3 and, alternating with the node's parity, entry tiles {0, 2} or {1}
                const bool heavy = (w < 4) == ((x & 1) == 0);
                const double *kb = &kb_s[buf][0];
                const int c16 = ct * 16 + (l & 15);
                if (BFS) {
                    // bf16 slices: A operand lane l = entry 16 et + l % 16, k = 32 kb + 8 (l / 16) .. + 7;
                    // slice products grouped by level p + q, FP32 accumulation per level, levels
                    // summed in FP64; output rows 4 (l / 16) + r, column = cell
                    auto tile = [&](int et) __attribute__((always_inline)) {
                        lat_f32x4 acc[NLV];
#pragma unroll
                        for (int v = 0; v < NLV; ++v) acc[v] = lat_f32x4{0.f, 0.f, 0.f, 0.f};
                        const int er = 16 * et + (l & 15);        // rows 36..47 feed unused outputs
#pragma unroll
                        for (int kbi = 0; kbi < NKB; ++kbi) {
                            const int k0 = 32 * kbi + 8 * (l >> 4);
                            lat_bf16x8 ap[NLV];
#pragma unroll
                            for (int v = 0; v < NLV; ++v) {
                                lat_s16x8 z = {0, 0, 0, 0, 0, 0, 0, 0};
                                if (k0 < NR) z = *reinterpret_cast<const lat_s16x8 *>(&ks_s[buf][v][er * KSR + k0]);
                                ap[v] = __builtin_bit_cast(lat_bf16x8, z);
                            }
#pragma unroll
                            for (int lev = 0; lev < NLV; ++lev)
#pragma unroll
                                for (int pc = 0; pc <= lev; ++pc)
                                    acc[lev] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[lev - pc], cB[pc][kbi], acc[lev], 0, 0, 0);
                        }
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int e = 16 * et + 4 * (l >> 4) + r;
                            double v = 0.0;
#pragma unroll
                            for (int lev = NLV - 1; lev >= 0; --lev) v += (double)acc[lev][r];
                            if (e < E) {
                                kt_s[buf][e][c16] = v;
                                if (x == xsamp) kts[e * 64 + c16] = v;
                            }
                        }
                    };
                    if (heavy) {
                        tile(0);
                        tile(2);
                    } else {
                        tile(1);
                    }
                } else if (F32M) {
                    // FP32 operands (rounded from the staged FP64 block and alpha) on
                    // v_mfma_f32_16x16x4f32: output rows 4 (l / 16) + r of the tile
                    auto tile32 = [&](int et) __attribute__((always_inline)) {
                        lat_f32x4 c = {0.f, 0.f, 0.f, 0.f};
                        const int er = 16 * et + (l & 15) < E ? 16 * et + (l & 15) : E - 1;
                        const double *rp = kb + er * KSTR + (l >> 4);
#pragma unroll
                        for (int s2 = 0; s2 < NR / 4; ++s2)
                            c = __builtin_amdgcn_mfma_f32_16x16x4f32((float)rp[4 * s2], (float)aB[s2], c, 0, 0, 0);
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int e = 16 * et + 4 * (l >> 4) + r;
                            if (e < E) {
                                kt_s[buf][e][c16] = (double)c[r];
                                if (x == xsamp) kts[e * 64 + c16] = (double)c[r];
                            }
                        }
                    };
                    if (heavy) {
                        tile32(0);
                        tile32(2);
                    } else {
                        tile32(1);
                    }
                } else if (heavy) {
                    v4d c0 = {0.0, 0.0, 0.0, 0.0}, c2 = {0.0, 0.0, 0.0, 0.0};
                    const double *r0p = kb + (l & 15) * KSTR + (l >> 4);
                    const int e2 = 32 + (l & 15) < E ? 32 + (l & 15) : E - 1;
                    const double *r2p = kb + e2 * KSTR + (l >> 4);
#pragma unroll
                    for (int s2 = 0; s2 < NR / 4; ++s2) {
                        c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(r0p[4 * s2], aB[s2], c0, 0, 0, 0);
                        c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(r2p[4 * s2], aB[s2], c2, 0, 0, 0);
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        kt_s[buf][(l >> 4) + 4 * r][c16] = c0[r];
                        if ((l >> 4) + 4 * r < E - 32) kt_s[buf][32 + (l >> 4) + 4 * r][c16] = c2[r];
                    }
                } else {
                    v4d c1 = {0.0, 0.0, 0.0, 0.0};
                    const double *r1p = kb + (16 + (l & 15)) * KSTR + (l >> 4);
#pragma unroll
                    for (int s2 = 0; s2 < NR / 4; ++s2)
                        c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(r1p[4 * s2], aB[s2], c1, 0, 0, 0);
#pragma unroll
                    for (int r = 0; r < 4; ++r) kt_s[buf][16 + (l >> 4) + 4 * r][c16] = c1[r];
                }
            }
        }
        // (2) stage the next node's block, prefetch the one after, and the next X column
        store_block(buf ^ 1, x + 1);
        fetch_block(x + 2);
        fetch_plain(x + 1);
        load_col(xw[sf], x + 2);
        __syncthreads();
        // (3) apply
        if (qi >= 0 && act) {
            double acc[2][MW];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int c = 0; c < MW; ++c) acc[i][c] = 0.0;
#pragma unroll
            for (int o = 0; o < 9; ++o) {
                const int dx = o % 3, dy = o / 3;
                const double (&col)[3][2][MW] = dx == 0 ? xw[sp] : (dx == 1 ? xw[sc] : xw[sn]);
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        const double kt = kt_s[buf][(o * 2 + i) * 2 + j][l];
#pragma unroll
                        for (int c = 0; c < MW; ++c) acc[i][c] = fma(kt, col[dy][j][c], acc[i][c]);
                    }
            }
            const int64_t q = gq + qi;
            const bool own = (umask[q] >> l) & 1;
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int c = 0; c < MW; ++c) Y[((q * 2 + i) * m + r0 + c) * LAT_WAVE + l] = own ? acc[i][c] : 0.0;
        }
    };
    // prologue: window columns x0-1, x0, x0+1; block of node x0 staged, x0+1 in flight; plain entries of x0
    // (slot of column c is (c - x0 + 1) % 4 within the segment; the LDS parity follows x)
    load_col(xw[0], xs0 - 1);
    load_col(xw[1], xs0);
    load_col(xw[2], xs0 + 1);
    fetch_block(xs0);
    store_block(xs0 & 1, xs0);
    fetch_block(xs0 + 1);
    fetch_plain(xs0);
    __syncthreads();
    int x = xs0;
    for (; x + 3 < xs1; x += 4) {
        step(x, 0, 1, 2, 3);
        step(x + 1, 1, 2, 3, 0);
        step(x + 2, 2, 3, 0, 1);
        step(x + 3, 3, 0, 1, 2);
    }
    if (x < xs1) step(x, 0, 1, 2, 3);
    if (x + 1 < xs1) step(x + 1, 1, 2, 3, 0);
    if (x + 2 < xs1) step(x + 2, 2, 3, 0, 1);
    if (SAMPLE && A.errp) {
        // the sampled node once more in FP64 (v_mfma_f64_16x16x4, output rows l / 16 + 4 r): each wave
        // its formation tiles of that node, against the reduced-precision values kept in kts
        __syncthreads();
        double d2 = 0.0, r2 = 0.0;
        if (ui[xsamp + nn * y] >= 0) {
            const bool heavy = (w < 4) == ((xsamp & 1) == 0);
            const int c16 = ct * 16 + (l & 15);
            auto ref_tile = [&](int et) {
                v4d c = {0.0, 0.0, 0.0, 0.0};
                const int er = 16 * et + (l & 15) < E ? 16 * et + (l & 15) : E - 1;
                const double *rp = kb64 + er * KSTR + (l >> 4);
                for (int s2 = 0; s2 < NR / 4; ++s2) {
                    const double a64 = alpha_il[(int64_t)(4 * s2 + (l >> 4)) * A.ld + (int64_t)g * LAT_WAVE + c16];
                    c = __builtin_amdgcn_mfma_f64_16x16x4f64(rp[4 * s2], a64, c, 0, 0, 0);
                }
                for (int r = 0; r < 4; ++r) {
                    const int e = 16 * et + (l >> 4) + 4 * r;
                    if (e < E) {
                        const double dv = kts[e * 64 + c16] - c[r];
                        d2 = fma(dv, dv, d2);
                        r2 = fma(c[r], c[r], r2);
                    }
                }
            };
            if (heavy) {
                ref_tile(0);
                ref_tile(2);
            } else {
                ref_tile(1);
            }
        }
        block_sum2_512(d2, r2, red, A.errp + 2 * (int64_t)blockIdx.x);
    }
}

// 3D ROM apply (and its transpose), formation on the matrix cores.  One workgroup of 8 waves =
// a run of APPLY3_RUN packed nodes (their group's 64 cells are the lanes).  A node's 27 stencil
// offsets are taken in 9 slices of 3 (27 entries, two 16-row tiles); per slice step:
//   - each wave issues the loads of the X values its right-hand sides need for the NEXT slice's
//     three neighbour nodes (consumed one step later, so they overlap a whole step);
//   - formation: Ktilde[e][cell] = sum_k K_k[e] alpha[k][cell] with v_mfma_f64_16x16x4 (A operand =
//     the principal block slice, staged in LDS; B operand = alpha, in registers); wave w forms
//     entry tile w / 4 of cell tile w % 4 and writes it to LDS;
//   - the next slice's principal block (fetched with coalesced loads one step earlier) goes to
//     LDS and the one after is fetched;
//   - one barrier; apply: wave w accumulates Ktilde[(o,i,j)] X[a+o, j] for right-hand sides
//     2w, 2w+1 (X masked to owned neighbour DOFs).
// Both LDS buffers are double-buffered (33 KB each for 64 principal cells), so one barrier per
// step suffices and two workgroups fit on a CU.
// Node order: each XCD takes one contiguous eighth of the runs, in bands of APPLY3_BAND workgroups
// (what one XCD holds at once); a band covers the packed nodes of its runs and its workgroup j
// takes nodes j, j + nb, j + 2 nb, ... of them (nb = workgroups in the band), so the nodes in
// flight on an XCD at any moment are one compact stretch whose shared neighbour X blocks meet in
// its L2.
constexpr int APPLY3_RUN = 16;
constexpr int APPLY3_BAND = 32;

template <int NR, int MODE, int LP>
__global__ __launch_bounds__(512) void k_apply3d_mfma(
    ApplyArgs A, const int32_t *__restrict__ goff, const int32_t *__restrict__ unode,
    const int32_t *__restrict__ unbr, const uint64_t *__restrict__ umask, const double *__restrict__ K,
    const double *__restrict__ alpha_il, const double *__restrict__ X, double *__restrict__ Y, int npacked,
    const int32_t *__restrict__ qgroup)
{
    constexpr int E = 243, NO = 27, ES = 27, ER = 32, KR = NR + 1, TR = 65, NSL = 9;
    constexpr bool BFS = LP >= 1 && LP <= 3;            // bf16 slice products (LP levels)
    constexpr bool F32M = LP == 4;                       // FP32 operands on the FP32 matrix cores
    constexpr int NLV = BFS ? LP : 1;
    constexpr int SPT = (ER * NR + 511) / 512;           // staged values per thread and slice
    __shared__ double kb_s[2][BFS ? 1 : ER * KR];
    __shared__ double kt_s[2][ER * TR];
    // BFS: the staged slice as bf16 slices [buf][slice][ER rows][KSR]
    constexpr int KSR = 32 * (NR <= 32 ? 1 : NR / 32) + 8;
    __shared__ __align__(16) uint16_t ks_s[2][NLV][BFS ? ER * KSR : 1];
    // reduced precision: one slice per workgroup (the run's middle slice) is formed again in FP64
    constexpr bool SAMPLE = LP >= 1;
    __shared__ double kb64[SAMPLE ? ER * KR : 1];
    __shared__ double kts[SAMPLE ? ER * 64 : 1];         // the sampled slice's reduced-precision stencils
    __shared__ double red[16];
    if (A.gate && *A.gate == 0) return;                  // a refinement pass that is not needed
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int l = threadIdx.x & 63, tid = threadIdx.x;
    // XCD x (blocks b with b % 8 == x) owns the runs [rx0, rx0 + nrx); its s-th block is in band
    // s / APPLY3_BAND of them
    const int ng = (int)gridDim.x, x8 = (int)blockIdx.x & 7, s8 = (int)blockIdx.x >> 3;
    const int rx0 = x8 * (ng >> 3) + min(x8, ng & 7), nrx = (ng >> 3) + (x8 < (ng & 7) ? 1 : 0);
    const int bnd = s8 / APPLY3_BAND;
    const int qs = min(APPLY3_BAND, nrx - bnd * APPLY3_BAND);              // node stride
    const int qb = (rx0 + bnd * APPLY3_BAND) * APPLY3_RUN + s8 % APPLY3_BAND; // first node of this workgroup
    if (qb >= npacked) return;
    const int cnt = min(APPLY3_RUN, (npacked - qb + qs - 1) / qs);       // nodes qb + qs t, t < cnt
    const int nn = A.nn, m = A.m, cap = A.cap;
    const int ct = w & 3, et = w >> 2;                   // formation tile of this wave
    const int r0 = A.rb + 2 * w;                         // this wave's right-hand sides (apply)
    const int nrw = max(0, min(2, A.mc - 2 * w));
    const int nsl = cnt * NSL;
    const int ssamp = SAMPLE && A.errp ? nsl / 2 : -1;
    // ---- principal block slice sl (node t = sl / 9, offsets 3 (sl % 9) ..): coalesced fetch
    double kpre[SPT];
    bool kval[SPT];
    auto fetch = [&](int sl) __attribute__((always_inline)) {
        const bool live = sl < nsl;
        const int a = live ? unode[qb + qs * (sl / NSL)] : 0;
        const int h = sl % NSL;
#pragma unroll
        for (int t = 0; t < SPT; ++t) {
            const int idx = tid + 512 * t < ER * NR ? tid + 512 * t : 0;
            const int el = idx / NR, k = idx % NR;
            const int e = ES * h + (el < ES ? el : ES - 1);
            bool valid = live && el < ES;
            int arow = a, ent = e;
            if (MODE == 1) {             // transposed block K[(a+o, j), (a, i)]
                const int o = e / 9, i = (e / 3) % 3, j = e % 3;
                const int xn = a % nn + o % 3 - 1, yn = (a / nn) % nn + (o / 3) % 3 - 1, zn = a / (nn * nn) + o / 9 - 1;
                const bool in = xn >= 0 && xn < nn && yn >= 0 && yn < nn && zn >= 0 && zn < nn;
                valid = valid && in;
                arow = in ? xn + nn * (yn + nn * zn) : 0;
                ent = ((NO - 1 - o) * 3 + j) * 3 + i;
            }
            kpre[t] = K[((int64_t)arow * E + ent) * cap + k];
            kval[t] = valid;
        }
    };
    auto store = [&](int buf, int sl) __attribute__((always_inline)) {
#pragma unroll
        for (int t = 0; t < SPT; ++t) {
            const int idx = tid + 512 * t;
            if (idx < ER * NR) {
                const double v = kval[t] ? kpre[t] : 0.0;
                if (SAMPLE && sl == ssamp) kb64[(idx / NR) * KR + idx % NR] = v;
                if (BFS) {
                    uint16_t b3[3];
                    lat_slice3(v, b3);
#pragma unroll
                    for (int lv = 0; lv < NLV; ++lv) ks_s[buf][lv][(idx / NR) * KSR + idx % NR] = b3[lv];
                } else {
                    kb_s[buf][(idx / NR) * KR + idx % NR] = v;
                }
            }
        }
    };
    // neighbour table of the workgroup's node t, one offset per lane: packed index and owner mask
    auto nbr_load = [&](int t, int &nbv, uint32_t &mlo, uint32_t &mhi) __attribute__((always_inline)) {
        nbv = (t < cnt && l < NO) ? unbr[(int64_t)(qb + qs * t) * NO + l] : -1;
        const uint64_t mk = nbv >= 0 ? umask[nbv] : 0ull;
        mlo = (uint32_t)mk;
        mhi = (uint32_t)(mk >> 32);
    };
    int gcur = -1;
    double aB[BFS ? 1 : NR / 4];
    constexpr int NKB = NR <= 32 ? 1 : NR / 32;
    lat_bf16x8 cB[NLV][NKB];
    int nbv, nbv_n;
    uint32_t mlo, mhi, mlo_n, mhi_n;
    nbr_load(0, nbv, mlo, mhi);
    // X of a slice's three neighbour nodes for this wave's right-hand sides (raw), issued one
    // slice step before it is used
    double xn[3][3][2];
    int nbn[3];
    bool ownn[3];
    auto load_x = [&](int tab, uint32_t tlo, uint32_t thi, int h) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            const int o = 3 * h + u;
            const int nb = __builtin_amdgcn_readlane(tab, o);
            const uint32_t lo = __builtin_amdgcn_readlane(tlo, o), hi = __builtin_amdgcn_readlane(thi, o);
            nbn[u] = nb;
            ownn[u] = ((l < 32 ? lo >> l : hi >> (l - 32)) & 1u) != 0;
            const int64_t nq = nb >= 0 ? nb : 0;
#pragma unroll
            for (int j = 0; j < 3; ++j)
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const int rr = r < nrw ? r0 + r : 0;
                    xn[u][j][r] = X[((nq * 3 + j) * m + rr) * LAT_WAVE + l];
                }
        }
    };
    load_x(nbv, mlo, mhi, 0);
    fetch(0);
    store(0, 0);
    fetch(1);
    __syncthreads();
    for (int q = qb; q < qb + qs * cnt; q += qs) {
        const int t = (q - qb) / qs;
        const int g = qgroup[q];
        if (g != gcur) {                                 // alpha of this group as the B operand
            gcur = g;
            if (!BFS) {
#pragma unroll
                for (int s2 = 0; s2 < NR / 4; ++s2)
                    aB[s2] = alpha_il[(int64_t)(4 * s2 + (l >> 4)) * A.ld + (int64_t)g * LAT_WAVE + ct * 16 + (l & 15)];
            } else {
                // bf16 slices of the coefficients: lane l holds c[k = 32 kb + 8 (l / 16) ..][cell]
#pragma unroll
                for (int kb = 0; kb < NKB; ++kb) {
                    lat_s16x8 sl[NLV];
#pragma unroll
                    for (int t = 0; t < 8; ++t) {
                        const int k = 32 * kb + 8 * (l >> 4) + t;
                        const double c = k < NR ? alpha_il[(int64_t)k * A.ld + (int64_t)g * LAT_WAVE + ct * 16 + (l & 15)] : 0.0;
                        uint16_t b3[3];
                        lat_slice3(c, b3);
#pragma unroll
                        for (int v = 0; v < NLV; ++v) sl[v][t] = (short)b3[v];
                    }
#pragma unroll
                    for (int v = 0; v < NLV; ++v) cB[v][kb] = __builtin_bit_cast(lat_bf16x8, sl[v]);
                }
            }
        }
        nbr_load(t + 1, nbv_n, mlo_n, mhi_n);            // next node's table, used one node later
        double acc[3][2];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int r = 0; r < 2; ++r) acc[i][r] = 0.0;
        const int sl0 = t * NSL;
#pragma unroll
        for (int h = 0; h < NSL; ++h) {
            const int buf = (sl0 + h) & 1;
            // (0) this slice's X (loaded a step ago); issue the next slice's (next node's first
            // slice after the last one: its table was loaded at the start of this node)
            double xv[3][3][2];
            int nbs[3];
            bool ownb[3];
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                nbs[u] = nbn[u];
                ownb[u] = ownn[u];
#pragma unroll
                for (int j = 0; j < 3; ++j)
#pragma unroll
                    for (int r = 0; r < 2; ++r) xv[u][j][r] = xn[u][j][r];
            }
            if (h + 1 < NSL) load_x(nbv, mlo, mhi, h + 1);
            else load_x(nbv_n, mlo_n, mhi_n, 0);
            // (1) formation of entry tile et of this slice for cell tile ct -> kt_s[buf]
            if (F32M) {
                lat_f32x4 c = {0.f, 0.f, 0.f, 0.f};
                const double *pa = &kb_s[buf][(16 * et + (l & 15)) * KR + (l >> 4)];
#pragma unroll
                for (int s2 = 0; s2 < NR / 4; ++s2)
                    c = __builtin_amdgcn_mfma_f32_16x16x4f32((float)pa[4 * s2], (float)aB[s2], c, 0, 0, 0);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    kt_s[buf][(16 * et + 4 * (l >> 4) + r) * TR + ct * 16 + (l & 15)] = (double)c[r];
                    if (sl0 + h == ssamp) kts[(16 * et + 4 * (l >> 4) + r) * 64 + ct * 16 + (l & 15)] = (double)c[r];
                }
            } else if (!BFS) {
                v4d c = {0.0, 0.0, 0.0, 0.0};
                const double *pa = &kb_s[buf][(16 * et + (l & 15)) * KR + (l >> 4)];
#pragma unroll
                for (int s2 = 0; s2 < NR / 4; ++s2) c = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[4 * s2], aB[s2], c, 0, 0, 0);
#pragma unroll
                for (int r = 0; r < 4; ++r) kt_s[buf][(16 * et + (l >> 4) + 4 * r) * TR + ct * 16 + (l & 15)] = c[r];
            } else {
                // bf16 slice products by level p + q, FP32 accumulation, FP64 level sums; output
                // rows 4 (l / 16) + r of the tile
                lat_f32x4 acc32[NLV];
#pragma unroll
                for (int v = 0; v < NLV; ++v) acc32[v] = lat_f32x4{0.f, 0.f, 0.f, 0.f};
                const int er = 16 * et + (l & 15);
#pragma unroll
                for (int kbi = 0; kbi < NKB; ++kbi) {
                    const int k0 = 32 * kbi + 8 * (l >> 4);
                    lat_bf16x8 ap[NLV];
#pragma unroll
                    for (int v = 0; v < NLV; ++v) {
                        lat_s16x8 z = {0, 0, 0, 0, 0, 0, 0, 0};
                        if (k0 < NR) z = *reinterpret_cast<const lat_s16x8 *>(&ks_s[buf][v][er * KSR + k0]);
                        ap[v] = __builtin_bit_cast(lat_bf16x8, z);
                    }
#pragma unroll
                    for (int lev = 0; lev < NLV; ++lev)
#pragma unroll
                        for (int pc = 0; pc <= lev; ++pc)
                            acc32[lev] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[lev - pc], cB[pc][kbi], acc32[lev], 0, 0, 0);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    double v = 0.0;
#pragma unroll
                    for (int lev = NLV - 1; lev >= 0; --lev) v += (double)acc32[lev][r];
                    kt_s[buf][(16 * et + 4 * (l >> 4) + r) * TR + ct * 16 + (l & 15)] = v;
                    if (sl0 + h == ssamp) kts[(16 * et + 4 * (l >> 4) + r) * 64 + ct * 16 + (l & 15)] = v;
                }
            }
            // (2) stage the next slice, fetch the one after
            store(buf ^ 1, sl0 + h + 1);
            fetch(sl0 + h + 2);
            __syncthreads();
            // (3) apply the slice's 27 entries
            if (nrw > 0) {
#pragma unroll
                for (int u = 0; u < 3; ++u) {
                    if (nbs[u] < 0) continue;
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int j = 0; j < 3; ++j) {
                            const double kt = kt_s[buf][((u * 3 + i) * 3 + j) * TR + l];
#pragma unroll
                            for (int r = 0; r < 2; ++r) acc[i][r] = fma(kt, ownb[u] ? xv[u][j][r] : 0.0, acc[i][r]);
                        }
                }
            }
        }
        const bool own = (umask[q] >> l) & 1;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int r = 0; r < 2; ++r)
                if (r < nrw) Y[(((int64_t)q * 3 + i) * m + r0 + r) * LAT_WAVE + l] = own ? acc[i][r] : 0.0;
        nbv = nbv_n; mlo = mlo_n; mhi = mhi_n;
    }
    if (SAMPLE && A.errp) {
        // the sampled slice once more in FP64 (output rows l / 16 + 4 r): each wave its formation tile,
        // against the reduced-precision values kept in kts; rows past the slice's 27 entries are padding
        __syncthreads();
        const int gs = qgroup[qb + qs * (ssamp / NSL)];
        const int c16 = ct * 16 + (l & 15);
        v4d c = {0.0, 0.0, 0.0, 0.0};
        const double *pa = &kb64[(16 * et + (l & 15)) * KR + (l >> 4)];
        for (int s2 = 0; s2 < NR / 4; ++s2) {
            const double a64 = alpha_il[(int64_t)(4 * s2 + (l >> 4)) * A.ld + (int64_t)gs * LAT_WAVE + c16];
            c = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[4 * s2], a64, c, 0, 0, 0);
        }
        double d2 = 0.0, r2 = 0.0;
        for (int r = 0; r < 4; ++r) {
            const int e = 16 * et + (l >> 4) + 4 * r;
            if (e < ES) {
                const double dv = kts[e * 64 + c16] - c[r];
                d2 = fma(dv, dv, d2);
                r2 = fma(c[r], c[r], r2);
            }
        }
        block_sum2_512(d2, r2, red, A.errp + 2 * (int64_t)blockIdx.x);
    }
}

// Adjoint forms: partial sums over a run of nodes of G_ik = sum_{a,o,i,j} K_k[a,o,i,j] W_i[a,o,i,j],
// W_i[a,o,i,j] = sum_r Ybar_i[a,i,r] X_i[a+o,j,r].  Output [chunk][lane][cap].
constexpr int FORM_MC = 8;

template <int DIM, int NR>
__global__ __launch_bounds__(256) void k_forms(ApplyArgs A, const int32_t *__restrict__ goff,
                                               const int32_t *__restrict__ unode, const int32_t *__restrict__ unbr,
                                               const uint64_t *__restrict__ umask, const double *__restrict__ K,
                                               const double *__restrict__ X, const double *__restrict__ Ybar,
                                               double *__restrict__ part)
{
    using G = Geo<DIM>;
    constexpr int E = G::E;
    const int wave = __builtin_amdgcn_readfirstlane(lat_xcd_block(blockIdx.x, gridDim.x) * 4 + (int)(threadIdx.x >> 6));
    const int l = threadIdx.x & 63;
    const int g = wave / A.chunks_per_group, ch = wave % A.chunks_per_group;
    if (g >= (int)(A.ld / LAT_WAVE)) return;
    const int q0 = goff[g] + ch * A.nch;
    const int q1 = min(goff[g + 1], q0 + A.nch);
    const int64_t p = (int64_t)g * LAT_WAVE + l;
    const int m = A.m;
    const int cap = A.cap;
    double gk[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) gk[k] = 0.0;
    for (int q = q0; q < q1; ++q) {
        const int a = unode[q];
        if (!((umask[q] >> l) & 1)) continue;          // Ybar only counts at owned DOFs
        for (int r0 = 0; r0 < m; r0 += FORM_MC) {
            const int mc = min(FORM_MC, m - r0);
            double yb[DIM][FORM_MC];
#pragma unroll
            for (int i = 0; i < DIM; ++i)
#pragma unroll
                for (int r = 0; r < FORM_MC; ++r)
                    yb[i][r] = r < mc ? Ybar[(((int64_t)q * DIM + i) * m + r0 + r) * LAT_WAVE + l] : 0.0;
            for (int o = 0; o < G::NO; ++o) {
                const int nb = unbr[(int64_t)q * G::NO + o];
                if (nb < 0 || !((umask[nb] >> l) & 1)) continue;
                double xv[DIM][FORM_MC];
#pragma unroll
                for (int j = 0; j < DIM; ++j)
#pragma unroll
                    for (int r = 0; r < FORM_MC; ++r)
                        xv[j][r] = r < mc ? X[(((int64_t)nb * DIM + j) * m + r0 + r) * LAT_WAVE + l] : 0.0;
#pragma unroll
                for (int i = 0; i < DIM; ++i)
#pragma unroll
                    for (int j = 0; j < DIM; ++j) {
                        double w = 0.0;
#pragma unroll
                        for (int r = 0; r < FORM_MC; ++r) w = fma(yb[i][r], xv[j][r], w);
                        const double *kp = K + ((int64_t)a * E + (o * DIM + i) * DIM + j) * cap;
#pragma unroll
                        for (int k = 0; k < NR; ++k) gk[k] = fma(w, kp[k], gk[k]);
                    }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) part[((int64_t)ch * A.ld + p) * cap + k] = gk[k];
    for (int k = NR; k < cap; ++k) part[((int64_t)ch * A.ld + p) * cap + k] = 0.0;
}

// Adjoint forms on the matrix cores: G^s_ik = <Ybar_i, K^s_k X_i> for up to three principal
// stacks s in one pass over X and Ybar.  G^s = sum over nodes a of K^s[a]^T W[a] with
// W[a][(o,i,j)][cell] = sum_r Ybar[cell][a,i,r] X[cell][a+o,j,r]: the second factor is per cell
// (VALU, lanes = cells), the contraction over the stencil entries is a dense
// (principals x entries) x (entries x cells) product shared by the group (v_mfma_f64_16x16x4).
// One workgroup of 8 waves = a run of FORMS_RUN packed nodes of one group.  A node's entries are
// taken in slices of 12 rows (2D: 3 offsets x 4 entries; 3D: 1 offset x 9 entries + 3 zero rows);
// per slice:
//   - wave w accumulates its right-hand sides (w, w + 8) into a partial W slice -> LDS, and the
//     slice's principal rows of every stack are staged in LDS;
//   - one barrier; each wave forms the B operand W = sum of the 8 partials (fixed order) for its
//     cell tile w % 4 and accumulates its output tiles (stack, principal tile, cell tile);
//   - one barrier.
// The run's partial G goes to part[stack][chunk][lane][cap]; chunks are summed by the fixed tree.
constexpr int FORMS_RUN = 32;

template <int DIM, int NR, int NS>
__global__ __launch_bounds__(512) void k_forms_mfma(ApplyArgs A, const int32_t *__restrict__ goff,
                                                    const int32_t *__restrict__ unode,
                                                    const int32_t *__restrict__ unbr,
                                                    const uint64_t *__restrict__ umask, const double *__restrict__ K0,
                                                    const double *__restrict__ K1, const double *__restrict__ K2,
                                                    const double *__restrict__ X, const double *__restrict__ Ybar,
                                                    double *__restrict__ part, int cpg)
{
    constexpr int NO = DIM == 2 ? 9 : 27, D2 = DIM * DIM, E = NO * D2;
    constexpr int OPS = DIM == 2 ? 3 : 1;                // offsets per slice
    constexpr int ES = OPS * D2;                         // entries per slice (12 / 9)
    constexpr int ER = 12;                               // slice rows: 3 k-steps of 4
    constexpr int NSL = NO / OPS;                        // slices per node (3 / 27)
    constexpr int KR = NR + 1;
    constexpr int NKT = NR / 16;                         // principal tiles
    constexpr int NT = NS * NKT * 4;                     // output tiles
    constexpr int TPW = (NT + 7) / 8;                    // output tiles per wave
    __shared__ double wp_s[8][ER * 64];
    __shared__ double kb_s[NS][ER * KR];
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int l = threadIdx.x & 63, tid = threadIdx.x;
    const int blk = lat_xcd_block(blockIdx.x, gridDim.x);
    const int g = blk / cpg, ch = blk % cpg;
    const int G = (int)(A.ld / LAT_WAVE);
    if (g >= G) return;
    const int q0 = goff[g] + ch * FORMS_RUN;
    const int q1 = min(goff[g + 1], q0 + FORMS_RUN);
    const int m = A.m, cap = A.cap, nn = A.nn;
    const int ct = w & 3;                                // this wave's cell tile (all its output tiles)
    (void)nn;
    v4d acc[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int q = q0; q < q1; ++q) {
        const int a = unode[q];
        const bool own = (umask[q] >> l) & 1;            // Ybar counts at owned DOFs only
        const int nbv = l < NO ? unbr[(int64_t)q * NO + l] : -1;
        const uint64_t mk = nbv >= 0 ? umask[nbv] : 0ull;
        const uint32_t mlo = (uint32_t)mk, mhi = (uint32_t)(mk >> 32);
        double yb[DIM][2];
#pragma unroll
        for (int i = 0; i < DIM; ++i)
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int rr = w + 8 * r;
                const double v = Ybar[(((int64_t)q * DIM + i) * m + (rr < m ? rr : 0)) * LAT_WAVE + l];
                yb[i][r] = (own && rr < m) ? v : 0.0;
            }
        for (int sl = 0; sl < NSL; ++sl) {
            // ---- partial W of this wave's right-hand sides -> wp_s[w]
#pragma unroll
            for (int u = 0; u < OPS; ++u) {
                const int o = sl * OPS + u;
                const int nb = __builtin_amdgcn_readlane(nbv, o);
                const uint32_t lo = __builtin_amdgcn_readlane(mlo, o), hi = __builtin_amdgcn_readlane(mhi, o);
                const bool nbo = nb >= 0 && ((((l < 32 ? lo >> l : hi >> (l - 32)) & 1u)) != 0);
                const int64_t nq = nb >= 0 ? nb : 0;
                double xv[DIM][2];
#pragma unroll
                for (int j = 0; j < DIM; ++j)
#pragma unroll
                    for (int r = 0; r < 2; ++r) {
                        const int rr = w + 8 * r;
                        const double v = X[((nq * DIM + j) * m + (rr < m ? rr : 0)) * LAT_WAVE + l];
                        xv[j][r] = (nbo && rr < m) ? v : 0.0;
                    }
#pragma unroll
                for (int i = 0; i < DIM; ++i)
#pragma unroll
                    for (int j = 0; j < DIM; ++j) {
                        double wv = 0.0;
#pragma unroll
                        for (int r = 0; r < 2; ++r) wv = fma(yb[i][r], xv[j][r], wv);
                        wp_s[w][((u * DIM + i) * DIM + j) * 64 + l] = wv;
                    }
            }
#pragma unroll
            for (int e = ES; e < ER; ++e) wp_s[w][e * 64 + l] = 0.0;
            // ---- the slice's principal rows of every stack -> kb_s (rows >= ES are zero)
            for (int idx = tid; idx < NS * ER * NR; idx += 512) {
                const int st = idx / (ER * NR), rem = idx % (ER * NR);
                const int el = rem / NR, k = rem % NR;
                const double *Ks = st == 0 ? K0 : (st == 1 ? K1 : K2);
                double v = 0.0;
                if (el < ES) v = Ks[((int64_t)a * E + sl * ES + el) * cap + k];
                kb_s[st][el * KR + k] = v;
            }
            __syncthreads();
            // ---- contraction: G^T[k][cell] += K^T[k][e] W[e][cell]
#pragma unroll
            for (int ks = 0; ks < ER / 4; ++ks) {
                const int row = ks * 4 + (l >> 4);
                double b = 0.0;
#pragma unroll
                for (int ww = 0; ww < 8; ++ww) b += wp_s[ww][row * 64 + ct * 16 + (l & 15)];
#pragma unroll
                for (int t = 0; t < TPW; ++t) {
                    const int j = w + 8 * t;
                    if (j < NT) {
                        const int st = j / (NKT * 4), kt = (j / 4) % NKT;
                        const double av = kb_s[st][row * KR + kt * 16 + (l & 15)];
                        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b, acc[t], 0, 0, 0);
                    }
                }
            }
            __syncthreads();
        }
    }
    // ---- this run's partial G: lane l, reg r -> principal kt*16 + l/16 + 4 r, cell ct*16 + l%16
    const int64_t ldc = A.ld * cap;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        const int j = w + 8 * t;
        if (j < NT) {
            const int st = j / (NKT * 4), kt = (j / 4) % NKT;
            const int64_t base = ((int64_t)(st * cpg + ch)) * ldc + ((int64_t)g * LAT_WAVE + ct * 16 + (l & 15)) * cap;
#pragma unroll
            for (int r = 0; r < 4; ++r) part[base + kt * 16 + (l >> 4) + 4 * r] = acc[t][r];
        }
    }
    if (cap > NR) {
        for (int idx = tid; idx < NS * 64 * (cap - NR); idx += 512) {
            const int st = idx / (64 * (cap - NR)), rem = idx % (64 * (cap - NR));
            const int cell = rem / (cap - NR), k = NR + rem % (cap - NR);
            part[((int64_t)(st * cpg + ch)) * ldc + ((int64_t)g * LAT_WAVE + cell) * cap + k] = 0.0;
        }
    }
}

// The adjoint forms' cell data W[(a, e)][p] = sum_r Ybar[a, i, r] X[a + o, j, r] (e = (o d + i) d + j)
// for every local node a and plan lane p, Ybar counted at the cell's owned DOFs and X at its owned
// neighbour DOFs, zero where the node is not in the lane's group union; then
// <Ybar_p, K_k X_p> = sum_(a, e) K_k[a][e] W[(a, e)][p] is one row contraction per stack.
// Lanes p0 .. p0 + ldw - 1 (a batch; W holds only these columns, row stride ldw).
template <int DIM, class WT>
__global__ __launch_bounds__(256) void k_forms_W(int64_t ld, int64_t p0, int64_t ldw, int nloc, int m,
                                                 const int32_t *__restrict__ goff, const int32_t *__restrict__ uidx,
                                                 const int32_t *__restrict__ unbr, const uint64_t *__restrict__ umask,
                                                 const double *__restrict__ X, const double *__restrict__ Ybar,
                                                 WT *__restrict__ W)
{
    constexpr int NO = DIM == 2 ? 9 : 27, E = NO * DIM * DIM, MM = 16;
    const int64_t pb = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t p = p0 + pb;
    const int a = blockIdx.y;
    if (pb >= ldw || p >= ld) return;
    const int g = (int)(p / LAT_WAVE), l = (int)(p % LAT_WAVE);
    const int qi = uidx[(int64_t)g * nloc + a];
    WT *wr = W + (int64_t)a * E * ldw + pb;
    if (qi < 0) {
        for (int e = 0; e < E; ++e) wr[(int64_t)e * ldw] = (WT)0;
        return;
    }
    const int64_t q = (int64_t)goff[g] + qi;
    const bool own = (umask[q] >> l) & 1;
    double yb[DIM][MM];
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int r = 0; r < MM; ++r)
            yb[i][r] = (own && r < m) ? Ybar[((q * DIM + i) * m + r) * LAT_WAVE + l] : 0.0;
    for (int o = 0; o < NO; ++o) {
        const int nb = unbr[q * NO + o];
        const bool nbo = nb >= 0 && ((umask[nb] >> l) & 1);
        double xv[DIM][MM];
#pragma unroll
        for (int j = 0; j < DIM; ++j)
#pragma unroll
            for (int r = 0; r < MM; ++r)
                xv[j][r] = (nbo && r < m) ? X[(((int64_t)nb * DIM + j) * m + r) * LAT_WAVE + l] : 0.0;
#pragma unroll
        for (int i = 0; i < DIM; ++i)
#pragma unroll
            for (int j = 0; j < DIM; ++j) {
                double v = 0.0;
#pragma unroll
                for (int r = 0; r < MM; ++r) v = fma(yb[i][r], xv[j][r], v);
                wr[(int64_t)((o * DIM + i) * DIM + j) * ldw] = (WT)v;
            }
    }
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

// direct Lame part: bar_{s_k} = sum_i alpha_ik G_ik, zero for non-principal cells.
__global__ void k_zero_vec(int64_t n, double *__restrict__ x)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.0;
}

// one workgroup per slot k: strided partial sums over the cells (canonical order), then a
// fixed-shape tree in LDS (deterministic)
__global__ __launch_bounds__(256) void k_direct_lame(int64_t ncells, int cap, const int32_t *__restrict__ S,
                                                     const int32_t *__restrict__ lane,
                                                     const double *__restrict__ alpha,
                                                     const double *__restrict__ f, double *__restrict__ bar)
{
    __shared__ double sh[256];
    const int k = blockIdx.x;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < ncells; i += 256) s = fma(alpha[i * cap + k], f[(int64_t)lane[i] * cap + k], s);
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) bar[S[k]] = sh[0];
}

template <int DIM, int MC, int MODE>
lat_status launch_apply_nr(const ApplyArgs &A, int nwaves, hipStream_t s)
{
    dim3 grid((unsigned)lat_cdiv(nwaves, 4)), block(256);
    const int nr = A.n_r;
#define APPLY(NRV) hipLaunchKernelGGL((k_apply<DIM, MC, NRV, MODE>), grid, block, 0, s, A, A.goff, A.unode, A.unbr, \
                                      A.umask, A.K, A.alpha_il, A.X, A.Y)
    if (MODE == 2 || nr <= 8) APPLY(8);
    else if (nr <= 16) APPLY(16);
    else if (nr <= 32) APPLY(32);
    else APPLY(64);
#undef APPLY
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

// 2D row walk grid: one workgroup per (group, node row, x-segment); rows are split into two
// segments when that is needed to fill the chip with whole waves of workgroups
int rowwalk_nseg(const lat_plan *P) { return P->ngroups * P->nn >= 1024 ? 1 : (P->nn >= 16 ? 2 : 1); }
int64_t rowwalk_grid(const lat_plan *P) { return (int64_t)P->ngroups * P->nn * rowwalk_nseg(P); }
int64_t apply3d_grid(const lat_plan *P) { return lat_cdiv(P->npacked, APPLY3_RUN); }

template <int MW, int MODE, int LP, bool IDLE>
lat_status launch_rowwalk_nr(const lat_plan *P, const ApplyArgs &A, hipStream_t s)
{
    ApplyArgs B = A;
    B.nseg = rowwalk_nseg(P);
    dim3 grid((unsigned)rowwalk_grid(P)), block(512);
#define RW(NRV) hipLaunchKernelGGL((k_apply2d_rw<MW, NRV, MODE, LP, IDLE>), grid, block, 0, s, B, P->goff, P->uidx, \
                                   P->umask, A.K, A.alpha_il, A.X, A.Y)
    if (MODE == 2 || A.n_r <= 8) RW(8);
    else if (A.n_r <= 16) RW(16);
    else if (A.n_r <= 32) RW(32);
    else RW(64);
#undef RW
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

// One row walk over the right-hand sides A.rb .. A.rb + A.mc - 1: 16 (two per wave), 8 (one per
// wave) or fewer (one per wave, the waves past them only form and stage)
template <int MODE, int LP>
lat_status launch_rowwalk_chunk(const lat_plan *P, const ApplyArgs &A, hipStream_t s)
{
    if (A.mc == 16) return launch_rowwalk_nr<2, MODE, LP, false>(P, A, s);
    if (A.mc == 8) return launch_rowwalk_nr<1, MODE, LP, false>(P, A, s);
    return launch_rowwalk_nr<1, MODE, LP, true>(P, A, s);
}

template <int LP>
lat_status launch_apply3d(const lat_plan *P, const ApplyArgs &A, int mode, hipStream_t s)
{
    dim3 grid((unsigned)apply3d_grid(P)), block(512);
    const int32_t *qgroup = P->goff + P->ngroups + 1;
#define A3(NRV, MD) hipLaunchKernelGGL((k_apply3d_mfma<NRV, MD, LP>), grid, block, 0, s, A, A.goff, A.unode, A.unbr, \
                                       A.umask, A.K, A.alpha_il, A.X, A.Y, (int)P->npacked, qgroup)
#define A3M(MD)                          \
    do {                                 \
        if (A.n_r <= 8) A3(8, MD);        \
        else if (A.n_r <= 16) A3(16, MD); \
        else if (A.n_r <= 32) A3(32, MD); \
        else A3(64, MD);                  \
    } while (0)
    if (mode == 0) A3M(0);
    else A3M(1);
#undef A3M
#undef A3
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

ApplyArgs base_args(const lat_plan *P, int m, int nch)
{
    ApplyArgs A{};
    A.nn = P->nn; A.m = m; A.cap = P->cap; A.ld = P->ld; A.nch = nch;
    A.rb = 0; A.mc = m;
    A.chunks_per_group = (int)lat_cdiv(std::max(P->maxunion, 1), nch);
    A.goff = P->goff; A.unode = P->unode; A.unbr = P->unbr; A.umask = P->umask;
    return A;
}

constexpr int APPLY_NODES_PER_WAVE = 4;
constexpr int FORM_NODES_PER_WAVE = 8;

lat_status interleave_alpha(const lat_plan *P, int n_r, const double *alpha, hipStream_t s)
{
    hipLaunchKernelGGL(k_alpha_il, dim3((unsigned)lat_cdiv(P->ld, 256), (unsigned)P->cap), dim3(256), 0, s, P->ld,
                       P->cap, n_r, P->perm, alpha, P->alpha_il);
    LAT_LAUNCH_CHECK();
    return LAT_OK;
}

// One pass of the ROM apply (mode 0, or 1 = transposed) through the walk kernels, over all right-hand
// sides in chunks of 16, 8 or fewer columns.  LP: 0 = FP64 combination, 1..3 = bf16 slice levels,
// 4 = FP32 operands.  A.errp (reduced precision) receives the error partials of the first chunk
// (the combination is the same for every chunk).
template <int LP>
lat_status walk_pass_lp(const lat_plan *P, ApplyArgs A, int mode, hipStream_t s)
{
    const int m = A.m;
    for (int rb = 0; rb < m;) {
        const int rest = m - rb;
        A.rb = rb;
        A.mc = rest >= 16 ? 16 : (rest >= 8 ? 8 : rest);
        lat_status st;
        if (P->dim == 2) st = mode == 0 ? launch_rowwalk_chunk<0, LP>(P, A, s) : launch_rowwalk_chunk<1, LP>(P, A, s);
        else st = launch_apply3d<LP>(P, A, mode, s);
        if (st != LAT_OK) return st;
        A.errp = nullptr;
        rb += A.mc;
    }
    return LAT_OK;
}

lat_status walk_pass(const lat_plan *P, const ApplyArgs &A, int mode, int lev, hipStream_t s)
{
    switch (lev) {
    case 0: return walk_pass_lp<0>(P, A, mode, s);
    case 1: return walk_pass_lp<1>(P, A, mode, s);
    case 2: return walk_pass_lp<2>(P, A, mode, s);
    case 3: return walk_pass_lp<3>(P, A, mode, s);
    default: return walk_pass_lp<4>(P, A, mode, s);
    }
}

// FP64 apply: ROM (mode 0), transposed ROM (mode 1) or plain per-cell (mode 2).
lat_status run_apply(const lat_plan *P, int mode, const double *K, int n_r, const double *alpha, const double *X,
                     double *Y, int m, hipStream_t s)
{
    if (P->npacked == 0) return LAT_OK;              // no owned DOF anywhere: nothing to write
    ApplyArgs A = base_args(P, m, APPLY_NODES_PER_WAVE);
    A.K = K; A.X = X; A.Y = Y; A.n_r = n_r;
    lat_status st;
    if (mode != 2) {
        if ((st = interleave_alpha(P, n_r, alpha, s)) != LAT_OK) return st;
        A.alpha_il = P->alpha_il;
    }
    const int nwaves = P->ngroups * A.chunks_per_group;
    if (mode == 2) {
        // the per-cell stencil apply: the 2D row walk for m in {8, 16}; with fewer right-hand sides
        // the per-group kernel streams the stencils faster
        if (P->dim == 2 && P->nn >= 3 && (m == 8 || m == 16))
            return m == 16 ? launch_rowwalk_nr<2, 2, 0, false>(P, A, s) : launch_rowwalk_nr<1, 2, 0, false>(P, A, s);
        return P->dim == 2 ? launch_apply<2, 2>(A, nwaves, s) : launch_apply<3, 2>(A, nwaves, s);
    }
    if (P->dim == 2 && P->nn < 3) return mode == 0 ? launch_apply<2, 0>(A, nwaves, s) : launch_apply<2, 1>(A, nwaves, s);
    return walk_pass(P, A, mode, 0, s);
}

// Relative error estimate of one reduced-precision pass: err = sqrt(sum d2 / sum r2) over the
// per-block partials (fixed order: strided per-thread sums, then a tree); the next pass's gate
// opens when err > tol (or err is not a number).  A pass that its own gate skipped leaves the
// estimate as it is and closes the next gate.
__global__ __launch_bounds__(256) void k_lp_err(int64_t nblk, const double *__restrict__ part, double tol,
                                                const int32_t *gate_in, int32_t *gate_out, double *err_est)
{
    __shared__ double sa[256], sb[256];
    if (gate_in && *gate_in == 0) {
        if (threadIdx.x == 0) *gate_out = 0;
        return;
    }
    double a = 0.0, b = 0.0;
    for (int64_t i = threadIdx.x; i < nblk; i += 256) {
        a += part[2 * i];
        b += part[2 * i + 1];
    }
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sa[threadIdx.x] += sa[threadIdx.x + w];
            sb[threadIdx.x] += sb[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double d = sa[0], r = sb[0];
        const double err = r > 0.0 ? sqrt(d / r) : (d > 0.0 ? INFINITY : 0.0);
        if (err_est) *err_est = err;
        *gate_out = (err <= tol) ? 0 : 1;
    }
}

// The FP64 pass of a refinement chain ran: its combination is the FP64 one, estimate 0.
__global__ void k_lp_exact(const int32_t *gate, double *err_est)
{
    if (threadIdx.x == 0 && *gate && err_est) *err_est = 0.0;
}

__global__ void k_fill_scalar(double *x, double v)
{
    if (threadIdx.x == 0) *x = v;
}

// Reduced-precision ROM apply with FP64-measured refinement.  The combination sum_k c_ik K_k runs
// in reduced precision (prec F32: FP32 operands on the FP32 matrix cores; BF16: bf16 slices in
// levels), the apply of the combined stencil in FP64.  Every pass measures its combination
// against the FP64 one at one node (2D) or stencil slice (3D) per workgroup; when that relative
// estimate exceeds refine_tol the apply runs again with one more bf16 level, and after the third
// level (or after FP32) with the FP64 combination.  The passes are chained by device gates: no host
// synchronisation, the skipped passes exit at once.
lat_status run_apply_lowp(const lat_plan *P, int mode, const double *K, int n_r, const double *coef, const double *X,
                          double *Y, int m, int prec, double refine_tol, double *err_est, hipStream_t s)
{
    lat_status st;
    if (n_r < 1 || P->npacked == 0 || (P->dim == 2 && P->nn < 3)) {
        // nothing to combine, or a lattice too small for the walks: the FP64 apply, estimate 0
        if ((st = run_apply(P, mode, K, n_r, coef, X, Y, m, s)) != LAT_OK) return st;
        if (err_est) {
            hipLaunchKernelGGL(k_fill_scalar, dim3(1), dim3(64), 0, s, err_est, 0.0);
            LAT_LAUNCH_CHECK();
        }
        return LAT_OK;
    }
    ApplyArgs A = base_args(P, m, APPLY_NODES_PER_WAVE);
    A.K = K; A.X = X; A.Y = Y; A.n_r = n_r;
    if ((st = interleave_alpha(P, n_r, coef, s)) != LAT_OK) return st;
    A.alpha_il = P->alpha_il;
    const int64_t nblk = P->dim == 2 ? rowwalk_grid(P) : apply3d_grid(P);
    int lev = prec == LAT_F32 ? 4 : (refine_tol >= 0x1p-8 ? 1 : (refine_tol >= 0x1p-16 ? 2 : 3));
    const int32_t *gate = nullptr;
    for (int gi = 0;; ++gi) {
        A.gate = gate;
        A.errp = lev ? P->lp_err : nullptr;
        if ((st = walk_pass(P, A, mode, lev, s)) != LAT_OK) return st;
        if (lev == 0) {
            hipLaunchKernelGGL(k_lp_exact, dim3(1), dim3(64), 0, s, gate, err_est);
            LAT_LAUNCH_CHECK();
            return LAT_OK;
        }
        hipLaunchKernelGGL(k_lp_err, dim3(1), dim3(256), 0, s, nblk, P->lp_err, refine_tol, gate, P->lp_gate + gi,
                           err_est);
        LAT_LAUNCH_CHECK();
        gate = P->lp_gate + gi;
        lev = lev >= 3 ? 0 : lev + 1;
    }
}

// Fused forms for ns (1..3) stacks -> P->form_part laid out [stack][chunk][ld][cap].
lat_status run_forms_fused(const lat_plan *P, const double *const *stk, int ns, int n_r, const double *X,
                           const double *Ybar, int m, int *cpg_out, hipStream_t s)
{
    ApplyArgs A = base_args(P, m, FORMS_RUN);
    A.X = X; A.Ybar = Ybar; A.n_r = n_r;
    const int cpg = A.chunks_per_group;
    if ((int64_t)ns * cpg > P->napc) return LAT_E_SHAPE;
    dim3 grid((unsigned)(P->ngroups * cpg)), block(512);
    const double *k0 = stk[0], *k1 = ns > 1 ? stk[1] : stk[0], *k2 = ns > 2 ? stk[2] : stk[0];
#define FF(D, NRV, NSV) hipLaunchKernelGGL((k_forms_mfma<D, NRV, NSV>), grid, block, 0, s, A, A.goff, A.unode, A.unbr, \
                                           A.umask, k0, k1, k2, X, Ybar, P->form_part, cpg)
#define FFS(D, NRV)                     \
    do {                                \
        if (ns == 1) FF(D, NRV, 1);     \
        else if (ns == 2) FF(D, NRV, 2); \
        else FF(D, NRV, 3);             \
    } while (0)
#define FFD(D)                                 \
    do {                                       \
        if (n_r <= 16) FFS(D, 16);             \
        else if (n_r <= 32) FFS(D, 32);        \
        else FFS(D, 64);                       \
    } while (0)
    if (P->dim == 2) FFD(2);
    else FFD(3);
#undef FFD
#undef FFS
#undef FF
    LAT_LAUNCH_CHECK();
    *cpg_out = cpg;
    return LAT_OK;
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
#define FORMS1(D, NRV) hipLaunchKernelGGL((k_forms<D, NRV>), grid, block, 0, s, A, A.goff, A.unode, A.unbr, A.umask, \
                                           A.K, A.X, A.Ybar, A.Y)
#define FORMS(D)                                                                                   \
    do {                                                                                           \
        if (n_r <= 8) FORMS1(D, 8);                                                                \
        else if (n_r <= 16) FORMS1(D, 16);                                                         \
        else if (n_r <= 32) FORMS1(D, 32);                                                         \
        else FORMS1(D, 64);                                                                        \
    } while (0)
    if (P->dim == 2) FORMS(2);
    else FORMS(3);
#undef FORMS
#undef FORMS1
    LAT_LAUNCH_CHECK();
    return lat_tree_reduce(P->form_part, A.chunks_per_group, P->ld * P->cap, 0, out_pl, P->g_t1, P->g_t2, s);
}

// The adjoint forms of the requested stacks (ROM coefficients, Lame parts) with the plan copy V's
// scratch.  With room for W past the workspace minimum: the cells' W (FP64, or FP32 when
// prec != LAT_F64) in lane batches as large as that room allows (whole 64-lane groups), each batch
// a streaming W pass followed by one row contraction per stack (one pass for all of them when
// n_r <= 32); without it the fused per-node kernel (m <= 16), or one per-node pass per stack.
lat_status run_adjoint_forms(const lat_plan *V, const double *K, const double *K_mu, const double *K_lam,
                             const int32_t *S, int n_r, const double *alpha, const double *X, const double *Ybar,
                             int m, double *alpha_bar, double *mu_bar, double *lam_bar, int prec, hipStream_t stream)
{
    lat_status st;
    const dim3 lg((unsigned)lat_cdiv(V->ld, 256));
    const double *stk[3];
    int role[3], ns = 0;
    if (alpha_bar) { stk[ns] = K; role[ns++] = 0; }
    if (mu_bar) { stk[ns] = K_mu; role[ns++] = 1; }
    if (lam_bar) { stk[ns] = K_lam; role[ns++] = 2; }
    if (ns == 0) return LAT_OK;
    const int64_t ld = V->ld, cap = V->cap, ldc = ld * cap;
    auto finish = [&](int t, const double *forms) -> lat_status {   // forms [ld][cap] -> the output
        if (role[t] == 0) {
            hipLaunchKernelGGL(k_forms_scatter, lg, dim3(256), 0, stream, ld, V->cap, V->perm, forms, alpha_bar);
        } else {
            double *bar = role[t] == 1 ? mu_bar : lam_bar;
            hipLaunchKernelGGL(k_zero_vec, dim3((unsigned)lat_cdiv(V->ncells, 256)), dim3(256), 0, stream, V->ncells,
                               bar);
            if (n_r > 0)
                hipLaunchKernelGGL(k_direct_lame, dim3((unsigned)n_r), dim3(256), 0, stream, V->ncells, V->cap, S,
                                   V->lane, alpha, forms, bar);
        }
        LAT_LAUNCH_CHECK();
        return LAT_OK;
    };
    if (V->npacked == 0 || m > 16 || V->cap < 16) {
        // one per-node pass per stack
        for (int t = 0; t < ns; ++t) {
            if ((st = run_forms(V, stk[t], n_r, X, Ybar, m, V->form_out, stream)) != LAT_OK) return st;
            if ((st = finish(t, V->form_out)) != LAT_OK) return st;
        }
        return LAT_OK;
    }
    // lanes per W batch from the workspace past its minimum (FP32 W: half the W bytes per lane)
    const bool low = prec != LAT_F64;
    const size_t esz = low ? 4 : 8;
    auto batch_bytes = [&](int64_t lanes) {
        return ((size_t)V->nsnap * lanes * esz + 255) / 256 * 256 + ((size_t)3 * V->aa_nchunk * lanes * cap * 8 + 255) / 256 * 256;
    };
    int64_t lanes = 0;
    if (V->ws_rest) {
        lanes = std::min<int64_t>(ld, (int64_t)(V->ws_rest_bytes / (V->nsnap * esz + 3 * V->aa_nchunk * cap * 8)) / 64 * 64);
        while (lanes > 0 && batch_bytes(lanes) > V->ws_rest_bytes) lanes -= 64;
    }
    if (lanes < 64) {
        int cpg = 0;
        if ((st = run_forms_fused(V, stk, ns, n_r, X, Ybar, m, &cpg, stream)) != LAT_OK) return st;
        for (int t = 0; t < ns; ++t) {
            if ((st = lat_tree_reduce(V->form_part + (int64_t)t * cpg * ldc, cpg, ldc, 0, V->form_out, V->g_t1,
                                      V->g_t2, stream)) != LAT_OK)
                return st;
            if ((st = finish(t, V->form_out)) != LAT_OK) return st;
        }
        return LAT_OK;
    }
    char *wbase = V->ws_rest;
    double *W64 = low ? nullptr : (double *)wbase;
    float *W32 = low ? (float *)wbase : nullptr;
    double *parts = (double *)(wbase + ((size_t)V->nsnap * lanes * esz + 255) / 256 * 256);
    // n_r <= 32: the stacks' contractions share one pass over W (chunk partials per stack)
    const bool multi = n_r <= 32;
    for (int64_t p0 = 0; p0 < ld; p0 += lanes) {
        const int64_t ldw = std::min<int64_t>(lanes, ld - p0);
        const dim3 wg((unsigned)lat_cdiv(ldw, 256), (unsigned)V->nloc);
        if (low) {
            if (V->dim == 2)
                hipLaunchKernelGGL((k_forms_W<2, float>), wg, dim3(256), 0, stream, ld, p0, ldw, V->nloc, m, V->goff,
                                   V->uidx, V->unbr, V->umask, X, Ybar, W32);
            else
                hipLaunchKernelGGL((k_forms_W<3, float>), wg, dim3(256), 0, stream, ld, p0, ldw, V->nloc, m, V->goff,
                                   V->uidx, V->unbr, V->umask, X, Ybar, W32);
        } else {
            if (V->dim == 2)
                hipLaunchKernelGGL((k_forms_W<2, double>), wg, dim3(256), 0, stream, ld, p0, ldw, V->nloc, m, V->goff,
                                   V->uidx, V->unbr, V->umask, X, Ybar, W64);
            else
                hipLaunchKernelGGL((k_forms_W<3, double>), wg, dim3(256), 0, stream, ld, p0, ldw, V->nloc, m, V->goff,
                                   V->uidx, V->unbr, V->umask, X, Ybar, W64);
        }
        LAT_LAUNCH_CHECK();
        // the batch as a plan of ldw lanes: contractions and trees write rows p0 .. p0 + ldw - 1
        lat_plan Vb = *V;
        Vb.ld = ldw;
        const int64_t ldcb = ldw * cap;
        double *bparts[3] = {parts, parts + V->aa_nchunk * ldcb, parts + 2 * V->aa_nchunk * ldcb};
        if (multi && (st = lat_contract_rows_multi(&Vb, n_r, W64, W32, stk, ns, bparts, stream)) != LAT_OK) return st;
        for (int t = 0; t < ns; ++t) {
            double *out = V->form_out3 + t * ldc + p0 * cap;
            if (multi) st = lat_tree_reduce(bparts[t], V->aa_nchunk, ldcb, 0, out, V->g_t1, V->g_t2, stream);
            else st = lat_contract_rows(&Vb, n_r, W64, W32, stk[t], out, stream);
            if (st != LAT_OK) return st;
        }
    }
    for (int t = 0; t < ns; ++t)
        if ((st = finish(t, V->form_out3 + t * ldc)) != LAT_OK) return st;
    return LAT_OK;
}

}  // namespace

extern "C" {

lat_status lat_apply_combo(const lat_plan *P, const double *K, int32_t n_r, const double *alpha, const double *X,
                           double *Y, int32_t m, lat_prec prec, double refine_tol, int32_t transpose, double *err_est,
                           void *work, size_t work_bytes, hipStream_t stream)
{
    if (!P || !K || !alpha || !X || !Y || m < 1) return LAT_E_ARG;
    if (n_r < 0 || n_r > P->cap) return LAT_E_SHAPE;
    if (prec != LAT_F64 && prec != LAT_F32 && prec != LAT_BF16) return LAT_E_ARG;
    if (!(refine_tol >= 0.0)) return LAT_E_ARG;
    lat_plan V;
    lat_status st = lat_ws_bind(P, LAT_CALL_APPLY_COMBO, work, work_bytes, &V);
    if (st != LAT_OK) return st;
    const int mode = transpose ? 1 : 0;
    if (prec == LAT_F64) {
        if ((st = run_apply(&V, mode, K, n_r, alpha, X, Y, m, stream)) != LAT_OK) return st;
        if (err_est) {
            hipLaunchKernelGGL(k_fill_scalar, dim3(1), dim3(64), 0, stream, err_est, 0.0);
            LAT_LAUNCH_CHECK();
        }
        return LAT_OK;
    }
    return run_apply_lowp(&V, mode, K, n_r, alpha, X, Y, m, prec, refine_tol, err_est, stream);
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
                                   double *lam_bar, lat_prec prec, double refine_tol, double *err_est, void *work,
                                   size_t work_bytes, hipStream_t stream)
{
    if (!P || !K || !alpha || !X || !Ybar || m < 1) return LAT_E_ARG;
    if (n_r < 0 || n_r > P->cap) return LAT_E_SHAPE;
    if ((mu_bar && !K_mu) || (lam_bar && !K_lam) || ((mu_bar || lam_bar) && !S)) return LAT_E_ARG;
    if (prec != LAT_F64 && prec != LAT_F32 && prec != LAT_BF16) return LAT_E_ARG;
    if (!(refine_tol >= 0.0)) return LAT_E_ARG;
    lat_plan V;
    lat_status st = lat_ws_bind(P, LAT_CALL_APPLY_COMBO_ADJOINT, work, work_bytes, &V);
    if (st != LAT_OK) return st;
    if (Xbar) {
        if (prec == LAT_F64) st = run_apply(&V, 1, K, n_r, alpha, Ybar, Xbar, m, stream);
        else st = run_apply_lowp(&V, 1, K, n_r, alpha, Ybar, Xbar, m, prec, refine_tol, err_est, stream);
        if (st != LAT_OK) return st;
    }
    if (err_est && (prec == LAT_F64 || !Xbar)) {
        hipLaunchKernelGGL(k_fill_scalar, dim3(1), dim3(64), 0, stream, err_est, 0.0);
        LAT_LAUNCH_CHECK();
    }
    return run_adjoint_forms(&V, K, K_mu, K_lam, S, n_r, alpha, X, Ybar, m, alpha_bar, mu_bar, lam_bar, prec, stream);
}

}  // extern "C"
