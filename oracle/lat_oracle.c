/*
 * FP64 CPU oracle for the principal-cell lattice operators.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls this
 * file; it exists so that tests, the smoke check and the CPU baseline of the benchmark
 * can compare the GPU library against a plain, slow, obviously correct implementation
 * written from the paper's definitions.  It shares no code with the GPU library.
 *
 * Conventions (cell-major, "canonical" layouts):
 *   cell edge 1, n elements per axis, h = 1/n; element e = ex + n(ey + n ez);
 *   node a = ix + (n+1)(iy + (n+1) iz); local DOF = d*a + i;
 *   element corner c in {0..2^d-1} sits at offset (c&1, (c>>1)&1, (c>>2)&1);
 *   stencil offset o in {-1,0,1}^d has index (o0+1) + 3(o1+1) + 9(o2+1);
 *   snapshot / stencil of a cell: [(n+1)^d][3^d][d][d], entry (a,o,i,j) = K[(a,i),(a+o,j)].
 *
 * Passages followed (paper: "Efficient Fine-Scale Simulation of Nonlinear Hyperelastic
 * Lattice Structures"):
 *   deformation gradient: eq. (def_grad) and its indicial form in Sec. 3.1.3;
 *   neo-Hookean stress: eq. (sig_eq); tangent: eq. (const_eq), the K^c/K^sigma split and
 *     the tensor D of Sec. 3.1.4 -- written here in the equivalent material form
 *     (first Piola stress P and its derivative A = dP/dF), Sec. 2.2.1 notes both
 *     descriptions give the same predictions;
 *   internal force: eq. (internalloadvec); residual assembly: eq. (residualvector);
 *   Gauss-Legendre quadrature: eq. (fullquadraturerule) and eq. (snapshots);
 *   greedy: Algorithm 1 (Sec. 3.2.2); coefficients: the least-squares formula of Sec. 3.2.2;
 *   ROM operator: eq. (romstiffnessmatrix).
 * Where the paper leaves a choice open, the choice taken is stated at the function that makes it.
 *
 * Compiled with -ffp-contract=off: every fused multiply-add below is an explicit fma().
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_INVERTED 5
#define ORC_E_NONFINITE 6
#define ORC_W_CAP 7

static int ipow(int b, int e) { int r = 1; while (e-- > 0) r *= b; return r; }

/* ------------------------------------------------------------------------ DOF maps */
/* Active local nodes, global numbering of the union lattice's active nodes
 * (lexicographic over the background grid, x fastest), local-to-global map.
 * Returns the number of global active nodes. (eq. residualvector: A^s Boolean.) */
int64_t orc_dofmap(int dim, const int32_t *ncell, int nel, const uint8_t *keep,
                   int32_t *l2g, int32_t *n_active, int64_t *g2bg)
{
    int nn = nel + 1, nloc = ipow(nn, dim), nelem = ipow(nel, dim);
    int64_t ncells = 1, G = 1, gs[3] = {1, 1, 1};
    for (int ax = 0; ax < dim; ++ax) ncells *= ncell[ax];
    for (int ax = 0; ax < dim; ++ax) { gs[ax] = (int64_t)ncell[ax] * nel + 1; G *= gs[ax]; }
    uint8_t *gact = (uint8_t *)calloc((size_t)G, 1);
    uint8_t *lact = (uint8_t *)malloc((size_t)ncells * nloc);
    for (int64_t c = 0; c < ncells; ++c) {
        int cc[3] = {0, 0, 0}; int64_t r = c;
        for (int ax = 0; ax < dim; ++ax) { cc[ax] = (int)(r % ncell[ax]); r /= ncell[ax]; }
        int cnt = 0;
        for (int a = 0; a < nloc; ++a) {
            int ia[3] = {0, 0, 0}, t = a;
            for (int ax = 0; ax < dim; ++ax) { ia[ax] = t % nn; t /= nn; }
            int act = 0;
            /* the node is active when one of its (up to 2^d) elements is kept */
            for (int k = 0; k < (1 << dim) && !act; ++k) {
                int ie[3] = {0, 0, 0}, ok = 1;
                for (int ax = 0; ax < dim; ++ax) {
                    ie[ax] = ia[ax] - ((k >> ax) & 1);
                    if (ie[ax] < 0 || ie[ax] >= nel) ok = 0;
                }
                if (!ok) continue;
                int e = ie[0] + nel * (ie[1] + nel * ie[2]);
                if (keep[c * nelem + e]) act = 1;
            }
            lact[c * nloc + a] = (uint8_t)act;
            cnt += act;
            if (act) {
                int64_t g = 0, st = 1;
                for (int ax = 0; ax < dim; ++ax) { g += ((int64_t)cc[ax] * nel + ia[ax]) * st; st *= gs[ax]; }
                gact[g] = 1;
            }
        }
        n_active[c] = cnt;
    }
    int32_t *gid = (int32_t *)malloc((size_t)G * sizeof(int32_t));
    int64_t ng = 0;
    for (int64_t g = 0; g < G; ++g) {
        if (gact[g]) { if (g2bg) g2bg[ng] = g; gid[g] = (int32_t)ng++; }
        else gid[g] = -1;
    }
    for (int64_t c = 0; c < ncells; ++c) {
        int cc[3] = {0, 0, 0}; int64_t r = c;
        for (int ax = 0; ax < dim; ++ax) { cc[ax] = (int)(r % ncell[ax]); r /= ncell[ax]; }
        for (int a = 0; a < nloc; ++a) {
            int ia[3] = {0, 0, 0}, t = a;
            for (int ax = 0; ax < dim; ++ax) { ia[ax] = t % nn; t /= nn; }
            int64_t g = 0, st = 1;
            for (int ax = 0; ax < dim; ++ax) { g += ((int64_t)cc[ax] * nel + ia[ax]) * st; st *= gs[ax]; }
            l2g[c * nloc + a] = lact[c * nloc + a] ? gid[g] : -1;
        }
    }
    free(gact); free(lact); free(gid);
    return ng;
}

/* ------------------------------------------------------------------------ constitutive law */
static void inv3(const double F[9], double Fi[9], double *J)
{
    double d = F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6])
             + F[2] * (F[3] * F[7] - F[4] * F[6]);
    *J = d;
    Fi[0] = (F[4] * F[8] - F[5] * F[7]) / d;
    Fi[1] = (F[2] * F[7] - F[1] * F[8]) / d;
    Fi[2] = (F[1] * F[5] - F[2] * F[4]) / d;
    Fi[3] = (F[5] * F[6] - F[3] * F[8]) / d;
    Fi[4] = (F[0] * F[8] - F[2] * F[6]) / d;
    Fi[5] = (F[2] * F[3] - F[0] * F[5]) / d;
    Fi[6] = (F[3] * F[7] - F[4] * F[6]) / d;
    Fi[7] = (F[1] * F[6] - F[0] * F[7]) / d;
    Fi[8] = (F[0] * F[4] - F[1] * F[3]) / d;
}

/* Compressible neo-Hookean law in material form, F is 3x3 row-major (F[iJ] = F[3i+J]).
 *   W = mu/2 (tr F^T F - 3) - mu ln J + lam/2 (ln J)^2
 *   P = dW/dF = mu (F - F^{-T}) + lam ln J F^{-T}        (push-forward J^{-1} P F^T = eq. sig_eq)
 *   A_{iJjL} = dP_{iJ}/dF_{jL} = mu d_ij d_JL + (mu - lam ln J) Fi_{Li} Fi_{Jj} + lam Fi_{Ji} Fi_{Lj}
 * (A equals J Fi_{Jk} Fi_{Ll} D_{ijkl} with D of Sec. 3.1.4.)  Returns 0 when J <= 0. */
int orc_neo_hooke(const double F[9], double mu, double lam, double *W, double P[9], double A[81])
{
    double Fi[9], J;
    inv3(F, Fi, &J);
    if (!(J > 0.0)) return 0;
    double lnJ = log(J);
    double I1 = 0.0;
    for (int k = 0; k < 9; ++k) I1 += F[k] * F[k];
    if (W) *W = 0.5 * mu * (I1 - 3.0) - mu * lnJ + 0.5 * lam * lnJ * lnJ;
    if (P)
        for (int i = 0; i < 3; ++i)
            for (int J_ = 0; J_ < 3; ++J_) {
                double FiT = Fi[3 * J_ + i];            /* (F^{-T})_{iJ} = Fi_{Ji} */
                P[3 * i + J_] = mu * (F[3 * i + J_] - FiT) + lam * lnJ * FiT;
            }
    if (A)
        for (int i = 0; i < 3; ++i)
            for (int J_ = 0; J_ < 3; ++J_)
                for (int j = 0; j < 3; ++j)
                    for (int L = 0; L < 3; ++L) {
                        double v = (mu - lam * lnJ) * Fi[3 * L + i] * Fi[3 * J_ + j]
                                 + lam * Fi[3 * J_ + i] * Fi[3 * L + j];
                        if (i == j && J_ == L) v += mu;
                        A[((3 * i + J_) * 3 + j) * 3 + L] = v;
                    }
    return 1;
}

/* ------------------------------------------------------------------------ element quadrature */
/* Q1 shape functions on the element reference square/cube [0,1]^d:
 *   N_c(xi) = prod_ax (bit_ax(c) ? xi_ax : 1 - xi_ax);  g_c = grad_X N_c = grad_xi N_c / h.
 * Gauss-Legendre: 2 points per axis at 1/2 -+ 1/(2 sqrt 3) with weight 1/2 (FULL),
 * or 1 point at 1/2 with weight 1 (REDUCED). */
static int gauss_rule(int dim, int rule, double xi[8][3], double w[8])
{
    double p[2], pw[2]; int np;
    if (rule == 0) { p[0] = 0.5 - 0.5 / sqrt(3.0); p[1] = 0.5 + 0.5 / sqrt(3.0); pw[0] = pw[1] = 0.5; np = 2; }
    else { p[0] = 0.5; pw[0] = 1.0; np = 1; }
    int nq = ipow(np, dim);
    for (int q = 0; q < nq; ++q) {
        int t = q; w[q] = 1.0;
        for (int ax = 0; ax < 3; ++ax) {
            if (ax < dim) { int k = t % np; t /= np; xi[q][ax] = p[k]; w[q] *= pw[k]; }
            else xi[q][ax] = 0.0;
        }
    }
    return nq;
}

static void shape_grads(int dim, double h, const double xi[3], double g[8][3])
{
    int nc = 1 << dim;
    for (int c = 0; c < nc; ++c)
        for (int ax = 0; ax < 3; ++ax) {
            if (ax >= dim) { g[c][ax] = 0.0; continue; }
            double v = 1.0;
            for (int bx = 0; bx < dim; ++bx) {
                int bit = (c >> bx) & 1;
                if (bx == ax) v *= bit ? 1.0 : -1.0;
                else v *= bit ? xi[bx] : 1.0 - xi[bx];
            }
            g[c][ax] = v / h;
        }
}

/* One element: f_e [2^d][d], K_e [2^d d][2^d d], energy. u_e [2^d][d]. Returns 0 if J <= 0. */
static int element_eval(int dim, double h, int rule, const double *u_e, double mu, double lam,
                        double *f_e, double *K_e, double *energy)
{
    double xi[8][3], w[8], g[8][3];
    int nq = gauss_rule(dim, rule, xi, w);
    int nc = 1 << dim, ne = nc * dim;
    double vol = 1.0;
    for (int ax = 0; ax < dim; ++ax) vol *= h;              /* element measure h^d */
    int ok = 1;
    if (f_e) memset(f_e, 0, sizeof(double) * ne);
    if (K_e) memset(K_e, 0, sizeof(double) * ne * ne);
    for (int q = 0; q < nq; ++q) {
        shape_grads(dim, h, xi[q], g);
        double F[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};            /* plane strain: F_33 = 1 in 2D */
        for (int c = 0; c < nc; ++c)
            for (int i = 0; i < dim; ++i)
                for (int J = 0; J < dim; ++J)
                    F[3 * i + J] += u_e[c * dim + i] * g[c][J];
        double Wq, P[9], A[81];
        if (!orc_neo_hooke(F, mu, lam, &Wq, P, A)) { ok = 0; continue; }
        double cq = w[q] * vol;
        if (energy) *energy += cq * Wq;
        if (f_e)
            for (int c = 0; c < nc; ++c)
                for (int i = 0; i < dim; ++i) {
                    double s = 0.0;
                    for (int J = 0; J < dim; ++J) s += P[3 * i + J] * g[c][J];
                    f_e[c * dim + i] += cq * s;
                }
        if (K_e)
            for (int c = 0; c < nc; ++c)
                for (int i = 0; i < dim; ++i)
                    for (int c2 = 0; c2 < nc; ++c2)
                        for (int j = 0; j < dim; ++j) {
                            double s = 0.0;
                            for (int J = 0; J < dim; ++J)
                                for (int L = 0; L < dim; ++L)
                                    s += g[c][J] * A[((3 * i + J) * 3 + j) * 3 + L] * g[c2][L];
                            K_e[(c * dim + i) * ne + c2 * dim + j] += cq * s;
                        }
    }
    return ok;
}

/* ------------------------------------------------------------------------ one cell */
/* Evaluates one cell at local displacement u_c [(n+1)^d][d]:
 *   f_c [(n+1)^d][d]   internal force (cell-local, unassembled)   -- may be NULL
 *   energy             stored energy of the cell                 -- may be NULL
 *   st  [(n+1)^d][3^d][d][d] assembled tangent in stencil layout -- may be NULL
 *   Kd  dense [(n+1)^d d]^2 assembled tangent (small cells only)  -- may be NULL
 * Only kept elements contribute.  Returns ORC_OK or ORC_E_INVERTED (J <= 0 somewhere). */
int orc_cell_eval(int dim, int nel, const uint8_t *keep_c, const double *u_c, double mu, double lam,
                  int rule, double *f_c, double *energy, double *st, double *Kd)
{
    int nn = nel + 1, nloc = ipow(nn, dim), nelem = ipow(nel, dim), nc = 1 << dim;
    int no = ipow(3, dim), ne = nc * dim, ndof = nloc * dim;
    double h = 1.0 / nel;
    double u_e[24], f_e[24], K_e[576];
    int status = ORC_OK;
    if (f_c) memset(f_c, 0, sizeof(double) * ndof);
    if (st) memset(st, 0, sizeof(double) * (size_t)nloc * no * dim * dim);
    if (Kd) memset(Kd, 0, sizeof(double) * (size_t)ndof * ndof);
    if (energy) *energy = 0.0;
    for (int e = 0; e < nelem; ++e) {
        if (!keep_c[e]) continue;
        int ie[3] = {0, 0, 0}, t = e;
        for (int ax = 0; ax < dim; ++ax) { ie[ax] = t % nel; t /= nel; }
        int node[8];
        for (int c = 0; c < nc; ++c) {
            int a = 0, s = 1;
            for (int ax = 0; ax < dim; ++ax) { a += (ie[ax] + ((c >> ax) & 1)) * s; s *= nn; }
            node[c] = a;
            for (int i = 0; i < dim; ++i) u_e[c * dim + i] = u_c[a * dim + i];
        }
        double en = 0.0;
        if (!element_eval(dim, h, rule, u_e, mu, lam, f_c ? f_e : NULL, (st || Kd) ? K_e : NULL,
                          energy ? &en : NULL))
            status = ORC_E_INVERTED;
        if (energy) *energy += en;
        if (f_c)
            for (int c = 0; c < nc; ++c)
                for (int i = 0; i < dim; ++i) f_c[node[c] * dim + i] += f_e[c * dim + i];
        if (st)
            for (int c = 0; c < nc; ++c)
                for (int c2 = 0; c2 < nc; ++c2) {
                    int oi = 0, s = 1;
                    for (int ax = 0; ax < dim; ++ax) { oi += (((c2 >> ax) & 1) - ((c >> ax) & 1) + 1) * s; s *= 3; }
                    for (int i = 0; i < dim; ++i)
                        for (int j = 0; j < dim; ++j)
                            st[(((size_t)node[c] * no + oi) * dim + i) * dim + j] += K_e[(c * dim + i) * ne + c2 * dim + j];
                }
        if (Kd)
            for (int c = 0; c < nc; ++c)
                for (int i = 0; i < dim; ++i)
                    for (int c2 = 0; c2 < nc; ++c2)
                        for (int j = 0; j < dim; ++j)
                            Kd[(size_t)(node[c] * dim + i) * ndof + node[c2] * dim + j] += K_e[(c * dim + i) * ne + c2 * dim + j];
    }
    return status;
}

/* Batched over cells (OpenMP over cells; cells are independent). u_loc [Ns][(n+1)^d][d]. */
int orc_cells_eval(int dim, int nel, int64_t ncells, const uint8_t *keep, const double *u_loc,
                   const double *mu, const double *lam, int rule, double *f, double *energy, double *T,
                   int32_t *status_cell)
{
    int nloc = ipow(nel + 1, dim), nelem = ipow(nel, dim);
    int64_t nsnap = (int64_t)nloc * ipow(3, dim) * dim * dim;
    int worst = ORC_OK;
#pragma omp parallel for schedule(dynamic, 1) reduction(max : worst)
    for (int64_t c = 0; c < ncells; ++c) {
        int s = orc_cell_eval(dim, nel, keep + c * nelem, u_loc + c * (int64_t)nloc * dim, mu[c], lam[c], rule,
                              f ? f + c * (int64_t)nloc * dim : NULL, energy ? energy + c : NULL,
                              T ? T + c * nsnap : NULL, NULL);
        if (status_cell) status_cell[c] = s;
        if (s > worst) worst = s;
    }
    return worst;
}

/* ------------------------------------------------------------------------ greedy (Algorithm 1) */
/* Dot product in the fixed arithmetic order the library specifies for decisions:
 * contiguous chunks of 256 entries in index order, each accumulated from 0 by
 * s = fma(x_j, y_j, s); the chunk sums are then combined by a pairwise tree
 * (level by level, neighbours (2k, 2k+1) added, an odd last element carried up). */
#define ORC_CHUNK 256
double orc_dot(const double *x, const double *y, int64_t n)
{
    int64_t nc = (n + ORC_CHUNK - 1) / ORC_CHUNK;
    if (nc == 0) return 0.0;
    double *p = (double *)malloc(sizeof(double) * (size_t)nc);
    for (int64_t b = 0; b < nc; ++b) {
        double s = 0.0;
        int64_t j1 = (b + 1) * ORC_CHUNK < n ? (b + 1) * ORC_CHUNK : n;
        for (int64_t j = b * ORC_CHUNK; j < j1; ++j) s = fma(x[j], y[j], s);
        p[b] = s;
    }
    int64_t m = nc;
    while (m > 1) {
        int64_t half = m / 2;
        for (int64_t k = 0; k < half; ++k) p[k] = p[2 * k] + p[2 * k + 1];
        if (m & 1) p[half] = p[m - 1];
        m = half + (m & 1);
    }
    double r = p[0];
    free(p);
    return r;
}

static double inf_norm(const double *x, int64_t n)
{
    double m = 0.0;
    for (int64_t j = 0; j < n; ++j) { double a = fabs(x[j]); if (a > m) m = a; }
    return m;
}

/* Algorithm 1.  D [Ns][nsnap] holds the snapshots on entry and the residuals Delta on exit.
 * Outputs: S[cap] principal cells (0-based, -1 past n_r), n_r, beta [Ns][cap] (coordinates
 * beta_i^s), nu [Ns] = ||t^s||_2, R [cap][cap] with R[j][k] = nu_{s_k} beta_j^{s_k} (j <= k),
 * Z [cap][nsnap] the orthonormal basis (may be NULL), achieved = max_s ||Delta^s||_inf at exit.
 * Readings: ties of the argmax go to the lowest cell index; a zero snapshot gives Delta = 0
 * and is never selected; the loop also stops at `cap` selections (status ORC_W_CAP when the
 * tolerance is then still not met). */
int orc_greedy(int64_t nsnap, int64_t Ns, double *D, double tol, int cap, int32_t *S, int32_t *n_r,
               double *beta, double *nu, double *R, double *Z, double *achieved)
{
    double *mx = (double *)malloc(sizeof(double) * (size_t)Ns);
    double *zeta = (double *)malloc(sizeof(double) * (size_t)nsnap);
    for (int k = 0; k < cap; ++k) S[k] = -1;
    memset(beta, 0, sizeof(double) * (size_t)Ns * cap);
    memset(R, 0, sizeof(double) * (size_t)cap * cap);
    /* normalisation: Delta_0^s = t^s / ||t^s||_2 */
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < Ns; ++s) {
        double *x = D + s * nsnap;
        double nrm = sqrt(orc_dot(x, x, nsnap));
        nu[s] = nrm;
        if (nrm > 0.0) for (int64_t j = 0; j < nsnap; ++j) x[j] = x[j] / nrm;
        else for (int64_t j = 0; j < nsnap; ++j) x[j] = 0.0;
        mx[s] = inf_norm(x, nsnap);
    }
    int i = 0, status = ORC_OK;
    for (;;) {
        int64_t best = 0;
        for (int64_t s = 1; s < Ns; ++s) if (mx[s] > mx[best]) best = s;   /* strict: lowest index wins ties */
        double top = mx[best];
        if (!(top > tol)) break;
        if (i == cap) { status = ORC_W_CAP; break; }
        const double *xs = D + best * nsnap;
        double rho = sqrt(orc_dot(xs, xs, nsnap));
        for (int64_t j = 0; j < nsnap; ++j) zeta[j] = xs[j] / rho;
        if (Z) memcpy(Z + (int64_t)i * nsnap, zeta, sizeof(double) * (size_t)nsnap);
        S[i] = (int32_t)best;
#pragma omp parallel for schedule(static)
        for (int64_t s = 0; s < Ns; ++s) {
            double *x = D + s * nsnap;
            double b = orc_dot(x, zeta, nsnap);
            beta[s * cap + i] = b;
            for (int64_t j = 0; j < nsnap; ++j) x[j] = fma(-b, zeta[j], x[j]);
            mx[s] = inf_norm(x, nsnap);
        }
        ++i;
    }
    *n_r = i;
    double ach = 0.0;
    for (int64_t s = 0; s < Ns; ++s) if (mx[s] > ach) ach = mx[s];
    *achieved = ach;
    for (int k = 0; k < i; ++k)
        for (int j = 0; j <= k; ++j) R[j * cap + k] = nu[S[k]] * beta[(int64_t)S[k] * cap + j];
    free(mx); free(zeta);
    return status;
}

/* RB coefficients alpha^s: the least-squares coordinates of t^s in the principal snapshots,
 * obtained from the greedy's certified decomposition as R alpha^s = nu_s beta^s
 * (R upper triangular), solved by back-substitution from the last row. alpha [Ns][cap]. */
void orc_alpha(int64_t Ns, int cap, int n_r, const double *R, const double *nu, const double *beta,
               double *alpha)
{
    for (int64_t s = 0; s < Ns; ++s) {
        double *a = alpha + s * cap;
        for (int k = 0; k < cap; ++k) a[k] = 0.0;
        for (int k = n_r - 1; k >= 0; --k) {
            double acc = nu[s] * beta[s * cap + k];
            for (int l = k + 1; l < n_r; ++l) acc = fma(-R[k * cap + l], a[l], acc);
            a[k] = acc / R[k * cap + k];
        }
    }
}

/* ------------------------------------------------------------------------ operator applies */
/* y = M K M x for one cell, K in stencil layout, M the active-DOF mask (l2g >= 0);
 * transpose != 0 applies K^T instead. x, y [(n+1)^d][d][m]. */
void orc_stencil_apply(int dim, int nel, const double *st, const int32_t *l2g_c, const double *x, int m,
                       int transpose, double *y)
{
    int nn = nel + 1, nloc = ipow(nn, dim), no = ipow(3, dim);
    memset(y, 0, sizeof(double) * (size_t)nloc * dim * m);
    for (int a = 0; a < nloc; ++a) {
        if (l2g_c[a] < 0) continue;
        int ia[3] = {0, 0, 0}, t = a;
        for (int ax = 0; ax < dim; ++ax) { ia[ax] = t % nn; t /= nn; }
        for (int o = 0; o < no; ++o) {
            int ib[3] = {0, 0, 0}, to = o, ok = 1, b = 0, s = 1;
            for (int ax = 0; ax < dim; ++ax) {
                ib[ax] = ia[ax] + (to % 3) - 1; to /= 3;
                if (ib[ax] < 0 || ib[ax] >= nn) ok = 0;
                b += ib[ax] * s; s *= nn;
            }
            if (!ok || l2g_c[b] < 0) continue;
            if (!transpose) {
                /* y[a,i] += K[(a,i),(b,j)] x[b,j],  K[(a,i),(b,j)] = st[a,o,i,j] */
                const double *K = st + ((size_t)a * no + o) * dim * dim;
                for (int i = 0; i < dim; ++i)
                    for (int j = 0; j < dim; ++j)
                        for (int c = 0; c < m; ++c)
                            y[((size_t)a * dim + i) * m + c] += K[i * dim + j] * x[((size_t)b * dim + j) * m + c];
            } else {
                /* y[a,i] += K[(b,j),(a,i)] x[b,j],  K[(b,j),(a,i)] = st[b,-o,j,i] */
                int onegi = no - 1 - o;
                const double *K = st + ((size_t)b * no + onegi) * dim * dim;
                for (int i = 0; i < dim; ++i)
                    for (int j = 0; j < dim; ++j)
                        for (int c = 0; c < m; ++c)
                            y[((size_t)a * dim + i) * m + c] += K[j * dim + i] * x[((size_t)b * dim + j) * m + c];
            }
        }
    }
}

/* Plain per-cell apply Y_i = M_i K_i M_i X_i with each cell's own stencil Kst [Ns][nsnap]. */
void orc_plain_apply(int dim, int nel, int64_t Ns, const double *Kst, const int32_t *l2g, const double *X,
                     int m, int transpose, double *Y)
{
    int nloc = ipow(nel + 1, dim);
    int64_t nsnap = (int64_t)nloc * ipow(3, dim) * dim * dim;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < Ns; ++c)
        orc_stencil_apply(dim, nel, Kst + c * nsnap, l2g + c * nloc, X + c * (int64_t)nloc * dim * m, m,
                          transpose, Y + c * (int64_t)nloc * dim * m);
}

/* ROM apply (eq. romstiffnessmatrix): Ktilde_i = sum_k alpha_ik K_k, then Y_i = M_i Ktilde_i M_i X_i.
 * Kp [n_r][nsnap] principal stencils, alpha [Ns][cap]. */
void orc_combo_apply(int dim, int nel, int64_t Ns, int n_r, const double *Kp, const double *alpha, int cap,
                     const int32_t *l2g, const double *X, int m, int transpose, double *Y)
{
    int nloc = ipow(nel + 1, dim);
    int64_t nsnap = (int64_t)nloc * ipow(3, dim) * dim * dim;
#pragma omp parallel
    {
        double *Kt = (double *)malloc(sizeof(double) * (size_t)nsnap);
#pragma omp for schedule(static)
        for (int64_t c = 0; c < Ns; ++c) {
            for (int64_t q = 0; q < nsnap; ++q) Kt[q] = 0.0;
            for (int k = 0; k < n_r; ++k) {
                double a = alpha[c * cap + k];
                const double *K = Kp + (int64_t)k * nsnap;
                for (int64_t q = 0; q < nsnap; ++q) Kt[q] += a * K[q];
            }
            orc_stencil_apply(dim, nel, Kt, l2g + c * nloc, X + c * (int64_t)nloc * dim * m, m, transpose,
                              Y + c * (int64_t)nloc * dim * m);
        }
        free(Kt);
    }
}

/* Bilinear forms G[i][k] = <M_i Ybar_i, K_k M_i X_i> for all cells i and principal operators k
 * (the derivative of Y_i = sum_k alpha_ik K_k X_i with respect to alpha_ik). G [Ns][cap]. */
void orc_combo_forms(int dim, int nel, int64_t Ns, int n_r, const double *Kp, int cap, const int32_t *l2g,
                     const double *X, const double *Ybar, int m, double *G)
{
    int nloc = ipow(nel + 1, dim);
    int64_t nsnap = (int64_t)nloc * ipow(3, dim) * dim * dim, nv = (int64_t)nloc * dim * m;
#pragma omp parallel
    {
        double *y = (double *)malloc(sizeof(double) * (size_t)nv);
#pragma omp for schedule(static)
        for (int64_t c = 0; c < Ns; ++c) {
            const int32_t *lc = l2g + c * nloc;
            for (int k = 0; k < cap; ++k) G[c * cap + k] = 0.0;
            for (int k = 0; k < n_r; ++k) {
                orc_stencil_apply(dim, nel, Kp + (int64_t)k * nsnap, lc, X + c * nv, m, 0, y);
                double s = 0.0;
                for (int64_t q = 0; q < nv; ++q) s += Ybar[c * nv + q] * y[q];   /* y is already masked */
                G[c * cap + k] = s;
            }
        }
        free(y);
    }
}
