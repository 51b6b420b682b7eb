/*
 * FP64 CPU oracle for the Brillouin-kernel overlap operator.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant generator
 * with the HIP library.
 *
 * What it computes, each piece written out from its plain definition
 * (Duerr & Koutsou, "On the suitability of the Brillouin action as a kernel
 * to the overlap procedure", arXiv:1701.00726):
 *
 *   orc_links      off-axis links W_d(x) for all 81 displacements d in
 *                  {-1,0,1}^4: the average over all k! shortest lattice
 *                  paths from x to x+d (k = number of non-zero d_mu) of the
 *                  ordered product of the links along the path; no
 *                  projection back to SU(3) (App. C.1: the average, not the
 *                  projection, is the favoured choice, and it keeps the
 *                  operator gamma5-hermitian).
 *   orc_dirac      the Brillouin operator, eq. (def_bril) with c_SW = 0, as
 *                  the direct sum over the 81-point hypercube,
 *                  (D psi)(x) = sum_d S_d (x) W_d(x) psi(x+d).
 *                  The spin matrices S_d are the position-space weights of
 *                  the isotropic derivative and the Brillouin Laplacian,
 *                  read off from their momentum-space forms (App. A:
 *                  p~_mu = sin p_mu prod_{nu!=mu} (cos p_nu + 2)/3 and
 *                  lap^bri = (1/4) prod_mu (cos p_mu + 1) - 4).
 *                  Each factor (cos p + 2)/3 is the one-axis stencil
 *                  {1/6, 2/3, 1/6}; i sin p is {-1/2, 0, +1/2}; (cos p + 1)
 *                  is {1/2, 1, 1/2}.  The bare mass sits on the 0-hop term
 *                  (App. C.1 (ii)).
 *   orc_dirac_adj  the adjoint D^dag by its definition D^dag(x,y) = D(y,x)^dag
 *                  (transposed sum; gamma5-hermiticity is NOT used here, so a
 *                  test can check it).
 *   orc_dirac_dense  the same operator as a dense matrix (small lattices).
 *   orc_dirac_at, orc_dirac_adj_at  D psi and D^dag psi at listed sites only, with
 *                  the links of those sites (and their neighbours) built on the
 *                  fly, for lattices too large for the full link array.
 *   orc_wilson, orc_wilson_adj, orc_wilson_dense  the Wilson operator of eq. (def_wils)
 *                  (c_SW = 0) from its covariant derivative and 9-point Laplacian, applied
 *                  block by block straight from U; the adjoint as the transposed sum.
 *   orc_clover, orc_clover_apply  the clover term -(c_SW/2) sum sigma_mu_nu F_mu_nu with the
 *                  clover-leaf F_mu_nu (the paper gives no discretisation; see orc_clover),
 *                  and its site-local application (any kernel, and its adjoint).
 *   orc_cg         textbook conjugate gradient on (D^dag D + sigma) x = b, for either kernel
 *                  (kern 0: Brillouin with its link array W; kern 1: Wilson with U and tbc).
 *   orc_rational   y = c0 b + sum_i omega_i (D^dag D + sigma_i)^{-1} b, every
 *                  shift solved separately (eq. (KLnn_parfrac) with
 *                  X^dag X = D^dag D).
 *   orc_link_force derivative of Re sum_p w_p u_p^dag D v_p with respect to
 *                  the Gell-Mann components of log U (Sec. 9), by the product
 *                  rule along every path of every W_d(x).
 *
 * Gamma matrices: the paper only says "chiral representation" (App. C.1).
 * Used here: gamma_k = [[0, -i s_k], [i s_k, 0]] (s_k the Pauli matrices),
 * gamma_4 = [[0, 1], [1, 0]], gamma5 = gamma_1 gamma_2 gamma_3 gamma_4.
 *
 * Layouts (oracle-private, site-major):
 *   U   [4][V][3][3]      W   [V][81][3][3]      psi [nrhs][V][4][3]
 *   site s = x + Lx*(y + Ly*(z + Lz*t)); displacement index
 *   j = sum_mu (d_mu + 1) 3^mu, so j = 40 is d = 0 and j, 80-j are opposite.
 * tbc = 1 makes the fermion field antiperiodic in t: a path step that crosses
 * the t boundary picks up a factor -1.
 */
#include <complex.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ geometry */

static long vol(const int L[4]) { return (long)L[0] * L[1] * L[2] * L[3]; }

static void coords(const int L[4], long s, int c[4]) {
    for (int mu = 0; mu < 4; ++mu) {
        c[mu] = (int)(s % L[mu]);
        s /= L[mu];
    }
}

static long site_of(const int L[4], const int c[4]) {
    long s = 0;
    for (int mu = 3; mu >= 0; --mu) {
        int v = ((c[mu] % L[mu]) + L[mu]) % L[mu];
        s = s * L[mu] + v;
    }
    return s;
}

static void disp_of(int j, int d[4]) {
    for (int mu = 0; mu < 4; ++mu) {
        d[mu] = j % 3 - 1;
        j /= 3;
    }
}

/* ------------------------------------------------------------- gamma basis */

static cplx GAM[5][4][4];
static int gam_ready = 0;

static void init_gammas(void) {
    if (gam_ready) return;
    const cplx iu = _Complex_I;
    cplx pauli[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -iu}, {iu, 0}},
        {{1, 0}, {0, -1}},
    };
    memset(GAM, 0, sizeof(GAM));
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                GAM[k][a][2 + b] = -iu * pauli[k][a][b];
                GAM[k][2 + a][b] = iu * pauli[k][a][b];
            }
    for (int a = 0; a < 2; ++a) {
        GAM[3][a][2 + a] = 1;
        GAM[3][2 + a][a] = 1;
    }
    /* gamma5 = gamma_1 gamma_2 gamma_3 gamma_4 */
    cplx t1[4][4], t2[4][4];
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            cplx s = 0;
            for (int c = 0; c < 4; ++c) s += GAM[0][a][c] * GAM[1][c][b];
            t1[a][b] = s;
        }
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            cplx s = 0;
            for (int c = 0; c < 4; ++c) s += t1[a][c] * GAM[2][c][b];
            t2[a][b] = s;
        }
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            cplx s = 0;
            for (int c = 0; c < 4; ++c) s += t2[a][c] * GAM[3][c][b];
            GAM[4][a][b] = s;
        }
    gam_ready = 1;
}

void orc_gamma(int mu, cplx *out16) {
    init_gammas();
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) out16[4 * a + b] = GAM[mu][a][b];
}

/* ------------------------------------------------------- stencil weights */

/* one-axis factors read off from the momentum forms */
static double w_iso(int dnu) { return dnu == 0 ? 2.0 / 3.0 : 1.0 / 6.0; } /* (cos p + 2)/3 */
static double w_lap(int dnu) { return dnu == 0 ? 1.0 : 0.5; }             /* (cos p + 1)   */

/* S_d for displacement index j: 4x4 spin matrix multiplying W_d(x) psi(x+d) */
static void spin_matrix(int j, double m0, cplx S[4][4]) {
    init_gammas();
    int d[4];
    disp_of(j, d);
    int zero = (d[0] == 0 && d[1] == 0 && d[2] == 0 && d[3] == 0);
    /* -(1/2) lap^bri : (1/4) prod f - 4 delta  ->  -(1/8) prod f + 2 delta */
    double prodf = 1.0;
    for (int mu = 0; mu < 4; ++mu) prodf *= w_lap(d[mu]);
    double scal = -prodf / 8.0 + (zero ? 2.0 + m0 : 0.0);
    memset(S, 0, sizeof(cplx) * 16);
    for (int a = 0; a < 4; ++a) S[a][a] = scal;
    /* sum_mu gamma_mu nabla^iso_mu : weight (d_mu/2) prod_{nu != mu} w_iso(d_nu) */
    for (int mu = 0; mu < 4; ++mu) {
        if (d[mu] == 0) continue;
        double c = 0.5 * d[mu];
        for (int nu = 0; nu < 4; ++nu)
            if (nu != mu) c *= w_iso(d[nu]);
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) S[a][b] += c * GAM[mu][a][b];
    }
}

void orc_spin_matrix(int j, double m0, cplx *out16) {
    cplx S[4][4];
    spin_matrix(j, m0, S);
    memcpy(out16, S, sizeof(S));
}

/* ------------------------------------------------------- off-axis links */

static void mat_mul(const cplx *A, const cplx *B, cplx *C) {
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            cplx s = 0;
            for (int c = 0; c < 3; ++c) s += A[3 * a + c] * B[3 * c + b];
            C[3 * a + b] = s;
        }
}

static void mat_mul_dag(const cplx *A, const cplx *B, cplx *C) { /* A B^dag */
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            cplx s = 0;
            for (int c = 0; c < 3; ++c) s += A[3 * a + c] * conj(B[3 * b + c]);
            C[3 * a + b] = s;
        }
}

/* all permutations of {0..k-1} for k = 0..4, generated once by recursive swapping */
static int PERM[5][24][4];
static int NPERM[5];
static int perm_ready = 0;

static void gen_perm(int k, int *a, int pos) {
    if (pos == k) {
        memcpy(PERM[k][NPERM[k]++], a, sizeof(int) * 4);
        return;
    }
    for (int i = pos; i < k; ++i) {
        int t = a[pos]; a[pos] = a[i]; a[i] = t;
        gen_perm(k, a, pos + 1);
        t = a[pos]; a[pos] = a[i]; a[i] = t;
    }
}

static void init_perms(void) {
    if (perm_ready) return;
    for (int k = 0; k <= 4; ++k) {
        int a[4] = {0, 1, 2, 3};
        NPERM[k] = 0;
        gen_perm(k, a, 0);
    }
    perm_ready = 1;
}

/* the 81 path-averaged links W_d(x) of one site x, out[81][9] */
static void links_site(const int *L, int tbc, const cplx *U, long x, cplx *out81) {
    const long V = vol(L);
    int cx[4];
    coords(L, x, cx);
    for (int j = 0; j < 81; ++j) {
        int d[4];
        disp_of(j, d);
        int axes[4], k = 0;
        for (int mu = 0; mu < 4; ++mu)
            if (d[mu] != 0) axes[k++] = mu;
        cplx *out = out81 + (size_t)j * 9;
        cplx acc[9] = {0};
        /* enumerate the k! orderings of the non-zero axes */
        const int np_local = NPERM[k];
        const int (*pl)[4] = PERM[k];
        for (int p = 0; p < np_local; ++p) {
            cplx M[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
            int cy[4] = {cx[0], cx[1], cx[2], cx[3]};
            double sign = 1.0;
            for (int st = 0; st < k; ++st) {
                int mu = axes[pl[p][st]];
                cplx T[9];
                if (d[mu] > 0) {
                    /* step +mu: multiply by U_mu(y), then y -> y + mu */
                    long sy = site_of(L, cy);
                    mat_mul(M, U + ((size_t)mu * V + sy) * 9, T);
                    if (tbc && mu == 3 && cy[3] == L[3] - 1) sign = -sign;
                    cy[mu] += 1;
                } else {
                    /* step -mu: y -> y - mu, multiply by U_mu(y)^dag */
                    if (tbc && mu == 3 && cy[3] == 0) sign = -sign;
                    cy[mu] -= 1;
                    long sy = site_of(L, cy);
                    mat_mul_dag(M, U + ((size_t)mu * V + sy) * 9, T);
                }
                memcpy(M, T, sizeof(T));
            }
            for (int e = 0; e < 9; ++e) acc[e] += sign * M[e];
        }
        for (int e = 0; e < 9; ++e) out[e] = acc[e] / (double)np_local;
    }
}

void orc_links(const int *L, int tbc, const cplx *U, cplx *W) {
    const long V = vol(L);
    init_perms();
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x) links_site(L, tbc, U, x, W + (size_t)x * 81 * 9);
}

/* ------------------------------------------------------------ the operator */

static void neighbour_table(const int L[4], long x, long nb[81]) {
    int cx[4];
    coords(L, x, cx);
    for (int j = 0; j < 81; ++j) {
        int d[4], cy[4];
        disp_of(j, d);
        for (int mu = 0; mu < 4; ++mu) cy[mu] = cx[mu] + d[mu];
        nb[j] = site_of(L, cy);
    }
}

void orc_dirac(const int *L, const cplx *W, double m0, const cplx *in, cplx *out, int nrhs) {
    const long V = vol(L);
    cplx S[81][4][4];
    for (int j = 0; j < 81; ++j) spin_matrix(j, m0, S[j]);
    for (int r = 0; r < nrhs; ++r) {
        const cplx *src = in + (size_t)r * V * 12;
        cplx *dst = out + (size_t)r * V * 12;
#pragma omp parallel for schedule(static)
        for (long x = 0; x < V; ++x) {
            long nb[81];
            neighbour_table(L, x, nb);
            cplx acc[4][3] = {{0}};
            for (int j = 0; j < 81; ++j) {
                const cplx *Wd = W + ((size_t)x * 81 + j) * 9;
                const cplx *p = src + (size_t)nb[j] * 12;
                cplx tp[4][3]; /* W_d(x) psi(x+d), colour rotated, per spin */
                for (int s = 0; s < 4; ++s)
                    for (int a = 0; a < 3; ++a) {
                        cplx v = 0;
                        for (int b = 0; b < 3; ++b) v += Wd[3 * a + b] * p[3 * s + b];
                        tp[s][a] = v;
                    }
                for (int s = 0; s < 4; ++s)
                    for (int a = 0; a < 3; ++a) {
                        cplx v = 0;
                        for (int t = 0; t < 4; ++t) v += S[j][s][t] * tp[t][a];
                        acc[s][a] += v;
                    }
            }
            for (int s = 0; s < 4; ++s)
                for (int a = 0; a < 3; ++a) dst[(size_t)x * 12 + 3 * s + a] = acc[s][a];
        }
    }
}

/* D^dag(x, x+d) = D(x+d, x)^dag = S_{-d}^dag (x) W_{-d}(x+d)^dag */
void orc_dirac_adj(const int *L, const cplx *W, double m0, const cplx *in, cplx *out, int nrhs) {
    const long V = vol(L);
    cplx S[81][4][4];
    for (int j = 0; j < 81; ++j) spin_matrix(j, m0, S[j]);
    for (int r = 0; r < nrhs; ++r) {
        const cplx *src = in + (size_t)r * V * 12;
        cplx *dst = out + (size_t)r * V * 12;
#pragma omp parallel for schedule(static)
        for (long x = 0; x < V; ++x) {
            long nb[81];
            neighbour_table(L, x, nb);
            cplx acc[4][3] = {{0}};
            for (int j = 0; j < 81; ++j) {
                int jm = 80 - j; /* the displacement -d */
                long y = nb[j];  /* y = x + d */
                const cplx *Wy = W + ((size_t)y * 81 + jm) * 9; /* W_{-d}(x+d) */
                const cplx *p = src + (size_t)y * 12;
                cplx tp[4][3];
                for (int s = 0; s < 4; ++s)
                    for (int a = 0; a < 3; ++a) {
                        cplx v = 0;
                        for (int b = 0; b < 3; ++b) v += conj(Wy[3 * b + a]) * p[3 * s + b];
                        tp[s][a] = v;
                    }
                for (int s = 0; s < 4; ++s)
                    for (int a = 0; a < 3; ++a) {
                        cplx v = 0;
                        for (int t = 0; t < 4; ++t) v += conj(S[jm][t][s]) * tp[t][a];
                        acc[s][a] += v;
                    }
            }
            for (int s = 0; s < 4; ++s)
                for (int a = 0; a < 3; ++a) dst[(size_t)x * 12 + 3 * s + a] = acc[s][a];
        }
    }
}

/* dense matrix, row/col index = 12*site + 3*spin + colour */
void orc_dirac_dense(const int *L, const cplx *W, double m0, cplx *M) {
    const long V = vol(L);
    const long n = 12 * V;
    cplx S[81][4][4];
    for (int j = 0; j < 81; ++j) spin_matrix(j, m0, S[j]);
    memset(M, 0, sizeof(cplx) * (size_t)n * n);
    for (long x = 0; x < V; ++x) {
        long nb[81];
        neighbour_table(L, x, nb);
        for (int j = 0; j < 81; ++j) {
            const cplx *Wd = W + ((size_t)x * 81 + j) * 9;
            for (int s = 0; s < 4; ++s)
                for (int a = 0; a < 3; ++a)
                    for (int t = 0; t < 4; ++t)
                        for (int b = 0; b < 3; ++b)
                            M[(size_t)(12 * x + 3 * s + a) * n + 12 * nb[j] + 3 * t + b] +=
                                S[j][s][t] * Wd[3 * a + b];
        }
    }
}

/* (D psi)(x) and (D^dag psi)(x) at the listed sites only, with the links built
 * on the fly from U (for lattices too large for the full link array).  Same sums
 * as orc_dirac / orc_dirac_adj.  out[nsites][4][3]. */
void orc_dirac_at(const int *L, int tbc, const cplx *U, double m0, const cplx *in, int nsites, const long *sites,
                  cplx *out) {
    init_perms();
    cplx S[81][4][4];
    for (int j = 0; j < 81; ++j) spin_matrix(j, m0, S[j]);
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < nsites; ++i) {
        const long x = sites[i];
        cplx Wx[81 * 9];
        links_site(L, tbc, U, x, Wx);
        long nb[81];
        neighbour_table(L, x, nb);
        cplx acc[4][3] = {{0}};
        for (int j = 0; j < 81; ++j) {
            const cplx *Wd = Wx + (size_t)j * 9;
            const cplx *p = in + (size_t)nb[j] * 12;
            for (int s = 0; s < 4; ++s)
                for (int a = 0; a < 3; ++a) {
                    cplx v = 0;
                    for (int t = 0; t < 4; ++t)
                        for (int b = 0; b < 3; ++b) v += S[j][s][t] * Wd[3 * a + b] * p[3 * t + b];
                    acc[s][a] += v;
                }
        }
        for (int s = 0; s < 4; ++s)
            for (int a = 0; a < 3; ++a) out[(size_t)i * 12 + 3 * s + a] = acc[s][a];
    }
}

void orc_dirac_adj_at(const int *L, int tbc, const cplx *U, double m0, const cplx *in, int nsites, const long *sites,
                      cplx *out) {
    init_perms();
    cplx S[81][4][4];
    for (int j = 0; j < 81; ++j) spin_matrix(j, m0, S[j]);
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < nsites; ++i) {
        const long x = sites[i];
        long nb[81];
        neighbour_table(L, x, nb);
        cplx acc[4][3] = {{0}};
        cplx Wy[81 * 9];
        for (int j = 0; j < 81; ++j) {
            /* D^dag(x, x+d) = D(x+d, x)^dag = S_{-d}^dag W_{-d}(x+d)^dag */
            const int jm = 80 - j;
            const long y = nb[j];
            links_site(L, tbc, U, y, Wy);
            const cplx *Wd = Wy + (size_t)jm * 9;
            const cplx *p = in + (size_t)y * 12;
            for (int s = 0; s < 4; ++s)
                for (int a = 0; a < 3; ++a) {
                    cplx v = 0;
                    for (int t = 0; t < 4; ++t)
                        for (int b = 0; b < 3; ++b) v += conj(S[jm][t][s]) * conj(Wd[3 * b + a]) * p[3 * t + b];
                    acc[s][a] += v;
                }
        }
        for (int s = 0; s < 4; ++s)
            for (int a = 0; a < 3; ++a) out[(size_t)i * 12 + 3 * s + a] = acc[s][a];
    }
}

/* ------------------------------------------------------------ Wilson kernel */

/*
 * The Wilson operator, eq. (def_wils) with c_SW = 0:
 *   D_wil = sum_mu gamma_mu nabla_mu - (1/2) lap + m0,
 *   nabla_mu psi(x) = (1/2) [U_mu(x) psi(x+mu) - U_mu(x-mu)^dag psi(x-mu)],
 *   lap psi(x) = sum_mu [U_mu(x) psi(x+mu) + U_mu(x-mu)^dag psi(x-mu) - 2 psi(x)].
 * Collecting the terms per neighbour gives the blocks
 *   D(x, x+mu) = (+gamma_mu/2 - 1/2) U_mu(x),   D(x, x-mu) = (-gamma_mu/2 - 1/2) U_mu(x-mu)^dag,
 *   D(x, x) = 4 + m0,
 * with a factor -1 on a hop across the t boundary when tbc = 1.  The operator is applied from
 * these blocks; the adjoint by D^dag(x, y) = D(y, x)^dag, without the gamma5 trick.
 */

/* block D(x, x + s mu) (s = +1 or -1): spin matrix S and colour matrix M; returns the neighbour */
static long wilson_block(const int *L, int tbc, const cplx *U, long x, int mu, int s, cplx S[4][4], cplx M[9]) {
    const long V = vol(L);
    init_gammas();
    int c[4];
    coords(L, x, c);
    double sign = 1.0;
    if (s > 0) {
        memcpy(M, U + ((size_t)mu * V + x) * 9, sizeof(cplx) * 9);
        if (tbc && mu == 3 && c[3] == L[3] - 1) sign = -1.0;
        c[mu] += 1;
    } else {
        if (tbc && mu == 3 && c[3] == 0) sign = -1.0;
        c[mu] -= 1;
        const cplx *u = U + ((size_t)mu * V + site_of(L, c)) * 9;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) M[3 * a + b] = conj(u[3 * b + a]);
    }
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) S[a][b] = sign * (0.5 * s * GAM[mu][a][b] - (a == b ? 0.5 : 0.0));
    return site_of(L, c);
}

static void wilson_site(const int *L, int tbc, const cplx *U, double m0, const cplx *src, long x, int adj,
                        cplx *dst) {
    cplx acc[4][3];
    for (int s = 0; s < 4; ++s)
        for (int a = 0; a < 3; ++a) acc[s][a] = (4.0 + m0) * src[(size_t)x * 12 + 3 * s + a];
    for (int mu = 0; mu < 4; ++mu)
        for (int sg = -1; sg <= 1; sg += 2) {
            cplx S[4][4], M[9];
            long y;
            if (!adj) {
                y = wilson_block(L, tbc, U, x, mu, sg, S, M);
            } else {
                /* D^dag(x, y) = D(y, x)^dag with y = x + sg mu, i.e. the block of y towards -sg */
                int c[4];
                coords(L, x, c);
                c[mu] += sg;
                y = site_of(L, c);
                cplx S2[4][4], M2[9];
                wilson_block(L, tbc, U, y, mu, -sg, S2, M2);
                for (int a = 0; a < 4; ++a)
                    for (int b = 0; b < 4; ++b) S[a][b] = conj(S2[b][a]);
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) M[3 * a + b] = conj(M2[3 * b + a]);
            }
            const cplx *p = src + (size_t)y * 12;
            for (int s = 0; s < 4; ++s)
                for (int a = 0; a < 3; ++a) {
                    cplx v = 0;
                    for (int t = 0; t < 4; ++t)
                        for (int b = 0; b < 3; ++b) v += S[s][t] * M[3 * a + b] * p[3 * t + b];
                    acc[s][a] += v;
                }
        }
    for (int s = 0; s < 4; ++s)
        for (int a = 0; a < 3; ++a) dst[(size_t)x * 12 + 3 * s + a] = acc[s][a];
}

void orc_wilson(const int *L, int tbc, const cplx *U, double m0, const cplx *in, cplx *out, int nrhs) {
    const long V = vol(L);
    init_gammas();
    for (int r = 0; r < nrhs; ++r) {
#pragma omp parallel for schedule(static)
        for (long x = 0; x < V; ++x) wilson_site(L, tbc, U, m0, in + (size_t)r * V * 12, x, 0, out + (size_t)r * V * 12);
    }
}

void orc_wilson_adj(const int *L, int tbc, const cplx *U, double m0, const cplx *in, cplx *out, int nrhs) {
    const long V = vol(L);
    init_gammas();
    for (int r = 0; r < nrhs; ++r) {
#pragma omp parallel for schedule(static)
        for (long x = 0; x < V; ++x) wilson_site(L, tbc, U, m0, in + (size_t)r * V * 12, x, 1, out + (size_t)r * V * 12);
    }
}

void orc_wilson_dense(const int *L, int tbc, const cplx *U, double m0, cplx *M) {
    const long V = vol(L);
    const long n = 12 * V;
    memset(M, 0, sizeof(cplx) * (size_t)n * n);
    for (long x = 0; x < V; ++x) {
        for (int i = 0; i < 12; ++i) M[(size_t)(12 * x + i) * n + 12 * x + i] += 4.0 + m0;
        for (int mu = 0; mu < 4; ++mu)
            for (int sg = -1; sg <= 1; sg += 2) {
                cplx S[4][4], C[9];
                const long y = wilson_block(L, tbc, U, x, mu, sg, S, C);
                for (int s = 0; s < 4; ++s)
                    for (int a = 0; a < 3; ++a)
                        for (int t = 0; t < 4; ++t)
                            for (int b = 0; b < 3; ++b)
                                M[(size_t)(12 * x + 3 * s + a) * n + 12 * y + 3 * t + b] += S[s][t] * C[3 * a + b];
            }
    }
}

/* ------------------------------------------------------------------- clover */

/*
 * Clover term of eqs. (def_wils), (def_bril): -(c_SW/2) sum_{mu<nu} sigma_mu_nu F_mu_nu on the
 * diagonal.  The paper does not give the discretisation of F_mu_nu; used here (a reading):
 *   sigma_mu_nu = (i/2) [gamma_mu, gamma_nu],
 *   Q_mu_nu(x)  = the four plaquettes in the mu-nu plane that start and end at x, each taken
 *                 counter-clockwise (mu first, then nu),
 *   F_mu_nu(x)  = (Q_mu_nu - Q_mu_nu^dag) / (8 i), minus its trace / 3 (hermitian, traceless).
 * The gauge loops are closed, so the fermion boundary condition does not enter.
 * out[V][12][12], index 3*spin + colour.
 */
static void plaq_leaves(const int *L, const cplx *U, long x, int mu, int nu, cplx Q[9]) {
    const long V = vol(L);
    int c[4];
    coords(L, x, c);
    /* a leaf is a closed path of four steps (+-mu, +-nu), given by the signs of its first two steps */
    const int leaf[4][2] = {{+1, +1}, {+1, -1}, {-1, -1}, {-1, +1}};
    memset(Q, 0, sizeof(cplx) * 9);
    for (int l = 0; l < 4; ++l) {
        /* counter-clockwise in the (mu, nu) plane: steps a*mu, b*nu, -a*mu, -b*nu with a*b = +1, or
         * b*nu, a*mu, -b*nu, -a*mu with a*b = -1 */
        const int a = leaf[l][0], b = leaf[l][1];
        int dirs[4], sg[4];
        if (a * b > 0) {
            dirs[0] = mu; sg[0] = a; dirs[1] = nu; sg[1] = b; dirs[2] = mu; sg[2] = -a; dirs[3] = nu; sg[3] = -b;
        } else {
            dirs[0] = nu; sg[0] = b; dirs[1] = mu; sg[1] = a; dirs[2] = nu; sg[2] = -b; dirs[3] = mu; sg[3] = -a;
        }
        cplx M[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
        int y[4] = {c[0], c[1], c[2], c[3]};
        for (int st = 0; st < 4; ++st) {
            cplx T[9];
            const int d = dirs[st];
            if (sg[st] > 0) {
                mat_mul(M, U + ((size_t)d * V + site_of(L, y)) * 9, T);
                y[d] += 1;
            } else {
                y[d] -= 1;
                mat_mul_dag(M, U + ((size_t)d * V + site_of(L, y)) * 9, T);
            }
            memcpy(M, T, sizeof(T));
        }
        for (int e = 0; e < 9; ++e) Q[e] += M[e];
    }
}

void orc_clover(const int *L, const cplx *U, double csw, cplx *out) {
    const long V = vol(L);
    init_gammas();
    /* sigma_mu_nu = (i/2)(gamma_mu gamma_nu - gamma_nu gamma_mu) */
    cplx sig[4][4][4][4];
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = 0; nu < 4; ++nu)
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) {
                    cplx v = 0;
                    for (int k = 0; k < 4; ++k) v += GAM[mu][a][k] * GAM[nu][k][b] - GAM[nu][a][k] * GAM[mu][k][b];
                    sig[mu][nu][a][b] = 0.5 * _Complex_I * v;
                }
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x) {
        cplx *C = out + (size_t)x * 144;
        memset(C, 0, sizeof(cplx) * 144);
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                cplx Q[9], F[9];
                plaq_leaves(L, U, x, mu, nu, Q);
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) F[3 * i + j] = (Q[3 * i + j] - conj(Q[3 * j + i])) / (8.0 * _Complex_I);
                const cplx tr = (F[0] + F[4] + F[8]) / 3.0;
                for (int i = 0; i < 3; ++i) F[4 * i] -= tr;
                for (int s = 0; s < 4; ++s)
                    for (int t = 0; t < 4; ++t)
                        for (int i = 0; i < 3; ++i)
                            for (int j = 0; j < 3; ++j)
                                C[(3 * s + i) * 12 + 3 * t + j] += -0.5 * csw * sig[mu][nu][s][t] * F[3 * i + j];
            }
    }
}

/* out[x] += C(x) in[x] (adj: C(x)^dag in[x]) for nrhs right-hand sides */
void orc_clover_apply(const int *L, const cplx *Cf, const cplx *in, cplx *out, int nrhs, int adj) {
    const long V = vol(L);
    for (int r = 0; r < nrhs; ++r) {
#pragma omp parallel for schedule(static)
        for (long x = 0; x < V; ++x) {
            const cplx *C = Cf + (size_t)x * 144;
            const cplx *p = in + ((size_t)r * V + x) * 12;
            cplx *o = out + ((size_t)r * V + x) * 12;
            for (int i = 0; i < 12; ++i) {
                cplx v = 0;
                for (int j = 0; j < 12; ++j) v += (adj ? conj(C[j * 12 + i]) : C[i * 12 + j]) * p[j];
                o[i] += v;
            }
        }
    }
}

/* ------------------------------------------------------------------ solvers */

static cplx dotc(const cplx *a, const cplx *b, long n) {
    double re = 0, im = 0;
#pragma omp parallel for reduction(+ : re, im) schedule(static)
    for (long i = 0; i < n; ++i) {
        cplx v = conj(a[i]) * b[i];
        re += creal(v);
        im += cimag(v);
    }
    return re + _Complex_I * im;
}

static double norm2(const cplx *a, long n) { return creal(dotc(a, a, n)); }

/* The kernel operator of the solvers: kern 0 = Brillouin (W = the 81 links per site), kern 1 =
 * Wilson (W = the gauge field U, tbc applied on the fly). */
typedef struct {
    int kern, tbc;
    const cplx *W;
    const cplx *clov; /* clover field [V][12][12] or NULL */
} kernel_t;

static void kernel_apply(const int *L, const kernel_t *K, double m0, const cplx *x, cplx *y, int adj) {
    if (K->kern == 1) {
        if (adj)
            orc_wilson_adj(L, K->tbc, K->W, m0, x, y, 1);
        else
            orc_wilson(L, K->tbc, K->W, m0, x, y, 1);
    } else {
        if (adj)
            orc_dirac_adj(L, K->W, m0, x, y, 1);
        else
            orc_dirac(L, K->W, m0, x, y, 1);
    }
    if (K->clov) orc_clover_apply(L, K->clov, x, y, 1, adj);
}

/* y = (D^dag D + sigma) x */
static void normal_op(const int *L, const kernel_t *K, double m0, double sigma, const cplx *x, cplx *y, cplx *tmp) {
    const long n = 12 * vol(L);
    kernel_apply(L, K, m0, x, tmp, 0);
    kernel_apply(L, K, m0, tmp, y, 1);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) y[i] += sigma * x[i];
}

/* Textbook CG for (D^dag D + sigma) x = b, x0 = 0.  Iterates until the
 * recursive residual is below tol*|b|, then recomputes the true residual and
 * restarts from the current x if that is still above tol*|b|.
 * Returns the iteration count; *true_rel receives |b - (A+sigma)x|/|b|. */
int orc_cg(const int *L, int kern, int tbc, const cplx *W, const cplx *clov, double m0, double sigma,
           const cplx *b, cplx *x, double tol, int maxit, double *true_rel) {
    const long n = 12 * vol(L);
    const kernel_t Kv = {kern, tbc, W, clov};
    const kernel_t *K = &Kv;
    cplx *r = malloc(sizeof(cplx) * n), *p = malloc(sizeof(cplx) * n);
    cplx *Ap = malloc(sizeof(cplx) * n), *tmp = malloc(sizeof(cplx) * n);
    const double bn = sqrt(norm2(b, n));
    memset(x, 0, sizeof(cplx) * n);
    int it = 0;
    double rel = 1.0;
    if (bn == 0) {
        *true_rel = 0;
        free(r); free(p); free(Ap); free(tmp);
        return 0;
    }
    while (it < maxit) {
        /* (re)start: r = b - A x */
        normal_op(L, K, m0, sigma, x, Ap, tmp);
        for (long i = 0; i < n; ++i) r[i] = b[i] - Ap[i];
        double rr = norm2(r, n);
        rel = sqrt(rr) / bn;
        if (rel <= tol) break;
        memcpy(p, r, sizeof(cplx) * n);
        while (it < maxit) {
            normal_op(L, K, m0, sigma, p, Ap, tmp);
            double pAp = creal(dotc(p, Ap, n));
            double alpha = rr / pAp;
            for (long i = 0; i < n; ++i) {
                x[i] += alpha * p[i];
                r[i] -= alpha * Ap[i];
            }
            double rr_new = norm2(r, n);
            ++it;
            if (sqrt(rr_new) <= tol * bn) break;
            double beta = rr_new / rr;
            rr = rr_new;
            for (long i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        }
    }
    normal_op(L, K, m0, sigma, x, Ap, tmp);
    double rr = 0;
    for (long i = 0; i < n; ++i) {
        cplx e = b[i] - Ap[i];
        rr += creal(e) * creal(e) + cimag(e) * cimag(e);
    }
    *true_rel = sqrt(rr) / bn;
    free(r); free(p); free(Ap); free(tmp);
    return it;
}

/* y = c0 b + sum_i omega_i (D^dag D + sigma_i)^{-1} b, each shift separately.
 * iters[i], rel[i] receive the per-shift CG iteration count and true residual. */
int orc_rational(const int *L, int kern, int tbc, const cplx *W, const cplx *clov, double m0, int nshift, double c0,
                 const double *omega, const double *sigma, const cplx *b, cplx *y, double tol, int maxit, int *iters,
                 double *rel) {
    const long n = 12 * vol(L);
    cplx *xs = malloc(sizeof(cplx) * n);
    for (long i = 0; i < n; ++i) y[i] = c0 * b[i];
    int worst = 0;
    for (int s = 0; s < nshift; ++s) {
        iters[s] = orc_cg(L, kern, tbc, W, clov, m0, sigma[s], b, xs, tol, maxit, &rel[s]);
        if (rel[s] > tol) worst = 1;
        for (long i = 0; i < n; ++i) y[i] += omega[s] * xs[i];
    }
    free(xs);
    return worst;
}

/* ------------------------------------------------------------- link force */

/* Gell-Mann matrices lambda_1..lambda_8, written out from their definition */
static cplx LAM[8][3][3];
static int lam_ready = 0;

static void init_lambdas(void) {
    if (lam_ready) return;
    const cplx iu = _Complex_I;
    memset(LAM, 0, sizeof(LAM));
    LAM[0][0][1] = 1;   LAM[0][1][0] = 1;
    LAM[1][0][1] = -iu; LAM[1][1][0] = iu;
    LAM[2][0][0] = 1;   LAM[2][1][1] = -1;
    LAM[3][0][2] = 1;   LAM[3][2][0] = 1;
    LAM[4][0][2] = -iu; LAM[4][2][0] = iu;
    LAM[5][1][2] = 1;   LAM[5][2][1] = 1;
    LAM[6][1][2] = -iu; LAM[6][2][1] = iu;
    LAM[7][0][0] = 1.0 / sqrt(3.0);
    LAM[7][1][1] = 1.0 / sqrt(3.0);
    LAM[7][2][2] = -2.0 / sqrt(3.0);
    lam_ready = 1;
}

void orc_lambda(int a, cplx *out9) {
    init_lambdas();
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) out9[3 * i + k] = LAM[a][i][k];
}

/* Link force of S = Re sum_p w_p u_p^dag D v_p (D the Brillouin operator; the
 * 0-hop term does not depend on the links).  Sec. 9 takes the derivative with
 * respect to the Gell-Mann components of log U; here
 *   F[mu][z][a] = dS/d omega at omega = 0 for U_mu(z) -> exp(i omega lambda_a / 2) U_mu(z).
 * Each W_d(x) is the average over its k! paths of the ordered product of the
 * step matrices (orc_links); the product rule puts the perturbed step between
 * the product of the steps before it (P) and of those after it (Q):
 *   a +mu step from z carries U = U_mu(z),       dU   = X U,
 *   a -mu step onto z carries U_mu(z)^dag,       dU^dag = -U^dag X,
 * with X = i lambda_a / 2 (anti-hermitian).  With
 *   M_ab = sum_p w_p sum_{s,t} conj(u_p(x)_{s a}) (S_d)_{s t} v_p(x+d)_{t b},
 * a step contributes Re sum_ab M_ab (P dT Q)_ab = Re tr(Q M^T P dT).
 * Layouts: U [4][V][3][3]; u, v [npairs][V][4][3]; F [4][V][8]. */
void orc_link_force(const int *L, int tbc, const cplx *U, int npairs, const double *w, const cplx *u,
                    const cplx *v, double *F) {
    const long V = vol(L);
    init_perms();
    init_lambdas();
    cplx S[81][4][4];
    for (int j = 0; j < 81; ++j) spin_matrix(j, 0.0, S[j]);
    int nthr = orc_num_threads();
    double *part = calloc((size_t)nthr * 4 * V * 8, sizeof(double));
#pragma omp parallel
    {
#ifdef _OPENMP
        double *Fl = part + (size_t)omp_get_thread_num() * 4 * V * 8;
#else
        double *Fl = part;
#endif
#pragma omp for schedule(dynamic, 1)
        for (long x = 0; x < V; ++x) {
            int cx[4];
            coords(L, x, cx);
            for (int j = 0; j < 81; ++j) {
                if (j == 40) continue;
                int d[4];
                disp_of(j, d);
                int cy[4];
                for (int mu = 0; mu < 4; ++mu) cy[mu] = cx[mu] + d[mu];
                const long y = site_of(L, cy);
                /* M (colour 3x3) */
                cplx M[9] = {0};
                for (int p = 0; p < npairs; ++p) {
                    const cplx *up = u + ((size_t)p * V + x) * 12;
                    const cplx *vp = v + ((size_t)p * V + y) * 12;
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) {
                            cplx acc = 0;
                            for (int s = 0; s < 4; ++s)
                                for (int t = 0; t < 4; ++t) acc += conj(up[3 * s + a]) * S[j][s][t] * vp[3 * t + b];
                            M[3 * a + b] += w[p] * acc;
                        }
                }
                int nonzero = 0;
                for (int e = 0; e < 9; ++e) nonzero |= (M[e] != 0);
                if (!nonzero) continue; /* this (x, d) term does not enter S */
                cplx MT[9];
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) MT[3 * a + b] = M[3 * b + a];
                int axes[4], k = 0;
                for (int mu = 0; mu < 4; ++mu)
                    if (d[mu] != 0) axes[k++] = mu;
                const int np_local = NPERM[k];
                for (int pth = 0; pth < np_local; ++pth) {
                    /* the steps of this path */
                    cplx T[4][9];
                    int smu[4], plus[4];
                    long lsite[4];
                    double sign = 1.0;
                    int cz[4] = {cx[0], cx[1], cx[2], cx[3]};
                    for (int st = 0; st < k; ++st) {
                        const int mu = axes[PERM[k][pth][st]];
                        smu[st] = mu;
                        if (d[mu] > 0) {
                            if (tbc && mu == 3 && ((cz[3] % L[3]) + L[3]) % L[3] == L[3] - 1) sign = -sign;
                            lsite[st] = site_of(L, cz);
                            memcpy(T[st], U + ((size_t)mu * V + lsite[st]) * 9, sizeof(cplx) * 9);
                            plus[st] = 1;
                            cz[mu] += 1;
                        } else {
                            if (tbc && mu == 3 && ((cz[3] % L[3]) + L[3]) % L[3] == 0) sign = -sign;
                            cz[mu] -= 1;
                            lsite[st] = site_of(L, cz);
                            const cplx *Um = U + ((size_t)mu * V + lsite[st]) * 9;
                            for (int a = 0; a < 3; ++a)
                                for (int b = 0; b < 3; ++b) T[st][3 * a + b] = conj(Um[3 * b + a]);
                            plus[st] = 0;
                        }
                    }
                    /* prefix P[i] = T_0 ... T_{i-1}, suffix Q[i] = T_i ... T_{k-1} */
                    cplx P[5][9], Q[5][9];
                    const cplx I3[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
                    memcpy(P[0], I3, sizeof(I3));
                    for (int i = 0; i < k; ++i) mat_mul(P[i], T[i], P[i + 1]);
                    memcpy(Q[k], I3, sizeof(I3));
                    for (int i = k - 1; i >= 0; --i) mat_mul(T[i], Q[i + 1], Q[i]);
                    const double f = sign / (double)np_local;
                    for (int i = 0; i < k; ++i) {
                        cplx R[9], t1[9], Y[9];
                        mat_mul(Q[i + 1], MT, t1);
                        mat_mul(t1, P[i], R);
                        const cplx *Ul = U + ((size_t)smu[i] * V + lsite[i]) * 9;
                        if (plus[i]) {
                            mat_mul(Ul, R, Y); /* Re tr(R X U) = Re tr(U R X) */
                        } else {
                            mat_mul_dag(R, Ul, t1); /* -Re tr(R U^dag X) */
                            for (int e = 0; e < 9; ++e) Y[e] = -t1[e];
                        }
                        double *Fz = Fl + ((size_t)smu[i] * V + lsite[i]) * 8;
                        for (int a = 0; a < 8; ++a) {
                            cplx tr = 0;
                            for (int r = 0; r < 3; ++r)
                                for (int c = 0; c < 3; ++c) tr += Y[3 * r + c] * LAM[a][c][r];
                            /* Re tr(Y i lambda / 2) */
                            Fz[a] += f * creal(0.5 * _Complex_I * tr);
                        }
                    }
                }
            }
        }
    }
    memset(F, 0, sizeof(double) * 4 * V * 8);
    for (int t = 0; t < nthr; ++t)
        for (long e = 0; e < 4 * V * 8; ++e) F[e] += part[(size_t)t * 4 * V * 8 + e];
    free(part);
}

/*
 * Link force of S = Re sum_p w_p u_p^dag D_wil v_p (Sec. 9 convention: U_mu(z) -> exp(i omega^a
 * lambda_a / 2) U_mu(z), F^a = dS/d omega^a at 0).  U_mu(z) enters two blocks: the forward hop
 * D(z, z+mu) = S_+ (s U_mu(z)), whose colour matrix changes by i (lambda_a/2) M, and the backward
 * hop D(z+mu, z) = S_- (s U_mu(z)^dag), whose colour matrix changes by -i M (lambda_a/2).
 * F[mu][z][a]; u, v [npairs][V][4][3].
 */
void orc_wilson_force(const int *L, int tbc, const cplx *U, int npairs, const double *w, const cplx *u,
                      const cplx *v, double *F) {
    const long V = vol(L);
    init_gammas();
    init_lambdas();
#pragma omp parallel for schedule(static)
    for (long z = 0; z < V; ++z) {
        for (int mu = 0; mu < 4; ++mu) {
            cplx Sf[4][4], Mf[9], Sb[4][4], Mb[9];
            const long zp = wilson_block(L, tbc, U, z, mu, +1, Sf, Mf);
            wilson_block(L, tbc, U, zp, mu, -1, Sb, Mb);
            for (int a = 0; a < 8; ++a) {
                /* dMf = i (lambda/2) Mf ; dMb = -i Mb (lambda/2) */
                cplx dMf[9], dMb[9];
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) {
                        cplx sf = 0, sb = 0;
                        for (int k = 0; k < 3; ++k) {
                            sf += LAM[a][i][k] * Mf[3 * k + j];
                            sb += Mb[3 * i + k] * LAM[a][k][j];
                        }
                        dMf[3 * i + j] = 0.5 * _Complex_I * sf;
                        dMb[3 * i + j] = -0.5 * _Complex_I * sb;
                    }
                double acc = 0.0;
                for (int p = 0; p < npairs; ++p) {
                    const cplx *up = u + (size_t)p * V * 12, *vp = v + (size_t)p * V * 12;
                    cplx sum = 0;
                    for (int s = 0; s < 4; ++s)
                        for (int t = 0; t < 4; ++t)
                            for (int i = 0; i < 3; ++i)
                                for (int j = 0; j < 3; ++j) {
                                    sum += conj(up[z * 12 + 3 * s + i]) * Sf[s][t] * dMf[3 * i + j] * vp[zp * 12 + 3 * t + j];
                                    sum += conj(up[zp * 12 + 3 * s + i]) * Sb[s][t] * dMb[3 * i + j] * vp[z * 12 + 3 * t + j];
                                }
                    acc += w[p] * creal(sum);
                }
                F[((size_t)mu * V + z) * 8 + a] = acc;
            }
        }
    }
}
