// Link force of S = Re sum_p w_p u_p^dag D_bri v_p, and of S = Re chi^dag D_ov psi.
//
// Convention: U_mu(x) -> exp(i omega^a lambda_a / 2) U_mu(x), F^a_mu(x) = dS/d omega^a at 0.
// For any complex matrix M entering S write dS = Re tr(G_M^T dM) (plain transpose);
// G_M is "the coefficient of M".  Then
//   * D_bri(x, x+d) = S_d (x) W_d(x) with S_d = a_k + c_k sum d_mu gamma_mu Hermitian, so
//     G_{W_d}(x) = sum_p w_p sum_t conj((S_d u_p(x))_t) v_p(x+d)_t^T      (colour outer product)
//     for every displacement d != 0 (App. C.1 stencil);
//   * W_d(x) = (1/k) sum_mu T_mu(x) W_r(x + s_mu e_mu), r = d - s_mu e_mu (the k-hop recursion of
//     the path average): a product M = A X B gives G_X = A^T G_M B^T, so
//       G_T  += (1/k) G_W W_r^T,      G_{W_r} += (1/k) T^T G_W,
//     and a daggered matrix M = Y^dag gives G_Y = G_M^dag;
//   * T = U_mu(x) for a + step, U_mu(x - e_mu)^dag for a - step (times -1 across the t boundary
//     when the fermions are antiperiodic);
//   * F^a = Re tr(G_U^T (i lambda_a / 2) U) = -Im tr(lambda_a U G_U^T) / 2.
// The pull-back through the recursion runs level by level from 4 hops down to 1 in gather form:
// each level-(k-1) entry G_r(y) collects from its parents d = r + s e_mu (mu not in supp r,
// s = +-1) at x = y - s e_mu, so no two threads write the same entry.
//
// Overlap: with X = D_bri(-rho), A = X^dag X, a_i = (A + sigma_i)^{-1} psi,
// b_i = (A + sigma_i)^{-1} X^dag chi and y = c0 psi + sum omega_i a_i,
//   dS = rho Re[chi^dag dX y] - rho sum_i omega_i Re[(X a_i)^dag dX b_i + (X b_i)^dag dX a_i],
// i.e. 1 + 2n pairs of the form above (differentiating the partial fractions of eq.
// (KLnn_parfrac) inside eq. (def_over)), and the spinor gradient is
//   dS/d psi = D_ov^dag chi = rho (chi + c0 X^dag chi + sum_i omega_i b_i).
#include <chrono>
#include <cstring>
#include <vector>

#include "stencil.hpp"
#include "stencil_core.hpp"

namespace bri {

// Multi-shift solve of (A + sigma_i) x = b over the Kenney-Laub shifts, every x kept in FP64
// ([shift][ncol][12 V] in the workspace); with work == NULL only *need is set (solver.hip).
int ov_solve_shifts(const Geom &g, const void *W64, const void *Wlo, const ov_params *prm, const void *b, int ncol,
                    void *work, size_t work_bytes, size_t *need, hipStream_t s, void **x_out, ov_stats *st,
                    int i0 = -1, int i1 = -1);
// the rational of `prm` (diagonal or upper-diagonal coefficients, per-shift tolerance factors) and
// the validity check of its fields (solver.hip)
void shift_coeffs(const ov_params *prm, double *c0, double *omega, double *sigma, double *tolf);
bool params_ok(const ov_params *prm);

__device__ __forceinline__ int dj(int j, int mu) { return disp_comp(j, mu); }

__device__ __forceinline__ unsigned site_of(const Geom &g, const int c[4]) {
    return (unsigned)(c[0] + g.L[0] * (c[1] + g.L[1] * (c[2] + g.L[2] * c[3])));
}

__device__ __forceinline__ int wrapc(int v, int L) { return v < 0 ? v + L : (v >= L ? v - L : v); }

// W_d(y) for any displacement index j (stored, daggered partner, or the identity)
__device__ void link_any(const Geom &g, const double2 *__restrict__ W, int j, const int cy[4], double2 M[3][3]) {
    const size_t V = (size_t)g.V;
    if (j == 40) {
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) M[a][b] = make_double2(a == b ? 1.0 : 0.0, 0.0);
        return;
    }
    if (j < 40) {
        const unsigned ys = site_of(g, cy);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) M[a][b] = W[((size_t)j * 9 + a * 3 + b) * V + ys];
        return;
    }
    int cz[4];
    for (int mu = 0; mu < 4; ++mu) cz[mu] = wrapc(cy[mu] + dj(j, mu), g.L[mu]);
    const unsigned zs = site_of(g, cz);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            const double2 w = W[((size_t)(80 - j) * 9 + b * 3 + a) * V + zs];
            M[a][b] = make_double2(w.x, -w.y);
        }
}

// T_mu^{s}(x) (with the antiperiodic sign) for the first step of a path from x
__device__ void first_step(const Geom &g, const double2 *__restrict__ U, int mu, int s, const int cx[4],
                           double2 T[3][3]) {
    const size_t V = (size_t)g.V;
    if (s > 0) {
        const unsigned xs = site_of(g, cx);
        const double sg = (g.tbc && mu == 3 && cx[3] == g.L[3] - 1) ? -1.0 : 1.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                const double2 u = U[((size_t)(mu * 3 + a) * 3 + b) * V + xs];
                T[a][b] = make_double2(sg * u.x, sg * u.y);
            }
    } else {
        int cm[4] = {cx[0], cx[1], cx[2], cx[3]};
        cm[mu] = wrapc(cm[mu] - 1, g.L[mu]);
        const unsigned ms = site_of(g, cm);
        const double sg = (g.tbc && mu == 3 && cx[3] == 0) ? -1.0 : 1.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                const double2 u = U[((size_t)(mu * 3 + b) * 3 + a) * V + ms];
                T[a][b] = make_double2(sg * u.x, -sg * u.y);
            }
    }
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// ------------------------------------------------------------ outer products

struct PairTable {
    const double2 *u[BRI_MAX_PAIRS];
    const double2 *v[BRI_MAX_PAIRS];
    double w[BRI_MAX_PAIRS];
    int n;
    int accumulate;  // add to G instead of overwriting it
};

// G[j][a][b](x) = sum_p w_p sum_t conj((S_d u_p(x))_{t,a}) v_p(x+d)_{t,b}, all d != 0.
// A workgroup owns 64 consecutive sites and 8 of the 80 displacements (the block index modulo
// the group count picks which 8, so the ten groups of a tile are dispatched side by side);
// each wave keeps the 3x3 accumulators of 2 displacements in registers while the pairs stream
// through, so u_p(x) and the neighbourhood of v_p are read while hot in L2 (a pass per
// displacement would stream every pair from HBM 80 times).
// The Wilson operator has only the 8 one-hop displacements (one group), with its own weights.
constexpr int OUTER_WAVES = 4;
constexpr int OUTER_PER_WAVE = 2;
template <int KIND> struct OuterDisp {
    static constexpr int n = KIND == KERN_WIL ? 8 : 80;
    static constexpr int groups = n / (OUTER_WAVES * OUTER_PER_WAVE);
    // displacement index of the jj-th displacement (the centre j = 40 is skipped)
    __device__ __forceinline__ static int at(int jj) {
        if constexpr (KIND == KERN_WIL) {
            const int half = jj < 4 ? jj : 7 - jj;  // 13, 31, 37, 39 and their opposites 67, 49, 43, 41
            const int j = 40 - (half == 0 ? 27 : half == 1 ? 9 : half == 2 ? 3 : 1);
            return jj < 4 ? j : 80 - j;
        }
        return jj < 40 ? jj : jj + 1;
    }
};

template <int KIND>
__global__ __launch_bounds__(64 * OUTER_WAVES) void grad_outer_kernel(Geom g, PairTable pt,
                                                                      double2 *__restrict__ G) {
    constexpr int GROUPS = OuterDisp<KIND>::groups;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const unsigned grp = blockIdx.x % GROUPS;
    const unsigned x = (blockIdx.x / GROUPS) * 64 + lane;
    const bool live = x < (unsigned)g.V;
    const size_t V = (size_t)g.V;
    const int jbase = (grp * OUTER_WAVES + w) * OUTER_PER_WAVE;
    int cx[4];
    {
        int s = live ? (int)x : 0;
        for (int mu = 0; mu < 4; ++mu) {
            cx[mu] = s % g.L[mu];
            s /= g.L[mu];
        }
    }
    unsigned ys[OUTER_PER_WAVE];
#pragma unroll
    for (int i = 0; i < OUTER_PER_WAVE; ++i) {
        const int j = OuterDisp<KIND>::at(jbase + i);
        int cy[4];
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) cy[mu] = wrapc(cx[mu] + dj(j, mu), g.L[mu]);
        ys[i] = site_of(g, cy);
    }
    double2 acc[OUTER_PER_WAVE][3][3];
#pragma unroll
    for (int i = 0; i < OUTER_PER_WAVE; ++i)
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) acc[i][a][b] = make_double2(0.0, 0.0);
    if (!live) return;
    for (int p = 0; p < pt.n; ++p) {
        const double2 *__restrict__ up = pt.u[p];
        const double2 *__restrict__ vp = pt.v[p];
        const double wp = pt.w[p];
        double2 u[4][3];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double2 t = up[(size_t)(s * 3 + c) * V + x];
                u[s][c] = make_double2(wp * t.x, wp * t.y);
            }
#pragma unroll
        for (int i = 0; i < OUTER_PER_WAVE; ++i) {
            const DirW<double, false, KIND> dw(OuterDisp<KIND>::at(jbase + i));  // S_d of the kernel
            double2 e[4][3];
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int c = 0; c < 3; ++c) e[s][c] = make_double2(0.0, 0.0);
            spin_accumulate(e, u, dw.a, dw.c0, dw.c1, dw.c2, dw.c3);  // e = w_p S_d u
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int bb = 0; bb < 3; ++bb) {
                    const double2 v = vp[(size_t)(t * 3 + bb) * V + ys[i]];
#pragma unroll
                    for (int aa = 0; aa < 3; ++aa) {
                        // acc += conj(e) v
                        acc[i][aa][bb].x += e[t][aa].x * v.x + e[t][aa].y * v.y;
                        acc[i][aa][bb].y += e[t][aa].x * v.y - e[t][aa].y * v.x;
                    }
                }
            // keep the scheduler from hoisting the next displacement's loads above this one
            __builtin_amdgcn_sched_barrier(0);
        }
    }
#pragma unroll
    for (int i = 0; i < OUTER_PER_WAVE; ++i) {
        const int j = OuterDisp<KIND>::at(jbase + i);
#pragma unroll
        for (int aa = 0; aa < 3; ++aa)
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) {
                double2 *gp = G + ((size_t)j * 9 + aa * 3 + bb) * V + x;
                if (pt.accumulate) {
                    const double2 o = *gp;
                    *gp = make_double2(o.x + acc[i][aa][bb].x, o.y + acc[i][aa][bb].y);
                } else {
                    *gp = acc[i][aa][bb];
                }
            }
    }
}

// Displacement indices with a given number of hops (8, 24, 32 or 16 of them).
struct HopDirs {
    int n;
    int j[32];
};

// Level k -> k-1 in gather form: G_r(y) += (1/k) T^T G_d(x), d = r + s e_mu, x = y - s e_mu;
// one thread per (site, (k-1)-hop displacement r).  r is the fastest-varying part of the block
// index, so the children of one parent entry run together and share its L2 line.
__global__ __launch_bounds__(128) void grad_level_kernel(Geom g, const double2 *__restrict__ U, double2 *__restrict__ G,
                                                         int k, HopDirs lower) {
    const unsigned y = (blockIdx.x / lower.n) * blockDim.x + threadIdx.x;
    if (y >= (unsigned)g.V) return;
    const size_t V = (size_t)g.V;
    int cy[4];
    {
        int s = (int)y;
        for (int mu = 0; mu < 4; ++mu) {
            cy[mu] = s % g.L[mu];
            s /= g.L[mu];
        }
    }
    const double invk = 1.0 / (double)k;
    {
        const int jr = lower.j[blockIdx.x % lower.n];
        int r[4];
        for (int mu = 0; mu < 4; ++mu) r[mu] = dj(jr, mu);
        double2 acc[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) acc[a][b] = G[((size_t)jr * 9 + a * 3 + b) * V + y];
        for (int mu = 0; mu < 4; ++mu) {
            if (r[mu] != 0) continue;
            for (int s = -1; s <= 1; s += 2) {
                int cx[4] = {cy[0], cy[1], cy[2], cy[3]};
                cx[mu] = wrapc(cx[mu] - s, g.L[mu]);
                const int jd = jr + s * (mu == 0 ? 1 : mu == 1 ? 3 : mu == 2 ? 9 : 27);
                double2 T[3][3];
                first_step(g, U, mu, s, cx, T);
                const unsigned xs = site_of(g, cx);
                double2 Gd[3][3];
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) Gd[a][b] = G[((size_t)jd * 9 + a * 3 + b) * V + xs];
                // acc += (1/k) T^T Gd
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) {
                        double2 t = make_double2(0.0, 0.0);
                        for (int c = 0; c < 3; ++c) {
                            const double2 m = cmul(T[c][a], Gd[c][b]);
                            t.x += m.x;
                            t.y += m.y;
                        }
                        acc[a][b].x += invk * t.x;
                        acc[a][b].y += invk * t.y;
                    }
            }
        }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) G[((size_t)jr * 9 + a * 3 + b) * V + y] = acc[a][b];
    }
}

// G_U_mu(z) from every level's first step, then F^a_mu(z) = -Im tr(lambda_a U G_U^T) / 2
// (kind = KERN_WIL: only the one-hop displacements carry a coefficient, and their remainder link
// is the identity)
__global__ __launch_bounds__(128) void grad_force_kernel(Geom g, const double2 *__restrict__ U,
                                                         const double2 *__restrict__ W, const double2 *__restrict__ G,
                                                         double *__restrict__ F, double2 *__restrict__ GUo, int kind) {
    const unsigned z = (blockIdx.x >> 2) * blockDim.x + threadIdx.x;
    if (z >= (unsigned)g.V) return;
    const size_t V = (size_t)g.V;
    int cz[4];
    {
        int s = (int)z;
        for (int mu = 0; mu < 4; ++mu) {
            cz[mu] = s % g.L[mu];
            s /= g.L[mu];
        }
    }
    {
        const int mu = blockIdx.x & 3;  // one thread per (site, link direction); mu varies fastest
        double2 GU[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) GU[a][b] = make_double2(0.0, 0.0);
        const int emu = mu == 0 ? 1 : mu == 1 ? 3 : mu == 2 ? 9 : 27;
        int cp[4] = {cz[0], cz[1], cz[2], cz[3]};
        cp[mu] = wrapc(cp[mu] + 1, g.L[mu]);
        const unsigned ps = site_of(g, cp);
        // + step at z: T = sg U_mu(z); G_T = (1/k) G_d(z) W_{d - e_mu}(z + e_mu)^T, G_U += sg G_T
        const double sgp = (g.tbc && mu == 3 && cz[3] == g.L[3] - 1) ? -1.0 : 1.0;
        // - step at z + e_mu: T = sg U_mu(z)^dag; G_T = (1/k) G_d(z+e) W_{d + e_mu}(z)^T, G_U += sg G_T^dag
        const double sgm = (g.tbc && mu == 3 && cp[3] == 0) ? -1.0 : 1.0;
        for (int jd = 0; jd < 81; ++jd) {
            const int dmu = dj(jd, mu);
            if (dmu == 0) continue;
            int k = 0;
            for (int nu = 0; nu < 4; ++nu) k += dj(jd, nu) != 0;
            if (kind == KERN_WIL && k != 1) continue;
            const double invk = 1.0 / (double)k;
            double2 Gd[3][3], Wr[3][3];
            if (dmu > 0) {
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) Gd[a][b] = G[((size_t)jd * 9 + a * 3 + b) * V + z];
                link_any(g, W, jd - emu, cp, Wr);
            } else {
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) Gd[a][b] = G[((size_t)jd * 9 + a * 3 + b) * V + ps];
                link_any(g, W, jd + emu, cz, Wr);
            }
            // GT = Gd Wr^T
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    double2 t = make_double2(0.0, 0.0);
                    for (int c = 0; c < 3; ++c) {
                        const double2 m = cmul(Gd[a][c], Wr[b][c]);
                        t.x += m.x;
                        t.y += m.y;
                    }
                    if (dmu > 0) {
                        GU[a][b].x += sgp * invk * t.x;
                        GU[a][b].y += sgp * invk * t.y;
                    } else {  // dagger: G_U[b][a] += conj(t)
                        GU[b][a].x += sgm * invk * t.x;
                        GU[b][a].y -= sgm * invk * t.y;
                    }
                }
        }
        // P = U G_U^T ; F^a = -Im tr(lambda_a P) / 2
        double2 Um[3][3], P[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) Um[a][b] = U[((size_t)(mu * 3 + a) * 3 + b) * V + z];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double2 t = make_double2(0.0, 0.0);
                for (int c = 0; c < 3; ++c) {
                    const double2 m = cmul(Um[a][c], GU[b][c]);
                    t.x += m.x;
                    t.y += m.y;
                }
                P[a][b] = t;
            }
        // tr(lambda_a P) = sum_{ij} (lambda_a)_{ij} P_{ji}; F^a = -Im tr(lambda_a P) / 2
        const double s3 = 0.57735026918962576451;  // 1/sqrt(3)
        // only the imaginary parts are needed: lambda_{1,4,6} are real symmetric, lambda_{2,5,7}
        // carry -i above and +i below the diagonal, so tr(lambda P) = i (P_ij - P_ji) for them
        double im[8];
        im[0] = P[1][0].y + P[0][1].y;
        im[1] = P[0][1].x - P[1][0].x;
        im[2] = P[0][0].y - P[1][1].y;
        im[3] = P[2][0].y + P[0][2].y;
        im[4] = P[0][2].x - P[2][0].x;
        im[5] = P[2][1].y + P[1][2].y;
        im[6] = P[1][2].x - P[2][1].x;
        im[7] = s3 * (P[0][0].y + P[1][1].y - 2.0 * P[2][2].y);
        if (F)
            for (int a = 0; a < 8; ++a) F[((size_t)mu * 8 + a) * V + z] = -0.5 * im[a];
        if (GUo)  // torch's complex gradient dS/dRe U + i dS/dIm U = conj(G_U)
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    GUo[((size_t)(mu * 3 + a) * 3 + b) * V + z] = make_double2(GU[a][b].x, -GU[a][b].y);
    }
}

// ---------------------------------------------------------------- helpers

// out = alpha x + beta y + gam sum_k omega_k z_k  (one FP64 column; z_k at stride zstride)
__global__ void grad_combine_kernel(size_t n, double alpha, const double2 *__restrict__ x, double beta,
                                    const double2 *__restrict__ y, double gam, int nz,
                                    const double *__restrict__ omega, const double2 *__restrict__ z, size_t zstride,
                                    double2 *__restrict__ out) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        double2 v = make_double2(alpha * x[i].x, alpha * x[i].y);
        if (y) {
            v.x += beta * y[i].x;
            v.y += beta * y[i].y;
        }
        double2 t = make_double2(0.0, 0.0);
        for (int k = 0; k < nz; ++k) {
            const double2 zv = z[(size_t)k * zstride + i];
            t.x += omega[k] * zv.x;
            t.y += omega[k] * zv.y;
        }
        v.x += gam * t.x;
        v.y += gam * t.y;
        out[i] = v;
    }
}

static inline size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

// G buffer [81][9][V] complex double
static size_t grad_g_bytes(const Geom &g) { return al256((size_t)81 * 9 * g.V * sizeof(double2)); }

// G (=, or += with pt.accumulate) the outer products of the pairs of pt
static void outer_pairs(const Geom &g, const PairTable &pt, double2 *G, hipStream_t s, int kind) {
    const int tiles = (g.V + 63) / 64;
    if (kind == KERN_WIL)
        hipLaunchKernelGGL(grad_outer_kernel<KERN_WIL>, dim3(OuterDisp<KERN_WIL>::groups * tiles),
                           dim3(64 * OUTER_WAVES), 0, s, g, pt, G);
    else
        hipLaunchKernelGGL(grad_outer_kernel<KERN_BRI>, dim3(OuterDisp<KERN_BRI>::groups * tiles),
                           dim3(64 * OUTER_WAVES), 0, s, g, pt, G);
}

// pull-back of the accumulated G through the path average (Brillouin kernel) and the force
static int force_from_outer(const Geom &g, const double2 *U, const double2 *W, double2 *G, double *F, double2 *GU,
                            hipStream_t s, int kind) {
    const int threads = 128;
    const int blocks = (g.V + threads - 1) / threads;
    if (kind == KERN_WIL) {
        // one-hop displacements only: no pull-back through the path average
        hipLaunchKernelGGL(grad_force_kernel, dim3(4 * blocks), dim3(threads), 0, s, g, U, W, G, F, GU, kind);
        return hipGetLastError() == hipSuccess ? BRI_OK : BRI_EHIP;
    }
    for (int k = 4; k >= 2; --k) {
        HopDirs lower{};
        for (int j = 0; j < 81; ++j) {
            int nh = 0;
            for (int r = j, mu = 0; mu < 4; ++mu, r /= 3) nh += (r % 3) != 1;
            if (nh == k - 1) lower.j[lower.n++] = j;
        }
        hipLaunchKernelGGL(grad_level_kernel, dim3(lower.n * blocks), dim3(threads), 0, s, g, U, G, k, lower);
    }
    hipLaunchKernelGGL(grad_force_kernel, dim3(4 * blocks), dim3(threads), 0, s, g, U, W, G, F, GU, kind);
    return hipGetLastError() == hipSuccess ? BRI_OK : BRI_EHIP;
}

static int force_from_pairs(const Geom &g, const double2 *U, const double2 *W, const PairTable &pt, double2 *G,
                            double *F, double2 *GU, hipStream_t s, int kind) {
    outer_pairs(g, pt, G, s, kind);
    return force_from_outer(g, U, W, G, F, GU, s, kind);
}

// workspace of ov_apply_grad, carved in this order
struct GradPlan {
    size_t g_off, xab_off, bin_off, y_off, om_off, solver_off, bytes, solver_bytes;
};

// shifts per solve of the gradient: all of them, or recompute at a time
static int grad_chunk(const ov_params *prm) {
    return prm->recompute > 0 && prm->recompute < prm->kl_n ? prm->recompute : prm->kl_n;
}

static int plan_grad(const Geom &g, const ov_params *prm, GradPlan &pl) {
    const size_t nel = (size_t)12 * g.V;
    const size_t vb = al256(nel * sizeof(double2));
    const int m = grad_chunk(prm);
    size_t solver_need = 0;
    void *xdummy = nullptr;
    const int rc = ov_solve_shifts(g, nullptr, nullptr, prm, nullptr, 2, nullptr, 0, &solver_need, nullptr, &xdummy,
                                   nullptr, 0, m);
    if (rc != BRI_OK) return rc;
    size_t off = 0;
    pl.g_off = off;
    off += grad_g_bytes(g);
    pl.xab_off = off;  // X applied to the 2m shift solutions of one solve
    off += vb * 2 * m;
    pl.bin_off = off;  // [psi | X^dag chi]
    off += vb * 2;
    pl.y_off = off;
    off += vb;
    pl.om_off = off;
    off += al256(sizeof(double) * MAXS);
    pl.solver_off = off;
    pl.solver_bytes = solver_need;
    off += solver_need;
    pl.bytes = off;
    return BRI_OK;
}

}  // namespace bri

extern "C" {

static int link_grad_impl(const bri_geom *geom, const void *U, const void *W, int npairs, const double *weights,
                          const void *u, const void *v, void *F, void *GU, void *work, size_t *work_bytes,
                          void *stream, int kind) {
    using namespace bri;
    Geom g;
    int rc = geom_check(geom, &g);
    if (rc != BRI_OK) return rc;
    if (g.csw != 0.0) return BRI_EINVAL;  // the clover term's derivative is not built
    if (!work_bytes || npairs < 1 || npairs > BRI_MAX_PAIRS) return BRI_EINVAL;
    const size_t need = grad_g_bytes(g);
    if (!work) {
        *work_bytes = need;
        return BRI_OK;
    }
    if (*work_bytes < need || !U || !W || !weights || !u || !v || (!F && !GU)) return BRI_EINVAL;
    {
        // the outputs and the workspace must not alias each other or any input
        const size_t V = (size_t)g.V, sp = (size_t)npairs * 192 * V;
        const void *ins[4] = {U, W, u, v};
        const size_t inb[4] = {576 * V, 5760 * V, sp, sp};
        const void *outs[3] = {F, GU, work};
        const size_t outb[3] = {256 * V, 576 * V, need};
        for (int i = 0; i < 3; ++i) {
            if (!outs[i]) continue;
            for (int k = 0; k < 4; ++k)
                if (ranges_overlap(outs[i], outb[i], ins[k], inb[k])) return BRI_EINVAL;
            for (int k = i + 1; k < 3; ++k)
                if (outs[k] && ranges_overlap(outs[i], outb[i], outs[k], outb[k])) return BRI_EINVAL;
        }
    }
    PairTable pt;
    std::memset(&pt, 0, sizeof(pt));
    pt.n = npairs;
    const size_t nel = (size_t)12 * g.V;
    for (int p = 0; p < npairs; ++p) {
        pt.u[p] = (const double2 *)u + p * nel;
        pt.v[p] = (const double2 *)v + p * nel;
        pt.w[p] = weights[p];
    }
    return force_from_pairs(g, (const double2 *)U, (const double2 *)W, pt, (double2 *)work, (double *)F,
                            (double2 *)GU, (hipStream_t)stream, kind);
}

int bri_link_grad(const bri_geom *geom, const void *U, const void *W, int npairs, const double *weights,
                  const void *u, const void *v, void *F, void *GU, void *work, size_t *work_bytes, void *stream) {
    return link_grad_impl(geom, U, W, npairs, weights, u, v, F, GU, work, work_bytes, stream, bri::KERN_BRI);
}

int wil_link_grad(const bri_geom *geom, const void *U, const void *W, int npairs, const double *weights,
                  const void *u, const void *v, void *F, void *GU, void *work, size_t *work_bytes, void *stream) {
    return link_grad_impl(geom, U, W, npairs, weights, u, v, F, GU, work, work_bytes, stream, bri::KERN_WIL);
}

int ov_apply_grad(const bri_geom *geom, const void *U, const void *W64, const void *Wlo, const ov_params *prm,
                  const void *chi, const void *psi, void *F, void *GU, void *gpsi, void *work, size_t *work_bytes,
                  ov_stats *stats, void *stream) {
    using namespace bri;
    const auto t0 = std::chrono::steady_clock::now();
    Geom g;
    int rc = geom_check(geom, &g);
    if (rc != BRI_OK) return rc;
    if (!prm || !work_bytes || g.csw != 0.0) return BRI_EINVAL;
    const int n = prm->kl_n;
    if (!params_ok(prm) || prm->relax == 2 || g.V % 64) return BRI_EINVAL;  // (the bound is the apply's)
    GradPlan pl;
    rc = plan_grad(g, prm, pl);
    if (rc != BRI_OK) return rc;
    if (!work) {
        *work_bytes = pl.bytes;
        return BRI_OK;
    }
    if (*work_bytes < pl.bytes || !U || !W64 || !chi || !psi || (!F && !GU) || !gpsi ||
        (prm->inner != BRI_F64 && !Wlo))
        return BRI_EINVAL;
    {
        // the outputs and the workspace must not alias each other or any input
        const size_t V = (size_t)g.V;
        const void *ins[4] = {U, W64, chi, psi};
        const size_t inb[4] = {576 * V, 5760 * V, 192 * V, 192 * V};
        const void *outs[4] = {F, GU, gpsi, work};
        const size_t outb[4] = {256 * V, 576 * V, 192 * V, pl.bytes};
        for (int i = 0; i < 4; ++i) {
            if (!outs[i]) continue;
            for (int k = 0; k < 4; ++k)
                if (ranges_overlap(outs[i], outb[i], ins[k], inb[k])) return BRI_EINVAL;
            for (int k = i + 1; k < 4; ++k)
                if (outs[k] && ranges_overlap(outs[i], outb[i], outs[k], outb[k])) return BRI_EINVAL;
        }
    }
    hipStream_t s = (hipStream_t)stream;
    const size_t nel = (size_t)12 * g.V;
    char *base = (char *)work;
    double2 *G = (double2 *)(base + pl.g_off);
    double2 *XAB = (double2 *)(base + pl.xab_off);
    double2 *BIN = (double2 *)(base + pl.bin_off);
    double2 *Y = (double2 *)(base + pl.y_off);
    double *om_dev = (double *)(base + pl.om_off);
    void *swork = base + pl.solver_off;
    const double m0 = -prm->rho;

    // BIN = [psi | X^dag chi]
    BRI_HIP_CHECK(hipMemcpyAsync(BIN, psi, nel * sizeof(double2), hipMemcpyDeviceToDevice, s));
    StencilArgs a{};
    a.g = g;
    a.W = W64;
    a.ncol = 1;
    a.in = chi;
    a.out = BIN + nel;
    a.kind = prm->kernel;
    a.diag = kernel_diag(prm->kernel) + m0;
    rc = stencil_launch(a, BRI_F64, true, EPI_PLAIN, default_config(g, BRI_F64, 1, prm->kernel), s);
    if (rc != BRI_OK) return rc;
    // a_i = (A + sigma_i)^{-1} psi and b_i = (A + sigma_i)^{-1} X^dag chi by two-column multi-shift
    // solves over the shifts, m at a time (m = n: one solve keeping every solution); a solve's X
    // holds them as [i][2][12 V], i.e. a_i = X[2 i], b_i = X[2 i + 1].  Per solve the pairs
    // (X a_i, b_i), (X b_i, a_i) (weight -rho omega_i) are added to the outer products G, and
    // y = c0 psi + sum omega_i a_i, gpsi = rho (chi + c0 X^dag chi + sum omega_i b_i) accumulate;
    // the pair (chi, y) (weight rho) joins the last solve's.
    double c0, om[MAXS], sg[MAXS], tf[MAXS];
    shift_coeffs(prm, &c0, om, sg, tf);
    BRI_HIP_CHECK(hipMemcpyAsync(om_dev, om, sizeof(double) * n, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(grad_combine_kernel, dim3(1024), dim3(256), 0, s, nel, c0, (const double2 *)psi, 0.0,
                       (const double2 *)nullptr, 0.0, 0, (const double *)om_dev, (const double2 *)nullptr, 0, Y);
    hipLaunchKernelGGL(grad_combine_kernel, dim3(1024), dim3(256), 0, s, nel, prm->rho, (const double2 *)chi,
                       prm->rho * c0, (const double2 *)(BIN + nel), 0.0, 0, (const double *)om_dev,
                       (const double2 *)nullptr, 0, (double2 *)gpsi);
    BRI_HIP_CHECK(hipGetLastError());
    const int m = grad_chunk(prm);
    int rcs = BRI_OK;
    ov_stats sst;
    std::memset(&sst, 0, sizeof(sst));
    for (int i0 = 0; i0 < n; i0 += m) {
        const int i1 = i0 + m < n ? i0 + m : n, mc = i1 - i0;
        const bool last = i1 == n;
        void *xs = nullptr;
        ov_stats cst;
        const int r = ov_solve_shifts(g, W64, Wlo, prm, BIN, 2, swork, pl.solver_bytes, nullptr, s, &xs, &cst, i0, i1);
        if (r != BRI_OK && r != BRI_ENOCONV) return r;
        if (r == BRI_ENOCONV) rcs = r;
        sst.iters += cst.iters;
        sst.refine += cst.refine;
        for (int k = 0; k < mc; ++k) {
            sst.shift_iters[i0 + k] = cst.shift_iters[k];
            sst.rel_resid[i0 + k] = cst.rel_resid[k];
        }
        const double2 *X = (const double2 *)xs;
        hipLaunchKernelGGL(grad_combine_kernel, dim3(1024), dim3(256), 0, s, nel, 1.0, (const double2 *)Y, 0.0,
                           (const double2 *)nullptr, 1.0, mc, (const double *)(om_dev + i0), X, 2 * nel, Y);
        hipLaunchKernelGGL(grad_combine_kernel, dim3(1024), dim3(256), 0, s, nel, 1.0, (const double2 *)gpsi, 0.0,
                           (const double2 *)nullptr, prm->rho, mc, (const double *)(om_dev + i0), X + nel, 2 * nel,
                           (double2 *)gpsi);
        BRI_HIP_CHECK(hipGetLastError());
        // X applied to this solve's 2 mc shift solutions
        StencilArgs ax = a;
        ax.ncol = 2 * mc;
        ax.in = X;
        ax.out = XAB;
        rc = stencil_launch(ax, BRI_F64, false, EPI_PLAIN, default_config(g, BRI_F64, 2 * mc, prm->kernel), s);
        if (rc != BRI_OK) return rc;
        PairTable pt;
        std::memset(&pt, 0, sizeof(pt));
        pt.accumulate = i0 > 0;
        for (int k = 0; k < mc; ++k) {
            const double w = -prm->rho * om[i0 + k];
            pt.u[pt.n] = XAB + (size_t)(2 * k) * nel;
            pt.v[pt.n] = X + (size_t)(2 * k + 1) * nel;
            pt.w[pt.n++] = w;
            pt.u[pt.n] = XAB + (size_t)(2 * k + 1) * nel;
            pt.v[pt.n] = X + (size_t)(2 * k) * nel;
            pt.w[pt.n++] = w;
        }
        if (last) {
            pt.u[pt.n] = (const double2 *)chi;
            pt.v[pt.n] = Y;
            pt.w[pt.n++] = prm->rho;
        }
        outer_pairs(g, pt, G, s, prm->kernel);
        BRI_HIP_CHECK(hipGetLastError());
    }
    rc = force_from_outer(g, (const double2 *)U, (const double2 *)W64, G, (double *)F, (double2 *)GU, s, prm->kernel);
    if (rc != BRI_OK) return rc;
    if (hipStreamSynchronize(s) != hipSuccess) return BRI_EHIP;
    if (stats) {
        *stats = sst;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return rcs;
}

}  // extern "C"
