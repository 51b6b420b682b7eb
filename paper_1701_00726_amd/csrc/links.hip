// bri_build_links: off-axis links of the Brillouin stencil (App. C.1).
//
// The average over the k! shortest paths from x to x+d obeys the hop-by-hop
// recursion
//   W_d(x) = (1/k) sum_{mu in supp d} T_mu(x) W_{d - s_mu e_mu}(x + s_mu e_mu),
// with s_mu = d_mu, T_mu(x) = U_mu(x) for s_mu = +1 and U_mu(x - e_mu)^dag for
// s_mu = -1: grouping the paths by their first step, each first step mu is
// followed by all (k-1)! orderings of the remaining axes.  The links are built
// level by level (k = 1..4 hops), one kernel per level, in FP64.  A level-(k-1)
// link that is not stored is the hermitian conjugate of a stored one at the
// far end, W_{d'}(y) = W_{-d'}(y + d')^dag.
#include <cmath>

#include "common.hpp"

namespace bri {

__device__ __forceinline__ int wrap(int v, int L) { return v < 0 ? v + L : (v >= L ? v - L : v); }

__device__ __forceinline__ int site_index(const Geom &g, const int c[4]) {
    return c[0] + g.L[0] * (c[1] + g.L[1] * (c[2] + g.L[2] * c[3]));
}

// Stored directions j < 40 with k non-zero components, per level k = 1..4 (4, 12, 16, 8 of them).
struct LevelDirs {
    int n;
    int j[16];
};

// One thread per (site, stored direction of level k): blockIdx.y picks the direction.
__global__ __launch_bounds__(128) void build_level_kernel(Geom g, const double2 *__restrict__ U,
                                                          double2 *__restrict__ W, int k, LevelDirs dirs) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= g.V) return;
    const size_t V = (size_t)g.V;
    const int j = dirs.j[blockIdx.y];
    int cx[4];
    {
        int s = x;
        for (int mu = 0; mu < 4; ++mu) {
            cx[mu] = s % g.L[mu];
            s /= g.L[mu];
        }
    }
    int d[4];
    for (int mu = 0; mu < 4; ++mu) d[mu] = disp_comp(j, mu);
    double2 acc[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) acc[a][b] = make_double2(0.0, 0.0);
    for (int mu = 0; mu < 4; ++mu) {
        if (d[mu] == 0) continue;
        const int s = d[mu];
        // first step T_mu(x)
        double2 T[3][3];
        double sgn = 1.0;
        if (s > 0) {
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) T[a][b] = U[((size_t)(mu * 3 + a) * 3 + b) * V + x];
            if (g.tbc && mu == 3 && cx[3] == g.L[3] - 1) sgn = -1.0;
        } else {
            int cm[4] = {cx[0], cx[1], cx[2], cx[3]};
            cm[mu] = wrap(cm[mu] - 1, g.L[mu]);
            const int xs = site_index(g, cm);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    double2 u = U[((size_t)(mu * 3 + b) * 3 + a) * V + xs];
                    T[a][b] = make_double2(u.x, -u.y);
                }
            if (g.tbc && mu == 3 && cx[3] == 0) sgn = -1.0;
        }
        // remainder W_{d - s e_mu}(x + s e_mu)
        int cy[4] = {cx[0], cx[1], cx[2], cx[3]};
        cy[mu] = wrap(cy[mu] + s, g.L[mu]);
        int dr[4] = {d[0], d[1], d[2], d[3]};
        dr[mu] = 0;
        double2 M[3][3];
        if (k == 1) {
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) M[a][b] = make_double2(a == b ? 1.0 : 0.0, 0.0);
        } else {
            const int jr = (dr[0] + 1) + 3 * (dr[1] + 1) + 9 * (dr[2] + 1) + 27 * (dr[3] + 1);
            if (jr < 40) {
                const int ys = site_index(g, cy);
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) M[a][b] = W[((size_t)jr * 9 + a * 3 + b) * V + ys];
            } else {
                // W_{dr}(y) = W_{-dr}(y + dr)^dag, -dr stored at index 80 - jr
                int cz[4];
                for (int nu = 0; nu < 4; ++nu) cz[nu] = wrap(cy[nu] + dr[nu], g.L[nu]);
                const int zs = site_index(g, cz);
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) {
                        double2 w = W[((size_t)(80 - jr) * 9 + b * 3 + a) * V + zs];
                        M[a][b] = make_double2(w.x, -w.y);
                    }
            }
        }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double2 t = make_double2(0.0, 0.0);
                for (int c = 0; c < 3; ++c) cmac(t, T[a][c], M[c][b]);
                acc[a][b].x = fma(sgn, t.x, acc[a][b].x);
                acc[a][b].y = fma(sgn, t.y, acc[a][b].y);
            }
    }
    const double inv_k = 1.0 / (double)k;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double2 v = acc[a][b];
            W[((size_t)j * 9 + a * 3 + b) * V + x] = make_double2(v.x * inv_k, v.y * inv_k);
        }
}

__global__ void convert_f32_kernel(size_t n, const double2 *__restrict__ src, float2 *__restrict__ dst) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        double2 v = src[i];
        dst[i] = make_float2((float)v.x, (float)v.y);
    }
}

__global__ void convert_bf16_kernel(size_t n, const double2 *__restrict__ src, uint32_t *__restrict__ dst) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        double2 v = src[i];
        // round the double to float first (exact for the bfloat16 grid), then to bfloat16
        uint32_t re = f32_to_bf16((float)v.x), im = f32_to_bf16((float)v.y);
        dst[i] = re | (im << 16);
    }
}

// n link entries of an FP64 array rounded into W (complex float, or a (re, im) bfloat16 pair)
static int round_links(size_t n, const double2 *src, void *W, int wprec, hipStream_t s) {
    const int blocks = (int)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    if (wprec == BRI_F32)
        hipLaunchKernelGGL(convert_f32_kernel, dim3(blocks), dim3(256), 0, s, n, src, (float2 *)W);
    else
        hipLaunchKernelGGL(convert_bf16_kernel, dim3(blocks), dim3(256), 0, s, n, src, (uint32_t *)W);
    return hipGetLastError() == hipSuccess ? BRI_OK : BRI_EHIP;
}

int geom_check(const bri_geom *geom, Geom *g) {
    if (!geom) return BRI_EINVAL;
    long long V = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (geom->L[mu] < 1 || geom->L[mu] > 4096) return BRI_EINVAL;
        g->L[mu] = geom->L[mu];
        V *= geom->L[mu];
    }
    // site indices are 32-bit; every element offset into the link, clover, spinor and
    // workspace arrays is formed in 64 bits
    if (!std::isfinite(geom->csw)) return BRI_EINVAL;
    if (V >= (1LL << 31)) return BRI_EINVAL;
    if (geom->tbc != 0 && geom->tbc != 1) return BRI_EINVAL;
    g->V = (int)V;
    g->tbc = geom->tbc;
    g->csw = geom->csw;
    return BRI_OK;
}

// ------------------------------------------------------------------- clover

// One site: the clover-leaf field strength of every plane and its contribution to the two
// chirality blocks of -(c_SW/2) sum_{mu<nu} sigma_mu_nu F_mu_nu.
//   Q_mu_nu(x) = sum of the four plaquettes at x in the mu-nu plane, all counter-clockwise
//               (mu before nu): steps (+mu,+nu,-mu,-nu), (+nu,-mu,-nu,+mu), (-mu,-nu,+mu,+nu),
//               (-nu,+mu,+nu,-mu);
//   F_mu_nu = (Q - Q^dag) / (8i) minus its trace / 3.
// With sigma_mu_nu = (i/2)[gamma_mu, gamma_nu] in the chiral basis, sigma_jk = -eps_jkl s_l in
// both blocks and sigma_j4 = +s_j (spins 0,1) and -s_j (spins 2,3), s_l the Pauli matrices, so
// plane (mu, nu) enters with one Pauli matrix s_l and a sign per block:
//   xy: s_3, (-,-)   xz: s_2, (+,+)   yz: s_1, (-,-)   xt: s_1, (+,-)   yt: s_2, (+,-)   zt: s_3, (+,-)
__device__ void leaf_walk(const Geom &g, const double2 *__restrict__ U, const int c0[4], const int dir[4],
                          const int sgn[4], double2 (&M)[3][3]) {
    int c[4] = {c0[0], c0[1], c0[2], c0[3]};
    const unsigned V = (unsigned)g.V;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) M[a][b] = make_double2(a == b ? 1.0 : 0.0, 0.0);
    for (int st = 0; st < 4; ++st) {
        const int d = dir[st];
        if (sgn[st] < 0) c[d] = c[d] == 0 ? g.L[d] - 1 : c[d] - 1;
        const unsigned y = (unsigned)(c[0] + g.L[0] * (c[1] + g.L[1] * (c[2] + g.L[2] * c[3])));
        double2 u[3][3], T[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                const double2 e = U[((size_t)(d * 3 + a) * 3 + b) * V + y];
                if (sgn[st] > 0)
                    u[a][b] = e;
                else
                    u[b][a] = make_double2(e.x, -e.y);
            }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double re = 0.0, im = 0.0;
                for (int k = 0; k < 3; ++k) {
                    re += M[a][k].x * u[k][b].x - M[a][k].y * u[k][b].y;
                    im += M[a][k].x * u[k][b].y + M[a][k].y * u[k][b].x;
                }
                T[a][b] = make_double2(re, im);
            }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) M[a][b] = T[a][b];
        if (sgn[st] > 0) c[d] = c[d] == g.L[d] - 1 ? 0 : c[d] + 1;
    }
}

__global__ void clover_build_kernel(Geom g, const double2 *__restrict__ U, double2 *__restrict__ C) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= g.V) return;
    const unsigned V = (unsigned)g.V;
    int c[4];
    for (int mu = 0, r = x; mu < 4; ++mu) {
        c[mu] = r % g.L[mu];
        r /= g.L[mu];
    }
    double2 blk[2][6][6];
    for (int k = 0; k < 2; ++k)
        for (int a = 0; a < 6; ++a)
            for (int b = 0; b < 6; ++b) blk[k][a][b] = make_double2(0.0, 0.0);
    const double h = -0.5 * g.csw;
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = mu + 1; nu < 4; ++nu) {
            double2 Q[3][3];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) Q[a][b] = make_double2(0.0, 0.0);
            const int dirs[4][4] = {{mu, nu, mu, nu}, {nu, mu, nu, mu}, {mu, nu, mu, nu}, {nu, mu, nu, mu}};
            const int sgns[4][4] = {{1, 1, -1, -1}, {1, -1, -1, 1}, {-1, -1, 1, 1}, {-1, 1, 1, -1}};
            for (int l = 0; l < 4; ++l) {
                double2 M[3][3];
                leaf_walk(g, U, c, dirs[l], sgns[l], M);
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) {
                        Q[a][b].x += M[a][b].x;
                        Q[a][b].y += M[a][b].y;
                    }
            }
            // F = (Q - Q^dag) / (8i): F_ab = [ (Q_ab - conj Q_ba) ] / (8i)
            double2 F[3][3];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    const double dre = Q[a][b].x - Q[b][a].x, dim = Q[a][b].y + Q[b][a].y;
                    F[a][b] = make_double2(dim / 8.0, -dre / 8.0);  // (dre + i dim) / (8i)
                }
            const double tr = (F[0][0].x + F[1][1].x + F[2][2].x) / 3.0;  // F hermitian: real trace
            for (int a = 0; a < 3; ++a) F[a][a].x -= tr;
            // Pauli matrix and block signs of this plane
            const bool tplane = nu == 3;
            const int l = tplane ? mu + 1 : 4 - mu - nu;  // xy -> 3, xz -> 2, yz -> 1; xt,yt,zt -> 1,2,3
            const int sgn_sp = (mu == 0 && nu == 2) ? 1 : -1;  // xz: +, xy and yz: -
            for (int k = 0; k < 2; ++k) {
                const double kap = h * (tplane ? (k == 0 ? 1.0 : -1.0) : (double)sgn_sp);
                // nonzero entries z of s_l at (s, t)
                for (int s = 0; s < 2; ++s)
                    for (int t = 0; t < 2; ++t) {
                        double zr = 0.0, zi = 0.0;
                        if (l == 1 && s != t) zr = 1.0;
                        if (l == 2 && s == 0 && t == 1) zi = -1.0;
                        if (l == 2 && s == 1 && t == 0) zi = 1.0;
                        if (l == 3 && s == t) zr = s == 0 ? 1.0 : -1.0;
                        if (zr == 0.0 && zi == 0.0) continue;
                        for (int a = 0; a < 3; ++a)
                            for (int b = 0; b < 3; ++b) {
                                const double fr = F[a][b].x, fi = F[a][b].y;
                                double2 &o = blk[k][s * 3 + a][t * 3 + b];
                                o.x += kap * (zr * fr - zi * fi);
                                o.y += kap * (zr * fi + zi * fr);
                            }
                    }
            }
        }
    for (int k = 0; k < 2; ++k)
        for (int a = 0; a < 6; ++a)
            for (int b = 0; b < 6; ++b) C[((size_t)(k * 6 + a) * 6 + b) * V + x] = blk[k][a][b];
}

int build_clover(const Geom &g, const double2 *U, double2 *C, hipStream_t st) {
    const int threads = 64;
    hipLaunchKernelGGL(clover_build_kernel, dim3((g.V + threads - 1) / threads), dim3(threads), 0, st, g, U, C);
    BRI_HIP_CHECK(hipGetLastError());
    return BRI_OK;
}

int build_links_f64(const Geom &g, const double2 *U, double2 *W, hipStream_t st) {
    const int threads = 128;
    const int blocks = (g.V + threads - 1) / threads;
    for (int k = 1; k <= 4; ++k) {
        LevelDirs dirs{};
        for (int j = 0; j < 40; ++j) {
            int nh = 0;
            for (int r = j, mu = 0; mu < 4; ++mu, r /= 3) nh += (r % 3) != 1;
            if (nh == k) dirs.j[dirs.n++] = j;
        }
        hipLaunchKernelGGL(build_level_kernel, dim3(blocks, dirs.n), dim3(threads), 0, st, g, U, W, k, dirs);
        BRI_HIP_CHECK(hipGetLastError());
    }
    return BRI_OK;
}

}  // namespace bri

extern "C" int bri_build_links(const bri_geom *geom, const void *U, void *W, int wprec, void *stream) {
    using namespace bri;
    Geom g;
    int st = geom_check(geom, &g);
    if (st != BRI_OK) return st;
    if (!U || !W) return BRI_EINVAL;
    if (wprec != BRI_F64 && wprec != BRI_F32 && wprec != BRI_F32_BF16W) return BRI_EINVAL;
    const size_t wbytes = link_entries(g) * (wprec == BRI_F64 ? 16 : (wprec == BRI_F32 ? 8 : 4));
    if (ranges_overlap(U, (size_t)576 * g.V, W, wbytes)) return BRI_EINVAL;  // W is written while U is read
    hipStream_t s = (hipStream_t)stream;
    if (wprec == BRI_F64) {
        st = build_links_f64(g, (const double2 *)U, (double2 *)W, s);
        if (st == BRI_OK && g.csw != 0.0) st = build_clover(g, (const double2 *)U, (double2 *)W + (size_t)LINK_SLAB_ENTRIES * g.V, s);
        return st;
    }
    const size_t n = link_entries(g);
    double2 *tmp = nullptr;
    BRI_HIP_CHECK(hipMalloc(&tmp, n * sizeof(double2)));
    st = build_links_f64(g, (const double2 *)U, tmp, s);
    if (st == BRI_OK && g.csw != 0.0) st = build_clover(g, (const double2 *)U, tmp + (size_t)LINK_SLAB_ENTRIES * g.V, s);
    if (st == BRI_OK) st = round_links(n, tmp, W, wprec, s);
    if (hipStreamSynchronize(s) != hipSuccess) st = BRI_EHIP;
    if (hipFree(tmp) != hipSuccess) st = BRI_EHIP;
    return st;
}

extern "C" int bri_round_links(const bri_geom *geom, const void *W64, void *W, int wprec, void *stream) {
    using namespace bri;
    Geom g;
    const int st = geom_check(geom, &g);
    if (st != BRI_OK) return st;
    if (!W64 || !W || (wprec != BRI_F32 && wprec != BRI_F32_BF16W)) return BRI_EINVAL;
    const size_t n = link_entries(g);
    if (ranges_overlap(W64, n * sizeof(double2), W, n * (wprec == BRI_F32 ? 8 : 4))) return BRI_EINVAL;
    return round_links(n, (const double2 *)W64, W, wprec, (hipStream_t)stream);
}
