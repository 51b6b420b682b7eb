// Outer solve of the massive overlap equation (Sec. 4, Sec. 7):
//   (D_ov + mt) x = bt,   mt = m / (1 - m/(2 rho)),
//   bt = [1 + (m/(2 rho)) (1 - D_ov/(2 rho))] b / (1 - m/(2 rho))     complete form, eq. (upshot_complete)
//   bt = b / (1 - m/(2 rho))                                           traditional, eq. (upshot_traditional)
// (lattice spacing 1) by BiCGstab, each operator application being one ov_apply (the
// multi-shift evaluation of the rational) plus mt x.
//
// Cascaded preconditioning (Sec. 8, eqs. (cascaded_one), (cascaded_two)): with D^(0) = D_bri(-rho)
// and D^(k) = X r_{n_k}(X^dag X) the overlap approximants of growing Kenney-Laub order, every
// level works with A_k = rho [D^(k) + 1 + mt/rho] = D_ov^(n_k) + mt (and, at the Brillouin level,
// rho D_bri(-rho) + rho + mt).  A level's operator is inverted by BiCGstab preconditioned from the
// right by the next level's approximate inverse, itself an inner BiCGstab to a loose tolerance.
// Because the preconditioner changes from call to call, x is updated with the preconditioned
// vectors themselves (phat = K p, shat = K s, v = A phat, t = A shat), so the recursive residual
// stays the residual of x.
//
// The host drives the recurrences; every vector operation and reduction runs on the device,
// reductions in FP64 with fixed block partial sums added in order on the host (deterministic).
#include <chrono>
#include <complex>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace bri {

int geom_check(const bri_geom *geom, Geom *g);

using cplx = std::complex<double>;

constexpr int DOT_BLOCKS = 512;
constexpr int DOT_THREADS = 256;

// partial sums of up to three complex dot products <a_k, b_k> = sum conj(a_k) b_k
__global__ __launch_bounds__(DOT_THREADS) void outer_dots_kernel(size_t n, int nd, const double2 *__restrict__ a0,
                                                                 const double2 *__restrict__ b0,
                                                                 const double2 *__restrict__ a1,
                                                                 const double2 *__restrict__ b1,
                                                                 const double2 *__restrict__ a2,
                                                                 const double2 *__restrict__ b2,
                                                                 double *__restrict__ partial) {
    double acc[3][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    const double2 *as[3] = {a0, a1, a2};
    const double2 *bs[3] = {b0, b1, b2};
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        for (int k = 0; k < nd; ++k) {
            const double2 u = as[k][i], v = bs[k][i];
            acc[k][0] += u.x * v.x + u.y * v.y;
            acc[k][1] += u.x * v.y - u.y * v.x;
        }
    }
    __shared__ double sh[DOT_THREADS];
    for (int k = 0; k < nd; ++k)
        for (int c = 0; c < 2; ++c) {
            sh[threadIdx.x] = acc[k][c];
            __syncthreads();
            for (int w = DOT_THREADS / 2; w > 0; w >>= 1) {
                if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
                __syncthreads();
            }
            if (threadIdx.x == 0) partial[((size_t)k * gridDim.x + blockIdx.x) * 2 + c] = sh[0];
            __syncthreads();
        }
}

// out = c0 x0 + c1 x1 + c2 x2 (complex coefficients; unused terms have a null vector); out may
// be one of the inputs (elementwise)
__global__ void outer_lincomb_kernel(size_t n, double2 *out, double2 c0, const double2 *x0, double2 c1,
                                     const double2 *x1, double2 c2, const double2 *x2) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        double2 v = make_double2(0.0, 0.0);
        const double2 *xs[3] = {x0, x1, x2};
        const double2 cs[3] = {c0, c1, c2};
        for (int k = 0; k < 3; ++k) {
            if (!xs[k]) continue;
            const double2 u = xs[k][i];
            v.x += cs[k].x * u.x - cs[k].y * u.y;
            v.y += cs[k].x * u.y + cs[k].y * u.x;
        }
        out[i] = v;
    }
}

static inline size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }
static inline double2 c2d(cplx c) { return make_double2(c.real(), c.imag()); }

// one level of the cascade: its operator and the BiCGstab vectors of its solves
struct Level {
    int kl_n;       // 0: Brillouin operator, else overlap approximant of this order
    ov_params prm;  // overlap apply parameters (kl_n > 0)
    double tol;
    int max_iter;
    double2 *r, *r0, *p, *v, *s, *t, *ph, *sh;
    int iters = 0, calls = 0, applies = 0;
};
constexpr int NVEC = 8;

struct Cascade {
    const bri_geom *geom;
    Geom g;
    const void *W64, *Wlo;
    double rho, mt;
    size_t n;
    hipStream_t s;
    void *ov;
    size_t ov_bytes;
    double *partial;
    std::vector<double> hp;
    std::vector<Level> lev;
    int inner_iters = 0;
    ov_stats ist;

    void lincomb(double2 *dst, cplx c0, const double2 *x0, cplx c1 = 0.0, const double2 *x1 = nullptr,
                 cplx c2 = 0.0, const double2 *x2 = nullptr) {
        hipLaunchKernelGGL(outer_lincomb_kernel, dim3(2048), dim3(256), 0, s, n, dst, c2d(c0), x0, c2d(c1), x1,
                           c2d(c2), x2);
    }

    // up to three dot products, summed on the host in a fixed order; synchronises the stream
    int dots(int nd, const double2 *a0, const double2 *b0, const double2 *a1, const double2 *b1, const double2 *a2,
             const double2 *b2, cplx *res) {
        hipLaunchKernelGGL(outer_dots_kernel, dim3(DOT_BLOCKS), dim3(DOT_THREADS), 0, s, n, nd, a0, b0, a1, b1, a2,
                           b2, partial);
        if (hipGetLastError() != hipSuccess) return BRI_EHIP;
        if (hipMemcpyAsync(hp.data(), partial, sizeof(double) * 2 * nd * DOT_BLOCKS, hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return BRI_EHIP;
        for (int k = 0; k < nd; ++k) {
            double re = 0.0, im = 0.0;
            for (int i = 0; i < DOT_BLOCKS; ++i) {
                re += hp[((size_t)k * DOT_BLOCKS + i) * 2];
                im += hp[((size_t)k * DOT_BLOCKS + i) * 2 + 1];
            }
            res[k] = cplx(re, im);
        }
        return BRI_OK;
    }

    // dst = D_ov^(n_k) v (kl_n > 0) or rho D_bri(-rho) v (kl_n = 0); dst != v
    int apply_d(Level &L, const double2 *v, double2 *dst) {
        ++L.applies;
        if (L.kl_n == 0) {
            const int r = L.prm.kernel == BRI_KERNEL_WILSON ? ::wil_apply(geom, W64, BRI_F64, -rho, v, dst, 1, s)
                                                            : ::bri_apply(geom, W64, BRI_F64, -rho, v, dst, 1, s);
            if (r != BRI_OK) return r;
            lincomb(dst, rho, dst);
            return hipGetLastError() == hipSuccess ? BRI_OK : BRI_EHIP;
        }
        size_t ob = ov_bytes;
        const int r = ::ov_apply(geom, W64, Wlo, &L.prm, v, dst, 1, ov, &ob, &ist, s);
        inner_iters += ist.iters;
        // a loose preconditioner may stop its multi-shift at the cap
        return (r == BRI_ENOCONV && &L != &lev[0]) ? BRI_OK : r;
    }

    // dst = A_k v
    int apply_a(Level &L, const double2 *v, double2 *dst) {
        const int r = apply_d(L, v, dst);
        if (r != BRI_OK) return r;
        lincomb(dst, 1.0, dst, L.kl_n == 0 ? rho + mt : mt, v);
        return hipGetLastError() == hipSuccess ? BRI_OK : BRI_EHIP;
    }

    // dst = approximate A_{k+1}^{-1} v, or v itself below the last level
    int precondition(int k, const double2 *v, double2 *dst) {
        if (k + 1 >= (int)lev.size()) {
            lincomb(dst, 1.0, v);
            return hipGetLastError() == hipSuccess ? BRI_OK : BRI_EHIP;
        }
        double rel;
        int it;
        const int r = solve(k + 1, v, dst, rel, it);
        // an inner level that stops at its cap (or breaks down after progress) still preconditions
        return (r == BRI_ENOCONV) ? BRI_OK : r;
    }

    // BiCGstab on A_k x = b from x = 0 (shadow residual r0 = b), right-preconditioned by level k+1
    int solve(int k, const double2 *b, double2 *x, double &rel, int &it) {
        Level &L = lev[k];
        ++L.calls;
        cplx d[3];
        lincomb(x, 0.0, nullptr);
        lincomb(L.r, 1.0, b);
        lincomb(L.r0, 1.0, b);
        lincomb(L.p, 0.0, nullptr);
        lincomb(L.v, 0.0, nullptr);
        int rc = dots(1, b, b, nullptr, nullptr, nullptr, nullptr, d);
        if (rc != BRI_OK) return rc;
        const double bn = std::sqrt(d[0].real());
        it = 0;
        rel = 0.0;
        if (bn == 0.0) return BRI_OK;
        if (!std::isfinite(bn)) return BRI_ENAN;
        rel = 1.0;
        cplx rho_new = d[0], rho_old = 1.0, alpha = 1.0, omega = 1.0;
        while (it < L.max_iter) {
            ++it;
            ++L.iters;
            const cplx beta = (rho_new / rho_old) * (alpha / omega);
            lincomb(L.p, 1.0, L.r, beta, L.p, -beta * omega, L.v);  // p = r + beta (p - omega v)
            if ((rc = precondition(k, L.p, L.ph)) != BRI_OK) return rc;
            if ((rc = apply_a(L, L.ph, L.v)) != BRI_OK) return rc;  // v = A K p
            if ((rc = dots(1, L.r0, L.v, nullptr, nullptr, nullptr, nullptr, d)) != BRI_OK) return rc;
            if (std::abs(d[0]) == 0.0 || !std::isfinite(d[0].real())) return k == 0 || it == 1 ? BRI_ENAN : BRI_ENOCONV;
            alpha = rho_new / d[0];
            lincomb(L.s, 1.0, L.r, -alpha, L.v);  // s = r - alpha v
            if ((rc = dots(1, L.s, L.s, nullptr, nullptr, nullptr, nullptr, d)) != BRI_OK) return rc;
            const double srel = std::sqrt(d[0].real()) / bn;
            if (!std::isfinite(srel)) return BRI_ENAN;
            if (srel <= L.tol) {
                lincomb(x, 1.0, x, alpha, L.ph);
                rel = srel;
                return BRI_OK;
            }
            if ((rc = precondition(k, L.s, L.sh)) != BRI_OK) return rc;
            if ((rc = apply_a(L, L.sh, L.t)) != BRI_OK) return rc;  // t = A K s
            if ((rc = dots(2, L.t, L.s, L.t, L.t, nullptr, nullptr, d)) != BRI_OK) return rc;
            if (d[1].real() == 0.0 || !std::isfinite(d[1].real())) return k == 0 ? BRI_ENAN : BRI_ENOCONV;
            omega = d[0] / d[1].real();
            lincomb(x, 1.0, x, alpha, L.ph, omega, L.sh);  // x += alpha K p + omega K s
            lincomb(L.r, 1.0, L.s, -omega, L.t);           // r = s - omega t
            rho_old = rho_new;
            if ((rc = dots(2, L.r, L.r, L.r0, L.r, nullptr, nullptr, d)) != BRI_OK) return rc;
            rel = std::sqrt(d[0].real()) / bn;
            rho_new = d[1];
            if (!std::isfinite(rel)) return BRI_ENAN;
            if (rel <= L.tol) return BRI_OK;
            if (std::abs(omega) == 0.0 || std::abs(rho_new) == 0.0) return k == 0 ? BRI_ENAN : BRI_ENOCONV;
        }
        return BRI_ENOCONV;
    }
};

static int check_levels(const ov_params *prm, const ov_mass_params *mp, int nprec, const ov_level *prec) {
    const double rho = prm->rho, m = mp->mass;
    if (!(m >= 0.0 && m < 2.0 * rho) || !(mp->tol > 0.0) || mp->max_iter < 1 ||
        (mp->complete != 0 && mp->complete != 1))
        return BRI_EINVAL;
    if (nprec < 0 || nprec > BRI_MAX_LEVELS || (nprec > 0 && !prec)) return BRI_EINVAL;
    for (int k = 0; k < nprec; ++k) {
        const ov_level &l = prec[k];
        if (l.kl_n < 0 || l.kl_n > BRI_MAX_SHIFTS || !(l.tol > 0.0) || l.max_iter < 1) return BRI_EINVAL;
        if (l.kl_n > 0 && !(l.ms_tol > 0.0)) return BRI_EINVAL;
        if (l.kl_n > 0 && l.inner != BRI_F64 && l.inner != BRI_F32 && l.inner != BRI_F32_BF16W) return BRI_EINVAL;
        if (l.kl_n == 0 && k != nprec - 1) return BRI_EINVAL;  // the Brillouin level ends the chain
    }
    return BRI_OK;
}

static ov_params level_params(const ov_params *top, const ov_level &l) {
    ov_params p = *top;
    p.kl_n = l.kl_n;
    p.tol = l.ms_tol;
    p.inner = l.inner;
    p.kind = BRI_KL_DIAG;  // the cascade nests f_{1,1}: diagonal approximants only
    p.relax = 0;
    if (p.inner != BRI_F64 && p.max_refine == 0) p.max_refine = 10;
    return p;
}

}  // namespace bri

extern "C" {

int ov_solve(const bri_geom *geom, const void *W64, const void *Wlo, const ov_params *params,
             const ov_mass_params *mp, int nprec, const ov_level *prec, const void *in, void *out, void *work,
             size_t *work_bytes, ov_solve_stats *stats, void *stream) {
    using namespace bri;
    const auto t0 = std::chrono::steady_clock::now();
    Geom g;
    int rc = geom_check(geom, &g);
    if (rc != BRI_OK) return rc;
    if (!params || !mp || !work_bytes) return BRI_EINVAL;
    if ((rc = check_levels(params, mp, nprec, prec)) != BRI_OK) return rc;
    // workspace: the largest ov_apply workspace of all levels, NVEC vectors per level, bt, partials
    size_t ovb = 0;
    bool low = false;
    for (int k = -1; k < nprec; ++k) {
        if (k >= 0 && prec[k].kl_n == 0) continue;
        const ov_params p = k < 0 ? *params : level_params(params, prec[k]);
        low = low || p.inner != BRI_F64;
        size_t b = 0;
        rc = ov_apply(geom, nullptr, nullptr, &p, nullptr, nullptr, 1, nullptr, &b, nullptr, nullptr);
        if (rc != BRI_OK) return rc;
        ovb = b > ovb ? b : ovb;
    }
    const size_t vb = al256((size_t)12 * g.V * sizeof(double2));
    const size_t nvec = (size_t)NVEC * (nprec + 1) + 1;
    const size_t pb = al256(sizeof(double) * 2 * 3 * DOT_BLOCKS);
    const size_t need = nvec * vb + pb + al256(ovb);
    if (!work) {
        *work_bytes = need;
        return BRI_OK;
    }
    if (*work_bytes < need || !W64 || !in || !out || in == out || (low && !Wlo)) return BRI_EINVAL;

    Cascade c;
    c.geom = geom;
    c.g = g;
    c.W64 = W64;
    c.Wlo = Wlo;
    c.rho = params->rho;
    const double m = mp->mass, rho = params->rho;
    const double den = 1.0 - m / (2.0 * rho);
    c.mt = m / den;
    c.n = (size_t)12 * g.V;
    c.s = (hipStream_t)stream;
    c.hp.resize(2 * 3 * DOT_BLOCKS);
    char *base = (char *)work;
    auto take = [&](size_t b) {
        char *p = base;
        base += b;
        return p;
    };
    double2 *bt = (double2 *)take(vb);
    c.lev.resize(nprec + 1);
    for (int k = 0; k <= nprec; ++k) {
        Level &L = c.lev[k];
        if (k == 0) {
            L.kl_n = params->kl_n;
            L.prm = *params;
            L.tol = mp->tol;
            L.max_iter = mp->max_iter;
        } else {
            L.kl_n = prec[k - 1].kl_n;
            L.prm = level_params(params, prec[k - 1]);
            L.tol = prec[k - 1].tol;
            L.max_iter = prec[k - 1].max_iter;
        }
        double2 **vs[NVEC] = {&L.r, &L.r0, &L.p, &L.v, &L.s, &L.t, &L.ph, &L.sh};
        for (auto vp : vs) *vp = (double2 *)take(vb);
    }
    c.partial = (double *)take(pb);
    c.ov = take(al256(ovb));
    c.ov_bytes = ovb;

    // bt
    const double2 *b = (const double2 *)in;
    double2 *x = (double2 *)out;
    Level &top = c.lev[0];
    if (mp->complete) {
        rc = c.apply_d(top, b, top.t);
        if (rc != BRI_OK) return rc;
        c.lincomb(bt, (1.0 + m / (2.0 * rho)) / den, b, -m / (4.0 * rho * rho) / den, top.t);
    } else {
        c.lincomb(bt, 1.0 / den, b);
    }
    double rel = 0.0;
    int it = 0;
    const int result = c.solve(0, bt, x, rel, it);
    if (result != BRI_OK && result != BRI_ENOCONV) return result;
    // true residual |bt - A x| / |bt|
    double true_rel = 0.0;
    {
        cplx d[1];
        if ((rc = c.dots(1, bt, bt, nullptr, nullptr, nullptr, nullptr, d)) != BRI_OK) return rc;
        const double bn = std::sqrt(d[0].real());
        if (bn > 0.0) {
            if ((rc = c.apply_a(top, x, top.t)) != BRI_OK) return rc;
            c.lincomb(top.t, 1.0, bt, -1.0, top.t);
            if ((rc = c.dots(1, top.t, top.t, nullptr, nullptr, nullptr, nullptr, d)) != BRI_OK) return rc;
            true_rel = std::sqrt(d[0].real()) / bn;
        }
    }
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->iters = it;
        stats->inner_iters = c.inner_iters;
        stats->applies = top.applies;
        stats->rel_resid = true_rel;
        for (int k = 1; k <= nprec; ++k) {
            stats->level_iters[k - 1] = c.lev[k].iters;
            stats->level_calls[k - 1] = c.lev[k].calls;
            stats->level_applies[k - 1] = c.lev[k].applies;
        }
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return result;
}

}  // extern "C"
