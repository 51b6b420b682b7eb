// Outer solve of the massive overlap equation (Sec. 4, Sec. 7):
//   (D_ov + mt) x = bt,   mt = m / (1 - m/(2 rho)),
//   bt = [1 + (m/(2 rho)) (1 - D_ov/(2 rho))] b / (1 - m/(2 rho))     complete form, eq. (upshot_complete)
//   bt = b / (1 - m/(2 rho))                                           traditional, eq. (upshot_traditional)
// (lattice spacing 1) by BiCGstab, each operator application being one ov_apply (the
// multi-shift evaluation of the rational) plus mt x.  The host drives the outer recurrences;
// every vector operation and reduction runs on the device, reductions in FP64 with fixed
// block partial sums summed in order on the host (deterministic).
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

struct OuterWork {
    double2 *bt, *r, *r0, *p, *v, *s, *t;
    double *partial;
    void *ov;  // ov_apply workspace
    size_t ov_bytes, bytes;
};

static int plan_outer(const bri_geom *geom, const Geom &g, const void *W64, const void *Wlo, const ov_params *prm,
                      void *work, OuterWork &w) {
    size_t ovb = 0;
    const int rc = ov_apply(geom, nullptr, nullptr, prm, nullptr, nullptr, 1, nullptr, &ovb, nullptr, nullptr);
    if (rc != BRI_OK) return rc;
    (void)W64;
    (void)Wlo;
    const size_t vb = al256((size_t)12 * g.V * sizeof(double2));
    char *base = (char *)work;
    size_t off = 0;
    double2 **vecs[7] = {&w.bt, &w.r, &w.r0, &w.p, &w.v, &w.s, &w.t};
    for (auto vp : vecs) {
        *vp = base ? (double2 *)(base + off) : nullptr;
        off += vb;
    }
    w.partial = base ? (double *)(base + off) : nullptr;
    off += al256(sizeof(double) * 2 * 3 * DOT_BLOCKS);
    w.ov = base ? (void *)(base + off) : nullptr;
    w.ov_bytes = ovb;
    off += al256(ovb);
    w.bytes = off;
    return BRI_OK;
}

}  // namespace bri

extern "C" {

int ov_solve(const bri_geom *geom, const void *W64, const void *Wlo, const ov_params *params,
             const ov_mass_params *mp, const void *in, void *out, void *work, size_t *work_bytes,
             ov_solve_stats *stats, void *stream) {
    using namespace bri;
    const auto t0 = std::chrono::steady_clock::now();
    Geom g;
    int rc = geom_check(geom, &g);
    if (rc != BRI_OK) return rc;
    if (!params || !mp || !work_bytes) return BRI_EINVAL;
    const double rho = params->rho, m = mp->mass;
    if (!(m >= 0.0 && m < 2.0 * rho) || !(mp->tol > 0.0) || mp->max_iter < 1 ||
        (mp->complete != 0 && mp->complete != 1))
        return BRI_EINVAL;
    OuterWork w{};
    rc = plan_outer(geom, g, W64, Wlo, params, nullptr, w);
    if (rc != BRI_OK) return rc;
    if (!work) {
        *work_bytes = w.bytes;
        return BRI_OK;
    }
    if (*work_bytes < w.bytes || !W64 || !in || !out || in == out) return BRI_EINVAL;
    plan_outer(geom, g, W64, Wlo, params, work, w);
    hipStream_t s = (hipStream_t)stream;
    const size_t n = (size_t)12 * g.V;
    const double2 *b = (const double2 *)in;
    double2 *x = (double2 *)out;
    const dim3 vg(2048), vt(256);
    const double2 one = make_double2(1.0, 0.0), zero = make_double2(0.0, 0.0);
    const double den = 1.0 - m / (2.0 * rho);
    const double mt = m / den;
    int applies = 0, inner = 0;
    ov_stats ist;

    // A v = D_ov v + mt v into dst (dst != v)
    auto apply = [&](const double2 *vin, double2 *dst) -> int {
        size_t ob = w.ov_bytes;
        const int r = ::ov_apply(geom, W64, Wlo, params, vin, dst, 1, w.ov, &ob, &ist, stream);
        ++applies;
        inner += ist.iters;
        if (r != BRI_OK) return r;
        hipLaunchKernelGGL(outer_lincomb_kernel, vg, vt, 0, s, n, dst, one, (const double2 *)dst,
                           make_double2(mt, 0.0), vin, zero, (const double2 *)nullptr);
        return hipGetLastError() == hipSuccess ? BRI_OK : BRI_EHIP;
    };
    // up to three dot products, summed on the host in a fixed order
    std::vector<double> hp(2 * 3 * DOT_BLOCKS);
    auto dots = [&](int nd, const double2 *a0, const double2 *b0, const double2 *a1, const double2 *b1,
                    const double2 *a2, const double2 *b2, cplx *res) -> int {
        hipLaunchKernelGGL(outer_dots_kernel, dim3(DOT_BLOCKS), dim3(DOT_THREADS), 0, s, n, nd, a0, b0, a1, b1, a2,
                           b2, w.partial);
        if (hipGetLastError() != hipSuccess) return BRI_EHIP;
        if (hipMemcpyAsync(hp.data(), w.partial, sizeof(double) * 2 * nd * DOT_BLOCKS, hipMemcpyDeviceToHost, s) !=
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
    };
    auto lincomb = [&](double2 *dst, cplx c0, const double2 *x0, cplx c1, const double2 *x1, cplx c2,
                       const double2 *x2) {
        hipLaunchKernelGGL(outer_lincomb_kernel, vg, vt, 0, s, n, dst, c2d(c0), x0, c2d(c1), x1, c2d(c2), x2);
    };

    // bt
    if (mp->complete) {
        size_t ob = w.ov_bytes;
        rc = ::ov_apply(geom, W64, Wlo, params, b, w.t, 1, w.ov, &ob, &ist, stream);
        ++applies;
        inner += ist.iters;
        if (rc != BRI_OK) return rc;
        lincomb(w.bt, cplx((1.0 + m / (2.0 * rho)) / den, 0.0), b, cplx(-m / (4.0 * rho * rho) / den, 0.0), w.t,
                cplx(0.0, 0.0), nullptr);
    } else {
        lincomb(w.bt, cplx(1.0 / den, 0.0), b, cplx(0.0, 0.0), nullptr, cplx(0.0, 0.0), nullptr);
    }
    // BiCGstab from x = 0, shadow residual r0 = bt
    lincomb(x, cplx(0.0, 0.0), nullptr, cplx(0.0, 0.0), nullptr, cplx(0.0, 0.0), nullptr);
    lincomb(w.r, cplx(1.0, 0.0), w.bt, cplx(0.0, 0.0), nullptr, cplx(0.0, 0.0), nullptr);
    lincomb(w.r0, cplx(1.0, 0.0), w.bt, cplx(0.0, 0.0), nullptr, cplx(0.0, 0.0), nullptr);
    lincomb(w.p, cplx(0.0, 0.0), nullptr, cplx(0.0, 0.0), nullptr, cplx(0.0, 0.0), nullptr);
    lincomb(w.v, cplx(0.0, 0.0), nullptr, cplx(0.0, 0.0), nullptr, cplx(0.0, 0.0), nullptr);
    cplx d[3];
    rc = dots(2, w.bt, w.bt, w.r0, w.r, nullptr, nullptr, d);
    if (rc != BRI_OK) return rc;
    const double bn = sqrt(d[0].real());
    cplx rho_new = d[1], rho_old(1.0, 0.0), alpha(1.0, 0.0), omega(1.0, 0.0);
    int it = 0, result = BRI_ENOCONV;
    double rel = bn > 0 ? 1.0 : 0.0;
    if (bn == 0.0) result = BRI_OK;
    while (result == BRI_ENOCONV && it < mp->max_iter) {
        ++it;
        const cplx beta = (rho_new / rho_old) * (alpha / omega);
        lincomb(w.p, cplx(1.0, 0.0), w.r, beta, w.p, -beta * omega, w.v);  // p = r + beta (p - omega v)
        if ((rc = apply(w.p, w.v)) != BRI_OK) return rc;                     // v = A p
        if ((rc = dots(1, w.r0, w.v, nullptr, nullptr, nullptr, nullptr, d)) != BRI_OK) return rc;
        if (std::abs(d[0]) == 0.0 || !std::isfinite(d[0].real())) return BRI_ENAN;
        alpha = rho_new / d[0];
        lincomb(w.s, cplx(1.0, 0.0), w.r, -alpha, w.v, cplx(0.0, 0.0), nullptr);  // s = r - alpha v
        if ((rc = dots(1, w.s, w.s, nullptr, nullptr, nullptr, nullptr, d)) != BRI_OK) return rc;
        rel = sqrt(d[0].real()) / bn;
        if (rel <= mp->tol) {
            lincomb(x, cplx(1.0, 0.0), x, alpha, w.p, cplx(0.0, 0.0), nullptr);
            result = BRI_OK;
            break;
        }
        if ((rc = apply(w.s, w.t)) != BRI_OK) return rc;  // t = A s
        if ((rc = dots(2, w.t, w.s, w.t, w.t, nullptr, nullptr, d)) != BRI_OK) return rc;
        if (d[1].real() == 0.0 || !std::isfinite(d[1].real())) return BRI_ENAN;
        omega = d[0] / d[1].real();
        lincomb(x, cplx(1.0, 0.0), x, alpha, w.p, omega, w.s);            // x += alpha p + omega s
        lincomb(w.r, cplx(1.0, 0.0), w.s, -omega, w.t, cplx(0.0, 0.0), nullptr);  // r = s - omega t
        rho_old = rho_new;
        if ((rc = dots(2, w.r, w.r, w.r0, w.r, nullptr, nullptr, d)) != BRI_OK) return rc;
        rel = sqrt(d[0].real()) / bn;
        rho_new = d[1];
        if (!std::isfinite(rel)) return BRI_ENAN;
        if (rel <= mp->tol) result = BRI_OK;
    }
    // true residual |bt - A x| / |bt|
    double true_rel = 0.0;
    if (bn > 0.0) {
        if ((rc = apply(x, w.t)) != BRI_OK) return rc;
        lincomb(w.t, cplx(1.0, 0.0), w.bt, cplx(-1.0, 0.0), w.t, cplx(0.0, 0.0), nullptr);
        if ((rc = dots(1, w.t, w.t, nullptr, nullptr, nullptr, nullptr, d)) != BRI_OK) return rc;
        true_rel = sqrt(d[0].real()) / bn;
    }
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->iters = it;
        stats->inner_iters = inner;
        stats->applies = applies;
        stats->rel_resid = true_rel;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return result;
}

}  // extern "C"
