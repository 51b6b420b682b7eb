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
// Several right-hand sides run side by side, each with its own BiCGstab scalars; every operator
// application treats all of them in one batched call.  A column that has converged keeps its x
// and r (its coefficients become those of the identity) until every column is done.  The host
// drives the recurrences; every vector operation and reduction runs on the device, reductions in
// FP64 with fixed block partial sums added in order on the host (deterministic).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace bri {

int geom_check(const bri_geom *geom, Geom *g);

using cplx = std::complex<double>;

constexpr int MAXC = BRI_MAX_SOLVE_RHS;
constexpr int DOT_BLOCKS = 256;  // per column
constexpr int DOT_THREADS = 256;

// partial sums of up to three complex dot products <a_k, b_k> = sum conj(a_k) b_k per column
// (column = blockIdx.y, vectors [ncol][n]); partial[k][col][block][2]
__global__ __launch_bounds__(DOT_THREADS) void outer_dots_kernel(size_t n, int nd, const double2 *__restrict__ a0,
                                                                 const double2 *__restrict__ b0,
                                                                 const double2 *__restrict__ a1,
                                                                 const double2 *__restrict__ b1,
                                                                 const double2 *__restrict__ a2,
                                                                 const double2 *__restrict__ b2,
                                                                 double *__restrict__ partial) {
    const size_t off = (size_t)blockIdx.y * n;
    double acc[3][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    const double2 *as[3] = {a0, a1, a2};
    const double2 *bs[3] = {b0, b1, b2};
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        for (int k = 0; k < nd; ++k) {
            const double2 u = as[k][off + i], v = bs[k][off + i];
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
            if (threadIdx.x == 0)
                partial[(((size_t)k * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x) * 2 + c] = sh[0];
            __syncthreads();
        }
}

// per-column coefficients of a three-term combination
struct Coef3 {
    double2 c[MAXC][3];
};

// out = c0 x0 + c1 x1 + c2 x2 per column (column = blockIdx.y, vectors [ncol][n]); a null vector is
// a zero term; out may be one of the inputs (elementwise)
__global__ void outer_lincomb_kernel(size_t n, double2 *out, Coef3 cf, const double2 *x0, const double2 *x1,
                                     const double2 *x2) {
    const int col = blockIdx.y;
    const size_t off = (size_t)col * n;
    const double2 *xs[3] = {x0, x1, x2};
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        double2 v = make_double2(0.0, 0.0);
        for (int k = 0; k < 3; ++k) {
            if (!xs[k]) continue;
            const double2 u = xs[k][off + i], c = cf.c[col][k];
            v.x += c.x * u.x - c.y * u.y;
            v.y += c.x * u.y + c.y * u.x;
        }
        out[off + i] = v;
    }
}

// Column maps of the kernel level: only the columns still iterating go through its stencil.
struct ColMap {
    int idx[MAXC];
};

template <typename T> __device__ __forceinline__ T conv(double2 v);
template <> __device__ __forceinline__ double2 conv<double2>(double2 v) { return v; }
template <> __device__ __forceinline__ float2 conv<float2>(double2 v) { return make_float2((float)v.x, (float)v.y); }

// out column k = in column map.idx[k] (k = blockIdx.y), converted to T (complex float narrows)
template <typename T>
__global__ void outer_gather_kernel(size_t n, ColMap map, const double2 *__restrict__ in, T *__restrict__ out) {
    const double2 *src = in + (size_t)map.idx[blockIdx.y] * n;
    T *dst = out + (size_t)blockIdx.y * n;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = conv<T>(src[i]);
}

// out column c = scale * in column inv.idx[c], or zero where inv.idx[c] < 0 (c = blockIdx.y)
template <typename T>
__global__ void outer_scatter_kernel(size_t n, ColMap inv, double scale, const T *__restrict__ in,
                                     double2 *__restrict__ out) {
    const int k = inv.idx[blockIdx.y];
    double2 *dst = out + (size_t)blockIdx.y * n;
    const T *src = in + (size_t)(k < 0 ? 0 : k) * n;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = k < 0 ? make_double2(0.0, 0.0) : make_double2(scale * (double)src[i].x, scale * (double)src[i].y);
}

static inline size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

using Cols = std::vector<cplx>;  // one coefficient per column

// one level of the cascade: its operator and the BiCGstab vectors of its solves
struct Level {
    int kl_n;       // 0: kernel operator, else overlap approximant of this order
    ov_params prm;  // overlap apply parameters (kl_n > 0)
    double tol;
    int max_iter;
    int kprec;  // kernel level: precision of its stencil (BRI_F64, or BRI_F32 / BRI_F32_BF16W on Wlo)
    double2 *r, *r0, *p, *v, *s, *t, *ph, *sh;  // [ncol][12 V] each
    int iters = 0, calls = 0, applies = 0;
};
constexpr int NVEC = 8;

struct Cascade {
    const bri_geom *geom;
    Geom g;
    const void *W64, *Wlo;
    double rho, mt;
    size_t n;  // complex entries per column
    int ncol;
    hipStream_t s;
    void *ov;
    size_t ov_bytes;
    float2 *lo_in = nullptr, *lo_out = nullptr;  // low-precision kernel level: [ncol][12 V] each
    double2 *k_in = nullptr, *k_out = nullptr;   // FP64 kernel level, compacted columns
    double *partial;
    std::vector<double> hp;
    std::vector<Level> lev;
    int inner_iters = 0;
    ov_stats ist;

    Cols all(cplx v) const { return Cols(ncol, v); }

    int lincomb(double2 *dst, const Cols &c0, const double2 *x0, const Cols &c1 = Cols(), const double2 *x1 = nullptr,
                const Cols &c2 = Cols(), const double2 *x2 = nullptr) {
        Coef3 cf{};
        for (int c = 0; c < ncol; ++c) {
            const cplx k[3] = {c0.empty() ? 0.0 : c0[c], c1.empty() ? 0.0 : c1[c], c2.empty() ? 0.0 : c2[c]};
            for (int j = 0; j < 3; ++j) cf.c[c][j] = make_double2(k[j].real(), k[j].imag());
        }
        hipLaunchKernelGGL(outer_lincomb_kernel, dim3(1024, ncol), dim3(256), 0, s, n, dst, cf, x0, x1, x2);
        return hipGetLastError() == hipSuccess ? BRI_OK : BRI_EHIP;
    }

    // up to three dot products per column, summed on the host in a fixed order; res[k][col];
    // synchronises the stream
    int dots(int nd, const double2 *a0, const double2 *b0, const double2 *a1, const double2 *b1, const double2 *a2,
             const double2 *b2, std::vector<Cols> &res) {
        hipLaunchKernelGGL(outer_dots_kernel, dim3(DOT_BLOCKS, ncol), dim3(DOT_THREADS), 0, s, n, nd, a0, b0, a1,
                           b1, a2, b2, partial);
        if (hipGetLastError() != hipSuccess) return BRI_EHIP;
        const size_t cnt = (size_t)2 * nd * ncol * DOT_BLOCKS;
        if (hipMemcpyAsync(hp.data(), partial, sizeof(double) * cnt, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return BRI_EHIP;
        res.assign(nd, Cols(ncol));
        for (int k = 0; k < nd; ++k)
            for (int c = 0; c < ncol; ++c) {
                double re = 0.0, im = 0.0;
                const double *q = hp.data() + ((size_t)k * ncol + c) * DOT_BLOCKS * 2;
                for (int i = 0; i < DOT_BLOCKS; ++i) {
                    re += q[2 * i];
                    im += q[2 * i + 1];
                }
                res[k][c] = cplx(re, im);
            }
        return BRI_OK;
    }

    // dst = D_ov^(n_k) v (kl_n > 0) or rho D_kernel(-rho) v (kl_n = 0); dst != v.  Columns outside
    // `act` are zero in v and come out zero: the multi-shift drops zero columns at its start, and
    // the kernel level applies its stencil to the active columns only (gathered, in the level's
    // precision, and scattered back).
    int apply_d(Level &L, const double2 *v, double2 *dst, const std::vector<char> &act) {
        ++L.applies;
        if (L.kl_n == 0) {
            const bool wil = L.prm.kernel == BRI_KERNEL_WILSON;
            ColMap map{}, inv{};
            int k = 0;
            for (int c = 0; c < ncol; ++c) {
                inv.idx[c] = act[c] ? k : -1;
                if (act[c]) map.idx[k++] = c;
            }
            if (k == 0) return lincomb(dst, all(0.0), nullptr);
            const bool lo = L.kprec != BRI_F64;
            if (!lo && k == ncol) {  // every column active: no compaction
                const int r = wil ? ::wil_apply(geom, W64, BRI_F64, -rho, v, dst, ncol, s)
                                  : ::bri_apply(geom, W64, BRI_F64, -rho, v, dst, ncol, s);
                if (r != BRI_OK) return r;
                return lincomb(dst, all(rho), dst);
            }
            if (lo)
                hipLaunchKernelGGL(outer_gather_kernel<float2>, dim3(1024, k), dim3(256), 0, s, n, map, v, lo_in);
            else
                hipLaunchKernelGGL(outer_gather_kernel<double2>, dim3(1024, k), dim3(256), 0, s, n, map, v, k_in);
            const void *Wk = lo ? Wlo : W64;
            const void *in_k = lo ? (const void *)lo_in : (const void *)k_in;
            void *out_k = lo ? (void *)lo_out : (void *)k_out;
            const int r = wil ? ::wil_apply(geom, Wk, L.kprec, -rho, in_k, out_k, k, s)
                              : ::bri_apply(geom, Wk, L.kprec, -rho, in_k, out_k, k, s);
            if (r != BRI_OK) return r;
            if (lo)
                hipLaunchKernelGGL(outer_scatter_kernel<float2>, dim3(1024, ncol), dim3(256), 0, s, n, inv, rho,
                                   lo_out, dst);
            else
                hipLaunchKernelGGL(outer_scatter_kernel<double2>, dim3(1024, ncol), dim3(256), 0, s, n, inv, rho,
                                   k_out, dst);
            return hipGetLastError() == hipSuccess ? BRI_OK : BRI_EHIP;
        }
        size_t ob = ov_bytes;
        const int r = ::ov_apply(geom, W64, Wlo, &L.prm, v, dst, ncol, ov, &ob, &ist, s);
        inner_iters += ist.iters;
        // a loose preconditioner may stop its multi-shift at the cap
        return (r == BRI_ENOCONV && &L != &lev[0]) ? BRI_OK : r;
    }

    // dst = A_k v
    int apply_a(Level &L, const double2 *v, double2 *dst, const std::vector<char> &act) {
        const int r = apply_d(L, v, dst, act);
        if (r != BRI_OK) return r;
        return lincomb(dst, all(1.0), dst, all(L.kl_n == 0 ? rho + mt : mt), v);
    }

    // dst = approximate A_{k+1}^{-1} v, or v itself below the last level
    int precondition(int k, const double2 *v, double2 *dst) {
        if (k + 1 >= (int)lev.size()) return lincomb(dst, all(1.0), v);
        int it;
        const int r = solve(k + 1, v, dst, it, nullptr);
        // an inner level that stops at its cap (or breaks down after progress) still preconditions
        return (r == BRI_ENOCONV) ? BRI_OK : r;
    }

    // BiCGstab on A_k x = b from x = 0 (shadow residual r0 = b) for every column, right-
    // preconditioned by level k+1.  A column stops at its own tolerance; at the outer level a
    // breakdown is an error, inside the cascade the column keeps what it has.
    int solve(int k, const double2 *b, double2 *x, int &it, std::vector<double> *rel_out) {
        Level &L = lev[k];
        ++L.calls;
        std::vector<Cols> d;
        int rc;
        if ((rc = lincomb(x, all(0.0), nullptr)) != BRI_OK) return rc;
        if ((rc = lincomb(L.r, all(1.0), b)) != BRI_OK) return rc;
        if ((rc = lincomb(L.r0, all(1.0), b)) != BRI_OK) return rc;
        if ((rc = lincomb(L.p, all(0.0), nullptr)) != BRI_OK) return rc;
        if ((rc = lincomb(L.v, all(0.0), nullptr)) != BRI_OK) return rc;
        if ((rc = dots(1, b, b, nullptr, nullptr, nullptr, nullptr, d)) != BRI_OK) return rc;
        std::vector<double> bn(ncol), rel(ncol, 0.0);
        std::vector<char> active(ncol, 0);
        Cols rho_new(ncol), rho_old(ncol, 1.0), alpha(ncol, 1.0), omega(ncol, 1.0);
        int nact = 0;
        for (int c = 0; c < ncol; ++c) {
            bn[c] = std::sqrt(d[0][c].real());
            if (!std::isfinite(bn[c])) return BRI_ENAN;
            active[c] = bn[c] > 0.0;
            nact += active[c];
            rel[c] = active[c] ? 1.0 : 0.0;
            rho_new[c] = d[0][c];
        }
        const bool outer = k == 0;
        auto finish = [&](int status) {
            if (rel_out) *rel_out = rel;
            return status;
        };
        it = 0;
        while (nact > 0 && it < L.max_iter) {
            ++it;
            ++L.iters;
            Cols beta(ncol, 0.0), mbw(ncol, 0.0);
            for (int c = 0; c < ncol; ++c)
                if (active[c]) {
                    beta[c] = (rho_new[c] / rho_old[c]) * (alpha[c] / omega[c]);
                    mbw[c] = -beta[c] * omega[c];
                }
            // p = r + beta (p - omega v); a finished column gets p = 0, so the inner solves and the
            // multi-shift skip it
            Cols one_act(ncol, 0.0);
            for (int c = 0; c < ncol; ++c) one_act[c] = active[c] ? 1.0 : 0.0;
            if ((rc = lincomb(L.p, one_act, L.r, beta, L.p, mbw, L.v)) != BRI_OK) return rc;
            if ((rc = precondition(k, L.p, L.ph)) != BRI_OK) return rc;
            if ((rc = apply_a(L, L.ph, L.v, active)) != BRI_OK) return rc;  // v = A K p
            if ((rc = dots(1, L.r0, L.v, nullptr, nullptr, nullptr, nullptr, d)) != BRI_OK) return rc;
            Cols ma(ncol, 0.0), half(ncol, 0.0);
            for (int c = 0; c < ncol; ++c) {
                if (!active[c]) continue;
                if (std::abs(d[0][c]) == 0.0 || !std::isfinite(d[0][c].real())) {
                    if (outer) return finish(BRI_ENAN);
                    active[c] = 0;
                    --nact;
                    continue;
                }
                alpha[c] = rho_new[c] / d[0][c];
                ma[c] = -alpha[c];
            }
            for (int c = 0; c < ncol; ++c) one_act[c] = active[c] ? 1.0 : 0.0;
            if ((rc = lincomb(L.s, one_act, L.r, ma, L.v)) != BRI_OK) return rc;  // s = r - alpha v
            if ((rc = dots(1, L.s, L.s, nullptr, nullptr, nullptr, nullptr, d)) != BRI_OK) return rc;
            bool any_half = false;
            for (int c = 0; c < ncol; ++c) {
                if (!active[c]) continue;
                const double srel = std::sqrt(d[0][c].real()) / bn[c];
                if (!std::isfinite(srel)) return finish(BRI_ENAN);
                if (srel <= L.tol) {  // converged half way: x += alpha K p
                    half[c] = alpha[c];
                    rel[c] = srel;
                    active[c] = 0;
                    --nact;
                    any_half = true;
                }
            }
            if (any_half && (rc = lincomb(x, all(1.0), x, half, L.ph)) != BRI_OK) return rc;
            if (nact == 0) break;
            if (any_half) {  // the columns that just finished leave s as well
                for (int c = 0; c < ncol; ++c) one_act[c] = active[c] ? 1.0 : 0.0;
                if ((rc = lincomb(L.s, one_act, L.s)) != BRI_OK) return rc;
            }
            if ((rc = precondition(k, L.s, L.sh)) != BRI_OK) return rc;
            if ((rc = apply_a(L, L.sh, L.t, active)) != BRI_OK) return rc;  // t = A K s
            if ((rc = dots(2, L.t, L.s, L.t, L.t, nullptr, nullptr, d)) != BRI_OK) return rc;
            Cols ax(ncol, 0.0), ox(ncol, 0.0), keep(ncol, 1.0), rs(ncol, 0.0), rt(ncol, 0.0);
            for (int c = 0; c < ncol; ++c) {
                if (!active[c]) continue;
                if (d[1][c].real() == 0.0 || !std::isfinite(d[1][c].real())) {
                    if (outer) return finish(BRI_ENAN);
                    active[c] = 0;
                    --nact;
                    continue;
                }
                omega[c] = d[0][c] / d[1][c].real();
                ax[c] = alpha[c];
                ox[c] = omega[c];
                keep[c] = 0.0;
                rs[c] = 1.0;
                rt[c] = -omega[c];
            }
            if ((rc = lincomb(x, all(1.0), x, ax, L.ph, ox, L.sh)) != BRI_OK) return rc;  // x += alpha Kp + omega Ks
            if ((rc = lincomb(L.r, keep, L.r, rs, L.s, rt, L.t)) != BRI_OK) return rc;    // r = s - omega t
            rho_old = rho_new;
            if ((rc = dots(2, L.r, L.r, L.r0, L.r, nullptr, nullptr, d)) != BRI_OK) return rc;
            for (int c = 0; c < ncol; ++c) {
                if (!active[c]) continue;
                rel[c] = std::sqrt(d[0][c].real()) / bn[c];
                rho_new[c] = d[1][c];
                if (!std::isfinite(rel[c])) return finish(BRI_ENAN);
                if (rel[c] <= L.tol) {
                    active[c] = 0;
                    --nact;
                } else if (std::abs(omega[c]) == 0.0 || std::abs(rho_new[c]) == 0.0) {
                    if (outer) return finish(BRI_ENAN);
                    active[c] = 0;
                    --nact;
                }
            }
        }
        return finish(nact > 0 ? BRI_ENOCONV : BRI_OK);
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
        if (l.inner != BRI_F64 && l.inner != BRI_F32 && l.inner != BRI_F32_BF16W) return BRI_EINVAL;
        if (l.kl_n == 0 && k != nprec - 1) return BRI_EINVAL;  // the kernel level ends the chain
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
             const ov_mass_params *mp, int nprec, const ov_level *prec, const void *in, void *out, int nrhs,
             void *work, size_t *work_bytes, ov_solve_stats *stats, void *stream) {
    using namespace bri;
    const auto t0 = std::chrono::steady_clock::now();
    Geom g;
    int rc = geom_check(geom, &g);
    if (rc != BRI_OK) return rc;
    if (!params || !mp || !work_bytes || nrhs < 1 || nrhs > MAXC) return BRI_EINVAL;
    if ((rc = check_levels(params, mp, nprec, prec)) != BRI_OK) return rc;
    // every low-precision piece reads the one array Wlo, so they must agree on its precision
    int lo_prec = params->inner != BRI_F64 ? params->inner : -1;
    bool lo_kernel = false;
    for (int k = 0; k < nprec; ++k) {
        if (prec[k].inner == BRI_F64) continue;
        if (lo_prec >= 0 && prec[k].inner != lo_prec) return BRI_EINVAL;
        lo_prec = prec[k].inner;
        lo_kernel = lo_kernel || prec[k].kl_n == 0;
    }
    // workspace: the largest ov_apply workspace of all levels, NVEC vectors per level, bt, partials
    size_t ovb = 0;
    bool low = false;
    for (int k = -1; k < nprec; ++k) {
        if (k >= 0 && prec[k].kl_n == 0) continue;
        const ov_params p = k < 0 ? *params : level_params(params, prec[k]);
        low = low || p.inner != BRI_F64;
        size_t b = 0;
        rc = ov_apply(geom, nullptr, nullptr, &p, nullptr, nullptr, nrhs, nullptr, &b, nullptr, nullptr);
        if (rc != BRI_OK) return rc;
        ovb = b > ovb ? b : ovb;
    }
    const size_t vb = al256((size_t)12 * g.V * sizeof(double2) * nrhs);
    const size_t nvec = (size_t)NVEC * (nprec + 1) + 1;
    const size_t pb = al256(sizeof(double) * 2 * 3 * DOT_BLOCKS * nrhs);
    bool f64_kernel = false;
    for (int k = 0; k < nprec; ++k) f64_kernel = f64_kernel || (prec[k].kl_n == 0 && prec[k].inner == BRI_F64);
    const size_t lb = lo_kernel ? al256((size_t)12 * g.V * sizeof(float2) * nrhs) : 0;
    const size_t kb = f64_kernel ? vb : 0;
    const size_t need = nvec * vb + pb + al256(ovb) + 2 * lb + 2 * kb;
    if (!work) {
        *work_bytes = need;
        return BRI_OK;
    }
    if (*work_bytes < need || !W64 || !in || !out || ((low || lo_kernel) && !Wlo)) return BRI_EINVAL;
    {
        const size_t vbytes = (size_t)12 * g.V * nrhs * sizeof(double2);
        if (ranges_overlap(in, vbytes, out, vbytes) || ranges_overlap(in, vbytes, work, need) ||
            ranges_overlap(out, vbytes, work, need))
            return BRI_EINVAL;
    }

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
    c.ncol = nrhs;
    c.s = (hipStream_t)stream;
    c.hp.resize((size_t)2 * 3 * DOT_BLOCKS * nrhs);
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
            L.kprec = BRI_F64;
        } else {
            L.kl_n = prec[k - 1].kl_n;
            L.prm = level_params(params, prec[k - 1]);
            L.tol = prec[k - 1].tol;
            L.max_iter = prec[k - 1].max_iter;
            L.kprec = prec[k - 1].kl_n == 0 ? prec[k - 1].inner : BRI_F64;
        }
        double2 **vs[NVEC] = {&L.r, &L.r0, &L.p, &L.v, &L.s, &L.t, &L.ph, &L.sh};
        for (auto vp : vs) *vp = (double2 *)take(vb);
    }
    c.partial = (double *)take(pb);
    c.ov = take(al256(ovb));
    c.ov_bytes = ovb;
    if (lo_kernel) {
        c.lo_in = (float2 *)take(lb);
        c.lo_out = (float2 *)take(lb);
    }
    if (f64_kernel) {
        c.k_in = (double2 *)take(kb);
        c.k_out = (double2 *)take(kb);
    }

    // bt
    const double2 *b = (const double2 *)in;
    double2 *x = (double2 *)out;
    Level &top = c.lev[0];
    const std::vector<char> every(nrhs, 1);
    if (mp->complete) {
        if ((rc = c.apply_d(top, b, top.t, every)) != BRI_OK) return rc;
        rc = c.lincomb(bt, c.all((1.0 + m / (2.0 * rho)) / den), b, c.all(-m / (4.0 * rho * rho) / den), top.t);
    } else {
        rc = c.lincomb(bt, c.all(1.0 / den), b);
    }
    if (rc != BRI_OK) return rc;
    int it = 0;
    const int result = c.solve(0, bt, x, it, nullptr);
    if (result != BRI_OK && result != BRI_ENOCONV) return result;
    // true residual |bt - A x| / |bt|, worst column
    double true_rel = 0.0;
    {
        std::vector<Cols> d, e;
        if ((rc = c.dots(1, bt, bt, nullptr, nullptr, nullptr, nullptr, d)) != BRI_OK) return rc;
        if ((rc = c.apply_a(top, x, top.t, every)) != BRI_OK) return rc;
        if ((rc = c.lincomb(top.t, c.all(1.0), bt, c.all(-1.0), top.t)) != BRI_OK) return rc;
        if ((rc = c.dots(1, top.t, top.t, nullptr, nullptr, nullptr, nullptr, e)) != BRI_OK) return rc;
        for (int k = 0; k < nrhs; ++k) {
            const double bn = std::sqrt(d[0][k].real());
            if (bn > 0.0) true_rel = std::max(true_rel, std::sqrt(e[0][k].real()) / bn);
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
