// Overlap operator apply: D_ov psi = rho (psi + X r_n(X^dag X) psi), X = D_bri(-rho)
// (eq. (def_over)), with the Kenney-Laub partial fractions
//   r_n(t) = c0 + sum_i omega_i / (t + sigma_i)            (eq. (KLnn_parfrac))
// evaluated by a multi-shift conjugate gradient on A + sigma_0, A = X^dag X,
// sigma_0 the smallest shift (Sec. 3.3).  Many right-hand sides ("columns")
// run side by side, each with its own Krylov space and FP64 scalars.
//
// Multi-shift CG.  The base system (A + sigma_0) x = b runs plain CG:
//   alpha_k = (r_k, r_k) / (p_k, (A + sigma_0) p_k),  r_{k+1} = r_k - alpha_k (A + sigma_0) p_k,
//   beta_k = (r_{k+1}, r_{k+1}) / (r_k, r_k),          p_{k+1} = r_{k+1} + beta_k p_k.
// For sigma = sigma_0 + delta the residuals stay collinear, r^sigma_k = zeta^sigma_k r_k,
// because every Krylov polynomial of the shifted system is a rescaled base polynomial.
// Matching the three-term residual recurrences of the two systems gives
//   zeta_{k+1} = zeta_k zeta_{k-1} alpha_{k-1} /
//                [alpha_k beta_{k-1} (zeta_{k-1} - zeta_k) + zeta_{k-1} alpha_{k-1} (1 + delta alpha_k)],
//   alpha^sigma_k = alpha_k zeta_{k+1} / zeta_k,   beta^sigma_k = beta_k (zeta_{k+1} / zeta_k)^2,
//   x^sigma_{k+1} = x^sigma_k + alpha^sigma_k p^sigma_k,
//   p^sigma_{k+1} = zeta_{k+1} r_{k+1} + beta^sigma_k p^sigma_k,
// with zeta_0 = zeta_{-1} = 1, alpha_{-1} = 1, beta_{-1} = 0.  Shift sigma stops once
// |zeta^sigma| |r| <= tol |b|.  The base shift has zeta = 1, so its search
// direction is p itself.  When only y = c0 b + sum_sigma omega_sigma x^sigma is
// needed the x^sigma are never stored: y accumulates omega_sigma alpha^sigma p^sigma, and the
// applies defer even that: within a window of iterations y and the p^sigma are carried as
// coefficients of the stored residuals and written once per window (WinState below), so an
// iteration streams r and p instead of every p^sigma and y.
//
// Mixed precision (inner = BRI_F32 or BRI_F32_BF16W): the same multi-shift recurrences, with the
// precision of the operator and of the Krylov vectors relaxed as the residual falls.  A matrix-
// vector product whose relative error is u perturbs the recursively updated residual, and with
// it every shifted solution, by about u |r_k| (inexact Krylov methods: van den Eshof and Sleijpen,
// SIAM J. Matrix Anal. Appl. 26 (2004) 125; Simoncini and Szyld, SIAM J. Sci. Comput. 25 (2003)
// 454).  So the iterations run in FP64 until the base residual of every column has fallen to
// |r| <= (tol / u_lo) |b|, u_lo the unit roundoff of the low precision (2^-24 for FP32 links
// and vectors, 2^-8 for bfloat16 links); then r, p and the p^sigma are rounded to FP32 once and
// the remaining iterations apply the stencil with the low-precision links on FP32 vectors,
// while y (or every x^sigma) keeps accumulating in FP64 and all scalars stay FP64.  Each late
// iteration's rounding is then of order tol |b|, the level the shifts stop at; no shift needs
// a separate correction solve, so the multi-shift structure (one Krylov space for all shifts)
// is kept to the end.  The output is formed from the FP64 y with the FP64 links.
//
// All solver scalars live on the device (ColState) and are updated by small
// kernels; the host only polls a done flag every few iterations, and every
// loop kernel returns at once for columns that are done.  Because no launch
// argument changes between iterations, a block of iterations is captured once
// into a HIP graph and replayed (one launch per block instead of six per
// iteration); the instantiated graphs are cached per solve layout.
#include <math.h>

#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <vector>

#include "stencil.hpp"

namespace bri {

constexpr int RED_THREADS = 256;
constexpr int CHECK_EVERY = 8;
constexpr double LONG_ITER_SEC = 2e-3;  // iterations this long are polled one by one before the switch
constexpr int INIT_BLOCKS = 256;  // vector-kernel blocks per column

// --------------------------------------------------------------- reductions

// deterministic sums of n partial pairs (stride 2) by one block: each lane sums a strided slice,
// each wave folds its lanes with shuffles, and every thread adds the wave sums in the same order,
// so all threads return the same (x, y) = (sum of component 0, sum of component 1)
static_assert(RED_THREADS % 64 == 0 && MAXS <= RED_THREADS, "one thread per shift");
__device__ double2 block_sum2(const double *partial, int n) {
    __shared__ double2 sh[RED_THREADS / 64];
    double sx = 0.0, sy = 0.0;
    for (int i = threadIdx.x; i < n; i += RED_THREADS) {
        sx += partial[2 * i];
        sy += partial[2 * i + 1];
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        sx += __shfl_down(sx, off, 64);
        sy += __shfl_down(sy, off, 64);
    }
    if (threadIdx.x % 64 == 0) sh[threadIdx.x / 64] = make_double2(sx, sy);
    __syncthreads();
    double2 t = sh[0];
#pragma unroll
    for (int w = 1; w < RED_THREADS / 64; ++w) {
        t.x += sh[w].x;
        t.y += sh[w].y;
    }
    __syncthreads();
    return t;
}

// ------------------------------------------------------------------ kernels

// Deferred shift updates.  Within a window of at most WIN iterations the shifted directions and
// y are carried as linear combinations of the vectors at the window's start and the residuals
// r_{k0+1}, ..., r_{k0+m} the window stores (slots 1..m):
//   p^sigma = a_sigma P_sigma + sum_j c[sigma][j] R_j,    y = y_0 + sum_sigma e_sigma P_sigma + sum_j f_j R_j,
// with P_sigma = p^sigma_{k0} (P_0 = p_{k0}, the base direction) and y_0 = y_{k0}.  An iteration
// then writes only p and one residual slot; the scalar recurrences of the multi-shift update
// (x^sigma += alpha^sigma p^sigma, p^sigma = zeta r + beta^sigma p^sigma) act on the coefficients,
// and a fold materialises y and the p^sigma once per window.  The sums are those of the
// per-iteration updates, taken in another order.
// When every x^sigma is kept (the gradient's shift solutions) the same holds per shift:
//   x^sigma = x^sigma_0 + e_sigma P_sigma + sum_j h[sigma][j] R_j.
constexpr int WIN = 8;
struct WinState {
    int wn;                   // residuals stored in the window
    double a[MAXS], e[MAXS];  // coefficients of P_sigma in p^sigma and in y (or in x^sigma)
    double c[MAXS][WIN + 1];  // c[sigma][j]: of R_j in p^sigma (j = 1..WIN)
    double f[WIN + 1];        // f[j]: of R_j in y
    double h[MAXS][WIN + 1];  // h[sigma][j]: of R_j in x^sigma
};

// column c = blockIdx.y.  r = p = b, p_sigma = b, and y = c0 b (or x_sigma = 0);
// partial |b|^2.  B is the input type (double2 or float2), C the solver type.  With deferred
// updates y and ps are NULL: the first window reads b in their place.
template <typename B, typename C>
__global__ void ms_init_kernel(size_t n, const B *__restrict__ b, C *__restrict__ r, C *__restrict__ p,
                               C *__restrict__ y, C *__restrict__ x, C *__restrict__ ps, int ncol, int nshift,
                               double c0, double *partial) {
    const int col = blockIdx.y;
    const size_t off = (size_t)col * n;
    double s = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const B bv = b[off + i];
        C v;
        v.x = bv.x;
        v.y = bv.y;
        r[off + i] = v;
        p[off + i] = v;
        if (y) {
            C yv;
            yv.x = c0 * bv.x;
            yv.y = c0 * bv.y;
            y[off + i] = yv;
        }
        if (x) {
            C z;
            z.x = 0;
            z.y = 0;
            for (int k = 0; k < nshift; ++k) x[((size_t)k * ncol + col) * n + i] = z;
        }
        if (ps)
            for (int k = 1; k < nshift; ++k) ps[((size_t)(k - 1) * ncol + col) * n + i] = v;
        s += (double)v.x * v.x + (double)v.y * v.y;
    }
    __shared__ double sh[256];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * ((size_t)col * gridDim.x + blockIdx.x)] = sh[0];
        partial[2 * ((size_t)col * gridDim.x + blockIdx.x) + 1] = 0.0;
    }
}

// one block per column
__global__ void ms_scalar_init_kernel(ColState *states, const double *partial, int nblk, double tol) {
    ColState *st = states + blockIdx.x;
    const double b2 = block_sum2(partial + 2 * (size_t)blockIdx.x * nblk, nblk).x;
    if (threadIdx.x == 0) {
        st->bnorm2 = b2;
        st->rr = b2;
        st->tol2 = tol * tol * b2;
        st->alpha = 0.0;
        st->alpha_old = 1.0;
        st->beta = 0.0;
        st->beta_old = 0.0;
        st->iter = 0;
        st->status = 0;
        st->done = (b2 == 0.0) ? 1 : 0;
        if (!isfinite(b2)) {
            st->status = BRI_ENAN;
            st->done = 1;
        }
        for (int i = 0; i < st->nshift; ++i) {
            st->zeta[i] = 1.0;
            st->zeta_old[i] = 1.0;
            st->zeta_new[i] = 1.0;
            st->alpha_s[i] = 0.0;
            st->beta_s[i] = 0.0;
            st->active[i] = st->done ? 0 : 1;
            st->upd_x[i] = 0;
            st->conv_iter[i] = 0;
            st->conv_res[i] = 0.0;
        }
    }
}

// alpha and the shifted alpha^sigma after t = X p (partials: |t|^2, |p|^2).  Every thread forms
// alpha from the same sums; thread i < nshift updates shift i, thread 0 the column scalars.
__global__ void ms_alpha_kernel(ColState *states, const double *partial, int nblk) {
    ColState *st = states + blockIdx.x;
    if (st->done) return;
    const double2 sums = block_sum2(partial + 2 * (size_t)blockIdx.x * nblk, nblk);
    const double pAp = sums.x + st->sigma0 * sums.y;
    const double alpha = st->rr / pAp;
    const bool bad = !isfinite(alpha) || pAp <= 0.0;
    const int i = threadIdx.x;
    if (i < st->nshift) {
        const int act = bad ? 0 : st->active[i];
        st->upd_x[i] = act;
        if (act) {
            const double z = st->zeta[i], zo = st->zeta_old[i];
            const double den =
                alpha * st->beta_old * (zo - z) + zo * st->alpha_old * (1.0 + st->delta[i] * alpha);
            const double zn = z * zo * st->alpha_old / den;
            st->zeta_new[i] = zn;
            st->alpha_s[i] = alpha * zn / z;
        }
    }
    if (i == 0) {
        if (bad) {
            st->status = BRI_ENAN;
            st->done = 1;
        } else {
            st->alpha = alpha;
        }
    }
}

// beta, beta^sigma, convergence after r -= alpha (A + sigma0) p (partials: |r|^2).  Thread
// i < nshift updates shift i; the column scalars are written by thread 0 after a block-wide
// vote on whether any shift is still active (every read of them precedes that barrier).
// Stopping: shift i by itself once |r_i| <= tol_i |b|; with the result bound (joint), shift i
// once ebw_i |r_i| <= tol |b| / (2 nshift), and every shift once sum_i ebw_i |r_i| <= tol |b|
// (a stopped shift counts with its residual when it stopped).
__global__ void ms_beta_kernel(ColState *states, const double *partial, int nblk, WinState *ws, int xmode) {
    ColState *st = states + blockIdx.x;
    if (st->done) return;
    const double rr_new = block_sum2(partial + 2 * (size_t)blockIdx.x * nblk, nblk).x;
    const bool bad = !isfinite(rr_new);
    const double beta = rr_new / st->rr;
    const int it = st->iter + 1;
    const int i = threadIdx.x;
    const int ns = st->nshift;
    int still = 0;
    double res2 = 0.0, term = 0.0;  // |r_i|^2 of a shift still running; its bound term
    if (i < ns) {
        if (bad) {
            st->active[i] = 0;
            st->upd_x[i] = 0;
        } else if (st->active[i]) {
            const double zn = st->zeta_new[i], z = st->zeta[i];
            const double ratio = zn / z;
            st->beta_s[i] = beta * ratio * ratio;
            st->zeta_old[i] = z;
            st->zeta[i] = zn;
            res2 = zn * zn * rr_new;
            const double e2 = st->ebw[i] * st->ebw[i] * res2;
            const bool stop = st->joint ? e2 * (4.0 * ns * ns) <= st->tol2 : res2 <= st->tol2 * st->tolf2[i];
            if (stop) {
                st->active[i] = 0;
                st->conv_iter[i] = it;
                st->conv_res[i] = sqrt(res2 / st->bnorm2);
            } else {
                still = 1;
            }
            term = sqrt(e2);
        } else {
            term = st->ebw[i] * st->conv_res[i] * sqrt(st->bnorm2);
        }
    }
    // the bound over all shifts (they sit in the first wave); fixed-order sum
    static_assert(MAXS <= 64, "one wave holds every shift");
    if (st->joint && !bad && i < 64) {
        double tot = term;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) tot += __shfl_xor(tot, off, 64);
        if (still && tot * tot <= st->tol2) {
            st->active[i] = 0;
            st->conv_iter[i] = it;
            st->conv_res[i] = sqrt(res2 / st->bnorm2);
            still = 0;
        }
    }
    // deferred updates: this iteration's y steps and next directions act on the coefficients
    // (wave 0 holds every shift, so the reads of c precede its writes in program order)
    bool overflow = false;
    if (ws && !bad && i < 64) {
        WinState *w = ws + blockIdx.x;
        const int m = w->wn;
        overflow = m >= WIN;  // the host folds every WIN iterations; never reached
        if (!overflow) {
            // y += sum_sigma omega alpha^sigma p^sigma, or x^sigma += alpha^sigma p^sigma (the
            // shifts that took their step)
            const bool step = i < ns && st->upd_x[i];
            const double wgt = step ? (xmode ? 1.0 : st->omega[i]) * st->alpha_s[i] : 0.0;
            if (i < ns) w->e[i] += wgt * w->a[i];
            if (xmode) {
                if (step)
                    for (int j = 1; j <= m; ++j) w->h[i][j] += wgt * w->c[i][j];
            } else {
                for (int j = 1; j <= m; ++j) {
                    double v = i < ns ? wgt * w->c[i][j] : 0.0;
#pragma unroll
                    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
                    if (i == 0) w->f[j] += v;
                }
            }
            // p^sigma <- zeta_{k+1} r_{k+1} + beta^sigma p^sigma for the shifts still running;
            // the base direction p <- r_{k+1} + beta p always
            if (i < ns && (i == 0 || st->active[i])) {
                const double bs = i == 0 ? beta : st->beta_s[i];
                w->a[i] *= bs;
                for (int j = 1; j <= m; ++j) w->c[i][j] *= bs;
                w->c[i][m + 1] = i == 0 ? 1.0 : st->zeta[i];
            }
            if (i == 0) w->wn = m + 1;
        }
    }
    const int any = __syncthreads_or(still);
    if (i == 0) {
        st->iter = it;
        if (overflow) {
            st->status = BRI_EINVAL;
            st->done = 1;
            return;
        }
        if (bad) {
            st->status = BRI_ENAN;
            st->done = 1;
            return;
        }
        st->alpha_old = st->alpha;
        st->beta_old = beta;
        st->beta = beta;
        st->rr = rr_new;
        if (!any) st->done = 2;  // converged: this iteration's vector update still runs
    }
}

// column c = blockIdx.y:
//   y += sum_sigma omega alpha^sigma p^sigma   (or x^sigma += alpha^sigma p^sigma)
//   p^sigma = zeta^sigma r + beta^sigma p^sigma,  p = r + beta p
// The shifted directions are streamed UPD_BATCH at a time: all loads of a batch are issued
// before any store, so the independent streams overlap in flight.
constexpr int UPD_BATCH = 8;

template <typename C, typename Y>
__global__ __launch_bounds__(256) void ms_update_kernel(const ColState *__restrict__ states, size_t n, int ncol,
                                                        const C *__restrict__ r, C *__restrict__ p,
                                                        Y *__restrict__ y, Y *__restrict__ x, C *__restrict__ ps) {
    const int col = blockIdx.y;
    const ColState *st = states + col;
    const int done = st->done;
    if (done == 1) return;
    const int ns = st->nshift;
    const double beta = st->beta;
    const size_t off = (size_t)col * n;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const C ri = r[off + i];
        C pi = p[off + i];
        Y yi;
        if (y) yi = y[off + i];
        for (int k0 = 0; k0 < ns; k0 += UPD_BATCH) {
            C v[UPD_BATCH];
            Y xv[UPD_BATCH];
#pragma unroll
            for (int b = 0; b < UPD_BATCH; ++b) {
                const int k = k0 + b;
                if (k >= ns || !st->upd_x[k]) continue;
                v[b] = k == 0 ? pi : ps[((size_t)(k - 1) * ncol + col) * n + i];
                if (!y) xv[b] = x[((size_t)k * ncol + col) * n + i];
            }
#pragma unroll
            for (int b = 0; b < UPD_BATCH; ++b) {
                const int k = k0 + b;
                if (k >= ns || !st->upd_x[k]) continue;
                const double as = st->alpha_s[k];
                if (y) {
                    const double w = st->omega[k] * as;
                    yi.x += w * v[b].x;
                    yi.y += w * v[b].y;
                } else {
                    xv[b].x += as * v[b].x;
                    xv[b].y += as * v[b].y;
                    x[((size_t)k * ncol + col) * n + i] = xv[b];
                }
                if (k > 0 && st->active[k]) {
                    const double z = st->zeta[k], bs = st->beta_s[k];
                    C u;
                    u.x = z * ri.x + bs * v[b].x;
                    u.y = z * ri.y + bs * v[b].y;
                    ps[((size_t)(k - 1) * ncol + col) * n + i] = u;
                }
            }
        }
        if (y) y[off + i] = yi;
        if (done == 0) {
            pi.x = ri.x + beta * pi.x;
            pi.y = ri.y + beta * pi.y;
            p[off + i] = pi;
        }
    }
}

// blocks per column of the vector-update kernel: about two elements per thread
static inline int update_blocks(size_t n) {
    const size_t b = (n + 511) / 512;
    return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

// Deferred updates, per iteration: R_m = r_{k+1} (m = the window count the beta kernel just
// advanced) and p = r_{k+1} + beta p.  Column c = blockIdx.y; slot j of column c at
// R + ((j - 1) ncol + c) n.
template <typename C>
__global__ __launch_bounds__(256) void ms_pupdate_kernel(const ColState *__restrict__ states,
                                                         const WinState *__restrict__ ws, size_t n, int ncol,
                                                         const C *__restrict__ r, C *__restrict__ p,
                                                         C *__restrict__ R) {
    const int col = blockIdx.y;
    const ColState *st = states + col;
    if (st->done == 1) return;
    const int m = ws[col].wn;
    if (m < 1 || m > WIN) return;
    const double beta = st->beta;
    const size_t off = (size_t)col * n;
    C *__restrict__ Rm = R + ((size_t)(m - 1) * ncol + col) * n;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const C ri = r[off + i];
        C pi = p[off + i];
        Rm[i] = ri;
        pi.x = ri.x + beta * pi.x;
        pi.y = ri.y + beta * pi.y;
        p[off + i] = pi;
    }
}

// The fold: y += e_0 P_0 + sum_{sigma>=1} e_sigma P_sigma + sum_j f_j R_j (or, with x != NULL,
// x^sigma += e_sigma P_sigma + sum_j h[sigma][j] R_j for every shift), and for a running column
// P_sigma <- a_sigma P_sigma + sum_j c[sigma][j] R_j for the shifts still active and P_0 <- p, all
// in FP64 arithmetic.  CI is the type of the window's vectors, CO that of the P written (FP32
// at the switch to the low-precision phase, where Pout / P0out are the FP32 vectors).  In the
// first window (first = 1) every P_sigma is the right-hand side b, which P_0 holds, y starts
// at c0 b and every x^sigma at 0, so P_0 is read in their place (neither y, the x^sigma nor the
// P_sigma was written at the start) and every x^sigma is written.
template <typename CI, typename CO>
__global__ __launch_bounds__(256) void ms_fold_kernel(const ColState *__restrict__ states,
                                                      const WinState *__restrict__ ws, size_t n, int ncol,
                                                      const CI *__restrict__ R, const CI *__restrict__ p,
                                                      const CI *P0in, CO *P0out, const CI *Pin, CO *Pout,
                                                      double2 *__restrict__ y, double2 *__restrict__ x, int convert,
                                                      int first) {
    const int col = blockIdx.y;
    const ColState *st = states + col;
    const WinState *w = ws + col;
    const int m = w->wn < WIN ? w->wn : WIN;
    if (m == 0 && !convert && !first) return;  // no iteration since the last fold: nothing changed
    const int ns = st->nshift;
    const bool running = st->done == 0;
    const bool xmode = x != nullptr;
    const size_t off = (size_t)col * n;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        double2 rj[WIN];
#pragma unroll
        for (int j = 0; j < WIN; ++j) {
            if (j < m) {
                const CI v = R[((size_t)j * ncol + col) * n + i];
                rj[j] = make_double2(v.x, v.y);
            } else {
                rj[j] = make_double2(0.0, 0.0);
            }
        }
        double2 yv = make_double2(0.0, 0.0), bv = make_double2(0.0, 0.0);
        if (first) {
            const CI u = P0in[off + i];
            bv = make_double2(u.x, u.y);
        }
        if (!xmode) yv = first ? make_double2(st->c0 * bv.x, st->c0 * bv.y) : y[off + i];
        // x^sigma += e_sigma P_sigma + sum_j h[sigma][j] R_j for a shift with steps in this window
        auto x_step = [&](int k, const double2 &v) {
            const double e = w->e[k];
            if (e == 0.0 && !first) return;
            const size_t xi = ((size_t)k * ncol + col) * n + i;
            double2 xv = first ? make_double2(0.0, 0.0) : x[xi];
            xv.x += e * v.x;
            xv.y += e * v.y;
#pragma unroll
            for (int j = 0; j < WIN; ++j) {
                if (j < m) {
                    xv.x += w->h[k][j + 1] * rj[j].x;
                    xv.y += w->h[k][j + 1] * rj[j].y;
                }
            }
            x[xi] = xv;
        };
        // a direction is read only where it enters: a shift without a step in this window (e = 0)
        // that no longer runs may hold a stale or never-written vector
        if (w->e[0] != 0.0 || (xmode && first)) {
            double2 v = bv;
            if (!first) {
                const CI u = P0in[off + i];
                v = make_double2(u.x, u.y);
            }
            if (xmode) {
                x_step(0, v);
            } else {
                yv.x += w->e[0] * v.x;
                yv.y += w->e[0] * v.y;
            }
        }
        for (int k = 1; k < ns; ++k) {
            const double e = w->e[k];
            const bool adv = running && st->active[k];
            if (e == 0.0 && !adv && !(xmode && first)) continue;
            const size_t pidx = ((size_t)(k - 1) * ncol + col) * n + i;
            double2 v = bv;
            if (!first) {
                const CI u = Pin[pidx];
                v = make_double2(u.x, u.y);
            }
            if (xmode) {
                x_step(k, v);
            } else {
                yv.x += e * v.x;
                yv.y += e * v.y;
            }
            if (adv) {
                const double a = w->a[k];
                double ux = a * v.x, uy = a * v.y;
#pragma unroll
                for (int j = 0; j < WIN; ++j) {
                    if (j < m) {
                        const double c = w->c[k][j + 1];
                        ux += c * rj[j].x;
                        uy += c * rj[j].y;
                    }
                }
                CO u;
                u.x = ux;
                u.y = uy;
                Pout[pidx] = u;
            }
        }
        if (!xmode) {
#pragma unroll
            for (int j = 0; j < WIN; ++j) {
                if (j < m) {
                    yv.x += w->f[j + 1] * rj[j].x;
                    yv.y += w->f[j + 1] * rj[j].y;
                }
            }
            y[off + i] = yv;
        }
        if (running) {
            const CI v = p[off + i];
            CO u;
            u.x = v.x;
            u.y = v.y;
            P0out[off + i] = u;
        }
    }
}

// empties every column's window after a fold (one block per column)
__global__ void ms_window_reset_kernel(WinState *ws) {
    WinState *w = ws + blockIdx.x;
    const int i = threadIdx.x;
    if (i < MAXS) {
        w->a[i] = 1.0;
        w->e[i] = 0.0;
        for (int j = 0; j <= WIN; ++j) {
            w->c[i][j] = 0.0;
            w->h[i][j] = 0.0;
        }
    }
    if (i <= WIN) w->f[i] = 0.0;
    if (i == 0) w->wn = 0;
}

// done 2 -> 1 for every column; *alldone = 1 once every column is done, else 2 when sw2 > 0 and
// every column still iterating has |r|^2 <= sw2 |b|^2 (time for the low-precision phase), else 0
__global__ void ms_finish_kernel(ColState *states, int ncol, int *alldone, double sw2) {
    __shared__ int cnt[256], low[256];
    int mine = 0, below = 0;
    for (int c = threadIdx.x; c < ncol; c += blockDim.x) {
        if (states[c].done == 2) states[c].done = 1;
        mine += states[c].done != 0;
        below += states[c].done != 0 || states[c].rr <= sw2 * states[c].bnorm2;
    }
    cnt[threadIdx.x] = mine;
    low[threadIdx.x] = below;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            cnt[threadIdx.x] += cnt[threadIdx.x + w];
            low[threadIdx.x] += low[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *alldone = (cnt[0] == ncol) ? 1 : ((sw2 > 0.0 && low[0] == ncol) ? 2 : 0);
}

// dst = src rounded to FP32 (the Krylov vectors entering the low-precision phase)
__global__ void narrow_kernel(size_t count, const double2 *__restrict__ src, float2 *__restrict__ dst) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
        const double2 v = src[i];
        dst[i] = make_float2((float)v.x, (float)v.y);
    }
}

// ----------------------------------------------------------------- host side

void kl_coeffs(int n, double *c0, double *omega, double *sigma) {
    // eq. (KLnn_parfrac): theta_i = (2i+1) pi / (4n+2), omega_i = 2 / ((2n+1) cos^2 theta_i),
    // sigma_i = tan^2 theta_i, i < n.  Past pi/4 the complementary angle
    // phi_i = pi/2 - theta_i = (n - i) pi / (2n+1) is used (cos theta = sin phi,
    // tan theta = 1 / tan phi), so that both stay accurate to a few ulp as theta -> pi/2.
    const double pi = 3.14159265358979323846;
    *c0 = 1.0 / (2.0 * n + 1.0);
    for (int i = 0; i < n; ++i) {
        if (2 * (2 * i + 1) <= 2 * n + 1) {  // theta <= pi/4
            const double th = (2.0 * i + 1.0) * pi / (4.0 * n + 2.0);
            const double cs = cos(th), tn = tan(th);
            omega[i] = 2.0 / ((2.0 * n + 1.0) * cs * cs);
            sigma[i] = tn * tn;
        } else {
            const double ph = (double)(n - i) * pi / (2.0 * n + 1.0);
            const double sn = sin(ph), tn = tan(ph);
            omega[i] = 2.0 / ((2.0 * n + 1.0) * sn * sn);
            sigma[i] = 1.0 / (tn * tn);
        }
    }
}

// First upper diagonal f_{n-1,n} = g_{2n} (Sec. 3.3, App. B): g_2n(x) = (x/n) sum_{i<n}
// 1 / (sin^2 theta_i + cos^2 theta_i x^2), theta_i = (2i+1) pi / (4n), i.e. no constant term,
// omega_i = 1 / (n cos^2 theta_i), sigma_i = tan^2 theta_i (complementary angle past pi/4).
void kl_upper_coeffs(int n, double *omega, double *sigma) {
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        if (2 * i + 1 <= n) {  // theta <= pi/4
            const double th = (2.0 * i + 1.0) * pi / (4.0 * n);
            const double cs = cos(th), tn = tan(th);
            omega[i] = 1.0 / (n * cs * cs);
            sigma[i] = tn * tn;
        } else {
            const double ph = (2.0 * (n - i) - 1.0) * pi / (4.0 * n);
            const double sn = sin(ph), tn = tan(ph);
            omega[i] = 1.0 / (n * sn * sn);
            sigma[i] = 1.0 / (tn * tn);
        }
    }
}

// The rational of an overlap apply: c0, omega, sigma of the diagonal or first upper diagonal
// Kenney-Laub function, and the per-shift factor on the stopping tolerance: 1, or with
// relaxation 1 omega_max / omega_i (App. B: the weights grow with the shift, so the small
// shifts, whose terms carry small weights, may stop at a larger residual).  Relaxation 2 (the
// result bound) stops on the weighted sum instead; plan_shifts sets its weights.
void shift_coeffs(const ov_params *prm, double *c0, double *omega, double *sigma, double *tolf) {
    const int n = prm->kl_n;
    if (prm->kind == BRI_KL_UPPER) {
        *c0 = 0.0;
        kl_upper_coeffs(n, omega, sigma);
    } else {
        kl_coeffs(n, c0, omega, sigma);
    }
    double wmax = 0.0;
    for (int i = 0; i < n; ++i) wmax = omega[i] > wmax ? omega[i] : wmax;
    for (int i = 0; i < n; ++i) tolf[i] = prm->relax == 1 ? wmax / omega[i] : 1.0;
}

bool params_ok(const ov_params *prm) {
    const int n = prm->kl_n;
    if (n < 1 || n > MAXS || !(prm->rho > 0.0 && prm->rho < 2.0) || !(prm->tol > 0.0) || prm->max_iter < 1)
        return false;
    if (prm->inner != BRI_F64 && prm->inner != BRI_F32 && prm->inner != BRI_F32_BF16W) return false;
    if (prm->max_refine < 0 || prm->max_refine > 100) return false;
    if (prm->kind != BRI_KL_DIAG && prm->kind != BRI_KL_UPPER) return false;
    if (prm->kernel != BRI_KERNEL_BRILLOUIN && prm->kernel != BRI_KERNEL_WILSON) return false;
    if (prm->recompute < 0 || prm->recompute > MAXS) return false;
    return prm->relax >= 0 && prm->relax <= 2;
}

static inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// bump allocator over the caller's workspace (only counts bytes when base is NULL)
struct Arena {
    char *base;
    size_t used = 0;
    explicit Arena(void *b) : base((char *)b) {}
    void *take(size_t bytes) {
        void *p = base ? base + used : nullptr;
        used += align256(bytes);
        return p;
    }
};

// unit roundoff of the low-precision operator: FP32 links and vectors, or bfloat16 links
inline double unit_roundoff(int prec) { return prec == BRI_F32_BF16W ? 0x1p-8 : 0x1p-24; }

// One batched multi-shift solve: ncol columns, nshift shifts each.
struct MsSolve {
    Geom g;
    int prec = BRI_F64;  // vectors and stencil of the first phase (FP64)
    const void *W = nullptr;
    // low-precision phase: once every column has |r| <= lo_switch |b| the
    // iterations continue on FP32 vectors with the links Wlo of precision prec_lo; y / x stay FP64
    int prec_lo = -1;
    const void *Wlo = nullptr;
    double lo_switch = 0.0;
    void *r_lo = nullptr, *p_lo = nullptr, *t_lo = nullptr, *ps_lo = nullptr;
    double m0 = 0.0;
    int kind = KERN_BRI;  // kernel operator X = D_kind(m0)
    int ncol = 1, nshift = 1;
    bool store_x = false;  // keep x^sigma (else accumulate y)
    double c0 = 0.0;
    std::vector<double> omega;  // [nshift]
    std::vector<double> sigma;  // [ncol][nshift], ascending per column
    std::vector<double> tolf;   // [nshift] factor on tol per shift (empty: 1)
    std::vector<double> ebw;    // [nshift] result-bound weights (empty: stop shift by shift)
    double tol = 1e-12;
    int max_iter = 1000;
    // workspace pieces
    ColState *st = nullptr;
    double *partial = nullptr;
    int *alldone = nullptr;
    void *r = nullptr, *p = nullptr, *t = nullptr, *y = nullptr, *x = nullptr, *ps = nullptr;
    int nblk_st = 0;
    // deferred shift updates: window state, the base direction at the
    // window's start and the stored residuals, per phase
    bool windowed = false;
    WinState *ws = nullptr;
    void *P0 = nullptr, *R = nullptr, *P0_lo = nullptr, *R_lo = nullptr;


    void carve(Arena &ar) {
        nblk_st = stencil_blocks(g);
        const int nb = nblk_st > INIT_BLOCKS ? nblk_st : INIT_BLOCKS;
        st = (ColState *)ar.take(sizeof(ColState) * ncol);
        partial = (double *)ar.take(sizeof(double) * 2 * (size_t)nb * ncol);
        alldone = (int *)ar.take(sizeof(int));
        const size_t vb = (size_t)12 * g.V * sizeof(double2) * ncol;
        r = ar.take(vb);
        p = ar.take(vb);
        t = ar.take(vb);
        if (store_x)
            x = ar.take(vb * nshift);
        else
            y = ar.take(vb);
        if (nshift > 1) ps = ar.take(vb * (nshift - 1));
        if (windowed) {
            ws = (WinState *)ar.take(sizeof(WinState) * ncol);
            P0 = ar.take(vb);
            R = ar.take(vb * WIN);
        }
        if (prec_lo >= 0) {
            const size_t vl = (size_t)12 * g.V * sizeof(float2) * ncol;
            r_lo = ar.take(vl);
            p_lo = ar.take(vl);
            t_lo = ar.take(vl);
            if (nshift > 1) ps_lo = ar.take(vl * (nshift - 1));
            if (windowed) {
                P0_lo = ar.take(vl);
                R_lo = ar.take(vl * WIN);
            }
        }
    }
};

struct RunStats {
    int iters = 0;
    int lo_iters = 0;  // iterations of the low-precision phase (launched; columns done earlier return)
    int status = BRI_OK;
    std::vector<ColState> fin;
};

// ------------------------------------------------------------ graph cache

// Instantiated graphs of a block of solver iterations, keyed by everything their launches
// depend on (device, geometry, precision, buffers, launch configuration).  Bounded; the
// oldest entry is destroyed first.  Capture runs on a library stream per device (capture
// is not possible on the null stream); the graph is then launched on the caller's stream.
// Each entry carries an event recorded after every launch of it, and an entry is destroyed
// only after that event has completed, so a graph another host thread launched on its own
// stream is never destroyed while it runs.
namespace {
constexpr size_t GRAPH_CACHE_MAX = 16;
struct CachedGraph {
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;  // recorded after each launch
};
std::mutex g_graph_mu;
bool g_graphs_on = true;
std::map<std::vector<uint64_t>, CachedGraph> g_graphs;
std::deque<std::vector<uint64_t>> g_graph_order;
std::map<int, hipStream_t> g_capture_streams;

void graph_release(CachedGraph &c) {
    if (c.done) {
        (void)hipEventSynchronize(c.done);  // the last launch has finished
        (void)hipEventDestroy(c.done);
    }
    if (c.exec) (void)hipGraphExecDestroy(c.exec);
    c = CachedGraph{};
}

void graph_cache_clear_locked() {
    for (auto &kv : g_graphs) graph_release(kv.second);
    g_graphs.clear();
    g_graph_order.clear();
}
}  // namespace

// Launches the graph cached under `key` on `strm`, capturing it first from `enqueue` if absent.
// The launch happens under the cache lock, so another host thread cannot evict (destroy) the
// executable graph between lookup and launch.
template <typename F>
static int graph_launch(const std::vector<uint64_t> &key, F enqueue, hipStream_t strm, bool *captured = nullptr) {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    auto it = g_graphs.find(key);
    if (captured) *captured = it == g_graphs.end();
    if (it != g_graphs.end()) {
        if (hipGraphLaunch(it->second.exec, strm) != hipSuccess) return BRI_EHIP;
        return hipEventRecord(it->second.done, strm) == hipSuccess ? BRI_OK : BRI_EHIP;
    }
    int dev = 0;
    BRI_HIP_CHECK(hipGetDevice(&dev));
    hipStream_t cs = g_capture_streams[dev];
    if (!cs) {
        BRI_HIP_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        g_capture_streams[dev] = cs;
    }
    BRI_HIP_CHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue(cs);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &graph);
    if (rc != BRI_OK || ec != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc != BRI_OK ? rc : BRI_EHIP;
    }
    CachedGraph c;
    const hipError_t ei = hipGraphInstantiate(&c.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return BRI_EHIP;
    if (hipEventCreateWithFlags(&c.done, hipEventDisableTiming) != hipSuccess) {
        c.done = nullptr;
        graph_release(c);
        return BRI_EHIP;
    }
    if (g_graphs.size() >= GRAPH_CACHE_MAX) {
        auto old = g_graph_order.front();
        g_graph_order.pop_front();
        graph_release(g_graphs[old]);
        g_graphs.erase(old);
    }
    g_graphs[key] = c;
    g_graph_order.push_back(key);
    if (hipGraphLaunch(c.exec, strm) != hipSuccess) return BRI_EHIP;
    return hipEventRecord(c.done, strm) == hipSuccess ? BRI_OK : BRI_EHIP;
}

// The pinned host word the solvers poll the all-done flag into: one per (host thread, device),
// allocated on first use and kept for the life of the thread (a page of pinned memory), so that no
// apply allocates or frees pinned memory on its path.
static int pinned_flag(int **out) {
    thread_local std::map<int, int *> flags;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return BRI_EHIP;
    auto it = flags.find(dev);
    if (it == flags.end()) {
        int *p = nullptr;
        if (hipHostMalloc((void **)&p, sizeof(int), hipHostMallocDefault) != hipSuccess) return BRI_EHIP;
        it = flags.emplace(dev, p).first;
    }
    *out = it->second;
    return BRI_OK;
}

static bool graphs_enabled() {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    return g_graphs_on;
}

// Runs one batched multi-shift solve; b is [ncol][12 V] complex double.  Returns a HIP /
// argument status; convergence and NaN status land in rs.
static int ms_run(MsSolve &s, const void *b, hipStream_t strm, int *hflag, RunStats &rs, bool allow_graphs = true) {
    if (s.prec != BRI_F64) return BRI_EINVAL;  // FP64 vectors; the low-precision phase has its own
    const size_t n = (size_t)12 * s.g.V;
    std::vector<ColState> h(s.ncol);
    for (int c = 0; c < s.ncol; ++c) {
        ColState &cs = h[c];
        std::memset(&cs, 0, sizeof(cs));
        cs.nshift = s.nshift;
        cs.c0 = s.c0;
        cs.sigma0 = s.sigma[(size_t)c * s.nshift];
        cs.joint = s.ebw.empty() ? 0 : 1;
        for (int i = 0; i < s.nshift; ++i) {
            cs.omega[i] = s.omega[i];
            cs.delta[i] = s.sigma[(size_t)c * s.nshift + i] - cs.sigma0;
            const double f = s.tolf.empty() ? 1.0 : s.tolf[i];
            cs.tolf2[i] = f * f;
            cs.ebw[i] = s.ebw.empty() ? 0.0 : s.ebw[i];
        }
    }
    BRI_HIP_CHECK(hipMemcpyAsync(s.st, h.data(), sizeof(ColState) * s.ncol, hipMemcpyHostToDevice, strm));
    const dim3 vgrid(INIT_BLOCKS, s.ncol);
    const dim3 ugrid(update_blocks(n), s.ncol);
    // (with deferred updates y and the p^sigma are c0 b and b until the first fold, which reads the
    // window's base direction P_0 = b in their place)
    hipLaunchKernelGGL((ms_init_kernel<double2, double2>), vgrid, dim3(256), 0, strm, n, (const double2 *)b,
                       (double2 *)s.r, (double2 *)s.p, s.windowed ? nullptr : (double2 *)s.y,
                       s.windowed ? nullptr : (double2 *)s.x, s.windowed ? nullptr : (double2 *)s.ps, s.ncol,
                       s.nshift, s.c0, s.partial);
    hipLaunchKernelGGL(ms_scalar_init_kernel, dim3(s.ncol), dim3(RED_THREADS), 0, strm, s.st, s.partial, INIT_BLOCKS,
                       s.tol);
    if (s.windowed) {
        BRI_HIP_CHECK(hipMemcpyAsync(s.P0, b, n * s.ncol * sizeof(double2), hipMemcpyDeviceToDevice, strm));
        hipLaunchKernelGGL(ms_window_reset_kernel, dim3(s.ncol), dim3(64), 0, strm, s.ws);
    }
    BRI_HIP_CHECK(hipGetLastError());

    // phase 0 runs at s.prec on (r, p, t, ps); phase 1 (FP64 solves with a low-precision phase)
    // on the FP32 vectors (r_lo, p_lo, t_lo, ps_lo) with the links Wlo, accumulating into the
    // FP64 y / x
    struct Phase {
        int prec;
        StencilConfig cfg;
        StencilArgs a1, a2;
        void *r, *p, *ps;
        void *P0, *R;  // deferred updates: base direction at the window's start, stored residuals
    };
    auto make_phase = [&](int prec, const void *W, void *r, void *p, void *t, void *ps, void *P0, void *R) {
        Phase ph;
        ph.prec = prec;
        ph.cfg = default_config(s.g, prec, s.ncol, s.kind);
        ph.a1 = StencilArgs{};
        ph.a1.g = s.g;
        ph.a1.W = W;
        ph.a1.ncol = s.ncol;
        ph.a1.in = p;
        ph.a1.out = t;
        ph.a1.kind = s.kind;
        ph.a1.diag = kernel_diag(s.kind) + s.m0;
        ph.a1.partial = s.partial;
        ph.a1.st = s.st;
        ph.a2 = ph.a1;
        ph.a2.in = t;
        ph.a2.out = nullptr;
        ph.a2.p = p;
        ph.a2.r = r;
        ph.r = r;
        ph.p = p;
        ph.ps = ps;
        ph.P0 = P0;
        ph.R = R;
        return ph;
    };
    const bool has_lo = s.prec == BRI_F64 && s.prec_lo >= 0;
    Phase phases[2] = {make_phase(s.prec, s.W, s.r, s.p, s.t, s.ps, s.P0, s.R),
                       has_lo ? make_phase(s.prec_lo, s.Wlo, s.r_lo, s.p_lo, s.t_lo, s.ps_lo, s.P0_lo, s.R_lo)
                              : Phase{}};
    const double sw2 = has_lo ? s.lo_switch * s.lo_switch : 0.0;

    // one CG iteration for every column: t = X p, alpha, r update, beta, vector updates, done flags
    auto iteration = [&](const Phase &ph, bool lo, hipStream_t q) -> int {
        const int e1 = stencil_launch(ph.a1, ph.prec, false, EPI_NORMS, ph.cfg, q);
        hipLaunchKernelGGL(ms_alpha_kernel, dim3(s.ncol), dim3(RED_THREADS), 0, q, s.st, s.partial, s.nblk_st);
        const int e2 = stencil_launch(ph.a2, ph.prec, true, EPI_CG_R, ph.cfg, q);
        hipLaunchKernelGGL(ms_beta_kernel, dim3(s.ncol), dim3(RED_THREADS), 0, q, s.st, s.partial, s.nblk_st,
                           s.windowed ? s.ws : nullptr, s.store_x ? 1 : 0);
        if (s.windowed && !lo)
            hipLaunchKernelGGL((ms_pupdate_kernel<double2>), ugrid, dim3(256), 0, q, s.st, s.ws, n, s.ncol,
                               (const double2 *)ph.r, (double2 *)ph.p, (double2 *)ph.R);
        else if (s.windowed)
            hipLaunchKernelGGL((ms_pupdate_kernel<float2>), ugrid, dim3(256), 0, q, s.st, s.ws, n, s.ncol,
                               (const float2 *)ph.r, (float2 *)ph.p, (float2 *)ph.R);
        else if (!lo)
            hipLaunchKernelGGL((ms_update_kernel<double2, double2>), ugrid, dim3(256), 0, q, s.st, n, s.ncol,
                               (const double2 *)ph.r, (double2 *)ph.p, (double2 *)s.y, (double2 *)s.x,
                               (double2 *)ph.ps);
        else
            hipLaunchKernelGGL((ms_update_kernel<float2, double2>), ugrid, dim3(256), 0, q, s.st, n, s.ncol,
                               (const float2 *)ph.r, (float2 *)ph.p, (double2 *)s.y, (double2 *)s.x,
                               (float2 *)ph.ps);
        hipLaunchKernelGGL(ms_finish_kernel, dim3(1), dim3(256), 0, q, s.st, s.ncol, s.alldone, lo ? 0.0 : sw2);
        if (e1 != BRI_OK || e2 != BRI_OK) return e1 != BRI_OK ? e1 : e2;
        return hipGetLastError() == hipSuccess ? BRI_OK : BRI_EHIP;
    };
    // rounds phase 0's r, p, p^sigma into phase 1's FP32 vectors
    auto narrow = [&]() -> int {
        const size_t cnt = n * s.ncol;
        hipLaunchKernelGGL(narrow_kernel, dim3(4096), dim3(256), 0, strm, cnt, (const double2 *)s.r, (float2 *)s.r_lo);
        hipLaunchKernelGGL(narrow_kernel, dim3(4096), dim3(256), 0, strm, cnt, (const double2 *)s.p, (float2 *)s.p_lo);
        if (s.nshift > 1)
            hipLaunchKernelGGL(narrow_kernel, dim3(4096), dim3(256), 0, strm, cnt * (s.nshift - 1),
                               (const double2 *)s.ps, (float2 *)s.ps_lo);
        return hipGetLastError() == hipSuccess ? BRI_OK : BRI_EHIP;
    };
    // deferred updates: materialise y and the p^sigma of the phase's window, then empty it
    // (first: no fold yet, so P_0 = b stands for y / c0 and every direction)
    double2 *xv = s.store_x ? (double2 *)s.x : nullptr;
    auto fold = [&](const Phase &ph, bool lo, hipStream_t q, int first) -> int {
        if (!lo)
            hipLaunchKernelGGL((ms_fold_kernel<double2, double2>), ugrid, dim3(256), 0, q, s.st, s.ws, n, s.ncol,
                               (const double2 *)ph.R, (const double2 *)ph.p, (const double2 *)ph.P0,
                               (double2 *)ph.P0, (const double2 *)ph.ps, (double2 *)ph.ps, (double2 *)s.y, xv, 0,
                               first);
        else
            hipLaunchKernelGGL((ms_fold_kernel<float2, float2>), ugrid, dim3(256), 0, q, s.st, s.ws, n, s.ncol,
                               (const float2 *)ph.R, (const float2 *)ph.p, (const float2 *)ph.P0, (float2 *)ph.P0,
                               (const float2 *)ph.ps, (float2 *)ph.ps, (double2 *)s.y, xv, 0, first);
        hipLaunchKernelGGL(ms_window_reset_kernel, dim3(s.ncol), dim3(64), 0, q, s.ws);
        return hipGetLastError() == hipSuccess ? BRI_OK : BRI_EHIP;
    };
    // the switch to the low-precision phase with deferred updates: the fold writes the FP32
    // p^sigma and base direction from the FP64 window, then r and p are rounded
    auto fold_switch = [&](int first) -> int {
        hipLaunchKernelGGL((ms_fold_kernel<double2, float2>), ugrid, dim3(256), 0, strm, s.st, s.ws, n, s.ncol,
                           (const double2 *)s.R, (const double2 *)s.p, (const double2 *)s.P0, (float2 *)s.P0_lo,
                           (const double2 *)s.ps, (float2 *)s.ps_lo, (double2 *)s.y, xv, 1, first);
        hipLaunchKernelGGL(ms_window_reset_kernel, dim3(s.ncol), dim3(64), 0, strm, s.ws);
        const size_t cnt = n * s.ncol;
        hipLaunchKernelGGL(narrow_kernel, dim3(4096), dim3(256), 0, strm, cnt, (const double2 *)s.r, (float2 *)s.r_lo);
        hipLaunchKernelGGL(narrow_kernel, dim3(4096), dim3(256), 0, strm, cnt, (const double2 *)s.p, (float2 *)s.p_lo);
        return hipGetLastError() == hipSuccess ? BRI_OK : BRI_EHIP;
    };
    const bool use_graph = allow_graphs && graphs_enabled();
    std::vector<uint64_t> key0;
    if (use_graph) {
        int dev = 0;
        BRI_HIP_CHECK(hipGetDevice(&dev));
        // everything the captured launches bake in: geometry (with the clover switch), precision,
        // kernel, mass, every buffer address and the launch configuration
        uint64_t m0bits, cswbits, swbits;
        std::memcpy(&m0bits, &s.m0, sizeof(m0bits));
        std::memcpy(&cswbits, &s.g.csw, sizeof(cswbits));
        std::memcpy(&swbits, &sw2, sizeof(swbits));
        key0 = {(uint64_t)dev, (uint64_t)s.g.L[0], (uint64_t)s.g.L[1], (uint64_t)s.g.L[2], (uint64_t)s.g.L[3],
                (uint64_t)s.g.tbc, cswbits, (uint64_t)s.prec, (uint64_t)s.kind, (uint64_t)s.ncol, m0bits,
                (uint64_t)(uintptr_t)s.W, (uint64_t)(uintptr_t)s.st, (uint64_t)(uintptr_t)s.partial,
                (uint64_t)(uintptr_t)s.alldone, (uint64_t)(uintptr_t)s.r, (uint64_t)(uintptr_t)s.p,
                (uint64_t)(uintptr_t)s.t, (uint64_t)(uintptr_t)s.y, (uint64_t)(uintptr_t)s.x,
                (uint64_t)(uintptr_t)s.ps, (uint64_t)(int64_t)s.prec_lo, (uint64_t)(uintptr_t)s.Wlo,
                (uint64_t)(uintptr_t)s.r_lo, (uint64_t)(uintptr_t)s.p_lo, (uint64_t)(uintptr_t)s.t_lo,
                (uint64_t)(uintptr_t)s.ps_lo, swbits, (uint64_t)s.windowed, (uint64_t)(uintptr_t)s.ws,
                (uint64_t)(uintptr_t)s.P0, (uint64_t)(uintptr_t)s.R, (uint64_t)(uintptr_t)s.P0_lo,
                (uint64_t)(uintptr_t)s.R_lo};
    }
    auto key_of = [&](int phase, int nblock, int win_at, int first) {
        std::vector<uint64_t> k = key0;
        const StencilConfig &cfg = phases[phase].cfg;
        for (uint64_t v : {(uint64_t)phase, (uint64_t)nblock, (uint64_t)cfg.tile[0], (uint64_t)cfg.tile[1],
                           (uint64_t)cfg.tile[2], (uint64_t)cfg.tile[3], (uint64_t)cfg.colz, (uint64_t)cfg.coly, (uint64_t)cfg.nsplit,
                           (uint64_t)cfg.rpt, (uint64_t)cfg.xcd_remap, (uint64_t)cfg.variant, (uint64_t)win_at,
                           (uint64_t)first})
            k.push_back(v);
        return k;
    };
    // the switch to the low-precision phase
    bool first_window = s.windowed;  // no fold yet
    auto to_low = [&]() -> int {
        if (!s.windowed) return narrow();
        const int e = fold_switch(first_window ? 1 : 0);
        first_window = false;
        return e;
    };

    // a solve whose tolerance is already within the low precision's reach starts in phase 1
    int phase = 0;
    if (has_lo && s.lo_switch >= 1.0) {
        const int e = to_low();
        if (e != BRI_OK) return e;
        phase = 1;
    }
    int it = 0, it_switch = 0;
    int since_fold = 0;  // iterations launched since the window was last folded
    rs.lo_iters = 0;
    double sec_per_iter = 0.0;  // host wall time per iteration of the last polling block
    for (;;) {
        // shorter polling blocks while the switch to the low-precision phase is pending: one
        // iteration per poll once iterations are long enough that a host round trip (tens of us)
        // costs little against them, so the switch comes at the first iteration that allows it
        int blk = CHECK_EVERY;
        if (phase == 0 && has_lo) blk = sec_per_iter > LONG_ITER_SEC ? 1 : CHECK_EVERY / 2;
        const auto tb = std::chrono::steady_clock::now();
        const int it_before = it;
        const Phase &ph = phases[phase];
        const bool lo = phase == 1;
        // one iteration, then the fold whenever the window is full (every WIN iterations)
        auto step = [&](int &sf, bool &fw, hipStream_t q) -> int {
            int e = iteration(ph, lo, q);
            if (e == BRI_OK && s.windowed && ++sf == WIN) {
                e = fold(ph, lo, q, fw ? 1 : 0);
                sf = 0;
                fw = false;
            }
            return e;
        };
        bool captured = false;  // a block whose graph was captured now: its time is not an iteration's
        if (use_graph && it + blk <= s.max_iter) {
            const int at = since_fold;
            const bool fw0 = first_window;
            const int rc = graph_launch(
                key_of(phase, blk, s.windowed ? at : 0, fw0 ? 1 : 0),
                [&](hipStream_t q) -> int {
                    int sf = at;
                    bool fw = fw0;
                    for (int k = 0; k < blk; ++k) {
                        const int e = step(sf, fw, q);
                        if (e != BRI_OK) return e;
                    }
                    return BRI_OK;
                },
                strm, &captured);
            if (rc != BRI_OK) return rc;
            it += blk;
            if (s.windowed) {
                if (first_window && at + blk >= WIN) first_window = false;  // the block folded
                since_fold = (since_fold + blk) % WIN;
            }
        } else {
            for (int k = 0; k < blk && it < s.max_iter; ++k, ++it) {
                const int e = step(since_fold, first_window, strm);
                if (e != BRI_OK) return e;
            }
        }
        BRI_HIP_CHECK(hipMemcpyAsync(hflag, s.alldone, sizeof(int), hipMemcpyDeviceToHost, strm));
        BRI_HIP_CHECK(hipStreamSynchronize(strm));
        if (it > it_before && !captured)
            sec_per_iter = std::chrono::duration<double>(std::chrono::steady_clock::now() - tb).count() /
                           (it - it_before);
        if (*hflag == 1 || it >= s.max_iter) break;
        if (*hflag == 2 && phase == 0 && has_lo) {
            // iterations done so far (the last of a polling block may find a column done)
            std::vector<ColState> cur(s.ncol);
            BRI_HIP_CHECK(hipMemcpyAsync(cur.data(), s.st, sizeof(ColState) * s.ncol, hipMemcpyDeviceToHost, strm));
            BRI_HIP_CHECK(hipStreamSynchronize(strm));
            for (const ColState &c : cur) it_switch = c.iter > it_switch ? c.iter : it_switch;
            const int e = to_low();
            if (e != BRI_OK) return e;
            since_fold = 0;
            phase = 1;
        }
    }
    // the last window's steps into y (and y itself, if no fold has written it yet)
    if (s.windowed && (since_fold > 0 || first_window)) {
        const int e = fold(phases[phase], phase == 1, strm, first_window ? 1 : 0);
        if (e != BRI_OK) return e;
    }
    rs.fin.resize(s.ncol);
    BRI_HIP_CHECK(hipMemcpyAsync(rs.fin.data(), s.st, sizeof(ColState) * s.ncol, hipMemcpyDeviceToHost, strm));
    BRI_HIP_CHECK(hipStreamSynchronize(strm));
    rs.iters = 0;
    rs.status = BRI_OK;
    for (const ColState &c : rs.fin) {
        if (c.iter > rs.iters) rs.iters = c.iter;
        if (phase == 1 && c.iter - it_switch > rs.lo_iters) rs.lo_iters = c.iter - it_switch;
        if (c.status == BRI_ENAN)
            rs.status = BRI_ENAN;
        else if (c.done == 0 && rs.status == BRI_OK)
            rs.status = BRI_ENOCONV;
    }
    return BRI_OK;
}

// ---------------------------------------------------------------- overlap

// The multi-shift solve behind an overlap apply or the gradient: FP64, or FP64 with a low-
// precision phase for inner = BRI_F32 / BRI_F32_BF16W, entered once the base residual has
// fallen to tol / u_lo (u_lo the inner precision's unit roundoff; at once when that exceeds 1).
// i0, i1: the shifts [i0, i1) of the rational only (the gradient's recompute mode); -1: all.
static void plan_shifts(MsSolve &m, const Geom &g, const ov_params *prm, int ncol, const void *W64, const void *Wlo,
                        bool store_x, int i0 = -1, int i1 = -1) {
    double om_all[MAXS], sg_all[MAXS], tf_all[MAXS];
    shift_coeffs(prm, &m.c0, om_all, sg_all, tf_all);
    if (i0 < 0) {
        i0 = 0;
        i1 = prm->kl_n;
    }
    const int n = i1 - i0;
    const double *om = om_all + i0, *sg = sg_all + i0, *tf = tf_all + i0;
    m.g = g;
    m.prec = BRI_F64;
    m.W = W64;
    m.m0 = -prm->rho;
    m.kind = prm->kernel;
    m.ncol = ncol;
    m.nshift = n;
    m.store_x = store_x;
    m.omega.assign(om, om + n);
    m.tolf.assign(tf, tf + n);
    m.ebw.clear();
    if (prm->relax == 2)  // |X (X^dag X + sigma)^-1| <= max_s s / (s^2 + sigma) = 1 / (2 sqrt(sigma))
        for (int i = 0; i < n; ++i) m.ebw.push_back(om[i] / (2.0 * sqrt(sg[i])));
    m.sigma.resize((size_t)ncol * n);
    for (int c = 0; c < ncol; ++c)
        for (int i = 0; i < n; ++i) m.sigma[(size_t)c * n + i] = sg[i];
    m.tol = prm->tol;
    m.max_iter = prm->max_iter;
    if (prm->inner != BRI_F64) {
        m.prec_lo = prm->inner;
        m.Wlo = Wlo;
        const double sw = prm->tol / unit_roundoff(prm->inner);
        m.lo_switch = sw < 1.0 ? sw : 1.0;
    }
}

// iterations and residual per shift, the worst column of the solve
static void fill_stats(const RunStats &rs, int n, ov_stats *st) {
    st->iters = rs.iters;
    st->refine = rs.lo_iters;
    for (int i = 0; i < n; ++i) {
        int it = 0;
        double res = 0.0;
        for (const ColState &c : rs.fin) {
            const int ci = c.conv_iter[i] ? c.conv_iter[i] : c.iter;
            const double cr =
                c.conv_iter[i] ? c.conv_res[i] : fabs(c.zeta[i]) * sqrt(c.rr / (c.bnorm2 > 0 ? c.bnorm2 : 1));
            if (ci > it) it = ci;
            if (cr > res) res = cr;
        }
        st->shift_iters[i] = it;
        st->rel_resid[i] = res;
    }
}

// Static workspace of the entry point that allocates nothing (ov_apply_noalloc): one per GPU,
// held until the process ends, resolved once per device with hipGetSymbolAddress (the array's
// name is only a host-side stand-in).  Every call on a GPU shares it.
constexpr size_t SCRATCH_BYTES = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];
constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[SCRATCH_MAX_DEVICES];

// device address of the current device's scratch array (resolved on the first call per device)
static int scratch_address(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return BRI_EHIP;
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return BRI_EINVAL;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return BRI_EHIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return BRI_OK;
}

// noalloc: the workspace is the static scratch (work / work_bytes ignored), the polling word a
// host variable, and the CG loop is launched without HIP graphs (instantiating one allocates)
static int ov_impl(const bri_geom *geom, const void *W64, const void *Wlo, const ov_params *prm, const void *in,
                   void *out, int nrhs, void *work, size_t *work_bytes, ov_stats *stats, void *stream,
                   bool overlap, bool noalloc = false) {
    const auto t0 = std::chrono::steady_clock::now();
    Geom g;
    int rc = geom_check(geom, &g);
    if (rc != BRI_OK) return rc;
    if (!prm || (!work_bytes && !noalloc)) return BRI_EINVAL;
    const int n = prm->kl_n;
    if (!params_ok(prm)) return BRI_EINVAL;
    if (g.V % 64 || nrhs < 1 || nrhs > 4096) return BRI_EINVAL;
    const bool mixed = prm->inner != BRI_F64;
    MsSolve m;
    plan_shifts(m, g, prm, nrhs, W64, Wlo, false);
    m.windowed = !noalloc;  // (the static scratch holds the per-iteration form only)
    size_t scratch_bytes = 0;
    if (noalloc) {
        Arena ar(nullptr);
        m.carve(ar);
        if (ar.used > SCRATCH_BYTES) return BRI_ESCRATCH;
        rc = scratch_address(&work);
        if (rc != BRI_OK) return rc;
        scratch_bytes = SCRATCH_BYTES;
        work_bytes = &scratch_bytes;
    }
    {
        Arena ar(nullptr);
        m.carve(ar);
        if (!work) {
            *work_bytes = ar.used;
            return BRI_OK;
        }
        if (*work_bytes < ar.used || !W64 || !in || !out || (mixed && !Wlo)) return BRI_EINVAL;
        const size_t vb = (size_t)12 * g.V * nrhs * sizeof(double2);
        if (ranges_overlap(in, vb, out, vb) || ranges_overlap(in, vb, work, ar.used) ||
            ranges_overlap(out, vb, work, ar.used))
            return BRI_EINVAL;
    }
    Arena ar(work);
    m.carve(ar);
    hipStream_t s = (hipStream_t)stream;

    int *hflag = nullptr, host_flag = 0;
    if (noalloc)
        hflag = &host_flag;
    else if (pinned_flag(&hflag) != BRI_OK)
        return BRI_EHIP;
    RunStats rs;
    rc = ms_run(m, in, s, hflag, rs, !noalloc);
    int result = rc != BRI_OK ? rc : rs.status;
    if (result == BRI_OK || result == BRI_ENOCONV) {  // (the best iterate on ENOCONV)
        // out = rho (b + X y)  or  gamma5 X y, in FP64
        StencilArgs a3{};
        a3.g = g;
        a3.W = W64;
        a3.ncol = nrhs;
        a3.in = m.y;
        a3.out = out;
        a3.kind = prm->kernel;
        a3.diag = kernel_diag(prm->kernel) - prm->rho;
        a3.b = in;
        a3.rho = prm->rho;
        rc = stencil_launch(a3, BRI_F64, false, overlap ? EPI_OV : EPI_SIGN,
                            default_config(g, BRI_F64, nrhs, prm->kernel), s);
        if (rc != BRI_OK && result == BRI_OK) result = rc;
    }
    if (hipStreamSynchronize(s) != hipSuccess) result = BRI_EHIP;
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        if (!rs.fin.empty()) fill_stats(rs, n, stats);
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return result;
}

// Multi-shift solve of (A + sigma_i) x_i = b over the Kenney-Laub shifts i0 <= i < i1 (all for
// i0 = -1) with every x_i kept in FP64, [shift][ncol][12 V] inside the workspace (the gradient
// needs the individual shift solutions).  inner = BRI_F64 runs it in FP64; a low-precision inner relaxes the precision
// of the late iterations as the overlap apply does.  With work == NULL only *need is set.
// st (may be NULL) receives iterations and the final residual of each shift (the worst column).
int ov_solve_shifts(const Geom &g, const void *W64, const void *Wlo, const ov_params *prm, const void *b, int ncol,
                    void *work, size_t work_bytes, size_t *need, hipStream_t s, void **x_out, ov_stats *st, int i0,
                    int i1) {
    if (prm->kl_n < 1 || prm->kl_n > MAXS || ncol < 1) return BRI_EINVAL;
    if (i0 < 0) {
        i0 = 0;
        i1 = prm->kl_n;
    }
    if (i1 <= i0 || i1 > prm->kl_n) return BRI_EINVAL;
    const int n = i1 - i0;
    const bool mixed = prm->inner != BRI_F64;
    MsSolve m;
    plan_shifts(m, g, prm, ncol, W64, Wlo, true, i0, i1);
    m.windowed = true;
    Arena ar(work);
    m.carve(ar);
    if (!work) {
        if (need) *need = ar.used;
        return BRI_OK;
    }
    if (work_bytes < ar.used || !W64 || !b || !x_out || (mixed && !Wlo)) return BRI_EINVAL;
    int *hflag = nullptr;
    if (pinned_flag(&hflag) != BRI_OK) return BRI_EHIP;
    RunStats rs;
    const int rc = ms_run(m, b, s, hflag, rs);
    const int result = rc != BRI_OK ? rc : rs.status;
    if (result != BRI_OK && result != BRI_ENOCONV) return result;
    *x_out = m.x;
    if (st) {
        std::memset(st, 0, sizeof(*st));
        fill_stats(rs, n, st);
    }
    return result;
}

}  // namespace bri

extern "C" {

int bri_set_solver_graphs(int enable) {
    if (enable != 0 && enable != 1) return BRI_EINVAL;
    std::lock_guard<std::mutex> lk(bri::g_graph_mu);
    bri::g_graphs_on = enable == 1;
    if (!bri::g_graphs_on) bri::graph_cache_clear_locked();
    return BRI_OK;
}

int bri_kl_upper_coeffs(int n, double *omega, double *sigma) {
    if (n < 1 || n > BRI_MAX_SHIFTS || !omega || !sigma) return BRI_EINVAL;
    bri::kl_upper_coeffs(n, omega, sigma);
    return BRI_OK;
}

int bri_kl_coeffs(int n, double *c0, double *omega, double *sigma) {
    if (n < 1 || n > BRI_MAX_SHIFTS || !c0 || !omega || !sigma) return BRI_EINVAL;
    bri::kl_coeffs(n, c0, omega, sigma);
    return BRI_OK;
}

int ov_sign_apply(const bri_geom *geom, const void *W64, const void *Wlo, const ov_params *params, const void *in,
                  void *out, int nrhs, void *work, size_t *work_bytes, ov_stats *stats, void *stream) {
    return bri::ov_impl(geom, W64, Wlo, params, in, out, nrhs, work, work_bytes, stats, stream, false);
}

int ov_apply(const bri_geom *geom, const void *W64, const void *Wlo, const ov_params *params, const void *in,
             void *out, int nrhs, void *work, size_t *work_bytes, ov_stats *stats, void *stream) {
    return bri::ov_impl(geom, W64, Wlo, params, in, out, nrhs, work, work_bytes, stats, stream, true);
}

int ov_apply_noalloc(const bri_geom *geom, const void *W64, const void *Wlo, const ov_params *params, const void *in,
                     void *out, int nrhs, ov_stats *stats, void *stream) {
    return bri::ov_impl(geom, W64, Wlo, params, in, out, nrhs, nullptr, nullptr, stats, stream, true, true);
}

size_t ov_noalloc_max_bytes(void) { return bri::SCRATCH_BYTES; }

}  // extern "C"
