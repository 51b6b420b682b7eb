// Overlap operator apply: D_ov psi = rho (psi + X r_n(X^dag X) psi), X = D_bri(-rho)
// (eq. (def_over)), with the Kenney-Laub partial fractions
//   r_n(t) = c0 + sum_i omega_i / (t + sigma_i)            (eq. (KLnn_parfrac))
// evaluated by one multi-shift conjugate gradient on A + sigma_0, A = X^dag X,
// sigma_0 the smallest shift (Sec. 3.3).
//
// Multi-shift CG (Krylov space shared by all shifted systems).  The base
// system (A + sigma_0) x = b runs plain CG:
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
// |zeta^sigma| |r| <= tol |b|.  Only y = c0 b + sum_sigma omega_sigma x^sigma is
// needed, so the x^sigma are never stored: y accumulates omega_sigma alpha^sigma p^sigma.
// The base shift has zeta = 1, so its search direction is p itself.
//
// All scalars live on the device (MsState) and are updated by single-block
// kernels; the host only polls the `done` flag every few iterations, and every
// loop kernel returns at once when `done` is set.
#include <math.h>

#include <chrono>
#include <cstring>

#include "stencil.hpp"

namespace bri {

constexpr int MAXS = BRI_MAX_SHIFTS;
constexpr int RED_THREADS = 256;
constexpr int CHECK_EVERY = 8;

struct MsState {
    double rr, bnorm2, tol2;
    double alpha, alpha_old, beta, beta_old;
    double sigma0;
    int iter, done, status, nshift;
    double c0;
    double delta[MAXS], omega[MAXS];
    double zeta[MAXS], zeta_old[MAXS], zeta_new[MAXS];
    double alpha_s[MAXS], beta_s[MAXS];
    int active[MAXS];       // shift still iterating
    int upd_x[MAXS];        // shift contributes alpha^sigma p^sigma in this iteration
    int conv_iter[MAXS];
    double conv_res[MAXS];  // |zeta r| / |b| when the shift stopped
};

// --------------------------------------------------------------- reductions

// deterministic sum of n partials (stride 2, component comp) by one block
__device__ double block_sum(const double *partial, int n, int comp) {
    __shared__ double sh[RED_THREADS];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += RED_THREADS) s += partial[2 * i + comp];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// ------------------------------------------------------------------ kernels

// r = p = b, p_sigma = b (sigma >= 1), y = c0 b; partial |b|^2
template <typename C>
__global__ void ms_init_kernel(size_t n, const C *__restrict__ b, C *__restrict__ r, C *__restrict__ p,
                               C *__restrict__ y, C *__restrict__ ps, int nps, double c0, double *partial) {
    double s = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const C v = b[i];
        r[i] = v;
        p[i] = v;
        y[i].x = c0 * v.x;
        y[i].y = c0 * v.y;
        for (int k = 0; k < nps; ++k) ps[(size_t)k * n + i] = v;
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
        partial[2 * blockIdx.x] = sh[0];
        partial[2 * blockIdx.x + 1] = 0.0;
    }
}

__global__ void ms_scalar_init_kernel(MsState *st, const double *partial, int nblk, double tol) {
    const double b2 = block_sum(partial, nblk, 0);
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

// alpha and the shifted alpha^sigma after t = X p (partials: |t|^2, |p|^2)
__global__ void ms_alpha_kernel(MsState *st, const double *partial, int nblk) {
    if (st->done) return;
    const double tt = block_sum(partial, nblk, 0);
    const double pp = block_sum(partial, nblk, 1);
    if (threadIdx.x == 0) {
        const double pAp = tt + st->sigma0 * pp;
        const double alpha = st->rr / pAp;
        if (!isfinite(alpha) || pAp <= 0.0) {
            st->status = BRI_ENAN;
            st->done = 1;
            for (int i = 0; i < st->nshift; ++i) st->upd_x[i] = 0;
            return;
        }
        st->alpha = alpha;
        for (int i = 0; i < st->nshift; ++i) {
            st->upd_x[i] = st->active[i];
            if (!st->active[i]) continue;
            const double z = st->zeta[i], zo = st->zeta_old[i];
            const double den =
                alpha * st->beta_old * (zo - z) + zo * st->alpha_old * (1.0 + st->delta[i] * alpha);
            const double zn = z * zo * st->alpha_old / den;
            st->zeta_new[i] = zn;
            st->alpha_s[i] = alpha * zn / z;
        }
    }
}

// beta, beta^sigma, convergence after r -= alpha (A + sigma0) p (partials: |r|^2)
__global__ void ms_beta_kernel(MsState *st, const double *partial, int nblk) {
    if (st->done) return;
    const double rr_new = block_sum(partial, nblk, 0);
    if (threadIdx.x == 0) {
        const int it = st->iter + 1;
        st->iter = it;
        if (!isfinite(rr_new)) {
            st->status = BRI_ENAN;
            st->done = 1;
            for (int i = 0; i < st->nshift; ++i) st->active[i] = 0;
            return;
        }
        const double beta = rr_new / st->rr;
        int any = 0;
        for (int i = 0; i < st->nshift; ++i) {
            if (!st->active[i]) continue;
            const double ratio = st->zeta_new[i] / st->zeta[i];
            st->beta_s[i] = beta * ratio * ratio;
            st->zeta_old[i] = st->zeta[i];
            st->zeta[i] = st->zeta_new[i];
            const double res2 = st->zeta[i] * st->zeta[i] * rr_new;
            if (res2 <= st->tol2) {
                st->active[i] = 0;
                st->conv_iter[i] = it;
                st->conv_res[i] = sqrt(res2 / st->bnorm2);
            } else {
                any = 1;
            }
        }
        st->alpha_old = st->alpha;
        st->beta_old = beta;
        st->beta = beta;
        st->rr = rr_new;
        if (!any) st->done = 2;  // converged: the last vector update still runs
    }
}

// y += sum_sigma omega alpha^sigma p^sigma (base shift: p); then
// p^sigma = zeta^sigma r + beta^sigma p^sigma, p = r + beta p
template <typename C>
__global__ void ms_update_kernel(const MsState *__restrict__ st, size_t n, const C *__restrict__ r,
                                 C *__restrict__ p, C *__restrict__ y, C *__restrict__ ps) {
    const int done = st->done;
    if (done == 1) return;
    const int ns = st->nshift;
    const double beta = st->beta;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const C ri = r[i];
        C pi = p[i];
        C yi = y[i];
        if (st->upd_x[0]) {
            const double w = st->omega[0] * st->alpha_s[0];
            yi.x += w * pi.x;
            yi.y += w * pi.y;
        }
        for (int k = 1; k < ns; ++k) {
            if (!st->upd_x[k]) continue;
            C *pk = ps + (size_t)(k - 1) * n;
            C v = pk[i];
            const double w = st->omega[k] * st->alpha_s[k];
            yi.x += w * v.x;
            yi.y += w * v.y;
            if (st->active[k]) {
                const double z = st->zeta[k], bs = st->beta_s[k];
                v.x = z * ri.x + bs * v.x;
                v.y = z * ri.y + bs * v.y;
                pk[i] = v;
            }
        }
        y[i] = yi;
        if (done == 0) {
            pi.x = ri.x + beta * pi.x;
            pi.y = ri.y + beta * pi.y;
            p[i] = pi;
        }
    }
}

__global__ void ms_finish_kernel(MsState *st) {
    if (st->done == 2) st->done = 1;
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

struct Workspace {
    size_t bytes;
    size_t off_state, off_partial, off_vec;
    int nblk_red;
};

static inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

static Workspace plan_workspace(const Geom &g, int nshift) {
    Workspace w;
    const size_t vec = (size_t)12 * g.V * sizeof(double2);
    const int nblk_st = stencil_blocks(g);
    const int nblk_init = 1024;
    w.nblk_red = nblk_st > nblk_init ? nblk_st : nblk_init;
    w.off_state = 0;
    w.off_partial = align256(sizeof(MsState));
    w.off_vec = align256(w.off_partial + sizeof(double) * 2 * (size_t)w.nblk_red);
    // r, p, t, y, and nshift - 1 shifted directions
    w.bytes = w.off_vec + align256(vec) * (size_t)(4 + nshift - 1);
    return w;
}

static int ov_impl(const bri_geom *geom, const void *W64, const void *Wlo, const ov_params *prm, const void *in,
                   void *out, int nrhs, void *work, size_t *work_bytes, ov_stats *stats, void *stream,
                   bool overlap) {
    const auto t0 = std::chrono::steady_clock::now();
    Geom g;
    int rc = geom_check(geom, &g);
    if (rc != BRI_OK) return rc;
    if (!prm || !work_bytes) return BRI_EINVAL;
    const int n = prm->kl_n;
    if (n < 1 || n > MAXS || !(prm->rho > 0.0 && prm->rho < 2.0) || !(prm->tol > 0.0) || prm->max_iter < 1)
        return BRI_EINVAL;
    if (prm->inner != BRI_F64 || prm->max_refine != 0) return BRI_EINVAL;
    if (g.V % 64 || nrhs < 1) return BRI_EINVAL;
    (void)Wlo;
    const Workspace ws = plan_workspace(g, n);
    if (!work) {
        *work_bytes = ws.bytes;
        return BRI_OK;
    }
    if (*work_bytes < ws.bytes || !W64 || !in || !out) return BRI_EINVAL;
    hipStream_t s = (hipStream_t)stream;

    char *base = (char *)work;
    MsState *st = (MsState *)(base + ws.off_state);
    double *partial = (double *)(base + ws.off_partial);
    const size_t vbytes = align256((size_t)12 * g.V * sizeof(double2));
    double2 *r = (double2 *)(base + ws.off_vec);
    double2 *p = (double2 *)(base + ws.off_vec + vbytes);
    double2 *t = (double2 *)(base + ws.off_vec + 2 * vbytes);
    double2 *y = (double2 *)(base + ws.off_vec + 3 * vbytes);
    double2 *ps = (double2 *)(base + ws.off_vec + 4 * vbytes);
    // ps is laid out with stride n = 12 V complex between shifts; vbytes is n * 16 rounded
    // to 256 bytes and 12 V * 16 is a multiple of 256 whenever V % 64 == 0.

    // coefficients, shifts ascending (sigma_0 smallest)
    MsState hst;
    std::memset(&hst, 0, sizeof(hst));
    double c0, om[MAXS], sg[MAXS];
    kl_coeffs(n, &c0, om, sg);
    hst.nshift = n;
    hst.c0 = c0;
    hst.sigma0 = sg[0];
    for (int i = 0; i < n; ++i) {
        hst.omega[i] = om[i];
        hst.delta[i] = sg[i] - sg[0];
    }

    const double m0 = -prm->rho;
    const StencilConfig cfg = default_config(g, BRI_F64);
    const int nblk = stencil_blocks(g);
    const size_t nel = (size_t)12 * g.V;
    const int vblocks = 1024;

    int *hdone = nullptr;
    BRI_HIP_CHECK(hipHostMalloc((void **)&hdone, 2 * sizeof(int), hipHostMallocDefault));
    int result = BRI_OK;
    MsState fin;
    for (int rhs = 0; rhs < nrhs && result != BRI_EHIP; ++rhs) {
        const double2 *b = (const double2 *)in + rhs * nel;
        double2 *o = (double2 *)out + rhs * nel;
        if (hipMemcpyAsync(st, &hst, sizeof(MsState), hipMemcpyHostToDevice, s) != hipSuccess) {
            result = BRI_EHIP;
            break;
        }
        hipLaunchKernelGGL(ms_init_kernel<double2>, dim3(vblocks), dim3(256), 0, s, nel, b, r, p, y, ps, n - 1, c0,
                           partial);
        hipLaunchKernelGGL(ms_scalar_init_kernel, dim3(1), dim3(RED_THREADS), 0, s, st, partial, vblocks,
                           prm->tol);
        if (hipGetLastError() != hipSuccess) {
            result = BRI_EHIP;
            break;
        }

        StencilArgs a1{};
        a1.g = g;
        a1.W = W64;
        a1.in = p;
        a1.out = t;
        a1.diag = 15.0 / 8.0 + m0;
        a1.partial = partial;
        a1.done = &st->done;
        StencilArgs a2 = a1;
        a2.in = t;
        a2.out = nullptr;
        a2.p = p;
        a2.r = r;
        a2.alpha = &st->alpha;
        a2.sigma0 = sg[0];

        int it = 0;
        bool finished = false;
        while (!finished) {
            for (int k = 0; k < CHECK_EVERY && it < prm->max_iter; ++k, ++it) {
                int e1 = stencil_launch(a1, BRI_F64, false, EPI_NORMS, 1, cfg, s);
                hipLaunchKernelGGL(ms_alpha_kernel, dim3(1), dim3(RED_THREADS), 0, s, st, partial, nblk);
                int e2 = stencil_launch(a2, BRI_F64, true, EPI_CG_R, 1, cfg, s);
                hipLaunchKernelGGL(ms_beta_kernel, dim3(1), dim3(RED_THREADS), 0, s, st, partial, nblk);
                hipLaunchKernelGGL(ms_update_kernel<double2>, dim3(vblocks), dim3(256), 0, s, st, nel, r, p, y,
                                   ps);
                hipLaunchKernelGGL(ms_finish_kernel, dim3(1), dim3(1), 0, s, st);
                if (e1 != BRI_OK || e2 != BRI_OK || hipGetLastError() != hipSuccess) {
                    result = BRI_EHIP;
                    break;
                }
            }
            if (result == BRI_EHIP) break;
            if (hipMemcpyAsync(hdone, &st->done, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                result = BRI_EHIP;
                break;
            }
            if (hdone[0] != 0 || it >= prm->max_iter) finished = true;
        }
        if (result == BRI_EHIP) break;

        // out = rho (b + X y)  or  gamma5 X y
        StencilArgs a3{};
        a3.g = g;
        a3.W = W64;
        a3.in = y;
        a3.out = o;
        a3.diag = 15.0 / 8.0 + m0;
        a3.b = b;
        a3.rho = prm->rho;
        if (stencil_launch(a3, BRI_F64, false, overlap ? EPI_OV : EPI_SIGN, 1, cfg, s) != BRI_OK) {
            result = BRI_EHIP;
            break;
        }
        if (hipMemcpyAsync(&fin, st, sizeof(MsState), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            result = BRI_EHIP;
            break;
        }
        if (fin.status == BRI_ENAN)
            result = BRI_ENAN;
        else if (fin.done == 0 && result == BRI_OK)
            result = BRI_ENOCONV;
        if (stats) {
            stats->iters = fin.iter;
            stats->refine = 0;
            for (int i = 0; i < MAXS; ++i) {
                stats->shift_iters[i] = i < n ? (fin.conv_iter[i] ? fin.conv_iter[i] : fin.iter) : 0;
                stats->rel_resid[i] =
                    i < n ? (fin.conv_iter[i] ? fin.conv_res[i]
                                              : fabs(fin.zeta[i]) * sqrt(fin.rr / (fin.bnorm2 > 0 ? fin.bnorm2 : 1)))
                          : 0.0;
            }
        }
    }
    (void)hipHostFree(hdone);
    if (stats)
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return result;
}

}  // namespace bri

extern "C" {

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

}  // extern "C"
