// Brillouin stencil y = D_bri(m0) x on gfx950 (App. C.1).
//
//   (D psi)(x) = (15/8 + m0) psi(x) + sum_{d != 0} S_d W_d(x) psi(x + d)
//   S_d = a_k + c_k sum_mu d_mu gamma_mu      (k = number of hops of d)
//
// Work decomposition.  A block owns a tile of 64 sites (one site per lane) and
// NSPLIT waves; wave q handles the stored link slabs j = q, q + NSPLIT, ...
// (uniform per wave, so the displacement, its weights and the branches on
// them live in scalar registers).  For each stored slab j the wave applies the
// pair of opposite displacements:
//   own:        S_{d}  W_j(x)            psi(x + d)
//   neighbour:  S_{-d} W_j(x - d)^dag    psi(x - d)
// so each stored link is read twice close together in time: once by its own
// site and once, as W^dag, by the site across the link, which is usually a
// lane of the same or an adjacent tile (L2 hit).  The NSPLIT partial sums meet
// in LDS; wave q then finishes 12/NSPLIT of the spin-colour components and runs
// the fused epilogue on them.
//
// The adjoint uses D^dag = gamma5 D gamma5, i.e. the same stencil with the
// derivative weights c_k negated (gamma5 anticommutes with every gamma_mu).
//
// Gamma matrices, chiral basis: gamma_k = [[0, -i s_k], [i s_k, 0]],
// gamma_4 = [[0, 1], [1, 0]].  Acting on the four spin components chi_s:
//   gamma_1 chi = (-i chi3, -i chi2,  i chi1,  i chi0)
//   gamma_2 chi = (  -chi3,    chi2,    chi1,   -chi0)
//   gamma_3 chi = (-i chi2,  i chi3,  i chi0, -i chi1)
//   gamma_4 chi = (   chi2,    chi3,    chi0,    chi1)
#include "stencil.hpp"

namespace bri {

template <typename C, typename R>
__device__ __forceinline__ void axpy_c(C &acc, R a, const C &v) {
    acc.x = fma(a, v.x, acc.x);
    acc.y = fma(a, v.y, acc.y);
}

// acc += i * a * v
template <typename C, typename R>
__device__ __forceinline__ void axpy_ic(C &acc, R a, const C &v) {
    acc.x = fma(-a, v.y, acc.x);
    acc.y = fma(a, v.x, acc.y);
}

// acc[s][c] += (a + sum_mu cmu gamma_mu) chi[s][c];  branches are wave-uniform.
template <typename C, typename R>
__device__ __forceinline__ void spin_accumulate(C (&acc)[4][3], const C (&chi)[4][3], R a, R c0, R c1, R c2, R c3) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int s = 0; s < 4; ++s) axpy_c(acc[s][c], a, chi[s][c]);
    }
    if (c0 != (R)0) {  // gamma_1 (x)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            axpy_ic(acc[0][c], -c0, chi[3][c]);
            axpy_ic(acc[1][c], -c0, chi[2][c]);
            axpy_ic(acc[2][c], c0, chi[1][c]);
            axpy_ic(acc[3][c], c0, chi[0][c]);
        }
    }
    if (c1 != (R)0) {  // gamma_2 (y)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            axpy_c(acc[0][c], -c1, chi[3][c]);
            axpy_c(acc[1][c], c1, chi[2][c]);
            axpy_c(acc[2][c], c1, chi[1][c]);
            axpy_c(acc[3][c], -c1, chi[0][c]);
        }
    }
    if (c2 != (R)0) {  // gamma_3 (z)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            axpy_ic(acc[0][c], -c2, chi[2][c]);
            axpy_ic(acc[1][c], c2, chi[3][c]);
            axpy_ic(acc[2][c], c2, chi[0][c]);
            axpy_ic(acc[3][c], -c2, chi[1][c]);
        }
    }
    if (c3 != (R)0) {  // gamma_4 (t)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            axpy_c(acc[0][c], c3, chi[2][c]);
            axpy_c(acc[1][c], c3, chi[3][c]);
            axpy_c(acc[2][c], c3, chi[0][c]);
            axpy_c(acc[3][c], c3, chi[1][c]);
        }
    }
}

template <class LS, bool ADJ>
__device__ __forceinline__ void transport(typename Cx<typename LS::R>::T (&chi)[4][3],
                                          const typename LS::store_t *__restrict__ Wj, unsigned ws,
                                          const typename Cx<typename LS::R>::T *__restrict__ ps, unsigned ys,
                                          unsigned V) {
    using R = typename LS::R;
    using C = typename Cx<R>::T;
    C w[3][3], p[4][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) w[a][b] = LS::load(Wj, (size_t)(a * 3 + b) * V + ws);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int b = 0; b < 3; ++b) p[s][b] = ps[(size_t)(s * 3 + b) * V + ys];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            C v = cmake<C>((R)0, (R)0);
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                if (ADJ)
                    cmac_conj(v, w[b][a], p[s][b]);
                else
                    cmac(v, w[a][b], p[s][b]);
            }
            chi[s][a] = v;
        }
}

__device__ __forceinline__ unsigned sel3(int d, unsigned m, unsigned z, unsigned p) {
    return d < 0 ? m : (d > 0 ? p : z);
}

template <class LS, int NSPLIT, bool DAG, int MODE>
__global__ __launch_bounds__(64 * NSPLIT) void stencil_kernel(StencilArgs args) {
    using R = typename LS::R;
    using C = typename Cx<R>::T;
    constexpr int NCOMP = 12 / NSPLIT;

    if (MODE != EPI_PLAIN && args.done && *args.done) return;  // solver already converged

    const Geom &g = args.g;
    const unsigned V = (unsigned)g.V;
    const int lane = threadIdx.x & 63;
    const int q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    // tile of 64 sites; optional XCD-aware order of the tiles
    int blk = blockIdx.x;
    const int nblk = gridDim.x;
    if (args.xcd_remap && (nblk & 7) == 0) blk = (blk & 7) * (nblk >> 3) + (blk >> 3);
    int t = blk;
    int c[4];
    {
        int l = lane;
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const int bm = t % args.nb[mu];
            t /= args.nb[mu];
            c[mu] = bm * args.tile[mu] + l % args.tile[mu];
            l /= args.tile[mu];
        }
    }
    // wrapped neighbour offsets per axis, premultiplied by the axis stride
    unsigned om[4], o0[4], op[4];
    {
        unsigned stride = 1;
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const int Lm = g.L[mu];
            const int cm = c[mu] == 0 ? Lm - 1 : c[mu] - 1;
            const int cp = c[mu] == Lm - 1 ? 0 : c[mu] + 1;
            om[mu] = (unsigned)cm * stride;
            o0[mu] = (unsigned)c[mu] * stride;
            op[mu] = (unsigned)cp * stride;
            stride *= (unsigned)Lm;
        }
    }
    const unsigned x = o0[0] + o0[1] + o0[2] + o0[3];

    const size_t rhs_off = (size_t)blockIdx.y * 12 * V;
    const C *__restrict__ in = (const C *)args.in + rhs_off;
    const typename LS::store_t *__restrict__ W = (const typename LS::store_t *)args.W;

    C acc[4][3];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[s][a] = cmake<C>((R)0, (R)0);
    if (q == 0) {
        const R diag = (R)args.diag;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                C v = in[(size_t)(s * 3 + a) * V + x];
                acc[s][a] = cmake<C>(diag * v.x, diag * v.y);
            }
    }

    for (int j = q; j < 40; j += NSPLIT) {
        const int d0 = j % 3 - 1, d1 = (j / 3) % 3 - 1, d2 = (j / 9) % 3 - 1, d3 = j / 27 - 1;
        const int k = (d0 != 0) + (d1 != 0) + (d2 != 0) + (d3 != 0);
        const R a = (R)lap_weight(k);
        const R ck = (R)(DAG ? -iso_weight(k) : iso_weight(k));
        const R c0 = ck * (R)d0, c1 = ck * (R)d1, c2 = ck * (R)d2, c3 = ck * (R)d3;
        const typename LS::store_t *__restrict__ Wj = W + (size_t)j * 9 * V;

        C chi[4][3];
        // own link: S_d W_j(x) psi(x + d)
        {
            const unsigned y = sel3(d0, om[0], o0[0], op[0]) + sel3(d1, om[1], o0[1], op[1]) +
                               sel3(d2, om[2], o0[2], op[2]) + sel3(d3, om[3], o0[3], op[3]);
            transport<LS, false>(chi, Wj, x, in, y, V);
            spin_accumulate(acc, chi, a, c0, c1, c2, c3);
        }
        // opposite displacement: S_{-d} W_j(x - d)^dag psi(x - d)
        {
            const unsigned z = sel3(-d0, om[0], o0[0], op[0]) + sel3(-d1, om[1], o0[1], op[1]) +
                               sel3(-d2, om[2], o0[2], op[2]) + sel3(-d3, om[3], o0[3], op[3]);
            transport<LS, true>(chi, Wj, z, in, z, V);
            spin_accumulate(acc, chi, a, -c0, -c1, -c2, -c3);
        }
    }

    // ---- combine the NSPLIT partial sums through LDS
    __shared__ C red[NSPLIT > 1 ? NSPLIT : 1][12][64];
    __shared__ double wsum[NSPLIT][2];
    C res[NCOMP];
    if constexpr (NSPLIT > 1) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int a = 0; a < 3; ++a) red[q][s * 3 + a][lane] = acc[s][a];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NCOMP; ++i) {
            const int comp = q * NCOMP + i;
            C v = red[0][comp][lane];
#pragma unroll
            for (int w = 1; w < NSPLIT; ++w) {
                C u = red[w][comp][lane];
                v.x += u.x;
                v.y += u.y;
            }
            res[i] = v;
        }
    } else {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int a = 0; a < 3; ++a) res[s * 3 + a] = acc[s][a];
    }

    // ---- fused epilogues on components [q*NCOMP, (q+1)*NCOMP)
    double n0 = 0.0, n1 = 0.0;
    C *__restrict__ out = (C *)args.out + rhs_off;
#pragma unroll
    for (int i = 0; i < NCOMP; ++i) {
        const int comp = q * NCOMP + i;
        const size_t idx = (size_t)comp * V + x;
        C v = res[i];
        if constexpr (MODE == EPI_PLAIN) {
            out[idx] = v;
        } else if constexpr (MODE == EPI_NORMS) {
            out[idx] = v;
            const C u = in[idx];
            n0 += (double)v.x * v.x + (double)v.y * v.y;
            n1 += (double)u.x * u.x + (double)u.y * u.y;
        } else if constexpr (MODE == EPI_CG_R) {
            // Ap = v + sigma0 p ; r -= alpha Ap ; |r|^2
            const C pp = ((const C *)args.p + rhs_off)[idx];
            C *rr = (C *)args.r + rhs_off;
            C r = rr[idx];
            const R al = (R)*args.alpha;
            const R s0 = (R)args.sigma0;
            const R apx = v.x + s0 * pp.x, apy = v.y + s0 * pp.y;
            r.x = fma(-al, apx, r.x);
            r.y = fma(-al, apy, r.y);
            rr[idx] = r;
            n0 += (double)r.x * r.x + (double)r.y * r.y;
        } else if constexpr (MODE == EPI_OV) {
            const C b = ((const C *)args.b + rhs_off)[idx];
            const R rho = (R)args.rho;
            out[idx] = cmake<C>(rho * (b.x + v.x), rho * (b.y + v.y));
        } else if constexpr (MODE == EPI_SIGN) {
            const R sg = comp < 6 ? (R)1 : (R)-1;  // gamma5 = diag(1, 1, -1, -1)
            out[idx] = cmake<C>(sg * v.x, sg * v.y);
        }
    }
    if constexpr (MODE == EPI_NORMS || MODE == EPI_CG_R) {
        // deterministic block reduction: wave sums, then the NSPLIT wave totals in order
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            n0 += __shfl_xor(n0, off, 64);
            n1 += __shfl_xor(n1, off, 64);
        }
        if (lane == 0) {
            wsum[q][0] = n0;
            wsum[q][1] = n1;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double s0 = 0.0, s1 = 0.0;
            for (int w = 0; w < NSPLIT; ++w) {
                s0 += wsum[w][0];
                s1 += wsum[w][1];
            }
            const size_t pb = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
            args.partial[2 * pb] = s0;
            args.partial[2 * pb + 1] = s1;
        }
    }
}

// ------------------------------------------------------------------ launch

template <class LS, int NSPLIT, bool DAG>
static hipError_t launch_mode(const StencilArgs &a, int mode, dim3 grid, hipStream_t st) {
    const dim3 block(64 * NSPLIT);
    switch (mode) {
    case EPI_PLAIN:
        hipLaunchKernelGGL((stencil_kernel<LS, NSPLIT, DAG, EPI_PLAIN>), grid, block, 0, st, a);
        break;
    case EPI_NORMS:
        hipLaunchKernelGGL((stencil_kernel<LS, NSPLIT, DAG, EPI_NORMS>), grid, block, 0, st, a);
        break;
    case EPI_CG_R:
        hipLaunchKernelGGL((stencil_kernel<LS, NSPLIT, DAG, EPI_CG_R>), grid, block, 0, st, a);
        break;
    case EPI_OV:
        hipLaunchKernelGGL((stencil_kernel<LS, NSPLIT, DAG, EPI_OV>), grid, block, 0, st, a);
        break;
    case EPI_SIGN:
        hipLaunchKernelGGL((stencil_kernel<LS, NSPLIT, DAG, EPI_SIGN>), grid, block, 0, st, a);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class LS, bool DAG>
static hipError_t launch_split(const StencilArgs &a, int nsplit, int mode, dim3 grid, hipStream_t st) {
    switch (nsplit) {
    case 1:
        return launch_mode<LS, 1, DAG>(a, mode, grid, st);
    case 2:
        return launch_mode<LS, 2, DAG>(a, mode, grid, st);
    case 4:
        return launch_mode<LS, 4, DAG>(a, mode, grid, st);
    default:
        return hipErrorInvalidValue;
    }
}

// Chooses a 64-site tile that divides the lattice: x first (coalescing), then
// y, z, t.  Falls back to BRI_EINVAL when no such tile exists.
int plan_tile(const Geom &g, const StencilConfig &cfg, int tile[4], int nb[4]) {
    if (cfg.tile[0] > 0) {
        int prod = 1;
        for (int mu = 0; mu < 4; ++mu) {
            if (cfg.tile[mu] < 1 || g.L[mu] % cfg.tile[mu]) return BRI_EINVAL;
            prod *= cfg.tile[mu];
        }
        if (prod != 64) return BRI_EINVAL;
        for (int mu = 0; mu < 4; ++mu) {
            tile[mu] = cfg.tile[mu];
            nb[mu] = g.L[mu] / tile[mu];
        }
        return BRI_OK;
    }
    int rem = 64;
    for (int mu = 0; mu < 4; ++mu) {
        int t = 1;
        while (rem % (2 * t) == 0 && g.L[mu] % (2 * t) == 0 && 2 * t <= rem && 2 * t <= 16) t *= 2;
        tile[mu] = t;
        rem /= t;
    }
    if (rem != 1) {
        // absorb the rest wherever it still divides
        for (int mu = 0; mu < 4 && rem > 1; ++mu)
            while (rem > 1 && g.L[mu] % (tile[mu] * 2) == 0) {
                tile[mu] *= 2;
                rem /= 2;
            }
        if (rem != 1) return BRI_EINVAL;
    }
    for (int mu = 0; mu < 4; ++mu) nb[mu] = g.L[mu] / tile[mu];
    return BRI_OK;
}

int stencil_launch(StencilArgs a, int prec, bool dag, int mode, int nrhs, const StencilConfig &cfg, hipStream_t st) {
    int rc = plan_tile(a.g, cfg, a.tile, a.nb);
    if (rc != BRI_OK) return rc;
    a.xcd_remap = cfg.xcd_remap;
    const int nsplit = cfg.nsplit;
    const dim3 grid((unsigned)(a.g.V / 64), (unsigned)nrhs);
    hipError_t e;
    if (prec == BRI_F64)
        e = dag ? launch_split<LinkF64, true>(a, nsplit, mode, grid, st)
                : launch_split<LinkF64, false>(a, nsplit, mode, grid, st);
    else if (prec == BRI_F32)
        e = dag ? launch_split<LinkF32, true>(a, nsplit, mode, grid, st)
                : launch_split<LinkF32, false>(a, nsplit, mode, grid, st);
    else if (prec == BRI_F32_BF16W)
        e = dag ? launch_split<LinkBF16, true>(a, nsplit, mode, grid, st)
                : launch_split<LinkBF16, false>(a, nsplit, mode, grid, st);
    else
        return BRI_EINVAL;
    return e == hipSuccess ? BRI_OK : (e == hipErrorInvalidValue ? BRI_EINVAL : BRI_EHIP);
}

StencilConfig default_config(const Geom &g, int prec) {
    StencilConfig c;
    for (int mu = 0; mu < 4; ++mu) c.tile[mu] = 0;
    // few sites -> split each site's directions over more waves to fill 1024 SIMDs
    const int waves_1 = g.V / 64;
    c.nsplit = waves_1 >= 8192 ? 2 : 4;
    c.xcd_remap = 1;
    (void)prec;
    return c;
}

}  // namespace bri

extern "C" {

int bri_apply(const bri_geom *geom, const void *W, int prec, double m0, const void *in, void *out, int nrhs,
              void *stream) {
    using namespace bri;
    StencilArgs a{};
    int rc = geom_check(geom, &a.g);
    if (rc != BRI_OK) return rc;
    if (!W || !in || !out || nrhs < 1 || nrhs > 65535 || a.g.V % 64) return BRI_EINVAL;
    a.W = W;
    a.in = in;
    a.out = out;
    a.diag = 15.0 / 8.0 + m0;
    return stencil_launch(a, prec, false, EPI_PLAIN, nrhs, default_config(a.g, prec), (hipStream_t)stream);
}

int bri_apply_dag(const bri_geom *geom, const void *W, int prec, double m0, const void *in, void *out, int nrhs,
                  void *stream) {
    using namespace bri;
    StencilArgs a{};
    int rc = geom_check(geom, &a.g);
    if (rc != BRI_OK) return rc;
    if (!W || !in || !out || nrhs < 1 || nrhs > 65535 || a.g.V % 64) return BRI_EINVAL;
    a.W = W;
    a.in = in;
    a.out = out;
    a.diag = 15.0 / 8.0 + m0;
    return stencil_launch(a, prec, true, EPI_PLAIN, nrhs, default_config(a.g, prec), (hipStream_t)stream);
}

}  // extern "C"
