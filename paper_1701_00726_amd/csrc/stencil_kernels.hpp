// Brillouin stencil y = D_bri(m0) x on gfx950 (App. C.1), and the Wilson stencil y = D_wil(m0) x
// (eq. (def_wils)) as the same kernels restricted to the four one-hop slabs with Wilson weights.
//
//   (D psi)(x) = (15/8 + m0) psi(x) + C(x) psi(x) + sum_{d != 0} S_d W_d(x) psi(x + d)
//   S_d = a_k + c_k sum_mu d_mu gamma_mu      (k = number of hops of d)
// with C(x) the clover term stored after the link slabs (only when the geometry's csw != 0;
// it commutes with gamma5 and is hermitian, so the adjoint uses it unchanged).
//
// Both kernels walk the 40 stored link slabs j and apply, for each, the pair
// of opposite displacements
//   own:        S_{d}  W_j(x)            psi(x + d)
//   neighbour:  S_{-d} W_j(x - d)^dag    psi(x - d)
// so that a stored link is read by its own site and, as W^dag, by the site
// across the link at nearly the same time.  The adjoint uses
// D^dag = gamma5 D gamma5: the same stencil with the derivative weights c_k
// negated (gamma5 anticommutes with every gamma_mu).
//
// stencil_kernel (one right-hand side per block row): a block owns a tile of
// 64 sites and NSPLIT waves; wave q takes the slabs j = q, q + NSPLIT, ... so
// that small lattices still fill the 1024 SIMDs.  The NSPLIT partial sums meet
// in LDS; wave q finishes 12/NSPLIT of the spin-colour components.
//
// stencil_mrhs_kernel (many right-hand sides): a block owns a tile of 64 sites
// and R right-hand sides; its MRHS_SPLIT waves split the slabs as above and
// every thread carries all R right-hand sides, so each link entry is loaded
// once per R right-hand sides while the tile still spreads over MRHS_SPLIT
// waves.  The partial sums meet in LDS one column at a time.
//
// The templates are instantiated by the per-variant translation units
// stencil_<precision>_<kernel>.hip, one (link precision, kernel) pair each, so that the variants
// compile in parallel.
#pragma once

#include <cstdlib>
#include <type_traits>

#include "stencil.hpp"
#include "stencil_core.hpp"

namespace bri {

template <typename C> __device__ __forceinline__ double norm2(const C &v) {
    return (double)v.x * (double)v.x + (double)v.y * (double)v.y;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Epilogue for component comp of column col at site x.  Returns the two norm
// contributions (n0, n1) where the mode has any.
template <int MODE, typename C, typename R>
__device__ __forceinline__ void epilogue(const StencilArgs &a, int col, int comp, unsigned x, unsigned V, C v,
                                         double &n0, double &n1) {
    const size_t idx = ((size_t)col * 12 + comp) * V + x;
    if constexpr (MODE == EPI_PLAIN) {
        ((C *)a.out)[idx] = v;
    } else if constexpr (MODE == EPI_NORMS) {
        ((C *)a.out)[idx] = v;
        n0 += norm2(v);
        n1 += norm2(((const C *)a.in)[idx]);
    } else if constexpr (MODE == EPI_CG_R) {
        const C pp = ((const C *)a.p)[idx];
        C *rr = (C *)a.r;
        C r = rr[idx];
        const R al = (R)a.st[col].alpha;
        const R s0 = (R)a.st[col].sigma0;
        const R apx = v.x + s0 * pp.x, apy = v.y + s0 * pp.y;
        r.x = fma(-al, apx, r.x);
        r.y = fma(-al, apy, r.y);
        rr[idx] = r;
        n0 += norm2(r);
    } else if constexpr (MODE == EPI_OV) {
        const C b = ((const C *)a.b)[idx];
        const R rho = (R)a.rho;
        ((C *)a.out)[idx] = cmake<C>(rho * (b.x + v.x), rho * (b.y + v.y));
    } else if constexpr (MODE == EPI_SIGN) {
        const R sg = comp < 6 ? (R)1 : (R)-1;  // gamma5 = diag(1, 1, -1, -1)
        ((C *)a.out)[idx] = cmake<C>(sg * v.x, sg * v.y);
    } else if constexpr (MODE == EPI_RESID) {
        const size_t bidx = ((size_t)(col % a.b_mod) * 12 + comp) * V + x;
        const C b = ((const C *)a.b)[bidx];
        const C xv = ((const C *)a.xs)[idx];
        const R s = (R)a.sig[col];
        const C o = cmake<C>(b.x - (v.x + s * xv.x), b.y - (v.y + s * xv.y));
        ((C *)a.out)[idx] = o;
        n0 += norm2(o);
    }
}

template <int MODE> __device__ __forceinline__ bool col_done(const StencilArgs &a, int col) {
    if constexpr (MODE == EPI_NORMS || MODE == EPI_CG_R) return a.st && a.st[col].done;
    return false;
}

// ------------------------------------------------------- one right-hand side

template <class LS, int NSPLIT, bool DAG, int MODE, int KIND>
__global__ __launch_bounds__(64 * NSPLIT) void stencil_kernel(StencilArgs a) {
    using R = typename LS::R;
    using C = typename Cx<R>::T;
    constexpr int NCOMP = 12 / NSPLIT;
    int blk, col;
    tile_and_group(a.nslots, a.xcd_remap, blk, col);
    if (col >= a.ncol || col_done<MODE>(a, col)) return;  // whole block: this column has converged

    const unsigned V = (unsigned)a.g.V;
    const int lane = threadIdx.x & 63;
    const int q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    unsigned om[4], o0[4], op[4];
    const unsigned x = tile_site(a.g, a.tile, a.nb, a.colz, a.coly, blk, lane, om, o0, op);

    const C *__restrict__ in = (const C *)a.in + (size_t)col * 12 * V;
    const typename LS::store_t *__restrict__ W = (const typename LS::store_t *)a.W;

    C acc[4][3];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int b = 0; b < 3; ++b) acc[s][b] = cmake<C>((R)0, (R)0);
    if (q == 0) {
        const R diag = (R)a.diag;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const C v = in[(size_t)(s * 3 + b) * V + x];
                acc[s][b] = cmake<C>(diag * v.x, diag * v.y);
            }
    }

    for (int k = q; k < Slabs<KIND>::n; k += NSPLIT) {
        const int j = Slabs<KIND>::at(k);
        const DirW<R, DAG, KIND> dw(j);
        const typename LS::store_t *__restrict__ Wj = W + (size_t)j * 9 * V;
        C chi[4][3];
        const unsigned y = neighbour(j, +1, om, o0, op);
        transport<LS, false>(chi, Wj, x, in, y, V);
        spin_accumulate(acc, chi, dw.a, dw.c0, dw.c1, dw.c2, dw.c3);
        const unsigned z = neighbour(j, -1, om, o0, op);
        transport<LS, true>(chi, Wj, z, in, z, V);
        spin_accumulate(acc, chi, dw.a, -dw.c0, -dw.c1, -dw.c2, -dw.c3);
    }

    // combine the NSPLIT partial sums through LDS
    __shared__ C red[NSPLIT > 1 ? NSPLIT : 1][12][64];
    __shared__ double wsum[NSPLIT][2];
    C res[NCOMP];
    if constexpr (NSPLIT > 1) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int b = 0; b < 3; ++b) red[q][s * 3 + b][lane] = acc[s][b];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NCOMP; ++i) {
            const int comp = q * NCOMP + i;
            C v = red[0][comp][lane];
#pragma unroll
            for (int w = 1; w < NSPLIT; ++w) {
                const C u = red[w][comp][lane];
                v.x += u.x;
                v.y += u.y;
            }
            res[i] = v;
        }
    } else {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int b = 0; b < 3; ++b) res[s * 3 + b] = acc[s][b];
    }

    if (a.g.csw != 0.0) {
#pragma unroll
        for (int i = 0; i < NCOMP; ++i) clover_row<LS>(res[i], W + (size_t)LINK_SLAB_ENTRIES * V, in, q * NCOMP + i, x, V);
    }
    double n0 = 0.0, n1 = 0.0;
#pragma unroll
    for (int i = 0; i < NCOMP; ++i) epilogue<MODE, C, R>(a, col, q * NCOMP + i, x, V, res[i], n0, n1);
    if constexpr (MODE == EPI_NORMS || MODE == EPI_CG_R || MODE == EPI_RESID) {
        // deterministic: wave sums, then the NSPLIT wave totals in order
        n0 = wave_sum(n0);
        n1 = wave_sum(n1);
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
            const size_t pb = (size_t)col * a.nslots + blk;
            a.partial[2 * pb] = s0;
            a.partial[2 * pb + 1] = s1;
        }
    }
}

// ------------------------------------------------ whole x-lines, one right-hand side
//
// stencil_xline_kernel: as stencil_kernel, with 64-site tiles whose x extent is the lattice's
// (every x-line of a tile lies in one wave).  The 80 displacements fall into 27 groups of equal
// (d_y, d_z, d_t), each with d_x = -1, 0, +1; a group's three neighbour spinors psi(x + d) are the
// one spinor loaded at x + (0, d_y, d_z, d_t), moved one lane left or right inside the x-line
// (cross-lane moves through the LDS crossbar instead of two more loads through the vector-memory
// address unit, and every spinor load aligned to the x-line).  A displacement d whose index
// j(d) < 40 uses the stored link W_j(x) (own term); otherwise the stored link of -d at x + d,
// daggered (partner term).  Wave q takes the groups q, q + NSPLIT, ...

template <typename C> __device__ __forceinline__ C lane_fetch(const C &v, int src) {
    C r;
    r.x = __shfl(v.x, src, 64);
    r.y = __shfl(v.y, src, 64);
    return r;
}

// chi = w p' (ADJ: w^dag p') where p' is p as held by lane src (shift) or by this lane; each
// component is moved right before its use, so no shifted copy of the spinor is kept
template <typename C, typename R, bool ADJ>
__device__ __forceinline__ void transport_shift(C (&chi)[4][3], const C (&w)[3][3], const C (&p)[4][3], bool shift,
                                                int src) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
#pragma unroll
        for (int a = 0; a < 3; ++a) chi[s][a] = cmake<C>((R)0, (R)0);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const C v = shift ? lane_fetch(p[s][b], src) : p[s][b];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (ADJ)
                    cmac_conj(chi[s][a], w[b][a], v);
                else
                    cmac(chi[s][a], w[a][b], v);
            }
        }
    }
}

template <class LS, int NSPLIT, bool DAG, int MODE>
__global__ __launch_bounds__(64 * NSPLIT) void stencil_xline_kernel(StencilArgs a) {
    using R = typename LS::R;
    using C = typename Cx<R>::T;
    using S = typename LS::store_t;
    constexpr int NCOMP = 12 / NSPLIT;
    int blk, col;
    tile_and_group(a.nslots, a.xcd_remap, blk, col);
    if (col >= a.ncol || col_done<MODE>(a, col)) return;

    const unsigned V = (unsigned)a.g.V;
    const int lane = threadIdx.x & 63;
    const int q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    unsigned om[4], o0[4], op[4];
    const unsigned x = tile_site(a.g, a.tile, a.nb, a.colz, a.coly, blk, lane, om, o0, op);
    const int tx = a.tile[0];  // = L_x
    const int lx = lane % tx;
    const int lane_m = lane - lx + (lx == 0 ? tx - 1 : lx - 1);  // holds x - 1 (periodic in x)
    const int lane_p = lane - lx + (lx == tx - 1 ? 0 : lx + 1);  // holds x + 1

    const C *__restrict__ in = (const C *)a.in + (size_t)col * 12 * V;
    const S *__restrict__ W = (const S *)a.W;

    C acc[4][3];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int b = 0; b < 3; ++b) acc[s][b] = cmake<C>((R)0, (R)0);
    if (q == 0) {
        const R diag = (R)a.diag;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const C v = in[(size_t)(s * 3 + b) * V + x];
                acc[s][b] = cmake<C>(diag * v.x, diag * v.y);
            }
    }

    for (int gi = q; gi < 27; gi += NSPLIT) {
        const int dy = gi % 3 - 1, dz = (gi / 3) % 3 - 1, dt = gi / 9 - 1;
        const unsigned yzt = sel3(dy, om[1], o0[1], op[1]) + sel3(dz, om[2], o0[2], op[2]) +
                             sel3(dt, om[3], o0[3], op[3]);
        C pc[4][3];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int b = 0; b < 3; ++b) pc[s][b] = in[(size_t)(s * 3 + b) * V + o0[0] + yzt];
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            if (gi == 13 && dx == 0) continue;  // d = 0: the diagonal term
            const int jd = (dx + 1) + 3 * gi;    // index of d = (dx, dy, dz, dt)
            const int src = dx < 0 ? lane_m : lane_p;
            C w[3][3], chi[4][3];
            if (jd < 40) {  // own term: S_d W_d(x) psi(x + d)
                const DirW<R, DAG, KERN_BRI> dw(jd);
                load_link<LS>(w, W + (size_t)jd * 9 * V, x, V);
                transport_shift<C, R, false>(chi, w, pc, dx != 0, src);
                spin_accumulate(acc, chi, dw.a, dw.c0, dw.c1, dw.c2, dw.c3);
            } else {  // partner term: S_d W_{-d}(x + d)^dag psi(x + d)
                const int j = 80 - jd;
                const DirW<R, DAG, KERN_BRI> dw(j);
                load_link<LS>(w, W + (size_t)j * 9 * V, sel3(dx, om[0], o0[0], op[0]) + yzt, V);
                transport_shift<C, R, true>(chi, w, pc, dx != 0, src);
                spin_accumulate(acc, chi, dw.a, -dw.c0, -dw.c1, -dw.c2, -dw.c3);
            }
        }
    }

    __shared__ C red[NSPLIT > 1 ? NSPLIT : 1][12][64];
    __shared__ double wsum[NSPLIT][2];
    C res[NCOMP];
    if constexpr (NSPLIT > 1) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int b = 0; b < 3; ++b) red[q][s * 3 + b][lane] = acc[s][b];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NCOMP; ++i) {
            const int comp = q * NCOMP + i;
            C v = red[0][comp][lane];
#pragma unroll
            for (int w = 1; w < NSPLIT; ++w) {
                const C u = red[w][comp][lane];
                v.x += u.x;
                v.y += u.y;
            }
            res[i] = v;
        }
    } else {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int b = 0; b < 3; ++b) res[s * 3 + b] = acc[s][b];
    }
    if (a.g.csw != 0.0) {
#pragma unroll
        for (int i = 0; i < NCOMP; ++i) clover_row<LS>(res[i], W + (size_t)LINK_SLAB_ENTRIES * V, in, q * NCOMP + i, x, V);
    }
    double n0 = 0.0, n1 = 0.0;
#pragma unroll
    for (int i = 0; i < NCOMP; ++i) epilogue<MODE, C, R>(a, col, q * NCOMP + i, x, V, res[i], n0, n1);
    if constexpr (MODE == EPI_NORMS || MODE == EPI_CG_R || MODE == EPI_RESID) {
        n0 = wave_sum(n0);
        n1 = wave_sum(n1);
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
            const size_t pb = (size_t)col * a.nslots + blk;
            a.partial[2 * pb] = s0;
            a.partial[2 * pb + 1] = s1;
        }
    }
}

// stencil_xline_mrhs_kernel: the x-line grouping with R right-hand sides per thread, as
// stencil_mrhs_kernel: MRHS_SPLIT waves split a whole-x-line tile's 27 groups, each group's R
// neighbour spinors are loaded once and shifted across lanes, and each link is loaded once for
// the R right-hand sides.  The partial sums meet in LDS one column at a time.
template <class LS, int R, bool DAG, int MODE>
__global__ __launch_bounds__(64 * MRHS_SPLIT) void stencil_xline_mrhs_kernel(StencilArgs a) {
    using RT = typename LS::R;
    using C = typename Cx<RT>::T;
    using S = typename LS::store_t;
    constexpr int NSPLIT = MRHS_SPLIT;
    constexpr int NCOMP = 12 / NSPLIT;
    const unsigned V = (unsigned)a.g.V;
    const int lane = threadIdx.x & 63;
    const int q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int blk, grp;
    tile_and_group(a.nslots, a.xcd_remap, blk, grp);
    const int col0 = grp * R;
    bool live[R];
    bool any = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        live[r] = (col0 + r < a.ncol) && !col_done<MODE>(a, col0 + r);
        any |= live[r];
    }
    if (!any) return;

    unsigned om[4], o0[4], op[4];
    const unsigned x = tile_site(a.g, a.tile, a.nb, a.colz, a.coly, blk, lane, om, o0, op);
    const int tx = a.tile[0];  // = L_x
    const int lx = lane % tx;
    const int lane_m = lane - lx + (lx == 0 ? tx - 1 : lx - 1);
    const int lane_p = lane - lx + (lx == tx - 1 ? 0 : lx + 1);
    const C *__restrict__ in = (const C *)a.in + (size_t)col0 * 12 * V;
    const S *__restrict__ W = (const S *)a.W;

    C acc[R][4][3];
    const RT diag = (RT)a.diag;
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                C v = cmake<C>((RT)0, (RT)0);
                if (q == 0 && live[r]) {
                    const C u = in[((size_t)r * 12 + s * 3 + b) * V + x];
                    v = cmake<C>(diag * u.x, diag * u.y);
                }
                acc[r][s][b] = v;
            }

    for (int gi = q; gi < 27; gi += NSPLIT) {
        const int dy = gi % 3 - 1, dz = (gi / 3) % 3 - 1, dt = gi / 9 - 1;
        const unsigned yzt = sel3(dy, om[1], o0[1], op[1]) + sel3(dz, om[2], o0[2], op[2]) +
                             sel3(dt, om[3], o0[3], op[3]);
        C pc[R][4][3];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    pc[r][s][b] = live[r] ? in[((size_t)r * 12 + s * 3 + b) * V + o0[0] + yzt] : cmake<C>((RT)0, (RT)0);
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            if (gi == 13 && dx == 0) continue;  // d = 0: the diagonal term
            const int jd = (dx + 1) + 3 * gi;
            const int src = dx < 0 ? lane_m : lane_p;
            const bool own = jd < 40;
            const int j = own ? jd : 80 - jd;
            const DirW<RT, DAG, KERN_BRI> dw(j);
            C w[3][3], chi[4][3];
            load_link<LS>(w, W + (size_t)j * 9 * V, own ? x : sel3(dx, om[0], o0[0], op[0]) + yzt, V);
            const RT sg = own ? (RT)1 : (RT)-1;  // the partner term has S_{-d}: derivative weights negated
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (!live[r]) continue;
                if (own)
                    transport_shift<C, RT, false>(chi, w, pc[r], dx != 0, src);
                else
                    transport_shift<C, RT, true>(chi, w, pc[r], dx != 0, src);
                spin_accumulate(acc[r], chi, dw.a, sg * dw.c0, sg * dw.c1, sg * dw.c2, sg * dw.c3);
            }
        }
    }

    __shared__ C red[NSPLIT][12][64];
    __shared__ double wsum[NSPLIT][2];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!live[r]) continue;
        const int col = col0 + r;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int b = 0; b < 3; ++b) red[q][s * 3 + b][lane] = acc[r][s][b];
        __syncthreads();
        double n0 = 0.0, n1 = 0.0;
#pragma unroll
        for (int i = 0; i < NCOMP; ++i) {
            const int comp = q * NCOMP + i;
            C v = red[0][comp][lane];
#pragma unroll
            for (int w = 1; w < NSPLIT; ++w) {
                const C u = red[w][comp][lane];
                v.x += u.x;
                v.y += u.y;
            }
            if (a.g.csw != 0.0)
                clover_row<LS>(v, W + (size_t)LINK_SLAB_ENTRIES * V, in + (size_t)r * 12 * V, comp, x, V);
            epilogue<MODE, C, RT>(a, col, comp, x, V, v, n0, n1);
        }
        if constexpr (MODE == EPI_NORMS || MODE == EPI_CG_R || MODE == EPI_RESID) {
            n0 = wave_sum(n0);
            n1 = wave_sum(n1);
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
                const size_t pb = (size_t)col * a.nslots + blk;
                a.partial[2 * pb] = s0;
                a.partial[2 * pb + 1] = s1;
            }
        }
        __syncthreads();  // red and wsum are reused by the next column
    }
}

// ------------------------------------------------ t-streaming, one right-hand side
//
// stencil_stream_kernel: a block of STREAM_THREADS threads owns a tile of tile[0] x tile[1] x
// tile[2] sites of the xyz volume (one site per thread) and walks the tile[3] t-slices of its
// chunk.  At slice s every stored slab j (displacement d, with d_t = -1 for j < 27 and d_t = 0
// for 27 <= j < 40) is read twice inside that slice:
//   at the site x itself, for the own term     S_d W_j(x) psi(x + d)            of y(s);
//   at the xyz-shifted site x - d_xyz, for the partner term S_{-d} W_j(x - d_xyz)^dag psi(x - d_xyz)
//                                              of y(s - 1) (d_t = -1) or y(s) (d_t = 0),
// since the partner site x - d of the output site (x, s - 1) lies in slice s.  Both reads of a
// stored link thus happen in the same slice at nearly the same time, mostly inside the block's
// own tile, instead of a slice apart.  Every thread keeps the two output slices it is building:
// y(s - 1) is complete after the d_t = -1 slabs of step s and is written out then.  A chunk
// [t0, t1) also visits slice t1 for the partner terms of y(t1 - 1) and leaves the partner terms of
// y(t0 - 1) to the chunk before it.
template <class LS, bool DAG, int MODE>
__global__ __launch_bounds__(STREAM_THREADS) void stencil_stream_kernel(StencilArgs a) {
    using R = typename LS::R;
    using C = typename Cx<R>::T;
    using S = typename LS::store_t;
    const int col = blockIdx.y;
    if (col_done<MODE>(a, col)) return;

    const unsigned V = (unsigned)a.g.V;
    const int Lt = a.g.L[3];
    const unsigned S3 = (unsigned)a.g.L[0] * (unsigned)a.g.L[1] * (unsigned)a.g.L[2];
    const int blk = xcd_order(blockIdx.x, gridDim.x, a.xcd_remap);
    const int ntile = a.nb[0] * a.nb[1] * a.nb[2];
    const int chunk = blk / ntile;
    unsigned om[3], o0[3], op[3];
    {
        int tl = blk - chunk * ntile;
        int l = threadIdx.x;
        unsigned stride = 1;
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
            const int bm = tl % a.nb[mu];
            tl /= a.nb[mu];
            const int cm = bm * a.tile[mu] + l % a.tile[mu];
            l /= a.tile[mu];
            const int Lm = a.g.L[mu];
            om[mu] = (unsigned)(cm == 0 ? Lm - 1 : cm - 1) * stride;
            o0[mu] = (unsigned)cm * stride;
            op[mu] = (unsigned)(cm == Lm - 1 ? 0 : cm + 1) * stride;
            stride *= (unsigned)Lm;
        }
    }
    const unsigned xyz = o0[0] + o0[1] + o0[2];
    const int t0 = chunk * a.tile[3], t1 = t0 + a.tile[3];

    const C *__restrict__ in = (const C *)a.in + (size_t)col * 12 * V;
    const S *__restrict__ W = (const S *)a.W;
    const R diag = (R)a.diag;

    C accp[4][3], accc[4][3];  // y(s - 1), y(s)
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            accp[s][b] = cmake<C>((R)0, (R)0);
            accc[s][b] = cmake<C>((R)0, (R)0);
        }
    double n0 = 0.0, n1 = 0.0;

    for (int s = t0; s <= t1; ++s) {
        const bool first = s == t0, last = s == t1;
        const unsigned ts = (unsigned)(s == Lt ? 0 : s) * S3;         // slice s
        const unsigned tm = (unsigned)(s == 0 ? Lt - 1 : s - 1) * S3;  // slice s - 1
        if (!last) {
#pragma unroll
            for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    const C v = in[(size_t)(sp * 3 + b) * V + xyz + ts];
                    accc[sp][b] = cmake<C>(diag * v.x, diag * v.y);
                }
        }
        // d_t = -1: own terms of y(s) (spinor from slice s - 1), partner terms of y(s - 1)
        for (int j = 0; j < 27; ++j) {
            const DirW<R, DAG, KERN_BRI> dw(j);
            const S *__restrict__ Wj = W + (size_t)j * 9 * V;
            C chi[4][3];
            if (!last) {
                const unsigned yp = neighbour3(j, +1, om, o0, op) + tm;
                transport<LS, false>(chi, Wj, xyz + ts, in, yp, V);
                spin_accumulate(accc, chi, dw.a, dw.c0, dw.c1, dw.c2, dw.c3);
            }
            if (!first) {
                const unsigned ym = neighbour3(j, -1, om, o0, op) + ts;
                transport<LS, true>(chi, Wj, ym, in, ym, V);
                spin_accumulate(accp, chi, dw.a, -dw.c0, -dw.c1, -dw.c2, -dw.c3);
            }
        }
        if (!first) {  // y(s - 1) is complete
            const unsigned x = xyz + tm;
#pragma unroll
            for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    C v = accp[sp][b];
                    if (a.g.csw != 0.0) clover_row<LS>(v, W + (size_t)LINK_SLAB_ENTRIES * V, in, sp * 3 + b, x, V);
                    epilogue<MODE, C, R>(a, col, sp * 3 + b, x, V, v, n0, n1);
                }
        }
        if (last) break;
        // d_t = 0: own and partner terms of y(s), everything in slice s
        for (int j = 27; j < 40; ++j) {
            const DirW<R, DAG, KERN_BRI> dw(j);
            const S *__restrict__ Wj = W + (size_t)j * 9 * V;
            C chi[4][3];
            const unsigned yp = neighbour3(j, +1, om, o0, op) + ts;
            transport<LS, false>(chi, Wj, xyz + ts, in, yp, V);
            spin_accumulate(accc, chi, dw.a, dw.c0, dw.c1, dw.c2, dw.c3);
            const unsigned ym = neighbour3(j, -1, om, o0, op) + ts;
            transport<LS, true>(chi, Wj, ym, in, ym, V);
            spin_accumulate(accc, chi, dw.a, -dw.c0, -dw.c1, -dw.c2, -dw.c3);
        }
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int b = 0; b < 3; ++b) accp[sp][b] = accc[sp][b];
    }

    if constexpr (MODE == EPI_NORMS || MODE == EPI_CG_R || MODE == EPI_RESID) {
        // deterministic: wave sums, then the wave totals in order; blocks fill slots
        // [0, gridDim.x) of the column and zero the rest of its nslots
        constexpr int NW = STREAM_THREADS / 64;
        __shared__ double wsum[NW][2];
        const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
        n0 = wave_sum(n0);
        n1 = wave_sum(n1);
        if (lane == 0) {
            wsum[q][0] = n0;
            wsum[q][1] = n1;
        }
        __syncthreads();
        double *pc = a.partial + 2 * (size_t)col * a.nslots;
        if (threadIdx.x == 0) {
            double s0 = 0.0, s1 = 0.0;
            for (int w = 0; w < NW; ++w) {
                s0 += wsum[w][0];
                s1 += wsum[w][1];
            }
            pc[2 * blockIdx.x] = s0;
            pc[2 * blockIdx.x + 1] = s1;
        }
        for (int i = gridDim.x + blockIdx.x * STREAM_THREADS + threadIdx.x; i < a.nslots;
             i += gridDim.x * STREAM_THREADS) {
            pc[2 * i] = 0.0;
            pc[2 * i + 1] = 0.0;
        }
    }
}

// ------------------------------------------------------ many right-hand sides

// waves per SIMD the multi-RHS kernel is compiled for: three for single-precision arithmetic
// with four right-hand sides per thread (168 VGPRs, a few spilled: 12 RHS at 32^3x64 in 18.5
// against 20.4 ms at the two waves its 177 VGPRs would allow, when each column group was a pass
// of its own over the lattice), else what the registers give
template <class LS, int R> constexpr int mrhs_waves() { return sizeof(typename LS::R) == 4 && R == 4 ? 3 : 1; }

template <class LS, int R, bool DAG, int MODE, int KIND>
__global__ __launch_bounds__(64 * MRHS_SPLIT) __attribute__((amdgpu_waves_per_eu(mrhs_waves<LS, R>())))
void stencil_mrhs_kernel(StencilArgs a) {
    using RT = typename LS::R;
    using C = typename Cx<RT>::T;
    constexpr int NSPLIT = MRHS_SPLIT;
    constexpr int NCOMP = 12 / NSPLIT;
    const unsigned V = (unsigned)a.g.V;
    const int lane = threadIdx.x & 63;
    const int q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int blk, grp;
    tile_and_group(a.nslots, a.xcd_remap, blk, grp);
    const int col0 = grp * R;
    // block-uniform: every wave of the block carries the same R columns
    bool live[R];
    bool any = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        live[r] = (col0 + r < a.ncol) && !col_done<MODE>(a, col0 + r);
        any |= live[r];
    }
    if (!any) return;

    unsigned om[4], o0[4], op[4];
    const unsigned x = tile_site(a.g, a.tile, a.nb, a.colz, a.coly, blk, lane, om, o0, op);
    const C *__restrict__ in = (const C *)a.in + (size_t)col0 * 12 * V;
    const typename LS::store_t *__restrict__ W = (const typename LS::store_t *)a.W;

    C acc[R][4][3];
    const RT diag = (RT)a.diag;
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                C v = cmake<C>((RT)0, (RT)0);
                if (q == 0 && live[r]) {
                    const C u = in[((size_t)r * 12 + s * 3 + b) * V + x];
                    v = cmake<C>(diag * u.x, diag * u.y);
                }
                acc[r][s][b] = v;
            }

    for (int k = q; k < Slabs<KIND>::n; k += NSPLIT) {
        const int j = Slabs<KIND>::at(k);
        const DirW<RT, DAG, KIND> dw(j);
        const typename LS::store_t *__restrict__ Wj = W + (size_t)j * 9 * V;
        C wl[3][3];
        C chi[4][3];
        {
            const unsigned y = neighbour(j, +1, om, o0, op);
            load_link<LS>(wl, Wj, x, V);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (!live[r]) continue;
                transport_reg<C, RT, false>(chi, wl, in + (size_t)r * 12 * V, y, V);
                spin_accumulate(acc[r], chi, dw.a, dw.c0, dw.c1, dw.c2, dw.c3);
            }
        }
        {
            const unsigned z = neighbour(j, -1, om, o0, op);
            load_link<LS>(wl, Wj, z, V);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (!live[r]) continue;
                transport_reg<C, RT, true>(chi, wl, in + (size_t)r * 12 * V, z, V);
                spin_accumulate(acc[r], chi, dw.a, -dw.c0, -dw.c1, -dw.c2, -dw.c3);
            }
        }
    }

    // per column: the NSPLIT partial sums meet in LDS, wave q finishes NCOMP components
    __shared__ C red[NSPLIT][12][64];
    __shared__ double wsum[NSPLIT][2];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!live[r]) continue;
        const int col = col0 + r;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int b = 0; b < 3; ++b) red[q][s * 3 + b][lane] = acc[r][s][b];
        __syncthreads();
        double n0 = 0.0, n1 = 0.0;
#pragma unroll
        for (int i = 0; i < NCOMP; ++i) {
            const int comp = q * NCOMP + i;
            C v = red[0][comp][lane];
#pragma unroll
            for (int w = 1; w < NSPLIT; ++w) {
                const C u = red[w][comp][lane];
                v.x += u.x;
                v.y += u.y;
            }
            if (a.g.csw != 0.0)
                clover_row<LS>(v, W + (size_t)LINK_SLAB_ENTRIES * V, in + (size_t)r * 12 * V, comp, x, V);
            epilogue<MODE, C, RT>(a, col, comp, x, V, v, n0, n1);
        }
        if constexpr (MODE == EPI_NORMS || MODE == EPI_CG_R || MODE == EPI_RESID) {
            // deterministic: wave sums, then the NSPLIT wave totals in order
            n0 = wave_sum(n0);
            n1 = wave_sum(n1);
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
                const size_t pb = (size_t)col * a.nslots + blk;
                a.partial[2 * pb] = s0;
                a.partial[2 * pb + 1] = s1;
            }
        }
        __syncthreads();  // red and wsum are reused by the next column
    }
}

}  // namespace bri

#include "stencil_mfma.hpp"

namespace bri {

// ------------------------------------------------------------------ launch

// Grid of a launch of ngroups column groups (tile_and_group): one block per 64-site tile and group,
// the groups of a tile consecutive along x, as many as keep grid.x * threads within 32 bits (HIP's
// limit on a dimension's work-items); further groups continue along y.  BRI_GROUPS_ALONG_X (a
// positive integer in the environment) lowers that count, so that tests reach the y split with
// small lattices; it is read at every launch (a captured graph keeps the grid it was captured with).
inline dim3 group_grid(const StencilArgs &a, int ngroups, int threads) {
    const long long ntiles = a.nslots;
    long long fit = 0xffffffffLL / (ntiles * threads);
    if (const char *cap = std::getenv("BRI_GROUPS_ALONG_X")) {
        const long long c = std::atoll(cap);
        if (c > 0 && c < fit) fit = c;
    }
    const long long gin = fit < 1 ? 1 : (fit < ngroups ? fit : ngroups);
    return dim3((unsigned)(ntiles * gin), (unsigned)((ngroups + gin - 1) / gin));
}

template <class LS, int NSPLIT, bool DAG, int KIND>
inline hipError_t launch_1rhs(const StencilArgs &a, int mode, hipStream_t st) {
    const dim3 grid = group_grid(a, a.ncol, 64 * NSPLIT), block(64 * NSPLIT);
    switch (mode) {
    case EPI_PLAIN: hipLaunchKernelGGL((stencil_kernel<LS, NSPLIT, DAG, EPI_PLAIN, KIND>), grid, block, 0, st, a); break;
    case EPI_NORMS: hipLaunchKernelGGL((stencil_kernel<LS, NSPLIT, DAG, EPI_NORMS, KIND>), grid, block, 0, st, a); break;
    case EPI_CG_R: hipLaunchKernelGGL((stencil_kernel<LS, NSPLIT, DAG, EPI_CG_R, KIND>), grid, block, 0, st, a); break;
    case EPI_OV: hipLaunchKernelGGL((stencil_kernel<LS, NSPLIT, DAG, EPI_OV, KIND>), grid, block, 0, st, a); break;
    case EPI_SIGN: hipLaunchKernelGGL((stencil_kernel<LS, NSPLIT, DAG, EPI_SIGN, KIND>), grid, block, 0, st, a); break;
    case EPI_RESID: hipLaunchKernelGGL((stencil_kernel<LS, NSPLIT, DAG, EPI_RESID, KIND>), grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class LS, int R, bool DAG, int KIND>
inline hipError_t launch_mrhs(const StencilArgs &a, int mode, hipStream_t st) {
    const int groups = (a.ncol + R - 1) / R;
    const dim3 grid = group_grid(a, groups, 64 * MRHS_SPLIT), block(64 * MRHS_SPLIT);
    switch (mode) {
    case EPI_PLAIN: hipLaunchKernelGGL((stencil_mrhs_kernel<LS, R, DAG, EPI_PLAIN, KIND>), grid, block, 0, st, a); break;
    case EPI_NORMS: hipLaunchKernelGGL((stencil_mrhs_kernel<LS, R, DAG, EPI_NORMS, KIND>), grid, block, 0, st, a); break;
    case EPI_CG_R: hipLaunchKernelGGL((stencil_mrhs_kernel<LS, R, DAG, EPI_CG_R, KIND>), grid, block, 0, st, a); break;
    case EPI_OV: hipLaunchKernelGGL((stencil_mrhs_kernel<LS, R, DAG, EPI_OV, KIND>), grid, block, 0, st, a); break;
    case EPI_SIGN: hipLaunchKernelGGL((stencil_mrhs_kernel<LS, R, DAG, EPI_SIGN, KIND>), grid, block, 0, st, a); break;
    case EPI_RESID: hipLaunchKernelGGL((stencil_mrhs_kernel<LS, R, DAG, EPI_RESID, KIND>), grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class LS, bool DAG>
inline hipError_t launch_stream(const StencilArgs &a, int mode, hipStream_t st) {
    const dim3 grid((unsigned)(a.nb[0] * a.nb[1] * a.nb[2] * a.nb[3]), (unsigned)a.ncol), block(STREAM_THREADS);
    switch (mode) {
    case EPI_PLAIN: hipLaunchKernelGGL((stencil_stream_kernel<LS, DAG, EPI_PLAIN>), grid, block, 0, st, a); break;
    case EPI_NORMS: hipLaunchKernelGGL((stencil_stream_kernel<LS, DAG, EPI_NORMS>), grid, block, 0, st, a); break;
    case EPI_CG_R: hipLaunchKernelGGL((stencil_stream_kernel<LS, DAG, EPI_CG_R>), grid, block, 0, st, a); break;
    case EPI_OV: hipLaunchKernelGGL((stencil_stream_kernel<LS, DAG, EPI_OV>), grid, block, 0, st, a); break;
    case EPI_SIGN: hipLaunchKernelGGL((stencil_stream_kernel<LS, DAG, EPI_SIGN>), grid, block, 0, st, a); break;
    case EPI_RESID: hipLaunchKernelGGL((stencil_stream_kernel<LS, DAG, EPI_RESID>), grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class LS, int NSPLIT, bool DAG>
inline hipError_t launch_xline(const StencilArgs &a, int mode, hipStream_t st) {
    const dim3 grid = group_grid(a, a.ncol, 64 * NSPLIT), block(64 * NSPLIT);
    switch (mode) {
    case EPI_PLAIN: hipLaunchKernelGGL((stencil_xline_kernel<LS, NSPLIT, DAG, EPI_PLAIN>), grid, block, 0, st, a); break;
    case EPI_NORMS: hipLaunchKernelGGL((stencil_xline_kernel<LS, NSPLIT, DAG, EPI_NORMS>), grid, block, 0, st, a); break;
    case EPI_CG_R: hipLaunchKernelGGL((stencil_xline_kernel<LS, NSPLIT, DAG, EPI_CG_R>), grid, block, 0, st, a); break;
    case EPI_OV: hipLaunchKernelGGL((stencil_xline_kernel<LS, NSPLIT, DAG, EPI_OV>), grid, block, 0, st, a); break;
    case EPI_SIGN: hipLaunchKernelGGL((stencil_xline_kernel<LS, NSPLIT, DAG, EPI_SIGN>), grid, block, 0, st, a); break;
    case EPI_RESID: hipLaunchKernelGGL((stencil_xline_kernel<LS, NSPLIT, DAG, EPI_RESID>), grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class LS, int R, bool DAG>
inline hipError_t launch_xline_mrhs(const StencilArgs &a, int mode, hipStream_t st) {
    const int groups = (a.ncol + R - 1) / R;
    const dim3 grid = group_grid(a, groups, 64 * MRHS_SPLIT), block(64 * MRHS_SPLIT);
    switch (mode) {
    case EPI_PLAIN: hipLaunchKernelGGL((stencil_xline_mrhs_kernel<LS, R, DAG, EPI_PLAIN>), grid, block, 0, st, a); break;
    case EPI_NORMS: hipLaunchKernelGGL((stencil_xline_mrhs_kernel<LS, R, DAG, EPI_NORMS>), grid, block, 0, st, a); break;
    case EPI_CG_R: hipLaunchKernelGGL((stencil_xline_mrhs_kernel<LS, R, DAG, EPI_CG_R>), grid, block, 0, st, a); break;
    case EPI_OV: hipLaunchKernelGGL((stencil_xline_mrhs_kernel<LS, R, DAG, EPI_OV>), grid, block, 0, st, a); break;
    case EPI_SIGN: hipLaunchKernelGGL((stencil_xline_mrhs_kernel<LS, R, DAG, EPI_SIGN>), grid, block, 0, st, a); break;
    case EPI_RESID: hipLaunchKernelGGL((stencil_xline_mrhs_kernel<LS, R, DAG, EPI_RESID>), grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class LS, int R, bool DAG>
inline hipError_t launch_mfma(const StencilArgs &a, int mode, hipStream_t st) {
    const int groups = (a.ncol + R - 1) / R;
    const dim3 grid = group_grid(a, groups, 256), block(256);
    switch (mode) {
    case EPI_PLAIN: hipLaunchKernelGGL((stencil_mfma_kernel<LS, R, DAG, EPI_PLAIN>), grid, block, 0, st, a); break;
    case EPI_NORMS: hipLaunchKernelGGL((stencil_mfma_kernel<LS, R, DAG, EPI_NORMS>), grid, block, 0, st, a); break;
    case EPI_CG_R: hipLaunchKernelGGL((stencil_mfma_kernel<LS, R, DAG, EPI_CG_R>), grid, block, 0, st, a); break;
    case EPI_OV: hipLaunchKernelGGL((stencil_mfma_kernel<LS, R, DAG, EPI_OV>), grid, block, 0, st, a); break;
    case EPI_SIGN: hipLaunchKernelGGL((stencil_mfma_kernel<LS, R, DAG, EPI_SIGN>), grid, block, 0, st, a); break;
    case EPI_RESID: hipLaunchKernelGGL((stencil_mfma_kernel<LS, R, DAG, EPI_RESID>), grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class LS, bool DAG, int KIND>
inline hipError_t launch_cfg(const StencilArgs &a, int mode, const StencilConfig &cfg, hipStream_t st) {
    if (cfg.variant == VAR_MFMA) {
        if constexpr (KIND == KERN_BRI && !std::is_same<LS, LinkF64>::value) {
            switch (cfg.rpt) {
            case 1: return launch_mfma<LS, 1, DAG>(a, mode, st);
            case 2: return launch_mfma<LS, 2, DAG>(a, mode, st);
            case 3: return launch_mfma<LS, 3, DAG>(a, mode, st);
            case 4: return launch_mfma<LS, 4, DAG>(a, mode, st);
            default: return hipErrorInvalidValue;
            }
        }
        return hipErrorInvalidValue;
    }
    if (cfg.variant == VAR_XLINE) {
        if constexpr (KIND == KERN_BRI) {
            switch (cfg.rpt) {
            case 0: break;
            case 2: return launch_xline_mrhs<LS, 2, DAG>(a, mode, st);
            case 3: return launch_xline_mrhs<LS, 3, DAG>(a, mode, st);
            case 4: return launch_xline_mrhs<LS, 4, DAG>(a, mode, st);
            default: return hipErrorInvalidValue;
            }
            if (cfg.rpt == 0) {
                switch (cfg.nsplit) {
                case 1: return launch_xline<LS, 1, DAG>(a, mode, st);
                case 2: return launch_xline<LS, 2, DAG>(a, mode, st);
                case 4: return launch_xline<LS, 4, DAG>(a, mode, st);
                default: return hipErrorInvalidValue;
                }
            }
        }
        return hipErrorInvalidValue;
    }
    if (cfg.variant == VAR_TSTREAM) {
        if constexpr (KIND == KERN_BRI) {
            if (cfg.rpt == 0) return launch_stream<LS, DAG>(a, mode, st);
        }
        return hipErrorInvalidValue;
    }
    switch (cfg.rpt) {
    case 0:
        switch (cfg.nsplit) {
        case 1: return launch_1rhs<LS, 1, DAG, KIND>(a, mode, st);
        case 2: return launch_1rhs<LS, 2, DAG, KIND>(a, mode, st);
        case 4: return launch_1rhs<LS, 4, DAG, KIND>(a, mode, st);
        default: return hipErrorInvalidValue;
        }
    case 1: return launch_mrhs<LS, 1, DAG, KIND>(a, mode, st);
    case 2: return launch_mrhs<LS, 2, DAG, KIND>(a, mode, st);
    case 3: return launch_mrhs<LS, 3, DAG, KIND>(a, mode, st);
    case 4: return launch_mrhs<LS, 4, DAG, KIND>(a, mode, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace bri
