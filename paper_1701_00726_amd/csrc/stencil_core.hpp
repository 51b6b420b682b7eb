// Device helpers shared by the Brillouin stencil kernels: complex axpy forms,
// the spin weights S_d = a + sum_mu c_mu gamma_mu, the colour transport
// W psi / W^dag psi, and site / neighbour addressing.
//
// Gamma matrices, chiral basis: gamma_k = [[0, -i s_k], [i s_k, 0]],
// gamma_4 = [[0, 1], [1, 0]].  Acting on the four spin components chi_s:
//   gamma_1 chi = (-i chi3, -i chi2,  i chi1,  i chi0)
//   gamma_2 chi = (  -chi3,    chi2,    chi1,   -chi0)
//   gamma_3 chi = (-i chi2,  i chi3,  i chi0, -i chi1)
//   gamma_4 chi = (   chi2,    chi3,    chi0,    chi1)
#pragma once

#include "common.hpp"

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

// chi = w p (ADJ: w^dag p) with link and spinor both in registers
template <typename C, typename R, bool ADJ>
__device__ __forceinline__ void transport_vals(C (&chi)[4][3], const C (&w)[3][3], const C (&p)[4][3]) {
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


// the nine entries of link slab Wj at site ws, converted to the compute type
template <class LS>
__device__ __forceinline__ void load_link(typename Cx<typename LS::R>::T (&w)[3][3],
                                          const typename LS::store_t *__restrict__ Wj, unsigned ws, unsigned V) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) w[a][b] = LS::load(Wj, (size_t)(a * 3 + b) * V + ws);
}

// chi = w psi(ys) (ADJ: w^dag psi(ys)) with the link already in registers
template <typename C, typename R, bool ADJ>
__device__ __forceinline__ void transport_reg(C (&chi)[4][3], const C (&w)[3][3], const C *__restrict__ ps,
                                              unsigned ys, unsigned V) {
    C p[4][3];
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

// Site of lane `lane` in (logical) tile `blk`, and the wrapped neighbour
// offsets om/o0/op per axis, premultiplied by the axis stride.  Two traversals:
//   colz == 0: tiles of extents tile[4] in lexicographic order (x fastest);
//   colz  > 0: tiles of tile[0] x tile[1] x 1 x 1 sites grouped in columns of
//              coly tile rows along y, colz z-planes and all t; inside a column
//              the tiles run y fastest, then z, then t, and the columns run x, y,
//              z.  A tile's neighbours in y, z and t are then 1, coly and
//              coly * colz tiles away: tiles an XCD runs together hold most stencil
//              neighbours of each other, so the second read of a link (by the
//              partner site) and re-read spinors stay in that XCD's L2.
__device__ __forceinline__ unsigned tile_site(const Geom &g, const int tile[4], const int nb[4], int colz, int coly,
                                              int blk, int lane, unsigned om[4], unsigned o0[4], unsigned op[4]) {
    int c[4];
    if (colz > 0) {
        const int per_col = coly * colz * g.L[3];
        const int col = blk / per_col, rem = blk - col * per_col;
        const int yy = rem % coly, r1 = rem / coly;
        const int zt = r1 % colz, tt = r1 / colz;
        const int ncy = nb[1] / coly;
        const int cx = col % nb[0], r2 = col / nb[0];
        const int cy = r2 % ncy, cz = r2 / ncy;
        c[0] = cx * tile[0] + lane % tile[0];
        c[1] = (cy * coly + yy) * tile[1] + lane / tile[0];
        c[2] = cz * colz + zt;
        c[3] = tt;
    } else {
        int t = blk;
        int l = lane;
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const int bm = t % nb[mu];
            t /= nb[mu];
            c[mu] = bm * tile[mu] + l % tile[mu];
            l /= tile[mu];
        }
    }
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
    return o0[0] + o0[1] + o0[2] + o0[3];
}

__device__ __forceinline__ int xcd_order(int blk, int nblk, int remap) {
    return (remap && (nblk & 7) == 0) ? (blk & 7) * (nblk >> 3) + (blk >> 3) : blk;
}

// Tile and column group of this block.  The column groups (one column, or R of them) of a tile are
// consecutive along x, gridDim.x / ntiles of them (all, unless grid.x would grow too large, the
// rest follow in blockIdx.y), so that after the XCD ordering the blocks that read the same links
// run together on one XCD and share those links in its L2 instead of re-reading them from HBM or
// the Infinity Cache one pass over the lattice later.
__device__ __forceinline__ void tile_and_group(int ntiles, int remap, int &blk, int &grp) {
    const int gin = gridDim.x / ntiles;
    const int lin = xcd_order(blockIdx.x, gridDim.x, remap);
    blk = lin / gin;
    grp = blockIdx.y * gin + (lin - blk * gin);
}

// v += (C(x) psi(x))_comp for the clover term stored after the link slabs: two chirality blocks
// of 6x6 entries, component index comp = 3*spin + colour, block k holding spins 2k and 2k+1.
// Applied where a wave finishes its output components, after the slab loop, so the term adds
// nothing to the loop's register footprint.
template <class LS>
__device__ __forceinline__ void clover_row(typename Cx<typename LS::R>::T &v,
                                           const typename LS::store_t *__restrict__ Cf,
                                           const typename Cx<typename LS::R>::T *__restrict__ ps, int comp,
                                           unsigned x, unsigned V) {
    const int k = comp / 6, a = comp % 6;
#pragma unroll
    for (int b = 0; b < 6; ++b)
        cmac(v, LS::load(Cf, (size_t)((k * 6 + a) * 6 + b) * V + x), ps[(size_t)(k * 6 + b) * V + x]);
}

// stored slabs a kernel walks: all 40 (Brillouin), or the one-hop slabs j = 40 - 3^(3-k) (Wilson:
// displacements -t, -z, -y, -x)
template <int KIND> struct Slabs {
    static constexpr int n = KIND == KERN_WIL ? 4 : 40;
    __device__ __forceinline__ static int at(int k) {
        if constexpr (KIND == KERN_WIL) return 40 - (k == 0 ? 27 : k == 1 ? 9 : k == 2 ? 3 : 1);
        return k;
    }
};

// neighbour x + s*d of a stored displacement index j (s = +1 or -1)
__device__ __forceinline__ unsigned neighbour(int j, int s, const unsigned om[4], const unsigned o0[4],
                                              const unsigned op[4]) {
    const int d0 = s * (j % 3 - 1), d1 = s * ((j / 3) % 3 - 1), d2 = s * ((j / 9) % 3 - 1), d3 = s * (j / 27 - 1);
    return sel3(d0, om[0], o0[0], op[0]) + sel3(d1, om[1], o0[1], op[1]) + sel3(d2, om[2], o0[2], op[2]) +
           sel3(d3, om[3], o0[3], op[3]);
}

// xyz part of the neighbour x + s*d of a stored displacement index j (s = +1 or -1); the t step
// is added by the caller
__device__ __forceinline__ unsigned neighbour3(int j, int s, const unsigned om[3], const unsigned o0[3],
                                               const unsigned op[3]) {
    const int d0 = s * (j % 3 - 1), d1 = s * ((j / 3) % 3 - 1), d2 = s * ((j / 9) % 3 - 1);
    return sel3(d0, om[0], o0[0], op[0]) + sel3(d1, om[1], o0[1], op[1]) + sel3(d2, om[2], o0[2], op[2]);
}

// weights of stored displacement j: a_k and c_mu = c_k d_mu (negated for the adjoint).
// Brillouin: the Laplacian and isotropic-derivative weights of a k-hop point.  Wilson (one-hop
// slabs only): -1/2 from -(1/2) lap^std and 1/2 d_mu from gamma_mu nabla^std_mu, i.e.
// S_{+-mu} = -(1/2)(1 -+ gamma_mu).
template <typename R, bool DAG, int KIND = KERN_BRI> struct DirW {
    R a, c0, c1, c2, c3;
    __device__ __forceinline__ explicit DirW(int j) {
        const int d0 = j % 3 - 1, d1 = (j / 3) % 3 - 1, d2 = (j / 9) % 3 - 1, d3 = j / 27 - 1;
        const int k = (d0 != 0) + (d1 != 0) + (d2 != 0) + (d3 != 0);
        a = (R)(KIND == KERN_WIL ? -0.5 : lap_weight(k));
        const double cw = KIND == KERN_WIL ? 0.5 : iso_weight(k);
        const R ck = (R)(DAG ? -cw : cw);
        c0 = ck * (R)d0;
        c1 = ck * (R)d1;
        c2 = ck * (R)d2;
        c3 = ck * (R)d3;
    }
};

}  // namespace bri
