// Multi-RHS Brillouin stencil with the colour transport on the matrix cores (FP32 MFMA), for FP32
// or bfloat16 links and FP32 spinors.
//
// v_mfma_f32_4x4x1_16b_f32 computes 16 independent 4x4 outer products per wave: in the block of
// lanes 4b..4b+3, D[i][j] += A[i] B[j] with A[i] from lane 4b+i, B[j] from lane 4b+j, and lane
// 4b+j holds D[0..3][j] in its four result registers.  Here a block is one site and its four
// lanes are that site's four spins j: with A[i] = W[i][c] (colour row i; the fourth lane gives 0)
// and B[j] = psi[j][c], three steps c = 0..2 give D[i][j] = (W psi)[spin j][colour i], the
// transport of the neighbour spinor, left in the lane of its spin.  A complex product takes
// four real steps (re.re - im.im into the real part, re.im + im.re into the imaginary part).
// The spin weights S_d = a_k + sum_mu c_mu gamma_mu then act across the four lanes of a site:
// gamma_1 and gamma_2 pair spin j with j^3, gamma_3 and gamma_4 with j^2 (quad permutes), with
// the signs and factors i of the chiral basis:
//   (gamma_1 chi)_j = i s1_j chi_{j^3},  s1 = (-1, -1, +1, +1)
//   (gamma_2 chi)_j =   s2_j chi_{j^3},  s2 = (-1, +1, +1, -1)
//   (gamma_3 chi)_j = i s3_j chi_{j^2},  s3 = (-1, +1, +1, -1)
//   (gamma_4 chi)_j =        chi_{j^2}.
// A wave covers 16 sites, a block of four waves a 64-site tile; every thread walks the 40 stored
// slabs as own / partner pairs (as the other kernels) for its R right-hand sides, the link entry
// being shared by them.  The per-thread accumulators are the site's spin-j row: 3 colours x R.
#pragma once

namespace bri {

typedef float mfma_f4 __attribute__((ext_vector_type(4)));

// value of v in the lane of the same site holding spin (j ^ 3) / (j ^ 2)
__device__ __forceinline__ float quad_xor3(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x1B, 0xF, 0xF, true));
}
__device__ __forceinline__ float quad_xor2(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, true));
}

template <class LS, int R, bool DAG, int MODE>
__global__ __launch_bounds__(256) void stencil_mfma_kernel(StencilArgs a) {
    using C = float2;
    using S = typename LS::store_t;
    const unsigned V = (unsigned)a.g.V;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int sub = lane & 3;                 // spin of this lane; colour row of the link it feeds
    const int site_in_tile = 16 * w + (lane >> 2);
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
    const unsigned x = tile_site(a.g, a.tile, a.nb, a.colz, a.coly, blk, site_in_tile, om, o0, op);
    const C *__restrict__ in = (const C *)a.in + (size_t)col0 * 12 * V;
    const S *__restrict__ W = (const S *)a.W;
    // chiral-basis signs of this lane's spin
    const float s1 = sub < 2 ? -1.f : 1.f;
    const float s23 = (sub == 0 || sub == 3) ? -1.f : 1.f;

    C acc[R][3];  // (D psi)[spin sub][colour b] of column col0 + r
    const float diag = (float)a.diag;
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            C v = make_float2(0.f, 0.f);
            if (live[r]) {
                const C u = in[((size_t)r * 12 + sub * 3 + b) * V + x];
                v = make_float2(diag * u.x, diag * u.y);
            }
            acc[r][b] = v;
        }

    const mfma_f4 zero = {0.f, 0.f, 0.f, 0.f};
    for (int j = 0; j < 40; ++j) {
        const DirW<float, DAG, KERN_BRI> dw(j);
        const S *__restrict__ Wj = W + (size_t)j * 9 * V;
#pragma unroll
        for (int side = 0; side < 2; ++side) {  // own term, then the partner term
            const unsigned y = neighbour(j, side == 0 ? +1 : -1, om, o0, op);
            // A: row `sub` of W_j(x) (own) or of W_j(x - d)^dag (partner); the fourth row is 0
            C arow[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (sub < 3) {
                    if (side == 0) {
                        arow[c] = LS::load(Wj, (size_t)(sub * 3 + c) * V + x);
                    } else {
                        const C t = LS::load(Wj, (size_t)(c * 3 + sub) * V + y);
                        arow[c] = make_float2(t.x, -t.y);
                    }
                } else {
                    arow[c] = make_float2(0.f, 0.f);
                }
            }
            const float sg = side == 0 ? 1.f : -1.f;  // S_{-d}: derivative weights negated
            const float ca = dw.a, c0 = sg * dw.c0, c1 = sg * dw.c1, c2 = sg * dw.c2, c3 = sg * dw.c3;
            const bool t13 = c0 != 0.f || c1 != 0.f, t24 = c2 != 0.f || c3 != 0.f;
            // term coefficients of this lane: (c1 s2 + i c0 s1) chi_{j^3} + (c3 + i c2 s3) chi_{j^2}
            const float al = c1 * s23, be = c0 * s1, ga = c3, de = c2 * s23;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (!live[r]) continue;
                const C *__restrict__ pr = in + (size_t)r * 12 * V;
                mfma_f4 dre = zero, dim = zero;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const C p = pr[(size_t)(sub * 3 + c) * V + y];
                    dre = __builtin_amdgcn_mfma_f32_4x4x1f32(arow[c].x, p.x, dre, 0, 0, 0);
                    dre = __builtin_amdgcn_mfma_f32_4x4x1f32(-arow[c].y, p.y, dre, 0, 0, 0);
                    dim = __builtin_amdgcn_mfma_f32_4x4x1f32(arow[c].x, p.y, dim, 0, 0, 0);
                    dim = __builtin_amdgcn_mfma_f32_4x4x1f32(arow[c].y, p.x, dim, 0, 0, 0);
                }
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    const float xr = dre[b], xi = dim[b];  // chi[spin sub][colour b]
                    C v = acc[r][b];
                    v.x = fmaf(ca, xr, v.x);
                    v.y = fmaf(ca, xi, v.y);
                    if (t13) {
                        const float tr = quad_xor3(xr), ti = quad_xor3(xi);
                        v.x = fmaf(al, tr, fmaf(-be, ti, v.x));
                        v.y = fmaf(al, ti, fmaf(be, tr, v.y));
                    }
                    if (t24) {
                        const float tr = quad_xor2(xr), ti = quad_xor2(xi);
                        v.x = fmaf(ga, tr, fmaf(-de, ti, v.x));
                        v.y = fmaf(ga, ti, fmaf(de, tr, v.y));
                    }
                    acc[r][b] = v;
                }
            }
        }
    }

    __shared__ double wsum[4][2];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!live[r]) continue;
        const int col = col0 + r;
        double n0 = 0.0, n1 = 0.0;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            C v = acc[r][b];
            if (a.g.csw != 0.0)
                clover_row<LS>(v, W + (size_t)LINK_SLAB_ENTRIES * V, in + (size_t)r * 12 * V, sub * 3 + b, x, V);
            epilogue<MODE, C, float>(a, col, sub * 3 + b, x, V, v, n0, n1);
        }
        if constexpr (MODE == EPI_NORMS || MODE == EPI_CG_R || MODE == EPI_RESID) {
            n0 = wave_sum(n0);
            n1 = wave_sum(n1);
            if (lane == 0) {
                wsum[w][0] = n0;
                wsum[w][1] = n1;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                double t0 = 0.0, t1 = 0.0;
                for (int q = 0; q < 4; ++q) {
                    t0 += wsum[q][0];
                    t1 += wsum[q][1];
                }
                const size_t pb = (size_t)col * a.nslots + blk;
                a.partial[2 * pb] = t0;
                a.partial[2 * pb + 1] = t1;
            }
            __syncthreads();  // wsum is reused by the next column
        }
    }
}

}  // namespace bri
