// Device-side building blocks of the Brillouin / overlap library (gfx950).
//
// Field layouts (structure of arrays, site index fastest, complex interleaved):
//   U   [4][3][3][V]     W   [40][3][3][V]     psi [nrhs][4][3][V]
// Displacement index j = sum_mu (d_mu + 1) 3^mu; the 40 stored off-axis links
// are the j < 40 ones, whose last non-zero d_mu is -1.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/brillouin.h"

namespace bri {

// ---------------------------------------------------------------- geometry

struct Geom {
    int L[4];
    int V;
    int tbc;
    double csw;  // clover coefficient; nonzero: the link array carries the clover field
};

// Link array layout: 40 stored slabs of 3x3 complex entries ([40][3][3][V]), followed when
// csw != 0 by the clover term -(c_SW/2) sum_{mu<nu} sigma_mu_nu F_mu_nu as its two chirality
// blocks of 6x6 complex entries ([2][6][6][V], row and column index 3*spin + colour within the
// block; spins 0,1 and 2,3).
constexpr int LINK_SLAB_ENTRIES = 360;   // per site
constexpr int CLOVER_ENTRIES = 72;       // per site
inline size_t link_entries(const Geom &g) {
    return (size_t)g.V * (LINK_SLAB_ENTRIES + (g.csw != 0.0 ? CLOVER_ENTRIES : 0));
}

__host__ __device__ inline int disp_comp(int j, int mu) {
    int p = 1;
    for (int i = 0; i < mu; ++i) p *= 3;
    return (j / p) % 3 - 1;
}

// Kernel operator of the stencils: the 81-point Brillouin operator (all 40 stored slabs) or the
// 9-point Wilson operator (the four one-hop slabs of the same link array).
enum KernelKind { KERN_BRI = BRI_KERNEL_BRILLOUIN, KERN_WIL = BRI_KERNEL_WILSON };

// diagonal of the operator without the bare mass: 15/8 (Brillouin), 4 (Wilson)
inline double kernel_diag(int kind) { return kind == KERN_WIL ? 4.0 : 15.0 / 8.0; }

// true when the byte ranges [a, a + na) and [b, b + nb) share a byte (argument aliasing checks)
inline bool ranges_overlap(const void *a, size_t na, const void *b, size_t nb) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

// ---------------------------------------------------------- stencil weights
//
// S_d = a_k + c_k sum_mu d_mu gamma_mu for a k-hop displacement d (k >= 1),
// and 15/8 + m0 on the 0-hop term.  a_k is the Brillouin-Laplacian weight
// -(1/2) * (1/4) * (1/2)^k, c_k the isotropic-derivative weight
// (1/2) (1/6)^(k-1) (2/3)^(4-k); both are the position-space coefficients of
// the momentum forms (cos p + 1)/2 and sin p (cos p + 2)/3 per axis.

__host__ __device__ constexpr double lap_weight(int k) { return -1.0 / (double)(8 << k); }

__host__ __device__ constexpr double iso_weight(int k) {
    return k == 1 ? 4.0 / 27.0 : k == 2 ? 1.0 / 27.0 : k == 3 ? 1.0 / 108.0 : k == 4 ? 1.0 / 432.0 : 0.0;
}

// ----------------------------------------------------------- complex types

template <typename R> struct Cx;
template <> struct Cx<double> { using T = double2; };
template <> struct Cx<float> { using T = float2; };

template <typename C> __device__ __forceinline__ C cmake(decltype(C{}.x) r, decltype(C{}.x) i) {
    C c;
    c.x = r;
    c.y = i;
    return c;
}

// acc += w * v   (complex multiply-accumulate, 4 FMA)
template <typename C> __device__ __forceinline__ void cmac(C &acc, const C &w, const C &v) {
    acc.x = fma(w.x, v.x, acc.x);
    acc.x = fma(-w.y, v.y, acc.x);
    acc.y = fma(w.x, v.y, acc.y);
    acc.y = fma(w.y, v.x, acc.y);
}

// acc += conj(w) * v
template <typename C> __device__ __forceinline__ void cmac_conj(C &acc, const C &w, const C &v) {
    acc.x = fma(w.x, v.x, acc.x);
    acc.x = fma(w.y, v.y, acc.x);
    acc.y = fma(w.x, v.y, acc.y);
    acc.y = fma(-w.y, v.x, acc.y);
}

// ----------------------------------------------------------------- bfloat16
// round-to-nearest-even from float; NaN kept quiet.

__host__ __device__ inline uint16_t f32_to_bf16(float f) {
    union {
        float f;
        uint32_t u;
    } v;
    v.f = f;
    if ((v.u & 0x7f800000u) == 0x7f800000u && (v.u & 0x007fffffu)) return (uint16_t)((v.u >> 16) | 0x40u);
    uint32_t lsb = (v.u >> 16) & 1u;
    v.u += 0x7fffu + lsb;
    return (uint16_t)(v.u >> 16);
}

__host__ __device__ inline float bf16_to_f32(uint16_t h) {
    union {
        float f;
        uint32_t u;
    } v;
    v.u = (uint32_t)h << 16;
    return v.f;
}

// ------------------------------------------------------- link storage types
// LinkStore<P>::load returns element e of link slab j at site x as Cx<R>.

struct LinkF64 {
    using store_t = double2;
    using R = double;
    __device__ __forceinline__ static double2 load(const store_t *W, size_t idx) { return W[idx]; }
};
struct LinkF32 {
    using store_t = float2;
    using R = float;
    __device__ __forceinline__ static float2 load(const store_t *W, size_t idx) { return W[idx]; }
};
struct LinkBF16 {
    using store_t = uint32_t;  // (re, im) packed: re in the low half
    using R = float;
    __device__ __forceinline__ static float2 load(const store_t *W, size_t idx) {
        uint32_t u = W[idx];
        float2 c;
        c.x = __uint_as_float(u << 16);
        c.y = __uint_as_float(u & 0xffff0000u);
        return c;
    }
};

// ---------------------------------------------------------------- launches

#define BRI_HIP_CHECK(expr)                           \
    do {                                              \
        hipError_t _e = (expr);                       \
        if (_e != hipSuccess) return BRI_EHIP;        \
    } while (0)

}  // namespace bri
