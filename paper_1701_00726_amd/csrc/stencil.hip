// Stencil launches: tile planning, default configurations, the dispatch to the per-variant
// instantiations (stencil_<precision>_<kernel>.hip) and the bri_apply / wil_apply entry points.
#include "stencil.hpp"

namespace bri {

// one translation unit per (link precision, kernel) pair
hipError_t launch_f64_bri(const StencilArgs &, bool, int, const StencilConfig &, hipStream_t);
hipError_t launch_f64_wil(const StencilArgs &, bool, int, const StencilConfig &, hipStream_t);
hipError_t launch_f32_bri(const StencilArgs &, bool, int, const StencilConfig &, hipStream_t);
hipError_t launch_f32_wil(const StencilArgs &, bool, int, const StencilConfig &, hipStream_t);
hipError_t launch_bf16_bri(const StencilArgs &, bool, int, const StencilConfig &, hipStream_t);
hipError_t launch_bf16_wil(const StencilArgs &, bool, int, const StencilConfig &, hipStream_t);

// A 64-site tile that divides the lattice.  Column traversal: tile
// tile[0] x tile[1] x 1 x 1 with colz | Lz.  Otherwise x first (coalescing),
// then y, z, t.
static int plan_tile_base(const Geom &g, const StencilConfig &cfg, int tile[4], int nb[4]) {
    if (g.V % 64) return BRI_EINVAL;
    if (cfg.colz <= 0 && cfg.coly > 1) return BRI_EINVAL;  // y-blocked columns need the column traversal
    if (cfg.variant == VAR_TSTREAM) {
        // t-streaming: an xyz tile of STREAM_THREADS sites and chunks of tile[3] t-slices
        if (cfg.rpt != 0) return BRI_EINVAL;
        int prod = 1;
        for (int mu = 0; mu < 4; ++mu) {
            if (cfg.tile[mu] < 1 || g.L[mu] % cfg.tile[mu]) return BRI_EINVAL;
            if (mu < 3) prod *= cfg.tile[mu];
        }
        if (prod != STREAM_THREADS) return BRI_EINVAL;
        for (int mu = 0; mu < 4; ++mu) {
            tile[mu] = cfg.tile[mu];
            nb[mu] = g.L[mu] / tile[mu];
        }
        return BRI_OK;
    }
    if (cfg.colz > 0) {
        const int tx = cfg.tile[0], ty = cfg.tile[1];
        if (tx < 1 || ty < 1 || tx * ty != 64 || g.L[0] % tx || g.L[1] % ty || g.L[2] % cfg.colz) return BRI_EINVAL;
        tile[0] = tx;
        tile[1] = ty;
        tile[2] = tile[3] = 1;
        nb[0] = g.L[0] / tx;
        nb[1] = g.L[1] / ty;
        nb[2] = g.L[2];
        nb[3] = g.L[3];
        if (cfg.coly < 0 || (cfg.coly > 0 && nb[1] % cfg.coly)) return BRI_EINVAL;
        return BRI_OK;
    }
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
    for (int mu = 0; mu < 4 && rem > 1; ++mu)
        while (rem > 1 && g.L[mu] % (tile[mu] * 2) == 0) {
            tile[mu] *= 2;
            rem /= 2;
        }
    if (rem != 1) return BRI_EINVAL;
    for (int mu = 0; mu < 4; ++mu) nb[mu] = g.L[mu] / tile[mu];
    return BRI_OK;
}

// the tile plan, and for the x-line kernel the requirement that a tile spans whole x-lines
int plan_tile(const Geom &g, const StencilConfig &cfg, int tile[4], int nb[4]) {
    const int rc = plan_tile_base(g, cfg, tile, nb);
    if (rc != BRI_OK) return rc;
    if (cfg.variant == VAR_XLINE && (tile[0] != g.L[0] || cfg.rpt == 1 || cfg.rpt > 4)) return BRI_EINVAL;
    if (cfg.variant == VAR_MFMA && (cfg.rpt < 1 || cfg.rpt > 4)) return BRI_EINVAL;
    if (cfg.variant < VAR_STANDARD || cfg.variant > VAR_MFMA) return BRI_EINVAL;
    return BRI_OK;
}

int stencil_launch(StencilArgs a, int prec, bool dag, int mode, const StencilConfig &cfg, hipStream_t st) {
    if (a.ncol < 1 || a.ncol > 65535) return BRI_EINVAL;
    int rc = plan_tile(a.g, cfg, a.tile, a.nb);
    if (rc != BRI_OK) return rc;
    a.colz = cfg.colz;
    a.coly = cfg.coly > 0 ? cfg.coly : 1;
    a.xcd_remap = cfg.xcd_remap;
    a.nslots = a.g.V / 64;
    if (a.kind != KERN_BRI && a.kind != KERN_WIL) return BRI_EINVAL;
    const bool wil = a.kind == KERN_WIL;
    hipError_t e;
    if (prec == BRI_F64)
        e = wil ? launch_f64_wil(a, dag, mode, cfg, st) : launch_f64_bri(a, dag, mode, cfg, st);
    else if (prec == BRI_F32)
        e = wil ? launch_f32_wil(a, dag, mode, cfg, st) : launch_f32_bri(a, dag, mode, cfg, st);
    else if (prec == BRI_F32_BF16W)
        e = wil ? launch_bf16_wil(a, dag, mode, cfg, st) : launch_bf16_bri(a, dag, mode, cfg, st);
    else
        return BRI_EINVAL;
    return e == hipSuccess ? BRI_OK : (e == hipErrorInvalidValue ? BRI_EINVAL : BRI_EHIP);
}

// Column traversal when the lattice allows a 16 x 4 tile (two full 128-byte lines per row in
// FP64) and a column depth of 8 (or 4, 2) z-planes; lexicographic tiles otherwise, which
// measured faster than 8 x 8 or 4 x 16 columns (24^3 x 48: 1.86 against 2.04 ms).
static void default_traversal(const Geom &g, StencilConfig &c) {
    for (int mu = 0; mu < 4; ++mu) c.tile[mu] = 0;
    c.colz = 0;
    if (g.L[0] % 16 || g.L[1] % 4) return;
    for (int cz : {8, 4, 2}) {
        if (g.L[2] % cz) continue;
        c.tile[0] = 16;
        c.tile[1] = 4;
        c.colz = cz;
        return;
    }
}

// a large lattice whose x-lines fill whole rows of a 64-lane wave (the x-line kernels' default)
static bool xline_fits(const Geom &g) {
    return g.V / 64 >= 8192 && (g.L[0] == 16 || g.L[0] == 32 || g.L[0] == 64) && g.L[1] % (64 / g.L[0]) == 0;
}

StencilConfig default_config(const Geom &g, int prec, int ncol, int kind) {
    StencilConfig c;
    // the tuned table holds Brillouin launches; the Wilson stencil keeps the defaults
    if (kind == KERN_BRI && tuned_config(g, prec, ncol, &c)) return c;
    default_traversal(g, c);
    c.xcd_remap = 1;
    if (ncol >= 2) {
        // link loads amortised over R right-hand sides per thread (a last, partial group of
        // columns is allowed); four waves still split each tile's displacements.  Below 4096
        // tiles (up to 16^4) more column groups keep the chip busy: R = 2 (FP64, and FP32 up to 8
        // columns) or 3 measured 5-40% faster than R = 4 at 8^4 and 16^4; at 24^3x48 R = 4 is
        // fastest (by up to 25% in FP32).
        c.nsplit = MRHS_SPLIT;
        if (ncol < 4)
            c.rpt = ncol;
        else if (g.V / 64 < 4096)
            c.rpt = (prec == BRI_F64 || ncol <= 8) ? 2 : 3;
        else
            c.rpt = (ncol % 4 == 0 || ncol % 3 != 0) ? 4 : 3;
        // large lattices whose x-lines fit a wave: whole-line tiles (Lx x 64/Lx) in columns of 4
        // z-slices (FP64: one tile row wide; FP32 and bfloat16 links: two), the column groups of
        // a tile run together (tile_and_group).  12 RHS at 32^3x64 measured 28.8-29.2 ms (FP64, R
        // = 2; 30.2 / 31.4 ms in columns of 8 / 16 z-slices; two rows wide the same time with 8%
        // more bytes fetched), 16.4 ms (FP32, R = 3; 16.8 ms one row wide, 17.4 ms with R = 4) and
        // 14.9 ms (bfloat16 links: the x-line kernel, one RHS per thread; 15.1 ms for the
        // multi-RHS kernel with R = 3).  Before the tiles' column groups ran together (each group
        // a separate pass over the lattice, re-reading every link) the same launches took 37.6 /
        // 18.5 / 18.7 ms.
        if (kind == KERN_BRI && ncol >= 3 && xline_fits(g)) {
            c.tile[0] = g.L[0];
            c.tile[1] = 64 / g.L[0];
            c.tile[2] = c.tile[3] = 1;
            c.xcd_remap = 1;
            c.colz = g.L[2] % 4 == 0 ? 4 : (g.L[2] % 2 == 0 ? 2 : 1);
            c.coly = prec != BRI_F64 && (g.L[1] / c.tile[1]) % 2 == 0 ? 2 : 1;
            if (prec == BRI_F32_BF16W) {
                c.variant = VAR_XLINE;
                c.rpt = 0;
            } else {
                c.rpt = prec == BRI_F64 ? 2 : 3;
            }
        }
    } else {
        // four waves split each tile's directions: fills the 1024 SIMDs on small lattices, and on
        // large ones keeps fewer tiles (and their link lines) in flight per XCD than two waves do
        c.rpt = 0;
        c.nsplit = 4;
        // large lattices whose x-lines fit a wave: the x-line kernel (one spinor load per three
        // x-displacements) on whole-line tiles in XCD-ordered columns of 4 z-slices and 8 (FP64)
        // or 16 tile rows, whose tiles run together with their y, z and t neighbours, where the
        // partner sites re-read the links.  At 32^3x64 it measured 3.59-3.63 / 2.00 / 1.47 ms
        // (FP64 / FP32 / bfloat16 links) against 4.17 / 2.21 / 1.71 ms for lexicographic tiles
        // (the fastest traversal without y-blocked columns) and 5.52 / 3.37 / 2.64 ms for the 16 x
        // 4 column traversal above; at 16^4 the kernels tie.
        if (kind == KERN_BRI && xline_fits(g)) {
            c.variant = VAR_XLINE;
            c.tile[0] = g.L[0];
            c.tile[1] = 64 / g.L[0];
            c.tile[2] = c.tile[3] = 1;
            const int rows = g.L[1] / c.tile[1];
            c.colz = g.L[2] % 4 == 0 ? 4 : (g.L[2] % 2 == 0 ? 2 : 1);
            const int widest = prec == BRI_F64 ? 8 : 16;
            c.coly = 1;
            for (int cy = widest; cy > 1; cy /= 2)
                if (rows % cy == 0) {
                    c.coly = cy;
                    break;
                }
            c.xcd_remap = 1;
        }
    }
    return c;
}

}  // namespace bri

extern "C" {

static int apply_common(const bri_geom *geom, const void *W, int prec, double m0, const void *in, void *out, int nrhs,
                        void *stream, bool dag, int kind) {
    using namespace bri;
    StencilArgs a{};
    int rc = geom_check(geom, &a.g);
    if (rc != BRI_OK) return rc;
    if (!W || !in || !out || nrhs < 1 || nrhs > 65535 || a.g.V % 64) return BRI_EINVAL;
    if (prec != BRI_F64 && prec != BRI_F32 && prec != BRI_F32_BF16W) return BRI_EINVAL;
    const size_t sb = (size_t)12 * a.g.V * nrhs * (prec == BRI_F64 ? 16 : 8);
    if (ranges_overlap(in, sb, out, sb)) return BRI_EINVAL;  // neighbours are read while out is written
    a.W = W;
    a.in = in;
    a.out = out;
    a.ncol = nrhs;
    a.kind = kind;
    a.diag = kernel_diag(kind) + m0;
    return stencil_launch(a, prec, dag, EPI_PLAIN, default_config(a.g, prec, nrhs, kind), (hipStream_t)stream);
}

int bri_apply(const bri_geom *geom, const void *W, int prec, double m0, const void *in, void *out, int nrhs,
              void *stream) {
    return apply_common(geom, W, prec, m0, in, out, nrhs, stream, false, bri::KERN_BRI);
}

int bri_apply_dag(const bri_geom *geom, const void *W, int prec, double m0, const void *in, void *out, int nrhs,
                  void *stream) {
    return apply_common(geom, W, prec, m0, in, out, nrhs, stream, true, bri::KERN_BRI);
}

int wil_apply(const bri_geom *geom, const void *W, int prec, double m0, const void *in, void *out, int nrhs,
              void *stream) {
    return apply_common(geom, W, prec, m0, in, out, nrhs, stream, false, bri::KERN_WIL);
}

int wil_apply_dag(const bri_geom *geom, const void *W, int prec, double m0, const void *in, void *out, int nrhs,
                  void *stream) {
    return apply_common(geom, W, prec, m0, in, out, nrhs, stream, true, bri::KERN_WIL);
}

}  // extern "C"
