// Stencil launch autotuner.  For one lattice, precision and column count it
// times a set of candidate launch configurations (tile shape and traversal,
// waves per tile or right-hand sides per thread, XCD-aware tile order) with
// HIP events and keeps the fastest in a process-wide table that
// default_config consults.
#include <array>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "stencil.hpp"

namespace bri {

using TuneKey = std::tuple<int, int, int, int, int, int>;  // L[4], prec, ncol

static std::mutex g_tune_mu;
static std::map<TuneKey, StencilConfig> g_tuned;

static TuneKey key_of(const Geom &g, int prec, int ncol) {
    return TuneKey(g.L[0], g.L[1], g.L[2], g.L[3], prec, ncol);
}

bool tuned_config(const Geom &g, int prec, int ncol, StencilConfig *out) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(key_of(g, prec, ncol));
    if (it == g_tuned.end()) return false;
    *out = it->second;
    return true;
}

static StencilConfig from_public(const bri_stencil_cfg &c) {
    StencilConfig s;
    s.tile[0] = c.tile_x;
    s.tile[1] = c.tile_y;
    s.tile[2] = c.tile_z;
    s.tile[3] = c.tile_t;
    s.colz = c.col_z;
    s.nsplit = c.nsplit;
    s.rpt = c.rpt;
    s.xcd_remap = c.xcd;
    s.variant = c.variant;
    s.coly = c.col_y;
    return s;
}

static bri_stencil_cfg to_public(const StencilConfig &s) {
    bri_stencil_cfg c;
    c.tile_x = s.tile[0];
    c.tile_y = s.tile[1];
    c.tile_z = s.tile[2];
    c.tile_t = s.tile[3];
    c.col_z = s.colz;
    c.nsplit = s.nsplit;
    c.rpt = s.rpt;
    c.xcd = s.xcd_remap;
    c.variant = s.variant;
    c.col_y = s.coly;
    return c;
}

static int time_config(const Geom &g, const void *W, int prec, const void *in, void *out, int ncol,
                       const StencilConfig &cfg, int reps, hipStream_t st, double *us) {
    StencilArgs a{};
    a.g = g;
    a.W = W;
    a.in = in;
    a.out = out;
    a.ncol = ncol;
    a.diag = 0.875;
    int rc = stencil_launch(a, prec, false, EPI_PLAIN, cfg, st);  // warm-up, and rejects invalid configs
    if (rc != BRI_OK) return rc;
    hipEvent_t e0, e1;
    BRI_HIP_CHECK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return BRI_EHIP;
    }
    rc = BRI_OK;
    if (hipEventRecord(e0, st) != hipSuccess) rc = BRI_EHIP;
    for (int i = 0; i < reps && rc == BRI_OK; ++i) rc = stencil_launch(a, prec, false, EPI_PLAIN, cfg, st);
    float ms = 0.f;
    if (rc == BRI_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = BRI_EHIP;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *us = 1e3 * ms / reps;
    return rc;
}

static std::vector<StencilConfig> candidates(const Geom &g, int prec, int ncol) {
    std::vector<StencilConfig> out;
    std::vector<std::array<int, 6>> trav;  // tile x, y, z, t, colz, coly
    const int tx_opts[5][2] = {{8, 8}, {16, 4}, {4, 16}, {32, 2}, {64, 1}};
    for (const auto &t : tx_opts)
        for (int cz : {2, 4, 8, 16})
            if (g.L[0] % t[0] == 0 && g.L[1] % t[1] == 0 && g.L[2] % cz == 0) {
                trav.push_back({t[0], t[1], 1, 1, cz, 1});
                // whole-line tiles also in columns several tile rows wide (y fastest inside), the
                // widths of the defaults among them
                for (int cy : {2, 8, 16})
                    if (t[0] == g.L[0] && cz <= 4 && (g.L[1] / t[1]) % cy == 0)
                        trav.push_back({t[0], t[1], 1, 1, cz, cy});
            }
    trav.push_back({0, 0, 0, 0, 0, 0});  // automatic lexicographic tile
    std::vector<std::pair<int, int>> work;  // (nsplit, rpt)
    if (ncol == 1) {
        work = {{2, 0}, {4, 0}};
    } else if (ncol < 4) {
        work = {{4, 0}, {4, ncol}};
    } else {
        // one right-hand side per thread too: the column groups of a tile run together and share
        // its links in L2 (the bfloat16-link default for batches on whole-line tiles)
        work = {{4, 0}, {4, 2}, {4, 3}, {4, 4}};
    }
    for (const auto &t : trav)
        for (const auto &w : work)
            for (int xcd : {0, 1}) {
                StencilConfig c;
                for (int mu = 0; mu < 4; ++mu) c.tile[mu] = t[mu];
                c.colz = t[4];
                c.coly = t[5];
                c.nsplit = w.first;
                c.rpt = w.second;
                c.xcd_remap = xcd;
                out.push_back(c);
                // the x-line kernels where the tile spans whole x-lines
                if (w.second != 1 && t[0] == g.L[0]) {
                    c.variant = VAR_XLINE;
                    out.push_back(c);
                }
            }
    // the matrix-core transport (FP32 / bfloat16 links), on the tiles and traversals above
    if (prec != BRI_F64)
        for (const auto &t : trav)
            for (int rpt : {1, 2, 3, 4}) {
                if (rpt > 1 && ncol < 2) continue;
                StencilConfig c;
                for (int mu = 0; mu < 4; ++mu) c.tile[mu] = t[mu];
                c.colz = t[4];
                c.coly = t[5];
                c.nsplit = 4;
                c.rpt = rpt;
                c.xcd_remap = 1;
                c.variant = VAR_MFMA;
                out.push_back(c);
            }
    // t-streaming kernel (one right-hand side per block row): xyz tiles of 256 sites, t-chunks
    if (ncol <= 4) {
        const int xyz[6][3] = {{8, 8, 4}, {16, 4, 4}, {8, 4, 8}, {16, 8, 2}, {32, 8, 1}, {16, 16, 1}};
        for (const auto &t : xyz)
            for (int ct : {4, 8, 16})
                for (int xcd : {0, 1}) {
                    StencilConfig c;
                    c.tile[0] = t[0];
                    c.tile[1] = t[1];
                    c.tile[2] = t[2];
                    c.tile[3] = ct;
                    c.colz = 0;
                    c.nsplit = 1;
                    c.rpt = 0;
                    c.xcd_remap = xcd;
                    c.variant = VAR_TSTREAM;
                    int tile[4], nb[4];
                    if (plan_tile(g, c, tile, nb) == BRI_OK) out.push_back(c);
                }
    }
    return out;
}

}  // namespace bri

extern "C" {

int bri_stencil_time(const bri_geom *geom, const void *W, int prec, const void *in, void *out, int nrhs,
                     const bri_stencil_cfg *cfg, int reps, double *us_per_launch, void *stream) {
    using namespace bri;
    Geom g;
    int rc = geom_check(geom, &g);
    if (rc != BRI_OK) return rc;
    if (!W || !in || !out || !us_per_launch || nrhs < 1 || reps < 1 || g.V % 64) return BRI_EINVAL;
    if (prec != BRI_F64 && prec != BRI_F32 && prec != BRI_F32_BF16W) return BRI_EINVAL;
    const StencilConfig c = cfg ? from_public(*cfg) : default_config(g, prec, nrhs);
    if (c.rpt == 0 && nrhs > 65535) return BRI_EINVAL;
    return time_config(g, W, prec, in, out, nrhs, c, reps, (hipStream_t)stream, us_per_launch);
}

int bri_autotune(const bri_geom *geom, const void *W, int prec, const void *in, void *out, int nrhs, int reps,
                 bri_stencil_cfg *best, double *best_us, void *stream) {
    using namespace bri;
    Geom g;
    int rc = geom_check(geom, &g);
    if (rc != BRI_OK) return rc;
    if (!W || !in || !out || nrhs < 1 || reps < 1 || g.V % 64) return BRI_EINVAL;
    if (prec != BRI_F64 && prec != BRI_F32 && prec != BRI_F32_BF16W) return BRI_EINVAL;
    double bus = 1e300;
    StencilConfig bc{};
    bool found = false;
    for (const StencilConfig &c : candidates(g, prec, nrhs)) {
        double us = 0.0;
        rc = time_config(g, W, prec, in, out, nrhs, c, reps, (hipStream_t)stream, &us);
        if (rc == BRI_EINVAL) continue;  // configuration does not fit this lattice
        if (rc != BRI_OK) return rc;
        if (us < bus) {
            bus = us;
            bc = c;
            found = true;
        }
    }
    if (!found) return BRI_EINVAL;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[key_of(g, prec, nrhs)] = bc;
    }
    if (best) *best = to_public(bc);
    if (best_us) *best_us = bus;
    return BRI_OK;
}

int bri_set_stencil_cfg(const bri_geom *geom, int prec, int nrhs, const bri_stencil_cfg *cfg) {
    using namespace bri;
    Geom g;
    int rc = geom_check(geom, &g);
    if (rc != BRI_OK) return rc;
    if (nrhs < 1) return BRI_EINVAL;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!cfg) {
        g_tuned.erase(key_of(g, prec, nrhs));
        return BRI_OK;
    }
    StencilConfig c = from_public(*cfg);
    int tile[4], nb[4];
    if (plan_tile(g, c, tile, nb) != BRI_OK) return BRI_EINVAL;
    if (c.variant < VAR_STANDARD || c.variant > VAR_MFMA) return BRI_EINVAL;
    if (c.rpt < 0 || c.rpt > 4 || (c.variant != VAR_TSTREAM && c.rpt == 0 && c.nsplit != 1 && c.nsplit != 2 &&
                                   c.nsplit != 4))
        return BRI_EINVAL;
    g_tuned[key_of(g, prec, nrhs)] = c;
    return BRI_OK;
}

int bri_get_stencil_cfg(const bri_geom *geom, int prec, int nrhs, bri_stencil_cfg *cfg) {
    using namespace bri;
    Geom g;
    int rc = geom_check(geom, &g);
    if (rc != BRI_OK) return rc;
    if (!cfg || nrhs < 1) return BRI_EINVAL;
    *cfg = to_public(default_config(g, prec, nrhs));
    return BRI_OK;
}

}  // extern "C"
