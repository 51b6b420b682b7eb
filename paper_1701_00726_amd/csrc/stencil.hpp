// Internal interface of the Brillouin stencil kernels.
#pragma once

#include "common.hpp"

namespace bri {

// fused epilogues of the stencil kernel
enum EpiMode {
    EPI_PLAIN = 0,  // out = D in
    EPI_NORMS = 1,  // out = D in; partial sums of |out|^2 and |in|^2
    EPI_CG_R = 2,   // r -= alpha (D in + sigma0 p); partial sums of |r|^2
    EPI_OV = 3,     // out = rho (b + D in)
    EPI_SIGN = 4    // out = gamma5 D in
};

struct StencilArgs {
    Geom g;
    int tile[4];  // 64-site tile extents
    int nb[4];    // tiles per axis
    int xcd_remap;
    const void *W;
    const void *in;
    void *out;
    double diag;  // 15/8 + m0
    // epilogue operands
    double *partial;       // EPI_NORMS / EPI_CG_R: 2 doubles per block
    const void *p;         // EPI_CG_R
    void *r;               // EPI_CG_R
    const double *alpha;   // EPI_CG_R (device scalar)
    double sigma0;         // EPI_CG_R
    const void *b;         // EPI_OV
    double rho;            // EPI_OV
    const int *done;       // solver loop: skip the launch body once converged
};

struct StencilConfig {
    int tile[4];    // 0 = automatic
    int nsplit;     // waves per 64-site tile (1, 2, 4)
    int xcd_remap;  // 1 = give each XCD a contiguous range of tiles
};

int geom_check(const bri_geom *geom, Geom *g);
int plan_tile(const Geom &g, const StencilConfig &cfg, int tile[4], int nb[4]);
StencilConfig default_config(const Geom &g, int prec);
int stencil_launch(StencilArgs a, int prec, bool dag, int mode, int nrhs, const StencilConfig &cfg, hipStream_t st);

inline int stencil_blocks(const Geom &g) { return g.V / 64; }

}  // namespace bri
