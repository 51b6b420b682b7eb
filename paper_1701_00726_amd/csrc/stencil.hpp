// Internal interface of the Brillouin stencil kernels and of the per-column
// state the multi-shift solver shares with their fused epilogues.
#pragma once

#include "common.hpp"

namespace bri {

constexpr int MAXS = BRI_MAX_SHIFTS;
constexpr int MRHS_SPLIT = 4;  // waves per tile of the multi-RHS stencil kernel


// FP64 scalars of one column (one right-hand side) of a batched multi-shift CG.
struct ColState {
    double rr, bnorm2, tol2;
    double alpha, alpha_old, beta, beta_old;
    double sigma0;
    int iter, done, status, nshift;
    double c0;
    double delta[MAXS], omega[MAXS];
    double tolf2[MAXS];     // squared per-shift factor on the stopping tolerance
    int joint;              // stop on the result bound sum_i ebw_i |r_i| <= tol |b| (else per shift)
    double ebw[MAXS];       // omega_i / (2 sqrt(sigma_i)): weight of |r_i| in that bound
    double zeta[MAXS], zeta_old[MAXS], zeta_new[MAXS];
    double alpha_s[MAXS], beta_s[MAXS];
    int active[MAXS];       // shift still iterating
    int upd_x[MAXS];        // shift takes its alpha^sigma step in this iteration
    int conv_iter[MAXS];
    double conv_res[MAXS];  // |zeta r| / |b| when the shift stopped
};

// fused epilogues of the stencil kernels (per column c)
enum EpiMode {
    EPI_PLAIN = 0,  // out = D in
    EPI_NORMS = 1,  // out = D in; partial sums of |out|^2 and |in|^2
    EPI_CG_R = 2,   // r -= alpha_c (D in + sigma0_c p); partial sums of |r|^2
    EPI_OV = 3,     // out = rho (b + D in)
    EPI_SIGN = 4,   // out = gamma5 D in
    EPI_RESID = 5   // out = b_{c mod b_mod} - (D in + sig_c xs); partial sums of |out|^2
};

struct StencilArgs {
    Geom g;
    int tile[4];  // 64-site tile extents (t-streaming: xyz tile of 256 sites and the t-chunk length)
    int nb[4];    // tiles per axis
    int colz;     // column traversal depth in z (0 = lexicographic tiles)
    int coly;     // column traversal width in tile rows along y (>= 1)
    int xcd_remap;
    int ncol;     // columns (right-hand sides); column c lives at offset c * 12 V
    int nslots;   // partial-sum slots per column the reductions read (V / 64, one per 64-site tile,
                  // filled by the tile's block); a kernel with fewer blocks zeroes the slots it does
                  // not fill
    const void *W;
    const void *in;
    void *out;
    double diag;  // kernel_diag(kind) + m0
    int kind;     // KernelKind
    // epilogue operands
    double *partial;        // EPI_NORMS / EPI_CG_R / EPI_RESID: [ncol][nblk][2]
    const void *p;          // EPI_CG_R
    void *r;                // EPI_CG_R
    const ColState *st;     // EPI_NORMS / EPI_CG_R: alpha, sigma0 and the done flag per column
    const void *b;          // EPI_OV / EPI_RESID
    int b_mod;              // EPI_RESID: column c uses b column (c % b_mod)
    const void *xs;         // EPI_RESID
    const double *sig;      // EPI_RESID: shift per column
    double rho;             // EPI_OV
};

struct StencilConfig {
    int tile[4];    // 0 = automatic
    int colz;       // column traversal: z-planes per column (0 = lexicographic tiles)
    int coly = 0;   // column traversal: tile rows along y per column (0 = 1)
    int nsplit;     // 1-RHS kernel: waves per 64-site tile (1, 2, 4)
    int rpt;        // multi-RHS kernel: right-hand sides per thread (0 = use the 1-RHS kernel)
    int xcd_remap;  // 1 = give each XCD a contiguous range of tiles
    int variant = 0;  // 1-RHS kernel variant (rpt must be 0 for 1 and 2):
                      //   VAR_STANDARD  the 64-site tile kernel above;
                      //   VAR_TSTREAM   t-streaming: xyz tile tile[0..2] (256 sites), chunks of
                      //                 tile[3] t-slices;
                      //   VAR_XLINE     64-site tiles spanning whole x-lines (tile[0] = L_x): the
                      //                 three x-displacements of every (dy, dz, dt) share one
                      //                 spinor load, the x-neighbours come by cross-lane moves
                      //   VAR_MFMA      FP32 / bfloat16 links only: rpt (1..4) right-hand sides
                      //                 per thread, the colour transport on the matrix cores
};

enum StencilVariant { VAR_STANDARD = 0, VAR_TSTREAM = 1, VAR_XLINE = 2, VAR_MFMA = 3 };

constexpr int STREAM_THREADS = 256;  // sites (threads) per block of the t-streaming kernel

// process-wide table of tuned configurations, keyed by lattice, precision and
// number of columns; default_config consults it first
bool tuned_config(const Geom &g, int prec, int ncol, StencilConfig *out);

int geom_check(const bri_geom *geom, Geom *g);
int plan_tile(const Geom &g, const StencilConfig &cfg, int tile[4], int nb[4]);
StencilConfig default_config(const Geom &g, int prec, int ncol, int kind = KERN_BRI);
int stencil_launch(StencilArgs a, int prec, bool dag, int mode, const StencilConfig &cfg, hipStream_t st);

inline int stencil_blocks(const Geom &g) { return g.V / 64; }

}  // namespace bri
