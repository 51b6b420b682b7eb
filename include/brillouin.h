/*
 * brillouin.h -- C ABI of the MI355X library for the Brillouin-kernel overlap
 * operator (S. Duerr, G. Koutsou, arXiv:1701.00726).
 *
 * Operator conventions (lattice spacing a = 1):
 *   D_bri(m0) = sum_mu gamma_mu nabla^iso_mu - (1/2) lap^bri + m0   eq. (def_bril)
 *               [- (c_SW/2) sum_{mu<nu} sigma_mu_nu F_mu_nu when bri_geom.csw != 0]
 *   D_wil(m0)   likewise with the standard derivative and 9-point Laplacian, eq. (def_wils)
 *   X         = D_bri(-rho),  H = gamma5 X,  A = X^dag X = H^2
 *   D_ov      = rho (1 + gamma5 sign(H))                               eq. (def_over)
 *   sign(H)  ~= g_{2n+1}(H) = H r_n(H^2),
 *   r_n(t)    = c0 + sum_{i<n} omega_i / (t + sigma_i)                 eq. (KLnn_parfrac)
 *   so D_ov psi ~= rho (psi + X r_n(A) psi), sign(H) psi ~= gamma5 X r_n(A) psi.
 *
 * Lattice and layouts.  Extents L = {Lx, Ly, Lz, Lt}, direction mu = 0..3 is
 * x, y, z, t; site s = x + Lx*(y + Ly*(z + Lz*t)), V = Lx*Ly*Lz*Lt.  All fields
 * are structure-of-arrays with the site index fastest and complex numbers
 * interleaved (re, im):
 *   U    [4][3][3][V]        thin (or smeared) gauge links, complex double
 *   W    [40][3][3][V]       off-axis links, complex double / float / bfloat16, followed
 *                            when csw != 0 by the clover term [2][6][6][V] (48 slabs in all)
 *   psi  [nrhs][4][3][V]     spinors: spin, colour, site
 * Gamma matrices (chiral basis): gamma_k = [[0, -i s_k], [i s_k, 0]] with the
 * Pauli matrices s_k, gamma_4 = [[0, 1], [1, 0]], gamma5 = diag(1, 1, -1, -1).
 * Displacements d in {-1,0,1}^4 carry the index j = sum_mu (d_mu + 1) 3^mu,
 * so that j and 80 - j are opposite and j = 40 is d = 0 (App. C.1).  Only the
 * 40 links with j < 40 are stored; W_{80-j}(x) = W_j(x + d_{80-j})^dag.
 *
 * Memory: every pointer argument named U, W*, in, out, work is a DEVICE pointer
 * owned by the caller; the library never frees caller memory.  Host pointers
 * are the geometry, parameter and statistics structs and work_bytes.
 * Streams: `stream` is a hipStream_t (NULL = the null stream); the stencil, FP64 link and
 * force calls are asynchronous on it; the solver calls (ov_*) and the autotuner
 * synchronise it before returning (they read convergence flags or timings on the host).
 * Errors: no call aborts, prints or throws.  A call returns BRI_OK or a
 * negative status; on BRI_EINVAL nothing was launched.
 */
#ifndef BRILLOUIN_H
#define BRILLOUIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* lattice geometry; tbc = 1 makes the fermion field antiperiodic in t.
 * Accepted: L_mu in 1..4096, tbc 0 or 1, finite csw, and V = L_0 L_1 L_2 L_3 < 2^31 sites
 * (site indices are 32-bit, element offsets 64-bit; device memory is the practical bound:
 * 5760 V bytes of FP64 links, e.g. 61 GB at 48^3 x 96).  Every operator call also needs V to
 * be a multiple of 64 (the stencil tiles 64 sites per wave).  Anything else returns
 * BRI_EINVAL. */
typedef struct {
    int32_t L[4];
    int32_t tbc;
    double csw; /* clover coefficient c_SW of eqs. (def_wils), (def_bril); 0 = no clover term.
                   bri_build_links then appends the clover field to the link array, and
                   every operator built on that array applies it (pass the same value). */
} bri_geom;

/* storage / arithmetic precision of a field */
typedef enum {
    BRI_F64 = 0,      /* complex double spinors, complex double links          */
    BRI_F32 = 1,      /* complex float spinors, complex float links            */
    BRI_F32_BF16W = 2 /* complex float spinors, links as (re, im) bfloat16     */
} bri_prec;

typedef enum {
    BRI_OK = 0,
    BRI_EINVAL = -1,  /* bad geometry, pointer, precision, size or workspace  */
    BRI_ENOCONV = -2, /* solver hit max_iter; out holds the last iterate      */
    BRI_ENAN = -3,    /* non-finite value met in a reduction                  */
    BRI_EHIP = -4,    /* a HIP runtime call failed                            */
    BRI_ESCRATCH = -5 /* ov_apply_noalloc: the problem's workspace exceeds the
                         library's static scratch (ov_noalloc_max_bytes)       */
} bri_status;

/* Largest supported Kenney-Laub order n (number of shifts). */
#define BRI_MAX_SHIFTS 32

/*
 * bri_build_links -- off-axis links of the Brillouin stencil (App. C.1).
 * W_d(x) is the average over the k! shortest paths from x to x + d
 * (k = number of non-zero d_mu) of the ordered product of links along the
 * path; a step +mu at y contributes U_mu(y), a step -mu contributes
 * U_mu(y - mu)^dag.  No projection back to SU(3).  Computed in FP64 and rounded
 * to `wprec` on store.
 * With geom->csw != 0 the clover term -(c_SW/2) sum_{mu<nu} sigma_mu_nu F_mu_nu follows the
 * links: F_mu_nu the hermitian traceless part of the clover-leaf average of the four
 * plaquettes at x, sigma_mu_nu = (i/2)[gamma_mu, gamma_nu]; stored as its two chirality
 * blocks (spins 0,1 and 2,3), 6x6 entries each, index 3*spin + colour within the block.
 *   U  : [4][3][3][V] complex double (device, read)
 *   W  : [40][3][3][V] (csw = 0) or [48][3][3][V] (csw != 0) in precision wprec (device, written)
 * Returns BRI_EINVAL for a geometry outside the limits stated at bri_geom, a null pointer or W
 * overlapping U,
 * BRI_EHIP on a HIP failure.  Asynchronous on `stream` for wprec = BRI_F64; for the lower
 * precisions a temporary FP64 buffer of 5760*V bytes (6912*V with the clover term) is
 * allocated, and the call synchronises `stream` before freeing it (bri_round_links takes an
 * FP64 array already built instead, without either).
 */
int bri_build_links(const bri_geom *geom, const void *U, void *W, int wprec, void *stream);

/*
 * bri_round_links -- the link array of bri_build_links rounded from FP64 to wprec = BRI_F32 or
 * BRI_F32_BF16W, entry by entry (the rounding bri_build_links applies on store), for a caller
 * that holds the FP64 array already: the mixed-precision applies take both.  geom->csw != 0:
 * the clover slabs are rounded with the links.
 *   W64 : [40 or 48][3][3][V] complex double (device, read)
 *   W   : the same shape in precision wprec (device, written); must not overlap W64
 * Returns BRI_EINVAL for a bad geometry, precision or pointer, or overlapping arrays; BRI_EHIP
 * on a launch failure.  Asynchronous on `stream`; allocates nothing.
 */
int bri_round_links(const bri_geom *geom, const void *W64, void *W, int wprec, void *stream);

/*
 * bri_apply -- out = D_bri(m0) in, the 81-point sum (App. C.1)
 *   (D psi)(x) = (15/8 + m0) psi(x) + sum_{d != 0} S_d W_d(x) psi(x + d),
 *   S_d = -2^{-(k+3)} + c_k sum_{mu in supp d} d_mu gamma_mu,
 *   c_k = 4/27, 1/27, 1/108, 1/432 for k = 1..4 hops
 * (position-space weights of the isotropic derivative and the Brillouin
 * Laplacian, App. A momentum forms), plus the clover term on the diagonal when
 * geom->csw != 0 (W must then hold it; only whether csw is zero matters here).
 *   W   : [40][3][3][V] in precision prec (F64: double; F32: float;
 *         F32_BF16W: bfloat16 links with float spinors)
 *   in, out : [nrhs][4][3][V], complex double for BRI_F64, complex float
 *         otherwise; in and out must not overlap (BRI_EINVAL if they do).
 */
int bri_apply(const bri_geom *geom, const void *W, int prec, double m0, const void *in, void *out, int nrhs,
              void *stream);

/* bri_apply_dag -- out = D_bri(m0)^dag in = gamma5 D_bri(m0) gamma5 in
 * (gamma5-hermiticity, Sec. 4).  Arguments as bri_apply. */
int bri_apply_dag(const bri_geom *geom, const void *W, int prec, double m0, const void *in, void *out, int nrhs,
                  void *stream);

/* Kernel operator X of the overlap (ov_params.kernel). */
enum bri_kernel {
    BRI_KERNEL_BRILLOUIN = 0, /* D_bri, eq. (def_bril): the 81-point stencil                   */
    BRI_KERNEL_WILSON = 1     /* D_wil, eq. (def_wils): the 9-point stencil, reading the four
                                 one-hop slabs of the same link array (either with the clover
                                 term when the geometry's csw != 0)                          */
};

/* Kenney-Laub family member used for sign(H) (ov_params.kind). */
enum bri_kl_kind {
    BRI_KL_DIAG = 0, /* diagonal f_{n,n} = g_{2n+1}, eq. (KLnn_parfrac): c0 + n poles           */
    BRI_KL_UPPER = 1 /* first upper diagonal f_{n-1,n} = g_{2n} (Sec. 3.3, Tab. 6): n poles, no
                        constant term                                                         */
};

/* Stopping rule of the multi-shift solve (ov_params.relax); r_i = b - (A + sigma_i) x_i. */
enum bri_relax {
    BRI_RELAX_OFF = 0,   /* every shift stops at |r_i| <= tol |psi|                          */
    BRI_RELAX_OMEGA = 1, /* shift i stops at |r_i| <= tol |psi| omega_max / omega_i (App. B: the
                            small shifts carry small weights, so they may stop earlier)       */
    BRI_RELAX_BOUND = 2  /* tol bounds the result instead: the solve stops once
                              sum_i omega_i |r_i| / (2 sqrt(sigma_i)) <= tol |psi|,
                            which bounds the error of sign(H) psi (and of D_ov psi / rho),
                            because |X (X^dag X + sigma)^-1| = max_s s / (s^2 + sigma)
                            <= 1 / (2 sqrt(sigma)) over the singular values s of X; shift i
                            stops by itself once its term is at most tol |psi| / (2n).
                            ov_apply, ov_sign_apply and ov_solve only (the gradient and the
                            cascade's levels reject or ignore it)                           */
};

/*
 * wil_apply     -- out = D_wil(m0) in,  eq. (def_wils):
 *   (D psi)(x) = (4 + m0) psi(x) - (1/2) sum_mu [(1 - gamma_mu) U_mu(x) psi(x+mu)
 *                                               + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu)]
 *               [+ the clover term when geom->csw != 0]
 * wil_apply_dag -- out = D_wil(m0)^dag in = gamma5 D_wil(m0) gamma5 in.
 * W is the link array of bri_build_links (its four one-hop slabs are U_mu(x - mu)^dag with the
 * boundary signs folded in; the other slabs are not read), so both kernels share one set-up.
 * Arguments, layouts and errors as bri_apply.
 */
int wil_apply(const bri_geom *geom, const void *W, int prec, double m0, const void *in, void *out, int nrhs,
              void *stream);
int wil_apply_dag(const bri_geom *geom, const void *W, int prec, double m0, const void *in, void *out, int nrhs,
                  void *stream);

/* Parameters of the overlap applies. */
typedef struct {
    int kl_n;       /* Kenney-Laub order n: f_{n,n} = g_{2n+1}, 1..BRI_MAX_SHIFTS */
    double rho;     /* 0 < rho < 2; kernel mass m0 = -rho                        */
    double tol;     /* per-shift stop |b - (A + sigma) x_sigma| <= tol |psi|, or
                       the result bound (relax = BRI_RELAX_BOUND)                */
    int max_iter;   /* multi-shift CG iteration cap                              */
    int inner;      /* bri_prec of the late iterations: BRI_F64 (all FP64), or
                       BRI_F32 / BRI_F32_BF16W (FP32 vectors on Wlo once the base
                       residual has fallen to tol / u_lo |psi|, see ov_apply)   */
    int max_refine; /* unused (0..100 accepted)                                 */
    int kind;       /* bri_kl_kind; BRI_KL_DIAG unless stated                   */
    int relax;      /* bri_relax; BRI_RELAX_OFF unless stated (ov_apply_grad:
                       BRI_EINVAL for BRI_RELAX_BOUND)                          */
    int kernel;     /* bri_kernel: X = D_kernel(-rho); BRI_KERNEL_BRILLOUIN unless
                       stated                                                  */
    int recompute;  /* ov_apply_grad only: 0 keeps all 2n shift solutions of one
                       multi-shift solve; m in 1..kl_n solves the shifts m at a
                       time and keeps only those (workspace for 4m instead of
                       ~6n vectors, at the cost of a solve per group)           */
} ov_params;

/* Statistics of one overlap apply; for nrhs > 1 each figure is the worst column's. */
typedef struct {
    int iters;                          /* multi-shift CG iterations            */
    int refine;                         /* of those, run in the low-precision phase */
    int shift_iters[BRI_MAX_SHIFTS];    /* iteration at which each shift stopped */
    double rel_resid[BRI_MAX_SHIFTS];   /* |zeta_sigma r| / |psi| at that point (the
                                           recursively updated residual)        */
    double seconds;                     /* host wall time of the call            */
} ov_stats;

/*
 * ov_sign_apply -- out ~= sign(H) in = gamma5 X r_n(X^dag X) in, H = gamma5 X, X = D_kernel(-rho)
 *                  (params->kernel: Brillouin or Wilson; with the clover term when csw != 0)
 * ov_apply      -- out ~= D_ov in   = rho (in + X r_n(X^dag X) in)          eq. (def_over)
 * r_n(A) in is evaluated by one multi-shift CG on A + sigma_min for all n
 * shifts at once (Sec. 3.3), with the coefficients of eq. (KLnn_parfrac) (or of the
 * first upper diagonal, params->kind); the
 * nrhs right-hand sides run side by side, each with its own Krylov space.
 * Mixed precision (inner = BRI_F32 or BRI_F32_BF16W): the multi-shift runs in FP64
 * until the base residual of every right-hand side is at most (tol / u_lo) |psi|,
 * u_lo = 2^-24 (BRI_F32) or 2^-8 (BRI_F32_BF16W); from there (at once if that
 * bound exceeds 1) its vectors r, p, p_sigma are FP32 and its stencils read Wlo,
 * while y = c0 psi + sum omega_sigma x_sigma keeps accumulating in FP64 and every
 * scalar stays FP64.  A low-precision product then perturbs the result by about
 * tol |psi| (the relaxation rule of inexact Krylov methods), so no shift needs a
 * separate correction.  The final X y uses W64.
 * The shifted directions and y are written once per window of 8 iterations: in between
 * they are carried as coefficients of the residuals the window stores (8 per right-hand
 * side in the workspace, and 8 FP32 ones for a low-precision inner), so an iteration
 * streams r and p rather than every p_sigma and y.  The result is the same sum taken in
 * another order.
 *   W64 : [40][3][3][V] complex double off-axis links ([48]... with the clover term)
 *   Wlo : links in precision `inner` (from bri_build_links); NULL when inner = BRI_F64
 *   in, out : [nrhs][4][3][V] complex double (device); must not overlap each other or the
 *         used part of the workspace (BRI_EINVAL if they do)
 *   work, work_bytes : device workspace; with work == NULL the call only writes
 *         the required size into *work_bytes and returns BRI_OK.
 *   stats : may be NULL.
 * Returns BRI_ENOCONV when max_iter is reached before every shift met tol
 * (out then holds the result of the last iterate), BRI_ENAN on a non-finite
 * residual.
 */
int ov_sign_apply(const bri_geom *geom, const void *W64, const void *Wlo, const ov_params *params, const void *in,
                  void *out, int nrhs, void *work, size_t *work_bytes, ov_stats *stats, void *stream);
int ov_apply(const bri_geom *geom, const void *W64, const void *Wlo, const ov_params *params, const void *in,
             void *out, int nrhs, void *work, size_t *work_bytes, ov_stats *stats, void *stream);

/*
 * ov_apply_noalloc -- ov_apply for callers that cannot allocate (no hipMalloc, hipFree, pinned
 * host memory or HIP-graph instantiation on their path): the same computation and kernels, with
 * the shifted directions and y updated every iteration (no window of stored residuals, so a
 * smaller workspace) taken from a static device array of ov_noalloc_max_bytes() = 256 MiB that
 * the library holds on each GPU it runs on until the process ends (enough for a 16^4 FP64 apply
 * of one right-hand side with 16 shifts).  The caller passes inputs and outputs as for ov_apply;
 * stats may be NULL.  Returns BRI_ESCRATCH, before launching anything, when that workspace
 * exceeds the array.  The array's address is resolved on the first call
 * on each device.  Every call on a GPU uses that GPU's one array and nothing in it needs to be
 * cleared between calls (each call initialises what it reads); calls that overlap in time on
 * one GPU (other streams or host threads) race on it and must be serialised by the caller.
 * Synchronises `stream` (it polls the solver's convergence flag, as ov_apply does).
 */
int ov_apply_noalloc(const bri_geom *geom, const void *W64, const void *Wlo, const ov_params *params, const void *in,
                     void *out, int nrhs, ov_stats *stats, void *stream);
size_t ov_noalloc_max_bytes(void);

/*
 * Outer solve of the massive overlap equation (Sec. 4; BiCGstab outer solver of Sec. 7):
 *   (D_ov + mt) x = bt,  mt = m / (1 - m/(2 rho)),
 *   complete form (eq. (upshot_complete)):   bt = [1 + (m/(2 rho)) (1 - D_ov/(2 rho))] b / (1 - m/(2 rho))
 *   traditional (eq. (upshot_traditional)):  bt = b / (1 - m/(2 rho))
 * with lattice spacing 1.  Every application of D_ov is one ov_apply with `params` (the inner
 * multi-shift); its tolerance should be well below the outer one.
 *
 * Cascaded preconditioning (Sec. 8, eqs. (cascaded_one), (cascaded_two)): the outer BiCGstab can
 * be preconditioned from the right by a chain of cheaper operators of the same massive form,
 *   A_k = rho [D^(k) + 1 + mt/rho],  D^(k) = X r_{n_k}(X^dag X)  (the overlap approximant of
 *   Kenney-Laub order n_k, so A_k = D_ov^(n_k) + mt),  D^(0) = X = D_kernel(-rho),
 * each inverted approximately by its own BiCGstab (stopped at a loose tolerance or an iteration
 * cap) that is preconditioned by the next operator of the chain.  The paper's one-level scheme
 * for f_{1,1} is params->kl_n = 1 with prec = {Brillouin}; its two-level scheme for f_{4,4} is
 * kl_n = 4 with prec = {n = 1, Brillouin}.  The same bare mass is used at every level.
 */
#define BRI_MAX_LEVELS 4
#define BRI_MAX_SOLVE_RHS 16

typedef struct {
    double mass;  /* bare quark mass m, 0 <= m < 2 rho                               */
    int complete; /* 1: complete massive form, 0: traditional                        */
    double tol;   /* outer stop: recursive |bt - (D_ov + mt) x| <= tol |bt|          */
    int max_iter; /* outer BiCGstab iterations                                       */
} ov_mass_params;

/* One preconditioner level. */
typedef struct {
    int kl_n;      /* 0: the kernel operator itself (Brillouin or Wilson as params->kernel; must
                      be the last level), else 1..BRI_MAX_SHIFTS                          */
    double tol;    /* stop of this level's BiCGstab, relative to the vector it is applied to   */
    int max_iter;  /* iteration cap of this level's BiCGstab, per application                  */
    double ms_tol; /* multi-shift CG tolerance of this level's overlap applies (kl_n > 0)       */
    int inner;     /* bri_prec of this level's multi-shift (kl_n > 0) or of its kernel stencil
                      (kl_n = 0: vectors narrowed to complex float around each apply); low
                      precision reads Wlo, so every low-precision level must name Wlo's
                      precision                                                           */
} ov_level;

typedef struct {
    int iters;                          /* outer BiCGstab iterations (until every column met
                                           tol)                                               */
    int inner_iters;                    /* multi-shift CG iterations summed over every level  */
    int applies;                        /* D_ov applies of the outer level (bt, two per
                                           iteration, the final check)                        */
    double rel_resid;                   /* true |bt - (D_ov + mt) x| / |bt| at exit, worst
                                           column                                             */
    int level_iters[BRI_MAX_LEVELS];    /* BiCGstab iterations summed per preconditioner level */
    int level_calls[BRI_MAX_LEVELS];    /* applications of each preconditioner level          */
    int level_applies[BRI_MAX_LEVELS];  /* operator applies of each preconditioner level      */
    double seconds;                     /* host wall time of the call                         */
} ov_solve_stats;

/*
 * ov_solve -- x = (D_ov + mt)^{-1} bt for nrhs right-hand sides side by side (each with its own
 * BiCGstab scalars and stopping test; every operator application treats all of them in one
 * batched call, as the paper's 12-source solves do).
 *   W64, Wlo, params : as ov_apply (params->kl_n is the order of the operator solved for; Wlo is
 *          needed when params->inner or any level's inner is low precision)
 *   mp    : mass, form, outer tolerance and iteration cap
 *   nprec, prec : preconditioner chain, 0..BRI_MAX_LEVELS levels (prec may be NULL for 0);
 *          prec[0] preconditions the outer operator, prec[k+1] preconditions prec[k]
 *   in    : b, [nrhs][4][3][V] complex double;  out : x, same layout; in, out and the used
 *           workspace must not overlap (BRI_EINVAL if they do)
 *   nrhs  : 1..BRI_MAX_SOLVE_RHS
 *   work, work_bytes : device workspace (query with work == NULL)
 *   stats : may be NULL
 * Synchronises `stream`.  Returns BRI_ENOCONV when max_iter outer iterations did not reach tol
 * (out holds the last iterate), BRI_ENAN on a non-finite or breaking-down outer recurrence, the
 * status of a failing outer ov_apply, BRI_EINVAL for bad arguments (m outside [0, 2 rho), a
 * kernel level that is not the last one, low-precision levels of different precisions, no Wlo
 * for a low-precision level).  Preconditioner levels that stop at their cap are not errors.
 */
int ov_solve(const bri_geom *geom, const void *W64, const void *Wlo, const ov_params *params,
             const ov_mass_params *mp, int nprec, const ov_level *prec, const void *in, void *out, int nrhs,
             void *work, size_t *work_bytes, ov_solve_stats *stats, void *stream);

/*
 * Stencil launch configuration and autotuner.  A configuration picks the
 * 64-site tile (tile_x * tile_y * tile_z * tile_t = 64, each dividing its
 * lattice extent; all zero = automatic), the traversal (col_z > 0: tiles of
 * tile_x x tile_y x 1 x 1 walked inside columns of col_y tile rows along y
 * (0 = 1; must divide L_y / tile_y) by col_z z-planes by all of t, y fastest,
 * then z, then t, so that stencil neighbours run together on one XCD; col_z = 0:
 * lexicographic tiles and col_y 0 or 1), the work split (rpt = 0: one right-hand side per
 * block row with nsplit = 1, 2 or 4 waves sharing the 80 displacements;
 * rpt = 1..4: rpt right-hand sides per thread, four waves sharing the
 * displacements, nsplit ignored) and xcd = 1 to give each XCD a
 * contiguous range of tiles.  variant selects the kernel for one right-hand
 * side per block row (rpt = 0; Brillouin kernel only for 1 and 2):
 *   0  the 64-site tile kernel described above;
 *   1  t-streaming: a block of 256 threads owns a tile_x x tile_y x tile_z tile of
 *      the xyz volume (product 256, each dividing its extent) and walks tile_t
 *      consecutive t-slices (dividing L_t), reading both uses of every stored
 *      link inside one slice; col_z and nsplit are ignored;
 *   2  x-line: as 0 with tile_x = L_x (whole x-lines in every wave), the three
 *      x-displacements of each (dy, dz, dt) sharing one spinor load; with
 *      rpt = 2, 3 or 4 right-hand sides per thread as the multi-RHS kernel;
 *   3  matrix cores (BRI_F32 and BRI_F32_BF16W only): rpt = 1..4 right-hand sides
 *      per thread, the colour transport by FP32 MFMA (16 sites per wave, a site's
 *      four spins in four lanes), the spin weights applied across those lanes.
 */
typedef struct {
    int tile_x, tile_y, tile_z, tile_t;
    int col_z;
    int nsplit;
    int rpt;
    int xcd;
    int variant;
    int col_y;
} bri_stencil_cfg;

/* bri_stencil_time -- average time of `reps` back-to-back bri_apply launches
 * (after one warm-up) with configuration cfg (NULL: the current default), in
 * microseconds, measured with HIP events on `stream` (synchronises it).
 * in / out as bri_apply; out is overwritten.  BRI_EINVAL if cfg does not fit. */
int bri_stencil_time(const bri_geom *geom, const void *W, int prec, const void *in, void *out, int nrhs,
                     const bri_stencil_cfg *cfg, int reps, double *us_per_launch, void *stream);

/* bri_autotune -- times every candidate configuration for (geom, prec, nrhs)
 * as bri_stencil_time does and installs the fastest in a process-wide table
 * used by the Brillouin stencils (bri_apply, bri_apply_dag and the overlap solvers on the
 * Brillouin kernel) for that lattice, precision and column count; the Wilson stencil keeps
 * the default configuration.  best / best_us may be NULL. */
int bri_autotune(const bri_geom *geom, const void *W, int prec, const void *in, void *out, int nrhs, int reps,
                 bri_stencil_cfg *best, double *best_us, void *stream);

/* bri_set_stencil_cfg -- installs cfg for (geom, prec, nrhs); cfg = NULL removes
 * the entry.  bri_get_stencil_cfg -- the configuration a launch would use. */
int bri_set_stencil_cfg(const bri_geom *geom, int prec, int nrhs, const bri_stencil_cfg *cfg);
int bri_get_stencil_cfg(const bri_geom *geom, int prec, int nrhs, bri_stencil_cfg *cfg);

/* bri_set_solver_graphs -- enable (1, the default) or disable (0) HIP-graph replay of
 * the multi-shift CG loop.  When enabled, each block of 8 iterations (six launches per
 * iteration) is captured once per solve layout (device, lattice, boundary condition, clover
 * switch, precision, kernel, mass, column count, workspace and link addresses, launch
 * configuration) on a library-owned stream and
 * replayed on the caller's stream; up to 16 instantiated graphs are cached per process and
 * disabling clears them.  Results are identical either way (same kernels, same order).
 * Cached graphs are looked up and launched under a lock, and an evicted or cleared graph is
 * destroyed only after its last launch has completed, so solves in several host threads may
 * share the cache; switching graphs off while other threads solve is not supported (their
 * solves keep launching graphs).  BRI_EINVAL for
 * other values. */
int bri_set_solver_graphs(int enable);

/* Kenney-Laub coefficients c0, omega[n], sigma[n] of f_{n,n} (eq. (KLnn_parfrac)),
 * computed in double precision on the host; sigma ascending. */
int bri_kl_coeffs(int n, double *c0, double *omega, double *sigma);

/* Coefficients omega[n], sigma[n] of the first upper diagonal f_{n-1,n} = g_{2n}
 * = x sum_i omega_i / (x^2 + sigma_i) (Sec. 3.3; Tab. 6 for n <= 3), host double precision,
 * sigma ascending.  BRI_EINVAL for n outside 1..BRI_MAX_SHIFTS or NULL pointers. */
int bri_kl_upper_coeffs(int n, double *omega, double *sigma);

/*
 * Differentiation (Sec. 9: the molecular-dynamics force is the derivative with
 * respect to the Gell-Mann components of log U).  The links are perturbed as
 *   U_mu(x) -> exp(i omega^a lambda_a / 2) U_mu(x),  a = 1..8,
 * and the force is F^a_mu(x) = dS/d omega^a at omega = 0, stored
 *   F    [4][8][V]     double
 * The complex gradient with respect to the link entries, in the convention
 * dS/dRe U + i dS/dIm U (the one torch uses for a real loss), is stored
 *   GU   [4][3][3][V]  complex double (same layout as U).
 * Both follow the off-axis links through their path averages (App. C.1) down
 * to U, with the t-boundary sign of tbc.  The 0-hop term does not depend on U.
 */

/* Most (u, v) pairs bri_link_grad takes in one call. */
#define BRI_MAX_PAIRS (2 * BRI_MAX_SHIFTS + 1)

/*
 * bri_link_grad -- force of S = Re sum_p weights[p] u_p^dag D_bri v_p.
 *   U       [4][3][3][V] complex double links the FP64 W was built from, with
 *           the same geom->tbc
 *   W       [40][3][3][V] complex double off-axis links (bri_build_links, BRI_F64)
 *   npairs  1..BRI_MAX_PAIRS; weights[npairs] on the host
 *   u, v    [npairs][4][3][V] complex double spinors
 *   F       [4][8][V] double, or NULL;  GU [4][3][3][V] complex double, or NULL
 *           (at least one of the two); both overwritten
 *   work, work_bytes: device workspace of 81 * 9 * V complex doubles; with
 *           work == NULL the call only writes the size into *work_bytes.
 * Asynchronous on `stream`.  BRI_EINVAL for bad geometry, npairs or pointers, or when F, GU
 * or work overlap each other or an input.
 */
int bri_link_grad(const bri_geom *geom, const void *U, const void *W, int npairs, const double *weights,
                  const void *u, const void *v, void *F, void *GU, void *work, size_t *work_bytes, void *stream);

/* wil_link_grad -- the same force for S = Re sum_p w_p u_p^dag D_wil v_p (eq. (def_wils)): each
 * link U_mu(z) enters the hops z -> z+mu and z+mu -> z.  W is the link array of bri_build_links
 * (only its one-hop slabs are read); arguments, workspace and errors as bri_link_grad. */
int wil_link_grad(const bri_geom *geom, const void *U, const void *W, int npairs, const double *weights,
                  const void *u, const void *v, void *F, void *GU, void *work, size_t *work_bytes, void *stream);

/*
 * ov_apply_grad -- gradient of S = Re chi^dag D_ov psi (one right-hand side),
 * D_ov = rho (1 + X r_n(A)), with the fixed-order rational of eq.
 * (KLnn_parfrac) differentiated through its partial fractions (Sec. 9):
 *   a_i = (A + sigma_i)^{-1} psi, b_i = (A + sigma_i)^{-1} X^dag chi,
 *   y = c0 psi + sum_i omega_i a_i,
 *   dS = rho Re[chi^dag dX y] - rho sum_i omega_i Re[(X a_i)^dag dX b_i + (X b_i)^dag dX a_i],
 *   gpsi = D_ov^dag chi = rho (chi + c0 X^dag chi + sum_i omega_i b_i)
 *        (= dS/dRe psi + i dS/dIm psi).
 * The a_i and b_i come from one two-column multi-shift solve that keeps every
 * shift solution (x_sigma accumulated in FP64): all FP64 (params->inner = BRI_F64), or
 * with the late iterations on FP32 vectors and the links Wlo, as ov_apply does.
 *   U, W64  as bri_link_grad (W64 built from U with geom->tbc)
 *   Wlo     links in precision params->inner; NULL when inner = BRI_F64
 *   chi, psi, gpsi  [4][3][V] complex double
 *   F, GU   as bri_link_grad (at least one non-NULL)
 *   work, work_bytes  device workspace (query with work == NULL)
 *   stats   may be NULL: iterations (of them in low precision) and the final residual
 *           of each shift (worst of the two columns)
 * Synchronises `stream`.  Returns BRI_ENOCONV when a shift missed tol within
 * max_iter (the outputs then use the last iterates), BRI_ENAN on a non-finite
 * residual, BRI_EINVAL for bad arguments (V must be a multiple of 64; F, GU, gpsi and work must
 * not overlap each other or an input).
 */
int ov_apply_grad(const bri_geom *geom, const void *U, const void *W64, const void *Wlo, const ov_params *params,
                  const void *chi, const void *psi, void *F, void *GU, void *gpsi, void *work, size_t *work_bytes,
                  ov_stats *stats, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* BRILLOUIN_H */
