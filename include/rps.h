/*
 * rps.h -- robust-pseudospectral (rPS) occ-RI exchange for periodic Gaussian
 * basis sets on AMD Instinct MI355X (gfx950).  C ABI, version 1.
 *
 * Method: Sharma, White, Beylkin, "Fast exchange with Gaussian basis set using
 * robust pseudospectral method" (arXiv:2207.04636).  Interpolation points and
 * fitting functions chi_g (ISDF, Sec. 3.1, 4.3), the potentials V of chi_g and
 * W = V chi^T (Sec. 3.2, Eq. 12 and 14) are set up once per geometry.  Each
 * exchange build then evaluates Eq. 16 (occ-RI, Sec. 3.3) without any FFT.
 *
 * Conventions (all public floating point is IEEE binary64, row-major):
 *  - Basis values are plain function values; the paper's pSinc coefficients
 *    are sqrt(dV) times them, dV = Omega / N_g.  Every contraction carries a
 *    single factor dV.
 *  - Coulomb kernel 4 pi / |G|^2 on the plane waves of the grid (Sec. 2.2,
 *    Eq. 7-8) with the G = 0 term removed (Sec. 4.5).  No Madelung term is
 *    added: the paper's nM/2 correction is a constant per (n, cell).
 *  - Grid point R(i1,i2,i3) = sum_k (i_k/N_k) a_k, linear index
 *    (i1*N2 + i2)*N3 + i3.
 *  - Shells: s; p in the order x, y, z; d as five real-spherical components
 *    xy, yz, zx, x^2-y^2, 3z^2-r^2; free-space normalised primitives, one
 *    exponent per shell, periodized by summing lattice images (Sec. 2.1.3).
 *    Basis function order = shell order, components in the order above.
 *  - K_occ[mu][i] = sum_j (mu j | j i)  (N x n_occ), the occ-RI exchange of
 *    Eq. 16; E_x = -tr(C^T K_occ), closed shell with doubly occupied spatial
 *    orbitals.
 *
 * Ownership: the caller owns every input and output buffer; the library copies
 * what it keeps.  A context owns all device memory it allocates and frees it
 * in rps_destroy.  Errors: no function aborts or throws; on failure the
 * outputs are left untouched and rps_last_error() (thread-local) explains.
 * Threading: a context is not thread-safe; use it from one host thread.
 */
#ifndef RPS_H
#define RPS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rps_context rps_context;

typedef enum {
    RPS_OK = 0,
    RPS_ERR_ARG = 1,      /* null pointer, negative size, bad enum value */
    RPS_ERR_SHAPE = 2,    /* inconsistent sizes (e.g. n_aux > N_g, duplicate points) */
    RPS_ERR_NOMEM = 3,    /* memory estimate exceeds free device memory (checked before allocating) */
    RPS_ERR_NOT_PD = 4,   /* fitting metric not positive definite even after the shift */
    RPS_ERR_DEVICE = 5,   /* HIP runtime error */
    RPS_ERR_STATE = 6     /* call out of order (e.g. build before a completed setup) */
} rps_status;

/* Arithmetic of the per-build contractions. */
typedef enum {
    RPS_PREC_FP64 = 0,    /* FP64 MFMA and FP64 accumulation throughout */
    RPS_PREC_FP32 = 1,    /* V stored FP32; FP32 MFMA tiles, FP64 cross-tile accumulation */
    RPS_PREC_BF16X3 = 2   /* V stored FP32; split hi+lo BF16 MFMA products, FP32 in tile, FP64 across */
} rps_precision;

/* Interpolation-point selection (Sec. 4.3). */
typedef enum {
    RPS_SELECT_VORONOI = 0,  /* per-atom randomized selection, then a global pass over the union */
    RPS_SELECT_GLOBAL = 1    /* one randomized selection over the whole grid */
} rps_select_mode;

/* Exchange variants of Eq. 13 (Sec. 3.2). */
typedef enum {
    RPS_VARIANT_RPS = 0,  /* fit.exact + exact.fit - fit.fit (robust, error O(eps^2)) */
    RPS_VARIANT_PS = 1,   /* first line only (pseudospectral, O(eps), asymmetric) */
    RPS_VARIANT_THC = 2   /* third line only (tensor hypercontraction, O(eps)) */
} rps_variant;

#define RPS_PTRS_HOST 0    /* C, K, ex are host pointers; the call is synchronous */
#define RPS_PTRS_DEVICE 1  /* C, K, ex are device pointers; stream-ordered, asynchronous */

/* Periodic cell and grid (Sec. 2.1): lattice rows a1, a2, a3 in bohr; mesh points
 * per axis, each in [2, 256] (RPS_ERR_SHAPE otherwise). */
typedef struct {
    double lattice[9];
    int32_t mesh[3];
} rps_cell;

/* Gaussian basis (Sec. 2.1.3).  Arrays are host memory, read during the call. */
typedef struct {
    int32_t natom;
    int32_t nshell;
    const double *atom_xyz;     /* [natom][3] cartesian positions, bohr */
    const int32_t *shell_atom;  /* [nshell] atom index of each shell (its centre) */
    const int32_t *shell_l;     /* [nshell] 0, 1 or 2 */
    const double *shell_exp;    /* [nshell] exponent > 0, bohr^-2 */
} rps_basis;

/* Sizes and set-up diagnostics of a context. */
typedef struct {
    int64_t ngrid;        /* N_g */
    int64_t nbas;         /* N */
    int64_t naux;         /* N_chi */
    int64_t ngrid_pad, nbas_pad, naux_pad;   /* padded extents of the device arrays */
    int64_t n_candidates; /* |R_h| of the Voronoi selection (0 if points were given) */
    double dvol;          /* Omega / N_g */
    double chol_shift;    /* diagonal shift used by the fitting-metric Cholesky (0 if none) */
    double setup_seconds; /* wall time of rps_setup_isdf */
    int64_t device_bytes; /* device memory held by the context */
    int32_t precision;
    int32_t exact;        /* 1 if n_aux == N_g (chi = identity) */
    double madelung;      /* Madelung constant M of the cell (see rps_madelung_constant) */
    double basis_fill;    /* screened set-up: fraction of the N_g x N basis values held in the
                             atom blocks (1.0 without screening) */
    double basis_pair_fill; /* screened set-up: sum over atoms of |kappa_I| n_I^2 / (N_g N^2),
                               the fraction of the dense J product's work (1.0 without) */
    int32_t build_arith;  /* arithmetic the last exchange build used for its V products, as an
                             rps_precision value (-1 before the first build).  RPS_PREC_BF16X3
                             contexts report RPS_PREC_FP32 where that form runs FP32 products:
                             the fused kernels for n_occ <= 16 and N <= 128, and the GEMM form
                             for n_occ > 128 */
} rps_info;

/*
 * One-time set-up per geometry (Sec. 3.1, 3.2, 4.1, 4.3):
 *   basis values Phi on the grid; interpolation points (points_in, or the
 *   randomized selection of Sec. 4.3 with sketch matrices drawn from
 *   Philox4x32-10 with the given seed); fitting metric X_gg = (Phi_g Phi_g^T)^2
 *   and its FP64 Cholesky factor (retried once with the diagonal shift
 *   1e-13 * max diag(X_gg) if the plain factorisation fails); chi = X_gg^-1
 *   X_gR (Eq. 11); V[g,:] = Vc(chi_g) by FFT; W = V chi^T, symmetrised.
 * cell, basis       : host structures (see above)
 * n_aux             : number of interpolation points, 1 <= n_aux <= N_g.
 *                     n_aux == N_g selects chi = identity (the exact case).
 * seed              : 64-bit seed of the sketch matrices (ignored with points_in)
 * select_mode       : rps_select_mode (ignored with points_in)
 * precision         : rps_precision of later builds
 * points_in         : NULL, or host array of n_aux distinct grid indices
 * hip_stream        : hipStream_t to run on (NULL = default stream); the call
 *                     is synchronous with respect to the host
 * out               : receives the new context (unchanged on failure)
 * Errors: RPS_ERR_ARG, RPS_ERR_SHAPE, RPS_ERR_NOMEM (before allocating),
 *         RPS_ERR_NOT_PD, RPS_ERR_DEVICE.
 */
rps_status rps_setup_isdf(const rps_cell *cell, const rps_basis *basis, int64_t n_aux,
                          uint64_t seed, int32_t select_mode, int32_t precision,
                          const int64_t *points_in, void *hip_stream, rps_context **out);

/*
 * rps_setup_isdf with the screened basis of Sec. 4.1: every basis value whose
 * pSinc coefficient sqrt(dV) |phi_mu(R)| is below basis_eps (the paper's
 * eps1, 1e-8 there) is dropped before anything reads the basis, so the set-up
 * (points, chi, V, W) and every build use the screened values.  Each atom I
 * then holds one dense block: the grid points of its Voronoi set times the
 * basis functions not all zero there.  The general-size build (N > 128, or n
 * above the fused kernels' limit) forms U = Phi C and K1 = Phi^T M1^T from
 * these blocks, and rps_build_coulomb forms the density and J from them
 * (bases with N > 128 or n > 64); the fused kernels for small bases read the
 * screened values in dense form.  Sums over the atoms holding a function run
 * in a fixed order, so results are deterministic.  basis_eps = 0 is exactly
 * rps_setup_isdf.  rps_info.basis_fill reports the fraction of values held.
 * Errors: as rps_setup_isdf; RPS_ERR_ARG for a negative or non-finite basis_eps.
 */
rps_status rps_setup_isdf_screened(const rps_cell *cell, const rps_basis *basis, int64_t n_aux,
                                   uint64_t seed, int32_t select_mode, int32_t precision,
                                   const int64_t *points_in, double basis_eps, void *hip_stream,
                                   rps_context **out);

/*
 * Set-up from potentials computed elsewhere: the basis on the grid (Sec. 2.1.3)
 * and Phi_g as in rps_setup_isdf, but the interpolation points, the potentials V
 * of the fitting functions (Eq. 12) and W (Eq. 14) are the caller's; no point
 * selection, fit or FFT runs.  For reusing set-up products across processes or
 * codes (save them with rps_get_points and rps_get_array), and for timing builds
 * apart from the fit.
 * points   : host array of n_aux distinct grid indices (required)
 * precision: rps_precision of later builds; it also fixes V's element type
 * V        : [n_aux][ldv] row-major, ldv >= N_g: FP64 for RPS_PREC_FP64, FP32
 *            (the stored form) for RPS_PREC_FP32 and RPS_PREC_BF16X3
 * W        : [n_aux][ldw] FP64, ldw >= n_aux, symmetric
 * flags    : RPS_PTRS_HOST or RPS_PTRS_DEVICE (V and W); the call is synchronous
 * n_aux == N_g (the exact case) is refused: use rps_setup_isdf.
 * Errors: RPS_ERR_ARG, RPS_ERR_SHAPE, RPS_ERR_NOMEM (before allocating), RPS_ERR_DEVICE.
 */
rps_status rps_setup_isdf_from_potentials(const rps_cell *cell, const rps_basis *basis, int64_t n_aux,
                                          const int64_t *points, int32_t precision, const void *V, int64_t ldv,
                                          const double *W, int64_t ldw, int32_t flags, void *hip_stream,
                                          rps_context **out);

/*
 * One exchange build, Eq. 16 (Sec. 3.3) with the contraction order of
 * Sec. 4.4 for the second line:
 *   U = Phi C, U_g = U[points], P = U_g U^T, A = V o P, P_g = U_g U_g^T,
 *   B = W o P_g,  K_occ = dV [Phi^T (A^T U_g) + Phi_g^T (A U) - Phi_g^T (B U_g)],
 *   E_x = -dV (2 sum A o P - sum B o P_g).
 * nocc  : number of occupied orbitals n >= 1
 * C     : [N][nocc] FP64 coefficients (host or device, see flags)
 * K     : [N][nocc] FP64 output K_occ (host or device)
 * ex    : FP64 output E_x, or NULL
 * flags : RPS_PTRS_HOST or RPS_PTRS_DEVICE
 * hip_stream : stream for device-pointer mode (NULL = default stream)
 * Errors: RPS_ERR_ARG, RPS_ERR_STATE, RPS_ERR_NOMEM, RPS_ERR_DEVICE.
 */
rps_status rps_build_exchange_occRI(rps_context *ctx, int32_t nocc, const double *C, double *K,
                                    double *ex, int32_t flags, void *hip_stream);

/*
 * rps_build_exchange_occRI for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The call allocates nothing.  The build's workspace (orbitals at
 * the points, the ordered partial sums of lines 1-3, the energy partials and
 * counter) comes from a static device array of 64 MiB that the library holds
 * on every device it runs on until the process ends; the caller passes only
 * C, K and ex, all device pointers (stream-ordered on hip_stream, asynchronous).
 * Results equal rps_build_exchange_occRI's on the same context.
 * Limits: the fused path only (N <= 128 with n_occ <= 64 for FP64 contexts,
 * n_occ <= 16 for the precision forms; about 38 MiB at most for the 8-atom
 * 48^3 cell) and at most 64 MiB of workspace; anything else returns
 * RPS_ERR_SHAPE before any launch.  All calls on one device share the array:
 * calls that overlap on one device (two streams, two host threads) race and
 * give wrong results; order them on one stream.
 * Errors: RPS_ERR_ARG, RPS_ERR_STATE, RPS_ERR_SHAPE, RPS_ERR_DEVICE.
 */
rps_status rps_build_exchange_occRI_noalloc(rps_context *ctx, int32_t nocc, const double *C, double *K,
                                            double *ex, void *hip_stream);

/*
 * Same as rps_build_exchange_occRI for the PS and THC approximations
 * (variant = rps_variant; Sec. 3.2: PS keeps the first line of Eq. 13, THC the
 * third).  RPS_VARIANT_RPS gives exactly rps_build_exchange_occRI.
 */
rps_status rps_build_exchange_variant(rps_context *ctx, int32_t variant, int32_t nocc,
                                      const double *C, double *K, double *ex, int32_t flags,
                                      void *hip_stream);

/*
 * Full exchange matrix K_{mu nu} = sum_i (mu i | i nu) with rPS integrals
 * (Eq. 15 and its two partner terms of Eq. 13):
 *   K = dV [Phi_g^T A Phi + (Phi_g^T A Phi)^T - Phi_g^T B Phi_g],
 * A = V o (U_g U^T), B = W o (U_g U_g^T); K_full C equals K_occ.  Needed once
 * at the end of an SCF run (Sec. 3.3).  nocc, C as for
 * rps_build_exchange_occRI; K: [N][N] FP64 output (host or device per flags).
 * Works on any context (FP64 products; the precision form reads its FP32 V).
 * Allocates its temporaries for the call (about 2 GB plus 8 N_aux^2 bytes)
 * and synchronises hip_stream before returning.
 * Errors: RPS_ERR_ARG, RPS_ERR_STATE, RPS_ERR_NOMEM, RPS_ERR_DEVICE.
 */
rps_status rps_build_exchange_full(rps_context *ctx, int32_t nocc, const double *C, double *K,
                                   int32_t flags, void *hip_stream);

/*
 * Coulomb matrix on the same grid (Sec. 2.3, "Coulomb matrix", steps 1-4, with
 * the density matrix D = C C^T of Sec. 2.3):
 *   rho(R) = sum_i u_i(R)^2 (u = Phi C), V_H = Vc rho (G = 0 removed),
 *   J_{mu nu} = dV sum_R phi_mu(R) phi_nu(R) V_H(R),
 *   ej = dV sum_R rho(R) V_H(R) = sum_ij (ii|jj) = tr(D J).
 * With doubly occupied spatial orbitals the closed-shell two-electron energy
 * is 2 ej + ex (ex from rps_build_exchange_occRI).  Every step runs in FP64 on
 * any context (the precision option applies to exchange only); Phi is dense,
 * so the cost is 2 N_g N n + N_g N^2 multiply-adds.
 * nocc, C : as for rps_build_exchange_occRI
 * J       : [N][N] FP64 output, symmetric (host or device per flags)
 * ej      : FP64 output E_J, or NULL (host or device per flags)
 * Device-pointer calls are asynchronous on hip_stream; host-pointer calls
 * synchronise it.  Workspace (about 256 MB plus 24 N_g bytes and the split
 * partials of J) is allocated on the first call and kept by the context.
 * Errors: RPS_ERR_ARG, RPS_ERR_STATE, RPS_ERR_NOMEM, RPS_ERR_DEVICE.
 */
rps_status rps_build_coulomb(rps_context *ctx, int32_t nocc, const double *C, double *J, double *ej,
                             int32_t flags, void *hip_stream);

/*
 * Madelung constant of a lattice (Sec. 4.5: the exchange drops G = 0 and adds
 * nM/2 back for n electrons).  M is minus the potential at a lattice site of
 * unit point charges on all sites with a uniform neutralising background, the
 * site's own 1/r removed, by Ewald's splitting (M L = 2.8372975 for a simple
 * cubic cell of side L).  lattice: rows a1, a2, a3 in bohr.  Host only.
 * Errors: RPS_ERR_ARG (NULL or degenerate lattice).
 */
rps_status rps_madelung_constant(const double lattice[9], double *M);

/*
 * Madelung term of an exchange build (Sec. 4.5), applied in place to the
 * outputs of rps_build_exchange_occRI: K += M S C and, if ex is not NULL,
 * ex -= M tr(C^T S C), with S = dV Phi^T Phi the grid overlap (formed on the
 * first call and kept by the context, 8 N^2 bytes).  For S-orthonormal C the
 * energy shift is n_occ M = nM/2 (n = 2 n_occ electrons).
 * nocc, C, K, ex, flags, hip_stream as for rps_build_exchange_occRI.
 * Errors: RPS_ERR_ARG, RPS_ERR_STATE, RPS_ERR_NOMEM, RPS_ERR_DEVICE.
 */
rps_status rps_madelung_correct(rps_context *ctx, int32_t nocc, const double *C, double *K, double *ex,
                                int32_t flags, void *hip_stream);

/*
 * Batched builds over several contexts (cells of different sizes), one call,
 * issued one after another on hip_stream: C[b], K[b] as for
 * rps_build_exchange_occRI, ex[b] per cell (ex may be NULL).  All pointers are
 * of the kind given by flags.  The graph-captured form is rps_batch_create.
 */
rps_status rps_build_exchange_occRI_batched(rps_context *const *ctx, int32_t nbatch,
                                            const int32_t *nocc, const double *const *C,
                                            double *const *K, double *ex, int32_t flags,
                                            void *hip_stream);

/*
 * Autotuner.  Times the launch parameters that matter for this context's
 * build path on the given device-pointer inputs (the work-group target of the
 * streaming passes, or the R tiles per work-group and g blocks of the fused
 * kernel), keeps the fastest in the context for every later build, and writes
 * its mean build time in ms to best_ms (may be NULL).  Results of later builds
 * stay deterministic; they may differ from untuned builds in the last bits
 * (another summation order).  C, K: device [N][nocc]; ex device or NULL.
 * The call synchronises hip_stream.
 * Errors: RPS_ERR_ARG, RPS_ERR_STATE, RPS_ERR_NOMEM, RPS_ERR_DEVICE.
 */
rps_status rps_autotune(rps_context *ctx, int32_t nocc, const double *C, double *K, double *ex,
                        void *hip_stream, double *best_ms);

/*
 * Batching form: the builds of many independent cells (contexts of any sizes)
 * captured once into one HIP graph and replayed with one launch.  Cells are
 * ordered by work (n N_aux N_g, largest first) and dealt to parallel graph
 * branches by least accumulated work.  rps_batch_create takes device pointers
 * only (C[b], K[b] as for rps_build_exchange_occRI; ex: device array [nbatch]
 * or NULL); they are baked into the graph, so every rps_batch_run reads the
 * current contents of C[b] and overwrites K[b] and ex[b].  flags:
 *   RPS_BATCH_AUTOTUNE     run rps_autotune on every context first;
 *   RPS_BATCH_BRANCHES(k)  use k parallel branches (1..15) instead of timing
 *                          1, 2 and 4 and keeping the fastest.
 * A context may appear once per batch and must not be used by other builds
 * while a replay of the batch runs (the builds share its workspace).
 * The graph holds the addresses of each context's build workspace: after
 * rps_autotune on one of its contexts, or a build there with another number of
 * occupied orbitals (either may reallocate that workspace), rps_batch_run
 * returns RPS_ERR_STATE without launching; destroy and recreate the batch.
 * Destroy the batch before any of its contexts.
 * rps_batch_info: nbranch, and seconds[3] = {create (tuning + capture),
 * last capture, mean replay measured at creation}.
 * Errors: RPS_ERR_ARG, RPS_ERR_STATE, RPS_ERR_NOMEM, RPS_ERR_DEVICE.
 */
typedef struct rps_batch rps_batch;
#define RPS_BATCH_AUTOTUNE 1
#define RPS_BATCH_FIXED_BRANCHES_MASK 0xF00
#define RPS_BATCH_BRANCHES(k) (((k) & 15) << 8)
rps_status rps_batch_create(rps_context *const *ctx, int32_t nbatch, const int32_t *nocc,
                            const double *const *C, double *const *K, double *ex, int32_t flags,
                            void *hip_stream, rps_batch **out);
rps_status rps_batch_run(rps_batch *batch, void *hip_stream);
rps_status rps_batch_info(const rps_batch *batch, int32_t *nbranch, double *seconds);
void rps_batch_destroy(rps_batch *batch);

/* E_x = -tr(C^T K) = -sum_{mu,i} C[mu][i] K[mu][i]; host FP64 arrays [nbas][nocc]. */
rps_status rps_exchange_energy(int32_t nbas, int32_t nocc, const double *C, const double *K,
                               double *ex);

/* Grid overlap S = dV Phi^T Phi, host output [N][N] (for orthonormalising C). */
rps_status rps_overlap(rps_context *ctx, double *S);

/* Interpolation point indices in selection order, host output [n_aux]. */
rps_status rps_get_points(const rps_context *ctx, int64_t *points_out);

/* Sizes and diagnostics. */
rps_status rps_get_info(const rps_context *ctx, rps_info *info);

/*
 * Copies of set-up products to host memory (inspection and tests).
 * which: 0 = Phi rows [row0, row0+nrows) x N;   1 = V rows x N_g;
 *        2 = W rows x N_chi;  3 = Voronoi owner of grid points row0.. (as double).
 */
rps_status rps_get_array(const rps_context *ctx, int32_t which, int64_t row0, int64_t nrows,
                         double *out);

/*
 * Kernel timing for measurement.  With enable = 1 every later build records
 * HIP events on its stream around the V-streaming kernel(s) (Eq. 16, lines 1-2;
 * in the GEMM form of n_occ > 128, the chunk products A_c = V o P, M1^T and M2
 * with their split-K reductions), around the fit-fit kernel (line 3) and
 * around the whole build.
 * rps_get_profile synchronises the stream of the last build, writes
 *   out[0] = builds timed, out[1] = total ms in the V-streaming kernel,
 *   out[2] = total ms in the fit-fit kernel, out[3] = total ms of whole builds,
 * and clears the record.  At most 65536 builds are recorded between reads.
 */
rps_status rps_set_profiling(rps_context *ctx, int32_t enable);
rps_status rps_get_profile(rps_context *ctx, double *out);

/* Frees every device buffer of the context.  NULL is allowed. */
void rps_destroy(rps_context *ctx);

/* Message of the last failure on the calling thread ("" if none). */
const char *rps_last_error(void);

/* ABI version (1). */
int32_t rps_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RPS_H */
