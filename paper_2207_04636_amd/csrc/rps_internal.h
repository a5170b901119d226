// Internal launchers of the rPS exchange library (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rps {

// ---------------------------------------------------------------- GEMM
// C[M x N] = epilogue(alpha * op(A)[M x K] op(B)[K x N], beta, C)
//   op(A)[m][k] = transA ? A[k*lda + m] : A[m*lda + k]
//   op(B)[k][n] = transB ? B[n*ldb + k] : B[k*ldb + n]
enum GemmEpi {
  EPI_AXPBY = 0,     // C = alpha*AB + beta*C
  EPI_SQUARE = 1,    // C = (alpha*AB)^2 (elementwise)
  EPI_HADAMARD = 2,  // C = C o (alpha*AB)
  EPI_HADAMARD_SRC = 3   // C = D o (alpha*AB), D a separate matrix (ldd)
};
struct Gemm {
  int64_t M = 0, N = 0, K = 0;
  const double* A = nullptr; int64_t lda = 0; bool transA = false;
  const double* B = nullptr; int64_t ldb = 0; bool transB = false;
  double* C = nullptr; int64_t ldc = 0;
  double alpha = 1.0, beta = 0.0;
  int epi = EPI_AXPBY;
  bool lower_only = false;   // skip output tiles strictly above the diagonal
  const double* D = nullptr; int64_t ldd = 0;   // EPI_HADAMARD_SRC operand
  const float* D32 = nullptr;                    // FP32 form of that operand (used when D is NULL)
  int splitk = 1;            // > 1: K split over workgroups, partials in work (EPI_AXPBY only)
  double* work = nullptr;    // splitk * M * N doubles
  bool keep_partials = false;          // splitk > 1: leave the partials in work, no reduction
  const double* kscale = nullptr;      // op(B)[k][n] *= kscale[k] (transA && !transB, or N <= 16)
  int tile_n = 0;                      // output tile width 64 or 128 (0: chosen from N)
  float* Cf = nullptr; int64_t ldcf = 0;   // also the final C rounded to FP32 here (EPI_AXPBY only)
};
hipError_t gemm_f64(const Gemm& g, hipStream_t s);
// Split count and tile width of an AXPBY product together: the pair whose workgroups fill
// their last round (two per CU) best, weighted by the share of the tile columns that
// are not padding; splits keep >= 256 of K and fit work_cap doubles.
void gemm_plan(Gemm& g, int64_t work_cap_doubles);
// One launch of many independent products: item i computes C_i = alpha op(A_i) op(B_i)
// + beta C_i with A_i = base.A + aofs etc. (its own sizes and pitches), and with
// base.kscale + kofs as the row scale when base.kscale is set (transA only).  Items
// live in device memory; maxM / maxN bound their sizes.  No K split; EPI_AXPBY only.
struct GemmItem {
  int64_t M, N, K, lda, ldb, ldc, aofs, bofs, cofs, kofs;
};
hipError_t gemm_f64_grouped(const Gemm& base, const GemmItem* items, int nitems, int64_t maxM, int64_t maxN,
                            hipStream_t s);
// Split count giving enough workgroups for a long-K product within work_cap doubles.
int gemm_splitk_for(int64_t M, int64_t N, int64_t K, int64_t work_cap_doubles);

// FP32 operands on the FP32 matrix cores:
//   C32 != NULL: C32[M x N] (ldc) = D32 o (alpha * op(A) op(B)), FP32 sums (no split)
//   else:        C[M x N] (ldc, FP64) = alpha * op(A) op(B) + beta * C; FP32 sums over
//                64 terms of K at a time, FP64 beyond, the K splits summed in FP64 in a
//                fixed order (partials in work, splitk * M * N)
struct Gemm32 {
  int64_t M = 0, N = 0, K = 0;
  const float* A = nullptr; int64_t lda = 0; bool transA = false;
  const float* B = nullptr; int64_t ldb = 0; bool transB = false;
  double* C = nullptr; int64_t ldc = 0;
  double alpha = 1.0, beta = 0.0;
  float* C32 = nullptr;
  const float* D32 = nullptr; int64_t ldd = 0;
  int splitk = 1;
  double* work = nullptr;
  // B holds Nread >= N columns (zero beyond N) that may be read: tiles reaching
  // past N but not past Nread load B whole; outputs stay within N (0: Nread = N)
  int64_t Nread = 0;
  float* Cf = nullptr; int64_t ldcf = 0;   // FP64 output: also the final C rounded to FP32 here
};
hipError_t gemm_f32(const Gemm32& g, hipStream_t s);
// Split count with at most kmax of K per split and enough workgroups, within work_cap doubles
// (a split count whose K range exceeds kmax is returned when the workspace allows no more).
int gemm32_splitk_for(int64_t M, int64_t N, int64_t K, int64_t kmax, int64_t work_cap_doubles);

// ---------------------------------------------------------------- screened basis (k_sparse.hip)
// Phi[i] = 0 where |Phi[i]| < thr (i < count)
hipError_t screen_basis(double* Phi, int64_t count, double thr, hipStream_t s);
// flags[owner[R] * N + mu] = 1 where Phi[R][mu] != 0 (flags zeroed by the caller)
hipError_t basis_flags(const double* Phi, int64_t ng, int Np, int N, const int32_t* owner, int32_t* flags,
                       hipStream_t s);
// dst[r][c] = Phi[rows[r]][cols[c]] (dst row-major, pitch nc)
hipError_t pack_block(const double* Phi, int Np, const int64_t* rows, int64_t nr, const int64_t* cols, int nc,
                      double* dst, hipStream_t s);
// out[mu][i] = sum_{e in [ofs[mu], ofs[mu+1])} part[rows[e]][i], in order (mu < N; rows N..Np-1 zero)
hipError_t csr_rowsum(const double* part, int np, const int64_t* ofs, const int64_t* rows, int N, int Np,
                      double* out, hipStream_t s);
// J[mu][nu] = J[nu][mu] = scale * sum_{e in ofs[mu]..} Q_atom[e][pos(mu)][pos(nu)] (lower triangles read)
hipError_t j_reduce(const double* Q, const int64_t* qofs, const int64_t* fofs, const int32_t* pos,
                    const int64_t* ofs, const int32_t* atom, int N, double scale, double* J, hipStream_t s);

// ---------------------------------------------------------------- basis / grid
struct ShellDev {        // one Gaussian shell, device copy
  double cx, cy, cz;     // centre wrapped into the cell
  double expo;
  int l;                 // 0, 1, 2
  int fofs;              // first basis-function column
  int m0, m1, m2;        // image range along a1, a2, a3
};
struct CellDev {
  double a[9];           // rows a1, a2, a3
  double ainv[9];        // inverse of the row matrix (cartesian -> fractional)
  int mesh[3];
};
// Phi[R][mu] for R in [0, ngrid), rows >= ngrid up to nrows_pad left as is.
hipError_t basis_eval(const CellDev& cell, const ShellDev* shells, int nshell, int64_t ngrid,
                      double* Phi, int64_t ldphi, hipStream_t s);
// owner[R] = nearest atom over periodic images (ties -> lower index).
hipError_t voronoi_assign(const CellDev& cell, const double* atoms, int natom, int64_t ngrid,
                          int32_t* owner, hipStream_t s);
// dst[r][0:ncols] = src[idx[r]][0:ncols] for r < nidx, 0 for nidx <= r < nrows.
hipError_t gather_rows(const double* src, int64_t lds, const int64_t* idx, int64_t nidx,
                       int64_t nrows, int64_t ncols, double* dst, int64_t ldd, hipStream_t s);
// X[g][idx[g]] = 1 for g < n (fitting functions of the exact case, chi = identity)
hipError_t set_unit_rows(double* X, int64_t ld, const int64_t* idx, int64_t n, hipStream_t s);
// Y[r][c] = X[r][idx[c]] for r, c < n
hipError_t gather_cols(const double* X, int64_t ldx, const int64_t* idx, int64_t n, double* Y,
                       int64_t ldy, hipStream_t s);
hipError_t to_f32(const double* X, int64_t count, float* Y, hipStream_t s);
// Y[r][c] = X[r][c] for c < n, 0 for n <= c < ldy (X rows x n contiguous, Y pitch ldy >= n)
hipError_t to_f32_pad(const double* X, int64_t rows, int64_t n, float* Y, int64_t ldy, hipStream_t s);
// x[i*ld + i] += v for i in [i0, i1)
hipError_t add_diag(double* X, int64_t ld, int64_t i0, int64_t i1, double v, hipStream_t s);
hipError_t fill(double* X, int64_t count, double v, hipStream_t s);
// B = (A + A^T)/2 in place for an n x n matrix (ld)
hipError_t symmetrize(double* A, int64_t n, int64_t ld, hipStream_t s);
// A[i][j] = A[j][i] for i > j: the lower triangle copied from the upper
hipError_t mirror_upper(double* A, int64_t n, int64_t ld, hipStream_t s);
// out[j*ldo + i] = in[i*ldi + j] (i < rows, j < cols)
hipError_t transpose(const double* in, int64_t ldi, int64_t rows, int64_t cols, double* out,
                     int64_t ldo, hipStream_t s);

// ---------------------------------------------------------------- dense linear algebra
// Blocked right-looking lower Cholesky in place on an n x n matrix (n % 64 == 0).
// status[0] = 0 on success, 1 + (first failing row) otherwise.
hipError_t cholesky_lower(double* A, int64_t n, int64_t lda, int32_t* status, hipStream_t s);
// Solve L X = B (trans = false) or L^T X = B (trans = true) in place,
// L lower n x n (n % 64 == 0), B n x ncols with leading dimension ldb.
hipError_t tri_solve_lower(const double* L, int64_t n, int64_t ldl, double* B, int64_t ncols,
                           int64_t ldb, bool trans, hipStream_t s);
// Blocked pivoted Cholesky on an explicit symmetric Gram matrix G (n x n, ld),
// destroyed.  Writes the first k pivots (indices into 0..n-1, argmax of the
// updated diagonal, ties to the lowest index) to piv (device int64[k]).
// Work buffers: Lbuf (n x k doubles), diag (n + k doubles).
hipError_t pivoted_cholesky(double* G, int64_t n, int64_t ld, int64_t k, int64_t* piv,
                            double* Lbuf, double* diag, hipStream_t s);

// ---------------------------------------------------------------- Poisson solve
// In place V <- Vc V for nrows real rows (split-complex pairs of rows, nrows even)
// of the grid mesh, leading dimension ld.  kern[N_g]: k(G) / N_g in FFT order.
hipError_t poisson_rows(double* V, int64_t nrows, int64_t ld, const int mesh[3],
                        const double* kern, hipStream_t s);

// ---------------------------------------------------------------- Coulomb matrix
// For r < rows: out[r] = out[2 ld + r] = sum_{i < np} U[r][i]^2 (U pitch np, np even)
// and out[ld + r] = 0, i.e. the density as the real row of a Poisson pair plus a copy.
hipError_t density_rows(const double* U, int64_t rows, int np, double* out, int64_t ld, hipStream_t s);
// *out = scale * sum_{p < n} x[p] y[p], summed in a fixed order over nparts blocks
// (part: nparts doubles of workspace).
hipError_t dot_scaled(const double* x, const double* y, int64_t n, double scale, double* part, int nparts,
                      double* out, hipStream_t s);
// J[i][j] = scale * sum_{z < nz} work[z][max(i,j)][min(i,j)] for i, j < N (work [nz][Np][Np],
// lower triangle valid).
hipError_t sym_from_lower(const double* work, int nz, int64_t Np, int64_t N, double scale, double* J,
                          hipStream_t s);

// Small-basis Coulomb path (Np <= 128): rho of rows [0, rows) of Phi [rows][Np] with
// U = Phi C (np <= 64) written as density_rows does; and the lower 16 x 16 tiles of the
// partials part[b][Np][Np] = sum over workgroup b's 64-row chunks of v[R] phi[R] phi[R]^T
// (rows % 64 == 0; coulomb_small_blocks(rows) partials).
hipError_t density_small(const double* Phi, int64_t rows, int Np, const double* C, int N, int n, int np,
                         double* out, int64_t ld, hipStream_t s);
int coulomb_small_blocks(int64_t rows);
hipError_t coulomb_small(const double* Phi, int64_t rows, int Np, const double* v, double* part, hipStream_t s);

// Madelung term: K[mu][i] += M SC[mu][i] (K, C: [N][n]; SC pitch ldsc) and, if ex,
// *ex -= M sum C o SC, summed over nparts (<= 256) blocks in a fixed order (part: workspace).
hipError_t madelung_apply(const double* SC, int64_t ldsc, const double* C, int64_t N, int64_t n, double M,
                          double* K, double* ex, double* part, int nparts, hipStream_t s);

// ---------------------------------------------------------------- exchange build
struct FusedArgs {
  // A = Vm o (Ug Ur^T); Vm: [G x R] row pitch ldv
  const double* Vm; int64_t ldv;
  const float* Vm32;        // FP32 copy (precision forms), ldv pitch
  const double* Ug;         // [Gp x np]  (row operand)
  const double* Ugp;        // permuted copy [Gp][i % 4][i / 4] (np == 16 only), or NULL
  int use_m4;               // use the 4x4x4 FP64 MFMA form (np == 16)
  const double* Ur;         // [Rp x np]  (column operand)
  const double* Phir;       // [Rp x Np]  basis at the columns (for K1)
  int64_t G, R;             // padded extents (multiples of 64)
  int64_t R_valid;          // columns beyond it are zero
  int np;                   // padded n (multiple of 16)
  int Np;                   // padded N (multiple of 16)
  int rtiles;               // 64-column tiles per workgroup
  int gblocks;              // workgroups along G
  int nwaves;               // waves per workgroup (4 or 8)
  int want_m2;              // write M2 partials
  int want_k1;              // accumulate K1 partials (Phir^T (A^T Ug))
  int want_m1;              // write M1^T = A^T Ug rows (when K1 is not fused)
  int want_e;               // accumulate sum A o P into e1p (else the caller forms it from M2)
  int prec;                 // rps_precision
  // precision form with the orbitals of each R tile formed in the kernel (NULL Phi32: U from Ur)
  const float* Phi32;       // [Rp x Np] FP32 basis values
  const double* Cm;         // [N x n] occupied coefficients (row pitch n)
  int N, n;
  // fit-fit line folded into that kernel (Wl NULL: not computed).  Unit (g subtile ys,
  // h subtile hc) of Y = (Wl o (U_g U_g^T)) U_g is written NEGATED as rows ys of partial
  // hc of Yneg ([G/16][G][np]; placed after the M2 partials, so that their ordered sum
  // is M2 - Y), and sum U_g o Y over the unit goes to e3u[ys * (G/16) + hc].
  const double* Wl; int64_t ldw;   // W [G x G] FP64, row pitch ldw (symmetric)
  double* Yneg;
  double* e3u;
  // outputs
  double* M2p;              // [rblocks][G][np]
  double* K1p;              // [gblocks*rblocks][Np][np]
  double* M1T;              // [gblocks][R][np]
  double* e1p;              // [gblocks*rblocks]
};
int fused_rblocks(const FusedArgs& a);
// g subtiles per wave of the in-kernel-orbitals precision kernel (Phi32 set; at most 8)
// and its LDS bytes (at most 160 KiB).
int64_t fused_f32u_nmy(const FusedArgs& a);
int64_t fused_f32u_lds(const FusedArgs& a);
int64_t fused_lds_bytes(const FusedArgs& a);
hipError_t fused_exchange(const FusedArgs& a, hipStream_t s);
// U [R x np] = Phi [R x Np] C and U_g [G x np] = Phi_g [G x Np] C, with C [N x n]
// (row pitch n) zero padded to [Np x np] (R, G % 16 == 0, np <= 64, Np <= 128).
// Ugp (may be NULL; np == 16 only): permuted copy [g][i % 4][i / 4] of U_g.
hipError_t orbitals(const double* Phi, int64_t R, const double* Phig, int64_t G, int Np, const double* C,
                    int N, int n, int np, double* U, double* Ug, double* Ugp, hipStream_t s);
// Cp [rows_p x ldp] = C [rows x cols] zero padded.
hipError_t pack_matrix(const double* C, int64_t rows, int64_t cols, int64_t ldc, double* Cp, int64_t rows_p,
                       int64_t ldp, hipStream_t s);
// Up to three partial sums in one launch: out_k[i] = sum_p in_k[p*count_k + i]
// (fixed order); a segment with a NULL input is skipped.
hipError_t sum_partials3(const double* in0, int64_t n0, int64_t c0, double* o0, const double* in1, int64_t n1,
                         int64_t c1, double* o1, const double* in2, int64_t n2, int64_t c2, double* o2,
                         hipStream_t s);
// Energy terms given as dot products: e1 += x1 . y1 (n1 terms), e3 += x3 . y3.
// Long dots are split over several blocks whose partials go to part[nparts]
// (summed in order by a second kernel); NULL part keeps one block.
struct EnergyDots {
  const double* x1 = nullptr; const double* y1 = nullptr; int64_t n1 = 0;
  const double* x3 = nullptr; const double* y3 = nullptr; int64_t n3 = 0;
  double* part = nullptr; int nparts = 0;
  // with part: a device counter, zero between builds, by which the last energy block
  // sums the partials itself (NULL: a second kernel does)
  unsigned* count = nullptr;
};
// K[mu][i] = dV (s1 K1 + s2 Phi_g^T M2 + s3 K3) for mu < N, i < n ([Np][np] arrays,
// any may be NULL); ex = -dV (ce1 e1 + ce3 e3) if ex is not NULL, with
// e1 = sum e1p + x1 . y1 and e3 = sum e3p + x3 . y3 (fixed summation order).
hipError_t finalize(const double* Phig, const double* M2, int64_t G, const double* K1, const double* K3, int N,
                    int n, int np, int Np, double s1, double s2, double s3, double dV, double* K, const double* e1p,
                    int64_t ne1, const double* e3p, int64_t ne3, double ce1, double ce3, double* ex, hipStream_t s,
                    const EnergyDots& dots = EnergyDots());

// Full exchange matrix: K[i][j] = dV (T[i][j] + T[j][i] - K3[i][j]) for i, j < N
// from [Np][Np] arrays T = Phi_g^T (A Phi) and K3 = Phi_g^T (B Phi_g).
hipError_t full_combine(const double* T, const double* K3, int64_t Np, int64_t N, double dV, double* K,
                        hipStream_t s);

// ---------------------------------------------------------------- streaming form (general sizes)
// O[x][c] = sum_y S[x][y] (sum_d X[x][d] Y[y][d]) Y[y][c], S = V (or W) stored
// row-major [rows][cols] with pitch ldv; trans = 0: x indexes rows of S,
// trans = 1: x indexes columns.  X [nx][ldx], Y [ny][np] (ldy == np), np a
// multiple of 16 up to 128, nx % 16 == 0, ny % 32 == 0.  The y range is split
// over nsplit workgroup columns; out holds nsplit partials [nsplit][nx][np].
struct StreamArgs {
  const double* V = nullptr;
  const float* V32 = nullptr;
  int64_t ldv = 0;
  int trans = 0;
  const double* X = nullptr; int64_t ldx = 0;
  const double* Y = nullptr; int64_t ldy = 0;
  const float* Y32 = nullptr;  // FP32 copy of Y (same pitch), read by the FP32 and split-BF16 forms
  int64_t nx = 0, ny = 0;
  int64_t ysplit = 0;       // set by stream_product
  int np = 0;
  double* out = nullptr;
};
// Split count along y giving about target_blocks workgroups.
int stream_splits(int64_t nx, int64_t ny, int target_blocks);
// prec: 0 FP64 (V), 1 FP32 (V32, FP32 products), 2 split-BF16 products on V32.
hipError_t stream_product(const StreamArgs& a, int prec, int nsplit, hipStream_t s);

// Persistent form of the passes for the batching form.  A work item is one
// workgroup's share of one cell's pass: x block bx (128 rows) and y split by.
struct StreamItem {
  int32_t cell, bx, by;
};
// Checks a pass as stream_product does and returns it with its split length set.
hipError_t stream_prepare(const StreamArgs& a, int prec, int nsplit, StreamArgs& out);
// x blocks of a pass with nx rows.
int64_t stream_xblocks(int64_t nx);
// Workgroups that stay resident for the passes of class (prec, np, trans).
int stream_queue_blocks(int prec, int np, int trans);
// One launch over items[0..nitems) (device arrays) of cells whose passes share
// prec, np and trans; args[cell] as returned by stream_prepare; *counter (device)
// must be zero at launch and is left at nitems + the number of workgroups.
hipError_t stream_product_queue(const StreamArgs* args, const StreamItem* items, int nitems, int prec, int np,
                                int trans, unsigned* counter, int nblocks, hipStream_t s);

}  // namespace rps
