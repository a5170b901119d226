// Dense FP64 linear algebra of the ISDF set-up.
//
// * Cholesky factorisation of the fitting metric X_gg (Sec. 4.3 solves the
//   least-squares fit of Sec. 3.1, Eq. 11, with a Cholesky factorisation):
//   blocked right-looking, 64-column panels factored in LDS, the block column
//   below by substitution, the trailing matrix by the FP64 MFMA product.
// * Triangular solves with many right-hand sides (the N_g columns of X_gR, or
//   the N_chi columns when forming W): 64-row diagonal blocks by substitution,
//   one thread per right-hand side, the rest by matrix products.
// * Pivoted Cholesky of an explicit Gram matrix.  QR with column pivoting of a
//   matrix M (Sec. 3.1, 4.3) picks as pivot k the column whose norm, after
//   projecting out the columns picked before, is largest.  That residual norm
//   squared is the updated diagonal of a Cholesky factorisation of M^T M with
//   the same pivot order, so the pivots are those of QRCP in exact arithmetic.
//   Panels of 32 steps; the Gram matrix is updated after each panel.
#include <math.h>

#include "mfma.h"
#include "rps_internal.h"

namespace rps {
namespace {

constexpr int NB = 64;

__global__ __launch_bounds__(256) void chol_panel_kernel(double* A, int64_t lda, int64_t k0, int32_t* status) {
  __shared__ double L[NB][NB + 1];
  __shared__ double piv;
  const int tid = threadIdx.x;
  for (int e = tid; e < NB * NB; e += 256) {
    const int i = e / NB, j = e % NB;
    L[i][j] = (j <= i) ? A[(k0 + i) * lda + k0 + j] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < NB; ++j) {
    if (tid == 0) {
      double d = L[j][j];
      if (!(d > 0.0)) {
        if (status[0] == 0) status[0] = (int32_t)(1 + k0 + j);
        d = 1.0;
      }
      piv = sqrt(d);
      L[j][j] = piv;
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < NB; i += 256) L[i][j] /= piv;
    __syncthreads();
    for (int e = tid; e < NB * NB; e += 256) {
      const int i = e / NB, k = e % NB;
      if (i > j && k > j && k <= i) L[i][k] -= L[i][j] * L[k][j];
    }
    __syncthreads();
  }
  for (int e = tid; e < NB * NB; e += 256) {
    const int i = e / NB, j = e % NB;
    if (j <= i) A[(k0 + i) * lda + k0 + j] = L[i][j];
  }
}

// Solve a 64-vector v against the 64x64 lower triangle Ls (in LDS):
// TRANS = false: L x = v (forward), TRANS = true: L^T x = v (backward).
// Vector v number t has component j at base[t*sv + j*sj].
template <bool TRANS>
__global__ __launch_bounds__(256) void tri64_kernel(const double* __restrict__ Lg, int64_t ldl, double* base,
                                                   int64_t sv, int64_t sj, int64_t nvec) {
  __shared__ double Ls[NB][NB + 1];
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int i = e / NB, j = e % NB;
    Ls[i][j] = (j <= i) ? Lg[i * ldl + j] : 0.0;
  }
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= nvec) return;
  double* v = base + t * sv;
  double x[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) x[j] = v[j * sj];
  if (!TRANS) {
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      double s = x[i];
#pragma unroll
      for (int k = 0; k < i; ++k) s -= Ls[i][k] * x[k];
      x[i] = s / Ls[i][i];
    }
  } else {
#pragma unroll
    for (int i = NB - 1; i >= 0; --i) {
      double s = x[i];
#pragma unroll
      for (int k = i + 1; k < NB; ++k) s -= Ls[k][i] * x[k];
      x[i] = s / Ls[i][i];
    }
  }
#pragma unroll
  for (int j = 0; j < NB; ++j) v[j * sj] = x[j];
}

// ---------------- pivoted Cholesky
__global__ void diag_init_kernel(const double* G, int64_t n, int64_t ld, double* diag) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) diag[j] = G[j * ld + j];
}

__global__ __launch_bounds__(1024) void argmax_kernel(const double* __restrict__ diag, int64_t n,
                                                     int64_t* __restrict__ piv, double* __restrict__ dsel,
                                                     int64_t k) {
  __shared__ double sv[1024];
  __shared__ int64_t si[1024];
  double bv = -INFINITY;
  int64_t bi = n;
  for (int64_t j = threadIdx.x; j < n; j += 1024) {
    const double v = diag[j];
    if (v > bv) { bv = v; bi = j; }     // strided scan visits j in increasing order
  }
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      const double v2 = sv[threadIdx.x + off];
      const int64_t i2 = si[threadIdx.x + off];
      if (v2 > sv[threadIdx.x] || (v2 == sv[threadIdx.x] && i2 < si[threadIdx.x])) {
        sv[threadIdx.x] = v2;
        si[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t p = (si[0] < n) ? si[0] : 0;
    piv[k] = p;
    dsel[k] = (si[0] < n) ? sv[0] : 0.0;
  }
}

// Column k of the factor: L[j][k] = (G[p][j] - sum_{t=kb}^{k-1} L[j][t] L[p][t]) / sqrt(d_p)
__global__ __launch_bounds__(256) void pchol_column_kernel(const double* __restrict__ G, int64_t n, int64_t ld,
                                                          double* __restrict__ L, int64_t ldl, int64_t k,
                                                          int64_t kb, const int64_t* __restrict__ piv,
                                                          const double* __restrict__ dsel,
                                                          double* __restrict__ diag) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t p = piv[k];
  const double dp = dsel[k];                 // pivot value saved by the argmax step
  const double dj = diag[j];
  if (dj == -INFINITY && j != p) {           // already selected: its residual is zero
    L[j * ldl + k] = 0.0;
    return;
  }
  double s = G[p * ld + j];
  for (int64_t t = kb; t < k; ++t) s -= L[j * ldl + t] * L[p * ldl + t];
  double l = 0.0;
  if (dp > 0.0) l = s / sqrt(dp);
  L[j * ldl + k] = l;
  if (j == p) {
    diag[j] = -INFINITY;
  } else {
    diag[j] = dj - l * l;
  }
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t cholesky_lower(double* A, int64_t n, int64_t lda, int32_t* status, hipStream_t s) {
  hipError_t e = hipMemsetAsync(status, 0, sizeof(int32_t), s);
  if (e != hipSuccess) return e;
  for (int64_t k0 = 0; k0 < n; k0 += NB) {
    hipLaunchKernelGGL(chol_panel_kernel, dim3(1), dim3(256), 0, s, A, lda, k0, status);
    const int64_t rest = n - k0 - NB;
    if (rest <= 0) break;
    // A21 <- A21 L11^-T : each row x solves L11 x = a
    hipLaunchKernelGGL(tri64_kernel<false>, dim3(nblk(rest, 256)), dim3(256), 0, s,
                       A + k0 * lda + k0, lda, A + (k0 + NB) * lda + k0, lda, (int64_t)1, rest);
    Gemm g;
    g.M = rest; g.N = rest; g.K = NB;
    g.A = A + (k0 + NB) * lda + k0; g.lda = lda;
    g.B = A + (k0 + NB) * lda + k0; g.ldb = lda; g.transB = true;
    g.C = A + (k0 + NB) * lda + k0 + NB; g.ldc = lda;
    g.alpha = -1.0; g.beta = 1.0; g.lower_only = true;
    e = gemm_f64(g, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

// Two-level blocked solve.  Outer blocks of NB2 rows: the block is solved 64 rows
// at a time (the 64 x 64 triangle in LDS, one thread per right-hand side, and
// rank-64 updates confined to the block's rows), then the rest of B takes one
// rank-NB2 update.  The updates that sweep all of B are therefore NB2 deep, so B
// streams through HBM n / NB2 times instead of n / 64 times.
hipError_t tri_solve_lower(const double* L, int64_t n, int64_t ldl, double* B, int64_t ncols,
                           int64_t ldb, bool trans, hipStream_t s) {
  constexpr int64_t NB2 = 512;
  if (n % NB != 0) return hipErrorInvalidValue;
  const int64_t nout = (n + NB2 - 1) / NB2;
  auto update = [&](int64_t r0, int64_t r1, int64_t k0, int64_t kb) -> hipError_t {
    // rows [r0, r1) of B minus the contribution of the solved rows [k0, k0 + kb)
    if (r1 <= r0) return hipSuccess;
    Gemm g;
    g.M = r1 - r0; g.N = ncols; g.K = kb;
    g.B = B + k0 * ldb; g.ldb = ldb;
    g.C = B + r0 * ldb; g.ldc = ldb;
    g.alpha = -1.0; g.beta = 1.0;
    if (!trans) { g.A = L + r0 * ldl + k0; g.lda = ldl; }                     // L[r0:r1, k0:k0+kb]
    else { g.A = L + k0 * ldl + r0; g.lda = ldl; g.transA = true; }           // L[k0:k0+kb, r0:r1]^T
    return gemm_f64(g, s);
  };
  for (int64_t oq = 0; oq < nout; ++oq) {
    const int64_t ob = trans ? (nout - 1 - oq) : oq;
    const int64_t o0 = ob * NB2, o1 = (o0 + NB2 < n) ? o0 + NB2 : n;
    const int64_t nin = (o1 - o0) / NB;
    for (int64_t q = 0; q < nin; ++q) {
      const int64_t k0 = o0 + (trans ? (nin - 1 - q) : q) * NB;
      if (!trans)
        hipLaunchKernelGGL(tri64_kernel<false>, dim3(nblk(ncols, 256)), dim3(256), 0, s,
                           L + k0 * ldl + k0, ldl, B + k0 * ldb, (int64_t)1, ldb, ncols);
      else
        hipLaunchKernelGGL(tri64_kernel<true>, dim3(nblk(ncols, 256)), dim3(256), 0, s,
                           L + k0 * ldl + k0, ldl, B + k0 * ldb, (int64_t)1, ldb, ncols);
      const hipError_t e = trans ? update(o0, k0, k0, NB) : update(k0 + NB, o1, k0, NB);
      if (e != hipSuccess) return e;
    }
    const hipError_t e = trans ? update(0, o0, o0, o1 - o0) : update(o1, n, o0, o1 - o0);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t pivoted_cholesky(double* G, int64_t n, int64_t ld, int64_t k, int64_t* piv,
                            double* Lbuf, double* diag, hipStream_t s) {
  constexpr int64_t PB = 32;
  hipLaunchKernelGGL(diag_init_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, G, n, ld, diag);
  for (int64_t kb = 0; kb < k; kb += PB) {
    const int64_t ke = (kb + PB < k) ? kb + PB : k;
    for (int64_t kk = kb; kk < ke; ++kk) {
      hipLaunchKernelGGL(argmax_kernel, dim3(1), dim3(1024), 0, s, diag, n, piv, diag + n, kk);
      hipLaunchKernelGGL(pchol_column_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, G, n, ld, Lbuf, k,
                         kk, kb, piv, diag + n, diag);
    }
    if (ke < k) {   // G -= L[:, kb:ke] L[:, kb:ke]^T
      Gemm g;
      g.M = n; g.N = n; g.K = ke - kb;
      g.A = Lbuf + kb; g.lda = k;
      g.B = Lbuf + kb; g.ldb = k; g.transB = true;
      g.C = G; g.ldc = ld; g.alpha = -1.0; g.beta = 1.0;
      hipError_t e = gemm_f64(g, s);
      if (e != hipSuccess) return e;
    }
  }
  return hipGetLastError();
}

}  // namespace rps
