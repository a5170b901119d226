// Coulomb matrix on the grid (Sec. 2.3, "Coulomb matrix", steps 1-4; Sec. 4.2):
//   1. rho(R) = sum_i U(R, i)^2 with U = Phi C, the density of D = C C^T,
//   2-3. V_H = Vc rho (the set-up's Poisson solve, one row pair),
//   4. J = dV Phi^T diag(V_H) Phi, a matrix-core product over the grid whose
//      second operand is scaled row by row as it is loaded (lower tiles only,
//      mirrored here),
// and E_J = dV sum_R rho(R) V_H(R) = sum_ij (ii|jj).
//
// The kernels below are the small steps around the products: the density of a
// block of grid rows, a fixed-order dot product and the symmetric reduction of
// the split-K partials of J; and the Madelung term of the exchange (Sec. 4.5):
// K_occ += M S C, E_x -= M tr(C^T S C).
#include "rps_internal.h"

namespace rps {
namespace {

// rho[r] = sum_i U[r][i]^2 for r < rows, written to out[r] and out[2 ld + r];
// out[ld + r] = 0 (the imaginary row of the Poisson pair).  np is even.
__global__ __launch_bounds__(256) void density_rows_kernel(const double* __restrict__ U, int64_t rows, int np,
                                                           double* __restrict__ out, int64_t ld) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const double2* u = reinterpret_cast<const double2*>(U + r * np);
  double s0 = 0.0, s1 = 0.0;
  for (int i = 0; i < np / 2; ++i) {
    const double2 v = u[i];
    s0 += v.x * v.x;
    s1 += v.y * v.y;
  }
  const double rho = s0 + s1;
  out[r] = rho;
  out[ld + r] = 0.0;
  out[2 * ld + r] = rho;
}

// part[b] = sum over block b's slice of x[p] y[p]
__global__ __launch_bounds__(256) void dot_blocks_kernel(const double* __restrict__ x, const double* __restrict__ y,
                                                         int64_t n, double* __restrict__ part) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * per;
  const int64_t b1 = (b0 + per < n) ? b0 + per : n;
  double s = 0.0;
  for (int64_t p = b0 + tid; p < b1; p += 256) s += x[p] * y[p];
  red[tid] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0) part[blockIdx.x] = red[0];
}

// *out = scale * sum_i part[i]: one block, strided partial sums, fixed-order tree
__global__ __launch_bounds__(256) void sum_scaled_kernel(const double* __restrict__ part, int n, double scale,
                                                         double* __restrict__ out) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int i = tid; i < n; i += 256) s += part[i];
  red[tid] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0) *out = scale * red[0];
}

// J[i][j] = J[j][i] = scale * sum_z work[z][i][j] for j <= i < N.  Block (64, ZG):
// 64 consecutive elements of the [Np][Np] partials, ZG interleaved groups of z
// summed separately, then combined in a fixed order.
constexpr int ZG = 4;
__global__ __launch_bounds__(64 * ZG) void sym_from_lower_kernel(const double* __restrict__ work, int nz, int64_t Np,
                                                                 int64_t N, double scale, double* __restrict__ J) {
  __shared__ double red[ZG][64];
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 64 + tx;
  const int64_t i = e / Np, j = e % Np;
  const bool live = (i < N) && (j <= i);
  double s = 0.0;
  if (live)
    for (int z = ty; z < nz; z += ZG) s += work[(int64_t)z * Np * Np + e];
  red[ty][tx] = s;
  __syncthreads();
  if (ty == 0 && live) {
    double t = red[0][tx];
    for (int g = 1; g < ZG; ++g) t += red[g][tx];
    t *= scale;
    J[i * N + j] = t;
    J[j * N + i] = t;
  }
}

// K[mu][i] += M SC[mu][i] for mu < N, i < n (K pitch n, SC pitch ldsc);
// part[b] = sum over block b's slice of C[mu][i] SC[mu][i] (C pitch n)
__global__ __launch_bounds__(256) void madelung_k_kernel(const double* __restrict__ SC, int64_t ldsc,
                                                         const double* __restrict__ C, int64_t N, int64_t n,
                                                         double M, double* __restrict__ K,
                                                         double* __restrict__ part) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int64_t cnt = N * n;
  const int64_t per = (cnt + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * per;
  const int64_t b1 = (b0 + per < cnt) ? b0 + per : cnt;
  double s = 0.0;
  for (int64_t e = b0 + tid; e < b1; e += 256) {
    const int64_t mu = e / n, i = e % n;
    const double sc = SC[mu * ldsc + i];
    K[e] += M * sc;
    s += C[e] * sc;
  }
  red[tid] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0) part[blockIdx.x] = red[0];
}

// ex -= M * sum_b part[b] (one block, fixed-order tree)
__global__ __launch_bounds__(256) void madelung_e_kernel(const double* __restrict__ part, int n, double M,
                                                         double* __restrict__ ex) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int i = tid; i < n; i += 256) s += part[i];
  red[tid] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0) *ex -= M * red[0];
}

}  // namespace

hipError_t madelung_apply(const double* SC, int64_t ldsc, const double* C, int64_t N, int64_t n, double M,
                          double* K, double* ex, double* part, int nparts, hipStream_t s) {
  if (nparts < 1 || nparts > 256 || N * n <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(madelung_k_kernel, dim3((unsigned)nparts), dim3(256), 0, s, SC, ldsc, C, N, n, M, K, part);
  if (ex) hipLaunchKernelGGL(madelung_e_kernel, dim3(1), dim3(256), 0, s, part, nparts, M, ex);
  return hipGetLastError();
}

hipError_t density_rows(const double* U, int64_t rows, int np, double* out, int64_t ld, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  if (np % 2 != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(density_rows_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, U, rows, np, out, ld);
  return hipGetLastError();
}

hipError_t dot_scaled(const double* x, const double* y, int64_t n, double scale, double* part, int nparts,
                      double* out, hipStream_t s) {
  if (nparts < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(dot_blocks_kernel, dim3((unsigned)nparts), dim3(256), 0, s, x, y, n, part);
  hipLaunchKernelGGL(sum_scaled_kernel, dim3(1), dim3(256), 0, s, part, nparts, scale, out);
  return hipGetLastError();
}

hipError_t sym_from_lower(const double* work, int nz, int64_t Np, int64_t N, double scale, double* J,
                          hipStream_t s) {
  if (N <= 0) return hipSuccess;
  const int64_t cnt = N * Np;   // rows below N of the partials
  hipLaunchKernelGGL(sym_from_lower_kernel, dim3((unsigned)((cnt + 63) / 64)), dim3(64, ZG), 0, s, work, nz, Np, N,
                     scale, J);
  return hipGetLastError();
}

}  // namespace rps
