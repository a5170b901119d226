// Basis functions on the grid, Voronoi assignment and small utility kernels.
//
// Basis (Sec. 2.1.3): phi_P(R) = sum_T phi(R - A - T) over lattice images T.
// The displacement R - A is first reduced to fractional coordinates in
// [-1/2, 1/2); the images n1 a1 + n2 a2 + n3 a3 with |n_k| <= m_k (m_k from the
// cutoff radius and the plane spacings, computed on the host) are summed while
// a |d|^2 <= 50.  Components and normalisation:
//   s  N_s e^{-a r^2}, N_s = (2a/pi)^{3/4}
//   p  N_s 2 sqrt(a) (x, y, z) e^{-a r^2}
//   d  N_s 4a (xy, yz, zx), N_s 2a (x^2 - y^2), N_s 2a/sqrt(3) (3z^2 - r^2), times e^{-a r^2}
// Voronoi (Sec. 4.1): nearest atom under periodic images, ties to the lower index.
#include <math.h>

#include "mfma.h"
#include "rps_internal.h"

namespace rps {
namespace {

// 1-D launches over more than 2^32 work-items (e.g. N_aux x N_g at the largest
// sizes) do not fit one grid dimension: blocks are laid out over x and y.
__device__ __forceinline__ int64_t flat_id() {
  return ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x;
}
inline dim3 flat_grid(int64_t n) {
  const int64_t b = (n + 255) / 256;
  const int64_t gx = b < 65536 ? (b > 0 ? b : 1) : 65536;
  return dim3((unsigned)gx, (unsigned)((b + gx - 1) / gx));
}

constexpr double kCutoff = 50.0;

__device__ __forceinline__ void grid_point(const CellDev& c, int64_t idx, double r[3]) {
  const int64_t n23 = (int64_t)c.mesh[1] * c.mesh[2];
  const int i1 = (int)(idx / n23);
  const int i2 = (int)((idx / c.mesh[2]) % c.mesh[1]);
  const int i3 = (int)(idx % c.mesh[2]);
  const double f1 = (double)i1 / c.mesh[0], f2 = (double)i2 / c.mesh[1], f3 = (double)i3 / c.mesh[2];
#pragma unroll
  for (int k = 0; k < 3; ++k) r[k] = f1 * c.a[k] + f2 * c.a[3 + k] + f3 * c.a[6 + k];
}

// Reduce d to fractional coordinates in [-1/2, 1/2) (componentwise) and back.
__device__ __forceinline__ void reduce_disp(const CellDev& c, double d[3]) {
  double f[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    f[k] = d[0] * c.ainv[k] + d[1] * c.ainv[3 + k] + d[2] * c.ainv[6 + k];
    f[k] -= rint(f[k]);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) d[k] = f[0] * c.a[k] + f[1] * c.a[3 + k] + f[2] * c.a[6 + k];
}

// One thread per (grid point, shell); shells vary fastest so that a wave
// writes neighbouring columns of the same row.
__global__ __launch_bounds__(256) void basis_kernel(CellDev cell, const ShellDev* __restrict__ shells,
                                                   int nshell, int64_t ngrid, double* __restrict__ Phi,
                                                   int64_t ld) {
  const int64_t t = flat_id();
  if (t >= ngrid * nshell) return;
  const int64_t R = t / nshell;
  const ShellDev sh = shells[t % nshell];
  double r[3];
  grid_point(cell, R, r);
  double d0[3] = {r[0] - sh.cx, r[1] - sh.cy, r[2] - sh.cz};
  reduce_disp(cell, d0);
  const double a = sh.expo;
  double acc[5] = {0, 0, 0, 0, 0};
  for (int n1 = -sh.m0; n1 <= sh.m0; ++n1)
    for (int n2 = -sh.m1; n2 <= sh.m1; ++n2)
      for (int n3 = -sh.m2; n3 <= sh.m2; ++n3) {
        const double x = d0[0] + n1 * cell.a[0] + n2 * cell.a[3] + n3 * cell.a[6];
        const double y = d0[1] + n1 * cell.a[1] + n2 * cell.a[4] + n3 * cell.a[7];
        const double z = d0[2] + n1 * cell.a[2] + n2 * cell.a[5] + n3 * cell.a[8];
        const double r2 = x * x + y * y + z * z;
        if (a * r2 > kCutoff) continue;
        const double e = exp(-a * r2);
        if (sh.l == 0) {
          acc[0] += e;
        } else if (sh.l == 1) {
          acc[0] += x * e; acc[1] += y * e; acc[2] += z * e;
        } else {
          acc[0] += x * y * e; acc[1] += y * z * e; acc[2] += z * x * e;
          acc[3] += (x * x - y * y) * e; acc[4] += (2.0 * z * z - x * x - y * y) * e;
        }
      }
  const double ns = pow(2.0 * a / M_PI, 0.75);
  double* out = Phi + R * ld + sh.fofs;
  if (sh.l == 0) {
    out[0] = ns * acc[0];
  } else if (sh.l == 1) {
    const double c = ns * 2.0 * sqrt(a);
    out[0] = c * acc[0]; out[1] = c * acc[1]; out[2] = c * acc[2];
  } else {
    const double c1 = ns * 4.0 * a, c2 = ns * 2.0 * a, c3 = ns * 2.0 * a / sqrt(3.0);
    out[0] = c1 * acc[0]; out[1] = c1 * acc[1]; out[2] = c1 * acc[2];
    out[3] = c2 * acc[3]; out[4] = c3 * acc[4];
  }
}

__global__ __launch_bounds__(256) void voronoi_kernel(CellDev cell, const double* __restrict__ atoms,
                                                     int natom, int64_t ngrid, int32_t* __restrict__ owner) {
  const int64_t R = flat_id();
  if (R >= ngrid) return;
  double r[3];
  grid_point(cell, R, r);
  double best = INFINITY;
  int who = 0;
  for (int I = 0; I < natom; ++I) {
    double d0[3] = {r[0] - atoms[3 * I], r[1] - atoms[3 * I + 1], r[2] - atoms[3 * I + 2]};
    reduce_disp(cell, d0);
    double dmin = INFINITY;
    for (int s1 = -1; s1 <= 1; ++s1)
      for (int s2 = -1; s2 <= 1; ++s2)
        for (int s3 = -1; s3 <= 1; ++s3) {
          const double x = d0[0] + s1 * cell.a[0] + s2 * cell.a[3] + s3 * cell.a[6];
          const double y = d0[1] + s1 * cell.a[1] + s2 * cell.a[4] + s3 * cell.a[7];
          const double z = d0[2] + s1 * cell.a[2] + s2 * cell.a[5] + s3 * cell.a[8];
          dmin = fmin(dmin, x * x + y * y + z * z);
        }
    if (dmin < best) { best = dmin; who = I; }
  }
  owner[R] = who;
}

__global__ void gather_kernel(const double* __restrict__ src, int64_t lds, const int64_t* __restrict__ idx,
                              int64_t nidx, int64_t nrows, int64_t ncols, double* __restrict__ dst, int64_t ldd) {
  const int64_t t = flat_id();
  if (t >= nrows * ncols) return;
  const int64_t r = t / ncols, c = t % ncols;
  dst[r * ldd + c] = (r < nidx) ? src[idx[r] * lds + c] : 0.0;
}

__global__ void add_diag_kernel(double* X, int64_t ld, int64_t i0, int64_t i1, double v) {
  const int64_t i = i0 + flat_id();
  if (i < i1) X[i * ld + i] += v;
}

__global__ void fill_kernel(double* X, int64_t count, double v) {
  const int64_t i = flat_id();
  if (i < count) X[i] = v;
}

__global__ void symmetrize_kernel(double* A, int64_t n, int64_t ld) {
  const int64_t t = flat_id();
  if (t >= n * n) return;
  const int64_t i = t / n, j = t % n;
  if (j >= i) return;
  const double v = 0.5 * (A[i * ld + j] + A[j * ld + i]);
  A[i * ld + j] = v;
  A[j * ld + i] = v;
}

__global__ void mirror_upper_kernel(double* A, int64_t n, int64_t ld) {
  const int64_t t = flat_id();
  if (t >= n * n) return;
  const int64_t i = t / n, j = t % n;
  if (j < i) A[i * ld + j] = A[j * ld + i];
}

__global__ void transpose_kernel(const double* __restrict__ in, int64_t ldi, int64_t rows, int64_t cols,
                                 double* __restrict__ out, int64_t ldo) {
  __shared__ double tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  for (int k = threadIdx.y; k < 32; k += 8) {
    const int64_t r = r0 + k, c = c0 + threadIdx.x;
    tile[k][threadIdx.x] = (r < rows && c < cols) ? in[r * ldi + c] : 0.0;
  }
  __syncthreads();
  for (int k = threadIdx.y; k < 32; k += 8) {
    const int64_t c = c0 + k, r = r0 + threadIdx.x;
    if (r < rows && c < cols) out[c * ldo + r] = tile[threadIdx.x][k];
  }
}

__global__ void unit_rows_kernel(double* X, int64_t ld, const int64_t* __restrict__ idx, int64_t n) {
  const int64_t g = flat_id();
  if (g < n) X[g * ld + idx[g]] = 1.0;
}

__global__ void gather_cols_kernel(const double* __restrict__ X, int64_t ldx, const int64_t* __restrict__ idx,
                                   int64_t n, double* __restrict__ Y, int64_t ldy) {
  const int64_t t = flat_id();
  if (t >= n * n) return;
  const int64_t r = t / n, c = t % n;
  Y[r * ldy + c] = X[r * ldx + idx[c]];
}

__global__ void to_f32_kernel(const double* __restrict__ X, int64_t count, float* __restrict__ Y) {
  const int64_t i = flat_id();
  if (i < count) Y[i] = (float)X[i];
}

__global__ void to_f32_pad_kernel(const double* __restrict__ X, int64_t rows, int64_t n, float* __restrict__ Y,
                                  int64_t ldy) {
  const int64_t i = flat_id();
  if (i >= rows * ldy) return;
  const int64_t r = i / ldy, c = i % ldy;
  Y[i] = (c < n) ? (float)X[r * n + c] : 0.f;
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t set_unit_rows(double* X, int64_t ld, const int64_t* idx, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(unit_rows_kernel, flat_grid(n), dim3(256), 0, s, X, ld, idx, n);
  return hipGetLastError();
}

hipError_t gather_cols(const double* X, int64_t ldx, const int64_t* idx, int64_t n, double* Y,
                       int64_t ldy, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_cols_kernel, flat_grid(n * n), dim3(256), 0, s, X, ldx, idx, n, Y, ldy);
  return hipGetLastError();
}

hipError_t to_f32(const double* X, int64_t count, float* Y, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(to_f32_kernel, flat_grid(count), dim3(256), 0, s, X, count, Y);
  return hipGetLastError();
}

hipError_t to_f32_pad(const double* X, int64_t rows, int64_t n, float* Y, int64_t ldy, hipStream_t s) {
  if (rows <= 0 || ldy < n) return rows <= 0 ? hipSuccess : hipErrorInvalidValue;
  hipLaunchKernelGGL(to_f32_pad_kernel, flat_grid(rows * ldy), dim3(256), 0, s, X, rows, n, Y, ldy);
  return hipGetLastError();
}

hipError_t basis_eval(const CellDev& cell, const ShellDev* shells, int nshell, int64_t ngrid,
                      double* Phi, int64_t ldphi, hipStream_t s) {
  hipLaunchKernelGGL(basis_kernel, flat_grid(ngrid * nshell), dim3(256), 0, s, cell, shells,
                     nshell, ngrid, Phi, ldphi);
  return hipGetLastError();
}

hipError_t voronoi_assign(const CellDev& cell, const double* atoms, int natom, int64_t ngrid,
                          int32_t* owner, hipStream_t s) {
  hipLaunchKernelGGL(voronoi_kernel, flat_grid(ngrid), dim3(256), 0, s, cell, atoms, natom,
                     ngrid, owner);
  return hipGetLastError();
}

hipError_t gather_rows(const double* src, int64_t lds, const int64_t* idx, int64_t nidx,
                       int64_t nrows, int64_t ncols, double* dst, int64_t ldd, hipStream_t s) {
  if (nrows * ncols == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_kernel, flat_grid(nrows * ncols), dim3(256), 0, s, src, lds, idx,
                     nidx, nrows, ncols, dst, ldd);
  return hipGetLastError();
}

hipError_t add_diag(double* X, int64_t ld, int64_t i0, int64_t i1, double v, hipStream_t s) {
  if (i1 <= i0) return hipSuccess;
  hipLaunchKernelGGL(add_diag_kernel, flat_grid(i1 - i0), dim3(256), 0, s, X, ld, i0, i1, v);
  return hipGetLastError();
}

hipError_t fill(double* X, int64_t count, double v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, flat_grid(count), dim3(256), 0, s, X, count, v);
  return hipGetLastError();
}

hipError_t symmetrize(double* A, int64_t n, int64_t ld, hipStream_t s) {
  hipLaunchKernelGGL(symmetrize_kernel, flat_grid(n * n), dim3(256), 0, s, A, n, ld);
  return hipGetLastError();
}

hipError_t mirror_upper(double* A, int64_t n, int64_t ld, hipStream_t s) {
  hipLaunchKernelGGL(mirror_upper_kernel, flat_grid(n * n), dim3(256), 0, s, A, n, ld);
  return hipGetLastError();
}

hipError_t transpose(const double* in, int64_t ldi, int64_t rows, int64_t cols, double* out,
                     int64_t ldo, hipStream_t s) {
  dim3 grid(nblk(cols, 32), nblk(rows, 32));
  hipLaunchKernelGGL(transpose_kernel, grid, dim3(32, 8), 0, s, in, ldi, rows, cols, out, ldo);
  return hipGetLastError();
}

}  // namespace rps
