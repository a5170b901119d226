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
#include <algorithm>

#include "mfma.h"
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
constexpr int ZG = 16;
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

// Small-basis path (Np = 16 MT <= 128, np = 16 NI <= 64), Coulomb steps 1 and 4 in
// one pass over Phi each, FP64 matrix cores.
//
// Density: each wave takes 16-row subtiles of Phi (A operand straight from global,
// all Np/4 k slices requested before the products), U = Phi C against C staged in
// LDS, and rho = sum_i U^2 reduced over the 16 lanes holding a row.  rho goes to
// out[r] and out[2 ld + r], 0 to out[ld + r].
template <int NI, int MT>
__global__ __launch_bounds__(256) void density_small_kernel(const double* __restrict__ Phi, int64_t rows,
                                                           const double* __restrict__ C, int N, int n,
                                                           double* __restrict__ out, int64_t ld) {
  constexpr int NP = 16 * NI, NPK = 16 * MT;
  __shared__ double sC[NPK * NP];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, lq = lane >> 4;
  for (int e = tid; e < NPK * NP; e += 256) {
    const int r = e / NP, c = e % NP;
    sC[e] = (r < N && c < n) ? C[(int64_t)r * n + c] : 0.0;
  }
  __syncthreads();
  const int64_t nsub = rows / 16;
  for (int64_t sidx = (int64_t)blockIdx.x * 4 + w; sidx < nsub; sidx += (int64_t)gridDim.x * 4) {
    const double* src = Phi + (sidx * 16 + l16) * NPK + lq;
    double x[4 * MT];
#pragma unroll
    for (int kk = 0; kk < 4 * MT; ++kk) x[kk] = src[4 * kk];
    d4_t acc[NI];
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[j] = zero_d4();
#pragma unroll
    for (int kk = 0; kk < 4 * MT; ++kk)
#pragma unroll
      for (int j = 0; j < NI; ++j) acc[j] = mfma_f64(x[kk], sC[(4 * kk + lq) * NP + 16 * j + l16], acc[j]);
    // lane (lq, l16), reg r holds U[4 r + lq][16 j + l16]
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double v = 0.0;
#pragma unroll
      for (int j = 0; j < NI; ++j) v += acc[j][r] * acc[j][r];
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) v += __shfl_xor(v, off, 64);
      if (l16 == 0) {
        const int64_t row = sidx * 16 + 4 * r + lq;
        out[row] = v;
        out[ld + row] = 0.0;
        out[2 * ld + row] = v;
      }
    }
  }
}

// J partials: workgroup b sums v[R] phi[R][mu] phi[R][nu] over its chunks of 64 grid
// rows (b, b + gridDim.x, ...) for the lower 16 x 16 tiles (mb >= nb) and writes them
// to part[b][Np][Np] (upper tiles untouched).  Chunks are staged in LDS with the next
// one requested into registers meanwhile; tile t of the lower triangle belongs to wave
// t % 8.
template <int MT>
__global__ __launch_bounds__(512) void coulomb_small_kernel(const double* __restrict__ Phi, int64_t rows,
                                                           const double* __restrict__ v,
                                                           double* __restrict__ part) {
  constexpr int NPK = 16 * MT, RC = 64, PPD = NPK + 1;
  constexpr int NT = MT * (MT + 1) / 2, TPW = (NT + 7) / 8;
  constexpr int PER = RC * NPK / 512;          // doubles per thread of a chunk
  static_assert(PER * 512 == RC * NPK, "chunk split");
  __shared__ double sP[RC * PPD];
  __shared__ double sv[RC];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, lq = lane >> 4;
  const int64_t nchunk = rows / RC;
  // this wave's tiles (mb, nb), mb >= nb
  int tmb[TPW], tnb[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    int t = w + 8 * q, mb = 0;
    while (t > mb) { t -= mb + 1; ++mb; }
    tmb[q] = (w + 8 * q < NT) ? mb : -1;
    tnb[q] = t;
  }
  d4_t acc[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) acc[q] = zero_d4();
  double nx[PER];
  double nv = 0.0;
  auto fetch = [&](int64_t c) {
    const double* src = Phi + c * RC * NPK;
#pragma unroll
    for (int i = 0; i < PER; ++i) nx[i] = src[tid + 512 * i];
    if (tid < RC) nv = v[c * RC + tid];
  };
  int64_t c = blockIdx.x;
  if (c < nchunk) fetch(c);
  for (; c < nchunk; c += gridDim.x) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = tid + 512 * i;
      sP[(e / NPK) * PPD + e % NPK] = nx[i];
    }
    if (tid < RC) sv[tid] = nv;
    __syncthreads();
    if (c + gridDim.x < nchunk) fetch(c + gridDim.x);
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      if (tmb[q] < 0) continue;
      const double* pa = sP + lq * PPD + 16 * tmb[q] + l16;
      const double* pb = sP + lq * PPD + 16 * tnb[q] + l16;
#pragma unroll
      for (int kk = 0; kk < RC / 4; ++kk)
        acc[q] = mfma_f64(pa[4 * kk * PPD], sv[4 * kk + lq] * pb[4 * kk * PPD], acc[q]);
    }
  }
  double* o = part + (int64_t)blockIdx.x * NPK * NPK;
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    if (tmb[q] < 0) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) o[(16 * tmb[q] + 4 * r + lq) * NPK + 16 * tnb[q] + l16] = acc[q][r];
  }
}

}  // namespace

int coulomb_small_blocks(int64_t rows) {
  const int64_t nchunk = rows / 64;
  return (int)std::min<int64_t>(256, std::max<int64_t>(1, nchunk));
}

hipError_t density_small(const double* Phi, int64_t rows, int Np, const double* C, int N, int n, int np,
                         double* out, int64_t ld, hipStream_t s) {
  if (rows % 16 != 0 || Np % 16 != 0 || Np > 128 || np % 16 != 0 || np > 64) return hipErrorInvalidValue;
  const unsigned blocks = (unsigned)std::min<int64_t>((rows / 16 + 3) / 4, 1024);
#define RPS_DEN(NI_, MT_) \
  hipLaunchKernelGGL((density_small_kernel<NI_, MT_>), dim3(blocks), dim3(256), 0, s, Phi, rows, C, N, n, out, ld)
#define RPS_DEN_MT(NI_)                                                                                     \
  switch (Np / 16) {                                                                                         \
    case 1: RPS_DEN(NI_, 1); break; case 2: RPS_DEN(NI_, 2); break; case 3: RPS_DEN(NI_, 3); break;          \
    case 4: RPS_DEN(NI_, 4); break; case 5: RPS_DEN(NI_, 5); break; case 6: RPS_DEN(NI_, 6); break;          \
    case 7: RPS_DEN(NI_, 7); break; default: RPS_DEN(NI_, 8); break;                                         \
  }
  switch (np / 16) {
    case 1: RPS_DEN_MT(1); break;
    case 2: RPS_DEN_MT(2); break;
    case 3: RPS_DEN_MT(3); break;
    default: RPS_DEN_MT(4); break;
  }
#undef RPS_DEN_MT
#undef RPS_DEN
  return hipGetLastError();
}

hipError_t coulomb_small(const double* Phi, int64_t rows, int Np, const double* v, double* part, hipStream_t s) {
  if (rows % 64 != 0 || Np % 16 != 0 || Np > 128) return hipErrorInvalidValue;
  const int blocks = coulomb_small_blocks(rows);
  switch (Np / 16) {
    case 1: hipLaunchKernelGGL((coulomb_small_kernel<1>), dim3(blocks), dim3(512), 0, s, Phi, rows, v, part); break;
    case 2: hipLaunchKernelGGL((coulomb_small_kernel<2>), dim3(blocks), dim3(512), 0, s, Phi, rows, v, part); break;
    case 3: hipLaunchKernelGGL((coulomb_small_kernel<3>), dim3(blocks), dim3(512), 0, s, Phi, rows, v, part); break;
    case 4: hipLaunchKernelGGL((coulomb_small_kernel<4>), dim3(blocks), dim3(512), 0, s, Phi, rows, v, part); break;
    case 5: hipLaunchKernelGGL((coulomb_small_kernel<5>), dim3(blocks), dim3(512), 0, s, Phi, rows, v, part); break;
    case 6: hipLaunchKernelGGL((coulomb_small_kernel<6>), dim3(blocks), dim3(512), 0, s, Phi, rows, v, part); break;
    case 7: hipLaunchKernelGGL((coulomb_small_kernel<7>), dim3(blocks), dim3(512), 0, s, Phi, rows, v, part); break;
    default: hipLaunchKernelGGL((coulomb_small_kernel<8>), dim3(blocks), dim3(512), 0, s, Phi, rows, v, part); break;
  }
  return hipGetLastError();
}

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
