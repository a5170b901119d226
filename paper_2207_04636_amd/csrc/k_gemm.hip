// General FP64 matrix product on the FP64 matrix cores (v_mfma_f64_16x16x4_f64).
//
// Used by the one-time set-up (fitting metric, fitting functions, W, Gram
// matrices of the point selection, trailing updates of the factorisations)
// and by the small contractions of an exchange build.
//
// Tiling: 256 threads = 4 waves in a WGM x (4/WGM) grid; each wave owns a
// (16*TM) x (16*TN) block of C.  Square problems use 2 x 2 waves of 32 x 32
// (64 x 64 tiles); products with at most 16 columns use 4 x 1 waves of 32 x 16.
// K advances in steps of 16 through LDS, stored k-major so that both operand
// fetches of the MFMA read consecutive addresses across the 16 lanes of a row.
#include "mfma.h"
#include "rps_internal.h"

namespace rps {
namespace {

constexpr int BK = 16;

template <int WGM, int TM, int TN>
__global__ __launch_bounds__(256) void gemm_kernel(Gemm g) {
  constexpr int WGN = 4 / WGM;
  constexpr int BM = WGM * 16 * TM, BN = WGN * 16 * TN;
  __shared__ double As[BK][BM + 1];
  __shared__ double Bs[BK][BN + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
  if (g.lower_only && n0 > m0 + BM - 1) return;

  d4_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = zero_d4();

  // split-K: blockIdx.z owns K range [kbeg, kend)
  int64_t kbeg = 0, kend = g.K;
  if (g.splitk > 1) {
    const int64_t per = ((g.K + g.splitk - 1) / g.splitk + BK - 1) / BK * BK;
    kbeg = (int64_t)blockIdx.z * per;
    kend = (kbeg + per < g.K) ? kbeg + per : g.K;
  }
  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
    // stage op(A)[m0:m0+BM, k0:k0+BK] -> As[k][m]
    for (int e = tid; e < BM * BK; e += 256) {
      int m, k;
      if (g.transA) { m = e % BM; k = e / BM; } else { k = e % BK; m = e / BK; }
      int64_t gm = m0 + m, gk = k0 + k;
      double v = 0.0;
      if (gm < g.M && gk < kend) v = g.transA ? g.A[gk * g.lda + gm] : g.A[gm * g.lda + gk];
      As[k][m] = v;
    }
    for (int e = tid; e < BN * BK; e += 256) {
      int n, k;
      if (g.transB) { k = e % BK; n = e / BK; } else { n = e % BN; k = e / BN; }
      int64_t gn = n0 + n, gk = k0 + k;
      double v = 0.0;
      if (gn < g.N && gk < kend) v = g.transB ? g.B[gn * g.ldb + gk] : g.B[gk * g.ldb + gn];
      Bs[k][n] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4);
      double a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = As[kr][wm * 16 * TM + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = Bs[kr][wn * 16 * TN + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = mfma_f64(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int64_t gm = m0 + wm * 16 * TM + i * 16 + d64_row(lane, r);
        int64_t gn = n0 + wn * 16 * TN + j * 16 + (lane & 15);
        if (gm < g.M && gn < g.N) {
          double v = g.alpha * acc[i][j][r];
          if (g.splitk > 1) {
            g.work[((int64_t)blockIdx.z * g.M + gm) * g.N + gn] = v;
            continue;
          }
          double* c = g.C + gm * g.ldc + gn;
          if (g.epi == EPI_SQUARE) *c = v * v;
          else if (g.epi == EPI_HADAMARD) *c = *c * v;
          else if (g.epi == EPI_HADAMARD_SRC) *c = g.D[gm * g.ldd + gn] * v;
          else *c = (g.beta == 0.0) ? v : v + g.beta * *c;
        }
      }
}

// C = alpha * sum_z work[z] + beta * C (fixed order over z)
__global__ void splitk_reduce_kernel(const double* __restrict__ work, int splitk, int64_t M, int64_t N,
                                     double* __restrict__ C, int64_t ldc, double beta) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= M * N) return;
  double s = 0.0;
  for (int z = 0; z < splitk; ++z) s += work[(int64_t)z * M * N + t];
  const int64_t m = t / N, n = t % N;
  double* c = C + m * ldc + n;
  *c = (beta == 0.0) ? s : s + beta * *c;
}

}  // namespace

hipError_t gemm_f64(const Gemm& g0, hipStream_t s) {
  Gemm g = g0;
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  if (g.K <= 0) {
    // alpha*AB = 0
    if (g.epi == EPI_AXPBY && g.beta == 1.0) return hipSuccess;
  }
  if (g.splitk > 1 && (!g.work || g.epi != EPI_AXPBY)) return hipErrorInvalidValue;
  if (g.splitk < 1) g.splitk = 1;
  if (g.N <= 16) {
    dim3 grid((unsigned)((g.N + 15) / 16), (unsigned)((g.M + 127) / 128), (unsigned)g.splitk);
    hipLaunchKernelGGL((gemm_kernel<4, 2, 1>), grid, dim3(256), 0, s, g);
  } else {
    dim3 grid((unsigned)((g.N + 63) / 64), (unsigned)((g.M + 63) / 64), (unsigned)g.splitk);
    hipLaunchKernelGGL((gemm_kernel<2, 2, 2>), grid, dim3(256), 0, s, g);
  }
  if (g.splitk > 1) {
    const int64_t cnt = g.M * g.N;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, g.work,
                       g.splitk, g.M, g.N, g.C, g.ldc, g.beta);
  }
  return hipGetLastError();
}

int gemm_splitk_for(int64_t M, int64_t N, int64_t K, int64_t work_cap_doubles) {
  // aim for >= 512 workgroups, at least 256 K per split, bounded by the workspace
  const int64_t tiles = (N <= 16) ? ((M + 127) / 128) * ((N + 15) / 16) : ((M + 63) / 64) * ((N + 63) / 64);
  int64_t z = 1;
  while (tiles * z < 512 && K / (z * 2) >= 256 && (z * 2) * M * N <= work_cap_doubles) z *= 2;
  return (int)z;
}

}  // namespace rps
