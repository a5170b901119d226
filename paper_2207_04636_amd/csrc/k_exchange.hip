// Per-build exchange contractions, Eq. 16 (occ-RI rPS, Sec. 3.3), FP64.
//
// With U = Phi C (orbitals on the grid), U_g = U at the interpolation points,
// P = U_g U^T and A = V o P (o: elementwise), the first two lines of Eq. 16 are
//   line 1:  K1 = Phi^T (A^T U_g)        (contraction over the points g, then grid R)
//   line 2:  K2 = Phi_g^T (A U)          (contraction over R first, Sec. 4.4 order)
// and the energy needs e1 = sum A o P.  The fused kernel streams the stored
// potential V from HBM exactly once: for each 64 x 64 tile it forms P with the
// FP64 matrix cores (inner dimension n), multiplies by the V tile in registers,
// stages A through LDS (the second contraction needs the transposed fragment
// layout), and accumulates both products with the matrix cores:
//   M1^T[R][i] = sum_g A[g][R] U_g[g][i]   (registers, summed over the g loop)
//   M2[g][i]   = sum_R A[g][R] U[R][i]     (registers, summed over the R loop)
// A workgroup owns a block of g rows and a block of R columns; g tiles are the
// outer loop and R tiles the inner one.  M2 partials (one per R block) go to
// global memory and are reduced in a fixed order.  When N and n are small, the
// K1 product Phi^T M1^T is also fused (Phi rows of the R block are read once at
// the end), so M1 never leaves the chip; K1 partials are reduced in order.
//
// The third line (fit-fit) has the same structure with V -> W, U -> U_g and
// Phi -> Phi_g, because W and P_g are symmetric: K3 = Phi_g^T (B U_g) with
// B = W o P_g; the same kernel computes it with M2 disabled.
#include <math.h>

#include "mfma.h"
#include "rps_internal.h"

namespace rps {
namespace {

constexpr int T = 64;        // tile edge
constexpr int LDA = T + 1;   // LDS pitch of the A tile (doubles)

template <int NI, int RT, int MT>
__global__ __launch_bounds__(256) void fused_f64_kernel(FusedArgs a) {
  constexpr int NP = 16 * NI;          // padded n
  constexpr int LDU = NP + 1;          // LDS pitch of the U tiles
  __shared__ double sA[T][LDA];
  __shared__ double sUg[T][LDU];       // U_g rows of the current g tile
  __shared__ double sUr[T][LDU];       // U rows of the current R tile
  __shared__ double sRed[4][64];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, lq = lane >> 4;

  const int64_t gtiles = a.G / T;
  const int64_t gper = (gtiles + a.gblocks - 1) / a.gblocks;
  const int gb = blockIdx.x % a.gblocks;
  const int rb = blockIdx.x / a.gblocks;
  const int64_t gt0 = gb * gper;
  const int64_t gt1 = (gt0 + gper < gtiles) ? gt0 + gper : gtiles;
  const int64_t rtiles_valid = (a.R_valid + T - 1) / T;
  const int64_t rt0 = (int64_t)rb * RT;
  const int64_t rt1 = (rt0 + RT < rtiles_valid) ? rt0 + RT : rtiles_valid;
  const int nrt = (int)(rt1 - rt0);
  const int64_t ntile = (gt1 > gt0 && nrt > 0) ? (gt1 - gt0) * nrt : 0;

  d4_t m1[RT][NI];
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int j = 0; j < NI; ++j) m1[r][j] = zero_d4();
  d4_t m2[NI];
  double e1 = 0.0;

  // V fragment of tile t: lane holds V[g0 + 16w + 4r + lq][R0 + 16c + l16]
  double vnext[4][4];
  auto load_v = [&](int64_t t) {
    const int64_t g0 = (gt0 + t / nrt) * T, R0 = (rt0 + t % nrt) * T;
    const double* base = a.Vm + (g0 + 16 * w + lq) * a.ldv + R0 + l16;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double* row = base + (int64_t)(4 * r) * a.ldv;
#pragma unroll
      for (int c = 0; c < 4; ++c) vnext[r][c] = row[16 * c];
    }
  };
  // stage 64 rows x NP of a U matrix into LDS (rows contiguous, NP doubles each)
  auto stage = [&](double (*dst)[LDU], const double* src) {
#pragma unroll
    for (int e = tid; e < T * NP; e += 256) dst[e / NP][e % NP] = src[e];
  };
  if (ntile > 0) load_v(0);

  for (int64_t gt = gt0; gt < gt1 && nrt > 0; ++gt) {
    const int64_t g0 = gt * T;
#pragma unroll
    for (int j = 0; j < NI; ++j) m2[j] = zero_d4();
    stage(sUg, a.Ug + g0 * NP);
#pragma unroll
    for (int rl = 0; rl < RT; ++rl) {
      if (rl >= nrt) break;
      const int64_t t = (gt - gt0) * nrt + rl;
      const int64_t R0 = (rt0 + rl) * T;
      stage(sUr, a.Ur + R0 * NP);
      double v[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) v[r][c] = vnext[r][c];
      if (t + 1 < ntile) load_v(t + 1);
      __syncthreads();

      // P for rows g0+16w.. and the 4 column subtiles: D[g][R] += U_g[g][k] U^T[k][R]
      d4_t p[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) p[c] = zero_d4();
#pragma unroll
      for (int kk = 0; kk < NI * 4; ++kk) {
        const double x = sUg[16 * w + l16][4 * kk + lq];
#pragma unroll
        for (int c = 0; c < 4; ++c) p[c] = mfma_f64(x, sUr[16 * c + l16][4 * kk + lq], p[c]);
      }
      // A = V o P, energy, stage A
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double av = v[r][c] * p[c][r];
          e1 += av * p[c][r];
          sA[16 * w + 4 * r + lq][16 * c + l16] = av;
        }
      __syncthreads();

      // M1^T for column subtile w: D[R][i] += sum_g A^T[R][g] U_g[g][i]
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) {
        const double x = sA[4 * kk + lq][16 * w + l16];
#pragma unroll
        for (int j = 0; j < NI; ++j) m1[rl][j] = mfma_f64(x, sUg[4 * kk + lq][16 * j + l16], m1[rl][j]);
      }
      // M2 for row subtile w: D[g][i] += sum_R A[g][R] U[R][i]
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) {
        const double x = sA[16 * w + l16][4 * kk + lq];
#pragma unroll
        for (int j = 0; j < NI; ++j) m2[j] = mfma_f64(x, sUr[4 * kk + lq][16 * j + l16], m2[j]);
      }
      __syncthreads();
    }
    if (a.want_m2) {
      double* out = a.M2p + ((int64_t)rb * a.G + g0 + 16 * w) * NP + l16;
#pragma unroll
      for (int j = 0; j < NI; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) out[(int64_t)(4 * r + lq) * NP + 16 * j] = m2[j][r];
    }
  }

  const int wg = blockIdx.x;
  // M1^T rows of this workgroup (when K1 is not fused): lane holds
  // M1^T[R0 + 16w + 4r + lq][16j + l16]
  if (a.want_m1) {
#pragma unroll
    for (int rl = 0; rl < RT; ++rl) {
      if (rl >= nrt) break;
      const int64_t R0 = (rt0 + rl) * T;
      double* out = a.M1T + ((int64_t)gb * a.R + R0 + 16 * w) * NP + l16;
#pragma unroll
      for (int j = 0; j < NI; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) out[(int64_t)(4 * r + lq) * NP + 16 * j] = m1[rl][j][r];
    }
  }
  if (MT > 0 && a.want_k1) {
    // K1[mu][i] += sum_R Phi[R][mu] M1^T[R][i]; the M1 fragment registers are
    // already the B operand (reg r <-> k = 4r + lq of this wave's 16 rows).
    d4_t k1[MT > 0 ? MT : 1][NI];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int j = 0; j < NI; ++j) k1[m][j] = zero_d4();
    const int mt = a.Np / 16;
#pragma unroll
    for (int rl = 0; rl < RT; ++rl) {
      if (rl >= nrt) break;
      const int64_t R0 = (rt0 + rl) * T;
      const double* ph = a.Phir + (R0 + 16 * w + lq) * a.Np + l16;
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          if (m < mt) {
            const double x = ph[(int64_t)(4 * r) * a.Np + 16 * m];
#pragma unroll
            for (int j = 0; j < NI; ++j) {
              d4_t one = m1[rl][j];
              k1[m][j] = mfma_f64(x, one[r], k1[m][j]);
            }
          }
        }
    }
    // reduce over the 4 waves through LDS, one (m, j) fragment at a time
    double* out = a.K1p + (int64_t)wg * a.Np * NP;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      if (m >= mt) break;
#pragma unroll
      for (int j = 0; j < NI; ++j) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          sRed[w][lane] = k1[m][j][r];
          __syncthreads();
          if (w == 0) {
            const double s = sRed[0][lane] + sRed[1][lane] + sRed[2][lane] + sRed[3][lane];
            out[(int64_t)(16 * m + 4 * r + lq) * NP + 16 * j + l16] = s;
          }
          __syncthreads();
        }
      }
    }
  }
  // energy partial
  const double es = wave_sum(e1);
  if (lane == 0) sRed[w][0] = es;
  __syncthreads();
  if (tid == 0) a.e1p[wg] = ((sRed[0][0] + sRed[1][0]) + sRed[2][0]) + sRed[3][0];
}

__global__ void sum_partials_kernel(const double* __restrict__ in, int64_t nparts, int64_t stride,
                                    int64_t count, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  double s = 0.0;
  for (int64_t p = 0; p < nparts; ++p) s += in[p * stride + i];
  out[i] = s;
}

__global__ void pack_kernel(const double* __restrict__ C, int64_t rows, int64_t cols, int64_t ldc,
                            double* __restrict__ Cp, int64_t rows_p, int64_t ldp) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows_p * ldp) return;
  const int64_t r = t / ldp, c = t % ldp;
  Cp[t] = (r < rows && c < cols) ? C[r * ldc + c] : 0.0;
}

__global__ __launch_bounds__(256) void combine_kernel(const double* K1, const double* K2, const double* K3,
                                                     int N, int n, int np, double s1, double s2, double s3,
                                                     double dV, double* K, const double* e1p, int64_t ne1,
                                                     const double* e3p, int64_t ne3, double ce1, double ce3,
                                                     double* ex) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < (int64_t)N * n) {
    const int64_t mu = t / n, i = t % n;
    const int64_t q = mu * np + i;
    double v = 0.0;
    if (K1) v += s1 * K1[q];
    if (K2) v += s2 * K2[q];
    if (K3) v += s3 * K3[q];
    K[t] = dV * v;
  }
  if (ex && t == 0) {
    double e1 = 0.0, e3 = 0.0;
    for (int64_t p = 0; p < ne1; ++p) e1 += e1p[p];
    for (int64_t p = 0; p < ne3; ++p) e3 += e3p[p];
    *ex = -dV * (ce1 * e1 + ce3 * e3);
  }
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

template <int NI, int RT>
hipError_t launch_fused_mt(const FusedArgs& a, int blocks, hipStream_t s) {
  const int mt = a.want_k1 ? a.Np / 16 : 0;
  if (mt == 0) {
    hipLaunchKernelGGL((fused_f64_kernel<NI, RT, 0>), dim3(blocks), dim3(256), 0, s, a);
  } else if (mt <= 4) {
    hipLaunchKernelGGL((fused_f64_kernel<NI, RT, 4>), dim3(blocks), dim3(256), 0, s, a);
  } else if (mt <= 8) {
    hipLaunchKernelGGL((fused_f64_kernel<NI, RT, 8>), dim3(blocks), dim3(256), 0, s, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int NI>
hipError_t launch_fused_rt(const FusedArgs& a, int blocks, hipStream_t s) {
  switch (a.rtiles) {
    case 1: return launch_fused_mt<NI, 1>(a, blocks, s);
    case 2: return launch_fused_mt<NI, 2>(a, blocks, s);
    case 4: return launch_fused_mt<NI, 4>(a, blocks, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int fused_rblocks(const FusedArgs& a) {
  const int64_t rt = (a.R_valid + T - 1) / T;
  return (int)((rt + a.rtiles - 1) / a.rtiles);
}

hipError_t fused_exchange(const FusedArgs& a, hipStream_t s) {
  if (a.G % T != 0 || a.R % T != 0 || a.np % 16 != 0 || a.Np % 16 != 0) return hipErrorInvalidValue;
  if (a.want_k1 && a.Np / 16 > 8) return hipErrorInvalidValue;
  const int blocks = fused_rblocks(a) * a.gblocks;
  if (blocks <= 0) return hipSuccess;
  switch (a.np / 16) {
    case 1: return launch_fused_rt<1>(a, blocks, s);
    case 2: return launch_fused_rt<2>(a, blocks, s);
    case 3: return launch_fused_rt<3>(a, blocks, s);
    case 4: return launch_fused_rt<4>(a, blocks, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t sum_partials(const double* in, int64_t nparts, int64_t stride, int64_t count,
                        double* out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(sum_partials_kernel, dim3(nblk(count, 256)), dim3(256), 0, s, in, nparts, stride,
                     count, out);
  return hipGetLastError();
}

hipError_t pack_matrix(const double* C, int64_t rows, int64_t cols, int64_t ldc, double* Cp,
                       int64_t rows_p, int64_t ldp, hipStream_t s) {
  hipLaunchKernelGGL(pack_kernel, dim3(nblk(rows_p * ldp, 256)), dim3(256), 0, s, C, rows, cols, ldc,
                     Cp, rows_p, ldp);
  return hipGetLastError();
}

hipError_t combine(const double* K1, const double* K2, const double* K3, int N, int n, int np,
                   double s1, double s2, double s3, double dV, double* K,
                   const double* e1p, int64_t ne1, const double* e3p, int64_t ne3,
                   double ce1, double ce3, double* ex, hipStream_t s) {
  const int64_t cnt = (int64_t)N * n;
  hipLaunchKernelGGL(combine_kernel, dim3(nblk(cnt > 0 ? cnt : 1, 256)), dim3(256), 0, s, K1, K2, K3, N,
                     n, np, s1, s2, s3, dV, K, e1p, ne1, e3p, ne3, ce1, ce3, ex);
  return hipGetLastError();
}

}  // namespace rps
