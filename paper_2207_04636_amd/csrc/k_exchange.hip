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

#include <algorithm>
#include <type_traits>

#include "mfma.h"
#include "rps_internal.h"

namespace rps {
namespace {

constexpr int T = 64;        // R tile width; g rows are processed in 16-row subtiles
constexpr int SLAB = T + 1;  // LDS pitch of a wave's A slab (doubles)

// Dynamic LDS layout of the fused kernel (doubles):
//   slabs [NW][16][SLAB]   each wave's A = V o P for its 16 rows (wave-private)
//   sU    [T][NP+1]        U rows of the current R tile
//   sM2   [BG][NP]         M2 rows of this workgroup's g block (row owner = one wave)
template <int NW, int NI>
__host__ __device__ constexpr int64_t fused_lds_doubles(int64_t bg) {
  return (int64_t)NW * 16 * SLAB + (int64_t)T * (16 * NI + 1) + bg * 16 * NI;
}

template <int NW, int NI, int MT, bool WM2>
__global__ __launch_bounds__(NW * 64) void fused_f64_kernel(FusedArgs a) {
  constexpr int NP = 16 * NI;
  constexpr int LDU = NP + 1;
  extern __shared__ double smem[];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, lq = lane >> 4;

  // g block of this workgroup
  const int64_t gsub_total = a.G / 16;
  const int64_t gper = ((a.G / T + a.gblocks - 1) / a.gblocks) * (T / 16);   // subtiles per g block
  const int gb = blockIdx.x % a.gblocks;
  const int rb = blockIdx.x / a.gblocks;
  const int64_t gs0 = gb * gper;
  const int64_t gs1 = (gs0 + gper < gsub_total) ? gs0 + gper : gsub_total;
  const int64_t bg = gper * 16;                            // rows of sM2
  // R tiles of this workgroup
  const int64_t rtiles_valid = (a.R_valid + T - 1) / T;
  const int64_t rt0 = (int64_t)rb * a.rtiles;
  const int64_t rt1 = (rt0 + a.rtiles < rtiles_valid) ? rt0 + a.rtiles : rtiles_valid;

  double* slab = smem + (int64_t)w * 16 * SLAB;
  double* sU = smem + (int64_t)NW * 16 * SLAB;
  double* sM2 = sU + (int64_t)T * LDU;
  double* red = smem;                                      // reuses the slabs between phases

  // this wave's subtiles: gs0 + w, gs0 + w + NW, ...
  const int64_t nmy = (gs1 - gs0 > w) ? (gs1 - gs0 - w + NW - 1) / NW : 0;
  const int64_t nstep = nmy * (rt1 > rt0 ? rt1 - rt0 : 0);

  if constexpr (WM2)
    for (int64_t e = tid; e < bg * NP; e += NW * 64) sM2[e] = 0.0;

  // V fragment of step t: lane holds V[g0 + 4r + lq][R0 + 16c + l16]
  double vnext[4][4];
  // coordinates of step (ri, si): R tile rt0 + ri, this wave's si-th g subtile
  auto step_coords = [&](int64_t ri, int64_t si, int64_t& g0, int64_t& R0) {
    R0 = (rt0 + ri) * T;
    g0 = (gs0 + w + si * NW) * 16;
  };
  // U_g operands of step t: A operand of P, B operand of M1
  double ugAn[NI * 4], ugBn[4][NI];
  auto load_v = [&](int64_t ri, int64_t si) {
    int64_t g0, R0;
    step_coords(ri, si, g0, R0);
    const double* base = a.Vm + (g0 + lq) * a.ldv + R0 + l16;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double* row = base + (int64_t)(4 * r) * a.ldv;
#pragma unroll
      for (int c = 0; c < 4; ++c) vnext[r][c] = row[16 * c];
    }
    const double* ug = a.Ug + g0 * NP;
#pragma unroll
    for (int kk = 0; kk < NI * 4; ++kk) ugAn[kk] = ug[l16 * NP + 4 * kk + lq];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int j = 0; j < NI; ++j) ugBn[r][j] = ug[(4 * r + lq) * NP + 16 * j + l16];
  };
  if (nstep > 0) load_v(0, 0);

  double e1 = 0.0;
  // K1 output tiles owned by this wave: m = w, w + NW, ...  (MTW of them)
  constexpr int MTW = (MT + NW - 1) / NW > 0 ? (MT + NW - 1) / NW : 1;
  d4_t k1[MTW][NI];
#pragma unroll
  for (int mm = 0; mm < MTW; ++mm)
#pragma unroll
    for (int j = 0; j < NI; ++j) k1[mm][j] = zero_d4();
  const int mt = a.Np / 16;

  int64_t t = 0;
  for (int64_t rt = rt0; rt < rt1; ++rt) {
    const int64_t R0 = rt * T;
    __syncthreads();
    for (int e = tid; e < T * NP; e += NW * 64) sU[(e / NP) * LDU + (e % NP)] = a.Ur[R0 * NP + e];
    __syncthreads();
    d4_t m1[4][NI];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int j = 0; j < NI; ++j) m1[c][j] = zero_d4();

    for (int64_t si = 0; si < nmy; ++si, ++t) {
      const int64_t g0 = (gs0 + w + si * NW) * 16;
      double v[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) v[r][c] = vnext[r][c];
      double ugA[NI * 4], ugB[4][NI];
#pragma unroll
      for (int kk = 0; kk < NI * 4; ++kk) ugA[kk] = ugAn[kk];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int j = 0; j < NI; ++j) ugB[r][j] = ugBn[r][j];
      if (t + 1 < nstep) load_v(si + 1 < nmy ? rt - rt0 : rt - rt0 + 1, si + 1 < nmy ? si + 1 : 0);

      // P[g][R] = sum_k U_g[g][k] U[R][k]
      d4_t p[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) p[c] = zero_d4();
#pragma unroll
      for (int kk = 0; kk < NI * 4; ++kk)
#pragma unroll
        for (int c = 0; c < 4; ++c) p[c] = mfma_f64(ugA[kk], sU[(16 * c + l16) * LDU + 4 * kk + lq], p[c]);
      // A = V o P; energy; M1^T from the registers (reg r is the k-slice g = 4r + lq)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        d4_t av;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          av[r] = v[r][c] * p[c][r];
          if constexpr (!WM2) e1 += av[r] * p[c][r];   // fit-fit line: no M2 to form it from
          slab[(4 * r + lq) * SLAB + 16 * c + l16] = av[r];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int j = 0; j < NI; ++j) m1[c][j] = mfma_f64(av[r], ugB[r][j], m1[c][j]);
      }
      __builtin_amdgcn_wave_barrier();
      if constexpr (WM2) {
        // M2[g][i] = sum_R A[g][R] U[R][i]: A operand from the wave's own slab
        d4_t m2[NI];
#pragma unroll
        for (int j = 0; j < NI; ++j) m2[j] = zero_d4();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
          const double x = slab[l16 * SLAB + 4 * kk + lq];
#pragma unroll
          for (int j = 0; j < NI; ++j) m2[j] = mfma_f64(x, sU[(4 * kk + lq) * LDU + 16 * j + l16], m2[j]);
        }
        double* acc = sM2 + (g0 - gs0 * 16) * NP + l16;
#pragma unroll
        for (int j = 0; j < NI; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[(4 * r + lq) * NP + 16 * j] += m2[j][r];
      }
      __builtin_amdgcn_wave_barrier();
    }

    // M1^T of this R tile summed over the waves (fixed order) into LDS, then
    // K1 += Phi[R tile]^T M1^T with each wave owning whole K1 output tiles.
    if (MT > 0 || a.want_m1) {
      double* m1s = sU;                       // the U tile is not needed until the next R tile
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
          for (int r = 0; r < 4; ++r) red[(w * 64 + 16 * c + 4 * r + lq) * 16 + l16] = m1[c][j][r];
        __syncthreads();
        if (w < 4) {
          const int q = w;   // R subtile
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            double s = 0.0;
            for (int ww = 0; ww < NW; ++ww) s += red[(ww * 64 + 16 * q + 4 * r + lq) * 16 + l16];
            m1s[(16 * q + 4 * r + lq) * 16 + l16] = s;
            if (a.want_m1) a.M1T[((int64_t)gb * a.R + R0 + 16 * q + 4 * r + lq) * NP + 16 * j + l16] = s;
          }
        }
        __syncthreads();
        if (MT > 0 && a.want_k1) {
          // slice (q, r) <-> R = R0 + 16q + 4r + lq
#pragma unroll
          for (int mm = 0; mm < MTW; ++mm) {
            const int m = w + mm * NW;
            if (m < mt) {
              const double* ph = a.Phir + (R0 + lq) * a.Np + 16 * m + l16;
#pragma unroll
              for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                  k1[mm][j] = mfma_f64(ph[(int64_t)(16 * q + 4 * r) * a.Np], m1s[(16 * q + 4 * r + lq) * 16 + l16],
                                       k1[mm][j]);
            }
          }
        }
      }
    }
  }

  const int wg = blockIdx.x;
  __syncthreads();
  if (MT > 0 && a.want_k1) {
    double* out = a.K1p + (int64_t)wg * a.Np * NP;
#pragma unroll
    for (int mm = 0; mm < MTW; ++mm) {
      const int m = w + mm * NW;
      if (m < mt)
#pragma unroll
        for (int j = 0; j < NI; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) out[(int64_t)(16 * m + 4 * r + lq) * NP + 16 * j + l16] = k1[mm][j][r];
    }
  }
  if constexpr (WM2) {
    double* out = a.M2p + ((int64_t)rb * a.G + gs0 * 16) * NP;
    const int64_t rows = (gs1 - gs0) * 16;
    for (int64_t e = tid; e < rows * NP; e += NW * 64) out[e] = sM2[e];
  }
  // energy partial (fit-fit line): waves in fixed order
  if constexpr (!WM2) {
    const double es = wave_sum(e1);
    __syncthreads();
    if (lane == 0) red[w] = es;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int ww = 0; ww < NW; ++ww) s += red[ww];
      a.e1p[wg] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// n <= 16 variant on v_mfma_f64_4x4x4_f64 (4 blocks).  On gfx950 this
// instruction sustains nearly the FP64 peak while the 16x16x4 form does not.
// With lane l, q = l / 16, c4 = l % 4, b = (l / 4) % 4 (the block):
//   A_b[c4][q], B_b[q][c4] -> D_b[q][c4].
// Two views of one instruction are used:
//   shared A (4 x 16 output): A[l%4][l/16], B[l/16][l%16] -> D[l/16][l%16]
//   shared B (16 x 4 output): A[l%16][l/16], B[l/16][l%4] -> D[4b + l/16][l%4]
// P = U_g U^T uses the first (rows g, columns R, k = orbital): its fragment
// P[g0 + 4 gq + l/16][R0 + 16c + l%16] is the same as the 16x16 layout, so the
// V fragment and the wave's A slab are unchanged.  M1^T = A^T U_g uses the
// second with A^T taken straight from those registers (k = 4 rows of g).  M2 =
// A U uses the second with A read transposed from the wave's slab.
// Orbital operands are read from a permuted copy [row][i % 4][i / 4] so that
// the four k slices a lane needs are contiguous.
__device__ __forceinline__ double mfma4(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

template <int NW, int MT, int M2MODE>
__global__ __launch_bounds__(NW * 64) void fused_m4_kernel(FusedArgs a) {
  constexpr int NP = 16;
  constexpr int LDP = 18;               // pitch of the permuted U tile rows (doubles, 16-byte aligned)
  extern __shared__ double smem[];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, lq = lane >> 4, c4 = lane & 3, bq = (lane >> 2) & 3;

  const int64_t gsub_total = a.G / 16;
  const int64_t gper = ((a.G / T + a.gblocks - 1) / a.gblocks) * (T / 16);
  const int gb = blockIdx.x % a.gblocks;
  const int rb = blockIdx.x / a.gblocks;
  const int64_t gs0 = gb * gper;
  const int64_t gs1 = (gs0 + gper < gsub_total) ? gs0 + gper : gsub_total;
  const int64_t bg = gper * 16;
  const int64_t rtiles_valid = (a.R_valid + T - 1) / T;
  const int64_t rt0 = (int64_t)rb * a.rtiles;
  const int64_t rt1 = (rt0 + a.rtiles < rtiles_valid) ? rt0 + a.rtiles : rtiles_valid;

  double* slab = smem + (int64_t)w * 16 * SLAB;
  double* sU = smem + (int64_t)NW * 16 * SLAB;          // [T][LDP] permuted: [R][j4*4 + ich]
  double* sM2 = sU + (int64_t)T * LDP;                   // [bg][NP]
  double* red = smem;

  const int64_t nmy = (gs1 - gs0 > w) ? (gs1 - gs0 - w + NW - 1) / NW : 0;
  const int64_t nstep = nmy * (rt1 > rt0 ? rt1 - rt0 : 0);
  if (a.want_m2)
    for (int64_t e = tid; e < bg * NP; e += NW * 64) sM2[e] = 0.0;

  double vnext[4][4];
  auto load_v = [&](int64_t ri, int64_t si) {
    const int64_t R0 = (rt0 + ri) * T, g0 = (gs0 + w + si * NW) * 16;
    const double* base = a.Vm + (g0 + lq) * a.ldv + R0 + l16;
#pragma unroll
    for (int gq = 0; gq < 4; ++gq) {
      const double* row = base + (int64_t)(4 * gq) * a.ldv;
#pragma unroll
      for (int c = 0; c < 4; ++c) vnext[gq][c] = row[16 * c];
    }
  };
  if (nstep > 0) load_v(0, 0);

  double e1 = 0.0;
  constexpr int MTW = (MT + NW - 1) / NW > 0 ? (MT + NW - 1) / NW : 1;
  d4_t k1[MTW];
#pragma unroll
  for (int mm = 0; mm < MTW; ++mm) k1[mm] = zero_d4();
  const int mt = a.Np / 16;

  int64_t t = 0;
  for (int64_t rt = rt0; rt < rt1; ++rt) {
    const int64_t R0 = rt * T;
    __syncthreads();
    // U tile, permuted: sU[R][(i % 4) * 4 + i / 4] = U[R0 + R][i]
    for (int e = tid; e < T * NP; e += NW * 64) {
      const int r = e / NP, i = e % NP;
      sU[r * LDP + (i & 3) * 4 + (i >> 2)] = a.Ur[(R0 + r) * NP + i];
    }
    __syncthreads();
    double m1[4][4];                       // [c][ich]: M1^T[R0 + 16c + 4bq + lq][4 ich + c4]
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int k = 0; k < 4; ++k) m1[c][k] = 0.0;

    for (int64_t si = 0; si < nmy; ++si, ++t) {
      const int64_t g0 = (gs0 + w + si * NW) * 16;
      double v[4][4];
#pragma unroll
      for (int gq = 0; gq < 4; ++gq)
#pragma unroll
        for (int c = 0; c < 4; ++c) v[gq][c] = vnext[gq][c];
      if (t + 1 < nstep) load_v(si + 1 < nmy ? rt - rt0 : rt - rt0 + 1, si + 1 < nmy ? si + 1 : 0);
      const double* ugp = a.Ugp + g0 * NP;   // permuted U_g rows of this subtile
      double pA[4][4];                      // P A operand: U_g[g0 + 4gq + c4][4kk + lq] = ugp[.. + lq*4 + kk]
      double mB[4][4];                      // M1 B operand: U_g[g0 + 4gq + lq][4ich + c4] = ugp[.. + c4*4 + ich]
#pragma unroll
      for (int gq = 0; gq < 4; ++gq) {
        const double2* x = reinterpret_cast<const double2*>(ugp + (4 * gq + c4) * NP + lq * 4);
        const double2 x0 = x[0], x1 = x[1];
        pA[gq][0] = x0.x; pA[gq][1] = x0.y; pA[gq][2] = x1.x; pA[gq][3] = x1.y;
        const double2* y = reinterpret_cast<const double2*>(ugp + (4 * gq + lq) * NP + c4 * 4);
        const double2 y0 = y[0], y1 = y[1];
        mB[gq][0] = y0.x; mB[gq][1] = y0.y; mB[gq][2] = y1.x; mB[gq][3] = y1.y;
      }
      // P[g0 + 4gq + lq][R0 + 16c + l16] = sum_k U_g[g][k] U[R][k]  (shared-A view)
      double p[4][4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double2* u = reinterpret_cast<const double2*>(sU + (16 * c + l16) * LDP + lq * 4);
        const double2 u0 = u[0], u1 = u[1];
        const double ub[4] = {u0.x, u0.y, u1.x, u1.y};     // U[R][4kk + lq]
#pragma unroll
        for (int gq = 0; gq < 4; ++gq) {
          double acc = 0.0;
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) acc = mfma4(pA[gq][kk], ub[kk], acc);
          p[gq][c] = acc;
        }
      }
      // A = V o P, energy, slab; M1^T[R][i] += sum_g A^T[R][g] U_g[g][i]  (shared-B view)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
#pragma unroll
        for (int gq = 0; gq < 4; ++gq) {
          const double av = v[gq][c] * p[gq][c];
          e1 += av * p[gq][c];
          slab[(4 * gq + lq) * SLAB + 16 * c + l16] = av;
#pragma unroll
          for (int ich = 0; ich < 4; ++ich) m1[c][ich] = mfma4(av, mB[gq][ich], m1[c][ich]);
        }
      }
      __builtin_amdgcn_wave_barrier();
      if (a.want_m2) {
        if (M2MODE == 0) {
          // M2[g0 + 4bq + lq][4 ich + c4] += sum_R A[g][R] U[R][i]  (shared-B view, A^T from the slab);
          // four partial chains per output (R slices s % 4) for independent MFMAs
          double m2[4][4];
#pragma unroll
          for (int ich = 0; ich < 4; ++ich)
#pragma unroll
            for (int h = 0; h < 4; ++h) m2[ich][h] = 0.0;
#pragma unroll
          for (int s = 0; s < 16; ++s) {
            const double x = slab[l16 * SLAB + 4 * s + lq];
            const double2* u = reinterpret_cast<const double2*>(sU + (4 * s + lq) * LDP + c4 * 4);
            const double2 u0 = u[0], u1 = u[1];
            m2[0][s & 3] = mfma4(x, u0.x, m2[0][s & 3]);
            m2[1][s & 3] = mfma4(x, u0.y, m2[1][s & 3]);
            m2[2][s & 3] = mfma4(x, u1.x, m2[2][s & 3]);
            m2[3][s & 3] = mfma4(x, u1.y, m2[3][s & 3]);
          }
          double* acc = sM2 + (g0 - gs0 * 16 + 4 * bq + lq) * NP + c4;
#pragma unroll
          for (int ich = 0; ich < 4; ++ich)
            acc[4 * ich] += (m2[ich][0] + m2[ich][1]) + (m2[ich][2] + m2[ich][3]);
        } else {
          // 16x16x4 form: D[g][i] += A[g][R] U[R][i], A from the slab, U (unpermuted index) from the tile
          d4_t m2 = zero_d4();
#pragma unroll
          for (int s = 0; s < 16; ++s) {
            const double x = slab[l16 * SLAB + 4 * s + lq];
            m2 = mfma_f64(x, sU[(4 * s + lq) * LDP + (l16 & 3) * 4 + (l16 >> 2)], m2);
          }
          double* acc = sM2 + (g0 - gs0 * 16 + lq) * NP + l16;
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[4 * r * NP] += m2[r];
        }
      }
      __builtin_amdgcn_wave_barrier();
    }

    if (MT > 0 || a.want_m1) {
      double* m1s = sU;
      __syncthreads();
      // wave w's partial M1^T -> red[w][R][i]
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int ich = 0; ich < 4; ++ich)
          red[(w * 64 + 16 * c + 4 * bq + lq) * 16 + 4 * ich + c4] = m1[c][ich];
      __syncthreads();
      if (w < 4) {
        const int q = w;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          double s = 0.0;
          for (int ww = 0; ww < NW; ++ww) s += red[(ww * 64 + 16 * q + 4 * r + lq) * 16 + l16];
          m1s[(16 * q + 4 * r + lq) * 16 + l16] = s;
          if (a.want_m1) a.M1T[((int64_t)gb * a.R + R0 + 16 * q + 4 * r + lq) * NP + l16] = s;
        }
      }
      __syncthreads();
      if (MT > 0 && a.want_k1) {
#pragma unroll
        for (int mm = 0; mm < MTW; ++mm) {
          const int m = w + mm * NW;
          if (m < mt) {
            const double* ph = a.Phir + (R0 + lq) * a.Np + 16 * m + l16;
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
              for (int r = 0; r < 4; ++r)
                k1[mm] = mfma_f64(ph[(int64_t)(16 * q + 4 * r) * a.Np], m1s[(16 * q + 4 * r + lq) * 16 + l16], k1[mm]);
          }
        }
      }
    }
  }

  const int wg = blockIdx.x;
  __syncthreads();
  if (MT > 0 && a.want_k1) {
    double* out = a.K1p + (int64_t)wg * a.Np * NP;
#pragma unroll
    for (int mm = 0; mm < MTW; ++mm) {
      const int m = w + mm * NW;
      if (m < mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) out[(int64_t)(16 * m + 4 * r + lq) * NP + l16] = k1[mm][r];
    }
  }
  if (a.want_m2) {
    double* out = a.M2p + ((int64_t)rb * a.G + gs0 * 16) * NP;
    const int64_t rows = (gs1 - gs0) * 16;
    for (int64_t e = tid; e < rows * NP; e += NW * 64) out[e] = sM2[e];
  }
  const double es = wave_sum(e1);
  __syncthreads();
  if (lane == 0) red[w] = es;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int ww = 0; ww < NW; ++ww) s += red[ww];
    a.e1p[wg] = s;
  }
}

// ---------------------------------------------------------------------------
// Precision form, n <= 16: V stored in FP32, the in-tile products on the FP32
// matrix cores (v_mfma_f32_16x16x4_f32) with FP32 accumulation inside a tile,
// FP64 accumulation across tiles (M2 in the LDS accumulators, M1 when the waves'
// partials are combined, K1 and the energy in FP64).  Same structure as the
// FP64 kernel; the FP32 fragment layout has rows 4*(l/16) + r, so the V
// fragment and the k-slices of the M1 product follow that layout.
template <int NW, int MT>
__global__ __launch_bounds__(NW * 64) void fused_f32_kernel(FusedArgs a) {
  constexpr int NP = 16;
  constexpr int LDU = NP + 1;
  constexpr int SL = T + 4;                // FP32 slab pitch (floats): conflict-free rows for both access patterns
  extern __shared__ double smem[];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, lq = lane >> 4;

  const int64_t gsub_total = a.G / 16;
  const int64_t gper = ((a.G / T + a.gblocks - 1) / a.gblocks) * (T / 16);
  const int gb = blockIdx.x % a.gblocks;
  const int rb = blockIdx.x / a.gblocks;
  const int64_t gs0 = gb * gper;
  const int64_t gs1 = (gs0 + gper < gsub_total) ? gs0 + gper : gsub_total;
  const int64_t bg = gper * 16;
  const int64_t rtiles_valid = (a.R_valid + T - 1) / T;
  const int64_t rt0 = (int64_t)rb * a.rtiles;
  const int64_t rt1 = (rt0 + a.rtiles < rtiles_valid) ? rt0 + a.rtiles : rtiles_valid;

  // layout (doubles): slabs NW*16*SLAB (holds the FP32 slabs and the reduction area),
  // sU [T][LDU] (FP32 copy in the first half), sM2 [bg][NP] FP64
  float* slab = reinterpret_cast<float*>(smem + (int64_t)w * 16 * SLAB);
  double* red = smem;
  float* sU = reinterpret_cast<float*>(smem + (int64_t)NW * 16 * SLAB);
  double* m1s = smem + (int64_t)NW * 16 * SLAB;          // reuses the sU area between R tiles
  double* sM2 = smem + (int64_t)NW * 16 * SLAB + (int64_t)T * LDU;

  const int64_t nmy = (gs1 - gs0 > w) ? (gs1 - gs0 - w + NW - 1) / NW : 0;
  const int64_t nstep = nmy * (rt1 > rt0 ? rt1 - rt0 : 0);
  if (a.want_m2)
    for (int64_t e = tid; e < bg * NP; e += NW * 64) sM2[e] = 0.0;

  // V fragment: lane holds V[g0 + 4lq + r][R0 + 16c + l16]; U_g operands of the
  // step are prefetched in FP64 and rounded when used (a conversion right after
  // the load would wait for the whole prefetch)
  float vnext[4][4];
  double ugAn[4], ugBn[4];
  auto load_v = [&](int64_t ri, int64_t si) {
    const int64_t R0 = (rt0 + ri) * T, g0 = (gs0 + w + si * NW) * 16;
    const float* base = a.Vm32 + (g0 + 4 * lq) * a.ldv + R0 + l16;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float* row = base + (int64_t)r * a.ldv;
#pragma unroll
      for (int c = 0; c < 4; ++c) vnext[r][c] = row[16 * c];
    }
    const double* ug = a.Ug + g0 * NP;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) ugAn[kk] = ug[l16 * NP + 4 * kk + lq];
#pragma unroll
    for (int r = 0; r < 4; ++r) ugBn[r] = ug[(4 * lq + r) * NP + l16];
  };
  if (nstep > 0) load_v(0, 0);

  constexpr int MTW = (MT + NW - 1) / NW > 0 ? (MT + NW - 1) / NW : 1;
  d4_t k1[MTW];
#pragma unroll
  for (int mm = 0; mm < MTW; ++mm) k1[mm] = zero_d4();
  const int mt = a.Np / 16;

  int64_t t = 0;
  for (int64_t rt = rt0; rt < rt1; ++rt) {
    const int64_t R0 = rt * T;
    __syncthreads();
    for (int e = tid; e < T * NP; e += NW * 64) sU[(e / NP) * LDU + (e % NP)] = (float)a.Ur[R0 * NP + e];
    __syncthreads();
    f4_t m1[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) m1[c] = zero_f4();

    for (int64_t si = 0; si < nmy; ++si, ++t) {
      const int64_t g0 = (gs0 + w + si * NW) * 16;
      float v[4][4], ugA[4], ugB[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        ugA[r] = (float)ugAn[r];
        ugB[r] = (float)ugBn[r];
#pragma unroll
        for (int c = 0; c < 4; ++c) v[r][c] = vnext[r][c];
      }
      if (t + 1 < nstep) load_v(si + 1 < nmy ? rt - rt0 : rt - rt0 + 1, si + 1 < nmy ? si + 1 : 0);
      // P[g0 + 4lq + r][R0 + 16c + l16]
      f4_t p[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) p[c] = zero_f4();
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
#pragma unroll
        for (int c = 0; c < 4; ++c) p[c] = mfma_f32(ugA[kk], sU[(16 * c + l16) * LDU + 4 * kk + lq], p[c]);
      // A = V o P; slab; M1^T from the registers (slice r <-> g = 4lq + r).  The
      // energy term sum A o P is formed afterwards as tr(U_g^T M2).
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        f4_t av;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          av[r] = v[r][c] * p[c][r];
          slab[(4 * lq + r) * SL + 16 * c + l16] = av[r];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) m1[c] = mfma_f32(av[r], ugB[r], m1[c]);
      }
      __builtin_amdgcn_wave_barrier();
      if (a.want_m2) {
        f4_t m2 = zero_f4();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk)
          m2 = mfma_f32(slab[l16 * SL + 4 * kk + lq], sU[(4 * kk + lq) * LDU + l16], m2);
        double* acc = sM2 + (g0 - gs0 * 16 + 4 * lq) * NP + l16;
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r * NP] += (double)m2[r];
      }
      __builtin_amdgcn_wave_barrier();
    }

    if (MT > 0 || a.want_m1) {
      __syncthreads();
      // wave w's partial M1^T[R0 + 16c + 4lq + r][l16] -> red (FP64)
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[(w * 64 + 16 * c + 4 * lq + r) * 16 + l16] = (double)m1[c][r];
      __syncthreads();
      if (w < 4) {
        const int q = w;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          double s = 0.0;
          for (int ww = 0; ww < NW; ++ww) s += red[(ww * 64 + 16 * q + 4 * r + lq) * 16 + l16];
          m1s[(16 * q + 4 * r + lq) * 16 + l16] = s;
          if (a.want_m1) a.M1T[((int64_t)gb * a.R + R0 + 16 * q + 4 * r + lq) * NP + l16] = s;
        }
      }
      __syncthreads();
      if (MT > 0 && a.want_k1) {
#pragma unroll
        for (int mm = 0; mm < MTW; ++mm) {
          const int m = w + mm * NW;
          if (m < mt) {
            const double* ph = a.Phir + (R0 + lq) * a.Np + 16 * m + l16;
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
              for (int r = 0; r < 4; ++r)
                k1[mm] = mfma_f64(ph[(int64_t)(16 * q + 4 * r) * a.Np], m1s[(16 * q + 4 * r + lq) * 16 + l16], k1[mm]);
          }
        }
      }
    }
  }

  const int wg = blockIdx.x;
  __syncthreads();
  if (MT > 0 && a.want_k1) {
    double* out = a.K1p + (int64_t)wg * a.Np * NP;
#pragma unroll
    for (int mm = 0; mm < MTW; ++mm) {
      const int m = w + mm * NW;
      if (m < mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) out[(int64_t)(16 * m + 4 * r + lq) * NP + l16] = k1[mm][r];
    }
  }
  if (a.want_m2) {
    double* out = a.M2p + ((int64_t)rb * a.G + gs0 * 16) * NP;
    const int64_t rows = (gs1 - gs0) * 16;
    for (int64_t e = tid; e < rows * NP; e += NW * 64) out[e] = sM2[e];
  }
}

// Precision form, n <= 16, with the orbitals formed tile by tile in the kernel.
// Per R tile (64 grid rows) the FP32 basis rows are staged in LDS once and serve
// both ends of the tile:
//   start: U = Phi C on the FP32 matrix cores (FP32 basis values, C rounded to
//          FP32), the in-tile operand of the products below;
//   end:   the eight waves' M1 partials summed in FP32, K1_tile = Phi^T M1^T on
//          the FP32 matrix cores, added to an FP64 sum over the tiles.
// The orbitals therefore never leave the chip and the basis is read once per
// build in FP32.  Other choices, all for the latency of the V stream:
//  * every wave steps through NMY g subtiles per tile (the workgroup's block of
//    g rows split over 8 waves; a wave with fewer subtiles idles on the rest),
//    so the double buffer of V fragments has a fixed parity per step and V is
//    requested two steps ahead (tiles are processed in pairs for that);
//  * inside a tile, position p = 16 c + j of the 64 columns is grid row
//    R0 + 4 j + c, so a lane's four V values of a row are one 16-byte load;
//  * U_g rows of the workgroup sit in LDS in FP32; M2 accumulates in FP64
//    registers; the U operands of the tile's products sit in registers.
// NW = 8 waves; Np <= 128.
template <int NMY>
__global__ __launch_bounds__(512) void fused_f32u_kernel(FusedArgs a) {
  constexpr int NW = 8;
  constexpr int NP = 16;
  constexpr int LDU = NP + 1;              // sU pitch (floats): rows 4 j + c read across j
  constexpr int LDM = NP + 4;              // sU2 / sUg pitch: rows 4 lq + r read across lq
  constexpr int RP = NP + 1;               // M1 partial pitch
  constexpr int SL = T + 4;                // FP32 slab pitch (floats)
  extern __shared__ double smem[];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, lq = lane >> 4;
  const int Np = a.Np, PP = Np + 4;

  const int64_t gsub_total = a.G / 16;
  const int64_t gper = ((a.G / T + a.gblocks - 1) / a.gblocks) * (T / 16);
  const int gb = blockIdx.x % a.gblocks;
  const int rb = blockIdx.x / a.gblocks;
  const int64_t gs0 = gb * gper;
  const int64_t gs1 = (gs0 + gper < gsub_total) ? gs0 + gper : gsub_total;
  const int64_t rtiles_valid = (a.R_valid + T - 1) / T;
  const int64_t rt0 = (int64_t)rb * a.rtiles;
  const int64_t rt1 = (rt0 + a.rtiles < rtiles_valid) ? rt0 + a.rtiles : rtiles_valid;

  // LDS (bytes): area0 | sPhi [T][PP] f32 | sC [Np][16] f64 | m1s [T][16] f64 | sU [T][LDU] f32
  //              | sU2 [T][LDM] f32 | sUg [gper*16][LDM] f32
  // area0 holds, one after another within a tile: the waves' A slabs [NW][16][SL] f32,
  // the M1 partials [NW][T][RP] f32.  The pitches keep the lanes of each access pattern
  // on distinct banks.
  constexpr int AREA0 = NW * 16 * SL * 4;
  char* base = reinterpret_cast<char*>(smem);
  float* slab = reinterpret_cast<float*>(base) + w * 16 * SL;
  float* red = reinterpret_cast<float*>(base);
  float* sPhi = reinterpret_cast<float*>(base + AREA0);
  double* sC = reinterpret_cast<double*>(base + AREA0 + (int64_t)T * PP * 4);
  double* m1s = sC + Np * NP;
  float* sU = reinterpret_cast<float*>(m1s + T * NP);
  float* sU2 = sU + T * LDU;
  float* sUg = sU2 + T * LDM;

  const int nmy = (gs1 - gs0 > w) ? (int)((gs1 - gs0 - w + NW - 1) / NW) : 0;   // <= NMY (host check)

  // operands of this wave's first fit-fit unit (see below), requested before anything else
  const int64_t nsub3 = a.Wl ? a.G / 16 : 0, n3 = nsub3 * nsub3;
  int64_t u3 = (int64_t)blockIdx.x * NW + w;
  double l3ha[4], l3ya[4], l3w[4], l3hb[4], l3yr[4];
  auto l3_load = [&](int64_t u) {
    const int64_t y0 = (u / nsub3) * 16, h0 = (u % nsub3) * 16;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      l3ha[q] = a.Ug[(h0 + l16) * NP + 4 * q + lq];
      l3ya[q] = a.Ug[(y0 + l16) * NP + 4 * q + lq];
      l3w[q] = a.Wl[(h0 + 4 * q + lq) * a.ldw + y0 + l16];
      l3hb[q] = a.Ug[(h0 + 4 * q + lq) * NP + l16];
      l3yr[q] = a.Ug[(y0 + 4 * q + lq) * NP + l16];
    }
  };
  if (u3 < n3) l3_load(u3);

  // staging loops unrolled so that their global loads are in flight together
  float* sCf = reinterpret_cast<float*>(sC);   // C rounded to FP32 (first half of its area)
#pragma unroll 4
  for (int e = tid; e < Np * NP; e += NW * 64) {
    const int r = e / NP, c = e % NP;
    sCf[e] = (r < a.N && c < a.n) ? (float)a.Cm[(int64_t)r * a.n + c] : 0.0f;
  }
  {
    // U_g rows of the workgroup, two doubles per load
    const double2* ug2 = reinterpret_cast<const double2*>(a.Ug + gs0 * 16 * NP);
    const int n2 = (int)((gs1 - gs0) * 16 * NP / 2);
#pragma unroll 8
    for (int e = tid; e < n2; e += NW * 64) {
      const double2 v = ug2[e];
      float* d = sUg + ((2 * e) / NP) * LDM + (2 * e) % NP;
      d[0] = (float)v.x;
      d[1] = (float)v.y;
    }
  }

  // V fragment of step (tile rt, subtile si): lane holds V[g0 + 4lq + r][R0 + 4 l16 + c]
  float vb[2][4][4];
  // Loads are issued unconditionally (a step that does not exist re-reads V row 0 of
  // the first tile), so that the wait before each use counts only older loads.
  auto load_v = [&](float (&dst)[4][4], int64_t rt, int si) {
    const bool ok = rt < rt1 && si < nmy;
    const int64_t R0 = (ok ? rt : rt0) * T, g0 = ok ? (gs0 + w + (int64_t)si * NW) * 16 : 0;
    const float* src = a.Vm32 + (g0 + 4 * lq) * a.ldv + R0 + 4 * l16;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float4 q = *reinterpret_cast<const float4*>(src + (int64_t)r * a.ldv);
      dst[r][0] = q.x; dst[r][1] = q.y; dst[r][2] = q.z; dst[r][3] = q.w;
    }
  };
  double m2acc[NMY][4];
#pragma unroll
  for (int si = 0; si < NMY; ++si)
#pragma unroll
    for (int r = 0; r < 4; ++r) m2acc[si][r] = 0.0;
  double k1[4] = {0.0, 0.0, 0.0, 0.0};   // K1[16 w + 4 lq + r][l16], summed over the tiles in FP64
  const int mt = Np / 16;

  // Basis rows of a tile (T x Np floats, contiguous): float4 piece q = tid + 512 j of
  // the tile goes to sPhi row q / (Np/4), column 4 (q % (Np/4)).  The next tile's
  // pieces are requested into registers while the current tile runs.
  constexpr int PFJ = 4;                   // pieces per thread: T * 128 / 4 / 512
  const int nq = Np / 4;
  static_assert(PFJ == 4, "four named prefetch registers");
  // pieces past the tile go to the pad columns [Np, Np + 4) of a row (never read), so
  // that every store is unconditional and the wait before it counts the loads exactly
  auto lds_of = [&](int j) {
    const int q = tid + 512 * j;
    return (q < T * nq) ? (q / nq) * PP + 4 * (q % nq) : (tid & 63) * PP + Np;
  };
  const int pl0 = lds_of(0), pl1 = lds_of(1), pl2 = lds_of(2), pl3 = lds_of(3);
  // named registers, not an array: an array captured by the lambdas ends up in scratch
  float4 pf0, pf1, pf2, pf3;
  const int qlast = T * nq - 1;
  auto fetch_phi = [&](int64_t rt) {
    // unconditional loads (pieces past the tile re-read its last one)
    const float4* src = reinterpret_cast<const float4*>(a.Phi32 + rt * T * Np);
    pf0 = src[min(tid, qlast)];
    pf1 = src[min(tid + 512, qlast)];
    pf2 = src[min(tid + 1024, qlast)];
    pf3 = src[min(tid + 1536, qlast)];
  };
  // The first tile's basis rows go out before its first two V fragments: at the head
  // of the tile loop the basis registers are then older than the last eight loads on
  // every path into it (as after a tile, where the next tile's first two fragments are
  // the most recent loads), so the wait for them never waits for V.
  fetch_phi(rt0);
#pragma unroll
  for (int s = 0; s < 2; ++s) load_v(vb[s & 1], rt0 + s / NMY, s % NMY);

  // Fit-fit line (Eq. 16 line 3), folded in while the first loads are in flight.  Unit
  // (ys, hc) = one 16 x 16 block of B = W o P_g times U_g rows hc: P_g^T is formed for
  // the h rows of the unit (W is symmetric, so W o P_g^T is B^T), and its registers feed
  // the product directly.  Units go round-robin over all waves of the grid, FP64; the
  // operands of a wave's first unit were requested at the top of the kernel.
  for (; u3 < n3; u3 += (int64_t)gridDim.x * NW) {
    const int64_t ys = u3 / nsub3, hc = u3 % nsub3;
    const int64_t y0 = ys * 16;
    d4_t pt = zero_d4();    // P_g^T[h0 + 4r + lq][y0 + l16]
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) pt = mfma_f64(l3ha[kk], l3ya[kk], pt);
    d4_t yacc = zero_d4();  // Y[y0 + 4r + lq][l16], this unit's part
#pragma unroll
    for (int r = 0; r < 4; ++r) yacc = mfma_f64(l3w[r] * pt[r], l3hb[r], yacc);
    double* yo = a.Yneg + (hc * a.G + y0) * NP;
    double e = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      yo[(4 * r + lq) * NP + l16] = -yacc[r];
      e += l3yr[r] * yacc[r];
    }
    e = wave_sum(e);
    if (lane == 0) a.e3u[u3] = e;
    if (u3 + (int64_t)gridDim.x * NW < n3) l3_load(u3 + (int64_t)gridDim.x * NW);
  }

  auto tile = [&](auto tau, int64_t rt) {
    constexpr int TAU = decltype(tau)::value;
    __syncthreads();   // the previous tile is done with sPhi, m1s and area0
    *reinterpret_cast<float4*>(sPhi + pl0) = pf0;
    *reinterpret_cast<float4*>(sPhi + pl1) = pf1;
    *reinterpret_cast<float4*>(sPhi + pl2) = pf2;
    *reinterpret_cast<float4*>(sPhi + pl3) = pf3;
    __syncthreads();
    fetch_phi(rt + 1 < rt1 ? rt + 1 : rt);   // unconditional (the last tile re-reads itself)
    if (w < 4) {
      // U rows 16 w .. 16 w + 15 over all basis functions on the FP32 matrix cores (two
      // accumulator chains, C rounded to FP32), straight into sU / sU2.  Waves 4-7 have no
      // share: split over eight waves the halves would need a sum through LDS and one more
      // barrier, while the matrix cores of each SIMD do the same work either way.
      const int ksteps = Np / 4;             // even, since Np % 16 == 0
      const float* pa = sPhi + (16 * w + l16) * PP + lq;
      const float* pb = sCf + lq * NP + l16;
      f4_t acc0 = zero_f4(), acc1 = zero_f4();
#pragma unroll 4
      for (int kk = 0; kk < ksteps; kk += 2) {
        acc0 = mfma_f32(pa[4 * kk], pb[4 * kk * NP], acc0);
        acc1 = mfma_f32(pa[4 * kk + 4], pb[(4 * kk + 4) * NP], acc1);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * w + 4 * lq + r;
        const float u = acc0[r] + acc1[r];
        sU[row * LDU + l16] = u;
        sU2[row * LDM + l16] = u;
      }
    }
    __syncthreads();
    // U operands of the tile's products (column position p = 16 c + j is row 4 j + c):
    // P = U_g U^T: B[k = i][n = p]; M2 = A U: B[k = p][n = i], in registers when room
    constexpr bool BMREG = (NMY <= 5);
    float bP[4][4], bM[16];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int c = 0; c < 4; ++c) bP[kk][c] = sU[(4 * l16 + c) * LDU + 4 * kk + lq];
    auto bm_row = [&](int kk) { return 4 * ((4 * kk + lq) & 15) + (kk >> 2); };
    if (BMREG)
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) bM[kk] = sU2[bm_row(kk) * LDM + l16];

    f4_t m1[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) m1[c] = zero_f4();

#pragma unroll
    for (int si = 0; si < NMY; ++si) {
      const int b = (TAU * NMY + si) & 1;
      float (&v)[4][4] = vb[b];
      if (si < nmy) {
        const int gl = (w + si * NW) * 16;     // local row of the subtile in sUg
        float ugA[4], ugB[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) ugA[kk] = sUg[(gl + l16) * LDM + 4 * kk + lq];
#pragma unroll
        for (int r = 0; r < 4; ++r) ugB[r] = sUg[(gl + 4 * lq + r) * LDM + l16];
        f4_t p[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) p[c] = zero_f4();
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
          for (int c = 0; c < 4; ++c) p[c] = mfma_f32(ugA[kk], bP[kk][c], p[c]);
        // A to the slab, arranged for the M2 operand: row g holds position p = 4 kk + q
        // at chunk (q, kk / 4) of four floats, chunk index XORed with (g / 4) % 4 in its
        // low bits (conflict-free writes; each reader lane gets four 16-byte chunks)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          f4_t av;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            av[r] = v[r][c] * p[c][r];
            slab[(4 * lq + r) * SL + 4 * ((l16 & 3) * 4 + (c ^ lq)) + (l16 >> 2)] = av[r];
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) m1[c] = mfma_f32(av[r], ugB[r], m1[c]);
        }
        __builtin_amdgcn_wave_barrier();
        float4 ach[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          ach[j] = *reinterpret_cast<const float4*>(slab + l16 * SL + 4 * (lq * 4 + (j ^ ((l16 >> 2) & 3))));
        f4_t m2 = zero_f4();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
          const float4 q = ach[kk >> 2];
          const float av = (kk & 3) == 0 ? q.x : (kk & 3) == 1 ? q.y : (kk & 3) == 2 ? q.z : q.w;
          m2 = mfma_f32(av, BMREG ? bM[kk] : sU2[bm_row(kk) * LDM + l16], m2);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) m2acc[si][r] += (double)m2[r];
        __builtin_amdgcn_wave_barrier();
      }
      // request the V fragment two steps ahead into the buffer just used
      load_v(vb[b], rt + (si + 2) / NMY, (si + 2) % NMY);
    }

    __syncthreads();
    // wave w's partial M1^T: m1[c][r] is row R0 + 4 (4 lq + r) + c, column l16 -> red (FP32)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[(w * 64 + 16 * lq + 4 * r + c) * RP + l16] = m1[c][r];
    __syncthreads();
    // the eight partials summed in FP32 (the sum feeds the FP32 K1 product), two elements
    // of the 64 x 16 block per thread
    float* m1f = reinterpret_cast<float*>(m1s);
    for (int e = tid; e < T * NP; e += NW * 64) {
      const int row = e / NP, col = e % NP;
      float sm = 0.0f;
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) sm += red[(ww * 64 + row) * RP + col];
      m1f[e] = sm;
    }
    __syncthreads();
    if (a.want_k1 && w < mt) {
      // K1 += Phi^T M1^T over the tile's 64 rows on the FP32 matrix cores in two
      // independent chains of 32 rows, added to the FP64 sum of the tiles
      const float* ph = sPhi + lq * PP + 16 * w + l16;
      f4_t t0 = zero_f4(), t1 = zero_f4();
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          t0 = mfma_f32(ph[(16 * q + 4 * r) * PP], m1f[(16 * q + 4 * r + lq) * 16 + l16], t0);
          t1 = mfma_f32(ph[(16 * q + 32 + 4 * r) * PP], m1f[(16 * q + 32 + 4 * r + lq) * 16 + l16], t1);
        }
#pragma unroll
      for (int r = 0; r < 4; ++r) k1[r] += (double)t0[r] + (double)t1[r];
    }
  };

  for (int64_t rt = rt0; rt < rt1; rt += 2) {
    tile(std::integral_constant<int, 0>{}, rt);
    if (rt + 1 < rt1) tile(std::integral_constant<int, 1>{}, rt + 1);
  }

  const int wg = blockIdx.x;
  if (a.want_k1 && w < mt) {
    double* out = a.K1p + (int64_t)wg * a.Np * NP;
#pragma unroll
    for (int r = 0; r < 4; ++r) out[(int64_t)(16 * w + 4 * lq + r) * NP + l16] = k1[r];
  }
  // M2 rows of the wave's subtiles: M2[g0 + 4lq + r][l16]
  double* out = a.M2p + (int64_t)rb * a.G * NP;
#pragma unroll
  for (int si = 0; si < NMY; ++si)
    if (si < nmy) {
      const int64_t g0 = (gs0 + w + si * NW) * 16;
#pragma unroll
      for (int r = 0; r < 4; ++r) out[(g0 + 4 * lq + r) * NP + l16] = m2acc[si][r];
    }
}

// Orbitals on the grid and at the points: U = Phi C and U_g = Phi_g C.
// Row subtiles 16 at a time on the FP64 matrix cores; rows [0, R) come from
// Phi, rows [R, R + G) from Phi_g.  C [N x n] (row pitch n) is read once into
// LDS as the zero-padded [Np x NP] operand.  Each wave loads its 16 x Np block
// of basis values up front (MT = Np/16 <= 8) so that the loads overlap.
template <int NI, int MT>
__global__ __launch_bounds__(256) void orbitals_kernel(const double* __restrict__ Phi, int64_t R,
                                                      const double* __restrict__ Phig, int64_t G, int /*Np*/,
                                                      const double* __restrict__ C, int N, int n,
                                                      double* __restrict__ U, double* __restrict__ Ug,
                                                      double* __restrict__ Ugp) {
  constexpr int NP = 16 * NI;
  constexpr int NPK = 16 * MT;                 // padded N (the Np argument equals it)
  extern __shared__ double lds[];
  double* sC = lds;                            // [Np][NP]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, lq = lane >> 4;
  constexpr int ldb = NPK + 1;
  double* sB = lds + NPK * NP + w * 16 * ldb;  // this wave's 16 x Np block, pitch Np + 1
  const int64_t nsub = (R + G) / 16;
  constexpr int nvec = 16 * NPK / 2;           // 16-byte pieces of a 16-row block
  constexpr int NQ = (nvec + 63) / 64;
  // the 16 rows of a subtile are contiguous in memory (16*Np doubles); the
  // next subtile's rows are loaded while the current one is multiplied
  double2 buf[NQ];
  auto fetch = [&](int64_t sidx) {
    const int64_t row0 = sidx * 16;
    const double* src = (row0 < R) ? Phi + row0 * NPK : Phig + (row0 - R) * NPK;
    const double2* src2 = reinterpret_cast<const double2*>(src);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int v = q * 64 + lane;
      if (v < nvec) buf[q] = src2[v];
    }
  };
  const int64_t sfirst = (int64_t)blockIdx.x * 4 + w, sstep = (int64_t)gridDim.x * 4;
  // the first block of basis values is in flight while C is staged
  if (sfirst < nsub) fetch(sfirst);
  for (int e = tid; e < NPK * NP; e += 256) {
    const int r = e / NP, c = e % NP;
    sC[e] = (r < N && c < n) ? C[(int64_t)r * n + c] : 0.0;
  }
  __syncthreads();
  for (int64_t sidx = sfirst; sidx < nsub; sidx += sstep) {
    const int64_t row0 = sidx * 16;
    double* dst = (row0 < R) ? U + row0 * NP : Ug + (row0 - R) * NP;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int v = q * 64 + lane;
      if (v < nvec) {
        const int e = 2 * v, r = e / NPK, c = e % NPK;
        sB[r * ldb + c] = buf[q].x;
        sB[r * ldb + c + 1] = buf[q].y;
      }
    }
    if (sidx + sstep < nsub) fetch(sidx + sstep);
    __builtin_amdgcn_wave_barrier();
    d4_t acc[NI];
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[j] = zero_d4();
#pragma unroll
    for (int kk = 0; kk < MT * 4; ++kk) {
      const double x = sB[l16 * ldb + 4 * kk + lq];
#pragma unroll
      for (int j = 0; j < NI; ++j) acc[j] = mfma_f64(x, sC[(4 * kk + lq) * NP + 16 * j + l16], acc[j]);
    }
    __builtin_amdgcn_wave_barrier();
    double* out = dst + lq * NP + l16;
#pragma unroll
    for (int j = 0; j < NI; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) out[(int64_t)(4 * r) * NP + 16 * j] = acc[j][r];
    if (NI == 1 && Ugp && row0 >= R) {
      // permuted copy [g][i % 4][i / 4] of U_g for the n <= 16 exchange kernel
      double* op = Ugp + (row0 - R + lq) * 16 + (l16 & 3) * 4 + (l16 >> 2);
#pragma unroll
      for (int r = 0; r < 4; ++r) op[(int64_t)(4 * r) * 16] = acc[0][r];
    }
  }
}

// Deterministic sums over partials for up to three segments in one launch:
// out_s[i] = sum_p in_s[p * count_s + i].  A block owns 16 outputs of one
// segment; its 16 partial lanes per output take p = q, q + 16, ... with 8 loads
// in flight, and are combined in a fixed order.
struct ReduceSeg {
  const double* in;
  int64_t nparts, count;
  double* out;
  int64_t block0;     // first block of this segment
};
struct ReduceArgs {
  ReduceSeg seg[3];
  int nseg;
};

__global__ __launch_bounds__(256) void reduce_partials_kernel(ReduceArgs ra) {
  // 16 outputs per block, 16 partial lanes per output (lane q takes p = q, q + 16, ...,
  // eight loads in flight), lanes combined in a fixed order
  __shared__ double red[16][17];
  int si = 0;
  for (int k = 1; k < ra.nseg; ++k)
    if ((int64_t)blockIdx.x >= ra.seg[k].block0) si = k;
  const ReduceSeg sg = ra.seg[si];
  const int x = threadIdx.x & 15, q = threadIdx.x >> 4;
  const int64_t i = ((int64_t)blockIdx.x - sg.block0) * 16 + x;
  double s = 0.0;
  if (i < sg.count) {
    int64_t p = q;
    for (; p + 112 < sg.nparts; p += 128) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = sg.in[(p + 16 * u) * sg.count + i];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; p < sg.nparts; p += 16) s += sg.in[p * sg.count + i];
  }
  red[q][x] = s;
  __syncthreads();
  if (q == 0 && i < sg.count) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) t += red[k][x];
    sg.out[i] = t;
  }
}

// Final step of a build.  Workgroup (m, j) owns the 16 x 16 output tile
// K[16m.., 16j..]: it forms K2 = Phi_g^T M2 for the tile on the matrix cores
// with the inner dimension split over the 8 waves (fixed-order reduction) and
// writes K = dV (s1 K1 + s2 K2 + s3 K3) for mu < N, i < n.  The last workgroup
// sums the energy partials with a fixed tree.
__global__ __launch_bounds__(512) void finalize_kernel(const double* __restrict__ Phig, const double* __restrict__ M2,
                                                      int64_t G, const double* __restrict__ K1,
                                                      const double* __restrict__ K3, int N, int n,
                                                      int np, int Np, double s1, double s2, double s3, double dV,
                                                      double* __restrict__ K, const double* __restrict__ e1p,
                                                      int64_t ne1, const double* __restrict__ e3p, int64_t ne3,
                                                      double ce1, double ce3, double* __restrict__ ex,
                                                      EnergyDots dots) {
  __shared__ double red[8][64][4];
  __shared__ int last_blk;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, lq = lane >> 4;
  const int ntile = (Np / 16) * (np / 16);
  if ((int)blockIdx.x >= ntile) {
    // energy: block eb of neb takes a contiguous slice of the dot products; with
    // one block the result goes to ex, else to the partial list summed later
    if (!ex) return;
    const int eb = (int)blockIdx.x - ntile, neb = (int)gridDim.x - ntile;
    auto slice = [&](int64_t n, int64_t& b0, int64_t& b1) {
      const int64_t per = (n + neb - 1) / neb;
      b0 = (int64_t)eb * per;
      b1 = (b0 + per < n) ? b0 + per : n;
    };
    double sa = 0.0, sb = 0.0;
    int64_t b0, b1;
    slice(ne1, b0, b1);
    for (int64_t p = b0 + tid; p < b1; p += 512) sa += e1p[p];
    slice(ne3, b0, b1);
    for (int64_t p = b0 + tid; p < b1; p += 512) sb += e3p[p];
    slice(dots.n1, b0, b1);
#pragma unroll 8
    for (int64_t p = b0 + tid; p < b1; p += 512) sa += dots.x1[p] * dots.y1[p];
    slice(dots.n3, b0, b1);
#pragma unroll 4
    for (int64_t p = b0 + tid; p < b1; p += 512) sb += dots.x3[p] * dots.y3[p];
    double* r1 = &red[0][0][0];
    r1[tid] = ce1 * sa + ce3 * sb;
    __syncthreads();
    for (int off = 256; off > 0; off >>= 1) {
      if (tid < off) r1[tid] += r1[tid + off];
      __syncthreads();
    }
    if (tid == 0) {
      if (neb == 1) *ex = -dV * r1[0];
      else dots.part[eb] = r1[0];
    }
    if (neb > 1 && dots.count) {
      // the last energy block to finish sums the partials in a fixed order and resets
      // the counter for the next build (device-scope release / acquire around it)
      __threadfence();
      __syncthreads();
      if (tid == 0) last_blk = (atomicAdd(dots.count, 1u) == (unsigned)(neb - 1));
      __syncthreads();
      if (last_blk) {
        __threadfence();
        double v = 0.0;
        for (int i = tid; i < neb; i += 512)
          v += __hip_atomic_load(dots.part + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        r1[tid] = v;
        __syncthreads();
        for (int off = 256; off > 0; off >>= 1) {
          if (tid < off) r1[tid] += r1[tid + off];
          __syncthreads();
        }
        if (tid == 0) {
          *ex = -dV * r1[0];
          *dots.count = 0u;
        }
      }
    }
    return;
  }
  const int m = blockIdx.x / (np / 16), j = blockIdx.x % (np / 16);
  d4_t acc = zero_d4();
  if (M2) {
    // wave w takes the k slices sl = w + 8 q (G is a multiple of 64), sixteen at a time
    // with all their loads in flight together (clamped, unconditional; slices past the
    // end contribute zero)
    const int64_t per = G / 32;
    for (int64_t q0 = 0; q0 < per; q0 += 16) {
      double a[16], b[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int64_t q = (q0 + u < per) ? q0 + u : per - 1;
        const int64_t g = 4 * (w + 8 * q) + lq;
        a[u] = Phig[g * Np + 16 * m + l16];
        b[u] = M2[g * np + 16 * j + l16];
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) acc = mfma_f64(a[u], (q0 + u < per) ? b[u] : 0.0, acc);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) red[w][lane][r] = acc[r];
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double s = 0.0;
      for (int ww = 0; ww < 8; ++ww) s += red[ww][lane][r];
      const int mu = 16 * m + 4 * r + lq, i = 16 * j + l16;
      const int64_t q = (int64_t)mu * np + i;
      double v = s2 * s;
      if (K1) v += s1 * K1[q];
      if (K3) v += s3 * K3[q];
      if (mu < N && i < n) K[(int64_t)mu * n + i] = dV * v;
    }
  }
}

// Zero-padded copy Cp [rows_p x ldp] of C [rows x cols] (row pitch ldc).
__global__ void pack_kernel(const double* __restrict__ C, int64_t rows, int64_t cols, int64_t ldc,
                            double* __restrict__ Cp, int64_t rows_p, int64_t ldp) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows_p * ldp) return;
  const int64_t r = t / ldp, c = t % ldp;
  Cp[t] = (r < rows && c < cols) ? C[r * ldc + c] : 0.0;
}

// ex = -dV sum of the energy partials of the finalize kernel (one block of 256,
// strided partial sums, fixed-order tree).
__global__ __launch_bounds__(256) void energy_sum_kernel(const double* __restrict__ part, int n, double dV,
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
  if (tid == 0) *ex = -dV * red[0];
}

// K[i][j] = dV (T[i][j] + T[j][i] - K3[i][j]) for i, j < N (T, K3 pitch Np).
__global__ void full_combine_kernel(const double* __restrict__ T, const double* __restrict__ K3, int64_t Np,
                                    int64_t N, double dV, double* __restrict__ K) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * N) return;
  const int64_t i = t / N, j = t % N;
  K[t] = dV * (T[i * Np + j] + T[j * Np + i] - K3[i * Np + j]);
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

template <int NW, int NI, int MT>
hipError_t launch_fused3(const FusedArgs& a, int blocks, hipStream_t s) {
  const int64_t gper = ((a.G / T + a.gblocks - 1) / a.gblocks) * (T / 16);
  const int64_t lds = fused_lds_doubles<NW, NI>(a.want_m2 ? gper * 16 : 0) * 8;
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  // the energy term is accumulated in the kernel exactly when M2 is not formed
  if ((a.want_e != 0) == (a.want_m2 != 0)) return hipErrorInvalidValue;
  auto k = a.want_m2 ? fused_f64_kernel<NW, NI, MT, true> : fused_f64_kernel<NW, NI, MT, false>;
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(blocks), dim3(NW * 64), (size_t)lds, s, a);
  return hipGetLastError();
}

template <int NW, int NI>
hipError_t launch_fused2(const FusedArgs& a, int blocks, hipStream_t s) {
  const int mt = a.want_k1 ? a.Np / 16 : 0;
  if (mt == 0) return launch_fused3<NW, NI, 0>(a, blocks, s);
  if (mt <= 4) return launch_fused3<NW, NI, 4>(a, blocks, s);
  if (mt <= 8) return launch_fused3<NW, NI, 8>(a, blocks, s);
  return hipErrorInvalidValue;
}

template <int NW, int MT, int M2MODE>
hipError_t launch_m4(const FusedArgs& a, int blocks, hipStream_t s) {
  const int64_t gper = ((a.G / T + a.gblocks - 1) / a.gblocks) * (T / 16);
  const int64_t lds = ((int64_t)NW * 16 * SLAB + (int64_t)T * 18 + (a.want_m2 ? gper * 16 : 0) * 16) * 8;
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  auto k = fused_m4_kernel<NW, MT, M2MODE>;
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(blocks), dim3(NW * 64), (size_t)lds, s, a);
  return hipGetLastError();
}

template <int NW, int M2MODE>
hipError_t launch_m4_mt(const FusedArgs& a, int blocks, hipStream_t s) {
  const int mt = a.want_k1 ? a.Np / 16 : 0;
  if (mt == 0) return launch_m4<NW, 0, M2MODE>(a, blocks, s);
  if (mt <= 4) return launch_m4<NW, 4, M2MODE>(a, blocks, s);
  if (mt <= 8) return launch_m4<NW, 8, M2MODE>(a, blocks, s);
  return hipErrorInvalidValue;
}

template <int NW, int MT>
hipError_t launch_f32(const FusedArgs& a, int blocks, hipStream_t s) {
  if (a.want_e) return hipErrorInvalidValue;   // this kernel leaves the energy to tr(U_g^T M2)
  const int64_t gper = ((a.G / T + a.gblocks - 1) / a.gblocks) * (T / 16);
  const int64_t lds = ((int64_t)NW * 16 * SLAB + (int64_t)T * 17 + (a.want_m2 ? gper * 16 : 0) * 16) * 8;
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  auto k = fused_f32_kernel<NW, MT>;
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(blocks), dim3(NW * 64), (size_t)lds, s, a);
  return hipGetLastError();
}

// LDS bytes of fused_f32u_kernel (8 waves) for gper g subtiles per workgroup
int64_t f32u_lds_bytes(int Np, int64_t gper) {
  return (int64_t)8 * 16 * (T + 4) * 4 + (int64_t)T * (Np + 4) * 4 + (int64_t)Np * 16 * 8 + (int64_t)T * 16 * 8 +
         (int64_t)T * 17 * 4 + (int64_t)T * 20 * 4 + gper * 16 * 20 * 4;
}

template <int NMY>
hipError_t launch_f32u(const FusedArgs& a, int blocks, hipStream_t s) {
  const int64_t gper = ((a.G / T + a.gblocks - 1) / a.gblocks) * (T / 16);
  const int64_t lds = f32u_lds_bytes(a.Np, gper);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  auto k = fused_f32u_kernel<NMY>;
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(blocks), dim3(512), (size_t)lds, s, a);
  return hipGetLastError();
}

template <int NW>
hipError_t launch_f32_mt(const FusedArgs& a, int blocks, hipStream_t s) {
  const int mt = a.want_k1 ? a.Np / 16 : 0;
  if (mt == 0) return launch_f32<NW, 0>(a, blocks, s);
  if (mt <= 4) return launch_f32<NW, 4>(a, blocks, s);
  if (mt <= 8) return launch_f32<NW, 8>(a, blocks, s);
  return hipErrorInvalidValue;
}

template <int NI>
hipError_t launch_fused1(const FusedArgs& a, int blocks, hipStream_t s) {
  if (NI == 1 && a.prec != 0 && a.Vm32 && a.Phi32) {
    // orbitals formed in the kernel: M2 (and K1) fused, no M1 output, no energy partials
    if (!a.Cm || !a.want_m2 || a.want_m1 || a.want_e || a.nwaves != 8 || a.Np > 128)
      return hipErrorInvalidValue;
    switch (fused_f32u_nmy(a)) {   // subtiles per wave, exactly (the kernel's step count per tile)
      case 1: return launch_f32u<1>(a, blocks, s);
      case 2: return launch_f32u<2>(a, blocks, s);
      case 3: return launch_f32u<3>(a, blocks, s);
      case 4: return launch_f32u<4>(a, blocks, s);
      case 5: return launch_f32u<5>(a, blocks, s);
      case 6: return launch_f32u<6>(a, blocks, s);
      case 7: return launch_f32u<7>(a, blocks, s);
      case 8: return launch_f32u<8>(a, blocks, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (NI == 1 && a.prec != 0 && a.Vm32) {
    if (a.nwaves == 8) return launch_f32_mt<8>(a, blocks, s);
    return launch_f32_mt<4>(a, blocks, s);
  }
  if (NI == 1 && a.use_m4 && a.Ugp) {
    if (a.use_m4 == 2) {
      if (a.nwaves == 8) return launch_m4_mt<8, 1>(a, blocks, s);
      return launch_m4_mt<4, 1>(a, blocks, s);
    }
    if (a.nwaves == 8) return launch_m4_mt<8, 0>(a, blocks, s);
    return launch_m4_mt<4, 0>(a, blocks, s);
  }
  if (a.nwaves == 8) return launch_fused2<8, NI>(a, blocks, s);
  return launch_fused2<4, NI>(a, blocks, s);
}

}  // namespace

int64_t fused_f32u_nmy(const FusedArgs& a) {
  const int64_t gper = ((a.G / T + a.gblocks - 1) / a.gblocks) * (T / 16);
  return (gper + 7) / 8;
}

int64_t fused_f32u_lds(const FusedArgs& a) {
  const int64_t gper = ((a.G / T + a.gblocks - 1) / a.gblocks) * (T / 16);
  return f32u_lds_bytes(a.Np, gper);
}

int fused_rblocks(const FusedArgs& a) {
  const int64_t rt = (a.R_valid + T - 1) / T;
  return (int)((rt + a.rtiles - 1) / a.rtiles);
}

int64_t fused_lds_bytes(const FusedArgs& a) {
  const int64_t gper = ((a.G / T + a.gblocks - 1) / a.gblocks) * (T / 16);
  const int64_t bg = a.want_m2 ? gper * 16 : 0;
  const int64_t per = (int64_t)(a.nwaves == 8 ? 8 : 4) * 16 * SLAB + (int64_t)T * (a.np + 2) + bg * a.np;
  return per * 8;
}

hipError_t fused_exchange(const FusedArgs& a, hipStream_t s) {
  if (a.G % T != 0 || a.R % T != 0 || a.np % 16 != 0 || a.Np % 16 != 0) return hipErrorInvalidValue;
  if (a.want_k1 && a.Np / 16 > 8) return hipErrorInvalidValue;
  if (a.rtiles < 1 || a.gblocks < 1) return hipErrorInvalidValue;
  const int blocks = fused_rblocks(a) * a.gblocks;
  if (blocks <= 0) return hipSuccess;
  switch (a.np / 16) {
    case 1: return launch_fused1<1>(a, blocks, s);
    case 2: return launch_fused1<2>(a, blocks, s);
    case 3: return launch_fused1<3>(a, blocks, s);
    case 4: return launch_fused1<4>(a, blocks, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t sum_partials3(const double* in0, int64_t n0, int64_t c0, double* o0, const double* in1, int64_t n1,
                         int64_t c1, double* o1, const double* in2, int64_t n2, int64_t c2, double* o2,
                         hipStream_t s) {
  ReduceArgs ra{};
  int64_t blocks = 0;
  const double* ins[3] = {in0, in1, in2};
  const int64_t ns[3] = {n0, n1, n2}, cs[3] = {c0, c1, c2};
  double* outs[3] = {o0, o1, o2};
  for (int k = 0; k < 3; ++k) {
    if (!ins[k] || ns[k] <= 0 || cs[k] <= 0) continue;
    ReduceSeg& g = ra.seg[ra.nseg++];
    g.in = ins[k]; g.nparts = ns[k]; g.count = cs[k]; g.out = outs[k]; g.block0 = blocks;
    blocks += (cs[k] + 15) / 16;
  }
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)blocks), dim3(256), 0, s, ra);
  return hipGetLastError();
}

hipError_t orbitals(const double* Phi, int64_t R, const double* Phig, int64_t G, int Np, const double* C,
                    int N, int n, int np, double* U, double* Ug, double* Ugp, hipStream_t s) {
  if (R % 16 != 0 || G % 16 != 0 || Np % 16 != 0 || np % 16 != 0 || Np > 128) return hipErrorInvalidValue;
  const int64_t nsub = (R + G) / 16;
  const unsigned blocks = (unsigned)std::min<int64_t>((nsub + 3) / 4, 512);   // two workgroups per CU
  const int mt = Np / 16;
  const size_t lds = (size_t)Np * np * 8 + (size_t)4 * 16 * (Np + 1) * 8;
#define RPS_ORB(NI_, MT_)                                                                                   \
  do {                                                                                                       \
    hipError_t e_ = hipFuncSetAttribute((const void*)orbitals_kernel<NI_, MT_>,                              \
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);               \
    if (e_ != hipSuccess) return e_;                                                                         \
    hipLaunchKernelGGL((orbitals_kernel<NI_, MT_>), dim3(blocks), dim3(256), lds, s, Phi, R, Phig, G, Np, C, \
                       N, n, U, Ug, Ugp);                                                                    \
  } while (0)
#define RPS_ORB_NI(NI_)                                                                                     \
  do {                                                                                                       \
    switch (mt) {                                                                                            \
      case 1: RPS_ORB(NI_, 1); break; case 2: RPS_ORB(NI_, 2); break; case 3: RPS_ORB(NI_, 3); break;        \
      case 4: RPS_ORB(NI_, 4); break; case 5: RPS_ORB(NI_, 5); break; case 6: RPS_ORB(NI_, 6); break;        \
      case 7: RPS_ORB(NI_, 7); break; default: RPS_ORB(NI_, 8); break;                                       \
    }                                                                                                        \
  } while (0)
  switch (np / 16) {
    case 1: RPS_ORB_NI(1); break;
    case 2: RPS_ORB_NI(2); break;
    case 3: RPS_ORB_NI(3); break;
    case 4: RPS_ORB_NI(4); break;
    default: return hipErrorInvalidValue;
  }
#undef RPS_ORB_NI
#undef RPS_ORB
  return hipGetLastError();
}

hipError_t finalize(const double* Phig, const double* M2, int64_t G, const double* K1, const double* K3, int N,
                    int n, int np, int Np, double s1, double s2, double s3, double dV, double* K, const double* e1p,
                    int64_t ne1, const double* e3p, int64_t ne3, double ce1, double ce3, double* ex, hipStream_t s,
                    const EnergyDots& dots) {
  if (G % 64) return hipErrorInvalidValue;   // the K2 tiles take G in slices of 8 x 4 rows
  const int ntile = (Np / 16) * (np / 16);
  // energy blocks: one per 4K dot-product terms and partials (up to the partial list size)
  // (up to 16K terms one block does it all: no device-scope fence, no counter)
  const int64_t nterms = dots.n1 + dots.n3 + ne1 + ne3;
  int neb = (nterms <= 16384) ? 1 : (int)std::min<int64_t>((nterms + 4095) / 4096, dots.part ? dots.nparts : 1);
  if (neb < 1) neb = 1;
  hipLaunchKernelGGL(finalize_kernel, dim3(ntile + neb), dim3(512), 0, s, Phig, M2, G, K1, K3, N, n, np, Np, s1, s2,
                     s3, dV, K, e1p, ne1, e3p, ne3, ce1, ce3, ex, dots);
  if (neb > 1 && ex && !dots.count)
    hipLaunchKernelGGL(energy_sum_kernel, dim3(1), dim3(256), 0, s, dots.part, neb, dV, ex);
  return hipGetLastError();
}

hipError_t pack_matrix(const double* C, int64_t rows, int64_t cols, int64_t ldc, double* Cp, int64_t rows_p,
                       int64_t ldp, hipStream_t s) {
  hipLaunchKernelGGL(pack_kernel, dim3(nblk(rows_p * ldp, 256)), dim3(256), 0, s, C, rows, cols, ldc, Cp, rows_p,
                     ldp);
  return hipGetLastError();
}

hipError_t full_combine(const double* T, const double* K3, int64_t Np, int64_t N, double dV, double* K,
                        hipStream_t s) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(full_combine_kernel, dim3(nblk(N * N, 256)), dim3(256), 0, s, T, K3, Np, N, dV, K);
  return hipGetLastError();
}

}  // namespace rps
