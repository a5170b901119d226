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
#include <stdlib.h>

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
      if (gn < g.N && gk < kend) {
        v = g.transB ? g.B[gn * g.ldb + gk] : g.B[gk * g.ldb + gn];
        if (g.kscale) v *= g.kscale[gk];
      }
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
          else if (g.epi == EPI_HADAMARD_SRC) *c = (g.D ? g.D[gm * g.ldd + gn] : (double)g.D32[gm * g.ldd + gn]) * v;
          else {
            *c = (g.beta == 0.0) ? v : v + g.beta * *c;
            if (g.Cf) g.Cf[gm * g.ldcf + gn] = (float)*c;
          }
        }
      }
}

// Large tiles: 4 waves in 2 x 2, each wave (16*TM) x (16*TN) of C, BK = 16,
// operands prefetched into registers while the matrix cores work on the
// current LDS buffer (two buffers, one barrier per K step).  KS: row k of
// op(B) is scaled by kscale[k] as it is loaded.  The body computes the output
// tile at (m0, n0) of K split bz; gemm_big_kernel and the grouped kernel below
// differ only in how they pick the tile and the operands.
template <int TM, int TN, bool TA, bool TB, bool KS>
__device__ __forceinline__ void gemm_big_body(const Gemm& g, int64_t m0, int64_t n0, int bz) {
  constexpr int BM = 32 * TM, BN = 32 * TN;
  constexpr int PA = BM * BK / 256, PB = BN * BK / 256;
  constexpr int LA = BM + 1, LB = BN + 1;
  __shared__ double As[2][BK * LA];
  __shared__ double Bs[2][BK * LB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int l16 = lane & 15, lq = lane >> 4;
  if (g.lower_only && n0 > m0 + BM - 1) return;

  int64_t kbeg = 0, kend = g.K;
  if (g.splitk > 1) {
    const int64_t per = ((g.K + g.splitk - 1) / g.splitk + BK - 1) / BK * BK;
    kbeg = (int64_t)bz * per;
    kend = (kbeg + per < g.K) ? kbeg + per : g.K;
  }
  const int64_t nk = (kend > kbeg) ? (kend - kbeg + BK - 1) / BK : 0;

  // Element e = tid + 256 i of a tile maps to consecutive addresses across
  // consecutive threads for either storage order of each operand.  Addresses
  // are a uniform tile base plus 32-bit per-lane offsets (a tile spans less
  // than 2^31 elements for every leading dimension used here).
  const bool interior = (m0 + BM <= g.M) && (n0 + BN <= g.N);
  const int lda = (int)g.lda, ldb = (int)g.ldb;
  double ra[PA], rb[PB];
  auto load = [&](int64_t k0) {
    const bool full = interior && (k0 + BK <= kend);
    const int64_t kc = (k0 < kend) ? k0 : kbeg;   // keeps the base in bounds past the last step
    const double* ba = g.A + (TA ? kc * g.lda + m0 : m0 * g.lda + kc);
    const double* bb = g.B + (TB ? n0 * g.ldb + kc : kc * g.ldb + n0);
    const double* bk = KS ? g.kscale + kc : nullptr;
    if (full) {     // uniform: whole tile inside, straight-line loads
#pragma unroll
      for (int i = 0; i < PA; ++i) {
        const int e = tid + 256 * i;
        const int m = TA ? e % BM : e / BK, k = TA ? e / BM : e % BK;
        ra[i] = ba[TA ? k * lda + m : m * lda + k];
      }
#pragma unroll
      for (int i = 0; i < PB; ++i) {
        const int e = tid + 256 * i;
        const int n = TB ? e / BK : e % BN, k = TB ? e % BK : e / BN;
        rb[i] = bb[TB ? n * ldb + k : k * ldb + n];
        if constexpr (KS) rb[i] *= bk[k];
      }
    } else {
#pragma unroll
      for (int i = 0; i < PA; ++i) {
        const int e = tid + 256 * i;
        const int m = TA ? e % BM : e / BK, k = TA ? e / BM : e % BK;
        ra[i] = (m0 + m < g.M && k0 + k < kend) ? ba[TA ? k * lda + m : m * lda + k] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < PB; ++i) {
        const int e = tid + 256 * i;
        const int n = TB ? e / BK : e % BN, k = TB ? e % BK : e / BN;
        rb[i] = (n0 + n < g.N && k0 + k < kend) ? bb[TB ? n * ldb + k : k * ldb + n] * (KS ? bk[k] : 1.0) : 0.0;
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < PA; ++i) {
      const int e = tid + 256 * i;
      const int m = TA ? e % BM : e / BK, k = TA ? e / BM : e % BK;
      As[buf][k * LA + m] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < PB; ++i) {
      const int e = tid + 256 * i;
      const int n = TB ? e / BK : e % BN, k = TB ? e % BK : e / BN;
      Bs[buf][k * LB + n] = rb[i];
    }
  };

  d4_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = zero_d4();

  if (nk > 0) {
    load(kbeg);
    store(0);
  }
  __syncthreads();
  // The loop body is one basic block (the prefetch past the last step reads
  // in-bounds addresses and is discarded), which keeps the accumulators in
  // the matrix-core registers across iterations.
  for (int64_t t = 0; t < nk; ++t) {
    load(kbeg + (t + 1) * BK);
    const double* as = As[t & 1] + lq * LA + wm * 16 * TM + l16;
    const double* bs = Bs[t & 1] + lq * LB + wn * 16 * TN + l16;
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      double a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = as[4 * kk * LA + 16 * i];
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = bs[4 * kk * LB + 16 * j];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = mfma_f64(a[i], b[j], acc[i][j]);
    }
    store((t + 1) & 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gm = m0 + wm * 16 * TM + i * 16 + d64_row(lane, r);
        const int64_t gn = n0 + wn * 16 * TN + j * 16 + l16;
        if (gm < g.M && gn < g.N) {
          const double v = g.alpha * acc[i][j][r];
          if (g.splitk > 1) {
            g.work[((int64_t)bz * g.M + gm) * g.N + gn] = v;
            continue;
          }
          double* c = g.C + gm * g.ldc + gn;
          if (g.epi == EPI_SQUARE) *c = v * v;
          else if (g.epi == EPI_HADAMARD) *c = *c * v;
          else if (g.epi == EPI_HADAMARD_SRC) *c = (g.D ? g.D[gm * g.ldd + gn] : (double)g.D32[gm * g.ldd + gn]) * v;
          else {
            *c = (g.beta == 0.0) ? v : v + g.beta * *c;
            if (g.Cf) g.Cf[gm * g.ldcf + gn] = (float)*c;
          }
        }
      }
}

// FP32 operands on the FP32 matrix cores (v_mfma_f32_16x16x4_f32), the
// products of the precision form's GEMM form.  Tiling as gemm_big_kernel:
// 2 x 2 waves of (16*TM) x (16*TN), BK = 16, double-buffered LDS with the next
// step's operands prefetched into registers.  The LDS pitch BM + 16 puts the
// four k rows of an operand fetch on disjoint banks.  Outputs:
//   OUT32: C32 = D32 o (alpha * AB), FP32 (the A = V o P chunk, short K);
//   else   C = alpha * AB + beta * C in FP64, or FP64 partials per K split,
//          with the FP32 sums moved into FP64 registers every 64 terms of K.
template <int TM, int TN, bool TA, bool TB, bool OUT32>
__global__ __launch_bounds__(256, 2) void gemm32_kernel(Gemm32 g) {
  constexpr int BM = 32 * TM, BN = 32 * TN;
  constexpr int PA = BM * BK / 256, PB = BN * BK / 256;
  constexpr int LA = BM + 16, LB = BN + 16;
  __shared__ float As[2][BK * LA];
  __shared__ float Bs[2][BK * LB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int l16 = lane & 15, lq = lane >> 4;
  const int bz = blockIdx.z;
  const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;

  int64_t kbeg = 0, kend = g.K;
  if (g.splitk > 1) {
    const int64_t per = ((g.K + g.splitk - 1) / g.splitk + BK - 1) / BK * BK;
    kbeg = (int64_t)bz * per;
    kend = (kbeg + per < g.K) ? kbeg + per : g.K;
  }
  const int64_t nk = (kend > kbeg) ? (kend - kbeg + BK - 1) / BK : 0;

  const bool interior = (m0 + BM <= g.M) && (n0 + BN <= g.N);
  const int lda = (int)g.lda, ldb = (int)g.ldb;
  float ra[PA], rb[PB];
  auto load = [&](int64_t k0) {
    const bool full = interior && (k0 + BK <= kend);
    const int64_t kc = (k0 < kend) ? k0 : kbeg;   // keeps the base in bounds past the last step
    const float* ba = g.A + (TA ? kc * g.lda + m0 : m0 * g.lda + kc);
    const float* bb = g.B + (TB ? n0 * g.ldb + kc : kc * g.ldb + n0);
    if (full) {
#pragma unroll
      for (int i = 0; i < PA; ++i) {
        const int e = tid + 256 * i;
        const int m = TA ? e % BM : e / BK, k = TA ? e / BM : e % BK;
        ra[i] = ba[TA ? k * lda + m : m * lda + k];
      }
#pragma unroll
      for (int i = 0; i < PB; ++i) {
        const int e = tid + 256 * i;
        const int n = TB ? e / BK : e % BN, k = TB ? e % BK : e / BN;
        rb[i] = bb[TB ? n * ldb + k : k * ldb + n];
      }
    } else {
#pragma unroll
      for (int i = 0; i < PA; ++i) {
        const int e = tid + 256 * i;
        const int m = TA ? e % BM : e / BK, k = TA ? e / BM : e % BK;
        ra[i] = (m0 + m < g.M && k0 + k < kend) ? ba[TA ? k * lda + m : m * lda + k] : 0.f;
      }
#pragma unroll
      for (int i = 0; i < PB; ++i) {
        const int e = tid + 256 * i;
        const int n = TB ? e / BK : e % BN, k = TB ? e % BK : e / BN;
        rb[i] = (n0 + n < g.N && k0 + k < kend) ? bb[TB ? n * ldb + k : k * ldb + n] : 0.f;
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < PA; ++i) {
      const int e = tid + 256 * i;
      const int m = TA ? e % BM : e / BK, k = TA ? e / BM : e % BK;
      As[buf][k * LA + m] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < PB; ++i) {
      const int e = tid + 256 * i;
      const int n = TB ? e / BK : e % BN, k = TB ? e % BK : e / BN;
      Bs[buf][k * LB + n] = rb[i];
    }
  };

  f4_t acc[TM][TN];
  // FP64 output: the FP32 sums cover FLUSH K steps (64 terms), then go into FP64
  // registers, so rounding does not grow with the length of K
  constexpr int FLUSH = OUT32 ? (1 << 30) : 4;
  double acc64[OUT32 ? 1 : TM][OUT32 ? 1 : TN][4];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = zero_f4();
  if constexpr (!OUT32) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc64[i][j][r] = 0.0;
  }

  if (nk > 0) {
    load(kbeg);
    store(0);
  }
  __syncthreads();
  for (int64_t t0 = 0; t0 < nk; t0 += FLUSH) {
    const int64_t t1 = (t0 + FLUSH < nk) ? t0 + FLUSH : nk;
    for (int64_t t = t0; t < t1; ++t) {
      load(kbeg + (t + 1) * BK);
      const float* as = As[t & 1] + lq * LA + wm * 16 * TM + l16;
      const float* bs = Bs[t & 1] + lq * LB + wn * 16 * TN + l16;
#pragma unroll
      for (int kk = 0; kk < BK / 4; ++kk) {
        float a[TM], b[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) a[i] = as[4 * kk * LA + 16 * i];
#pragma unroll
        for (int j = 0; j < TN; ++j) b[j] = bs[4 * kk * LB + 16 * j];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[i][j] = mfma_f32(a[i], b[j], acc[i][j]);
      }
      store((t + 1) & 1);
      __syncthreads();
    }
    if constexpr (!OUT32) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[i][j][r] += (double)acc[i][j][r];
          acc[i][j] = zero_f4();
        }
    }
  }

#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gm = m0 + wm * 16 * TM + i * 16 + d32_row(lane, r);
        const int64_t gn = n0 + wn * 16 * TN + j * 16 + l16;
        if (gm < g.M && gn < g.N) {
          if constexpr (OUT32) {
            g.C32[gm * g.ldc + gn] = g.D32[gm * g.ldd + gn] * ((float)g.alpha * acc[i][j][r]);
          } else {
            const double v = g.alpha * acc64[i][j][r];
            if (g.splitk > 1) {
              g.work[((int64_t)bz * g.M + gm) * g.N + gn] = v;
              continue;
            }
            double* c = g.C + gm * g.ldc + gn;
            *c = (g.beta == 0.0) ? v : v + g.beta * *c;
            if (g.Cf) g.Cf[gm * g.ldcf + gn] = (float)*c;
          }
        }
      }
}

// FP32 products with 16-byte operand traffic.  Same outputs and tiling as
// gemm32_kernel (2 x 2 waves of (16*TM) x (16*TN), FP32 sums over 64 terms of K
// then FP64), but every operand moves in 16-byte pieces: float4 loads from global
// memory, 16-byte LDS stores, and 16-byte LDS reads where K is the contiguous
// dimension.  Each operand tile keeps the storage order it has in global memory:
//   K-major  ([mn][k], pitch BK + 4): op(A) with TA = false, op(B) with TB = true;
//   MN-major ([k][mn], pitch BMN + 4): op(A) with TA = true, op(B) with TB = false.
// The matrix-core step kk (0..3) of a 16-wide K slice h takes from lane group
// q = lane / 16 the element k = 16 h + 4 q + kk (a fixed permutation of K that
// both operands share, so the products are the same sums), which makes the four
// values a lane needs from a K-major tile one 16-byte read.  The pitches keep the
// reads of a wave off shared banks: K-major rows are BK + 4 = 20 floats apart, so
// eight consecutive rows cover the 32 banks once; MN-major row groups 4 rows apart
// are 16 banks apart.  The 16-byte stores are conflict-free for MN-major tiles and
// at most two-way for K-major ones.
// Requires lda, ldb (and ldd for OUT32) multiples of 4 and 16-byte aligned bases.
// Row of a K-major tile filled by piece row q.  With 16-wide K steps four
// consecutive lanes fill one row (16 floats), so eight lanes fill two rows; rows
// 4 apart sit 80 = 16 (mod 32) banks apart, so pairing q = 2t, 2t + 1 with rows
// 4 apart puts the eight lanes' 16-byte stores on distinct banks (rows next to
// each other would share four).  A bijection on every block of eight rows.
template <int CW>
__device__ __forceinline__ int kmajor_row(int q) {
  if constexpr (CW != 4) return q;
  const int t = q >> 1;
  return ((t >> 2) << 3) + (t & 3) + ((q & 1) << 2);
}

// The same products with the operands moved from global memory straight into LDS
// (global_load_lds_dwordx4: lane L of a wave writes bytes [16 L, 16 L + 16) after a
// wave-uniform LDS base), three LDS stages, loads issued two K steps ahead.  With
// no staging registers and no LDS store instructions, each 16-deep step is: wait
// for this step's loads (vmcnt, issue order), one barrier, issue the loads of step
// t + 2 into the stage step t - 1 used, then the LDS reads and the matrix-core
// instructions of step t.  The loads past the last step re-read the last step (in
// bounds), so every step has the same number of loads in flight.  The loop is
// unrolled over the three stages (one LDS array each, passed to each step as
// restrict pointers), so the compiler can tell a step's reads from the loads in
// flight to the other stages and adds no wait of its own beyond the explicit one.
// FP64 output on 128 x 64 tiles (on 128 x 128 its accumulators spill registers);
// FP32 output on 128 x 128 tiles, or 128 x 64 where those pad N less.
//
// LDS layouts are unpadded, with 16-byte chunks permuted within a row (the DMA
// writes whole 1 KB runs): K-major rows (16 floats, 4 chunks) hold logical chunk q
// at q ^ ((row >> 1) & 3); MN-major rows (tile width W floats) hold chunk c at
// c ^ (k & 4).  The matrix-core operand reads of a wave then fall on distinct banks
// (eight 16-byte reads at a time for K-major rows: 16 row + 4 chunk dwords cover
// 32 banks; for MN-major rows lanes 0-31 read rows k and k + 4, whose chunk
// groups the permutation puts 16 banks apart).
// Requires K (and every K split) a multiple of 16; whole 16-byte pieces past M or
// the readable N are read from the matrix's edge instead (their products only
// reach outputs that are not stored).
template <int TM, int TN, bool TA, bool TB, bool OUT32>
__global__ __launch_bounds__(256, 2) void gemm32d_kernel(Gemm32 g) {
  constexpr int BK = 16;
  constexpr int BM = 32 * TM, BN = 32 * TN;
  constexpr int ASZ = BM * BK, BSZ = BN * BK;                // floats per stage
  constexpr int NA = ASZ / 4 / 256, NB = BSZ / 4 / 256;      // 16-byte pieces per thread per stage
  constexpr int NPER = NA + NB;                              // loads per thread per stage
  static_assert(NA >= 1 && NB >= 1 && NPER < 16, "stage split");
  // one array per stage: the loop is unrolled by the three stages, so the compiler
  // sees that a step's LDS reads and the loads it issues touch different arrays
  __shared__ __attribute__((aligned(16))) float A0[ASZ], A1[ASZ], A2[ASZ];
  __shared__ __attribute__((aligned(16))) float B0[BSZ], B1[BSZ], B2[BSZ];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int l16 = lane & 15, lq = lane >> 4;
  // tile order: as gemm32v_kernel (XCD-contiguous ranges, K splits outermost, groups of 8 row panels)
  const int64_t tiles_n = (g.N + BN - 1) / BN, tiles_m = (g.M + BM - 1) / BM;
  const int64_t ntile = tiles_n * tiles_m * g.splitk;
  const int64_t per = ((ntile + 7) / 8);
  const int64_t T = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (T >= ntile) return;
  constexpr int64_t GROUP = 8;
  const int bz = (int)(T / (tiles_n * tiles_m));
  const int64_t T2 = T % (tiles_n * tiles_m);
  const int64_t grp = T2 / (GROUP * tiles_n), r2 = T2 % (GROUP * tiles_n);
  const int64_t gh = (tiles_m - grp * GROUP < GROUP) ? tiles_m - grp * GROUP : GROUP;
  const int64_t m0 = (grp * GROUP + r2 % gh) * BM, n0 = (r2 / gh) * BN;

  int64_t kbeg = 0, kend = g.K;
  if (g.splitk > 1) {
    const int64_t kper = ((g.K + g.splitk - 1) / g.splitk + BK - 1) / BK * BK;
    kbeg = (int64_t)bz * kper;
    kend = (kbeg + kper < g.K) ? kbeg + kper : g.K;
  }
  const int64_t nk = (kend > kbeg) ? (kend - kbeg) / BK : 0;
  const int64_t nread = (g.Nread > g.N) ? g.Nread : g.N;
  const int64_t lda = g.lda, ldb = g.ldb;

  // global source of piece P (0 <= P < 512 or < BSZ / 4) of a stage for K step k0
  auto src_a = [&](int P, int64_t k0) -> const float* {
    if constexpr (!TA) {                     // K-major: row P / 4, slot P % 4
      const int r = P >> 2, q = (P & 3) ^ ((r >> 1) & 3);
      int64_t gm = m0 + r;
      if (gm >= g.M) gm = g.M - 1;
      return g.A + gm * lda + k0 + 4 * q;
    } else {                                 // MN-major: row k = P / (BM / 4), slot P % (BM / 4)
      constexpr int CW = BM / 4;
      const int k = P / CW, c = (P % CW) ^ (k & 4);
      const int64_t gc = (m0 + 4 * c < g.M) ? m0 + 4 * c : m0;
      return g.A + (k0 + k) * lda + gc;
    }
  };
  auto src_b = [&](int P, int64_t k0) -> const float* {
    if constexpr (TB) {                      // K-major: row n = P / 4
      const int r = P >> 2, q = (P & 3) ^ ((r >> 1) & 3);
      int64_t gn = n0 + r;
      if (gn >= nread) gn = nread - 1;
      return g.B + gn * ldb + k0 + 4 * q;
    } else {                                 // MN-major: row k = P / (BN / 4)
      constexpr int CW = BN / 4;
      const int k = P / CW, c = (P % CW) ^ (k & 4);
      const int64_t gc = (n0 + 4 * c < nread) ? n0 + 4 * c : n0;
      return g.B + (k0 + k) * ldb + gc;
    }
  };
  auto issue = [&](int64_t t, float* as, float* bs) {
    const int64_t k0 = kbeg + ((t < nk) ? t : nk - 1) * BK;   // past the end: the last step again
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int run = i * 4 + wave;          // 1 KB run of this wave instruction
      __builtin_amdgcn_global_load_lds((const void*)src_a(run * 64 + lane, k0),
                                       (__attribute__((address_space(3))) void*)&as[run * 256], 16, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int run = i * 4 + wave;
      __builtin_amdgcn_global_load_lds((const void*)src_b(run * 64 + lane, k0),
                                       (__attribute__((address_space(3))) void*)&bs[run * 256], 16, 0, 0);
    }
  };

  f4_t acc[TM][TN];
  constexpr int FLUSH = OUT32 ? (1 << 30) : 64 / BK;   // FP64 output: FP32 sums over 64 terms of K
  double acc64[OUT32 ? 1 : TM][OUT32 ? 1 : TN][4];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = zero_f4();
  if constexpr (!OUT32) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc64[i][j][r] = 0.0;
  }

  if (nk > 0) {
    issue(0, A0, B0);
    issue(1, A1, B1);
  }
  // step t: its stage (as, bs) and the stage of step t - 1, which receives step t + 2.
  // The four are distinct arrays; saying so (restrict) lets the compiler's own wait
  // for loads into LDS tell them apart across the loop's back edge too, where it
  // otherwise waits for every load in flight once per three steps.
  auto step = [&](int64_t t, const float* __restrict__ as, const float* __restrict__ bs,
                  float* __restrict__ an, float* __restrict__ bn) {
    // this step's loads landed (the next step's NPER may still be in flight)
    __builtin_amdgcn_s_waitcnt(0xF70 | NPER);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    issue(t + 2, an, bn);
    f4_t a[TM], b[TN];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int m = wm * 16 * TM + i * 16 + l16;
      if constexpr (!TA) {
        a[i] = *reinterpret_cast<const f4_t*>(&as[m * 16 + ((lq ^ ((m >> 1) & 3)) << 2)]);
      } else {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int k = 4 * lq + kk;
          a[i][kk] = as[k * BM + (((m >> 2) ^ (k & 4)) << 2) + (m & 3)];
        }
      }
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int n = wn * 16 * TN + j * 16 + l16;
      if constexpr (TB) {
        b[j] = *reinterpret_cast<const f4_t*>(&bs[n * 16 + ((lq ^ ((n >> 1) & 3)) << 2)]);
      } else {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int k = 4 * lq + kk;
          b[j][kk] = bs[k * BN + (((n >> 2) ^ (k & 4)) << 2) + (n & 3)];
        }
      }
    }
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = mfma_f32(a[i][kk], b[j][kk], acc[i][j]);
    if constexpr (!OUT32) {
      if ((t + 1) % FLUSH == 0 || t + 1 == nk) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) {
#pragma unroll
            for (int r = 0; r < 4; ++r) acc64[i][j][r] += (double)acc[i][j][r];
            acc[i][j] = zero_f4();
          }
      }
    }
  };
  // Loop form, measured per product at the 3x3x3 cell's shapes.  Whole triples of
  // steps in the loop and the last one or two after it: no exits inside the loop,
  // which keeps the FP32-output tiles at 102-113 registers on 128 x 64 (four waves
  // per SIMD) and lets 128 x 128 fit without spilling, and ran the MN-major-A
  // products 1.5% faster.  The K-major-A, FP64-output product (M2 += A_c U_c) ran 7%
  // faster with an exit after each step, so it keeps that form.
  constexpr bool kExitEachStep = !OUT32 && !TA;
  if constexpr (kExitEachStep) {
    for (int64_t t = 0; t < nk; t += 3) {
      step(t, A0, B0, A2, B2);
      if (t + 1 >= nk) break;
      step(t + 1, A1, B1, A0, B0);
      if (t + 2 >= nk) break;
      step(t + 2, A2, B2, A1, B1);
    }
  } else {
    int64_t t = 0;
    for (; t + 3 <= nk; t += 3) {
      step(t, A0, B0, A2, B2);
      step(t + 1, A1, B1, A0, B0);
      step(t + 2, A2, B2, A1, B1);
    }
    if (t < nk) {
      step(t, A0, B0, A2, B2);
      if (t + 1 < nk) step(t + 1, A1, B1, A0, B0);
    }
  }
  // the two loads issued past the last step are still in flight: let them land
  // before the workgroup's LDS can be reused
  __builtin_amdgcn_s_waitcnt(0xF70);
  asm volatile("" ::: "memory");

#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gm = m0 + wm * 16 * TM + i * 16 + d32_row(lane, r);
        const int64_t gn = n0 + wn * 16 * TN + j * 16 + l16;
        if (gm < g.M && gn < g.N) {
          if constexpr (OUT32) {
            g.C32[gm * g.ldc + gn] = g.D32[gm * g.ldd + gn] * ((float)g.alpha * acc[i][j][r]);
          } else {
            const double v = g.alpha * acc64[i][j][r];
            if (g.splitk > 1) {
              g.work[((int64_t)bz * g.M + gm) * g.N + gn] = v;
              continue;
            }
            double* c = g.C + gm * g.ldc + gn;
            *c = (g.beta == 0.0) ? v : v + g.beta * *c;
            if (g.Cf) g.Cf[gm * g.ldcf + gn] = (float)*c;
          }
        }
      }
}

template <int TM, int TN, bool TA, bool TB, bool OUT32, int BK>
__global__ __launch_bounds__(256, 2) void gemm32v_kernel(Gemm32 g) {
  constexpr int BM = 32 * TM, BN = 32 * TN;
  constexpr int PKM = BK + 4;                      // K-major pitch
  constexpr int PAM = BM + 4, PBM = BN + 4;        // MN-major pitches
  constexpr int ASZ = TA ? BK * PAM : BM * PKM;
  constexpr int BSZ = TB ? BN * PKM : BK * PBM;
  constexpr int NA4 = BM * BK / 4 / 256, NB4 = BN * BK / 4 / 256;   // float4 per thread per step
  __shared__ __attribute__((aligned(16))) float As[2][ASZ];
  __shared__ __attribute__((aligned(16))) float Bs[2][BSZ];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int l16 = lane & 15, lq = lane >> 4;
  // Tile order (1-D grid).  Workgroups go to the eight XCDs in turn (workgroup L to
  // XCD L % 8), and each XCD has its own L2, so XCD j takes the contiguous range
  // [j per, (j + 1) per) of the tile sequence; in that sequence the K splits are
  // outermost and the output tiles run in groups of GROUP row panels, column by
  // column, so that the tiles an XCD has in flight share their row panels (A) and
  // column panels (B) in its L2.
  const int64_t tiles_n = (g.N + BN - 1) / BN, tiles_m = (g.M + BM - 1) / BM;
  const int64_t ntile = tiles_n * tiles_m * g.splitk;
  const int64_t per = ((ntile + 7) / 8);
  const int64_t T = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (T >= ntile) return;
  constexpr int64_t GROUP = 8;
  const int bz = (int)(T / (tiles_n * tiles_m));
  const int64_t T2 = T % (tiles_n * tiles_m);
  const int64_t grp = T2 / (GROUP * tiles_n), r2 = T2 % (GROUP * tiles_n);
  const int64_t gh = (tiles_m - grp * GROUP < GROUP) ? tiles_m - grp * GROUP : GROUP;
  const int64_t m0 = (grp * GROUP + r2 % gh) * BM, n0 = (r2 / gh) * BN;

  int64_t kbeg = 0, kend = g.K;
  if (g.splitk > 1) {
    const int64_t kper = ((g.K + g.splitk - 1) / g.splitk + BK - 1) / BK * BK;
    kbeg = (int64_t)bz * kper;
    kend = (kbeg + kper < g.K) ? kbeg + kper : g.K;
  }
  const int64_t nk = (kend > kbeg) ? (kend - kbeg + BK - 1) / BK : 0;
  const int64_t nread = (g.Nread > g.N) ? g.Nread : g.N;   // readable columns of B
  const bool interior = (m0 + BM <= g.M) && (n0 + BN <= nread);
  const int lda = (int)g.lda, ldb = (int)g.ldb;

  f4_t ra[NA4], rb[NB4];
  // piece i of a thread: row r = e / (C / 4), 4 columns from c = 4 (e % (C / 4)),
  // e = tid + 256 i, C the contiguous extent of the tile in global memory
  auto load = [&](int64_t k0) {
    const bool full = interior && (k0 + BK <= kend);
    const int64_t kc = (k0 < kend) ? k0 : kbeg;       // keeps the base in bounds past the last step
    const float* ba = g.A + (TA ? kc * g.lda + m0 : m0 * g.lda + kc);
    const float* bb = g.B + (TB ? n0 * g.ldb + kc : kc * g.ldb + n0);
#pragma unroll
    for (int i = 0; i < NA4; ++i) {
      const int e = tid + 256 * i;
      constexpr int CW = (TA ? BM : BK) / 4;
      const int r = TA ? e / CW : kmajor_row<CW>(e / CW), c = 4 * (e % CW);
      const float* src = ba + r * lda + c;
      if (full) {
        ra[i] = *reinterpret_cast<const f4_t*>(src);
      } else {
        // rows: m (TA = false) or k (TA = true); columns: the other.  A piece wholly
        // inside is one 16-byte load, one wholly outside is zero; only a piece that
        // straddles the edge is read element by element.
        const int64_t rm = TA ? k0 + r : m0 + r, rlim = TA ? kend : g.M;
        const int64_t cm = TA ? m0 + c : k0 + c, clim = TA ? g.M : kend;
        if (rm < rlim && cm + 4 <= clim) {
          ra[i] = *reinterpret_cast<const f4_t*>(src);
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) ra[i][j] = (rm < rlim && cm + j < clim) ? src[j] : 0.f;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NB4; ++i) {
      const int e = tid + 256 * i;
      constexpr int CW = (TB ? BK : BN) / 4;
      const int r = TB ? kmajor_row<CW>(e / CW) : e / CW, c = 4 * (e % CW);
      const float* src = bb + r * ldb + c;
      if (full) {
        rb[i] = *reinterpret_cast<const f4_t*>(src);
      } else {
        const int64_t rn = TB ? n0 + r : k0 + r, rlim = TB ? nread : kend;
        const int64_t cn = TB ? k0 + c : n0 + c, clim = TB ? kend : nread;
        if (rn < rlim && cn + 4 <= clim) {
          rb[i] = *reinterpret_cast<const f4_t*>(src);
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) rb[i][j] = (rn < rlim && cn + j < clim) ? src[j] : 0.f;
        }
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NA4; ++i) {
      const int e = tid + 256 * i;
      constexpr int CW = (TA ? BM : BK) / 4;
      const int r = TA ? e / CW : kmajor_row<CW>(e / CW), c = 4 * (e % CW);
      *reinterpret_cast<f4_t*>(&As[buf][r * (TA ? PAM : PKM) + c]) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < NB4; ++i) {
      const int e = tid + 256 * i;
      constexpr int CW = (TB ? BK : BN) / 4;
      const int r = TB ? kmajor_row<CW>(e / CW) : e / CW, c = 4 * (e % CW);
      *reinterpret_cast<f4_t*>(&Bs[buf][r * (TB ? PKM : PBM) + c]) = rb[i];
    }
  };

  f4_t acc[TM][TN];
  constexpr int FLUSH = OUT32 ? (1 << 30) : 64 / BK;   // FP64 output: FP32 sums over 64 terms of K
  double acc64[OUT32 ? 1 : TM][OUT32 ? 1 : TN][4];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = zero_f4();
  if constexpr (!OUT32) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc64[i][j][r] = 0.0;
  }

  if (nk > 0) {
    load(kbeg);
    store(0);
  }
  __syncthreads();
  for (int64_t t0 = 0; t0 < nk; t0 += FLUSH) {
    const int64_t t1 = (t0 + FLUSH < nk) ? t0 + FLUSH : nk;
    for (int64_t t = t0; t < t1; ++t) {
      load(kbeg + (t + 1) * BK);
      const float* as = As[t & 1];
      const float* bs = Bs[t & 1];
#pragma unroll
      for (int h = 0; h < BK / 16; ++h) {
        f4_t a[TM], b[TN];      // a[i][kk]: operand of step kk for row block i
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          const int m = wm * 16 * TM + i * 16 + l16;
          if constexpr (TA) {
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) a[i][kk] = as[(16 * h + 4 * lq + kk) * PAM + m];
          } else {
            a[i] = *reinterpret_cast<const f4_t*>(&as[m * PKM + 16 * h + 4 * lq]);
          }
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int n = wn * 16 * TN + j * 16 + l16;
          if constexpr (TB) {
            b[j] = *reinterpret_cast<const f4_t*>(&bs[n * PKM + 16 * h + 4 * lq]);
          } else {
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) b[j][kk] = bs[(16 * h + 4 * lq + kk) * PBM + n];
          }
        }
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
          for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = mfma_f32(a[i][kk], b[j][kk], acc[i][j]);
      }
      store((t + 1) & 1);
      __syncthreads();
    }
    if constexpr (!OUT32) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[i][j][r] += (double)acc[i][j][r];
          acc[i][j] = zero_f4();
        }
    }
  }

#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gm = m0 + wm * 16 * TM + i * 16 + d32_row(lane, r);
        const int64_t gn = n0 + wn * 16 * TN + j * 16 + l16;
        if (gm < g.M && gn < g.N) {
          if constexpr (OUT32) {
            g.C32[gm * g.ldc + gn] = g.D32[gm * g.ldd + gn] * ((float)g.alpha * acc[i][j][r]);
          } else {
            const double v = g.alpha * acc64[i][j][r];
            if (g.splitk > 1) {
              g.work[((int64_t)bz * g.M + gm) * g.N + gn] = v;
              continue;
            }
            double* c = g.C + gm * g.ldc + gn;
            *c = (g.beta == 0.0) ? v : v + g.beta * *c;
            if (g.Cf) g.Cf[gm * g.ldcf + gn] = (float)*c;
          }
        }
      }
}

// FP64 products with the operands moved from global memory straight into LDS, as
// gemm32d_kernel does for FP32: global_load_lds_dwordx4 (two doubles per lane),
// three LDS stages, loads issued two K steps ahead, one barrier per step, the loop
// unrolled over the stages with restrict stage pointers and no exit inside it.  A
// K step is 8 deep (two v_mfma_f64_16x16x4_f64 per output block); lane group q of
// instruction kk takes k = 2 q + kk, so a lane reads its two K values of a K-major
// row as one 16-byte LDS read.  K-major rows (8 doubles, four 16-byte chunks) hold
// chunk q at q ^ ((row >> 1) & 3); MN-major rows are unpermuted (a 16-lane group of
// an 8-byte read covers one 128-byte row segment).  Tiles follow the XCD-grouped
// one-dimensional order of the FP32 kernels.  Requires K and every K split a
// multiple of 8, even leading dimensions, 16-byte aligned bases and an even width
// for an MN-major operand; whole 16-byte pieces past M or N are read from the
// matrix's edge (their products reach only outputs that are not stored).
template <int TM, int TN, bool TA, bool TB>
__global__ __launch_bounds__(256, 2) void gemm64d_kernel(Gemm g) {
  constexpr int BK8 = 8;
  constexpr int BM = 32 * TM, BN = 32 * TN;
  constexpr int ASZ = BM * BK8, BSZ = BN * BK8;              // doubles per stage
  constexpr int NA = ASZ / 2 / 256, NB = BSZ / 2 / 256;      // 16-byte pieces per thread per stage
  constexpr int NPER = NA + NB;
  static_assert(NA >= 1 && NB >= 1 && NPER < 16, "stage split");
  __shared__ __attribute__((aligned(16))) double A0[ASZ], A1[ASZ], A2[ASZ];
  __shared__ __attribute__((aligned(16))) double B0[BSZ], B1[BSZ], B2[BSZ];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int l16 = lane & 15, lq = lane >> 4;
  const int64_t tiles_n = (g.N + BN - 1) / BN, tiles_m = (g.M + BM - 1) / BM;
  const int64_t ntile = tiles_n * tiles_m * g.splitk;
  const int64_t per = ((ntile + 7) / 8);
  const int64_t T = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (T >= ntile) return;
  constexpr int64_t GROUP = 8;
  const int bz = (int)(T / (tiles_n * tiles_m));
  const int64_t T2 = T % (tiles_n * tiles_m);
  const int64_t grp = T2 / (GROUP * tiles_n), r2 = T2 % (GROUP * tiles_n);
  const int64_t gh = (tiles_m - grp * GROUP < GROUP) ? tiles_m - grp * GROUP : GROUP;
  const int64_t m0 = (grp * GROUP + r2 % gh) * BM, n0 = (r2 / gh) * BN;
  if (g.lower_only && n0 > m0 + BM - 1) return;

  int64_t kbeg = 0, kend = g.K;
  if (g.splitk > 1) {
    const int64_t kper = ((g.K + g.splitk - 1) / g.splitk + BK8 - 1) / BK8 * BK8;
    kbeg = (int64_t)bz * kper;
    kend = (kbeg + kper < g.K) ? kbeg + kper : g.K;
  }
  const int64_t nk = (kend > kbeg) ? (kend - kbeg) / BK8 : 0;
  const int64_t lda = g.lda, ldb = g.ldb;

  auto src_a = [&](int P, int64_t k0) -> const double* {
    if constexpr (!TA) {                     // K-major: row P / 4, chunk P % 4
      const int r = P >> 2, q = (P & 3) ^ ((r >> 1) & 3);
      int64_t gm = m0 + r;
      if (gm >= g.M) gm = g.M - 1;
      return g.A + gm * lda + k0 + 2 * q;
    } else {                                 // MN-major: row k = P / (BM / 2)
      constexpr int CW = BM / 2;
      const int k = P / CW, c = P % CW;
      const int64_t gc = (m0 + 2 * c < g.M) ? m0 + 2 * c : m0;
      return g.A + (k0 + k) * lda + gc;
    }
  };
  auto src_b = [&](int P, int64_t k0) -> const double* {
    if constexpr (TB) {                      // K-major: row n = P / 4
      const int r = P >> 2, q = (P & 3) ^ ((r >> 1) & 3);
      int64_t gn = n0 + r;
      if (gn >= g.N) gn = g.N - 1;
      return g.B + gn * ldb + k0 + 2 * q;
    } else {                                 // MN-major: row k = P / (BN / 2)
      constexpr int CW = BN / 2;
      const int k = P / CW, c = P % CW;
      const int64_t gc = (n0 + 2 * c < g.N) ? n0 + 2 * c : n0;
      return g.B + (k0 + k) * ldb + gc;
    }
  };
  auto issue = [&](int64_t t, double* as, double* bs) {
    const int64_t k0 = kbeg + ((t < nk) ? t : nk - 1) * BK8;   // past the end: the last step again
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int run = i * 4 + wave;          // 1 KB run of this wave instruction
      __builtin_amdgcn_global_load_lds((const void*)src_a(run * 64 + lane, k0),
                                       (__attribute__((address_space(3))) void*)&as[run * 128], 16, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int run = i * 4 + wave;
      __builtin_amdgcn_global_load_lds((const void*)src_b(run * 64 + lane, k0),
                                       (__attribute__((address_space(3))) void*)&bs[run * 128], 16, 0, 0);
    }
  };

  d4_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = zero_d4();

  if (nk > 0) {
    issue(0, A0, B0);
    issue(1, A1, B1);
  }
  auto step = [&](int64_t t, const double* __restrict__ as, const double* __restrict__ bs,
                  double* __restrict__ an, double* __restrict__ bn) {
    __builtin_amdgcn_s_waitcnt(0xF70 | NPER);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    issue(t + 2, an, bn);
    double a[TM][2], b[TN][2];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int m = wm * 16 * TM + i * 16 + l16;
      if constexpr (!TA) {
        const d2_t v = *reinterpret_cast<const d2_t*>(&as[m * 8 + ((lq ^ ((m >> 1) & 3)) << 1)]);
        a[i][0] = v[0];
        a[i][1] = v[1];
      } else {
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) a[i][kk] = as[(2 * lq + kk) * BM + m];
      }
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int n = wn * 16 * TN + j * 16 + l16;
      if constexpr (TB) {
        const d2_t v = *reinterpret_cast<const d2_t*>(&bs[n * 8 + ((lq ^ ((n >> 1) & 3)) << 1)]);
        b[j][0] = v[0];
        b[j][1] = v[1];
      } else {
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) b[j][kk] = bs[(2 * lq + kk) * BN + n];
      }
    }
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = mfma_f64(a[i][kk], b[j][kk], acc[i][j]);
  };
  int64_t t = 0;
  for (; t + 3 <= nk; t += 3) {
    step(t, A0, B0, A2, B2);
    step(t + 1, A1, B1, A0, B0);
    step(t + 2, A2, B2, A1, B1);
  }
  if (t < nk) {
    step(t, A0, B0, A2, B2);
    if (t + 1 < nk) step(t + 1, A1, B1, A0, B0);
  }
  // the two loads issued past the last step are still in flight: let them land
  // before the workgroup's LDS can be reused
  __builtin_amdgcn_s_waitcnt(0xF70);
  asm volatile("" ::: "memory");

#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gm = m0 + wm * 16 * TM + i * 16 + d64_row(lane, r);
        const int64_t gn = n0 + wn * 16 * TN + j * 16 + l16;
        if (gm < g.M && gn < g.N) {
          const double v = g.alpha * acc[i][j][r];
          if (g.splitk > 1) {
            g.work[((int64_t)bz * g.M + gm) * g.N + gn] = v;
            continue;
          }
          double* c = g.C + gm * g.ldc + gn;
          if (g.epi == EPI_SQUARE) *c = v * v;
          else if (g.epi == EPI_HADAMARD) *c = *c * v;
          else if (g.epi == EPI_HADAMARD_SRC) *c = (g.D ? g.D[gm * g.ldd + gn] : (double)g.D32[gm * g.ldd + gn]) * v;
          else {
            *c = (g.beta == 0.0) ? v : v + g.beta * *c;
            if (g.Cf) g.Cf[gm * g.ldcf + gn] = (float)*c;
          }
        }
      }
}

// 128 x 64 tiles without the row scale fit three waves per SIMD (168 registers)
template <int TM, int TN, bool TA, bool TB, bool KS = false>
__global__ __launch_bounds__(256, (TN == 2 && !KS) ? 3 : 2) void gemm_big_kernel(Gemm g) {
  gemm_big_body<TM, TN, TA, TB, KS>(g, (int64_t)blockIdx.y * 32 * TM, (int64_t)blockIdx.x * 32 * TN, blockIdx.z);
}

// Many independent products in one launch: item blockIdx.z takes the base operands
// at its own offsets, sizes and pitches (no K split).
template <int TM, int TN, bool TA, bool TB, bool KS>
__global__ __launch_bounds__(256, 2) void gemm_grouped_kernel(Gemm base, const GemmItem* __restrict__ items) {
  const GemmItem it = items[blockIdx.z];
  const int64_t m0 = (int64_t)blockIdx.y * 32 * TM, n0 = (int64_t)blockIdx.x * 32 * TN;
  if (m0 >= it.M || n0 >= it.N) return;
  Gemm g = base;
  g.M = it.M; g.N = it.N; g.K = it.K;
  g.lda = it.lda; g.ldb = it.ldb; g.ldc = it.ldc;
  g.A = base.A + it.aofs; g.B = base.B + it.bofs; g.C = base.C + it.cofs;
  if (KS) g.kscale = base.kscale + it.kofs;
  g.splitk = 1;
  gemm_big_body<TM, TN, TA, TB, KS>(g, m0, n0, 0);
}

// C = alpha * sum_z work[z] + beta * C (fixed order over z)
__global__ void splitk_reduce_kernel(const double* __restrict__ work, int splitk, int64_t M, int64_t N,
                                     double* __restrict__ C, int64_t ldc, double beta, float* __restrict__ Cf,
                                     int64_t ldcf) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= M * N) return;
  double s = 0.0;
  for (int z = 0; z < splitk; ++z) s += work[(int64_t)z * M * N + t];
  const int64_t m = t / N, n = t % N;
  double* c = C + m * ldc + n;
  *c = (beta == 0.0) ? s : s + beta * *c;
  if (Cf) Cf[m * ldcf + n] = (float)*c;
}

template <int TM, int TN>
void launch_big(const Gemm& g, dim3 grid, hipStream_t s) {
  if (g.kscale) hipLaunchKernelGGL((gemm_big_kernel<TM, TN, true, false, true>), grid, dim3(256), 0, s, g);
  else if (!g.transA && !g.transB) hipLaunchKernelGGL((gemm_big_kernel<TM, TN, false, false>), grid, dim3(256), 0, s, g);
  else if (g.transA && !g.transB) hipLaunchKernelGGL((gemm_big_kernel<TM, TN, true, false>), grid, dim3(256), 0, s, g);
  else if (!g.transA && g.transB) hipLaunchKernelGGL((gemm_big_kernel<TM, TN, false, true>), grid, dim3(256), 0, s, g);
  else hipLaunchKernelGGL((gemm_big_kernel<TM, TN, true, true>), grid, dim3(256), 0, s, g);
}

template <int TN>
void launch64d(const Gemm& g, dim3 grid, hipStream_t s) {
  if (!g.transA && !g.transB) hipLaunchKernelGGL((gemm64d_kernel<4, TN, false, false>), grid, dim3(256), 0, s, g);
  else if (g.transA && !g.transB) hipLaunchKernelGGL((gemm64d_kernel<4, TN, true, false>), grid, dim3(256), 0, s, g);
  else if (!g.transA && g.transB) hipLaunchKernelGGL((gemm64d_kernel<4, TN, false, true>), grid, dim3(256), 0, s, g);
  else hipLaunchKernelGGL((gemm64d_kernel<4, TN, true, true>), grid, dim3(256), 0, s, g);
}

// the LDS-direct FP64 kernel's requirements (see gemm64d_kernel)
bool direct64_ok(const Gemm& g) {
  auto al = [](const void* p) { return ((uintptr_t)p & 15u) == 0; };
  if (g.kscale || g.K % 8 != 0 || g.lda % 2 || g.ldb % 2 || !al(g.A) || !al(g.B)) return false;
  if ((g.transA && g.M % 2) || (!g.transB && g.N % 2)) return false;
  // both operands K-major over a long K (W = V chi^T at set-up): each 8-deep step
  // touches 64 bytes of every one of 192 rows megabytes apart, and the register-staged
  // kernel's 16-deep steps ran faster there
  if (!g.transA && g.transB && g.K > 16384) return false;
  const char* v = getenv("RPS_GEMM64_DIRECT");    // "0": the register-staged kernel (comparison runs)
  return !(v && v[0] == '0');
}

// Output tile width: 16 for skinny products, 64 when N <= 64, else 128 (all 128 rows high).
int gemm_tile_n(int64_t M, int64_t N) {
  (void)M;
  return (N <= 16) ? 16 : (N <= 64) ? 64 : 128;
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
  if (g.epi == EPI_HADAMARD_SRC && !g.D && !g.D32) return hipErrorInvalidValue;
  if (g.Cf && (g.epi != EPI_AXPBY || g.keep_partials)) return hipErrorInvalidValue;
  if (g.splitk < 1) g.splitk = 1;
  int bn = gemm_tile_n(g.M, g.N);
  if (g.tile_n) {
    if ((g.tile_n != 64 && g.tile_n != 128) || g.N <= 16) return hipErrorInvalidValue;
    bn = g.tile_n;
  }
  if (g.kscale && bn != 16 && !(g.transA && !g.transB)) return hipErrorInvalidValue;
  if (bn == 16) {
    dim3 grid((unsigned)((g.N + 15) / 16), (unsigned)((g.M + 127) / 128), (unsigned)g.splitk);
    hipLaunchKernelGGL((gemm_kernel<4, 2, 1>), grid, dim3(256), 0, s, g);
  } else if (direct64_ok(g)) {
    // 128 x 64 tiles (three waves per SIMD; 128 x 128 holds two and ran slower on the
    // set-up's updates), one-dimensional grid in XCD-grouped tile order, padded to
    // whole rounds of eight
    const int64_t ntile = ((g.N + 63) / 64) * ((g.M + 127) / 128) * g.splitk;
    if (ntile > (int64_t)UINT32_MAX - 8) return hipErrorInvalidValue;
    launch64d<2>(g, dim3((unsigned)((ntile + 7) / 8 * 8)), s);
  } else if (bn == 64) {
    dim3 grid((unsigned)((g.N + 63) / 64), (unsigned)((g.M + 127) / 128), (unsigned)g.splitk);
    launch_big<4, 2>(g, grid, s);
  } else {
    dim3 grid((unsigned)((g.N + 127) / 128), (unsigned)((g.M + 127) / 128), (unsigned)g.splitk);
    launch_big<4, 4>(g, grid, s);
  }
  if (g.splitk > 1 && !g.keep_partials) {
    const int64_t cnt = g.M * g.N;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, g.work,
                       g.splitk, g.M, g.N, g.C, g.ldc, g.beta, g.Cf, g.ldcf);
  }
  return hipGetLastError();
}

namespace {
template <int TN, bool OUT32>
void launch32(const Gemm32& g, dim3 grid, hipStream_t s) {
  if (!g.transA && !g.transB) hipLaunchKernelGGL((gemm32_kernel<4, TN, false, false, OUT32>), grid, dim3(256), 0, s, g);
  else if (g.transA && !g.transB) hipLaunchKernelGGL((gemm32_kernel<4, TN, true, false, OUT32>), grid, dim3(256), 0, s, g);
  else if (!g.transA && g.transB) hipLaunchKernelGGL((gemm32_kernel<4, TN, false, true, OUT32>), grid, dim3(256), 0, s, g);
  else hipLaunchKernelGGL((gemm32_kernel<4, TN, true, true, OUT32>), grid, dim3(256), 0, s, g);
}
template <int TN, bool OUT32, int BK>
void launch32v_bk(const Gemm32& g, dim3 grid, hipStream_t s) {
  if (!g.transA && !g.transB) hipLaunchKernelGGL((gemm32v_kernel<4, TN, false, false, OUT32, BK>), grid, dim3(256), 0, s, g);
  else if (g.transA && !g.transB) hipLaunchKernelGGL((gemm32v_kernel<4, TN, true, false, OUT32, BK>), grid, dim3(256), 0, s, g);
  else if (!g.transA && g.transB) hipLaunchKernelGGL((gemm32v_kernel<4, TN, false, true, OUT32, BK>), grid, dim3(256), 0, s, g);
  else hipLaunchKernelGGL((gemm32v_kernel<4, TN, true, true, OUT32, BK>), grid, dim3(256), 0, s, g);
}
// K steps of 16: at the 3x3x3 cell's chunk shapes they measured 102-110 TF/s against
// 98-106 TF/s with steps of 32 (twice the LDS and prefetch registers per workgroup)
template <int TN, bool OUT32>
void launch32d(const Gemm32& g, dim3 grid, hipStream_t s) {
  if (!g.transA && !g.transB) hipLaunchKernelGGL((gemm32d_kernel<4, TN, false, false, OUT32>), grid, dim3(256), 0, s, g);
  else if (g.transA && !g.transB) hipLaunchKernelGGL((gemm32d_kernel<4, TN, true, false, OUT32>), grid, dim3(256), 0, s, g);
  else if (!g.transA && g.transB) hipLaunchKernelGGL((gemm32d_kernel<4, TN, false, true, OUT32>), grid, dim3(256), 0, s, g);
  else hipLaunchKernelGGL((gemm32d_kernel<4, TN, true, true, OUT32>), grid, dim3(256), 0, s, g);
}

template <int TN, bool OUT32>
void launch32v(const Gemm32& g, dim3 grid, hipStream_t s) {
  launch32v_bk<TN, OUT32, 16>(g, grid, s);
}
// 16-byte operand traffic needs 4-float aligned rows and bases
bool vec4_ok(const Gemm32& g) {
  auto al = [](const void* p) { return ((uintptr_t)p & 15u) == 0; };
  if (g.lda % 4 || g.ldb % 4 || !al(g.A) || !al(g.B)) return false;
  if (g.C32 && (g.ldd % 4 || !al(g.D32))) return false;
  const char* v = getenv("RPS_GEMM32_SCALAR");     // comparison runs: the scalar-traffic kernel
  return !(v && v[0] == '1');
}
}  // namespace

int gemm32_tile_n(int64_t N) {
  // 128-wide output tiles unless 64-wide ones pad N less (N = 432: 448 against 512)
  const int64_t p128 = (N + 127) / 128 * 128, p64 = (N + 63) / 64 * 64;
  return (p64 < p128) ? 64 : 128;
}

hipError_t gemm_f32(const Gemm32& g0, hipStream_t s) {
  Gemm32 g = g0;
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  const bool out32 = g.C32 != nullptr;
  if (out32 && (!g.D32 || g.splitk > 1 || g.Cf)) return hipErrorInvalidValue;
  if (!out32 && !g.C) return hipErrorInvalidValue;
  if (g.splitk > 1 && !g.work) return hipErrorInvalidValue;
  if (g.splitk < 1) g.splitk = 1;
  // 32-bit per-lane offsets inside a tile (at most 128 rows of either operand)
  if (g.lda > INT32_MAX / 128 || g.ldb > INT32_MAX / 128) return hipErrorInvalidValue;
  // operands straight into LDS when every K step is whole (K a multiple of 16),
  // otherwise the register-staged kernel; FP64 output on 128 x 64 tiles, FP32 output
  // on 128 x 128 unless 128 x 64 pads N less
  const char* dv = getenv("RPS_GEMM32_DIRECT");    // "0": the register-staged kernel (comparison runs)
  const bool vec = vec4_ok(g);
  const bool direct = vec && g.K % 16 == 0 && !(dv && dv[0] == '0');
  const int bn = out32 ? gemm32_tile_n(g.N) : 64;
  dim3 grid((unsigned)((g.N + bn - 1) / bn), (unsigned)((g.M + 127) / 128), (unsigned)g.splitk);
  if (grid.y > 65535u) return hipErrorInvalidValue;
  // the 16-byte kernels order their tiles themselves: one dimension, padded to whole rounds
  // of the eight XCDs (the padding workgroups exit at once)
  const int64_t ntile = (int64_t)grid.x * grid.y * grid.z;
  const dim3 grid1((unsigned)((ntile + 7) / 8 * 8));
  if (vec && ntile > (int64_t)UINT32_MAX - 8) return hipErrorInvalidValue;
  if (bn == 64) {
    if (direct) { if (out32) launch32d<2, true>(g, grid1, s); else launch32d<2, false>(g, grid1, s); }
    else if (vec) { if (out32) launch32v<2, true>(g, grid1, s); else launch32v<2, false>(g, grid1, s); }
    else { if (out32) launch32<2, true>(g, grid, s); else launch32<2, false>(g, grid, s); }
  } else {
    if (direct) launch32d<4, true>(g, grid1, s);
    else if (vec) launch32v<4, true>(g, grid1, s);
    else launch32<4, true>(g, grid, s);
  }
  if (g.splitk > 1) {
    const int64_t cnt = g.M * g.N;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, g.work,
                       g.splitk, g.M, g.N, g.C, g.ldc, g.beta, g.Cf, g.ldcf);
  }
  return hipGetLastError();
}

int gemm32_splitk_for(int64_t M, int64_t N, int64_t K, int64_t kmax, int64_t work_cap_doubles) {
  // K per split at most kmax, then >= 1024 workgroups while each split keeps
  // >= 1024 of K, within the workspace (FP64-output tiles are 128 x 64)
  const int bn = 64;
  const int64_t tiles = ((M + 127) / 128) * ((N + bn - 1) / bn);
  // among the split counts that keep >= 1024 of K per split, the one whose workgroups
  // fill the last round of 768 (three per CU, as the FP64-output tiles run) best, the
  // smaller on a tie
  int64_t z0 = 1;
  while ((K + z0 - 1) / z0 > kmax) ++z0;
  int64_t best = z0;
  double best_fill = -1.0;
  for (int64_t z = z0; z <= z0 + 7; ++z) {
    if (z > z0 && K / z < 1024) break;
    if (z > 1 && z * M * N > work_cap_doubles) break;
    const int64_t wgs = tiles * z, rounds = (wgs + 767) / 768;
    const double fill = (double)wgs / (double)(rounds * 768) + (rounds > 1 ? 0.0 : -0.5);
    if (fill > best_fill + 1e-9) { best_fill = fill; best = z; }
  }
  return (int)best;
}

namespace {
template <int TN>
void launch_grouped(const Gemm& g, const GemmItem* items, dim3 grid, hipStream_t s) {
  if (g.kscale) hipLaunchKernelGGL((gemm_grouped_kernel<4, TN, true, false, true>), grid, dim3(256), 0, s, g, items);
  else if (!g.transA && !g.transB)
    hipLaunchKernelGGL((gemm_grouped_kernel<4, TN, false, false, false>), grid, dim3(256), 0, s, g, items);
  else if (g.transA && !g.transB)
    hipLaunchKernelGGL((gemm_grouped_kernel<4, TN, true, false, false>), grid, dim3(256), 0, s, g, items);
  else if (!g.transA && g.transB)
    hipLaunchKernelGGL((gemm_grouped_kernel<4, TN, false, true, false>), grid, dim3(256), 0, s, g, items);
  else hipLaunchKernelGGL((gemm_grouped_kernel<4, TN, true, true, false>), grid, dim3(256), 0, s, g, items);
}
}  // namespace

hipError_t gemm_f64_grouped(const Gemm& base, const GemmItem* items, int nitems, int64_t maxM, int64_t maxN,
                            hipStream_t s) {
  if (nitems <= 0 || maxM <= 0 || maxN <= 0) return hipSuccess;
  if (nitems > 65535 || base.splitk > 1 || base.epi != EPI_AXPBY || base.Cf) return hipErrorInvalidValue;
  if (base.kscale && !(base.transA && !base.transB)) return hipErrorInvalidValue;
  const int bn = (maxN <= 64) ? 64 : 128;
  dim3 grid((unsigned)((maxN + bn - 1) / bn), (unsigned)((maxM + 127) / 128), (unsigned)nitems);
  if (grid.y > 65535u) return hipErrorInvalidValue;
  if (bn == 64) launch_grouped<2>(base, items, grid, s);
  else launch_grouped<4>(base, items, grid, s);
  return hipGetLastError();
}

void gemm_plan(Gemm& g, int64_t work_cap_doubles) {
  g.tile_n = 0;
  g.splitk = 1;
  if (g.epi != EPI_AXPBY || g.kscale || g.N <= 64) {
    g.splitk = gemm_splitk_for(g.M, g.N, g.K, work_cap_doubles);
    return;
  }
  // the LDS-direct kernel runs 128 x 64 tiles, three workgroups per CU; the
  // register-staged one 128 x 64 or 128 x 128, two per CU
  const bool direct = direct64_ok(g);
  const int64_t slots = direct ? 768 : 512;
  double best = -1.0;
  for (int bn = direct ? 64 : 128; bn >= 64; bn -= 64) {
    const int64_t padn = (g.N + bn - 1) / bn * bn;
    const int64_t tiles = ((g.M + 127) / 128) * (padn / bn);
    for (int64_t z = 1; z <= 64; ++z) {
      if (z > 1 && (g.K / z < 256 || z * g.M * g.N > work_cap_doubles)) break;
      const int64_t wgs = tiles * z, rounds = (wgs + slots - 1) / slots;
      const double score = (double)g.N / (double)padn * (double)wgs / (double)(rounds * slots);
      if (score > best + 1e-9) {
        best = score;
        g.tile_n = bn;
        g.splitk = (int)z;
      }
    }
  }
}

int gemm_splitk_for(int64_t M, int64_t N, int64_t K, int64_t work_cap_doubles) {
  // aim for >= 512 workgroups, at least 256 K per split, bounded by the workspace
  const int bn = gemm_tile_n(M, N);
  const int64_t tiles = ((M + 127) / 128) * ((N + bn - 1) / bn);
  int64_t z = 1;
  while (tiles * z < 512 && K / (z * 2) >= 256 && (z * 2) * M * N <= work_cap_doubles) z *= 2;
  return (int)z;
}

}  // namespace rps
