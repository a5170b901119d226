// Streaming contractions of lines 1-2 (and 3) of Eq. 16 for general sizes.
//
// For the product  O[x][c] = sum_y S[x][y] (sum_d X[x][d] Y[y][d]) Y[y][c]
// with S the stored potential (V or W) and X, Y orbital values, one workgroup
// owns 16 NW rows x and streams all (or a split of the) y: for every 32-row
// tile of Y (staged through LDS, double buffered) each wave forms the 16 x 16
// tile P^T[y][x] with the matrix cores (inner dimension n), multiplies it by the
// matching S values in registers, and feeds the result straight back into the
// matrix cores as the A operand of O += A Y (inner dimension y).  O stays in
// registers for the whole pass: nothing of size N_aux x N_g is ever stored.
//
// Two passes cover Eq. 16 (Sec. 3.3, Sec. 4.4 order):
//   x = g (rows of V),    y = R, X = U_g, Y = U:   O = M2   = (V o P) U
//   x = R (columns of V), y = g, X = U,   Y = U_g: O = M1^T = (V o P)^T U_g
// and the fit-fit line is the first form on W with X = Y = U_g.
//
// Fragment layout (16x16x4 MFMA, lane l, q = l / 16, l16 = l % 16): the S tile
// register r of lane l holds y = 4q + r, x = l16 for both FP64 and FP32 (the
// FP64 form reads its Y operand rows in the order 4(m % 4) + m / 4 to get it),
// which is exactly the A operand of the O product at k-step r.  So V is read
// as four consecutive values of one row per lane (x = rows) or as coalesced
// rows (x = columns), and P never leaves the registers.
//
// Precision: TM = double is FP64 throughout.  TM = float reads the FP32 copy
// of V, rounds X and Y to FP32, accumulates each 32-row tile in FP32 and adds
// it to FP64 accumulators, so error does not grow with N_g.  The split-BF16
// form is a separate kernel below.
#include <type_traits>

#include "mfma.h"
#include "rps_internal.h"

namespace rps {
namespace {

constexpr int BY = 32;   // y rows per LDS tile

template <typename TM>
struct Frag;
template <>
struct Frag<double> {
  using acc = d4_t;
  static __device__ __forceinline__ acc zero() { return zero_d4(); }
  static __device__ __forceinline__ acc mma(double a, double b, acc c) { return mfma_f64(a, b, c); }
};
template <>
struct Frag<float> {
  using acc = f4_t;
  static __device__ __forceinline__ acc zero() { return zero_f4(); }
  static __device__ __forceinline__ acc mma(float a, float b, acc c) { return mfma_f32(a, b, c); }
};

// Y tile pitch.  FP32: 16 NC + 4 = 4 x odd, so the two read patterns of a wave
// (row l16 at column 4 j + lq, and row 4 lq + r at column l16 + 16 cb) fall on
// 64 distinct banks.
template <typename TM, int NC>
__host__ __device__ constexpr int stream_ldy() {
  return std::is_same<TM, float>::value ? 16 * NC + 4 : 16 * NC + 1;
}

// One work item of a pass: x block bx (16 NW rows) and y split by.
template <typename TM, int NC, int TRANS, int NW>
__device__ __forceinline__ void stream_body(const StreamArgs& a, int64_t bx, int64_t by, unsigned char* smem_raw) {
  using F = Frag<TM>;
  using acc_t = typename F::acc;
  constexpr bool F64 = std::is_same<TM, double>::value;
  constexpr int NP = 16 * NC;
  constexpr int NK = NP / 4;
  constexpr int LDY = stream_ldy<TM, NC>();
  constexpr int PER = BY * NP / (NW * 64);   // staged Y elements per thread
  static_assert(PER * NW * 64 == BY * NP, "tile split");
  TM* sY = reinterpret_cast<TM*>(smem_raw);

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, lq = lane >> 4;
  const int64_t x0 = (bx * NW + w) * 16;
  const bool xvalid = x0 < a.nx;
  const int64_t xrow = xvalid ? x0 : a.nx - 16;   // rows read by a wave past the end (discarded)
  const int64_t ys = by * a.ysplit;
  const int64_t ye = (ys + a.ysplit < a.ny) ? ys + a.ysplit : a.ny;
  const int64_t ntile = (ye > ys) ? (ye - ys) / BY : 0;

  // X operand (B of the P^T product): lane holds X[x0 + l16][4j + lq]
  TM xr[NK];
#pragma unroll
  for (int j = 0; j < NK; ++j) xr[j] = xvalid ? (TM)a.X[(x0 + l16) * a.ldx + 4 * j + lq] : (TM)0;

  acc_t o[NC];
#pragma unroll
  for (int cb = 0; cb < NC; ++cb) o[cb] = F::zero();
  double od[F64 ? 1 : NC][4];
  if constexpr (!F64) {
#pragma unroll
    for (int cb = 0; cb < NC; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) od[cb][r] = 0.0;
  }

  // Y tile staging (rows are contiguous: ldy == np); the FP32 form reads the FP32
  // copy of Y (Y is re-read by every x block, so this halves the dominant traffic)
  TM ystage[PER];
  auto stage_load = [&](int64_t t) {
    if constexpr (F64) {
      const double* src = a.Y + (ys + t * BY) * a.ldy;
#pragma unroll
      for (int k = 0; k < PER; ++k) ystage[k] = src[tid + k * NW * 64];
    } else {
      const float* src = a.Y32 + (ys + t * BY) * a.ldy;
#pragma unroll
      for (int k = 0; k < PER; ++k) ystage[k] = src[tid + k * NW * 64];
    }
  };
  auto stage_store = [&](int buf) {
    TM* dst = sY + buf * BY * LDY;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = tid + k * NW * 64;
      dst[(e / NP) * LDY + (e % NP)] = (TM)ystage[k];
    }
  };

  // S operand row of the P^T product for lane l16 (see the header)
  const int yrowA = F64 ? 4 * (l16 & 3) + (l16 >> 2) : l16;

  // S values of a tile: lane holds S[x0 + l16][y] for y = tile + 16 sb + 4 lq + r
  TM vv[2][4], vn[2][4];
  auto load_s = [&](int64_t t, TM (&d)[2][4]) {
    const int64_t yb = ys + ((t < ntile) ? t : ntile - 1) * BY;   // past the last tile: re-read it
#pragma unroll
    for (int sb = 0; sb < 2; ++sb) {
      const int64_t y0 = yb + 16 * sb + 4 * lq;
      if constexpr (TRANS == 0) {
        if constexpr (F64) {
          const double* p = a.V + (xrow + l16) * a.ldv + y0;
          const double2 u0 = *reinterpret_cast<const double2*>(p);
          const double2 u1 = *reinterpret_cast<const double2*>(p + 2);
          d[sb][0] = u0.x; d[sb][1] = u0.y; d[sb][2] = u1.x; d[sb][3] = u1.y;
        } else {
          const float4 u = *reinterpret_cast<const float4*>(a.V32 + (xrow + l16) * a.ldv + y0);
          d[sb][0] = u.x; d[sb][1] = u.y; d[sb][2] = u.z; d[sb][3] = u.w;
        }
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if constexpr (F64) d[sb][r] = a.V[(y0 + r) * a.ldv + xrow + l16];
          else d[sb][r] = a.V32[(y0 + r) * a.ldv + xrow + l16];
        }
      }
    }
  };

  if (ntile > 0) {
    stage_load(0);
    stage_store(0);
    load_s(0, vv);
  }
  __syncthreads();
  // Every load of the loop is unconditional (past the last tile the last one is re-read
  // and staged into the idle buffer), so the wait before each use counts the loads
  // exactly instead of falling back to waiting for all of them.
  for (int64_t t = 0; t < ntile; ++t) {
    stage_load(t + 1 < ntile ? t + 1 : t);
    load_s(t + 1, vn);    // the next tile's S values, a tile ahead
    const TM* sy = sY + (t & 1) * BY * LDY;
    if (xvalid) {
#pragma unroll
      for (int sb = 0; sb < 2; ++sb) {
        // operands of the two products read from LDS into registers first, so that
        // the reads are in flight together instead of one per matrix-core step
        const TM* ya = sy + (16 * sb + yrowA) * LDY + lq;
        const TM* yb_ = sy + (16 * sb + 4 * lq) * LDY + l16;
        TM pa[NK], ob[4][NC];
#pragma unroll
        for (int j = 0; j < NK; ++j) pa[j] = ya[4 * j];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int cb = 0; cb < NC; ++cb) ob[r][cb] = yb_[r * LDY + 16 * cb];
        // FP32: keep the reads above the products (the scheduler otherwise interleaves
        // one read and its full wait per two matrix-core steps); the FP64 operands would
        // not fit in registers together
        if constexpr (!F64) __builtin_amdgcn_sched_barrier(0);
        // P^T[y][x] = sum_d Y[y][d] X[x][d]
        acc_t s = F::zero();
#pragma unroll
        for (int j = 0; j < NK; ++j) s = F::mma(pa[j], xr[j], s);
        // A = S o P, straight into the O product (k-step r <-> y = 4 lq + r)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const TM av = s[r] * vv[sb][r];
#pragma unroll
          for (int cb = 0; cb < NC; ++cb) o[cb] = F::mma(av, ob[r][cb], o[cb]);
        }
      }
      if constexpr (!F64) {
#pragma unroll
        for (int cb = 0; cb < NC; ++cb) {
#pragma unroll
          for (int r = 0; r < 4; ++r) od[cb][r] += (double)o[cb][r];
          o[cb] = F::zero();
        }
      }
    }
#pragma unroll
    for (int sb = 0; sb < 2; ++sb)
#pragma unroll
      for (int r = 0; r < 4; ++r) vv[sb][r] = vn[sb][r];
    stage_store((t + 1) & 1);
    __syncthreads();
  }

  if (!xvalid) return;
  double* out = a.out + (by * a.nx) * a.np;
#pragma unroll
  for (int cb = 0; cb < NC; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t x = F64 ? x0 + 4 * r + lq : x0 + 4 * lq + r;
      double v;
      if constexpr (F64) v = o[cb][r];
      else v = od[cb][r];
      out[x * a.np + 16 * cb + l16] = v;
    }
}


template <typename TM, int NC, int TRANS, int NW>
__global__ __launch_bounds__(NW * 64) void stream_kernel(StreamArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  stream_body<TM, NC, TRANS, NW>(a, blockIdx.x, blockIdx.y, smem_raw);
}

// Persistent form for the batching form: the work items of one pass class
// (precision, n, orientation) over many cells, taken from a device queue in
// list order (longest first) until it runs dry; every workgroup ends when the
// counter passes the last item.  items[i] = (cell, x block, y split) and
// args[cell] the cell's pass; *counter is zero at launch.
template <typename TM, int NC, int TRANS, int NW>
__global__ __launch_bounds__(NW * 64) void stream_queue_kernel(const StreamArgs* __restrict__ args,
                                                              const StreamItem* __restrict__ items, int nitems,
                                                              unsigned* __restrict__ counter) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int s_item;
  while (true) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int i = s_item;
    __syncthreads();
    if (i >= nitems) break;
    const StreamItem it = items[i];
    const StreamArgs a = args[it.cell];
    stream_body<TM, NC, TRANS, NW>(a, it.bx, it.by, smem_raw);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Split-BF16 form (precision RPS_PREC_BF16X3) on v_mfma_f32_16x16x32_bf16
// with FP32 accumulation inside a tile and FP64 across tiles.  Every operand
// is split into three BF16 terms by repeated round-to-nearest, x = h + m + l
// (24 significant bits, as FP32), and each product keeps the six term
// products down to 2^-16 of the leading one (the dropped ones are at or below
// 2^-24, FP32 rounding level):
//   a b ~ ah bh + ah bm + am bh + ah bl + al bh + am bm
// A two-term split (16 bits) was not enough: the orbital values X and Y enter
// every product with the same rounding error, which then acts like a fixed
// perturbation of the orbitals, and the sums over the points behind K cancel
// strongly; both put |dE_x| above 1e-6 Ha on test cells.
// Dataflow as in the FP64/FP32 kernel with K = 32 per instruction:
//   P^T tile: A operand = Y rows (LDS, row-major planes), B = X (registers),
//             k <-> d = 32 j + 8 q + e;
//   O += A Y: A operand straight from the two P^T tiles of a 32-row tile with
//             k = 8 q + e <-> y = 4 q + e (e < 4) or 16 + 4 q + e - 4 (e >= 4),
//             B operand from transposed planes of the Y tile in LDS.
typedef __bf16 bf4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void split3_bf16(float x, __bf16& h, __bf16& m, __bf16& l) {
  h = (__bf16)x;
  const float r = x - (float)h;
  m = (__bf16)r;
  l = (__bf16)(r - (float)m);
}

template <int NC>
struct Bf16Layout {
  static constexpr int NP = 16 * NC;
  static constexpr int NKC = (NP + 31) / 32;   // K chunks of the P^T product
  static constexpr int NPP = NKC * 32;         // n padded to whole chunks (zero tail)
  static constexpr int LR = NPP + 8;           // row-major plane pitch (bf16), 16-byte rows
  static constexpr int LT = BY + 4;            // transposed plane pitch (bf16): 18 dwords, so the
                                               // 8-byte reads of 16 consecutive columns hit 32 banks
  static constexpr int SZR = BY * LR, SZT = NP * LT;
  static constexpr int BUF = 3 * SZR + 3 * SZT;   // bf16 per buffer: Y h/m/l, Y^T h/m/l
  // Two staging buffers (one barrier per tile), 108 KB at n = 128: one workgroup of
  // eight waves per CU.  One buffer (two barriers, two workgroups per CU) measured
  // the same at n = 128.
  static constexpr int NBUF = 2;
  static constexpr size_t LDS_BYTES = (size_t)NBUF * BUF * 2;
};

template <int NC, int TRANS, int NW>
__device__ __forceinline__ void bf16x3_body(const StreamArgs& a, int64_t bx, int64_t by, unsigned char* smem_raw) {
  using L = Bf16Layout<NC>;
  constexpr int NP = L::NP, NKC = L::NKC, NPP = L::NPP, LR = L::LR, LT = L::LT;
  constexpr int SZR = L::SZR, SZT = L::SZT;
  constexpr int PER = BY * NP / (NW * 64);
  static_assert(PER * NW * 64 == BY * NP, "tile split");
  __bf16* sm = reinterpret_cast<__bf16*>(smem_raw);

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, lq = lane >> 4;
  const int64_t x0 = (bx * NW + w) * 16;
  const bool xvalid = x0 < a.nx;
  const int64_t xrow = xvalid ? x0 : a.nx - 16;   // rows read by a wave past the end (discarded)
  const int64_t ys = by * a.ysplit;
  const int64_t ye = (ys + a.ysplit < a.ny) ? ys + a.ysplit : a.ny;
  const int64_t ntile = (ye > ys) ? (ye - ys) / BY : 0;

  // X operand of the P^T product in three terms: lane holds X[x0 + l16][32 j + 8 lq + e]
  bf8_t xh[NKC], xm[NKC], xl[NKC];
#pragma unroll
  for (int j = 0; j < NKC; ++j)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int d = 32 * j + 8 * lq + e;
      const float v = (xvalid && d < NP) ? (float)a.X[(x0 + l16) * a.ldx + d] : 0.f;
      __bf16 h, m, l;
      split3_bf16(v, h, m, l);
      xh[j][e] = h;
      xm[j][e] = m;
      xl[j][e] = l;
    }

  // zero tail columns [NP, NPP) of the row-major planes of every buffer (never staged)
  if constexpr (NPP > NP) {
    constexpr int TAIL = BY * (NPP - NP);
    for (int e = tid; e < L::NBUF * 3 * TAIL; e += NW * 64) {
      const int plane = e / TAIL, rem = e % TAIL;
      const int r = rem / (NPP - NP), c = NP + rem % (NPP - NP);
      sm[(plane / 3) * L::BUF + (plane % 3) * SZR + r * LR + c] = (__bf16)0.f;
    }
  }

  f4_t o[NC];
  double od[NC][4];
#pragma unroll
  for (int cb = 0; cb < NC; ++cb) {
    o[cb] = zero_f4();
#pragma unroll
    for (int r = 0; r < 4; ++r) od[cb][r] = 0.0;
  }

  // Staging order: element k of a wave is one 8 x 8 block of the tile (rows
  // 8 (b % 4) + lane / 8, columns 8 (b / 4) + lane % 8, b = w + NW k).  With row
  // pitch LR/2 = 4 or 20 (mod 32) dwords such a block puts its 64 two-byte stores
  // on 32 distinct banks of the row-major planes (two lanes per dword) and, with
  // column pitch LT/2 = 18 dwords, on at most two dwords per bank of the
  // transposed planes; a row of 64 consecutive columns hit each bank of the
  // transposed planes from up to eight dwords.
  static_assert(NW == 8 && PER == NC, "8 x 8 staging blocks: one per wave per element");
  float ystage[PER];   // from the FP32 copy of Y (the split keeps 24 bits anyway)
  const int sr = lane >> 3, sc = lane & 7;
  auto stage_rc = [&](int k, int& r, int& c) {
    const int b = w + NW * k;
    r = 8 * (b & 3) + sr;
    c = 8 * (b >> 2) + sc;
  };
  auto stage_load = [&](int64_t t) {
    const float* src = a.Y32 + (ys + t * BY) * a.ldy;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      int r, c;
      stage_rc(k, r, c);
      ystage[k] = src[r * NP + c];
    }
  };
  auto stage_store = [&](int buf) {
    __bf16* b = sm + buf * L::BUF;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      int r, c;
      stage_rc(k, r, c);
      __bf16 h, m, l;
      split3_bf16(ystage[k], h, m, l);
      b[r * LR + c] = h;
      b[SZR + r * LR + c] = m;
      b[2 * SZR + r * LR + c] = l;
      b[3 * SZR + c * LT + r] = h;
      b[3 * SZR + SZT + c * LT + r] = m;
      b[3 * SZR + 2 * SZT + c * LT + r] = l;
    }
  };

  // S values at (x0 + l16, tile + y(e)), y(e) = 4 lq + e (e < 4), 16 + 4 lq + e - 4 (e >= 4)
  float vv[8], vn[8];
  auto load_s = [&](int64_t t, float (&d)[8]) {
    const int64_t yb = ys + ((t < ntile) ? t : ntile - 1) * BY;   // past the last tile: re-read it
    if constexpr (TRANS == 0) {
      const float* p = a.V32 + (xrow + l16) * a.ldv + yb + 4 * lq;
      const float4 u0 = *reinterpret_cast<const float4*>(p);
      const float4 u1 = *reinterpret_cast<const float4*>(p + 16);
      d[0] = u0.x; d[1] = u0.y; d[2] = u0.z; d[3] = u0.w;
      d[4] = u1.x; d[5] = u1.y; d[6] = u1.z; d[7] = u1.w;
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t y = yb + ((e < 4) ? 4 * lq + e : 16 + 4 * lq + e - 4);
        d[e] = a.V32[y * a.ldv + xrow + l16];
      }
    }
  };

  if (ntile > 0) {
    stage_load(0);
    stage_store(0);
    load_s(0, vv);
  }
  __syncthreads();
  // unconditional loads, as in the FP64/FP32 kernel
  for (int64_t t = 0; t < ntile; ++t) {
    stage_load(t + 1 < ntile ? t + 1 : t);
    load_s(t + 1, vn);    // the next tile's S values, a tile ahead
    const __bf16* b = sm + ((L::NBUF == 2) ? (int)(t & 1) : 0) * L::BUF;
    if (xvalid) {
      // P^T tiles of the two 16-row halves: reg r <-> y = 16 sb + 4 lq + r, x = l16
      f4_t sp[2];
#pragma unroll
      for (int sb = 0; sb < 2; ++sb) {
        sp[sb] = zero_f4();
        const __bf16* yr = b + (16 * sb + l16) * LR + 8 * lq;
#pragma unroll
        for (int j = 0; j < NKC; ++j) {
          const bf8_t yh = *reinterpret_cast<const bf8_t*>(yr + 32 * j);
          const bf8_t ym = *reinterpret_cast<const bf8_t*>(yr + SZR + 32 * j);
          const bf8_t yl = *reinterpret_cast<const bf8_t*>(yr + 2 * SZR + 32 * j);
          sp[sb] = mfma_bf16(yl, xh[j], sp[sb]);     // smallest terms first
          sp[sb] = mfma_bf16(yh, xl[j], sp[sb]);
          sp[sb] = mfma_bf16(ym, xm[j], sp[sb]);
          sp[sb] = mfma_bf16(ym, xh[j], sp[sb]);
          sp[sb] = mfma_bf16(yh, xm[j], sp[sb]);
          sp[sb] = mfma_bf16(yh, xh[j], sp[sb]);
        }
      }
      bf8_t ah, am, al;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float av = sp[e >> 2][e & 3] * vv[e];
        __bf16 h, m, l;
        split3_bf16(av, h, m, l);
        ah[e] = h;
        am[e] = m;
        al[e] = l;
      }
      // O[x][c] += A[x][y] Y[y][c], column blocks in pairs: the pair's operands are read
      // together ahead of its products, and the two accumulation chains alternate
      const __bf16* yt = b + 3 * SZR + l16 * LT + 4 * lq;
#pragma unroll
      for (int c0 = 0; c0 < NC; c0 += 2) {
        const int npair = (c0 + 1 < NC) ? 2 : 1;
        bf8_t bt[2][3];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          if (u < npair) {
            const __bf16* ph = yt + 16 * (c0 + u) * LT;
#pragma unroll
            for (int pl = 0; pl < 3; ++pl) {
              const bf4_t v0 = *reinterpret_cast<const bf4_t*>(ph + pl * SZT);
              const bf4_t v1 = *reinterpret_cast<const bf4_t*>(ph + pl * SZT + 16);
              bt[u][pl] = bf8_t{v0[0], v0[1], v0[2], v0[3], v1[0], v1[1], v1[2], v1[3]};
            }
          }
        }
        __builtin_amdgcn_sched_barrier(0);
        // smallest terms first
#pragma unroll
        for (int u = 0; u < 2; ++u)
          if (u < npair) o[c0 + u] = mfma_bf16(al, bt[u][0], o[c0 + u]);
#pragma unroll
        for (int u = 0; u < 2; ++u)
          if (u < npair) o[c0 + u] = mfma_bf16(ah, bt[u][2], o[c0 + u]);
#pragma unroll
        for (int u = 0; u < 2; ++u)
          if (u < npair) o[c0 + u] = mfma_bf16(am, bt[u][1], o[c0 + u]);
#pragma unroll
        for (int u = 0; u < 2; ++u)
          if (u < npair) o[c0 + u] = mfma_bf16(am, bt[u][0], o[c0 + u]);
#pragma unroll
        for (int u = 0; u < 2; ++u)
          if (u < npair) o[c0 + u] = mfma_bf16(ah, bt[u][1], o[c0 + u]);
#pragma unroll
        for (int u = 0; u < 2; ++u)
          if (u < npair) o[c0 + u] = mfma_bf16(ah, bt[u][0], o[c0 + u]);
      }
      if ((t & 1) || t + 1 == ntile) {
#pragma unroll
        for (int cb = 0; cb < NC; ++cb) {
#pragma unroll
          for (int r = 0; r < 4; ++r) od[cb][r] += (double)o[cb][r];
          o[cb] = zero_f4();
        }
      }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) vv[e] = vn[e];
    if constexpr (L::NBUF == 2) {
      stage_store((t + 1) & 1);
    } else {
      __syncthreads();     // every wave has read tile t
      stage_store(0);
    }
    __syncthreads();
  }

  if (!xvalid) return;
  double* out = a.out + (by * a.nx) * a.np;
#pragma unroll
  for (int cb = 0; cb < NC; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) out[(x0 + 4 * lq + r) * a.np + 16 * cb + l16] = od[cb][r];
}

template <int NC, int TRANS, int NW>
__global__ __launch_bounds__(NW * 64) void stream_bf16x3_kernel(StreamArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  bf16x3_body<NC, TRANS, NW>(a, blockIdx.x, blockIdx.y, smem_raw);
}

// Persistent split-BF16 form (see stream_queue_kernel).
template <int NC, int TRANS, int NW>
__global__ __launch_bounds__(NW * 64) void bf16x3_queue_kernel(const StreamArgs* __restrict__ args,
                                                              const StreamItem* __restrict__ items, int nitems,
                                                              unsigned* __restrict__ counter) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int s_item;
  while (true) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int i = s_item;
    __syncthreads();
    if (i >= nitems) break;
    const StreamItem it = items[i];
    const StreamArgs a = args[it.cell];
    bf16x3_body<NC, TRANS, NW>(a, it.bx, it.by, smem_raw);
    __syncthreads();
  }
}

template <int NC, int TRANS>
hipError_t launch_bf16x3(const StreamArgs& a, int nsplit, hipStream_t s) {
  constexpr int NW = 8;
  const size_t lds = Bf16Layout<NC>::LDS_BYTES;
  auto kern = stream_bf16x3_kernel<NC, TRANS, NW>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  dim3 grid((unsigned)((a.nx + 16 * NW - 1) / (16 * NW)), (unsigned)nsplit);
  hipLaunchKernelGGL(kern, grid, dim3(NW * 64), lds, s, a);
  return hipGetLastError();
}

template <int TRANS>
hipError_t dispatch_bf16x3(const StreamArgs& a, int nsplit, hipStream_t s) {
  switch (a.np / 16) {
    case 1: return launch_bf16x3<1, TRANS>(a, nsplit, s);
    case 2: return launch_bf16x3<2, TRANS>(a, nsplit, s);
    case 3: return launch_bf16x3<3, TRANS>(a, nsplit, s);
    case 4: return launch_bf16x3<4, TRANS>(a, nsplit, s);
    case 5: return launch_bf16x3<5, TRANS>(a, nsplit, s);
    case 6: return launch_bf16x3<6, TRANS>(a, nsplit, s);
    case 7: return launch_bf16x3<7, TRANS>(a, nsplit, s);
    case 8: return launch_bf16x3<8, TRANS>(a, nsplit, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename TM, int NC, int TRANS>
hipError_t launch_stream(const StreamArgs& a, int nsplit, hipStream_t s) {
  constexpr int NW = 8;
  const size_t lds = (size_t)2 * BY * stream_ldy<TM, NC>() * sizeof(TM);
  auto kern = stream_kernel<TM, NC, TRANS, NW>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  dim3 grid((unsigned)((a.nx + 16 * NW - 1) / (16 * NW)), (unsigned)nsplit);
  hipLaunchKernelGGL(kern, grid, dim3(NW * 64), lds, s, a);
  return hipGetLastError();
}

template <typename TM, int TRANS>
hipError_t dispatch_nc(const StreamArgs& a, int nsplit, hipStream_t s) {
  switch (a.np / 16) {
    case 1: return launch_stream<TM, 1, TRANS>(a, nsplit, s);
    case 2: return launch_stream<TM, 2, TRANS>(a, nsplit, s);
    case 3: return launch_stream<TM, 3, TRANS>(a, nsplit, s);
    case 4: return launch_stream<TM, 4, TRANS>(a, nsplit, s);
    case 5: return launch_stream<TM, 5, TRANS>(a, nsplit, s);
    case 6: return launch_stream<TM, 6, TRANS>(a, nsplit, s);
    case 7: return launch_stream<TM, 7, TRANS>(a, nsplit, s);
    case 8: return launch_stream<TM, 8, TRANS>(a, nsplit, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int stream_splits(int64_t nx, int64_t ny, int target_blocks) {
  const int64_t xb = (nx + 127) / 128;
  int64_t sp = target_blocks / xb;            // whole rounds of workgroups, no ragged last round
  const int64_t maxsp = ny / (4 * BY);        // at least four tiles per split
  if (sp > maxsp) sp = maxsp;
  if (sp < 1) sp = 1;
  return (int)sp;
}

hipError_t stream_prepare(const StreamArgs& a, int prec, int nsplit, StreamArgs& b) {
  if (a.np < 16 || a.np > 128 || a.np % 16 || a.nx % 16 || a.ny % BY || a.ldy != a.np) return hipErrorInvalidValue;
  if (nsplit < 1 || prec < 0 || prec > 2) return hipErrorInvalidValue;
  if (prec == 0 ? !a.V : (!a.V32 || !a.Y32)) return hipErrorInvalidValue;
  b = a;
  // y rows per split, a multiple of the tile
  const int64_t tiles = a.ny / BY;
  b.ysplit = ((tiles + nsplit - 1) / nsplit) * BY;
  return hipSuccess;
}

int64_t stream_xblocks(int64_t nx) { return (nx + 127) / 128; }

namespace {
template <typename K>
int resident_blocks(K kern, size_t lds) {
  int per_cu = 0, dev = 0, cus = 0;
  if (lds > 65536) (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 512, lds) != hipSuccess || per_cu < 1) per_cu = 1;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  return per_cu * cus;
}

template <typename TM, int NC, int TRANS>
hipError_t queue_stream(const StreamArgs* args, const StreamItem* items, int nitems, unsigned* counter, int nblocks,
                        hipStream_t s, int* resident) {
  constexpr int NW = 8;
  const size_t lds = (size_t)2 * BY * stream_ldy<TM, NC>() * sizeof(TM);
  auto kern = stream_queue_kernel<TM, NC, TRANS, NW>;
  if (resident) { *resident = resident_blocks(kern, lds); return hipSuccess; }
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)nblocks), dim3(NW * 64), lds, s, args, items, nitems, counter);
  return hipGetLastError();
}

template <int NC, int TRANS>
hipError_t queue_bf16x3(const StreamArgs* args, const StreamItem* items, int nitems, unsigned* counter, int nblocks,
                        hipStream_t s, int* resident) {
  constexpr int NW = 8;
  const size_t lds = Bf16Layout<NC>::LDS_BYTES;
  auto kern = bf16x3_queue_kernel<NC, TRANS, NW>;
  if (resident) { *resident = resident_blocks(kern, lds); return hipSuccess; }
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)nblocks), dim3(NW * 64), lds, s, args, items, nitems, counter);
  return hipGetLastError();
}

template <int TRANS>
hipError_t queue_dispatch(int prec, int np, const StreamArgs* args, const StreamItem* items, int nitems,
                          unsigned* counter, int nblocks, hipStream_t s, int* resident) {
#define RPS_QCASE(NC_)                                                                                    \
  case NC_:                                                                                               \
    return prec == 0 ? queue_stream<double, NC_, TRANS>(args, items, nitems, counter, nblocks, s, resident) \
         : prec == 1 ? queue_stream<float, NC_, TRANS>(args, items, nitems, counter, nblocks, s, resident)  \
                     : queue_bf16x3<NC_, TRANS>(args, items, nitems, counter, nblocks, s, resident);
  switch (np / 16) {
    RPS_QCASE(1) RPS_QCASE(2) RPS_QCASE(3) RPS_QCASE(4) RPS_QCASE(5) RPS_QCASE(6) RPS_QCASE(7) RPS_QCASE(8)
    default: return hipErrorInvalidValue;
  }
#undef RPS_QCASE
}
}  // namespace

int stream_queue_blocks(int prec, int np, int trans) {
  int r = 0;
  if (prec < 0 || prec > 2 || np < 16 || np > 128 || np % 16) return 0;
  if (trans) (void)queue_dispatch<1>(prec, np, nullptr, nullptr, 0, nullptr, 0, nullptr, &r);
  else (void)queue_dispatch<0>(prec, np, nullptr, nullptr, 0, nullptr, 0, nullptr, &r);
  return r;
}

hipError_t stream_product_queue(const StreamArgs* args, const StreamItem* items, int nitems, int prec, int np,
                                int trans, unsigned* counter, int nblocks, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  if (!args || !items || !counter || nblocks < 1 || prec < 0 || prec > 2) return hipErrorInvalidValue;
  return trans ? queue_dispatch<1>(prec, np, args, items, nitems, counter, nblocks, s, nullptr)
               : queue_dispatch<0>(prec, np, args, items, nitems, counter, nblocks, s, nullptr);
}

hipError_t stream_product(const StreamArgs& a, int prec, int nsplit, hipStream_t s) {
  StreamArgs b;
  const hipError_t pe = stream_prepare(a, prec, nsplit, b);
  if (pe != hipSuccess) return pe;
  if (prec == 2) {
    if (!a.V32 || !a.Y32) return hipErrorInvalidValue;
    return a.trans ? dispatch_bf16x3<1>(b, nsplit, s) : dispatch_bf16x3<0>(b, nsplit, s);
  }
  if (prec == 1) {
    if (!a.V32 || !a.Y32) return hipErrorInvalidValue;
    return a.trans ? dispatch_nc<float, 1>(b, nsplit, s) : dispatch_nc<float, 0>(b, nsplit, s);
  }
  if (!a.V) return hipErrorInvalidValue;
  return a.trans ? dispatch_nc<double, 1>(b, nsplit, s) : dispatch_nc<double, 0>(b, nsplit, s);
}

}  // namespace rps
