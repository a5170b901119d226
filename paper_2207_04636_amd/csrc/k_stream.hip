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
// it to FP64 accumulators, so error does not grow with N_g.
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

template <typename TM, int NC>
__host__ __device__ constexpr int stream_ldy() {
  return 16 * NC + 1;
}

template <typename TM, int NC, int TRANS, int NW>
__global__ __launch_bounds__(NW * 64) void stream_kernel(StreamArgs a) {
  using F = Frag<TM>;
  using acc_t = typename F::acc;
  constexpr bool F64 = std::is_same<TM, double>::value;
  constexpr int NP = 16 * NC;
  constexpr int NK = NP / 4;
  constexpr int LDY = stream_ldy<TM, NC>();
  constexpr int PER = BY * NP / (NW * 64);   // staged Y elements per thread
  static_assert(PER * NW * 64 == BY * NP, "tile split");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TM* sY = reinterpret_cast<TM*>(smem_raw);

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, lq = lane >> 4;
  const int64_t x0 = ((int64_t)blockIdx.x * NW + w) * 16;
  const bool xvalid = x0 < a.nx;
  const int64_t ys = (int64_t)blockIdx.y * a.ysplit;
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

  // Y tile staging (rows are contiguous: ldy == np)
  double ystage[PER];
  auto stage_load = [&](int64_t t) {
    const double* src = a.Y + (ys + t * BY) * a.ldy;
#pragma unroll
    for (int k = 0; k < PER; ++k) ystage[k] = src[tid + k * NW * 64];
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

  if (ntile > 0) {
    stage_load(0);
    stage_store(0);
  }
  __syncthreads();
  for (int64_t t = 0; t < ntile; ++t) {
    if (t + 1 < ntile) stage_load(t + 1);
    const TM* sy = sY + (t & 1) * BY * LDY;
    const int64_t yb = ys + t * BY;
    if (xvalid) {
      TM vv[2][4];
#pragma unroll
      for (int sb = 0; sb < 2; ++sb) {
        const int64_t y0 = yb + 16 * sb + 4 * lq;
        if constexpr (TRANS == 0) {
          if constexpr (F64) {
            const double* p = a.V + (x0 + l16) * a.ldv + y0;
            const double2 u0 = *reinterpret_cast<const double2*>(p);
            const double2 u1 = *reinterpret_cast<const double2*>(p + 2);
            vv[sb][0] = u0.x; vv[sb][1] = u0.y; vv[sb][2] = u1.x; vv[sb][3] = u1.y;
          } else {
            const float4 u = *reinterpret_cast<const float4*>(a.V32 + (x0 + l16) * a.ldv + y0);
            vv[sb][0] = u.x; vv[sb][1] = u.y; vv[sb][2] = u.z; vv[sb][3] = u.w;
          }
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            if constexpr (F64) vv[sb][r] = a.V[(y0 + r) * a.ldv + x0 + l16];
            else vv[sb][r] = a.V32[(y0 + r) * a.ldv + x0 + l16];
          }
        }
      }
#pragma unroll
      for (int sb = 0; sb < 2; ++sb) {
        // P^T[y][x] = sum_d Y[y][d] X[x][d]
        acc_t s = F::zero();
        const TM* ya = sy + (16 * sb + yrowA) * LDY + lq;
#pragma unroll
        for (int j = 0; j < NK; ++j) s = F::mma(ya[4 * j], xr[j], s);
        // A = S o P, straight into the O product (k-step r <-> y = 4 lq + r)
        const TM* yb_ = sy + (16 * sb + 4 * lq) * LDY + l16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const TM av = s[r] * vv[sb][r];
#pragma unroll
          for (int cb = 0; cb < NC; ++cb) o[cb] = F::mma(av, yb_[r * LDY + 16 * cb], o[cb]);
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
    if (t + 1 < ntile) stage_store((t + 1) & 1);
    __syncthreads();
  }

  if (!xvalid) return;
  double* out = a.out + ((int64_t)blockIdx.y * a.nx) * a.np;
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

hipError_t stream_product(const StreamArgs& a, bool fp32, int nsplit, hipStream_t s) {
  if (a.np < 16 || a.np > 128 || a.np % 16 || a.nx % 16 || a.ny % BY || a.ldy != a.np) return hipErrorInvalidValue;
  if (nsplit < 1) return hipErrorInvalidValue;
  StreamArgs b = a;
  // y rows per split, a multiple of the tile
  const int64_t tiles = a.ny / BY;
  b.ysplit = ((tiles + nsplit - 1) / nsplit) * BY;
  if (fp32) {
    if (!a.V32) return hipErrorInvalidValue;
    return a.trans ? dispatch_nc<float, 1>(b, nsplit, s) : dispatch_nc<float, 0>(b, nsplit, s);
  }
  if (!a.V) return hipErrorInvalidValue;
  return a.trans ? dispatch_nc<double, 1>(b, nsplit, s) : dispatch_nc<double, 0>(b, nsplit, s);
}

}  // namespace rps
