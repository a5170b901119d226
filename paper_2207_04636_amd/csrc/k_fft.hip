// Coulomb potential of the fitting functions, V[g, :] = Vc chi_g (Sec. 3.2;
// the Coulomb operator is diagonal on the plane waves, Sec. 2.2 Eq. 7-8,
// with the G = 0 term removed, Sec. 4.5):
//     Vc f = IDFT( k(G) / N_g * DFT(f) ),  k(G) = 4 pi / |G|^2,  k(0) = 0.
//
// Two real rows f, h are transformed together as the complex row f + i h
// (split storage: the real parts stay in row 2c, the imaginary parts in row
// 2c + 1), which works because Vc is real: Vc(f + i h) = Vc f + i Vc h.
//
// The 3-D transform is separable: one pass per axis, each pass moving 16
// pencils of one axis into LDS and applying the length-L transform there with
// twiddles from sincospi in FP64 (axes up to 256 points): a self-sorting
// mixed-radix FFT (radices 2, 3, 4, 5) when L has no other prime factor, else
// the DFT by direct summation.  Passes:
// forward along axis 2, forward along axis 1, [forward along axis 0, multiply
// by k/N_g, inverse along axis 0] in one kernel, inverse along axis 1, inverse
// along axis 2.  This is a set-up step (once per geometry); the per-build path
// uses no transform.
#include <math.h>

#include "mfma.h"
#include "rps_internal.h"

namespace rps {
namespace {

constexpr int LMAX = 256;    // longest supported axis

// Pencil p (of outer*inner) starts at o*L*inner + i with o = p / inner, i = p % inner;
// element j of it is at start + j*inner.  PEN pencils per workgroup: 16 for the
// set-up's many rows, 4 when a single row pair would leave most CUs idle.  LM is
// the longest axis the LDS arrays hold: 128 (68 KB at PEN = 16), or 256 for longer
// axes with at most 8 pencils (70 KB).
template <int MODE, int PEN, int LM>   // 0: forward, 1: inverse, 2: forward, multiply by kern, inverse
__global__ __launch_bounds__(256) void dft_axis_kernel(double* __restrict__ V, int64_t ld, int L,
                                                      int64_t inner, int64_t npencil,
                                                      const double* __restrict__ kern) {
  __shared__ double br[2][PEN][LM + 1], bi[2][PEN][LM + 1];
  __shared__ double wr[LM], wi[LM];
  const int tid = threadIdx.x;
  double* re = V + (int64_t)(2 * blockIdx.y) * ld;
  double* im = re + ld;
  const int64_t p0 = (int64_t)blockIdx.x * PEN;
  const bool contiguous = (inner == 1);
  for (int m = tid; m < L; m += 256) {
    double s, c;
    sincospi(2.0 * (double)m / (double)L, &s, &c);
    wr[m] = c;
    wi[m] = s;
  }
  // element e of the workgroup block -> (pencil q, position j); coalesced either way
  auto split = [&](int e, int& q, int& j) {
    if (contiguous) { q = e / L; j = e % L; } else { j = e / PEN; q = e % PEN; }
  };
  for (int e = tid; e < PEN * L; e += 256) {
    int q, j;
    split(e, q, j);
    const int64_t p = p0 + q;
    double a = 0.0, b = 0.0;
    if (p < npencil) {
      const int64_t at = (p / inner) * (int64_t)L * inner + (p % inner) + (int64_t)j * inner;
      a = re[at];
      b = im[at];
    }
    br[0][q][j] = a;
    bi[0][q][j] = b;
  }
  __syncthreads();
  constexpr int PASSES = (MODE == 2) ? 2 : 1;
  int cur = 0;
  // lengths whose factors are all 2, 3 and 5 take the fast transform
  int rest = L;
  while (rest % 2 == 0) rest /= 2;
  while (rest % 3 == 0) rest /= 3;
  while (rest % 5 == 0) rest /= 5;
  const bool fast = (rest == 1);
#pragma unroll
  for (int pass = 0; pass < PASSES; ++pass) {
    // out[k] = sum_j x[j] exp(sg * 2 pi i j k / L), sg = -1 forward, +1 inverse
    const double sg = (MODE == 1 || pass == 1) ? 1.0 : -1.0;
    if (fast) {
      // Self-sorting (Stockham) mixed-radix transform, radices 4, 2, 3, 5: stage with
      // radix R after sub-transforms of length ns: butterfly j (< L / R) takes the R
      // points j + r L / R, turns them by exp(sg 2 pi i r (j mod ns) / (ns R)), applies
      // the R-point transform and writes point r' to (j / ns) ns R + (j mod ns) + r' ns.
      // Twiddles come from the table exp(2 pi i m / L) (ns R divides L).
      int ns = 1, left = L;
      while (left > 1) {
        const int R = (left % 4 == 0) ? 4 : (left % 2 == 0) ? 2 : (left % 3 == 0) ? 3 : 5;
        const int nb = L / R;
        const int tstep = L / (ns * R);
        for (int e = tid; e < PEN * nb; e += 256) {
          const int q = e / nb, j = e % nb;
          const int k = j % ns;
          double vr[5], vi[5];
#pragma unroll
          for (int r = 0; r < 5; ++r) {
            if (r < R) {
              const double a = br[cur][q][j + r * nb], b = bi[cur][q][j + r * nb];
              const int m = (r * k * tstep) % L;
              const double c = wr[m], sn = sg * wi[m];
              vr[r] = a * c - b * sn;
              vi[r] = a * sn + b * c;
            }
          }
          const int d0 = (j / ns) * ns * R + k;
#pragma unroll
          for (int o = 0; o < 5; ++o) {
            if (o < R) {
              double yr = 0.0, yi = 0.0;
#pragma unroll
              for (int r = 0; r < 5; ++r) {
                if (r < R) {
                  const int m = ((r * o) % R) * nb;
                  const double c = wr[m], sn = sg * wi[m];
                  yr += vr[r] * c - vi[r] * sn;
                  yi += vr[r] * sn + vi[r] * c;
                }
              }
              br[cur ^ 1][q][d0 + o * ns] = yr;
              bi[cur ^ 1][q][d0 + o * ns] = yi;
            }
          }
        }
        __syncthreads();
        cur ^= 1;
        ns *= R;
        left /= R;
      }
      if (MODE == 2 && pass == 0) {
        for (int e = tid; e < PEN * L; e += 256) {
          int q, k;
          split(e, q, k);
          const int64_t p = p0 + q;
          double kv = 0.0;
          if (p < npencil) kv = kern[(p / inner) * (int64_t)L * inner + (p % inner) + (int64_t)k * inner];
          br[cur][q][k] *= kv;
          bi[cur][q][k] *= kv;
        }
        __syncthreads();
      }
      continue;
    }
    for (int e = tid; e < PEN * L; e += 256) {
      int q, k;
      split(e, q, k);
      double sr = 0.0, si = 0.0;
      int m = 0;
      for (int j = 0; j < L; ++j) {
        const double c = wr[m], s = sg * wi[m];
        const double a = br[cur][q][j], b = bi[cur][q][j];
        sr += a * c - b * s;
        si += a * s + b * c;
        m += k;
        if (m >= L) m -= L;
      }
      if (MODE == 2 && pass == 0) {
        const int64_t p = p0 + q;
        double kv = 0.0;
        if (p < npencil) kv = kern[(p / inner) * (int64_t)L * inner + (p % inner) + (int64_t)k * inner];
        sr *= kv;
        si *= kv;
      }
      br[cur ^ 1][q][k] = sr;
      bi[cur ^ 1][q][k] = si;
    }
    __syncthreads();
    cur ^= 1;
  }
  for (int e = tid; e < PEN * L; e += 256) {
    int q, j;
    split(e, q, j);
    const int64_t p = p0 + q;
    if (p < npencil) {
      const int64_t at = (p / inner) * (int64_t)L * inner + (p % inner) + (int64_t)j * inner;
      re[at] = br[cur][q][j];
      im[at] = bi[cur][q][j];
    }
  }
}

template <int PEN, int LM>
void go(double* V, int64_t ld, int L, int64_t inner, int64_t np, const double* kern, int64_t npairs, int mode,
        hipStream_t s) {
  dim3 grid((unsigned)((np + PEN - 1) / PEN), (unsigned)npairs);
  if (mode == 0)
    hipLaunchKernelGGL((dft_axis_kernel<0, PEN, LM>), grid, dim3(256), 0, s, V, ld, L, inner, np, kern);
  else if (mode == 1)
    hipLaunchKernelGGL((dft_axis_kernel<1, PEN, LM>), grid, dim3(256), 0, s, V, ld, L, inner, np, kern);
  else
    hipLaunchKernelGGL((dft_axis_kernel<2, PEN, LM>), grid, dim3(256), 0, s, V, ld, L, inner, np, kern);
}

}  // namespace

hipError_t poisson_rows(double* V, int64_t nrows, int64_t ld, const int mesh[3],
                        const double* kern, hipStream_t s) {
  if (nrows % 2 != 0) return hipErrorInvalidValue;
  for (int a = 0; a < 3; ++a)
    if (mesh[a] > LMAX || mesh[a] < 1) return hipErrorInvalidValue;
  const int64_t ng = (int64_t)mesh[0] * mesh[1] * mesh[2];
  const int64_t npairs = nrows / 2;
  const int64_t inner[3] = {(int64_t)mesh[1] * mesh[2], (int64_t)mesh[2], 1};
  // grid.y <= 65535 pairs per launch
  for (int64_t c0 = 0; c0 < npairs; c0 += 65535) {
    const int64_t cn = (npairs - c0 < 65535) ? npairs - c0 : 65535;
    double* Vc = V + 2 * c0 * ld;
    auto launch = [&](int axis, int mode) {
      const int L = mesh[axis];
      const int64_t np = ng / L;
      if (L > 128) {
        go<8, 256>(Vc, ld, L, inner[axis], np, kern, cn, mode, s);
      } else if ((np + 15) / 16 * cn >= 1024) {
        go<16, 128>(Vc, ld, L, inner[axis], np, kern, cn, mode, s);
      } else {
        go<4, 128>(Vc, ld, L, inner[axis], np, kern, cn, mode, s);
      }
    };
    launch(2, 0);
    launch(1, 0);
    launch(0, 2);
    launch(1, 1);
    launch(2, 1);
  }
  return hipGetLastError();
}

}  // namespace rps
