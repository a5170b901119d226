// Host-side helpers of the set-up: geometry, the Coulomb kernel table and the
// random sketch matrices of the point selection.
#include "host_util.h"

#include <math.h>

#include <cmath>

namespace rps {

double det3(const double a[9]) {
  return a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
         a[2] * (a[3] * a[7] - a[4] * a[6]);
}

bool inv3(const double a[9], double o[9]) {
  const double d = det3(a);
  if (!(fabs(d) > 0.0)) return false;
  o[0] = (a[4] * a[8] - a[5] * a[7]) / d;
  o[1] = (a[2] * a[7] - a[1] * a[8]) / d;
  o[2] = (a[1] * a[5] - a[2] * a[4]) / d;
  o[3] = (a[5] * a[6] - a[3] * a[8]) / d;
  o[4] = (a[0] * a[8] - a[2] * a[6]) / d;
  o[5] = (a[2] * a[3] - a[0] * a[5]) / d;
  o[6] = (a[3] * a[7] - a[4] * a[6]) / d;
  o[7] = (a[1] * a[6] - a[0] * a[7]) / d;
  o[8] = (a[0] * a[4] - a[1] * a[3]) / d;
  return true;
}

static inline int fftfreq_int(int i, int n) { return (i < (n + 1) / 2) ? i : i - n; }

std::vector<double> coulomb_kernel_table(const double lat[9], const int mesh[3]) {
  // reciprocal rows B_j with a_i . B_j = 2 pi delta_ij: B = 2 pi (a^-1)^T
  double ai[9];
  inv3(lat, ai);
  double B[9];
  for (int j = 0; j < 3; ++j)
    for (int k = 0; k < 3; ++k) B[j * 3 + k] = 2.0 * M_PI * ai[k * 3 + j];
  const int64_t n1 = mesh[0], n2 = mesh[1], n3 = mesh[2];
  const int64_t ng = n1 * n2 * n3;
  auto kval = [&](int64_t i1, int64_t i2, int64_t i3) {
    const int f1 = fftfreq_int((int)i1, (int)n1), f2 = fftfreq_int((int)i2, (int)n2),
              f3 = fftfreq_int((int)i3, (int)n3);
    double g[3];
    for (int k = 0; k < 3; ++k) g[k] = f1 * B[k] + f2 * B[3 + k] + f3 * B[6 + k];
    const double g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
    return (g2 > 0.0) ? 4.0 * M_PI / g2 : 0.0;
  };
  std::vector<double> k(ng);
  for (int64_t i1 = 0; i1 < n1; ++i1)
    for (int64_t i2 = 0; i2 < n2; ++i2)
      for (int64_t i3 = 0; i3 < n3; ++i3) {
        const double v = kval(i1, i2, i3);
        const double vm = kval((n1 - i1) % n1, (n2 - i2) % n2, (n3 - i3) % n3);
        k[(i1 * n2 + i2) * n3 + i3] = 0.5 * (v + vm) / (double)ng;
      }
  return k;
}

double madelung_constant(const double lat[9]) {
  // phi(0) = sum_{T != 0} erfc(a |T|)/|T| + (4 pi / Omega) sum_{G != 0} exp(-G^2 / 4a^2) / G^2
  //          - 2a / sqrt(pi) - pi / (a^2 Omega),  with a = sqrt(pi) / Omega^(1/3);
  // both lattice sums run over a box of images wide enough for 1e-17 terms.
  const double om = std::fabs(det3(lat));
  const double a = std::sqrt(M_PI) / std::cbrt(om);
  double ai[9];
  inv3(lat, ai);
  double B[9];
  for (int j = 0; j < 3; ++j)
    for (int k = 0; k < 3; ++k) B[j * 3 + k] = 2.0 * M_PI * ai[k * 3 + j];
  auto norm = [](const double* v) { return std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); };
  // image boxes: a lattice vector n . a of length <= cut has |n_i| <= cut |b_i| / (2 pi)
  // (b_i the reciprocal rows), and a reciprocal vector m . b has |m_i| <= cut |a_i| / (2 pi)
  const double rcut = 6.5 / a;      // erfc(6.5) ~ 4e-20
  int mr[3];
  for (int i = 0; i < 3; ++i) mr[i] = (int)std::ceil(rcut * norm(B + 3 * i) / (2.0 * M_PI)) + 1;
  double real = 0.0;
  for (int i = -mr[0]; i <= mr[0]; ++i)
    for (int j = -mr[1]; j <= mr[1]; ++j)
      for (int k = -mr[2]; k <= mr[2]; ++k) {
        if (i == 0 && j == 0 && k == 0) continue;
        double t[3];
        for (int c = 0; c < 3; ++c) t[c] = i * lat[c] + j * lat[3 + c] + k * lat[6 + c];
        const double r = norm(t);
        real += std::erfc(a * r) / r;
      }
  const double gcut = 2.0 * a * std::sqrt(-std::log(1e-17));
  int mg[3];
  for (int i = 0; i < 3; ++i) mg[i] = (int)std::ceil(gcut * norm(lat + 3 * i) / (2.0 * M_PI)) + 1;
  double recip = 0.0;
  for (int i = -mg[0]; i <= mg[0]; ++i)
    for (int j = -mg[1]; j <= mg[1]; ++j)
      for (int k = -mg[2]; k <= mg[2]; ++k) {
        if (i == 0 && j == 0 && k == 0) continue;
        double g[3];
        for (int c = 0; c < 3; ++c) g[c] = i * B[c] + j * B[3 + c] + k * B[6 + c];
        const double g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
        recip += std::exp(-g2 / (4.0 * a * a)) / g2;
      }
  recip *= 4.0 * M_PI / om;
  const double phi0 = real + recip - 2.0 * a / std::sqrt(M_PI) - M_PI / (a * a * om);
  return -phi0;
}

void philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

std::vector<double> sketch_normal(int64_t nrow, int64_t ncol, uint64_t seed, uint32_t stream) {
  std::vector<double> z(nrow * ncol);
  const uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  for (int64_t idx = 0; idx < nrow * ncol; ++idx) {
    const uint32_t ctr[4] = {(uint32_t)((uint64_t)idx & 0xffffffffu), (uint32_t)((uint64_t)idx >> 32), stream, 0u};
    uint32_t x[4];
    philox4x32_10(ctr, key, x);
    const double u0 = ((double)x[0] + 0.5) / 4294967296.0;
    const double u1 = ((double)x[1] + 0.5) / 4294967296.0;
    z[idx] = sqrt(-2.0 * log(u0)) * cos(2.0 * M_PI * u1);
  }
  return z;
}

void orthonormalize_columns(std::vector<double>& A, int64_t nrow, int64_t ncol) {
  for (int64_t j = 0; j < ncol; ++j) {
    for (int pass = 0; pass < 2; ++pass) {
      for (int64_t i = 0; i < j; ++i) {
        double d = 0.0;
        for (int64_t r = 0; r < nrow; ++r) d += A[r * ncol + i] * A[r * ncol + j];
        for (int64_t r = 0; r < nrow; ++r) A[r * ncol + j] -= d * A[r * ncol + i];
      }
    }
    double nrm = 0.0;
    for (int64_t r = 0; r < nrow; ++r) nrm += A[r * ncol + j] * A[r * ncol + j];
    nrm = sqrt(nrm);
    if (nrm > 0.0)
      for (int64_t r = 0; r < nrow; ++r) A[r * ncol + j] /= nrm;
  }
}

}  // namespace rps
