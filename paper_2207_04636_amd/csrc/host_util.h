// Host-side helpers: cell geometry, Coulomb kernel table, sketch matrices.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

namespace rps {

// 3x3 row-matrix helpers (rows a1, a2, a3).
double det3(const double a[9]);
bool inv3(const double a[9], double out[9]);

// k(G)/N_g on the grid in FFT index order (fftfreq convention, G = 0 -> 0),
// symmetrised over G <-> -G (mod mesh).
std::vector<double> coulomb_kernel_table(const double lattice[9], const int mesh[3]);

// Madelung constant M of the lattice (rows a1, a2, a3): minus the potential at a
// site of unit point charges on all sites with a uniform neutralising background,
// the site's own 1/r removed (Ewald splitting; M L = 2.8372975 for a simple cubic
// lattice of side L).
double madelung_constant(const double lattice[9]);

// Philox4x32-10 (Salmon et al., SC'11): ten rounds, multipliers 0xD2511F53 and
// 0xCD9E8D57, Weyl key increments 0x9E3779B9 and 0xBB67AE85.
void philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

// nrow x ncol (row-major) standard normal sketch matrix of stream `stream`:
// element (r, c) uses counter (idx lo, idx hi, stream, 0), idx = r*ncol + c,
// key (seed lo, seed hi); z = sqrt(-2 ln u0) cos(2 pi u1), u_k = (x_k + 0.5)/2^32.
std::vector<double> sketch_normal(int64_t nrow, int64_t ncol, uint64_t seed, uint32_t stream);

// Orthonormalise the columns of a row-major nrow x ncol matrix in place
// (modified Gram-Schmidt, applied twice).
void orthonormalize_columns(std::vector<double>& A, int64_t nrow, int64_t ncol);

}  // namespace rps
