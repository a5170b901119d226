// Voronoi-screened basis (Sec. 4.1).
//
// Per atom I the grid points of its Voronoi set kappa_I and the basis functions
// whose screened values are not all zero there form one dense block
// Phi_I = Phi[kappa_I][S_I] (row-major, |kappa_I| x n_I).  The screened value is
// dropped when its pSinc coefficient sqrt(dV) |phi| is below eps1.  The blocks
// replace the dense basis in the products with the grid of the general path:
//   U = Phi C:            U[kappa_I] = Phi_I C[S_I]                   (per atom)
//   K1 = Phi^T M1^T:      K1[mu] = sum_{I : mu in S_I} (Phi_I^T M1^T[kappa_I])[pos_I(mu)]
//   J = Phi^T diag(v) Phi: J[mu][nu] = sum_{I : mu, nu in S_I} (Phi_I^T diag(v) Phi_I)[pos_I(mu)][pos_I(nu)]
// The per-atom products run as ordinary matrix-core GEMMs; the kernels here are
// the screening, the block structure and the fixed-order sums over atoms.
#include "rps_internal.h"

namespace rps {
namespace {

__device__ __forceinline__ int64_t flat_id2() {
  return ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x;
}
inline dim3 flat_grid2(int64_t n) {
  const int64_t b = (n + 255) / 256;
  const int64_t gx = b < 65536 ? (b > 0 ? b : 1) : 65536;
  return dim3((unsigned)gx, (unsigned)((b + gx - 1) / gx));
}

__global__ void screen_kernel(double* __restrict__ Phi, int64_t count, double thr) {
  const int64_t i = flat_id2();
  if (i < count && fabs(Phi[i]) < thr) Phi[i] = 0.0;
}

// flags[owner[R] * N + mu] = 1 where Phi[R][mu] != 0 (every writer stores the same value)
__global__ void sig_flags_kernel(const double* __restrict__ Phi, int64_t ng, int Np, int N,
                                 const int32_t* __restrict__ owner, int32_t* __restrict__ flags) {
  const int64_t t = flat_id2();
  if (t >= ng * N) return;
  const int64_t R = t / N;
  const int mu = (int)(t % N);
  if (Phi[R * Np + mu] != 0.0) flags[(int64_t)owner[R] * N + mu] = 1;
}

// dst[r][c] = Phi[rows[r]][cols[c]] for r < nr, c < nc
__global__ void pack_block_kernel(const double* __restrict__ Phi, int Np, const int64_t* __restrict__ rows,
                                  int64_t nr, const int64_t* __restrict__ cols, int nc, double* __restrict__ dst) {
  const int64_t t = flat_id2();
  if (t >= nr * nc) return;
  const int64_t r = t / nc;
  const int c = (int)(t % nc);
  dst[t] = Phi[rows[r] * Np + cols[c]];
}

// out[mu][i] = sum over e in [ofs[mu], ofs[mu+1]) of part[rows[e]][i] (in order), mu < N;
// rows N..Np-1 of out are zero
__global__ void csr_rowsum_kernel(const double* __restrict__ part, int np, const int64_t* __restrict__ ofs,
                                  const int64_t* __restrict__ rows, int N, int Np, double* __restrict__ out) {
  const int64_t t = flat_id2();
  if (t >= (int64_t)Np * np) return;
  const int mu = (int)(t / np), i = (int)(t % np);
  double s = 0.0;
  if (mu < N)
    for (int64_t e = ofs[mu]; e < ofs[mu + 1]; ++e) s += part[rows[e] * np + i];
  out[t] = s;
}

// J[mu][nu] = J[nu][mu] = scale * sum over the atoms I holding mu (in order) of
// Q_I[pos_I(mu)][pos_I(nu)] where nu is held too; nu <= mu, so pos_I(nu) <= pos_I(mu)
// (function lists ascending) and only the lower triangle of each Q_I is read
__global__ void j_reduce_kernel(const double* __restrict__ Q, const int64_t* __restrict__ qofs,
                                const int64_t* __restrict__ fofs, const int32_t* __restrict__ pos,
                                const int64_t* __restrict__ ofs, const int32_t* __restrict__ atom, int N,
                                double scale, double* __restrict__ J) {
  const int64_t t = flat_id2();
  if (t >= (int64_t)N * N) return;
  const int mu = (int)(t / N), nu = (int)(t % N);
  if (nu > mu) return;
  double s = 0.0;
  for (int64_t e = ofs[mu]; e < ofs[mu + 1]; ++e) {
    const int I = atom[e];
    const int pn = pos[(int64_t)I * N + nu];
    if (pn < 0) continue;
    const int pm = pos[(int64_t)I * N + mu];
    const int64_t nI = fofs[I + 1] - fofs[I];
    s += Q[qofs[I] + (int64_t)pm * nI + pn];
  }
  J[(int64_t)mu * N + nu] = scale * s;
  J[(int64_t)nu * N + mu] = scale * s;
}

}  // namespace

hipError_t screen_basis(double* Phi, int64_t count, double thr, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(screen_kernel, flat_grid2(count), dim3(256), 0, s, Phi, count, thr);
  return hipGetLastError();
}

hipError_t basis_flags(const double* Phi, int64_t ng, int Np, int N, const int32_t* owner, int32_t* flags,
                       hipStream_t s) {
  if (ng * N <= 0) return hipSuccess;
  hipLaunchKernelGGL(sig_flags_kernel, flat_grid2(ng * N), dim3(256), 0, s, Phi, ng, Np, N, owner, flags);
  return hipGetLastError();
}

hipError_t pack_block(const double* Phi, int Np, const int64_t* rows, int64_t nr, const int64_t* cols, int nc,
                      double* dst, hipStream_t s) {
  if (nr * nc <= 0) return hipSuccess;
  hipLaunchKernelGGL(pack_block_kernel, flat_grid2(nr * nc), dim3(256), 0, s, Phi, Np, rows, nr, cols, nc, dst);
  return hipGetLastError();
}

hipError_t csr_rowsum(const double* part, int np, const int64_t* ofs, const int64_t* rows, int N, int Np,
                      double* out, hipStream_t s) {
  hipLaunchKernelGGL(csr_rowsum_kernel, flat_grid2((int64_t)Np * np), dim3(256), 0, s, part, np, ofs, rows, N, Np,
                     out);
  return hipGetLastError();
}

hipError_t j_reduce(const double* Q, const int64_t* qofs, const int64_t* fofs, const int32_t* pos,
                    const int64_t* ofs, const int32_t* atom, int N, double scale, double* J, hipStream_t s) {
  hipLaunchKernelGGL(j_reduce_kernel, flat_grid2((int64_t)N * N), dim3(256), 0, s, Q, qofs, fofs, pos, ofs, atom, N,
                     scale, J);
  return hipGetLastError();
}

}  // namespace rps
