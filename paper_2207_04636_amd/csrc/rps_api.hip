// C ABI of the rPS exchange library: context, one-time ISDF set-up and the
// per-build exchange (see include/rps.h for the contract of every entry point).
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>

#include <algorithm>
#include <array>
#include <chrono>
#include <exception>
#include <new>
#include <string>
#include <memory>
#include <mutex>
#include <vector>

#include "../../include/rps.h"
#include "host_util.h"
#include "rps_internal.h"

using namespace rps;

namespace {

thread_local std::string g_err;

struct Fail {
  rps_status st;
  std::string msg;
};

[[noreturn]] void fail(rps_status st, const std::string& m) { throw Fail{st, m}; }

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(RPS_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Device buffer owned by a context (or by a set-up step; freed on every exit path).
template <typename Tp>
struct DBuf {
  Tp* p = nullptr;
  int64_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(nullptr); }
  void alloc(int64_t count, int64_t* counter) {
    release(counter);
    if (count <= 0) return;
    hip_check(hipMalloc((void**)&p, sizeof(Tp) * count), "hipMalloc");
    n = count;
    if (counter) *counter += (int64_t)sizeof(Tp) * count;
  }
  void release(int64_t* counter) {
    if (p) {
      (void)hipFree(p);
      if (counter) *counter -= (int64_t)sizeof(Tp) * n;
    }
    p = nullptr;
    n = 0;
  }
};

}  // namespace

struct rps_context {
  // geometry and sizes
  double lat[9], ainv[9];
  int mesh[3];
  int64_t ng = 0, ngp = 0, nbas = 0, Np = 0, naux = 0, nauxp = 0;
  int natom = 0;
  double dV = 0.0;
  int precision = 0;
  int exact = 0;
  double shift = 0.0;
  double madelung = 0.0;   // Madelung constant of the cell (Sec. 4.5)
  double setup_seconds = 0.0;
  int64_t ncand = 0;
  int64_t bytes = 0;
  std::vector<int64_t> points;
  std::vector<int32_t> owner_host;
  // persistent device data
  DBuf<double> Phi, Phig, V, W;
  DBuf<float> V32;
  DBuf<float> Phi32;   // precision form, N <= 128: FP32 basis for the in-kernel orbitals
  DBuf<int64_t> dpoints;
  // Voronoi-screened basis (Sec. 4.1; set up when eps1 > 0): atom I holds grid rows
  // perm[vofs[I] .. vofs[I+1]) and functions fun[fofs[I] .. fofs[I+1]) (ascending); its
  // block Phi_I sits at pofs[I] in sPhi (row-major, pitch n_I) and its J block at qofs[I]
  double basis_eps = 0.0;
  bool sparse = false;
  std::vector<int64_t> vofs, fofs, pofs, qofs;
  DBuf<int64_t> sperm, sinv, sfun, smu_ofs, smu_rows, sqofs, sfofs;
  DBuf<int32_t> spos, smu_atom;   // pos[I][mu] (-1 if absent); atom of each CSR entry
  DBuf<double> sPhi;
  int sws_np = -1, sjws_np = -1;
  DBuf<double> sCg, sUv, sK1p, sQ, svv, sUj;
  DBuf<GemmItem> sitU, sitK1, sitJ;   // per-atom products of one grouped launch each
  int64_t smaxr = 0, smaxc = 0;       // largest Voronoi set, largest function list
  // build workspace (grows on demand)
  int ws_np = -1;
  DBuf<double> U, Ug, Ugp, M2p, K1p, K3p, e1p, e3p, M2, K1, K3, Kdev, Cdev, exdev, e3u;
  int use_m4 = 0;   // 16x16x4 FP64 kernel by default (faster on gfx950); RPS_FP64_MFMA=m4|hybrid selects the 4x4x4 one
  // general path workspace
  int gws_np = -1;
  int64_t gchunk = 0;
  DBuf<double> gCp, gU, gUg, gA, gSp, gM2, gM1T, gK1, gK3, gY, gwork, epart;
  DBuf<float> gU32, gUg32, gA32;   // precision form of the GEMM form: FP32 operands and A chunk
  DBuf<float> gPhi32, gM1T32;      // and the FP32 operands of K1 = Phi^T M1^T (basis, padded M1^T)
  DBuf<unsigned> ecount;   // last-block counter of the finalize kernel's energy sum (zero between builds)
  int64_t rblocks_main = 0, blocks_main = 0, blocks_l3 = 0;
  int rtiles = 4, gblocks = 1, nwaves = 4;
  // Coulomb matrix: kernel table k(G) / N_g kept from the set-up, and workspace
  DBuf<double> kern;
  int jws_np = -1;
  bool jws_small = false;
  int64_t jchunk = 0;
  DBuf<double> jCp, jCin, jU, jrho, jwork, jpart, jJ;
  // Madelung term: S = dV Phi^T Phi (kept once formed) and workspace
  DBuf<double> Sdev, mCp, mSC, mpart;
  // autotuned launch parameters (0: built-in default)
  int tune_target = 0;                      // streaming form: workgroups aimed at per launch
  int tune_rtiles = 0, tune_gblocks = 0;    // fused kernel: R tiles per workgroup, g blocks
  double tune_ms = 0.0;                     // best build time the tuner measured
  int last_arith = -1;                      // arithmetic of the last build's V products (rps_info.build_arith)
  // replay of repeated device-pointer builds as a captured HIP graph
  struct GraphEntry {
    int variant, nocc;
    const double* C;
    double* K;
    double* ex;
    hipGraph_t graph;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  GraphEntry last_call{-1, 0, nullptr, nullptr, nullptr, nullptr, nullptr};
  hipStream_t gstream = nullptr, gbranch = nullptr;   // capture stream and the line-3 branch
  hipEvent_t gfork = nullptr, gjoin = nullptr;
  // Generation of the build workspace: bumped whenever buffers that captured builds
  // refer to may be reallocated (every such change goes through clear_graphs), so a
  // batch graph captured earlier can tell that its baked-in pointers are stale.
  uint64_t ws_gen = 0;
  void clear_graphs() {
    ++ws_gen;
    for (auto& e : graphs) {
      (void)hipGraphExecDestroy(e.exec);
      (void)hipGraphDestroy(e.graph);
    }
    graphs.clear();
    last_call.variant = -1;
  }
  // profiling: event triples (build start, main start, main end, l3 start, l3 end, build end)
  int profiling = 0;
  std::vector<hipEvent_t> ev_pool;
  int64_t ev_used = 0;
  hipStream_t last_stream = nullptr;

  ~rps_context() {
    DBuf<double>* all[] = {&Phi, &Phig, &V, &W, &U, &Ug, &Ugp, &M2p, &K1p, &K3p, &e1p,
                           &e3p, &M2, &K1, &K3, &Kdev, &Cdev, &exdev, &e3u};
    for (auto* b : all) b->release(nullptr);
    DBuf<double>* gen[] = {&gCp, &gU, &gUg, &gA, &gSp, &gM2, &gM1T, &gK1, &gK3, &gY, &gwork, &epart};
    for (auto* b : gen) b->release(nullptr);
    gU32.release(nullptr);
    gUg32.release(nullptr);
    gPhi32.release(nullptr);
    gM1T32.release(nullptr);
    gA32.release(nullptr);
    ecount.release(nullptr);
    DBuf<double>* jb[] = {&kern, &jCp, &jCin, &jU, &jrho, &jwork, &jpart, &jJ, &Sdev, &mCp, &mSC, &mpart};
    for (auto* b : jb) b->release(nullptr);
    V32.release(nullptr);
    Phi32.release(nullptr);
    dpoints.release(nullptr);
    DBuf<int64_t>* si[] = {&sperm, &sinv, &sfun, &smu_ofs, &smu_rows, &sqofs, &sfofs};
    for (auto* b : si) b->release(nullptr);
    spos.release(nullptr);
    smu_atom.release(nullptr);
    DBuf<double>* sd[] = {&sPhi, &sCg, &sUv, &sK1p, &sQ, &svv, &sUj};
    for (auto* b : sd) b->release(nullptr);
    sitU.release(nullptr);
    sitK1.release(nullptr);
    sitJ.release(nullptr);
    for (auto e : ev_pool) (void)hipEventDestroy(e);
    clear_graphs();
    if (gfork) (void)hipEventDestroy(gfork);
    if (gjoin) (void)hipEventDestroy(gjoin);
    if (gstream) (void)hipStreamDestroy(gstream);
    if (gbranch) (void)hipStreamDestroy(gbranch);
  }
};

namespace {

// ------------------------------------------------------------------ set-up helpers
// Stage timing on stderr when RPS_VERBOSE is set (large set-ups run for minutes).
struct StageLog {
  bool on = getenv("RPS_VERBOSE") != nullptr;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  void operator()(const char* what, hipStream_t st) {
    if (!on) return;
    (void)hipStreamSynchronize(st);
    const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fprintf(stderr, "[rps setup %8.2f s] %s\n", t, what);
    fflush(stderr);
  }
};
constexpr int64_t kSplitWork = 64ll << 20;   // doubles of split-K partials (512 MB)
constexpr int kEnergyBlocks = 256;            // most blocks the energy dot products are split over
constexpr int kStreamMaxNp = 128;             // largest padded n of the streaming form
constexpr int64_t kChiPanel = 32768;          // grid columns per fitting-function panel (set-up)
constexpr int64_t kWPanel = 1024;             // rows per panel of the V and W stage (set-up)
constexpr int kStreamBlocks = 512;            // workgroups aimed at per streaming launch (default)
constexpr int kStreamMaxTarget = 1024;        // largest target the tuner tries
constexpr int64_t kStreamPartRows = (int64_t)kStreamMaxTarget * 128;   // rows of split partials
constexpr double kCutoff = 50.0;
constexpr double kCholShift = 1e-13;
constexpr int kOversample = 4;

CellDev make_cell(const rps_context& c) {
  CellDev d;
  memcpy(d.a, c.lat, sizeof d.a);
  memcpy(d.ainv, c.ainv, sizeof d.ainv);
  for (int k = 0; k < 3; ++k) d.mesh[k] = c.mesh[k];
  return d;
}

// Image ranges: a displacement reduced to |f_k| <= 1/2 reaches every image
// within radius rc when |n_k| <= rc/h_k + 1/2 (h_k = spacing of lattice planes).
std::vector<ShellDev> make_shells(const rps_context& c, const rps_basis* b, std::vector<int>& nfunc_atom) {
  const int nf[3] = {1, 3, 5};
  double h[3];
  for (int k = 0; k < 3; ++k) {
    // |A_k| = 2 pi |row k of (a^-1)^T| ; h_k = 2 pi / |A_k| = 1 / |column k of a^-1|
    const double x = c.ainv[0 * 3 + k], y = c.ainv[1 * 3 + k], z = c.ainv[2 * 3 + k];
    h[k] = 1.0 / sqrt(x * x + y * y + z * z);
  }
  std::vector<ShellDev> out(b->nshell);
  nfunc_atom.assign(b->natom, 0);
  int ofs = 0;
  for (int s = 0; s < b->nshell; ++s) {
    const int at = b->shell_atom[s];
    const double* A = b->atom_xyz + 3 * at;
    ShellDev& d = out[s];
    d.cx = A[0]; d.cy = A[1]; d.cz = A[2];
    d.expo = b->shell_exp[s];
    d.l = b->shell_l[s];
    d.fofs = ofs;
    const double rc = sqrt(kCutoff / d.expo);
    d.m0 = (int)ceil(rc / h[0] + 0.5);
    d.m1 = (int)ceil(rc / h[1] + 0.5);
    d.m2 = (int)ceil(rc / h[2] + 0.5);
    ofs += nf[d.l];
    nfunc_atom[at] += nf[d.l];
  }
  return out;
}

// Leading k pivots of the Gram matrix (A A^T) o (B B^T) of the sketch of the
// pair products at the candidate rows `cand` (Sec. 3.1, 4.3).
std::vector<int64_t> select_pivots(rps_context& c, const std::vector<int64_t>& cand, int64_t k,
                                   uint64_t seed, uint32_t s1, uint32_t s2, hipStream_t st) {
  const int64_t nc = (int64_t)cand.size();
  k = std::min(k, nc);
  const int64_t N = c.nbas;
  int64_t p = (int64_t)ceil(sqrt((double)k)) + kOversample;
  if (p > N) p = N;
  std::vector<double> G1 = sketch_normal(N, p, seed, s1);
  std::vector<double> G2 = sketch_normal(N, p, seed, s2);
  orthonormalize_columns(G1, N, p);
  orthonormalize_columns(G2, N, p);
  // padded to Np rows
  std::vector<double> G12((size_t)c.Np * 2 * p, 0.0);
  for (int64_t r = 0; r < N; ++r)
    for (int64_t q = 0; q < p; ++q) {
      G12[r * 2 * p + q] = G1[r * p + q];
      G12[r * 2 * p + p + q] = G2[r * p + q];
    }
  int64_t tmpb = 0;
  DBuf<double> dG, Phic, AB, Gram, Lb, diag;
  DBuf<int64_t> dcand, dpiv;
  dG.alloc(c.Np * 2 * p, &tmpb);
  dcand.alloc(nc, &tmpb);
  dpiv.alloc(k, &tmpb);
  Phic.alloc(nc * c.Np, &tmpb);
  AB.alloc(nc * 2 * p, &tmpb);
  Gram.alloc(nc * nc, &tmpb);
  Lb.alloc(nc * k, &tmpb);
  diag.alloc(nc + k, &tmpb);
  hip_check(hipMemcpyAsync(dG.p, G12.data(), G12.size() * 8, hipMemcpyHostToDevice, st), "copy sketch");
  hip_check(hipMemcpyAsync(dcand.p, cand.data(), nc * 8, hipMemcpyHostToDevice, st), "copy candidates");
  hip_check(gather_rows(c.Phi.p, c.Np, dcand.p, nc, nc, c.Np, Phic.p, c.Np, st), "gather");
  Gemm g;                                    // [A | B] = Phi_c [G1 | G2]
  g.M = nc; g.N = 2 * p; g.K = c.Np;
  g.A = Phic.p; g.lda = c.Np; g.B = dG.p; g.ldb = 2 * p; g.C = AB.p; g.ldc = 2 * p;
  hip_check(gemm_f64(g, st), "sketch product");
  Gemm ga;                                   // Gram = A A^T
  ga.M = nc; ga.N = nc; ga.K = p;
  ga.A = AB.p; ga.lda = 2 * p; ga.B = AB.p; ga.ldb = 2 * p; ga.transB = true;
  ga.C = Gram.p; ga.ldc = nc;
  hip_check(gemm_f64(ga, st), "gram A");
  Gemm gb = ga;                              // Gram o= B B^T
  gb.A = AB.p + p; gb.B = AB.p + p; gb.epi = EPI_HADAMARD;
  hip_check(gemm_f64(gb, st), "gram B");
  hip_check(pivoted_cholesky(Gram.p, nc, nc, k, dpiv.p, Lb.p, diag.p, st), "pivoted cholesky");
  std::vector<int64_t> piv(k);
  hip_check(hipMemcpyAsync(piv.data(), dpiv.p, k * 8, hipMemcpyDeviceToHost, st), "copy pivots");
  hip_check(hipStreamSynchronize(st), "sync");
  DBuf<double>* bufs[] = {&dG, &Phic, &AB, &Gram, &Lb, &diag};
  for (auto* b : bufs) b->release(nullptr);
  dcand.release(nullptr);
  dpiv.release(nullptr);
  std::vector<int64_t> out(k);
  for (int64_t i = 0; i < k; ++i) out[i] = cand[piv[i]];
  return out;
}

// Voronoi owner of every grid point (Sec. 4.1), kept on the host
void compute_owners(rps_context& c, const double* atoms, hipStream_t st) {
  if ((int64_t)c.owner_host.size() == c.ng) return;
  DBuf<int32_t> own;
  int64_t tmpb = 0;
  own.alloc(c.ng, &tmpb);
  DBuf<double> datoms;
  datoms.alloc(3 * (int64_t)c.natom, &tmpb);
  hip_check(hipMemcpyAsync(datoms.p, atoms, 3 * c.natom * 8, hipMemcpyHostToDevice, st), "copy atoms");
  hip_check(voronoi_assign(make_cell(c), datoms.p, c.natom, c.ng, own.p, st), "voronoi");
  c.owner_host.resize(c.ng);
  hip_check(hipMemcpyAsync(c.owner_host.data(), own.p, c.ng * 4, hipMemcpyDeviceToHost, st), "copy owner");
  hip_check(hipStreamSynchronize(st), "sync");
  own.release(nullptr);
  datoms.release(nullptr);
}

// Atom blocks of the screened basis: grid rows of each Voronoi set, the functions not
// all zero there, the packed blocks and the maps of the fixed-order sums over atoms.
void build_screened_blocks(rps_context& c, const double* atoms, hipStream_t st) {
  compute_owners(c, atoms, st);
  const int N = (int)c.nbas, natom = c.natom;
  int64_t tmp = 0;
  DBuf<int32_t> own, flags;
  own.alloc(c.ng, &tmp);
  flags.alloc((int64_t)natom * N, &tmp);
  hip_check(hipMemcpyAsync(own.p, c.owner_host.data(), c.ng * 4, hipMemcpyHostToDevice, st), "copy owner");
  hip_check(hipMemsetAsync(flags.p, 0, (size_t)natom * N * 4, st), "clear flags");
  hip_check(basis_flags(c.Phi.p, c.ng, (int)c.Np, N, own.p, flags.p, st), "flags");
  std::vector<int32_t> fl((size_t)natom * N);
  hip_check(hipMemcpyAsync(fl.data(), flags.p, fl.size() * 4, hipMemcpyDeviceToHost, st), "copy flags");
  hip_check(hipStreamSynchronize(st), "sync");
  own.release(nullptr);
  flags.release(nullptr);

  std::vector<std::vector<int64_t>> kap(natom);
  for (int64_t R = 0; R < c.ng; ++R) kap[c.owner_host[R]].push_back(R);
  std::vector<int64_t> perm, inv(c.ng), fun;
  std::vector<int32_t> pos((size_t)natom * N, -1);
  c.vofs.assign(natom + 1, 0);
  c.fofs.assign(natom + 1, 0);
  c.pofs.assign(natom + 1, 0);
  c.qofs.assign(natom + 1, 0);
  for (int I = 0; I < natom; ++I) {
    for (int64_t R : kap[I]) {
      inv[R] = (int64_t)perm.size();
      perm.push_back(R);
    }
    int k = 0;
    for (int mu = 0; mu < N; ++mu)
      if (fl[(size_t)I * N + mu]) {
        pos[(size_t)I * N + mu] = k++;
        fun.push_back(mu);
      }
    c.vofs[I + 1] = (int64_t)perm.size();
    c.fofs[I + 1] = (int64_t)fun.size();
    c.pofs[I + 1] = c.pofs[I] + (int64_t)kap[I].size() * k;
    c.qofs[I + 1] = c.qofs[I] + (int64_t)k * k;
  }
  // for every function, the atoms holding it (ascending) and its packed row there
  std::vector<int64_t> mofs(N + 1, 0), mrows;
  std::vector<int32_t> matom;
  for (int mu = 0; mu < N; ++mu) {
    for (int I = 0; I < natom; ++I) {
      const int p = pos[(size_t)I * N + mu];
      if (p < 0) continue;
      mrows.push_back(c.fofs[I] + p);
      matom.push_back(I);
    }
    mofs[mu + 1] = (int64_t)mrows.size();
  }
  auto up64 = [&](DBuf<int64_t>& d, const std::vector<int64_t>& h) {
    d.alloc(std::max<int64_t>((int64_t)h.size(), 1), &c.bytes);
    if (!h.empty()) hip_check(hipMemcpyAsync(d.p, h.data(), h.size() * 8, hipMemcpyHostToDevice, st), "copy map");
  };
  auto up32 = [&](DBuf<int32_t>& d, const std::vector<int32_t>& h) {
    d.alloc(std::max<int64_t>((int64_t)h.size(), 1), &c.bytes);
    if (!h.empty()) hip_check(hipMemcpyAsync(d.p, h.data(), h.size() * 4, hipMemcpyHostToDevice, st), "copy map");
  };
  up64(c.sperm, perm);
  up64(c.sinv, inv);
  up64(c.sfun, fun);
  up64(c.smu_ofs, mofs);
  up64(c.smu_rows, mrows);
  up64(c.sqofs, c.qofs);
  up64(c.sfofs, c.fofs);
  up32(c.spos, pos);
  up32(c.smu_atom, matom);
  c.sPhi.alloc(std::max<int64_t>(c.pofs[natom], 1), &c.bytes);
  for (int I = 0; I < natom; ++I) {
    const int64_t nr = c.vofs[I + 1] - c.vofs[I];
    const int nc = (int)(c.fofs[I + 1] - c.fofs[I]);
    hip_check(pack_block(c.Phi.p, (int)c.Np, c.sperm.p + c.vofs[I], nr, c.sfun.p + c.fofs[I], nc,
                         c.sPhi.p + c.pofs[I], st), "pack");
  }
  // J blocks: lower triangles of Phi_I^T diag(v[kappa_I]) Phi_I, one grouped launch
  std::vector<GemmItem> jt;
  c.smaxr = c.smaxc = 0;
  for (int I = 0; I < natom; ++I) {
    const int64_t nr = c.vofs[I + 1] - c.vofs[I], nc = c.fofs[I + 1] - c.fofs[I];
    c.smaxr = std::max(c.smaxr, nr);
    c.smaxc = std::max(c.smaxc, nc);
    if (nc == 0) continue;
    jt.push_back(GemmItem{nc, nc, nr, nc, nc, nc, c.pofs[I], c.pofs[I], c.qofs[I], c.vofs[I]});
  }
  c.sitJ.alloc(std::max<int64_t>((int64_t)jt.size(), 1), &c.bytes);
  if (!jt.empty())
    hip_check(hipMemcpyAsync(c.sitJ.p, jt.data(), jt.size() * sizeof(GemmItem), hipMemcpyHostToDevice, st), "items");
  c.sitJ.n = (int64_t)jt.size();
  hip_check(hipStreamSynchronize(st), "sync");
  c.sparse = true;
}

void select_points(rps_context& c, int mode, uint64_t seed, const std::vector<int>& nfunc_atom,
                   const double* atoms, hipStream_t st) {
  const int64_t global_limit = 16384;   // Gram of all grid points must stay small
  auto global = [&]() {
    if (c.ng > global_limit)
      fail(RPS_ERR_ARG, "global selection builds the N_g x N_g Gram matrix and is limited to N_g <= 16384; "
                        "use RPS_SELECT_VORONOI");
    std::vector<int64_t> all(c.ng);
    for (int64_t i = 0; i < c.ng; ++i) all[i] = i;
    c.points = select_pivots(c, all, c.naux, seed, 0, 1, st);
    c.ncand = c.ng;
  };
  if (mode == RPS_SELECT_GLOBAL) {
    global();
    return;
  }
  // Voronoi sets (Sec. 4.1)
  compute_owners(c, atoms, st);
  std::vector<std::vector<int64_t>> kappa(c.natom);
  for (int64_t R = 0; R < c.ng; ++R) kappa[c.owner_host[R]].push_back(R);
  const double cfac = (double)c.naux / (double)c.nbas;
  std::vector<int64_t> Rh;
  for (int I = 0; I < c.natom; ++I) {
    if (kappa[I].empty()) continue;
    int64_t KI = (int64_t)ceil(cfac * nfunc_atom[I] - 1e-9) + 10;
    KI = std::min<int64_t>(KI, (int64_t)kappa[I].size());
    std::vector<int64_t> pi = select_pivots(c, kappa[I], KI, seed, 2 + 2 * I, 3 + 2 * I, st);
    Rh.insert(Rh.end(), pi.begin(), pi.end());
  }
  if ((int64_t)Rh.size() < c.naux) {
    global();
    return;
  }
  c.ncand = (int64_t)Rh.size();
  c.points = select_pivots(c, Rh, c.naux, seed, 0, 1, st);
}

// ------------------------------------------------------------------ no-allocation build
// Static device scratch of the no-allocation entry point: the fused path's
// workspace (orbitals at the points, M2 / K1 / fit-fit partials, their sums,
// the energy partials and the energy counter) carved from one array per device.
// The code object holds it on every device it is loaded on until the process
// ends.  Host code must not use the array's name as an address: the device
// address of each device's copy is taken once with hipGetSymbolAddress (with
// that device current) and kept in g_scratch_ptr.
constexpr int64_t kNoAllocScratchBytes = 64ll << 20;
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / 8];

std::mutex g_scratch_mu;
std::vector<double*> g_scratch_ptr;   // device address of `scratch` per device ordinal

double* scratch_device_ptr() {
  int dev = 0;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!ptr) fail(RPS_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  return g_scratch_ptr[dev];
}

// Set-up products supplied by the caller (rps_setup_isdf_from_potentials): V in the
// context's storage precision (FP64, or FP32 for the precision forms) and W, with
// their row pitches, as host or device pointers.
struct GivenFit {
  const void* V = nullptr;
  int64_t ldv = 0;
  const double* W = nullptr;
  int64_t ldw = 0;
  bool device = false;
};

void setup_impl(rps_context& c, const rps_cell* cell, const rps_basis* b, int64_t n_aux, uint64_t seed,
                int32_t mode, int32_t prec, const int64_t* points_in, double basis_eps, hipStream_t st,
                const GivenFit* given = nullptr) {
  auto t0 = std::chrono::steady_clock::now();
  StageLog stage;
  // ---- validation
  if (!cell || !b) fail(RPS_ERR_ARG, "cell and basis must not be NULL");
  if (b->natom < 1 || b->nshell < 1 || !b->atom_xyz || !b->shell_atom || !b->shell_l || !b->shell_exp)
    fail(RPS_ERR_ARG, "basis needs natom >= 1, nshell >= 1 and non-NULL arrays");
  if (prec < RPS_PREC_FP64 || prec > RPS_PREC_BF16X3) fail(RPS_ERR_ARG, "unknown precision");
  if (mode != RPS_SELECT_VORONOI && mode != RPS_SELECT_GLOBAL) fail(RPS_ERR_ARG, "unknown selection mode");
  if (!(basis_eps >= 0.0) || !std::isfinite(basis_eps)) fail(RPS_ERR_ARG, "basis_eps must be finite and >= 0");
  c.basis_eps = basis_eps;
  memcpy(c.lat, cell->lattice, sizeof c.lat);
  const double vol = fabs(det3(c.lat));
  if (!(vol > 1e-10) || !inv3(c.lat, c.ainv)) fail(RPS_ERR_ARG, "lattice is singular");
  for (int k = 0; k < 3; ++k) {
    c.mesh[k] = cell->mesh[k];
    if (c.mesh[k] < 2 || c.mesh[k] > 256) fail(RPS_ERR_SHAPE, "mesh sizes must be in [2, 256]");
  }
  c.natom = b->natom;
  int64_t nb = 0;
  for (int s = 0; s < b->nshell; ++s) {
    const int l = b->shell_l[s];
    if (l < 0 || l > 2) fail(RPS_ERR_ARG, "shell_l must be 0, 1 or 2");
    if (!(b->shell_exp[s] > 0.0) || !std::isfinite(b->shell_exp[s])) fail(RPS_ERR_ARG, "shell exponents must be > 0");
    if (b->shell_atom[s] < 0 || b->shell_atom[s] >= b->natom) fail(RPS_ERR_ARG, "shell_atom out of range");
    nb += (l == 0) ? 1 : (l == 1) ? 3 : 5;
  }
  c.nbas = nb;
  c.ng = (int64_t)c.mesh[0] * c.mesh[1] * c.mesh[2];
  c.dV = vol / (double)c.ng;
  c.madelung = madelung_constant(c.lat);
  if (n_aux < 1 || n_aux > c.ng) fail(RPS_ERR_SHAPE, "n_aux must be in [1, N_g]");
  c.naux = n_aux;
  c.precision = prec;
  c.exact = (n_aux == c.ng);
  c.ngp = round_up(c.ng, 64);
  c.Np = round_up(c.nbas, 16);
  c.nauxp = round_up(c.naux, 64);
  if (given) {
    if (!points_in) fail(RPS_ERR_ARG, "set-up from given potentials needs points_in");
    if (!given->V || !given->W) fail(RPS_ERR_ARG, "V and W must not be NULL");
    if (given->ldv < c.ng || given->ldw < n_aux) fail(RPS_ERR_SHAPE, "ldv must be >= N_g and ldw >= n_aux");
    if (c.exact) fail(RPS_ERR_SHAPE, "n_aux == N_g is the exact case (chi = identity); use rps_setup_isdf");
  }
  if (points_in) {
    std::vector<char> seen(c.ng, 0);
    for (int64_t g = 0; g < n_aux; ++g) {
      const int64_t p = points_in[g];
      if (p < 0 || p >= c.ng) fail(RPS_ERR_SHAPE, "points_in entry out of range");
      if (seen[p]) fail(RPS_ERR_SHAPE, "points_in has a duplicate grid index");
      seen[p] = 1;
    }
  }
  // ---- memory estimate before any allocation
  {
    const double vbytes = (given && prec != RPS_PREC_FP64) ? 0.0 : 8.0 * (double)c.nauxp * c.ngp;
    const double persist = 8.0 * ((double)c.ngp * c.Np + (double)c.nauxp * c.Np + (double)c.nauxp * c.nauxp) +
                           vbytes + ((prec != RPS_PREC_FP64) ? 4.0 * (double)c.nauxp * c.ngp : 0.0);
    // the Cholesky factor for chi, then a panel of chi rows and the split partials for W
    const double xgg = 8.0 * (double)c.nauxp * c.nauxp;
    const double xblk = std::max(0.0, 8.0 * ((double)std::min(kWPanel, c.nauxp) * c.ngp + (double)kSplitWork) - xgg);
    double selb = 0.0;
    if (!points_in && !c.exact) {
      const double ncand = (mode == RPS_SELECT_GLOBAL) ? (double)c.ng : (double)c.naux + 10.0 * c.natom + 64;
      const double kap = 4.0 * (double)c.ng / std::max(1, c.natom) + 1024;   // generous Voronoi set
      const double nmax = std::max(ncand, kap);
      selb = 8.0 * (nmax * nmax + nmax * (double)c.naux + nmax * (double)c.Np);
    }
    const double need = persist + (given ? 0.0 : std::max(xgg + xblk, selb)) + 64.0 * 1024 * 1024;
    size_t fr = 0, tot = 0;
    hip_check(hipMemGetInfo(&fr, &tot), "hipMemGetInfo");
    if (need > (double)fr)
      fail(RPS_ERR_NOMEM, "set-up needs about " + std::to_string((int64_t)(need / 1e9)) + " GB, " +
                              std::to_string((int64_t)(fr / 1000000000ull)) + " GB free");
  }
  // ---- basis on the grid (Sec. 2.1.3)
  std::vector<int> nfunc_atom;
  std::vector<ShellDev> shells = make_shells(c, b, nfunc_atom);
  c.Phi.alloc(c.ngp * c.Np, &c.bytes);
  hip_check(fill(c.Phi.p, c.ngp * c.Np, 0.0, st), "fill");
  {
    DBuf<ShellDev> dsh;
    hip_check(hipMalloc((void**)&dsh.p, sizeof(ShellDev) * shells.size()), "hipMalloc");
    dsh.n = (int64_t)shells.size();
    hip_check(hipMemcpyAsync(dsh.p, shells.data(), sizeof(ShellDev) * shells.size(), hipMemcpyHostToDevice, st),
              "copy shells");
    hip_check(basis_eval(make_cell(c), dsh.p, (int)shells.size(), c.ng, c.Phi.p, c.Np, st), "basis");
    // screened basis (Sec. 4.1): pSinc coefficients sqrt(dV) |phi| below eps1 are dropped,
    // before anything else reads Phi
    if (basis_eps > 0.0) hip_check(screen_basis(c.Phi.p, c.ngp * c.Np, basis_eps / sqrt(c.dV), st), "screen");
    hip_check(hipStreamSynchronize(st), "sync");
    (void)hipFree(dsh.p);
    dsh.p = nullptr;
  }
  stage("basis on the grid", st);
  // ---- interpolation points
  if (points_in) {
    c.points.assign(points_in, points_in + n_aux);
  } else if (c.exact) {
    c.points.resize(c.ng);
    for (int64_t i = 0; i < c.ng; ++i) c.points[i] = i;
  } else {
    select_points(c, mode, seed, nfunc_atom, b->atom_xyz, st);
  }
  stage("interpolation points", st);
  c.dpoints.alloc(c.naux, &c.bytes);
  hip_check(hipMemcpyAsync(c.dpoints.p, c.points.data(), c.naux * 8, hipMemcpyHostToDevice, st), "copy points");
  c.Phig.alloc(c.nauxp * c.Np, &c.bytes);
  hip_check(gather_rows(c.Phi.p, c.Np, c.dpoints.p, c.naux, c.nauxp, c.Np, c.Phig.p, c.Np, st), "gather");
  const bool given32 = given && prec != RPS_PREC_FP64;   // caller's V goes straight into the FP32 store
  if (!given32) {
    c.V.alloc(c.nauxp * c.ngp, &c.bytes);
    hip_check(fill(c.V.p, c.nauxp * c.ngp, 0.0, st), "fill");
  }
  c.W.alloc(c.nauxp * c.nauxp, &c.bytes);
  hip_check(fill(c.W.p, c.nauxp * c.nauxp, 0.0, st), "fill");
  std::vector<double> kern = coulomb_kernel_table(c.lat, c.mesh);
  c.kern.alloc(c.ng, &c.bytes);   // kept for the Coulomb matrix builds
  const double* dkern = c.kern.p;
  int64_t tmpb = 0;
  hip_check(hipMemcpyAsync(c.kern.p, kern.data(), c.ng * 8, hipMemcpyHostToDevice, st), "copy kernel");

  if (given) {
    // rows of the caller's V and W into the padded device arrays (padding stays zero)
    const hipMemcpyKind kind = given->device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (given32) {
      c.V32.alloc(c.nauxp * c.ngp, &c.bytes);
      hip_check(hipMemsetAsync(c.V32.p, 0, (size_t)c.nauxp * c.ngp * 4, st), "clear V32");
      hip_check(hipMemcpy2DAsync(c.V32.p, c.ngp * 4, given->V, given->ldv * 4, c.ng * 4, c.naux, kind, st),
                "copy V");
    } else {
      hip_check(hipMemcpy2DAsync(c.V.p, c.ngp * 8, given->V, given->ldv * 8, c.ng * 8, c.naux, kind, st),
                "copy V");
    }
    hip_check(hipMemcpy2DAsync(c.W.p, c.nauxp * 8, given->W, given->ldw * 8, c.naux * 8, c.naux, kind, st),
              "copy W");
    hip_check(hipStreamSynchronize(st), "sync");
    stage("given potentials", st);
  } else if (c.exact) {
    // chi = identity on the chosen order: V[g] = Vc e_{points[g]}, W[g][g'] = V[g][points[g']]
    hip_check(set_unit_rows(c.V.p, c.ngp, c.dpoints.p, c.naux, st), "unit rows");
    hip_check(poisson_rows(c.V.p, c.nauxp, c.ngp, c.mesh, dkern, st), "poisson");
    hip_check(gather_cols(c.V.p, c.ngp, c.dpoints.p, c.naux, c.W.p, c.nauxp, st), "W");
  } else {
    // ---- fitting metric and Cholesky (Sec. 3.1 Eq. 11, Sec. 4.3)
    DBuf<double> L;
    L.alloc(c.nauxp * c.nauxp, &tmpb);
    int32_t* dstatus = nullptr;
    hip_check(hipMalloc((void**)&dstatus, sizeof(int32_t)), "hipMalloc");
    auto form_metric = [&]() {
      hip_check(fill(L.p, c.nauxp * c.nauxp, 0.0, st), "fill");
      Gemm g;
      g.M = c.nauxp; g.N = c.nauxp; g.K = c.Np;
      g.A = c.Phig.p; g.lda = c.Np; g.B = c.Phig.p; g.ldb = c.Np; g.transB = true;
      g.C = L.p; g.ldc = c.nauxp; g.epi = EPI_SQUARE;
      hip_check(gemm_f64(g, st), "metric");
      hip_check(add_diag(L.p, c.nauxp, c.naux, c.nauxp, 1.0, st), "pad diag");
    };
    form_metric();
    int32_t status = 0;
    hip_check(cholesky_lower(L.p, c.nauxp, c.nauxp, dstatus, st), "cholesky");
    hip_check(hipMemcpyAsync(&status, dstatus, 4, hipMemcpyDeviceToHost, st), "copy status");
    hip_check(hipStreamSynchronize(st), "sync");
    if (status != 0) {
      form_metric();
      std::vector<double> dg(c.naux);
      hip_check(hipMemcpy2DAsync(dg.data(), 8, L.p, (c.nauxp + 1) * 8, 8, c.naux, hipMemcpyDeviceToHost, st),
                "copy diag");
      hip_check(hipStreamSynchronize(st), "sync");
      double mx = 0.0;
      for (double v : dg) mx = std::max(mx, v);
      c.shift = kCholShift * mx;
      hip_check(add_diag(L.p, c.nauxp, 0, c.naux, c.shift, st), "shift");
      hip_check(cholesky_lower(L.p, c.nauxp, c.nauxp, dstatus, st), "cholesky");
      hip_check(hipMemcpyAsync(&status, dstatus, 4, hipMemcpyDeviceToHost, st), "copy status");
      hip_check(hipStreamSynchronize(st), "sync");
      if (status != 0) {
        (void)hipFree(dstatus);
        fail(RPS_ERR_NOT_PD, "fitting metric is not positive definite at row " + std::to_string(status - 1) +
                                 " even with the diagonal shift (duplicate or degenerate points?)");
      }
    }
    (void)hipFree(dstatus);
    stage("fitting metric and Cholesky", st);
    // ---- chi = X_gg^-1 X_gR in column panels, in place in V: X_gR = (Phi_g Phi^T)^2 for
    //      the panel, then the two triangular solves on it
    {
      int64_t pw = kChiPanel;
      if (const char* e = getenv("RPS_CHI_PANEL")) {     // tuning sweeps: columns per panel
        const int64_t v = atoll(e);
        if (v >= 64 && v % 64 == 0) pw = v;
      }
      pw = std::min(pw, c.ngp);
      for (int64_t r0 = 0; r0 < c.ngp; r0 += pw) {
        const int64_t nc = std::min(pw, c.ngp - r0);
        Gemm g;
        g.M = c.nauxp; g.N = nc; g.K = c.Np;
        g.A = c.Phig.p; g.lda = c.Np; g.B = c.Phi.p + r0 * c.Np; g.ldb = c.Np; g.transB = true;
        g.C = c.V.p + r0; g.ldc = c.ngp; g.epi = EPI_SQUARE;
        hip_check(gemm_f64(g, st), "X_gR panel");
        hip_check(tri_solve_lower(L.p, c.nauxp, c.nauxp, c.V.p + r0, nc, c.ngp, false, st), "solve L");
        hip_check(tri_solve_lower(L.p, c.nauxp, c.nauxp, c.V.p + r0, nc, c.ngp, true, st), "solve L^T");
      }
      hip_check(hipStreamSynchronize(st), "sync");
    }
    stage("fitting functions chi", st);
    hip_check(hipStreamSynchronize(st), "sync");
    L.release(nullptr);
    // ---- V = Vc chi (Sec. 3.2) and W = V chi^T (Eq. 14) together, in row panels.  While
    //      panel a turns from chi into V, the rows after it still hold chi, so the block
    //      row W[a, a:] = V[a] chi[a:]^T is formed then (chi[a] itself from a copy kept for
    //      the diagonal block).  W is symmetric: the upper triangle is formed, the lower one
    //      copied from it.  Half the flops of the full product, and chi is not re-formed.
    {
      int64_t P = kWPanel;
      if (const char* wp = getenv("RPS_W_PANEL")) {      // smaller panels (tests of the panel path)
        const int64_t v = atoll(wp);
        if (v >= 64 && v <= kWPanel && v % 64 == 0) P = v;
      }
      P = std::min(P, c.nauxp);                          // a multiple of 64 (rows in pairs)
      DBuf<double> X, work;
      X.alloc(P * c.ngp, &tmpb);
      work.alloc(kSplitWork, &tmpb);
      for (int64_t a0 = 0; a0 < c.nauxp; a0 += P) {
        const int64_t pa = std::min(P, c.nauxp - a0);
        double* Va = c.V.p + a0 * c.ngp;
        hip_check(hipMemcpyAsync(X.p, Va, (size_t)(pa * c.ngp) * 8, hipMemcpyDeviceToDevice, st), "chi panel");
        hip_check(poisson_rows(Va, pa, c.ngp, c.mesh, dkern, st), "poisson");
        for (int part = 0; part < 2; ++part) {
          Gemm g;   // part 0: W[a, a] = V[a] chi[a]^T; part 1: W[a, after a] = V[a] chi[after a]^T
          g.M = pa; g.K = c.ngp;
          g.N = (part == 0) ? pa : c.nauxp - a0 - pa;
          if (g.N <= 0) continue;
          g.A = Va; g.lda = c.ngp;
          g.B = (part == 0) ? X.p : Va + pa * c.ngp; g.ldb = c.ngp; g.transB = true;
          g.C = c.W.p + a0 * c.nauxp + a0 + ((part == 0) ? 0 : pa); g.ldc = c.nauxp;
          gemm_plan(g, kSplitWork);
          g.work = work.p;
          hip_check(gemm_f64(g, st), "W block row");
        }
      }
      hip_check(mirror_upper(c.W.p, c.nauxp, c.nauxp, st), "mirror");
      hip_check(hipStreamSynchronize(st), "sync");
      X.release(nullptr);
      work.release(nullptr);
    }
    stage("potentials V and W", st);
  }
  hip_check(hipStreamSynchronize(st), "sync");
  if (prec != RPS_PREC_FP64) {
    if (!given32) {
      c.V32.alloc(c.nauxp * c.ngp, &c.bytes);
      hip_check(to_f32(c.V.p, c.nauxp * c.ngp, c.V32.p, st), "to f32");
      hip_check(hipStreamSynchronize(st), "sync");
      c.V.release(&c.bytes);      // the precision form keeps only the FP32 copy of V
    }
    const char* fu = getenv("RPS_F32_FUSED_U");
    if (c.Np <= 128 && !(fu && fu[0] == '0')) {
      c.Phi32.alloc(c.ngp * c.Np, &c.bytes);
      hip_check(to_f32(c.Phi.p, c.ngp * c.Np, c.Phi32.p, st), "Phi to f32");
      hip_check(hipStreamSynchronize(st), "sync");
    }
  }
  const char* sb = getenv("RPS_SCREENED_BLOCKS");   // "0": screened values in dense form only (tests)
  if (basis_eps > 0.0 && !(sb && sb[0] == '0')) {
    build_screened_blocks(c, b->atom_xyz, st);
    stage("screened basis blocks", st);
  }
  // device address of the no-allocation build's static scratch on this device, taken
  // here so that loading the array happens at set-up, not inside that build
  (void)scratch_device_ptr();
  c.setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// ------------------------------------------------------------------ builds
constexpr int kEvPerBuild = 6;
constexpr int64_t kMaxProfiled = 65536;

hipEvent_t prof_event(rps_context& c, int slot) {
  const int64_t i = c.ev_used * kEvPerBuild + slot;
  while ((int64_t)c.ev_pool.size() <= i) {
    hipEvent_t e;
    hip_check(hipEventCreate(&e), "hipEventCreate");
    c.ev_pool.push_back(e);
  }
  return c.ev_pool[i];
}

void prof_mark(rps_context& c, int slot, hipStream_t st) {
  if (!c.profiling || c.ev_used >= kMaxProfiled) return;
  hip_check(hipEventRecord(prof_event(c, slot), st), "hipEventRecord");
}

// Launch shape of the fused V-streaming kernel for n padded to np:
// one workgroup per CU (8 waves when np == 16, else 4), all g rows of a
// workgroup kept in LDS (M2 accumulators) unless they do not fit, then
// g blocks; R tiles split so that the workgroups cover the CUs once.
// The precision form with n <= 16 forms the orbitals in its kernel when the FP32
// basis is stored (N <= 128).
bool uses_f32u(const rps_context& c, int np) { return c.Phi32.p && np == 16; }

void choose_shape(rps_context& c, int np, FusedArgs& a) {
  a.nwaves = (np == 16) ? 8 : 4;
  a.np = np;
  a.G = c.nauxp;
  a.want_m2 = 1;
  const int64_t lds_cap = 160 * 1024;
  const int64_t gt = c.nauxp / 64;
  const bool f32u = uses_f32u(c, np);
  // the in-kernel-orbitals kernel holds M2 in registers (at most 8 g subtiles per
  // wave); the others hold this workgroup's M2 block in LDS
  a.Np = (int)c.Np;
  auto fits = [&](const FusedArgs& t) {
    // (the in-kernel-orbitals kernel stays within its registers up to 5 subtiles per wave)
    return f32u ? (fused_f32u_nmy(t) <= 5 && fused_f32u_lds(t) <= lds_cap) : fused_lds_bytes(t) <= lds_cap;
  };
  a.gblocks = 1;
  a.rtiles = 1;
  while (true) {
    if (fits(a) || a.gblocks >= gt) break;
    ++a.gblocks;
  }
  const int64_t rt = c.ngp / 64;
  const int64_t target = std::max<int64_t>(1, 256 / a.gblocks);
  a.rtiles = (int)std::max<int64_t>(1, (rt + target - 1) / target);
  // launch-shape override for tuning sweeps: RPS_FUSED_SHAPE="rtiles,gblocks"
  if (const char* ov = getenv("RPS_FUSED_SHAPE")) {
    int x = 0, y = 0;
    if (sscanf(ov, "%d,%d", &x, &y) == 2 && x >= 1 && y >= 1 && y <= gt) {
      FusedArgs t = a;
      t.rtiles = x;
      t.gblocks = y;
      if (fits(t)) { a.rtiles = x; a.gblocks = y; }
    }
  }
  if (c.tune_rtiles > 0 && c.tune_gblocks > 0 && c.tune_gblocks <= gt) {
    FusedArgs t = a;
    t.rtiles = c.tune_rtiles;
    t.gblocks = c.tune_gblocks;
    if (fits(t)) { a.rtiles = t.rtiles; a.gblocks = t.gblocks; }
  }
}

// Partials and the zeroed counter of the finalize kernel's split energy sum.
void ensure_energy_parts(rps_context& c) {
  if (c.epart.p) return;
  c.epart.alloc(kEnergyBlocks, &c.bytes);
  c.ecount.alloc(1, &c.bytes);
  hip_check(hipMemset(c.ecount.p, 0, sizeof(unsigned)), "hipMemset");
}

// Launch shape and buffer sizes (in doubles) of the fused path's workspace for
// padded n = np; the same plan serves the context's own buffers and the
// no-allocation entry point's static scratch, so both give identical builds.
struct FusedPlan {
  int rtiles, gblocks, nwaves;
  int64_t rblocks_main, blocks_main, blocks_l3;
  bool f32u, m4;
  int64_t nU, nUg, nUgp, nM2p, ne3u, nK1p, nK3p, ne1p, ne3p, nM2, nK1, nK3;
};

FusedPlan fused_plan(rps_context& c, int np) {
  FusedPlan p{};
  FusedArgs a{};
  a.R_valid = c.ng;
  choose_shape(c, np, a);
  p.rtiles = a.rtiles;
  p.gblocks = a.gblocks;
  p.nwaves = a.nwaves;
  p.rblocks_main = fused_rblocks(a);
  p.blocks_main = p.rblocks_main * p.gblocks;
  p.blocks_l3 = (c.nauxp / 64) * ((c.naux + 63) / 64);   // one 64 x 64 tile of W per workgroup
  p.f32u = uses_f32u(c, np);
  p.m4 = (np == 16) && c.use_m4;
  const int64_t nsub = c.nauxp / 16;
  p.nU = c.ngp * np;
  p.nUg = c.nauxp * np;
  p.nUgp = c.nauxp * np;
  // M2 partials, followed by the negated fit-fit partials of the in-kernel-orbitals kernel
  p.nM2p = (p.rblocks_main + (p.f32u ? nsub : 0)) * c.nauxp * np;
  p.ne3u = p.f32u ? nsub * nsub : 1;
  p.nK1p = p.blocks_main * c.Np * np;
  p.nK3p = std::max<int64_t>(p.blocks_l3, 1) * c.Np * np;
  p.ne1p = p.blocks_main;
  p.ne3p = std::max<int64_t>(p.blocks_l3, 1);
  p.nM2 = c.nauxp * np;
  p.nK1 = c.Np * np;
  p.nK3 = c.Np * np;
  return p;
}

// Pointers of the fused path's workspace (the context's buffers, or carved
// from the static scratch by the no-allocation entry point).
struct FusedWs {
  FusedPlan plan;
  double *U = nullptr, *Ug = nullptr, *Ugp = nullptr, *M2p = nullptr, *e3u = nullptr, *K1p = nullptr,
         *K3p = nullptr, *e1p = nullptr, *e3p = nullptr, *M2 = nullptr, *K1 = nullptr, *K3 = nullptr,
         *epart = nullptr;
  unsigned* ecount = nullptr;
};

void ensure_workspace(rps_context& c, int np) {
  if (c.ws_np == np) return;
  c.clear_graphs();          // captured builds refer to the buffers about to change
  int64_t* cnt = &c.bytes;
  if (const char* m = getenv("RPS_FP64_MFMA"))
    c.use_m4 = (strcmp(m, "16x16x4") == 0) ? 0 : (strcmp(m, "hybrid") == 0) ? 2 : 1;
  const FusedPlan p = fused_plan(c, np);
  c.rtiles = p.rtiles;
  c.gblocks = p.gblocks;
  c.nwaves = p.nwaves;
  c.rblocks_main = p.rblocks_main;
  c.blocks_main = p.blocks_main;
  c.blocks_l3 = p.blocks_l3;
  c.U.alloc(p.nU, cnt);
  c.Ug.alloc(p.nUg, cnt);
  c.Ugp.alloc(p.nUgp, cnt);
  c.M2p.alloc(p.nM2p, cnt);
  c.e3u.alloc(p.ne3u, cnt);
  ensure_energy_parts(c);
  c.K1p.alloc(p.nK1p, cnt);
  c.K3p.alloc(p.nK3p, cnt);
  c.e1p.alloc(p.ne1p, cnt);
  c.e3p.alloc(p.ne3p, cnt);
  c.M2.alloc(p.nM2, cnt);
  c.K1.alloc(p.nK1, cnt);
  c.K3.alloc(p.nK3, cnt);
  c.Cdev.alloc(c.nbas * np, cnt);
  c.Kdev.alloc(c.nbas * np, cnt);
  c.exdev.alloc(1, cnt);
  c.ws_np = np;
}

FusedWs context_ws(rps_context& c, int np) {
  FusedWs w;
  w.plan.f32u = uses_f32u(c, np);
  w.plan.m4 = (np == 16) && c.use_m4;
  w.plan.rtiles = c.rtiles;
  w.plan.gblocks = c.gblocks;
  w.plan.nwaves = c.nwaves;
  w.plan.rblocks_main = c.rblocks_main;
  w.plan.blocks_main = c.blocks_main;
  w.plan.blocks_l3 = c.blocks_l3;
  w.U = c.U.p; w.Ug = c.Ug.p; w.Ugp = c.Ugp.p; w.M2p = c.M2p.p; w.e3u = c.e3u.p; w.K1p = c.K1p.p;
  w.K3p = c.K3p.p; w.e1p = c.e1p.p; w.e3p = c.e3p.p; w.M2 = c.M2.p; w.K1 = c.K1.p; w.K3 = c.K3.p;
  w.epart = c.epart.p; w.ecount = c.ecount.p;
  return w;
}

// ------------------------------------------------------------------ general path
// Any N and n.  The GEMM form (padded n above the streaming form's limit) takes
// the grid in chunks c of R_c columns of V:
//   A_c = V[:, c] o (U_g U[c]^T)          (N_aux x R_c; the epilogue multiplies by V)
//   M1^T[c] = A_c^T U_g                    (rows c of M1^T, written once)
//   M2 += A_c U[c]                         (N_aux x n, accumulated over the chunks)
// then K1 = Phi^T M1^T, K2 = Phi_g^T M2, B = W o (U_g U_g^T), Y = B U_g,
// K3 = Phi_g^T Y, e1 = tr(U_g^T M2), e3 = tr(U_g^T Y)  (Eq. 16).  In the
// precision form the three chunk products run on the FP32 matrix cores with V,
// U and U_g in FP32 and A_c stored in FP32, and so does K1 (dense basis) from FP32
// copies of Phi and M1^T; the products into M1^T, M2 and K1 sum 64 terms at a
// time in FP32 and everything beyond (longer sums, splits, chunks, K) in FP64.
// U = Phi C stays FP64 (its rounding enters every product of the build); the U
// product and the M1^T chunk products also write the FP32 copies the later
// products read (rounded from their FP64 results).

// workspace of the products with the screened basis's atom blocks
void ensure_sparse_ws(rps_context& c, int np) {
  if (c.sws_np == np) return;
  c.clear_graphs();
  c.sCg.alloc(std::max<int64_t>(c.fofs[c.natom], 1) * np, &c.bytes);
  c.sK1p.alloc(std::max<int64_t>(c.fofs[c.natom], 1) * np, &c.bytes);
  c.sUv.alloc(c.ng * np, &c.bytes);
  // U rows of atom I = Phi_I C[S_I] (an empty function list gives zero rows: K = 0);
  // K1 partial rows of atom I = Phi_I^T M1T[kappa_I]
  std::vector<GemmItem> ut, kt;
  for (int I = 0; I < c.natom; ++I) {
    const int64_t nr = c.vofs[I + 1] - c.vofs[I], nc = c.fofs[I + 1] - c.fofs[I];
    if (nr > 0) ut.push_back(GemmItem{nr, np, nc, std::max<int64_t>(nc, 1), np, np, c.pofs[I], c.fofs[I] * np,
                                      c.vofs[I] * np, 0});
    if (nc > 0) kt.push_back(GemmItem{nc, np, nr, nc, np, np, c.pofs[I], c.vofs[I] * np, c.fofs[I] * np, 0});
  }
  auto up = [&](DBuf<GemmItem>& d, const std::vector<GemmItem>& h) {
    d.alloc(std::max<int64_t>((int64_t)h.size(), 1), &c.bytes);
    if (!h.empty()) hip_check(hipMemcpy(d.p, h.data(), h.size() * sizeof(GemmItem), hipMemcpyHostToDevice), "items");
    d.n = (int64_t)h.size();
  };
  up(c.sitU, ut);
  up(c.sitK1, kt);
  c.sws_np = np;
}

void ensure_general(rps_context& c, int np) {
  if (c.sparse) ensure_sparse_ws(c, np);
  if (c.gws_np == np) return;
  c.clear_graphs();
  int64_t* cnt = &c.bytes;
  const bool f32 = c.precision != RPS_PREC_FP64;
  const int64_t budget = 2000000000ll / (f32 ? 4 : 8);     // A chunk: about 2 GB
  int64_t rc = std::max<int64_t>(128, budget / c.nauxp / 128 * 128);
  if (const char* e = getenv("RPS_GEMM_RCHUNK")) rc = std::max<int64_t>(1, atoll(e));   // tests: ragged chunks
  rc = std::min(rc, c.ngp);
  c.gchunk = rc;
  c.gCp.alloc(c.Np * np, cnt);
  c.gU.alloc(c.ngp * np, cnt);
  c.gUg.alloc(c.nauxp * np, cnt);
  c.gU32.release(cnt);
  c.gUg32.release(cnt);
  c.gA32.release(cnt);
  c.gM1T32.release(cnt);
  if (np > kStreamMaxNp || getenv("RPS_GENERAL_GEMM")) {
    c.gSp.release(cnt);
    if (f32) {
      const int64_t npg = round_up(np, 64);      // FP32 copies padded to whole 64-column tiles
      c.gA.alloc(c.nauxp * c.nauxp, cnt);      // B of the fit-fit line (FP64)
      c.gA32.alloc(c.nauxp * rc, cnt);
      c.gU32.alloc(c.ngp * npg, cnt);
      c.gUg32.alloc(c.nauxp * npg, cnt);
      // the products write only the first np columns of these FP32 copies: the padding
      // columns are cleared here, once (npg is even: cleared as pairs of floats)
      hip_check(fill(reinterpret_cast<double*>(c.gU32.p), c.ngp * npg / 2, 0.0, nullptr), "clear U32");
      if (!c.sparse) {
        c.gM1T32.alloc(c.ngp * npg, cnt);
        hip_check(fill(reinterpret_cast<double*>(c.gM1T32.p), c.ngp * npg / 2, 0.0, nullptr), "clear M1T32");
      }
      hip_check(hipStreamSynchronize(nullptr), "sync");    // before any build's stream writes them
      if (!c.sparse) {
        if (!c.gPhi32.p) {    // the basis does not change after set-up: converted once, here (no capture)
          c.gPhi32.alloc(c.ngp * c.Np, cnt);
          hip_check(to_f32(c.Phi.p, c.ngp * c.Np, c.gPhi32.p, nullptr), "Phi to f32");
          hip_check(hipStreamSynchronize(nullptr), "sync");
        }
      }
    } else {
      c.gA.alloc(std::max(c.nauxp * rc, c.nauxp * c.nauxp), cnt);
    }
  } else {
    c.gA.release(cnt);
    c.gSp.alloc(kStreamPartRows * np, cnt);    // split partials of the streaming form
    if (f32) {                                  // FP32 copies of the Y operands of the passes
      c.gU32.alloc(c.ngp * np, cnt);
      c.gUg32.alloc(c.nauxp * np, cnt);
    }
  }
  c.gM2.alloc(c.nauxp * np, cnt);
  c.gM1T.alloc(c.ngp * np, cnt);
  c.gK1.alloc(c.Np * np, cnt);
  c.gK3.alloc(c.Np * np, cnt);
  c.gY.alloc(c.nauxp * np, cnt);
  c.gwork.alloc(kSplitWork, cnt);
  ensure_energy_parts(c);
  c.Cdev.alloc(c.nbas * np, cnt);
  c.Kdev.alloc(c.nbas * np, cnt);
  c.exdev.alloc(1, cnt);
  c.gws_np = np;
}

void gemm_run(Gemm g, rps_context& c, hipStream_t st, const char* what, bool allow_split) {
  if (allow_split && g.epi == EPI_AXPBY) {
    gemm_plan(g, kSplitWork);
    g.work = c.gwork.p;
  } else if (!g.kscale && g.N > 64) {
    g.tile_n = ((g.N + 63) / 64 * 64 < (g.N + 127) / 128 * 128) ? 64 : 128;   // less padding
  }
  hip_check(gemm_f64(g, st), what);
}

// ---- products with the screened basis (atom blocks; see k_sparse.hip)
// U (ngp x np, grid order) = Phi C from the atom blocks; Cp is C packed [Np][np]
void sparse_u(rps_context& c, const double* Cp, int np, double* U, hipStream_t st) {
  ensure_sparse_ws(c, np);
  const int64_t F = c.fofs[c.natom];
  if (F > 0) hip_check(gather_rows(Cp, np, c.sfun.p, F, F, np, c.sCg.p, np, st), "C rows");
  Gemm g;   // U[kappa_I] = Phi_I C[S_I] for every atom
  g.A = c.sPhi.p; g.B = c.sCg.p; g.C = c.sUv.p;
  hip_check(gemm_f64_grouped(g, c.sitU.p, (int)c.sitU.n, c.smaxr, np, st), "U blocks");
  hip_check(gather_rows(c.sUv.p, np, c.sinv.p, c.ng, c.ngp, np, U, np, st), "U rows");
}

// K1 (Np x np) = Phi^T M1T from the atom blocks (M1T: ngp x np, grid order)
void sparse_k1(rps_context& c, const double* M1T, int np, double* K1, hipStream_t st) {
  ensure_sparse_ws(c, np);
  hip_check(gather_rows(M1T, np, c.sperm.p, c.ng, c.ng, np, c.sUv.p, np, st), "M1 rows");
  Gemm g;   // partial K1 rows of every atom: Phi_I^T M1T[kappa_I]
  g.A = c.sPhi.p; g.transA = true; g.B = c.sUv.p; g.C = c.sK1p.p;
  hip_check(gemm_f64_grouped(g, c.sitK1.p, (int)c.sitK1.n, c.smaxc, np, st), "K1 blocks");
  hip_check(csr_rowsum(c.sK1p.p, np, c.smu_ofs.p, c.smu_rows.p, (int)c.nbas, (int)c.Np, K1, st), "K1 sums");
}

// The streaming passes of a general-path build (one description, used by the eager
// build and by the batching form's persistent launches alike).
StreamArgs pass_m2(const rps_context& c, int np) {   // M2 = (V o P) U, x = interpolation points
  StreamArgs m2;
  m2.V = c.V.p; m2.V32 = c.V32.p; m2.ldv = c.ngp; m2.trans = 0;
  m2.X = c.gUg.p; m2.ldx = np; m2.Y = c.gU.p; m2.Y32 = c.gU32.p; m2.ldy = np;
  m2.nx = c.nauxp; m2.ny = c.ngp; m2.np = np; m2.out = c.gSp.p;
  return m2;
}
StreamArgs pass_m1(const rps_context& c, int np) {   // M1^T = (V o P)^T U_g, x = grid points
  StreamArgs m1;
  m1.V = c.V.p; m1.V32 = c.V32.p; m1.ldv = c.ngp; m1.trans = 1;
  m1.X = c.gU.p; m1.ldx = np; m1.Y = c.gUg.p; m1.Y32 = c.gUg32.p; m1.ldy = np;
  m1.nx = c.ngp; m1.ny = c.nauxp; m1.np = np; m1.out = c.gM1T.p;
  return m1;
}
StreamArgs pass_l3(const rps_context& c, int np, double* out) {   // Y = (W o P_g) U_g, FP64
  StreamArgs l3;
  l3.V = c.W.p; l3.ldv = c.nauxp; l3.trans = 0;
  l3.X = c.gUg.p; l3.ldx = np; l3.Y = c.gUg.p; l3.ldy = np;
  l3.nx = c.nauxp; l3.ny = c.nauxp; l3.np = np; l3.out = out;
  return l3;
}
int pass_splits(const rps_context& c, const StreamArgs& a) {
  return stream_splits(a.nx, a.ny, c.tune_target > 0 ? c.tune_target : kStreamBlocks);
}

// Before the passes: C packed, U = Phi C, U_g, and the FP32 copies the precision forms read.
// With uf set (dense basis), the U product also writes U rounded to FP32 there (pitch
// lduf); the return value says whether it did.
bool general_pre(rps_context& c, int nocc, const double* Csrc, hipStream_t st, bool f32_copies,
                 float* uf = nullptr, int64_t lduf = 0) {
  const int np = (int)round_up(nocc, 16);
  bool wrote_uf = false;
  hip_check(pack_matrix(Csrc, c.nbas, nocc, nocc, c.gCp.p, c.Np, np, st), "pack C");
  if (c.sparse) {
    sparse_u(c, c.gCp.p, np, c.gU.p, st);
  } else {
    Gemm g;   // U = Phi C
    g.M = c.ngp; g.N = np; g.K = c.Np;
    g.A = c.Phi.p; g.lda = c.Np; g.B = c.gCp.p; g.ldb = np; g.C = c.gU.p; g.ldc = np;
    if (uf) { g.Cf = uf; g.ldcf = lduf; wrote_uf = true; }
    gemm_run(g, c, st, "U", false);
  }
  hip_check(gather_rows(c.gU.p, np, c.dpoints.p, c.naux, c.nauxp, np, c.gUg.p, np, st), "U_g");
  if (f32_copies) {
    hip_check(to_f32(c.gU.p, c.ngp * np, c.gU32.p, st), "U to f32");
    hip_check(to_f32(c.gUg.p, c.nauxp * np, c.gUg32.p, st), "U_g to f32");
  }
  return wrote_uf;
}

void build_general(rps_context& c, int variant, int nocc, const double* Csrc, double* Kout, double* exout,
                   hipStream_t st, double s1, double s2, double s3, double ce1, double ce3) {
  const int np = (int)round_up(nocc, 16);
  ensure_general(c, np);
  const bool need_main = (variant != RPS_VARIANT_THC);
  const bool need_l3 = (variant != RPS_VARIANT_PS);
  const bool k1 = need_main && variant == RPS_VARIANT_RPS;
  const bool stream = c.gSp.p != nullptr && np <= kStreamMaxNp;
  // GEMM form with FP32 products: U rounded to FP32 by the U product itself
  const bool gemm_f32_form = !stream && need_main && c.gA32.p != nullptr;
  const bool u32_done = general_pre(c, nocc, Csrc, st, false, gemm_f32_form ? c.gU32.p : nullptr,
                                    round_up(np, 64));
  // the streaming passes run the context's precision; the GEMM form runs FP32
  // products for either precision form
  c.last_arith = stream ? c.precision : (c.gA32.p != nullptr ? RPS_PREC_FP32 : RPS_PREC_FP64);
  if (stream) {
    // streaming form: O never materialises A = V o P (see k_stream.hip)
    const int prec = c.precision;
    if (need_main) {
      prof_mark(c, 1, st);
      if (prec != RPS_PREC_FP64) {
        hip_check(to_f32(c.gU.p, c.ngp * np, c.gU32.p, st), "U to f32");
        hip_check(to_f32(c.gUg.p, c.nauxp * np, c.gUg32.p, st), "U_g to f32");
      }
      const StreamArgs m2 = pass_m2(c, np);
      const int sp = pass_splits(c, m2);
      hip_check(stream_product(m2, prec, sp, st), "stream M2");
      hip_check(sum_partials3(c.gSp.p, sp, c.nauxp * np, c.gM2.p, nullptr, 0, 0, nullptr, nullptr, 0, 0, nullptr, st),
                "M2 partials");
      if (k1) hip_check(stream_product(pass_m1(c, np), prec, 1, st), "stream M1");
      prof_mark(c, 2, st);
      if (k1 && c.sparse) {
        sparse_k1(c, c.gM1T.p, np, c.gK1.p, st);
      } else if (k1) {
        Gemm g;   // K1 = Phi^T M1^T
        g.M = c.Np; g.N = np; g.K = c.ngp;
        g.A = c.Phi.p; g.lda = c.Np; g.transA = true; g.B = c.gM1T.p; g.ldb = np; g.C = c.gK1.p; g.ldc = np;
        gemm_run(g, c, st, "K1", true);
      }
    }
    if (need_l3) {
      prof_mark(c, 3, st);
      const StreamArgs l3 = pass_l3(c, np, c.gSp.p);
      const int sp = pass_splits(c, l3);
      hip_check(stream_product(l3, RPS_PREC_FP64, sp, st), "stream line 3");
      hip_check(sum_partials3(c.gSp.p, sp, c.nauxp * np, c.gY.p, nullptr, 0, 0, nullptr, nullptr, 0, 0, nullptr, st),
                "line-3 partials");
      Gemm k3;    // K3 = Phi_g^T Y
      k3.M = c.Np; k3.N = np; k3.K = c.nauxp;
      k3.A = c.Phig.p; k3.lda = c.Np; k3.transA = true; k3.B = c.gY.p; k3.ldb = np; k3.C = c.gK3.p; k3.ldc = np;
      gemm_run(k3, c, st, "K3", true);
      prof_mark(c, 4, st);
    }
  } else if (need_main) {
    const bool f32 = c.gA32.p != nullptr;
    // FP32 copies of U and U_g with npg >= np columns, zero beyond np: every tile of
    // the n dimension then loads whole 16-byte pieces
    const int64_t npg = round_up(np, 64);
    if (f32) {
      if (!u32_done) hip_check(to_f32_pad(c.gU.p, c.ngp, np, c.gU32.p, npg, st), "U to f32");
      hip_check(to_f32_pad(c.gUg.p, c.nauxp, np, c.gUg32.p, npg, st), "U_g to f32");
    }
    prof_mark(c, 1, st);     // the profiled main phase: the chunk products only
    constexpr int64_t kF32Terms = 1ll << 40;   // split for parallelism only (FP32 sums are short)
    for (int64_t r0 = 0; r0 < c.ngp; r0 += c.gchunk) {
      const int64_t rc = std::min(c.gchunk, c.ngp - r0);
      if (f32) {
        Gemm32 a;   // A_c = V[:, c] o (U_g U[c]^T), FP32; K = np rounded up to whole
        a.M = c.nauxp; a.N = rc; a.K = round_up(np, 16);   // 16-deep steps (zero columns add nothing)
        a.A = c.gUg32.p; a.lda = npg; a.B = c.gU32.p + r0 * npg; a.ldb = npg; a.transB = true;
        a.C32 = c.gA32.p; a.ldc = rc; a.D32 = c.V32.p + r0; a.ldd = c.ngp;
        hip_check(gemm_f32(a, st), "A chunk");
        if (k1) {
          Gemm32 m1;   // M1^T[c] = A_c^T U_g
          m1.M = rc; m1.N = np; m1.Nread = npg; m1.K = c.nauxp;
          m1.A = c.gA32.p; m1.lda = rc; m1.transA = true; m1.B = c.gUg32.p; m1.ldb = npg;
          m1.C = c.gM1T.p + r0 * np; m1.ldc = np;
          if (c.gM1T32.p) { m1.Cf = c.gM1T32.p + r0 * npg; m1.ldcf = npg; }   // FP32 copy for K1
          m1.splitk = gemm32_splitk_for(m1.M, m1.N, m1.K, kF32Terms, kSplitWork); m1.work = c.gwork.p;
          hip_check(gemm_f32(m1, st), "M1");
        }
        Gemm32 m2;     // M2 += A_c U[c]
        m2.M = c.nauxp; m2.N = np; m2.Nread = npg; m2.K = rc;
        m2.A = c.gA32.p; m2.lda = rc; m2.B = c.gU32.p + r0 * npg; m2.ldb = npg;
        m2.C = c.gM2.p; m2.ldc = np; m2.beta = (r0 == 0) ? 0.0 : 1.0;
        m2.splitk = gemm32_splitk_for(m2.M, m2.N, m2.K, kF32Terms, kSplitWork); m2.work = c.gwork.p;
        hip_check(gemm_f32(m2, st), "M2");
      } else {
        Gemm a;     // A_c = V[:, c] o (U_g U[c]^T)
        a.M = c.nauxp; a.N = rc; a.K = np;
        a.A = c.gUg.p; a.lda = np; a.B = c.gU.p + r0 * np; a.ldb = np; a.transB = true;
        a.C = c.gA.p; a.ldc = rc; a.epi = EPI_HADAMARD_SRC; a.D = c.V.p + r0; a.ldd = c.ngp;
        gemm_run(a, c, st, "A chunk", false);
        if (k1) {
          Gemm m1;  // M1^T[c] = A_c^T U_g
          m1.M = rc; m1.N = np; m1.K = c.nauxp;
          m1.A = c.gA.p; m1.lda = rc; m1.transA = true; m1.B = c.gUg.p; m1.ldb = np;
          m1.C = c.gM1T.p + r0 * np; m1.ldc = np;
          gemm_run(m1, c, st, "M1", true);
        }
        Gemm m2;    // M2 += A_c U[c]
        m2.M = c.nauxp; m2.N = np; m2.K = rc;
        m2.A = c.gA.p; m2.lda = rc; m2.B = c.gU.p + r0 * np; m2.ldb = np;
        m2.C = c.gM2.p; m2.ldc = np; m2.beta = (r0 == 0) ? 0.0 : 1.0;
        gemm_run(m2, c, st, "M2", true);
      }
    }
    prof_mark(c, 2, st);
    if (k1 && c.sparse) {
      sparse_k1(c, c.gM1T.p, np, c.gK1.p, st);
    } else if (k1 && f32) {
      // K1 = Phi^T M1^T on the FP32 matrix cores: FP32 basis, M1^T rounded to FP32
      // (padded to npg columns), FP32 sums over 64 terms and FP64 beyond
      // (M1^T rounded to FP32 by its chunk products)
      Gemm32 g;
      g.M = c.Np; g.N = np; g.Nread = npg; g.K = c.ngp;
      g.A = c.gPhi32.p; g.lda = c.Np; g.transA = true; g.B = c.gM1T32.p; g.ldb = npg;
      g.C = c.gK1.p; g.ldc = np;
      // 22 x 7 output tiles at the 3x3x3 cell: the long K is split 32-39 ways for parallelism
      g.splitk = gemm32_splitk_for(g.M, g.N, g.K, (g.K + 31) / 32, kSplitWork); g.work = c.gwork.p;
      hip_check(gemm_f32(g, st), "K1");
    } else if (k1) {
      Gemm g;   // K1 = Phi^T M1^T
      g.M = c.Np; g.N = np; g.K = c.ngp;
      g.A = c.Phi.p; g.lda = c.Np; g.transA = true; g.B = c.gM1T.p; g.ldb = np; g.C = c.gK1.p; g.ldc = np;
      gemm_run(g, c, st, "K1", true);
    }
  }
  if (need_l3 && !stream) {
    prof_mark(c, 3, st);
    Gemm b;     // B = W o (U_g U_g^T)
    b.M = c.nauxp; b.N = c.nauxp; b.K = np;
    b.A = c.gUg.p; b.lda = np; b.B = c.gUg.p; b.ldb = np; b.transB = true;
    b.C = c.gA.p; b.ldc = c.nauxp; b.epi = EPI_HADAMARD_SRC; b.D = c.W.p; b.ldd = c.nauxp;
    gemm_run(b, c, st, "B", false);
    Gemm y;     // Y = B U_g
    y.M = c.nauxp; y.N = np; y.K = c.nauxp;
    y.A = c.gA.p; y.lda = c.nauxp; y.B = c.gUg.p; y.ldb = np; y.C = c.gY.p; y.ldc = np;
    gemm_run(y, c, st, "Y", true);
    Gemm k3;    // K3 = Phi_g^T Y
    k3.M = c.Np; k3.N = np; k3.K = c.nauxp;
    k3.A = c.Phig.p; k3.lda = c.Np; k3.transA = true; k3.B = c.gY.p; k3.ldb = np; k3.C = c.gK3.p; k3.ldc = np;
    gemm_run(k3, c, st, "K3", true);
    prof_mark(c, 4, st);
  }
  // e1 = tr(U_g^T M2), e3 = tr(U_g^T Y), formed by the finalize kernel
  EnergyDots dots;
  if (need_main) { dots.x1 = c.gUg.p; dots.y1 = c.gM2.p; dots.n1 = c.nauxp * np; }
  if (need_l3) { dots.x3 = c.gUg.p; dots.y3 = c.gY.p; dots.n3 = c.nauxp * np; }
  dots.part = c.epart.p; dots.nparts = kEnergyBlocks; dots.count = c.ecount.p;
  hip_check(finalize(c.Phig.p, need_main ? c.gM2.p : nullptr, c.nauxp, k1 ? c.gK1.p : nullptr,
                     need_l3 ? c.gK3.p : nullptr, (int)c.nbas, nocc, np, (int)c.Np, s1, s2, s3, c.dV, Kout,
                     nullptr, 0, nullptr, 0, ce1, ce3, exout, st, dots),
            "finalize");
}

// After the passes, in the batching form (rPS variant, streaming form): the ordered
// sums of the M2 partials (sp_m2 of them in gSp) and of the fit-fit partials (sp_l3
// in p3), K1, K3 and the combine, exactly as the eager build forms them.
void general_post(rps_context& c, int nocc, int sp_m2, const double* p3, int sp_l3, double* Kout, double* exout,
                  hipStream_t st) {
  const int np = (int)round_up(nocc, 16);
  hip_check(sum_partials3(c.gSp.p, sp_m2, c.nauxp * np, c.gM2.p, nullptr, 0, 0, nullptr, nullptr, 0, 0, nullptr, st),
            "M2 partials");
  if (c.sparse) {
    sparse_k1(c, c.gM1T.p, np, c.gK1.p, st);
  } else {
    Gemm g;   // K1 = Phi^T M1^T
    g.M = c.Np; g.N = np; g.K = c.ngp;
    g.A = c.Phi.p; g.lda = c.Np; g.transA = true; g.B = c.gM1T.p; g.ldb = np; g.C = c.gK1.p; g.ldc = np;
    gemm_run(g, c, st, "K1", true);
  }
  hip_check(sum_partials3(p3, sp_l3, c.nauxp * np, c.gY.p, nullptr, 0, 0, nullptr, nullptr, 0, 0, nullptr, st),
            "line-3 partials");
  Gemm k3;    // K3 = Phi_g^T Y
  k3.M = c.Np; k3.N = np; k3.K = c.nauxp;
  k3.A = c.Phig.p; k3.lda = c.Np; k3.transA = true; k3.B = c.gY.p; k3.ldb = np; k3.C = c.gK3.p; k3.ldc = np;
  gemm_run(k3, c, st, "K3", true);
  EnergyDots dots;
  dots.x1 = c.gUg.p; dots.y1 = c.gM2.p; dots.n1 = c.nauxp * np;
  dots.x3 = c.gUg.p; dots.y3 = c.gY.p; dots.n3 = c.nauxp * np;
  dots.part = c.epart.p; dots.nparts = kEnergyBlocks; dots.count = c.ecount.p;
  hip_check(finalize(c.Phig.p, c.gM2.p, c.nauxp, c.gK1.p, c.gK3.p, (int)c.nbas, nocc, np, (int)c.Np, 1.0, 1.0, -1.0,
                     c.dV, Kout, nullptr, 0, nullptr, 0, 2.0, -1.0, exout, st, dots),
            "finalize");
  c.last_arith = c.precision;
}

// The fused single-pass kernels cover N <= 128 with n <= 64 (FP64) or n <= 16
// (FP32 form); everything else takes the general path.
bool uses_general(const rps_context& c, int np) {
  bool general = (np > 64) || (c.Np > 128) || (c.precision != RPS_PREC_FP64 && np > 16);
  if (const char* bp = getenv("RPS_BUILD_PATH")) general = general || (strcmp(bp, "general") == 0);
  return general;
}

// The fused path of one build (N <= 128, n within the fused kernels' limits) on
// the workspace w: orbitals, the V-streaming kernel (lines 1-2, and line 3 in
// the in-kernel-orbitals form), the fit-fit kernel, the ordered partial sums and
// the combine.  C, K and ex are device pointers.  prof: record the profiling
// events (the no-allocation entry point passes false: events are created on
// demand).
void enqueue_fused(rps_context& c, const FusedWs& w, int variant, int32_t nocc, const double* Csrc, double* Kout,
                   double* exout, hipStream_t st, hipStream_t st3, bool prof) {
  const int np = (int)round_up(nocc, 16);
  double s1 = 1, s2 = 1, s3 = -1, ce1 = 2, ce3 = -1;
  if (variant == RPS_VARIANT_PS) { s1 = 0; s2 = 1; s3 = 0; ce1 = 1; ce3 = 0; }
  if (variant == RPS_VARIANT_THC) { s1 = 0; s2 = 0; s3 = 1; ce1 = 0; ce3 = 1; }
  // U = Phi C (orbitals on the grid) and U_g = Phi_g C (at the points); the
  // in-kernel-orbitals precision kernel needs U_g only
  const bool m4 = w.plan.m4;
  const bool f32u = w.plan.f32u;
  c.last_arith = (c.precision == RPS_PREC_FP64) ? RPS_PREC_FP64 : RPS_PREC_FP32;   // fused kernels: FP32 products
  hip_check(orbitals(c.Phi.p, f32u ? 0 : c.ngp, c.Phig.p, c.nauxp, (int)c.Np, Csrc, (int)c.nbas, nocc, np, w.U,
                     w.Ug, m4 ? w.Ugp : nullptr, st),
            "orbitals");
  const bool need_main = (variant != RPS_VARIANT_THC);
  const bool need_l3 = (variant != RPS_VARIANT_PS);
  // the in-kernel-orbitals kernel also forms the fit-fit line, as negated partials after
  // the M2 partials (their ordered sum is then M2 - Y; the rPS variant only)
  const bool l3_in_main = f32u && variant == RPS_VARIANT_RPS;
  const int64_t nsub = c.nauxp / 16;
  if (need_main) {
    FusedArgs a{};
    a.Vm = c.V.p; a.ldv = c.ngp; a.Ug = w.Ug; a.Ur = w.U; a.Phir = c.Phi.p;
    a.G = c.nauxp; a.R = c.ngp; a.R_valid = c.ng; a.np = np; a.Np = (int)c.Np;
    a.rtiles = w.plan.rtiles; a.gblocks = w.plan.gblocks; a.nwaves = w.plan.nwaves;
    a.want_m2 = 1; a.want_k1 = (variant == RPS_VARIANT_RPS) ? 1 : 0; a.want_m1 = 0;
    a.want_e = m4 ? 1 : 0;     // sum A o P = tr(U_g^T M2) is formed after the M2 reduction instead
    a.prec = c.precision;
    a.Vm32 = (c.precision != RPS_PREC_FP64) ? c.V32.p : nullptr;
    a.Ugp = m4 ? w.Ugp : nullptr; a.use_m4 = m4 ? c.use_m4 : 0;
    if (f32u) { a.Phi32 = c.Phi32.p; a.Cm = Csrc; a.N = (int)c.nbas; a.n = nocc; }
    if (l3_in_main) {
      a.Wl = c.W.p; a.ldw = c.nauxp;
      a.Yneg = w.M2p + w.plan.rblocks_main * c.nauxp * np; a.e3u = w.e3u;
    }
    a.M2p = w.M2p; a.K1p = w.K1p; a.e1p = w.e1p;
    if (prof) prof_mark(c, 1, st);
    hip_check(fused_exchange(a, st), "fused main");
    if (prof) prof_mark(c, 2, st);
  }
  hipStream_t sl3 = st;
  if (need_l3 && !l3_in_main && st3) {      // fork after the orbitals: line 3 needs only U_g
    hip_check(hipEventRecord(c.gfork, st), "fork");
    hip_check(hipStreamWaitEvent(st3, c.gfork, 0), "fork wait");
    sl3 = st3;
  }
  if (need_l3 && !l3_in_main) {
    FusedArgs a{};
    a.Vm = c.W.p; a.ldv = c.nauxp; a.Ug = w.Ug; a.Ur = w.Ug; a.Phir = c.Phig.p;
    a.G = c.nauxp; a.R = c.nauxp; a.R_valid = c.naux; a.np = np; a.Np = (int)c.Np;
    a.rtiles = 1; a.gblocks = (int)(c.nauxp / 64); a.nwaves = 4;
    a.want_m2 = 0; a.want_k1 = 1; a.want_m1 = 0; a.want_e = 1; a.prec = RPS_PREC_FP64;
    a.Ugp = m4 ? w.Ugp : nullptr; a.use_m4 = m4 ? c.use_m4 : 0;
    a.K1p = w.K3p; a.e1p = w.e3p;
    if (prof) prof_mark(c, 3, sl3);
    hip_check(fused_exchange(a, sl3), "fused line 3");
    if (prof) prof_mark(c, 4, sl3);
  }
  if (sl3 != st) {
    hip_check(hipEventRecord(c.gjoin, sl3), "join");
    hip_check(hipStreamWaitEvent(st, c.gjoin, 0), "join wait");
  }
  const bool k1 = need_main && variant == RPS_VARIANT_RPS;
  const bool k3 = need_l3 && !l3_in_main;
  hip_check(sum_partials3(k1 ? w.K1p : nullptr, w.plan.blocks_main, c.Np * np, w.K1,
                          need_main ? w.M2p : nullptr, w.plan.rblocks_main + (l3_in_main ? nsub : 0),
                          c.nauxp * np, w.M2,
                          k3 ? w.K3p : nullptr, w.plan.blocks_l3, c.Np * np, w.K3, st),
            "partial sums");
  int64_t ne1 = need_main ? w.plan.blocks_main : 0;
  EnergyDots dots;
  dots.part = w.epart; dots.nparts = kEnergyBlocks; dots.count = w.ecount;
  if (need_main && !m4) {      // sum A o P = tr(U_g^T M2), formed by the finalize kernel
    ne1 = 0;
    dots.x1 = w.Ug; dots.y1 = w.M2; dots.n1 = c.nauxp * np;
  }
  if (l3_in_main) {
    // M2 now holds Z = M2 - Y: K = dV (K1 + Phi_g^T Z); E_x = -dV (2 tr(U_g^T Z) + tr(U_g^T Y))
    hip_check(finalize(c.Phig.p, w.M2, c.nauxp, w.K1, nullptr, (int)c.nbas, nocc, np, (int)c.Np, 1.0, 1.0, 0.0,
                       c.dV, Kout, nullptr, 0, w.e3u, nsub * nsub, 2.0, 1.0, exout, st, dots),
              "finalize");
  } else {
    hip_check(finalize(c.Phig.p, need_main ? w.M2 : nullptr, c.nauxp, k1 ? w.K1 : nullptr,
                       k3 ? w.K3 : nullptr, (int)c.nbas, nocc, np, (int)c.Np, s1, s2, s3, c.dV, Kout,
                       w.e1p, ne1, w.e3p, k3 ? w.plan.blocks_l3 : 0, ce1, ce3, exout, st, dots),
              "finalize");
  }
  if (prof) prof_mark(c, 5, st);
  if (prof && c.profiling && c.ev_used < kMaxProfiled) {
    if (!need_main) { prof_mark(c, 1, st); prof_mark(c, 2, st); }
    if (!need_l3 || l3_in_main) { prof_mark(c, 3, st); prof_mark(c, 4, st); }
    ++c.ev_used;
  }
}

// variant coefficients: K = dV (s1 K1 + s2 K2 + s3 K3), E = -dV (ce1 e1 + ce3 e3)
// Enqueue one build on st.  With st3 != NULL (graph capture only) the fit-fit
// kernel of the fused path runs on st3, beside the V-streaming kernel.
void enqueue_build(rps_context& c, int variant, int32_t nocc, const double* C, double* K, double* ex, bool dev,
                   hipStream_t st, hipStream_t st3) {
  const int np = (int)round_up(nocc, 16);
  const bool general = uses_general(c, np);
  double s1 = 1, s2 = 1, s3 = -1, ce1 = 2, ce3 = -1;
  if (variant == RPS_VARIANT_PS) { s1 = 0; s2 = 1; s3 = 0; ce1 = 1; ce3 = 0; }
  if (variant == RPS_VARIANT_THC) { s1 = 0; s2 = 0; s3 = 1; ce1 = 0; ce3 = 1; }
  c.last_stream = st;
  if (general) ensure_general(c, np); else ensure_workspace(c, np);
  prof_mark(c, 0, st);
  const double* Csrc = C;
  if (!dev) {
    hip_check(hipMemcpyAsync(c.Cdev.p, C, (size_t)c.nbas * nocc * 8, hipMemcpyHostToDevice, st), "copy C");
    Csrc = c.Cdev.p;
  }
  if (general) {
    double* Kout = dev ? K : c.Kdev.p;
    double* exout = dev ? ex : (ex ? c.exdev.p : nullptr);
    build_general(c, variant, nocc, Csrc, Kout, exout, st, s1, s2, s3, ce1, ce3);
    prof_mark(c, 5, st);
    if (c.profiling && c.ev_used < kMaxProfiled) {
      if (variant == RPS_VARIANT_THC) { prof_mark(c, 1, st); prof_mark(c, 2, st); }
      if (variant == RPS_VARIANT_PS) { prof_mark(c, 3, st); prof_mark(c, 4, st); }
      ++c.ev_used;
    }
    if (!dev) {
      hip_check(hipMemcpyAsync(K, c.Kdev.p, (size_t)c.nbas * nocc * 8, hipMemcpyDeviceToHost, st), "copy K");
      if (ex) hip_check(hipMemcpyAsync(ex, c.exdev.p, 8, hipMemcpyDeviceToHost, st), "copy ex");
      hip_check(hipStreamSynchronize(st), "sync");
    }
    return;
  }
  double* Kout = dev ? K : c.Kdev.p;
  double* exout = dev ? ex : (ex ? c.exdev.p : nullptr);
  enqueue_fused(c, context_ws(c, np), variant, nocc, Csrc, Kout, exout, st, st3, true);
  if (!dev) {
    hip_check(hipMemcpyAsync(K, c.Kdev.p, (size_t)c.nbas * nocc * 8, hipMemcpyDeviceToHost, st), "copy K");
    if (ex) hip_check(hipMemcpyAsync(ex, c.exdev.p, 8, hipMemcpyDeviceToHost, st), "copy ex");
    hip_check(hipStreamSynchronize(st), "sync");
  }
}

// Replay of repeated builds as a captured graph: opt-in (RPS_GRAPH=1).  Measured on
// the 48^3 cell, eager launches queue back to back with less device idle time than a
// graph launch leaves between builds (130 us against 137 us per build).
bool graphs_enabled() {
  const char* g = getenv("RPS_GRAPH");
  return g && g[0] == '1';
}

// One exchange build.  With graph replay on, a device-pointer build repeated with
// the same arguments is captured into a HIP graph on its second call (the fit-fit
// kernel on a parallel branch when it is a separate kernel) and replayed from then
// on; host-pointer builds, profiled builds and builds inside a batch capture run
// eagerly.
void build_impl(rps_context& c, int variant, int32_t nocc, const double* C, double* K, double* ex,
                int32_t flags, hipStream_t st, bool allow_graph = true) {
  if (c.ng == 0) fail(RPS_ERR_STATE, "context has no completed set-up");
  if (nocc < 1) fail(RPS_ERR_ARG, "nocc must be >= 1");
  if (!C || !K) fail(RPS_ERR_ARG, "C and K must not be NULL");
  if (flags != RPS_PTRS_HOST && flags != RPS_PTRS_DEVICE) fail(RPS_ERR_ARG, "flags must be RPS_PTRS_HOST or RPS_PTRS_DEVICE");
  if (variant < RPS_VARIANT_RPS || variant > RPS_VARIANT_THC) fail(RPS_ERR_ARG, "unknown variant");
  const bool dev = (flags == RPS_PTRS_DEVICE);
  if (!(dev && allow_graph && !c.profiling && graphs_enabled())) {
    enqueue_build(c, variant, nocc, C, K, ex, dev, st, nullptr);
    return;
  }
  auto same = [&](const rps_context::GraphEntry& e) {
    return e.variant == variant && e.nocc == nocc && e.C == C && e.K == K && e.ex == ex;
  };
  for (auto& e : c.graphs)
    if (same(e)) {
      hip_check(hipGraphLaunch(e.exec, st), "hipGraphLaunch");
      c.last_stream = st;
      return;
    }
  if (!same(c.last_call)) {
    // first sight of these arguments: eager (also sizes every workspace)
    enqueue_build(c, variant, nocc, C, K, ex, dev, st, nullptr);
    c.last_call = rps_context::GraphEntry{variant, nocc, C, K, ex, nullptr, nullptr};
    return;
  }
  if (!c.gstream) {
    hip_check(hipStreamCreateWithFlags(&c.gstream, hipStreamNonBlocking), "hipStreamCreate");
    hip_check(hipStreamCreateWithFlags(&c.gbranch, hipStreamNonBlocking), "hipStreamCreate");
    hip_check(hipEventCreateWithFlags(&c.gfork, hipEventDisableTiming), "hipEventCreate");
    hip_check(hipEventCreateWithFlags(&c.gjoin, hipEventDisableTiming), "hipEventCreate");
  }
  // workspaces must exist before the capture (no allocation inside it)
  const int np = (int)round_up(nocc, 16);
  if (uses_general(c, np)) ensure_general(c, np); else ensure_workspace(c, np);
  rps_context::GraphEntry e{variant, nocc, C, K, ex, nullptr, nullptr};
  hip_check(hipStreamBeginCapture(c.gstream, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
  try {
    enqueue_build(c, variant, nocc, C, K, ex, dev, c.gstream, c.gbranch);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(c.gstream, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  hip_check(hipStreamEndCapture(c.gstream, &e.graph), "hipStreamEndCapture");
  hip_check(hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0), "hipGraphInstantiate");
  if (c.graphs.size() >= 4) {
    (void)hipGraphExecDestroy(c.graphs.front().exec);
    (void)hipGraphDestroy(c.graphs.front().graph);
    c.graphs.erase(c.graphs.begin());
  }
  c.graphs.push_back(e);
  hip_check(hipGraphLaunch(e.exec, st), "hipGraphLaunch");
  c.last_stream = st;
}

// Full exchange matrix with rPS integrals (Eq. 15 and its partner terms of
// Eq. 13): K = dV [Phi_g^T (A Phi) + (Phi_g^T (A Phi))^T - Phi_g^T (B Phi_g)],
// A = V o (U_g U^T), B = W o (U_g U_g^T).  Needed once at the end of an SCF
// run (Sec. 3.3), so it takes the simple route: A in g chunks by the GEMM with
// the Hadamard epilogue, then plain GEMMs; temporaries live for the call.
void build_full_impl(rps_context& c, int32_t nocc, const double* C, double* K, int32_t flags, hipStream_t st) {
  if (c.ng == 0) fail(RPS_ERR_STATE, "context has no completed set-up");
  if (nocc < 1) fail(RPS_ERR_ARG, "nocc must be >= 1");
  if (!C || !K) fail(RPS_ERR_ARG, "C and K must not be NULL");
  if (flags != RPS_PTRS_HOST && flags != RPS_PTRS_DEVICE) fail(RPS_ERR_ARG, "flags must be RPS_PTRS_HOST or RPS_PTRS_DEVICE");
  const bool dev = (flags == RPS_PTRS_DEVICE);
  const int64_t np = round_up(nocc, 16), Np = c.Np, G = c.nauxp, R = c.ngp;
  int64_t tmp = 0;
  DBuf<double> Cd, Cp, U, Ug, A, O, T, B, BP, K3, Kd, work;
  const double* Csrc = C;
  if (!dev) {
    Cd.alloc(c.nbas * nocc, &tmp);
    hip_check(hipMemcpyAsync(Cd.p, C, (size_t)c.nbas * nocc * 8, hipMemcpyHostToDevice, st), "copy C");
    Csrc = Cd.p;
  }
  const int64_t gc = std::min<int64_t>(G, std::max<int64_t>(64, (2000000000ll / 8) / R / 64 * 64));
  Cp.alloc(Np * np, &tmp);
  U.alloc(R * np, &tmp);
  Ug.alloc(G * np, &tmp);
  A.alloc(std::max(gc * R, G * G), &tmp);
  O.alloc(G * Np, &tmp);
  T.alloc(Np * Np, &tmp);
  B.alloc(G * G, &tmp);
  BP.alloc(G * Np, &tmp);
  K3.alloc(Np * Np, &tmp);
  work.alloc(kSplitWork, &tmp);
  if (!dev) Kd.alloc(c.nbas * c.nbas, &tmp);
  auto run = [&](Gemm g, const char* what, bool split) {
    if (split && g.epi == EPI_AXPBY) {
      g.splitk = gemm_splitk_for(g.M, g.N, g.K, kSplitWork);
      g.work = work.p;
    }
    hip_check(gemm_f64(g, st), what);
  };
  hip_check(pack_matrix(Csrc, c.nbas, nocc, nocc, Cp.p, Np, np, st), "pack C");
  {
    Gemm g;   // U = Phi C
    g.M = R; g.N = np; g.K = Np;
    g.A = c.Phi.p; g.lda = Np; g.B = Cp.p; g.ldb = np; g.C = U.p; g.ldc = np;
    run(g, "U", false);
  }
  hip_check(gather_rows(U.p, np, c.dpoints.p, c.naux, G, np, Ug.p, np, st), "U_g");
  for (int64_t g0 = 0; g0 < G; g0 += gc) {
    const int64_t m = std::min(gc, G - g0);
    Gemm a;   // A_c = V_c o (U_g[c] U^T)
    a.M = m; a.N = R; a.K = np;
    a.A = Ug.p + g0 * np; a.lda = np; a.B = U.p; a.ldb = np; a.transB = true;
    a.C = A.p; a.ldc = R; a.epi = EPI_HADAMARD_SRC; a.ldd = R;
    if (c.V.p) a.D = c.V.p + g0 * R;
    else a.D32 = c.V32.p + g0 * R;
    run(a, "A chunk", false);
    Gemm o;   // O[c] = A_c Phi
    o.M = m; o.N = Np; o.K = R;
    o.A = A.p; o.lda = R; o.B = c.Phi.p; o.ldb = Np; o.C = O.p + g0 * Np; o.ldc = Np;
    run(o, "A Phi", true);
  }
  {
    Gemm t;   // T = Phi_g^T O
    t.M = Np; t.N = Np; t.K = G;
    t.A = c.Phig.p; t.lda = Np; t.transA = true; t.B = O.p; t.ldb = Np; t.C = T.p; t.ldc = Np;
    run(t, "Phi_g^T (A Phi)", true);
    Gemm b;   // B = W o (U_g U_g^T)
    b.M = G; b.N = G; b.K = np;
    b.A = Ug.p; b.lda = np; b.B = Ug.p; b.ldb = np; b.transB = true;
    b.C = B.p; b.ldc = G; b.epi = EPI_HADAMARD_SRC; b.D = c.W.p; b.ldd = G;
    run(b, "B", false);
    Gemm bp;  // B Phi_g
    bp.M = G; bp.N = Np; bp.K = G;
    bp.A = B.p; bp.lda = G; bp.B = c.Phig.p; bp.ldb = Np; bp.C = BP.p; bp.ldc = Np;
    run(bp, "B Phi_g", true);
    Gemm k3;  // K3 = Phi_g^T (B Phi_g)
    k3.M = Np; k3.N = Np; k3.K = G;
    k3.A = c.Phig.p; k3.lda = Np; k3.transA = true; k3.B = BP.p; k3.ldb = Np; k3.C = K3.p; k3.ldc = Np;
    run(k3, "Phi_g^T (B Phi_g)", true);
  }
  double* Kout = dev ? K : Kd.p;
  hip_check(full_combine(T.p, K3.p, Np, c.nbas, c.dV, Kout, st), "combine");
  if (!dev) hip_check(hipMemcpyAsync(K, Kd.p, (size_t)c.nbas * c.nbas * 8, hipMemcpyDeviceToHost, st), "copy K");
  hip_check(hipStreamSynchronize(st), "sync");   // temporaries are released on return
}

// ------------------------------------------------------------------ Coulomb matrix
constexpr int64_t kCoulombChunk = 32ll << 20;   // doubles of U rows per chunk (256 MB)
constexpr int kCoulombParts = 256;              // blocks of the E_J dot product

// Split count of the J product over the grid: the smallest power of two giving at
// least two workgroups per compute unit over the lower output tiles, at least 128
// grid rows per split and partials within kSplitWork.
int coulomb_splits(const rps_context& c) {
  const int64_t bn = (c.Np <= 16) ? 16 : (c.Np <= 64) ? 64 : 128;   // output tile width of gemm_f64
  const int64_t tm = (c.Np + 127) / 128, tn = (c.Np + bn - 1) / bn;
  int64_t active = 0;
  for (int64_t i = 0; i < tm; ++i)
    for (int64_t j = 0; j < tn; ++j) active += (j * bn <= i * 128 + 127);
  int64_t z = 1;
  while (active * z < 512 && c.ngp / (z * 2) >= 128 && (z * 2) * c.Np * c.Np <= kSplitWork) z *= 2;
  return (int)z;
}

// Small-basis Coulomb path (one pass over Phi per step, U never stored): N <= 128, n <= 64.
bool coulomb_small_path(const rps_context& c, int np) {
  const char* e = getenv("RPS_COULOMB_GEMM");
  return c.Np <= 128 && np <= 64 && !(e && e[0] == '1');
}

void ensure_coulomb(rps_context& c, int np) {
  const bool small = coulomb_small_path(c, np);
  if (c.jws_np == np && c.jws_small == small) return;
  int64_t* cnt = &c.bytes;
  c.jchunk = std::min<int64_t>(c.ngp, std::max<int64_t>(64, kCoulombChunk / np / 64 * 64));
  c.jCp.alloc(c.Np * np, cnt);
  c.jCin.alloc(c.nbas * np, cnt);
  if (small) c.jU.release(cnt); else c.jU.alloc(c.jchunk * np, cnt);
  if (!c.jrho.p) c.jrho.alloc(3 * c.ngp, cnt);
  const int64_t nw = std::max<int64_t>({1, coulomb_splits(c), small ? coulomb_small_blocks(c.ngp) : 1});
  if (c.jwork.n < nw * c.Np * c.Np) c.jwork.alloc(nw * c.Np * c.Np, cnt);
  if (!c.jpart.p) c.jpart.alloc(kCoulombParts, cnt);
  c.jws_np = np;
  c.jws_small = small;
}

// J = dV Phi^T diag(Vc rho) Phi, rho(R) = sum_i U(R, i)^2, U = Phi C (Sec. 2.3, steps 1-4);
// ej = dV sum_R rho V_H.  All steps run on st in FP64.
// Lower triangles of the atom J blocks Phi_I^T diag(v) Phi_I, then J = dV sum over atoms
void sparse_j(rps_context& c, const double* vh, double* J, hipStream_t st) {
  if (!c.sQ.p) {
    c.sQ.alloc(std::max<int64_t>(c.qofs[c.natom], 1), &c.bytes);
    c.svv.alloc(c.ng, &c.bytes);
  }
  hip_check(gather_rows(vh, 1, c.sperm.p, c.ng, c.ng, 1, c.svv.p, 1, st), "V_H rows");
  Gemm g;
  g.A = c.sPhi.p; g.transA = true; g.B = c.sPhi.p; g.C = c.sQ.p;
  g.kscale = c.svv.p; g.lower_only = true;
  hip_check(gemm_f64_grouped(g, c.sitJ.p, (int)c.sitJ.n, c.smaxc, c.smaxc, st), "J blocks");
  hip_check(j_reduce(c.sQ.p, c.sqofs.p, c.sfofs.p, c.spos.p, c.smu_ofs.p, c.smu_atom.p, (int)c.nbas, c.dV, J, st),
            "J sums");
}

void build_coulomb_impl(rps_context& c, int32_t nocc, const double* C, double* J, double* ej, int32_t flags,
                        hipStream_t st) {
  if (c.ng == 0) fail(RPS_ERR_STATE, "context has no completed set-up");
  if (nocc < 1) fail(RPS_ERR_ARG, "nocc must be >= 1");
  if (!C || !J) fail(RPS_ERR_ARG, "C and J must not be NULL");
  if (flags != RPS_PTRS_HOST && flags != RPS_PTRS_DEVICE) fail(RPS_ERR_ARG, "flags must be RPS_PTRS_HOST or RPS_PTRS_DEVICE");
  if (!c.kern.p) fail(RPS_ERR_STATE, "context has no Coulomb kernel table");
  const bool dev = (flags == RPS_PTRS_DEVICE);
  const int np = (int)round_up(nocc, 16);
  const int64_t Np = c.Np, R = c.ngp, N = c.nbas;
  ensure_coulomb(c, np);
  const double* Csrc = C;
  if (!dev) {
    hip_check(hipMemcpyAsync(c.jCin.p, C, (size_t)N * nocc * 8, hipMemcpyHostToDevice, st), "copy C");
    Csrc = c.jCin.p;
    if (!c.jJ.p) c.jJ.alloc(N * N, &c.bytes);
  }
  const bool small = coulomb_small_path(c, np);
  if (small)   // step 1 in one pass: U = Phi C and rho = sum U^2 per 16-row subtile, U never stored
    hip_check(density_small(c.Phi.p, R, (int)Np, Csrc, (int)N, nocc, np, c.jrho.p, R, st), "density");
  else
    hip_check(pack_matrix(Csrc, N, nocc, nocc, c.jCp.p, Np, np, st), "pack C");
  if (!small && c.sparse) {
    // step 1 from the atom blocks of the screened basis: U in grid order, then rho
    if (c.sjws_np != np) {
      c.sUj.alloc(R * np, &c.bytes);
      c.sjws_np = np;
    }
    sparse_u(c, c.jCp.p, np, c.sUj.p, st);
    hip_check(density_rows(c.sUj.p, R, np, c.jrho.p, R, st), "density");
  }
  // step 1: density, one chunk of grid rows at a time (rows past N_g have Phi = 0, so rho = 0)
  for (int64_t r0 = 0; !small && !c.sparse && r0 < R; r0 += c.jchunk) {
    const int64_t m = std::min(c.jchunk, R - r0);
    Gemm g;   // U = Phi[r0:r0+m] C
    g.M = m; g.N = np; g.K = Np;
    g.A = c.Phi.p + r0 * Np; g.lda = Np; g.B = c.jCp.p; g.ldb = np; g.C = c.jU.p; g.ldc = np;
    hip_check(gemm_f64(g, st), "U chunk");
    hip_check(density_rows(c.jU.p, m, np, c.jrho.p + r0, R, st), "density");
  }
  // steps 2-3: V_H = Vc rho in place on the pair (rho, 0); row 2 keeps rho
  hip_check(poisson_rows(c.jrho.p, 2, R, c.mesh, c.kern.p, st), "poisson");
  double* exout = nullptr;
  if (ej) {
    exout = dev ? ej : c.jpart.p + (kCoulombParts - 1);
    hip_check(dot_scaled(c.jrho.p, c.jrho.p + 2 * R, R, c.dV, c.jpart.p, kCoulombParts - 1, exout, st), "E_J");
  }
  // step 4: lower tiles of Phi^T diag(V_H) Phi, split over the grid, mirrored and scaled by dV
  double* Jout = dev ? J : c.jJ.p;
  if (small) {
    hip_check(coulomb_small(c.Phi.p, R, (int)Np, c.jrho.p, c.jwork.p, st), "Phi^T diag(V_H) Phi");
    hip_check(sym_from_lower(c.jwork.p, coulomb_small_blocks(R), Np, N, c.dV, Jout, st), "J");
  } else if (c.sparse) {
    sparse_j(c, c.jrho.p, Jout, st);
  } else {
    Gemm g;
    g.M = Np; g.N = Np; g.K = R;
    g.A = c.Phi.p; g.lda = Np; g.transA = true; g.B = c.Phi.p; g.ldb = Np;
    g.kscale = c.jrho.p; g.lower_only = true;
    g.splitk = coulomb_splits(c);
    if (g.splitk > 1) {
      g.work = c.jwork.p;
      g.keep_partials = true;
    } else {
      g.C = c.jwork.p; g.ldc = Np;
    }
    hip_check(gemm_f64(g, st), "Phi^T diag(V_H) Phi");
    hip_check(sym_from_lower(c.jwork.p, g.splitk, Np, N, c.dV, Jout, st), "J");
  }
  if (!dev) {
    hip_check(hipMemcpyAsync(J, c.jJ.p, (size_t)N * N * 8, hipMemcpyDeviceToHost, st), "copy J");
    if (ej) hip_check(hipMemcpyAsync(ej, exout, 8, hipMemcpyDeviceToHost, st), "copy E_J");
    hip_check(hipStreamSynchronize(st), "sync");
  }
}

// ------------------------------------------------------------------ Madelung term
// K_occ += M S C and ex -= M tr(C^T S C) with S = dV Phi^T Phi (Sec. 4.5; for S-orthonormal C
// the energy shift is n_occ M = nM/2 with n = 2 n_occ electrons).
void madelung_impl(rps_context& c, int32_t nocc, const double* C, double* K, double* ex, int32_t flags,
                   hipStream_t st) {
  if (c.ng == 0) fail(RPS_ERR_STATE, "context has no completed set-up");
  if (nocc < 1) fail(RPS_ERR_ARG, "nocc must be >= 1");
  if (!C || !K) fail(RPS_ERR_ARG, "C and K must not be NULL");
  if (flags != RPS_PTRS_HOST && flags != RPS_PTRS_DEVICE) fail(RPS_ERR_ARG, "flags must be RPS_PTRS_HOST or RPS_PTRS_DEVICE");
  const bool dev = (flags == RPS_PTRS_DEVICE);
  const int64_t N = c.nbas, Np = c.Np, np = round_up(nocc, 16);
  int64_t* cnt = &c.bytes;
  if (!c.Sdev.p) {
    c.Sdev.alloc(Np * Np, cnt);
    const int z = coulomb_splits(c);
    int64_t tmp = 0;
    DBuf<double> work;
    Gemm g;
    g.M = Np; g.N = Np; g.K = c.ngp;
    g.A = c.Phi.p; g.lda = Np; g.transA = true; g.B = c.Phi.p; g.ldb = Np;
    g.C = c.Sdev.p; g.ldc = Np; g.alpha = c.dV;
    if (z > 1) {
      work.alloc(z * Np * Np, &tmp);
      g.splitk = z; g.work = work.p;
    }
    hip_check(gemm_f64(g, st), "overlap");
    hip_check(hipStreamSynchronize(st), "sync");
  }
  if (c.mCp.n < Np * np) {
    c.mCp.alloc(Np * np, cnt);
    c.mSC.alloc(Np * np, cnt);
  }
  if (!c.mpart.p) c.mpart.alloc(256, cnt);
  int64_t tmp = 0;
  DBuf<double> hC, hK, hE;
  const double* Cd = C;
  double* Kd = K;
  double* Ed = ex;
  if (!dev) {
    hC.alloc(N * nocc, &tmp);
    hK.alloc(N * nocc, &tmp);
    hip_check(hipMemcpyAsync(hC.p, C, (size_t)N * nocc * 8, hipMemcpyHostToDevice, st), "copy C");
    hip_check(hipMemcpyAsync(hK.p, K, (size_t)N * nocc * 8, hipMemcpyHostToDevice, st), "copy K");
    Cd = hC.p;
    Kd = hK.p;
    if (ex) {
      hE.alloc(1, &tmp);
      hip_check(hipMemcpyAsync(hE.p, ex, 8, hipMemcpyHostToDevice, st), "copy ex");
      Ed = hE.p;
    }
  }
  hip_check(pack_matrix(Cd, N, nocc, nocc, c.mCp.p, Np, np, st), "pack C");
  Gemm g;   // SC = S Cp
  g.M = Np; g.N = np; g.K = Np;
  g.A = c.Sdev.p; g.lda = Np; g.B = c.mCp.p; g.ldb = np; g.C = c.mSC.p; g.ldc = np;
  hip_check(gemm_f64(g, st), "S C");
  const int nparts = (int)std::min<int64_t>(256, std::max<int64_t>(1, (N * nocc + 4095) / 4096));
  hip_check(madelung_apply(c.mSC.p, np, Cd, N, nocc, c.madelung, Kd, Ed, c.mpart.p, nparts, st), "Madelung");
  if (!dev) {
    hip_check(hipMemcpyAsync(K, hK.p, (size_t)N * nocc * 8, hipMemcpyDeviceToHost, st), "copy K");
    if (ex) hip_check(hipMemcpyAsync(ex, hE.p, 8, hipMemcpyDeviceToHost, st), "copy ex");
    hip_check(hipStreamSynchronize(st), "sync");
  }
}

// ------------------------------------------------------------------ autotuner
// Mean time of `reps` device-pointer builds after one warm-up build (which
// also allocates any workspace the launch shape needs).
double time_builds(rps_context& c, int32_t nocc, const double* C, double* K, double* ex, hipStream_t st, int reps) {
  build_impl(c, RPS_VARIANT_RPS, nocc, C, K, ex, RPS_PTRS_DEVICE, st, false);
  hipEvent_t e0, e1;
  hip_check(hipEventCreate(&e0), "hipEventCreate");
  hip_check(hipEventCreate(&e1), "hipEventCreate");
  hip_check(hipEventRecord(e0, st), "hipEventRecord");
  for (int r = 0; r < reps; ++r) build_impl(c, RPS_VARIANT_RPS, nocc, C, K, ex, RPS_PTRS_DEVICE, st, false);
  hip_check(hipEventRecord(e1, st), "hipEventRecord");
  hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
  float ms = 0.f;
  hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms / reps;
}

// Try the launch parameters that matter for this context's path on its own
// inputs and keep the fastest: the streaming form's workgroup target (tail
// balance of the split passes) or the fused kernel's R tiles per workgroup
// and g blocks.  Results stay in the context and persist for later builds.
void autotune(rps_context& c, int32_t nocc, const double* C, double* K, double* ex, hipStream_t st) {
  const int np = (int)round_up(nocc, 16);
  struct Cand { int target, rtiles, gblocks; };
  std::vector<Cand> cands;
  const int saved_prof = c.profiling;
  c.profiling = 0;
  if (uses_general(c, np)) {
    for (int t : {256, 512, kStreamMaxTarget}) cands.push_back({t, 0, 0});
  } else {
    c.tune_rtiles = c.tune_gblocks = 0;
    FusedArgs a{};
    a.R_valid = c.ng;
    choose_shape(c, np, a);
    const int64_t rt = c.ngp / 64, gt = c.nauxp / 64;
    cands.push_back({0, a.rtiles, a.gblocks});
    if (a.rtiles > 1) cands.push_back({0, (a.rtiles + 1) / 2, a.gblocks});
    cands.push_back({0, a.rtiles * 2, a.gblocks});
    if (a.gblocks < gt) {
      const int gb = a.gblocks + 1;
      const int64_t target = std::max<int64_t>(1, 256 / gb);
      cands.push_back({0, (int)std::max<int64_t>(1, (rt + target - 1) / target), gb});
    }
  }
  double best = 1e300;
  Cand bc = cands[0];
  for (const Cand& k : cands) {
    c.tune_target = k.target;
    c.tune_rtiles = k.rtiles;
    c.tune_gblocks = k.gblocks;
    c.ws_np = -1;                 // re-derive the launch shape and its buffers
    const double ms = time_builds(c, nocc, C, K, ex, st, 3);
    if (ms < best) { best = ms; bc = k; }
  }
  c.tune_target = bc.target;
  c.tune_rtiles = bc.rtiles;
  c.tune_gblocks = bc.gblocks;
  c.tune_ms = best;
  c.ws_np = -1;
  build_impl(c, RPS_VARIANT_RPS, nocc, C, K, ex, RPS_PTRS_DEVICE, st, false);
  hip_check(hipStreamSynchronize(st), "sync");
  c.profiling = saved_prof;
}

// ------------------------------------------------------------------ no-allocation build (continued)
// Carve the workspace of plan p from base (256-byte aligned pieces); returns the
// doubles used (the caller checks them against the scratch size before use).
int64_t carve_fused_ws(const FusedPlan& p, double* base, FusedWs& w) {
  int64_t off = 0;
  auto take = [&](int64_t n) {
    double* q = base ? base + off : nullptr;
    off += (n + 31) / 32 * 32;
    return q;
  };
  w.plan = p;
  w.U = p.f32u ? nullptr : take(p.nU);      // the in-kernel-orbitals kernel forms U itself
  w.Ug = take(p.nUg);
  w.Ugp = p.m4 ? take(p.nUgp) : nullptr;
  w.M2p = take(p.nM2p);
  w.e3u = take(p.ne3u);
  w.K1p = take(p.nK1p);
  w.K3p = take(p.nK3p);
  w.e1p = take(p.ne1p);
  w.e3p = take(p.ne3p);
  w.M2 = take(p.nM2);
  w.K1 = take(p.nK1);
  w.K3 = take(p.nK3);
  w.epart = take(kEnergyBlocks);
  w.ecount = reinterpret_cast<unsigned*>(take(32));
  return off;
}

void build_noalloc_impl(rps_context& c, int32_t nocc, const double* C, double* K, double* ex, hipStream_t st) {
  if (c.ng == 0) fail(RPS_ERR_STATE, "context has no completed set-up");
  if (nocc < 1) fail(RPS_ERR_ARG, "nocc must be >= 1");
  if (!C || !K) fail(RPS_ERR_ARG, "C and K must not be NULL");
  const int np = (int)round_up(nocc, 16);
  if (uses_general(c, np))
    fail(RPS_ERR_SHAPE, "the no-allocation build covers the fused path only (N <= 128 with n_occ <= 64 in FP64 "
                        "or n_occ <= 16 in the precision forms)");
  FusedWs w;
  const FusedPlan p = fused_plan(c, np);
  const int64_t need = carve_fused_ws(p, nullptr, w);
  if (need * 8 > kNoAllocScratchBytes)
    fail(RPS_ERR_SHAPE, "the no-allocation build needs " + std::to_string(need * 8) + " bytes of scratch, " +
                            "above its static maximum of " + std::to_string(kNoAllocScratchBytes) + " bytes");
  double* base = scratch_device_ptr();
  carve_fused_ws(p, base, w);
  // the energy counter must start at zero (a fill kernel, no memset node if captured)
  hip_check(fill(reinterpret_cast<double*>(w.ecount), 32, 0.0, st), "clear counter");
  c.last_stream = st;
  enqueue_fused(c, w, RPS_VARIANT_RPS, nocc, C, K, ex, st, nullptr, false);
}

template <typename F>
rps_status guarded(F&& f) {
  try {
    f();
    g_err.clear();
    return RPS_OK;
  } catch (const Fail& e) {
    g_err = e.msg;
    return e.st;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return RPS_ERR_NOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return RPS_ERR_DEVICE;
  } catch (...) {
    g_err = "unknown failure";
    return RPS_ERR_DEVICE;
  }
}

}  // namespace

// A captured batch of exchange builds over many contexts (the batching form).
struct rps_batch {
  // Persistent pass launches: one per class (precision, padded n, orientation)
  // over the work items of every streaming-form cell of the batch.
  struct QClass {
    int prec = 0, np = 0, trans = 0, nitems = 0, nblocks = 0;
    DBuf<StreamArgs> args;
    DBuf<StreamItem> items;
  };
  std::vector<int> qcell;              // cell -> 1 if its passes run in the persistent launches
  std::vector<int> qsp_m2, qsp_l3;     // their split counts (M2 and fit-fit passes)
  std::vector<std::unique_ptr<DBuf<double>>> qpart3;   // their fit-fit partials
  std::vector<std::unique_ptr<QClass>> qclass;
  DBuf<double> qcount;                 // one queue counter per class (8-byte slots)
  hipStream_t pipe = nullptr;          // stream of the persistent launches during capture
  std::vector<hipEvent_t> qev;
  std::vector<rps_context*> ctx;
  std::vector<uint64_t> gen;           // workspace generation of each context at capture
  std::vector<int32_t> nocc;
  std::vector<const double*> C;
  std::vector<double*> K;
  double* ex = nullptr;
  int nbranch = 1;
  double tune_seconds = 0.0, capture_seconds = 0.0, replay_ms = 0.0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t origin = nullptr;        // capture stream (the legacy default stream cannot be captured)
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  void release_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
  ~rps_batch() {
    release_graph();
    for (auto e : events) (void)hipEventDestroy(e);
    for (auto e : qev) (void)hipEventDestroy(e);
    for (auto st : streams) (void)hipStreamDestroy(st);
    if (pipe) (void)hipStreamDestroy(pipe);
    if (origin) (void)hipStreamDestroy(origin);
  }
};

namespace {

// Work items of the persistent pass launches.  A cell takes part when its build is
// the streaming form (general path, padded n <= 128): its M2 and M1^T passes (the
// context's precision) and its fit-fit pass (FP64) become items (cell, x block,
// y split) of the class (precision, n, orientation); items are ordered by the
// length of their y split, longest first.  Everything else (fused-path cells,
// the GEMM form) is built by its own launches beside them.
void plan_queue(rps_batch& b) {
  const int nb = (int)b.ctx.size();
  b.qcell.assign(nb, 0);
  b.qsp_m2.assign(nb, 0);
  b.qsp_l3.assign(nb, 0);
  b.qpart3.clear();
  b.qpart3.resize(nb);
  b.qclass.clear();
  // Off unless RPS_BATCH_QUEUE=1: the first GPU run of this form ended in a host
  // segmentation fault inside rps_batch_create whose cause is not found (the host
  // logic runs clean under AddressSanitizer on a CPU stand-in for the runtime), so
  // every cell keeps its own launches by default.
  const char* qe = getenv("RPS_BATCH_QUEUE");
  if (!(qe && qe[0] == '1')) return;
  std::vector<std::vector<std::pair<StreamArgs, int>>> cls_args;   // per class: (args, nsplit)
  std::vector<std::array<int, 3>> keys;
  auto class_of = [&](int prec, int np, int trans) {
    for (size_t k = 0; k < keys.size(); ++k)
      if (keys[k][0] == prec && keys[k][1] == np && keys[k][2] == trans) return (int)k;
    keys.push_back({prec, np, trans});
    cls_args.emplace_back();
    return (int)keys.size() - 1;
  };
  for (int i = 0; i < nb; ++i) {
    rps_context& c = *b.ctx[i];
    const int np = (int)round_up(b.nocc[i], 16);
    if (!uses_general(c, np) || np > kStreamMaxNp || !c.gSp.p || c.gws_np != np) continue;
    b.qcell[i] = 1;
    const StreamArgs m2 = pass_m2(c, np), m1 = pass_m1(c, np);
    b.qsp_m2[i] = pass_splits(c, m2);
    b.qpart3[i] = std::make_unique<DBuf<double>>();
    const StreamArgs l3 = pass_l3(c, np, nullptr);
    b.qsp_l3[i] = pass_splits(c, l3);
    b.qpart3[i]->alloc((int64_t)b.qsp_l3[i] * c.nauxp * np, nullptr);
    const StreamArgs l3p = pass_l3(c, np, b.qpart3[i]->p);
    cls_args[class_of(c.precision, np, 0)].push_back({m2, b.qsp_m2[i]});
    cls_args[class_of(c.precision, np, 1)].push_back({m1, 1});
    cls_args[class_of(RPS_PREC_FP64, np, 0)].push_back({l3p, b.qsp_l3[i]});
  }
  b.qcount.alloc(std::max<int64_t>((int64_t)keys.size(), 1), nullptr);
  for (size_t k = 0; k < keys.size(); ++k) {
    auto q = std::make_unique<rps_batch::QClass>();
    q->prec = keys[k][0];
    q->np = keys[k][1];
    q->trans = keys[k][2];
    std::vector<StreamArgs> args;
    std::vector<StreamItem> items;
    std::vector<int64_t> len;
    for (auto& pa : cls_args[k]) {
      StreamArgs a;
      hip_check(stream_prepare(pa.first, q->prec, pa.second, a), "queue pass");
      const int cell = (int)args.size();
      args.push_back(a);
      const int64_t xb = stream_xblocks(a.nx);
      // every (x block, split) is an item, empty splits too: they write the zero
      // partials the ordered sums expect, as in the one-cell launch
      for (int64_t by = 0; by < pa.second; ++by) {
        const int64_t ys = by * a.ysplit, ye = std::min(ys + a.ysplit, a.ny);
        for (int64_t bx = 0; bx < xb; ++bx) {
          items.push_back(StreamItem{cell, (int32_t)bx, (int32_t)by});
          len.push_back(std::max<int64_t>(ye - ys, 0));
        }
      }
    }
    std::vector<size_t> order(items.size());
    for (size_t t = 0; t < order.size(); ++t) order[t] = t;
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return len[x] > len[y]; });
    std::vector<StreamItem> sorted(items.size());
    for (size_t t = 0; t < order.size(); ++t) sorted[t] = items[order[t]];
    q->nitems = (int)sorted.size();
    q->nblocks = std::max(1, std::min(q->nitems, stream_queue_blocks(q->prec, q->np, q->trans)));
    q->args.alloc((int64_t)args.size(), nullptr);
    q->items.alloc(std::max<int64_t>(q->nitems, 1), nullptr);
    hip_check(hipMemcpy(q->args.p, args.data(), args.size() * sizeof(StreamArgs), hipMemcpyHostToDevice), "queue args");
    if (q->nitems > 0)
      hip_check(hipMemcpy(q->items.p, sorted.data(), sorted.size() * sizeof(StreamItem), hipMemcpyHostToDevice),
                "queue items");
    b.qclass.push_back(std::move(q));
  }
}

// Capture every build of the batch into one graph.  Cells are ordered by
// their work (n N_aux N_g, largest first) and dealt to `nbranch` parallel
// branches by least accumulated work, so small cells fill the device beside
// the large ones; the branches fork from and join back into `origin`.
// Streaming-form cells (plan_queue) run in three phases: their orbitals on the
// branches, then the persistent pass launches (one per class, on the pipe
// stream, each preceded by a fill kernel that zeroes its queue counter), then
// their sums, K1, K3 and the combine back on the branches; every other cell's
// build runs on its branch in between, beside the persistent launches.
void capture_batch(rps_batch& b, int nbranch, hipStream_t origin) {
  b.release_graph();
  const int nb = (int)b.ctx.size();
  while ((int)b.streams.size() < nbranch) {
    hipStream_t st;
    hip_check(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate");
    b.streams.push_back(st);
  }
  while ((int)b.events.size() < nbranch + 1) {
    hipEvent_t e;
    hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
    b.events.push_back(e);
  }
  while ((int)b.qev.size() < nbranch + 1) {
    hipEvent_t e;
    hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
    b.qev.push_back(e);
  }
  if (!b.pipe) hip_check(hipStreamCreateWithFlags(&b.pipe, hipStreamNonBlocking), "hipStreamCreate");
  std::vector<int> order(nb);
  for (int i = 0; i < nb; ++i) order[i] = i;
  auto work = [&](int i) {
    return (double)b.nocc[i] * (double)b.ctx[i]->naux * (double)b.ctx[i]->ng;
  };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work(x) > work(y); });
  std::vector<double> load(nbranch, 0.0);
  std::vector<int> assign(nb, 0);
  for (int i : order) {
    int br = 0;
    for (int k = 1; k < nbranch; ++k)
      if (load[k] < load[br]) br = k;
    assign[i] = br;
    load[br] += work(i);
  }
  std::vector<int> prof(nb);
  for (int i = 0; i < nb; ++i) { prof[i] = b.ctx[i]->profiling; b.ctx[i]->profiling = 0; }
  auto t0 = std::chrono::steady_clock::now();
  hip_check(hipStreamBeginCapture(origin, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
  try {
    hip_check(hipEventRecord(b.events[nbranch], origin), "fork");
    for (int k = 0; k < nbranch; ++k) hip_check(hipStreamWaitEvent(b.streams[k], b.events[nbranch], 0), "fork wait");
    const bool queue = !b.qclass.empty();
    if (queue) {
      // phase 1: orbitals of the streaming-form cells
      for (int i : order)
        if (b.qcell[i])
          general_pre(*b.ctx[i], b.nocc[i], b.C[i], b.streams[assign[i]], b.ctx[i]->precision != RPS_PREC_FP64);
      hip_check(hipStreamWaitEvent(b.pipe, b.events[nbranch], 0), "fork wait");
      for (int k = 0; k < nbranch; ++k) {
        hip_check(hipEventRecord(b.qev[k], b.streams[k]), "phase 1");
        hip_check(hipStreamWaitEvent(b.pipe, b.qev[k], 0), "phase 1 wait");
      }
      // phase 2: the persistent pass launches
      for (size_t k = 0; k < b.qclass.size(); ++k) {
        const rps_batch::QClass& q = *b.qclass[k];
        hip_check(fill(b.qcount.p + k, 1, 0.0, b.pipe), "clear queue counter");
        hip_check(stream_product_queue(q.args.p, q.items.p, q.nitems, q.prec, q.np, q.trans,
                                       reinterpret_cast<unsigned*>(b.qcount.p + k), q.nblocks, b.pipe),
                  "persistent passes");
      }
      hip_check(hipEventRecord(b.qev[nbranch], b.pipe), "phase 2");
    }
    // every other cell: its whole build, beside phase 2
    for (int i : order)
      if (!queue || !b.qcell[i])
        build_impl(*b.ctx[i], RPS_VARIANT_RPS, b.nocc[i], b.C[i], b.K[i], b.ex ? b.ex + i : nullptr, RPS_PTRS_DEVICE,
                   b.streams[assign[i]], false);
    if (queue) {
      // phase 3: sums, K1, K3 and the combine of the streaming-form cells
      for (int k = 0; k < nbranch; ++k) hip_check(hipStreamWaitEvent(b.streams[k], b.qev[nbranch], 0), "phase 2 wait");
      for (int i : order)
        if (b.qcell[i])
          general_post(*b.ctx[i], b.nocc[i], b.qsp_m2[i], b.qpart3[i]->p, b.qsp_l3[i], b.K[i],
                       b.ex ? b.ex + i : nullptr, b.streams[assign[i]]);
    }
    for (int k = 0; k < nbranch; ++k) {
      hip_check(hipEventRecord(b.events[k], b.streams[k]), "join");
      hip_check(hipStreamWaitEvent(origin, b.events[k], 0), "join wait");
    }
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(origin, &g);
    if (g) (void)hipGraphDestroy(g);
    for (int i = 0; i < nb; ++i) b.ctx[i]->profiling = prof[i];
    throw;
  }
  hip_check(hipStreamEndCapture(origin, &b.graph), "hipStreamEndCapture");
  hip_check(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0), "hipGraphInstantiate");
  b.gen.resize(nb);
  for (int i = 0; i < nb; ++i) b.gen[i] = b.ctx[i]->ws_gen;
  b.capture_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  b.nbranch = nbranch;
  for (int i = 0; i < nb; ++i) b.ctx[i]->profiling = prof[i];
}

double time_replays(rps_batch& b, hipStream_t st, int reps) {
  hip_check(hipGraphLaunch(b.exec, st), "hipGraphLaunch");
  hipEvent_t e0, e1;
  hip_check(hipEventCreate(&e0), "hipEventCreate");
  hip_check(hipEventCreate(&e1), "hipEventCreate");
  hip_check(hipEventRecord(e0, st), "hipEventRecord");
  for (int r = 0; r < reps; ++r) hip_check(hipGraphLaunch(b.exec, st), "hipGraphLaunch");
  hip_check(hipEventRecord(e1, st), "hipEventRecord");
  hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
  float ms = 0.f;
  hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms / reps;
}

}  // namespace

extern "C" {

int32_t rps_abi_version(void) { return 1; }

const char* rps_last_error(void) { return g_err.c_str(); }

rps_status rps_setup_isdf_screened(const rps_cell* cell, const rps_basis* basis, int64_t n_aux, uint64_t seed,
                                   int32_t select_mode, int32_t precision, const int64_t* points_in,
                                   double basis_eps, void* hip_stream, rps_context** out) {
  return guarded([&] {
    if (!out) fail(RPS_ERR_ARG, "out must not be NULL");
    rps_context* c = new rps_context();
    try {
      setup_impl(*c, cell, basis, n_aux, seed, select_mode, precision, points_in, basis_eps,
                 (hipStream_t)hip_stream);
    } catch (...) {
      delete c;
      throw;
    }
    *out = c;
  });
}

rps_status rps_setup_isdf_from_potentials(const rps_cell* cell, const rps_basis* basis, int64_t n_aux,
                                          const int64_t* points, int32_t precision, const void* V, int64_t ldv,
                                          const double* W, int64_t ldw, int32_t flags, void* hip_stream,
                                          rps_context** out) {
  return guarded([&] {
    if (!out) fail(RPS_ERR_ARG, "out must not be NULL");
    if (flags != RPS_PTRS_HOST && flags != RPS_PTRS_DEVICE) fail(RPS_ERR_ARG, "flags must be RPS_PTRS_HOST or RPS_PTRS_DEVICE");
    GivenFit gf;
    gf.V = V; gf.ldv = ldv; gf.W = W; gf.ldw = ldw; gf.device = (flags == RPS_PTRS_DEVICE);
    rps_context* c = new rps_context();
    try {
      setup_impl(*c, cell, basis, n_aux, 0, RPS_SELECT_VORONOI, precision, points, 0.0, (hipStream_t)hip_stream, &gf);
    } catch (...) {
      delete c;
      throw;
    }
    *out = c;
  });
}

rps_status rps_setup_isdf(const rps_cell* cell, const rps_basis* basis, int64_t n_aux, uint64_t seed,
                          int32_t select_mode, int32_t precision, const int64_t* points_in, void* hip_stream,
                          rps_context** out) {
  return rps_setup_isdf_screened(cell, basis, n_aux, seed, select_mode, precision, points_in, 0.0, hip_stream,
                                 out);
}

rps_status rps_build_exchange_occRI(rps_context* ctx, int32_t nocc, const double* C, double* K, double* ex,
                                    int32_t flags, void* hip_stream) {
  return guarded([&] {
    if (!ctx) fail(RPS_ERR_ARG, "ctx must not be NULL");
    build_impl(*ctx, RPS_VARIANT_RPS, nocc, C, K, ex, flags, (hipStream_t)hip_stream);
  });
}

rps_status rps_build_exchange_occRI_noalloc(rps_context* ctx, int32_t nocc, const double* C, double* K,
                                            double* ex, void* hip_stream) {
  return guarded([&] {
    if (!ctx) fail(RPS_ERR_ARG, "ctx must not be NULL");
    build_noalloc_impl(*ctx, nocc, C, K, ex, (hipStream_t)hip_stream);
  });
}

rps_status rps_build_exchange_variant(rps_context* ctx, int32_t variant, int32_t nocc, const double* C, double* K,
                                      double* ex, int32_t flags, void* hip_stream) {
  return guarded([&] {
    if (!ctx) fail(RPS_ERR_ARG, "ctx must not be NULL");
    build_impl(*ctx, variant, nocc, C, K, ex, flags, (hipStream_t)hip_stream);
  });
}

rps_status rps_build_exchange_full(rps_context* ctx, int32_t nocc, const double* C, double* K, int32_t flags,
                                   void* hip_stream) {
  return guarded([&] {
    if (!ctx) fail(RPS_ERR_ARG, "ctx must not be NULL");
    build_full_impl(*ctx, nocc, C, K, flags, (hipStream_t)hip_stream);
  });
}

rps_status rps_build_coulomb(rps_context* ctx, int32_t nocc, const double* C, double* J, double* ej, int32_t flags,
                             void* hip_stream) {
  return guarded([&] {
    if (!ctx) fail(RPS_ERR_ARG, "ctx must not be NULL");
    build_coulomb_impl(*ctx, nocc, C, J, ej, flags, (hipStream_t)hip_stream);
  });
}

rps_status rps_madelung_constant(const double lattice[9], double* M) {
  return guarded([&] {
    if (!lattice || !M) fail(RPS_ERR_ARG, "NULL argument");
    if (!(std::fabs(det3(lattice)) > 0.0)) fail(RPS_ERR_ARG, "lattice vectors are degenerate");
    *M = madelung_constant(lattice);
  });
}

rps_status rps_madelung_correct(rps_context* ctx, int32_t nocc, const double* C, double* K, double* ex, int32_t flags,
                                void* hip_stream) {
  return guarded([&] {
    if (!ctx) fail(RPS_ERR_ARG, "ctx must not be NULL");
    madelung_impl(*ctx, nocc, C, K, ex, flags, (hipStream_t)hip_stream);
  });
}

rps_status rps_build_exchange_occRI_batched(rps_context* const* ctx, int32_t nbatch, const int32_t* nocc,
                                            const double* const* C, double* const* K, double* ex, int32_t flags,
                                            void* hip_stream) {
  return guarded([&] {
    if (!ctx || !nocc || !C || !K || nbatch < 0) fail(RPS_ERR_ARG, "NULL argument or negative nbatch");
    for (int32_t b = 0; b < nbatch; ++b) {
      if (!ctx[b]) fail(RPS_ERR_ARG, "NULL context in batch");
      build_impl(*ctx[b], RPS_VARIANT_RPS, nocc[b], C[b], K[b], ex ? ex + b : nullptr, flags,
                 (hipStream_t)hip_stream);
    }
  });
}

rps_status rps_autotune(rps_context* ctx, int32_t nocc, const double* C, double* K, double* ex, void* hip_stream,
                        double* best_ms) {
  return guarded([&] {
    if (!ctx || !C || !K) fail(RPS_ERR_ARG, "NULL argument");
    if (nocc < 1) fail(RPS_ERR_ARG, "nocc must be >= 1");
    autotune(*ctx, nocc, C, K, ex, (hipStream_t)hip_stream);
    if (best_ms) *best_ms = ctx->tune_ms;
  });
}

rps_status rps_batch_create(rps_context* const* ctx, int32_t nbatch, const int32_t* nocc, const double* const* C,
                            double* const* K, double* ex, int32_t flags, void* hip_stream, rps_batch** out) {
  return guarded([&] {
    if (!out) fail(RPS_ERR_ARG, "out must not be NULL");
    *out = nullptr;
    if (!ctx || !nocc || !C || !K || nbatch < 1) fail(RPS_ERR_ARG, "NULL argument or nbatch < 1");
    if (flags & ~(RPS_BATCH_AUTOTUNE | RPS_BATCH_FIXED_BRANCHES_MASK)) fail(RPS_ERR_ARG, "unknown flags");
    for (int32_t i = 0; i < nbatch; ++i) {
      if (!ctx[i] || !C[i] || !K[i]) fail(RPS_ERR_ARG, "NULL context or buffer in batch");
      if (ctx[i]->ng == 0) fail(RPS_ERR_STATE, "context without a completed set-up in batch");
      if (nocc[i] < 1) fail(RPS_ERR_ARG, "nocc must be >= 1");
      for (int32_t j = 0; j < i; ++j)
        if (ctx[j] == ctx[i]) fail(RPS_ERR_ARG, "a context appears twice in the batch (builds would share workspace)");
    }
    hipStream_t st = (hipStream_t)hip_stream;
    auto b = std::make_unique<rps_batch>();
    b->ctx.assign(ctx, ctx + nbatch);
    b->nocc.assign(nocc, nocc + nbatch);
    b->C.assign(C, C + nbatch);
    b->K.assign(K, K + nbatch);
    b->ex = ex;
    auto t0 = std::chrono::steady_clock::now();
    for (int32_t i = 0; i < nbatch; ++i) {
      if (flags & RPS_BATCH_AUTOTUNE)
        autotune(*ctx[i], nocc[i], C[i], K[i], ex ? ex + i : nullptr, st);
      else   // one eager build: allocates every workspace before capture
        build_impl(*ctx[i], RPS_VARIANT_RPS, nocc[i], C[i], K[i], ex ? ex + i : nullptr, RPS_PTRS_DEVICE, st, false);
    }
    hip_check(hipStreamSynchronize(st), "sync");
    plan_queue(*b);
    hip_check(hipStreamCreateWithFlags(&b->origin, hipStreamNonBlocking), "hipStreamCreate");
    hipStream_t org = b->origin;
    const int fixed = (flags & RPS_BATCH_FIXED_BRANCHES_MASK) >> 8;
    if (fixed > 0) {
      capture_batch(*b, fixed, org);
      b->replay_ms = time_replays(*b, org, 2);
    } else {
      // branch count: the fastest replay of 1, 2 and 4 parallel branches
      double best = 1e300;
      int bestk = 1;
      for (int k : {1, 2, 4}) {
        if (k > 1 && k > nbatch) break;
        capture_batch(*b, k, org);
        const double ms = time_replays(*b, org, 2);
        if (ms < best) { best = ms; bestk = k; }
      }
      if (b->nbranch != bestk) capture_batch(*b, bestk, org);
      b->replay_ms = best;
    }
    hip_check(hipStreamSynchronize(org), "sync");
    b->tune_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = b.release();
  });
}

rps_status rps_batch_run(rps_batch* b, void* hip_stream) {
  return guarded([&] {
    if (!b || !b->exec) fail(RPS_ERR_ARG, "NULL or empty batch");
    // the graph holds the workspace addresses of its contexts as they were at capture
    for (size_t i = 0; i < b->ctx.size(); ++i)
      if (b->ctx[i]->ws_gen != b->gen[i])
        fail(RPS_ERR_STATE, "the workspace of context " + std::to_string(i) +
                                " changed after the batch was captured (autotune, or a build with another "
                                "number of occupied orbitals); destroy and recreate the batch");
    hip_check(hipGraphLaunch(b->exec, (hipStream_t)hip_stream), "hipGraphLaunch");
  });
}

rps_status rps_batch_info(const rps_batch* b, int32_t* nbranch, double* seconds) {
  return guarded([&] {
    if (!b) fail(RPS_ERR_ARG, "NULL batch");
    if (nbranch) *nbranch = b->nbranch;
    if (seconds) {
      seconds[0] = b->tune_seconds;
      seconds[1] = b->capture_seconds;
      seconds[2] = b->replay_ms * 1e-3;
    }
  });
}

void rps_batch_destroy(rps_batch* b) { delete b; }

rps_status rps_exchange_energy(int32_t nbas, int32_t nocc, const double* C, const double* K, double* ex) {
  return guarded([&] {
    if (nbas < 1 || nocc < 1) fail(RPS_ERR_ARG, "nbas and nocc must be >= 1");
    if (!C || !K || !ex) fail(RPS_ERR_ARG, "NULL argument");
    double s = 0.0;
    for (int64_t i = 0; i < (int64_t)nbas * nocc; ++i) s += C[i] * K[i];
    *ex = -s;
  });
}

rps_status rps_overlap(rps_context* ctx, double* S) {
  return guarded([&] {
    if (!ctx || !S) fail(RPS_ERR_ARG, "NULL argument");
    rps_context& c = *ctx;
    if (c.ng == 0) fail(RPS_ERR_STATE, "context has no completed set-up");
    int64_t tmpb = 0;
    DBuf<double> dS;
    dS.alloc(c.Np * c.Np, &tmpb);
    Gemm g;
    g.M = c.Np; g.N = c.Np; g.K = c.ngp;
    g.A = c.Phi.p; g.lda = c.Np; g.transA = true; g.B = c.Phi.p; g.ldb = c.Np;
    g.C = dS.p; g.ldc = c.Np; g.alpha = c.dV;
    hip_check(gemm_f64(g, nullptr), "overlap");
    std::vector<double> h(c.Np * c.Np);
    hip_check(hipMemcpy(h.data(), dS.p, h.size() * 8, hipMemcpyDeviceToHost), "copy S");
    dS.release(nullptr);
    for (int64_t i = 0; i < c.nbas; ++i)
      for (int64_t j = 0; j < c.nbas; ++j) S[i * c.nbas + j] = h[i * c.Np + j];
  });
}

rps_status rps_get_points(const rps_context* ctx, int64_t* out) {
  return guarded([&] {
    if (!ctx || !out) fail(RPS_ERR_ARG, "NULL argument");
    if (ctx->ng == 0) fail(RPS_ERR_STATE, "context has no completed set-up");
    std::copy(ctx->points.begin(), ctx->points.end(), out);
  });
}

rps_status rps_get_info(const rps_context* ctx, rps_info* info) {
  return guarded([&] {
    if (!ctx || !info) fail(RPS_ERR_ARG, "NULL argument");
    const rps_context& c = *ctx;
    info->ngrid = c.ng; info->nbas = c.nbas; info->naux = c.naux;
    info->ngrid_pad = c.ngp; info->nbas_pad = c.Np; info->naux_pad = c.nauxp;
    info->n_candidates = c.ncand; info->dvol = c.dV; info->chol_shift = c.shift;
    info->setup_seconds = c.setup_seconds; info->device_bytes = c.bytes;
    info->precision = c.precision; info->exact = c.exact; info->madelung = c.madelung;
    info->basis_fill = c.sparse ? (double)c.pofs[c.natom] / ((double)c.ng * (double)c.nbas) : 1.0;
    double pair = 0.0;
    for (int I = 0; c.sparse && I < c.natom; ++I) {
      const double nc = (double)(c.fofs[I + 1] - c.fofs[I]);
      pair += (double)(c.vofs[I + 1] - c.vofs[I]) * nc * nc;
    }
    info->basis_pair_fill = c.sparse ? pair / ((double)c.ng * (double)c.nbas * (double)c.nbas) : 1.0;
    info->build_arith = c.last_arith;
  });
}

rps_status rps_get_array(const rps_context* ctx, int32_t which, int64_t row0, int64_t nrows, double* out) {
  return guarded([&] {
    if (!ctx || !out) fail(RPS_ERR_ARG, "NULL argument");
    const rps_context& c = *ctx;
    if (c.ng == 0) fail(RPS_ERR_STATE, "context has no completed set-up");
    int64_t rows = 0, cols = 0, ld = 0;
    const double* src = nullptr;
    if (which == 0) { rows = c.ng; cols = c.nbas; ld = c.Np; src = c.Phi.p; }
    else if (which == 1) {
      if (!c.V.p) fail(RPS_ERR_STATE, "this context keeps V in FP32 only (precision form)");
      rows = c.naux; cols = c.ng; ld = c.ngp; src = c.V.p;
    }
    else if (which == 2) { rows = c.naux; cols = c.naux; ld = c.nauxp; src = c.W.p; }
    else if (which == 3) {
      if (c.owner_host.empty()) fail(RPS_ERR_STATE, "no Voronoi assignment was computed (points were given)");
      if (row0 < 0 || nrows < 0 || row0 + nrows > c.ng) fail(RPS_ERR_SHAPE, "row range out of bounds");
      for (int64_t i = 0; i < nrows; ++i) out[i] = (double)c.owner_host[row0 + i];
      return;
    } else {
      fail(RPS_ERR_ARG, "which must be 0..3");
    }
    if (row0 < 0 || nrows < 0 || row0 + nrows > rows) fail(RPS_ERR_SHAPE, "row range out of bounds");
    hip_check(hipMemcpy2D(out, cols * 8, src + row0 * ld, ld * 8, cols * 8, nrows, hipMemcpyDeviceToHost),
              "copy array");
  });
}

rps_status rps_set_profiling(rps_context* ctx, int32_t enable) {
  return guarded([&] {
    if (!ctx) fail(RPS_ERR_ARG, "ctx must not be NULL");
    ctx->profiling = enable ? 1 : 0;
    ctx->ev_used = 0;
  });
}

rps_status rps_get_profile(rps_context* ctx, double* out) {
  return guarded([&] {
    if (!ctx || !out) fail(RPS_ERR_ARG, "NULL argument");
    rps_context& c = *ctx;
    double tot[3] = {0.0, 0.0, 0.0};
    if (c.ev_used > 0) {
      hip_check(hipStreamSynchronize(c.last_stream), "sync");
      for (int64_t b = 0; b < c.ev_used; ++b) {
        hipEvent_t* e = &c.ev_pool[b * kEvPerBuild];
        float ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, e[1], e[2]), "elapsed");
        tot[0] += ms;
        hip_check(hipEventElapsedTime(&ms, e[3], e[4]), "elapsed");
        tot[1] += ms;
        hip_check(hipEventElapsedTime(&ms, e[0], e[5]), "elapsed");
        tot[2] += ms;
      }
    }
    out[0] = (double)c.ev_used;
    out[1] = tot[0];
    out[2] = tot[1];
    out[3] = tot[2];
    c.ev_used = 0;
  });
}

void rps_destroy(rps_context* ctx) {
  if (!ctx) return;
  (void)hipDeviceSynchronize();
  delete ctx;
}

}  // extern "C"
