"""Pins of the FP64 oracle against facts that do not come from the oracle itself:
published test vectors, closed forms, brute-force sums without FFTs, exact
algebraic identities of the rPS derivation (Sec. 3.2), special cases and
invariants.  All CPU; no GPU code is involved."""
import dataclasses
import math
import os

import numpy as np
import pytest

import rps_inputs as ri
from oracle import basis, brute, conventional, coulomb, grid, isdf, madelung, rng, rps

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- generator
def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = rng.philox4x32_10(*v[:6])
        assert [int(o) for o in out] == v[6:]


def test_sketch_normal_statistics():
    z = rng.sketch_normal(400, 50, seed=12345, stream=3)
    assert abs(z.mean()) < 0.02 and abs(z.std() - 1.0) < 0.02
    z2 = rng.sketch_normal(400, 50, seed=12345, stream=4)
    assert abs(np.corrcoef(z.ravel(), z2.ravel())[0, 1]) < 0.02


# ---------------------------------------------------------------- Coulomb on the grid
@pytest.mark.parametrize("skew", [False, True])
@pytest.mark.parametrize("mesh", [(6, 6, 6), (5, 6, 7)])
def test_poisson_equals_direct_g_sum(skew, mesh):
    """FFT Poisson solve == dense matrix from explicit cos(G.(R-R')) sums."""
    lat = np.eye(3) * 5.0
    if skew:
        lat = np.array([[5.0, 0.0, 0.0], [1.3, 4.6, 0.0], [0.4, -0.9, 5.5]])
    Vd = brute.dense_coulomb(lat, mesh)
    f = np.random.default_rng(1).standard_normal((3, int(np.prod(mesh))))
    got = grid.poisson(f, lat, mesh)
    np.testing.assert_allclose(got, f @ Vd.T, rtol=0, atol=1e-12 * np.abs(got).max())
    # symmetric positive semi-definite, null vector = constant (G = 0 removed)
    np.testing.assert_allclose(Vd, Vd.T, atol=1e-12)
    ev = np.linalg.eigvalsh(Vd)
    assert ev.min() > -1e-10
    assert abs(np.ones(Vd.shape[0]) @ Vd @ np.ones(Vd.shape[0])) < 1e-9


@pytest.mark.parametrize("a,b", [(0.8, 1.1), (0.5, 0.5)])
def test_grid_coulomb_matches_analytic_lattice_sum(a, b):
    """dV sum rho_A Vc rho_B for periodized s Gaussians == the reciprocal
    lattice sum of their analytic transforms (Eq. 4), G = 0 removed.  Pins dV,
    1/Omega, 4 pi / G^2, the G = 0 rule, the FFT convention and the s
    normalisation together."""
    L = 7.0
    lat = np.eye(3) * L
    mesh = (40, 40, 40)
    A = np.array([1.0, 2.0, 3.0])
    B = np.array([4.5, 0.7, 5.9])
    w = ri.Workload("t", lat, np.array(mesh), np.stack([A, B]), np.array([0, 1]),
                    np.array([0, 0]), np.array([a, b]), 1, 1, 0)
    Phi = basis.eval_basis(w)
    dV = grid.dvol(lat, mesh)
    got = dV * Phi[:, 0] @ grid.poisson(Phi[:, 1], lat, mesh)
    ref = brute.analytic_s_coulomb(lat, A, a, B, b)
    assert abs(got - ref) < 1e-11 * max(1.0, abs(ref))


# ---------------------------------------------------------------- basis functions
def _one_shell_workload(l, a, L=10.0, mesh=64, center=(3.1, 4.7, 5.3)):
    return ri.Workload("t", np.eye(3) * L, np.array([mesh] * 3), np.array([center]),
                       np.array([0]), np.array([l]), np.array([a]), 1, 1, 0)


@pytest.mark.parametrize("l,a", [(0, 1.3), (1, 0.9), (2, 1.1), (2, 0.6)])
def test_shell_components_orthonormal(l, a):
    """Tight shell in a large cell: the grid overlap of its components is the
    identity (free-space normalisation, mutually orthogonal components)."""
    w = _one_shell_workload(l, a)
    Phi = basis.eval_basis(w)
    S = basis.overlap(Phi, grid.dvol(w.lattice, w.mesh))
    np.testing.assert_allclose(S, np.eye(2 * l + 1), atol=1e-10)


def test_d_shell_sum_of_squares_is_spherical():
    """For correctly normalised real spherical d functions sum_m d_m(r)^2
    depends only on |r| (addition theorem)."""
    d = np.random.default_rng(3).standard_normal((50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    v = basis.shell_values(2, 0.7, 1.3 * d)
    s = (v * v).sum(axis=1)
    np.testing.assert_allclose(s, s[0], rtol=1e-13)


def test_basis_is_periodic_and_sums_images():
    lat = np.array([[6.0, 0, 0], [0.8, 5.5, 0], [0.3, 0.2, 6.2]])
    w = ri.Workload("t", lat, np.array([8, 8, 8]), np.array([[0.2, 0.1, 5.9]]),
                    np.array([0, 0, 0]), np.array([0, 1, 2]), np.array([0.12, 0.3, 0.25]), 1, 1, 0)
    p = np.random.default_rng(0).uniform(0, 6, size=(20, 3))
    v0 = basis.eval_basis(w, p)
    for k in range(3):
        np.testing.assert_allclose(basis.eval_basis(w, p + lat[k]), v0, atol=1e-12, rtol=1e-12)
    # brute force over a wide block of images for the s shell
    A = w.atoms[0]
    acc = np.zeros(len(p))
    for i in range(-12, 13):
        for j in range(-12, 13):
            for k in range(-12, 13):
                T = i * lat[0] + j * lat[1] + k * lat[2]
                r2 = ((p - A - T) ** 2).sum(1)
                acc += (2 * 0.12 / math.pi) ** 0.75 * np.exp(-0.12 * r2)
    np.testing.assert_allclose(v0[:, 0], acc, rtol=1e-13, atol=1e-16)


def test_voronoi_brute_force():
    lat = np.array([[5.0, 0, 0], [1.1, 4.8, 0], [0.2, 0.4, 5.1]])
    atoms = np.array([[0.1, 0.2, 0.3], [2.5, 2.4, 2.6], [4.0, 1.0, 4.5]])
    w = ri.Workload("t", lat, np.array([7, 6, 5]), atoms, np.arange(3), np.zeros(3, int),
                    np.ones(3), 1, 1, 0)
    own = basis.voronoi(w)
    pts = grid.grid_points(lat, w.mesh)
    best = np.full(len(pts), np.inf)
    ref = np.zeros(len(pts), int)
    for I, A in enumerate(atoms):
        for i in range(-3, 4):
            for j in range(-3, 4):
                for k in range(-3, 4):
                    T = i * lat[0] + j * lat[1] + k * lat[2]
                    d2 = ((pts - A - T) ** 2).sum(1)
                    upd = d2 < best - 1e-12
                    best[upd] = d2[upd]
                    ref[upd] = I
    assert np.array_equal(own, ref)


# ---------------------------------------------------------------- conventional exchange
def test_conventional_exchange_closed_form():
    """Two s orbitals far from their images: E = -[(AA|AA) + (BB|BB) + 2 (AB|BA)]
    with every pair density a Gaussian (product theorem) whose Coulomb energy is
    the analytic lattice sum."""
    L, a, b = 10.0, 1.2, 1.6
    lat = np.eye(3) * L
    A = np.array([3.0, 3.5, 4.0])
    B = np.array([5.0, 4.6, 4.9])
    w = ri.Workload("t", lat, np.array([64] * 3), np.stack([A, B]), np.array([0, 1]),
                    np.array([0, 0]), np.array([a, b]), 2, 1, 0)
    Phi = basis.eval_basis(w)
    K, E = conventional.exchange_occ(Phi, np.eye(2), lat, w.mesh)

    def nrm(x):
        return (2 * x / math.pi) ** 0.75

    def self_energy(x, X):      # (rho|rho) for rho = N_x^2 exp(-2 x |r-X|^2)
        c = nrm(x) ** 2 / nrm(2 * x)
        return c * c * brute.analytic_s_coulomb(lat, X, 2 * x, X, 2 * x)
    p = a + b
    P = (a * A + b * B) / p
    cab = nrm(a) * nrm(b) * math.exp(-a * b / p * np.sum((A - B) ** 2)) / nrm(p)
    cross = cab * cab * brute.analytic_s_coulomb(lat, P, p, P, p)
    ref = -(self_energy(a, A) + self_energy(b, B) + 2 * cross)
    assert abs(E - ref) < 1e-10 * abs(ref)
    assert abs(E + np.trace(K)) < 1e-12 * abs(E)   # C = I: E = -tr(K)


def test_conventional_matches_dense_and_full():
    w = ri.tiny_s_cell(5, 6, 4.0, 2, 8, lmax=1)
    Phi = basis.eval_basis(w)
    dV = grid.dvol(w.lattice, w.mesh)
    C = ri.lowdin(ri.random_coefficients(w), basis.overlap(Phi, dV))
    K, E = conventional.exchange_occ(Phi, C, w.lattice, w.mesh)
    Vd = brute.dense_coulomb(w.lattice, w.mesh)
    U = Phi @ C
    Kref = np.zeros_like(K)
    Eref = 0.0
    for j in range(U.shape[1]):
        for i in range(U.shape[1]):
            Vij = Vd @ (U[:, i] * U[:, j])
            Kref[:, j] += dV * Phi.T @ (U[:, i] * Vij)
            Eref -= dV * (U[:, i] * U[:, j]) @ Vij
    np.testing.assert_allclose(K, Kref, atol=1e-13)
    assert abs(E - Eref) < 1e-13
    Kf = conventional.exchange_full(Phi, C, w.lattice, w.mesh)
    np.testing.assert_allclose(Kf @ C, K, atol=1e-13)
    np.testing.assert_allclose(Kf, Kf.T, atol=1e-13)
    assert np.linalg.eigvalsh(Kf).min() > -1e-12      # exchange operator is PSD
    assert E < 0


# ---------------------------------------------------------------- ISDF + rPS
@pytest.fixture(scope="module")
def tiny():
    w = ri.tiny_s_cell(6, 8, 4.0, 2, 8, lmax=1)
    Phi = basis.eval_basis(w)
    dV = grid.dvol(w.lattice, w.mesh)
    C = ri.lowdin(ri.random_coefficients(w), basis.overlap(Phi, dV))
    Kc, Ec = conventional.exchange_occ(Phi, C, w.lattice, w.mesh)
    return w, Phi, dV, C, Kc, Ec


def _delta(rho, pts, chi):
    return rho - rho[..., pts] @ chi


@pytest.mark.parametrize("naux", [10, 18, 30])
def test_rps_error_identities(tiny, naux):
    """Sec. 3.2: rPS keeps three of the four terms of the exact expansion and
    drops the fit-error term.  Hence, with delta_ab = rho_ab - sum_g
    rho_ab(R_g) chi_g computed independently:
      E_rPS - E_conv         = + dV sum_ij <delta_ij, Vc delta_ij>  (>= 0)
      K_rPS(mu,j) - K_conv   = - dV sum_i <delta_{mu i}, Vc delta_ij>
    A dropped line, a wrong sign or a transposed operand breaks these."""
    w, Phi, dV, C, Kc, Ec = tiny
    st = isdf.setup(w.with_naux(naux), Phi, mode="global")
    pts, chi = st["points"], st["chi"]
    K, E, Etr = rps.build_occ(Phi, pts, st["V"], st["W"], C, dV)
    U = Phi @ C
    n = U.shape[1]
    dij = np.stack([_delta(U[:, i] * U[:, j], pts, chi) for i in range(n) for j in range(n)])
    eref = dV * np.sum(dij * grid.poisson(dij, w.lattice, w.mesh))
    assert abs((E - Ec) - eref) < 1e-13 * max(1, abs(Ec))
    assert E - Ec >= -1e-14
    dK = np.zeros_like(K)
    for i in range(n):
        dmu = _delta((Phi * U[:, i][:, None]).T, pts, chi)           # (N, N_g)
        for j in range(n):
            vij = grid.poisson(_delta(U[:, i] * U[:, j], pts, chi), w.lattice, w.mesh)
            dK[:, j] -= dV * dmu @ vij
    np.testing.assert_allclose(K - Kc, dK, atol=1e-13)
    assert abs(E - Etr) < 1e-13


@pytest.mark.parametrize("naux", [10, 18, 30])
def test_ps_and_thc_error_identities(tiny, naux):
    """Sec. 3.2's expansion of the exact integral around the fit, for the two
    one-line approximations.  With rho_ab = u_a u_b, its fit rhobar_ab =
    sum_g rho_ab(R_g) chi_g and delta_ab = rho_ab - rhobar_ab (all computed
    here by FFT, not by the oracle's build):
      PS  (fitted pair times exact pair):  (mu i|i j) = dV <rhobar_mu i, Vc rho_ij>
          E_PS  - E_conv = + dV sum_ij <delta_ij, Vc rho_ij>
          K_PS  - K_conv = - dV sum_i <delta_mu i, Vc rho_ij>
      THC (fit times fit):                 (mu i|i j) = dV <rhobar_mu i, Vc rhobar_ij>
          E_THC - E_conv = + dV sum_ij (2 <delta_ij, Vc rho_ij> - <delta_ij, Vc delta_ij>)
          K_THC - K_conv = dV sum_i (<delta_mu i, Vc delta_ij> - <delta_mu i, Vc rho_ij>
                                     - <rho_mu i, Vc delta_ij>)
    A dropped term, a wrong sign, the wrong side fitted or a transposed
    operand in ps_occ / thc_occ breaks one of these."""
    w, Phi, dV, C, Kc, Ec = tiny
    st = isdf.setup(w.with_naux(naux), Phi, mode="global")
    pts, chi = st["points"], st["chi"]
    args = (Phi, pts, st["V"], st["W"], C, dV)
    Kps, Eps = rps.ps_occ(*args)
    Kthc, Ethc = rps.thc_occ(*args)
    U = Phi @ C
    n = U.shape[1]
    rho = np.stack([U[:, i] * U[:, j] for i in range(n) for j in range(n)])
    dlt = _delta(rho, pts, chi)
    vrho = grid.poisson(rho, w.lattice, w.mesh)
    vdlt = grid.poisson(dlt, w.lattice, w.mesh)
    d_r = dV * np.sum(dlt * vrho)          # sum_ij <delta_ij, Vc rho_ij>
    d_d = dV * np.sum(dlt * vdlt)          # sum_ij <delta_ij, Vc delta_ij>
    scale = max(1.0, abs(Ec))
    assert abs((Eps - Ec) - d_r) < 1e-13 * scale
    assert abs((Ethc - Ec) - (2.0 * d_r - d_d)) < 1e-13 * scale
    assert d_d > 0                          # the G != 0 Coulomb kernel is positive definite
    dps = np.zeros_like(Kc)
    dthc = np.zeros_like(Kc)
    for i in range(n):
        r_mu = (Phi * U[:, i][:, None]).T                             # rho_{mu i}, (N, N_g)
        d_mu = _delta(r_mu, pts, chi)
        for j in range(n):
            k = i * n + j
            dps[:, j] -= dV * d_mu @ vrho[k]
            dthc[:, j] += dV * (d_mu @ vdlt[k] - d_mu @ vrho[k] - r_mu @ vdlt[k])
    np.testing.assert_allclose(Kps - Kc, dps, atol=1e-13)
    np.testing.assert_allclose(Kthc - Kc, dthc, atol=1e-13)


def test_cholesky_shift_retry_rank_deficient_metric():
    """Sec. 4.3 solves the fit with a Cholesky factorisation of X_gg and names
    no regularisation.  X_gg = (Phi_g Phi_g^T)^2 has rank at most N(N+1)/2
    (the pair space), so with more points than that it is singular and the
    plain factorisation fails; the oracle then retries once with the shift
    lambda = 1e-13 max diag(X_gg) (reading of the paper).  Pinned here:
    numpy's own Cholesky rejects X_gg, the shifted factor reproduces
    X_gg + lambda I, and the fit made with it still obeys the exact rPS error
    identity (which holds for any chi with V = Vc chi and W = V chi^T)."""
    w = ri.tiny_s_cell(3, 8, 4.0, 2, 24, cid=91)        # 3 s functions: pair rank 6
    Phi = basis.eval_basis(w)
    dV = grid.dvol(w.lattice, w.mesh)
    C = ri.lowdin(ri.random_coefficients(w), basis.overlap(Phi, dV))
    Kc, Ec = conventional.exchange_occ(Phi, C, w.lattice, w.mesh)
    pts = np.random.default_rng(3).choice(w.ngrid, 24, replace=False)
    X = isdf.fitting_metric(Phi[pts])
    assert np.linalg.matrix_rank(X, tol=1e-10 * np.abs(X).max()) <= 6
    with pytest.raises(np.linalg.LinAlgError):
        np.linalg.cholesky(X)
    L, lam = isdf.cholesky_with_shift(X)
    assert lam == pytest.approx(1e-13 * float(np.max(np.diag(X))), rel=1e-15)
    np.testing.assert_allclose(L @ L.T, X + lam * np.eye(len(pts)), atol=1e-12 * np.abs(X).max())
    st = isdf.setup(w, Phi, points=pts)
    assert st["shift"] == lam
    K, E, Etr = rps.build_occ(Phi, pts, st["V"], st["W"], C, dV)
    U = Phi @ C
    dij = np.stack([_delta(U[:, i] * U[:, j], pts, st["chi"]) for i in range(2) for j in range(2)])
    eref = dV * np.sum(dij * grid.poisson(dij, w.lattice, w.mesh))
    assert abs((E - Ec) - eref) < 1e-12 * max(1.0, abs(Ec))
    assert abs(E - Etr) < 1e-12


def test_cholesky_fails_when_metric_vanishes():
    """A metric with zero diagonal (every basis value at the points zero) gets
    a zero shift and stays singular: the oracle raises, as the library returns
    its not-positive-definite error."""
    with pytest.raises(np.linalg.LinAlgError):
        isdf.cholesky_with_shift(np.zeros((8, 8)))


def test_rps_exact_with_all_points(tiny):
    """N_chi = N_g: chi is the identity and rPS reproduces exact exchange."""
    w, Phi, dV, C, Kc, Ec = tiny
    pts = np.random.default_rng(5).permutation(w.ngrid)
    st = isdf.setup(w.with_naux(w.ngrid), Phi, points=pts)
    K, E, _ = rps.build_occ(Phi, pts, st["V"], st["W"], C, dV)
    np.testing.assert_allclose(K, Kc, atol=1e-13)
    assert abs(E - Ec) < 1e-13


def test_rps_structure_and_invariants(tiny):
    w, Phi, dV, C, Kc, Ec = tiny
    st = isdf.setup(w.with_naux(18), Phi, mode="global")
    pts = st["points"]
    K, E, Etr, parts = rps.build_occ(Phi, pts, st["V"], st["W"], C, dV, return_parts=True)
    CK = C.T @ K
    np.testing.assert_allclose(CK, CK.T, atol=1e-14)                   # symmetric integrals
    np.testing.assert_allclose(C.T @ parts["K1"], (C.T @ parts["K2"]).T, atol=1e-14)
    Kf = rps.build_full(Phi, pts, st["V"], st["W"], C, dV)
    np.testing.assert_allclose(Kf, Kf.T, atol=1e-14)
    np.testing.assert_allclose(Kf @ C, K, atol=1e-14)
    assert E < 0 and abs(E - Etr) < 1e-13
    Q, _ = np.linalg.qr(np.random.default_rng(2).standard_normal((C.shape[1],) * 2))
    K2, E2, _ = rps.build_occ(Phi, pts, st["V"], st["W"], C @ Q, dV)
    assert abs(E2 - E) < 1e-13
    np.testing.assert_allclose(K2, K @ Q, atol=1e-13)
    np.testing.assert_allclose(st["W"], st["W"].T, atol=0)
    assert np.linalg.eigvalsh(st["W"]).min() > -1e-10 * np.abs(st["W"]).max()


@pytest.fixture(scope="module")
def cfg1():
    w = ri.tiny_cell()
    Phi = basis.eval_basis(w)
    dV = grid.dvol(w.lattice, w.mesh)
    C = ri.lowdin(ri.random_coefficients(w), basis.overlap(Phi, dV))
    Kc, Ec = conventional.exchange_occ(Phi, C, w.lattice, w.mesh)
    return w, Phi, dV, C, Kc, Ec, basis.voronoi(w)


@pytest.mark.parametrize("c", [5, 6])
def test_ps_and_thc_errors_are_first_order(cfg1, c):
    """Sec. 3.2: PS (line 1) and THC (line 3) carry O(eps) errors, rPS O(eps^2):
    once the fit is good the rPS error is far below both."""
    w, Phi, dV, C, Kc, Ec, own = cfg1
    st = isdf.setup(w.with_naux(c * w.nbas), Phi, owner=own)
    args = (Phi, st["points"], st["V"], st["W"], C, dV)
    _, E, _ = rps.build_occ(*args)
    _, Eps = rps.ps_occ(*args)
    _, Ethc = rps.thc_occ(*args)
    err = abs(E - Ec)
    assert abs(Eps - Ec) > 10 * err and abs(Ethc - Ec) > 10 * err


def test_fit_interpolates_and_solves_normal_equations(tiny):
    w, Phi, dV, C, Kc, Ec = tiny
    st = isdf.setup(w.with_naux(12), Phi, mode="global")
    pts, chi = st["points"], st["chi"]
    np.testing.assert_allclose(chi[:, pts], np.eye(len(pts)), atol=1e-8)
    X = isdf.fitting_metric(Phi[pts])
    XgR = (Phi[pts] @ Phi.T) ** 2
    assert np.abs(X @ chi - XgR).max() < 1e-10 * np.abs(XgR).max()


def test_randomized_qrcp_equals_full_qrcp_when_sketch_is_square():
    """With p = N the sketch matrices are square orthogonal, the sketch is an
    orthogonal row transform of the full pair matrix, and the pivots agree."""
    w = ri.tiny_s_cell(4, 6, 4.0, 2, 8)
    Phi = basis.eval_basis(w)
    full = isdf.qrcp_full(Phi, 8)
    sk = isdf.randomized_qrcp(Phi, 8, seed=77, streams=(0, 1))
    assert isdf.sketch_size(8, 4) == 4
    assert np.array_equal(full, sk)


def test_qrcp_pivots_are_greedy_max_residual():
    """QRCP pivot k = column of largest norm after projecting out pivots < k."""
    w = ri.tiny_s_cell(5, 6, 4.0, 2, 8, lmax=1)
    Phi = basis.eval_basis(w)
    N = Phi.shape[1]
    M = (Phi[:, :, None] * Phi[:, None, :]).reshape(Phi.shape[0], N * N).T
    piv = isdf.qrcp_full(Phi, 10)
    chosen = []
    for k in range(10):
        if chosen:
            Q, _ = np.linalg.qr(M[:, chosen])
            R = M - Q @ (Q.T @ M)
        else:
            R = M
        nr = np.linalg.norm(R, axis=0)
        nr[chosen] = -1
        chosen.append(int(np.argmax(nr)))
    assert list(piv) == chosen


def test_voronoi_isdf_quality_config1(cfg1):
    """Config-1 cell: the rPS energy error is non-negative and falls roughly
    exponentially with c = N_chi/N (Sec. 5.2, 5.3); the global randomized ISDF
    gives an error of the same size as v-ISDF (Sec. 5.1, Table 3)."""
    w, Phi, dV, C, Kc, Ec, own = cfg1
    errs = []
    for c in (2, 3, 4, 5, 6):
        st = isdf.setup(w.with_naux(c * w.nbas), Phi, owner=own)
        _, E, _ = rps.build_occ(Phi, st["points"], st["V"], st["W"], C, dV)
        errs.append(E - Ec)
    assert all(e >= -1e-12 for e in errs)
    assert all(errs[i + 1] < errs[i] / 3 for i in range(len(errs) - 1))
    assert errs[-1] < 1e-3 * errs[0]
    stg = isdf.setup(w, Phi, mode="global")
    _, Eg, _ = rps.build_occ(Phi, stg["points"], stg["V"], stg["W"], C, dV)
    assert 0 <= Eg - Ec < 10 * errs[2]


# ---------------------------------------------------------------- inputs
def test_workload_recipes():
    w1 = ri.tiny_cell()
    assert (w1.nbas, w1.nocc, w1.naux, w1.ngrid) == (40, 8, 160, 24 ** 3)
    w2 = ri.diamond_cell(6.0)
    assert (w2.nbas, w2.nocc, w2.naux, w2.ngrid, w2.natom) == (104, 16, 624, 48 ** 3, 8)
    assert [ri.diamond_cell(c).naux for c in (4, 6, 8, 10)] == [416, 624, 832, 1040]
    w3 = ri.diamond_2x2x2()
    assert (w3.nbas, w3.nocc, w3.naux, w3.ngrid) == (832, 128, 4992, 72 ** 3)
    w4 = ri.diamond_3x3x3()
    assert (w4.nbas, w4.nocc, w4.naux, w4.ngrid) == (2808, 432, 12000, 108 ** 3)
    assert np.array_equal(ri.diamond_cell().atoms, ri.diamond_cell().atoms)
    b = ri.batch_cells()
    assert len(b) == 64 and all(32 <= m <= 72 for x in b for m in x.mesh)
    assert all(ri.smooth_235(int(m)) == int(m) for x in b for m in x.mesh)
    assert all(x.naux == 6 * x.nbas and x.nocc == 2 * x.natom for x in b)


def test_lowdin_orthonormal():
    rg = np.random.default_rng(0)
    X = rg.standard_normal((30, 30))
    S = X @ X.T + 30 * np.eye(30)
    C = ri.lowdin(rg.standard_normal((30, 7)), S)
    np.testing.assert_allclose(C.T @ S @ C, np.eye(7), atol=1e-12)
    C2 = ri.perturbed(C, S, 1, cid=3)
    np.testing.assert_allclose(C2.T @ S @ C2, np.eye(7), atol=1e-12)
    assert 1e-4 < np.abs(C2 - C).max() < 0.2


# ---------------------------------------------------------------- Coulomb matrix (Sec. 2.3)
def test_coulomb_matrix_equals_four_index_contraction():
    """J_{mu nu} = sum_{lambda sigma} D_{lambda sigma} (mu nu|lambda sigma) with the
    four-index integrals formed explicitly from the dense Coulomb matrix of
    direct G sums (no FFT, no density on the grid), D = C C^T."""
    w = ri.tiny_s_cell(5, 6, 4.0, 2, 8, lmax=1)
    Phi = basis.eval_basis(w)
    dV = grid.dvol(w.lattice, w.mesh)
    C = ri.lowdin(ri.random_coefficients(w), basis.overlap(Phi, dV))
    J, E, vh = coulomb.build_j(Phi, C, w.lattice, w.mesh)
    N = Phi.shape[1]
    pairs = (Phi[:, :, None] * Phi[:, None, :]).reshape(Phi.shape[0], N * N)
    # (f|g) = dV f . Vc g with Vc the dense matrix (it carries the other dV)
    eri = dV * pairs.T @ brute.dense_coulomb(w.lattice, w.mesh) @ pairs   # (N^2, N^2)
    D = C @ C.T
    Jref = (eri @ D.reshape(-1)).reshape(N, N)
    assert np.abs(J - Jref).max() < 1e-13 * np.abs(Jref).max()
    Eref = 0.0
    for i in range(C.shape[1]):          # sum_ij (ii|jj) from the same tensor
        ci = np.outer(C[:, i], C[:, i]).reshape(-1)
        for j in range(C.shape[1]):
            Eref += ci @ eri @ np.outer(C[:, j], C[:, j]).reshape(-1)
    assert abs(E - Eref) < 1e-13 * abs(Eref)
    assert E > 0


def test_coulomb_single_orbital_equals_exchange():
    """One occupied orbital: (mu 1|1 1) is both the Coulomb and the exchange
    integral, so J C = K_occ and E_J = -E_x of the conventional exchange."""
    w = ri.tiny_s_cell(5, 6, 4.0, 1, 8, lmax=1)
    Phi = basis.eval_basis(w)
    dV = grid.dvol(w.lattice, w.mesh)
    C = ri.lowdin(ri.random_coefficients(w), basis.overlap(Phi, dV))
    assert C.shape[1] == 1
    J, E, _ = coulomb.build_j(Phi, C, w.lattice, w.mesh)
    K, Ex = conventional.exchange_occ(Phi, C, w.lattice, w.mesh)
    np.testing.assert_allclose(J @ C, K, atol=1e-14 * np.abs(K).max())
    assert abs(E + Ex) < 1e-14 * abs(Ex)


def test_coulomb_closed_form_two_s():
    """Two s functions far from their images, density of the second one:
    J_00 = (phi_a^2 | phi_b^2) and J_11 = E_J = (phi_b^2 | phi_b^2), each
    squared Gaussian an s Gaussian of twice the exponent whose Coulomb energy
    is the analytic lattice sum."""
    L, a, b = 10.0, 1.2, 1.6
    lat = np.eye(3) * L
    A = np.array([3.0, 3.5, 4.0])
    B = np.array([5.0, 4.6, 4.9])
    w = ri.Workload("t", lat, np.array([64] * 3), np.stack([A, B]), np.array([0, 1]),
                    np.array([0, 0]), np.array([a, b]), 1, 1, 0)
    Phi = basis.eval_basis(w)
    J, E, _ = coulomb.build_j(Phi, np.array([[0.0], [1.0]]), lat, w.mesh)

    def nrm(x):
        return (2 * x / math.pi) ** 0.75
    ca, cb = nrm(a) ** 2 / nrm(2 * a), nrm(b) ** 2 / nrm(2 * b)
    j00 = ca * cb * brute.analytic_s_coulomb(lat, A, 2 * a, B, 2 * b)
    j11 = cb * cb * brute.analytic_s_coulomb(lat, B, 2 * b, B, 2 * b)
    assert abs(J[0, 0] - j00) < 1e-10 * abs(j00)
    assert abs(J[1, 1] - j11) < 1e-10 * abs(j11)
    assert abs(E - j11) < 1e-10 * abs(j11)


def test_coulomb_invariants():
    """J is symmetric, depends on C only through D (occupied rotations leave
    it unchanged), is additive over blocks of orbitals, and E_J = tr(D J) > 0."""
    w = ri.tiny_s_cell(6, 8, 4.0, 3, 8, lmax=1)
    Phi = basis.eval_basis(w)
    dV = grid.dvol(w.lattice, w.mesh)
    C = ri.lowdin(ri.random_coefficients(w), basis.overlap(Phi, dV))
    J, E, _ = coulomb.build_j(Phi, C, w.lattice, w.mesh)
    np.testing.assert_allclose(J, J.T, atol=1e-15 * np.abs(J).max())
    Q, _ = np.linalg.qr(np.random.default_rng(4).standard_normal((3, 3)))
    JQ, EQ, _ = coulomb.build_j(Phi, C @ Q, w.lattice, w.mesh)
    np.testing.assert_allclose(JQ, J, atol=1e-13 * np.abs(J).max())
    J1, _, _ = coulomb.build_j(Phi, C[:, :1], w.lattice, w.mesh)
    J2, _, _ = coulomb.build_j(Phi, C[:, 1:], w.lattice, w.mesh)
    np.testing.assert_allclose(J1 + J2, J, atol=1e-13 * np.abs(J).max())
    assert abs(E - np.trace(C.T @ J @ C)) < 1e-13 * abs(E) and E > 0 and abs(EQ - E) < 1e-13 * E


# ---------------------------------------------------------------- Madelung term (Sec. 4.5)
def _lattice(kind, unit=1.0):
    if kind == "sc":
        return np.eye(3) * unit
    if kind == "bcc":
        return np.array([[-.5, .5, .5], [.5, -.5, .5], [.5, .5, -.5]]) * unit
    return np.array([[0, .5, .5], [.5, 0, .5], [.5, .5, 0]]) * unit


def test_madelung_published_constants():
    """Wigner-lattice constants from the literature (tests/golden/madelung_constants.txt)."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "madelung_constants.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for kind, unit, val in rows:
        lat = _lattice(kind, 1.7)
        om = abs(np.linalg.det(lat))
        length = 1.7 if unit == "L" else (3 * om / (4 * math.pi)) ** (1 / 3)
        assert abs(madelung.madelung(lat) * length - float(val)) < 2e-9


@pytest.mark.parametrize("kind", ["sc", "fcc", "skew"])
def test_madelung_independent_of_splitting(kind):
    lat = _lattice(kind, 5.0) if kind != "skew" else np.array([[6.0, 0, 0], [0.8, 5.5, 0], [0.3, 0.2, 6.2]])
    om = abs(np.linalg.det(lat))
    ref = madelung.madelung(lat)
    for f in (0.4, 0.7, 1.5, 2.5):
        assert abs(madelung.madelung(lat, eta=f * math.sqrt(math.pi) / om ** (1 / 3)) - ref) < 1e-12 * abs(ref)


def test_madelung_from_grid_potential():
    """The G = 0-free grid potential of a periodized normalised Gaussian charge
    (exponent a) at its centre is -M + 2 sqrt(a/pi) + pi/(a Omega) when the
    images are far apart (Ewald's identity with the splitting at sqrt(a))."""
    lat = np.array([[4.0, 0, 0], [0.5, 4.2, 0], [0.2, -0.3, 4.4]])
    mesh = (48, 50, 52)
    a = 3.0
    R = grid.grid_points(lat, mesh)
    f = (R @ np.linalg.inv(lat))
    rho = np.zeros(len(R))
    for i in (-1, 0, 1):
        for j in (-1, 0, 1):
            for k in (-1, 0, 1):
                d = (f - np.round(f) + np.array([i, j, k])) @ lat
                rho += (a / math.pi) ** 1.5 * np.exp(-a * np.einsum("ij,ij->i", d, d))
    v0 = grid.poisson(rho, lat, mesh)[0]          # grid point 0 is the charge centre
    om = abs(np.linalg.det(lat))
    ref = -madelung.madelung(lat) + 2 * math.sqrt(a / math.pi) + math.pi / (a * om)
    assert abs(v0 - ref) < 1e-10 * abs(ref)


def test_madelung_correction_shifts():
    """For S-orthonormal C the energy drops by n_occ M (= nM/2 for n = 2 n_occ
    electrons) and K_occ gains M S C."""
    w = ri.tiny_s_cell(5, 6, 4.0, 2, 8, lmax=1)
    Phi = basis.eval_basis(w)
    dV = grid.dvol(w.lattice, w.mesh)
    S = basis.overlap(Phi, dV)
    C = ri.lowdin(ri.random_coefficients(w), S)
    K, E = conventional.exchange_occ(Phi, C, w.lattice, w.mesh)
    M = madelung.madelung(w.lattice)
    K2, E2 = madelung.correct(K, E, C, S, M)
    assert abs((E - E2) - C.shape[1] * M) < 1e-12
    np.testing.assert_allclose(K2 - K, M * S @ C, atol=1e-14)



# ---------------------------------------------------------------- screened basis (Sec. 4.1)
def test_screen_s_function_radius():
    """One normalised s Gaussian in a large cubic cell (images below 1e-30): the
    kept points are exactly those inside the radius where sqrt(dV) N e^(-a r^2)
    equals eps, a closed form independent of the screening code."""
    L, m, a, eps = 24.0, 48, 0.7, 1e-6
    w = ri.tiny_s_cell(1, m, L, 1, 1, lmax=0)
    w = dataclasses.replace(w, atoms=np.array([[L / 2, L / 2, L / 2]]), shell_exp=np.array([a]))
    Phi = basis.eval_basis(w)
    dV = grid.dvol(w.lattice, w.mesh)
    Ps = basis.screen(Phi, eps, dV)
    ns = (2.0 * a / math.pi) ** 0.75
    rstar2 = math.log(math.sqrt(dV) * ns / eps) / a
    pts = grid.grid_points(w.lattice, w.mesh)
    r2 = np.sum((pts - L / 2) ** 2, axis=1)
    inside = r2 <= rstar2
    assert np.array_equal(Ps[:, 0] != 0.0, inside)
    assert np.array_equal(Ps[inside, 0], Phi[inside, 0])
    assert 0 < inside.sum() < len(inside)


def test_screen_monotone_and_identity(cfg1):
    w, Phi, dV, *_ = cfg1
    assert np.array_equal(basis.screen(Phi, 0.0, dV), Phi)
    a, b = basis.screen(Phi, 1e-6, dV), basis.screen(Phi, 1e-3, dV)
    assert np.all((b != 0) <= (a != 0))          # a larger eps keeps a subset
    kept = b != 0
    assert np.array_equal(b[kept], Phi[kept])    # kept values are untouched


def test_screen_at_paper_eps_leaves_exchange(cfg1):
    """At eps1 = 1e-8 the screened exchange (same points, V and W from the
    screened basis) differs from the unscreened one far below the fit error."""
    w, Phi, dV, C, Kc, Ec, _ = cfg1
    Ps = basis.screen(Phi, 1e-8, dV)
    st = isdf.setup(w, Phi)
    K0, E0, _ = rps.build_occ(Phi, st["points"], st["V"], st["W"], C, dV)
    st2 = isdf.setup(w, Ps, points=st["points"])
    K1, E1, _ = rps.build_occ(Ps, st2["points"], st2["V"], st2["W"], C, dV)
    assert abs(E1 - E0) < 1e-7 * abs(E0)
    assert np.abs(K1 - K0).max() < 1e-6 * np.abs(K0).max()
