"""Write the stored oracle results used by the GPU parity tests.

Calls only ``oracle/`` and the seeded workload recipes in ``rps_inputs``; no
value here comes from the HIP library.  For the 8-atom diamond-like cell
(48^3 grid, N = 104, n_occ = 16) and c = N_chi/N in {4, 6, 8, 10} it stores:
the S-orthonormal occupied coefficients C, the oracle's Voronoi-ISDF points,
the rPS occ-RI exchange K_occ and E_x for those points (Eq. 16), the PS and THC
variants, the conventional exact exchange, and samples of Phi, V and W.

    python tests/golden/make_golden.py            # all c values
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import rps_inputs as ri  # noqa: E402
from oracle import basis, conventional, grid, isdf, rps  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))


def main(cs=(4, 6, 8, 10)):
    w0 = ri.diamond_cell(6.0)
    t = time.time()
    Phi = basis.eval_basis(w0)
    dV = grid.dvol(w0.lattice, w0.mesh)
    S = basis.overlap(Phi, dV)
    C = ri.lowdin(ri.random_coefficients(w0), S)
    own = basis.voronoi(w0)
    Kc, Ec = conventional.exchange_occ(Phi, C, w0.lattice, w0.mesh)
    print(f"basis/conventional {time.time() - t:.1f}s  E_conv={Ec:.12f}", flush=True)
    rng = np.random.default_rng(1234)
    phi_rows = np.sort(rng.choice(w0.ngrid, 256, replace=False))
    for c in cs:
        w = ri.diamond_cell(float(c))
        t = time.time()
        st = isdf.setup(w, Phi, owner=own)
        args = (Phi, st["points"], st["V"], st["W"], C, dV)
        K, E, Etr = rps.build_occ(*args)
        Kps, Eps = rps.ps_occ(*args)
        Kthc, Ethc = rps.thc_occ(*args)
        vr = np.sort(rng.choice(w.naux, 16, replace=False))
        vc = np.sort(rng.choice(w.ngrid, 64, replace=False))
        wr = np.sort(rng.choice(w.naux, 48, replace=False))
        np.savez_compressed(
            os.path.join(OUT, f"diamond1x1x1_c{c}.npz"),
            C=C, points=st["points"], K=K, E=E, E_trace=Etr, K_ps=Kps, E_ps=Eps, K_thc=Kthc, E_thc=Ethc,
            K_conv=Kc, E_conv=Ec, shift=st["shift"], phi_rows=phi_rows, Phi_s=Phi[phi_rows],
            v_rows=vr, v_cols=vc, V_s=st["V"][np.ix_(vr, vc)], w_rows=wr, W_s=st["W"][np.ix_(wr, wr)],
            owner=own.astype(np.int32), S=S, naux=w.naux)
        print(f"c={c} N_chi={w.naux} setup+build {time.time() - t:.1f}s  E={E:.12f}  err={E - Ec:.3e}",
              flush=True)


if __name__ == "__main__":
    main(tuple(int(x) for x in sys.argv[1:]) or (4, 6, 8, 10))
