"""Write the stored ground energies used by the GPU Lanczos tests.

Calls only the oracle (tuple-built Hamiltonian, Eq. Talpha2, bisection ranks)
and LAPACK/ARPACK through it.  Run from the repository root:
    python tests/golden/make_golden.py [chain|anderson|all]
Outputs tests/golden/hubbard_chain_L14.json and tests/golden/anderson_12.json.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import hamiltonian as H  # noqa: E402
from oracle import lanczos as LZ  # noqa: E402
import synth  # noqa: E402

# Anderson impurity: impurity site 0 with eps_d and U, 11 bath sites.
AIM_SEED, AIM_NBATH, AIM_U, AIM_EPSD = 5, 11, 8.0, -4.0


def chain():
    L, U, nu, nd, seed, steps = 14, 4.0, 7, 7, 2, 200
    t0 = time.time()
    s = H.sector(L, nu, nd)
    A = H.sparse(s, H.terms(L, H.chain_bonds(L), U))
    e_exact = LZ.lowest_eigenvalue(A)
    v0 = synth.start_vector(seed, s.size)
    a, b = LZ.lanczos(lambda v: A @ v, v0, steps)
    e_200 = LZ.tridiag_lowest(a, b)
    out = {
        "about": "periodic Hubbard chain L=14, t=1, U=4, (N_up, N_dn) = (7, 7); oracle values",
        "L": L, "U": U, "n_up": nu, "n_dn": nd, "dim": int(s.size),
        "e0_exact": e_exact,
        "lanczos_steps": steps, "start_seed": seed, "e0_lanczos": e_200,
        "alpha_first10": [float(x) for x in a[:10]], "beta_first10": [float(x) for x in b[:10]],
        "seconds": time.time() - t0,
    }
    json.dump(out, open(os.path.join(HERE, "hubbard_chain_L14.json"), "w"), indent=1)
    print("chain", out["e0_exact"], out["e0_lanczos"], out["seconds"])


def anderson():
    t0 = time.time()
    L = AIM_NBATH + 1
    eps_b, V = synth.anderson_parameters(AIM_SEED, AIM_NBATH)
    eps = np.concatenate([[AIM_EPSD], eps_b])
    U = [AIM_U] + [0.0] * AIM_NBATH
    bonds = H.star_bonds(V)
    tl = H.terms(L, bonds, U, eps)
    res = {}
    for nu in range(L + 1):
        for nd in range(L + 1):
            s = H.sector(L, nu, nd)
            A = H.sparse(s, tl)
            res[f"{nu},{nd}"] = LZ.lowest_eigenvalue(A)
    free = {f"{nu},{nd}": H.free_energy(L, bonds, nu, nd, eps)
            for nu in range(L + 1) for nd in range(L + 1)}
    out = {
        "about": "Anderson impurity, 1 impurity + 11 bath sites, U=8, eps_d=-4, "
                 "bath from synth.anderson_parameters(5, 11); oracle values per sector",
        "seed": AIM_SEED, "U": AIM_U, "eps_d": AIM_EPSD,
        "eps_bath": [float(x) for x in eps_b], "V": [float(x) for x in V],
        "e0": res, "e0_U0": free, "seconds": time.time() - t0,
    }
    json.dump(out, open(os.path.join(HERE, "anderson_12.json"), "w"), indent=1)
    print("anderson", min(res.values()), out["seconds"])


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "all"
    if what in ("anderson", "all"):
        anderson()
    if what in ("chain", "all"):
        chain()
