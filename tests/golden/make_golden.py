"""Writes oracle-derived expected values used by the GPU parity tests.

Calls only the oracle and the seeded instance generators; nothing here comes
from the GPU path.  Run from the repository root:
    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np
import scipy.linalg

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2001_01978_amd import inputs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def c1_dense(seeds):
    out = []
    for seed in seeds:
        om, n, eps, V = inputs.c1_instance(seed)
        basis = oracle.basis_alg1(om, n)
        H = oracle.dense_h(om, n, eps, V, basis)
        w, Z = scipy.linalg.eigh(H, subset_by_index=[0, 1], driver="evr")
        psi = Z[:, 0] / np.linalg.norm(Z[:, 0])
        if psi.sum() < 0:
            psi = -psi
        occ = oracle.occupations(om, basis, psi)
        out.append(dict(seed=seed, E0=float(w[0]), E1=float(w[1]), occ=[float(v) for v in occ],
                        monopole_min=oracle.monopole_min(om, n, eps, V)))
        print("c1 seed", seed, w[0], flush=True)
    return out


def main():
    res = {
        "what": "oracle dense diagonalisation of the Omega=16, n=8 random family (eps = 10*sort(U[0,1)^16), "
                "G_ij = 0.3(1+0.2u)) and the Richardson value of Omega=28, n=14, eps_i=i, G=0.4",
        "c1": c1_dense([0, 1, 2]),
    }
    eps = np.arange(1, 29, dtype=float)
    E, _ = oracle.richardson_evb(eps, 0.4, 14)
    res["c2a_richardson_E0"] = E
    with open(os.path.join(HERE, "oracle_expected.json"), "w") as f:
        json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
