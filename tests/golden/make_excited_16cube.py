"""Writes excited_16cube.json: the FP64 oracle's lowest eigenvalues of h(t_f) and the
excited-electron density n_ex (Sec. IV B, Eqs. (25)-(26)) on a 16^3 grid, from
dense N_r x N_r Hamiltonians (numpy.linalg.eigh). Calls only oracle/ and the seeded
input generator. Run from the repository root:

    python tests/golden/make_excited_16cube.py
"""

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import excited  # noqa: E402
from paper_1507_05156_amd import synth  # noqa: E402

CASE = dict(n=16, mesh=[2, 1, 1], nb=16, seed=2026, alpha=0.25, omega=synth.OMEGA_HSE, a_over_c=[0.0, 0.0, 0.05],
            vloc="synth.model_vloc(16)", psi="synth.orbitals(16, cell, kpts, 16, seed)")


def inputs(case=CASE):
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(case["mesh"][0], cell, case["mesh"][1], case["mesh"][2])
    psi = synth.orbitals(case["n"], cell, kp, case["nb"], seed=case["seed"])
    v = synth.model_vloc(case["n"])
    return cell, kp, psi, v


def main():
    t0 = time.time()
    cell, kp, psi, v = inputs()
    eps, phi = excited.eigenstates_dense(psi, kp, cell, CASE["omega"], np.array(CASE["a_over_c"]), CASE["alpha"],
                                         CASE["nb"], vloc=v, extra=1)
    nb = CASE["nb"]
    nex = excited.excited_density(phi[:, :nb], psi, cell)
    out = dict(case=CASE, eigenvalues=eps.tolist(), n_ex=nex,
               note="eigenvalues[k] holds the nb + 1 lowest (the last shows the gap); n_ex for phi = the nb lowest")
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "excited_16cube.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote excited_16cube.json in {time.time() - t0:.0f} s; gaps {eps[:, nb] - eps[:, nb - 1]}, n_ex {nex}")


if __name__ == "__main__":
    main()
