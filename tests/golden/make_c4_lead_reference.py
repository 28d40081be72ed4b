"""Write tests/golden/c4_lead_reference.npz: oracle values for the spinful W=256 strip.

The headline workload's lead (spinful square lattice, slice dimension 512,
Rashba 0.2t, Zeeman 0.1t) at two energies of its 64-point midpoint grid in
(-3.9, 3.9), computed by the oracle only:
  * the exact Bloch-mode self-energies of both leads (oracle.leads.sigma_modes),
    stored as sampled rows (0, 1, 255, 256, 510, 511) and the full diagonal;
  * the open-channel count of each lead (eigenvalues of Gamma above 1e-8);
  * end to end on realization 0 of the workload (seed 10102627, disorder
    U[-1, 1], L = 512): the Fisher-Lee transmission with those self-energies
    (oracle.rgf) and the transmission eigenvalues (oracle.noise).
One Bloch-mode self-energy at this size takes about a minute on a CPU, so the
GPU tests read these stored values instead of recomputing them.

Run from the repository root:  python tests/golden/make_c4_lead_reference.py
"""

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import leads as OL      # noqa: E402
from oracle import noise as ON      # noqa: E402
from oracle import rgf as OR        # noqa: E402
from paper_1010_2627_amd import inputs   # noqa: E402

ENERGY_INDEX = (17, 50)
ROWS = (0, 1, 255, 256, 510, 511)


def main():
    st = inputs.rashba_strip(256, alpha=0.2, ez=0.1)
    V = st.V_dense()
    grid = inputs.midpoint_grid(-3.9, 3.9, 64)
    E = grid[list(ENERGY_INDEX)]
    sL = np.stack([OL.sigma_modes(st.H0, V, e, "L") for e in E])
    sR = np.stack([OL.sigma_modes(st.H0, V, e, "R") for e in E])
    nopen = np.array([[(np.linalg.eigvalsh(OL.gamma_of(s)) > 1e-8).sum() for s in S] for S in (sL, sR)])
    on = inputs.onsite_disorder(st, 512, 2.0, inputs.SEED_BASE)
    res = OR.rgf_forward(st.H0, V, on, E, sL, sR)
    T = OR.transmission_lr(sL, sR, res["G1N"])
    Tn = ON.transmission_eigenvalues(sL, sR, res["GN1"])
    rows = np.array(ROWS)
    np.savez_compressed(
        os.path.join(ROOT, "tests", "golden", "c4_lead_reference.npz"),
        energy_index=np.array(ENERGY_INDEX), E=E, rows=rows,
        sigmaL_rows=sL[:, rows, :], sigmaR_rows=sR[:, rows, :],
        sigmaL_diag=np.diagonal(sL, axis1=1, axis2=2), sigmaR_diag=np.diagonal(sR, axis1=1, axis2=2),
        nopen=nopen, T=T, Tn=Tn[:, :int(nopen.min())])
    print("E", E, "N_open", nopen.tolist(), "T", T)


if __name__ == "__main__":
    main()
