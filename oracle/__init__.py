"""CPU oracle for the two-lead strip transport path (FP64, numpy).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check of the entry module and
the CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library (``paper_1010_2627_amd``); its inputs are plain numpy arrays built by
the seeded generators of ``paper_1010_2627_amd.inputs``.

Contents
--------
``leads``   lead surface Green function by decimation, the analytic modal
            self-energy of a square-lattice lead, the 1D closed form, and the
            open-channel count.
``rgf``     the slice-by-slice Dyson recursion, propagators G_1N / G_N1,
            Fisher-Lee transmission, the Ward-identity check and the LDOS
            backward sweep.
``dense``   brute force: the retarded Green function of the whole finite
            system by one dense inverse (plain definition, section 2.3 Eq. (2)),
            for tiny systems and for the worked example of section 2.2.
``lesser``  the lesser Green function of injection from one lead,
            G_l^< = i G Gamma_l G^dagger (section 2.3), and the local
            observables built on it: injected density and spin (on-site
            blocks), longitudinal and transverse currents into every site.
``multiterminal``  the conductance matrix T_kl = Tr[Gamma_k G_kl Gamma_l
            G_kl^dagger] of a strip with further leads attached to single
            slices (section 2.3, section 6.1), by one dense inverse.
``noise``   transmission eigenvalues (eigenvalues of t t^dagger with
            t = Gamma_R^{1/2} G_N1 Gamma_L^{1/2}) and the shot-noise Fano
            factor, section 2.1 item (a).

Every function names the passage it follows.  Parity status: every function is
pinned by a test in ``tests/test_oracle_*.py`` against closed forms, brute
force or the worked example's printed values; the decimation is pinned by the
modal closed form only away from channel thresholds.
"""

from .leads import (surface_gf_decimation, sigma_left, sigma_right, sigma_square_modal, sigma_modes,
                    sigma_chain_closed_form, n_open_square, gamma_of)
from .rgf import (rgf_forward, transmission_lr, transmission_rl, transmission_ward, ldos_rgf,
                  slice_hamiltonians, transmission_full)
from .dense import dense_green, dense_strip_hamiltonian, dense_transmission, dense_ldos
from .noise import psd_sqrt, transmission_amplitude, transmission_eigenvalues, fano_factor
from .lesser import strip_green_dense, injected_spectral, local_observables
from .multiterminal import green_with_leads, conductance_matrix

__all__ = [
    "surface_gf_decimation", "sigma_left", "sigma_right", "sigma_square_modal", "sigma_modes",
    "sigma_chain_closed_form", "n_open_square", "gamma_of", "rgf_forward", "transmission_lr",
    "transmission_rl", "transmission_ward", "ldos_rgf", "slice_hamiltonians", "transmission_full",
    "dense_green", "dense_strip_hamiltonian", "dense_transmission", "dense_ldos",
    "psd_sqrt", "transmission_amplitude", "transmission_eigenvalues", "fano_factor",
    "strip_green_dense", "injected_spectral", "local_observables",
    "green_with_leads", "conductance_matrix",
]
