"""FP64 CPU oracle for the FFT phase-field twin-propagation step.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
link anything in this package; only the tests, the smoke check and the
benchmark's CPU-baseline leg use it. It shares no code with the HIP library.

The oracle is a plain, slow, obviously correct NumPy/SciPy implementation of
what one step of the method computes, written from the paper (Zhang, Ma &
Llorca, "Simulation of dislocation slip and twin propagation in Mg through
coupling crystal plasticity and phase field models"):

* ``crystal``   - Mg twin crystallography and stiffness rotation
                  (Sec. 2.1, eq. (5); the twin eigenstrain of eq. (6)).
* ``spectral``  - FFT conventions, wavevectors, the Green's operator of the
                  Moulinec-Suquet scheme (textbook; the paper takes its
                  strain from the FE solution instead, Sec. 2.2).
* ``mech``      - stress, mixed boundary condition, Moulinec-Suquet fixed
                  point (small-strain analogue of eq. (4) with the mixture
                  stiffness of eq. (5)).
* ``phasefield``- driving forces of eq. (17), the linearised semi-implicit
                  update of eqs. (19)-(20) solved in Fourier space
                  (Table 1), energies of eqs. (12)-(15).

Where the paper is silent or garbled the reading taken is stated in the
docstring of the function that depends on it.
"""

from . import crystal, spectral, mech, phasefield  # noqa: F401
