"""FP64 CPU oracle of the reduced-frequency Lippmann-Schwinger solver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy implementation of what the GPU path computes, written from the paper
(Gierden, Waimann, Svendsen, Reese: "A geometrically adapted reduced set of
frequencies for a FFT-based microstructure simulation", arXiv 2103.10203).
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the HIP path and imports
nothing from the product package; the only shared module is ``synth`` (seeded
input generators, which hold none of the method's arithmetic).

Every tensor is a full 3x3 array (2D plane strain = 3D with the out-of-plane
wave-vector component and strains set to zero), every float is FP64, and
steps follow the paper's order:

* ``pattern``   - adapted sampling pattern: spectrum of g, top-R% amplitudes
                  (Sec. 4.2), with the tie and pair rules stated in pattern.py.
* ``green``     - Green operator Gamma^0 from its definition (Sec. 3, eq. Gamma),
                  continuous and rotated finite-difference wave vectors.
* ``material``  - Hooke and J2 with linear isotropic hardening (Sec. 2).
* ``solver``    - basic fixed-point scheme, full and reduced (Sec. 3 and 4).
* ``bounds``    - closed forms used as pins (Voigt/Reuss, laminate, HS).
* ``mlp``       - FP64 reference of the warm-start network (forward, backward,
                  Adam) for gradient checks.

Functions without an independent pin say "parity unpinned" in their docstring.
"""
from . import pattern, green, material, solver, bounds, mlp  # noqa: F401

__all__ = ["pattern", "green", "material", "solver", "bounds", "mlp"]
