"""Shared helpers of the GPU parity tests (HIP path through the C ABI vs the
FP64 oracle on the same seeded inputs)."""
import numpy as np

import synth
from oracle import material, pattern, solver

LM, MM = synth.phase_lame(synth.MATRIX_E, synth.MATRIX_NU)
LI, MI = synth.phase_lame(synth.FIBRE_E, synth.FIBRE_NU)
ORACLE_PH = (material.Phase(LM, MM), material.Phase(LI, MI))
ORACLE_J2 = (material.Phase(LM, MM, sigma_y0=0.25, H=1.0, plastic=True), material.Phase(LI, MI))


def native_phases(j2=False):
    import paper_2103_10203_amd as mor
    m = mor.Phase(LM, MM, 0.25, 1.0, True) if j2 else mor.Phase(LM, MM)
    return [m, mor.Phase(LI, MI)]


def oracle_reduced(g, eb_comps, M, tol, max_iter=5000, j2=False, gamma="rotated"):
    dim = g.ndim
    p = pattern.build_pattern(g, M)
    eb = solver.macro_tensor(eb_comps, dim)
    ph = ORACLE_J2 if j2 else ORACLE_PH
    r = solver.solve(g, ph, eb, mask=p.mask(), tol=tol, max_iter=max_iter, gamma_kind=gamma)
    return p, r


def stress_comps(sig_bar, dim):
    return solver.tensor_comps(sig_bar, dim, with_s33=True)


def rel_l2(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))
