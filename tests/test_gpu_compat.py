"""GPU parity of the compatibility step (paper Sec. 4.1 post-processing and
Sec. 5.1, fig. OneIncCircComp): one full-set pass from a reduced solution,
through mor_compat, against the oracle's step from its own reduced solution
(solved to 1e-12).  Also its fixed point: from the full-set solution it
changes nothing."""
import math

import numpy as np
import pytest

import synth
from oracle import pattern, solver
from tests.gpu_common import ORACLE_J2, ORACLE_PH, native_phases, rel_l2, stress_comps

pytestmark = pytest.mark.gpu


def _fields(t, dim):
    return np.moveaxis(t.double().cpu().numpy(), 0, -1)


def _check(out, ref, dim, b=0):
    want = stress_comps(ref.sigma_bar, dim)
    assert np.max(np.abs(out.eff_stress[b] - want)) / np.max(np.abs(want)) < 1e-5
    eps = _fields(out.strain[b], dim)
    assert rel_l2(eps, solver.tensor_comps(ref.eps, dim)) < 1e-4
    sig = _fields(out.stress[b], dim)
    assert rel_l2(sig, stress_comps(ref.sigma, dim)) < 1e-4
    assert abs(out.residual[b] - ref.residuals[0]) < 1e-3 * ref.residuals[0] + 1e-6


@pytest.mark.parametrize("kind", ["adapted", "radial"])
@pytest.mark.parametrize("n", [64, 256])
def test_compat_2d_matches_oracle(kind, n):
    import paper_2103_10203_amd as mor
    g = synth.rsa_fibres(n, n, n / 16, n / 8, seed=700 + n, target_vf=0.35).g
    eb = np.array([[1e-3, -4e-4, 3e-4], [-2e-3, 1e-3, 0.0]])
    if kind == "adapted":
        M = int(math.ceil(0.02 * g.size))
        plan = mor.Plan(g, M)
        mask = pattern.build_pattern(g, M).mask()
    else:
        plan = mor.Plan(g, 1, radial_lines=8)
        mask = pattern.build_radial_pattern(g.shape, 8).mask()
    full = mor.Plan(g, g.size)
    red = mor.solve(plan, eb, native_phases(), 1e-6, want_coeffs=True)
    assert red.status == mor.MOR_OK
    out = mor.compat(plan, full, red.coeffs, eb, native_phases())
    assert out.status == mor.MOR_OK and np.all(out.iterations == 1)
    for b in range(2):
        E = solver.macro_tensor(eb[b], 2)
        r = solver.solve(g, ORACLE_PH, E, mask=mask, tol=1e-12, max_iter=5000)
        ref = solver.compatibility_step(g, ORACLE_PH, E, r.eps)
        _check(out, ref, 2, b)


def test_compat_3d_matches_oracle():
    import paper_2103_10203_amd as mor
    g = synth.rsa_spheres(32, 32, 32, 3.0, 5.0, seed=710, target_vf=0.2).g
    eb = np.array([[1e-3, -2e-4, 0.0, 1e-4, -3e-4, 2e-4]])
    M = int(math.ceil(0.03 * g.size))
    plan = mor.Plan(g, M)
    full = mor.Plan(g, g.size)
    red = mor.solve(plan, eb, native_phases(), 1e-6, want_coeffs=True)
    out = mor.compat(plan, full, red.coeffs, eb, native_phases())
    E = solver.macro_tensor(eb[0], 3)
    r = solver.solve(g, ORACLE_PH, E, mask=pattern.build_pattern(g, M).mask(), tol=1e-12, max_iter=5000)
    _check(out, solver.compatibility_step(g, ORACLE_PH, E, r.eps), 3)


def test_compat_j2_single_step():
    """J2 matrix, one load step from the virgin state: the reduced solve and
    the step both use the virgin committed state."""
    import paper_2103_10203_amd as mor
    n = 64
    g = synth.rsa_fibres(n, n, 4.0, 8.0, seed=720, target_vf=0.35).g
    eb = np.array([[8e-3, -2e-3, 1e-3]])
    M = int(math.ceil(0.05 * g.size))
    plan = mor.Plan(g, M)
    full = mor.Plan(g, g.size)
    red = mor.solve(plan, eb, native_phases(j2=True), 1e-6, want_coeffs=True)
    assert red.status == mor.MOR_OK
    out = mor.compat(plan, full, red.coeffs, eb, native_phases(j2=True))
    E = solver.macro_tensor(eb[0], 2)
    r = solver.solve(g, ORACLE_J2, E, mask=pattern.build_pattern(g, M).mask(), tol=1e-12, max_iter=5000)
    ref = solver.compatibility_step(g, ORACLE_J2, E, r.eps)
    assert r.alpha.max() > 0.0
    _check(out, ref, 2)


def test_compat_fixed_point_of_full_solution():
    import paper_2103_10203_amd as mor
    g = synth.rsa_fibres(64, 64, 4.0, 8.0, seed=730, target_vf=0.35).g
    eb = np.array([[1e-3, 5e-4, -2e-4]])
    full = mor.Plan(g, g.size)
    sol = mor.solve(full, eb, native_phases(), 1e-7, want_coeffs=True)
    out = mor.compat(full, full, sol.coeffs, eb, native_phases())
    assert out.residual[0] < 1e-6
    assert np.max(np.abs(out.eff_stress[0] - sol.eff_stress[0])) < 1e-6 * np.max(np.abs(sol.eff_stress[0]))


def test_compat_rejects_mismatched_plans():
    import paper_2103_10203_amd as mor
    g = synth.disk(32, 32, 8.0)
    plan = mor.Plan(g, 51)
    eb = np.array([[1e-3, 0.0, 0.0]])
    red = mor.solve(plan, eb, native_phases(), 1e-6, want_coeffs=True)
    for bad in (mor.Plan(g, 100), mor.Plan(synth.disk(32, 32, 5.0), g.size), mor.Plan(synth.disk(64, 64, 8.0), 4096)):
        with pytest.raises(mor.MorError) as ei:
            mor.compat(plan, bad, red.coeffs, eb, native_phases())
        assert ei.value.status == mor.MOR_E_INVALID_ARG
