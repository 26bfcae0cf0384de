"""mor_solve_noalloc (the solve whose workspace is the library's fixed device
scratch array) against mor_solve on the same inputs: two calls in a row, the
second with fewer RVEs, so the second call runs on what the first left in
the array.  The kernels and summation orders are the same, so the results
are compared bit for bit; the J2 case checks that the internal plastic state
starts from zero on every call."""
import math

import numpy as np
import pytest

import synth
from tests.gpu_common import native_phases

pytestmark = pytest.mark.gpu


def _both(mor, plan, eb, ph, **kw):
    a = mor.solve(plan, eb, ph, 1e-6, want_fields=True, want_coeffs=True, **kw)
    b = mor.solve(plan, eb, ph, 1e-6, want_fields=True, want_coeffs=True, noalloc=True, **kw)
    return a, b


def _same(a, b):
    assert a.status == b.status == 0
    assert np.array_equal(a.iterations, b.iterations)
    assert np.array_equal(a.eff_stress, b.eff_stress)
    assert np.array_equal(a.residual, b.residual)
    assert bool((a.strain == b.strain).all()) and bool((a.stress == b.stress).all())
    assert bool((a.coeffs == b.coeffs).all())


@pytest.mark.parametrize("j2", [False, True])
def test_noalloc_equals_solve_twice_shrinking(j2):
    import paper_2103_10203_amd as mor
    g = synth.rsa_fibres(64, 64, 4.0, 8.0, seed=501, target_vf=0.35).g
    plan = mor.Plan(g, int(math.ceil(0.05 * g.size)))
    ph = native_phases(j2=j2)
    scale = 4.0 if j2 else 1.0  # J2: strains beyond yield
    for B, seed in ((9, 1), (4, 2)):
        eb = synth.macro_strains(B, 3, 5e-3 * scale, seed=seed)
        a, b = _both(mor, plan, eb, ph)
        _same(a, b)


def test_noalloc_3d_and_fp64():
    import paper_2103_10203_amd as mor
    g3 = synth.rsa_spheres(32, 32, 32, 3.0, 5.0, seed=502, target_vf=0.2).g
    p3 = mor.Plan(g3, int(math.ceil(0.05 * g3.size)))
    eb3 = synth.macro_strains(3, 6, 1e-3, seed=3)
    _same(*_both(mor, p3, eb3, native_phases()))
    g2 = synth.rsa_fibres(64, 64, 4.0, 8.0, seed=503, target_vf=0.35).g
    p2 = mor.Plan(g2, 205)
    eb2 = synth.macro_strains(2, 3, 5e-3, seed=4)
    _same(*_both(mor, p2, eb2, native_phases(), precision=mor.PREC_FP64))


def test_noalloc_rejects_beyond_scratch():
    """A batch whose workspace exceeds the scratch array is refused on the
    host before any kernel runs; a batch that fits still solves after it."""
    import paper_2103_10203_amd as mor
    g = synth.rsa_fibres(256, 256, 8.0, 16.0, seed=504, target_vf=0.35).g
    plan = mor.Plan(g, 3277)
    eb = synth.macro_strains(1024, 3, 5e-3, seed=5)
    with pytest.raises(mor.MorError) as ei:
        mor.solve(plan, eb, native_phases(), 1e-6, noalloc=True)
    assert ei.value.status == mor.MOR_E_INVALID_ARG
    assert "scratch" in str(ei.value)
    a = mor.solve(plan, eb[:8], native_phases(), 1e-6)
    b = mor.solve(plan, eb[:8], native_phases(), 1e-6, noalloc=True)
    assert np.array_equal(a.eff_stress, b.eff_stress) and np.array_equal(a.iterations, b.iterations)
