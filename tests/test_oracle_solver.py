"""Pins of the oracle's fixed-point solver (paper Secs. 2-4) against results the
mathematics fixes: homogeneous media, the mean-strain condition, the Voigt
limit of a one-frequency pattern, the full-set special case, the exact
laminate solution, energy bounds over nested patterns, Hill/Hashin bulk
bounds, a directly solved Galerkin system on a tiny grid, and J2 material-point
closed forms."""
import numpy as np
import pytest

import synth
from oracle import bounds, green, material, pattern, solver

LM, MM = synth.phase_lame(synth.MATRIX_E, synth.MATRIX_NU)
LI, MI = synth.phase_lame(synth.FIBRE_E, synth.FIBRE_NU)
PH = (material.Phase(LM, MM), material.Phase(LI, MI))


def _hooke_tensor_apply(lam, mu, e):
    return lam * np.trace(e) * np.eye(3) + 2 * mu * e


def test_lame_conversion_values():
    # fibre E=400, nu=0.2; matrix E=70, nu=0.3 (GPa)
    assert abs(LI - 111.1111111111111) < 1e-9 and abs(MI - 166.6666666666667) < 1e-9
    assert abs(LM - 40.38461538461539) < 1e-9 and abs(MM - 26.92307692307692) < 1e-9


@pytest.mark.parametrize("fill", [0, 1])
@pytest.mark.parametrize("dim", [2, 3])
def test_homogeneous_medium_one_step(fill, dim):
    shape = (8, 12) if dim == 2 else (6, 4, 8)
    g = np.full(shape, fill, np.uint8)
    comps = [1e-3, -4e-4, 2.5e-4] if dim == 2 else [1e-3, -4e-4, 3e-4, 1e-4, -2e-4, 2.5e-4]
    eb = solver.macro_tensor(comps, dim)
    res = solver.solve(g, PH, eb, tol=1e-12)
    assert res.iterations == 1 and res.residuals[0] == 0.0
    p = PH[fill]
    ref = _hooke_tensor_apply(p.lam, p.mu, eb)
    assert np.max(np.abs(res.sigma_bar - ref)) < 1e-13 * np.max(np.abs(ref))


def test_mean_strain_equals_macro_strain():
    g = synth.rsa_fibres(32, 32, 3, 6, seed=2, target_vf=0.3).g
    eb = solver.macro_tensor([2e-3, -1e-3, 7e-4], 2)
    p = pattern.build_pattern(g, 60)
    res = solver.solve(g, PH, eb, mask=p.mask(), tol=1e-10)
    mean = res.eps.reshape(-1, 3, 3).mean(axis=0)
    assert np.max(np.abs(mean - eb)) < 1e-17
    # plane strain: no out-of-plane strain appears
    assert np.max(np.abs(res.eps[..., 2, :])) == 0.0


def test_single_frequency_gives_voigt():
    g = synth.rsa_fibres(32, 32, 3, 6, seed=4, target_vf=0.35).g
    eb = solver.macro_tensor([1e-3, 5e-4, -3e-4], 2)
    p = pattern.build_pattern(g, 1)
    assert p.M_actual == 1
    res = solver.solve(g, PH, eb, mask=p.mask(), tol=1e-12)
    ref = bounds.voigt_stress(PH, float(g.mean()), eb)
    assert res.iterations == 1
    assert np.max(np.abs(res.sigma_bar - ref)) < 1e-13 * np.max(np.abs(ref))


def test_all_frequencies_equals_full_scheme_bitwise():
    g = synth.disk(16, 16, 5.1)
    eb = solver.macro_tensor([1e-3, 0, 0], 2)
    p = pattern.build_pattern(g, g.size)
    r1 = solver.solve(g, PH, eb, mask=p.mask(), tol=1e-10)
    r2 = solver.solve(g, PH, eb, mask=None, tol=1e-10)
    assert r1.iterations == r2.iterations
    assert np.array_equal(r1.sigma_bar, r2.sigma_bar)
    assert np.array_equal(r1.eps, r2.eps)


@pytest.mark.parametrize("kind", [green.ROTATED, green.CONTINUOUS])
@pytest.mark.parametrize("reduced", [False, True])
def test_laminate_closed_form(kind, reduced):
    shape = (32, 16)
    g = synth.laminate(shape, 11, offset=5)
    eb = solver.macro_tensor([1e-3, -6e-4, 4e-4], 2)
    mask = None
    if reduced:
        keys, _ = pattern.spectrum_keys(g)
        M = int(np.count_nonzero(keys))
        mask = pattern.build_pattern(g, M).mask()
        assert mask.sum() < g.size // 4
    res = solver.solve(g, PH, eb, mask=mask, tol=1e-13, gamma_kind=kind, max_iter=500)
    eps_ref, sig_ref, sbar_ref = bounds.laminate_fields(g[:, 0], PH, eb)
    assert np.max(np.abs(res.eps - eps_ref[:, None])) < 1e-14
    assert np.max(np.abs(res.sigma_bar - sbar_ref)) < 1e-11


def test_laminate_fails_when_pattern_misses_support():
    shape = (32, 16)
    g = synth.laminate(shape, 11, offset=5)
    eb = solver.macro_tensor([1e-3, 0, 0], 2)
    keys, _ = pattern.spectrum_keys(g)
    M = int(np.count_nonzero(keys))
    mask = pattern.build_pattern(g, M - 3).mask()
    res = solver.solve(g, PH, eb, mask=mask, tol=1e-13, max_iter=500)
    eps_ref, _, _ = bounds.laminate_fields(g[:, 0], PH, eb)
    assert np.max(np.abs(res.eps - eps_ref[:, None])) > 1e-7


def test_energy_bounds_nested_patterns():
    g = synth.rsa_fibres(32, 32, 3, 7, seed=11, target_vf=0.35).g
    eb = solver.macro_tensor([1e-3, -2e-4, 3e-4], 2)
    f = float(g.mean())
    w_reuss, w_voigt = bounds.voigt_reuss_energy(PH, f, eb, 2)
    full = solver.solve(g, PH, eb, tol=1e-12, max_iter=2000)
    ws = []
    for M in [1, 8, 40, 160, 512]:
        r = solver.solve(g, PH, eb, mask=pattern.build_pattern(g, M).mask(), tol=1e-12, max_iter=2000)
        ws.append(float(np.einsum("ij,ij", eb, r.sigma_bar)))
    w_full = float(np.einsum("ij,ij", eb, full.sigma_bar))
    tol = 1e-9 * w_voigt
    assert w_reuss <= w_full + tol
    assert abs(ws[0] - w_voigt) < tol
    for a, b in zip(ws[1:], ws[:-1]):
        assert a <= b + tol
    assert w_full <= ws[-1] + tol


def test_plane_strain_bulk_bounds_full_solution():
    n = 64
    g = synth.disk(n, n, np.sqrt(0.3 * n * n / np.pi))
    e = 1e-3
    res = solver.solve(g, PH, solver.macro_tensor([e, e, 0], 2), tol=1e-12, max_iter=2000)
    k = (res.sigma_bar[0, 0] + res.sigma_bar[1, 1]) / (4 * e)
    lo, hi = bounds.plane_strain_bulk_bounds(PH, float(g.mean()))
    assert lo * (1 - 1e-6) <= k <= hi * (1 + 1e-6)


def _galerkin_direct(g, phases, eb, mask, kind):
    """Solve the reduced problem directly: eps = eps_bar + sum_m sym(n (x) a_m)
    e^{2 pi i m.x/N}/N, with equilibrium sigma^(m) n(m) = 0 on every pattern
    frequency (dense complex linear system, tiny grids only)."""
    shape = g.shape
    N = g.size
    idx = np.flatnonzero(mask.ravel())
    n, live = green.directions(shape, idx, kind)
    act = idx[live]
    nv = n[live]
    L = act.size
    ks = np.array(np.unravel_index(act, shape)).T
    xs = np.array(np.unravel_index(np.arange(N), shape)).T
    phase = np.exp(2j * np.pi * (xs / np.array(shape)) @ ks.T)  # [N, L]
    lam = np.where(g.ravel() > 0, phases[1].lam, phases[0].lam)
    mu = np.where(g.ravel() > 0, phases[1].mu, phases[0].mu)
    dim = g.ndim

    def stress_of(eps):  # eps [N,3,3]
        tr = np.trace(eps, axis1=1, axis2=2)
        return lam[:, None, None] * tr[:, None, None] * np.eye(3) + 2 * mu[:, None, None] * eps

    def residual(u):  # u [L, dim] complex -> equilibrium residual [L, dim]
        a = np.zeros((L, 3), complex)
        a[:, :dim] = u
        sym = 0.5 * (nv[:, :, None] * a[:, None, :] + a[:, :, None] * nv[:, None, :])
        eps = eb[None].astype(complex) + np.einsum("xl,lij->xij", phase, sym) / N
        sig = stress_of(eps)
        sh = np.einsum("xl,xij->lij", np.conj(phase), sig)
        return np.einsum("lij,lj->li", sh, nv)[:, :dim]

    b = -residual(np.zeros((L, dim), complex)).ravel()
    A = np.zeros((L * dim, L * dim), complex)
    for c in range(L * dim):
        e = np.zeros(L * dim, complex)
        e[c] = 1.0
        A[:, c] = residual(e.reshape(L, dim)).ravel() + b
    u = np.linalg.solve(A, b).reshape(L, dim)
    a = np.zeros((L, 3), complex)
    a[:, :dim] = u
    sym = 0.5 * (nv[:, :, None] * a[:, None, :] + a[:, :, None] * nv[:, None, :])
    eps = (eb[None] + np.einsum("xl,lij->xij", phase, sym) / N)
    assert np.max(np.abs(eps.imag)) < 1e-12
    sig = stress_of(eps.real)
    return eps.real.reshape(shape + (3, 3)), sig.mean(axis=0)


@pytest.mark.parametrize("kind", [green.ROTATED, green.CONTINUOUS])
@pytest.mark.parametrize("case", ["2d", "3d"])
def test_matches_direct_galerkin_solution(kind, case):
    rng = np.random.default_rng(7)
    if case == "2d":
        g = (rng.random((8, 10)) < 0.4).astype(np.uint8)
        eb = solver.macro_tensor([1e-3, -5e-4, 3e-4], 2)
        M = 23
    else:
        g = (rng.random((4, 6, 4)) < 0.4).astype(np.uint8)
        eb = solver.macro_tensor([1e-3, -5e-4, 2e-4, 1e-4, -3e-4, 3e-4], 3)
        M = 21
    mask = pattern.build_pattern(g, M).mask()
    res = solver.solve(g, PH, eb, mask=mask, tol=1e-14, max_iter=3000, gamma_kind=kind)
    assert res.converged
    eps_d, sbar_d = _galerkin_direct(g, PH, eb, mask, kind)
    assert np.max(np.abs(res.eps - eps_d)) < 1e-12
    assert np.max(np.abs(res.sigma_bar - sbar_d)) < 1e-10


def test_fields_are_real_and_hermitian():
    g = synth.rsa_fibres(32, 32, 3, 6, seed=9, target_vf=0.3).g
    eb = solver.macro_tensor([1e-3, 2e-4, -1e-4], 2)
    p = pattern.build_pattern(g, 103)
    res = solver.solve(g, PH, eb, mask=p.mask(), tol=1e-9)
    # the field lives on the pattern: its spectrum vanishes off the pattern
    sp = np.fft.fftn(res.eps - eb, axes=(0, 1))
    off = ~p.mask()
    assert np.max(np.abs(sp[off])) < 1e-15 * g.size


# ---------------------------------------------------------------- J2 pins

J2M = material.Phase(LM, MM, sigma_y0=0.25, H=1.0, plastic=True)


def test_j2_elastic_below_yield():
    eps = np.zeros((1, 3, 3))
    eps[0, 0, 0] = 1e-4
    s, ep, al = material.j2_return(eps, np.zeros_like(eps), np.zeros(1), J2M.lam, J2M.mu, J2M.sigma_y0, J2M.H, True)
    assert np.array_equal(s[0], _hooke_tensor_apply(J2M.lam, J2M.mu, eps[0]))
    assert al[0] == 0.0 and not ep.any()


def test_j2_return_consistency():
    rng = np.random.default_rng(3)
    for _ in range(50):
        e = rng.normal(size=(3, 3)) * 5e-3
        e = 0.5 * (e + e.T)
        ep0 = rng.normal(size=(3, 3)) * 1e-3
        ep0 = 0.5 * (ep0 + ep0.T)
        ep0 -= np.trace(ep0) / 3 * np.eye(3)
        a0 = abs(rng.normal()) * 1e-3
        s, ep, al = material.j2_return(e[None], ep0[None], np.array([a0]), J2M.lam, J2M.mu, 0.25, 1.0, True)
        q = material.von_mises(s)[0]
        sig_tr = _hooke_tensor_apply(J2M.lam, J2M.mu, e - ep0)
        q_tr = material.von_mises(sig_tr[None])[0]
        f_tr = q_tr - (0.25 + 1.0 * a0)
        if f_tr > 0:
            # on the updated yield surface, closed-form multiplier, deviatoric flow
            assert abs(q - (0.25 + 1.0 * al[0])) < 1e-12
            assert abs((al[0] - a0) - f_tr / (3 * J2M.mu + 1.0)) < 1e-15
            assert abs(np.trace(ep[0] - ep0)) < 1e-17
            # accumulated strain increment = sqrt(2/3) ||d eps_p||
            d = ep[0] - ep0
            assert abs(np.sqrt(2.0 / 3.0 * np.sum(d * d)) - (al[0] - a0)) < 1e-15
        else:
            assert al[0] == a0


def test_j2_uniaxial_stress_hardening_slope():
    # Uniaxial stress, monotonic loading: d sigma / d eps = E H / (E + H) after yield.
    E = synth.MATRIX_E
    nu = synth.MATRIX_NU
    lam, mu = synth.phase_lame(E, nu)
    H = 1.0
    state = (np.zeros((1, 3, 3)), np.zeros(1))
    pts = []
    for e11 in np.linspace(0.0, 0.02, 41)[1:]:
        # solve for lateral strain giving sigma22 = sigma33 = 0 by Newton on the return map
        el = -nu * e11
        for _ in range(60):
            def s_of(x):
                e = np.diag([e11, x, x])[None]
                return material.j2_return(e, state[0], state[1], lam, mu, 0.25, H, True)
            s = s_of(el)[0][0]
            h = 1e-9
            ds = (s_of(el + h)[0][0][1, 1] - s[1, 1]) / h
            el -= s[1, 1] / ds
        sig, ep, al = s_of(el)
        state = (ep, al)
        pts.append((e11, sig[0, 0, 0]))
    e = np.array(pts)
    slope = np.diff(e[-10:, 1]) / np.diff(e[-10:, 0])
    assert np.allclose(slope, E * H / (E + H), rtol=1e-5)


def test_homogeneous_j2_rve_matches_material_point():
    shape = (8, 8)
    g = np.zeros(shape, np.uint8)
    ph = (J2M, material.Phase(LI, MI))
    eb = solver.macro_tensor([0.02, 0.0, 0.0], 2)
    path = solver.solve_path(g, ph, eb, 10, tol=1e-12)
    ep = np.zeros((1, 3, 3))
    al = np.zeros(1)
    for n, res in enumerate(path, 1):
        assert res.iterations == 1
        s, ep, al = material.j2_return((eb * n / 10)[None], ep, al, J2M.lam, J2M.mu, 0.25, 1.0, True)
        assert np.max(np.abs(res.sigma_bar - s[0])) < 1e-13


# ---------------------------------------------------------------- compatibility step (Secs. 4.1, 5.1)
def test_compatibility_step_fixed_point_of_full_solution():
    """The full-set solution is the fixed point of the full scheme, so the
    compatibility step leaves it unchanged."""
    g = synth.disk(24, 24, 7.0)
    eb = solver.macro_tensor([1e-3, -4e-4, 3e-4], 2)
    full = solver.solve(g, PH, eb, tol=1e-14, max_iter=2000)
    c = solver.compatibility_step(g, PH, eb, full.eps)
    assert np.max(np.abs(c.eps - full.eps)) < 1e-12 * np.max(np.abs(full.eps)) * 1e3
    assert np.allclose(c.sigma_bar, full.sigma_bar, rtol=0, atol=1e-12 * np.abs(full.sigma_bar).max())
    assert c.residuals[0] < 1e-10


@pytest.mark.parametrize("dim", [2, 3])
def test_compatibility_step_contracts_towards_full_solution(dim):
    """One pass of the basic scheme contracts the distance to its fixed point
    (the full-set solution): the reduced solution moves closer to it in L2.
    A sign or index error in the pass would push it away."""
    if dim == 2:
        g = synth.rsa_fibres(32, 32, 3.0, 6.0, seed=9, target_vf=0.35).g
        eb = solver.macro_tensor([1e-3, -4e-4, 3e-4], 2)
    else:
        g = synth.rsa_spheres(12, 12, 12, 2.0, 3.0, seed=9, target_vf=0.2).g
        eb = solver.macro_tensor([1e-3, 0, -2e-4, 1e-4, 0, 3e-4], 3)
    N = g.size
    full = solver.solve(g, PH, eb, tol=1e-13, max_iter=3000)
    for M in (max(1, N // 50), N // 10):
        red = solver.solve(g, PH, eb, mask=pattern.build_pattern(g, M).mask(), tol=1e-13, max_iter=3000)
        c = solver.compatibility_step(g, PH, eb, red.eps)
        d_red = np.linalg.norm(red.eps - full.eps)
        d_c = np.linalg.norm(c.eps - full.eps)
        assert d_c < d_red
        assert np.allclose(c.eps.reshape(N, 3, 3).mean(axis=0), eb, atol=1e-15)


def test_compatibility_step_reference_medium_returns_macro_strain():
    """When both phases equal the reference medium, the polarisation is zero
    for any input field, so the step returns the macro strain everywhere
    (the input need not even be compatible)."""
    g = synth.disk(16, 16, 5.0)
    same = (material.Phase(LM, MM), material.Phase(LM, MM))
    eb = solver.macro_tensor([2e-3, 1e-3, -5e-4], 2)
    rng = np.random.default_rng(3)
    junk = rng.normal(size=g.shape + (3, 3))
    junk = 0.5 * (junk + np.swapaxes(junk, -1, -2))
    c = solver.compatibility_step(g, same, eb, junk)
    assert np.max(np.abs(c.eps - eb)) < 1e-15


# ---------------------------------------------------------------- error measures of Sec. 5
def test_macro_and_micro_error_hand_computed():
    """E_bar and E (Sec. 5) on hand-computed cases: a uniform 10 % scaling,
    and a two-point field whose values were worked out by hand."""
    ref = np.broadcast_to(np.diag([1.0, 2.0, 3.0]), (4, 5, 3, 3)).copy()
    assert abs(solver.macro_error(1.1 * ref.mean(axis=(0, 1)), ref.mean(axis=(0, 1))) - 0.1) < 1e-14
    assert abs(solver.micro_error(1.1 * ref, ref) - 0.1) < 1e-14
    r1 = np.zeros((3, 3)); r1[0, 0] = 1.0
    r2 = np.zeros((3, 3)); r2[0, 1] = r2[1, 0] = 1.0
    s1 = r1.copy(); s1[2, 2] = 1.0          # |s1 - r1| = 1, |r1| = 1      -> 1
    s2 = 0.5 * r2                             # |s2 - r2| = sqrt(2)/2, |r2| = sqrt(2) -> 0.5
    ref2 = np.stack([r1, r2])
    sig2 = np.stack([s1, s2])
    assert abs(solver.micro_error(sig2, ref2) - 0.75) < 1e-15
    # means: ref [[.5,.5,0],[.5,0,0],[0,0,0]] (norm^2 0.75), difference
    # [[0,-.25,0],[-.25,0,0],[0,0,.5]] (norm^2 0.375): E_bar = sqrt(1/2)
    assert abs(solver.macro_error(sig2.mean(axis=0), ref2.mean(axis=0)) - np.sqrt(0.5)) < 1e-15


def test_micro_error_skips_vanishing_reference_points():
    r = np.zeros((3, 3, 3))
    r[0, 0, 0] = 2.0
    r[1, 1, 1] = 4.0                          # point 2 has sigma_ref = 0: skipped
    s = r.copy()
    s[0, 0, 0] = 3.0                          # ratio 0.5
    s[2, 2, 2] = 7.0
    assert abs(solver.micro_error(s, r) - 0.25) < 1e-15
