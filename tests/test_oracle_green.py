"""Pins of the oracle's Green operator (paper Sec. 3, eq. Gamma) that do not
reuse its implementation: an independent closed form for isotropic C0, the
projection identities that define Gamma^, and the rotated finite-difference
wave vector evaluated from its complex symbol."""
import numpy as np
import pytest

from oracle import green

LAM0, MU0 = 75.7, 96.8


def _closed_form_apply(n, tau, lam, mu):
    # For isotropic C0 and unit n: G = (I - (lam+mu)/(lam+2mu) n n)/mu, hence
    # Gamma:tau = sym(n (x) G tau n) written out component-wise.
    v = tau @ n
    s = n @ v
    k = (lam + mu) / (mu * (lam + 2.0 * mu))
    return -((np.outer(n, v) + np.outer(v, n)) / (2.0 * mu) - k * s * np.outer(n, n))


def _rand_sym(rng, cplx=True):
    a = rng.normal(size=(3, 3)) + (1j * rng.normal(size=(3, 3)) if cplx else 0)
    return 0.5 * (a + a.T)


def test_definition_matches_closed_form():
    rng = np.random.default_rng(0)
    n = rng.normal(size=(50, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    Gam = green.gamma_tensor(n, LAM0, MU0)
    for f in range(50):
        tau = _rand_sym(rng)
        got = green.apply_gamma(Gam[f:f + 1], tau[None])[0]
        ref = _closed_form_apply(n[f], tau, LAM0, MU0)
        assert np.max(np.abs(got - ref)) < 1e-14 * max(1.0, np.max(np.abs(ref)))


def test_projection_identities():
    rng = np.random.default_rng(1)
    n = rng.normal(size=(20, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    Gam = green.gamma_tensor(n, LAM0, MU0)
    C0 = green.stiffness(LAM0, MU0)
    for f in range(20):
        G = Gam[f]
        GCG = np.einsum("ijab,abcd,cdkl->ijkl", G, C0, G)
        assert np.max(np.abs(GCG - G)) < 1e-15
        a = rng.normal(size=3)
        e = 0.5 * (np.outer(n[f], a) + np.outer(a, n[f]))
        back = np.einsum("ijkl,klab,ab->ij", G, C0, e)
        assert np.max(np.abs(back - e)) < 1e-14
        # an equilibrated polarisation (tau . n = 0) produces no strain
        t = _rand_sym(rng, cplx=False)
        P = np.eye(3) - np.outer(n[f], n[f])
        teq = P @ t @ P
        assert np.max(np.abs(np.einsum("ijkl,kl->ij", G, teq))) < 1e-15
        # Gamma is positive semi-definite on symmetric tensors
        assert np.einsum("ij,ijkl,kl->", t, G, t) >= -1e-15


def test_direction_symmetry_and_limit():
    shape = (64, 48)
    idx = np.arange(64 * 48)
    conj = ((-np.arange(64)[:, None]) % 64) * 48 + ((-np.arange(48)[None, :]) % 48)
    n, live = green.directions(shape, idx, green.ROTATED)
    nc, livec = green.directions(shape, conj.ravel(), green.ROTATED)
    # Gamma(-m) = Gamma(m): directions agree up to sign
    dots = np.abs(np.sum(n * nc, axis=1))
    assert np.all(dots[live] > 1 - 1e-14)
    assert np.array_equal(live, livec)
    # rotated -> continuous as |m|/N -> 0
    big = (256, 256)
    sel = np.array([1 * 256 + 1, 2 * 256 + 1, 1 * 256 + 3])
    nr, _ = green.directions(big, sel, green.ROTATED)
    ncn, _ = green.directions(big, sel, green.CONTINUOUS)
    assert np.max(np.abs(nr - ncn)) < 1e-3


def _complex_symbol(k, shape):
    # Rotated first-order finite-difference symbol, written with the identity
    # tan(x/2) (1 + e^{ix}) = 2 sin(x/2) e^{ix/2} so that it is finite at Nyquist.
    xi = [2 * np.pi * kk / n for kk, n in zip(k, shape)]
    fac = [1 + np.exp(1j * x) for x in xi]
    out = np.zeros(3, dtype=complex)
    for j in range(len(shape)):
        v = 1j * np.sin(xi[j] / 2) * np.exp(1j * xi[j] / 2)
        for m in range(len(shape)):
            if m != j:
                v *= fac[m]
        out[j] = v
    return out


def _gamma_from_symbol(kv, tau, lam, mu):
    # eps = sym(k (x) u), equilibrium with the adjoint symbol conj(k):
    # K_ik = C_ijkl conj(k_j) k_l,  u = -K^-1 (tau conj(k)).
    C0 = green.stiffness(lam, mu)
    K = np.einsum("ijkl,j,l->ik", C0, np.conj(kv), kv)
    u = -np.linalg.solve(K, tau @ np.conj(kv))
    return 0.5 * (np.outer(kv, u) + np.outer(u, kv))


@pytest.mark.parametrize("shape", [(8, 8), (6, 10), (4, 6, 8)])
def test_rotated_direction_rule_matches_symbol(shape):
    rng = np.random.default_rng(2)
    N = int(np.prod(shape))
    idx = np.arange(N)
    n, live = green.directions(shape, idx, green.ROTATED)
    Gam = green.gamma_tensor(n[live], LAM0, MU0)
    li = np.flatnonzero(live)
    ks = np.unravel_index(idx, shape)
    pos = {int(f): j for j, f in enumerate(li)}
    for f in range(N):
        k = [int(ks[a][f]) for a in range(len(shape))]
        kv = _complex_symbol(k, shape)
        if not live[f]:
            # m = 0 or >= 2 Nyquist components: the discrete wave vector vanishes
            assert np.max(np.abs(kv)) < 1e-15
            continue
        tau = _rand_sym(rng)
        ref = _gamma_from_symbol(kv, tau, LAM0, MU0)
        got = green.apply_gamma(Gam[pos[f]:pos[f] + 1], tau[None])[0]
        assert np.max(np.abs(got - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))
