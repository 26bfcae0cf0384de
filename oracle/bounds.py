"""Closed-form results that pin the solver independently of its iteration.

* Voigt / Reuss: the energy of every kinematically admissible strain field is
  bounded by the uniform-strain and uniform-stress estimates.  In plane strain
  the 2D problem has the in-plane stiffness C_ab cd, so both bounds use it.
* Laminate (g depends on x along axis 0 only): traction continuity across the
  layers plus compatibility of the tangential strains give the exact,
  piecewise constant solution (textbook).
* Plane-strain bulk modulus k = lambda + mu: Hill / Hashin bounds for fibre
  composites of arbitrary transverse geometry under equi-biaxial strain.
These are not taken from the paper (which prints no closed forms); they are the
mathematics the paper's discretised problem must reproduce.
"""
from __future__ import annotations

import numpy as np

from .green import stiffness

_M6 = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
_M3 = [(0, 0), (1, 1), (0, 1)]


def _mandel(C, pairs):
    n = len(pairs)
    A = np.zeros((n, n))
    for a, (i, j) in enumerate(pairs):
        for b, (k, l) in enumerate(pairs):
            wa = 1.0 if i == j else np.sqrt(2.0)
            wb = 1.0 if k == l else np.sqrt(2.0)
            A[a, b] = C[i, j, k, l] * wa * wb
    return A


def _vec(e, pairs):
    return np.array([e[i, j] * (1.0 if i == j else np.sqrt(2.0)) for (i, j) in pairs])


def voigt_reuss_energy(phases, vf_incl: float, eps_bar: np.ndarray, dim: int):
    """(W_reuss, W_voigt) with W = eps_bar : C_eff : eps_bar."""
    pairs = _M3 if dim == 2 else _M6
    Cm = _mandel(stiffness(phases[0].lam, phases[0].mu), pairs)
    Ci = _mandel(stiffness(phases[1].lam, phases[1].mu), pairs)
    f = vf_incl
    CV = (1.0 - f) * Cm + f * Ci
    CR = np.linalg.inv((1.0 - f) * np.linalg.inv(Cm) + f * np.linalg.inv(Ci))
    e = _vec(eps_bar, pairs)
    return float(e @ CR @ e), float(e @ CV @ e)


def voigt_stress(phases, vf_incl: float, eps_bar: np.ndarray) -> np.ndarray:
    """sigma_bar = <C> : eps_bar (uniform strain), full 3x3."""
    f = vf_incl
    C = (1.0 - f) * stiffness(phases[0].lam, phases[0].mu) + f * stiffness(phases[1].lam, phases[1].mu)
    return np.einsum("ijkl,kl->ij", C, eps_bar)


def laminate_fields(g_profile: np.ndarray, phases, eps_bar: np.ndarray):
    """Exact laminate solution for layers normal to axis 0.

    g_profile: phase indicator along axis 0 (length N0).  Returns
    (eps [N0,3,3], sigma [N0,3,3], sigma_bar [3,3]) per layer position.
    """
    g_profile = np.asarray(g_profile).astype(bool)
    f_i = g_profile.mean()
    fr = [1.0 - f_i, f_i]
    lam = [p.lam for p in phases]
    mu = [p.mu for p in phases]
    Mp = [l + 2.0 * m for l, m in zip(lam, mu)]
    et = eps_bar[1, 1] + eps_bar[2, 2]
    S = (eps_bar[0, 0] + et * sum(f * l / M for f, l, M in zip(fr, lam, Mp))) / sum(f / M for f, M in zip(fr, Mp))
    T12 = eps_bar[0, 1] / sum(f / (2.0 * m) for f, m in zip(fr, mu))
    T13 = eps_bar[0, 2] / sum(f / (2.0 * m) for f, m in zip(fr, mu))
    eps_p, sig_p = [], []
    for p in range(2):
        e = eps_bar.copy()
        e[0, 0] = (S - lam[p] * et) / Mp[p]
        e[0, 1] = e[1, 0] = T12 / (2.0 * mu[p])
        e[0, 2] = e[2, 0] = T13 / (2.0 * mu[p])
        s = lam[p] * np.trace(e) * np.eye(3) + 2.0 * mu[p] * e
        eps_p.append(e)
        sig_p.append(s)
    eps = np.where(g_profile[:, None, None], eps_p[1], eps_p[0])
    sig = np.where(g_profile[:, None, None], sig_p[1], sig_p[0])
    sigma_bar = fr[0] * sig_p[0] + fr[1] * sig_p[1]
    return eps, sig, sigma_bar


def plane_strain_bulk_bounds(phases, vf_incl: float):
    """(k_lower, k_upper) for k = lambda + mu of a two-phase fibre composite.

    Requires well-ordered phases (inclusion stiffer in k and mu).
    """
    km = phases[0].lam + phases[0].mu
    ki = phases[1].lam + phases[1].mu
    mm, mi = phases[0].mu, phases[1].mu
    fi, fm = vf_incl, 1.0 - vf_incl
    lo = km + fi / (1.0 / (ki - km) + fm / (km + mm))
    hi = ki + fm / (1.0 / (km - ki) + fi / (ki + mi))
    return lo, hi
