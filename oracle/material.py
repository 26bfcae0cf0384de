"""Pointwise constitutive laws of the two phases (paper Sec. 2).

* Linear elasticity: sigma = C(x) : eps_e with isotropic C (lambda, mu).
* Elasto-plasticity: von Mises yield Phi = sigma_eq - [sigma_y0 + H * eps_acc],
  associative flow eps_p_dot = gamma_dot dPhi/dsigma and the KKT conditions.
  The paper states the model but not its integration; the oracle uses the
  textbook backward-Euler radial return (Simo & Hughes 1998, Box 3.1) with
  eps_acc the accumulated equivalent plastic strain (eps_acc_dot = gamma_dot).

Tensors are full 3x3 arrays [..., 3, 3] in FP64.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Phase:
    lam: float
    mu: float
    sigma_y0: float = 0.0
    H: float = 0.0
    plastic: bool = False


def hooke(eps: np.ndarray, lam, mu) -> np.ndarray:
    """sigma = lam tr(eps) I + 2 mu eps; lam and mu broadcast over the points."""
    lam = np.asarray(lam)[..., None, None]
    mu = np.asarray(mu)[..., None, None]
    tr = np.trace(eps, axis1=-2, axis2=-1)[..., None, None]
    return lam * tr * np.eye(3) + 2.0 * mu * eps


def point_params(g: np.ndarray, phases):
    """Per-point (lam, mu, sigma_y0, H, plastic) arrays from the phase indicator."""
    m, i = phases
    sel = g.astype(bool)
    lam = np.where(sel, i.lam, m.lam)
    mu = np.where(sel, i.mu, m.mu)
    sy = np.where(sel, i.sigma_y0, m.sigma_y0)
    H = np.where(sel, i.H, m.H)
    pl = np.where(sel, i.plastic, m.plastic)
    return lam, mu, sy, H, pl


def j2_return(eps, eps_p_n, alpha_n, lam, mu, sy, H, plastic):
    """Radial return for J2 with linear isotropic hardening.

    Returns (sigma, eps_p, alpha).  Points with plastic == False are elastic.
    """
    eps_e = eps - eps_p_n
    sig_tr = hooke(eps_e, lam, mu)
    tr = np.trace(sig_tr, axis1=-2, axis2=-1)[..., None, None]
    s_tr = sig_tr - tr / 3.0 * np.eye(3)
    norm_s = np.sqrt(np.einsum("...ij,...ij->...", s_tr, s_tr))
    q_tr = np.sqrt(1.5) * norm_s
    f = q_tr - (sy + H * alpha_n)
    yielding = plastic & (f > 0.0)
    dgam = np.where(yielding, f / (3.0 * mu + H), 0.0)
    safe = np.where(norm_s > 0.0, norm_s, 1.0)
    nhat = s_tr / safe[..., None, None]
    flow = (np.sqrt(1.5) * dgam)[..., None, None] * nhat
    sigma = sig_tr - 2.0 * np.asarray(mu)[..., None, None] * flow
    eps_p = eps_p_n + flow
    alpha = alpha_n + dgam
    return sigma, eps_p, alpha


def von_mises(sigma: np.ndarray) -> np.ndarray:
    tr = np.trace(sigma, axis1=-2, axis2=-1)[..., None, None]
    s = sigma - tr / 3.0 * np.eye(3)
    return np.sqrt(1.5 * np.einsum("...ij,...ij->...", s, s))
