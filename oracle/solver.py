"""Basic fixed-point scheme of Moulinec and Suquet with a full or reduced set of
frequencies (paper Sec. 3 and the reduced scheme a)-d) of Sec. 4).

Per iteration i (all in FP64, full 3x3 tensors, unnormalised forward FFT):
  a) tau = sigma(eps^i) - C0 : eps^i at every grid point,
  b) tau^ = FFT(tau),
  c) eps^(m) = -Gamma^(m) : tau^(m) for m in the pattern, m != 0;
     eps^(0) = N eps_bar; eps^ = 0 off the pattern,
  d) eps^{i+1} = Re iFFT(eps^).
Convergence (a reading: the paper's loop condition and norms disagree): after producing eps^{i+1},
  r = sqrt(mean_x ||eps^{i+1} - eps^i||_F^2) / ||eps_bar||_F
(denominator 1 if eps_bar = 0), stop at the first r < tol; the iteration count
is the number of Green-operator applications.  Finally sigma = sigma(eps_final)
by one more constitutive evaluation and sigma_bar is its grid mean (paper
Sec. 2, volume averages).  The reference medium is the arithmetic mean of the
two phases' Lame constants (Sec. 3).  ``mask = None`` is the full set; the
reduced scheme with every frequency selected is the same code path.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import green, material

_VOIGT2 = [(0, 0), (1, 1), (0, 1)]
_VOIGT3 = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


def comp_pairs(dim: int):
    """Component order of macro strains: 2D [11,22,12], 3D [11,22,33,23,13,12]."""
    return _VOIGT2 if dim == 2 else _VOIGT3


def macro_tensor(comps, dim: int) -> np.ndarray:
    """3x3 symmetric tensor from the component list (tensor shear components)."""
    e = np.zeros((3, 3))
    for v, (i, j) in zip(comps, comp_pairs(dim)):
        e[i, j] = v
        e[j, i] = v
    return e


def tensor_comps(t: np.ndarray, dim: int, with_s33: bool = False) -> np.ndarray:
    """Component list of a (field of) 3x3 tensor(s); 2D may append the 33 entry."""
    out = [t[..., i, j] for (i, j) in comp_pairs(dim)]
    if dim == 2 and with_s33:
        out.append(t[..., 2, 2])
    return np.stack(out, axis=-1)


def reference_medium(phases):
    """C0 from the arithmetic mean of the phase Lame constants."""
    m, i = phases
    return 0.5 * (m.lam + i.lam), 0.5 * (m.mu + i.mu)


@dataclass
class Result:
    eps: np.ndarray
    sigma: np.ndarray
    sigma_bar: np.ndarray
    iterations: int
    converged: bool
    residuals: list = field(default_factory=list)
    eps_p: np.ndarray | None = None
    alpha: np.ndarray | None = None


def _constitutive(eps, params, state):
    lam, mu, sy, H, pl = params
    if state is None:
        return material.hooke(eps, lam, mu), None, None
    sig, ep, al = material.j2_return(eps, state[0], state[1], lam, mu, sy, H, pl)
    return sig, ep, al


def _frob_rms(d: np.ndarray) -> float:
    return float(np.sqrt(np.mean(np.einsum("...ij,...ij->...", d, d))))


def solve(g, phases, eps_bar, mask=None, tol=1e-8, max_iter=1000, gamma_kind=green.ROTATED,
          eps0=None, state=None, C0=None) -> Result:
    """One solve of the (reduced) basic scheme.

    g: uint8 phase map (2D or 3D); phases: (matrix, inclusion) material.Phase;
    eps_bar: 3x3 macro strain; mask: bool array of the frequency grid or None;
    eps0: initial strain field [*shape,3,3] (default: eps_bar everywhere);
    state: committed J2 state (eps_p [*shape,3,3], alpha [*shape]) or None for
    purely elastic phases.
    """
    shape = g.shape
    dim = g.ndim
    axes = tuple(range(dim))
    N = int(np.prod(shape))
    if C0 is None:
        C0 = reference_medium(phases)
    lam0, mu0 = C0
    C0t = green.stiffness(lam0, mu0)
    params = material.point_params(g, phases)
    if state is None and (phases[0].plastic or phases[1].plastic):
        state = (np.zeros(shape + (3, 3)), np.zeros(shape))
    if mask is None:
        idx = np.arange(N)
    else:
        idx = np.flatnonzero(np.asarray(mask).ravel())
    n, live = green.directions(shape, idx, gamma_kind)
    act = idx[live]
    Gam = green.gamma_tensor(n[live], lam0, mu0)
    eb_norm = float(np.linalg.norm(eps_bar))
    denom = eb_norm if eb_norm > 0.0 else 1.0
    eps = np.broadcast_to(eps_bar, shape + (3, 3)).copy() if eps0 is None else np.array(eps0, dtype=np.float64)
    residuals = []
    converged = False
    it = 0
    while it < max_iter:
        sig, _, _ = _constitutive(eps, params, state)
        tau = sig - np.einsum("ijkl,...kl->...ij", C0t, eps)
        tau_hat = np.fft.fftn(tau, axes=axes).reshape(N, 3, 3)
        eps_hat = np.zeros((N, 3, 3), dtype=np.complex128)
        eps_hat[act] = green.apply_gamma(Gam, tau_hat[act])
        eps_hat[0] = N * eps_bar
        eps_new = np.fft.ifftn(eps_hat.reshape(shape + (3, 3)), axes=axes).real
        r = _frob_rms(eps_new - eps) / denom
        eps = eps_new
        it += 1
        residuals.append(r)
        if r < tol:
            converged = True
            break
    sig, ep, al = _constitutive(eps, params, state)
    sigma_bar = sig.reshape(N, 3, 3).mean(axis=0)
    return Result(eps=eps, sigma=sig, sigma_bar=sigma_bar, iterations=it, converged=converged,
                  residuals=residuals, eps_p=ep, alpha=al)


def solve_path(g, phases, eps_bar_final, steps, mask=None, tol=1e-8, max_iter=1000,
               gamma_kind=green.ROTATED, C0=None):
    """Load path with ``steps`` equal increments eps_bar_n = (n/steps) eps_bar_final.

    Step n starts from the converged strain of step n-1 plus the macro increment,
    with the committed J2 state of step n-1 held fixed during its iterations;
    the state of the final constitutive evaluation is committed.
    """
    shape = g.shape
    state = (np.zeros(shape + (3, 3)), np.zeros(shape))
    eps = None
    prev_bar = np.zeros((3, 3))
    out = []
    for n in range(1, steps + 1):
        bar = eps_bar_final * (n / steps)
        eps0 = None if eps is None else eps + (bar - prev_bar)
        res = solve(g, phases, bar, mask=mask, tol=tol, max_iter=max_iter, gamma_kind=gamma_kind,
                    eps0=eps0, state=state, C0=C0)
        out.append(res)
        state = (res.eps_p, res.alpha)
        eps = res.eps
        prev_bar = bar
    return out


def compatibility_step(g, phases, eps_bar, eps_red, state=None, gamma_kind=green.ROTATED, C0=None) -> Result:
    """Compatibility step (paper Sec. 4.1 post-processing, applied alone to the
    adapted-pattern solutions in Sec. 5.1): the Lippmann-Schwinger equation is
    solved once on the full set of frequencies from the fields of a reduced
    solution, i.e. one pass of steps a)-d) with every frequency kept,
    starting from eps_red:
      tau = sigma(eps_red) - C0 : eps_red,  eps^(xi) = -Gamma^(xi) : tau^(xi)
      (xi != 0),  eps^(0) = N eps_bar,  eps_comp = iFFT(eps^),
    followed by sigma(eps_comp) and its grid mean.  ``state`` is the committed
    J2 state the reduced solution was computed with (None: virgin material);
    it is used, not updated.  ``residuals[0]`` is the RMS change
    ||eps_comp - eps_red|| / ||eps_bar||."""
    r = solve(g, phases, eps_bar, mask=None, tol=0.0, max_iter=1, gamma_kind=gamma_kind, eps0=eps_red,
              state=state, C0=C0)
    r.eps_p = None
    r.alpha = None
    return r


def macro_error(sigma_bar, sigma_bar_ref) -> float:
    """E_bar = ||sigma_bar - sigma_bar_ref|| / ||sigma_bar_ref|| (paper Sec. 5)."""
    return float(np.linalg.norm(sigma_bar - sigma_bar_ref) / np.linalg.norm(sigma_bar_ref))


def micro_error(sigma, sigma_ref, skip_rel: float = 1e-12) -> float:
    """E = mean over points of ||sigma - sigma_ref|| / ||sigma_ref|| (paper Sec. 5).

    Points with ||sigma_ref|| below skip_rel * max are skipped (the definition
    divides by a pointwise norm that may vanish).
    """
    d = np.sqrt(np.einsum("...ij,...ij->...", sigma - sigma_ref, sigma - sigma_ref)).ravel()
    r = np.sqrt(np.einsum("...ij,...ij->...", sigma_ref, sigma_ref)).ravel()
    keep = r > skip_rel * r.max()
    return float(np.mean(d[keep] / r[keep]))
