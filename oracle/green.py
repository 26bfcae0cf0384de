"""Green operator of the homogeneous reference medium (paper Sec. 3, eqs. homoBVP,
LippmannSchwinger and Gamma).

For an isotropic reference stiffness C0 (Lame constants lambda0, mu0) and a
wave vector k, the acoustic tensor is K_ik = C0_ijkl k_j k_l, its inverse is
G^_ik, and the Green operator is the symmetrised product
    Gamma^_ijkl = 1/4 (G^_jk k_l k_i + G^_ik k_l k_j + G^_jl k_k k_i + G^_il k_k k_j),
so that eps^ = -Gamma^ : tau^ for k != 0 and eps^(0) = N * eps_bar.
(The paper's comma notation is read as this standard form, a reading of the
paper's garbled index notation.)  Gamma^ is homogeneous of degree 0 in k, so only the unit direction
n = k/|k| matters.

Wave vectors (paper Sec. 3, last paragraph, first-order finite differences):

* ``continuous``: n = s/|s| with s the signed centred frequency.  On an even
  axis the Nyquist index has no sign, so for an m that has a Nyquist component
  and is not its own conjugate, s(-m) != -s(m), Gamma^(m) != Gamma^(-m) and the
  iterate would not stay real; such modes are dropped (Gamma^ = 0) in this
  option.  Self-conjugate modes (every component 0 or N_a/2) are kept.
* ``rotated`` (default): the rotated first-order finite-difference scheme.
  Its discrete wave vector is a common complex factor times the real vector
  t_a = tan(pi m_a / N_a); hence n = t/|t|.  Where exactly one component sits
  at the Nyquist index N_a/2 the factor vanishes in every other component and
  n = e_a; with two or more Nyquist components the discrete wave vector is zero
  and the mode carries no strain (Gamma^ = 0).

All tensors are full 3x3 (2D: the third wave-vector component is zero).
"""
from __future__ import annotations

import numpy as np

ROTATED = "rotated"
CONTINUOUS = "continuous"


def stiffness(lam: float, mu: float) -> np.ndarray:
    """Isotropic 4th-order stiffness C_ijkl = lam d_ij d_kl + mu (d_ik d_jl + d_il d_jk)."""
    d = np.eye(3)
    return (lam * np.einsum("ij,kl->ijkl", d, d)
            + mu * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))


def directions(shape, freq_idx, kind: str = ROTATED):
    """Unit directions n [len(freq_idx), 3] and a 'live' flag per frequency.

    ``freq_idx`` are linear FFT indices on ``shape`` (C order).  live = False
    marks m = 0 and the dropped multi-Nyquist modes of the rotated scheme.
    """
    shape = tuple(shape)
    freq_idx = np.asarray(freq_idx, dtype=np.int64)
    ks = np.unravel_index(freq_idx, shape)
    nf = freq_idx.size
    n = np.zeros((nf, 3))
    live = np.ones(nf, dtype=bool)
    for i in range(nf):
        k = [int(ks[a][i]) for a in range(len(shape))]
        if all(v == 0 for v in k):
            live[i] = False
            continue
        if kind == CONTINUOUS:
            nyq = any(N % 2 == 0 and v == N // 2 for v, N in zip(k, shape))
            selfconj = all(v == 0 or (N % 2 == 0 and v == N // 2) for v, N in zip(k, shape))
            if nyq and not selfconj:
                live[i] = False
                continue
            s = np.array([v if v <= N // 2 else v - N for v, N in zip(k, shape)], dtype=np.float64)
            n[i, :len(shape)] = s / np.linalg.norm(s)
        elif kind == ROTATED:
            nyq = [a for a, (v, N) in enumerate(zip(k, shape)) if N % 2 == 0 and v == N // 2]
            if len(nyq) >= 2:
                live[i] = False
                continue
            if len(nyq) == 1:
                n[i, nyq[0]] = 1.0
                continue
            t = np.array([np.tan(np.pi * v / N) for v, N in zip(k, shape)])
            n[i, :len(shape)] = t / np.linalg.norm(t)
        else:
            raise ValueError(kind)
    return n, live


def gamma_tensor(n: np.ndarray, lam0: float, mu0: float) -> np.ndarray:
    """Gamma^_ijkl [F,3,3,3,3] from the definition (acoustic tensor inverse)."""
    C0 = stiffness(lam0, mu0)
    K = np.einsum("ijkl,fj,fl->fik", C0, n, n)
    G = np.linalg.inv(K)
    return 0.25 * (np.einsum("fjk,fl,fi->fijkl", G, n, n)
                   + np.einsum("fik,fl,fj->fijkl", G, n, n)
                   + np.einsum("fjl,fk,fi->fijkl", G, n, n)
                   + np.einsum("fil,fk,fj->fijkl", G, n, n))


def apply_gamma(Gam: np.ndarray, tau_hat: np.ndarray) -> np.ndarray:
    """eps^ = -Gamma^ : tau^ for tau_hat [F,3,3] (complex)."""
    return -np.einsum("fijkl,fkl->fij", Gam, tau_hat)
