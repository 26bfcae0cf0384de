"""Geometrically adapted sampling pattern (paper Sec. 4.2, Figs. GeoRealFourier /
SamplingReduced): FFT of the binary phase indicator g, then keep the given
fraction R of frequencies with the highest amplitudes |g^(xi)|.

The paper is silent on ties, conjugate pairs, xi = 0, the rounding of R*N and
floating-point noise.  The oracle fixes them as follows (listed in the design doc):

1. M = ceil(R*N) is passed in directly as an integer.
2. P(m) = |FFT(g)(m)|^2 in FP64 (unnormalised forward DFT, e^{-2 pi i m.x/N}),
   with P(0) = (number of inclusion voxels)^2 taken exactly.
3. key(m) = 0 if P(m) <= 2^-80 P(0) (flushes FFT noise at exact zeros), else
   float32_round_nearest_even(P(m) / P(0)); g == 0 gives all keys 0.
4. Pairs {m, -m} are ranked as units: key descending, then |s(m)|^2 ascending
   (s = signed centred frequency, N/2 counted as +N/2), then the lexicographic
   rank of the pair representative ascending.  The representative is the
   member with the smaller lexicographic rank, where
   lexrank(m) = mixed radix over axes (axis 0 most significant) of
   u_a = s_a + (N_a - 1) // 2.
5. Pairs are taken whole, in rank order, until at least M frequencies are in;
   a self-conjugate m (every component 0 or N/2) counts once.  M' = M or M+1.
6. xi = 0 is always in (it has key 1 and |s|^2 = 0, so it ranks first).
7. The pattern is the sorted list of linear FFT indices; ``rank_idx`` lists the
   same frequencies in selection order (representative, then its partner).
8. ``unstable`` is set when some frequency's FP64 ratio P/P(0) lies within a
   relative 1e-10 of a rounding boundary of the cut key's float32 interval (or
   of the 2^-80 flush threshold when the cut key is 0): an independent FP64
   spectrum could then round to a different key and select another set.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

FLUSH = 2.0 ** -80
UNSTABLE_REL = 1e-10


@dataclass
class Pattern:
    shape: tuple
    M: int                  # requested count
    sorted_idx: np.ndarray  # int64 [M'] linear FFT indices, ascending
    rank_idx: np.ndarray    # int64 [M'] same set, in selection order
    keys: np.ndarray        # float32 [N] key of every frequency
    unstable: bool

    @property
    def M_actual(self) -> int:
        return int(self.sorted_idx.size)

    def mask(self) -> np.ndarray:
        m = np.zeros(int(np.prod(self.shape)), dtype=bool)
        m[self.sorted_idx] = True
        return m.reshape(self.shape)


def signed_freq(k: np.ndarray, n: int) -> np.ndarray:
    """Signed centred frequency of FFT index k on a period-n axis; n/2 -> +n/2."""
    k = np.asarray(k)
    return np.where(k <= n // 2, k, k - n)


def power_spectrum(g: np.ndarray) -> np.ndarray:
    """P(m) = |g^(m)|^2, FP64, with P(0) replaced by the exact count^2."""
    gh = np.fft.fftn(g.astype(np.float64))
    P = gh.real * gh.real + gh.imag * gh.imag
    cnt = float(int(g.astype(np.int64).sum()))
    P.flat[0] = cnt * cnt
    return P


def spectrum_keys(g: np.ndarray):
    """(keys float32 [shape], ratio float64 [shape]) of the amplitude ranking."""
    P = power_spectrum(g)
    P0 = P.flat[0]
    if P0 == 0.0:
        z = np.zeros(g.shape, dtype=np.float64)
        return z.astype(np.float32), z
    ratio = P / P0
    keys = np.where(P <= FLUSH * P0, 0.0, ratio).astype(np.float32)
    return keys, ratio


def _coords(shape):
    """Per-frequency integer index arrays k_a, flattened in C order."""
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    return [gr.ravel() for gr in grids]


def _lexrank(s_list, shape):
    r = np.zeros_like(s_list[0], dtype=np.int64)
    for s, n in zip(s_list, shape):
        r = r * n + (s + (n - 1) // 2)
    return r


def conjugate_index(shape) -> np.ndarray:
    """Linear index of -m for every linear index m."""
    ks = _coords(shape)
    neg = [(-k) % n for k, n in zip(ks, shape)]
    lin = np.zeros_like(neg[0], dtype=np.int64)
    for k, n in zip(neg, shape):
        lin = lin * n + k
    return lin


def build_pattern(g: np.ndarray, M: int) -> Pattern:
    """Adapted pattern of ``M`` frequencies (pair-closed, so M' in {M, M+1})."""
    shape = tuple(int(n) for n in g.shape)
    N = int(np.prod(shape))
    if not 1 <= M <= N:
        raise ValueError("M must lie in [1, N]")
    keys, ratio = spectrum_keys(g)
    kf = keys.ravel()
    ks = _coords(shape)
    s = [signed_freq(k, n) for k, n in zip(ks, shape)]
    s2 = np.zeros(N, dtype=np.int64)
    for sa in s:
        s2 += sa.astype(np.int64) ** 2
    lex = _lexrank(s, shape)
    conj = conjugate_index(shape)
    lex_conj = lex[conj]
    lin = np.arange(N, dtype=np.int64)
    # one entry per pair: the representative (smaller lexrank; self-conjugate -> itself)
    is_rep = (lex <= lex_conj)
    reps = lin[is_rep]
    # Ranking: key descending, |s|^2 ascending, lexrank ascending (np.lexsort: last key primary).
    order = np.lexsort((lex[reps], s2[reps], -kf[reps].astype(np.float64)))
    reps = reps[order]
    sizes = np.where(conj[reps] == reps, 1, 2)
    csum = np.cumsum(sizes)
    npairs = int(np.searchsorted(csum, M) + 1)
    chosen = reps[:npairs]
    partner = conj[chosen]
    rank = []
    for a, b in zip(chosen.tolist(), partner.tolist()):
        rank.append(a)
        if b != a:
            rank.append(b)
    rank_idx = np.asarray(rank, dtype=np.int64)
    sorted_idx = np.sort(rank_idx)
    unstable = _unstable_cut(kf, ratio.ravel(), kf[chosen[-1]])
    return Pattern(shape=shape, M=M, sorted_idx=sorted_idx, rank_idx=rank_idx,
                   keys=keys, unstable=unstable)


def _unstable_cut(keys, ratio, cut_key) -> bool:
    """True if a float32 rounding boundary next to the cut key is within reach."""
    ck = np.float32(cut_key)
    if ck == 0.0:
        bounds = [FLUSH]
    else:
        lo = np.nextafter(ck, np.float32(0.0))
        hi = np.nextafter(ck, np.float32(np.inf))
        bounds = [(float(lo) + float(ck)) / 2.0, (float(ck) + float(hi)) / 2.0]
    for b in bounds:
        if np.any(np.abs(ratio - b) <= UNSTABLE_REL * b):
            return True
    return False
