"""Geometrically adapted sampling pattern (paper Sec. 4.2, Figs. GeoRealFourier /
SamplingReduced): FFT of the binary phase indicator g, then keep the given
fraction R of frequencies with the highest amplitudes |g^(xi)|.  Also the
fixed radial pattern it is compared with (Sec. 4.1, fig. FixedSampling):
straight lines through xi = 0 at equally spaced angles, independent of g.

The paper is silent on ties, conjugate pairs, xi = 0, the rounding of R*N and
floating-point noise.  The oracle fixes them as follows (readings, not the paper's statements):

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


# ---------------------------------------------------------------- fixed radial pattern
RADIAL_TIE_MARGIN = 1e-9


def _round_half_away(x: np.ndarray) -> np.ndarray:
    """Nearest integer, halves away from zero (odd-symmetric: r(-x) = -r(x))."""
    return np.sign(x) * np.floor(np.abs(x) + 0.5)


def radial_lines(shape, L: int):
    """Signed frequencies (s0, s1) of the fixed radial sampling pattern with L
    straight lines through xi = 0 (paper Sec. 4.1, fig. FixedSampling; the
    paper does not give the rasterisation, so this is a reading):

    line l = 0..L-1 has the angle theta_l = l pi / L, measured from the axis-1
    direction towards axis 0.  A line with theta in [0, pi/4] or [3 pi/4, pi)
    (integer test 4l <= L or 4l >= 3L) advances one step along axis 1 at a
    time: s1 = -(n1/2 - 1) .. n1/2 - 1 and s0 = round(s1 tan theta).  The
    other lines advance along axis 0: s0 = -(n0/2 - 1) .. n0/2 - 1 and
    s1 = round(s0 tan(pi/2 - theta)).  round = nearest, halves away from
    zero; points beyond |s_a| <= n_a/2 - 1 are dropped.  The Nyquist index
    n_a/2 is never used, so every line is closed under m -> -m.

    Returns (s0, s1, margin): the points (with repeats) and the smallest
    distance of any rounded product from a half-integer (rounding ties do not
    occur: tan(l pi / L) is irrational unless it is 0 or +-1)."""
    n0, n1 = int(shape[0]), int(shape[1])
    h0, h1 = n0 // 2 - 1, n1 // 2 - 1
    S0, S1 = [], []
    margin = np.inf
    for l in range(int(L)):
        if 4 * l <= L or 4 * l >= 3 * L:
            u = np.arange(-h1, h1 + 1, dtype=np.float64)
            x = u * np.tan(np.pi * l / L)
            v = _round_half_away(x)
            keep = np.abs(v) <= h0
            S0.append(v[keep].astype(np.int64))
            S1.append(u[keep].astype(np.int64))
        else:
            u = np.arange(-h0, h0 + 1, dtype=np.float64)
            x = u * np.tan(np.pi * (L - 2 * l) / (2 * L))
            v = _round_half_away(x)
            keep = np.abs(v) <= h1
            S0.append(u[keep].astype(np.int64))
            S1.append(v[keep].astype(np.int64))
        frac = np.abs(x - np.floor(x) - 0.5)
        margin = min(margin, float(frac.min()) if frac.size else np.inf)
    return np.concatenate(S0), np.concatenate(S1), margin


def build_radial_pattern(shape, L: int) -> Pattern:
    """Fixed radial pattern of L lines (2D only; Sec. 4.1).  The pattern does
    not depend on the microstructure.  Its rank order (``rank_idx``, used for
    the warm-start slots) is the adapted ranking with every selected
    frequency given the same key: pairs by |s|^2 ascending, then lexrank of
    the representative.  ``unstable`` flags a rounding product within
    RADIAL_TIE_MARGIN of a half-integer."""
    shape = tuple(int(n) for n in shape)
    if len(shape) != 2:
        raise ValueError("the radial pattern is defined for 2D grids")
    if L < 1:
        raise ValueError("L must be >= 1")
    n0, n1 = shape
    N = n0 * n1
    s0, s1, margin = radial_lines(shape, L)
    sel = np.zeros(N, dtype=bool)
    sel[(s0 % n0) * n1 + (s1 % n1)] = True
    ks = _coords(shape)
    s = [signed_freq(k, n) for k, n in zip(ks, shape)]
    s2 = s[0].astype(np.int64) ** 2 + s[1].astype(np.int64) ** 2
    lex = _lexrank(s, shape)
    conj = conjugate_index(shape)
    lin = np.arange(N, dtype=np.int64)
    if not np.array_equal(sel, sel[conj]):
        raise AssertionError("radial pattern not closed under m -> -m")
    reps = lin[sel & (lex <= lex[conj])]
    reps = reps[np.lexsort((lex[reps], s2[reps]))]
    rank = []
    for a in reps.tolist():
        rank.append(a)
        if conj[a] != a:
            rank.append(int(conj[a]))
    rank_idx = np.asarray(rank, dtype=np.int64)
    keys = sel.astype(np.float32).reshape(shape)
    M = int(rank_idx.size)
    return Pattern(shape=shape, M=M, sorted_idx=np.sort(rank_idx), rank_idx=rank_idx, keys=keys,
                   unstable=bool(margin < RADIAL_TIE_MARGIN))
