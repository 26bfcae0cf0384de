"""Pins of the adapted sampling pattern (paper Sec. 4.2): a brute-force
selection from a directly summed DFT on tiny grids, and properties the paper
states or the construction implies (symmetry, nestedness, anisotropy of the
ellipse pattern, independence of material data, degenerate geometries)."""
import itertools
import math

import numpy as np
import pytest

import synth
from oracle import pattern


def _brute_pattern(g, M):
    # Independent of the oracle: O(N^2) DFT by direct summation, python tuples
    # for the ranking, explicit pair bookkeeping.
    shape = g.shape
    pts = list(itertools.product(*[range(n) for n in shape]))
    cnt = int(g.sum())
    entries = {}
    for m in pts:
        acc = 0j
        for x in pts:
            if g[x]:
                ph = sum(mi * xi / n for mi, xi, n in zip(m, x, shape))
                acc += complex(math.cos(2 * math.pi * ph), -math.sin(2 * math.pi * ph))
        P = acc.real ** 2 + acc.imag ** 2
        if all(v == 0 for v in m):
            P = float(cnt * cnt)
        if cnt == 0 or P <= 2.0 ** -80 * cnt * cnt:
            key = 0.0
        else:
            key = float(np.float32(P / (cnt * cnt)))
        entries[m] = key

    def signed(v, n):
        return v if v <= n // 2 else v - n

    def lexrank(m):
        r = 0
        for v, n in zip(m, shape):
            r = r * n + signed(v, n) + (n - 1) // 2
        return r

    seen, pairs = set(), []
    for m in pts:
        if m in seen:
            continue
        c = tuple((-v) % n for v, n in zip(m, shape))
        seen.add(m)
        seen.add(c)
        rep = m if lexrank(m) <= lexrank(c) else c
        s2 = sum(signed(v, n) ** 2 for v, n in zip(rep, shape))
        members = [rep] if c == m else [rep, c if rep == m else m]
        pairs.append(((-entries[rep], s2, lexrank(rep)), members))
    pairs.sort(key=lambda p: p[0])
    chosen, count = [], 0
    for _, mem in pairs:
        if count >= M:
            break
        chosen.extend(mem)
        count += len(mem)
    lin = sorted(int(np.ravel_multi_index(m, shape)) for m in chosen)
    return np.array(lin)


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_small_grids(seed):
    rng = np.random.default_rng(100 + seed)
    shape = [(8, 8), (12, 12), (10, 16), (16, 16), (6, 8), (4, 4, 6)][seed]
    g = (rng.random(shape) < 0.35).astype(np.uint8)
    N = int(np.prod(shape))
    for M in sorted({1, 2, 3, N // 20 + 1, N // 7, N // 3, N - 1, N}):
        p = pattern.build_pattern(g, M)
        if p.unstable:
            continue
        ref = _brute_pattern(g, M)
        assert np.array_equal(p.sorted_idx, ref), (shape, M)


def test_symmetric_disk_ties_are_resolved_deterministically():
    g = synth.disk(16, 16, 5.0)
    for M in range(1, 60):
        p = pattern.build_pattern(g, M)
        if p.unstable:
            continue
        assert np.array_equal(p.sorted_idx, _brute_pattern(g, M))


def test_pair_closure_zero_first_and_count():
    g, _ = synth.metric_rve(3, n=64)
    N = g.size
    conj = pattern.conjugate_index(g.shape)
    for M in [1, 2, 5, 50, 205, 1000, N]:
        p = pattern.build_pattern(g, M)
        s = set(p.sorted_idx.tolist())
        assert p.rank_idx[0] == 0
        assert all(int(conj[i]) in s for i in s)
        assert p.M_actual in (M, M + 1)
        assert np.array_equal(np.sort(p.rank_idx), p.sorted_idx)


def test_nested_in_M():
    g = synth.rsa_fibres(64, 64, 4, 8, seed=5, target_vf=0.3).g
    prev = set()
    for M in [1, 10, 50, 205, 600, 2000]:
        cur = set(pattern.build_pattern(g, M).sorted_idx.tolist())
        assert prev <= cur
        prev = cur


def test_disk_pattern_square_symmetry_up_to_cut_orbit():
    n = 64
    g = synth.disk(n, n, 12.3)
    p = pattern.build_pattern(g, 205)
    mask = p.mask()
    keys = p.keys
    cut = keys.ravel()[p.rank_idx[-1]]
    k0, k1 = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    for (a, b) in [(k1, k0), ((-k0) % n, k1), (k0, (-k1) % n)]:
        img = mask[a, b]
        diff = img != mask
        # only frequencies in the tie class at the cut may break the symmetry
        assert np.all(keys[diff] == cut)


def test_ellipse_pattern_is_anisotropic():
    # An ellipse elongated along axis 0 is narrow along axis 1: its spectrum,
    # and so the pattern, reaches further along frequency axis 1.
    n = 128
    g = synth.ellipse(n, n, 40.0, 12.0)
    p = pattern.build_pattern(g, int(math.ceil(0.0154 * n * n)))
    k0, k1 = np.unravel_index(p.sorted_idx, g.shape)
    s0 = np.abs(pattern.signed_freq(k0, n))
    s1 = np.abs(pattern.signed_freq(k1, n))
    assert s1.max() > 1.5 * s0.max()


def test_degenerate_geometries():
    n = 16
    N = n * n
    for g in [np.zeros((n, n), np.uint8), np.ones((n, n), np.uint8)]:
        keys, _ = pattern.spectrum_keys(g)
        if g.any():
            assert keys.ravel()[0] == 1.0 and np.all(keys.ravel()[1:] == 0.0)
        else:
            assert np.all(keys == 0.0)
        p = pattern.build_pattern(g, 9)
        # all keys (beyond xi=0) tie at zero: the ranking is by |s|^2, then lexrank
        s = pattern.signed_freq(np.array(np.unravel_index(p.sorted_idx, g.shape)), n)
        assert np.max(np.sum(s * s, axis=0)) <= 2
        assert p.M_actual in (9, 10)
    assert pattern.build_pattern(np.ones((n, n), np.uint8), N).M_actual == N


def test_laminate_pattern_covers_support():
    g = synth.laminate((32, 32), 11, offset=3)
    keys, _ = pattern.spectrum_keys(g)
    support = np.flatnonzero(keys.ravel() > 0)
    p = pattern.build_pattern(g, support.size)
    assert set(support.tolist()) <= set(p.sorted_idx.tolist())
    k0, k1 = np.unravel_index(support, g.shape)
    assert np.all(k1 == 0)
