"""Seeded input generators: determinism, voxelisation and the recorded stats."""
import numpy as np

import synth


def test_disk_volume_fraction_and_symmetry():
    n = 64
    g = synth.disk(n, n, np.sqrt(0.3 * n * n / np.pi))
    assert abs(g.mean() - 0.3) < 0.01
    assert np.array_equal(g, g[::-1, :]) and np.array_equal(g, g.T)


def test_rsa_deterministic_and_non_overlapping():
    a = synth.rsa_fibres(128, 128, 6, 10, seed=3, target_vf=0.35)
    b = synth.rsa_fibres(128, 128, 6, 10, seed=3, target_vf=0.35)
    assert np.array_equal(a.g, b.g) and a.count == b.count
    assert a.vf >= 0.35
    vol = sum(np.pi * r * r for r in a.radii) / 128 ** 2
    assert abs(vol - a.vf) < 0.02


def test_metric_rve_reproducible():
    g1, e1 = synth.metric_rve(5, n=64)
    g2, e2 = synth.metric_rve(5, n=64)
    assert np.array_equal(g1, g2) and np.array_equal(e1, e2)
    assert np.all(np.abs(e1) <= 5e-3)


def test_laminate_profile():
    g = synth.laminate((16, 8), 5, offset=14)
    assert g[:, 0].tolist() == [1, 1, 1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1]
    assert np.all(g == g[:, :1])
