"""GPU parity of the reduced fixed-point solve (paper Sec. 4, steps a-d) against
the FP64 oracle, through the C ABI.

Tolerances: effective stress rel. 1e-5 and fields rel. L2 1e-4 against the
oracle's fixed point (oracle run to 1e-12, GPU FP32 to 1e-6 or 1e-7); iteration
counts within +-1 of the oracle run to the same tolerance."""
import math

import numpy as np
import pytest

import synth
from oracle import bounds, pattern, solver
from tests.gpu_common import ORACLE_PH, native_phases, oracle_reduced, rel_l2, stress_comps

pytestmark = pytest.mark.gpu


def _mor():
    import paper_2103_10203_amd as mor
    return mor


def _fields_from_oracle(res, dim):
    eps = solver.tensor_comps(res.eps, dim)          # [..., C]
    sig = solver.tensor_comps(res.sigma, dim, with_s33=True)
    return np.moveaxis(eps, -1, 0), np.moveaxis(sig, -1, 0)


def _check_against_oracle(g, eb, M, gpu_tol=1e-6, check_fields=True, iters=True):
    mor = _mor()
    dim = g.ndim
    plan = mor.Plan(g, M)
    out = mor.solve(plan, np.array([eb]), native_phases(), gpu_tol, want_fields=check_fields)
    assert out.status == mor.MOR_OK
    _, ref = oracle_reduced(g, eb, M, tol=1e-12)
    sref = stress_comps(ref.sigma_bar, dim)
    err = np.max(np.abs(out.eff_stress[0] - sref)) / np.max(np.abs(sref))
    assert err < 1e-5, err
    if check_fields:
        e_ref, s_ref = _fields_from_oracle(ref, dim)
        assert rel_l2(out.strain[0].cpu().numpy(), e_ref) < 1e-4
        assert rel_l2(out.stress[0].cpu().numpy(), s_ref) < 1e-4
    if iters:
        _, r6 = oracle_reduced(g, eb, M, tol=gpu_tol)
        assert abs(int(out.iterations[0]) - r6.iterations) <= 1, (out.iterations[0], r6.iterations)
    return out


def test_centred_disk_64():
    n = 64
    g = synth.disk(n, n, math.sqrt(0.3 * n * n / math.pi))
    _check_against_oracle(g, [1e-3, 0.0, 0.0], 205)


def test_fibres_256_metric_sample():
    g, eb = synth.metric_rve(0)
    _check_against_oracle(g, list(eb), 3277)


def test_batched_macro_strains_one_plan():
    mor = _mor()
    g = synth.rsa_fibres(128, 128, 4, 8, seed=5, target_vf=0.35).g
    M = 820
    ebs = synth.macro_strains(6, 3, 5e-3, seed=17)
    plan = mor.Plan(g, M)
    out = mor.solve(plan, ebs, native_phases(), 1e-6)
    assert out.status == mor.MOR_OK
    for b in range(len(ebs)):
        _, ref = oracle_reduced(g, list(ebs[b]), M, tol=1e-12)
        sref = stress_comps(ref.sigma_bar, 2)
        assert np.max(np.abs(out.eff_stress[b] - sref)) / np.max(np.abs(sref)) < 1e-5


def test_multi_uneven_grids():
    mor = _mor()
    gs = [synth.rsa_fibres(n, n, n / 32, n / 16, seed=40 + n, target_vf=0.35).g for n in (32, 64, 48)]
    Ms = [int(math.ceil(0.05 * g.size)) for g in gs]
    plans = [mor.Plan(g, M) for g, M in zip(gs, Ms)]
    plan_of = np.array([0, 1, 2, 1, 0, 2, 2])
    ebs = synth.macro_strains(len(plan_of), 3, 5e-3, seed=3)
    out = mor.solve_multi(plans, plan_of, ebs, native_phases(), 1e-6)
    assert out.status == mor.MOR_OK
    for b, p in enumerate(plan_of):
        _, ref = oracle_reduced(gs[p], list(ebs[b]), Ms[p], tol=1e-12)
        sref = stress_comps(ref.sigma_bar, 2)
        assert np.max(np.abs(out.eff_stress[b] - sref)) / np.max(np.abs(sref)) < 1e-5


def test_homogeneous_and_single_frequency():
    mor = _mor()
    eb = [1e-3, -4e-4, 2.5e-4]
    for fill in (0, 1):
        g = np.full((32, 32), fill, np.uint8)
        out = mor.solve(mor.Plan(g, 51), np.array([eb]), native_phases(), 1e-6)
        assert out.iterations[0] == 1
        p = ORACLE_PH[fill]
        e = solver.macro_tensor(eb, 2)
        ref = stress_comps(p.lam * np.trace(e) * np.eye(3) + 2 * p.mu * e, 2)
        assert np.max(np.abs(out.eff_stress[0] - ref)) < 1e-6 * np.max(np.abs(ref))
    g = synth.rsa_fibres(32, 32, 3, 6, seed=4, target_vf=0.35).g
    out = mor.solve(mor.Plan(g, 1), np.array([eb]), native_phases(), 1e-6)
    ref = stress_comps(bounds.voigt_stress(ORACLE_PH, float(g.mean()), solver.macro_tensor(eb, 2)), 2)
    assert out.iterations[0] == 1
    assert np.max(np.abs(out.eff_stress[0] - ref)) < 1e-6 * np.max(np.abs(ref))


def test_laminate_exact_fields():
    mor = _mor()
    g = synth.laminate((64, 32), 23, offset=5)
    keys, _ = pattern.spectrum_keys(g)
    M = int(np.count_nonzero(keys))
    eb = [1e-3, -6e-4, 4e-4]
    out = mor.solve(mor.Plan(g, M), np.array([eb]), native_phases(), 1e-7, want_fields=True)
    eps_ref, sig_ref, sbar = bounds.laminate_fields(g[:, 0], ORACLE_PH, solver.macro_tensor(eb, 2))
    e = out.strain[0].cpu().numpy()
    ref = np.moveaxis(solver.tensor_comps(eps_ref, 2), -1, 0)[:, :, None]
    assert np.max(np.abs(e - ref)) < 2e-8
    assert np.max(np.abs(out.eff_stress[0] - stress_comps(sbar, 2))) < 1e-5 * np.max(np.abs(sbar))


def test_zero_macro_strain_and_mean_strain():
    mor = _mor()
    g, _ = synth.metric_rve(2, n=64)
    plan = mor.Plan(g, 205)
    out = mor.solve(plan, np.zeros((1, 3)), native_phases(), 1e-6, want_fields=True, want_coeffs=True)
    assert out.iterations[0] == 1 and np.all(out.eff_stress == 0.0)
    eb = np.array([[2e-3, -1e-3, 7e-4]])
    out = mor.solve(plan, eb, native_phases(), 1e-6, want_fields=True, want_coeffs=True)
    mean = out.strain[0].double().mean(dim=(1, 2)).cpu().numpy()
    assert np.max(np.abs(mean - eb[0])) < 1e-9
    ci = plan.coeff_index()
    z = np.flatnonzero(ci == 0)[0]
    c0 = out.coeffs[0, :, z].cpu().numpy()
    assert np.array_equal(c0.real, (g.size * eb[0]).astype(np.float32)) and np.all(c0.imag == 0)


def test_max_iter_reports_not_converged():
    mor = _mor()
    g, eb = synth.metric_rve(1, n=64)
    out = mor.solve(mor.Plan(g, 205), np.array([eb]), native_phases(), 1e-9, max_iter=5)
    assert out.status == mor.MOR_E_NOT_CONVERGED
    assert out.iterations[0] == 5 and out.residual[0] > 1e-9


def test_deterministic_rerun():
    mor = _mor()
    g, eb = synth.metric_rve(4, n=128)
    plan = mor.Plan(g, 820)
    a = mor.solve(plan, np.array([eb]), native_phases(), 1e-6)
    b = mor.solve(plan, np.array([eb]), native_phases(), 1e-6)
    assert np.array_equal(a.eff_stress, b.eff_stress) and np.array_equal(a.residual, b.residual)


@pytest.mark.parametrize("n,R", [(384, 0.05), (512, 0.01), (128, 0.2)])
def test_other_grid_sizes(n, R):
    mor = _mor()
    g = synth.rsa_fibres(n, n, n / 32, n / 16, seed=70 + n, target_vf=0.35).g
    M = int(math.ceil(R * g.size))
    eb = [2e-3, -1e-3, 1.5e-3]
    plan = mor.Plan(g, M)
    out = mor.solve(plan, np.array([eb]), native_phases(), 1e-6)
    _, ref = oracle_reduced(g, eb, M, tol=1e-10)
    sref = stress_comps(ref.sigma_bar, 2)
    assert np.max(np.abs(out.eff_stress[0] - sref)) / np.max(np.abs(sref)) < 1e-5


# (24, 128, 32) and (36, 64, 16): the axis-1 kernels of n1 = 128 and 64 with a
# ragged last block of x0 values (16 per workgroup)
@pytest.mark.parametrize("shape", [(16, 16, 16), (32, 64, 64), (64, 32, 128), (24, 128, 32), (36, 64, 16)])
def test_3d_parity(shape):
    mor = _mor()
    g = synth.rsa_spheres(*shape, r_lo=min(shape) / 8, r_hi=min(shape) / 5, seed=sum(shape), target_vf=0.2).g
    M = int(math.ceil(0.03 * g.size))
    eb = [1e-3, -4e-4, 3e-4, 2e-4, -1e-4, 5e-4]
    plan = mor.Plan(g, M)
    out = mor.solve(plan, np.array([eb]), native_phases(), 1e-6, want_fields=True)
    assert out.status == mor.MOR_OK
    _, ref = oracle_reduced(g, eb, M, tol=1e-10)
    sref = stress_comps(ref.sigma_bar, 3)
    assert np.max(np.abs(out.eff_stress[0] - sref)) / np.max(np.abs(sref)) < 1e-5
    e_ref, s_ref = _fields_from_oracle(ref, 3)
    assert rel_l2(out.strain[0].cpu().numpy(), e_ref) < 1e-4


@pytest.mark.parametrize("n", [64, 128, 256, 384, 512])
def test_row_kernel_variants(n):
    """Every row-kernel variant of a size (factorisation, row block) against
    the FP64 oracle on a random-fibre RVE."""
    mor = _mor()
    g = synth.fibre_rve_256(11, n).g
    eb = [2e-3, -1e-3, 5e-4]
    M = int(math.ceil(0.05 * n * n))
    _, ref = oracle_reduced(g, eb, M, tol=1e-11)
    sref = stress_comps(ref.sigma_bar, 2)
    e_ref, s_ref = _fields_from_oracle(ref, 2)
    plan = mor.Plan(g, M)
    keep = mor.tune_get(2, n)
    nv = mor.tune_variants(2, n)
    assert nv >= 1
    try:
        for v in range(nv):
            mor.tune_set(2, n, v)
            out = mor.solve(plan, np.array([eb]), native_phases(), 1e-7, want_fields=True)
            assert out.status == mor.MOR_OK
            err = np.max(np.abs(out.eff_stress[0] - sref)) / np.max(np.abs(sref))
            assert err < 1e-5, (v, err)
            assert rel_l2(out.strain[0].cpu().numpy(), e_ref) < 1e-4, v
            assert rel_l2(out.stress[0].cpu().numpy(), s_ref) < 1e-4, v
    finally:
        mor.tune_set(2, n, keep)


def test_autotune_keeps_results():
    """The autotuner leaves a valid variant selected for each size of a mixed
    batch, and solves after tuning agree with solves before it."""
    mor = _mor()
    gs = [synth.fibre_rve_256(20 + i, n).g for i, n in enumerate((128, 256, 256, 128))]
    plans = [mor.Plan(g, int(math.ceil(0.05 * g.size))) for g in gs]
    po = np.array([0, 1, 2, 3, 1, 0])
    ebs = synth.macro_strains(len(po), 3, 5e-3, seed=5)
    keep = {n: mor.tune_get(2, n) for n in (128, 256)}
    try:
        before = mor.solve_multi(plans, po, ebs, native_phases(), 1e-7)
        mor.autotune(plans, po, ebs, native_phases(), 1e-7, reps=1)
        for n in (128, 256):
            assert 0 <= mor.tune_get(2, n) < mor.tune_variants(2, n)
        after = mor.solve_multi(plans, po, ebs, native_phases(), 1e-7)
        rel = np.max(np.abs(after.eff_stress - before.eff_stress)) / np.max(np.abs(before.eff_stress))
        assert rel < 2e-6
    finally:
        for n, v in keep.items():
            mor.tune_set(2, n, v)


def test_graph_replay_matches_eager():
    """Iteration chunks replayed from a captured hipGraph give exactly the eager
    results (same kernels, same order), over several solves in a row with eager
    solves in between, for one plan, a mixed batch and the J2 load path."""
    mor = _mor()
    gs = [synth.fibre_rve_256(40 + i, n).g for i, n in enumerate((64, 128, 64))]
    plans = [mor.Plan(g, int(math.ceil(0.05 * g.size))) for g in gs]
    po = np.array([0, 1, 2, 1, 0])
    ebs = synth.macro_strains(len(po), 3, 5e-3, seed=9)
    ref = mor.solve_multi(plans, po, ebs, native_phases(), 1e-6)
    for rep in range(3):
        got = mor.solve_multi(plans, po, ebs, native_phases(), 1e-6, use_graph=1, check_every=4 + rep)
        assert np.array_equal(got.eff_stress, ref.eff_stress)
        assert np.array_equal(got.iterations, ref.iterations)
        eager = mor.solve_multi(plans, po, ebs, native_phases(), 1e-6, check_every=4 + rep)
        assert np.array_equal(got.eff_stress, eager.eff_stress)
        assert np.array_equal(got.iterations, eager.iterations)
    one_e = mor.solve(plans[1], ebs[:2], native_phases(), 1e-6, want_fields=True)
    one_g = mor.solve(plans[1], ebs[:2], native_phases(), 1e-6, want_fields=True, use_graph=1)
    assert np.array_equal(one_e.eff_stress, one_g.eff_stress)
    assert bool((one_e.strain == one_g.strain).all())


@pytest.mark.parametrize("shape", [(16, 16, 64), (8, 16, 128), (8, 8, 256)])
def test_row_kernel_variants_3d(shape):
    """Every 3D row-kernel variant (six strain components) against the oracle."""
    mor = _mor()
    g = synth.rsa_spheres(*shape, r_lo=3.0, r_hi=5.0, seed=sum(shape), target_vf=0.2).g
    M = int(math.ceil(0.03 * g.size))
    eb = [1e-3, -4e-4, 3e-4, 2e-4, -1e-4, 5e-4]
    _, ref = oracle_reduced(g, eb, M, tol=1e-10)
    sref = stress_comps(ref.sigma_bar, 3)
    e_ref, _ = _fields_from_oracle(ref, 3)
    plan = mor.Plan(g, M)
    L = shape[-1]
    keep = mor.tune_get(3, L)
    try:
        for v in range(mor.tune_variants(3, L)):
            mor.tune_set(3, L, v)
            out = mor.solve(plan, np.array([eb]), native_phases(), 1e-7, want_fields=True)
            assert out.status == mor.MOR_OK
            err = np.max(np.abs(out.eff_stress[0] - sref)) / np.max(np.abs(sref))
            assert err < 1e-5, (v, err)
            assert rel_l2(out.strain[0].cpu().numpy(), e_ref) < 1e-4, v
    finally:
        mor.tune_set(3, L, keep)


@pytest.mark.parametrize("shape", [(64, 64), (128, 128), (256, 256), (384, 96), (512, 64), (128, 16, 16)])
def test_col_kernel_variants(shape):
    """Every column-kernel variant (axis-0 FFT factorisation, columns per
    workgroup) against the FP64 oracle."""
    mor = _mor()
    nd = len(shape)
    if nd == 2:
        g = synth.rsa_fibres(*shape, r_lo=min(shape) / 16, r_hi=min(shape) / 8, seed=sum(shape), target_vf=0.35).g
        eb = [2e-3, -1e-3, 5e-4]
        M = int(math.ceil(0.05 * g.size))
    else:
        g = synth.rsa_spheres(*shape, r_lo=3.0, r_hi=5.0, seed=sum(shape), target_vf=0.2).g
        eb = [1e-3, -4e-4, 3e-4, 2e-4, -1e-4, 5e-4]
        M = int(math.ceil(0.03 * g.size))
    _, ref = oracle_reduced(g, eb, M, tol=1e-11 if nd == 2 else 1e-10)
    sref = stress_comps(ref.sigma_bar, nd)
    e_ref, _ = _fields_from_oracle(ref, nd)
    plan = mor.Plan(g, M)
    n0 = shape[0]
    keep = mor.tune_get(nd, n0, mor.KERNEL_COL)
    try:
        for v in range(mor.tune_variants(nd, n0, mor.KERNEL_COL)):
            mor.tune_set(nd, n0, v, mor.KERNEL_COL)
            out = mor.solve(plan, np.array([eb]), native_phases(), 1e-7, want_fields=True)
            assert out.status == mor.MOR_OK
            err = np.max(np.abs(out.eff_stress[0] - sref)) / np.max(np.abs(sref))
            assert err < 1e-5, (v, err)
            assert rel_l2(out.strain[0].cpu().numpy(), e_ref) < 1e-4, v
    finally:
        mor.tune_set(nd, n0, keep, mor.KERNEL_COL)


def test_persistent_schedule_matches_grid():
    """The persistent (RVE, tile)-queue schedule gives bit-identical results
    to the grid schedule: mixed grids with different iteration counts, a 3D
    batch, the J2 load path, and under hipGraph replay."""
    import torch
    mor = _mor()
    gs = [synth.fibre_rve_256(80 + i, n).g for i, n in enumerate((64, 128, 256, 128, 64))]
    plans = [mor.Plan(g, int(math.ceil(0.05 * g.size))) for g in gs]
    po = np.array([0, 1, 2, 3, 4, 2, 1, 0, 3])
    ebs = synth.macro_strains(len(po), 3, 5e-3, seed=21)
    ebs[3] = 0.0  # converges at once
    grid = mor.solve_multi(plans, po, ebs, native_phases(), 1e-6)
    pers = mor.solve_multi(plans, po, ebs, native_phases(), 1e-6, schedule=mor.SCHED_PERSISTENT)
    assert np.array_equal(grid.eff_stress, pers.eff_stress)
    assert np.array_equal(grid.iterations, pers.iterations)
    assert len(set(grid.iterations.tolist())) > 1
    pg = mor.solve_multi(plans, po, ebs, native_phases(), 1e-6, schedule=mor.SCHED_PERSISTENT, use_graph=1)
    assert np.array_equal(grid.eff_stress, pg.eff_stress)
    g3 = synth.rsa_spheres(16, 32, 64, r_lo=3.0, r_hi=5.0, seed=4, target_vf=0.2).g
    p3 = mor.Plan(g3, int(math.ceil(0.03 * g3.size)))
    e3 = synth.macro_strains(3, 6, 1e-3, seed=2)
    a = mor.solve(p3, e3, native_phases(), 1e-6)
    b = mor.solve(p3, e3, native_phases(), 1e-6, schedule=mor.SCHED_PERSISTENT)
    assert np.array_equal(a.eff_stress, b.eff_stress)
    g2 = synth.rsa_fibres(64, 64, 5.0, 10.0, seed=75, target_vf=0.4).g
    plan2 = mor.Plan(g2, 205)
    path = np.stack([[0.005 * k, 0.0, 0.0] for k in range(1, 4)])
    s1 = torch.zeros(5 * g2.size, dtype=torch.float32, device="cuda")
    s2 = torch.zeros(5 * g2.size, dtype=torch.float32, device="cuda")
    o1 = mor.solve_path(plan2, path, native_phases(j2=True), 1e-6, s1)
    o2 = mor.solve_path(plan2, path, native_phases(j2=True), 1e-6, s2, schedule=mor.SCHED_PERSISTENT)
    assert np.array_equal(o1.eff_stress, o2.eff_stress)
    assert bool((s1 == s2).all())


@pytest.mark.parametrize("shape", [(72, 256), (36, 128), (24, 64), (36, 512), (18, 384)])
def test_ragged_row_tiles(shape):
    """Row counts that are not a multiple of the row kernel's rows per
    workgroup (the last workgroup's spare rows gather neighbouring or
    out-of-range entries and must never be stored): every row variant of the
    size against the FP64 oracle."""
    mor = _mor()
    n0, n1 = shape
    g = synth.rsa_fibres(n0, n1, min(shape) / 10, min(shape) / 6, seed=n0 * 7 + n1, target_vf=0.3).g
    eb = [1.5e-3, -5e-4, 8e-4]
    M = int(math.ceil(0.05 * g.size))
    _, ref = oracle_reduced(g, eb, M, tol=1e-11)
    sref = stress_comps(ref.sigma_bar, 2)
    e_ref, _ = _fields_from_oracle(ref, 2)
    plan = mor.Plan(g, M)
    keep = mor.tune_get(2, n1)
    try:
        for v in range(mor.tune_variants(2, n1)):
            mor.tune_set(2, n1, v)
            out = mor.solve(plan, np.array([eb]), native_phases(), 1e-7, want_fields=True)
            assert out.status == mor.MOR_OK
            err = np.max(np.abs(out.eff_stress[0] - sref)) / np.max(np.abs(sref))
            assert err < 1e-5, (v, err)
            assert rel_l2(out.strain[0].cpu().numpy(), e_ref) < 1e-4, v
    finally:
        mor.tune_set(2, n1, keep)


@pytest.mark.parametrize("shape,R", [((4, 4), 0.5), ((6, 1024), 0.05), ((1024, 6), 0.05), ((4, 96), 0.2),
                                     ((1024, 1024), 0.005)])
def test_extreme_grid_shapes(shape, R):
    """The smallest and largest grids the plan accepts (every n even,
    2^a 3^b, 4..1024) and the most elongated ones, against the oracle."""
    rng = np.random.default_rng(sum(shape))
    if shape == (1024, 1024):
        g = synth.rsa_fibres(1024, 1024, 32.0, 64.0, seed=1024, target_vf=0.35).g
    else:
        # a smooth two-phase map, so the pattern keeps meaningful frequencies
        x = np.linspace(0.0, 2.0 * np.pi, shape[0], endpoint=False)[:, None]
        y = np.linspace(0.0, 2.0 * np.pi, shape[1], endpoint=False)[None, :]
        f = np.sin(x + rng.uniform(0, 6)) + np.cos(2 * y + rng.uniform(0, 6)) + 0.3 * rng.standard_normal(shape)
        g = (f > 0.2).astype(np.uint8)
    assert 0 < g.sum() < g.size
    M = max(1, int(math.ceil(R * g.size)))
    _check_against_oracle(g, [1.5e-3, -5e-4, 8e-4], M, check_fields=True, iters=shape != (1024, 1024))


def test_subbatches_match_one_batch():
    """Cutting the batch into cache-sized sub-batches (iterated one after the
    other) changes no result: uneven grids with different iteration counts,
    fields, 3D, the persistent schedule, hipGraph replay, the FP64 path, the
    split-bf16 DFT path and batched J2 paths, each bit for bit against the
    same call with the limit off; the split runs also match the oracle."""
    import torch
    mor = _mor()
    gs = [synth.fibre_rve_256(90 + i, n).g for i, n in enumerate((64, 128, 256, 128, 64))]
    Ms = [int(math.ceil(0.05 * g.size)) for g in gs]
    plans = [mor.Plan(g, M) for g, M in zip(gs, Ms)]
    po = np.array([0, 1, 2, 3, 4, 2, 1, 0, 3, 2, 2])
    ebs = synth.macro_strains(len(po), 3, 5e-3, seed=23)
    ebs[4] = 0.0  # converges at once
    g3 = synth.rsa_spheres(16, 32, 64, r_lo=3.0, r_hi=5.0, seed=5, target_vf=0.2).g
    p3 = mor.Plan(g3, int(math.ceil(0.03 * g3.size)))
    e3 = synth.macro_strains(4, 6, 1e-3, seed=3)
    g2 = synth.rsa_fibres(64, 64, 5.0, 10.0, seed=76, target_vf=0.4).g
    plan2 = mor.Plan(g2, 205)
    paths = np.stack([np.stack([[0.004 * k * (1 + r), -0.001 * k, 0.0] for k in range(1, 4)]) for r in range(5)])

    def run_all():
        res = {"multi": mor.solve_multi(plans, po, ebs, native_phases(), 1e-6, want_fields=True),
               "pers": mor.solve_multi(plans, po, ebs, native_phases(), 1e-6, schedule=mor.SCHED_PERSISTENT),
               "graph": mor.solve_multi(plans, po, ebs, native_phases(), 1e-6, use_graph=1),
               "fp64": mor.solve_multi(plans, po, ebs, native_phases(), 1e-9, precision=mor.PREC_FP64),
               "dft": mor.solve_multi(plans, po, ebs, native_phases(), 1e-5, precision=mor.PREC_BF16X3),
               "3d": mor.solve(p3, e3, native_phases(), 1e-6)}
        state = torch.zeros(5 * 5 * g2.size, dtype=torch.float32, device="cuda")
        res["j2"] = mor.solve_path_multi([plan2], np.zeros(5, dtype=np.int64), paths, native_phases(j2=True), 1e-6,
                                         state)
        res["j2state"] = state.cpu().numpy()
        return res

    keep = mor.tune_subbatch(0)
    try:
        whole = run_all()
        mor.tune_subbatch(1, 1)  # every RVE its own sub-batch
        ones = run_all()
        mor.tune_subbatch(600 << 10, 1)  # a few RVEs per sub-batch
        some = run_all()
    finally:
        mor.tune_subbatch(*keep)
    for split in (ones, some):
        for key in ("multi", "pers", "graph", "fp64", "dft", "3d", "j2"):
            assert np.array_equal(split[key].eff_stress, whole[key].eff_stress), key
            assert np.array_equal(split[key].iterations, whole[key].iterations), key
        assert bool(torch.equal(split["multi"].strain, whole["multi"].strain))
        assert bool(torch.equal(split["multi"].stress, whole["multi"].stress))
        assert np.array_equal(split["j2state"], whole["j2state"])
    assert len(set(whole["multi"].iterations.tolist())) > 1
    for b in (0, 2, 4):
        _, ref = oracle_reduced(gs[po[b]], list(ebs[b]), Ms[po[b]], tol=1e-12)
        sref = stress_comps(ref.sigma_bar, 2)
        if np.max(np.abs(sref)) > 0:
            assert np.max(np.abs(ones["multi"].eff_stress[b] - sref)) / np.max(np.abs(sref)) < 1e-5
        else:
            assert np.max(np.abs(ones["multi"].eff_stress[b])) == 0.0


@pytest.mark.parametrize("shape", [(256, 256, 256), (1024, 1024), (384, 64, 512)])
def test_large_laminates_exact(shape):
    """Largest grids, against a closed form rather than the oracle (which
    would take minutes there): a laminate normal to axis 0 with every
    frequency of its spectrum in the pattern has the exact laminate fields
    (uniform strain in each phase) as the fixed point of the reduced scheme.
    Checks the kernels' indexing at 16.8 M points (3D), 1024² and a 3D grid
    with unequal axes, for every strain component."""
    mor = _mor()
    dim = len(shape)
    g = synth.laminate(shape, shape[0] // 3, offset=shape[0] // 7)
    prof = g.reshape(shape[0], -1)[:, 0]
    # the spectrum lives on the axis-0 line: pattern = its nonzero frequencies
    ph = np.fft.fft(prof.astype(np.float64))
    M = int(np.count_nonzero(np.abs(ph) ** 2 > 2.0 ** -80 * (prof.sum() ** 2)))
    eb = [1e-3, -6e-4, 4e-4] if dim == 2 else [1e-3, -6e-4, 2e-4, 3e-4, -1e-4, 4e-4]
    plan = mor.Plan(g, M)
    assert plan.info["M_actual"] == M
    out = mor.solve(plan, np.array([eb]), native_phases(), 1e-7, want_fields=True)
    assert out.status == mor.MOR_OK
    eps_ref, _, sbar = bounds.laminate_fields(prof, ORACLE_PH, solver.macro_tensor(eb, dim))
    ref = np.moveaxis(solver.tensor_comps(eps_ref, dim), -1, 0)  # [C][n0]
    e = out.strain[0].reshape(len(eb), shape[0], -1)
    emax = e.amax(dim=2).cpu().numpy()
    emin = e.amin(dim=2).cpu().numpy()
    assert np.max(np.abs(emax - ref)) < 5e-8 and np.max(np.abs(emin - ref)) < 5e-8
    assert np.max(np.abs(out.eff_stress[0] - stress_comps(sbar, dim))) < 1e-5 * np.max(np.abs(sbar))


def test_plan_list_member_replaced_and_staging_reused():
    """Batched solves on a PlanList (make_plans) whose member is replaced
    between calls use the new plan (the cached handle array is rebuilt), and
    a run of solves of changing batch size on one stream (pinned staging of
    the small transfers grown, then reused) repeats each result bit for bit."""
    mor = _mor()
    gs = [synth.rsa_fibres(64, 64, 2.0, 4.0, seed=90 + k, target_vf=0.35).g for k in range(3)]
    plans = mor.make_plans(gs[:2], 205)
    assert isinstance(plans, mor.PlanList)
    po = np.array([0, 1, 1, 0])
    ebs = synth.macro_strains(len(po), 3, 5e-3, seed=17)
    first = mor.solve_multi(plans, po, ebs, native_phases(), 1e-6)
    plans[1] = mor.Plan(gs[2], 205)
    swapped = mor.solve_multi(plans, po, ebs, native_phases(), 1e-6)
    fresh = mor.solve_multi([mor.Plan(gs[0], 205), mor.Plan(gs[2], 205)], po, ebs, native_phases(), 1e-6)
    assert np.array_equal(swapped.eff_stress, fresh.eff_stress)
    assert np.array_equal(swapped.eff_stress[0], first.eff_stress[0])
    assert not np.array_equal(swapped.eff_stress[1], first.eff_stress[1])
    # sizes 4, 64, 4, 64: the 64-RVE call outgrows the staging of the first
    big_po = np.arange(64) % 2
    big_eb = synth.macro_strains(64, 3, 5e-3, seed=18)
    runs = [(po, ebs), (big_po, big_eb), (po, ebs), (big_po, big_eb)]
    outs = [mor.solve_multi(plans, p, e, native_phases(), 1e-6) for p, e in runs]
    for a, b in ((outs[0], outs[2]), (outs[1], outs[3])):
        assert np.array_equal(a.eff_stress, b.eff_stress) and np.array_equal(a.iterations, b.iterations)
    assert np.array_equal(outs[0].eff_stress, swapped.eff_stress)
