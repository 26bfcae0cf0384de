"""GPU parity of the elasto-plastic load path (paper Sec. 2 J2 model; load
steps as in Sec. 5.2) against the FP64 oracle: effective stress per step and
the accumulated plastic strain field after the last step, at the FP32
tolerances of the other solves (effective stress rel. 1e-5, fields rel. L2
1e-4).  The GPU stops at residual 1e-6, the oracle at 1e-10; the J2
iteration contracts slowly (hundreds of iterations per step), so most of the
difference is the GPU's stopping error, not FP32 rounding.  Points whose
elastic/plastic status differs from the oracle's (a yield function within
rounding of zero) are counted and must stay rare."""
import math

import numpy as np
import pytest

import synth
from oracle import pattern, solver
from tests.gpu_common import ORACLE_J2, native_phases, rel_l2, stress_comps

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,R,steps", [(64, 0.05, 5), (128, 0.05, 4)])
def test_load_path_matches_oracle(n, R, steps):
    import torch
    import paper_2103_10203_amd as mor
    g = synth.rsa_fibres(n, n, n / 12.8, n / 6.4, seed=11 + n, target_vf=0.4).g
    M = int(math.ceil(R * g.size))
    final = np.array([0.02, 0.0, 0.0])
    path = np.stack([final * (k + 1) / steps for k in range(steps)])
    plan = mor.Plan(g, M)
    state = torch.zeros(5 * g.size, dtype=torch.float32, device="cuda")
    out = mor.solve_path(plan, path, native_phases(j2=True), 1e-6, state)
    assert out.status == mor.MOR_OK
    p = pattern.build_pattern(g, M)
    ref = solver.solve_path(g, ORACLE_J2, solver.macro_tensor(final, 2), steps, mask=p.mask(), tol=1e-10)
    for k in range(steps):
        want = stress_comps(ref[k].sigma_bar, 2)
        err = np.max(np.abs(out.eff_stress[k] - want)) / np.max(np.abs(want))
        assert err < 1e-5, (k, err)
    alpha = state.view(5, n, n)[4].double().cpu().numpy()
    assert rel_l2(alpha, ref[-1].alpha) < 1e-4
    ep = state.view(5, n, n)[0].double().cpu().numpy()
    assert rel_l2(ep, ref[-1].eps_p[..., 0, 0]) < 1e-4
    assert np.max(alpha) > 0.0
    # elastic/plastic status after the path: differing points are those whose
    # plastic strain is at rounding level on one side
    flips = np.count_nonzero((alpha > 0.0) != (ref[-1].alpha > 0.0))
    assert flips <= max(2, 0.002 * alpha.size), flips


@pytest.mark.parametrize("n1", [384, 512])
def test_load_path_long_rows(n1):
    """Rows of 384 and 512 points, where J2 phases select their own row-kernel
    variant (a radix-4 register pass), against the oracle."""
    import torch
    import paper_2103_10203_amd as mor
    n0, steps = 32, 3
    g = synth.rsa_fibres(n0, n1, 3.0, 6.0, seed=n1, target_vf=0.35).g
    M = int(math.ceil(0.05 * g.size))
    final = np.array([0.015, -0.002, 0.004])
    path = np.stack([final * (k + 1) / steps for k in range(steps)])
    plan = mor.Plan(g, M)
    state = torch.zeros(5 * g.size, dtype=torch.float32, device="cuda")
    out = mor.solve_path(plan, path, native_phases(j2=True), 1e-6, state)
    assert out.status == mor.MOR_OK
    p = pattern.build_pattern(g, M)
    ref = solver.solve_path(g, ORACLE_J2, solver.macro_tensor(final, 2), steps, mask=p.mask(), tol=1e-10)
    for k in range(steps):
        want = stress_comps(ref[k].sigma_bar, 2)
        err = np.max(np.abs(out.eff_stress[k] - want)) / np.max(np.abs(want))
        assert err < 1e-5, (k, err)
    alpha = state.view(5, n0, n1)[4].double().cpu().numpy()
    assert np.max(alpha) > 0.0
    assert rel_l2(alpha, ref[-1].alpha) < 1e-4


def test_homogeneous_j2_one_iteration_per_step():
    import torch
    import paper_2103_10203_amd as mor
    g = np.zeros((32, 32), np.uint8)
    plan = mor.Plan(g, 51)
    path = np.stack([[0.004 * k, 0.0, 0.0] for k in range(1, 6)])
    state = torch.zeros(5 * g.size, dtype=torch.float32, device="cuda")
    out = mor.solve_path(plan, path, native_phases(j2=True), 1e-6, state)
    assert np.all(out.iterations == 1)
    ref = solver.solve_path(g, ORACLE_J2, solver.macro_tensor([0.02, 0, 0], 2), 5, tol=1e-12)
    for k in range(5):
        want = stress_comps(ref[k].sigma_bar, 2)
        assert np.max(np.abs(out.eff_stress[k] - want)) < 1e-5 * np.max(np.abs(want))


def test_load_path_graph_replay_matches_eager():
    """The J2 load path with hipGraph-replayed iteration chunks equals the
    eager path exactly (stress per step, iterations, final state)."""
    import torch
    import paper_2103_10203_amd as mor
    g = synth.rsa_fibres(64, 64, 5.0, 10.0, seed=75, target_vf=0.4).g
    plan = mor.Plan(g, 205)
    path = np.stack([[0.005 * k, 0.0, 0.0] for k in range(1, 5)])
    se = torch.zeros(5 * g.size, dtype=torch.float32, device="cuda")
    sg = torch.zeros(5 * g.size, dtype=torch.float32, device="cuda")
    oe = mor.solve_path(plan, path, native_phases(j2=True), 1e-6, se)
    og = mor.solve_path(plan, path, native_phases(j2=True), 1e-6, sg, use_graph=1)
    assert np.array_equal(oe.eff_stress, og.eff_stress)
    assert np.array_equal(oe.iterations, og.iterations)
    assert bool((se == sg).all())


def test_batched_load_paths_equal_single_paths():
    """mor_solve_path_multi: RVEs on different grids and microstructures,
    each with its own macro strain history, in one call; every RVE's stresses,
    iteration counts and final state equal its own mor_solve_path bit for
    bit (the same kernels and start rules), and RVE 0 matches the oracle."""
    import torch
    import paper_2103_10203_amd as mor
    gs = [synth.rsa_fibres(64, 64, 5.0, 10.0, seed=91, target_vf=0.4).g,
          synth.rsa_fibres(128, 128, 10.0, 20.0, seed=92, target_vf=0.4).g]
    plans = [mor.Plan(g, int(math.ceil(0.05 * g.size))) for g in gs]
    plan_of = [0, 1, 0, 1, 0]
    steps = 4
    finals = np.array([[0.02, 0.0, 0.0], [0.0, 0.015, 0.003], [-0.01, 0.01, 0.0], [0.012, -0.004, 0.002],
                       [0.0, 0.0, 0.0]])
    paths = np.stack([np.stack([f * (k + 1) / steps for k in range(steps)]) for f in finals])
    ph = native_phases(j2=True)
    sizes = [gs[i].size for i in plan_of]
    state = torch.zeros(5 * sum(sizes), dtype=torch.float32, device="cuda")
    out = mor.solve_path_multi(plans, plan_of, paths, ph, 1e-6, state, want_coeffs=True)
    assert out.status == mor.MOR_OK
    off = np.concatenate([[0], np.cumsum(sizes)]) * 5
    coff = np.concatenate([[0], np.cumsum([3 * plans[i].n_coeff for i in plan_of])])
    for b, i in enumerate(plan_of):
        st1 = torch.zeros(5 * gs[i].size, dtype=torch.float32, device="cuda")
        one = mor.solve_path(plans[i], paths[b], ph, 1e-6, st1, want_coeffs=True)
        assert np.array_equal(out.iterations[b], one.iterations)
        assert np.array_equal(out.eff_stress[b][:, :4], one.eff_stress)
        assert bool((state[off[b]:off[b + 1]] == st1).all())
        assert bool((out.coeffs[coff[b]:coff[b + 1]] == one.coeffs.reshape(-1)).all())
    g = gs[0]
    p = pattern.build_pattern(g, plans[0].info["M"])
    ref = solver.solve_path(g, ORACLE_J2, solver.macro_tensor(finals[0], 2), steps, mask=p.mask(), tol=1e-10)
    for k in range(steps):
        want = stress_comps(ref[k].sigma_bar, 2)
        assert np.max(np.abs(out.eff_stress[0, k, :4] - want)) / np.max(np.abs(want)) < 1e-5
