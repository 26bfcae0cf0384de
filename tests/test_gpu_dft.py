"""The last-axis partial DFT on the matrix cores (FP32 MFMA and split-bf16
"bf16x3" MFMA with FP32 accumulation) against the FP64 oracle, and against
the FFT path of the same library.

Tolerances: FP32 MFMA as the FFT path (effective stress rel. 1e-5, fields
rel. L2 1e-4); bf16x3: effective stress rel. 1e-4, fields rel. L2 1e-4, solved
to residual 1e-5 (the split-bf16 products carry ~2^-16 relative error per
term, which sets the residual floor)."""
import math

import numpy as np
import pytest

import synth
from oracle import pattern, solver
from tests.gpu_common import ORACLE_J2, native_phases, oracle_reduced, rel_l2, stress_comps

pytestmark = pytest.mark.gpu


def _mor():
    import paper_2103_10203_amd as mor
    return mor


def _fields(res, dim):
    eps = np.moveaxis(solver.tensor_comps(res.eps, dim), -1, 0)
    sig = np.moveaxis(solver.tensor_comps(res.sigma, dim, with_s33=True), -1, 0)
    return eps, sig


CASES = [
    ("disk64", 2), ("fibres256", 2), ("box3d", 3), ("rect192x384", 2),
]


def _case(name):
    if name == "disk64":
        n = 64
        return synth.disk(n, n, math.sqrt(0.3 * n * n / math.pi)), [1e-3, 0.0, 0.0], 205
    if name == "fibres256":
        g, eb = synth.metric_rve(5)
        return g, list(eb), 3277
    if name == "rect192x384":
        # a last axis that is not a power of two (twiddle indices reduced
        # modulo 384) and rows that split into 64-row tiles only
        g = synth.rsa_fibres(192, 384, 8.0, 16.0, seed=19, target_vf=0.35).g
        return g, [1e-3, -4e-4, 6e-4], int(math.ceil(0.05 * g.size))
    g = synth.rsa_spheres(32, 64, 64, 5.0, 9.0, seed=3, target_vf=0.25).g
    eb = [1e-3, -5e-4, 2e-4, 3e-4, -1e-4, 4e-4]
    return g, eb, int(math.ceil(0.02 * g.size))


@pytest.mark.parametrize("name,dim", CASES)
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_dft_against_oracle(name, dim, prec):
    mor = _mor()
    g, eb, M = _case(name)
    plan = mor.Plan(g, M)
    p = mor.PREC_FP32 if prec == "fp32" else mor.PREC_BF16X3
    tol = 1e-6 if prec == "fp32" else 1e-5
    out = mor.solve(plan, np.array([eb]), native_phases(), tol, want_fields=True,
                    transform=mor.TRANSFORM_DFT, precision=p)
    assert out.status == mor.MOR_OK
    _, ref = oracle_reduced(g, eb, M, tol=1e-12 if dim == 2 else 1e-10)
    sref = stress_comps(ref.sigma_bar, dim)
    err = np.max(np.abs(out.eff_stress[0] - sref)) / np.max(np.abs(sref))
    assert err < (1e-5 if prec == "fp32" else 1e-4), err
    e_ref, s_ref = _fields(ref, dim)
    assert rel_l2(out.strain[0].cpu().numpy(), e_ref) < 1e-4
    assert rel_l2(out.stress[0].cpu().numpy(), s_ref) < 1e-4
    fft = mor.solve(plan, np.array([eb]), native_phases(), tol, transform=mor.TRANSFORM_FFT)
    assert abs(int(out.iterations[0]) - int(fft.iterations[0])) <= 1


def test_dft_batched_uneven_grids():
    """Uneven batch on the DFT path (FP32 MFMA and bf16x3) against the
    oracle: every RVE's effective stress against the oracle's effective
    stiffness of its microstructure (linear in the macro strain)."""
    mor = _mor()
    gs = [synth.fibre_rve_256(60 + i, n).g for i, n in enumerate((64, 128, 256))]
    Ms = [int(math.ceil(0.05 * g.size)) for g in gs]
    plans = [mor.Plan(g, M) for g, M in zip(gs, Ms)]
    po = np.array([0, 1, 2, 2, 1, 0, 2])
    ebs = synth.macro_strains(len(po), 3, 5e-3, seed=13)
    C = []
    for g, M in zip(gs, Ms):
        cols = []
        for k in range(3):
            e = np.zeros(3)
            e[k] = 1.0
            _, r = oracle_reduced(g, e, M, tol=1e-12)
            cols.append(stress_comps(r.sigma_bar, 2))
        C.append(np.stack(cols, axis=1))
    want = np.stack([C[po[b]] @ ebs[b] for b in range(len(po))])
    d32 = mor.solve_multi(plans, po, ebs, native_phases(), 1e-6, transform=mor.TRANSFORM_DFT)
    x3 = mor.solve_multi(plans, po, ebs, native_phases(), 1e-5, precision=mor.PREC_BF16X3)
    for out, bound in ((d32, 1e-5), (x3, 1e-4)):
        err = np.max(np.abs(out.eff_stress[:, :4] - want), axis=1) / np.max(np.abs(want), axis=1)
        assert np.max(err) < bound, (bound, float(np.max(err)))


def test_dft_j2_load_path():
    import torch
    mor = _mor()
    g = synth.rsa_fibres(64, 64, 5.0, 10.0, seed=75, target_vf=0.4).g
    plan = mor.Plan(g, 205)
    path = np.stack([[0.005 * k, 0.0, 0.0] for k in range(1, 4)])
    s1 = torch.zeros(5 * g.size, dtype=torch.float32, device="cuda")
    s2 = torch.zeros(5 * g.size, dtype=torch.float32, device="cuda")
    a = mor.solve_path(plan, path, native_phases(j2=True), 1e-6, s1)
    b = mor.solve_path(plan, path, native_phases(j2=True), 1e-6, s2, transform=mor.TRANSFORM_DFT)
    ref = solver.solve_path(g, ORACLE_J2, solver.macro_tensor(path[-1], 2), 3,
                             mask=pattern.build_pattern(g, 205).mask(), tol=1e-10)
    for k in range(3):
        want = stress_comps(ref[k].sigma_bar, 2)
        for out in (a, b):
            assert np.max(np.abs(out.eff_stress[k] - want)) < 1e-5 * np.max(np.abs(want)), k
    for s in (s1, s2):
        alpha = s.view(5, 64, 64)[4].double().cpu().numpy()
        assert rel_l2(alpha, ref[-1].alpha) < 1e-4


def test_dft_rejects_unsupported_sizes():
    mor = _mor()
    g = synth.disk(96, 96, 20.0)
    plan = mor.Plan(g, 461)
    with pytest.raises(mor.MorError):
        mor.solve(plan, np.array([[1e-3, 0, 0]]), native_phases(), 1e-6, transform=mor.TRANSFORM_DFT)
    with pytest.raises(mor.MorError):
        mor.solve(plan, np.array([[1e-3, 0, 0]]), native_phases(), 1e-6, precision=mor.PREC_BF16X3,
                  transform=mor.TRANSFORM_FFT)
