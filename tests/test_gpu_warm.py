"""Learned warm start on the GPU: the network's hand-written kernels against
the FP64 CPU reference (gradients, Adam), BF16 inference against FP32, the
slot gather/scatter round trip, and the gain of the trained network over the
cold start on held-out microstructures (measured, not pinned)."""
import math

import numpy as np
import pytest

import synth
from oracle import mlp as omlp
from oracle import pattern as opattern
from oracle import solver as osolver
from tests.gpu_common import ORACLE_PH, native_phases

pytestmark = pytest.mark.gpu


def _mor():
    import paper_2103_10203_amd as mor
    return mor


def _oracle_params(net, flat):
    return [p.astype(np.float64) for p in net.split(flat)]


@pytest.mark.parametrize("dims", [(7, 8, 5, 6), (65, 96, 130, 37)])
def test_gradients_match_fp64_reference(dims):
    import torch
    mor = _mor()
    i, h, o, B = dims
    net = mor.MLP(i, h, o, seed=3)
    rng = np.random.default_rng(1)
    flat = net.params()
    # nonzero biases so every term of the backward pass is exercised
    parts = net.split(flat)
    for p in parts[1::2]:
        p[:] = rng.normal(size=p.shape) * 0.1
    net.set_params(flat)
    X = rng.normal(size=(B, i)).astype(np.float32)
    T = rng.normal(size=(B, o)).astype(np.float32)
    loss = net.grad(torch.tensor(X, device="cuda"), torch.tensor(T, device="cuda"))
    P = _oracle_params(net, net.params())
    y, cache = omlp.forward(P, X.astype(np.float64))
    want = omlp.backward(P, cache, y, T.astype(np.float64))
    assert abs(loss - omlp.mse(y, T)) < 1e-5 * abs(omlp.mse(y, T))
    got = net.split(net.grads())
    for g, w in zip(got, want):
        assert np.max(np.abs(g - w)) <= 1e-4 * np.max(np.abs(w)) + 1e-9


def test_gradients_real_shape_sampled_coordinates():
    import torch
    mor = _mor()
    S = 1024
    net = mor.MLP(4 * S + 1, 512, 18 * S, seed=5)
    rng = np.random.default_rng(2)
    B = 6
    X = (rng.normal(size=(B, 4 * S + 1)) * 0.05).astype(np.float32)
    T = (rng.normal(size=(B, 18 * S)) * 0.05).astype(np.float32)
    net.grad(torch.tensor(X, device="cuda"), torch.tensor(T, device="cuda"))
    P = _oracle_params(net, net.params())
    y, cache = omlp.forward(P, X.astype(np.float64))
    want = omlp.backward(P, cache, y, T.astype(np.float64))
    got = net.split(net.grads())
    for g, w in zip(got, want):
        idx = rng.integers(0, w.size, size=200)
        gv, wv = g.reshape(-1)[idx], w.reshape(-1)[idx]
        assert np.max(np.abs(gv - wv)) <= 2e-4 * np.max(np.abs(w)) + 1e-12


def test_adam_matches_reference():
    import torch
    mor = _mor()
    net = mor.MLP(9, 16, 4, seed=7)
    rng = np.random.default_rng(3)
    X = torch.tensor(rng.normal(size=(5, 9)).astype(np.float32), device="cuda")
    T = torch.tensor(rng.normal(size=(5, 4)).astype(np.float32), device="cuda")
    P = _oracle_params(net, net.params())
    m = [np.zeros_like(p) for p in P]
    v = [np.zeros_like(p) for p in P]
    for step in range(1, 4):
        net.grad(X, T)
        g = [x.astype(np.float64) for x in net.split(net.grads())]
        omlp.adam_step(P, g, m, v, step, lr=1e-2)
        net.adam(1e-2)
        got = net.split(net.params())
        for a, b in zip(got, P):
            assert np.max(np.abs(a - b)) < 1e-5
        P = _oracle_params(net, net.params())


def test_bf16_inference_close_to_fp32():
    import torch
    mor = _mor()
    net = mor.MLP(300, 128, 200, seed=9)
    rng = np.random.default_rng(4)
    X = torch.tensor(rng.normal(size=(70, 300)).astype(np.float32), device="cuda")
    y32 = net.forward(X, mor.MLP_FP32)
    y16 = net.forward(X, mor.MLP_BF16)
    P = _oracle_params(net, net.params())
    yref, _ = omlp.forward(P, X.cpu().double().numpy())
    assert np.max(np.abs(y32.cpu().numpy() - yref)) < 1e-4 * np.max(np.abs(yref))
    rel = float(torch.linalg.norm(y16 - y32) / torch.linalg.norm(y32))
    assert rel < 2e-2, rel


def test_slot_targets_and_apply_round_trip():
    import torch
    mor = _mor()
    g, _ = synth.metric_rve(3, n=64)
    plan = mor.Plan(g, 205)
    S = plan.info["M_actual"]  # more slots than pairs: every pair gets one
    plan_of = np.zeros(3, np.int64)
    out = mor.solve_multi([plan], plan_of, np.eye(3), native_phases(), 1e-7, want_coeffs=True)
    T = mor.warm_targets([plan], [0], S, native_phases(), out.coeffs)
    eb = np.array([[1.3e-3, -4e-4, 6e-4]])
    W = mor.warm_apply([plan], [0], S, native_phases(), T, eb).view(3, plan.n_coeff)
    ref = mor.solve(plan, eb, native_phases(), 1e-7, want_coeffs=True).coeffs[0]
    ci = plan.coeff_index()
    nz = ci != 0
    err = torch.linalg.norm((W - ref)[:, torch.tensor(nz, device="cuda")]) / torch.linalg.norm(ref)
    assert float(err) < 1e-5
    # the exact response as warm start converges in one or two iterations
    o2 = mor.solve(plan, eb, native_phases(), 1e-6, warm_start=W)
    assert o2.iterations[0] <= 3


@pytest.mark.parametrize("S", [8, 400])
def test_zero_correction_is_the_first_cold_iterate(S):
    """With a zero network output the warm start is the Born prior, which is
    the FP64 oracle's first iterate from the cold start at every coefficient
    of the pattern (also beyond the network's slots); starting there saves
    exactly one iteration."""
    import torch
    from paper_2103_10203_amd import warm
    mor = _mor()
    n, M = 64, 205
    gs = [synth.metric_rve(i, n=n)[0] for i in range(6)]
    ebs = synth.macro_strains(6, 3, 5e-3, seed=77)
    plans = [mor.Plan(g, M) for g in gs]
    po = np.arange(6)
    W = warm.born_warm(plans, po, ebs, native_phases(), S)
    off = 0
    for b, (g, p) in enumerate(zip(gs, plans)):
        pat = opattern.build_pattern(g, M)
        mask = np.zeros(g.size, bool)
        mask[pat.sorted_idx] = True
        E = osolver.macro_tensor(ebs[b], 2)
        r1 = osolver.solve(g, ORACLE_PH, E, mask=mask, tol=0.0, max_iter=1)
        eh = np.fft.fft2(r1.eps, axes=(0, 1)).reshape(g.size, 3, 3)
        ci = p.coeff_index()
        want = np.stack([eh[ci, 0, 0], eh[ci, 1, 1], eh[ci, 0, 1]])
        got = W[off:off + 3 * p.n_coeff].view(3, p.n_coeff).cpu().numpy()
        off += 3 * p.n_coeff
        nz = ci != 0
        err = np.linalg.norm((got - want)[:, nz]) / np.linalg.norm(want[:, nz])
        assert err < 1e-5, (b, err)
    cold = mor.solve_multi(plans, po, ebs, native_phases(), 1e-6)
    born = mor.solve_multi(plans, po, ebs, native_phases(), 1e-6, warm_start=W)
    assert np.all(np.abs(born.iterations - (cold.iterations - 1)) <= 1)
    assert born.iterations.mean() < cold.iterations.mean() - 0.5


def test_trained_network_gain_small_grid():
    """Train on 64^2 fibre RVEs (the headline recipe scaled by 1/4) and compare
    held-out iterations and effective stress with the cold start and with the
    Born prior alone.  This test documents the measured gain rather than
    pinning one: the start saves the prior's iteration over the cold start,
    and the learned correction adds no measurable gain over the prior (held-
    out means within 0.1 iteration; the analysis is in the design notes), so
    the assertions are that the network start beats the cold start and is
    not worse than the prior."""
    import torch
    from paper_2103_10203_amd import warm
    mor = _mor()
    n, M, S = 64, 205, 96
    gs = warm.generate_microstructures(range(0, 600), n=n)
    data = warm.build_training_set(gs, M, native_phases(), S)
    cfg = warm.WarmConfig(nslots=S, hidden=512, epochs=80, batch=128, lr=1e-3)
    net = mor.MLP(4 * S + 1, 512, 18 * S, seed=0)
    hist, _ = warm.train(net, data, cfg)
    assert hist[-1] < 0.2 * hist[0]
    test_g = warm.generate_microstructures(range(1_000_000, 1_000_064), n=n)
    ebs = synth.macro_strains(64, 3, 5e-3, seed=123)
    plans = [mor.Plan(g, M) for g in test_g]
    po = np.arange(64)
    held = warm.build_training_set(test_g, M, native_phases(), S)
    cold = mor.solve_multi(plans, po, ebs, native_phases(), 1e-6)
    Wb = warm.born_warm(plans, po, ebs, native_phases(), S)
    born = mor.solve_multi(plans, po, ebs, native_phases(), 1e-6, warm_start=Wb)
    W = warm.predict_warm(net, plans, po, ebs, native_phases(), S)
    hot = mor.solve_multi(plans, po, ebs, native_phases(), 1e-6, warm_start=W)
    assert cold.status == mor.MOR_OK and hot.status == mor.MOR_OK
    print(f"mean iterations: cold {cold.iterations.mean():.3f} born {born.iterations.mean():.3f} "
          f"network {hot.iterations.mean():.3f}; held-out correction error "
          f"{warm.relative_error(net, held):.3f}")
    assert hot.iterations.mean() < cold.iterations.mean() - 0.5
    assert hot.iterations.mean() <= born.iterations.mean() + 0.1
    rel = np.max(np.abs(hot.eff_stress - cold.eff_stress)) / np.max(np.abs(cold.eff_stress))
    assert rel < 2e-5


def test_bf16_inference_real_shape():
    """The tiled BF16 MFMA inference at the warm-start network's real shape
    (4097 -> 512 -> 512 -> 18432, batch 1024 plus a ragged batch) against the
    FP32 path."""
    import torch
    mor = _mor()
    S = 1024
    net = mor.MLP(4 * S + 1, 512, 18 * S, seed=11)
    rng = np.random.default_rng(8)
    for B in (1024, 37):
        X = torch.tensor((rng.normal(size=(B, 4 * S + 1)) * 0.1).astype(np.float32), device="cuda")
        y32 = net.forward(X, mor.MLP_FP32)
        y16 = net.forward(X, mor.MLP_BF16)
        rel = float(torch.linalg.norm(y16 - y32) / torch.linalg.norm(y32))
        assert rel < 2e-2, (B, rel)
