"""Benchmark: RVE solves/s to residual 1e-6 on held-out 256x256 random-fibre
RVEs with the adapted 5% pattern (M = 3277), one MI355X.

A step is one batched solve (mor_solve_multi) of the whole batch of RVEs,
each RVE with its own microstructure and macro strain, from its start to
residual < 1e-6 (every RVE), including the final stress evaluation.  Inputs
(plans, macro strains) are resident on the device before the timed region.

The headline value is the learned, batched path: the warm-start network
(trained first, untimed, on the method's own solves of separate training
microstructures) runs inside every timed step (features, BF16 inference,
scatter), then the batched solve.  Beside it: the cold-start batched rate,
the Born-prior-only rate, the plain single-RVE rates (cold and learned), the
iteration statistics of each start, the training cost, and the effective
stress difference between learned and cold starts.

The timed steps record no per-kernel events (events around every launch
cost about 9 % of the step); --graph 1 replays each chunk of iterations from a
hipGraph (measured equal to eager launches).  Prints one JSON
line (rank 0).  It also reports the per-kernel roofline of the dominant kernel
(HIP events around each of its launches on the solve stream, in an eager
repetition of the same steps right after the timed ones; algorithmic bytes
counted from the plans and iteration counts), the plan-construction cost, and
the FP64 CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import gc
import json
import math
import os
import subprocess
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TF = 157.3
FP32_NONPACKED_TF = 78.6
METRIC = "RVE solves/s at residual 1e-6, 256² 2D 5% freqs: learned/batched vs plain"
GRID = 256
M_FREQ = int(math.ceil(0.05 * GRID * GRID))
TOL = 1e-6


def _gen(i):
    return synth.metric_rve(i, n=GRID)


def workload(count, workers=8):
    with ProcessPoolExecutor(max_workers=workers) as ex:
        items = list(ex.map(_gen, range(count), chunksize=8))
    gs = [g for g, _ in items]
    ebs = np.stack([e for _, e in items])
    return gs, ebs


def settle_heap():
    """Collect the Python heap and exempt what is left from later
    collections: the workload, training and evaluation stages leave millions
    of long-lived objects, and a full collection over them (tens of ms) must
    not land inside a timed region."""
    gc.collect()
    gc.freeze()


def itstats(it):
    return {"mean": float(np.mean(it)), "p50": float(np.percentile(it, 50)),
            "p95": float(np.percentile(it, 95)), "max": int(np.max(it))}


def phases():
    import paper_2103_10203_amd as mor
    lm, mm = synth.phase_lame(synth.MATRIX_E, synth.MATRIX_NU)
    li, mi = synth.phase_lame(synth.FIBRE_E, synth.FIBRE_NU)
    return [mor.Phase(lm, mm), mor.Phase(li, mi)]


def _oracle_solve(args):
    """One oracle solve of the workload (pattern construction timed apart)."""
    g, eb = args
    from oracle import material, pattern, solver
    lm, mm = synth.phase_lame(synth.MATRIX_E, synth.MATRIX_NU)
    li, mi = synth.phase_lame(synth.FIBRE_E, synth.FIBRE_NU)
    ph = (material.Phase(lm, mm), material.Phase(li, mi))
    tp = time.perf_counter()
    p = pattern.build_pattern(g, M_FREQ)
    ts = time.perf_counter()
    r = solver.solve(g, ph, solver.macro_tensor(eb, 2), mask=p.mask(), tol=TOL)
    te = time.perf_counter()
    return te - ts, ts - tp, r.iterations, solver.tensor_comps(r.sigma_bar, 2, with_s33=True)


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(gs, ebs, budget_s=12.0):
    """The FP64 oracle, as it stands, on the same workload: first one thread
    (NumPy's FFT is single-threaded), then one oracle process per core over
    further RVEs of the workload.  Returns the line's cpu_baseline object and
    the oracle's effective stresses of the RVEs it solved (index -> sigma_bar)."""
    done, t_solve, t_plan, its, sig = 0, 0.0, 0.0, [], {}
    t0 = time.perf_counter()
    while done < len(gs) and time.perf_counter() - t0 < budget_s:
        ts, tp, it, sb = _oracle_solve((gs[done], ebs[done]))
        t_solve += ts
        t_plan += tp
        its.append(it)
        sig[done] = sb
        done += 1
    single = done / t_solve
    workers = max(1, min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", "16"))))
    n_all = min(len(gs) - done, workers * max(2, int(round(budget_s * single))))
    idx = list(range(done, done + n_all))
    all_rate = None
    if n_all > 0:
        with ProcessPoolExecutor(max_workers=workers) as ex:
            list(ex.map(_oracle_solve, [(gs[0], ebs[0])] * workers))  # start the workers and import
            t = time.perf_counter()
            res = list(ex.map(_oracle_solve, [(gs[i], ebs[i]) for i in idx]))
            wall = time.perf_counter() - t
        all_rate = n_all / wall
        for i, r in zip(idx, res):
            its.append(r[2])
            sig[i] = r[3]
    base = {
        "value": all_rate if all_rate else single,
        "unit": "RVE solves/s",
        "cores": workers if all_rate else 1,
        "kind": "oracle",
        "sample": f"held-out 256x256 RVEs of the same workload (M={M_FREQ}, residual {TOL:g}), FP64 NumPy "
                  f"oracle: {done} solved on one thread, then {n_all} by {workers} single-threaded oracle "
                  f"processes (one per core); pattern construction excluded (single thread with it: "
                  f"{done / (t_solve + t_plan):.3f}/s)",
        "single_thread": {"value": single, "cores": 1, "rves": done},
        "all_cores": {"value": all_rate, "cores": workers, "rves": n_all},
        "cpu_model": cpu_model(),
        "os_cpu_count": os.cpu_count(),
        "mean_iterations": float(np.mean(its)),
    }
    return base, sig


SOLVE_SOURCES = ("fft_lds.h", "fft_reg.h", "mor_internal.h", "solve_fast.h", "solve_kernels.h", "solve.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "solve_256x256_m3277_b1024_hbm_traffic.txt")


def solve_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in SOLVE_SOURCES:
        with open(os.path.join(ROOT, "paper_2103_10203_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


VALU_FILE = os.path.join(ROOT, "profiles", "solve_256x256_m3277_b1024_valu_issue.txt")


def measured_valu_issue(kernel):
    """Fraction of the chip's VALU issue slots `kernel` used (rocprofv3 SQ
    counters, committed summary), or None when the kernel sources changed."""
    if not os.path.exists(VALU_FILE):
        return None
    want = solve_source_hash()
    with open(VALU_FILE) as fh:
        for line in fh:
            f = line.split()
            if len(f) == 6 and f[0] == "valu" and f[1] == kernel and f[5] == want:
                return float(f[2])
    return None


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE/WRITE_SIZE
    summary (copy-calibrated), or None when the kernel sources changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    want = solve_source_hash()
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            f = line.split()
            if len(f) == 6 and f[0] == "traffic" and f[1] == kernel and f[5] == want:
                return float(f[2])
    return None


SOLVE_KW = {}  # transform / precision / schedule of every solve (command line)
BATCH_KW = {}  # options of the batched solves only


def timed_batched(mor, plans, plan_of, ebs, ph, steps, warmup, warm_fn=None):
    """Batched solves of the whole workload; warm_fn (if given) builds the warm
    start inside the timed region (features, network, scatter).

    The throughput is timed without per-kernel events (optionally with
    hipGraph replay of the iteration chunks); the per-kernel durations of the
    roofline come from a repetition of the same steps, launched eagerly with
    HIP events around every kernel on the solve stream."""
    import torch

    def step(**kw):
        w = warm_fn() if warm_fn else None
        return mor.solve_multi(plans, plan_of, ebs, ph, TOL, warm_start=w, **SOLVE_KW, **kw)

    for _ in range(warmup):
        step(**BATCH_KW)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(steps):
        out = step(**BATCH_KW)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert out.status == mor.MOR_OK, out.status
    # profiled repetition: eager launches, events around each kernel
    mor.profile_reset()
    mor.profile_enable(True)
    for _ in range(steps):
        prof = step(use_graph=0)
    torch.cuda.synchronize()
    mor.profile_enable(False)
    assert np.array_equal(prof.iterations, out.iterations)
    kern = {k: mor.profile_query(k) for k in ("row", "col", "final", "init")}
    return out, elapsed, kern


def end_to_end_pipelined(mor, gs, ebs, ph, batch, s_plan, warm_fn=None):
    """End to end over several batches as an FE-FFT driver would run them:
    the plans of batch k+1 are built (host checks and staging, plan kernels on
    the stream s_plan, from a second host thread) while batch k is solved on
    the current stream.  Returns solves/s over the whole run, plan
    construction of the first batch (not overlapped) included."""
    import queue
    import threading

    import torch
    nb = len(gs) // batch
    s_solve = torch.cuda.current_stream()
    q = queue.Queue(maxsize=2)
    err = []

    def producer():
        try:
            with torch.cuda.stream(s_plan):
                for k in range(nb):
                    plans = mor.make_plans(gs[k * batch:(k + 1) * batch], M_FREQ, stream=s_plan)
                    s_plan.synchronize()
                    q.put(plans)
        except Exception as e:  # noqa: BLE001 - reported by the consumer
            err.append(e)
            q.put(None)

    keep = []
    marks = []
    po = np.arange(batch)
    torch.cuda.synchronize()
    t = time.perf_counter()
    th = threading.Thread(target=producer)
    th.start()
    with torch.cuda.stream(s_solve):
        for k in range(nb):
            plans = q.get()
            if plans is None:
                break
            eb = ebs[k * batch:(k + 1) * batch]
            w = warm_fn(plans, po, eb) if warm_fn else None
            out = mor.solve_multi(plans, po, eb, ph, TOL, warm_start=w, stream=s_solve, **SOLVE_KW)
            assert out.status == mor.MOR_OK, out.status
            keep.append(plans)  # released after the timed region (destroying a plan drains the device)
            marks.append(time.perf_counter() - t)
    th.join()
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    if err:
        raise err[0]
    del keep
    return nb * batch / el, nb, [round(1e3 * (b - a), 2) for a, b in zip([0.0] + marks[:-1], marks)]


def timed_single(mor, plans, ebs, ph, count, warm_fn=None, use_graph=0):
    """Plain path: one RVE per call (mor_solve), optionally warm-started and
    with the iteration chunks replayed from a hipGraph."""
    import torch

    def one(i):
        w = warm_fn(i) if warm_fn else None
        return mor.solve(plans[i], ebs[i:i + 1], ph, TOL, warm_start=w, use_graph=use_graph, **SOLVE_KW)

    for i in range(2):
        one(i)
    torch.cuda.synchronize()
    t = time.perf_counter()
    its = []
    for i in range(count):
        its.append(int(one(i).iterations[0]))
    torch.cuda.synchronize()
    return count / (time.perf_counter() - t), float(np.mean(its))


def train_network(mor, ph, ntrain, nslots, epochs, log):
    """Training data from the method's own solves on seeded training
    microstructures (seeds 0..ntrain-1), then Adam on the GPU."""
    import torch
    from paper_2103_10203_amd import warm
    cfg = warm.WarmConfig(nslots=nslots, hidden=512, epochs=epochs, batch=512)
    t = time.perf_counter()
    gs = warm.generate_microstructures(range(ntrain), n=GRID, workers=min(16, os.cpu_count() or 8))
    t_gen = time.perf_counter() - t
    log(f"generated {ntrain} training microstructures in {t_gen:.1f} s")
    data = warm.build_training_set(gs, M_FREQ, ph, nslots, log=log if ntrain >= 4096 else None)
    del gs
    log(f"training set: {data.solves} unit-strain solves, plans {data.gen_s['plans']:.1f} s, "
        f"solves {data.gen_s['solves']:.1f} s")
    net = mor.MLP(4 * nslots + 1, cfg.hidden, 18 * nslots, seed=cfg.seed)
    hist, t_train = warm.train(net, data, cfg)
    log(f"trained {epochs} epochs in {t_train:.1f} s, loss {hist[0]:.3e} -> {hist[-1]:.3e}")
    info = {"microstructures": ntrain, "unit_solves": data.solves, "gen_s": t_gen,
            "plans_s": data.gen_s["plans"], "solves_s": data.gen_s["solves"], "train_s": t_train,
            "epochs": epochs, "params": int(net.num_params), "loss_first": hist[0], "loss_last": hist[-1]}
    del data
    torch.cuda.empty_cache()
    return net, info


GOLDEN = os.path.join(ROOT, "tests", "golden")


def _golden(name):
    """Expected values written by tests/golden/make_golden.py from the FP64
    oracle (None if the fixture is missing)."""
    path = os.path.join(GOLDEN, name + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        return json.load(fh)


def _max_rel(got, want):
    got = np.atleast_2d(np.asarray(got, dtype=np.float64))
    want = np.atleast_2d(np.asarray(want, dtype=np.float64))
    d = np.max(np.abs(got[:, :want.shape[1]] - want), axis=1)
    return float(np.max(d / np.max(np.abs(want), axis=1)))


def cube128(mor, ph, timed, reps=1, variants=("fft", "dft_bf16x3")):
    """3D: 128^3 spheres (vf 0.25), M = 2 %, 8 macro strains in one
    mor_solve call, with the FFT and (if listed) the split-bf16 MFMA DFT."""
    res = {}
    g3 = synth.rsa_spheres(128, 128, 128, 8.0, 14.0, seed=7, target_vf=0.25).g
    p3 = mor.Plan(g3, int(math.ceil(0.02 * g3.size)))
    e3 = synth.macro_strains(8, 6, 1e-3, seed=3)
    G4 = _golden("c4_128")
    runs = {"fft": ({}, 1e-6), "dft_bf16x3": ({"precision": mor.PREC_BF16X3}, 1e-5)}
    for name in variants:
        kw, tol = runs[name]
        el, out = timed(lambda: mor.solve(p3, e3, ph, tol, **kw), reps)
        res[f"cube128_{name}"] = {"workload": "128³ spheres (vf 0.25), M = 2 %, 8 macro strains in one call, "
                                              f"residual {tol:g}",
                                  "solves_per_s": 8 / el, "ms": el * 1e3,
                                  "mean_iterations": float(out.iterations.mean())}
        if G4:
            e_one = np.array([G4["macro_strain"]])
            one = mor.solve(p3, e_one, ph, tol, **kw)
            res[f"cube128_{name}"]["oracle_rel_err"] = _max_rel(one.eff_stress, [G4["sigma_bar"]])
    return res


def other_configs(mor, ph):
    """Throughput of the other configured workloads (one timed call each,
    after one untimed call): the 4096-RVE uneven batch (also autotuned with
    hipGraph replay), 3D 128^3 with the FFT and the split-bf16 MFMA DFT, the
    64^2 disk in FP64 to 1e-8, and the 512^2 J2 load path.  Each result
    carries its largest effective-stress difference from the FP64 oracle
    (from the oracle's fixtures under tests/golden)."""
    import torch

    def timed(fn, reps=1):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps, r

    res = {}
    gs = [synth.rsa_fibres(n, n, n / 32, n / 16, seed=seed, target_vf=0.35).g
          for n, seed in ((128, 31), (256, 32), (384, 33))]
    plans = mor.make_plans(gs, [int(math.ceil(0.05 * g.size)) for g in gs])
    B = 4096
    po = np.arange(B) % 3
    ebs = synth.macro_strains(B, 3, 5e-3, seed=2026)
    el, out = timed(lambda: mor.solve_multi(plans, po, ebs, ph, TOL), 2)
    res["uneven_4096"] = {"workload": "4096 RVEs round robin over 128², 256², 384² fibre RVEs (vf 0.35), M = 5 %, "
                                      "one mor_solve_multi call, residual 1e-6",
                          "solves_per_s": B / el, "ms": el * 1e3, "mean_iterations": float(out.iterations.mean())}
    G3 = _golden("c3_stiffness")
    if G3:
        C = [np.array(gr["C_eff"]) for gr in G3["grids"]]
        res["uneven_4096"]["oracle_rel_err"] = _max_rel(out.eff_stress, np.stack([C[po[b]] @ ebs[b]
                                                                                 for b in range(B)]))
    # the same after the autotuner has measured every row and column variant of
    # the three sizes on this workload, with the iteration chunks replayed from
    # a captured hipGraph; the selections are put back afterwards
    keep = {(k, n): mor.tune_get(2, n, k) for k in (mor.KERNEL_ROW, mor.KERNEL_COL) for n in (128, 256, 384)}
    t = time.perf_counter()
    mor.autotune(plans, po, ebs, ph, TOL, reps=2)
    t_tune = time.perf_counter() - t
    picked = {f"{'row' if k == mor.KERNEL_ROW else 'col'}{n}": mor.tune_get(2, n, k) for (k, n) in keep}
    el, out = timed(lambda: mor.solve_multi(plans, po, ebs, ph, TOL, use_graph=1), 2)
    res["uneven_4096_autotuned_graph"] = {"solves_per_s": B / el, "ms": el * 1e3, "tune_s": t_tune,
                                          "variants": picked, "mean_iterations": float(out.iterations.mean())}
    for (k, n), v in keep.items():
        mor.tune_set(2, n, v, k)
    del plans
    res.update(cube128(mor, ph, timed))
    # the paper's 64^2 centred disk (M = 205) to its residual 1e-8, FP64 throughout
    n1 = 64
    g1 = synth.disk(n1, n1, math.sqrt(0.3 * n1 * n1 / math.pi))
    p1 = mor.Plan(g1, 205)
    e1 = synth.macro_strains(256, 3, 1e-3, seed=64)
    el, out = timed(lambda: mor.solve(p1, e1, ph, 1e-8, precision=mor.PREC_FP64))
    res["disk64_fp64_1e-8"] = {"workload": "64² centred disk (vf 0.3), M = 205, 256 macro strains in one call, "
                                           "FP64 throughout, residual 1e-8",
                               "solves_per_s": 256 / el, "ms": el * 1e3,
                               "mean_iterations": float(out.iterations.mean())}
    # against the oracle's effective stiffness of the disk (linear in the macro strain)
    G1 = _golden("disk64_stiffness")
    if G1:
        res["disk64_fp64_1e-8"]["oracle_rel_err"] = _max_rel(out.eff_stress, e1 @ np.array(G1["C_eff"]).T)
    del p1
    res["radial_vs_adapted_256"] = radial_and_compat(mor, ph, timed)
    g2 = synth.rsa_fibres(512, 512, 20.0, 40.0, seed=2103, target_vf=0.40).g
    p2 = mor.Plan(g2, int(math.ceil(0.05 * g2.size)))
    path = np.stack([[0.02 * (k + 1) / 20, 0.0, 0.0] for k in range(20)])
    lm, mm = synth.phase_lame(synth.MATRIX_E, synth.MATRIX_NU)
    li, mi = synth.phase_lame(synth.FIBRE_E, synth.FIBRE_NU)
    j2 = [mor.Phase(lm, mm, 0.25, 1.0, True), mor.Phase(li, mi)]

    def run_path():
        state = torch.zeros(5 * g2.size, dtype=torch.float32, device="cuda")
        return mor.solve_path(p2, path, j2, TOL, state)

    el, out = timed(run_path)
    res["j2_512_path"] = {"workload": "512² J2 fibres (vf 0.4), M = 5 %, 20 load steps to 2 %, residual 1e-6",
                          "ms_per_path": el * 1e3, "iterations": int(out.iterations.sum())}
    G2 = _golden("c2_j2_512")
    if G2:
        case = G2["cases"][str(p2.info["M"])]
        res["j2_512_path"]["oracle_rel_err"] = _max_rel(out.eff_stress, case["sigma_bar"])
    res["j2_512_paths_b64"] = j2_paths_batched(mor, j2)
    return res


def radial_and_compat(mor, ph, timed, L=16, B=256):
    """The fixed radial pattern of L lines (Sec. 4.1) against the adapted
    pattern of the same size and the full set, on one 256^2 fibre
    microstructure with B macro strains, and the compatibility step (one
    full-set pass) from the radial solution: solves/s of each, and the
    largest effective-stress difference from the full-set solution."""
    g, _ = synth.metric_rve(0)
    eb = synth.macro_strains(B, 3, 5e-3, seed=5)
    rad = mor.Plan(g, 1, radial_lines=L)
    ada = mor.Plan(g, rad.info["M_actual"])
    full = mor.Plan(g, g.size)
    el_f, out_f = timed(lambda: mor.solve(full, eb, ph, TOL))
    el_r, out_r = timed(lambda: mor.solve(rad, eb, ph, TOL, want_coeffs=True))
    el_a, out_a = timed(lambda: mor.solve(ada, eb, ph, TOL))
    el_c, out_c = timed(lambda: mor.compat(rad, full, out_r.coeffs, eb, ph, want_fields=False))
    ref = out_f.eff_stress
    return {"workload": f"256² fibre RVE, {B} macro strains in one call, residual {TOL:g}; radial pattern of {L} "
                        f"lines (M = {rad.info['M_actual']}, {100 * rad.info['M_actual'] / g.size:.2f} %) vs the "
                        "adapted pattern of the same size vs the full set; compatibility step from the radial "
                        "solution",
            "solves_per_s": {"radial": B / el_r, "adapted": B / el_a, "full_set": B / el_f,
                             "compat_step": B / el_c},
            "mean_iterations": {"radial": float(out_r.iterations.mean()), "adapted": float(out_a.iterations.mean()),
                                "full_set": float(out_f.iterations.mean())},
            "eff_stress_rel_diff_vs_full": {"radial": _max_rel(out_r.eff_stress, ref),
                                            "adapted": _max_rel(out_a.eff_stress, ref),
                                            "radial_then_compat": _max_rel(out_c.eff_stress, ref)}}


def j2_paths_batched(mor, j2, B=64, R=0.05):
    """Load paths of B integration points on the 512^2 J2 microstructure in
    one mor_solve_path_multi call: 20 steps to a macro strain of norm 2 %
    along seeded random directions (the first uniaxial).  Reports ms per
    path and the row kernel's share of the HBM peak on its algorithmic bytes
    (J2 state included), from HIP events around its launches."""
    import torch
    g2 = synth.rsa_fibres(512, 512, 20.0, 40.0, seed=2103, target_vf=0.40).g
    p2 = mor.Plan(g2, int(math.ceil(R * g2.size)))
    rng = np.random.default_rng(B)
    dirs = rng.normal(size=(B, 3))
    dirs[0] = [1.0, 0.0, 0.0]
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    paths = np.stack([np.stack([0.02 * d * (k + 1) / 20 for k in range(20)]) for d in dirs])
    state = torch.zeros(5 * g2.size * B, dtype=torch.float32, device="cuda")
    mor.solve_path_multi([p2], [0] * B, paths[:, :2], j2, TOL, state)  # warm-up
    state.zero_()
    torch.cuda.synchronize()
    t = time.perf_counter()
    out = mor.solve_path_multi([p2], [0] * B, paths, j2, TOL, state)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    assert out.status == mor.MOR_OK, out.status
    state.zero_()
    mor.profile_reset()
    mor.profile_enable(True)
    mor.solve_path_multi([p2], [0] * B, paths, j2, TOL, state)
    torch.cuda.synchronize()
    mor.profile_enable(False)
    row = mor.profile_query("row")
    gbs = row["bytes"] / (row["ms"] * 1e-3) / 1e9
    return {"workload": f"{B} integration points on the 512² J2 fibres (vf 0.4), M = {R:.0%}, 20 load steps "
                        "to |eps| = 2 % along seeded random directions, one mor_solve_path_multi call, "
                        "residual 1e-6",
            "ms_per_path": el * 1e3 / B, "ms_per_call": el * 1e3, "iterations": int(out.iterations.sum()),
            "row_us_per_launch": row["ms"] * 1e3 / max(row["launches"], 1), "row_GBps": gbs,
            "row_hbm_frac": gbs / HBM_PEAK_GBS}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--single", type=int, default=32, help="RVEs timed one launch each (plain path)")
    ap.add_argument("--train", type=int, default=20000,
                    help="training microstructures of the warm-start network (0: cold start only)")
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--nslots", type=int, default=256,
                    help="network slots (ranked conjugate pairs); the Born prior covers every pair")
    ap.add_argument("--transform", choices=["auto", "fft", "dft"], default="auto",
                    help="last-axis transform of every solve (auto = the pruned FFT)")
    ap.add_argument("--precision", choices=["fp32", "bf16x3"], default="fp32",
                    help="bf16x3: split-bf16 MFMA partial DFT (implies --transform dft)")
    ap.add_argument("--graph", type=int, default=0,
                    help="1: replay each chunk of iterations of the batched solves from a hipGraph")
    ap.add_argument("--schedule", choices=["grid", "persistent"], default="grid",
                    help="workgroup schedule of the iteration kernels")
    ap.add_argument("--no-other-configs", action="store_true",
                    help="skip the timings of the other configured workloads")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--only", choices=["j2paths", "cube128"], default=None,
                    help="run one other workload alone and print its JSON (for profiling runs)")
    ap.add_argument("--e2e-batches", type=int, default=4,
                    help="batches of the pipelined end-to-end run (plans of the next batch built meanwhile)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the batched RVE solves would shard across GPUs without per-iteration "
              "communication).", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    import paper_2103_10203_amd as mor
    from paper_2103_10203_amd import warm

    if args.only == "j2paths":
        lm, mm = synth.phase_lame(synth.MATRIX_E, synth.MATRIX_NU)
        li, mi = synth.phase_lame(synth.FIBRE_E, synth.FIBRE_NU)
        print(json.dumps(j2_paths_batched(mor, [mor.Phase(lm, mm, 0.25, 1.0, True), mor.Phase(li, mi)])))
        return
    if args.only == "cube128":
        def timed_only(fn, reps=1):
            fn()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                r = fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t) / reps, r
        print(json.dumps(cube128(mor, phases(), timed_only, reps=3, variants=("fft",))))
        return

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    global TOL
    SOLVE_KW["transform"] = {"auto": mor.TRANSFORM_AUTO, "fft": mor.TRANSFORM_FFT,
                             "dft": mor.TRANSFORM_DFT}[args.transform]
    SOLVE_KW["precision"] = mor.PREC_BF16X3 if args.precision == "bf16x3" else mor.PREC_FP32
    SOLVE_KW["schedule"] = mor.SCHED_PERSISTENT if args.schedule == "persistent" else mor.SCHED_GRID
    BATCH_KW["use_graph"] = args.graph
    dft = args.transform == "dft" or args.precision == "bf16x3"
    if args.precision == "bf16x3":
        TOL = 1e-5  # split-bf16 products set a residual floor near 1e-6

    B = args.batch
    t = time.perf_counter()
    gs, ebs = workload(B)
    t_gen = time.perf_counter() - t
    ph = phases()
    log(f"generated {B} held-out RVEs in {t_gen:.1f} s")

    # plans: all RVEs in one batched construction (end to end); one
    # mor_plan_create per RVE on a sample is reported beside it
    nseq = min(B, 128)
    warmup_plans = mor.make_plans(gs[:4], M_FREQ)  # first launches load the plan kernels
    del warmup_plans
    torch.cuda.synchronize()
    t = time.perf_counter()
    seq = [mor.Plan(g, M_FREQ) for g in gs[:nseq]]
    torch.cuda.synchronize()
    plan_ms_seq = (time.perf_counter() - t) * 1e3 / nseq
    del seq
    torch.cuda.synchronize()
    t = time.perf_counter()
    plans = mor.make_plans(gs, M_FREQ)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t) * 1e3 / B
    plan_of = np.arange(B)

    # cold start, batched
    settle_heap()
    cold, el_cold, kern_cold = timed_batched(mor, plans, plan_of, ebs, ph, args.steps, args.warmup)
    cold_rate = B * args.steps / el_cold
    log(f"cold batched: {cold_rate:.0f} solves/s, mean iterations {cold.iterations.mean():.2f}")

    # prior alone (Born term, zero network output)
    S = args.nslots
    born_fn = lambda: warm.born_warm(plans, plan_of, ebs, ph, S)  # noqa: E731
    born, el_born, _ = timed_batched(mor, plans, plan_of, ebs, ph, args.steps, 1, born_fn)
    born_rate = B * args.steps / el_born

    learned = None
    net = None
    if args.train > 0:
        net, tinfo = train_network(mor, ph, args.train, S, args.epochs, log)
        warm_fn = lambda: warm.predict_warm(net, plans, plan_of, ebs, ph, S)  # noqa: E731
        settle_heap()
        hot, el_hot, kern_hot = timed_batched(mor, plans, plan_of, ebs, ph, args.steps, args.warmup, warm_fn)
        hot_rate = B * args.steps / el_hot
        log(f"learned batched: {hot_rate:.0f} solves/s, mean iterations {hot.iterations.mean():.2f}")
        dstress = float(np.max(np.abs(hot.eff_stress - cold.eff_stress)) / np.max(np.abs(cold.eff_stress)))
        learned = {"rate": hot_rate, "elapsed": el_hot, "kern": kern_hot, "out": hot, "train": tinfo,
                   "eff_stress_rel_diff_vs_cold": dstress}

    # iterations on 2 batches of held-out RVEs (the timed batch and the next
    # one): cold, prior alone and learned start on the same microstructures
    heldout = None
    if learned is not None:
        gs_n, ebs_n = workload(2 * B)
        gs_n, ebs_n = gs_n[B:], ebs_n[B:]
        plans_n = mor.make_plans(gs_n, M_FREQ)
        its = {"cold": [cold.iterations], "born_prior": [born.iterations], "learned": [learned["out"].iterations]}
        starts = {"cold": None,
                  "born_prior": lambda: warm.born_warm(plans_n, plan_of, ebs_n, ph, S),
                  "learned": lambda: warm.predict_warm(net, plans_n, plan_of, ebs_n, ph, S)}
        for key, fn in starts.items():
            o = mor.solve_multi(plans_n, plan_of, ebs_n, ph, TOL, warm_start=fn() if fn else None, **SOLVE_KW)
            assert o.status == mor.MOR_OK, o.status
            its[key].append(o.iterations)
        heldout = {"rves": 2 * B, "iterations": {k: itstats(np.concatenate(v)) for k, v in its.items()}}
        del plans_n, gs_n, ebs_n
        log(f"held-out {2 * B}: mean iterations cold {heldout['iterations']['cold']['mean']:.3f}, "
            f"learned {heldout['iterations']['learned']['mean']:.3f}")

    # end to end: plan construction of the next batch overlapped with the solve
    # of the current one (second stream, second host thread)
    e2e_pipe = None
    if args.e2e_batches > 0:
        gs_e, ebs_e = workload(args.e2e_batches * B)
        wf = None
        if learned is not None:
            wf = lambda pl, po_, eb: warm.predict_warm(net, pl, po_, eb, ph, S)  # noqa: E731
        s_plan = torch.cuda.Stream()
        settle_heap()
        end_to_end_pipelined(mor, gs_e[:2 * B], ebs_e[:2 * B], ph, B, s_plan, wf)  # warm-up: buffers, pools
        rate, nbat, bms = end_to_end_pipelined(mor, gs_e, ebs_e, ph, B, s_plan, wf)
        steady = (B * (len(bms) - 2) / (sum(bms[2:]) * 1e-3)) if len(bms) > 2 else None
        e2e_pipe = {"solves_per_s": rate, "batches": nbat, "batch": B, "batch_done_ms": bms,
                    "steady_solves_per_s": steady,
                    "steady_note": "batches after the first two (the pipeline is full: plans of the next batch "
                                   "overlap the solve of this one)",
                    "note": "plans of batch k+1 built on a second stream from a second host thread while batch "
                            "k is solved (learned start when trained); first batch's plans not overlapped"}
        del gs_e, ebs_e
        log(f"end to end, pipelined: {rate:.0f} solves/s")

    if learned is not None:
        head_out, head_el, kern, start = learned["out"], learned["elapsed"], learned["kern"], "learned"
    else:
        head_out, head_el, kern, start = cold, el_cold, kern_cold, "cold"
    value = B * args.steps / head_el
    ms_per_step = head_el * 1e3 / args.steps
    iters = head_out.iterations
    dom = max(kern, key=lambda k: kern[k]["ms"])
    kd = kern[dom]
    achieved = kd["bytes"] / (kd["ms"] * 1e-3) / 1e9 if kd["ms"] > 0 else 0.0
    traffic = measured_traffic(dom)
    hbm = {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
           "traffic": traffic,
           "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
           "bytes_note": "algorithmic bytes per RVE-iteration: rows (16 C nlast + L) for the row kernel, "
                         "ncol 16 C n0 + ncoef (16 C + 17) for the column kernel"}
    # The fused row kernel keeps the fields in registers: it is bound by
    # VALU issue, so its roofline is the FP32 vector peak.  Algorithmic flops
    # per RVE-iteration: the inverse and forward real FFTs of every row and
    # strain component (2.5 L log2 L each) and the Hooke law (25 per point).
    def row_flops(p):
        L = p.shape[-1]
        return p.ncomp * (p.N // L) * 2 * 2.5 * L * math.log2(L) + 25.0 * p.N

    row_fl = args.steps * sum(row_flops(plans[plan_of[b]]) * int(it) for b, it in enumerate(head_out.iterations))
    kr = kern["row"]
    alu = row_fl / (kr["ms"] * 1e-3) / 1e12 if kr["ms"] > 0 else 0.0
    roof = {"bound": "alu", "kernel": "row", "achieved": alu, "peak": FP32_PEAK_TF, "unit": "TFLOP/s",
            "frac": alu / FP32_PEAK_TF, "traffic": measured_traffic("row"),
            "frac_nonpacked": alu / FP32_NONPACKED_TF,
            "flops_note": "per RVE-iteration rows * C * 2 * 2.5 L log2 L + 25 N (FFT-path flops of the fused "
                          "row pass); peak = FP32 vector 157.3 TFLOP/s; frac_nonpacked against the 78.6 "
                          "TFLOP/s that FP32 FMAs reach without packed instructions (not generated here)",
            "timing": "HIP events around every launch of the kernel in an eager repetition of the timed steps",
            "avg_launch_us": kr["ms"] * 1e3 / max(kr["launches"], 1), "launches": kr["launches"],
            "valu_issue_frac": measured_valu_issue("row"),
            "valu_note": "share of the 1024 SIMDs' VALU issue slots the kernel used (rocprofv3 SQ_INSTS_VALU, "
                         "SQ_BUSY_CYCLES); near 1 means arithmetic issue, not HBM, bounds it",
            "hbm": dict(hbm, kernel=dom)}
    if dft:
        # the last-axis stage is two dense GEMMs: 8 C rows nlast L flops per RVE-iteration
        fl = sum(8.0 * p.ncomp * (p.N // p.shape[-1]) * p.info["n_last"] * p.shape[-1] * it
                 for p, it in zip(plans, head_out.iterations)) * args.steps
        kr = kern["row"]
        bf = args.precision == "bf16x3"
        mfma = fl * (3.0 if bf else 1.0) / (kr["ms"] * 1e-3) / 1e12
        peak = 2500.0 if bf else 157.3
        roof = {"bound": "mfma", "kernel": "row (DFT GEMMs + pointwise)", "achieved": mfma, "peak": peak,
                "unit": "TFLOP/s", "frac": mfma / peak, "traffic": None,
                "flops_note": "MFMA flops (bf16x3: three bf16 products per FP32 product)",
                "avg_launch_us": kr["ms"] * 1e3 / max(kr["launches"], 1), "launches": kr["launches"]}

    # plain path: one RVE per launch, cold and warm
    ns = min(args.single, B)
    single_cold = single_warm = single_graph = None
    if ns > 0:
        single_cold = timed_single(mor, plans, ebs, ph, ns)
        single_graph = timed_single(mor, plans, ebs, ph, ns, use_graph=1)
        if net is not None:
            single_warm = timed_single(
                mor, plans, ebs, ph, ns,
                lambda i: warm.predict_warm(net, [plans[i]], [0], ebs[i:i + 1], ph, S))

    if args.copy_mib > 0:
        n = args.copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    start_desc = ("learned warm start (Born prior + MLP correction, BF16 MFMA inference inside the timed step)"
                  if start == "learned" else "cold start")
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "RVE solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3" if args.precision == "bf16x3" else "f32",
        "data": "synthetic",
        "config": {
            "workload": f"held-out random-fibre RVEs {GRID}x{GRID} (vf~U[0.2,0.5], r~U[8,16] px), "
                        f"adapted pattern M={M_FREQ} (5%), batch {B} in one mor_solve_multi call, "
                        f"residual {TOL:g}, {start_desc}",
            "grid": [GRID, GRID],
            "M": M_FREQ,
            "batch": B,
            "tol": TOL,
            "start": start,
            "fields": "FP32, FP64 residual and stress sums",
            "transform": args.transform, "precision": args.precision, "schedule": args.schedule,
            "hipgraph": bool(args.graph),
        },
        "roofline": roof,
        "kernels": {k: {"ms": v["ms"], "launches": v["launches"],
                        "GBps": (v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 else 0.0}
                    for k, v in kern.items()},
        "iterations": itstats(iters),
        "table_solves_per_s": {
            "batched_cold": cold_rate,
            "batched_born_prior": born_rate,
            "batched_learned": learned["rate"] if learned else None,
            "single_cold": single_cold[0] if single_cold else None,
            "single_cold_hipgraph": single_graph[0] if single_graph else None,
            "single_learned": single_warm[0] if single_warm else None,
        },
        "learned_vs_plain": {
            "vs_batched_cold": (learned["rate"] / cold_rate) if learned else None,
            "vs_single_cold": (learned["rate"] / single_cold[0]) if (learned and single_cold) else None,
        },
        "iterations_by_start": {
            "cold": itstats(cold.iterations),
            "born_prior": itstats(born.iterations),
            "learned": itstats(learned["out"].iterations) if learned else None,
        },
        "heldout_iterations": heldout,
        "plan_ms_per_rve": plan_ms,
        "plan_ms_per_rve_single_calls": plan_ms_seq,
        "end_to_end_solves_per_s": 1.0 / (1.0 / value + plan_ms * 1e-3),
        "end_to_end_pipelined": e2e_pipe,
        "workload_gen_s": t_gen,
    }
    if learned:
        line["training"] = learned["train"]
        line["eff_stress_rel_diff_learned_vs_cold"] = learned["eff_stress_rel_diff_vs_cold"]
    if not args.no_other_configs:
        line["other_configs"] = other_configs(mor, ph)
    if not args.no_cpu_baseline:
        base, osig = cpu_baseline(gs, ebs, args.cpu_budget)
        line["cpu_baseline"] = base
        idx = sorted(osig)
        want = np.stack([osig[i] for i in idx])

        def rel_err(out):
            d = np.max(np.abs(out.eff_stress[idx, :want.shape[1]] - want), axis=1)
            return float(np.max(d / np.max(np.abs(want), axis=1)))

        line["oracle_rel_err"] = {
            "eff_stress": {"learned": rel_err(head_out) if learned else None, "cold": rel_err(cold),
                           "born_prior": rel_err(born)},
            "rves": len(idx), "oracle_tol": TOL,
            "note": "largest effective-stress difference of the GPU from the FP64 oracle over the RVEs the "
                    "oracle solved, relative to each RVE's largest component (both stop at the same residual)"}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
