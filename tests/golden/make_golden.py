"""Expected values of the full-size GPU tests, written from the FP64 oracle.

This script calls only the oracle (``oracle/``) and the seeded generators
(``synth/``); nothing here comes from the HIP path.  Each fixture states the
workload recipe and the passage of the paper it exercises.  Usage:

    python tests/golden/make_golden.py [c2_j2_512] [c3_stiffness] [c4_128] [disk64_stiffness]
        [headline_sample]
"""
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import material, pattern, solver  # noqa: E402

LM, MM = synth.phase_lame(synth.MATRIX_E, synth.MATRIX_NU)
LI, MI = synth.phase_lame(synth.FIBRE_E, synth.FIBRE_NU)
PH = (material.Phase(LM, MM), material.Phase(LI, MI))
PH_J2 = (material.Phase(LM, MM, sigma_y0=0.25, H=1.0, plastic=True), material.Phase(LI, MI))
NSAMPLE = 4096


def sample_points(shape, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(int(np.prod(shape)), size=NSAMPLE, replace=False))


def c2_geometry():
    return synth.rsa_fibres(512, 512, 20.0, 40.0, seed=2103, target_vf=0.40).g


def c3_geometries():
    out = []
    for n, seed in ((128, 31), (256, 32), (384, 33)):
        out.append(synth.rsa_fibres(n, n, n / 32, n / 16, seed=seed, target_vf=0.35).g)
    return out


def c4_geometry():
    return synth.rsa_spheres(128, 128, 128, 8.0, 14.0, seed=7, target_vf=0.25).g


def c4_macro():
    return synth.macro_strains(1, 6, 1e-3, seed=4)[0]


def _c2_case(R):
    g = c2_geometry()
    pts = sample_points(g.shape, 77)
    M = int(math.ceil(R * g.size))
    p = pattern.build_pattern(g, M)
    t = time.perf_counter()
    steps = solver.solve_path(g, PH_J2, solver.macro_tensor([0.02, 0.0, 0.0], 2), 20, mask=p.mask(), tol=1e-10,
                              max_iter=5000)
    sig = [solver.tensor_comps(s.sigma_bar, 2, with_s33=True).tolist() for s in steps]
    alpha = steps[-1].alpha.reshape(-1)
    ep11 = steps[-1].eps_p[..., 0, 0].reshape(-1)
    print(f"c2 M={M}: {time.perf_counter() - t:.0f} s, iterations {[s.iterations for s in steps]}", flush=True)
    return str(M), {"R": R, "M": M, "sigma_bar": sig, "alpha_sample": alpha[pts].tolist(),
                    "eps_p11_sample": ep11[pts].tolist(),
                    "alpha_mean": float(alpha.mean()), "alpha_max": float(alpha.max()),
                    "plastic_count": int(np.count_nonzero(alpha > 0.0))}


def make_c2():
    """Elasto-plastic load path (Sec. 2 J2 model, Sec. 5.2 load stepping):
    512^2 fibres, 20 equal steps to eps_11 = 2 %, M = 1, 5, 20 % of N (the
    three cases run in parallel processes)."""
    from concurrent.futures import ProcessPoolExecutor
    g = c2_geometry()
    res = {"recipe": "synth.rsa_fibres(512, 512, 20, 40, seed=2103, target_vf=0.40); J2 matrix sigma_y0 0.25 GPa, "
                     "H 1 GPa; 20 equal steps to eps_11 = 0.02; oracle tol 1e-10",
           "cite": "Sec. 2 (J2 plasticity), Sec. 4 steps a-d, Sec. 5.2 (load steps)",
           "oracle_tol": 1e-10,
           "vf": float(g.mean()), "sample_points": sample_points(g.shape, 77).tolist(), "cases": {}}
    with ProcessPoolExecutor(max_workers=3) as ex:
        for key, case in ex.map(_c2_case, (0.01, 0.05, 0.20)):
            res["cases"][key] = case
    return res


def make_c3():
    """Effective stiffness of the three microstructures of the uneven batch
    (Sec. 4 reduced scheme, linear elastic): sigma_bar = C_eff eps_bar for any
    macro strain, from three unit-strain solves."""
    res = {"recipe": "synth.rsa_fibres(n, n, n/32, n/16, seed, target_vf=0.35) for (n, seed) in "
                     "((128, 31), (256, 32), (384, 33)); M = ceil(0.05 N); oracle tol 1e-11",
           "cite": "Sec. 4 steps a-d (linear in the macro strain for Hooke phases)", "grids": []}
    for g in c3_geometries():
        M = int(math.ceil(0.05 * g.size))
        p = pattern.build_pattern(g, M)
        cols = []
        for k in range(3):
            e = np.zeros(3)
            e[k] = 1.0
            r = solver.solve(g, PH, solver.macro_tensor(e, 2), mask=p.mask(), tol=1e-11)
            cols.append(solver.tensor_comps(r.sigma_bar, 2, with_s33=True))
        res["grids"].append({"n": g.shape[0], "M": M, "C_eff": np.stack(cols, axis=1).tolist()})
        print(f"c3 n={g.shape[0]} done", flush=True)
    return res


def make_c4():
    """3D 128^3 spheres, M = 2 % (Sec. 4 reduced scheme in 3D)."""
    g = c4_geometry()
    eb = c4_macro()
    M = int(math.ceil(0.02 * g.size))
    p = pattern.build_pattern(g, M)
    t = time.perf_counter()
    r = solver.solve(g, PH, solver.macro_tensor(eb, 3), mask=p.mask(), tol=1e-10, max_iter=5000)
    pts = sample_points(g.shape, 78)
    eps = solver.tensor_comps(r.eps, 3).reshape(-1, 6)
    print(f"c4: {time.perf_counter() - t:.0f} s, {r.iterations} iterations", flush=True)
    return {"recipe": "synth.rsa_spheres(128, 128, 128, 8, 14, seed=7, target_vf=0.25); macro strain "
                      "synth.macro_strains(1, 6, 1e-3, seed=4); M = ceil(0.02 N); oracle tol 1e-10",
            "cite": "Sec. 4 steps a-d, 3D", "vf": float(g.mean()), "M": M, "macro_strain": eb.tolist(),
            "sigma_bar": solver.tensor_comps(r.sigma_bar, 3, with_s33=True).tolist(),
            "sample_points": pts.tolist(), "eps_sample": eps[pts].tolist()}


def make_disk64():
    """Effective stiffness of the 64^2 centred disk (vf 0.3), M = 205 (Sec. 4
    reduced scheme, linear elastic; the paper's single-inclusion example)."""
    n = 64
    g = synth.disk(n, n, math.sqrt(0.3 * n * n / math.pi))
    p = pattern.build_pattern(g, 205)
    cols = []
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1.0
        r = solver.solve(g, PH, solver.macro_tensor(e, 2), mask=p.mask(), tol=1e-12, max_iter=5000)
        cols.append(solver.tensor_comps(r.sigma_bar, 2, with_s33=True))
    return {"recipe": "synth.disk(64, 64, sqrt(0.3 * 64^2 / pi)); M = 205; oracle tol 1e-12",
            "cite": "Sec. 4 steps a-d, Sec. 5.1 (single inclusion)", "M": 205,
            "C_eff": np.stack(cols, axis=1).tolist()}


HEADLINE_SAMPLE = (0, 137, 300, 511, 512, 700, 901, 1023)


def _headline_case(i):
    import hashlib
    g, eb = synth.metric_rve(i)
    p = pattern.build_pattern(g, 3277)
    r = solver.solve(g, PH, solver.macro_tensor(eb, 2), mask=p.mask(), tol=1e-10, max_iter=5000)
    r6 = solver.solve(g, PH, solver.macro_tensor(eb, 2), mask=p.mask(), tol=1e-6, max_iter=5000)
    return {"index": i, "sigma_bar": solver.tensor_comps(r.sigma_bar, 2, with_s33=True).tolist(),
            "iterations_1e-6": int(r6.iterations), "unstable": bool(p.unstable),
            "sorted_idx_sha256": hashlib.sha256(p.sorted_idx.astype("<i8").tobytes()).hexdigest()}


def make_headline():
    """Sampled RVEs of the headline batch (held-out 256^2 fibre RVEs 0..1023,
    M = 3277, Sec. 4 reduced scheme): effective stress at oracle residual
    1e-10, the oracle's iteration count at 1e-6 and a digest of the pattern."""
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=8) as ex:
        cases = list(ex.map(_headline_case, HEADLINE_SAMPLE))
    return {"recipe": "synth.metric_rve(i) for i in 0..1023 (256^2, seeds 1000000 + i); M = 3277; "
                      "oracle tol 1e-10 (sigma_bar) and 1e-6 (iterations); pattern digest = sha256 of the "
                      "sorted linear indices as little-endian int64",
            "cite": "Sec. 4 steps a-d, Sec. 4.2 (pattern)", "M": 3277, "cases": cases}


MAKERS = {"c2_j2_512": make_c2, "c3_stiffness": make_c3, "c4_128": make_c4, "disk64_stiffness": make_disk64,
          "headline_sample": make_headline}

if __name__ == "__main__":
    names = sys.argv[1:] or list(MAKERS)
    for name in names:
        data = MAKERS[name]()
        with open(os.path.join(HERE, name + ".json"), "w") as fh:
            json.dump(data, fh, separators=(",", ":"))
            fh.write("\n")
        print("wrote", name, flush=True)
