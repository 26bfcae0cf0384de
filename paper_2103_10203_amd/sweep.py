"""Reduced-versus-full error sweep (paper Sec. 5): the macroscopic and
microscopic errors E_bar and E of reduced solutions against the solution with
the full set of frequencies, for the fixed radial pattern (Sec. 4.1) and the
geometrically adapted pattern (Sec. 4.2) at equal numbers of frequencies,
before and after the compatibility step (Secs. 4.1, 5.1).  2D elastic and
elasto-plastic (a load path, errors at its last step; figs. OneIncError and
ErrorPlast) and 3D elastic (adapted patterns only, as in Sec. 5.3).

Orchestration only: plans, solves, the compatibility step and the error
measures all run in the library (mor_plan_create, mor_solve /
mor_solve_path, mor_compat, mor_stress_error).

    python -m paper_2103_10203_amd.sweep [--n 256] [--j2-steps 0] [--lines 1,2,4]

prints one JSON document with the sweep of the 2D one-inclusion example of
Sec. 5.1 (centred disk, lambda = mu = 2 GPa inclusion in lambda = mu = 1 GPa
matrix, eps_11 = 0.01, eps_22 = -0.01), or with --j2-steps of the
elasto-plastic example of Sec. 5.2 on seeded random fibres.
"""
from __future__ import annotations

import argparse
import json
import math

import numpy as np

from . import _native as mor

DEFAULT_LINES = (1, 2, 4, 8, 16, 32, 64, 128)


def _solve(plan, eb, phases, tol, steps):
    """Fields and coefficients of the solution (steps = 0: one elastic solve;
    else the last step of a load path of `steps` equal increments), and the
    committed J2 state that step iterated with (None for steps = 0)."""
    import torch
    if steps == 0:
        out = mor.solve(plan, eb[None, :], phases, tol, want_fields=True, want_coeffs=True)
        return out, None
    nst = 5 if plan.ndim == 2 else 7
    state = torch.zeros(nst * plan.N, dtype=torch.float32, device="cuda")
    path = np.stack([eb * (k + 1) / steps for k in range(steps)])
    if steps > 1:
        mor.solve_path(plan, path[:-1], phases, tol, state, allow=())
    committed = state.clone()
    last = mor.solve_path(plan, path[-1:], phases, tol, state, want_fields=True, want_coeffs=True, allow=())
    last.strain = last.strain[None]
    last.stress = last.stress[None]
    last.coeffs = last.coeffs[None]
    return last, committed


def error_sweep(g, phases, macro_strain, lines=DEFAULT_LINES, fractions=None, tol=1e-6, compat=True,
                j2_steps=0, skip_rel=1e-12):
    """Rows of E_bar and E for each pattern.  2D: for every L in `lines` the
    radial pattern of L lines and the adapted pattern with the same number of
    frequencies; 3D: adapted patterns with M = ceil(R N) for R in
    `fractions`.  j2_steps > 0 runs a load path of that many equal steps to
    `macro_strain` (phases with J2) and measures at its last step."""
    g = np.ascontiguousarray(g, dtype=np.uint8)
    eb = np.asarray(macro_strain, dtype=np.float64)
    ndim = g.ndim
    N = g.size
    full = mor.Plan(g, N)
    ref, _ = _solve(full, eb, phases, tol, j2_steps)
    cases = []
    if ndim == 2:
        for L in lines:
            rp = mor.Plan(g, 1, radial_lines=L)
            cases.append(("radial", L, rp))
            cases.append(("adapted", L, mor.Plan(g, rp.info["M_actual"])))
    else:
        for R in fractions or (0.0039, 0.0078, 0.0154, 0.0306, 0.0602, 0.1164):
            cases.append(("adapted", None, mor.Plan(g, int(math.ceil(R * N)))))
    rows = []
    for kind, L, plan in cases:
        out, committed = _solve(plan, eb, phases, tol, j2_steps)
        Eb, E = mor.stress_error(out.stress, ref.stress, out.eff_stress, ref.eff_stress, ndim, skip_rel)
        row = {"kind": kind, "lines": L, "M": plan.info["M_actual"], "R": plan.info["M_actual"] / N,
               "E_bar": float(Eb[0]), "E": float(E[0]), "iterations": int(np.sum(out.iterations))}
        if compat:
            c = mor.compat(plan, full, out.coeffs, eb[None, :], phases, state=committed)
            Ebc, Ec = mor.stress_error(c.stress, ref.stress, c.eff_stress, ref.eff_stress, ndim, skip_rel)
            row.update({"E_bar_compat": float(Ebc[0]), "E_compat": float(Ec[0])})
        rows.append(row)
    return {"N": N, "shape": list(g.shape), "tol": tol, "j2_steps": j2_steps, "rows": rows,
            "reference_eff_stress": ref.eff_stress[-1].tolist()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--j2-steps", type=int, default=0,
                    help="> 0: the elasto-plastic example of Sec. 5.2 (several inclusions, J2 matrix) "
                         "as a load path of this many steps")
    ap.add_argument("--lines", type=str, default=",".join(str(v) for v in DEFAULT_LINES))
    args = ap.parse_args()
    import synth
    n = args.n
    lines = tuple(int(v) for v in args.lines.split(","))
    if args.j2_steps > 0:
        # Sec. 5.2: several inclusions, lambda = mu = 2 / 1 GPa, J2 matrix with
        # sigma_y0 = H = 0.01 GPa, eps = [[0.01, 0.002], [0.002, -0.01]]
        g = synth.rsa_fibres(n, n, n / 16, n / 8, seed=52, target_vf=0.3).g
        phases = [mor.Phase(1.0, 1.0, 0.01, 0.01, True), mor.Phase(2.0, 2.0)]
        eb = [0.01, -0.01, 0.002]
    else:
        # Sec. 5.1: one centred circular inclusion, eps_11 = 0.01, eps_22 = -0.01
        g = synth.disk(n, n, n * 0.25)
        phases = [mor.Phase(1.0, 1.0), mor.Phase(2.0, 2.0)]
        eb = [0.01, -0.01, 0.0]
    print(json.dumps(error_sweep(g, phases, eb, lines=lines, j2_steps=args.j2_steps)))


if __name__ == "__main__":
    main()
