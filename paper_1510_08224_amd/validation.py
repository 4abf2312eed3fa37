"""Steady natural convection in the square cavity against the paper's
Table 3 (Sec. 3.4), on the GPU.

    python -m paper_1510_08224_amd.validation [--md out.md]

For each row of Table 3 (Ra = 1e3 on 128^2, 1e4 on 192^2, 1e5 and 1e6 on
256^2; Pr = 0.71, u_c = 0.1, hot left and cold right walls, adiabatic top
and bottom) and each wall family (link-wise halfway walls, and the paper's
non-equilibrium extrapolation), the solver runs in FP64 until the residual
over 20000 steps falls below 1e-11, then reports the mean Nusselt number
of both walls (Eq. 39), the largest local one on the cold (right) wall and
its position (the wall the paper reports), the largest horizontal velocity on the vertical centre line and
the largest vertical velocity on the horizontal centre line in units of
alpha / L, with their positions in units of L.  Node positions: (i + 1/2)/N
for halfway walls, i/(N - 1) for walls through the edge nodes; centre lines
average the two middle columns (rows).
"""
from __future__ import annotations

import argparse
import json

import numpy as np

from . import lbm
from . import workloads as W

# The "Present" rows of Table 3 (Sec. 3.4): Ra, N, ux_max, y, uy_max, x,
# Nu_max, y(Nu_max), Nu_mean.
TABLE3 = {
    1e3: (128, 3.6528, 0.8125, 3.7004, 0.1797, 1.5005, 0.9141, 1.1161),
    1e4: (192, 16.177, 0.8229, 19.6184, 0.1198, 3.5301, 0.8542, 2.2447),
    1e5: (256, 34.6891, 0.8555, 68.5034, 0.0664, 7.7480, 0.9219, 4.5273),
    1e6: (256, 64.6968, 0.8516, 219.149, 0.0391, 17.6722, 0.9648, 8.8258),
}


def steady_cavity(ra: float, n: int, nee: bool, tol: float = 1e-11, check: int = 20000,
                  max_steps: int = 4_000_000) -> dict:
    pb = W.cavity(n, ra)
    if nee:
        pb = W.with_nee_walls(pb)
    S = lbm.Solver(n, n, "f64")
    try:
        S.set_params(pb)
        L = S.derived()["length"]
        alpha = pb.u_c * L / np.sqrt(ra * pb.pr)        # Eq. 40: Pr = nu/alpha, Ra = u_c^2 L^2/(nu alpha)
        S.residual()
        steps, r = 0, float("inf")
        while steps < max_steps and r > tol:
            S.step(check)
            steps += check
            r, _ = S.residual()
        _, ux, uy, _ = S.moments()
        c = np.arange(n) / (n - 1) if nee else (np.arange(n) + 0.5) / n
        i0, i1 = (n - 1) // 2, n // 2
        uxc = 0.5 * (ux[:, i0] + ux[:, i1]) * L / alpha
        uyc = 0.5 * (uy[i0, :] + uy[i1, :]) * L / alpha
        j, k = int(np.argmax(uxc)), int(np.argmax(uyc))
        nu_left = S.nusselt(lbm.LBM_LEFT)[0]
        nu_right, nu_max, i_max = S.nusselt(lbm.LBM_RIGHT)
        return {"ra": ra, "n": n, "walls": "nee" if nee else "link-wise", "steps": steps, "residual": r,
                "ux_max": float(uxc[j]), "y_ux_max": float(c[j]), "uy_max": float(uyc[k]), "x_uy_max": float(c[k]),
                "nu_max": nu_max, "y_nu_max": float(c[i_max]), "nu_mean_left": nu_left, "nu_mean_right": nu_right}
    finally:
        S.close()


def markdown(rows) -> str:
    out = ["# Steady heated cavity against Table 3 of the paper (MI355X, FP64)", "", "Command:", "", "```",
           "python -m paper_1510_08224_amd.validation", "```", "",
           "Each run stops when the residual over 20000 steps falls below 1e-11.  Velocities in units of "
           "alpha/L on the centre lines, positions in units of L; Nu_mean of both walls (Eq. 39); Nu_max and "
           "its position on the cold (right) wall.  Paper: the \"Present\" rows of Table 3 (non-equilibrium "
           "extrapolation walls).", "",
           "| Ra | N | walls | steps | ux_max (paper) | y | uy_max (paper) | x | Nu_max (paper) | y (paper) | "
           "Nu_mean left / right (paper) |",
           "|---:|---:|---|---:|---|---:|---|---:|---|---:|---|"]
    for r in rows:
        p = TABLE3[r["ra"]]
        out.append(f"| {r['ra']:g} | {r['n']} | {r['walls']} | {r['steps']} | {r['ux_max']:.4f} ({p[1]}) | "
                   f"{r['y_ux_max']:.4f} ({p[2]}) | {r['uy_max']:.4f} ({p[3]}) | {r['x_uy_max']:.4f} ({p[4]}) | "
                   f"{r['nu_max']:.4f} ({p[5]}) | {r['y_nu_max']:.4f} ({p[6]}) | "
                   f"{r['nu_mean_left']:.5f} / {r['nu_mean_right']:.5f} ({p[7]}) |")
    return "\n".join(out) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--md", default=None)
    a = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    rows = []
    for ra, p in TABLE3.items():
        for nee in (False, True):
            rows.append(steady_cavity(ra, p[0], nee))
            print(json.dumps(rows[-1]), flush=True)
    if a.md:
        with open(a.md, "w") as fh:
            fh.write(markdown(rows))


if __name__ == "__main__":
    main()
