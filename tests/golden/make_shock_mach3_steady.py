"""Writes shock_mach3_steady.json: the FP64 oracle's steady Mach-3 normal shock.

Calls only the oracle (``oracle.kinetics.ShockSolver``).  Set-up (appendix on
the shock: Rankine--Hugoniot states, tanh initial profile; Sec. 3.4 and Alg. 2:
LLF in local Hermite gauges with ES-BGK halves):

* Mach 3, gamma = 5/3, 1000 cells on [-20, 20] (upstream mean free path 1),
  tanh half-width 5.44, 12^3 Gauss--Hermite nodes, CFL 0.5, Pr = 2/3.

Steady state.  The paper gives no criterion.  The profile settles long before
the shock's position does (the position moves by a slow drift), and the
profiles are compared after moving both shock centres to x = 0.  The run stops
when, over the last 100 steps, both

* the density profile moved by at most ``--tol-raw`` of (n+ - n-), and
* the centred profiles of n, T and q_x (normalised as in the test, sampled on
  the offsets of the output grid) moved by at most ``--tol-centred``.

The centred change decays slowly (a few per cent per 100 steps near t = 13)
while the start-up transient is carried out through the downstream boundary,
so the centred tolerance is 1e-4: a tenth of the bar the profiles are held to.
The raw change does not go to zero: from t ~ 25 on it stays at ~2.6e-5 per 100
steps, the trace of a slow drift of the shock position (about 3e-4 per 1000
steps) while the centred profiles keep settling; its tolerance, 3e-5, only
confirms that nothing but that drift is left.
The GPU test steps its own solver the same number of steps and compares at
that time, so the golden need not be fully stationary for the comparison to be
exact up to precision.

The shock centre is where n = (n- + n+)/2, by linear interpolation between
cell centres.

Usage:
    python tests/golden/make_shock_mach3_steady.py [--checkpoint FILE]

With ``--checkpoint`` the state is saved every 500 steps and a later run
resumes from it.  The output records the sha256 of this script.
"""

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import kinetics  # noqa: E402

MACH, CELLS, X_LO, X_HI, THICK = 3.0, 1000, -20.0, 20.0, 5.44
OFFSETS = np.linspace(-12.0, 12.0, 481)     # centred sample points (0.05 apart)


def profiles(solver):
    mac = kinetics.macroscopic(solver.M, solver.g)
    return mac["n"], mac["T"], mac["qx"]


def centre(x, n, n_lo, n_hi):
    half = 0.5 * (n_lo + n_hi)
    k = int(np.nonzero((n[:-1] - half) * (n[1:] - half) <= 0.0)[0][0])
    return x[k] + (half - n[k]) / (n[k + 1] - n[k]) * (x[k + 1] - x[k])


def normalised(n, T, qx, up, down):
    (n1, _, T1), (n2, _, T2) = up, down
    return ((n - n1) / (n2 - n1), (T - T1) / (T2 - T1), qx / (n1 * T1 ** 1.5))


def centred(x, prof, xc):
    return np.stack([np.interp(OFFSETS, x - xc, p) for p in prof])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--checkpoint", default=None)
    ap.add_argument("--tol-raw", type=float, default=3e-5)
    ap.add_argument("--tol-centred", type=float, default=1e-4)
    ap.add_argument("--max-steps", type=int, default=24000)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                  "shock_mach3_steady.json"))
    args = ap.parse_args()

    s = kinetics.ShockSolver(MACH, CELLS, X_LO, X_HI, THICK)
    up, down = s.rh
    x = X_LO + s.dx * (np.arange(CELLS) + 0.5)
    step = 0
    if args.checkpoint and os.path.exists(args.checkpoint):
        z = np.load(args.checkpoint)
        s.M, s.beta, s.g = z["M"], z["beta"], z["g"]
        s.t, s.dt, step = float(z["t"]), float(z["dt"]), int(z["step"])
        print(f"resumed at step {step}, t = {s.t:.4f}", flush=True)

    hist_n, hist_c = {}, {}
    t0 = time.time()
    raw = cen = math.inf
    while step < args.max_steps:
        s.step()
        step += 1
        n, T, qx = profiles(s)
        if step % 100 == 0:
            xc = centre(x, n, up[0], down[0])
            c = centred(x, normalised(n, T, qx, up, down), xc)
            if step - 100 in hist_n:
                raw = np.max(np.abs(n - hist_n[step - 100])) / (down[0] - up[0])
                cen = float(np.max(np.abs(c - hist_c[step - 100])))
            hist_n = {step: n.copy()}
            hist_c = {step: c}
            print(f"step {step} t {s.t:.4f} centre {xc:.5f} raw {raw:.3e} centred {cen:.3e} "
                  f"wall {time.time() - t0:.0f}s", flush=True)
            if args.checkpoint and step % 500 == 0:
                np.savez(args.checkpoint + ".tmp.npz", M=s.M, beta=s.beta, g=s.g, t=s.t,
                         dt=s.dt, step=step)
                os.replace(args.checkpoint + ".tmp.npz", args.checkpoint)
            if raw <= args.tol_raw and cen <= args.tol_centred:
                break

    n, T, qx = profiles(s)
    xc = centre(x, n, up[0], down[0])
    with open(os.path.abspath(__file__), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    out = dict(
        description="FP64 oracle steady state of the Mach-3 normal shock (LLF, ES-BGK, "
                    "1000 cells on [-20, 20], 12^3 Gauss-Hermite nodes, CFL 0.5)",
        script="tests/golden/make_shock_mach3_steady.py", script_sha256=sha,
        mach=MACH, cells=CELLS, x_lo=X_LO, x_hi=X_HI, thickness=THICK,
        upstream=list(up), downstream=list(down),
        steps=step, t=s.t, reached=bool(raw <= args.tol_raw and cen <= args.tol_centred),
        last_change_raw=raw, last_change_centred=cen,
        tol_raw=args.tol_raw, tol_centred=args.tol_centred, centre=xc,
        x=x.tolist(), n=n.tolist(), T=T.tolist(), qx=qx.tolist())
    with open(args.out, "w") as f:
        json.dump(out, f)
    print(f"wrote {args.out}: steps {step}, t {s.t:.4f}, centre {xc:.5f}, reached {out['reached']}")


if __name__ == "__main__":
    main()
