"""Confined-cylinder Nusselt study (Sec. 4.4, Tables 3 and 4) on the GPU library.

Steady forced convection from a cylinder in a channel, Re = 10, for a set of
Prandtl numbers, lattice refinements S (1000 S x 150 S nodes, D = 30 S), kernel
pairs and boundary-condition orders.  Each case runs until the Nusselt number
from the heater flux is steady, then reports it with the Nusselt number of the
Sec. 4.4 definition (heater and section fluxes averaged) and the balance of the
two fluxes.  The inputs are those of workloads.confined_cylinder (EQ inlet in
place of the paper's Zou-He inlet, periodic y in place of its symmetry planes).

    python -m paper_2203_01316_amd.confined_cylinder --S 1 2 --Pr 10 100 1000 \\
        --pairs cm cucm cucu --bc 2 1 --out study.json

Kernel pairs: cm = central-moment f with CM-TRT h; cucm = cumulant f with
CM-TRT h (the paper's "CM-TRT" configuration); cucu = cumulant f with
Cumulants-1st h (the paper's "Cumulants-1st").  BC order 2 = IBB/IABB on the
cylinder, 1 = BB/ABB.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import lbm as L
from . import workloads as W

PAIRS = {"cm": dict(cumulant_f=False, cumulant_h=False, relax_h="trt"),
         "cucm": dict(cumulant_f=True, cumulant_h=False, relax_h="trt"),
         "cucu": dict(cumulant_f=True, cumulant_h=True, relax_h="1st")}


def run_case(S, Pr, pair, bc, *, xc_frac=0.2, tol=1e-3, bal_tol=0.02, min_flow=1.0, max_flow=15.0,
             storage="fp32_dev", stream="aa", log=print, progress=False):
    """One case; returns a dict of its results.  The Nusselt numbers are read
    every eighth of the flow-through time nx / U, for at least min_flow and
    at most max_flow flow-through times.  Steady means that the heater
    Nusselt number moved less than tol (relative) over the last half
    flow-through and that the heater flux and the flow's gain between the
    sections agree within bal_tol."""
    flags, q, groups, u, rho0, H0, info = W.confined_cylinder(S, Pr, bc == 2, xc_frac=xc_frac)
    nx, ny = info["nx"], info["ny"]
    g = L.LBM(L.D2Q9, nx, ny, with_ns=True, storage=storage, nu=info["nu"], k=info["k"], flags=flags, q=q,
              groups=groups, rho_ref=1.0, H_ref=info["T_in"],
              stream=L.STREAM_AA if stream == "aa" else L.STREAM_AB, **PAIRS[pair])
    uf = np.asarray(u, np.float32)
    g.set_velocity(uf)
    g.init(H0, u=uf.astype(np.float64), rho=rho0)
    flow = nx / info["U"]
    chunk = max(1, int(round(flow / 8)))
    hist = []
    t0 = time.time()
    converged = False
    while g.t < max_flow * flow:
        g.step(chunk)
        nu, nu_s, q_s, q_in, q_out = g.nusselt(1, *info["sections"], info["T_cyl"], info["T_in"])
        hist.append((g.t, nu_s))
        if progress:
            log(f"  S={S} Pr={Pr:g} {pair} bc{bc}: t = {g.t} ({g.t / flow:.2f} flow-throughs), Nu {nu:.4f}, "
                f"heater Nu {nu_s:.4f}, balance {(q_out - q_in) / q_s:.4f}")
        window = [h for t, h in hist if t >= g.t - 0.5 * flow]
        if g.t >= min_flow * flow and len(window) >= 4:
            if (max(window) - min(window)) <= tol * abs(nu_s) and abs((q_out - q_in) / q_s - 1.0) <= bal_tol:
                converged = True
                break
    bal = (q_out - q_in) / q_s
    # the heater flux of the high-Prandtl cases keeps fluctuating by a few
    # per cent: report the mean and spread of the readings over the last half
    # flow-through next to the last reading
    window = [h for t, h in hist if t >= g.t - 0.5 * flow]
    mean = sum(window) / len(window)
    res = dict(S=S, Pr=Pr, pair=pair, bc=bc, xc_frac=xc_frac, steps=g.t,
               flow_throughs=round(g.t / flow, 2), Nu=round(nu, 4), Nu_heater=round(nu_s, 4),
               Nu_heater_mean=round(mean, 4), Nu_heater_spread=round((max(window) - min(window)) / mean, 4),
               balance=round(bal, 4), converged=converged, seconds=round(time.time() - t0, 1))
    log(json.dumps(res))
    del g
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--S", type=int, nargs="+", default=[1])
    ap.add_argument("--Pr", type=float, nargs="+", default=[10.0, 100.0, 1000.0])
    ap.add_argument("--pairs", nargs="+", default=["cm", "cucm", "cucu"], choices=sorted(PAIRS))
    ap.add_argument("--bc", type=int, nargs="+", default=[2, 1], choices=[1, 2])
    ap.add_argument("--xc-frac", type=float, nargs="+", default=[0.2])
    ap.add_argument("--max-flow", type=float, default=15.0)
    ap.add_argument("--min-flow", type=float, default=1.0)
    ap.add_argument("--tol", type=float, default=1e-3)
    ap.add_argument("--bal-tol", type=float, default=0.02)
    ap.add_argument("--out", default=None)
    ap.add_argument("--progress", action="store_true", help="print every reading of Nu")
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    results = []
    for S in args.S:
        for Pr in args.Pr:
            for pair in args.pairs:
                for bc in args.bc:
                    for xc in args.xc_frac:
                        results.append(run_case(S, Pr, pair, bc, xc_frac=xc, tol=args.tol, bal_tol=args.bal_tol,
                                                min_flow=args.min_flow,
                                                max_flow=args.max_flow, log=log, progress=args.progress))
                        if args.out:
                            with open(args.out, "w") as fh:
                                json.dump(results, fh, indent=1)
    return results


if __name__ == "__main__":
    main(sys.argv[1:])
