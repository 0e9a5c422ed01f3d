"""Writes tests/golden/alpha0.json: the step-size constant alpha0 of each
workload, from the oracle only.

Reading of the unstated step size (the paper tunes alpha0 per problem,
Sec. 5): alpha0 is chosen so that the first design step moves no density
by more than 0.2, alpha0 = 0.2 / max|g_P(x_1) / 2|, computed once with the
oracle's FP64 first-iteration gradient and then frozen into the workload
definition (synth.ALPHA0) so that the oracle and the GPU path use the same
double.  Plane problems ("plane_*") take their first step with Alg. 3's
Krylov step of the problem's degree.
Run:  python tests/golden/make_alpha0.py [cfg ...]
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth                                     # noqa: E402
from oracle.outer import OuterContext, default_alpha0   # noqa: E402
from oracle.plane import PlaneContext            # noqa: E402


def main(names):
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "alpha0.json")
    out = json.load(open(path)) if os.path.exists(path) else {}
    for name in names:
        if name.startswith("plane_"):
            # plane grids run Alg. 3: the first step uses the Krylov step of
            # the problem's degree, on the box [lo, 1]
            p = synth.plane_config(name)
            ctx = PlaneContext(p.nx, p.ny, p.fixed_mask)
            a0 = default_alpha0(ctx, p.x0, p.loads, 0, p.lo, 1.0, p.vmax,
                                low_level=("krylov", p.degree, p.beta))
        else:
            p = synth.config(name)
            ctx = OuterContext(p.nx, p.ny, p.nz, p.filter_radius, p.fixed_mask, p.springs)
            a0 = default_alpha0(ctx, p.x0, p.loads,
                                p.inner_steps, 0.0, 1.0, p.vmax)
        out[name] = float(a0)
        print(name, repr(a0), flush=True)
        json.dump(out, open(path, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["cfg1", "cfg2", "cfg3", "plane_small", "plane_a"])
