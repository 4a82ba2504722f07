"""Write adjoint64_tangent.json: directional derivatives of the mean hot-wall
Nusselt number on the differentiation workload, from the complex-step
tangent oracle (oracle/tangent.py).  Calls nothing but oracle/.

Workload: 64^3 cells, Ra 1e4, Pr 0.71, 400 pseudo-time steps from the seeded
initial state (seed 5, noise 1e-3); hot-wall temperatures
Theta_jk = 1 + 0.05 (2 r - 1), r the 53-bit uniform of SplitMix64(seed 5)
output j + nj k.  Directions: one seeded unit wall direction (numpy
default_rng(11) normals, normalised) and the Ra direction dRa = Ra.

The complex step follows the same side of every kink (|u| at 0, the maxima
and minima of the time step and beta^2) as the discrete adjoint does, so the
two agree to rounding; finite differences do not separate the two errors.

    python tests/golden/make_adjoint64_tangent.py      (about 4 minutes)
"""
import json
import os
import sys
import time
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from oracle import tangent as TG  # noqa: E402

N, RA, STEPS, SEED, AMP, NOISE, DIR_SEED = 64, 1e4, 400, 5, 0.05, 1e-3, 11
OUT = os.path.join(HERE, "adjoint64_tangent.json")


def theta():
    r = np.array([(O.splitmix64(SEED, m) >> 11) * 2.0 ** -53 for m in range(N * N)])
    return 1.0 + AMP * (2.0 * r - 1.0)


def wall_direction():
    v = np.random.default_rng(DIR_SEED).standard_normal(N * N)
    return v / np.linalg.norm(v)


def one(which):
    th = theta()
    q0 = O.init(O.Problem(N, Ra=RA), SEED, NOISE)
    t0 = time.time()
    if which == "theta":
        J, d = TG.nusselt_tangent(N, N, N, RA, th, q0, STEPS, dtheta=wall_direction())
    else:
        J, d = TG.nusselt_tangent(N, N, N, RA, th, q0, STEPS, dRa=RA)
    return which, J, d, time.time() - t0


def main():
    with Pool(2) as pool:
        res = pool.map(one, ["theta", "Ra"])
    out = {"workload": "64^3 FP64, Ra 1e4, Pr 0.71, 400 steps, state seed 5 (noise 1e-3), "
                       "Theta = 1 + 0.05 (2r - 1) from SplitMix64(5) output j + nj k",
           "n": N, "Ra": RA, "steps": STEPS, "state_seed": SEED, "noise": NOISE, "theta_amp": AMP,
           "wall_direction": "numpy default_rng(%d).standard_normal(nj*nk), unit norm" % DIR_SEED,
           "wall_direction_seed": DIR_SEED,
           "made_by": "tests/golden/make_adjoint64_tangent.py (complex-step tangent oracle, h = 1e-30)"}
    for which, J, d, sec in res:
        out["nusselt"] = J
        out["dJ_%s" % ("dir_theta" if which == "theta" else "dRa_times_Ra")] = d
        print("%s: J = %.17g, derivative %.17g (%.0f s)" % (which, J, d, sec), flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
