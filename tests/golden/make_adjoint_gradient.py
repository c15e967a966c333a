"""Write the oracle's reference gradient of the full-size adjoint workload.

Runs the CPU oracle's forward-mode derivative (``oracle.tlm_run``) of the two-stream
workload with 1,000,000 particles, 256 cells, 500 steps and 8 density modes, for the
loss J = dt * sum_n W_E^n, one parameter direction per process (8 amplitudes, beam
speed, beam spread), and stores J, the gradient and the fallback count in
``adjoint_two_stream_256c_1M.json`` beside this script.  Calls only ``oracle`` and the
seeded generators.  Takes a few minutes per direction.

    python tests/golden/make_adjoint_gradient.py [processes]
"""
import json
import os
import sys
import time
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "adjoint_two_stream_256c_1M.json")


def direction(i):
    import numpy as np
    import oracle
    import workloads
    wl = workloads.by_name("adjoint_two_stream_256c_1M")
    modes = wl.meta["modes"]
    n = wl.n_particles
    dx = np.zeros((1, n))
    dv = np.zeros((1, n))
    if i < len(modes):
        dx[0] = oracle.density_mode_tangents(wl.x, modes)[i]
    elif i == len(modes):
        dv[0] = wl.meta["sign"]
    else:
        dv[0] = wl.meta["g"]
    t0 = time.time()
    out = oracle.tlm_run(wl, wl.steps, dx, dv, wl.dt)
    return i, out["J"], float(out["dJ"][0]), int(out["records"]["fallbacks"].sum()), time.time() - t0


def main():
    procs = int(sys.argv[1]) if len(sys.argv) > 1 else 5
    with Pool(procs) as pool:
        res = sorted(pool.map(direction, range(10)))
    J = [r[1] for r in res]
    assert max(J) == min(J), "every direction runs the same forward"
    doc = {
        "workload": "adjoint_two_stream_256c_1M",
        "what": "oracle forward-mode gradient of J = dt * sum_{n=1..500} W_E^n",
        "parameters": [f"alpha_{m + 1}" for m in range(8)] + ["v_beam", "v_spread"],
        "J": J[0],
        "grad": [r[2] for r in res],
        "fallbacks": res[0][3],
        "seconds_per_direction": [round(r[4], 1) for r in res],
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    print(json.dumps(doc))


if __name__ == "__main__":
    main()
