"""Full-length energy trace of the 2048^2 FP32 workload against the FP64 oracle.

Not collected by pytest (about 7 minutes of CPU on 16 threads): run it by
name on a machine with a HIP device,

    python tests/full_length_trace.py [--steps 20000] [--log-every 500]

It steps the 2048^2 periodic lattice (r = 0.1, A1 = -4.9, seed 1, tau = 1)
on the GPU in the library's default launch configuration, and the oracle in
chunks of log_every steps, and prints for every log point the relative
differences of the mass, of the pseudo-potential energy E = E_s + E_m and of
sum psi^2 (section V), and their maxima over the run.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import oracle as O  # noqa: E402
from paper_1008_2865_amd import inputs  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--log-every", type=int, default=500)
    ap.add_argument("--r", type=float, default=0.1)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    import torch

    from paper_1008_2865_amd.sim import LBSim

    n, T, le = args.n, args.steps, args.log_every
    G1, G2 = inputs.couplings(args.r)
    rho0 = inputs.rho_noise(n, n, args.seed)

    sim = LBSim(rho0, G1=G1, G2=G2, storage="f32", log_every=le, max_steps=T)
    t0 = time.perf_counter()
    sim.step(T)
    tg = sim.trace()
    torch.cuda.synchronize()
    print(f"gpu: {T} steps, {len(tg)} trace rows, {time.perf_counter() - t0:.2f} s", flush=True)
    sim.close()

    f = O.init(rho0)
    rows = []
    t0 = time.perf_counter()
    for c in range(T // le):
        f, tr = O.run(f, le, 1.0, 1.0, G1, G2, le)
        row = tr[0].copy()
        row[0] = c * le  # the chunk's trace counts time from its start
        rows.append(row)
        print(f"oracle: t = {(c + 1) * le} ({time.perf_counter() - t0:.0f} s)", flush=True)
    ob = O.observables(f, 1.0, G1, G2)
    rows.append(np.concatenate([[T], ob]))
    to = np.array(rows)

    assert tg.shape == to.shape and np.array_equal(tg[:, 0], to[:, 0]), (tg.shape, to.shape)
    Eg, Eo = tg[:, 2] + tg[:, 3], to[:, 2] + to[:, 3]
    dM = (tg[:, 1] - to[:, 1]) / to[:, 1]
    dE = (Eg - Eo) / np.abs(Eo)
    dP = (tg[:, 4] - to[:, 4]) / to[:, 4]
    print("     t        dM/M        dE/E   dsum(psi^2)", flush=True)
    for k in range(len(to)):
        print(f"{int(to[k, 0]):6d} {dM[k]: .3e} {dE[k]: .3e} {dP[k]: .3e}", flush=True)
    res = {"n": n, "steps": T, "log_every": le, "max_abs_dM_over_M": float(np.max(np.abs(dM))),
           "max_abs_dE_over_E": float(np.max(np.abs(dE))),
           "max_abs_dpsi2": float(np.max(np.abs(dP))), "E_oracle_first_last": [Eo[0], Eo[-1]]}
    print(json.dumps(res), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(res, fh)


if __name__ == "__main__":
    main()
