"""Oracle trajectories for the full-size parity tests (tests/test_gpu_configs.py).

For each case the oracle steps the configuration's domain for its whole length
and stores, after every Crank-Nicolson step, the state at a seeded sample of
active nodes (compact indices, shared with the GPU path, whose ordering is
checked bit-exact against the oracle's) and the max norms of s and c over all
active nodes, with the oracle's Newton and V-cycle counts.  Only the oracle and
the seeded input generators are called.  Cases whose oracle run takes minutes
are stored here; the faster ones are stepped live by the tests.

    python tests/golden/make_oracle_trajectories.py [case ...]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import lsmg_inputs as I  # noqa: E402
import oracle  # noqa: E402

# the solver parameters the library resolves by default in 3-D
PARAMS3 = dict(ghost_sweeps=15, ghost_sweeps_coarse=30, sweeps_lambda=0.1)
SAMPLES = 512


def _request(rid):
    return [r for r in I.serving_requests(24, seed=0) if r["id"] == rid][0]


CASES = {
    # configuration 3: the torus at 257^3, all 20 steps
    "torus257": lambda: (I.torus(257), 257, 20, 1e-4),
    # configuration 5: served requests to completion (seeded stream, the served union of
    # ellipsoids): request 12 (129^3, 3 ellipsoids, 31 steps), request 17 (257^3, 4, 52)
    "serve_r12": lambda: (I.ellipsoids(129, _request(12)["centres"], _request(12)["semi"]), 129,
                          _request(12)["steps"], _request(12)["dt"]),
    "serve_r17": lambda: (I.ellipsoids(257, _request(17)["centres"], _request(17)["semi"]), 257,
                          _request(17)["steps"], _request(17)["dt"]),
}


def path_of(case):
    return os.path.join(HERE, f"trajectory_{case}.npz")


def make(case):
    phi, n, steps, dt = CASES[case]()
    O = oracle.Hierarchy(phi, 3, n, coarsest_n=9, params=PARAMS3)
    info = O.level_info(0)
    na = info["na"]
    s0, c0 = I.initial_state(n, 3)
    W = O.to_compact(0, s0, c0)
    sb = np.ones(info["ng"])
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(na, size=min(SAMPLES, na), replace=False))
    vals = np.zeros((steps, 2, idx.size))
    norms = np.zeros((steps, 2))
    counts = np.zeros((steps, 2), dtype=np.int64)
    t0 = time.time()
    for k in range(steps):
        rc, W, st = O.newton_cn_step(W, dt, sb)
        if rc != 0:
            raise RuntimeError(f"{case}: oracle step {k} failed with {rc}")
        vals[k, 0], vals[k, 1] = W[idx], W[na + idx]
        norms[k] = np.max(np.abs(W[:na])), np.max(np.abs(W[na:]))
        counts[k] = st["newton_iters"], st["vcycles"]
        print(f"{case}: step {k + 1}/{steps} newton {st['newton_iters']} cycles {st['vcycles']} "
              f"({time.time() - t0:.0f} s)", flush=True)
    np.savez_compressed(path_of(case), n=n, steps=steps, dt=dt, na=na, ng=info["ng"], idx=idx, vals=vals,
                        norms=norms, counts=counts,
                        params=np.array([PARAMS3["ghost_sweeps"], PARAMS3["ghost_sweeps_coarse"]]),
                        sweeps_lambda=PARAMS3["sweeps_lambda"])


if __name__ == "__main__":
    for c in (sys.argv[1:] or list(CASES)):
        make(c)
