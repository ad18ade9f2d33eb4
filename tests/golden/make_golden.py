"""Writes the oracle's temperatures after each workload's full step count at a
seeded sample of nodes, the reference of the full-horizon GPU parity tests
(tests/test_gpu_horizon.py) and of the benchmark's error line.

Calls only the FP64 oracle (``oracle``) and the seeded input generators
(``workloads``); nothing here comes from the GPU path.  Usage:

    python tests/golden/make_golden.py [workload ...]

Each file ``<workload>_<steps>.txt`` holds a header of ``# key value`` lines
(workload, steps, the sample's seed, max |T_ref| over all nodes, min and max
T_ref over all nodes, the oracle's threads and seconds) and then one
``node value`` line per sampled node (caller order, %.17g).  The sample is
4,096 nodes drawn without replacement (numpy PCG64, seed 1909_0100) plus the
nodes of the smallest and largest T_ref."""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import problems as P  # noqa: E402

SAMPLE_SEED = 1909_0100
N_SAMPLE = 4096

# workload name -> (builder, steps)
WORKLOADS = {
    "nonlinear_hex64": (lambda: P.cube_nonlinear_hex(64, 10000), 10000),
    "aniso_tet128": (lambda: P.cube_aniso_tet(128, 2000), 2000),
    "batched_hex256": (lambda: P.batched_hex(256, nsteps=5000), 5000),
}


def sample_nodes(N, Tref):
    g = np.random.default_rng(SAMPLE_SEED)
    idx = g.choice(N, size=min(N_SAMPLE, N), replace=False)
    idx = np.union1d(idx, [int(np.argmin(Tref)), int(np.argmax(Tref))])
    return idx.astype(np.int64)


def path_of(name, steps):
    return os.path.join(HERE, f"{name}_{steps}.txt")


def write(name):
    build, steps = WORKLOADS[name]
    p = build()
    t0 = time.time()
    Tref = oracle.Oracle(p).run(steps)
    secs = time.time() - t0
    idx = sample_nodes(Tref.size, Tref)
    with open(path_of(name, steps), "w") as f:
        f.write(f"# workload {name}\n# steps {steps}\n# sample_seed {SAMPLE_SEED}\n")
        f.write(f"# n_nodes {Tref.size}\n")
        f.write(f"# max_abs {np.max(np.abs(Tref)):.17g}\n")
        f.write(f"# min {Tref.min():.17g}\n# max {Tref.max():.17g}\n")
        f.write(f"# oracle_threads {os.environ.get('OMP_NUM_THREADS', os.cpu_count())}\n")
        f.write(f"# oracle_seconds {secs:.1f}\n")
        for k in idx:
            f.write(f"{k} {Tref[k]:.17g}\n")
    print(f"{name}: {steps} steps in {secs:.1f} s, T in [{Tref.min():.4f}, {Tref.max():.4f}]",
          flush=True)


def read(name, steps):
    """(header dict, node ids, values) of a golden file."""
    head, ids, vals = {}, [], []
    with open(path_of(name, steps)) as f:
        for line in f:
            if line.startswith("#"):
                k, v = line[1:].split(None, 1)
                head[k] = v.strip()
            else:
                a, b = line.split()
                ids.append(int(a))
                vals.append(float(b))
    return head, np.array(ids, dtype=np.int64), np.array(vals)


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(WORKLOADS)):
        write(name)
