#!/usr/bin/env python3
"""Write the stored oracle results for the 64^3 lid-driven cavity.

The cavity: 64^3 fluid nodes, lid on the +y face moving at 0.05 along x,
Re = 100 with Re = rho H^n U^(2-n) / K, power-law index n in {0.5, 1.0, 1.5},
rest start (f = w), 20000 steps.  Each run calls only the FP64 CPU oracle
(about 40 minutes of 8 cores per index); nothing here touches the GPU
library.  The files keep the velocity on the two mid-planes z = 31, 32, on
every fourth node of the lattice, and the total mass, together with a hash of
the oracle source they were computed with.

Usage:  python tests/golden/make_cavity64_fixtures.py [n ...]
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

STEPS = 20000
CHUNK = 500
SUB = slice(1, 64, 4)          # every fourth node, 16 per axis
PLANES = (31, 32)


def oracle_source_hash() -> str:
    with open(os.path.join(ROOT, "oracle", "clbm_oracle.c"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def fixture_path(n: float) -> str:
    return os.path.join(HERE, f"cavity64_re100_n{n:g}_steps{STEPS}.npz")


def make(n: float) -> None:
    spec = W.config_cavity64(n)
    f = W.rest_populations(spec).numpy()
    t0 = time.time()
    done = 0
    while done < STEPS:
        f = oracle.run(spec, f, CHUNK)
        done += CHUNK
        print(f"n={n:g}: {done}/{STEPS} steps, {time.time() - t0:.0f} s", flush=True)
    rho, u = oracle.macroscopic(spec, f)
    np.savez_compressed(
        fixture_path(n),
        u_planes=u[:, list(PLANES)],            # (3, 2, 64, 64): components, z, y, x
        u_sub=u[:, SUB, SUB, SUB],              # (3, 16, 16, 16)
        mass=np.array(rho.sum()),
        steps=np.array(STEPS), n=np.array(n), K=np.array(spec.K), nu_min=np.array(spec.nu_min),
        nu_max=np.array(spec.nu_max), lid_velocity=np.array(spec.lid_velocity),
        oracle_source=np.array(oracle_source_hash()))
    print(f"wrote {fixture_path(n)}", flush=True)


if __name__ == "__main__":
    if os.environ.get("ORACLE_THREADS"):
        oracle.set_threads(int(os.environ["ORACLE_THREADS"]))
    for arg in (sys.argv[1:] or ["0.5", "1.0", "1.5"]):
        make(float(arg))
