"""The 64^3 lid-driven cavity at Re 100 (n = 0.5, 1, 1.5; lid velocity 0.05;
rest start; 20000 steps) in FP64 and FP32 storage against the stored FP64
oracle results of tests/golden/make_cavity64_fixtures.py (the velocity on the
mid-planes z = 31, 32 and on every fourth node), normwise over those values.
"""
import hashlib
import os

import numpy as np
import pytest
import torch

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")
STEPS = 20000
TOL_U = {"f64": 1e-12, "f32": 1e-5}


def _fixture(n):
    path = os.path.join(GOLDEN, f"cavity64_re100_n{n:g}_steps{STEPS}.npz")
    if not os.path.exists(path):
        pytest.skip(f"{os.path.basename(path)} not generated (tests/golden/make_cavity64_fixtures.py)")
    return np.load(path)


def _oracle_hash():
    with open(os.path.join(ROOT, "oracle", "clbm_oracle.c"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


@pytest.mark.parametrize("n", [0.5, 1.0, 1.5])
def test_fixture_matches_current_oracle_and_spec(n):
    """A stored result is only valid for the oracle source and parameters it
    was computed with."""
    fx = _fixture(n)
    spec = W.config_cavity64(n)
    assert str(fx["oracle_source"]) == _oracle_hash(), "regenerate: the oracle changed"
    assert float(fx["K"]) == spec.K and float(fx["nu_min"]) == spec.nu_min and float(fx["nu_max"]) == spec.nu_max
    assert int(fx["steps"]) == STEPS
    assert abs(float(fx["mass"]) - spec.nodes) < 1e-9 * spec.nodes     # the closed cavity conserves mass


@pytest.mark.gpu
@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("n", [0.5, 1.0, 1.5])
def test_cavity64_against_stored_oracle(n, storage):
    fx = _fixture(n)
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1908_05396_amd import clbm
    spec = W.config_cavity64(n)
    print(f"[gpu] cavity64 n={n} {storage} {STEPS} steps", flush=True)
    lat = clbm.Lattice(spec, storage=storage, track_residual=False)
    lat.init_rest()
    lat.step(STEPS)
    _, u = lat.macroscopic()
    u = u.cpu().numpy()
    lat.close()
    got = np.concatenate([u[:, [31, 32]].ravel(), u[:, 1::4, 1::4, 1::4].ravel()])
    ref = np.concatenate([fx["u_planes"].ravel(), fx["u_sub"].ravel()])
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"    normwise error over {ref.size} stored values: {err:.3e}")
    assert err < TOL_U[storage]
