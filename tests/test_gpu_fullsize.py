"""Parity at full size, in the launch configuration the benchmark times.

One step moves information by at most one node, so after k steps a node
depends only on the initial state within distance k.  The oracle therefore
reproduces sampled nodes of a 512^3 run exactly from a (2k+1)^3 sub-box of the
same counter-generated initial state: where the sub-box reaches a real wall or
the lid it has that wall; where it is cut, the cut's (wrong) boundary value
cannot reach the sample within k steps.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

K_STEPS = 6
TOL_U = {"f64": 1e-12, "f32": 1e-5, "f16": 2e-3}


@pytest.fixture(scope="module")
def clbm():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1908_05396_amd import clbm as c
    c.load()
    return c


def _samples(spec):
    nx, ny, nz = spec.nx, spec.ny, spec.nz
    rng = np.random.default_rng(2024)
    pts = [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (0, ny - 1, 0), (nx - 1, ny - 1, nz // 2),
           (nx // 2, ny - 1, nz // 2), (nx // 2, ny - 2, 0), (nx // 2, ny // 2, nz // 2),
           (1, ny // 3, nz - 1), (nx - 1, 0, nz // 4)]
    pts += [tuple(int(v) for v in (rng.integers(0, nx), rng.integers(0, ny), rng.integers(0, nz)))
            for _ in range(5)]
    return pts


def _oracle_at(spec, seed, eps, pt, k):
    """Oracle velocity and post-collision populations at node pt after k steps."""
    lo = [max(0, c - k) for c in pt]
    hi = [min(n, c + k + 1) for c, n in zip(pt, (spec.nx, spec.ny, spec.nz))]
    lid = spec.lid_face if hi[1] == spec.ny else W.LID_NONE     # the lid is the +y face
    sub = spec.with_(nx=hi[0] - lo[0], ny=hi[1] - lo[1], nz=hi[2] - lo[2], lid_face=lid)
    box = ((lo[0], hi[0]), (lo[1], hi[1]), (lo[2], hi[2]))
    f0 = W.perturbed_populations(spec, seed, eps, box=box).numpy()
    f = oracle.run(sub, f0, k)
    _, u = oracle.macroscopic(sub, f)
    ft = oracle.collide(sub, f)
    ix, iy, iz = (pt[0] - lo[0], pt[1] - lo[1], pt[2] - lo[2])
    return u[:, iz, iy, ix], ft[:, iz, iy, ix]


@pytest.mark.parametrize("config,storage,layout", [
    ("cavity512", "f32", "rows"), ("cavity512", "f16", "rows"), ("cavity512", "f64", "rows"),
    ("cavity512", "f32", "planes"), ("cavity512", "f16", "planes"), ("cavity256", "f32", "rows"),
    ("cavity256", "f16", "rows"), ("cavity512", "f32", "two-step"), ("cavity512", "f64", "two-step"),
    ("cavity512", "f32", "two-step-rows")])
def test_light_cone_samples(clbm, config, storage, layout):
    """layout "two-step": the planes layout with the two-steps-per-launch
    configuration that bench.py times for this storage type; "two-step-rows":
    the same configuration in the row layout (the autotuner's pick for the
    row-layout lattice).  K_STEPS is even: two-step launches only."""
    from bench import TWO_STEP
    spec = W.config_cavity512() if config == "cavity512" else W.config_cavity256()
    seed, eps = 77, 2e-3
    print(f"[gpu] full-size {spec.name} {storage} {layout} k={K_STEPS}", flush=True)
    if layout.startswith("two-step"):
        lat = clbm.Lattice(spec, storage=storage, track_residual=False,
                           layout="rows" if layout.endswith("rows") else "planes", launch=TWO_STEP[storage])
        assert lat.get_launch()["fuse_steps"] == 2 and K_STEPS % 2 == 0
    else:
        lat = clbm.Lattice(spec, storage=storage, track_residual=False, layout=layout)
    f0 = W.perturbed_populations(spec, seed, eps, device="cuda")
    lat.init_populations(f0)
    del f0
    torch.cuda.empty_cache()
    lat.step(K_STEPS)
    _, u = lat.macroscopic()
    pts = _samples(spec)
    idx = torch.tensor([[p[2], p[1], p[0]] for p in pts], device="cuda")
    u_gpu = u[:, idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy().T
    del u
    st = lat.state_view()
    d_gpu = st[:, idx[:, 0], idx[:, 1], idx[:, 2]].to(torch.float64).cpu().numpy().T
    lat.close()
    del lat, st
    torch.cuda.empty_cache()
    w = W.INPUT_WEIGHTS
    refs = [_oracle_at(spec, seed, eps, p, K_STEPS) for p in pts]
    u_ref = np.array([r[0] for r in refs])
    f_ref = np.array([r[1] for r in refs])
    err_u = np.abs(u_gpu - u_ref).max() / np.abs(u_ref).max()
    err_f = np.abs((d_gpu + w) - f_ref).max()
    print(f"full-size {spec.name} {storage}: u {err_u:.3e}, populations {err_f:.3e}")
    assert err_u < TOL_U[storage]
    assert err_f < {"f64": 5e-15, "f32": 1e-6, "f16": 2e-5}[storage]
