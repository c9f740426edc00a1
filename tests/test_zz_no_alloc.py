"""clbm_reduce_noalloc (the reduction entry point that allocates nothing and
keeps its block partials in the library's static scratch) against
clbm_reduce, through the C-ABI, on two twin lattices stepped identically.

Two calls in a row on a lattice (the second with a residual against the
first), then a call on a smaller lattice, then a lattice holding a NaN: the
eight values must agree to the FP64 reduction bar (bit for bit: both run the
same block partition and summation order; the residual's square root to one
ulp)."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("mass", "momentum_x", "momentum_y", "momentum_z", "residual", "nonfinite", "umax", "kinetic")


@pytest.fixture(scope="module")
def clbm():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1908_05396_amd import clbm as c
    c.load()
    return c


def _twins(clbm, spec, storage, f0=None):
    lats = []
    for _ in range(2):
        lat = clbm.Lattice(spec, storage=storage, track_residual=True)
        if f0 is None:
            lat.init_rest()
        else:
            lat.init_populations(f0.to("cuda"))
        lats.append(lat)
    return lats


def _compare(clbm, a, b, label):
    ref = a.reduce(raise_unstable=False)
    out = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
    b.reduce_noalloc(out)
    torch.cuda.synchronize()
    got = dict(zip(KEYS, out.cpu().tolist()))
    print(f"[no-alloc] {label}: " + ", ".join(f"{k}={got[k]:.6e}" for k in KEYS), flush=True)
    for k in KEYS:
        if k == "residual":
            assert got[k] == pytest.approx(ref[k], rel=2.3e-16, abs=0.0), (label, k)
        else:
            same = got[k] == ref[k] or (np.isnan(got[k]) and np.isnan(ref[k]))
            assert same, (label, k, got[k], ref[k])
    return got


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_noalloc_reduce_matches_reduce(clbm, storage):
    big = W.cavity(48, 0.05, 0.7, 200.0).with_(nx=70, ny=48, nz=40, name="cavity70x48x40")
    small = W.cavity(12, 0.05, 1.2, 50.0).with_(nz=9, name="cavity12x12x9")
    a, b = _twins(clbm, big, storage, W.perturbed_populations(big, 3, 1e-3))
    for lat in (a, b):
        lat.step(30)
    first = _compare(clbm, a, b, f"{storage} {big.name} first call")
    assert first["residual"] == 0.0 and first["nonfinite"] == 0
    for lat in (a, b):
        lat.step(20)
    second = _compare(clbm, a, b, f"{storage} {big.name} second call")
    assert second["residual"] > 0.0
    c, d = _twins(clbm, small, storage)
    for lat in (c, d):
        lat.step(15)
    third = _compare(clbm, c, d, f"{storage} {small.name} (smaller)")
    assert third["mass"] == pytest.approx(small.nodes, rel=1e-12 if storage == "f64" else 1e-9)


def test_noalloc_reduce_reports_nonfinite(clbm):
    spec = W.cavity(8, 0.05, 1.0, 10.0, name="cavity8_nan")
    f0 = W.rest_populations(spec).clone()
    f0[3, 2, 2, 2] = float("nan")
    a, b = _twins(clbm, spec, "f32", f0)
    got = _compare(clbm, a, b, "nan")
    assert got["nonfinite"] >= 1
