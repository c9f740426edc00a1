"""Two time steps per launch (temporal blocking) against one step per launch
and against the FP64 oracle.

The two-step kernel evaluates the operations of two one-step launches (the
first step's state is rounded to the storage type before it is used), so
after any number of steps both give the same populations up to the
compiler's choice of fused multiply-adds in the two inlined copies of the
collision: rounding-level differences (measured ~1e-16 relative in FP64).
The bounds below sit far under what a misplaced population would cause
(~1e-2 relative after a few steps from a 1e-2 perturbation) in FP64 and FP32;
in FP16 a one-ulp difference in FP32 can flip a rounding of the stored half,
so its bound is looser and the FP64/FP32 cases carry the check.  The cases
cover every wall kind (half-way bounce-back on each axis, the moving lid on
+y, -x and +z, periodic axes), lattices narrower than one patch and spanning
several patches along x, y and z, odd step counts (the remainder runs as one
one-step launch), every patch height (12 rows: in the planes layout the FP32
variant whose loads go straight to LDS), several z chunk lengths, the forced
kernel, the printed-moment collision form, and both state layouts (the row
layout reads and writes through the one-step row kernel's gather and store).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL_U = {"f64": 1e-12, "f32": 1e-5, "f16": 2e-3}


@pytest.fixture(scope="module")
def clbm():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1908_05396_amd import clbm as c
    c.load()
    return c


def _geometries():
    cav = W.cavity(16, 0.05, 0.7, 100.0)
    return {
        "ragged_lid_py": W.cavity(70, 0.05, 0.8, 200.0).with_(ny=20, nz=9, name="ragged"),
        "multi_patch": W.cavity(130, 0.04, 1.3, 300.0).with_(ny=40, nz=11, name="multi"),
        "poiseuille_forced": W.config_poiseuille(),
        "periodic_xz_lid": cav.with_(periodic=(1, 0, 1)),
        "lid_mx": cav.with_(nx=12, ny=18, nz=10, lid_face=W.LID_MX, lid_velocity=(0.0, 0.05, 0.01)),
        "lid_pz": cav.with_(nx=9, ny=7, nz=13, lid_face=W.LID_PZ, lid_velocity=(0.05, -0.02, 0.0)),
        "channel_1xNx1": W.poiseuille(1, 12, 1, n=0.6, Re=5.0, umax=0.02),
        "periodic_box": W.LatticeSpec(nx=5, ny=7, nz=6, K=0.02, n=0.9, periodic=(1, 1, 1), name="box"),
    }


def _run(clbm, spec, storage, steps, launch, seed=11, eps=1e-2, collision="auto", layout="planes"):
    lat = clbm.Lattice(spec, storage=storage, track_residual=False, launch=launch, collision=collision,
                       layout=layout)
    lat.init_populations(W.perturbed_populations(spec, seed, eps, device="cuda"))
    lat.step(steps)
    st = lat.state_view().reshape(19, -1).clone()
    _, u = lat.macroscopic()
    torch.cuda.synchronize()
    lat.close()
    return st, u


REL_BOUND = {"f64": 1e-13, "f32": 1e-5, "f16": 2e-2}


def _compare(a, b, storage):
    """max |a - b| and its bound, relative to max |b|."""
    da, db = a.to(torch.float64), b.to(torch.float64)
    return (da - db).abs().max().item(), REL_BOUND[storage] * db.abs().max().item()


@pytest.mark.parametrize("layout", ["rows", "planes"])
@pytest.mark.parametrize("geom", list(_geometries()))
@pytest.mark.parametrize("storage,rows", [("f64", 8), ("f32", 8), ("f32", 12), ("f32", 16), ("f16", 8), ("f16", 16)])
def test_two_step_equals_one_step(clbm, geom, storage, rows, layout):
    spec = _geometries()[geom]
    for steps, planes in ((7, 3), (4, 1), (6, max(1, spec.nz))):
        print(f"[gpu] fused {layout} {geom} {spec.nx}x{spec.ny}x{spec.nz} {storage} rows={rows} planes={planes} "
              f"steps={steps}", flush=True)
        ref, _ = _run(clbm, spec, storage, steps, {"fuse_steps": 1}, layout=layout)
        got, _ = _run(clbm, spec, storage, steps, {"fuse_steps": 2, "fuse_rows": rows, "fuse_planes": planes},
                      layout=layout)
        diff, bound = _compare(got, ref, storage)
        print(f"    max |diff| {diff:.3e} (bound {bound:.3e})")
        assert diff <= bound, f"{geom} {storage} rows={rows} planes={planes}: max diff {diff}"


@pytest.mark.parametrize("layout", ["rows", "planes"])
@pytest.mark.parametrize("storage,rows", [("f32", 16), ("f32", 12), ("f16", 8), ("f64", 8)])
def test_two_step_tile_order_and_store_hint(clbm, storage, rows, layout):
    """The XCD-contiguous patch order and the store hint change only where and
    how each output is written: every combination gives the same bits.  With
    16 rows the lattice has 36 patches (3 x 3 x 4) and with 8 rows 84, so the
    remapped range (a multiple of 8) and a remainder left in dispatch order
    both occur."""
    spec = _geometries()["multi_patch"]
    outs = []
    for mode in range(4):
        launch = {"fuse_steps": 2, "fuse_rows": rows, "fuse_planes": 3, "xcd_remap": mode & 1,
                  "nt_stores": mode >> 1}
        print(f"[gpu] fused order/hint {layout} {storage} rows={rows} {launch}", flush=True)
        st, _ = _run(clbm, spec, storage, 6, launch, layout=layout)
        outs.append(st.cpu())
    for o in outs[1:]:
        assert torch.equal(o, outs[0])


@pytest.mark.parametrize("layout", ["rows", "planes"])
@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_two_step_printed_moment_form(clbm, storage, layout):
    spec = W.cavity(20, 0.05, 0.8, 100.0).with_(omega_bulk=1.2, omega_high=(1.1, 0.9, 1.3, 1.0, 1.2, 0.8, 1.1, 1.4, 0.95))
    ref, _ = _run(clbm, spec, storage, 5, {"fuse_steps": 1}, collision="ghat", layout=layout)
    got, _ = _run(clbm, spec, storage, 5, {"fuse_steps": 2, "fuse_rows": 8, "fuse_planes": 4}, collision="ghat",
                  layout=layout)
    diff, bound = _compare(got, ref, storage)
    assert diff <= bound, f"max diff {diff}"


@pytest.mark.parametrize("layout", ["rows", "planes"])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("n", [0.5, 1.5])
def test_two_step_cavity_vs_oracle(clbm, storage, n, layout):
    spec = W.cavity(16, 0.05, n, 100.0)
    steps = 40
    f0 = W.perturbed_populations(spec, 5, 1e-3).numpy()
    _, u_ref = oracle.macroscopic(spec, oracle.run(spec, f0, steps))
    rows = {"f64": 8, "f32": 12, "f16": 16}[storage]
    _, u = _run(clbm, spec, storage, steps, {"fuse_steps": 2, "fuse_rows": rows, "fuse_planes": 5}, seed=5, eps=1e-3,
                layout=layout)
    err = np.abs(u.cpu().numpy() - u_ref).max() / np.abs(u_ref).max()
    print(f"two-step cavity16 n={n} {storage} {layout}: {err:.3e}")
    assert err < TOL_U[storage]


def test_two_step_poiseuille_vs_oracle(clbm):
    spec = W.config_poiseuille()
    f0 = W.rest_populations(spec).numpy()
    _, u_ref = oracle.macroscopic(spec, oracle.run(spec, f0, 2000))
    lat = clbm.Lattice(spec, storage="f64", launch={"fuse_steps": 2, "fuse_rows": 8, "fuse_planes": 8}, layout="rows")
    lat.init_rest()
    lat.step(2000)
    _, u = lat.macroscopic()
    err = np.abs(u.cpu().numpy() - u_ref).max() / np.abs(u_ref).max()
    lat.close()
    assert err < TOL_U["f64"]


def test_launch_validation(clbm):
    lat = clbm.Lattice(W.cavity(8, 0.05, 1.0, 10.0), storage="f64")
    for bad in ({"fuse_steps": 3}, {"fuse_steps": 2, "fuse_rows": 16}, {"fuse_planes": 0}, {"fuse_rows": 12},
                {"fuse_rows": 10}):
        with pytest.raises(clbm.ClbmError):
            lat.set_launch(**bad)
    lat.close()
