"""The row layout against the planes layout and against the FP64 oracle.

Both layouts hold the same values and run the same collision; the row
kernels address a wave's 19 sources through scalar row bases, take the full
wall rule on rows of a y or z face and the x-face rule on the lanes of the
x faces.  The cases put whole 64-lane waves on lattices with every wall kind
(half-way bounce-back on each axis, the lid on +y, -x, +x and +z, periodic
axes), forced and unforced kernels, the printed-moment form with general
rates, the BGK comparison model, the three storage types, and block widths
that are and are not multiples of 64.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL_U = {"f64": 1e-12, "f32": 1e-5, "f16": 2e-3}
# rows vs planes after a few steps, relative to the largest stored deviation:
# the same arithmetic on the same inputs (the bound only allows for the
# compiler contracting a product differently in the two kernels)
TOL_SAME = {"f64": 1e-13, "f32": 2e-6, "f16": 2e-3}


@pytest.fixture(scope="module")
def clbm():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1908_05396_amd import clbm as c
    c.load()
    return c


def _geometries():
    base = W.cavity(64, 0.05, 0.8, 200.0)
    omegas = dict(omega_bulk=1.15, omega_high=(1.2, 1.1, 1.3, 0.95, 0.9, 1.05, 1.1, 1.2, 0.85))
    return {
        "lid_py_130x12x9": base.with_(nx=130, ny=12, nz=9, name="rows_py"),
        "lid_mx_64x10x7": base.with_(nx=64, ny=10, nz=7, lid_face=W.LID_MX, lid_velocity=(0.0, 0.05, 0.01)),
        "lid_px_96x9x8": base.with_(nx=96, ny=9, nz=8, lid_face=W.LID_PX, lid_velocity=(0.0, -0.03, 0.02)),
        "lid_pz_70x8x11": base.with_(nx=70, ny=8, nz=11, lid_face=W.LID_PZ, lid_velocity=(0.05, -0.02, 0.0)),
        "periodic_xz_lid_128x10x6": base.with_(nx=128, ny=10, nz=6, periodic=(1, 0, 1)),
        "periodic_box_64x5x6": W.LatticeSpec(nx=64, ny=5, nz=6, K=0.02, n=0.9, periodic=(1, 1, 1), name="box"),
        "periodic_y_lid_pz_64x9x7": base.with_(nx=64, ny=9, nz=7, periodic=(0, 1, 0), lid_face=W.LID_PZ,
                                               lid_velocity=(0.04, 0.01, 0.0)),
        "channel_forced_64x16x4": W.poiseuille(64, 16, 4, n=0.6, Re=5.0, umax=0.02),
        # one row per y (ny = 1) or per z (nz = 1): every row is a face row
        "slab_ny1_64x1x5": W.LatticeSpec(nx=64, ny=1, nz=5, K=0.02, n=0.8, periodic=(1, 1, 0), name="slab_ny1"),
        "slab_nz1_96x6x1": base.with_(nx=96, ny=6, nz=1, periodic=(0, 0, 1)),
        "slab_ny2_nz2_64x2x2": W.LatticeSpec(nx=64, ny=2, nz=2, K=0.03, n=1.2, lid_face=W.LID_PY,
                                             lid_velocity=(0.05, 0.0, 0.01), name="slab_2x2"),
        "ghat_general_80x9x7": base.with_(nx=80, ny=9, nz=7, **omegas),
        "srt_72x9x8": base.with_(nx=72, ny=9, nz=8, model="srt"),
    }


def _run(clbm, spec, storage, layout, steps, seed, eps, block=None):
    lat = clbm.Lattice(spec, storage=storage, track_residual=False, layout=layout, block=block)
    lat.init_populations(W.perturbed_populations(spec, seed, eps, device="cuda"))
    lat.step(steps)
    st = lat.state_view().to(torch.float64).cpu().numpy()
    _, u = lat.macroscopic()
    u = u.cpu().numpy()
    f = lat.populations().cpu().numpy()
    lat.close()
    return st, u, f


@pytest.mark.parametrize("geom", list(_geometries()))
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_rows_match_planes_and_oracle(clbm, geom, storage):
    spec = _geometries()[geom]
    steps, seed, eps = 6, 31, 1e-2
    print(f"[gpu] layouts {geom} {storage} steps={steps}", flush=True)
    st_r, u_r, f_r = _run(clbm, spec, storage, "rows", steps, seed, eps)
    st_p, u_p, f_p = _run(clbm, spec, storage, "planes", steps, seed, eps)
    same = np.abs(st_r - st_p).max()
    print(f"    rows vs planes: max |d| diff {same:.3e} (bitwise equal: {np.array_equal(st_r, st_p)})")
    assert same <= TOL_SAME[storage] * np.abs(st_p).max()
    assert np.abs(f_r - f_p).max() <= TOL_SAME[storage] * np.abs(st_p).max()
    f_ref = oracle.run(spec, W.perturbed_populations(spec, seed, eps).numpy(), steps)
    _, u_ref = oracle.macroscopic(spec, f_ref)
    err = np.abs(u_r - u_ref).max() / np.abs(u_ref).max()
    print(f"    rows u vs oracle {err:.3e}")
    assert err < TOL_U[storage]


@pytest.mark.parametrize("block", [(64, 1), (128, 1), (64, 4), (192, 2), (32, 4), (100, 1)])
def test_row_block_shapes(clbm, block):
    """Fast (width a multiple of 64) and full-rule kernels give the same bits."""
    spec = _geometries()["lid_py_130x12x9"]
    print(f"[gpu] rows block {block}", flush=True)
    st, u, _ = _run(clbm, spec, "f32", "rows", 5, 8, 1e-2, block=block)
    ref, u_ref, _ = _run(clbm, spec, "f32", "rows", 5, 8, 1e-2, block=(256, 1))
    assert np.array_equal(st, ref) and np.array_equal(u, u_ref)


def test_rows_rest_state_and_reductions(clbm):
    """Rest initial state in the row layout: mass N, zero momentum, and a lid
    that starts the flow; reductions read the row layout."""
    spec = W.cavity(64, 0.05, 0.7, 100.0).with_(ny=20, nz=12)
    lat = clbm.Lattice(spec, storage="f64", layout="rows")
    lat.init_rest()
    r0 = lat.reduce()
    assert abs(r0["mass"] - spec.nodes) < 1e-12 * spec.nodes and r0["umax"] < 1e-15
    lat.step(50)
    r1 = lat.reduce()
    two = clbm.Lattice(spec, storage="f64", layout="planes")
    two.init_rest()
    two.step(50)
    r2 = two.reduce()
    lat.close()
    two.close()
    assert abs(r1["mass"] - spec.nodes) < 1e-11 * spec.nodes
    for k in ("mass", "momentum_x", "momentum_y", "momentum_z", "umax", "kinetic"):
        assert abs(r1[k] - r2[k]) <= 1e-12 * max(1.0, abs(r2[k])), k


@pytest.mark.parametrize("layout,storage", [("rows", "f32"), ("planes", "f32"), ("rows", "f64")])
def test_autotune_keeps_state_and_results(clbm, layout, storage):
    """clbm_autotune times launches into the spare buffer: the state is
    unchanged, and stepping with the chosen launch gives the same bits as the
    default launch (one step per launch), or the same values to rounding (two
    steps per launch: the two inlined collisions may contract multiply-adds
    differently)."""
    spec = _geometries()["lid_py_130x12x9"]
    print(f"[gpu] autotune {layout} {storage}", flush=True)
    tol = {"f32": 1e-6, "f64": 1e-14}[storage]      # two vs one step per launch: rounding only
    outs = []
    for tune in (False, True):
        lat = clbm.Lattice(spec, storage=storage, track_residual=False, layout=layout)
        lat.init_populations(W.perturbed_populations(spec, 12, 1e-2, device="cuda"))
        lat.step(3)
        if tune:
            before = lat.populations().cpu().numpy()
            cfg, ms = lat.autotune()
            print(f"    chose {cfg} {ms:.4f} ms/step")
            assert ms > 0 and cfg["bx"] % 64 == 0 and lat.get_launch() == cfg
            assert np.array_equal(before, lat.populations().cpu().numpy())
            assert lat.state() == (1, 3)
        lat.step(6)
        outs.append(lat.populations().cpu().numpy())
        lat.close()
    if cfg["fuse_steps"] == 1:
        assert np.array_equal(outs[0], outs[1])
    else:
        assert np.abs(outs[0] - outs[1]).max() <= tol
    # a two-step candidate alone, on the same lattice, as the autotuner would run it
    rows = 16 if storage != "f64" else 8
    lat = clbm.Lattice(spec, storage=storage, track_residual=False, layout=layout,
                       launch={"fuse_steps": 2, "fuse_rows": rows, "fuse_planes": 16, "xcd_remap": 1, "nt_stores": 0})
    lat.init_populations(W.perturbed_populations(spec, 12, 1e-2, device="cuda"))
    lat.step(9)
    assert np.abs(lat.populations().cpu().numpy() - outs[0]).max() <= tol
    lat.close()
    ip = clbm.Lattice(spec, storage=storage, in_place=True, layout=layout)
    ip.init_rest()
    with pytest.raises(clbm.ClbmError):
        ip.autotune()
    ip.close()
