"""In-place stepping with one state buffer (AA pattern) against the FP64
oracle and against the two-buffer form.

The in-place buffer holds pre-collision populations, which are exactly what
the oracle's run() returns, so the populations are compared element by
element; velocities are compared with the two-buffer form (whose buffer holds
the post-collision state of the same time).  The cases cover every wall kind
(half-way bounce-back on each axis, the lid on +y, -x and +z, periodic axes),
the forced kernel, the printed-moment collision form, the BGK comparison
model, the three storage types, both state layouts (narrow lattices take the
full-rule kernels, lattices of whole 64-lane waves the row kernels with scalar
row bases), and the 512^3 benchmark lattice by light cone.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL_U = {"f64": 1e-12, "f32": 1e-5, "f16": 2e-3}
# element-wise bounds on populations after a few steps: FP64 rounding of
# populations of size ~1/3 (ulp 5.6e-17) over 8 steps, up to ~70 ulp; FP32
# ~16 ulp of the largest population; FP16 the rounding of deviations of size
# ~1e-2
TOL_F = {"f64": 4e-15, "f32": 1e-6, "f16": 3e-5}


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
        "poiseuille_forced": W.config_poiseuille(),
        "periodic_xz_lid": cav.with_(periodic=(1, 0, 1)),
        "lid_mx": cav.with_(nx=12, ny=18, nz=10, lid_face=W.LID_MX, lid_velocity=(0.0, 0.05, 0.01)),
        "lid_pz": cav.with_(nx=9, ny=7, nz=13, lid_face=W.LID_PZ, lid_velocity=(0.05, -0.02, 0.0)),
        "channel_1xNx1": W.poiseuille(1, 12, 1, n=0.6, Re=5.0, umax=0.02),
        "periodic_box": W.LatticeSpec(nx=5, ny=7, nz=6, K=0.02, n=0.9, periodic=(1, 1, 1), name="box"),
        "srt_cavity": cav.with_(nx=11, ny=13, nz=10, model="srt"),
        # whole 64-lane waves: the row-layout kernels with scalar row bases
        "wide_lid_mx": cav.with_(nx=64, ny=10, nz=7, lid_face=W.LID_MX, lid_velocity=(0.0, 0.05, 0.01)),
        "wide_lid_px": cav.with_(nx=96, ny=9, nz=8, lid_face=W.LID_PX, lid_velocity=(0.0, -0.03, 0.02)),
        "wide_lid_pz": cav.with_(nx=70, ny=8, nz=11, lid_face=W.LID_PZ, lid_velocity=(0.05, -0.02, 0.0)),
        "wide_periodic_xz_lid": cav.with_(nx=128, ny=10, nz=6, periodic=(1, 0, 1)),
        "wide_periodic_y": cav.with_(nx=64, ny=9, nz=7, periodic=(0, 1, 0), lid_face=W.LID_PZ,
                                     lid_velocity=(0.04, 0.01, 0.0)),
        "wide_box": W.LatticeSpec(nx=64, ny=5, nz=6, K=0.02, n=0.9, periodic=(1, 1, 1), name="wide_box"),
        "wide_forced": W.poiseuille(64, 16, 4, n=0.6, Re=5.0, umax=0.02),
        "wide_srt": cav.with_(nx=72, ny=9, nz=8, model="srt"),
        "wide_slab_ny1": W.LatticeSpec(nx=64, ny=1, nz=5, K=0.02, n=0.8, periodic=(1, 1, 0), name="wide_slab_ny1"),
        "wide_slab_2x2": W.LatticeSpec(nx=64, ny=2, nz=2, K=0.03, n=1.2, lid_face=W.LID_PY,
                                       lid_velocity=(0.05, 0.0, 0.01), name="wide_slab_2x2"),
    }


@pytest.mark.parametrize("layout", ["rows", "planes"])
@pytest.mark.parametrize("geom", list(_geometries()))
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_in_place_matches_oracle_and_two_buffer_form(clbm, geom, storage, layout):
    spec = _geometries()[geom]
    steps, seed, eps = 8, 21, 1e-2
    print(f"[gpu] in-place {geom} {spec.nx}x{spec.ny}x{spec.nz} {storage} {layout} steps={steps}", flush=True)
    f0 = W.perturbed_populations(spec, seed, eps)
    f_ref = oracle.run(spec, f0.numpy(), steps)
    _, u_ref = oracle.macroscopic(spec, f_ref)

    lat = clbm.Lattice(spec, storage=storage, track_residual=False, in_place=True, layout=layout)
    lat.init_populations(f0.to("cuda"))
    lat.step(steps)
    f_gpu = lat.populations().cpu().numpy()
    _, u_in = lat.macroscopic()
    u_in = u_in.cpu().numpy()
    lat.close()

    two = clbm.Lattice(spec, storage=storage, track_residual=False, layout=layout)
    two.init_populations(f0.to("cuda"))
    two.step(steps)
    _, u_two = two.macroscopic()
    u_two = u_two.cpu().numpy()
    two.close()

    err_f = np.abs(f_gpu - f_ref).max()
    err_u = np.abs(u_in - u_ref).max() / np.abs(u_ref).max()
    err_2 = np.abs(u_in - u_two).max() / np.abs(u_two).max()
    print(f"    populations {err_f:.3e}, u vs oracle {err_u:.3e}, u vs two-buffer {err_2:.3e}")
    assert err_f < TOL_F[storage]
    assert err_u < TOL_U[storage]
    assert err_2 < TOL_U[storage]


def test_in_place_rules(clbm):
    lat = clbm.Lattice(W.cavity(8, 0.05, 1.0, 10.0), storage="f32", in_place=True)
    lat.init_rest()
    with pytest.raises(clbm.ClbmError):
        lat.step(3)
    with pytest.raises(clbm.ClbmError):
        lat.set_launch(fuse_steps=2, fuse_rows=16, fuse_planes=4)
    lat.step(4)
    assert lat.state() == (0, 4)
    r = lat.reduce()
    assert r["nonfinite"] == 0 and abs(r["mass"] - 512) < 1e-6 * 512     # FP32 rounding of the sums
    lat.close()


@pytest.mark.parametrize("storage,layout", [("f32", "rows"), ("f64", "rows"), ("f16", "rows"), ("f32", "planes")])
def test_in_place_full_size_light_cone(clbm, storage, layout):
    """512^3 cavity (the benchmark lattice) in place for 6 steps from a
    perturbed start; sampled nodes against the oracle on (2k+1)^3 sub-boxes."""
    spec = W.config_cavity512()
    k, seed, eps = 6, 77, 2e-3
    print(f"[gpu] in-place full size {storage} {layout}", flush=True)
    lat = clbm.Lattice(spec, storage=storage, track_residual=False, in_place=True, layout=layout)
    f0 = W.perturbed_populations(spec, seed, eps, device="cuda")
    lat.init_populations(f0)
    del f0
    torch.cuda.empty_cache()
    lat.step(k)
    nx, ny, nz = spec.nx, spec.ny, spec.nz
    pts = [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (nx // 2, ny - 1, nz // 2), (1, ny // 3, nz - 1),
           (nx - 1, 0, nz // 4), (nx // 2, ny // 2, nz // 2)]
    st = lat.state_view()
    idx = torch.tensor([(p[2], p[1], p[0]) for p in pts], device="cuda")
    d = st[:, idx[:, 0], idx[:, 1], idx[:, 2]].to(torch.float64).cpu().numpy().T
    lat.close()
    del lat, st
    torch.cuda.empty_cache()
    for p, dp in zip(pts, d):
        lo = [max(0, c - k) for c in p]
        hi = [min(n, c + k + 1) for c, n in zip(p, (nx, ny, nz))]
        lid = spec.lid_face if hi[1] == ny else W.LID_NONE
        sub = spec.with_(nx=hi[0] - lo[0], ny=hi[1] - lo[1], nz=hi[2] - lo[2], lid_face=lid)
        f0s = W.perturbed_populations(spec, seed, eps, box=((lo[0], hi[0]), (lo[1], hi[1]), (lo[2], hi[2])))
        ref = oracle.run(sub, f0s.numpy(), k)[:, p[2] - lo[2], p[1] - lo[1], p[0] - lo[0]]
        err = np.abs(dp + W.INPUT_WEIGHTS - ref).max()
        print(f"   {p}: {err:.3e}")
        assert err < TOL_F[storage]
