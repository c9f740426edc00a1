"""Lattices with per-node solid flags (the nullable flag array of
clbm_create), and the host/device and output-precision options of the
boundary, on the GPU against the FP64 oracle.

Half-way bounce-back at a flagged node is the rule of the box walls
(Sec. 4.1), with the moving-wall term for a moving-wall node (Sec. 4.3).
Tolerances (normwise on u): FP64 1e-12, FP32 1e-5, as for the box."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL_U = {"f64": 1e-12, "f32": 1e-5}


@pytest.fixture(scope="module")
def clbm():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1908_05396_amd import clbm as c
    c.load()
    return c


def _normwise(u, ref):
    return np.abs(u - ref).max() / np.abs(ref).max()


def _walled_cavity_flags(nx, ny, nz):
    """An (nx+2) x (ny+2) x (nz+2) lattice whose outer layers are walls and
    whose +y layer (edges and corners included) moves: the nx x ny x nz lid
    cavity with its walls as flagged nodes."""
    fl = np.zeros((nz + 2, ny + 2, nx + 2), dtype=np.uint8)
    fl[0], fl[-1] = 1, 1
    fl[:, 0], fl[:, -1] = 1, 1
    fl[:, :, 0], fl[:, :, -1] = 1, 1
    fl[:, -1, :] = 2
    return fl


def _obstacle_channel():
    spec = W.LatticeSpec(nx=70, ny=14, nz=5, K=0.05, n=0.8, periodic=(1, 0, 1), force=(2e-5, 0.0, 0.0),
                         lid_velocity=(0.01, 0.0, 0.0), name="obstacle_channel")
    fl = np.zeros((5, 14, 70), dtype=np.uint8)
    fl[:, 5:9, 20:24] = oracle.WALL
    fl[2, 0:2, 50:53] = oracle.MOVING_WALL   # a solid moving with the lid velocity, touching the wall
    return spec, fl


def _run(clbm, spec, storage, layout, f0, steps, flags):
    print(f"[gpu] flagged {spec.name} {spec.nx}x{spec.ny}x{spec.nz} {storage} {layout} steps={steps}", flush=True)
    lat = clbm.Lattice(spec, storage=storage, layout=layout, flags=torch.from_numpy(flags))
    lat.init_populations(torch.from_numpy(f0).to("cuda"))
    lat.step(steps)
    rho, u = lat.macroscopic()
    r = lat.reduce()
    torch.cuda.synchronize()
    return rho.cpu().numpy(), u.cpu().numpy(), r, lat


@pytest.mark.parametrize("layout", ["rows", "planes"])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_flagged_cavity_matches_oracle_and_box(clbm, storage, layout):
    """A 9 x 8 x 7 lattice with flagged walls and moving lid layer: against
    the oracle on the same flags, and (its interior) against the 7 x 6 x 5
    box cavity run by the tuned kernels."""
    box = W.cavity(6, 0.05, 0.7, 50.0).with_(nx=7, ny=6, nz=5, name="cavity7x6x5")
    big = box.with_(nx=9, ny=8, nz=7, lid_face=W.LID_NONE, name="flagged9x8x7")
    fl = _walled_cavity_flags(7, 6, 5)
    f0 = W.perturbed_populations(box, 5, 1e-3).numpy()
    g0 = np.broadcast_to(oracle.weights()[:, None, None, None], (19, 7, 8, 9)).copy()
    g0[:, 1:-1, 1:-1, 1:-1] = f0
    ref = oracle.run(big, g0, 60, flags=fl)
    rho_ref, u_ref = oracle.macroscopic(big, ref, flags=fl)
    rho, u, r, _ = _run(clbm, big, storage, layout, g0, 60, fl)
    err = _normwise(u, u_ref)
    print(f"flagged cavity {storage} {layout}: {err:.3e}")
    assert err < TOL_U[storage]
    assert np.all(u[:, fl != 0] == 0.0) and np.all(rho[fl != 0] == 1.0)
    # reductions over the fluid nodes only: mass of the 210 fluid nodes (FP32:
    # the rounding of the stored deviations, ~1e-10 per node after 60 steps)
    fluid = fl == 0
    assert abs(r["mass"] - rho_ref[fluid].sum()) < {"f64": 1e-11, "f32": 1e-9}[storage] * fluid.sum()
    # the box run through the tuned (unflagged) kernels
    lat = clbm.Lattice(box, storage=storage, layout=layout)
    lat.init_populations(torch.from_numpy(f0).to("cuda"))
    lat.step(60)
    _, ub = lat.macroscopic()
    assert _normwise(u[:, 1:-1, 1:-1, 1:-1], ub.cpu().numpy()) < TOL_U[storage]


@pytest.mark.parametrize("layout", ["rows", "planes"])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_flagged_obstacle_channel(clbm, storage, layout):
    """Force-driven channel around a solid block (periodic x and z, walls on
    y), 70 nodes along x (a 64-wide tile and a ragged tail): velocity field
    and fluid mass against the oracle."""
    spec, fl = _obstacle_channel()
    f0 = W.perturbed_populations(spec, 11, 1e-3).numpy()
    ref = oracle.run(spec, f0, 200, flags=fl)
    rho_ref, u_ref = oracle.macroscopic(spec, ref, flags=fl)
    rho, u, r, _ = _run(clbm, spec, storage, layout, f0, 200, fl)
    err = _normwise(u, u_ref)
    print(f"obstacle channel {storage} {layout}: {err:.3e}")
    assert err < TOL_U[storage]
    fluid = fl == 0
    assert abs(r["mass"] - rho_ref[fluid].sum()) < {"f64": 1e-11, "f32": 1e-9}[storage] * fluid.sum()
    mom = (rho_ref[None] * u_ref)[:, fluid].sum(axis=1)
    assert abs(r["momentum_x"] - mom[0]) < (1e-12 if storage == "f64" else 1e-5) * abs(mom[0])


def test_flag_restrictions(clbm):
    """Invalid flag values are refused at creation; flagged lattices run one
    step per launch and are not autotuned."""
    spec, fl = _obstacle_channel()
    bad = fl.copy()
    bad[0, 7, 7] = 3
    with pytest.raises(clbm.ClbmError) as ei:
        clbm.Lattice(spec, storage="f32", flags=torch.from_numpy(bad))
    assert ei.value.status == clbm.CLBM_EINVAL and "flags" in str(ei.value)
    lat = clbm.Lattice(spec, storage="f32", flags=torch.from_numpy(fl))
    lat.init_rest()
    with pytest.raises(clbm.ClbmError):
        lat.set_launch(fuse_steps=2)
    with pytest.raises(clbm.ClbmError):
        lat.autotune()
    with pytest.raises(ValueError):
        clbm.Lattice(spec, storage="f32", in_place=True, flags=torch.from_numpy(fl))


@pytest.mark.parametrize("in_place", [False, True])
def test_host_initial_state_and_float_outputs(clbm, in_place):
    """clbm_init_populations from host memory gives the same state as from
    device memory; clbm_macroscopic in FP32 is the FP64 output rounded."""
    spec = W.cavity(12, 0.05, 0.9, 80.0).with_(nz=9, name="cavity12x12x9")
    f0 = W.perturbed_populations(spec, 21, 1e-3)
    a = clbm.Lattice(spec, storage="f64", in_place=in_place)
    a.init_populations(f0.to("cuda"))
    b = clbm.Lattice(spec, storage="f64", in_place=in_place)
    b.init_populations(f0.cpu())
    assert torch.equal(a.populations(), b.populations())
    a.step(20)
    b.step(20)
    rho64, u64 = b.macroscopic()
    rho32, u32 = b.macroscopic(out_prec="f32")
    assert u32.dtype == torch.float32 and rho32.dtype == torch.float32
    assert torch.equal(u32, u64.float()) and torch.equal(rho32, rho64.float())
    assert torch.equal(a.macroscopic()[1], u64)


def test_batch_host_initial_state_and_float_outputs(clbm):
    specs = [W.cavity(10, 0.05, 0.8, 50.0, name="b10"), W.cavity(14, 0.05, 1.2, 50.0, name="b14")]
    b = clbm.Batch(specs, storage="f32")
    b.init_rest()
    f0 = W.perturbed_populations(specs[1], 3, 1e-3)
    b.init_populations(1, f0.cpu())
    b.step(10)
    rho64, u64 = b.macroscopic(1)
    _, u32 = b.macroscopic(1, out_prec="f32")
    assert torch.equal(u32, u64.float())
    with pytest.raises(clbm.ClbmError):
        rho = torch.empty(specs[0].nodes, dtype=torch.float16, device="cuda")
        clbm._check(clbm.load().clbm_batch_macroscopic(b._h, 0, ctypes.c_void_p(rho.data_ptr()), None, 2,
                                                       clbm._stream(None)))
