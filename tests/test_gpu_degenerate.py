"""Degenerate lattices and empty step counts.

Single-node and single-row lattices put every node on several faces at once
(a 1 x 1 x 1 cavity bounces every direction back, with the lid term on the
+y side; a fully periodic single node streams every population onto itself),
so the face-row kernels, the x-face lanes and the two-step patch ring all
meet their corner cases.  The stored (post-collision) populations after a few
steps are compared element by element with the oracle's collision of its
state at the same step, in both layouts and both launch forms.  Zero steps
change nothing.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL_F = {"f64": 1e-13, "f32": 2e-6}


@pytest.fixture(scope="module")
def clbm():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1908_05396_amd import clbm as c
    c.load()
    return c


def _specs():
    return {
        "cube1_lid": W.cavity(1, 0.05, 0.8, 10.0, name="cube1"),
        "cube1_periodic_forced": W.LatticeSpec(nx=1, ny=1, nz=1, K=0.02, n=0.9, periodic=(1, 1, 1),
                                               force=(1e-4, -2e-5, 0.0), name="cube1p"),
        "line2_periodic_x_lid": W.cavity(4, 0.05, 1.0, 20.0, name="line2").with_(nx=2, ny=1, nz=1,
                                                                                   periodic=(1, 0, 0)),
        "column1x3x1": W.LatticeSpec(nx=1, ny=3, nz=1, K=0.02, n=1.2, name="col3"),
        "plate3x1x2_lid_pz": W.cavity(4, 0.04, 0.7, 30.0, name="plate").with_(nx=3, ny=1, nz=2, lid_face=W.LID_PZ,
                                                                                lid_velocity=(0.04, 0.0, 0.0)),
    }


FORMS = {"one": None, "two": {"fuse_steps": 2, "fuse_rows": 8, "fuse_planes": 1}}


@pytest.mark.parametrize("form", ["one", "two"])
@pytest.mark.parametrize("layout", ["rows", "planes"])
@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("geom", list(_specs()))
def test_degenerate_lattice_vs_oracle(clbm, geom, storage, layout, form):
    spec = _specs()[geom]
    steps, seed, eps = 6, 9, 1e-2
    print(f"[gpu] degenerate {geom} {storage} {layout} {form}", flush=True)
    f0 = W.perturbed_populations(spec, seed, eps)
    lat = clbm.Lattice(spec, storage=storage, track_residual=False, layout=layout, launch=FORMS[form])
    lat.init_populations(f0.to("cuda"))
    lat.step(steps)
    f = lat.populations().cpu().numpy()
    lat.close()
    ref = oracle.collide(spec, oracle.run(spec, f0.numpy(), steps))
    err = np.abs(f - ref).max()
    print(f"    max |f - oracle| {err:.3e}")
    assert err < TOL_F[storage]


@pytest.mark.parametrize("form", ["one", "two"])
def test_zero_steps_change_nothing(clbm, form):
    spec = W.cavity(16, 0.05, 0.8, 100.0).with_(nx=20, ny=9, nz=7)
    lat = clbm.Lattice(spec, storage="f32", track_residual=False, launch=FORMS[form],
                       layout="planes" if form == "two" else "rows")
    lat.init_populations(W.perturbed_populations(spec, 4, 1e-2, device="cuda"))
    lat.step(3)
    before, state = lat.populations().cpu().numpy(), lat.state()
    lat.step(0)
    assert lat.state() == state and np.array_equal(before, lat.populations().cpu().numpy())
    lat.close()
    b = clbm.Batch([spec, spec.with_(nx=33)], storage="f32")
    b.init_rest()
    b.step(2)
    before, state = [b.populations(i).cpu().numpy() for i in range(2)], b.state()
    b.step(0)
    assert b.state() == state
    for i in range(2):
        assert np.array_equal(before[i], b.populations(i).cpu().numpy())
    b.close()


@pytest.mark.parametrize("layout", ["rows", "planes"])
def test_degenerate_instances_in_a_batch(clbm, layout):
    """The same lattices as instances of one batch (one launch per step, graph
    replay), beside an ordinary one."""
    specs = list(_specs().values()) + [W.cavity(12, 0.05, 0.9, 50.0, name="b12")]
    steps, eps = 6, 1e-2
    b = clbm.Batch(specs, storage="f64", layout=layout)
    b.init_rest()
    for i, sp in enumerate(specs):
        b.init_populations(i, W.perturbed_populations(sp, 20 + i, eps, device="cuda"))
    b.set_config(graph_steps=4)
    b.step(steps)
    for i, sp in enumerate(specs):
        f = b.populations(i).cpu().numpy()
        ref = oracle.collide(sp, oracle.run(sp, W.perturbed_populations(sp, 20 + i, eps).numpy(), steps))
        err = np.abs(f - ref).max()
        print(f"[gpu] batch {layout} {sp.name}: {err:.3e}", flush=True)
        assert err < TOL_F["f64"], (sp.name, err)
    b.close()
