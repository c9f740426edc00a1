"""Batched stepping (many lattices in one launch per step, graph
replay, autotuned tiles) against the oracle and against the one-launch-per-
instance reference path."""
import os

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def clbm():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1908_05396_amd import clbm as c
    c.load()
    return c


def _mixed_specs():
    return [
        W.cavity(12, 0.05, 0.6, 50.0, name="b_cav12"),
        W.cavity(16, 0.05, 1.4, 80.0, name="b_cav16").with_(nx=70, ny=9, name="b_cav70x9x16"),
        W.cavity(10, 0.04, 0.9, 60.0, name="b_cav128").with_(nx=128, ny=6, nz=5, lid_face=W.LID_MX,
                                                             lid_velocity=(0.0, 0.04, 0.01)),
        W.poiseuille(6, 20, 5, n=0.8, Re=10.0, umax=0.02, name="b_chan"),
        W.LatticeSpec(nx=9, ny=11, nz=7, K=0.02, n=1.0, periodic=(1, 1, 1), force=(2e-5, -1e-5, 0.0),
                      name="b_periodic"),
        # a periodic x axis wider than one wave, and a lattice whose rows all lie on a z face (nz = 2)
        W.cavity(8, 0.05, 1.1, 70.0, name="b_px100").with_(nx=100, ny=7, nz=6, periodic=(1, 0, 0)),
        W.cavity(8, 0.04, 0.7, 40.0, name="b_slab").with_(nx=40, ny=5, nz=2, periodic=(0, 0, 1)),
    ]


# the fully periodic box has no walls to drive it: a larger perturbation
# keeps its velocities well above the FP64 noise floor
EPS = [1e-3, 1e-3, 1e-3, 1e-3, 5e-2, 1e-3, 1e-3]


@pytest.mark.parametrize("layout,passes", [("rows", 0), ("rows", 1), ("rows", 3), ("planes", 0)])
def test_batch_matches_oracle_per_instance(clbm, layout, passes):
    """Row layout: items of one row run (passes = 0) or packed passes of 64
    consecutive nodes of a z layer (1 and 3 passes per item)."""
    specs = _mixed_specs()
    steps = 70
    b = clbm.Batch(specs, storage="f64", layout=layout)
    b.init_rest()
    for i, sp in enumerate(specs):
        b.init_populations(i, W.perturbed_populations(sp, 40 + i, EPS[i], device="cuda"))
    b.set_config(graph_steps=20, passes=passes)
    b.step(steps)          # three graph replays and ten plain launches
    torch.cuda.synchronize()
    for i, sp in enumerate(specs):
        print(f"[gpu] batch {layout} instance {i} {sp.name}", flush=True)
        _, u = b.macroscopic(i)
        f = oracle.run(sp, W.perturbed_populations(sp, 40 + i, EPS[i]).numpy(), steps)
        _, u_ref = oracle.macroscopic(sp, f)
        err = np.abs(u.cpu().numpy() - u_ref).max() / np.abs(u_ref).max()
        assert err < 1e-12, (sp.name, err)


# The batch kernel and the single-lattice kernel inline the same collision
# code but may contract multiply-adds differently, so they agree to rounding
# rather than bit for bit: a few ulp of the populations (FP32) or of the
# stored FP16 deviations.
ATOL = {"f32": 2e-6, "f16": 2e-4}


@pytest.mark.parametrize("layout", ["rows", "planes"])
@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_batch_equals_per_instance_launches(clbm, storage, layout):
    specs = _mixed_specs()
    outs = []
    for mode in ("batch", "each"):
        b = clbm.Batch(specs, storage=storage, layout=layout)
        b.init_rest()
        for i, sp in enumerate(specs):
            b.init_populations(i, W.perturbed_populations(sp, 7 + i, 1e-3, device="cuda"))
        (b.step if mode == "batch" else b.step_each)(33)
        outs.append([b.populations(i).cpu().numpy() for i in range(len(specs))])
        assert b.state() == (1, 33)
        b.close()
    for x, y in zip(*outs):
        err = np.abs(x - y).max()
        print(f"batch vs per-instance {storage}: {err:.3e}")
        assert err < ATOL[storage]


@pytest.mark.parametrize("layout", ["rows", "planes"])
def test_graph_replay_equals_plain_launches(clbm, layout):
    specs = _mixed_specs()
    outs = []
    for k in (0, 8, 9):
        b = clbm.Batch(specs, storage="f32", layout=layout)
        b.init_rest()
        b.set_config(graph_steps=k)
        b.step(5)
        b.step(27)
        b.step(3)
        outs.append([b.populations(i).cpu().numpy() for i in range(len(specs))])
    for other in outs[1:]:
        for x, y in zip(outs[0], other):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_packings_agree(clbm, storage):
    """Row layout: one row run per item and packed items of 1, 2 and 5
    passes give the same state to rounding (the kernels may contract
    multiply-adds differently; FP16 stores the same stochastic rounding)."""
    specs = _mixed_specs()
    outs = []
    for passes in (0, 1, 2, 5):
        b = clbm.Batch(specs, storage=storage, layout="rows")
        b.set_config(passes=passes)
        b.init_rest()
        for i, sp in enumerate(specs):
            b.init_populations(i, W.perturbed_populations(sp, 17 + i, 1e-3, device="cuda"))
        b.step(21)
        outs.append([b.populations(i).cpu().numpy() for i in range(len(specs))])
        b.close()
    for other in outs[1:]:
        for x, y in zip(outs[0], other):
            assert np.abs(x - y).max() < ATOL[storage]
    with pytest.raises(clbm.ClbmError):
        clbm.Batch(specs, storage="f32", layout="planes").set_config(passes=2)


@pytest.mark.parametrize("layout", ["rows", "planes"])
def test_store_hint_gives_same_bits(clbm, layout):
    """Plain and non-temporal stores (the nt_stores choice of the batch
    configuration) write the same values."""
    specs = _mixed_specs()
    outs = []
    for nt in (0, 1):
        b = clbm.Batch(specs, storage="f32", layout=layout)
        b.init_rest()
        for i, sp in enumerate(specs):
            b.init_populations(i, W.perturbed_populations(sp, 3 + i, 1e-3, device="cuda"))
        b.set_config(nt_stores=nt)
        assert b.get_config()["nt_stores"] == nt
        b.step(12)
        outs.append([b.populations(i).cpu().numpy() for i in range(len(specs))])
        if nt == 1:
            with pytest.raises(clbm.ClbmError):
                b.set_config(nt_stores=2)
        b.close()
    for x, y in zip(*outs):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("layout", ["rows", "planes"])
def test_grid_size_gives_same_bits(clbm, layout):
    """A persistent grid (one workgroup per CU, each wave striding over many
    items), a mid-size one and the default (at most one item per wave) write
    the same values; the configuration rejects grids outside 1..1024
    workgroups per CU."""
    specs = _mixed_specs()
    outs = []
    for bpc in (1024, 1, 3):
        b = clbm.Batch(specs, storage="f32", layout=layout)
        b.init_rest()
        for i, sp in enumerate(specs):
            b.init_populations(i, W.perturbed_populations(sp, 5 + i, 1e-3, device="cuda"))
        b.set_config(blocks_per_cu=bpc, graph_steps=4)
        assert b.get_config()["blocks_per_cu"] == bpc
        b.step(11)
        outs.append([b.populations(i).cpu().numpy() for i in range(len(specs))])
        for bad in (0, 1025):
            with pytest.raises(clbm.ClbmError):
                b.set_config(blocks_per_cu=bad)
        b.close()
    for other in outs[1:]:
        for x, y in zip(outs[0], other):
            assert np.array_equal(x, y)


def test_autotune_keeps_state_and_caches(clbm, tmp_path):
    specs = _mixed_specs()
    cache = str(tmp_path / "tune.txt")
    b = clbm.Batch(specs, storage="f32", tune_cache=cache)
    b.init_rest()
    b.step(10)
    before = [b.populations(i).cpu().numpy() for i in range(len(specs))]
    cfg, ms = b.autotune()
    after = [b.populations(i).cpu().numpy() for i in range(len(specs))]
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    assert ms > 0 and os.path.exists(cache)
    b2 = clbm.Batch(specs, storage="f32", tune_cache=cache)
    assert b2.get_config() == cfg
    # different instance set: no cached entry applies
    b3 = clbm.Batch(specs[:2], storage="f32", tune_cache=cache)
    assert b3.get_config() != cfg or cfg == clbm.Batch(specs[:2], storage="f32").get_config()


@pytest.mark.parametrize("layout", ["rows", "planes"])
def test_cavity_batch64_full_size(clbm, layout):
    """The 64-cavity batch (edges 32..96, n in [0.4, 1.6], Re in [50, 1000])
    at full size: the graph-replayed batch launch agrees with one launch
    per instance, and every instance keeps its mass (closed cavities)."""
    specs = W.config_batch()
    print(f"[gpu] 64-cavity batch {layout}", flush=True)
    b = clbm.Batch(specs, storage="f32", layout=layout)
    b.init_rest()
    r0 = b.reduce()
    b.autotune()
    b.step(40)
    ref = clbm.Batch(specs, storage="f32", layout=layout)
    ref.init_rest()
    ref.step_each(40)
    r1 = b.reduce(raise_unstable=False)
    for i in range(len(specs)):
        err = np.abs(b.populations(i).cpu().numpy() - ref.populations(i).cpu().numpy()).max()
        assert err < ATOL["f32"], (i, err)
        assert r1[i]["nonfinite"] == 0
        assert abs(r1[i]["mass"] - r0[i]["mass"]) < 1e-5 * r0[i]["mass"]


def _oracle_post_collision(spec, seed, eps, pt, k):
    """Oracle post-collision populations at node pt of a cavity after k steps,
    from the (2k+1)^3 sub-box of the same counter-generated initial state
    (the node cannot see beyond it within k steps)."""
    lo = [max(0, c - k) for c in pt]
    hi = [min(n, c + k + 1) for c, n in zip(pt, (spec.nx, spec.ny, spec.nz))]
    lid = spec.lid_face if hi[1] == spec.ny else W.LID_NONE     # the lid is the +y face
    sub = spec.with_(nx=hi[0] - lo[0], ny=hi[1] - lo[1], nz=hi[2] - lo[2], lid_face=lid)
    box = ((lo[0], hi[0]), (lo[1], hi[1]), (lo[2], hi[2]))
    f = oracle.run(sub, W.perturbed_populations(spec, seed, eps, box=box).numpy(), k)
    return oracle.collide(sub, f)[:, pt[2] - lo[2], pt[1] - lo[1], pt[0] - lo[0]]


@pytest.mark.parametrize("layout", ["rows", "planes"])
def test_cavity_batch64_light_cone(clbm, layout):
    """The 64-cavity batch at full size in the tuned launch the benchmark times,
    from a perturbed start: sampled nodes of six instances (lid corner, x face,
    interior, bottom wall) against the oracle after k steps."""
    specs = W.config_batch()
    k, eps, seed0 = 6, 2e-3, 500
    print(f"[gpu] 64-cavity batch light cone {layout}", flush=True)
    b = clbm.Batch(specs, storage="f32", layout=layout)
    b.init_rest()
    for i, sp in enumerate(specs):
        b.init_populations(i, W.perturbed_populations(sp, seed0 + i, eps, device="cuda"))
    b.autotune()            # trial launches write the spare pool only
    b.step(k)
    torch.cuda.synchronize()
    picks = sorted(int(i) for i in np.random.default_rng(7).choice(len(specs), 6, replace=False))
    for i in picks:
        sp = specs[i]
        f = b.populations(i).cpu().numpy()
        for p in [(0, sp.ny - 1, 0), (sp.nx - 1, sp.ny // 2, sp.nz - 1), (sp.nx // 2, sp.ny // 2, sp.nz // 2),
                  (sp.nx // 3, 0, sp.nz // 2)]:
            ref = _oracle_post_collision(sp, seed0 + i, eps, p, k)
            err = np.abs(f[:, p[2], p[1], p[0]] - ref).max()
            assert err < 1e-6, (i, sp.nx, p, err)
    b.close()
