"""GPU (HIP, through the C-ABI) versus the FP64 CPU oracle on the same seeded
inputs.

Tolerances (normwise: max over nodes and components of |u_gpu - u_ref|
divided by max |u_ref|): FP64 storage 1e-12, FP32 storage 1e-5, FP16
deviation storage 2e-3.  Post-collision populations after a single collision
are compared element by element with bounds derived from the storage
precision (see each test).
"""
import functools

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


@functools.lru_cache(maxsize=None)
def _oracle_u(spec, seed, eps, steps):
    if seed is None:
        f0 = W.rest_populations(spec).numpy()
    else:
        f0 = W.perturbed_populations(spec, seed, eps).numpy()
    f = oracle.run(spec, f0, steps)
    rho, u = oracle.macroscopic(spec, f)
    return rho, u


def _gpu_run(clbm, spec, storage, seed, eps, steps, block=None, layout="rows"):
    print(f"[gpu] {spec.name} {spec.nx}x{spec.ny}x{spec.nz} storage={storage} layout={layout} seed={seed} "
          f"steps={steps} block={block}", flush=True)
    lat = clbm.Lattice(spec, storage=storage, block=block, layout=layout)
    if seed is None:
        lat.init_rest()
    else:
        lat.init_populations(W.perturbed_populations(spec, seed, eps, device="cuda"))
    lat.step(steps)
    rho, u = lat.macroscopic()
    torch.cuda.synchronize()
    out = (rho.cpu().numpy(), u.cpu().numpy(), lat)
    return out


def _normwise(u, ref):
    return np.abs(u - ref).max() / np.abs(ref).max()


@pytest.mark.parametrize("storage,tol", [("f64", 5e-15), ("f32", 1e-6), ("f16", 2e-5)])
def test_single_collision_populations(clbm, storage, tol):
    """One collision of a strongly perturbed state (eps = 2e-2, so every
    non-equilibrium moment is present): post-collision populations agree
    element by element.  Bounds: FP64 a few ulp of O(1) values; FP32 about 16
    ulp of the largest population; FP16 the rounding of deviations of size
    ~1e-2 (2^-11 relative) plus FP32 arithmetic."""
    spec = W.cavity(16, 0.05, 0.6, 100.0).with_(nx=13, ny=11, nz=9, name="collide13x11x9")
    f0 = W.perturbed_populations(spec, 7, 2e-2)
    lat = clbm.Lattice(spec, storage=storage)
    lat.init_populations(f0.to("cuda"))
    f_gpu = lat.populations().cpu().numpy()
    f_ref = oracle.collide(spec, f0.numpy())
    err = np.abs(f_gpu - f_ref).max()
    print(f"collide {storage}: max abs diff {err:.3e}")
    assert err < tol


@pytest.mark.parametrize("layout", ["rows", "planes"])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_poiseuille_config(clbm, storage, layout):
    """8x32x8 power-law channel (n = 0.5, Re = 10, u_max = 0.01, body force),
    2000 steps from rest.  The force changes the populations by ~1e-7 per
    step, below half an FP16 ulp of the stored deviations: nearest-even
    rounding would drop it, stochastic rounding keeps it on average."""
    spec = W.config_poiseuille()
    rho_ref, u_ref = _oracle_u(spec, None, 0.0, 2000)
    rho, u, _ = _gpu_run(clbm, spec, storage, None, 0.0, 2000, layout=layout)
    err = _normwise(u, u_ref)
    print(f"poiseuille {storage} {layout}: {err:.3e}")
    assert err < TOL_U[storage]


@pytest.mark.parametrize("storage,stop,cap", [("f64", 1e-9, 300000), ("f32", 1e-7, 300000)])
def test_poiseuille_config_steady_state(clbm, storage, stop, cap):
    """The 8x32x8 power-law channel (n = 0.5, Re = 10, u_max = 0.01) from
    rest, run until the residual |u(t) - u(t - 1000)| / |u(t)| falls below
    `stop` (FP32: its rounding floor is higher), then against the closed-form
    profile of Sec. 4.1, u(y) = n/(n+1) (F/K)^(1/n) [(H/2)^((n+1)/n) -
    |y|^((n+1)/n)].  The closed form is the unclipped power law, so the
    viscosity clip is kept below the near-wall viscosity (omega up to 1.99).
    Expected relative L2 error at H = 32: of order 1e-3 (second order)."""
    spec = W.config_poiseuille().with_(nu_min=(1.0 / 1.99 - 0.5) / 3.0)
    n, K, F, H = spec.n, spec.K, spec.force[0], spec.ny
    yc = np.arange(H) - (H - 1) / 2
    ua = n / (n + 1) * (F / K) ** (1 / n) * ((H / 2) ** ((n + 1) / n) - np.abs(yc) ** ((n + 1) / n))
    print(f"[gpu] poiseuille steady state {storage}", flush=True)
    lat = clbm.Lattice(spec, storage=storage, track_residual=True)
    lat.init_rest()
    lat.reduce()
    steps, r = 0, 1.0
    while steps < cap:
        lat.step(1000)
        steps += 1000
        r = lat.reduce()["residual"]
        if r < stop:
            break
    _, u = lat.macroscopic()
    u = u.cpu().numpy()
    prof = u[0].mean(axis=(0, 2))                    # uniform along x and z
    assert np.abs(u[0] - prof[None, :, None]).max() < 1e-12 * np.abs(prof).max() + (0 if storage == "f64" else 1e-6)
    err = np.sqrt(((prof - ua) ** 2).sum() / (ua ** 2).sum())
    print(f"poiseuille {storage}: {steps} steps, residual {r:.2e}, L2 error vs closed form {err:.3e}, "
          f"u_max {prof.max():.6e} (closed form {ua.max():.6e})")
    assert r < stop
    assert err < 5e-3


@pytest.mark.parametrize("layout", ["rows", "planes"])
@pytest.mark.parametrize("n", [0.5, 1.0, 1.5])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_cavity16_power_law(clbm, n, storage, layout):
    """16^3 lid-driven cavity, U = 0.05, Re = 100, perturbed start (seed 1234,
    eps 1e-3), 300 steps (16 nodes along x: every lane takes the full wall
    rule in the row layout)."""
    spec = W.cavity(16, 0.05, n, 100.0, name=f"cavity16_n{n}")
    rho_ref, u_ref = _oracle_u(spec, 1234, 1e-3, 300)
    rho, u, _ = _gpu_run(clbm, spec, storage, 1234, 1e-3, 300, layout=layout)
    err = _normwise(u, u_ref)
    print(f"cavity16 n={n} {storage} {layout}: {err:.3e}")
    assert err < TOL_U[storage]


@pytest.mark.parametrize("layout", ["rows", "planes"])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_ragged_lattice(clbm, storage, layout):
    """70 x 20 x 9 cavity: two 64-wide tiles along x with a ragged tail of 6,
    odd y and z extents."""
    spec = W.cavity(20, 0.05, 0.8, 50.0).with_(nx=70, ny=20, nz=9, name="cavity70x20x9")
    rho_ref, u_ref = _oracle_u(spec, 99, 1e-3, 80)
    rho, u, _ = _gpu_run(clbm, spec, storage, 99, 1e-3, 80, layout=layout)
    err = _normwise(u, u_ref)
    print(f"ragged {storage} {layout}: {err:.3e}")
    assert err < TOL_U[storage]


@pytest.mark.parametrize("layout", ["rows", "planes"])
@pytest.mark.parametrize("nx", [12, 64])
def test_periodic_mixed_walls(clbm, nx, layout):
    """A duct periodic along x with walls in y and z and a lid on +z (a lid on
    a periodic axis would be invalid).  nx = 64: whole waves, so the row
    layout takes its fast kernel with the periodic x-face rule."""
    spec = W.LatticeSpec(nx=nx, ny=10, nz=8, K=0.02, n=1.3, periodic=(1, 0, 0), lid_face=W.LID_PZ,
                         lid_velocity=(0.03, 0.01, 0.0), name=f"duct_lidz_{nx}")
    rho_ref, u_ref = _oracle_u(spec, 5, 1e-3, 150)
    rho, u, _ = _gpu_run(clbm, spec, "f64", 5, 1e-3, 150, layout=layout)
    assert _normwise(u, u_ref) < TOL_U["f64"]


@pytest.mark.parametrize("layout", ["rows", "planes"])
def test_block_shape_does_not_change_results(clbm, layout):
    """Row layout: widths that are multiples of 64 take the fast kernel, the
    others the full-rule kernel; both give the same bits."""
    spec = W.cavity(20, 0.05, 0.7, 100.0).with_(nx=96, name="cavity96x20x20")
    results = []
    for block in [(64, 1), (64, 4), (32, 2), (128, 2), (96, 2)]:
        _, u, _ = _gpu_run(clbm, spec, "f32", 4, 1e-3, 30, block=block, layout=layout)
        results.append(u)
    for u in results[1:]:
        assert np.array_equal(u, results[0])


def test_reductions(clbm):
    """FP64 reductions: total mass of a closed cavity is conserved (the lid
    terms cancel pairwise), momentum matches the oracle, no NaN."""
    spec = W.cavity(16, 0.05, 0.5, 100.0, name="cavity16_red")
    lat = clbm.Lattice(spec, storage="f64")
    lat.init_populations(W.perturbed_populations(spec, 1234, 1e-3, device="cuda"))
    r0 = lat.reduce()
    lat.step(300)
    r1 = lat.reduce()
    assert abs(r1["mass"] - r0["mass"]) < 1e-12 * spec.nodes
    rho_ref, u_ref = _oracle_u(spec, 1234, 1e-3, 300)
    mom = (rho_ref[None] * u_ref).reshape(3, -1).sum(axis=1)
    assert np.allclose([r1["momentum_x"], r1["momentum_y"], r1["momentum_z"]], mom, rtol=0, atol=1e-12)
    assert r1["nonfinite"] == 0
    assert r1["umax"] == pytest.approx(np.sqrt((u_ref ** 2).sum(axis=0)).max(), rel=1e-12)
    assert r0["residual"] == 0.0       # no earlier velocity to compare with


@pytest.mark.parametrize("in_place", [False, True])
@pytest.mark.parametrize("storage,tol", [("f64", 1e-9), ("f32", 1e-3)])
def test_residual_matches_oracle_fields(clbm, storage, tol, in_place):
    """The steady-state residual |u(t) - u(t - k)|_2 / |u(t)|_2 of clbm_reduce
    (its velocity snapshot is kept in FP64) against the same quantity
    computed from two oracle velocity fields k = 100 steps apart.  Bounds:
    FP64 rounding of a 1e-2 relative difference; FP32 the 1e-6 relative
    error of each velocity field over that difference."""
    spec = W.cavity(16, 0.05, 0.7, 100.0, name="cavity16_residual")
    lat = clbm.Lattice(spec, storage=storage, track_residual=True, in_place=in_place)
    lat.init_populations(W.perturbed_populations(spec, 77, 1e-3, device="cuda"))
    lat.step(200)
    assert lat.reduce()["residual"] == 0.0
    lat.step(100)
    r = lat.reduce()["residual"]
    _, ua = _oracle_u(spec, 77, 1e-3, 200)
    _, ub = _oracle_u(spec, 77, 1e-3, 300)
    ref = np.sqrt(((ub - ua) ** 2).sum() / (ub ** 2).sum())
    print(f"residual {storage} in_place={in_place}: {r:.6e} vs oracle {ref:.6e}")
    assert ref > 1e-3
    assert abs(r - ref) <= tol * ref


def test_reduce_reports_nonfinite(clbm):
    spec = W.cavity(8, 0.05, 1.0, 10.0, name="cavity8_nan")
    f0 = W.rest_populations(spec).clone()
    f0[3, 2, 2, 2] = float("nan")
    lat = clbm.Lattice(spec, storage="f32")
    lat.init_populations(f0.to("cuda"))
    with pytest.raises(clbm.ClbmError) as ei:
        lat.reduce()
    assert ei.value.status == clbm.CLBM_EUNSTABLE
    assert lat.reduce(raise_unstable=False)["nonfinite"] >= 1


def test_init_rest_with_force_matches_oracle(clbm):
    spec = W.config_poiseuille()
    lat = clbm.Lattice(spec, storage="f64")
    lat.init_rest()
    f = lat.populations().cpu().numpy()
    ref = oracle.collide(spec, W.rest_populations(spec).numpy())
    assert np.abs(f - ref).max() < 1e-15


# ---------------------------------------------------------------------------
# The paper's printed form of the collision (changes of moments g4..g18 and
# f~ = f + K.g) and relaxation rates other than one for the bulk and the
# higher moments
# ---------------------------------------------------------------------------

# an anisotropic set that the oracle keeps stable in the 16^3 cavity at
# Re = 100 (some choices of higher-order rates are not)
GENERAL_OMEGAS = dict(omega_bulk=1.15, omega_high=(1.2, 1.1, 1.3, 0.95, 0.9, 1.05, 1.1, 1.2, 0.85))


@pytest.mark.parametrize("storage,tol", [("f64", 5e-15), ("f32", 1e-6)])
@pytest.mark.parametrize("omegas", ["unit", "general"])
def test_ghat_single_collision(clbm, storage, tol, omegas):
    spec = W.cavity(16, 0.05, 0.6, 100.0).with_(nx=13, ny=11, nz=9, name="ghat13x11x9")
    if omegas == "general":
        spec = spec.with_(**GENERAL_OMEGAS)
    f0 = W.perturbed_populations(spec, 7, 2e-2)
    lat = clbm.Lattice(spec, storage=storage, collision="ghat")
    lat.init_populations(f0.to("cuda"))
    f_gpu = lat.populations().cpu().numpy()
    f_ref = oracle.collide(spec, f0.numpy())
    err = np.abs(f_gpu - f_ref).max()
    print(f"ghat collide {storage} {omegas}: {err:.3e}")
    assert err < tol


@pytest.mark.parametrize("forced", [False, True])
def test_ghat_and_central_forms_agree(clbm, forced):
    spec = W.cavity(16, 0.05, 1.3, 100.0).with_(nx=10, ny=12, nz=8, name="forms10x12x8")
    if forced:
        spec = spec.with_(force=(2e-5, -1e-5, 5e-6))
    f0 = W.perturbed_populations(spec, 21, 2e-2).to("cuda")
    out = []
    for form in ("central", "ghat"):
        lat = clbm.Lattice(spec, storage="f64", collision=form)
        lat.init_populations(f0)
        out.append(lat.populations().cpu().numpy())
    assert np.abs(out[0] - out[1]).max() < 5e-16


def test_ghat_poiseuille_config(clbm):
    spec = W.config_poiseuille()
    rho_ref, u_ref = _oracle_u(spec, None, 0.0, 2000)
    print(f"[gpu] {spec.name} ghat f64", flush=True)
    lat = clbm.Lattice(spec, storage="f64", collision="ghat")
    lat.init_rest()
    lat.step(2000)
    _, u = lat.macroscopic()
    assert _normwise(u.cpu().numpy(), u_ref) < TOL_U["f64"]


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_general_omegas_cavity(clbm, storage):
    """omega_9 and omega_10..18 away from one (tunable higher-order rates):
    the printed-form kernel against the oracle's direct relaxation of each
    central-moment combination with its own rate."""
    spec = W.cavity(16, 0.05, 0.8, 100.0, name="cavity16_general").with_(**GENERAL_OMEGAS)
    rho_ref, u_ref = _oracle_u(spec, 1234, 1e-3, 200)
    rho, u, _ = _gpu_run(clbm, spec, storage, 1234, 1e-3, 200)
    err = _normwise(u, u_ref)
    print(f"general omegas {storage}: {err:.3e}")
    assert err < TOL_U[storage]


def test_literal_attractor_single_collision(clbm):
    spec = W.cavity(8, 0.05, 0.9, 50.0).with_(attractor_literal=1, name="literal8")
    f0 = W.perturbed_populations(spec, 5, 3e-2)
    for form in ("central", "ghat"):
        lat = clbm.Lattice(spec, storage="f64", collision=form)
        lat.init_populations(f0.to("cuda"))
        err = np.abs(lat.populations().cpu().numpy() - oracle.collide(spec, f0.numpy())).max()
        assert err < 5e-15, (form, err)


def test_central_form_rejects_general_omegas(clbm):
    spec = W.cavity(8, 0.05, 1.0, 50.0).with_(**GENERAL_OMEGAS)
    with pytest.raises(clbm.ClbmError):
        clbm.Lattice(spec, storage="f32", collision="central")


# ---------------------------------------------------------------------------
# Square duct (Sec. 4.2): body force along the periodic axis, walls on two
# axes.  Parity with the oracle for Newtonian and power-law fluids, and the
# Newtonian steady state against the series solution printed in Sec. 4.2.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("n", [1.0, 0.7, 1.4])
def test_duct_parity(clbm, storage, n):
    """Square duct (3 x 45 x 45, F = 1e-6, Re = 80) from a perturbed start,
    2000 steps; the force per step lies below the FP16 resolution of the
    stored deviations, which stochastic rounding carries on average."""
    # at 2000 steps the forced flow (F t = 2e-3) dominates the decayed start
    # perturbation and |u| stays far above the FP64 rounding of the oracle's
    # full populations (~1e-17 absolute per operation)
    spec = W.duct(3, 45, n, 80.0)
    steps = 2000
    rho_ref, u_ref = _oracle_u(spec, 3, 1e-3, steps)
    _, u, lat = _gpu_run(clbm, spec, storage, 3, 1e-3, steps)
    lat.close()
    err = _normwise(u, u_ref)
    print(f"duct n={n} {storage}: {err:.3e} (max |u| {np.abs(u_ref).max():.2e})")
    assert err < TOL_U[storage]


def _series(H, F, nu, terms=80):
    a = H / 2.0
    c = np.arange(H) - (H - 1) / 2.0
    Y, Z = np.meshgrid(c, c, indexing="ij")
    u = np.zeros_like(Y)
    for k in range(1, terms + 1):
        m = 2 * k - 1
        u += ((-1.0) ** (k - 1) * (1.0 - np.cosh(m * np.pi * Z / (2 * a)) / np.cosh(m * np.pi / 2))
              * np.cos(m * np.pi * Y / (2 * a)) / m ** 3)
    return 16.0 * a ** 2 * F / (nu * np.pi ** 3) * u


@pytest.mark.parametrize("Re", [80.0, 20.0])
def test_duct_steady_state_matches_series(clbm, Re):
    """3 x 45 x 45 duct, F = 1e-6 (the paper's set-up), FP64, run until the
    velocity changes by less than 1e-7 relative per 5000 steps (the residual
    compares with an FP32 snapshot, whose rounding floor is ~3e-8).  Bound: the
    oracle's second-order pin gives 4.8e-3 at H = 16 (Re 2); scaled by
    (16/45)^2 that is 6e-4 at H = 45, and the bound allows a factor 5 for the
    relaxation-rate dependence of the half-way wall position (omega 1.93 and
    1.86 here against 1.79 there)."""
    spec = W.duct(3, 45, 1.0, Re)
    lat = clbm.Lattice(spec, storage="f64", track_residual=True)
    lat.init_rest()
    steps = 0
    while steps < 600000:
        lat.step(5000)
        steps += 5000
        r = lat.reduce()
        if steps > 20000 and r["residual"] < 1e-7:
            break
    _, u = lat.macroscopic()
    lat.close()
    got = u[0].cpu().numpy()                       # (z, y, x)
    ua = _series(45, spec.force[0], spec.K)        # [y, z]
    prof = got[:, :, 1].T                          # [y, z]
    assert np.abs(got[:, :, 0] - got[:, :, 2]).max() < 1e-14 * np.abs(got).max()   # uniform along x
    err = np.sqrt(((prof - ua) ** 2).sum() / (ua ** 2).sum())
    print(f"duct Re={Re}: {steps} steps, residual {r['residual']:.2e}, L2 error vs series {err:.3e}, "
          f"u_max {prof.max():.4e} (series {ua.max():.4e})")
    assert r["residual"] < 1e-7
    assert err < 3e-3


# ---------------------------------------------------------------------------
# The single-relaxation-time comparison model (Sec. 5), same power law
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("storage,tol", [("f64", 5e-15), ("f32", 1e-6), ("f16", 2e-5)])
def test_srt_single_collision_populations(clbm, storage, tol):
    """One BGK collision of a strongly perturbed state, element by element
    (bounds as for the cascaded collision)."""
    spec = W.cavity(16, 0.05, 0.6, 100.0).with_(nx=13, ny=11, nz=9, model="srt", name="srt13x11x9")
    f0 = W.perturbed_populations(spec, 7, 2e-2)
    lat = clbm.Lattice(spec, storage=storage)
    lat.init_populations(f0.to("cuda"))
    f_gpu = lat.populations().cpu().numpy()
    lat.close()
    f_ref = oracle.collide(spec, f0.numpy())
    err = np.abs(f_gpu - f_ref).max()
    print(f"srt collide {storage}: max abs diff {err:.3e}")
    assert err < tol


SRT_F16_XFAIL = pytest.mark.xfail(
    strict=True, reason="BGK comparison model, n = 0.5, FP16 storage: 6.2e-3 normwise at 300 steps (measured); its "
                        "near-wall relaxation rates close to the clip leave the higher moments undamped, which keeps "
                        "the FP16 rounding noise; the paper's cascaded scheme meets 2e-3 on the same case")


@pytest.mark.parametrize("storage,n", [(st, n) for st in ("f64", "f32") for n in (0.5, 1.0, 1.5)] +
                         [pytest.param("f16", 0.5, marks=SRT_F16_XFAIL), ("f16", 1.0), ("f16", 1.5)])
def test_srt_cavity16(clbm, n, storage):
    """16^3 cavity with the BGK model, perturbed start, 300 steps."""
    spec = W.cavity(16, 0.05, n, 100.0, name=f"srt_cavity16_n{n}").with_(model="srt")
    rho_ref, u_ref = _oracle_u(spec, 1234, 1e-3, 300)
    rho, u, lat = _gpu_run(clbm, spec, storage, 1234, 1e-3, 300)
    lat.close()
    err = _normwise(u, u_ref)
    print(f"srt cavity16 n={n} {storage}: {err:.3e}")
    assert err < TOL_U[storage]
