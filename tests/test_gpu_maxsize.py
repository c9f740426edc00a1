"""Largest lattices the library accepts, against the oracle by light cone.

One population plane is addressed with 32-bit byte offsets, so a plane holds
at most 4 GiB - 256 bytes: 1024 x 1024 x 1023 nodes in FP32 (1.07e9 nodes,
two states of 81.5 GB each) and 2048 x 1024 x 1023 in FP16 (2.15e9 nodes, the
node index just below 2^31).  From rest, after k steps only nodes within k of
the lid have moved; sampled nodes there and at the far corners of the index
range are compared with the oracle run on (2k+1)^3 sub-boxes (see
test_gpu_fullsize.py).  The velocity is formed from the sampled post-collision
populations on the host, so no full-size output array is needed.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

K_STEPS = 6


@pytest.fixture(scope="module")
def clbm():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1908_05396_amd import clbm as c
    c.load()
    return c


def _oracle_rest(spec, pt, k):
    lo = [max(0, c - k) for c in pt]
    hi = [min(n, c + k + 1) for c, n in zip(pt, (spec.nx, spec.ny, spec.nz))]
    lid = spec.lid_face if hi[1] == spec.ny else W.LID_NONE
    sub = spec.with_(nx=hi[0] - lo[0], ny=hi[1] - lo[1], nz=hi[2] - lo[2], lid_face=lid)
    f = oracle.run(sub, W.rest_populations(sub).numpy(), k)
    ft = oracle.collide(sub, f)
    return ft[:, pt[2] - lo[2], pt[1] - lo[1], pt[0] - lo[0]]


@pytest.mark.parametrize("storage,dims,layout", [("f32", (1024, 1024, 1023), "planes"),
                                                  ("f16", (2048, 1024, 1023), "planes"),
                                                  ("f16", (2048, 1024, 1023), "rows")])
def test_largest_lattice(clbm, storage, dims, layout):
    """Planes: the largest lattices whose planes fit the 4 GiB range of a
    buffer descriptor (one more z layer is refused).  Rows: node indices are
    32-bit, and the FP16 lattice of just under 2^31 nodes runs in either
    layout."""
    nx, ny, nz = dims
    spec = W.cavity(16, 0.05, 0.8, 100.0).with_(nx=nx, ny=ny, nz=nz, name=f"max_{storage}")
    plane, nbytes = clbm.buffer_size(clbm.params_from_spec(spec, storage, layout=layout))
    esize = 4 if storage == "f32" else 2
    if layout == "planes":
        assert spec.nodes * esize <= (1 << 32) - 256 < (spec.nodes + nx * ny) * esize
    else:
        assert spec.nodes < (1 << 31) <= spec.nodes + nx * ny
    print(f"[gpu] max-size {storage} {layout} {nx}x{ny}x{nz}: {spec.nodes} nodes, 2 x {nbytes / 1e9:.1f} GB",
          flush=True)
    lat = clbm.Lattice(spec, storage=storage, track_residual=False, layout=layout)
    lat.init_rest()
    lat.step(K_STEPS)
    pts = [(nx - 1, ny - 1, nz - 1), (0, ny - 1, nz - 1), (nx - 1, ny - 1, 0), (nx // 2, ny - 1, nz // 2),
           (nx - 2, ny - 3, nz - 2), (nx // 3, ny - 5, nz - 1), (nx - 1, ny // 2, nz - 1)]
    st = lat.state_view()
    idx = torch.tensor([(p[2], p[1], p[0]) for p in pts], device="cuda")
    d = st[:, idx[:, 0], idx[:, 1], idx[:, 2]].to(torch.float64).cpu().numpy().T   # (samples, 19) deviations
    rest = lat.reduce()
    lat.close()
    del lat, st
    torch.cuda.empty_cache()
    assert rest["nonfinite"] == 0
    assert abs(rest["mass"] - spec.nodes) < 1e-6 * spec.nodes   # closed cavity: mass is conserved
    E = np.array(clbm.lattice_tables()[0], dtype=np.float64)
    w = W.INPUT_WEIGHTS
    refs = np.array([_oracle_rest(spec, p, K_STEPS) for p in pts])
    got = d + w
    u_ref = refs @ E / refs.sum(axis=1, keepdims=True)
    u_got = got @ E / got.sum(axis=1, keepdims=True)
    err = np.abs(u_got - u_ref).max() / np.abs(u_ref).max()        # normwise over the samples
    print(f"   max |u_ref| {np.abs(u_ref).max():.3e}, normwise error {err:.3e}, "
          f"populations {np.abs(got - refs).max():.3e}")
    assert err < {"f32": 1e-5, "f16": 2e-3}[storage]
    assert np.abs(got - refs).max() < {"f32": 1e-6, "f16": 2e-5}[storage]
