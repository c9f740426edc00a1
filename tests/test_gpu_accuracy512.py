"""FP16-deviation storage against FP64 storage on the 512^3 lid-driven cavity
(Re 3200, n 0.75, lid velocity 0.04, from rest), the workload of the
benchmark: the velocity field after 5000 steps, normwise (max |du| / max |u|).

The 2e-3 bound on FP16 velocity fields is met at the benchmark's 6100 steps
(1.75e-3) but not at 5000 steps, where the measured error is 2.06e-3: the case
is carried as a strict expected failure with that number.  Stochastic rounding
is keyed by node and collision index, so the result is reproducible."""
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

STEPS = 5000


@pytest.fixture(scope="module")
def clbm():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1908_05396_amd import clbm as c
    c.load()
    return c


def _field(clbm, spec, storage):
    print(f"[gpu] cavity512 {storage} {STEPS} steps", flush=True)
    lat = clbm.Lattice(spec, storage=storage, track_residual=False)
    lat.init_rest()
    lat.step(STEPS)
    _, u = lat.macroscopic()
    torch.cuda.synchronize()
    lat.close()
    return u


@pytest.mark.xfail(strict=True, reason="FP16 storage, 512^3 Re 3200 cavity at 5000 steps: field error 2.06e-3 "
                                       "against FP64 (measured), over the 2e-3 bound (1.75e-3 at 6100 steps)")
def test_fp16_field_error_cavity512(clbm):
    spec = W.config_cavity512()
    u64 = _field(clbm, spec, "f64")
    u16 = _field(clbm, spec, "f16")
    err = ((u16 - u64).abs().max() / u64.abs().max()).item()
    del u16, u64
    torch.cuda.empty_cache()
    print(f"    FP16 vs FP64 field error after {STEPS} steps: {err:.4e}")
    assert err < 2e-3
