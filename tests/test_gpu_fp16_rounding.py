"""The FP16 rounding of the state (clbm_f16_round, the conversion every FP16
step kernel applies to its collision results), checked against its
definition: stochastic rounding returns one of the two FP16 values that
bracket the FP32 input, the upper one with probability (x - lo)/(hi - lo)
(so the expected result is x), and exact FP16 values unchanged; nearest-even
mode equals IEEE round-to-nearest-even (numpy's float16 conversion)."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

TRIALS = 8192


@pytest.fixture(scope="module")
def clbm():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1908_05396_amd import clbm as c
    c.load()
    return c


def _bracket(x32):
    """FP16 neighbours lo <= x <= hi of float32 values (equal when exact)."""
    h = x32.astype(np.float16)
    hd = h.astype(np.float64)
    xd = x32.astype(np.float64)
    lo = np.where(hd <= xd, h, np.nextafter(h, np.float16(-np.inf)))
    hi = np.where(hd >= xd, h, np.nextafter(h, np.float16(np.inf)))
    return lo.astype(np.float64), hi.astype(np.float64)


def _values():
    rng = np.random.default_rng(42)
    v = [1e-2 * (1 + k / 7) for k in range(7)] + [-3.3e-3, 4.7e-4, -5.1e-5, 7.0e-6, -2.3e-7, 1.3e-2, 0.21, -0.33]
    v += list(rng.uniform(-0.05, 0.05, size=24))
    x = np.array(v, dtype=np.float32)
    lo, hi = _bracket(x)
    mid = ((lo + hi) / 2).astype(np.float32)                  # exact halfway points
    exact = np.array([0.25, -1.0 / 64, 2.0 ** -20, 0.0], dtype=np.float32)
    return np.concatenate([x, mid[:6], exact])


def test_stochastic_rounding_is_unbiased(clbm):
    x = _values()
    lo, hi = _bracket(x)
    rng = np.random.default_rng(7)
    seeds = rng.integers(0, 2 ** 32, size=(x.size, TRIALS), dtype=np.uint64).astype(np.uint32).view(np.int32)
    xs = torch.from_numpy(np.repeat(x[:, None], TRIALS, axis=1)).cuda()
    out = clbm.f16_round(xs, torch.from_numpy(seeds).cuda()).cpu().numpy().astype(np.float64)
    for i in range(x.size):
        o = out[i]
        assert np.all((o == lo[i]) | (o == hi[i])), (x[i], np.unique(o))
        if lo[i] == hi[i]:
            continue
        p = (float(x[i]) - lo[i]) / (hi[i] - lo[i])
        got = np.mean(o == hi[i])
        sigma = np.sqrt(p * (1 - p) / TRIALS)
        print(f"x={x[i]: .4e}  P(up) expected {p:.4f} got {got:.4f}")
        assert abs(got - p) <= 5 * sigma + 2.0 ** -12, (x[i], p, got)


def test_nearest_even_mode_is_ieee(clbm):
    x = _values()
    out = clbm.f16_round(torch.from_numpy(x).cuda()).cpu().numpy()
    assert np.array_equal(out.view(np.uint16), x.astype(np.float16).view(np.uint16))


def test_state_rounding_keeps_the_mean(clbm):
    """A periodic box at rest with a uniform density excess delta: every step
    stores the deviations w_a delta again.  Nearest-even rounding stores the
    same rounded values every step, so the total mass keeps the rounding error
    of w_a delta (predicted here from IEEE float16); stochastic rounding draws
    new bits for every node, direction and step, and the mass stays at the
    exact value up to the noise of the draws."""
    import workloads as W
    spec = W.LatticeSpec(nx=64, ny=32, nz=16, K=0.02, n=1.0, periodic=(1, 1, 1), name="periodic_rest")
    delta = 2.9e-3
    w = np.asarray(W.INPUT_WEIGHTS)
    f0 = torch.from_numpy(np.broadcast_to((w * (1 + delta))[:, None, None, None], (19, 16, 32, 64)).copy())
    rne_excess = float(np.sum((w * delta).astype(np.float32).astype(np.float16).astype(np.float64)))
    assert abs(rne_excess - delta) > 1e-4 * delta          # nearest-even is visibly biased here
    excess = {}
    for mode in ("stochastic", "nearest"):
        lat = clbm.Lattice(spec, storage="f16", f16_rounding=mode)
        lat.init_populations(f0.cuda())
        lat.step(20)
        excess[mode] = lat.reduce()["mass"] / spec.nodes - 1.0
    print(f"mass excess per node: exact {delta:.8e}, stochastic {excess['stochastic']:.8e}, "
          f"nearest {excess['nearest']:.8e} (predicted {rne_excess:.8e})")
    assert abs(excess["stochastic"] - delta) < 2e-5 * delta
    assert abs(excess["nearest"] - rne_excess) < 2e-5 * delta
