"""Seeded synthetic inputs and workload descriptions.

This module is shared by the tests, the benchmark and the smoke check, which
hand its outputs both to the GPU library and to the CPU oracle.  It holds no
part of the method's arithmetic: only problem descriptions (lattice sizes,
boundary types, power-law parameters, driving), the Reynolds-number bookkeeping
that turns a stated Re into a consistency coefficient, and a counter-based
random generator for perturbed initial states.

Workloads follow the benchmark problems of the paper (Sec. 4): a power-law
Poiseuille channel driven by a body force (Sec. 4.1), and the lid-driven cubic
cavity (Sec. 4.3) at several sizes, power-law indices and Reynolds numbers.
The paper's own data (figures, the comparison benchmark of its Sec. 4.3) are
not used; every input here is synthetic.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Tuple

import numpy as np

#: textbook D3Q19 lattice weights (rest 1/3, faces 1/18, edges 1/36) in the
#: paper's velocity order; used only to shape perturbed initial states.
INPUT_WEIGHTS = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12, dtype=np.float64)

#: default viscosity clip: omega^nu kept in [0.1, 1.95], i.e. nu = (1/omega - 1/2)/3
NU_MIN_DEFAULT = (1.0 / 1.95 - 0.5) / 3.0
NU_MAX_DEFAULT = (1.0 / 0.1 - 0.5) / 3.0

# lid faces
LID_NONE, LID_MX, LID_PX, LID_MY, LID_PY, LID_MZ, LID_PZ = range(7)


@dataclass(frozen=True)
class LatticeSpec:
    """One lattice problem, in lattice units (dx = dt = 1)."""

    nx: int
    ny: int
    nz: int
    K: float                      # consistency coefficient mu_p
    n: float                      # power-law index
    periodic: Tuple[int, int, int] = (0, 0, 0)
    lid_face: int = LID_NONE
    lid_velocity: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    force: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    nu_min: float = NU_MIN_DEFAULT
    nu_max: float = NU_MAX_DEFAULT
    omega_bulk: float = 1.0
    omega_high: Tuple[float, ...] = (1.0,) * 9
    rho_wall: float = 1.0
    attractor_literal: int = 0     # 1: fourth-order attractors without the 1/rho factor
    model: str = "cascaded"        # "cascaded" (the paper's scheme) or "srt" (its BGK comparison model)
    name: str = ""

    @property
    def nodes(self) -> int:
        return self.nx * self.ny * self.nz

    def with_(self, **kw) -> "LatticeSpec":
        return replace(self, **kw)


# ---------------------------------------------------------------------------
# Reynolds-number bookkeeping (definitions stated with each benchmark)
# ---------------------------------------------------------------------------

def cavity_K(H: float, U: float, n: float, Re: float, rho: float = 1.0) -> float:
    """Consistency coefficient for a cavity: Re = rho H^n U^(2-n) / mu_p (Sec. 4.3)."""
    return rho * H ** n * U ** (2.0 - n) / Re


def channel_K(H: float, umax: float, n: float, Re: float, rho: float = 1.0) -> float:
    """Channel: Re = rho (H/2)^n u_max^(2-n) / mu_p (Sec. 4.1)."""
    return rho * (H / 2.0) ** n * umax ** (2.0 - n) / Re


def channel_force(H: float, umax: float, n: float, K: float) -> float:
    """Body force giving centreline velocity umax in the power-law channel:
    u_max = n/(n+1) (F/mu_p)^(1/n) (H/2)^((n+1)/n) (Sec. 4.1), solved for F."""
    return K * (umax * (n + 1.0) / n / (H / 2.0) ** ((n + 1.0) / n)) ** n


def cavity(L: int, U: float, n: float, Re: float, lid_axis_len=None, name="") -> LatticeSpec:
    """Cubic lid-driven cavity: all six faces are half-way bounce-back walls,
    the +y face moves with velocity (U, 0, 0)."""
    return LatticeSpec(nx=L, ny=L, nz=L, K=cavity_K(L, U, n, Re), n=n, periodic=(0, 0, 0),
                       lid_face=LID_PY, lid_velocity=(U, 0.0, 0.0), name=name or f"cavity{L}")


def poiseuille(nx: int, ny: int, nz: int, n: float, Re: float, umax: float, name="") -> LatticeSpec:
    """Channel between walls normal to y (width H = ny), periodic in x and z,
    driven by a body force along x."""
    K = channel_K(ny, umax, n, Re)
    F = channel_force(ny, umax, n, K)
    return LatticeSpec(nx=nx, ny=ny, nz=nz, K=K, n=n, periodic=(1, 0, 1), force=(F, 0.0, 0.0),
                       name=name or f"poiseuille{nx}x{ny}x{nz}")


def duct_centre_coefficient(terms: int = 60) -> float:
    """C in u_max = C F a^2 / nu for the Newtonian square duct of half width a:
    the centre value (y = z = 0) of the series solution quoted in Sec. 4.2,
    C = 16/pi^3 sum_k (-1)^(k-1) [1 - 1/cosh((2k-1) pi/2)] / (2k-1)^3."""
    k = np.arange(1, terms + 1)
    m = 2 * k - 1
    return float(16.0 / np.pi ** 3 * np.sum((-1.0) ** (k - 1) * (1.0 - 1.0 / np.cosh(m * np.pi / 2)) / m ** 3))


def duct(nx: int, H: int, n: float, Re: float, F: float = 1e-6, name="") -> LatticeSpec:
    """Square duct (Sec. 4.2): walls normal to y and z, H fluid nodes across
    (half width a = H/2 with half-way walls), periodic along x, body force F
    along x.  Re = u_max a / nu with the Newtonian centre velocity
    u_max = C F a^2 / nu, so nu = sqrt(C F a^3 / Re); that nu is used as the
    consistency K for every n (rho = 1)."""
    a = H / 2.0
    K = float(np.sqrt(duct_centre_coefficient() * F * a ** 3 / Re))
    return LatticeSpec(nx=nx, ny=H, nz=H, K=K, n=n, periodic=(1, 0, 0), force=(F, 0.0, 0.0),
                       name=name or f"duct{nx}x{H}x{H}_n{n}_re{Re:g}")


# ---------------------------------------------------------------------------
# The five benchmark workloads
# ---------------------------------------------------------------------------

def config_poiseuille() -> LatticeSpec:
    """8x32x8 power-law channel, n = 0.5, Re = 10, u_max = 0.01 (FP64, 2000 steps)."""
    return poiseuille(8, 32, 8, n=0.5, Re=10.0, umax=0.01, name="poiseuille_8x32x8_n0.5_re10")


def config_cavity64(n: float) -> LatticeSpec:
    """64^3 cavity, U = 0.05, Re = 100, n in {0.5, 1.0, 1.5} (20000 steps)."""
    return cavity(64, 0.05, n, 100.0, name=f"cavity64_re100_n{n}")


def config_cavity256() -> LatticeSpec:
    """256^3 cavity, Re = 1000, n = 0.5, U = 0.05 (50000 steps)."""
    return cavity(256, 0.05, 0.5, 1000.0, name="cavity256_re1000_n0.5")


def config_cavity512() -> LatticeSpec:
    """512^3 cavity, Re = 3200, n = 0.75, U = 0.04 (5000 steps)."""
    return cavity(512, 0.04, 0.75, 3200.0, name="cavity512_re3200_n0.75")


def config_batch(count: int = 64, seed: int = 0, lmin: int = 32, lmax: int = 96):
    """Batch of cubic cavities: L ~ U{lmin..lmax}, n ~ U[0.4, 1.6],
    Re ~ U[50, 1000], U = 0.05 (numpy PCG64, fixed seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Ls = rng.integers(lmin, lmax + 1, size=count)
    ns = rng.uniform(0.4, 1.6, size=count)
    Res = rng.uniform(50.0, 1000.0, size=count)
    return [cavity(int(L), 0.05, float(n), float(Re), name=f"batch{i}_L{int(L)}")
            for i, (L, n, Re) in enumerate(zip(Ls, ns, Res))]


# ---------------------------------------------------------------------------
# Counter-based random numbers (SplitMix64, Steele, Lea & Flood 2014)
# ---------------------------------------------------------------------------
# Evaluated with torch int64 tensors so the same values come out on the CPU
# and on the GPU, for the whole lattice or for any sub-box of it.

_GOLDEN = -7046029254386353131      # 0x9E3779B97F4A7C15 as int64
_MIX1 = -4658895280553007687        # 0xBF58476D1CE4E5B9
_MIX2 = -7723592293110705685        # 0x94D049BB133111EB


def _lsr(z, s: int):
    """Logical right shift of int64 tensors (torch's >> is arithmetic)."""
    return (z >> s) & ((1 << (64 - s)) - 1)


def splitmix_uniform(counter, seed: int):
    """Uniform doubles in [-1, 1) from int64 counters (torch tensor)."""
    import torch
    z = counter + (int(seed) * 0x100000000 + 0x5DEECE66D)
    z = z + _GOLDEN
    z = (z ^ _lsr(z, 30)) * _MIX1
    z = (z ^ _lsr(z, 27)) * _MIX2
    z = z ^ _lsr(z, 31)
    top = _lsr(z, 11).to(torch.float64)          # 53 random bits, exact in double
    return top * (2.0 / 9007199254740992.0) - 1.0


def perturbed_populations(spec: LatticeSpec, seed: int, eps: float = 1e-3, device="cpu",
                          box=None, dtype=None):
    """Initial populations f0 = w (1 + eps * xi), xi ~ U[-1, 1) i.i.d. per
    (alpha, node), drawn by counter from the global node coordinates, so any
    sub-box reproduces the values of the full lattice.

    Returns a torch float64 tensor of shape (19, nz', ny', nx') for the box
    ``((x0, x1), (y0, y1), (z0, z1))`` (half-open, default the whole lattice).
    """
    import torch
    if box is None:
        box = ((0, spec.nx), (0, spec.ny), (0, spec.nz))
    (x0, x1), (y0, y1), (z0, z1) = box
    nxy = spec.nx * spec.ny
    N = spec.nx * spec.ny * spec.nz
    xs = torch.arange(x0, x1, dtype=torch.int64, device=device)
    ys = torch.arange(y0, y1, dtype=torch.int64, device=device)
    zs = torch.arange(z0, z1, dtype=torch.int64, device=device)
    node = (zs.view(-1, 1, 1) * nxy + ys.view(1, -1, 1) * spec.nx + xs.view(1, 1, -1))
    w = torch.tensor(INPUT_WEIGHTS, dtype=torch.float64, device=device)
    out = torch.empty((19, z1 - z0, y1 - y0, x1 - x0), dtype=torch.float64, device=device)
    for a in range(19):
        xi = splitmix_uniform(node + a * N, seed)
        out[a] = w[a] * (1.0 + eps * xi)
    return out if dtype is None else out.to(dtype)


def rest_populations(spec: LatticeSpec, device="cpu"):
    import torch
    w = torch.tensor(INPUT_WEIGHTS, dtype=torch.float64, device=device)
    return w.view(19, 1, 1, 1).expand(19, spec.nz, spec.ny, spec.nx).contiguous()
