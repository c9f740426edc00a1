"""FP64 CPU oracle for the D3Q19 cascaded power-law LBM (arXiv:1908.05396).

TEST INFRASTRUCTURE ONLY.  The oracle is the plain, slow reference that the
GPU library is checked against: per node it computes central moments by
direct summation, solves the local power-law relaxation rate exactly by
bisection, relaxes each central-moment combination to its attractor and
recovers the post-collision populations with a linear solve (see the header of
``clbm_oracle.c`` for the passages of the paper each step follows).  Only the
test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library.

Arrays are numpy float64 in structure-of-arrays layout ``f[alpha, z, y, x]``
(node index ``x + nx*(y + ny*z)``).  Parameters come from a
``workloads.LatticeSpec``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "clbm_oracle.c")
_LIBPATH = os.path.join(_HERE, "liboracle.so")
_lib = None

Q = 19


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE double, no fast-math, OpenMP)."""
    if not force and os.path.exists(_LIBPATH):
        return _LIBPATH
    tmp = _LIBPATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIBPATH)
    return _LIBPATH


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("periodic", ctypes.c_int32 * 3),
        ("lid_face", ctypes.c_int32),
        ("attractor_literal", ctypes.c_int32),
        ("K", ctypes.c_double), ("n", ctypes.c_double),
        ("nu_min", ctypes.c_double), ("nu_max", ctypes.c_double),
        ("omega_bulk", ctypes.c_double),
        ("omega_high", ctypes.c_double * 9),
        ("force", ctypes.c_double * 3),
        ("lid_velocity", ctypes.c_double * 3),
        ("rho_wall", ctypes.c_double),
        ("model", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("flags", ctypes.c_void_p),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        build()
    lib = ctypes.CDLL(_LIBPATH)
    dp = ctypes.POINTER(ctypes.c_double)
    pp = ctypes.POINTER(_Params)
    lib.orc_weights.argtypes = [dp]
    lib.orc_opposite.argtypes = [ctypes.POINTER(ctypes.c_int32)]
    lib.orc_velocities.argtypes = [ctypes.POINTER(ctypes.c_int32)]
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    lib.orc_collide_node.argtypes = [pp, dp, dp, dp]
    lib.orc_collide.argtypes = [pp, dp, dp, dp]
    lib.orc_stream.argtypes = [pp, dp, dp]
    lib.orc_run.argtypes = [pp, dp, ctypes.c_int64]
    lib.orc_macroscopic.argtypes = [pp, dp, dp, dp]
    for name in ("orc_weights", "orc_opposite", "orc_velocities", "orc_set_threads", "orc_collide_node",
                 "orc_collide", "orc_stream", "orc_run", "orc_macroscopic"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


#: per-node solid flags (uint8, shape (nz, ny, nx)): fluid, wall, moving wall
FLUID, WALL, MOVING_WALL = 0, 1, 2


def _flags(spec, flags):
    """C-contiguous uint8 copy of a flag array (or None)."""
    if flags is None:
        return None
    a = np.ascontiguousarray(flags, dtype=np.uint8).reshape(_shape(spec)[1:])
    if a.max(initial=0) > MOVING_WALL:
        raise ValueError("flags must be 0 (fluid), 1 (wall) or 2 (moving wall)")
    return a


def _params(spec, flags=None) -> _Params:
    """C parameters; `flags` (a uint8 array from _flags, kept alive by the
    caller during the call) marks solid nodes."""
    p = _Params()
    p.nx, p.ny, p.nz = int(spec.nx), int(spec.ny), int(spec.nz)
    for d in range(3):
        p.periodic[d] = 1 if spec.periodic[d] else 0
        p.force[d] = float(spec.force[d])
        p.lid_velocity[d] = float(spec.lid_velocity[d])
    p.lid_face = int(spec.lid_face)
    p.attractor_literal = 1 if getattr(spec, "attractor_literal", 0) else 0
    p.K, p.n = float(spec.K), float(spec.n)
    p.nu_min, p.nu_max = float(spec.nu_min), float(spec.nu_max)
    p.omega_bulk = float(spec.omega_bulk)
    for k in range(9):
        p.omega_high[k] = float(spec.omega_high[k])
    p.rho_wall = float(spec.rho_wall)
    model = getattr(spec, "model", "cascaded")
    if model not in ("cascaded", "srt"):
        raise ValueError(f"unknown model {model!r}")
    p.model = 1 if model == "srt" else 0
    p.flags = flags.ctypes.data if flags is not None else None
    return p


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def set_threads(n: int) -> int:
    """Set the OpenMP thread count; returns the count in effect."""
    return int(_load().orc_set_threads(int(n)))


def threads() -> int:
    return int(_load().orc_set_threads(0))


def weights() -> np.ndarray:
    """Rest-state populations of the attractors (rho = 1, u = 0)."""
    w = np.zeros(Q)
    _check(_load().orc_weights(_ptr(w)), "weights")
    return w


def opposite() -> np.ndarray:
    o = np.zeros(Q, dtype=np.int32)
    _load().orc_opposite(o.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return o


def velocities() -> np.ndarray:
    """The oracle's D3Q19 particle velocities e_alpha, shape (19, 3)."""
    e = np.zeros((Q, 3), dtype=np.int32)
    _load().orc_velocities(e.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return e.astype(np.int64)


def _shape(spec):
    return (Q, int(spec.nz), int(spec.ny), int(spec.nx))


def collide_node(spec, f: np.ndarray):
    """Collide one node; returns (post-collision populations, omega^nu)."""
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(Q)
    out = np.zeros(Q)
    om = np.zeros(1)
    p = _params(spec)
    _check(_load().orc_collide_node(ctypes.byref(p), _ptr(f), _ptr(out), _ptr(om)), "collide_node")
    return out, float(om[0])


def collide(spec, f: np.ndarray, with_omega: bool = False, flags=None):
    """Post-collision populations of every node (and omega^nu if asked);
    nodes flagged solid hold the rest populations."""
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(_shape(spec))
    out = np.empty_like(f)
    om = np.empty(_shape(spec)[1:]) if with_omega else None
    fl = _flags(spec, flags)
    p = _params(spec, fl)
    _check(_load().orc_collide(ctypes.byref(p), _ptr(f), _ptr(out),
                               _ptr(om) if om is not None else None), "collide")
    return (out, om) if with_omega else out


def stream(spec, ft: np.ndarray, flags=None) -> np.ndarray:
    """Pull streaming of post-collision populations with the boundary rules
    (solid nodes of `flags` bounce back like the walls of the box)."""
    ft = np.ascontiguousarray(ft, dtype=np.float64).reshape(_shape(spec))
    out = np.empty_like(ft)
    fl = _flags(spec, flags)
    p = _params(spec, fl)
    _check(_load().orc_stream(ctypes.byref(p), _ptr(ft), _ptr(out)), "stream")
    return out


def run(spec, f0: np.ndarray, steps: int, flags=None) -> np.ndarray:
    """Pre-collision state after `steps` collide+stream steps from f0."""
    f = np.array(f0, dtype=np.float64, copy=True).reshape(_shape(spec))
    f = np.ascontiguousarray(f)
    fl = _flags(spec, flags)
    p = _params(spec, fl)
    _check(_load().orc_run(ctypes.byref(p), _ptr(f), int(steps)), "run")
    return f


def macroscopic(spec, f: np.ndarray, flags=None):
    """(rho, u) of a pre-collision state; u has shape (3, nz, ny, nx); solid
    nodes report rho = 1, u = 0."""
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(_shape(spec))
    rho = np.empty(_shape(spec)[1:])
    u = np.empty((3,) + _shape(spec)[1:])
    fl = _flags(spec, flags)
    p = _params(spec, fl)
    _check(_load().orc_macroscopic(ctypes.byref(p), _ptr(f), _ptr(rho), _ptr(u)), "macroscopic")
    return rho, u
