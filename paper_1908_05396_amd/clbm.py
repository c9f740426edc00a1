"""ctypes binding of libclbm.so (the C-ABI declared in include/clbm.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of the library.  PyTorch provides device memory and streams.  If the library
is not built, importing this module raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libclbm.so")

Q = 19
STORAGE = {"f64": 0, "f32": 1, "f16": 2}
COLLISION = {"auto": 0, "central": 1, "ghat": 2, "srt": 3}
LAYOUT = {"planes": 0, "rows": 1}
STORAGE_DTYPE = {0: torch.float64, 1: torch.float32, 2: torch.float16}

CLBM_OK, CLBM_EINVAL, CLBM_ENOMEM, CLBM_EHIP, CLBM_EUNSTABLE, CLBM_ESTATE = 0, -1, -2, -3, -4, -5
CLBM_FLUID, CLBM_WALL, CLBM_MOVING_WALL = 0, 1, 2
OUT_PREC = {"f64": 0, "f32": 1}
OUT_DTYPE = {"f64": torch.float64, "f32": torch.float32}


class ClbmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"clbm error {status}: {message}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("periodic", ctypes.c_int32 * 3),
        ("lid_face", ctypes.c_int32),
        ("storage", ctypes.c_int32),
        ("attractor_literal", ctypes.c_int32),
        ("track_residual", ctypes.c_int32),
        ("plane_pad", ctypes.c_int32),
        ("collision", ctypes.c_int32),
        ("layout", ctypes.c_int32),
        ("f16_rounding", ctypes.c_int32),
        ("K", ctypes.c_double), ("n", ctypes.c_double),
        ("nu_min", ctypes.c_double), ("nu_max", ctypes.c_double),
        ("omega_bulk", ctypes.c_double),
        ("omega_high", ctypes.c_double * 9),
        ("force", ctypes.c_double * 3),
        ("lid_velocity", ctypes.c_double * 3),
        ("rho_wall", ctypes.c_double),
    ]


class Launch(ctypes.Structure):
    _fields_ = [("bx", ctypes.c_int32), ("by", ctypes.c_int32), ("xcd_remap", ctypes.c_int32),
                ("nt_loads", ctypes.c_int32), ("nt_stores", ctypes.c_int32), ("fuse_steps", ctypes.c_int32),
                ("fuse_rows", ctypes.c_int32), ("fuse_planes", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class BatchConfig(ctypes.Structure):
    _fields_ = [("bx", ctypes.c_int32), ("by", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("graph_steps", ctypes.c_int32), ("nt_stores", ctypes.c_int32), ("passes", ctypes.c_int32)]


_lib = None

#: every function the header declares, with (restype, argtypes)
_VP, _DP, _I32P, _I64P = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), \
    ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)
_PP = ctypes.POINTER(Params)
SIGNATURES = {
    "clbm_params_default": (ctypes.c_int, [_PP]),
    "clbm_buffer_size": (ctypes.c_int, [_PP, _I64P, ctypes.POINTER(ctypes.c_size_t)]),
    "clbm_create": (ctypes.c_int, [_PP, _VP, _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
    "clbm_create_in_place": (ctypes.c_int, [_PP, _VP, ctypes.c_size_t, ctypes.POINTER(_VP)]),
    "clbm_init_rest": (ctypes.c_int, [_VP, _VP]),
    "clbm_init_populations": (ctypes.c_int, [_VP, _VP, ctypes.c_int, _VP]),
    "clbm_step": (ctypes.c_int, [_VP, ctypes.c_int64, _VP]),
    "clbm_macroscopic": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int32, _VP]),
    "clbm_populations": (ctypes.c_int, [_VP, _VP, _VP]),
    "clbm_reduce": (ctypes.c_int, [_VP, _DP, _VP]),
    "clbm_reduce_noalloc": (ctypes.c_int, [_VP, _VP, _VP]),
    "clbm_state": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int), _I64P]),
    "clbm_set_launch": (ctypes.c_int, [_VP, ctypes.POINTER(Launch)]),
    "clbm_get_launch": (ctypes.c_int, [_VP, ctypes.POINTER(Launch)]),
    "clbm_set_block": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32]),
    "clbm_get_block": (ctypes.c_int, [_VP, _I32P, _I32P]),
    "clbm_autotune": (ctypes.c_int, [_VP, _VP, ctypes.POINTER(Launch), _DP]),
    "clbm_destroy": (ctypes.c_int, [_VP]),
    "clbm_last_error": (ctypes.c_char_p, []),
    "clbm_version": (ctypes.c_char_p, []),
    "clbm_lattice_tables": (ctypes.c_int, [_I32P, _I32P, _DP]),
    "clbm_copy_probe": (ctypes.c_int, [_VP, _VP, ctypes.c_size_t, _VP]),
    "clbm_f16_round": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int64, ctypes.c_int32, _VP]),
    "clbm_batch_size": (ctypes.c_int, [_PP, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "clbm_batch_create": (ctypes.c_int, [_PP, ctypes.c_int32, _VP, _VP, ctypes.c_size_t, ctypes.c_char_p,
                                         ctypes.POINTER(_VP)]),
    "clbm_batch_init_rest": (ctypes.c_int, [_VP, _VP]),
    "clbm_batch_init_populations": (ctypes.c_int, [_VP, ctypes.c_int32, _VP, ctypes.c_int, _VP]),
    "clbm_batch_step": (ctypes.c_int, [_VP, ctypes.c_int64, _VP]),
    "clbm_batch_step_each": (ctypes.c_int, [_VP, ctypes.c_int64, _VP]),
    "clbm_batch_macroscopic": (ctypes.c_int, [_VP, ctypes.c_int32, _VP, _VP, ctypes.c_int32, _VP]),
    "clbm_batch_populations": (ctypes.c_int, [_VP, ctypes.c_int32, _VP, _VP]),
    "clbm_batch_reduce": (ctypes.c_int, [_VP, _DP, _VP]),
    "clbm_batch_autotune": (ctypes.c_int, [_VP, _VP, ctypes.POINTER(BatchConfig), _DP]),
    "clbm_batch_set_config": (ctypes.c_int, [_VP, ctypes.POINTER(BatchConfig)]),
    "clbm_batch_get_config": (ctypes.c_int, [_VP, ctypes.POINTER(BatchConfig)]),
    "clbm_batch_state": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int), _I64P]),
    "clbm_batch_destroy": (ctypes.c_int, [_VP]),
}


def load():
    """Load libclbm.so.  Raises if it has not been built, or if it was built
    from other sources than those in the tree (stale library)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise ImportError(f"{LIBPATH} is not built; run __graft_entry__.build() "
                          "(python -m paper_1908_05396_amd.build)")
    lib = ctypes.CDLL(LIBPATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    from . import build as _build
    built = lib.clbm_version().decode().rsplit(" src ", 1)[-1]
    want = _build.source_hash()
    if built != want:
        raise ImportError(f"{LIBPATH} was built from other sources (hash {built}, tree {want}); rebuild it "
                          "with __graft_entry__.build()")
    _lib = lib
    return lib


def _check(rc: int):
    if rc != CLBM_OK:
        raise ClbmError(rc, load().clbm_last_error().decode())


def version() -> str:
    return load().clbm_version().decode()


def lattice_tables():
    """(e[19,3], opposite[19], w[19]) compiled into the kernels."""
    import numpy as np
    e = (ctypes.c_int32 * (3 * Q))()
    o = (ctypes.c_int32 * Q)()
    w = (ctypes.c_double * Q)()
    _check(load().clbm_lattice_tables(e, o, w))
    return (np.array(list(e), dtype=np.int64).reshape(Q, 3), np.array(list(o)), np.array(list(w)))


def copy_probe(src: torch.Tensor, dst: torch.Tensor, stream=None):
    """Plain device copy of src into dst (bandwidth reference)."""
    nbytes = min(src.numel() * src.element_size(), dst.numel() * dst.element_size())
    nbytes -= nbytes % 16
    _check(load().clbm_copy_probe(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                  ctypes.c_size_t(nbytes), _stream(stream)))
    return nbytes


F16_ROUNDING = {"stochastic": 0, "nearest": 1}


def f16_round(x: torch.Tensor, seeds: torch.Tensor = None, stream=None) -> torch.Tensor:
    """The library's FP16 rounding of float32 device values: stochastic with
    the given uint32 seeds (stored as int32), or nearest even if seeds is
    None.  Returns float16."""
    x = x.contiguous()
    assert x.is_cuda and x.dtype == torch.float32
    out = torch.empty(x.shape, dtype=torch.float16, device=x.device)
    mode = 1 if seeds is None else 0
    sp = None
    if seeds is not None:
        seeds = seeds.contiguous()
        assert seeds.is_cuda and seeds.dtype == torch.int32 and seeds.numel() == x.numel()
        sp = ctypes.c_void_p(seeds.data_ptr())
    _check(load().clbm_f16_round(ctypes.c_void_p(x.data_ptr()), sp, ctypes.c_void_p(out.data_ptr()),
                                 int(x.numel()), mode, _stream(stream)))
    return out


def params_from_spec(spec, storage: str = "f32", track_residual: bool = True, plane_pad: int = -1,
                     collision: str = "auto", layout: str = "rows", f16_rounding: str = "stochastic") -> Params:
    """Fill the C parameter struct from a problem description with the
    attributes of workloads.LatticeSpec."""
    p = Params()
    _check(load().clbm_params_default(ctypes.byref(p)))
    p.nx, p.ny, p.nz = int(spec.nx), int(spec.ny), int(spec.nz)
    for d in range(3):
        p.periodic[d] = 1 if spec.periodic[d] else 0
        p.force[d] = float(spec.force[d])
        p.lid_velocity[d] = float(spec.lid_velocity[d])
    p.lid_face = int(spec.lid_face)
    p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    p.attractor_literal = int(getattr(spec, "attractor_literal", 0))
    p.track_residual = 1 if track_residual else 0
    p.plane_pad = int(plane_pad)
    if getattr(spec, "model", "cascaded") == "srt":
        collision = "srt"
    p.collision = COLLISION[collision] if isinstance(collision, str) else int(collision)
    p.layout = LAYOUT[layout] if isinstance(layout, str) else int(layout)
    p.f16_rounding = F16_ROUNDING[f16_rounding] if isinstance(f16_rounding, str) else int(f16_rounding)
    p.K, p.n = float(spec.K), float(spec.n)
    p.nu_min, p.nu_max = float(spec.nu_min), float(spec.nu_max)
    p.omega_bulk = float(spec.omega_bulk)
    for k in range(9):
        p.omega_high[k] = float(spec.omega_high[k])
    p.rho_wall = float(spec.rho_wall)
    return p


def buffer_size(p: Params):
    plane = ctypes.c_int64()
    nbytes = ctypes.c_size_t()
    _check(load().clbm_buffer_size(ctypes.byref(p), ctypes.byref(plane), ctypes.byref(nbytes)))
    return int(plane.value), int(nbytes.value)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Lattice:
    """One lattice on one GPU: two state buffers owned by torch, a library
    handle, and thin wrappers of the C calls."""

    def __init__(self, spec, storage: str = "f32", device="cuda", track_residual: bool = True,
                 block=None, plane_pad: int = -1, launch: dict = None, collision: str = "auto",
                 in_place: bool = False, layout: str = None, flags: torch.Tensor = None,
                 f16_rounding: str = "stochastic"):
        """layout: "rows" or "planes"; None picks planes for two steps per
        launch (which need them), rows otherwise.  flags: optional uint8
        tensor of shape (nz, ny, nx) with CLBM_FLUID / CLBM_WALL /
        CLBM_MOVING_WALL per node (kept on the device for the lattice's
        lifetime)."""
        lib = load()
        self.spec = spec
        self.storage = storage
        self.in_place = bool(in_place)
        if layout is None:
            two_step = bool(launch) and int(launch.get("fuse_steps", 1)) == 2
            layout = "planes" if two_step else "rows"
        self.layout = layout
        self.params = params_from_spec(spec, storage, track_residual, plane_pad, collision, layout, f16_rounding)
        self.plane, self.nbytes = buffer_size(self.params)
        self.device = torch.device(device)
        nbuf = 1 if self.in_place else 2
        self.buffers = [torch.empty(self.nbytes, dtype=torch.uint8, device=self.device) for _ in range(nbuf)]
        self.flags = None
        if flags is not None:
            if self.in_place:
                raise ValueError("the one-buffer form takes no per-node flags")
            self.flags = flags.to(device=self.device, dtype=torch.uint8).contiguous()
            assert self.flags.numel() == self.nodes, "flags must hold nx*ny*nz values"
        h = ctypes.c_void_p()
        if self.in_place:
            _check(lib.clbm_create_in_place(ctypes.byref(self.params), ctypes.c_void_p(self.buffers[0].data_ptr()),
                                            ctypes.c_size_t(self.nbytes), ctypes.byref(h)))
        else:
            fl = ctypes.c_void_p(self.flags.data_ptr()) if self.flags is not None else None
            _check(lib.clbm_create(ctypes.byref(self.params), ctypes.c_void_p(self.buffers[0].data_ptr()),
                                   ctypes.c_void_p(self.buffers[1].data_ptr()), ctypes.c_size_t(self.nbytes),
                                   fl, ctypes.byref(h)))
        self._h = h
        if block is not None:
            self.set_block(*block)
        if launch:
            self.set_launch(**launch)

    @property
    def nodes(self) -> int:
        return self.params.nx * self.params.ny * self.params.nz

    @property
    def shape(self):
        return (self.params.nz, self.params.ny, self.params.nx)

    def close(self):
        if getattr(self, "_h", None):
            load().clbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- state -------------------------------------------------------------
    def init_rest(self, stream=None):
        _check(load().clbm_init_rest(self._h, _stream(stream)))

    def init_populations(self, f0: torch.Tensor, stream=None):
        """f0: float64 tensor of shape (19, nz, ny, nx) on the device, or on
        the host (the library then stages it and synchronizes)."""
        on_device = f0.is_cuda
        f0 = f0.to(device=self.device if on_device else "cpu", dtype=torch.float64).contiguous()
        assert f0.numel() == Q * self.nodes, "f0 must hold 19 x nx*ny*nz values"
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        _check(load().clbm_init_populations(self._h, ctypes.c_void_p(f0.data_ptr()), 1 if on_device else 0,
                                            _stream(s)))
        if on_device and s != torch.cuda.current_stream(self.device):
            f0.record_stream(s)     # the launch may still read f0 after this returns

    def step(self, nsteps: int, stream=None):
        _check(load().clbm_step(self._h, int(nsteps), _stream(stream)))

    def state(self):
        idx = ctypes.c_int()
        steps = ctypes.c_int64()
        _check(load().clbm_state(self._h, ctypes.byref(idx), ctypes.byref(steps)))
        return idx.value, steps.value

    def state_tensor(self) -> torch.Tensor:
        """The current state buffer of a planes-layout lattice as
        (19, plane_stride) deviations f - w."""
        if self.layout != "planes":
            raise ValueError("state_tensor: planes layout only (state_view works for both)")
        idx, _ = self.state()
        dt = STORAGE_DTYPE[self.params.storage]
        return self.buffers[idx].view(dt).view(Q, self.plane)

    def state_view(self) -> torch.Tensor:
        """The current state buffer as a (19, nz, ny, nx) view of the stored
        deviations f - w, in either layout (no copy)."""
        idx, _ = self.state()
        dt = STORAGE_DTYPE[self.params.storage]
        nz, ny, nx = self.shape
        flat = self.buffers[idx].view(dt)
        if self.layout == "planes":
            return flat[:Q * self.plane].view(Q, self.plane)[:, :self.nodes].view(Q, nz, ny, nx)
        return flat[:Q * self.nodes].view(nz, ny, Q, nx).permute(2, 0, 1, 3)

    # -- outputs -----------------------------------------------------------
    def macroscopic(self, stream=None, out_prec: str = "f64"):
        """(rho, u) at the current time, u of shape (3, nz, ny, nx), as float64
        (out_prec "f64") or float32 ("f32")."""
        dt = OUT_DTYPE[out_prec]
        rho = torch.empty(self.shape, dtype=dt, device=self.device)
        u = torch.empty((3,) + self.shape, dtype=dt, device=self.device)
        _check(load().clbm_macroscopic(self._h, ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                       OUT_PREC[out_prec], _stream(stream)))
        return rho, u

    def populations(self, stream=None) -> torch.Tensor:
        f = torch.empty((Q,) + self.shape, dtype=torch.float64, device=self.device)
        _check(load().clbm_populations(self._h, ctypes.c_void_p(f.data_ptr()), _stream(stream)))
        return f

    def reduce(self, stream=None, raise_unstable: bool = True) -> dict:
        out = (ctypes.c_double * 8)()
        rc = load().clbm_reduce(self._h, out, _stream(stream))
        if rc != CLBM_OK and not (rc == CLBM_EUNSTABLE and not raise_unstable):
            _check(rc)
        keys = ("mass", "momentum_x", "momentum_y", "momentum_z", "residual", "nonfinite", "umax", "kinetic")
        return dict(zip(keys, list(out)))

    def reduce_noalloc(self, out: torch.Tensor, stream=None):
        """clbm_reduce_noalloc: the eight reductions of reduce() written
        asynchronously into `out` (a float64 device tensor of 8 values)."""
        assert out.is_cuda and out.dtype == torch.float64 and out.numel() >= 8 and out.is_contiguous()
        _check(load().clbm_reduce_noalloc(self._h, ctypes.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    # -- launch shape ------------------------------------------------------
    def set_block(self, bx: int, by: int):
        _check(load().clbm_set_block(self._h, int(bx), int(by)))

    def autotune(self, stream=None):
        """Time block shapes, tile orders and cache hints on the current state
        (left unchanged) and keep the fastest; returns (launch dict, ms per step)."""
        c = Launch()
        ms = ctypes.c_double()
        _check(load().clbm_autotune(self._h, _stream(stream), ctypes.byref(c), ctypes.byref(ms)))
        return {k: getattr(c, k) for k, _ in Launch._fields_ if k != "reserved"}, float(ms.value)

    def set_launch(self, **kw):
        c = Launch()
        _check(load().clbm_get_launch(self._h, ctypes.byref(c)))
        for k, v in kw.items():
            setattr(c, k, int(v))
        _check(load().clbm_set_launch(self._h, ctypes.byref(c)))

    def get_launch(self) -> dict:
        c = Launch()
        _check(load().clbm_get_launch(self._h, ctypes.byref(c)))
        return {k: getattr(c, k) for k, _ in Launch._fields_ if k != "reserved"}

    def get_block(self):
        bx, by = ctypes.c_int32(), ctypes.c_int32()
        _check(load().clbm_get_block(self._h, ctypes.byref(bx), ctypes.byref(by)))
        return bx.value, by.value


class Batch:
    """Many lattices (one problem description each, shared storage type)
    stepped together, one batched launch per step."""

    def __init__(self, specs, storage: str = "f32", device="cuda", track_residual: bool = False,
                 tune_cache: str = None, collision: str = "auto", layout: str = "rows",
                 f16_rounding: str = "stochastic"):
        lib = load()
        self.specs = list(specs)
        self.storage = storage
        self.layout = layout
        n = len(self.specs)
        arr = (Params * n)()
        for i, sp in enumerate(self.specs):
            arr[i] = params_from_spec(sp, storage, track_residual, -1, collision, layout, f16_rounding)
        self._params = arr
        nbytes = ctypes.c_size_t()
        _check(lib.clbm_batch_size(arr, n, ctypes.byref(nbytes)))
        self.nbytes = int(nbytes.value)
        self.device = torch.device(device)
        self.pools = [torch.empty(self.nbytes, dtype=torch.uint8, device=self.device) for _ in range(2)]
        h = ctypes.c_void_p()
        _check(lib.clbm_batch_create(arr, n, ctypes.c_void_p(self.pools[0].data_ptr()),
                                     ctypes.c_void_p(self.pools[1].data_ptr()), ctypes.c_size_t(self.nbytes),
                                     tune_cache.encode() if tune_cache else None, ctypes.byref(h)))
        self._h = h

    @property
    def count(self) -> int:
        return len(self.specs)

    @property
    def nodes(self) -> int:
        return sum(s.nx * s.ny * s.nz for s in self.specs)

    def close(self):
        if getattr(self, "_h", None):
            load().clbm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_rest(self, stream=None):
        _check(load().clbm_batch_init_rest(self._h, _stream(stream)))

    def init_populations(self, i: int, f0: torch.Tensor, stream=None):
        sp = self.specs[i]
        on_device = f0.is_cuda
        f0 = f0.to(device=self.device if on_device else "cpu", dtype=torch.float64).contiguous()
        assert f0.numel() == Q * sp.nx * sp.ny * sp.nz
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        _check(load().clbm_batch_init_populations(self._h, int(i), ctypes.c_void_p(f0.data_ptr()),
                                                  1 if on_device else 0, _stream(s)))
        if on_device and s != torch.cuda.current_stream(self.device):
            f0.record_stream(s)

    def step(self, nsteps: int, stream=None):
        _check(load().clbm_batch_step(self._h, int(nsteps), _stream(stream)))

    def step_each(self, nsteps: int, stream=None):
        _check(load().clbm_batch_step_each(self._h, int(nsteps), _stream(stream)))

    def macroscopic(self, i: int, stream=None, out_prec: str = "f64"):
        sp = self.specs[i]
        shape = (sp.nz, sp.ny, sp.nx)
        dt = OUT_DTYPE[out_prec]
        rho = torch.empty(shape, dtype=dt, device=self.device)
        u = torch.empty((3,) + shape, dtype=dt, device=self.device)
        _check(load().clbm_batch_macroscopic(self._h, int(i), ctypes.c_void_p(rho.data_ptr()),
                                             ctypes.c_void_p(u.data_ptr()), OUT_PREC[out_prec], _stream(stream)))
        return rho, u

    def populations(self, i: int, stream=None):
        sp = self.specs[i]
        f = torch.empty((Q, sp.nz, sp.ny, sp.nx), dtype=torch.float64, device=self.device)
        _check(load().clbm_batch_populations(self._h, int(i), ctypes.c_void_p(f.data_ptr()), _stream(stream)))
        return f

    def reduce(self, stream=None, raise_unstable: bool = True):
        out = (ctypes.c_double * (8 * self.count))()
        rc = load().clbm_batch_reduce(self._h, out, _stream(stream))
        if rc != CLBM_OK and not (rc == CLBM_EUNSTABLE and not raise_unstable):
            _check(rc)
        keys = ("mass", "momentum_x", "momentum_y", "momentum_z", "residual", "nonfinite", "umax", "kinetic")
        vals = list(out)
        return [dict(zip(keys, vals[8 * i:8 * i + 8])) for i in range(self.count)]

    def autotune(self, stream=None):
        c = BatchConfig()
        ms = ctypes.c_double()
        _check(load().clbm_batch_autotune(self._h, _stream(stream), ctypes.byref(c), ctypes.byref(ms)))
        return {k: getattr(c, k) for k, _ in BatchConfig._fields_}, ms.value

    def set_config(self, **kw):
        c = BatchConfig()
        _check(load().clbm_batch_get_config(self._h, ctypes.byref(c)))
        for k, v in kw.items():
            setattr(c, k, int(v))
        _check(load().clbm_batch_set_config(self._h, ctypes.byref(c)))

    def get_config(self) -> dict:
        c = BatchConfig()
        _check(load().clbm_batch_get_config(self._h, ctypes.byref(c)))
        return {k: getattr(c, k) for k, _ in BatchConfig._fields_}

    def state(self):
        idx = ctypes.c_int()
        steps = ctypes.c_int64()
        _check(load().clbm_batch_state(self._h, ctypes.byref(idx), ctypes.byref(steps)))
        return idx.value, steps.value
