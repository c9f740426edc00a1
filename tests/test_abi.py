"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function declared in include/clbm.h, carries the paper's lattice
tables, and validates parameters."""
import ctypes
import os
import re
from fractions import Fraction

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


@pytest.fixture(scope="module")
def clbm():
    from paper_1908_05396_amd import clbm as c
    c.load()
    return c


def _declared_functions():
    with open(os.path.join(ROOT, "include", "clbm.h")) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(clbm_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(clbm):
    names = _declared_functions()
    assert len(names) >= 16
    lib = clbm.load()
    for name in names:
        assert hasattr(lib, name), name
        assert name in clbm.SIGNATURES, f"binding lacks {name}"


def test_version(clbm):
    assert "gfx950" in clbm.version()


def test_library_built_from_the_sources_in_the_tree(clbm):
    """clbm_version() carries the hash of the sources the library was built
    from; it must be the hash of the sources in the tree (load() refuses a
    stale library, so this also holds for every other test)."""
    from paper_1908_05396_amd import build
    assert clbm.version().endswith(" src " + build.source_hash())


def _prototypes():
    """{name: (return type, [parameter types])} of the header's functions,
    parameter names removed, whitespace normalised."""
    with open(os.path.join(ROOT, "include", "clbm.h")) as fh:
        text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
    out = {}
    for ret, name, args in re.findall(r"([A-Za-z_][\w \*]*?)\s*\b(clbm_\w+)\s*\(([^)]*)\)\s*;", text):
        params = []
        for a in args.split(","):
            a = " ".join(a.replace("*", " * ").split())
            if a in ("void", ""):
                continue
            a = re.sub(r"\[\d*\]$", "", a).strip()          # double out[8] -> double out
            toks = a.split(" ")
            if toks[-1] != "*" and len(toks) > 1:
                toks = toks[:-1]                              # drop the parameter name
            params.append(" ".join(toks).replace(" *", "*"))
        out[name] = (" ".join(ret.replace("*", " * ").split()).replace(" *", "*"), params)
    return out


# The boundary of the hot path as the scope table states it, call by call.
# Deliberate differences, each kept identical in meaning: streams are passed
# as void* (a hipStream_t is a pointer; the header then needs no HIP include,
# so plain C callers compile without ROCm), and out_prec is an int32_t
# holding a clbm_storage value (the same 4 bytes as the enum).
SCOPE_BOUNDARY = {
    "clbm_create": ["const clbm_params*", "void*", "void*", "size_t", "const uint8_t*", "clbm_lattice**"],
    "clbm_init_rest": ["clbm_lattice*", "void*"],
    "clbm_init_populations": ["clbm_lattice*", "const double*", "int", "void*"],
    "clbm_step": ["clbm_lattice*", "int64_t", "void*"],
    "clbm_macroscopic": ["clbm_lattice*", "void*", "void*", "int32_t", "void*"],
    "clbm_reduce": ["clbm_lattice*", "double", "void*"],
    "clbm_destroy": ["clbm_lattice*"],
    "clbm_last_error": [],
    "clbm_batch_create": ["const clbm_params*", "int32_t", "void*", "void*", "size_t", "const char*",
                          "clbm_batch**"],
    "clbm_batch_step": ["clbm_batch*", "int64_t", "void*"],
    "clbm_batch_reduce": ["clbm_batch*", "double*", "void*"],
    "clbm_batch_destroy": ["clbm_batch*"],
}


def test_header_matches_the_scope_boundary():
    """Every call of the scope table's boundary is declared with its
    parameter list (status return, const char* for the error message)."""
    protos = _prototypes()
    for name, params in SCOPE_BOUNDARY.items():
        assert name in protos, name
        ret, got = protos[name]
        assert got == params, (name, got)
        assert ret == ("const char*" if name == "clbm_last_error" else "clbm_status"), (name, ret)
    with open(os.path.join(ROOT, "include", "clbm.h")) as fh:
        text = fh.read()
    assert re.search(r"CLBM_FLUID\s*=\s*0,\s*CLBM_WALL\s*=\s*1,\s*CLBM_MOVING_WALL\s*=\s*2", text)
    for st, v in (("CLBM_OK", 0), ("CLBM_EINVAL", -1), ("CLBM_ENOMEM", -2), ("CLBM_EHIP", -3),
                  ("CLBM_EUNSTABLE", -4), ("CLBM_ESTATE", -5), ("CLBM_F64", 0), ("CLBM_F32", 1),
                  ("CLBM_F16_DEV", 2)):
        assert re.search(rf"\b{st}\s*=\s*{v}\b", text), st


def test_every_call_cites_the_paper():
    """Each declared call's comment block names the section or equation of
    the paper it implements, or says what non-method utility it is."""
    with open(os.path.join(ROOT, "include", "clbm.h")) as fh:
        text = fh.read()
    method_calls = ["clbm_create", "clbm_create_in_place", "clbm_init_rest", "clbm_init_populations", "clbm_step",
                    "clbm_macroscopic", "clbm_populations", "clbm_reduce", "clbm_batch_create", "clbm_batch_step",
                    "clbm_params_default"]
    for name in method_calls:
        decl = re.search(rf"^clbm_status\s+{name}\s*\(", text, flags=re.M)
        assert decl, name
        start = text.rfind("/*", 0, decl.start())
        block = text[start:decl.start()]
        assert re.search(r"Sec\. \d|Eq\.", block), name


def test_kernel_tables_match_paper(clbm):
    e, opp, w = clbm.lattice_tables()
    printed = np.loadtxt(os.path.join(GOLDEN, "paper_velocity_components.txt"))
    assert np.array_equal(e.T, printed)
    assert np.array_equal(e[opp], -e)
    with open(os.path.join(GOLDEN, "d3q19_weights.txt")) as fh:
        vals = [float(Fraction(l.strip())) for l in fh if l.strip() and not l.startswith("#")]
    assert np.array_equal(w, np.array(vals))


def test_batch_config_struct_matches_header(clbm):
    """The binding's clbm_batch_config has the header's int32 fields in order."""
    with open(os.path.join(ROOT, "include", "clbm.h")) as fh:
        text = fh.read()
    body = text[text.index("typedef struct {", text.index("typedef struct clbm_batch clbm_batch;")):
                text.index("} clbm_batch_config;")]
    names = []
    for line in body.splitlines():
        line = line.split("/*")[0].strip()
        if line.startswith("int32_t"):
            names += [n.strip() for n in line[len("int32_t"):].rstrip(";").split(",")]
    assert names == [k for k, _ in clbm.BatchConfig._fields_]
    assert ctypes.sizeof(clbm.BatchConfig) == 4 * len(names)


def test_params_struct_layout(clbm):
    assert ctypes.sizeof(clbm.Params) == 56 + 8 * (5 + 9 + 3 + 3 + 1)
    p = clbm.Params()
    assert clbm.load().clbm_params_default(ctypes.byref(p)) == 0
    assert (p.nx, p.ny, p.nz) == (1, 1, 1)
    assert p.storage == 1 and p.omega_bulk == 1.0 and p.rho_wall == 1.0
    assert p.layout == clbm.LAYOUT["rows"] and p.f16_rounding == clbm.F16_ROUNDING["stochastic"]
    assert list(p.omega_high) == [1.0] * 9


@pytest.mark.parametrize("storage,esize", [("f64", 8), ("f32", 4), ("f16", 2)])
def test_buffer_size_padding(clbm, storage, esize):
    spec = W.cavity(37, 0.05, 1.0, 100.0)
    plane, nbytes = clbm.buffer_size(clbm.params_from_spec(spec, storage, layout="planes"))
    assert plane >= spec.nodes and (plane * esize) % 256 == 0 and plane * esize - spec.nodes * esize < 256
    # a plane of 2^k bytes gets 256 bytes of padding by default (HBM channel spread)
    pow2 = W.cavity(64, 0.05, 1.0, 100.0)
    plane2, _ = clbm.buffer_size(clbm.params_from_spec(pow2, storage, layout="planes"))
    assert plane2 * esize == pow2.nodes * esize + 256
    plane3, _ = clbm.buffer_size(clbm.params_from_spec(pow2, storage, plane_pad=0, layout="planes"))
    assert plane3 == pow2.nodes
    assert nbytes == 19 * plane * esize
    # row layout: populations a and a + 1 of a node are nx apart, no padding
    stride, rbytes = clbm.buffer_size(clbm.params_from_spec(spec, storage, layout="rows"))
    assert stride == spec.nx and rbytes == 19 * spec.nodes * esize


@pytest.mark.parametrize("field,value", [
    ("nx", 0), ("K", 0.0), ("K", float("nan")), ("n", -1.0), ("nu_min", 0.0), ("nu_max", 1e-6),
    ("omega_bulk", 2.0), ("rho_wall", 0.0), ("storage", 7), ("lid_face", 9), ("attractor_literal", 2),
    ("collision", 4), ("plane_pad", -2), ("layout", 2), ("layout", -1), ("f16_rounding", 2),
])
def test_invalid_parameters_rejected(clbm, field, value):
    p = clbm.params_from_spec(W.cavity(8, 0.05, 1.0, 10.0), "f32")
    setattr(p, field, value)
    with pytest.raises(clbm.ClbmError) as ei:
        clbm.buffer_size(p)
    assert ei.value.status == clbm.CLBM_EINVAL


def test_lid_on_periodic_axis_rejected(clbm):
    spec = W.cavity(8, 0.05, 1.0, 10.0).with_(periodic=(0, 1, 0))
    with pytest.raises(clbm.ClbmError):
        clbm.buffer_size(clbm.params_from_spec(spec, "f32"))


def test_create_rejects_bad_buffers(clbm):
    p = clbm.params_from_spec(W.cavity(8, 0.05, 1.0, 10.0), "f32")
    h = ctypes.c_void_p()
    lib = clbm.load()
    assert lib.clbm_create(ctypes.byref(p), None, None, 0, None, ctypes.byref(h)) == clbm.CLBM_EINVAL
    # misaligned pointers are refused before any device call
    assert lib.clbm_create(ctypes.byref(p), ctypes.c_void_p(0x1004), ctypes.c_void_p(0x2000), 1 << 30,
                           None, ctypes.byref(h)) == clbm.CLBM_EINVAL
    assert "aligned" in lib.clbm_last_error().decode()
    # too small
    assert lib.clbm_create(ctypes.byref(p), ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), 16,
                           None, ctypes.byref(h)) == clbm.CLBM_EINVAL


def test_batch_size_validates_each_instance(clbm):
    specs = [W.cavity(8, 0.05, 1.0, 10.0), W.cavity(12, 0.05, 0.7, 10.0)]
    arr = (clbm.Params * 2)()
    for i, sp in enumerate(specs):
        arr[i] = clbm.params_from_spec(sp, "f32", layout="planes")
    n = ctypes.c_size_t()
    assert clbm.load().clbm_batch_size(arr, 2, ctypes.byref(n)) == 0
    assert n.value == sum(clbm.buffer_size(arr[i])[1] for i in range(2))
    arr[1].storage = 0
    assert clbm.load().clbm_batch_size(arr, 2, ctypes.byref(n)) == clbm.CLBM_EINVAL
    assert "instance 1" in clbm.load().clbm_last_error().decode()
    arr[1] = clbm.params_from_spec(specs[1], "f32", layout="rows")
    assert clbm.load().clbm_batch_size(arr, 2, ctypes.byref(n)) == clbm.CLBM_EINVAL
    assert "layout differs" in clbm.load().clbm_last_error().decode()
    # all in the row layout: each instance rounded up to 256 bytes
    rows = (clbm.Params * 2)()
    for i, sp in enumerate(specs):
        rows[i] = clbm.params_from_spec(sp, "f32", layout="rows")
    assert clbm.load().clbm_batch_size(rows, 2, ctypes.byref(n)) == 0
    assert n.value == sum((clbm.buffer_size(rows[i])[1] + 255) // 256 * 256 for i in range(2))
    arr[1] = clbm.params_from_spec(specs[1], "f32", layout="planes")
    arr[1].K = -1.0
    assert clbm.load().clbm_batch_size(arr, 2, ctypes.byref(n)) == clbm.CLBM_EINVAL
    assert clbm.load().clbm_batch_size(arr, 0, ctypes.byref(n)) == clbm.CLBM_EINVAL


def test_srt_model_restrictions(clbm):
    """The single-relaxation-time comparison model is unforced and is not
    offered in batches."""
    spec = W.poiseuille(4, 8, 4, n=1.0, Re=5.0, umax=0.01).with_(model="srt")
    with pytest.raises(clbm.ClbmError):
        clbm.buffer_size(clbm.params_from_spec(spec, "f32"))
    cav = W.cavity(8, 0.05, 1.0, 10.0).with_(model="srt")
    p = clbm.params_from_spec(cav, "f32")
    assert p.collision == clbm.COLLISION["srt"]
    clbm.buffer_size(p)
    arr = (clbm.Params * 1)()
    arr[0] = p
    n = ctypes.c_size_t()
    assert clbm.load().clbm_batch_size(arr, 1, ctypes.byref(n)) == clbm.CLBM_EINVAL


@pytest.mark.parametrize("layout", ["rows", "planes"])
def test_in_place_create_checks_buffer_first(clbm, layout):
    """The one-buffer form takes either layout; a misaligned buffer is refused
    before any device call."""
    lib = clbm.load()
    h = ctypes.c_void_p()
    p = clbm.params_from_spec(W.cavity(8, 0.05, 1.0, 10.0), "f32", layout=layout)
    assert lib.clbm_create_in_place(ctypes.byref(p), ctypes.c_void_p(0x1004), ctypes.c_size_t(1 << 30),
                                    ctypes.byref(h)) == clbm.CLBM_EINVAL
    assert "aligned" in lib.clbm_last_error().decode()


def test_size_limits_per_layout(clbm):
    """Planes: one plane must fit the 4 GiB range of a buffer descriptor.
    Rows: no plane limit, node indices are 32-bit (fewer than 2^31 nodes)."""
    big = W.cavity(16, 0.05, 0.8, 100.0).with_(nx=1024, ny=1024, nz=1024)
    with pytest.raises(clbm.ClbmError):
        clbm.buffer_size(clbm.params_from_spec(big, "f32", layout="planes"))
    stride, nbytes = clbm.buffer_size(clbm.params_from_spec(big, "f32", layout="rows"))
    assert stride == 1024 and nbytes == 19 * 4 * 1024 ** 3
    too_many = big.with_(nx=2048)
    with pytest.raises(clbm.ClbmError):
        clbm.buffer_size(clbm.params_from_spec(too_many, "f16", layout="rows"))
    clbm.buffer_size(clbm.params_from_spec(too_many.with_(nz=1023), "f16", layout="rows"))
    # rows: a wave's descriptors span up to 20 runs of nx + 64 values, within a 2 GiB byte range
    long_row = big.with_(nx=1 << 24, ny=1, nz=1)
    with pytest.raises(clbm.ClbmError):
        clbm.buffer_size(clbm.params_from_spec(long_row, "f64", layout="rows"))
    clbm.buffer_size(clbm.params_from_spec(long_row, "f16", layout="rows"))
    clbm.buffer_size(clbm.params_from_spec(long_row, "f64", layout="planes"))
