"""bench.py's output contract and its ties to the committed profiles (CPU only).

The benchmark itself needs a GPU; these checks cover what it computes on the
host: the roofline object, the launch forms it times, the refusal of more
than one GPU, and that every committed profile summary was taken on the
current kernel sources (otherwise the benchmark reports no traffic)."""
import glob
import json
import os
import re
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WORKLOAD = "cavity512_re3200_n0.75"


def test_roofline_object():
    n = 512 ** 3
    for storage, spl, layout in (("f32", 2, "rows"), ("f16", 1, "rows"), ("f64", 1, "rows")):
        r = bench.roofline(storage, n, 3.0, WORKLOAD, spl, layout)
        for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
            assert k in r
        assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
        assert abs(r["achieved"] - bench.BYTES_PER_LUP[storage] * n / 3e-3 / 1e9) < 0.1
        assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-4
        assert r["kernel"] == ("stream_collide2" if spl == 2 else "stream_collide_rows")


def test_launch_forms():
    spec_nz = type("S", (), {"nz": 512})()
    for storage, form in bench.BEST_FORM.items():
        c = bench.launch_of(form, storage, spec_nz)
        if form == "two":
            assert c["fuse_steps"] == 2
            assert c["fuse_rows"] in ((8,) if storage == "f64" else (8, 12, 16))
            assert c["xcd_remap"] in (0, 1) and c["nt_stores"] in (0, 1) and c["fuse_planes"] >= 1
            assert bench.TWO_STEP_LAYOUT[storage] in ("rows", "planes")
        else:
            assert c is None
    short = type("S", (), {"nz": 5})()
    assert bench.launch_of("two", "f32", short)["fuse_planes"] == 5


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "error" in line and line["n_gpus"] == 2


def test_traffic_comes_only_from_profiles_of_the_current_kernels(tmp_path, monkeypatch):
    """Every committed counter summary names the kernel-source hash it was
    taken on; the benchmark takes measured traffic from a summary only when
    that hash is the hash of the current sources (else it reports null)."""
    files = glob.glob(os.path.join(ROOT, "profiles", "*_traffic.md"))
    assert files
    for path in files:
        assert re.search(r"kernel_source_hash:\s*[0-9a-f]{16}", open(path).read()), path
    h = bench.kernel_source_hash()
    monkeypatch.setattr(bench, "PROFILE_DIR", str(tmp_path))
    for tag, want in ((h, 1.5e10), ("0" * 16, None)):
        (tmp_path / f"stream_collide2_{WORKLOAD}_f32_traffic.md").write_text(
            f"kernel_source_hash: {tag}\nhbm_bytes_per_launch: 1.5e10\n")
        assert bench.measured_traffic("f32", WORKLOAD, "stream_collide2") == want
