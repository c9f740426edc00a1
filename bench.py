#!/usr/bin/env python3
"""Throughput benchmark of the D3Q19 cascaded power-law stream-collide step.

Workload (default): lid-driven cubic cavity 512^3 (134.2 M nodes), Re = 3200,
n = 0.75, lid velocity 0.04, rest start; FP32 storage of f - w with FP32
arithmetic; the FP64 mass reduction every 100 steps tracks the mass drift.
Every timed run starts from rest and first takes --spinup untimed steps (1000
by default), which set the whole cavity moving: from rest most nodes have no
shear and skip the relaxation-rate solve, so steps timed near rest would be
faster than the developed flow of the 5000-step run.  The first --rest-steps
of the main run's spin-up are timed on their own and reported as a secondary
figure.  Each storage type runs in its faster launch form: FP32 two steps per
launch (temporal blocking in the row-interleaved layout; one launch = two
full steps of the fused pull stream-collide), FP16 deviations (stochastic rounding) and FP64
one step per launch in the row-interleaved layout (a launch for the rows off
the y and z faces and one for the face rows).  All storage types run the same
spin-up, warm-up and timed steps, and the errors of FP32 and FP16 against FP64
are reported on the centrelines u_x(y), u_y(x) and normwise over the whole
field.

Prints ONE JSON line: MLUPS of the timed region (exactly --steps steps after
the spin-up and --warmup untimed ones, bracketed by device synchronisation),
the roofline of the stream-collide kernel (algorithmic bytes of the steps a
launch advances / average launch time measured with events on the launch
stream, with the measured HBM traffic of the committed counter summary
beside it), the other launch form and the planes layout of each storage
type, the FP16-deviation and FP64 storage variants of the same workload, the
64-cavity batch (one graph-replayed launch per step vs one launch per
instance, with its roofline), the achievable copy bandwidth, and the CPU
oracle timed on the host cores on a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, published
BYTES_PER_LUP = {"f64": 304, "f32": 152, "f16": 76}   # 19 reads + 19 writes per node update
PROFILE_DIR = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1908_05396_amd", "csrc", f)
                  for f in ("clbm_device.hpp", "clbm_internal.hpp", "clbm_rows.hpp", "clbm_kernels.hip",
                            "clbm_rows.hip", "clbm_fused.hip", "clbm_batch.hip")]
# the one-step kernel of each state layout
STEP_KERNEL = {"rows": "stream_collide_rows", "planes": "stream_collide"}


def kernel_source_hash() -> str:
    """Hash of the step kernels' code: the sources with comments and blank
    lines removed, so that a profile stays valid across comment edits."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        code = "\n".join(line.rstrip() for line in text.splitlines() if line.strip())
        h.update(code.encode())
    return h.hexdigest()[:16]


def measured_traffic(storage: str, workload: str, kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this kernel and workload, or None if absent or taken on other sources."""
    path = os.path.join(PROFILE_DIR, f"{kernel}_{workload}_{storage}_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"kernel_source_hash:\s*([0-9a-f]+)", text)
    m_bytes = re.search(r"hbm_bytes_per_(?:launch|step):\s*([0-9.eE+]+)", text)
    if not m_hash or not m_bytes or m_hash.group(1) != kernel_source_hash():
        return None
    return float(m_bytes.group(1))


def centrelines(u, L):
    """u_x(y) on x = H/2 and u_y(x) on y = H/2, both in the plane z = H/2; for
    an even edge length the two middle node columns (planes) are averaged."""
    c0, c1 = L // 2 - 1, L // 2
    mid = (u[:, c0] + u[:, c1]) / 2                     # (3, y, x) at z = H/2
    ux_y = (mid[0, :, c0] + mid[0, :, c1]) / 2
    uy_x = (mid[1, c0, :] + mid[1, c1, :]) / 2
    return ux_y, uy_x


def accuracy_vs(torch, runs, ref_key, U, L):
    """Errors of each run's velocity field against the reference run's:
    centreline max |du| / U and the normwise max |du| / max |u_ref|."""
    ref = runs[ref_key]
    rx, ry = centrelines(ref, L)
    out = {"reference": f"{ref_key} storage on the GPU, same workload and step count"}
    for key, u in runs.items():
        if key == ref_key:
            continue
        ax, ay = centrelines(u, L)
        cl = max((ax - rx).abs().max().item(), (ay - ry).abs().max().item()) / U
        out[key] = {"centreline_max_abs_over_U": float(f"{cl:.3e}"),
                    "field_normwise": float(f"{((u - ref).abs().max() / ref.abs().max()).item():.3e}")}
    return out


# Two steps per launch for each storage type: the fastest layout, patch
# height, z chunk, tile order and store hint of a sweep at 512^3 (rows
# 8/12/16 x planes 4..48 x both orders x both hints x both layouts).  FP32 in
# the row layout with 16-plane chunks: 3.156 ms per step against 3.238 in the
# planes layout with 32-plane chunks, the better one there.
TWO_STEP = {"f32": {"fuse_steps": 2, "fuse_rows": 16, "fuse_planes": 16, "xcd_remap": 1, "nt_stores": 0},
            "f16": {"fuse_steps": 2, "fuse_rows": 16, "fuse_planes": 16, "xcd_remap": 1, "nt_stores": 0},
            "f64": {"fuse_steps": 2, "fuse_rows": 8, "fuse_planes": 32, "xcd_remap": 0, "nt_stores": 1}}
TWO_STEP_LAYOUT = {"f32": "rows", "f16": "planes", "f64": "planes"}
# The faster form per storage type at 512^3: FP32 two steps per launch (it
# moves about 0.6 of the bytes of two one-step launches); FP16 storage, bound
# by its arithmetic, and FP64 one step per launch in the row layout.
BEST_FORM = {"f32": "two", "f16": "one", "f64": "one"}


def launch_of(form, storage, spec):
    """Launch dict of a form ("one": library default, "two": TWO_STEP)."""
    if form != "two":
        return None
    c = dict(TWO_STEP[storage])
    c["fuse_planes"] = min(spec.nz, c["fuse_planes"])
    return c


def time_lattice(clbm, torch, spec, storage, steps, warmup, reduce_every, block=None, keep_u=False, launch=None,
                 in_place=False, layout=None, spinup=0, rest_steps=0):
    """Rest start, then `spinup` untimed steps (the first `rest_steps` of them
    timed on their own: the near-rest transient), `warmup` untimed steps, and
    `steps` timed steps; returns timing and reduction results (and the final
    velocity field, FP64 on the device, if `keep_u`).  `launch`: a launch
    dict or None (the library default)."""
    lat = clbm.Lattice(spec, storage=storage, track_residual=False, block=block, in_place=in_place, launch=launch,
                       layout=layout)
    lat.init_rest()
    r0 = lat.reduce()
    stream = torch.cuda.current_stream()
    rest_ms = None
    if rest_steps > 0:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        lat.step(rest_steps)
        e1.record(stream)
        torch.cuda.synchronize()
        rest_ms = e0.elapsed_time(e1) / rest_steps
    lat.step(max(spinup - rest_steps, 0) + warmup)
    torch.cuda.synchronize()
    starts, ends = [], []
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        chunk = min(reduce_every, steps - done)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        lat.step(chunk)
        e1.record(stream)
        starts.append((e0, chunk))
        ends.append(e1)
        done += chunk
        if done < steps or done % reduce_every == 0:
            lat.reduce()          # FP64 mass/NaN check every `reduce_every` steps (synchronizes)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = sum(e0.elapsed_time(e1) for (e0, _), e1 in zip(starts, ends))
    r1 = lat.reduce()
    out = {
        "wall_s": wall,
        "ms_per_step": wall * 1e3 / steps,
        "kernel_ms_per_step": kernel_ms / steps,
        "rest_kernel_ms_per_step": rest_ms,
        "mass_drift": (r1["mass"] - r0["mass"]) / r0["mass"],
        "umax": r1["umax"],
        "nonfinite": r1["nonfinite"],
        "block": list(lat.get_block()),
        "launch": lat.get_launch(),
        "layout": lat.layout,
    }
    if keep_u:
        out["u"] = lat.macroscopic()[1]
    lat.close()
    del lat
    torch.cuda.empty_cache()
    return out


def roofline(storage, nodes, kernel_ms_per_step, workload, steps_per_launch, layout, kernel=None):
    """HBM roofline of the stream-collide kernel: `achieved` is the
    algorithmic bytes of one launch (19 reads + 19 writes per node and step,
    times the steps one launch advances) over the launch's average duration;
    `traffic` is the measured HBM bytes per launch from the committed counter
    summary (null if absent or taken on other kernel sources), and
    `hbm_gbs_measured` those bytes over the same duration."""
    launch_ms = kernel_ms_per_step * steps_per_launch
    achieved = BYTES_PER_LUP[storage] * nodes / (kernel_ms_per_step * 1e-3) / 1e9
    if kernel is None:
        kernel = STEP_KERNEL[layout] if steps_per_launch == 1 else "stream_collide2"
    traffic = measured_traffic(storage, workload, kernel)
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernel,
           "achieved_is": "algorithmic bytes per launch / launch time",
           "bytes_per_lup": BYTES_PER_LUP[storage], "steps_per_launch": steps_per_launch,
           "kernel_ms_per_launch": round(launch_ms, 4)}
    if traffic is not None:
        # measured HBM bytes over the algorithmic bytes of one launch (below 1: temporal blocking)
        out["traffic_over_algorithmic"] = round(traffic / (BYTES_PER_LUP[storage] * nodes * steps_per_launch), 3)
        out["hbm_gbs_measured"] = round(traffic / (launch_ms * 1e-3) / 1e9, 1)
    return out


BATCH_WORKLOAD = "batch64_cavities_L32-96_n0.4-1.6_re50-1000"


def batched(clbm, torch, W, storage, steps, spinup, tune=True):
    """The 64-cavity batch: one launch per step for all instances (graph-replayed,
    autotuned after an untimed spin-up from rest) against one launch per
    instance per step, both timed with events on the launch stream over
    `steps` steps; the roofline of the batch kernel in algorithmic bytes
    per node update."""
    specs = W.config_batch()
    nodes = sum(s.nodes for s in specs)
    b = clbm.Batch(specs, storage=storage)
    b.init_rest()
    b.step(spinup)
    cfg = b.autotune()[0] if tune else b.get_config()
    out = {"workload": BATCH_WORKLOAD, "instances": len(specs), "nodes": nodes, "storage": storage,
           "steps": steps, "spinup_steps": spinup, "config": cfg}
    stream = torch.cuda.current_stream()
    ms = {}
    for key, fn in (("mlups", b.step), ("mlups_one_launch_per_instance", b.step_each)):
        fn(10)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        fn(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms[key] = e0.elapsed_time(e1) / steps
        out[key] = round(nodes * steps / (time.perf_counter() - t0) / 1e6, 1)
    out["speedup"] = round(out["mlups"] / out["mlups_one_launch_per_instance"], 3)
    kernel = "batch_packed" if cfg.get("passes", 0) > 0 else "batch_rows"
    out["roofline"] = roofline(storage, nodes, ms["mlups"], BATCH_WORKLOAD, 1, "rows", kernel=kernel)
    r = b.reduce(raise_unstable=False)
    out["nonfinite_instances"] = sum(1 for x in r if x["nonfinite"] > 0)
    b.close()
    del b
    torch.cuda.empty_cache()
    return out


# storage variants of the accuracy runs: (name, storage, FP16 rounding)
ACCURACY_VARIANTS = (("f64", "f64", "stochastic"), ("f32", "f32", "stochastic"), ("f16", "f16", "stochastic"),
                     ("f16_nearest", "f16", "nearest"))


def accuracy_run(clbm, torch, spec, steps, report_every, variants=ACCURACY_VARIANTS):
    """The same cavity from rest for `steps` steps in FP64, FP32 and
    FP16-deviation storage (stochastic and nearest-even rounding); errors of
    each against FP64 on the centrelines and over the whole field."""
    fields, history = {}, {}
    for key, st, rounding in variants:
        lat = clbm.Lattice(spec, storage=st, track_residual=True, f16_rounding=rounding)
        lat.init_rest()
        m0 = lat.reduce()["mass"]
        t0 = time.perf_counter()
        done, hist = 0, []
        while done < steps:
            k = min(report_every, steps - done)
            lat.step(k)
            done += k
            r = lat.reduce(raise_unstable=False)
            hist.append({"step": done, "umax": r["umax"], "residual": r["residual"],
                         "mass_drift": (r["mass"] - m0) / m0, "nonfinite": r["nonfinite"]})
            print(f"[accuracy] {spec.name} {key} step {done}: {time.perf_counter() - t0:.1f} s, "
                  f"residual {r['residual']:.3e}, umax {r['umax']:.5f}", file=sys.stderr, flush=True)
        fields[key] = lat.macroscopic()[1]
        history[key] = hist[-1]
        lat.close()
        del lat
        torch.cuda.empty_cache()
    out = accuracy_vs(torch, fields, "f64", spec.lid_velocity[0], spec.nx)
    out.update({"workload": spec.name, "steps": steps, "final": history})
    return out, fields


def accuracy64(clbm, torch, W, steps=20000):
    """The 64^3 cavity at Re 100 (n = 0.5, 1, 1.5), every storage variant
    against GPU FP64 and, where the stored FP64 oracle results exist, against
    them (the velocity on the mid-planes z = 31, 32 and every fourth node)."""
    import numpy as np
    out = []
    for n in (0.5, 1.0, 1.5):
        spec = W.config_cavity64(n)
        acc, fields = accuracy_run(clbm, torch, spec, steps, 5000)
        path = os.path.join(ROOT, "tests", "golden", f"cavity64_re100_n{n:g}_steps{steps}.npz")
        if os.path.exists(path):
            fx = np.load(path)
            sub = slice(1, 64, 4)
            ref = np.concatenate([fx["u_planes"].ravel(), fx["u_sub"].ravel()])
            vs = {}
            for key, u in fields.items():
                uu = u.cpu().numpy()
                got = np.concatenate([uu[:, [31, 32]].ravel(), uu[:, sub, sub, sub].ravel()])
                vs[key] = float(f"{np.abs(got - ref).max() / np.abs(ref).max():.3e}")
            acc["vs_stored_oracle"] = vs
        out.append(acc)
        print(json.dumps(acc), file=sys.stderr, flush=True)
    return {"workload": "cavity64_re100, n = 0.5, 1, 1.5", "steps": steps, "runs": out}


def stability(clbm, torch, W, steps=50000, check_every=5000):
    """Largest stable lid velocity of the 64^3 cavity (the protocol of Sec. 5:
    mu_p = c_s^2 (tau_p - 1/2), stable = finite with max |u| below 1 after
    `steps` steps) for the cascaded scheme and the BGK comparison model, by
    bisection on U.  The viscosity clip is opened to omega < 2 - 1e-6, as the
    protocol has none."""
    nu_min = (1.0 / (2.0 - 1e-6) - 0.5) / 3.0
    out = []
    for n in (0.8, 1.0, 1.5):
        for tau_p in (0.51, 0.55, 0.6):
            row = {"n": n, "tau_p": tau_p}
            for model in ("cascaded", "srt"):
                lo, hi = 0.0, 0.4
                for _ in range(7):
                    U = 0.5 * (lo + hi)
                    spec = W.LatticeSpec(nx=64, ny=64, nz=64, K=(tau_p - 0.5) / 3.0, n=n, lid_face=W.LID_PY,
                                         lid_velocity=(U, 0.0, 0.0), nu_min=nu_min, model=model)
                    lat = clbm.Lattice(spec, storage="f32", track_residual=False)
                    lat.init_rest()
                    ok, done = True, 0
                    while done < steps:
                        lat.step(check_every)
                        done += check_every
                        r = lat.reduce(raise_unstable=False)
                        if r["nonfinite"] > 0 or not (r["umax"] < 1.0):
                            ok = False
                            break
                    lat.close()
                    lo, hi = (U, hi) if ok else (lo, U)
                row[model + "_max_U"] = round(lo, 4)
                print(f"[stability] n={n} tau_p={tau_p} {model}: max stable U in [{lo:.4f}, {hi:.4f})",
                      file=sys.stderr, flush=True)
            out.append(row)
    return {"workload": "cavity64, FP32, 50000 steps, bisection on U in (0, 0.4)", "rows": out}


def stability_re(clbm, torch, W, steps=50000, check_every=5000, U=0.05, grids=(48, 64, 96, 128), iters=8,
                 re_lo=10.0, re_hi=1.0e5):
    """Largest stable Reynolds number against grid size (the first stability
    protocol of Sec. 5): lid-driven cavity at a fixed lid velocity, the
    consistency coefficient lowered (Re = H^n U^(2-n) / mu_p raised) until
    the run becomes unstable, for the cascaded scheme and the BGK comparison
    model.  Bisection on log Re in [re_lo, re_hi]; a probe is stable when the
    state stays finite with max |u| below 1 for `steps` steps (checked every
    `check_every`, the run stops at the first failure).  The viscosity clip
    is opened to omega < 2 - 1e-6, as the protocol has none."""
    import math
    nu_min = (1.0 / (2.0 - 1e-6) - 0.5) / 3.0
    out = []
    for n in (0.8, 1.0, 1.5):
        for L in grids:
            row = {"n": n, "grid": L}
            for model in ("cascaded", "srt"):
                lo, hi = math.log(re_lo), math.log(re_hi)
                stable_lo = None
                for _ in range(iters):
                    Re = math.exp(0.5 * (lo + hi))
                    spec = W.cavity(L, U, n, Re).with_(nu_min=nu_min, model=model, name=f"stab{L}")
                    lat = clbm.Lattice(spec, storage="f32", track_residual=False)
                    lat.init_rest()
                    ok, done = True, 0
                    while done < steps:
                        lat.step(check_every)
                        done += check_every
                        r = lat.reduce(raise_unstable=False)
                        if r["nonfinite"] > 0 or not (r["umax"] < 1.0):
                            ok = False
                            break
                    lat.close()
                    del lat
                    if ok:
                        lo, stable_lo = math.log(Re), Re
                    else:
                        hi = math.log(Re)
                    print(f"[stability-re] n={n} L={L} {model}: Re {Re:.1f} {'stable' if ok else 'unstable'} "
                          f"({done} steps)", file=sys.stderr, flush=True)
                row[model + "_max_Re"] = round(math.exp(lo), 1) if stable_lo is not None else None
                row[model + "_unstable_Re"] = round(math.exp(hi), 1)
            out.append(row)
            torch.cuda.empty_cache()
    return {"workload": f"lid-driven cavity, U = {U}, FP32, {steps} steps per probe, bisection on log Re in "
                        f"[{re_lo:g}, {re_hi:g}] ({iters} probes), clip omega < 2 - 1e-6",
            "rows": out}


def copy_bandwidth(clbm, torch, nbytes=4 << 30, reps=10):
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    clbm.copy_probe(a, b)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        clbm.copy_probe(a, b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def cpu_baseline(spec_full, min_seconds=10.0, max_seconds=30.0):
    """The FP64 oracle on the host cores, on a 64^3 cavity with the same
    power-law parameters (K, n, lid velocity) as the full workload, stepped
    until at least `min_seconds` have elapsed."""
    import numpy as np

    import oracle
    import workloads as W
    threads = oracle.set_threads(len(os.sched_getaffinity(0)))
    sub = spec_full.with_(nx=64, ny=64, nz=64, name="cpu_sample")
    f = W.rest_populations(sub).numpy()
    steps = 0
    t0 = time.perf_counter()
    while True:
        f = oracle.run(sub, f, 2)
        steps += 2
        el = time.perf_counter() - t0
        if el >= min_seconds or el >= max_seconds:
            break
    mlups = sub.nodes * steps / el / 1e6
    assert np.isfinite(f).all()
    return {"value": round(mlups, 4), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle, 64^3 cavity with the workload's K, n and lid velocity, "
                      f"{steps} steps from rest, {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--size", type=int, default=512, help="cavity edge length")
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "f64"])
    ap.add_argument("--layout", default="rows", choices=["rows", "planes"],
                    help="state layout of the one-step runs")
    ap.add_argument("--form", default="best", choices=["best", "one", "two"],
                    help="launch form of the main run and the storage variants: the faster one per storage type "
                         "(FP32 two steps per launch, FP16 and FP64 one), or one / two steps per launch for all")
    ap.add_argument("--reduce-every", type=int, default=100)
    ap.add_argument("--spinup", type=int, default=1000,
                    help="untimed steps from rest before the warm-up of every timed run: the lid sets the whole "
                         "cavity moving, so the timed steps see the developed flow (from rest most nodes have no "
                         "shear and skip the relaxation-rate solve)")
    ap.add_argument("--rest-steps", type=int, default=100,
                    help="the first steps of the main run's spin-up, timed on their own (secondary figure)")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-copy", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other launch form, the planes layout, the BGK comparison and the one-buffer "
                         "form (short runs under a profiler)")
    ap.add_argument("--batch-steps", type=int, default=10000)
    ap.add_argument("--batch-only", action="store_true",
                    help="only the 64-cavity batch (its own JSON line; for profiling the batch kernel)")
    ap.add_argument("--batch-no-tune", action="store_true",
                    help="time the batch in its default launch configuration (no autotuner trials)")
    ap.add_argument("--stability", action="store_true",
                    help="instead of the benchmark: largest stable lid velocity of the 64^3 cavity, cascaded "
                         "scheme vs the single-relaxation-time comparison model")
    ap.add_argument("--stability-re", action="store_true",
                    help="instead of the benchmark: largest stable Re against grid size (48^3 .. 128^3), cascaded "
                         "scheme vs the single-relaxation-time comparison model")
    ap.add_argument("--accuracy256", type=int, default=0, metavar="STEPS",
                    help="instead of the benchmark: run the 256^3 cavity (Re 1000, n 0.5) for STEPS steps in "
                         "FP64, FP32 and FP16-deviation storage and print the centreline errors vs FP64")
    ap.add_argument("--accuracy64", type=int, default=0, metavar="STEPS",
                    help="instead of the benchmark: the 64^3 cavity (Re 100, n = 0.5, 1, 1.5) for STEPS steps in "
                         "every storage variant, errors vs GPU FP64 and vs the stored oracle results")
    ap.add_argument("--accuracy512", type=int, default=0, metavar="STEPS",
                    help="instead of the benchmark: the 512^3 cavity for STEPS steps in every storage variant")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the method's "
                                   "multi-GPU decomposition (z slabs with ghost planes) is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    import workloads as W
    from paper_1908_05396_amd import clbm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.stability:
        print(json.dumps(stability(clbm, torch, W)), flush=True)
        return
    if args.stability_re:
        print(json.dumps(stability_re(clbm, torch, W)), flush=True)
        return
    if args.accuracy256:
        print(json.dumps(accuracy_run(clbm, torch, W.config_cavity256(), args.accuracy256, 5000)[0]), flush=True)
        return
    if args.accuracy64:
        print(json.dumps(accuracy64(clbm, torch, W, args.accuracy64)), flush=True)
        return
    if args.batch_only:
        out = batched(clbm, torch, W, "f32", args.batch_steps, args.spinup, not args.batch_no_tune)
        if not args.no_copy:
            out["copy_gbs"] = copy_bandwidth(clbm, torch)     # the counters' calibration in the same run
        print(json.dumps(out), flush=True)
        return
    if args.accuracy512:
        print(json.dumps(accuracy_run(clbm, torch, W.config_cavity512(), args.accuracy512, 1000)[0]), flush=True)
        return
    spec = W.config_cavity512() if args.size == 512 else \
        W.cavity(args.size, 0.04, 0.75, 3200.0, name=f"cavity{args.size}_re3200_n0.75")
    workload = spec.name
    spin = args.spinup
    compare = not args.no_variants

    def form_of(st):
        return BEST_FORM[st] if args.form == "best" else args.form

    def run_form(st, form, steps, warmup, keep_u=False, rest_steps=0):
        launch = launch_of(form, st, spec)
        return time_lattice(clbm, torch, spec, st, steps, warmup, args.reduce_every, keep_u=keep_u, launch=launch,
                            layout=TWO_STEP_LAYOUT[st] if launch else args.layout, spinup=spin,
                            rest_steps=rest_steps)

    def frac_of(st, ms):
        return round(BYTES_PER_LUP[st] * spec.nodes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)

    rest_steps = min(args.rest_steps, spin)
    main_run = run_form(args.storage, form_of(args.storage), args.steps, args.warmup, keep_u=compare,
                        rest_steps=rest_steps)
    mlups = spec.nodes * args.steps / (main_run["ms_per_step"] * args.steps * 1e-3) / 1e6
    print(f"[bench] main run {args.storage}: {main_run['kernel_ms_per_step']:.4f} ms/step in the developed flow",
          file=sys.stderr, flush=True)

    # every storage runs the same spin-up, warm-up and timed steps, so all end at the same step
    variants = {}
    fields = {args.storage: main_run.pop("u", None)}
    if not args.no_variants:
        for st in ("f16", "f64", "f32"):
            if st == args.storage:
                continue
            r = run_form(st, form_of(st), args.steps, args.warmup, keep_u=compare)
            fields[st] = r.pop("u", None)
            spl = r["launch"]["fuse_steps"]
            variants[st] = {
                "mlups": round(spec.nodes / (r["ms_per_step"] * 1e-3) / 1e6, 1),
                "roofline": roofline(st, spec.nodes, r["kernel_ms_per_step"], workload, spl, r["layout"]),
                "kernel_ms_per_launch": round(r["kernel_ms_per_step"] * spl, 4),
                "steps_per_launch": spl,
                "mass_drift": r["mass_drift"], "steps": args.steps,
            }
            print(f"[bench] variant {st}: {r['kernel_ms_per_step']:.4f} ms/step", file=sys.stderr, flush=True)
    # the other launch form of each storage (one vs two steps per launch), after the same spin-up
    launch_forms = {}
    if not (args.no_variants or args.no_extras):
        for st in ("f32", "f64", "f16"):
            r = run_form(st, "one" if form_of(st) == "two" else "two", 300, 20)
            launch_forms[st] = {
                "launch": r["launch"], "layout": r["layout"],
                "mlups": round(spec.nodes / (r["ms_per_step"] * 1e-3) / 1e6, 1),
                "kernel_ms_per_step": round(r["kernel_ms_per_step"], 4),
                "roofline_frac": frac_of(st, r["kernel_ms_per_step"])}

    # the planes layout, one step per launch, for each storage
    planes_layout = {}
    if not (args.no_variants or args.no_extras):
        for st in ("f32", "f16", "f64"):
            r = time_lattice(clbm, torch, spec, st, 300, 20, args.reduce_every, layout="planes", spinup=spin)
            planes_layout[st] = {
                "mlups": round(spec.nodes / (r["ms_per_step"] * 1e-3) / 1e6, 1),
                "kernel_ms_per_step": round(r["kernel_ms_per_step"], 4),
                "roofline_frac": frac_of(st, r["kernel_ms_per_step"])}

    # the library's autotuner on the same workload (FP32, row layout, after the spin-up)
    autotuned = None
    if not (args.no_variants or args.no_extras):
        lat = clbm.Lattice(spec, storage="f32", track_residual=False)
        lat.init_rest()
        lat.step(spin)
        default = lat.get_launch()
        cfg, ms = lat.autotune()
        autotuned = {"storage": "f32", "default_launch": default, "best_launch": cfg,
                     "best_ms_per_step": round(ms, 4), "roofline_frac": frac_of("f32", ms)}
        lat.close()
        del lat
        torch.cuda.empty_cache()

    # the single-relaxation-time comparison model on the same workload (FP32)
    comparison = None
    if not (args.no_variants or args.no_extras):
        r = time_lattice(clbm, torch, spec.with_(model="srt"), "f32", 300, 20, args.reduce_every, spinup=spin)
        comparison = {"model": "single-relaxation-time (BGK), same power law, FP32, 300 steps after the spin-up",
                      "mlups": round(spec.nodes / (r["ms_per_step"] * 1e-3) / 1e6, 1),
                      "kernel_ms_per_step": round(r["kernel_ms_per_step"], 4),
                      "roofline_frac": frac_of("f32", r["kernel_ms_per_step"])}

    # one state buffer, stepped in place (AA pattern), FP32
    in_place = None
    if not (args.no_variants or args.no_extras):
        r = time_lattice(clbm, torch, spec, "f32", 300, 20, args.reduce_every, in_place=True, spinup=spin)
        in_place = {"storage": "f32", "steps": 300, "mlups": round(spec.nodes / (r["ms_per_step"] * 1e-3) / 1e6, 1),
                    "kernel_ms_per_step": round(r["kernel_ms_per_step"], 4),
                    "roofline_frac": frac_of("f32", r["kernel_ms_per_step"]),
                    "state_bytes": 1 * 19 * spec.nodes * 4}

    accuracy = None
    if compare:
        accuracy = accuracy_vs(torch, fields, "f64", spec.lid_velocity[0], args.size)
        accuracy["steps"] = spin + args.warmup + args.steps
        accuracy["f16_rounding"] = "stochastic"
    del fields
    torch.cuda.empty_cache()

    line = {
        "metric": "MLUPS & %HBM roofline, D3Q19 cascaded power-law; FP32/FP16-store vs FP64",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_run["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage != "f64" else "f64",
        "data": "synthetic",
        "config": {"workload": workload, "nodes": spec.nodes, "storage": args.storage,
                   "lid_velocity": spec.lid_velocity[0], "Re": 3200.0, "n": spec.n, "K": spec.K,
                   "init": "rest", "spinup_steps": spin,
                   "timed": f"{args.steps} steps after {spin} untimed spin-up steps from rest (the whole cavity "
                            f"moving) and {args.warmup} warm-up steps",
                   "reduce_every": args.reduce_every, "layout": main_run["layout"],
                   "launch": main_run["launch"]},
        "roofline": roofline(args.storage, spec.nodes, main_run["kernel_ms_per_step"], workload,
                             main_run["launch"]["fuse_steps"], main_run["layout"]),
        "kernel_ms_per_launch": round(main_run["kernel_ms_per_step"] * main_run["launch"]["fuse_steps"], 4),
        "rest_start": None if main_run["rest_kernel_ms_per_step"] is None else {
            "steps": rest_steps, "kernel_ms_per_step": round(main_run["rest_kernel_ms_per_step"], 4),
            "roofline_frac": frac_of(args.storage, main_run["rest_kernel_ms_per_step"]),
            "note": "the first steps from rest, most of the cavity still at rest (secondary figure)"},
        "mass_drift": main_run["mass_drift"],
        "variants": variants,
        "other_launch_form": launch_forms,
        "planes_layout": planes_layout,
        "autotune": autotuned,
        "srt_comparison": comparison,
        "in_place": in_place,
        "accuracy": accuracy,
    }
    if not args.no_batch:
        line["batched"] = batched(clbm, torch, W, "f32", args.batch_steps, spin, not args.batch_no_tune)
    if not args.no_copy:
        line["copy_gbs"] = round(copy_bandwidth(clbm, torch), 1)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(spec)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
