"""Throughput of the fused central-moment stream-and-collide step on one GPU.

Workload: coupled D2Q9 flow (f) + heat (h) lattices on a 2048 x 2048 grid in
FP32 storage, in-place (AA) streaming by default: heated cylinder of radius 64 (IBB for
f, IABB for h), equilibrium inlet column with a seeded perturbation of the
inlet velocity, zero-gradient outlet column, periodic in y; Re = 100 (u = 0.04,
D = 128, nu = 0.0512), Pr = 0.71.  Synthetic inputs, all resident in HBM before
the timed region.

Prints one JSON line: MLUPS (nodes x steps / s / 1e6) of the whole job, the HBM
roofline of the step kernel (one launch per step) from HIP events around the
timed region, and the FP64 CPU oracle timed on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import ctypes as C
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12  # MI355X HBM3E, B/s
METRIC = "MLUPS + % HBM roofline (fwd CM stream-collide); adjoint/forward step-time ratio"


def source_digest() -> str:
    """Digest of the kernel sources and build script with comments and blank
    lines removed, so that it changes with the code only."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2203_01316_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp")) or name == "build.py":
            with open(os.path.join(csrc, name), encoding="utf-8") as fh:
                text = fh.read()
            if name.endswith((".hip", ".hpp")):
                text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
                text = re.sub(r"//[^\n]*", "", text)
            else:
                text = re.sub(r"#[^\n]*", "", text)
            lines = [ln.rstrip() for ln in text.splitlines() if ln.strip()]
            h.update(name.encode() + b"\0" + "\n".join(lines).encode())
    return h.hexdigest()[:16]


MALL_BYTES = 256 * 2**20  # MI355X Infinity Cache


def cache_note(stream: str, bytes_per_step: int) -> str:
    """Whether the step's population set can sit partly in the Infinity Cache.
    The in-place layout keeps one copy (half the bytes moved per step); on
    MI355X it measured 79-85% of the roofline while that copy fits in about
    300 MB and 70-72% above, while the two-array layout stayed at 76-78%."""
    copy = bytes_per_step // 2
    if stream == "aa" and copy <= 1.25 * MALL_BYTES:
        return (f"one population set of {copy / 1e6:.0f} MB, partly resident in the {MALL_BYTES >> 20} MB "
                "Infinity Cache between steps: the rate is partly cache-assisted")
    copies = "one population set" if stream == "aa" else "two population sets"
    return f"{copies} of {copy / 1e6:.0f} MB"


def read_traffic(workload: str):
    """HBM bytes per bulk launch from the committed rocprofv3 counter summary,
    or None if there is none or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_digest") != source_digest():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_ceiling(torch, L, dev, nbytes=2 << 30, reps=20):
    """Practical HBM ceiling: device-to-device copies of 2 GiB (read 2 GiB,
    write 2 GiB: far above the 256 MB Infinity Cache), by torch's copy and by
    the library's streaming copy kernel (lbm_device_copy: 16-byte
    non-temporal loads and stores) in two launch shapes.  GB/s counts the
    bytes read plus the bytes written."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    a.fill_(1.0)
    stream = torch.cuda.current_stream(dev)

    def rate(fn):
        for _ in range(3):
            fn()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return 2 * nbytes / (e0.elapsed_time(e1) / 1e3 / reps)

    out = {"bytes_each_way": nbytes, "torch_copy_GBps": round(rate(lambda: b.copy_(a)) / 1e9, 1)}
    best = None
    hs = C.c_void_p(stream.cuda_stream)
    for blocks in (0, 8192):
        r = rate(lambda: L.device_copy(b, a, blocks, hs))
        if best is None or r > best[0]:
            best = (r, blocks)
    assert torch.equal(a, b)
    out["lbm_copy_GBps"] = round(best[0] / 1e9, 1)
    out["lbm_copy_blocks"] = best[1]
    del a, b
    torch.cuda.empty_cache()
    return out


def time_steps(torch, g, steps, warmup):
    """GPU seconds per step over `steps` back-to-back steps (events on the stream).
    The legs warm up for as many steps as they time: on MI355X the first few
    hundred steps after a lattice is set up run up to 6% slower."""
    g.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    g.step(steps)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / steps


def leg_cylinder(torch, L, W, np, storage, stream, nx, ny, steps, cu_f=False, cu_h=False):
    nu = 0.04 * 128 / 100.0
    flags, q, groups, u, rho0, H0 = W.heated_cylinder(nx, ny, 64, u_in=0.04, amp=1e-3, seed=0)
    uf = np.asarray(u, np.float32)
    g = L.LBM(L.D2Q9, nx, ny, with_ns=True, storage=storage, nu=nu, k=nu / 0.71, flags=flags, q=q,
              groups=groups, rho_ref=1.0, H_ref=10.0, stream=L.STREAM_AA if stream == "aa" else L.STREAM_AB,
              relax_h="1st" if cu_h else "trt", cumulant_f=cu_f, cumulant_h=cu_h)
    g.set_velocity(uf)
    g.init(H0, u=uf.astype(np.float64), rho=rho0)
    sec = time_steps(torch, g, steps, steps)
    bpn = 2 * 2 * 9 * (8 if storage == "fp64" else 2 if storage.startswith("fp16") else 4)
    mlups = nx * ny / sec / 1e6
    del g
    torch.cuda.empty_cache()
    return {"workload": f"d2q9_ns_ade_heated_cylinder_{nx}x{ny}", "storage": storage, "stream": stream.upper(),
            "collision": ("f cumulant" if cu_f else "f CM-NS") + (", h Cumulants-1st" if cu_h else ", h CM-TRT"),
            "MLUPS": round(mlups, 1),
            "bytes_per_node": bpn, "pct_hbm_roofline": round(100 * mlups * 1e6 * bpn / HBM_PEAK, 2),
            "us_per_step": round(sec * 1e6, 2)}


def leg_tgv(torch, L, W, storage, n1, steps, cu=False, stream="ab"):
    rho, u, H = W.taylor_green_3d(n1, 0.04)
    g = L.LBM(L.D3Q27, n1, n1, n1, with_ns=True, storage=storage, nu=0.002, k=0.002,
              relax_h="1st" if cu else "trt", rho_ref=1.0, H_ref=1.0, cumulant_f=cu, cumulant_h=cu,
              stream=L.STREAM_AA if stream == "aa" else L.STREAM_AB)
    g.init(H, u=u, rho=rho)
    del rho, u, H
    sec = time_steps(torch, g, steps, steps)
    red = g.reduce()
    bpn = 2 * 2 * 27 * (2 if storage.startswith("fp16") else 4)
    mlups = n1 ** 3 / sec / 1e6
    out = {"workload": f"d3q27_ns_ade_taylor_green_{n1}^3", "storage": storage, "stream": stream.upper(),
           "collision": "f cumulant, h Cumulants-1st" if cu else "f CM-NS, h CM-TRT",
           "MLUPS": round(mlups, 1),
           "bytes_per_node": bpn, "pct_hbm_roofline": round(100 * mlups * 1e6 * bpn / HBM_PEAK, 2),
           "us_per_step": round(sec * 1e6, 2), "mass": red[0], "energy": red[1]}
    del g
    torch.cuda.empty_cache()
    return out


def leg_adjoint(torch, L, np, n1=512, steps=2000, interval=45):
    """Adjoint/forward step-time ratio: 512^2 advection-diffusion with a source,
    FP32 forward and FP32 adjoint, checkpoints every `interval` steps."""
    from paper_2203_01316_amd.adjoint import source_objective

    n = n1 * n1
    src = 0.01 * np.random.Generator(np.random.PCG64(1)).standard_normal(n)
    target = 1.0 + 0.01 * np.random.Generator(np.random.PCG64(2)).standard_normal(n)
    g = L.LBM(L.D2Q9, n1, n1, storage="fp32", k=0.01, u0=(0.03, 0.0, 0.0), with_source=True)
    H0 = np.ones(n)
    out = {"workload": f"d2q9_ade_source_{n1}x{n1}", "steps": steps, "checkpoint_interval": interval}
    for rec in (False, True):
        q = torch.tensor(src, dtype=torch.float32, device=g.device, requires_grad=True)
        source_objective(q, g, H0, target, 20, interval=5, recompute=rec).backward()  # warm-up
        q = torch.tensor(src, dtype=torch.float32, device=g.device, requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J = source_objective(q, g, H0, target, steps, interval=interval, recompute=rec)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        J.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        key = "with_replay" if rec else "no_replay"
        out[key] = {"forward_us_per_step": round((t1 - t0) / steps * 1e6, 2),
                    "backward_us_per_step": round((t2 - t1) / steps * 1e6, 2),
                    "ratio": round((t2 - t1) / (t1 - t0), 3)}
    # an objective summed over every 10th step: the reverse sweep needs the
    # residual of each observation time, recomputed by replaying the segments
    from paper_2203_01316_amd.adjoint import tracking_objective
    q = torch.tensor(src, dtype=torch.float32, device=g.device, requires_grad=True)
    tracking_objective(q, g, H0, target, 20, 10, interval=5).backward()  # warm-up
    q = torch.tensor(src, dtype=torch.float32, device=g.device, requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = tracking_objective(q, g, H0, target, steps, 10, interval=interval)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    J.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    out["tracking_every_10"] = {"forward_us_per_step": round((t1 - t0) / steps * 1e6, 2),
                                "backward_us_per_step": round((t2 - t1) / steps * 1e6, 2),
                                "ratio": round((t2 - t1) / (t1 - t0), 3)}
    # kernel-only ratio: step kernel vs adjoint kernel, events around each region
    g.set_source(src.astype(np.float32))
    g.init(H0)
    fwd = time_steps(torch, g, steps, 20)
    lam = torch.zeros(9, n, dtype=torch.float32, device=g.device)
    other = torch.empty_like(lam)
    dq = torch.zeros(n, dtype=torch.float64, device=g.device)
    for _ in range(20):
        g.adjoint_step(lam, other, dq)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps // 2):
        g.adjoint_step(lam, other, dq)
        g.adjoint_step(other, lam, dq)
    e1.record()
    torch.cuda.synchronize()
    adj = e0.elapsed_time(e1) / 1e3 / (2 * (steps // 2))
    out["kernels"] = {"forward_us_per_step": round(fwd * 1e6, 2), "adjoint_us_per_step": round(adj * 1e6, 2),
                      "ratio": round(adj / fwd, 3)}
    out["walls"] = leg_adjoint_walls(torch, L, np, n1, steps)
    return out


def leg_adjoint_walls(torch, L, np, n1, steps):
    """Kernel-only adjoint/forward ratio of the same lattice with walls: a
    channel periodic in x with ABB walls, an IABB disc and EQ nodes."""
    from paper_2203_01316_amd import workloads as W

    flags, q, groups, u = W.walled_box(n1, n1, 0.3 * n1, 0.45 * n1, 0.15 * n1)
    n = n1 * n1
    g = L.LBM(L.D2Q9, n1, n1, storage="fp32", k=0.01, with_source=True, u_mode=1, flags=flags, q=q,
              groups=groups)
    g.set_velocity(np.asarray(u, np.float32))
    g.set_source(np.zeros(n, np.float32))
    g.init(np.ones(n))
    fwd = time_steps(torch, g, steps, 20)
    lam = torch.zeros(9, n, dtype=torch.float32, device=g.device)
    other = torch.empty_like(lam)
    dq = torch.zeros(n, dtype=torch.float64, device=g.device)
    for _ in range(20):
        g.adjoint_step(lam, other, dq)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps // 2):
        g.adjoint_step(lam, other, dq)
        g.adjoint_step(other, lam, dq)
    e1.record()
    torch.cuda.synchronize()
    adj = e0.elapsed_time(e1) / 1e3 / (2 * (steps // 2))
    return {"workload": f"d2q9_ade_walled_box_{n1}x{n1}", "forward_us_per_step": round(fwd * 1e6, 2),
            "adjoint_us_per_step": round(adj * 1e6, 2), "ratio": round(adj / fwd, 3)}


def cpu_baseline(inputs, steps, single_thread=True):
    from oracle import oracle as O

    flags, q, groups, u, rho0, H0, nx, ny, nu, k = inputs
    cores = len(os.sched_getaffinity(0))
    O.lib().ora_set_threads(cores)
    sf = O.preset(9, "ns", O.s_main(nu))
    sh = O.preset(9, "trt", O.s_main(k))
    o = O.Sim(9, nx, ny, with_ns=True, s_f=sf, s_h=sh, uvel=u, flags=flags, qlink=q, groups=groups, s_bulk_f=1.0)
    o.init(H0, u=u, rho=rho0)
    t0 = time.perf_counter()
    o.step(steps)
    sec = time.perf_counter() - t0
    out = {"value": nx * ny * steps / sec / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
           "sample": f"{steps} steps of the same {nx}x{ny} coupled workload, FP64 oracle ({sec:.1f} s)"}
    if single_thread:
        # one more step on one thread (the OpenMP node loop is the only parallelism)
        O.lib().ora_set_threads(1)
        t0 = time.perf_counter()
        o.step(1)
        sec1 = time.perf_counter() - t0
        O.lib().ora_set_threads(cores)
        out["single_thread_value"] = nx * ny / sec1 / 1e6
        out["single_thread_sample"] = f"1 step of the same workload on 1 thread ({sec1:.1f} s)"
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--nx", type=int, default=2048)
    ap.add_argument("--ny", type=int, default=2048)
    ap.add_argument("--storage", default="fp32")
    ap.add_argument("--stream", default="aa", choices=["aa", "ab"],
                    help="population layout: in place (aa, measured faster for D2Q9 FP32) or two arrays (ab)")
    ap.add_argument("--cpu-steps", type=int, default=40)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-cpu-single", action="store_true", help="skip the single-thread oracle step")
    ap.add_argument("--no-extra", action="store_true", help="skip the FP16, D3Q27 and adjoint legs")
    ap.add_argument("--extra-scale", type=float, default=1.0, help="scale the step counts of those legs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: one GPU only (got --gpus {args.gpus}); the step would shard by slabs, "
              "but the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2203_01316_amd import lbm as L
    from paper_2203_01316_amd import workloads as W

    dev = torch.device("cuda:0")
    nx, ny = args.nx, args.ny
    nu = 0.04 * 128 / 100.0
    k = nu / 0.71
    flags, q, groups, u, rho0, H0 = W.heated_cylinder(nx, ny, 64, u_in=0.04, amp=1e-3, seed=0)
    uf = np.asarray(u, np.float32)
    g = L.LBM(L.D2Q9, nx, ny, with_ns=True, storage=args.storage, nu=nu, k=k, relax_f="ns", relax_h="trt",
              flags=flags, q=q, groups=groups, device=dev,
              stream=L.STREAM_AA if args.stream == "aa" else L.STREAM_AB)
    g.set_velocity(uf)
    g.init(H0, u=uf.astype(np.float64), rho=rho0)
    n = nx * ny
    nl, nspecial = L.count_geometry(g.params, flags)
    nsolid = int(np.count_nonzero((flags & 15) == L.SOLID))

    ceiling = copy_ceiling(torch, L, dev)

    g.step(args.warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    g.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_sec = e0.elapsed_time(e1) / 1e3
    sec = max(wall, gpu_sec)
    red = g.reduce(group=1, columns=[50, nx - 101])

    bytes_node = 2 * 2 * 9 * (8 if args.storage == "fp64" else 4 if args.storage.startswith("fp32") else 2)
    mlups = n * args.steps / sec / 1e6
    # One fused launch per step covers every non-solid node (bulk and
    # boundary), launched back to back on this stream (AA: the two layout
    # phases alternate): the HIP events around the timed region divided by the
    # step count give the average launch duration (inter-launch gaps
    # included, so this errs low).
    n_work = n - nsolid
    launch_avg = gpu_sec / args.steps
    achieved = n_work * bytes_node / launch_avg
    traffic = read_traffic(f"d2q9_ns_ade_{nx}x{ny}_{args.storage}_{args.stream}")
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.storage in ("fp64", "fp32_sr") else "f32",
        "data": "synthetic",
        "config": {"workload": f"d2q9_ns_ade_heated_cylinder_{nx}x{ny}", "lattice": "D2Q9",
                   "lattices": "f (NS, CM) + h (ADE, CM-TRT)", "nx": nx, "ny": ny,
                   "storage": args.storage, "stream": args.stream.upper(), "Re": 100, "Pr": 0.71,
                   "bytes_per_node": bytes_node, "boundary_nodes": nspecial, "solid_nodes": nsolid},
        "pct_hbm_roofline": round(100.0 * mlups * 1e6 * bytes_node / HBM_PEAK, 2),
        "roofline": {"bound": "hbm", "achieved": round(achieved / 1e9, 1), "peak": HBM_PEAK / 1e9,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK, 4),
                     "traffic": None if traffic is None else int(traffic),
                     "kernel": "k_fused" + (" (AA: swapped and streamed layout phases alternate)"
                                            if args.stream == "aa" else ""),
                     "avg_launch_us": round(launch_avg * 1e6, 2),
                     "bytes_per_launch": n_work * bytes_node,
                     "note": cache_note(args.stream, n_work * bytes_node),
                     "frac_of_copy": round(achieved / (ceiling["lbm_copy_GBps"] * 1e9), 4)},
        "copy_ceiling_GBps": ceiling["lbm_copy_GBps"],
        "copy_ceiling": ceiling,
        "mass": red[0],
        "energy": red[1],
    }
    del g
    torch.cuda.empty_cache()
    sc = args.extra_scale
    # the same step in the other layout; with two arrays (AB) the population
    # sets (604 MB at 2048^2 FP32) exceed the Infinity Cache, so that rate is
    # the step's rate from HBM alone
    other = "ab" if args.stream == "aa" else "aa"
    leg_other = leg_cylinder(torch, L, W, np, args.storage, other, nx, ny, max(10, int(1000 * sc)))
    ab = leg_other if other == "ab" else None
    if args.stream == "ab":
        ab = {"us_per_step": round(launch_avg * 1e6, 2)}
    if ab is not None:
        ab_rate = n_work * bytes_node / (ab["us_per_step"] * 1e-6)
        out["roofline"]["hbm_only"] = {"stream": "AB", "achieved": round(ab_rate / 1e9, 1),
                                       "frac": round(ab_rate / HBM_PEAK, 4),
                                       "frac_of_copy": round(ab_rate / (ceiling["lbm_copy_GBps"] * 1e9), 4),
                                       "avg_launch_us": ab["us_per_step"]}
    if not args.no_extra:
        out["also"] = [leg_other,
                       leg_cylinder(torch, L, W, np, "fp16_dev", "aa", nx, ny, max(10, int(1000 * sc))),
                       leg_cylinder(torch, L, W, np, "fp16_dev", "ab", nx, ny, max(10, int(1000 * sc))),
                       leg_tgv(torch, L, W, "fp32", 256, max(5, int(100 * sc))),
                       leg_tgv(torch, L, W, "fp32", 256, max(5, int(100 * sc)), stream="aa"),
                       leg_tgv(torch, L, W, "fp16_dev", 256, max(5, int(100 * sc))),
                       # the paper's kernels: cumulant f with CM-TRT or Cumulants-1st h
                       leg_cylinder(torch, L, W, np, "fp32", "aa", nx, ny, max(10, int(1000 * sc)), cu_f=True),
                       leg_cylinder(torch, L, W, np, "fp32", "aa", nx, ny, max(10, int(1000 * sc)), cu_f=True,
                                    cu_h=True),
                       leg_tgv(torch, L, W, "fp32", 256, max(5, int(100 * sc)), cu=True),
                       # FP32 storage, FP64 arithmetic, stochastic rounding on store
                       leg_cylinder(torch, L, W, np, "fp32_sr", "ab", nx, ny, max(10, int(1000 * sc))),
                       leg_cylinder(torch, L, W, np, "fp32_sr", "aa", nx, ny, max(10, int(1000 * sc))),
                       leg_tgv(torch, L, W, "fp32_sr", 256, max(5, int(100 * sc))),
                       # FP16 deviations rounded stochastically
                       leg_cylinder(torch, L, W, np, "fp16_sr", "ab", nx, ny, max(10, int(1000 * sc))),
                       leg_tgv(torch, L, W, "fp16_sr", 256, max(5, int(100 * sc)))]
        out["adjoint"] = leg_adjoint(torch, L, np, steps=max(90, int(2000 * sc)))
        # headline: the checkpointed gradient with its forward replay (sqrt(T)
        # checkpoints); without the replay alongside
        out["adjoint_forward_ratio"] = out["adjoint"]["with_replay"]["ratio"]
        out["adjoint_forward_ratio_no_replay"] = out["adjoint"]["no_replay"]["ratio"]
        out["adjoint_forward_ratio_tracking"] = out["adjoint"]["tracking_every_10"]["ratio"]
    if not args.no_cpu:
        inputs = (flags, q, groups, uf.astype(np.float64), rho0, H0, nx, ny, nu, k)
        out["cpu_baseline"] = cpu_baseline(inputs, args.cpu_steps, not args.no_cpu_single)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
