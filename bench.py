#!/usr/bin/env python3
"""Benchmark of the exact symmetric product A A^T mod p on one MI355X.

Metric: effective Gop/s = sum of n^2 k over the step / time (the classical
cost of A A^T counted as n^2 k operations).  Default workload: A of shape
8192 x 8192 and 8192 x 32768 with entries uniform in [0, 131071), p = 131071
(a sum of two squares builds Y), three levels of Algorithm 2 over FP64
matrix-core base products.  One step = fsyrk_modp on both shapes.

Inputs are drawn on the host with numpy's PCG64 (seed 1) and are resident in
HBM before the timed region.  Besides the JSON line the run prints nothing
on stdout.  Roofline figures come from HIP events around every product
launch in the timed region; the CPU baseline is the oracle on a bounded row
panel of the same product.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "effective Gop/s (n²k/s) for A·Aᵀ mod p, batched vs plain; p50/p99 latency"
PEAK_F64 = 78.6      # TFLOP/s, MI355X FP64 matrix
PEAK_I8 = 5000.0     # TOP/s, MI355X dense int8
HBM = 8000.0         # GB/s

WORKLOADS = {
    "syrk_8192_p131071_depth3": dict(shapes=[(8192, 8192), (8192, 32768)], p=131071, depth=3,
                                     seed=1, dtype="u32", cls=0),
    "syrk_16384_p251_int8": dict(shapes=[(16384, 16384)], p=251, depth=0, seed=2, dtype="i8",
                                 cls=1),
    "syrk_16384_p65521_limb2": dict(shapes=[(16384, 16384)], p=65521, depth=0, seed=2,
                                    dtype="limb2", cls=2),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def upload(A, p, dtype):
    import torch
    from tests.gpu_util import centred_i8, limbs
    if dtype == "u32":
        return torch.from_numpy(A.view(np.int32)).cuda()
    if dtype == "i8":
        return torch.from_numpy(centred_i8(A, p)).cuda()
    return torch.from_numpy(limbs(A, p)).cuda()


def profile_hooks():
    import ctypes
    from paper_2001_04109_amd import ffp
    L = ffp.lib()
    L.ffp_debug_profile.argtypes = [ctypes.c_int]
    L.ffp_debug_profile.restype = None
    L.ffp_debug_profile_read.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int64)]
    L.ffp_debug_profile_read.restype = ctypes.c_int

    L.ffp_debug_profile_read_variant.argtypes = L.ffp_debug_profile_read.argtypes
    L.ffp_debug_profile_read_variant.restype = ctypes.c_int
    L.ffp_debug_variant_name.argtypes = [ctypes.c_int]
    L.ffp_debug_variant_name.restype = ctypes.c_char_p

    def read(cls):
        ms, fl, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        L.ffp_debug_profile_read(cls, ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(n))
        return ms.value, fl.value, n.value

    def read_variants():
        """{variant: (ms, flops, launches, name)} of the recorded launches."""
        out = {}
        for v in range(6):
            ms, fl, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
            L.ffp_debug_profile_read_variant(v, ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(n))
            if n.value:
                out[v] = (ms.value, fl.value, n.value, L.ffp_debug_variant_name(v).decode())
        return out
    return L.ffp_debug_profile, read, read_variants


def run_workload(name, steps, warmup, check=True):
    import torch
    from paper_2001_04109_amd import ffp, inputs
    import oracle

    w = WORKLOADS[name]
    p = w["p"]
    a_dtype = {"u32": ffp.FFP_U32, "i8": ffp.FFP_I8_CENTERED, "limb2": ffp.FFP_I8_LIMB2}[w["dtype"]]
    mats, devs, outs = [], [], []
    for (n, k) in w["shapes"]:
        A = inputs.uniform(w["seed"], n, k, p)
        mats.append(A)
        devs.append(upload(A, p, w["dtype"]))
        outs.append(torch.zeros((n, n), dtype=torch.int32, device="cuda"))
    torch.cuda.synchronize()

    def step():
        for Ad, Cd in zip(devs, outs):
            ffp.syrk(Ad, p, C=Cd, depth=w["depth"], a_dtype=a_dtype)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    prof_enable, prof_read, prof_variants = profile_hooks()
    prof_read(-1)
    prof_enable(1)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    prof_enable(0)
    ms = e0.elapsed_time(e1) / steps
    variants = prof_variants()
    # dominant product kernel: the variant with the most time in the step
    dom = max(variants.items(), key=lambda kv: kv[1][0]) if variants else None
    eff = sum(n * n * k for (n, k) in w["shapes"])
    res = dict(ms_per_step=ms, gops=eff / (ms * 1e-3) / 1e9)
    if dom:
        v, (kms, kflops, nl, kname) = dom
        res.update(kernel=kname, kernel_ms=kms / steps, kernel_flops=kflops / steps,
                   launches=nl // max(steps, 1), kernel_avg_ms=kms / nl,
                   all_kernels={name: round(t / steps, 4) for (t, _, _, name) in variants.values()})
    if check:
        # sampled bit-exact check of the last step's results against the oracle
        for A, Cd in zip(mats, outs):
            n = A.shape[0]
            rng = np.random.default_rng(7)
            r = rng.integers(0, n, 64)
            c = rng.integers(0, n, 64)
            lo, hi = np.maximum(r, c), np.minimum(r, c)
            got = Cd.cpu().numpy().view(np.uint32)[lo, hi]
            if not np.array_equal(got, oracle.syrk_entries(A, p, lo, hi)):
                raise SystemExit(f"bench: {name} result differs from the oracle")
    del devs, outs
    torch.cuda.empty_cache()
    return res


def cpu_baseline(name):
    """Oracle on a bounded sample: rows [n-r, n) of the lower triangle of the
    first shape, i.e. r*(2n-r+1)/2 dot products of length k (r = n for the
    8192 x 8192 product: its whole lower triangle)."""
    import oracle
    from paper_2001_04109_amd import inputs
    w = WORKLOADS[name]
    n, k = w["shapes"][0]
    p = w["p"]
    A = inputs.uniform(w["seed"], n, k, p)
    r = n if n * n * k <= 8192 ** 3 else max(64, int(8192 ** 3 / (n * k)))
    t0 = time.perf_counter()
    oracle.syrk_rows(A, p, n - r, n)
    dt = time.perf_counter() - t0
    macs = r * (2 * n - r + 1) // 2 * k
    return {"value": round(2.0 * macs / dt / 1e9, 3), "unit": "Gop/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"rows [{n - r},{n}) of lower(A A^T) for A {n}x{k} mod {p} "
                      f"({macs:.3e} multiply-adds, {dt:.1f} s)"}


def traffic_for(kernel, workload):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    return d.get(f"{kernel}:{workload}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="syrk_8192_p131071_depth3", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (--gpus {args.gpus} "
              "requested)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a ROCm GPU")
    from paper_2001_04109_amd import ffp
    ffp.lib()

    name = args.workload
    w = WORKLOADS[name]
    log(f"bench: {name} steps={args.steps} warmup={args.warmup}")
    res = run_workload(name, args.steps, args.warmup)
    log(f"bench: {name} {res['ms_per_step']:.3f} ms/step {res['gops']:.1f} Gop/s")
    if w["cls"] == 0:
        peak, unit = PEAK_F64, "TFLOP/s"
    else:
        peak, unit = PEAK_I8, "TOP/s"
    kname = res.get("kernel", "")
    achieved = res["kernel_flops"] / (res["kernel_ms"] * 1e-3) / 1e12 if res.get("kernel_ms") else 0.0
    roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 4), "traffic": traffic_for(kname, name),
            "kernel": kname, "kernel_avg_launch_ms": round(res.get("kernel_avg_ms", 0.0), 5),
            "kernel_ms_per_step": round(res.get("kernel_ms", 0.0), 4),
            "launches_per_step": res.get("launches", 0),
            "product_kernels_ms_per_step": res.get("all_kernels", {})}
    extra = {}
    if not args.no_extra:
        for other in ("syrk_16384_p251_int8", "syrk_16384_p65521_limb2"):
            if other == name:
                continue
            log(f"bench: extra {other}")
            r2 = run_workload(other, max(3, args.steps // 3), 1)
            a2 = r2["kernel_flops"] / (r2["kernel_ms"] * 1e-3) / 1e12 if r2.get("kernel_ms") else 0.0
            extra[other] = {"gops": round(r2["gops"], 1), "ms_per_step": round(r2["ms_per_step"], 4),
                            "frac_int8_peak_effective": round(r2["gops"] / 1e3 / PEAK_I8, 4),
                            "kernel_achieved_TOPs": round(a2, 2)}
    cpu = None
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        cpu = cpu_baseline(name)
    n0, _ = w["shapes"][0]
    out = {
        "metric": METRIC,
        "value": round(res["gops"], 2),
        "unit": "Gop/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if w["cls"] == 0 else "int8",
        "data": "synthetic (seeded uniform residues, numpy PCG64)",
        "config": {"workload": name, "n": n0, "k": [k for (_, k) in w["shapes"]], "p": w["p"],
                   "depth": w["depth"], "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
