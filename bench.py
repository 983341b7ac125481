"""ST-HOSVD throughput on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--path fp64|mixed]

A step is one full ST-HOSVD (Alg. 1: every mode's Gram, FP64 eigensolve,
rank rule and TTM) of the combustion-shaped 128x128x128x32x32 tensor
(planted ranks (16,16,16,8,8), spectra decaying by 0.7, cosine factors,
noise 1e-5), eps = 1e-4, modes in order 1..5, with the tensor resident in
HBM.  The timed region is exactly K steps bracketed by device
synchronisation.  Prints one JSON line with the input throughput (GB/s of
input tensor per second), the roofline of the dominant kernel (the mode-1
Gram), and the CPU oracle timed on a bounded slab of the same tensor.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import torch  # noqa: E402

import synth  # noqa: E402
from paper_1510_06689_amd import tucker  # noqa: E402

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_MFMA_PEAK_TFS = 78.6      # MI355X dense FP64 matrix
BF16_MFMA_PEAK_TFS = 2500.0    # MI355X dense BF16 matrix


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def gram_flops(j: int, numel: int) -> float:
    """Symmetric Gram count: J (J + 1) multiply-adds per column pair set,
    i.e. (J + 1) * #Y flops for a J x (#Y / J) unfolding."""
    return float(j + 1) * numel


def time_gram(x, mode, precision, reps, stream):
    """Average duration of one gram_mode_n launch on the library's stream,
    measured with HIP events recorded on that same stream."""
    import ctypes
    lib = tucker.library()
    sh = tucker.shape_of(x)
    prec = tucker.GRAM_PRECISIONS[precision]
    need = lib.gram_workspace_bytes(ctypes.byref(sh), mode, prec)
    ws = tucker._workspace(need, x.device)
    j = x.shape[mode]
    s = torch.empty((j, j), dtype=torch.float64, device=x.device)
    args = (ctypes.byref(sh), x.data_ptr(), mode, prec, s.data_ptr(), None,
            tucker._aligned(ws), need, ctypes.c_void_p(stream.cuda_stream))
    tucker._check(lib.gram_mode_n(*args))  # warm
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        start.record(stream)
        for _ in range(reps):
            tucker._check(lib.gram_mode_n(*args))
        end.record(stream)
    end.synchronize()
    return start.elapsed_time(end) / 1e3 / reps


def cpu_baseline(x_dev, eps, path):
    """The FP64 CPU oracle on one time-step slab of the same tensor."""
    import oracle
    import numpy as np
    sample = x_dev[..., 0:1]
    xs = np.asfortranarray(sample.double().cpu().numpy())
    t0 = time.perf_counter()
    oracle.sthosvd(xs, eps)
    dt = time.perf_counter() - t0
    in_bytes = xs.size * x_dev.element_size()
    return {"value": round(in_bytes / dt / 1e9, 4), "unit": "GB/s", "cores": 1,
            "kind": "oracle",
            "sample": f"one time step of the same tensor, dims {list(xs.shape)}, "
                      f"{path} input bytes {in_bytes}, {dt:.1f} s single-threaded"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--path", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--gram-reps", type=int, default=10)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    w = synth.WORKLOADS["combustion128"]
    dtype = torch.float64 if args.path == "fp64" else torch.float32
    gp, tp = ("fp64", "fp64") if args.path == "fp64" else ("split_bf16", "bf16x3")
    log(f"generating {w.name} {w.dims} on {dev}")
    x = w.make(dtype=dtype, device=dev)
    torch.cuda.synchronize()
    comp = tucker.Compressor(w.dims, dtype, dev, w.eps, gram_precision=gp, ttm_precision=tp)
    stream = torch.cuda.current_stream(dev)

    for i in range(args.warmup):
        comp.run(x)
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        comp.run(x)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt / args.steps * 1e3
    in_bytes = x.numel() * x.element_size()
    value = in_bytes / (ms / 1e3) / 1e9
    res = comp.result()
    log(f"timed {args.steps} steps: {ms:.3f} ms/step, {value:.1f} GB/s, ranks {res.ranks}")

    # accuracy of the timed configuration (untimed)
    xh = tucker.reconstruct(res.core, res.factors, precision="fp64")
    e2, mx, n2 = tucker.error_metrics(x, xh)
    relerr = math.sqrt(e2 / n2)
    del xh
    torch.cuda.empty_cache()

    # roofline of the dominant kernel: the mode-1 Gram
    tg = time_gram(x, 0, gp, args.gram_reps, stream)
    flops = gram_flops(w.dims[0], x.numel())
    if args.path == "fp64":
        achieved = flops / tg / 1e12
        roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_MFMA_PEAK_TFS,
                "unit": "TFLOP/s", "frac": round(achieved / FP64_MFMA_PEAK_TFS, 4),
                "traffic": None, "kernel": "gram_partial_f64 (mode 1, J=128)",
                "gram_ms": round(tg * 1e3, 4), "algorithmic_flops": flops}
    else:
        achieved = in_bytes / tg / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "gram_partial_split_bf16 (mode 1, J=128)",
                "gram_ms": round(tg * 1e3, 4), "algorithmic_bytes": in_bytes}
    log(f"mode-1 gram: {tg * 1e3:.3f} ms")

    out = {
        "metric": "ST-HOSVD input GB/s + Gram/TTM TFLOP/s, mixed vs FP64 GPU at rel err <=1e-4",
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.path == "fp64" else "bf16-split/f32/f64",
        "data": "synthetic",
        "config": {"workload": "combustion128: 128x128x128x32x32 planted Tucker, ranks "
                               "(16,16,16,8,8), decay 0.7, noise 1e-5, eps 1e-4, order 1..5",
                   "dims": list(w.dims), "eps": w.eps, "path": args.path,
                   "storage": str(dtype).replace("torch.", ""),
                   "gram": gp, "ttm": tp},
        "ranks": list(res.ranks), "relerr": relerr, "max_abs_err": mx,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(x, w.eps, args.path)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
