"""Benchmark of the four-phonon rate path on one MI355X.

Workload: the 8x8x8 four-phonon FP64 configuration (2-atom diamond cell,
Oh-irreducible q1 set, 32 cubic + 94 quartic force-constant terms, Gaussian
width 0.1 THz, |Delta| <= 3 sigma, T = 300 K).  Lists are enumerated once on
the host by the library and uploaded before timing.  One step is the whole hot
path: force-constant load (order 3 and 4, device-resident values), 3ph and 4ph
rates accumulated into Gamma = Gamma3 + Gamma4, and kappa_RTA.

Prints one JSON line.  value = 4ph processes per second of the whole step.
roofline: the dominant kernel (the order-4 rate kernel) timed with HIP events
on its own stream, algorithmic FLOP = (320 n4 + 60) per process, against the
FP64 vector peak.  cpu_baseline: the FP64 oracle (list mode) on a bounded
sample of the same lists on this host's cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 FP64 lanes x 2 FLOP x 2.4 GHz
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_rates4_fcc8_4ph.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2510_00518_amd", "csrc", f) for f in ("fp_kernels.h", "fp_batched.h", "fp_lib.hip")]


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(cfg, lists, seconds, seed=251000518 + 6):
    """Oracle list-mode throughput on seeded slices of the 4ph lists (bounded time)."""
    import oracle
    from paper_2510_00518_amd import fp
    S = oracle.System(cfg)
    rm, off, rec = lists[fp.FP_4PM]
    rng = np.random.default_rng(seed)
    slice_len = 20000
    done, spent, rows_used = 0, 0.0, 0
    while spent < seconds:
        r = int(rng.integers(len(rm)))
        n = int(off[r + 1] - off[r])
        if n == 0:
            continue
        a = int(off[r]) + int(rng.integers(max(1, n - slice_len)))
        sub = rec[a:min(a + slice_len, int(off[r + 1]))]
        t0 = time.perf_counter()
        S.rates(fp.FP_4PM, rm[r:r + 1], [300.0], cfg["sigma"], row_off=np.array([0, len(sub)]), rec=sub)
        spent += time.perf_counter() - t0
        done += len(sub)
        rows_used += 1
    return {"value": done / spent, "unit": "processes/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{done} four-phonon (+-) records in {rows_used} seeded slices of {slice_len} from the "
                      f"benchmark's lists, FP64 list mode, {spent:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (reference kernel for HBM counter scaling)")
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--ppl", type=int, default=None)
    ap.add_argument("--blocks-per-cu", type=int, default=None)
    ap.add_argument("--variant", type=int, default=None, help="order-4 contraction form (library knob)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the rate path is built and timed on a single MI355X; "
              "multi-GPU sharding is a design in DESIGN.md, not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2510_00518_amd import fp
    from paper_2510_00518_amd.driver import TYPES3, TYPES4, RatePath, host_lists
    from paper_2510_00518_amd.synth import make_config

    if not os.path.exists(fp.LIB_PATH):
        from __graft_entry__ import build
        build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    cfg = make_config("fcc8_4ph")
    n4 = int(cfg["ifc4"]["n_terms"])
    T = [float(x) for x in cfg["T"]]
    log("bench: enumerating lists on the host")
    t0 = time.perf_counter()
    lists = host_lists(cfg, TYPES3 + TYPES4)
    t_enum = time.perf_counter() - t0
    path = RatePath(cfg, device=0)
    if args.ppl:
        fp.fp_set_knob(path.ctx, "ppl", args.ppl)
    if args.blocks_per_cu:
        fp.fp_set_knob(path.ctx, "blocks_per_cu", args.blocks_per_cu)
    if args.variant is not None:
        fp.fp_set_knob(path.ctx, "variant", args.variant)
    path.set_lists(lists)
    n_proc4, n_proc3 = path.n_proc4, path.n_proc3
    log(f"bench: {n_proc4} 4ph + {n_proc3} 3ph processes, enumeration {t_enum:.1f} s")
    gamma = torch.zeros((len(T), path.n_modes), dtype=torch.float64, device="cuda")
    kappa = torch.zeros((len(T), 9), dtype=torch.float64, device="cuda")

    if args.copy_calibration:
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        src.fill_(1.0)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for i in range(args.warmup):
        path.step(T, gamma, kappa)
        torch.cuda.synchronize()
        log(f"bench: warmup step {i + 1}/{args.warmup} done")
    fp.fp_check(path.ctx)
    fp.fp_profile(path.ctx, True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        path.step(T, gamma, kappa)
    e1.record()
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    rates_ms, launches = fp.fp_profile_read(path.ctx, 4)
    fp.fp_profile(path.ctx, False)
    fp.fp_check(path.ctx)
    ms_step = ms_total / args.steps
    kern_ms = rates_ms / max(1, launches)
    log(f"bench: {args.steps} steps, {ms_step:.3f} ms/step, order-4 rate kernel {kern_ms:.3f} ms/launch")
    kap = kappa.cpu().numpy()
    finite = bool(np.all(np.isfinite(kap)))

    # backward step: dkappa/dGamma, then the adjoint of both rate orders
    bwd = None
    if not args.no_backward:
        dk = torch.zeros_like(gamma)
        d3 = torch.zeros_like(path.phi3)
        d4 = torch.zeros_like(path.phi4)

        def backward_step():
            path.kappa(T, gamma, kappa, dk)
            fp.fp_rates_backward(path.ctx, path.lists3 + path.lists4, T, cfg["sigma"], dk, d3, d4)

        backward_step()
        torch.cuda.synchronize()
        fp.fp_check(path.ctx)
        fp.fp_profile(path.ctx, True)
        b0, b1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        b0.record()
        for _ in range(args.steps):
            backward_step()
        b1.record()
        torch.cuda.synchronize()
        g4_ms, g4_n = fp.fp_profile_read(path.ctx, 14)
        fp.fp_profile(path.ctx, False)
        fp.fp_check(path.ctx)
        ms_bwd = b0.elapsed_time(b1) / args.steps
        bwd = {"ms_per_step": ms_bwd, "bwd_fwd_ratio": ms_bwd / ms_step,
               "adjoint4_kernel_ms": g4_ms / max(1, g4_n),
               "step": "kappa_RTA with dkappa/dGamma + adjoint of the 3ph and 4ph rates (V recomputed)"}
        log(f"bench: backward {ms_bwd:.3f} ms/step, ratio {ms_bwd / ms_step:.2f}")

    flop_per_proc = 320 * n4 + 60
    achieved = flop_per_proc * n_proc4 / (kern_ms * 1e-3) / 1e12
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        if tr.get("kernel_source_hash") == kernel_source_hash():
            traffic = tr.get("hbm_bytes_per_launch")
    out = {
        "metric": "4ph processes/sec at 1 GPU, FP64 vs mixed (rel err vs oracle); bwd/fwd time ratio",
        "value": n_proc4 / (ms_step * 1e-3),
        "unit": "processes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "4ph FP64, 2-atom diamond cell, 8x8x8 mesh, Oh-irreducible q1 (29), "
                        f"32 cubic + {n4} quartic terms, sigma 0.1 THz, |Delta| <= 3 sigma, T = 300 K",
            "processes_4ph": n_proc4,
            "processes_3ph": n_proc3,
            "step": "load_ifc(3,4) + rates3 + rates4 (Gamma3+Gamma4) + kappa_RTA",
            "host_enumeration_s": round(t_enum, 2),
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": traffic,
            "kernel": "k_rates<4,1> (order-4 rate kernel)",
            "kernel_ms": kern_ms,
            "flop_per_process": flop_per_proc,
        },
        "kappa_finite": finite,
        "mixed": None,
        "bwd_fwd_ratio": None if bwd is None else bwd["bwd_fwd_ratio"],
        "backward": bwd,
    }
    if not args.no_cpu_baseline:
        log("bench: timing the oracle on the host")
        out["cpu_baseline"] = cpu_baseline(cfg, lists, args.cpu_seconds)
    path.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
