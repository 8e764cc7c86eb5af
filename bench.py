"""Benchmark of the four-phonon rate path on one MI355X.

Workload: the 8x8x8 four-phonon FP64 configuration (2-atom diamond cell,
Oh-irreducible q1 set, 32 cubic + 94 quartic force-constant terms, Gaussian
width 0.1 THz, |Delta| <= 3 sigma, T = 300 K).  Lists are enumerated once on
the host by the library and uploaded before timing.  One step is the whole hot
path: force-constant load (order 3 and 4, device-resident values), 3ph and 4ph
rates accumulated into Gamma = Gamma3 + Gamma4, and kappa_RTA.

Prints one JSON line.  value = 4ph processes per second of the whole FP64 step;
"mixed" holds the same step with the order-4 rates in mixed precision (bf16
split MFMA, FP32 contraction, FP64 weights) and its errors against FP64.
roofline: the dominant kernel (the order-4 rate kernel) timed with HIP events
on its own stream, with the algorithmic FLOP of the form that ran: (320 n4 + 60)
per process for the per-process forms; 216 n4 per (lambda, q', q'') tuple on
FP64 MFMA (and 312 n_groups + 60 per process on the VALU) for the tuple-batched
form.  backward: kappa_RTA with dkappa/dGamma and the adjoint of both orders.
adaptive: the same step with the per-process width sigma_p = max(0.1 sigma0_p,
0.01 THz) from the group velocities (the paper's broadening scale 0.1) on lists
the host enumerates with that width.
cpu_baseline: the FP64 oracle (list mode) on a bounded sample of the same lists
on this host's cores.  --paper-scale adds the 16x16x16 two-atom cell (every row,
three types, T = 300/600/900 K) through GPU-side enumeration, FP64 and mixed,
each with a roofline from the library's tuple count; with --paper-scale-adaptive
the adaptive width too.  They hold the GPU for about a minute, so they are not
part of the default run.
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

PEAK_FP64_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 FP64 lanes x 2 FLOP x 2.4 GHz (vector; FP64 MFMA the same)
PEAK_BF16_TFLOPS = 2500.0  # dense bf16 MFMA
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_rates4_fcc8_4ph.json")
# device code of the tuple-batched FP64 kernel (its launch shape is the variant knob)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2510_00518_amd", "csrc", f) for f in ("fp_kernels.h", "fp_batched.h")]


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


def tuple_stats(lists, nb, unit=128):
    """Distinct (lambda, q', q'') tuples of the 4ph lists, and the tuples the
    tuple-batched kernels form (a tuple split by a 128-record unit boundary
    counts once per unit)."""
    from paper_2510_00518_amd import fp
    n_tup = n_unit_tup = 0
    for t, (rm, off, rec) in lists.items():
        if fp.ORDER[t] != 4 or len(rec) == 0:
            continue
        q1 = (rec & np.uint64(0xFFFFFF)).astype(np.int64) // nb
        q2 = ((rec >> np.uint64(24)) & np.uint64(0xFFFFFF)).astype(np.int64) // nb
        key = q1 * (1 << 24) + q2
        del q1, q2
        row_start = np.zeros(len(rec), dtype=bool)
        row_start[off[:-1][np.diff(off) > 0]] = True
        new = row_start.copy()
        new[1:] |= key[1:] != key[:-1]
        n_tup += int(new.sum())
        pos = np.arange(len(rec), dtype=np.int64) - np.repeat(off[:-1], np.diff(off))
        n_unit_tup += int((new | (pos % unit == 0)).sum())
    return n_tup, n_unit_tup


def partner_groups(ifc):
    """Partner-atom groups of a force-constant list (distinct atoms of slots 1..m-1)."""
    return len({tuple(a[1:]) for a in np.asarray(ifc["atoms"]).tolist()})


def paper_scale(torch, fp, RatePath, adaptive=False, precision=None):
    """The 16^3 two-atom cell: every active row and the three four-phonon types
    in one fp_rates4_fused call (lists generated on the GPU), T = 300/600/900 K;
    with adaptive, the per-process width max(0.1 sigma0_p, 0.01 THz)."""
    from paper_2510_00518_amd.synth import SIGMA_FLOOR, adaptive_broadening, make_config, row_modes
    cfg = make_config("fcc16_34ph")
    if adaptive:
        cfg = dict(cfg, sigma=SIGMA_FLOOR)
    T = [float(x) for x in cfg["T"]]
    p = RatePath(cfg, device=0, precision=fp.FP_FP64 if precision is None else precision)
    if adaptive:
        p.set_broadening(adaptive_broadening(cfg))
    p.set_fused(row_modes(cfg), 7)
    gam, wp = p.outputs(len(T))
    p.load_ifc()
    fp.fp_profile(p.ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p.rates(T, gam, wp, order=4)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    k_ms, n = fp.fp_profile_read(p.ctx, 34)
    fp.fp_profile(p.ctx, False)
    fp.fp_check(p.ctx)
    kept = int(p.kept.cpu()[0])
    n_proc, n_tup = fp.fp_fused_counts(p.ctx)
    n4 = int(cfg["ifc4"]["n_terms"])
    n_groups = partner_groups(cfg["ifc4"])
    p.close()
    mixed = precision == fp.FP_MIXED
    # the fused kernel's algorithmic work in the tuple form that ran: 216 n4 FLOP per
    # (lambda, q', q'') tuple on matrix cores, (312 n_groups + 60) per process on the VALU
    sec = k_ms / max(1, n) * 1e-3
    f_build = 216 * n4 * n_tup
    f_contract = (312 * n_groups + 60) * n_proc
    if mixed:
        roof = {"bound": "mfma", "achieved": 6 * f_build / sec / 1e12, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                "kernel": "k_fused4 mixed (bf16 split MFMA + FP32 VALU)",
                "work": f"6 bf16 products per FP32-accurate product, 216*n4 FLOP per tuple, n4 = {n4}, {n_tup} tuples",
                "fp32_equivalent_tflops": f_build / sec / 1e12}
    else:
        roof = {"bound": "mfma", "achieved": f_build / sec / 1e12, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "kernel": "k_fused4 (GPU enumeration + tuple-batched FP64 MFMA + FP64 VALU)",
                "work": f"216*n4 FLOP per (lambda, q', q'') tuple on FP64 MFMA, n4 = {n4}, {n_tup} tuples"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["valu_achieved"] = f_contract / sec / 1e12
    roof["per_process_form_equivalent_tflops"] = (320 * n4 + 60) * n_proc / sec / 1e12
    roof["kernel_ms"] = k_ms / max(1, n)
    roof["traffic"] = None
    log(f"bench: 16^3 fused{' adaptive' if adaptive else ''}{' mixed' if mixed else ''}: {kept} processes in {dt:.2f} s")
    width = "adaptive width max(0.1 sigma0, 0.01 THz)" if adaptive else "sigma 0.1 THz"
    return {"workload": f"4ph {'mixed' if mixed else 'FP64'}, 2-atom diamond cell, 16x16x16 mesh, "
                        "Oh-irreducible q1 (145), 62 cubic + "
                        f"{int(cfg['ifc4']['n_terms'])} quartic terms, T = 300/600/900 K, {width}, "
                        "lists generated on the GPU",
            "processes_4ph": kept, "tuples_4ph": n_tup, "seconds": dt, "value": kept / dt, "unit": "processes/s",
            "kernel_ms": k_ms / max(1, n), "rows": int(len(row_modes(cfg))), "roofline": roof}


def run_forward(path, T, steps, warmup, tag, torch, fp):
    """Warm up, then time `steps` whole steps; returns ms/step, the tagged
    kernel's ms/launch, and the last step's Gamma and kappa (host copies)."""
    gamma = torch.zeros((len(T), path.n_modes), dtype=torch.float64, device="cuda")
    kappa = torch.zeros((len(T), 9), dtype=torch.float64, device="cuda")
    for i in range(warmup):
        path.step(T, gamma, kappa)
        torch.cuda.synchronize()
        log(f"bench: warmup step {i + 1}/{warmup} done")
    fp.fp_check(path.ctx)
    fp.fp_profile(path.ctx, True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        path.step(T, gamma, kappa)
    e1.record()
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / steps
    k_ms, launches = fp.fp_profile_read(path.ctx, tag)
    fp.fp_profile(path.ctx, False)
    fp.fp_check(path.ctx)
    return ms_step, k_ms / max(1, launches), gamma, kappa


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
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-adaptive", action="store_true")
    ap.add_argument("--paper-scale-adaptive", action="store_true",
                    help="also run the 16^3 cell with the adaptive width (about a minute)")
    ap.add_argument("--paper-scale", action="store_true",
                    help="also run the 16^3 two-atom cell through GPU-side enumeration (about a minute)")
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
    from paper_2510_00518_amd.synth import ADAPTIVE_FACTOR, SIGMA_FLOOR, adaptive_broadening, make_config

    if not os.path.exists(fp.LIB_PATH):
        from __graft_entry__ import build
        build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    cfg = make_config("fcc8_4ph")
    n4 = int(cfg["ifc4"]["n_terms"])
    n_groups = partner_groups(cfg["ifc4"])
    T = [float(x) for x in cfg["T"]]
    log("bench: enumerating lists on the host")
    t0 = time.perf_counter()
    lists = host_lists(cfg, TYPES3 + TYPES4)
    t_enum = time.perf_counter() - t0
    n_tup, n_unit_tup = tuple_stats(lists, cfg["nb"])
    path = RatePath(cfg, device=0)
    if args.ppl:
        fp.fp_set_knob(path.ctx, "ppl", args.ppl)
    if args.blocks_per_cu:
        fp.fp_set_knob(path.ctx, "blocks_per_cu", args.blocks_per_cu)
    if args.variant is not None:
        fp.fp_set_knob(path.ctx, "variant", args.variant)
    variant = fp.fp_get_knob(path.ctx, "variant")
    path.set_lists(lists)
    n_proc4, n_proc3 = path.n_proc4, path.n_proc3
    log(f"bench: {n_proc4} 4ph + {n_proc3} 3ph processes in {n_tup} (lambda, q', q'') tuples, "
        f"enumeration {t_enum:.1f} s")

    if args.copy_calibration:
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        src.fill_(1.0)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---- FP64 forward
    ms_step, kern_ms, gamma, kappa = run_forward(path, T, args.steps, args.warmup, 4, torch, fp)
    log(f"bench: FP64 {args.steps} steps, {ms_step:.3f} ms/step, order-4 rate kernel {kern_ms:.3f} ms/launch")
    g64 = gamma.cpu().numpy()
    k64 = kappa.cpu().numpy()
    finite = bool(np.all(np.isfinite(k64)))

    # algorithmic work of the order-4 kernel, per formulation
    f4 = (320 * n4 + 60) * n_proc4                  # per-process form: 320 n4 + 60 FLOP per process
    f_build = 216 * n4 * n_tup                      # tuple form: phase-weighted constants, 216 n4 per tuple
    f_contract = (312 * n_groups + 60) * n_proc4    # tuple form: 39 complex MACs per group, + weights
    sec = kern_ms * 1e-3
    if variant >= 4:
        roof = {"bound": "mfma", "achieved": f_build / sec / 1e12, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "kernel": f"k_rates4b variant {variant} (tuple-batched, FP64 MFMA + FP64 VALU)",
                "work": f"216*n4 FLOP per (lambda, q', q'') tuple on FP64 MFMA, n4 = {n4}, {n_tup} tuples",
                "valu_achieved": f_contract / sec / 1e12}
    else:
        roof = {"bound": "alu", "achieved": f4 / sec / 1e12, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "kernel": f"k_rates<4,...> variant {variant} (per-process, FP64 VALU)",
                "work": f"320*n4 + 60 FLOP per process, n4 = {n4}"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["kernel_ms"] = kern_ms
    roof["per_process_form_equivalent_tflops"] = f4 / sec / 1e12
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        if tr.get("kernel_source_hash") == kernel_source_hash() and tr.get("variant") == variant:
            traffic = tr.get("hbm_bytes_per_launch")
    roof["traffic"] = traffic

    # ---- mixed-precision forward (order 4 on bf16-split MFMA + FP32 contraction)
    mixed = None
    if not args.no_mixed:
        path.precision = fp.FP_MIXED
        ms_m, kern_m, gam_m, kap_m = run_forward(path, T, args.steps, 1, 24, torch, fp)
        path.precision = fp.FP_FP64
        gm = gam_m.cpu().numpy()
        km = kap_m.cpu().numpy()
        big = np.abs(g64) > 1e-6 * np.abs(g64).max()
        rel = np.abs(gm[big] - g64[big]) / np.abs(g64[big])
        kr = (km[:, 0] + km[:, 4] + km[:, 8]) / 3
        k0 = (k64[:, 0] + k64[:, 4] + k64[:, 8]) / 3
        sec_m = kern_m * 1e-3
        mixed = {
            "value": n_proc4 / (ms_m * 1e-3), "unit": "processes/s", "ms_per_step": ms_m,
            "speedup_vs_fp64": ms_step / ms_m,
            "kappa_rel_err": float(np.max(np.abs(kr - k0) / np.abs(k0))),
            "gamma_rel_err_max": float(rel.max()), "gamma_rel_err_median": float(np.median(rel)),
            "error_reference": "the FP64 GPU path of this run (held to the oracle at 1e-10 per mode by the tests)",
            "roofline": {"bound": "mfma", "achieved": 6 * f_build / sec_m / 1e12, "peak": PEAK_BF16_TFLOPS,
                         "unit": "TFLOP/s", "frac": 6 * f_build / sec_m / 1e12 / PEAK_BF16_TFLOPS,
                         "kernel": "k_rates4m (bf16 split MFMA + FP32 VALU)", "kernel_ms": kern_m,
                         "work": "6 bf16 products per FP32-accurate product, 216*n4 FLOP per tuple",
                         "fp32_equivalent_tflops": f_build / sec_m / 1e12,
                         "valu_achieved": f_contract / sec_m / 1e12,
                         "per_process_form_equivalent_tflops": f4 / sec_m / 1e12},
        }
        log(f"bench: mixed {ms_m:.3f} ms/step (kernel {kern_m:.3f} ms), kappa rel err {mixed['kappa_rel_err']:.2e}, "
            f"Gamma rel err max {mixed['gamma_rel_err_max']:.2e}")

    # ---- backward: dkappa/dGamma, then the adjoint of both rate orders
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

    # ---- adaptive broadening: per-process width, lists enumerated with it
    adaptive = None
    if not args.no_adaptive:
        b = adaptive_broadening(cfg)
        log("bench: enumerating adaptive-width lists on the host")
        t0 = time.perf_counter()
        lists_a = host_lists(cfg, TYPES3 + TYPES4, sigma=SIGMA_FLOOR, broadening=b)
        t_enum_a = time.perf_counter() - t0
        path_a = RatePath(dict(cfg, sigma=SIGMA_FLOOR), device=0)
        if args.variant is not None:
            fp.fp_set_knob(path_a.ctx, "variant", args.variant)
        path_a.set_broadening(b)
        path_a.set_lists(lists_a)
        del lists_a
        ms_a, kern_a, gam_a, kap_a = run_forward(path_a, T, args.steps, 1, 4, torch, fp)
        adaptive = {
            "value": path_a.n_proc4 / (ms_a * 1e-3), "unit": "processes/s", "ms_per_step": ms_a,
            "processes_4ph": path_a.n_proc4, "processes_3ph": path_a.n_proc3, "kernel_ms": kern_a,
            "ns_per_process_kernel": kern_a * 1e6 / path_a.n_proc4,
            "ns_per_process_kernel_fixed_width": kern_ms * 1e6 / n_proc4,
            "factor": ADAPTIVE_FACTOR, "floor_rad_per_ps": SIGMA_FLOOR, "host_enumeration_s": round(t_enum_a, 2),
            "kappa_finite": bool(np.all(np.isfinite(kap_a.cpu().numpy()))),
        }
        path_a.close()
        log(f"bench: adaptive {ms_a:.3f} ms/step, {path_a.n_proc4} 4ph processes, kernel {kern_a:.3f} ms")

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
            "tuples_4ph": n_tup,
            "tuples_4ph_per_unit": n_unit_tup,
            "partner_groups_4ph": n_groups,
            "variant": variant,
            "step": "load_ifc(3,4) + rates3 + rates4 (Gamma3+Gamma4) + kappa_RTA",
            "host_enumeration_s": round(t_enum, 2),
        },
        "roofline": roof,
        "kappa_finite": finite,
        "mixed": mixed,
        "bwd_fwd_ratio": None if bwd is None else bwd["bwd_fwd_ratio"],
        "backward": bwd,
        "adaptive": adaptive,
    }
    if args.paper_scale:
        out["paper_scale"] = paper_scale(torch, fp, RatePath)
        out["paper_scale_mixed"] = paper_scale(torch, fp, RatePath, precision=fp.FP_MIXED)
    if args.paper_scale_adaptive:
        out["paper_scale_adaptive"] = paper_scale(torch, fp, RatePath, adaptive=True)
    if not args.no_cpu_baseline:
        log("bench: timing the oracle on the host")
        out["cpu_baseline"] = cpu_baseline(cfg, lists, args.cpu_seconds)
    path.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
