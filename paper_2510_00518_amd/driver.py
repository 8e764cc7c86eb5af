"""One pass of the rate path for a workload: sequencing of libfp calls.

This module holds no arithmetic of the method.  It uploads a workload's lists
to device tensors, loads modes and force constants, and issues, in order,
fp_load_ifc (order 3 and 4), fp_rates3, fp_rates4 (accumulating into the same
Gamma) and fp_kappa_rta, all on one stream.
"""
import json
import os

import numpy as np

from . import fp
from .synth import row_modes

TYPES3 = (fp.FP_3P, fp.FP_3M)
TYPES4 = (fp.FP_4PP, fp.FP_4PM, fp.FP_4MM)


def host_lists(cfg, types, rows=None, sigma=None, nsigma=None, keep_fraction=1.0, seed=0, n_threads=0,
               broadening=None):
    """{type: (row_mode, row_off, rec)} from the library's host enumerator
    (broadening: None or {"factor": a, "recip": (3, 3)} for the adaptive width)."""
    out = {}
    for t in types:
        out[t] = fp.enumerate_list(t, cfg, row_mode=rows, sigma=sigma, nsigma=nsigma, keep_fraction=keep_fraction,
                                   seed=seed, n_threads=n_threads, broadening=broadening)
    return out


def uneven_lists(cfg, types, lengths, pilot=1e-5, seed=0, n_threads=0):
    """Lists whose length per irreducible q1 follows `lengths` (one target per
    entry of cfg["q1"], summed over that q1's branches and the given types).
    Each q1's rows are enumerated with the (q', q'')-pair sampling fraction that
    a pilot pass at fraction `pilot` predicts, so every kept pair carries all of
    its branch combinations, as in a full list.  Returns {type: (row_mode,
    row_off, rec)} and the fraction used per q1."""
    nb = cfg["nb"]
    rows_all = np.asarray(row_modes(cfg))
    per_q = [rows_all[rows_all // nb == q] for q in np.asarray(cfg["q1"])]
    frac = []
    for k, rows in enumerate(per_q):
        n = sum(int(fp.enumerate_list(t, cfg, row_mode=rows, keep_fraction=pilot, seed=seed,
                                      n_threads=n_threads)[1][-1]) for t in types) if len(rows) else 0
        frac.append(min(1.0, float(lengths[k]) * pilot / n) if n > 0 else 1.0)
    out = {}
    for t in types:
        rms, recs, offs, base = [], [], [np.zeros(1, np.int64)], 0
        for k, rows in enumerate(per_q):
            if len(rows) == 0:
                continue
            rm, off, rec = fp.enumerate_list(t, cfg, row_mode=rows, keep_fraction=frac[k], seed=seed + 1,
                                             n_threads=n_threads)
            rms.append(rm)
            recs.append(rec)
            offs.append(off[1:] + base)
            base += int(off[-1])
        out[t] = (np.concatenate(rms).astype(np.int32), np.concatenate(offs).astype(np.int64),
                  np.concatenate(recs).astype(np.uint64))
    return out, np.asarray(frac)


class RatePath:
    def __init__(self, cfg, device=0, ctx=None, precision=fp.FP_FP64):
        """precision applies to the order-4 rates (fp.FP_FP64 or fp.FP_MIXED);
        order 3 always runs in FP64."""
        import torch
        self.torch = torch
        self.cfg = cfg
        self.precision = precision
        self.device = torch.device("cuda", device)
        self.ctx = ctx if ctx is not None else fp.fp_create(device)
        self.own_ctx = ctx is None
        fp.fp_load_modes(self.ctx, cfg["mesh"], cfg["n_atoms"], cfg["lattice"], cfg["masses"], cfg["omega"],
                         cfg["evec"], cfg["vel"], cfg["omega_floor"])
        self.n_modes = int(cfg["omega"].size)
        self.lists3, self.lists4 = [], []
        self.phi3 = self.phi4 = None
        if cfg.get("ifc3") is not None:
            self.phi3 = torch.as_tensor(cfg["ifc3"]["phi"]).to(self.device)
        if cfg.get("ifc4") is not None:
            self.phi4 = torch.as_tensor(cfg["ifc4"]["phi"]).to(self.device)
        self.fused_rows = None
        self.fused_mask = 0
        self.stream_rows = None
        self.broadening = None
        self.q1 = torch.as_tensor(np.ascontiguousarray(cfg["q1"], dtype=np.int32)).to(self.device)
        self.q1w = torch.as_tensor(np.ascontiguousarray(cfg["q1_weight"], dtype=np.float64)).to(self.device)

    def set_broadening(self, broadening):
        """None: the fixed width; {"factor": a, "recip": (3, 3)}: the adaptive
        width, with the sigma of each call as its floor."""
        fp.fp_set_broadening(self.ctx, broadening)
        self.broadening = broadening

    def close(self):
        if self.own_ctx and self.ctx is not None:
            fp.fp_destroy(self.ctx)
        self.ctx = None

    def set_lists(self, lists):
        """lists: {type: (row_mode, row_off, rec)} host arrays."""
        self.lists3, self.lists4 = [], []
        for t, (rm, off, rec) in sorted(lists.items()):
            pl = fp.PList.from_host(t, rm, off, rec, self.device)
            (self.lists3 if fp.ORDER[t] == 3 else self.lists4).append(pl)

    def set_fused(self, rows=None, type_mask=7):
        """Evaluate the order-4 rates with GPU-side enumeration (fp_rates4_fused)
        over `rows` (default: every active mode of the q1 set) instead of lists."""
        torch = self.torch
        rows = row_modes(self.cfg) if rows is None else rows
        self.fused_rows = torch.as_tensor(np.ascontiguousarray(rows, dtype=np.int32)).to(self.device)
        self.fused_mask = type_mask
        self.lists4 = []
        self.kept = torch.zeros(1, dtype=torch.int64, device=self.device)

    def set_streamed(self, type_mask=31, rows=None, chunk_records=1 << 26, n_threads=0):
        """Evaluate through fp_rates_streamed: the library enumerates the lists of
        `rows` (default: every active mode of the q1 set) chunk by chunk on the
        host, so no whole list is ever held."""
        self.stream_rows = np.ascontiguousarray(row_modes(self.cfg) if rows is None else rows, dtype=np.int32)
        self.stream_mask = int(type_mask)
        self.stream_chunk = int(chunk_records)
        self.stream_threads = int(n_threads)
        self.lists3, self.lists4 = [], []
        self.fused_rows = None
        self.stream_stats = None

    @property
    def n_proc4(self):
        return sum(pl.n_rec for pl in self.lists4)

    @property
    def n_proc3(self):
        return sum(pl.n_rec for pl in self.lists3)

    def signature(self, order, n_T):
        """Key of the autotuner cache: what the best launch depends on."""
        lists = self.lists3 if order == 3 else self.lists4
        return "|".join(str(x) for x in (order, self.precision if order == 4 else fp.FP_FP64, n_T,
                                          int(self.broadening is not None), self.cfg["nb"], self.n_modes, len(lists),
                                          sum(pl.n_rows for pl in lists), sum(pl.n_rec for pl in lists)))

    def autotune(self, T, order=4, cache=None, reps=2):
        """Pick the launch knobs for this workload with the library's autotuner.
        With `cache` (a JSON file path) a previous choice for the same workload
        signature is reused instead of measured, and new choices are stored."""
        key = self.signature(order, len(T))
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
        if key in table:
            for k in ("variant", "ppl", "blocks_per_cu"):
                fp.fp_set_knob(self.ctx, k, table[key][k])
            return table[key], []
        lists = self.lists3 if order == 3 else self.lists4
        self.load_ifc()
        prec = self.precision if order == 4 else fp.FP_FP64
        report = fp.fp_autotune(self.ctx, order, lists, T, self.cfg["sigma"], prec, reps=reps)
        best = {k: fp.fp_get_knob(self.ctx, k) for k in ("variant", "ppl", "blocks_per_cu")}
        best["ms"] = min(r["ms"] for r in report) if report else None
        if cache:
            table[key] = best
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return best, report

    def outputs(self, n_T):
        t = self.torch
        return (t.zeros((n_T, self.n_modes), dtype=t.float64, device=self.device),
                t.zeros((n_T, self.n_modes), dtype=t.float64, device=self.device))

    def load_ifc(self, phi3=None, phi4=None):
        cfg = self.cfg
        if self.fused_rows is not None and phi4 is None:
            phi4 = self.phi4
        if self.stream_rows is not None:
            if phi3 is None and self.stream_mask & 3 and self.phi3 is not None:
                phi3 = self.phi3
            if phi4 is None and self.stream_mask & 28 and self.phi4 is not None:
                phi4 = self.phi4
        if self.lists3 or phi3 is not None:
            p = self.phi3 if phi3 is None else phi3
            fp.fp_load_ifc(self.ctx, 3, cfg["ifc3"]["atoms"], cfg["ifc3"]["cells"], p)
        if self.lists4 or phi4 is not None:
            p = self.phi4 if phi4 is None else phi4
            fp.fp_load_ifc(self.ctx, 4, cfg["ifc4"]["atoms"], cfg["ifc4"]["cells"], p)

    def rates(self, T, gamma, wp=None, order=None):
        """Gamma (and WP) over every loaded list: order 3 then order 4, accumulated."""
        sigma = self.cfg["sigma"]
        first = True
        if self.lists3 and order in (None, 3):
            fp.fp_rates3(self.ctx, self.lists3, T, sigma, fp.FP_FP64, gamma, wp)
            first = False
        if self.lists4 and order in (None, 4):
            prec = self.precision if first else self.precision | fp.FP_ACCUMULATE
            fp.fp_rates4(self.ctx, self.lists4, T, sigma, prec, gamma, wp)
            first = False
        if self.fused_rows is not None and order in (None, 4):
            prec = self.precision if first else self.precision | fp.FP_ACCUMULATE
            fp.fp_rates4_fused(self.ctx, self.fused_rows, self.fused_mask, T, sigma, self.cfg["nsigma"], prec, gamma, wp,
                               n_kept=self.kept)
            first = False
        if self.stream_rows is not None:
            mask = self.stream_mask & {None: 31, 3: 3, 4: 28}[order]
            if mask:
                prec = self.precision if first else self.precision | fp.FP_ACCUMULATE
                self.stream_stats = fp.fp_rates_streamed(self.ctx, mask, self.stream_rows, T, sigma, self.cfg["nsigma"],
                                                         prec, self.stream_chunk, gamma, wp,
                                                         n_threads=self.stream_threads)
                first = False
        if first:
            gamma.zero_()
            if wp is not None:
                wp.zero_()

    def kappa(self, T, gamma, kappa_out, dkappa=None):
        fp.fp_kappa_rta(self.ctx, self.q1, self.q1w, T, gamma, kappa_out, dkappa)

    def step(self, T, gamma, kappa_out, wp=None):
        """The whole hot path once: force-constant load, 3ph + 4ph rates, kappa."""
        self.load_ifc()
        self.rates(T, gamma, wp)
        self.kappa(T, gamma, kappa_out)


def rates_autograd():
    """torch.autograd.Function classes over the library: Gamma(phi3, phi4) with the
    library's adjoint as backward, and kappa_RTA(Gamma) with dkappa/dGamma."""
    import torch

    class Rates(torch.autograd.Function):
        @staticmethod
        def forward(ctx, phi3, phi4, path, T):
            gamma = torch.zeros((len(T), path.n_modes), dtype=torch.float64, device=path.device)
            path.load_ifc(phi3=phi3.detach().contiguous() if phi3 is not None else None,
                          phi4=phi4.detach().contiguous() if phi4 is not None else None)
            path.rates(T, gamma)
            ctx.path, ctx.T = path, T
            ctx.has3, ctx.has4 = phi3 is not None, phi4 is not None
            ctx.save_for_backward(phi3 if phi3 is not None else torch.empty(0),
                                  phi4 if phi4 is not None else torch.empty(0))
            return gamma

        @staticmethod
        def backward(ctx, grad_gamma):
            path = ctx.path
            phi3, phi4 = ctx.saved_tensors
            d3 = torch.zeros_like(phi3) if ctx.has3 else None
            d4 = torch.zeros_like(phi4) if ctx.has4 else None
            path.load_ifc(phi3=phi3.detach() if ctx.has3 else None, phi4=phi4.detach() if ctx.has4 else None)
            fp.fp_rates_backward(path.ctx, path.lists3 + path.lists4, ctx.T, path.cfg["sigma"],
                                 grad_gamma.contiguous(), d3 if path.lists3 else None, d4 if path.lists4 else None,
                                 precision=path.precision)
            if d3 is not None and not path.lists3:
                d3.zero_()
            if d4 is not None and not path.lists4:
                d4.zero_()
            return d3, d4, None, None

    class KappaRTA(torch.autograd.Function):
        @staticmethod
        def forward(ctx, gamma, path, T):
            kap = torch.zeros((len(T), 9), dtype=torch.float64, device=path.device)
            dk = torch.zeros_like(gamma)
            path.kappa(T, gamma.contiguous(), kap, dk)
            ctx.save_for_backward(dk)
            return kap[:, [0, 4, 8]].sum(dim=1) / 3.0

        @staticmethod
        def backward(ctx, grad_k):
            (dk,) = ctx.saved_tensors
            return grad_k[:, None] * dk, None, None

    return Rates, KappaRTA
