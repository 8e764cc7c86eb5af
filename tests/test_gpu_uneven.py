"""The uneven 8-atom workload in one persistent, autotuned launch.

8-atom cubic diamond cell (24 branches), 10^3 mesh, 56 irreducible q1 whose
four-phonon list lengths are drawn log-uniform in [1e4, 1e7] (about 7e7
records in all), 198 quartic terms in 80 partner-atom groups.  The lists of all
q1 go to one fp_rates4 call (one persistent launch); the library's autotuner
picks the contraction form and work distribution.

Parity: the rates of sampled rows (short lists of several q1) against the
oracle's list-mode sums over the same records, per mode within 1e-10; the
chosen launch agrees with the per-process FP64 form on every mode within 1e-12;
the mixed-precision path is held to the mixed bars (per mode 2e-5 relative,
kappa_RTA 1e-5) against FP64.
"""
import sys

import numpy as np
import pytest

import knob_util
import oracle
from paper_2510_00518_amd import fp
from paper_2510_00518_amd.synth import make_config

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def workload():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2510_00518_amd.driver import TYPES4, RatePath, uneven_lists
    cfg = make_config("sc10_4ph_uneven")
    lists, frac = uneven_lists(cfg, TYPES4, cfg["q1_lengths"])
    say("sc10_4ph_uneven: records", {t: int(v[1][-1]) for t, v in lists.items()},
        "pair fractions", float(frac.min()), "..", float(frac.max()))
    ctx = fp.fp_create(0)
    p = RatePath(cfg, ctx=ctx)
    p.set_lists(lists)
    yield cfg, lists, p
    p.close()
    fp.fp_destroy(ctx)


def rates(p, T):
    import torch
    gam, _ = p.outputs(len(T))
    p.load_ifc()
    p.rates(T, gam)
    fp.fp_check(p.ctx)
    torch.cuda.synchronize()
    return gam.cpu().numpy()


def test_uneven_autotuned_launch_matches_oracle(workload, tmp_path):
    cfg, lists, p = workload
    T = [300.0]
    p.precision = fp.FP_FP64
    best, report = p.autotune(T, cache=str(tmp_path / "tune.json"), reps=1)
    for r in report:
        say(f"  candidate variant={r['variant']} ppl={r['ppl']} blocks/CU={r['blocks_per_cu']}: {r['ms']:.2f} ms")
    say("autotuner choice", best)
    assert len(report) >= 10
    assert best["ms"] == min(r["ms"] for r in report)
    # a second call with the cache reuses the choice without measuring
    again, rep2 = p.autotune(T, cache=str(tmp_path / "tune.json"))
    assert rep2 == [] and all(again[k] == best[k] for k in ("variant", "ppl", "blocks_per_cu"))
    g = rates(p, T)[0]

    # every mode: the chosen launch against the per-process FP64 form
    with knob_util.knobs(p.ctx, variant=1, ppl=2, blocks_per_cu=0):
        g1 = rates(p, T)[0]
    scale = np.abs(g1).max()
    np.testing.assert_allclose(g, g1, rtol=1e-12, atol=1e-12 * scale)

    # sampled rows against the oracle: the shortest non-empty +- rows of three q1
    S = oracle.System(cfg)
    rm, off, _ = lists[fp.FP_4PM]
    lens = np.diff(off)
    order = [r for r in np.argsort(lens) if lens[r] > 0]
    nb = cfg["nb"]
    picked, seen = [], set()
    for r in order:
        q = int(rm[r]) // nb
        if q not in seen:
            seen.add(q)
            picked.append(int(rm[r]))
        if len(picked) == 3:
            break
    for gm in picked:
        want = 0.0
        n_rec = 0
        for t, (rmt, offt, rect) in lists.items():
            idx = np.nonzero(rmt == gm)[0]
            if len(idx) == 0:
                continue
            r = int(idx[0])
            sub = rect[offt[r]:offt[r + 1]]
            n_rec += len(sub)
            if len(sub):
                go, _, _, _ = S.rates(t, rmt[r:r + 1], T, cfg["sigma"], row_off=np.array([0, len(sub)]), rec=sub)
                want += float(go[0, 0])
        err = abs(g[gm] - want) / max(abs(want), 1e-300)
        say(f"row g={gm}: {n_rec} records, GPU {g[gm]:.15e} oracle {want:.15e} rel {err:.2e}")
        assert err <= 1e-10 or abs(g[gm] - want) <= 1e-12 * scale


def test_uneven_mixed_precision(workload):
    import torch
    cfg, lists, p = workload
    T = [300.0]
    out = {}
    for name, prec in (("fp64", fp.FP_FP64), ("mixed", fp.FP_MIXED)):
        p.precision = prec
        g = rates(p, T)
        gt = torch.as_tensor(g).cuda()
        kap = torch.zeros((1, 9), dtype=torch.float64, device="cuda")
        p.kappa(T, gt, kap)
        torch.cuda.synchronize()
        k = kap.cpu().numpy()[0]
        out[name] = (g[0], (k[0] + k[4] + k[8]) / 3)
    p.precision = fp.FP_FP64
    g64, k64 = out["fp64"]
    gmx, kmx = out["mixed"]
    scale = np.abs(g64).max()
    big = np.abs(g64) > 1e-6 * scale
    rel = np.abs(gmx[big] - g64[big]) / np.abs(g64[big])
    kerr = abs(kmx - k64) / abs(k64)
    say(f"uneven mixed vs FP64: per-mode rel max {rel.max():.3e} median {np.median(rel):.3e}; kappa rel {kerr:.3e}")
    assert rel.max() <= 2e-5
    assert np.abs(gmx[~big] - g64[~big]).max() <= 1e-6 * scale
    assert kerr <= 1e-5
