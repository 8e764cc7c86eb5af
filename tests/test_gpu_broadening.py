"""Adaptive broadening on the GPU: the per-process width
sigma_p = max(a sigma0_p, sigma) from the partners' group velocities.

Parity: on small meshes (one anisotropic, with reciprocal vectors tilted off any
symmetry) the rates over the oracle's own adaptive enumeration equal the
oracle's list-mode sums per mode within 1e-10 for every FP64 contraction form,
within the mixed-precision bar (2e-5 per mode) for FP_MIXED, and the adjoint
equals the oracle's gradient within 1e-10.  At the 8^3 workload with the
paper's scale a = 0.1, the library's host lists of sampled modes equal the
oracle's enumeration exactly and their rates, from the launch over every row,
equal the oracle's sums within 1e-10.
"""
import sys

import numpy as np
import pytest

import knob_util
import oracle
from paper_2510_00518_amd import fp
from paper_2510_00518_amd.synth import SIGMA_FLOOR, adaptive_broadening, make_config, row_modes, small_config

pytestmark = pytest.mark.gpu

TYPES3 = (fp.FP_3P, fp.FP_3M)
TYPES4 = (fp.FP_4PP, fp.FP_4PM, fp.FP_4MM)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    h = fp.fp_create(0)
    yield h
    fp.fp_destroy(h)


def tilted(cfg):
    rng = np.random.default_rng(99)
    return {"factor": 0.5, "recip": cfg["recip"] + rng.uniform(-0.3, 0.3, size=(3, 3))}


def oracle_lists(S, types, rows, floor, nsigma):
    out = {}
    for t in types:
        recs = [S.enumerate_row(t, int(g), floor, nsigma) for g in rows]
        off = np.concatenate([[0], np.cumsum([len(r) for r in recs])]).astype(np.int64)
        rec = np.concatenate(recs).astype(np.uint64) if off[-1] else np.zeros(0, np.uint64)
        out[t] = (np.asarray(rows, dtype=np.int32), off, rec)
    return out


def oracle_mode_rates(S, n_modes, lists, T, floor):
    gam = np.zeros((len(T), n_modes))
    wp = np.zeros((len(T), n_modes))
    for t, (rm, off, rec) in lists.items():
        if off[-1] == 0:
            continue
        g, w, _, _ = S.rates(t, rm, T, floor, row_off=off, rec=rec)
        gam[:, rm] += g.T
        wp[:, rm] += w.T
    return gam, wp


def gpu_rates(ctx, cfg, b, lists, T, floor, variant=knob_util.DEFAULT_VARIANT, precision=fp.FP_FP64):
    import torch
    from paper_2510_00518_amd.driver import RatePath
    with knob_util.knobs(ctx, variant=variant):
        p = RatePath(dict(cfg, sigma=floor), ctx=ctx, precision=precision)
        p.set_broadening(b)
        p.set_lists(lists)
        gam, wp = p.outputs(len(T))
        p.load_ifc()
        p.rates(T, gam, wp)
        fp.fp_check(ctx)
        torch.cuda.synchronize()
    return gam.cpu().numpy(), wp.cpu().numpy()


def assert_parity(got, want, what, rtol=1e-10):
    floor = 1e-12 * np.abs(want).max()
    err = np.abs(got - want) / np.maximum(np.abs(want), floor)
    say(f"  {what}: max rel err {err.max():.2e}, median {np.median(err):.1e}")
    assert err.max() <= rtol, what


CASES = [((2, 3, 4), 0.05, 1), (4, 0.2, 9), (3, 0.1, 2)]


@pytest.mark.parametrize("mesh,floor,stride", CASES)
def test_adaptive_three_phonon(ctx, mesh, floor, stride):
    cfg = small_config(mesh)
    b = tilted(cfg)
    S = oracle.System(cfg, broadening=b)
    rows = row_modes(cfg)[::stride]
    lists = oracle_lists(S, TYPES3, rows, floor, cfg["nsigma"])
    say(f"3ph adaptive {mesh}: records", {t: int(v[1][-1]) for t, v in lists.items()})
    T = [300.0, 900.0]
    g, w = gpu_rates(ctx, cfg, b, lists, T, floor)
    go, wo = oracle_mode_rates(S, cfg["omega"].size, lists, T, floor)
    assert_parity(g, go, "Gamma3 adaptive")
    assert_parity(w, wo, "WP3 adaptive")


_CACHE4 = {}


def four_phonon_case(mesh, floor, stride):
    """Oracle lists and rates of one case, shared by the variants (the +- lists,
    the longest, over a third of the rows)."""
    key = (mesh, floor, stride)
    if key not in _CACHE4:
        cfg = small_config(mesh)
        b = tilted(cfg)
        S = oracle.System(cfg, broadening=b)
        rows = row_modes(cfg)[::stride * 3]
        lists = oracle_lists(S, (fp.FP_4PP, fp.FP_4MM), rows, floor, cfg["nsigma"])
        lists.update(oracle_lists(S, (fp.FP_4PM,), rows[::3], floor, cfg["nsigma"]))
        T = [300.0, 1200.0]
        _CACHE4[key] = (cfg, b, lists, T, oracle_mode_rates(S, cfg["omega"].size, lists, T, floor))
    return _CACHE4[key]


@pytest.mark.parametrize("variant", [0, 1, 4, 5, 6, 7])
@pytest.mark.parametrize("mesh,floor,stride", CASES)
def test_adaptive_four_phonon(ctx, mesh, floor, stride, variant):
    cfg, b, lists, T, (go, wo) = four_phonon_case(mesh, floor, stride)
    say(f"4ph adaptive {mesh} variant {variant}: records", {t: int(v[1][-1]) for t, v in lists.items()})
    g, w = gpu_rates(ctx, cfg, b, lists, T, floor, variant=variant)
    assert_parity(g, go, f"Gamma4 adaptive variant {variant}")
    assert_parity(w, wo, f"WP4 adaptive variant {variant}")


def test_adaptive_mixed_precision(ctx):
    cfg = small_config(4)
    b = tilted(cfg)
    S = oracle.System(cfg, broadening=b)
    rows = row_modes(cfg)[::13]
    lists = oracle_lists(S, TYPES4, rows, 0.2, cfg["nsigma"])
    g, _ = gpu_rates(ctx, cfg, b, lists, [300.0], 0.2, precision=fp.FP_MIXED)
    go, _ = oracle_mode_rates(S, cfg["omega"].size, lists, [300.0], 0.2)
    assert_parity(g, go, "Gamma4 adaptive, mixed precision", rtol=2e-5)


def test_adaptive_backward(ctx):
    import torch
    from paper_2510_00518_amd.driver import RatePath
    cfg = small_config((2, 3, 4))
    b = tilted(cfg)
    floor = 0.05
    S = oracle.System(cfg, broadening=b)
    rows = row_modes(cfg)[::2]
    lists = oracle_lists(S, (fp.FP_3M, fp.FP_4PP, fp.FP_4PM), rows, floor, cfg["nsigma"])
    T = [300.0, 900.0]
    dLdG = np.random.default_rng(6).uniform(0.5, 1.5, size=(len(T), cfg["omega"].size))
    p = RatePath(dict(cfg, sigma=floor), ctx=ctx)
    p.set_broadening(b)
    p.set_lists(lists)
    p.load_ifc(phi3=p.phi3, phi4=p.phi4)
    d3 = torch.zeros_like(p.phi3)
    d4 = torch.zeros_like(p.phi4)
    fp.fp_rates_backward(ctx, p.lists3 + p.lists4, T, floor, torch.as_tensor(dLdG).cuda(), d3, d4)
    fp.fp_check(ctx)
    torch.cuda.synchronize()
    for m, got in ((3, d3.cpu().numpy()), (4, d4.cpu().numpy())):
        want = np.zeros_like(got)
        for t, (rm, off, rec) in lists.items():
            if oracle.ORDER[t] == m and off[-1]:
                S.grad(t, rm, T, floor, off, rec, dLdG[:, rm].T, out=want)
        fl = 1e-5 * np.abs(want).max()  # rounding-noise entries sit near 1e-16 of the largest
        err = np.abs(got - want) / np.maximum(np.abs(want), fl)
        say(f"  adaptive dPhi{m}: max rel err {err.max():.2e}")
        assert err.max() <= 1e-10


def test_adaptive_errors_and_reset(ctx):
    import torch
    from paper_2510_00518_amd.driver import RatePath
    cfg = small_config(3)
    p = RatePath(cfg, ctx=ctx)
    for bad in ({"factor": -1.0, "recip": cfg["recip"]}, {"factor": 0.1, "recip": np.full((3, 3), np.inf)}):
        with pytest.raises(fp.FpError) as e:
            p.set_broadening(bad)
        assert e.value.status == fp.FP_ERR_ARG
    p.set_broadening(tilted(cfg))
    p.load_ifc(phi4=p.phi4)
    rows = torch.as_tensor(np.asarray(row_modes(cfg)[:2], np.int32)).cuda()
    gam = torch.zeros((1, p.n_modes), dtype=torch.float64, device="cuda")
    # without velocities there is nothing to take the width from
    fp.fp_load_modes(ctx, cfg["mesh"], cfg["n_atoms"], cfg["lattice"], cfg["masses"], cfg["omega"], cfg["evec"],
                     None, cfg["omega_floor"])
    with pytest.raises(fp.FpError) as e:
        fp.fp_set_broadening(ctx, tilted(cfg))
    assert e.value.status == fp.FP_ERR_STATE
    # a new load of the modes returns to the fixed width
    p = RatePath(cfg, ctx=ctx)
    p.load_ifc(phi4=p.phi4)
    fp.fp_rates4_fused(ctx, rows, 7, [300.0], cfg["sigma"], 3.0, fp.FP_FP64, gam)
    fp.fp_check(ctx)
    torch.cuda.synchronize()
    assert np.all(np.isfinite(gam.cpu().numpy()))


@pytest.mark.slow
def test_adaptive_fcc8_full_size_sampled(ctx):
    """The 8^3 four-phonon workload with a = 0.1 and a 0.01 THz floor, every row
    in the default launch; two sampled modes against the oracle."""
    import torch
    from paper_2510_00518_amd.driver import RatePath, host_lists
    assert fp.fp_get_knob(ctx, "variant") == knob_util.DEFAULT_VARIANT
    cfg = make_config("fcc8_4ph")
    b = adaptive_broadening(cfg)
    say("fcc8_4ph adaptive: enumerating (library, host)")
    lists = host_lists(cfg, TYPES4, sigma=SIGMA_FLOOR, broadening=b)
    p = RatePath(dict(cfg, sigma=SIGMA_FLOOR), ctx=ctx)
    p.set_broadening(b)
    p.set_lists(lists)
    say("fcc8_4ph adaptive: records", p.n_proc4)
    gam, _ = p.outputs(1)
    p.load_ifc()
    p.rates([300.0], gam)
    fp.fp_check(ctx)
    torch.cuda.synchronize()
    g = gam.cpu().numpy()[0]
    rows = lists[fp.FP_4PM][0]
    lens = np.diff(lists[fp.FP_4PM][1])
    rng = np.random.default_rng(251000518 + 8)
    short = np.argsort(lens)[: len(lens) // 2]
    pick = rows[rng.choice(short, size=2, replace=False)]
    S = oracle.System(cfg, broadening=b)
    for gm in pick:
        total = 0.0
        for t in TYPES4:
            rm, off, rec = lists[t]
            r = int(np.nonzero(rm == gm)[0][0])
            mine = np.sort(rec[off[r]:off[r + 1]])
            ref = S.enumerate_row(t, int(gm), SIGMA_FLOOR, cfg["nsigma"])
            np.testing.assert_array_equal(mine, ref)
            if len(ref):
                go, _, _, _ = S.rates(t, [gm], [300.0], SIGMA_FLOOR, row_off=np.array([0, len(ref)]), rec=ref)
                total += go[0, 0]
        say(f"fcc8_4ph adaptive mode {gm}: gpu {g[gm]:.12e} oracle {total:.12e}")
        assert g[gm] == pytest.approx(total, rel=1e-10)
