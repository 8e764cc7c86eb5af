"""GPU parity: libfp's HIP path against the FP64 oracle, per mode.

Inputs of the oracle never come from the HIP path: the small cases evaluate
lists produced by the oracle's own brute-force enumeration on both sides; the
full-size case (the benchmark's 8^3 four-phonon workload in the benchmark's
launch configuration) checks the library's lists of sampled modes against the
oracle's enumeration and their rates against the oracle's list-mode sums.

Tolerance: per-mode relative error <= 1e-10 (FP64 bar).  Modes whose rate is
at the rounding level of the largest one (symmetry-forbidden processes, below
1e-12 of the maximum) are compared with that absolute floor instead.
"""
import sys

import numpy as np
import pytest

import knob_util
import oracle
from paper_2510_00518_amd import fp
from paper_2510_00518_amd.synth import make_config, row_modes, small_config

pytestmark = pytest.mark.gpu

RTOL = 1e-10


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


def oracle_lists(cfg, types, rows, sigma):
    S = oracle.System(cfg)
    out = {}
    for t in types:
        recs = [S.enumerate_row(t, g, sigma, cfg["nsigma"]) for g in rows]
        off = np.concatenate([[0], np.cumsum([len(r) for r in recs])]).astype(np.int64)
        rec = np.concatenate(recs).astype(np.uint64) if off[-1] else np.zeros(0, np.uint64)
        out[t] = (np.asarray(rows, dtype=np.int32), off, rec)
    return out


def oracle_mode_rates(cfg, lists, T, sigma):
    S = oracle.System(cfg)
    n = cfg["omega"].size
    gam = np.zeros((len(T), n))
    wp = np.zeros((len(T), n))
    for t, (rm, off, rec) in lists.items():
        if off[-1] == 0:
            continue
        g, w, _, _ = S.rates(t, rm, T, sigma, row_off=off, rec=rec)
        gam[:, rm] += g.T
        wp[:, rm] += w.T
    return gam, wp


def gpu_rates(ctx, cfg, lists, T, sigma=None, knobs=None):
    import torch
    from paper_2510_00518_amd.driver import RatePath
    cfg = dict(cfg)
    if sigma is not None:
        cfg["sigma"] = sigma
    with knob_util.knobs(ctx, **(knobs or {})):
        p = RatePath(cfg, ctx=ctx)
        p.set_lists(lists)
        gam, wp = p.outputs(len(T))
        p.load_ifc()
        p.rates(T, gam, wp)
        fp.fp_check(ctx)
        torch.cuda.synchronize()
    return gam.cpu().numpy(), wp.cpu().numpy()


def assert_parity(got, want, what, rtol=RTOL):
    floor = 1e-12 * np.abs(want).max()
    err = np.abs(got - want) / np.maximum(np.abs(want), floor)
    i = np.unravel_index(int(err.argmax()), err.shape)
    say(f"  {what}: max rel err {err.max():.2e} at {i} (value {want[i]:.6e}), median {np.median(err):.1e}")
    assert err.max() <= rtol, what


def test_fcc4_three_phonon(ctx):
    cfg = make_config("fcc4_3ph")
    rows = row_modes(cfg)
    say("fcc4_3ph: rows", len(rows))
    lists = oracle_lists(cfg, (fp.FP_3P, fp.FP_3M), rows, cfg["sigma"])
    for T in ([300.0], [300.0, 600.0, 900.0]):
        g, w = gpu_rates(ctx, cfg, lists, T)
        go, wo = oracle_mode_rates(cfg, lists, T, cfg["sigma"])
        assert_parity(g, go, f"fcc4_3ph Gamma3 T={T}")
        assert_parity(w, wo, f"fcc4_3ph WP3 T={T}")
        inactive = np.setdiff1d(np.arange(cfg["omega"].size), rows)
        assert np.all(g[:, inactive] == 0.0)


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("mesh,sigma,stride", [(4, None, 5), (4, 10.0, 17), (3, 4.0, 3)])
def test_four_phonon_small(ctx, mesh, sigma, stride, variant):
    cfg = small_config(mesh)
    sig = cfg["sigma"] if sigma is None else sigma
    rows = row_modes(cfg)[::stride]
    lists = oracle_lists(cfg, (fp.FP_4PP, fp.FP_4PM, fp.FP_4MM), rows, sig)
    say(f"4ph {mesh}^3 sigma={sig}: records", {t: int(v[1][-1]) for t, v in lists.items()})
    T = [300.0, 1200.0]
    g, w = gpu_rates(ctx, cfg, lists, T, sigma=sig, knobs={"variant": variant})
    go, wo = oracle_mode_rates(cfg, lists, T, sig)
    assert_parity(g, go, f"Gamma4 {mesh}^3")
    assert_parity(w, wo, f"WP4 {mesh}^3")


def test_launch_knobs_do_not_change_results(ctx):
    cfg = small_config(4)
    rows = row_modes(cfg)[::9]
    lists = oracle_lists(cfg, (fp.FP_4PM, fp.FP_4MM), rows, 6.0)
    go, _ = oracle_mode_rates(cfg, lists, [300.0], 6.0)
    ref = None
    for variant, ppl, bpc in ((0, 1, 1), (0, 2, 0), (1, 3, 1), (2, 3, 0), (3, 8, 2), (2, 64, 1), (4, 5, 1), (4, 1, 0), (5, 3, 0), (5, 1, 1), (7, 2, 0), (1, 2, 0)):
        g, _ = gpu_rates(ctx, cfg, lists, [300.0], sigma=6.0,
                         knobs={"variant": variant, "ppl": ppl, "blocks_per_cu": bpc})
        assert_parity(g, go, f"variant={variant} ppl={ppl} blocks/CU={bpc}")
        if ref is not None:
            np.testing.assert_allclose(g, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
        ref = g


@pytest.mark.parametrize("order", ["enumerator", "shuffled"])
def test_tuple_batched_any_record_order(ctx, order):
    """The tuple-batched form finds (q', q'') tuples from consecutive records, so
    it must give the same rates whether a row's records of one tuple are
    contiguous (the enumerator's order) or scattered."""
    from paper_2510_00518_amd.driver import host_lists
    cfg = small_config(4)
    rows = row_modes(cfg)[::7]
    lists = host_lists(cfg, (fp.FP_4PP, fp.FP_4PM, fp.FP_4MM), rows=rows, sigma=6.0)
    if order == "shuffled":
        rng = np.random.default_rng(7)
        for t, (rm, off, rec) in lists.items():
            rec = rec.copy()
            for r in range(len(rm)):
                rec[off[r]:off[r + 1]] = rng.permutation(rec[off[r]:off[r + 1]])
            lists[t] = (rm, off, rec)
    say(f"tuple-batched, {order} records:", {t: int(v[1][-1]) for t, v in lists.items()})
    go, wo = oracle_mode_rates(cfg, lists, [300.0], 6.0)
    g, w = gpu_rates(ctx, cfg, lists, [300.0], sigma=6.0, knobs={"variant": 4})
    assert_parity(g, go, f"Gamma4 variant 4, {order}")
    assert_parity(w, wo, f"WP4 variant 4, {order}")


@pytest.mark.parametrize("variant", [0, 2, 4, 5])
def test_eight_atom_cell(ctx, variant):
    cfg = small_config(2, n3=0, n4=200, cell="conv")
    rows = row_modes(cfg)[::13]
    lists = oracle_lists(cfg, (fp.FP_4PM,), rows, cfg["sigma"])
    say("8-atom 2^3: records", int(lists[fp.FP_4PM][1][-1]), "groups of terms over 8 atoms")
    T = [300.0, 600.0, 700.0, 800.0, 900.0]  # five temperatures: the 8-wide temperature variant
    g, w = gpu_rates(ctx, cfg, lists, T, knobs={"variant": variant})
    go, wo = oracle_mode_rates(cfg, lists, T, cfg["sigma"])
    assert_parity(g, go, "Gamma4 8-atom")
    assert_parity(w, wo, "WP4 8-atom")


def test_edge_cases(ctx):
    import torch
    from paper_2510_00518_amd.driver import RatePath
    cfg = small_config(3)
    S = oracle.System(cfg)
    # four rows whose +- lists hold at least two records each
    rows = np.array([g for g in row_modes(cfg) if len(S.enumerate_row(fp.FP_4PM, g, cfg["sigma"])) >= 2][:4],
                    dtype=np.int32)
    dev = torch.device("cuda", 0)
    p = RatePath(cfg, ctx=ctx)
    p.load_ifc(phi3=p.phi3, phi4=p.phi4)
    gam, wp = p.outputs(1)
    # no lists at all: outputs are cleared
    gam.fill_(7.0)
    fp.fp_rates4(ctx, [], [300.0], cfg["sigma"], fp.FP_FP64, gam, wp)
    torch.cuda.synchronize()
    assert float(gam.abs().max()) == 0.0
    # rows without records, and a single-record row
    lists = oracle_lists(cfg, (fp.FP_4PM,), rows, cfg["sigma"])
    rm, off, rec = lists[fp.FP_4PM]
    own = rec[int(off[1]):int(off[1]) + 1]  # first record of the second row's own list
    one = fp.PList.from_host(fp.FP_4PM, rm[:2], np.array([0, 0, 1]), own, dev)
    empty = fp.PList.from_host(fp.FP_4MM, rm[:2], np.array([0, 0, 0]), np.zeros(0, np.uint64), dev)
    fp.fp_rates4(ctx, [empty, one], [300.0], cfg["sigma"], fp.FP_FP64, gam, wp)
    fp.fp_check(ctx)
    g1 = gam.cpu().numpy()
    go, wo, _, _ = S.rates(fp.FP_4PM, rm[1:2], [300.0], cfg["sigma"], row_off=np.array([0, 1]), rec=own)
    assert g1[0, rm[1]] == pytest.approx(go[0, 0], rel=RTOL)
    assert np.count_nonzero(g1) == 1
    # a record outside the mesh is skipped and reported; the others still count
    bad_rec = rec[: int(off[2])].copy()
    bad_rec[0] = np.uint64(0xFFFFFF)
    bad = fp.PList.from_host(fp.FP_4PM, rm[:2], off[:3], bad_rec, dev)
    fp.fp_rates4(ctx, [bad], [300.0], cfg["sigma"], fp.FP_FP64, gam, wp)
    with pytest.raises(fp.FpError) as e:
        fp.fp_check(ctx)
    assert e.value.status == fp.FP_ERR_RANGE
    fp.fp_check(ctx)  # the flag was cleared
    gb = gam.cpu().numpy()
    ref, _, _, _ = S.rates(fp.FP_4PM, rm[:2], [300.0], cfg["sigma"], row_off=np.array([0, off[1] - 1, off[2] - 1]),
                           rec=rec[1:int(off[2])])
    np.testing.assert_allclose(gb[0, rm[:2]], ref[:, 0], rtol=RTOL)
    # a row naming a mode outside the mesh, and a decreasing row offset
    for bad_mode, bad_off in ((10 ** 6, off[:2]), (int(rm[0]), np.array([int(off[1]), 0]))):
        badrow = fp.PList.from_host(fp.FP_4PM, np.array([bad_mode], np.int32), bad_off, rec[: int(off[1])], dev)
        fp.fp_rates4(ctx, [badrow], [300.0], cfg["sigma"], fp.FP_FP64, gam, wp)
        with pytest.raises(fp.FpError):
            fp.fp_check(ctx)
        assert float(gam.abs().max()) == 0.0
    # argument errors are synchronous
    with pytest.raises(fp.FpError) as e:
        fp.fp_rates4(ctx, [one], [], cfg["sigma"], fp.FP_FP64, gam, wp)
    assert e.value.status == fp.FP_ERR_ARG
    with pytest.raises(fp.FpError) as e:
        fp.fp_rates3(ctx, [one], [300.0], cfg["sigma"], fp.FP_FP64, gam, wp)
    assert e.value.status == fp.FP_ERR_ARG
    with pytest.raises(fp.FpError) as e:
        fp.fp_rates4(ctx, [one], [300.0], cfg["sigma"], fp.FP_MIXED + 7, gam, wp)
    assert e.value.status == fp.FP_ERR_ARG
    torch.cuda.synchronize()


def test_kappa(ctx):
    import torch
    from paper_2510_00518_amd.driver import RatePath
    cfg = make_config("fcc8_4ph")
    S_gamma = np.random.default_rng(1).uniform(0.01, 0.5, size=(2, cfg["omega"].size))
    T = [300.0, 700.0]
    p = RatePath(cfg, ctx=ctx)
    gam = torch.as_tensor(S_gamma).cuda()
    kap = torch.zeros((2, 9), dtype=torch.float64, device="cuda")
    dk = torch.zeros_like(gam)
    p.kappa(T, gam, kap, dk)
    torch.cuda.synchronize()
    k = kap.cpu().numpy()
    for it, TT in enumerate(T):
        ko = oracle.kappa(cfg, S_gamma[it], TT).reshape(-1)
        np.testing.assert_allclose(k[it], ko, rtol=1e-12, atol=1e-12 * np.abs(ko).max())
        # d(tr kappa / 3)/dGamma against a central difference of the oracle
        g = int(cfg["q1"][3]) * cfg["nb"] + 4
        h = 1e-6 * S_gamma[it, g]
        gp, gm = S_gamma[it].copy(), S_gamma[it].copy()
        gp[g] += h
        gm[g] -= h
        fd = (np.trace(oracle.kappa(cfg, gp, TT)) - np.trace(oracle.kappa(cfg, gm, TT))) / (6 * h)
        assert float(dk[it, g]) == pytest.approx(fd, rel=1e-6)


@pytest.mark.slow
def test_fcc8_4ph_full_size_sampled(ctx):
    """The 8^3 four-phonon workload at full size, in the benchmark's launch
    configuration; sampled modes checked against the oracle one by one."""
    import torch
    from paper_2510_00518_amd.driver import TYPES3, TYPES4, RatePath, host_lists
    assert fp.fp_get_knob(ctx, "variant") == knob_util.DEFAULT_VARIANT
    cfg = make_config("fcc8_4ph")
    say("fcc8_4ph: enumerating (library, host)")
    lists = host_lists(cfg, TYPES3 + TYPES4)
    p = RatePath(cfg, ctx=ctx)
    p.set_lists(lists)
    say("fcc8_4ph: records 4ph", p.n_proc4, "3ph", p.n_proc3)
    gam, wp = p.outputs(1)
    p.load_ifc()
    p.rates([300.0], gam, wp)
    fp.fp_check(ctx)
    torch.cuda.synchronize()
    g = gam.cpu().numpy()[0]
    rows = lists[fp.FP_4PM][0]
    lens = np.diff(lists[fp.FP_4PM][1])
    rng = np.random.default_rng(251000518 + 5)
    # two sampled modes among the shorter half of the rows (the oracle sums them one record at a time)
    short = np.argsort(lens)[: len(lens) // 2]
    pick = rows[rng.choice(short, size=2, replace=False)]
    S = oracle.System(cfg)
    for gm in pick:
        total = 0.0
        for t in TYPES3 + TYPES4:
            rm, off, rec = lists[t]
            r = int(np.nonzero(rm == gm)[0][0])
            mine = np.sort(rec[off[r]:off[r + 1]])
            ref = S.enumerate_row(t, gm, cfg["sigma"], cfg["nsigma"])
            np.testing.assert_array_equal(mine, ref)
            if len(ref):
                go, _, _, _ = S.rates(t, [gm], [300.0], cfg["sigma"], row_off=np.array([0, len(ref)]), rec=ref)
                total += go[0, 0]
        say(f"fcc8_4ph mode {gm}: gpu {g[gm]:.12e} oracle {total:.12e}")
        assert g[gm] == pytest.approx(total, rel=RTOL)
