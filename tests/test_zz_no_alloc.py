"""fp_rates4_noalloc (every per-call table in the library's fixed workspace)
against fp_rates4 on the same inputs: identical kernels, so identical results
bit for bit, on two calls in a row, the second with a smaller input (fewer
rows and records, which must not see the first call's leftovers), FP64 and
mixed precision; and a call whose tables exceed the workspace is refused."""
import sys

import numpy as np
import pytest

from paper_2510_00518_amd import fp
from paper_2510_00518_amd.synth import make_config, row_modes, small_config

pytestmark = pytest.mark.gpu

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


def both(ctx, cfg, rows, T, precision):
    import torch
    from paper_2510_00518_amd.driver import RatePath, host_lists
    lists = host_lists(cfg, TYPES4, rows=rows, sigma=6.0)
    p = RatePath(cfg, ctx=ctx, precision=precision)
    p.set_lists(lists)
    p.load_ifc()
    out = []
    for fn in (fp.fp_rates4, fp.fp_rates4_noalloc):
        gam, wp = p.outputs(len(T))
        gam.fill_(3.0)  # overwritten, not added to
        fn(ctx, p.lists4, T, 6.0, precision, gam, wp)
        fp.fp_check(ctx)
        torch.cuda.synchronize()
        out.append((gam.cpu().numpy(), wp.cpu().numpy()))
    say(f"  {len(rows)} rows, {p.n_proc4} records, precision {precision}")
    return out, p.n_proc4


@pytest.mark.parametrize("precision", [fp.FP_FP64, fp.FP_MIXED])
def test_noalloc_matches_rates4(ctx, precision):
    cfg = small_config(4)
    rows_all = row_modes(cfg)
    T = [300.0, 900.0]
    sizes = []
    for rows in (rows_all[::3], rows_all[::11]):  # the second call is smaller
        ((g, w), (gn, wn)), n = both(ctx, cfg, rows, T, precision)
        sizes.append(n)
        assert np.abs(g).max() > 0
        np.testing.assert_array_equal(gn, g)
        np.testing.assert_array_equal(wn, w)
    assert sizes[1] < sizes[0]


def test_noalloc_refuses_beyond_workspace(ctx):
    import torch
    from paper_2510_00518_amd.driver import RatePath
    cfg = make_config("fcc8_4ph")
    p = RatePath(cfg, ctx=ctx)
    p.load_ifc(phi4=p.phi4)
    dev = torch.device("cuda", 0)
    rows = np.asarray(row_modes(cfg), np.int32)
    lists = [fp.PList.from_host(t, rows, np.zeros(len(rows) + 1, np.int64), np.zeros(0, np.uint64), dev)
             for t in TYPES4]
    gam, wp = p.outputs(1)
    # empty rows within the workspace: accepted, outputs cleared
    gam.fill_(1.0)
    fp.fp_rates4_noalloc(ctx, lists, [300.0], cfg["sigma"], fp.FP_FP64, gam, wp)
    torch.cuda.synchronize()
    assert float(gam.abs().max()) == 0.0
    # more rows than the workspace has per-row force-constant tables for: refused
    # before anything is launched
    n_keys = fp.fp_ifc_info(ctx, 4)["n_keys"]
    n_big = int(fp.FP_NOALLOC_BYTES // (n_keys * 27 * 16)) + 1024
    big = [fp.PList.from_host(fp.FP_4PM, np.arange(n_big, dtype=np.int32) % cfg["omega"].size,
                              np.zeros(n_big + 1, np.int64), np.zeros(0, np.uint64), dev)]
    with pytest.raises(fp.FpError) as e:
        fp.fp_rates4_noalloc(ctx, big, [300.0], cfg["sigma"], fp.FP_FP64, gam, wp)
    assert e.value.status == fp.FP_ERR_UNSUPPORTED
