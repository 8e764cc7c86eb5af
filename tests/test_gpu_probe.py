"""Peak probes of the device (fp_peak_probe): each kernel keeps one pipe busy and
reports a positive, finite rate no larger than a generous bound on the chip's
published peak (MI355X: FP64 78.6 TFLOP/s vector and matrix, FP32 matrix 157.3,
dense bf16 2500, HBM 8000 GB/s).  Argument errors come back as statuses."""
import numpy as np
import pytest

from paper_2510_00518_amd import fp

pytestmark = pytest.mark.gpu

PUBLISHED = {0: 78.6, 1: 78.6, 2: 157.3, 3: 2500.0, 4: 8000.0}


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"  # torch's runtime first, as elsewhere
    c = fp.fp_create(0)
    yield c
    fp.fp_destroy(c)


@pytest.mark.parametrize("kind", [0, 1, 2, 3, 4])
def test_probe_rates(ctx, kind):
    v = fp.fp_peak_probe(ctx, kind, reps=2)
    print(f"probe {kind}: {v:.1f} (published {PUBLISHED[kind]})", flush=True)
    assert np.isfinite(v) and v > 0.05 * PUBLISHED[kind]
    assert v < 1.5 * PUBLISHED[kind]


def test_probe_argument_errors(ctx):
    for kind, reps in ((5, 1), (-1, 1), (0, 0), (0, 101)):
        with pytest.raises(fp.FpError):
            fp.fp_peak_probe(ctx, kind, reps=reps)
