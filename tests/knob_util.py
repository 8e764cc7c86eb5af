"""Launch knobs set for one block of a test and restored afterwards to the
values the context held before (the library defaults, unless a test changed
them on purpose), so no test leaks a knob into the tests after it."""
import contextlib

from paper_2510_00518_amd import fp

# the library's defaults, which the benchmark runs with
DEFAULT_VARIANT = 6


@contextlib.contextmanager
def knobs(ctx, **values):
    saved = {k: fp.fp_get_knob(ctx, k) for k in values}
    try:
        for k, v in values.items():
            fp.fp_set_knob(ctx, k, v)
        yield
    finally:
        for k, v in saved.items():
            fp.fp_set_knob(ctx, k, v)
