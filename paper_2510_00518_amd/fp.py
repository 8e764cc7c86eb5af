"""Python binding of libfp (include/fp.h): the same entry points, argument
marshalling only.  Every step of the rate computation runs in the library;
this module converts numpy arrays and torch tensors to pointers and raises on
a non-zero status.  There is no fallback: without libfp.so it raises.

Device buffers are torch tensors on the library's device (int64 tensors carry
the uint64 records bit for bit); host arrays are numpy arrays.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfp.so")

FP_OK, FP_ERR_ARG, FP_ERR_STATE, FP_ERR_RANGE, FP_ERR_NOMEM, FP_ERR_HIP, FP_ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
FP_FP64, FP_MIXED = 0, 1
FP_ACCUMULATE = 0x100
FP_3P, FP_3M, FP_4PP, FP_4PM, FP_4MM, FP_3E = 0, 1, 2, 3, 4, 5
ORDER = {FP_3P: 3, FP_3M: 3, FP_4PP: 4, FP_4PM: 4, FP_4MM: 4, FP_3E: 3}
FP_MAX_T = 8
FP_MAX_LISTS = 8
FP_NOALLOC_BYTES = 128 << 20

EXPORTS = ["fp_create", "fp_destroy", "fp_last_error", "fp_load_modes", "fp_load_ifc", "fp_rates3", "fp_rates4",
           "fp_rates4_fused", "fp_rates_backward", "fp_kappa_rta", "fp_check", "fp_set_knob", "fp_get_knob", "fp_autotune", "fp_profile", "fp_profile_read",
           "fp_enumerate_count", "fp_enumerate_fill", "fp_set_broadening", "fp_rates_streamed", "fp_fused_counts",
           "fp_ifc_info", "fp_rates4_noalloc", "fp_peak_probe"]


class FpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libfp status {status}: {msg}")
        self.status = status


class fp_plist(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("reserved", ctypes.c_int32), ("n_rows", ctypes.c_int64),
                ("n_rec", ctypes.c_int64), ("row_mode", ctypes.c_void_p), ("row_off", ctypes.c_void_p),
                ("rec", ctypes.c_void_p)]


class fp_tune_entry(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("ppl", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("ms", ctypes.c_double)]


class fp_stream_stats(ctypes.Structure):
    _fields_ = [("n_records", ctypes.c_int64), ("n_chunks", ctypes.c_int64), ("max_chunk", ctypes.c_int64),
                ("count_ms", ctypes.c_double), ("fill_ms", ctypes.c_double), ("wait_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double)]


class fp_broadening(ctypes.Structure):
    _fields_ = [("adaptive", ctypes.c_int32), ("reserved", ctypes.c_int32), ("factor", ctypes.c_double),
                ("recip", ctypes.c_double * 9)]


def _broadening(b):
    """None (fixed width) or {"factor": a, "recip": (3, 3) rows b_d} -> fp_broadening pointer or None."""
    if b is None:
        return None
    out = fp_broadening()
    out.adaptive = 1
    out.factor = float(b["factor"])
    rc = np.asarray(b["recip"], dtype=np.float64).reshape(9)
    for i in range(9):
        out.recip[i] = float(rc[i])
    return ctypes.pointer(out)


_lib = None


def lib():
    """Load libfp.so; raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2510_00518_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64
        L.fp_create.argtypes = [ctypes.POINTER(vp), i32]
        L.fp_destroy.argtypes = [vp]
        L.fp_destroy.restype = None
        L.fp_last_error.argtypes = [vp]
        L.fp_last_error.restype = ctypes.c_char_p
        L.fp_load_modes.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp, dbl]
        L.fp_load_ifc.argtypes = [vp, i32, i64, vp, vp, vp, i32, vp]
        for f in (L.fp_rates3, L.fp_rates4, L.fp_rates4_noalloc):
            f.argtypes = [vp, ctypes.POINTER(fp_plist), i32, i32, vp, dbl, i32, vp, vp, vp]
        L.fp_rates4_fused.argtypes = [vp, i64, vp, i32, i32, vp, dbl, dbl, i32, vp, vp, vp, vp]
        L.fp_fused_counts.argtypes = [vp, vp, vp]
        L.fp_peak_probe.argtypes = [vp, i32, i32, vp, vp]
        L.fp_ifc_info.argtypes = [vp, i32, vp]
        L.fp_rates_backward.argtypes = [vp, ctypes.POINTER(fp_plist), i32, i32, vp, dbl, i32, vp, vp, vp, vp]
        L.fp_kappa_rta.argtypes = [vp, i32, vp, vp, i32, vp, vp, vp, vp, vp]
        L.fp_check.argtypes = [vp, vp]
        L.fp_set_knob.argtypes = [vp, ctypes.c_char_p, i64]
        L.fp_get_knob.argtypes = [vp, ctypes.c_char_p, vp]
        L.fp_autotune.argtypes = [vp, i32, ctypes.POINTER(fp_plist), i32, i32, vp, dbl, i32, i32,
                                  ctypes.POINTER(fp_tune_entry), i32, vp, vp]
        L.fp_profile.argtypes = [vp, i32]
        L.fp_profile_read.argtypes = [vp, i32, vp, vp]
        bp = ctypes.POINTER(fp_broadening)
        L.fp_enumerate_count.argtypes = [i32, vp, i32, vp, dbl, i64, vp, dbl, dbl, dbl, u64, i32, vp, bp, vp]
        L.fp_enumerate_fill.argtypes = [i32, vp, i32, vp, dbl, i64, vp, dbl, dbl, dbl, u64, i32, vp, bp, vp, vp]
        L.fp_set_broadening.argtypes = [vp, bp]
        L.fp_rates_streamed.argtypes = [vp, i32, i64, vp, i32, vp, dbl, dbl, i32, i64, i32, vp, vp,
                                        ctypes.POINTER(fp_stream_stats), vp]
        for name in EXPORTS:
            if name not in ("fp_destroy", "fp_last_error"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _hp(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dp(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _check(ctx, status):
    if status != FP_OK:
        msg = lib().fp_last_error(ctx).decode() if ctx else ""
        raise FpError(status, msg)


def fp_create(device=0):
    h = ctypes.c_void_p()
    _check(None, lib().fp_create(ctypes.byref(h), int(device)))
    return h


def fp_destroy(ctx):
    lib().fp_destroy(ctx)


def fp_last_error(ctx):
    return lib().fp_last_error(ctx).decode()


def fp_set_knob(ctx, name, value):
    _check(ctx, lib().fp_set_knob(ctx, name.encode(), int(value)))


def fp_get_knob(ctx, name):
    v = ctypes.c_int64(0)
    _check(ctx, lib().fp_get_knob(ctx, name.encode(), ctypes.byref(v)))
    return int(v.value)


def fp_load_modes(ctx, mesh, n_atoms, lattice, masses, omega, evec, vel, omega_floor):
    keep = [_host(mesh, np.int32), _host(lattice, np.float64).reshape(-1), _host(masses, np.float64),
            _host(omega, np.float64).reshape(-1), _host(np.asarray(evec, dtype=np.complex128), np.complex128),
            None if vel is None else _host(vel, np.float64).reshape(-1)]
    _check(ctx, lib().fp_load_modes(ctx, _hp(keep[0]), int(n_atoms), _hp(keep[1]), _hp(keep[2]), _hp(keep[3]),
                                    _hp(keep[4]), None if keep[5] is None else _hp(keep[5]), float(omega_floor)))


def fp_load_ifc(ctx, order, atoms, cells, phi, stream=None):
    """phi: numpy array (host) or a contiguous float64 device tensor [n_terms, 3**order]."""
    atoms = _host(atoms, np.int32)
    cells = _host(cells, np.int32)
    n = atoms.shape[0]
    if hasattr(phi, "is_cuda") and phi.is_cuda:
        ptr, on_dev, keep = _dp(phi), 1, phi
    else:
        keep = _host(phi, np.float64)
        ptr, on_dev = _hp(keep), 0
    _check(ctx, lib().fp_load_ifc(ctx, int(order), n, _hp(atoms), _hp(cells), ptr, on_dev, _stream(stream)))


class PList:
    """A device-resident CSR list (torch tensors) in the fp_plist layout."""

    def __init__(self, ptype, row_mode, row_off, rec):
        self.type = int(ptype)
        self.row_mode, self.row_off, self.rec = row_mode, row_off, rec
        self.n_rec = int(rec.numel())

    @property
    def n_rows(self):
        return int(self.row_mode.numel())

    def struct(self):
        return fp_plist(self.type, 0, self.n_rows, self.n_rec, _dp(self.row_mode), _dp(self.row_off),
                        _dp(self.rec) if self.n_rec else None)

    @classmethod
    def from_host(cls, ptype, row_mode, row_off, rec, device):
        import torch
        rm = torch.as_tensor(_host(row_mode, np.int32)).to(device)
        ro = torch.as_tensor(_host(row_off, np.int64)).to(device)
        rc = torch.as_tensor(_host(rec, np.uint64).view(np.int64)).to(device)
        return cls(ptype, rm, ro, rc)


def _lists(lists):
    arr = (fp_plist * max(1, len(lists)))()
    for i, pl in enumerate(lists):
        arr[i] = pl.struct()
    return arr


def _rates(fn, ctx, lists, T, sigma, precision, gamma_out, wp_out, stream):
    T = _host(np.atleast_1d(T), np.float64)
    arr = _lists(lists)
    _check(ctx, fn(ctx, arr, len(lists), len(T), _hp(T), float(sigma), int(precision), _dp(gamma_out),
                   _dp(wp_out), _stream(stream)))


def fp_rates3(ctx, lists, T, sigma, precision=FP_FP64, gamma_out=None, wp_out=None, stream=None):
    _rates(lib().fp_rates3, ctx, lists, T, sigma, precision, gamma_out, wp_out, stream)


def fp_rates4(ctx, lists, T, sigma, precision=FP_FP64, gamma_out=None, wp_out=None, stream=None):
    _rates(lib().fp_rates4, ctx, lists, T, sigma, precision, gamma_out, wp_out, stream)


def fp_rates4_noalloc(ctx, lists, T, sigma, precision=FP_FP64, gamma_out=None, wp_out=None, stream=None):
    """fp_rates4 with every per-call table in the library's fixed workspace (no allocation)."""
    _rates(lib().fp_rates4_noalloc, ctx, lists, T, sigma, precision, gamma_out, wp_out, stream)


def fp_rates4_fused(ctx, row_mode, type_mask, T, sigma, nsigma, precision=FP_FP64, gamma_out=None, wp_out=None,
                    n_kept=None, stream=None):
    """row_mode: int32 device tensor of distinct modes; n_kept: int64 device tensor [1] or None."""
    T = _host(np.atleast_1d(T), np.float64)
    _check(ctx, lib().fp_rates4_fused(ctx, int(row_mode.numel()), _dp(row_mode), int(type_mask), len(T), _hp(T),
                                      float(sigma), float(nsigma), int(precision), _dp(gamma_out), _dp(wp_out),
                                      _dp(n_kept), _stream(stream)))



def fp_ifc_info(ctx, order):
    """{"n_terms", "n_keys", "n_groups", "n_pkeys", "n_pgroups"} of the loaded
    force constants of `order`."""
    out = np.zeros(5, np.int64)
    _check(ctx, lib().fp_ifc_info(ctx, int(order), _hp(out)))
    return {"n_terms": int(out[0]), "n_keys": int(out[1]), "n_groups": int(out[2]), "n_pkeys": int(out[3]),
            "n_pgroups": int(out[4])}


PROBES = {"fp64_vector_tflops": 0, "fp64_matrix_tflops": 1, "fp32_matrix_tflops": 2, "bf16_matrix_tflops": 3,
          "hbm_copy_gbs": 4}


def fp_peak_probe(ctx, kind, reps=3, stream=None):
    """The device's measured peak for probe `kind` (0-3: TFLOP/s, 4: GB/s)."""
    out = np.zeros(1, np.float64)
    _check(ctx, lib().fp_peak_probe(ctx, int(kind), int(reps), _hp(out), _stream(stream)))
    return float(out[0])


def fp_fused_counts(ctx, stream=None):
    """(processes, tuples) of the last fp_rates4_fused call; waits on `stream`."""
    out = np.zeros(2, np.int64)
    _check(ctx, lib().fp_fused_counts(ctx, _hp(out), _stream(stream)))
    return int(out[0]), int(out[1])

def fp_autotune(ctx, order, lists, T, sigma, precision=FP_FP64, reps=2, stream=None):
    """Run the library's autotuner; returns the measured candidates as dicts
    (the fastest is left in the context's knobs)."""
    T = _host(np.atleast_1d(T), np.float64)
    arr = _lists(lists)
    rep = (fp_tune_entry * 64)()
    n = ctypes.c_int32(0)
    _check(ctx, lib().fp_autotune(ctx, int(order), arr, len(lists), len(T), _hp(T), float(sigma), int(precision),
                                  int(reps), rep, 64, ctypes.byref(n), _stream(stream)))
    return [{"variant": rep[i].variant, "ppl": rep[i].ppl, "blocks_per_cu": rep[i].blocks_per_cu, "ms": rep[i].ms}
            for i in range(n.value)]


def fp_rates_backward(ctx, lists, T, sigma, dL_dgamma, dphi3=None, dphi4=None, precision=FP_FP64, stream=None):
    T = _host(np.atleast_1d(T), np.float64)
    arr = _lists(lists)
    _check(ctx, lib().fp_rates_backward(ctx, arr, len(lists), len(T), _hp(T), float(sigma), int(precision),
                                        _dp(dL_dgamma), _dp(dphi3), _dp(dphi4), _stream(stream)))


def fp_kappa_rta(ctx, q1, q1_weight, T, gamma, kappa_out, dkappa_dgamma=None, stream=None):
    T = _host(np.atleast_1d(T), np.float64)
    _check(ctx, lib().fp_kappa_rta(ctx, int(q1.numel()), _dp(q1), _dp(q1_weight), len(T), _hp(T), _dp(gamma),
                                   _dp(kappa_out), _dp(dkappa_dgamma), _stream(stream)))


def fp_profile(ctx, enable=True):
    _check(ctx, lib().fp_profile(ctx, int(bool(enable))))


def fp_profile_read(ctx, order):
    """(total milliseconds, launch count) of the order-`order` rate kernel since fp_profile(ctx, True)."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(ctx, lib().fp_profile_read(ctx, int(order), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def fp_set_broadening(ctx, broadening):
    """broadening: None (the fixed width of each call) or {"factor": a, "recip": (3, 3)}."""
    _check(ctx, lib().fp_set_broadening(ctx, _broadening(broadening)))


def fp_rates_streamed(ctx, type_mask, row_mode, T, sigma, nsigma, precision, chunk_records, gamma_out, wp_out=None,
                      n_threads=0, stream=None):
    """Rates over host-enumerated lists streamed through bounded staging slots
    (row_mode: host array).  Synchronous; returns the call's figures as a dict."""
    rm = _host(row_mode, np.int32)
    T = _host(np.atleast_1d(T), np.float64)
    st = fp_stream_stats()
    _check(ctx, lib().fp_rates_streamed(ctx, int(type_mask), len(rm), _hp(rm), len(T), _hp(T), float(sigma),
                                        float(nsigma), int(precision), int(chunk_records), int(n_threads),
                                        _dp(gamma_out), _dp(wp_out), ctypes.byref(st), _stream(stream)))
    return {k: getattr(st, k) for k, _ in fp_stream_stats._fields_}


def fp_check(ctx, stream=None):
    _check(ctx, lib().fp_check(ctx, _stream(stream)))


def _vel(vel, broadening):
    if broadening is None:
        return None, None
    if vel is None:
        raise ValueError("adaptive broadening needs the group velocities")
    v = _host(vel, np.float64).reshape(-1)
    return v, _hp(v)


def fp_enumerate_count(ptype, mesh, nb, omega, omega_floor, row_mode, sigma, nsigma, keep_fraction=1.0, seed=0,
                       n_threads=0, vel=None, broadening=None):
    mesh = _host(mesh, np.int32)
    omega = _host(omega, np.float64).reshape(-1)
    row_mode = _host(row_mode, np.int32)
    row_off = np.zeros(len(row_mode) + 1, dtype=np.int64)
    v, vp = _vel(vel, broadening)
    st = lib().fp_enumerate_count(int(ptype), _hp(mesh), int(nb), _hp(omega), float(omega_floor), len(row_mode),
                                  _hp(row_mode), float(sigma), float(nsigma), float(keep_fraction), int(seed),
                                  int(n_threads), vp, _broadening(broadening), _hp(row_off))
    _check(None, st)
    return row_off


def fp_enumerate_fill(ptype, mesh, nb, omega, omega_floor, row_mode, sigma, nsigma, row_off, keep_fraction=1.0,
                      seed=0, n_threads=0, vel=None, broadening=None):
    mesh = _host(mesh, np.int32)
    omega = _host(omega, np.float64).reshape(-1)
    row_mode = _host(row_mode, np.int32)
    row_off = _host(row_off, np.int64)
    rec = np.zeros(max(1, int(row_off[-1])), dtype=np.uint64)
    v, vp = _vel(vel, broadening)
    st = lib().fp_enumerate_fill(int(ptype), _hp(mesh), int(nb), _hp(omega), float(omega_floor), len(row_mode),
                                 _hp(row_mode), float(sigma), float(nsigma), float(keep_fraction), int(seed),
                                 int(n_threads), vp, _broadening(broadening), _hp(row_off), _hp(rec))
    _check(None, st)
    return rec[: int(row_off[-1])]


def enumerate_list(ptype, cfg, row_mode=None, nsigma=None, sigma=None, keep_fraction=1.0, seed=0, n_threads=0,
                   broadening=None):
    """Both enumeration passes for one list of a synthetic workload (host arrays).
    broadening: None or {"factor": a, "recip": (3, 3)} (adaptive width, floor sigma)."""
    from .synth import row_modes
    rm = row_modes(cfg) if row_mode is None else np.asarray(row_mode, dtype=np.int32)
    sig = cfg["sigma"] if sigma is None else sigma
    ns = cfg["nsigma"] if nsigma is None else nsigma
    vel = cfg["vel"] if broadening is not None else None
    off = fp_enumerate_count(ptype, cfg["mesh"], cfg["nb"], cfg["omega"], cfg["omega_floor"], rm, sig, ns,
                             keep_fraction, seed, n_threads, vel, broadening)
    rec = fp_enumerate_fill(ptype, cfg["mesh"], cfg["nb"], cfg["omega"], cfg["omega_floor"], rm, sig, ns, off,
                            keep_fraction, seed, n_threads, vel, broadening)
    return rm, off, rec
