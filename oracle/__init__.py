"""ctypes access to the FP64 CPU oracle (oracle/oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it; the product path never does.  It shares no code with
the HIP library; both read the same seeded inputs from the synthetic generator.
"""
import ctypes
import os

import numpy as np

from .build import LIB, build

c_i32p = ctypes.POINTER(ctypes.c_int32)

# process types (same numbering as the library interface)
T3P, T3M, T4PP, T4PM, T4MM = 0, 1, 2, 3, 4
ORDER = {T3P: 3, T3M: 3, T4PP: 4, T4PM: 4, T4MM: 4}
SIGNS = {T3P: (1, 1, -1), T3M: (1, -1, -1), T4PP: (1, 1, 1, -1), T4PM: (1, 1, -1, -1), T4MM: (1, -1, -1, -1)}


class _Sys(ctypes.Structure):
    _fields_ = [
        ("mesh", ctypes.c_int32 * 3), ("n_atoms", ctypes.c_int32),
        ("masses", ctypes.c_void_p), ("omega", ctypes.c_void_p), ("evec", ctypes.c_void_p),
        ("omega_floor", ctypes.c_double),
        ("n3", ctypes.c_int64), ("atoms3", ctypes.c_void_p), ("cells3", ctypes.c_void_p), ("phi3", ctypes.c_void_p),
        ("n4", ctypes.c_int64), ("atoms4", ctypes.c_void_p), ("cells4", ctypes.c_void_p), ("phi4", ctypes.c_void_p),
        ("adaptive", ctypes.c_int32), ("factor", ctypes.c_double), ("vel", ctypes.c_void_p),
        ("recip", ctypes.c_double * 9),
    ]


_lib = None


def lib():
    """Load the oracle; ORACLE_LIB may name another build of oracle.c (mutation tests)."""
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIB", LIB)
        if path == LIB and not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(path)
        vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.orc_constants.argtypes = [vp]
        L.orc_threads.argtypes = []
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = None
        L.orc_bose.argtypes = [dbl, dbl]
        L.orc_bose.restype = dbl
        L.orc_gauss.argtypes = [dbl, dbl]
        L.orc_gauss.restype = dbl
        L.orc_vertex.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp]
        L.orc_rates.argtypes = [vp, ctypes.c_int, ctypes.c_int, i64, vp, vp, vp, dbl, dbl, ctypes.c_int, vp, vp,
                                vp, vp, vp]
        L.orc_enumerate.argtypes = [vp, ctypes.c_int, i32, dbl, dbl, vp, i64]
        L.orc_enumerate.restype = i64
        L.orc_occupation.argtypes = [ctypes.c_int, vp]
        L.orc_occupation.restype = dbl
        L.orc_grad.argtypes = [vp, ctypes.c_int, i64, vp, vp, vp, dbl, ctypes.c_int, vp, vp, vp]
        L.orc_kappa.argtypes = [i32, vp, vp, i32, vp, vp, vp, dbl, dbl, i64, dbl, vp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def constants():
    out = np.zeros(4)
    lib().orc_constants(_p(out))
    return dict(hbar=out[0], kb=out[1], ev=out[2], kappa_unit=out[3])


def threads():
    return int(lib().orc_threads())


def set_threads(n):
    """Threads of the rate sums that follow."""
    lib().orc_set_threads(int(n))


def bose(omega, T):
    return lib().orc_bose(float(omega), float(T))


def occupation(ptype, n):
    n = np.ascontiguousarray(n, dtype=np.float64)
    return lib().orc_occupation(ptype, _p(n))


def gauss(delta, sigma):
    return lib().orc_gauss(float(delta), float(sigma))


class System:
    """The oracle's view of one workload (mesh, modes, force constants).

    broadening: None for the fixed width of each call, or {"factor": a,
    "recip": (3, 3) reciprocal vectors as rows} for the per-process width
    max(a sigma0_p, sigma) from the partners' group velocities cfg["vel"].
    """

    def __init__(self, cfg, phi3=None, phi4=None, broadening=None):
        self._keep = []

        def arr(x, dt):
            a = np.ascontiguousarray(x, dtype=dt)
            self._keep.append(a)
            return _p(a)

        s = _Sys()
        for d in range(3):
            s.mesh[d] = int(cfg["mesh"][d])
        s.n_atoms = int(cfg["n_atoms"])
        s.masses = arr(cfg["masses"], np.float64)
        s.omega = arr(cfg["omega"].reshape(-1), np.float64)
        ev = np.ascontiguousarray(cfg["evec"], dtype=np.complex128).reshape(-1)
        s.evec = arr(ev.view(np.float64), np.float64)
        s.omega_floor = float(cfg["omega_floor"])
        for m, key, phi in ((3, "ifc3", phi3), (4, "ifc4", phi4)):
            ifc = cfg.get(key)
            if ifc is None:
                setattr(s, f"n{m}", 0)
                continue
            setattr(s, f"n{m}", int(ifc["atoms"].shape[0]))
            setattr(s, f"atoms{m}", arr(ifc["atoms"], np.int32))
            setattr(s, f"cells{m}", arr(ifc["cells"], np.int32))
            setattr(s, f"phi{m}", arr(ifc["phi"] if phi is None else phi, np.float64))
        if broadening is not None:
            s.adaptive = 1
            s.factor = float(broadening["factor"])
            s.vel = arr(cfg["vel"].reshape(-1), np.float64)
            rc = np.asarray(broadening["recip"], dtype=np.float64).reshape(9)
            for i in range(9):
                s.recip[i] = float(rc[i])
        self.s = s
        self.cfg = cfg
        self.nb = int(cfg["nb"])
        self.N = int(np.prod(cfg["mesh"]))

    @property
    def ptr(self):
        return ctypes.cast(ctypes.pointer(self.s), ctypes.c_void_p)

    def vertex(self, qc, br, sg):
        """Matrix element for slots at integer mesh coordinates qc (m, 3), branches br, signs sg."""
        qc = np.ascontiguousarray(qc, dtype=np.int32)
        br = np.ascontiguousarray(br, dtype=np.int32)
        sg = np.ascontiguousarray(sg, dtype=np.int32)
        out = np.zeros(2)
        rc = lib().orc_vertex(self.ptr, len(br), _p(qc), _p(br), _p(sg), _p(out))
        if rc:
            raise ValueError("orc_vertex failed")
        return complex(out[0], out[1])

    def rates(self, ptype, row_mode, T, sigma, nsigma=3.0, row_off=None, rec=None):
        """Per-row (Gamma, WP, kept, candidates); brute mode when no list is given."""
        row_mode = np.ascontiguousarray(row_mode, dtype=np.int32)
        T = np.ascontiguousarray(np.atleast_1d(T), dtype=np.float64)
        n_rows, n_T = len(row_mode), len(T)
        gam = np.zeros((n_rows, n_T))
        wp = np.zeros((n_rows, n_T))
        kept = np.zeros(n_rows, dtype=np.int64)
        cand = np.zeros(n_rows, dtype=np.int64)
        if rec is None:
            mode, ro, rc_ = 0, np.zeros(1, np.int64), np.zeros(1, np.uint64)
        else:
            mode = 1
            ro = np.ascontiguousarray(row_off, dtype=np.int64)
            rc_ = np.ascontiguousarray(rec, dtype=np.uint64)
        rc = lib().orc_rates(self.ptr, ptype, mode, n_rows, _p(row_mode), _p(ro), _p(rc_), float(sigma),
                             float(nsigma), n_T, _p(T), _p(gam), _p(wp), _p(kept), _p(cand))
        if rc:
            raise ValueError(f"orc_rates failed ({rc})")
        return gam, wp, kept, cand

    def grad(self, ptype, row_mode, T, sigma, row_off, rec, dLdG, out=None):
        """d(sum dLdG[r][T] Gamma_r(T))/d(raw force constants of the list's order), added into out."""
        row_mode = np.ascontiguousarray(row_mode, dtype=np.int32)
        T = np.ascontiguousarray(np.atleast_1d(T), dtype=np.float64)
        m = ORDER[ptype]
        n_terms = int(self.s.n3 if m == 3 else self.s.n4)
        if out is None:
            out = np.zeros((n_terms, 3 ** m))
        dl = np.ascontiguousarray(dLdG, dtype=np.float64).reshape(len(row_mode), len(T))
        ro = np.ascontiguousarray(row_off, dtype=np.int64)
        rc_ = np.ascontiguousarray(rec, dtype=np.uint64) if len(rec) else np.zeros(1, np.uint64)
        rc = lib().orc_grad(self.ptr, ptype, len(row_mode), _p(row_mode), _p(ro), _p(rc_), float(sigma), len(T),
                            _p(T), _p(dl), _p(out))
        if rc:
            raise ValueError(f"orc_grad failed ({rc})")
        return out

    def enumerate_row(self, ptype, g, sigma, nsigma=3.0):
        """Canonical packed records of one row by brute force (sorted)."""
        cap = 1 << 16
        while True:
            out = np.zeros(cap, dtype=np.uint64)
            n = lib().orc_enumerate(self.ptr, ptype, int(g), float(sigma), float(nsigma), _p(out), cap)
            if n <= cap:
                return np.sort(out[:n])
            cap = int(n)


def kappa(cfg, gamma_by_mode, T):
    """3x3 kappa (W/m/K) from per-mode Gamma (indexed by global mode g) at temperature T."""
    q1 = np.ascontiguousarray(cfg["q1"], dtype=np.int32)
    w = np.ascontiguousarray(cfg["q1_weight"], dtype=np.float64)
    om = np.ascontiguousarray(cfg["omega"].reshape(-1), dtype=np.float64)
    vel = np.ascontiguousarray(cfg["vel"].reshape(-1), dtype=np.float64)
    gam = np.ascontiguousarray(gamma_by_mode, dtype=np.float64)
    out = np.zeros(9)
    lib().orc_kappa(len(q1), _p(q1), _p(w), int(cfg["nb"]), _p(om), _p(vel), _p(gam), float(T),
                    float(cfg["volume"]), int(np.prod(cfg["mesh"])), float(cfg["omega_floor"]), _p(out))
    return out.reshape(3, 3)
