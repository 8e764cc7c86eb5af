"""The five seeded synthetic workloads (diamond-structure, silicon-like mass).

  fcc4_3ph         3ph, 2-atom FCC, 4^3 mesh, every q1 (weight 1), 32 cubic terms
  fcc8_4ph         4ph, 2-atom FCC, 8^3 mesh, Oh-irreducible q1, the same 32 cubic
                   terms + 96 quartic terms
  fcc16_34ph       3ph+4ph, 2-atom FCC, 16^3 mesh, irreducible q1, 64 cubic + 160
                   quartic terms, T in {300, 600, 900} K
  sc10_4ph_uneven  4ph, 8-atom simple-cubic conventional cell, 10^3 mesh,
                   irreducible q1, 200 quartic terms, per-q1 list lengths drawn
                   log-uniform in [1e4, 1e7]
  fcc8_adjoint     adjoint workload: 2-atom FCC, 8^3 mesh, the 64 cubic + 160
                   quartic terms of fcc16_34ph

Common recipe: a = 5.431 A, masses 28 amu, per-shell spring constants
k1, k2 ~ U[5, 15] eV/A^2, cubic coefficients scaled to RMS 1 eV/A^3, quartic to
RMS 0.3 eV/A^4, Gaussian width sigma = 0.1 THz = 2 pi * 0.1 rad/ps, filter
|Delta| <= 3 sigma, omega floor 1e-3 rad/ps.  Adaptive-width variant of a
workload: sigma_p = max(0.1 sigma0_p, 0.01 THz) from the group velocities.  Seeds: default_rng(251000518 + k)
with k = 0 springs, 1 cubic, 2 quartic, 3 gradient-component pick, 4 uneven list lengths.
"""
import functools

import numpy as np

from .cells import diamond_conventional, diamond_primitive
from .harmonic import phonons, spring_fc2
from .ifc import build_ifc
from .qsym import irreducible_q

SEED = 251000518
SIGMA = 2.0 * np.pi * 0.1   # rad/ps
NSIGMA = 3.0
OMEGA_FLOOR = 1e-3          # rad/ps
# adaptive broadening: scale 0.1 (the paper's setting for three- plus
# four-phonon runs) and a floor of 0.01 THz where the partner velocities coincide
ADAPTIVE_FACTOR = 0.1
SIGMA_FLOOR = 2.0 * np.pi * 0.01   # rad/ps

_SPEC = {
    "fcc4_3ph": dict(cell="prim", mesh=4, q1="all", n3=32, n4=0, T=[300.0]),
    "fcc8_4ph": dict(cell="prim", mesh=8, q1="irr", n3=32, n4=96, T=[300.0]),
    "fcc16_34ph": dict(cell="prim", mesh=16, q1="irr", n3=64, n4=160, T=[300.0, 600.0, 900.0]),
    "sc10_4ph_uneven": dict(cell="conv", mesh=10, q1="irr", n3=0, n4=200, T=[300.0]),
    "fcc8_adjoint": dict(cell="prim", mesh=8, q1="irr", n3=64, n4=160, T=[300.0]),
}

DESCRIPTION = {
    "fcc4_3ph": "3ph FP64, 2-atom diamond cell, 4x4x4 mesh, all q1, 32 cubic terms",
    "fcc8_4ph": "4ph FP64, 2-atom diamond cell, 8x8x8 mesh, irreducible q1, 32 cubic + 96 quartic terms",
    "fcc16_34ph": "3ph+4ph, 2-atom diamond cell, 16x16x16 mesh, irreducible q1, 64 cubic + 160 quartic terms",
    "sc10_4ph_uneven": "4ph, 8-atom cubic diamond cell, 10x10x10 mesh, irreducible q1, 200 quartic terms, uneven lists",
    "fcc8_adjoint": "adjoint, 2-atom diamond cell, 8x8x8 mesh, 64 cubic + 160 quartic terms",
}


def springs():
    rng = np.random.default_rng(SEED + 0)
    return rng.uniform(5.0, 15.0, size=2)


@functools.lru_cache(maxsize=None)
def _cell(kind):
    return diamond_primitive() if kind == "prim" else diamond_conventional()


@functools.lru_cache(maxsize=None)
def _harmonic(kind, mesh):
    cell = _cell(kind)
    fc2 = spring_fc2(cell, springs())
    return phonons(cell, fc2, (mesh, mesh, mesh) if isinstance(mesh, int) else mesh)


@functools.lru_cache(maxsize=None)
def _ifc(kind, order, n_terms):
    if n_terms == 0:
        return None
    rng = np.random.default_rng(SEED + (1 if order == 3 else 2))
    return build_ifc(_cell(kind), order, n_terms, rng, rms=1.0 if order == 3 else 0.3)


def c4_lengths(n_q1):
    rng = np.random.default_rng(SEED + 4)
    return np.floor(10.0 ** rng.uniform(4.0, 7.0, size=n_q1)).astype(np.int64)


def make_config(name):
    """Return a dict with every input of the scattering-rate path for workload `name`."""
    s = _SPEC[name]
    cell = _cell(s["cell"])
    mesh = (s["mesh"],) * 3
    omega, evec, vel = _harmonic(s["cell"], s["mesh"])
    nq = omega.shape[0]
    if s["q1"] == "all":
        q1 = np.arange(nq, dtype=np.int32)
        w = np.ones(nq)
    else:
        q1, w = irreducible_q(cell, mesh)
    cfg = dict(
        name=name, description=DESCRIPTION[name], mesh=np.array(mesh, dtype=np.int32),
        n_atoms=cell.n_at, nb=cell.nb, lattice=cell.lattice.copy(), masses=cell.masses.copy(),
        volume=cell.volume, recip=cell.recip.copy(), omega=omega, evec=evec, vel=vel, q1=q1, q1_weight=w,
        sigma=SIGMA, nsigma=NSIGMA, omega_floor=OMEGA_FLOOR, T=np.array(s["T"]),
        ifc3=_ifc(s["cell"], 3, s["n3"]), ifc4=_ifc(s["cell"], 4, s["n4"]),
    )
    if name == "sc10_4ph_uneven":
        cfg["q1_lengths"] = c4_lengths(len(q1))
    return cfg


def small_config(mesh, n3=32, n4=96, cell="prim", T=(300.0,)):
    """Same recipe as the named workloads on a small mesh (N or (N0, N1, N2)),
    every q1 with weight 1."""
    c = _cell(cell)
    m3 = (int(mesh),) * 3 if np.isscalar(mesh) else tuple(int(x) for x in mesh)
    omega, evec, vel = _harmonic(cell, m3)
    nq = omega.shape[0]
    return dict(
        name=f"small{m3[0]}x{m3[1]}x{m3[2]}", description=f"{cell} cell, {m3[0]}x{m3[1]}x{m3[2]} mesh",
        mesh=np.array(m3, dtype=np.int32),
        n_atoms=c.n_at, nb=c.nb, lattice=c.lattice.copy(), masses=c.masses.copy(), volume=c.volume, recip=c.recip.copy(),
        omega=omega, evec=evec, vel=vel, q1=np.arange(nq, dtype=np.int32), q1_weight=np.ones(nq),
        sigma=SIGMA, nsigma=NSIGMA, omega_floor=OMEGA_FLOOR, T=np.array(T),
        ifc3=_ifc(cell, 3, n3), ifc4=_ifc(cell, 4, n4),
    )


def adaptive_broadening(cfg, factor=ADAPTIVE_FACTOR):
    """The adaptive-width setting of a workload: {"factor", "recip"} (its floor is SIGMA_FLOOR)."""
    return {"factor": float(factor), "recip": np.asarray(cfg["recip"], dtype=np.float64)}


def row_modes(cfg):
    """Global mode indices g = iq*nb + j of the active q1 modes (rows of the lists)."""
    nb = cfg["nb"]
    g = (cfg["q1"][:, None].astype(np.int64) * nb + np.arange(nb)[None, :]).ravel()
    active = cfg["omega"].reshape(-1)[g] >= cfg["omega_floor"]
    return g[active].astype(np.int32)
