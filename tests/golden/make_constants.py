"""Writes constants.txt: the physical constants of the scattering-rate path in
its internal units (amu, Angstrom, ps, K), from their SI definitions.

Inputs (no other source): the SI 2019 exact values of h, k_B and e, and the
CODATA 2018 atomic mass constant m_u = 1.66053906660e-27 kg.  Every derived value
is computed at 40 significant digits with mpmath and rounded to 15.

    python tests/golden/make_constants.py          # rewrites constants.txt
    python tests/golden/make_constants.py --check  # exit 1 if the file differs
"""
import os
import sys

import mpmath

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "constants.txt")

HEADER = """# Physical constants in the units of the scattering-rate path (amu, Angstrom, ps, K).
# Source: SI 2019 exact definitions of h, k_B and e; CODATA 2018 atomic mass
# constant m_u = 1.66053906660e-27 kg.  Derived values computed at 40 digits
# (mpmath) from h/(2 pi), k_B, e and m_u; rounded to 15 significant figures.
"""


def values():
    mpmath.mp.dps = 40
    h = mpmath.mpf("6.62607015e-34")      # J s, exact
    kb = mpmath.mpf("1.380649e-23")       # J/K, exact
    e = mpmath.mpf("1.602176634e-19")     # C, exact (1 eV = e J)
    mu = mpmath.mpf("1.66053906660e-27")  # kg, CODATA 2018
    angstrom, ps = mpmath.mpf("1e-10"), mpmath.mpf("1e-12")
    energy = mu * angstrom ** 2 / ps ** 2  # J per amu A^2 / ps^2
    action = mu * angstrom ** 2 / ps       # J s per amu A^2 / ps
    hbar = h / (2 * mpmath.pi) / action
    kB = kb / energy
    return [
        ("hbar_amu_A2_per_ps", hbar),
        ("kB_amu_A2_per_ps2_per_K", kB),
        ("eV_amu_A2_per_ps2", e / energy),
        ("hbar_over_kB_ps_K", hbar / kB),
        # kappa in amu A / ps^3 / K, expressed in W / (m K)
        ("kappa_unit_W_per_m_K", mu * angstrom / ps ** 3),
    ]


def render():
    lines = [HEADER.rstrip("\n")]
    width = max(len(k) for k, _ in values())
    for k, v in values():
        lines.append(f"{k:<{width}} {mpmath.nstr(v, 15, strip_zeros=False)}")
    return "\n".join(lines) + "\n"


if __name__ == "__main__":
    text = render()
    if "--check" in sys.argv:
        with open(OUT) as f:
            sys.exit(0 if f.read() == text else 1)
    with open(OUT, "w") as f:
        f.write(text)
