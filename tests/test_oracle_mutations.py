"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of oracle.c (on the CPU, in a temporary
directory), builds it, and runs the pin tests (the physics pins and the
golden-rule pin of the prefactors) against that build; the pins must fail.  The unmodified source must pass the same selection.
"""
import os
import subprocess
import sys

import pytest

from oracle.build import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTATIONS = {
    "emitted partner not conjugated": ("cplx r = {p[0], sign > 0 ? p[1] : -p[1]};", "cplx r = {p[0], p[1]};"),
    "phase sign flipped": ("k[d] += (int64_t)sg[r] * qc[r][d] * ce[(r - 1) * 3 + d];",
                           "k[d] -= (int64_t)sg[r] * qc[r][d] * ce[(r - 1) * 3 + d];"),
    "transposed force-constant index": ("double f = ph[((a0 * 3 + a1) * 3 + a2) * 3 + a3];",
                                        "double f = ph[((a0 * 3 + a2) * 3 + a1) * 3 + a3];"),
    "last term dropped": ("cplx V = {0.0, 0.0};\n    for (int64_t t = 0; t < n_terms; ++t) {",
                          "cplx V = {0.0, 0.0};\n    for (int64_t t = 0; t < n_terms - 1; ++t) {"),
    "gradient without the factor 2 of |V|^2": ("            c *= 2.0;\n", "            c *= 1.0;\n"),
    "gradient with V not conjugated": ("cplx Vc = {V.re, -V.im};", "cplx Vc = {V.re, V.im};"),
    "one mass factor dropped": ("for (int r = 0; r < m; ++r) msc *= s->masses[at[r]];",
                                "for (int r = 1; r < m; ++r) msc *= s->masses[at[r]];"),
    "wrong 4+- occupation": ("case T4PM: return n[1] * (1.0 + n[2]) * (1.0 + n[3]) - (1.0 + n[1]) * n[2] * n[3];",
                             "case T4PM: return n[1] * (1.0 + n[2]) * (1.0 + n[3]) - n[1] * n[2] * n[3];"),
    "wrong 3- occupation": ("case T3M: return 1.0 + n[1] + n[2];", "case T3M: return n[1] + n[2];"),
    "wrong -- ordered weight": ("if (ptype == T4MM) return 1.0 / 6.0;", "if (ptype == T4MM) return 0.5;"),
    "wrong 3- triangle weight": ("case T3M: return g[1] == g[2] ? 0.5 : 1.0;", "case T3M: return 1.0;"),
    "Gaussian width convention": ("return exp(-(delta * delta) / (sigma * sigma)) / (sigma * sqrt(M_PI));",
                                  "return exp(-(delta * delta) / (2.0 * sigma * sigma)) / (sigma * sqrt(M_PI));"),
    "Bose with exp instead of expm1": ("return 1.0 / expm1(c_hbar() * omega / (c_kb() * T));",
                                       "return 1.0 / exp(c_hbar() * omega / (c_kb() * T));"),
    "momentum closed with wrong sign": ("qc[m - 1][d] = wrap(sg[m - 1] * (-Q), s->mesh[d]);",
                                        "qc[m - 1][d] = wrap(sg[m - 1] * Q, s->mesh[d]);"),
    "filter with strict bound on wrong side": ("if (filter && !(fabs(delta) <= pc->nsigma * sp)) return 0;",
                                               "if (filter && !(fabs(delta) <= 2.0 * pc->nsigma * sp)) return 0;"),
    "adaptive width with the variance, not 2 var": ("double sigma0 = sqrt(s2 / (3.0 * (double)(m - 1)));",
                                                    "double sigma0 = sqrt(s2 / (6.0 * (double)(m - 1)));",
                                                    "adaptive"),
    "adaptive width with reciprocal vectors transposed": (
        "double p = (w0 * s->recip[d * 3 + 0] + w1 * s->recip[d * 3 + 1] + w2 * s->recip[d * 3 + 2]) /",
        "double p = (w0 * s->recip[0 * 3 + d] + w1 * s->recip[1 * 3 + d] + w2 * s->recip[2 * 3 + d]) /",
        "adaptive"),
    "adaptive width divided by the wrong mesh axis": ("                           (double)s->mesh[d];",
                                                      "                           (double)s->mesh[2 - d];", "adaptive"),
    "adaptive four-phonon width from one partner pair": (
        "        for (int j = i + 1; j < m; ++j) {\n            const double* vi",
        "        for (int j = i + 1; j < (i == 1 ? m : 0); ++j) {\n            const double* vi", "adaptive"),
    "adaptive width taken before the floor": ("    return sp > sigma ? sp : sigma;", "    return sp;", "adaptive"),
    "three-phonon prefactor pi hbar / 2N": ("if (m == 3) return M_PI * hb / (4.0 * (double)N);",
                                            "if (m == 3) return M_PI * hb / (2.0 * (double)N);"),
    "four-phonon prefactor with 1/N": ("return M_PI * hb * hb / (8.0 * (double)N * (double)N);",
                                       "return M_PI * hb * hb / (8.0 * (double)N);"),
    "four-phonon prefactor with hbar, not hbar^2": ("return M_PI * hb * hb / (8.0 * (double)N * (double)N);",
                                                    "return M_PI * hb / (8.0 * (double)N * (double)N);"),
}


def _run_pins(lib_path, select=None):
    env = dict(os.environ, ORACLE_LIB=lib_path, OMP_NUM_THREADS="4")
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
           os.path.join(ROOT, "tests", "test_oracle_golden_rule.py"),
           os.path.join(ROOT, "tests", "test_oracle_pins.py")] + (["-k", select] if select else [])
    return subprocess.run(cmd, env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_mutation(name, tmp_path):
    old, new, *select = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not found once: {old}"
    mutated = tmp_path / "oracle_mut.c"
    mutated.write_text(src.replace(old, new))
    lib = build(source=str(mutated), out=str(tmp_path / "liboracle_mut.so"))
    res = _run_pins(lib, *select)
    # 5 would mean that no pin ran at all
    assert res.returncode not in (0, 5), f"pins did not catch: {name}\n{res.stdout[-2000:]}"
