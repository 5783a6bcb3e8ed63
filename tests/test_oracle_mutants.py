"""The oracle's pins catch plausible mistakes: each case below plants one
mistake in a copy of the oracle's C source (a dropped term, a wrong sign, a
missing conjugate, a wrong order or rule), builds it into a library of its
own, loads it in place of the oracle and runs the pins that should catch it;
at least one of them must fail. CPU only; the oracle itself is untouched."""
from __future__ import annotations

import os
import subprocess

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(os.path.abspath(oracle.__file__)), "vrk_oracle.c")

# (label, text in vrk_oracle.c, planted replacement, pins that must catch it)
MUTANTS = [
    ("sign of xi q in the residual",
     "return s[i] - acc - p->xi * q[i];", "return s[i] - acc + p->xi * q[i];",
     [lambda: pins.test_iterations_converge_to_rzf("grk", "baiwu"),
      lambda: pins.test_iterations_converge_to_rzf("vr_oahk", "baiwu")]),
    ("missing conjugate in the single-row update",
     "if (seen(p, i, n)) x[n] += gamma * conj(p->H[i * p->ldh + n]);",
     "if (seen(p, i, n)) x[n] += gamma * p->H[i * p->ldh + n];",
     [lambda: pins.test_iterations_converge_to_rzf("grk", "max")]),
    ("threshold term of the greedy randomized rule",
     "theta = 0.5 * (rho_max + rr / fro2);", "theta = 0.5 * rho_max;",
     [pins.test_selection_rules_against_definitions]),
    ("xi ||phi||^2 term of the aggregated step",
     "    den += p->xi * phin;\n", "\n",
     [pins.test_aggregated_step_decrease_and_rate, lambda: pins.test_iterations_converge_to_rzf("ahk", "baiwu")]),
    ("conjugate in the Cholesky update",
     "for (int t = 0; t < j; ++t) acc -= L[i * K + t] * conj(L[j * K + t]);",
     "for (int t = 0; t < j; ++t) acc -= L[i * K + t] * L[j * K + t];",
     [lambda: pins.test_rzf_cholesky_matches_numpy_and_scipy(64, 8, 0)]),
    ("MIS greedy ordered by start instead of end",
     "    if (vr_end(p, i) != vr_end(p, j)) return vr_end(p, i) < vr_end(p, j);\n    if (p->vs[i] != p->vs[j]) return p->vs[i] < p->vs[j];",
     "    if (p->vs[i] != p->vs[j]) return p->vs[i] < p->vs[j];\n    if (vr_end(p, i) != vr_end(p, j)) return vr_end(p, i) < vr_end(p, j);",
     [pins.test_mis_is_maximum_independent_set_bruteforce]),
    ("degree-1 reduction keeps the neighbour",
     "if (u != pick1 && alive[u] && vr_overlap(p, u, pick1)) alive[u] = 0;",
     "if (u != pick1 && alive[u] && vr_overlap(p, u, pick1)) alive[u] = 1;",
     [pins.test_reducing_peeling_exact_on_forests_and_maximal_on_graphs, pins.test_reducing_peeling_small_cases]),
    ("peeling a smallest-degree vertex",
     "if (d > dmax) { dmax = d; pickp = v; }", "if (dmax < 0 || d < dmax) { dmax = d; pickp = v; }",
     [pins.test_reducing_peeling_small_cases]),
    ("hull overlap instead of mask overlap",
     "if (p->mask) return (p->mask[i] & p->mask[j]) != 0;", "if (0) return (p->mask[i] & p->mask[j]) != 0;",
     [pins.test_subarray_graph_matches_antenna_indicators]),
    ("energy criterion weighted uniformly",
     "for (int i = 0; i < K; ++i) W += rule == ORC_SEL_ENERGY ? nrm[i] : 1.0;",
     "for (int i = 0; i < K; ++i) W += 1.0;",
     [pins.test_randomized_criteria_against_definitions]),
    ("sign of the mu x^H term of the gradient",
     "gH[k * ldgh + n] += vk * conj(g[n] - xh[n]) - muk * conj(x[n]);",
     "gH[k * ldgh + n] += vk * conj(g[n] - xh[n]) + muk * conj(x[n]);",
     [pins.test_rzf_gradient_matches_finite_differences]),
    ("one Philox multiplier digit",
     "M1 = 0xCA5A826395121157ULL", "M1 = 0xCA5A826395121155ULL",
     [lambda: pins.test_philox_matches_numpy((0, 0), (0, 0, 0, 0))]),
]


@pytest.fixture
def mutant_loader(tmp_path, monkeypatch):
    def load(old, new, tag):
        src = open(SRC).read()
        assert src.count(old) >= 1, "mutation anchor not found: %r" % old
        d = tmp_path / tag
        d.mkdir()
        c = d / "vrk_oracle.c"
        c.write_text(src.replace(old, new))
        so = d / "liboracle.so"
        subprocess.run(["gcc", "-O1", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", str(so), str(c), "-lm"],
                       check=True, capture_output=True)
        monkeypatch.setattr(oracle, "LIB", str(so))
        monkeypatch.setattr(oracle, "_lib", None)
    yield load
    # the real oracle again for whatever runs next
    oracle._lib = None


@pytest.mark.parametrize("idx", range(len(MUTANTS)), ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(idx, mutant_loader):
    label, old, new, checks = MUTANTS[idx]
    mutant_loader(old, new, "m%d" % idx)
    caught = []
    for check in checks:
        try:
            check()
        except (AssertionError, ValueError, FloatingPointError, OverflowError):
            caught.append(check)
    assert caught, "no pin caught the planted mistake: %s" % label
