"""Pins of the oracle's DVM construction against what the paper fixes.

* every table printed in Appendices A and B (tests/golden/dvm_tables.txt):
  velocity count V, stencil energy E, group sizes V_g, quadrature order exactly
  Q (exact to degree Q, wrong at Q+1), and, for minimal DVMs, c* and the group
  weights re-solved from the null space of K(S) (Section II, Eqs. defK, dimker);
* the D2V16 closed form c = sqrt(3)/2, w = 64/405, 5/81, 1/36, 1/405 (table
  tab:dvmSet5Amin) and the D3V39 closed form c^2 = 3/2, w = 1/12, 1/12, 1/27,
  2/135, 1/432, 1/1620;
* the Hermite recurrence defH against the separable product of 1D Hermite
  polynomials, and the orthogonality relation (Eq. orth) under a DVM.
"""
import itertools
import math
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest

from oracle import dvm
from tests.golden.tables import load_dvm_tables

TABLES = load_dvm_tables()


def _mpq(fr):
    mp.mp.dps = dvm.MP_DPS
    return mp.mpf(fr.numerator) / fr.denominator


@pytest.mark.parametrize("m", TABLES, ids=[t["label"] for t in TABLES])
def test_printed_table_structure_and_degree(m):
    d = dvm.make_dvm(m["D"], m["gens"], m["weights"], m["c"], m["Q"])
    assert d.V == m["V"]
    assert d.energy == m["E"]
    assert [len(dvm.orbit(g)) for g in m["gens"]] == m["sizes"]
    assert abs(d.weights.sum() - 1.0) < 1e-15
    # printed weights carry 17 significant digits: exact to Q, not beyond
    assert dvm.quadrature_errors(d, m["Q"]) < 1e-13
    assert dvm.quadrature_errors(d, m["Q"] + 1) > 1e-6 or dvm.quadrature_errors(d, m["Q"] + 2) > 1e-6


MINIMAL = [t for t in TABLES if t["kind"] == "minimal"]


@pytest.mark.parametrize("m", MINIMAL, ids=[t["label"] for t in MINIMAL])
def test_minimal_tables_resolved_from_null_space(m):
    s = dvm.solve_dvm(m["D"], m["gens"], m["Q"], m["c"] * 0.97, m["c"] * 1.03, n_scan=600)
    assert abs(s.c - m["c"]) <= 2e-15 * m["c"]
    for got, want in zip(s.group_weights, m["weights"]):
        assert abs(got - want) <= 4e-15 * want


def test_d2v16_closed_form():
    s = dvm.solve_dvm(2, [(1, 0), (2, 0), (2, 2), (4, 0)], 7, 0.5, 1.2, n_scan=800)
    assert abs(s.c_mp ** 2 - 0.75) < 1e-30
    want = [Fraction(64, 405), Fraction(5, 81), Fraction(1, 36), Fraction(1, 405)]
    for got, w in zip(s.group_weights_mp, want):
        assert abs(got - _mpq(w)) < 1e-30


def test_d3v39_closed_form_and_config_dvms():
    s = dvm.named_dvm("D3V39")
    assert abs(s.c_mp ** 2 - 1.5) < 1e-30
    want = [Fraction(1, 12), Fraction(1, 12), Fraction(1, 27), Fraction(2, 135),
            Fraction(1, 432), Fraction(1, 1620)]
    for got, w in zip(s.group_weights_mp, want):
        assert abs(got - _mpq(w)) < 1e-30
    for name, V, Q in (("D2V17", 17, 7), ("D2V37", 37, 9), ("D3V39", 39, 7)):
        d = dvm.named_dvm(name)
        assert d.V == V
        assert np.all(d.weights > 0)
        assert dvm.quadrature_degree(d) == Q


def test_d2v17_positive_root_is_selected():
    # two roots of the nullity condition in [0.2, 3]; the smaller one has a
    # negative weight and is rejected (only positive weights are admitted)
    roots = dvm.solve_roots(2, dvm.D2V17_GENS, 7, 0.2, 3.0)
    cs = sorted(float(r[0]) for r in roots)
    assert len(cs) >= 2
    positive = [float(c) for c, w, _ in roots if all(x > 0 for x in w)]
    assert len(positive) == 1
    assert abs(dvm.named_dvm("D2V17").c - positive[0]) < 1e-15
    assert min(cs) < positive[0]


def _product_form(ms, x):
    out = 1.0
    for d in range(len(x)):
        n = ms.count(d)
        h0, h1 = 1.0, x[d]
        if n == 0:
            continue
        for k in range(1, n):
            h0, h1 = h1, x[d] * h1 - k * h0
        out *= h1
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_hermite_recurrence_matches_product_form(dim):
    rng = np.random.default_rng(7)
    for m in range(0, 6):
        for idx in itertools.product(range(dim), repeat=m):
            poly = dvm.hermite_component(tuple(idx), dim)
            # the tensor is symmetric: any ordering of the same multiset agrees
            poly_sorted = dvm.hermite_component(tuple(sorted(idx)), dim)
            assert dict(poly) == dict(poly_sorted)
            for _ in range(2):
                x = rng.normal(size=dim)
                got = float(dvm.eval_poly(poly, [Fraction(v) for v in x]))
                assert abs(got - _product_form(list(idx), x)) < 1e-9 * (1 + abs(got))


def test_orthogonality_relation_under_dvm():
    d = dvm.named_dvm("D2V17")
    xi = d.xi
    comps = []
    for m in range(0, 4):
        for ms, _ in dvm.component_multisets(2, m):
            comps.append((m, ms))
    for (m1, a), (m2, b) in itertools.product(comps, comps):
        if m1 + m2 > d.Q:
            continue
        q = sum(d.weights[k] * _product_form(list(a), xi[k]) * _product_form(list(b), xi[k])
                for k in range(d.V))
        # continuous value: prod over directions of n_d! if multisets equal, else 0
        if sorted(a) == sorted(b):
            want = math.prod(math.factorial(list(a).count(dd)) for dd in range(2))
        else:
            want = 0.0
        assert abs(q - want) < 1e-12 * max(1.0, want)
