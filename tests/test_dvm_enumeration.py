"""The library's enumeration of minimal DVMs (lbm_dvm_enumerate, Section II.B)
against what the paper prints.

Pinned:
* the minimal velocity count V_min of every set of Table tab:dvmSummary that
  the enumeration covers (S1: 38, S2: 79, S4: 80, S5: 16, S6: 33, S7: 20);
* every printed minimal model (Appendices A and B) found in its set, at its
  printed energy E, lattice speed c* and group weights;
* the example of Eq. Ssymbol (D3Q19 = S^{D3V19}_{Q5E15}) and the minimal D3V15
  of Table tab:ExampleIntro;
* the wall accuracy index Lambda_index of Table tab:dvmSummary for the models
  with the fewest velocities (0 for the bulk sets, 549 for the scattering set
  S7, 6245 for S4), from the library's wall-moment diagnostics;
* the three DVMs of the channel and duct configurations (D2V17, D2V37, D3V39)
  at the speeds and weights solved independently.

Parity unpinned: the model counts # of Table tab:dvmSummary. Under this
enumeration's reading (a stencil is a set of distinct velocity groups with
group-constant weights, Eq. wdach; it is minimal at c* when the moment
conditions have exactly one solution there and none nearby, all weights
positive; integer multiples and 45-degree images count as separate stencils)
the 3D sets come out within 1 % of the printed counts and the 2D sets do not;
the tests only record them."""
import math

import pytest

from paper_1510_08886_amd import lbm
from tests.golden.tables import load_dvm_tables

SETS = {  # name: (dim, Q, E_max, scattering, printed V_min, printed Lambda_index)
    "S1": (3, 7, 500, False, 38, 0),
    "S2": (3, 9, 625, False, 79, 0),
    "S4": (3, 7, 2500, True, 80, 6245),
    "S5": (2, 7, 250, False, 16, 0),
    "S6": (2, 9, 300, False, 33, 0),
    "S7": (2, 7, 1000, True, 20, 549),
}
# printed minimal models and the set each belongs to (by D, Q, E <= E_max)
PRINTED = {"D3V38a": "S1", "D3V38b": "S1", "D3V59": "S1", "D3V64": "S1", "D3V66": "S1",
           "D3V79": "S2", "D3V121": "S2", "D3V96": "S4", "D3V112": "S4", "D2V16": "S5",
           "D2V33": "S6", "D2V32": "S7"}

_cache = {}


def models(name):
    if name not in _cache:
        dim, Q, emax, scat, _, _ = SETS[name]
        _cache[name] = lbm.enumerate_dvms(dim, Q, emax, scattering=scat)
    return _cache[name]


def _canon(g):
    return tuple(sorted(abs(int(x)) for x in g))


def _find(ms, gens, E):
    key = sorted(_canon(g) for g in gens)
    return [m for m in ms if m["E"] == E and sorted(m["gens"]) == key]


@pytest.mark.parametrize("name", sorted(SETS))
def test_minimal_velocity_count(name):
    ms = models(name)
    assert ms, name
    assert min(m["V"] for m in ms) == SETS[name][4]


@pytest.mark.parametrize("label", sorted(PRINTED))
def test_printed_minimal_models_are_found(label):
    t = {m["label"]: m for m in load_dvm_tables()}[label]
    hits = _find(models(PRINTED[label]), t["gens"], t["E"])
    hits = [m for m in hits if abs(m["c"] - t["c"]) <= 1e-13 * t["c"]]
    assert len(hits) == 1, (label, [m["c"] for m in _find(models(PRINTED[label]), t["gens"], t["E"])])
    m = hits[0]
    assert m["V"] == t["V"]
    want = {_canon(g): w for g, w in zip(t["gens"], t["weights"])}
    for g, w in zip(m["gens"], m["weights"]):
        assert abs(w - want[g]) <= 1e-12 * want[g], (label, g, w, want[g])


@pytest.mark.parametrize("name", sorted(SETS))
def test_wall_accuracy_index_of_the_smallest_models(name):
    """Lambda_index of each model with V = V_min equals the set's printed
    value (Eq. defbin; Table tab:dvmSummary)."""
    dim, Q, _, _, vmin, lam = SETS[name]
    for m in [m for m in models(name) if m["V"] == vmin]:
        d = lbm.Dvm(dim, m["gens"], m["weights"], m["c"], Q)
        assert d.wall_errors(normal_axis=dim - 1)["lambda_index"] == lam, (name, m)


def test_symbol_example_and_intro_model():
    ms = lbm.enumerate_dvms(3, 5, 30)
    # D3Q19 -> S^{D3V19}_{Q5E15} (Eq. Ssymbol); the D3V15 of tab:ExampleIntro at E = 24
    d3q19 = _find(ms, [(0, 0, 0), (1, 0, 0), (1, 1, 0)], 15)
    assert len(d3q19) == 1 and d3q19[0]["V"] == 19 and abs(d3q19[0]["c"] - math.sqrt(3)) < 1e-14
    t = {m["label"]: m for m in load_dvm_tables()}["D3V15"]
    hit = _find(ms, t["gens"], t["E"])
    assert len(hit) == 1 and abs(hit[0]["c"] - t["c"]) <= 1e-14 * t["c"]


@pytest.mark.parametrize("name,dim,Q,emax,E", [("D2V17", 2, 7, 250, 40), ("D2V37", 2, 9, 300, 108),
                                             ("D3V39", 3, 7, 500, 102)])
def test_configuration_dvms(name, dim, Q, emax, E):
    """The channel and duct DVMs appear at their energies, with the lattice
    speed and weights that lbm_dvm_solve finds for their generators."""
    spec = lbm.NAMED_DVMS[name]
    d = lbm.Dvm.named(name)
    ms = models({(2, 7): "S5", (2, 9): "S6", (3, 7): "S1"}[(dim, Q)])
    hits = [m for m in _find(ms, spec["gens"], E) if abs(m["c"] - d.c) <= 1e-13 * d.c]
    assert len(hits) == 1
    assert hits[0]["V"] == d.V


def test_counts_are_recorded():
    """Parity unpinned (see the module docstring): the counts only have to be
    positive and ordered by construction; their values are listed in the
    design notes next to the printed ones."""
    counts = {n: len(models(n)) for n in SETS}
    assert all(v > 0 for v in counts.values())
    print("enumerated counts:", counts)


@pytest.mark.parametrize("name", ["S5", "S6", "S7", "S1"])
def test_enumerated_models_are_quadratures_by_the_oracle(name):
    """A seeded sample of each enumerated set, checked with the oracle's own
    code (independent of the library): the velocities integrate every monomial
    of degree <= Q exactly (Eqs. genQua / orth), the weights are positive, V
    and E are those of the expanded stencil, and the oracle's nullity condition
    (Eq. dimker) has a root at the enumerated c* with the same weights."""
    import numpy as np

    from oracle import dvm as odvm
    dim, Q, emax, scat, _, _ = SETS[name]
    ms = models(name)
    rng = np.random.default_rng(1510)
    pick = [ms[int(k)] for k in rng.choice(len(ms), size=min(6, len(ms)), replace=False)]
    for m in pick:
        gens = [tuple(int(x) for x in g) for g in m["gens"]]
        d = odvm.make_dvm(dim, gens, m["weights"], m["c"], Q)
        assert d.V == m["V"] and d.energy == m["E"]
        assert all(w > 0 for w in m["weights"])
        for deg in range(1, Q + 1):
            assert odvm.quadrature_errors(d, deg) < 1e-10, (m, deg)
        if scat:
            assert all(0 not in e for e in d.velocities.tolist())
        roots = odvm.solve_roots(dim, gens, Q, 0.995 * m["c"], 1.005 * m["c"], n_scan=400)
        near = [r for r in roots if abs(float(r[0]) - m["c"]) <= 1e-9 * m["c"]]
        assert len(near) == 1, (m, [float(r[0]) for r in roots])
        wbar = [float(x) for x in near[0][1]]
        for a, b in zip(wbar, m["weights"]):
            assert abs(a - b) <= 1e-9 * abs(b), (m, wbar)
