"""Slip velocity and Knudsen-layer analysis of a channel profile (Section VI of
the paper, Eqs. defSlip, uNS, uNEQ): the oracle pinned to exact cases, and the
library's host function (lbm_profile_analysis through the C ABI) against it.

Pins of the oracle:
* a sampled slip parabola u = a + b y (1 - y): wall value a and centre value
  a + b/4 exactly (quadratic extrapolation and the centre rule are exact for
  it), no non-equilibrium part (u^neq = 0);
* u^NS keeps the node-averaged mass flow and the centre value of any profile;
* the discrete u^NS tends to the continuum formula of Eq. uNS as O(1/ny^2);
* a cubic profile: the even-ny centre value is exact.
"""
import numpy as np
import pytest

from oracle import profile


def nodes(ny):
    return (np.arange(ny) + 0.5) / ny


@pytest.mark.parametrize("ny", [3, 4, 5, 8, 17, 40, 41])
def test_slip_parabola_is_exact(ny):
    a, b = 0.3, 2.5
    y = nodes(ny)
    r = profile.analyse(a + b * y * (1 - y))
    assert r["u_wall"] == pytest.approx(a, rel=1e-13)
    assert r["u_center"] == pytest.approx(a + b / 4, rel=1e-13)
    assert r["slip"] == pytest.approx(a / (a + b / 4), rel=1e-13)
    np.testing.assert_allclose(r["u_neq"], 0.0, atol=1e-14)


@pytest.mark.parametrize("ny", [4, 9, 40])
def test_ns_profile_keeps_mass_flow_and_centre(ny):
    y = nodes(ny)
    u = 1.0 + 0.2 * np.cos(3 * (y - 0.5)) - 0.7 * (y - 0.5) ** 4 + 0.05 * np.exp(-30 * y)
    r = profile.analyse(u)
    assert np.mean(r["u_ns"]) == pytest.approx(np.mean(u), rel=1e-14)
    assert abs(np.mean(r["u_neq"])) < 1e-15
    if ny % 2:
        assert r["u_ns"][ny // 2] == pytest.approx(r["u_center"], rel=1e-15)
    assert np.max(np.abs(r["u_neq"])) > 1e-4      # a genuine non-parabolic part


def test_discrete_ns_profile_tends_to_continuum_formula():
    def continuum(u, ny):
        y = nodes(ny)
        z = y - 0.5
        r = profile.analyse(u)
        m = np.mean(u)   # the integral in Eq. uNS by the midpoint rule
        return r["u_center"] * (1 - 3 * (1 - m / r["u_center"]) * (z / 0.5) ** 2), r["u_ns"]
    scaled = []
    for ny in (11, 21, 41, 81, 161):
        y = nodes(ny)
        u = 1.0 + 0.4 * y * (1 - y) + 0.3 * (y * (1 - y)) ** 2
        c, d = continuum(u, ny)
        scaled.append(np.max(np.abs(c - d)) * ny ** 2)
    # second order: err * ny^2 settles to a constant
    assert all(0.7 < scaled[k] / scaled[-1] <= 1.0 for k in range(4)), scaled
    assert abs(scaled[-2] / scaled[-1] - 1) < 0.02, scaled


def test_even_centre_is_exact_for_cubics():
    ny = 10
    y = nodes(ny)
    u = 1 + y - 2 * y ** 2 + 0.7 * y ** 3
    r = profile.analyse(u)
    assert r["u_center"] == pytest.approx(1 + 0.5 - 0.5 + 0.7 / 8, rel=1e-14)


# ---------------------------------------------------------------------------
# library (host, C ABI) against the oracle
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("ny", [3, 4, 5, 8, 40, 41, 512])
def test_library_matches_oracle(ny):
    from paper_1510_08886_amd import lbm
    try:
        lbm.lib()
    except Exception as e:  # pragma: no cover - library not built
        pytest.skip(f"library not built: {e}")
    rng = np.random.default_rng(ny)
    u = 1.0 + rng.standard_normal(ny) * 0.1
    ro, rg = profile.analyse(u), lbm.profile_analysis(u)
    for k in ("u_wall", "u_center", "slip", "mean"):
        assert rg[k] == pytest.approx(ro[k], rel=1e-14, abs=1e-15), k
    np.testing.assert_allclose(rg["u_ns"], ro["u_ns"], rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(rg["u_neq"], ro["u_neq"], rtol=0, atol=1e-13)


def test_library_rejects_short_profiles():
    from paper_1510_08886_amd import lbm
    try:
        lbm.lib()
    except Exception as e:  # pragma: no cover
        pytest.skip(f"library not built: {e}")
    for ny in (1, 2):
        with pytest.raises(lbm.LbmError):
            lbm.profile_analysis(np.ones(ny))
