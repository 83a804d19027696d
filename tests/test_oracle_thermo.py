"""Pins of the oracle's Peng-Robinson thermodynamics (Sec. 3.1): the brute-force
equal-area construction against the closed-form equal chemical potential
condition, corresponding states, and the paper's T_r = 0.59 for ratio 1000."""
import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import oracle as O

SQ2 = np.sqrt(2.0)


def _pr(a, b, R, acentric, Tr):
    Tc = 0.0778 * a / (0.45724 * b * R)
    m = 0.37464 + 1.54226 * acentric - 0.26992 * acentric ** 2
    aal = a * (1 + m * (1 - np.sqrt(Tr))) ** 2
    RT = R * Tr * Tc

    def P(r):
        return r * RT / (1 - b * r) - aal * r * r / (1 + 2 * b * r - b * b * r * r)

    def G(r):  # antiderivative of P / rho^2
        return RT * np.log(r / (1 - b * r)) - aal / (2 * SQ2 * b) * np.log(
            (1 + (1 + SQ2) * b * r) / (1 + (1 - SQ2) * b * r))

    return P, G


CASES = [
    (2 / 49, 2 / 21, 0.8),
    (2 / 49, 2 / 21, 0.6),
    (0.003, 0.095, 0.8),
    (0.003, 0.095, 0.592454),
    (0.0017, 0.095, 0.7),
    (0.0011, 0.095, 0.95),
]


@pytest.mark.parametrize("a,b,Tr", CASES)
def test_maxwell_bruteforce_vs_closed_form(a, b, Tr):
    """Equal area (Sec. 3.1.1) <=> P(rho_v) = P(rho_l) = P_sat and
    P_sat (1/rho_v - 1/rho_l) = G(rho_l) - G(rho_v) with G the exact
    antiderivative of P/rho^2."""
    rv, rl, ps = O.maxwell(a, b, 1.0, 0.344, Tr)
    P, G = _pr(a, b, 1.0, 0.344, Tr)
    assert rv < rl
    # the two PR terms nearly cancel in the liquid: roundoff scales with rho
    assert abs(P(rv) - ps) < 1e-14 * rv
    assert abs(P(rl) - ps) < 1e-14 * rl
    area = ps * (1 / rv - 1 / rl) - (G(rl) - G(rv))
    assert abs(area) < 1e-10 * ps / rv
    # independent closed-form solve: Newton-free root finding in P_sat
    def resid(psat):
        # outer roots of P = psat
        grid = np.linspace(1e-9, 1 / b * (1 - 1e-9), 200001)
        s = P(grid) - psat
        idx = np.where(np.sign(s[:-1]) != np.sign(s[1:]))[0]
        r1 = brentq(lambda r: P(r) - psat, grid[idx[0]], grid[idx[0] + 1], xtol=1e-15)
        r3 = brentq(lambda r: P(r) - psat, grid[idx[-1]], grid[idx[-1] + 1], xtol=1e-15)
        return psat * (1 / r1 - 1 / r3) - (G(r3) - G(r1))
    psat_cf = brentq(resid, ps * 0.9, ps * 1.1, xtol=1e-16, rtol=1e-15)
    assert abs(psat_cf - ps) < 1e-9 * ps


def test_corresponding_states():
    """The density ratio depends on T_r only (the reduced PR equation does not
    contain a, b)."""
    for Tr in (0.6, 0.8, 0.9):
        r1 = O.maxwell(2 / 49, 2 / 21, 1.0, 0.344, Tr)
        r2 = O.maxwell(0.003, 0.095, 1.0, 0.344, Tr)
        assert abs(r1[1] / r1[0] - r2[1] / r2[0]) < 1e-9 * (r1[1] / r1[0])
        # rho b is also invariant
        assert abs(r1[1] * 2 / 21 - r2[1] * 0.095) < 1e-11


def test_ratio_1000_temperature():
    """Sec. 3.2: T_r = 0.59 gives a density ratio of 10^3 (water/air)."""
    def ratio(Tr):
        rv, rl, _ = O.maxwell(0.003, 0.095, 1.0, 0.344, Tr)
        return rl / rv
    Tr = brentq(lambda t: ratio(t) - 1000.0, 0.55, 0.65, xtol=1e-10)
    assert round(Tr, 2) == 0.59
    assert abs(Tr - 0.592454) < 2e-6


def test_critical_temperature_definition():
    """Tc from a = 0.45724 R^2 Tc^2/Pc, b = 0.0778 R Tc/Pc: eliminating Pc."""
    for a, b, R in [(2 / 49, 2 / 21, 1.0), (0.003, 0.095, 1.0), (0.01, 0.2, 0.5)]:
        Tc = O.Tc(a, b, R)
        Pc = 0.0778 * R * Tc / b
        assert abs(0.45724 * R * R * Tc * Tc / Pc - a) < 1e-15 * a
