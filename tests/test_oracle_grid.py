"""Pins of the oracle's grid operations: force stencils on polynomial fields
(Sec. 2.3), conservation, invariance of uniform states and mirror symmetry.
CPU only, small grids."""
import numpy as np
import pytest
from scipy.optimize import brentq

import basis_np as B
from oracle import oracle as O


def _grid(D, n):
    axes = [np.arange(k, dtype=float) for k in n[:D]]
    mesh = np.meshgrid(*axes, indexing="ij")          # mesh[a][x, y, (z)]
    # flatten in cell order x fastest: transpose to (z, y, x)
    return [m.transpose(tuple(range(D))[::-1]).reshape(-1) for m in mesh]


def _interior(D, n, margin=2):
    X = _grid(D, n)
    ok = np.ones(X[0].size, dtype=bool)
    for a in range(D):
        ok &= (X[a] >= margin) & (X[a] <= n[a] - 1 - margin)
    return ok


def _pr(p):
    Tc = 0.0778 * p.a / (0.45724 * p.b * p.R)
    m = 0.37464 + 1.54226 * p.acentric - 0.26992 * p.acentric ** 2
    aal = p.a * (1 + m * (1 - np.sqrt(p.Tr))) ** 2
    RT = p.R * p.Tr * Tc
    return lambda r: r * RT / (1 - p.b * r) - aal * r * r / (1 + 2 * p.b * r - p.b ** 2 * r * r)


@pytest.mark.parametrize("D,n", [(2, (12, 11, 1)), (3, (9, 8, 10))])
def test_capillary_stencil_is_grad_laplacian_on_cubics(D, n):
    """kappa part of the force: kappa rho sum (w/cs^2) c [rho(r+2c) - 2 rho(r+c)]
    equals kappa rho grad(lap rho) exactly for cubic rho (reading R2)."""
    rng = np.random.default_rng(7)
    X = _grid(D, n)
    cen = [x - (k - 1) / 2 for x, k in zip(X, n)]
    coef = rng.uniform(-1e-3, 1e-3, (D, D, D))
    lin = rng.uniform(-0.02, 0.02, D)
    rho = 4.0 + sum(lin[a] * cen[a] for a in range(D))
    for a in range(D):
        for b in range(D):
            for c in range(D):
                rho = rho + coef[a, b, c] * cen[a] * cen[b] * cen[c]
    # analytic grad(lap rho) of the cubic: symmetrise the coefficient tensor
    S = np.zeros((D, D, D))
    import itertools
    for a, b, c in itertools.product(range(D), repeat=3):
        for perm in set(itertools.permutations((a, b, c))):
            S[perm] += coef[a, b, c] / len(set(itertools.permutations((a, b, c))))
    # rho = sum S_abc x_a x_b x_c ; d_a lap rho = 6 sum_b S_abb
    expect = np.array([6 * sum(S[a, b, b] for b in range(D)) for a in range(D)])
    p1 = O.Params(D=D, n=n, kappa=1.0, a=0.003, b=0.095, Tr=0.8)
    p0 = O.Params(D=D, n=n, kappa=0.0, a=0.003, b=0.095, Tr=0.8)
    K = (O.force_field(p1, rho) - O.force_field(p0, rho)) / rho
    ok = _interior(D, n)
    for a in range(D):
        np.testing.assert_allclose(K[a][ok], expect[a], atol=1e-12)


@pytest.mark.parametrize("D,n", [(2, (12, 11, 1)), (3, (9, 10, 9))])
def test_psi_stencil_is_fourth_order_gradient(D, n):
    """psi part: +2 psi sum (w/cs^2) c [4/3 psi(r+c) - 1/6 psi(r+2c)] equals
    2 psi grad(psi) exactly for quartic psi (error O(dr^5)), where P <= P0."""
    rng = np.random.default_rng(8)
    p = O.Params(D=D, n=n, kappa=0.0, a=0.003, b=0.095, Tr=0.8)
    P = _pr(p)
    psi_of = lambda r: np.sqrt(r / 3.0 - P(r))
    X = _grid(D, n)
    cen = [x - (k - 1) / 2 for x, k in zip(X, n)]
    # quartic psi field in the liquid range where psi(rho) is monotone
    lin = rng.uniform(-0.01, 0.01, D)
    quad = rng.uniform(-2e-4, 2e-4, D)
    quart = rng.uniform(-1e-5, 1e-5, D)
    target = 1.4 + sum(lin[a] * cen[a] + quad[a] * cen[a] ** 2 + quart[a] * cen[a] ** 4
                       for a in range(D))
    rho = np.array([brentq(lambda r: psi_of(r) - t, 3.0, 9.0, xtol=1e-15, rtol=1e-15)
                    for t in target])
    psi = psi_of(rho)
    assert np.all(P(rho) <= rho / 3.0)
    G = O.force_field(p, rho) / (2 * psi)
    ok = _interior(D, n)
    for a in range(D):
        grad = lin[a] + 2 * quad[a] * cen[a] + 4 * quart[a] * cen[a] ** 3
        np.testing.assert_allclose(G[a][ok], grad[ok], atol=3e-13)


def test_force_sign_follows_minus_grad_nonideal_pressure():
    """Continuum model (Sec. 2): the psi term approximates -grad(P - P0)."""
    n = (40, 3, 1)
    p = O.Params(D=2, n=n, kappa=0.0, a=0.003, b=0.095, Tr=0.8)
    P = _pr(p)
    x = np.tile(np.arange(40, dtype=float), 3)
    rho = 3.0 + 0.5 * np.sin(2 * np.pi * x / 40)
    F = O.force_field(p, rho)
    g = -(P(rho) - rho / 3)
    dg = (np.roll(g.reshape(3, 40), -1, 1) - np.roll(g.reshape(3, 40), 1, 1)).reshape(-1) / 2
    assert np.corrcoef(F[0], dg)[0, 1] > 0.999
    np.testing.assert_allclose(F[0], dg, atol=0.02 * np.abs(dg).max())


def _drop_state(D, n, seed=0, noise=1e-4, centre=None, R=None):
    rv, rl = 0.19712191, 7.2038517
    X = _grid(D, n)
    c = centre if centre is not None else [(k - 1) / 2 for k in n[:D]]
    r = np.sqrt(sum((X[a] - c[a]) ** 2 for a in range(D)))
    R = R if R is not None else min(n[:D]) / 4
    rho = (rl + rv) / 2 - (rl - rv) / 2 * np.tanh(2 * (r - R) / 4)
    rng = np.random.default_rng(seed)
    u = rng.uniform(-noise, noise, (D, rho.size))
    return rho, u, rv, rl


@pytest.mark.parametrize("D,n,bc", [(2, (24, 20, 1), (0, 0, 0)), (2, (24, 20, 1), (0, 1, 0)),
                                    (3, (12, 10, 11), (0, 0, 0)), (3, (12, 10, 11), (0, 0, 1))])
@pytest.mark.parametrize("collision", [0, 1])
def test_mass_and_momentum_conservation(D, n, bc, collision):
    """Mass is conserved to roundoff by every step; momentum too when every
    axis is periodic (both stencils are pairwise antisymmetric)."""
    rho0, u0, rv, rl = _drop_state(D, n)
    p = O.Params(D=D, n=n, bc=bc, collision=collision, kappa=0.03, nu_l=0.05, nu_v=0.05,
                 rho_l=rl, rho_v=rv)
    f = O.init_equilibrium(p, rho0, u0)
    _, _, s0 = O.macros(p, f)
    st = O.step(p, f, 20)
    _, _, s1 = O.macros(p, f)
    assert st.nonfinite == 0
    assert abs(s1[0] - s0[0]) <= 1e-13 * s0[0]
    if bc == (0, 0, 0):
        np.testing.assert_allclose(s1[1:1 + D], s0[1:1 + D], atol=1e-12 * s0[0])


@pytest.mark.parametrize("D,n", [(2, (10, 9, 1)), (3, (7, 6, 8))])
@pytest.mark.parametrize("u", [0.0, 1.0])
def test_uniform_states_are_invariant(D, n, u):
    """A uniform state (at rest or moving) has F = 0 and Phi = 0, so f = f^eq
    is a fixed point of the step."""
    vel = u * np.array([0.05, -0.03, 0.02])[:D]
    p = O.Params(D=D, n=n, kappa=0.03, rho_l=7.2, rho_v=0.2)
    N = p.N
    rho0 = np.full(N, 2.3)
    u0 = np.tile(vel[:, None], (1, N))
    f = O.init_equilibrium(p, rho0, u0)
    f0 = f.copy()
    O.step(p, f, 5)
    np.testing.assert_allclose(f, f0, atol=2e-15 * 2.3)


def _mirror_x_index(D):
    c = B.velocities(D)
    cm = c.copy()
    cm[:, 0] *= -1
    return np.array([np.where((c == v).all(axis=1))[0][0] for v in cm])


@pytest.mark.parametrize("D,n", [(2, (20, 18, 1)), (3, (10, 9, 8))])
def test_mirror_symmetry_of_centred_drop(D, n):
    """A drop centred on a symmetric grid with zero initial velocity keeps its
    mirror symmetry x -> n-1-x (up to summation order)."""
    rho0, _, rv, rl = _drop_state(D, n, noise=0.0)
    u0 = np.zeros((D, rho0.size))
    p = O.Params(D=D, n=n, kappa=0.03, rho_l=rl, rho_v=rv)
    f = O.init_equilibrium(p, rho0, u0)
    O.step(p, f, 30)
    fx = f.reshape(tuple(n[::-1][(3 - D):]) + (p.Q,)) if D == 3 else f.reshape(n[1], n[0], p.Q)
    mir = _mirror_x_index(D)
    flipped = np.flip(fx, axis=-2)[..., mir]
    np.testing.assert_allclose(flipped, fx, atol=1e-12 * rl)


def test_update_cells_matches_full_step():
    """The sampled single-cell update equals the whole-grid step."""
    for D, n, bc in [(2, (14, 12, 1), (0, 1, 0)), (3, (8, 7, 9), (0, 0, 1))]:
        rho0, u0, rv, rl = _drop_state(D, n, R=3)
        p = O.Params(D=D, n=n, bc=bc, kappa=0.03, rho_l=rl, rho_v=rv, nu_l=0.02, nu_v=0.05)
        f = O.init_equilibrium(p, rho0, u0)
        O.step(p, f, 3)
        cells = np.random.default_rng(3).choice(p.N, 25, replace=False)
        part = O.update_cells(p, f, cells)
        O.step(p, f, 1)
        np.testing.assert_allclose(part, f[cells], rtol=0, atol=1e-15 * rl)


@pytest.mark.parametrize("D,n,bc", [(2, (20, 18, 1), (0, 0, 0)), (2, (20, 18, 1), (0, 1, 0)),
                                    (3, (9, 8, 10), (0, 0, 1))])
def test_fluid_velocity_initialisation(D, n, bc):
    """With the exact-difference forcing the fluid velocity is u + F/(2 rho);
    the initial state built from a prescribed fluid velocity u0 has density
    rho0 and u + F(rho)/(2 rho) = u0 (definition checked from the populations)."""
    rho0, _, rv, rl = _drop_state(D, n, R=4)
    u0 = np.random.default_rng(2).uniform(-0.01, 0.01, (D, rho0.size))
    p = O.Params(D=D, n=n, bc=bc, kappa=0.03, rho_l=rl, rho_v=rv)
    f = O.init_fluid(p, rho0, u0)
    rho, u, _ = O.macros(p, f)
    F = O.force_field(p, rho)
    np.testing.assert_allclose(rho, rho0, rtol=0, atol=1e-14 * rl)
    np.testing.assert_allclose(u + F / (2 * rho), u0, rtol=0, atol=1e-14)
    # and it is the equilibrium there: the non-equilibrium part vanishes
    c = B.velocities(D).astype(float)
    for cell in (0, rho0.size // 2, rho0.size - 1):
        np.testing.assert_allclose(f[cell], O.equilibrium(D, rho[cell], u[:, cell]), atol=1e-15 * rl)


@pytest.mark.parametrize("bad", [float("nan"), -0.1, 0.0])
def test_step_counts_cells_without_a_valid_density(bad):
    """The failure mode of the method is a density that stops being finite
    and positive: a state holding one such cell is reported by the step's
    statistics (the check the library's instability flag mirrors)."""
    rho0, u0, rv, rl = _drop_state(2, (24, 20, 1))
    p = O.Params(D=2, n=(24, 20, 1), bc=(0, 0, 0), kappa=0.03, nu_l=0.05, nu_v=0.05, rho_l=rl, rho_v=rv)
    f = O.init_equilibrium(p, rho0, u0)
    st = O.step(p, f, 1)
    assert st.nonfinite == 0
    rho1 = rho0.copy()
    rho1[5 + 24 * 7] = bad
    f = O.init_equilibrium(p, rho1, u0)
    st = O.step(p, f, 1)
    assert st.nonfinite >= 1
