"""Pins of the oracle parts that the paper leaves to a reading: the viscosity
of the two phases (R14) through the relaxation rate (Sec. 2), the stencil
ghosts at walls (R15), and the sign of the psi term where P > P0 (R3,
Sec. 2.3).  Each test compares the oracle with something it does not compute
itself: a measured decay rate against the closed form nu = cs^2 (1/omega -
1/2), the walled grid against a doubled periodic grid that holds the mirror
image explicitly, and the force against a finite difference of -(P - P0).
CPU only."""
import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import oracle as O


@pytest.fixture(autouse=True)
def _one_thread():
    """The grids here are tiny: one oracle thread avoids OpenMP overhead."""
    prev = O.set_threads(0)
    O.set_threads(1)
    yield
    O.set_threads(prev)


def _grid(D, n):
    axes = [np.arange(k, dtype=float) for k in n[:D]]
    mesh = np.meshgrid(*axes, indexing="ij")
    return [m.transpose(tuple(range(D))[::-1]).reshape(-1) for m in mesh]


# ------------------------------------------------------------- R14 and omega

# viscosity anchors of the interpolation (reading R14) and the two phase
# viscosities; the EOS (set a = 2/49, b = 2/21 at T/Tc = 0.8) has its stable
# vapour branch up to rho ~ 0.9, so every uniform state below stays uniform
RHO_V, RHO_L, NU_V, NU_L = 0.1, 0.2, 0.1, 0.02


def _nu_of(rho):
    """R14 written out: nu_v at and below rho_v, nu_l at and above rho_l,
    linear in rho between."""
    x = min(max((rho - RHO_V) / (RHO_L - RHO_V), 0.0), 1.0)
    return NU_V + (NU_L - NU_V) * x


def _shear_wave_nu(D, rho0, collision, L=32, U=1e-3, t1=20, t2=220):
    """Kinematic viscosity measured from the decay of u_y = U sin(2 pi x / L)
    on a uniform density rho0 (F = 0 and Phi = 0 there): the mode decays as
    exp(-nu k^2 t)."""
    n = (L, 4, 1) if D == 2 else (L, 4, 4)
    p = O.Params(D=D, n=n, collision=collision, kappa=0.03, nu_l=NU_L, nu_v=NU_V, rho_l=RHO_L, rho_v=RHO_V)
    X = _grid(D, n)
    k = 2 * np.pi / L
    rho = np.full(p.N, rho0)
    u = np.zeros((D, p.N))
    u[1] = U * np.sin(k * X[0])
    f = O.init_equilibrium(p, rho, u)
    amp = []
    for t in (t1, t2 - t1):
        O.step(p, f, t)
        r, uu, _ = O.macros(p, f)
        assert np.abs(r - rho0).max() < 1e-6 * rho0           # stays uniform (to O(U^2))
        amp.append(2 * np.mean(uu[1] * np.sin(k * X[0])))
    return np.log(amp[0] / amp[1]) / (k * k * (t2 - t1))


@pytest.mark.parametrize("D,collision,rho0", [(2, c, r) for c in (0, 1) for r in (0.05, 0.1, 0.125, 0.18, 0.2, 0.3)]
                         + [(3, 0, r) for r in (0.1, 0.125, 0.2)] + [(3, 1, 0.18)])
def test_viscosity_of_each_density_from_shear_wave_decay(D, collision, rho0):
    """The shear-wave decay measures nu = cs^2 (1/omega - 1/2), so it pins
    omega = 1/(3 nu + 1/2) (Sec. 2) and the interpolation of nu in rho (R14)
    at both anchors, inside and beyond them, within 1 %."""
    nu = _shear_wave_nu(D, rho0, collision)
    expect = _nu_of(rho0)
    assert abs(nu / expect - 1) < 0.01, (nu, expect)


def test_relaxation_rate_closed_form():
    """omega = dt / (rho nu / P0 + dt/2) with P0 = rho cs^2 (Sec. 2)."""
    p = O.Params(D=2, n=(4, 4, 1), nu_l=NU_L, nu_v=NU_V, rho_l=RHO_L, rho_v=RHO_V)
    for rho0 in (0.05, 0.1, 0.15, 0.2, 0.3):
        assert abs(O.omega(p, rho0) - 1.0 / (3.0 * _nu_of(rho0) + 0.5)) < 1e-15


# ------------------------------------------------------------------ R15 walls


def _mirror_velocity_index(D, axis):
    c = O.velocities(D)
    m = c.copy()
    m[:, axis] *= -1
    return np.array([int(np.where((c == v).all(axis=1))[0][0]) for v in m])


def _mirror_doubled(D, n, axis, f):
    """A grid twice as long along 'axis' holding f in its first half and the
    mirror image about the plane -1/2 (equivalently n - 1/2) in the second:
    cell 2n-1-k of the copy = cell k with the axis component of every
    velocity reversed.  Periodic along the doubled axis, the copy's cells -1
    and -2 are the mirror images of cells 0 and 1."""
    shape = tuple(n[:D][::-1]) + (f.shape[1],)
    g = f.reshape(shape)
    ax = D - 1 - axis                      # numpy axis of the grid axis
    mir = np.flip(g, axis=ax)[..., _mirror_velocity_index(D, axis)]
    return np.concatenate([g, mir], axis=ax).reshape(-1, f.shape[1])


def _drop_near_wall(D, n, axis, seed=4):
    rv, rl = 0.19712191, 7.2038517
    X = _grid(D, n)
    c = [(k - 1) / 2 for k in n[:D]]
    c[axis] = 2.5                          # the interface crosses the wall rows
    r = np.sqrt(sum((X[a] - c[a]) ** 2 for a in range(D)))
    rho = (rl + rv) / 2 - (rl - rv) / 2 * np.tanh(2 * (r - 4.0) / 4.0)
    u = np.random.default_rng(seed).uniform(-0.02, 0.02, (D, rho.size))
    return rho, u, rv, rl


@pytest.mark.parametrize("D,n,axis", [(2, (14, 12, 1), 1), (2, (12, 14, 1), 0), (3, (9, 8, 10), 2),
                                      (3, (10, 9, 8), 1)])
def test_wall_ghosts_equal_mirrored_periodic_grid(D, n, axis):
    """Reading R15: at a wall the stencils see the density mirrored about the
    wall plane (rho(-1) = rho(0), rho(-2) = rho(1)) and the wall-normal flux of
    Phi odd.  The force on the walled grid equals the force on the doubled
    periodic grid that holds the mirror image; one step on both (the walled
    one with half-way bounce-back, the doubled one plain periodic) gives the
    same populations in every cell that is not next to a wall, whose pulls
    then come from post-collision states that include the wall rows and hence
    the ghosts of both stencils and of Phi."""
    rho, u, rv, rl = _drop_near_wall(D, n, axis)
    bc = [0, 0, 0]
    bc[axis] = 1
    pw = O.Params(D=D, n=n, bc=tuple(bc), kappa=0.03, nu_l=0.05, nu_v=0.08, rho_l=rl, rho_v=rv)
    n2 = list(n)
    n2[axis] *= 2
    pp = O.Params(D=D, n=tuple(n2), bc=(0, 0, 0), kappa=0.03, nu_l=0.05, nu_v=0.08, rho_l=rl, rho_v=rv)
    # force: the walled grid against the mirrored doubled grid
    fw = O.init_equilibrium(pw, rho, u)
    fp = _mirror_doubled(D, n, axis, fw)
    rw, _, _ = O.macros(pw, fw)
    rp, _, _ = O.macros(pp, fp)
    Fw = O.force_field(pw, rw)
    Fp = O.force_field(pp, rp)
    half = _grid(D, n2)[axis] < n[axis]
    np.testing.assert_allclose(Fw, Fp[:, half], rtol=0, atol=1e-13)
    # one step
    O.step(pw, fw, 1)
    O.step(pp, fp, 1)
    X = _grid(D, n)
    inner = (X[axis] >= 1) & (X[axis] <= n[axis] - 2)
    np.testing.assert_allclose(fw[inner], fp[half][inner], rtol=0, atol=1e-14 * rl)


# ------------------------------------------------------------- R3: P > P0

EOS_B = dict(a=0.003, b=0.095, Tr=0.592454)   # density ratio 1000; P = P0 at rho = 10.4318


def _pr(p):
    Tc = 0.0778 * p.a / (0.45724 * p.b * p.R)
    m = 0.37464 + 1.54226 * p.acentric - 0.26992 * p.acentric ** 2
    aal = p.a * (1 + m * (1 - np.sqrt(p.Tr))) ** 2
    RT = p.R * p.Tr * Tc
    return lambda r: r * RT / (1 - p.b * r) - aal * r * r / (1 + 2 * p.b * r - p.b ** 2 * r * r)


@pytest.mark.parametrize("D,n", [(2, (12, 11, 1)), (3, (9, 10, 9))])
def test_psi_term_above_p0_is_minus_grad(D, n):
    """Where P > P0 the psi term takes the minus sign (R3): with psi = sqrt(P
    - P0) it is -2 psi grad(psi) = -grad(P - P0), and the fourth-order psi
    stencil makes it exact for quartic psi.  The field lies in the compressed
    liquid 10.44 <= rho <= 10.5 of the ratio-1000 EOS, above the crossing
    P = P0 at rho = 10.432."""
    rng = np.random.default_rng(9)
    p = O.Params(D=D, n=n, kappa=0.0, **EOS_B)
    P = _pr(p)
    psi_of = lambda r: np.sqrt(P(r) - r / 3.0)
    X = _grid(D, n)
    cen = [x - (k - 1) / 2 for x, k in zip(X, n)]
    lin = rng.uniform(-0.02, 0.02, D)
    quad = rng.uniform(-4e-4, 4e-4, D)
    quart = rng.uniform(-2e-5, 2e-5, D)
    target = 1.5 + sum(lin[a] * cen[a] + quad[a] * cen[a] ** 2 + quart[a] * cen[a] ** 4 for a in range(D))
    rho = np.array([brentq(lambda r: psi_of(r) - t, 10.435, 10.52, xtol=1e-15, rtol=1e-15) for t in target])
    assert rho.min() >= 10.44 and rho.max() <= 10.5
    assert np.all(P(rho) > rho / 3.0)
    psi = psi_of(rho)
    G = -O.force_field(p, rho) / (2 * psi)
    ok = np.ones(p.N, dtype=bool)
    for a in range(D):
        ok &= (X[a] >= 2) & (X[a] <= n[a] - 3)
    for a in range(D):
        grad = lin[a] + 2 * quad[a] * cen[a] + 4 * quart[a] * cen[a] ** 3
        np.testing.assert_allclose(G[a][ok], grad[ok], atol=3e-12)


def test_psi_term_follows_minus_grad_on_both_sides_of_the_crossing():
    """A 1-D density field through the crossing P = P0 (rho from 10.2 to
    10.47): the psi term follows -grad(P - P0) on both sides; the cells whose
    stencil reaches within a cell of the crossing (where |psi| has a cusp and
    steep derivatives) are excluded."""
    L = 64
    p = O.Params(D=2, n=(L, 3, 1), kappa=0.0, **EOS_B)
    P = _pr(p)
    x = np.tile(np.arange(L, dtype=float), 3)
    rho = 10.335 + 0.135 * np.sin(2 * np.pi * x / L)
    F = O.force_field(p, rho)[0]
    g = -(P(rho) - rho / 3)
    gg = g.reshape(3, L)
    dg = ((-np.roll(gg, -2, 1) + 8 * np.roll(gg, -1, 1) - 8 * np.roll(gg, 1, 1) + np.roll(gg, 2, 1)) / 12).reshape(-1)
    above = P(rho) > rho / 3
    assert above.any() and (~above).any()
    near = np.zeros(L, dtype=bool)
    ab = above.reshape(3, L)[0]
    for s in range(-3, 4):
        near |= ab != np.roll(ab, s)
    far = ~np.tile(near, 3)
    for side in (above & far, ~above & far):
        err = np.abs(F[side] - dg[side]).max() / np.abs(dg[side]).max()
        assert err < 0.03, err
        assert np.corrcoef(F[side], dg[side])[0, 1] > 0.999


# ------------------------------------------------------------------ Phi


@pytest.mark.parametrize("D,n", [(2, (16, 12, 1)), (3, (10, 8, 6))])
def test_phi_correction_enters_the_extended_equilibrium(D, n):
    """Sec. 2.2: Phi_aa = (1 - omega/2) dt d_a q_a with the flux q_a = rho u_a
    (u_a^2 + 3 P0/rho - 3 cs^2) = rho u_a^3 (P0 = rho cs^2), differentiated by
    a central difference (R5), enters zeta*_a = P0/rho + u_a^2 + Phi_aa/rho of
    the extended equilibrium.  On a uniform density (F = 0) started at f =
    f^eq, the non-equilibrium parts vanish and the post-collision state is f*
    itself, so one step must give f_i(r) = f*_i(r - c_i) with f* the product
    form (Sec. 2.1) at those values, written out here from the definitions."""
    rho0, nu = 0.15, 0.05
    p = O.Params(D=D, n=n, kappa=0.03, nu_l=nu, nu_v=nu)
    X = _grid(D, n)
    u = np.zeros((D, p.N))
    u[0] = 0.02 + 0.08 * np.sin(2 * np.pi * X[0] / n[0]) + 0.01 * np.cos(2 * np.pi * X[1] / n[1])
    u[1] = 0.01 + 0.05 * np.cos(2 * np.pi * X[1] / n[1]) + 0.02 * np.sin(2 * np.pi * X[0] / n[0])
    if D == 3:
        u[2] = -0.01 + 0.04 * np.sin(2 * np.pi * X[2] / n[2])
    f = O.init_equilibrium(p, np.full(p.N, rho0), u)
    O.step(p, f, 1)
    omega = 1.0 / (3.0 * nu + 0.5)
    shape = tuple(n[:D][::-1])
    q = rho0 * u ** 3
    phi = np.zeros((D, p.N))
    for a in range(D):
        qa = q[a].reshape(shape)
        ax = D - 1 - a
        phi[a] = ((1 - omega / 2) * (np.roll(qa, -1, ax) - np.roll(qa, 1, ax)) / 2).reshape(-1)
    zeta = 1.0 / 3.0 + u ** 2 + phi / rho0
    c = O.velocities(D)
    fstar = np.full((p.N, len(c)), rho0)
    for i, ci in enumerate(c):
        for a in range(D):
            fstar[:, i] *= (1 - zeta[a]) if ci[a] == 0 else 0.5 * (ci[a] * u[a] + zeta[a])
    expect = np.empty_like(fstar)
    for i, ci in enumerate(c):
        g = fstar[:, i].reshape(shape)
        for a in range(D):
            g = np.roll(g, int(ci[a]), D - 1 - a)
        expect[:, i] = g.reshape(-1)
    np.testing.assert_allclose(f, expect, rtol=0, atol=1e-15)
    assert np.abs(phi).max() > 1e-5


# --------------------------------------------------------------- body force


@pytest.mark.parametrize("D,nu,collision", [(2, 1.0 / 6.0, 0), (2, 1.0 / 6.0, 1), (2, 0.1, 0), (3, 0.1, 0)])
def test_body_force_poiseuille_between_halfway_walls(D, nu, collision):
    """A uniform body force rho g along x between walls (half-way bounce-back,
    reading R15) drives plane Poiseuille flow whose fluid velocity u + F/(2
    rho) is the parabola g/(2 nu) (y + 1/2)(H - 1/2 - y): the walls sit half a
    cell outside the first and last nodes.  Within 1 % of the peak (the
    measured departure is 0.15-0.5 %; a wall on the nodes or a force of the
    wrong size misses by > 10 %)."""
    H, g = 16, 1e-5
    n = (4, H, 1) if D == 2 else (4, 4, H)
    bc = (0, 1, 0) if D == 2 else (0, 0, 1)
    p = O.Params(D=D, n=n, bc=bc, collision=collision, kappa=0.03, nu_l=nu, nu_v=nu, g=(g, 0.0, 0.0))
    rho0 = 0.15
    f = O.init_fluid(p, np.full(p.N, rho0), np.zeros((D, p.N)))
    O.step(p, f, int(6 * H * H / nu / 10))
    r, u, _ = O.macros(p, f)
    assert np.abs(r - rho0).max() < 1e-6 * rho0
    ux = u[0] + g / 2.0
    wall_axis = _grid(D, n)[D - 1]
    exact = g / (2 * nu) * (wall_axis + 0.5) * (H - 0.5 - wall_axis)
    err = np.abs(ux - exact).max() / exact.max()
    assert err < 0.01, err
    assert np.abs(u[1:]).max() < 1e-5 * exact.max()


# ------------------------------------------------------- kappa from a width


def _slab(tr, W, nu=0.1, phi=0, steps=None, kappa=None):
    """Liquid slab in vapour (EOS a = 0.003, b = 0.095), 1-D along x, tanh
    interfaces of width W, run to equilibrium; returns (rho along x, rho_v,
    rho_l of the Maxwell rule)."""
    a, b = 0.003, 0.095
    rv, rl, _ = O.maxwell(a, b, 1.0, 0.344, tr)
    k = O.kappa_for_width(a, b, 1.0, 0.344, tr, W) if kappa is None else kappa
    L = int(12 * W)
    p = O.Params(D=2, n=(L, 3, 1), a=a, b=b, Tr=tr, kappa=k, nu_l=nu, nu_v=nu, phi_velocity=phi)
    x = np.tile(np.arange(L, dtype=float), 3)
    rho0 = rv + (rl - rv) * 0.5 * (np.tanh(2 * (x - L / 4) / W) - np.tanh(2 * (x - 3 * L / 4) / W))
    f = O.init_fluid(p, rho0, np.zeros((2, p.N)))
    O.step(p, f, steps if steps is not None else int(20 * W * W))
    r, _, _ = O.macros(p, f)
    return r[:L], rv, rl


def test_kappa_for_width_vanishing_potential_at_coexistence():
    """The excess grand potential behind kappa~(W) vanishes at both
    coexistence densities (Maxwell's equal areas), so kappa~ scales as W^2
    exactly and is positive."""
    for tr in (0.6, 0.8, 0.9):
        k1 = O.kappa_for_width(0.003, 0.095, 1.0, 0.344, tr, 5.0)
        k2 = O.kappa_for_width(0.003, 0.095, 1.0, 0.344, tr, 10.0)
        assert k1 > 0 and abs(k2 / k1 - 4.0) < 1e-12


@pytest.mark.slow
def test_kappa_for_width_gives_that_width_in_the_continuum_limit():
    """kappa~(W) is the square-gradient capillarity of an interface of width
    W = (rho_l - rho_v) / max |d rho/dx| (Sec. 3.1.1).  The model's force
    (Sec. 2.3) has the square-gradient equilibrium as its continuum limit, so
    the converged width of a flat interface approaches W as W grows: the
    measured ratios at W = 16 and 24 (1.18, 1.085 at T/Tc = 0.9) fall off as
    W^-2, and their quadratic extrapolation is 1 within 2 %.  A kappa~ off by a
    factor c would extrapolate to sqrt(c)."""
    ratios = {}
    for W in (16, 24):
        r, _, _ = _slab(0.9, W)
        grad = np.abs(np.roll(r, -1) - np.roll(r, 1)) / 2
        ratios[W] = (r.max() - r.min()) / grad.max() / W
    limit = (ratios[24] * 24 ** 2 - ratios[16] * 16 ** 2) / (24 ** 2 - 16 ** 2)
    assert ratios[16] > ratios[24] > 1.0
    assert abs(limit - 1.0) < 0.02, (ratios, limit)


# ------------------------------------------------- readings R4 and R6


def test_phi_with_fluid_velocity_makes_coexistence_independent_of_viscosity():
    """Reading R4 and its alternative: at rest the bare velocity is -F/(2 rho)
    near an interface, so with the bare velocity the flux of Phi, and the
    vapour density it leaves, depend on nu; with the fluid velocity u + F/(2
    rho) (phi_velocity = 1) the flux vanishes at rest and the coexistence no
    longer depends on nu (flat interface, T/Tc = 0.6, nu = 0.1 and 0.03)."""
    out = {}
    for phi in (0, 1):
        out[phi] = [(_slab(0.6, 6, nu=nu, phi=phi, steps=6000, kappa=O.kappa_for_width(0.003, 0.095, 1.0, 0.344, 0.6, 6)))
                    for nu in (0.1, 0.03)]
    rv_of = {phi: [r.min() / rv - 1 for r, rv, _ in out[phi]] for phi in out}
    assert abs(rv_of[1][0] - rv_of[1][1]) < 0.003, rv_of
    assert abs(rv_of[0][0] - rv_of[0][1]) > 0.05, rv_of
    for phi in out:
        for r, _, rl in out[phi]:
            assert abs(r.max() / rl - 1) < 0.001


@pytest.mark.parametrize("D", [2, 3])
def test_trace_in_s_split_equals_explicit_projection(D):
    """Reading R6 and its alternative: with trace_in_s the trace of the
    second-order central moments moves from h to s; both splits equal the
    projections by explicit inversion of the modified central Hermite basis
    (Appendix A), and k + s + h = f either way."""
    import basis_np as B
    rng = np.random.default_rng(5)
    for _ in range(5):
        u = rng.uniform(-0.1, 0.1, D)
        f = O.equilibrium(D, 1.3, u) * (1 + rng.uniform(-0.05, 0.05, 3 ** D))
        for tis in (False, True):
            k, s, h = O.split(D, u, f, trace_in_s=int(tis))
            np.testing.assert_allclose(s, B.project(D, u, f, "stress", tis), atol=1e-14)
            np.testing.assert_allclose(h, B.project(D, u, f, "h", tis), atol=1e-14)
            np.testing.assert_allclose(k + s + h, f, atol=1e-14)
        s0 = O.split(D, u, f, 0)[1]
        assert np.abs(s - s0).max() > 1e-6
