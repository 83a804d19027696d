"""Pins of the oracle's per-cell algebra against what the paper and the
mathematics fix (Sec. 2.1-2.4 and Appendix A).  CPU only."""
import numpy as np
import pytest
from scipy.optimize import minimize_scalar

import basis_np as B
from oracle import oracle as O

CS2 = 1.0 / 3.0


@pytest.mark.parametrize("D", [2, 3])
def test_weights_values_and_isotropy(D):
    """w_i = prod Psi(0, cs^2) (Sec. 2.3): D2Q9 {4/9, 1/9, 1/36};
    D3Q27 {8/27, 2/27, 1/54, 1/216}; isotropic to fourth order."""
    w = O.weights(D)
    c = B.velocities(D)
    nz = np.abs(c).sum(axis=1)
    table = {2: [4 / 9, 1 / 9, 1 / 36], 3: [8 / 27, 2 / 27, 1 / 54, 1 / 216]}[D]
    for k, val in enumerate(table):
        np.testing.assert_allclose(w[nz == k], val, rtol=0, atol=1e-15)
    assert abs(w.sum() - 1) < 1e-15
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, c, c), CS2 * np.eye(D), atol=1e-15)
    assert abs(np.einsum("i,i->", w, c[:, 0] ** 4) - 3 * CS2 ** 2) < 1e-15
    assert abs(np.einsum("i,i,i->", w, c[:, 0] ** 2, c[:, 1] ** 2) - CS2 ** 2) < 1e-15


@pytest.mark.parametrize("D", [2, 3])
def test_equilibrium_moments(D):
    """Central Hermite moments of f^eq are (rho, 0, ..., 0) (Appendix A); raw
    moments are rho, rho u, rho u u + rho cs^2 I."""
    rng = np.random.default_rng(1)
    c = B.velocities(D).astype(float)
    for _ in range(20):
        rho = rng.uniform(0.005, 9.0)
        u = rng.uniform(-0.15, 0.15, D)
        feq = O.equilibrium(D, rho, u)
        labs, M = B.matrix(D, u)
        a = M @ feq
        expect = np.array([rho if l == (0,) * D else 0.0 for l in labs])
        np.testing.assert_allclose(a, expect, rtol=0, atol=1e-14 * rho)
        np.testing.assert_allclose(feq @ c, rho * u, atol=1e-14 * rho)
        P = np.einsum("i,ia,ib->ab", feq, c, c)
        np.testing.assert_allclose(P, rho * np.outer(u, u) + rho * CS2 * np.eye(D), atol=1e-14 * rho)
        # the oracle's own moment routine agrees with the explicit basis
        ao = O.moments(D, u, feq)
        order = _oracle_order(D, labs)
        np.testing.assert_allclose(ao[order], a, atol=1e-14 * rho)


def _oracle_order(D, labs):
    """Index of each numpy label in the oracle's moment vector (tensor index
    m_x + 3 m_y + 9 m_z, diagonal block rows replaced in place)."""
    diag = {2: {"xx-yy": 2, "trace": 6}, 3: {"xx-yy": 2, "xx-zz": 6, "trace": 18}}[D]
    out = []
    for l in labs:
        if isinstance(l, tuple):
            out.append(sum(m * 3 ** a for a, m in enumerate(l)))
        else:
            out.append(diag[l])
    return np.array(out)


@pytest.mark.parametrize("D", [2, 3])
def test_extended_equilibrium_matches_appendix(D):
    """Central Hermite moments of f* equal the closed-form a* vectors of
    Appendix A, for random rho, u, F, Phi (reading R1 of zeta*)."""
    rng = np.random.default_rng(2)
    for _ in range(30):
        rho = rng.uniform(0.005, 9.0)
        u = rng.uniform(-0.1, 0.1, D)
        F = rng.uniform(-0.05, 0.05, D) * rho
        Phi = rng.uniform(-0.01, 0.01, D) * rho
        fs = O.extended_equilibrium(D, rho, u, F, Phi)
        labs, M = B.matrix(D, u)
        a = M @ fs
        ref = B.appendix_astar(D, rho, F, Phi)
        for k, l in enumerate(labs):
            assert abs(a[k] - ref[l]) <= 1e-14 * max(1.0, rho), (l, a[k], ref[l])


def _random_cell(rng, D, amp):
    rho = rng.uniform(0.01, 9.0)
    u = rng.uniform(-0.1, 0.1, D)
    feq = O.equilibrium(D, rho, u)
    f = feq * (1 + amp * rng.uniform(-1, 1, feq.size))
    c = B.velocities(D).astype(float)
    u_f = (f @ c) / f.sum()
    return f, f.sum(), u_f


@pytest.mark.parametrize("D", [2, 3])
def test_split_matches_explicit_inverse(D):
    """k + s + h = f; each part equals the projection computed with an
    explicit inverse of the Q x Q modified central Hermite matrix (Sec. 2.4)."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        f, rho, u = _random_cell(rng, D, 0.2)
        k, s, h = O.split(D, u, f)
        np.testing.assert_allclose(k + s + h, f, atol=1e-13 * rho)
        np.testing.assert_allclose(s, B.project(D, u, f, "stress"), atol=1e-13 * rho)
        np.testing.assert_allclose(k, B.project(D, u, f, "conserved"), atol=1e-13 * rho)
        np.testing.assert_allclose(h, B.project(D, u, f, "h"), atol=1e-13 * rho)
        # k carries only rho (the central first moments vanish), so k = f^eq
        np.testing.assert_allclose(k, O.equilibrium(D, rho, u), atol=1e-13 * rho)


@pytest.mark.parametrize("D", [2, 3])
def test_split_classes(D):
    """Trace of the second-order moments goes to h, differences and
    off-diagonals to s (reading R6); everything third order and up to h."""
    cls = O.moment_classes(D)
    Q = 3 ** D
    assert (cls == 0).sum() == 1 + D
    assert (cls == 1).sum() == (2 if D == 2 else 5)
    assert (cls == 2).sum() == 1
    assert (cls == 3).sum() == Q - (1 + D) - (cls == 1).sum() - 1


@pytest.mark.parametrize("D", [2, 3])
@pytest.mark.parametrize("collision", [0, 1])
def test_collision_closed_form_and_invariants(D, collision):
    """The LBGK update with the mirror state of Sec. 2.4 equals
    f* + (1-omega) s + (1 - omega gamma/2) h; it conserves mass and adds F to
    the momentum; with gamma = 2 it is BGK: f + omega (f^eq - f) + f* - f^eq."""
    rng = np.random.default_rng(4)
    c = B.velocities(D).astype(float)
    for _ in range(20):
        f, rho, u = _random_cell(rng, D, 0.1)
        F = rng.uniform(-0.03, 0.03, D) * rho
        Phi = rng.uniform(-0.005, 0.005, D) * rho
        omega = rng.uniform(0.5, 1.95)
        fp, gamma, _ = O.collide(D, collision, omega, f, F, Phi)
        feq = O.equilibrium(D, rho, u)
        fs = O.extended_equilibrium(D, rho, u, F, Phi)
        s = B.project(D, u, f, "stress")
        h = f - feq - s
        closed = fs + (1 - omega) * s + (1 - omega * gamma / 2) * h
        np.testing.assert_allclose(fp, closed, atol=2e-14 * rho)
        assert abs(fp.sum() - rho) < 1e-13 * rho
        np.testing.assert_allclose(fp @ c, rho * u + F, atol=1e-13 * rho)
        if collision == 1:
            assert gamma == 2.0
            np.testing.assert_allclose(fp, f + omega * (feq - f) + fs - feq, atol=2e-14 * rho)


@pytest.mark.parametrize("D", [2, 3])
def test_gamma_minimises_entropy_to_first_order(D):
    """Sec. 2.4: gamma comes from dH(f')/dgamma = 0 expanded to first
    non-vanishing order.  For u = F = Phi = 0 the oracle's gamma must approach
    the exact minimiser of H = sum f' ln(f'/w) as the non-equilibrium part
    shrinks (difference O(amplitude))."""
    rng = np.random.default_rng(5)
    w = O.weights(D)
    Q = w.size
    c = B.velocities(D).astype(float)
    # a fixed non-equilibrium direction with zero mass and momentum
    base = rng.normal(size=Q) * w
    A = np.vstack([np.ones(Q), c.T])
    base -= A.T @ np.linalg.solve(A @ A.T, A @ base)
    omega = 1.6
    errs = []
    for amp in (1e-2, 1e-3):
        rho = 1.0
        f = rho * w + amp * rho * base
        u = (f @ c) / f.sum()
        assert np.abs(u).max() < 1e-14
        fp_g, gamma, _ = O.collide(D, 0, omega, f, np.zeros(D), np.zeros(D))
        feq = O.equilibrium(D, f.sum(), u)
        s = B.project(D, u, f, "stress")
        h = f - feq - s

        def H(g):
            fp = feq + (1 - omega) * s + (1 - omega * g / 2) * h
            return np.sum(fp * np.log(fp / w))

        res = minimize_scalar(H, bracket=(gamma - 0.5, gamma + 0.5), tol=1e-14)
        errs.append(abs(res.x - gamma))
    assert errs[1] < 0.2 * errs[0] + 1e-6, errs
    assert errs[1] < 5e-3


@pytest.mark.parametrize("D", [2, 3])
def test_gamma_fallback_at_equilibrium(D):
    """At exact equilibrium <dh|dh> = 0 and gamma falls back to 2/omega
    (reading R10); the post-collision state is f* itself."""
    rho, u = 2.5, np.array([0.03, -0.02, 0.01])[:D]
    feq = O.equilibrium(D, rho, u)
    fp, gamma, fb = O.collide(D, 0, 1.7, feq, np.zeros(D), np.zeros(D))
    assert fb and abs(gamma - 2 / 1.7) < 1e-15
    np.testing.assert_allclose(fp, feq, atol=1e-15 * rho)
