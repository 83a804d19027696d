"""Crown-radius post-processing of drop impacts (Sec. 3.2, 3.3), on
synthetic density fields whose liquid extent is known in closed form."""
import numpy as np
import pytest

from paper_2201_12404_amd import studies as S
from paper_2201_12404_amd import workloads as W


def _field(w, zc, R, sharp=1.0):
    """Film of thickness w.film plus a drop of radius R centred over the axis
    at height zc, with tanh interfaces of width 'sharp'."""
    X = W._coords(w.n)
    D = w.D
    r = np.sqrt(sum((X[a] - w.centre[a]) ** 2 for a in range(D - 1)) + (X[D - 1] - zc) ** 2)
    phi = np.maximum(0.5 * (1 - np.tanh(2 * (X[D - 1] - w.film) / sharp)), 0.5 * (1 - np.tanh(2 * (r - R) / sharp)))
    return w.rho_v + (w.rho_l - w.rho_v) * phi


@pytest.mark.parametrize("D", [2, 3])
@pytest.mark.parametrize("pen", [3.0, 8.0, 15.0])
def test_crown_radius_is_the_chord_of_the_drop(D, pen):
    """A drop that has sunk 'pen' cells below the probe plane: the liquid
    extent there is the chord 2 sqrt(R^2 - (R - pen)^2) of the sphere."""
    R = 20.0
    w = S.impact_we_re(93, 400, R, 0.01, D=D, extent=(6, 3) if D == 2 else (4, 4, 3))
    zp = round(w.film + w.width)
    zc = zp + R - pen
    rho = _field(w, zc, R)
    expect = np.sqrt(R * R - (R - pen) ** 2)
    got = S.crown_radius(rho, w)
    assert abs(got - expect) < 0.35, (got, expect)


def test_crown_radius_before_contact_and_full_row():
    w = S.impact_we_re(93, 400, 20.0, 0.01, extent=(6, 3))
    rho = _field(w, w.centre[-1], w.radius)        # drop still above the probe row
    assert S.crown_radius(rho, w) == 0.0
    rho = np.full(w.N, w.rho_l)                    # liquid across the whole row
    assert S.crown_radius(rho, w) == w.n[0] / 2.0


def test_ray_extent_interpolates_and_finds_the_crown_wall():
    line = np.zeros(40)
    line[10:21] = 1.0
    line[9], line[21] = 0.75, 0.25
    # rightward from 15: cell 20 (1) to 21 (0.25) crosses 0.5 at 20 + 2/3
    assert S._ray_extent(line, 15, 1, 0.5) == pytest.approx(20 + 2 / 3 - 15)
    # leftward: cell 9 (0.75) to 8 (0) crosses at 9 - 1/3
    assert S._ray_extent(line, 15, -1, 0.5) == pytest.approx(15 - (9 - 1 / 3))
    # periodic wrap: the same run rolled across the end of the line
    wrapped = np.roll(line, 25)
    assert S._ray_extent(wrapped, (15 + 25) % 40, 1, 0.5) == pytest.approx(20 + 2 / 3 - 15)
    # vapour on the axis (a crater): the ray skips it to the wall's outer edge
    assert S._ray_extent(line, 4, 1, 0.5) == pytest.approx(20 + 2 / 3 - 4)
    # no liquid within half the line
    assert S._ray_extent(np.zeros(40), 3, 1, 0.5) == 0.0
    assert S._ray_extent(np.ones(40), 3, -1, 0.5) == 20.0


def test_crown_radius_of_a_ring():
    """3-D crown wall: a liquid ring of inner radius 10 and outer radius 14
    around a vapour crater, in the probe plane: radius 14."""
    w = S.impact_we_re(93, 400, 20.0, 0.01, D=3, extent=(4, 4, 3))
    X = W._coords(w.n)
    r = np.sqrt((X[0] - w.centre[0]) ** 2 + (X[1] - w.centre[1]) ** 2)
    ring = 0.5 * (np.tanh(2 * (r - 10)) - np.tanh(2 * (r - 14)))
    rho = w.rho_v + (w.rho_l - w.rho_v) * ring
    assert S.crown_radius(rho, w) == pytest.approx(14.0, abs=0.3)


def test_fit_sqrt_recovers_power_law():
    t = np.linspace(0.02, 1.0, 40)
    n, c = S.fit_sqrt(t, 2.0 * np.sqrt(t))
    assert n == pytest.approx(0.5, abs=1e-12) and c == pytest.approx(2.0, rel=1e-12)
    n, c = S.fit_sqrt(t, 1.3 * t ** 0.7, lo=0.1, hi=0.9)
    assert n == pytest.approx(0.7, abs=1e-12) and c == pytest.approx(1.3, rel=1e-12)
    with pytest.raises(ValueError):
        S.fit_sqrt(t, np.zeros_like(t))


def test_fit_sqrt_offset_recovers_origin_and_flags_other_laws():
    t = np.linspace(0.05, 0.5, 20)
    c, tc, res = S.fit_sqrt_offset(t, 3.0 * np.sqrt(t + 0.12))
    assert c == pytest.approx(3.0, rel=1e-10) and tc == pytest.approx(-0.12, abs=1e-10) and res < 1e-12
    _, _, res = S.fit_sqrt_offset(t, t ** 0.25)    # a different power law leaves a residual
    assert res > 1e-2


def test_impact_we_re_dimensionless_groups():
    sigma, R0 = 0.0123, 50.0
    for D in (2, 3):
        w = S.impact_we_re(238, 4000, R0, sigma, D=D)
        We = 2 * w.rho_l * R0 * w.u_impact ** 2 / sigma
        Re = 2 * w.u_impact * R0 / w.nu_liquid
        assert We == pytest.approx(238, rel=1e-12) and Re == pytest.approx(4000, rel=1e-12)
        assert w.nu_vapour == pytest.approx(15 * w.nu_liquid, rel=1e-12)
        assert w.centre[-1] - w.radius - w.film == pytest.approx(2 * w.width)
    assert S.impact_we_re(93, 100, R0, sigma).n == (1200, 600)
    assert S.impact_we_re(93, 100, R0, sigma, D=3).n == (700, 700, 300)


def test_fixed_kappa_drops_differ_from_the_default_only_in_kappa():
    """The fixed-kappa~ resting drops of the temperature study use the same
    EOS, coexistence densities and geometry as the default ones; only kappa~
    is the one of T/Tc = 0.7 for every T."""
    k07 = W.kappa_w5(0.7)
    for tr in (0.6, 0.65, 0.7, 0.75, 0.8):
        ref = S.drop(tr, 0.03)
        w = S.drop_a(tr, 0.003, 0.03, k07)
        assert w.eos == W.EOS_B
        assert (w.rho_v, w.rho_l) == (ref.rho_v, ref.rho_l)
        assert (w.n, w.radius, w.width, w.centre, w.nu_liquid, w.nu_vapour) == \
            (ref.n, ref.radius, ref.width, ref.centre, ref.nu_liquid, ref.nu_vapour)
        assert w.kappa_tilde == k07
        assert (ref.kappa_tilde == k07) == (tr == 0.7)


def test_paper_3d_impacts_groups_and_box():
    """Sec. 3.3: We 82, 167, 328 over Re 3500..6900 with Re / sqrt(We)
    constant (a fixed drop and fluid), R0 = 80 in a 14 R0 x 14 R0 x 6 R0 box
    (6.0e8 cells) with h / 2R0 = 0.22."""
    wes = [we for we, _ in S.PAPER_3D_IMPACTS]
    res = [re for _, re in S.PAPER_3D_IMPACTS]
    assert wes == [82.0, 167.0, 328.0]
    assert res[-1] == 6900 and 3400 <= res[0] <= 3500
    ratios = [re / np.sqrt(we) for we, re in S.PAPER_3D_IMPACTS]
    assert max(ratios) / min(ratios) < 1.001
    w = S.impact_we_re(82.0, res[0], 80.0, 0.06, D=3, a=5e-4)
    assert w.n == (1120, 1120, 480) and w.N == 602112000
    assert abs(w.film / (2 * w.radius) - 0.22) < 1e-12
    assert abs(S.reynolds(w) - res[0]) < 1e-9 * res[0]


def test_liquid_noise_is_seeded_gaussian_in_the_liquid_only():
    """White noise on the liquid velocity (Sec. 3.3): std noise_liquid * U0
    in the bulk liquid, none in the bulk vapour, the same for the same seed."""
    from dataclasses import replace
    w = S.impact_case(30.0, 0.05, 0.005)
    w = replace(w, noise_liquid=0.05, seed=3)
    rho, u = W.initial_fields(w)
    rho2, u2 = W.initial_fields(w)
    assert np.array_equal(u, u2) and np.array_equal(rho, rho2)
    base_rho, base_u = W.initial_fields(replace(w, noise_liquid=0.0))
    assert np.array_equal(rho, base_rho)
    du = u - base_u
    lam = (rho - w.rho_v) / (w.rho_l - w.rho_v)    # the liquid indicator
    liquid, vapour = lam > 0.999, lam < 1e-9
    assert liquid.sum() > 1000 and vapour.sum() > 1000
    assert np.abs(du[:, vapour]).max() < 1e-8 * w.u_impact
    s = du[:, liquid].std()
    assert abs(s / (0.05 * w.u_impact) - 1) < 0.05
    assert abs(du[:, liquid].mean()) < 0.1 * s
    other = W.initial_fields(replace(w, seed=4))[1]
    assert not np.array_equal(other, u)


def test_tracked_reading_follows_the_crown_wall_past_an_inner_ring():
    """With an inner liquid ring inside the crown wall on the probe plane,
    the first-edge reading gives the ring's outer edge; the tracked reading
    (the edge closest to a given radius) gives the wall's, on every ray."""
    w = S.impact_case(12.0, 0.05, 0.005, D=3, extent=(8, 8, 3))
    nx, ny, nz = w.n
    z = int(round(w.film + w.width))
    X, Y = np.meshgrid(np.arange(nx) - w.centre[0], np.arange(ny) - w.centre[1])
    R = np.hypot(X, Y)
    rho = np.full((nz, ny, nx), w.rho_v)
    rho[z] = np.where(((R >= 8) & (R <= 12)) | ((R >= 26) & (R <= 30)), w.rho_l, w.rho_v)
    first = S.crown_radius(rho.ravel(), w)
    tracked = S.crown_radius(rho.ravel(), w, near=28.0)
    assert 12.0 <= first <= 13.5
    assert 30.0 <= tracked <= 31.5
    assert S.crown_radius(rho.ravel(), w, near=1.0) == first
    assert S._ray_edges(rho[z][int(round(w.centre[1]))], int(round(w.centre[0])), 1, 0.5 * (w.rho_l + w.rho_v))[:2] \
        == pytest.approx([first, tracked], abs=1.5)
