"""Pins of the oracle's elementary pieces against what the paper and the
mathematics fix independently (quadratures, limits, Monte Carlo, the paper's
printed values)."""
import json
import os

import numpy as np
import pytest
from scipy import integrate

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")
R = np.sqrt(3.0 / (4.0 * np.pi))


# ----------------------------------------------------------------- K(r, h)
def sphere_average_quadrature(r, a):
    """Volume average over a ball of radius a of 1/(4 pi d^2), d the distance
    to a point source at distance r from the centre.  Integrates over shells
    about the source: the fraction of each shell inside the ball times
    4 pi d^2 / (4 pi d^2)."""
    def frac(d):
        if d == 0:
            return 1.0 if r < a else 0.0
        c0 = (d * d + r * r - a * a) / (2 * d * r) if r > 0 else (-1.0 if d < a else 1.0)
        return min(1.0, max(0.0, (1.0 - c0) / 2.0))
    pts = [abs(r - a), r + a] if r > 0 else [a]
    val, _ = integrate.quad(frac, 0.0, r + a, points=pts, limit=400, epsabs=1e-14, epsrel=1e-12)
    return val / (4.0 / 3.0 * np.pi * a ** 3)


@pytest.mark.parametrize("x", [0.0, 0.05, 0.3, 0.8, 0.999, 1.0, 1.001, 1.7, 3.0, 9.99, 10.0, 40.0])
def test_kernel_is_sphere_average(x):
    """Section 2.2: eq. intint is the volume average over a sphere of radius
    (3/4pi)^(1/2) h of the intensity of a point source at distance r."""
    h = 0.37
    r = x * R * h
    ref = sphere_average_quadrature(r, R * h)
    assert oracle.kernel_K(r, h) == pytest.approx(ref, rel=1e-9)


def test_kernel_limits():
    h = 2.0
    # peak 1/h^2 at zero separation (Section 2.2)
    assert oracle.kernel_K(0.0, h) == pytest.approx(1.0 / h ** 2, rel=1e-15)
    # inverse-square law far away
    for r in (50.0, 500.0, 5e4):
        assert oracle.kernel_K(r, h) * 4 * np.pi * r * r == pytest.approx(1.0, rel=2.0 * (R * h / r) ** 2)
    # close to inverse square by r ~ 2h (within a few percent)
    assert oracle.kernel_K(2 * h, h) * 4 * np.pi * (2 * h) ** 2 == pytest.approx(1.0, rel=0.05)
    # monotone decreasing and continuous across the branch points x = 1, 10
    xs = np.concatenate([np.linspace(0, 20, 4001), [1 - 1e-12, 1 + 1e-12, 10 - 1e-12, 10 + 1e-12]])
    xs.sort()
    ks = np.array([oracle.kernel_K(x * R * h, h) for x in xs])
    assert np.all(np.diff(ks) <= 1e-15)
    for x0 in (1.0, 10.0):
        a = oracle.kernel_K((x0 - 1e-9) * R * h, h)
        b = oracle.kernel_K((x0 + 1e-9) * R * h, h)
        assert a == pytest.approx(b, rel=1e-7)


# ----------------------------------------------------------------- C(tau)
@pytest.mark.parametrize("tau", [1e-12, 1e-6, 0.01, 0.5, 1.0, 7.0, 50.0, 1e4])
def test_thick_correction_is_element_average(tau):
    """Section 2.1, eq. taucorr: the mean of e^{-tau'} over the element depth."""
    ref, _ = integrate.quad(lambda t: np.exp(-t), 0.0, tau, epsabs=0, epsrel=1e-13)
    assert oracle.thick_C(tau) == pytest.approx(ref / tau, rel=1e-11)


def test_thick_correction_limits():
    assert oracle.thick_C(0.0) == 1.0
    t = 1e-3
    assert oracle.thick_C(t) == pytest.approx(1 - t / 2 + t * t / 6 - t ** 3 / 24, rel=1e-12)
    assert oracle.thick_C(1e5) * 1e5 == pytest.approx(1.0, rel=1e-12)           # 1/tau limit


# -------------------------------------------------------------- Sigma(b)
def test_column_profile_normalisation():
    """Section 2.4: the column falls linearly with b/h and its area integral
    over b < h is the particle mass."""
    m, h = 0.3, 0.7
    tot, _ = integrate.quad(lambda b: oracle.column_sigma(b, m, h) * 2 * np.pi * b, 0, h)
    assert tot == pytest.approx(m, rel=1e-12)
    assert oracle.column_sigma(h, m, h) == 0.0
    assert oracle.column_sigma(2 * h, m, h) == 0.0
    a = oracle.column_sigma(0.2 * h, m, h)
    b = oracle.column_sigma(0.6 * h, m, h)
    assert a / b == pytest.approx(0.8 / 0.4, rel=1e-14)


# ---------------------------------------------------------------- HEALPix
@pytest.mark.parametrize("nside", [1, 2, 4, 8])
def test_healpix_centres_and_membership(nside):
    v = oracle.healpix_centres(nside)
    npix = 12 * nside * nside
    assert v.shape == (npix, 3)
    assert np.allclose((v * v).sum(1), 1.0, atol=1e-14)
    assert np.array_equal(oracle.healpix_pixel(nside, v), np.arange(npix))
    # rings: 4N-1 distinct z values, symmetric about the equator
    z = np.unique(np.round(v[:, 2], 12))
    assert len(z) == 4 * nside - 1
    assert np.allclose(np.sort(z), -np.sort(z)[::-1])
    # antipodes: a fixed-point-free involution
    anti = oracle.healpix_pixel(nside, -v)
    assert np.array_equal(anti[anti], np.arange(npix))
    assert np.all(anti != np.arange(npix))


@pytest.mark.parametrize("nside", [1, 2, 4])
def test_healpix_equal_area(nside):
    """Gorski et al. 2005: equal-area pixels; Monte Carlo directions land in
    each pixel with probability 1/N_pix."""
    rng = np.random.default_rng(nside)
    n = 600000
    d = rng.normal(size=(n, 3))
    pix = oracle.healpix_pixel(nside, d)
    npix = 12 * nside * nside
    cnt = np.bincount(pix, minlength=npix)
    exp = n / npix
    assert np.all(np.abs(cnt - exp) < 5.5 * np.sqrt(exp))


@pytest.mark.parametrize("nside", [1, 2, 4])
def test_healpix_pixel_is_compact_region(nside):
    """A direction lies in a pixel whose centre is within the largest
    centre-to-vertex angle (a pixel is a compact region around its centre)."""
    rng = np.random.default_rng(7)
    v = oracle.healpix_centres(nside)
    d = rng.normal(size=(20000, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    pix = oracle.healpix_pixel(nside, d)
    ang = np.degrees(np.arccos(np.clip((d * v[pix]).sum(1), -1, 1)))
    # nearest-centre angle is a lower bound; the assigned centre is close
    near = np.degrees(np.arccos(np.clip((d @ v.T).max(1), -1, 1)))
    assert np.all(ang >= near - 1e-9)
    assert ang.max() < 2.0 * np.degrees(np.sqrt(4 * np.pi / (12 * nside * nside)))
    assert (np.abs(ang - near) < 1e-9).mean() > 0.8


# ------------------------------------------------------------- combining
def _two_cell(phi_deg, a1=10.0, a2=0.0):
    ph = np.radians(phi_deg)
    n = [np.cos(ph), np.sin(ph), 0.0]
    a, g = oracle.combine([2.0, 1.0, 1.0], 0, n, a1, a2, return_geom=True)
    return a, g


def test_two_cell_table_exact_rows():
    """Section 2.6 table: the thinnest (rays along the joining face) and
    thickest (rays through both cells) rows of transmission averaging."""
    rows = {(r["method"], r["direction"]): r for r in
            json.load(open(os.path.join(GOLD, "two_cell_table.json")))["rows"]}
    a, g = _two_cell(90.0)
    r = rows[("transmission", "thinnest_vertical")]
    assert a == pytest.approx(r["alpha"], abs=5e-4)
    assert a * g[2] == pytest.approx(r["tau"], abs=5e-4)
    assert np.exp(-a * g[2]) == pytest.approx(r["T"], abs=5e-5)
    a, g = _two_cell(0.0)
    r = rows[("transmission", "thickest_horizontal")]
    assert a == pytest.approx(r["alpha"], rel=1e-12)
    assert a * g[2] == pytest.approx(r["tau"], rel=1e-12)
    assert np.exp(-a * g[2]) == pytest.approx(r["T"], rel=0.02)
    # absorption average of the same pair is the volume mean 5, tau = 5 d
    ra = rows[("absorption", "thinnest_vertical")]
    assert 5.0 * g[2] / 2.0 == pytest.approx(ra["tau"], rel=1e-12)


@pytest.mark.parametrize("key", ["A", "B"])
def test_two_cell_table_directions_loose(key):
    """Rows A and B give no direction; find the in-plane angle that
    reproduces the printed transmission and check the printed alpha and tau
    (and the absorption-average tau at the same angle) loosely."""
    from scipy.optimize import brentq
    rows = {(r["method"], r["direction"]): r for r in
            json.load(open(os.path.join(GOLD, "two_cell_table.json")))["rows"]}
    rt, ra = rows[("transmission", key)], rows[("absorption", key)]
    def f(p):
        a, g = _two_cell(p)
        return np.exp(-a * g[2]) - rt["T"]
    grid = np.linspace(0.5, 89.5, 400)
    vals = np.array([f(p) for p in grid])
    k = np.nonzero(np.sign(vals[:-1]) != np.sign(vals[1:]))[0]
    assert len(k) >= 1
    phi = brentq(f, grid[k[0]], grid[k[0] + 1])
    a, g = _two_cell(phi)
    assert a == pytest.approx(rt["alpha"], abs=0.06)
    assert a * g[2] == pytest.approx(rt["tau"], abs=0.01)
    assert 5.0 * g[2] == pytest.approx(ra["tau"], rel=0.03)


def test_half_blocked_node_transmits_half():
    """Section 2.6: a node half blocked by opaque material (tau = 1000) should
    pass half the light, tau_eff = ln 2, where linear averaging gives 500."""
    a, g = oracle.combine([2.0, 1.0, 1.0], 0, [0.0, 1.0, 0.0], 1000.0, 0.0, return_geom=True)
    assert a * g[2] == pytest.approx(np.log(2.0), rel=1e-12)


def test_combine_identities():
    rng = np.random.default_rng(3)
    for _ in range(200):
        sides = np.array([1.0, 1.0, 1.0]) * np.array([rng.choice([0.5, 1.0]), 1, 1])
        ax = int(rng.integers(3))
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        a1, a2 = rng.exponential(3.0, size=2)
        c = oracle.combine(sides, ax, n, a1, a2)
        # symmetric in the children and under n -> -n (Section 2.6: N_ray/2 stored)
        assert c == pytest.approx(oracle.combine(sides, ax, n, a2, a1), rel=1e-13)
        assert c == pytest.approx(oracle.combine(sides, ax, -n, a1, a2), rel=1e-13)
        # uniform children keep their alpha; result bounded by the children
        assert oracle.combine(sides, ax, n, a1, a1) == pytest.approx(a1, rel=1e-12)
        assert min(a1, a2) * (1 - 1e-12) <= c <= max(a1, a2) * (1 + 1e-12)
        assert c <= 0.5 * (a1 + a2) * (1 + 1e-12)   # never above the linear average
        # first order: the volume-weighted linear average (Section 2.6)
        e1, e2 = 1e-7 * a1, 1e-7 * a2
        assert oracle.combine(sides, ax, n, e1, e2) == pytest.approx(0.5 * (e1 + e2), rel=1e-6)


@pytest.mark.parametrize("seed", range(6))
def test_combine_geometry_monte_carlo(seed):
    """V12/V is the fraction of the box whose points lie on a line along n
    that crosses the joining face inside the box; d is the chord through the
    box centre.  Both checked by sampling."""
    rng = np.random.default_rng(100 + seed)
    sides = np.array([1.0, 1.0, 1.0])
    if seed % 3:
        sides[rng.integers(3)] = 0.5
    ax = int(np.argmax(sides)) if seed % 2 else int(rng.integers(3))
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    _, g = oracle.combine(sides, ax, n, 1.0, 2.0, return_geom=True)
    p = rng.random((400000, 3)) * sides
    t = (0.5 * sides[ax] - p[:, ax]) / n[ax]
    q = p + t[:, None] * n
    inside = np.all((q >= 0) & (q <= sides), axis=1)
    assert inside.mean() == pytest.approx(g[1], abs=4e-3)
    assert 2 * g[0] + g[1] == pytest.approx(1.0, abs=1e-12)
    # chord through the centre by stepping
    c = 0.5 * sides
    tmax = np.min(np.where(np.abs(n) > 0, (0.5 * sides) / np.maximum(np.abs(n), 1e-300), np.inf))
    assert g[2] == pytest.approx(2 * tmax, rel=1e-12)


# --------------------------------------------------------------- opening
def test_opening_angle_threshold():
    """Section 2.5.2: at theta = 0.75 a cube with a centred source is accepted
    once its face-on half-angle drops to 16.8 deg (23 deg across the
    diagonal)."""
    g = json.load(open(os.path.join(GOLD, "opening_angles.json")))
    lo, hi, cen = np.zeros(3), np.ones(3), np.full(3, 0.5)
    dcrit = np.sqrt(0.75) / g["theta"]           # B = half diagonal
    # bucket on the x axis, face-on
    for d, expect in ((dcrit * (1 - 1e-9), True), (dcrit * (1 + 1e-9), False)):
        c = np.array([1.0 + d, 0.5, 0.5])
        assert oracle.open_cell(lo, hi, cen, c, 0.0, g["theta"]) is expect
    half_face = np.degrees(np.arctan(0.5 / (dcrit + 0.5)))
    half_diag = np.degrees(np.arctan(np.sqrt(0.5) / (dcrit + 0.5)))
    assert half_face == pytest.approx(g["half_angle_face_deg"], abs=0.05)
    assert half_diag == pytest.approx(g["half_angle_diag_deg"], abs=0.2)
    # a cell always opens itself; and it opens when reaching into the p-p sphere
    assert oracle.open_cell(lo, hi, cen, cen, 0.0, 100.0)
    assert oracle.open_cell(lo, hi, cen, np.array([3.0, 0.5, 0.5]), 2.5, 100.0)
    assert not oracle.open_cell(lo, hi, cen, np.array([3.0, 0.5, 0.5]), 1.5, 100.0)
