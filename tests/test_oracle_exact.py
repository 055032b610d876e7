"""Exact pins of the oracle's absorber path, background, p-p radius rule and
linear absorption average.

Each test builds a case whose answer the paper's definitions fix in closed
form, and computes that answer here with numpy (`tests/bruteforce.py`), not
with the oracle's code:

* a gap-free lattice (32^3 cell-centred elements in the unit cube, buckets of
  8 = 2x2x2 blocks) is a uniform medium whose buckets tile space, so the cell
  chords on any ray beyond the p-p radius add up to the ray length there and
  every transmission average equals kappa rho (Sections 2.5.1, 2.6);
* with theta = 0 every cell opens, so every source outside the p-p sphere is
  a point source at its own position (Section 2.5.2);
* the p-p columns (Section 2.4) are summed here element by element.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2310_15235_amd import scenes
from tests import bruteforce as bf

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _lattice(kappa=(4.0, 1.0), nside=2, theta=0.0, **kw):
    return scenes.lattice_scene(per_side=32, rho=1.0, kappa=kappa, nside=nside, theta=theta,
                                thick_corr=False, **kw)


def _bucket_centre(pos):
    """Centre of the 2x2x2 block (bucket) holding each lattice element."""
    return (np.floor(pos * 16.0) + 0.5) / 16.0


def _h(sc):
    return np.cbrt(sc.m.astype(np.float64) / sc.rho.astype(np.float64))


def _rpp_of(sc, act):
    """p-p radius per active element, from the oracle's bucket report."""
    T = oracle.OracleTree(sc)
    _, _, info = T.compute_J(act, bucket_info=True)
    nd = T.nodes(with_alpha=False)
    perm, _ = T.perm()
    r = np.full(sc.n, np.nan)
    for row in info:
        leaf = int(row[0])
        slots = perm[nd["first"][leaf]:nd["first"][leaf] + nd["count"][leaf]]
        r[slots] = row[1]
    return r


# ------------------------------------------------------------ background
def test_background_transparent_is_4pi_intensity():
    """No absorption and no sources: every ray carries 4 pi / N_ray of the
    isotropic background unattenuated, so J = 4 pi I_bg exactly (abstract,
    Section 4)."""
    sc = scenes.lognormal_scene(n=3000, seed=81, grid=16, bands=(0.0, 0.0), nside=2,
                                thick_corr=False)
    sc.lum[:] = 0.0
    sc = sc.with_(background=True, bg=np.array([0.7, 2.5], np.float32))
    J, c = oracle.compute_J(sc)
    ref = 4.0 * np.pi * sc.bg.astype(np.float64)[:, None]
    assert np.max(np.abs(J - ref) / ref) < 1e-13
    assert c["source_entries"] == 0 and c["absorber_entries"] == 0


@pytest.mark.parametrize("near", [False, True])
def test_background_lattice_exit_depth(near):
    """A uniform gap-free medium: each ray is attenuated by kappa rho times
    its length from the p-p radius to the root-cube exit, plus (near field
    on) the p-p columns ahead of the receiver on that ray."""
    sc = _lattice(theta=0.75, near_field=near)
    sc.lum[:] = 0.0
    sc = sc.with_(background=True, bg=np.array([1.0, 3.0], np.float32))
    pos = sc.positions().astype(np.float64)
    rng = np.random.default_rng(5)
    act = np.zeros(sc.n, np.uint8)
    act[rng.choice(sc.n, 40, replace=False)] = 1
    J, _ = oracle.OracleTree(sc).compute_J(act)
    r = _rpp_of(sc, act) if near else np.zeros(sc.n)
    h = _h(sc)
    kap = sc.kappa.astype(np.float64)
    m = sc.m.astype(np.float64)
    ar = kap[:, 0] * 1.0                          # kappa rho per band
    nv = oracle.healpix_centres(sc.nside)
    K = nv.shape[0]
    bg = sc.bg.astype(np.float64)
    cen = _bucket_centre(pos)
    for i in np.flatnonzero(act):
        c = cen[i]
        near_set = np.flatnonzero(np.linalg.norm(pos - c, axis=1) < r[i]) if near else []
        ref = np.zeros(2)
        for k in range(K):
            s_exit = bf.box_exit(c, nv[k], (0.0, 0.0, 0.0), 1.0)
            tpp = bf.ray_depth(pos, m, h, kap, i, nv[k], near_set)
            ref += (4 * np.pi / K) * bg * np.exp(-tpp - ar * max(0.0, s_exit - r[i]))
        assert np.max(np.abs(J[:, i] - ref) / ref) < 1e-12, (i, J[:, i], ref)


# ------------------------------------------------------- absorber path
@pytest.mark.parametrize("nside,near", [(1, False), (2, False), (2, True), (4, True)])
def test_lattice_absorber_path_closed_form(nside, near):
    """Sources and receivers near the middle of a gap-free lattice, theta = 0.
    Every far source j sits on the ray k whose pixel holds its direction from
    the bucket centre c, at projected distance s; the cell chords on that ray
    from the p-p radius r to s add up to s - r, so its optical depth is
    kappa rho (s - r), scaled by the true over the projected distance
    (Section 2.5.1), plus the receiver's p-p column on ray k; near sources
    (inside r) see the p-p column of the segment (Section 2.4).  This fixes
    the slab test, the clip at r, the sum of chords, the r/s projection and
    the per-beam p-p column together:

      J_i = sum_far L_j K(r_ij, h_i) exp(-tpp_i(k_j) - kappa rho (s_j - r) r_ij / s_j)
          + sum_near L_j K(r_ij, h_i) exp(-tpp(i -> j)).
    """
    sc = _lattice(nside=nside, near_field=near)
    pos = sc.positions().astype(np.float64)
    rc = np.linalg.norm(pos - 0.5, axis=1)
    rng = np.random.default_rng(10 + nside)
    src = rng.choice(np.flatnonzero(rc < 0.1), 24, replace=False)
    sc.lum[:, src] = np.array([1.0, 2.0])[:, None] * rng.uniform(0.5, 2.0, src.size)[None, :]
    act = (rc < 0.1).astype(np.uint8)
    J, c = oracle.OracleTree(sc).compute_J(act)
    assert c["absorber_entries"] > 0 and c["source_entries"] > 0
    if near:
        assert c["near_pairs"] > 0
    r = _rpp_of(sc, act) if near else np.zeros(sc.n)
    h = _h(sc)
    kap = sc.kappa.astype(np.float64)
    m = sc.m.astype(np.float64)
    lum = sc.lum.astype(np.float64)
    ar = kap[:, 0]
    nv = oracle.healpix_centres(nside)
    cen = _bucket_centre(pos)
    checked = 0
    for i in np.flatnonzero(act):
        cb = cen[i]
        # every ray from cb to a source stays inside the lattice (so the
        # chords tile it): |cb - middle| + |x_j - cb| < 1/2
        assert np.all(np.linalg.norm(cb - 0.5) + np.linalg.norm(pos[src] - cb, axis=1) < 0.5)
        dist_c = np.linalg.norm(pos - cb, axis=1)
        near_set = np.flatnonzero(dist_c < r[i])
        ref = np.zeros(2)
        for j in src:
            rij = np.linalg.norm(pos[j] - pos[i])
            Kv = bf.kernel(rij, h[i])
            if dist_c[j] < r[i]:
                tau = bf.segment_depth(pos, m, h, kap, i, j, near_set)
            else:
                v = pos[j] - cb
                k = int(oracle.healpix_pixel(nside, v)[0])
                s = float(v @ nv[k])
                tpp = bf.ray_depth(pos, m, h, kap, i, nv[k], near_set)
                tcell = ar * (s - r[i]) * rij / s if s > r[i] else 0.0
                tau = tpp + tcell
            ref += lum[:, j] * Kv * np.exp(-tau)
        assert np.max(np.abs(J[:, i] - ref) / ref) < 1e-12, (i, J[:, i], ref)
        checked += 1
    assert checked > 100


# ------------------------------------------------------------ p-p radius
def _beam_w(nray):
    return 2.0 * np.tan(np.arccos(1.0 - 2.0 / nray))


@pytest.mark.parametrize("nside,rpp_min", [(2, 0.0), (4, 0.0), (4, 0.03)])
def test_rpp_is_first_fixed_point_of_the_beam_rule(nside, rpp_min):
    """Section 2.4: the p-p sphere about the bucket centre reaches past every
    bucket member by its size h, and grows until no element inside it is
    wider than the beam at that distance.  Checked per bucket from the
    oracle's report: (1) r >= max(rpp_min, |x_i - c| + h_i) over members;
    (2) every element inside has h_j <= w r; (3) r is that start value or the
    h_j / w of an element inside, and no smaller candidate (the start value
    or any h_j / w in between) already satisfies (2)."""
    sc = scenes.lognormal_scene(n=2 ** 13, seed=83, grid=16, bands=(1.0,), nside=nside,
                                rpp_min=rpp_min)
    T = oracle.OracleTree(sc)
    _, _, info = T.compute_J(scenes.active_subset(sc, 0.05, 2), bucket_info=True)
    nd = T.nodes(with_alpha=False)
    perm, _ = T.perm()
    pos = sc.positions().astype(np.float64)
    h = _h(sc)
    w = _beam_w(12 * nside * nside)
    grew = 0
    rng = np.random.default_rng(1)
    for row in info[rng.permutation(len(info))[:300]]:
        leaf, r = int(row[0]), float(row[1])
        c = 0.5 * (nd["lo"][leaf] + nd["hi"][leaf])
        mem = perm[nd["first"][leaf]:nd["first"][leaf] + nd["count"][leaf]]
        d = np.linalg.norm(pos - c, axis=1)
        r0 = max(rpp_min, float(np.max(d[mem] + h[mem])))
        assert r >= r0 * (1 - 1e-15)
        inside = d < r
        assert np.all(h[inside] <= w * r * (1 + 1e-12))
        assert int(row[2]) == int(inside.sum())
        if abs(r - r0) > 1e-14 * r0:
            grew += 1
            assert np.min(np.abs(h[inside] / w - r)) < 1e-14 * r
        # largest h among the elements closer than rc, for any rc
        order = np.argsort(d)
        ds, hmax = d[order], np.maximum.accumulate(h[order])
        cand = np.concatenate([[r0], h[inside] / w])
        cand = cand[(cand >= r0) & (cand < r * (1 - 1e-12))]
        cnt = np.searchsorted(ds, cand, side="left")        # elements with d < rc
        assert np.all((cnt > 0) & (hmax[np.maximum(cnt - 1, 0)] > w * cand * (1 + 1e-12))), \
            (leaf, r)
    if nside == 4 and rpp_min == 0.0:
        assert grew > 0


def test_beam_half_angle_from_oracle_growth():
    """Section 2.5.2 quotes an average half-angle of 16.5 degrees for 48
    beams.  Where a p-p sphere grew, its radius is h_j / w for the element j
    that set it, so the beam width w and half-angle atan(w/2) can be read off
    the oracle's output (not recomputed from the beam rule)."""
    g = json.load(open(os.path.join(GOLD, "opening_angles.json")))
    sc = scenes.lognormal_scene(n=2 ** 13, seed=84, grid=16, bands=(1.0,), nside=2)
    T = oracle.OracleTree(sc)
    _, _, info = T.compute_J(sc.active, bucket_info=True)
    nd = T.nodes(with_alpha=False)
    perm, _ = T.perm()
    pos = sc.positions().astype(np.float64)
    h = _h(sc)
    ws = []
    for row in info:
        leaf, r = int(row[0]), float(row[1])
        c = 0.5 * (nd["lo"][leaf] + nd["hi"][leaf])
        mem = perm[nd["first"][leaf]:nd["first"][leaf] + nd["count"][leaf]]
        d = np.linalg.norm(pos - c, axis=1)
        r0 = float(np.max(d[mem] + h[mem]))
        if r > r0 * (1 + 1e-12):
            inside = d < r
            ws.append(float(np.max(h[inside])) / r)
    assert len(ws) > 5
    ws = np.array(ws)
    assert np.ptp(ws) < 1e-12 * ws.max()
    half = np.degrees(np.arctan(ws[0] / 2))
    assert half == pytest.approx(g["beam48_half_angle_deg"], abs=0.15)


# --------------------------------------------------- absorption average
def _half_filled_lattice(avg):
    """Two uniform halves along x (x < 1/2 with alpha = 10, the other
    transparent): the root's two children are the figure's two cells."""
    sc = scenes.lattice_scene(per_side=16, rho=1.0, kappa=(10.0,), nside=2,
                              absorption_avg=avg)
    sc.kappa[0, sc.x >= 0.5] = 0.0
    return sc


def test_absorption_average_table_rows():
    """Section 2.6 figure table, absorption-average rows: the linear average of
    alpha = 10 and 0 is 5 in every direction; tau along the chord through the
    centre of the pair is 5 across (thinnest) and 5 sqrt(5) = 11.2 along the
    diagonal of the 2:1 pair (thickest)."""
    g = json.load(open(os.path.join(GOLD, "two_cell_table.json")))
    rows = {(r["method"], r["direction"]): r for r in g["rows"]}
    T = oracle.OracleTree(_half_filled_lattice(True))
    al = T.nodes()["alpha"][0]                      # root [dir][band]
    assert np.allclose(al, rows[("absorption", "A")]["alpha"], rtol=1e-14, atol=0)
    # tau = alpha d on the two-cell figure geometry (2 x 1 cells)
    _, geo_v = oracle.combine([2.0, 1.0, 1.0], 0, [0.0, 1.0, 0.0], 10.0, 0.0, return_geom=True)
    dg = np.array([2.0, 1.0, 0.0]) / np.sqrt(5.0)
    _, geo_d = oracle.combine([2.0, 1.0, 1.0], 0, dg, 10.0, 0.0, return_geom=True)
    assert al[0, 0] * geo_v[2] == pytest.approx(rows[("absorption", "thinnest_vertical")]["tau"],
                                                abs=0.05)
    assert al[0, 0] * geo_d[2] == pytest.approx(rows[("absorption", "thickest_diagonal")]["tau"],
                                                abs=0.05)


def test_absorption_average_vacuum_halving_and_first_order_limit():
    """Linear averaging weighs by volume: a cell whose particles fill one
    octant of its owned box has 1/8 of their absorption (empty space is
    vacuum), and for a weakly absorbing medium the transmission average
    agrees with it to first order in tau (Section 2.6)."""
    sc = scenes.lattice_scene(per_side=16, rho=1.0, kappa=(2.0,), nside=2, absorption_avg=True)
    keep = (sc.x < 0.5) & (sc.y < 0.5) & (sc.z < 0.5)
    sub = sc.with_(x=sc.x[keep], y=sc.y[keep], z=sc.z[keep], m=sc.m[keep], rho=sc.rho[keep],
                   kappa=sc.kappa[:, keep], lum=sc.lum[:, keep], active=sc.active[keep])
    al = oracle.OracleTree(sub).nodes()["alpha"][0]
    assert np.allclose(al, 2.0 / 8.0, rtol=1e-14, atol=0)
    # weak, non-uniform medium: the two averages agree to first order
    wk = scenes.lognormal_scene(n=4000, seed=85, grid=16, bands=(1e-4,), nside=2)
    a_lin = oracle.OracleTree(wk.with_(absorption_avg=True)).nodes()["alpha"]
    a_tr = oracle.OracleTree(wk).nodes()["alpha"]
    big = a_lin > 0
    assert np.max(np.abs(a_tr[big] - a_lin[big]) / a_lin[big]) < 1e-2
    # and the transmission average never exceeds the linear one (Jensen's
    # inequality; -ln(T)/d at T = 1 - 1e-5 carries ~1e-11 relative rounding)
    assert np.all(a_tr <= a_lin * (1 + 1e-9))


# ------------------------------------------------------- directed rays
@pytest.mark.parametrize("nside", [1, 2])
def test_directed_ray_lattice_closed_form(nside):
    """Directed rays (Sections 3.4.1, 4) on the gap-free lattice with one
    source p: the ray that carries p is aimed at it, so p sits on the ray at
    s = |p - c| and the chords from r to s add up to s - r along the aimed
    direction u; the p-p column of that ray is taken along u:
      J_i = L K(r_i, h_i) exp(-tpp_i(u) - kappa rho (|p - c| - r) r_i / |p - c|)."""
    sc = _lattice(nside=nside, near_field=True)
    pos = sc.positions().astype(np.float64)
    rc = np.linalg.norm(pos - 0.5, axis=1)
    j = int(np.flatnonzero(rc < 0.05)[0])
    sc.lum[:, j] = [1.0, 2.0]
    sc = sc.with_(directed=tuple(float(v) for v in pos[j]))
    act = ((rc < 0.12) & (rc > 0.06)).astype(np.uint8)
    J, c = oracle.OracleTree(sc).compute_J(act)
    r = _rpp_of(sc, act)
    h = _h(sc)
    kap = sc.kappa.astype(np.float64)
    m = sc.m.astype(np.float64)
    cen = _bucket_centre(pos)
    checked = 0
    for i in np.flatnonzero(act):
        cb = cen[i]
        v = pos[j] - cb
        d = np.sqrt(v @ v)
        if d < r[i]:
            continue                      # a near source: p-p path, pinned above
        u = v / d
        near_set = np.flatnonzero(np.linalg.norm(pos - cb, axis=1) < r[i])
        rij = np.linalg.norm(pos[j] - pos[i])
        tau = bf.ray_depth(pos, m, h, kap, i, u, near_set) + kap[:, 0] * (d - r[i]) * rij / d
        ref = sc.lum[:, j].astype(np.float64) * bf.kernel(rij, h[i]) * np.exp(-tau)
        assert np.max(np.abs(J[:, i] - ref) / ref) < 1e-12, (i, J[:, i], ref)
        checked += 1
    assert checked > 100


# ------------------------------------------------- complex source model
def _exit(lo, hi, p, n):
    t = np.inf
    for a in range(3):
        if n[a] > 0:
            t = min(t, (hi[a] - p[a]) / n[a])
        elif n[a] < 0:
            t = min(t, (lo[a] - p[a]) / n[a])
    return max(t, 0.0)


@pytest.mark.parametrize("nside", [1, 2])
def test_complex_source_single_source_uniform_medium(nside):
    """Section 2.7 with one source in a uniform gap-free medium: every cell
    holding the source has its luminosity centre at the source, the child
    rays are extended (never clipped) through a cell of the same absorption,
    so the stored optical depth of the source's own ray in direction k is
    kappa rho times the distance from the source to the cell's edge along
    n_k; buckets store their absorption in every direction."""
    sc = _lattice(kappa=(4.0, 1.0), nside=nside, theta=0.75, complex_source=True)
    j = (17 * 32 + 9) * 32 + 21
    sc.lum[:, j] = [1.0, 3.0]
    T = oracle.OracleTree(sc)
    nd = T.nodes(with_alpha=False)
    cd, ca, ap = T.complex_tables()
    hp = oracle.healpix_centres(nside)
    pos = sc.positions().astype(np.float64)
    perm, _ = T.perm()
    slot = int(np.flatnonzero(perm == j)[0])
    lum_nodes = np.flatnonzero((nd["first"] <= slot) & (slot < nd["first"] + nd["count"]))
    assert len(lum_nodes) > 5
    for n_ in lum_nodes:
        for k in range(hp.shape[0]):
            d = _exit(nd["lo"][n_], nd["hi"][n_], pos[j], hp[k])
            assert cd[n_, k] == pytest.approx(d, rel=1e-12, abs=1e-15)
            np.testing.assert_allclose(ca[n_, k] * cd[n_, k], np.array([4.0, 1.0]) * d,
                                       rtol=1e-12, atol=1e-15)
    leaves = np.flatnonzero(nd["split"] < 0)
    assert np.allclose(ca[leaves], np.array([4.0, 1.0])[None, None, :], rtol=1e-14)
    # antipodes: opposite directions
    np.testing.assert_allclose(hp[ap], -hp, atol=1e-12)


def test_complex_source_transparent_equals_standard():
    """Without absorption the complex source model changes nothing: the
    sources' own rays and the shortened cell trace carry no optical depth."""
    sc = scenes.lognormal_scene(n=3000, seed=86, grid=16, bands=(0.0, 0.0), nside=2)
    J0, c0 = oracle.compute_J(sc)
    J1, c1 = oracle.compute_J(sc.with_(complex_source=True))
    assert c0 == c1
    assert np.max(np.abs(J1 - J0) / J0) < 1e-13
