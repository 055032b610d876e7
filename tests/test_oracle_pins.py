"""Scene-level pins of the oracle: exact reductions to brute force, closed
forms, invariances and the cost law (Sections 2.2-2.6, 3.1)."""
import numpy as np
import pytest

import oracle
from paper_2310_15235_amd import scenes
from tests import bruteforce as bf


def _h(sc):
    return np.cbrt(sc.m.astype(np.float64) / sc.rho.astype(np.float64))


def _pos(sc):
    return sc.positions().astype(np.float64)


def _rel(a, b, floor=1e-300):
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), floor))


# -------------------------------------------------------------------- tree
@pytest.mark.parametrize("maker", [
    lambda: scenes.uniform_scene(n=3000, seed=4, n_src=40, nside=2),
    lambda: scenes.lognormal_scene(n=6000, seed=5, grid=16, nside=1),
    lambda: scenes.uniform_scene(n=500, seed=6, n_src=5, nside=1, leaf_size=12, box=None),
])
def test_tree_invariants(maker):
    """Section 2.3: binary tree of cubes or 2:1 boxes split half-way along the
    longest axis; buckets of at most leaf_size particles (unless their keys
    coincide); children tile their parent's split box."""
    sc = maker()
    T = oracle.OracleTree(sc)
    nd = T.nodes(with_alpha=False)
    nn = T.num_nodes
    assert nn <= 2 * sc.n - 1
    first, count, lown, split = nd["first"], nd["count"], nd["lown"], nd["split"]
    c0, c1, nxt = nd["child0"], nd["child1"], nd["next"]
    assert count[0] == sc.n and first[0] == 0 and lown[0] == 0 and nxt[0] == nn
    leaf = split < 0
    assert np.all(count[leaf] <= sc.leaf_size)
    perm, keys = T.perm()
    assert np.array_equal(np.sort(perm), np.arange(sc.n))
    assert np.all(np.diff(keys.astype(np.float64)) >= 0)
    pos = _pos(sc)[perm]
    lo, hi = nd["lo"], nd["hi"]
    side = hi - lo
    for i in range(nn):
        # cube or 2:1, longest axis first in x, y, z order
        s = side[i]
        assert s.max() / s.min() in (1.0, 2.0)
        p = pos[first[i]:first[i] + count[i]]
        tol = 1e-12 * T.root_box()[3]
        assert np.all(p >= lo[i] - tol) and np.all(p <= hi[i] + tol)
        if not leaf[i]:
            a, b = c0[i], c1[i]
            assert a == i + 1 and b == nxt[a] and nxt[b] == nxt[i]
            assert count[a] + count[b] == count[i] and first[b] == first[a] + count[a]
            assert lown[a] == lown[b] == split[i] + 1 and split[i] >= lown[i]
            ax = split[i] % 3
            # children are the two halves of the split box along axis ax
            assert hi[a][ax] == lo[b][ax]
            assert hi[a][ax] - lo[a][ax] == pytest.approx(hi[b][ax] - lo[b][ax], rel=1e-15)
            for q in range(3):
                if q != ax:
                    assert lo[a][q] == lo[b][q] and hi[a][q] == hi[b][q]
            assert np.all(lo[a] >= lo[i]) and np.all(hi[b] <= hi[i])
        else:
            assert nxt[i] == i + 1


def test_uniform_lattice_alpha_tables_exact():
    """Section 2.6: volume-weighted bucket absorption of a uniform medium is
    kappa*rho, and transmission averaging of equal children keeps it, in
    every direction (a 16^3 lattice with leaf 8 has no empty sub-boxes)."""
    sc = scenes.lattice_scene(per_side=16, rho=2.0, kappa=(0.5, 3.0), nside=2)
    T = oracle.OracleTree(sc)
    nd = T.nodes()
    al = nd["alpha"]
    target = np.array([1.0, 6.0])
    assert np.allclose(al, target[None, None, :], rtol=1e-14, atol=0)
    assert np.all(nd["count"][nd["split"] < 0] == 8)


def test_random_medium_alpha_bounded_by_vacuum_inflation():
    """Empty prefix boxes are vacuum, so transmission averaging never raises
    alpha above the uniform value and only lowers it where boxes have gaps."""
    sc = scenes.uniform_scene(n=4000, seed=9, n_src=10, bands=(1.0, 4.0), nside=2)
    T = oracle.OracleTree(sc)
    al = T.nodes()["alpha"]
    assert np.all(al <= np.array([1.0, 4.0])[None, None, :] * (1 + 1e-12))
    assert np.all(al >= 0)


# ------------------------------------------------------ optically thin limit
def test_thin_theta0_equals_brute_force_sum():
    """No absorption and theta = 0: every cell opens, every bucket resolves
    into point sources, so J is the direct sum of L K(r, h) (Section 2.2)."""
    sc = scenes.uniform_scene(n=2048, seed=11, n_src=200, bands=(0.0, 0.0), nside=1, theta=0.0,
                              near_field=False, thick_corr=False)
    sc.lum[1] *= 3.0
    J, c = oracle.compute_J(sc)
    ref = bf.thin_sum(_pos(sc), sc.lum.astype(np.float64), _h(sc))
    assert _rel(J, ref) < 1e-12
    assert c["absorber_entries"] == 0


def test_thin_theta0_with_near_field_partitions_sources():
    """With the p-p sphere on, sources split into near (particle-particle)
    and far (point sources of opened buckets); their union is every source
    exactly once."""
    sc = scenes.uniform_scene(n=2048, seed=12, n_src=300, bands=(0.0,), nside=2, theta=0.0,
                              thick_corr=False)
    J, c = oracle.compute_J(sc)
    ref = bf.thin_sum(_pos(sc), sc.lum.astype(np.float64), _h(sc))
    assert _rel(J, ref) < 1e-12
    assert c["near_pairs"] > 0


def test_thin_theta_default_multipole_error_small():
    """theta = 0.75 in a transparent medium: the merged-source (monopole at
    the luminosity centre) error stays small (Section 2.5.2 bounds the
    higher moments)."""
    sc = scenes.uniform_scene(n=4096, seed=13, n_src=400, bands=(0.0,), nside=2, thick_corr=False)
    J, _ = oracle.compute_J(sc)
    ref = bf.thin_sum(_pos(sc), sc.lum.astype(np.float64), _h(sc))
    err = np.abs(J - ref) / ref
    assert np.median(err) < 0.01
    assert np.percentile(err, 99) < 0.05


def test_single_source_inverse_square():
    """One source in a transparent medium: J = L K(r, h) exactly for every
    receiver (its cell's luminosity centre is the source), which is
    L/(4 pi r^2) far from it."""
    sc = scenes.uniform_scene(n=3000, seed=14, n_src=1, bands=(0.0,), nside=2, thick_corr=False)
    J, _ = oracle.compute_J(sc)
    s = int(np.nonzero(sc.lum[0])[0][0])
    pos, h = _pos(sc), _h(sc)
    r = np.linalg.norm(pos - pos[s], axis=1)
    ref = sc.lum[0, s] * bf.kernel(r, h)
    assert _rel(J[0], ref) < 1e-12
    far = r > 8 * h
    assert far.sum() > 100
    assert _rel(J[0][far], sc.lum[0, s] / (4 * np.pi * r[far] ** 2)) < 3e-3


# ------------------------------------------------------ pure p-p reduction
@pytest.mark.parametrize("seed", [21, 22])
def test_pp_sphere_covering_scene_is_pairwise_transfer(seed):
    """A p-p radius larger than the root-cube diagonal puts every particle in
    every bucket's near set and leaves no cell work: J must equal pairwise
    particle-particle transfer (Section 2.4) computed by brute force."""
    rng = np.random.default_rng(seed)
    sc = scenes.uniform_scene(n=256, seed=seed, n_src=70, bands=(1.0, 10.0), nside=1)
    sc.rho[:] = rng.uniform(0.5, 2.0, sc.n).astype(np.float32)
    sc.lum[1] *= rng.uniform(0.5, 2.0, sc.n).astype(np.float32)
    sc = sc.with_(rpp_min=2.0)
    J, c = oracle.compute_J(sc)
    ref = bf.pairwise_pp(_pos(sc), sc.m.astype(np.float64), sc.rho.astype(np.float64),
                         sc.kappa.astype(np.float64), sc.lum.astype(np.float64))
    assert _rel(J, ref) < 1e-12
    assert c["cells"] == 0 and c["source_entries"] == 0 and c["absorber_entries"] == 0
    assert c["max_near"] == sc.n


# -------------------------------------------------------- uniform absorber
def test_uniform_lattice_attenuation():
    """A source in a uniform medium (kappa rho = 1, h = 1/16): far from the
    source J follows L K(r) e^{-kappa rho r} (cell chords tile the rays
    beyond r_pp; p-p columns approximate the continuum inside it)."""
    n1 = 16
    src = (5 * n1 + 6) * n1 + 4
    sc = scenes.lattice_scene(per_side=n1, rho=1.0, kappa=(1.0,), src_index=src, nside=2,
                              thick_corr=False)
    J, _ = oracle.compute_J(sc)
    pos, h = _pos(sc), _h(sc)
    r = np.linalg.norm(pos - pos[src], axis=1)
    sel = r > 4 * h
    ref = bf.kernel(r[sel], h[sel]) * np.exp(-r[sel])
    lr = np.log(J[0][sel] / ref)
    assert np.median(np.abs(lr)) < 0.05
    assert np.max(np.abs(lr)) < 0.35


# -------------------------------------------------------------- invariances
def _scene_small(seed=31, **kw):
    sc = scenes.lognormal_scene(n=3000, seed=seed, grid=16, bands=(1.0, 10.0), nside=2, **kw)
    return sc


def test_luminosity_linearity():
    sc = _scene_small()
    J1, _ = oracle.compute_J(sc)
    J2, _ = oracle.compute_J(sc.with_(lum=(sc.lum * np.float32(4.0))))
    assert _rel(J2, 4.0 * J1) < 1e-12


def test_length_scale_invariance():
    """x -> s x, rho -> rho/s^3, kappa -> kappa s^2 (same optical depths):
    J -> J/s^2, decisions unchanged (s a power of two)."""
    sc = _scene_small(seed=32)
    s = np.float32(2.0)
    sc2 = sc.with_(x=sc.x * s, y=sc.y * s, z=sc.z * s, rho=sc.rho / s ** 3, kappa=sc.kappa * s * s,
                   box=(0.0, 0.0, 0.0, 2.0))
    J1, c1 = oracle.compute_J(sc)
    J2, c2 = oracle.compute_J(sc2)
    assert c1 == c2
    assert _rel(J2, J1 / 4.0) < 1e-12


def test_permutation_invariance():
    sc = _scene_small(seed=33)
    rng = np.random.default_rng(0)
    p = rng.permutation(sc.n)
    scp = sc.with_(x=sc.x[p], y=sc.y[p], z=sc.z[p], m=sc.m[p], rho=sc.rho[p],
                   kappa=sc.kappa[:, p], lum=sc.lum[:, p], active=sc.active[p])
    J1, c1 = oracle.compute_J(sc)
    J2, c2 = oracle.compute_J(scp)
    assert c1 == c2
    assert _rel(J2, J1[:, p]) < 1e-13


def test_band_permutation_equivariance():
    sc = scenes.lognormal_scene(n=3000, seed=34, grid=16, bands=(1.0, 10.0, 100.0), nside=1)
    sc.lum[1] *= 2.0
    sc.lum[2] *= 0.5
    p = [2, 0, 1]
    J1, _ = oracle.compute_J(sc)
    J2, _ = oracle.compute_J(sc.with_(kappa=sc.kappa[p], lum=sc.lum[p]))
    assert _rel(J2, J1[p]) < 1e-10


def test_translation_invariance():
    """Shift by a power of two with the root box: quantised positions shift
    exactly, J is unchanged."""
    sc = _scene_small(seed=35)
    q = lambda a: (np.round(a.astype(np.float64) * 2 ** 20) / 2 ** 20).astype(np.float32)
    sc = sc.with_(x=q(sc.x), y=q(sc.y), z=q(sc.z))
    sh = np.float32(4.0)
    sc2 = sc.with_(x=sc.x + sh, y=sc.y - sh, z=sc.z + sh, box=(4.0, -4.0, 4.0, 1.0))
    J1, c1 = oracle.compute_J(sc)
    J2, c2 = oracle.compute_J(sc2)
    assert c1 == c2
    assert _rel(J2, J1) < 1e-12


def test_active_subset_matches_full_run():
    """Buckets are independent given the tree: the J of an active subset is
    the full run's J on those rows, other rows untouched."""
    sc = _scene_small(seed=36)
    J1, _ = oracle.compute_J(sc)
    act = scenes.active_subset(sc, 0.1, 3)
    T = oracle.OracleTree(sc)
    J2, c2 = T.compute_J(act, J_init=np.full_like(J1, -7.0))
    a = act.astype(bool)
    assert np.array_equal(J2[:, a], J1[:, a])
    assert np.all(J2[:, ~a] == -7.0)


# ------------------------------------------------------------- cost law
@pytest.mark.parametrize("kind", ["uniform", "lognormal"])
def test_cost_grows_as_log2_n(kind):
    """Section 3.1 (and 2.5.1): work per active receiver grows as log2 N,
    over N = 2^12 .. 2^21 (linear fit in log2 N, R^2 >= 0.98)."""
    lg = np.arange(12, 22)
    seg = []
    for k in lg:
        n = 2 ** int(k)
        if kind == "uniform":
            sc = scenes.uniform_scene(n=n, seed=int(k), n_src=n // 10, bands=(1.0,), nside=2)
        else:
            sc = scenes.lognormal_scene(n=n, seed=int(k), grid=32, bands=(1.0,), nside=2)
        act = scenes.active_subset(sc, min(1.0, 1500 / n), 5)
        J, c = oracle.OracleTree(sc).compute_J(act)
        seg.append(c["segments"] / act.sum())
    seg = np.array(seg)
    A = np.vstack([lg, np.ones_like(lg)]).T.astype(np.float64)
    coef, res, _, _ = np.linalg.lstsq(A, seg, rcond=None)
    r2 = 1 - res[0] / ((seg - seg.mean()) ** 2).sum()
    assert coef[0] > 0
    assert r2 >= 0.98
