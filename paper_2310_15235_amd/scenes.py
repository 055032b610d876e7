"""Seeded synthetic scenes (inputs only).

The paper's own workloads (a zoomed galaxy snapshot, glass initial conditions)
are not available, so these generators stand in for them with the structure
the paper describes: gas elements that absorb, receive and may emit, point
sources with a wide luminosity spread, multi-band opacities, off-centre
features (Appendix A) and active subsets (Section 1.2).

This module holds inputs and nothing of the method: no element sizes,
absorption coefficients, tree or ray arithmetic.  Both the HIP path and the
oracle consume the same arrays.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

import numpy as np


@dataclass
class Scene:
    x: np.ndarray          # float32 [n]
    y: np.ndarray
    z: np.ndarray
    m: np.ndarray          # float32 [n] element mass
    rho: np.ndarray        # float32 [n] element density
    kappa: np.ndarray      # float32 [B, n] opacity per band (per unit mass)
    lum: np.ndarray        # float32 [B, n] luminosity per band
    active: np.ndarray     # uint8 [n]
    nside: int = 2
    leaf_size: int = 8
    theta: float = 0.75
    thick_corr: bool = True
    near_field: bool = True
    background: bool = False
    absorption_avg: bool = False      # linear absorption averaging instead of transmission
    directed: Optional[Tuple[float, float, float]] = None   # target of directed rays
    complex_source: bool = False      # complex source model (per-direction source absorption)
    bg: Optional[np.ndarray] = None   # float32 [B] isotropic background intensity
    rpp_min: float = 0.0
    box: Optional[Tuple[float, float, float, float]] = (0.0, 0.0, 0.0, 1.0)
    name: str = "scene"
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_bands(self) -> int:
        return int(self.kappa.shape[0])

    def with_(self, **kw) -> "Scene":
        return replace(self, **kw)

    def positions(self) -> np.ndarray:
        return np.stack([self.x, self.y, self.z], axis=1)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _lognormal_sources(rng, n, n_src, sigma_dex=1.0):
    lum = np.zeros(n, dtype=np.float64)
    idx = rng.choice(n, size=n_src, replace=False)
    lum[idx] = 10.0 ** rng.normal(0.0, sigma_dex, size=n_src)
    return lum


def uniform_scene(n=4096, seed=1, n_src=64, bands=(1.0,), nside=1, leaf_size=8, theta=0.75,
                  rho=1.0, name=None, **kw) -> Scene:
    """Uniform-random elements in the unit cube, uniform density, a set of
    sources at random element positions with log-normal luminosities
    (sigma 1 dex), grey spectra."""
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3))
    m = np.full(n, rho / n)
    rh = np.full(n, rho)
    L = _lognormal_sources(rng, n, n_src)
    B = len(bands)
    kappa = np.repeat(np.asarray(bands, dtype=np.float64)[:, None], n, axis=1)
    lum = np.repeat(L[None, :], B, axis=0)
    return Scene(x=_f32(pos[:, 0]), y=_f32(pos[:, 1]), z=_f32(pos[:, 2]), m=_f32(m), rho=_f32(rh),
                 kappa=_f32(kappa), lum=_f32(lum), active=np.ones(n, np.uint8), nside=nside,
                 leaf_size=leaf_size, theta=theta, name=name or f"uniform{n}", **kw)


def gaussian_random_field(rng, grid, slope=-3.0, sigma=1.5):
    """Periodic Gaussian random field: white noise shaped by sqrt(P(k)),
    P ~ k^slope, k = 0 removed, scaled to standard deviation sigma."""
    white = rng.normal(size=(grid, grid, grid))
    fk = np.fft.rfftn(white)
    kx = np.fft.fftfreq(grid) * grid
    kz = np.fft.rfftfreq(grid) * grid
    k2 = kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2
    amp = np.zeros_like(k2)
    nz = k2 > 0
    amp[nz] = k2[nz] ** (slope / 4.0)  # sqrt(P) with P ~ k^slope
    delta = np.fft.irfftn(fk * amp, s=(grid, grid, grid), axes=(0, 1, 2))
    delta *= sigma / delta.std()
    return delta


def lognormal_scene(n=2 ** 18, seed=2, grid=64, bands=(1.0, 10.0, 100.0), src_frac=0.10,
                    nside=2, leaf_size=8, theta=0.75, sigma_ln=1.5, name=None, **kw) -> Scene:
    """Clumpy medium: a log-normal density field (Gaussian random field with
    P(k) ~ k^-3, sigma_ln rho = 1.5) on a periodic grid over the unit cube;
    elements drawn per cell in proportion to the cell mass and placed
    uniformly inside it, carrying the cell density; equal masses; a fraction
    of elements are sources with log-normal luminosities."""
    rng = np.random.default_rng(seed)
    delta = gaussian_random_field(rng, grid, sigma=sigma_ln)
    rho_grid = np.exp(delta - 0.5 * sigma_ln ** 2)
    p = (rho_grid / rho_grid.sum()).ravel()
    counts = rng.multinomial(n, p)
    cells = np.repeat(np.arange(grid ** 3), counts)
    ix, iy, iz = np.unravel_index(cells, (grid, grid, grid))
    off = rng.random((n, 3))
    pos = (np.stack([ix, iy, iz], axis=1) + off) / grid
    rh = rho_grid.ravel()[cells]
    m = np.full(n, rho_grid.mean() / n)
    L = _lognormal_sources(rng, n, int(round(src_frac * n)))
    B = len(bands)
    kappa = np.repeat(np.asarray(bands, dtype=np.float64)[:, None], n, axis=1)
    lum = np.repeat(L[None, :], B, axis=0)
    return Scene(x=_f32(pos[:, 0]), y=_f32(pos[:, 1]), z=_f32(pos[:, 2]), m=_f32(m), rho=_f32(rh),
                 kappa=_f32(kappa), lum=_f32(lum), active=np.ones(n, np.uint8), nside=nside,
                 leaf_size=leaf_size, theta=theta, name=name or f"lognormal{n}", **kw)


def isothermal_scene(n=2 ** 21, seed=3, core=0.05, centre=(0.37, 0.41, 0.29),
                     bands=(1.0, 10.0), nside=4, leaf_size=8, theta=0.75, active_frac=1.0,
                     name=None, **kw) -> Scene:
    """Diffuse emission: rho(x) = 1/(|x - x_c|^2 + a^2) + 1 in the unit cube
    (an isothermal-sphere profile with core radius a, off-centre in one
    octant) sampled with equal masses; every element emits L = rho/<rho>;
    an isotropic background equal to the emission-weighted thin field at
    distance 0.5 divided by 4 pi; an active subset drawn uniformly."""
    rng = np.random.default_rng(seed)
    c = np.asarray(centre)
    corners = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], float)
    rmax = np.sqrt(((corners - c) ** 2).sum(1)).max()
    # Radial inverse CDF of 4 pi r^2 / (r^2 + a^2) on [0, rmax].
    rg = np.linspace(0.0, rmax, 200001)
    cdf = 4 * np.pi * (rg - core * np.arctan(rg / core))
    m_ball = cdf[-1]
    # Mass of the sphere term inside the box (Monte Carlo acceptance).
    u = np.interp(rng.random(400000) * m_ball, cdf, rg)
    d = rng.normal(size=(400000, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    pts = c + u[:, None] * d
    acc = np.all((pts >= 0) & (pts < 1), axis=1).mean()
    m_sph = m_ball * acc
    frac_sph = m_sph / (m_sph + 1.0)
    out = []
    need = n
    while need > 0:
        k = int(need * 1.3) + 1024
        comp = rng.random(k) < frac_sph
        u = np.interp(rng.random(k) * m_ball, cdf, rg)
        d = rng.normal(size=(k, 3))
        d /= np.linalg.norm(d, axis=1)[:, None]
        sph = c + u[:, None] * d
        uni = rng.random((k, 3))
        pts = np.where(comp[:, None], sph, uni)
        ok = np.all((pts >= 0) & (pts < 1), axis=1)
        pts = pts[ok][:need]
        out.append(pts)
        need -= pts.shape[0]
    pos = np.concatenate(out, axis=0)
    rr2 = ((pos - c) ** 2).sum(1)
    rh = 1.0 / (rr2 + core ** 2) + 1.0
    m = np.full(n, (m_sph + 1.0) / n)
    L = rh / rh.mean()
    B = len(bands)
    kappa = np.repeat(np.asarray(bands, dtype=np.float64)[:, None], n, axis=1)
    lum = np.repeat(L[None, :], B, axis=0)
    bg = lum.sum(axis=1) / (16 * np.pi ** 2 * 0.5 ** 2)
    active = np.zeros(n, np.uint8)
    na = int(round(active_frac * n))
    active[rng.choice(n, size=na, replace=False)] = 1
    return Scene(x=_f32(pos[:, 0]), y=_f32(pos[:, 1]), z=_f32(pos[:, 2]), m=_f32(m), rho=_f32(rh),
                 kappa=_f32(kappa), lum=_f32(lum), active=active, nside=nside, leaf_size=leaf_size,
                 theta=theta, background=True, bg=_f32(bg), name=name or f"isothermal{n}", **kw)


def lattice_scene(per_side=16, rho=1.0, kappa=(1.0,), src_index=None, src_lum=1.0, nside=2,
                  leaf_size=8, theta=0.75, name=None, **kw) -> Scene:
    """Cell-centred cubic lattice in the unit cube, uniform density."""
    g = (np.arange(per_side) + 0.5) / per_side
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    n = per_side ** 3
    m = np.full(n, rho / n)
    L = np.zeros(n)
    if src_index is not None:
        L[src_index] = src_lum
    B = len(kappa)
    kap = np.repeat(np.asarray(kappa, dtype=np.float64)[:, None], n, axis=1)
    lum = np.repeat(L[None, :], B, axis=0)
    return Scene(x=_f32(X.ravel()), y=_f32(Y.ravel()), z=_f32(Z.ravel()), m=_f32(m),
                 rho=_f32(np.full(n, rho)), kappa=_f32(kap), lum=_f32(lum),
                 active=np.ones(n, np.uint8), nside=nside, leaf_size=leaf_size, theta=theta,
                 name=name or f"lattice{per_side}", **kw)


# ------------------------------------------------------------ named workloads
def config_tiny() -> Scene:
    """4096 uniform elements, rho = 1, one band with box optical depth 1,
    64 log-normal point sources at element positions, N_side 1, leaf 8."""
    return uniform_scene(n=4096, seed=1, n_src=64, bands=(1.0,), nside=1, name="tiny4096")


def config_clumpy(n=2 ** 18, seed=2, grid=64) -> Scene:
    """2^18 elements in a log-normal medium, 10% sources, 3 bands with
    opacity ratios 1:10:100, N_side 2, all active."""
    return lognormal_scene(n=n, seed=seed, grid=grid, bands=(1.0, 10.0, 100.0), nside=2,
                           name=f"clumpy{n}")


def config_diffuse(active_frac=1.0, n=2 ** 21, seed=3) -> Scene:
    """2^21 elements in an off-centre isothermal sphere plus uniform
    background, every element emits, isotropic background, N_side 4,
    2 bands, an active fraction."""
    return isothermal_scene(n=n, seed=seed, active_frac=active_frac,
                            name=f"diffuse{n}_a{active_frac:g}")


def config_differentiation(n=2 ** 18, seed=5, grid=64) -> Scene:
    """2^18-element log-normal medium, 2 bands (opacity 1, 10), N_side 2."""
    return lognormal_scene(n=n, seed=seed, grid=grid, bands=(1.0, 10.0), nside=2,
                           name=f"diff{n}")


def config_differentiation_small() -> Scene:
    return lognormal_scene(n=2 ** 12, seed=6, grid=16, bands=(1.0, 10.0), nside=2, name="diff4096")


def batched_scenes(count=64, seed0=1000):
    """Independent scenes with log-uniform sizes 2^12..2^17, a random mix of
    uniform and log-normal media, 1-4 bands and N_side in {1, 2, 4}."""
    out = []
    for s in range(count):
        rng = np.random.default_rng(seed0 + s)
        n = int(round(2 ** rng.uniform(12, 17)))
        B = int(rng.integers(1, 5))
        bands = (1.0, 10.0, 100.0, 1000.0)[:B]
        nside = int(rng.choice([1, 2, 4]))
        if rng.random() < 0.5:
            sc = uniform_scene(n=n, seed=seed0 + s, n_src=max(1, n // 64), bands=bands,
                               nside=nside, name=f"batch{s}_uniform{n}")
        else:
            grid = 32 if n < 2 ** 15 else 64
            sc = lognormal_scene(n=n, seed=seed0 + s, grid=grid, bands=bands, nside=nside,
                                 name=f"batch{s}_lognormal{n}")
        out.append(sc)
    return out


def active_subset(scene: Scene, frac: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    a = np.zeros(scene.n, np.uint8)
    a[rng.choice(scene.n, size=max(1, int(round(frac * scene.n))), replace=False)] = 1
    return a


# ------------------------------------------- the paper's fixed-opacity tests
def _jittered_lattice(rng, lo, hi, spacing, jitter=0.25):
    """Cubic lattice of the given spacing filling the box [lo, hi)^3, each
    point moved by up to +-jitter*spacing per axis: a stand-in for the glass
    initial conditions of Section 3.3, with the same spacing and no two
    elements at one position."""
    axes = [np.arange(lo[a] + 0.5 * spacing, hi[a], spacing) for a in range(3)]
    X, Y, Z = np.meshgrid(*axes, indexing="ij")
    p = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    return p + rng.uniform(-jitter, jitter, p.shape) * spacing


def _escape_scene(pos, spacing, alpha, src_pos, src_lum, box, meta, nside, theta, leaf_size,
                  avg, name):
    """Elements of density 1 and volume spacing^3 (so h is the local
    spacing) with opacity alpha (alpha = kappa rho), one band, plus a source
    element at each of src_pos with luminosity src_lum and the local medium
    around it.  The thick-element factor is off: these tests measure the
    incident intensity.  All elements are receivers (the tests pick a shell
    as the active set)."""
    n_med = pos.shape[0]
    pos = np.concatenate([pos, np.asarray(src_pos, float)], axis=0)
    spacing = np.concatenate([spacing, meta.pop("src_spacing")])
    alpha = np.concatenate([alpha, meta.pop("src_alpha")])
    n = pos.shape[0]
    lum = np.zeros(n)
    lum[n_med:] = src_lum
    meta.update(sources=np.arange(n_med, n), src_pos=np.asarray(src_pos, float),
                src_lum=np.asarray(src_lum, float))
    return Scene(x=_f32(pos[:, 0]), y=_f32(pos[:, 1]), z=_f32(pos[:, 2]), m=_f32(spacing ** 3),
                 rho=_f32(np.ones(n)), kappa=_f32(alpha[None, :]), lum=_f32(lum[None, :]),
                 active=np.ones(n, np.uint8), nside=nside, leaf_size=leaf_size, theta=theta,
                 thick_corr=False, box=box, absorption_avg=avg, name=name, meta=meta)


def source_features_scene(feature="clouds", seed=7, avg=False, nside=2, theta=0.75,
                          leaf_size=12, outer=0.0625, inner=0.0209) -> Scene:
    """Section 3.4 tests: a source of L = 1 at (0.17, 0.17, 0.17) in a
    medium of alpha = 1 filling the sphere of radius 2.5 about the origin,
    element spacing 0.0625 outside and 0.0209 within 0.4 of the source, and
      feature = "none":   nothing else (escape at r = 2 is e^-2);
      feature = "clouds": two clouds of radius 0.1 and alpha = 10 offset by
                          +-0.25 along the main diagonal (Section 3.4.1);
      feature = "wall":   alpha = 10 beyond the plane 0.25 from the source
                          along -(1,1,1)/sqrt(3) (Section 3.4.2).
    Escape fractions are measured at distance 2 from the source."""
    rng = np.random.default_rng(seed)
    src = np.array([0.17, 0.17, 0.17])
    diag = np.ones(3) / np.sqrt(3.0)
    po = _jittered_lattice(rng, (-2.5,) * 3, (2.5,) * 3, outer)
    po = po[(np.linalg.norm(po, axis=1) < 2.5) & (np.linalg.norm(po - src, axis=1) >= 0.4)]
    pi = _jittered_lattice(rng, src - 0.4, src + 0.4, inner)
    pi = pi[np.linalg.norm(pi - src, axis=1) < 0.4]
    pos = np.concatenate([po, pi], axis=0)
    spacing = np.concatenate([np.full(len(po), outer), np.full(len(pi), inner)])

    def alpha_at(p):
        a = np.ones(len(p))
        if feature == "clouds":
            for sgn in (1.0, -1.0):
                a[np.linalg.norm(p - (src + sgn * 0.25 * diag), axis=1) < 0.1] = 10.0
        elif feature == "wall":
            a[(p - src) @ diag < -0.25] = 10.0
        elif feature != "none":
            raise ValueError(feature)
        return a

    meta = dict(test=f"source+{feature}", centre=src, radius=2.0, medium_alpha=1.0,
                src_spacing=np.array([inner]), src_alpha=alpha_at(src[None, :]))
    return _escape_scene(pos, spacing, alpha_at(pos), [src], [1.0], (-2.5, -2.5, -2.5, 5.0),
                         meta, nside, theta, leaf_size, avg,
                         f"source_{feature}{'_absavg' if avg else ''}")


def two_sources_cloud_scene(seed=8, avg=False, nside=2, theta=0.75, leaf_size=12,
                            outer=0.25, inner=0.0625, cloud=True) -> Scene:
    """Section 3.3: a sphere of radius 0.5 at the origin with alpha = 10^4
    (element spacing 0.0625) in a medium of alpha = 10^-4 (spacing 0.25), two
    sources of L = 0.5 at (-2, 0, 0) and (0, -2, 0); the volume is centred on
    (-2.1, -2.1, -2.1) so that the sources and the cloud share a moderately
    sized tree cell (Appendix A), and reaches past radius 6 about the origin,
    where escape fractions are measured."""
    rng = np.random.default_rng(seed)
    half = 8.2
    c = np.array([-2.1, -2.1, -2.1])
    po = _jittered_lattice(rng, c - half, c + half, outer)
    pos_list, sp_list = [po[np.linalg.norm(po, axis=1) >= 0.5]], []
    sp_list.append(np.full(len(pos_list[0]), outer))
    if cloud:
        pi = _jittered_lattice(rng, (-0.5,) * 3, (0.5,) * 3, inner)
        pi = pi[np.linalg.norm(pi, axis=1) < 0.5]
        pos_list.append(pi)
        sp_list.append(np.full(len(pi), inner))
    pos = np.concatenate(pos_list, axis=0)
    spacing = np.concatenate(sp_list)
    alpha = np.where(np.linalg.norm(pos, axis=1) < 0.5, 1e4 if cloud else 1e-4, 1e-4)
    srcs = np.array([[-2.0, 0.0, 0.0], [0.0, -2.0, 0.0]])
    meta = dict(test="two sources+cloud" if cloud else "two sources", centre=np.zeros(3),
                radius=6.0, medium_alpha=1e-4, src_spacing=np.full(2, outer),
                src_alpha=np.full(2, 1e-4))
    box = (c[0] - half, c[1] - half, c[2] - half, 2 * half)
    return _escape_scene(pos, spacing, alpha, srcs, [0.5, 0.5], box, meta, nside, theta,
                         leaf_size, avg, f"two_sources_cloud{'_absavg' if avg else ''}")


def shell_active(scene: Scene, width=None) -> np.ndarray:
    """Receivers of an escape measurement: elements within `width` (default
    one outer spacing, 0.0625 or 0.25) of the measuring radius about the
    test's centre."""
    c, R = scene.meta["centre"], scene.meta["radius"]
    if width is None:
        width = 0.25 if R > 3 else 0.0625
    r = np.linalg.norm(scene.positions().astype(np.float64) - c, axis=1)
    a = (np.abs(r - R) < width).astype(np.uint8)
    a[scene.meta["sources"]] = 0
    return a
