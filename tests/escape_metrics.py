"""Figures of merit of the paper's fixed-opacity tests (Section 3.3, 3.4,
Table 'escape'), computed from J on the receivers of a measuring shell.

The escape fraction is the fraction of the emitted flux that reaches the
measuring radius R: per receiver, J over the exact no-feature value
J0 = sum_s L_s e^{-alpha0 r_s} / (4 pi r_s^2) (point sources in the uniform
medium alpha0), averaged over the shell (its receivers are spread evenly in
solid angle), times the no-feature escape e^{-alpha0 R}.  The covering
factor is the fraction of the shell where J is at most half of J0."""
import numpy as np


def no_feature_J(scene, active):
    pos = scene.positions().astype(np.float64)[active.astype(bool)]
    a0 = scene.meta["medium_alpha"]
    J0 = np.zeros(pos.shape[0])
    for p, L in zip(scene.meta["src_pos"], scene.meta["src_lum"]):
        r = np.linalg.norm(pos - p, axis=1)
        J0 += L * np.exp(-a0 * r) / (4 * np.pi * r * r)
    return J0


def escape_covering(scene, J, active):
    """(escape fraction, covering factor) from J [1, n] (or [n])."""
    J = np.asarray(J).reshape(-1, scene.n)[0]
    a = active.astype(bool)
    ratio = J[a] / no_feature_J(scene, active)
    e0 = np.exp(-scene.meta["medium_alpha"] * scene.meta["radius"])
    return float(e0 * ratio.mean()), float((ratio <= 0.5).mean())
