"""Independent brute-force references (numpy) that pin the oracle.

These do not share code with the oracle: they evaluate the paper's
particle-level model directly, O(N^2) or O(N^3), on tiny inputs.
"""
from __future__ import annotations

import numpy as np

R_SPHERE = np.sqrt(3.0 / (4.0 * np.pi))   # Section 2.2: sphere radius over element size


def f_sphere(x):
    """Shape of the element-averaged intensity (Section 2.2, eq. intint),
    evaluated from the printed logarithmic form, with its limits."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    z = x == 0
    one = x == 1
    big = x >= 10
    mid = ~(z | one | big)
    xm = x[mid]
    out[mid] = 1.0 + (xm * xm - 1.0) / (4.0 * xm) * np.log((xm - 1.0) ** 2 / (xm + 1.0) ** 2)
    out[z] = 2.0
    out[one] = 1.0
    xb = x[big]
    y2 = 1.0 / (xb * xb)
    s = np.zeros_like(xb)
    t = y2.copy()
    for k in range(1, 40):
        s += 2.0 * t / (4.0 * k * k - 1.0)
        t *= y2
    out[big] = s
    return out


def kernel(r, h):
    return f_sphere(np.asarray(r) / (R_SPHERE * np.asarray(h))) / (2.0 * np.asarray(h) ** 2)


def thick(tau):
    tau = np.asarray(tau, dtype=np.float64)
    out = np.ones_like(tau)
    nz = tau > 0
    out[nz] = -np.expm1(-tau[nz]) / tau[nz]
    return out


def thin_sum(pos, lum, h):
    """J_ib = sum_j L_jb K(|x_i - x_j|, h_i): every source as a point, no
    absorption (the optically thin limit, Section 2.2)."""
    d = np.sqrt(((pos[:, None, :] - pos[None, :, :]) ** 2).sum(-1))
    K = kernel(d, h[:, None])
    return lum @ K.T


def pairwise_pp(pos, m, rho, kappa, lum, thick_corr=True):
    """Pure particle-particle transfer (Section 2.4) between every receiver i
    and every source j: particles l (not i, not j) closer to the source than
    the receiver is, and within their size h_l of the segment i-j, attenuate
    by exp(-kappa_l Sigma_l(b)), Sigma_l(b) = 3 m_l/(pi h_l^2) (1 - b/h_l);
    the receiver's own column is excluded; self emission K(0) = 1/h_i^2."""
    n = pos.shape[0]
    B = kappa.shape[0]
    h = np.cbrt(m / rho)
    sig0 = 3.0 * m / (np.pi * h * h)
    J = np.zeros((B, n))
    srcs = np.nonzero(lum.sum(0) > 0)[0]
    for i in range(n):
        w = pos - pos[i]
        for j in srcs:
            if j == i:
                J[:, i] += lum[:, j] / h[i] ** 2
                continue
            e = pos[j] - pos[i]
            rij2 = e @ e
            front = ((pos - pos[j]) ** 2).sum(1) < rij2
            front[i] = False
            front[j] = False
            u = np.clip((w @ e) / rij2, 0.0, 1.0)
            f = w - u[:, None] * e
            b = np.sqrt((f * f).sum(1))
            hit = front & (b < h)
            col = sig0[hit] * (1.0 - b[hit] / h[hit])
            tau = kappa[:, hit] @ col
            J[:, i] += lum[:, j] * kernel(np.sqrt(rij2), h[i]) * np.exp(-tau)
    if thick_corr:
        J *= thick(kappa * rho[None, :] * h[None, :])
    return J


def column_sigma(b, m, h):
    """Section 2.4: the column of an element at impact parameter b falls
    linearly to zero at b = h and integrates to m over the disc b < h."""
    return np.where(b < h, 3.0 * m / (np.pi * h * h) * (1.0 - b / h), 0.0)


def ray_depth(pos, m, h, kappa, i, n, members):
    """Optical depth [B] of the elements `members` (not i) on the ray from
    element i along unit vector n: those ahead of it (positive projection)
    within their size of the ray line (Section 2.4)."""
    idx = np.asarray([l for l in members if l != i], dtype=np.int64)
    if idx.size == 0:
        return np.zeros(kappa.shape[0])
    d = pos[idx] - pos[i]
    proj = d @ n
    b = np.linalg.norm(np.cross(d, n), axis=1)
    ok = (proj > 0) & (b < h[idx])
    return kappa[:, idx[ok]] @ column_sigma(b[ok], m[idx[ok]], h[idx[ok]])


def segment_depth(pos, m, h, kappa, i, j, members):
    """Optical depth [B] of the elements `members` (not i, not j) between
    element i and a source j: those closer to j than i is, within their size
    of the segment (Section 2.4)."""
    idx = np.asarray([l for l in members if l != i and l != j], dtype=np.int64)
    e = pos[j] - pos[i]
    r2 = e @ e
    if idx.size == 0 or r2 == 0.0:          # no column between i and itself
        return np.zeros(kappa.shape[0])
    w = pos[idx] - pos[i]
    front = ((pos[idx] - pos[j]) ** 2).sum(1) < r2
    u = np.clip((w @ e) / r2, 0.0, 1.0)
    b = np.linalg.norm(w - u[:, None] * e, axis=1)
    ok = front & (b < h[idx])
    return kappa[:, idx[ok]] @ column_sigma(b[ok], m[idx[ok]], h[idx[ok]])


def box_exit(c, n, lo, L):
    """Distance from c (inside the cube [lo, lo + L]^3) along unit n to the
    cube's boundary."""
    t = np.inf
    for a in range(3):
        if n[a] > 0:
            t = min(t, (lo[a] + L - c[a]) / n[a])
        elif n[a] < 0:
            t = min(t, (lo[a] - c[a]) / n[a])
    return t
