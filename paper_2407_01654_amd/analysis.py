"""Host-side measurements on order-parameter fields (read back from the device):
the apparent contact angle of a sessile drop and the deformation factor of a
suspended one.  Plain numpy; they take fields, not simulations."""
from __future__ import annotations

import numpy as np


def interface_points(phi: np.ndarray, level: float = 0.5) -> np.ndarray:
    """Points (x, y) where phi crosses `level` between horizontally or
    vertically adjacent nodes, by linear interpolation (x periodic)."""
    pts = []
    a, b = phi, np.roll(phi, -1, axis=1)
    ys, xs = np.nonzero((a - level) * (b - level) < 0)
    t = (level - a[ys, xs]) / (b[ys, xs] - a[ys, xs])
    pts.append(np.stack([xs + t, ys.astype(float)], axis=1))
    a, b = phi[:-1], phi[1:]
    ys, xs = np.nonzero((a - level) * (b - level) < 0)
    t = (level - a[ys, xs]) / (b[ys, xs] - a[ys, xs])
    pts.append(np.stack([xs.astype(float), ys + t], axis=1))
    return np.concatenate(pts)


def fit_circle(x: np.ndarray, y: np.ndarray):
    """Least-squares circle through the points (algebraic fit:
    x^2 + y^2 = 2 a x + 2 b y + c, R^2 = c + a^2 + b^2)."""
    A = np.stack([2 * x, 2 * y, np.ones_like(x)], axis=1)
    sol, *_ = np.linalg.lstsq(A, x * x + y * y, rcond=None)
    a, b, c = sol
    return a, b, float(np.sqrt(c + a * a + b * b))


def contact_angle(phi: np.ndarray, wall_y: float = -0.5, exclude: float = 8.0) -> dict:
    """Apparent contact angle (inside the phase phi = 1) of a sessile drop on
    the bottom wall at y = wall_y: a circle is fitted to the phi = 1/2
    contour at least `exclude` lattice units above the wall (the diffuse
    contact-line region is left out), unwrapped about the drop's centre in x;
    for a circular cap with centre height y_c above the wall and radius R,
    cos(theta) = -(y_c - wall_y) / R."""
    nx = phi.shape[1]
    pts = interface_points(phi)
    # unwrap x about the drop's centre of mass (periodic x)
    col = np.clip(phi, 0, 1).sum(axis=0)
    ang = 2 * np.pi * np.arange(nx) / nx
    cx = (np.arctan2((col * np.sin(ang)).sum(), (col * np.cos(ang)).sum()) % (2 * np.pi)) * nx / (2 * np.pi)
    x = (pts[:, 0] - cx + nx / 2.0) % nx - nx / 2.0
    y = pts[:, 1]
    keep = y >= wall_y + exclude
    if keep.sum() < 6:
        raise ValueError(f"only {int(keep.sum())} interface points lie {exclude} units above the wall")
    a, b, R = fit_circle(x[keep], y[keep])
    cos_t = -(b - wall_y) / R
    return {"theta_deg": float(np.degrees(np.arccos(np.clip(cos_t, -1, 1)))), "cos_theta": float(cos_t),
            "radius": R, "centre_height": float(b - wall_y), "points": int(keep.sum())}


def deformation(phi: np.ndarray) -> float:
    """D = (L - B) / (L + B) of a drop, L along y (the field) and B along x,
    from the second moments of the region phi > 1/2 (a uniform ellipse of
    semi-axes L, B has moments L^2 / 4, B^2 / 4)."""
    w = np.where(phi > 0.5, np.clip(phi, 0, 1), 0.0)
    y, x = np.mgrid[0:phi.shape[0], 0:phi.shape[1]].astype(float)
    m = w.sum()
    cx, cy = (w * x).sum() / m, (w * y).sum() / m
    a = np.sqrt((w * (y - cy) ** 2).sum() / m)
    b = np.sqrt((w * (x - cx) ** 2).sum() / m)
    return float((a - b) / (a + b))


def deformation_contour(phi: np.ndarray, level: float = 0.5) -> float:
    """D = (L - B) / (L + B) of a drop from the ellipse fitted to its phi = 1/2
    contour (points interpolated between nodes, so the value changes smoothly
    as the drop deforms; the thresholded moments of `deformation` jump when a
    node crosses 1/2, by up to ~0.008 at radius 10).  The axis-aligned conic
    a x^2 + c y^2 + d x + e y = 1 is fitted by least squares about the
    contour's centroid: B^2 = k / a along x, L^2 = k / c along y, with
    k = 1 + d^2 / (4 a) + e^2 / (4 c).  The drop must not touch the domain's
    edges."""
    pts = interface_points(phi, level)
    x = pts[:, 0] - pts[:, 0].mean()
    y = pts[:, 1] - pts[:, 1].mean()
    A = np.stack([x * x, y * y, x, y], axis=1)
    (a, c, d, e), *_ = np.linalg.lstsq(A, np.ones_like(x), rcond=None)
    k = 1.0 + d * d / (4.0 * a) + e * e / (4.0 * c)
    B, L = np.sqrt(k / a), np.sqrt(k / c)
    return float((L - B) / (L + B))
