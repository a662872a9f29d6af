"""Density-compensation weights: the measure of each point's Voronoi cell,
clipped to a bandwidth region (App. B).

Reading of the undefined bandwidth region Y_K: in 1D the interval [-K, K];
for spiral patterns the disk of radius r_max + (arm gap)/2; for jittered
grids the square band that holds the grid.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.spatial import Voronoi


def voronoi_weights_1d(xi: np.ndarray, K: float) -> np.ndarray:
    """Cell lengths (xi_{m+1} - xi_{m-1}) / 2, end cells clipped to [-K, K]."""
    xi = np.asarray(xi, dtype=np.float64)
    order = np.argsort(xi, kind="stable")
    s = xi[order]
    mid = 0.5 * (s[1:] + s[:-1])
    lo = np.concatenate([[-K], mid])
    hi = np.concatenate([mid, [K]])
    w = np.empty_like(s)
    w[order] = np.clip(hi, -K, K) - np.clip(lo, -K, K)
    return w


def _shoelace(vx, vy, starts, counts):
    """Polygon areas from flattened vertex lists (counter-clockwise or not)."""
    nxt = np.arange(vx.size) + 1
    ends = starts + counts
    nxt[ends - 1] = starts
    cross = vx * vy[nxt] - vx[nxt] * vy
    return 0.5 * np.abs(np.add.reduceat(cross, starts))


def _seg_disk_area(ax, ay, bx, by, R):
    """Signed area of triangle (0, a, b) intersected with the disk |z| <= R."""
    def sector(ux, uy, vx, vy):
        ang = math.atan2(ux * vy - uy * vx, ux * vx + uy * vy)
        return 0.5 * R * R * ang

    da = math.hypot(ax, ay)
    db = math.hypot(bx, by)
    dx, dy = bx - ax, by - ay
    A = dx * dx + dy * dy
    if A == 0:
        return 0.0
    Bq = 2 * (ax * dx + ay * dy)
    C = ax * ax + ay * ay - R * R
    disc = Bq * Bq - 4 * A * C
    if da <= R and db <= R:
        return 0.5 * (ax * by - ay * bx)
    if disc <= 0:
        return sector(ax, ay, bx, by)
    sq = math.sqrt(disc)
    t1 = (-Bq - sq) / (2 * A)
    t2 = (-Bq + sq) / (2 * A)
    p1 = (ax + t1 * dx, ay + t1 * dy)
    p2 = (ax + t2 * dx, ay + t2 * dy)
    if da <= R:                      # a inside, b outside: exit at t2
        return 0.5 * (ax * p2[1] - ay * p2[0]) + sector(p2[0], p2[1], bx, by)
    if db <= R:                      # a outside, b inside: enter at t1
        return sector(ax, ay, p1[0], p1[1]) + 0.5 * (p1[0] * by - p1[1] * bx)
    if t1 >= 1 or t2 <= 0 or t1 >= t2:   # chord misses the segment
        return sector(ax, ay, bx, by)
    return (sector(ax, ay, p1[0], p1[1]) + 0.5 * (p1[0] * p2[1] - p1[1] * p2[0])
            + sector(p2[0], p2[1], bx, by))


def _clip_square(poly, H):
    """Sutherland-Hodgman clip of a convex polygon to [-H, H]^2."""
    def clip(pts, inside, inter):
        out = []
        n = len(pts)
        for i in range(n):
            cur, prev = pts[i], pts[i - 1]
            ci, pi_ = inside(cur), inside(prev)
            if ci:
                if not pi_:
                    out.append(inter(prev, cur))
                out.append(cur)
            elif pi_:
                out.append(inter(prev, cur))
        return out

    def ix(a, b, x):
        t = (x - a[0]) / (b[0] - a[0])
        return (x, a[1] + t * (b[1] - a[1]))

    def iy(a, b, y):
        t = (y - a[1]) / (b[1] - a[1])
        return (a[0] + t * (b[0] - a[0]), y)

    pts = [tuple(v) for v in poly]
    pts = clip(pts, lambda q: q[0] <= H, lambda a, b: ix(a, b, H))
    if pts:
        pts = clip(pts, lambda q: q[0] >= -H, lambda a, b: ix(a, b, -H))
    if pts:
        pts = clip(pts, lambda q: q[1] <= H, lambda a, b: iy(a, b, H))
    if pts:
        pts = clip(pts, lambda q: q[1] >= -H, lambda a, b: iy(a, b, -H))
    if len(pts) < 3:
        return 0.0
    a = 0.0
    for i in range(len(pts)):
        x0, y0 = pts[i - 1]
        x1, y1 = pts[i]
        a += x0 * y1 - x1 * y0
    return 0.5 * abs(a)


def voronoi_weights_2d(pts: np.ndarray, region: str, size: float, guard_spacing: float) -> np.ndarray:
    """Voronoi cell areas of ``pts`` (M, 2) clipped to ``region``:
    'disk' of radius ``size`` or 'square' [-size, size]^2.  A ring of guard
    points outside the region keeps every real cell bounded."""
    pts = np.asarray(pts, dtype=np.float64)
    M = pts.shape[0]
    if region == "disk":
        Rg = size + 2 * guard_spacing
        ng = max(64, int(2 * math.pi * Rg / guard_spacing))
        ang = 2 * math.pi * np.arange(ng) / ng
        guards = [np.stack([Rg * np.cos(ang), Rg * np.sin(ang)], 1),
                  np.stack([2 * Rg * np.cos(ang), 2 * Rg * np.sin(ang)], 1)]
    elif region == "square":
        Hg = size + 2 * guard_spacing
        ng = max(16, int(2 * Hg / guard_spacing))
        c = np.linspace(-Hg, Hg, ng + 1)
        ring = np.concatenate([np.stack([c, np.full_like(c, -Hg)], 1), np.stack([c, np.full_like(c, Hg)], 1),
                               np.stack([np.full_like(c, -Hg), c], 1), np.stack([np.full_like(c, Hg), c], 1)])
        guards = [ring, 2 * ring]
    else:
        raise ValueError(region)
    allp = np.concatenate([pts] + guards)
    vor = Voronoi(allp)
    regs = [vor.regions[vor.point_region[i]] for i in range(M)]
    counts = np.fromiter((len(r) for r in regs), dtype=np.int64, count=M)
    if np.any(counts < 3) or any(-1 in r for r in regs):
        raise RuntimeError("unbounded Voronoi cell for a real point; enlarge the guard ring")
    flat = np.fromiter((v for r in regs for v in r), dtype=np.int64, count=int(counts.sum()))
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    V = vor.vertices
    vx, vy = V[flat, 0], V[flat, 1]
    area = _shoelace(vx, vy, starts, counts)
    if region == "disk":
        rad = np.hypot(vx, vy)
        rmax = np.maximum.reduceat(rad, starts)
        for i in np.nonzero(rmax > size)[0]:
            poly = V[regs[i]]
            a = 0.0
            for q in range(len(poly)):
                a += _seg_disk_area(poly[q - 1][0], poly[q - 1][1], poly[q][0], poly[q][1], size)
            area[i] = abs(a)
    else:
        amax = np.maximum.reduceat(np.maximum(np.abs(vx), np.abs(vy)), starts)
        for i in np.nonzero(amax > size)[0]:
            area[i] = _clip_square(V[regs[i]], size)
    return area
