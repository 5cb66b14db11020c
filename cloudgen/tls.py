"""Terrestrial (TLS-like) synthetic scan with range-dependent density.

Recipe: a scanner at the origin shoots rays on a regular azimuth x elevation
grid (azimuth over the full circle, elevation in [-45, +45] degrees).  Each ray
keeps its first hit, found by exact ray intersection, among: the ground plane
z = -1.8 m, about 200 vertical cylinders (tree trunks, radius 0.1-0.5 m, 10 m
tall) and about 20 axis-aligned boxes (5-20 m wide, 3-10 m tall) placed
within 100 m; hits farther than 100 m are dropped.  Because the ray spacing is
angular, point density falls roughly as 1 / range^2.  The grid is chosen to
give more hits than needed and a seeded subset of exactly ``n`` is kept.
"""
import math

import numpy as np

GROUND_Z = -1.8
MAX_RANGE = 100.0


def _objects(rng, ncyl=200, nbox=20):
    cd = np.sqrt(rng.uniform(3.0 ** 2, 95.0 ** 2, ncyl))
    ca = rng.uniform(0.0, 2 * math.pi, ncyl)
    cyl = dict(cx=cd * np.cos(ca), cy=cd * np.sin(ca), r=rng.uniform(0.1, 0.5, ncyl),
               z0=np.full(ncyl, GROUND_Z), z1=np.full(ncyl, GROUND_Z + 10.0))
    bw = rng.uniform(5.0, 20.0, nbox); bd = rng.uniform(5.0, 20.0, nbox)
    dist = rng.uniform(15.0, 85.0, nbox) + 0.5 * np.hypot(bw, bd)
    ba = rng.uniform(0.0, 2 * math.pi, nbox)
    bx, by = dist * np.cos(ba), dist * np.sin(ba)
    box = dict(x0=bx - bw / 2, x1=bx + bw / 2, y0=by - bd / 2, y1=by + bd / 2,
               z0=np.full(nbox, GROUND_Z), z1=GROUND_Z + rng.uniform(3.0, 10.0, nbox))
    return cyl, box


def _az_window(n_az, a_lo, a_hi):
    """Azimuth grid indices in [a_lo, a_hi] (radians, may wrap)."""
    step = 2 * math.pi / n_az
    i0 = int(math.floor(a_lo / step)) - 1
    i1 = int(math.ceil(a_hi / step)) + 1
    return np.arange(i0, i1 + 1) % n_az


def tls_cloud(rng, n, n_az=None, n_el=None):
    cyl, box = _objects(rng)
    if n_az is None:
        # about half of the rays point downwards and hit the ground
        per = math.sqrt(n * 2.4 / 0.5)
        n_az = int(per * 1.4)
        n_el = int(per / 1.4)
    az = (np.arange(n_az) + 0.5) * (2 * math.pi / n_az)
    el = np.deg2rad(-45.0 + (np.arange(n_el) + 0.5) * (90.0 / n_el))
    cos_az, sin_az = np.cos(az), np.sin(az)
    out = []
    rows = max(1, int(4_000_000 // n_az))
    for e0 in range(0, n_el, rows):
        ce = np.cos(el[e0:e0 + rows])[:, None]
        se = np.sin(el[e0:e0 + rows])[:, None]
        dx = ce * cos_az[None, :]; dy = ce * sin_az[None, :]
        dz = np.broadcast_to(se, dx.shape)
        with np.errstate(divide="ignore", invalid="ignore"):
            t = np.where(dz < 0, GROUND_Z / dz, np.inf)
        t = np.where(t <= MAX_RANGE, t, np.inf)
        # cylinders: 2D circle along the horizontal direction
        for c in range(len(cyl["cx"])):
            cx, cy, r = cyl["cx"][c], cyl["cy"][c], cyl["r"][c]
            d = math.hypot(cx, cy)
            a = math.atan2(cy, cx) % (2 * math.pi)
            half = math.asin(min(1.0, r / d))
            w = _az_window(n_az, a - half, a + half)
            ux, uy = cos_az[w][None, :], sin_az[w][None, :]
            cu = cx * ux + cy * uy
            disc = cu * cu - (cx * cx + cy * cy - r * r)
            s = cu - np.sqrt(np.maximum(disc, 0.0))
            tt = s / ce
            z = tt * se
            hit = (disc >= 0) & (s > 0) & (z >= cyl["z0"][c]) & (z <= cyl["z1"][c])
            sub = t[:, w]
            t[:, w] = np.where(hit & (tt < sub), tt, sub)
        # boxes: slab method
        for b in range(len(box["x0"])):
            corners = [(box["x0"][b], box["y0"][b]), (box["x1"][b], box["y0"][b]),
                       (box["x0"][b], box["y1"][b]), (box["x1"][b], box["y1"][b])]
            angs = np.array([math.atan2(cy_, cx_) for cx_, cy_ in corners])
            ang0 = angs[0]
            rel = (angs - ang0 + math.pi) % (2 * math.pi) - math.pi
            lo, hi = ang0 + rel.min(), ang0 + rel.max()
            w = _az_window(n_az, lo % (2 * math.pi), (lo % (2 * math.pi)) + (hi - lo))
            bdx, bdy = dx[:, w], dy[:, w]
            bdz = dz[:, w]
            with np.errstate(divide="ignore", invalid="ignore"):
                tx0 = box["x0"][b] / bdx; tx1 = box["x1"][b] / bdx
                ty0 = box["y0"][b] / bdy; ty1 = box["y1"][b] / bdy
                tz0 = box["z0"][b] / bdz; tz1 = box["z1"][b] / bdz
            tmin = np.maximum(np.maximum(np.minimum(tx0, tx1), np.minimum(ty0, ty1)),
                              np.minimum(tz0, tz1))
            tmax = np.minimum(np.minimum(np.maximum(tx0, tx1), np.maximum(ty0, ty1)),
                              np.maximum(tz0, tz1))
            hit = np.isfinite(tmin) & (tmax >= tmin) & (tmin > 0)
            sub = t[:, w]
            t[:, w] = np.where(hit & (tmin < sub), tmin, sub)
        ok = np.isfinite(t) & (t <= MAX_RANGE)
        tk = t[ok]
        out.append(np.stack([tk * dx[ok], tk * dy[ok], tk * dz[ok]], axis=1))
    allp = np.concatenate(out, axis=0)
    if allp.shape[0] < n:
        raise ValueError(f"ray grid gave {allp.shape[0]} hits < {n}")
    keep = rng.permutation(allp.shape[0])[:n]
    return np.ascontiguousarray(allp[keep])


def config2(seed=2, n=20_000_000, nq=2_000_000):
    """TLS-like scan: 20 M points, 2 M query indices; radii 0.1, 0.25, 0.5 m;
    k = 32; sparse and mixed flavors."""
    rng = np.random.default_rng(seed)
    xyz = tls_cloud(rng, n)
    q = rng.choice(n, nq, replace=False).astype(np.int32)
    return dict(xyz=xyz, queries=q, radii=(0.1, 0.25, 0.5), k=32)
