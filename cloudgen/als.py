"""Airborne (ALS-like) synthetic tiles.

Recipe (all lengths in metres, coordinates FP64, XY shifted by a UTM-like
offset so that the FP64 -> FP32 recentring is exercised):

* terrain: sum of four sinusoids of amplitude 2.5 m along random directions
  (|z| <= 10 m), wavelengths uniform in a configurable range;
* buildings: axis-aligned boxes 10-40 m wide, 5-30 m tall standing on the
  terrain height at their centre; pulses inside a footprint return once from
  the roof; extra wall points (about 10 % of the pulse budget) are spread
  uniformly over the four walls;
* vegetation: discs of radius 5-30 m covering about 30 % of the open ground,
  canopy height 5-25 m; a pulse inside a disc gives 1-4 returns, the last on
  the ground and the others uniformly between the ground and the canopy top;
* open ground: one return on the terrain.

Pulses are uniform over the tile; enough are drawn to exceed the point budget
and a seeded subset of exactly ``n`` points is kept, in random order.
"""
import math

import numpy as np

UTM_OFFSET = (5.0e5, 5.4e6)


def terrain_params(rng, lam_lo, lam_hi, nwaves=4, amp=2.5):
    theta = rng.uniform(0.0, 2.0 * math.pi, nwaves)
    lam = rng.uniform(lam_lo, lam_hi, nwaves)
    phi = rng.uniform(0.0, 2.0 * math.pi, nwaves)
    return dict(ux=np.cos(theta), uy=np.sin(theta), lam=lam, phi=phi, amp=amp)


def terrain_height(tp, x, y):
    z = np.zeros(np.broadcast(x, y).shape, dtype=np.float64)
    for m in range(len(tp["lam"])):
        z += tp["amp"] * np.sin(2.0 * math.pi * (tp["ux"][m] * x + tp["uy"][m] * y)
                                / tp["lam"][m] + tp["phi"][m])
    return z


def _bin_table(bx0, by0, bx1, by1, binsz, nbx, nby):
    """Map each bin of a coarse grid to the shapes whose bbox touches it."""
    lists = [[] for _ in range(nbx * nby)]
    for s in range(len(bx0)):
        i0 = max(0, int(bx0[s] // binsz)); i1 = min(nbx - 1, int(bx1[s] // binsz))
        j0 = max(0, int(by0[s] // binsz)); j1 = min(nby - 1, int(by1[s] // binsz))
        for i in range(i0, i1 + 1):
            for j in range(j0, j1 + 1):
                lists[i * nby + j].append(s)
    width = max(1, max(len(l) for l in lists))
    table = np.full((nbx * nby, width), -1, dtype=np.int64)
    for b, l in enumerate(lists):
        table[b, :len(l)] = l
    return table


def _shape_lookup(x, y, ex, ey, bx0, by0, bx1, by1, inside, pick_max=None):
    """Per point, the shape containing it (or -1); if several, the one with the
    largest ``pick_max`` value (or the lowest id)."""
    n = x.shape[0]
    out = np.full(n, -1, dtype=np.int64)
    if len(bx0) == 0:
        return out
    binsz = 64.0
    nbx = max(1, int(math.ceil(ex / binsz))); nby = max(1, int(math.ceil(ey / binsz)))
    table = _bin_table(bx0, by0, bx1, by1, binsz, nbx, nby)
    bi = np.clip((x // binsz).astype(np.int64), 0, nbx - 1)
    bj = np.clip((y // binsz).astype(np.int64), 0, nby - 1)
    b = bi * nby + bj
    best = np.full(n, -np.inf)
    for slot in range(table.shape[1]):
        s = table[b, slot]
        ok = s >= 0
        sid = np.where(ok, s, 0)
        hit = ok & inside(sid, x, y)
        if pick_max is None:
            take = hit & (out < 0)
        else:
            val = pick_max[sid]
            take = hit & (val > best)
            best = np.where(take, val, best)
        out = np.where(take, sid, out)
    return out


def als_cloud(rng, n, ex, ey, lam_lo=50.0, lam_hi=500.0, buildings_per_km2=250.0,
              veg_cover=0.30, wall_frac=0.10, density=None):
    """An ALS-like tile of exactly ``n`` points over ``ex`` x ``ey`` metres.

    Returns (xyz [n,3] float64 absolute coordinates, info dict).
    ``density`` is informational (points per square metre = n / area).
    """
    area = ex * ey
    tp = terrain_params(rng, lam_lo, lam_hi)
    # buildings
    nb = int(round(buildings_per_km2 * area / 1.0e6))
    bw = rng.uniform(10.0, 40.0, nb); bd = rng.uniform(10.0, 40.0, nb)
    bcx = rng.uniform(0.0, ex, nb); bcy = rng.uniform(0.0, ey, nb)
    bh = rng.uniform(5.0, 30.0, nb)
    bbase = terrain_height(tp, bcx, bcy)
    bx0, bx1 = bcx - bw / 2, bcx + bw / 2
    by0, by1 = bcy - bd / 2, bcy + bd / 2
    # vegetation discs: Poisson coverage 1 - exp(-lambda * E[area]) = veg_cover
    mean_r2 = (30.0 ** 3 - 5.0 ** 3) / (3.0 * 25.0)
    nv = int(round(-math.log(1.0 - veg_cover) * area / (math.pi * mean_r2)))
    vr = rng.uniform(5.0, 30.0, nv)
    vcx = rng.uniform(0.0, ex, nv); vcy = rng.uniform(0.0, ey, nv)
    vcan = rng.uniform(5.0, 25.0, nv)

    def in_bldg(s, x, y):
        return (x >= bx0[s]) & (x < bx1[s]) & (y >= by0[s]) & (y < by1[s])

    def in_veg(s, x, y):
        return (x - vcx[s]) ** 2 + (y - vcy[s]) ** 2 < vr[s] ** 2

    chunks = []
    total = 0
    # expected points per pulse ~ 1 + 1.5 * veg share + wall share
    per_pulse = 1.0 + 1.5 * veg_cover * 0.9 + wall_frac
    while total < n:
        npulse = int((n - total) / per_pulse * 1.05) + 1024
        px = rng.uniform(0.0, ex, npulse); py = rng.uniform(0.0, ey, npulse)
        gz = terrain_height(tp, px, py)
        bid = _shape_lookup(px, py, ex, ey, bx0, by0, bx1, by1, in_bldg, pick_max=bh + bbase)
        vid = _shape_lookup(px, py, ex, ey, vcx - vr, vcy - vr, vcx + vr, vcy + vr, in_veg,
                            pick_max=vcan)
        inb = bid >= 0
        inv = (~inb) & (vid >= 0)
        # roof / ground returns (one per pulse: roof if in a building, else ground)
        z0 = np.where(inb, bbase[np.where(inb, bid, 0)] + bh[np.where(inb, bid, 0)], gz)
        pts = [np.stack([px, py, z0], axis=1)]
        # extra (intermediate) returns in vegetation
        nret = rng.integers(1, 5, npulse)
        extra = np.where(inv, nret - 1, 0)
        if extra.sum() > 0:
            rep = np.repeat(np.arange(npulse), extra)
            can = vcan[vid[rep]]
            ez = gz[rep] + rng.uniform(0.0, 1.0, rep.shape[0]) * can
            pts.append(np.stack([px[rep], py[rep], ez], axis=1))
        # wall points
        nw = int(round(wall_frac * npulse))
        if nb > 0 and nw > 0:
            per = 2.0 * (bw + bd)
            wb = rng.choice(nb, nw, p=per / per.sum())
            t = rng.uniform(0.0, 1.0, nw) * per[wb]
            w_, d_ = bw[wb], bd[wb]
            wx = np.where(t < w_, bx0[wb] + t,
                 np.where(t < w_ + d_, bx1[wb],
                 np.where(t < 2 * w_ + d_, bx1[wb] - (t - w_ - d_), bx0[wb])))
            wy = np.where(t < w_, by0[wb],
                 np.where(t < w_ + d_, by0[wb] + (t - w_),
                 np.where(t < 2 * w_ + d_, by1[wb], by1[wb] - (t - 2 * w_ - d_))))
            wz = bbase[wb] + rng.uniform(0.0, 1.0, nw) * bh[wb]
            ok = (wx >= 0) & (wx < ex) & (wy >= 0) & (wy < ey)
            pts.append(np.stack([wx[ok], wy[ok], wz[ok]], axis=1))
        c = np.concatenate(pts, axis=0)
        chunks.append(c)
        total += c.shape[0]
    allp = np.concatenate(chunks, axis=0)
    keep = rng.permutation(allp.shape[0])[:n]
    xyz = allp[keep]
    xyz[:, 0] += UTM_OFFSET[0]
    xyz[:, 1] += UTM_OFFSET[1]
    info = dict(n=n, extent=(ex, ey), buildings=nb, veg_patches=nv,
                density=n / area if density is None else density)
    return np.ascontiguousarray(xyz), info


def config0(seed=0):
    """Tiny ALS-like cloud: 100 000 points over 200 m x 200 m, terrain of four
    sinusoids (wavelength 20-200 m) and 30 % of points lifted 0-20 m; 10 000
    query indices drawn without replacement.  Radius 1 m, k = 16, cell 1 m."""
    rng = np.random.default_rng(seed)
    n = 100_000
    tp = terrain_params(rng, 20.0, 200.0)
    x = rng.uniform(0.0, 200.0, n)
    y = rng.uniform(0.0, 200.0, n)
    z = terrain_height(tp, x, y)
    lift = rng.uniform(0.0, 1.0, n) < 0.30
    z = z + np.where(lift, rng.uniform(0.0, 20.0, n), 0.0)
    xyz = np.stack([x + UTM_OFFSET[0], y + UTM_OFFSET[1], z], axis=1)
    q = rng.choice(n, 10_000, replace=False).astype(np.int32)
    return dict(xyz=np.ascontiguousarray(xyz), queries=q, r=1.0, k=16, cell=1.0)


def config1(seed=1, n=10_000_000, extent=1000.0):
    """Large ALS tile: 10 M points over 1 km x 1 km (about 10 points per square
    metre) with terrain, buildings and multi-return vegetation.  All points are
    queries.  Radii 0.5, 1, 2, 3 m; k = 8, 16, 32."""
    rng = np.random.default_rng(seed)
    xyz, info = als_cloud(rng, n, extent, extent)
    return dict(xyz=xyz, queries=None, radii=(0.5, 1.0, 2.0, 3.0), ks=(8, 16, 32),
                cell=1.0, info=info)


def small_als(seed, n, density=10.0):
    """A smaller tile built exactly like the large ALS tile (same density),
    for parity tests that the CPU oracle finishes in seconds."""
    rng = np.random.default_rng(seed)
    e = math.sqrt(n / density)
    xyz, info = als_cloud(rng, n, e, e, buildings_per_km2=250.0 * max(1.0, 1.0e4 / (e * e)))
    return xyz


def config3_tiles(seed=3, ntiles=256, total=60_000_000, lo=10_000, hi=2_000_000,
                  scale=1.0):
    """Per-tile sizes and densities of the batched workload: sizes log-uniform in
    [1e4, 2e6], rescaled so that they sum to about ``total``; densities
    log-uniform in [2, 20] points per square metre.  ``scale`` shrinks every
    size (for tests).  Tile t's cloud comes from ``tile_cloud(t)``."""
    rng = np.random.default_rng(seed)
    nt = np.exp(rng.uniform(math.log(lo), math.log(hi), ntiles))
    for _ in range(50):
        nt = np.clip(nt * (total / nt.sum()), lo, hi)
    nt = np.maximum(1, np.round(nt * scale)).astype(np.int64)
    dens = np.exp(rng.uniform(math.log(2.0), math.log(20.0), ntiles))

    def tile_cloud(t):
        trng = np.random.default_rng([seed, t])
        e = math.sqrt(nt[t] / dens[t])
        xyz, _ = als_cloud(trng, int(nt[t]), e, e,
                           buildings_per_km2=250.0 * max(1.0, 1.0e4 / (e * e)))
        return xyz

    return nt, dens, tile_cloud


def config4(seed=4, n=1_000_000, nq=250_000, channels=64, side=None):
    """Aggregation workload: an ALS-like cloud (config-0 generator) at about
    50 points per square metre, 64-channel N(0,1) features and query centres
    drawn from the points.  Radius 0.5 m, 64 nearest, sigma 0.25 m."""
    rng = np.random.default_rng(seed)
    if side is None:
        side = math.sqrt(n / 50.0)
    tp = terrain_params(rng, 20.0, 200.0)
    x = rng.uniform(0.0, side, n)
    y = rng.uniform(0.0, side, n)
    z = terrain_height(tp, x, y)
    lift = rng.uniform(0.0, 1.0, n) < 0.30
    z = z + np.where(lift, rng.uniform(0.0, 20.0, n), 0.0)
    xyz = np.ascontiguousarray(np.stack([x + UTM_OFFSET[0], y + UTM_OFFSET[1], z], axis=1))
    f = rng.standard_normal((n, channels)).astype(np.float32)
    q = rng.choice(n, nq, replace=False).astype(np.int32)
    return dict(xyz=xyz, f=f, queries=q, r=0.5, k=64, sigma=0.25)
