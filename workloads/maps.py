"""Seeded synthetic normal maps.

All height fields are in texel units and periodic on the N x N torus.  A normal
map stores, per texel, the xy components of the unit surface normal (the
"projected hemisphere" coordinates of the paper's Preliminaries section), as a
float32 array of shape (N, N, 2) indexed [j, i, :] with i running along u.

Normals come from central differences with wrap-around, computed in float64 and
stored in float32.
"""
import numpy as np

MAP_KINDS = ("bumps", "powerlaw", "scratched")


def normals_from_height(h):
    """(s, t) = -g / sqrt(1 + |g|^2), g the central-difference gradient (wrapped)."""
    h = np.asarray(h, dtype=np.float64)
    gx = 0.5 * (np.roll(h, -1, axis=1) - np.roll(h, 1, axis=1))
    gy = 0.5 * (np.roll(h, -1, axis=0) - np.roll(h, 1, axis=0))
    inv = 1.0 / np.sqrt(1.0 + gx * gx + gy * gy)
    out = np.empty(h.shape + (2,), dtype=np.float32)
    out[..., 0] = -gx * inv
    out[..., 1] = -gy * inv
    return out


def _rms_slope(h):
    gx = 0.5 * (np.roll(h, -1, axis=1) - np.roll(h, 1, axis=1))
    gy = 0.5 * (np.roll(h, -1, axis=0) - np.roll(h, 1, axis=0))
    return float(np.sqrt(np.mean(gx * gx + gy * gy)))


def bumps_height(n, count, seed, amp=0.5, width=(2.0, 8.0)):
    """Sum of `count` Gaussian bumps of amplitude +-amp (random sign) and standard
    deviation U[width], centred uniformly, using torus distance."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cx = rng.uniform(0.0, n, count)
    cy = rng.uniform(0.0, n, count)
    sg = rng.uniform(width[0], width[1], count)
    sign = np.where(rng.uniform(0.0, 1.0, count) < 0.5, -1.0, 1.0)
    h = np.zeros((n, n), dtype=np.float64)
    coords = np.arange(n, dtype=np.float64)
    for k in range(count):
        # each bump only touches a (10 sigma)^2 window: evaluate there
        rad = int(np.ceil(5.0 * sg[k]))
        if 2 * rad + 1 >= n:
            dx = coords - cx[k]
            dx -= n * np.round(dx / n)
            dy = coords - cy[k]
            dy -= n * np.round(dy / n)
            g = np.exp(-(dy[:, None] ** 2 + dx[None, :] ** 2) / (2 * sg[k] ** 2))
            h += sign[k] * amp * g
            continue
        ix = np.arange(int(np.floor(cx[k])) - rad, int(np.floor(cx[k])) + rad + 2)
        iy = np.arange(int(np.floor(cy[k])) - rad, int(np.floor(cy[k])) + rad + 2)
        dx = ix - cx[k]
        dy = iy - cy[k]
        g = np.exp(-(dy[:, None] ** 2 + dx[None, :] ** 2) / (2 * sg[k] ** 2))
        h[np.ix_(iy % n, ix % n)] += sign[k] * amp * g
    return h


def powerlaw_height(n, seed, rms_slope=0.15, exponent=3.0, f_max=None):
    """Isotropic power-law noise: white complex Gaussian shaped by |f|^(-exponent/2)
    (so the power spectrum falls as f^-exponent), zero mean, optionally low-passed
    at |f| < f_max cycles/texel, scaled so the RMS central-difference slope equals
    `rms_slope`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    fy = np.fft.fftfreq(n)[:, None]
    fx = np.fft.rfftfreq(n)[None, :]
    f = np.sqrt(fx * fx + fy * fy)
    shape = (n, n // 2 + 1)
    spec = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    with np.errstate(divide="ignore"):
        amp = np.where(f > 0, f ** (-0.5 * exponent), 0.0)
    if f_max is not None:
        amp = np.where(f < f_max, amp, 0.0)
    spec *= amp
    del amp, f
    h = np.fft.irfft2(spec, s=(n, n))
    del spec
    s = _rms_slope(h)
    if s > 0:
        h *= rms_slope / s
    return h


def _scratch_carve(n, rng, count, length, width, depth):
    """Minimum over V-shaped scratch profiles (<= 0), rasterised by walking each
    scratch's rectangle at half-texel spacing."""
    carve = np.zeros(n * n, dtype=np.float64)
    cx = rng.uniform(0.0, n, count)
    cy = rng.uniform(0.0, n, count)
    ang = rng.uniform(0.0, np.pi, count)
    ln = rng.uniform(length[0], length[1], count)
    wd = rng.uniform(width[0], width[1], count)
    dp = rng.uniform(depth[0], depth[1], count)
    chunk = 256
    for s0 in range(0, count, chunk):
        sl = slice(s0, min(count, s0 + chunk))
        for k in range(sl.start, sl.stop):
            tdir = np.array([np.cos(ang[k]), np.sin(ang[k])])
            ndir = np.array([-np.sin(ang[k]), np.cos(ang[k])])
            a = np.arange(-0.5 * ln[k] - 1.0, 0.5 * ln[k] + 1.0, 0.5)
            b = np.arange(-0.5 * wd[k] - 1.0, 0.5 * wd[k] + 1.0, 0.5)
            px = cx[k] + a[:, None] * tdir[0] + b[None, :] * ndir[0]
            py = cy[k] + a[:, None] * tdir[1] + b[None, :] * ndir[1]
            ix = np.floor(px + 0.5).astype(np.int64).ravel()
            iy = np.floor(py + 0.5).astype(np.int64).ravel()
            # exact profile at the chosen texel centres
            rx = ix - cx[k]
            ry = iy - cy[k]
            along = rx * tdir[0] + ry * tdir[1]
            perp = np.abs(rx * ndir[0] + ry * ndir[1])
            half = 0.5 * wd[k]
            inside = (np.abs(along) <= 0.5 * ln[k]) & (perp < half)
            if not np.any(inside):
                continue
            prof = -dp[k] * (1.0 - perp[inside] / half)
            flat = (iy[inside] % n) * n + (ix[inside] % n)
            np.minimum.at(carve, flat, prof)
    return carve.reshape(n, n)


def scratched_normals(n, seed, scratches=20000, flakes=50000,
                      base_rms_slope=0.02, base_fmax=1.0 / 32.0,
                      scratch_length=(32.0, 512.0), scratch_width=(1.0, 4.0),
                      scratch_depth=(0.2, 1.0), flake_radius=(2.0, 6.0),
                      flake_sigma=0.1):
    """Scratched metal: low-passed power-law base, V-scratches carved by min, then
    hexagonal flakes whose constant normals override the map (highest flake index
    wins where flakes overlap)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    base_seed = int(rng.integers(0, 2**31 - 1))
    h = powerlaw_height(n, base_seed, rms_slope=base_rms_slope, f_max=base_fmax)
    h += _scratch_carve(n, rng, scratches, scratch_length, scratch_width, scratch_depth)
    nrm = normals_from_height(h)
    del h
    if flakes > 0:
        fcx = rng.uniform(0.0, n, flakes)
        fcy = rng.uniform(0.0, n, flakes)
        frad = rng.uniform(flake_radius[0], flake_radius[1], flakes)
        frot = rng.uniform(0.0, np.pi / 3.0, flakes)
        fn = rng.normal(0.0, flake_sigma, (flakes, 2))
        mag = np.sqrt(np.sum(fn * fn, axis=1))
        fn *= np.where(mag > 0.95, 0.95 / np.maximum(mag, 1e-30), 1.0)[:, None]
        owner = np.full(n * n, -1, dtype=np.int64)
        w = int(np.ceil(flake_radius[1])) + 1
        off = np.arange(-w, w + 1)
        ox, oy = np.meshgrid(off, off)
        ox = ox.ravel()
        oy = oy.ravel()
        apothem_scale = np.sqrt(3.0) / 2.0
        chunk = 4096
        for s0 in range(0, flakes, chunk):
            s1 = min(flakes, s0 + chunk)
            k = np.arange(s0, s1)
            ix = np.floor(fcx[k])[:, None].astype(np.int64) + ox[None, :]
            iy = np.floor(fcy[k])[:, None].astype(np.int64) + oy[None, :]
            rx = ix - fcx[k][:, None]
            ry = iy - fcy[k][:, None]
            inside = np.ones(rx.shape, dtype=bool)
            for m in range(3):
                a = frot[k] + m * np.pi / 3.0
                d = np.abs(rx * np.cos(a)[:, None] + ry * np.sin(a)[:, None])
                inside &= d <= (frad[k] * apothem_scale)[:, None]
            flat = (iy % n) * n + (ix % n)
            ids = np.broadcast_to(k[:, None], flat.shape)
            np.maximum.at(owner, flat[inside], ids[inside])
        sel = owner >= 0
        flat_nrm = nrm.reshape(-1, 2)
        flat_nrm[sel] = fn[owner[sel]].astype(np.float32)
    return nrm


def make_map(kind, n, seed, **kw):
    """Normal map (N, N, 2) float32 for one of MAP_KINDS."""
    if kind == "bumps":
        count = kw.pop("count", max(1, (32 * n * n) // (64 * 64)))
        return normals_from_height(bumps_height(n, count, seed, **kw))
    if kind == "powerlaw":
        return normals_from_height(powerlaw_height(n, seed, **kw))
    if kind == "scratched":
        return scratched_normals(n, seed, **kw)
    raise ValueError(f"unknown map kind {kind!r}")
