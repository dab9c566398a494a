"""Seeded query batches and the named workload configurations.

A query is six float32 values (x, y, sx, sy, hx, hy): footprint centre in texel
units on the torus, Gaussian footprint standard deviations per axis, and the
query normal on the projected hemisphere.
"""
import numpy as np

QUERY_FIELDS = ("x", "y", "sx", "sy", "hx", "hy")


def uniform_queries(n, count, seed, sigma, radius, anisotropic=False):
    """x uniform on [0, n)^2; h uniform in the disk |h| < radius; sigma either a
    constant or a (lo, hi) pair drawn log-uniformly (isotropic unless asked)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    q = np.empty((count, 6), dtype=np.float32)
    q[:, 0] = rng.uniform(0.0, n, count)
    q[:, 1] = rng.uniform(0.0, n, count)
    if np.isscalar(sigma):
        sx = np.full(count, float(sigma))
        sy = sx
    else:
        lo, hi = float(sigma[0]), float(sigma[1])
        sx = np.exp(rng.uniform(np.log(lo), np.log(hi), count))
        sy = np.exp(rng.uniform(np.log(lo), np.log(hi), count)) if anisotropic else sx
    q[:, 2] = sx
    q[:, 3] = sy
    rad = radius * np.sqrt(rng.uniform(0.0, 1.0, count))
    phi = rng.uniform(0.0, 2.0 * np.pi, count)
    q[:, 4] = rad * np.cos(phi)
    q[:, 5] = rad * np.sin(phi)
    return q


def tile_request(n, seed, tile=64, spp=4, sigma_range=(0.5, 4096.0),
                 max_view_deg=80.0):
    """One render-tile request: tile x tile pixels x spp samples on a plane seen at
    a view angle theta ~ U[0, max_view_deg] (tilt along u).  Footprints come from
    synthetic ray differentials: sigma_y = s0, sigma_x = s0 / cos(theta), with s0
    log-uniform in sigma_range and both clipped to it.  The query normal is the xy
    of the half vector between the view direction and a light direction drawn
    uniformly on the hemisphere per sample."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi = sigma_range
    theta = np.deg2rad(rng.uniform(0.0, max_view_deg))
    s0 = float(np.exp(rng.uniform(np.log(lo), np.log(hi))))
    sx = float(np.clip(s0 / np.cos(theta), lo, hi))
    sy = float(np.clip(s0, lo, hi))
    ox = rng.uniform(0.0, n)
    oy = rng.uniform(0.0, n)
    count = tile * tile * spp
    px = np.repeat(np.arange(tile * tile) % tile, spp).astype(np.float64)
    py = np.repeat(np.arange(tile * tile) // tile, spp).astype(np.float64)
    jx = rng.uniform(0.0, 1.0, count)
    jy = rng.uniform(0.0, 1.0, count)
    x = np.mod(ox + (px + jx) * sx, n)
    y = np.mod(oy + (py + jy) * sy, n)
    wo = np.array([np.sin(theta), 0.0, np.cos(theta)])
    # uniform hemisphere directions
    z = rng.uniform(0.0, 1.0, count)
    phi = rng.uniform(0.0, 2.0 * np.pi, count)
    rr = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    wi = np.stack([rr * np.cos(phi), rr * np.sin(phi), z], axis=1)
    hv = wi + wo[None, :]
    hv /= np.linalg.norm(hv, axis=1, keepdims=True)
    q = np.empty((count, 6), dtype=np.float32)
    q[:, 0] = x
    q[:, 1] = y
    q[:, 2] = sx
    q[:, 3] = sy
    q[:, 4] = hv[:, 0]
    q[:, 5] = hv[:, 1]
    return q


# Named workloads: map recipe + query recipe.  Sizes and distributions follow the
# synthetic stand-ins for the paper's isotropic / scratch / flake maps.
CONFIGS = {
    "bumps64": dict(map=dict(kind="bumps", n=64, seed=101, count=32),
                    queries=dict(count=4096, seed=102, sigma=2.0, radius=0.3),
                    tau=0.0),
    "powerlaw2048": dict(map=dict(kind="powerlaw", n=2048, seed=201, rms_slope=0.15),
                         queries=dict(count=1 << 20, seed=202, sigma=(1.0, 64.0), radius=0.4),
                         tau=0.0),
    "scratched4096": dict(map=dict(kind="scratched", n=4096, seed=301),
                          queries=dict(count=4 << 20, seed=302, sigma=(4.0, 1024.0), radius=0.4),
                          tau=1e-4),
    "powerlaw8192": dict(map=dict(kind="powerlaw", n=8192, seed=501, rms_slope=0.15),
                         queries=dict(count=16 << 20, seed=502, sigma=(1.0, 8192.0), radius=0.6),
                         tau=1e-3),
}
