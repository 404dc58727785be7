"""Seeded synthetic magnetization fields and upstream gradients.

These generators only draw inputs; they hold none of the demagnetizing-field
arithmetic.  Every field is drawn in FP64 with numpy's default_rng(seed) and
returned as float32, SoA shape (3, nz, ny, nx), x fastest.  The paper's own
benchmark workload is not published with it, so these stand in for it:
  * uniform unit vectors on the sphere (normalized Gaussian triples),
  * a vortex-like field m = (-y, x, c)/|.| plus Gaussian noise, renormalized,
  * random domains: 3D Voronoi grains of about 50 cells, one random direction
    per grain,
  * Gaussian upstream gradients G for the backward.
"""
import numpy as np


def _normalize(v, rng):
    norm = np.sqrt(np.sum(v * v, axis=0))
    bad = norm == 0
    while bad.any():                       # redraw exact zeros (measure zero)
        v[:, bad] = rng.standard_normal((3, int(bad.sum())))
        norm = np.sqrt(np.sum(v * v, axis=0))
        bad = norm == 0
    return v / norm


def unit_sphere(n, seed):
    """Unit vectors uniform on the sphere, one per cell of an (nx, ny, nz) mesh."""
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((3, nz, ny, nx))
    return _normalize(v, rng).astype(np.float32)


def vortex(n, h_nm, core, seed, noise=0.1):
    """m = (-y, x, core)/|.| with (x, y) the cell centre relative to the mesh
    centre in nanometres, plus noise * N(0, 1) per component, renormalized.
    The same in-plane pattern is used in every z layer."""
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    x = (np.arange(nx) - (nx - 1) / 2.0) * h_nm[0]
    y = (np.arange(ny) - (ny - 1) / 2.0) * h_nm[1]
    Y, X = np.meshgrid(y, x, indexing="ij")
    base = np.stack([-Y, X, np.full_like(X, float(core))])
    base = base / np.sqrt(np.sum(base * base, axis=0))
    v = np.broadcast_to(base[:, None], (3, nz, ny, nx)).copy()
    v += noise * rng.standard_normal(v.shape)
    return _normalize(v, rng).astype(np.float32)


def voronoi(n, h_nm, seed, cells_per_grain=50):
    """Random domains: S = round(cells / cells_per_grain) grain seeds uniform in
    the physical box, each with a random unit direction; every cell takes the
    direction of its nearest seed (Euclidean distance in nm, no wrap)."""
    from scipy.spatial import cKDTree
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    S = max(1, int(round(nx * ny * nz / cells_per_grain)))
    box = np.array([nx * h_nm[0], ny * h_nm[1], nz * h_nm[2]])
    seeds = rng.random((S, 3)) * box
    dirs = _normalize(rng.standard_normal((3, S)), rng)
    tree = cKDTree(seeds)
    z = (np.arange(nz) + 0.5) * h_nm[2]
    y = (np.arange(ny) + 0.5) * h_nm[1]
    x = (np.arange(nx) + 0.5) * h_nm[0]
    out = np.empty((3, nz, ny, nx), dtype=np.float32)
    Y, X = np.meshgrid(y, x, indexing="ij")
    pts_xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    for k in range(nz):                    # one layer at a time keeps memory flat
        pts = np.concatenate([pts_xy, np.full((pts_xy.shape[0], 1), z[k])], axis=1)
        _, idx = tree.query(pts, workers=-1)
        out[:, k] = dirs[:, idx].reshape(3, ny, nx)
    return out


def gaussian(n, seed):
    """Upstream gradient G ~ N(0, 1) per component and cell."""
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    return rng.standard_normal((3, nz, ny, nx)).astype(np.float32)


def uniform(count, lo, hi, seed):
    """`count` values uniform in [lo, hi) (e.g. Ms per mesh)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=count)
