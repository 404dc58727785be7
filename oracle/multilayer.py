"""Demagnetizing field of a collection of meshes with independent
discretizations (Sec. 3, Eq. 4): H(r'_kl) = -sum_i sum_{r_ij in V_i}
N(r'_kl - r_ij, h_k, h_i) M(r_ij), with N the inter-mesh tensor between a
target cell of size h_k and a source cell of size h_i.  The paper cites its
generalization of the Newell formulas without printing it; here:

  * closed form: the Newell f/g functions under a 4-point stencil per axis,
    X +- (a + b)/2 with weight -1 and X +- (a - b)/2 with weight +1 (a the
    target size, b the source size along that axis), over 4 pi V_target.  For
    a == b the two inner points coincide and this is the 27-point stencil of
    the equal-cell tensor.
  * far field: the defining integral, N(R) = 1/(4 pi V_target) * integral of
    prod_axes w_ab(u) D(R + u) du, where w_ab (the overlap of a box of width a
    with one of width b) is a trapezoid of base a + b and plateau min(a, b);
    Gauss-Legendre on each linear piece.

Meshes are given as (n, h, origin): n = (nx, ny, nz) cells of size
h = (dx, dy, dz) whose lower corner sits at origin (metres); cell (i, j, k)
has its centre at origin + (i + 1/2, j + 1/2, k + 1/2) * h.  FP64 throughout.
"""
import math

import numpy as np

from .newell import newell_f, newell_g

NEAR_RADIUS = 3.0
GL_BANDS = ((6.0, 8), (16.0, 6), (40.0, 4), (math.inf, 3))


def _stencil4(phi, X, Y, Z, ta, sa, tb, sb, tc, sc):
    """4-point second difference per axis of phi, over 4 pi ta tb tc."""
    pts = []
    for (t, s) in ((ta, sa), (tb, sb), (tc, sc)):
        pts.append(((0.5 * (t + s), -1.0), (-0.5 * (t + s), -1.0), (0.5 * (t - s), 1.0), (-0.5 * (t - s), 1.0)))
    acc = np.zeros(np.broadcast(X, Y, Z).shape)
    for (ox, wx) in pts[0]:
        for (oy, wy) in pts[1]:
            for (oz, wz) in pts[2]:
                acc = acc + wx * wy * wz * phi(X + ox, Y + oy, Z + oz)
    return acc / (4.0 * math.pi * ta * tb * tc)


def near_unequal(X, Y, Z, ht, hs):
    """All six components [6, ...] by the generalized closed form; the
    permutations follow the equal-cell case, each axis keeping its own
    (target, source) sizes."""
    (tx, ty, tz), (sx, sy, sz) = ht, hs
    return np.stack([
        _stencil4(newell_f, X, Y, Z, tx, sx, ty, sy, tz, sz),   # xx
        _stencil4(newell_f, Y, X, Z, ty, sy, tx, sx, tz, sz),   # yy
        _stencil4(newell_f, Z, Y, X, tz, sz, ty, sy, tx, sx),   # zz
        _stencil4(newell_g, X, Y, Z, tx, sx, ty, sy, tz, sz),   # xy
        _stencil4(newell_g, X, Z, Y, tx, sx, tz, sz, ty, sy),   # xz
        _stencil4(newell_g, Y, Z, X, ty, sy, tz, sz, tx, sx),   # yz
    ])


def _trapezoid_nodes(a, b, n):
    """Nodes and weights of int w_ab(u) F(u) du, w_ab the overlap length of
    a box of width a centred at 0 shifted by u with one of width b."""
    lo, hi = 0.5 * abs(a - b), 0.5 * (a + b)
    t, w = np.polynomial.legendre.leggauss(n)
    us, ws = [], []
    # ramps on [lo, hi] and [-hi, -lo]: weight hi - |u|
    u = lo + 0.5 * (hi - lo) * (1.0 + t)
    wt = 0.5 * (hi - lo) * w * (hi - u)
    us += [u, -u]
    ws += [wt, wt]
    if lo > 0:   # plateau of height min(a, b) on [-lo, lo]
        u = lo * t
        us.append(u)
        ws.append(lo * w * min(a, b))
    return np.concatenate(us), np.concatenate(ws)


def far_unequal(X, Y, Z, ht, hs, n):
    X, Y, Z = (np.asarray(v, dtype=np.float64) for v in (X, Y, Z))
    shape = np.broadcast(X, Y, Z).shape
    acc = np.zeros((6,) + shape)
    ux, wx = _trapezoid_nodes(ht[0], hs[0], n)
    uy, wy = _trapezoid_nodes(ht[1], hs[1], n)
    uz, wz = _trapezoid_nodes(ht[2], hs[2], n)
    for a in range(len(ux)):
        vx = X + ux[a]
        for b in range(len(uy)):
            vy = Y + uy[b]
            for c in range(len(uz)):
                vz = Z + uz[c]
                r2 = vx * vx + vy * vy + vz * vz
                wgt = wx[a] * wy[b] * wz[c] / (r2 * r2 * np.sqrt(r2))
                acc[0] += wgt * (r2 - 3.0 * vx * vx)
                acc[1] += wgt * (r2 - 3.0 * vy * vy)
                acc[2] += wgt * (r2 - 3.0 * vz * vz)
                acc[3] += wgt * (-3.0 * vx * vy)
                acc[4] += wgt * (-3.0 * vx * vz)
                acc[5] += wgt * (-3.0 * vy * vz)
    return acc / (4.0 * math.pi * ht[0] * ht[1] * ht[2])


def tensor_unequal(X, Y, Z, ht, hs):
    """N(R; h_target, h_source) at offsets R = target centre - source centre,
    closed form near, quadrature far (distance in units of the largest edge
    of either cell).  Returns [6, ...]."""
    X, Y, Z = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64) for v in (X, Y, Z)))
    hmax = max(max(ht), max(hs))
    dist = np.sqrt(X * X + Y * Y + Z * Z) / hmax
    out = np.zeros((6,) + X.shape)
    near = dist < NEAR_RADIUS
    if near.any():
        out[:, near] = near_unequal(X[near], Y[near], Z[near], ht, hs)
    lo = NEAR_RADIUS
    for hi, nodes in GL_BANDS:
        sel = (dist >= lo) & (dist < hi)
        if sel.any():
            out[:, sel] = far_unequal(X[sel], Y[sel], Z[sel], ht, hs, nodes)
        lo = hi
    return out


def centres(n, h, origin):
    """Cell centres of a mesh, arrays (Z, Y, X) of shape (nz, ny, nx)."""
    nx, ny, nz = n
    z = origin[2] + (np.arange(nz) + 0.5) * h[2]
    y = origin[1] + (np.arange(ny) + 0.5) * h[1]
    x = origin[0] + (np.arange(nx) + 0.5) * h[0]
    return np.meshgrid(z, y, x, indexing="ij")


def field_at(meshes, Ms, targets):
    """H at target cells by the direct sum of Eq. 4 over every source cell of
    every mesh.  meshes: list of (n, h, origin); Ms: list of arrays
    (3, nz, ny, nx) of magnetization (A/m); targets: list of (mesh index,
    (k, j, i)).  Returns [len(targets), 3]."""
    src = [(centres(n, h, o), h, np.asarray(M, np.float64)) for (n, h, o), M in zip(meshes, Ms)]
    out = np.zeros((len(targets), 3))
    for q, (p, (k, j, i)) in enumerate(targets):
        (n_p, h_p, o_p) = meshes[p]
        tz = o_p[2] + (k + 0.5) * h_p[2]
        ty = o_p[1] + (j + 0.5) * h_p[1]
        tx = o_p[0] + (i + 0.5) * h_p[0]
        H = np.zeros(3)
        for (Zc, Yc, Xc), h_s, M in src:
            N = tensor_unequal(tx - Xc, ty - Yc, tz - Zc, h_p, h_s)
            xx, yy, zz, xy, xz, yz = N
            H[0] -= np.sum(xx * M[0] + xy * M[1] + xz * M[2])
            H[1] -= np.sum(xy * M[0] + yy * M[1] + yz * M[2])
            H[2] -= np.sum(xz * M[0] + yz * M[1] + zz * M[2])
        out[q] = H
    return out


def field(meshes, Ms, only=None):
    """H of every cell of every mesh by the direct sum (small meshes only):
    all target cells of mesh p against all source cells of mesh q at once.
    only: indices of the target meshes to evaluate (default: all).
    Returns a list of arrays (3, nz, ny, nx), one per evaluated mesh."""
    res = []
    for p, (n_p, h_p, o_p) in enumerate(meshes):
        if only is not None and p not in only:
            continue
        Zt, Yt, Xt = (a.ravel() for a in centres(n_p, h_p, o_p))
        H = np.zeros((3, Xt.size))
        for (n_q, h_q, o_q), M in zip(meshes, Ms):
            Zs, Ys, Xs = (a.ravel() for a in centres(n_q, h_q, o_q))
            M = np.asarray(M, np.float64).reshape(3, -1)
            N = tensor_unequal(Xt[:, None] - Xs[None, :], Yt[:, None] - Ys[None, :], Zt[:, None] - Zs[None, :],
                               h_p, h_q)
            xx, yy, zz, xy, xz, yz = N
            H[0] -= xx @ M[0] + xy @ M[1] + xz @ M[2]
            H[1] -= xy @ M[0] + yy @ M[1] + yz @ M[2]
            H[2] -= xz @ M[0] + yz @ M[1] + zz @ M[2]
        nx, ny, nz = n_p
        res.append(H.reshape(3, nz, ny, nx))
    return res


def periods(meshes, pbc):
    """Period of a coupled collection along each periodic axis (Sec. 3,
    multiple images): the collection repeats as a whole, so every mesh must
    start at the same coordinate and span the same length along that axis;
    the period is that length.  pbc = (bool, bool, bool).  Returns (Px, Py, Pz),
    0 along open axes."""
    out = []
    for a in range(3):
        if not pbc[a]:
            out.append(0.0)
            continue
        spans = {round(n[a] * h[a] / 1e-15) for n, h, _ in meshes}
        starts = {round(o[a] / 1e-15) for _, _, o in meshes}
        if len(spans) != 1 or len(starts) != 1:
            raise ValueError("periodic axis: every mesh must share its start and its span")
        n, h, _ = meshes[0]
        out.append(n[a] * h[a])
    return tuple(out)


def image_shifts(meshes, pbc, images):
    """Shift vectors k o P of the symmetric image set, |k_a| <= images on the
    periodic axes."""
    P = periods(meshes, pbc)
    rng = [range(-images, images + 1) if pbc[a] else range(0, 1) for a in range(3)]
    return [(i * P[0], j * P[1], k * P[2]) for i in rng[0] for j in rng[1] for k in rng[2]]


def field_periodic(meshes, Ms, pbc, images):
    """Eq. 4 over a coupled collection with periodic axes by multiple images:
    the field of the collection repeated `images` times on either side of
    each periodic axis, read in its central copy,
    H_t = -sum_q sum_j sum_k N(r_t - r_j - k o P, h_p, h_q) M_j.
    Direct sum (small meshes).  Returns a list of arrays (3, nz, ny, nx)."""
    shifts = np.asarray(image_shifts(meshes, pbc, images))
    res = []
    for p, (n_p, h_p, o_p) in enumerate(meshes):
        Zt, Yt, Xt = (a.ravel() for a in centres(n_p, h_p, o_p))
        H = np.zeros((3, Xt.size))
        for (n_q, h_q, o_q), M in zip(meshes, Ms):
            Zs, Ys, Xs = (a.ravel() for a in centres(n_q, h_q, o_q))
            M = np.asarray(M, np.float64).reshape(3, -1)
            dX, dY, dZ = Xt[:, None] - Xs[None, :], Yt[:, None] - Ys[None, :], Zt[:, None] - Zs[None, :]
            # all images of every pair at once, in groups of about 2^20 offsets
            N = np.zeros((6,) + dX.shape)
            per = max(1, (1 << 20) // dX.size)
            for g0 in range(0, len(shifts), per):
                sh = shifts[g0:g0 + per]
                N += tensor_unequal(dX[None] - sh[:, 0, None, None], dY[None] - sh[:, 1, None, None],
                                    dZ[None] - sh[:, 2, None, None], h_p, h_q).sum(axis=1)
            xx, yy, zz, xy, xz, yz = N
            H[0] -= xx @ M[0] + xy @ M[1] + xz @ M[2]
            H[1] -= xy @ M[0] + yy @ M[1] + yz @ M[2]
            H[2] -= xz @ M[0] + yz @ M[1] + zz @ M[2]
        nx, ny, nz = n_p
        res.append(H.reshape(3, nz, ny, nx))
    return res
