"""Oersted field of a current density on the mesh: H = K * J.

Test infrastructure only (like the rest of this package).

Paper: Table 1, row "Oersted" (H(r0) = sum_r K(r - r0) J_C(r), a convolution
sum with an Oersted tensor) and the Sec. 4 passage on computing it from the
transport solver's current density; the tensor formulas are in a reference
the paper cites but does not print.  The kernel here is written from the
definition (the reading is recorded with the design notes): K is the field of
a cuboid cell carrying a uniform unit current density, averaged over the
target cell, from the Biot-Savart law

    H(r0) = 1/(4 pi) sum_s J_s x g(r0 - r_s),
    g(d)  = 1/V  int_{target at d} int_{source at 0} (r - r') / |r - r'|^3 dV' dV,

so K(r_s - r0) J = 1/(4 pi) J x g(r0 - r_s), an antisymmetric 3x3 matrix per
offset built from the vector g.  g_a is odd along axis a and even along the
other two; g(0) = 0.

Numerics:
  * |d| < 3 h_max: (r - r')_x / |r - r'|^3 = d/dx' (1/|r - r'|), so the six
    integrals reduce to second differences over the 27 points
    (X + i a, Y + j b, Z + k c) of a function Q with
    d/dX d^2/dY^2 d^2/dZ^2 Q = 1/R:
        g_x = -(1/V) sum w_i w_j w_k Q(X + i a, Y + j b, Z + k c),
    w_0 = -2, w_{+-1} = 1.  Newell's f satisfies d^2/dY^2 d^2/dZ^2 f = 1/R
    exactly, so Q(X, Y, Z) = int_0^X f(s, Y, Z) ds, taken by Gauss-Legendre
    quadrature on panels halving towards s = 0 (f is even in s and its only
    non-analytic point on the path is s = 0).
  * |d| >= 3 h_max: the defining integral against the tent weight
    prod_a (h_a - |u_a|) (the overlap of two cells displaced by u),
    g(d) = 1/V int T(u) (d + u) / |d + u|^3 du, by Gauss-Legendre on each
    half-axis with the same node counts by distance as the demagnetizing
    tensor.
"""
import math

import numpy as np
import scipy.fft

from .conv import _WORKERS, padded_len
from .newell import GL_BANDS, NEAR_RADIUS, newell_f

# parity of g_a under r_b -> -r_b (b = x, y, z): odd along its own axis only
PARITY = ((-1, 1, 1), (1, -1, 1), (1, 1, -1))

Q_PANELS = 24        # panels [X 2^-(p+1), X 2^-p], p < Q_PANELS, plus [0, X 2^-Q_PANELS]
Q_NODES = 20         # Gauss-Legendre nodes per panel


def _q_rule():
    t, w = np.polynomial.legendre.leggauss(Q_NODES)
    nodes, weights = [], []
    for p in range(Q_PANELS + 1):
        hi = 2.0 ** -p
        lo = 0.0 if p == Q_PANELS else hi / 2.0
        nodes.append(lo + (hi - lo) * 0.5 * (1.0 + t))
        weights.append((hi - lo) * 0.5 * w)
    return np.concatenate(nodes), np.concatenate(weights)


_QS, _QW = _q_rule()


def q_integral(X, Y, Z):
    """Q(X, Y, Z) = int_0^X f(s, Y, Z) ds with Newell's f (vectorized, FP64).
    Odd in X (f is even in s), even in Y and Z."""
    X, Y, Z = np.broadcast_arrays(*(np.asarray(a, dtype=np.float64) for a in (X, Y, Z)))
    ax = np.abs(X)[..., None]
    vals = newell_f(ax * _QS, Y[..., None], Z[..., None])
    return np.sign(X) * np.abs(X) * np.sum(vals * _QW, axis=-1)


def _stencil_q(X, Y, Z, a, b, c):
    """-(1/(a b c)) times the 27-point second difference of Q, weights
    (1, -2, 1) per axis: the target-averaged integral for the component
    along the first argument."""
    w = {-1: 1.0, 0: -2.0, 1: 1.0}
    acc = np.zeros(np.broadcast(X, Y, Z).shape)
    for i in (-1, 0, 1):
        for j in (-1, 0, 1):
            for k in (-1, 0, 1):
                acc = acc + w[i] * w[j] * w[k] * q_integral(X + i * a, Y + j * b, Z + k * c)
    return -acc / (a * b * c)


def g_near(X, Y, Z, h):
    """g at offsets (X, Y, Z) by the closed reduction; returns [3, ...]."""
    dx, dy, dz = h
    return np.stack([
        _stencil_q(X, Y, Z, dx, dy, dz),
        _stencil_q(Y, X, Z, dy, dx, dz),
        _stencil_q(Z, X, Y, dz, dx, dy),
    ])


def _tent_nodes(hi, n):
    t, w = np.polynomial.legendre.leggauss(n)
    u = 0.5 * hi * (1.0 + t)
    wt = 0.5 * hi * w * (hi - u)
    return np.concatenate([u, -u]), np.concatenate([wt, wt])


def g_far(X, Y, Z, h, n):
    """g from the defining tent-weighted integral with n Gauss-Legendre nodes
    per half-axis (accurate away from the source cell); returns [3, ...]."""
    X, Y, Z = (np.asarray(a, dtype=np.float64) for a in (X, Y, Z))
    acc = np.zeros((3,) + np.broadcast(X, Y, Z).shape)
    ux, wx = _tent_nodes(h[0], n)
    uy, wy = _tent_nodes(h[1], n)
    uz, wz = _tent_nodes(h[2], n)
    for a in range(len(ux)):
        vx = X + ux[a]
        for b in range(len(uy)):
            vy = Y + uy[b]
            for c in range(len(uz)):
                vz = Z + uz[c]
                r2 = vx * vx + vy * vy + vz * vz
                wgt = wx[a] * wy[b] * wz[c] / (r2 * np.sqrt(r2))
                acc[0] += wgt * vx
                acc[1] += wgt * vy
                acc[2] += wgt * vz
    return acc / (h[0] * h[1] * h[2])


def g_at(X, Y, Z, h):
    """g at offsets (X, Y, Z) (metres, any sign, any value): the reduction
    near the source, quadrature beyond.  Returns [3, ...]."""
    X, Y, Z = np.broadcast_arrays(*(np.asarray(a, dtype=np.float64) for a in (X, Y, Z)))
    dist = np.sqrt(X * X + Y * Y + Z * Z) / max(h)
    out = np.zeros((3,) + X.shape)
    near = dist < NEAR_RADIUS
    if near.any():
        out[:, near] = g_near(X[near], Y[near], Z[near], h)
    lo = NEAR_RADIUS
    for hi, nodes in GL_BANDS:
        sel = (dist >= lo) & (dist < hi)
        if sel.any():
            out[:, sel] = g_far(X[sel], Y[sel], Z[sel], h, nodes)
        lo = hi
    return out


def g_octant(n, h, pbc=(False, False, False), images=0):
    """g at the non-negative lattice offsets; [3, nz, ny, nx].  With periodic
    axes (multiple images, Sec. 3, the reading taken for the demagnetizing
    tensor): the sum of g over the shifts k o L, |k_a| <= images on the
    periodic axes, L_a = n_a h_a, i.e. the field of the (2K+1)-times repeated
    mesh read in its central copy.  The image set is symmetric, so the sum
    keeps g's parities."""
    from .pbc import image_shifts
    nx, ny, nz = n
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    X, Y, Z = i * h[0], j * h[1], k * h[2]
    out = np.zeros((3, nz, ny, nx))
    for sx, sy, sz in image_shifts(n, h, pbc, images if any(pbc) else 0):
        out += g_at(X + sx, Y + sy, Z + sz, h)
    return out


def g_full(n, h, pbc=(False, False, False), images=0):
    """g at every lattice offset -(n_a - 1) .. (n_a - 1) from the octant and
    the parities; [3, 2nz-1, 2ny-1, 2nx-1], zero offset at (nz-1, ny-1, nx-1)."""
    nx, ny, nz = n
    octn = g_octant(n, h, pbc, images)
    idx = [np.arange(-(m - 1), m) for m in (nx, ny, nz)]
    full = np.zeros((3, 2 * nz - 1, 2 * ny - 1, 2 * nx - 1))
    for c in range(3):
        vals = octn[c][np.ix_(np.abs(idx[2]), np.abs(idx[1]), np.abs(idx[0]))]
        px, py, pz = PARITY[c]
        s = np.ones(vals.shape)
        if px < 0:
            s = s * np.where(idx[0] < 0, -1.0, 1.0)[None, None, :]
        if py < 0:
            s = s * np.where(idx[1] < 0, -1.0, 1.0)[None, :, None]
        if pz < 0:
            s = s * np.where(idx[2] < 0, -1.0, 1.0)[:, None, None]
        full[c] = vals * s
    return full


def field_direct(J, h, gfull=None):
    """H_t = 1/(4 pi) sum_s J_s x g(r_t - r_s) over every cell pair (A/m for
    J in A/m^2 and h in metres).  O(N^2): tiny meshes only."""
    J = np.asarray(J, dtype=np.float64)
    _, nz, ny, nx = J.shape
    if gfull is None:
        gfull = g_full((nx, ny, nz), h)
    H = np.zeros_like(J)
    for sz in range(nz):
        for sy in range(ny):
            for sx in range(nx):
                win = (slice(nz - 1 - sz, 2 * nz - 1 - sz),
                       slice(ny - 1 - sy, 2 * ny - 1 - sy),
                       slice(nx - 1 - sx, 2 * nx - 1 - sx))
                j = J[:, sz, sy, sx]
                g = [gfull[c][win] for c in range(3)]
                H[0] += j[1] * g[2] - j[2] * g[1]
                H[1] += j[2] * g[0] - j[0] * g[2]
                H[2] += j[0] * g[1] - j[1] * g[0]
    return H / (4.0 * math.pi)


def field_fft(J, h, gfull=None):
    """The same sum by the convolution theorem on the zero-padded grid:
    H^ = 1/(4 pi) J^ x g^ point-wise."""
    J = np.asarray(J, dtype=np.float64)
    _, nz, ny, nx = J.shape
    Nz, Ny, Nx = padded_len(nz), padded_len(ny), padded_len(nx)
    if gfull is None:
        gfull = g_full((nx, ny, nz), h)
    grid = np.zeros((3, Nz, Ny, Nx))
    ix = np.arange(-(nx - 1), nx) % Nx
    iy = np.arange(-(ny - 1), ny) % Ny
    iz = np.arange(-(nz - 1), nz) % Nz
    grid[:, iz[:, None, None], iy[None, :, None], ix[None, None, :]] = gfull
    shape = (Nz, Ny, Nx)
    G = scipy.fft.rfftn(grid, s=shape, axes=(1, 2, 3), workers=_WORKERS)
    Jh = scipy.fft.rfftn(J, s=shape, axes=(1, 2, 3), workers=_WORKERS)
    Hh = np.stack([Jh[1] * G[2] - Jh[2] * G[1],
                   Jh[2] * G[0] - Jh[0] * G[2],
                   Jh[0] * G[1] - Jh[1] * G[0]]) / (4.0 * math.pi)
    H = scipy.fft.irfftn(Hh, s=shape, axes=(1, 2, 3), workers=_WORKERS)
    return np.ascontiguousarray(H[:, :nz, :ny, :nx])
