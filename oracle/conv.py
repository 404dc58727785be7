"""H = -N * M on a regular finite-difference mesh, two independent routes.

Paper: Table 1, row "Demagnetizing Field": H(r0) = -sum_r N(r - r0) M(r), and
Sec. 3, Eq. 4 for a single mesh.  Sec. 7 evaluates that sum by the
convolution theorem with zero padding to (at least) double the size when the
boundaries are open.  The field/energy relation H = -1/(mu0 Ms) d(eps)/dm of
Appendix A gives, for this quadratic self-energy, the density
eps = -(mu0/2) M.H and the total E = -(mu0/2) V sum_cells M.H.

Arrays are SoA, shape (3, nz, ny, nx) with x fastest; positions are cell
centres r = (i dx, j dy, k dz).  Everything here is FP64.
"""
import math
import os

import numpy as np
import scipy.fft

from .newell import tensor_full

MU0 = 4.0e-7 * math.pi
# FFT threads: the CPUs this process may use, at most 16
_WORKERS = max(1, min(16, len(os.sched_getaffinity(0))))


def fft_workers():
    """Threads the FFT convolution uses."""
    return _WORKERS


def padded_len(n):
    """Smallest power of two >= 2n - 1 (open boundary), 1 for n == 1."""
    if n == 1:
        return 1
    p = 1
    while p < 2 * n - 1:
        p *= 2
    return p


def _as_matrix(N6):
    xx, yy, zz, xy, xz, yz = N6
    return ((xx, xy, xz), (xy, yy, yz), (xz, yz, zz))


def direct_sum(M, h, Nfull=None):
    """Brute force H_t = -sum_s N(r_t - r_s) M_s over every ordered cell pair.

    O(N^2); meant for meshes of at most a few thousand cells."""
    M = np.asarray(M, dtype=np.float64)
    _, nz, ny, nx = M.shape
    if Nfull is None:
        Nfull = tensor_full((nx, ny, nz), h)
    N = _as_matrix(Nfull)
    H = np.zeros_like(M)
    for sz in range(nz):
        for sy in range(ny):
            for sx in range(nx):
                # window of N(r_t - r_s) over all targets t
                win = (slice(nz - 1 - sz, 2 * nz - 1 - sz),
                       slice(ny - 1 - sy, 2 * ny - 1 - sy),
                       slice(nx - 1 - sx, 2 * nx - 1 - sx))
                m = M[:, sz, sy, sx]
                for a in range(3):
                    H[a] -= (N[a][0][win] * m[0] + N[a][1][win] * m[1]
                             + N[a][2][win] * m[2])
    return H


def direct_sum_at(M, h, targets, Noct):
    """H at the listed target cells (tz, ty, tx) by the direct sum over every
    source, H_t = -sum_s N(r_t - r_s) M_s, with N looked up in the octant
    Noct [6, nz, ny, nx] and reflected by each component's parity.
    Returns [len(targets), 3]."""
    from .newell import COMPONENTS, PARITY
    M = np.asarray(M, dtype=np.float64)
    _, nz, ny, nx = M.shape
    out = np.zeros((len(targets), 3))
    for q, (tz, ty, tx) in enumerate(targets):
        oz = tz - np.arange(nz)
        oy = ty - np.arange(ny)
        ox = tx - np.arange(nx)
        az, ay, ax = np.abs(oz), np.abs(oy), np.abs(ox)
        sgn = [np.where(o < 0, -1.0, 1.0) for o in (ox, oy, oz)]
        N = []
        for c, name in enumerate(COMPONENTS):
            v = Noct[c][np.ix_(az, ay, ax)]
            px, py, pz = PARITY[name]
            if px < 0:
                v = v * sgn[0][None, None, :]
            if py < 0:
                v = v * sgn[1][None, :, None]
            if pz < 0:
                v = v * sgn[2][:, None, None]
            N.append(v)
        Nm = _as_matrix(N)
        for a in range(3):
            out[q, a] = -float(np.sum(Nm[a][0] * M[0] + Nm[a][1] * M[1] + Nm[a][2] * M[2]))
    return out


def kernel_grid(n, h, Nfull=None):
    """N placed on the zero-padded periodic grid (6, Nz, Ny, Nx): lattice
    offset o in -(n-1)..(n-1) goes to index o mod N_pad; every other index
    (the unused band n..N_pad-n) is zero."""
    nx, ny, nz = n
    Nx, Ny, Nz = padded_len(nx), padded_len(ny), padded_len(nz)
    if Nfull is None:
        Nfull = tensor_full(n, h)
    grid = np.zeros((6, Nz, Ny, Nx))
    ix = np.arange(-(nx - 1), nx) % Nx
    iy = np.arange(-(ny - 1), ny) % Ny
    iz = np.arange(-(nz - 1), nz) % Nz
    grid[:, iz[:, None, None], iy[None, :, None], ix[None, None, :]] = Nfull
    return grid


def fft_conv(M, h, Nfull=None):
    """H = -N * M by the convolution theorem on the zero-padded grid:
    forward FFT of M and of N, point-wise 3x3 product, inverse FFT, crop."""
    M = np.asarray(M, dtype=np.float64)
    _, nz, ny, nx = M.shape
    shape = (padded_len(nz), padded_len(ny), padded_len(nx))
    Khat = scipy.fft.rfftn(kernel_grid((nx, ny, nz), h, Nfull), s=shape,
                           axes=(1, 2, 3), workers=_WORKERS)
    Mhat = scipy.fft.rfftn(M, s=shape, axes=(1, 2, 3), workers=_WORKERS)
    K = _as_matrix(Khat)
    Hhat = np.stack([-(K[a][0] * Mhat[0] + K[a][1] * Mhat[1] + K[a][2] * Mhat[2])
                     for a in range(3)])
    H = scipy.fft.irfftn(Hhat, s=shape, axes=(1, 2, 3), workers=_WORKERS)
    return np.ascontiguousarray(H[:, :nz, :ny, :nx])


def energy(M, H, h):
    """E = -(mu0/2) V sum_cells M . H  (joules)."""
    V = h[0] * h[1] * h[2]
    return -0.5 * MU0 * V * float(np.sum(np.asarray(M, np.float64) * np.asarray(H, np.float64)))


def grad_energy_m(m, Ms, h, conv=fft_conv):
    """dE/dm for M = Ms m: E is quadratic in M with a symmetric, self-adjoint
    operator, so dE/dM = -mu0 V H[M] and dE/dm = -mu0 V Ms H[Ms m]."""
    V = h[0] * h[1] * h[2]
    M = np.asarray(Ms, np.float64) * np.asarray(m, np.float64)
    return -MU0 * V * np.asarray(Ms, np.float64) * conv(M, h)


def grad_inner_m(m, Ms, G, h, conv=fft_conv):
    """d<G, H[Ms m]>/dm = Ms H[G], since <G, H[M]> = <H[G], M>."""
    return np.asarray(Ms, np.float64) * conv(np.asarray(G, np.float64), h)
