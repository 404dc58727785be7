"""Periodic boundaries by the multiple-images method.

Test infrastructure: only the tests, the package smoke check and the
benchmark's CPU baseline use this module.

Paper: Sec. 3 extends the convolution to periodic boundary conditions with
the multiple images method (cited, not printed).  Reading taken here: along
each periodic axis a (with period L_a = n_a h_a) the mesh is repeated K times
on either side, and the field is that of the (2K+1)-times repeated mesh read
in its central copy:

    H_i = -sum_j sum_{|k_a| <= K} N(r_i - r_j - k o L) M_j,

i.e. the ordinary convolution sum with the image-summed tensor

    N_K(d) = sum_{|k_a| <= K, periodic a} N(d + k o L)

at every lattice offset d with |d_a| < n_a.  The image set is symmetric, so
N_K keeps the parity of N and everything downstream (zero padding, FFT
convolution, direct sum) applies unchanged.  Summing over the cube of images
makes the fully 3D-periodic case depend on that summation shape
(conditionally convergent sum); 1D and 2D periodicity converge absolutely.
"""
import itertools

import numpy as np

from .newell import COMPONENTS, PARITY, tensor_at

DEFAULT_IMAGES = 10


def image_shifts(n, h, pbc, images):
    """Shift vectors k o L of the image set: k_a in [-K, K] on the periodic
    axes (pbc = (bool, bool, bool)), 0 on the others."""
    rng = [range(-images, images + 1) if p else range(0, 1) for p in pbc]
    L = [n[a] * h[a] for a in range(3)]
    return [(kx * L[0], ky * L[1], kz * L[2]) for kx, ky, kz in itertools.product(*rng)]


def tensor_octant_pbc(n, h, pbc, images=DEFAULT_IMAGES):
    """N_K at the non-negative lattice offsets (i dx, j dy, k dz), i < nx,
    j < ny, k < nz.  Returns [6, nz, ny, nx]."""
    nx, ny, nz = n
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    X, Y, Z = i * h[0], j * h[1], k * h[2]
    out = np.zeros((6, nz, ny, nx))
    shifts = np.asarray(image_shifts(n, h, pbc, images))
    # images in groups of about 2^20 points per evaluation
    per = max(1, (1 << 20) // X.size)
    for g0 in range(0, len(shifts), per):
        sh = shifts[g0:g0 + per]
        Nim = tensor_at(X[None] + sh[:, 0, None, None, None], Y[None] + sh[:, 1, None, None, None],
                        Z[None] + sh[:, 2, None, None, None], h)
        out += Nim.sum(axis=1)
    return out


def tensor_full_pbc(n, h, pbc, images=DEFAULT_IMAGES):
    """N_K at every lattice offset -(n_a - 1) .. (n_a - 1) (zero offset at index
    n_a - 1), from the octant by each component's parity.  Same layout as
    newell.tensor_full, so conv.direct_sum / conv.fft_conv take it as Nfull."""
    nx, ny, nz = n
    octn = tensor_octant_pbc(n, h, pbc, images)
    full = np.zeros((6, 2 * nz - 1, 2 * ny - 1, 2 * nx - 1))
    offs = [np.arange(-(m - 1), m) for m in (nx, ny, nz)]
    for c, name in enumerate(COMPONENTS):
        px, py, pz = PARITY[name]
        vals = octn[c][np.ix_(np.abs(offs[2]), np.abs(offs[1]), np.abs(offs[0]))]
        if px < 0:
            vals = vals * np.where(offs[0] < 0, -1.0, 1.0)[None, None, :]
        if py < 0:
            vals = vals * np.where(offs[1] < 0, -1.0, 1.0)[None, :, None]
        if pz < 0:
            vals = vals * np.where(offs[2] < 0, -1.0, 1.0)[:, None, None]
        full[c] = vals
    return full
