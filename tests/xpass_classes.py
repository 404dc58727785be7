"""Representative meshes of every compile-time class of the x passes.

The x passes are instantiated per (log2 Nx, log2 Nz) of the padded lengths
(Sec. 7: zero padding to double size along open axes).  One mesh per class:
nx in the middle of the class (ragged), the smallest nz of the class (if the
library accepts any nz of the class, it accepts that one), a few y rows."""

LNX = (0, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12)
LNZ = (0, 2, 3, 4, 5, 6, 7)


def _n_of(l):
    """A cell count whose padded length (next power of two >= 2n - 1) is 2^l."""
    if l == 0:
        return 1
    if l == 2:
        return 2
    lo = (1 << (l - 2)) + 1          # smallest n with padded length 2^l
    hi = 1 << (l - 1)                # largest
    return (lo + hi) // 2 if l > 3 else lo


def _nz_of(l):
    if l == 0:
        return 1
    if l == 2:
        return 2
    return (1 << (l - 2)) + 1


def representatives(ny=3):
    """[((lnx, lnz), (nx, ny, nz)), ...] over every class."""
    return [((a, b), (_n_of(a), ny, _nz_of(b))) for a in LNX for b in LNZ]


def padded(n):
    if n == 1:
        return 1
    p = 1
    while p < 2 * n - 1:
        p *= 2
    return p
