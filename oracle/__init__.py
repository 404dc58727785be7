"""FP64 CPU oracle for the demagnetizing-field path (test infrastructure).

This package is test infrastructure only: the tests, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does.
It shares no code with the HIP implementation.

Contents
  newell.py  cell-averaged demagnetizing tensor N(r) (Sec. 3, Eq. 4 and the
             demagnetizing-field row of Table 1; Newell closed forms near,
             Gauss-Legendre quadrature of the dipole kernel far)
  conv.py    H = -N * M by brute-force direct sum and by zero-padded FP64 FFT
             convolution (Sec. 7), demag energy (Appendix A field/energy
             relation), gradients of the energy and of <G, H>.
  multilayer.py  inter-mesh tensor for unequal cells and the Eq. 4 direct sum
             over a collection of meshes (Sec. 3).
  pbc.py     image-summed tensor for periodic boundaries (Sec. 3, multiple
             images).
  llg.py     a minimal evaluation loop: exchange and applied fields, the LLG
             equation (Sec. 2, Eq. 1), RK4 steps (Sec. 7), the two-sublattice
             demagnetizing input (Sec. 6).
  oersted.py Oersted field of a current density, H = K * J (Table 1,
             Oersted row; Sec. 4): the cell-averaged Biot-Savart kernel, its
             direct sum and its zero-padded FFT convolution.
"""
from .newell import (COMPONENTS, newell_f, newell_g, newell_near, gl_far,
                     tensor_at, tensor_octant, tensor_full)
from .conv import (MU0, padded_len, direct_sum, fft_conv, energy,
                   grad_energy_m, grad_inner_m)
