"""MI355X-native demagnetizing-field path: H_d = -N * M on a regular
finite-difference mesh by zero-padded FFT convolution with the Newell tensor
(hand-written HIP kernels for gfx950 behind a C ABI)."""
