// Plan geometry and kernel argument blocks shared by the host launcher and the
// HIP kernels of the demagnetizing-field path.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>

namespace demag {

constexpr int TILE = 8;          // kx points per tile of the spectrum work buffer
constexpr int FWD_THREADS = 256;
constexpr int INV_THREADS = 256;
constexpr int RED_THREADS = 256;

// Sizes of one mesh.  Padded lengths are powers of two >= 2n-1 (1 for n == 1).
struct Geom {
  int nx, ny, nz;
  int Nx, Ny, Nz;
  int lnx, lny, lnz;   // log2 of the padded lengths
  int Kx;              // Nx/2 + 1 (1 when Nx == 1): half spectrum along x
  int Kyh, Kzh;        // Ny/2 + 1, Nz/2 + 1 (1 for unit lengths): stored octant
  int nTiles;          // ceil(Kx / TILE)
  int yg;              // y rows per workgroup in the x passes
  double dx, dy, dz;
};

// Work buffer layout: spectrum T[c][kz][tile][y][TILE] (float2), then the
// FP64 energy partials.
inline size_t spectrum_elems(const Geom& g) {
  return (size_t)3 * g.Nz * g.nTiles * g.ny * TILE;
}

// Gauss-Legendre nodes and weights on [0, 1] for the far-field quadrature of
// the tensor, one row per distance band (orders 8, 6, 4, 3).
struct GLTable {
  double u[4][8];
  double w[4][8];
  int n[4];
};

struct FwdArgs {
  const float* m; const float* Ms; float ms;
  float2* T; const float2* tw;
  int nx, ny, nz, nTiles, Kx, yg;
};

struct MidArgs {
  float2* T; const float* K; const float2* tw;
  double* epart;               // one partial per workgroup, or nullptr
  int ny, Nz, Nx, nTiles, Kx, Kyh, Kzh, kw_halves;
};

struct InvArgs {
  const float2* T; float* H; const float2* tw;
  int nx, ny, nz, nTiles, Kx, yg;
  int accumulate;
  // optional epilogue for the backward: out = s * (conv + beta * aux), with
  // s = per-cell Ms (or the scalar) and beta = *beta_ptr (device scalar)
  const float* aux; const double* beta_ptr; double beta_scale; const float* Ms; float ms; int scale_out;
};

}  // namespace demag
