// Plan geometry and kernel argument blocks shared by the host launcher and the
// HIP kernels of the demagnetizing-field path.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>

namespace demag {

constexpr int TILE = 16;         // kx points per tile of the spectrum work buffer (128-byte rows)
constexpr int FWD_THREADS = 512;
constexpr int INV_THREADS = 512;
constexpr int RED_THREADS = 256;
constexpr int FINAL_THREADS = 1024;   // threads of the single-workgroup final reductions

// Points per lane (R) of an M-point line FFT, and its padded LDS footprint
// (one pad point after every 2^3 points for radix 8, 2^5 for radix 16).
// Kernel spectrum storage for a padded y length Ny: rows K[kz][kx][component][ky]
// of kernel_row_pitch(Ny) floats holding ky < Ny/2 (ky = 0 when Ny = 1; zero
// padding up to the pitch), and the Nyquist entries ky = Ny/2 (Ny >= 4) in a
// side array KN[kz][kx][component] after the rows.  The pitch is a multiple of
// 4 floats, so rows start 16-byte aligned and a block of rows splits evenly
// over the lanes that fetch it.
constexpr int kernel_row_pitch(int Ny) { return Ny >= 8 ? Ny / 2 : 4; }

constexpr int line_radix(int M) { return M >= 1024 ? 16 : (M >= 8 ? 8 : M); }
constexpr int line_pad_shift(int R) { return R >= 16 ? 5 : 3; }
constexpr int line_lds_points(int M) { return M + (M >> line_pad_shift(line_radix(M))); }

// Radices the middle pass may use for its M-point y lines (M = Ny/2): the
// default, plus the alternatives the schedule tuner may pick from for the
// long lines (4 to 64 lanes per line, at most 16 points per lane; radix 8 for
// 1024-point lines spans two wavefronts per line).
constexpr bool mid_radix_ok(int M, int R) {
  if (R == line_radix(M)) return true;
  if (M == 1024) return R == 8;      // 128 lanes per line: two wavefronts, barrier exchanges
  if (M != 256 && M != 512) return false;
  return (R == 4 || R == 8 || R == 16) && M / R <= 64;
}

// Threads of a middle-pass workgroup: two residue jobs per kx line (one for
// unit lengths) of M/R lanes each, KW lines, at least one wavefront.
constexpr int mid_threads_rt(int M, int kw, int R) {
  const int nt = (M > 1 ? 2 : 1) * kw * (M / R);
  return nt < 64 ? 64 : nt;
}

// Schedules offered for the middle pass: a supported radix, and 1024-thread
// workgroups only for radix <= 4 (at 16 wavefronts per workgroup a lane has
// 128 registers, too few for 3 components of 8 or 16 points plus twiddles).
constexpr bool mid_schedule_ok(int M, int kw, int R) {
  return (kw == 2 || kw == 4 || kw == 8) && mid_radix_ok(M, R) && (mid_threads_rt(M, kw, R) <= 512 || R <= 4);
}

// LDS points per row of the x passes for Nx = 2^lnx: the half spectrum
// (Nx/2 + 1 points) and, while the row is transformed, the padded scratch of
// its two Nx/4-point residue FFTs.
constexpr int xrow_pitch_rt(int lnx) {
  if (lnx < 2) return 2;
  const int L = (1 << lnx) / 2, P = L / 2;
  const int sc = 2 * line_lds_points(P);
  return sc > L + 1 ? sc : L + 1;
}

// Sizes of one mesh.  Padded lengths are powers of two >= 2n-1 (1 for n == 1).
struct Geom {
  int nx, ny, nz;
  int Nx, Ny, Nz;
  int lnx, lny, lnz;   // log2 of the padded lengths
  int Kx;              // Nx/2 + 1 (1 when Nx == 1): half spectrum along x
  int Kyh, Kzh;        // Ny/2 + 1, Nz/2 + 1 (1 for unit lengths): stored octant
  int Kyp;             // row pitch of the stored kernel spectrum (kernel_row_pitch)
  int nTiles;          // ceil(Kx / TILE)
  int yg;              // y rows per workgroup in the x passes
  int mid_kw;          // kx lines per workgroup of the middle pass (2, 4 or 8)
  int mid_r;           // points per lane of its y line FFT (0: line_radix)
  int zsep;            // 1: z transformed by separate passes (x passes on the mesh flattened to ny nz rows)
  int yg_sep;          // rows per workgroup of those flattened x passes
  unsigned pbc;        // periodic axes (bit 0 x, 1 y, 2 z): image-summed tensor
  int images;          // images K on either side along each periodic axis
  int kind;            // KERNEL_DEMAG or KERNEL_OERSTED
  double dx, dy, dz;
};

// The convolution kernel of a plan: the demagnetizing tensor (6 real
// spectrum rows per (kz, kx): xx yy zz xy xz yz) or the Oersted kernel (3
// rows: the imaginary parts of the Biot-Savart vector's spectrum, x y z).
enum { KERNEL_DEMAG = 0, KERNEL_OERSTED = 1 };
inline int kernel_comps(const Geom& g) { return g.kind == KERNEL_OERSTED ? 3 : 6; }

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

// Batches: nb meshes of one geometry share the kernel spectrum.  Member b
// reads and writes its vectors at moff[b] floats into the caller's
// concatenated buffers (moff == nullptr: offset 0), uses Ms = ms_mesh[b]
// (ms_mesh == nullptr: the scalar ms), its spectrum slab at b * Tb points and
// its energy partials at b * (partials per member).

// One plane pair (target p, source q) of a coupled group on the padded fine
// in-plane grid: R = (u fx + ox, v fy + oy, oz) for lattice offsets (u, v).
struct PairGeom {
  double ht[3], hs[3];
  double fx, fy, ox, oy, oz;
  int Nx, Ny, Lx, Ly;
  // periodic in-plane axes (multiple images): images on either side along x
  // and y (0: open axis) and the periods (the lattice spans) in metres
  int kx, ky;
  double px, py;
};

// Coupled layers (Sec. 3, Eq. 4): every z plane of every mesh of a group is
// embedded in one fine in-plane lattice (the finest pitch of the group).
// Plane p's cell (i, j) sits at fine (ox + i sx, oy + j sy); its true centre is
// offset by (dxo, dyo) from that lattice point (coarser cells), which the
// pair kernels carry.
constexpr int MAXP = 8;
struct PlaneInfo {
  long long moff;      // float offset of the owning mesh in the batch vectors
  int nx, ny, nz, k;   // owning mesh dims and this plane's z index
  int sx, sy, ox, oy;  // embedding strides and offsets on the fine lattice
  int gid;             // global mesh index (Ms, energy, gE)
  float vol;           // cell volume of the owning mesh (m^3)
};

struct LayerArgs {
  const PlaneInfo* pl;         // device table of P planes
  int P, Ly, nTiles, Kx;
  const float* m; float* H; float2* T; const float2* tw;
  const float* ms_mesh; float ms;
  int backward;                // input times 1/V, output times Ms V (adjoint)
  int accumulate;
  const float* aux; const double* beta_ptr; double beta_scale;
};

struct CoupleArgs {
  float2* S;                   // S[c][p][kx][ky]
  const float* K;              // pair spectra, pair after pair (p <= q): [component][kx][ky]
  const PlaneInfo* pl;
  int Kx, NY, Nx;
  double* epart;               // per workgroup and plane, or nullptr
  // bit i set: pair i has no in-plane centre offset, so each component of its
  // spectrum is purely real (xx yy zz xy) or purely imaginary (xz yz) and is
  // stored as one float per frequency; other pairs store complex values
  unsigned long long parity_pairs;
};

struct FwdArgs {
  const float* m; const float* Ms; float ms;
  float2* T; const float2* tw;
  int nx, ny, nz, nTiles, Kx, yg;
  int nb; const long long* moff; const float* ms_mesh; size_t Tb; const int* gid;
  // second sublattice (nullptr: none): the input is (ms m + ms2 m2) / 2
  const float* m2; float ms2;
  // flattened x pass of a plan with separate z passes (0: off): row y' of the
  // (nx, ny nz, 1) mesh is spectrum plane z = y' / ysplit, row y' % ysplit, of
  // nzp planes per component
  int ysplit; int nzp;
};

struct MidArgs {
  float2* T; const float* K; const float2* tw;  // K: rows of pitch kernel_row_pitch(Ny), then KN
  double* epart;               // one partial per workgroup, or nullptr
  int ny, Nz, Nx, nTiles, Kx, Kyh, Kzh, kw_halves;
  int nb; size_t Tb; int nblk1; // workgroups per member
  float2* S;                    // full y spectra [c][plane][kx][ky] (split y passes)
};

struct InvArgs {
  const float2* T; float* H; const float2* tw;
  int nx, ny, nz, nTiles, Kx, yg;
  int accumulate;
  // optional epilogue for the backward: out = s * (conv + beta * aux), with
  // s = per-cell Ms (or the scalar) and beta = beta_scale * beta_ptr[member]
  const float* aux; const double* beta_ptr; double beta_scale; const float* Ms; float ms; int scale_out;
  int nb; const long long* moff; const float* ms_mesh; size_t Tb; const int* gid;
  int ysplit; int nzp;         // as in FwdArgs
};

// Separate z passes (k_zpass.hip): in place on the spectrum T of nb members.
struct ZArgs {
  float2* T; const float2* tw;
  int ny, nz, nTiles;
  int nb; size_t Tb;
};

// One RK4 stage of the LLG evaluation loop (k_llg.hip).
struct LlgArgs {
  const float* m0;     // state at the start of the step
  const float* mi;     // stage input
  const float* Hd;     // demagnetizing field of the stage input
  float* acc;          // running sum of the stage slopes
  float* next;         // next stage input (stages 0..2)
  float* mout;         // new state (stage 3; may alias m0)
  int nx, ny, nz;
  unsigned pbc;        // periodic axes of the exchange Laplacian
  float ihx2, ihy2, ihz2;
  float cex;           // 2 A / (mu0 Ms)
  float hx, hy, hz;    // applied field (A/m)
  float gp;            // gamma / (1 + alpha^2)
  float alpha, dt;
  int stage;
};

}  // namespace demag
