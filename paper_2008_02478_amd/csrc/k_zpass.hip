// Separate z transforms of the spectrum, for meshes whose z lines are too long
// to be transformed inside the x passes (Sec. 7: the pipelined form, z
// transform fused with its neighbours, pays up to 2^4 cells along z; beyond,
// the z transform runs as passes of its own).
//
// The x passes then run on the mesh flattened to (nx, ny nz, 1) rows and read
// or write the spectrum planes z < nz of T[c][kz][tile][y][16] directly.  The
// z passes work in place on T: one workgroup owns one (member, component,
// tile, y) block of 16 kx columns through all planes, so no other workgroup
// touches its elements.
//
//   k_zpass<LNZ, false>: X(kz) = sum_{z < nz} x(z) W_Nz^(z kz), all Nz planes
//   k_zpass<LNZ, true> : x(z) = sum_kz X(kz) W_Nz^(-z kz), planes z < nz
//
// A padded z line has at most Nz/2 non-zero inputs (forward) or needed outputs
// (inverse), so each line splits into its even and odd kz residues: M = Nz/2
// point FFTs of x(z) and of x(z) W_Nz^z (forward); the inverse is the sum of
// the two residue inverses, the odd one times W_Nz^(-z).  Both unnormalized.
#include "fft_core.hpp"
#include "plan.hpp"
#include "xrows.hpp"

namespace demag {

// points per lane of the M-point residue lines of the z passes
constexpr int zline_radix(int M) { return M <= 8 ? M : (M <= 128 ? 8 : 16); }
constexpr int zpass_threads(int lnz) {
  const int M = (1 << lnz) / 2;
  const int n = 32 * (M / zline_radix(M));   // 16 columns x 2 residues
  return n < 64 ? 64 : n;
}
// LDS points of one z-pass workgroup (after the two twiddle tables): the
// largest of the forward and inverse stagings and the 32 lines' FFT scratch
template <int M, int R>
constexpr int zpass_region_points() {
  const int fin = 16 * (M + 1), scr = 32 * lds_points<M, R>(), fout = 2 * M * 17, iin = 32 * (M + 1);
  int m = fin > scr ? fin : scr;
  m = m > fout ? m : fout;
  return m > iin ? m : iin;
}
template <int M>
constexpr int zpass_rtab_points() { return ((M + 31) / 32) * 32; }

template <int LNZ, bool INV>
__global__ void __launch_bounds__(zpass_threads(LNZ)) k_zpass(ZArgs a) {
  constexpr int NZ = 1 << LNZ;
  constexpr int M = NZ / 2;
  constexpr int R = zline_radix(M);
  constexpr int T = M / R;
  constexpr int NT = 32 * T;
  constexpr int NTH = zpass_threads(LNZ);
  constexpr int SP = M + 1;                 // staging pitch of one line (odd)
  extern __shared__ float2 smem_base[];
  float2* const tab = smem_base;
  float2* const rtab = tab + tab_points<M, R>();
  float2* const reg = rtab + zpass_rtab_points<M>();

  const int per_member = 3 * a.nTiles * a.ny;
  const int lg = xcd_logical(blockIdx.x, gridDim.x);
  const int b = lg / per_member;
  int rem = lg - b * per_member;
  const int c = rem / (a.nTiles * a.ny);
  rem -= c * a.nTiles * a.ny;
  const int tile = rem / a.ny;
  const int y = rem - tile * a.ny;
  const size_t plane = (size_t)a.nTiles * a.ny * TILE;
  float2* const col = a.T + (size_t)b * a.Tb + (size_t)c * NZ * plane + ((size_t)tile * a.ny + y) * TILE;
  const int nz = a.nz;

  const int tid = threadIdx.x;
  const bool act = tid < NT;
  const int gi = act ? tid / T : 0;         // line: column kxl, residue r (idle lanes shadow line 0)
  const int t = tid % T;
  const int kxl = gi & 15, r = gi >> 4;
  float2* const scr = reg + gi * lds_points<M, R>();

  if constexpr (M > R) fill_stage_table<M, R>(tab, a.tw, tid, NTH);
  fill_residue_table<M>(rtab, a.tw, tid, NTH);

  float2 v[R];
  if constexpr (!INV) {
    // planes z < nz of the 16 columns into LDS, column-major, zeros up to M
    for (int e = tid; e < 16 * M; e += NTH) {
      const int z = e >> 4, k = e & 15;
      reg[k * SP + z] = z < nz ? col[(size_t)z * plane + k] : make_float2(0.f, 0.f);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < R; ++j) v[j] = reg[kxl * SP + t + T * j];
    if (r) residue_twiddle_tab<R, T, false>(v, rtab, t);
    __syncthreads();                        // staging read before the scratch (same region) is written
    if (act) group_fft<M, R, false>(v, scr, t, tab);
    __syncthreads();                        // every line done with its scratch
    // X(kz), kz = 2 (t + T j) + r, to LDS as rows of 16 columns (pitch 17)
    if (act) {
#pragma unroll
      for (int j = 0; j < R; ++j) reg[(2 * (t + T * j) + r) * 17 + kxl] = v[j];
    }
    __syncthreads();
    for (int e = tid; e < 16 * NZ; e += NTH) {
      const int kz = e >> 4, k = e & 15;
      col[(size_t)kz * plane + k] = reg[kz * 17 + k];
    }
  } else {
    // all Nz planes into LDS, each line's residue contiguous: line (k, r)
    // holds X(2 k' + r) at k'
    for (int e = tid; e < 16 * NZ; e += NTH) {
      const int kz = e >> 4, k = e & 15;
      reg[(2 * k + (kz & 1)) * SP + (kz >> 1)] = col[(size_t)kz * plane + k];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < R; ++j) v[j] = reg[(2 * kxl + r) * SP + t + T * j];
    __syncthreads();
    if (act) {
      group_fft<M, R, true>(v, scr, t, tab);
      if (r) residue_twiddle_tab<R, T, true>(v, rtab, t);
    }
    __syncthreads();
    // x(z) = even-residue inverse + odd-residue inverse, z = t + T j < nz
    if (act && r == 1) {
#pragma unroll
      for (int j = 0; j < R; ++j) reg[(t + T * j) * 17 + kxl] = v[j];
    }
    __syncthreads();
    if (act && r == 0) {
#pragma unroll
      for (int j = 0; j < R; ++j) {
        float2* const d = reg + (t + T * j) * 17 + kxl;
        *d = cadd(*d, v[j]);
      }
    }
    __syncthreads();
    for (int e = tid; e < 16 * nz; e += NTH) {
      const int z = e >> 4, k = e & 15;
      col[(size_t)z * plane + k] = reg[z * 17 + k];
    }
  }
}

template <int LNZ, bool INV>
static hipError_t zpass_one(const ZArgs& a, hipStream_t s) {
  constexpr int M = (1 << LNZ) / 2;
  constexpr int R = zline_radix(M);
  const size_t lds = (size_t)(tab_points<M, R>() + zpass_rtab_points<M>() + zpass_region_points<M, R>()) *
                     sizeof(float2);
  if (lds > 65536) {
    const hipError_t e =
        hipFuncSetAttribute((const void*)k_zpass<LNZ, INV>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const dim3 grid((unsigned)(a.nb * 3 * a.nTiles * a.ny));
  hipLaunchKernelGGL((k_zpass<LNZ, INV>), grid, dim3(zpass_threads(LNZ)), lds, s, a);
  return hipGetLastError();
}

template <bool INV>
static hipError_t zpass_switch(int lnz, const ZArgs& a, hipStream_t s) {
  switch (lnz) {
    case 2: return zpass_one<2, INV>(a, s);
    case 3: return zpass_one<3, INV>(a, s);
    case 4: return zpass_one<4, INV>(a, s);
    case 5: return zpass_one<5, INV>(a, s);
    case 6: return zpass_one<6, INV>(a, s);
    case 7: return zpass_one<7, INV>(a, s);
    case 8: return zpass_one<8, INV>(a, s);
    case 9: return zpass_one<9, INV>(a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_zpass(int lnz, const ZArgs& a, bool inverse, hipStream_t s) {
  return inverse ? zpass_switch<true>(lnz, a, s) : zpass_switch<false>(lnz, a, s);
}

}  // namespace demag
