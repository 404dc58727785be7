// Coupled layers (Sec. 3, Eq. 4): meshes with their own cell sizes and
// positions whose fields couple through inter-mesh tensors N(r, h_k, h_i);
// "the summation of inter-mesh contributions moved to the transform space".
//
// All z planes of a group share one fine in-plane lattice (coarser layers
// are zero-inserted at their stride).  Per evaluation:
//   k_lfwd   : per (fine row, component): real-to-complex x FFT of every
//              plane's row (zeros where a plane has no cell) -> T
//   k_mid<1> : y FFT of every (plane, kx) line -> S (full ky range)
//   k_couple : per (kx, ky): H_p = sum_q K_pq M_q over all plane pairs, the
//              pair kernels of q > p from p < q by reciprocity
//              (V_p N_pq(r) = V_q N_qp(-r) -> K_qp = V_p/V_q conj K_pq);
//              Parseval energy partials
//   k_mid<2> : inverse y FFT -> T
//   k_linv   : inverse x FFT, keeping each plane's own cells -> H
#include "fft_core.hpp"
#include "plan.hpp"
#include "xrows.hpp"
#include "launch.hpp"

namespace demag {

// Index of the fine-lattice offset i on a plane of stride s and n cells: i / s
// when i is a non-negative multiple of s below s n, else -1.  The quotient is
// the nearest integer to i (1/s), exact for |i| < 2^22 (no integer division).
__device__ __forceinline__ int on_stride(int i, int s, int n) {
  const int q = (int)rintf((float)i * __frcp_rn((float)s));
  return (q * s == i && q >= 0 && q < n) ? q : -1;
}

template <int LNX>
__global__ void __launch_bounds__(FWD_THREADS) __attribute__((amdgpu_waves_per_eu(LNX >= 12 ? 2 : 4, 8))) k_lfwd(LayerArgs a) {
  extern __shared__ float2 smem_base[];
  constexpr int PITCH = xrow_pitch<LNX>();
  float2* const tab = smem_base;
  float2* const smem = smem_base + xtab_points<LNX>();
  const int lg = xcd_logical(blockIdx.x, gridDim.x);
  const int c = lg / a.Ly, v = lg - c * a.Ly;
  // A fine-lattice point (2 mm + h, v) holds a cell of plane p when it falls on
  // the plane's stride inside its extent.  Loads read a clamped in-range cell
  // and the scale step zeroes the points without one, so that no load sits
  // under a condition (its wait would be taken at once).
  auto cell_x = [&](const PlaneInfo& pi, int ix) -> int { return on_stride(ix, pi.sx, pi.nx); };
  auto cell_y = [&](const PlaneInfo& pi) -> int { return on_stride(v - pi.oy, pi.sy, pi.ny); };
  xfwd_rows<LNX, FWD_THREADS>(smem, tab, a.tw, a.P, PITCH, [&](int p, int mm) -> float2 {
    const PlaneInfo pi = a.pl[p];
    const int yy = cell_y(pi);
    const float* src = a.m + pi.moff + (((size_t)c * pi.nz + pi.k) * pi.ny + (yy < 0 ? 0 : yy)) * pi.nx;
    const int x0 = cell_x(pi, 2 * mm - pi.ox), x1 = cell_x(pi, 2 * mm + 1 - pi.ox);
    return make_float2(src[x0 < 0 ? 0 : x0], src[x1 < 0 ? 0 : x1]);
  }, [&](int p, int mm, float2 u) -> float2 {
    const PlaneInfo pi = a.pl[p];
    const float sc = a.backward ? 1.0f / pi.vol : (a.ms_mesh ? a.ms_mesh[pi.gid] : a.ms);
    const bool row = cell_y(pi) >= 0;
    const bool in0 = row && cell_x(pi, 2 * mm - pi.ox) >= 0, in1 = row && cell_x(pi, 2 * mm + 1 - pi.ox) >= 0;
    return make_float2(in0 ? sc * u.x : 0.f, in1 ? sc * u.y : 0.f);
  });
  const int Kx = a.Kx;
  for (int it = threadIdx.x; it < a.P * Kx; it += FWD_THREADS) {
    const int p = it / Kx, kx = it - p * Kx;
    a.T[((((size_t)c * a.P + p) * a.nTiles + kx / TILE) * a.Ly + v) * TILE + (kx % TILE)] = smem[p * PITCH + kx];
  }
}

template <int LNX>
__global__ void __launch_bounds__(INV_THREADS) __attribute__((amdgpu_waves_per_eu(LNX >= 12 ? 2 : 4, 8))) k_linv(LayerArgs a) {
  extern __shared__ float2 smem_base[];
  constexpr int PITCH = xrow_pitch<LNX>();
  float2* const tab = smem_base;
  float2* const smem = smem_base + xtab_points<LNX>();
  const int lg = xcd_logical(blockIdx.x, gridDim.x);
  const int c = lg / a.Ly, v = lg - c * a.Ly;
  const int Kx = a.Kx;
  for (int it = threadIdx.x; it < a.P * Kx; it += INV_THREADS) {
    const int p = it / Kx, kx = it - p * Kx;
    smem[p * PITCH + kx] = a.T[((((size_t)c * a.P + p) * a.nTiles + kx / TILE) * a.Ly + v) * TILE + (kx % TILE)];
  }
  __syncthreads();
  xinv_rows<LNX, INV_THREADS>(smem, tab, a.tw, a.P, PITCH, [&](int p, int mm, float2 uu) {
    const PlaneInfo pi = a.pl[p];
    const int yy = on_stride(v - pi.oy, pi.sy, pi.ny);
    if (yy < 0) return;
    const size_t row = pi.moff + (((size_t)c * pi.nz + pi.k) * pi.ny + yy) * pi.nx;
    float post = 1.f, beta = 0.f;
    if (a.backward) {
      post = (a.ms_mesh ? a.ms_mesh[pi.gid] : a.ms) * pi.vol;
      if (a.beta_ptr) beta = (float)(a.beta_scale * a.beta_ptr[pi.gid]);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int xx = on_stride(2 * mm + h - pi.ox, pi.sx, pi.nx);
      if (xx >= 0) {
        const size_t o = row + xx;
        float val = h ? uu.y : uu.x;
        if (a.backward) val = post * (val + (a.beta_ptr ? beta * a.aux[o] : 0.f));
        a.H[o] = a.accumulate ? a.H[o] + val : val;
      }
    }
  });
}

// complex 3x3 symmetric K (xx yy zz xy xz yz) times complex vector, added to h
__device__ __forceinline__ void sym_mac(float2 (&h)[3], const float2 (&k)[6], const float2 (&m)[3], float s,
                                       bool conj_k) {
  auto mul = [&](float2 kk, float2 mm) {
    const float2 kc = conj_k ? cconj(kk) : kk;
    return cscale(cmul(kc, mm), s);
  };
  h[0] = cadd(h[0], cadd(mul(k[0], m[0]), cadd(mul(k[3], m[1]), mul(k[4], m[2]))));
  h[1] = cadd(h[1], cadd(mul(k[3], m[0]), cadd(mul(k[1], m[1]), mul(k[5], m[2]))));
  h[2] = cadd(h[2], cadd(mul(k[4], m[0]), cadd(mul(k[5], m[1]), mul(k[2], m[2]))));
}

// plane pair n of the order (0,0), (0,1) .. (0,P-1), (1,1) .. (P-1,P-1)
template <int P>
constexpr int pair_p(int n) {
  int p = 0;
  while (n >= P - p) { n -= P - p; ++p; }
  return p;
}
template <int P>
constexpr int pair_q(int n) {
  int p = 0;
  while (n >= P - p) { n -= P - p; ++p; }
  return p + n;
}

// One pair's spectrum for this point as raw words: a pair stored one float
// per component (parity) reads that float twice; a full pair reads the real
// and imaginary words.  Branch-free, so that the next pair's reads can be in
// flight while this pair is summed.
struct PairWords {
  float x[6], y[6];
};
__device__ __forceinline__ void load_pair(PairWords& w, const float* __restrict__ K, size_t koff, bool par,
                                          size_t npt, size_t pt) {
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const size_t i = (size_t)e * npt + pt;
    const float* const ax = K + koff + (par ? i : 2 * i);
    w.x[e] = ax[0];
    w.y[e] = ax[par ? 0 : 1];
  }
}

template <int P, int N>
__device__ __forceinline__ void couple_pairs(const CoupleArgs& a, size_t npt, size_t pt, size_t koff,
                                             PairWords& cur, PairWords& nxt, float2 (&M)[P][3],
                                             float2 (&H)[P][3], const float (&vol)[P]) {
  constexpr int NP = P * (P + 1) / 2;
  if constexpr (N < NP) {
    constexpr int p = pair_p<P>(N), q = pair_q<P>(N);
    const bool par = (a.parity_pairs >> N) & 1ull;
    const size_t knext = koff + (size_t)(par ? 6 : 12) * npt;
    // the next pair's words are requested before this pair is summed
    if constexpr (N + 1 < NP) load_pair(nxt, a.K, knext, (a.parity_pairs >> (N + 1)) & 1ull, npt, pt);
    float2 k6[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      // parity pairs: real xx yy zz xy, imaginary xz yz
      if (e < 4) k6[e] = make_float2(cur.x[e], par ? 0.f : cur.y[e]);
      else k6[e] = make_float2(par ? 0.f : cur.x[e], cur.y[e]);
    }
    sym_mac(H[p], k6, M[q], 1.f, false);
    if constexpr (q != p) sym_mac(H[q], k6, M[p], vol[p] / vol[q], true);
    couple_pairs<P, N + 1>(a, npt, pt, knext, nxt, cur, M, H, vol);
  }
}

template <int P>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P <= 6 ? 4 : 2, 8))) k_couple(CoupleArgs a) {
  __shared__ double red[4][P];
  const size_t npt = (size_t)a.Kx * a.NY;
  const size_t pt = (size_t)blockIdx.x * 256 + threadIdx.x;
  const bool act = pt < npt;
  const size_t ptc = act ? pt : 0;          // lanes past the end read point 0
  const int kx = act ? (int)(pt / a.NY) : 0;
  float2 M[P][3], H[P][3];
  float vol[P];
  PairWords wa, wb;
  load_pair(wa, a.K, 0, a.parity_pairs & 1ull, npt, ptc);
#pragma unroll
  for (int p = 0; p < P; ++p) {
    vol[p] = a.pl[p].vol;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      M[p][c] = a.S[((size_t)c * P + p) * npt + ptc];
      H[p][c] = make_float2(0.f, 0.f);
    }
  }
  couple_pairs<P, 0>(a, npt, ptc, 0, wa, wb, M, H, vol);
  if (act) {
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int c = 0; c < 3; ++c) a.S[((size_t)c * P + p) * npt + pt] = H[p][c];
  }
  if (a.epart) {
    const float w = (kx == 0 || 2 * kx == a.Nx) ? 1.f : 2.f;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      double e = 0.0;
      if (act) {
        float d = 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c) d += M[p][c].x * H[p][c].x + M[p][c].y * H[p][c].y;
        e = (double)(w * vol[p] * d);
      }
      for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o);
      if (lane == 0) red[wv][p] = e;
    }
    __syncthreads();
    if (threadIdx.x < P) {
      const double s = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
      a.epart[(size_t)blockIdx.x * P + threadIdx.x] = s;
    }
  }
}

// energies of the meshes of a group: out[gid] = scale * sum over the mesh's
// planes and all workgroups' partials (fixed order)
template <int P>
__global__ void __launch_bounds__(FINAL_THREADS) k_lenergy(const double* part, int nblk, const PlaneInfo* pl,
                                                           double scale, double* out) {
  static_assert(P >= 1 && P <= MAXP, "planes per group");
  constexpr int NW = FINAL_THREADS / 64;
  constexpr int U = 4;                      // workgroup entries per thread and sweep
  __shared__ double red[NW][MAXP];
  __shared__ double tot[MAXP];
  __shared__ int gid[MAXP];
  // every plane's partials of U workgroup entries at once (P contiguous words
  // each), all reads issued before any is summed; entries past nblk read
  // entry 0 and add nothing.  Each plane's sum runs over the entries in
  // increasing order.
  double acc[P];
#pragma unroll
  for (int p = 0; p < P; ++p) acc[p] = 0.0;
  for (int i0 = threadIdx.x; i0 < nblk; i0 += U * FINAL_THREADS) {
    double v[U][P];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * FINAL_THREADS;
#pragma unroll
      for (int p = 0; p < P; ++p) v[u][p] = part[(size_t)(i < nblk ? i : 0) * P + p];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int p = 0; p < P; ++p) acc[p] += i0 + u * FINAL_THREADS < nblk ? v[u][p] : 0.0;
  }
  if ((int)threadIdx.x < P) gid[threadIdx.x] = pl[threadIdx.x].gid;
  // all planes' wavefront sums together (independent butterflies), then the
  // wavefronts in order
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
    for (int p = 0; p < P; ++p) acc[p] += __shfl_xor(acc[p], o);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int p = 0; p < P; ++p) red[w][p] = acc[p];
  }
  __syncthreads();
  if ((int)threadIdx.x < P) {
    double t = 0.0;
    for (int i = 0; i < NW; ++i) t += red[i][threadIdx.x];
    tot[threadIdx.x] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int p = 0; p < P; ++p) {
      bool first = true;
      for (int q = 0; q < p; ++q) first = first && gid[q] != gid[p];
      if (!first) continue;
      double t = 0.0;
      for (int q = p; q < P; ++q)
        if (gid[q] == gid[p]) t += tot[q];
      out[gid[p]] = scale * t;
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename K>
static hipError_t prep(K kern, size_t lds) {
  if (lds > 65536)
    return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return hipSuccess;
}

template <int LNX>
static hipError_t lx_one(const LayerArgs& a, bool inverse, hipStream_t s) {
  const size_t lds = ((size_t)a.P * xrow_pitch<LNX>() + xtab_points<LNX>()) * sizeof(float2);
  dim3 grid(a.Ly * 3);
  if (inverse) {
    hipError_t e = prep(k_linv<LNX>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_linv<LNX>), grid, dim3(INV_THREADS), lds, s, a);
  } else {
    hipError_t e = prep(k_lfwd<LNX>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_lfwd<LNX>), grid, dim3(FWD_THREADS), lds, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_layer_x(int lnx, const LayerArgs& a, bool inverse, hipStream_t s) {
  switch (lnx) {
    case 2: return lx_one<2>(a, inverse, s);
    case 3: return lx_one<3>(a, inverse, s);
    case 4: return lx_one<4>(a, inverse, s);
    case 5: return lx_one<5>(a, inverse, s);
    case 6: return lx_one<6>(a, inverse, s);
    case 7: return lx_one<7>(a, inverse, s);
    case 8: return lx_one<8>(a, inverse, s);
    case 9: return lx_one<9>(a, inverse, s);
    case 10: return lx_one<10>(a, inverse, s);
    case 11: return lx_one<11>(a, inverse, s);
    case 12: return lx_one<12>(a, inverse, s);
    default: return hipErrorInvalidValue;
  }
}

int couple_blocks(int Kx, int NY) { return (int)(((size_t)Kx * NY + 255) / 256); }

template <int P>
static hipError_t couple_one(const CoupleArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_couple<P>), dim3(couple_blocks(a.Kx, a.NY)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_couple(int P, const CoupleArgs& a, hipStream_t s) {
  switch (P) {
    case 1: return couple_one<1>(a, s);
    case 2: return couple_one<2>(a, s);
    case 3: return couple_one<3>(a, s);
    case 4: return couple_one<4>(a, s);
    case 5: return couple_one<5>(a, s);
    case 6: return couple_one<6>(a, s);
    case 7: return couple_one<7>(a, s);
    case 8: return couple_one<8>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <int P>
static hipError_t lenergy_one(const double* part, int nblk, const PlaneInfo* pl, double scale, double* out,
                              hipStream_t s) {
  hipLaunchKernelGGL((k_lenergy<P>), dim3(1), dim3(FINAL_THREADS), 0, s, part, nblk, pl, scale, out);
  return hipGetLastError();
}

hipError_t launch_layer_energy(const double* part, int nblk, int P, const PlaneInfo* pl, double scale, double* out,
                               hipStream_t s) {
  switch (P) {
    case 1: return lenergy_one<1>(part, nblk, pl, scale, out, s);
    case 2: return lenergy_one<2>(part, nblk, pl, scale, out, s);
    case 3: return lenergy_one<3>(part, nblk, pl, scale, out, s);
    case 4: return lenergy_one<4>(part, nblk, pl, scale, out, s);
    case 5: return lenergy_one<5>(part, nblk, pl, scale, out, s);
    case 6: return lenergy_one<6>(part, nblk, pl, scale, out, s);
    case 7: return lenergy_one<7>(part, nblk, pl, scale, out, s);
    case 8: return lenergy_one<8>(part, nblk, pl, scale, out, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace demag
