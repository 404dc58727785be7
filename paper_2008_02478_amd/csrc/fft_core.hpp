// Device FFT building blocks for gfx950 (wave64).
//
// A "group" is T consecutive lanes of one wavefront (T divides 64) that
// together transform one line of M complex points (M = T * R).  Lane t of the
// group holds R points in registers, v[j] = x[t + T*j] ("stride-T layout"), and
// gets back X[t + T*j] in the same layout.  The transform is a mixed-radix
// Stockham autosort FFT: the first radix-R stage runs on the registers as
// loaded, later stages exchange through a per-group LDS scratch of M points.
// Because a group never spans two wavefronts, exchanges need only wavefront
// ordering, never a workgroup barrier.
//
// Twiddle factors come from a table W_4096^k = exp(-2 pi i k / 4096) computed
// in FP64 on the host and rounded once to FP32 (no recurrences).
#pragma once
#include <hip/hip_runtime.h>

namespace demag {

constexpr int TW_LOG2 = 12;
constexpr int TW_SIZE = 1 << TW_LOG2;

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// All lanes of the wavefront have finished their LDS accesses before any lane
// continues (LDS traffic of one wavefront is ordered; this also stops the
// compiler from moving LDS accesses across the point).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// exp(-2 pi i m / N) (forward) or its conjugate (INV), N a power of two <= 4096.
template <bool INV>
__device__ __forceinline__ float2 twiddle(const float2* __restrict__ tw, int m, int log2N) {
  const int idx = (m & ((1 << log2N) - 1)) << (TW_LOG2 - log2N);
  float2 w = tw[idx];
  if (INV) w.y = -w.y;
  return w;
}

// Compile-time twiddles W_16^k for the in-register butterflies.
__device__ __forceinline__ constexpr float c16(int k) {
  return k == 0 ? 1.0f : k == 1 ? 0.92387953251128674f : k == 2 ? 0.70710678118654752f
       : k == 3 ? 0.38268343236508977f : k == 4 ? 0.0f : k == 5 ? -0.38268343236508977f
       : k == 6 ? -0.70710678118654752f : k == 7 ? -0.92387953251128674f : -1.0f;
}
// a * W_LEN^J (forward: exp(-2 pi i J/LEN); INV: conjugate), LEN <= 16, J < LEN/2.
template <int LEN, int J, bool INV>
__device__ __forceinline__ float2 tw_const(float2 a) {
  constexpr int k = J * (16 / LEN);  // index into W_16, 0 <= k < 8
  if constexpr (k == 0) {
    return a;
  } else if constexpr (k == 4) {     // -i (forward) / +i (inverse)
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
  } else {
    constexpr float c = c16(k);
    constexpr float s = (k < 4) ? c16(4 - k) : c16(k - 4);  // sin(2 pi k/16) for 0 < k < 8
    // forward multiplies by (c - i s), inverse by (c + i s)
    if constexpr (INV) return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
    else return make_float2(a.x * c + a.y * s, a.y * c - a.x * s);
  }
}

template <int R>
__device__ __forceinline__ constexpr int bitrev(int i) {
  int r = 0;
  for (int b = 1; b < R; b <<= 1) { r = (r << 1) | (i & 1); i >>= 1; }
  return r;
}

template <int LEN, int BASE, int J, int R, bool INV>
__device__ __forceinline__ void bfly_j(float2 (&b)[R]) {
  if constexpr (J < LEN / 2) {
    const float2 u = b[BASE + J];
    const float2 t = tw_const<LEN, J, INV>(b[BASE + J + LEN / 2]);
    b[BASE + J] = cadd(u, t);
    b[BASE + J + LEN / 2] = csub(u, t);
    bfly_j<LEN, BASE, J + 1, R, INV>(b);
  }
}
template <int LEN, int BASE, int R, bool INV>
__device__ __forceinline__ void bfly_blocks(float2 (&b)[R]) {
  if constexpr (BASE < R) {
    bfly_j<LEN, BASE, 0, R, INV>(b);
    bfly_blocks<LEN, BASE + LEN, R, INV>(b);
  }
}
template <int LEN, int R, bool INV>
__device__ __forceinline__ void bfly_levels(float2 (&b)[R]) {
  if constexpr (LEN <= R) {
    bfly_blocks<LEN, 0, R, INV>(b);
    bfly_levels<LEN * 2, R, INV>(b);
  }
}

// In-register DFT of R <= 16 points (radix-2 DIT, fully unrolled).
template <int R, bool INV>
__device__ __forceinline__ void dft(float2 (&a)[R]) {
  if constexpr (R == 1) {
    return;
  } else {
    float2 b[R];
#pragma unroll
    for (int i = 0; i < R; ++i) b[bitrev<R>(i)] = a[i];
    bfly_levels<2, R, INV>(b);
#pragma unroll
    for (int i = 0; i < R; ++i) a[i] = b[i];
  }
}

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x >> 1); }

// One Stockham stage (not the first): NS = product of earlier radices, RS = this radix.
template <int M, int R, int NS, int RS, bool INV>
__device__ __forceinline__ void stockham_stage(float2 (&v)[R], float2* __restrict__ lds, int t,
                                               const float2* __restrict__ tw) {
  constexpr int T = M / R;
  constexpr int NB = R / RS;        // butterflies per lane
  constexpr bool LAST = (NS * RS == M);
  float2 a[NB][RS];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = t + T * i;
#pragma unroll
    for (int r = 0; r < RS; ++r) a[i][r] = lds[b + r * (M / RS)];
  }
  wave_sync();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = t + T * i;
    const int k = b & (NS - 1);
#pragma unroll
    for (int r = 1; r < RS; ++r)
      a[i][r] = cmul(a[i][r], twiddle<INV>(tw, r * k, ilog2(NS * RS)));
    dft<RS, INV>(a[i]);
  }
  if constexpr (LAST) {
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int r = 0; r < RS; ++r) v[i + r * NB] = a[i][r];
  } else {
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int b = t + T * i;
      const int k = b & (NS - 1);
      const int base = (b / NS) * NS * RS + k;
#pragma unroll
      for (int r = 0; r < RS; ++r) lds[base + r * NS] = a[i][r];
    }
    wave_sync();
  }
}

template <int M, int R, int NS, bool INV>
__device__ __forceinline__ void stockham_rest(float2 (&v)[R], float2* __restrict__ lds, int t,
                                              const float2* __restrict__ tw) {
  if constexpr (NS < M) {
    constexpr int left = M / NS;
    constexpr int RS = left >= R ? R : left;
    stockham_stage<M, R, NS, RS, INV>(v, lds, t, tw);
    stockham_rest<M, R, NS * RS, INV>(v, lds, t, tw);
  }
}

// Group FFT of M points, lane t in [0, M/R) of its group, stride-T layout in
// and out.  lds: M points of scratch owned by this group (unused when M == R).
// Unnormalized in both directions.
template <int M, int R, bool INV>
__device__ __forceinline__ void group_fft(float2 (&v)[R], float2* __restrict__ lds, int t,
                                          const float2* __restrict__ tw) {
  static_assert(M % R == 0, "R must divide M");
  constexpr int T = M / R;
  static_assert(T <= 64 && (64 % T) == 0, "a group must fit in one wavefront");
  dft<R, INV>(v);
  if constexpr (M > R) {
    // first stage output index b*R + r for butterfly b = t
#pragma unroll
    for (int r = 0; r < R; ++r) lds[t * R + r] = v[r];
    wave_sync();
    stockham_rest<M, R, R, INV>(v, lds, t, tw);
  }
}

// Points per lane used for an M-point line.
template <int M>
struct LineShape {
  static constexpr int R = M >= 1024 ? 16 : (M >= 8 ? 8 : M);
  static constexpr int T = M / R;
};

}  // namespace demag
