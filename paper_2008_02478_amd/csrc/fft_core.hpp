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

#include "plan.hpp"

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

// Exchange point of a group of T lanes: wavefront ordering for groups within
// one wavefront; a workgroup barrier for groups spanning several wavefronts
// (then every lane of the workgroup must run the same transforms).
template <int T>
__device__ __forceinline__ void group_sync() {
  if constexpr (T > 64) __syncthreads();
  else wave_sync();
}

// exp(-2 pi i m / N) (forward) or its conjugate (INV), N a power of two <= 4096.
template <bool INV>
__device__ __forceinline__ float2 twiddle(const float2* __restrict__ tw, int m, int log2N) {
  const int idx = (m & ((1 << log2N) - 1)) << (TW_LOG2 - log2N);
  float2 w = tw[idx];
  if (INV) w.y = -w.y;
  return w;
}

// Compile-time cos(2 pi k / 128), 0 <= k <= 64, for the in-register
// butterflies (values of the double-precision cosine, rounded to float).
__device__ __forceinline__ constexpr float cos128(int k) {
  return k == 0 ? 1.0f : k == 1 ? 0.9987954562051724f : k == 2 ? 0.9951847266721969f :
       k == 3 ? 0.989176509964781f : k == 4 ? 0.9807852804032304f : k == 5 ? 0.970031253194544f :
       k == 6 ? 0.9569403357322088f : k == 7 ? 0.9415440651830208f : k == 8 ? 0.9238795325112867f :
       k == 9 ? 0.9039892931234433f : k == 10 ? 0.881921264348355f : k == 11 ? 0.8577286100002721f :
       k == 12 ? 0.8314696123025452f : k == 13 ? 0.8032075314806449f : k == 14 ? 0.773010453362737f :
       k == 15 ? 0.7409511253549591f : k == 16 ? 0.7071067811865476f : k == 17 ? 0.6715589548470183f :
       k == 18 ? 0.6343932841636455f : k == 19 ? 0.5956993044924335f : k == 20 ? 0.5555702330196023f :
       k == 21 ? 0.5141027441932217f : k == 22 ? 0.4713967368259978f : k == 23 ? 0.4275550934302822f :
       k == 24 ? 0.38268343236508984f : k == 25 ? 0.33688985339222005f : k == 26 ? 0.29028467725446233f :
       k == 27 ? 0.24298017990326398f : k == 28 ? 0.19509032201612833f : k == 29 ? 0.14673047445536175f :
       k == 30 ? 0.09801714032956077f : k == 31 ? 0.049067674327418126f : k == 32 ? 0.0f
       : -cos128(64 - k);
}

// a * W_LEN^J (forward: exp(-2 pi i J/LEN); INV: conjugate), LEN <= 128, J < LEN/2.
template <int LEN, int J, bool INV>
__device__ __forceinline__ float2 tw_const(float2 a) {
  static_assert(LEN <= 128 && J < LEN / 2, "constant twiddle out of range");
  constexpr int k = J * (128 / LEN);  // angle 2 pi k / 128, 0 <= k < 64
  if constexpr (k == 0) {
    return a;
  } else if constexpr (k == 32) {    // -i (forward) / +i (inverse)
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
  } else {
    constexpr float c = cos128(k);
    constexpr float s = cos128(k < 32 ? 32 - k : k - 32);  // sin(2 pi k/128) > 0
    // forward multiplies by (c - i s), inverse by (c + i s)
    if constexpr (INV) return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
    else return make_float2(a.x * c + a.y * s, a.y * c - a.x * s);
  }
}

// f(i, base W_LEN^i) for i = 0 .. N-1 (forward, or the conjugate factors for
// INV), the factors compile-time constants: the twiddles of points spaced
// LEN-th of a turn apart from one table read.
template <int LEN, int N, bool INV, int I = 0, typename F>
__device__ __forceinline__ void for_const_twiddles(float2 base, F&& f) {
  if constexpr (I < N) {
    f(I, tw_const<LEN, I, INV>(base));
    for_const_twiddles<LEN, N, INV, I + 1>(base, f);
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

// In-register DFT of R <= 128 points (radix-2 DIT, fully unrolled).
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

// LDS placement of point i of an M-point line: one pad point after every
// 2^s points (s = 3 for radix 8, 5 for radix 16).  It spreads the strided
// Stockham accesses over the LDS banks while keeping every address an affine
// function of the lane, so paired ds_read2/ds_write2 offsets still apply.
template <int M, int R>
__device__ __forceinline__ int swz(int i) { return i + (i >> line_pad_shift(R)); }
// LDS points a group needs for an M-point line with this padding.
template <int M, int R>
constexpr int lds_points() { return M + (M >> line_pad_shift(R)); }

// Twiddles of the later Stockham stages of an M-point line, kept in LDS in
// the order [stage][r - 1][k] (k = butterfly index mod NS), so that lanes with
// consecutive k read consecutive entries.  Stage s with NS and radix RS holds
// W_{NS RS}^(r k) for 1 <= r < RS and 0 <= k < NS.
template <int M, int R>
constexpr int stage_table_size() {
  int n = 0, ns = R;
  while (ns < M) {
    const int left = M / ns, rs = left >= R ? R : left;
    n += (rs - 1) * ns;
    ns *= rs;
  }
  return n;
}

// Fill the table cooperatively from the FP32 W_4096 table (threads nth).  The
// stages are walked at compile time, so each entry costs a shift, a mask and
// one table read.
template <int M, int R, int NS, int OFF>
__device__ __forceinline__ void fill_stage_table_from(float2* __restrict__ tab, const float2* __restrict__ tw,
                                                      int tid, int nth) {
  if constexpr (NS < M) {
    constexpr int left = M / NS;
    constexpr int RS = left >= R ? R : left;
    constexpr int CNT = (RS - 1) * NS;
    for (int e = tid; e < CNT; e += nth) {
      const int r = e / NS + 1, k = e % NS;      // NS a power of two: shift and mask
      tab[OFF + e] = twiddle<false>(tw, r * k, ilog2(NS * RS));
    }
    fill_stage_table_from<M, R, NS * RS, OFF + CNT>(tab, tw, tid, nth);
  }
}
template <int M, int R>
__device__ __forceinline__ void fill_stage_table(float2* __restrict__ tab, const float2* __restrict__ tw, int tid,
                                                 int nth) {
  fill_stage_table_from<M, R, R, 0>(tab, tw, tid, nth);
}

// The same tables (stage table and, if RES, the odd-residue table rtab of
// fill_residue_table) staged through registers: load() issues the reads of the
// W_4096 table, store() writes LDS.  A kernel issues load() before its bulk
// loads and store() after them, so the table reads overlap them; memory
// counters retire in issue order, so store() waits only for the table reads.
// Lanes past an entry count read an in-range table entry (indices are masked)
// and store it to a discard slot, so that no store is conditional (a
// conditional store would let the compiler sink the read next to it, where
// it is waited for at once).  NTH: threads of the workgroup (compile time).
template <int M, int R, int NTH, bool RES>
struct TabRegs {
  template <int NS>
  static constexpr int iters_from() {
    if constexpr (NS >= M) {
      return 0;
    } else {
      constexpr int left = M / NS, RS = left >= R ? R : left, CNT = (RS - 1) * NS;
      return (CNT + NTH - 1) / NTH + iters_from<NS * RS>();
    }
  }
  static constexpr int NRI = RES ? (M + NTH - 1) / NTH : 0;
  static constexpr int K = iters_from<R>() + NRI;
  float2 v[K > 0 ? K : 1];

  template <int NS, int SLOT>
  __device__ __forceinline__ void load_from(const float2* __restrict__ tw, int tid) {
    if constexpr (NS < M) {
      constexpr int left = M / NS, RS = left >= R ? R : left, CNT = (RS - 1) * NS, IT = (CNT + NTH - 1) / NTH;
#pragma unroll
      for (int i = 0; i < IT; ++i) {
        const int e = tid + i * NTH;
        v[SLOT + i] = twiddle<false>(tw, (e / NS + 1) * (e % NS), ilog2(NS * RS));
      }
      load_from<NS * RS, SLOT + IT>(tw, tid);
    }
  }
  template <int NS, int SLOT, int OFF>
  __device__ __forceinline__ void store_from(float2* __restrict__ tab, float2* sink, int tid) const {
    if constexpr (NS < M) {
      constexpr int left = M / NS, RS = left >= R ? R : left, CNT = (RS - 1) * NS, IT = (CNT + NTH - 1) / NTH;
#pragma unroll
      for (int i = 0; i < IT; ++i) {
        const int e = tid + i * NTH;
        *((CNT % NTH == 0 || e < CNT) ? tab + OFF + e : sink) = v[SLOT + i];
      }
      store_from<NS * RS, SLOT + IT, OFF + CNT>(tab, sink, tid);
    }
  }
  __device__ __forceinline__ void load(const float2* __restrict__ tw, int tid) {
    load_from<R, 0>(tw, tid);
    if constexpr (RES) {
#pragma unroll
      for (int i = 0; i < NRI; ++i) v[K - NRI + i] = twiddle<false>(tw, tid + i * NTH, ilog2(2 * M));
    }
  }
  __device__ __forceinline__ void store(float2* __restrict__ tab, float2* __restrict__ rtab, int tid) const {
    __shared__ float2 sink;   // written by lanes past an entry count, never read
    store_from<R, 0, 0>(tab, &sink, tid);
    if constexpr (RES) {
#pragma unroll
      for (int i = 0; i < NRI; ++i) {
        const int k = tid + i * NTH;
        *((M % NTH == 0 || k < M) ? rtab + k : &sink) = v[K - NRI + i];
      }
    }
  }
};

// One Stockham stage (not the first): NS = product of earlier radices, RS = this radix.
template <int M, int R, int NS, int RS, bool INV, int OFF>
__device__ __forceinline__ void stockham_stage(float2 (&v)[R], float2* __restrict__ lds, int t,
                                               const float2* __restrict__ tab) {
  constexpr int T = M / R;
  constexpr int NB = R / RS;        // butterflies per lane
  constexpr bool LAST = (NS * RS == M);
  float2 a[NB][RS];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = t + T * i;
#pragma unroll
    for (int r = 0; r < RS; ++r) a[i][r] = lds[swz<M, R>(b + r * (M / RS))];
  }
  group_sync<T>();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int k = (t + T * i) & (NS - 1);
#pragma unroll
    for (int r = 1; r < RS; ++r) {
      const float2 wv = tab[OFF + (r - 1) * NS + k];
      a[i][r] = INV ? cmulc(a[i][r], wv) : cmul(a[i][r], wv);
    }
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
      for (int r = 0; r < RS; ++r) lds[swz<M, R>(base + r * NS)] = a[i][r];
    }
    group_sync<T>();
  }
}

template <int M, int R, int NS, bool INV, int OFF>
__device__ __forceinline__ void stockham_rest(float2 (&v)[R], float2* __restrict__ lds, int t,
                                              const float2* __restrict__ tab) {
  if constexpr (NS < M) {
    constexpr int left = M / NS;
    constexpr int RS = left >= R ? R : left;
    stockham_stage<M, R, NS, RS, INV, OFF>(v, lds, t, tab);
    stockham_rest<M, R, NS * RS, INV, OFF + (RS - 1) * NS>(v, lds, t, tab);
  }
}

// Group FFT of M points, lane t in [0, M/R) of its group, stride-T layout in
// and out.  lds: M points of scratch owned by this group (unused when M == R);
// tab: the stage twiddle table in LDS.  Unnormalized in both directions.  A
// group of more than 64 lanes exchanges through workgroup barriers.
template <int M, int R, bool INV>
__device__ __forceinline__ void group_fft(float2 (&v)[R], float2* __restrict__ lds, int t,
                                          const float2* __restrict__ tab) {
  static_assert(M % R == 0, "R must divide M");
  constexpr int T = M / R;
  static_assert((T <= 64 && (64 % T) == 0) || T % 64 == 0, "a group is part of a wavefront or whole wavefronts");
  dft<R, INV>(v);
  if constexpr (M > R) {
    // a group spanning wavefronts waits until every wavefront has finished
    // reading this scratch (the previous transform's last stage)
    if constexpr (T > 64) __syncthreads();
    // first stage output index b*R + r for butterfly b = t
#pragma unroll
    for (int r = 0; r < R; ++r) lds[swz<M, R>(t * R + r)] = v[r];
    group_sync<T>();
    stockham_rest<M, R, R, INV, 0>(v, lds, t, tab);
  }
}

// v[j] *= W_{2M}^(t + T j) for j < R (INV: conjugate), where T = M / R, on
// lanes with `on` set; other lanes multiply by 1.  The factor is one table
// value W_{2M}^t (base) times the compile-time W_{2R}^j, picked by a select
// rather than a branch so that divergent lanes do not keep two copies.
template <int R, int J, bool INV>
__device__ __forceinline__ void residue_twiddle_j(float2 (&v)[R], float2 base, bool on) {
  if constexpr (J < R) {
    float2 f = tw_const<2 * R, J, false>(base);
    f.x = on ? f.x : 1.0f;
    f.y = on ? f.y : 0.0f;
    v[J] = INV ? cmulc(v[J], f) : cmul(v[J], f);
    residue_twiddle_j<R, J + 1, INV>(v, base, on);
  }
}
template <int R, bool INV>
__device__ __forceinline__ void residue_twiddle(float2 (&v)[R], float2 base, bool on) {
  residue_twiddle_j<R, 0, INV>(v, base, on);
}

// Odd-residue twiddles of an M-point line: the odd outputs of a 2M-point
// transform of M non-zero points are the M-point transform of x[n] W_2M^n.
// rtab[k] = W_2M^k for k < M, filled cooperatively into LDS.
template <int M>
__device__ __forceinline__ void fill_residue_table(float2* __restrict__ rtab, const float2* __restrict__ tw,
                                                   int tid, int nth) {
  for (int k = tid; k < M; k += nth) rtab[k] = twiddle<false>(tw, k, ilog2(2 * M));
}
// v[j] *= rtab[t + T j] (INV: conjugate), stride-T layout of lane t.
template <int R, int T, bool INV>
__device__ __forceinline__ void residue_twiddle_tab(float2 (&v)[R], const float2* __restrict__ rtab, int t) {
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const float2 w = rtab[t + T * j];
    v[j] = INV ? cmulc(v[j], w) : cmul(v[j], w);
  }
}

// Points per lane used for an M-point line.
template <int M>
struct LineShape {
  static constexpr int R = line_radix(M);
  static constexpr int T = M / R;
};

__device__ __forceinline__ int xcd_logical(int b, int nblk) {
  // workgroups are handed to the 8 XCDs round-robin; give each XCD a
  // contiguous range of logical work so neighbours share its L2
  const int x = b & 7, idx = b >> 3;
  const int per = nblk >> 3, rem = nblk & 7;
  return x * per + min(x, rem) + idx;
}

}  // namespace demag
