// Real-to-complex and complex-to-real transforms of rows along x, shared by
// the single-mesh and the coupled-layer x passes.
//
// A row of NX = 2^LNX points (NX >= 4, at most NX/2 of them non-zero) is
// packed as u[m] = x[2m] + i x[2m+1]; its L = NX/2-point FFT is split into the
// even and odd output residues (two P = L/2-point FFTs, the input upper half
// being zero), and X[k], 0 <= k <= L, follows from U[k] and U[L-k].  Rows live
// in LDS at smem + row * pitch; each row's two residue FFTs use its own slots
// as scratch.  A row is handled by 2T lanes (T = lanes of one residue FFT).
#pragma once
#include "fft_core.hpp"
#include "plan.hpp"

namespace demag {

// LDS points reserved for the stage twiddle table of an M-point line FFT
// (rounded up to 32 points so that the data after it stays 256-byte aligned).
template <int M, int R = LineShape<M>::R>
constexpr int tab_points() {
  return (M > R) ? ((stage_table_size<M, R>() + 31) / 32) * 32 : 0;
}
template <int LNX>
constexpr int xrow_pitch() { return xrow_pitch_rt(LNX); }
template <int LNX>
constexpr int xtab_points() {
  return (LNX >= 2) ? tab_points<((1 << LNX) / 4 > 0 ? (1 << LNX) / 4 : 1)>() : 0;
}


// load(row, m) returns the raw (x[2m], x[2m+1]) of that row and scale(row,
// m, v) the value transformed, zeroed past the row's end, so that a round's
// loads can be issued one round ahead: round i + 1's loads are in flight while
// round i is transformed.  load must read in-range memory for every m < L/2
// (clamping its index, or returning zeros itself) and is called for row <
// rows only; branch-free loads are issued unconditionally, so the waits for
// them count exactly.  On return row r of smem holds X[0..L].  Ends with a
// workgroup barrier.
template <int LNX, int NTH, typename Load, typename Scale>
__device__ __forceinline__ void xfwd_rows(float2* __restrict__ smem, float2* __restrict__ tab,
                                          const float2* __restrict__ tw, int rows, int pitch, Load&& load,
                                          Scale&& scale) {
  constexpr int NX = 1 << LNX;
  constexpr int L = NX / 2;
  constexpr int P = L / 2;
  constexpr int R = LineShape<P>::R;
  constexpr int T = LineShape<P>::T;
  constexpr int RPR = NTH / (2 * T);
  const int tid = threadIdx.x;
  const int sub = tid / (2 * T);
  const int r = (tid / T) & 1;
  const int t = tid % T;
  // table reads first; the first round's rows behind them (lanes past the
  // last row re-read it)
  TabRegs<P, R, NTH, false> tabr;
  tabr.load(tw, tid);
  const float2 rbase = twiddle<false>(tw, t, ilog2(2 * P));
  // the split step's twiddles W_NX^k, k = k0 + i 2T: W_NX^k0 times constants
  const int k0 = tid % (2 * T);
  const float2 wk0 = twiddle<false>(tw, k0, LNX);
  float2 nxt[R];
  {
    const int r0 = sub < rows ? sub : rows - 1;
#pragma unroll
    for (int j = 0; j < R; ++j) nxt[j] = load(r0, t + T * j);
  }
  tabr.store(tab, nullptr, tid);
  __syncthreads();
  for (int start = 0; start < rows; start += RPR) {
    const int row = start + sub;
    const bool act = row < rows;
    float2* rb = smem + row * pitch;
    float2 u[R];
#pragma unroll
    for (int j = 0; j < R; ++j) u[j] = nxt[j];
    {
      // next round's rows (the last row again past the end: a cache hit)
      const int rn = row + RPR < rows ? row + RPR : rows - 1;
#pragma unroll
      for (int j = 0; j < R; ++j) nxt[j] = load(rn, t + T * j);
    }
    if (act) {
#pragma unroll
      for (int j = 0; j < R; ++j) u[j] = scale(row, t + T * j, u[j]);
      residue_twiddle<R, false>(u, rbase, r != 0);
      group_fft<P, R, false>(u, rb + r * lds_points<P, R>(), t, tab);
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int j = 0; j < R; ++j) rb[2 * (t + T * j) + r] = u[j];
    }
    __syncthreads();
    if (act) {
      // X[k] = E + W^k O and X[L-k] = conj(E - W^k O), with
      // E = (U[k] + conj U[L-k]) / 2 and O = -i (U[k] - conj U[L-k]) / 2.
      // k = k0 + i 2T <= L/2 needs i <= R/2 (2T = L/R)
      for_const_twiddles<2 * R, R / 2 + 1, false>(wk0, [&](int i, float2 w) {
        const int k = k0 + i * (2 * T);
        if (k > L / 2) return;
        const float2 Uk = rb[k];
        const float2 Um = rb[(L - k) & (L - 1)];
        const float2 E = make_float2(0.5f * (Uk.x + Um.x), 0.5f * (Uk.y - Um.y));
        const float2 O = make_float2(0.5f * (Uk.y + Um.y), -0.5f * (Uk.x - Um.x));
        const float2 WO = cmul(O, w);
        if (k == 0) {
          rb[0] = make_float2(E.x + O.x, E.y + O.y);
          rb[L] = make_float2(E.x - O.x, E.y - O.y);
        } else {
          rb[k] = cadd(E, WO);
          if (k != L - k) rb[L - k] = cconj(csub(E, WO));
        }
      });
    }
    __syncthreads();
  }
}

// The stage table of the x passes' Nx/4-point residue FFTs and the lane's
// odd-residue twiddle base, read into registers by load() (issued ahead of a
// kernel's bulk loads) and the table written to LDS by store().
template <int LNX, int NTH>
struct XTabPre {
  static constexpr int P = (1 << LNX) / 4;
  static constexpr int R = LineShape<P>::R;
  static constexpr int T = LineShape<P>::T;
  TabRegs<P, R, NTH, false> tabr;
  float2 rbase;
  float2 kbase;   // W_NX^-(2t + r), the split step's twiddle of the lane's first point
  __device__ __forceinline__ void load(const float2* __restrict__ tw, int tid) {
    tabr.load(tw, tid);
    rbase = twiddle<false>(tw, tid % T, ilog2(2 * P));
    kbase = twiddle<true>(tw, 2 * (tid % T) + ((tid / T) & 1), LNX);
  }
  __device__ __forceinline__ void store(float2* __restrict__ tab, int tid) const { tabr.store(tab, nullptr, tid); }
};

// Rows of smem hold X[0..L]; store(row, m, (x[2m], x[2m+1])) receives the
// unnormalized inverse for m < NX/4.  pre: the tables, read earlier by the
// caller and already stored to LDS (the barrier at entry publishes them).
// Ends with a workgroup barrier.
template <int LNX, int NTH, typename Store>
__device__ __forceinline__ void xinv_rows_pre(float2* __restrict__ smem, float2* __restrict__ tab,
                                              const float2* __restrict__ tw, int rows, int pitch,
                                              const XTabPre<LNX, NTH>& pre, Store&& store) {
  constexpr int NX = 1 << LNX;
  constexpr int L = NX / 2;
  constexpr int P = L / 2;
  constexpr int R = LineShape<P>::R;
  constexpr int T = LineShape<P>::T;
  constexpr int RPR = NTH / (2 * T);
  const int tid = threadIdx.x;
  const int sub = tid / (2 * T);
  const int r = (tid / T) & 1;
  const int t = tid % T;
  const float2 rbase = pre.rbase;
  __syncthreads();
  for (int start = 0; start < rows; start += RPR) {
    const int row = start + sub;
    const bool act = row < rows;
    float2* rb = smem + row * pitch;
    float2 u[R];
    if (act) {
      // U[k] = (X[k] + conj X[L-k]) + i W^-k (X[k] - conj X[L-k]): inverse of
      // the packed FFT of (x[2m], x[2m+1]), scaled to match X
      // W_NX^-k for k = 2t + r + 2T j: the lane's base times W_2R^-j (2T = NX/2R)
      for_const_twiddles<2 * R, R, true>(pre.kbase, [&](int j, float2 w) {
        const int k = 2 * (t + T * j) + r;
        const float2 Xk = rb[k];
        const float2 Xm = rb[L - k];
        const float2 S = make_float2(Xk.x + Xm.x, Xk.y - Xm.y);
        const float2 D = make_float2(Xk.x - Xm.x, Xk.y + Xm.y);
        const float2 WD = cmul(D, w);
        u[j] = make_float2(S.x - WD.y, S.y + WD.x);
      });
    }
    __syncthreads();
    if (act) {
      group_fft<P, R, true>(u, rb + r * lds_points<P, R>(), t, tab);
      residue_twiddle<R, true>(u, rbase, r != 0);
    }
    __syncthreads();
    if (act && r == 1) {
#pragma unroll
      for (int j = 0; j < R; ++j) rb[t + T * j] = u[j];
    }
    __syncthreads();
    if (act && r == 0) {
#pragma unroll
      for (int j = 0; j < R; ++j) store(row, t + T * j, cadd(u[j], rb[t + T * j]));
    }
    __syncthreads();
  }
}

// xinv_rows_pre with the tables read here.
template <int LNX, int NTH, typename Store>
__device__ __forceinline__ void xinv_rows(float2* __restrict__ smem, float2* __restrict__ tab,
                                          const float2* __restrict__ tw, int rows, int pitch, Store&& store) {
  XTabPre<LNX, NTH> pre;
  pre.load(tw, threadIdx.x);
  pre.store(tab, threadIdx.x);
  xinv_rows_pre<LNX, NTH>(smem, tab, tw, rows, pitch, pre, store);
}

}  // namespace demag
