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


// load(row, m) returns the raw (x[2m], x[2m+1]) of that row (zeros past its
// end) and scale(row, m, v) the value transformed, so that a round's loads
// can be issued one round ahead: round i + 1's loads are in flight while
// round i is transformed.  On return row r of smem holds X[0..L].  Ends with
// a workgroup barrier.
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
  float2 nxt[R];
#pragma unroll
  for (int j = 0; j < R; ++j) nxt[j] = sub < rows ? load(sub, t + T * j) : make_float2(0.f, 0.f);
  fill_stage_table<P, R>(tab, tw, tid, NTH);
  const float2 rbase = twiddle<false>(tw, t, ilog2(2 * P));
  __syncthreads();
  for (int start = 0; start < rows; start += RPR) {
    const int row = start + sub;
    const bool act = row < rows;
    float2* rb = smem + row * pitch;
    float2 u[R];
#pragma unroll
    for (int j = 0; j < R; ++j) u[j] = nxt[j];
    if (row + RPR < rows) {
#pragma unroll
      for (int j = 0; j < R; ++j) nxt[j] = load(row + RPR, t + T * j);
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
      for (int k = tid % (2 * T); k <= L / 2; k += 2 * T) {
        const float2 Uk = rb[k];
        const float2 Um = rb[(L - k) & (L - 1)];
        const float2 E = make_float2(0.5f * (Uk.x + Um.x), 0.5f * (Uk.y - Um.y));
        const float2 O = make_float2(0.5f * (Uk.y + Um.y), -0.5f * (Uk.x - Um.x));
        const float2 WO = cmul(O, twiddle<false>(tw, k, LNX));
        if (k == 0) {
          rb[0] = make_float2(E.x + O.x, E.y + O.y);
          rb[L] = make_float2(E.x - O.x, E.y - O.y);
        } else {
          rb[k] = cadd(E, WO);
          if (k != L - k) rb[L - k] = cconj(csub(E, WO));
        }
      }
    }
    __syncthreads();
  }
}

// The stage table of the x passes' Nx/4-point residue FFTs.
template <int LNX, int NTH>
__device__ __forceinline__ void fill_x_tables(float2* __restrict__ tab, const float2* __restrict__ tw, int tid) {
  constexpr int P = (1 << LNX) / 4;
  fill_stage_table<P, LineShape<P>::R>(tab, tw, tid, NTH);
}

// Rows of smem hold X[0..L]; store(row, m, (x[2m], x[2m+1])) receives the
// unnormalized inverse for m < NX/4.  Ends with a workgroup barrier.
// tables_ready: the caller filled the stage table earlier (fill_x_tables), so
// its latency overlapped other work.
template <int LNX, int NTH, bool TABLES_READY = false, typename Store>
__device__ __forceinline__ void xinv_rows(float2* __restrict__ smem, float2* __restrict__ tab,
                                          const float2* __restrict__ tw, int rows, int pitch, Store&& store) {
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
  if constexpr (!TABLES_READY) fill_stage_table<P, R>(tab, tw, tid, NTH);
  const float2 rbase = twiddle<false>(tw, t, ilog2(2 * P));
  __syncthreads();
  for (int start = 0; start < rows; start += RPR) {
    const int row = start + sub;
    const bool act = row < rows;
    float2* rb = smem + row * pitch;
    float2 u[R];
    if (act) {
      // U[k] = (X[k] + conj X[L-k]) + i W^-k (X[k] - conj X[L-k]): inverse of
      // the packed FFT of (x[2m], x[2m+1]), scaled to match X
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const int k = 2 * (t + T * j) + r;
        const float2 Xk = rb[k];
        const float2 Xm = rb[L - k];
        const float2 S = make_float2(Xk.x + Xm.x, Xk.y - Xm.y);
        const float2 D = make_float2(Xk.x - Xm.x, Xk.y + Xm.y);
        const float2 WD = cmul(D, twiddle<true>(tw, k, LNX));
        u[j] = make_float2(S.x - WD.y, S.y + WD.x);
      }
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

}  // namespace demag
