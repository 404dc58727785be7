// Field passes of H = -N * M by zero-padded FFT convolution (Sec. 7: 1D
// transforms along x, y, z, point-wise product with the transformed kernel,
// inverse transforms; Sec. 3 Eq. 4 and Table 1 for the sum itself).
//
//   k_fwd_xz : per (y rows, component): M = Ms m, real-to-complex FFT along x
//              (two-for-one packing), then the z FFT per kx; writes the
//              spectrum T[c][kz][tile][y][8].
//   k_mid    : per (kz, kx tile): y FFT of the three components, 3x3 product
//              with the real kernel spectrum (plus Parseval energy partials),
//              inverse y FFT, in place in T.
//   k_inv_zx : per (y rows, component): inverse z FFT keeping z < nz, then the
//              complex-to-real inverse along x keeping x < nx; stores H.
//
// Zero padding is never transformed: every padded axis of length N has at most
// N/2 non-zero inputs, so its FFT splits into the even and odd output residues,
// each an N/2-point FFT of the (pre-twiddled) non-zero half; the inverse keeps
// only the first N/2 outputs, which is the sum of the two residue inverses.
#include "fft_core.hpp"
#include "plan.hpp"
#include "xrows.hpp"
#include "reduce.hpp"

namespace demag {


// v[z] *= W_NZ^z (forward) or its conjugate, z < NZ/2, as compile-time constants.
template <int NZ, int Z, bool INV>
__device__ __forceinline__ void zodd_twiddle(float2 (&v)[NZ / 2]) {
  if constexpr (Z < NZ / 2) {
    v[Z] = tw_const<NZ, Z, INV>(v[Z]);
    zodd_twiddle<NZ, Z + 1, INV>(v);
  }
}

// ---------------------------------------------------------------------------
// forward: x real-to-complex + z
// ---------------------------------------------------------------------------
template <int LNX, int LNZ>
__global__ void __launch_bounds__(FWD_THREADS) __attribute__((amdgpu_waves_per_eu(LNX >= 12 || LNZ >= 6 ? 2 : 4, 8))) k_fwd_xz(FwdArgs a) {
  constexpr int NX = 1 << LNX;
  constexpr int NZ = 1 << LNZ;
  extern __shared__ float2 smem_base[];
  const int nyb = (a.ny + a.yg - 1) / a.yg;
  const int lg0 = xcd_logical(blockIdx.x, gridDim.x);
  const int b = lg0 / (3 * nyb);            // batch member
  const int lg = lg0 - b * 3 * nyb;
  if (a.moff) a.m += a.moff[b];
  if (a.ms_mesh) a.ms = a.ms_mesh[a.gid ? a.gid[b] : b];
  a.T += (size_t)b * a.Tb;
  const int c = lg / nyb;
  const int y0 = (lg - c * nyb) * a.yg;
  const int yg = min(a.yg, a.ny - y0);
  const int nz = a.nz, nx = a.nx, ny = a.ny;
  const int rows = yg * nz;
  const int tid = threadIdx.x;
  constexpr int L = (NX >= 4) ? NX / 2 : 1;   // packed complex length
  constexpr int PITCH = xrow_pitch<LNX>();    // LDS points per row
  float2* const tab = smem_base;
  float2* const smem = smem_base + xtab_points<LNX>();

  if constexpr (NX == 1) {
    for (int row = tid; row < rows; row += FWD_THREADS) {
      const int yl = row / nz, z = row - yl * nz;
      const size_t off = ((size_t)z * ny + (y0 + yl)) * nx;
      const float ms = a.Ms ? a.Ms[off] : a.ms;
      float v = a.m[(size_t)c * nz * ny * nx + off] * ms;
      if (a.m2) v = 0.5f * (v + a.ms2 * a.m2[(size_t)c * nz * ny * nx + off]);
      smem[row * PITCH] = make_float2(v, 0.f);
    }
  } else {
    const float* const mc = a.m + (size_t)c * nz * ny * nx;
    // row offsets of the mesh arrays
    auto roff = [&](int row) -> size_t {
      const int yl = row / nz, z = row - yl * nz;
      return ((size_t)z * ny + (y0 + yl)) * nx;
    };
    // loads read in-range memory for every m (indices past the row clamp to
    // its start); the scale step zeroes what lies past nx
    auto scale = [&](int row, int mm, float2 v) -> float2 {
      const int xi = 2 * mm;
      const bool in0 = xi < nx, in1 = xi + 1 < nx;
      if (a.m2) {
        // two sublattices: (ms m + ms2 m2) / 2, the second read here
        const float* src2 = a.m2 + (size_t)c * nz * ny * nx + roff(row);
        const float w0 = src2[in0 ? xi : 0], w1 = src2[in1 ? xi + 1 : 0];
        return make_float2(in0 ? 0.5f * (a.ms * v.x + a.ms2 * w0) : 0.f,
                           in1 ? 0.5f * (a.ms * v.y + a.ms2 * w1) : 0.f);
      }
      if (!a.Ms) return make_float2(in0 ? v.x * a.ms : 0.f, in1 ? v.y * a.ms : 0.f);
      const float* msr = a.Ms + roff(row);
      const float s0 = msr[in0 ? xi : 0], s1 = msr[in1 ? xi + 1 : 0];
      return make_float2(in0 ? v.x * s0 : 0.f, in1 ? v.y * s1 : 0.f);
    };
    if ((nx & 1) == 0 && !a.m2 && !a.Ms) {
      // the common case, branch-free: even rows start 8-byte aligned (one
      // 8-byte load per point), one saturation for the whole mesh
      const float ms = a.ms;
      xfwd_rows<LNX, FWD_THREADS>(smem, tab, a.tw, rows, PITCH, [&](int row, int mm) -> float2 {
        const float2* src = reinterpret_cast<const float2*>(mc + roff(row));
        return src[2 * mm < nx ? mm : 0];
      }, [&](int, int mm, float2 v) -> float2 {
        return 2 * mm < nx ? make_float2(v.x * ms, v.y * ms) : make_float2(0.f, 0.f);
      });
    } else {
      xfwd_rows<LNX, FWD_THREADS>(smem, tab, a.tw, rows, PITCH, [&](int row, int mm) -> float2 {
        const float* src = mc + roff(row);
        const int xi = 2 * mm;
        return make_float2(src[xi < nx ? xi : 0], src[xi + 1 < nx ? xi + 1 : 0]);
      }, scale);
    }
  }
  __syncthreads();

  // z transform per (y, kx) and store of the spectrum
  const int Kx = a.Kx;
  const int items = yg * Kx;
  const unsigned kzstride = (unsigned)a.nTiles * ny * TILE;   // float2 elements
  float2* const Tc = a.T + (size_t)c * NZ * kzstride;
  for (int it = tid; it < items; it += FWD_THREADS) {
    const int yl = it / Kx, kx = it - yl * Kx;
    const unsigned o = ((unsigned)(kx / TILE) * ny + (y0 + yl)) * TILE + (kx % TILE);
    if constexpr (NZ == 1) {
      if (a.ysplit) {
        // flattened rows: plane z = y' / ysplit of nzp per component
        const int yy = y0 + yl, zz = yy / a.ysplit, yr = yy - zz * a.ysplit;
        const size_t psz = (size_t)a.nTiles * a.ysplit * TILE;
        a.T[((size_t)c * a.nzp + zz) * psz + ((size_t)(kx / TILE) * a.ysplit + yr) * TILE + (kx % TILE)] =
            smem[(yl * nz) * PITCH + kx];
      } else {
        Tc[o] = smem[(yl * nz) * PITCH + kx];
      }
    } else {
      constexpr int Q = NZ / 2;
      // one residue in registers at a time, the column read from LDS once
      // per residue
      const float2* const col = smem + (yl * nz) * PITCH + kx;
      float2 v[Q];
#pragma unroll
      for (int z = 0; z < Q; ++z) v[z] = (z < nz) ? col[z * PITCH] : make_float2(0.f, 0.f);
      dft<Q, false>(v);
#pragma unroll
      for (int k = 0; k < Q; ++k) Tc[o + (unsigned)(2 * k) * kzstride] = v[k];
#pragma unroll
      for (int z = 0; z < Q; ++z) v[z] = (z < nz) ? col[z * PITCH] : make_float2(0.f, 0.f);
      zodd_twiddle<NZ, 0, false>(v);
      dft<Q, false>(v);
#pragma unroll
      for (int k = 0; k < Q; ++k) Tc[o + (unsigned)(2 * k + 1) * kzstride] = v[k];
    }
  }
}

// ---------------------------------------------------------------------------
// middle: y FFT, kernel product, inverse y FFT
// ---------------------------------------------------------------------------

__device__ __forceinline__ int kz_of(int i, int Nz) {
  // 0, Nz/2, 1, Nz-1, 2, Nz-2, ...: +-kz share kernel lines
  if (Nz == 1) return 0;
  if (i == 0) return 0;
  if (i == 1) return Nz / 2;
  const int p = (i - 2) / 2 + 1;
  return (i & 1) ? Nz - p : p;
}

// threads of the middle pass: two residue jobs per kx (one for a unit y
// length), each a group of LineShape<M>::T lanes, at least one wavefront
constexpr int mid_radix_of(int lny) { return line_radix(lny > 0 ? (1 << lny) / 2 : 1); }
// LDS points of the middle pass' odd-residue twiddle table (M entries, padded
// to 32 points so the data after it stays 256-byte aligned)
template <int M, int NRES>
constexpr int mid_rtab_points() { return NRES == 2 ? ((M + 31) / 32) * 32 : 0; }
constexpr int mid_threads(int lny, int kw, int r) { return mid_threads_rt(lny > 0 ? (1 << lny) / 2 : 1, kw, r); }


// MODE 0: y FFT, kernel product, inverse y FFT (the pipelined pass).
// MODE 1: y FFT only; spectra to S[c][kz][kx][ky] with ky ordered by residue
//         (r * NY/2 + k' for ky = 2k' + r).
// MODE 2: inverse y FFT only, from S.
// MODE 3: as MODE 0 with the Oersted kernel: H^ = i (P x J^), P the real
//         3-row spectrum (x even in ky and kz, y odd in ky, z odd in kz).
// R: points per lane of the M-point y lines (M / R lanes per line).
template <int LNY, int KW, bool ENERGY, int MODE = 0, int R = mid_radix_of(LNY)>
__global__ void __launch_bounds__(mid_threads(LNY, KW, R)) __attribute__((amdgpu_waves_per_eu(R >= 16 ? 2 : 4, 8)))
k_mid(MidArgs a) {
  constexpr int NY = 1 << LNY;
  constexpr int M = NY > 1 ? NY / 2 : 1;
  constexpr int NRES = NY > 1 ? 2 : 1;
  static_assert(mid_radix_ok(M, R), "unsupported radix for this line length");
  constexpr int T = M / R;
  constexpr int JOBS = NRES * KW;
  constexpr int NT = JOBS * T;
  __shared__ double red[16];
  extern __shared__ float2 smem_base[];
  float2* const tab = smem_base;
  float2* const rtab = smem_base + tab_points<M, R>();      // odd-residue twiddles W_2M^k, k < M
  float2* const smem = rtab + mid_rtab_points<M, NRES>();

  const int lg0 = xcd_logical(blockIdx.x, gridDim.x);
  const int bm = lg0 / a.nblk1;             // batch member
  const int lg = lg0 - bm * a.nblk1;
  a.T += (size_t)bm * a.Tb;
  if (ENERGY) a.epart += (size_t)bm * a.nblk1;
  const int halves = a.kw_halves;
  const int half = lg % halves;
  const int kzi = (lg / halves) % a.Nz;
  const int tile = lg / (halves * a.Nz);
  constexpr bool PROD = MODE == 0 || MODE == 3;   // kernel product in this pass
  constexpr int NKC = MODE == 3 ? 3 : 6;          // kernel rows per (kz, kx)
  const int kz = PROD ? kz_of(kzi, a.Nz) : kzi;
  const int ny = a.ny;

  const int tid = threadIdx.x;
  const bool lane_act = tid < NT;
  const int job = (T >= 64) ? __builtin_amdgcn_readfirstlane(tid / T) : tid / T;
  const int t = tid % T;
  // jobs r-major: the KW lines of residue 0, then those of residue 1, so
  // that the residue is uniform over a wavefront when KW T >= 64
  constexpr bool R_UNIFORM = (KW * T) % 64 == 0;
  const int w = job % KW;
  const int r = NRES == 1 ? 0 : (R_UNIFORM ? __builtin_amdgcn_readfirstlane(tid / (KW * T)) : job / KW);
  const int kx = tile * TILE + half * KW + w;
  const bool valid = lane_act && kx < a.Kx;
  if (tile * TILE + half * KW >= a.Kx) {    // nothing but padding columns
    if (ENERGY && tid == 0) a.epart[lg] = 0.0;
    return;
  }
  // staging of the three components' blocks: rows of KWP = KW + 1 points per
  // y (an odd pitch, so the lanes of a job, which read consecutive y, hit
  // distinct LDS banks)
  constexpr int KWP = KW + 1;
  constexpr int CST = M * KWP;              // component stride of the staging: M rows (zeros past ny)
  float2* stage = smem;                     // 3 components x M * KWP points
  float2* scr = smem + (size_t)job * lds_points<M, R>();   // per-job scratch (aliases stage)
  const size_t cstride = (size_t)a.Nz * a.nTiles * ny * TILE;
  float2* blk0 = a.T + ((size_t)kz * a.nTiles + tile) * ny * TILE + half * KW;

  // The kernel spectrum of this workgroup (KW consecutive kx lines of NKC rows
  // of KYP floats, contiguous in K[kz][kx][c][ky], plus their NKC KW Nyquist
  // entries) is requested with the components and held in registers through
  // the forward transforms, so its latency overlaps them; it moves to LDS
  // just before the product.  In LDS a row (pitch KLP) holds the even-ky
  // half, the Nyquist entry at KYP/2, and the odd-ky half from OH.
  constexpr int KYP = kernel_row_pitch(NY);
  constexpr int KLP = NRES == 2 ? KYP + 4 : KYP;
  constexpr int OH = KYP / 2 + 2;
  constexpr int NTHK = mid_threads(LNY, KW, R);
  constexpr int KF4 = KW * NKC * KYP / 4;         // float4 per workgroup block
  constexpr int KIT = PROD ? (KF4 + NTHK - 1) / NTHK : 1;
  const int kzf = (kz <= a.Nz / 2) ? kz : a.Nz - kz;
  const int kx0 = tile * TILE + half * KW;
  float4 kp[KIT];
  float knv = 0.f;
  float2 v[3][R];
  // S index of (c, kz, kx, residue r, k') in MODE 1 / 2
  auto sidx = [&](int c, int j) -> size_t {
    return (((size_t)c * a.Nz + kz) * a.Kx + kx) * NY + (size_t)r * M + (t + T * j);
  };
  if constexpr (MODE == 2) {
    // tables first, then the spectra (lanes of columns past Kx read S[0]: their
    // results land only in padding columns), then the tables to LDS
    TabRegs<M, R, NTHK, NRES == 2> tabs;
    tabs.load(a.tw, tid);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int j = 0; j < R; ++j) v[c][j] = a.S[valid ? sidx(c, j) : 0];
    tabs.store(tab, rtab, tid);
    __syncthreads();   // tables complete before any transform reads them
  } else {
    // the three components' blocks are loaded at once (16-byte copies, KW/2
    // float4 per y row of the half tile) and staged through LDS together,
    // so a workgroup waits for memory once
    constexpr int V = KW / 2;
    constexpr int NYMAX = NY > 1 ? NY / 2 : 1;
    constexpr int NTH = mid_threads(LNY, KW, R);
    constexpr int ITER = (NYMAX * V + NTH - 1) / NTH;
    const int nv = ny * V;
    // twiddle-table reads first, written to LDS once the bulk loads are issued
    TabRegs<M, R, NTHK, NRES == 2> tabr;
    tabr.load(a.tw, tid);
    float4 pre[3][ITER];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float4* b4 = reinterpret_cast<const float4*>(blk0 + c * cstride);
#pragma unroll
      for (int i = 0; i < ITER; ++i) {
        // unconditional (rows past ny read row 0 and are zeroed when staged),
        // so that the waits for these loads count exactly
        const int e = tid + i * NTH;
        const int y = e < nv ? e / V : 0, q = e < nv ? e - y * V : 0;
        pre[c][i] = b4[(unsigned)y * (TILE / 2) + q];
      }
    }
    // kernel rows after the components: the staging below waits only for the
    // components (memory counters retire in issue order) and the kernel rows
    // stay in flight through the forward transforms
    if constexpr (PROD) {
      const float4* Kb4 = reinterpret_cast<const float4*>(a.K + ((size_t)kzf * a.Kx + kx0) * NKC * KYP);
      // unconditional loads (rows past the block read its first float4,
      // which exists), so that no moves of a loaded value sit right behind
      // its load; entries out of range are dropped as they move to LDS
#pragma unroll
      for (int i = 0; i < KIT; ++i) {
        const int e = tid + i * NTHK;
        const bool in = e < KF4 && kx0 + e / (NKC * KYP / 4) < a.Kx;
        kp[i] = Kb4[in ? e : 0];
      }
      if constexpr (NY >= 4) {
        const bool in = tid < NKC * KW && kx0 + tid / NKC < a.Kx;
        knv = a.K[(size_t)NKC * a.Kzh * a.Kx * KYP + ((size_t)kzf * a.Kx + kx0) * NKC + (in ? tid : 0)];
      }
    }
    tabr.store(tab, rtab, tid);   // read by the transforms after the staging barrier
    // all M rows staged (rows past ny as zeros), so the reads
    // below need no bounds and their offsets are compile-time constants
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int i = 0; i < ITER; ++i) {
        const int e = tid + i * NTH;
        if ((NYMAX * V) % NTH == 0 || e < NYMAX * V) {
          const int y = e / V, q = e - y * V;
          float2* const d = stage + c * CST + y * KWP + 2 * q;
          const float4 p4 = e < nv ? pre[c][i] : make_float4(0.f, 0.f, 0.f, 0.f);
          d[0] = make_float2(p4.x, p4.y);
          d[1] = make_float2(p4.z, p4.w);
        }
      }
    }
    __syncthreads();
    {
      const float2* const src = stage + t * KWP + w;
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < R; ++j) v[c][j] = src[c * CST + T * j * KWP];
    }
    if constexpr (NRES == 2) {
      if (r) {
#pragma unroll
        for (int c = 0; c < 3; ++c) residue_twiddle_tab<R, T, false>(v[c], rtab, t);
      }
    }
    __syncthreads();
    if (lane_act) {
#pragma unroll
      for (int c = 0; c < 3; ++c) group_fft<M, R, false>(v[c], scr, t, tab);
    }
    if constexpr (MODE == 1) {
      if (valid) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int j = 0; j < R; ++j) a.S[sidx(c, j)] = v[c][j];
      }
      return;
    }
  }

  // point-wise product with the real kernel spectrum.  In LDS each kernel row
  // is split by the parity of ky (the parity of a job's folded ky is its
  // residue r), so the lanes of a job read consecutive words.
  float* const kl = reinterpret_cast<float*>(smem);   // aliases stage and FFT scratch
  // kernel rows odd in z (xz, yz; the Oersted P_z) change sign for kz > Nz/2:
  // folded in while the rows move to LDS
  constexpr unsigned ZODD = MODE == 3 ? 0x4u : 0x30u;
  const float sz = (kz <= a.Nz / 2) ? 1.f : -1.f;
  if constexpr (PROD) {
    __syncthreads();   // every job is done with its forward FFT scratch
#pragma unroll
    for (int i = 0; i < KIT; ++i) {
      const int e = tid + i * NTHK;
      if (e < KF4) {
        const int row = (4 * e) / KYP, ky0 = 4 * e - row * KYP;
        // sign of the rows odd in z, zero for kx lines past the spectrum
        const float f = kx0 + e / (NKC * KYP / 4) >= a.Kx ? 0.f : ((ZODD >> (row % NKC)) & 1u) ? sz : 1.f;
        float* const dst = kl + row * KLP;
        if constexpr (NRES == 2) {
          dst[ky0 / 2] = f * kp[i].x;
          dst[ky0 / 2 + 1] = f * kp[i].z;
          dst[OH + ky0 / 2] = f * kp[i].y;
          dst[OH + ky0 / 2 + 1] = f * kp[i].w;
        } else {
          *reinterpret_cast<float4*>(dst + ky0) = make_float4(f * kp[i].x, f * kp[i].y, f * kp[i].z, f * kp[i].w);
        }
      }
    }
    if (NY >= 4 && tid < NKC * KW)
      kl[tid * KLP + KYP / 2] = kx0 + tid / NKC >= a.Kx ? 0.f : ((ZODD >> (tid % NKC)) & 1u) ? sz * knv : knv;
    __syncthreads();
  }
  double e = 0.0;
  if (lane_act && PROD) {
    const float* const Kb = kl + w * NKC * KLP;
    const float wkx = (kx == 0 || 2 * kx == a.Nx) ? 1.f : 2.f;
    float ef = 0.f;
    // 3x3 product at one frequency: kernel entries k[0..NKC) read at row
    // offset ki of this line's NKC rows, sy the sign of the rows odd in y
    auto product = [&](int j, const float* kp0, float sy) __attribute__((always_inline)) {
      if constexpr (MODE == 3) {
        // H^ = i (P x J^), P real: i (a + i b) = -b + i a
        const float px = kp0[0 * KLP];
        const float py = sy * kp0[1 * KLP];
        const float pz = kp0[2 * KLP];
        const float2 jx = v[0][j], jy = v[1][j], jz = v[2][j];
        const float2 cx = make_float2(py * jz.x - pz * jy.x, py * jz.y - pz * jy.y);
        const float2 cy = make_float2(pz * jx.x - px * jz.x, pz * jx.y - px * jz.y);
        const float2 cz = make_float2(px * jy.x - py * jx.x, px * jy.y - py * jx.y);
        v[0][j] = make_float2(-cx.y, cx.x);
        v[1][j] = make_float2(-cy.y, cy.x);
        v[2][j] = make_float2(-cz.y, cz.x);
      } else {
        const float kxx = kp0[0 * KLP];
        const float kyy = kp0[1 * KLP];
        const float kzz = kp0[2 * KLP];
        const float kxy = sy * kp0[3 * KLP];
        const float kxz = kp0[4 * KLP];
        const float kyz = sy * kp0[5 * KLP];
        const float2 mx = v[0][j], my = v[1][j], mz = v[2][j];
        const float2 hx = make_float2(kxx * mx.x + kxy * my.x + kxz * mz.x, kxx * mx.y + kxy * my.y + kxz * mz.y);
        const float2 hy = make_float2(kxy * mx.x + kyy * my.x + kyz * mz.x, kxy * mx.y + kyy * my.y + kyz * mz.y);
        const float2 hz = make_float2(kxz * mx.x + kyz * my.x + kzz * mz.x, kxz * mx.y + kyz * my.y + kzz * mz.y);
        if constexpr (ENERGY)
          ef += mx.x * hx.x + mx.y * hx.y + my.x * hy.x + my.y * hy.y + mz.x * hz.x + mz.y * hz.y;
        v[0][j] = hx; v[1][j] = hy; v[2][j] = hz;
      }
    };
    if constexpr (NRES == 2 && NY >= 8) {
      // ky = 2u + r with u = t + T j.  For j < R/2, ky < NY/2: folded
      // ky = ky, row index u in the residue's half.  For j >= R/2 the
      // frequency folds to NY - ky, row index M - u - r, sign -1 for the rows
      // odd in y (at ky = NY/2, reached by t = r = 0, j = R/2, those rows are
      // zero, so the sign does not matter there).  Both indices are affine in
      // t with compile-time offsets per j.
      const float* const plo = Kb + (r ? OH : 0) + t;
      const float* const phi = Kb + (r ? OH : 0) + M - r - t;
#pragma unroll
      for (int j = 0; j < R; ++j) {
        if (j < R / 2) product(j, plo + T * j, 1.f);
        else product(j, phi - T * j, -1.f);
      }
    } else {
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const int ky = NRES * (t + T * j) + r;
        const bool lo = 2 * ky <= NY;
        const int kyf = lo ? ky : NY - ky;
        // index in the LDS row: even/odd half by the residue, the Nyquist
        // entry at KYP/2
        int ki = NRES == 2 ? (r ? OH : 0) + (kyf >> 1) : kyf;
        if constexpr (NY == 4) ki = kyf == 2 ? KYP / 2 : ki;
        product(j, Kb + ki, lo ? 1.f : -1.f);
      }
    }
    if (ENERGY && valid) e = (double)(wkx * ef);
  }
  if constexpr (PROD) __syncthreads();   // kernel rows read before the scratch is reused
  if (lane_act) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      group_fft<M, R, true>(v[c], scr, t, tab);
    }
    if constexpr (NRES == 2) {
      if (r) {
#pragma unroll
        for (int c = 0; c < 3; ++c) residue_twiddle_tab<R, T, true>(v[c], rtab, t);
      }
    }
  }

  // sum the two residues of the three components in LDS and store
  __syncthreads();
  float2* const dstg = stage + t * KWP + w;   // row y = t + T j of this lane's line
  if (lane_act && r == NRES - 1) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int j = 0; j < R; ++j) dstg[c * CST + T * j * KWP] = v[c][j];
  }
  __syncthreads();
  if constexpr (NRES == 2) {
    if (lane_act && r == 0) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < R; ++j) dstg[c * CST + T * j * KWP] = cadd(dstg[c * CST + T * j * KWP], v[c][j]);
    }
    __syncthreads();
  }
  {
    constexpr int V = KW / 2;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float4* b4 = reinterpret_cast<float4*>(blk0 + c * cstride);
      for (int q = tid; q < ny * V; q += blockDim.x) {
        const int y = q / V, s2 = q - y * V;
        const float2* const src = stage + c * CST + y * KWP + 2 * s2;
        const float2 lo = src[0], hi = src[1];
        b4[(unsigned)y * (TILE / 2) + s2] = make_float4(lo.x, lo.y, hi.x, hi.y);
      }
    }
  }
  if constexpr (ENERGY) {
    const double s = block_sum(e, red);
    if (tid == 0) a.epart[lg] = s;
  }
}

// ---------------------------------------------------------------------------
// inverse: z + x complex-to-real
// ---------------------------------------------------------------------------
template <int LNX, int LNZ>
__global__ void __launch_bounds__(INV_THREADS) __attribute__((amdgpu_waves_per_eu(LNX >= 12 || LNZ >= 6 ? 2 : 4, 8))) k_inv_zx(InvArgs a) {
  constexpr int NX = 1 << LNX;
  constexpr int NZ = 1 << LNZ;
  extern __shared__ float2 smem_base[];
  const int nyb = (a.ny + a.yg - 1) / a.yg;
  const int lg0 = xcd_logical(blockIdx.x, gridDim.x);
  const int b = lg0 / (3 * nyb);            // batch member
  const int lg = lg0 - b * 3 * nyb;
  if (a.moff) {
    a.H += a.moff[b];
    if (a.aux) a.aux += a.moff[b];
  }
  if (a.ms_mesh) a.ms = a.ms_mesh[a.gid ? a.gid[b] : b];
  if (a.beta_ptr && a.gid) a.beta_ptr += a.gid[b];
  a.T += (size_t)b * a.Tb;
  const int c = lg / nyb;
  const int y0 = (lg - c * nyb) * a.yg;
  const int yg = min(a.yg, a.ny - y0);
  const int nz = a.nz, nx = a.nx, ny = a.ny;
  const int rows = yg * nz;
  const int tid = threadIdx.x;
  constexpr int L = (NX >= 4) ? NX / 2 : 1;
  constexpr int PITCH = xrow_pitch<LNX>();
  const int Kx = a.Kx;
  float2* const tab = smem_base;
  float2* const smem = smem_base + xtab_points<LNX>();

  // the x transform's twiddle tables first, so that their reads overlap the
  // z phase (stored to LDS after it)
  XTabPre<(NX >= 4 ? LNX : 2), INV_THREADS> xpre;
  if constexpr (NX >= 4) xpre.load(a.tw, tid);
  // inverse z per (y, kx), keeping z < nz: the even kz residue, then the
  // odd one added through LDS (one residue live at a time)
  const int items = yg * Kx;
  const unsigned kzstride = (unsigned)a.nTiles * ny * TILE;
  const float2* const Tc = a.T + (size_t)c * NZ * kzstride;
  for (int it = tid; it < items; it += INV_THREADS) {
    const int yl = it / Kx, kx = it - yl * Kx;
    const unsigned o = ((unsigned)(kx / TILE) * ny + (y0 + yl)) * TILE + (kx % TILE);
    float2* const d0 = &smem[(yl * nz) * PITCH + kx];
    if constexpr (NZ == 1) {
      if (a.ysplit) {
        const int yy = y0 + yl, zz = yy / a.ysplit, yr = yy - zz * a.ysplit;
        const size_t psz = (size_t)a.nTiles * a.ysplit * TILE;
        d0[0] = a.T[((size_t)c * a.nzp + zz) * psz + ((size_t)(kx / TILE) * a.ysplit + yr) * TILE + (kx % TILE)];
      } else {
        d0[0] = Tc[o];
      }
    } else {
      constexpr int Q = NZ / 2;
      // both residues requested before either is transformed (one at a time
      // for the longest lines, whose two residues would not fit in registers)
      constexpr int QW = NZ >= 128 ? 1 : Q;
      float2 v[Q], w[QW];
      // residue loads of the longest lines go in chunks of 16, so that few
      // addresses are live at once
      auto load_res = [&](int par) __attribute__((always_inline)) {
        constexpr int CH = Q > 16 ? 16 : Q;
#pragma unroll
        for (int k0 = 0; k0 < Q; k0 += CH) {
#pragma unroll
          for (int k = k0; k < k0 + CH; ++k) v[k] = Tc[o + (unsigned)(2 * k + par) * kzstride];
          if constexpr (NZ >= 128) asm volatile("" ::: "memory");
        }
      };
      load_res(0);
      if constexpr (NZ < 128) {
#pragma unroll
        for (int k = 0; k < Q; ++k) w[k] = Tc[o + (unsigned)(2 * k + 1) * kzstride];
      }
      dft<Q, true>(v);
#pragma unroll
      for (int z = 0; z < Q; ++z)
        if (z < nz) d0[z * PITCH] = v[z];
      if constexpr (NZ < 128) {
#pragma unroll
        for (int k = 0; k < Q; ++k) v[k] = w[k];
      } else {
        load_res(1);
      }
      dft<Q, true>(v);
      zodd_twiddle<NZ, 0, true>(v);
#pragma unroll
      for (int z = 0; z < Q; ++z)
        if (z < nz) d0[z * PITCH] = cadd(d0[z * PITCH], v[z]);
    }
  }
  __syncthreads();

  const size_t cbase = (size_t)c * nz * ny * nx;
  if constexpr (NX == 1) {
    for (int row = tid; row < rows; row += INV_THREADS) {
      const int yl = row / nz, z = row - yl * nz;
      const size_t off = ((size_t)z * ny + (y0 + yl)) * nx;
      float val = smem[row * PITCH].x;
      if (a.scale_out) {
        const float s = a.Ms ? a.Ms[off] : a.ms;
        val = s * (val + (a.beta_ptr ? (float)(a.beta_scale * *a.beta_ptr) * a.aux[cbase + off] : 0.f));
      }
      float* dst = a.H + cbase + off;
      dst[0] = a.accumulate ? dst[0] + val : val;
    }
  } else {
    const float beta = (a.scale_out && a.beta_ptr) ? (float)(a.beta_scale * *a.beta_ptr) : 0.f;
    xpre.store(tab, tid);
    xinv_rows_pre<LNX, INV_THREADS>(smem, tab, a.tw, rows, PITCH, xpre, [&](int row, int mm, float2 uu) {
      const int yl = row / nz, z = row - yl * nz;
      const size_t off = ((size_t)z * ny + (y0 + yl)) * nx;
      float* dst = a.H + cbase + off;
      const int xi = 2 * mm;
      // reads at clamped (in-range) indices, not under the bounds tests, so
      // that they are not waited for one by one
      const bool in0 = xi < nx, in1 = xi + 1 < nx;
      const int x0 = in0 ? xi : 0, x1 = in1 ? xi + 1 : 0;
      float v0 = uu.x, v1 = uu.y;
      if (a.scale_out) {
        if (a.beta_ptr) {
          const float* aux = a.aux + cbase + off;
          v0 += beta * aux[x0];
          v1 += beta * aux[x1];
        }
        const float s0 = a.Ms ? a.Ms[off + x0] : a.ms, s1 = a.Ms ? a.Ms[off + x1] : a.ms;
        v0 *= s0;
        v1 *= s1;
      }
      if (a.accumulate) {
        v0 += dst[x0];
        v1 += dst[x1];
      }
      if (in0) dst[xi] = v0;
      if (in1) dst[xi + 1] = v1;
    });
  }
}

// ---------------------------------------------------------------------------
// energy reductions
// ---------------------------------------------------------------------------
// Sum of the middle pass' Parseval partials in a fixed order:
// E = scale * sum(partials), scale = -(mu0/2) V.
// One workgroup per batch member; out index gid[member] (or the member).
__global__ void __launch_bounds__(FINAL_THREADS) k_energy_final(const double* part, int n, double scale,
                                                                double* out, const int* gid) {
  __shared__ double red[FINAL_THREADS / 64];
  const int b = blockIdx.x;
  part += (size_t)b * n;
  // eight partials per thread and sweep, all read before any is added (one
  // memory round trip up to 8 FINAL_THREADS partials); each thread adds its
  // partials in increasing order, entries past n read entry 0 and add nothing
  constexpr int U = 8;
  double acc = 0.0;
  for (int i0 = threadIdx.x; i0 < n; i0 += U * FINAL_THREADS) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = part[i0 + u * FINAL_THREADS < n ? i0 + u * FINAL_THREADS : 0];
#pragma unroll
    for (int u = 0; u < U; ++u) acc += i0 + u * FINAL_THREADS < n ? v[u] : 0.0;
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) out[gid ? gid[b] : b] = scale * s;
}

// Per-workgroup partials of sum_c Ms m_c H_c over the cells.
__global__ void __launch_bounds__(RED_THREADS) k_energy_cells(const float* m, const float* Ms, float ms,
                                                              const float* H, size_t ncell, double* part) {
  __shared__ double red[RED_THREADS / 64];
  double s = 0.0;
  for (size_t i = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; i < ncell; i += (size_t)gridDim.x * RED_THREADS) {
    const float msv = Ms ? Ms[i] : ms;
    const float d = m[i] * H[i] + m[ncell + i] * H[ncell + i] + m[2 * ncell + i] * H[2 * ncell + i];
    s += (double)(msv * d);
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

}  // namespace demag

// ---------------------------------------------------------------------------
// host-side launchers (compile-time FFT lengths dispatched from the plan)
// ---------------------------------------------------------------------------
#include "launch.hpp"

namespace demag {

static size_t xpass_lds(const Geom& g) {
  return (size_t)g.yg * g.nz * xrow_pitch_rt(g.lnx) * sizeof(float2);
}

template <typename K>
static hipError_t prep_lds(K kern, size_t lds) {
  if (lds > 65536)
    return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return hipSuccess;
}

template <int LNX, int LNZ>
static hipError_t fwd_one(const Geom& g, const FwdArgs& a, hipStream_t s) {
  const size_t lds = xpass_lds(g) + xtab_points<LNX>() * sizeof(float2);
  hipError_t e = prep_lds(k_fwd_xz<LNX, LNZ>, lds);
  if (e != hipSuccess) return e;
  dim3 grid(((g.ny + g.yg - 1) / g.yg) * 3 * a.nb);
  hipLaunchKernelGGL((k_fwd_xz<LNX, LNZ>), grid, dim3(FWD_THREADS), lds, s, a);
  return hipGetLastError();
}

template <int LNX, int LNZ>
static hipError_t inv_one(const Geom& g, const InvArgs& a, hipStream_t s) {
  const size_t lds = xpass_lds(g) + xtab_points<LNX>() * sizeof(float2);
  hipError_t e = prep_lds(k_inv_zx<LNX, LNZ>, lds);
  if (e != hipSuccess) return e;
  dim3 grid(((g.ny + g.yg - 1) / g.yg) * 3 * a.nb);
  hipLaunchKernelGGL((k_inv_zx<LNX, LNZ>), grid, dim3(INV_THREADS), lds, s, a);
  return hipGetLastError();
}

// Nz = 64 (17 <= nz <= 32) only for Nx <= 1024 and Nz = 128 (33 <= nz <= 64)
// only for Nx <= 512: longer rows do not leave room for that many of them in
// LDS (the plan rejects those sizes first)
#define DEMAG_Z_SWITCH(FN, LNX, ...)                      \
  switch (g.lnz) {                                        \
    case 0: return FN<LNX, 0>(__VA_ARGS__);               \
    case 2: return FN<LNX, 2>(__VA_ARGS__);               \
    case 3: return FN<LNX, 3>(__VA_ARGS__);               \
    case 4: return FN<LNX, 4>(__VA_ARGS__);               \
    case 5: return FN<LNX, 5>(__VA_ARGS__);               \
    case 6:                                               \
      if constexpr (LNX <= 10) return FN<LNX, 6>(__VA_ARGS__); \
      else return hipErrorInvalidValue;                   \
    case 7:                                               \
      if constexpr (LNX <= 9) return FN<LNX, 7>(__VA_ARGS__); \
      else return hipErrorInvalidValue;                   \
    default: return hipErrorInvalidValue;                 \
  }

template <int LNX>
static hipError_t fwd_z(const Geom& g, const FwdArgs& a, hipStream_t s) { DEMAG_Z_SWITCH(fwd_one, LNX, g, a, s) }
template <int LNX>
static hipError_t inv_z(const Geom& g, const InvArgs& a, hipStream_t s) { DEMAG_Z_SWITCH(inv_one, LNX, g, a, s) }

#define DEMAG_X_SWITCH(FN, ...)                           \
  switch (g.lnx) {                                        \
    case 0: return FN<0>(__VA_ARGS__);                    \
    case 2: return FN<2>(__VA_ARGS__);                    \
    case 3: return FN<3>(__VA_ARGS__);                    \
    case 4: return FN<4>(__VA_ARGS__);                    \
    case 5: return FN<5>(__VA_ARGS__);                    \
    case 6: return FN<6>(__VA_ARGS__);                    \
    case 7: return FN<7>(__VA_ARGS__);                    \
    case 8: return FN<8>(__VA_ARGS__);                    \
    case 9: return FN<9>(__VA_ARGS__);                    \
    case 10: return FN<10>(__VA_ARGS__);                  \
    case 11: return FN<11>(__VA_ARGS__);                  \
    case 12: return FN<12>(__VA_ARGS__);                  \
    default: return hipErrorInvalidValue;                 \
  }

hipError_t launch_fwd(const Geom& g, const FwdArgs& a, hipStream_t s) { DEMAG_X_SWITCH(fwd_z, g, a, s) }
hipError_t launch_inv(const Geom& g, const InvArgs& a, hipStream_t s) { DEMAG_X_SWITCH(inv_z, g, a, s) }

int mid_kw(const Geom& g) {
  if (g.mid_kw == 2 || g.mid_kw == 4 || g.mid_kw == 8) return g.mid_kw;
  return 4;
}

int mid_radix(const Geom& g) {
  const int M = g.Ny > 1 ? g.Ny / 2 : 1;
  return (g.mid_r > 0 && mid_radix_ok(M, g.mid_r)) ? g.mid_r : line_radix(M);
}

int mid_blocks(const Geom& g) { return g.nTiles * (TILE / mid_kw(g)) * g.Nz; }
int mid_blocks_max(const Geom& g) { return g.nTiles * (TILE / 2) * g.Nz; }

template <int LNY, int KW, bool ENERGY, int MODE, int R>
static hipError_t mid_launch(const Geom& g, const MidArgs& a, hipStream_t s) {
  constexpr int NY = 1 << LNY;
  constexpr int M = NY > 1 ? NY / 2 : 1;
  constexpr int NRES = NY > 1 ? 2 : 1;
  size_t lds = (size_t)NRES * KW * lds_points<M, R>() * sizeof(float2);
  const size_t st = (size_t)3 * M * (KW + 1) * sizeof(float2);   // staging of the three components
  if (st > lds) lds = st;
  const size_t klp = NRES == 2 ? kernel_row_pitch(NY) + 4 : kernel_row_pitch(NY);
  const size_t kr = (MODE == 0 || MODE == 3) ? (size_t)KW * (MODE == 3 ? 3 : 6) * klp * sizeof(float) : 0;
  if (kr > lds) lds = kr;
  lds += (tab_points<M, R>() + mid_rtab_points<M, NRES>()) * sizeof(float2);
  hipError_t e = prep_lds(k_mid<LNY, KW, ENERGY, MODE, R>, lds);
  if (e != hipSuccess) return e;
  const int blocks = g.nTiles * (TILE / KW) * g.Nz;
  hipLaunchKernelGGL((k_mid<LNY, KW, ENERGY, MODE, R>), dim3(blocks * a.nb), dim3(mid_threads(LNY, KW, R)), lds, s,
                     a);
  return hipGetLastError();
}

// mode 0: the pipelined pass (energy partials when a.epart is set);
// 1 / 2: the split y passes of coupled layers; 3: the pipelined pass with the
// Oersted kernel
template <int LNY, int KW, int R>
static hipError_t mid_mode(const Geom& g, const MidArgs& a, int mode, hipStream_t s) {
  if constexpr (!mid_schedule_ok(LNY > 0 ? (1 << LNY) / 2 : 1, KW, R)) {
    return hipErrorInvalidConfiguration;   // not offered (rejected by the plan before launch)
  } else {
  if (mode == 1) return mid_launch<LNY, KW, false, 1, R>(g, a, s);
  if (mode == 2) return mid_launch<LNY, KW, false, 2, R>(g, a, s);
  if (mode == 3) return mid_launch<LNY, KW, false, 3, R>(g, a, s);
  return a.epart ? mid_launch<LNY, KW, true, 0, R>(g, a, s) : mid_launch<LNY, KW, false, 0, R>(g, a, s);
  }
}

template <int LNY, int KW>
static hipError_t mid_radix_switch(const Geom& g, const MidArgs& a, int mode, hipStream_t s) {
  constexpr int M = LNY > 0 ? (1 << LNY) / 2 : 1;
  constexpr int R0 = line_radix(M);
  const int r = mid_radix(g);
  if constexpr (mid_radix_ok(M, 4) && R0 != 4)
    if (r == 4) return mid_mode<LNY, KW, 4>(g, a, mode, s);
  if constexpr (mid_radix_ok(M, 8) && R0 != 8)
    if (r == 8) return mid_mode<LNY, KW, 8>(g, a, mode, s);
  if constexpr (mid_radix_ok(M, 16) && R0 != 16)
    if (r == 16) return mid_mode<LNY, KW, 16>(g, a, mode, s);
  return mid_mode<LNY, KW, R0>(g, a, mode, s);
}

template <int LNY>
static hipError_t mid_kw_switch(const Geom& g, const MidArgs& a, int mode, hipStream_t s) {
  switch (mid_kw(g)) {
    case 2: return mid_radix_switch<LNY, 2>(g, a, mode, s);
    case 8: return mid_radix_switch<LNY, 8>(g, a, mode, s);
    default: return mid_radix_switch<LNY, 4>(g, a, mode, s);
  }
}

static hipError_t mid_dispatch(const Geom& g, const MidArgs& a, int mode, hipStream_t s) {
  switch (g.lny) {
    case 0: return mid_kw_switch<0>(g, a, mode, s);
    case 2: return mid_kw_switch<2>(g, a, mode, s);
    case 3: return mid_kw_switch<3>(g, a, mode, s);
    case 4: return mid_kw_switch<4>(g, a, mode, s);
    case 5: return mid_kw_switch<5>(g, a, mode, s);
    case 6: return mid_kw_switch<6>(g, a, mode, s);
    case 7: return mid_kw_switch<7>(g, a, mode, s);
    case 8: return mid_kw_switch<8>(g, a, mode, s);
    case 9: return mid_kw_switch<9>(g, a, mode, s);
    case 10: return mid_kw_switch<10>(g, a, mode, s);
    case 11: return mid_kw_switch<11>(g, a, mode, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_mid(const Geom& g, const MidArgs& a, hipStream_t s) {
  return mid_dispatch(g, a, g.kind == KERNEL_OERSTED ? 3 : 0, s);
}

// y passes without the kernel product (coupled layers): mode 1 forward into
// S, mode 2 inverse from S
hipError_t launch_mid_split(const Geom& g, const MidArgs& a, int mode, hipStream_t s) {
  return mid_dispatch(g, a, mode, s);
}

hipError_t launch_energy_final(const double* part, int n, double scale, double* out, hipStream_t s, int nb,
                               const int* gid) {
  hipLaunchKernelGGL(k_energy_final, dim3(nb), dim3(FINAL_THREADS), 0, s, part, n, scale, out, gid);
  return hipGetLastError();
}

int energy_cell_blocks(size_t ncell) {
  size_t b = (ncell + RED_THREADS - 1) / RED_THREADS;
  return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

hipError_t launch_energy_cells(const float* m, const float* Ms, float ms, const float* H, size_t ncell,
                               double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_energy_cells, dim3(energy_cell_blocks(ncell)), dim3(RED_THREADS), 0, s, m, Ms, ms, H,
                     ncell, part);
  return hipGetLastError();
}

}  // namespace demag
