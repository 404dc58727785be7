// Set-up of the kernel spectrum (once per geometry), all in FP64.
//
//  k_tensor   : cell-averaged demagnetizing tensor N(r) at the non-negative
//               lattice offsets (Sec. 3, Eq. 4; Table 1 demagnetizing field,
//               formulas of Newell et al.).  Near the source (|r| < 3 h_max)
//               the Newell closed form; farther out Gauss-Legendre quadrature
//               of the point-dipole kernel against the tent weight
//               prod_a (h_a - |u_a|), the exact overlap of two cells.
//  k_axis     : the transform of the zero-padded, wrapped tensor along one
//               axis.  Each component is even or odd along each axis, so the
//               DFT of the wrapped line is real up to a factor -i per odd axis:
//               even: N(0) + 2 sum_{i>0} N(i) cos(2 pi i k / Npad)
//               odd : -i * 2 sum_{i>0} N(i) sin(2 pi i k / Npad)
//               kept for 0 <= k <= Npad/2 (the rest follows by symmetry).
//  k_pack     : scale by -s/(Nx Ny Nz) (s = -1 for off-diagonal components,
//               from (-i)^2) and store FP32 in the layout read by the middle
//               pass, K[kz][kx][component][ky].
//
// The Oersted kernel (Table 1, Oersted row; Sec. 4) takes the same route with
// three components: g(d), the field of a cuboid cell of unit current density
// averaged over the target cell at offset d (H = 1/(4 pi) J x g), built by
// k_oe_far (then, with periodic axes, summed over the images like the
// tensor) and k_oe_near (|d| < 3 h_max); g_a is odd along axis a only, so
// its spectrum is -i times a real octant, packed as 1/(4 pi Nx Ny Nz) times
// that real part.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <climits>
#include <cmath>
#include "plan.hpp"

namespace demag {


__device__ double nf(double x, double y, double z) {
  const double x2 = x * x, y2 = y * y, z2 = z * z;
  const double R = sqrt(x2 + y2 + z2);
  double s = (2.0 * x2 - y2 - z2) * R / 6.0;
  const double rxz = sqrt(x2 + z2), rxy = sqrt(x2 + y2);
  if (y != 0.0 && rxz > 0.0) s += 0.5 * y * (z2 - x2) * asinh(y / rxz);
  if (z != 0.0 && rxy > 0.0) s += 0.5 * z * (y2 - x2) * asinh(z / rxy);
  if (x != 0.0 && y != 0.0 && z != 0.0) s -= x * y * z * atan(y * z / (x * R));
  return s;
}

__device__ double ng(double x, double y, double z) {
  const double x2 = x * x, y2 = y * y, z2 = z * z;
  const double R = sqrt(x2 + y2 + z2);
  const double rxy = sqrt(x2 + y2), ryz = sqrt(y2 + z2), rxz = sqrt(x2 + z2);
  double s = -x * y * R / 3.0;
  if (x != 0.0 && y != 0.0 && z != 0.0) s += x * y * z * asinh(z / rxy);
  if (y != 0.0 && x != 0.0) s += y / 6.0 * (3.0 * z2 - y2) * asinh(x / ryz);
  if (x != 0.0 && y != 0.0) s += x / 6.0 * (3.0 * z2 - x2) * asinh(y / rxz);
  if (z != 0.0 && x != 0.0 && y != 0.0) {
    s -= z * z2 / 6.0 * atan(x * y / (z * R));
    s -= z * y2 / 2.0 * atan(x * z / (y * R));
    s -= z * x2 / 2.0 * atan(y * z / (x * R));
  }
  return s;
}

// second difference over the 27 points (X + i a, Y + j b, Z + k c), weights
// 2 (centre) and -1 (sides) per axis, over 4 pi a b c
template <bool OFFDIAG>
__device__ double stencil27(double X, double Y, double Z, double a, double b, double c) {
  double acc = 0.0;
  for (int i = -1; i <= 1; ++i) {
    const double wi = i == 0 ? 2.0 : -1.0;
    for (int j = -1; j <= 1; ++j) {
      const double wj = j == 0 ? 2.0 : -1.0;
      for (int k = -1; k <= 1; ++k) {
        const double wk = k == 0 ? 2.0 : -1.0;
        const double px = X + i * a, py = Y + j * b, pz = Z + k * c;
        acc += wi * wj * wk * (OFFDIAG ? ng(px, py, pz) : nf(px, py, pz));
      }
    }
  }
  return acc / (4.0 * M_PI * a * b * c);
}

// N at one offset (X, Y, Z): closed form within 3 h_max, Gauss-Legendre
// quadrature of the tent-weighted dipole kernel beyond (order by distance).
__device__ void tensor_point(double X, double Y, double Z, double dx, double dy, double dz, const GLTable& gl,
                             double (&N)[6]) {
  const double hmax = fmax(dx, fmax(dy, dz));
  const double dist = sqrt(X * X + Y * Y + Z * Z) / hmax;
  if (dist < 3.0) {
    N[0] = stencil27<false>(X, Y, Z, dx, dy, dz);
    N[1] = stencil27<false>(Y, X, Z, dy, dx, dz);
    N[2] = stencil27<false>(Z, Y, X, dz, dy, dx);
    N[3] = stencil27<true>(X, Y, Z, dx, dy, dz);
    N[4] = stencil27<true>(X, Z, Y, dx, dz, dy);
    N[5] = stencil27<true>(Y, Z, X, dy, dz, dx);
    return;
  }
  const int b = dist < 6.0 ? 0 : dist < 16.0 ? 1 : dist < 40.0 ? 2 : 3;
  const int n = gl.n[b];
  for (int q = 0; q < 6; ++q) N[q] = 0.0;
  for (int ax = 0; ax < 2 * n; ++ax) {
    const double ux = (ax < n ? 1.0 : -1.0) * gl.u[b][ax % n] * dx;
    const double wx = gl.w[b][ax % n] * dx * (dx - fabs(ux));
    const double vx = X + ux;
    for (int ay = 0; ay < 2 * n; ++ay) {
      const double uy = (ay < n ? 1.0 : -1.0) * gl.u[b][ay % n] * dy;
      const double wy = gl.w[b][ay % n] * dy * (dy - fabs(uy));
      const double vy = Y + uy;
      for (int az = 0; az < 2 * n; ++az) {
        const double uz = (az < n ? 1.0 : -1.0) * gl.u[b][az % n] * dz;
        const double wz = gl.w[b][az % n] * dz * (dz - fabs(uz));
        const double vz = Z + uz;
        const double r2 = vx * vx + vy * vy + vz * vz;
        const double wt = wx * wy * wz / (r2 * r2 * sqrt(r2));
        N[0] += wt * (r2 - 3.0 * vx * vx);
        N[1] += wt * (r2 - 3.0 * vy * vy);
        N[2] += wt * (r2 - 3.0 * vz * vz);
        N[3] -= wt * 3.0 * vx * vy;
        N[4] -= wt * 3.0 * vx * vz;
        N[5] -= wt * 3.0 * vy * vz;
      }
    }
  }
  const double s = 1.0 / (4.0 * M_PI * dx * dy * dz);
  for (int q = 0; q < 6; ++q) N[q] *= s;
}

// Octant of the tensor, out[c][k][j][i] = N at (i dx, j dy, k dz).  Periodic
// axes (multiple images, Sec. 3): the sum of N over the shifts
// (kx Lx, ky Ly, kz Lz), |k_a| <= K_a, with L_a = n_a h_a and K_a = images on
// a periodic axis, 0 otherwise.
__global__ void k_tensor(double* __restrict__ out, int nx, int ny, int nz, double dx, double dy, double dz,
                         GLTable gl, int Kx, int Ky, int Kz) {
  const size_t cnt = (size_t)nx * ny * nz;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= cnt) return;
  const int i = (int)(idx % nx);
  const int j = (int)((idx / nx) % ny);
  const int k = (int)(idx / ((size_t)nx * ny));
  const double X = i * dx, Y = j * dy, Z = k * dz;
  const double Lx = nx * dx, Ly = ny * dy, Lz = nz * dz;
  double S[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int a = -Kx; a <= Kx; ++a)
    for (int b = -Ky; b <= Ky; ++b)
      for (int c = -Kz; c <= Kz; ++c) {
        double N[6];
        tensor_point(X + a * Lx, Y + b * Ly, Z + c * Lz, dx, dy, dz, gl, N);
        for (int q = 0; q < 6; ++q) S[q] += N[q];
      }
  for (int q = 0; q < 6; ++q) out[q * cnt + idx] = S[q];
}

// ---------------------------------------------------------------------------
// Oersted kernel g(d) = 1/V int_target int_source (r - r') / |r - r'|^3
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool oe_near(double X, double Y, double Z, double hmax) {
  return sqrt(X * X + Y * Y + Z * Z) / hmax < 3.0;
}

// Q(X, Y, Z) = int_0^X f(s, Y, Z) ds with Newell's f (even in s, so Q is odd
// in X): the rule (qs, qw) on [0, 1], panels that halve towards s = 0, where
// f's only non-analytic point on the path lies.  d/dX d^2/dY^2 d^2/dZ^2 Q = 1/R.
__device__ double q_path(double X, double Y, double Z, const double* __restrict__ qs,
                         const double* __restrict__ qw, int nq) {
  const double ax = fabs(X);
  if (ax == 0.0) return 0.0;
  double acc = 0.0;
  for (int i = 0; i < nq; ++i) acc += qw[i] * nf(ax * qs[i], Y, Z);
  return (X < 0.0 ? -ax : ax) * acc;
}

// weight of stencil point p (0..26) and its offsets along the three axes
__device__ __forceinline__ double oe_stencil(int p, int& di, int& dj, int& dk) {
  di = p % 3 - 1;
  dj = (p / 3) % 3 - 1;
  dk = p / 9 - 1;
  return (di ? 1.0 : -2.0) * (dj ? 1.0 : -2.0) * (dk ? 1.0 : -2.0);
}

// term p of component c at offset (X, Y, Z): (A, B, C) is the offset taken
// along (c, then the other two axes), f being symmetric in its last two
__device__ double oe_term(int c, int p, double X, double Y, double Z, double dx, double dy, double dz,
                          const double* __restrict__ qs, const double* __restrict__ qw, int nq) {
  int di, dj, dk;
  const double w = oe_stencil(p, di, dj, dk);
  const double A = c == 0 ? X : c == 1 ? Y : Z, ha = c == 0 ? dx : c == 1 ? dy : dz;
  const double B = c == 0 ? Y : X, hb = c == 0 ? dy : dx;
  const double C = c == 2 ? Y : Z, hc = c == 2 ? dy : dz;
  return w * q_path(A + di * ha, B + dj * hb, C + dk * hc, qs, qw, nq);
}

// Near offsets (|d| < 3 h_max) of the central image, one workgroup each over
// the box bx x by x bz of candidates:
// (r - r')_a / |r - r'|^3 = d/dr'_a (1/|r - r'|), so
//   g_a = -(1/V) sum_{i,j,k} w_i w_j w_k Q(A + i h_a, B + j h_b, C + k h_c),
// w_0 = -2, w_{+-1} = 1.  81 lanes take one (component, stencil point)
// each; lane c sums its component's 27 terms in a fixed order and adds the
// result to what k_oe_far left there (the other images' sum, or 0).
__global__ void __launch_bounds__(128) k_oe_near(double* __restrict__ out, int nx, int ny, int nz, double dx,
                                                 double dy, double dz, int bx, int by, const double* __restrict__ qs,
                                                 const double* __restrict__ qw, int nq) {
  const int b = blockIdx.x;
  const int i = b % bx, j = (b / bx) % by, k = b / (bx * by);
  const double X = i * dx, Y = j * dy, Z = k * dz;
  if (i >= nx || j >= ny || k >= nz || !oe_near(X, Y, Z, fmax(dx, fmax(dy, dz)))) return;   // whole workgroup
  __shared__ double part[81];
  const int t = threadIdx.x;
  if (t < 81) part[t] = oe_term(t / 27, t % 27, X, Y, Z, dx, dy, dz, qs, qw, nq);
  __syncthreads();
  if (t < 3) {
    double acc = 0.0;
    for (int p = 0; p < 27; ++p) acc += part[t * 27 + p];
    out[(size_t)t * nx * ny * nz + ((size_t)k * ny + j) * nx + i] += -acc / (dx * dy * dz);
  }
}

// Far offsets, and with periodic axes the sum over the images
// d + (a Lx, b Ly, c Lz), |a| <= Kx, ...: far images by the defining integral
// against the tent weight (the overlap of two cells displaced by u),
//   g = 1/V int prod_a (h_a - |u_a|) (d + u)/|d + u|^3 du,
// Gauss-Legendre on each half-axis with the tensor's node counts by distance;
// near images other than the central one by the path-integral reduction in
// this thread (only short periods have any).  The central image's near
// offsets are left at 0 for k_oe_near.
__global__ void __launch_bounds__(128) k_oe_far(double* __restrict__ out, int nx, int ny, int nz, double dx,
                                                double dy, double dz, GLTable gl, int Kx, int Ky, int Kz,
                                                const double* __restrict__ qs, const double* __restrict__ qw,
                                                int nq) {
  const size_t cnt = (size_t)nx * ny * nz;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= cnt) return;
  const int i = (int)(idx % nx);
  const int j = (int)((idx / nx) % ny);
  const int k = (int)(idx / ((size_t)nx * ny));
  const double hmax = fmax(dx, fmax(dy, dz));
  const double Lx = nx * dx, Ly = ny * dy, Lz = nz * dz;
  double g0 = 0.0, g1 = 0.0, g2 = 0.0;
  for (int ia = -Kx; ia <= Kx; ++ia)
    for (int ib = -Ky; ib <= Ky; ++ib)
      for (int ic = -Kz; ic <= Kz; ++ic) {
        const double X = i * dx + ia * Lx, Y = j * dy + ib * Ly, Z = k * dz + ic * Lz;
        if (oe_near(X, Y, Z, hmax)) {
          if (ia == 0 && ib == 0 && ic == 0) continue;   // k_oe_near
          double a0 = 0.0, a1 = 0.0, a2 = 0.0;
          for (int p = 0; p < 27; ++p) {
            a0 += oe_term(0, p, X, Y, Z, dx, dy, dz, qs, qw, nq);
            a1 += oe_term(1, p, X, Y, Z, dx, dy, dz, qs, qw, nq);
            a2 += oe_term(2, p, X, Y, Z, dx, dy, dz, qs, qw, nq);
          }
          const double s = -1.0 / (dx * dy * dz);
          g0 += s * a0;
          g1 += s * a1;
          g2 += s * a2;
          continue;
        }
        const double dist = sqrt(X * X + Y * Y + Z * Z) / hmax;
        const int b = dist < 6.0 ? 0 : dist < 16.0 ? 1 : dist < 40.0 ? 2 : 3;
        const int n = gl.n[b];
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int ax = 0; ax < 2 * n; ++ax) {
          const double ux = (ax < n ? 1.0 : -1.0) * gl.u[b][ax % n] * dx;
          const double wx = gl.w[b][ax % n] * dx * (dx - fabs(ux));
          const double vx = X + ux;
          for (int ay = 0; ay < 2 * n; ++ay) {
            const double uy = (ay < n ? 1.0 : -1.0) * gl.u[b][ay % n] * dy;
            const double wy = gl.w[b][ay % n] * dy * (dy - fabs(uy));
            const double vy = Y + uy;
            for (int az = 0; az < 2 * n; ++az) {
              const double uz = (az < n ? 1.0 : -1.0) * gl.u[b][az % n] * dz;
              const double wz = gl.w[b][az % n] * dz * (dz - fabs(uz));
              const double vz = Z + uz;
              const double r2 = vx * vx + vy * vy + vz * vz;
              const double wt = wx * wy * wz / (r2 * sqrt(r2));
              s0 += wt * vx;
              s1 += wt * vy;
              s2 += wt * vz;
            }
          }
        }
        const double s = 1.0 / (dx * dy * dz);
        g0 += s * s0;
        g1 += s * s1;
        g2 += s * s2;
      }
  out[idx] = g0;
  out[cnt + idx] = g1;
  out[2 * cnt + idx] = g2;
}

// out[c][o][k][q] = sum_i coef_i * in[c][o][i][q] * trig(i k), 0 <= k < nout,
// trig = cos (component even along this axis) or sin (odd), coef_0 = 1 and
// coef_i = 2 for i > 0.  cs holds cos, sn sin of 2 pi m / npad, m < npad.
__global__ void k_axis(const double* __restrict__ in, double* __restrict__ out, int nc, int outer, int nin, int nout,
                       int inner, int npad, unsigned odd_mask, const double* __restrict__ cs,
                       const double* __restrict__ sn) {
  const size_t per_c = (size_t)outer * nout * inner;
  const size_t tot = (size_t)nc * per_c;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tot) return;
  const int c = (int)(idx / per_c);
  size_t rem = idx - (size_t)c * per_c;
  const int q = (int)(rem % inner);
  rem /= inner;
  const int k = (int)(rem % nout);
  const int o = (int)(rem / nout);
  const bool odd = (odd_mask >> c) & 1u;
  const double* src = in + (((size_t)c * outer + o) * nin) * inner + q;
  const double* tab = odd ? sn : cs;
  double acc = odd ? 0.0 : src[0];
  const int mask = npad - 1;
  int m = k & mask;
  for (int i = 1; i < nin; ++i) {
    acc += 2.0 * src[(size_t)i * inner] * tab[m];
    m = (m + k) & mask;
  }
  out[idx] = acc;
}

// in [nc][Kzh][Kyh][Kx] (FP64) -> K[kz][kx][c][ky] (FP32, rows of pitch Kyp
// holding ky < Ny/2, or ky = 0 for Ny = 1, zero padded) and KN[kz][kx][c]
// (ky = Ny/2, Ny >= 4) after the rows; times -sign_c / npad (demagnetizing
// tensor, nc = 6) or 1 / (4 pi npad) (Oersted kernel, nc = 3)
__global__ void k_pack(const double* __restrict__ in, float* __restrict__ K, int nc, int Kx, int Kyh, int Kyp, int Kzh,
                       int Ny, double inv_npad) {
  const size_t per_c = (size_t)Kzh * Kyh * Kx;
  const size_t nrow = (size_t)nc * Kzh * Kyp * Kx;
  const size_t tot = nrow + (size_t)nc * Kzh * Kx;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tot) return;
  int ky, c, kx, kz;
  bool have;
  if (idx < nrow) {
    ky = (int)(idx % Kyp);
    size_t rem = idx / Kyp;
    c = (int)(rem % nc);
    rem /= nc;
    kx = (int)(rem % Kx);
    kz = (int)(rem / Kx);
    have = Ny >= 4 ? ky < Ny / 2 : ky == 0;
  } else {
    size_t rem = idx - nrow;
    c = (int)(rem % nc);
    rem /= nc;
    kx = (int)(rem % Kx);
    kz = (int)(rem / Kx);
    ky = Ny / 2;
    have = Ny >= 4;
  }
  const double s = nc == 3 ? inv_npad / (4.0 * M_PI) : (c < 3 ? -1.0 : 1.0) * inv_npad;
  K[idx] = have ? (float)(s * in[c * per_c + ((size_t)kz * Kyh + ky) * Kx + kx]) : 0.f;
}

}  // namespace demag

namespace demag {

// ---------------------------------------------------------------------------
// Inter-mesh tensor between cells of different sizes (Sec. 3, Eq. 4:
// N(r, h_k, h_i)).  Closed form: f/g under a 4-point stencil per axis,
// X +- (a+b)/2 weight -1 and X +- (a-b)/2 weight +1 (a target, b source
// size), over 4 pi V_target.  Far field: Gauss-Legendre quadrature of the
// dipole kernel against the overlap weight of the two boxes per axis, a
// trapezoid of base a + b and plateau min(a, b).
// ---------------------------------------------------------------------------
template <bool OFFDIAG>
__device__ double stencil64(double X, double Y, double Z, double ta, double sa, double tb, double sb, double tc,
                            double sc) {
  const double ox[4] = {0.5 * (ta + sa), -0.5 * (ta + sa), 0.5 * (ta - sa), -0.5 * (ta - sa)};
  const double oy[4] = {0.5 * (tb + sb), -0.5 * (tb + sb), 0.5 * (tb - sb), -0.5 * (tb - sb)};
  const double oz[4] = {0.5 * (tc + sc), -0.5 * (tc + sc), 0.5 * (tc - sc), -0.5 * (tc - sc)};
  double acc = 0.0;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j)
      for (int k = 0; k < 4; ++k) {
        const double w = (i < 2 ? -1.0 : 1.0) * (j < 2 ? -1.0 : 1.0) * (k < 2 ? -1.0 : 1.0);
        acc += w * (OFFDIAG ? ng(X + ox[i], Y + oy[j], Z + oz[k]) : nf(X + ox[i], Y + oy[j], Z + oz[k]));
      }
  return acc / (4.0 * M_PI * ta * tb * tc);
}

// idx-th quadrature node of the overlap weight of widths a and b along one
// axis (3 pieces of n nodes: two ramps, then the plateau when a != b)
__device__ bool trap_node(double a, double b, int n, int idx, const GLTable& gl, int band, double& u, double& w) {
  const double lo = 0.5 * fabs(a - b), hi = 0.5 * (a + b);
  const int piece = idx / n, i = idx - piece * n;
  const double x = gl.u[band][i], wx = gl.w[band][i];
  if (piece < 2) {
    const double v = lo + (hi - lo) * x;
    u = piece == 0 ? v : -v;
    w = (hi - lo) * wx * (hi - v);
    return true;
  }
  if (lo <= 0.0) return false;
  u = -lo + 2.0 * lo * x;
  w = 2.0 * lo * wx * fmin(a, b);
  return true;
}

__device__ void tensor_unequal_dev(double X, double Y, double Z, const double* ht, const double* hs,
                                   const GLTable& gl, double* N) {
  const double hmax = fmax(fmax(fmax(ht[0], ht[1]), ht[2]), fmax(fmax(hs[0], hs[1]), hs[2]));
  const double dist = sqrt(X * X + Y * Y + Z * Z) / hmax;
  if (dist < 3.0) {
    N[0] = stencil64<false>(X, Y, Z, ht[0], hs[0], ht[1], hs[1], ht[2], hs[2]);
    N[1] = stencil64<false>(Y, X, Z, ht[1], hs[1], ht[0], hs[0], ht[2], hs[2]);
    N[2] = stencil64<false>(Z, Y, X, ht[2], hs[2], ht[1], hs[1], ht[0], hs[0]);
    N[3] = stencil64<true>(X, Y, Z, ht[0], hs[0], ht[1], hs[1], ht[2], hs[2]);
    N[4] = stencil64<true>(X, Z, Y, ht[0], hs[0], ht[2], hs[2], ht[1], hs[1]);
    N[5] = stencil64<true>(Y, Z, X, ht[1], hs[1], ht[2], hs[2], ht[0], hs[0]);
    return;
  }
  const int band = dist < 6.0 ? 0 : dist < 16.0 ? 1 : dist < 40.0 ? 2 : 3;
  const int n = gl.n[band];
  for (int q = 0; q < 6; ++q) N[q] = 0.0;
  for (int ia = 0; ia < 3 * n; ++ia) {
    double ux, wx;
    if (!trap_node(ht[0], hs[0], n, ia, gl, band, ux, wx)) continue;
    const double vx = X + ux;
    for (int ib = 0; ib < 3 * n; ++ib) {
      double uy, wy;
      if (!trap_node(ht[1], hs[1], n, ib, gl, band, uy, wy)) continue;
      const double vy = Y + uy;
      for (int ic = 0; ic < 3 * n; ++ic) {
        double uz, wz;
        if (!trap_node(ht[2], hs[2], n, ic, gl, band, uz, wz)) continue;
        const double vz = Z + uz;
        const double r2 = vx * vx + vy * vy + vz * vz;
        const double wt = wx * wy * wz / (r2 * r2 * sqrt(r2));
        N[0] += wt * (r2 - 3.0 * vx * vx);
        N[1] += wt * (r2 - 3.0 * vy * vy);
        N[2] += wt * (r2 - 3.0 * vz * vz);
        N[3] -= wt * 3.0 * vx * vy;
        N[4] -= wt * 3.0 * vx * vz;
        N[5] -= wt * 3.0 * vy * vz;
      }
    }
  }
  const double s = 1.0 / (4.0 * M_PI * ht[0] * ht[1] * ht[2]);
  for (int q = 0; q < 6; ++q) N[q] *= s;
}

// One plane pair on the padded fine grid [6][Ny][Nx] (FP64 complex, imaginary
// part 0): lattice offset u = i for i < Lx, i - Nx for i > Nx - Lx, none
// (zero) in between; the same along y.  Along periodic in-plane axes the
// tensor is summed over the images, offsets shifted by whole periods (Sec. 3,
// multiple images).
__global__ void k_pair_tensor(double2* __restrict__ out, PairGeom pg, GLTable gl) {
  const size_t cnt = (size_t)pg.Nx * pg.Ny;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= cnt) return;
  const int i = (int)(idx % pg.Nx), j = (int)(idx / pg.Nx);
  const int u = i < pg.Lx ? i : (i > pg.Nx - pg.Lx ? i - pg.Nx : INT_MIN);
  const int v = j < pg.Ly ? j : (j > pg.Ny - pg.Ly ? j - pg.Ny : INT_MIN);
  double N[6] = {0, 0, 0, 0, 0, 0};
  if (u != INT_MIN && v != INT_MIN) {
    // summed over the images of periodic in-plane axes (kx = ky = 0: open)
    for (int a = -pg.kx; a <= pg.kx; ++a)
      for (int b = -pg.ky; b <= pg.ky; ++b) {
        double Ni[6];
        tensor_unequal_dev(u * pg.fx + pg.ox + a * pg.px, v * pg.fy + pg.oy + b * pg.py, pg.oz, pg.ht, pg.hs, gl, Ni);
        for (int q = 0; q < 6; ++q) N[q] += Ni[q];
      }
  }
  for (int q = 0; q < 6; ++q) out[q * cnt + idx] = make_double2(N[q], 0.0);
}

// In-place FP64 FFT of lines of N = 2^logN points (radix 2, in LDS).  Line l
// starts at (l / lpb) * bstride + (l % lpb) * ls, elements es apart.
__global__ void k_fft64_lines(double2* __restrict__ data, int logN, long long es, long long ls, int lpb,
                              long long bstride, const double2* __restrict__ tw64) {
  extern __shared__ double2 buf[];
  const int N = 1 << logN;
  const int l = blockIdx.x;
  double2* base = data + (long long)(l / lpb) * bstride + (long long)(l % lpb) * ls;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    int r = 0, x = i;
    for (int b = 0; b < logN; ++b) { r = (r << 1) | (x & 1); x >>= 1; }
    buf[r] = base[(long long)i * es];
  }
  __syncthreads();
  for (int len = 2; len <= N; len <<= 1) {
    const int half = len >> 1, step = 4096 / len;
    for (int k = threadIdx.x; k < N / 2; k += blockDim.x) {
      const int j = k % half, s0 = (k / half) * len;
      const double2 w = tw64[j * step];
      const double2 a = buf[s0 + j], b = buf[s0 + j + half];
      const double2 bw = make_double2(b.x * w.x - b.y * w.y, b.x * w.y + b.y * w.x);
      buf[s0 + j] = make_double2(a.x + bw.x, a.y + bw.y);
      buf[s0 + j + half] = make_double2(a.x - bw.x, a.y - bw.y);
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < N; i += blockDim.x) base[(long long)i * es] = buf[i];
}

// [6][Ny][Nx] FP64 spectrum -> one pair's block K[6][Kx][NY] times scale, ky
// stored by residue (r * NY/2 + k' for ky = 2k' + r).  FP32 complex, or for a
// pair without in-plane centre offset (parity != 0) one FP32 per frequency:
// the real part of xx yy zz xy, the imaginary part of xz yz (the other part
// is zero by the parity of the tensor in the in-plane offsets).
__global__ void k_pair_pack(const double2* __restrict__ in, float* __restrict__ K, int Nx, int Ny, int Kx,
                            double scale, int parity) {
  const size_t tot = (size_t)6 * Kx * Ny;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tot) return;
  const int ry = (int)(idx % Ny);
  const int kx = (int)((idx / Ny) % Kx);
  const int c = (int)(idx / ((size_t)Ny * Kx));
  const int M = Ny > 1 ? Ny / 2 : 1;
  const int ky = Ny > 1 ? 2 * (ry % M) + ry / M : 0;
  const double2 v = in[(size_t)c * Nx * Ny + (size_t)ky * Nx + kx];
  if (parity) {
    K[idx] = (float)(scale * (c < 4 ? v.x : v.y));
  } else {
    reinterpret_cast<float2*>(K)[idx] = make_float2((float)(scale * v.x), (float)(scale * v.y));
  }
}

}  // namespace demag

#include "launch.hpp"

namespace demag {

hipError_t launch_tensor(double* out, const Geom& g, const GLTable& gl, hipStream_t s) {
  const size_t cnt = (size_t)g.nx * g.ny * g.nz;
  const int K = g.images;
  hipLaunchKernelGGL(k_tensor, dim3((unsigned)((cnt + 127) / 128)), dim3(128), 0, s, out, g.nx, g.ny, g.nz, g.dx,
                     g.dy, g.dz, gl, (g.pbc & 1u) ? K : 0, (g.pbc & 2u) ? K : 0, (g.pbc & 4u) ? K : 0);
  return hipGetLastError();
}

hipError_t launch_axis(const double* in, double* out, int nc, int outer, int nin, int nout, int inner, int npad,
                       unsigned odd_mask, const double* cs, const double* sn, hipStream_t s) {
  const size_t tot = (size_t)nc * outer * nout * inner;
  hipLaunchKernelGGL(k_axis, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, in, out, nc, outer, nin, nout,
                     inner, npad, odd_mask, cs, sn);
  return hipGetLastError();
}

hipError_t launch_pack(const double* in, float* K, const Geom& g, hipStream_t s) {
  const int nc = kernel_comps(g);
  const size_t tot = (size_t)nc * g.Kzh * g.Kx * (g.Kyp + 1);
  hipLaunchKernelGGL(k_pack, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, in, K, nc, g.Kx, g.Kyh, g.Kyp,
                     g.Kzh, g.Ny, 1.0 / ((double)g.Nx * g.Ny * g.Nz));
  return hipGetLastError();
}

hipError_t launch_oe_tensor(double* out, const Geom& g, const GLTable& gl, const double* qs, const double* qw, int nq,
                            hipStream_t s) {
  const size_t cnt = (size_t)g.nx * g.ny * g.nz;
  const int K = g.images;
  hipLaunchKernelGGL(k_oe_far, dim3((unsigned)((cnt + 127) / 128)), dim3(128), 0, s, out, g.nx, g.ny, g.nz, g.dx, g.dy,
                     g.dz, gl, (g.pbc & 1u) ? K : 0, (g.pbc & 2u) ? K : 0, (g.pbc & 4u) ? K : 0, qs, qw, nq);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // candidates for |d| < 3 h_max along each axis: index < 3 h_max / h_a
  const double hmax = std::fmax(g.dx, std::fmax(g.dy, g.dz));
  const int bx = std::min(g.nx, (int)(3.0 * hmax / g.dx) + 1);
  const int by = std::min(g.ny, (int)(3.0 * hmax / g.dy) + 1);
  const int bz = std::min(g.nz, (int)(3.0 * hmax / g.dz) + 1);
  hipLaunchKernelGGL(k_oe_near, dim3((unsigned)(bx * by * bz)), dim3(128), 0, s, out, g.nx, g.ny, g.nz, g.dx, g.dy,
                     g.dz, bx, by, qs, qw, nq);
  return hipGetLastError();
}

}  // namespace demag

namespace demag {

hipError_t launch_pair_tensor(double2* out, const PairGeom& pg, const GLTable& gl, hipStream_t s) {
  const size_t cnt = (size_t)pg.Nx * pg.Ny;
  hipLaunchKernelGGL(k_pair_tensor, dim3((unsigned)((cnt + 127) / 128)), dim3(128), 0, s, out, pg, gl);
  return hipGetLastError();
}

hipError_t launch_fft64(double2* data, int logN, long long es, long long ls, int lpb, long long bstride, int nlines,
                        const double2* tw64, hipStream_t s) {
  const size_t lds = (size_t)sizeof(double2) << logN;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k_fft64_lines, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_fft64_lines, dim3(nlines), dim3(256), lds, s, data, logN, es, ls, lpb, bstride, tw64);
  return hipGetLastError();
}

hipError_t launch_pair_pack(const double2* in, float* K, int Nx, int Ny, int Kx, double scale, int parity,
                            hipStream_t s) {
  const size_t tot = (size_t)6 * Kx * Ny;
  hipLaunchKernelGGL(k_pair_pack, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, in, K, Nx, Ny, Kx, scale,
                     parity);
  return hipGetLastError();
}

}  // namespace demag
