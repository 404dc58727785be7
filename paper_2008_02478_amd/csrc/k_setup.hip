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
#include <hip/hip_runtime.h>
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

__global__ void k_tensor(double* __restrict__ out, int nx, int ny, int nz, double dx, double dy, double dz,
                         GLTable gl) {
  const size_t cnt = (size_t)nx * ny * nz;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= cnt) return;
  const int i = (int)(idx % nx);
  const int j = (int)((idx / nx) % ny);
  const int k = (int)(idx / ((size_t)nx * ny));
  const double X = i * dx, Y = j * dy, Z = k * dz;
  const double hmax = fmax(dx, fmax(dy, dz));
  const double dist = sqrt(X * X + Y * Y + Z * Z) / hmax;
  double N[6];
  if (dist < 3.0) {
    N[0] = stencil27<false>(X, Y, Z, dx, dy, dz);
    N[1] = stencil27<false>(Y, X, Z, dy, dx, dz);
    N[2] = stencil27<false>(Z, Y, X, dz, dy, dx);
    N[3] = stencil27<true>(X, Y, Z, dx, dy, dz);
    N[4] = stencil27<true>(X, Z, Y, dx, dz, dy);
    N[5] = stencil27<true>(Y, Z, X, dy, dz, dx);
  } else {
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
  for (int q = 0; q < 6; ++q) out[q * cnt + idx] = N[q];
}

// out[c][o][k][q] = sum_i coef_i * in[c][o][i][q] * trig(i k), 0 <= k < nout,
// trig = cos (component even along this axis) or sin (odd), coef_0 = 1 and
// coef_i = 2 for i > 0.  cs holds cos, sn sin of 2 pi m / npad, m < npad.
__global__ void k_axis(const double* __restrict__ in, double* __restrict__ out, int outer, int nin, int nout,
                       int inner, int npad, unsigned odd_mask, const double* __restrict__ cs,
                       const double* __restrict__ sn) {
  const size_t per_c = (size_t)outer * nout * inner;
  const size_t tot = 6 * per_c;
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

// in [6][Kzh][Kyh][Kx] (FP64) -> K[kz][kx][c][ky] (FP32) times -sign_c / npad
__global__ void k_pack(const double* __restrict__ in, float* __restrict__ K, int Kx, int Kyh, int Kzh,
                       double inv_npad) {
  const size_t per_c = (size_t)Kzh * Kyh * Kx;
  const size_t tot = 6 * per_c;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tot) return;
  const int ky = (int)(idx % Kyh);
  size_t rem = idx / Kyh;
  const int c = (int)(rem % 6);
  rem /= 6;
  const int kx = (int)(rem % Kx);
  const int kz = (int)(rem / Kx);
  const double s = (c < 3 ? -1.0 : 1.0) * inv_npad;
  K[idx] = (float)(s * in[c * per_c + ((size_t)kz * Kyh + ky) * Kx + kx]);
}

}  // namespace demag

#include "launch.hpp"

namespace demag {

hipError_t launch_tensor(double* out, const Geom& g, const GLTable& gl, hipStream_t s) {
  const size_t cnt = (size_t)g.nx * g.ny * g.nz;
  hipLaunchKernelGGL(k_tensor, dim3((unsigned)((cnt + 127) / 128)), dim3(128), 0, s, out, g.nx, g.ny, g.nz, g.dx,
                     g.dy, g.dz, gl);
  return hipGetLastError();
}

hipError_t launch_axis(const double* in, double* out, int outer, int nin, int nout, int inner, int npad,
                       unsigned odd_mask, const double* cs, const double* sn, hipStream_t s) {
  const size_t tot = (size_t)6 * outer * nout * inner;
  hipLaunchKernelGGL(k_axis, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, in, out, outer, nin, nout, inner,
                     npad, odd_mask, cs, sn);
  return hipGetLastError();
}

hipError_t launch_pack(const double* in, float* K, const Geom& g, hipStream_t s) {
  const size_t tot = (size_t)6 * g.Kzh * g.Kyh * g.Kx;
  hipLaunchKernelGGL(k_pack, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, in, K, g.Kx, g.Kyh, g.Kzh,
                     1.0 / ((double)g.Nx * g.Ny * g.Nz));
  return hipGetLastError();
}

}  // namespace demag
