// One stage of a classical RK4 step of the LLG equation (Sec. 2, Eq. 1,
// solved for dm/dt: dm/dt = -gamma' [m x H + alpha m x (m x H)], gamma' =
// gamma / (1 + alpha^2)) with the effective field of Sec. 7's benchmark:
// demagnetizing (computed by the field passes before this kernel), applied,
// and direct exchange H = (2A / (mu0 Ms)) lap(m) (Appendix A, Table 1) with
// the discrete Neumann condition (a missing neighbour is the cell itself) or
// periodic neighbours along periodic axes.
//
// Stages s = 0..3 with slopes k_s:
//   s = 0: acc = k0;        next = m0 + dt/2 k0
//   s = 1: acc += 2 k1;     next = m0 + dt/2 k1
//   s = 2: acc += 2 k2;     next = m0 + dt k2
//   s = 3: m = m0 + dt/6 (acc + k3), renormalized to unit length.
// One thread per cell; SoA vectors [3][nz][ny][nx].
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "plan.hpp"

namespace demag {

__device__ __forceinline__ int neighbour(int v, int n, int d, bool periodic) {
  int w = v + d;
  if (w < 0) w = periodic ? w + n : v;
  else if (w >= n) w = periodic ? w - n : v;
  return w;
}

__global__ void __launch_bounds__(256) k_llg_stage(LlgArgs a) {
  const size_t n = (size_t)a.nx * a.ny * a.nz;
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int x = (int)(i % a.nx);
  const int y = (int)((i / a.nx) % a.ny);
  const int z = (int)(i / ((size_t)a.nx * a.ny));
  const size_t row = (size_t)z * a.ny * a.nx + (size_t)y * a.nx;
  const size_t xm = row + neighbour(x, a.nx, -1, a.pbc & 1u), xp = row + neighbour(x, a.nx, 1, a.pbc & 1u);
  const size_t base_z = (size_t)z * a.ny * a.nx;
  const size_t ym = base_z + (size_t)neighbour(y, a.ny, -1, a.pbc & 2u) * a.nx + x;
  const size_t yp = base_z + (size_t)neighbour(y, a.ny, 1, a.pbc & 2u) * a.nx + x;
  const size_t zm = (size_t)neighbour(z, a.nz, -1, a.pbc & 4u) * a.ny * a.nx + (size_t)y * a.nx + x;
  const size_t zp = (size_t)neighbour(z, a.nz, 1, a.pbc & 4u) * a.ny * a.nx + (size_t)y * a.nx + x;
  const float hext[3] = {a.hx, a.hy, a.hz};
  float m[3], H[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float* v = a.mi + (size_t)c * n;
    const float mc = v[i];
    const float lap = (v[xp] - 2.f * mc + v[xm]) * a.ihx2 + (v[yp] - 2.f * mc + v[ym]) * a.ihy2 +
                      (v[zp] - 2.f * mc + v[zm]) * a.ihz2;
    m[c] = mc;
    H[c] = a.Hd[(size_t)c * n + i] + hext[c] + a.cex * lap;
  }
  const float t0 = m[1] * H[2] - m[2] * H[1];
  const float t1 = m[2] * H[0] - m[0] * H[2];
  const float t2 = m[0] * H[1] - m[1] * H[0];
  const float d0 = m[1] * t2 - m[2] * t1;
  const float d1 = m[2] * t0 - m[0] * t2;
  const float d2 = m[0] * t1 - m[1] * t0;
  const float k[3] = {-a.gp * (t0 + a.alpha * d0), -a.gp * (t1 + a.alpha * d1), -a.gp * (t2 + a.alpha * d2)};
  if (a.stage < 3) {
    const float cn = a.stage == 2 ? a.dt : 0.5f * a.dt;
    const float ca = a.stage == 0 ? 1.f : 2.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const size_t j = (size_t)c * n + i;
      a.acc[j] = a.stage == 0 ? k[c] : a.acc[j] + ca * k[c];
      a.next[j] = a.m0[j] + cn * k[c];
    }
  } else {
    float o[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const size_t j = (size_t)c * n + i;
      o[c] = a.m0[j] + (a.dt / 6.f) * (a.acc[j] + k[c]);
    }
    const float inv = 1.f / sqrtf(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]);
#pragma unroll
    for (int c = 0; c < 3; ++c) a.mout[(size_t)c * n + i] = o[c] * inv;
  }
}

hipError_t launch_llg_stage(const LlgArgs& a, hipStream_t s) {
  const size_t n = (size_t)a.nx * a.ny * a.nz;
  hipLaunchKernelGGL(k_llg_stage, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace demag
