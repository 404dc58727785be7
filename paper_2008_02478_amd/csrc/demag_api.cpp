// C ABI of the demagnetizing-field library: argument checks, plan geometry,
// kernel-spectrum set-up and the launch sequence of one field evaluation.
//
// A plan holds one or more sub-plans, each a group of meshes with identical
// geometry that share one kernel spectrum and run through the same three
// passes with a batch dimension.  A single-mesh plan is one sub-plan with one
// member and no offset tables.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/demag.h"
#include "fft_core.hpp"
#include "launch.hpp"
#include "plan.hpp"
#include "tune_cache.hpp"

using namespace demag;

namespace {

struct Sub {
  Geom g{};
  std::vector<int> members;          // global mesh ids
  size_t k_off = 0, tab_off = 0;     // offsets into the kernel buffer
  size_t t_off = 0, e_off = 0;       // offsets into the work buffer
  size_t parts = 0;                  // energy partials per member
  float* K = nullptr;
  long long* moff = nullptr;
  int* gid = nullptr;
  float2* T = nullptr;
  double* epart = nullptr;
};

// A coupled group: planes of several meshes on one fine in-plane lattice.
struct Group {
  std::vector<int> members;
  std::vector<PlaneInfo> planes;
  std::vector<double> ph;          // 3 cell sizes per plane
  std::vector<double> pdx, pdy, pz;
  Geom g{};                        // fine lattice: nx = Lx, ny = Ly, nz = Nz = P
  double fx = 0, fy = 0;
  unsigned pbc = 0;                // periodic in-plane axes (bit 0 x, bit 1 y)
  int images = 0;
  size_t k_off = 0, pl_off = 0, t_off = 0, s_off = 0, e_off = 0;
  float* K = nullptr;               // pair spectra (complex, or one float per frequency for parity pairs)
  PlaneInfo* pl = nullptr;
  float2* T = nullptr;
  float2* S = nullptr;
  double* epart = nullptr;
  int npairs() const { const int P = (int)planes.size(); return P * (P + 1) / 2; }
  // pairs (p <= q, in order) whose planes share the in-plane cell centres:
  // their spectra are stored as one float per frequency and component
  unsigned long long parity_pairs() const {
    unsigned long long m = 0;
    const int P = (int)planes.size();
    int i = 0;
    for (int p = 0; p < P; ++p)
      for (int q = p; q < P; ++q, ++i)
        if (pdx[p] == pdx[q] && pdy[p] == pdy[q]) m |= 1ull << i;
    return m;
  }
  // floats of all pair spectra (6 components per frequency each)
  size_t pair_floats(size_t npt) const {
    const unsigned long long m = parity_pairs();
    size_t n = 0;
    for (int i = 0; i < npairs(); ++i) n += ((m >> i) & 1ull) ? 6 * npt : 12 * npt;
    return n;
  }
};

}  // namespace

struct demag_plan {
  std::vector<Sub> subs;
  std::vector<Group> groups;
  bool batch = false;
  bool oersted = false;              // Oersted-field plan (demag_setup_oersted)
  std::vector<long long> offsets;    // float offset of each mesh in concatenated buffers
  size_t total_floats = 0;
  bool bound = false;
  bool has_work = false;             // bound with a work buffer (else demag_field_noalloc only)
  int device = -1;
  char* noalloc_work = nullptr;      // this device's static scratch (demag_field_noalloc)
  float2* tw = nullptr;
  size_t kernel_bytes = 0, work_bytes = 0;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  bool timing = false;
};

namespace {

thread_local std::string g_err;
constexpr double MU0 = 4.0e-7 * M_PI;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int fail_hip(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return DEMAG_EHIP;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Work space of demag_field_noalloc: the spectrum and energy partials of one
// single-mesh plan, in a device array of fixed size instead of a buffer the
// caller allocates.  Every GPU the library runs on holds its own copy until
// the process ends.  In host code the array's name is only a stand-in: its
// device address, per device, comes from hipGetSymbolAddress, taken once per
// device with that device current (at the first demag_bind on it) and kept
// in scratch_ptr.
static __device__ __align__(256) unsigned char scratch[DEMAG_NOALLOC_WORK_BYTES];
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
char* scratch_ptr[MAX_DEVICES] = {};

int noalloc_scratch(int dev, char** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return fail(DEMAG_EUNSUPPORTED, "device index out of range for the static scratch");
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(DEMAG_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    scratch_ptr[dev] = static_cast<char*>(ptr);
  }
  *out = scratch_ptr[dev];
  return DEMAG_OK;
}

int padded(int n) {
  if (n == 1) return 1;
  int p = 1;
  while (p < 2 * n - 1) p *= 2;
  return p;
}

int ilog2i(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

int line_threads(int M) { return M / line_radix(M); }  // lanes per line of the x passes

// Gauss-Legendre rule of order n on [-1, 1] by Newton iteration on P_n.
void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

bool aligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255) == 0; }

constexpr size_t XTAB_BYTES = 8192;   // stage twiddle table of the x passes (upper bound)

// Whether the fused x+z passes support a geometry: the nz rows of one y line
// fit in LDS, and the z lines fit the in-register transforms (padded length
// 64 for nx <= 512, 128 for nx <= 256).
bool fused_ok(const Geom& g) {
  if (g.nz > 64 || (g.nz > 16 && g.nx > 512) || (g.nz > 32 && g.nx > 256)) return false;
  return (size_t)g.nz * xrow_pitch_rt(g.lnx) * sizeof(float2) + XTAB_BYTES <= 160 * 1024;
}
// Separate z passes exist for padded z lengths 4..512.
bool zsep_ok(const Geom& g) { return g.nz >= 2 && g.Nz <= 512; }

// Validate one mesh and derive its geometry (host only).
constexpr int DEFAULT_IMAGES = 10;
constexpr int MAX_IMAGES = 1000;

int make_geom(int nx, int ny, int nz, double dx, double dy, double dz, unsigned pbc, int images, Geom& g,
              const char* who) {
  if (nx < 1 || ny < 1 || nz < 1) return fail(DEMAG_EINVAL, std::string(who) + ": mesh dimensions must be >= 1");
  if (!(std::isfinite(dx) && std::isfinite(dy) && std::isfinite(dz)) || dx <= 0 || dy <= 0 || dz <= 0)
    return fail(DEMAG_EINVAL, std::string(who) + ": cell sizes must be finite and > 0");
  if (nx > 2048 || ny > 1024 || nz > 256)
    return fail(DEMAG_EUNSUPPORTED, std::string(who) + ": supported sizes are nx <= 2048, ny <= 1024, nz <= 256");
  g = Geom{};
  g.nx = nx; g.ny = ny; g.nz = nz;
  g.Nx = padded(nx); g.Ny = padded(ny); g.Nz = padded(nz);
  g.lnx = ilog2i(g.Nx); g.lny = ilog2i(g.Ny); g.lnz = ilog2i(g.Nz);
  g.Kx = g.Nx > 1 ? g.Nx / 2 + 1 : 1;
  g.Kyh = g.Ny > 1 ? g.Ny / 2 + 1 : 1;
  g.Kzh = g.Nz > 1 ? g.Nz / 2 + 1 : 1;
  g.Kyp = kernel_row_pitch(g.Ny);
  g.nTiles = (g.Kx + TILE - 1) / TILE;
  g.dx = dx; g.dy = dy; g.dz = dz;
  // y rows per workgroup of the x passes: enough rows for one round of the
  // workgroup, within 64 KiB of LDS; for the fused x+z passes a y row brings
  // its nz rows, for the flattened x passes of separate z passes one row
  const size_t pitch_bytes = (size_t)xrow_pitch_rt(g.lnx) * sizeof(float2);
  const int P = g.Nx >= 4 ? g.Nx / 4 : 1;
  const int rpr = FWD_THREADS / (2 * line_threads(P));
  auto rows_per_wg = [&](int zrows, int nrows) {
    int yg = (rpr + zrows - 1) / zrows;
    while (yg > 1 && (size_t)yg * zrows * pitch_bytes + XTAB_BYTES > 65536) --yg;
    if (yg > nrows) yg = nrows;
    return yg < 1 ? 1 : yg;
  };
  g.yg = rows_per_wg(nz, ny);
  g.yg_sep = rows_per_wg(1, ny * nz);
  // the fused x+z passes need the nz rows of a y line in LDS and their z
  // lines in registers; beyond that the z transform runs as separate passes
  g.zsep = fused_ok(g) ? 0 : 1;
  g.mid_kw = 4;
  g.mid_r = 0;
  g.pbc = pbc;
  g.images = pbc ? (images > 0 ? images : DEFAULT_IMAGES) : 0;
  return DEMAG_OK;
}

// Buffer layout of a plan (sizes only; pointers are attached at bind).
void layout(demag_plan* p) {
  size_t kb = align256((size_t)TW_SIZE * sizeof(float2));
  size_t wb = 0;
  for (Sub& s : p->subs) {
    const Geom& g = s.g;
    const size_t nb = s.members.size();
    s.k_off = kb;
    kb += align256((size_t)kernel_comps(g) * g.Kzh * g.Kx * (g.Kyp + 1) * sizeof(float));   // rows, then KN
    s.tab_off = kb;
    kb += align256(nb * sizeof(long long)) + align256(nb * sizeof(int));
    s.t_off = wb;
    wb += align256(nb * spectrum_elems(g) * sizeof(float2));
    const size_t ncell = (size_t)g.nx * g.ny * g.nz;
    s.parts = (size_t)mid_blocks_max(g);   // room for every middle-pass schedule
    const size_t ecb = (size_t)energy_cell_blocks(ncell);
    if (ecb > s.parts) s.parts = ecb;
    s.e_off = wb;
    wb += align256(nb * s.parts * sizeof(double));
  }
  for (Group& G : p->groups) {
    const Geom& g = G.g;
    const int P = (int)G.planes.size();
    const size_t npt = (size_t)g.Kx * g.Ny;
    G.k_off = kb;
    kb += align256(G.pair_floats(npt) * sizeof(float));
    G.pl_off = kb;
    kb += align256((size_t)P * sizeof(PlaneInfo));
    G.t_off = wb;
    wb += align256(spectrum_elems(g) * sizeof(float2));
    G.s_off = wb;
    wb += align256((size_t)3 * P * npt * sizeof(float2));
    G.e_off = wb;
    wb += align256((size_t)couple_blocks(g.Kx, g.Ny) * P * sizeof(double));
  }
  p->kernel_bytes = kb;
  p->work_bytes = wb;
}

// Coupled group from meshes idx (validated; host only).
int make_group(const std::vector<int>& idx, const int* dims, const double* cells, const double* origins,
               const std::vector<long long>& offsets, unsigned pbc, int images, Group& G) {
  const char* who = "demag_setup_batch";
  double fx = 1e300, fy = 1e300, X0 = 1e300, Y0 = 1e300;
  for (int i : idx) {
    fx = std::min(fx, cells[3 * i]);
    fy = std::min(fy, cells[3 * i + 1]);
    X0 = std::min(X0, origins[3 * i]);
    Y0 = std::min(Y0, origins[3 * i + 1]);
  }
  auto pow2ratio = [](double a, double f, int& s) {
    const double r = a / f;
    s = (int)std::lround(r);
    return s >= 1 && std::fabs(r - s) < 1e-9 * r && (s & (s - 1)) == 0;
  };
  auto lattice = [](double d, double f, int& o) {
    const double r = d / f;
    o = (int)std::lround(r);
    return std::fabs(r - o) < 1e-6;
  };
  int Lx = 0, Ly = 0;
  G = Group{};
  G.members = idx;
  for (int i : idx) {
    const int nx = dims[3 * i], ny = dims[3 * i + 1], nz = dims[3 * i + 2];
    const double dx = cells[3 * i], dy = cells[3 * i + 1], dz = cells[3 * i + 2];
    if (nx < 1 || ny < 1 || nz < 1 || !(dx > 0 && dy > 0 && dz > 0) || !std::isfinite(dx * dy * dz) ||
        !std::isfinite(origins[3 * i] + origins[3 * i + 1] + origins[3 * i + 2]))
      return fail(DEMAG_EINVAL, std::string(who) + ": invalid mesh in a coupled group");
    int sx, sy, ox, oy;
    if (!pow2ratio(dx, fx, sx) || !pow2ratio(dy, fy, sy))
      return fail(DEMAG_EUNSUPPORTED, std::string(who) + ": coupled in-plane cell sizes must be power-of-two multiples");
    if (!lattice(origins[3 * i] - X0, fx, ox) || !lattice(origins[3 * i + 1] - Y0, fy, oy))
      return fail(DEMAG_EUNSUPPORTED, std::string(who) + ": coupled origins must lie on the finest in-plane lattice");
    Lx = std::max(Lx, ox + nx * sx);
    Ly = std::max(Ly, oy + ny * sy);
    for (int k = 0; k < nz; ++k) {
      PlaneInfo pi{};
      pi.moff = offsets[i];
      pi.nx = nx; pi.ny = ny; pi.nz = nz; pi.k = k;
      pi.sx = sx; pi.sy = sy; pi.ox = ox; pi.oy = oy;
      pi.gid = i;
      pi.vol = (float)(dx * dy * dz);
      G.planes.push_back(pi);
      G.ph.insert(G.ph.end(), {dx, dy, dz});
      G.pdx.push_back(0.5 * (dx - fx));
      G.pdy.push_back(0.5 * (dy - fy));
      G.pz.push_back(origins[3 * i + 2] + (k + 0.5) * dz);
    }
  }
  const int P = (int)G.planes.size();
  if (P > MAXP) return fail(DEMAG_EUNSUPPORTED, std::string(who) + ": a coupled group has at most 8 z planes");
  // periodic in-plane axes: the group repeats as a whole, so every mesh spans
  // the whole lattice along such an axis
  for (int i : idx) {
    const int n[2] = {dims[3 * i], dims[3 * i + 1]};
    int s[2], o[2];
    pow2ratio(cells[3 * i], fx, s[0]);
    pow2ratio(cells[3 * i + 1], fy, s[1]);
    lattice(origins[3 * i] - X0, fx, o[0]);
    lattice(origins[3 * i + 1] - Y0, fy, o[1]);
    const int L[2] = {Lx, Ly};
    for (int a = 0; a < 2; ++a)
      if (((pbc >> a) & 1u) && (o[a] != 0 || n[a] * s[a] != L[a]))
        return fail(DEMAG_EUNSUPPORTED, std::string(who) + ": along a periodic axis every mesh of a coupled group "
                                                          "must span the whole group");
  }
  G.pbc = pbc & 3u;
  G.images = G.pbc ? images : 0;
  if (Lx < 2 || Lx > 2048 || Ly > 1024)
    return fail(DEMAG_EUNSUPPORTED, std::string(who) + ": coupled lattice must span 2..2048 x 1..1024 fine cells");
  Geom& g = G.g;
  g.nx = Lx; g.ny = Ly; g.nz = P;
  g.Nx = padded(Lx); g.Ny = padded(Ly); g.Nz = P;
  g.lnx = ilog2i(g.Nx); g.lny = ilog2i(g.Ny); g.lnz = 0;
  g.Kx = g.Nx / 2 + 1;
  g.Kyh = g.Ny > 1 ? g.Ny / 2 + 1 : 1;
  g.Kzh = 1;
  g.Kyp = kernel_row_pitch(g.Ny);
  g.nTiles = (g.Kx + TILE - 1) / TILE;
  g.dx = fx; g.dy = fy; g.dz = 1.0;
  g.yg = 1;
  g.zsep = 0;
  g.yg_sep = 1;
  g.mid_kw = 4;
  g.mid_r = 0;
  g.pbc = 0;
  g.images = 0;
  if ((size_t)P * xrow_pitch_rt(g.lnx) * sizeof(float2) + 8192 > 160 * 1024)
    return fail(DEMAG_EUNSUPPORTED, std::string(who) + ": coupled planes of one fine row must fit in 160 KiB of LDS");
  G.fx = fx;
  G.fy = fy;
  return DEMAG_OK;
}

// Pair kernel spectra of a group: FP64 tensor on the padded fine grid, FP64
// 2D FFT, times -1/(Nx Ny), FP32.
int build_group(const Group& G, hipStream_t s) {
  const Geom& g = G.g;
  const int P = (int)G.planes.size();
  const size_t cnt = (size_t)g.Nx * g.Ny;
  GLTable gl{};
  const int orders[4] = {8, 6, 4, 3};
  for (int b = 0; b < 4; ++b) {
    double x[8], w[8];
    gauss_legendre(orders[b], x, w);
    gl.n[b] = orders[b];
    for (int i = 0; i < orders[b]; ++i) {
      gl.u[b][i] = 0.5 * (1.0 + x[i]);
      gl.w[b][i] = 0.5 * w[i];
    }
  }
  std::vector<double2> tw(TW_SIZE);
  for (int k = 0; k < TW_SIZE; ++k) {
    const double ang = -2.0 * M_PI * k / TW_SIZE;
    tw[k] = make_double2(std::cos(ang), std::sin(ang));
  }
  double2 *buf = nullptr, *d_tw = nullptr;
  int rc = DEMAG_OK;
  hipError_t e;
  do {
    if (hipMalloc(&buf, 6 * cnt * sizeof(double2)) != hipSuccess || hipMalloc(&d_tw, TW_SIZE * sizeof(double2)) != hipSuccess) {
      rc = fail(DEMAG_ENOMEM, "demag_bind: set-up temporaries could not be allocated"); break;
    }
    if ((e = hipMemcpyAsync(d_tw, tw.data(), TW_SIZE * sizeof(double2), hipMemcpyHostToDevice, s)) != hipSuccess) {
      rc = fail_hip(e, "twiddle upload"); break;
    }
    int pair = 0;
    size_t koff = 0;   // float offset of the pair's spectrum
    for (int p = 0; p < P && rc == DEMAG_OK; ++p) {
      for (int q = p; q < P; ++q, ++pair) {
        PairGeom pg{};
        for (int a = 0; a < 3; ++a) {
          pg.ht[a] = G.ph[3 * p + a];
          pg.hs[a] = G.ph[3 * q + a];
        }
        pg.fx = G.fx; pg.fy = G.fy;
        pg.ox = G.pdx[p] - G.pdx[q];
        pg.oy = G.pdy[p] - G.pdy[q];
        pg.oz = G.pz[p] - G.pz[q];
        pg.Nx = g.Nx; pg.Ny = g.Ny; pg.Lx = g.nx; pg.Ly = g.ny;
        pg.kx = (G.pbc & 1u) ? G.images : 0;
        pg.ky = (G.pbc & 2u) ? G.images : 0;
        pg.px = g.nx * G.fx;
        pg.py = g.ny * G.fy;
        if ((e = launch_pair_tensor(buf, pg, gl, s)) != hipSuccess) { rc = fail_hip(e, "pair tensor"); break; }
        if ((e = launch_fft64(buf, g.lnx, 1, g.Nx, g.Ny, (long long)cnt, 6 * g.Ny, d_tw, s)) != hipSuccess) {
          rc = fail_hip(e, "pair x transform"); break;
        }
        if (g.Ny > 1 && (e = launch_fft64(buf, g.lny, g.Nx, 1, g.Nx, (long long)cnt, 6 * g.Nx, d_tw, s)) != hipSuccess) {
          rc = fail_hip(e, "pair y transform"); break;
        }
        const int parity = (int)((G.parity_pairs() >> pair) & 1ull);
        float* dst = G.K + koff;
        koff += (parity ? 6 : 12) * (size_t)g.Kx * g.Ny;
        if ((e = launch_pair_pack(buf, dst, g.Nx, g.Ny, g.Kx, -1.0 / ((double)g.Nx * g.Ny), parity, s)) != hipSuccess) {
          rc = fail_hip(e, "pair pack"); break;
        }
      }
    }
    if (rc == DEMAG_OK && (e = hipStreamSynchronize(s)) != hipSuccess) rc = fail_hip(e, "group set-up");
  } while (false);
  if (buf) (void)hipFree(buf);
  if (d_tw) (void)hipFree(d_tw);
  return rc;
}

MidArgs group_mid_args(const demag_plan* p, const Group& G) {
  const Geom& g = G.g;
  return MidArgs{G.T, nullptr, p->tw, nullptr, g.ny, g.Nz, g.Nx, g.nTiles, g.Kx, g.Kyh, g.Kzh,
                 TILE / mid_kw(g), 1, spectrum_elems(g), mid_blocks(g), G.S};
}

int run_groups(const demag_plan* p, const float* d_in, const float* ms_mesh, float Ms, float* d_out, unsigned flags,
               double* d_energy, bool backward, const float* d_H, const double* d_gE, hipStream_t s) {
  for (const Group& G : p->groups) {
    const Geom& g = G.g;
    const int P = (int)G.planes.size();
    LayerArgs la{G.pl, P, g.ny, g.nTiles, g.Kx, d_in, d_out, G.T, p->tw, ms_mesh, Ms, backward ? 1 : 0,
                 (flags & DEMAG_ACCUMULATE) ? 1 : 0, d_H, d_gE, -MU0};
    hipError_t e = launch_layer_x(g.lnx, la, false, s);
    if (e != hipSuccess) return fail_hip(e, "layer forward pass");
    const MidArgs ma = group_mid_args(p, G);
    if ((e = launch_mid_split(g, ma, 1, s)) != hipSuccess) return fail_hip(e, "layer y pass");
    CoupleArgs ca{G.S, G.K, G.pl, g.Kx, g.Ny, g.Nx, (d_energy && !backward) ? G.epart : nullptr, G.parity_pairs()};
    if ((e = launch_couple(P, ca, s)) != hipSuccess) return fail_hip(e, "layer coupling");
    if ((e = launch_mid_split(g, ma, 2, s)) != hipSuccess) return fail_hip(e, "layer inverse y pass");
    if ((e = launch_layer_x(g.lnx, la, true, s)) != hipSuccess) return fail_hip(e, "layer inverse pass");
    if (d_energy && !backward) {
      e = launch_layer_energy(G.epart, couple_blocks(g.Kx, g.Ny), P, G.pl, -0.5 * MU0, d_energy, s);
      if (e != hipSuccess) return fail_hip(e, "layer energy");
    }
  }
  return DEMAG_OK;
}

int build_spectrum(const Geom& g, float* d_K, hipStream_t s) {
  // FP64 cos/sin tables per axis
  const int Ns[3] = {g.Nx, g.Ny, g.Nz};
  int Nmax = 1;
  for (int a = 0; a < 3; ++a) Nmax = Ns[a] > Nmax ? Ns[a] : Nmax;
  std::vector<double> trig((size_t)6 * Nmax);
  for (int a = 0; a < 3; ++a)
    for (int m = 0; m < Ns[a]; ++m) {
      const double ang = 2.0 * M_PI * m / Ns[a];
      double c = std::cos(ang), sn = std::sin(ang);
      if ((4 * m) % Ns[a] == 0) {
        // multiples of a quarter turn exactly, so that the odd components'
        // sine transforms vanish exactly at the Nyquist frequency
        const int q = 4 * m / Ns[a];
        c = q == 0 ? 1.0 : (q == 2 ? -1.0 : 0.0);
        sn = q == 1 ? 1.0 : (q == 3 ? -1.0 : 0.0);
      }
      trig[(size_t)(2 * a) * Nmax + m] = c;
      trig[(size_t)(2 * a + 1) * Nmax + m] = sn;
    }
  GLTable gl{};
  const int orders[4] = {8, 6, 4, 3};
  for (int b = 0; b < 4; ++b) {
    double x[8], w[8];
    gauss_legendre(orders[b], x, w);
    gl.n[b] = orders[b];
    for (int i = 0; i < orders[b]; ++i) {
      gl.u[b][i] = 0.5 * (1.0 + x[i]);
      gl.w[b][i] = 0.5 * w[i];
    }
  }
  // path rule of the Oersted kernel's near offsets: QN_NODES Gauss-Legendre
  // nodes on each of the panels [2^-(p+1), 2^-p], p < QN_PANELS, and
  // [0, 2^-QN_PANELS] of [0, 1]
  constexpr int QN_PANELS = 24, QN_NODES = 20, QN = (QN_PANELS + 1) * QN_NODES;
  std::vector<double> qrule;
  const bool oersted = g.kind == KERNEL_OERSTED;
  if (oersted) {
    double x[QN_NODES], w[QN_NODES];
    gauss_legendre(QN_NODES, x, w);
    qrule.resize(2 * QN);
    for (int p = 0; p <= QN_PANELS; ++p) {
      const double hi = std::ldexp(1.0, -p), lo = p == QN_PANELS ? 0.0 : hi / 2;
      for (int i = 0; i < QN_NODES; ++i) {
        qrule[p * QN_NODES + i] = lo + (hi - lo) * 0.5 * (1.0 + x[i]);
        qrule[QN + p * QN_NODES + i] = (hi - lo) * 0.5 * w[i];
      }
    }
  }
  const int nc = kernel_comps(g);
  const size_t s0 = (size_t)g.nz * g.ny * g.nx;
  const size_t s1 = (size_t)g.nz * g.ny * g.Kx;
  const size_t s2 = (size_t)g.nz * g.Kyh * g.Kx;
  const size_t s3 = (size_t)g.Kzh * g.Kyh * g.Kx;
  size_t smax = s0;
  for (size_t v : {s1, s2, s3}) smax = v > smax ? v : smax;
  double *bufA = nullptr, *bufB = nullptr, *d_trig = nullptr;
  int rc = DEMAG_OK;
  hipError_t e;
  do {
    if (hipMalloc(&bufA, nc * smax * sizeof(double)) != hipSuccess ||
        hipMalloc(&bufB, nc * smax * sizeof(double)) != hipSuccess ||
        hipMalloc(&d_trig, (trig.size() + qrule.size()) * sizeof(double)) != hipSuccess) {
      rc = fail(DEMAG_ENOMEM, "demag_bind: set-up temporaries could not be allocated"); break;
    }
    if ((e = hipMemcpyAsync(d_trig, trig.data(), trig.size() * sizeof(double), hipMemcpyHostToDevice, s)) != hipSuccess) {
      rc = fail_hip(e, "trig upload"); break;
    }
    if (oersted && (e = hipMemcpyAsync(d_trig + trig.size(), qrule.data(), qrule.size() * sizeof(double),
                                       hipMemcpyHostToDevice, s)) != hipSuccess) {
      rc = fail_hip(e, "rule upload"); break;
    }
    const double* cs[3];
    const double* sn[3];
    for (int a = 0; a < 3; ++a) {
      cs[a] = d_trig + (size_t)(2 * a) * Nmax;
      sn[a] = d_trig + (size_t)(2 * a + 1) * Nmax;
    }
    // demagnetizing tensor: component order xx yy zz xy xz yz; odd along x:
    // xy xz; y: xy yz; z: xz yz.  Oersted kernel: x y z, each odd along its own axis.
    const unsigned odd[3] = {oersted ? 0x1u : 0x18u, oersted ? 0x2u : 0x28u, oersted ? 0x4u : 0x30u};
    e = oersted ? launch_oe_tensor(bufA, g, gl, d_trig + trig.size(), d_trig + trig.size() + QN, QN, s)
                : launch_tensor(bufA, g, gl, s);
    if (e != hipSuccess) { rc = fail_hip(e, "tensor kernel"); break; }
    if ((e = launch_axis(bufA, bufB, nc, g.nz * g.ny, g.nx, g.Kx, 1, g.Nx, odd[0], cs[0], sn[0], s)) != hipSuccess) {
      rc = fail_hip(e, "x transform"); break;
    }
    if ((e = launch_axis(bufB, bufA, nc, g.nz, g.ny, g.Kyh, g.Kx, g.Ny, odd[1], cs[1], sn[1], s)) != hipSuccess) {
      rc = fail_hip(e, "y transform"); break;
    }
    if ((e = launch_axis(bufA, bufB, nc, 1, g.nz, g.Kzh, g.Kyh * g.Kx, g.Nz, odd[2], cs[2], sn[2], s)) != hipSuccess) {
      rc = fail_hip(e, "z transform"); break;
    }
    if ((e = launch_pack(bufB, d_K, g, s)) != hipSuccess) { rc = fail_hip(e, "pack"); break; }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) { rc = fail_hip(e, "set-up"); break; }
  } while (false);
  if (bufA) (void)hipFree(bufA);
  if (bufB) (void)hipFree(bufB);
  if (d_trig) (void)hipFree(d_trig);
  return rc;
}

int mark(const demag_plan* p, int i, hipStream_t s) {
  if (!p->timing) return DEMAG_OK;
  hipError_t e = hipEventRecord(p->ev[i], s);
  return e == hipSuccess ? DEMAG_OK : fail_hip(e, "hipEventRecord");
}

// Where a sub-plan's spectrum and energy partials live: the bound work buffer,
// or the same offsets into another base (the static scratch of
// demag_field_noalloc).
struct Slab {
  float2* T;
  double* epart;
};

Slab slab_of(const Sub& sb, char* base) {
  if (!base) return Slab{sb.T, sb.epart};
  return Slab{reinterpret_cast<float2*>(base + sb.t_off), reinterpret_cast<double*>(base + sb.e_off)};
}

// Geometry the x passes run on: the mesh itself (fused x+z passes), or with
// separate z passes the mesh flattened to (nx, ny nz, 1) rows.
Geom xgeom(const Geom& g) {
  if (!g.zsep) return g;
  Geom f = g;
  f.ny = g.ny * g.nz;
  f.nz = 1; f.Nz = 1; f.lnz = 0; f.Kzh = 1;
  f.yg = g.yg_sep;
  f.zsep = 0;
  return f;
}

FwdArgs fwd_args(const demag_plan* p, const Sub& sb, const float* src, const float* Ms, float ms,
                 const float* ms_mesh, const float* src2 = nullptr, float ms2 = 0.f, char* base = nullptr) {
  const Geom& g = sb.g;
  const Geom x = xgeom(g);
  FwdArgs a{src, Ms, ms, slab_of(sb, base).T, p->tw, x.nx, x.ny, x.nz, x.nTiles, x.Kx, x.yg,
            (int)sb.members.size(), p->batch ? sb.moff : nullptr, ms_mesh, spectrum_elems(g),
            p->batch ? sb.gid : nullptr, src2, ms2};
  a.ysplit = g.zsep ? g.ny : 0;
  a.nzp = g.Nz;
  return a;
}

ZArgs z_args(const demag_plan* p, const Sub& sb, char* base = nullptr) {
  const Geom& g = sb.g;
  return ZArgs{slab_of(sb, base).T, p->tw, g.ny, g.nz, g.nTiles, (int)sb.members.size(), spectrum_elems(g)};
}

// The inverse x pass (after the inverse z pass of separate z passes).
int run_inv(const demag_plan* p, const Sub& sb, InvArgs ia, hipStream_t s, char* base = nullptr) {
  const Geom& g = sb.g;
  hipError_t e = hipSuccess;
  if (g.zsep) {
    e = launch_zpass(g.lnz, z_args(p, sb, base), true, s);
    if (e != hipSuccess) return fail_hip(e, "inverse z pass");
    const Geom x = xgeom(g);
    ia.ny = x.ny; ia.nz = 1; ia.yg = x.yg;
    ia.ysplit = g.ny;
    ia.nzp = g.Nz;
    e = launch_inv(x, ia, s);
  } else {
    e = launch_inv(g, ia, s);
  }
  return e == hipSuccess ? DEMAG_OK : fail_hip(e, "inverse pass");
}

MidArgs mid_args(const demag_plan* p, const Sub& sb, bool energy, char* base = nullptr) {
  const Geom& g = sb.g;
  const Slab w = slab_of(sb, base);
  return MidArgs{w.T, sb.K, p->tw, energy ? w.epart : nullptr, g.ny, g.Nz, g.Nx, g.nTiles, g.Kx, g.Kyh, g.Kzh,
                 TILE / mid_kw(g), (int)sb.members.size(), spectrum_elems(g), mid_blocks(g)};
}

// forward and middle passes of one sub-plan (src2: optional second sublattice)
int run_conv(const demag_plan* p, const Sub& sb, const float* src, const float* Ms, float ms,
             const float* ms_mesh, bool energy, hipStream_t s, const float* src2 = nullptr, float ms2 = 0.f,
             char* base = nullptr) {
  const Geom& g = sb.g;
  int rc = mark(p, 0, s);
  if (rc != DEMAG_OK) return rc;
  hipError_t e = launch_fwd(xgeom(g), fwd_args(p, sb, src, Ms, ms, ms_mesh, src2, ms2, base), s);
  if (e != hipSuccess) return fail_hip(e, "forward pass");
  if (g.zsep) {
    e = launch_zpass(g.lnz, z_args(p, sb, base), false, s);
    if (e != hipSuccess) return fail_hip(e, "forward z pass");
  }
  if ((rc = mark(p, 1, s)) != DEMAG_OK) return rc;
  e = launch_mid(g, mid_args(p, sb, energy, base), s);
  if (e != hipSuccess) return fail_hip(e, "middle pass");
  return mark(p, 2, s);
}

// base: NULL for the bound work buffer, else the base of another buffer with
// the same layout (the static scratch of demag_field_noalloc)
int run_field(const demag_plan* p, const float* d_m, const float* d_Ms, float Ms, const float* ms_mesh, float* d_H,
              unsigned flags, double* d_energy, hipStream_t s, const float* d_m2 = nullptr, float Ms2 = 0.f,
              char* base = nullptr) {
  for (const Sub& sb : p->subs) {
    const Geom& g = sb.g;
    const int nb = (int)sb.members.size();
    const Slab w = slab_of(sb, base);
    int rc = run_conv(p, sb, d_m, d_Ms, Ms, ms_mesh, d_energy != nullptr, s, d_m2, Ms2, base);
    if (rc != DEMAG_OK) return rc;
    InvArgs ia{w.T, d_H, p->tw, g.nx, g.ny, g.nz, g.nTiles, g.Kx, g.yg, (flags & DEMAG_ACCUMULATE) ? 1 : 0,
               nullptr, nullptr, 0.0, nullptr, 0.f, 0,
               nb, p->batch ? sb.moff : nullptr, ms_mesh, spectrum_elems(g), p->batch ? sb.gid : nullptr};
    if ((rc = run_inv(p, sb, ia, s, base)) != DEMAG_OK) return rc;
    if ((rc = mark(p, 3, s)) != DEMAG_OK) return rc;
    if (d_energy) {
      const double V = g.dx * g.dy * g.dz;
      const hipError_t e = launch_energy_final(w.epart, mid_blocks(g), -0.5 * MU0 * V, d_energy, s, nb, p->batch ? sb.gid : nullptr);
      if (e != hipSuccess) return fail_hip(e, "energy reduction");
    }
  }
  return DEMAG_OK;
}

int run_backward(const demag_plan* p, const float* d_G, const float* d_Ms, float Ms, const float* ms_mesh,
                 const float* d_H, const double* d_gE, float* d_grad, unsigned flags, hipStream_t s) {
  for (const Sub& sb : p->subs) {
    const Geom& g = sb.g;
    const int nb = (int)sb.members.size();
    int rc = run_conv(p, sb, d_G, nullptr, 1.0f, nullptr, false, s);
    if (rc != DEMAG_OK) return rc;
    const double V = g.dx * g.dy * g.dz;
    InvArgs ia{sb.T, d_grad, p->tw, g.nx, g.ny, g.nz, g.nTiles, g.Kx, g.yg, (flags & DEMAG_ACCUMULATE) ? 1 : 0,
               d_H, d_gE, -MU0 * V, d_Ms, Ms, 1,
               nb, p->batch ? sb.moff : nullptr, ms_mesh, spectrum_elems(g), p->batch ? sb.gid : nullptr};
    if ((rc = run_inv(p, sb, ia, s)) != DEMAG_OK) return rc;
    if ((rc = mark(p, 3, s)) != DEMAG_OK) return rc;
  }
  return DEMAG_OK;
}

// ---------------------------------------------------------------------------
// launch-shape schedules and their tuner
// ---------------------------------------------------------------------------
// A plan has one schedule per part: parts 0 .. subs-1 are the same-geometry
// sub-plans, the following ones the coupled groups.  The tunables are the y
// rows per workgroup of the x passes (sub-plans only), the kx lines per
// workgroup of the middle pass and the radix of its y lines.  Every schedule
// computes the same convolution; they differ in rounding order and speed.

int part_count(const demag_plan* p) { return (int)(p->subs.size() + p->groups.size()); }

Geom& part_geom(demag_plan* p, int i) {
  return i < (int)p->subs.size() ? p->subs[i].g : p->groups[i - p->subs.size()].g;
}

// y rows per workgroup of the active x passes (fused: y lines of nz rows;
// separate z passes: rows of the flattened mesh)
int& active_yg(Geom& g) { return g.zsep ? g.yg_sep : g.yg; }
int active_yg(const Geom& g) { return g.zsep ? g.yg_sep : g.yg; }

bool yg_ok(const Geom& g, int yg) {
  const int rows = g.zsep ? g.ny * g.nz : g.ny;
  const int zr = g.zsep ? 1 : g.nz;
  if (yg < 1 || yg > rows) return false;
  return (size_t)yg * zr * xrow_pitch_rt(g.lnx) * sizeof(float2) + XTAB_BYTES <= 160 * 1024;
}

bool kw_ok(int kw) { return kw == 2 || kw == 4 || kw == 8; }

int line_m(const Geom& g) { return g.Ny > 1 ? g.Ny / 2 : 1; }

bool sched_ok(const Geom& g, int kw, int r) { return mid_schedule_ok(line_m(g), kw, r); }

// Radices the tuner times.  Lines spanning two wavefronts (radix 8 at 1024
// points) stay selectable by demag_set_schedule but are not tuned: timed alone
// the middle pass looked faster with them, inside the field sequence it was
// slower (422 vs 340 us at 1024x1024x4).
std::vector<int> radix_candidates(const Geom& g) {
  const int M = line_m(g);
  std::vector<int> r{line_radix(M)};
  for (int c : {4, 8, 16})
    if (c != r[0] && mid_radix_ok(M, c) && M / c <= 64) r.push_back(c);
  return r;
}

InvArgs inv_plain_args(const demag_plan* p, const Sub& sb, float* d_H, unsigned flags, const float* ms_mesh) {
  const Geom& g = sb.g;
  return InvArgs{sb.T, d_H, p->tw, g.nx, g.ny, g.nz, g.nTiles, g.Kx, g.yg, (flags & DEMAG_ACCUMULATE) ? 1 : 0,
                 nullptr, nullptr, 0.0, nullptr, 0.f, 0,
                 (int)sb.members.size(), p->batch ? sb.moff : nullptr, ms_mesh, spectrum_elems(g),
                 p->batch ? sb.gid : nullptr};
}

// Microseconds per call of fn (a launch sequence on s): two warm-up calls,
// then the best of three timed runs of `reps` calls (reps sized for ~2 ms).
template <class F>
int time_calls(hipStream_t s, F&& fn, double& us) {
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e;
  if ((e = hipEventCreate(&a)) != hipSuccess) return fail_hip(e, "hipEventCreate");
  if ((e = hipEventCreate(&b)) != hipSuccess) {
    (void)hipEventDestroy(a);
    return fail_hip(e, "hipEventCreate");
  }
  auto run = [&](int n) -> int {
    for (int i = 0; i < n; ++i) {
      const int rc = fn();
      if (rc != DEMAG_OK) return rc;
    }
    return DEMAG_OK;
  };
  auto timed = [&](int n, double& t) -> int {
    hipError_t he;
    if ((he = hipEventRecord(a, s)) != hipSuccess) return fail_hip(he, "hipEventRecord");
    const int rc = run(n);
    if (rc != DEMAG_OK) return rc;
    if ((he = hipEventRecord(b, s)) != hipSuccess) return fail_hip(he, "hipEventRecord");
    if ((he = hipEventSynchronize(b)) != hipSuccess) return fail_hip(he, "hipEventSynchronize");
    float ms = 0.f;
    if ((he = hipEventElapsedTime(&ms, a, b)) != hipSuccess) return fail_hip(he, "hipEventElapsedTime");
    t = 1000.0 * ms / n;
    return DEMAG_OK;
  };
  int rc = run(2);
  double t1 = 0.0;
  if (rc == DEMAG_OK) rc = timed(1, t1);
  if (rc == DEMAG_OK) {
    int reps = (int)(2000.0 / (t1 > 1.0 ? t1 : 1.0));
    reps = reps < 3 ? 3 : (reps > 50 ? 50 : reps);
    us = 1e300;
    for (int trial = 0; trial < 3 && rc == DEMAG_OK; ++trial) {
      double t = 0.0;
      rc = timed(reps, t);
      if (rc == DEMAG_OK && t < us) us = t;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return rc;
}

// Measure the candidates of sub-plan sb and keep the fastest in its geometry.
int tune_sub(demag_plan* p, Sub& sb, const float* d_m, float* d_H, hipStream_t s, TuneEntry& out,
             bool keep_form) {
  Geom& g = sb.g;
  // one field sequence without energy: forward x (and z) passes, middle
  // pass, inverse (z and) x passes
  auto sequence = [&]() -> int {
    hipError_t e = launch_fwd(xgeom(g), fwd_args(p, sb, d_m, nullptr, 1.0f, nullptr), s);
    if (e == hipSuccess && g.zsep) e = launch_zpass(g.lnz, z_args(p, sb), false, s);
    if (e == hipSuccess) e = launch_mid(g, mid_args(p, sb, false), s);
    if (e != hipSuccess) return fail_hip(e, "field sequence");
    return run_inv(p, sb, inv_plain_args(p, sb, d_H, 0u, nullptr), s);
  };
  // fused x+z passes or separate z passes, where both exist
  if (!keep_form && fused_ok(g) && zsep_ok(g)) {
    const int z0 = g.zsep;
    double t[2] = {0.0, 0.0};
    for (int z = 0; z < 2; ++z) {
      g.zsep = z;
      const int rc = time_calls(s, sequence, t[z]);
      if (rc != DEMAG_OK) {
        g.zsep = z0;
        return rc;
      }
    }
    g.zsep = t[1] < t[0] ? 1 : 0;
  }
  out.zsep = g.zsep;
  const int d = active_yg(g);
  std::vector<int> ygs;
  for (int c : {d / 2, d, 2 * d, 4 * d})
    if (yg_ok(g, c) && std::find(ygs.begin(), ygs.end(), c) == ygs.end()) ygs.push_back(c);
  double best = 1e300;
  int best_yg = d;
  for (int yg : ygs) {
    active_yg(g) = yg;
    double us = 0.0;
    const int rc = time_calls(s, [&]() -> int {
      const Geom x = xgeom(g);
      hipError_t e = launch_fwd(x, fwd_args(p, sb, d_m, nullptr, 1.0f, nullptr), s);
      if (e == hipSuccess) {
        InvArgs ia = inv_plain_args(p, sb, d_H, 0u, nullptr);
        ia.ny = x.ny; ia.nz = x.nz; ia.yg = x.yg;
        ia.ysplit = g.zsep ? g.ny : 0;
        ia.nzp = g.Nz;
        e = launch_inv(x, ia, s);
      }
      return e == hipSuccess ? DEMAG_OK : fail_hip(e, "x passes");
    }, us);
    if (rc != DEMAG_OK) {
      active_yg(g) = d;
      return rc;
    }
    if (us < best) {
      best = us;
      best_yg = yg;
    }
  }
  active_yg(g) = best_yg;
  out.yg = best_yg;
  out.x_us = best;
  const int kw0 = g.mid_kw, r0 = g.mid_r;
  best = 1e300;
  int best_kw = mid_kw(g), best_r = mid_radix(g);
  for (int kw : {2, 4, 8}) {
    for (int r : radix_candidates(g)) {
      if (!sched_ok(g, kw, r)) continue;
      g.mid_kw = kw;
      g.mid_r = r;
      // timed inside the whole field sequence: alone, the middle pass can
      // rank its candidates differently (cache state, clocks)
      double us = 0.0;
      const int rc = time_calls(s, sequence, us);
      if (rc != DEMAG_OK) {
        g.mid_kw = kw0;
        g.mid_r = r0;
        return rc;
      }
      if (us < best) {
        best = us;
        best_kw = kw;
        best_r = r;
      }
    }
  }
  g.mid_kw = best_kw;
  g.mid_r = best_r;
  out.kw = best_kw;
  out.radix = best_r;
  out.mid_us = best > out.x_us ? best - out.x_us : best;   // the middle pass's share of the sequence
  return DEMAG_OK;
}

// Coupled group: the two split y passes are the tunable ones.
int tune_group(demag_plan* p, Group& G, hipStream_t s, TuneEntry& out) {
  Geom& g = G.g;
  const int kw0 = g.mid_kw, r0 = g.mid_r;
  double best = 1e300;
  int best_kw = mid_kw(g), best_r = mid_radix(g);
  for (int kw : {2, 4, 8}) {
    for (int r : radix_candidates(g)) {
      if (!sched_ok(g, kw, r)) continue;
      g.mid_kw = kw;
      g.mid_r = r;
      double us = 0.0;
      const int rc = time_calls(s, [&]() -> int {
        const MidArgs ma = group_mid_args(p, G);
        hipError_t e = launch_mid_split(g, ma, 1, s);
        if (e == hipSuccess) e = launch_mid_split(g, ma, 2, s);
        return e == hipSuccess ? DEMAG_OK : fail_hip(e, "layer y passes");
      }, us);
      if (rc != DEMAG_OK) {
        g.mid_kw = kw0;
        g.mid_r = r0;
        return rc;
      }
      if (us < best) {
        best = us;
        best_kw = kw;
        best_r = r;
      }
    }
  }
  g.mid_kw = best_kw;
  g.mid_r = best_r;
  out.yg = 0;
  out.kw = best_kw;
  out.radix = best_r;
  out.mid_us = best;
  return DEMAG_OK;
}

std::string part_key(const demag_plan* p, int i, const std::string& dev) {
  char buf[160];
  if (i < (int)p->subs.size()) {
    const Sub& sb = p->subs[i];
    std::snprintf(buf, sizeof buf, "|%s %dx%dx%d nb=%d", sb.g.kind == KERNEL_OERSTED ? "oersted" : "mesh", sb.g.nx,
                  sb.g.ny, sb.g.nz, (int)sb.members.size());
  } else {
    const Group& G = p->groups[i - p->subs.size()];
    std::snprintf(buf, sizeof buf, "|layers %dx%d planes=%d", G.g.nx, G.g.ny, (int)G.planes.size());
  }
  return dev + buf;
}

}  // namespace

extern "C" {

const char* demag_last_error(void) { return g_err.c_str(); }

int demag_setup(demag_plan** out, int nx, int ny, int nz, double dx, double dy, double dz, unsigned pbc_flags,
                int pbc_images) {
  if (!out) return fail(DEMAG_EINVAL, "demag_setup: out is NULL");
  *out = nullptr;
  Geom g;
  if (pbc_flags & ~7u) return fail(DEMAG_EINVAL, "demag_setup: unknown boundary flags");
  if (pbc_flags && pbc_images > MAX_IMAGES)
    return fail(DEMAG_EINVAL, "demag_setup: at most 1000 images per side");
  int rc = make_geom(nx, ny, nz, dx, dy, dz, pbc_flags, pbc_images, g, "demag_setup");
  if (rc != DEMAG_OK) return rc;
  demag_plan* p = new (std::nothrow) demag_plan;
  if (!p) return fail(DEMAG_ENOMEM, "demag_setup: out of host memory");
  Sub sb;
  sb.g = g;
  sb.members = {0};
  p->subs.push_back(sb);
  p->offsets = {0};
  p->total_floats = (size_t)3 * nx * ny * nz;
  layout(p);
  *out = p;
  return DEMAG_OK;
}

int demag_setup_oersted(demag_plan** out, int nx, int ny, int nz, double dx, double dy, double dz, unsigned pbc_flags,
                        int pbc_images) {
  if (!out) return fail(DEMAG_EINVAL, "demag_setup_oersted: out is NULL");
  *out = nullptr;
  Geom g;
  if (pbc_flags & ~7u) return fail(DEMAG_EINVAL, "demag_setup_oersted: unknown boundary flags");
  if (pbc_flags && pbc_images > MAX_IMAGES)
    return fail(DEMAG_EINVAL, "demag_setup_oersted: at most 1000 images per side");
  int rc = make_geom(nx, ny, nz, dx, dy, dz, pbc_flags, pbc_images, g, "demag_setup_oersted");
  if (rc != DEMAG_OK) return rc;
  g.kind = KERNEL_OERSTED;
  demag_plan* p = new (std::nothrow) demag_plan;
  if (!p) return fail(DEMAG_ENOMEM, "demag_setup_oersted: out of host memory");
  Sub sb;
  sb.g = g;
  sb.members = {0};
  p->subs.push_back(sb);
  p->offsets = {0};
  p->total_floats = (size_t)3 * nx * ny * nz;
  p->oersted = true;
  layout(p);
  *out = p;
  return DEMAG_OK;
}

int demag_setup_batch(demag_plan** out, int nmesh, const int* dims, const double* cells, const double* origins,
                      const int* groups, unsigned pbc_flags, int pbc_images) {
  if (!out) return fail(DEMAG_EINVAL, "demag_setup_batch: out is NULL");
  *out = nullptr;
  if (nmesh < 1 || !dims || !cells) return fail(DEMAG_EINVAL, "demag_setup_batch: need nmesh >= 1 and dims/cells");
  if (pbc_flags & ~7u) return fail(DEMAG_EINVAL, "demag_setup_batch: unknown boundary flags");
  if (pbc_flags && pbc_images > MAX_IMAGES)
    return fail(DEMAG_EINVAL, "demag_setup_batch: at most 1000 images per side");
  if ((pbc_flags & DEMAG_PBC_Z) && groups)
    for (int i = 0; i < nmesh; ++i)
      if (groups[i] >= 0)
        return fail(DEMAG_EUNSUPPORTED, "demag_setup_batch: coupled groups take periodic x and y only");
  demag_plan* p = new (std::nothrow) demag_plan;
  if (!p) return fail(DEMAG_ENOMEM, "demag_setup_batch: out of host memory");
  p->batch = true;
  size_t off = 0;
  if (groups && !origins) {
    delete p;
    return fail(DEMAG_EINVAL, "demag_setup_batch: coupled groups need origins");
  }
  for (int i = 0; i < nmesh; ++i) {
    const int nx = dims[3 * i], ny = dims[3 * i + 1], nz = dims[3 * i + 2];
    if (nx < 1 || ny < 1 || nz < 1) {
      delete p;
      return fail(DEMAG_EINVAL, "demag_setup_batch: mesh dimensions must be >= 1");
    }
    p->offsets.push_back((long long)off);
    off += (size_t)3 * nx * ny * nz;
  }
  // coupled groups
  std::vector<bool> coupled(nmesh, false);
  if (groups) {
    std::vector<int> ids;
    for (int i = 0; i < nmesh; ++i)
      if (groups[i] >= 0 && std::find(ids.begin(), ids.end(), groups[i]) == ids.end()) ids.push_back(groups[i]);
    for (int id : ids) {
      std::vector<int> idx;
      for (int i = 0; i < nmesh; ++i)
        if (groups[i] == id) idx.push_back(i);
      Group G;
      const int rc = make_group(idx, dims, cells, origins, p->offsets, pbc_flags,
                                pbc_flags ? (pbc_images > 0 ? pbc_images : DEFAULT_IMAGES) : 0, G);
      if (rc != DEMAG_OK) {
        delete p;
        return rc;
      }
      for (int i : idx) coupled[i] = true;
      p->groups.push_back(G);
    }
  }
  for (int i = 0; i < nmesh; ++i) {
    if (coupled[i]) continue;
    Geom g;
    const int rc = make_geom(dims[3 * i], dims[3 * i + 1], dims[3 * i + 2], cells[3 * i], cells[3 * i + 1],
                             cells[3 * i + 2], pbc_flags, pbc_images, g, "demag_setup_batch");
    if (rc != DEMAG_OK) {
      delete p;
      return rc;
    }
    bool placed = false;
    for (Sub& sb : p->subs) {
      const Geom& h = sb.g;
      if (h.nx == g.nx && h.ny == g.ny && h.nz == g.nz && h.dx == g.dx && h.dy == g.dy && h.dz == g.dz) {
        sb.members.push_back(i);
        placed = true;
        break;
      }
    }
    if (!placed) {
      Sub sb;
      sb.g = g;
      sb.members = {i};
      p->subs.push_back(sb);
    }
  }
  p->total_floats = off;
  layout(p);
  *out = p;
  return DEMAG_OK;
}

int demag_batch_layout(const demag_plan* p, int* nmesh, long long* offsets, size_t* total_floats) {
  if (!p || !nmesh || !total_floats) return fail(DEMAG_EINVAL, "demag_batch_layout: NULL argument");
  *nmesh = (int)p->offsets.size();
  *total_floats = p->total_floats;
  if (offsets)
    for (size_t i = 0; i < p->offsets.size(); ++i) offsets[i] = p->offsets[i];
  return DEMAG_OK;
}

int demag_padded_dims(const demag_plan* p, int* Nx, int* Ny, int* Nz) {
  if (!p || !Nx || !Ny || !Nz) return fail(DEMAG_EINVAL, "demag_padded_dims: NULL argument");
  if (p->batch || p->subs.size() != 1)
    return fail(DEMAG_EINVAL, "demag_padded_dims: a batch plan has one padded size per geometry");
  *Nx = p->subs[0].g.Nx; *Ny = p->subs[0].g.Ny; *Nz = p->subs[0].g.Nz;
  return DEMAG_OK;
}

int demag_buffer_bytes(const demag_plan* p, size_t* kernel_bytes, size_t* work_bytes) {
  if (!p || !kernel_bytes || !work_bytes) return fail(DEMAG_EINVAL, "demag_buffer_bytes: NULL argument");
  *kernel_bytes = p->kernel_bytes;
  *work_bytes = p->work_bytes;
  return DEMAG_OK;
}

int demag_bind(demag_plan* p, void* d_kernel, void* d_work, void* stream) {
  if (!p) return fail(DEMAG_EINVAL, "demag_bind: plan is NULL");
  if (p->bound) return fail(DEMAG_ESTATE, "demag_bind: plan is already bound");
  if (!d_kernel) return fail(DEMAG_EINVAL, "demag_bind: NULL kernel buffer");
  if (!d_work && (p->batch || p->oersted))
    return fail(DEMAG_EINVAL, "demag_bind: only single-mesh demagnetizing plans may be bound without a work buffer");
  if (!aligned(d_kernel) || (d_work && !aligned(d_work)))
    return fail(DEMAG_EINVAL, "demag_bind: buffers must be 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
  {
    const int rc = noalloc_scratch(p->device, &p->noalloc_work);
    if (rc != DEMAG_OK) return rc;
  }
  char* kb = static_cast<char*>(d_kernel);
  char* wb = static_cast<char*>(d_work);

  // twiddles W_4096^k in FP64, rounded once to FP32
  std::vector<float2> tw(TW_SIZE);
  for (int k = 0; k < TW_SIZE; ++k) {
    const double ang = -2.0 * M_PI * k / TW_SIZE;
    tw[k] = make_float2((float)std::cos(ang), (float)std::sin(ang));
  }
  if ((e = hipMemcpyAsync(kb, tw.data(), TW_SIZE * sizeof(float2), hipMemcpyHostToDevice, s)) != hipSuccess)
    return fail_hip(e, "twiddle upload");
  for (Sub& sb : p->subs) {
    sb.K = reinterpret_cast<float*>(kb + sb.k_off);
    sb.moff = reinterpret_cast<long long*>(kb + sb.tab_off);
    sb.gid = reinterpret_cast<int*>(kb + sb.tab_off + align256(sb.members.size() * sizeof(long long)));
    sb.T = wb ? reinterpret_cast<float2*>(wb + sb.t_off) : nullptr;
    sb.epart = wb ? reinterpret_cast<double*>(wb + sb.e_off) : nullptr;
    std::vector<long long> mo;
    for (int m : sb.members) mo.push_back(p->offsets[m]);
    if ((e = hipMemcpyAsync(sb.moff, mo.data(), mo.size() * sizeof(long long), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(sb.gid, sb.members.data(), sb.members.size() * sizeof(int), hipMemcpyHostToDevice, s)) !=
            hipSuccess)
      return fail_hip(e, "batch table upload");
    const int rc = build_spectrum(sb.g, sb.K, s);
    if (rc != DEMAG_OK) return rc;
  }
  p->tw = reinterpret_cast<float2*>(kb);
  for (Group& G : p->groups) {
    G.K = reinterpret_cast<float*>(kb + G.k_off);
    G.pl = reinterpret_cast<PlaneInfo*>(kb + G.pl_off);
    G.T = reinterpret_cast<float2*>(wb + G.t_off);
    G.S = reinterpret_cast<float2*>(wb + G.s_off);
    G.epart = reinterpret_cast<double*>(wb + G.e_off);
    if ((e = hipMemcpyAsync(G.pl, G.planes.data(), G.planes.size() * sizeof(PlaneInfo), hipMemcpyHostToDevice, s)) !=
        hipSuccess)
      return fail_hip(e, "plane table upload");
    const int rc = build_group(G, s);
    if (rc != DEMAG_OK) return rc;
  }
  p->bound = true;
  p->has_work = wb != nullptr;
  return DEMAG_OK;
}

int demag_field(const demag_plan* p, const float* d_m, const float* d_Ms, float Ms, float* d_H, unsigned flags,
                double* d_energy, void* stream) {
  if (!p) return fail(DEMAG_EINVAL, "demag_field: plan is NULL");
  if (p->oersted) return fail(DEMAG_EINVAL, "demag_field: an Oersted plan (use demag_oersted_field)");
  if (p->batch) return fail(DEMAG_EINVAL, "demag_field: batch plans use demag_field_batch");
  if (!p->bound) return fail(DEMAG_ESTATE, "demag_field: plan is not bound");
  if (!p->has_work) return fail(DEMAG_ESTATE, "demag_field: plan was bound without a work buffer");
  if (!d_m || !d_H) return fail(DEMAG_EINVAL, "demag_field: NULL m or H");
  if (flags & ~(unsigned)DEMAG_ACCUMULATE) return fail(DEMAG_EINVAL, "demag_field: unknown flags");
  if (!d_Ms && !std::isfinite(Ms)) return fail(DEMAG_EINVAL, "demag_field: Ms is not finite");
  return run_field(p, d_m, d_Ms, Ms, nullptr, d_H, flags, d_energy, static_cast<hipStream_t>(stream));
}

int demag_field_noalloc(const demag_plan* p, const float* d_m, const float* d_Ms, float Ms, float* d_H,
                        unsigned flags, double* d_energy, void* stream) {
  if (!p) return fail(DEMAG_EINVAL, "demag_field_noalloc: plan is NULL");
  if (p->oersted) return fail(DEMAG_EINVAL, "demag_field_noalloc: an Oersted plan");
  if (p->batch) return fail(DEMAG_EINVAL, "demag_field_noalloc: single-mesh plans only");
  if (p->work_bytes > (size_t)DEMAG_NOALLOC_WORK_BYTES)
    return fail(DEMAG_EUNSUPPORTED, "demag_field_noalloc: the plan needs " + std::to_string(p->work_bytes) +
                                        " bytes of work space, more than the " +
                                        std::to_string((size_t)DEMAG_NOALLOC_WORK_BYTES) + " of the static scratch");
  if (!p->bound) return fail(DEMAG_ESTATE, "demag_field_noalloc: plan is not bound");
  if (!d_m || !d_H) return fail(DEMAG_EINVAL, "demag_field_noalloc: NULL m or H");
  if (flags & ~(unsigned)DEMAG_ACCUMULATE) return fail(DEMAG_EINVAL, "demag_field_noalloc: unknown flags");
  if (!d_Ms && !std::isfinite(Ms)) return fail(DEMAG_EINVAL, "demag_field_noalloc: Ms is not finite");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
  if (dev != p->device) return fail(DEMAG_EINVAL, "demag_field_noalloc: the current device is not the plan's");
  return run_field(p, d_m, d_Ms, Ms, nullptr, d_H, flags, d_energy, static_cast<hipStream_t>(stream), nullptr, 0.f,
                   p->noalloc_work);
}

int demag_oersted_field(const demag_plan* p, const float* d_J, float scale, float* d_H, unsigned flags,
                        void* stream) {
  if (!p) return fail(DEMAG_EINVAL, "demag_oersted_field: plan is NULL");
  if (!p->oersted) return fail(DEMAG_EINVAL, "demag_oersted_field: not an Oersted plan (use demag_setup_oersted)");
  if (!p->bound) return fail(DEMAG_ESTATE, "demag_oersted_field: plan is not bound");
  if (!p->has_work) return fail(DEMAG_ESTATE, "demag_oersted_field: plan was bound without a work buffer");
  if (!d_J || !d_H) return fail(DEMAG_EINVAL, "demag_oersted_field: NULL J or H");
  if (flags & ~(unsigned)DEMAG_ACCUMULATE) return fail(DEMAG_EINVAL, "demag_oersted_field: unknown flags");
  if (!std::isfinite(scale)) return fail(DEMAG_EINVAL, "demag_oersted_field: scale is not finite");
  return run_field(p, d_J, nullptr, scale, nullptr, d_H, flags, nullptr, static_cast<hipStream_t>(stream));
}

int demag_field_2sub(const demag_plan* p, const float* d_mA, const float* d_mB, float MsA, float MsB, float* d_H,
                     unsigned flags, double* d_energy, void* stream) {
  if (!p) return fail(DEMAG_EINVAL, "demag_field_2sub: plan is NULL");
  if (p->oersted) return fail(DEMAG_EINVAL, "demag_field_2sub: an Oersted plan");
  if (p->batch) return fail(DEMAG_EINVAL, "demag_field_2sub: single-mesh plans only");
  if (!p->bound) return fail(DEMAG_ESTATE, "demag_field_2sub: plan is not bound");
  if (!p->has_work) return fail(DEMAG_ESTATE, "demag_field_2sub: plan was bound without a work buffer");
  if (!d_mA || !d_mB || !d_H) return fail(DEMAG_EINVAL, "demag_field_2sub: NULL mA, mB or H");
  if (flags & ~(unsigned)DEMAG_ACCUMULATE) return fail(DEMAG_EINVAL, "demag_field_2sub: unknown flags");
  if (!std::isfinite(MsA) || !std::isfinite(MsB)) return fail(DEMAG_EINVAL, "demag_field_2sub: Ms is not finite");
  return run_field(p, d_mA, nullptr, MsA, nullptr, d_H, flags, d_energy, static_cast<hipStream_t>(stream), d_mB,
                   MsB);
}

int demag_field_batch(const demag_plan* p, const float* d_m, const float* d_Ms_mesh, float Ms, float* d_H,
                      unsigned flags, double* d_energy, void* stream) {
  if (!p) return fail(DEMAG_EINVAL, "demag_field_batch: plan is NULL");
  if (!p->batch) return fail(DEMAG_EINVAL, "demag_field_batch: not a batch plan");
  if (!p->bound) return fail(DEMAG_ESTATE, "demag_field_batch: plan is not bound");
  if (!p->has_work) return fail(DEMAG_ESTATE, "demag_field_batch: plan was bound without a work buffer");
  if (!d_m || !d_H) return fail(DEMAG_EINVAL, "demag_field_batch: NULL m or H");
  if (flags & ~(unsigned)DEMAG_ACCUMULATE) return fail(DEMAG_EINVAL, "demag_field_batch: unknown flags");
  if (!d_Ms_mesh && !std::isfinite(Ms)) return fail(DEMAG_EINVAL, "demag_field_batch: Ms is not finite");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int rc = run_field(p, d_m, nullptr, Ms, d_Ms_mesh, d_H, flags, d_energy, s);
  if (rc != DEMAG_OK) return rc;
  return run_groups(p, d_m, d_Ms_mesh, Ms, d_H, flags, d_energy, false, nullptr, nullptr, s);
}

int demag_energy(const demag_plan* p, const float* d_m, const float* d_Ms, float Ms, const float* d_H,
                 double* d_energy, void* stream) {
  if (!p) return fail(DEMAG_EINVAL, "demag_energy: plan is NULL");
  if (p->oersted) return fail(DEMAG_EINVAL, "demag_energy: an Oersted plan");
  if (p->batch) return fail(DEMAG_EINVAL, "demag_energy: single-mesh plans only");
  if (!p->bound) return fail(DEMAG_ESTATE, "demag_energy: plan is not bound");
  if (!p->has_work) return fail(DEMAG_ESTATE, "demag_energy: plan was bound without a work buffer");
  if (!d_m || !d_H || !d_energy) return fail(DEMAG_EINVAL, "demag_energy: NULL argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Sub& sb = p->subs[0];
  const Geom& g = sb.g;
  const size_t ncell = (size_t)g.nx * g.ny * g.nz;
  hipError_t e = launch_energy_cells(d_m, d_Ms, Ms, d_H, ncell, sb.epart, s);
  if (e != hipSuccess) return fail_hip(e, "energy partials");
  const double V = g.dx * g.dy * g.dz;
  e = launch_energy_final(sb.epart, energy_cell_blocks(ncell), -0.5 * MU0 * V, d_energy, s);
  if (e != hipSuccess) return fail_hip(e, "energy reduction");
  return DEMAG_OK;
}

int demag_backward(const demag_plan* p, const float* d_G, const float* d_Ms, float Ms, const float* d_H,
                   const double* d_gE, float* d_grad_m, unsigned flags, void* stream) {
  if (!p) return fail(DEMAG_EINVAL, "demag_backward: plan is NULL");
  if (p->oersted) return fail(DEMAG_EINVAL, "demag_backward: an Oersted plan (its operator is self-adjoint: "
                                            "demag_oersted_field is its own backward)");
  if (p->batch) return fail(DEMAG_EINVAL, "demag_backward: batch plans use demag_backward_batch");
  if (!p->bound) return fail(DEMAG_ESTATE, "demag_backward: plan is not bound");
  if (!p->has_work) return fail(DEMAG_ESTATE, "demag_backward: plan was bound without a work buffer");
  if (!d_G || !d_grad_m) return fail(DEMAG_EINVAL, "demag_backward: NULL G or grad_m");
  if (d_gE && !d_H) return fail(DEMAG_EINVAL, "demag_backward: the energy term needs the forward field H");
  if (flags & ~(unsigned)DEMAG_ACCUMULATE) return fail(DEMAG_EINVAL, "demag_backward: unknown flags");
  return run_backward(p, d_G, d_Ms, Ms, nullptr, d_H, d_gE, d_grad_m, flags, static_cast<hipStream_t>(stream));
}

int demag_backward_batch(const demag_plan* p, const float* d_G, const float* d_Ms_mesh, float Ms, const float* d_H,
                         const double* d_gE, float* d_grad_m, unsigned flags, void* stream) {
  if (!p) return fail(DEMAG_EINVAL, "demag_backward_batch: plan is NULL");
  if (!p->batch) return fail(DEMAG_EINVAL, "demag_backward_batch: not a batch plan");
  if (!p->bound) return fail(DEMAG_ESTATE, "demag_backward_batch: plan is not bound");
  if (!p->has_work) return fail(DEMAG_ESTATE, "demag_backward_batch: plan was bound without a work buffer");
  if (!d_G || !d_grad_m) return fail(DEMAG_EINVAL, "demag_backward_batch: NULL G or grad_m");
  if (d_gE && !d_H) return fail(DEMAG_EINVAL, "demag_backward_batch: the energy term needs the forward field H");
  if (flags & ~(unsigned)DEMAG_ACCUMULATE) return fail(DEMAG_EINVAL, "demag_backward_batch: unknown flags");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int rc = run_backward(p, d_G, nullptr, Ms, d_Ms_mesh, d_H, d_gE, d_grad_m, flags, s);
  if (rc != DEMAG_OK) return rc;
  return run_groups(p, d_G, d_Ms_mesh, Ms, d_grad_m, flags, nullptr, true, d_H, d_gE, s);
}

int demag_set_timing_events(demag_plan* p, void* const* events, int count) {
  if (!p) return fail(DEMAG_EINVAL, "demag_set_timing_events: plan is NULL");
  if (!events || count == 0) {
    p->timing = false;
    return DEMAG_OK;
  }
  if (count != 4) return fail(DEMAG_EINVAL, "demag_set_timing_events: expected 4 events");
  for (int i = 0; i < 4; ++i) {
    if (!events[i]) return fail(DEMAG_EINVAL, "demag_set_timing_events: NULL event");
    p->ev[i] = static_cast<hipEvent_t>(events[i]);
  }
  p->timing = true;
  return DEMAG_OK;
}

int demag_schedule_count(const demag_plan* p, int* nparts) {
  if (!p || !nparts) return fail(DEMAG_EINVAL, "demag_schedule_count: NULL argument");
  *nparts = part_count(p);
  return DEMAG_OK;
}

int demag_get_schedule(const demag_plan* p, int part, int* yg, int* kw, int* radix) {
  if (!p || !yg || !kw || !radix) return fail(DEMAG_EINVAL, "demag_get_schedule: NULL argument");
  if (part < 0 || part >= part_count(p)) return fail(DEMAG_EINVAL, "demag_get_schedule: part out of range");
  const Geom& g = part_geom(const_cast<demag_plan*>(p), part);
  *yg = part < (int)p->subs.size() ? active_yg(g) : 0;
  *kw = mid_kw(g);
  *radix = mid_radix(g);
  return DEMAG_OK;
}

int demag_get_z_passes(const demag_plan* p, int part, int* separate) {
  if (!p || !separate) return fail(DEMAG_EINVAL, "demag_get_z_passes: NULL argument");
  if (part < 0 || part >= part_count(p)) return fail(DEMAG_EINVAL, "demag_get_z_passes: part out of range");
  *separate = part_geom(const_cast<demag_plan*>(p), part).zsep;
  return DEMAG_OK;
}

int demag_set_z_passes(demag_plan* p, int part, int separate) {
  if (!p) return fail(DEMAG_EINVAL, "demag_set_z_passes: plan is NULL");
  if (part < 0 || part >= part_count(p)) return fail(DEMAG_EINVAL, "demag_set_z_passes: part out of range");
  if (separate != 0 && separate != 1) return fail(DEMAG_EINVAL, "demag_set_z_passes: separate must be 0 or 1");
  if (part >= (int)p->subs.size())
    return fail(DEMAG_EUNSUPPORTED, "demag_set_z_passes: coupled groups have no z transform");
  Geom& g = part_geom(p, part);
  if (separate ? !zsep_ok(g) : !fused_ok(g))
    return fail(DEMAG_EUNSUPPORTED, separate ? "demag_set_z_passes: separate z passes need 2 <= nz <= 256"
                                             : "demag_set_z_passes: this mesh is too deep for the fused x+z passes");
  g.zsep = separate;
  return DEMAG_OK;
}

int demag_set_schedule(demag_plan* p, int part, int yg, int kw, int radix) {
  if (!p) return fail(DEMAG_EINVAL, "demag_set_schedule: plan is NULL");
  if (part < 0 || part >= part_count(p)) return fail(DEMAG_EINVAL, "demag_set_schedule: part out of range");
  Geom& g = part_geom(p, part);
  const bool sub = part < (int)p->subs.size();
  if (yg != 0 && (!sub || !yg_ok(g, yg)))
    return fail(DEMAG_EINVAL, sub ? "demag_set_schedule: yg must be in 1..ny and fit the x pass in 160 KiB of LDS"
                                  : "demag_set_schedule: coupled groups take yg = 0");
  if (kw != 0 && !kw_ok(kw)) return fail(DEMAG_EINVAL, "demag_set_schedule: kw must be 2, 4 or 8");
  if (radix != 0 && !mid_radix_ok(line_m(g), radix))
    return fail(DEMAG_EUNSUPPORTED, "demag_set_schedule: radix not available for this y length");
  if (!sched_ok(g, kw ? kw : mid_kw(g), radix ? radix : mid_radix(g)))
    return fail(DEMAG_EUNSUPPORTED, "demag_set_schedule: this kw and radix need more than 128 registers per lane");
  if (yg) active_yg(g) = yg;
  if (kw) g.mid_kw = kw;
  if (radix) g.mid_r = radix;
  return DEMAG_OK;
}

int demag_autotune(demag_plan* p, const float* d_m, float* d_H, const char* cache_path, unsigned flags,
                   int* measured, void* stream) {
  if (!p) return fail(DEMAG_EINVAL, "demag_autotune: plan is NULL");
  if (flags & ~(unsigned)(DEMAG_TUNE_FORCE | DEMAG_TUNE_KEEP_FORM))
    return fail(DEMAG_EINVAL, "demag_autotune: unknown flags");
  const bool keep_form = (flags & DEMAG_TUNE_KEEP_FORM) != 0;
  if (measured) *measured = 0;
  TuneMap cache;
  std::string err;
  if (cache_path && !tune_cache_read(cache_path, cache, err)) return fail(DEMAG_EINVAL, "demag_autotune: " + err);
  int dev = p->device;
  hipError_t e;
  if (dev < 0 && (e = hipGetDevice(&dev)) != hipSuccess) return fail_hip(e, "hipGetDevice");
  hipDeviceProp_t prop;
  if ((e = hipGetDeviceProperties(&prop, dev)) != hipSuccess) return fail_hip(e, "hipGetDeviceProperties");
  const std::string devkey = std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount) + "CU";
  hipStream_t s = static_cast<hipStream_t>(stream);
  int nmeas = 0;
  for (int i = 0; i < part_count(p); ++i) {
    const std::string key = part_key(p, i, devkey);
    const bool sub = i < (int)p->subs.size();
    auto it = cache.find(key);
    // with the z form kept, an entry for the other form does not apply
    const bool other_form = it != cache.end() && keep_form && sub && it->second.zsep >= 0 &&
                            it->second.zsep != p->subs[i].g.zsep;
    if (it != cache.end() && !(flags & DEMAG_TUNE_FORCE) && !other_form) {
      const TuneEntry& c = it->second;
      Geom& g = part_geom(p, i);
      const int z0 = g.zsep;
      if (c.zsep >= 0) {
        if (!sub || c.zsep > 1 || (c.zsep ? !zsep_ok(g) : !fused_ok(g)))
          return fail(DEMAG_EINVAL, "demag_autotune: cache entry '" + key + "' holds an unsupported z mode");
        g.zsep = c.zsep;
      }
      if ((sub ? !yg_ok(g, c.yg) : c.yg != 0) || !sched_ok(g, c.kw, c.radix)) {
        g.zsep = z0;
        return fail(DEMAG_EINVAL, "demag_autotune: cache entry '" + key + "' holds an unsupported schedule");
      }
      if (sub) active_yg(g) = c.yg;
      g.mid_kw = c.kw;
      g.mid_r = c.radix;
      continue;
    }
    if (!p->bound) return fail(DEMAG_ESTATE, "demag_autotune: measuring needs a bound plan");
    if (!p->has_work) return fail(DEMAG_ESTATE, "demag_autotune: plan was bound without a work buffer");
    if (sub && (!d_m || !d_H)) return fail(DEMAG_EINVAL, "demag_autotune: measuring needs m and H buffers");
    TuneEntry t;
    const int rc = sub ? tune_sub(p, p->subs[i], d_m, d_H, s, t, keep_form)
                       : tune_group(p, p->groups[i - p->subs.size()], s, t);
    if (rc != DEMAG_OK) return rc;
    cache[key] = t;
    ++nmeas;
  }
  if (measured) *measured = nmeas;
  if (cache_path && nmeas > 0 && !tune_cache_write(cache_path, cache, err))
    return fail(DEMAG_EINVAL, "demag_autotune: " + err);
  return DEMAG_OK;
}

int demag_llg_workspace_bytes(const demag_plan* p, size_t* bytes) {
  if (!p || !bytes) return fail(DEMAG_EINVAL, "demag_llg_workspace_bytes: NULL argument");
  if (p->oersted) return fail(DEMAG_EINVAL, "demag_llg_workspace_bytes: an Oersted plan");
  if (p->batch) return fail(DEMAG_EINVAL, "demag_llg_workspace_bytes: single-mesh plans only");
  const Geom& g = p->subs[0].g;
  *bytes = 4 * align256((size_t)3 * g.nx * g.ny * g.nz * sizeof(float));
  return DEMAG_OK;
}

int demag_llg_rk4(const demag_plan* p, float* d_m, const demag_llg_params* prm, void* d_work, void* stream) {
  if (!p || !d_m || !prm || !d_work) return fail(DEMAG_EINVAL, "demag_llg_rk4: NULL argument");
  if (p->oersted) return fail(DEMAG_EINVAL, "demag_llg_rk4: an Oersted plan");
  if (p->batch) return fail(DEMAG_EINVAL, "demag_llg_rk4: single-mesh plans only");
  if (!p->bound) return fail(DEMAG_ESTATE, "demag_llg_rk4: plan is not bound");
  if (!p->has_work) return fail(DEMAG_ESTATE, "demag_llg_rk4: plan was bound without a work buffer");
  if (!aligned(d_work)) return fail(DEMAG_EINVAL, "demag_llg_rk4: workspace must be 256-byte aligned");
  const float vals[8] = {prm->Ms, prm->A, prm->alpha, prm->gamma, prm->dt, prm->Hext[0], prm->Hext[1], prm->Hext[2]};
  for (float v : vals)
    if (!std::isfinite(v)) return fail(DEMAG_EINVAL, "demag_llg_rk4: parameters must be finite");
  if (!(prm->Ms > 0.f) || !(prm->dt > 0.f) || prm->A < 0.f || prm->alpha < 0.f)
    return fail(DEMAG_EINVAL, "demag_llg_rk4: need Ms > 0, dt > 0, A >= 0, alpha >= 0");
  const Geom& g = p->subs[0].g;
  const size_t n = (size_t)g.nx * g.ny * g.nz;
  const size_t vb = align256(3 * n * sizeof(float));
  char* w = static_cast<char*>(d_work);
  float* sA = reinterpret_cast<float*>(w);
  float* sB = reinterpret_cast<float*>(w + vb);
  float* acc = reinterpret_cast<float*>(w + 2 * vb);
  float* H = reinterpret_cast<float*>(w + 3 * vb);
  const double gamma = prm->gamma > 0.f ? (double)prm->gamma : MU0 * 1.76085963023e11;
  const double alpha = prm->alpha;
  LlgArgs la{};
  la.m0 = d_m;
  la.acc = acc;
  la.nx = g.nx; la.ny = g.ny; la.nz = g.nz;
  la.pbc = g.pbc;
  la.ihx2 = (float)(1.0 / (g.dx * g.dx));
  la.ihy2 = (float)(1.0 / (g.dy * g.dy));
  la.ihz2 = (float)(1.0 / (g.dz * g.dz));
  la.cex = (float)(2.0 * prm->A / (MU0 * prm->Ms));
  la.hx = prm->Hext[0]; la.hy = prm->Hext[1]; la.hz = prm->Hext[2];
  la.gp = (float)(gamma / (1.0 + alpha * alpha));
  la.alpha = prm->alpha;
  la.dt = prm->dt;
  la.Hd = H;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // stage inputs: m, sA, sB, sA; stage 3 writes the new state over m
  const float* in[4] = {d_m, sA, sB, sA};
  float* nxt[3] = {sA, sB, sA};
  for (int st = 0; st < 4; ++st) {
    int rc = run_field(p, in[st], nullptr, prm->Ms, nullptr, H, 0u, nullptr, s);
    if (rc != DEMAG_OK) return rc;
    la.mi = in[st];
    la.stage = st;
    la.next = st < 3 ? nxt[st] : nullptr;
    la.mout = st == 3 ? d_m : nullptr;
    const hipError_t e = launch_llg_stage(la, s);
    if (e != hipSuccess) return fail_hip(e, "LLG stage");
  }
  return DEMAG_OK;
}

int demag_stream_copy(const void* d_src, void* d_dst, size_t bytes, void* stream) {
  if (!d_src || !d_dst) return fail(DEMAG_EINVAL, "demag_stream_copy: NULL buffer");
  if ((bytes & 15) || (reinterpret_cast<uintptr_t>(d_src) & 15) || (reinterpret_cast<uintptr_t>(d_dst) & 15))
    return fail(DEMAG_EINVAL, "demag_stream_copy: pointers and size must be multiples of 16 bytes");
  const hipError_t e = launch_stream_copy(d_src, d_dst, bytes, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? DEMAG_OK : fail_hip(e, "stream copy");
}

int demag_destroy(demag_plan* p) {
  delete p;
  return DEMAG_OK;
}

}  // extern "C"
