// Host launchers of the demagnetizing-field kernels.
#pragma once
#include <hip/hip_runtime.h>
#include "plan.hpp"

namespace demag {

hipError_t launch_fwd(const Geom& g, const FwdArgs& a, hipStream_t s);
hipError_t launch_mid(const Geom& g, const MidArgs& a, hipStream_t s);
hipError_t launch_zpass(int lnz, const ZArgs& a, bool inverse, hipStream_t s);
hipError_t launch_inv(const Geom& g, const InvArgs& a, hipStream_t s);
hipError_t launch_energy_final(const double* part, int n, double scale, double* out, hipStream_t s, int nb = 1,
                               const int* gid = nullptr);
hipError_t launch_energy_cells(const float* m, const float* Ms, float ms, const float* H, size_t ncell,
                               double* part, hipStream_t s);
hipError_t launch_mid_split(const Geom& g, const MidArgs& a, int mode, hipStream_t s);
hipError_t launch_layer_x(int lnx, const LayerArgs& a, bool inverse, hipStream_t s);
hipError_t launch_couple(int P, const CoupleArgs& a, hipStream_t s);
hipError_t launch_layer_energy(const double* part, int nblk, int P, const PlaneInfo* pl, double scale, double* out,
                               hipStream_t s);
int couple_blocks(int Kx, int NY);
int mid_kw(const Geom& g);
int mid_blocks(const Geom& g);
int mid_blocks_max(const Geom& g);
int mid_radix(const Geom& g);
int energy_cell_blocks(size_t ncell);

hipError_t launch_tensor(double* out, const Geom& g, const GLTable& gl, hipStream_t s);
hipError_t launch_axis(const double* in, double* out, int nc, int outer, int nin, int nout, int inner, int npad,
                       unsigned odd_mask, const double* cs, const double* sn, hipStream_t s);
hipError_t launch_pack(const double* in, float* K, const Geom& g, hipStream_t s);
hipError_t launch_oe_tensor(double* out, const Geom& g, const GLTable& gl, const double* qs, const double* qw, int nq,
                            hipStream_t s);
hipError_t launch_pair_tensor(double2* out, const PairGeom& pg, const GLTable& gl, hipStream_t s);
hipError_t launch_fft64(double2* data, int logN, long long es, long long ls, int lpb, long long bstride, int nlines,
                        const double2* tw64, hipStream_t s);
hipError_t launch_pair_pack(const double2* in, float* K, int Nx, int Ny, int Kx, double scale, int parity,
                            hipStream_t s);
hipError_t launch_llg_stage(const LlgArgs& a, hipStream_t s);
hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s);

}  // namespace demag
