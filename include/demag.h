/*
 * demag.h - C ABI of the MI355X demagnetizing-field library.
 *
 * Computes H_d = -N * M on a regular finite-difference mesh: the
 * demagnetizing-field term of Table 1 (H(r0) = -sum_r N(r - r0) M(r), N the
 * cell-averaged Newell tensor) and the single-mesh form of Sec. 3, Eq. 4,
 * evaluated with the convolution theorem on a zero-padded grid (Sec. 7: 1D
 * transforms along x, y and z, point-wise product with the transformed
 * kernel, inverse transforms; the z transform, product and inverse z
 * transform fused into one pass, the paper's pipelined convolution).  The
 * energy follows from the field/energy relation of Appendix A,
 * E = -(mu0/2) V sum_cells M . H.
 *
 * Conventions
 *  - Every function returns DEMAG_OK (0) or a negative status; no other error
 *    channel crosses the ABI.  demag_last_error() gives a message for the
 *    calling thread's last failure.
 *  - Arguments and sizes are checked on the host before any HIP call.
 *  - Device pointers are allocated and owned by the caller; the library never
 *    frees them.  `stream` is a hipStream_t (NULL = the default stream).
 *  - demag_field(_batch), demag_energy and demag_backward(_batch) only
 *    enqueue work on `stream`: they neither allocate nor synchronize, so a
 *    caller may capture them in a HIP graph and replay it.  Calls that share a
 *    plan share its work buffer and must be ordered on one stream.
 *  - Arrays of vectors are SoA [3][nz][ny][nx], x fastest, FP32.  Lengths in
 *    metres, M and H in A/m, energies in joules (FP64).
 *  - Supported sizes: 1 <= nx <= 2048, 1 <= ny <= 1024, 1 <= nz <= 256; each
 *    axis zero-padded to the next power of two >= 2n-1.  Short z lines are
 *    transformed inside the x passes, long ones by separate z passes
 *    (demag_set_z_passes).
 *  - Periodic boundaries (Sec. 3, multiple images): along a periodic axis a
 *    (period L_a = n_a h_a) the mesh is repeated pbc_images times on either
 *    side and the field is that of the repeated mesh in its central copy,
 *    H_i = -sum_j sum_{|k_a| <= K} N(r_i - r_j - k o L) M_j.  The tensor is
 *    summed over the images at set-up; the field passes are those of open
 *    boundaries.  All three axes periodic sums the cube of images, a
 *    conditionally convergent sum whose value depends on that shape.
 */
#ifndef DEMAG_H
#define DEMAG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct demag_plan demag_plan;

enum {
  DEMAG_OK = 0,
  DEMAG_EINVAL = -1,        /* invalid argument (null pointer, bad size, NaN cell) */
  DEMAG_EUNSUPPORTED = -2,  /* valid but not supported (size limits, group shapes) */
  DEMAG_ENOMEM = -3,        /* host or set-up device allocation failed */
  DEMAG_EHIP = -4,          /* a HIP runtime call failed */
  DEMAG_ESTATE = -5         /* wrong call order (field before bind, bind twice) */
};

enum { DEMAG_PBC_X = 1, DEMAG_PBC_Y = 2, DEMAG_PBC_Z = 4 };
enum { DEMAG_ACCUMULATE = 1 };   /* H += H_d instead of H = H_d */

/* Validate a mesh of nx*ny*nz cells of size dx*dy*dz metres and create a plan
 * (host memory only, no HIP call).  pbc_flags: OR of DEMAG_PBC_* (periodic
 * axes); pbc_images: images K on either side of each periodic axis (<= 0: 10;
 * more than 1000: DEMAG_EINVAL), ignored without periodic axes.  Set-up cost
 * grows with (2K+1)^(periodic axes).  On success *out owns the plan (free
 * with demag_destroy). */
int demag_setup(demag_plan** out, int nx, int ny, int nz, double dx, double dy, double dz,
                unsigned pbc_flags, int pbc_images);

/* Padded FFT lengths of a single-mesh plan: powers of two >= 2n-1, or 1 for
 * n = 1 (Sec. 7: zero padding to double the size; periodic axes are padded
 * too, their image-summed tensor is convolved like an open one).  A batch
 * plan has one padded size per geometry: DEMAG_EINVAL. */
int demag_padded_dims(const demag_plan* plan, int* Nx, int* Ny, int* Nz);

/* Bytes of the two device buffers the caller provides to demag_bind:
 * kernel_bytes - twiddle table and the FP32 kernel spectrum (read-only after
 *                bind);
 * work_bytes   - the padded spectrum of M and energy partials (scratch that
 *                every field call overwrites). */
int demag_buffer_bytes(const demag_plan* plan, size_t* kernel_bytes, size_t* work_bytes);

/* Attach the caller's buffers (256-byte aligned device memory on the current
 * device) and build the kernel spectrum on `stream`: the Newell tensor in FP64
 * (Sec. 3 Eq. 4; Table 1), its transform on the padded grid in FP64, stored in
 * FP32 with the factor -1/(Nx Ny Nz).  Set-up only: allocates FP64
 * temporaries, synchronizes `stream` and frees them before returning.  A plan
 * binds once (DEMAG_ESTATE otherwise).  d_work may be NULL for a
 * single-mesh demagnetizing plan: it can then be used only with
 * demag_field_noalloc (every call that needs the work buffer returns
 * DEMAG_ESTATE). */
int demag_bind(demag_plan* plan, void* d_kernel, void* d_work, void* stream);

/* H_d = -N * M with M = Ms * m (Table 1, demagnetizing field).  d_m: unit
 * magnetization [3][nz][ny][nx]; d_Ms: per-cell saturation magnetization
 * [nz][ny][nx] or NULL to use the scalar Ms; d_H: output [3][nz][ny][nx]
 * (overwritten, or incremented with DEMAG_ACCUMULATE).  d_energy: NULL or a
 * device double that receives E = -(mu0/2) V sum M . H_d, evaluated in the
 * transform domain (Parseval) without extra memory traffic.  d_m and d_H must
 * not overlap. */
int demag_field(const demag_plan* plan, const float* d_m, const float* d_Ms, float Ms, float* d_H,
                unsigned flags, double* d_energy, void* stream);

/* Size of the library's static work space per GPU (64 MiB), the limit of
 * demag_field_noalloc. */
#define DEMAG_NOALLOC_WORK_BYTES (64u << 20)

/* demag_field for callers that cannot allocate device memory while they run
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same passes, with the spectrum and energy partials in a
 * static device array of DEMAG_NOALLOC_WORK_BYTES that each GPU holds for the
 * lifetime of the process, instead of the plan's work buffer.  Arguments,
 * layouts and results are those of demag_field (bitwise the same output).
 * Single-mesh demagnetizing plans only (DEMAG_EINVAL otherwise), bound on the
 * current device (DEMAG_EINVAL for another device; DEMAG_ESTATE before
 * demag_bind), whose work_bytes (demag_buffer_bytes) are at most
 * DEMAG_NOALLOC_WORK_BYTES (DEMAG_EUNSUPPORTED otherwise, checked before the
 * bind state).  Calls no allocator.  All calls on one GPU share that GPU's
 * array, which keeps the last call's contents: calls that overlap in time on
 * one GPU (other streams, other threads, other plans) race and give wrong
 * results; order them on one stream. */
int demag_field_noalloc(const demag_plan* plan, const float* d_m, const float* d_Ms, float Ms, float* d_H,
                        unsigned flags, double* d_energy, void* stream);

/* E = -(mu0/2) V sum_cells Ms m . H for a given field H (any H, e.g. an
 * accumulated effective field), written to the device double d_energy.
 * Appendix A: the field/energy relation H = -1/(mu0 Ms) d(eps)/dm gives, for
 * the quadratic demagnetizing self-energy, the density eps = -(mu0/2) M . H.
 * d_m, d_H: [3][nz][ny][nx] FP32; d_Ms: per-cell [nz][ny][nx] or NULL for the
 * scalar Ms.  Products in FP32, sum in FP64 (fixed order).  Single-mesh plans
 * only (DEMAG_EINVAL otherwise); DEMAG_ESTATE before demag_bind. */
int demag_energy(const demag_plan* plan, const float* d_m, const float* d_Ms, float Ms, const float* d_H,
                 double* d_energy, void* stream);

/* Gradient of L(m) = <G, H_d(m)> + gE * E_demag(m) with respect to m, where
 * H_d(m) = -N * (Ms m).  N is symmetric and even in r, so the operator is
 * self-adjoint and d<G,H>/dM = -N * G; with dE/dM = -mu0 V H_d:
 *   grad_m = Ms * ( -N * G  - mu0 V gE H_d ).
 * d_G: upstream gradient [3][nz][ny][nx]; d_H: the forward field H_d (read
 * only when d_gE is not NULL); d_gE: NULL or a device double holding gE;
 * d_grad_m: output (overwritten, or incremented with DEMAG_ACCUMULATE).
 * d_G may alias neither d_H nor d_grad_m. */
int demag_backward(const demag_plan* plan, const float* d_G, const float* d_Ms, float Ms, const float* d_H,
                   const double* d_gE, float* d_grad_m, unsigned flags, void* stream);

/* A collection of meshes with independent discretizations (Sec. 3, Eq. 4).
 * Mesh i has dims[3i..3i+2] cells of cells[3i..3i+2] metres, its lower corner
 * at origins[3i..3i+2] (metres; NULL: all at the origin, only allowed without
 * groups).  groups: NULL, or one id per mesh; meshes sharing an id >= 0 are
 * coupled: each one's field includes the fields of the others through the
 * inter-mesh tensors N(r, h_k, h_i), summed in the transform space.  A
 * coupled group needs in-plane cell sizes that are power-of-two multiples of
 * the finest one, origins on the finest in-plane lattice, at most 8 z planes
 * in all and a fine lattice of at most 2048 x 1024 cells (else
 * DEMAG_EUNSUPPORTED).  Other meshes (id < 0) are independent; those of
 * identical geometry share one kernel spectrum and one launch per pass.
 * Vectors of all meshes are concatenated in mesh order, each mesh SoA
 * [3][nz][ny][nx], at the float offsets given by demag_batch_layout.
 * pbc_flags / pbc_images apply to every independent mesh as in demag_setup
 * and to every coupled group along x and y (Sec. 3, multiple images: the
 * group repeats as a whole, with the pair tensors summed over the images;
 * every mesh of the group must span the whole group along a periodic axis,
 * else DEMAG_EUNSUPPORTED).  A coupled group with periodic z returns
 * DEMAG_EUNSUPPORTED.  Host only, like demag_setup. */
int demag_setup_batch(demag_plan** out, int nmesh, const int* dims, const double* cells, const double* origins,
                      const int* groups, unsigned pbc_flags, int pbc_images);

/* Number of meshes, float offset of each mesh's block (offsets may be NULL;
 * otherwise room for nmesh entries) and total floats of one batch vector. */
int demag_batch_layout(const demag_plan* plan, int* nmesh, long long* offsets, size_t* total_floats);

/* H_d of every mesh of a batch plan in one launch sequence (one launch per
 * pass and geometry).  d_Ms_mesh: device float[nmesh] saturation
 * magnetizations, or NULL for the scalar Ms; d_energy: NULL or device
 * double[nmesh].  Otherwise as demag_field. */
int demag_field_batch(const demag_plan* plan, const float* d_m, const float* d_Ms_mesh, float Ms, float* d_H,
                      unsigned flags, double* d_energy, void* stream);

/* demag_backward for every mesh of a batch plan; d_gE: NULL or device
 * double[nmesh].  For coupled meshes the adjoint follows from reciprocity,
 * V_k N_ki(r) = V_i N_ik(-r): d<G,H>/dM_i = V_i H_i[G_k / V_k]. */
int demag_backward_batch(const demag_plan* plan, const float* d_G, const float* d_Ms_mesh, float Ms,
                         const float* d_H, const double* d_gE, float* d_grad_m, unsigned flags, void* stream);

/* Per-pass timing: `events` points to 4 hipEvent_t created by the caller; each
 * later demag_field / demag_backward call on this plan records them on its
 * stream before the forward pass, after the forward pass, after the middle
 * pass and after the inverse pass (the optional energy reduction follows).
 * NULL (or count 0) turns recording off.  Host-only bookkeeping. */
int demag_set_timing_events(demag_plan* plan, void* const* events, int count);

/* Demagnetizing field of two sublattices (Sec. 6): the field of the mean
 * magnetization (MsA mA + MsB mB) / 2, with d_mA, d_mB unit-vector fields of
 * the plan's mesh and scalar saturation magnetizations.  d_energy, when
 * given, receives -(mu0/2) V sum M . H_d of that mean M.  Single-mesh plans;
 * otherwise as demag_field. */
int demag_field_2sub(const demag_plan* plan, const float* d_mA, const float* d_mB, float MsA, float MsB,
                     float* d_H, unsigned flags, double* d_energy, void* stream);

/* A minimal evaluation loop around the demagnetizing field: one classical
 * RK4 step of the LLG equation (Sec. 2, Eq. 1, in its explicit form
 * dm/dt = -gamma/(1 + alpha^2) [m x H + alpha m x (m x H)]), with
 * H = demagnetizing + applied + direct exchange (Appendix A, Table 1:
 * (2A / (mu0 Ms)) lap(m), discrete Neumann condition, periodic along the
 * plan's periodic axes).  Four field evaluations per step (Sec. 7's
 * benchmark counts time per evaluation); m is renormalized after the step.
 *   Ms     saturation magnetization (A/m), > 0
 *   A      exchange stiffness (J/m), >= 0
 *   alpha  Gilbert damping, >= 0
 *   gamma  mu0 g_rel |gamma_e| in m/(A s); <= 0 selects mu0 * 1.76085963023e11
 *   dt     time step (s), > 0
 *   Hext   applied field (A/m) */
typedef struct {
  float Ms, A, alpha, gamma, dt;
  float Hext[3];
} demag_llg_params;

/* Device workspace of demag_llg_rk4 (4 vectors of the mesh, 256-byte aligned
 * slices).  Single-mesh plans. */
int demag_llg_workspace_bytes(const demag_plan* plan, size_t* bytes);

/* One RK4 step in place on d_m (unit vectors, SoA) on `stream`; d_work as
 * sized by demag_llg_workspace_bytes (caller-owned, 256-byte aligned).  Only
 * enqueues work (graph-capturable).  DEMAG_EINVAL for NULL or non-finite
 * parameters, Ms <= 0, dt <= 0, A < 0 or alpha < 0; single-mesh plans. */
int demag_llg_rk4(const demag_plan* plan, float* d_m, const demag_llg_params* params, void* d_work, void* stream);

/* Oersted field of a current density (Table 1, Oersted row; Sec. 4: the
 * field is a convolution sum of the current density with an Oersted kernel):
 *   H_t = scale / (4 pi) sum_s J_s x g(r_t - r_s),
 * g(d) the field integral of a cuboid cell carrying a uniform unit current
 * density, averaged over the target cell at offset d,
 *   g(d) = 1/V int_target int_source (r - r') / |r - r'|^3 dV' dV,
 * built in FP64 at set-up (reduced to one-dimensional integrals of Newell's f
 * near the source, Gauss-Legendre quadrature of the defining integral
 * beyond).  The field passes are those of demag_field with this kernel's
 * product, H^ = i (P x J^) per frequency.  J is SoA [3][nz][ny][nx] FP32 in
 * A/m^2 (scale = 1) and H is in A/m.
 *
 * demag_setup_oersted: as demag_setup, same size limits and periodic axes
 * (the kernel summed over pbc_images images on either side, the field of the
 * repeated mesh in its central copy); bind with demag_buffer_bytes /
 * demag_bind as any plan.  An Oersted plan is
 * refused (DEMAG_EINVAL) by demag_field, _2sub, _energy, _backward and the
 * LLG calls; schedules and the tuner apply as for a demagnetizing plan.
 *
 * demag_oersted_field: H = scale K*J, or H += scale K*J with
 * DEMAG_ACCUMULATE; only enqueues work (graph-capturable).  J -> H is
 * self-adjoint (K_ab(d) = K_ba(-d)), so this call is also its own backward:
 * d<G, H[J]>/dJ = scale K*G.  DEMAG_EINVAL for NULL buffers, unknown flags,
 * a non-finite scale or a plan that is not an Oersted plan; DEMAG_ESTATE
 * before demag_bind. */
int demag_setup_oersted(demag_plan** out, int nx, int ny, int nz, double dx, double dy, double dz,
                        unsigned pbc_flags, int pbc_images);
int demag_oersted_field(const demag_plan* plan, const float* d_J, float scale, float* d_H, unsigned flags,
                        void* stream);

/* Launch schedules.  Each plan has parts: one per group of identical
 * independent meshes (a single-mesh plan has one), then one per coupled
 * group.  A part's schedule is its launch shape:
 *   yg    y rows per workgroup of the x passes (meshes only; 0 for groups),
 *   kw    kx lines per workgroup of the middle (y) pass: 2, 4 or 8,
 *   radix points per lane of its y line FFTs (Ny/2 points per line): the
 *         default for the length, or 4 / 8 / 16 for Ny/2 of 256 and 512 when
 *         that leaves at most 64 lanes per line, or 8 for Ny/2 = 1024 (128
 *         lanes, a line spanning two wavefronts; selectable, not tuned).
 * All schedules compute the same convolution (Sec. 3, Eq. 4); they differ
 * only in speed and FP32 rounding order.  Host only. */
int demag_schedule_count(const demag_plan* plan, int* nparts);
int demag_get_schedule(const demag_plan* plan, int part, int* yg, int* kw, int* radix);

/* Sets part's schedule; 0 keeps a field.  DEMAG_EINVAL for a yg outside
 * 1..ny or beyond 160 KiB of LDS, a kw other than 2/4/8, a non-zero yg on a
 * coupled group; DEMAG_EUNSUPPORTED for a radix not offered for the length.
 * Affects later calls only (graphs captured earlier keep their launches);
 * not safe against concurrent calls on the same plan. */
int demag_set_schedule(demag_plan* plan, int part, int yg, int kw, int radix);

/* How a part transforms along z (Sec. 7: the z transform fused with the
 * passes around it, the paper's pipelined form, pays for short z lines; long
 * lines take separate passes).  separate = 0: the z transform runs inside the
 * x passes (needs the nz rows of a y line in LDS: nz <= 64, nz <= 32 for
 * nx > 256, nz <= 16 for nx > 512); separate = 1: the x passes run on the
 * mesh flattened to (nx, ny nz, 1) and two z passes transform the spectrum in
 * place (2 <= nz <= 256).  demag_setup picks the fused form where it exists;
 * demag_autotune times both where both exist.  yg of demag_get_schedule /
 * demag_set_schedule refers to the x passes of the current form.
 * DEMAG_EUNSUPPORTED for a form the part cannot take (coupled groups have no
 * z transform); DEMAG_EINVAL for bad arguments.  Host only. */
int demag_get_z_passes(const demag_plan* plan, int part, int* separate);
int demag_set_z_passes(demag_plan* plan, int part, int separate);

enum { DEMAG_TUNE_FORCE = 1,      /* measure even where the cache has an entry */
       DEMAG_TUNE_KEEP_FORM = 2 }; /* keep each part's current z form (fused or separate) */

/* Launch-shape tuner.  For each part: if cache_path names a schedule cache
 * (JSON, "demag-schedule-cache/1") holding an entry for this device and
 * geometry, apply it; else time every candidate schedule on `stream` with
 * HIP events (the fused and the separate z form where both exist, unless
 * DEMAG_TUNE_KEEP_FORM; then the x passes over the yg candidates; then the
 * whole field sequence over the middle pass's kw x radix), keep the fastest
 * and, when cache_path
 * is given, write it back
 * (temporary file + rename).  Measuring needs a bound plan (DEMAG_ESTATE) and,
 * for mesh parts, d_m and d_H laid out like the plan's vectors: d_m is only
 * read (its values do not matter), d_H and the plan's work buffer are
 * overwritten.  It synchronizes the stream: set-up time, not for graph
 * capture.  *measured (may be NULL) receives the number of parts timed.
 * DEMAG_EINVAL for an unreadable or malformed cache or an entry holding an
 * unsupported schedule; DEMAG_EHIP without a device. */
int demag_autotune(demag_plan* plan, const float* d_m, float* d_H, const char* cache_path, unsigned flags,
                   int* measured, void* stream);

/* Plain streaming copy of `bytes` from d_src to d_dst on `stream` (device
 * pointers, non-overlapping; both and `bytes` multiples of 16, else
 * DEMAG_EINVAL): the HBM read + write rate of a trivially bandwidth-bound
 * kernel, the measured ceiling the benchmark reports the field passes
 * against.  Measurement only; not an operation of the method. */
int demag_stream_copy(const void* d_src, void* d_dst, size_t bytes, void* stream);

/* Free a plan (host memory only).  NULL is accepted. */
int demag_destroy(demag_plan* plan);

/* Message for the calling thread's last non-OK return ("" if none). */
const char* demag_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DEMAG_H */
