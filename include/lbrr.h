/*
 * lbrr.h -- C ABI of the recursive-regularised lattice Boltzmann library
 * (MI355X / gfx950).
 *
 * The library advances athermal flows on a periodic lattice with the
 * regularised update of O. Malaspinas, "Increasing stability and accuracy of
 * the lattice Boltzmann scheme: recursivity and regularization"
 * (arXiv:1505.06900):
 *
 *   f_i(x + xi_i, t + 1) = f0_i + (1 - 1/tau) f1_i          (Sec. 3.5, Eq. discr_bgk_reg)
 *
 * f0 and f1 are Hermite expansions (Sec. 3.2, Eqs. fzero_d2q9 / fone_d2q9,
 * fzero_d3q27 / fone_d3q27) truncated at order N; their coefficients are
 * a0^(n) = rho u...u (Sec. 2) and a1^(n) from a1^(2) = P^(1) by the recursion
 * of Sec. 3.1 (Eq. rel_a1, App. B).  tau is the shifted relaxation time of
 * Sec. 3.4 (Eq. full_discr_bgk), so the kinematic viscosity is
 * nu = (tau - 1/2) / 3 in lattice units.
 *
 * Conventions shared by every entry point
 *  - Every function is extern "C"; none throws.  Functions returning int
 *    return LB_OK (0) or a negative LB_ERR_* code; lb_last_error() gives a
 *    message for the calling thread.
 *  - Field arrays are structure-of-arrays, x fastest: rho[z][y][x],
 *    u[d][z][y][x] (d = x, y[, z]), pi1[c][z][y][x] with the symmetric
 *    components c = (xx, xy, yy) in 2D and (xx, xy, xz, yy, yz, zz) in 3D.
 *    2D lattices require nz == 1.
 *  - dtype selects the element type of caller field arrays: LB_F64 (double)
 *    or LB_F32 (float).  on_device = 1 means the pointer is device memory of
 *    the current HIP device, 0 means host memory.  Caller arrays are only
 *    accessed during the call (stream-ordered on the handle's stream) and
 *    stay owned by the caller.
 *  - Population velocity order: i = (cx+1) + 3(cy+1) + 9(cz+1) for D2Q9
 *    (cz = 0) and D3Q27; D3Q19 keeps the D3Q27 order without the 8 corners.
 *  - The library owns two state buffers per handle (allocated with
 *    hipMalloc in lb_init_fields / lb_set_populations, freed by lb_destroy).
 *    With population storage they hold post-collision populations as
 *    deviations f_i - w_i rho0 in the storage type; rho and u of the stored
 *    state equal those of the pre-collision state at the same time because
 *    the collision conserves them (Sec. 2, mass and momentum conservation).
 *    With moment storage they hold the pre-collision moments (lb_config).
 *  - All device work is enqueued on the handle's stream (default: the null
 *    stream).  Entry points that return host data synchronise that stream.
 *  - Tuning overrides (environment variables; the defaults are the choices
 *    measured fastest on MI355X).  They change where data lives or how work
 *    is launched, not what is computed; a value out of range is ignored.
 *      LBRR_LAYOUT=0|1|2        state layout, read when a handle's buffers
 *                               are allocated: 0 [q][z][y][x], 1 [z][y][q][x],
 *                               2 [z][q][y][x] (q: population or field)
 *      LBRR_PLANE_PAD_BYTES=n   bytes after each population plane in layouts
 *                               0 and 2, rounded up to 256 (read at allocation)
 *      LBRR_MOM_LZ=n            z-planes (3D) or rows (2D) per block of the
 *                               moment-storage step, n >= 1 (read every step)
 *      LBRR_CLOSURE_WPR=1|2     waves per row of the fused closure step with
 *                               FP32 or FP16 storage (read every step)
 *      LBRR_STEP_BLOCKS_PER_CU=n  blocks of the population step per compute
 *                               unit, 1..8, 0 for no limit (read every step)
 */
#ifndef LBRR_H
#define LBRR_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lb_ctx* lb_handle;

enum lb_lattice { LB_D2Q9 = 0, LB_D3Q19 = 1, LB_D3Q27 = 2 };
enum lb_storage {
  LB_STORE_FP64 = 0, /* populations f_i - w_i rho0, FP64 */
  LB_STORE_FP32 = 1, /* populations f_i - w_i rho0, FP32 */
  LB_STORE_FP16 = 2, /* populations f_i - w_i rho0, binary16 */
  LB_STORE_MOM_FP64 = 3, /* moments rho - rho0, rho u, a1^(2) of each node, FP64 */
  LB_STORE_MOM_FP32 = 4  /* moments rho - rho0, rho u, a1^(2) of each node, FP32 */
};
enum lb_dtype { LB_F64 = 0, LB_F32 = 1 };
enum lb_status {
  LB_OK = 0,
  LB_ERR_INVALID_ARG = -1, /* argument out of range, NULL pointer, wrong dims */
  LB_ERR_UNSUPPORTED = -2, /* valid combination the library does not provide */
  LB_ERR_OOM = -3,         /* device allocation failed */
  LB_ERR_HIP = -4,         /* a HIP runtime call failed (message has the HIP error) */
  LB_ERR_UNSTABLE = -5,    /* non-finite density or velocity found by a check */
  LB_ERR_STATE = -6        /* call out of order (e.g. lb_step before lb_init_fields) */
};

/* Create a simulation handle.
 * lattice: LB_D2Q9, LB_D3Q19 or LB_D3Q27 (velocity sets of Sec. 3.2).
 * nx, ny, nz: periodic box, each >= 1, nz == 1 for D2Q9, nx*ny*nz < 2^31.
 * tau: shifted relaxation time of Sec. 3.4, finite and > 0.5.
 * order: Hermite truncation N of f0 and f1 (Sec. 3.2, Sec. 3.8.1 for N = 2):
 *        2..4 for D2Q9 and D3Q19, 2..6 for D3Q27.
 * Default storage: LB_STORE_FP32 with rho0 = 1.  No device memory is
 * allocated and no device work is launched.  Returns NULL on error. */
lb_handle lb_create(int lattice, int nx, int ny, int nz, double tau, int order);

/* Choose the state storage (LB_STORE_*) and the reference density rho0 of
 * the deviation form f_i - w_i rho0 (rho0 > 0, finite).  FP32 and FP16
 * storage collide in FP32, FP64 storage in FP64; FP16 values are rounded to
 * nearest-even on store, subnormals kept.
 * Moment storage (LB_STORE_MOM_*): after the collision of Eq. discr_bgk_reg
 * the populations of a node are a function of its rho, u and a1^(2) only
 * (a0 and the recursion of Sec. 3.1, reconstruction of Sec. 3.2), so the
 * library stores each node's pre-collision (rho - rho0, rho u, a1^(2)) --
 * 6 values in 2D, 10 in 3D -- and lb_step rebuilds each population of the
 * source node before streaming it: the same update with 20 instead of 54
 * stored values moved per D3Q27 node update.  Collision in FP64 or FP32 as
 * the storage.  lb_set_populations and the learned closure are not available
 * with moment storage (LB_ERR_UNSUPPORTED).
 * Must precede lb_init_fields / lb_set_populations; calling it again discards
 * the state. */
int lb_config(lb_handle h, int storage, double rho0);

/* Use hip_stream (a hipStream_t, may be NULL for the null stream) for all
 * later device work of this handle.  Work already enqueued on the previous
 * stream is ordered before it (the new stream waits for an event recorded on
 * the old one; the host does not block). */
int lb_set_stream(lb_handle h, void* hip_stream);

/* Set the state at t = 0 from macroscopic fields.  The pre-collision
 * populations are f0^(N)(rho, u) (Sec. 3.2) plus, if pi1 != NULL, the
 * off-equilibrium part f1^(N) whose second-order coefficient is
 * a1^(2) = pi1 (P^(1) of Sec. 2) and whose higher orders follow from the
 * recursion of Sec. 3.1; the stored state is their collision.
 * rho: [nz][ny][nx], u: [D][nz][ny][nx], pi1: [D(D+1)/2][nz][ny][nx] or NULL.
 * Resets the step counter to 0. */
int lb_init_fields(lb_handle h, const void* rho, const void* u, const void* pi1,
                   int dtype, int on_device);

/* Advance n >= 0 steps of Eq. discr_bgk_reg (pull streaming fused with the
 * regularised collision).  Stream-ordered, asynchronous unless a stability
 * check interval is set (lb_set_check_interval), in which case the density
 * and velocity are checked every k steps and LB_ERR_UNSTABLE is returned
 * after the first check that finds a non-finite value (the state then holds
 * the failing step).  Without a check interval the call only launches
 * kernels (no allocation, memset or synchronisation), so it can be captured
 * in a HIP graph on the handle's stream.  Each step swaps the handle's two
 * state buffers: replays of a captured run keep the handle's bookkeeping
 * right only if n is even. */
int lb_step(lb_handle h, long long n);

/* Resting no-slip walls (u = 0) on the first and last node of each axis in
 * the mask `walls` (bit 0 x, bit 1 y, bit 2 z; 0 = fully periodic, the
 * default); the other axes stay periodic.  The regularised Dirichlet
 * boundary of Sec. 3.7: at a wall node the populations whose source lies
 * outside the box are unknown; an unknown one takes the off-equilibrium part
 * of its opposite if that one is known (here f_i = f_opp), else its
 * equilibrium value (edges and corners); rho is the zeroth moment of the
 * completed set, a1^(2) its second moment minus rho c_s^2 I, and the node
 * collides with (rho, u = 0, a1^(2)).  Velocities given to lb_init_fields on
 * wall nodes should be 0.  A walled axis needs at least 3 nodes.  Population
 * and moment storage (a wall node of the moment state keeps rho - rho0,
 * j = 0 and that a1^(2)); not with the learned closure (lb_step returns
 * LB_ERR_UNSUPPORTED).  lb_enstrophy uses one-sided differences on the walls.
 * Takes effect at the next lb_step. */
int lb_set_walls(lb_handle h, int walls);

/* Stability check interval k for lb_step (0 = never, the default). */
int lb_set_check_interval(lb_handle h, long long k);

/* Macroscopic fields of the current state: rho [nz][ny][nx], u [D][nz][ny][nx]
 * and, if pi1 != NULL, the off-equilibrium stress a1^(2) of the pre-collision
 * populations (Sec. 2, P^(1) = a1^(2)), recovered from a stored
 * post-collision population state as its a1^(2) divided by (1 - 1/tau)
 * (LB_ERR_UNSUPPORTED when tau == 1; moment storage holds it directly).  Any of the outputs may be NULL.  Synchronises the stream. */
int lb_moments(lb_handle h, void* rho, void* u, void* pi1, int dtype, int on_device);

/* Global FP64 totals of the current state: out[0] = sum rho, out[1..3] =
 * sum rho u (z component 0 in 2D), out[4] = sum rho |u|^2 / 2 (the kinetic
 * energy followed in Sec. 4.1).  Per-wave shuffles, per-block partials, then
 * a fixed-order final sum: bitwise reproducible.  Returns LB_ERR_UNSTABLE if
 * any total is not finite.  Synchronises the stream. */
int lb_reduce(lb_handle h, double out[5]);

/* FP64 totals of a population state held by the caller, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Computes what lb_reduce computes
 * (out[0] = sum rho, out[1..3] = sum rho u, out[4] = sum rho |u|^2 / 2), with
 * the same kernels and the same partition into blocks, so the same bits,
 * but allocates nothing and does not synchronise: the per-block partials
 * live in a static device array of LB_REDUCE_STATIC_MAX_BLOCKS x 5 doubles
 * (82 KB per GPU, held until the process ends), and the five totals are
 * written to device memory on the given stream (the caller checks them for
 * non-finite values).
 * lattice: LB_D2Q9 / LB_D3Q19 / LB_D3Q27; storage: LB_STORE_FP64, _FP32 or
 * _FP16 (moment storages: LB_ERR_UNSUPPORTED); populations: device pointer,
 * compact SoA [q][nz][ny][nx] of the deviations f_i - w_i rho0 in the storage
 * type (what lb_get_populations writes); out: device pointer to 5 doubles;
 * hip_stream: a hipStream_t or NULL.  nx*ny*nz < 2^31 (nz = 1 for D2Q9),
 * which keeps the partials within the static array; anything else returns
 * LB_ERR_INVALID_ARG.  All calls on one GPU share its static array: calls
 * that overlap in time on one GPU (two streams, two threads) race; calls in
 * one stream are ordered.  No part of the array needs clearing: every call
 * writes every partial it reads. */
#define LB_REDUCE_STATIC_MAX_BLOCKS 2048
int lb_reduce_static(int lattice, int storage, int nx, int ny, int nz, double rho0, const void* populations,
                     double* out, void* hip_stream);

/* Volume mean of |omega|^2 / 2, omega = curl u by second-order periodic
 * central differences (second-order one-sided on walls, lb_set_walls),
 * accumulated in FP64: the enstrophy of Sec. 4.1 (half the integral of
 * omega^2) divided by the volume.  On a walled axis the integral is the
 * trapezoid rule over the box whose faces are the wall nodes (those nodes
 * weigh 1/2, and n nodes span n - 1 cells); a periodic axis of n nodes
 * spans n cells of weight 1.  Synchronises the stream. */
int lb_enstrophy(lb_handle h, double* out);

/* Copy the stored post-collision deviations f_i - w_i rho0 out of / into the
 * library, in the storage type, compact SoA [q][nz][ny][nx].  dst/src hold
 * q*nx*ny*nz elements.  lb_set_populations makes the handle ready to step
 * (step counter unchanged).  With moment storage lb_get_populations returns
 * the post-collision deviations rebuilt from the stored moments (FP64 or FP32
 * as the storage) and lb_set_populations returns LB_ERR_UNSUPPORTED. */
int lb_get_populations(lb_handle h, void* dst, int on_device);
int lb_set_populations(lb_handle h, const void* src, int on_device);

/* Number of completed steps since lb_init_fields. */
long long lb_step_count(lb_handle h);

/* Bytes of state storage moved per lattice-node update by lb_step: each
 * stored value read once and written once, 2 * q * sizeof(element) for
 * population storage, 2 * (1 + D + D(D+1)/2) * sizeof(element) for moment
 * storage.  Returns 0 for a NULL handle. */
double lb_bytes_per_update(lb_handle h);

/* Release the handle and its device buffers (NULL-safe). */
void lb_destroy(lb_handle h);

/* Thread-local description of the last error ("" if none). */
const char* lb_last_error(void);

/* ------------------------------------------------------------------------
 * Learned closure of a1^(2) on coarse D2Q9 runs.  Not part of the paper: a
 * per-node MLP (36 -> 64 -> 64 -> 3, exact-erf GELU, BF16 matrix-core
 * operands with FP32 accumulation) predicts a correction that is added to
 * the pre-collision a1^(2) (P^(1) of Sec. 2) before the recursion of
 * Sec. 3.1 (Eq. rel_a1) builds the higher orders and Eq. discr_bgk_reg
 * reconstructs the populations.
 *
 * Parameter vector: LB_MLP_NPARAM FP32 values, in order W1 (64 x 36, row =
 * output), b1 (64), W2 (64 x 64), b2 (64), W3 (3 x 64), b3 (3).
 * Normalisation vector: LB_MLP_NNORM FP32 values: feature mean (36), feature
 * std (36, > 0), output mean (3), output std (3, > 0); the network maps
 * (x - mean)/std to (y - mean)/std.
 * Features of a node for the step from a stored state g (36 FP32): the 9
 * pulled pre-collision deviations f_i - w_i rho0, f_i(x) = g_i(x - xi_i), then
 * for the neighbours x + (dx, dy), dy = -1, 0, 1 (outer), dx = -1, 0, 1
 * (inner): rho - rho0, u_x, u_y of g.  Outputs: corrections of a1^(2)
 * (xx, xy, yy).
 * All pointers of these entry points are device pointers.  The MLP entry
 * points share one library-owned workspace per process: calls that overlap
 * on one device race.
 */
#define LB_MLP_NPARAM 6723
#define LB_MLP_NNORM 78
#define LB_MLP_NIN 36

/* Enable (enable = 1) or disable the closure for lb_step of a D2Q9 handle
 * (LB_ERR_UNSUPPORTED otherwise).  params / norm are copied (stream-ordered);
 * with the closure on, each step first writes (rho - rho0, u) of the stored
 * state to a handle-owned buffer, then runs the fused step with the MLP. */
int lb_set_closure(lb_handle h, const float* params, const float* norm, int enable);

/* Features (nodes x 36, row-major) of the step that would follow the current
 * state, and labels (nodes x 3) = a_target - plain_weight * (a1^(2) of the
 * pulled populations); a_target is packed [3][ny][nx] FP64 or NULL (read as
 * 0).  D2Q9 only; the state is not advanced; asynchronous on the stream. */
int lb_closure_features(lb_handle h, const double* a_target, double plain_weight, float* features, float* labels);

/* Coarse-grain fine D2Q9 fields by factor x factor box averages (acoustic
 * scaling, velocities and stresses keep their lattice-unit values):
 *   rho_c = box(rho), u_c = box(rho u) / rho_c,
 *   pi1_c = alpha box(pi1) + beta (box(rho u u) - rho_c u_c u_c),
 * the second term being the sub-filter stress.  Inputs: rho [nfy][nfx],
 * u [2][nfy][nfx], pi1 [3][nfy][nfx] (packed xx, xy, yy) of element type
 * dtype; outputs FP64, [nfy/f][nfx/f] per component.  nfx, nfy multiples of
 * factor. */
int lb_closure_coarsen(const void* rho, const void* u, const void* pi1, int dtype, int nfx, int nfy, int factor,
                       double alpha, double beta, double* rho_c, double* u_c, double* pi1_c, void* hip_stream);

/* MLP outputs y (n x 3, de-normalised) for raw features x (n x 36). */
int lb_mlp_forward(const float* params, const float* norm, const float* x, long long n, float* y, void* hip_stream);

/* Gradient (LB_MLP_NPARAM) of the mean squared error of normalised outputs
 * over the batch rows idx[0..batch) of x (raw features, n x 36) and t (raw
 * targets, n x 3), and the loss itself (loss may be NULL).  Row indices
 * outside [0, n) are clamped.  Per-block partial sums reduced in a fixed
 * order: bitwise reproducible. */
int lb_mlp_gradient(const float* params, const float* norm, const float* x, const float* t, long long n,
                    const int* idx, int batch, float* grad, float* loss, void* hip_stream);

/* Column mean and standard deviation (population form, FP64 accumulation in a
 * fixed order) of x (n x dim, row-major), e.g. for the normalisation vector;
 * a zero deviation is reported as 1. */
int lb_column_stats(const float* x, long long n, int dim, float* mean, float* std, void* hip_stream);

/* One bias-corrected Adam update of params (FP32 master copy) with moments m,
 * v; step counts from 1. */
int lb_mlp_adam(float* params, float* m, float* v, const float* grad, long long step, float lr, float beta1,
                float beta2, float eps, void* hip_stream);

/* Plain device copy of n bytes (n a multiple of 16, 16-byte aligned
 * pointers) on hip_stream: the bandwidth probe and hardware-counter
 * calibration kernel. */
int lb_probe_copy(const void* src, void* dst, size_t n, void* hip_stream);

/* Bandwidth probes of n bytes on hip_stream (no lattice arithmetic): kind 0
 * copy src -> dst, 1 read src (dst is written only for values a zero-filled
 * src cannot give), 2 write dst, 3 copy of `streams` (1..32) equal planes,
 * each thread copying its element of every plane.  vec_bytes 4, 8 or 16 per
 * lane; blocks_per_cu 0 = one thread per element, 1..64 = that many
 * 256-thread blocks per compute unit striding over the buffer (kinds 0-2);
 * nontemporal != 0 uses non-temporal loads and stores.  16-byte aligned
 * pointers, n a multiple of 16 (kind 3: of vec_bytes * streams).  They give
 * the HBM rate simple patterns reach on this GPU, beside the vendor peak. */
int lb_probe_bandwidth(int kind, int vec_bytes, int blocks_per_cu, int nontemporal, int streams, const void* src,
                       void* dst, size_t n, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LBRR_H */
