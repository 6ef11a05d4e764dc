// C ABI of the library (declarations and contracts in include/lbrr.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>

#include "closure.hpp"
#include "lbrr.h"
#include "ops.hpp"

using lbrr::LatticeOps;
using lbrr::StepArgs;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(LB_ERR_HIP, "%s: %s (%d)", what, hipGetErrorString(e), int(e));
}

#define HIP_TRY(expr, what)            \
  do {                                 \
    hipError_t e_ = (expr);            \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

size_t elem_size(int storage) {
  switch (storage) {
    case LB_STORE_FP64:
    case LB_STORE_MOM_FP64: return 8;
    case LB_STORE_FP32:
    case LB_STORE_MOM_FP32: return 4;
  }
  return 2;
}

// Chunk length of the moment-state step: rows per block in 2D, z-planes per
// block in 3D (each block rebuilds lz + 2/3 planes' worth: the two planes next
// to the chunk rebuild one layer).  Measured on MI355X:
//   2D, rows of 256 nodes: 4 rows best (see kRowX).
//   3D FP32 (row-aligned tiles of 64 x 9 nodes, x-neighbouring tiles on one
//   XCD), D3Q27 order 4, GLUPS at lz = 9 / 12 / 16 / 24 / 32 / 43 / 64:
//     256^3 49.1 / 51.5 / 51.0 / 53.4 / 53.4 / 53.9 / 54.4
//     512^3 50.9 / 52.6 / 53.9 / 55.0 / 55.9 / 56.1 / 55.7
//     D3Q19 order 4 512^3 (lz 9 / 12 / 16 / 24): 51.0 / 53.0 / 54.6 / 55.8
//   Longer chunks re-read fewer edge planes but give fewer blocks, so the host
//   takes the longest of 24, 16, 12, 9, 6, 4 planes that still gives four
//   blocks per compute unit (at 256^3: 24 planes, 1408 blocks).
//   3D FP64 (64 x 8 / 32 x 8 patches, k_mstep), lz = 3 / 4 / 6:
//     D3Q27 256^3 20.8 / 21.4 / 22.0, 512^3 19.8 / 20.3 / 21.7; D3Q19 on
//     planes of 448^2 nodes and more prefers 4.  So lz = 6 there, except 4 for
//     D3Q19 on large planes.
// LBRR_MOM_LZ overrides the choice.
int moment_lz(int nvalues, int q, int nx, int ny, int nz, size_t es) {
  if (const char* e = std::getenv("LBRR_MOM_LZ")) {
    const int v = std::atoi(e);
    if (v >= 1) return v;
  }
  if (nvalues == 6) return 4;
  if (es == 4) {  // row-aligned tiles of 64 x kTileRows nodes, tile rows in groups of eight
    int cus = 256;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    for (int lz : {24, 16, 12, 9, 6}) {
      const int64_t rows = int64_t((ny + lbrr::kTileRows - 1) / lbrr::kTileRows) * ((nz + lz - 1) / lz);
      if (int64_t((nx + 63) / 64) * 8 * ((rows + 7) / 8) >= int64_t(4) * cus) return lz;
    }
    return 4;
  }
  if (q == 19 && int64_t(nx) * ny >= 448 * 448) return 4;
  return 6;
}

// Extra bytes after each population plane (layouts 0 and 2).  Planes whose
// size is a large power of two would otherwise start at addresses that map to
// the same HBM channels; the default adds 4 KiB + 256 B when the plane is a
// multiple of 64 KiB.  LBRR_PLANE_PAD_BYTES overrides it (rounded up to 256 B).
size_t plane_pad_bytes(size_t plane_bytes) {
  if (const char* e = std::getenv("LBRR_PLANE_PAD_BYTES")) {
    const long long v = std::atoll(e);
    if (v >= 0) return size_t((v + 255) / 256 * 256);
  }
  return (plane_bytes % 65536 == 0) ? 4352 : 0;
}

// Scratch of lb_reduce_static: the per-block partial totals (5 doubles per
// block, at most LB_REDUCE_STATIC_MAX_BLOCKS blocks) and nothing else.  A
// file-scope device array: every GPU the library runs on holds its own copy
// (82 KB) until the process ends.  Host code never uses the name `scratch`
// as an address; it uses the per-device address that hipGetSymbolAddress
// returns (static_scratch below).
static __device__ __align__(256) double scratch[5 * LB_REDUCE_STATIC_MAX_BLOCKS];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

// Address of `scratch` on the current device, looked up once per device.
int static_scratch(double** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(LB_ERR_UNSUPPORTED, "device index %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    g_scratch[dev] = static_cast<double*>(p);
  }
  *out = g_scratch[dev];
  return LB_OK;
}

// Per-block partial count of the totals: one block per 2048 nodes, at most
// LB_REDUCE_STATIC_MAX_BLOCKS (the handle path and lb_reduce_static use the
// same partition, so their sums are the same bits).
int totals_blocks(int64_t nodes) {
  const int64_t nb = (nodes + 2047) / 2048;
  return int(nb < 1 ? 1 : (nb > LB_REDUCE_STATIC_MAX_BLOCKS ? LB_REDUCE_STATIC_MAX_BLOCKS : nb));
}

}  // namespace

struct lb_ctx {
  int lattice = 0;
  const LatticeOps* ops = nullptr;
  int nx = 0, ny = 0, nz = 0;
  double tau = 0.0;
  int order = 0;
  int storage = LB_STORE_FP32;
  double rho0 = 1.0;
  int device = 0;
  hipStream_t stream = nullptr;
  void* buf[2] = {nullptr, nullptr};
  int cur = 0;
  int layout = 0;                  // 0 [q][z][y][x], 1 [z][y][q][x], 2 [z][q][y][x]
  int64_t si = 0, sy = 0, sz = 0;  // element strides of population, row, plane
  size_t buf_elems = 0;
  bool ready = false;
  long long steps = 0;
  long long check_every = 0;
  int walls = 0;  // bit 0 x, bit 1 y, bit 2 z: resting no-slip walls on the first and last node
  double* partials = nullptr;
  int nblocks = 0;
  double* dev_out = nullptr;
  double* vel = nullptr;
  // learned closure (D2Q9)
  bool closure_on = false;
  float* cl_params = nullptr;   // kMlpNParam
  float* cl_norm = nullptr;     // kMlpNNorm
  uint16_t* cl_packed = nullptr;

  int64_t nodes() const { return int64_t(nx) * ny * nz; }
  int q() const { return ops->q; }
  int d() const { return ops->d; }
  bool moment() const { return lbrr::is_moment_storage(storage); }
  // stored values per node: q populations, or rho - rho0, j and a1^(2)
  int nvalues() const { return moment() ? 1 + d() + d() * (d() + 1) / 2 : q(); }
  StepArgs args() const {
    StepArgs a;
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.si = si;
    a.sy = sy;
    a.sz = sz;
    a.rho0 = rho0;
    a.omega1 = 1.0 - 1.0 / tau;
    a.lz = moment() ? moment_lz(nvalues(), q(), nx, ny, nz, elem_size(storage)) : 1;
    a.walls = moment() ? walls : 0;
    return a;
  }
  void release() {
    for (void*& b : buf) {
      if (b) (void)hipFree(b);
      b = nullptr;
    }
    if (partials) (void)hipFree(partials);
    if (dev_out) (void)hipFree(dev_out);
    if (vel) (void)hipFree(vel);
    partials = nullptr;
    dev_out = nullptr;
    vel = nullptr;
    ready = false;
  }
  void release_closure() {
    for (void* p : {static_cast<void*>(cl_params), static_cast<void*>(cl_norm), static_cast<void*>(cl_packed)})
      if (p) (void)hipFree(p);
    cl_params = nullptr;
    cl_norm = nullptr;
    cl_packed = nullptr;
    closure_on = false;
  }
};

namespace {

// Population layout.  Measured on MI355X for the step kernel (GLUPS, each
// layout three times in one run, interleaved; runs agree to 1%):
//   * planes of at most 256 KiB (256^2 FP32, 256^2 / 320^2 FP16): keeping the
//     q planes of a z-slab together ([z][q][y][x], layout 2) is best
//     (D3Q27 256^3 FP32 27.5 against 26.7 for layout 1);
//   * larger planes: the q rows of a (y, z) row together ([z][y][q][x],
//     layout 1) for FP32 at every size and for the rest up to 448^2 planes
//     (D3Q27 384^3 FP16 55.3 against 53.1 / 53.0);
//   * planes of 512^2 nodes and more: FP16 keeps layout 2 (D3Q27 512^3 50.3
//     against 46.4 for layout 1, D3Q19 78.5 against 70.4) and FP64 one volume
//     per population ([q][z][y][x], layout 0; D3Q27 12.7 against 11.1,
//     D3Q19 18.2 against 16.4).
// LBRR_LAYOUT=0|1|2 overrides the choice.
int layout_choice(int d, int64_t nx, int64_t ny, size_t es) {
  if (const char* e = std::getenv("LBRR_LAYOUT")) {
    const int v = std::atoi(e);
    if (v >= 0 && v <= 2) return v;
  }
  if (d != 3) return 1;
  const int64_t plane_nodes = nx * ny;
  if (size_t(plane_nodes) * es <= 262144) return 2;
  if (plane_nodes >= 512 * 512) {
    if (es == 2) return 2;
    if (es == 8) return 0;
  }
  return 1;
}

// Moment-state layout: the fields of a (y, z) row together ([z][y][c][x],
// layout 1), so the patch of a step block reads one contiguous run per row.
// LBRR_LAYOUT=0|1|2 overrides the choice.
int moment_layout_choice() {
  if (const char* e = std::getenv("LBRR_LAYOUT")) {
    const int v = std::atoi(e);
    if (v >= 0 && v <= 2) return v;
  }
  return 1;
}

int ensure_buffers(lb_ctx* h) {
  if (h->buf[0]) return LB_OK;
  const size_t es = elem_size(h->storage);
  const int64_t nx = h->nx, ny = h->ny, nz = h->nz, q = h->nvalues();
  h->layout = h->moment() ? moment_layout_choice() : layout_choice(h->d(), nx, ny, es);
  // Row pitch: nx rounded up to whole 128-byte lines, so that every row starts
  // on a line and a wave's 64 consecutive x stay within the fewest lines (with
  // nx = 300 unpadded, D3Q27 FP32 ran at 13.9 GLUPS against 27 for 256 or 320).
  const int64_t px = int64_t((size_t(nx) * es + 127) / 128 * 128 / es);
  size_t elems = 0;
  if (h->layout == 1) {  // rows of all populations together
    h->si = px;
    h->sy = q * px;
    h->sz = ny * q * px;
    elems = size_t(nz * ny * q * px);
  } else {
    const size_t plane = size_t(h->layout == 0 ? px * ny * nz : px * ny) * es;
    const size_t plane_al = (plane + 255) / 256 * 256;
    const size_t plane_bytes = plane_al + plane_pad_bytes(plane_al);
    const int64_t p = int64_t(plane_bytes / es);
    if (h->layout == 0) {
      h->si = p;
      h->sy = px;
      h->sz = px * ny;
      elems = size_t(q * p);
    } else {
      h->si = p;
      h->sy = px;
      h->sz = q * p;
      elems = size_t(nz * q * p);
    }
  }
  // every kernel index i*si + z*sz + y*sy + x must stay inside the allocation
  const int64_t max_index = (q - 1) * h->si + (nz - 1) * h->sz + (ny - 1) * h->sy + (nx - 1);
  if (max_index < 0 || size_t(max_index) >= elems)
    return fail(LB_ERR_INVALID_ARG, "internal layout error: max index %lld >= %zu", (long long)max_index, elems);
  h->buf_elems = elems;
  const size_t total = elems * es;
  for (int k = 0; k < 2; ++k) {
    hipError_t e = hipMalloc(&h->buf[k], total);
    if (e != hipSuccess) {
      h->release();
      (void)hipGetLastError();
      return fail(LB_ERR_OOM, "hipMalloc of %zu bytes for populations failed: %s", total, hipGetErrorString(e));
    }
  }
  h->nblocks = totals_blocks(h->nodes());
  // a failure here frees the population buffers too: buf[0] marks a complete set
  hipError_t e = hipMalloc(&h->partials, sizeof(double) * 5 * h->nblocks);
  if (e == hipSuccess) e = hipMalloc(&h->dev_out, sizeof(double) * 8);
  if (e != hipSuccess) {
    h->release();
    (void)hipGetLastError();
    return fail(LB_ERR_OOM, "hipMalloc of the reduction buffers failed: %s", hipGetErrorString(e));
  }
  return LB_OK;
}

int check_handle(lb_ctx* h) {
  if (!h) return fail(LB_ERR_INVALID_ARG, "NULL handle");
  HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
  return LB_OK;
}

int totals(lb_ctx* h, double out[5]) {
  hipError_t e = h->ops->totals(h->storage, h->buf[h->cur], h->partials, h->nblocks, h->dev_out, h->args(), h->stream);
  if (e != hipSuccess) return hip_fail(e, "totals kernel launch");
  HIP_TRY(hipMemcpyAsync(out, h->dev_out, sizeof(double) * 5, hipMemcpyDeviceToHost, h->stream), "copy totals");
  HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  for (int c = 0; c < 5; ++c)
    if (!std::isfinite(out[c])) return fail(LB_ERR_UNSTABLE, "non-finite total after step %lld", h->steps);
  return LB_OK;
}

}  // namespace

extern "C" {

const char* lb_last_error(void) { return g_err.c_str(); }

lb_handle lb_create(int lattice, int nx, int ny, int nz, double tau, int order) {
  const LatticeOps* ops = nullptr;
  switch (lattice) {
    case LB_D2Q9: ops = &lbrr::ops_d2q9(); break;
    case LB_D3Q19: ops = &lbrr::ops_d3q19(); break;
    case LB_D3Q27: ops = &lbrr::ops_d3q27(); break;
    default: fail(LB_ERR_INVALID_ARG, "unknown lattice %d", lattice); return nullptr;
  }
  if (nx < 1 || ny < 1 || nz < 1 || ny > 65535 || nz > 65535) {
    fail(LB_ERR_INVALID_ARG, "dims must be >= 1 (ny, nz <= 65535), got %d x %d x %d", nx, ny, nz);
    return nullptr;
  }
  if (int64_t(nx) * ny * nz >= (int64_t(1) << 31)) {
    fail(LB_ERR_INVALID_ARG, "nx*ny*nz must be < 2^31");
    return nullptr;
  }
  if (ops->d == 2 && nz != 1) {
    fail(LB_ERR_INVALID_ARG, "D2Q9 requires nz == 1, got %d", nz);
    return nullptr;
  }
  if (!std::isfinite(tau) || !(tau > 0.5)) {
    fail(LB_ERR_INVALID_ARG, "tau must be finite and > 0.5, got %g", tau);
    return nullptr;
  }
  if (order < 2 || order > ops->nmax) {
    fail(LB_ERR_INVALID_ARG, "order must be in [2, %d] for this lattice, got %d", ops->nmax, order);
    return nullptr;
  }
  lb_ctx* h = new (std::nothrow) lb_ctx();
  if (!h) {
    fail(LB_ERR_OOM, "host allocation failed");
    return nullptr;
  }
  h->lattice = lattice;
  h->ops = ops;
  h->nx = nx;
  h->ny = ny;
  h->nz = nz;
  h->tau = tau;
  h->order = order;
  const hipError_t e = hipGetDevice(&h->device);
  if (e != hipSuccess) {
    delete h;
    fail(LB_ERR_HIP, "hipGetDevice failed: %s (%d)", hipGetErrorString(e), int(e));
    return nullptr;
  }
  g_err.clear();
  return h;
}

int lb_config(lb_handle h, int storage, double rho0) {
  if (int r = check_handle(h)) return r;
  if (storage < LB_STORE_FP64 || storage > LB_STORE_MOM_FP32) return fail(LB_ERR_INVALID_ARG, "bad storage %d", storage);
  if (!std::isfinite(rho0) || !(rho0 > 0)) return fail(LB_ERR_INVALID_ARG, "rho0 must be finite and > 0");
  if (h->buf[0]) HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  h->release();
  h->storage = storage;
  h->rho0 = rho0;
  h->steps = 0;
  return LB_OK;
}

int lb_set_stream(lb_handle h, void* hip_stream) {
  if (int r = check_handle(h)) return r;
  hipStream_t next = static_cast<hipStream_t>(hip_stream);
  if (next != h->stream && h->buf[0]) {
    // work already enqueued on the old stream comes first: the new stream
    // waits for an event recorded behind it (nothing blocks the host)
    hipEvent_t ev;
    HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate");
    hipError_t e = hipEventRecord(ev, h->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(next, ev, 0);
    (void)hipEventDestroy(ev);
    if (e != hipSuccess) return hip_fail(e, "ordering the new stream after the old one");
  }
  h->stream = next;
  return LB_OK;
}

int lb_set_walls(lb_handle h, int walls) {
  if (int r = check_handle(h)) return r;
  if (walls < 0 || walls > 7) return fail(LB_ERR_INVALID_ARG, "walls must be a mask of bits 0 (x), 1 (y), 2 (z)");
  if ((walls & 4) && h->d() == 2) return fail(LB_ERR_INVALID_ARG, "a 2D lattice has no z walls");
  const int dims[3] = {h->nx, h->ny, h->nz};
  for (int k = 0; k < 3; ++k)
    if ((walls >> k & 1) && dims[k] < 3) return fail(LB_ERR_INVALID_ARG, "a walled axis needs at least 3 nodes");
  h->walls = walls;
  return LB_OK;
}

int lb_set_check_interval(lb_handle h, long long k) {
  if (int r = check_handle(h)) return r;
  if (k < 0) return fail(LB_ERR_INVALID_ARG, "check interval must be >= 0");
  h->check_every = k;
  return LB_OK;
}

int lb_init_fields(lb_handle h, const void* rho, const void* u, const void* pi1, int dtype, int on_device) {
  if (int r = check_handle(h)) return r;
  if (!rho || !u) return fail(LB_ERR_INVALID_ARG, "rho and u must not be NULL");
  if (dtype != LB_F64 && dtype != LB_F32) return fail(LB_ERR_INVALID_ARG, "bad dtype %d", dtype);
  if (int r = ensure_buffers(h)) return r;
  const size_t es = dtype == LB_F64 ? 8 : 4;
  const size_t nodes = size_t(h->nodes());
  const int d = h->d(), nc = d * (d + 1) / 2;
  const void *drho = rho, *du = u, *dpi = pi1;
  void* tmp = nullptr;
  if (!on_device) {
    const size_t n = nodes * (1 + d + (pi1 ? nc : 0));
    HIP_TRY(hipMalloc(&tmp, n * es), "hipMalloc staging");
    char* t = static_cast<char*>(tmp);
    hipError_t e = hipMemcpyAsync(t, rho, nodes * es, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(t + nodes * es, u, nodes * d * es, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess && pi1)
      e = hipMemcpyAsync(t + nodes * (1 + d) * es, pi1, nodes * nc * es, hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) {
      (void)hipFree(tmp);
      return hip_fail(e, "staging copy");
    }
    drho = t;
    du = t + nodes * es;
    dpi = pi1 ? t + nodes * (1 + d) * es : nullptr;
  }
  hipError_t e = h->ops->init(h->order, h->storage, dtype, drho, du, dpi, h->buf[0], h->args(), h->stream);
  if (tmp) {
    hipError_t s = hipStreamSynchronize(h->stream);
    (void)hipFree(tmp);
    if (e == hipSuccess) e = s;
  }
  if (e != hipSuccess) return hip_fail(e, "init kernel");
  h->cur = 0;
  h->steps = 0;
  h->ready = true;
  return LB_OK;
}

int lb_step(lb_handle h, long long n) {
  if (int r = check_handle(h)) return r;
  if (n < 0) return fail(LB_ERR_INVALID_ARG, "n must be >= 0");
  if (!h->ready) return fail(LB_ERR_STATE, "lb_step before lb_init_fields / lb_set_populations");
  if (h->closure_on && h->moment()) return fail(LB_ERR_UNSUPPORTED, "the learned closure needs population storage");
  if (h->walls && h->closure_on) return fail(LB_ERR_UNSUPPORTED, "walls and the learned closure exclude each other");
  const StepArgs a = h->args();
  for (long long k = 0; k < n; ++k) {
    hipError_t e;
    if (h->closure_on)
      e = lbrr::closure_step(h->order, h->storage, h->buf[h->cur], h->buf[1 - h->cur], a, h->cl_packed, h->cl_params,
                             h->cl_norm, h->stream);
    else if (h->walls && !h->moment())
      e = h->ops->step_walls(h->order, h->storage, h->buf[h->cur], h->buf[1 - h->cur], a, h->walls, h->stream);
    else
      e = h->ops->step(h->order, h->storage, h->buf[h->cur], h->buf[1 - h->cur], a, h->stream);
    if (e != hipSuccess) return hip_fail(e, "step kernel launch");
    h->cur ^= 1;
    ++h->steps;
    if (h->check_every > 0 && h->steps % h->check_every == 0) {
      double t[5];
      if (int r = totals(h, t)) return r;
    }
  }
  return LB_OK;
}

int lb_moments(lb_handle h, void* rho, void* u, void* pi1, int dtype, int on_device) {
  if (int r = check_handle(h)) return r;
  if (!h->ready) return fail(LB_ERR_STATE, "no state: call lb_init_fields or lb_set_populations first");
  if (dtype != LB_F64 && dtype != LB_F32) return fail(LB_ERR_INVALID_ARG, "bad dtype %d", dtype);
  const double om = 1.0 - 1.0 / h->tau;
  if (pi1 && om == 0.0 && !h->moment())
    return fail(LB_ERR_UNSUPPORTED, "pi1 is not recoverable from the stored state when tau == 1");
  const double inv_om = (pi1 && !h->moment()) ? 1.0 / om : 0.0;
  const size_t es = dtype == LB_F64 ? 8 : 4;
  const size_t nodes = size_t(h->nodes());
  const int d = h->d(), nc = d * (d + 1) / 2;
  if (on_device) {
    hipError_t e = h->ops->moments(h->storage, dtype, h->buf[h->cur], rho, u, pi1, h->args(), inv_om, h->stream);
    if (e != hipSuccess) return hip_fail(e, "moments kernel");
    HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    return LB_OK;
  }
  void* tmp = nullptr;
  HIP_TRY(hipMalloc(&tmp, nodes * (1 + d + nc) * es), "hipMalloc staging");
  char* t = static_cast<char*>(tmp);
  void* drho = rho ? t : nullptr;
  void* du = u ? t + nodes * es : nullptr;
  void* dpi = pi1 ? t + nodes * (1 + d) * es : nullptr;
  hipError_t e = h->ops->moments(h->storage, dtype, h->buf[h->cur], drho, du, dpi, h->args(), inv_om, h->stream);
  if (e == hipSuccess && rho) e = hipMemcpyAsync(rho, drho, nodes * es, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess && u) e = hipMemcpyAsync(u, du, nodes * d * es, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess && pi1) e = hipMemcpyAsync(pi1, dpi, nodes * nc * es, hipMemcpyDeviceToHost, h->stream);
  hipError_t s = hipStreamSynchronize(h->stream);
  (void)hipFree(tmp);
  if (e == hipSuccess) e = s;
  if (e != hipSuccess) return hip_fail(e, "moments");
  return LB_OK;
}

int lb_reduce(lb_handle h, double out[5]) {
  if (int r = check_handle(h)) return r;
  if (!out) return fail(LB_ERR_INVALID_ARG, "out must not be NULL");
  if (!h->ready) return fail(LB_ERR_STATE, "no state");
  return totals(h, out);
}

int lb_reduce_static(int lattice, int storage, int nx, int ny, int nz, double rho0, const void* populations,
                     double* out, void* hip_stream) {
  const LatticeOps* ops = nullptr;
  switch (lattice) {
    case LB_D2Q9: ops = &lbrr::ops_d2q9(); break;
    case LB_D3Q19: ops = &lbrr::ops_d3q19(); break;
    case LB_D3Q27: ops = &lbrr::ops_d3q27(); break;
    default: return fail(LB_ERR_INVALID_ARG, "unknown lattice %d", lattice);
  }
  if (storage != LB_STORE_FP64 && storage != LB_STORE_FP32 && storage != LB_STORE_FP16)
    return fail(LB_ERR_UNSUPPORTED, "lb_reduce_static takes population storage (FP64, FP32, FP16), got %d", storage);
  if (nx < 1 || ny < 1 || nz < 1 || (ops->d == 2 && nz != 1))
    return fail(LB_ERR_INVALID_ARG, "bad dims %d x %d x %d for this lattice", nx, ny, nz);
  const int64_t nodes = int64_t(nx) * ny * nz;
  if (nodes >= (int64_t(1) << 31)) return fail(LB_ERR_INVALID_ARG, "nx*ny*nz must be < 2^31");
  if (!std::isfinite(rho0) || !(rho0 > 0)) return fail(LB_ERR_INVALID_ARG, "rho0 must be finite and > 0");
  if (!populations || !out) return fail(LB_ERR_INVALID_ARG, "populations and out must not be NULL");
  const int nblocks = totals_blocks(nodes);
  if (nblocks > LB_REDUCE_STATIC_MAX_BLOCKS)
    return fail(LB_ERR_INVALID_ARG, "%d partial blocks exceed the static scratch (%d)", nblocks,
                LB_REDUCE_STATIC_MAX_BLOCKS);
  double* partials = nullptr;
  if (int r = static_scratch(&partials)) return r;
  StepArgs a{};
  a.nx = nx;
  a.ny = ny;
  a.nz = nz;
  a.si = nodes;  // compact [q][nz][ny][nx]
  a.sy = nx;
  a.sz = int64_t(nx) * ny;
  a.rho0 = rho0;
  a.omega1 = 0.0;
  a.lz = 1;
  a.walls = 0;
  const hipError_t e =
      ops->totals(storage, populations, partials, nblocks, out, a, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "totals kernel launch");
  return LB_OK;
}

int lb_enstrophy(lb_handle h, double* out) {
  if (int r = check_handle(h)) return r;
  if (!out) return fail(LB_ERR_INVALID_ARG, "out must not be NULL");
  if (!h->ready) return fail(LB_ERR_STATE, "no state");
  if (!h->vel) HIP_TRY(hipMalloc(&h->vel, sizeof(double) * size_t(h->nodes()) * h->d()), "hipMalloc velocity");
  hipError_t e = h->ops->velocity(h->storage, h->buf[h->cur], h->vel, h->args(), h->stream);
  if (e == hipSuccess)
    e = lbrr::launch_enstrophy(h->vel, h->d(), h->nx, h->ny, h->nz, h->walls, h->partials, h->nblocks, h->dev_out,
                               h->stream);
  if (e != hipSuccess) return hip_fail(e, "enstrophy kernels");
  double s = 0.0;
  HIP_TRY(hipMemcpyAsync(&s, h->dev_out, sizeof(double), hipMemcpyDeviceToHost, h->stream), "copy enstrophy");
  HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  // trapezoid volume: a walled axis of n nodes spans n - 1 cells, a periodic one n
  double vol = 1.0;
  const int dims[3] = {h->nx, h->ny, h->nz};
  for (int k = 0; k < h->d(); ++k) vol *= double((h->walls >> k & 1) ? dims[k] - 1 : dims[k]);
  *out = s / vol;
  if (!std::isfinite(*out)) return fail(LB_ERR_UNSTABLE, "non-finite enstrophy");
  return LB_OK;
}

int lb_get_populations(lb_handle h, void* dst, int on_device) {
  if (int r = check_handle(h)) return r;
  if (!dst) return fail(LB_ERR_INVALID_ARG, "dst must not be NULL");
  if (!h->ready) return fail(LB_ERR_STATE, "no state");
  const size_t bytes = size_t(h->nodes()) * h->q() * elem_size(h->storage);
  void* d = dst;
  if (!on_device) HIP_TRY(hipMalloc(&d, bytes), "hipMalloc staging");
  hipError_t e = h->moment() ? h->ops->mpopulations(h->order, h->storage, h->buf[h->cur], d, h->args(), h->stream)
                             : h->ops->repack(h->storage, h->buf[h->cur], d, true, h->args(), h->stream);
  if (e == hipSuccess && !on_device) e = hipMemcpyAsync(dst, d, bytes, hipMemcpyDeviceToHost, h->stream);
  hipError_t s = hipStreamSynchronize(h->stream);
  if (!on_device) (void)hipFree(d);
  if (e == hipSuccess) e = s;
  if (e != hipSuccess) return hip_fail(e, "copy populations out");
  return LB_OK;
}

int lb_set_populations(lb_handle h, const void* src, int on_device) {
  if (int r = check_handle(h)) return r;
  if (!src) return fail(LB_ERR_INVALID_ARG, "src must not be NULL");
  if (h->moment())
    return fail(LB_ERR_UNSUPPORTED, "moment storage holds only states reachable by the collision; use lb_init_fields");
  if (int r = ensure_buffers(h)) return r;
  const size_t bytes = size_t(h->nodes()) * h->q() * elem_size(h->storage);
  const void* d = src;
  void* tmp = nullptr;
  if (!on_device) {
    HIP_TRY(hipMalloc(&tmp, bytes), "hipMalloc staging");
    hipError_t e = hipMemcpyAsync(tmp, src, bytes, hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) {
      (void)hipFree(tmp);
      return hip_fail(e, "copy populations in");
    }
    d = tmp;
  }
  hipError_t e = h->ops->repack(h->storage, d, h->buf[h->cur], false, h->args(), h->stream);
  hipError_t s = hipStreamSynchronize(h->stream);
  if (tmp) (void)hipFree(tmp);
  if (e == hipSuccess) e = s;
  if (e != hipSuccess) return hip_fail(e, "copy populations in");
  h->ready = true;
  return LB_OK;
}

long long lb_step_count(lb_handle h) { return h ? h->steps : -1; }

double lb_bytes_per_update(lb_handle h) {
  if (!h) return 0.0;
  return 2.0 * h->nvalues() * double(elem_size(h->storage));
}

void lb_destroy(lb_handle h) {
  if (!h) return;
  (void)hipSetDevice(h->device);
  if (h->buf[0]) (void)hipStreamSynchronize(h->stream);
  h->release();
  h->release_closure();
  delete h;
}

// ---------------------------------------------------------------------------
// Learned closure (D2Q9).

namespace {

// Reusable device workspace of the MLP entry points (grown on demand; calls
// that overlap on one device must not share it).
struct Workspace {
  void* ptr = nullptr;
  size_t size = 0;
  int device = -1;
};
Workspace g_ws;

int workspace(size_t bytes, void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (g_ws.ptr && (g_ws.size < bytes || g_ws.device != dev)) {
    int cur = dev;
    (void)hipSetDevice(g_ws.device);
    (void)hipDeviceSynchronize();
    (void)hipFree(g_ws.ptr);
    (void)hipSetDevice(cur);
    g_ws.ptr = nullptr;
  }
  if (!g_ws.ptr) {
    const size_t sz = bytes < (size_t(1) << 20) ? (size_t(1) << 20) : bytes;
    HIP_TRY(hipMalloc(&g_ws.ptr, sz), "hipMalloc MLP workspace");
    g_ws.size = sz;
    g_ws.device = dev;
  }
  *out = g_ws.ptr;
  return LB_OK;
}

}  // namespace

int lb_set_closure(lb_handle h, const float* params, const float* norm, int enable) {
  if (int r = check_handle(h)) return r;
  if (h->lattice != LB_D2Q9) return fail(LB_ERR_UNSUPPORTED, "the learned closure is implemented for D2Q9 only");
  if (enable && h->moment()) return fail(LB_ERR_UNSUPPORTED, "the learned closure needs population storage");
  if (!enable) {
    h->closure_on = false;
    return LB_OK;
  }
  if (!params || !norm) return fail(LB_ERR_INVALID_ARG, "params and norm must not be NULL");
  // each buffer on its own, through a temporary: after a failed allocation the
  // handle holds only complete buffers, and the next call allocates the rest
  auto alloc = [](auto*& dst, size_t bytes) {
    void* p = nullptr;
    const hipError_t e = dst ? hipSuccess : hipMalloc(&p, bytes);
    if (e == hipSuccess && !dst) dst = static_cast<std::remove_reference_t<decltype(dst)>>(p);
    return e;
  };
  HIP_TRY(alloc(h->cl_params, sizeof(float) * lbrr::kMlpNParam), "hipMalloc closure params");
  HIP_TRY(alloc(h->cl_norm, sizeof(float) * lbrr::kMlpNNorm), "hipMalloc closure norm");
  HIP_TRY(alloc(h->cl_packed, sizeof(uint16_t) * (lbrr::kMlpNPacked + lbrr::kMlpNRegImage)),
          "hipMalloc closure weights");
  HIP_TRY(hipMemcpyAsync(h->cl_params, params, sizeof(float) * lbrr::kMlpNParam, hipMemcpyDeviceToDevice, h->stream),
          "copy closure params");
  HIP_TRY(hipMemcpyAsync(h->cl_norm, norm, sizeof(float) * lbrr::kMlpNNorm, hipMemcpyDeviceToDevice, h->stream),
          "copy closure norm");
  hipError_t e = lbrr::mlp_pack_step(h->cl_params, h->cl_packed, h->stream);
  if (e != hipSuccess) return hip_fail(e, "pack closure weights");
  h->closure_on = true;
  return LB_OK;
}

int lb_closure_features(lb_handle h, const double* a_target, double plain_weight, float* features, float* labels) {
  if (int r = check_handle(h)) return r;
  if (h->lattice != LB_D2Q9) return fail(LB_ERR_UNSUPPORTED, "the learned closure is implemented for D2Q9 only");
  if (!features || !labels) return fail(LB_ERR_INVALID_ARG, "features and labels must not be NULL");
  if (h->moment()) return fail(LB_ERR_UNSUPPORTED, "closure features need population storage");
  if (!h->ready) return fail(LB_ERR_STATE, "no state");
  void* m = nullptr;
  if (int r = workspace(sizeof(float) * 3 * size_t(h->nodes()), &m)) return r;
  hipError_t e = lbrr::closure_features(h->storage, h->buf[h->cur], static_cast<float*>(m), h->args(), a_target,
                                        plain_weight, features, labels, h->stream);
  if (e != hipSuccess) return hip_fail(e, "closure features");
  return LB_OK;
}

int lb_closure_coarsen(const void* rho, const void* u, const void* pi1, int dtype, int nfx, int nfy, int factor,
                       double alpha, double beta, double* rho_c, double* u_c, double* pi1_c, void* hip_stream) {
  if (!rho || !u || !pi1 || !rho_c || !u_c || !pi1_c) return fail(LB_ERR_INVALID_ARG, "NULL pointer");
  if (dtype != LB_F64 && dtype != LB_F32) return fail(LB_ERR_INVALID_ARG, "bad dtype %d", dtype);
  if (factor < 1 || nfx < factor || nfy < factor || nfx % factor || nfy % factor)
    return fail(LB_ERR_INVALID_ARG, "fine dims must be positive multiples of the factor");
  if (!std::isfinite(alpha) || !std::isfinite(beta)) return fail(LB_ERR_INVALID_ARG, "alpha, beta must be finite");
  hipError_t e = lbrr::closure_coarsen(dtype, rho, u, pi1, nfx, nfy, factor, alpha, beta, rho_c, u_c, pi1_c,
                                       static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "coarsen kernel");
  return LB_OK;
}

int lb_mlp_forward(const float* params, const float* norm, const float* x, long long n, float* y, void* hip_stream) {
  if (!params || !norm || (n > 0 && (!x || !y))) return fail(LB_ERR_INVALID_ARG, "NULL pointer");
  if (n < 0) return fail(LB_ERR_INVALID_ARG, "n must be >= 0");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  void* ws = nullptr;
  if (int r = workspace(sizeof(uint16_t) * lbrr::kMlpNPacked, &ws)) return r;
  uint16_t* packed = static_cast<uint16_t*>(ws);
  hipError_t e = lbrr::mlp_pack(params, packed, s);
  if (e == hipSuccess) e = lbrr::mlp_infer(x, n, packed, params, norm, y, s);
  if (e != hipSuccess) return hip_fail(e, "MLP forward");
  return LB_OK;
}

int lb_mlp_gradient(const float* params, const float* norm, const float* x, const float* t, long long n,
                    const int* idx, int batch, float* grad, float* loss, void* hip_stream) {
  if (!params || !norm || !x || !t || !idx || !grad) return fail(LB_ERR_INVALID_ARG, "NULL pointer");
  if (batch < 1 || n < 1) return fail(LB_ERR_INVALID_ARG, "batch and n must be >= 1");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int nb = lbrr::mlp_train_blocks(batch);
  const size_t packed_bytes = sizeof(uint16_t) * lbrr::kMlpNPacked;
  const size_t part_bytes = sizeof(float) * size_t(nb) * lbrr::kMlpNParam;
  void* ws = nullptr;
  if (int r = workspace(packed_bytes + part_bytes + sizeof(float) * size_t(nb) + 256, &ws)) return r;
  char* base = static_cast<char*>(ws);
  uint16_t* packed = reinterpret_cast<uint16_t*>(base);
  float* gpart = reinterpret_cast<float*>(base + packed_bytes);
  float* lpart = reinterpret_cast<float*>(base + packed_bytes + part_bytes);
  hipError_t e = lbrr::mlp_pack(params, packed, s);
  if (e == hipSuccess) e = lbrr::mlp_gradient(x, t, n, idx, batch, packed, params, norm, gpart, lpart, grad, loss, s);
  if (e != hipSuccess) return hip_fail(e, "MLP gradient");
  return LB_OK;
}

int lb_column_stats(const float* x, long long n, int dim, float* mean, float* std, void* hip_stream) {
  if (!x || !mean || !std) return fail(LB_ERR_INVALID_ARG, "NULL pointer");
  if (n < 1 || dim < 1) return fail(LB_ERR_INVALID_ARG, "n and dim must be >= 1");
  hipError_t e = lbrr::column_stats(x, n, dim, mean, std, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "column stats kernel");
  return LB_OK;
}

int lb_mlp_adam(float* params, float* m, float* v, const float* grad, long long step, float lr, float beta1,
                float beta2, float eps, void* hip_stream) {
  if (!params || !m || !v || !grad) return fail(LB_ERR_INVALID_ARG, "NULL pointer");
  if (step < 1) return fail(LB_ERR_INVALID_ARG, "step counts from 1");
  hipError_t e = lbrr::mlp_adam(params, m, v, grad, step, lr, beta1, beta2, eps, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "Adam kernel");
  return LB_OK;
}

int lb_probe_copy(const void* src, void* dst, size_t n, void* hip_stream) {
  if (!src || !dst) return fail(LB_ERR_INVALID_ARG, "NULL pointer");
  if (n % 16 || (reinterpret_cast<uintptr_t>(src) % 16) || (reinterpret_cast<uintptr_t>(dst) % 16))
    return fail(LB_ERR_INVALID_ARG, "copy needs 16-byte aligned pointers and a size multiple of 16");
  hipError_t e = lbrr::launch_copy(src, dst, n, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "copy kernel");
  return LB_OK;
}

int lb_probe_bandwidth(int kind, int vec_bytes, int blocks_per_cu, int nontemporal, int streams, const void* src,
                       void* dst, size_t n, void* hip_stream) {
  if (kind < 0 || kind > 3) return fail(LB_ERR_INVALID_ARG, "kind must be 0 (copy), 1 (read), 2 (write) or 3 (streams)");
  if (vec_bytes != 4 && vec_bytes != 8 && vec_bytes != 16) return fail(LB_ERR_INVALID_ARG, "vec_bytes must be 4, 8 or 16");
  if (blocks_per_cu < 0 || blocks_per_cu > 64) return fail(LB_ERR_INVALID_ARG, "blocks_per_cu must be in [0, 64]");
  if (kind == 3 && (streams < 1 || streams > 32)) return fail(LB_ERR_INVALID_ARG, "streams must be in [1, 32]");
  if (kind == 3 && blocks_per_cu != 0) return fail(LB_ERR_INVALID_ARG, "the stream copy launches one thread per element");
  if (!src || !dst) return fail(LB_ERR_INVALID_ARG, "NULL pointer");
  if (n % 16 || (reinterpret_cast<uintptr_t>(src) % 16) || (reinterpret_cast<uintptr_t>(dst) % 16))
    return fail(LB_ERR_INVALID_ARG, "probes need 16-byte aligned pointers and a size multiple of 16");
  if (kind == 3 && (n / size_t(vec_bytes)) % size_t(streams))
    return fail(LB_ERR_INVALID_ARG, "the stream copy needs a whole number of elements per stream");
  int dev = 0, cus = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "hipDeviceGetAttribute");
  const hipError_t e = lbrr::launch_probe(kind, vec_bytes, blocks_per_cu, nontemporal, streams, src, dst, n, cus,
                                          static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "probe kernel");
  return LB_OK;
}

}  // extern "C"
