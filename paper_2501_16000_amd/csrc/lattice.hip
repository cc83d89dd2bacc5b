// lattice.hip -- the C ABI of include/oreg.h: lattice handles, validation,
// device buffers, stream ordering and error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "kernels.hpp"
#include "oreg.h"

using namespace oreg;

struct lb_lattice {
  lb_options opt{};
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  void* buf[2] = {nullptr, nullptr};  // A/B population buffers
  int cur = 0;                        // buffer holding the current state
  size_t elem = 8;                    // bytes per stored population
  Geometry geo{};
  int fused_rows[8] = {};             // output rows per strip of fused launches, by step count
  Coef64 coef{};
  double theta_energy = 0.0;          // theta of p = rho theta in the energy sum
  bool initialized = false;
  int64_t t = 0;
  double* tmp = nullptr;              // 3 * plane FP64 staging (lazy)
  double* aux = nullptr;              // kDiagBlocks*6 partials + 8 results
  unsigned int* counter = nullptr;    // invalid-input count of lb_init*
  std::string err;
};

namespace {

thread_local std::string t_err;

lb_status fail(lb_lattice* h, lb_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (h) h->err = buf;
  t_err = buf;
  return st;
}

lb_status hip_fail(lb_lattice* h, hipError_t e, const char* what) {
  const lb_status st = (e == hipErrorOutOfMemory) ? LB_ENOMEM : LB_EDEVICE;
  return fail(h, st, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

#define HIP_TRY(h, call)                                 \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return hip_fail((h), e_, #call); \
  } while (0)

// Makes the lattice's device current for the scope of one call.
struct DeviceScope {
  int prev = -1;
  bool ok = true;
  explicit DeviceScope(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = (hipSetDevice(dev) == hipSuccess);
  }
  ~DeviceScope() {
    if (prev >= 0) {
      int now = -1;
      if (hipGetDevice(&now) == hipSuccess && now != prev) (void)hipSetDevice(prev);
    }
  }
};

bool is_finite(double v) { return std::isfinite(v); }

size_t storage_bytes(lb_storage s) {
  switch (s) {
    case LB_F64: return 8;
    case LB_F32S: return 4;
    case LB_F16S:
    case LB_BF16S: return 2;
  }
  return 0;
}

lb_status validate(const lb_options* o) {
  if (!o) return fail(nullptr, LB_EINVAL, "options pointer is NULL");
  if (o->nx < 1 || o->ny < 1) return fail(nullptr, LB_EINVAL, "nx and ny must be >= 1 (got %d x %d)", o->nx, o->ny);
  if (o->equilibrium != LB_EQ_GUIDED && o->equilibrium != LB_EQ_POLY2)
    return fail(nullptr, LB_EINVAL, "unknown equilibrium %d", (int)o->equilibrium);
  if (o->storage < LB_F64 || o->storage > LB_BF16S)
    return fail(nullptr, LB_EINVAL, "unknown storage %d", (int)o->storage);
  if (o->collision != LB_COLL_OREG && o->collision != LB_COLL_BGK)
    return fail(nullptr, LB_EINVAL, "unknown collision %d", (int)o->collision);
  if (o->boundary_x != LB_BC_PERIODIC && o->boundary_x != LB_BC_BOUNCEBACK)
    return fail(nullptr, LB_EINVAL, "unknown boundary %d", (int)o->boundary_x);
  // A HIP launch covers fewer than 2^32 work-items per dimension: the
  // single-step sweep launches sweep_work_items() of them (the row rounded up
  // to the storage's workgroup tile), the per-node kernels nx * ny rounded up
  // to 256.
  const int64_t plane = (int64_t)o->nx * (int64_t)o->ny;
  const int64_t items = std::max(sweep_work_items(o->storage, o->nx, o->ny), (plane + 255) / 256 * 256);
  if (items > (int64_t)4294967040LL)
    return fail(nullptr, LB_EINVAL, "lattice %d x %d is too large for one launch", o->nx, o->ny);
  if (!is_finite(o->tau) || !(o->tau > 0.5))
    return fail(nullptr, LB_EINVAL, "tau must be finite and > 1/2 (got %g)", o->tau);
  if (!is_finite(o->theta)) return fail(nullptr, LB_EINVAL, "theta must be finite");
  if (o->equilibrium == LB_EQ_GUIDED && !(o->theta > 0.0 && o->theta < 1.0))
    return fail(nullptr, LB_EINVAL, "guided equilibrium needs 0 < theta < 1 (got %g)", o->theta);
  if (o->equilibrium == LB_EQ_POLY2 && std::fabs(o->theta - 1.0 / 3.0) > 1e-12)
    return fail(nullptr, LB_EINVAL, "polynomial equilibrium needs theta = 1/3 (got %.17g)", o->theta);
  if (o->storage != LB_F64 && (!is_finite(o->rho0) || !(o->rho0 > 0.0)))
    return fail(nullptr, LB_EINVAL, "rho0 must be finite and > 0 for shifted storage");
  if (o->fuse_steps < 0 || o->fuse_steps > 2)
    return fail(nullptr, LB_EINVAL, "fuse_steps must be 0, 1 or 2 (got %d)", o->fuse_steps);
  return LB_OK;
}

Coef64 make_coef(const lb_options& o) {
  const double th = (o.equilibrium == LB_EQ_POLY2) ? 1.0 / 3.0 : o.theta;
  Coef64 c;
  c.theta = th;
  c.a0 = 1.0 - th;
  c.a1 = 0.5 * th;
  c.kappa0 = (1.0 - 1.0 / o.tau) / (2.0 * th * th);
  c.omega = 1.0 / o.tau;
  c.rho0 = (o.storage == LB_F64) ? 0.0 : o.rho0;
  return c;
}

lb_status ensure_tmp(lb_lattice* h) {
  if (h->tmp) return LB_OK;
  HIP_TRY(h, hipMalloc((void**)&h->tmp, 3 * (size_t)h->geo.plane * sizeof(double)));
  return LB_OK;
}

lb_status check_handle(lb_lattice* h) {
  if (!h) return fail(nullptr, LB_EINVAL, "lattice handle is NULL");
  return LB_OK;
}

// Partial sums of lb_diagnostics_device_noalloc: one row of six per
// reduction workgroup, in a file-scope device array instead of an allocation.
// Every GPU the library runs on holds its own copy until the process ends.
// In host code `scratch` only names the symbol: its device address comes
// from hipGetSymbolAddress, once per device, and only that address is passed
// to kernels.
constexpr int kMaxScratchDevices = 64;
static __device__ __align__(256) double scratch[kDiagBlocks * 6];
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of `scratch` on `dev` (the current device), looked up on
// the first call for that device.
lb_status scratch_ptr(lb_lattice* h, int dev, double** out) {
  if (dev < 0 || dev >= kMaxScratchDevices)
    return fail(h, LB_EDEVICE, "device %d: no scratch slot (at most %d devices)", dev,
                kMaxScratchDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(h, e != hipSuccess ? e : hipErrorUnknown,
                                               "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<double*>(g_scratch_ptr[dev]);
  return LB_OK;
}

lb_status finish_init(lb_lattice* h) {
  unsigned int bad = 0;
  HIP_TRY(h, hipMemcpyAsync(&bad, h->counter, sizeof bad, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  if (bad) {
    h->initialized = false;
    return fail(h, LB_EINVAL, "%u node(s) with a non-finite field or rho <= 0", bad);
  }
  h->initialized = true;
  h->t = 0;
  return LB_OK;
}

}  // namespace

extern "C" {

void lb_options_init(lb_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->tau = 1.0;
  o->theta = 1.0 / 3.0;
  o->equilibrium = LB_EQ_GUIDED;
  o->storage = LB_F64;
  o->collision = LB_COLL_OREG;
  o->boundary_x = LB_BC_PERIODIC;
  o->rho0 = 1.0;
  o->stream = nullptr;
  o->use_stream = 0;
  o->device = -1;
  o->check_nonfinite = 0;
  o->fuse_steps = 0;
}

lb_status lb_create(int nx, int ny, double tau, double theta, lb_equilibrium eq,
                    lb_lattice** out) {
  lb_options o;
  lb_options_init(&o);
  o.nx = nx;
  o.ny = ny;
  o.tau = tau;
  o.theta = theta;
  o.equilibrium = eq;
  return lb_create_ex(&o, out);
}

lb_status lb_create_ex(const lb_options* opt, lb_lattice** out) {
  if (!out) return fail(nullptr, LB_EINVAL, "out pointer is NULL");
  *out = nullptr;
  lb_status st = validate(opt);
  if (st != LB_OK) return st;

  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev < 1)
    return fail(nullptr, LB_EDEVICE, "no HIP device available (%s)",
                e != hipSuccess ? hipGetErrorString(e) : "count is 0");
  int dev = opt->device;
  if (dev < 0) {
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  }
  if (dev >= ndev) return fail(nullptr, LB_EINVAL, "device %d out of range (%d devices)", dev, ndev);

  lb_lattice* h = new (std::nothrow) lb_lattice;
  if (!h) return fail(nullptr, LB_ENOMEM, "host allocation failed");
  h->opt = *opt;
  h->opt.device = dev;
  h->device = dev;
  h->elem = storage_bytes(opt->storage);
  h->geo.nx = opt->nx;
  h->geo.ny = opt->ny;
  h->geo.plane = (int64_t)opt->nx * (int64_t)opt->ny;
  h->coef = make_coef(*opt);
  h->theta_energy = h->coef.theta;

  DeviceScope ds(dev);
  if (!ds.ok) {
    delete h;
    return fail(nullptr, LB_EDEVICE, "cannot select device %d", dev);
  }
  auto cleanup = [&](lb_status s) {
    lb_destroy(h);
    return s;
  };
  if (opt->use_stream) {
    h->stream = static_cast<hipStream_t>(opt->stream);
  } else {
    e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return cleanup(hip_fail(nullptr, e, "hipStreamCreateWithFlags"));
    h->own_stream = true;
  }
  const size_t bytes = 9 * (size_t)h->geo.plane * h->elem;
  for (int b = 0; b < 2; ++b) {
    e = hipMalloc(&h->buf[b], bytes);
    if (e != hipSuccess) return cleanup(hip_fail(nullptr, e, "hipMalloc(populations)"));
  }
  e = hipMalloc((void**)&h->aux, (kDiagBlocks * 6 + 8) * sizeof(double));
  if (e != hipSuccess) return cleanup(hip_fail(nullptr, e, "hipMalloc(aux)"));
  e = hipMalloc((void**)&h->counter, sizeof(unsigned int));
  if (e != hipSuccess) return cleanup(hip_fail(nullptr, e, "hipMalloc(counter)"));
  for (int L = 2; L <= fused_levels(h->opt.storage); ++L)
    if (fused_levels_available(h->opt.collision, h->opt.boundary_x, h->opt.storage, L))
      h->fused_rows[L] = fused_rows(h->opt.storage, h->geo.nx, h->geo.ny,
                                    fused_shape(h->opt.storage, L), L);
  *out = h;
  return LB_OK;
}

lb_status lb_init(lb_lattice* h, const double* rho, const double* ux, const double* uy) {
  if (check_handle(h) != LB_OK) return LB_EINVAL;
  if (!rho || !ux || !uy) return fail(h, LB_EINVAL, "field pointer is NULL");
  const int64_t n = h->geo.plane;
  for (int64_t i = 0; i < n; ++i) {
    if (!is_finite(rho[i]) || !is_finite(ux[i]) || !is_finite(uy[i]) || !(rho[i] > 0.0))
      return fail(h, LB_EINVAL, "node %lld has a non-finite field or rho <= 0", (long long)i);
  }
  DeviceScope ds(h->device);
  if (!ds.ok) return fail(h, LB_EDEVICE, "cannot select device %d", h->device);
  lb_status st = ensure_tmp(h);
  if (st != LB_OK) return st;
  const size_t bytes = (size_t)n * sizeof(double);
  HIP_TRY(h, hipMemcpyAsync(h->tmp, rho, bytes, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(h, hipMemcpyAsync(h->tmp + n, ux, bytes, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(h, hipMemcpyAsync(h->tmp + 2 * n, uy, bytes, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(h, hipMemsetAsync(h->counter, 0, sizeof(unsigned int), h->stream));
  HIP_TRY(h, launch_init(h->opt.equilibrium, h->opt.storage, h->tmp, h->tmp + n, h->tmp + 2 * n,
                         h->buf[h->cur], h->geo, h->coef, h->counter, h->stream));
  return finish_init(h);
}

lb_status lb_init_device(lb_lattice* h, const double* rho, const double* ux, const double* uy) {
  if (check_handle(h) != LB_OK) return LB_EINVAL;
  if (!rho || !ux || !uy) return fail(h, LB_EINVAL, "field pointer is NULL");
  DeviceScope ds(h->device);
  if (!ds.ok) return fail(h, LB_EDEVICE, "cannot select device %d", h->device);
  HIP_TRY(h, hipMemsetAsync(h->counter, 0, sizeof(unsigned int), h->stream));
  HIP_TRY(h, launch_init(h->opt.equilibrium, h->opt.storage, rho, ux, uy, h->buf[h->cur], h->geo,
                         h->coef, h->counter, h->stream));
  return finish_init(h);
}

lb_status lb_step(lb_lattice* h, int64_t n) {
  if (check_handle(h) != LB_OK) return LB_EINVAL;
  if (n < 0) return fail(h, LB_EINVAL, "n must be >= 0 (got %lld)", (long long)n);
  if (!h->initialized) return fail(h, LB_ESTATE, "lattice is not initialized");
  if (n == 0) return LB_OK;
  DeviceScope ds(h->device);
  if (!ds.ok) return fail(h, LB_EDEVICE, "cannot select device %d", h->device);
  // Fused launches advance K steps each.  A remainder of two or more steps
  // runs as one shorter fused launch where that is compiled (periodic OReg:
  // it reads and writes the state once, where single steps would do so per
  // step), otherwise, and for a single step, one step per launch.
  const bool fuse =
      h->opt.fuse_steps == 2 ||
      (h->opt.fuse_steps == 0 && fused_worthwhile(h->opt.storage, h->geo.nx, h->geo.ny));
  const int64_t K = fuse ? fused_levels(h->opt.storage) : 1;
  int64_t left = n;
  while (K > 1 && left >= 2) {
    const int L = (int)std::min<int64_t>(K, left);
    if (!fused_levels_available(h->opt.collision, h->opt.boundary_x, h->opt.storage, L)) break;
    HIP_TRY(h, launch_fused_sweep(h->opt.equilibrium, h->opt.collision, h->opt.boundary_x,
                                  h->opt.storage, h->buf[h->cur], h->buf[1 - h->cur], h->geo,
                                  h->coef, h->fused_rows[L], L, h->stream));
    h->cur = 1 - h->cur;
    h->t += L;
    left -= L;
  }
  for (; left > 0; --left) {
    HIP_TRY(h, launch_sweep(h->opt.equilibrium, h->opt.collision, h->opt.boundary_x,
                            h->opt.storage, h->buf[h->cur], h->buf[1 - h->cur], h->geo, h->coef,
                            h->stream));
    h->cur = 1 - h->cur;
    h->t += 1;
  }
  if (h->opt.check_nonfinite) {
    double d[6];
    lb_status st = lb_diagnostics(h, d);
    if (st != LB_OK) return st;
    if (d[5] > 0) return fail(h, LB_ENONFINITE, "%.0f node(s) hold non-finite populations", d[5]);
  }
  return LB_OK;
}

lb_status lb_moments_device(lb_lattice* h, double* out_dev) {
  if (check_handle(h) != LB_OK) return LB_EINVAL;
  if (!out_dev) return fail(h, LB_EINVAL, "output pointer is NULL");
  if (!h->initialized) return fail(h, LB_ESTATE, "lattice is not initialized");
  DeviceScope ds(h->device);
  if (!ds.ok) return fail(h, LB_EDEVICE, "cannot select device %d", h->device);
  HIP_TRY(h, launch_moments(h->opt.storage, h->buf[h->cur], out_dev, h->geo, h->coef, h->stream));
  return LB_OK;
}

lb_status lb_moments(lb_lattice* h, double* out) {
  if (check_handle(h) != LB_OK) return LB_EINVAL;
  if (!out) return fail(h, LB_EINVAL, "output pointer is NULL");
  if (!h->initialized) return fail(h, LB_ESTATE, "lattice is not initialized");
  DeviceScope ds(h->device);
  if (!ds.ok) return fail(h, LB_EDEVICE, "cannot select device %d", h->device);
  lb_status st = ensure_tmp(h);
  if (st != LB_OK) return st;
  HIP_TRY(h, launch_moments(h->opt.storage, h->buf[h->cur], h->tmp, h->geo, h->coef, h->stream));
  HIP_TRY(h, hipMemcpyAsync(out, h->tmp, 3 * (size_t)h->geo.plane * sizeof(double),
                            hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return LB_OK;
}

lb_status lb_populations(lb_lattice* h, double* out) {
  if (check_handle(h) != LB_OK) return LB_EINVAL;
  if (!out) return fail(h, LB_EINVAL, "output pointer is NULL");
  if (!h->initialized) return fail(h, LB_ESTATE, "lattice is not initialized");
  DeviceScope ds(h->device);
  if (!ds.ok) return fail(h, LB_EDEVICE, "cannot select device %d", h->device);
  lb_status st = ensure_tmp(h);
  if (st != LB_OK) return st;
  const int64_t n = h->geo.plane;
  for (int i = 0; i < 9; ++i) {
    // The staging buffer holds three planes; cycle through them so that a
    // plane is not overwritten before its copy has been issued.
    double* stage = h->tmp + (i % 3) * n;
    HIP_TRY(h, launch_export_plane(h->opt.storage, i, h->buf[h->cur], stage, h->geo, h->coef,
                                   h->stream));
    HIP_TRY(h, hipMemcpyAsync(out + (size_t)i * n, stage, (size_t)n * sizeof(double),
                              hipMemcpyDeviceToHost, h->stream));
  }
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return LB_OK;
}

lb_status lb_set_populations(lb_lattice* h, const double* in) {
  if (check_handle(h) != LB_OK) return LB_EINVAL;
  if (!in) return fail(h, LB_EINVAL, "input pointer is NULL");
  const int64_t n = h->geo.plane;
  for (int64_t c = 0; c < n; ++c) {
    double rho = 0.0;
    for (int i = 0; i < 9; ++i) {
      const double v = in[(size_t)i * n + c];
      if (!is_finite(v)) return fail(h, LB_EINVAL, "population %d of node %lld is not finite", i, (long long)c);
      rho += v;
    }
    if (!(rho > 0.0)) return fail(h, LB_EINVAL, "node %lld has sum_i f_i <= 0", (long long)c);
  }
  DeviceScope ds(h->device);
  if (!ds.ok) return fail(h, LB_EDEVICE, "cannot select device %d", h->device);
  lb_status st = ensure_tmp(h);
  if (st != LB_OK) return st;
  for (int i = 0; i < 9; ++i) {
    double* stage = h->tmp + (i % 3) * n;
    HIP_TRY(h, hipMemcpyAsync(stage, in + (size_t)i * n, (size_t)n * sizeof(double),
                              hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, launch_import_plane(h->opt.storage, i, stage, h->buf[h->cur], h->geo, h->coef,
                                   h->stream));
  }
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  h->initialized = true;
  h->t = 0;
  return LB_OK;
}

lb_status lb_diagnostics(lb_lattice* h, double out[6]) {
  if (check_handle(h) != LB_OK) return LB_EINVAL;
  if (!out) return fail(h, LB_EINVAL, "output pointer is NULL");
  if (!h->initialized) return fail(h, LB_ESTATE, "lattice is not initialized");
  DeviceScope ds(h->device);
  if (!ds.ok) return fail(h, LB_EDEVICE, "cannot select device %d", h->device);
  double* result = h->aux + kDiagBlocks * 6;
  HIP_TRY(h, launch_diagnostics(h->opt.storage, h->buf[h->cur], h->aux, result, h->geo, h->coef,
                                h->theta_energy, h->stream));
  HIP_TRY(h, hipMemcpyAsync(out, result, 6 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return LB_OK;
}

lb_status lb_diagnostics_device_noalloc(lb_lattice* h, double* out_dev) {
  if (check_handle(h) != LB_OK) return LB_EINVAL;
  if (!out_dev) return fail(h, LB_EINVAL, "output pointer is NULL");
  if (!h->initialized) return fail(h, LB_ESTATE, "lattice is not initialized");
  DeviceScope ds(h->device);
  if (!ds.ok) return fail(h, LB_EDEVICE, "cannot select device %d", h->device);
  double* partials = nullptr;
  lb_status st = scratch_ptr(h, h->device, &partials);
  if (st != LB_OK) return st;
  // The same two kernels as lb_diagnostics, in the same reduction order; every
  // partial is written before the final kernel reads it, so nothing is cleared.
  HIP_TRY(h, launch_diagnostics(h->opt.storage, h->buf[h->cur], partials, out_dev, h->geo,
                                h->coef, h->theta_energy, h->stream));
  return LB_OK;
}

lb_status lb_density_profile(lb_lattice* h, double* out) {
  if (check_handle(h) != LB_OK) return LB_EINVAL;
  if (!out) return fail(h, LB_EINVAL, "output pointer is NULL");
  if (!h->initialized) return fail(h, LB_ESTATE, "lattice is not initialized");
  DeviceScope ds(h->device);
  if (!ds.ok) return fail(h, LB_EDEVICE, "cannot select device %d", h->device);
  lb_status st = ensure_tmp(h);
  if (st != LB_OK) return st;
  HIP_TRY(h, launch_profile(h->opt.storage, h->buf[h->cur], h->tmp, h->geo, h->coef, h->stream));
  HIP_TRY(h, hipMemcpyAsync(out, h->tmp, (size_t)h->geo.nx * sizeof(double),
                            hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return LB_OK;
}

lb_status lb_sync(lb_lattice* h) {
  if (check_handle(h) != LB_OK) return LB_EINVAL;
  DeviceScope ds(h->device);
  if (!ds.ok) return fail(h, LB_EDEVICE, "cannot select device %d", h->device);
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return LB_OK;
}

int64_t lb_time(const lb_lattice* h) { return h ? h->t : -1; }

lb_status lb_get_options(const lb_lattice* h, lb_options* out) {
  if (!h || !out) return fail(nullptr, LB_EINVAL, "NULL argument");
  *out = h->opt;
  return LB_OK;
}

int64_t lb_device_bytes(const lb_lattice* h) {
  if (!h) return 0;
  int64_t b = 2 * 9 * h->geo.plane * (int64_t)h->elem;
  b += (kDiagBlocks * 6 + 8) * (int64_t)sizeof(double) + (int64_t)sizeof(unsigned int);
  if (h->tmp) b += 3 * h->geo.plane * (int64_t)sizeof(double);
  return b;
}

lb_status lb_destroy(lb_lattice* h) {
  if (!h) return LB_OK;
  lb_status st = LB_OK;
  {
    DeviceScope ds(h->device);
    if ((h->stream || !h->own_stream) && hipStreamSynchronize(h->stream) != hipSuccess)
      st = LB_EDEVICE;
    for (int b = 0; b < 2; ++b)
      if (h->buf[b]) (void)hipFree(h->buf[b]);
    if (h->tmp) (void)hipFree(h->tmp);
    if (h->aux) (void)hipFree(h->aux);
    if (h->counter) (void)hipFree(h->counter);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  }
  delete h;
  return st;
}

lb_status lb_copy_device(const void* src, void* dst, int64_t bytes, void* hip_stream) {
  if (!src || !dst) return fail(nullptr, LB_EINVAL, "lb_copy_device: NULL buffer");
  if (bytes < 0 || bytes % 16 != 0)
    return fail(nullptr, LB_EINVAL, "lb_copy_device: %lld bytes is not a multiple of 16",
                (long long)bytes);
  const uintptr_t a = reinterpret_cast<uintptr_t>(src), b = reinterpret_cast<uintptr_t>(dst);
  if ((a | b) % 16 != 0)
    return fail(nullptr, LB_EINVAL, "lb_copy_device: buffers must be 16-byte aligned");
  if (bytes > 0 && a < b + (uintptr_t)bytes && b < a + (uintptr_t)bytes)
    return fail(nullptr, LB_EINVAL, "lb_copy_device: buffers overlap");
  if (bytes == 0) return LB_OK;
  const hipError_t e = launch_copy(src, dst, bytes, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(nullptr, e, "copy_kernel launch");
  return LB_OK;
}

const char* lb_status_string(lb_status s) {
  switch (s) {
    case LB_OK: return "LB_OK";
    case LB_EINVAL: return "LB_EINVAL: invalid argument";
    case LB_ENOMEM: return "LB_ENOMEM: device allocation failed";
    case LB_EDEVICE: return "LB_EDEVICE: HIP error or no device";
    case LB_ESTATE: return "LB_ESTATE: lattice not initialized";
    case LB_ENONFINITE: return "LB_ENONFINITE: non-finite populations";
    case LB_EAGAIN: return "LB_EAGAIN: not now, retry later";
  }
  return "unknown lb_status";
}

const char* lb_last_error(const lb_lattice* h) {
  if (h) return h->err.c_str();
  return t_err.c_str();
}

}  // extern "C"
