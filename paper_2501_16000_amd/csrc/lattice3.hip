// lattice3.hip -- the C ABI of include/oreg3.h: D3Q27 lattice handles,
// validation, device buffers, stream ordering and error reporting.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "kernels3.hpp"
#include "oreg3.h"

using namespace oreg;

struct lb3_lattice {
  lb3_options opt{};
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  void* buf[2] = {nullptr, nullptr};  // A/B population buffers
  int cur = 0;
  size_t elem = 8;
  Geometry3 geo{};
  Coef64 coef{};
  bool initialized = false;
  int64_t t = 0;
  double* tmp = nullptr;              // 4 * cells FP64 staging (lazy)
  double* aux = nullptr;              // kDiag3Blocks * 7 partials + 8 results
  unsigned int* counter = nullptr;
  std::string err;
};

namespace {

thread_local std::string t_err3;

lb_status fail(lb3_lattice* h, lb_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (h) h->err = buf;
  t_err3 = buf;
  return st;
}

lb_status hip_fail(lb3_lattice* h, hipError_t e, const char* what) {
  const lb_status st = (e == hipErrorOutOfMemory) ? LB_ENOMEM : LB_EDEVICE;
  return fail(h, st, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

#define HIP_TRY(h, call)                                   \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return hip_fail((h), e_, #call); \
  } while (0)

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

lb_status validate(const lb3_options* o) {
  if (!o) return fail(nullptr, LB_EINVAL, "options pointer is NULL");
  if (o->nx < 1 || o->ny < 1 || o->nz < 1)
    return fail(nullptr, LB_EINVAL, "nx, ny and nz must be >= 1 (got %d x %d x %d)", o->nx, o->ny,
                o->nz);
  if (o->equilibrium != LB_EQ_GUIDED && o->equilibrium != LB_EQ_POLY2)
    return fail(nullptr, LB_EINVAL, "unknown equilibrium %d", (int)o->equilibrium);
  if (o->storage < LB_F64 || o->storage > LB_BF16S)
    return fail(nullptr, LB_EINVAL, "unknown storage %d", (int)o->storage);
  if (o->collision != LB_COLL_OREG && o->collision != LB_COLL_BGK)
    return fail(nullptr, LB_EINVAL, "unknown collision %d", (int)o->collision);
  // The sweep launches one wavefront per 64-node row segment (a 32-bit task
  // count); the per-node kernels launch cells / 256 workgroups.
  const double tasks = std::ceil(o->nx / 64.0) * (double)o->ny * (double)o->nz;
  const double cells = (double)o->nx * (double)o->ny * (double)o->nz;
  if (tasks > 4294967040.0 || cells > 4294967040.0 * 64.0)
    return fail(nullptr, LB_EINVAL, "box %d x %d x %d is too large for one launch", o->nx, o->ny,
                o->nz);
  if (!is_finite(o->tau) || !(o->tau > 0.5))
    return fail(nullptr, LB_EINVAL, "tau must be finite and > 1/2 (got %g)", o->tau);
  if (!is_finite(o->theta)) return fail(nullptr, LB_EINVAL, "theta must be finite");
  if (o->equilibrium == LB_EQ_GUIDED && !(o->theta > 0.0 && o->theta < 1.0))
    return fail(nullptr, LB_EINVAL, "guided equilibrium needs 0 < theta < 1 (got %g)", o->theta);
  if (o->equilibrium == LB_EQ_POLY2 && std::fabs(o->theta - 1.0 / 3.0) > 1e-12)
    return fail(nullptr, LB_EINVAL, "polynomial equilibrium needs theta = 1/3 (got %.17g)", o->theta);
  if (o->storage != LB_F64 && (!is_finite(o->rho0) || !(o->rho0 > 0.0)))
    return fail(nullptr, LB_EINVAL, "rho0 must be finite and > 0 for shifted storage");
  return LB_OK;
}

Coef64 make_coef(const lb3_options& o) {
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

lb_status ensure_tmp(lb3_lattice* h) {
  if (h->tmp) return LB_OK;
  HIP_TRY(h, hipMalloc((void**)&h->tmp, 4 * (size_t)h->geo.cells * sizeof(double)));
  return LB_OK;
}

lb_status ready(lb3_lattice* h, const void* ptr, bool need_init) {
  if (!h) return fail(nullptr, LB_EINVAL, "lattice handle is NULL");
  if (!ptr) return fail(h, LB_EINVAL, "array pointer is NULL");
  if (need_init && !h->initialized) return fail(h, LB_ESTATE, "lattice is not initialized");
  return LB_OK;
}

lb_status finish_init(lb3_lattice* h) {
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

void lb3_options_init(lb3_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->tau = 1.0;
  o->theta = 1.0 / 3.0;
  o->equilibrium = LB_EQ_GUIDED;
  o->storage = LB_F64;
  o->collision = LB_COLL_OREG;
  o->rho0 = 1.0;
  o->stream = nullptr;
  o->use_stream = 0;
  o->device = -1;
}

lb_status lb3_create(const lb3_options* opt, lb3_lattice** out) {
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
  if (dev < 0 && hipGetDevice(&dev) != hipSuccess) dev = 0;
  if (dev >= ndev) return fail(nullptr, LB_EINVAL, "device %d out of range (%d devices)", dev, ndev);

  lb3_lattice* h = new (std::nothrow) lb3_lattice;
  if (!h) return fail(nullptr, LB_ENOMEM, "host allocation failed");
  h->opt = *opt;
  h->opt.device = dev;
  h->device = dev;
  h->elem = storage_bytes(opt->storage);
  h->geo.nx = opt->nx;
  h->geo.ny = opt->ny;
  h->geo.nz = opt->nz;
  h->geo.cells = (int64_t)opt->nx * opt->ny * opt->nz;
  h->coef = make_coef(*opt);

  DeviceScope ds(dev);
  if (!ds.ok) {
    delete h;
    return fail(nullptr, LB_EDEVICE, "cannot select device %d", dev);
  }
  auto cleanup = [&](lb_status s) {
    lb3_destroy(h);
    return s;
  };
  if (opt->use_stream) {
    h->stream = static_cast<hipStream_t>(opt->stream);
  } else {
    e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return cleanup(hip_fail(nullptr, e, "hipStreamCreateWithFlags"));
    h->own_stream = true;
  }
  const size_t bytes = 27 * (size_t)h->geo.cells * h->elem;
  for (int b = 0; b < 2; ++b) {
    e = hipMalloc(&h->buf[b], bytes);
    if (e != hipSuccess) return cleanup(hip_fail(nullptr, e, "hipMalloc(populations)"));
  }
  e = hipMalloc((void**)&h->aux, (kDiag3Blocks * 7 + 8) * sizeof(double));
  if (e != hipSuccess) return cleanup(hip_fail(nullptr, e, "hipMalloc(aux)"));
  e = hipMalloc((void**)&h->counter, sizeof(unsigned int));
  if (e != hipSuccess) return cleanup(hip_fail(nullptr, e, "hipMalloc(counter)"));
  *out = h;
  return LB_OK;
}

lb_status lb3_init(lb3_lattice* h, const double* rho, const double* ux, const double* uy,
                   const double* uz) {
  lb_status st = ready(h, (rho && ux && uy && uz) ? rho : nullptr, false);
  if (st != LB_OK) return st;
  const int64_t n = h->geo.cells;
  for (int64_t i = 0; i < n; ++i) {
    if (!is_finite(rho[i]) || !is_finite(ux[i]) || !is_finite(uy[i]) || !is_finite(uz[i]) ||
        !(rho[i] > 0.0))
      return fail(h, LB_EINVAL, "node %lld has a non-finite field or rho <= 0", (long long)i);
  }
  DeviceScope ds(h->device);
  if (!ds.ok) return fail(h, LB_EDEVICE, "cannot select device %d", h->device);
  if ((st = ensure_tmp(h)) != LB_OK) return st;
  const size_t bytes = (size_t)n * sizeof(double);
  const double* src[4] = {rho, ux, uy, uz};
  for (int a = 0; a < 4; ++a)
    HIP_TRY(h, hipMemcpyAsync(h->tmp + a * n, src[a], bytes, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(h, hipMemsetAsync(h->counter, 0, sizeof(unsigned int), h->stream));
  HIP_TRY(h, launch_init3(h->opt.equilibrium, h->opt.storage, h->tmp, h->tmp + n, h->tmp + 2 * n,
                          h->tmp + 3 * n, h->buf[h->cur], h->geo, h->coef, h->counter, h->stream));
  return finish_init(h);
}

lb_status lb3_init_device(lb3_lattice* h, const double* rho, const double* ux, const double* uy,
                          const double* uz) {
  lb_status st = ready(h, (rho && ux && uy && uz) ? rho : nullptr, false);
  if (st != LB_OK) return st;
  DeviceScope ds(h->device);
  if (!ds.ok) return fail(h, LB_EDEVICE, "cannot select device %d", h->device);
  HIP_TRY(h, hipMemsetAsync(h->counter, 0, sizeof(unsigned int), h->stream));
  HIP_TRY(h, launch_init3(h->opt.equilibrium, h->opt.storage, rho, ux, uy, uz, h->buf[h->cur],
                          h->geo, h->coef, h->counter, h->stream));
  return finish_init(h);
}

lb_status lb3_step(lb3_lattice* h, int64_t n) {
  if (!h) return fail(nullptr, LB_EINVAL, "lattice handle is NULL");
  if (n < 0) return fail(h, LB_EINVAL, "n must be >= 0 (got %lld)", (long long)n);
  if (!h->initialized) return fail(h, LB_ESTATE, "lattice is not initialized");
  if (n == 0) return LB_OK;
  DeviceScope ds(h->device);
  if (!ds.ok) return fail(h, LB_EDEVICE, "cannot select device %d", h->device);
  for (int64_t s = 0; s < n; ++s) {
    HIP_TRY(h, launch_sweep3(h->opt.equilibrium, h->opt.collision, h->opt.storage, h->buf[h->cur],
                             h->buf[1 - h->cur], h->geo, h->coef, h->stream));
    h->cur = 1 - h->cur;
    h->t += 1;
  }
  return LB_OK;
}

lb_status lb3_moments_device(lb3_lattice* h, double* out_dev) {
  lb_status st = ready(h, out_dev, true);
  if (st != LB_OK) return st;
  DeviceScope ds(h->device);
  if (!ds.ok) return fail(h, LB_EDEVICE, "cannot select device %d", h->device);
  HIP_TRY(h, launch_moments3(h->opt.storage, h->buf[h->cur], out_dev, h->geo, h->coef, h->stream));
  return LB_OK;
}

lb_status lb3_moments(lb3_lattice* h, double* out) {
  lb_status st = ready(h, out, true);
  if (st != LB_OK) return st;
  DeviceScope ds(h->device);
  if (!ds.ok) return fail(h, LB_EDEVICE, "cannot select device %d", h->device);
  if ((st = ensure_tmp(h)) != LB_OK) return st;
  HIP_TRY(h, launch_moments3(h->opt.storage, h->buf[h->cur], h->tmp, h->geo, h->coef, h->stream));
  HIP_TRY(h, hipMemcpyAsync(out, h->tmp, 4 * (size_t)h->geo.cells * sizeof(double),
                            hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return LB_OK;
}

lb_status lb3_populations(lb3_lattice* h, double* out) {
  lb_status st = ready(h, out, true);
  if (st != LB_OK) return st;
  DeviceScope ds(h->device);
  if (!ds.ok) return fail(h, LB_EDEVICE, "cannot select device %d", h->device);
  if ((st = ensure_tmp(h)) != LB_OK) return st;
  const int64_t n = h->geo.cells;
  for (int i = 0; i < 27; ++i) {
    // Four staging planes, used in turn, so a plane is not overwritten
    // before its copy has been issued (same stream, so ordered).
    double* stage = h->tmp + (i % 4) * n;
    HIP_TRY(h, launch_export3(h->opt.storage, i, h->buf[h->cur], stage, h->geo, h->coef, h->stream));
    HIP_TRY(h, hipMemcpyAsync(out + (size_t)i * n, stage, (size_t)n * sizeof(double),
                              hipMemcpyDeviceToHost, h->stream));
  }
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return LB_OK;
}

lb_status lb3_set_populations(lb3_lattice* h, const double* in) {
  lb_status st = ready(h, in, false);
  if (st != LB_OK) return st;
  const int64_t n = h->geo.cells;
  for (int64_t c = 0; c < n; ++c) {
    double rho = 0.0;
    for (int i = 0; i < 27; ++i) {
      const double v = in[(size_t)i * n + c];
      if (!is_finite(v))
        return fail(h, LB_EINVAL, "population %d of node %lld is not finite", i, (long long)c);
      rho += v;
    }
    if (!(rho > 0.0)) return fail(h, LB_EINVAL, "node %lld has sum_i f_i <= 0", (long long)c);
  }
  DeviceScope ds(h->device);
  if (!ds.ok) return fail(h, LB_EDEVICE, "cannot select device %d", h->device);
  if ((st = ensure_tmp(h)) != LB_OK) return st;
  for (int i = 0; i < 27; ++i) {
    double* stage = h->tmp + (i % 4) * n;
    HIP_TRY(h, hipMemcpyAsync(stage, in + (size_t)i * n, (size_t)n * sizeof(double),
                              hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, launch_import3(h->opt.storage, i, stage, h->buf[h->cur], h->geo, h->coef, h->stream));
  }
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  h->initialized = true;
  h->t = 0;
  return LB_OK;
}

lb_status lb3_diagnostics(lb3_lattice* h, double out[7]) {
  lb_status st = ready(h, out, true);
  if (st != LB_OK) return st;
  DeviceScope ds(h->device);
  if (!ds.ok) return fail(h, LB_EDEVICE, "cannot select device %d", h->device);
  double* result = h->aux + kDiag3Blocks * 7;
  HIP_TRY(h, launch_diagnostics3(h->opt.storage, h->buf[h->cur], h->aux, result, h->geo, h->coef,
                                 h->coef.theta, h->stream));
  HIP_TRY(h, hipMemcpyAsync(out, result, 7 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return LB_OK;
}

lb_status lb3_sync(lb3_lattice* h) {
  if (!h) return fail(nullptr, LB_EINVAL, "lattice handle is NULL");
  DeviceScope ds(h->device);
  if (!ds.ok) return fail(h, LB_EDEVICE, "cannot select device %d", h->device);
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return LB_OK;
}

int64_t lb3_time(const lb3_lattice* h) { return h ? h->t : -1; }

int64_t lb3_device_bytes(const lb3_lattice* h) {
  if (!h) return 0;
  int64_t b = 2 * 27 * h->geo.cells * (int64_t)h->elem;
  b += (kDiag3Blocks * 7 + 8) * (int64_t)sizeof(double) + (int64_t)sizeof(unsigned int);
  if (h->tmp) b += 4 * h->geo.cells * (int64_t)sizeof(double);
  return b;
}

lb_status lb3_destroy(lb3_lattice* h) {
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

const char* lb3_last_error(const lb3_lattice* h) {
  if (h) return h->err.c_str();
  return t_err3.c_str();
}

}  // extern "C"
