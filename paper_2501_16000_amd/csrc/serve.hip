// serve.hip -- continuous-batching server of many independent D2Q9 OReg
// lattices on one GPU (the lb_server_* part of include/oreg.h).
//
// Resources:
//   * a device arena (one hipMalloc of memory_budget bytes) carved by a
//     first-fit allocator: each admitted lattice holds 2 * 9 * sizeof(storage)
//     bytes per node of populations plus 24 bytes per node that first receive
//     the initial fields and at the end the result moments;
//   * a pinned host arena for field uploads and one for results;
//   * a compute stream (init, batched sweeps, gathers) and a copy stream
//     (uploads, downloads), ordered by events.
// Per step the host enqueues one batched sweep over every resident lattice.
// Lattices whose step count is reached are gathered on the compute stream and
// copied to pinned memory on the copy stream; their arena block is released
// once that copy has completed.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "oreg.h"

using namespace oreg;

namespace {

constexpr size_t kAlign = 256;

size_t round_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size) in kAlign units, with coalescing frees.
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
    used_ = 0;
  }
  bool alloc(size_t n, size_t* off) {
    n = round_up(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n;
        const size_t noff = it->first + n;
        free_.erase(it);
        if (rest) free_[noff] = rest;
        used_ += n;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = round_up(n);
    used_ -= n;
    auto it = free_.emplace(off, n).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0;
};

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

size_t storage_size(lb_storage s) { return s == LB_F64 ? 8 : s == LB_F32S ? 4 : 2; }

}  // namespace

struct ServedLattice {
  int64_t tag;
  int nx, ny;
  int64_t steps;
  double tau;
  size_t dev_off, dev_bytes;  // arena block
  size_t in_off, in_bytes;    // pinned upload block (released after the upload)
  hipEvent_t upload_done = nullptr;
  bool upload_pending = false;
  int64_t admit_T;
  int64_t done = 0;     // time steps run
  int64_t nlaunch = 0;  // batched launches taken part in (state in buf[nlaunch % 2])
  int kl = 1;           // steps of the next launch
  double t_submit;
  // retirement
  size_t out_off = 0, out_bytes = 0;  // pinned result block
  std::vector<double> heap_out;       // result when the pinned space was full
  hipEvent_t download_done = nullptr;
  double t_done = 0;
};

struct lb_server {
  lb_server_options opt{};
  int device = 0;
  hipStream_t compute = nullptr, copy = nullptr;
  char* arena_base = nullptr;
  Arena arena;
  char* pin_in = nullptr;
  Arena pin_in_arena;
  char* pin_out = nullptr;
  Arena pin_out_arena;
  Coef64 base{};                    // theta, a0, a1, rho0 of every lattice
  std::vector<ServedLattice*> active;
  std::deque<ServedLattice*> retiring;
  std::deque<ServedLattice*> ready;
  std::vector<ServedLattice*> uploading;  // pinned upload blocks to reclaim
  // descriptors
  LatticeDesc* d_desc = nullptr;
  unsigned int* d_bad = nullptr;    // init_kernel's invalid-node counter (fields are pre-checked)
  int* d_map = nullptr;
  int64_t map_capacity = 0;
  LatticeDesc* h_desc[2] = {nullptr, nullptr};  // pinned staging
  hipEvent_t desc_done[2] = {nullptr, nullptr};
  int desc_slot = 0;
  bool dirty = true;
  int64_t tiles = 0;
  int64_t T = 0;
  int64_t launches = 0, node_updates = 0;
  bool broken = false;                  // a retire failed: no further work
  std::string broken_msg;
  std::vector<ServedLattice*> orphans;  // lattices whose retire failed (freed at destroy)
  std::string err;
};

namespace {

thread_local std::string t_server_err;  // last failure without a server handle

lb_status fail(lb_server* s, lb_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (s) s->err = buf;
  else t_server_err = buf;
  return st;
}

lb_status hfail(lb_server* s, hipError_t e, const char* what) {
  return fail(s, e == hipErrorOutOfMemory ? LB_ENOMEM : LB_EDEVICE, "%s: %s (%d)", what,
              hipGetErrorString(e), (int)e);
}

#define STRY(s, call)                                  \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hfail((s), e_, #call); \
  } while (0)

struct DeviceScope {
  int prev = -1;
  bool ok = true;
  explicit DeviceScope(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = (hipSetDevice(dev) == hipSuccess);
  }
  ~DeviceScope() {
    int now = -1;
    if (prev >= 0 && hipGetDevice(&now) == hipSuccess && now != prev) (void)hipSetDevice(prev);
  }
};

size_t population_bytes(const lb_server* s, int64_t cells) {
  return round_up(2 * 9 * (size_t)cells * storage_size(s->opt.storage));
}

LatticeDesc describe(const lb_server* s, const ServedLattice* L) {
  LatticeDesc d{};
  char* base = s->arena_base + L->dev_off;
  const int64_t cells = (int64_t)L->nx * L->ny;
  const size_t half = 9 * (size_t)cells * storage_size(s->opt.storage);
  d.buf[0] = base;
  d.buf[1] = base + half;
  d.fields = reinterpret_cast<double*>(base + population_bytes(s, cells));
  d.nx = L->nx;
  d.ny = L->ny;
  d.plane = cells;
  d.admit_T = L->admit_T;
  const int W = fused_strip_width(s->opt.storage);
  d.kl = L->kl;
  // Rows per work item: the lattice's rows in equal blocks of at most 132
  // (rounded up to a multiple of 3, the strip loop's unroll).  Measured on
  // the 2000-request stream: 2 % (F32S) and 3 % (FP64) more capacity than
  // blocks of 66 rows with a ragged last one.
  const int nblk = (L->ny + 131) / 132;
  d.rows = ((L->ny + nblk - 1) / nblk + 2) / 3 * 3;
  d.strips = (L->nx + W - 1) / W;
  d.coef = s->base;
  d.coef.kappa0 = (1.0 - 1.0 / L->tau) / (2.0 * s->base.theta * s->base.theta);
  d.coef.omega = 1.0 / L->tau;
  return d;
}

// Reclaim pinned upload blocks whose copies have finished.
lb_status reclaim_uploads(lb_server* s) {
  for (size_t i = 0; i < s->uploading.size();) {
    ServedLattice* L = s->uploading[i];
    const hipError_t q = hipEventQuery(L->upload_done);
    if (q == hipSuccess) {
      s->pin_in_arena.release(L->in_off, L->in_bytes);
      L->upload_pending = false;
      s->uploading[i] = s->uploading.back();
      s->uploading.pop_back();
    } else if (q == hipErrorNotReady) {
      ++i;
    } else {
      return hfail(s, q, "hipEventQuery(upload)");
    }
  }
  return LB_OK;
}

// Move retiring lattices whose results reached host memory to `ready`, and
// give their arena blocks back.
lb_status reclaim_results(lb_server* s) {
  while (!s->retiring.empty()) {
    ServedLattice* L = s->retiring.front();
    const hipError_t q = hipEventQuery(L->download_done);
    if (q == hipErrorNotReady) break;
    if (q != hipSuccess) return hfail(s, q, "hipEventQuery(download)");
    L->t_done = now_s();
    s->arena.release(L->dev_off, L->dev_bytes);
    s->retiring.pop_front();
    s->ready.push_back(L);
  }
  return LB_OK;
}

lb_status upload_descriptors(lb_server* s) {
  const int n = (int)s->active.size();
  int64_t tiles = 0;
  const int slot = s->desc_slot;
  STRY(s, hipEventSynchronize(s->desc_done[slot]));  // staging slot free again
  for (int i = 0; i < n; ++i) {
    LatticeDesc d = describe(s, s->active[i]);
    d.tile_begin = tiles;
    tiles += (int64_t)d.strips * ((d.ny + d.rows - 1) / d.rows);
    s->h_desc[slot][i] = d;
  }
  if (tiles > s->map_capacity) {
    // grow the tile map (stream-ordered: the old map is no longer read after
    // the synchronization)
    STRY(s, hipStreamSynchronize(s->compute));
    if (s->d_map) STRY(s, hipFree(s->d_map));
    s->d_map = nullptr;
    const int64_t cap = tiles * 2;
    STRY(s, hipMalloc((void**)&s->d_map, (size_t)cap * sizeof(int)));
    s->map_capacity = cap;
  }
  if (n > 0) {
    STRY(s, hipMemcpyAsync(s->d_desc, s->h_desc[slot], (size_t)n * sizeof(LatticeDesc),
                           hipMemcpyHostToDevice, s->compute));
    STRY(s, launch_tile_map(s->d_desc, n, s->d_map, tiles, s->compute));
  }
  STRY(s, hipEventRecord(s->desc_done[slot], s->compute));
  s->desc_slot = 1 - slot;
  s->tiles = tiles;
  s->dirty = false;
  return LB_OK;
}

// Gather the moments of a finished lattice and start their download.
lb_status retire(lb_server* s, ServedLattice* L) {
  const LatticeDesc d = describe(s, L);
  const int64_t cells = d.plane;
  const Geometry g{L->nx, L->ny, cells};
  const size_t bytes = 3 * (size_t)cells * sizeof(double);
  const bool pinned = s->pin_out_arena.alloc(bytes, &L->out_off);
  L->out_bytes = bytes;
  STRY(s, launch_moments(s->opt.storage, d.buf[L->nlaunch & 1], d.fields, g, d.coef,
                         s->compute));
  hipEvent_t gathered;
  STRY(s, hipEventCreateWithFlags(&gathered, hipEventDisableTiming));
  STRY(s, hipEventRecord(gathered, s->compute));
  STRY(s, hipStreamWaitEvent(s->copy, gathered, 0));
  STRY(s, hipEventDestroy(gathered));
  if (!pinned) {
    // Unfetched results fill the pinned space: download synchronously.
    L->heap_out.resize(3 * (size_t)cells);
    STRY(s, hipMemcpyAsync(L->heap_out.data(), d.fields, bytes, hipMemcpyDeviceToHost, s->copy));
    STRY(s, hipStreamSynchronize(s->copy));
    STRY(s, hipEventCreateWithFlags(&L->download_done, hipEventDisableTiming));
    STRY(s, hipEventRecord(L->download_done, s->copy));
    s->retiring.push_back(L);
    return LB_OK;
  }
  STRY(s, hipMemcpyAsync(s->pin_out + L->out_off, d.fields, bytes, hipMemcpyDeviceToHost,
                         s->copy));
  STRY(s, hipEventCreateWithFlags(&L->download_done, hipEventDisableTiming));
  STRY(s, hipEventRecord(L->download_done, s->copy));
  s->retiring.push_back(L);
  return LB_OK;
}

void free_lattice(ServedLattice* L) {
  if (L->upload_done) (void)hipEventDestroy(L->upload_done);
  if (L->download_done) (void)hipEventDestroy(L->download_done);
  delete L;
}

}  // namespace

extern "C" {

void lb_server_options_init(lb_server_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->memory_budget = (int64_t)16 << 30;
  o->pinned_bytes = (int64_t)1 << 30;
  o->max_active = 256;
  o->equilibrium = LB_EQ_GUIDED;
  o->storage = LB_F32S;
  o->theta = 1.0 / 3.0;
  o->rho0 = 1.0;
  o->device = -1;
}

lb_status lb_server_create(const lb_server_options* o, lb_server** out) {
  if (!out) return LB_EINVAL;
  *out = nullptr;
  if (!o) return LB_EINVAL;
  // Reuse the lattice validation for the shared parameters.
  lb_options lo;
  lb_options_init(&lo);
  lo.nx = lo.ny = 1;
  lo.tau = 1.0;
  lo.theta = o->theta;
  lo.equilibrium = o->equilibrium;
  lo.storage = o->storage;
  lo.rho0 = o->rho0;
  if (o->memory_budget <= 0 || o->pinned_bytes <= 0 || o->max_active < 1 ||
      o->max_active > 65536)
    return fail(nullptr, LB_EINVAL, "need memory_budget > 0, pinned_bytes > 0, 1 <= max_active <= 65536");
  if (o->equilibrium != LB_EQ_GUIDED && o->equilibrium != LB_EQ_POLY2)
    return fail(nullptr, LB_EINVAL, "unknown equilibrium %d", (int)o->equilibrium);
  if (o->storage < LB_F64 || o->storage > LB_BF16S)
    return fail(nullptr, LB_EINVAL, "unknown storage %d", (int)o->storage);
  if (!std::isfinite(o->theta)) return fail(nullptr, LB_EINVAL, "theta must be finite");
  if (o->equilibrium == LB_EQ_GUIDED && !(o->theta > 0.0 && o->theta < 1.0))
    return fail(nullptr, LB_EINVAL, "guided equilibrium needs 0 < theta < 1 (got %g)", o->theta);
  if (o->equilibrium == LB_EQ_POLY2 && std::fabs(o->theta - 1.0 / 3.0) > 1e-12)
    return fail(nullptr, LB_EINVAL, "polynomial equilibrium needs theta = 1/3");
  if (o->storage != LB_F64 && (!std::isfinite(o->rho0) || !(o->rho0 > 0.0)))
    return fail(nullptr, LB_EINVAL, "rho0 must be finite and > 0 for shifted storage");

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return fail(nullptr, LB_EDEVICE, "no HIP device available");
  int dev = o->device;
  if (dev < 0 && hipGetDevice(&dev) != hipSuccess) dev = 0;
  if (dev >= ndev) return fail(nullptr, LB_EINVAL, "device %d out of range (%d devices)", dev, ndev);

  lb_server* s = new (std::nothrow) lb_server;
  if (!s) return LB_ENOMEM;
  s->opt = *o;
  s->opt.device = dev;
  s->device = dev;
  const double th = o->equilibrium == LB_EQ_POLY2 ? 1.0 / 3.0 : o->theta;
  s->base.theta = th;
  s->base.a0 = 1.0 - th;
  s->base.a1 = 0.5 * th;
  s->base.rho0 = o->storage == LB_F64 ? 0.0 : o->rho0;

  DeviceScope ds(dev);
  auto bail = [&](lb_status st) {
    lb_server_destroy(s);
    return st;
  };
  if (!ds.ok) return bail(LB_EDEVICE);
  if (hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking) != hipSuccess)
    return bail(LB_EDEVICE);
  if (hipMalloc((void**)&s->arena_base, (size_t)o->memory_budget) != hipSuccess)
    return bail(LB_ENOMEM);
  s->arena.reset((size_t)o->memory_budget);
  if (hipHostMalloc((void**)&s->pin_in, (size_t)o->pinned_bytes, hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc((void**)&s->pin_out, (size_t)o->pinned_bytes, hipHostMallocDefault) !=
          hipSuccess)
    return bail(LB_ENOMEM);
  s->pin_in_arena.reset((size_t)o->pinned_bytes);
  s->pin_out_arena.reset((size_t)o->pinned_bytes);
  if (hipMalloc((void**)&s->d_desc, (size_t)o->max_active * sizeof(LatticeDesc)) != hipSuccess ||
      hipMalloc((void**)&s->d_bad, sizeof(unsigned int)) != hipSuccess)
    return bail(LB_ENOMEM);
  for (int k = 0; k < 2; ++k) {
    if (hipHostMalloc((void**)&s->h_desc[k], (size_t)o->max_active * sizeof(LatticeDesc),
                      hipHostMallocDefault) != hipSuccess)
      return bail(LB_ENOMEM);
    if (hipEventCreateWithFlags(&s->desc_done[k], hipEventDisableTiming) != hipSuccess)
      return bail(LB_EDEVICE);
    if (hipEventRecord(s->desc_done[k], s->compute) != hipSuccess) return bail(LB_EDEVICE);
  }
  *out = s;
  return LB_OK;
}

lb_status lb_server_submit(lb_server* s, const lb_request* r) {
  if (!s) return LB_EINVAL;
  if (!r || !r->rho || !r->ux || !r->uy) return fail(s, LB_EINVAL, "NULL request or field");
  if (r->nx < 1 || r->ny < 1) return fail(s, LB_EINVAL, "lattice %d x %d", r->nx, r->ny);
  if (!std::isfinite(r->tau) || !(r->tau > 0.5)) return fail(s, LB_EINVAL, "tau %g", r->tau);
  if (r->steps < 1) return fail(s, LB_EINVAL, "steps %lld", (long long)r->steps);
  const int64_t cells = (int64_t)r->nx * r->ny;
  const size_t dev_bytes = population_bytes(s, cells) + round_up(3 * (size_t)cells * 8);
  const size_t in_bytes = 3 * (size_t)cells * sizeof(double);
  if (dev_bytes > (size_t)s->opt.memory_budget || in_bytes > (size_t)s->opt.pinned_bytes)
    return fail(s, LB_EINVAL, "lattice %d x %d does not fit the server's memory", r->nx, r->ny);
  for (int64_t i = 0; i < cells; ++i)
    if (!std::isfinite(r->rho[i]) || !std::isfinite(r->ux[i]) || !std::isfinite(r->uy[i]) ||
        !(r->rho[i] > 0.0))
      return fail(s, LB_EINVAL, "node %lld has a non-finite field or rho <= 0", (long long)i);

  if (s->broken) return fail(s, LB_EDEVICE, "server failed earlier: %s", s->broken_msg.c_str());
  DeviceScope ds(s->device);
  if (!ds.ok) return fail(s, LB_EDEVICE, "cannot select device %d", s->device);
  lb_status st = reclaim_uploads(s);
  if (st != LB_OK) return st;
  st = reclaim_results(s);
  if (st != LB_OK) return st;
  if ((int)s->active.size() >= s->opt.max_active)
    return fail(s, LB_EAGAIN, "all %d slots are busy", s->opt.max_active);
  size_t dev_off, in_off;
  if (!s->arena.alloc(dev_bytes, &dev_off)) return fail(s, LB_EAGAIN, "device arena full");
  if (!s->pin_in_arena.alloc(in_bytes, &in_off)) {
    s->arena.release(dev_off, dev_bytes);
    return fail(s, LB_EAGAIN, "pinned upload space full");
  }
  ServedLattice* L = new (std::nothrow) ServedLattice;
  if (!L) {
    s->arena.release(dev_off, dev_bytes);
    s->pin_in_arena.release(in_off, in_bytes);
    return fail(s, LB_ENOMEM, "host allocation failed");
  }
  L->tag = r->tag;
  L->nx = r->nx;
  L->ny = r->ny;
  L->steps = r->steps;
  L->tau = r->tau;
  L->dev_off = dev_off;
  L->dev_bytes = dev_bytes;
  L->in_off = in_off;
  L->in_bytes = in_bytes;
  L->admit_T = s->T;
  L->t_submit = now_s();

  // Fields -> pinned -> device (copy stream) -> f^eq into buffer A (compute stream).
  double* pin = reinterpret_cast<double*>(s->pin_in + in_off);
  std::memcpy(pin, r->rho, (size_t)cells * sizeof(double));
  std::memcpy(pin + cells, r->ux, (size_t)cells * sizeof(double));
  std::memcpy(pin + 2 * cells, r->uy, (size_t)cells * sizeof(double));
  const LatticeDesc d = describe(s, L);
  // Error exits give back everything the request holds (after the streams
  // have let go of the pinned upload block and the arena block).
  auto undo = [&](lb_status e) {
    (void)hipStreamSynchronize(s->copy);
    (void)hipStreamSynchronize(s->compute);
    s->arena.release(dev_off, dev_bytes);
    s->pin_in_arena.release(in_off, in_bytes);
    free_lattice(L);
    return e;
  };
  hipError_t e = hipMemcpyAsync(d.fields, pin, in_bytes, hipMemcpyHostToDevice, s->copy);
  if (e != hipSuccess) return undo(hfail(s, e, "hipMemcpyAsync(fields)"));
  if ((e = hipEventCreateWithFlags(&L->upload_done, hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventRecord(L->upload_done, s->copy)) != hipSuccess ||
      (e = hipStreamWaitEvent(s->compute, L->upload_done, 0)) != hipSuccess)
    return undo(hfail(s, e, "upload event"));
  const Geometry g{L->nx, L->ny, cells};
  // The fields were validated above, so init_kernel's invalid-node counter
  // is never incremented and not read back.
  e = launch_init(s->opt.equilibrium, s->opt.storage, d.fields, d.fields + cells,
                  d.fields + 2 * cells, d.buf[0], g, d.coef, s->d_bad, s->compute);
  if (e != hipSuccess) return undo(hfail(s, e, "launch_init"));
  L->upload_pending = true;
  s->uploading.push_back(L);
  s->active.push_back(L);
  s->dirty = true;
  return LB_OK;
}

lb_status lb_server_step(lb_server* s, int64_t n) {
  if (!s) return LB_EINVAL;
  if (n < 0) return fail(s, LB_EINVAL, "n %lld", (long long)n);
  DeviceScope ds(s->device);
  if (!ds.ok) return fail(s, LB_EDEVICE, "cannot select device %d", s->device);
  if (s->broken) return fail(s, LB_EDEVICE, "server failed earlier: %s", s->broken_msg.c_str());
  const int K = fused_levels(s->opt.storage);
  for (int64_t k = 0; k < n && !s->active.empty(); ++k) {
    // a lattice's last launch may advance it fewer than K steps (at least 1:
    // a lattice is retired as soon as it has run its steps)
    for (ServedLattice* L : s->active) {
      const int want = (int)std::max<int64_t>(1, std::min<int64_t>(K, L->steps - L->done));
      if (want != L->kl) {
        L->kl = want;
        s->dirty = true;
      }
    }
    if (s->dirty) {
      lb_status st = upload_descriptors(s);
      if (st != LB_OK) return st;
    }
    STRY(s, launch_batched_fused(s->opt.equilibrium, s->opt.storage, s->d_desc, s->d_map,
                                 s->tiles, s->T, s->compute));
    s->T += 1;
    s->launches += 1;
    // retire lattices that have run their steps
    for (size_t i = 0; i < s->active.size();) {
      ServedLattice* L = s->active[i];
      L->done += L->kl;
      L->nlaunch += 1;
      s->node_updates += (int64_t)L->nx * L->ny * L->kl;
      if (L->done >= L->steps) {
        // Out of the active set whatever retire() returns, so that no later
        // launch advances it again.  A failed retire leaves its gather or
        // download half enqueued: the server refuses further work (its
        // memory may still be in use by the device) and reports the error.
        s->active.erase(s->active.begin() + (long)i);
        s->dirty = true;
        lb_status st = retire(s, L);
        if (st != LB_OK) {
          s->broken = true;
          s->broken_msg = s->err;
          s->orphans.push_back(L);
          return st;
        }
      } else {
        ++i;
      }
    }
  }
  lb_status st = reclaim_uploads(s);
  if (st != LB_OK) return st;
  return reclaim_results(s);
}

lb_status lb_server_poll(lb_server* s, lb_result* out) {
  if (!s || !out) return LB_EINVAL;
  DeviceScope ds(s->device);
  lb_status st = reclaim_results(s);
  if (st != LB_OK) return st;
  if (s->ready.empty()) return LB_EAGAIN;
  const ServedLattice* L = s->ready.front();
  out->tag = L->tag;
  out->nx = L->nx;
  out->ny = L->ny;
  out->steps = L->steps;
  out->t_submit = L->t_submit;
  out->t_done = L->t_done;
  return LB_OK;
}

lb_status lb_server_fetch(lb_server* s, int64_t tag, double* out) {
  if (!s || !out) return LB_EINVAL;
  for (auto it = s->ready.begin(); it != s->ready.end(); ++it) {
    ServedLattice* L = *it;
    if (L->tag != tag) continue;
    if (!L->heap_out.empty()) {
      std::memcpy(out, L->heap_out.data(), L->out_bytes);
    } else {
      std::memcpy(out, s->pin_out + L->out_off, L->out_bytes);
      s->pin_out_arena.release(L->out_off, L->out_bytes);
    }
    s->ready.erase(it);
    if (L->upload_pending) {
      // still referenced by the upload list; it is reclaimed there
      for (auto& u : s->uploading)
        if (u == L) {
          DeviceScope ds(s->device);
          (void)hipEventSynchronize(L->upload_done);
          s->pin_in_arena.release(L->in_off, L->in_bytes);
          u = s->uploading.back();
          s->uploading.pop_back();
          break;
        }
    }
    free_lattice(L);
    return LB_OK;
  }
  return fail(s, LB_EINVAL, "no ready result with tag %lld", (long long)tag);
}

lb_status lb_server_stats_get(lb_server* s, lb_server_stats* out) {
  if (!s || !out) return LB_EINVAL;
  DeviceScope ds(s->device);
  lb_status st = reclaim_results(s);
  if (st != LB_OK) return st;
  out->active = (int)s->active.size();
  out->retiring = (int)s->retiring.size();
  out->ready = (int)s->ready.size();
  out->device_bytes_used = (int64_t)s->arena.used();
  out->launches = s->launches;
  out->node_updates = s->node_updates;
  out->clock = now_s();
  return LB_OK;
}

lb_status lb_server_sync(lb_server* s) {
  if (!s) return LB_EINVAL;
  DeviceScope ds(s->device);
  STRY(s, hipStreamSynchronize(s->compute));
  STRY(s, hipStreamSynchronize(s->copy));
  lb_status st = reclaim_uploads(s);
  if (st != LB_OK) return st;
  return reclaim_results(s);
}

lb_status lb_server_destroy(lb_server* s) {
  if (!s) return LB_OK;
  {
    DeviceScope ds(s->device);
    if (s->compute) (void)hipStreamSynchronize(s->compute);
    if (s->copy) (void)hipStreamSynchronize(s->copy);
    for (ServedLattice* L : s->active) free_lattice(L);
    for (ServedLattice* L : s->retiring) free_lattice(L);
    for (ServedLattice* L : s->ready) free_lattice(L);
    for (ServedLattice* L : s->orphans) free_lattice(L);
    if (s->d_map) (void)hipFree(s->d_map);
    if (s->d_desc) (void)hipFree(s->d_desc);
    if (s->d_bad) (void)hipFree(s->d_bad);
    for (int k = 0; k < 2; ++k) {
      if (s->h_desc[k]) (void)hipHostFree(s->h_desc[k]);
      if (s->desc_done[k]) (void)hipEventDestroy(s->desc_done[k]);
    }
    if (s->arena_base) (void)hipFree(s->arena_base);
    if (s->pin_in) (void)hipHostFree(s->pin_in);
    if (s->pin_out) (void)hipHostFree(s->pin_out);
    if (s->compute) (void)hipStreamDestroy(s->compute);
    if (s->copy) (void)hipStreamDestroy(s->copy);
  }
  delete s;
  return LB_OK;
}

const char* lb_server_last_error(const lb_server* s) {
  return s ? s->err.c_str() : t_server_err.c_str();
}

}  // extern "C"
