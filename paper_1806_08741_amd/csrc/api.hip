// api.hip -- the C ABI of libsslic.so (include/sslic.h, include/sslic_steps.h):
// argument checks, the context's device workspace and the order of launches.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/sslic_profile.h"
#include "../../include/sslic_steps.h"
#include "literal.h"
#include "sslic_ctx.h"

using namespace sslic;

namespace {
thread_local std::string g_err;
}  // namespace

namespace sslic {

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int64_t grid_count(int64_t n, int64_t s) {
  int64_t k = (2 * n + s) / (2 * s);
  return k < 1 ? 1 : k;
}

// Geometry of a request; checks every validity rule of sslic.h.
int make_geo(Geo* g, int ndim, const int64_t* dims, int channels, int dtype, const int32_t* S,
             double m, int64_t K_override) {
  if (ndim < 1 || ndim > kMaxDim) return fail(SSLIC_EINVAL, "ndim %d outside [1, 4]", ndim);
  if (!dims || !S) return fail(SSLIC_EINVAL, "dims and S must be given");
  if (channels < 1 || channels > kMaxChan)
    return fail(SSLIC_EINVAL, "channels %d outside [1, 8]", channels);
  if (dtype != kU8 && dtype != kU16 && dtype != kF32) return fail(SSLIC_EINVAL, "unknown dtype %d", dtype);
  if (!(m > 0.0) || !std::isfinite(m)) return fail(SSLIC_EINVAL, "m must be positive and finite");
  memset(g, 0, sizeof *g);
  g->nd_out = ndim;
  g->nd = ndim < 2 ? 2 : ndim;
  g->C = channels;
  g->dtype = dtype;
  int64_t N = 1, K = 1, nbins = 1, prodS = 1;
  for (int i = 0; i < kMaxDim; ++i) {
    int64_t n = i < ndim ? dims[i] : 1;
    int64_t s = i < ndim ? S[i] : 1;
    if (n < 1) return fail(SSLIC_EINVAL, "dims[%d] = %lld < 1", i, (long long)n);
    if (s < 1) return fail(SSLIC_EINVAL, "S[%d] = %lld < 1", i, (long long)s);
    if (s > (1LL << 30)) return fail(SSLIC_EINVAL, "S[%d] = %lld is above 2^30", i, (long long)s);
    if (n > ((1LL << 40) - 1) / N) return fail(SSLIC_EINVAL, "image has 2^40 voxels or more");
    N *= n;
  }
  // Valid up to 2^40 voxels; the kernels index voxels, clusters and new labels
  // in 32 bits, so larger images are refused as unsupported.
  if (N >= (1LL << 31))
    return fail(SSLIC_EUNSUPPORTED, "images of 2^31 voxels or more are not supported (%lld voxels)",
                (long long)N);
  N = 1;
  for (int i = 0; i < kMaxDim; ++i) {
    int64_t n = i < ndim ? dims[i] : 1;
    int64_t s = i < ndim ? S[i] : 1;
    g->n[i] = (int)n;
    g->st[i] = N;
    N *= n;
    g->S[i] = (int)s;
    g->Ka[i] = (int)grid_count(n, s);
    K *= g->Ka[i];
    g->nb[i] = (int)((n + s - 1) / s);
    g->bst[i] = nbins;
    nbins *= g->nb[i];
    prodS *= s;
    g->wd[i] = (m * m) / ((double)s * (double)s);
    g->swd[i] = m / (double)s;
    g->sw[i] = (float)g->swd[i];
  }
  g->N = N;
  g->K = K_override > 0 ? K_override : K;
  if (g->K + N >= (1LL << 31))
    return fail(SSLIC_EUNSUPPORTED, "K + N must stay below 2^31 (labels K, K+1, ... are int32)");
  g->nbins = nbins;
  g->prodS = prodS;
  g->rs = rec_words(channels, g->nd);
  g->F = 1 + g->nd + channels;
  g->row = channels + ndim;
  return SSLIC_OK;
}

size_t al(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

Layout layout(const Geo& g, int iterations, bool cc, bool part, bool persist) {
  Layout L{};
  size_t o = 0;
  auto put = [&](size_t bytes) {
    size_t at = o;
    o += al(bytes);
    return at;
  };
  L.ctab = put((size_t)g.K * g.rs * 4);
  L.bin_of = put((size_t)g.K * 4);
  L.bin_cnt = put((size_t)g.nbins * 4);
  L.bin_start = put((size_t)(g.nbins + 1) * 4);
  L.bin_items = put((size_t)g.K * 4);
  L.scan_part = put((size_t)(g.nbins / 4096 + 2) * 4);
  L.acc = put((size_t)g.K * g.F * 8);
  L.accf = put((size_t)(g.K + 3) / 4 * 4);
  L.part = put(part ? (size_t)g.K * ((size_t)1 << g.nd) * (g.F + 1) * 8 : 0);
  L.res_acc = put((size_t)2 * kResSlots * (iterations > 0 ? iterations : 1) * 8);
  L.flags = put(64);
  if (cc) {
    L.cc_parent = put((size_t)g.N * 4);
    L.cc_size = put((size_t)g.N * 4);
    L.cc_newlab = put((size_t)g.N * 4);
    L.cc_part = put((size_t)cc_part_ints(g.N) * 4);
    L.cc_roots = put((size_t)g.N * 4);
    L.cc_xface = put((size_t)cc_xface_ints(g) * 4);
  }
  L.dist = put(persist ? (size_t)g.N * 4 : 0);
  L.total = o;
  return L;
}

int ensure_ws(sslic_ctx* ctx, size_t need) {
  if (need <= ctx->ws_size) return SSLIC_OK;
  if (ctx->ws) {
    // earlier work on any stream may still use the old workspace
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_size = 0;
  }
  size_t sz = need + (need >> 3);
  if (hipMalloc((void**)&ctx->ws, sz) != hipSuccess) {
    (void)hipGetLastError();
    ctx->ws = nullptr;
    return fail(SSLIC_ENOMEM, "cannot allocate %zu bytes of device workspace", sz);
  }
  ctx->ws_size = sz;
  return SSLIC_OK;
}

Iter iter_view(char* b, const Layout& L) {
  Iter it;
  it.ctab = (float*)(b + L.ctab);
  it.bin_of = (int32_t*)(b + L.bin_of);
  it.bin_cnt = (int32_t*)(b + L.bin_cnt);
  it.bin_start = (int32_t*)(b + L.bin_start);
  it.bin_items = (int32_t*)(b + L.bin_items);
  it.scan_part = (int32_t*)(b + L.scan_part);
  it.acc = (uint64_t*)(b + L.acc);
  it.accf = (uint8_t*)(b + L.accf);
  it.part = (uint64_t*)(b + L.part);
  it.res_acc = (double*)(b + L.res_acc);
  it.done = (int32_t*)(b + L.flags);
  it.iters = it.done + 1;
  return it;
}

CCBuf cc_view(char* b, const Layout& L, int64_t N) {
  CCBuf c;
  c.parent = (int32_t*)(b + L.cc_parent);
  c.size = (int32_t*)(b + L.cc_size);
  c.newlab = (int32_t*)(b + L.cc_newlab);
  cc_carve(c, (int32_t*)(b + L.cc_part), N);
  c.roots = (int32_t*)(b + L.cc_roots);
  c.xface = (int32_t*)(b + L.cc_xface);
  c.total = (int32_t*)(b + L.flags) + 2;  // flags: done, iters, total, n_labels
  return c;
}

int32_t* nlab_slot(char* base, const Layout& L) { return (int32_t*)(base + L.flags) + 3; }

int select_device(sslic_ctx* ctx) {
  HIP_TRY(hipSetDevice(ctx->device));
  return SSLIC_OK;
}

hipEvent_t next_event(sslic_ctx* ctx) {
  if (ctx->ev_used == ctx->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ctx->ev_pool.push_back(e);
  }
  return ctx->ev_pool[ctx->ev_used++];
}

Mark::Mark(sslic_ctx* c, const char* n, hipStream_t st) : ctx(c), name(n), s(st) {
  if (ctx && ctx->prof && (a = next_event(ctx))) (void)hipEventRecord(a, s);
}

Mark::~Mark() {
  if (!a) return;
  hipEvent_t b = next_event(ctx);
  if (!b) return;
  (void)hipEventRecord(b, s);
  ctx->marks[name].emplace_back(a, b);
}

// Copy device int32 scalars to host outputs (waits for the stream).
int read_ints(sslic_ctx* ctx, hipStream_t s, const int32_t* dev_a, int32_t* out_a,
              const int32_t* dev_b, int32_t* out_b) {
  if (!out_a && !out_b) return SSLIC_OK;
  if (out_a) HIP_TRY(hipMemcpyAsync(ctx->host_ints, dev_a, 4, hipMemcpyDeviceToHost, s));
  if (out_b) HIP_TRY(hipMemcpyAsync(ctx->host_ints + 1, dev_b, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (out_a) *out_a = ctx->host_ints[0];
  if (out_b) *out_b = ctx->host_ints[1];
  return SSLIC_OK;
}

// The iteration loop of one image on the context workspace.  Centres are in
// `cen` (seeded or given) when called.  With `dist` the loop keeps that
// distance image across iterations (set to +inf once, here): each iteration
// is then the persistent assignment step followed by the stand-alone update
// (map step by atomics into acc, then the reduce step); otherwise the sweep
// assigns and maps in one pass on a distance reset every iteration.
int run_iterations(sslic_ctx* ctx, const Geo& g, const Iter& it, const void* image, int iterations,
                   double tol, int32_t* labels, double* cen, int64_t* counts, double* residuals,
                   float* dist, hipStream_t s) {
  const int slots = dist ? 0 : sweep_slots(g);
  HIP_TRY(launch_fill_i32(it.bin_cnt, 0, g.nbins, s));
  HIP_TRY(launch_fill_u64(it.acc, 0, g.K * g.F, s));
  HIP_TRY(launch_fill_i32((int32_t*)it.accf, 0, (g.K + 3) / 4, s));
  if (slots) HIP_TRY(launch_fill_u64(it.part, 0, g.K * ((int64_t)1 << g.nd) * (g.F + 1), s));
  HIP_TRY(launch_fill_f64(it.res_acc, 0.0, 2 * kResSlots * iterations, s));
  HIP_TRY(launch_fill_i32(it.done, 0, 2, s));
  if (residuals) HIP_TRY(launch_fill_f64(residuals, 0.0, iterations, s));
  HIP_TRY(launch_prep(g, cen, it, s));
  // +inf; the first assignment writes the grid cell where no window reaches
  if (dist) HIP_TRY(launch_fill_i32(reinterpret_cast<int32_t*>(dist), 0x7f800000, g.N, s));
  for (int t = 0; t < iterations; ++t) {
    {
      Mark mk(ctx, "bins", s);
      HIP_TRY(launch_bins(g, it, s));
    }
    if (dist) {
      {
        Mark mk(ctx, "assign_persist", s);
        HIP_TRY(launch_assign_persist(g, image, it, labels, dist, t == 0, s));
      }
      Mark mk(ctx, "update", s);
      HIP_TRY(launch_update(g, image, labels, it, s));
    } else {
      Mark mk(ctx, "sweep", s);
      HIP_TRY(launch_sweep(g, image, it, labels, t, 1, s));
    }
    {
      Mark mk(ctx, "finalize", s);
      HIP_TRY(launch_finalize(g, cen, counts, it, t, t + 1 < iterations, slots, s));
      HIP_TRY(launch_residual_finish(it, t, tol, residuals, s));
    }
  }
  return SSLIC_OK;
}

// The whole filter on a workspace laid out by `L` at device address `ws`:
// seeding (or the given centres), the iteration loop, then connectivity.  The
// label count and the iterations run stay on the device (flags of `ws`), and
// go to opt's device outputs when given.  `ctx` only brackets launches for
// the profiler and may be null.
int run_on(sslic_ctx* ctx, char* ws, const Layout& L, const Geo& g, const void* image,
           int iterations, const sslic_options& o, int32_t* labels, double* centres,
           int64_t* counts, hipStream_t s) {
  Iter it = iter_view(ws, L);
  if (o.init_centres) {
    if (o.init_centres != centres)
      HIP_TRY(hipMemcpyAsync(centres, o.init_centres, (size_t)g.K * g.row * 8,
                             hipMemcpyDeviceToDevice, s));
  } else {
    Mark mk(ctx, "seed", s);
    HIP_TRY(launch_seed(g, image, centres, s));
  }
  float* dist = o.persist_distance ? reinterpret_cast<float*>(ws + L.dist) : nullptr;
  int rc = run_iterations(ctx, g, it, image, iterations, o.tol, labels, centres, counts,
                          o.residuals, dist, s);
  if (rc) return rc;
  int32_t* nl = nlab_slot(ws, L);
  if (!o.no_connectivity) {
    Mark mk(ctx, "connectivity", s);
    HIP_TRY(launch_connectivity(g, centres, labels, cc_view(ws, L, g.N), nl, s));
  } else {
    HIP_TRY(launch_fill_i32(nl, (int32_t)g.K, 1, s));
  }
  if (o.n_labels_dev) HIP_TRY(hipMemcpyAsync(o.n_labels_dev, nl, 4, hipMemcpyDeviceToDevice, s));
  if (o.iters_done_dev)
    HIP_TRY(hipMemcpyAsync(o.iters_done_dev, it.iters, 4, hipMemcpyDeviceToDevice, s));
  return SSLIC_OK;
}

// Checks of sslic_run's arguments that need no device (shared with
// sslic_run_static).
int check_run(const void* image, int ndim, const int64_t* dims, int channels, int dtype,
              const int32_t* S, double m, int iterations, const sslic_options* opt,
              const int32_t* labels, const double* centres, Geo* g, sslic_options* o) {
  if (!image || !labels || !centres) return fail(SSLIC_EINVAL, "image, labels and centres must be given");
  if (iterations < 1) return fail(SSLIC_EINVAL, "iterations %d < 1", iterations);
  *o = sslic_options{};
  if (opt) *o = *opt;
  if (!(o->tol >= 0.0)) return fail(SSLIC_EINVAL, "tol must be >= 0");
  return make_geo(g, ndim, dims, channels, dtype, S, m, 0);
}

}  // namespace sslic

// ---- the entry point that allocates nothing (sslic_run_static) -------------
//
// Its workspace is this array: one copy on every GPU the library runs on,
// held until the process ends.  On the host `scratch` is only a stand-in for
// the symbol, not a device address: host code looks up the array's address
// on each device once (static_scratch) and passes that address to kernels
// and copies, never the name itself.
static __device__ __align__(256) char scratch[SSLIC_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};  // device address of `scratch`, per device ordinal

// The device address of `scratch` on `device` (the current device).
int static_scratch(int device, char** out) {
  if (device < 0 || device >= kMaxDevices)
    return fail(SSLIC_EUNSUPPORTED, "device ordinal %d above %d", device, kMaxDevices - 1);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(SSLIC_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device,
                  hipGetErrorString(e));
    }
    g_scratch[device] = static_cast<char*>(p);
  }
  *out = g_scratch[device];
  return SSLIC_OK;
}
}  // namespace

extern "C" {

const char* sslic_last_error(void) { return g_err.c_str(); }

int sslic_create(sslic_ctx** out, int device_ordinal) {
  if (!out) return fail(SSLIC_EINVAL, "out is NULL");
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    return fail(SSLIC_EDEVICE, "no HIP device available");
  }
  if (device_ordinal < 0 || device_ordinal >= n)
    return fail(SSLIC_EINVAL, "device %d outside [0, %d)", device_ordinal, n);
  sslic_ctx* c = new sslic_ctx;
  c->device = device_ordinal;
  if (hipSetDevice(device_ordinal) != hipSuccess ||
      hipHostMalloc((void**)&c->host_ints, 64, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return fail(SSLIC_EDEVICE, "cannot initialise device %d", device_ordinal);
  }
  *out = c;
  return SSLIC_OK;
}

void sslic_destroy(sslic_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  release_batch(ctx);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->host_ints) (void)hipHostFree(ctx->host_ints);
  delete ctx;
}

int sslic_num_clusters(int ndim, const int64_t* dims, const int32_t* S, int64_t* K_out,
                       int64_t* K_axis) {
  Geo g;
  int rc = make_geo(&g, ndim, dims, 1, kU8, S, 1.0, 0);
  if (rc) return rc;
  if (K_out) *K_out = g.K;
  if (K_axis)
    for (int i = 0; i < ndim; ++i) K_axis[i] = g.Ka[i];
  return SSLIC_OK;
}

int sslic_run(sslic_ctx* ctx, const void* image, int ndim, const int64_t* dims, int channels,
              sslic_dtype dtype, const int32_t* S, double m, int iterations,
              const sslic_options* opt, int32_t* labels, double* centres, int64_t* counts,
              int32_t* n_labels_out, int32_t* iters_done_out, sslic_stream_t stream) {
  if (!ctx) return fail(SSLIC_EINVAL, "ctx is NULL");
  Geo g;
  sslic_options o;
  int rc = check_run(image, ndim, dims, channels, dtype, S, m, iterations, opt, labels, centres,
                     &g, &o);
  if (rc) return rc;
  if ((rc = select_device(ctx))) return rc;
  const bool cc = !o.no_connectivity;
  const bool persist = o.persist_distance != 0;
  Layout L = layout(g, iterations, cc, !persist, persist);
  if ((rc = ensure_ws(ctx, L.total))) return rc;
  hipStream_t s = (hipStream_t)stream;
  if ((rc = run_on(ctx, ctx->ws, L, g, image, iterations, o, labels, centres, counts, s))) return rc;
  return read_ints(ctx, s, nlab_slot(ctx->ws, L), n_labels_out, iter_view(ctx->ws, L).iters,
                   iters_done_out);
}

int sslic_run_static(const void* image, int ndim, const int64_t* dims, int channels,
                     sslic_dtype dtype, const int32_t* S, double m, int iterations,
                     const sslic_options* opt, int32_t* labels, double* centres, int64_t* counts,
                     sslic_stream_t stream) {
  Geo g;
  sslic_options o;
  int rc = check_run(image, ndim, dims, channels, dtype, S, m, iterations, opt, labels, centres,
                     &g, &o);
  if (rc) return rc;
  const bool persist = o.persist_distance != 0;
  const Layout L = layout(g, iterations, !o.no_connectivity, !persist, persist);
  if (L.total > (size_t)SSLIC_STATIC_SCRATCH_BYTES)
    return fail(SSLIC_ENOMEM,
                "sslic_run_static: this request needs %zu bytes of workspace, above the static "
                "scratch of %zu bytes (use sslic_run)",
                L.total, (size_t)SSLIC_STATIC_SCRATCH_BYTES);
  int device = 0;
  HIP_TRY(hipGetDevice(&device));
  char* ws = nullptr;
  if ((rc = static_scratch(device, &ws))) return rc;
  return run_on(nullptr, ws, L, g, image, iterations, o, labels, centres, counts,
                (hipStream_t)stream);
}

int sslic_run_batch(sslic_ctx* ctx, const sslic_image_desc* images, int n, const sslic_options* opt,
                    int32_t* n_labels_out, sslic_stream_t stream) {
  if (!ctx) return fail(SSLIC_EINVAL, "ctx is NULL");
  if (n < 0 || (n > 0 && !images)) return fail(SSLIC_EINVAL, "bad image list");
  return run_batch(ctx, images, n, opt, n_labels_out, (hipStream_t)stream);
}

int sslic_seed(sslic_ctx* ctx, const void* image, int ndim, const int64_t* dims, int channels,
               sslic_dtype dtype, const int32_t* S, double* centres_out, sslic_stream_t stream) {
  if (!ctx || !image || !centres_out) return fail(SSLIC_EINVAL, "ctx, image and centres_out must be given");
  Geo g;
  int rc = make_geo(&g, ndim, dims, channels, dtype, S, 1.0, 0);
  if (rc) return rc;
  if ((rc = select_device(ctx))) return rc;
  HIP_TRY(launch_seed(g, image, centres_out, (hipStream_t)stream));
  return SSLIC_OK;
}

int sslic_grid_labels(sslic_ctx* ctx, int ndim, const int64_t* dims, const int32_t* S, int32_t* labels,
                      sslic_stream_t stream) {
  if (!ctx || !labels) return fail(SSLIC_EINVAL, "ctx and labels must be given");
  Geo g;
  int rc = make_geo(&g, ndim, dims, 1, kU8, S, 1.0, 0);
  if (rc) return rc;
  if ((rc = select_device(ctx))) return rc;
  HIP_TRY(launch_grid_labels(g, labels, (hipStream_t)stream));
  return SSLIC_OK;
}

int sslic_assign(sslic_ctx* ctx, const void* image, int ndim, const int64_t* dims, int channels,
                 sslic_dtype dtype, const int32_t* S, double m, const double* centres, int64_t K,
                 int32_t* labels, sslic_stream_t stream) {
  if (!ctx || !image || !centres || !labels) return fail(SSLIC_EINVAL, "missing pointer");
  if (K < 1) return fail(SSLIC_EINVAL, "K = %lld < 1", (long long)K);
  Geo g;
  int rc = make_geo(&g, ndim, dims, channels, dtype, S, m, K);
  if (rc) return rc;
  if ((rc = select_device(ctx))) return rc;
  Layout L = layout(g, 1, false, false);
  if ((rc = ensure_ws(ctx, L.total))) return rc;
  hipStream_t s = (hipStream_t)stream;
  Iter it = iter_view(ctx->ws, L);
  HIP_TRY(launch_fill_i32(it.bin_cnt, 0, g.nbins, s));
  HIP_TRY(launch_fill_i32(it.done, 0, 2, s));
  HIP_TRY(launch_prep(g, centres, it, s));
  HIP_TRY(launch_bins(g, it, s));
  // as a later iteration: voxels outside every window keep the given label
  HIP_TRY(launch_sweep(g, image, it, labels, 1, 0, s));
  return SSLIC_OK;
}

int sslic_assign_persist(sslic_ctx* ctx, const void* image, int ndim, const int64_t* dims,
                         int channels, sslic_dtype dtype, const int32_t* S, double m,
                         const double* centres, int64_t K, int32_t* labels, float* dist,
                         sslic_stream_t stream) {
  if (!ctx || !image || !centres || !labels || !dist) return fail(SSLIC_EINVAL, "missing pointer");
  if (K < 1) return fail(SSLIC_EINVAL, "K = %lld < 1", (long long)K);
  Geo g;
  int rc = make_geo(&g, ndim, dims, channels, dtype, S, m, K);
  if (rc) return rc;
  const size_t nd4 = (size_t)g.N * 4;
  const size_t ib = (size_t)g.N * channels * (dtype == kU8 ? 1 : dtype == kU16 ? 2 : 4);
  const char *d = (const char*)dist, *a = (const char*)image, *l = (const char*)labels;
  if (d < a + ib && a < d + nd4) return fail(SSLIC_EINVAL, "dist overlaps image");
  if (d < l + nd4 && l < d + nd4) return fail(SSLIC_EINVAL, "dist overlaps labels");
  if ((rc = select_device(ctx))) return rc;
  Layout L = layout(g, 1, false, false);
  if ((rc = ensure_ws(ctx, L.total))) return rc;
  hipStream_t s = (hipStream_t)stream;
  Iter it = iter_view(ctx->ws, L);
  HIP_TRY(launch_fill_i32(it.bin_cnt, 0, g.nbins, s));
  HIP_TRY(launch_fill_i32(it.done, 0, 2, s));
  HIP_TRY(launch_prep(g, centres, it, s));
  HIP_TRY(launch_bins(g, it, s));
  HIP_TRY(launch_assign_persist(g, image, it, labels, dist, 0, s));
  return SSLIC_OK;
}

int sslic_update(sslic_ctx* ctx, const void* image, int ndim, const int64_t* dims, int channels,
                 sslic_dtype dtype, const int32_t* S, double m, const int32_t* labels, int64_t K,
                 double* centres, int64_t* counts, double* residual, sslic_stream_t stream) {
  if (!ctx || !image || !centres || !labels) return fail(SSLIC_EINVAL, "missing pointer");
  if (K < 1) return fail(SSLIC_EINVAL, "K = %lld < 1", (long long)K);
  Geo g;
  int rc = make_geo(&g, ndim, dims, channels, dtype, S, m, K);
  if (rc) return rc;
  if ((rc = select_device(ctx))) return rc;
  Layout L = layout(g, 1, false, false);
  if ((rc = ensure_ws(ctx, L.total))) return rc;
  hipStream_t s = (hipStream_t)stream;
  Iter it = iter_view(ctx->ws, L);
  HIP_TRY(launch_fill_u64(it.acc, 0, g.K * g.F, s));
  HIP_TRY(launch_fill_f64(it.res_acc, 0.0, 2 * kResSlots, s));
  HIP_TRY(launch_fill_i32(it.done, 0, 2, s));
  HIP_TRY(launch_update(g, image, labels, it, s));
  HIP_TRY(launch_finalize(g, centres, counts, it, 0, 0, 0, s));
  HIP_TRY(launch_residual_finish(it, 0, -1.0, residual, s));
  return SSLIC_OK;
}

int sslic_connectivity(sslic_ctx* ctx, int ndim, const int64_t* dims, const int32_t* S, int channels,
                       const double* centres, int64_t K, int32_t* labels, int32_t* n_labels_out,
                       int32_t* n_labels_dev, sslic_stream_t stream) {
  if (!ctx || !centres || !labels) return fail(SSLIC_EINVAL, "missing pointer");
  if (K < 1) return fail(SSLIC_EINVAL, "K = %lld < 1", (long long)K);
  Geo g;
  int rc = make_geo(&g, ndim, dims, channels, kU8, S, 1.0, K);
  if (rc) return rc;
  if ((rc = select_device(ctx))) return rc;
  Layout L = layout(g, 1, true, false);
  if ((rc = ensure_ws(ctx, L.total))) return rc;
  hipStream_t s = (hipStream_t)stream;
  int32_t* nl = nlab_slot(ctx->ws, L);
  HIP_TRY(launch_connectivity(g, centres, labels, cc_view(ctx->ws, L, g.N), nl, s));
  if (n_labels_dev) HIP_TRY(hipMemcpyAsync(n_labels_dev, nl, 4, hipMemcpyDeviceToDevice, s));
  return read_ints(ctx, s, nl, n_labels_out, nullptr, nullptr);
}

int sslic_mask_contours(sslic_ctx* ctx, const void* image, int ndim, const int64_t* dims,
                        int channels, sslic_dtype dtype, const int32_t* labels, void* out,
                        sslic_stream_t stream) {
  if (!ctx || !image || !labels || !out) return fail(SSLIC_EINVAL, "missing pointer");
  if (ndim < 1 || ndim > kMaxDim || !dims) return fail(SSLIC_EINVAL, "ndim %d outside [1, 4]", ndim);
  int32_t S[kMaxDim];
  for (int i = 0; i < ndim; ++i) S[i] = (int32_t)std::min<int64_t>(std::max<int64_t>(dims[i], 1), 1 << 30);
  Geo g;
  int rc = make_geo(&g, ndim, dims, channels, dtype, S, 1.0, 0);
  if (rc) return rc;
  const size_t bytes = (size_t)g.N * channels * (dtype == kU8 ? 1 : dtype == kU16 ? 2 : 4);
  const char *a = (const char*)image, *o = (const char*)out;
  if (a < o + bytes && o < a + bytes) return fail(SSLIC_EINVAL, "out overlaps image");
  if ((rc = select_device(ctx))) return rc;
  HIP_TRY(launch_mask_contours(g, image, labels, out, (hipStream_t)stream));
  return SSLIC_OK;
}

int sslic_rgb_to_lab(sslic_ctx* ctx, const uint8_t* rgb, int64_t n_pixels, float* lab,
                     sslic_stream_t stream) {
  if (!ctx || !rgb || !lab) return fail(SSLIC_EINVAL, "missing pointer");
  if (n_pixels < 0) return fail(SSLIC_EINVAL, "n_pixels = %lld < 0", (long long)n_pixels);
  if (n_pixels == 0) return SSLIC_OK;
  const char *a = (const char*)rgb, *o = (const char*)lab;
  if (a < o + 12 * (size_t)n_pixels && o < a + 3 * (size_t)n_pixels)
    return fail(SSLIC_EINVAL, "lab overlaps rgb");
  int rc = select_device(ctx);
  if (rc) return rc;
  HIP_TRY(launch_rgb_to_lab(rgb, n_pixels, lab, (hipStream_t)stream));
  return SSLIC_OK;
}

int sslic_profile_enable(sslic_ctx* ctx, int enable) {
  if (!ctx) return fail(SSLIC_EINVAL, "ctx is NULL");
  int rc = select_device(ctx);
  if (rc) return rc;
  if (enable) {
    HIP_TRY(hipDeviceSynchronize());  // recorded events may still be pending
    ctx->marks.clear();
    ctx->ev_used = 0;
  }
  ctx->prof = enable != 0;
  return SSLIC_OK;
}

int sslic_profile_read(sslic_ctx* ctx, const char* kernel, double* total_ms, int64_t* launches) {
  if (!ctx || !kernel) return fail(SSLIC_EINVAL, "ctx and kernel must be given");
  int rc = select_device(ctx);
  if (rc) return rc;
  double tot = 0.0;
  int64_t n = 0;
  auto f = ctx->marks.find(kernel);
  if (f != ctx->marks.end()) {
    for (auto& pr : f->second) {
      HIP_TRY(hipEventSynchronize(pr.second));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second));
      tot += ms;
      ++n;
    }
    f->second.clear();
  }
  bool empty = true;
  for (auto& kv : ctx->marks) empty = empty && kv.second.empty();
  if (empty) ctx->ev_used = 0;
  if (total_ms) *total_ms = tot;
  if (launches) *launches = n;
  return SSLIC_OK;
}

}  // extern "C"
