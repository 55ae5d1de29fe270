// batch.hip -- sslic_run_batch (include/sslic.h): many independent images
// through one set of shared tables.
//
//   * Images are ordered by group (pixel type, ndim, channels, tile shape);
//     each group has one flat list of the tiles of all its images.
//   * Per iteration: one bin sort over all centres of the batch, one
//     persistent sweep per group over its tile list, one reduce step per
//     group over its clusters, one residual / stop kernel over the images.
//     An image that has converged (or run its own iteration count) drops out
//     of every later launch; nothing returns to the host between iterations.
//   * The sequence is captured into a HIP graph on the context's own stream
//     and launched on the caller's stream; a later call with the same
//     descriptors and options replays that instance.
//   * Tile shape per (ndim, channels, dtype, S): the first time such an image
//     comes, every candidate shape times the sweep on the largest one of the
//     batch, and the fastest is kept for the context's lifetime.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "sslic_ctx.h"

namespace sslic {
namespace {

struct Group {
  int dtype, nd, C, var;
  int i0, i1;          // images [i0, i1) in batch order
  int64_t k0, k1;      // their global clusters
  int tile0, ntiles;   // their global tiles
};

// sections of the batch workspace; imgs, cl_img and tile_img are contiguous
// so that one copy uploads them
struct BLayout {
  size_t imgs, cl_img, tile_img, upload_bytes;
  size_t ctab, bin_of, bin_cnt, bin_start, bin_items, scan_part;
  size_t acc, accf, part, res, flags, nlab;
  size_t cc_parent, cc_size, cc_newlab, cc_part, cc_roots, cc_xface, total;
};

std::array<int, 7> key_of(const Geo& g) {
  return {g.dtype, g.nd, g.C, g.S[0], g.S[1], g.S[2], g.S[3]};
}

int tiles_of(const Geo& g, int var, int* nt) {
  int T[kMaxDim];
  sweep_tile_shape(g.nd, T, var);
  int n = 1;
  for (int i = 0; i < kMaxDim; ++i) nt[i] = 1;
  for (int i = 0; i < g.nd; ++i) {
    nt[i] = (g.n[i] + T[i] - 1) / T[i];
    n *= nt[i];
  }
  return n;
}

// The sweep's view of image g (tile variant var) with the given tables.
BImg make_bimg(const Geo& g, int var, const sslic_image_desc& d) {
  BImg b;
  memset(&b, 0, sizeof b);
  b.g = g;
  b.img = d.image;
  b.cen = d.centres;
  b.counts = d.counts;
  b.residuals = d.residuals;
  b.iters_out = d.iters_done;
  b.iterations = d.iterations;
  b.a.labels = d.labels;
  b.a.ntiles = tiles_of(g, var, b.a.nt);
  b.a.slots = sweep_slots(g, var);
  b.a.table = sweep_table_suits(g, var);
  b.a.fast = var == 0;  // as sslic_run: the fast form where it applies, on its tile shape
  sweep_tile_shape(g.nd, b.tdim, var);
  for (int i = g.nd; i < kMaxDim; ++i) b.tdim[i] = 1;
  return b;
}

void drop_graph(sslic_ctx* ctx) {
  if (ctx->bgraph) (void)hipGraphExecDestroy(ctx->bgraph);
  ctx->bgraph = nullptr;
  ctx->bkey.clear();
}

int ensure_bws(sslic_ctx* ctx, size_t need) {
  if (need <= ctx->bws_size) return SSLIC_OK;
  drop_graph(ctx);  // it names the old buffer
  if (ctx->bws) {
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipFree(ctx->bws));
    ctx->bws = nullptr;
    ctx->bws_size = 0;
  }
  size_t sz = need + (need >> 3);
  if (hipMalloc((void**)&ctx->bws, sz) != hipSuccess) {
    (void)hipGetLastError();
    ctx->bws = nullptr;
    return fail(SSLIC_ENOMEM, "cannot allocate %zu bytes of batch workspace", sz);
  }
  ctx->bws_size = sz;
  return SSLIC_OK;
}

// Pinned staging for uploads: waits for the previous upload out of it.
int ensure_stage(sslic_ctx* ctx, size_t need) {
  if (!ctx->bstage_ev) HIP_TRY(hipEventCreateWithFlags(&ctx->bstage_ev, hipEventDisableTiming));
  else HIP_TRY(hipEventSynchronize(ctx->bstage_ev));
  if (need <= ctx->bstage_size) return SSLIC_OK;
  if (ctx->bstage) HIP_TRY(hipHostFree(ctx->bstage));
  ctx->bstage = nullptr;
  ctx->bstage_size = 0;
  size_t sz = need + (need >> 2);
  if (hipHostMalloc((void**)&ctx->bstage, sz, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    ctx->bstage = nullptr;
    return fail(SSLIC_ENOMEM, "cannot allocate %zu bytes of pinned staging", sz);
  }
  ctx->bstage_size = sz;
  return SSLIC_OK;
}

// Times every tile variant of the sweep on image d (alone, on the
// single-image workspace; its centres and labels serve as scratch) and
// returns the fastest.  Waits for the stream.
int autotune(sslic_ctx* ctx, const sslic_image_desc& d, const Geo& g, hipStream_t s, int* best) {
  Layout L = layout(g, 1, false, true);
  const size_t o_img = al(L.total);
  int ntmax = 0;
  int nt[kMaxDim];
  for (int v = 0; v < kTileVars; ++v) ntmax = std::max(ntmax, tiles_of(g, v, nt));
  const size_t o_tile = o_img + al(sizeof(BImg));
  int rc = ensure_ws(ctx, o_tile + al((size_t)ntmax * 4));
  if (rc) return rc;
  Iter it = iter_view(ctx->ws, L);
  BImg* dimg = reinterpret_cast<BImg*>(ctx->ws + o_img);
  int32_t* dtile = reinterpret_cast<int32_t*>(ctx->ws + o_tile);
  HIP_TRY(launch_seed(g, d.image, d.centres, s));
  HIP_TRY(launch_fill_i32(it.bin_cnt, 0, g.nbins, s));
  HIP_TRY(launch_fill_i32(it.done, 0, 2, s));
  HIP_TRY(launch_fill_i32(dtile, 0, ntmax, s));
  HIP_TRY(launch_prep(g, d.centres, it, s));
  HIP_TRY(launch_bins(g, it, s));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(SSLIC_EDEVICE, "hipEventCreate failed");
  }
  float best_ms = 0.0f;
  *best = 0;
  for (int v = 0; v < kTileVars && rc == SSLIC_OK; ++v) {
    BImg b = make_bimg(g, v, d);
    b.a.ctab = it.ctab;
    b.a.done = it.done;
    b.a.part = it.part;
    b.a.acc = it.acc;
    b.a.accf = it.accf;
    b.flags = it.done;
    if ((rc = ensure_stage(ctx, sizeof(BImg)))) break;
    memcpy(ctx->bstage, &b, sizeof b);
    hipError_t e = hipMemcpyAsync(dimg, ctx->bstage, sizeof b, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(ctx->bstage_ev, s);
    const unsigned grid = (unsigned)b.a.ntiles;  // as the batch launches it
    // one launch to warm up, then five timed (the sums are scratch)
    for (int r = 0; r < 6 && e == hipSuccess; ++r) {
      if (r == 1) e = hipEventRecord(e0, s);
      if (e == hipSuccess)
        e = launch_sweep_batch(g.dtype, g.nd, g.C, v, dimg, dtile, 0, b.a.ntiles, it.bin_start,
                               it.bin_items, it.ctab, 0, grid, s);
    }
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      rc = fail(SSLIC_EDEVICE, "tile autotuning: %s", hipGetErrorString(e));
      break;
    }
    if (v == 0 || ms < best_ms) {
      best_ms = ms;
      *best = v;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

struct Plan {
  const sslic_image_desc* desc = nullptr;  // the caller's, by caller's index
  int n = 0, tmax = 0;
  bool cc = false;
  std::vector<int> ord;       // batch order -> caller's index
  std::vector<Geo> geo;       // by caller's index
  std::vector<Group> groups;
  int64_t K = 0, nbins = 0, Nmax = 0, XFmax = 0;
  int ntiles = 0, rs = 4;
  BLayout L{};
};

// everything enqueued for one batch (captured or direct); `timed`: bracket
// the sweep and reduce launches with profiling events (direct launches only)
int enqueue(sslic_ctx* ctx, const Plan& P, hipStream_t q, bool timed) {
  sslic_ctx* mctx = timed ? ctx : nullptr;
  char* b = ctx->bws;
  const BImg* imgs = reinterpret_cast<const BImg*>(b + P.L.imgs);
  const int32_t* cl_img = reinterpret_cast<const int32_t*>(b + P.L.cl_img);
  const int32_t* tile_img = reinterpret_cast<const int32_t*>(b + P.L.tile_img);
  float* ctab = reinterpret_cast<float*>(b + P.L.ctab);
  int32_t* flags = reinterpret_cast<int32_t*>(b + P.L.flags);
  Iter it{};
  it.ctab = ctab;
  it.bin_of = reinterpret_cast<int32_t*>(b + P.L.bin_of);
  it.bin_cnt = reinterpret_cast<int32_t*>(b + P.L.bin_cnt);
  it.bin_start = reinterpret_cast<int32_t*>(b + P.L.bin_start);
  it.bin_items = reinterpret_cast<int32_t*>(b + P.L.bin_items);
  it.scan_part = reinterpret_cast<int32_t*>(b + P.L.scan_part);
  it.done = flags + 2 * P.n;  // the bin sort runs every iteration
  Geo gb;
  memset(&gb, 0, sizeof gb);
  gb.K = P.K;
  gb.nbins = P.nbins;
  gb.rs = P.rs;

  HIP_TRY(launch_fill_i32(it.bin_cnt, 0, P.nbins, q));
  // accumulators and their flags (adjacent)
  HIP_TRY(launch_fill_u64(reinterpret_cast<uint64_t*>(b + P.L.acc), 0,
                          (int64_t)((P.L.part - P.L.acc) / 8), q));
  HIP_TRY(launch_fill_u64(reinterpret_cast<uint64_t*>(b + P.L.part), 0,
                          (int64_t)((P.L.res - P.L.part) / 8), q));
  HIP_TRY(launch_fill_f64(reinterpret_cast<double*>(b + P.L.res), 0.0,
                          (int64_t)((P.L.flags - P.L.res) / 8), q));
  HIP_TRY(launch_fill_i32(flags, 0, 2 * P.n + 1, q));
  HIP_TRY(launch_batch_zero_residuals(imgs, P.n, P.tmax, q));
  // seeding, one launch per pixel type (groups are ordered by type first)
  for (size_t a = 0; a < P.groups.size();) {
    size_t e = a;
    while (e < P.groups.size() && P.groups[e].dtype == P.groups[a].dtype) ++e;
    HIP_TRY(launch_seed_batch(P.groups[a].dtype, imgs, cl_img, P.groups[a].k0, P.groups[e - 1].k1, q));
    a = e;
  }
  HIP_TRY(launch_prep_batch(imgs, cl_img, P.K, ctab, it.bin_of, it.bin_cnt, q));
  for (int t = 0; t < P.tmax; ++t) {
    HIP_TRY(launch_bins(gb, it, q));
    for (const Group& g : P.groups) {
      // a workgroup per tile: the hardware then overlaps one tile's drain
      // with the next tile's start (measured faster than a grid that walks
      // several tiles per workgroup)
      const unsigned grid = (unsigned)g.ntiles;
      Mark mk(mctx, "sweep_batch", q);
      HIP_TRY(launch_sweep_batch(g.dtype, g.nd, g.C, g.var, imgs, tile_img, g.tile0, g.ntiles,
                                 it.bin_start, it.bin_items, it.ctab, t, grid, q));
    }
    for (const Group& g : P.groups) {
      Mark mk(mctx, "finalize_batch", q);
      HIP_TRY(launch_finalize_batch(g.dtype, g.nd, g.C, imgs, cl_img, g.k0, g.k1, ctab, it.bin_of,
                                    it.bin_cnt, t, q));
    }
    HIP_TRY(launch_residual_finish_batch(imgs, P.n, t, q));
  }
  HIP_TRY(launch_batch_outputs(imgs, P.n, q));
  if (P.cc) {
    CCBuf c;
    c.parent = reinterpret_cast<int32_t*>(b + P.L.cc_parent);
    c.size = reinterpret_cast<int32_t*>(b + P.L.cc_size);
    c.newlab = reinterpret_cast<int32_t*>(b + P.L.cc_newlab);
    cc_carve(c, reinterpret_cast<int32_t*>(b + P.L.cc_part), P.Nmax);
    c.roots = reinterpret_cast<int32_t*>(b + P.L.cc_roots);
    c.xface = reinterpret_cast<int32_t*>(b + P.L.cc_xface);
    c.total = flags + 2 * P.n + 1;
    int32_t* nlab = reinterpret_cast<int32_t*>(b + P.L.nlab);
    for (int j = 0; j < P.n; ++j) {
      const int i = P.ord[j];
      HIP_TRY(launch_connectivity(P.geo[i], P.desc[i].centres, P.desc[i].labels, c, nlab + i, q));
    }
  }
  return SSLIC_OK;
}

}  // namespace

int run_batch(sslic_ctx* ctx, const sslic_image_desc* images, int n, const sslic_options* opt,
              int32_t* n_labels_out, hipStream_t s) {
  sslic_options o{};
  if (opt) o = *opt;
  if (!(o.tol >= 0.0)) return fail(SSLIC_EINVAL, "tol must be >= 0");
  if (o.persist_distance)
    return fail(SSLIC_EUNSUPPORTED, "persist_distance is a sslic_run option only");
  if (n == 0) return SSLIC_OK;
  int rc = SSLIC_OK;

  Plan P;
  P.desc = images;
  P.n = n;
  P.cc = !o.no_connectivity;
  P.geo.resize(n);
  for (int i = 0; i < n; ++i) {
    const sslic_image_desc& d = images[i];
    if (!d.image || !d.labels || !d.centres)
      return fail(SSLIC_EINVAL, "image %d: image, labels and centres must be given", i);
    if (d.iterations < 1) return fail(SSLIC_EINVAL, "image %d: iterations %d < 1", i, d.iterations);
    if ((rc = make_geo(&P.geo[i], d.ndim, d.dims, d.channels, d.dtype, d.S, d.m, 0)))
      return fail(rc, "image %d: %s", i, sslic_last_error());
    P.tmax = std::max(P.tmax, d.iterations);
  }
  if ((rc = select_device(ctx))) return rc;

  // tile variant per image: tuned once per (ndim, channels, dtype, S); the
  // images the fast form serves keep its tile shape, as in sslic_run, so
  // that a batch gives them the same results as a run of their own
  std::vector<int> var(n, 0);
  if (!o.no_autotune) {
    std::map<std::array<int, 7>, int> pick;
    for (int i = 0; i < n; ++i) {
      if (sweep_fast_applies(P.geo[i])) continue;
      auto k = key_of(P.geo[i]);
      if (ctx->tune.count(k)) continue;
      auto f = pick.find(k);
      if (f == pick.end() || P.geo[i].N > P.geo[f->second].N) pick[k] = i;
    }
    for (auto& kv : pick) {
      int v = 0;
      if ((rc = autotune(ctx, images[kv.second], P.geo[kv.second], s, &v))) return rc;
      ctx->tune[kv.first] = v;
    }
    for (int i = 0; i < n; ++i)
      var[i] = sweep_fast_applies(P.geo[i]) ? 0 : ctx->tune[key_of(P.geo[i])];
  }

  // what a captured graph would have been made for
  std::vector<char> key(sizeof(int) + (size_t)n * sizeof(sslic_image_desc) + sizeof(double) +
                        sizeof(int) + (size_t)n * sizeof(int));
  {
    char* k = key.data();
    memcpy(k, &n, sizeof n);
    k += sizeof n;
    memcpy(k, images, (size_t)n * sizeof(sslic_image_desc));
    k += (size_t)n * sizeof(sslic_image_desc);
    memcpy(k, &o.tol, sizeof o.tol);
    k += sizeof o.tol;
    memcpy(k, &o.no_connectivity, sizeof(int));
    k += sizeof(int);
    memcpy(k, var.data(), (size_t)n * sizeof(int));
  }
  const bool use_graph = !o.no_graph;
  if (use_graph && ctx->bgraph && key == ctx->bkey) {
    HIP_TRY(hipGraphLaunch(ctx->bgraph, s));
  } else {
    drop_graph(ctx);
    // batch order: by group
    P.ord.resize(n);
    std::iota(P.ord.begin(), P.ord.end(), 0);
    std::stable_sort(P.ord.begin(), P.ord.end(), [&](int a, int b) {
      const Geo &x = P.geo[a], &y = P.geo[b];
      return std::make_tuple(x.dtype, x.nd, x.C, var[a]) < std::make_tuple(y.dtype, y.nd, y.C, var[b]);
    });
    for (int i = 0; i < n; ++i) P.rs = std::max(P.rs, P.geo[i].rs);
    // offsets
    std::vector<BImg> bi(n);
    size_t acc_w = 0, part_w = 0, res_w = 0;
    for (int j = 0; j < n; ++j) {
      const int i = P.ord[j];
      Geo g = P.geo[i];
      g.rs = P.rs;
      if (j == 0 || var[i] != var[P.ord[j - 1]] || g.dtype != P.geo[P.ord[j - 1]].dtype ||
          g.nd != P.geo[P.ord[j - 1]].nd || g.C != P.geo[P.ord[j - 1]].C) {
        Group gr;
        gr.dtype = g.dtype;
        gr.nd = g.nd;
        gr.C = g.C;
        gr.var = var[i];
        gr.i0 = j;
        gr.k0 = P.K;
        gr.tile0 = P.ntiles;
        P.groups.push_back(gr);
      }
      BImg& b = bi[j];
      b = make_bimg(g, var[i], images[i]);
      b.tol = o.tol;
      b.koff = P.K;
      b.binoff = P.nbins;
      b.tile_off = P.ntiles;
      P.K += g.K;
      P.nbins += g.nbins;
      if ((int64_t)P.ntiles + b.a.ntiles >= (1LL << 31) || P.K >= (1LL << 31) || P.nbins >= (1LL << 31))
        return fail(SSLIC_EINVAL, "batch too large for 32-bit cluster, bin and tile indices");
      P.ntiles += b.a.ntiles;
      P.Nmax = std::max(P.Nmax, g.N);
      P.XFmax = std::max(P.XFmax, cc_xface_ints(g));
      b.a.bstart = nullptr;
      acc_w += (size_t)g.K * g.F;  // offsets in words, resolved below
      part_w += b.a.slots ? (size_t)g.K * ((size_t)1 << g.nd) * (g.F + 1) : 0;
      res_w += 2 * (size_t)kResSlots * images[i].iterations;
      Group& gr = P.groups.back();
      gr.i1 = j + 1;
      gr.k1 = P.K;
      gr.ntiles = P.ntiles - gr.tile0;
    }
    BLayout& L = P.L;
    size_t off = 0;
    auto put = [&](size_t bytes) {
      size_t at = off;
      off += al(bytes);
      return at;
    };
    L.imgs = put((size_t)n * sizeof(BImg));
    L.cl_img = off;
    off += (size_t)P.K * 4;
    L.tile_img = off;
    off += (size_t)P.ntiles * 4;
    L.upload_bytes = off - L.imgs;
    off = al(off);
    L.ctab = put((size_t)P.K * P.rs * 4);
    L.bin_of = put((size_t)P.K * 4);
    L.bin_cnt = put((size_t)P.nbins * 4);
    L.bin_start = put((size_t)(P.nbins + 1) * 4);
    L.bin_items = put((size_t)P.K * 4);
    L.scan_part = put((size_t)(P.nbins / 4096 + 2) * 4);
    L.acc = put(acc_w * 8);
    L.accf = put((size_t)P.K);
    L.part = put(part_w * 8);
    L.res = put(res_w * 8);
    L.flags = put(((size_t)2 * n + 2) * 4);
    L.nlab = put((size_t)n * 4);
    if (P.cc) {
      L.cc_parent = put((size_t)P.Nmax * 4);
      L.cc_size = put((size_t)P.Nmax * 4);
      L.cc_newlab = put((size_t)P.Nmax * 4);
      L.cc_part = put((size_t)cc_part_ints(P.Nmax) * 4);
      L.cc_roots = put((size_t)P.Nmax * 4);
      L.cc_xface = put((size_t)P.XFmax * 4);
    }
    L.total = off;
    if ((rc = ensure_bws(ctx, L.total))) return rc;
    ctx->bnlab = L.nlab;
    char* base = ctx->bws;
    // per-image pointers into the pools
    size_t ao = 0, po = 0, ro = 0;
    int32_t* flags = reinterpret_cast<int32_t*>(base + L.flags);
    for (int j = 0; j < n; ++j) {
      BImg& b = bi[j];
      const Geo& g = b.g;
      b.a.ctab = reinterpret_cast<const float*>(base + L.ctab) + b.koff * P.rs;
      b.a.acc = reinterpret_cast<uint64_t*>(base + L.acc) + ao;
      b.a.accf = reinterpret_cast<uint8_t*>(base + L.accf) + b.koff;
      b.a.part = b.a.slots ? reinterpret_cast<uint64_t*>(base + L.part) + po : nullptr;
      b.res = reinterpret_cast<double*>(base + L.res) + ro;
      b.flags = flags + 2 * j;
      b.a.done = b.flags;
      ao += (size_t)g.K * g.F;
      po += b.a.slots ? (size_t)g.K * ((size_t)1 << g.nd) * (g.F + 1) : 0;
      ro += 2 * (size_t)kResSlots * b.iterations;
    }
    // upload descriptors and the cluster / tile -> image maps
    if ((rc = ensure_stage(ctx, L.upload_bytes))) return rc;
    char* st = ctx->bstage;
    memcpy(st, bi.data(), (size_t)n * sizeof(BImg));
    int32_t* cl = reinterpret_cast<int32_t*>(st + (L.cl_img - L.imgs));
    int32_t* tl = reinterpret_cast<int32_t*>(st + (L.tile_img - L.imgs));
    for (int j = 0; j < n; ++j) {
      for (int64_t k = 0; k < bi[j].g.K; ++k) cl[bi[j].koff + k] = j;
      for (int t = 0; t < bi[j].a.ntiles; ++t) tl[bi[j].tile_off + t] = j;
    }
    HIP_TRY(hipMemcpyAsync(base + L.imgs, st, L.upload_bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(ctx->bstage_ev, s));

    if (use_graph) {
      if (!ctx->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
      HIP_TRY(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
      rc = enqueue(ctx, P, ctx->cap_stream, false);
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamEndCapture(ctx->cap_stream, &graph);
      if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
      }
      if (e != hipSuccess) return fail(SSLIC_EDEVICE, "graph capture: %s", hipGetErrorString(e));
      hipGraphExec_t exec = nullptr;
      e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) return fail(SSLIC_EDEVICE, "graph instantiation: %s", hipGetErrorString(e));
      ctx->bgraph = exec;
      ctx->bkey = key;
      HIP_TRY(hipGraphLaunch(exec, s));
    } else {
      if ((rc = enqueue(ctx, P, s, true))) return rc;
    }
  }

  if (n_labels_out) {
    if (o.no_connectivity) {
      for (int i = 0; i < n; ++i) n_labels_out[i] = (int32_t)P.geo[i].K;
    } else {
      if ((rc = ensure_stage(ctx, (size_t)n * 4))) return rc;
      HIP_TRY(hipMemcpyAsync(ctx->bstage, ctx->bws + ctx->bnlab, (size_t)n * 4, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipEventRecord(ctx->bstage_ev, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    if (!o.no_connectivity) memcpy(n_labels_out, ctx->bstage, (size_t)n * 4);
  }
  return SSLIC_OK;
}

void release_batch(sslic_ctx* ctx) {
  drop_graph(ctx);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->bstage_ev) (void)hipEventDestroy(ctx->bstage_ev);
  if (ctx->bstage) (void)hipHostFree(ctx->bstage);
  if (ctx->bws) (void)hipFree(ctx->bws);
  ctx->cap_stream = nullptr;
  ctx->bstage_ev = nullptr;
  ctx->bstage = nullptr;
  ctx->bws = nullptr;
  ctx->bstage_size = ctx->bws_size = 0;
}

}  // namespace sslic
