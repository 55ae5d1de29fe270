// sslic_ctx.h -- the state behind the opaque sslic_ctx handle and the host
// helpers that the C ABI sources (api.hip, batch.hip) share.
#pragma once

#include <array>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/sslic.h"
#include "sslic_internal.h"

struct sslic_ctx {
  int device = 0;
  char* ws = nullptr;  // device workspace of single-image calls
  size_t ws_size = 0;
  int32_t* host_ints = nullptr;  // pinned staging for *_out scalars
  // event timing of kernel classes (sslic_profile.h)
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::map<std::string, std::vector<std::pair<hipEvent_t, hipEvent_t>>> marks;
  // batched form (batch.hip)
  char* bws = nullptr;  // device workspace of batches
  size_t bws_size = 0;
  char* bstage = nullptr;  // pinned staging of batch descriptors
  size_t bstage_size = 0;
  hipEvent_t bstage_ev = nullptr;  // recorded after the last upload from bstage
  hipStream_t cap_stream = nullptr;  // stream the batch graph is captured on
  hipGraphExec_t bgraph = nullptr;  // instance of the last captured batch
  std::vector<char> bkey;           // what it was captured for
  size_t bnlab = 0;                 // offset of the per-image label counts in bws
  std::map<std::array<int, 7>, int> tune;  // (dtype, nd, C, S_0..S_3) -> tile variant
};

namespace sslic {

int fail(int code, const char* fmt, ...);

#define HIP_TRY(expr)                                                               \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return ::sslic::fail(SSLIC_EDEVICE, "%s: %s (%s:%d)", #expr,                  \
                           hipGetErrorString(e_), __FILE__, __LINE__);              \
  } while (0)

int64_t grid_count(int64_t n, int64_t s);
// geometry of a request; checks every validity rule of sslic.h
int make_geo(Geo* g, int ndim, const int64_t* dims, int channels, int dtype, const int32_t* S,
             double m, int64_t K_override);

constexpr size_t kAlign = 256;
size_t al(size_t v);

// sections of the single-image workspace
struct Layout {
  size_t ctab, bin_of, bin_cnt, bin_start, bin_items, scan_part, acc, accf, part, res_acc, flags;
  size_t cc_parent, cc_size, cc_newlab, cc_part, cc_roots, cc_xface, dist, total;
};
// persist: room for the distance image kept across iterations (f32 [N])
Layout layout(const Geo& g, int iterations, bool cc, bool part, bool persist = false);
int ensure_ws(sslic_ctx* ctx, size_t need);
// views of a workspace laid out by `layout` at device address `base`
Iter iter_view(char* base, const Layout& L);
CCBuf cc_view(char* base, const Layout& L, int64_t N);
int select_device(sslic_ctx* ctx);

// Brackets the launches of one kernel class with events when profiling
// (sslic_profile.h); a no-op unless the context's profiling is on.
struct Mark {
  sslic_ctx* ctx;
  const char* name;
  hipStream_t s;
  hipEvent_t a = nullptr;
  Mark(sslic_ctx* c, const char* n, hipStream_t st);
  ~Mark();
  Mark(const Mark&) = delete;
  Mark& operator=(const Mark&) = delete;
};

// the batched form behind sslic_run_batch (batch.hip)
int run_batch(sslic_ctx* ctx, const sslic_image_desc* images, int n, const sslic_options* opt,
              int32_t* n_labels_out, hipStream_t s);
// frees what the batched form holds (sslic_destroy)
void release_batch(sslic_ctx* ctx);

}  // namespace sslic
