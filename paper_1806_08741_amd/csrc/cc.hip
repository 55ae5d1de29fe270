// cc.hip -- connectivity enforcement (Sec. 2.2 stage 3, Sec. 3.1 stage 3).
//
// The paper's marker-image procedure is sequential in its second pass (a
// raster scan that flood-fills each non-final component).  Its result has a
// closed description that parallelises:
//   * components are the face-connected components of equal labels; the
//     union-find below gives every voxel the smallest linear index of its
//     component as root, which is the voxel where the raster scan meets it;
//   * the first pass marks the component of label k found at (or near) centre
//     k final when 4 size > prod S;
//   * non-final components are visited in increasing root order: large ones
//     get K, K+1, ... in that order (an exclusive scan over roots); small ones
//     take the final label of the face neighbour just before their root, which
//     lies in a component with a smaller root, so following these links ends
//     at a final, large or origin component after finitely many steps.
#include "sslic_internal.h"

namespace sslic {

namespace {

constexpr int kThreads = 256;
constexpr int kPer = 16;
constexpr int kBlockVox = kThreads * kPer;

inline int blocks_for(int64_t n) { return (int)((n + kThreads - 1) / kThreads); }

__device__ __forceinline__ int find_root(const int32_t* parent, int v) {
  int p = parent[v];
  while (p != v) {
    v = p;
    p = parent[v];
  }
  return v;
}

// Lock-free union: always hang the larger root under the smaller one, so a
// root is the smallest index of its set.
__device__ __forceinline__ void unite(int32_t* parent, int a, int b) {
  while (true) {
    a = find_root(parent, a);
    b = find_root(parent, b);
    if (a == b) return;
    if (a < b) {
      int t = a;
      a = b;
      b = t;
    }
    if (atomicCAS(&parent[a], a, b) == a) return;
  }
}

// ---- union-find of equal-label face neighbours, in two levels -------------
// Level 1: a workgroup loads a tile of 4096 voxels into LDS and unites inside
// it with LDS atomics; every voxel's parent becomes the smallest voxel of its
// component within the tile (local raster order is global order), and each
// such local root gets its local size.  Level 2: unions across the low faces
// of every tile on the global parents, then every voxel takes its global root
// and each local root adds its size to it.

template <int ND>
struct CCTile;
template <>
struct CCTile<2> {
  static constexpr int L[2] = {6, 6};  // log2 extents: 64 x 64
};
template <>
struct CCTile<3> {
  static constexpr int L[3] = {4, 4, 4};  // 16^3
};
template <>
struct CCTile<4> {
  static constexpr int L[4] = {4, 3, 3, 2};  // 16 x 8 x 8 x 4
};
constexpr int kTileVox = 4096;
constexpr int kSeg = kTileVox / kThreads;  // voxels a thread walks along axis 0

template <int ND>
__device__ __forceinline__ void tile_origin(const Geo& g, int tile, int* o) {
  int r = tile;
  for (int i = 0; i < ND; ++i) {
    const int nt = (g.n[i] + (1 << CCTile<ND>::L[i]) - 1) >> CCTile<ND>::L[i];
    o[i] = (r % nt) << CCTile<ND>::L[i];
    r /= nt;
  }
}

__device__ __forceinline__ int find_local(const int* par, int v) {
  int p = par[v];
  while (p != v) {
    v = p;
    p = par[v];
  }
  return v;
}

__device__ __forceinline__ void unite_local(int* par, int a, int b) {
  while (true) {
    a = find_local(par, a);
    b = find_local(par, b);
    if (a == b) return;
    if (a < b) {
      int t = a;
      a = b;
      b = t;
    }
    if (atomicCAS(&par[a], a, b) == a) return;
  }
}

template <int ND>
__global__ void __launch_bounds__(kThreads)
cc_local_kernel(Geo g, const int32_t* __restrict__ labels, CCBuf b) {
  __shared__ int s_lab[kTileVox];
  __shared__ int s_par[kTileVox];
  __shared__ int s_size[kTileVox];
  int o[ND];
  tile_origin<ND>(g, blockIdx.x, o);
  auto local_coords = [&](int j, int* x) {
    int sh = 0;
    for (int i = 0; i < ND; ++i) {
      x[i] = (j >> sh) & ((1 << CCTile<ND>::L[i]) - 1);
      sh += CCTile<ND>::L[i];
    }
  };
  auto global_index = [&](const int* x, bool& in) {
    int64_t v = 0;
    in = true;
    for (int i = 0; i < ND; ++i) {
      const int gx = o[i] + x[i];
      in = in && gx < g.n[i];
      v += (int64_t)gx * g.st[i];
    }
    return v;
  };
  for (int j = threadIdx.x; j < kTileVox; j += kThreads) {
    int x[ND];
    local_coords(j, x);
    bool in;
    const int64_t v = global_index(x, in);
    s_lab[j] = in ? labels[v] : -1;
    s_par[j] = j;
    s_size[j] = 0;
  }
  __syncthreads();
  // every thread walks kSeg consecutive voxels of one row along axis 0:
  // runs of equal labels point at their first voxel (no atomics) ...
  const int j0 = threadIdx.x * kSeg;
  {
    int start = j0;
    for (int q = 1; q < kSeg; ++q) {
      const int j = j0 + q;
      if (s_lab[j] != s_lab[j - 1]) start = j;
      s_par[j] = start;
    }
  }
  __syncthreads();
  // ... then runs are united with the voxel before the segment and with the
  // rows below, once where an overlap of two runs begins
  {
    int x0[ND];
    local_coords(j0, x0);
    if (x0[0] > 0 && s_lab[j0] >= 0 && s_lab[j0] == s_lab[j0 - 1]) unite_local(s_par, j0 - 1, j0);
    int sh = CCTile<ND>::L[0];
    for (int i = 1; i < ND; ++i) {
      if (x0[i] > 0) {
        const int d = 1 << sh;
        for (int q = 0; q < kSeg; ++q) {
          const int j = j0 + q, l = s_lab[j];
          if (l < 0 || s_lab[j - d] != l) continue;
          if (q > 0 && s_lab[j - 1] == l && s_lab[j - 1 - d] == l) continue;  // same pair of runs
          unite_local(s_par, j - d, j);
        }
      }
      sh += CCTile<ND>::L[i];
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < kTileVox; j += kThreads) s_par[j] = find_local(s_par, j);
  __syncthreads();
  {  // sizes: each thread counts 16 consecutive voxels, one atomic per run
    const int j0 = threadIdx.x * (kTileVox / kThreads);
    int cur = -1, n = 0;
    for (int q = 0; q < kTileVox / kThreads; ++q) {
      const int j = j0 + q;
      if (s_lab[j] < 0) continue;
      const int r = s_par[j];
      if (r != cur) {
        if (n) atomicAdd(&s_size[cur], n);
        cur = r;
        n = 0;
      }
      ++n;
    }
    if (n) atomicAdd(&s_size[cur], n);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < kTileVox; j += kThreads) {
    if (s_lab[j] < 0) continue;
    int x[ND], xr[ND];
    local_coords(j, x);
    bool in;
    const int64_t v = global_index(x, in);
    local_coords(s_par[j], xr);
    const int64_t r = global_index(xr, in);
    b.parent[v] = (int32_t)r;
    b.size[v] = s_size[j];  // non-zero exactly at local roots
  }
}

template <int ND>
__global__ void __launch_bounds__(kThreads)
cc_faces_kernel(Geo g, const int32_t* __restrict__ labels, CCBuf b) {
  int o[ND];
  tile_origin<ND>(g, blockIdx.x, o);
  for (int i = 0; i < ND; ++i) {
    if (o[i] == 0) continue;
    // the face x_i = o_i: 4096 >> L[i] voxels, the other axes in raster order
    const int nf = kTileVox >> CCTile<ND>::L[i];
    for (int f = threadIdx.x; f < nf; f += kThreads) {
      int r = f;
      int64_t v = 0;
      bool in = true;
      for (int a = 0; a < ND; ++a) {
        int xa;
        if (a == i) {
          xa = o[a];
        } else {
          xa = o[a] + (r & ((1 << CCTile<ND>::L[a]) - 1));
          r >>= CCTile<ND>::L[a];
        }
        in = in && xa < g.n[a];
        v += (int64_t)xa * g.st[a];
      }
      if (!in) continue;
      const int64_t u = v - g.st[i];
      if (labels[u] == labels[v]) unite(b.parent, (int)u, (int)v);
    }
  }
}

__global__ void cc_flatten_kernel(Geo g, CCBuf b) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < g.N;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int r = find_root(b.parent, (int)v);
    const int s = b.size[v];
    if (s > 0 && r != (int)v) atomicAdd(&b.size[r], s);  // a local root joins its global root
    if (r == (int)v) b.final_[v] = 0;
    b.parent[v] = r;
  }
}

// First pass: the component of label k at the rounded centre k, or the first
// voxel of label k in raster order within floor(S_i / 2) of it.
__global__ void cc_first_kernel(Geo g, const double* __restrict__ cen,
                                const int32_t* __restrict__ labels, CCBuf b) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= g.K) return;
  const double* row = cen + k * g.row;
  int p[kMaxDim], lo[kMaxDim], hi[kMaxDim], x[kMaxDim];
  int64_t pl = 0;
  for (int i = 0; i < g.nd; ++i) {
    double c = i < g.nd_out ? row[g.C + i] : 0.0;
    double f = floor(c + 0.5);
    f = fmin(fmax(f, 0.0), (double)(g.n[i] - 1));
    p[i] = isfinite(c) ? (int)f : 0;
    pl += p[i] * g.st[i];
  }
  int64_t seed = -1;
  if (labels[pl] == (int32_t)k) {
    seed = pl;
  } else {
    for (int i = 0; i < g.nd; ++i) {
      int h = g.S[i] / 2;
      lo[i] = max(p[i] - h, 0);
      hi[i] = min(p[i] + h, g.n[i] - 1);
      x[i] = lo[i];
    }
    while (true) {
      int64_t v = 0;
      for (int i = 0; i < g.nd; ++i) v += x[i] * g.st[i];
      if (labels[v] == (int32_t)k) {
        seed = v;
        break;
      }
      int i = 0;
      while (i < g.nd) {
        if (++x[i] <= hi[i]) break;
        x[i] = lo[i];
        ++i;
      }
      if (i == g.nd) break;
    }
  }
  if (seed < 0) return;
  int r = b.parent[seed];
  if (4 * (int64_t)b.size[r] > g.prodS) b.final_[r] = 1;
}

__device__ __forceinline__ bool large_open_root(const Geo& g, const CCBuf& b, int64_t v) {
  return !b.final_[v] && 4 * (int64_t)b.size[v] > g.prodS;
}

// The roots (and, among them, the large open ones) of block `blk`'s 4096
// voxels, visited as 16 coalesced rows of 256 in raster order; f(v, large,
// rank_large, rank_root) is called for every root with its ranks inside the
// block.  Returns the block totals (thread 0).
template <class Fn>
__device__ __forceinline__ void block_roots(const Geo& g, const CCBuf& b, int64_t blk, int* sh,
                                            int& tot_large, int& tot_root, Fn f) {
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  constexpr int W = kThreads / 64;
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  int run_l = 0, run_r = 0;
  for (int j = 0; j < kPer; ++j) {
    const int64_t v = blk * kBlockVox + (int64_t)j * kThreads + threadIdx.x;
    const bool root = v < g.N && b.parent[v] == (int32_t)v;
    const bool large = root && large_open_root(g, b, v);
    const uint64_t mr = __ballot(root), ml = __ballot(large);
    if (lane == 0) {
      sh[wv] = __popcll(ml);
      sh[W + wv] = __popcll(mr);
    }
    __syncthreads();
    int off_l = 0, off_r = 0, all_l = 0, all_r = 0;
    for (int w = 0; w < W; ++w) {
      if (w < wv) {
        off_l += sh[w];
        off_r += sh[W + w];
      }
      all_l += sh[w];
      all_r += sh[W + w];
    }
    __syncthreads();
    if (root) f(v, large, run_l + off_l + __popcll(ml & lt), run_r + off_r + __popcll(mr & lt));
    run_l += all_l;
    run_r += all_r;
  }
  tot_large = run_l;
  tot_root = run_r;
}

__global__ void __launch_bounds__(kThreads) cc_count_kernel(Geo g, CCBuf b) {
  __shared__ int sh[2 * (kThreads / 64)];
  int tl, tr;
  block_roots(g, b, blockIdx.x, sh, tl, tr, [](int64_t, bool, int, int) {});
  if (threadIdx.x == 0) {
    b.part[blockIdx.x] = tl;
    b.rpart[blockIdx.x] = tr;
  }
}

__device__ __forceinline__ int block_exclusive_scan(int v, int* sh, int* total) {
  int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kThreads; off <<= 1) {
    int a = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  int incl = sh[t];
  *total = sh[kThreads - 1];
  __syncthreads();
  return incl - v;
}

// exclusive scans of both block count arrays; totals to b.total / b.nroots
__global__ void cc_scan_parts_kernel(CCBuf b, int nparts) {
  __shared__ int sh[kThreads];
  for (int which = 0; which < 2; ++which) {
    int32_t* part = which ? b.rpart : b.part;
    int carry = 0;
    for (int b0 = 0; b0 < nparts; b0 += kThreads) {
      int i = b0 + threadIdx.x;
      int v = i < nparts ? part[i] : 0;
      int total;
      int ex = block_exclusive_scan(v, sh, &total);
      if (i < nparts) part[i] = ex + carry;
      carry += total;
      __syncthreads();
    }
    if (threadIdx.x == 0) *(which ? b.nroots : b.total) = carry;
  }
}

// Label of every root: final roots keep their label, large open roots get
// K + rank, the origin keeps its label, other small roots store a link
// -(root of their predecessor) - 1 to be resolved.  The roots are listed in
// raster order as they go.
__global__ void __launch_bounds__(kThreads)
cc_root_labels_kernel(Geo g, const int32_t* __restrict__ labels, CCBuf b) {
  __shared__ int sh[2 * (kThreads / 64)];
  const int base_l = b.part[blockIdx.x], base_r = b.rpart[blockIdx.x];
  int tl, tr;
  block_roots(g, b, blockIdx.x, sh, tl, tr, [&](int64_t v, bool large, int rl, int rr) {
    int lab;
    if (b.final_[v]) {
      lab = labels[v];
    } else if (large) {
      lab = (int)(g.K + base_l + rl);
    } else if (v == 0) {
      lab = labels[0];
    } else {
      int64_t pred = -1, r = v;
      for (int i = 0; i < g.nd && pred < 0; ++i) {
        int xi = (int)(r % g.n[i]);
        r /= g.n[i];
        if (xi > 0) pred = v - g.st[i];
      }
      lab = -(b.parent[pred]) - 1;
    }
    b.newlab[v] = lab;
    b.roots[base_r + rr] = (int32_t)v;
  });
}

// Small roots follow their links to a resolved label (links go to strictly
// smaller roots, so every chain ends).
__global__ void cc_resolve_kernel(Geo g, CCBuf b) {
  const int n = *b.nroots;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int v = b.roots[i];
    int lab = b.newlab[v];
    if (lab >= 0) continue;
    int t = -lab - 1;
    int lt = b.newlab[t];
    while (lt < 0) {
      t = -lt - 1;
      lt = b.newlab[t];
    }
    b.newlab[v] = lt;
  }
}

__global__ void cc_relabel_kernel(Geo g, int32_t* __restrict__ labels, CCBuf b, int32_t* n_labels) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < g.N;
       v += (int64_t)gridDim.x * blockDim.x)
    labels[v] = b.newlab[b.parent[v]];
  if (n_labels && blockIdx.x == 0 && threadIdx.x == 0) *n_labels = (int32_t)(g.K + *b.total);
}

}  // namespace

hipError_t launch_connectivity(const Geo& g, const double* cen, int32_t* labels, const CCBuf& b,
                               int32_t* n_labels_dev, hipStream_t s) {
  int nv = (int)std::min<int64_t>(blocks_for(g.N), 1 << 18);
  int nparts = (int)((g.N + kBlockVox - 1) / kBlockVox);
  int ntiles = 1;
  for (int i = 0; i < g.nd; ++i) {
    const int L = g.nd == 2 ? CCTile<2>::L[i] : g.nd == 3 ? CCTile<3>::L[i] : CCTile<4>::L[i];
    ntiles *= (g.n[i] + (1 << L) - 1) >> L;
  }
  switch (g.nd) {
    case 2:
      cc_local_kernel<2><<<ntiles, kThreads, 0, s>>>(g, labels, b);
      cc_faces_kernel<2><<<ntiles, kThreads, 0, s>>>(g, labels, b);
      break;
    case 3:
      cc_local_kernel<3><<<ntiles, kThreads, 0, s>>>(g, labels, b);
      cc_faces_kernel<3><<<ntiles, kThreads, 0, s>>>(g, labels, b);
      break;
    default:
      cc_local_kernel<4><<<ntiles, kThreads, 0, s>>>(g, labels, b);
      cc_faces_kernel<4><<<ntiles, kThreads, 0, s>>>(g, labels, b);
      break;
  }
  cc_flatten_kernel<<<nv, kThreads, 0, s>>>(g, b);
  cc_first_kernel<<<blocks_for(g.K), kThreads, 0, s>>>(g, cen, labels, b);
  cc_count_kernel<<<nparts, kThreads, 0, s>>>(g, b);
  cc_scan_parts_kernel<<<1, kThreads, 0, s>>>(b, nparts);
  cc_root_labels_kernel<<<nparts, kThreads, 0, s>>>(g, labels, b);
  cc_resolve_kernel<<<(int)std::min<int64_t>(blocks_for(g.N), 4096), kThreads, 0, s>>>(g, b);
  cc_relabel_kernel<<<nv, kThreads, 0, s>>>(g, labels, b, n_labels_dev);
  return hipGetLastError();
}

}  // namespace sslic
