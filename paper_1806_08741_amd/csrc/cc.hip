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

__global__ void cc_init_kernel(Geo g, CCBuf b) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < g.N;
       v += (int64_t)gridDim.x * blockDim.x) {
    b.parent[v] = (int32_t)v;
    b.size[v] = 0;
    b.final_[v] = 0;
  }
}

__global__ void cc_union_kernel(Geo g, const int32_t* __restrict__ labels, CCBuf b) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < g.N;
       v += (int64_t)gridDim.x * blockDim.x) {
    int l = labels[v];
    int64_t r = v;
    for (int i = 0; i < g.nd; ++i) {
      int xi = (int)(r % g.n[i]);
      r /= g.n[i];
      if (xi > 0) {
        int64_t u = v - g.st[i];
        if (labels[u] == l) unite(b.parent, (int)u, (int)v);
      }
    }
  }
}

__global__ void cc_flatten_kernel(Geo g, CCBuf b) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < g.N;
       v += (int64_t)gridDim.x * blockDim.x) {
    int r = find_root(b.parent, (int)v);
    b.parent[v] = r;
    atomicAdd(&b.size[r], 1);
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
  return b.parent[v] == (int32_t)v && !b.final_[v] && 4 * (int64_t)b.size[v] > g.prodS;
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

__global__ void cc_count_kernel(Geo g, CCBuf b) {
  __shared__ int sh[kThreads];
  int64_t base = (int64_t)blockIdx.x * kBlockVox + (int64_t)threadIdx.x * kPer;
  int cnt = 0;
  for (int j = 0; j < kPer; ++j) {
    int64_t v = base + j;
    if (v < g.N && large_open_root(g, b, v)) ++cnt;
  }
  int total;
  block_exclusive_scan(cnt, sh, &total);
  if (threadIdx.x == 0) b.part[blockIdx.x] = total;
}

__global__ void cc_scan_parts_kernel(CCBuf b, int nparts) {
  __shared__ int sh[kThreads];
  int carry = 0;
  for (int b0 = 0; b0 < nparts; b0 += kThreads) {
    int i = b0 + threadIdx.x;
    int v = i < nparts ? b.part[i] : 0;
    int total;
    int ex = block_exclusive_scan(v, sh, &total);
    if (i < nparts) b.part[i] = ex + carry;
    carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) *b.total = carry;
}

// Label of every root: final roots keep their label, large open roots get
// K + rank, the origin keeps its label, other small roots store a link
// -(root of their predecessor) - 1 to be resolved.
__global__ void cc_root_labels_kernel(Geo g, const int32_t* __restrict__ labels, CCBuf b) {
  __shared__ int sh[kThreads];
  int64_t base = (int64_t)blockIdx.x * kBlockVox + (int64_t)threadIdx.x * kPer;
  int cnt = 0;
  for (int j = 0; j < kPer; ++j) {
    int64_t v = base + j;
    if (v < g.N && large_open_root(g, b, v)) ++cnt;
  }
  int total;
  int rank = block_exclusive_scan(cnt, sh, &total) + b.part[blockIdx.x];
  for (int j = 0; j < kPer; ++j) {
    int64_t v = base + j;
    if (v >= g.N || b.parent[v] != (int32_t)v) continue;
    int lab;
    if (b.final_[v]) {
      lab = labels[v];
    } else if (4 * (int64_t)b.size[v] > g.prodS) {
      lab = (int)(g.K + rank);
      ++rank;
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
  }
}

__global__ void cc_resolve_kernel(Geo g, CCBuf b) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < g.N;
       v += (int64_t)gridDim.x * blockDim.x) {
    if (b.parent[v] != (int32_t)v) continue;
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
  cc_init_kernel<<<nv, kThreads, 0, s>>>(g, b);
  cc_union_kernel<<<nv, kThreads, 0, s>>>(g, labels, b);
  cc_flatten_kernel<<<nv, kThreads, 0, s>>>(g, b);
  cc_first_kernel<<<blocks_for(g.K), kThreads, 0, s>>>(g, cen, labels, b);
  cc_count_kernel<<<nparts, kThreads, 0, s>>>(g, b);
  cc_scan_parts_kernel<<<1, kThreads, 0, s>>>(b, nparts);
  cc_root_labels_kernel<<<nparts, kThreads, 0, s>>>(g, labels, b);
  cc_resolve_kernel<<<nv, kThreads, 0, s>>>(g, b);
  cc_relabel_kernel<<<nv, kThreads, 0, s>>>(g, labels, b, n_labels_dev);
  return hipGetLastError();
}

}  // namespace sslic
