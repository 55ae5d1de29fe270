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
constexpr int kWaves = kThreads / 64;
constexpr int kChunk = 1024;                     // voxels one wave ranks: 16 rows of 64
constexpr int kScanPer = 16;
constexpr int kScanBlock = kThreads * kScanPer;  // chunk counts one scan block takes

inline int blocks_for(int64_t n) { return (int)((n + kThreads - 1) / kThreads); }

// Workgroups are dealt to the 8 XCDs in turn.  This numbers them so that
// each XCD takes one contiguous eighth of the grid, in order: what
// neighbouring workgroups share (the rows just before, the roots just
// behind) is then in that XCD's own L2.  A bijection for any grid size.
__device__ __forceinline__ int xcd_block() {
  const int nb = (int)gridDim.x, b = (int)blockIdx.x;
  const int per = nb / 8, rem = nb % 8, x = b % 8;
  return x * per + min(x, rem) + b / 8;
}

__device__ __forceinline__ int find_root(const int32_t* parent, int v) {
  int p = parent[v];
  while (p != v) {
    v = p;
    p = parent[v];
  }
  return v;
}

// Lock-free union of the sets of two nodes of the forest of local roots
// (after the local pass every voxel points at its local root, and only local
// roots are ever linked): the larger root hangs under the smaller one, so a
// root is the smallest index of its set.  Paths are halved on the way with
// plain stores: a halving store writes a local root's parent, never another
// voxel's, and only moves it toward its root.
__device__ __forceinline__ int find_halving(int32_t* parent, int v) {
  while (true) {
    const int p = parent[v];
    const int gp = parent[p];
    if (p == gp) return p;
    parent[v] = gp;
    v = gp;
  }
}

__device__ __forceinline__ void unite_roots(int32_t* parent, int a, int b) {
  while (true) {
    a = find_halving(parent, a);
    b = find_halving(parent, b);
    if (a == b) return;
    if (a < b) {
      const int t = a;
      a = b;
      b = t;
    }
    const int old = atomicCAS(&parent[a], a, b);
    if (old == a) return;
    a = old;  // a's parent as the atomic saw it: progress even if plain loads lag
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
  // 64 x 8 x 8: rows of 256 bytes, so every pass over the tile reads and
  // writes whole lines, and the faces across axis 0 (each voxel on a line of
  // its own) hold 64 voxels instead of 256
  static constexpr int L[3] = {6, 3, 3};
};
template <>
struct CCTile<4> {
  static constexpr int L[4] = {4, 3, 3, 2};  // 16 x 8 x 8 x 4
};
constexpr int kTileVox = 4096;
constexpr int kSeg = kTileVox / kThreads;  // voxels a thread walks along axis 0

// A tile's first and last column along axis 0 (one voxel per line of the
// tile, each on a line of memory of its own) are also kept compact, per tile:
// [0] labels and [1] local roots of the first column, [2] and [3] of the
// last, so the face unions across axis 0 read them as whole lines.
template <int ND>
constexpr int xcol() { return kTileVox >> CCTile<ND>::L[0]; }
template <int ND>
constexpr int xface_ints() { return 4 * xcol<ND>(); }

template <int ND>
__device__ __forceinline__ void tile_origin(const Geo& g, int tile, int* o) {
  int r = tile;
  for (int i = 0; i < ND; ++i) {
    const int nt = (g.n[i] + (1 << CCTile<ND>::L[i]) - 1) >> CCTile<ND>::L[i];
    o[i] = (r % nt) << CCTile<ND>::L[i];
    r /= nt;
  }
}

// LDS position of local voxel j: one pad word after every 16, so the 64
// lanes of a wave, each walking its own 16 consecutive voxels, hit distinct
// banks.
__device__ __forceinline__ int pd(int j) { return j + (j >> 4); }
constexpr int kPadVox = kTileVox + kTileVox / 16;

__device__ __forceinline__ int find_local(const int* par, int v) {
  int p = par[pd(v)];
  while (p != v) {
    v = p;
    p = par[pd(v)];
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
    if (atomicCAS(&par[pd(a)], a, b) == a) return;
  }
}

// Voxel indices fit 32 bits (images hold fewer than 2^31 voxels), so the
// tile kernels index in int.
template <int ND>
struct TileIndex {
  int o[ND];
  int st[ND];
  int base;  // index of the tile origin
  __device__ TileIndex(const Geo& g, int tile) {
    tile_origin<ND>(g, tile, o);
    base = 0;
    for (int i = 0; i < ND; ++i) {
      st[i] = (int)g.st[i];
      base += o[i] * st[i];
    }
  }
  // global index of local voxel j, and whether it lies inside the image
  __device__ __forceinline__ int at(const Geo& g, int j, bool& in) const {
    int v = base, sh = 0;
    in = true;
    for (int i = 0; i < ND; ++i) {
      const int x = (j >> sh) & ((1 << CCTile<ND>::L[i]) - 1);
      sh += CCTile<ND>::L[i];
      in = in && o[i] + x < g.n[i];
      v += i == 0 ? x : x * st[i];
    }
    return v;
  }
};

template <int ND>
__global__ void __launch_bounds__(kThreads)
cc_local_kernel(Geo g, const int32_t* __restrict__ labels, CCBuf b) {
  __shared__ int s_lab[kPadVox];  // labels, then (once unions are done) local sizes
  __shared__ int s_par[kPadVox];
  int* s_size = s_lab;
  const TileIndex<ND> ti(g, blockIdx.x);
  constexpr int XL = CCTile<ND>::L[0], XE = 1 << XL;
  int32_t* xf = b.xface + (int64_t)blockIdx.x * xface_ints<ND>();
  {
    int lab[kSeg];  // all of this thread's loads in flight at once
#pragma unroll
    for (int q = 0; q < kSeg; ++q) {
      bool in;
      const int v = ti.at(g, threadIdx.x + q * kThreads, in);
      lab[q] = in ? labels[v] : -1;
    }

#pragma unroll
    for (int q = 0; q < kSeg; ++q) {
      const int j = threadIdx.x + q * kThreads;
      s_lab[pd(j)] = lab[q];
      s_par[pd(j)] = j;
    }
  }
  __syncthreads();
  // the first and last columns' labels, as whole lines
  for (int t = threadIdx.x; t < 2 * xcol<ND>(); t += kThreads) {
    const int c = t / xcol<ND>(), f = t % xcol<ND>();
    xf[2 * c * xcol<ND>() + f] = s_lab[pd((f << XL) + c * (XE - 1))];
  }
  // every thread walks kSeg consecutive voxels of one row along axis 0, with
  // their labels in registers (LDS reads issued together, not one per test):
  // runs of equal labels point at their first voxel (no atomics) ...
  const int j0 = threadIdx.x * kSeg;
  int own[kSeg];
#pragma unroll
  for (int q = 0; q < kSeg; ++q) own[q] = s_lab[pd(j0 + q)];
  uint32_t starts = 1;  // bit q: a run begins at j0 + q
  {
    int start = j0;
#pragma unroll
    for (int q = 1; q < kSeg; ++q) {
      if (own[q] != own[q - 1]) {
        start = j0 + q;
        starts |= 1u << q;
      }
      s_par[pd(j0 + q)] = start;
    }
  }
  __syncthreads();
  // ... then runs are united with the voxel before the segment and with the
  // rows below, once where an overlap of two runs begins.  The pairs to unite
  // are collected first (bit 16 (i - 1) + q: voxel q and its neighbour below
  // along axis i; bit 63: the first voxel and the one before the segment) and
  // then taken one by one, so the wave loops as often as its busiest lane
  // has pairs, not once per voxel that any lane unites.
  {
    uint64_t todo = 0;
    int sh = CCTile<ND>::L[0];
    const int x0 = j0 & ((1 << sh) - 1);
    if (x0 > 0 && own[0] >= 0 && own[0] == s_lab[pd(j0 - 1)]) todo |= 1ull << 63;
#pragma unroll
    for (int i = 1; i < ND; ++i) {
      if (((j0 >> sh) & ((1 << CCTile<ND>::L[i]) - 1)) > 0) {
        const int d = 1 << sh;
        int below[kSeg];
#pragma unroll
        for (int q = 0; q < kSeg; ++q) below[q] = s_lab[pd(j0 + q - d)];
#pragma unroll
        for (int q = 0; q < kSeg; ++q) {
          const int l = own[q];
          if (l < 0 || below[q] != l) continue;
          if (q > 0 && own[q - 1] == l && below[q - 1] == l) continue;  // same pair of runs
          todo |= 1ull << (16 * (i - 1) + q);
        }
      }
      sh += CCTile<ND>::L[i];
    }
    while (todo) {
      const int t = (int)__builtin_ctzll(todo);
      todo &= todo - 1;
      int a, c;
      if (t == 63) {
        a = j0 - 1;
        c = j0;
      } else {
        const int i = t >> 4;  // axis - 1
        int dsh = CCTile<ND>::L[0];
#pragma unroll
        for (int k = 1; k < ND - 1; ++k) dsh += k <= i ? CCTile<ND>::L[k] : 0;
        c = j0 + (t & 15);
        a = c - (1 << dsh);
      }
      unite_local(s_par, a, c);
    }
  }
  __syncthreads();
  int rt[kSeg];  // local root of each voxel of the segment
  {
    // each run's first voxel finds its root (one find per run, taken one by
    // one as above); the other voxels of the run take it from there
    uint32_t m = starts;
    while (m) {
      const int q = (int)__builtin_ctz(m);
      m &= m - 1;
      s_par[pd(j0 + q)] = find_local(s_par, j0 + q);
    }
    int cur = 0;
#pragma unroll
    for (int q = 0; q < kSeg; ++q) {
      if (starts & (1u << q)) cur = s_par[pd(j0 + q)];
      rt[q] = own[q] < 0 ? -1 : cur;  // voxels outside the image: -1
    }
  }
  __syncthreads();
  // labels are no longer needed: the label words become the size counters,
  // and every voxel's parent its local root
#pragma unroll
  for (int q = 0; q < kSeg; ++q) {
    s_par[pd(j0 + q)] = rt[q];
    s_size[pd(j0 + q)] = 0;
  }
  __syncthreads();
  {  // sizes: one atomic per run of equal roots
    int cur = -1, n = 0;
#pragma unroll
    for (int q = 0; q < kSeg; ++q) {
      if (rt[q] < 0) continue;
      if (rt[q] != cur) {
        if (n) atomicAdd(&s_size[pd(cur)], n);
        cur = rt[q];
        n = 0;
      }
      ++n;
    }
    if (n) atomicAdd(&s_size[pd(cur)], n);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kSeg; ++q) {
    const int j = threadIdx.x + q * kThreads;
    const int r = s_par[pd(j)];
    if (r < 0) continue;
    bool in;
    const int v = ti.at(g, j, in);
    const int gr = ti.at(g, r, in);
    b.parent[v] = gr;
    b.size[v] = s_size[pd(j)];  // non-zero exactly at local roots
  }
  // the first and last columns' local roots, as whole lines
  for (int t = threadIdx.x; t < 2 * xcol<ND>(); t += kThreads) {
    const int c = t / xcol<ND>(), f = t % xcol<ND>();
    const int j = (f << XL) + c * (XE - 1), r = s_par[pd(j)];
    bool in;
    xf[(2 * c + 1) * xcol<ND>() + f] = r < 0 ? -1 : ti.at(g, r, in);
  }
}

// Unions across the low face x_i = o_i of every tile, on the global parents.
// The faces of a tile are numbered one after the other (a wave stays within
// one face) and walked with the first other axis fastest, one voxel per lane;
// a pair equal to the pair one step before it along that axis (same label
// on both sides) is already joined through it, since each side's pair of
// voxels lies in one local component, so only the first pair of each such
// overlap unites.  All label and parent loads of a thread are issued before
// its unions, which are then taken one by one.
template <int ND>
struct Faces {
  static constexpr int nf(int i) { return kTileVox >> CCTile<ND>::L[i]; }
  static constexpr int total() {
    int t = 0;
    for (int i = 0; i < ND; ++i) t += nf(i);
    return t;
  }
  static constexpr int kItems = (total() + kThreads - 1) / kThreads;
};

template <int ND>
__global__ void __launch_bounds__(kThreads)
cc_faces_kernel(Geo g, const int32_t* __restrict__ labels, CCBuf b) {
  const TileIndex<ND> ti(g, blockIdx.x);
  constexpr int K = Faces<ND>::kItems;
  const int32_t* xf = b.xface + (int64_t)blockIdx.x * xface_ints<ND>();
  int v[K], u[K], lv[K], lu[K], ax[K], f[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    int F = (int)threadIdx.x + k * kThreads;
    int i = 0;
    while (i < ND - 1 && F >= Faces<ND>::nf(i)) F -= Faces<ND>::nf(i++);
    bool in = F < Faces<ND>::nf(i);
    int r = F, vi = ti.base, du = 0;
#pragma unroll
    for (int a = 0; a < ND; ++a) {
      int xa = 0;
      if (a != i) {
        xa = r & ((1 << CCTile<ND>::L[a]) - 1);
        r >>= CCTile<ND>::L[a];
      } else {
        in = in && ti.o[a] > 0;
        du = a == 0 ? 1 : ti.st[a];
      }
      in = in && ti.o[a] + xa < g.n[a];
      vi += a == 0 ? xa : xa * ti.st[a];
    }
    ax[k] = in ? i : -1;
    f[k] = F;
    v[k] = vi;
    u[k] = vi - du;
    if (i == 0) {
      // across axis 0: this tile's first column and the last of the tile
      // before it, from their compact copies
      lv[k] = in ? xf[F] : -1;
      lu[k] = in ? xf[2 * xcol<ND>() - xface_ints<ND>() + F] : -2;
    } else {
      lv[k] = in ? labels[vi] : -1;
      lu[k] = in ? labels[vi - du] : -2;
    }
  }
  uint32_t need = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    // the pair one step before along the fastest face axis (the lane before)
    const int pv = __shfl_up(lv[k], 1, 64), pu = __shfl_up(lu[k], 1, 64);
    const int i = ax[k];
    const int ea = 1 << CCTile<ND>::L[i == 0 ? 1 : 0];  // extent of the fastest face axis
    const bool first = f[k] % ea == 0 || pv != lv[k] || pu != lu[k];
    if (i >= 0 && lu[k] == lv[k] && first) need |= 1u << k;
  }
  int pa[K], pb[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const bool n = need & (1u << k);
    if (ax[k] == 0) {
      pa[k] = n ? xf[3 * xcol<ND>() - xface_ints<ND>() + f[k]] : 0;
      pb[k] = n ? xf[xcol<ND>() + f[k]] : 0;
    } else {
      pa[k] = n ? b.parent[u[k]] : 0;
      pb[k] = n ? b.parent[v[k]] : 0;
    }
  }
  while (need) {
    const int k = (int)__builtin_ctz(need);
    need &= need - 1;
    int a = pa[0], c = pb[0];
#pragma unroll
    for (int k2 = 1; k2 < K; ++k2) {
      if (k == k2) {
        a = pa[k2];
        c = pb[k2];
      }
    }
    unite_roots(b.parent, a, c);
  }
}

// Global roots, per tile: each local root (local size > 0) finds its root
// after the face unions and adds its size there; every other voxel of the
// tile points at a local root of the tile, whose global root it then takes
// from LDS.
template <int ND>
__global__ void __launch_bounds__(kThreads, 5)
cc_flatten_kernel(Geo g, CCBuf b) {
  __shared__ int s_root[kTileVox];  // global root, at the local roots' entries
  const TileIndex<ND> ti(g, xcd_block());
  float inv[ND];
  for (int i = 0; i < ND; ++i) inv[i] = 1.0f / (float)ti.st[i];
  // parents, sizes and indices of this thread's voxels, all loads in flight at
  // once; cur[q] then walks a linked local root's chain and otherwise stays
  // the voxel's parent
  int sz[kSeg], cur[kSeg], vq[kSeg];
  uint32_t inm = 0, lr = 0, lk = 0;  // bit q: inside the image / a local root / one linked
#pragma unroll
  for (int q = 0; q < kSeg; ++q) {
    bool in;
    vq[q] = ti.at(g, threadIdx.x + q * kThreads, in);
    sz[q] = in ? b.size[vq[q]] : 0;
    cur[q] = in ? b.parent[vq[q]] : -1;
    inm |= in ? 1u << q : 0u;
  }
#pragma unroll
  for (int q = 0; q < kSeg; ++q) {
    lr |= sz[q] > 0 ? 1u << q : 0u;
    lk |= (sz[q] > 0 && cur[q] != vq[q]) ? 1u << q : 0u;
  }
#pragma unroll
  for (int q = 0; q < kSeg; ++q)  // the linked roots' sizes wait in their LDS entries
    if (lk & (1u << q)) s_root[threadIdx.x + q * kThreads] = sz[q];
  // the linked local roots' chains, all of a thread's a step at a time, until
  // each reaches a node that is its own parent
  uint32_t todo = lk;
  while (todo) {
    int nx[kSeg];
#pragma unroll
    for (int q = 0; q < kSeg; ++q) nx[q] = (todo & (1u << q)) ? b.parent[cur[q]] : cur[q];
#pragma unroll
    for (int q = 0; q < kSeg; ++q) {
      todo &= nx[q] == cur[q] ? ~(1u << q) : ~0u;
      cur[q] = nx[q];
    }
  }
#pragma unroll
  for (int q = 0; q < kSeg; ++q) {
    const int j = threadIdx.x + q * kThreads;
    if (lk & (1u << q)) atomicAdd(&b.size[cur[q]], s_root[j]);  // a local root joins its global root
    if (lr & (1u << q)) s_root[j] = cur[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kSeg; ++q) {
    if (!(inm & (1u << q))) continue;
    int r = cur[q];
    if (!(lr & (1u << q))) {
      // the local root's tile-local index from its offset to the tile origin:
      // the FP32 quotient estimate is off by at most one (each quotient is
      // below the tile extent), and the remainder it leaves lies in
      // [-stride, 2 stride) and is at most the offset, so it fits in 32 bits
      int d = cur[q] - ti.base;
      int lj = 0, sh = 0;
      int xq[ND];
      for (int i = ND - 1; i >= 1; --i) {
        int qi = (int)((float)d * inv[i]);
        int rem = (int)((uint32_t)d - (uint32_t)qi * (uint32_t)ti.st[i]);
        const bool lo = rem < 0, hi = rem >= ti.st[i];
        qi += lo ? -1 : (hi ? 1 : 0);
        rem += lo ? ti.st[i] : (hi ? -ti.st[i] : 0);
        xq[i] = qi;
        d = rem;
      }
      xq[0] = d;
      for (int i = 0; i < ND; ++i) {
        lj |= xq[i] << sh;
        sh += CCTile<ND>::L[i];
      }
      r = s_root[lj];
    }
    b.parent[vq[q]] = r;
  }
}

// First pass: the component of label k at the rounded centre k, or the first
// voxel of label k in raster order within floor(S_i / 2) of it.  Each lane
// takes one cluster and checks its rounded centre; the wave then reads the
// window of every cluster whose centre missed, 64 voxels at a time in raster
// order, and a ballot finds the first of label k.
__global__ void __launch_bounds__(kThreads)
cc_first_kernel(Geo g, const double* __restrict__ cen, const int32_t* __restrict__ labels, CCBuf b) {
  const int lane = threadIdx.x % 64;
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool in = k < g.K;
  int p[kMaxDim];
  int64_t pl = 0;
  if (in) {
    const double* row = cen + k * g.row;
    for (int i = 0; i < g.nd; ++i) {
      const double c = i < g.nd_out ? row[g.C + i] : 0.0;
      double f = floor(c + 0.5);
      f = fmin(fmax(f, 0.0), (double)(g.n[i] - 1));
      p[i] = isfinite(c) ? (int)f : 0;
      pl += p[i] * g.st[i];
    }
  }
  int64_t seed = in && labels[pl] == (int32_t)k ? pl : -1;
  // the clusters of this wave whose rounded centre holds another label
  uint64_t miss = __ballot(in && seed < 0);
  while (miss) {
    const int j = (int)__builtin_ctzll(miss);
    miss &= miss - 1;
    const int kj = __shfl((int)k, j, 64);
    int lo[kMaxDim], w[kMaxDim];
    int64_t nwin = 1;
    for (int i = 0; i < g.nd; ++i) {
      const int pi = __shfl(i < kMaxDim ? p[i] : 0, j, 64);
      const int h = g.S[i] / 2;
      lo[i] = max(pi - h, 0);
      w[i] = min(pi + h, g.n[i] - 1) - lo[i] + 1;
      nwin *= w[i];
    }
    int64_t found = -1;
    for (int64_t t0 = 0; t0 < nwin; t0 += 64) {
      const int64_t t = t0 + lane;
      bool hit = false;
      int64_t v = 0;
      if (t < nwin) {
        int64_t r = t;
        for (int i = 0; i < g.nd; ++i) {
          v += (int64_t)(lo[i] + (int)(r % w[i])) * g.st[i];
          r /= w[i];
        }
        hit = labels[v] == kj;
      }
      const uint64_t m = __ballot(hit);
      if (m) {
        found = (int64_t)__shfl((long long)v, (int)__builtin_ctzll(m), 64);
        break;
      }
    }
    if (lane == j) seed = found;
  }
  if (seed < 0) return;
  const int r = b.parent[seed];
  // a component holds one label, so no other cluster marks it
  const int sz = b.size[r];
  if (sz >= 0 && 4 * (int64_t)sz > g.prodS) b.size[r] = ~sz;
}


// Wave w of the workgroup numbered x (XCD-ordered, as xcd_block) ranks chunk
// c = 4x + w: voxels [1024 c, 1024 c + 1024) as 16 coalesced rows of 64, in
// raster order.
__device__ __forceinline__ int64_t wave_chunk() {
  return (int64_t)xcd_block() * kWaves + threadIdx.x / 64;
}

constexpr int kRows = kChunk / 64;

// Which of this lane's voxels of chunk c (one per row) are roots, and large
// open ones; all loads of a kind in flight at once.
__device__ __forceinline__ void chunk_roots(const Geo& g, const CCBuf& b, int64_t c, bool* root,
                                            bool* large, bool* fin) {
  const int lane = threadIdx.x % 64;
  int par[kRows];
#pragma unroll
  for (int q = 0; q < kRows; ++q) {
    const int64_t v = c * kChunk + q * 64 + lane;
    par[q] = v < g.N ? b.parent[v] : -1;
  }
  int sz[kRows];
#pragma unroll
  for (int q = 0; q < kRows; ++q) {
    const int64_t v = c * kChunk + q * 64 + lane;
    root[q] = par[q] == (int32_t)v;
    sz[q] = root[q] ? b.size[v] : 0;
  }
#pragma unroll
  for (int q = 0; q < kRows; ++q) {
    fin[q] = sz[q] < 0;  // marked final by the first pass
    large[q] = root[q] && !fin[q] && 4 * (int64_t)sz[q] > g.prodS;
  }
}

// Roots and large open roots per chunk.
__global__ void __launch_bounds__(kThreads) cc_count_kernel(Geo g, CCBuf b, int64_t nchunks) {
  const int lane = threadIdx.x % 64;
  const int64_t c = wave_chunk();
  if (c >= nchunks) return;
  bool root[kRows], large[kRows], fin[kRows];
  chunk_roots(g, b, c, root, large, fin);
  int nl = 0, nr = 0;
#pragma unroll
  for (int q = 0; q < kRows; ++q) {
    nr += (int)__popcll(__ballot(root[q]));
    nl += (int)__popcll(__ballot(large[q]));
  }
  if (lane == 0) {
    b.part[c] = nl;
    b.rpart[c] = nr;
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

// Exclusive scan of both chunk count arrays, in three steps: each block
// scans kScanBlock counts in place and leaves its total ...
__global__ void __launch_bounds__(kThreads) cc_scan_local_kernel(CCBuf b, int64_t n) {
  __shared__ int sh[kThreads];
  for (int which = 0; which < 2; ++which) {
    int32_t* a = which ? b.rpart : b.part;
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
    int v[kScanPer];
    int sum = 0;
    for (int j = 0; j < kScanPer; ++j) {
      v[j] = base + j < n ? a[base + j] : 0;
      sum += v[j];
    }
    int total;
    int off = block_exclusive_scan(sum, sh, &total);
    for (int j = 0; j < kScanPer; ++j) {
      if (base + j < n) a[base + j] = off;
      off += v[j];
    }
    if (threadIdx.x == 0) (which ? b.brpart : b.bpart)[blockIdx.x] = total;
  }
}

// ... one block scans the block totals (grand totals to b.total, b.nroots) ...
__global__ void __launch_bounds__(kThreads) cc_scan_blocks_kernel(CCBuf b, int nblocks) {
  __shared__ int sh[kThreads];
  for (int which = 0; which < 2; ++which) {
    int32_t* p = which ? b.brpart : b.bpart;
    int carry = 0;
    for (int b0 = 0; b0 < nblocks; b0 += kThreads) {
      const int i = b0 + threadIdx.x;
      const int v = i < nblocks ? p[i] : 0;
      int total;
      const int ex = block_exclusive_scan(v, sh, &total);
      if (i < nblocks) p[i] = ex + carry;
      carry += total;
    }
    if (threadIdx.x == 0) *(which ? b.nroots : b.total) = carry;
  }
}

// ... and every count gets its block's offset.
__global__ void cc_scan_add_kernel(CCBuf b, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  b.part[i] += b.bpart[i / kScanBlock];
  b.rpart[i] += b.brpart[i / kScanBlock];
}

// Label of every root: final roots keep their label, large open roots get
// K + rank, the origin keeps its label, other small roots store a link
// -(root of their predecessor) - 1 to be resolved.  The roots are listed in
// raster order as they go.
__global__ void __launch_bounds__(kThreads)
cc_root_labels_kernel(Geo g, const int32_t* __restrict__ labels, CCBuf b, int64_t nchunks) {
  const int lane = threadIdx.x % 64;
  const int64_t c = wave_chunk();
  if (c >= nchunks) return;
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  int rl = b.part[c], rr = b.rpart[c];
  bool rootq[kRows], largeq[kRows], finq[kRows];
  chunk_roots(g, b, c, rootq, largeq, finq);
  // axis-0 coordinates from the chunk's first one, one division per chunk:
  // rows at least a chunk long wrap at most once within it
  const uint32_t n0 = (uint32_t)g.n[0];
  const bool one_wrap = n0 >= (uint32_t)kChunk;
  const uint32_t x0 = one_wrap ? (uint32_t)(c * kChunk) % n0 : 0u;
#pragma unroll
  for (int q = 0; q < kRows; ++q) {
    const int64_t v = c * kChunk + q * 64 + lane;
    const bool root = rootq[q], large = largeq[q];
    uint32_t x = x0 + (uint32_t)(q * 64 + lane);
    x -= x >= n0 ? n0 : 0u;
    const uint64_t mr = __ballot(root), ml = __ballot(large);
    if (root) {
      int lab;
      if (finq[q]) {
        lab = labels[v];
      } else if (large) {
        lab = (int)(g.K + rl + __popcll(ml & lt));
      } else if (v == 0) {
        lab = labels[0];
      } else {
        // the face neighbour before v: along the first axis where v is not
        // at the low border (indices fit 32 bits)
        uint32_t r = (uint32_t)v;
        int64_t pred = one_wrap && x != 0 ? v - g.st[0] : -1;
        for (int i = 0; i < g.nd && pred < 0; ++i) {
          const uint32_t q2 = r / (uint32_t)g.n[i];
          if (r - q2 * (uint32_t)g.n[i] > 0) pred = v - g.st[i];
          r = q2;
        }
        lab = -(b.parent[pred]) - 1;
      }
      b.newlab[v] = lab;
      b.roots[rr + __popcll(mr & lt)] = (int32_t)v;
    }
    rl += (int)__popcll(ml);
    rr += (int)__popcll(mr);
  }
}

// Small roots take the label their link leads to.  On a fragmented volume a
// link most often leads to the root just before in raster order (fragments
// chain back along the rows) and chains run to tens of links; shortcuts come
// from entries already resolved on the way.  The root list is cut into units
// of 1024 consecutive roots,
// and each XCD walks one contiguous eighth of the units in order: a link
// leads a few rows back, to roots its own XCD has just resolved.  Each
// thread follows four chains 256 roots apart.  Every root's entry is written
// once, by its own thread, from link to label, so any entry read on the way
// is valid.  The grid is a multiple of 8 workgroups.
__global__ void __launch_bounds__(kThreads) cc_resolve_kernel(CCBuf b) {
  constexpr int U = 4;
  const int n = *b.nroots;
  const int W = (n + kThreads * U - 1) / (kThreads * U);
  const int x = (int)(blockIdx.x % 8), per = (int)(gridDim.x / 8);
  const int ue = (int)((int64_t)W * (x + 1) / 8);
  for (int u = (int)((int64_t)W * x / 8) + (int)(blockIdx.x / 8); u < ue; u += per) {
    const int i0 = u * kThreads * U + (int)threadIdx.x;
    int v[U], lab[U];
#pragma unroll
    for (int k = 0; k < U; ++k) v[k] = i0 + k * kThreads < n ? b.roots[i0 + k * kThreads] : -1;
#pragma unroll
    for (int k = 0; k < U; ++k) lab[k] = v[k] >= 0 ? b.newlab[v[k]] : 0;
    int w[U];
#pragma unroll
    for (int k = 0; k < U; ++k) w[k] = lab[k] < 0 ? b.newlab[-lab[k] - 1] : 0;
#pragma unroll
    for (int k = 0; k < U; ++k) {
      if (lab[k] >= 0) continue;
      int lk = w[k];
      while (lk < 0) lk = b.newlab[-lk - 1];
      b.newlab[v[k]] = lk;
    }
  }
}

// Every voxel takes the label of its component's root, tile by tile (the
// tiles of the local union-find): the root of a fragment lies in or near its
// tile, so a tile's gathers fall on a few lines, where raster order would
// reach planes back for them.  Each thread's 16 gathers are in flight at
// once.
template <int ND>
__global__ void __launch_bounds__(kThreads)
cc_relabel_kernel(Geo g, int32_t* __restrict__ labels, CCBuf b, int32_t* n_labels) {
  const TileIndex<ND> ti(g, blockIdx.x);
  int v[kSeg], p[kSeg];
#pragma unroll
  for (int q = 0; q < kSeg; ++q) {
    bool in;
    v[q] = ti.at(g, threadIdx.x + q * kThreads, in);
    p[q] = in ? b.parent[v[q]] : -1;
  }
#pragma unroll
  for (int q = 0; q < kSeg; ++q) p[q] = p[q] >= 0 ? b.newlab[p[q]] : -1;
#pragma unroll
  for (int q = 0; q < kSeg; ++q)
    if (p[q] >= 0) labels[v[q]] = p[q];
  if (n_labels && blockIdx.x == 0 && threadIdx.x == 0) *n_labels = (int32_t)(g.K + *b.total);
}

}  // namespace

int64_t cc_xface_ints(const Geo& g) {
  int64_t ntiles = 1;
  for (int i = 0; i < g.nd; ++i) {
    const int L = g.nd == 2 ? CCTile<2>::L[i] : g.nd == 3 ? CCTile<3>::L[i] : CCTile<4>::L[i];
    ntiles *= (g.n[i] + (1 << L) - 1) >> L;
  }
  const int w = g.nd == 2 ? xface_ints<2>() : g.nd == 3 ? xface_ints<3>() : xface_ints<4>();
  return ntiles * w;
}

hipError_t launch_connectivity(const Geo& g, const double* cen, int32_t* labels, const CCBuf& b,
                               int32_t* n_labels_dev, hipStream_t s) {
  const int64_t nchunks = (g.N + kChunk - 1) / kChunk;
  const int nwg = (int)((nchunks + kWaves - 1) / kWaves);
  const int nsb = (int)((nchunks + kScanBlock - 1) / kScanBlock);
  int ntiles = 1;
  for (int i = 0; i < g.nd; ++i) {
    const int L = g.nd == 2 ? CCTile<2>::L[i] : g.nd == 3 ? CCTile<3>::L[i] : CCTile<4>::L[i];
    ntiles *= (g.n[i] + (1 << L) - 1) >> L;
  }
  switch (g.nd) {
    case 2:
      cc_local_kernel<2><<<ntiles, kThreads, 0, s>>>(g, labels, b);
      cc_faces_kernel<2><<<ntiles, kThreads, 0, s>>>(g, labels, b);
      cc_flatten_kernel<2><<<ntiles, kThreads, 0, s>>>(g, b);
      break;
    case 3:
      cc_local_kernel<3><<<ntiles, kThreads, 0, s>>>(g, labels, b);
      cc_faces_kernel<3><<<ntiles, kThreads, 0, s>>>(g, labels, b);
      cc_flatten_kernel<3><<<ntiles, kThreads, 0, s>>>(g, b);
      break;
    default:
      cc_local_kernel<4><<<ntiles, kThreads, 0, s>>>(g, labels, b);
      cc_faces_kernel<4><<<ntiles, kThreads, 0, s>>>(g, labels, b);
      cc_flatten_kernel<4><<<ntiles, kThreads, 0, s>>>(g, b);
      break;
  }
  cc_first_kernel<<<blocks_for(g.K), kThreads, 0, s>>>(g, cen, labels, b);
  cc_count_kernel<<<nwg, kThreads, 0, s>>>(g, b, nchunks);
  cc_scan_local_kernel<<<nsb, kThreads, 0, s>>>(b, nchunks);
  cc_scan_blocks_kernel<<<1, kThreads, 0, s>>>(b, nsb);
  cc_scan_add_kernel<<<blocks_for(nchunks), kThreads, 0, s>>>(b, nchunks);
  cc_root_labels_kernel<<<nwg, kThreads, 0, s>>>(g, labels, b, nchunks);
  const int64_t units = (g.N + 4 * kThreads - 1) / (4 * kThreads);
  cc_resolve_kernel<<<(int)((std::min<int64_t>(units, 1 << 16) + 7) / 8 * 8), kThreads, 0, s>>>(b);
  switch (g.nd) {
    case 2: cc_relabel_kernel<2><<<ntiles, kThreads, 0, s>>>(g, labels, b, n_labels_dev); break;
    case 3: cc_relabel_kernel<3><<<ntiles, kThreads, 0, s>>>(g, labels, b, n_labels_dev); break;
    default: cc_relabel_kernel<4><<<ntiles, kThreads, 0, s>>>(g, labels, b, n_labels_dev); break;
  }
  return hipGetLastError();
}

}  // namespace sslic
