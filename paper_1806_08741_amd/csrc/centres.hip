// centres.hip -- seeding (Sec. 2.2 / 3.1 stage 1), the per-iteration centre
// table and S-bin index, the mean update's final division and the residual
// (Sec. 3.1 stage 2, Sec. 3.2).
#include <cmath>

#include "sslic_internal.h"

namespace sslic {

namespace {

constexpr int kThreads = 256;

struct TileDims {
  int T[kMaxDim];
};

inline int blocks_for(int64_t n, int per = kThreads) { return (int)((n + per - 1) / per); }

template <typename T>
__global__ void fill_kernel(T* p, T v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

template <typename T>
hipError_t fill(T* p, T v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int nb = (int)std::min<int64_t>(blocks_for(n), 8192);
  fill_kernel<T><<<nb, kThreads, 0, s>>>(p, v, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Seeding: grid seed, then the lowest squared Frobenius norm of the central
// difference Jacobian among the in-image 3^n neighbours, visited in raster
// order (offset along axis 0 fastest) and replaced only when strictly lower.

template <typename T>
__device__ __forceinline__ int64_t grad_int(const Geo& g, const T* img, const int* p, int nd) {
  int64_t base = 0;
  for (int i = 0; i < nd; ++i) base += p[i] * g.st[i];
  int64_t acc = 0;
  for (int c = 0; c < g.C; ++c) {
    for (int i = 0; i < nd; ++i) {
      int pp = min(p[i] + 1, g.n[i] - 1), pm = max(p[i] - 1, 0);
      int64_t a = (int64_t)img[(base + (int64_t)(pp - p[i]) * g.st[i]) * g.C + c];
      int64_t b = (int64_t)img[(base + (int64_t)(pm - p[i]) * g.st[i]) * g.C + c];
      acc += (a - b) * (a - b);
    }
  }
  return acc;
}

__device__ __forceinline__ double grad_flt(const Geo& g, const float* img, const int* p, int nd) {
#pragma clang fp contract(off)
  int64_t base = 0;
  for (int i = 0; i < nd; ++i) base += p[i] * g.st[i];
  double acc = 0.0;
  for (int c = 0; c < g.C; ++c) {
    for (int i = 0; i < nd; ++i) {
      int pp = min(p[i] + 1, g.n[i] - 1), pm = max(p[i] - 1, 0);
      double a = (double)img[(base + (int64_t)(pp - p[i]) * g.st[i]) * g.C + c];
      double b = (double)img[(base + (int64_t)(pm - p[i]) * g.st[i]) * g.C + c];
      double d = a - b;
      acc = acc + d * d;
    }
  }
  return acc;
}

template <typename T, typename G>
__device__ __forceinline__ G grad_any(const Geo& g, const T* img, const int* p, int nd) {
  if constexpr (std::is_same<T, float>::value) return grad_flt(g, img, p, nd);
  else return grad_int<T>(g, img, p, nd);
}

template <typename T>
__device__ __forceinline__ void seed_one(const Geo& g, const T* __restrict__ img, double* __restrict__ cen,
                                         int64_t k) {
  using G = typename std::conditional<std::is_same<T, float>::value, double, int64_t>::type;
  const int nd = g.nd;
  int s[kMaxDim], q[kMaxDim], best[kMaxDim];
  int64_t r = k;
  for (int i = 0; i < nd; ++i) {
    int64_t j = r % g.Ka[i];
    r /= g.Ka[i];
    s[i] = (int)(((2 * j + 1) * (int64_t)g.n[i]) / (2 * (int64_t)g.Ka[i]));
    best[i] = s[i];
  }
  G gb = grad_any<T, G>(g, img, s, nd);
  int n3 = 1;
  for (int i = 0; i < nd; ++i) n3 *= 3;
  for (int o = 0; o < n3; ++o) {
    int oo = o;
    bool inside = true;
    for (int i = 0; i < nd; ++i) {
      q[i] = s[i] + (oo % 3) - 1;
      oo /= 3;
      inside = inside && q[i] >= 0 && q[i] < g.n[i];
    }
    if (!inside) continue;
    G v = grad_any<T, G>(g, img, q, nd);
    if (v < gb) {
      gb = v;
      for (int i = 0; i < nd; ++i) best[i] = q[i];
    }
  }
  int64_t bl = 0;
  for (int i = 0; i < nd; ++i) bl += best[i] * g.st[i];
  double* row = cen + k * g.row;
  for (int c = 0; c < g.C; ++c) row[c] = (double)img[bl * g.C + c];
  for (int i = 0; i < g.nd_out; ++i) row[g.C + i] = (double)best[i];
}

template <typename T>
__global__ void seed_kernel(Geo g, const T* __restrict__ img, double* __restrict__ cen) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= g.K) return;
  seed_one<T>(g, img, cen, k);
}

// The same search with ND and C fixed at compile time: the values the
// 3^ND gradients read (the clamped voxels s + d with every |d_i| <= 1 but
// at most one |d_i| = 2) are loaded first, all at once, then the gradients
// are formed from registers in the order above (c outer, axis inner).
constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

template <typename T, int ND, int CC>
__global__ void __launch_bounds__(kThreads)
seed_fixed_kernel(Geo g, const T* __restrict__ img, double* __restrict__ cen) {
  using G = typename std::conditional<std::is_same<T, float>::value, double, int64_t>::type;
  constexpr int P5 = ipow(5, ND), N3 = ipow(3, ND);
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= g.K) return;
  int s[ND];
  {
    int64_t r = k;
    for (int i = 0; i < ND; ++i) {
      const int64_t j = r % g.Ka[i];
      r /= g.Ka[i];
      s[i] = (int)(((2 * j + 1) * (int64_t)g.n[i]) / (2 * (int64_t)g.Ka[i]));
    }
  }
  // clamped offsets along each axis, and their contribution to the address
  int64_t off[ND][5];
#pragma unroll
  for (int i = 0; i < ND; ++i)
#pragma unroll
    for (int d = -2; d <= 2; ++d) off[i][d + 2] = (int64_t)min(max(s[i] + d, 0), g.n[i] - 1) * g.st[i];
  T P[P5][CC];
#pragma unroll
  for (int e = 0; e < P5; ++e) {
    int twos = 0;
    int64_t a = 0;
#pragma unroll
    for (int i = 0, r = e; i < ND; ++i, r /= 5) {
      twos += (r % 5 == 0 || r % 5 == 4) ? 1 : 0;
      a += off[i][r % 5];
    }
    if (twos > 1) continue;  // no gradient reads it
#pragma unroll
    for (int c = 0; c < CC; ++c) P[e][c] = img[a * CC + c];
  }
  auto grad = [&](int o) {  // o: index of the offset in {-1,0,1}^ND, axis 0 fastest
    int pe = 0;
#pragma unroll
    for (int i = 0, r = o, m = 1; i < ND; ++i, r /= 3, m *= 5) pe += (r % 3 + 1) * m;
    G acc = 0;
#pragma unroll
    for (int c = 0; c < CC; ++c) {
#pragma unroll
      for (int i = 0, m = 1; i < ND; ++i, m *= 5) {
        const G a = (G)P[pe + m][c], b = (G)P[pe - m][c];
        if constexpr (std::is_same<G, double>::value) {
#pragma clang fp contract(off)
          const double d = a - b;
          acc = acc + d * d;
        } else {
          acc += (a - b) * (a - b);
        }
      }
    }
    return acc;
  };
  constexpr int kSelf = (N3 - 1) / 2;  // offset 0 on every axis
  G gb = grad(kSelf);
  int best = kSelf;
#pragma unroll
  for (int o = 0; o < N3; ++o) {
    bool inside = true;
#pragma unroll
    for (int i = 0, r = o; i < ND; ++i, r /= 3) {
      const int q = s[i] + r % 3 - 1;
      inside = inside && q >= 0 && q < g.n[i];
    }
    const G v = grad(o);
    if (inside && v < gb) {
      gb = v;
      best = o;
    }
  }
  int64_t bl = 0;
  int bq[ND];
#pragma unroll
  for (int i = 0, r = best; i < ND; ++i, r /= 3) {
    bq[i] = s[i] + r % 3 - 1;
    bl += (int64_t)bq[i] * g.st[i];
  }
  double* row = cen + k * g.row;
  for (int c = 0; c < CC; ++c) row[c] = (double)img[bl * CC + c];
  for (int i = 0; i < g.nd_out; ++i) row[CC + i] = (double)bq[i];
}

// Calls f(descriptor) for the lanes with `in`.  A wave whose lanes all work
// on one image (the common case: images hold many clusters) reads that
// image's descriptor through scalar loads; a mixed wave reads it per lane.
template <class F>
__device__ __forceinline__ void with_image(const BImg* __restrict__ imgs, int im, bool in, F f) {
  const int first = __builtin_amdgcn_readfirstlane(im);
  if (__all(in && im == first)) {
    f(imgs[first]);
  } else if (in) {
    f(imgs[im]);
  }
}

// clusters [k0, k1) of a batch, all of one pixel type
template <typename T>
__global__ void seed_batch_kernel(const BImg* __restrict__ imgs, const int32_t* __restrict__ cl_img,
                                  int64_t k0, int64_t k1) {
  const int64_t gk = k0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool in = gk < k1;
  with_image(imgs, in ? cl_img[gk] : -1, in, [&](const BImg& d) {
    seed_one<T>(d.g, reinterpret_cast<const T*>(d.img), d.cen, gk - d.koff);
  });
}

__global__ void grid_labels_kernel(Geo g, int32_t* __restrict__ labels) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < g.N;
       v += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = v, k = 0, kst = 1;
    for (int i = 0; i < g.nd; ++i) {
      int64_t x = r % g.n[i];
      r /= g.n[i];
      k += (x * g.Ka[i] / g.n[i]) * kst;
      kst *= g.Ka[i];
    }
    labels[v] = (int32_t)k;
  }
}

// ---------------------------------------------------------------------------
// Centre table and bins.  The window of centre k on axis i is the integer
// range [ceil(c - S), floor(c + S)], computed in FP64 exactly as the closed
// condition |x - c| <= S reads.  Bin b = floor(lo / S) + 1 (clamped) is within
// one bin of the bin of every voxel the window holds, so a voxel finds every
// centre that covers it among the 3^n bins around its own.

__device__ __forceinline__ int floordiv(int a, int b) {
  int q = a / b;
  return (q * b > a) ? q - 1 : q;
}

__device__ __forceinline__ void prep_one(const Geo& g, const double* row, int64_t k, const Iter& it,
                                         int64_t binoff = 0) {
  float* rec = it.ctab + k * g.rs;
  int32_t* irec = reinterpret_cast<int32_t*>(rec);
  for (int c = 0; c < g.C; ++c) rec[c] = (float)row[c];
  int64_t bin = 0;
  for (int i = 0; i < g.nd; ++i) {
    double ci = i < g.nd_out ? row[g.C + i] : 0.0;
    rec[g.C + i] = (float)(ci * g.swd[i]);
    int lo, hi;
    if (isfinite(ci)) {
      double l = ceil(ci - (double)g.S[i]);
      double h = floor(ci + (double)g.S[i]);
      l = fmin(fmax(l, -1073741824.0), 1073741824.0);
      h = fmin(fmax(h, -1073741824.0), 1073741824.0);
      lo = (int)l;
      hi = (int)h;
    } else {
      lo = 1073741824;
      hi = -1073741824;
    }
    irec[rec_lo(g.C, g.nd) + i] = lo;
    irec[rec_hi(g.C, g.nd) + i] = hi;
    int b = floordiv(lo, g.S[i]) + 1;
    b = min(max(b, 0), g.nb[i] - 1);
    bin += b * g.bst[i];
  }
  irec[rec_k(g.C, g.nd)] = (int32_t)k;
  it.bin_of[k] = (int32_t)(bin + binoff);
  atomicAdd(&it.bin_cnt[bin + binoff], 1);
}

// The image's view of the batch's shared tables: its records and bins at its
// offsets, its own accumulators and tile slots.
__device__ __forceinline__ Iter batch_iter(const BImg& d, float* ctab, int32_t* bin_of,
                                           int32_t* bin_cnt) {
  Iter it{};
  it.ctab = ctab + d.koff * d.g.rs;
  it.bin_of = bin_of + d.koff;
  it.bin_cnt = bin_cnt;
  it.acc = d.a.acc;
  it.accf = d.a.accf;
  it.part = d.a.part;
  it.res_acc = d.res;
  it.done = d.flags;
  it.iters = d.flags + 1;
  return it;
}

__global__ void prep_batch_kernel(const BImg* __restrict__ imgs, const int32_t* __restrict__ cl_img,
                                  int64_t K, float* ctab, int32_t* bin_of, int32_t* bin_cnt) {
  const int64_t gk = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool in = gk < K;
  with_image(imgs, in ? cl_img[gk] : -1, in, [&](const BImg& d) {
    if (d.flags[0]) return;
    const int64_t k = gk - d.koff;
    prep_one(d.g, d.cen + k * d.g.row, k, batch_iter(d, ctab, bin_of, bin_cnt), d.binoff);
  });
}

__global__ void prep_kernel(Geo g, const double* __restrict__ cen, Iter it) {
  if (*it.done) return;
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= g.K) return;
  prep_one(g, cen + k * g.row, k, it);
}

// Exclusive scan of bin counts in blocks of 4096 (16 per thread), then a
// single-block scan of block totals, then the offsets.  The counts are reset
// to zero on the way so they can serve as scatter cursors.
constexpr int kScanPer = 16;
constexpr int kScanBlock = kThreads * kScanPer;

__device__ __forceinline__ int block_exclusive_scan(int v, int* sh, int* total) {
  // sh: kThreads ints.  Hillis-Steele over the block.
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

__global__ void scan_local_kernel(int32_t* __restrict__ cnt, int32_t* __restrict__ out,
                                  int32_t* __restrict__ part, int64_t n, const int32_t* done) {
  if (*done) return;
  __shared__ int sh[kThreads];
  int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
  int v[kScanPer];
  int sum = 0;
  for (int j = 0; j < kScanPer; ++j) {
    int64_t i = base + j;
    v[j] = i < n ? cnt[i] : 0;
    if (i < n) cnt[i] = 0;
    sum += v[j];
  }
  int total;
  int off = block_exclusive_scan(sum, sh, &total);
  for (int j = 0; j < kScanPer; ++j) {
    int64_t i = base + j;
    if (i < n) out[i] = off;
    off += v[j];
  }
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

__global__ void scan_parts_kernel(int32_t* __restrict__ part, int nparts, int32_t* __restrict__ out_last,
                                  const int32_t* done) {
  if (*done) return;
  __shared__ int sh[kThreads];
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
  if (threadIdx.x == 0) *out_last = carry;
}

__global__ void scan_add_kernel(int32_t* __restrict__ out, const int32_t* __restrict__ part, int64_t n,
                                const int32_t* done) {
  if (*done) return;
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] += part[i / kScanBlock];
}

__global__ void scatter_kernel(Geo g, Iter it) {
  if (*it.done) return;
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= g.K) return;
  int b = it.bin_of[k];
  if (b < 0) return;  // a cluster of a finished image (batches)
  int pos = it.bin_start[b] + atomicAdd(&it.bin_cnt[b], 1);
  it.bin_items[pos] = (int32_t)k;
}

// Order each bin's items by cluster index (bins hold a handful of centres)
// and reset the cursors for the next use.
__global__ void binsort_kernel(Geo g, Iter it) {
  if (*it.done) return;
  int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= g.nbins) return;
  int a = it.bin_start[b], e = it.bin_start[b + 1];
  for (int i = a + 1; i < e; ++i) {
    int v = it.bin_items[i];
    int j = i - 1;
    while (j >= a && it.bin_items[j] > v) {
      it.bin_items[j + 1] = it.bin_items[j];
      --j;
    }
    it.bin_items[j + 1] = v;
  }
  it.bin_cnt[b] = 0;
}

// ---------------------------------------------------------------------------
// Update, final step: sums / count in FP64 (correctly rounded, as the oracle),
// the residual term of the cluster, counts out, accumulators reset, and the
// table and bin of the new centre for the next assignment.

__device__ __forceinline__ double warp_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// The reduce step of cluster k at iteration t: accumulators (and, with
// use_part, the tile slots of the tiles its window meets, as the sweep chose
// them, that carry this iteration's tag) -> new centre in FP64, count,
// residual term (e_sum, e_cnt); then the next iteration's record and bin when
// prep_next.  With use_part the accumulators are read (and cleared) only where
// the sweep flagged them; without it they are the only source.
template <int ND, int CC, bool FLT>
__device__ __forceinline__ void finalize_one(const Geo& g, double* __restrict__ cen,
                                             int64_t* __restrict__ counts, const Iter& it,
                                             int64_t k, int t, int prep_next, int use_part,
                                             const int* tdT, int64_t binoff, double& e_sum,
                                             double& e_cnt) {
  constexpr int CM = CC > 0 ? CC : kMaxChan;
  const int C = CC > 0 ? CC : g.C;
  const int F = 1 + ND + C;

    uint64_t si[1 + ND];
    uint64_t sc[CM];
    double sf[CM];
    if (!use_part || it.accf[k]) {
      uint64_t* a = it.acc + k * F;
#pragma unroll
      for (int f = 0; f < 1 + ND; ++f) si[f] = a[f];
      for (int c = 0; c < C; ++c) {
        sc[c] = a[1 + ND + c];
        sf[c] = __longlong_as_double((long long)sc[c]);
      }
      for (int f = 0; f < F; ++f) a[f] = 0;
      if (use_part) it.accf[k] = 0;
    } else {
#pragma unroll
      for (int f = 0; f < 1 + ND; ++f) si[f] = 0;
      for (int c = 0; c < C; ++c) {
        sc[c] = 0;
        sf[c] = 0.0;
      }
    }
    if (use_part) {
      // the slots of the tiles this cluster's window meets (as the sweep chose them)
      const int32_t* irec = reinterpret_cast<const int32_t*>(it.ctab + k * g.rs);
      int lo[ND], hi[ND], t0[ND];
      bool any = true;
#pragma unroll
      for (int i = 0; i < ND; ++i) {
        lo[i] = max(irec[rec_lo(C, ND) + i], 0);
        hi[i] = min(irec[rec_hi(C, ND) + i], g.n[i] - 1);
        any = any && lo[i] <= hi[i];
        t0[i] = lo[i] / tdT[i];
      }
      constexpr int NQ = 1 << ND;
      uint32_t qm = 0;  // the slots of the tiles the window meets
      if (any) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          bool meets = true;
#pragma unroll
          for (int i = 0; i < ND; ++i) {
            if ((q >> i) & 1) meets = meets && (t0[i] + 1) * tdT[i] <= hi[i];
          }
          if (meets) qm |= 1u << q;
        }
      }
      auto add_slot = [&](const uint64_t* w) {
#pragma unroll
        for (int f = 0; f < 1 + ND; ++f) si[f] += w[f];
        for (int c = 0; c < C; ++c) {
          const uint64_t raw = w[1 + ND + c];
          if (FLT) sf[c] += __longlong_as_double((long long)raw);
          else sc[c] += raw;
        }
      };
      if constexpr (ND <= 3) {
        // every meeting slot's words and tag in flight at once, then the
        // slots written this iteration are added in slot order
        constexpr int FW = 1 + ND + CM;
        uint64_t w[NQ][FW + 1];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          if (!((qm >> q) & 1u)) continue;
          const uint64_t* p = it.part + (k * NQ + q) * (F + 1);
          w[q][FW] = p[F];
#pragma unroll
          for (int f = 0; f < 1 + ND; ++f) w[q][f] = p[f];
          for (int c = 0; c < C; ++c) w[q][1 + ND + c] = p[1 + ND + c];
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q)
          if (((qm >> q) & 1u) && w[q][FW] == (uint64_t)(t + 1)) add_slot(w[q]);
      } else {
        for (int q = 0; q < NQ; ++q) {
          if (!((qm >> q) & 1u)) continue;
          const uint64_t* p = it.part + (k * NQ + q) * (F + 1);
          if (p[F] != (uint64_t)(t + 1)) continue;  // not written this iteration
          add_slot(p);
        }
      }
    }
    const uint64_t n = si[0];
    double* row = cen + k * g.row;
    if (n > 0) {
      double dn = (double)n;
      double e = 0.0;
      for (int c = 0; c < C; ++c) {
        double nv = FLT ? sf[c] / dn : (double)sc[c] / dn;
        double d = nv - row[c];
        e = e + d * d;
        row[c] = nv;
      }
      for (int i = 0; i < g.nd_out; ++i) {
        double nv = (double)si[1 + i] / dn;
        double d = nv - row[C + i];
        e = e + g.wd[i] * (d * d);
        row[C + i] = nv;
      }
      e_sum = sqrt(e);
      e_cnt = 1.0;
    }
    if (counts) counts[k] = (int64_t)n;
    if (prep_next) prep_one(g, row, k, it, binoff);
  }

template <int ND, int CC, bool FLT>
__global__ void __launch_bounds__(kThreads)
finalize_kernel(Geo g, double* __restrict__ cen, int64_t* __restrict__ counts, Iter it, int t,
                int prep_next, int use_part, TileDims td) {
  if (*it.done) return;
  __shared__ double sh_e[kThreads / 64], sh_n[kThreads / 64];
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double e_sum = 0.0, e_cnt = 0.0;
  if (k < g.K)
    finalize_one<ND, CC, FLT>(g, cen, counts, it, k, t, prep_next, use_part, td.T, 0, e_sum, e_cnt);
  e_sum = warp_sum(e_sum);
  e_cnt = warp_sum(e_cnt);
  int wv = threadIdx.x / 64, ln = threadIdx.x % 64;
  if (ln == 0) {
    sh_e[wv] = e_sum;
    sh_n[wv] = e_cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0, c = 0.0;
    for (int i = 0; i < kThreads / 64; ++i) {
      s += sh_e[i];
      c += sh_n[i];
    }
    if (c > 0.0) {
      double* r = it.res_acc + 2 * ((int64_t)t * kResSlots + blockIdx.x % kResSlots);
      atomicAdd(r, s);
      atomicAdd(r + 1, c);
    }
  }
}

__global__ void residual_finish_kernel(Iter it, int t, double tol, double* residuals) {
  if (*it.done) return;
  double s = 0.0, c = 0.0;
  for (int q = 0; q < kResSlots; ++q) {
    s += it.res_acc[2 * (t * kResSlots + q)];
    c += it.res_acc[2 * (t * kResSlots + q) + 1];
  }
  double e = c > 0.0 ? s / c : 0.0;
  if (residuals) residuals[t] = e;
  *it.iters = t + 1;
  if (e < tol) *it.done = 1;
}

// Reduce step of the clusters [k0, k1) of a batch group.  Residual partials
// go to each image's own (sum, count) pair; a wave whose lanes all belong to
// one image adds its total once.
template <int ND, int CC, bool FLT>
__global__ void __launch_bounds__(kThreads)
finalize_batch_kernel(const BImg* __restrict__ imgs, const int32_t* __restrict__ cl_img, int64_t k0,
                      int64_t k1, float* ctab, int32_t* bin_of, int32_t* bin_cnt, int t) {
  const int64_t gk = k0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool in = gk < k1;
  const int im = in ? cl_img[gk] : -1;
  double e_sum = 0.0, e_cnt = 0.0;
  with_image(imgs, im, in, [&](const BImg& d) {
    const bool next = t + 1 < d.iterations;
    if (!d.flags[0]) {
      const int64_t k = gk - d.koff;
      finalize_one<ND, CC, FLT>(d.g, d.cen, d.counts, batch_iter(d, ctab, bin_of, bin_cnt), k, t,
                                next, d.a.slots, d.tdim, d.binoff, e_sum, e_cnt);
    }
    // an image that has stopped takes no part in later bin sorts
    if (d.flags[0] || !next) bin_of[gk] = -1;
  });
  // residual partials: summed per wave when the wave is one image, then per
  // workgroup over its waves of one image, into slot blockIdx mod kResSlots
  __shared__ double sh_s[kThreads / 64], sh_c[kThreads / 64];
  __shared__ int sh_im[kThreads / 64];
  const int first = __builtin_amdgcn_readfirstlane(im);
  const bool uni = __all(im == first);
  const int slot = (int)(blockIdx.x % kResSlots);
  if (uni) {
    e_sum = warp_sum(e_sum);
    e_cnt = warp_sum(e_cnt);
  } else if (in && e_cnt > 0.0) {
    double* r = imgs[im].res + 2 * ((int64_t)t * kResSlots + slot);
    atomicAdd(r, e_sum);
    atomicAdd(r + 1, e_cnt);
  }
  const int wv = threadIdx.x / 64;
  if (threadIdx.x % 64 == 0) {
    sh_im[wv] = uni ? first : -1;
    sh_s[wv] = e_sum;
    sh_c[wv] = e_cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int cur = -1;
    double s = 0.0, c = 0.0;
    for (int w = 0; w <= kThreads / 64; ++w) {
      const int i = w < kThreads / 64 ? sh_im[w] : -2;
      if (i != cur) {
        if (cur >= 0 && c > 0.0) {
          double* r = imgs[cur].res + 2 * ((int64_t)t * kResSlots + slot);
          atomicAdd(r, s);
          atomicAdd(r + 1, c);
        }
        cur = i;
        s = c = 0.0;
      }
      if (i >= 0) {
        s += sh_s[w];
        c += sh_c[w];
      }
    }
  }
}

// Per image: residual of iteration t, iteration count, done flag (converged,
// or its own iteration count reached).
__global__ void residual_finish_batch_kernel(const BImg* __restrict__ imgs, int n, int t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const BImg& d = imgs[i];
  if (d.flags[0]) return;
  double s = 0.0, c = 0.0;
  for (int q = 0; q < kResSlots; ++q) {
    s += d.res[2 * (t * kResSlots + q)];
    c += d.res[2 * (t * kResSlots + q) + 1];
  }
  const double e = c > 0.0 ? s / c : 0.0;
  if (d.residuals) d.residuals[t] = e;
  d.flags[1] = t + 1;
  if (e < d.tol || t + 1 >= d.iterations) d.flags[0] = 1;
}

// residuals[t] = 0 for every t of every image (iterations after a stop read 0)
__global__ void batch_zero_residuals_kernel(const BImg* __restrict__ imgs, int n, int tmax) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= (int64_t)n * tmax) return;
  const BImg& d = imgs[j / tmax];
  const int t = (int)(j % tmax);
  if (d.residuals && t < d.iterations) d.residuals[t] = 0.0;
}

__global__ void batch_outputs_kernel(const BImg* __restrict__ imgs, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && imgs[i].iters_out) *imgs[i].iters_out = imgs[i].flags[1];
}

}  // namespace

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) { return fill(p, v, n, s); }
hipError_t launch_fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t s) { return fill(p, v, n, s); }
hipError_t launch_fill_f64(double* p, double v, int64_t n, hipStream_t s) { return fill(p, v, n, s); }

template <typename T, int ND>
bool seed_fixed_c(const Geo& g, const void* img, double* cen, hipStream_t s) {
  const int nb = blocks_for(g.K);
  const T* p = (const T*)img;
  switch (g.C) {
    case 1: seed_fixed_kernel<T, ND, 1><<<nb, kThreads, 0, s>>>(g, p, cen); return true;
    case 3: seed_fixed_kernel<T, ND, 3><<<nb, kThreads, 0, s>>>(g, p, cen); return true;
    case 4: seed_fixed_kernel<T, ND, 4><<<nb, kThreads, 0, s>>>(g, p, cen); return true;
    default: return false;
  }
}

template <typename T>
bool seed_fixed(const Geo& g, const void* img, double* cen, hipStream_t s) {
  if (g.nd == 2) return seed_fixed_c<T, 2>(g, img, cen, s);
  if (g.nd == 3) return seed_fixed_c<T, 3>(g, img, cen, s);
  return false;
}

hipError_t launch_seed(const Geo& g, const void* img, double* cen, hipStream_t s) {
  int nb = blocks_for(g.K);
  bool done = false;
  switch (g.dtype) {
    case kU8: done = seed_fixed<uint8_t>(g, img, cen, s); break;
    case kU16: done = seed_fixed<uint16_t>(g, img, cen, s); break;
    default: done = seed_fixed<float>(g, img, cen, s); break;
  }
  if (done) return hipGetLastError();
  switch (g.dtype) {
    case kU8: seed_kernel<uint8_t><<<nb, kThreads, 0, s>>>(g, (const uint8_t*)img, cen); break;
    case kU16: seed_kernel<uint16_t><<<nb, kThreads, 0, s>>>(g, (const uint16_t*)img, cen); break;
    default: seed_kernel<float><<<nb, kThreads, 0, s>>>(g, (const float*)img, cen); break;
  }
  return hipGetLastError();
}

hipError_t launch_grid_labels(const Geo& g, int32_t* labels, hipStream_t s) {
  int nb = (int)std::min<int64_t>(blocks_for(g.N), 65536);
  grid_labels_kernel<<<nb, kThreads, 0, s>>>(g, labels);
  return hipGetLastError();
}

hipError_t launch_prep(const Geo& g, const double* cen, const Iter& it, hipStream_t s) {
  prep_kernel<<<blocks_for(g.K), kThreads, 0, s>>>(g, cen, it);
  return hipGetLastError();
}

hipError_t launch_bins(const Geo& g, const Iter& it, hipStream_t s) {
  int nparts = (int)((g.nbins + kScanBlock - 1) / kScanBlock);
  scan_local_kernel<<<nparts, kThreads, 0, s>>>(it.bin_cnt, it.bin_start, it.scan_part, g.nbins, it.done);
  scan_parts_kernel<<<1, kThreads, 0, s>>>(it.scan_part, nparts, it.bin_start + g.nbins, it.done);
  scan_add_kernel<<<blocks_for(g.nbins), kThreads, 0, s>>>(it.bin_start, it.scan_part, g.nbins, it.done);
  scatter_kernel<<<blocks_for(g.K), kThreads, 0, s>>>(g, it);
  binsort_kernel<<<blocks_for(g.nbins), kThreads, 0, s>>>(g, it);
  return hipGetLastError();
}

hipError_t launch_finalize(const Geo& g, double* cen, int64_t* counts, const Iter& it, int t,
                           int prep_next, int use_part, hipStream_t s) {
  TileDims td{};
  sweep_tile_shape(g.nd, td.T);
  const unsigned nb = blocks_for(g.K);
  const bool flt = g.dtype == kF32;
#define SSLIC_FIN(ND, CC)                                                                     \
  (flt ? (finalize_kernel<ND, CC, true><<<nb, kThreads, 0, s>>>(g, cen, counts, it, t, prep_next, \
                                                               use_part, td), 0)              \
       : (finalize_kernel<ND, CC, false><<<nb, kThreads, 0, s>>>(g, cen, counts, it, t,       \
                                                                prep_next, use_part, td), 0))
#define SSLIC_FIN_C(ND)                       \
  switch (g.C) {                              \
    case 1: SSLIC_FIN(ND, 1); break;          \
    case 3: SSLIC_FIN(ND, 3); break;          \
    case 4: SSLIC_FIN(ND, 4); break;          \
    default: SSLIC_FIN(ND, 0); break;         \
  }
  switch (g.nd) {
    case 2: SSLIC_FIN_C(2); break;
    case 3: SSLIC_FIN_C(3); break;
    default: SSLIC_FIN_C(4); break;
  }
#undef SSLIC_FIN_C
#undef SSLIC_FIN
  return hipGetLastError();
}

hipError_t launch_seed_batch(int dtype, const BImg* imgs, const int32_t* cl_img, int64_t k0,
                             int64_t k1, hipStream_t s) {
  if (k1 <= k0) return hipSuccess;
  const int nb = blocks_for(k1 - k0);
  switch (dtype) {
    case kU8: seed_batch_kernel<uint8_t><<<nb, kThreads, 0, s>>>(imgs, cl_img, k0, k1); break;
    case kU16: seed_batch_kernel<uint16_t><<<nb, kThreads, 0, s>>>(imgs, cl_img, k0, k1); break;
    default: seed_batch_kernel<float><<<nb, kThreads, 0, s>>>(imgs, cl_img, k0, k1); break;
  }
  return hipGetLastError();
}

hipError_t launch_prep_batch(const BImg* imgs, const int32_t* cl_img, int64_t K, float* ctab,
                             int32_t* bin_of, int32_t* bin_cnt, hipStream_t s) {
  if (K <= 0) return hipSuccess;
  prep_batch_kernel<<<blocks_for(K), kThreads, 0, s>>>(imgs, cl_img, K, ctab, bin_of, bin_cnt);
  return hipGetLastError();
}

hipError_t launch_finalize_batch(int dtype, int nd, int C, const BImg* imgs, const int32_t* cl_img,
                                 int64_t k0, int64_t k1, float* ctab, int32_t* bin_of,
                                 int32_t* bin_cnt, int t, hipStream_t s) {
  if (k1 <= k0) return hipSuccess;
  const unsigned nb = blocks_for(k1 - k0);
  const bool flt = dtype == kF32;
#define SSLIC_FINB(ND, CC)                                                                       \
  (flt ? (finalize_batch_kernel<ND, CC, true><<<nb, kThreads, 0, s>>>(imgs, cl_img, k0, k1, ctab,  \
                                                                     bin_of, bin_cnt, t), 0)    \
       : (finalize_batch_kernel<ND, CC, false><<<nb, kThreads, 0, s>>>(imgs, cl_img, k0, k1, ctab, \
                                                                      bin_of, bin_cnt, t), 0))
#define SSLIC_FINB_C(ND)                      \
  switch (C) {                                \
    case 1: SSLIC_FINB(ND, 1); break;         \
    case 3: SSLIC_FINB(ND, 3); break;         \
    case 4: SSLIC_FINB(ND, 4); break;         \
    default: SSLIC_FINB(ND, 0); break;        \
  }
  switch (nd) {
    case 2: SSLIC_FINB_C(2); break;
    case 3: SSLIC_FINB_C(3); break;
    default: SSLIC_FINB_C(4); break;
  }
#undef SSLIC_FINB_C
#undef SSLIC_FINB
  return hipGetLastError();
}

hipError_t launch_residual_finish_batch(const BImg* imgs, int n, int t, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  residual_finish_batch_kernel<<<blocks_for(n), kThreads, 0, s>>>(imgs, n, t);
  return hipGetLastError();
}

hipError_t launch_batch_zero_residuals(const BImg* imgs, int n, int tmax, hipStream_t s) {
  if (n <= 0 || tmax <= 0) return hipSuccess;
  batch_zero_residuals_kernel<<<blocks_for((int64_t)n * tmax), kThreads, 0, s>>>(imgs, n, tmax);
  return hipGetLastError();
}

hipError_t launch_batch_outputs(const BImg* imgs, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  batch_outputs_kernel<<<blocks_for(n), kThreads, 0, s>>>(imgs, n);
  return hipGetLastError();
}

hipError_t launch_residual_finish(const Iter& it, int t, double tol, double* residuals, hipStream_t s) {
  residual_finish_kernel<<<1, 1, 0, s>>>(it, t, tol, residuals);
  return hipGetLastError();
}

}  // namespace sslic
