// literal.hip -- assignment on a distance image that lives across iterations
// (Sec. 2.2 and Sec. 3.1: d is set to infinity once, in stage 1, and a voxel
// takes centre k only where D(x, k) < d(x)).  The main path resets d every
// iteration and fuses the map step of the update into its sweep; this step
// is a voxel-parallel gather whose labels the stand-alone update step then
// sums.
//
// One thread per voxel.  A workgroup takes 64 consecutive voxels along axis 0
// on 4 x kRowsPerWave rows (the other axes flattened); each wave walks
// kRowsPerWave rows.  Every centre whose closed window holds x lies in the
// 3^n bins around floor(x_i / S_i) (a centre's bin is the S-cell of its
// window's low corner, plus one); along axis 0 those bins are one contiguous
// range of the bin-ordered item list, so a voxel reads 3^(n-1) ranges.  The
// lanes of a wave share almost all of their ranges, so the records come from
// the caches.  Distances are FP32 in the scaled coordinates of the records,
// the same terms in the same order as the sweep.
#include "literal.h"

namespace sslic {

namespace {

constexpr int kThreads = 256;
constexpr int kRowsPerWave = 4;
constexpr int kRowsPerBlock = kRowsPerWave * (kThreads / 64);

template <typename T, int ND, int CC>
__global__ void __launch_bounds__(kThreads)
assign_persist_kernel(Geo g, const T* __restrict__ img, Iter it, int32_t* __restrict__ labels,
                      float* __restrict__ dist, int64_t nrows) {
  if (*it.done) return;
  constexpr int CM = CC > 0 ? CC : kMaxChan;
  const int C = CC > 0 ? CC : g.C;
  const int RS = g.rs;
  const float* __restrict__ recs = it.ctab;
  const int* __restrict__ irecs = reinterpret_cast<const int*>(it.ctab);
  const int* __restrict__ bstart = it.bin_start;
  const int* __restrict__ items = it.bin_items;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n0 = g.n[0];
  const int64_t tiles_x = (n0 + 63) / 64;
  const int x0 = (int)(blockIdx.x % tiles_x) * 64 + lane;
  if (x0 >= n0) return;  // no barrier below
  const int64_t rbase = (int64_t)(blockIdx.x / tiles_x) * kRowsPerBlock + wave * kRowsPerWave;

  const int b0 = x0 / g.S[0];
  const int lo0 = max(b0 - 1, 0), hi0 = min(b0 + 1, g.nb[0] - 1);
  const float xs0 = (float)x0 * g.sw[0];

  for (int j = 0; j < kRowsPerWave; ++j) {
    const int64_t r = rbase + j;
    if (r >= nrows) break;
    int x[ND];
    float xs[ND];
    int blo[ND], bhi[ND];
    x[0] = x0;
    xs[0] = xs0;
    int64_t rr = r;
    for (int i = 1; i < ND; ++i) {
      x[i] = (int)(rr % g.n[i]);
      rr /= g.n[i];
      xs[i] = (float)x[i] * g.sw[i];
      const int b = x[i] / g.S[i];
      blo[i] = max(b - 1, 0);
      bhi[i] = min(b + 1, g.nb[i] - 1);
    }
    const int64_t v = r * n0 + x0;
    float I[CM];
    for (int c = 0; c < C; ++c) I[c] = (float)img[v * C + c];

    float best = __builtin_inff();
    int bk = -1;
    int rc[ND];
    for (int i = 1; i < ND; ++i) rc[i] = blo[i];
    while (true) {
      int64_t bl = (int64_t)lo0 * g.bst[0];
      for (int i = 1; i < ND; ++i) bl += (int64_t)rc[i] * g.bst[i];
      const int ja = bstart[bl];
      const int jb = bstart[bl + (hi0 - lo0) + 1];
      for (int q = ja; q < jb; ++q) {
        const int k = items[q];
        const int* ir = irecs + (int64_t)k * RS;
        bool ok = true;
#pragma unroll
        for (int i = 0; i < ND; ++i)
          ok = ok && x[i] >= ir[rec_lo(C, ND) + i] && x[i] <= ir[rec_hi(C, ND) + i];
        if (!ok) continue;
        const float* rec = recs + (int64_t)k * RS;
        float D = 0.0f;
#pragma unroll
        for (int i = 0; i < ND; ++i) {
          const float d = xs[i] - rec[C + i];
          D = i == 0 ? d * d : fmaf(d, d, D);
        }
        for (int c = 0; c < C; ++c) {
          const float t = I[c] - rec[c];
          D = fmaf(t, t, D);
        }
        if (D < best || (D == best && k < bk)) {
          best = D;
          bk = k;
        }
      }
      int i = 1;
      while (i < ND) {
        if (++rc[i] <= bhi[i]) break;
        rc[i] = blo[i];
        ++i;
      }
      if (i >= ND) break;
    }
    if (bk >= 0 && best < dist[v]) {
      labels[v] = bk;
      dist[v] = best;
    }
  }
}

template <typename T, int ND>
hipError_t dispatch_c(const Geo& g, const void* img, const Iter& it, int32_t* labels, float* dist,
                      hipStream_t s) {
  const int64_t tiles_x = (g.n[0] + 63) / 64;
  const int64_t nrows = g.N / g.n[0];
  const int64_t nb = tiles_x * ((nrows + kRowsPerBlock - 1) / kRowsPerBlock);
  if (nb <= 0) return hipSuccess;
  if (nb > 0x7fffffff) return hipErrorInvalidValue;
  const T* p = (const T*)img;
  const unsigned grid = (unsigned)nb;
  switch (g.C) {
    case 1: assign_persist_kernel<T, ND, 1><<<grid, kThreads, 0, s>>>(g, p, it, labels, dist, nrows); break;
    case 3: assign_persist_kernel<T, ND, 3><<<grid, kThreads, 0, s>>>(g, p, it, labels, dist, nrows); break;
    case 4: assign_persist_kernel<T, ND, 4><<<grid, kThreads, 0, s>>>(g, p, it, labels, dist, nrows); break;
    default: assign_persist_kernel<T, ND, 0><<<grid, kThreads, 0, s>>>(g, p, it, labels, dist, nrows); break;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t dispatch_nd(const Geo& g, const void* img, const Iter& it, int32_t* labels, float* dist,
                       hipStream_t s) {
  switch (g.nd) {
    case 2: return dispatch_c<T, 2>(g, img, it, labels, dist, s);
    case 3: return dispatch_c<T, 3>(g, img, it, labels, dist, s);
    default: return dispatch_c<T, 4>(g, img, it, labels, dist, s);
  }
}

}  // namespace

hipError_t launch_assign_persist(const Geo& g, const void* img, const Iter& it, int32_t* labels,
                                 float* dist, hipStream_t s) {
  switch (g.dtype) {
    case kU8: return dispatch_nd<uint8_t>(g, img, it, labels, dist, s);
    case kU16: return dispatch_nd<uint16_t>(g, img, it, labels, dist, s);
    default: return dispatch_nd<float>(g, img, it, labels, dist, s);
  }
}

}  // namespace sslic
