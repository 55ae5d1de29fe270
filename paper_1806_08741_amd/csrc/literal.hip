// literal.hip -- assignment on a distance image that lives across iterations
// (Sec. 2.2 and Sec. 3.1: d is set to infinity once, in stage 1, and a voxel
// takes centre k only where D(x, k) < d(x)).  The main path resets d every
// iteration and fuses the map step of the update into its sweep; this step
// is a voxel-parallel gather whose labels the stand-alone update step then
// sums.
//
// A wave takes one block of 64 voxels (8x8 in 2D, 4x4x4 in 3D, 4x4x2x2 in
// 4D), one voxel per lane.  Every centre whose closed window holds a voxel of
// the block is in the bins within one bin of the block (a centre's bin is the
// S-cell of its window's low corner, plus one).  The wave first gathers those
// centres, lane j the j-th, with their records (all loads in flight at
// once), and ballots which windows meet the block; it then walks the meeting
// ones, broadcasting each record from its lane, while every lane tests its own
// voxel and evaluates the FP32 distance in the scaled coordinates of the
// records (the same terms in the same order as the sweep).  The least
// (D^2, k) is one 64-bit key.  A block with more than 64 such centres walks
// them one by one with scalar loads instead.
#include "literal.h"

namespace sslic {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

template <int ND>
struct Blk;
template <>
struct Blk<2> {
  static constexpr int B[2] = {8, 8};
};
template <>
struct Blk<3> {
  static constexpr int B[3] = {4, 4, 4};
};
template <>
struct Blk<4> {
  static constexpr int B[4] = {4, 4, 2, 2};
};

// Grid cell of voxel x: sum_i floor(x_i K_i / N_i) prod_{i'<i} K_i'.
template <int ND>
__device__ __forceinline__ int32_t cell_of(const Geo& g, const int* x) {
  int64_t k = 0, kst = 1;
#pragma unroll
  for (int i = 0; i < ND; ++i) {
    k += ((int64_t)x[i] * g.Ka[i] / g.n[i]) * kst;
    kst *= g.Ka[i];
  }
  return (int32_t)k;
}

// Workgroup w of a grid of G (a multiple of 8) takes the blocks of tile
// (w mod 8) * (G / 8) + w div 8: workgroups go round the 8 XCDs in turn, so
// neighbouring tiles, whose image and distance lines overlap, run on one XCD
// and share its L2.
template <typename T, int ND, int CC>
__global__ void __launch_bounds__(kThreads)
assign_persist_kernel(Geo g, const T* __restrict__ img, const float* __restrict__ recs,
                      const int* __restrict__ bstart, const int* __restrict__ items,
                      const int* __restrict__ done, int32_t* __restrict__ labels,
                      float* __restrict__ dist, uint32_t nblocks, int first) {
  if (*done) return;
  constexpr int CM = CC > 0 ? CC : kMaxChan;
  constexpr int RN = (CM + 3 * ND + 1 + 3) & ~3;  // record words (rec_words)
  const int C = CC > 0 ? CC : g.C;
  const int RS = g.rs;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t tile = (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
  const uint32_t b = tile * kWaves + (uint32_t)wave;
  if (b >= nblocks) return;  // no barrier in this kernel

  // the block (axis 0 fastest over blocks; 32-bit index arithmetic, the
  // last axis without a division) and this lane's voxel in it
  int org[ND], top[ND], x[ND];
  uint32_t rb = b;
  int lr = lane;
  bool valid = true;
#pragma unroll
  for (int i = 0; i < ND; ++i) {
    const int Bi = Blk<ND>::B[i];
    if (i + 1 < ND) {
      const uint32_t nbi = (uint32_t)(g.n[i] + Bi - 1) / Bi;
      const uint32_t q = rb / nbi;
      org[i] = (int)(rb - q * nbi) * Bi;
      rb = q;
    } else {
      org[i] = (int)rb * Bi;
    }
    top[i] = min(org[i] + Bi, g.n[i]) - 1;
    x[i] = org[i] + lr % Bi;
    lr /= Bi;
    valid = valid && x[i] <= top[i];
  }
  int64_t v = 0;
#pragma unroll
  for (int i = 0; i < ND; ++i) v += (int64_t)(valid ? x[i] : org[i]) * g.st[i];
  float xs[ND];
#pragma unroll
  for (int i = 0; i < ND; ++i) xs[i] = (float)x[i] * g.sw[i];
  float I[CM];
  for (int c = 0; c < C; ++c) I[c] = (float)img[v * C + c];

  int blo[ND], bhi[ND], rc[ND];
#pragma unroll
  for (int i = 0; i < ND; ++i) {
    blo[i] = max(org[i] / g.S[i] - 1, 0);
    bhi[i] = min(top[i] / g.S[i] + 1, g.nb[i] - 1);
    rc[i] = blo[i];
  }
  uint64_t best = ~0ull;
  auto consider = [&](const float* R, uint32_t k) {
    const int* Ri = reinterpret_cast<const int*>(R);
    bool in = valid;
#pragma unroll
    for (int i = 0; i < ND; ++i)
      in = in && x[i] >= Ri[rec_lo(C, ND) + i] && x[i] <= Ri[rec_hi(C, ND) + i];
    float D;
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      const float d = xs[i] - R[C + i];
      D = i == 0 ? d * d : fmaf(d, d, D);
    }
    for (int c = 0; c < C; ++c) {
      const float t = I[c] - R[c];
      D = fmaf(t, t, D);
    }
    const uint64_t key = (uint64_t)__float_as_uint(D) << 32 | k;
    if (in && key < best) best = key;
  };

  // Gather: lane j takes the j-th centre of the bin rows around the block, and
  // its record, with every load of the wave in flight at once.
  int myk = 0, cnt = 0;
  while (true) {
    int64_t bl = (int64_t)blo[0] * g.bst[0];
#pragma unroll
    for (int i = 1; i < ND; ++i) bl += (int64_t)rc[i] * g.bst[i];
    const int ja = __builtin_amdgcn_readfirstlane(bstart[bl]);
    const int jb = __builtin_amdgcn_readfirstlane(bstart[bl + (bhi[0] - blo[0]) + 1]);
    const int j = lane - cnt;
    if (j >= 0 && j < jb - ja) myk = items[ja + j];
    cnt += jb - ja;
    int i = 1;
    while (i < ND) {
      if (++rc[i] <= bhi[i]) break;
      rc[i] = blo[i];
      ++i;
    }
    if (i >= ND) break;
  }
  if (cnt <= 64) {
    const bool held = lane < cnt;
    const float* rec = recs + (int64_t)(held ? myk : 0) * RS;
    float MR[RN];
#pragma unroll
    for (int w = 0; w < RN; ++w) MR[w] = (CC > 0 || w < RS) ? rec[w] : 0.0f;
    const int* MRi = reinterpret_cast<const int*>(MR);
    bool meets = held;
#pragma unroll
    for (int i = 0; i < ND; ++i)
      meets = meets && MRi[rec_lo(C, ND) + i] <= top[i] && MRi[rec_hi(C, ND) + i] >= org[i];
    uint64_t mask = __ballot(meets);
    while (mask) {
      const int l = (int)__builtin_ctzll(mask);
      mask &= mask - 1;
      float R[RN];
#pragma unroll
      for (int w = 0; w < RN; ++w)
        R[w] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(MR[w]), l));
      consider(R, (uint32_t)__builtin_amdgcn_readlane(myk, l));
    }
  } else {
    // more centres than lanes (a crowded neighbourhood): walk them one by one
#pragma unroll
    for (int i = 0; i < ND; ++i) rc[i] = blo[i];
    while (true) {
      int64_t bl = (int64_t)blo[0] * g.bst[0];
#pragma unroll
      for (int i = 1; i < ND; ++i) bl += (int64_t)rc[i] * g.bst[i];
      const int ja = __builtin_amdgcn_readfirstlane(bstart[bl]);
      const int jb = __builtin_amdgcn_readfirstlane(bstart[bl + (bhi[0] - blo[0]) + 1]);
      for (int q = ja; q < jb; ++q) {
        const int k = __builtin_amdgcn_readfirstlane(items[q]);
        const float* rec = recs + (int64_t)k * RS;
        float R[RN];
#pragma unroll
        for (int w = 0; w < RN; ++w) R[w] = (CC > 0 || w < RS) ? rec[w] : 0.0f;
        const int* Ri = reinterpret_cast<const int*>(R);
        bool meets = true;
#pragma unroll
        for (int i = 0; i < ND; ++i)
          meets = meets && Ri[rec_lo(C, ND) + i] <= top[i] && Ri[rec_hi(C, ND) + i] >= org[i];
        if (meets) consider(R, (uint32_t)k);
      }
      int i = 1;
      while (i < ND) {
        if (++rc[i] <= bhi[i]) break;
        rc[i] = blo[i];
        ++i;
      }
      if (i >= ND) break;
    }
  }
  if (valid && best != ~0ull) {
    const float D = __uint_as_float((uint32_t)(best >> 32));
    if (D < dist[v]) {
      labels[v] = (int32_t)(uint32_t)best;
      dist[v] = D;
    } else if (first) {
      labels[v] = cell_of<ND>(g, x);
    }
  } else if (valid && first) {
    labels[v] = cell_of<ND>(g, x);
  }
}

template <typename T, int ND>
hipError_t dispatch_c(const Geo& g, const void* img, const Iter& it, int32_t* labels, float* dist,
                      int first, hipStream_t s) {
  int64_t nblocks = 1;
  for (int i = 0; i < ND; ++i) nblocks *= (g.n[i] + Blk<ND>::B[i] - 1) / Blk<ND>::B[i];
  const int64_t nwg = ((nblocks + kWaves - 1) / kWaves + 7) / 8 * 8;  // whole rounds of 8 XCDs
  if (nwg <= 0) return hipSuccess;
  if (nblocks > 0x7fffffff) return hipErrorInvalidValue;  // 32-bit block indices
  const T* p = (const T*)img;
  const unsigned grid = (unsigned)nwg;
  const float* r = it.ctab;
  const int *bs = it.bin_start, *items = it.bin_items, *done = it.done;
  switch (g.C) {
    case 1: assign_persist_kernel<T, ND, 1><<<grid, kThreads, 0, s>>>(g, p, r, bs, items, done, labels, dist, (uint32_t)nblocks, first); break;
    case 3: assign_persist_kernel<T, ND, 3><<<grid, kThreads, 0, s>>>(g, p, r, bs, items, done, labels, dist, (uint32_t)nblocks, first); break;
    case 4: assign_persist_kernel<T, ND, 4><<<grid, kThreads, 0, s>>>(g, p, r, bs, items, done, labels, dist, (uint32_t)nblocks, first); break;
    default: assign_persist_kernel<T, ND, 0><<<grid, kThreads, 0, s>>>(g, p, r, bs, items, done, labels, dist, (uint32_t)nblocks, first); break;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t dispatch_nd(const Geo& g, const void* img, const Iter& it, int32_t* labels, float* dist,
                       int first, hipStream_t s) {
  switch (g.nd) {
    case 2: return dispatch_c<T, 2>(g, img, it, labels, dist, first, s);
    case 3: return dispatch_c<T, 3>(g, img, it, labels, dist, first, s);
    default: return dispatch_c<T, 4>(g, img, it, labels, dist, first, s);
  }
}

}  // namespace

hipError_t launch_assign_persist(const Geo& g, const void* img, const Iter& it, int32_t* labels,
                                 float* dist, int first, hipStream_t s) {
  switch (g.dtype) {
    case kU8: return dispatch_nd<uint8_t>(g, img, it, labels, dist, first, s);
    case kU16: return dispatch_nd<uint16_t>(g, img, it, labels, dist, first, s);
    default: return dispatch_nd<float>(g, img, it, labels, dist, first, s);
  }
}

}  // namespace sslic
