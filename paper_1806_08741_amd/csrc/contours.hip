// contours.hip -- the superpixel contour mask the paper renders its results
// with (Sec. 4, visualisation): a voxel lies on a contour when a face
// neighbour inside the image carries another label; the output is the image
// with every contour voxel set to 0 in all channels, the other voxels copied.
#include "sslic_internal.h"

namespace sslic {

namespace {

constexpr int kThreads = 256;

// One workgroup per 256-voxel piece of a row along axis 0 (the row's
// coordinates on the higher axes are the same for the whole workgroup).
// Neighbour labels along axis 0 share the row's cache lines; those along the
// higher axes are the rows the neighbouring workgroups read.
template <typename T, int CC>
__global__ void __launch_bounds__(kThreads)
mask_contours_kernel(Geo g, const T* __restrict__ img, const int32_t* __restrict__ lab,
                     T* __restrict__ out, int segs) {
  const int C = CC > 0 ? CC : g.C;
  const int64_t row = blockIdx.x / segs;
  const int x = (int)(blockIdx.x % segs) * kThreads + (int)threadIdx.x;
  if (x >= g.n[0]) return;
  int xc[kMaxDim];
  {
    int64_t r = row;
    for (int i = 1; i < g.nd; ++i) {
      xc[i] = (int)(r % g.n[i]);
      r /= g.n[i];
    }
  }
  const int64_t v = row * g.n[0] + x;
  const int l = lab[v];
  bool edge = (x > 0 && lab[v - 1] != l) || (x + 1 < g.n[0] && lab[v + 1] != l);
  for (int i = 1; i < g.nd; ++i) {
    edge = edge || (xc[i] > 0 && lab[v - g.st[i]] != l);
    edge = edge || (xc[i] + 1 < g.n[i] && lab[v + g.st[i]] != l);
  }
  for (int c = 0; c < C; ++c) out[v * C + c] = edge ? (T)0 : img[v * C + c];
}

// Four voxels per thread: their labels are one 16-byte load (and so are the
// labels of the rows beside them), their channel values whole 32-bit words,
// in which the bytes of contour voxels are cleared.  Needs axis 0 a multiple
// of 4 and rows a multiple of 16 bytes, so every load is aligned.
template <typename T, int CC>
__global__ void __launch_bounds__(kThreads)
mask_contours_vec_kernel(Geo g, const T* __restrict__ img, const int32_t* __restrict__ lab,
                         T* __restrict__ out, int segs) {
  constexpr int V = 4;
  constexpr int VB = CC * (int)sizeof(T);  // bytes per voxel
  constexpr int W = V * VB / 4;            // 32-bit words per thread
  const int64_t row = blockIdx.x / segs;
  const int x = ((int)(blockIdx.x % segs) * kThreads + (int)threadIdx.x) * V;
  if (x >= g.n[0]) return;
  int xc[kMaxDim];
  {
    int64_t r = row;
    for (int i = 1; i < g.nd; ++i) {
      xc[i] = (int)(r % g.n[i]);
      r /= g.n[i];
    }
  }
  const int64_t v = row * g.n[0] + x;
  const int4 l4 = *reinterpret_cast<const int4*>(lab + v);
  const int L[V] = {l4.x, l4.y, l4.z, l4.w};
  bool e[V];
  e[0] = (x > 0 && lab[v - 1] != L[0]) || L[1] != L[0];
  e[1] = L[0] != L[1] || L[2] != L[1];
  e[2] = L[1] != L[2] || L[3] != L[2];
  e[3] = L[2] != L[3] || (x + V < g.n[0] && lab[v + V] != L[3]);
  for (int i = 1; i < g.nd; ++i) {
    if (xc[i] > 0) {
      const int4 b = *reinterpret_cast<const int4*>(lab + v - g.st[i]);
      e[0] |= b.x != L[0], e[1] |= b.y != L[1], e[2] |= b.z != L[2], e[3] |= b.w != L[3];
    }
    if (xc[i] + 1 < g.n[i]) {
      const int4 b = *reinterpret_cast<const int4*>(lab + v + g.st[i]);
      e[0] |= b.x != L[0], e[1] |= b.y != L[1], e[2] |= b.z != L[2], e[3] |= b.w != L[3];
    }
  }
  const uint32_t* src = reinterpret_cast<const uint32_t*>(img + v * CC);
  uint32_t* dst = reinterpret_cast<uint32_t*>(out + v * CC);
  uint32_t w[W];
#pragma unroll
  for (int k = 0; k < W; ++k) w[k] = src[k];
#pragma unroll
  for (int k = 0; k < W; ++k) {
    uint32_t keep = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) keep |= e[(4 * k + b) / VB] ? 0u : 0xffu << (8 * b);
    dst[k] = w[k] & keep;
  }
}

// 3D, four voxels per thread as above, walking axis 2 over kZChunk planes:
// the labels of planes z-1, z and z+1 stay in registers, so each label comes
// from HBM once (as the plane ahead) instead of three times (its own plane
// and the two beside it, 4 MB apart for a 1024^3 volume).  The rows y-1 and
// y+1 of the same plane are the rows the neighbouring workgroups read at the
// same time; workgroups are handed out XCD by XCD (workgroup w takes piece
// (w mod 8) * (G/8) + w div 8 of a grid of G, a multiple of 8), so those
// neighbours share one L2.  Pieces go x-segment fastest, then y, then z-chunk.
constexpr int kZChunk = 32;

template <typename T, int CC>
__global__ void __launch_bounds__(kThreads)
mask_contours_z_kernel(Geo g, const T* __restrict__ img, const int32_t* __restrict__ lab,
                       T* __restrict__ out, int segs, int64_t pieces) {
  constexpr int V = 4;
  constexpr int VB = CC * (int)sizeof(T);
  constexpr int W = V * VB / 4;
  const int64_t piece = (int64_t)(blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
  if (piece >= pieces) return;  // no barrier in this kernel
  const int x = ((int)(piece % segs) * kThreads + (int)threadIdx.x) * V;
  if (x >= g.n[0]) return;
  const int64_t rest = piece / segs;
  const int y = (int)(rest % g.n[1]);
  const int z0 = (int)(rest / g.n[1]) * kZChunk;
  const int z1 = min(z0 + kZChunk, g.n[2]);
  const int64_t sy = g.st[1], sz = g.st[2];
  const bool hy0 = y > 0, hy1 = y + 1 < g.n[1];
  const bool hx0 = x > 0, hx1 = x + V < g.n[0];
  auto ld4 = [&](int64_t v) { return *reinterpret_cast<const int4*>(lab + v); };

  int64_t v = (int64_t)z0 * sz + (int64_t)y * sy + x;
  int4 prev = z0 > 0 ? ld4(v - sz) : make_int4(0, 0, 0, 0);
  int4 cur = ld4(v);
  for (int z = z0; z < z1; ++z, v += sz) {
    const bool hz1 = z + 1 < g.n[2];
    const int4 next = hz1 ? ld4(v + sz) : cur;
    const int4 up = hy0 ? ld4(v - sy) : cur;
    const int4 dn = hy1 ? ld4(v + sy) : cur;
    const int left = hx0 ? lab[v - 1] : cur.x;
    const int right = hx1 ? lab[v + V] : cur.w;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(img + v * CC);
    uint32_t w[W];
#pragma unroll
    for (int k = 0; k < W; ++k) w[k] = src[k];
    const int4 pz = z > 0 ? prev : cur;
    bool e[V];
    e[0] = left != cur.x || cur.y != cur.x || up.x != cur.x || dn.x != cur.x || pz.x != cur.x ||
           next.x != cur.x;
    e[1] = cur.x != cur.y || cur.z != cur.y || up.y != cur.y || dn.y != cur.y || pz.y != cur.y ||
           next.y != cur.y;
    e[2] = cur.y != cur.z || cur.w != cur.z || up.z != cur.z || dn.z != cur.z || pz.z != cur.z ||
           next.z != cur.z;
    e[3] = cur.z != cur.w || right != cur.w || up.w != cur.w || dn.w != cur.w || pz.w != cur.w ||
           next.w != cur.w;
    uint32_t* dst = reinterpret_cast<uint32_t*>(out + v * CC);
#pragma unroll
    for (int k = 0; k < W; ++k) {
      uint32_t keep = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) keep |= e[(4 * k + b) / VB] ? 0u : 0xffu << (8 * b);
      dst[k] = w[k] & keep;
    }
    prev = cur;
    cur = next;
  }
}

template <typename T>
hipError_t launch_t(const Geo& g, const void* img, const int32_t* lab, void* out, hipStream_t s) {
  const int64_t rows = g.N / g.n[0];
  const int64_t vb = (int64_t)g.C * (int64_t)sizeof(T);
  const bool aligned = g.n[0] % 4 == 0 && (g.n[0] * vb) % 16 == 0 &&
                       reinterpret_cast<uintptr_t>(img) % 16 == 0 &&
                       reinterpret_cast<uintptr_t>(out) % 16 == 0 &&
                       reinterpret_cast<uintptr_t>(lab) % 16 == 0;
  if (aligned && g.nd == 3 && (g.C == 1 || g.C == 3 || g.C == 4)) {
    const int segs = (g.n[0] / 4 + kThreads - 1) / kThreads;
    const int64_t pieces = (int64_t)segs * g.n[1] * ((g.n[2] + kZChunk - 1) / kZChunk);
    const int64_t nwg = (pieces + 7) / 8 * 8;
    if (nwg >= (1LL << 31)) return hipErrorInvalidValue;
    const T* p = (const T*)img;
    T* o = (T*)out;
    switch (g.C) {
      case 1: mask_contours_z_kernel<T, 1><<<(unsigned)nwg, kThreads, 0, s>>>(g, p, lab, o, segs, pieces); break;
      case 3: mask_contours_z_kernel<T, 3><<<(unsigned)nwg, kThreads, 0, s>>>(g, p, lab, o, segs, pieces); break;
      default: mask_contours_z_kernel<T, 4><<<(unsigned)nwg, kThreads, 0, s>>>(g, p, lab, o, segs, pieces); break;
    }
    return hipGetLastError();
  }
  if (aligned && (g.C == 1 || g.C == 3 || g.C == 4)) {
    const int segs = (g.n[0] / 4 + kThreads - 1) / kThreads;
    if (rows * segs >= (1LL << 31)) return hipErrorInvalidValue;
    const unsigned grid = (unsigned)(rows * segs);
    const T* p = (const T*)img;
    T* o = (T*)out;
    switch (g.C) {
      case 1: mask_contours_vec_kernel<T, 1><<<grid, kThreads, 0, s>>>(g, p, lab, o, segs); break;
      case 3: mask_contours_vec_kernel<T, 3><<<grid, kThreads, 0, s>>>(g, p, lab, o, segs); break;
      default: mask_contours_vec_kernel<T, 4><<<grid, kThreads, 0, s>>>(g, p, lab, o, segs); break;
    }
    return hipGetLastError();
  }
  const int segs = (g.n[0] + kThreads - 1) / kThreads;
  const int64_t grid = g.N / g.n[0] * segs;
  if (grid >= (1LL << 31)) return hipErrorInvalidValue;
  const T* p = (const T*)img;
  T* o = (T*)out;
  switch (g.C) {
    case 1: mask_contours_kernel<T, 1><<<(unsigned)grid, kThreads, 0, s>>>(g, p, lab, o, segs); break;
    case 3: mask_contours_kernel<T, 3><<<(unsigned)grid, kThreads, 0, s>>>(g, p, lab, o, segs); break;
    case 4: mask_contours_kernel<T, 4><<<(unsigned)grid, kThreads, 0, s>>>(g, p, lab, o, segs); break;
    default: mask_contours_kernel<T, 0><<<(unsigned)grid, kThreads, 0, s>>>(g, p, lab, o, segs); break;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_mask_contours(const Geo& g, const void* img, const int32_t* labels, void* out,
                                hipStream_t s) {
  switch (g.dtype) {
    case kU8: return launch_t<uint8_t>(g, img, labels, out, s);
    case kU16: return launch_t<uint16_t>(g, img, labels, out, s);
    default: return launch_t<float>(g, img, labels, out, s);
  }
}

}  // namespace sslic
