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

template <typename T>
hipError_t launch_t(const Geo& g, const void* img, const int32_t* lab, void* out, hipStream_t s) {
  const int64_t rows = g.N / g.n[0];
  const int64_t vb = (int64_t)g.C * (int64_t)sizeof(T);
  const bool aligned = g.n[0] % 4 == 0 && (g.n[0] * vb) % 16 == 0 &&
                       reinterpret_cast<uintptr_t>(img) % 16 == 0 &&
                       reinterpret_cast<uintptr_t>(out) % 16 == 0 &&
                       reinterpret_cast<uintptr_t>(lab) % 16 == 0;
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
