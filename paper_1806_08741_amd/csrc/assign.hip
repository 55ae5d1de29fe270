// assign.hip -- the assignment step (Sec. 2.1 distance with the per-axis
// weights of Sec. 3.3; Sec. 2.2 / 3.1 stage 2), computed per voxel: a voxel
// takes the lowest-index centre minimising D^2 among the centres whose closed
// window holds it.  Those centres all sit in the 3^n S-bins around the
// voxel's own bin (see the table and bins in centres.hip).
#include "sslic_internal.h"

namespace sslic {

namespace {

constexpr int kThreads = 256;

template <typename T, int ND, int CC>
__global__ void __launch_bounds__(kThreads)
assign_voxel_kernel(Geo g, const T* __restrict__ img, Iter it, int32_t* __restrict__ labels,
                    int first) {
  if (*it.done) return;
  const int C = CC > 0 ? CC : g.C;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < g.N;
       v += (int64_t)gridDim.x * blockDim.x) {
    int x[ND], b[ND];
    int64_t r = v;
    for (int i = 0; i < ND; ++i) {
      x[i] = (int)(r % g.n[i]);
      r /= g.n[i];
      b[i] = x[i] / g.S[i];
    }
    float I[CC > 0 ? CC : kMaxChan];
    for (int c = 0; c < C; ++c) I[c] = (float)img[v * C + c];
    float best = __builtin_inff();
    int bk = -1;
    int n3 = 1;
    for (int i = 0; i < ND; ++i) n3 *= 3;
    for (int o = 0; o < n3; ++o) {
      int oo = o;
      int64_t bl = 0;
      bool ok = true;
      for (int i = 0; i < ND; ++i) {
        int bi = b[i] + (oo % 3) - 1;
        oo /= 3;
        ok = ok && bi >= 0 && bi < g.nb[i];
        bl += bi * g.bst[i];
      }
      if (!ok) continue;
      int e = it.bin_start[bl + 1];
      for (int j = it.bin_start[bl]; j < e; ++j) {
        int k = it.bin_items[j];
        const float* rec = it.ctab + (int64_t)k * g.rs;
        const int32_t* irec = reinterpret_cast<const int32_t*>(rec);
        bool inside = true;
        for (int i = 0; i < ND; ++i)
          inside = inside && x[i] >= irec[C + ND + i] && x[i] <= irec[C + 2 * ND + i];
        if (!inside) continue;
        float D = 0.0f;
        for (int c = 0; c < C; ++c) {
          float t = I[c] - rec[c];
          D = fmaf(t, t, D);
        }
        for (int i = 0; i < ND; ++i) {
          float t = (float)x[i] - rec[C + i];
          D = fmaf(g.w[i] * t, t, D);
        }
        if (D < best || (D == best && k < bk)) {
          best = D;
          bk = k;
        }
      }
    }
    if (bk < 0) {
      if (first) {
        int64_t kk = 0, kst = 1;
        for (int i = 0; i < ND; ++i) {
          kk += ((int64_t)x[i] * g.Ka[i] / g.n[i]) * kst;
          kst *= g.Ka[i];
        }
        bk = (int)kk;
      } else {
        bk = labels[v];
      }
    }
    labels[v] = bk;
  }
}

template <typename T, int ND>
hipError_t dispatch_c(const Geo& g, const void* img, const Iter& it, int32_t* labels, int first,
                      hipStream_t s) {
  int nb = (int)std::min<int64_t>((g.N + kThreads - 1) / kThreads, 1 << 20);
  const T* p = (const T*)img;
  switch (g.C) {
    case 1: assign_voxel_kernel<T, ND, 1><<<nb, kThreads, 0, s>>>(g, p, it, labels, first); break;
    case 3: assign_voxel_kernel<T, ND, 3><<<nb, kThreads, 0, s>>>(g, p, it, labels, first); break;
    case 4: assign_voxel_kernel<T, ND, 4><<<nb, kThreads, 0, s>>>(g, p, it, labels, first); break;
    default: assign_voxel_kernel<T, ND, 0><<<nb, kThreads, 0, s>>>(g, p, it, labels, first); break;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t dispatch_nd(const Geo& g, const void* img, const Iter& it, int32_t* labels, int first,
                       hipStream_t s) {
  switch (g.nd) {
    case 2: return dispatch_c<T, 2>(g, img, it, labels, first, s);
    case 3: return dispatch_c<T, 3>(g, img, it, labels, first, s);
    default: return dispatch_c<T, 4>(g, img, it, labels, first, s);
  }
}

}  // namespace

hipError_t launch_assign(const Geo& g, const void* img, const Iter& it, int32_t* labels, int first,
                         hipStream_t s) {
  switch (g.dtype) {
    case kU8: return dispatch_nd<uint8_t>(g, img, it, labels, first, s);
    case kU16: return dispatch_nd<uint16_t>(g, img, it, labels, first, s);
    default: return dispatch_nd<float>(g, img, it, labels, first, s);
  }
}

}  // namespace sslic
