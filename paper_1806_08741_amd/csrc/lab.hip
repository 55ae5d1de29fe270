// lab.hip -- RGB (8-bit sRGB) to CIE-Lab, the colour space the paper's 2D
// and Visible Human runs use (Sec. 2.1, Sec. 4 data; the lookup-table
// approach of jSLIC it cites).  Constants: the sRGB transfer curve, the
// four-digit sRGB-to-XYZ matrix and the D65 white (0.95047, 1, 1.08883),
// with which the Lab ranges the paper prints for 8-bit RGB come out.
#include <cmath>

#include "sslic_internal.h"

namespace sslic {

namespace {

constexpr int kThreads = 256;

// XYZ / white, with the white folded into the matrix rows (FP64, then FP32)
constexpr double kXn = 0.95047, kYn = 1.0, kZn = 1.08883;
constexpr float kM[9] = {
    (float)(0.4124 / kXn), (float)(0.3576 / kXn), (float)(0.1805 / kXn),
    (float)(0.2126 / kYn), (float)(0.7152 / kYn), (float)(0.0722 / kYn),
    (float)(0.0193 / kZn), (float)(0.1192 / kZn), (float)(0.9505 / kZn)};
constexpr float kEps = (float)(216.0 / 24389.0);   // (6/29)^3
constexpr float kKap = (float)(24389.0 / 27.0);    // (29/3)^3

// The cube root as 2^(log2(t) / 3) on the hardware base-2 log and exponent
// (about one ulp each): for t above (6/29)^3 the result is within a few
// 1e-7 relative, far inside what the Lab values need.
__device__ __forceinline__ float lab_f(float t) {
  return t > kEps ? __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(t) * (1.0f / 3.0f))
                  : (kKap * t + 16.0f) * (1.0f / 116.0f);
}

__device__ __forceinline__ void lab_of(const float* lin, uint32_t r, uint32_t g, uint32_t b,
                                       float* out) {
  const float R = lin[r], G = lin[g], B = lin[b];
  const float fx = lab_f(kM[0] * R + kM[1] * G + kM[2] * B);
  const float fy = lab_f(kM[3] * R + kM[4] * G + kM[5] * B);
  const float fz = lab_f(kM[6] * R + kM[7] * G + kM[8] * B);
  out[0] = 116.0f * fy - 16.0f;
  out[1] = 500.0f * (fx - fy);
  out[2] = 200.0f * (fy - fz);
}

// The linear value of every 8-bit level, computed in FP64 once per workgroup.
__device__ __forceinline__ void fill_lin(float* s_lin) {
  const double v = threadIdx.x / 255.0;
  s_lin[threadIdx.x] = (float)(v <= 0.04045 ? v / 12.92 : pow((v + 0.055) / 1.055, 2.4));
  __syncthreads();
}

// Four pixels per thread (12 bytes in as three words).  The 48 bytes of
// each thread go through LDS, so that each of the three 16-byte stores of
// the workgroup writes one contiguous 4 KB span.  Needs rgb 4-byte and lab
// 16-byte aligned.  Workgroups take chunks of 256 groups of four pixels; the
// trip count is the same for every thread of a workgroup.
__global__ void __launch_bounds__(kThreads)
rgb_to_lab_vec_kernel(const uint8_t* __restrict__ rgb, int64_t groups, float* __restrict__ lab) {
  __shared__ float s_lin[256];
  __shared__ float4 s_out[3 * kThreads];
  fill_lin(s_lin);
  for (int64_t base = blockIdx.x * (int64_t)kThreads; base < groups;
       base += (int64_t)gridDim.x * kThreads) {
    const int64_t q = base + threadIdx.x;
    if (q < groups) {
      const uint32_t* src = reinterpret_cast<const uint32_t*>(rgb) + 3 * q;
      const uint32_t w0 = src[0], w1 = src[1], w2 = src[2];
      const uint32_t c[12] = {w0 & 255u, (w0 >> 8) & 255u, (w0 >> 16) & 255u, w0 >> 24,
                              w1 & 255u, (w1 >> 8) & 255u, (w1 >> 16) & 255u, w1 >> 24,
                              w2 & 255u, (w2 >> 8) & 255u, (w2 >> 16) & 255u, w2 >> 24};
      float o[12];
#pragma unroll
      for (int p = 0; p < 4; ++p) lab_of(s_lin, c[3 * p], c[3 * p + 1], c[3 * p + 2], o + 3 * p);
      s_out[3 * threadIdx.x] = make_float4(o[0], o[1], o[2], o[3]);
      s_out[3 * threadIdx.x + 1] = make_float4(o[4], o[5], o[6], o[7]);
      s_out[3 * threadIdx.x + 2] = make_float4(o[8], o[9], o[10], o[11]);
    }
    __syncthreads();
    const int64_t n4 = 3 * (min(groups, base + kThreads) - base);  // float4s of this chunk
    float4* dst = reinterpret_cast<float4*>(lab) + 3 * base;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int i = k * kThreads + (int)threadIdx.x;
      if (i < n4) dst[i] = s_out[i];
    }
    __syncthreads();
  }
}

// One pixel per thread, any alignment (pixels [p0, n)).
__global__ void __launch_bounds__(kThreads)
rgb_to_lab_kernel(const uint8_t* __restrict__ rgb, int64_t p0, int64_t n, float* __restrict__ lab) {
  __shared__ float s_lin[256];
  fill_lin(s_lin);
  for (int64_t p = p0 + blockIdx.x * (int64_t)kThreads + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * kThreads)
    lab_of(s_lin, rgb[3 * p], rgb[3 * p + 1], rgb[3 * p + 2], lab + 3 * p);
}

inline int grid_for(int64_t items) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((items + kThreads - 1) / kThreads, 4096));
}

}  // namespace

hipError_t launch_rgb_to_lab(const uint8_t* rgb, int64_t n, float* lab, hipStream_t s) {
  int64_t done = 0;
  if (reinterpret_cast<uintptr_t>(rgb) % 4 == 0 && reinterpret_cast<uintptr_t>(lab) % 16 == 0) {
    const int64_t groups = n / 4;
    if (groups > 0)
      rgb_to_lab_vec_kernel<<<grid_for(groups), kThreads, 0, s>>>(rgb, groups, lab);
    done = groups * 4;
  }
  if (done < n) rgb_to_lab_kernel<<<grid_for(n - done), kThreads, 0, s>>>(rgb, done, n, lab);
  return hipGetLastError();
}

}  // namespace sslic
