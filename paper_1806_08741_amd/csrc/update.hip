// update.hip -- the map step of the update (Sec. 3.1 stage 2): per-cluster
// sums of [1, x, I(x)] over the voxels carrying each label.
//
// A workgroup owns a tile of 64 columns (axis 0) by 64 rows (the other axes
// flattened).  Each lane walks one column of 16 rows and keeps a running sum
// for the current label (labels are spatially coherent, so runs are long);
// when the label changes the run is added into a small LDS hash table keyed
// by label.  At the end the table is added into the global per-cluster
// accumulators with one atomic per field and label present in the tile.
// Integer images and all coordinates are summed as 64-bit integers (exact);
// float32 channels in FP64.
#include "sslic_internal.h"

namespace sslic {

namespace {

constexpr int kThreads = 256;
constexpr int kCols = 64;
constexpr int kRowsPerWave = 16;
constexpr int kRows = kRowsPerWave * (kThreads / 64);
constexpr int kHash = 256;
constexpr int kMaxF = 1 + kMaxDim + kMaxChan;

template <bool FLT>
struct ChanSum {
  using type = uint64_t;
};
template <>
struct ChanSum<true> {
  using type = double;
};

__device__ __forceinline__ void add_global(const Geo& g, uint64_t* acc, int64_t key, int f, uint64_t v) {
  atomicAdd(reinterpret_cast<unsigned long long*>(acc + key * g.F + f), (unsigned long long)v);
}
__device__ __forceinline__ void add_global_f(const Geo& g, uint64_t* acc, int64_t key, int f, double v) {
  atomicAdd(reinterpret_cast<double*>(acc + key * g.F + f), v);
}

// 2D and 3D integer images with 1, 3 or 4 channels pack an LDS entry into
// few 64-bit words whose fields no tile can overflow.  The count is <= 4096
// (13 bits) and the sum of the tile-relative axis-0 coordinates <= 4096 * 63
// (18 bits); a channel sum is <= 4096 * 255 (20 bits) for u8 and
// <= 4096 * 65535 (28 bits) for u16.
//   2D: word 0 = count | sum x << 13 | sum y << 31 (y tile-relative too);
//   3D: word 0 = count | sum x << 13 | channel 0 << 31, word 1 = sum y |
//       sum z << 28 (absolute, 28 bits each, so n1 and n2 must be <= 65536;
//       a tile's rows run over y and z);
// the other channel sums follow, as many to a word as fit.  A run then adds
// into its entry with 2 or 3 LDS atomics instead of 1 + ND + C, and the entry
// is unpacked once per tile.
template <typename T, int ND, int CC>
struct Packing {
  static constexpr bool on = (ND == 2 || ND == 3) && !std::is_same<T, float>::value && CC > 0 &&
                             kCols == 64 && kRows == 64;
  static constexpr int CW = sizeof(T) == 1 ? 20 : 28;
  static constexpr int PW = 64 / CW;
  static constexpr int C0 = ND == 3 ? 1 : 0;  // channels in word 0
  static constexpr int CB = ND == 3 ? 2 : 1;  // first word of the other channels
  static constexpr int NCW = CC > 0 ? (CC - C0 + PW - 1) / PW : 1;
  __device__ static int word(int c) { return CB + (c - C0) / PW; }
  __device__ static int shift(int c) { return CW * ((c - C0) % PW); }
};

template <typename T, int ND, int CC>
__global__ void __launch_bounds__(kThreads)
update_kernel(Geo g, const T* __restrict__ img, const int32_t* __restrict__ labels, Iter it) {
  if (*it.done) return;
  constexpr bool FLT = std::is_same<T, float>::value;
  using CS = typename ChanSum<FLT>::type;
  const int C = CC > 0 ? CC : g.C;
  const int F = g.F;
  __shared__ int keys[kHash];
  __shared__ uint64_t vals[kHash * kMaxF];

  for (int i = threadIdx.x; i < kHash; i += kThreads) keys[i] = -1;
  for (int i = threadIdx.x; i < kHash * F; i += kThreads) vals[i] = 0;
  __syncthreads();

  const int n0 = g.n[0];
  const int64_t nrows = g.N / n0;
  const int tiles_x = (n0 + kCols - 1) / kCols;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int64_t tile = blockIdx.x;
  const int x = (int)(tile % tiles_x) * kCols + lane;
  const int64_t r0 = (tile / tiles_x) * kRows + (int64_t)wave * kRowsPerWave;
  using PK = Packing<T, ND, CC>;
  const bool pk = PK::on && (ND == 2 || (g.n[1] <= 65536 && g.n[2] <= 65536));
  const uint64_t x_org = (uint64_t)(tile % tiles_x) * kCols;  // tile origin (packed entries)
  const uint64_t y_org = (uint64_t)(tile / tiles_x) * kRows;

  int cur = -1;
  uint32_t cnt = 0;
  uint64_t sc[ND];
  CS sch[CC > 0 ? CC : kMaxChan];
  for (int i = 0; i < ND; ++i) sc[i] = 0;
  for (int c = 0; c < C; ++c) sch[c] = 0;

  auto flush = [&]() {
    if (cur < 0 || cur >= g.K || cnt == 0) return;
    uint32_t h = ((uint32_t)cur * 2654435761u) >> (32 - 8);  // kHash = 256
    int slot = -1;
    volatile int* vkeys = keys;
    for (int p = 0; p < kHash; ++p) {
      // a slot that already holds the label needs no atomic; an empty one is
      // claimed by compare-and-swap (keys are never removed)
      const int k = vkeys[h];
      if (k == cur) {
        slot = (int)h;
        break;
      }
      if (k == -1) {
        const int old = atomicCAS(&keys[h], -1, cur);
        if (old == -1 || old == cur) {
          slot = (int)h;
          break;
        }
      }
      h = (h + 1) & (kHash - 1);
    }
    if constexpr (PK::on) {
      if (pk) {
        // the run's axis-0 sum is tile-relative here (and in 2D its y sum)
        if (slot >= 0) {
          uint64_t w[PK::CB + PK::NCW];
#pragma unroll
          for (int j = 0; j < PK::CB + PK::NCW; ++j) w[j] = 0;
          w[0] = (uint64_t)cnt | sc[0] << 13;
          if constexpr (ND == 2) {
            w[0] |= sc[1] << 31;
          } else {
            w[0] |= (uint64_t)sch[0] << 31;
            w[1] = sc[1] | sc[2] << 28;
          }
#pragma unroll
          for (int c = PK::C0; c < CC; ++c) w[PK::word(c)] |= (uint64_t)sch[c] << PK::shift(c);
          uint64_t* vv = vals + slot * F;
#pragma unroll
          for (int j = 0; j < PK::CB + PK::NCW; ++j)
            atomicAdd(reinterpret_cast<unsigned long long*>(vv + j), (unsigned long long)w[j]);
        } else {
          add_global(g, it.acc, cur, 0, cnt);
          add_global(g, it.acc, cur, 1, sc[0] + cnt * x_org);
          if constexpr (ND == 2) {
            add_global(g, it.acc, cur, 2, sc[1] + cnt * y_org);
          } else {
            add_global(g, it.acc, cur, 2, sc[1]);
            add_global(g, it.acc, cur, 3, sc[2]);
          }
          for (int c = 0; c < C; ++c) add_global(g, it.acc, cur, 1 + ND + c, (uint64_t)sch[c]);
        }
        return;
      }
    }
    if (slot >= 0) {
      uint64_t* vv = vals + slot * F;
      atomicAdd(reinterpret_cast<unsigned long long*>(vv), (unsigned long long)cnt);
      for (int i = 0; i < ND; ++i) atomicAdd(reinterpret_cast<unsigned long long*>(vv + 1 + i), (unsigned long long)sc[i]);
      for (int c = 0; c < C; ++c) {
        if constexpr (FLT) atomicAdd(reinterpret_cast<double*>(vv + 1 + ND + c), (double)sch[c]);
        else atomicAdd(reinterpret_cast<unsigned long long*>(vv + 1 + ND + c), (unsigned long long)sch[c]);
      }
    } else {  // table full: straight to the global accumulators
      add_global(g, it.acc, cur, 0, cnt);
      for (int i = 0; i < ND; ++i) add_global(g, it.acc, cur, 1 + i, sc[i]);
      for (int c = 0; c < C; ++c) {
        if constexpr (FLT) add_global_f(g, it.acc, cur, 1 + ND + c, (double)sch[c]);
        else add_global(g, it.acc, cur, 1 + ND + c, (uint64_t)sch[c]);
      }
    }
  };

  if (x < n0) {
    // load the column's labels and values first, so the reads are in flight together
    using VT = typename std::conditional<FLT, float, uint32_t>::type;
    const int nr = (int)min((int64_t)kRowsPerWave, nrows - r0);
    int lab[kRowsPerWave];
    VT val[kRowsPerWave][CC > 0 ? CC : kMaxChan];
#pragma unroll
    for (int j = 0; j < kRowsPerWave; ++j) {
      lab[j] = -1;
      if (j < nr) {
        const int64_t v = (r0 + j) * n0 + x;
        lab[j] = labels[v];
        for (int c = 0; c < C; ++c) val[j][c] = (VT)img[v * C + c];
      }
    }
    int y[ND];  // coordinates of row r0 (axes 1..), advanced with carries
    {
      int64_t rr = r0;
      for (int i = 1; i < ND; ++i) {
        y[i] = (int)(rr % g.n[i]);
        rr /= g.n[i];
      }
    }
#pragma unroll
    for (int j = 0; j < kRowsPerWave; ++j) {
      if (j >= nr) continue;  // (no break: the loop must unroll to keep lab/val in registers)
      const int l = lab[j];
      if (l != cur) {
        flush();
        cur = l;
        cnt = 0;
        for (int i = 0; i < ND; ++i) sc[i] = 0;
        for (int c = 0; c < C; ++c) sch[c] = 0;
      }
      ++cnt;
      if (pk) {  // tile-relative axis 0 (and, in 2D, the row within the tile)
        sc[0] += (uint64_t)lane;
        if constexpr (ND == 2) sc[1] += (uint64_t)(wave * kRowsPerWave + j);
        else for (int i = 1; i < ND; ++i) sc[i] += (uint64_t)y[i];
      } else {
        sc[0] += (uint64_t)x;
        for (int i = 1; i < ND; ++i) sc[i] += (uint64_t)y[i];
      }
      for (int c = 0; c < C; ++c) sch[c] += (CS)val[j][c];
      for (int i = 1; i < ND; ++i) {
        if (++y[i] < g.n[i]) break;
        y[i] = 0;
      }
    }
    flush();
  }
  __syncthreads();
  for (int s = threadIdx.x; s < kHash; s += kThreads) {
    int key = keys[s];
    if (key < 0) continue;
    const uint64_t* vv = vals + s * F;
    if constexpr (PK::on) {
      if (pk) {
        const uint64_t w0 = vv[0];
        const uint64_t n = w0 & 0x1fffu;
        constexpr uint64_t m = (1ull << PK::CW) - 1;
        add_global(g, it.acc, key, 0, n);
        add_global(g, it.acc, key, 1, ((w0 >> 13) & 0x3ffffu) + n * x_org);
        if constexpr (ND == 2) {
          add_global(g, it.acc, key, 2, ((w0 >> 31) & 0x3ffffu) + n * y_org);
        } else {
          add_global(g, it.acc, key, 2, vv[1] & 0xfffffffu);
          add_global(g, it.acc, key, 3, vv[1] >> 28);
          add_global(g, it.acc, key, 1 + ND, (w0 >> 31) & m);
        }
#pragma unroll
        for (int c = PK::C0; c < CC; ++c)
          add_global(g, it.acc, key, 1 + ND + c, (vv[PK::word(c)] >> PK::shift(c)) & m);
        continue;
      }
    }
    add_global(g, it.acc, key, 0, vv[0]);
    for (int i = 0; i < ND; ++i) add_global(g, it.acc, key, 1 + i, vv[1 + i]);
    for (int c = 0; c < C; ++c) {
      if constexpr (FLT) add_global_f(g, it.acc, key, 1 + ND + c, __longlong_as_double((long long)vv[1 + ND + c]));
      else add_global(g, it.acc, key, 1 + ND + c, vv[1 + ND + c]);
    }
  }
}

template <typename T, int ND>
hipError_t dispatch_c(const Geo& g, const void* img, const int32_t* labels, const Iter& it,
                      hipStream_t s) {
  const int64_t tiles_x = (g.n[0] + kCols - 1) / kCols;
  const int64_t nrows = g.N / g.n[0];
  const int64_t nb = tiles_x * ((nrows + kRows - 1) / kRows);
  const T* p = (const T*)img;
  switch (g.C) {
    case 1: update_kernel<T, ND, 1><<<(unsigned)nb, kThreads, 0, s>>>(g, p, labels, it); break;
    case 3: update_kernel<T, ND, 3><<<(unsigned)nb, kThreads, 0, s>>>(g, p, labels, it); break;
    case 4: update_kernel<T, ND, 4><<<(unsigned)nb, kThreads, 0, s>>>(g, p, labels, it); break;
    default: update_kernel<T, ND, 0><<<(unsigned)nb, kThreads, 0, s>>>(g, p, labels, it); break;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t dispatch_nd(const Geo& g, const void* img, const int32_t* labels, const Iter& it,
                       hipStream_t s) {
  switch (g.nd) {
    case 2: return dispatch_c<T, 2>(g, img, labels, it, s);
    case 3: return dispatch_c<T, 3>(g, img, labels, it, s);
    default: return dispatch_c<T, 4>(g, img, labels, it, s);
  }
}

}  // namespace

hipError_t launch_update(const Geo& g, const void* img, const int32_t* labels, const Iter& it,
                         hipStream_t s) {
  switch (g.dtype) {
    case kU8: return dispatch_nd<uint8_t>(g, img, labels, it, s);
    case kU16: return dispatch_nd<uint16_t>(g, img, labels, it, s);
    default: return dispatch_nd<float>(g, img, labels, it, s);
  }
}

}  // namespace sslic
