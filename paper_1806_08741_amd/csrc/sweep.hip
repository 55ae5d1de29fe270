// sweep.hip -- one pass over the image per iteration: the assignment step
// (Sec. 2.1 distance, Sec. 3.1 stage 2) and the map half of the update (per
// cluster sums of [1, x, I(x)]) in the same kernel, so the image is read once
// and the labels written once per iteration.
//
// Work decomposition
//   * A workgroup owns a tile (2D 64x64, 3D 32x32x32, 4D 16x16x8x8); each of
//     its four waves sweeps rows of blocks of 64 voxels (8x8, 4x4x4,
//     4x4x2x2) along axis 0, one voxel per lane.
//   * Candidates, one centre record per lane: either the tile's table (the
//     centres whose window meets the tile, when at most 64; lane l holds
//     entry l), or per row of blocks the records of the bins within one bin
//     of the row (a row of bins is one contiguous range of the bin-ordered
//     item list).  For a block, each lane tests whether its centre's window
//     meets the block and whether it covers it, and ballots keep the meeting
//     ones.  The wave then takes them one by one (s_ff1 on the ballot) and
//     reads each record with scalar loads, so the means and scaled
//     coordinates are scalar operands of the distance:
//       D^2 = sum_i (x_i m / S_i - c'_i)^2 + sum_c (I_c - mu_c)^2   (FP32).
//     The best is one 64-bit key (bits of D, then the cluster index, or the
//     index and the holding lane), so among equal distances the lowest
//     index wins.
//   * Each lane keeps a running sum for its current label across the blocks
//     of its run (labels are spatially coherent); when the label changes the
//     run is added to the tile's LDS sum table: at the winner's table entry,
//     or at the entry a hash of the label finds.
//   * At the end the table goes to global memory without atomics: each
//     cluster has 2^n slots, one per tile its window can meet (a window spans
//     at most two tiles per axis when the tile is at least 2S+1 wide), chosen
//     by the tile's offset from the tile that holds the window's low corner,
//     and tagged with the iteration.  Sums for labels outside the window's
//     tiles (voxels that no window reached keep an older label) and every
//     sum when the tiles are too small for slots go through 64-bit atomics
//     into the plain accumulators instead, which are flagged per cluster.
#include "sslic_internal.h"

namespace sslic {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

// Tile shapes: VAR 0 is the default; VAR 1 is a smaller tile that the batch
// autotuner may pick for small images.
template <int ND, int VAR>
struct Shape;
template <>
struct Shape<2, 0> {
  static constexpr int T[2] = {64, 64};
  static constexpr int B[2] = {8, 8};
  static constexpr int kHash = 256;
};
template <>
struct Shape<2, 1> {
  static constexpr int T[2] = {32, 32};
  static constexpr int B[2] = {8, 8};
  static constexpr int kHash = 128;
};
template <>
struct Shape<3, 0> {
  static constexpr int T[3] = {32, 32, 32};
  static constexpr int B[3] = {4, 4, 4};
  static constexpr int kHash = 512;
};
template <>
struct Shape<3, 1> {
  static constexpr int T[3] = {16, 16, 16};
  static constexpr int B[3] = {4, 4, 4};
  static constexpr int kHash = 256;
};
template <>
struct Shape<4, 0> {
  static constexpr int T[4] = {16, 16, 8, 8};
  static constexpr int B[4] = {4, 4, 2, 2};
  static constexpr int kHash = 512;
};
template <>
struct Shape<4, 1> {
  static constexpr int T[4] = {8, 8, 8, 8};
  static constexpr int B[4] = {4, 4, 2, 2};
  static constexpr int kHash = 256;
};

template <class SH, int ND>
__host__ __device__ constexpr int blocks_per_tile() {
  int n = 1;
  for (int i = 0; i < ND; ++i) n *= SH::T[i] / SH::B[i];
  return n;
}

__device__ __forceinline__ int grid_label(const Geo& g, const int* x, int nd) {
  int64_t kk = 0, kst = 1;
  for (int i = 0; i < nd; ++i) {
    kk += ((int64_t)x[i] * g.Ka[i] / g.n[i]) * kst;
    kst *= g.Ka[i];
  }
  return (int)kk;
}

// Per-tile sums of one cluster share few 64-bit LDS words: the voxel count,
// the coordinate sums relative to the tile and, for integer images with a
// compile-time channel count, the channel sums.  Each field is as wide as a
// whole tile's sum can get, so adding packed words never carries from one
// field into the next, and a flush costs one atomic per word.
__host__ __device__ constexpr int bits_for(uint64_t v) {
  int b = 0;
  while (v) {
    ++b;
    v >>= 1;
  }
  return b;
}

template <typename T, int ND, int CC, class SH>
struct TilePack {
  static constexpr bool kPackCh = !std::is_same<T, float>::value && CC > 0;
  static constexpr int kFields = 1 + ND + (kPackCh ? CC : 0);
  int word[1 + ND + 4];
  int shift[1 + ND + 4];
  int width[1 + ND + 4];
  int nw;
  int maxw;  // widest field (bits)
  constexpr TilePack() : word(), shift(), width(), nw(0), maxw(0) {
    uint64_t vox = 1;
    for (int i = 0; i < ND; ++i) vox *= (uint64_t)SH::T[i];
    const uint64_t vmax = std::is_same<T, uint8_t>::value ? 255u : 65535u;
    int w = 0, used = 0;
    for (int f = 0; f < kFields; ++f) {
      const uint64_t mx = f == 0 ? vox : f <= ND ? (uint64_t)(SH::T[f - 1] - 1) * vox : vmax * vox;
      const int b = bits_for(mx);
      if (used + b > 64) {
        ++w;
        used = 0;
      }
      word[f] = w;
      shift[f] = used;
      width[f] = b;
      maxw = b > maxw ? b : maxw;
      used += b;
    }
    nw = w + 1;
  }
  __device__ static uint64_t field(const uint64_t* pw, int f) {
    constexpr TilePack p{};
    const int hi = f + 1 < kFields && p.word[f + 1] == p.word[f] ? p.shift[f + 1] : 64;
    const uint64_t v = pw[p.word[f]] >> p.shift[f];
    return hi - p.shift[f] >= 64 ? v : v & ((1ull << (hi - p.shift[f])) - 1);
  }
};

// 64-bit LDS words per table entry
template <typename T, int ND, int CC, class SH>
__host__ __device__ constexpr int entry_words() {
  using PK = TilePack<T, ND, CC, SH>;
  return PK{}.nw + (PK::kPackCh ? 0 : (CC > 0 ? CC : kMaxChan));
}

template <bool FLT>
struct RunSum {
  using type = uint32_t;
};
template <>
struct RunSum<true> {
  using type = double;
};

// The packed words of one run (count, tile-relative coordinate sums and, for
// packed channels, channel sums) assembled on 32-bit halves; each value is
// below 2^width of its field, and no field is wider than 32 bits.
template <class PK>
__device__ __forceinline__ void pack_run(const uint32_t* v, uint64_t* pw) {
  constexpr PK pk{};
  static_assert(pk.maxw <= 32, "a run's field must fit 32 bits");
  uint32_t lo[pk.nw], hi[pk.nw];
#pragma unroll
  for (int w = 0; w < pk.nw; ++w) lo[w] = hi[w] = 0;
#pragma unroll
  for (int f = 0; f < PK::kFields; ++f) {
    const int w = pk.word[f], s = pk.shift[f];
    if (s >= 32) {
      hi[w] |= v[f] << (s - 32);
    } else {
      lo[w] |= v[f] << s;
      if (s + pk.width[f] > 32) hi[w] |= v[f] >> (32 - s);
    }
  }
#pragma unroll
  for (int w = 0; w < pk.nw; ++w) pw[w] = (uint64_t)hi[w] << 32 | lo[w];
}

__device__ __forceinline__ int lanes_below(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// One tile of the sweep: the assignment of its voxels and, with ACC, the
// per-cluster sums of the tile into the cluster's tile slot or accumulators.
//
// TBL (with ACC): the workgroup first lists every centre whose window meets
// the tile (from the bins within one bin of the tile), at most 64, in an LDS
// table: lane l of every wave holds entry l, which is also the cluster's
// entry in the sum table.  The rows of blocks take their candidates from the
// lanes, and the best candidate's key carries (k << 6 | lane), so the
// winner's entry is known without a lookup, and among equal distances the
// lowest k still wins.  Returns false, before any label is written, when more
// than 64 centres meet the tile; the caller then runs the hashed form (TBL
// false), whose sum table is keyed by label and filled from the bins of each
// row.
//
// s_keys: record index per entry (TBL) or hash keys (labels); s_vals: the
// packed sums per entry; s_tb: per axis, the window bounds relative to the
// tile, clamped to [-1, T] and biased by 1, low | high << 16 (TBL); s_n: the
// entry count (TBL).
template <typename T, int ND, int CC, bool ACC, class SH, bool TBL>
__device__ __forceinline__ bool sweep_tile(const Geo& g, const T* __restrict__ img,
                                           const int32_t* __restrict__ bstart,
                                           const int32_t* __restrict__ items,
                                           const float* __restrict__ recs, const SweepArgs& a,
                                           int iter, int tile, int* s_keys, uint64_t* s_vals,
                                           uint32_t* s_tb, int* s_n) {
  static_assert(ACC || !TBL, "the table form accumulates");
  using SS = SH;
  constexpr int CM = CC > 0 ? CC : kMaxChan;
  constexpr int RN = CM + 3 * ND + 1;  // record words read
  constexpr int HS = SS::kHash;
  constexpr int FM = 1 + ND + CM;
  constexpr bool FLT = std::is_same<T, float>::value;
  using RT = typename RunSum<FLT>::type;
  const int C = CC > 0 ? CC : g.C;
  const int RS = g.rs;
  const int F = 1 + ND + C;

  using PK = TilePack<T, ND, CC, SH>;
  constexpr PK pk{};
  constexpr int NW = pk.nw;                          // packed words per entry
  const int EW = NW + (PK::kPackCh ? 0 : C);         // + unpacked channel sums

  const int tid = threadIdx.x, lane = tid % 64;
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);

  int to[ND], tc[ND];
  {
    int r = tile;
    for (int i = 0; i < ND; ++i) {
      tc[i] = r % a.nt[i];
      r /= a.nt[i];
      to[i] = tc[i] * SS::T[i];
    }
  }
  int lx[ND];
  {
    int r = lane;
    for (int i = 0; i < ND; ++i) {
      lx[i] = r % SS::B[i];
      r /= SS::B[i];
    }
  }

  if constexpr (ACC) {
    if constexpr (!TBL) {
      for (int i = tid; i < HS; i += kThreads) s_keys[i] = -1;
    } else {
      if (tid == 0) *s_n = 0;
    }
    for (int i = tid; i < HS * EW; i += kThreads) s_vals[i] = 0;
    __syncthreads();
  }

  // --- TBL: the centres whose window meets the tile ---------------------------
  int n = 0;
  if constexpr (TBL) {
    int tl[ND], th[ND], b0[ND], b1[ND];
    int nrows = 1;
    for (int i = 0; i < ND; ++i) {
      tl[i] = to[i];
      th[i] = min(to[i] + SS::T[i], g.n[i]) - 1;
      b0[i] = max(tl[i] / g.S[i] - 1, 0);
      b1[i] = min(th[i] / g.S[i] + 1, g.nb[i] - 1);
      if (i > 0) nrows *= b1[i] - b0[i] + 1;
    }
    for (int r = wave; r < nrows; r += kWaves) {  // one row of bins along axis 0 at a time
      int bl = b0[0] * (int)g.bst[0], rr = r;
      for (int i = 1; i < ND; ++i) {
        const int w = b1[i] - b0[i] + 1;
        bl += (b0[i] + rr % w) * (int)g.bst[i];
        rr /= w;
      }
      const int ja = bstart[bl], jb = bstart[bl + (b1[0] - b0[0]) + 1];
      for (int j0 = ja; j0 < jb; j0 += 64) {
        const int j = j0 + lane;
        bool keep = j < jb;
        int rk = 0;
        uint32_t pb[ND];
        if (keep) {
          rk = items[j];
          const int* irec = reinterpret_cast<const int*>(recs + (int64_t)rk * RS);
#pragma unroll
          for (int i = 0; i < ND; ++i) {
            const int lo = irec[rec_lo(C, ND) + i], hi = irec[rec_hi(C, ND) + i];
            keep = keep && lo <= th[i] && hi >= tl[i];
            const int rl = lo < to[i] ? -1 : min(lo - to[i], SS::T[i]);
            const int rh = hi < to[i] ? -1 : min(hi - to[i], SS::T[i]);
            pb[i] = (uint32_t)(rl + 1) | (uint32_t)(rh + 1) << 16;
          }
        }
        const uint64_t m = __ballot(keep);
        if (m == 0) continue;
        int base = 0;
        if (lane == 0) base = atomicAdd(s_n, (int)__popcll(m));
        base = __builtin_amdgcn_readlane(base, 0);
        if (keep) {
          const int p = base + lanes_below(m);
          if (p < 64) {
            s_keys[p] = rk;
#pragma unroll
            for (int i = 0; i < ND; ++i) s_tb[i * 64 + p] = pb[i];
          }
        }
      }
    }
    __syncthreads();
    n = __builtin_amdgcn_readfirstlane(*s_n);
    if (n > 64) return false;
  }

  // running sum of this lane's current label (coordinates relative to the tile)
  int cur = -1, cslot = -1;
  uint32_t rcnt = 0;
  uint32_t rco[ND];
  RT rch[CM];
  for (int i = 0; i < ND; ++i) rco[i] = 0;
  for (int c = 0; c < C; ++c) rch[c] = 0;

  auto flush = [&]() {
    if (cur < 0 || rcnt == 0) return;
    int slot = -1;
    if constexpr (TBL) {
      slot = cslot;
    } else {
      uint32_t h = ((uint32_t)cur * 2654435761u) >> 8;
      for (int p = 0; p < HS; ++p) {
        h &= HS - 1;
        int old = s_keys[h];  // a key once written stays: look before inserting
        if (old == -1) old = atomicCAS(&s_keys[h], -1, cur);
        if (old == -1 || old == cur) {
          slot = (int)h;
          break;
        }
        ++h;
      }
    }
    if (slot >= 0) {
      uint32_t v[PK::kFields];
      v[0] = rcnt;
#pragma unroll
      for (int i = 0; i < ND; ++i) v[1 + i] = rco[i];
      unsigned long long* vv = reinterpret_cast<unsigned long long*>(s_vals + slot * EW);
      if constexpr (PK::kPackCh) {
#pragma unroll
        for (int c = 0; c < CM; ++c) v[1 + ND + c] = (uint32_t)rch[c];
      } else {
        for (int c = 0; c < C; ++c) {
          if constexpr (FLT) atomicAdd(reinterpret_cast<double*>(vv + NW + c), (double)rch[c]);
          else atomicAdd(vv + NW + c, (unsigned long long)rch[c]);
        }
      }
      uint64_t pw[NW];
      pack_run<PK>(v, pw);
#pragma unroll
      for (int w = 0; w < NW; ++w) atomicAdd(vv + w, (unsigned long long)pw[w]);
    } else {  // no table entry: global accumulators (coordinates made absolute)
      a.accf[cur] = 1;
      unsigned long long* gg = reinterpret_cast<unsigned long long*>(a.acc + (int64_t)cur * F);
      atomicAdd(gg, (unsigned long long)rcnt);
      for (int i = 0; i < ND; ++i)
        atomicAdd(gg + 1 + i, (unsigned long long)rco[i] + (unsigned long long)rcnt * to[i]);
      for (int c = 0; c < C; ++c) {
        if constexpr (FLT) atomicAdd(reinterpret_cast<double*>(gg + 1 + ND + c), (double)rch[c]);
        else atomicAdd(gg + 1 + ND + c, (unsigned long long)rch[c]);
      }
    }
  };

  // Lane-parallel gather: lane i <- position of the i-th record in the bins
  // b0..b1 (rows of bins along axis 0 are contiguous in the record array).
  auto gather = [&](const int* b0, const int* b1, int& jl) {
    int cnt = 0;
    int rc[ND];
    for (int i = 1; i < ND; ++i) rc[i] = b0[i];
    while (true) {
      int bl = b0[0] * (int)g.bst[0];
      for (int i = 1; i < ND; ++i) bl += rc[i] * (int)g.bst[i];
      const int ja = bstart[bl];
      const int jb = bstart[bl + (b1[0] - b0[0]) + 1];
      if (lane >= cnt && lane < cnt + (jb - ja)) jl = ja + lane - cnt;
      cnt += jb - ja;
      int i = 1;
      while (i < ND) {
        if (++rc[i] <= b1[i]) break;
        rc[i] = b0[i];
        ++i;
      }
      if (i >= ND) break;
    }
    return cnt;
  };

  // The best candidate so far is one 64-bit key: the bits of D (never
  // negative, so they order as the values do) above the candidate's id, so
  // the smaller key is the smaller D and, among equal D, the lower id.  The
  // id is the cluster index, or (index << 6 | holding lane) when TBL rows
  // find candidates in the table (same order: indices are distinct).
  auto pick = [&](float D, uint32_t id, uint64_t& bkey) {
    const uint64_t key = ((uint64_t)__float_as_uint(D) << 32) | id;
    bkey = key < bkey ? key : bkey;
  };

  // The meeting centres of a block, one at a time (their records are scalar
  // loads of record readlane(jr, l), addressed in 64 bits).  Centres whose window covers the
  // whole block (mask mf) need no window test; for the others (mask mc) the
  // closed window is tested on every axis as one unsigned range compare.
  auto scan = [&](uint64_t mf, uint64_t mc, int jr, const int* x, const float* xs,
                  const float* I, bool tagl, uint64_t& bkey) {
    constexpr int RF = CM + ND + 1;  // mu, c', k
    while (mf) {
      const int l = (int)__builtin_ctzll(mf);
      mf &= mf - 1;
      const uint32_t rk = (uint32_t)__builtin_amdgcn_readlane(jr, l);
      const float* rec = recs + (uint64_t)rk * (uint32_t)RS;
      float R[RF];
#pragma unroll
      for (int w = 0; w < RF; ++w) R[w] = (CC > 0 || w < RS) ? rec[w] : 0.0f;
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
      const uint32_t k = CC > 0 ? __float_as_uint(R[rec_k(CC, ND)])
                                : reinterpret_cast<const uint32_t*>(rec)[rec_k(C, ND)];
      pick(D, tagl ? k << 6 | (uint32_t)l : k, bkey);
    }
    while (mc) {
      const int l = (int)__builtin_ctzll(mc);
      mc &= mc - 1;
      const uint32_t rk = (uint32_t)__builtin_amdgcn_readlane(jr, l);
      const float* rec = recs + (uint64_t)rk * (uint32_t)RS;
      float R[RN];
#pragma unroll
      for (int w = 0; w < RN; ++w) R[w] = (CC > 0 || w < RS) ? rec[w] : 0.0f;
      const int* Ri = reinterpret_cast<const int*>(R);
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
      bool ok = true;
#pragma unroll
      for (int i = 0; i < ND; ++i) {
        const int lo = Ri[rec_lo(C, ND) + i], hi = Ri[rec_hi(C, ND) + i];
        ok &= (uint32_t)(x[i] - lo) <= (uint32_t)(hi - lo);
      }
      D = ok ? D : __builtin_inff();
      const uint32_t k = (uint32_t)Ri[rec_k(C, ND)];
      pick(D, tagl ? k << 6 | (uint32_t)l : k, bkey);
    }
  };

  // meets / covers test of the record held by this lane against a block box
  auto test = [&](bool held, const int* lo, const int* hi, const int* blo, const int* bhi,
                  uint64_t& mf, uint64_t& mc) {
    bool meets = held, covers = true;  // bitwise: the compares combine as masks
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      meets &= (lo[i] <= bhi[i]) & (hi[i] >= blo[i]);
      covers &= (lo[i] <= blo[i]) & (hi[i] >= bhi[i]);
    }
    const uint64_t m = __ballot(meets), cv = __ballot(covers);
    mf = m & cv;
    mc = m & ~cv;
  };

  constexpr int BX = SS::T[0] / SS::B[0];            // blocks per row (axis 0)
  constexpr int NROW = blocks_per_tile<SS, ND>() / BX;  // block rows per tile
  static_assert(NROW % kWaves == 0, "rows must split evenly over waves");
  constexpr int RPW = NROW / kWaves;

  for (int rw = 0; rw < RPW; ++rw) {
    // a row of blocks along axis 0 across the tile
    int rlo[ND], rhi[ND];
    bool rin = true;
    {
      int r = wave * RPW + rw;
      rlo[0] = to[0];
      rhi[0] = min(to[0] + SS::T[0], g.n[0]) - 1;
      for (int i = 1; i < ND; ++i) {
        const int nbk = SS::T[i] / SS::B[i];
        rlo[i] = to[i] + (r % nbk) * SS::B[i];
        r /= nbk;
        rin = rin && rlo[i] < g.n[i];
        rhi[i] = min(rlo[i] + SS::B[i], g.n[i]) - 1;
      }
    }
    if (!rin) continue;
    // the row's candidates, one per lane: the lane's record index, window
    // bounds (tile-relative for TBL) and, for TBL, its table entry
    bool rowfit, held;
    int hrk, hslot = 0;
    int hlo[ND], hhi[ND];
    if constexpr (TBL) {  // lane l holds entry l
      rowfit = true;
      held = lane < n;
      hslot = held ? lane : 0;
      hrk = held ? s_keys[hslot] : 0;
#pragma unroll
      for (int i = 0; i < ND; ++i) {
        const uint32_t pbv = s_tb[i * 64 + hslot];
        hlo[i] = (int)(pbv & 0xffffu) - 1;
        hhi[i] = (int)(pbv >> 16) - 1;
      }
    } else {
      // the records of the bins within one bin of the row
      int rb0[ND], rb1[ND];
      for (int i = 0; i < ND; ++i) {
        rb0[i] = max(rlo[i] / g.S[i] - 1, 0);
        rb1[i] = min(rhi[i] / g.S[i] + 1, g.nb[i] - 1);
      }
      int rjl = 0;
      const int nrec = gather(rb0, rb1, rjl);
      rowfit = nrec <= 64;
      held = rowfit && lane < nrec;
      hrk = items[held ? rjl : 0];  // the record of the cluster at that bin position
      const int* irec = reinterpret_cast<const int*>(recs + (int64_t)hrk * RS);
#pragma unroll
      for (int i = 0; i < ND; ++i) {
        hlo[i] = irec[rec_lo(C, ND) + i];
        hhi[i] = irec[rec_hi(C, ND) + i];
      }
    }

    // This lane's voxel in block 0 of the row; block bx is B_0 * bx voxels
    // further along axis 0.  Lanes outside the image read (and never write)
    // the first voxel of their block.
    int x[ND];
    float xs[ND];
    bool rowok = true;
    for (int i = 1; i < ND; ++i) {
      x[i] = rlo[i] + lx[i];
      rowok = rowok && x[i] <= rhi[i];
      xs[i] = (float)x[i] * g.sw[i];
    }
    int64_t vrow = to[0];
    for (int i = 1; i < ND; ++i) vrow += (int64_t)(rowok ? x[i] : rlo[i]) * g.st[i];
    const int lx0 = rowok ? lx[0] : 0;
    const T* prow = img + (vrow + lx0) * C;
    int32_t* lrow = a.labels + vrow + lx0;

    for (int bx = 0; bx < BX; ++bx) {
      int blo[ND], bhi[ND];
      blo[0] = to[0] + bx * SS::B[0];
      if (blo[0] >= g.n[0]) break;
      bhi[0] = min(blo[0] + SS::B[0], g.n[0]) - 1;
      for (int i = 1; i < ND; ++i) {
        blo[i] = rlo[i];
        bhi[i] = rhi[i];
      }
      x[0] = blo[0] + lx[0];
      const bool okx = x[0] <= bhi[0];
      const bool valid = rowok && okx;
      xs[0] = (float)x[0] * g.sw[0];
      const int step = bx * SS::B[0] - (okx ? 0 : lx0);
      const T* px = prow + (int64_t)step * C;
      int32_t* lp = lrow + step;
      float I[CM];
      for (int c = 0; c < C; ++c) I[c] = (float)px[c];

      // no candidate yet: FLT_MAX; out-of-window distances (+inf) never win
      constexpr uint64_t kNone = (uint64_t)0x7f7fffffu << 32 | 0xffffffffu;
      uint64_t bkey = kNone;
      if (rowfit) {
        uint64_t mf, mc;
        if constexpr (TBL) {
          int qlo[ND], qhi[ND];
          for (int i = 0; i < ND; ++i) {
            qlo[i] = blo[i] - to[i];
            qhi[i] = bhi[i] - to[i];
          }
          test(held, hlo, hhi, qlo, qhi, mf, mc);
        } else {
          test(held, hlo, hhi, blo, bhi, mf, mc);
        }
        scan(mf, mc, hrk, x, xs, I, TBL, bkey);
      } else {
        int b0[ND], b1[ND];
        for (int i = 0; i < ND; ++i) {
          b0[i] = max(blo[i] / g.S[i] - 1, 0);
          b1[i] = min(bhi[i] / g.S[i] + 1, g.nb[i] - 1);
        }
        int jl = 0;
        const int cnt = gather(b0, b1, jl);
        if (cnt <= 64) {
          const bool bheld = lane < cnt;
          int lo[ND], hi[ND];
          const int bk0 = items[bheld ? jl : 0];
          const int* irec = reinterpret_cast<const int*>(recs + (int64_t)bk0 * RS);
          for (int i = 0; i < ND; ++i) {
            lo[i] = irec[rec_lo(C, ND) + i];
            hi[i] = irec[rec_hi(C, ND) + i];
          }
          uint64_t mf, mc;
          test(bheld, lo, hi, blo, bhi, mf, mc);
          scan(mf, mc, bk0, x, xs, I, false, bkey);
        } else {
          // more centres than lanes (a crowded neighbourhood): each lane walks them
          int rc[ND];
          for (int i = 1; i < ND; ++i) rc[i] = b0[i];
          while (true) {
            int bl = b0[0] * (int)g.bst[0];
            for (int i = 1; i < ND; ++i) bl += rc[i] * (int)g.bst[i];
            const int ja = bstart[bl];
            const int jb = bstart[bl + (b1[0] - b0[0]) + 1];
            for (int j = ja; j < jb; ++j) {
              const float* rec = recs + (int64_t)items[j] * RS;
              const int* irec2 = reinterpret_cast<const int*>(rec);
              bool ok = true;
              for (int i = 0; i < ND; ++i)
                ok = ok && x[i] >= irec2[rec_lo(C, ND) + i] && x[i] <= irec2[rec_hi(C, ND) + i];
              if (!ok) continue;
              float D;
              for (int i = 0; i < ND; ++i) {
                const float d = xs[i] - rec[C + i];
                D = i == 0 ? d * d : fmaf(d, d, D);
              }
              for (int c = 0; c < C; ++c) {
                const float t = I[c] - rec[c];
                D = fmaf(t, t, D);
              }
              pick(D, (uint32_t)irec2[rec_k(C, ND)], bkey);
            }
            int i = 1;
            while (i < ND) {
              if (++rc[i] <= b1[i]) break;
              rc[i] = b0[i];
              ++i;
            }
            if (i >= ND) break;
          }
        }
      }
      int bk = bkey == kNone ? -1 : (int)(uint32_t)bkey;
      int bslot = -1;
      if constexpr (TBL) {
        if (rowfit) {  // the key holds (k << 6 | lane of the winner's entry)
          const uint32_t id = (uint32_t)bkey;
          if (bk >= 0) {
            bk = (int)(id >> 6);
            bslot = (int)(id & 63u);  // lane l holds entry l
          }
        }
      }
      if (valid) {
        if (bk < 0) bk = iter == 0 ? grid_label(g, x, ND) : *lp;
        *lp = bk;
        if constexpr (ACC) {
          if (bk != cur || (TBL && bslot != cslot)) {
            flush();
            cur = bk;
            cslot = bslot;
            rcnt = 0;
            for (int i = 0; i < ND; ++i) rco[i] = 0;
            for (int c = 0; c < C; ++c) rch[c] = 0;
          }
          ++rcnt;
          for (int i = 0; i < ND; ++i) rco[i] += (uint32_t)(x[i] - to[i]);
          for (int c = 0; c < C; ++c) {
            if constexpr (FLT) rch[c] += (double)I[c];
            else rch[c] += (uint32_t)I[c];
          }
        }
      }
    }
  }
  if constexpr (!ACC) {
    return true;
  } else {
  flush();
  __syncthreads();

  // --- the tile's sums to their cluster slots -------------------------------
  constexpr int NS = 1 << ND;
  for (int s = tid; s < (TBL ? n : HS); s += kThreads) {
    int k;
    if constexpr (TBL) {
      k = reinterpret_cast<const int*>(recs + (int64_t)s_keys[s] * RS)[rec_k(C, ND)];
    } else {
      k = s_keys[s];
      if (k < 0) continue;
    }
    const uint64_t* vv = s_vals + s * EW;
    const uint64_t nn = PK::field(vv, 0);
    if (nn == 0) continue;  // a table entry no voxel of the tile took
    uint64_t out[FM];
    out[0] = nn;
    for (int i = 0; i < ND; ++i) out[1 + i] = PK::field(vv, 1 + i) + nn * (uint64_t)to[i];
    if constexpr (PK::kPackCh) {
      for (int c = 0; c < CM; ++c) out[1 + ND + c] = PK::field(vv, 1 + ND + c);
    } else {
      for (int c = 0; c < C; ++c) out[1 + ND + c] = vv[NW + c];
    }
    int q = -1;
    if (a.slots) {
      const int* irec = reinterpret_cast<const int*>(a.ctab + (int64_t)k * g.rs);
      q = 0;
      for (int i = 0; i < ND; ++i) {
        const int lo = max(irec[rec_lo(g.C, g.nd) + i], 0), hi = min(irec[rec_hi(g.C, g.nd) + i], g.n[i] - 1);
        const int t0 = lo / SS::T[i];
        const int d = tc[i] - t0;
        const bool meets = to[i] <= hi && to[i] + SS::T[i] - 1 >= lo;
        if (!meets || d < 0 || d > 1) {
          q = -1;
          break;
        }
        q |= d << i;
      }
    }
    if (q >= 0) {  // the slot, tagged with the iteration that wrote it
      uint64_t* dst = a.part + ((int64_t)k * NS + q) * (F + 1);
      for (int f = 0; f < F; ++f) dst[f] = out[f];
      dst[F] = (uint64_t)(iter + 1);
    } else {
      a.accf[k] = 1;
      unsigned long long* gg = reinterpret_cast<unsigned long long*>(a.acc + (int64_t)k * F);
      for (int f = 0; f < 1 + ND; ++f) atomicAdd(gg + f, (unsigned long long)out[f]);
      for (int c = 0; c < C; ++c) {
        if constexpr (FLT) atomicAdd(reinterpret_cast<double*>(gg + 1 + ND + c), __longlong_as_double((long long)out[1 + ND + c]));
        else atomicAdd(gg + 1 + ND + c, (unsigned long long)out[1 + ND + c]);
      }
    }
  }
  return true;
  }
}

// ---------------------------------------------------------------------------
// Fast form for 3D integer images with up to 3 channels.
//
// The workgroup first lists in LDS every centre whose window meets its tile
// (from the bins within one bin of the tile), in ascending cluster index,
// with its distance terms relative to the tile's centre o.  With
//   xs_i = (x_i - o_i) m / S_i,   c_i = c'_i - o_i m / S_i,
//   D^2 - |xs|^2 = |c|^2 - 2 c . xs + |I - mu|^2,
// a candidate costs one FMA per axis and two operations per channel; |xs|^2
// is the same for every centre a voxel compares, so the argmin is that of
// D^2.  Each wave then sweeps rows of blocks (8 blocks of 4x4x4 voxels
// along axis 0, one voxel per lane, each lane holding its 8 voxels of the
// row): the table indices of the entries meeting the row form the wave's
// row list, and the wave walks that list once, entry by entry with its
// terms read from the table as wave-uniform values.  An entry's terms along
// axes 1 and 2, and along axis 0 at the row's first block, are summed once
// for the row; each block its window meets then costs one FMA for axis 0
// (a multiple of one per-entry step), two operations per channel, a select
// that gives lanes outside the window an infinite distance, a compare and
// two selects.  The lane mask is formed in scalar registers from the
// entry's coverage bits.  Because the list is in ascending cluster index
// and the compare is strict, equal distances go to the lowest index.
//
// Map step: every voxel adds its packed [1, x - o, I] to its winner's table
// entry with LDS atomics (no per-lane runs, no hashing: the winner's entry
// is its table index).  Labels are staged per row in LDS and leave as whole
// lines.  At the end the table goes to the cluster slots as in the other
// forms.  Returns false before writing anything when the tile's table would
// not fit (crowded centres); the caller then runs the general form.
template <int ND>
struct Fast;
template <>
struct Fast<3> {
  static constexpr int T[3] = {32, 32, 32};
  static constexpr int B[3] = {4, 4, 4};
  static constexpr int kTab = 320;      // table entries
  static constexpr int kBinRows = 256;  // bin rows (along axis 0) scanned for the table
  static constexpr int kRep = 1;        // copies of the sums (lanes alternate between them)
};

// Where the fast form is used: 3D integer images with 1 to 3 channels.  (Its
// 2D variants measured slower than the general form on the 16384^2 slide,
// 1.40 ms: block by block 1.54-1.57 ms, and as this row walk on 64x64 tiles
// 2.18 ms, a tile of 64 blocks paying for a whole table.)
template <typename T, int ND, int CC>
constexpr bool fast_ok() {
  return !std::is_same<T, float>::value && ND == 3 && CC > 0 && 1 + ND + CC <= 7;
}

template <typename T, int ND, int CC>
struct FastLds {
  using SH = Fast<ND>;
  using PK = TilePack<T, ND, CC, SH>;
  static constexpr int NW = PK{}.nw;
  alignas(16) float rec[SH::kTab][8];  // q, -2 c_i (ND), mu_c (C), entry index (int bits)
  int kk[SH::kTab];        // cluster index of each entry
  uint16_t tb[ND][SH::kTab];  // window bounds relative to the tile, (lo + 1) | (hi + 1) << 8
  // the rows of blocks each entry's window meets: bit b (axis 1) and bit 8 + b
  // (axis 2) for the b-th block along that axis
  uint32_t rb[SH::kTab];
  // packed sums of the tile's voxels per entry, in kRep copies: lane l adds
  // to copy l mod kRep, so lanes of one label meet at one address less often
  unsigned long long sum[SH::kRep][SH::kTab][NW];
  union alignas(16) {
    int rl[kWaves][64];  // per wave: the table index of each entry of the current row
    int tk[SH::kTab];           // while building: cluster of each unranked entry
  };
  union alignas(16) {
    int lab[kWaves][64 / SH::B[0] / 2 * SH::T[0]];  // per wave: the labels of half the current row's lines
    struct {
      int pre[SH::kBinRows + 1];  // while building: prefix of the bin-row counts
      int rstart[SH::kBinRows];   // and the first item of each bin row
      int wsum[kWaves];
    } b;
  };
  int n;
};

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return (uint64_t)hi << 32 | lo;
}

// bits [a, b] of a 64-bit word (empty when b < a); a, b in [0, 63]
__device__ __forceinline__ uint64_t bit_range(int a, int b) {
  const uint64_t r = (~0ull >> (63 - b)) & (~0ull << a);
  return b < a ? 0ull : r;
}

// v with bit l cleared, one scalar instruction
__device__ __forceinline__ uint64_t clear_bit(uint64_t v, int l) {
  asm("s_bitset0_b64 %0, %1" : "+s"(v) : "s"(l));
  return v;
}

template <typename T, int ND, int CC>
__device__ __forceinline__ bool sweep_tile_fast(const Geo& g, const T* __restrict__ img,
                                                const int32_t* __restrict__ bstart,
                                                const int32_t* __restrict__ items,
                                                const float* __restrict__ recs,
                                                const SweepArgs& a, int iter, int tile,
                                                FastLds<T, ND, CC>& L) {
  using SH = Fast<ND>;
  using PK = TilePack<T, ND, CC, SH>;
  constexpr PK pk{};
  constexpr int NW = PK::kFields > 0 ? pk.nw : 1;
  constexpr int C = CC;
  const int RS = g.rs;
  const int F = 1 + ND + C;
  constexpr int BXN = SH::T[0] / SH::B[0];                 // blocks per row
  constexpr int NROWS = blocks_per_tile<SH, ND>() / BXN;   // rows per tile
  static_assert(SH::T[0] * (64 / SH::B[0]) == 512, "a row holds 512 voxels");

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

  int to[ND], tc[ND], te[ND];
  {
    int r = tile;
    for (int i = 0; i < ND; ++i) {
      tc[i] = r % a.nt[i];
      r /= a.nt[i];
      to[i] = tc[i] * SH::T[i];
      te[i] = min(SH::T[i], g.n[i] - to[i]);
    }
  }

  // --- the tile's table --------------------------------------------------------
  int b0[ND], nbr[ND], nrows = 1;
  for (int i = 0; i < ND; ++i) {
    b0[i] = max(to[i] / g.S[i] - 1, 0);
    const int b1 = min((to[i] + te[i] - 1) / g.S[i] + 1, g.nb[i] - 1);
    nbr[i] = b1 - b0[i] + 1;
    if (i > 0) nrows *= nbr[i];
  }
  if (nrows > SH::kBinRows) return false;
  if (tid == 0) L.n = 0;
  {
    int cnt = 0;
    if (tid < nrows) {
      int bl = b0[0] * (int)g.bst[0], rr = tid;
      for (int i = 1; i < ND; ++i) {
        bl += (b0[i] + rr % nbr[i]) * (int)g.bst[i];
        rr /= nbr[i];
      }
      const int ja = bstart[bl];
      cnt = bstart[bl + nbr[0]] - ja;
      L.b.rstart[tid] = ja;
    }
    // inclusive scan of the counts: within each wave, then across waves
    int v = cnt;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int u = __shfl_up(v, d, 64);
      if (lane >= d) v += u;
    }
    if (lane == 63) L.b.wsum[wave] = v;
    __syncthreads();
    int add = 0;
    for (int w = 0; w < wave; ++w) add += L.b.wsum[w];
    if (tid < nrows) L.b.pre[tid + 1] = v + add;
    if (tid == 0) L.b.pre[0] = 0;
    __syncthreads();
  }
  const int nraw = L.b.pre[nrows];
  if (nraw > 4 * SH::kTab) return false;  // uniform: every thread read the same count
  for (int i0 = 0; i0 < nraw; i0 += kThreads) {
    const int i = i0 + tid;
    bool keep = i < nraw;
    int k = 0;
    if (keep) {
      int lo = 0, hi = nrows;  // the bin row r with pre[r] <= i < pre[r + 1]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (L.b.pre[mid] <= i) lo = mid;
        else hi = mid;
      }
      k = items[L.b.rstart[lo] + (i - L.b.pre[lo])];
      const int* irec = reinterpret_cast<const int*>(recs + (int64_t)k * RS);
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        const int wl = irec[rec_lo(C, ND) + d], wh = irec[rec_hi(C, ND) + d];
        keep = keep && wl <= to[d] + te[d] - 1 && wh >= to[d];
      }
    }
    const uint64_t m = __ballot(keep);
    int base = 0;
    if (lane == 0 && m) base = atomicAdd(&L.n, (int)__popcll(m));
    base = __builtin_amdgcn_readlane(base, 0);
    if (keep) {
      const int p = base + lanes_below(m);
      if (p < SH::kTab) L.tk[p] = k;
    }
  }
  __syncthreads();
  const int n = L.n;
  if (n > SH::kTab) return false;
  // Coordinates are taken from the tile's centre o_i = to_i + T_i / 2.  q
  // carries an offset, the smallest power of two above the largest |xs|^2
  // of the tile, so that the distance the lanes compare, D^2 - |xs|^2 +
  // offset, is never negative (its bits then order as its values), and
  // adding it rounds nothing that was exact: equal distances stay equal.
  double qoff = 1.0;
  {
    double mx = 1.0;
    for (int i = 0; i < ND; ++i) mx += (SH::T[i] / 2 * g.swd[i]) * (SH::T[i] / 2 * g.swd[i]);
    while (qoff < mx * (1.0 + 1e-6)) qoff *= 2.0;
  }
  // rank by cluster index; each entry is written at its rank
  for (int s = tid; s < n; s += kThreads) {
    const int k = L.tk[s];
    int rank = 0;
    for (int t = 0; t < n; ++t) rank += L.tk[t] < k;
    const float* rec = recs + (int64_t)k * RS;
    const int* irec = reinterpret_cast<const int*>(rec);
    float* R = L.rec[rank];
    double q = 0.0;
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      const float cr = (float)((double)rec[C + i] - (double)(to[i] + SH::T[i] / 2) * g.swd[i]);
      q += (double)cr * (double)cr;
      R[1 + i] = -2.0f * cr;
    }
    R[0] = (float)(q + qoff);
#pragma unroll
    for (int c = 0; c < C; ++c) R[1 + ND + c] = rec[c];
    R[1 + ND + C] = __int_as_float(rank);
    // the image's own cluster index, from the record (a batch shares one
    // record table: k there counts across its images)
    L.kk[rank] = irec[rec_k(C, ND)];
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      const int lo = min(max(irec[rec_lo(C, ND) + i] - to[i], -1), SH::T[i]);
      const int hi = min(max(irec[rec_hi(C, ND) + i] - to[i], -1), SH::T[i]);
      L.tb[i][rank] = (uint16_t)((lo + 1) | (hi + 1) << 8);  // both in [0, 33]
    }
    {
      uint32_t rb = 0;
#pragma unroll
      for (int i = 1; i < ND; ++i) {
        const int lo = max(irec[rec_lo(C, ND) + i] - to[i], 0);
        const int hi = min(irec[rec_hi(C, ND) + i] - to[i], SH::T[i] - 1);
        if (lo <= hi) {
          const int b0 = lo / SH::B[i], b1 = hi / SH::B[i];
          rb |= (((1u << (b1 - b0 + 1)) - 1u) << b0) << (8 * (i - 1));
        }
      }
      L.rb[rank] = rb;
    }
#pragma unroll
    for (int r = 0; r < SH::kRep; ++r)
#pragma unroll
      for (int w = 0; w < NW; ++w) L.sum[r][rank][w] = 0;
  }
  __syncthreads();

  // --- rows of blocks --------------------------------------------------------
  int lx[ND];
  {
    int r = lane;
    for (int i = 0; i < ND; ++i) {
      lx[i] = r % SH::B[i];
      r /= SH::B[i];
    }
  }

  // Copies the table entries meeting the box [blo, bhi] (tile-relative) that
  // sit at positions [c0, c0 + 64) of its list into the wave's list; returns
  // how many entries meet the box.
  // (a whole row, box = the row: an entry meets it when its window meets the
  // row's block on every axis >= 1, since every entry meets the tile along
  // axis 0; a block: the bounds on every axis)
  auto build = [&](const int* blo, const int* bhi, int c0, auto whole_row) {
    int cnt = 0;
    uint32_t rbit = 1;
    if constexpr (decltype(whole_row)::value) {
      rbit = 1u << (blo[1] / SH::B[1]);
      if constexpr (ND == 3) rbit |= 1u << (8 + blo[2] / SH::B[2]);
    }
    for (int e0 = 0; e0 < n; e0 += 64) {
      const int e = e0 + lane;
      const int ec = min(e, n - 1);
      bool m = e < n;
      if constexpr (decltype(whole_row)::value) {
        m = m & ((L.rb[ec] & rbit) == rbit);
      } else {
#pragma unroll
        for (int i = 0; i < ND; ++i) {
          const uint32_t w = L.tb[i][ec];
          const int lo = (int)(w & 0xffu) - 1, hi = (int)(w >> 8) - 1;
          m = m & (lo <= bhi[i]) & (hi >= blo[i]);
        }
      }
      const uint64_t bal = __ballot(m);
      const int p = cnt + lanes_below(bal) - c0;
      if (m && p >= 0 && p < 64) L.rl[wave][p] = e;
      cnt += (int)__popcll(bal);
    }
    __builtin_amdgcn_wave_barrier();
    return cnt;
  };

  for (int row = wave; row < NROWS; row += kWaves) {
    int rlo[ND], rhi[ND];
    bool rin = true;
    rlo[0] = 0;
    rhi[0] = te[0] - 1;
    {
      int rr = row;
      for (int i = 1; i < ND; ++i) {
        const int nbk = SH::T[i] / SH::B[i];
        rlo[i] = (rr % nbk) * SH::B[i];
        rr /= nbk;
        rhi[i] = min(rlo[i] + SH::B[i], te[i]) - 1;
        rin = rin && rlo[i] <= rhi[i];
      }
    }
    if (!rin) continue;
    // this lane's voxel in the row: axes >= 1 fixed, axis 0 per block
    bool rowok = true;
    float xs[ND];
    int64_t vrow = to[0];
    for (int i = 1; i < ND; ++i) {
      const int y = rlo[i] + lx[i];
      rowok = rowok && y <= rhi[i];
      xs[i] = (float)(y - SH::T[i] / 2) * g.sw[i];
      vrow += (int64_t)(to[i] + (rowok ? y : rlo[i])) * g.st[i];
    }
    const T* prow = img + vrow * C;
    // this lane's line of the row (its position along axes 1-2 in the block)
    const int lline = ND == 2 ? lx[1] : lx[2] * SH::B[1] + lx[1];

    // The list (or one 64-entry part of it) the lanes hold: lane j holds
    // entry j, its window bounds, the part of its lane mask along axes 1 and
    // 2, and its coverage of the row's axis-0 positions.
    bool held = false;
    int ej = 0;  // table index of the held entry
    int lo[ND], hi[ND];
    uint64_t myz = 0, hm = 0;
    uint32_t xb0 = 0;  // axis-0 positions of the row (tile-relative) in the window
    auto hold = [&](int nc) {
      held = lane < nc;
      ej = held ? L.rl[wave][lane] : 0;
#pragma unroll
      for (int i = 0; i < ND; ++i) {
        const uint32_t w = L.tb[i][ej];
        lo[i] = (int)(w & 0xffu) - 1;
        hi[i] = (int)(w >> 8) - 1;
      }
      const int a1 = min(max(lo[1] - rlo[1], 0), SH::B[1] - 1);
      const int b1 = max(min(hi[1] - rlo[1], SH::B[1] - 1), 0);
      const int a2 = min(max(lo[2] - rlo[2], 0), SH::B[2] - 1);
      const int b2 = max(min(hi[2] - rlo[2], SH::B[2] - 1), 0);
      const uint64_t p1 = bit_range(a1 * 4, b1 * 4 + 3);
      myz = (p1 | p1 << 16 | p1 << 32 | p1 << 48) & bit_range(a2 * 16, b2 * 16 + 15);
      hm = __ballot(held);
      const int xa = max(lo[0], 0), xe = min(hi[0], rhi[0]);
      xb0 = xa <= xe ? (uint32_t)bit_range(min(xa, 31), max(xe, 0)) : 0u;
    };

    // this lane's voxel in each block of the row: its channels, its axis-0
    // term, and the best distance and entry so far
    const int nbx = min(BXN, (rhi[0] + SH::B[0]) / SH::B[0]);  // blocks in the image
    float Iv[BXN][C], bD[BXN];
    int bE[BXN];
#pragma unroll
    for (int bx = 0; bx < BXN; ++bx) {
      const int x = bx * SH::B[0] + lx[0];
      // lanes past the image's edge (last block only) read its last voxel
      const T* px = prow + (uint32_t)min(x, rhi[0]) * C;
#pragma unroll
      for (int c = 0; c < C; ++c) Iv[bx][c] = bx < nbx ? (float)px[c] : 0.0f;
      bD[bx] = __builtin_inff();
      bE[bx] = -1;
    }
    // axis-0 coordinate of this lane's voxel in block 0, and the step from
    // one block to the next
    const float x00 = (float)(lx[0] - SH::T[0] / 2) * g.sw[0];
    const float xstep = (float)SH::B[0] * g.sw[0];

    // The held entries one at a time, in ascending table order: the terms of
    // axes 1 and 2 and of axis 0 at block 0 once, then each block of the row
    // the window meets (its axis-0 term a multiple of one step).  On
    // such a block the window is applied as a lane mask (its axis-0 bits for
    // the block, repeated over the block's 16 lines, and its part along
    // axes 1 and 2; all lanes when it covers the block); lanes outside it
    // see an infinite distance.  The compare is strict, so equal distances
    // keep the earlier entry, i.e. the lowest cluster index.
    constexpr int EW = 2 + ND + C;  // entry words: q, -2 c_i (ND), mu_c (C), entry index
    constexpr uint32_t kFull = (1u << SH::B[0]) - 1u;
    auto walk = [&]() {
      uint64_t m = hm;
      while (m) {
        const int j = (int)__builtin_ctzll(m);
        m = clear_bit(m, j);
        const uint32_t xb = (uint32_t)__builtin_amdgcn_readlane((int)xb0, j);
        const uint32_t yzl = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)myz, j);
        const uint32_t yzh = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(myz >> 32), j);
        float R[EW];
        {
          const float* src = L.rec[__builtin_amdgcn_readlane(ej, j)];
          const float4 r0 = *reinterpret_cast<const float4*>(src);
          const float4 r1 = *reinterpret_cast<const float4*>(src + 4);
          const float rr[8] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
#pragma unroll
          for (int w = 0; w < EW; ++w) R[w] = rr[w];
        }
        float P = R[0];
#pragma unroll
        for (int i = 1; i < ND; ++i) P = fmaf(xs[i], R[1 + i], P);
        // the terms up to the channels at block 0, and their step per block
        const float Q = fmaf(x00, R[1], P);
        const float dq = xstep * R[1];
        const int rk = __float_as_int(R[EW - 1]);
#pragma unroll
        for (int bx = 0; bx < BXN; ++bx) {
          const uint32_t nib = (xb >> (bx * SH::B[0])) & kFull;
          if (nib == 0u) continue;
          const uint32_t p = nib * 0x11111111u;
          const uint64_t mk = (uint64_t)(p & yzh) << 32 | (p & yzl);
          float D = fmaf((float)bx, dq, Q);
#pragma unroll
          for (int c = 0; c < C; ++c) {
            const float t = Iv[bx][c] - R[1 + ND + c];
            D = fmaf(t, t, D);
          }
          D = __builtin_amdgcn_inverse_ballot_w64(mk) ? D : __builtin_inff();
          const bool cm = D < bD[bx];
          bD[bx] = cm ? D : bD[bx];
          bE[bx] = cm ? rk : bE[bx];
        }
      }
    };

    const int cnt = build(rlo, rhi, 0, std::true_type{});
    for (int c0 = 0;;) {
      hold(min(cnt - c0, 64));
      walk();
      c0 += 64;
      if (c0 >= cnt) break;
      // more than 64 entries meet the row: the next 64
      __builtin_amdgcn_wave_barrier();
      build(rlo, rhi, c0, std::true_type{});
    }

    // no window holds this voxel: its grid cell (first iteration) or its
    // previous label, summed straight into the accumulators
    auto uncovered = [&](int x, const float* Ivc) {
      int xa[ND];
      xa[0] = to[0] + x;
      for (int i = 1; i < ND; ++i) xa[i] = to[i] + rlo[i] + lx[i];
      int64_t lin = 0;
      for (int i = 0; i < ND; ++i) lin += (int64_t)xa[i] * g.st[i];
      const int lab = iter == 0 ? grid_label(g, xa, ND) : a.labels[lin];
      a.accf[lab] = 1;
      unsigned long long* gg = reinterpret_cast<unsigned long long*>(a.acc + (int64_t)lab * F);
      atomicAdd(gg, 1ull);
      for (int i = 0; i < ND; ++i) atomicAdd(gg + 1 + i, (unsigned long long)xa[i]);
      for (int c = 0; c < C; ++c) atomicAdd(gg + 1 + ND + c, (unsigned long long)Ivc[c]);
      return lab;
    };

    // labels and sums of this lane's voxels (the labels replace the entry
    // indices in bE); the rare voxels no window holds afterwards, one at a time
    uint32_t unc = 0, own = 0;  // bit bx: voxel bx uncovered / in the image
#pragma unroll
    for (int bx = 0; bx < BXN; ++bx) {
      const int x = bx * SH::B[0] + lx[0];
      if (bx >= nbx || !rowok || x > rhi[0]) continue;
      own |= 1u << bx;
      const int e = bE[bx];
      if (e < 0) {
        unc |= 1u << bx;
        continue;
      }
      uint32_t v[PK::kFields];
      v[0] = 1;
      v[1] = (uint32_t)x;
      for (int i = 1; i < ND; ++i) v[1 + i] = (uint32_t)(rlo[i] + lx[i]);
#pragma unroll
      for (int c = 0; c < C; ++c) v[1 + ND + c] = (uint32_t)Iv[bx][c];
      uint64_t pw[NW];
      pack_run<PK>(v, pw);
#pragma unroll
      for (int w = 0; w < NW; ++w) atomicAdd(&L.sum[lane & (SH::kRep - 1)][e][w], (unsigned long long)pw[w]);
      bE[bx] = L.kk[e];
    }
    while (unc) {
      const int bx = (int)__builtin_ctz(unc);
      unc &= unc - 1;
      const int x = bx * SH::B[0] + lx[0];
      float Ivc[C];
#pragma unroll
      for (int c = 0; c < C; ++c) Ivc[c] = (float)prow[(uint32_t)x * C + c];
      const int lab = uncovered(x, Ivc);
#pragma unroll
      for (int b2 = 0; b2 < BXN; ++b2)
        if (b2 == bx) bE[b2] = lab;
    }
    // the row's labels leave half its lines at a time (LDS holds half a row
    // per wave), staged so that they go out as whole lines, four per store
    static_assert(BXN == 8 && 64 / SH::B[0] == 16, "a row of 16 lines of 8 blocks' voxels");
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
      if ((lline >> 3) == hf) {
#pragma unroll
        for (int bx = 0; bx < BXN; ++bx)
          if (own & (1u << bx)) L.lab[wave][(lline & 7) * SH::T[0] + bx * SH::B[0] + lx[0]] = bE[bx];
      }
      __builtin_amdgcn_wave_barrier();
      {
        constexpr int Q = SH::T[0] / 4;  // stores per line
        const int line = hf * 8 + lane / Q, x = (lane % Q) * 4;
        int yz[ND];
        bool ok = x <= rhi[0];
        {
          int rr = line;
          for (int i = 1; i < ND; ++i) {
            yz[i] = rlo[i] + rr % SH::B[i];
            rr /= SH::B[i];
            ok = ok && yz[i] <= rhi[i];
          }
        }
        if (ok) {
          int64_t lin = to[0] + x;
          for (int i = 1; i < ND; ++i) lin += (int64_t)(to[i] + yz[i]) * g.st[i];
          const int4 v = *reinterpret_cast<const int4*>(&L.lab[wave][(lane / Q) * SH::T[0] + x]);
          int32_t* dst = a.labels + lin;
          if (x + 3 <= rhi[0] && (reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
            *reinterpret_cast<int4*>(dst) = v;
          } else {
            dst[0] = v.x;
            if (x + 1 <= rhi[0]) dst[1] = v.y;
            if (x + 2 <= rhi[0]) dst[2] = v.z;
            if (x + 3 <= rhi[0]) dst[3] = v.w;
          }
        }
      }
      if (hf == 0) __builtin_amdgcn_wave_barrier();  // the second half reuses the staging
    }
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();

  // --- the tile's sums to their cluster slots -------------------------------
  constexpr int NS = 1 << ND;
  for (int s = tid; s < n; s += kThreads) {
    uint64_t vv[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      vv[w] = 0;
#pragma unroll
      for (int r = 0; r < SH::kRep; ++r) vv[w] += L.sum[r][s][w];
    }
    const uint64_t nn = PK::field(vv, 0);
    if (nn == 0) continue;
    const int k = L.kk[s];
    uint64_t out[1 + ND + 4];
    out[0] = nn;
    for (int i = 0; i < ND; ++i)
      out[1 + i] = PK::field(vv, 1 + i) + nn * (uint64_t)to[i];
    for (int c = 0; c < C; ++c) out[1 + ND + c] = PK::field(vv, 1 + ND + c);
    int q = -1;
    if (a.slots) {
      const int* irec = reinterpret_cast<const int*>(a.ctab + (int64_t)k * g.rs);
      q = 0;
      for (int i = 0; i < ND; ++i) {
        const int lo = max(irec[rec_lo(g.C, g.nd) + i], 0), hi = min(irec[rec_hi(g.C, g.nd) + i], g.n[i] - 1);
        const int t0 = lo / SH::T[i];
        const int d = tc[i] - t0;
        const bool meets = to[i] <= hi && to[i] + SH::T[i] - 1 >= lo;
        if (!meets || d < 0 || d > 1) {
          q = -1;
          break;
        }
        q |= d << i;
      }
    }
    if (q >= 0) {
      uint64_t* dst = a.part + ((int64_t)k * NS + q) * (F + 1);
      for (int f = 0; f < F; ++f) dst[f] = out[f];
      dst[F] = (uint64_t)(iter + 1);
    } else {
      a.accf[k] = 1;
      unsigned long long* gg = reinterpret_cast<unsigned long long*>(a.acc + (int64_t)k * F);
      for (int f = 0; f < F; ++f) atomicAdd(gg + f, (unsigned long long)out[f]);
    }
  }
  return true;
}

// LDS of one workgroup of the sweep
template <typename T, int ND, int CC, class SH>
struct SweepLds {
  int keys[SH::kHash];
  uint64_t vals[SH::kHash * entry_words<T, ND, CC, SH>()];
  uint32_t tb[ND * 64];
  int n;
};

// A tile with accumulation: through its table when the sweep allows it and
// the table holds every meeting centre, else hashed.
template <typename T, int ND, int CC, class SH>
__device__ __forceinline__ void sweep_tile_acc(const Geo& g, const T* img, const int32_t* bstart,
                                               const int32_t* items, const float* recs,
                                               const SweepArgs& a, int iter, int tile,
                                               SweepLds<T, ND, CC, SH>& L) {
  if (a.table && sweep_tile<T, ND, CC, true, SH, true>(g, img, bstart, items, recs, a, iter, tile,
                                                       L.keys, L.vals, L.tb, &L.n))
    return;
  if (a.table) __syncthreads();  // every lane has read the entry count
  sweep_tile<T, ND, CC, true, SH, false>(g, img, bstart, items, recs, a, iter, tile, L.keys, L.vals,
                                         L.tb, &L.n);
}

// The fast form's grey instantiations are held to 6 workgroups per CU (at
// most 80 VGPRs; its LDS, with the window bounds in 16 bits and labels
// staged half of a row's lines at a time, is 25.2 KB per workgroup): the walk's chains
// of vector, scalar and vector work are latency-bound, and each further wave
// per SIMD hides more of it (6.62 -> 6.44 ms from 5 to 6 on the 1024^3
// volume; a few per-tile values spill to scratch, outside the walk).
template <typename T, int ND, int CC, bool ACC>
__global__ void __launch_bounds__(kThreads, (ACC && fast_ok<T, ND, CC>() && CC == 1) ? 6 : 1)
sweep_kernel(Geo g, const T* __restrict__ img, const int32_t* __restrict__ bstart,
             const int32_t* __restrict__ items, const float* __restrict__ recs, SweepArgs a) {
  if (*a.done) return;
  using SH = Shape<ND, 0>;
  const int per = (int)(gridDim.x / 8);
  const int tile = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (tile >= a.ntiles) return;
  if constexpr (ACC && fast_ok<T, ND, CC>()) {
    __shared__ union {
      FastLds<T, ND, CC> f;
      SweepLds<T, ND, CC, SH> s;
    } L;
    if (a.fast && sweep_tile_fast<T, ND, CC>(g, img, bstart, items, recs, a, a.iter, tile, L.f))
      return;
    __syncthreads();  // the fast form's reads of its table are done
    sweep_tile_acc<T, ND, CC, SH>(g, img, bstart, items, recs, a, a.iter, tile, L.s);
  } else if constexpr (ACC) {
    __shared__ SweepLds<T, ND, CC, SH> L;
    sweep_tile_acc<T, ND, CC, SH>(g, img, bstart, items, recs, a, a.iter, tile, L);
  } else {
    sweep_tile<T, ND, CC, false, SH, false>(g, img, bstart, items, recs, a, a.iter, tile, nullptr,
                                            nullptr, nullptr, nullptr);
  }
}

// The sweep over the flat tile work-list of a group of images (same pixel
// type, dimensionality, channel count and tile shape).  The list is cut into
// 8 contiguous chunks, one per XCD (workgroups are dealt to XCDs round
// robin), so neighbouring tiles of an image share an L2; the workgroups of an
// XCD stride through its chunk (one tile each when the grid has a workgroup
// per tile).  Tiles of converged images are skipped.
// Its grey fast-form instantiations are held to 4 waves per SIMD (127 VGPRs,
// no spills; 129 and 3 waves unbounded, spills at 5 and 6).
template <typename T, int ND, int CC, class SH>
__global__ void __launch_bounds__(kThreads, (fast_ok<T, ND, CC>() && CC == 1 &&
                                             std::is_same<SH, Shape<ND, 0>>::value) ? 4 : 1)
sweep_batch_kernel(const BImg* __restrict__ imgs, const int32_t* __restrict__ tile_img, int tile0,
                   int ntiles, const int32_t* __restrict__ bin_start,
                   const int32_t* __restrict__ items, const float* __restrict__ recs, int iter) {
  constexpr bool kFast = fast_ok<T, ND, CC>() && std::is_same<SH, Shape<ND, 0>>::value;
  using LF = typename std::conditional<kFast, FastLds<T, ND, CC>, char>::type;
  __shared__ union {
    LF f;
    SweepLds<T, ND, CC, SH> s;
  } L;
  const int xcd = (int)(blockIdx.x % 8), per = (int)(gridDim.x / 8);
  const int chunk = (ntiles + 7) / 8;
  const int end = min((xcd + 1) * chunk, ntiles);
  for (int t = xcd * chunk + (int)(blockIdx.x / 8); t < end; t += per) {
    const BImg& d = imgs[tile_img[tile0 + t]];
    if (d.flags[0]) continue;
    __syncthreads();  // the previous tile's table is read out
    const T* img = reinterpret_cast<const T*>(d.img);
    const int tile = tile0 + t - d.tile_off;
    if constexpr (kFast) {
      // the same form sslic_run takes for this image, so the results agree
      if (d.a.fast && sweep_tile_fast<T, ND, CC>(d.g, img, bin_start + d.binoff, items, recs, d.a,
                                                 iter, tile, L.f))
        continue;
      __syncthreads();  // the fast form's reads of its table are done
    }
    sweep_tile_acc<T, ND, CC, SH>(d.g, img, bin_start + d.binoff, items, recs, d.a, iter, tile,
                                  L.s);
  }
}

template <typename T, int ND, bool ACC>
hipError_t dispatch_c(const Geo& g, const void* img, SweepArgs a, hipStream_t s) {
  using SS = Shape<ND, 0>;
  int nt = 1;
  a.slots = 1;
  for (int i = 0; i < kMaxDim; ++i) a.nt[i] = 1;
  for (int i = 0; i < ND; ++i) {
    a.nt[i] = (g.n[i] + SS::T[i] - 1) / SS::T[i];
    nt *= a.nt[i];
    if (SS::T[i] < 2 * g.S[i] + 1) a.slots = 0;
  }
  a.ntiles = nt;
  const unsigned grid = (unsigned)(((int64_t)nt + 7) / 8 * 8);  // a multiple of the XCD count
  const T* p = (const T*)img;
  switch (g.C) {
    case 1: sweep_kernel<T, ND, 1, ACC><<<grid, kThreads, 0, s>>>(g, p, a.bstart, a.items, a.recs, a); break;
    case 3: sweep_kernel<T, ND, 3, ACC><<<grid, kThreads, 0, s>>>(g, p, a.bstart, a.items, a.recs, a); break;
    case 4: sweep_kernel<T, ND, 4, ACC><<<grid, kThreads, 0, s>>>(g, p, a.bstart, a.items, a.recs, a); break;
    default: sweep_kernel<T, ND, 0, ACC><<<grid, kThreads, 0, s>>>(g, p, a.bstart, a.items, a.recs, a); break;
  }
  return hipGetLastError();
}

template <typename T, bool ACC>
hipError_t dispatch_nd(const Geo& g, const void* img, const SweepArgs& a, hipStream_t s) {
  switch (g.nd) {
    case 2: return dispatch_c<T, 2, ACC>(g, img, a, s);
    case 3: return dispatch_c<T, 3, ACC>(g, img, a, s);
    default: return dispatch_c<T, 4, ACC>(g, img, a, s);
  }
}

template <bool ACC>
hipError_t dispatch(const Geo& g, const void* img, const SweepArgs& a, hipStream_t s) {
  switch (g.dtype) {
    case kU8: return dispatch_nd<uint8_t, ACC>(g, img, a, s);
    case kU16: return dispatch_nd<uint16_t, ACC>(g, img, a, s);
    default: return dispatch_nd<float, ACC>(g, img, a, s);
  }
}

template <typename T, int ND, int CC, int VAR>
hipError_t batch_launch(const BImg* imgs, const int32_t* tile_img, int tile0, int ntiles,
                        const int32_t* bin_start, const int32_t* items, const float* recs,
                        int iter, unsigned grid, hipStream_t s) {
  sweep_batch_kernel<T, ND, CC, Shape<ND, VAR>><<<grid, kThreads, 0, s>>>(
      imgs, tile_img, tile0, ntiles, bin_start, items, recs, iter);
  return hipGetLastError();
}

template <typename T, int ND, int CC>
hipError_t batch_var(int var, const BImg* imgs, const int32_t* tile_img, int tile0, int ntiles,
                     const int32_t* bin_start, const int32_t* items, const float* recs, int iter, unsigned grid,
                     hipStream_t s) {
  return var == 1 ? batch_launch<T, ND, CC, 1>(imgs, tile_img, tile0, ntiles, bin_start, items, recs, iter, grid, s)
                  : batch_launch<T, ND, CC, 0>(imgs, tile_img, tile0, ntiles, bin_start, items, recs, iter, grid, s);
}

template <typename T, int ND>
hipError_t batch_c(int C, int var, const BImg* imgs, const int32_t* tile_img, int tile0, int ntiles,
                   const int32_t* bin_start, const int32_t* items, const float* recs, int iter, unsigned grid,
                   hipStream_t s) {
  switch (C) {
    case 1: return batch_var<T, ND, 1>(var, imgs, tile_img, tile0, ntiles, bin_start, items, recs, iter, grid, s);
    case 3: return batch_var<T, ND, 3>(var, imgs, tile_img, tile0, ntiles, bin_start, items, recs, iter, grid, s);
    case 4: return batch_var<T, ND, 4>(var, imgs, tile_img, tile0, ntiles, bin_start, items, recs, iter, grid, s);
    default: return batch_var<T, ND, 0>(var, imgs, tile_img, tile0, ntiles, bin_start, items, recs, iter, grid, s);
  }
}

template <typename T>
hipError_t batch_nd(int nd, int C, int var, const BImg* imgs, const int32_t* tile_img, int tile0,
                    int ntiles, const int32_t* bin_start, const int32_t* items, const float* recs, int iter,
                    unsigned grid, hipStream_t s) {
  switch (nd) {
    case 2: return batch_c<T, 2>(C, var, imgs, tile_img, tile0, ntiles, bin_start, items, recs, iter, grid, s);
    case 3: return batch_c<T, 3>(C, var, imgs, tile_img, tile0, ntiles, bin_start, items, recs, iter, grid, s);
    default: return batch_c<T, 4>(C, var, imgs, tile_img, tile0, ntiles, bin_start, items, recs, iter, grid, s);
  }
}

template <int ND>
void shape_of(int var, int* T) {
  for (int i = 0; i < ND; ++i) T[i] = var == 1 ? Shape<ND, 1>::T[i] : Shape<ND, 0>::T[i];
}

}  // namespace

void sweep_tile_shape(int nd, int* T, int var) {
  if (nd == 2) shape_of<2>(var, T);
  else if (nd == 3) shape_of<3>(var, T);
  else shape_of<4>(var, T);
}

bool sweep_fast_applies(const Geo& g) {
  // as fast_ok: integer pixels, 3 axes, 1 + axes + channels <= 7
  return g.dtype != kF32 && g.nd == 3 && g.C > 0 && 1 + g.nd + g.C <= 7;
}

int sweep_slots(const Geo& g, int var) {
  int T[kMaxDim];
  sweep_tile_shape(g.nd, T, var);
  for (int i = 0; i < g.nd; ++i)
    if (T[i] < 2 * g.S[i] + 1) return 0;
  return 1;
}

// The table form pays off when the centres meeting a tile usually fit one
// wave: about prod_i (T_i + 2 S_i) / S_i of them on the seed grid.
int sweep_table_suits(const Geo& g, int var) {
  if (g.K > kTableMaxK) return 0;
  int T[kMaxDim];
  sweep_tile_shape(g.nd, T, var);
  double e = 1.0;
  for (int i = 0; i < g.nd; ++i) e *= (double)(T[i] + 2 * g.S[i]) / g.S[i];
  return e <= 56.0;
}

hipError_t launch_sweep(const Geo& g, const void* img, const Iter& it, int32_t* labels, int iter,
                        int accumulate, hipStream_t s, int var) {
  (void)var;  // the single-image path uses the default tile
  SweepArgs a{};
  a.bstart = it.bin_start;
  a.items = it.bin_items;
  a.recs = it.ctab;
  a.ctab = it.ctab;
  a.labels = labels;
  a.iter = iter;
  a.done = it.done;
  a.part = it.part;
  a.acc = it.acc;
  a.accf = it.accf;
  a.table = accumulate && sweep_table_suits(g, 0);
  a.fast = 1;
  return accumulate ? dispatch<true>(g, img, a, s) : dispatch<false>(g, img, a, s);
}

hipError_t launch_sweep_batch(int dtype, int nd, int C, int var, const BImg* imgs,
                              const int32_t* tile_img, int tile0, int ntiles,
                              const int32_t* bin_start, const int32_t* items, const float* recs, int iter,
                              unsigned grid, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  grid = (grid + 7) / 8 * 8;
  switch (dtype) {
    case kU8: return batch_nd<uint8_t>(nd, C, var, imgs, tile_img, tile0, ntiles, bin_start, items, recs, iter, grid, s);
    case kU16: return batch_nd<uint16_t>(nd, C, var, imgs, tile_img, tile0, ntiles, bin_start, items, recs, iter, grid, s);
    default: return batch_nd<float>(nd, C, var, imgs, tile_img, tile0, ntiles, bin_start, items, recs, iter, grid, s);
  }
}

}  // namespace sslic
