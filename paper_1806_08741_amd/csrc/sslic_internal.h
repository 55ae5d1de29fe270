// sslic_internal.h -- geometry, workspace views and kernel launchers shared by
// the HIP sources of libsslic.so.  Nothing here is part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sslic {

constexpr int kMaxDim = 4;
constexpr int kMaxChan = 8;

enum Dtype { kU8 = 0, kU16 = 1, kF32 = 2 };

// Geometry of one image as the kernels see it.  Images with one axis are
// handled as two-dimensional with a second axis of size 1 (grid step 1),
// which leaves every result unchanged; `nd_out` is the caller's axis count
// and the number of coordinate columns of its centre table.
struct Geo {
  int nd;            // axes the kernels iterate (2..4)
  int nd_out;        // caller's axes (1..4)
  int C;             // channels
  int dtype;         // Dtype
  int n[kMaxDim];    // size per axis (1 beyond nd)
  int64_t st[kMaxDim];  // voxel stride per axis
  int64_t N;         // voxels
  int S[kMaxDim];    // grid step per axis (index units)
  int Ka[kMaxDim];   // clusters per axis
  int64_t K;         // clusters
  int nb[kMaxDim];   // S-bins per axis = ceil(n / S)
  int64_t bst[kMaxDim];  // bin stride per axis
  int64_t nbins;
  float sw[kMaxDim]; // m / S_i in FP32: coordinates are scaled by it in the assignment
  double swd[kMaxDim];  // m / S_i in FP64
  double wd[kMaxDim];  // (m / S_i)^2 in FP64 (residual)
  int rs;            // words per record of the assignment centre table
  int64_t prodS;     // prod S_i (connectivity threshold 4 size > prodS)
  int F;             // 8-byte accumulator words per cluster = 1 + nd + C
  int row;           // doubles per row of the caller's centre table = C + nd_out
};

// Record k of the assignment centre table (FP32 words, stride g.rs):
//   [0, C)            channel means mu_c
//   [C, C+nd)         scaled coordinates c'_i = c_i * m / S_i (rounded from FP64)
//   [C+nd]            int32 cluster index k
//   [C+nd+1, C+2nd+1) int32 lo_i = ceil(c_i - S_i)   (FP64, clamped)
//   [C+2nd+1, C+3nd+1) int32 hi_i = floor(c_i + S_i)
// so that x is inside the closed window of k iff lo_i <= x_i <= hi_i, and
// D^2(x, k) = sum_i (x_i * m / S_i - c'_i)^2 + sum_c (I_c(x) - mu_c)^2.  The
// words a distance needs (mu, c', k) come first and contiguous.
__host__ __device__ inline int rec_words(int C, int nd) { return (C + 3 * nd + 1 + 3) & ~3; }
__host__ __device__ constexpr int rec_k(int C, int nd) { return C + nd; }
__host__ __device__ constexpr int rec_lo(int C, int nd) { return C + nd + 1; }
__host__ __device__ constexpr int rec_hi(int C, int nd) { return C + 2 * nd + 1; }

// Device buffers used by one iteration loop.
struct Iter {
  float* ctab;        // [K][rs]
  int32_t* bin_of;    // [K]
  int32_t* bin_cnt;   // [nbins]   counts, then cursors; zero between uses
  int32_t* bin_start; // [nbins + 1]
  int32_t* bin_items; // [K]     cluster indices in bin order (ascending within a bin)
  int32_t* scan_part; // [ceil(nbins / 4096) + 1]
  uint64_t* acc;      // [K][F]    zero between uses (atomic sums)
  uint8_t* accf;      // [K]       1 where acc holds sums (the sweep's atomic path)
  uint64_t* part;     // [K][2^nd][F + 1] per-tile sums from the sweep, tagged with
                      // iteration + 1 (older tags are stale and ignored)
  double* res_acc;    // [iterations][kResSlots][2]  (sum, count) partials per iteration
  int32_t* done;      // converged flag: kernels return early when set
  int32_t* iters;     // iterations run
};

// Residual partials of one iteration are spread over this many (sum, count)
// pairs (workgroup b adds into pair b mod kResSlots), so that the FP64 atomic
// adds of the reduce step do not all meet at one address.
constexpr int kResSlots = 16;

// ---- launchers (each returns the hipError_t of its launches) -------------

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_f64(double* p, double v, int64_t n, hipStream_t s);

hipError_t launch_seed(const Geo& g, const void* img, double* cen, hipStream_t s);
hipError_t launch_grid_labels(const Geo& g, int32_t* labels, hipStream_t s);

// f64 centres -> assignment table + bin of every cluster + bin counts
hipError_t launch_prep(const Geo& g, const double* cen, const Iter& it, hipStream_t s);
// bin counts -> CSR (bin_start, bin_items sorted by cluster index); the sweep
// reads a bin's records through bin_items
hipError_t launch_bins(const Geo& g, const Iter& it, hipStream_t s);

// Arguments of the fused assignment + map sweep (sweep.hip).
struct SweepArgs {
  const int32_t* bstart;
  const int32_t* items;   // cluster index at every bin position (bin order)
  const float* recs;      // records, by cluster index
  const float* ctab;
  int32_t* labels;
  int iter;               // iteration (0: uncovered voxels take their grid cell)
  const int32_t* done;
  uint64_t* part;         // [K][2^n][F + 1] tile slots, word F = iteration + 1 that wrote it
  uint64_t* acc;
  uint8_t* accf;          // [K] 1 where acc holds sums
  int ntiles;
  int nt[kMaxDim];
  int slots;  // 1: per-cluster tile slots; 0: tiles narrower than a window, atomics only
  int table;  // 1: tiles list their meeting centres first (see sweep_table_suits)
  int fast;   // 1: 2D/3D integer images with few channels take the fast form (sweep.hip)
};
// largest cluster count for which a candidate key can carry (k << 6 | lane)
constexpr int64_t kTableMaxK = (int64_t)1 << 25;
// 1 when the sweep with tile variant `var` should list each tile's meeting
// centres first (few enough per tile, cluster indices small enough)
int sweep_table_suits(const Geo& g, int var);
// assignment of every voxel (labels) at iteration `iter` (0: voxels outside
// every window take their grid cell's label, else they keep theirs); with
// `accumulate`, also the per-cluster sums into it.part (tile slots tagged
// iter + 1) / it.acc (atomics, flagged in it.accf).  `var` picks the tile
// shape (0 default, 1 small).
hipError_t launch_sweep(const Geo& g, const void* img, const Iter& it, int32_t* labels,
                        int iter, int accumulate, hipStream_t s, int var = 0);
constexpr int kTileVars = 2;
int sweep_slots(const Geo& g, int var = 0);          // whether the sweep uses tile slots
// whether the sweep tries its fast form on image g (on the default tile shape)
bool sweep_fast_applies(const Geo& g);
void sweep_tile_shape(int nd, int* T, int var = 0);  // its tile extent per axis

// ---- batched form ----------------------------------------------------------
// One image of a batch.  The batch shares one centre table, bin index and
// record array (global cluster index = koff + k, global bin = binoff + bin,
// record stride g.rs common to the batch); accumulators, tile slots, residual
// partials and flags are the image's own.
struct BImg {
  Geo g;
  SweepArgs a;            // a.bstart unused (bin_start + binoff), a.iter per launch
  const void* img;
  double* cen;            // caller's [K][C + n]
  int64_t* counts;        // caller's [K] or null
  double* residuals;      // caller's [iterations] or null
  int32_t* iters_out;     // caller's device int32 or null
  double* res;            // [iterations][kResSlots][2] residual partials
  int32_t* flags;         // [0] done, [1] iterations run
  int64_t koff;           // first global cluster
  int64_t binoff;         // first global bin
  int tile_off;           // first tile in its group's work-list (global tile numbering)
  int iterations;
  double tol;
  int tdim[kMaxDim];      // tile extent of its group
};
// sweep of one group's tiles at iteration `iter` (grid = workgroups, each
// taking tiles grid apart)
hipError_t launch_sweep_batch(int dtype, int nd, int C, int var, const BImg* imgs,
                              const int32_t* tile_img, int tile0, int ntiles,
                              const int32_t* bin_start, const int32_t* items, const float* recs,
                              int iter,
                              unsigned grid, hipStream_t s);
// seeding of the clusters [k0, k1) of one pixel type (cluster -> image map cl_img)
hipError_t launch_seed_batch(int dtype, const BImg* imgs, const int32_t* cl_img, int64_t k0,
                             int64_t k1, hipStream_t s);
// records and bin counts of every cluster of images not done
hipError_t launch_prep_batch(const BImg* imgs, const int32_t* cl_img, int64_t K, float* ctab,
                             int32_t* bin_of, int32_t* bin_cnt, hipStream_t s);
// the reduce step of one group ([k0, k1) share nd, C, pixel type)
hipError_t launch_finalize_batch(int dtype, int nd, int C, const BImg* imgs, const int32_t* cl_img,
                                 int64_t k0, int64_t k1, float* ctab, int32_t* bin_of,
                                 int32_t* bin_cnt, int t, hipStream_t s);
// residual, done flags and iteration counts of every image
hipError_t launch_residual_finish_batch(const BImg* imgs, int n, int t, hipStream_t s);
// iteration counts to the callers' device ints
hipError_t launch_batch_outputs(const BImg* imgs, int n, hipStream_t s);
// every image's residuals to 0
hipError_t launch_batch_zero_residuals(const BImg* imgs, int n, int tmax, hipStream_t s);
hipError_t launch_update(const Geo& g, const void* img, const int32_t* labels,
                         const Iter& it, hipStream_t s);
// accumulators (and, with `use_part`, the sweep's tile slots) -> new centres,
// counts, residual partials; then prep for the next iteration (table, bins)
// when `prep_next`
hipError_t launch_finalize(const Geo& g, double* cen, int64_t* counts, const Iter& it,
                           int t, int prep_next, int use_part, hipStream_t s);
// residual of iteration t -> residuals[t] (if non-null), done flag, iteration count
hipError_t launch_residual_finish(const Iter& it, int t, double tol, double* residuals,
                                  hipStream_t s);

// connectivity scratch
struct CCBuf {
  int32_t* parent;    // [N]
  int32_t* size;      // [N] component sizes at roots (~size: marked final)
  int32_t* newlab;    // [N] label of each component root
  int32_t* part;      // [ceil(N / 1024) + 1] large open roots per chunk, then offsets
  int32_t* rpart;     // [ceil(N / 1024) + 1] roots per chunk, then offsets
  int32_t* bpart;     // [ceil(chunks / 4096) + 1] scan partials of part
  int32_t* brpart;    // [ceil(chunks / 4096) + 1] scan partials of rpart
  int32_t* roots;     // [N] the roots in raster order
  int32_t* xface;     // [tiles][4][tile voxels / tile extent along axis 0]: label and
                      // local root of each tile's first and last column along axis 0
  int32_t* total;     // [1] number of new labels
  int32_t* nroots;    // [1] number of roots
};
// ints the chunk counts of CCBuf take (part, rpart, bpart, brpart, nroots),
// and their carving
inline int64_t cc_chunks(int64_t N) { return N / 1024 + 2; }
inline int64_t cc_scan_blocks(int64_t N) { return cc_chunks(N) / 4096 + 2; }
inline int64_t cc_part_ints(int64_t N) { return 2 * cc_chunks(N) + 2 * cc_scan_blocks(N) + 2; }
inline void cc_carve(CCBuf& c, int32_t* region, int64_t N) {
  const int64_t nc = cc_chunks(N), nb = cc_scan_blocks(N);
  c.part = region;
  c.rpart = region + nc;
  c.bpart = region + 2 * nc;
  c.brpart = region + 2 * nc + nb;
  c.nroots = region + 2 * nc + 2 * nb;
}
// 8-bit sRGB pixels [n][3] to CIE-Lab floats [n][3]
hipError_t launch_rgb_to_lab(const uint8_t* rgb, int64_t n, float* lab, hipStream_t s);
// the image with its label contours set to 0 (out may not alias img)
hipError_t launch_mask_contours(const Geo& g, const void* img, const int32_t* labels, void* out,
                                hipStream_t s);
hipError_t launch_connectivity(const Geo& g, const double* cen, int32_t* labels,
                               const CCBuf& b, int32_t* n_labels_dev, hipStream_t s);
// ints of CCBuf::xface for an image
int64_t cc_xface_ints(const Geo& g);

}  // namespace sslic
