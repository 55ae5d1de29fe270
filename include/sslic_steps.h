/*
 * sslic_steps.h -- the single steps of the SSLIC path as separate C entry
 * points of libsslic.so, for one-step checks, resuming and composition.
 * Same conventions as sslic.h: device pointers for images, labels, centres and
 * counts; host pointers for dims, S and *_out scalars; work queued on
 * `stream`; SSLIC_OK or a negative code; validation before any work.
 */
#ifndef SSLIC_STEPS_H
#define SSLIC_STEPS_H

#include "sslic.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Stage 1 (Sec. 2.2 / 3.1): seeds on the grid, each moved to the lowest
 * squared Frobenius norm of the central-difference Jacobian (Sec. 2.2
 * footnote) among its in-image 3^n neighbours (clamped indices, index
 * space; ties keep the earlier position in raster order, the seed first).
 * centres_out: device double [K][channels + ndim], the value and location
 * found.  Integer images compute the gradient in int64, float32 images in
 * FP64 without fused multiply-add, so the result is bit-exact. */
int sslic_seed(sslic_ctx* ctx, const void* image, int ndim, const int64_t* dims,
               int channels, sslic_dtype dtype, const int32_t* S, double* centres_out,
               sslic_stream_t stream);

/* Write into labels [N] the index of the grid cell of every voxel,
 * sum_i floor(x_i K_i / N_i) prod_{i'<i} K_i': the label a voxel keeps when no
 * window reaches it in the first iteration. */
int sslic_grid_labels(sslic_ctx* ctx, int ndim, const int64_t* dims, const int32_t* S,
                      int32_t* labels, sslic_stream_t stream);

/* One assignment step (Sec. 2.2 / 3.1 stage 2) from the given centres:
 * for every voxel x, labels[x] = the smallest k minimising D^2(x, k) over the
 * clusters whose closed window contains x (|x_i - c_ki| <= S_i, evaluated as
 * ceil(c - S) <= x <= floor(c + S) in FP64); distances are FP32.  Voxels no
 * window reaches keep labels[x] (in/out).
 *   centres  device double [K][channels + ndim], read only. */
int sslic_assign(sslic_ctx* ctx, const void* image, int ndim, const int64_t* dims,
                 int channels, sslic_dtype dtype, const int32_t* S, double m,
                 const double* centres, int64_t K, int32_t* labels, sslic_stream_t stream);

/* One assignment step on a distance image the caller keeps between steps,
 * the literal reading of the loops of Sec. 2.2 and Sec. 3.1 (there d is set to
 * infinity once, in stage 1): for every voxel x, the least D^2(x, k) over
 * the clusters whose closed window contains x (as in sslic_assign, FP32, ties
 * to the smallest k) replaces dist[x], and its k replaces labels[x], only
 * where it is strictly below dist[x]; elsewhere both are left as they are.
 *   centres  device double [K][channels + ndim], read only
 *   labels   device int32 [N], in/out
 *   dist     device float [N], in/out: squared distances D^2 of Sec. 2.1 with
 *            the spatial weight m^2 / S_i^2 per axis (Sec. 3.3); +inf where no
 *            centre has reached yet.  Must not overlap image or labels. */
int sslic_assign_persist(sslic_ctx* ctx, const void* image, int ndim, const int64_t* dims,
                         int channels, sslic_dtype dtype, const int32_t* S, double m,
                         const double* centres, int64_t K, int32_t* labels, float* dist,
                         sslic_stream_t stream);

/* One update step (Sec. 3.1 stage 2, map-reduce): every cluster with members
 * becomes the mean of [I(x), x] over the voxels labelled k; clusters without
 * members keep their row.  Integer images sum in int64 (bit-exact), float32
 * images in FP64.  Labels outside [0, K) are ignored.
 *   centres   device double [K][channels + ndim], in/out
 *   counts    device int64 [K] or NULL (out)
 *   residual  device double or NULL (out): mean over clusters with members of
 *             D(old centre, new centre) (Sec. 3.2). */
int sslic_update(sslic_ctx* ctx, const void* image, int ndim, const int64_t* dims,
                 int channels, sslic_dtype dtype, const int32_t* S, double m,
                 const int32_t* labels, int64_t K, double* centres, int64_t* counts,
                 double* residual, sslic_stream_t stream);

/* Connectivity enforcement (Sec. 3.1 stage 3) in place on labels [N], with
 * face adjacency: the component of label k at the rounded centre k (or the
 * first voxel of label k in raster order within floor(S_i/2) of it) is final
 * when 4 * size > prod S_i; every other component, in the raster order of its
 * first voxel, gets a new label K, K+1, ... when 4 * size > prod S_i, and
 * otherwise the label of the face neighbour just before its first voxel
 * (x - e_0 if x_0 > 0, else x - e_1, ...), keeping its own at the origin.
 *   centres       device double [K][channels + ndim], read only
 *   n_labels_out  host or NULL (makes the call wait): K + new labels
 *   n_labels_dev  device int32 or NULL. */
int sslic_connectivity(sslic_ctx* ctx, int ndim, const int64_t* dims, const int32_t* S,
                       int channels, const double* centres, int64_t K, int32_t* labels,
                       int32_t* n_labels_out, int32_t* n_labels_dev, sslic_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* SSLIC_STEPS_H */
