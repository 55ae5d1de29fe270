/*
 * sslic.h -- C ABI of the MI355X (gfx950) Scalable SLIC library, libsslic.so.
 *
 * Scalable SLIC (Lowekamp, Chen, Yaniv, Yoo) clusters the voxels of an n-D
 * image with C channels in the joint (channels, coordinates) space:
 *
 *   D^2 = sum_c (I_c(x) - mu_kc)^2 + sum_i (m / S_i)^2 (x_i - c_ki)^2
 *
 * (Sec. 2.1 distance, per-axis grid S_i in index units from Sec. 3.3), with
 * centres seeded on a regular grid and moved to the lowest gradient magnitude
 * in their 3^n neighbourhood (Sec. 2.2 / 3.1 stage 1), iterated assignment
 * over each centre's closed window |x_i - c_ki| <= S_i and mean update
 * (Sec. 3.1 stage 2), and connectivity enforcement (Sec. 3.1 stage 3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.  `image`, `labels`, `centres`, `counts`, `residuals`,
 *   `init_centres` are DEVICE pointers owned by the caller; they must stay
 *   valid until `stream` has passed the call.  Only `dims`, `S`, option
 *   structs, descriptor arrays and the `*_out` scalars are host memory.
 * Layout.  The image is dense with interleaved channels: channel fastest, then
 *   axis 0, axis 1, ...  (element (x_0..x_{n-1}, c) lives at
 *   ((x_{n-1} * N_{n-2} + ...) * N_0 + x_0) * C + c).  Labels are int32, one
 *   per voxel, same linear order.  The centre table is double, K rows of
 *   [mu_0 .. mu_{C-1}, c_0 .. c_{n-1}] (channel means first, then
 *   coordinates in voxel units).
 * Clusters.  K = prod_i K_i with K_i = max(1, round-half-up(N_i / S_i));
 *   cluster k has grid index j_i with k = sum_i j_i prod_{i'<i} K_i' and its
 *   seed at floor((2 j_i + 1) N_i / (2 K_i)) (Sec. 2.2 "fixed intervals").
 * Validity.  1 <= ndim <= 4; every N_i >= 1; prod N_i < 2^40;
 *   1 <= channels <= 8; 1 <= S_i <= 2^30; m > 0 and finite; iterations >= 1.
 *   Violations return SSLIC_EINVAL.  Valid requests this build does not
 *   handle return SSLIC_EUNSUPPORTED: images of 2^31 voxels or more (voxel,
 *   cluster and label indices are 32-bit inside the kernels) and K + N of
 *   2^31 or more (new labels K, K+1, ... must fit int32).  Everything is
 *   checked before any work is enqueued.
 * Asynchrony.  All device work is enqueued on `stream` (0 = the null stream);
 *   an entry point returns as soon as the work is queued, unless a host
 *   `*_out` pointer is given, which makes it wait for `stream`.
 * Errors.  Every function returns SSLIC_OK (0) or a negative code and never
 *   throws; sslic_last_error() gives a message for the calling thread's last
 *   failure.  After SSLIC_EDEVICE the outputs are unspecified.
 * Threads.  A context is used by one host thread at a time; contexts are
 *   independent and may share a device.
 */
#ifndef SSLIC_H
#define SSLIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sslic_ctx sslic_ctx;         /* opaque; owns the scratch workspace */
typedef struct ihipStream_t* sslic_stream_t; /* a hipStream_t */

typedef enum { SSLIC_U8 = 0, SSLIC_U16 = 1, SSLIC_F32 = 2 } sslic_dtype;

enum {
  SSLIC_OK = 0,
  SSLIC_EINVAL = -1,      /* an argument is outside the validity rules */
  SSLIC_ENOMEM = -2,      /* device workspace could not be allocated */
  SSLIC_EDEVICE = -3,     /* a HIP runtime call or kernel launch failed */
  SSLIC_EUNSUPPORTED = -4 /* valid request the library does not handle */
};

/* Options of sslic_run; a zeroed struct (or NULL) means the defaults. */
typedef struct {
  double tol;                 /* stop after the iteration whose residual is < tol
                                 (Sec. 2.2 termination); 0 = run every iteration,
                                 as SSLIC does (Sec. 3.1) */
  int no_connectivity;        /* 1 = skip connectivity enforcement (Sec. 3.1 stage 3) */
  const double* init_centres; /* device, K rows; NULL = seed on the grid (stage 1) */
  double* residuals;          /* device, `iterations` doubles or NULL: residual of
                                 every iteration run (Sec. 3.2), 0 after a stop */
  int32_t* iters_done_dev;    /* device int32 or NULL: iterations actually run */
  int32_t* n_labels_dev;      /* device int32 or NULL: labels in use after stage 3 */
  int no_graph;               /* sslic_run_batch: 1 = enqueue the launches directly
                                 instead of replaying a captured HIP graph */
  int no_autotune;            /* sslic_run_batch: 1 = default tile shapes instead of
                                 the ones timed per (ndim, channels, dtype, S) */
  int persist_distance;       /* sslic_run: 1 = the loop as Sec. 2.2 and Sec. 3.1
                                 write it: the distance image is set to infinity once,
                                 in stage 1, and kept across iterations (a voxel
                                 changes label only where a centre comes strictly
                                 closer than every earlier one); 0 = reset it at every
                                 iteration, so that each assignment depends on the
                                 current centres only (the default).  Adds 4 N bytes
                                 of scratch; sslic_run_batch rejects it with
                                 SSLIC_EUNSUPPORTED */
} sslic_options;

/* Create a context bound to HIP device `device_ordinal`.
 * out: receives the context (NULL on failure).  Allocates nothing on the
 * device until the first run. */
int sslic_create(sslic_ctx** out, int device_ordinal);

/* Free the context and its workspace (waits for the work it queued). */
void sslic_destroy(sslic_ctx* ctx);

/* Host-only: number of clusters K (and per-axis counts K_axis[ndim], may be
 * NULL) for the given geometry.  Sec. 2.2 / 3.1 stage 1. */
int sslic_num_clusters(int ndim, const int64_t* dims, const int32_t* S, int64_t* K_out,
                       int64_t* K_axis);

/* The whole filter on one image (Sec. 3.1): seeding and gradient move (or
 * init_centres), `iterations` rounds of assignment + update with the residual
 * test, then connectivity enforcement unless disabled.
 *   image      device, N * channels elements of `dtype`
 *   dims, S    host, ndim entries each (axis 0 first)
 *   m          spatial weight (Sec. 3.2; 10 suits CIE-Lab 2D images)
 *   labels     device int32 [N] (output)
 *   centres    device double [K][channels + ndim] (output; the centres of the
 *              last update, not moved by connectivity)
 *   counts     device int64 [K] or NULL (output: members of each cluster
 *              after the last assignment)
 *   n_labels_out, iters_done_out  host or NULL; either one makes the call
 *              wait for `stream`.
 * Scratch: the context's workspace grows to about
 *   K * (64 + 8 (channels + ndim + 1) (1 + 2^ndim)) + 4 ceil-bins + (connectivity ? 16 N : 0)
 *   + (persist_distance ? 4 N : 0)
 * bytes and is reused across calls. */
int sslic_run(sslic_ctx* ctx, const void* image, int ndim, const int64_t* dims,
              int channels, sslic_dtype dtype, const int32_t* S, double m, int iterations,
              const sslic_options* opt, int32_t* labels, double* centres, int64_t* counts,
              int32_t* n_labels_out, int32_t* iters_done_out, sslic_stream_t stream);

/* Size of the device scratch of sslic_run_static, per GPU. */
#define SSLIC_STATIC_SCRATCH_BYTES (64u << 20)

/* sslic_run for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  It
 * allocates nothing (no hipMalloc, hipFree or pinned host memory) and needs
 * no context: its workspace is a static device array of
 * SSLIC_STATIC_SCRATCH_BYTES (64 MiB) that the library holds on every GPU it
 * runs on until the process ends; its device address is looked up once per
 * device, on the first call there.
 *   Arguments, outputs and results are those of sslic_run, except that the
 *   label count and the iterations run are returned only through
 *   opt->n_labels_dev and opt->iters_done_dev (device int32, may be NULL), so
 *   the call never waits for `stream`.  The work runs on the calling
 *   thread's current HIP device; `stream` must belong to it.
 *   A request whose workspace (as given under sslic_run; e.g. about 16.6 MiB
 *   for a 1024 x 1024 RGB image at S = 16 with connectivity) exceeds the
 *   scratch returns SSLIC_ENOMEM before any device work, with the size in
 *   the message; use sslic_run for it.
 *   Every call on one GPU shares that GPU's scratch and leaves its contents
 *   behind (each call clears what must start at zero): calls that overlap on
 *   one GPU, on any streams or threads, race and give undefined results, so
 *   serialise them (one stream, or events between streams). */
int sslic_run_static(const void* image, int ndim, const int64_t* dims, int channels,
                     sslic_dtype dtype, const int32_t* S, double m, int iterations,
                     const sslic_options* opt, int32_t* labels, double* centres, int64_t* counts,
                     sslic_stream_t stream);

/* One image of a batch. */
typedef struct {
  const void* image;  /* device */
  int ndim;
  int64_t dims[4];
  int channels;
  sslic_dtype dtype;
  int32_t S[4];
  double m;
  int iterations;
  int32_t* labels;    /* device int32 [N] */
  double* centres;    /* device double [K][channels + ndim] */
  int64_t* counts;    /* device int64 [K] or NULL */
  double* residuals;  /* device double [iterations] or NULL */
  int32_t* iters_done;/* device int32 or NULL: iterations this image ran */
} sslic_image_desc;

/* Many independent images in one pass (the batched form).  Images may differ
 * in size, ndim, channels, dtype, S, m and iterations.  Seeding, then the
 * iterations of every image interleaved: per iteration one launch per group
 * of images sharing (dtype, ndim, channels, tile shape) covers a flat
 * work-list of their tiles, one workgroup per tile; each image stops on its own residual test
 * (opt->tol) or after its own `iterations`; then connectivity per image
 * unless opt->no_connectivity.  Each image's result is the one sslic_run
 * gives for it alone (bit-identical labels and centres for integer images;
 * float images may differ in the last bits of FP64 sums).
 *   Tile shapes: the first time a (ndim, channels, dtype, S) appears, the
 * candidate shapes are timed on the largest such image of the batch and the
 * fastest is kept for the context's lifetime (opt->no_autotune: defaults).
 * This first call waits for the stream.
 *   Graphs: the launches are captured into a HIP graph; a later call with the
 * same descriptors and options on the same context replays it, reading the
 * images and writing the outputs at the same addresses (opt->no_graph:
 * enqueue directly).  The batch workspace is separate from the one sslic_run
 * uses.  opt->init_centres and the opt *_dev fields are ignored.
 * n_labels_out: host int32 [n] or NULL (makes the call wait). */
int sslic_run_batch(sslic_ctx* ctx, const sslic_image_desc* images, int n,
                    const sslic_options* opt, int32_t* n_labels_out, sslic_stream_t stream);

/* The superpixel contour mask the paper renders its results with (Sec. 4,
 * visualisation: the image masked by the label contour): a voxel lies on a
 * contour when one of its 2 ndim face neighbours inside the image carries a
 * different label (neighbours outside the image do not count).  out = image
 * with every contour voxel set to 0 in all channels, every other voxel
 * copied.
 *   image   device, N * channels elements of `dtype` (as for sslic_run)
 *   labels  device int32 [N], any values
 *   out     device, N * channels elements of `dtype`; must not overlap image
 * Enqueued on `stream`; uses no workspace.  Returns SSLIC_EINVAL for bad
 * sizes or NULL pointers (nothing enqueued). */
int sslic_mask_contours(sslic_ctx* ctx, const void* image, int ndim, const int64_t* dims,
                        int channels, sslic_dtype dtype, const int32_t* labels, void* out,
                        sslic_stream_t stream);

/* RGB to CIE-Lab, the colour space the paper's colour runs use (Sec. 2.1;
 * Sec. 4 converts its 8-bit RGB data to float Lab; the default m = 10
 * assumes it).  Input: 8-bit sRGB; output: L in [0, 100], a, b, as floats.
 * Conversion: the sRGB transfer curve, the four-digit sRGB-to-XYZ matrix and
 * the D65 white (0.95047, 1, 1.08883), then the CIE Lab function (epsilon =
 * 216/24389, kappa = 24389/27); with these constants the Lab ranges the
 * paper prints for 8-bit RGB come out.
 *   rgb  device uint8 [n_pixels][3]
 *   lab  device float [n_pixels][3] (output); must not overlap rgb
 * Enqueued on `stream`; uses no workspace.  Returns SSLIC_EINVAL for NULL
 * pointers, n_pixels < 0 or overlapping buffers (nothing enqueued). */
int sslic_rgb_to_lab(sslic_ctx* ctx, const uint8_t* rgb, int64_t n_pixels, float* lab,
                     sslic_stream_t stream);

/* Message for the calling thread's last failure ("" if none). */
const char* sslic_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SSLIC_H */
