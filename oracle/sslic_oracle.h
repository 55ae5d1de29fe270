/*
 * sslic_oracle.h -- FP64 reference of the SSLIC path.  Test infrastructure:
 * used by the test-suite, the smoke check and the CPU-baseline timing only.
 *
 * Conventions (all host memory, caller-owned):
 *   image   interleaved channels, channel fastest, then axis 0, 1, ...
 *   labels  int32, one per voxel, linear index with axis 0 fastest
 *   centres double, K rows of [mu_0 .. mu_{C-1}, c_0 .. c_{n-1}]
 * Every function returns OR_OK or a negative error code.
 */
#ifndef SSLIC_ORACLE_H
#define SSLIC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_U8 = 0, OR_U16 = 1, OR_F32 = 2 };
enum { OR_OK = 0, OR_EINVAL = -1, OR_ENOMEM = -2 };

int or_num_clusters(int nd, const int64_t* dims, const int32_t* S, int64_t* K_axis,
                    int64_t* K);
int or_grid_labels(int nd, const int64_t* dims, const int32_t* S, int32_t* labels);
int or_seed(const void* img, int nd, const int64_t* dims, int C, int dtype,
            const int32_t* S, double* centres);
int or_assign(const void* img, int nd, const int64_t* dims, int C, int dtype,
              const int32_t* S, double m, const double* centres, int64_t K,
              int32_t* labels);
int or_assign_persist(const void* img, int nd, const int64_t* dims, int C, int dtype,
                      const int32_t* S, double m, const double* centres, int64_t K,
                      int32_t* labels, double* dist);
int or_assign_points(const void* img, int nd, const int64_t* dims, int C, int dtype,
                     const int32_t* S, double m, const double* centres, int64_t K,
                     const int64_t* points, int64_t npts, int32_t* labels_out,
                     double* dist_out);
int or_update(const void* img, int nd, const int64_t* dims, int C, int dtype,
              const int32_t* S, double m, const int32_t* labels, int64_t K,
              double* centres, int64_t* counts, double* residual);
int or_connectivity(int nd, const int64_t* dims, const int32_t* S,
                    const double* centres, int C, int64_t K, int32_t* labels,
                    int32_t* n_labels);
int or_run(const void* img, int nd, const int64_t* dims, int C, int dtype,
           const int32_t* S, double m, int iterations, double tol, int connectivity,
           int persist_distance, const double* init_centres, int32_t* labels,
           double* centres, int64_t* counts, double* residuals, int* iters_done,
           int32_t* n_labels);

#ifdef __cplusplus
}
#endif
#endif
