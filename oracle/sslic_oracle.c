/*
 * sslic_oracle.c -- plain, slow FP64 reference implementation of the SSLIC
 * per-iteration path (Lowekamp, Chen, Yaniv, Yoo: "Scalable Simple Linear
 * Iterative Clustering (SSLIC) Using a Generic and Parallel Approach").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP library in paper_1806_08741_amd/, and
 * the product path never calls it.
 *
 * Everything is written the way the paper states it: cluster-centric
 * assignment over each centre's window (Sec. 2.2 / Sec. 3.1 stage 2), a
 * map-reduce style update that is here simply a sequential sum (Sec. 3.1),
 * and the marker-image connectivity enforcement (Sec. 3.1 stage 3).  All
 * arithmetic is FP64; integer images are summed in int64 so the update is
 * exact.  Build with -ffp-contract=off so that no multiply-add is fused.
 *
 * Where the paper is silent the following readings are taken (each one is
 * listed in the design notes of the repository):
 *   - grid: K_i = max(1, round-half-up(N_i/S_i)), seeds at the centres of K_i
 *     equal integer intervals (Sec. 2.2 "regularly sampling ... at fixed
 *     intervals");
 *   - gradient: squared Frobenius norm of the central-difference Jacobian
 *     with clamped indices, in index space; ties keep the earlier position
 *     (Sec. 2.2 footnote on the Jacobian);
 *   - window: closed, |x_i - c_i| <= S_i, evaluated as the integer range
 *     [ceil(c_i - S_i), floor(c_i + S_i)] (Sec. 2.2, Sec. 3.1);
 *   - the distance image is reset to +inf at the start of every iteration
 *     (or, with persist_distance, once before the first, as stage 1 of
 *     Sec. 2.2 and Sec. 3.1 initialises it);
 *     voxels no window covers keep their previous label, and before the
 *     first iteration every voxel carries the label of its grid cell;
 *   - equal distances: the lower cluster index wins (strict "<" while
 *     visiting clusters in ascending order);
 *   - empty clusters keep their centre and are left out of the residual;
 *   - residual: mean, over non-empty clusters, of the paper's distance D
 *     between the previous and the new centre (Sec. 3.2 "residuals");
 *   - connectivity: face adjacency; "size greater than S^n/4" is tested as
 *     4*size > prod(S_i); new labels are K, K+1, ... in raster order; a small
 *     component takes the label of the last face neighbour that precedes its
 *     first voxel in raster order (x - e_0 if x_0 > 0, else x - e_1, ...), and
 *     keeps its own label at the origin (Sec. 3.1 stage 3).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "sslic_oracle.h"

#define OR_MAXD 4

typedef struct {
  int nd;
  int64_t n[OR_MAXD];
  int64_t stride[OR_MAXD];
  int64_t N;
  int C;
  int dtype;
  const void* img;
} img_t;

static int make_img(img_t* g, const void* img, int nd, const int64_t* dims, int C,
                    int dtype) {
  if (nd < 1 || nd > OR_MAXD || C < 1 || C > 8) return OR_EINVAL;
  if (dtype != OR_U8 && dtype != OR_U16 && dtype != OR_F32) return OR_EINVAL;
  g->nd = nd;
  g->C = C;
  g->dtype = dtype;
  g->img = img;
  g->N = 1;
  for (int i = 0; i < nd; ++i) {
    if (dims[i] < 1) return OR_EINVAL;
    g->n[i] = dims[i];
    g->stride[i] = g->N;
    g->N *= dims[i];
  }
  return OR_OK;
}

/* Channel c of voxel `lin`, converted exactly to double. */
static double value_f(const img_t* g, int64_t lin, int c) {
  size_t off = (size_t)lin * (size_t)g->C + (size_t)c;
  switch (g->dtype) {
    case OR_U8: return (double)((const uint8_t*)g->img)[off];
    case OR_U16: return (double)((const uint16_t*)g->img)[off];
    default: return (double)((const float*)g->img)[off];
  }
}

static int64_t value_i(const img_t* g, int64_t lin, int c) {
  size_t off = (size_t)lin * (size_t)g->C + (size_t)c;
  if (g->dtype == OR_U8) return (int64_t)((const uint8_t*)g->img)[off];
  return (int64_t)((const uint16_t*)g->img)[off];
}

static void coords_of(const img_t* g, int64_t lin, int64_t* x) {
  for (int i = 0; i < g->nd; ++i) {
    x[i] = lin % g->n[i];
    lin /= g->n[i];
  }
}

static int64_t lin_of(const img_t* g, const int64_t* x) {
  int64_t l = 0;
  for (int i = 0; i < g->nd; ++i) l += x[i] * g->stride[i];
  return l;
}

/* ---------------------------------------------------------------------- */
/* Grid (Sec. 2.2 / Sec. 3.1 stage 1: centres sampled at fixed intervals). */

static int64_t grid_count(int64_t n, int64_t s) {
  /* round-half-up of n/s, at least one */
  int64_t k = (2 * n + s) / (2 * s);
  return k < 1 ? 1 : k;
}

int or_num_clusters(int nd, const int64_t* dims, const int32_t* S, int64_t* K_axis,
                    int64_t* K) {
  if (nd < 1 || nd > OR_MAXD) return OR_EINVAL;
  int64_t tot = 1;
  for (int i = 0; i < nd; ++i) {
    if (dims[i] < 1 || S[i] < 1) return OR_EINVAL;
    int64_t k = grid_count(dims[i], S[i]);
    if (K_axis) K_axis[i] = k;
    tot *= k;
  }
  if (K) *K = tot;
  return OR_OK;
}

/* Label every voxel with the index of the grid cell it lies in: the label
 * image before the first iteration (readings: "undefined" label made
 * concrete, Sec. 3.1 stage 1). */
int or_grid_labels(int nd, const int64_t* dims, const int32_t* S, int32_t* labels) {
  img_t g;
  int rc = make_img(&g, NULL, nd, dims, 1, OR_U8);
  if (rc) return rc;
  int64_t Ka[OR_MAXD];
  or_num_clusters(nd, dims, S, Ka, NULL);
  int64_t x[OR_MAXD];
  for (int64_t lin = 0; lin < g.N; ++lin) {
    coords_of(&g, lin, x);
    int64_t k = 0, kst = 1;
    for (int i = 0; i < nd; ++i) {
      k += (x[i] * Ka[i] / g.n[i]) * kst;
      kst *= Ka[i];
    }
    labels[lin] = (int32_t)k;
  }
  return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* Seeding and the move to the lowest gradient magnitude (Sec. 2.2 stage 1,
 * footnote: Frobenius norm of the Jacobian for multi-channel images; Sec. 3.1
 * stage 1: done independently for every centre). */

static int64_t clampi(int64_t v, int64_t lo, int64_t hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

/* Squared Frobenius norm of the central-difference Jacobian (without the
 * factor 1/2, which does not change the ordering), integer version. */
static int64_t grad_i(const img_t* g, const int64_t* p) {
  int64_t q[OR_MAXD];
  int64_t acc = 0;
  for (int c = 0; c < g->C; ++c) {
    for (int i = 0; i < g->nd; ++i) {
      memcpy(q, p, sizeof(int64_t) * (size_t)g->nd);
      q[i] = clampi(p[i] + 1, 0, g->n[i] - 1);
      int64_t a = value_i(g, lin_of(g, q), c);
      q[i] = clampi(p[i] - 1, 0, g->n[i] - 1);
      int64_t b = value_i(g, lin_of(g, q), c);
      acc += (a - b) * (a - b);
    }
  }
  return acc;
}

static double grad_f(const img_t* g, const int64_t* p) {
  int64_t q[OR_MAXD];
  double acc = 0.0;
  for (int c = 0; c < g->C; ++c) {
    for (int i = 0; i < g->nd; ++i) {
      memcpy(q, p, sizeof(int64_t) * (size_t)g->nd);
      q[i] = clampi(p[i] + 1, 0, g->n[i] - 1);
      double a = value_f(g, lin_of(g, q), c);
      q[i] = clampi(p[i] - 1, 0, g->n[i] - 1);
      double b = value_f(g, lin_of(g, q), c);
      double d = a - b;
      acc = acc + d * d;
    }
  }
  return acc;
}

int or_seed(const void* img, int nd, const int64_t* dims, int C, int dtype,
            const int32_t* S, double* centres) {
  img_t g;
  int rc = make_img(&g, img, nd, dims, C, dtype);
  if (rc) return rc;
  int64_t Ka[OR_MAXD], K;
  rc = or_num_clusters(nd, dims, S, Ka, &K);
  if (rc) return rc;
  const int row = C + nd;
  int64_t j[OR_MAXD], s[OR_MAXD], q[OR_MAXD], best[OR_MAXD];
  int n3 = 1;
  for (int i = 0; i < nd; ++i) n3 *= 3;
  for (int64_t k = 0; k < K; ++k) {
    /* grid index j of cluster k, axis 0 fastest */
    int64_t r = k;
    for (int i = 0; i < nd; ++i) {
      j[i] = r % Ka[i];
      r /= Ka[i];
      /* centre of the j-th of K equal intervals, rounded down */
      s[i] = ((2 * j[i] + 1) * g.n[i]) / (2 * Ka[i]);
    }
    memcpy(best, s, sizeof(int64_t) * (size_t)nd);
    int64_t gbi = 0;
    double gbf = 0.0;
    if (dtype == OR_F32) gbf = grad_f(&g, s);
    else gbi = grad_i(&g, s);
    /* the 3^n neighbourhood in raster order: offset of axis 0 varies fastest */
    for (int o = 0; o < n3; ++o) {
      int oo = o, inside = 1;
      for (int i = 0; i < nd; ++i) {
        q[i] = s[i] + (oo % 3) - 1;
        oo /= 3;
        if (q[i] < 0 || q[i] >= g.n[i]) inside = 0;
      }
      if (!inside) continue;
      if (dtype == OR_F32) {
        double v = grad_f(&g, q);
        if (v < gbf) {
          gbf = v;
          memcpy(best, q, sizeof(int64_t) * (size_t)nd);
        }
      } else {
        int64_t v = grad_i(&g, q);
        if (v < gbi) {
          gbi = v;
          memcpy(best, q, sizeof(int64_t) * (size_t)nd);
        }
      }
    }
    /* the centre takes the location and the value found there */
    int64_t bl = lin_of(&g, best);
    for (int c = 0; c < C; ++c) centres[k * row + c] = value_f(&g, bl, c);
    for (int i = 0; i < nd; ++i) centres[k * row + C + i] = (double)best[i];
  }
  return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* Assignment (Sec. 2.1 squared distance with per-axis weights m^2/S_i^2 as
 * extended in Sec. 3.3; Sec. 2.2 / Sec. 3.1 stage 2: every centre scans its
 * window and keeps a per-voxel minimum distance and label). */

/* The centre loop over the distance image d: every centre, in ascending k,
 * visits the voxels of its window and takes each one whose d it beats. */
static void assign_windows(const img_t* gp, int nd, int C, const int32_t* S, double m,
                           const double* centres, int64_t K, int32_t* labels, double* d) {
  const img_t g = *gp;
  const int row = C + nd;
  double w[OR_MAXD];
  for (int i = 0; i < nd; ++i) w[i] = (m * m) / ((double)S[i] * (double)S[i]);
  int64_t lo[OR_MAXD], hi[OR_MAXD], x[OR_MAXD];
  for (int64_t k = 0; k < K; ++k) {
    const double* ck = centres + k * row;
    int empty = 0;
    for (int i = 0; i < nd; ++i) {
      double c = ck[C + i];
      /* closed window |x_i - c_i| <= S_i over integer x_i */
      double l = ceil(c - (double)S[i]);
      double h = floor(c + (double)S[i]);
      lo[i] = l < 0.0 ? 0 : (int64_t)l;
      hi[i] = h > (double)(g.n[i] - 1) ? g.n[i] - 1 : (int64_t)h;
      if (lo[i] > hi[i]) empty = 1;
    }
    if (empty) continue;
    memcpy(x, lo, sizeof(int64_t) * (size_t)nd);
    for (;;) {
      int64_t v = lin_of(&g, x);
      double D = 0.0;
      for (int c = 0; c < C; ++c) {
        double t = value_f(&g, v, c) - ck[c];
        D = D + t * t;
      }
      for (int i = 0; i < nd; ++i) {
        double t = (double)x[i] - ck[C + i];
        D = D + w[i] * (t * t);
      }
      if (D < d[v]) {
        d[v] = D;
        labels[v] = (int32_t)k;
      }
      /* odometer over the window box, axis 0 fastest */
      int i = 0;
      while (i < nd) {
        if (++x[i] <= hi[i]) break;
        x[i] = lo[i];
        ++i;
      }
      if (i == nd) break;
    }
  }
}

int or_assign(const void* img, int nd, const int64_t* dims, int C, int dtype,
              const int32_t* S, double m, const double* centres, int64_t K,
              int32_t* labels) {
  img_t g;
  int rc = make_img(&g, img, nd, dims, C, dtype);
  if (rc) return rc;
  if (!(m > 0.0) || K < 1) return OR_EINVAL;
  double* d = (double*)malloc(sizeof(double) * (size_t)g.N);
  if (!d) return OR_ENOMEM;
  for (int64_t v = 0; v < g.N; ++v) d[v] = INFINITY; /* reset every iteration */
  assign_windows(&g, nd, C, S, m, centres, K, labels, d);
  free(d);
  return OR_OK;
}

/* The same step on a distance image the caller keeps between iterations, as
 * the loops of Sec. 2.2 and Sec. 3.1 write it: d is set to infinity once, in
 * stage 1, and a voxel changes label only where some
 * centre of this iteration comes strictly closer than the least distance it
 * has seen so far.
 *   dist  squared distances D^2 [N], read and updated in place */
int or_assign_persist(const void* img, int nd, const int64_t* dims, int C, int dtype,
                      const int32_t* S, double m, const double* centres, int64_t K,
                      int32_t* labels, double* dist) {
  img_t g;
  int rc = make_img(&g, img, nd, dims, C, dtype);
  if (rc) return rc;
  if (!(m > 0.0) || K < 1 || !dist) return OR_EINVAL;
  assign_windows(&g, nd, C, S, m, centres, K, labels, dist);
  return OR_OK;
}

/* Assignment of selected voxels one by one: the per-voxel reading of the same
 * step (Sec. 2.1, Sec. 3.1 stage 2).  The label of x is the lowest k that
 * attains the least D among the centres whose closed window holds x; every
 * centre is examined for every point, in ascending k.
 *   points     linear indices (axis 0 fastest), npts of them
 *   labels_out -1 where no window holds the voxel
 *   dist_out   the least D (INFINITY where none), or NULL */
int or_assign_points(const void* img, int nd, const int64_t* dims, int C, int dtype,
                     const int32_t* S, double m, const double* centres, int64_t K,
                     const int64_t* points, int64_t npts, int32_t* labels_out,
                     double* dist_out) {
  img_t g;
  int rc = make_img(&g, img, nd, dims, C, dtype);
  if (rc) return rc;
  if (!(m > 0.0) || K < 1 || npts < 0) return OR_EINVAL;
  const int row = C + nd;
  double w[OR_MAXD];
  for (int i = 0; i < nd; ++i) w[i] = (m * m) / ((double)S[i] * (double)S[i]);
  /* the window of every centre, as in or_assign */
  int64_t* win = (int64_t*)malloc(sizeof(int64_t) * 2 * (size_t)nd * (size_t)K);
  if (!win) return OR_ENOMEM;
  for (int64_t k = 0; k < K; ++k)
    for (int i = 0; i < nd; ++i) {
      double c = centres[k * row + C + i];
      win[(k * nd + i) * 2] = (int64_t)ceil(c - (double)S[i]);
      win[(k * nd + i) * 2 + 1] = (int64_t)floor(c + (double)S[i]);
    }
  int64_t x[OR_MAXD];
  for (int64_t p = 0; p < npts; ++p) {
    if (points[p] < 0 || points[p] >= g.N) {
      free(win);
      return OR_EINVAL;
    }
    coords_of(&g, points[p], x);
    double best = INFINITY;
    int32_t lab = -1;
    for (int64_t k = 0; k < K; ++k) {
      const int64_t* wk = win + k * nd * 2;
      int inside = 1;
      for (int i = 0; i < nd && inside; ++i) inside = wk[2 * i] <= x[i] && x[i] <= wk[2 * i + 1];
      if (!inside) continue;
      const double* ck = centres + k * row;
      double D = 0.0;
      for (int c = 0; c < C; ++c) {
        double t = value_f(&g, points[p], c) - ck[c];
        D = D + t * t;
      }
      for (int i = 0; i < nd; ++i) {
        double t = (double)x[i] - ck[C + i];
        D = D + w[i] * (t * t);
      }
      if (D < best) {
        best = D;
        lab = (int32_t)k;
      }
    }
    labels_out[p] = lab;
    if (dist_out) dist_out[p] = best;
  }
  free(win);
  return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* Update and residual (Sec. 2.2 / Sec. 3.1 stage 2: new centre = mean of
 * [I(x), x] over the voxels labelled k; Sec. 2.2 termination / Sec. 3.2:
 * change of the centres between iterations). */

int or_update(const void* img, int nd, const int64_t* dims, int C, int dtype,
              const int32_t* S, double m, const int32_t* labels, int64_t K,
              double* centres, int64_t* counts, double* residual) {
  img_t g;
  int rc = make_img(&g, img, nd, dims, C, dtype);
  if (rc) return rc;
  const int row = C + nd;
  int64_t* cnt = (int64_t*)calloc((size_t)K, sizeof(int64_t));
  int64_t* sx = (int64_t*)calloc((size_t)K * (size_t)nd, sizeof(int64_t));
  int64_t* si = (int64_t*)calloc((size_t)K * (size_t)C, sizeof(int64_t));
  double* sf = (double*)calloc((size_t)K * (size_t)C, sizeof(double));
  double* sc = (double*)calloc((size_t)K * (size_t)C, sizeof(double)); /* Neumaier */
  if (!cnt || !sx || !si || !sf || !sc) {
    free(cnt), free(sx), free(si), free(sf), free(sc);
    return OR_ENOMEM;
  }
  int64_t x[OR_MAXD];
  for (int64_t v = 0; v < g.N; ++v) {
    int64_t k = labels[v];
    if (k < 0 || k >= K) continue;
    cnt[k] += 1;
    coords_of(&g, v, x);
    for (int i = 0; i < nd; ++i) sx[k * nd + i] += x[i];
    for (int c = 0; c < C; ++c) {
      if (dtype == OR_F32) {
        double a = value_f(&g, v, c), s = sf[k * C + c], t = s + a;
        if (fabs(s) >= fabs(a)) sc[k * C + c] += (s - t) + a;
        else sc[k * C + c] += (a - t) + s;
        sf[k * C + c] = t;
      } else {
        si[k * C + c] += value_i(&g, v, c);
      }
    }
  }
  double w[OR_MAXD];
  for (int i = 0; i < nd; ++i) w[i] = (m * m) / ((double)S[i] * (double)S[i]);
  double esum = 0.0;
  int64_t ecnt = 0;
  for (int64_t k = 0; k < K; ++k) {
    if (counts) counts[k] = cnt[k];
    if (cnt[k] == 0) continue; /* empty cluster keeps its centre */
    double* ck = centres + k * row;
    double n = (double)cnt[k], e = 0.0;
    for (int c = 0; c < C; ++c) {
      double nv = dtype == OR_F32 ? (sf[k * C + c] + sc[k * C + c]) / n
                                  : (double)si[k * C + c] / n;
      double t = nv - ck[c];
      e = e + t * t;
      ck[c] = nv;
    }
    for (int i = 0; i < nd; ++i) {
      double nv = (double)sx[k * nd + i] / n;
      double t = nv - ck[C + i];
      e = e + w[i] * (t * t);
      ck[C + i] = nv;
    }
    esum += sqrt(e);
    ecnt += 1;
  }
  if (residual) *residual = ecnt ? esum / (double)ecnt : 0.0;
  free(cnt), free(sx), free(si), free(sf), free(sc);
  return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* Connectivity enforcement (Sec. 2.2 stage 3; Sec. 3.1 stage 3: marker
 * image, per-centre first pass, then a raster scan of the non-final voxels). */

/* Flood fill of the face-connected component of label `lab` containing
 * `seed`.  With `only_open`, voxels whose marker is set are not entered.
 * The component is written to `out` (length returned). */
static int64_t flood(const img_t* g, const int32_t* labels, const uint8_t* marker,
                     int only_open, int64_t seed, int32_t lab, int64_t* out,
                     uint8_t* seen) {
  int64_t head = 0, tail = 0;
  out[tail++] = seed;
  seen[seed] = 1;
  int64_t x[OR_MAXD];
  while (head < tail) {
    int64_t v = out[head++];
    coords_of(g, v, x);
    for (int i = 0; i < g->nd; ++i) {
      for (int dir = -1; dir <= 1; dir += 2) {
        int64_t xi = x[i] + dir;
        if (xi < 0 || xi >= g->n[i]) continue;
        int64_t u = v + dir * g->stride[i];
        if (seen[u] || labels[u] != lab) continue;
        if (only_open && marker[u]) continue;
        seen[u] = 1;
        out[tail++] = u;
      }
    }
  }
  for (int64_t t = 0; t < tail; ++t) seen[out[t]] = 0;
  return tail;
}

int or_connectivity(int nd, const int64_t* dims, const int32_t* S,
                    const double* centres, int C, int64_t K, int32_t* labels,
                    int32_t* n_labels) {
  img_t g;
  int rc = make_img(&g, NULL, nd, dims, 1, OR_U8);
  if (rc) return rc;
  const int row = C + nd;
  int64_t prodS = 1;
  int64_t half[OR_MAXD];
  for (int i = 0; i < nd; ++i) {
    prodS *= S[i];
    half[i] = S[i] / 2;
  }
  uint8_t* marker = (uint8_t*)calloc((size_t)g.N, 1);
  uint8_t* seen = (uint8_t*)calloc((size_t)g.N, 1);
  int64_t* comp = (int64_t*)malloc(sizeof(int64_t) * (size_t)g.N);
  if (!marker || !seen || !comp) {
    free(marker), free(seen), free(comp);
    return OR_ENOMEM;
  }
  int64_t p[OR_MAXD], lo[OR_MAXD], hi[OR_MAXD], x[OR_MAXD];
  /* first pass: the component of label k at (or near) centre k */
  for (int64_t k = 0; k < K; ++k) {
    const double* ck = centres + k * row;
    for (int i = 0; i < nd; ++i) p[i] = clampi((int64_t)floor(ck[C + i] + 0.5), 0, g.n[i] - 1);
    int64_t seed = -1;
    int64_t pl = lin_of(&g, p);
    if (labels[pl] == (int32_t)k) {
      seed = pl;
    } else {
      /* first voxel of label k in raster order within the S-box around p */
      for (int i = 0; i < nd; ++i) {
        lo[i] = clampi(p[i] - half[i], 0, g.n[i] - 1);
        hi[i] = clampi(p[i] + half[i], 0, g.n[i] - 1);
      }
      /* raster order = increasing linear index: last axis outermost */
      memcpy(x, lo, sizeof(int64_t) * (size_t)nd);
      for (;;) {
        int64_t v = lin_of(&g, x);
        if (labels[v] == (int32_t)k) {
          seed = v;
          break;
        }
        int i = 0;
        while (i < nd) {
          if (++x[i] <= hi[i]) break;
          x[i] = lo[i];
          ++i;
        }
        if (i == nd) break;
      }
    }
    if (seed < 0) continue;
    int64_t sz = flood(&g, labels, marker, 0, seed, (int32_t)k, comp, seen);
    if (4 * sz > prodS)
      for (int64_t t = 0; t < sz; ++t) marker[comp[t]] = 1;
  }
  /* second pass: raster scan over the voxels that are not final yet */
  int64_t next = K;
  for (int64_t v = 0; v < g.N; ++v) {
    if (marker[v]) continue;
    int64_t sz = flood(&g, labels, marker, 1, v, labels[v], comp, seen);
    int32_t nl;
    if (4 * sz > prodS) {
      nl = (int32_t)next++;
    } else {
      /* the face neighbour just before v in raster order; at the origin the
       * component keeps its label */
      coords_of(&g, v, x);
      nl = labels[v];
      for (int i = 0; i < nd; ++i) {
        if (x[i] > 0) {
          nl = labels[v - g.stride[i]];
          break;
        }
      }
    }
    for (int64_t t = 0; t < sz; ++t) {
      labels[comp[t]] = nl;
      marker[comp[t]] = 1;
    }
  }
  if (n_labels) *n_labels = (int32_t)next;
  free(marker), free(seen), free(comp);
  return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* RGB to CIE-Lab (Sec. 2.1 and the data paragraph of Sec. 4: the colour
 * runs work on Lab converted from 8-bit RGB).  Reading: 8-bit sRGB, the sRGB
 * transfer curve, the four-digit sRGB-to-XYZ matrix, the D65 white
 * (0.95047, 1, 1.08883) and the CIE Lab function; these constants give the
 * ranges of L, a and b the paper prints for 8-bit RGB. */
static double srgb_linear(double v) {
  return v <= 0.04045 ? v / 12.92 : pow((v + 0.055) / 1.055, 2.4);
}

static double lab_fn(double t) {
  const double eps = 216.0 / 24389.0, kappa = 24389.0 / 27.0;
  return t > eps ? cbrt(t) : (kappa * t + 16.0) / 116.0;
}

int or_rgb_to_lab(const uint8_t* rgb, int64_t n, double* lab) {
  if (n < 0) return OR_EINVAL;
  for (int64_t p = 0; p < n; ++p) {
    const double r = srgb_linear(rgb[3 * p] / 255.0);
    const double g = srgb_linear(rgb[3 * p + 1] / 255.0);
    const double b = srgb_linear(rgb[3 * p + 2] / 255.0);
    const double X = 0.4124 * r + 0.3576 * g + 0.1805 * b;
    const double Y = 0.2126 * r + 0.7152 * g + 0.0722 * b;
    const double Z = 0.0193 * r + 0.1192 * g + 0.9505 * b;
    const double fx = lab_fn(X / 0.95047), fy = lab_fn(Y / 1.0), fz = lab_fn(Z / 1.08883);
    lab[3 * p] = 116.0 * fy - 16.0;
    lab[3 * p + 1] = 500.0 * (fx - fy);
    lab[3 * p + 2] = 200.0 * (fy - fz);
  }
  return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* The contour mask the paper draws its superpixels with (Sec. 4, the
 * visualisation paragraph: the image is masked where the label contour is
 * non-zero).  Reading: a voxel is on the contour when one of its face
 * neighbours inside the image carries a different label (neighbours outside
 * the image do not count); such voxels become 0 in every channel and every
 * other voxel keeps its value. */
int or_mask_contours(const void* img, int nd, const int64_t* dims, int C, int dtype,
                     const int32_t* labels, void* out) {
  img_t g;
  int rc = make_img(&g, img, nd, dims, C, dtype);
  if (rc) return rc;
  const size_t vox_bytes = (size_t)C * (dtype == OR_U8 ? 1 : dtype == OR_U16 ? 2 : 4);
  for (int64_t v = 0; v < g.N; ++v) {
    int on_contour = 0;
    int64_t rest = v;
    for (int i = 0; i < nd; ++i) {
      const int64_t x = rest % g.n[i];
      rest /= g.n[i];
      if (x > 0 && labels[v - g.stride[i]] != labels[v]) on_contour = 1;
      if (x + 1 < g.n[i] && labels[v + g.stride[i]] != labels[v]) on_contour = 1;
    }
    unsigned char* dst = (unsigned char*)out + (size_t)v * vox_bytes;
    if (on_contour) memset(dst, 0, vox_bytes);
    else memcpy(dst, (const unsigned char*)img + (size_t)v * vox_bytes, vox_bytes);
  }
  return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* The whole filter: stage 1, the iterations of stage 2 and stage 3 (Sec. 3.1),
 * stopping early only when the residual drops below `tol` (Sec. 2.2
 * termination criterion; tol = 0 runs every iteration, as SSLIC does).  With
 * persist_distance the distance image lives across the iterations (stage 1
 * of Sec. 2.2 and Sec. 3.1 sets it to infinity once). */

int or_run(const void* img, int nd, const int64_t* dims, int C, int dtype,
           const int32_t* S, double m, int iterations, double tol, int connectivity,
           int persist_distance, const double* init_centres, int32_t* labels,
           double* centres, int64_t* counts, double* residuals, int* iters_done,
           int32_t* n_labels) {
  img_t g;
  int rc = make_img(&g, img, nd, dims, C, dtype);
  if (rc) return rc;
  if (iterations < 1 || !(m > 0.0)) return OR_EINVAL;
  int64_t K;
  rc = or_num_clusters(nd, dims, S, NULL, &K);
  if (rc) return rc;
  const int row = C + nd;
  if (init_centres) memcpy(centres, init_centres, sizeof(double) * (size_t)(K * row));
  else if ((rc = or_seed(img, nd, dims, C, dtype, S, centres))) return rc;
  or_grid_labels(nd, dims, S, labels);
  double* dist = NULL;
  if (persist_distance) {
    dist = (double*)malloc(sizeof(double) * (size_t)g.N);
    if (!dist) return OR_ENOMEM;
    for (int64_t v = 0; v < g.N; ++v) dist[v] = INFINITY; /* once, before the loop */
  }
  int t = 0;
  for (t = 0; t < iterations; ++t) {
    rc = dist ? or_assign_persist(img, nd, dims, C, dtype, S, m, centres, K, labels, dist)
              : or_assign(img, nd, dims, C, dtype, S, m, centres, K, labels);
    double e = 0.0;
    if (!rc) rc = or_update(img, nd, dims, C, dtype, S, m, labels, K, centres, counts, &e);
    if (rc) {
      free(dist);
      return rc;
    }
    if (residuals) residuals[t] = e;
    if (e < tol) {
      ++t;
      break;
    }
  }
  free(dist);
  if (iters_done) *iters_done = t;
  int32_t nl = (int32_t)K;
  if (connectivity) {
    if ((rc = or_connectivity(nd, dims, S, centres, C, K, labels, &nl))) return rc;
  }
  if (n_labels) *n_labels = nl;
  return OR_OK;
}
