/*
 * vgoracle.c -- plain, slow FP64 CPU oracle for the batched RayCast of the
 * Voronoi Graph method (Sikorski & Heida, "Voronoi Graph - Improved raycasting
 * and integration schemes for high dimensional Voronoi diagrams",
 * arXiv 2405.10050).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the package smoke check and the bench's CPU
 * baseline do.  It shares no code, header or table with the HIP library.
 *
 * Every floating-point quantity is FP64.  Inputs given as float32 by the
 * callers are promoted exactly before they get here.
 *
 * Contents
 *   vgo_raycast           definition of the RayCast result (Sec. 2.2, eq. (t),
 *                         with the half-space restriction `skip` of
 *                         Algorithm 1): brute force over all nodes.
 *   vgo_raycast_incircle  Algorithm 1 itself (iterative nearest-neighbour
 *                         projection, optional InitialHeuristic), with a
 *                         brute-force `nn`; used as a cross-check of
 *                         vgo_raycast and to count `nn` calls (Table nncalls).
 *   vgo_explore           Algorithm 2 (VoronoiGraph exhaustive search with the
 *                         edge visit counter), Descent, SearchDirection and
 *                         the vertex coordinates of Sec. 2.1.
 *   vgo_explore_clipped   Algorithm 2 on the diagram clipped to the unit
 *                         cube: the faces of the cube join the generators
 *                         as constraints of a vertex (face x_k = s has the
 *                         code n + 2k + s in a key).
 *   vgo_explore_periodic  Algorithm 2 on the periodic diagram (the torus
 *                         R^d / Z^d): key entries are node images coded by
 *                         node and lattice shift, rays are cast over the
 *                         images in [-1,2)^d.
 *   vgo_mc_ray_weights    per-ray terms of the Monte-Carlo estimators of
 *                         Sec. 3.1 / Algorithm 3 (volume, area, and the
 *                         second moment used for the centroidal energy).
 *   vgo_mc_adjoint        closed-form derivative of those estimators with
 *                         frozen directions (not in the paper; derived from
 *                         eq. (t)).
 *
 * Index convention of a ray result: idx >= 0 is a node; -1 means no hit
 * (the ray leaves to infinity); -2-(2k+s) is the face x_k = s of the unit
 * cube (s = 0 or 1) when clipping is on.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define VGO_INF (1.0 / 0.0)

/* ------------------------------------------------------------------------ */
/* small vector helpers                                                      */
/* ------------------------------------------------------------------------ */
static double dot(const double *a, const double *b, int d) {
  double s = 0.0;
  for (int k = 0; k < d; ++k) s += a[k] * b[k];
  return s;
}

static double dist2(const double *a, const double *b, int d) {
  double s = 0.0;
  for (int k = 0; k < d; ++k) {
    double e = a[k] - b[k];
    s += e * e;
  }
  return s;
}

static int in_list(int32_t v, const int32_t *list, int n) {
  for (int a = 0; a < n; ++a)
    if (list[a] == v) return 1;
  return 0;
}

/* Exit of the ray x + t u from the unit cube [0,1]^d: smallest positive
 * t over the faces crossed in direction u.  Returns the face code 2k+s. */
static double box_exit(const double *x, const double *u, int d, int *face) {
  double tb = VGO_INF;
  *face = -1;
  for (int k = 0; k < d; ++k) {
    double tk;
    int f;
    if (u[k] > 0.0) {
      tk = (1.0 - x[k]) / u[k];
      f = 2 * k + 1;
    } else if (u[k] < 0.0) {
      tk = (0.0 - x[k]) / u[k];
      f = 2 * k;
    } else {
      continue;
    }
    if (tk < tb) {
      tb = tk;
      *face = f;
    }
  }
  return tb;
}

/* ------------------------------------------------------------------------ */
/* O1: the RayCast result by definition.                                     */
/*                                                                           */
/* The ray starts at x (a point equidistant to the generators eta, in the    */
/* cell of g = X[eta_1]) and runs along u.  Along the ray the point          */
/* x + t u stays at least as close to g as to node r exactly while           */
/*     2 t u.(r - g) <= |r - x|^2 - |g - x|^2                                */
/* (expand both squared distances, Sec. 2.2).  So the first bisector hit is  */
/* the smallest t of eq. (t) over the nodes in the forward half-space        */
/* u.(r - g) > 0 (the `skip` predicate of Algorithm 1) that are not in eta.  */
/* Equal t: the lowest node index wins; a node wins against the cube on      */
/* equality.                                                                 */
/* ------------------------------------------------------------------------ */
static void raycast_one(int d, int64_t n, const double *X, const double *x,
                        const double *u, int32_t g, const int32_t *excl,
                        int n_excl, int clip, double *t1, int32_t *i1,
                        double *t2) {
  const double *xg = X + (int64_t)g * d;
  double best = VGO_INF, second = VGO_INF;
  int32_t bi = -1;
  for (int64_t r = 0; r < n; ++r) {
    if (excl && in_list((int32_t)r, excl, n_excl)) continue;
    const double *xr = X + r * d;
    double den = 0.0;
    for (int k = 0; k < d; ++k) den += u[k] * (xr[k] - xg[k]);
    if (!(den > 0.0)) continue;
    /* |r - x|^2 - |g - x|^2 written as the difference of squares
     * (r - g).((r - x) + (g - x)): the same quantity, without cancelling two
     * |x|^2-sized terms when the origin is a far vertex of the diagram */
    double num = 0.0;
    for (int k = 0; k < d; ++k) num += (xr[k] - xg[k]) * ((xr[k] - x[k]) + (xg[k] - x[k]));
    double t = num / (2.0 * den);
    if (t < best) {
      second = best;
      best = t;
      bi = (int32_t)r;
    } else if (t < second) {
      second = t;
    }
  }
  if (clip) {
    int face;
    double tb = box_exit(x, u, d, &face);
    if (face >= 0) {
      if (tb < best) {
        second = best;
        best = tb;
        bi = -2 - face;
      } else if (tb < second) {
        second = tb;
      }
    }
  }
  *t1 = best;
  *i1 = bi;
  *t2 = second;
}

/* Rays are rows of origin/dir ([m][d]); gen[m] is the index g of the known
 * generator; excl is [m][n_excl] (may be NULL when n_excl == 0).  Outputs:
 * t (INF when no hit), idx, and the second-smallest candidate t2 (INF when
 * there is none), which the tests use to mark near-ties. */
int vgo_raycast(int d, int64_t n, const double *X, int64_t m,
                const double *origin, const double *dir, const int32_t *gen,
                const int32_t *excl, int n_excl, int clip, double *t_out,
                int32_t *idx_out, double *t2_out) {
  if (d < 1 || n < 0 || m < 0) return -1;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < m; ++k) {
    raycast_one(d, n, X, origin + k * d, dir + k * d, gen[k],
                excl ? excl + k * n_excl : NULL, n_excl, clip, &t_out[k],
                &idx_out[k], &t2_out[k]);
  }
  return 0;
}

/* Monte-Carlo rays (Algorithm 3): the ray of cell i starts at x_i, eta = {i},
 * g = i, with clipping to the unit cube.  dirs is [n_cells][n_rays][d] for
 * the listed cells. */
int vgo_raycast_cells(int d, int64_t n, const double *X, int64_t n_cells,
                      const int64_t *cells, int n_rays, const double *dirs,
                      double *t_out, int32_t *idx_out, double *t2_out) {
  if (d < 1 || n < 1 || n_cells < 0 || n_rays < 0) return -1;
  int64_t m = n_cells * (int64_t)n_rays;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < m; ++k) {
    int64_t c = k / n_rays;
    int32_t i = (int32_t)cells[c];
    raycast_one(d, n, X, X + (int64_t)i * d, dirs + k * d, i, &i, 1, 1,
                &t_out[k], &idx_out[k], &t2_out[k]);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* O5: Algorithm 1, the iterative incircle RayCast, with a brute-force nn.   */
/* ------------------------------------------------------------------------ */
/* nn(p, skip): nearest node to p among those not skipped; skip(i) holds when
 * <X_i,u> <= max_{g in eta} <x_g,u>.  Returns -1 when every node is skipped.
 * Equal distances: lowest index. */
static int32_t nn_skip(int d, int64_t n, const double *X, const double *p,
                       const double *u, double hmax) {
  double bd = VGO_INF;
  int32_t bi = -1;
  for (int64_t r = 0; r < n; ++r) {
    const double *xr = X + r * d;
    if (dot(xr, u, d) <= hmax) continue;
    double e = dist2(xr, p, d);
    if (e < bd) {
      bd = e;
      bi = (int32_t)r;
    }
  }
  return bi;
}

/* One incircle RayCast (Algorithm 1).  eta has n_eta entries, eta[0] is the
 * generator x_0 used in eq. (t).  Returns the node j completing the vertex
 * (or -1), the new point in r_out and the number of nn calls in *calls.
 * heuristic != 0 applies InitialHeuristic first (only when |eta| >= 2: with
 * one generator its scale factor divides by zero). */
static int32_t incircle_one(int d, int64_t n, const double *X,
                            const int32_t *eta, int n_eta, const double *r0,
                            const double *u, int heuristic, double *r_out,
                            int64_t *calls) {
  const double *x0 = X + (int64_t)eta[0] * d;
  double r[64], rp[64];
  for (int k = 0; k < d; ++k) r[k] = r0[k];
  if (heuristic && n_eta >= 2) {
    /* project r onto the plane through x0 orthogonal to u, then walk the
     * height of a regular simplex over the face (Sec. 2.2, heuristic) */
    double a = 0.0;
    for (int k = 0; k < d; ++k) a += u[k] * (x0[k] - r[k]);
    for (int k = 0; k < d; ++k) r[k] += a * u[k];
    double rad = sqrt(dist2(r, x0, d));
    double dd = (double)n_eta;
    double h = rad / sqrt((dd - 1.0) * (dd + 1.0));
    for (int k = 0; k < d; ++k) r[k] += h * u[k];
  }
  double hmax = -VGO_INF;
  for (int a = 0; a < n_eta; ++a) {
    double v = dot(X + (int64_t)eta[a] * d, u, d);
    if (v > hmax) hmax = v;
  }
  int32_t i = nn_skip(d, n, X, r, u, hmax);
  (*calls)++;
  if (i < 0) return -1;
  for (int iter = 0; iter < 100000; ++iter) {
    const double *x = X + (int64_t)i * d;
    double num = dist2(r, x, d) - dist2(r, x0, d);
    double den = 0.0;
    for (int k = 0; k < d; ++k) den += u[k] * (x[k] - x0[k]);
    double t = num / (2.0 * den);
    for (int k = 0; k < d; ++k) rp[k] = r[k] + t * u[k];
    int32_t j = nn_skip(d, n, X, rp, u, hmax);
    (*calls)++;
    if (j == i) {
      for (int k = 0; k < d; ++k) r_out[k] = rp[k];
      return i;
    }
    if (j < 0) return -1;
    i = j;
  }
  return -1;
}

/* Batched entry for the cross-check: rays given like vgo_raycast with
 * excl = eta ([m][n_eta], eta[0] = g).  Clipping is off. */
int vgo_raycast_incircle(int d, int64_t n, const double *X, int64_t m,
                         const double *origin, const double *dir,
                         const int32_t *eta, int n_eta, int heuristic,
                         double *t_out, int32_t *idx_out, int64_t *calls_out) {
  if (d < 1 || d > 64 || n_eta < 1) return -1;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < m; ++k) {
    double rp[64];
    int64_t calls = 0;
    const double *x = origin + k * d, *u = dir + k * d;
    int32_t j = incircle_one(d, n, X, eta + k * n_eta, n_eta, x, u, heuristic,
                             rp, &calls);
    idx_out[k] = j;
    calls_out[k] = calls;
    if (j >= 0) {
      /* report t measured from the given origin along u */
      double t = 0.0;
      for (int a = 0; a < d; ++a) t += (rp[a] - x[a]) * u[a];
      t_out[k] = t;
    } else {
      t_out[k] = VGO_INF;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Dense linear algebra for Sec. 2.1 (vertex coordinates) and Algorithm 2's  */
/* SearchDirection.                                                          */
/* ------------------------------------------------------------------------ */
/* Solve A y = b (A is [d][d], row-major, overwritten) by Gaussian elimination
 * with partial pivoting.  Returns 0, or -1 when a pivot vanishes. */
static int solve_dense(int d, double *A, double *b, double *y) {
  for (int c = 0; c < d; ++c) {
    int p = c;
    double pv = fabs(A[c * d + c]);
    for (int r = c + 1; r < d; ++r)
      if (fabs(A[r * d + c]) > pv) {
        pv = fabs(A[r * d + c]);
        p = r;
      }
    if (pv == 0.0) return -1;
    if (p != c) {
      for (int k = 0; k < d; ++k) {
        double tmp = A[c * d + k];
        A[c * d + k] = A[p * d + k];
        A[p * d + k] = tmp;
      }
      double tmp = b[c];
      b[c] = b[p];
      b[p] = tmp;
    }
    for (int r = c + 1; r < d; ++r) {
      double f = A[r * d + c] / A[c * d + c];
      for (int k = c; k < d; ++k) A[r * d + k] -= f * A[c * d + k];
      b[r] -= f * b[c];
    }
  }
  for (int c = d - 1; c >= 0; --c) {
    double s = b[c];
    for (int k = c + 1; k < d; ++k) s -= A[c * d + k] * y[k];
    y[c] = s / A[c * d + c];
  }
  return 0;
}

/* The vertex of the generators sigma (d+1 of them) is the point equidistant
 * to all of them (Sec. 2.1): with y = v - x_a and e_b = x_b - x_a,
 * |v - x_b|^2 = |v - x_a|^2  <=>  2 e_b . y = |e_b|^2  for b != a. */
static int circumcentre(int d, const double *X, const int32_t *sigma,
                        double *v) {
  double A[64 * 64], b[64], y[64];
  const double *xa = X + (int64_t)sigma[0] * d;
  for (int r = 0; r < d; ++r) {
    const double *xb = X + (int64_t)sigma[r + 1] * d;
    double s = 0.0;
    for (int k = 0; k < d; ++k) {
      double e = xb[k] - xa[k];
      A[r * d + k] = 2.0 * e;
      s += e * e;
    }
    b[r] = s;
  }
  if (solve_dense(d, A, b, y)) return -1;
  for (int k = 0; k < d; ++k) v[k] = xa[k] + y[k];
  return 0;
}

/* Remove from w its components along the span of the vectors
 * {X[s_j] - X[s_0]} (j = 1..m-1), by Gram-Schmidt applied twice. */
static void project_out_span(int d, const double *X, const int32_t *s, int m,
                             double *w) {
  double Q[64 * 64];
  int q = 0;
  const double *x0 = X + (int64_t)s[0] * d;
  for (int j = 1; j < m; ++j) {
    double *e = Q + q * d;
    const double *xj = X + (int64_t)s[j] * d;
    for (int k = 0; k < d; ++k) e[k] = xj[k] - x0[k];
    for (int pass = 0; pass < 2; ++pass)
      for (int a = 0; a < q; ++a) {
        double c = dot(e, Q + a * d, d);
        for (int k = 0; k < d; ++k) e[k] -= c * Q[a * d + k];
      }
    double nr = sqrt(dot(e, e, d));
    if (nr == 0.0) continue;
    for (int k = 0; k < d; ++k) e[k] /= nr;
    ++q;
  }
  for (int pass = 0; pass < 2; ++pass)
    for (int a = 0; a < q; ++a) {
      double c = dot(w, Q + a * d, d);
      for (int k = 0; k < d; ++k) w[k] -= c * Q[a * d + k];
    }
}

/* SearchDirection(sigma, eta) of Algorithm 2: unit vector orthogonal to the
 * affine span of X_eta pointing away from the omitted generator.  It is the
 * normalised negative of the component of (x_omit - x_eta1) orthogonal to
 * that span.  Returns -1 when that component vanishes. */
static int search_direction(int d, const double *X, const int32_t *eta,
                            int32_t omit, double *u) {
  const double *x0 = X + (int64_t)eta[0] * d;
  const double *xo = X + (int64_t)omit * d;
  for (int k = 0; k < d; ++k) u[k] = xo[k] - x0[k];
  project_out_span(d, X, eta, d, u);
  double nr = sqrt(dot(u, u, d));
  if (!(nr > 0.0)) return -1;
  for (int k = 0; k < d; ++k) u[k] = -u[k] / nr;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Open-addressing map keyed by sorted int32 tuples of a fixed length.       */
/* ------------------------------------------------------------------------ */
typedef struct {
  int L;
  int64_t cap, size;
  int32_t *keys;
  int64_t *vals;
  uint8_t *used;
} tmap;

static uint64_t tuple_hash(const int32_t *k, int L) {
  uint64_t h = 0x9E3779B97F4A7C15ULL;
  for (int a = 0; a < L; ++a) {
    h ^= (uint64_t)(uint32_t)k[a];
    h *= 0xFF51AFD7ED558CCDULL;
    h ^= h >> 32;
  }
  return h;
}

static int tmap_init(tmap *m, int L, int64_t cap) {
  int64_t c = 1024;
  while (c < cap) c <<= 1;
  m->L = L;
  m->cap = c;
  m->size = 0;
  m->keys = (int32_t *)malloc(sizeof(int32_t) * (size_t)(c * L));
  m->vals = (int64_t *)malloc(sizeof(int64_t) * (size_t)c);
  m->used = (uint8_t *)calloc((size_t)c, 1);
  return (m->keys && m->vals && m->used) ? 0 : -1;
}

static void tmap_free(tmap *m) {
  free(m->keys);
  free(m->vals);
  free(m->used);
}

static int64_t *tmap_slot(tmap *m, const int32_t *key, int create, int *created);

static int tmap_grow(tmap *m) {
  tmap n;
  if (tmap_init(&n, m->L, m->cap * 2)) return -1;
  for (int64_t s = 0; s < m->cap; ++s)
    if (m->used[s]) {
      int cr;
      *tmap_slot(&n, m->keys + s * m->L, 1, &cr) = m->vals[s];
    }
  tmap_free(m);
  *m = n;
  return 0;
}

/* Find the value slot of key; insert (value 0) when create != 0. */
static int64_t *tmap_slot(tmap *m, const int32_t *key, int create, int *created) {
  *created = 0;
  if (create && 2 * (m->size + 1) > m->cap)
    if (tmap_grow(m)) return NULL;
  uint64_t s = tuple_hash(key, m->L) & (uint64_t)(m->cap - 1);
  for (;;) {
    if (!m->used[s]) {
      if (!create) return NULL;
      m->used[s] = 1;
      memcpy(m->keys + (int64_t)s * m->L, key, sizeof(int32_t) * m->L);
      m->vals[s] = 0;
      m->size++;
      *created = 1;
      return &m->vals[s];
    }
    if (!memcmp(m->keys + (int64_t)s * m->L, key, sizeof(int32_t) * m->L))
      return &m->vals[s];
    s = (s + 1) & (uint64_t)(m->cap - 1);
  }
}

static void sort_small(int32_t *a, int n) {
  for (int i = 1; i < n; ++i) {
    int32_t v = a[i];
    int j = i - 1;
    while (j >= 0 && a[j] > v) {
      a[j + 1] = a[j];
      --j;
    }
    a[j + 1] = v;
  }
}

/* ------------------------------------------------------------------------ */
/* O2: Algorithm 2 (VoronoiGraph).                                           */
/* ------------------------------------------------------------------------ */
typedef struct {
  int d;
  int64_t nv, capv, nb, capb;
  int32_t *sig;   /* [capv][d+1] sorted generator tuples, discovery order */
  double *coord;  /* [capv][d] */
  int32_t *bsig;  /* [capb][d+1] vertex of each unbounded edge */
  int32_t *bomit; /* [capb] generator omitted from that vertex */
  int64_t raycasts, nn_calls, duplicates;
} vgo_mesh;

static int mesh_push_vertex(vgo_mesh *M, const int32_t *s, const double *v) {
  int d = M->d;
  if (M->nv == M->capv) {
    int64_t c = M->capv ? 2 * M->capv : 1024;
    int32_t *ns = (int32_t *)realloc(M->sig, sizeof(int32_t) * (size_t)(c * (d + 1)));
    if (!ns) return -1;
    M->sig = ns;
    double *nc = (double *)realloc(M->coord, sizeof(double) * (size_t)(c * d));
    if (!nc) return -1;
    M->coord = nc;
    M->capv = c;
  }
  memcpy(M->sig + M->nv * (d + 1), s, sizeof(int32_t) * (d + 1));
  memcpy(M->coord + M->nv * d, v, sizeof(double) * d);
  M->nv++;
  return 0;
}

static int mesh_push_boundary(vgo_mesh *M, const int32_t *s, int32_t omit) {
  int d = M->d;
  if (M->nb == M->capb) {
    int64_t c = M->capb ? 2 * M->capb : 256;
    int32_t *ns = (int32_t *)realloc(M->bsig, sizeof(int32_t) * (size_t)(c * (d + 1)));
    if (!ns) return -1;
    M->bsig = ns;
    int32_t *no = (int32_t *)realloc(M->bomit, sizeof(int32_t) * (size_t)c);
    if (!no) return -1;
    M->bomit = no;
    M->capb = c;
  }
  memcpy(M->bsig + M->nb * (d + 1), s, sizeof(int32_t) * (d + 1));
  M->bomit[M->nb] = omit;
  M->nb++;
  return 0;
}

/* one RayCast along (eta, x, u) without clipping; mode 0 = definition,
 * 1 = Algorithm 1, 2 = Algorithm 1 with InitialHeuristic */
static int32_t cast(int d, int64_t n, const double *X, const int32_t *eta,
                    int n_eta, const double *x, const double *u, int mode,
                    double *t, vgo_mesh *M) {
  M->raycasts++;
  if (mode == 0) {
    double t2;
    int32_t j;
    raycast_one(d, n, X, x, u, eta[0], eta, n_eta, 0, t, &j, &t2);
    return j;
  }
  double rp[64];
  int32_t j = incircle_one(d, n, X, eta, n_eta, x, u, mode == 2, rp, &M->nn_calls);
  if (j >= 0) {
    double s = 0.0;
    for (int k = 0; k < d; ++k) s += (rp[k] - x[k]) * u[k];
    *t = s;
  }
  return j;
}

/* Descent of Algorithm 2: from sigma = {start}, r = X[start] (node 0 for
 * the unbounded diagram), cast rays onto faces of
 * decreasing dimension until d+1 generators are known.  Each step takes the
 * next Gaussian draw as the search direction, removes its component in the
 * span of X_sigma, and casts with eta = sigma; a step whose ray escapes is
 * retried with -u and then with the next draw. */
static int descent(int d, int64_t n, const double *X, int32_t start,
                   const double *draws, int n_draws, int mode, int32_t *sigma,
                   double *v, vgo_mesh *M) {
  int m = 1;
  int used = 0;
  double r[64], u[64];
  sigma[0] = start;
  for (int k = 0; k < d; ++k) r[k] = X[(int64_t)start * d + k];
  while (m < d + 1) {
    if (used >= n_draws) return -1;
    for (int k = 0; k < d; ++k) u[k] = draws[used * d + k];
    used++;
    project_out_span(d, X, sigma, m, u);
    double nr = sqrt(dot(u, u, d));
    if (!(nr > 0.0)) continue;
    for (int k = 0; k < d; ++k) u[k] /= nr;
    double t;
    int32_t j = cast(d, n, X, sigma, m, r, u, mode, &t, M);
    if (j < 0) {
      for (int k = 0; k < d; ++k) u[k] = -u[k];
      j = cast(d, n, X, sigma, m, r, u, mode, &t, M);
    }
    if (j < 0) continue;
    for (int k = 0; k < d; ++k) r[k] += t * u[k];
    sigma[m++] = j;
  }
  sort_small(sigma, d + 1);
  return circumcentre(d, X, sigma, v);
}

/* Algorithm 2.  Readings:
 *  - the queue is FIFO and the vertex set V is keyed by the sorted tuple;
 *  - the start vertex's d+1 edges are counted like any discovered vertex's
 *    (otherwise its neighbours would cast back onto it);
 *  - RayCast runs without clipping: V is the vertex set of the unbounded
 *    diagram and B holds its unbounded edges as (vertex, omitted generator);
 *  - vertex coordinates are solved from sigma in FP64 (Sec. 2.1 stores each
 *    vertex as (sigma, r)) and rays start from those coordinates.
 * mode selects the RayCast: 0 = definition (vgo_raycast), 1/2 = Algorithm 1
 * without/with InitialHeuristic (counts nn calls). */
void *vgo_explore(int d, int64_t n, const double *X, const double *draws,
                  int n_draws, int mode) {
  if (d < 1 || d > 63 || n < d + 1) return NULL;
  vgo_mesh *M = (vgo_mesh *)calloc(1, sizeof(vgo_mesh));
  if (!M) return NULL;
  M->d = d;
  tmap G, V;
  int ok = !tmap_init(&G, d, 1 << 12) && !tmap_init(&V, d + 1, 1 << 12);
  int32_t s0[64], eta[64], key[64];
  double v0[64], u[64], v[64];
  int cr;
  if (!ok || descent(d, n, X, 0, draws, n_draws, mode, s0, v0, M)) goto fail;
  if (mesh_push_vertex(M, s0, v0)) goto fail;
  *tmap_slot(&V, s0, 1, &cr) = 0;
  for (int o = 0; o <= d; ++o) { /* E(sigma): omit one generator */
    int a = 0;
    for (int b = 0; b <= d; ++b)
      if (b != o) eta[a++] = s0[b];
    *tmap_slot(&G, eta, 1, &cr) += 1;
  }
  for (int64_t head = 0; head < M->nv; ++head) { /* pop in FIFO order */
    int32_t sig[64];
    double r[64];
    memcpy(sig, M->sig + head * (d + 1), sizeof(int32_t) * (d + 1));
    memcpy(r, M->coord + head * d, sizeof(double) * d);
    for (int o = 0; o <= d; ++o) {
      int a = 0;
      for (int b = 0; b <= d; ++b)
        if (b != o) eta[a++] = sig[b];
      int64_t *gc = tmap_slot(&G, eta, 0, &cr);
      if (gc && *gc >= 2) continue;
      if (search_direction(d, X, eta, sig[o], u)) continue;
      double t;
      int32_t j = cast(d, n, X, eta, d, r, u, mode, &t, M);
      if (j < 0) {
        if (mesh_push_boundary(M, sig, sig[o])) goto fail;
        continue;
      }
      for (int b = 0; b < d; ++b) key[b] = eta[b];
      key[d] = j;
      sort_small(key, d + 1);
      int64_t *vs = tmap_slot(&V, key, 1, &cr);
      if (!vs) goto fail;
      if (!cr) {
        M->duplicates++;
        continue;
      }
      *vs = M->nv;
      if (circumcentre(d, X, key, v)) goto fail;
      if (mesh_push_vertex(M, key, v)) goto fail;
      for (int o2 = 0; o2 <= d; ++o2) {
        int a2 = 0;
        int32_t e2[64];
        for (int b = 0; b <= d; ++b)
          if (b != o2) e2[a2++] = key[b];
        int64_t *g2 = tmap_slot(&G, e2, 1, &cr);
        if (!g2) goto fail;
        *g2 += 1;
      }
    }
  }
  tmap_free(&G);
  tmap_free(&V);
  return M;
fail:
  tmap_free(&G);
  tmap_free(&V);
  free(M->sig);
  free(M->coord);
  free(M->bsig);
  free(M->bomit);
  free(M);
  return NULL;
}

/* ------------------------------------------------------------------------ */
/* O2b: Algorithm 2 on the clipped diagram.                                  */
/*                                                                           */
/* The cells are C_i intersected with the unit cube.  A vertex of the        */
/* clipped diagram is a point of the cube fixed by d+1 constraints: a >= 1   */
/* generators at a common smallest distance, and d+1-a faces x_k = s it lies */
/* on.  Its key is the sorted tuple of the generator indices and the face    */
/* codes n + 2k + s (so generators come first).  An edge keeps d of the      */
/* constraints (at least one generator): the points that satisfy them form a */
/* line, and the edge leaves the vertex along that line, away from the       */
/* dropped constraint: away from a dropped generator j (it gets farther than */
/* the kept ones), or off a dropped face into the cube.  RayCast with        */
/* clipping ends the edge at the next generator or face.  Every edge is      */
/* bounded, so every edge is found from both ends.  The search starts at the */
/* corner 0, which lies in the cell of its nearest generator and on the d    */
/* faces x_k = 0.                                                            */
/* ------------------------------------------------------------------------ */

/* The vertex fixed by the d+1 constraints `key` (generator key[0] first):
 * with y = v - x_a, each further generator b gives 2 (x_b - x_a).y =
 * |x_b - x_a|^2 and each face x_k = s gives y_k = s - x_a,k.  Face
 * coordinates are then set exactly. */
static int clipped_vertex(int d, int64_t n, const double *X, const int32_t *key,
                          double *v) {
  double A[64 * 64], b[64], y[64];
  const double *xa = X + (int64_t)key[0] * d;
  for (int r = 0; r < d; ++r) {
    int32_t c = key[r + 1];
    for (int k = 0; k < d; ++k) A[r * d + k] = 0.0;
    if (c < n) {
      const double *xb = X + (int64_t)c * d;
      double s2 = 0.0;
      for (int k = 0; k < d; ++k) {
        double e = xb[k] - xa[k];
        A[r * d + k] = 2.0 * e;
        s2 += e * e;
      }
      b[r] = s2;
    } else {
      int f = (int)(c - n), k = f / 2;
      A[r * d + k] = 1.0;
      b[r] = (double)(f % 2) - xa[k];
    }
  }
  if (solve_dense(d, A, b, y)) return -1;
  for (int k = 0; k < d; ++k) v[k] = xa[k] + y[k];
  for (int r = 1; r <= d; ++r)
    if (key[r] >= n) {
      int f = (int)(key[r] - n);
      v[f / 2] = (double)(f % 2);
    }
  return 0;
}

/* Direction of the edge that keeps the constraints eta (d of them, sorted,
 * eta[0] a generator) and drops `omit`: the unit vector orthogonal to the
 * kept faces' normals e_k and to x_g - x_eta0 for the kept generators g,
 * pointing away from x_omit (a generator) or into the cube (a face).  Built
 * as the component of w orthogonal to those vectors, by Gram-Schmidt applied
 * twice with the face normals first, where w = -(x_omit - x_eta0) for a
 * generator and w = +-e_k (into the cube) for a face.  Returns -1 when the
 * component vanishes. */
static int clipped_direction(int d, int64_t n, const double *X, const int32_t *eta,
                             int32_t omit, double *u) {
  double Q[64 * 64];
  int q = 0;
  const double *x0 = X + (int64_t)eta[0] * d;
  for (int pass_kind = 0; pass_kind < 2; ++pass_kind) {
    for (int a = 0; a < d; ++a) {
      int is_f = eta[a] >= n;
      if (is_f != (pass_kind == 0) || (!is_f && a == 0)) continue;
      double *e = Q + q * d;
      if (is_f) {
        int k = (int)(eta[a] - n) / 2;
        for (int c = 0; c < d; ++c) e[c] = (c == k) ? 1.0 : 0.0;
      } else {
        const double *xg = X + (int64_t)eta[a] * d;
        for (int c = 0; c < d; ++c) e[c] = xg[c] - x0[c];
      }
      for (int pass = 0; pass < 2; ++pass)
        for (int b = 0; b < q; ++b) {
          double c = dot(e, Q + b * d, d);
          for (int k = 0; k < d; ++k) e[k] -= c * Q[b * d + k];
        }
      double nr = sqrt(dot(e, e, d));
      if (nr == 0.0) continue;
      for (int k = 0; k < d; ++k) e[k] /= nr;
      ++q;
    }
  }
  if (omit < n) {
    const double *xo = X + (int64_t)omit * d;
    for (int k = 0; k < d; ++k) u[k] = x0[k] - xo[k];
  } else {
    int f = (int)(omit - n), k = f / 2;
    for (int c = 0; c < d; ++c) u[c] = 0.0;
    u[k] = (f % 2) ? -1.0 : 1.0;
  }
  for (int pass = 0; pass < 2; ++pass)
    for (int b = 0; b < q; ++b) {
      double c = dot(u, Q + b * d, d);
      for (int k = 0; k < d; ++k) u[k] -= c * Q[b * d + k];
    }
  double nr = sqrt(dot(u, u, d));
  if (!(nr > 0.0)) return -1;
  for (int k = 0; k < d; ++k) u[k] /= nr;
  return 0;
}

void *vgo_explore_clipped(int d, int64_t n, const double *X) {
  if (d < 1 || d > 62 || n < 1) return NULL;
  vgo_mesh *M = (vgo_mesh *)calloc(1, sizeof(vgo_mesh));
  if (!M) return NULL;
  M->d = d;
  tmap G, V;
  int ok = !tmap_init(&G, d, 1 << 12) && !tmap_init(&V, d + 1, 1 << 12);
  int32_t s0[64], eta[64], key[64], gens[64];
  double v[64], u[64];
  int cr;
  if (!ok) goto fail;
  {
    /* start: the corner 0 and its nearest generator (lowest index on ties) */
    int64_t g0 = 0;
    double best = VGO_INF;
    for (int64_t i = 0; i < n; ++i) {
      double s2 = dot(X + i * d, X + i * d, d);
      if (s2 < best) {
        best = s2;
        g0 = i;
      }
    }
    s0[0] = (int32_t)g0;
    for (int k = 0; k < d; ++k) s0[k + 1] = (int32_t)(n + 2 * k);
    for (int k = 0; k < d; ++k) v[k] = 0.0;
    if (mesh_push_vertex(M, s0, v)) goto fail;
    *tmap_slot(&V, s0, 1, &cr) = 0;
    for (int o = 0; o <= d; ++o) {
      int a = 0;
      for (int b = 0; b <= d; ++b)
        if (b != o) eta[a++] = s0[b];
      *tmap_slot(&G, eta, 1, &cr) += 1;
    }
  }
  for (int64_t head = 0; head < M->nv; ++head) {
    int32_t sig[64];
    double r[64];
    memcpy(sig, M->sig + head * (d + 1), sizeof(int32_t) * (d + 1));
    memcpy(r, M->coord + head * d, sizeof(double) * d);
    for (int o = 0; o <= d; ++o) {
      int a = 0, ng = 0;
      for (int b = 0; b <= d; ++b)
        if (b != o) eta[a++] = sig[b];
      for (int b = 0; b < d; ++b)
        if (eta[b] < n) gens[ng++] = eta[b];
      if (ng == 0) continue; /* d faces meet in a corner, not along an edge */
      int64_t *gc = tmap_slot(&G, eta, 0, &cr);
      if (gc && *gc >= 2) continue;
      if (clipped_direction(d, n, X, eta, sig[o], u)) continue;
      double t, t2;
      int32_t j;
      M->raycasts++;
      raycast_one(d, n, X, r, u, eta[0], gens, ng, 1, &t, &j, &t2);
      if (j == -1) goto fail; /* a clipped ray always ends */
      int32_t code = j >= 0 ? j : (int32_t)(n + (-2 - j));
      for (int b = 0; b < d; ++b) key[b] = eta[b];
      key[d] = code;
      sort_small(key, d + 1);
      int64_t *vs = tmap_slot(&V, key, 1, &cr);
      if (!vs) goto fail;
      if (!cr) {
        M->duplicates++;
        continue;
      }
      *vs = M->nv;
      if (clipped_vertex(d, n, X, key, v)) goto fail;
      if (mesh_push_vertex(M, key, v)) goto fail;
      for (int o2 = 0; o2 <= d; ++o2) {
        int a2 = 0;
        int32_t e2[64];
        for (int b = 0; b <= d; ++b)
          if (b != o2) e2[a2++] = key[b];
        int64_t *g2 = tmap_slot(&G, e2, 1, &cr);
        if (!g2) goto fail;
        *g2 += 1;
      }
    }
  }
  tmap_free(&G);
  tmap_free(&V);
  return M;
fail:
  tmap_free(&G);
  tmap_free(&V);
  free(M->sig);
  free(M->coord);
  free(M);
  return NULL;
}

/* Exposed for the tests. */
int vgo_clipped_vertex(int d, int64_t n, const double *X, const int32_t *key, double *v) {
  return clipped_vertex(d, n, X, key, v);
}

/* ------------------------------------------------------------------------ */
/* O2c: Algorithm 2 on the periodic diagram (the flat torus R^d / Z^d).      */
/*                                                                           */
/* Every node x_i in [0,1)^d stands for all its images x_i + k, k in Z^d; a  */
/* vertex is a point equidistant to d+1 images with no image closer.  A key  */
/* entry is an image, coded i S + c(k) with S = 3^d and                      */
/* c(k) = sum_a (k_a + 1) 3^a for k in {-1,0,1}^d.  The keys of one vertex   */
/* differ by a lattice translation; the canonical one is translated so that  */
/* the entry of the smallest node index has k = 0, and the vertex            */
/* coordinates are solved in that frame.  An edge (d entries) is             */
/* canonicalised the same way.  Requirement: every vertex's empty ball has   */
/* radius below 1/2.  Then the images of one key belong to distinct nodes    */
/* and their shifts relative to each other lie in {-1,0,1}^d, so keys stay   */
/* in the code range; anything else is reported as a failure.                */
/*                                                                           */
/* Rays are cast by definition over the 3^d images of every node with        */
/* k in {-1,0,1}^d, i.e. every image in [-1,2)^d.  A ray whose true first    */
/* hit w is outside that set ends at a point y' whose ball (radius |y'-g|)   */
/* holds w in its interior, so it leaves [-1,2]^d: each new vertex's ball is */
/* checked to lie inside, in the frame of its ray, and a failed check (or a  */
/* ray with no hit) fails the search.                                        */
/* ------------------------------------------------------------------------ */

/* Translate the sorted key (L entries i S + c) so that its first entry has
 * k = 0; returns -1 when a shift leaves {-1,0,1}^d or a node repeats. */
static int periodic_canon(int d, int L, int32_t *key) {
  int32_t S = 1;
  for (int a = 0; a < d; ++a) S *= 3;
  int32_t c0 = key[0] % S;
  for (int e = 0; e < L; ++e) {
    int32_t id = key[e] / S, c = key[e] % S, cn = 0, p = 1, r0 = c0, r = c;
    for (int a = 0; a < d; ++a) {
      int dig = (r % 3) - (r0 % 3) + 1; /* k_a - k0_a + 1 */
      if (dig < 0 || dig > 2) return -1;
      cn += dig * p;
      p *= 3;
      r /= 3;
      r0 /= 3;
    }
    if (e > 0 && id == key[e - 1] / S) return -1;
    key[e] = id * S + cn;
  }
  return 0;
}

/* Radius of the empty ball of the vertex v of key (images in Xi) and whether
 * it lies strictly inside [-1,2]^d. */
static int ball_inside(int d, const double *Xi, const int32_t *key, const double *v) {
  double R = sqrt(dist2(v, Xi + (int64_t)key[0] * d, d));
  for (int a = 0; a < d; ++a)
    if (!(v[a] - R > -1.0 && v[a] + R < 2.0)) return 0;
  return 1;
}

/* Algorithm 2 on the torus; *status is 0, or -1 (input out of range or
 * allocation), -2 (a ball reaching past the image layer, or a ray without a
 * hit), -3 (a key outside the code range: a ball of radius >= 1/2),
 * -4 (singular vertex or failed Descent). */
void *vgo_explore_periodic(int d, int64_t n, const double *X, const double *draws,
                           int n_draws, int *status) {
  *status = -1;
  if (d < 1 || d > 12 || n < 1) return NULL;
  int64_t S = 1;
  for (int a = 0; a < d; ++a) S *= 3;
  if (n * S >= ((int64_t)1 << 31)) return NULL;
  for (int64_t i = 0; i < n * d; ++i)
    if (!(X[i] >= 0.0 && X[i] < 1.0)) return NULL;
  /* every image with k in {-1,0,1}^d, row i S + c(k) */
  double *Xi = (double *)malloc(sizeof(double) * (size_t)(n * S * d));
  vgo_mesh *M = (vgo_mesh *)calloc(1, sizeof(vgo_mesh));
  tmap G, V;
  memset(&G, 0, sizeof G);
  memset(&V, 0, sizeof V);
  if (!Xi || !M) goto fail;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t c = 0; c < S; ++c) {
      int64_t r = c;
      for (int a = 0; a < d; ++a) {
        Xi[(i * S + c) * d + a] = X[i * d + a] + (double)(r % 3 - 1);
        r /= 3;
      }
    }
  M->d = d;
  if (tmap_init(&G, d, 1 << 12) || tmap_init(&V, d + 1, 1 << 12)) goto fail;
  {
    int32_t s0[64], key[64], eta[64];
    double v[64], u[64];
    int cr;
    const int32_t centre = (int32_t)((S - 1) / 2); /* c(0) */
    *status = -4;
    if (descent(d, n * S, Xi, centre, draws, n_draws, 0, s0, v, M)) goto fail;
    *status = -2;
    if (!ball_inside(d, Xi, s0, v)) goto fail;
    *status = -3;
    if (periodic_canon(d, d + 1, s0)) goto fail;
    *status = -4;
    if (circumcentre(d, Xi, s0, v)) goto fail;
    *status = -1;
    if (mesh_push_vertex(M, s0, v)) goto fail;
    *tmap_slot(&V, s0, 1, &cr) = 0;
    for (int o = 0; o <= d; ++o) {
      int a = 0;
      for (int b = 0; b <= d; ++b)
        if (b != o) eta[a++] = s0[b];
      *status = -3;
      if (periodic_canon(d, d, eta)) goto fail;
      *tmap_slot(&G, eta, 1, &cr) += 1;
    }
    for (int64_t head = 0; head < M->nv; ++head) {
      int32_t sig[64];
      double r[64];
      memcpy(sig, M->sig + head * (d + 1), sizeof(int32_t) * (d + 1));
      memcpy(r, M->coord + head * d, sizeof(double) * d);
      for (int o = 0; o <= d; ++o) {
        int a = 0;
        for (int b = 0; b <= d; ++b)
          if (b != o) eta[a++] = sig[b];
        int32_t ec[64];
        memcpy(ec, eta, sizeof(int32_t) * d);
        *status = -3;
        if (periodic_canon(d, d, ec)) goto fail;
        int64_t *gc = tmap_slot(&G, ec, 0, &cr);
        if (gc && *gc >= 2) continue;
        if (search_direction(d, Xi, eta, sig[o], u)) continue;
        double t, t2;
        int32_t j;
        M->raycasts++;
        raycast_one(d, n * S, Xi, r, u, eta[0], eta, d, 0, &t, &j, &t2);
        *status = -2;
        if (j < 0) goto fail;
        for (int b = 0; b < d; ++b) key[b] = eta[b];
        key[d] = j;
        sort_small(key, d + 1);
        /* the ball of the new vertex, in the frame of its ray */
        *status = -4;
        if (circumcentre(d, Xi, key, v)) goto fail;
        *status = -2;
        if (!ball_inside(d, Xi, key, v)) goto fail;
        *status = -3;
        if (periodic_canon(d, d + 1, key)) goto fail;
        int64_t *vs = tmap_slot(&V, key, 1, &cr);
        *status = -1;
        if (!vs) goto fail;
        if (!cr) {
          M->duplicates++;
          continue;
        }
        *vs = M->nv;
        *status = -4;
        if (circumcentre(d, Xi, key, v)) goto fail;
        *status = -1;
        if (mesh_push_vertex(M, key, v)) goto fail;
        for (int o2 = 0; o2 <= d; ++o2) {
          int a2 = 0;
          int32_t e2[64];
          for (int b = 0; b <= d; ++b)
            if (b != o2) e2[a2++] = key[b];
          *status = -3;
          if (periodic_canon(d, d, e2)) goto fail;
          int64_t *g2 = tmap_slot(&G, e2, 1, &cr);
          *status = -1;
          if (!g2) goto fail;
          *g2 += 1;
        }
      }
    }
  }
  *status = 0;
  tmap_free(&G);
  tmap_free(&V);
  free(Xi);
  return M;
fail:
  tmap_free(&G);
  tmap_free(&V);
  free(Xi);
  if (M) {
    free(M->sig);
    free(M->coord);
    free(M);
  }
  return NULL;
}

/* The star of generator i: every vertex of the unbounded diagram whose
 * generators include i, found by Algorithm 2 restricted to the edges that
 * keep i (a Descent from sigma = {i}, r = x_i starts it).  Its vertices'
 * other generators are the Voronoi neighbours of i.  Returns the number of
 * vertices written to sig_out ([cap][d+1], sorted tuples), or -1. */
int64_t vgo_star(int d, int64_t n, const double *X, int32_t i, const double *draws,
                 int n_draws, int32_t *sig_out, int64_t cap) {
  if (d < 1 || d > 63 || n < d + 1) return -1;
  /* Descent from sigma = {i}, r = x_i (the steps of Algorithm 2's Descent) */
  vgo_mesh tmp;
  memset(&tmp, 0, sizeof tmp);
  tmp.d = d;
  int32_t sigma[64];
  double r[64], u[64], v[64];
  int m = 1, used = 0;
  sigma[0] = i;
  for (int k = 0; k < d; ++k) r[k] = X[(int64_t)i * d + k];
  while (m < d + 1) {
    if (used >= n_draws) return -1;
    for (int k = 0; k < d; ++k) u[k] = draws[used * d + k];
    used++;
    project_out_span(d, X, sigma, m, u);
    double nr = sqrt(dot(u, u, d));
    if (!(nr > 0.0)) continue;
    for (int k = 0; k < d; ++k) u[k] /= nr;
    double t;
    int32_t j = cast(d, n, X, sigma, m, r, u, 0, &t, &tmp);
    if (j < 0) {
      for (int k = 0; k < d; ++k) u[k] = -u[k];
      j = cast(d, n, X, sigma, m, r, u, 0, &t, &tmp);
    }
    if (j < 0) continue;
    for (int k = 0; k < d; ++k) r[k] += t * u[k];
    sigma[m++] = j;
  }
  sort_small(sigma, d + 1);
  if (circumcentre(d, X, sigma, v)) return -1;
  tmap V;
  if (tmap_init(&V, d + 1, 1 << 10)) return -1;
  int cr;
  int64_t nv = 0;
  double *coord = (double *)malloc(sizeof(double) * (size_t)(cap * d));
  if (!coord || cap < 1) {
    free(coord);
    tmap_free(&V);
    return -1;
  }
  memcpy(sig_out, sigma, sizeof(int32_t) * (d + 1));
  memcpy(coord, v, sizeof(double) * d);
  *tmap_slot(&V, sigma, 1, &cr) = 0;
  nv = 1;
  for (int64_t head = 0; head < nv; ++head) {
    int32_t sig[64], eta[64], key[64];
    memcpy(sig, sig_out + head * (d + 1), sizeof(int32_t) * (d + 1));
    memcpy(r, coord + head * d, sizeof(double) * d);
    for (int o = 0; o <= d; ++o) {
      if (sig[o] == i) continue; /* keep i in the edge */
      int a = 0;
      for (int b = 0; b <= d; ++b)
        if (b != o) eta[a++] = sig[b];
      if (search_direction(d, X, eta, sig[o], u)) continue;
      double t;
      int32_t j = cast(d, n, X, eta, d, r, u, 0, &t, &tmp);
      if (j < 0) continue;
      for (int b = 0; b < d; ++b) key[b] = eta[b];
      key[d] = j;
      sort_small(key, d + 1);
      int64_t *vs = tmap_slot(&V, key, 1, &cr);
      if (!vs || !cr) continue;
      if (nv >= cap) {
        nv = -1;
        break;
      }
      *vs = nv;
      memcpy(sig_out + nv * (d + 1), key, sizeof(int32_t) * (d + 1));
      if (circumcentre(d, X, key, coord + nv * d)) {
        nv = -1;
        break;
      }
      nv++;
    }
    if (nv < 0) break;
  }
  free(coord);
  tmap_free(&V);
  return nv;
}

int64_t vgo_mesh_nv(const void *h) { return ((const vgo_mesh *)h)->nv; }
int64_t vgo_mesh_nb(const void *h) { return ((const vgo_mesh *)h)->nb; }
int64_t vgo_mesh_raycasts(const void *h) { return ((const vgo_mesh *)h)->raycasts; }
int64_t vgo_mesh_nn_calls(const void *h) { return ((const vgo_mesh *)h)->nn_calls; }
int64_t vgo_mesh_duplicates(const void *h) { return ((const vgo_mesh *)h)->duplicates; }

void vgo_mesh_copy(const void *h, int32_t *sig, double *coord, int32_t *bsig,
                   int32_t *bomit) {
  const vgo_mesh *M = (const vgo_mesh *)h;
  int d = M->d;
  if (sig) memcpy(sig, M->sig, sizeof(int32_t) * (size_t)(M->nv * (d + 1)));
  if (coord) memcpy(coord, M->coord, sizeof(double) * (size_t)(M->nv * d));
  if (bsig && M->nb) memcpy(bsig, M->bsig, sizeof(int32_t) * (size_t)(M->nb * (d + 1)));
  if (bomit && M->nb) memcpy(bomit, M->bomit, sizeof(int32_t) * (size_t)M->nb);
}

void vgo_mesh_free(void *h) {
  vgo_mesh *M = (vgo_mesh *)h;
  if (!M) return;
  free(M->sig);
  free(M->coord);
  free(M->bsig);
  free(M->bomit);
  free(M);
}

/* Exposed for the tests: the FP64 vertex solve and search direction. */
int vgo_circumcentre(int d, const double *X, const int32_t *sigma, double *v) {
  return circumcentre(d, X, sigma, v);
}

int vgo_search_direction(int d, const double *X, const int32_t *eta,
                         int32_t omit, double *u) {
  return search_direction(d, X, eta, omit, u);
}

/* ------------------------------------------------------------------------ */
/* Monte-Carlo terms of Sec. 3.1 / Algorithm 3.                              */
/*                                                                           */
/* For a ray of cell i with direction u, result l = t* and neighbour j:      */
/*   volume term  l^d                       (V = S_{d-1}/(d n) sum l^d)      */
/*   area term    l^{d-1} / |n_ij . u|      (eq. dS-dA; A_ij = S/n sum)     */
/*   energy term  l^{d+2}                   (int_0^l rho^2 rho^{d-1} d rho   */
/*                                           = l^{d+2}/(d+2): the second     */
/*                                           moment of the cell about x_i)  */
/* with n_ij = (x_j - x_i)/|x_j - x_i| for a node and n = e_k for the cube   */
/* face x_k = s.  Algorithm 3 divides by <n,u> without absolute value and    */
/* with n = (x_i - x_j)/|..|, which is negative; the absolute value of       */
/* eq. dS-dA is used.                                                        */
/* ------------------------------------------------------------------------ */
int vgo_mc_ray_weights(int d, int64_t n, const double *X, int64_t n_cells,
                       const int64_t *cells, int n_rays, const double *dirs,
                       const double *t, const int32_t *idx, double *w_vol,
                       double *w_area, double *w_energy) {
  int64_t m = n_cells * (int64_t)n_rays;
  for (int64_t k = 0; k < m; ++k) {
    int64_t i = cells[k / n_rays];
    const double *xi = X + i * d, *u = dirs + k * d;
    double l = t[k];
    double ld1 = 1.0;
    for (int a = 0; a < d - 1; ++a) ld1 *= l;
    double nu;
    int32_t j = idx[k];
    if (j >= 0) {
      const double *xj = X + (int64_t)j * d;
      double nr = sqrt(dist2(xj, xi, d));
      double c = 0.0;
      for (int a = 0; a < d; ++a) c += (xj[a] - xi[a]) / nr * u[a];
      nu = fabs(c);
    } else if (j <= -2) {
      int face = -2 - j;
      nu = fabs(u[face / 2]);
    } else {
      return -1;
    }
    w_vol[k] = ld1 * l;
    w_area[k] = ld1 / nu;
    w_energy[k] = ld1 * l * l * l;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* O4: derivative of the Monte-Carlo estimators with the directions frozen.  */
/*                                                                           */
/* For a node winner j, with D = x_j - x_i and delta = u.D > 0, eq. (t) at   */
/* x = g = x_i reads t = |D|^2 / (2 delta), so                               */
/*   dt/dD = (D - t u)/delta,  dt/dx_j = dt/dD,  dt/dx_i = -dt/dD.           */
/* For a cube face x_k = s: t = (s - x_ik)/u_k, so dt/dx_ik = -1/u_k.        */
/* The area term l^{d-1}/|n.u| with n.u = delta/|D| also depends on D        */
/* directly: d(|D|/delta)/dD = D/(|D| delta) - |D| u/delta^2.                */
/* Upstream weights gv[i], ge[i] multiply the scaled volume and energy of    */
/* cell i; ga[k] multiplies the scaled area term of ray k (the caller maps   */
/* the gradient of each facet area onto its rays).  grad is [n][d], added    */
/* to (not cleared).  Scales: volume S/(d n_rays), energy S/((d+2) n_rays),  */
/* area S/n_rays, with S = S_{d-1} passed in.                                */
/* ------------------------------------------------------------------------ */
int vgo_mc_adjoint(int d, int64_t n, const double *X, int64_t n_cells,
                   const int64_t *cells, int n_rays, const double *dirs,
                   const double *t, const int32_t *idx, double S,
                   const double *gv, const double *ge, const double *ga,
                   double *grad) {
  double cv = S / ((double)d * n_rays), ce = S / ((double)(d + 2) * n_rays),
         ca = S / (double)n_rays;
  int64_t m = n_cells * (int64_t)n_rays;
  for (int64_t k = 0; k < m; ++k) {
    int64_t c = k / n_rays;
    int64_t i = cells[c];
    const double *xi = X + i * d, *u = dirs + k * d;
    double l = t[k];
    int32_t j = idx[k];
    double ld2 = 1.0; /* l^{d-2} */
    for (int a = 0; a < d - 2; ++a) ld2 *= l;
    double ld1 = (d >= 2) ? ld2 * l : 1.0;
    if (d < 2) ld2 = 0.0;
    double dl = 0.0; /* d(loss)/dl for this ray */
    if (gv) dl += gv[c] * cv * (double)d * ld1;
    if (ge) dl += ge[c] * ce * (double)(d + 2) * ld1 * l * l;
    if (j >= 0) {
      const double *xj = X + (int64_t)j * d;
      double D[64], delta = 0.0, nD2 = 0.0;
      for (int a = 0; a < d; ++a) {
        D[a] = xj[a] - xi[a];
        delta += u[a] * D[a];
        nD2 += D[a] * D[a];
      }
      double nD = sqrt(nD2);
      double ratio = nD / delta; /* 1/|n.u| */
      double dA_dl = 0.0;
      double gD[64];
      for (int a = 0; a < d; ++a) gD[a] = 0.0;
      if (ga) {
        dA_dl = ga[k] * ca * (double)(d - 1) * ld2 * ratio;
        for (int a = 0; a < d; ++a)
          gD[a] += ga[k] * ca * ld1 *
                   (D[a] / (nD * delta) - nD * u[a] / (delta * delta));
      }
      double tot = dl + dA_dl;
      for (int a = 0; a < d; ++a) {
        double dtdD = (D[a] - l * u[a]) / delta;
        gD[a] += tot * dtdD;
      }
      for (int a = 0; a < d; ++a) {
        grad[(int64_t)j * d + a] += gD[a];
        grad[i * d + a] -= gD[a];
      }
    } else if (j <= -2) {
      int face = -2 - j, kk = face / 2;
      double tot = dl;
      if (ga) tot += ga[k] * ca * (double)(d - 1) * ld2 / fabs(u[kk]);
      grad[i * d + kk] += tot * (-1.0 / u[kk]);
    } else {
      return -1;
    }
  }
  return 0;
}

/* Threads of the OpenMP loops that follow (timing aid; results do not
 * depend on it). */
void vgo_set_threads(int k) {
#ifdef _OPENMP
  if (k > 0) omp_set_num_threads(k);
#else
  (void)k;
#endif
}

int vgo_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
