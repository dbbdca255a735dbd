/*
 * FP64 CPU oracle for the continuous Fourier series (CFS) of rectilinear
 * polygons.  TEST INFRASTRUCTURE ONLY: it is called by the tests, by the
 * package's smoke check and by the benchmark's CPU-baseline leg, never by the
 * product path.  It shares no code, header, table or constant with the HIP
 * library and includes nothing from it.
 *
 * What it computes (Scheibler, Hurley, Chebira, "Fast Continuous Haar and
 * Fourier Transforms of Rectilinear Polygons from VLSI Layouts"):
 *
 *   F[k,l] = <f, phi_{k,l}>,  phi_{k,l}(x,y) = T^{-1} e^{j 2 pi (k x + l y)/T}
 *   (Sec. II-C, Fourier basis over the tile, with Nx = Ny = T; inner product
 *   of Sec. III-A), for f = sum of the indicators of the polygons (Sec. III-A,
 *   signal model).
 *
 * It evaluates the closed forms of Prop. 3 (Sec. III-C1) directly, in the
 * paper's EDGE form: one sum over the horizontal edges (a -> b at height y)
 * for F[0,0], F[0,l] and F[k,l], and one over the vertical edges
 * (a -> b at abscissa x) for F[k,0], with the scale factors alpha_{k,l} of
 * Prop. 3 for a square tile:
 *
 *   F[0,0] = (1/T)               * sum_h  y (x_b - x_a)
 *   F[k,0] = (j/(2 pi k))        * sum_v  (y_a - y_b) e^{-j 2 pi k x / T}
 *   F[0,l] = (j/(2 pi l))        * sum_h  (x_b - x_a) e^{-j 2 pi l y / T}
 *   F[k,l] = (-T/(4 pi^2 k l))   * sum_h  e^{-j 2 pi l y/T}
 *                                    (e^{-j 2 pi k x_b/T} - e^{-j 2 pi k x_a/T})
 *
 * Several polygons add up (Sec. III-A, linearity; Sec. III-C1, multiple
 * polygons).  The paper orders vertices clockwise (Sec. II-A2); a loop given
 * counter-clockwise has a negative edge-form area and is counted with the
 * opposite sign, which is the same as reversing it.
 *
 * Two coordinate modes:
 *   lattice = 1: coordinates are integers; the phase index (k x) mod T is
 *                reduced exactly in int64 before cos/sin of 2 pi r / T.
 *   lattice = 0: real coordinates; angle 2 pi fmod(k x, T) / T.  Used for
 *                finite differences of the gradient.
 *
 * The gradient routine differentiates the same four closed forms with respect
 * to a shift of one edge (both of its endpoints move: a vertical edge along
 * +x, a horizontal edge along +y) and contracts with a complex cotangent G,
 * using dLoss/dtheta = Re sum conj(G[k,l]) dF[k,l]/dtheta, where
 * G = dLoss/dRe F + j dLoss/dIm F.
 *
 * Everything is FP64; loops over edges are plain, in input order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define FO_OK 0
#define FO_ERR_ARG -1
#define FO_ERR_NOT_RECTILINEAR -2
#define FO_ERR_RANGE -3
#define FO_ERR_NOMEM -7

static const double FO_PI = 3.14159265358979323846264338327950288;

typedef struct {
  double re, im;
} fo_c;

/* One edge of a loop: from vertex a to vertex b (input order), with the
 * loop's orientation sign (+1 clockwise, -1 counter-clockwise). */
typedef struct {
  double xa, ya, xb, yb;
  double sigma;
  int horizontal;
} fo_edge;

static int set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
  int used = 1;
#pragma omp parallel
  {
#pragma omp single
    used = omp_get_num_threads();
  }
  return used;
#else
  (void)nthreads;
  return 1;
#endif
}

int fo_threads(int nthreads) { return set_threads(nthreads); }

/* Check the loops: each has an even number (>= 4) of vertices, every edge is
 * horizontal or vertical with nonzero length, and edges alternate.  Fills the
 * edge list (edge e joins input vertex e to the next vertex of its loop) and
 * the orientation sign of every loop from its edge-form area. */
static int build_edges(const double *xy, const int64_t *off, int64_t n_loops,
                       int lattice, fo_edge **edges_out, int64_t *n_edges_out) {
  if (!xy || !off || n_loops < 0) return FO_ERR_ARG;
  if (off[0] != 0) return FO_ERR_ARG;
  int64_t n = off[n_loops];
  fo_edge *E = (fo_edge *)malloc(sizeof(fo_edge) * (size_t)(n > 0 ? n : 1));
  if (!E) return FO_ERR_NOMEM;
  for (int64_t m = 0; m < n_loops; ++m) {
    int64_t b0 = off[m], cnt = off[m + 1] - off[m];
    if (cnt < 4 || (cnt & 1)) { free(E); return FO_ERR_NOT_RECTILINEAR; }
    double area = 0.0;
    for (int64_t i = 0; i < cnt; ++i) {
      int64_t a = b0 + i, b = b0 + (i + 1) % cnt;
      double xa = xy[2 * a], ya = xy[2 * a + 1], xb = xy[2 * b], yb = xy[2 * b + 1];
      if (lattice) {
        if (xa != floor(xa) || ya != floor(ya) || fabs(xa) > 1073741823.0 ||
            fabs(ya) > 1073741823.0) { free(E); return FO_ERR_RANGE; }
      }
      int h = (ya == yb) && (xa != xb);
      int v = (xa == xb) && (ya != yb);
      if (!h && !v) { free(E); return FO_ERR_NOT_RECTILINEAR; }
      E[a].xa = xa; E[a].ya = ya; E[a].xb = xb; E[a].yb = yb;
      E[a].horizontal = h;
      if (h) area += ya * (xb - xa);
    }
    for (int64_t i = 0; i < cnt; ++i) {
      int64_t a = b0 + i, b = b0 + (i + 1) % cnt;
      if (E[a].horizontal == E[b].horizontal) { free(E); return FO_ERR_NOT_RECTILINEAR; }
    }
    if (area == 0.0) { free(E); return FO_ERR_NOT_RECTILINEAR; }
    double sg = area > 0 ? 1.0 : -1.0;
    for (int64_t i = 0; i < cnt; ++i) E[b0 + i].sigma = sg;
  }
  *edges_out = E;
  *n_edges_out = n;
  return FO_OK;
}

/* Evaluation context: tile period, coordinate mode and, in lattice mode, the
 * values e^{-j 2 pi r / T} for r = 0..T-1, computed once per call with
 * cos/sin of 2 pi r / T.  Looking r up returns exactly what calling cos/sin
 * at that point would. */
typedef struct {
  int64_t T;
  int lattice;
  fo_c *tab;
} fo_ctx;

static int ctx_init(fo_ctx *c, int64_t T, int lattice) {
  c->T = T;
  c->lattice = lattice;
  c->tab = NULL;
  if (!lattice) return FO_OK;
  c->tab = (fo_c *)malloc(sizeof(fo_c) * (size_t)T);
  if (!c->tab) return FO_ERR_NOMEM;
  for (int64_t r = 0; r < T; ++r) {
    double ang = 2.0 * FO_PI * (double)r / (double)T;
    c->tab[r].re = cos(ang);
    c->tab[r].im = -sin(ang);
  }
  return FO_OK;
}

static void ctx_free(fo_ctx *c) { free(c->tab); c->tab = NULL; }

/* e^{-j 2 pi k t / T} for one coordinate t.  Lattice mode: exact integer
 * reduction of k t modulo T, then the value at 2 pi r / T. */
static fo_c expo(const fo_ctx *c, int64_t k, double t) {
  if (c->lattice) {
    int64_t r = ((k * (int64_t)t) % c->T + c->T) % c->T;
    return c->tab[r];
  }
  double ang = 2.0 * FO_PI * fmod((double)k * t, (double)c->T) / (double)c->T;
  fo_c e = {cos(ang), -sin(ang)};
  return e;
}

static inline fo_c cmul(fo_c a, fo_c b) {
  fo_c r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
  return r;
}

/* One coefficient F[k,l] from the edge list (Prop. 3 with alpha_{k,l}). */
static fo_c coef(const fo_ctx *c, const fo_edge *E, int64_t n, int64_t k, int64_t l) {
  const int64_t T = c->T;
  fo_c acc = {0.0, 0.0};
  if (k == 0 && l == 0) {
    /* F[0,0] = alpha_00 * sum_h y (x_b - x_a): the signed area over T. */
    for (int64_t e = 0; e < n; ++e)
      if (E[e].horizontal) acc.re += E[e].sigma * E[e].ya * (E[e].xb - E[e].xa);
    acc.re /= (double)T;
    return acc;
  }
  if (l == 0) {
    /* F[k,0] = j/(2 pi k) * sum over vertical edges (y_a - y_b) e^{-j w k x}. */
    for (int64_t e = 0; e < n; ++e) {
      if (E[e].horizontal) continue;
      fo_c w = expo(c, k, E[e].xa);
      double len = E[e].sigma * (E[e].ya - E[e].yb);
      acc.re += len * w.re;
      acc.im += len * w.im;
    }
    double sc = 1.0 / (2.0 * FO_PI * (double)k);
    fo_c r = {-acc.im * sc, acc.re * sc}; /* multiply by j*sc */
    return r;
  }
  if (k == 0) {
    /* F[0,l] = j/(2 pi l) * sum over horizontal edges (x_b - x_a) e^{-j w l y}. */
    for (int64_t e = 0; e < n; ++e) {
      if (!E[e].horizontal) continue;
      fo_c w = expo(c, l, E[e].ya);
      double len = E[e].sigma * (E[e].xb - E[e].xa);
      acc.re += len * w.re;
      acc.im += len * w.im;
    }
    double sc = 1.0 / (2.0 * FO_PI * (double)l);
    fo_c r = {-acc.im * sc, acc.re * sc};
    return r;
  }
  /* F[k,l] = -T/(4 pi^2 k l) * sum_h e^{-j w l y} (e^{-j w k x_b} - e^{-j w k x_a}). */
  for (int64_t e = 0; e < n; ++e) {
    if (!E[e].horizontal) continue;
    fo_c wy = expo(c, l, E[e].ya);
    fo_c wb = expo(c, k, E[e].xb);
    fo_c wa = expo(c, k, E[e].xa);
    fo_c d = {wb.re - wa.re, wb.im - wa.im};
    fo_c t = cmul(wy, d);
    acc.re += E[e].sigma * t.re;
    acc.im += E[e].sigma * t.im;
  }
  double a = -(double)T / (4.0 * FO_PI * FO_PI * (double)k * (double)l);
  acc.re *= a;
  acc.im *= a;
  return acc;
}

/* Full centred grid |k| <= K, |l| <= L, k-major: F[(k+K)(2L+1) + (l+L)],
 * interleaved (re, im).  area_out (optional) receives the exact signed area
 * in lattice mode (sum over loops of |area|). */
int fo_cfs_grid(const double *xy, const int64_t *off, int64_t n_loops, int64_t T, int32_t K,
                int32_t L, int lattice, int nthreads, double *F, int64_t *area_out) {
  if (T < 1 || K < 0 || L < 0 || !F) return FO_ERR_ARG;
  fo_edge *E = NULL;
  int64_t n = 0;
  int st = build_edges(xy, off, n_loops, lattice, &E, &n);
  if (st) return st;
  fo_ctx ctx;
  if (ctx_init(&ctx, T, lattice)) { free(E); return FO_ERR_NOMEM; }
  set_threads(nthreads);
  const int64_t W = 2 * (int64_t)L + 1;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t k = -K; k <= K; ++k) {
    for (int64_t l = -L; l <= L; ++l) {
      fo_c v = coef(&ctx, E, n, k, l);
      int64_t idx = (k + K) * W + (l + L);
      F[2 * idx] = v.re;
      F[2 * idx + 1] = v.im;
    }
  }
  if (area_out) {
    int64_t A = 0;
    if (lattice)
      for (int64_t e = 0; e < n; ++e)
        if (E[e].horizontal)
          A += (int64_t)E[e].sigma * (int64_t)E[e].ya * ((int64_t)E[e].xb - (int64_t)E[e].xa);
    *area_out = A;
  }
  ctx_free(&ctx);
  free(E);
  return FO_OK;
}

/* ---------------------------------------------------------------------------
 * General tile: periods Nx along x and Ny along y (any positive integers, Sec.
 * II-C), vertices on the grid of step 2^-F (F = frac_bits >= 0; F = 0 is the
 * integer lattice of Sec. II-A2).  Prop. 3 with its general factors:
 *
 *   alpha_00 = 1 / sqrt(Nx Ny),              alpha_k0 = j/(2 pi k) sqrt(Nx/Ny),
 *   alpha_0l = j/(2 pi l) sqrt(Ny/Nx),       alpha_kl = -sqrt(Nx Ny) / (4 pi^2 k l),
 *
 * and phases w_x k x = 2 pi k x / Nx reduced exactly: with X = x 2^F (an
 * integer) and Mx = Nx 2^F, k x / Nx = (k X mod Mx) / Mx + an integer.
 * --------------------------------------------------------------------------- */
typedef struct {
  int64_t M;
  fo_c *tab; /* e^{-j 2 pi r / M}, r = 0..M-1 */
} fo_period;

static int period_init(fo_period *p, int64_t M) {
  p->M = M;
  p->tab = (fo_c *)malloc(sizeof(fo_c) * (size_t)M);
  if (!p->tab) return FO_ERR_NOMEM;
  for (int64_t r = 0; r < M; ++r) {
    double ang = 2.0 * FO_PI * (double)r / (double)M;
    p->tab[r].re = cos(ang);
    p->tab[r].im = -sin(ang);
  }
  return FO_OK;
}

/* e^{-j 2 pi k X / M} for an integer X (the coordinate times 2^F). */
static fo_c period_expo(const fo_period *p, int64_t k, int64_t X) {
  int64_t xr = ((X % p->M) + p->M) % p->M;
  int64_t r = ((k % p->M) * xr) % p->M;
  if (r < 0) r += p->M;
  return p->tab[r];
}

static fo_c coef_general(const fo_period *px, const fo_period *py, double Nx, double Ny,
                         double scale, const fo_edge *E, int64_t n, int64_t k, int64_t l) {
  fo_c acc = {0.0, 0.0};
  if (k == 0 && l == 0) {
    for (int64_t e = 0; e < n; ++e)
      if (E[e].horizontal) acc.re += E[e].sigma * E[e].ya * (E[e].xb - E[e].xa);
    acc.re /= sqrt(Nx * Ny);
    return acc;
  }
  if (l == 0) {
    for (int64_t e = 0; e < n; ++e) {
      if (E[e].horizontal) continue;
      fo_c w = period_expo(px, k, (int64_t)llround(E[e].xa * scale));
      double len = E[e].sigma * (E[e].ya - E[e].yb);
      acc.re += len * w.re;
      acc.im += len * w.im;
    }
    double sc = sqrt(Nx / Ny) / (2.0 * FO_PI * (double)k);
    fo_c r = {-acc.im * sc, acc.re * sc};
    return r;
  }
  if (k == 0) {
    for (int64_t e = 0; e < n; ++e) {
      if (!E[e].horizontal) continue;
      fo_c w = period_expo(py, l, (int64_t)llround(E[e].ya * scale));
      double len = E[e].sigma * (E[e].xb - E[e].xa);
      acc.re += len * w.re;
      acc.im += len * w.im;
    }
    double sc = sqrt(Ny / Nx) / (2.0 * FO_PI * (double)l);
    fo_c r = {-acc.im * sc, acc.re * sc};
    return r;
  }
  for (int64_t e = 0; e < n; ++e) {
    if (!E[e].horizontal) continue;
    fo_c wy = period_expo(py, l, (int64_t)llround(E[e].ya * scale));
    fo_c wb = period_expo(px, k, (int64_t)llround(E[e].xb * scale));
    fo_c wa = period_expo(px, k, (int64_t)llround(E[e].xa * scale));
    fo_c d = {wb.re - wa.re, wb.im - wa.im};
    fo_c t = cmul(wy, d);
    acc.re += E[e].sigma * t.re;
    acc.im += E[e].sigma * t.im;
  }
  double a = -sqrt(Nx * Ny) / (4.0 * FO_PI * FO_PI * (double)k * (double)l);
  acc.re *= a;
  acc.im *= a;
  return acc;
}

/* Full centred grid for the general tile; layout as fo_cfs_grid.  xy holds the
 * true coordinates (multiples of 2^-F).  area_out: sum over loops of the
 * signed area times 4^F (an integer). */
int fo_cfs_grid_general(const double *xy, const int64_t *off, int64_t n_loops, int64_t Nx,
                        int64_t Ny, int32_t frac_bits, int32_t K, int32_t L, int nthreads,
                        double *F, int64_t *area_out) {
  if (Nx < 1 || Ny < 1 || frac_bits < 0 || frac_bits > 20 || K < 0 || L < 0 || !F)
    return FO_ERR_ARG;
  const double scale = ldexp(1.0, frac_bits);
  const int64_t nv = off[n_loops];
  for (int64_t i = 0; i < 2 * nv; ++i) {
    double X = xy[i] * scale;
    if (X != floor(X) || fabs(X) > 1073741823.0) return FO_ERR_RANGE;
  }
  fo_edge *E = NULL;
  int64_t n = 0;
  int st = build_edges(xy, off, n_loops, 0, &E, &n);
  if (st) return st;
  fo_period px, py;
  if (period_init(&px, Nx << frac_bits)) { free(E); return FO_ERR_NOMEM; }
  if (period_init(&py, Ny << frac_bits)) { free(px.tab); free(E); return FO_ERR_NOMEM; }
  set_threads(nthreads);
  const int64_t W = 2 * (int64_t)L + 1;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t k = -K; k <= K; ++k)
    for (int64_t l = -L; l <= L; ++l) {
      fo_c v = coef_general(&px, &py, (double)Nx, (double)Ny, scale, E, n, k, l);
      int64_t idx = (k + K) * W + (l + L);
      F[2 * idx] = v.re;
      F[2 * idx + 1] = v.im;
    }
  if (area_out) {
    int64_t A = 0;
    for (int64_t e = 0; e < n; ++e)
      if (E[e].horizontal)
        A += (int64_t)E[e].sigma * llround(E[e].ya * scale) *
             (llround(E[e].xb * scale) - llround(E[e].xa * scale));
    *area_out = A;
  }
  free(px.tab);
  free(py.tab);
  free(E);
  return FO_OK;
}

/* Single coefficients (k[i], l[i]) of a general tile; out interleaved. */
int fo_cfs_points_general(const double *xy, const int64_t *off, int64_t n_loops, int64_t Nx,
                          int64_t Ny, int32_t frac_bits, int64_t npts, const int32_t *kk,
                          const int32_t *ll, int nthreads, double *F) {
  if (Nx < 1 || Ny < 1 || frac_bits < 0 || frac_bits > 20 || npts < 0 || !F ||
      (npts > 0 && (!kk || !ll)))
    return FO_ERR_ARG;
  const double scale = ldexp(1.0, frac_bits);
  const int64_t nv = off[n_loops];
  for (int64_t i = 0; i < 2 * nv; ++i) {
    double X = xy[i] * scale;
    if (X != floor(X) || fabs(X) > 1073741823.0) return FO_ERR_RANGE;
  }
  fo_edge *E = NULL;
  int64_t n = 0;
  int st = build_edges(xy, off, n_loops, 0, &E, &n);
  if (st) return st;
  fo_period px, py;
  if (period_init(&px, Nx << frac_bits)) { free(E); return FO_ERR_NOMEM; }
  if (period_init(&py, Ny << frac_bits)) { free(px.tab); free(E); return FO_ERR_NOMEM; }
  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < npts; ++i) {
    fo_c v = coef_general(&px, &py, (double)Nx, (double)Ny, scale, E, n, kk[i], ll[i]);
    F[2 * i] = v.re;
    F[2 * i + 1] = v.im;
  }
  free(px.tab);
  free(py.tab);
  free(E);
  return FO_OK;
}

/* A list of single coefficients (k[i], l[i]); out interleaved (re, im). */
int fo_cfs_points(const double *xy, const int64_t *off, int64_t n_loops, int64_t T, int lattice,
                  int64_t npts, const int32_t *kk, const int32_t *ll, int nthreads, double *F) {
  if (T < 1 || npts < 0 || !F || (npts > 0 && (!kk || !ll))) return FO_ERR_ARG;
  fo_edge *E = NULL;
  int64_t n = 0;
  int st = build_edges(xy, off, n_loops, lattice, &E, &n);
  if (st) return st;
  fo_ctx ctx;
  if (ctx_init(&ctx, T, lattice)) { free(E); return FO_ERR_NOMEM; }
  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < npts; ++i) {
    fo_c v = coef(&ctx, E, n, kk[i], ll[i]);
    F[2 * i] = v.re;
    F[2 * i + 1] = v.im;
  }
  ctx_free(&ctx);
  free(E);
  return FO_OK;
}

/* Derivative of F[k,l] with respect to a shift of edge e (both endpoints).
 * A vertical edge a -> b at abscissa X moves along +x; it changes the two
 * horizontal edges that end at a and start at b, and its own position in the
 * F[k,0] sum.  A horizontal edge a -> b at height Y moves along +y; it
 * changes its own terms and the lengths of the two vertical edges that end at
 * a and start at b.  Derived by differentiating the four closed forms of
 * Prop. 3 term by term. */
static fo_c dcoef(const fo_ctx *c, const fo_edge *e, int64_t k, int64_t l) {
  const int64_t T = c->T;
  const double w = 2.0 * FO_PI / (double)T;
  fo_c r = {0.0, 0.0};
  double sg = e->sigma;
  if (!e->horizontal) {
    double X = e->xa, ya = e->ya, yb = e->yb;
    if (k == 0 && l == 0) {
      r.re = sg * (ya - yb) / (double)T;
    } else if (l == 0) {
      /* j/(2 pi k) (y_a - y_b)(-j w k) e(kX) = (y_a - y_b) e(kX) / T */
      fo_c ex = expo(c, k, X);
      double s = sg * (ya - yb) / (double)T;
      r.re = s * ex.re;
      r.im = s * ex.im;
    } else if (k == 0) {
      /* j/(2 pi l) (e(l y_a) - e(l y_b)) */
      fo_c ea = expo(c, l, ya), eb = expo(c, l, yb);
      double s = sg / (2.0 * FO_PI * (double)l);
      double dre = ea.re - eb.re, dim = ea.im - eb.im;
      r.re = -dim * s;
      r.im = dre * s;
    } else {
      /* alpha (-j w k) e(kX) (e(l y_a) - e(l y_b)) */
      fo_c ex = expo(c, k, X);
      fo_c ea = expo(c, l, ya), eb = expo(c, l, yb);
      fo_c d = {ea.re - eb.re, ea.im - eb.im};
      fo_c t = cmul(ex, d);
      double a = -(double)T / (4.0 * FO_PI * FO_PI * (double)k * (double)l);
      double m = sg * a * w * (double)k; /* times -j */
      r.re = m * t.im;
      r.im = -m * t.re;
    }
  } else {
    double Y = e->ya, xa = e->xa, xb = e->xb;
    if (k == 0 && l == 0) {
      r.re = sg * (xb - xa) / (double)T;
    } else if (l == 0) {
      /* j/(2 pi k) (e(k x_b) - e(k x_a)) */
      fo_c ea = expo(c, k, xa), eb = expo(c, k, xb);
      double s = sg / (2.0 * FO_PI * (double)k);
      double dre = eb.re - ea.re, dim = eb.im - ea.im;
      r.re = -dim * s;
      r.im = dre * s;
    } else if (k == 0) {
      /* (x_b - x_a) e(lY) / T */
      fo_c ey = expo(c, l, Y);
      double s = sg * (xb - xa) / (double)T;
      r.re = s * ey.re;
      r.im = s * ey.im;
    } else {
      /* alpha (-j w l) e(lY) (e(k x_b) - e(k x_a)) */
      fo_c ey = expo(c, l, Y);
      fo_c ea = expo(c, k, xa), eb = expo(c, k, xb);
      fo_c d = {eb.re - ea.re, eb.im - ea.im};
      fo_c t = cmul(ey, d);
      double a = -(double)T / (4.0 * FO_PI * FO_PI * (double)k * (double)l);
      double m = sg * a * w * (double)l;
      r.re = m * t.im;
      r.im = -m * t.re;
    }
  }
  return r;
}

/* Gradient of a real loss with respect to every edge offset.
 * G: complex cotangent on the centred grid (interleaved re, im, k-major).
 * If edge_idx is NULL all edges are computed (g has off[n_loops] entries);
 * otherwise only the n_sel listed edges (g has n_sel entries). */
int fo_edge_grad(const double *xy, const int64_t *off, int64_t n_loops, int64_t T, int32_t K,
                 int32_t L, int lattice, const double *G, const int64_t *edge_idx, int64_t n_sel,
                 int nthreads, double *g) {
  if (T < 1 || K < 0 || L < 0 || !G || !g) return FO_ERR_ARG;
  fo_edge *E = NULL;
  int64_t n = 0;
  int st = build_edges(xy, off, n_loops, lattice, &E, &n);
  if (st) return st;
  int64_t cnt = edge_idx ? n_sel : n;
  for (int64_t i = 0; i < cnt; ++i)
    if (edge_idx && (edge_idx[i] < 0 || edge_idx[i] >= n)) { free(E); return FO_ERR_ARG; }
  fo_ctx ctx;
  if (ctx_init(&ctx, T, lattice)) { free(E); return FO_ERR_NOMEM; }
  set_threads(nthreads);
  const int64_t W = 2 * (int64_t)L + 1;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < cnt; ++i) {
    const fo_edge *e = &E[edge_idx ? edge_idx[i] : i];
    double acc = 0.0;
    for (int64_t k = -K; k <= K; ++k)
      for (int64_t l = -L; l <= L; ++l) {
        int64_t idx = (k + K) * W + (l + L);
        fo_c d = dcoef(&ctx, e, k, l);
        /* Re(conj(G) d) */
        acc += G[2 * idx] * d.re + G[2 * idx + 1] * d.im;
      }
    g[i] = acc;
  }
  ctx_free(&ctx);
  free(E);
  return FO_OK;
}

/* Derivative of F[k,l] of a general tile (Prop. 3 with its general factors)
 * with respect to the shift of edge e, in true units; the same four closed
 * forms as dcoef, with w_x = 2 pi / Nx, w_y = 2 pi / Ny and the alphas of
 * coef_general. */
static fo_c dcoef_general(const fo_period *px, const fo_period *py, double Nx, double Ny,
                          double scale, const fo_edge *e, int64_t k, int64_t l) {
  fo_c r = {0.0, 0.0};
  const double sg = e->sigma, rn = 1.0 / sqrt(Nx * Ny);
  const double wx = 2.0 * FO_PI / Nx, wy = 2.0 * FO_PI / Ny;
  if (!e->horizontal) {
    const double ya = e->ya, yb = e->yb;
    const int64_t Xg = llround(e->xa * scale);
    if (k == 0 && l == 0) {
      r.re = sg * (ya - yb) * rn;
    } else if (l == 0) {
      /* alpha_k0 (y_a - y_b) (-j w_x k) e(kX) = (y_a - y_b) e(kX) / sqrt(Nx Ny) */
      fo_c ex = period_expo(px, k, Xg);
      r.re = sg * (ya - yb) * rn * ex.re;
      r.im = sg * (ya - yb) * rn * ex.im;
    } else if (k == 0) {
      /* alpha_0l (e(l y_a) - e(l y_b)) */
      fo_c ea = period_expo(py, l, llround(ya * scale)), eb = period_expo(py, l, llround(yb * scale));
      double s = sg * sqrt(Ny / Nx) / (2.0 * FO_PI * (double)l);
      r.re = -(ea.im - eb.im) * s;
      r.im = (ea.re - eb.re) * s;
    } else {
      /* alpha_kl (-j w_x k) e(kX) (e(l y_a) - e(l y_b)) */
      fo_c ex = period_expo(px, k, Xg);
      fo_c ea = period_expo(py, l, llround(ya * scale)), eb = period_expo(py, l, llround(yb * scale));
      fo_c d = {ea.re - eb.re, ea.im - eb.im};
      fo_c t = cmul(ex, d);
      double a = -sqrt(Nx * Ny) / (4.0 * FO_PI * FO_PI * (double)k * (double)l);
      double m = sg * a * wx * (double)k; /* times -j */
      r.re = m * t.im;
      r.im = -m * t.re;
    }
  } else {
    const double xa = e->xa, xb = e->xb;
    const int64_t Yg = llround(e->ya * scale);
    if (k == 0 && l == 0) {
      r.re = sg * (xb - xa) * rn;
    } else if (l == 0) {
      /* alpha_k0 (e(k x_b) - e(k x_a)) */
      fo_c ea = period_expo(px, k, llround(xa * scale)), eb = period_expo(px, k, llround(xb * scale));
      double s = sg * sqrt(Nx / Ny) / (2.0 * FO_PI * (double)k);
      r.re = -(eb.im - ea.im) * s;
      r.im = (eb.re - ea.re) * s;
    } else if (k == 0) {
      /* alpha_0l (x_b - x_a) (-j w_y l) e(lY) = (x_b - x_a) e(lY) / sqrt(Nx Ny) */
      fo_c ey = period_expo(py, l, Yg);
      r.re = sg * (xb - xa) * rn * ey.re;
      r.im = sg * (xb - xa) * rn * ey.im;
    } else {
      /* alpha_kl (-j w_y l) e(lY) (e(k x_b) - e(k x_a)) */
      fo_c ey = period_expo(py, l, Yg);
      fo_c ea = period_expo(px, k, llround(xa * scale)), eb = period_expo(px, k, llround(xb * scale));
      fo_c d = {eb.re - ea.re, eb.im - ea.im};
      fo_c t = cmul(ey, d);
      double a = -sqrt(Nx * Ny) / (4.0 * FO_PI * FO_PI * (double)k * (double)l);
      double m = sg * a * wy * (double)l;
      r.re = m * t.im;
      r.im = -m * t.re;
    }
  }
  return r;
}

/* Gradient of a real loss with respect to edge offsets (true units) for a
 * general tile; arguments as fo_edge_grad plus Nx, Ny and frac_bits. */
int fo_edge_grad_general(const double *xy, const int64_t *off, int64_t n_loops, int64_t Nx,
                         int64_t Ny, int32_t frac_bits, int32_t K, int32_t L, const double *G,
                         const int64_t *edge_idx, int64_t n_sel, int nthreads, double *g) {
  if (Nx < 1 || Ny < 1 || frac_bits < 0 || frac_bits > 20 || K < 0 || L < 0 || !G || !g)
    return FO_ERR_ARG;
  const double scale = ldexp(1.0, frac_bits);
  const int64_t nv = off[n_loops];
  for (int64_t i = 0; i < 2 * nv; ++i) {
    double X = xy[i] * scale;
    if (X != floor(X) || fabs(X) > 1073741823.0) return FO_ERR_RANGE;
  }
  fo_edge *E = NULL;
  int64_t n = 0;
  int st = build_edges(xy, off, n_loops, 0, &E, &n);
  if (st) return st;
  int64_t cnt = edge_idx ? n_sel : n;
  for (int64_t i = 0; i < cnt; ++i)
    if (edge_idx && (edge_idx[i] < 0 || edge_idx[i] >= n)) { free(E); return FO_ERR_ARG; }
  fo_period px, py;
  if (period_init(&px, Nx << frac_bits)) { free(E); return FO_ERR_NOMEM; }
  if (period_init(&py, Ny << frac_bits)) { free(px.tab); free(E); return FO_ERR_NOMEM; }
  set_threads(nthreads);
  const int64_t W = 2 * (int64_t)L + 1;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < cnt; ++i) {
    const fo_edge *e = &E[edge_idx ? edge_idx[i] : i];
    double acc = 0.0;
    for (int64_t k = -K; k <= K; ++k)
      for (int64_t l = -L; l <= L; ++l) {
        int64_t idx = (k + K) * W + (l + L);
        fo_c d = dcoef_general(&px, &py, (double)Nx, (double)Ny, scale, e, k, l);
        acc += G[2 * idx] * d.re + G[2 * idx + 1] * d.im;
      }
    g[i] = acc;
  }
  free(px.tab);
  free(py.tab);
  free(E);
  return FO_OK;
}

/* Exact edge-form area of every loop (lattice coordinates), sign kept. */
int fo_loop_areas(const double *xy, const int64_t *off, int64_t n_loops, int64_t *areas) {
  fo_edge *E = NULL;
  int64_t n = 0;
  int st = build_edges(xy, off, n_loops, 1, &E, &n);
  if (st) return st;
  for (int64_t m = 0; m < n_loops; ++m) {
    int64_t A = 0;
    for (int64_t e = off[m]; e < off[m + 1]; ++e)
      if (E[e].horizontal)
        A += (int64_t)E[e].ya * ((int64_t)E[e].xb - (int64_t)E[e].xa);
    areas[m] = A;
  }
  free(E);
  return FO_OK;
}
