/*
 * CPU oracle for the pruned continuous Haar transform (PCHT) of rectilinear
 * polygons.  TEST INFRASTRUCTURE ONLY: called by the tests, the package's
 * smoke check and the benchmark's CPU-baseline leg, never by the product path.
 * It shares no code, header or constant with the HIP library.
 *
 * What it computes (Scheibler, Hurley, Chebira, "Fast Continuous Haar and
 * Fourier Transforms of Rectilinear Polygons from VLSI Layouts"):
 *
 *   the inner products of f (the sum of the polygon indicators, Sec. III-A)
 *   with the 2D Haar basis over the tile [0,Nx) x [0,Ny) of Sec. II-B:
 *     phi_{0,0,0}                     scaling function of level 0
 *     psi^{hg}, psi^{gh}, psi^{hh}    wavelets of levels j = 0..J-1,
 *                                     positions kx, ky in [0, 2^j)
 *   phi_{j,kx,ky} = 2^j / sqrt(Nx Ny) on the cell
 *                   [kx Nx/2^j, (kx+1) Nx/2^j) x [ky Ny/2^j, (ky+1) Ny/2^j),
 *   and psi^{ab}_{j,kx,ky} = sum_{n,m} a_n b_m phi_{j+1, 2kx+n, 2ky+m} with
 *   g = (1, 1)/sqrt 2 and h = (1, -1)/sqrt 2; n steps along x, m along y.
 *
 * So, with A_{nm} the area of the polygon inside child cell (n, m) of cell
 * (j, kx, ky), the wavelet coefficients are 2^j / sqrt(Nx Ny) times
 *     hg: A00 + A01 - A10 - A11
 *     gh: A00 + A10 - A01 - A11
 *     hh: A00 - A01 - A10 + A11
 * and the scaling coefficient is Area(P inside the tile) / sqrt(Nx Ny)
 * (Sec. III-B1: inner product with a scaling function = intersection area
 * times 2^j / sqrt(Nx Ny)).
 *
 * Algorithm (Sec. III-B1, PCHT): per polygon, divide the tile into four parts
 * recursively; a part wholly inside or outside the polygon ends the recursion
 * (the wavelets below it see a constant and give zero).  Every intersection
 * area is Algorithm 1 (IntersectionArea) over the polygon's horizontal edges.
 * The transform of several polygons is the sum of their transforms (Sec.
 * III-A, linearity).  Counting the recursive calls that compute four child
 * areas gives the number of non-terminating calls of the complexity model
 * (Sec. III-B2).
 *
 * Output layout (a convention of this implementation, the paper fixes none):
 * a 2^J x 2^J row-major pyramid P[row][col].  P[0][0] holds the scaling
 * coefficient; with p = 2^j, level j puts hg at [ky][p + kx], gh at
 * [p + ky][kx] and hh at [p + ky][p + kx].  U holds the integer sums (areas
 * before the factor 2^j / sqrt(Nx Ny)), W the coefficients.
 *
 * Vertices are on the integer lattice (Sec. II-A2); 2^J must divide Nx and
 * Ny so that every cell corner is a lattice point; all arithmetic on areas is
 * exact int64.  Loops may have either orientation: the paper orders vertices
 * clockwise, and a counter-clockwise loop (negative Algorithm-1 area over the
 * whole plane) is counted with the opposite sign.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define PO_OK 0
#define PO_ERR_ARG -1
#define PO_ERR_NOT_RECTILINEAR -2
#define PO_ERR_RANGE -3
#define PO_ERR_NOMEM -7

/* One horizontal edge (xa, y) -> (xb, y) of a loop, in input order. */
typedef struct {
  int64_t xa, xb, y;
} po_hedge;

typedef struct {
  int64_t Nx, Ny;
  int J;
  int64_t side;  /* 2^J */
  int64_t *U;
  int64_t nodes; /* calls that computed four child areas */
} po_ctx;

/* Algorithm 1: area of the polygon (clockwise) inside [a1,a2) x [b1,b2). */
static int64_t intersection_area(const po_hedge *E, int64_t n, int64_t a1, int64_t b1,
                                 int64_t a2, int64_t b2) {
  int64_t I = 0;
  for (int64_t e = 0; e < n; ++e) {
    int64_t u = E[e].xa < E[e].xb ? E[e].xa : E[e].xb;
    int64_t v = E[e].xa < E[e].xb ? E[e].xb : E[e].xa;
    if (a2 <= u || v <= a1 || E[e].y <= b1) continue;
    int64_t s = E[e].xb > E[e].xa ? 1 : -1;
    int64_t w = (v < a2 ? v : a2) - (u > a1 ? u : a1);
    int64_t h = (E[e].y < b2 ? E[e].y : b2) - b1;
    I += s * w * h;
  }
  return I;
}

/* One non-terminating call: cell (j, kx, ky) meets the polygon's boundary. */
static void visit(po_ctx *c, const po_hedge *E, int64_t n, int64_t sigma, int j, int64_t kx,
                  int64_t ky) {
  const int64_t wx = c->Nx >> j, wy = c->Ny >> j, hx = wx / 2, hy = wy / 2;
  const int64_t a1 = kx * wx, b1 = ky * wy;
  int64_t A[2][2];
  for (int nn = 0; nn < 2; ++nn)
    for (int m = 0; m < 2; ++m)
      A[nn][m] = sigma * intersection_area(E, n, a1 + nn * hx, b1 + m * hy, a1 + (nn + 1) * hx,
                                           b1 + (m + 1) * hy);
  c->nodes += 1;
  const int64_t p = (int64_t)1 << j, S = c->side;
  c->U[ky * S + p + kx] += A[0][0] + A[0][1] - A[1][0] - A[1][1];
  c->U[(p + ky) * S + kx] += A[0][0] + A[1][0] - A[0][1] - A[1][1];
  c->U[(p + ky) * S + p + kx] += A[0][0] - A[0][1] - A[1][0] + A[1][1];
  if (j + 1 >= c->J) return;
  for (int nn = 0; nn < 2; ++nn)
    for (int m = 0; m < 2; ++m)
      if (A[nn][m] > 0 && A[nn][m] < hx * hy) visit(c, E, n, sigma, j + 1, 2 * kx + nn, 2 * ky + m);
}

/*
 * xy: interleaved vertex coordinates (integers stored as doubles), off: loop
 * offsets (n_loops + 1).  U (int64) and W (double, may be NULL) receive the
 * 2^J x 2^J pyramid; nodes (may be NULL) the number of non-terminating calls.
 */
int po_pcht(const double *xy, const int64_t *off, int64_t n_loops, int64_t Nx, int64_t Ny,
            int J, int64_t *U, double *W, int64_t *nodes) {
  if (!xy || !off || !U || n_loops < 0 || J < 0 || J > 15 || Nx < 1 || Ny < 1) return PO_ERR_ARG;
  if ((Nx % ((int64_t)1 << J)) || (Ny % ((int64_t)1 << J))) return PO_ERR_ARG;
  if (Nx > ((int64_t)1 << 20) || Ny > ((int64_t)1 << 20)) return PO_ERR_RANGE;
  if (off[0] != 0) return PO_ERR_ARG;
  po_ctx c;
  c.Nx = Nx;
  c.Ny = Ny;
  c.J = J;
  c.side = (int64_t)1 << J;
  c.U = U;
  c.nodes = 0;
  const int64_t npy = c.side * c.side;
  for (int64_t i = 0; i < npy; ++i) U[i] = 0;
  int64_t cap = 0;
  for (int64_t m = 0; m < n_loops; ++m)
    if (off[m + 1] - off[m] > cap) cap = off[m + 1] - off[m];
  po_hedge *E = (po_hedge *)malloc(sizeof(po_hedge) * (size_t)(cap > 0 ? cap : 1));
  if (!E) return PO_ERR_NOMEM;
  int st = PO_OK;
  for (int64_t m = 0; m < n_loops && st == PO_OK; ++m) {
    const int64_t b0 = off[m], cnt = off[m + 1] - off[m];
    if (cnt < 4 || (cnt & 1)) { st = PO_ERR_NOT_RECTILINEAR; break; }
    int64_t n = 0, whole = 0;
    for (int64_t i = 0; i < cnt; ++i) {
      const int64_t a = b0 + i, b = b0 + (i + 1) % cnt;
      const double xa = xy[2 * a], ya = xy[2 * a + 1], xb = xy[2 * b], yb = xy[2 * b + 1];
      if (xa != floor(xa) || ya != floor(ya) || fabs(xa) > 1e9 || fabs(ya) > 1e9) {
        st = PO_ERR_RANGE;
        break;
      }
      const int h = (ya == yb) && (xa != xb), v = (xa == xb) && (ya != yb);
      if (!h && !v) { st = PO_ERR_NOT_RECTILINEAR; break; }
      if (h) {
        E[n].xa = (int64_t)xa;
        E[n].xb = (int64_t)xb;
        E[n].y = (int64_t)ya;
        whole += E[n].y * (E[n].xb - E[n].xa);
        ++n;
      }
    }
    if (st) break;
    if (whole == 0) { st = PO_ERR_NOT_RECTILINEAR; break; }
    const int64_t sigma = whole > 0 ? 1 : -1;
    const int64_t A = sigma * intersection_area(E, n, 0, 0, Nx, Ny);
    U[0] += A;
    if (J > 0 && A > 0 && A < Nx * Ny) visit(&c, E, n, sigma, 0, 0, 0);
  }
  free(E);
  if (st) return st;
  if (W) {
    const double r = 1.0 / sqrt((double)Nx * (double)Ny);
    for (int64_t row = 0; row < c.side; ++row)
      for (int64_t col = 0; col < c.side; ++col) {
        int64_t mx = row > col ? row : col;
        int j = 0;
        while (((int64_t)2 << j) <= mx) ++j; /* level: 2^j <= max(row, col) < 2^{j+1} */
        const double sc = mx == 0 ? r : ldexp(r, j);
        W[row * c.side + col] = (double)U[row * c.side + col] * sc;
      }
  }
  if (nodes) *nodes = c.nodes;
  return PO_OK;
}
