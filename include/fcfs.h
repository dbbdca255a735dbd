/*
 * fcfs.h -- C ABI of the MI355X (gfx950) library for the continuous Fourier
 * series (CFS) of rectilinear lattice polygons, after Scheibler, Hurley and
 * Chebira, "Fast Continuous Haar and Fourier Transforms of Rectilinear
 * Polygons from VLSI Layouts".
 *
 * The CFS coefficient over a T x T tile (Sec. II-C; inner product of
 * Sec. III-A with the orthonormal Fourier basis) is
 *
 *     F[k,l] = (1/T) * integral of f(x,y) e^{-j 2 pi (k x + l y) / T} dx dy,
 *
 * f being the sum of the polygons' indicators (Sec. III-A, signal model).
 * Prop. 3 (Sec. III-C1) gives it in closed form from the vertices.  The
 * library uses the equivalent signed-corner form: every vertex v is an
 * endpoint of exactly one horizontal edge; s_v = +1 if that edge ends at v in
 * clockwise loop order and -1 if it starts there (the +1/-1 entries of the
 * sparse image of Alg. 2, lines building V^{KL}).  With e(t) = e^{-j 2 pi t/T}:
 *
 *     F[0,0] = (1/T)            sum_v s_v x_v y_v        (area / T; Step 1)
 *     F[k,0] = j/(2 pi k)       sum_v s_v y_v e(k x_v)   (Step 2)
 *     F[0,l] = j/(2 pi l)       sum_v s_v x_v e(l y_v)   (Step 3)
 *     F[k,l] = -T/(4 pi^2 k l)  sum_v s_v e(k x_v) e(l y_v)   (Step 4)
 *
 * Conventions shared by every entry point:
 *  - Ownership: the caller owns every data buffer and every workspace; the
 *    handle owns only its constant twiddle tables and batch plans.
 *  - Pointers marked (device) are device memory on the handle's device;
 *    (host) pointers are ordinary host memory.
 *  - Execution: device work is enqueued on the handle's stream and the call
 *    returns without synchronising.  A fault on the device surfaces as
 *    FCFS_ERR_DEVICE on a later call.
 *  - Errors: a negative status; outputs are then unspecified.
 *    fcfs_last_error() gives a human-readable detail.
 *  - The device path trusts the corner data it is given: s_v in {+1,-1},
 *    corners polygon-contiguous (accuracy depends on it), |x|,|y| < 2^30.
 *  - The tile period T is a power of two in [2, 8192]; K, L >= 0.
 *  - Threading: calls on one handle must not overlap in time.  A handle keeps
 *    no per-thread state, so it may pass from one host thread to another
 *    between calls (e.g. a backward pass run by another thread while the
 *    caller waits).  Different handles may be used concurrently.
 */
#ifndef FCFS_H_
#define FCFS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FCFS_OK = 0,
  FCFS_ERR_INVALID_ARG = -1,
  FCFS_ERR_NOT_RECTILINEAR = -2,
  FCFS_ERR_RANGE = -3,
  FCFS_ERR_UNSUPPORTED = -4,
  FCFS_ERR_WORKSPACE = -5,
  FCFS_ERR_DEVICE = -6,
  FCFS_ERR_NO_MEMORY = -7
} fcfs_status;

/* Arithmetic of the vertex contraction (the F[k,l] sums, Step 4).  Phases,
 * the area and the axis sums are exact integer / FP64 in every mode.
 *   FCFS_FP32        FP32 twiddles, FP32 MFMA products, FP32 accumulation.
 *   FCFS_SPLIT_BF16  twiddle w = hi + lo with hi, lo bfloat16 (round to
 *                    nearest even); hi*hi' + hi*lo' + lo*hi' on bf16 MFMA,
 *                    FP32 accumulation.
 *   FCFS_SPLIT_FP16  the same with binary16 hi, lo.
 *   FCFS_AUTO        (fcfs_forward, fcfs_forward_noalloc, fcfs_workspace_size
 *                    and fcfs_forward_plan_info only) the form a cost model
 *                    expects to be fastest among those that meet the split
 *                    bound: the lattice form of fcfs_forward_fft (FP64) where
 *                    its work, about L T log2 T, is well below the
 *                    contraction's 24 (K+1)(L+1) V flop (large V, small T:
 *                    Step 4 of Sec. III-C1 as a 2-D DFT of the corner
 *                    image), else the split-bf16 contraction; the direct form
 *                    for small problems as always. */
typedef enum {
  FCFS_FP32 = 0,
  FCFS_SPLIT_BF16 = 1,
  FCFS_SPLIT_FP16 = 2,
  FCFS_AUTO = 3
} fcfs_precision;

typedef struct fcfs_handle fcfs_handle;
typedef struct fcfs_plan fcfs_plan;
typedef struct fcfs_step_plan fcfs_step_plan;

/* One clip: a signed corner list (the concatenated sparse lists of Alg. 2 for
 * all polygons of the tile, Sec. III-C1 "multiple polygons") and its output. */
typedef struct {
  const int32_t *x;  /* (device) [V] corner abscissae                        */
  const int32_t *y;  /* (device) [V] corner ordinates                        */
  const int8_t *s;   /* (device) [V] corner signs, +1 or -1                  */
  int64_t V;         /* number of corners, >= 0                              */
  int32_t T;         /* tile period, power of two in [2, 8192]               */
  int32_t K, L;      /* cut-offs: |k| <= K, |l| <= L                          */
  float *F;          /* (device) out: (2K+1)*(2L+1) complex64 as interleaved
                        (re, im) floats, k-major: F[(k+K)*(2L+1) + (l+L)]     */
  int64_t *area;     /* (device) out: exact sum_v s_v x_v y_v (= area), or NULL */
} fcfs_clip;

/* Creates a handle on `device`, enqueuing on `hip_stream` (a hipStream_t; NULL
 * = the device's null stream).  Builds the twiddle tables of Step 4 once:
 * e^{j 2 pi p / 8192}, p = 0..8191, in FP64, FP32 and bf16/fp16 hi+lo. */
fcfs_status fcfs_create(fcfs_handle **h, int device, void *hip_stream);
fcfs_status fcfs_destroy(fcfs_handle *h);
/* Makes `hip_stream` the handle's stream for later calls.  The new stream
 * waits (an event, no host wait) for everything enqueued on the previous one,
 * so a workspace, an output or a table used before the switch may be reused
 * after it.  The previous stream must still exist.  Neither stream may be
 * capturing a graph for this order to be taken (the entry points refuse a
 * capturing stream anyway).  Errors: FCFS_ERR_INVALID_ARG (NULL handle),
 * FCFS_ERR_DEVICE (a failed HIP call). */
fcfs_status fcfs_set_stream(fcfs_handle *h, void *hip_stream);

/* (host) Polygon loops -> signed corner list and edge map.
 * xy: [n_vertices][2] lattice coordinates; loop_off: [n_loops+1] offsets,
 * loop m = vertices loop_off[m] .. loop_off[m+1]-1 (Sec. II-A2: ordered
 * vertices of a rectilinear polygon).  Validates: >= 4 and an even number of
 * vertices per loop, every edge horizontal or vertical with nonzero length,
 * edges alternating, nonzero area.  A counter-clockwise loop is taken as its
 * clockwise reversal (its signs are negated).
 * Outputs (host, caller-allocated, [n_vertices] each, any may be NULL):
 *   x, y  copies of the coordinates, s the corner signs,
 *   hedge[v] / vedge[v] the index of the horizontal / vertical edge at v,
 *   edge e joining vertex e to the next vertex of its loop.
 * Returns FCFS_ERR_NOT_RECTILINEAR or FCFS_ERR_RANGE on invalid loops. */
fcfs_status fcfs_loops_to_corners(const int32_t *xy, const int64_t *loop_off, int64_t n_loops,
                                  int32_t *x, int32_t *y, int8_t *s, int64_t *hedge,
                                  int64_t *vedge);

/* Workspace (device bytes) that fcfs_forward (adjoint = 0) or fcfs_adjoint
 * (adjoint = 1) needs for clip `c` at precision `p`.  Depends only on V, T, K,
 * L and p.  Pointers in `c` are not read. */
fcfs_status fcfs_workspace_size(const fcfs_clip *c, fcfs_precision p, int adjoint,
                                size_t *bytes);

/* Forward transform (Prop. 3 / Alg. 2 for one tile): writes c->F and
 * c->area.  ws: (device) workspace of at least fcfs_workspace_size bytes,
 * 256-byte aligned.  Steps enqueued: pre-pass (phase reduction, area),
 * axis sums (FP64), vertex contraction on MFMA, epilogue.
 * Small problems (V <= 1024 corners and V (K+1)(2L+1) <= 2^22) are evaluated
 * in one launch by the direct form, in FP64 whatever `p` asks for (the same
 * exact integer phases; the result is at least as accurate as the requested
 * form); a tile variant forced with fcfs_set_tile selects the staged MFMA
 * path at every size.  The workspace size is the same either way. */
fcfs_status fcfs_forward(fcfs_handle *h, const fcfs_clip *c, fcfs_precision p, void *ws,
                         size_t ws_bytes);

/* fcfs_forward without a workspace argument, for callers that cannot
 * allocate device memory (serving loops and harnesses that forbid it): the
 * work runs in a scratch array the library holds on each device it runs on,
 * 96 MiB, for the life of the process (the precision clip of 200k corners at
 * T = 8192, K = L = 511 needs 84 MiB).  Same arguments, kernels and results as
 * fcfs_forward; a clip whose workspace (fcfs_workspace_size) exceeds the
 * scratch is refused with FCFS_ERR_WORKSPACE.  The call allocates nothing:
 * no hipMalloc or hipFree, no allocating library routine.  Every call on a
 * device shares that device's scratch, so calls that overlap on one device
 * (several streams or host threads) race; the scratch keeps the last call's
 * contents, none of which a later call reads.  Like every entry point it
 * refuses a stream the caller is capturing. */
fcfs_status fcfs_forward_noalloc(fcfs_handle *h, const fcfs_clip *c, fcfs_precision p);

/* Low-pass forward: fcfs_forward restricted to the band |k| <= kmax,
 * |l| <= lmax (clamped to K, L) and, when radius >= 0, to the disc
 * k^2 + l^2 <= radius^2 (a circular pupil, as needed by lithography models,
 * Sec. I and the outlook of Sec. V).  c->F keeps its full (2K+1) x (2L+1)
 * layout: the entries inside the band (and disc) equal those of fcfs_forward
 * up to rounding, every other entry is written as zero.  Contraction tiles
 * wholly outside the disc are skipped.  ws: at least fcfs_band_workspace_size
 * bytes (same arguments), 256-byte aligned.  FCFS_ERR_INVALID_ARG for a
 * negative kmax or lmax or a NaN radius. */
fcfs_status fcfs_band_workspace_size(const fcfs_clip *c, int32_t kmax, int32_t lmax,
                                     double radius, fcfs_precision p, size_t *bytes);
fcfs_status fcfs_forward_band(fcfs_handle *h, const fcfs_clip *c, int32_t kmax, int32_t lmax,
                              double radius, fcfs_precision p, void *ws, size_t ws_bytes);

/* Lattice (FFT) form of the forward transform: the same coefficients as
 * fcfs_forward, computed in FP64 from the corner image on the T x T lattice
 * (Sec. III-C1, Step 4: a 2-D DFT of the image of corner signs) instead of
 * the vertex contraction: a sparse DFT along y of every x-row's exact integer
 * image for l = 1..L, then a radix-2 FFT of length T along x per l, cropped to
 * |k| <= K; the axes and F[0,0] as in fcfs_forward.  Cost O(V L + L T log T),
 * independent of the precision forms.  ws: at least fcfs_fft_workspace_size
 * bytes (16 T L + 4 V + ... : ~68 MB at T = 8192, L = 511), 256-byte aligned. */
fcfs_status fcfs_fft_workspace_size(const fcfs_clip *c, size_t *bytes);
fcfs_status fcfs_forward_fft(fcfs_handle *h, const fcfs_clip *c, void *ws, size_t ws_bytes);

/* General tile (Prop. 3 for any periods): the tile is Nx x Ny lattice units
 * (any positive integers, Nx != Ny allowed, Sec. II-C with w_x = 2 pi / Nx,
 * w_y = 2 pi / Ny), and corners may sit on the finer grid of step 2^-F
 * (F = frac_bits; F = 0 is the integer lattice of Sec. II-A2): x[v], y[v] are
 * the coordinates times 2^F.  The phases k x / Nx are reduced exactly modulo
 * Mx = Nx 2^F (likewise My); Mx and My must lie in [2, 2^24].  Periods up to
 * 8192 use one table entry per residue; past 8192 the twiddle is the product
 * of two table entries, e(2 pi p / M) = Whi[p >> 12] Wlo[p mod 4096] (a
 * two-level twiddle for fine sub-lattice grids), the phase being reduced
 * exactly in FP64, and the axis sums are taken over the corners
 * directly instead of over residue histograms.  Output as
 * fcfs_forward with alpha_{k,l} = -sqrt(Nx Ny)/(4 pi^2 k l),
 * alpha_{k,0} = j sqrt(Nx/Ny)/(2 pi k), alpha_{0,l} = j sqrt(Ny/Nx)/(2 pi l),
 * F[0,0] = area / sqrt(Nx Ny); `area` receives sum_v s_v x[v] y[v] (the area
 * times 4^F).  The contraction uses per-period tables that the handle builds
 * on the first call with a period (a synchronous upload) and caches. */
typedef struct {
  const int32_t *x;   /* (device) [V] corner abscissae, times 2^frac_bits      */
  const int32_t *y;   /* (device) [V] corner ordinates, times 2^frac_bits      */
  const int8_t *s;    /* (device) [V] corner signs                             */
  int64_t V;
  int32_t Nx, Ny;     /* tile periods, lattice units                          */
  int32_t frac_bits;  /* F in [0, 13]                                         */
  int32_t K, L;       /* cut-offs, <= 4095                                    */
  float *F;           /* (device) out: (2K+1)(2L+1) complex64, as fcfs_forward */
  int64_t *area;      /* (device) out: sum s x y in grid units, or NULL        */
} fcfs_gclip;

/* Workspace of fcfs_forward_general (256-byte aligned).  FCFS_ERR_UNSUPPORTED
 * when Nx 2^F or Ny 2^F is outside [2, 2^24], F > 13 or K, L > 4095. */
fcfs_status fcfs_general_workspace_size(const fcfs_gclip *c, fcfs_precision p, size_t *bytes);
/* Forward transform of a general tile: pre-pass (residues, area), axis sums
 * and FP64 low-frequency block on the side stream, MFMA contraction with
 * exact phases (f x) mod M, epilogue with the alpha factors above.  The split
 * precisions run a software-pipelined contraction kernel (one wave per SIMD);
 * FP32, or a handle with a tile variant forced by fcfs_set_tile, an eight-wave
 * kernel; periods past 8192 an eight-wave kernel on two-level tables (the
 * split entries rounded from the FP32 product in the kernel).  The workspace
 * size covers either. */
fcfs_status fcfs_forward_general(fcfs_handle *h, const fcfs_gclip *c, fcfs_precision p, void *ws,
                                 size_t ws_bytes);
/* Low-pass form of fcfs_forward_general (the pupil of the lithography use in
 * Sec. I and Sec. V, as fcfs_forward_band for the square tile): writes the
 * whole (2K+1) x (2L+1) grid of c->F, computing only |k| <= kmax,
 * |l| <= lmax and, when radius >= 0, k^2 + l^2 <= radius^2; every other entry
 * is zero.  Frequency tiles wholly outside the disc are skipped.  ws: at least
 * fcfs_general_band_workspace_size bytes, 256-byte aligned.
 * FCFS_ERR_INVALID_ARG for a negative band or a NaN radius. */
fcfs_status fcfs_general_band_workspace_size(const fcfs_gclip *c, int32_t kmax, int32_t lmax,
                                             double radius, fcfs_precision p, size_t *bytes);
fcfs_status fcfs_forward_general_band(fcfs_handle *h, const fcfs_gclip *c, int32_t kmax,
                                      int32_t lmax, double radius, fcfs_precision p, void *ws,
                                      size_t ws_bytes);

/* Adjoint of fcfs_forward_general with respect to the corner coordinates, in
 * lattice units (the derivative of the general closed forms of Prop. 3):
 * gx[v] = dLoss/dx_v, gy[v] = dLoss/dy_v for the true coordinates
 * x[v] / 2^frac_bits.  grad_F, band (kmax, lmax) and radius as in
 * fcfs_adjoint_band.  ws: at least fcfs_general_adjoint_workspace_size bytes,
 * 256-byte aligned.  Uses the per-period tables of the handle (built on first
 * use, as for the forward).  Periods Mx, My up to 2^23 (two-level tables
 * past 8192, as for the forward): FCFS_ERR_UNSUPPORTED past that. */
fcfs_status fcfs_general_adjoint_workspace_size(const fcfs_gclip *c, fcfs_precision p,
                                                size_t *bytes);
fcfs_status fcfs_adjoint_general(fcfs_handle *h, const fcfs_gclip *c, const float *grad_F,
                                 int32_t kmax, int32_t lmax, double radius, float *gx, float *gy,
                                 fcfs_precision p, void *ws, size_t ws_bytes);

/* The loss of the edge-moving optimisation behind a pupil (the low-pass need
 * of lithography models, Sec. I): loss = sum_{k,l} |H[k,l] F[k,l] - G[k,l]|^2
 * and its cotangent grad = dLoss/dRe F + j dLoss/dIm F = 2 H (H F - G), for
 * the backward of fcfs_adjoint / fcfs_adjoint_band.  F, G, grad: (device)
 * (2K+1)(2L+1) complex64, layout of fcfs_clip.F; H: (device) real weights in
 * the same layout, or NULL for the indicator of the disc k^2 + l^2 <= radius^2
 * (radius < 0: H = 1).  loss: (device) one double.  Sums in FP64 in a fixed
 * order (deterministic).  ws: fcfs_pupil_loss_workspace_size bytes, 256-byte
 * aligned. */
fcfs_status fcfs_pupil_loss_workspace_size(size_t *bytes);
fcfs_status fcfs_pupil_loss(fcfs_handle *h, const float *F, const float *G, const float *H,
                            int32_t K, int32_t L, double radius, double *loss, float *grad,
                            void *ws, size_t ws_bytes);

/* One step of the edge-moving optimisation behind a pupil in a single call,
 * for loops that drive the step without an autograd engine: the launches of
 *   fcfs_apply_edge_offsets (corners from base_x, base_y and the offsets),
 *   fcfs_forward_band (kmax, lmax, radius),
 *   fcfs_pupil_loss (G, H or the disc of radius),
 *   fcfs_adjoint_band (same band and disc) and fcfs_edge_grad,
 * enqueued in that order on the handle's stream with no host work between
 * them; results are bit-identical to making those calls one by one.  All
 * arrays (device): base_x, base_y, s, hedge, vedge [V] as from
 * fcfs_loops_to_corners (E = V edges), offsets [V] (one per edge, rounded to
 * integers), G (and H unless NULL) (2K+1)(2L+1) complex64 (real for H).
 * Outputs: loss (one double), g_edge [V] = dLoss/d(edge offset), and F_out
 * ((2K+1)(2L+1) complex64, the low-pass spectrum) unless NULL.  T a power of
 * two.  ws: at least fcfs_pupil_step_workspace_size bytes, 256-byte aligned;
 * it also holds the moved corners, the spectrum (when F_out is NULL), the
 * cotangent and the per-corner gradients. */
fcfs_status fcfs_pupil_step_workspace_size(int64_t V, int32_t T, int32_t K, int32_t L,
                                           int32_t kmax, int32_t lmax, double radius,
                                           fcfs_precision p, size_t *bytes);
fcfs_status fcfs_pupil_step(fcfs_handle *h, const int32_t *base_x, const int32_t *base_y,
                            const int8_t *s, const int64_t *hedge, const int64_t *vedge,
                            const float *offsets, int64_t V, int32_t T, int32_t K, int32_t L,
                            int32_t kmax, int32_t lmax, double radius, const float *G,
                            const float *H, fcfs_precision p, double *loss, float *g_edge,
                            float *F_out, void *ws, size_t ws_bytes);

/* fcfs_pupil_step captured once into a HIP graph and replayed: for loops that
 * repeat the step with new values in the same buffers (offsets, G, H).
 * fcfs_pupil_step_plan takes the arguments of fcfs_pupil_step, runs one
 * step eagerly (argument checks, one-time kernel set-up; the outputs hold its
 * result) and captures the next one on a stream of its own.  Every buffer,
 * the workspace included, must stay allocated and unmoved while the plan
 * lives, and so must the handle (the graph reads its twiddle tables);
 * fcfs_step_plan_launch replays the step on the handle's stream (same
 * device).  The plan owns its graph; fcfs_step_plan_destroy frees it. */
fcfs_status fcfs_pupil_step_plan(fcfs_handle *h, const int32_t *base_x, const int32_t *base_y,
                                 const int8_t *s, const int64_t *hedge, const int64_t *vedge,
                                 const float *offsets, int64_t V, int32_t T, int32_t K, int32_t L,
                                 int32_t kmax, int32_t lmax, double radius, const float *G,
                                 const float *H, fcfs_precision p, double *loss, float *g_edge,
                                 float *F_out, void *ws, size_t ws_bytes, fcfs_step_plan **plan);
fcfs_status fcfs_step_plan_launch(fcfs_handle *h, fcfs_step_plan *plan);
fcfs_status fcfs_step_plan_destroy(fcfs_step_plan *plan);

/* Batch of general tiles (fcfs_forward_general for every clip c[0..n-1],
 * each with its own periods, grid step, cut-offs, corners and outputs) as one
 * captured graph, in the manner of fcfs_pupil_step_plan: the workspace holds
 * one 256-byte aligned slice per clip (fcfs_general_batch_workspace_size);
 * the plan runs every clip once eagerly (the outputs hold the result), then
 * captures all their launches on a stream of its own.  Replays
 * (fcfs_step_plan_launch) recompute every clip from the current contents of
 * the corner arrays.  The period tables the graph reads are pinned in the
 * handle's cache until the plan is destroyed (the cache grows past its 16
 * entries rather than evict a pinned table).  Buffers, workspace and handle
 * must outlive the plan, as for fcfs_pupil_step_plan. */
fcfs_status fcfs_general_batch_workspace_size(const fcfs_gclip *c, int32_t n, fcfs_precision p,
                                              size_t *bytes);
fcfs_status fcfs_general_batch_plan(fcfs_handle *h, const fcfs_gclip *c, int32_t n,
                                    fcfs_precision p, void *ws, size_t ws_bytes,
                                    fcfs_step_plan **plan);

/* Pruned continuous Haar transform (PCHT, Sec. III-B1) of the polygons of one
 * tile [0,Nx) x [0,Ny): the inner products of the sum of polygon indicators
 * with the 2-D Haar basis of Sec. II-B (scaling function phi_{0,0,0} and the
 * wavelets psi^{hg}, psi^{gh}, psi^{hh} of levels j = 0..J-1, positions
 * kx, ky < 2^j; psi^{ab} = sum_{n,m} a_n b_m phi_{j+1,2kx+n,2ky+m} with
 * g = (1,1)/sqrt2, h = (1,-1)/sqrt2, n along x, m along y).  Per polygon the
 * quadtree is refined where a cell meets the polygon's boundary; intersection
 * areas are exact integers.  Polygons may extend past the tile (clipped).
 * Output: a 2^J x 2^J row-major pyramid.  [0][0] holds the scaling
 * coefficient; with p = 2^j, level j has hg at [ky][p+kx], gh at [p+ky][kx]
 * and hh at [p+ky][p+kx].  U gets the integer sums (the coefficient times
 * sqrt(Nx Ny) / 2^j, i.e. signed sums of child areas), W the coefficients.
 * Requirements: 1 <= Nx, Ny <= 8192, 0 <= J <= 13, 2^J divides Nx and Ny.
 * Polygon offsets must be nondecreasing (they are clamped to [0, V]). */
typedef struct {
  const int32_t *x;         /* (device) [V] corner abscissae, loop order       */
  const int32_t *y;         /* (device) [V] corner ordinates                   */
  const int8_t *s;          /* (device) [V] corner signs (fcfs_loops_to_corners) */
  const int64_t *poly_off;  /* (device) [M+1] polygon m = corners
                               poly_off[m] .. poly_off[m+1]-1                  */
  int64_t V;                /* corners                                        */
  int64_t M;                /* polygons                                       */
  int32_t Nx, Ny;           /* tile size (lattice units)                      */
  int32_t J;                /* wavelet levels                                 */
  int64_t *U;               /* (device) out: [4^J] int64 integer sums          */
  double *W;                /* (device) out: [4^J] coefficients, or NULL       */
  int64_t *stats;           /* (device) out: [2] cells visited (calls that
                               split a cell) and cell-corner pairs, or NULL    */
} fcfs_haar_clip;

/* Workspace of fcfs_haar (depends on M only: control words, 64 copies of the
 * 64 x 64 int64 block of the levels j < 6 (2 MiB; the waves add into their
 * own copy instead of all into the same few entries), per-polygon task counts
 * and the task list of large polygons split over several waves; about
 * 2 MiB + 4 M + 8 max(M, 4096) bytes), 256-byte aligned.
 * FCFS_ERR_UNSUPPORTED / FCFS_ERR_INVALID_ARG for sizes outside the limits. */
fcfs_status fcfs_haar_workspace_size(const fcfs_haar_clip *c, size_t *bytes);
/* Enqueues the transform on the handle's stream: clears U (a fill kernel),
 * walks every polygon's quadtree (one wave per polygon), then adds the coarse
 * copies into U and scales U into W when W is not NULL.  Calls that overlap
 * on one workspace race. */
fcfs_status fcfs_haar(fcfs_handle *h, const fcfs_haar_clip *c, void *ws, size_t ws_bytes);

/* Adjoint of fcfs_forward with respect to the corner coordinates (the
 * derivative of the four closed forms of Prop. 3 in x_v and y_v).
 * grad_F: (device) cotangent, same layout as c->F, holding
 * dLoss/dRe F + j dLoss/dIm F.  Writes (device) gx[V] = dLoss/dx_v and
 * gy[V] = dLoss/dy_v.  c->F and c->area are not touched. */
fcfs_status fcfs_adjoint(fcfs_handle *h, const fcfs_clip *c, const float *grad_F, float *gx,
                         float *gy, fcfs_precision p, void *ws, size_t ws_bytes);

/* Adjoint of fcfs_forward_band with the same kmax, lmax, radius: only the
 * entries of grad_F with |k| <= kmax, |l| <= lmax (clamped to K, L) and, when
 * radius >= 0, k^2 + l^2 <= radius^2 are used; the GEMM and the axis sums then
 * cover only that band.  It is also the adjoint of fcfs_forward whenever
 * grad_F vanishes outside the band (e.g. a loss behind a pupil).  The
 * workspace of fcfs_workspace_size(adjoint = 1) always suffices.
 * FCFS_ERR_INVALID_ARG for a negative kmax or lmax or a NaN radius. */
fcfs_status fcfs_adjoint_band(fcfs_handle *h, const fcfs_clip *c, const float *grad_F,
                              int32_t kmax, int32_t lmax, double radius, float *gx, float *gy,
                              fcfs_precision p, void *ws, size_t ws_bytes);

/* Edge-offset gradient: a shift of edge e moves both of its endpoints (along
 * x for a vertical edge, along y for a horizontal one), so
 * g_edge[e] = sum of gx (vertical) or gy (horizontal) over the two corners of
 * e.  hedge/vedge: (device) [V] maps from fcfs_loops_to_corners; gx, gy:
 * (device) [V]; g_edge: (device) out [E]. */
fcfs_status fcfs_edge_grad(fcfs_handle *h, const float *gx, const float *gy,
                           const int64_t *hedge, const int64_t *vedge, int64_t V, int64_t E,
                           float *g_edge);

/* Corner coordinates after edge shifts (the parametrisation used for
 * edge-moving optimisation): x[v] = base_x[v] + rint(offsets[vedge[v]]),
 * y[v] = base_y[v] + rint(offsets[hedge[v]]).  All arrays (device); offsets
 * has one entry per edge and should hold integers (the lattice of Sec.
 * II-A2); fractional values are rounded to nearest. */
fcfs_status fcfs_apply_edge_offsets(fcfs_handle *h, const int32_t *base_x, const int32_t *base_y,
                                    const int64_t *hedge, const int64_t *vedge,
                                    const float *offsets, int64_t V, int32_t *x, int32_t *y);
/* The same on a grid of step 2^-frac_bits: base_x, base_y, x, y in grid units
 * (coordinates times 2^frac_bits), offsets in lattice units; each corner moves
 * by rint(offset 2^frac_bits) grid steps.  frac_bits in [0, 13]. */
fcfs_status fcfs_apply_edge_offsets_grid(fcfs_handle *h, const int32_t *base_x,
                                         const int32_t *base_y, const int64_t *hedge,
                                         const int64_t *vedge, const float *offsets, int64_t V,
                                         int32_t frac_bits, int32_t *x, int32_t *y);

/* Batched forward: n clips (each with its own V, T, K, L and outputs) in one
 * persistent contraction launch.  The first call with *plan == NULL builds a
 * plan (work list, tile shapes) and captures the enqueued sequence in a
 * hipGraph; later calls with the same plan and the same clip array contents
 * replay the graph.  ws: (device) workspace of at least
 * fcfs_batch_workspace_size bytes, queried with the same handle (its tuned
 * tile shape and corners per work item set the layout; h = NULL gives the
 * built-in choices). */
fcfs_status fcfs_batch_workspace_size(fcfs_handle *h, const fcfs_clip *c, int32_t n,
                                      fcfs_precision p, size_t *bytes);
fcfs_status fcfs_forward_batch(fcfs_handle *h, const fcfs_clip *c, int32_t n, fcfs_precision p,
                               void *ws, size_t ws_bytes, fcfs_plan **plan);
fcfs_status fcfs_plan_destroy(fcfs_plan *plan);

/* Debug export of the exact integer phase indices of Step 4:
 * p[i*V + v] = ((k0 + i) * x_v) mod T for i in [0, nk) (axis = 0), or with
 * y_v (axis = 1), computed by the same pre-pass and phase arithmetic as the
 * contraction.  p: (device) out [nk][V] int32.  ws: (device) caller
 * workspace of at least fcfs_debug_phases_workspace_size(V, T) bytes,
 * 256-byte aligned (else FCFS_ERR_WORKSPACE).  Only c->x, y, s, V and T are
 * read.  Asynchronous like every other call. */
fcfs_status fcfs_debug_phases_workspace_size(int64_t V, int32_t T, size_t *bytes);
fcfs_status fcfs_debug_phases(fcfs_handle *h, const fcfs_clip *c, int32_t axis, int32_t k0,
                              int32_t nk, int32_t *p, void *ws, size_t ws_bytes);

/* Times candidate tile shapes of the contraction on synthetic corners and
 * stores the fastest per (precision, K-bucket, V-bucket) in the handle, plus
 * the wave tile and corners per work item of the batched kernel; with
 * cache_path != NULL the table is also written there as JSON.  fcfs_create
 * reads such a file when the environment variable FCFS_AUTOTUNE_CACHE names
 * it; fcfs_load_tune reads one explicitly.  A missing or malformed cache
 * leaves the built-in choices.  effort: 0..2 (more shapes and sizes).
 * Synchronises the handle's stream. */
fcfs_status fcfs_autotune(fcfs_handle *h, const char *cache_path, int effort);

/* Reads an autotune cache written by fcfs_autotune (JSON) into the handle; a
 * missing or malformed file is refused (FCFS_ERR_INVALID_ARG) and the handle
 * keeps its choices. */
fcfs_status fcfs_load_tune(fcfs_handle *h, const char *cache_path);

/* The plan fcfs_forward makes for clip `c` at precision `p` with the automatic
 * tile choice (pointers in `c` are not read): vertex splits, corners per split,
 * frequency tiles, and the form: *direct = 1 when the one-launch direct form
 * runs instead, 2 when FCFS_AUTO takes the lattice form, else 0.  Any output
 * pointer may be NULL. */
fcfs_status fcfs_forward_plan_info(const fcfs_clip *c, fcfs_precision p, int32_t *nsplit,
                                   int64_t *chunk, int32_t *tiles, int32_t *direct);

/* Tuning and profiling hooks (forced tile variants, the batch autotuner,
 * per-kernel event timing) are declared in fcfs_tuning.h. */

const char *fcfs_status_string(fcfs_status s);
/* Detail of the last failing call on this handle (or of the last failing
 * handle-less call when h is NULL).  Never NULL. */
const char *fcfs_last_error(fcfs_handle *h);

#ifdef __cplusplus
}
#endif

#endif /* FCFS_H_ */
