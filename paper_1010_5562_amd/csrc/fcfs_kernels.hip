// HIP kernels of the FCFS forward path for gfx950 (MI355X).
//
// Steps (the four steps of Sec. III-C1, Alg. 2, evaluated directly on the
// corner list instead of through pruned FFTs):
//   pre-pass   exact phase reduction x mod T, y mod T; packing; area (Step 1)
//   axis       F[k,0], F[0,l] first-moment sums in FP64 (Steps 2 and 3)
//   contract   sum_v s_v e(k x_v) e(l y_v) as a real GEMM on MFMA (Step 4)
//   epilogue   split reduction, quadrant unfolding, alpha_{k,l} of Prop. 3,
//              Hermitian fill, axis and DC entries
#include "fcfs_device.h"

namespace fcfs {

// ---------------------------------------------------------------------------
// Pre-pass: pack corners, exact area.  Corners with index >= V (up to the
// padded count) become padding records.  The area sum is done modulo 2^64,
// which is exact whenever the true area fits in int64.  The same launch
// clears the axis histograms (the 2T bins in use) for the side-stream kernels
// that follow.
// ---------------------------------------------------------------------------
constexpr int kHistN = kTabN;  // bins per axis histogram (T <= 8192)

__device__ __forceinline__ void prepass_body(const int32_t *__restrict__ x,
                                             const int32_t *__restrict__ y,
                                             const int8_t *__restrict__ s, int64_t V, int64_t vpad,
                                             int T, int shift, uint4 *__restrict__ packed,
                                             unsigned long long *__restrict__ area_part,
                                             unsigned long long *__restrict__ hist, int blk,
                                             int nblk) {
  const uint32_t tmask = (uint32_t)(T - 1);
  unsigned long long acc = 0;
  for (int64_t i = (int64_t)blk * 256 + threadIdx.x; i < vpad; i += (int64_t)nblk * 256) {
    uint4 w;
    if (i < V) {
      const int32_t xv = x[i], yv = y[i];
      const int sv = s[i];
      w.x = (((uint32_t)xv & tmask) << shift) << 3;
      w.y = (((uint32_t)yv & tmask) << shift) << 3;
      w.z = sv < 0 ? kNegOff : 0u;
      w.w = 0u;
      acc += (unsigned long long)((long long)sv * (long long)xv * (long long)yv);
    } else {
      w = make_uint4(0u, 0u, 0u, kPadOff);
    }
    packed[i] = w;
  }
  if (hist)
    for (int i = blk * 256 + threadIdx.x; i < 2 * T; i += nblk * 256)
      hist[i < T ? i : kHistN + (i - T)] = 0ull;
  // fixed-order block reduction (integer, exact)
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  __shared__ unsigned long long red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) area_part[blk] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void k_prepass(const int32_t *__restrict__ x,
                                                 const int32_t *__restrict__ y,
                                                 const int8_t *__restrict__ s, int64_t V,
                                                 int64_t vpad, int T, int shift,
                                                 uint4 *__restrict__ packed,
                                                 unsigned long long *__restrict__ area_part,
                                                 unsigned long long *__restrict__ hist) {
  prepass_body(x, y, s, V, vpad, T, shift, packed, area_part, hist, blockIdx.x, gridDim.x);
}

hipError_t launch_prepass(const FwdPlan &p, const int32_t *x, const int32_t *y, const int8_t *s,
                          uint4 *packed, unsigned long long *area_part,
                          unsigned long long *hist, hipStream_t st) {
  hipLaunchKernelGGL(k_prepass, dim3(p.pre_blocks), dim3(256), 0, st, x, y, s, p.V, p.vpad, p.T,
                     p.shift, packed, area_part, hist);
  return hipGetLastError();
}

// General tile (periods Mx, My: any integers in [2, 8192], coordinates in
// units of the grid): records {x mod Mx, y mod My, sign mask, pad}.  The sign
// mask flips the sign bits of a y-side table entry (smask = 0x80008000 for the
// packed 16-bit split entries, 0x80000000 for FP32 pairs); padding records
// carry pad = 8 Mx, which sends the x-side lookup (an entry index or a byte
// offset, clamped to the zero entry) to the zero entry Mx.  Bins of the axis
// histograms are the residues themselves.
// Plans with a period past 8192 also write the corner words big_word (phi;
// nullptr otherwise).
__device__ __forceinline__ void gen_prepass_body(const int32_t *__restrict__ x,
                                                 const int32_t *__restrict__ y,
                                                 const int8_t *__restrict__ s, int64_t V,
                                                 int64_t vpad, int Mx, int My, uint32_t smask,
                                                 uint4 *__restrict__ packed,
                                                 unsigned long long *__restrict__ area_part,
                                                 unsigned long long *__restrict__ hist, int blk,
                                                 int nblk, uint4 *__restrict__ phi = nullptr) {
  unsigned long long acc = 0;
  for (int64_t i = (int64_t)blk * 256 + threadIdx.x; i < vpad; i += (int64_t)nblk * 256) {
    uint4 w;
    if (i < V) {
      const int32_t xv = x[i], yv = y[i];
      const int sv = s[i];
      const int xm = xv % Mx, ym = yv % My;
      w.x = (uint32_t)(xm < 0 ? xm + Mx : xm);
      w.y = (uint32_t)(ym < 0 ? ym + My : ym);
      w.z = sv < 0 ? smask : 0u;
      w.w = 0u;
      acc += (unsigned long long)((long long)sv * (long long)xv * (long long)yv);
    } else {
      w = make_uint4(0u, 0u, 0u, 8u * (uint32_t)Mx);
    }
    packed[i] = w;
    if (phi) phi[i] = big_word(w.x, w.y, (uint32_t)Mx, (uint32_t)My, w.z != 0u, w.w != 0u);
  }
  if (hist)
    for (int i = blk * 256 + threadIdx.x; i < Mx + My; i += nblk * 256)
      hist[i < Mx ? i : kHistN + (i - Mx)] = 0ull;
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  __shared__ unsigned long long red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) area_part[blk] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void k_gen_prepass(const int32_t *__restrict__ x,
                                                     const int32_t *__restrict__ y,
                                                     const int8_t *__restrict__ s, int64_t V,
                                                     int64_t vpad, int Mx, int My, uint32_t smask,
                                                     uint4 *__restrict__ packed,
                                                     unsigned long long *__restrict__ area_part,
                                                     unsigned long long *__restrict__ hist,
                                                     uint4 *__restrict__ phi) {
  gen_prepass_body(x, y, s, V, vpad, Mx, My, smask, packed, area_part, hist, blockIdx.x,
                   gridDim.x, phi);
}

hipError_t launch_gen_prepass(const FwdPlan &p, const int32_t *x, const int32_t *y,
                              const int8_t *s, uint32_t smask, void *ws, hipStream_t st) {
  char *w = (char *)ws;
  // the histograms (Mx + My bins, at most 2 x 8192) are not used by plans
  // with periods past 8192, which sum the axes over the corners and take the
  // phase magics instead
  hipLaunchKernelGGL(k_gen_prepass, dim3(p.pre_blocks), dim3(256), 0, st, x, y, s, p.V, p.vpad,
                     p.Mx, p.My, smask, (uint4 *)(w + p.off_packed),
                     (unsigned long long *)(w + p.off_area),
                     p.big ? nullptr : (unsigned long long *)(w + p.off_hist),
                     p.big ? (uint4 *)(w + p.off_phi) : nullptr);
  return hipGetLastError();
}

hipError_t launch_gen_prepass_records(const int32_t *x, const int32_t *y, const int8_t *s,
                                      int64_t V, int64_t vpad, int Mx, int My, int pre_blocks,
                                      uint4 *packed, unsigned long long *area_part,
                                      hipStream_t st) {
  hipLaunchKernelGGL(k_gen_prepass, dim3(pre_blocks), dim3(256), 0, st, x, y, s, V, vpad, Mx, My,
                     0x80008000u, packed, area_part, nullptr, nullptr);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Axis sums (Steps 2 and 3):
//   Sx[f] = sum_v s_v y_v e(f x_v), f = 1..K,   Sy[f] = sum_v s_v x_v e(f y_v), f = 1..L,
// taken, as in the paper's Steps 2 and 3, as 1-D DFTs of sparse images: the
// weights s_v y_v are binned by x_v mod T into Hx (the signed vertical edge
// lengths at each abscissa) and s_v x_v by y_v mod T into Hy, in exact int64
// arithmetic (the order of the atomic adds cannot change the result); then
//   Sx[f] = sum_{q < T} Hx[q] e(f q)
// in FP64.  Cost O(V + (K + L) T) instead of O(V (K + L)).
// ---------------------------------------------------------------------------

// Bins of one clip; hist = [Hx | Hy], kHistN int64 each, cleared beforehand.
// GEN: general-tile records (the residues are the bins).
template <bool GEN = false>
__device__ __forceinline__ void hist_body(const int32_t *__restrict__ x,
                                          const int32_t *__restrict__ y,
                                          const uint4 *__restrict__ packed, int64_t V, int shift,
                                          unsigned long long *__restrict__ hist, int blk,
                                          int nblk) {
  for (int64_t v = (int64_t)blk * 256 + threadIdx.x; v < V; v += (int64_t)nblk * 256) {
    const uint4 c = packed[v];
    const long long sg = c.z ? -1 : 1;
    const uint32_t qx = GEN ? c.x : (c.x >> 3) >> shift, qy = GEN ? c.y : (c.y >> 3) >> shift;
    atomicAdd(&hist[qx], (unsigned long long)(sg * (long long)y[v]));
    atomicAdd(&hist[kHistN + qy], (unsigned long long)(sg * (long long)x[v]));
  }
}

// Block (fb, chunk): 256 frequencies f = 1 + 256 fb' + t of one axis against
// the bins q in [chunk * kAxisBins, ...) < T.  e(f q) from the exact table at
// the first bin of every 32 and FP64 complex products in between.
// GEN: the axis has its own period (Mx or My) and table, and the table index
// is (f q) mod M; chunks past the axis's period write zero partials.
template <bool GEN = false>
__device__ __forceinline__ void dft_body(const unsigned long long *__restrict__ hist,
                                         const double2 *__restrict__ w64, int T, int shift, int K,
                                         int L, int fb_k, double2 *__restrict__ axis_part, int fb,
                                         int chunk, const double2 *__restrict__ w64y = nullptr,
                                         int My = 0) {
  __shared__ double s_h[kAxisBins];
  const bool xaxis = fb < fb_k;
  const int f = 1 + (xaxis ? fb : fb - fb_k) * 256 + threadIdx.x;
  const int nf = xaxis ? K : L;
  const unsigned long long *H = hist + (xaxis ? 0 : kHistN);
  const int M = GEN && !xaxis ? My : T;
  const double2 *W = GEN && !xaxis ? w64y : w64;
  const int q0 = chunk * kAxisBins;
  const int n = max(0, min(kAxisBins, M - q0));
  for (int i = threadIdx.x; i < n; i += 256) s_h[i] = (double)(long long)H[q0 + i];
  __syncthreads();
  double re = 0.0, im = 0.0;
  const uint32_t uf = (uint32_t)f, mask = (uint32_t)(kTabN - 1);
  const uint32_t um = (uint32_t)M, fr = GEN ? uf % um : 0u;
  const double2 w1 = GEN ? W[fr] : W[(uf << shift) & mask];
  double2 w = make_double2(1.0, 0.0);
  for (int i = 0; i < n; ++i) {
    if ((i & 31) == 0)
      w = GEN ? W[(fr * (uint32_t)(q0 + i)) % um] : W[((uf * (uint32_t)(q0 + i)) << shift) & mask];
    const double h = s_h[i];
    re = fma(h, w.x, re);  // e(f q) = conj(w)
    im = fma(-h, w.y, im);
    const double nx = w.x * w1.x - w.y * w1.y, ny = w.x * w1.y + w.y * w1.x;
    w = make_double2(nx, ny);
  }
  if (f <= nf) {
    const int slot = xaxis ? f - 1 : K + f - 1;
    axis_part[(size_t)chunk * (K + L) + slot] = make_double2(re, im);
  }
}

__global__ __launch_bounds__(256) void k_axis_dft(const unsigned long long *__restrict__ hist,
                                                  const double2 *__restrict__ w64, int T, int shift,
                                                  int K, int L, int fb_k,
                                                  double2 *__restrict__ axis_part) {
  dft_body(hist, w64, T, shift, K, L, fb_k, axis_part, blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------------------
// FP64 guard region: S(k, l) = sum_v s_v e(k x_v) e(l y_v) in FP64 for the
// 8 x 8 frequency blocks of the guard region (the core block k, l = 1..8 and,
// for a span n > 1, the strips next to the axes), replacing the MFMA values
// there.  The 1/(k l) factor of alpha_{k,l} amplifies the rounding of the
// contraction most at these frequencies.  The span follows from a rounding
// model of the split forms and the exact area (guard_span): clips of high
// fill keep the core block alone, clips of low fill widen the strips.
// Each block is the same real-trigonometric GEMM as the contraction,
// restricted to 16 x 16 and run on the FP64 matrix cores: rows a_i =
// cos(k_i th_x) for i < 8 and sin(k_{i-8} th_x) for i >= 8 (the block's 8 k),
// columns b_j likewise in th_y with the sign s_v.
// v_mfma_f64_16x16x4_f64 takes 4 corners per instruction: lane i + 16 q holds
// A[i][q] = a_i(v_q) and B[q][i] = s b_i(v_q); D[i][j] is element i / 4 of
// lane j + 16 (i % 4).
// A lane reads (cos, sin) of its frequency f = 1..8 and of 8 th for both
// coordinates from the FP64 table (exact integer phases); the strip blocks
// step from one block to the next by the angle-addition rotation through
// 8 th in FP64 (at most kGuardSpanMax - 1 steps, a few ulp).
// Each 256-thread block reduces its corner range to one 16 x 16 partial per
// slot in use, in a fixed order; the epilogue adds the ranges in order, so the
// result does not depend on scheduling.
// ---------------------------------------------------------------------------
// Corner groups in flight per wave: the side kernel has to fit in the
// registers the one-wave-per-SIMD contraction leaves free (about 88 per lane)
// to run beside it.
constexpr int kGuardUnroll = 8;     // one block per corner range
constexpr int kGuardUnrollRot = 1;  // several blocks (rotations)
typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double2 rot(double2 v, double2 r) {
  return make_double2(v.x * r.x - v.y * r.y, v.y * r.x + v.x * r.y);
}

// Span of the guard region (block-uniform) from the exact area partials,
// limited to the strips that reach into |k| <= K or |l| <= L; a split-bf16
// clip routed to split-fp16 (gscale_alt > 0) sizes it with the fp16 factor.
__device__ __forceinline__ int guard_span_block(const unsigned long long *__restrict__ area_part,
                                                int pre_blocks, int64_t V, double gscale,
                                                double gscale_alt, int K, int L) {
  const long long a = block_area(area_part, pre_blocks);
  const int nmax = (max(K, L) + kGuard - 1) / kGuard;
  return max(1, min(guard_span_routed(gscale, gscale_alt, V, a), nmax));
}

// Phases of a guard lane's three frequencies (its row fx, its column fy and
// the 8-step of the rotations) against a corner.  GEN: general-tile records
// (residues; one-level periods reduced with lane magics, gen_phase).  BIG:
// corner words of a two-level clip (big_word_phase; NARROW as big_narrow).
template <bool GEN, bool BIG, bool NARROW>
struct GuardPhases {
  uint32_t fx, fy, rx, ry, r8x, r8y, mx, my, m8x, m8y;
  __device__ __forceinline__ GuardPhases(uint32_t fx_, uint32_t fy_, uint32_t Mx, uint32_t My)
      : fx(fx_), fy(fy_) {
    if constexpr (GEN && !BIG) {
      rx = fx % Mx;
      ry = fy % My;
      r8x = 8u % Mx;
      r8y = 8u % My;
      mx = gen_magic(rx, Mx);
      my = gen_magic(ry, My);
      m8x = gen_magic(r8x, Mx);
      m8y = gen_magic(r8y, My);
    }
  }
  // (f x) mod Mx for f = fx (or 8 when EIGHT), from record/word c
  template <bool EIGHT>
  __device__ __forceinline__ uint32_t px(const uint4 &c, uint32_t Mx) const {
    if constexpr (BIG)
      return big_word_phase<NARROW, true>(EIGHT ? 8u : fx, c, Mx - 1u, -(int)Mx);
    else
      return EIGHT ? gen_phase(r8x, m8x, c.x, Mx) : gen_phase(rx, mx, c.x, Mx);
  }
  template <bool EIGHT>
  __device__ __forceinline__ uint32_t py(const uint4 &c, uint32_t My) const {
    if constexpr (BIG)
      return big_word_phase<NARROW, false>(EIGHT ? 8u : fy, c, My - 1u, -(int)My);
    else
      return EIGHT ? gen_phase(r8y, m8y, c.y, My) : gen_phase(ry, my, c.y, My);
  }
  // the corner's sign is -1
  __device__ __forceinline__ bool neg(const uint4 &c) const {
    if constexpr (BIG)
      return (c.z >> 30) & 1u;
    else
      return c.z != 0u;
  }
};

// Slot group gi of the guard region over corner range blk (guard_group).
// The group's blocks share one side: the l-strip groups keep the row
// frequencies k = 1..8 and step the columns along l, the k-strip groups keep
// l = 1..8 and step the rows along k.
// GEN: general-tile records (residues); x phases (f x) mod Mx index wx, y
// phases wy (BIG: the corner words of a two-level clip in place of the
// records, two-level tables with nhx, nhy entries of Whi).  Otherwise
// byte-offset records and the one table wx.  UR: corners in flight per lane
// on the rotation path.
template <bool GEN = false, bool BIG = false, bool NARROW = false, int UR = kGuardUnrollRot>
__device__ __forceinline__ void guard_body(const uint4 *__restrict__ packed,
                                           const double2 *__restrict__ wx, int64_t V,
                                           int64_t g_chunk, int blk, int gi,
                                           const unsigned long long *__restrict__ area_part,
                                           int pre_blocks, double gscale, double gscale_alt,
                                           int K, int L, double *__restrict__ gpart,
                                           unsigned int *__restrict__ gspan,
                                           const double2 *__restrict__ wy = nullptr, int Mx = 0,
                                           int My = 0, int nhx = 0, int nhy = 0) {
  __shared__ double red[4][kGuardD];
  const int n =
      __builtin_amdgcn_readfirstlane(guard_span_block(area_part, pre_blocks, V, gscale, gscale_alt, K, L));
  if (blk == 0 && gi == 0 && threadIdx.x == 0) *gspan = (unsigned int)n;
  const GuardGroup gg = guard_group(gi, n);
  const int ns = gg.ns;  // slots of the group in use (block-uniform)
  if (ns == 0) return;
  const bool ymove = gg.ymove != 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, q = lane >> 4;
  const uint32_t f = (uint32_t)(i & 7) + 1u;
  const uint32_t fx = f + (uint32_t)(kGuard * gg.kb);
  const uint32_t fy = f + (uint32_t)(kGuard * gg.lb);
  const bool sn = i >= 8;  // sin row / column
  const GuardPhases<GEN, BIG, NARROW> ph(fx, fy, (uint32_t)Mx, (uint32_t)My);
  const int64_t v0 = (int64_t)blk * g_chunk;
  const int64_t v1 = min(V, v0 + g_chunk);
  f64x4 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = f64x4{0.0, 0.0, 0.0, 0.0};
  if (ns == 1) {
    // one block: each lane reads only the entry it feeds (cos or sin)
    for (int64_t base = v0 + 4 * wave; base < v1; base += 16 * kGuardUnroll) {
      double ea[kGuardUnroll], eb[kGuardUnroll];
#pragma unroll
      for (int u = 0; u < kGuardUnroll; ++u) {
        const int64_t v = base + 16 * u + q;
        ea[u] = eb[u] = 0.0;
        if (v < v1) {
          const uint4 c = packed[v];
          if constexpr (BIG) {
            const double2 wa = big_entry64(wx, nhx, ph.template px<false>(c, Mx));
            const double2 wb = big_entry64(wy, nhy, ph.template py<false>(c, My));
            ea[u] = sn ? wa.y : wa.x;
            const double tb = sn ? wb.y : wb.x;
            eb[u] = ph.neg(c) ? -tb : tb;
          } else {
            uint32_t px, py;
            if constexpr (GEN) {
              px = ph.template px<false>(c, Mx);
              py = ph.template py<false>(c, My);
            } else {
              px = __umul24(fx, c.x >> 3) & (uint32_t)(kTabN - 1);
              py = __umul24(fy, c.y >> 3) & (uint32_t)(kTabN - 1);
            }
            const double *tx = (const double *)wx, *ty = (const double *)(GEN ? wy : wx);
            ea[u] = tx[2 * px + (sn ? 1 : 0)];
            const double tb = ty[2 * py + (sn ? 1 : 0)];
            eb[u] = c.z ? -tb : tb;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kGuardUnroll; ++u)
        acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(ea[u], eb[u], acc[0], 0, 0, 0);
    }
  } else {
    // several blocks: (cos, sin) of the first and of the 8-step, rotated
    for (int64_t base = v0 + 4 * wave; base < v1; base += 16 * UR) {
      double2 ex[UR], ey[UR], e8[UR];
      bool ng[UR];
#pragma unroll
      for (int u = 0; u < UR; ++u) {
        const int64_t v = base + 16 * u + q;
        ex[u] = ey[u] = make_double2(0.0, 0.0);
        e8[u] = make_double2(1.0, 0.0);
        ng[u] = false;
        if (v < v1) {
          const uint4 c = packed[v];
          ng[u] = ph.neg(c);
          if constexpr (BIG) {
            ex[u] = big_entry64(wx, nhx, ph.template px<false>(c, Mx));
            ey[u] = big_entry64(wy, nhy, ph.template py<false>(c, My));
            e8[u] = ymove ? big_entry64(wy, nhy, ph.template py<true>(c, My))
                          : big_entry64(wx, nhx, ph.template px<true>(c, Mx));
          } else {
            uint32_t px, py, p8;
            if constexpr (GEN) {
              px = ph.template px<false>(c, Mx);
              py = ph.template py<false>(c, My);
              p8 = ymove ? ph.template py<true>(c, My) : ph.template px<true>(c, Mx);
            } else {
              const uint32_t xs = c.x >> 3, ys = c.y >> 3;
              px = __umul24(fx, xs) & (uint32_t)(kTabN - 1);
              py = __umul24(fy, ys) & (uint32_t)(kTabN - 1);
              p8 = (8u * (ymove ? ys : xs)) & (uint32_t)(kTabN - 1);
            }
            ex[u] = wx[px];
            ey[u] = GEN ? wy[py] : wx[py];
            e8[u] = (GEN && ymove) ? wy[p8] : wx[p8];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < UR; ++u) {
        double2 a = ex[u], b = ng[u] ? make_double2(-ey[u].x, -ey[u].y) : ey[u];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (j < ns) {
            if (j > 0) {
              if (ymove)
                b = rot(b, e8[u]);
              else
                a = rot(a, e8[u]);
            }
            acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(sn ? a.y : a.x, sn ? b.y : b.x, acc[j],
                                                          0, 0, 0);
          }
      }
    }
  }
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (j >= ns) break;
    const int slot = gg.slot + j;
#pragma unroll
    for (int r = 0; r < 4; ++r) red[wave][(q + 4 * r) * 16 + i] = acc[j][r];
    __syncthreads();
    gpart[((size_t)blk * kGuardSlots + slot) * kGuardD + t] =
        ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
    __syncthreads();
  }
}

// Side-stream kernel of one clip: blocks [0, nh) bin the axis histograms,
// blocks [nh, nh + kGuardGroups g_chunks) compute the guard region (slot
// group b / g_chunks over corner range b % g_chunks: the core group first).
// At most 80 registers per lane (six workgroups per CU), so that its blocks
// fit beside the contraction: the interleaved kernel holds 424, two
// workgroups of the two-waves-per-SIMD kernel 432.
__global__ __launch_bounds__(256, 6) void k_side(const int32_t *__restrict__ x,
                                              const int32_t *__restrict__ y,
                                              const uint4 *__restrict__ packed, int64_t V,
                                              int shift, unsigned long long *__restrict__ hist,
                                              int nh, const double2 *__restrict__ w64,
                                              int64_t g_chunk, int g_chunks,
                                              const unsigned long long *__restrict__ area_part,
                                              int pre_blocks, double gscale, double gscale_alt,
                                              int K, int L, double *__restrict__ gpart,
                                              unsigned int *__restrict__ gspan) {
  if ((int)blockIdx.x < nh)
    hist_body(x, y, packed, V, shift, hist, blockIdx.x, nh);
  else
    guard_body(packed, w64, V, g_chunk, (blockIdx.x - nh) % g_chunks,
               (blockIdx.x - nh) / g_chunks, area_part, pre_blocks, gscale, gscale_alt, K, L,
               gpart, gspan);
}

// Adds the guard partials of every used slot over the corner ranges into
// range 0, in place.  A block takes 64 entries of one slot; wave w sums the
// w-th quarter of the ranges in range order from an FP64 zero and the four
// sums are added in wave order (a fixed order; four times shorter chains of
// dependent loads than one thread per entry).  It runs at the end of the side
// stream beside the contraction, so the epilogue reads one range.
__global__ __launch_bounds__(256, 6) void k_guard_fold(double *__restrict__ gpart, int g_chunks,
                                                       const unsigned int *__restrict__ gspan) {
  const int j = blockIdx.x;
  if (!guard_slot_used(j, (int)*gspan)) return;
  __shared__ double red[3][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double *e = gpart + (size_t)j * kGuardD + blockIdx.y * 64 + lane;
  const int q = (g_chunks + 3) / 4, c0 = w * q, c1 = min(g_chunks, c0 + q);
  double sum = 0.0;
#pragma unroll 16
  for (int c = c0; c < c1; ++c) sum += e[(size_t)c * kGuardSlots * kGuardD];
  if (w > 0) red[w - 1][lane] = sum;
  __syncthreads();
  // only wave 0 reads range 0, and it writes after its own reads
  if (w == 0) e[0] = ((sum + red[0][lane]) + red[1][lane]) + red[2][lane];
}

// The fold pays where the contraction hides the side stream (large frequency
// blocks); beside a short contraction (a low-pass band) the side stream is
// the longer path and the epilogue keeps the sum (0.184 -> 0.188 ms per
// differentiation step with the fold there, same box).
bool guard_folded(const FwdPlan &p) {
  return p.K > 0 && p.L > 0 && (int64_t)(p.K + 1) * (p.L + 1) >= 128 * 128;
}

void launch_guard_fold(const FwdPlan &p, void *ws, hipStream_t st) {
  char *w = (char *)ws;
  static_assert(kGuardD % 64 == 0, "64 entries per fold block");
  hipLaunchKernelGGL(k_guard_fold, dim3(kGuardSlots, kGuardD / 64), dim3(256), 0, st,
                     (double *)(w + p.off_guard), p.g_chunks,
                     (const unsigned int *)(w + p.off_gspan));
}

hipError_t launch_side(const FwdPlan &p, const int32_t *x, const int32_t *y, const double2 *w64,
                       void *ws, hipStream_t st, bool guard) {
  char *w = (char *)ws;
  const uint4 *packed = (const uint4 *)(w + p.off_packed);
  auto *hist = (unsigned long long *)(w + p.off_hist);
  const int nh = p.K + p.L > 0 ? p.hist_blocks : 0;
  const int ng = guard && p.K > 0 && p.L > 0 ? kGuardGroups * p.g_chunks : 0;
  if (nh + ng > 0)
    hipLaunchKernelGGL(k_side, dim3(nh + ng), dim3(256), 0, st, x, y, packed, p.V, p.shift, hist,
                       nh, w64, p.g_chunk, p.g_chunks, (const unsigned long long *)(w + p.off_area),
                       p.pre_blocks, p.gscale, p.gscale_alt, p.K, p.L, (double *)(w + p.off_guard),
                       (unsigned int *)(w + p.off_gspan));
  if (ng > 0 && guard_folded(p)) launch_guard_fold(p, ws, st);
  if (p.K + p.L > 0)
    hipLaunchKernelGGL(k_axis_dft, dim3(p.ax_fb_k + p.ax_fb_l, p.ax_chunks), dim3(256), 0, st,
                       hist, w64, p.T, p.shift, p.K, p.L, p.ax_fb_k,
                       (double2 *)(w + p.off_axis));
  return hipGetLastError();
}

// General-tile side-stream work: histogram blocks, guard blocks, then the
// axis DFTs of both periods.  Sized for six workgroups per CU (at most 80
// registers per lane): the pipelined general contraction holds 432 of the
// 512, so the side blocks can run beside it rather than after it.
__global__ __launch_bounds__(256, 6) void k_gen_side(const int32_t *__restrict__ x,
                                                  const int32_t *__restrict__ y,
                                                  const uint4 *__restrict__ packed, int64_t V,
                                                  unsigned long long *__restrict__ hist, int nh,
                                                  const double2 *__restrict__ wx,
                                                  const double2 *__restrict__ wy, int Mx, int My,
                                                  int64_t g_chunk, int g_chunks,
                                                  const unsigned long long *__restrict__ area_part,
                                                  int pre_blocks, double gscale,
                                                  double gscale_alt, int K, int L,
                                                  double *__restrict__ gpart,
                                                  unsigned int *__restrict__ gspan) {
  if ((int)blockIdx.x < nh)
    hist_body<true>(x, y, packed, V, 0, hist, blockIdx.x, nh);
  else
    guard_body<true>(packed, wx, V, g_chunk, (blockIdx.x - nh) % g_chunks,
                     (blockIdx.x - nh) / g_chunks, area_part, pre_blocks, gscale, gscale_alt, K,
                     L, gpart, gspan, wy, Mx, My);
}

__global__ __launch_bounds__(256) void k_gen_axis_dft(const unsigned long long *__restrict__ hist,
                                                      const double2 *__restrict__ wx,
                                                      const double2 *__restrict__ wy, int Mx,
                                                      int My, int K, int L, int fb_k,
                                                      double2 *__restrict__ axis_part) {
  dft_body<true>(hist, wx, Mx, 0, K, L, fb_k, axis_part, blockIdx.x, blockIdx.y, wy, My);
}

// Periods past 8192 (two-level tables): the guard blocks alone, over the
// corner words.
__global__ __launch_bounds__(256) void k_gen_side_big(
    const uint4 *__restrict__ words, int64_t V, const double2 *__restrict__ wx,
    const double2 *__restrict__ wy, int Mx, int My, int nhx, int nhy, int64_t g_chunk,
    int g_chunks, const unsigned long long *__restrict__ area_part, int pre_blocks, double gscale,
    double gscale_alt, int K, int L, double *__restrict__ gpart, unsigned int *__restrict__ gspan) {
  if (big_narrow(Mx, My))
    guard_body<true, true, true>(words, wx, V, g_chunk, blockIdx.x % g_chunks,
                                 blockIdx.x / g_chunks, area_part, pre_blocks, gscale, gscale_alt,
                                 K, L, gpart, gspan, wy, Mx, My, nhx, nhy);
  else
    guard_body<true, true, false>(words, wx, V, g_chunk, blockIdx.x % g_chunks,
                                  blockIdx.x / g_chunks, area_part, pre_blocks, gscale,
                                  gscale_alt, K, L, gpart, gspan, wy, Mx, My, nhx, nhy);
}

// Axis sums (Steps 2 and 3) over the corners directly, for periods past 8192
// where a histogram over the residues would be too large: block (fb, chunk)
// takes nb = axis_big_freqs(K, L) frequencies f = f0 + 1 + i of one axis
// against the corners of its range,
//   Sx[f] += sum_v s_v y_v e^{-j 2 pi f x_v / Mx},  Sy[f] += sum_v s_v x_v e^{-j 2 pi f y_v / My},
// raw coordinates as the moments.  With i = 16 a + b (a < na = nb / 16,
// b < 16) the twiddle factors as e((f0 + 1 + 16 a) x / M) e(b x / M).  Per
// step of 64 corners, four threads per corner build its na factors
// m_v e((f0 + 1 + 16 a) x) and 16 factors e(b x) in FP64 from four table
// lookups (exact phases of 1, 4 q, 16 and f0 + 1 + 4 na q times x from the
// corner word, big_word_phase, and the two-level FP64 table) and short
// products (a factor of e(x) or e(16 x) at most seven times: a few units in
// the last place).  Thread t then adds the 4 x 4 frequencies of its group
// t mod na over every (256 / na)-th corner (group t / na), one complex
// multiply-add each, and the corner groups are added in a fixed order at the
// end.  The same per-chunk partials as k_gen_axis_dft, reduced by the
// epilogue.
constexpr int kAxisBigStep = 64;  // corners per LDS step
constexpr int kAxisBigLds = 4096;  // double2 entries
static_assert(kAxisBigStep * 48 <= kAxisBigLds, "factor area");
template <bool NARROW>
__device__ __forceinline__ void gen_axis_big_body(
    const int32_t *__restrict__ x, const int32_t *__restrict__ y, const uint4 *__restrict__ words,
    int64_t V, int64_t ax_chunk, const double2 *__restrict__ wx, const double2 *__restrict__ wy,
    int Mx, int My, int nhx, int nhy, int K, int L, int fb_k, double2 *__restrict__ axis_part,
    int fb, int chunk, double2 *abuf) {
  // abuf (LDS, kAxisBigLds entries): the factors of a step, [j][32] a side,
  // then [j][16] b side; at the end the partials of the corner groups,
  // [group][16 a + b] (256 / na groups of 16 na: always 4096)
  double2 *fa = abuf, *fbv = abuf + kAxisBigStep * 32;
  const int nb = axis_big_freqs(K, L), na = nb >> 4, nq = na >> 2, ncg = 256 / na;
  const int t = threadIdx.x;
  const bool xaxis = fb < fb_k;
  const int f0 = (xaxis ? fb : fb - fb_k) * nb;
  const int nf = xaxis ? K : L;
  const double2 *W = xaxis ? wx : wy;
  const int nh = xaxis ? nhx : nhy;
  const uint32_t M = (uint32_t)(xaxis ? Mx : My);
  const int64_t v0 = (int64_t)chunk * ax_chunk, v1 = min(V, v0 + ax_chunk);
  const int jf = t >> 2, q = t & 3;  // factor stage: corner, quarter
  const int g = t % na, cg = t / na, a0 = 4 * (g >> 2), b0 = 4 * (g & 3);
  auto entry = [&](uint32_t f, const uint4 &c) {
    const uint32_t p = xaxis ? big_word_phase<NARROW, true>(f, c, M - 1u, -(int)M)
                             : big_word_phase<NARROW, false>(f, c, M - 1u, -(int)M);
    return big_entry64(W, nh, p);
  };
  auto cmul = [](const double2 &u, const double2 &v) {
    return make_double2(fma(u.x, v.x, -u.y * v.y), fma(u.x, v.y, u.y * v.x));
  };
  double accr[4][4], acci[4][4];
#pragma unroll
  for (int ia = 0; ia < 4; ++ia)
#pragma unroll
    for (int ib = 0; ib < 4; ++ib) accr[ia][ib] = acci[ia][ib] = 0.0;
  for (int64_t base = v0; base < v1; base += kAxisBigStep) {
    const int n = (int)min((int64_t)kAxisBigStep, v1 - base);
    __syncthreads();  // the previous step's factors are consumed
    {
      double2 e1 = make_double2(0.0, 0.0), eb = e1, e16 = e1, ea = e1;
      double m = 0.0;
      if (jf < n) {
        const int64_t v = base + jf;
        const uint4 c = words[v];
        e1 = entry(1u, c);
        eb = q ? entry(4u * (uint32_t)q, c) : make_double2(1.0, 0.0);
        e16 = entry(16u, c);
        ea = entry((uint32_t)(f0 + 1 + 16 * nq * q), c);
        const double r = (double)(xaxis ? y[v] : x[v]);
        m = (c.z >> 30) & 1u ? -r : r;
      }
      double2 w = eb;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        fbv[jf * 16 + 4 * q + i] = w;
        w = cmul(w, e1);
      }
      w = make_double2(m * ea.x, m * ea.y);
      for (int i = 0; i < nq; ++i) {
        fa[jf * 32 + nq * q + i] = w;
        w = cmul(w, e16);
      }
    }
    __syncthreads();
    for (int j = cg; j < n; j += ncg) {
      double2 A[4], B[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        A[i] = fa[j * 32 + a0 + i];
        B[i] = fbv[j * 16 + b0 + i];
      }
#pragma unroll
      for (int ia = 0; ia < 4; ++ia)
#pragma unroll
        for (int ib = 0; ib < 4; ++ib) {
          accr[ia][ib] = fma(A[ia].x, B[ib].x, fma(-A[ia].y, B[ib].y, accr[ia][ib]));
          acci[ia][ib] = fma(A[ia].x, B[ib].y, fma(A[ia].y, B[ib].x, acci[ia][ib]));
        }
    }
  }
  __syncthreads();
#pragma unroll
  for (int ia = 0; ia < 4; ++ia)
#pragma unroll
    for (int ib = 0; ib < 4; ++ib)
      abuf[cg * nb + 16 * (a0 + ia) + b0 + ib] = make_double2(accr[ia][ib], acci[ia][ib]);
  __syncthreads();
  for (int fl = t; fl < nb; fl += 256) {
    const int f = f0 + 1 + fl;
    if (f > nf) continue;
    double re = 0.0, im = 0.0;
    for (int k = 0; k < ncg; ++k) {
      re += abuf[k * nb + fl].x;
      im += abuf[k * nb + fl].y;
    }
    // W holds e^{+j theta}: the sum wanted is the conjugate
    axis_part[(size_t)chunk * (K + L) + (xaxis ? f - 1 : K + f - 1)] = make_double2(re, -im);
  }
}

__global__ __launch_bounds__(256) void k_gen_axis_big(
    const int32_t *__restrict__ x, const int32_t *__restrict__ y, const uint4 *__restrict__ words,
    int64_t V, int64_t ax_chunk, const double2 *__restrict__ wx, const double2 *__restrict__ wy,
    int Mx, int My, int nhx, int nhy, int K, int L, int fb_k, double2 *__restrict__ axis_part) {
  __shared__ double2 abuf[kAxisBigLds];
  if (big_narrow(Mx, My))
    gen_axis_big_body<true>(x, y, words, V, ax_chunk, wx, wy, Mx, My, nhx, nhy, K, L, fb_k,
                            axis_part, blockIdx.x, blockIdx.y, abuf);
  else
    gen_axis_big_body<false>(x, y, words, V, ax_chunk, wx, wy, Mx, My, nhx, nhy, K, L, fb_k,
                             axis_part, blockIdx.x, blockIdx.y, abuf);
}

hipError_t launch_gen_side(const FwdPlan &p, const int32_t *x, const int32_t *y,
                           const double2 *wx, const double2 *wy, void *ws, hipStream_t st) {
  char *w = (char *)ws;
  const uint4 *packed = (const uint4 *)(w + p.off_packed);
  if (p.big) {
    const uint4 *words = (const uint4 *)(w + p.off_phi);
    if (p.K > 0 && p.L > 0)
      hipLaunchKernelGGL(k_gen_side_big, dim3(kGuardGroups * p.g_chunks), dim3(256), 0, st, words,
                         p.V, wx, wy, p.Mx, p.My, p.nhx, p.nhy, p.g_chunk, p.g_chunks,
                         (const unsigned long long *)(w + p.off_area), p.pre_blocks, p.gscale,
                         p.gscale_alt, p.K, p.L, (double *)(w + p.off_guard),
                         (unsigned int *)(w + p.off_gspan));
    if (guard_folded(p)) launch_guard_fold(p, ws, st);
    if (p.K + p.L > 0) {
      const int64_t ax_chunk = std::max<int64_t>(1, (p.V + p.ax_chunks - 1) / p.ax_chunks);
      hipLaunchKernelGGL(k_gen_axis_big, dim3(p.ax_fb_k + p.ax_fb_l, p.ax_chunks), dim3(256), 0,
                         st, x, y, words, p.V, ax_chunk, wx, wy, p.Mx, p.My, p.nhx, p.nhy, p.K,
                         p.L, p.ax_fb_k, (double2 *)(w + p.off_axis));
    }
    return hipGetLastError();
  }
  auto *hist = (unsigned long long *)(w + p.off_hist);
  const int nh = p.K + p.L > 0 ? p.hist_blocks : 0;
  const int ng = p.K > 0 && p.L > 0 ? kGuardGroups * p.g_chunks : 0;
  if (nh + ng > 0)
    hipLaunchKernelGGL(k_gen_side, dim3(nh + ng), dim3(256), 0, st, x, y, packed, p.V, hist, nh,
                       wx, wy, p.Mx, p.My, p.g_chunk, p.g_chunks,
                       (const unsigned long long *)(w + p.off_area),
                       p.pre_blocks, p.gscale, p.gscale_alt, p.K, p.L, (double *)(w + p.off_guard),
                       (unsigned int *)(w + p.off_gspan));
  if (ng > 0 && guard_folded(p)) launch_guard_fold(p, ws, st);
  if (p.K + p.L > 0)
    hipLaunchKernelGGL(k_gen_axis_dft, dim3(p.ax_fb_k + p.ax_fb_l, p.ax_chunks), dim3(256), 0, st,
                       hist, wx, wy, p.Mx, p.My, p.K, p.L, p.ax_fb_k, (double2 *)(w + p.off_axis));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Direct store of a clip contracted in one split (batch form, two-wave-per-SIMD
// kernels): the work item unfolds its accumulators into F itself, as the
// epilogue would (the sum over one split is that split, added to an FP64 zero
// in the same way), so no quadrant partials are written or read back.  The
// core guard block's entries are left to the epilogue, which writes them from
// the FP64 sums; it overwrites the entries of wider guard strips after this
// kernel.  The one-wave-per-SIMD kernel keeps writing partials: with its
// 256 accumulators the unfolding does not fit beside them without spills.
// ---------------------------------------------------------------------------
struct DirectOut {
  OutGrid o;
  int K, L;
  int on;  // 0: this clip writes partials
};

// Output of a batch clip for the direct store (on when it has one split).
__device__ __forceinline__ DirectOut direct_out(const BatchClip &c) {
  return DirectOut{OutGrid{c.F, c.K, c.L, -1.0, (double)c.T, 1.0, 1.0, 1.0 / (double)c.T}, c.K,
                   c.L, c.direct};
}

template <int NKB, int NLB>
__device__ __forceinline__ void store_direct(const DirectOut &d, const f32x16 (&acc)[NKB][NLB][4],
                                             int k0, int l0, int li, int lh) {
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
    for (int lb = 0; lb < NLB; ++lb) {
      const int l = l0 + 32 * lb + li;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int k = k0 + 32 * kb + 8 * (r >> 2) + 4 * lh + (r & 3);
        if (k < 1 || k > d.K || l < 1 || l > d.L || (k <= kGuard && l <= kGuard)) continue;
        store_quad(d.o, k, l, 0.0, 0.0 + (double)acc[kb][lb][0][r],
                   0.0 + (double)acc[kb][lb][1][r], 0.0 + (double)acc[kb][lb][2][r],
                   0.0 + (double)acc[kb][lb][3][r]);
      }
    }
}

// ---------------------------------------------------------------------------
// Vertex contraction (Step 4) in real-trigonometric form:
//   Z = X diag(s) Y^T,  X = [cos; sin](2 pi k x_v / T), Y likewise in l,
// giving per (k, l >= 0) the four sums P = sum s c c', U = sum s c s',
// R = sum s s c', Q = sum s s s'.  Each workgroup (4 waves, 2 x 2) owns a tile
// of frequencies and one split of the vertices; each wave owns 32*NKB k's by
// 32*NLB l's.  The twiddle table sits in LDS; the X and Y operand fragments
// are gathered from it with exact integer phases, the sign s_v is folded into
// the y phase, and the products run on MFMA with FP32 accumulation.
// Output: part[split][q][kp][lp], q = 0:P 1:U 2:R 3:Q.
// 32x32 accumulator layout: element r of lane (i = lane&31, h = lane>>5) is
// row 8*(r/4) + 4*h + (r%4), column i.
// ---------------------------------------------------------------------------
template <int NKB, int NLB>
__device__ __forceinline__ void gather(Raw<NKB, NLB> &r, const uint2 *s_tab, const uint4 (&c)[8],
                                       const uint32_t (&kf)[NKB], const uint32_t (&lf)[NLB]) {
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
    for (int j = 0; j < 8; ++j) r.a[kb][j] = lds_entry(s_tab, phase_x(kf[kb], c[j]));
#pragma unroll
  for (int lb = 0; lb < NLB; ++lb)
#pragma unroll
    for (int j = 0; j < 8; ++j) r.b[lb][j] = lds_entry(s_tab, phase_y(lf[lb], c[j]));
}

// Split (hi + lo) contraction.  Software pipeline per 16-corner step s:
// the table lookups of step s+1 are in flight and the corners of step s+2 are
// being loaded while the MFMAs of step s run; operand fragments are double
// buffered (two unrolled half-iterations swap their roles).
template <int PREC, int NKB, int NLB>
__device__ __forceinline__ void contract_split_body(const uint2 *s_tab,
                                                    const uint4 *__restrict__ packed,
                                                    int64_t chunk, int tiles_l, int kp, int lp,
                                                    float *__restrict__ part) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 31, lh = lane >> 5;
  const int tk = blockIdx.x / tiles_l, tl = blockIdx.x % tiles_l;
  const int split = blockIdx.y;
  const int k0 = tk * (64 * NKB) + (wave >> 1) * (32 * NKB);
  const int l0 = tl * (64 * NLB) + (wave & 1) * (32 * NLB);

  uint32_t kf[NKB], lf[NLB];
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb) kf[kb] = (uint32_t)(k0 + 32 * kb + li);
#pragma unroll
  for (int lb = 0; lb < NLB; ++lb) lf[lb] = (uint32_t)(l0 + 32 * lb + li);

  f32x16 acc[NKB][NLB][4];
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
    for (int lb = 0; lb < NLB; ++lb)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[kb][lb][q][r] = 0.0f;

  // corners of step s for this lane: vp + 16 s + j
  const uint4 *vp = packed + (size_t)split * chunk + 8 * lh;
  const int nsteps = (int)(chunk >> 4);
  uint4 c[8];
  Raw<NKB, NLB> raw;
  Frag<NKB, NLB> f0, f1;
  load_corners(c, vp);
  gather(raw, s_tab, c, kf, lf);
  build(f0, raw);
  if (nsteps > 1) {
    load_corners(c, vp + 16);
    gather(raw, s_tab, c, kf, lf);
  }
  if (nsteps > 2) load_corners(c, vp + 32);
  int s = 0;
  // steady state: f0 = step s, raw = lookups of step s+1, c = corners of s+2
  for (; s + 4 <= nsteps; s += 2) {
    build(f1, raw);
    gather(raw, s_tab, c, kf, lf);
    load_corners(c, vp + 16 * (s + 3));
    mma<PREC>(acc, f0);
    build(f0, raw);
    gather(raw, s_tab, c, kf, lf);
    if (s + 4 < nsteps) load_corners(c, vp + 16 * (s + 4));
    mma<PREC>(acc, f1);
  }
  // drain: at most three steps left (s, s+1, s+2)
  for (; s < nsteps; ++s) {
    if (s + 1 < nsteps) build(f1, raw);
    if (s + 2 < nsteps) gather(raw, s_tab, c, kf, lf);
    if (s + 3 < nsteps) load_corners(c, vp + 16 * (s + 3));
    mma<PREC>(acc, f0);
    f0 = f1;
  }
  store_part<NKB, NLB>(part, acc, split, kp, lp, k0, l0, li, lh);
}

// Operand table of a contraction staged in LDS (8193 entries).
__device__ __forceinline__ void stage_table(uint2 *s_tab, const uint2 *__restrict__ tab) {
  stage_entries(s_tab, tab, kTabEntries);
  __syncthreads();
}

// Split-bf16 launches take the split-fp16 table as well: a clip the rounding
// model routes to split-fp16 (block_route_fp16) runs the fp16 form.
template <int PREC, int NKB, int NLB>
__global__ __launch_bounds__(256) void k_contract_split(const uint4 *__restrict__ packed,
                                                        const uint2 *__restrict__ tab,
                                                        int64_t chunk, int tiles_l, int kp,
                                                        int lp, float *__restrict__ part, double r2,
                                                        RouteArgs ra, const uint2 *__restrict__ tab16) {
  if (tile_outside(blockIdx.x, tiles_l, 64 * NKB, 64 * NLB, r2)) return;
  __shared__ uint2 s_tab[kTabEntries];
  if constexpr (PREC == kBF16) {
    if (block_route_fp16(ra)) {
      stage_table(s_tab, tab16);
      contract_split_body<kFP16, NKB, NLB>(s_tab, packed, chunk, tiles_l, kp, lp, part);
      return;
    }
  }
  stage_table(s_tab, tab);
  contract_split_body<PREC, NKB, NLB>(s_tab, packed, chunk, tiles_l, kp, lp, part);
}

// Lean form of the same contraction for two waves per SIMD: no software
// pipeline inside the wave (lookups, fragment build and MFMAs of a step in
// sequence); the second wave on the SIMD hides the latencies.
template <int PREC, int NKB, int NLB, bool DIRECT = false>
__device__ __forceinline__ void contract_lean_body(const uint2 *s_tab,
                                                   const uint4 *__restrict__ packed,
                                                   int64_t chunk, int tiles_l, int kp, int lp,
                                                   float *__restrict__ part, int tile, int split,
                                                   const BatchClip *bc = nullptr) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 31, lh = lane >> 5;
  const int tk = tile / tiles_l, tl = tile % tiles_l;
  const int k0 = tk * (64 * NKB) + (wave >> 1) * (32 * NKB);
  const int l0 = tl * (64 * NLB) + (wave & 1) * (32 * NLB);

  uint32_t kf[NKB], lf[NLB];
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb) kf[kb] = (uint32_t)(k0 + 32 * kb + li);
#pragma unroll
  for (int lb = 0; lb < NLB; ++lb) lf[lb] = (uint32_t)(l0 + 32 * lb + li);

  f32x16 acc[NKB][NLB][4];
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
    for (int lb = 0; lb < NLB; ++lb)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[kb][lb][q][r] = 0.0f;

  const uint4 *vp = packed + (size_t)split * chunk + 8 * lh;
  for (int64_t vb = 0; vb < chunk; vb += 16) {
    uint4 c[8];
    load_corners(c, vp + vb);
    Raw<NKB, NLB> raw;
    gather(raw, s_tab, c, kf, lf);
    Frag<NKB, NLB> f;
    build(f, raw);
    mma<PREC>(acc, f);
  }
  if constexpr (DIRECT) {
    // read after the loop, so that nothing of it stays live through the MFMAs
    if (bc->direct) {
      store_direct<NKB, NLB>(direct_out(*bc), acc, k0, l0, li, lh);
      return;
    }
  }
  store_part<NKB, NLB>(part, acc, split, kp, lp, k0, l0, li, lh);
}

// Lean form of the same contraction for two waves per SIMD: no software
// pipeline inside the wave (lookups, fragment build and MFMAs of a step in
// sequence); the second wave on the SIMD hides the latencies.
template <int PREC, int NKB, int NLB>
__global__ __launch_bounds__(256, 2) void k_contract_split_lean(const uint4 *__restrict__ packed,
                                                                const uint2 *__restrict__ tab,
                                                                int64_t chunk, int tiles_l,
                                                                int kp, int lp,
                                                                float *__restrict__ part, double r2,
                                                                RouteArgs ra,
                                                                const uint2 *__restrict__ tab16) {
  if (tile_outside(blockIdx.x, tiles_l, 64 * NKB, 64 * NLB, r2)) return;
  __shared__ uint2 s_tab[kTabEntries];
  if constexpr (PREC == kBF16) {
    if (block_route_fp16(ra)) {
      stage_table(s_tab, tab16);
      contract_lean_body<kFP16, NKB, NLB>(s_tab, packed, chunk, tiles_l, kp, lp, part,
                                          blockIdx.x, blockIdx.y);
      return;
    }
  }
  stage_table(s_tab, tab);
  contract_lean_body<PREC, NKB, NLB>(s_tab, packed, chunk, tiles_l, kp, lp, part, blockIdx.x,
                                     blockIdx.y);
}

// Software-pipelined form for one wave per SIMD: the MFMAs of step s are
// interleaved with the table lookups and operand packing of step s+1 and the
// corner loads of step s+2.  Each half-iteration of the loop is one basic
// block (the look-ahead loads clamp their step index instead of branching), so
// the scheduling groups can interleave the whole step: per MFMA one group of
// VALU work, with the LDS lookups front-loaded so that their results are back
// before the packing needs them.  chunk must be a multiple of 32 corners.
template <int NKB, int NLB>
__device__ __forceinline__ void pipe_schedule() {
  constexpr int NM = 12 * NKB * NLB;                          // MFMAs per step
  constexpr int ND = 8 * (NKB + NLB);                         // LDS lookups per step
  constexpr int NV = 8 * NKB + 16 * NLB + 16 * (NKB + NLB);   // phase and packing VALU
#pragma unroll
  for (int i = 0; i < NM; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                   // MFMA
    if (i % 6 == 0) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);   // corner load
    if (i < ND / 2) __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);   // LDS lookups
    __builtin_amdgcn_sched_group_barrier(0x002, (NV + NM - 1) / NM, 0);  // VALU
  }
}

template <int PREC, int NKB, int NLB>
__device__ __forceinline__ void contract_pipe_body(const uint2 *s_tab,
                                                   const uint4 *__restrict__ packed,
                                                   int64_t chunk, int tiles_l, int kp, int lp,
                                                   float *__restrict__ part, int tile, int split) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 31, lh = lane >> 5;
  const int tk = tile / tiles_l, tl = tile % tiles_l;
  const int k0 = tk * (64 * NKB) + (wave >> 1) * (32 * NKB);
  const int l0 = tl * (64 * NLB) + (wave & 1) * (32 * NLB);

  uint32_t kf[NKB], lf[NLB];
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb) kf[kb] = (uint32_t)(k0 + 32 * kb + li);
#pragma unroll
  for (int lb = 0; lb < NLB; ++lb) lf[lb] = (uint32_t)(l0 + 32 * lb + li);

  f32x16 acc[NKB][NLB][4];
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
    for (int lb = 0; lb < NLB; ++lb)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[kb][lb][q][r] = 0.0f;

  const uint4 *vp = packed + (size_t)split * chunk + 8 * lh;
  const int nsteps = (int)(chunk >> 4);  // even
  const int last = nsteps - 1;
  uint4 c0[8], c1[8];
  Raw<NKB, NLB> raw;
  Frag<NKB, NLB> fa, fb;
  load_corners(c0, vp);
  gather(raw, s_tab, c0, kf, lf);
  build(fa, raw);
  load_corners(c1, vp + 16);
  for (int s = 0; s < nsteps; s += 2) {
    // fa: operands of step s; c1: corners of step s+1
    load_corners(c0, vp + 16 * min(s + 2, last));
    gather(raw, s_tab, c1, kf, lf);
    build(fb, raw);
    mma<PREC>(acc, fa);
    pipe_schedule<NKB, NLB>();
    // fb: operands of step s+1; c0: corners of step s+2 (the last iteration
    // prepares a step that is never multiplied)
    load_corners(c1, vp + 16 * min(s + 3, last));
    gather(raw, s_tab, c0, kf, lf);
    build(fa, raw);
    mma<PREC>(acc, fb);
    pipe_schedule<NKB, NLB>();
  }
  store_part<NKB, NLB>(part, acc, split, kp, lp, k0, l0, li, lh);
}

template <int PREC>
__global__ __launch_bounds__(256, 1) void k_contract_split_pipe(const uint4 *__restrict__ packed,
                                                                const uint2 *__restrict__ tab,
                                                                int64_t chunk, int tiles_l,
                                                                int kp, int lp,
                                                                float *__restrict__ part, double r2,
                                                                RouteArgs ra,
                                                                const uint2 *__restrict__ tab16) {
  if (tile_outside(blockIdx.x, tiles_l, 128, 128, r2)) return;
  __shared__ uint2 s_tab[kTabEntries];
  if constexpr (PREC == kBF16) {
    if (block_route_fp16(ra)) {
      stage_table(s_tab, tab16);
      contract_pipe_body<kFP16, 2, 2>(s_tab, packed, chunk, tiles_l, kp, lp, part, blockIdx.x,
                                      blockIdx.y);
      return;
    }
  }
  stage_table(s_tab, tab);
  contract_pipe_body<PREC, 2, 2>(s_tab, packed, chunk, tiles_l, kp, lp, part, blockIdx.x,
                                 blockIdx.y);
}

// FP32 form: v_mfma_f32_32x32x2_f32, two corners per product (lanes 0-31
// carry corner j of the lane's group, lanes 32-63 corner 8 + j).
template <int NKB, int NLB, bool DIRECT = false>
__device__ __forceinline__ void contract_fp32_body(const float2 *s_tab,
                                                   const uint4 *__restrict__ packed,
                                                   int64_t chunk, int tiles_l, int kp, int lp,
                                                   float *__restrict__ part, int tile, int split,
                                                   const BatchClip *bc = nullptr) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 31, lh = lane >> 5;
  const int tk = tile / tiles_l, tl = tile % tiles_l;
  const int k0 = tk * (64 * NKB) + (wave >> 1) * (32 * NKB);
  const int l0 = tl * (64 * NLB) + (wave & 1) * (32 * NLB);

  uint32_t kf[NKB], lf[NLB];
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb) kf[kb] = (uint32_t)(k0 + 32 * kb + li);
#pragma unroll
  for (int lb = 0; lb < NLB; ++lb) lf[lb] = (uint32_t)(l0 + 32 * lb + li);

  f32x16 acc[NKB][NLB][4];
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
    for (int lb = 0; lb < NLB; ++lb)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[kb][lb][q][r] = 0.0f;

  const uint4 *vp = packed + (size_t)split * chunk + 8 * lh;
  for (int64_t vb = 0; vb < chunk; vb += 16) {
    uint4 c[8];
    load_corners(c, vp + vb);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      float2 a[NKB], b[NLB];
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb)
        a[kb] = *(const float2 *)((const char *)s_tab + phase_x(kf[kb], c[j]));
#pragma unroll
      for (int lb = 0; lb < NLB; ++lb)
        b[lb] = *(const float2 *)((const char *)s_tab + phase_y(lf[lb], c[j]));
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
        for (int lb = 0; lb < NLB; ++lb) {
          acc[kb][lb][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[kb].x, b[lb].x, acc[kb][lb][0], 0, 0, 0);
          acc[kb][lb][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[kb].x, b[lb].y, acc[kb][lb][1], 0, 0, 0);
          acc[kb][lb][2] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[kb].y, b[lb].x, acc[kb][lb][2], 0, 0, 0);
          acc[kb][lb][3] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[kb].y, b[lb].y, acc[kb][lb][3], 0, 0, 0);
        }
    }
  }
  if constexpr (DIRECT) {
    // read after the loop, so that nothing of it stays live through the MFMAs
    if (bc->direct) {
      store_direct<NKB, NLB>(direct_out(*bc), acc, k0, l0, li, lh);
      return;
    }
  }
  store_part<NKB, NLB>(part, acc, split, kp, lp, k0, l0, li, lh);
}

// FP32 form: v_mfma_f32_32x32x2_f32, two corners per product (lanes 0-31
// carry corner j of the lane's group, lanes 32-63 corner 8 + j).
template <int NKB, int NLB>
__global__ __launch_bounds__(256) void k_contract_fp32(const uint4 *__restrict__ packed,
                                                       const float2 *__restrict__ tab,
                                                       int64_t chunk, int tiles_l, int kp, int lp,
                                                       float *__restrict__ part, double r2) {
  if (tile_outside(blockIdx.x, tiles_l, 64 * NKB, 64 * NLB, r2)) return;
  __shared__ float2 s_tab[kTabEntries];
  stage_entries(s_tab, tab, kTabEntries);
  __syncthreads();
  contract_fp32_body<NKB, NLB>(s_tab, packed, chunk, tiles_l, kp, lp, part, blockIdx.x,
                               blockIdx.y);
}

// Tile variants: (id, precision mask, k per wave, l per wave, loop form,
// workgroups per CU, corners per split a multiple of).
static const TileVariant kVariants[] = {
    {0, 0x7, 32, 32, 1, 2, 16},
    {1, 0x7, 64, 32, 1, 2, 16},
    {2, 0x7, 64, 64, 1, 2, 16},
    {3, 0x6, 32, 32, 0, 2, 16},
    {4, 0x6, 64, 32, 0, 2, 16},
    {5, 0x6, 64, 64, 2, 1, 32},
};

int n_tile_variants() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }
const TileVariant &tile_variant(int i) { return kVariants[i]; }

template <int NKB, int NLB, bool PIPE>
static void launch_contract_t(const FwdPlan &p, const uint4 *packed, const Tables &t, float *part,
                              const RouteArgs &ra, hipStream_t st) {
  dim3 grid(p.tiles_k * p.tiles_l, p.nsplit), block(256);
  if (p.prec == kFP32) {
    hipLaunchKernelGGL((k_contract_fp32<NKB, NLB>), grid, block, 0, st, packed, t.w32, p.chunk,
                       p.tiles_l, p.kp, p.lp, part, p.r2);
  } else if constexpr (PIPE) {
    if (p.prec == kBF16)
      hipLaunchKernelGGL((k_contract_split<kBF16, NKB, NLB>), grid, block, 0, st, packed,
                         t.wbf16, p.chunk, p.tiles_l, p.kp, p.lp, part, p.r2, ra, t.wfp16);
    else
      hipLaunchKernelGGL((k_contract_split<kFP16, NKB, NLB>), grid, block, 0, st, packed,
                         t.wfp16, p.chunk, p.tiles_l, p.kp, p.lp, part, p.r2, ra, t.wfp16);
  } else {
    if (p.prec == kBF16)
      hipLaunchKernelGGL((k_contract_split_lean<kBF16, NKB, NLB>), grid, block, 0, st, packed,
                         t.wbf16, p.chunk, p.tiles_l, p.kp, p.lp, part, p.r2, ra, t.wfp16);
    else
      hipLaunchKernelGGL((k_contract_split_lean<kFP16, NKB, NLB>), grid, block, 0, st, packed,
                         t.wfp16, p.chunk, p.tiles_l, p.kp, p.lp, part, p.r2, ra, t.wfp16);
  }
}

RouteArgs route_args(const FwdPlan &p, const unsigned long long *area_part) {
  RouteArgs ra;
  ra.area_part = area_part;
  ra.pre_blocks = p.pre_blocks;
  ra.V = p.V;
  ra.gscale = p.gscale;
  ra.gscale_alt = area_part && p.prec == kBF16 ? p.gscale_alt : 0.0;
  return ra;
}

hipError_t launch_contract(const FwdPlan &p, const uint4 *packed, const Tables &t, float *part,
                           hipStream_t st, const unsigned long long *area_part) {
  const RouteArgs ra = route_args(p, area_part);
  switch (p.tile) {
    case 0: launch_contract_t<1, 1, true>(p, packed, t, part, ra, st); break;
    case 1: launch_contract_t<2, 1, true>(p, packed, t, part, ra, st); break;
    case 2: launch_contract_t<2, 2, true>(p, packed, t, part, ra, st); break;
    case 3: launch_contract_t<1, 1, false>(p, packed, t, part, ra, st); break;
    case 4: launch_contract_t<2, 1, false>(p, packed, t, part, ra, st); break;
    case 5: {
      const dim3 grid(p.tiles_k * p.tiles_l, p.nsplit), block(256);
      if (p.prec == kBF16)
        hipLaunchKernelGGL(k_contract_split_pipe<kBF16>, grid, block, 0, st, packed, t.wbf16,
                           p.chunk, p.tiles_l, p.kp, p.lp, part, p.r2, ra, t.wfp16);
      else if (p.prec == kFP16)
        hipLaunchKernelGGL(k_contract_split_pipe<kFP16>, grid, block, 0, st, packed, t.wfp16,
                           p.chunk, p.tiles_l, p.kp, p.lp, part, p.r2, ra, t.wfp16);
      else
        return hipErrorInvalidValue;
      break;
    }
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Epilogue.  For k, l >= 1 (quadrant unfolding of the real GEMM):
//   S(k, l)  = (P - Q) - j (R + U)
//   S(k, -l) = (P + Q) - j (R - U)
// F[k, l] = alpha_{k,l} S(k, l) with alpha_{k,l} = -T / (4 pi^2 k l) (Prop. 3),
// alpha_{k,-l} = -alpha_{k,l}; F[-k,-l] = conj F[k,l] (real signal).
// Split partials are summed in FP64 in a fixed order.  One launch covers the
// contraction grid (blocks [0, nmain), the guard region's entries excepted),
// the axes and DC (the next nax blocks) and the guard slots (the last
// kGuardSlots blocks; the span n the side kernel chose says which are used).
// The output grid and the unfolding (OutGrid, put, store_quad) are shared with
// the contraction kernels that write single-split clips directly.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void epilogue_body(const float *__restrict__ part, int nsplit, int kp,
                                              int lp, int K, int L, double T, const OutGrid &o,
                                              int bx, int by, int gn) {
  // 64 consecutive l per block, 4 threads per l summing splits q, q+4, ...
  __shared__ double4 red[4][64];
  const int t = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int l = 1 + bx * 64 + t;
  const int k = 1 + by;
  const size_t plane = (size_t)kp * lp;
  double P = 0.0, U = 0.0, R = 0.0, Q = 0.0;
  if (l <= L) {
    const size_t o = (size_t)k * lp + l;
    for (int s = q; s < nsplit; s += 4) {
      const float *b = part + (size_t)s * 4 * plane + o;
      P += (double)b[0];
      U += (double)b[plane];
      R += (double)b[2 * plane];
      Q += (double)b[3 * plane];
    }
  }
  red[q][t] = make_double4(P, U, R, Q);
  __syncthreads();
  if (q != 0 || l > L || guarded(k, l, gn)) return;
  for (int w = 1; w < 4; ++w) {
    P += red[w][t].x;
    U += red[w][t].y;
    R += red[w][t].z;
    Q += red[w][t].w;
  }
  store_quad(o, k, l, T, P, U, R, Q);
}

// Entries of guard slot j (span gn): the 16 x 16 sums D (row-major) are the
// corner-range partials added in range order; the block's a-th k and b-th l
// take P = D[a][b], U = D[a][8+b], R = D[8+a][b], Q = D[8+a][8+b].
__device__ __forceinline__ void guard_store(const double *__restrict__ gpart, int g_chunks,
                                            int gn, int K, int L, double T, const OutGrid &o,
                                            int j) {
  if (!guard_slot_used(j, gn)) return;
  __shared__ double d[kGuardD];
  const int t = threadIdx.x;
  double sum = 0.0;
#pragma unroll 16
  for (int c = 0; c < g_chunks; ++c) sum += gpart[((size_t)c * kGuardSlots + j) * kGuardD + t];
  d[t] = sum;
  __syncthreads();
  if (t >= kGuard * kGuard) return;
  const int a = t / kGuard, b = t % kGuard;
  int kb, lb;
  guard_slot_block(j, kb, lb);
  const int k = kGuard * kb + 1 + a, l = kGuard * lb + 1 + b;
  if (k > K || l > L) return;
  store_quad(o, k, l, T, d[a * 16 + b], d[a * 16 + 8 + b], d[(8 + a) * 16 + b],
             d[(8 + a) * 16 + 8 + b]);
}

// Axis entries (Steps 2, 3) and DC (Step 1):
//   F[k,0] = j/(2 pi k) Sx[k],  F[-k,0] = conj F[k,0];  likewise F[0,l];
//   F[0,0] = area / T.
// Block: 16 frequency slots x 16 partial sums over the axis chunks (fixed
// order: chunk c goes to sum c mod 16, the sums are added in order).
__device__ __forceinline__ void epilogue_axes_body(const double2 *__restrict__ axis_part,
                                                   int ax_chunks, int K, int L, double T,
                                                   const unsigned long long *__restrict__ area_part,
                                                   int pre_blocks, const OutGrid &o,
                                                   int64_t *__restrict__ area, int bx) {
  __shared__ double2 red[16][16];
  const int t = threadIdx.x & 15, q = threadIdx.x >> 4;
  const int i = bx * 16 + t;
  const int nslot = K + L;
  double re = 0.0, im = 0.0;
  if (i < nslot)
    for (int c = q; c < ax_chunks; c += 16) {
      const double2 v = axis_part[(size_t)c * nslot + i];
      re += v.x;
      im += v.y;
    }
  red[q][t] = make_double2(re, im);
  __syncthreads();
  if (q == 0 && i < nslot) {
    for (int w = 1; w < 16; ++w) {
      re += red[w][t].x;
      im += red[w][t].y;
    }
    const int f = i < K ? i + 1 : i - K + 1;
    const double sc = (i < K ? o.ax : o.ay) / (2.0 * kPi * (double)f);
    const float fre = (float)(-im * sc), fim = (float)(re * sc);
    if (i < K) {
      put(o, f, 0, fre, fim);
      put(o, -f, 0, fre, -fim);
    } else {
      put(o, 0, f, fre, fim);
      put(o, 0, -f, fre, -fim);
    }
  }
  if (bx == 0 && threadIdx.x >= 64 && threadIdx.x < 128) {
    const int a0 = threadIdx.x - 64;
    unsigned long long a = 0;
    for (int b = a0; b < pre_blocks; b += 64) a += area_part[b];
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    if (a0 == 0) {
      const long long A = (long long)a;
      put(o, 0, 0, (float)((double)A * o.dc), 0.0f);
      if (area) *area = A;
    }
  }
}

// Block b of the epilogue launch of one clip (block-uniform branch).
__device__ __forceinline__ void epilogue_block(const float *__restrict__ part, int nsplit, int kp,
                                               int lp, int K, int L, double T,
                                               const double2 *__restrict__ axis_part,
                                               int ax_chunks,
                                               const unsigned long long *__restrict__ area_part,
                                               int pre_blocks, const double *__restrict__ gpart,
                                               int g_chunks,
                                               const unsigned int *__restrict__ gspan,
                                               const OutGrid &o, int64_t *__restrict__ area,
                                               int b, bool direct = false) {
  const bool grid2d = K > 0 && L > 0;
  const int nbx = (L + 63) / 64;
  const int nmain = grid2d && !direct ? nbx * K : 0;
  const int nax = max(1, (K + L + 15) / 16);
  if (b < nmain)
    epilogue_body(part, nsplit, kp, lp, K, L, T, o, b % nbx, b / nbx, (int)*gspan);
  else if (b < nmain + nax)
    epilogue_axes_body(axis_part, ax_chunks, K, L, T, area_part, pre_blocks, o, area, b - nmain);
  else if (grid2d)
    guard_store(gpart, g_chunks, (int)*gspan, K, L, T, o, b - nmain - nax);
}

int epilogue_block_count(int K, int L, bool direct) {
  const int nmain = K > 0 && L > 0 && !direct ? ((L + 63) / 64) * K : 0;
  const int nax = std::max(1, (K + L + 15) / 16);
  return nmain + nax + (K > 0 && L > 0 ? kGuardSlots : 0);
}

__global__ __launch_bounds__(256) void k_epilogue(const float *__restrict__ part, int nsplit,
                                                  int kp, int lp, int K, int L, double T,
                                                  const double2 *__restrict__ axis_part,
                                                  int ax_chunks,
                                                  const unsigned long long *__restrict__ area_part,
                                                  int pre_blocks,
                                                  const double *__restrict__ gpart, int g_chunks,
                                                  const unsigned int *__restrict__ gspan,
                                                  OutGrid o, int64_t *__restrict__ area) {
  epilogue_block(part, nsplit, kp, lp, K, L, T, axis_part, ax_chunks, area_part, pre_blocks,
                 gpart, g_chunks, gspan, o, area, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_epilogue_axes(const double2 *__restrict__ axis_part,
                                                       int ax_chunks, int K, int L, double T,
                                                       const unsigned long long *__restrict__ area_part,
                                                       int pre_blocks, OutGrid o,
                                                       int64_t *__restrict__ area) {
  epilogue_axes_body(axis_part, ax_chunks, K, L, T, area_part, pre_blocks, o, area, blockIdx.x);
}

// Clears the output grid (band forward: entries outside the computed band).
__global__ __launch_bounds__(256) void k_zero_grid(float2 *__restrict__ F, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    F[i] = make_float2(0.0f, 0.0f);
}

hipError_t launch_zero_outside(const FwdPlan &p, float *F, hipStream_t st) {
  if (p.KO > p.K || p.LO > p.L) {
    const int64_t n = (2 * (int64_t)p.KO + 1) * (2 * (int64_t)p.LO + 1);
    hipLaunchKernelGGL(k_zero_grid, dim3((unsigned)std::min<int64_t>(2048, (n + 255) / 256)),
                       dim3(256), 0, st, (float2 *)F, n);
  }
  return hipGetLastError();
}

hipError_t launch_epilogue(const FwdPlan &p, const void *ws, float *F, int64_t *area,
                           hipStream_t st) {
  const char *w = (const char *)ws;
  const OutGrid o{(float2 *)F, p.KO, p.LO, p.r2, p.eg, p.eax, p.eay, p.edc};
  hipLaunchKernelGGL(k_epilogue, dim3(epilogue_block_count(p.K, p.L)), dim3(256), 0, st,
                     (const float *)(w + p.off_part), p.nsplit, p.kp, p.lp, p.K, p.L, (double)p.T,
                     (const double2 *)(w + p.off_axis), p.ax_chunks,
                     (const unsigned long long *)(w + p.off_area), p.pre_blocks,
                     // folded: the side stream added the guard ranges into range 0
                     (const double *)(w + p.off_guard), guard_folded(p) ? 1 : p.g_chunks,
                     (const unsigned int *)(w + p.off_gspan), o, area);
  return hipGetLastError();
}

hipError_t launch_epilogue_axes(const FwdPlan &p, const void *ws, float *F, int64_t *area,
                                hipStream_t st) {
  const char *w = (const char *)ws;
  const OutGrid o{(float2 *)F, p.KO, p.LO, p.r2, p.eg, p.eax, p.eay, p.edc};
  hipLaunchKernelGGL(k_epilogue_axes, dim3(std::max(1, (p.K + p.L + 15) / 16)), dim3(256), 0, st,
                     (const double2 *)(w + p.off_axis), p.ax_chunks, p.K, p.L, (double)p.T,
                     (const unsigned long long *)(w + p.off_area), p.pre_blocks, o, area);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Direct form for small problems: every coefficient of Prop. 3 as an FP64 sum
// over the corners, in one launch from the raw corner arrays (no pre-pass,
// workspace, partials or second pass).  At a few hundred corners and a few
// thousand frequencies the staged path is launch-bound; this form costs one
// launch and V/4 corner steps per wave.
// Block roles (block-uniform):
//   [0, nq)            P, U, R, Q of one k >= 1 and 64 consecutive l >= 1
//   [nq, nq + nax)     64 consecutive frequencies of one axis sum (Steps 2, 3)
//   nq + nax           the exact area (Step 1) and F[0, 0]
// A block first stages its per-corner factors in LDS (for a quadrant block
// s_v e(k x_v) from the exact table, for an axis block the integer weight),
// then wave w takes corners [w V4, (w + 1) V4), V4 = ceil(V / 4): the factor
// is an LDS broadcast, the lane's entry e(l y_v) a table lookup at the exact
// integer phase, as in the contraction.  The four wave sums are added in
// wave order, so the result does not depend on scheduling.
// ---------------------------------------------------------------------------
constexpr int kDirectUnroll = 8;
constexpr int kDirectMaxV = 1024;  // corners staged in LDS

__global__ __launch_bounds__(256) void k_direct(const int32_t *__restrict__ x,
                                                const int32_t *__restrict__ y,
                                                const int8_t *__restrict__ s, int64_t V, int T,
                                                int shift, int K, int L,
                                                const double2 *__restrict__ w64, OutGrid o,
                                                int64_t *__restrict__ area) {
  // per corner: the block's uniform factor (s_v e(k x_v) for a quadrant
  // block, s_v times the other coordinate for an axis block) and the scaled
  // residue of the coordinate whose phase varies along the lanes
  __shared__ double2 s_a[kDirectMaxV];
  __shared__ uint32_t s_c[kDirectMaxV];
  __shared__ double4 red[4][64];
  __shared__ unsigned long long ared[4];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nlb = (L + 63) / 64, nkb = (K + 63) / 64;
  const int nq = K > 0 && L > 0 ? K * nlb : 0;
  const int nax = nkb + nlb;
  const int b = blockIdx.x;
  const uint32_t tmask = (uint32_t)(T - 1), mask = (uint32_t)(kTabN - 1);
  const int nv = (int)V;

  if (b >= nq + nax) {
    // area = sum s x y modulo 2^64 (exact whenever the true area fits int64)
    unsigned long long acc = 0;
    for (int v = threadIdx.x; v < nv; v += 256)
      acc += (unsigned long long)((long long)s[v] * (long long)x[v] * (long long)y[v]);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) ared[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      const long long A = (long long)(ared[0] + ared[1] + ared[2] + ared[3]);
      put(o, 0, 0, (float)((double)A * o.dc), 0.0f);
      if (area) *area = A;
    }
    return;
  }

  const bool quad = b < nq;
  const bool xaxis = !quad && b - nq < nkb;
  const uint32_t k = quad ? 1u + (uint32_t)(b / nlb) : 0u;
  // the lane's frequency: l for a quadrant block, f for an axis block
  const int f = 1 + (quad ? (b % nlb) : xaxis ? b - nq : b - nq - nkb) * 64 + lane;
  for (int v = threadIdx.x; v < nv; v += 256) {
    const int32_t xv = x[v], yv = y[v];
    const int sv = s[v];
    if (quad) {
      const double2 w = w64[(k * (((uint32_t)xv & tmask) << shift)) & mask];
      s_a[v] = make_double2(sv * w.x, sv * w.y);
      s_c[v] = ((uint32_t)yv & tmask) << shift;
    } else {
      s_a[v] = make_double2((double)(sv * (xaxis ? yv : xv)), 0.0);
      s_c[v] = ((uint32_t)(xaxis ? xv : yv) & tmask) << shift;
    }
  }
  __syncthreads();
  const int per = (nv + 3) / 4;
  const int v0 = min(nv, wave * per), v1 = min(nv, v0 + per);
  double P = 0.0, U = 0.0, R = 0.0, Q = 0.0;
  for (int vb = v0; vb < v1; vb += kDirectUnroll) {
    double2 a[kDirectUnroll], w[kDirectUnroll];
#pragma unroll
    for (int u = 0; u < kDirectUnroll; ++u) {
      const int v = min(vb + u, v1 - 1);  // in range; the tail weight is zero
      const double2 av = s_a[v];
      const bool in = vb + u < v1;
      a[u] = make_double2(in ? av.x : 0.0, in ? av.y : 0.0);
      w[u] = w64[((uint32_t)f * s_c[v]) & mask];
    }
    if (quad) {
#pragma unroll
      for (int u = 0; u < kDirectUnroll; ++u) {
        P = fma(a[u].x, w[u].x, P);
        U = fma(a[u].x, w[u].y, U);
        R = fma(a[u].y, w[u].x, R);
        Q = fma(a[u].y, w[u].y, Q);
      }
    } else {
#pragma unroll
      for (int u = 0; u < kDirectUnroll; ++u) {
        P = fma(a[u].x, w[u].x, P);   // Re sum h e(f q), e = conj(w)
        U = fma(-a[u].x, w[u].y, U);  // Im
      }
    }
  }
  red[wave][lane] = make_double4(P, U, R, Q);
  __syncthreads();
  if (wave != 0) return;
  for (int wv = 1; wv < 4; ++wv) {
    P += red[wv][lane].x;
    U += red[wv][lane].y;
    R += red[wv][lane].z;
    Q += red[wv][lane].w;
  }
  if (quad) {
    if (f <= L) store_quad(o, (int)k, f, (double)T, P, U, R, Q);
    return;
  }
  if (f > (xaxis ? K : L)) return;
  // F[f,0] = j/(2 pi f) Sx[f] (and F[0,f] likewise), Hermitian partners
  const double sc = (xaxis ? o.ax : o.ay) / (2.0 * kPi * (double)f);
  const float fre = (float)(-U * sc), fim = (float)(P * sc);
  if (xaxis) {
    put(o, f, 0, fre, fim);
    put(o, -f, 0, fre, -fim);
  } else {
    put(o, 0, f, fre, fim);
    put(o, 0, -f, fre, -fim);
  }
}

int direct_block_count(int K, int L) {
  const int nlb = (L + 63) / 64, nkb = (K + 63) / 64;
  return (K > 0 && L > 0 ? K * nlb : 0) + nkb + nlb + 1;
}

hipError_t launch_direct(const FwdPlan &p, const int32_t *x, const int32_t *y, const int8_t *s,
                         const double2 *w64, float *F, int64_t *area, hipStream_t st) {
  if (p.V > kDirectMaxV) return hipErrorInvalidValue;
  const OutGrid o{(float2 *)F, p.KO, p.LO, p.r2, p.eg, p.eax, p.eay, p.edc};
  hipLaunchKernelGGL(k_direct, dim3(direct_block_count(p.K, p.L)), dim3(256), 0, st, x, y, s,
                     p.V, p.T, p.shift, p.K, p.L, w64, o, area);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Debug export of the integer phases used by the contraction:
// out[i*V + v] = ((k0+i) * x_v) mod T  (axis 0) or with y_v (axis 1, the
// sign-free phase), recovered from the same byte offsets the kernels use.
// ---------------------------------------------------------------------------
__global__ void k_debug_phases(const uint4 *__restrict__ packed, int64_t V, int axis, int k0,
                               int nk, int shift, int32_t *__restrict__ out) {
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int i = blockIdx.y;
  if (v >= V || i >= nk) return;
  uint4 w = packed[v];
  w.z = 0u;  // the sign-free y phase
  const uint32_t f = (uint32_t)(k0 + i);
  const uint32_t b = axis == 0 ? phase_x(f, w) : phase_y(f, w);
  out[(size_t)i * V + v] = (int32_t)((b >> 3) >> shift);
}

hipError_t launch_debug_phases(const FwdPlan &p, const uint4 *packed, int axis, int k0, int nk,
                               int32_t *out, hipStream_t st) {
  if (p.V == 0 || nk == 0) return hipSuccess;
  hipLaunchKernelGGL(k_debug_phases, dim3((unsigned)((p.V + 255) / 256), nk), dim3(256), 0, st,
                     packed, p.V, axis, k0, nk, p.shift, out);
  return hipGetLastError();
}

// ===========================================================================
// Batched form.  Every clip keeps its own workspace slices; a persistent
// contraction kernel loads the twiddle table into LDS once per workgroup and
// then pulls (clip, tile, split) work items, longest first, from an atomic
// counter until the list is exhausted.  The counter is reset by a kernel at
// the head of the sequence, so a captured graph can be replayed.
// ===========================================================================
// The work counters of the passes and the routed-clip flag (BatchLaunch).
__global__ void k_batch_reset(unsigned int *counter, int n) {
  if ((int)threadIdx.x < n && blockIdx.x == 0) counter[threadIdx.x] = 0u;
}

__global__ __launch_bounds__(256) void k_batch_prepass(const BatchClip *__restrict__ clips) {
  const BatchClip &c = clips[blockIdx.y];
  prepass_body(c.x, c.y, c.s, c.V, c.vpad, c.T, c.shift, c.packed, c.area_part, c.hist,
               blockIdx.x, gridDim.x);
}

// Precision routing of the clips of a split-bf16 batch (route_fp16), one block
// per clip, after the pre-pass: route[c] = 1 sends clip c's work items to the
// split-fp16 pass of the contraction.
__global__ __launch_bounds__(256) void k_batch_route(const BatchClip *__restrict__ clips,
                                                     int pre_blocks, unsigned int *route,
                                                     unsigned int *any) {
  const BatchClip &c = clips[blockIdx.x];
  const long long a = block_area(c.area_part, pre_blocks);
  if (threadIdx.x == 0) {
    const bool r = route_fp16(c.gscale, c.gscale_alt, c.V, a);
    route[blockIdx.x] = r ? 1u : 0u;
    if (r) *any = 1u;  // every writer stores the same value
  }
}

// Side-stream blocks of a batch, one descriptor each: (clip, 0, b) bins
// histogram block b of the clip, (clip, 1, b) its guard block b (slot group
// b / g_chunks over corner range b % g_chunks).
__global__ __launch_bounds__(256) void k_batch_side(const BatchClip *__restrict__ clips,
                                                    const int4 *__restrict__ desc,
                                                    const double2 *__restrict__ w64,
                                                    int pre_blocks) {
  const int4 d = desc[blockIdx.x];
  const BatchClip &c = clips[d.x];
  if (d.y == 0)
    hist_body(c.x, c.y, c.packed, c.V, c.shift, c.hist, d.z, c.hist_blocks);
  else
    guard_body(c.packed, w64, c.V, c.g_chunk, d.z % c.g_chunks, d.z / c.g_chunks, c.area_part,
               pre_blocks, c.gscale, c.gscale_alt, c.K, c.L, c.gpart, c.gspan);
}

__global__ __launch_bounds__(256) void k_batch_axis(const BatchClip *__restrict__ clips,
                                                    const int4 *__restrict__ desc,
                                                    const double2 *__restrict__ w64) {
  const int4 d = desc[blockIdx.x];
  const BatchClip &c = clips[d.x];
  dft_body(c.hist, w64, c.T, c.shift, c.K, c.L, c.ax_fb_k, c.axis_part, d.y, d.z);
}

// Next work item for the whole workgroup (-1 when the list is exhausted).
__device__ __forceinline__ int next_item(unsigned int *counter, int n_items, int *s_item) {
  __syncthreads();
  if (threadIdx.x == 0) *s_item = (int)atomicAdd(counter, 1u);
  __syncthreads();
  const int it = *s_item;
  return it < n_items ? it : -1;
}

// route (split-bf16 batches): the contraction runs as two passes over the work
// list, the bf16 pass (want 0) and the split-fp16 pass of routed clips (want
// 1), each skipping the other's items; nullptr: every item.
template <int PREC, int NKB, int NLB>
__global__ __launch_bounds__(256, 2) void k_batch_contract(const BatchClip *__restrict__ clips,
                                                           const int4 *__restrict__ items,
                                                           int n_items, unsigned int *counter,
                                                           const uint2 *__restrict__ tab,
                                                           const unsigned int *__restrict__ route,
                                                           unsigned int want,
                                                           const unsigned int *__restrict__ any) {
  if (any && *any == 0u) return;  // a routed-clip pass with no routed clip
  __shared__ uint2 s_tab[kTabEntries];
  __shared__ int s_item;
  stage_entries(s_tab, tab, kTabEntries);
  for (;;) {
    const int it = next_item(counter, n_items, &s_item);
    if (it < 0) break;
    const int4 d = items[it];
    if (route && route[d.x] != want) continue;
    const BatchClip &c = clips[d.x];
    contract_lean_body<PREC, NKB, NLB, true>(s_tab, c.packed, c.chunk, c.tiles_l, c.kp, c.lp,
                                             c.part, d.y, d.z, &c);
  }
}

template <int PREC>
__global__ __launch_bounds__(256, 1) void k_batch_contract_pipe(const BatchClip *__restrict__ clips,
                                                                const int4 *__restrict__ items,
                                                                int n_items,
                                                                unsigned int *counter,
                                                                const uint2 *__restrict__ tab,
                                                                const unsigned int *__restrict__ route,
                                                                unsigned int want,
                                                                const unsigned int *__restrict__ any) {
  if (any && *any == 0u) return;  // a routed-clip pass with no routed clip
  __shared__ uint2 s_tab[kTabEntries];
  __shared__ int s_item;
  stage_entries(s_tab, tab, kTabEntries);
  for (;;) {
    const int it = next_item(counter, n_items, &s_item);
    if (it < 0) break;
    const int4 d = items[it];
    if (route && route[d.x] != want) continue;
    const BatchClip &c = clips[d.x];
    contract_pipe_body<PREC, 2, 2>(s_tab, c.packed, c.chunk, c.tiles_l, c.kp, c.lp, c.part, d.y,
                                   d.z);
  }
}

template <int NKB, int NLB>
__global__ __launch_bounds__(256, 2) void k_batch_contract_fp32(const BatchClip *__restrict__ clips,
                                                                const int4 *__restrict__ items,
                                                                int n_items, unsigned int *counter,
                                                                const float2 *__restrict__ tab) {
  __shared__ float2 s_tab[kTabEntries];
  __shared__ int s_item;
  stage_entries(s_tab, tab, kTabEntries);
  for (;;) {
    const int it = next_item(counter, n_items, &s_item);
    if (it < 0) break;
    const int4 d = items[it];
    const BatchClip &c = clips[d.x];
    contract_fp32_body<NKB, NLB, true>(s_tab, c.packed, c.chunk, c.tiles_l, c.kp, c.lp, c.part,
                                       d.y, d.z, &c);
  }
}

// clip owning flat block b of a prefix array off[0..n]
__device__ __forceinline__ int owner(const int *__restrict__ off, int n, int b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_batch_epilogue(const BatchClip *__restrict__ clips,
                                                        const int *__restrict__ off, int n,
                                                        int pre_blocks) {
  const int ci = owner(off, n, blockIdx.x);
  const BatchClip &c = clips[ci];
  const OutGrid o{c.F, c.K, c.L, -1.0, (double)c.T, 1.0, 1.0, 1.0 / (double)c.T};
  epilogue_block(c.part, c.nsplit, c.kp, c.lp, c.K, c.L, (double)c.T, c.axis_part, c.ax_chunks,
                 c.area_part, pre_blocks, c.gpart, c.g_chunks, c.gspan, o, c.area,
                 blockIdx.x - off[ci], c.direct != 0);
}

// ===========================================================================
// Batch of general tiles: one launch per step over all clips (GBatchLaunch).
// ===========================================================================
__global__ __launch_bounds__(256) void k_gbatch_prepass(const GBatchClip *__restrict__ clips) {
  const GBatchClip &c = clips[blockIdx.y];
  if ((int)blockIdx.x >= c.pre_blocks) return;
  gen_prepass_body(c.x, c.y, c.s, c.V, c.vpad, c.Mx, c.My, c.smask, c.packed, c.area_part,
                   c.big ? nullptr : c.hist, blockIdx.x, c.pre_blocks, c.big ? c.words : nullptr);
}

// (clip, 0, b): histogram block b; (clip, 1 | 2, b): guard block b (slot group
// b / g_chunks over corner range b % g_chunks), 2 with two-level tables
__global__ __launch_bounds__(256) void k_gbatch_side(const GBatchClip *__restrict__ clips,
                                                     const int4 *__restrict__ desc) {
  const int4 d = desc[blockIdx.x];
  const GBatchClip &c = clips[d.x];
  constexpr int UR = 4;  // no contraction workgroup shares a CU with these blocks
  if (d.y == 0)
    hist_body<true>(c.x, c.y, c.packed, c.V, 0, c.hist, d.z, c.hist_blocks);
  else if (d.y == 1)
    guard_body<true, false, false, UR>(c.packed, c.w64x, c.V, c.g_chunk, d.z % c.g_chunks,
                                       d.z / c.g_chunks, c.area_part, c.pre_blocks, c.gscale,
                                       c.gscale_alt, c.K, c.L, c.gpart, c.gspan, c.w64y, c.Mx,
                                       c.My);
  else if (big_narrow(c.Mx, c.My))
    guard_body<true, true, true, UR>(c.words, c.w64x, c.V, c.g_chunk, d.z % c.g_chunks,
                                     d.z / c.g_chunks, c.area_part, c.pre_blocks, c.gscale,
                                     c.gscale_alt, c.K, c.L, c.gpart, c.gspan, c.w64y, c.Mx, c.My,
                                     c.nhx, c.nhy);
  else
    guard_body<true, true, false, UR>(c.words, c.w64x, c.V, c.g_chunk, d.z % c.g_chunks,
                                      d.z / c.g_chunks, c.area_part, c.pre_blocks, c.gscale,
                                      c.gscale_alt, c.K, c.L, c.gpart, c.gspan, c.w64y, c.Mx,
                                      c.My, c.nhx, c.nhy);
}

// (clip, 0, fb, chunk): DFT of the histograms; (clip, 1, fb, chunk): the
// direct sums of a two-level clip
__global__ __launch_bounds__(256) void k_gbatch_axis(const GBatchClip *__restrict__ clips,
                                                     const int4 *__restrict__ desc) {
  __shared__ double2 abuf[kAxisBigLds];
  const int4 d = desc[blockIdx.x];
  const GBatchClip &c = clips[d.x];
  if (d.y == 0)
    dft_body<true>(c.hist, c.w64x, c.Mx, 0, c.K, c.L, c.ax_fb_k, c.axis_part, d.z, d.w, c.w64y,
                   c.My);
  else if (big_narrow(c.Mx, c.My))
    gen_axis_big_body<true>(c.x, c.y, c.words, c.V, c.ax_chunk, c.w64x, c.w64y, c.Mx, c.My,
                            c.nhx, c.nhy, c.K, c.L, c.ax_fb_k, c.axis_part, d.z, d.w, abuf);
  else
    gen_axis_big_body<false>(c.x, c.y, c.words, c.V, c.ax_chunk, c.w64x, c.w64y, c.Mx, c.My,
                             c.nhx, c.nhy, c.K, c.L, c.ax_fb_k, c.axis_part, d.z, d.w, abuf);
}

__global__ __launch_bounds__(256) void k_gbatch_epilogue(const GBatchClip *__restrict__ clips,
                                                         const int *__restrict__ off, int n) {
  const int ci = owner(off, n, blockIdx.x);
  const GBatchClip &c = clips[ci];
  const OutGrid o{c.F, c.K, c.L, -1.0, c.eg, c.eax, c.eay, c.edc};
  epilogue_block(c.part, c.nsplit, c.kp, c.lp, c.K, c.L, (double)c.Mx, c.axis_part, c.ax_chunks,
                 c.area_part, c.pre_blocks, c.gpart, c.g_chunks, c.gspan, o, c.area,
                 blockIdx.x - off[ci]);
}

hipError_t launch_gbatch_prepass(const GBatchLaunch &b, hipStream_t st) {
  if (b.n_clips > 0)
    hipLaunchKernelGGL(k_gbatch_prepass, dim3(b.max_pre_blocks, b.n_clips), dim3(256), 0, st,
                       b.clips);
  return hipGetLastError();
}

hipError_t launch_gbatch_side(const GBatchLaunch &b, hipStream_t st) {
  if (b.n_side > 0)
    hipLaunchKernelGGL(k_gbatch_side, dim3(b.n_side), dim3(256), 0, st, b.clips, b.side_desc);
  if (b.n_ax > 0)
    hipLaunchKernelGGL(k_gbatch_axis, dim3(b.n_ax), dim3(256), 0, st, b.clips, b.ax_desc);
  return hipGetLastError();
}

hipError_t launch_gbatch_epilogue(const GBatchLaunch &b, hipStream_t st) {
  if (b.n_epi > 0)
    hipLaunchKernelGGL(k_gbatch_epilogue, dim3(b.n_epi), dim3(256), 0, st, b.clips, b.epi_off,
                       b.n_clips);
  return hipGetLastError();
}

hipError_t launch_batch_prepass(const BatchLaunch &b, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, st, b.counter, 2 * b.n_groups + 1);
  hipLaunchKernelGGL(k_batch_prepass, dim3(b.pre_blocks, b.n_clips), dim3(256), 0, st, b.clips);
  if (b.prec == kBF16 && b.route && b.n_clips > 0)
    hipLaunchKernelGGL(k_batch_route, dim3(b.n_clips), dim3(256), 0, st, b.clips, b.pre_blocks,
                       b.route, b.counter + 2 * b.n_groups);
  return hipGetLastError();
}

hipError_t launch_batch_side(const BatchLaunch &b, const double2 *w64, hipStream_t st) {
  if (b.n_side > 0)
    hipLaunchKernelGGL(k_batch_side, dim3(b.n_side), dim3(256), 0, st, b.clips, b.side_desc,
                       w64, b.pre_blocks);
  if (b.n_ax > 0)
    hipLaunchKernelGGL(k_batch_axis, dim3(b.n_ax), dim3(256), 0, st, b.clips, b.ax_desc, w64);
  return hipGetLastError();
}

int batch_grid(int tile, int prec) {
  (void)prec;
  return tile_variant(tile).wg_per_cu * 256;  // persistent workgroups on 256 CUs
}

// One persistent pass over items [0, n) in precision prec with tile variant
// `tile` (want: the route value of the clips it takes, or all clips when route
// is nullptr).  any: when given, the pass exits at once unless *any is set.
static void batch_pass(const BatchLaunch &b, const Tables &t, int prec, int tile,
                       const int4 *items, int n, const unsigned int *route, unsigned int want,
                       unsigned int *counter, hipStream_t st, const unsigned int *any = nullptr) {
  const dim3 grid(batch_grid(tile, prec)), block(256);
  const bool wide = tile_variant(tile).wk == 64;
  const uint2 *tab = prec == kBF16 ? t.wbf16 : t.wfp16;
  if (prec == kFP32) {
    if (wide)
      hipLaunchKernelGGL((k_batch_contract_fp32<2, 1>), grid, block, 0, st, b.clips, items, n,
                         counter, t.w32);
    else
      hipLaunchKernelGGL((k_batch_contract_fp32<1, 1>), grid, block, 0, st, b.clips, items, n,
                         counter, t.w32);
  } else if (tile == 5) {
    if (prec == kBF16)
      hipLaunchKernelGGL(k_batch_contract_pipe<kBF16>, grid, block, 0, st, b.clips, items, n,
                         counter, tab, route, want, any);
    else
      hipLaunchKernelGGL(k_batch_contract_pipe<kFP16>, grid, block, 0, st, b.clips, items, n,
                         counter, tab, route, want, any);
  } else if (prec == kBF16) {
    if (wide)
      hipLaunchKernelGGL((k_batch_contract<kBF16, 2, 1>), grid, block, 0, st, b.clips, items, n,
                         counter, tab, route, want, any);
    else
      hipLaunchKernelGGL((k_batch_contract<kBF16, 1, 1>), grid, block, 0, st, b.clips, items, n,
                         counter, tab, route, want, any);
  } else {
    if (wide)
      hipLaunchKernelGGL((k_batch_contract<kFP16, 2, 1>), grid, block, 0, st, b.clips, items, n,
                         counter, tab, route, want, any);
    else
      hipLaunchKernelGGL((k_batch_contract<kFP16, 1, 1>), grid, block, 0, st, b.clips, items, n,
                         counter, tab, route, want, any);
  }
}

hipError_t launch_batch_contract(const BatchLaunch &b, const Tables &t, hipStream_t st) {
  const int G = b.n_groups;
  for (int g = 0; g < G; ++g) {
    const int n = b.group_off[g + 1] - b.group_off[g];
    if (n == 0) continue;
    const int4 *items = b.items + b.group_off[g];
    const int tile = b.group_tile[g];
    if (b.prec == kBF16 && b.route) {
      // split-bf16: the clips the rounding model keeps in bf16, then the routed ones
      batch_pass(b, t, kBF16, tile, items, n, b.route, 0u, b.counter + g, st);
      batch_pass(b, t, kFP16, tile, items, n, b.route, 1u, b.counter + G + g, st,
                 b.counter + 2 * G);
    } else {
      batch_pass(b, t, b.prec, tile, items, n, nullptr, 0u, b.counter + g, st);
    }
  }
  return hipGetLastError();
}

hipError_t launch_batch_epilogue(const BatchLaunch &b, hipStream_t st) {
  if (b.n_epi > 0)
    hipLaunchKernelGGL(k_batch_epilogue, dim3(b.n_epi), dim3(256), 0, st, b.clips, b.epi_off,
                       b.n_clips, b.pre_blocks);
  return hipGetLastError();
}

}  // namespace fcfs
