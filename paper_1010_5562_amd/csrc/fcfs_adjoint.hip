// Adjoint of the FCFS forward transform with respect to the corner
// coordinates (gfx950).
//
// Differentiating the closed forms of Prop. 3 (Sec. III-C1), with
// e(t) = e^{-j 2 pi t / T} and the torch cotangent G = dL/dRe F + j dL/dIm F,
// dL/dtheta = Re sum conj(G[k,l]) dF[k,l]/dtheta:
//  * F[k,l] = alpha s e(kx) e(ly) gives dF/dx_v = s_v (j/(2 pi l)) e(k x_v) e(l y_v)
//    and dF/dy_v = s_v (j/(2 pi k)) e(k x_v) e(l y_v) (alpha (-j w k) = j/(2 pi l)).
//    Folding (k,l) with (-k,-l) leaves k > 0; writing e = c - j s for both
//    coordinates turns the sum into s_v X_v^T W Y_v with X_v = [cos; sin](k x_v),
//    Y_v = [cos; sin](l y_v) and a real matrix W built from G: one GEMM
//    (vertices x 2K) . (2K x 4L) for both gradients, whose rows are dotted
//    with Y_v on the fly (never stored).
//  * F[k,0] = (j/(2 pi k)) sum s y e(kx): dF/dx_v = s_v y_v e(k x_v)/T,
//    dF/dy_v = s_v (j/(2 pi k)) e(k x_v); F[0,l] likewise; F[0,0] = area/T:
//    dF/dx_v = s_v y_v / T, dF/dy_v = s_v x_v / T.  These are evaluated per
//    corner in FP64.
//  * General tile (periods Nx, Ny, corners on a 2^-F grid): the same forms
//    with alpha of Prop. 3 for Nx x Ny; the coefficients j/(2 pi l) of the x
//    gradient gain sqrt(Ny/Nx), those of the y gradient sqrt(Nx/Ny), and 1/T
//    becomes 2^-F / sqrt(Nx Ny) (coordinates in grid units); phases are
//    reduced modulo Mx = Nx 2^F, My = Ny 2^F with per-period tables.
#include "fcfs_device.h"

namespace fcfs {

// Position of W[row r][column n] in the MFMA operand records (see k_adj_split).
__device__ __forceinline__ size_t rec_index(int n, int r, int lb, int ncb) {
  const int q = n / lb, lm = n - q * lb;
  const int kstep = r >> 4, h = (r >> 3) & 1, j = r & 7, cb = (lm >> 5) * 4 + q, li = lm & 31;
  return ((((size_t)kstep * ncb + cb) * 64) + li + 32 * h) * 8 + j;
}

// Position of W[row r][column n] in the FP32 operand records: per 16-row step
// and column block (the blocks of rec_index), 8 sub-steps of two rows, each a
// 64-lane B operand of v_mfma_f32_32x32x2_f32 (lane li + 32 h: row 2 u + h,
// column li of the block).
__device__ __forceinline__ size_t rec_index_f32(int n, int r, int lb, int ncb) {
  const int q = n / lb, lm = n - q * lb;
  const int kstep = r >> 4, u = (r >> 1) & 7, h = r & 1, cb = (lm >> 5) * 4 + q, li = lm & 31;
  return ((((size_t)kstep * ncb + cb) * 8 + u) * 64) + li + 32 * h;
}

// ---------------------------------------------------------------------------
// W from the cotangent.  For 1 <= k <= kb, 1 <= l <= lb (zero outside the
// band), with M'[k,l] = M[k,l] + conj(M[-k,-l]) and a + jb = M'[k,l],
// a'' + jb'' = M'[k,-l]:
//   W(cos k, cos l) = a + a'',  W(cos k, sin l) = b - b'',
//   W(sin k, cos l) = b + b'',  W(sin k, sin l) = a'' - a.
// Columns: [x: cos l | x: sin l | y: cos l | y: sin l], each lb wide; rows:
// [cos k | sin k], each kb long.  Stored transposed, Wf[n * R + r], FP32.
// The largest |W| is folded into *wmax (float bits, non-negative).
// ---------------------------------------------------------------------------
// MODE 0: FP32 matrix Wf (transposed) and its largest |W| (the split-fp16
// path scales from it); 1: split-bf16 operand records; 2: FP32 operand
// records (rec_index_f32).
template <int MODE>
__global__ __launch_bounds__(256) void k_adj_w(const float2 *__restrict__ G, int K, int L, int kmax,
                                               int lmax, double r2, int kb, int lb, double rx,
                                               double ry, float *__restrict__ Wf,
                                               unsigned int *__restrict__ wmax,
                                               uint16_t *__restrict__ whi,
                                               uint16_t *__restrict__ wlo,
                                               int *__restrict__ scale) {
  const int l = 1 + blockIdx.x * 256 + threadIdx.x;
  const int k = 1 + blockIdx.y;
  // lanes past lb stay active (with zeros) for the wave-wide maximum below
  const bool live = l <= lb;
  const int R = 2 * kb;
  double Wcc = 0, Wcs = 0, Wsc = 0, Wss = 0, Ycc = 0, Ycs = 0, Ysc = 0, Yss = 0;
  if (live && k <= kmax && l <= lmax && (r2 < 0.0 || (double)k * k + (double)l * l <= r2)) {
    const size_t WL = 2 * (size_t)L + 1;
    const float2 gpp = G[(size_t)(K + k) * WL + (L + l)];  // G[k, l]
    const float2 gmm = G[(size_t)(K - k) * WL + (L - l)];  // G[-k, -l]
    const float2 gpm = G[(size_t)(K + k) * WL + (L - l)];  // G[k, -l]
    const float2 gmp = G[(size_t)(K - k) * WL + (L + l)];  // G[-k, l]
    // conj(G) * j c = (c gi, c gr); folded with the conjugate of the mirror
    const double cl = rx / (2.0 * kPi * l), ck = ry / (2.0 * kPi * k);
    // x gradient: c = 1/(2 pi l) with the sign of l
    double a = cl * ((double)gpp.y - gmm.y), b = cl * ((double)gpp.x + gmm.x);
    double a2 = -cl * ((double)gpm.y - gmp.y), b2 = -cl * ((double)gpm.x + gmp.x);
    Wcc = a + a2;
    Wss = a2 - a;
    Wsc = b + b2;
    Wcs = b - b2;
    // y gradient: c = 1/(2 pi k), k > 0 on both sides
    a = ck * ((double)gpp.y - gmm.y);
    b = ck * ((double)gpp.x + gmm.x);
    a2 = ck * ((double)gpm.y - gmp.y);
    b2 = ck * ((double)gpm.x + gmp.x);
    Ycc = a + a2;
    Yss = a2 - a;
    Ysc = b + b2;
    Ycs = b - b2;
  }
  const int rc = k - 1, rs = kb + k - 1;
  const size_t nxc = (size_t)(l - 1), nxs = (size_t)(lb + l - 1);
  const size_t nyc = (size_t)(2 * lb + l - 1), nys = (size_t)(3 * lb + l - 1);
  const float v[8] = {(float)Wcc, (float)Wsc, (float)Wcs, (float)Wss,
                      (float)Ycc, (float)Ysc, (float)Ycs, (float)Yss};
  if constexpr (MODE == 2) {
    if (!live) return;
    const int ncb = lb / 8;
    const int nn[8] = {(int)nxc, (int)nxc, (int)nxs, (int)nxs, (int)nyc, (int)nyc, (int)nys, (int)nys};
    const int rr[8] = {rc, rs, rc, rs, rc, rs, rc, rs};
#pragma unroll
    for (int i = 0; i < 8; ++i) Wf[rec_index_f32(nn[i], rr[i], lb, ncb)] = v[i];
    return;
  }
  if constexpr (MODE == 1) {
    // split-bf16: hi + lo records written here, scale 2^0
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) scale[0] = 0;
    if (!live) return;
    const int ncb = lb / 8;  // NC / 32 with NC = 4 lb
    const int nn[8] = {(int)nxc, (int)nxc, (int)nxs, (int)nxs, (int)nyc, (int)nyc, (int)nys, (int)nys};
    const int rr[8] = {rc, rs, rc, rs, rc, rs, rc, rs};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const __bf16 hi = (__bf16)v[i];
      const __bf16 lo = (__bf16)(v[i] - (float)hi);
      const size_t o = rec_index(nn[i], rr[i], lb, ncb);
      whi[o] = __builtin_bit_cast(uint16_t, hi);
      wlo[o] = __builtin_bit_cast(uint16_t, lo);
    }
    return;
  }
  if (live) {
    Wf[nxc * R + rc] = v[0];
    Wf[nxc * R + rs] = v[1];
    Wf[nxs * R + rc] = v[2];
    Wf[nxs * R + rs] = v[3];
    Wf[nyc * R + rc] = v[4];
    Wf[nyc * R + rs] = v[5];
    Wf[nys * R + rc] = v[6];
    Wf[nys * R + rs] = v[7];
  }
  float m = 0.f;
#pragma unroll
  for (int i = 0; i < 8; ++i) m = fmaxf(m, fabsf(v[i]));
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0 && m > 0.f) atomicMax(wmax, __float_as_uint(m));
}

// Split W into hi + lo 16-bit parts after scaling by 2^e, e chosen from the
// largest |W| so that the binary16 range is never exceeded (bf16 uses the
// same scale).  scale[0] = e (as int), written by block 0.
// The parts are stored in MFMA operand order: the 16 x 32 block (rows
// 16 kstep .. +15, columns of block cb) is one 1 KB record of 64 lanes x 8
// values, lane li + 32 h holding rows 16 kstep + 8 h .. +7 of the block's
// column li, so that a wave loads its B operand with one contiguous read.
// Block cb = 4 lblk + q holds the columns (q, l = 32 lblk + 1 .. 32 lblk + 32).
template <int PREC>
__global__ __launch_bounds__(256) void k_adj_split(const float *__restrict__ Wf, int R, int NC,
                                                   int lb,
                                                   const unsigned int *__restrict__ wmax,
                                                   uint16_t *__restrict__ whi,
                                                   uint16_t *__restrict__ wlo,
                                                   int *__restrict__ scale) {
  const float m = __uint_as_float(*wmax);
  int e = 0;
  if (m > 0.f) {
    int ex;
    frexpf(m, &ex);  // m < 2^ex
    e = 14 - ex;     // m * 2^e < 2^14
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) scale[0] = e;
  const int64_t n_all = (int64_t)R * NC;
  const int ncb = NC / 32;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n_all;
       i += (int64_t)gridDim.x * 256) {
    const int n = (int)(i / R), r = (int)(i % R);
    const float w = ldexpf(Wf[i], e);
    const size_t o = rec_index(n, r, lb, ncb);
    if constexpr (PREC == kBF16) {
      const __bf16 hi = (__bf16)w;
      const __bf16 lo = (__bf16)(w - (float)hi);
      whi[o] = __builtin_bit_cast(uint16_t, hi);
      wlo[o] = __builtin_bit_cast(uint16_t, lo);
    } else {
      const _Float16 hi = (_Float16)w;
      const _Float16 lo = (_Float16)(w - (float)hi);
      whi[o] = __builtin_bit_cast(uint16_t, hi);
      wlo[o] = __builtin_bit_cast(uint16_t, lo);
    }
  }
}

__global__ void k_fill_u32(unsigned int *p, int n, unsigned int v) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

// Axis and DC coefficients, folded over +-f:
//   P_k = conj(G[k,0]) + G[-k,0],  Q_l = conj(G[0,l]) + G[0,-l],  G00 real part.
// coef layout: [P_1..P_K | Q_1..Q_L | Re G00 | P_k/(2 pi k) | Q_l/(2 pi l)] as
// double2 (the scaled copies spare the per-corner loop a division).
__global__ void k_adj_axcoef(const float2 *__restrict__ G, int K, int L, int kmax, int lmax,
                             double rx, double ry, double2 *__restrict__ coef) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const size_t WL = 2 * (size_t)L + 1;
  double2 v = make_double2(0.0, 0.0);
  int f = 0;
  if (i < K) {
    const int k = i + 1;
    f = k;
    if (k <= kmax) {
      const float2 a = G[(size_t)(K + k) * WL + L], b = G[(size_t)(K - k) * WL + L];
      v = make_double2((double)a.x + b.x, (double)b.y - a.y);
    }
  } else if (i < K + L) {
    const int l = i - K + 1;
    f = l;
    if (l <= lmax) {
      const float2 a = G[(size_t)K * WL + (L + l)], b = G[(size_t)K * WL + (L - l)];
      v = make_double2((double)a.x + b.x, (double)b.y - a.y);
    }
  } else if (i == K + L) {
    coef[i] = make_double2((double)G[(size_t)K * WL + L].x, 0.0);
    return;
  } else {
    return;
  }
  coef[i] = v;
  // P_k enters the y gradient (sqrt(Nx/Ny)), Q_l the x gradient (sqrt(Ny/Nx))
  const double sc = (i < K ? ry : rx) / (2.0 * kPi * (double)f);
  coef[K + L + 1 + i] = make_double2(v.x * sc, v.y * sc);
}

// Slot s of the register-resident main term's partials (k_adj_gemm_regb)
// holds y-gradient sums when bit 1 of s is set (waves of types 2 and 3 hold
// the y cos l and y sin l column blocks).
__host__ __device__ inline bool adj_slot_y(int s) { return (s & 2) != 0; }

// Per corner, FP64: the axis and DC parts of gx, gy (written, not added),
// plus, when part is given, the main-term partials of the register-resident
// kernel (k_adj_gemm_regb) in slot order.
// sum_f Re[c_f e(f t)] with e(f t) = conj(w^f), w = e^{j 2 pi ts / N}: the
// powers come from repeated multiplication, restarted from the exact table
// every 32 steps.
// GEN: residue records of a general tile, tables wx (period Mx) and wy (My);
// BIG: two-level tables (nhx, nhy entries of Whi) for periods past 8192.
template <bool GEN, bool BIG = false>
__global__ __launch_bounds__(256) void k_adj_axis(const int32_t *__restrict__ x,
                                                  const int32_t *__restrict__ y,
                                                  const uint4 *__restrict__ packed,
                                                  const double2 *__restrict__ w64,
                                                  const double2 *__restrict__ coef, int64_t V,
                                                  int K, int L, int kmax, int lmax, double dcf,
                                                  float *__restrict__ gx, float *__restrict__ gy,
                                                  const double2 *__restrict__ wy = nullptr,
                                                  int Mx = 0, int My = 0, int nhx = 0,
                                                  int nhy = 0,
                                                  const float *__restrict__ part = nullptr,
                                                  int nslots = 0, int64_t vpad = 0) {
  // 64 corners per workgroup, four waves: wave r takes the frequencies
  // f = r + 1 + 4 i of every corner (the coefficient loads stay uniform), its
  // twiddle stepping by e(4 t) and re-read from the exact table every eighth
  // step; the four partial sums meet in LDS in a fixed order
  __shared__ double4 red[4][64];
  const int r = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int64_t v = (int64_t)blockIdx.x * 64 + lane;
  const double dMx = (double)Mx, dMy = (double)My;
  const bool live = v < V;
  const int64_t vv = live ? v : 0;
  const uint4 c = packed[vv];
  const double2 *coef_s = coef + (K + L + 1);  // scaled by 1/(2 pi f)
  double sx1 = 0.0, sx2 = 0.0;  // sum Re[P e(kx)],  sum Re[P j/(2 pi k) e(kx)]
  if (live) {
    const uint32_t ph = GEN ? c.x : c.x >> 3;
    auto tw = [&](uint32_t k) {
      return BIG ? big_entry64(w64, nhx, big_phase(k, ph, dMx, 1.0 / dMx))
           : GEN ? w64[(k * ph) % (uint32_t)Mx]
                 : w64[(k * ph) & (uint32_t)(kTabN - 1)];
    };
    const double2 w4 = tw(4u);
    double2 w = w4;
#pragma unroll 4
    for (int k = r + 1, i = 0; k <= kmax; k += 4, ++i) {
      if ((i & 7) == 0) w = tw((uint32_t)k);
      const double2 p = coef[k - 1], ps = coef_s[k - 1];
      // e(kx) = w.x - j w.y;  Re[j z] = -Im z
      sx1 += p.x * w.x + p.y * w.y;
      sx2 -= ps.y * w.x - ps.x * w.y;
      const double nx = w.x * w4.x - w.y * w4.y, ny = w.x * w4.y + w.y * w4.x;
      w = make_double2(nx, ny);
    }
  }
  double sy1 = 0.0, sy2 = 0.0;  // sum Re[Q e(ly)],  sum Re[Q j/(2 pi l) e(ly)]
  if (live) {
    const double2 *W = GEN ? wy : w64;
    const uint32_t ph = GEN ? c.y : c.y >> 3;
    auto tw = [&](uint32_t l) {
      return BIG ? big_entry64(W, nhy, big_phase(l, ph, dMy, 1.0 / dMy))
           : GEN ? W[(l * ph) % (uint32_t)My]
                 : W[(l * ph) & (uint32_t)(kTabN - 1)];
    };
    const double2 w4 = tw(4u);
    double2 w = w4;
#pragma unroll 4
    for (int l = r + 1, i = 0; l <= lmax; l += 4, ++i) {
      if ((i & 7) == 0) w = tw((uint32_t)l);
      const double2 q = coef[K + l - 1], qs = coef_s[K + l - 1];
      sy1 += q.x * w.x + q.y * w.y;
      sy2 -= qs.y * w.x - qs.x * w.y;
      const double nx = w.x * w4.x - w.y * w4.y, ny = w.x * w4.y + w.y * w4.x;
      w = make_double2(nx, ny);
    }
  }
  red[r][lane] = make_double4(sx1, sx2, sy1, sy2);
  __syncthreads();
  if (!live || r != 0) return;
  {
    const double4 a = red[0][lane], b = red[1][lane], d = red[2][lane], e = red[3][lane];
    sx1 = (a.x + b.x) + (d.x + e.x);
    sx2 = (a.y + b.y) + (d.y + e.y);
    sy1 = (a.z + b.z) + (d.z + e.z);
    sy2 = (a.w + b.w) + (d.w + e.w);
  }
  const double sg = c.z ? -1.0 : 1.0;
  const double xv = (double)x[v], yv = (double)y[v];
  const double g00 = coef[K + L].x;
  float fx = (float)(sg * (yv * dcf * sx1 + sy2 + yv * g00 * dcf));
  float fy = (float)(sg * (sx2 + xv * dcf * sy1 + xv * g00 * dcf));
  for (int sl = 0; sl < nslots; ++sl) {
    const float t = part[(size_t)sl * vpad + v];
    if (adj_slot_y(sl))
      fy += t;
    else
      fx += t;
  }
  gx[v] = fx;
  gy[v] = fy;
}

// ---------------------------------------------------------------------------
// Main term: t_v = X_v^T W on MFMA (rows = 32 corners per wave, inner = the
// 2*kb frequencies, four column blocks of 32 at a time), each finished column
// block dotted with Y_v at once; the per-corner partial sums are reduced
// across the 32 columns held by the lanes and added to gx, gy.
// The eight waves of a workgroup (256 corners) share the W operand records:
// per 16-frequency step the workgroup copies the 16 records it needs (4 column
// blocks x cos/sin rows x hi/lo, 16 KB) into one of two LDS buffers, then every
// wave reads them from there.  The step index runs on across column groups so
// that consecutive steps always alternate buffers: one barrier per step keeps
// a buffer from being refilled while a slower wave still reads it.
// ---------------------------------------------------------------------------
constexpr int kAdjNB = 4;
constexpr int kAdjWaves = 8;

// Exact (f t) mod M for a lane-constant t < M <= 8192 and f < 2^19, with
// m = ceil(t 2^32 / M): floor(f t / M) = floor(f m / 2^32) because the error
// f (m - t 2^32 / M) / 2^32 < 2^-13 <= 1 / M.
__device__ __forceinline__ uint32_t adj_magic(uint32_t t, uint32_t M) {
  return (uint32_t)((((uint64_t)t << 32) + M - 1u) / M);
}
__device__ __forceinline__ uint32_t adj_phase(uint32_t f, uint32_t t, uint32_t m, uint32_t M) {
  return __umul24(f, t) - __umul24(__umulhi(f, m), M);
}

// Operand tables of a general tile in dynamic LDS: x entries [0, Mx), then y
// entries [Mx, Mx + My) unless the periods are equal (one table).
template <typename E>
__device__ __forceinline__ void stage_period_tables(E *dyn, const void *tx, const void *ty, int Mx,
                                                    int My, const E *&px, const E *&py) {
  for (int i = threadIdx.x; i < Mx; i += 64 * kAdjWaves) dyn[i] = static_cast<const E *>(tx)[i];
  if (tx != ty)
    for (int i = threadIdx.x; i < My; i += 64 * kAdjWaves) dyn[Mx + i] = static_cast<const E *>(ty)[i];
  px = dyn;
  py = tx != ty ? dyn + Mx : dyn;
}

// GEN: a general tile (residue records, per-period tables tab / taby in
// dynamic LDS, exact phases by adj_phase).  BIG: periods past 8192, tab and
// taby two-level FP32 tables (nhx, nhy entries of Whi), phases by big_phase,
// the x-side split entries rounded from the FP32 product in the kernel.
template <int PREC, bool GEN, bool BIG = false>
__global__ __launch_bounds__(64 * kAdjWaves) void k_adj_gemm_split(
    const uint4 *__restrict__ packed, const uint2 *__restrict__ tab,
    const uint16_t *__restrict__ whi,
    const uint16_t *__restrict__ wlo, const int *__restrict__ scale, int64_t V, int kb, int lb,
    float *__restrict__ gx, float *__restrict__ gy, const uint2 *__restrict__ taby = nullptr,
    int Mx = 0, int My = 0, int nhx = 0, int nhy = 0) {
  __shared__ u32x4 s_w[2][4 * kAdjNB][64];
  const uint2 *s_tab = nullptr, *s_taby = nullptr;
  const float2 *b_tab = nullptr, *b_taby = nullptr;
  const double dMx = (double)Mx, dMy = (double)My;
  const double iMx = BIG ? 1.0 / dMx : 0.0, iMy = BIG ? 1.0 / dMy : 0.0;
  if constexpr (BIG) {
    extern __shared__ uint2 s_dyn[];
    stage_period_tables<float2>((float2 *)s_dyn, tab, taby, nhx + kBigLo, nhy + kBigLo, b_tab,
                                b_taby);
  } else if constexpr (GEN) {
    extern __shared__ uint2 s_dyn[];
    stage_period_tables<uint2>(s_dyn, tab, taby, Mx, My, s_tab, s_taby);
  } else {
    __shared__ uint2 s_fix[kTabEntries];
    for (int i = threadIdx.x; i < kTabEntries; i += 64 * kAdjWaves) s_fix[i] = tab[i];
    s_tab = s_taby = s_fix;
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 31, lh = lane >> 5;
  const int64_t vbase = (int64_t)blockIdx.x * (32 * kAdjWaves) + wave * 32;
  const int NC = 4 * lb, ncb = NC / 32, nks = kb / 16;
  const int nsteps = (NC / (32 * kAdjNB)) * nks;
  // operand record q of flat step it: column block nb = q & 3, sin rows if
  // q & 4, lo part if q & 8 (layout of k_adj_split)
  auto record = [&](int it, int q) -> const u32x4 * {
    const int cgi = it / nks, t = it - cgi * nks;
    const int kstep = (q & 4) ? nks + t : t;
    const size_t cb = (size_t)(cgi * kAdjNB + (q & 3));
    const uint16_t *base = (q & 8) ? wlo : whi;
    return (const u32x4 *)(base + ((((size_t)kstep * ncb + cb) * 64) * 8));
  };
  // this thread's share of a step's 16 records: entries idx = tid + 512 u
  constexpr int kPer = 4 * kAdjNB * 64 / (64 * kAdjWaves);
  u32x4 pre[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int idx = threadIdx.x + 64 * kAdjWaves * u;
    pre[u] = record(0, idx >> 6)[idx & 63];
  }
  const uint4 ca = packed[vbase + li];  // this lane's A row
  // the 16 output rows this lane holds
  uint32_t ys8[16], ym[16];
  bool neg[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const uint4 c = packed[vbase + 8 * (r >> 2) + 4 * lh + (r & 3)];
    ys8[r] = c.y;
    ym[r] = GEN && !BIG ? adj_magic(c.y, (uint32_t)My) : 0u;
    neg[r] = c.z != 0u;
  }
  const uint32_t xm = GEN && !BIG ? adj_magic(ca.x, (uint32_t)Mx) : 0u;
  float sx[16], sy[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) sx[r] = sy[r] = 0.f;
  int it = 0;
  for (int cg = 0; cg < NC; cg += 32 * kAdjNB) {
    f32x16 acc[kAdjNB];
#pragma unroll
    for (int nb = 0; nb < kAdjNB; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[nb][r] = 0.f;
    for (int ib = 0; ib < kb; ib += 16, ++it) {
      const int buf = it & 1;
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int idx = threadIdx.x + 64 * kAdjWaves * u;
        s_w[buf][idx >> 6][idx & 63] = pre[u];
      }
      __syncthreads();
      if (it + 1 < nsteps) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
          const int idx = threadIdx.x + 64 * kAdjWaves * u;
          pre[u] = record(it + 1, idx >> 6)[idx & 63];
        }
      }
      uint2 d[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const uint32_t f = (uint32_t)(1 + ib + 8 * lh + j);
        if constexpr (BIG)
          d[j] = split_entry<PREC>(big_entry(b_tab, nhx, big_phase(f, ca.x, dMx, iMx)));
        else
          d[j] = GEN ? s_tab[adj_phase(f, ca.x, xm, (uint32_t)Mx)] : lds_entry(s_tab, phase_x(f, ca));
      }
      u32x4 ach, ash, acl, asl;
      pack4(d, ach, ash, acl, asl);
#pragma unroll
      for (int nb = 0; nb < kAdjNB; ++nb) {
        const u32x4 bch = s_w[buf][nb][lane], bsh = s_w[buf][4 + nb][lane];
        const u32x4 bcl = s_w[buf][8 + nb][lane], bsl = s_w[buf][12 + nb][lane];
        acc[nb] = mfma16<PREC>(ach, bch, acc[nb]);
        acc[nb] = mfma16<PREC>(ach, bcl, acc[nb]);
        acc[nb] = mfma16<PREC>(acl, bch, acc[nb]);
        acc[nb] = mfma16<PREC>(ash, bsh, acc[nb]);
        acc[nb] = mfma16<PREC>(ash, bsl, acc[nb]);
        acc[nb] = mfma16<PREC>(asl, bsh, acc[nb]);
      }
    }
    // dot with Y_v: this lane's four accumulators hold the columns (q, l) of
    // one frequency l; (cos, sin)(l y) = hi + lo from the split table
    {
      const uint32_t l = (uint32_t)((cg >> 2) + li + 1);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        float yc, ys;
        if constexpr (BIG) {
          const float2 e = big_entry(b_taby, nhy, big_phase(l, ys8[r], dMy, iMy));
          yc = e.x;
          ys = e.y;
        } else if constexpr (PREC == kBF16) {
          const uint2 e = GEN ? s_taby[adj_phase(l, ys8[r], ym[r], (uint32_t)My)]
                              : lds_entry(s_taby, phase_x(l, make_uint4(ys8[r], 0u, 0u, 0u)));
          yc = __uint_as_float(e.x << 16) + __uint_as_float(e.y << 16);
          ys = __uint_as_float(e.x & 0xFFFF0000u) + __uint_as_float(e.y & 0xFFFF0000u);
        } else {
          const uint2 e = GEN ? s_taby[adj_phase(l, ys8[r], ym[r], (uint32_t)My)]
                              : lds_entry(s_taby, phase_x(l, make_uint4(ys8[r], 0u, 0u, 0u)));
          yc = (float)__builtin_bit_cast(_Float16, (uint16_t)(e.x & 0xFFFFu)) +
               (float)__builtin_bit_cast(_Float16, (uint16_t)(e.y & 0xFFFFu));
          ys = (float)__builtin_bit_cast(_Float16, (uint16_t)(e.x >> 16)) +
               (float)__builtin_bit_cast(_Float16, (uint16_t)(e.y >> 16));
        }
        sx[r] = fmaf(acc[0][r], yc, fmaf(acc[1][r], ys, sx[r]));
        sy[r] = fmaf(acc[2][r], yc, fmaf(acc[3][r], ys, sy[r]));
      }
    }
  }
  // sum over the 32 columns of each half-wave (fixed butterfly order)
#pragma unroll
  for (int r = 0; r < 16; ++r)
    for (int o = 1; o < 32; o <<= 1) {
      sx[r] += __shfl_xor(sx[r], o, 64);
      sy[r] += __shfl_xor(sy[r], o, 64);
    }
  const float inv = ldexpf(1.0f, -scale[0]);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    if (li != r) continue;
    const int64_t v = vbase + 8 * (r >> 2) + 4 * lh + (r & 3);
    if (v < V) {
      const float sg = neg[r] ? -inv : inv;
      gx[v] += sg * sx[r];
      gy[v] += sg * sy[r];
    }
  }
}

// ---------------------------------------------------------------------------
// Register-resident form of the split main term (square tiles, kb <= 128),
// computed transposed: C^T = W^T X^T, W's column blocks as the MFMA A operand
// (the same records serve: for 32 x 32 x 16 products A and B share the lane
// layout) and the corner twiddles as B.  A workgroup takes a set of CPS
// frequency chunks (32 frequencies l each) with 4 CPS waves: wave w holds the
// column block of type w mod 4 (x cos l, x sin l, y cos l, y sin l) of chunk
// w / 4 in registers for all 2 kb rows, loaded once; CPS waves per SIMD hide
// each other's latencies.  The B operands of a 32-corner tile (the corner
// twiddles of every 16-frequency step, gathered from the table and packed)
// are built once per tile, one step per wave, and passed through LDS to all
// waves (double buffered: the next tile's operands are built while the
// current tile is multiplied).  In C^T each lane holds 16 columns of one
// corner, so the dot with Y_v is a per-lane sum plus one exchange between the
// two half-waves.  Tiles go to the persistent grid in contiguous runs; wave w
// of set s writes part[4 CPS s + w][v], and k_adj_axis adds the slots of each
// gradient in slot order, so the result does not depend on scheduling.
// ---------------------------------------------------------------------------
template <int NKS>
struct RegB {
  static constexpr int CPS = NKS <= 6 ? 3 : 2;  // chunks per set: waves = 4 CPS
};

template <int PREC, bool SIN>
__device__ __forceinline__ float split_value(uint2 e) {
  // hi + lo of cos (low halves) or sin (high halves) of a split table entry
  if constexpr (PREC == kBF16) {
    return SIN ? __uint_as_float(e.x & 0xFFFF0000u) + __uint_as_float(e.y & 0xFFFF0000u)
               : __uint_as_float(e.x << 16) + __uint_as_float(e.y << 16);
  } else {
    return SIN ? (float)__builtin_bit_cast(_Float16, (uint16_t)(e.x >> 16)) +
                     (float)__builtin_bit_cast(_Float16, (uint16_t)(e.y >> 16))
               : (float)__builtin_bit_cast(_Float16, (uint16_t)(e.x & 0xFFFFu)) +
                     (float)__builtin_bit_cast(_Float16, (uint16_t)(e.y & 0xFFFFu));
  }
}

// Per-lane dot of the C^T columns with Y_v: the block covers frequencies
// l = 32 chunk + m + 1 for the rows m = 8 (r >> 2) + 4 lh + (r & 3) of the lane.
template <int PREC, bool SIN>
__device__ __forceinline__ float regb_dot(const f32x16 &acc, int chunk, const uint2 *s_tab,
                                          uint32_t ys8, int lh) {
  float p[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const uint32_t l = (uint32_t)(32 * chunk + 8 * (r >> 2) + 4 * lh + (r & 3) + 1);
    const uint2 e = lds_entry(s_tab, phase_x(l, make_uint4(ys8, 0u, 0u, 0u)));
    p[r & 3] = fmaf(acc[r], split_value<PREC, SIN>(e), p[r & 3]);
  }
  return (p[0] + p[1]) + (p[2] + p[3]);
}

template <int PREC, int NKS>
__global__ __launch_bounds__(256 * RegB<NKS>::CPS, 1) void k_adj_gemm_regb(
    const uint4 *__restrict__ packed, const uint2 *__restrict__ tab,
    const uint16_t *__restrict__ whi, const uint16_t *__restrict__ wlo,
    const int *__restrict__ scale, int64_t vpad, int lb, float *__restrict__ part) {
  constexpr int CPS = RegB<NKS>::CPS;
  __shared__ uint2 s_tab[kTabN];
  __shared__ u32x4 s_b[2][NKS][4][64];  // packed corner operands of two tiles
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int li = lane & 31, lh = lane >> 5;
  const int ncb = lb / 8, nchunk = lb / 32;
  const int chunk = blockIdx.y * CPS + (wave >> 2);
  const int64_t ntiles = vpad / 32;
  const int64_t t0 = (int64_t)blockIdx.x * ntiles / gridDim.x;
  const int64_t t1 = (int64_t)(blockIdx.x + 1) * ntiles / gridDim.x;
  // in the order they are needed (memory waits count in issue order): the
  // table, the first two corner records, then this wave's block of W, which
  // only the first products wait for
  stage_entries_once(s_tab, tab, kTabN);
  // records of tiles past t1 - 1 are never used: the load is clamped to the
  // last tile, unconditional (a conditional or selected load would leave the
  // memory waits of the loop unable to tell the look-ahead load from the
  // ones it needs); the grid is never wider than the tile count, so t0 < t1
  auto record = [&](int64_t t) { return packed[min(t, t1 - 1) * 32 + li]; };
  uint4 c_cur = record(t0);
  uint4 c_nxt = record(t0 + 1);
  // column block of type wave mod 4 in the wave's chunk (a chunk past the
  // last one of a partial set holds zeros and adds nothing)
  u32x4 wreg[NKS][4];  // cos hi, cos lo, sin hi, sin lo rows of each step
  {
    const bool valid = chunk < nchunk;
    const int cb = 4 * chunk + (wave & 3);
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const size_t rc = (((size_t)ks * ncb + cb) * 64 + lane) * 8;
      const size_t rs = (((size_t)(NKS + ks) * ncb + cb) * 64 + lane) * 8;
      const u32x4 z = {0u, 0u, 0u, 0u};
      wreg[ks][0] = valid ? *(const u32x4 *)(whi + rc) : z;
      wreg[ks][1] = valid ? *(const u32x4 *)(wlo + rc) : z;
      wreg[ks][2] = valid ? *(const u32x4 *)(whi + rs) : z;
      wreg[ks][3] = valid ? *(const u32x4 *)(wlo + rs) : z;
    }
  }
  const float inv = ldexpf(1.0f, -scale[0]);
  // step `wave` of the corner operands of a tile into buffer buf, from the
  // lane's corner record c (corner li of the tile)
  auto build = [&](const uint4 &c, int buf) {
    if (wave >= NKS) return;
    uint2 d[8];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      d[j] = lds_entry(s_tab, phase_x((uint32_t)(1 + 16 * wave + 8 * lh + j), c));
    u32x4 ch, sh, cl, sl;
    pack4(d, ch, sh, cl, sl);
    s_b[buf][wave][0][lane] = ch;
    s_b[buf][wave][1][lane] = sh;
    s_b[buf][wave][2][lane] = cl;
    s_b[buf][wave][3][lane] = sl;
  };
  __syncthreads();  // table staged
  build(c_cur, 0);
  // W and the first records have arrived before the loop: inside it the only
  // load in flight is the look-ahead record
  __builtin_amdgcn_s_waitcnt(0xc07f);  // vmcnt(0)
  __syncthreads();
  float *dst = part + (size_t)(4 * CPS * blockIdx.y + wave) * vpad;
  for (int64_t t = t0; t < t1; ++t) {
    const int buf = (int)((t - t0) & 1);
    // the record two tiles ahead is loaded while this tile runs
    const uint4 c_far = record(t + 2);
    if (t + 1 < t1) build(c_nxt, buf ^ 1);
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const u32x4 bch = s_b[buf][ks][0][lane], bsh = s_b[buf][ks][1][lane];
      const u32x4 bcl = s_b[buf][ks][2][lane], bsl = s_b[buf][ks][3][lane];
      acc = mfma16<PREC>(wreg[ks][0], bch, acc);
      acc = mfma16<PREC>(wreg[ks][1], bch, acc);
      acc = mfma16<PREC>(wreg[ks][0], bcl, acc);
      acc = mfma16<PREC>(wreg[ks][2], bsh, acc);
      acc = mfma16<PREC>(wreg[ks][3], bsh, acc);
      acc = mfma16<PREC>(wreg[ks][2], bsl, acc);
    }
    // dot with Y_v of this lane's corner: cos l for types 0 and 2, sin l for
    // types 1 and 3 (a uniform branch)
    float p = (wave & 1) ? regb_dot<PREC, true>(acc, chunk, s_tab, c_cur.y, lh)
                         : regb_dot<PREC, false>(acc, chunk, s_tab, c_cur.y, lh);
    p += __shfl_xor(p, 32, 64);  // the two half-waves hold the two row halves
    if (lh == 0) dst[t * 32 + li] = (c_cur.z ? -inv : inv) * p;
    c_cur = c_nxt;
    c_nxt = c_far;
    __syncthreads();  // buffer buf is rebuilt in the next iteration
  }
}

// FP32 main term: v_mfma_f32_32x32x2_f32, two frequencies per product, with
// the operand records of rec_index_f32 shared through LDS as in the split form
// (eight waves, 256 corners per workgroup, double-buffered 16-row steps).
template <bool GEN, bool BIG = false>
__global__ __launch_bounds__(64 * kAdjWaves) void k_adj_gemm_fp32(
    const uint4 *__restrict__ packed, const float2 *__restrict__ tab32g,
    const float *__restrict__ Wr, int64_t V, int kb, int lb, float *__restrict__ gx,
    float *__restrict__ gy, const float2 *__restrict__ taby = nullptr, int Mx = 0, int My = 0,
    int nhx = 0, int nhy = 0) {
  __shared__ float s_w[2][2 * kAdjNB][8][64];
  const float2 *s_tab, *s_taby;
  const double dMx = (double)Mx, dMy = (double)My;
  const double iMx = BIG ? 1.0 / dMx : 0.0, iMy = BIG ? 1.0 / dMy : 0.0;
  if constexpr (GEN) {
    extern __shared__ float2 s_dynf[];
    // BIG: two-level tables (nhx, nhy entries of Whi, then Wlo)
    stage_period_tables<float2>(s_dynf, tab32g, taby, BIG ? nhx + kBigLo : Mx,
                                BIG ? nhy + kBigLo : My, s_tab, s_taby);
  } else {
    __shared__ float2 s_fix[kTabEntries];
    for (int i = threadIdx.x; i < kTabEntries; i += 64 * kAdjWaves) s_fix[i] = tab32g[i];
    s_tab = s_taby = s_fix;
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 31, lh = lane >> 5;
  const int64_t vbase = (int64_t)blockIdx.x * (32 * kAdjWaves) + wave * 32;
  const int NC = 4 * lb, ncb = NC / 32, nks = kb / 16;
  const int nsteps = (NC / (32 * kAdjNB)) * nks;
  // block q of flat step it: column block nb = q & 3, sin rows if q & 4
  auto record = [&](int it, int q) -> const float4 * {
    const int cgi = it / nks, t = it - cgi * nks;
    const int kstep = (q & 4) ? nks + t : t;
    const size_t cb = (size_t)(cgi * kAdjNB + (q & 3));
    return (const float4 *)(Wr + (((size_t)kstep * ncb + cb) * 8) * 64);
  };
  // a step is 8 blocks x 512 floats = 1024 float4: two per thread
  constexpr int kPer = 2 * kAdjNB * 8 * 64 / 4 / (64 * kAdjWaves);
  float4 pre[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int idx = threadIdx.x + 64 * kAdjWaves * u;
    pre[u] = record(0, idx >> 7)[idx & 127];
  }
  const uint4 ca = packed[vbase + li];
  uint32_t ys8[16], ym[16];
  bool neg[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const uint4 c = packed[vbase + 8 * (r >> 2) + 4 * lh + (r & 3)];
    ys8[r] = c.y;
    ym[r] = GEN && !BIG ? adj_magic(c.y, (uint32_t)My) : 0u;
    neg[r] = c.z != 0u;
  }
  const uint32_t xm = GEN && !BIG ? adj_magic(ca.x, (uint32_t)Mx) : 0u;
  float sx[16], sy[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) sx[r] = sy[r] = 0.f;
  int it = 0;
  for (int cg = 0; cg < NC; cg += 32 * kAdjNB) {
    f32x16 acc[kAdjNB];
#pragma unroll
    for (int nb = 0; nb < kAdjNB; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[nb][r] = 0.f;
    for (int ib = 0; ib < kb; ib += 16, ++it) {
      const int buf = it & 1;
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int idx = threadIdx.x + 64 * kAdjWaves * u;
        *(float4 *)&s_w[buf][idx >> 7][(idx & 127) >> 4][(idx & 15) * 4] = pre[u];
      }
      __syncthreads();
      if (it + 1 < nsteps) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
          const int idx = threadIdx.x + 64 * kAdjWaves * u;
          pre[u] = record(it + 1, idx >> 7)[idx & 127];
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const uint32_t f = (uint32_t)(1 + ib + 2 * u + lh);
        const float2 a = BIG   ? big_entry(s_tab, nhx, big_phase(f, ca.x, dMx, iMx))
                         : GEN ? s_tab[adj_phase(f, ca.x, xm, (uint32_t)Mx)]
                               : *(const float2 *)((const char *)s_tab + phase_x(f, ca));
#pragma unroll
        for (int nb = 0; nb < kAdjNB; ++nb) {
          acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, s_w[buf][nb][u][lane], acc[nb], 0,
                                                         0, 0);
          acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, s_w[buf][4 + nb][u][lane],
                                                         acc[nb], 0, 0, 0);
        }
      }
    }
    // dot with Y_v: one (cos, sin)(l y) per row serves the four accumulators
    {
      const uint32_t l = (uint32_t)((cg >> 2) + li + 1);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float2 w = BIG   ? big_entry(s_taby, nhy, big_phase(l, ys8[r], dMy, iMy))
                         : GEN ? s_taby[adj_phase(l, ys8[r], ym[r], (uint32_t)My)]
                               : *(const float2 *)((const char *)s_taby +
                                                   phase_x(l, make_uint4(ys8[r], 0u, 0u, 0u)));
        sx[r] = fmaf(acc[0][r], w.x, fmaf(acc[1][r], w.y, sx[r]));
        sy[r] = fmaf(acc[2][r], w.x, fmaf(acc[3][r], w.y, sy[r]));
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 16; ++r)
    for (int o = 1; o < 32; o <<= 1) {
      sx[r] += __shfl_xor(sx[r], o, 64);
      sy[r] += __shfl_xor(sy[r], o, 64);
    }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    if (li != r) continue;
    const int64_t v = vbase + 8 * (r >> 2) + 4 * lh + (r & 3);
    if (v < V) {
      const float sg = neg[r] ? -1.f : 1.f;
      gx[v] += sg * sx[r];
      gy[v] += sg * sy[r];
    }
  }
}

namespace {
template <typename KernelT>
hipError_t allow_big_lds(KernelT k, bool &done) {
  if (done) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)(sizeof(uint2) * 2 * kTabN));
  done = e == hipSuccess;
  return e;
}
}  // namespace

hipError_t launch_adjoint(const AdjPlan &a, const int32_t *x, const int32_t *y, const int8_t *s,
                          const float *gradF, const Tables &t, void *ws, float *gx, float *gy,
                          hipStream_t st, const PeriodTables *gtab,
                          hipEvent_t *main_ev) {
  char *w = (char *)ws;
  const uint4 *packed = (const uint4 *)(w + a.off_packed);
  double2 *coef = (double2 *)(w + a.off_coef);
  float *Wf = (float *)(w + a.off_wf);
  uint16_t *whi = (uint16_t *)(w + a.off_whi), *wlo = (uint16_t *)(w + a.off_wlo);
  unsigned int *wmax = (unsigned int *)(w + a.off_scale);
  int *scale = (int *)(w + a.off_scale + 64);
  const float2 *G = (const float2 *)gradF;
  const bool gen = a.gen && gtab;
  if (a.gen && !gtab) return hipErrorInvalidValue;
  (void)s;
  hipLaunchKernelGGL(k_adj_axcoef, dim3((a.K + a.L + 1 + 255) / 256), dim3(256), 0, st, G, a.K,
                     a.L, a.kmax, a.lmax, a.rx, a.ry, coef);
  // register-resident main term (square tiles, split precisions): W and the
  // slot partials first, then the axis kernel writes gx, gy with them added
  const bool regb = a.regb_nks > 0 && !gen && a.kmax > 0 && a.lmax > 0 && a.V > 0;
  if (regb) {
    const dim3 wgrid((a.lb + 255) / 256, a.kb);
    if (a.prec == kBF16) {
      hipLaunchKernelGGL(k_adj_w<1>, wgrid, dim3(256), 0, st, G, a.K, a.L, a.kmax, a.lmax, a.r2,
                         a.kb, a.lb, a.rx, a.ry, Wf, wmax, whi, wlo, scale);
    } else {
      hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, wmax, 1, 0u);
      hipLaunchKernelGGL(k_adj_w<0>, wgrid, dim3(256), 0, st, G, a.K, a.L, a.kmax, a.lmax, a.r2,
                         a.kb, a.lb, a.rx, a.ry, Wf, wmax, whi, wlo, scale);
      const int64_t n = (int64_t)a.R * a.NC;
      const unsigned sb = (unsigned)std::min<int64_t>(1024, (n + 255) / 256);
      hipLaunchKernelGGL(k_adj_split<kFP16>, dim3(sb), dim3(256), 0, st, Wf, a.R, a.NC, a.lb,
                         wmax, whi, wlo, scale);
    }
    float *rpart = (float *)(w + a.off_rpart);
    const int64_t ntiles = a.vpad / 32;
    const dim3 grid((unsigned)std::max<int64_t>(
                        1, std::min<int64_t>(ntiles, kAdjRegbGrid / std::max(1, a.regb_sets))),
                    (unsigned)a.regb_sets);
    const uint2 *tb = a.prec == kBF16 ? t.wbf16 : t.wfp16;
    if (main_ev) (void)hipEventRecord(main_ev[0], st);
#define FCFS_REGB(P, N)                                                                       \
  hipLaunchKernelGGL((k_adj_gemm_regb<P, N>), grid, dim3(256 * RegB<N>::CPS), 0, st, packed, tb, \
                     whi, wlo, scale, a.vpad, a.lb, rpart)
    switch (a.regb_nks * 4 + (a.prec == kBF16 ? 0 : 1)) {
      case 8: FCFS_REGB(kBF16, 2); break;
      case 9: FCFS_REGB(kFP16, 2); break;
      case 16: FCFS_REGB(kBF16, 4); break;
      case 17: FCFS_REGB(kFP16, 4); break;
      case 24: FCFS_REGB(kBF16, 6); break;
      case 25: FCFS_REGB(kFP16, 6); break;
      case 32: FCFS_REGB(kBF16, 8); break;
      case 33: FCFS_REGB(kFP16, 8); break;
      default: return hipErrorInvalidValue;
    }
#undef FCFS_REGB
    if (main_ev) (void)hipEventRecord(main_ev[1], st);
    hipLaunchKernelGGL(k_adj_axis<false>, dim3((unsigned)((a.V + 63) / 64)), dim3(256), 0, st,
                       x, y, packed, t.w64, coef, a.V, a.K, a.L, a.kmax, a.lmax, a.dcf, gx, gy,
                       nullptr, 0, 0, 0, 0, rpart, 4 * adj_regb_nbw(a.regb_nks) * a.regb_sets,
                       a.vpad);
    return hipGetLastError();
  }
  // axis and DC parts first: they write gx, gy
  if (a.V > 0) {
    if (gen && a.big)
      hipLaunchKernelGGL((k_adj_axis<true, true>), dim3((unsigned)((a.V + 63) / 64)), dim3(256),
                         0, st, x, y, packed, gtab->w64x, coef, a.V, a.K, a.L, a.kmax, a.lmax,
                         a.dcf, gx, gy, gtab->w64y, a.Mx, a.My, a.nhx, a.nhy);
    else if (gen)
      hipLaunchKernelGGL(k_adj_axis<true>, dim3((unsigned)((a.V + 63) / 64)), dim3(256), 0, st,
                         x, y, packed, gtab->w64x, coef, a.V, a.K, a.L, a.kmax, a.lmax, a.dcf, gx,
                         gy, gtab->w64y, a.Mx, a.My);
    else
      hipLaunchKernelGGL(k_adj_axis<false>, dim3((unsigned)((a.V + 63) / 64)), dim3(256), 0, st,
                         x, y, packed, t.w64, coef, a.V, a.K, a.L, a.kmax, a.lmax, a.dcf, gx, gy,
                         nullptr, 0, 0);
  }
  if (a.kmax == 0 || a.lmax == 0 || a.V == 0) return hipGetLastError();
  const dim3 wgrid((a.lb + 255) / 256, a.kb);
  if (a.prec == kBF16) {
    hipLaunchKernelGGL(k_adj_w<1>, wgrid, dim3(256), 0, st, G, a.K, a.L, a.kmax, a.lmax, a.r2,
                       a.kb, a.lb, a.rx, a.ry, Wf, wmax, whi, wlo, scale);
  } else if (a.prec == kFP32) {
    hipLaunchKernelGGL(k_adj_w<2>, wgrid, dim3(256), 0, st, G, a.K, a.L, a.kmax, a.lmax, a.r2,
                       a.kb, a.lb, a.rx, a.ry, Wf, wmax, whi, wlo, scale);
  } else {
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, wmax, 1, 0u);
    hipLaunchKernelGGL(k_adj_w<0>, wgrid, dim3(256), 0, st, G, a.K, a.L, a.kmax, a.lmax, a.r2,
                       a.kb, a.lb, a.rx, a.ry, Wf, wmax, whi, wlo, scale);
  }
  const unsigned sblocks = (unsigned)(a.vpad / (32 * kAdjWaves));
  // general tile: both period tables in dynamic LDS (two-level: Whi and Wlo
  // of each period, FP32 pairs)
  const bool same = gen && gtab->opx == gtab->opy;
  const size_t glds =
      !gen ? 0
      : a.big ? sizeof(float2) * ((size_t)a.nhx + kBigLo + (same ? 0 : (size_t)a.nhy + kBigLo))
              : sizeof(uint2) * ((size_t)a.Mx + (same ? 0 : a.My));
  hipError_t e;
  if (main_ev) (void)hipEventRecord(main_ev[0], st);
  if (a.prec == kFP32) {
    if (gen && a.big) {
      static bool done = false;
      if ((e = allow_big_lds(k_adj_gemm_fp32<true, true>, done))) return e;
      hipLaunchKernelGGL((k_adj_gemm_fp32<true, true>), dim3(sblocks), dim3(64 * kAdjWaves), glds,
                         st, packed, (const float2 *)gtab->opx, Wf, a.V, a.kb, a.lb, gx, gy,
                         (const float2 *)gtab->opy, a.Mx, a.My, a.nhx, a.nhy);
    } else if (gen) {
      static bool done = false;
      if ((e = allow_big_lds(k_adj_gemm_fp32<true>, done))) return e;
      hipLaunchKernelGGL(k_adj_gemm_fp32<true>, dim3(sblocks), dim3(64 * kAdjWaves), glds, st,
                         packed, (const float2 *)gtab->opx, Wf, a.V, a.kb, a.lb, gx, gy,
                         (const float2 *)gtab->opy, a.Mx, a.My);
    } else {
      hipLaunchKernelGGL(k_adj_gemm_fp32<false>, dim3(sblocks), dim3(64 * kAdjWaves), 0, st,
                         packed, t.w32, Wf, a.V, a.kb, a.lb, gx, gy, nullptr, 0, 0);
    }
  } else {
    const int64_t n = (int64_t)a.R * a.NC;
    const unsigned sb = (unsigned)std::min<int64_t>(1024, (n + 255) / 256);
    if (a.prec == kFP16)
      hipLaunchKernelGGL(k_adj_split<kFP16>, dim3(sb), dim3(256), 0, st, Wf, a.R, a.NC, a.lb,
                         wmax, whi, wlo, scale);
    const uint2 *tb = a.prec == kBF16 ? t.wbf16 : t.wfp16;
    if (gen && a.big) {
      if (a.prec == kBF16) {
        static bool done = false;
        if ((e = allow_big_lds(k_adj_gemm_split<kBF16, true, true>, done))) return e;
        hipLaunchKernelGGL((k_adj_gemm_split<kBF16, true, true>), dim3(sblocks),
                           dim3(64 * kAdjWaves), glds, st, packed, (const uint2 *)gtab->opx, whi,
                           wlo, scale, a.V, a.kb, a.lb, gx, gy, (const uint2 *)gtab->opy, a.Mx,
                           a.My, a.nhx, a.nhy);
      } else {
        static bool done = false;
        if ((e = allow_big_lds(k_adj_gemm_split<kFP16, true, true>, done))) return e;
        hipLaunchKernelGGL((k_adj_gemm_split<kFP16, true, true>), dim3(sblocks),
                           dim3(64 * kAdjWaves), glds, st, packed, (const uint2 *)gtab->opx, whi,
                           wlo, scale, a.V, a.kb, a.lb, gx, gy, (const uint2 *)gtab->opy, a.Mx,
                           a.My, a.nhx, a.nhy);
      }
    } else if (gen) {
      if (a.prec == kBF16) {
        static bool done = false;
        if ((e = allow_big_lds(k_adj_gemm_split<kBF16, true>, done))) return e;
        hipLaunchKernelGGL((k_adj_gemm_split<kBF16, true>), dim3(sblocks), dim3(64 * kAdjWaves),
                           glds, st, packed, (const uint2 *)gtab->opx, whi, wlo, scale, a.V, a.kb,
                           a.lb, gx, gy, (const uint2 *)gtab->opy, a.Mx, a.My);
      } else {
        static bool done = false;
        if ((e = allow_big_lds(k_adj_gemm_split<kFP16, true>, done))) return e;
        hipLaunchKernelGGL((k_adj_gemm_split<kFP16, true>), dim3(sblocks), dim3(64 * kAdjWaves),
                           glds, st, packed, (const uint2 *)gtab->opx, whi, wlo, scale, a.V, a.kb,
                           a.lb, gx, gy, (const uint2 *)gtab->opy, a.Mx, a.My);
      }
    } else if (a.prec == kBF16) {
      hipLaunchKernelGGL((k_adj_gemm_split<kBF16, false>), dim3(sblocks), dim3(64 * kAdjWaves), 0,
                         st, packed, tb, whi, wlo, scale, a.V, a.kb, a.lb, gx, gy, nullptr, 0, 0);
    } else {
      hipLaunchKernelGGL((k_adj_gemm_split<kFP16, false>), dim3(sblocks), dim3(64 * kAdjWaves), 0,
                         st, packed, tb, whi, wlo, scale, a.V, a.kb, a.lb, gx, gy, nullptr, 0, 0);
    }
  }
  if (main_ev) (void)hipEventRecord(main_ev[1], st);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Pupil loss of the edge-moving optimisation: L = sum |H F - G|^2 over the
// grid, H a real weight (an array, or the indicator of the disc
// k^2 + l^2 <= r2), and its cotangent dL/dRe F + j dL/dIm F = 2 H (H F - G),
// written in the layout of F.  Each block sums its range in FP64 in a fixed
// order; the block partials are added in block order by one more block, so
// the value does not depend on scheduling.
// ---------------------------------------------------------------------------
constexpr int kLossBlocks = 512;

__global__ __launch_bounds__(256) void k_pupil_loss(const float2 *__restrict__ F,
                                                    const float2 *__restrict__ G,
                                                    const float *__restrict__ H, int K, int L,
                                                    double r2, float2 *__restrict__ grad,
                                                    double *__restrict__ part) {
  const int64_t n = (2 * (int64_t)K + 1) * (2 * (int64_t)L + 1);
  const int W = 2 * L + 1;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    double h;
    if (H) {
      h = (double)H[i];
    } else {
      const int k = (int)(i / W) - K, l = (int)(i % W) - L;
      h = r2 < 0.0 || (double)k * k + (double)l * l <= r2 ? 1.0 : 0.0;
    }
    const float2 f = F[i], g = G[i];
    const double dr = h * f.x - g.x, di = h * f.y - g.y;
    acc += dr * dr + di * di;
    grad[i] = make_float2((float)(2.0 * h * dr), (float)(2.0 * h * di));
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_sum_parts(const double *__restrict__ part, int n,
                                                   double *__restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += part[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

size_t pupil_loss_workspace_bytes() { return sizeof(double) * kLossBlocks; }

hipError_t launch_pupil_loss(const float *F, const float *G, const float *H, int K, int L, double r2,
                             double *loss, float *grad, void *ws, hipStream_t st) {
  const int64_t n = (2 * (int64_t)K + 1) * (2 * (int64_t)L + 1);
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kLossBlocks, (n + 255) / 256));
  hipLaunchKernelGGL(k_pupil_loss, dim3(nb), dim3(256), 0, st, (const float2 *)F, (const float2 *)G,
                     H, K, L, r2, (float2 *)grad, (double *)ws);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, st, (const double *)ws, nb, loss);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Edge-offset gradient: each edge collects the gradient of its two corners
// along its normal direction (x for vertical edges, y for horizontal).  Two
// contributions per edge, so the atomic sum is order independent.
// ---------------------------------------------------------------------------
__global__ void k_zero_f32(float *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

__global__ void k_edge_grad(const float *__restrict__ gx, const float *__restrict__ gy,
                            const int64_t *__restrict__ hedge, const int64_t *__restrict__ vedge,
                            int64_t V, int64_t E, float *__restrict__ g_edge) {
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= V) return;
  const int64_t h = hedge[v], e = vedge[v];
  if (h >= 0 && h < E) atomicAdd(&g_edge[h], gy[v]);
  if (e >= 0 && e < E) atomicAdd(&g_edge[e], gx[v]);
}

hipError_t launch_edge_grad(const float *gx, const float *gy, const int64_t *hedge,
                            const int64_t *vedge, int64_t V, int64_t E, float *g_edge,
                            hipStream_t st) {
  if (E > 0)
    hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)((E + 255) / 256)), dim3(256), 0, st, g_edge, E);
  if (V > 0)
    hipLaunchKernelGGL(k_edge_grad, dim3((unsigned)((V + 255) / 256)), dim3(256), 0, st, gx, gy,
                       hedge, vedge, V, E, g_edge);
  return hipGetLastError();
}

// Corner coordinates after edge shifts: a vertical edge moves its two corners
// along x, a horizontal edge along y.  Coordinates are in units of 2^-F
// (grid), offsets in lattice units: the shift is rint(offset 2^F) grid steps.
__global__ void k_apply_offsets(const int32_t *__restrict__ bx, const int32_t *__restrict__ by,
                                const int64_t *__restrict__ hedge, const int64_t *__restrict__ vedge,
                                const float *__restrict__ off, int64_t V, float scale,
                                int32_t *__restrict__ x, int32_t *__restrict__ y) {
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= V) return;
  x[v] = bx[v] + (int32_t)rintf(off[vedge[v]] * scale);
  y[v] = by[v] + (int32_t)rintf(off[hedge[v]] * scale);
}

hipError_t launch_apply_offsets(const int32_t *bx, const int32_t *by, const int64_t *hedge,
                                const int64_t *vedge, const float *off, int64_t V, int32_t *x,
                                int32_t *y, hipStream_t st, int frac_bits) {
  if (V > 0)
    hipLaunchKernelGGL(k_apply_offsets, dim3((unsigned)((V + 255) / 256)), dim3(256), 0, st, bx,
                       by, hedge, vedge, off, V, ldexpf(1.0f, frac_bits), x, y);
  return hipGetLastError();
}

}  // namespace fcfs
