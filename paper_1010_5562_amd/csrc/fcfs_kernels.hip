// HIP kernels of the FCFS forward path for gfx950 (MI355X).
//
// Steps (the four steps of Sec. III-C1, Alg. 2, evaluated directly on the
// corner list instead of through pruned FFTs):
//   pre-pass   exact phase reduction x mod T, y mod T; packing; area (Step 1)
//   axis       F[k,0], F[0,l] first-moment sums in FP64 (Steps 2 and 3)
//   contract   sum_v s_v e(k x_v) e(l y_v) as a real GEMM on MFMA (Step 4)
//   epilogue   split reduction, quadrant unfolding, alpha_{k,l} of Prop. 3,
//              Hermitian fill, axis and DC entries
#include "fcfs_internal.h"

namespace fcfs {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr double kPi = 3.14159265358979323846264338327950288;

// ---------------------------------------------------------------------------
// Phase helpers.  A phase is kept as a byte offset into an 8-byte-per-entry
// table of kTabN entries: offset = ((f * xs) mod 8192) * 8, computed exactly in
// 32-bit integers (f < 2^13, xs*8 < 2^16).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t phase_x(uint32_t f, uint32_t w0) {
  return __umul24(f, w0 & 0xFFFFu) & 0xFFF8u;
}
// y phase with the corner sign folded in (half a period = factor -1) and
// padding corners redirected to the zero entry kTabN.
__device__ __forceinline__ uint32_t phase_y(uint32_t f, uint32_t w0, uint32_t w1) {
  return ((__umul24(f, w0 >> 16) + (w1 & kNegFlag)) & 0xFFF8u) |
         (w1 & kPadFlag);
}

// ---------------------------------------------------------------------------
// Pre-pass: pack corners, exact area.  Corners with index >= V (up to the
// padded count) become padding records.  The area sum is done modulo 2^64,
// which is exact whenever the true area fits in int64.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_prepass(const int32_t *__restrict__ x,
                                                 const int32_t *__restrict__ y,
                                                 const int8_t *__restrict__ s, int64_t V,
                                                 int64_t vpad, uint32_t tmask, int shift,
                                                 uint2 *__restrict__ packed,
                                                 unsigned long long *__restrict__ area_part) {
  unsigned long long acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < vpad;
       i += (int64_t)gridDim.x * 256) {
    uint2 w;
    if (i < V) {
      const int32_t xv = x[i], yv = y[i];
      const int sv = s[i];
      const uint32_t xs = ((uint32_t)xv & tmask) << shift;
      const uint32_t ys = ((uint32_t)yv & tmask) << shift;
      w.x = (xs << 3) | ((ys << 3) << 16);
      w.y = sv < 0 ? kNegFlag : 0u;
      acc += (unsigned long long)((long long)sv * (long long)xv * (long long)yv);
    } else {
      w.x = 0u;
      w.y = kPadFlag;
    }
    packed[i] = w;
  }
  // fixed-order block reduction (integer, exact)
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  __shared__ unsigned long long red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) area_part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

hipError_t launch_prepass(const FwdPlan &p, const int32_t *x, const int32_t *y, const int8_t *s,
                          uint2 *packed, unsigned long long *area_part, hipStream_t st) {
  hipLaunchKernelGGL(k_prepass, dim3(p.pre_blocks), dim3(256), 0, st, x, y, s, p.V, p.vpad,
                     (uint32_t)(p.T - 1), p.shift, packed, area_part);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Axis sums (Steps 2 and 3): for f = 1..K,
//   Sx[f] = sum_v s_v y_v e(f x_v),  and for f = 1..L,  Sy[f] = sum_v s_v x_v e(f y_v),
// with raw (unreduced) coordinates as weights and FP64 twiddles indexed by the
// exact integer phase.  Block (fb, c): 256 frequencies, one vertex chunk;
// partial sums per chunk, reduced in fixed order by the epilogue.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_axis(const int32_t *__restrict__ x,
                                              const int32_t *__restrict__ y,
                                              const uint2 *__restrict__ packed,
                                              const double2 *__restrict__ w64, int64_t V,
                                              int64_t ax_chunk, int K, int L, int kblocks,
                                              double2 *__restrict__ axis_part) {
  __shared__ uint32_t s_ph[256];
  __shared__ double s_wt[256];
  const int fb = blockIdx.x;
  const bool xaxis = fb < kblocks;
  const int f = 1 + (xaxis ? fb : fb - kblocks) * 256 + threadIdx.x;
  const int nf = xaxis ? K : L;
  const int64_t v0 = (int64_t)blockIdx.y * ax_chunk;
  const int64_t v1 = min(V, v0 + ax_chunk);
  double re = 0.0, im = 0.0;
  for (int64_t vb = v0; vb < v1; vb += 256) {
    const int64_t v = vb + threadIdx.x;
    uint32_t ph = 0;
    double wt = 0.0;
    if (v < v1) {
      const uint2 w = packed[v];
      const double sg = (w.y & kNegFlag) ? -1.0 : 1.0;
      if (xaxis) {
        ph = (w.x & 0xFFFFu) >> 3;
        wt = sg * (double)y[v];
      } else {
        ph = w.x >> 19;
        wt = sg * (double)x[v];
      }
    }
    __syncthreads();
    s_ph[threadIdx.x] = ph;
    s_wt[threadIdx.x] = wt;
    __syncthreads();
    const int n = (int)min((int64_t)256, v1 - vb);
    if (f <= nf) {
      for (int j = 0; j < n; ++j) {
        const uint32_t idx = ((uint32_t)f * s_ph[j]) & (kTabN - 1);
        const double2 t = w64[idx];
        re = fma(s_wt[j], t.x, re);
        im = fma(-s_wt[j], t.y, im);
      }
    }
  }
  if (f <= nf) {
    const int slot = xaxis ? f - 1 : K + f - 1;
    axis_part[(size_t)blockIdx.y * (K + L) + slot] = make_double2(re, im);
  }
}

hipError_t launch_axis(const FwdPlan &p, const int32_t *x, const int32_t *y, const int8_t *s,
                       const uint2 *packed, const double2 *w64, double2 *axis_part,
                       hipStream_t st) {
  (void)s;
  if (p.K + p.L == 0 || p.ax_chunks == 0) return hipSuccess;
  const int kblocks = (p.K + 255) / 256, lblocks = (p.L + 255) / 256;
  hipLaunchKernelGGL(k_axis, dim3(kblocks + lblocks, p.ax_chunks), dim3(256), 0, st, x, y,
                     packed, w64, p.V, p.ax_chunk, p.K, p.L, kblocks, axis_part);
  return hipGetLastError();
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
__device__ __forceinline__ uint2 lds_entry(const uint2 *tab, uint32_t byte_off) {
  return *(const uint2 *)((const char *)tab + byte_off);
}

template <int NKB, int NLB>
__device__ __forceinline__ void store_part(float *__restrict__ part, const f32x16 (&acc)[NKB][NLB][4],
                                           int split, int kp, int lp, int k0, int l0, int li,
                                           int lh) {
  const size_t plane = (size_t)kp * lp;
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
    for (int lb = 0; lb < NLB; ++lb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float *base = part + ((size_t)split * 4 + q) * plane + (size_t)(l0 + 32 * lb + li);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = k0 + 32 * kb + 8 * (r >> 2) + 4 * lh + (r & 3);
          base[(size_t)row * lp] = acc[kb][lb][q][r];
        }
      }
}

template <int PREC, int NKB, int NLB>
__global__ __launch_bounds__(256) void k_contract_split(const uint2 *__restrict__ packed,
                                                        const uint2 *__restrict__ tab,
                                                        int64_t chunk, int tiles_l, int kp,
                                                        int lp, float *__restrict__ part) {
  __shared__ uint2 s_tab[kTabEntries];
  for (int i = threadIdx.x; i < kTabEntries; i += 256) s_tab[i] = tab[i];
  __syncthreads();

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

  const u32x4 *vp = (const u32x4 *)(packed + (size_t)split * chunk + 8 * lh);
  for (int64_t vb = 0; vb < chunk; vb += 16) {
    // this lane's 8 corners: vb + 8*lh + j
    uint32_t w0[8], w1[8];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const u32x4 q = vp[(vb >> 1) + j];
      w0[2 * j] = q.x;
      w1[2 * j] = q.y;
      w0[2 * j + 1] = q.z;
      w1[2 * j + 1] = q.w;
    }
    u32x4 ach[NKB], acl[NKB], ash[NKB], asl[NKB];
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) {
      uint2 d[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) d[j] = lds_entry(s_tab, phase_x(kf[kb], w0[j]));
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        ach[kb][j] = __builtin_amdgcn_perm(d[2 * j + 1].x, d[2 * j].x, 0x05040100u);
        ash[kb][j] = __builtin_amdgcn_perm(d[2 * j + 1].x, d[2 * j].x, 0x07060302u);
        acl[kb][j] = __builtin_amdgcn_perm(d[2 * j + 1].y, d[2 * j].y, 0x05040100u);
        asl[kb][j] = __builtin_amdgcn_perm(d[2 * j + 1].y, d[2 * j].y, 0x07060302u);
      }
    }
    u32x4 bch[NLB], bcl[NLB], bsh[NLB], bsl[NLB];
#pragma unroll
    for (int lb = 0; lb < NLB; ++lb) {
      uint2 d[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) d[j] = lds_entry(s_tab, phase_y(lf[lb], w0[j], w1[j]));
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        bch[lb][j] = __builtin_amdgcn_perm(d[2 * j + 1].x, d[2 * j].x, 0x05040100u);
        bsh[lb][j] = __builtin_amdgcn_perm(d[2 * j + 1].x, d[2 * j].x, 0x07060302u);
        bcl[lb][j] = __builtin_amdgcn_perm(d[2 * j + 1].y, d[2 * j].y, 0x05040100u);
        bsl[lb][j] = __builtin_amdgcn_perm(d[2 * j + 1].y, d[2 * j].y, 0x07060302u);
      }
    }
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
      for (int lb = 0; lb < NLB; ++lb) {
        if constexpr (PREC == kBF16) {
#define MF(A, B, C) \
  C = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, A), __builtin_bit_cast(bf16x8, B), C, 0, 0, 0)
          MF(ach[kb], bch[lb], acc[kb][lb][0]);
          MF(ach[kb], bcl[lb], acc[kb][lb][0]);
          MF(acl[kb], bch[lb], acc[kb][lb][0]);
          MF(ach[kb], bsh[lb], acc[kb][lb][1]);
          MF(ach[kb], bsl[lb], acc[kb][lb][1]);
          MF(acl[kb], bsh[lb], acc[kb][lb][1]);
          MF(ash[kb], bch[lb], acc[kb][lb][2]);
          MF(ash[kb], bcl[lb], acc[kb][lb][2]);
          MF(asl[kb], bch[lb], acc[kb][lb][2]);
          MF(ash[kb], bsh[lb], acc[kb][lb][3]);
          MF(ash[kb], bsl[lb], acc[kb][lb][3]);
          MF(asl[kb], bsh[lb], acc[kb][lb][3]);
#undef MF
        } else {
#define MF(A, B, C) \
  C = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, A), __builtin_bit_cast(f16x8, B), C, 0, 0, 0)
          MF(ach[kb], bch[lb], acc[kb][lb][0]);
          MF(ach[kb], bcl[lb], acc[kb][lb][0]);
          MF(acl[kb], bch[lb], acc[kb][lb][0]);
          MF(ach[kb], bsh[lb], acc[kb][lb][1]);
          MF(ach[kb], bsl[lb], acc[kb][lb][1]);
          MF(acl[kb], bsh[lb], acc[kb][lb][1]);
          MF(ash[kb], bch[lb], acc[kb][lb][2]);
          MF(ash[kb], bcl[lb], acc[kb][lb][2]);
          MF(asl[kb], bch[lb], acc[kb][lb][2]);
          MF(ash[kb], bsh[lb], acc[kb][lb][3]);
          MF(ash[kb], bsl[lb], acc[kb][lb][3]);
          MF(asl[kb], bsh[lb], acc[kb][lb][3]);
#undef MF
        }
      }
  }
  store_part<NKB, NLB>(part, acc, split, kp, lp, k0, l0, li, lh);
}

// FP32 form: v_mfma_f32_32x32x2_f32, two corners per product (lanes 0-31
// carry corner j of the lane's group, lanes 32-63 corner 8 + j).
template <int NKB, int NLB>
__global__ __launch_bounds__(256) void k_contract_fp32(const uint2 *__restrict__ packed,
                                                       const float2 *__restrict__ tab,
                                                       int64_t chunk, int tiles_l, int kp, int lp,
                                                       float *__restrict__ part) {
  __shared__ float2 s_tab[kTabEntries];
  for (int i = threadIdx.x; i < kTabEntries; i += 256) s_tab[i] = tab[i];
  __syncthreads();

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

  const u32x4 *vp = (const u32x4 *)(packed + (size_t)split * chunk + 8 * lh);
  for (int64_t vb = 0; vb < chunk; vb += 16) {
    uint32_t w0[8], w1[8];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const u32x4 q = vp[(vb >> 1) + j];
      w0[2 * j] = q.x;
      w1[2 * j] = q.y;
      w0[2 * j + 1] = q.z;
      w1[2 * j + 1] = q.w;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      float2 a[NKB], b[NLB];
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb)
        a[kb] = *(const float2 *)((const char *)s_tab + phase_x(kf[kb], w0[j]));
#pragma unroll
      for (int lb = 0; lb < NLB; ++lb)
        b[lb] = *(const float2 *)((const char *)s_tab + phase_y(lf[lb], w0[j], w1[j]));
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
  store_part<NKB, NLB>(part, acc, split, kp, lp, k0, l0, li, lh);
}

// Tile variants: (id, precision mask, k per wave, l per wave).
static const TileVariant kVariants[] = {
    {0, 0x7, 32, 32},
    {1, 0x7, 64, 32},
    {2, 0x7, 64, 64},
};

int n_tile_variants() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }
const TileVariant &tile_variant(int i) { return kVariants[i]; }

template <int NKB, int NLB>
static void launch_contract_t(const FwdPlan &p, const uint2 *packed, const Tables &t, float *part,
                              hipStream_t st) {
  dim3 grid(p.tiles_k * p.tiles_l, p.nsplit), block(256);
  if (p.prec == kFP32)
    hipLaunchKernelGGL((k_contract_fp32<NKB, NLB>), grid, block, 0, st, packed, t.w32, p.chunk,
                       p.tiles_l, p.kp, p.lp, part);
  else if (p.prec == kBF16)
    hipLaunchKernelGGL((k_contract_split<kBF16, NKB, NLB>), grid, block, 0, st, packed, t.wbf16,
                       p.chunk, p.tiles_l, p.kp, p.lp, part);
  else
    hipLaunchKernelGGL((k_contract_split<kFP16, NKB, NLB>), grid, block, 0, st, packed, t.wfp16,
                       p.chunk, p.tiles_l, p.kp, p.lp, part);
}

hipError_t launch_contract(const FwdPlan &p, const uint2 *packed, const Tables &t, float *part,
                           hipStream_t st) {
  switch (p.tile) {
    case 0: launch_contract_t<1, 1>(p, packed, t, part, st); break;
    case 1: launch_contract_t<2, 1>(p, packed, t, part, st); break;
    case 2: launch_contract_t<2, 2>(p, packed, t, part, st); break;
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
// Split partials are summed in FP64 in a fixed order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_epilogue(const float *__restrict__ part, int nsplit, int kp,
                                                  int lp, int K, int L, double T,
                                                  float2 *__restrict__ F) {
  const int l = 1 + blockIdx.x * 256 + threadIdx.x;
  const int k = 1 + blockIdx.y;
  if (l > L) return;
  const size_t plane = (size_t)kp * lp;
  const size_t o = (size_t)k * lp + l;
  double P = 0.0, U = 0.0, R = 0.0, Q = 0.0;
  for (int s = 0; s < nsplit; ++s) {
    const float *b = part + (size_t)s * 4 * plane + o;
    P += (double)b[0];
    U += (double)b[plane];
    R += (double)b[2 * plane];
    Q += (double)b[3 * plane];
  }
  const double a = -T / (4.0 * kPi * kPi * (double)k * (double)l);
  const double pre = a * (P - Q), pim = -a * (R + U);  // F[k, l]
  const double mre = -a * (P + Q), mim = a * (R - U);  // F[k, -l]
  const size_t W = 2 * (size_t)L + 1;
  F[(size_t)(K + k) * W + (L + l)] = make_float2((float)pre, (float)pim);
  F[(size_t)(K - k) * W + (L - l)] = make_float2((float)pre, (float)-pim);
  F[(size_t)(K + k) * W + (L - l)] = make_float2((float)mre, (float)mim);
  F[(size_t)(K - k) * W + (L + l)] = make_float2((float)mre, (float)-mim);
}

// Axis entries (Steps 2, 3) and DC (Step 1):
//   F[k,0] = j/(2 pi k) Sx[k],  F[-k,0] = conj F[k,0];  likewise F[0,l];
//   F[0,0] = area / T.
__global__ __launch_bounds__(256) void k_epilogue_axes(const double2 *__restrict__ axis_part,
                                                       int ax_chunks, int K, int L, double T,
                                                       const unsigned long long *__restrict__ area_part,
                                                       int pre_blocks, float2 *__restrict__ F,
                                                       int64_t *__restrict__ area) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const size_t W = 2 * (size_t)L + 1;
  if (i < K + L) {
    double re = 0.0, im = 0.0;
    for (int c = 0; c < ax_chunks; ++c) {
      const double2 v = axis_part[(size_t)c * (K + L) + i];
      re += v.x;
      im += v.y;
    }
    const int f = i < K ? i + 1 : i - K + 1;
    const double sc = 1.0 / (2.0 * kPi * (double)f);
    const float fre = (float)(-im * sc), fim = (float)(re * sc);
    if (i < K) {
      F[(size_t)(K + f) * W + L] = make_float2(fre, fim);
      F[(size_t)(K - f) * W + L] = make_float2(fre, -fim);
    } else {
      F[(size_t)K * W + (L + f)] = make_float2(fre, fim);
      F[(size_t)K * W + (L - f)] = make_float2(fre, -fim);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x < 64) {
    unsigned long long a = 0;
    for (int b = threadIdx.x; b < pre_blocks; b += 64) a += area_part[b];
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    if (threadIdx.x == 0) {
      const long long A = (long long)a;
      F[(size_t)K * W + L] = make_float2((float)((double)A / T), 0.0f);
      if (area) *area = A;
    }
  }
}

hipError_t launch_epilogue(const FwdPlan &p, const float *part, const double2 *axis_part,
                           const unsigned long long *area_part, float *F, int64_t *area,
                           hipStream_t st) {
  float2 *F2 = (float2 *)F;
  const int nax = (p.K + p.L + 255) / 256;
  hipLaunchKernelGGL(k_epilogue_axes, dim3(nax > 0 ? nax : 1), dim3(256), 0, st, axis_part,
                     p.ax_chunks, p.K, p.L, (double)p.T, area_part, p.pre_blocks, F2, area);
  if (p.K > 0 && p.L > 0)
    hipLaunchKernelGGL(k_epilogue, dim3((p.L + 255) / 256, p.K), dim3(256), 0, st, part,
                       p.nsplit, p.kp, p.lp, p.K, p.L, (double)p.T, F2);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Debug export of the integer phases used by the contraction:
// out[i*V + v] = ((k0+i) * x_v) mod T  (axis 0) or with y_v (axis 1, the
// sign-free phase), recovered from the same byte offsets the kernels use.
// ---------------------------------------------------------------------------
__global__ void k_debug_phases(const uint2 *__restrict__ packed, int64_t V, int axis, int k0,
                               int nk, int shift, int32_t *__restrict__ out) {
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int i = blockIdx.y;
  if (v >= V || i >= nk) return;
  const uint2 w = packed[v];
  const uint32_t f = (uint32_t)(k0 + i);
  const uint32_t b = axis == 0 ? phase_x(f, w.x) : phase_y(f, w.x, 0u);
  out[(size_t)i * V + v] = (int32_t)((b >> 3) >> shift);
}

hipError_t launch_debug_phases(const FwdPlan &p, const uint2 *packed, int axis, int k0, int nk,
                               int32_t *out, hipStream_t st) {
  if (p.V == 0 || nk == 0) return hipSuccess;
  hipLaunchKernelGGL(k_debug_phases, dim3((unsigned)((p.V + 255) / 256), nk), dim3(256), 0, st,
                     packed, p.V, axis, k0, nk, p.shift, out);
  return hipGetLastError();
}

}  // namespace fcfs
