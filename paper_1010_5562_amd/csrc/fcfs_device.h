// Device-side helpers shared by the FCFS kernels (gfx950).  Not part of the
// public ABI.
#pragma once

#include "fcfs_internal.h"

namespace fcfs {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr double kPi = 3.14159265358979323846264338327950288;

// ---------------------------------------------------------------------------
// Phase helpers.  A phase is kept as a byte offset into an 8-byte-per-entry
// table of kTabN entries: offset = ((f * xs) mod 8192) * 8, computed exactly in
// 32-bit integers (f < 2^13, xs*8 < 2^16).
// ---------------------------------------------------------------------------
// The multiplies are written as 24-bit integer ops (v_mul/v_mad_u32_u24, full
// rate); plain 32-bit multiplies would become quarter-rate v_mul_lo_u32.
// x side: (f * xs8) mod 65536, the product's high half dropped by the
// sub-dword destination select.
__device__ __forceinline__ uint32_t phase_x(uint32_t f, const uint4 &c) {
  uint32_t r;
  asm("v_mul_u32_u24_sdwa %0, %1, %2 dst_sel:WORD_0 dst_unused:UNUSED_PAD src0_sel:DWORD "
      "src1_sel:DWORD"
      : "=v"(r)
      : "v"(f), "v"(c.x));
  return r;
}
// y side: (f * ys8 + sign offset) mod 65536; padding records are sent to the
// zero entry kTabN.
__device__ __forceinline__ uint32_t phase_y(uint32_t f, const uint4 &c) {
  uint32_t t;
  asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(t) : "v"(f), "v"(c.y), "v"(c.z));
  return (t & 0xFFFFu) | c.w;
}

__device__ __forceinline__ uint2 lds_entry(const uint2 *tab, uint32_t byte_off) {
  return *(const uint2 *)((const char *)tab + byte_off);
}

// Packs 8 table entries (one per k-slot j) into the four MFMA operand
// registers of cos-hi, sin-hi, cos-lo, sin-lo: two 16-bit values per register,
// slot 2j in the low half.  Entry = {hi(c)|hi(s)<<16, lo(c)|lo(s)<<16}.
__device__ __forceinline__ void pack4(const uint2 (&d)[8], u32x4 &ch, u32x4 &sh, u32x4 &cl,
                                      u32x4 &sl) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    ch[j] = __builtin_amdgcn_perm(d[2 * j + 1].x, d[2 * j].x, 0x05040100u);
    sh[j] = __builtin_amdgcn_perm(d[2 * j + 1].x, d[2 * j].x, 0x07060302u);
    cl[j] = __builtin_amdgcn_perm(d[2 * j + 1].y, d[2 * j].y, 0x05040100u);
    sl[j] = __builtin_amdgcn_perm(d[2 * j + 1].y, d[2 * j].y, 0x07060302u);
  }
}

template <int PREC>
__device__ __forceinline__ f32x16 mfma16(const u32x4 &a, const u32x4 &b, const f32x16 &c) {
  if constexpr (PREC == kBF16)
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                  __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
}

// Output grid of one clip: F holds (2 KO + 1) x (2 LO + 1) coefficients,
// k-major, index (KO + k)(2 LO + 1) + (LO + l).  It may be larger than the
// computed band |k| <= K, |l| <= L (the rest is cleared beforehand); with
// r2 >= 0 the entries with k^2 + l^2 > r2 are written as zero (a pupil).
// The factors of alpha_{k,l} (Prop. 3) come with the grid: alpha_{k,l} =
// -g / (4 pi^2 k l), alpha_{k,0} = j ax / (2 pi k), alpha_{0,l} = j ay / (2 pi l),
// F[0,0] = dc * area.  A square tile of period T has g = T, ax = ay = 1,
// dc = 1 / T; a general one carries the sqrt(Nx/Ny)-type factors.
struct OutGrid {
  float2 *F;
  int KO, LO;
  double r2;
  double g, ax, ay, dc;
};

__device__ __forceinline__ void put(const OutGrid &o, int k, int l, float re, float im) {
  if (o.r2 >= 0.0 && (double)k * k + (double)l * l > o.r2) re = im = 0.0f;
  o.F[(size_t)(o.KO + k) * (2 * (size_t)o.LO + 1) + (o.LO + l)] = make_float2(re, im);
}

__device__ __forceinline__ void store_quad(const OutGrid &o, int k, int l, double T, double P,
                                           double U, double R, double Q) {
  (void)T;
  const double a = -o.g / (4.0 * kPi * kPi * (double)k * (double)l);
  const double pre = a * (P - Q), pim = -a * (R + U);  // F[k, l]
  const double mre = -a * (P + Q), mim = a * (R - U);  // F[k, -l]
  put(o, k, l, (float)pre, (float)pim);
  put(o, -k, -l, (float)pre, (float)-pim);
  put(o, k, -l, (float)mre, (float)mim);
  put(o, -k, l, (float)mre, (float)-mim);
}

// A frequency tile whose corner nearest the origin lies outside the pupil
// k^2 + l^2 <= r2 (r2 >= 0) holds only coefficients the epilogue writes as zero:
// its workgroups return at once.
__device__ __forceinline__ bool tile_outside(int tile, int tiles_l, int wgk, int wgl, double r2) {
  if (r2 < 0.0) return false;
  const double k0 = (double)(tile / tiles_l) * wgk, l0 = (double)(tile % tiles_l) * wgl;
  return k0 * k0 + l0 * l0 > r2;
}

// Exact area of a clip from the pre-pass partials (modulo 2^64, exact when
// the area fits in int64), for the whole block: every thread calls it and
// gets the same value.  Blocks of up to 1024 threads (16 waves).
__device__ __forceinline__ long long block_area(const unsigned long long *__restrict__ area_part,
                                                int pre_blocks) {
  __shared__ unsigned long long s_red[16];
  unsigned long long a = 0;
  for (int b = threadIdx.x; b < pre_blocks; b += blockDim.x) a += area_part[b];
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = a;
  __syncthreads();
  unsigned long long t = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += s_red[w];
  __syncthreads();
  return (long long)t;
}

// Inputs of the precision routing of a split-bf16 contraction (route_fp16):
// the pre-pass area partials and both guard factors; gscale_alt = 0 turns the
// routing off.
struct RouteArgs {
  const unsigned long long *area_part;
  int pre_blocks;
  int64_t V;
  double gscale, gscale_alt;
};

// Block-uniform routing decision (every thread of a 256-thread block calls it).
__device__ __forceinline__ bool block_route_fp16(const RouteArgs &r) {
  if (r.gscale_alt <= 0.0) return false;
  return route_fp16(r.gscale, r.gscale_alt, r.V, block_area(r.area_part, r.pre_blocks));
}

// ---------------------------------------------------------------------------
// Contraction building blocks shared by the power-of-two and general-period
// kernels: partial stores, corner loads, raw table entries, MFMA fragments.
// ---------------------------------------------------------------------------
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

// The 8 corners of this lane's half-wave for one 16-corner step.
__device__ __forceinline__ void load_corners(uint4 (&c)[8], const uint4 *__restrict__ vp) {
#pragma unroll
  for (int j = 0; j < 8; ++j) c[j] = vp[j];
}

// Raw table entries of one step: a[kb][j] = W[k x_j], b[lb][j] = s_j W[l y_j].
template <int NKB, int NLB>
struct Raw {
  uint2 a[NKB][8], b[NLB][8];
};

// MFMA operand fragments of one step: 8 corners (the lane's k-slots), two
// 16-bit values per register.  Table entry = {hi(c)|hi(s)<<16, lo(c)|lo(s)<<16}.
template <int NKB, int NLB>
struct Frag {
  u32x4 ach[NKB], acl[NKB], ash[NKB], asl[NKB];
  u32x4 bch[NLB], bcl[NLB], bsh[NLB], bsl[NLB];
};

template <int NKB, int NLB>
__device__ __forceinline__ void build(Frag<NKB, NLB> &f, const Raw<NKB, NLB> &r) {
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb) pack4(r.a[kb], f.ach[kb], f.ash[kb], f.acl[kb], f.asl[kb]);
#pragma unroll
  for (int lb = 0; lb < NLB; ++lb) pack4(r.b[lb], f.bch[lb], f.bsh[lb], f.bcl[lb], f.bsl[lb]);
}

// hi*hi' + hi*lo' + lo*hi' for the four quadrants of every (kb, lb) block.
template <int PREC, int NKB, int NLB>
__device__ __forceinline__ void mma(f32x16 (&acc)[NKB][NLB][4], const Frag<NKB, NLB> &f) {
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
    for (int lb = 0; lb < NLB; ++lb) {
      acc[kb][lb][0] = mfma16<PREC>(f.ach[kb], f.bch[lb], acc[kb][lb][0]);
      acc[kb][lb][1] = mfma16<PREC>(f.ach[kb], f.bsh[lb], acc[kb][lb][1]);
      acc[kb][lb][2] = mfma16<PREC>(f.ash[kb], f.bch[lb], acc[kb][lb][2]);
      acc[kb][lb][3] = mfma16<PREC>(f.ash[kb], f.bsh[lb], acc[kb][lb][3]);
      acc[kb][lb][0] = mfma16<PREC>(f.ach[kb], f.bcl[lb], acc[kb][lb][0]);
      acc[kb][lb][1] = mfma16<PREC>(f.ach[kb], f.bsl[lb], acc[kb][lb][1]);
      acc[kb][lb][2] = mfma16<PREC>(f.ash[kb], f.bcl[lb], acc[kb][lb][2]);
      acc[kb][lb][3] = mfma16<PREC>(f.ash[kb], f.bsl[lb], acc[kb][lb][3]);
      acc[kb][lb][0] = mfma16<PREC>(f.acl[kb], f.bch[lb], acc[kb][lb][0]);
      acc[kb][lb][1] = mfma16<PREC>(f.acl[kb], f.bsh[lb], acc[kb][lb][1]);
      acc[kb][lb][2] = mfma16<PREC>(f.asl[kb], f.bch[lb], acc[kb][lb][2]);
      acc[kb][lb][3] = mfma16<PREC>(f.asl[kb], f.bsh[lb], acc[kb][lb][3]);
    }
}

// ---------------------------------------------------------------------------
// Copy of n 8-byte table entries from device memory into LDS by the whole
// block (blockDim.x threads): 16-byte loads, eight in flight per thread, then
// the stores (src 16-byte aligned; dst 8-byte aligned).  Tables are staged
// once per workgroup, so the loads' latency, not their bandwidth, is the cost.
// ---------------------------------------------------------------------------
template <typename E>
__device__ __forceinline__ void stage_entries(E *dst, const E *__restrict__ src, int n) {
  static_assert(sizeof(E) == 8, "8-byte entries");
  const uint4 *s4 = reinterpret_cast<const uint4 *>(src);
  uint2 *d = reinterpret_cast<uint2 *>(dst);
  const int nt = blockDim.x, n2 = n >> 1;
  int i = threadIdx.x;
  for (; i + 7 * nt < n2; i += 8 * nt) {
    uint4 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = s4[i + u * nt];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      d[2 * (i + u * nt)] = make_uint2(v[u].x, v[u].y);
      d[2 * (i + u * nt) + 1] = make_uint2(v[u].z, v[u].w);
    }
  }
  for (; i < n2; i += nt) {
    const uint4 v = s4[i];
    d[2 * i] = make_uint2(v.x, v.y);
    d[2 * i + 1] = make_uint2(v.z, v.w);
  }
  if ((n & 1) && threadIdx.x == 0) dst[n - 1] = src[n - 1];
}

// The same for tables of at most 16 entries per thread: every thread's
// 16-byte loads (at most eight) are in flight before its first LDS write.
template <typename E>
__device__ __forceinline__ void stage_entries_once(E *dst, const E *__restrict__ src, int n) {
  static_assert(sizeof(E) == 8, "8-byte entries");
  const uint4 *s4 = reinterpret_cast<const uint4 *>(src);
  uint2 *d = reinterpret_cast<uint2 *>(dst);
  const int nt = blockDim.x, n2 = n >> 1;
  if (n2 > 8 * nt) {
    stage_entries(dst, src, n);
    return;
  }
  uint4 v[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int k = threadIdx.x + u * nt;
    if (k < n2) v[u] = s4[k];
  }
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int k = threadIdx.x + u * nt;
    if (k < n2) {
      d[2 * k] = make_uint2(v[u].x, v[u].y);
      d[2 * k + 1] = make_uint2(v[u].z, v[u].w);
    }
  }
  if ((n & 1) && threadIdx.x == 0) dst[n - 1] = src[n - 1];
}

// ---------------------------------------------------------------------------
// Exact phase reduction of one-level general periods (M <= 8192): (f x) mod M
// for x < M and a lane-constant frequency f is
//     f' x - floor(x m / 2^32) M,   f' = f mod M,  m = ceil(f' 2^32 / M),
// exact because x M < 2^32 (the error term x (m - f' 2^32 / M) / 2^32 is below
// x / 2^32 < 1 / M).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t gen_magic(uint32_t fr, uint32_t M) {
  return (uint32_t)((((uint64_t)fr << 32) + M - 1u) / M);
}

// (f x) mod M with fr = f mod M and m = gen_magic(fr, M), for x < M <= 8192.
__device__ __forceinline__ uint32_t gen_phase(uint32_t fr, uint32_t m, uint32_t x, uint32_t M) {
  return __umul24(fr, x) - __umul24(__umulhi(x, m), M);
}

// ---------------------------------------------------------------------------
// Two-level twiddles (periods past 8192): entry p of a table of nh entries of
// Whi followed by kBigLo of Wlo is Whi[p >> kBigBits] x Wlo[p mod kBigLo].
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cmulf(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

__device__ __forceinline__ float2 big_entry(const float2 *t, int nh, uint32_t p) {
  return cmulf(t[p >> kBigBits], t[nh + (p & (uint32_t)(kBigLo - 1))]);
}

__device__ __forceinline__ double2 big_entry64(const double2 *__restrict__ t, int nh, uint32_t p) {
  const double2 a = t[p >> kBigBits], b = t[nh + (p & (uint32_t)(kBigLo - 1))];
  return make_double2(a.x * b.x - a.y * b.y, a.y * b.x + a.x * b.y);
}

// Round to nearest even of an FP32 value to bf16 (bit pattern), finite input.
__device__ __forceinline__ uint32_t bf16_rne(float v) {
  const uint32_t u = __float_as_uint(v);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

// Split entry {hi(c)|hi(s)<<16, lo(c)|lo(s)<<16} of w (the layout of the
// host-built split tables), rounded in the kernel.
template <int PREC>
__device__ __forceinline__ uint2 split_entry(float2 w) {
  if constexpr (PREC == kBF16) {
    const uint32_t hc = bf16_rne(w.x), hs = bf16_rne(w.y);
    const uint32_t lc = bf16_rne(w.x - __uint_as_float(hc << 16));
    const uint32_t ls = bf16_rne(w.y - __uint_as_float(hs << 16));
    return make_uint2(hc | hs << 16, lc | ls << 16);
  } else {
    const _Float16 hc = (_Float16)w.x, hs = (_Float16)w.y;
    const _Float16 lc = (_Float16)(w.x - (float)hc), ls = (_Float16)(w.y - (float)hs);
    return make_uint2((uint32_t)__builtin_bit_cast(uint16_t, hc) |
                          (uint32_t)__builtin_bit_cast(uint16_t, hs) << 16,
                      (uint32_t)__builtin_bit_cast(uint16_t, lc) |
                          (uint32_t)__builtin_bit_cast(uint16_t, ls) << 16);
  }
}

}  // namespace fcfs
