// Device-side helpers shared by the FCFS kernels (gfx950).  Not part of the
// public ABI.
#pragma once

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

}  // namespace fcfs
