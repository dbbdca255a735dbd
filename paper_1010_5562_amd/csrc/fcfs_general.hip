// Vertex contraction (Step 4 of Sec. III-C1) for a general tile: periods Mx
// along x and My along y, any integers in [2, 8192], not only powers of two,
// and not necessarily equal (Prop. 3 with w_x = 2 pi / Nx, w_y = 2 pi / Ny;
// vertices on a finer grid are handled by scaling the periods, see the API).
//
// The same real-trigonometric GEMM as the power-of-two kernels: per (k, l)
// the four sums P, U, R, Q of s_v (cos, sin)(2 pi k x_v / Mx) x
// (cos, sin)(2 pi l y_v / My) on MFMA, operands gathered from per-period
// tables in LDS.  What differs is the exact phase reduction: (f x) mod M for
// x < M and a lane-constant frequency f is
//     f' x - floor(x m / 2^32) M,   f' = f mod M,  m = ceil(f' 2^32 / M),
// exact because x M < 2^32 (the error term x (m - f' 2^32 / M) / 2^32 is below
// x / 2^32 < 1 / M).  The sign s_v flips the sign bits of the y-side entry
// (record field z) and padding records send the x-side lookup to the zero
// entry (record field w = 8 Mx, added before the clamp to Mx).
//
// Two kernels.  Eight-wave form (FP32, and the split precisions on request):
// 8 waves (2 in k x 4 in l), each 64 k x 32 l, so a 128 x 128 frequency tile;
// one or two workgroups per CU depending on the table sizes (at most
// (8193 + 8192) 8-byte entries of LDS), i.e. two waves per SIMD or more.
// Pipelined form (the split precisions): 4 waves of 64 x 64, one per SIMD,
// software-pipelined as the power-of-two production kernel.
#include "fcfs_device.h"

namespace fcfs {
namespace {

constexpr int kGenWaves = 8;
constexpr int kGenNKB = 2, kGenNLB = 1;

template <int NKB, int NLB>
struct GenLane {
  uint32_t kr[NKB], km[NKB], lr[NLB], lm[NLB];
};

// Phase constants of the lane's frequencies k0 + 32 kb + li and l0 + 32 lb + li.
template <int NKB, int NLB>
__device__ __forceinline__ void gen_lane(GenLane<NKB, NLB> &g, int k0, int l0, int li,
                                         uint32_t ux, uint32_t uy) {
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb) {
    g.kr[kb] = (uint32_t)(k0 + 32 * kb + li) % ux;
    g.km[kb] = gen_magic(g.kr[kb], ux);
  }
#pragma unroll
  for (int lb = 0; lb < NLB; ++lb) {
    g.lr[lb] = (uint32_t)(l0 + 32 * lb + li) % uy;
    g.lm[lb] = gen_magic(g.lr[lb], uy);
  }
}

// Entries of one 16-corner step: a[kb][j] = Wx[(k x_j) mod Mx] (zero for
// padding), b[lb][j] = s_j Wy[(l y_j) mod My].
template <typename E>
__device__ __forceinline__ E flip(E e, uint32_t m) {
  uint2 u = __builtin_bit_cast(uint2, e);
  u.x ^= m;
  u.y ^= m;
  return __builtin_bit_cast(E, u);
}

template <typename E, int NKB, int NLB>
__device__ __forceinline__ void gen_gather(E (&a)[NKB][8], E (&b)[NLB][8], const E *tx,
                                           const E *ty, const uint4 (&c)[8],
                                           const GenLane<NKB, NLB> &g, uint32_t Mx, uint32_t My) {
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
    for (int j = 0; j < 8; ++j)
      a[kb][j] = tx[min(gen_phase(g.kr[kb], g.km[kb], c[j].x, Mx) + c[j].w, Mx)];
#pragma unroll
  for (int lb = 0; lb < NLB; ++lb)
#pragma unroll
    for (int j = 0; j < 8; ++j) b[lb][j] = flip(ty[gen_phase(g.lr[lb], g.lm[lb], c[j].y, My)], c[j].z);
}

// Both period tables in LDS (one when they coincide): Mx + 1 entries of tabx
// (the last the zero entry), then My of taby.
template <typename E>
__device__ __forceinline__ E *stage_gen_tables(E *tx, const void *__restrict__ tabx,
                                               const void *__restrict__ taby, int Mx, int My) {
  E *ty = tabx == taby ? tx : tx + (Mx + 1);
  stage_entries(tx, static_cast<const E *>(tabx), Mx + 1);
  if (tabx != taby) stage_entries(ty, static_cast<const E *>(taby), My);
  __syncthreads();
  return ty;
}

// PREC: kBF16 / kFP16 (E = uint2 split entries) or kFP32 (E = float2).
template <int PREC>
__device__ __forceinline__ void contract_gen_body(
    const uint4 *__restrict__ packed,
    const typename std::conditional<PREC == kFP32, float2, uint2>::type *tx,
    const typename std::conditional<PREC == kFP32, float2, uint2>::type *ty, int Mx, int My,
    int64_t chunk, int tiles_l, int kp, int lp, float *__restrict__ part) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 31, lh = lane >> 5;
  const int tk = blockIdx.x / tiles_l, tl = blockIdx.x % tiles_l;
  const int split = blockIdx.y;
  const int k0 = tk * 128 + (wave >> 2) * 64;
  const int l0 = tl * 128 + (wave & 3) * 32;
  const uint32_t ux = (uint32_t)Mx, uy = (uint32_t)My;
  GenLane<kGenNKB, kGenNLB> g;
  gen_lane(g, k0, l0, li, ux, uy);

  f32x16 acc[kGenNKB][kGenNLB][4];
#pragma unroll
  for (int kb = 0; kb < kGenNKB; ++kb)
#pragma unroll
    for (int lb = 0; lb < kGenNLB; ++lb)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[kb][lb][q][r] = 0.0f;

  const uint4 *vp = packed + (size_t)split * chunk + 8 * lh;
  for (int64_t vb = 0; vb < chunk; vb += 16) {
    uint4 c[8];
    load_corners(c, vp + vb);
    if constexpr (PREC == kFP32) {
      float2 a[kGenNKB][8], b[kGenNLB][8];
      gen_gather(a, b, tx, ty, c, g, ux, uy);
#pragma unroll
      for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int kb = 0; kb < kGenNKB; ++kb)
#pragma unroll
          for (int lb = 0; lb < kGenNLB; ++lb) {
            acc[kb][lb][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[kb][j].x, b[lb][j].x, acc[kb][lb][0], 0, 0, 0);
            acc[kb][lb][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[kb][j].x, b[lb][j].y, acc[kb][lb][1], 0, 0, 0);
            acc[kb][lb][2] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[kb][j].y, b[lb][j].x, acc[kb][lb][2], 0, 0, 0);
            acc[kb][lb][3] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[kb][j].y, b[lb][j].y, acc[kb][lb][3], 0, 0, 0);
          }
    } else {
      Raw<kGenNKB, kGenNLB> raw;
      gen_gather(raw.a, raw.b, tx, ty, c, g, ux, uy);
      Frag<kGenNKB, kGenNLB> f;
      build(f, raw);
      mma<PREC>(acc, f);
    }
  }
  store_part<kGenNKB, kGenNLB>(part, acc, split, kp, lp, k0, l0, li, lh);
}

// Split-bf16 launches take the split-fp16 tables of both periods as well: a
// clip the rounding model routes to split-fp16 (block_route_fp16) runs the
// fp16 form.
template <int PREC>
__global__ __launch_bounds__(64 * kGenWaves) void k_contract_gen(
    const uint4 *__restrict__ packed, const void *__restrict__ tabx, const void *__restrict__ taby,
    int Mx, int My, int64_t chunk, int tiles_l, int kp, int lp, float *__restrict__ part,
    double r2, RouteArgs ra, const void *__restrict__ tabx16, const void *__restrict__ taby16) {
  if (tile_outside(blockIdx.x, tiles_l, 128, 128, r2)) return;
  using E = typename std::conditional<PREC == kFP32, float2, uint2>::type;
  extern __shared__ uint2 lds[];
  if constexpr (PREC == kBF16) {
    if (block_route_fp16(ra)) {
      const uint2 *ty = stage_gen_tables<uint2>(lds, tabx16, taby16, Mx, My);
      contract_gen_body<kFP16>(packed, lds, ty, Mx, My, chunk, tiles_l, kp, lp, part);
      return;
    }
  }
  E *tx = reinterpret_cast<E *>(lds);
  const E *ty = stage_gen_tables<E>(tx, tabx, taby, Mx, My);
  contract_gen_body<PREC>(packed, tx, ty, Mx, My, chunk, tiles_l, kp, lp, part);
}

// Byte offset base + 8 ((f x) mod M) of the table entry, from the lane
// constants fr8 = 8 (f mod M), m = gen_magic(f mod M, M) and M8 = 8 M: the
// quotient is that of gen_phase, and both 24-bit products stay below 2^29.
__device__ __forceinline__ uint32_t gen_phase8(uint32_t fr8, uint32_t m, uint32_t x, uint32_t M8,
                                               uint32_t base) {
  return (__umul24(fr8, x) + base) - __umul24(__umulhi(x, m), M8);
}

// gen_gather for the pipelined kernel, with LDS byte addresses: the x table at
// byte 0 (padding records, w = 8 Mx, land on its zero entry at byte 8 Mx), the
// y table at byte ybase.
__device__ __forceinline__ void gen_gather8(Raw<2, 2> &r, const uint2 *lds,
                                            const uint4 (&c)[8], const uint32_t (&kr8)[2],
                                            const uint32_t (&km)[2], const uint32_t (&lr8)[2],
                                            const uint32_t (&lm)[2], uint32_t Mx8, uint32_t My8,
                                            uint32_t ybase) {
#pragma unroll
  for (int kb = 0; kb < 2; ++kb)
#pragma unroll
    for (int j = 0; j < 8; ++j)
      r.a[kb][j] = lds_entry(lds, min(gen_phase8(kr8[kb], km[kb], c[j].x, Mx8, c[j].w), Mx8));
#pragma unroll
  for (int lb = 0; lb < 2; ++lb)
#pragma unroll
    for (int j = 0; j < 8; ++j)
      r.b[lb][j] = flip(lds_entry(lds, gen_phase8(lr8[lb], lm[lb], c[j].y, My8, ybase)), c[j].z);
}

// Software-pipelined split form for one wave per SIMD, as the power-of-two
// production kernel: 4 waves of 64 x 64 frequencies (128 x 128 per
// workgroup), the 48 MFMAs of step s interleaved with the lookups and packing
// of step s+1 and the corner loads of step s+2.  chunk is a multiple of 32.
__device__ __forceinline__ void gen_pipe_schedule() {
  constexpr int NM = 48;                 // MFMAs per step
  constexpr int ND = 32;                 // LDS lookups per step
  constexpr int NV = 16 * 5 + 16 * 6 + 64;  // phases, clamps, sign flips, packing
#pragma unroll
  for (int i = 0; i < NM; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                   // MFMA
    if (i % 6 == 0) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);   // corner load
    if (i < ND / 2) __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);   // LDS lookups
    __builtin_amdgcn_sched_group_barrier(0x002, (NV + NM - 1) / NM, 0);  // VALU
  }
}

// lds: both tables staged (a static array at LDS address 0, so the lookups
// need no base add); one_tab: the two periods share one table.
template <int PREC>
__device__ __forceinline__ void contract_gen_pipe_body(const uint2 *lds, bool one_tab,
                                                       const uint4 *__restrict__ packed, int Mx,
                                                       int My, int64_t chunk, int tiles_l, int kp,
                                                       int lp, float *__restrict__ part, int tile,
                                                       int split) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 31, lh = lane >> 5;
  const int tk = tile / tiles_l, tl = tile % tiles_l;
  const int k0 = tk * 128 + (wave >> 1) * 64;
  const int l0 = tl * 128 + (wave & 1) * 64;
  const uint32_t ux = (uint32_t)Mx, uy = (uint32_t)My;
  GenLane<2, 2> g;
  gen_lane(g, k0, l0, li, ux, uy);
  const uint32_t kr8[2] = {g.kr[0] << 3, g.kr[1] << 3}, lr8[2] = {g.lr[0] << 3, g.lr[1] << 3};
  const uint32_t Mx8 = ux << 3, My8 = uy << 3;
  const uint32_t ybase = one_tab ? 0u : Mx8 + 8u;

  f32x16 acc[2][2][4];
#pragma unroll
  for (int kb = 0; kb < 2; ++kb)
#pragma unroll
    for (int lb = 0; lb < 2; ++lb)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[kb][lb][q][r] = 0.0f;

  const uint4 *vp = packed + (size_t)split * chunk + 8 * lh;
  const int nsteps = (int)(chunk >> 4);  // even
  const int last = nsteps - 1;
  uint4 c0[8], c1[8];
  Raw<2, 2> raw;
  Frag<2, 2> fa, fb;
  load_corners(c0, vp);
  gen_gather8(raw, lds, c0, kr8, g.km, lr8, g.lm, Mx8, My8, ybase);
  build(fa, raw);
  load_corners(c1, vp + 16);
  for (int s = 0; s < nsteps; s += 2) {
    // fa: operands of step s; c1: corners of step s+1
    load_corners(c0, vp + 16 * min(s + 2, last));
    gen_gather8(raw, lds, c1, kr8, g.km, lr8, g.lm, Mx8, My8, ybase);
    build(fb, raw);
    mma<PREC>(acc, fa);
    gen_pipe_schedule();
    // fb: operands of step s+1; c0: corners of step s+2 (the last iteration
    // prepares a step that is never multiplied)
    load_corners(c1, vp + 16 * min(s + 3, last));
    gen_gather8(raw, lds, c0, kr8, g.km, lr8, g.lm, Mx8, My8, ybase);
    build(fa, raw);
    mma<PREC>(acc, fb);
    gen_pipe_schedule();
  }
  store_part<2, 2>(part, acc, split, kp, lp, k0, l0, li, lh);
}

template <int PREC>
__global__ __launch_bounds__(256, 1) void k_contract_gen_pipe(
    const uint4 *__restrict__ packed, const uint2 *__restrict__ tabx,
    const uint2 *__restrict__ taby, int Mx, int My, int64_t chunk, int tiles_l, int kp, int lp,
    float *__restrict__ part, double r2, RouteArgs ra, const uint2 *__restrict__ tabx16,
    const uint2 *__restrict__ taby16) {
  if (tile_outside(blockIdx.x, tiles_l, 128, 128, r2)) return;
  // large enough for both tables
  __shared__ uint2 lds[2 * kTabN + 1];
  if constexpr (PREC == kBF16) {
    if (block_route_fp16(ra)) {
      stage_gen_tables<uint2>(lds, tabx16, taby16, Mx, My);
      contract_gen_pipe_body<kFP16>(lds, tabx16 == taby16, packed, Mx, My, chunk, tiles_l, kp,
                                    lp, part, blockIdx.x, blockIdx.y);
      return;
    }
  }
  stage_gen_tables<uint2>(lds, tabx, taby, Mx, My);
  contract_gen_pipe_body<PREC>(lds, tabx == taby, packed, Mx, My, chunk, tiles_l, kp, lp, part,
                               blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------------------
// Periods past 8192 grid units (two-level twiddles).  The eight-wave layout
// of k_contract_gen; per entry the phase (f x) mod M is reduced exactly in
// 32-bit integers from the corner's magic (big_phase_int) and the twiddle is
// the FP32 complex product of the two table entries (both tables of both
// periods in LDS, at most 4 x 4096 entries).  The split precisions round that
// product to hi + lo in the kernel (the FP32 product is accurate to a few
// 2^-24, far below the split's own rounding).  This form serves FP32, and the
// split precisions where the shared-operand kernel below does not fit in LDS.
// ---------------------------------------------------------------------------
template <int PREC, bool NARROW>
__device__ __forceinline__ void contract_big_body(const uint4 *__restrict__ phi,
                                                  const float2 *tx, const float2 *ty, int Mx,
                                                  int My, int nhx, int nhy, int64_t chunk,
                                                  int tiles_l, int kp, int lp,
                                                  float *__restrict__ part) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 31, lh = lane >> 5;
  const int tk = blockIdx.x / tiles_l, tl = blockIdx.x % tiles_l;
  const int split = blockIdx.y;
  const int k0 = tk * 128 + (wave >> 2) * 64;
  const int l0 = tl * 128 + (wave & 3) * 32;
  const uint32_t Mxm1 = (uint32_t)Mx - 1u, Mym1 = (uint32_t)My - 1u;
  uint32_t kf[kGenNKB], lf[kGenNLB];
#pragma unroll
  for (int kb = 0; kb < kGenNKB; ++kb) kf[kb] = (uint32_t)(k0 + 32 * kb + li);
#pragma unroll
  for (int lb = 0; lb < kGenNLB; ++lb) lf[lb] = (uint32_t)(l0 + 32 * lb + li);

  f32x16 acc[kGenNKB][kGenNLB][4];
#pragma unroll
  for (int kb = 0; kb < kGenNKB; ++kb)
#pragma unroll
    for (int lb = 0; lb < kGenNLB; ++lb)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[kb][lb][q][r] = 0.0f;

  const uint4 *pp = phi + (size_t)split * chunk + 8 * lh;
  for (int64_t vb = 0; vb < chunk; vb += 16) {
    uint4 m[8];
    load_corners(m, pp + vb);
    float2 a[kGenNKB][8], b[kGenNLB][8];
#pragma unroll
    for (int kb = 0; kb < kGenNKB; ++kb)
#pragma unroll
      for (int j = 0; j < 8; ++j)
        a[kb][j] = m[j].z >> 31 ? make_float2(0.0f, 0.0f)
                                : big_entry(tx, nhx,
                                            big_word_phase<NARROW, true>(kf[kb], m[j], Mxm1, -Mx));
#pragma unroll
    for (int lb = 0; lb < kGenNLB; ++lb)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float2 w = big_entry(ty, nhy, big_word_phase<NARROW, false>(lf[lb], m[j], Mym1, -My));
        b[lb][j] = (m[j].z >> 30) & 1u ? make_float2(-w.x, -w.y) : w;
      }
    if constexpr (PREC == kFP32) {
#pragma unroll
      for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int kb = 0; kb < kGenNKB; ++kb)
#pragma unroll
          for (int lb = 0; lb < kGenNLB; ++lb) {
            acc[kb][lb][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[kb][j].x, b[lb][j].x, acc[kb][lb][0], 0, 0, 0);
            acc[kb][lb][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[kb][j].x, b[lb][j].y, acc[kb][lb][1], 0, 0, 0);
            acc[kb][lb][2] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[kb][j].y, b[lb][j].x, acc[kb][lb][2], 0, 0, 0);
            acc[kb][lb][3] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[kb][j].y, b[lb][j].y, acc[kb][lb][3], 0, 0, 0);
          }
    } else {
      Raw<kGenNKB, kGenNLB> raw;
#pragma unroll
      for (int kb = 0; kb < kGenNKB; ++kb)
#pragma unroll
        for (int j = 0; j < 8; ++j) raw.a[kb][j] = split_entry<PREC>(a[kb][j]);
#pragma unroll
      for (int lb = 0; lb < kGenNLB; ++lb)
#pragma unroll
        for (int j = 0; j < 8; ++j) raw.b[lb][j] = split_entry<PREC>(b[lb][j]);
      Frag<kGenNKB, kGenNLB> f;
      build(f, raw);
      mma<PREC>(acc, f);
    }
  }
  store_part<kGenNKB, kGenNLB>(part, acc, split, kp, lp, k0, l0, li, lh);
}

// The split entries are rounded in the kernel from the FP32 tables, so a clip
// routed to split-fp16 (block_route_fp16) uses the same tables.
template <int PREC>
__global__ __launch_bounds__(64 * kGenWaves) void k_contract_big(
    const uint4 *__restrict__ phi, const float2 *__restrict__ tabx, const float2 *__restrict__ taby, int Mx, int My, int nhx,
    int nhy, int64_t chunk, int tiles_l, int kp, int lp, float *__restrict__ part, double r2,
    RouteArgs ra) {
  if (tile_outside(blockIdx.x, tiles_l, 128, 128, r2)) return;
  extern __shared__ float2 lds_big[];
  const int nx = nhx + kBigLo, ny = nhy + kBigLo;
  float2 *tx = lds_big;
  float2 *ty = tabx == taby ? tx : tx + nx;
  stage_entries(tx, tabx, nx);
  if (tabx != taby) stage_entries(ty, taby, ny);
  __syncthreads();
  if constexpr (PREC == kBF16) {
    if (block_route_fp16(ra)) {
      if (big_narrow(Mx, My))
        contract_big_body<kFP16, true>(phi, tx, ty, Mx, My, nhx, nhy, chunk, tiles_l, kp, lp,
                                       part);
      else
        contract_big_body<kFP16, false>(phi, tx, ty, Mx, My, nhx, nhy, chunk, tiles_l, kp, lp,
                                        part);
      return;
    }
  }
  if (big_narrow(Mx, My))
    contract_big_body<PREC, true>(phi, tx, ty, Mx, My, nhx, nhy, chunk, tiles_l, kp, lp, part);
  else
    contract_big_body<PREC, false>(phi, tx, ty, Mx, My, nhx, nhy, chunk, tiles_l, kp, lp, part);
}

// ---------------------------------------------------------------------------
// Shared-operand form for periods past 8192 (split precisions).  Four waves of
// 64 x 64 frequencies (128 x 128 per workgroup, the layout of the pipelined
// kernel), but each operand entry of a 16-corner step is built once per
// workgroup instead of once per wave that uses it: wave w takes the 8 corners
// of half h = w / 2 and the frequencies 64 (w mod 2) + lane of both sides,
// reduces the phases exactly (big_phase_int), multiplies the two FP32 table
// entries, rounds the products to hi + lo two corners at a time and stores
// the lane's four operand registers (cos-hi, sin-hi, cos-lo, sin-lo of its 8
// corners) with 16-byte LDS writes; every wave then reads the fragments of
// its 64 x 64 block.  The corner words (big_word) are wave-uniform: scalar
// loads.  The build of step s+1 runs as eight units of two entries, each unit
// finishing the entries whose table lookups the previous unit issued and
// interleaved with six of the 48 MFMAs of step s.
// LDS (bytes, from 0): x table (nhx + kBigLo FP32 pairs), y table (unless the
// periods coincide), rounded to 16; the operand buffers of the two sides, each
// [kind 4][half 2][frequency 128] x 16 bytes.
// ---------------------------------------------------------------------------
// Rounded pair {v0, v1} (low half v0) and the two values it rounds to.
template <int PREC>
__device__ __forceinline__ uint32_t bs_round2(float v0, float v1, float &r0, float &r1) {
  if constexpr (PREC == kBF16) {
    const bf16x2 h = {(__bf16)v0, (__bf16)v1};
    const uint32_t u = __builtin_bit_cast(uint32_t, h);
    r0 = __uint_as_float(u << 16);
    r1 = __uint_as_float(u & 0xffff0000u);
    return u;
  } else {
    const f16x2 h = {(_Float16)v0, (_Float16)v1};
    r0 = (float)h[0];
    r1 = (float)h[1];
    return __builtin_bit_cast(uint32_t, h);
  }
}

template <int PREC>
__device__ __forceinline__ uint32_t bs_round2(float v0, float v1) {
  if constexpr (PREC == kBF16) {
    const bf16x2 h = {(__bf16)v0, (__bf16)v1};
    return __builtin_bit_cast(uint32_t, h);
  } else {
    const f16x2 h = {(_Float16)v0, (_Float16)v1};
    return __builtin_bit_cast(uint32_t, h);
  }
}

// (a << b) + c as one instruction (the compiler splits it otherwise).
__device__ __forceinline__ uint32_t lshl_add(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t d;
  asm("v_lshl_add_u32 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
  return d;
}

// LDS byte address of a pointer into LDS, and the FP32 pair at an address.
typedef __attribute__((address_space(3))) const char lds_char;
__device__ __forceinline__ uint32_t lds_addr(const void *p) {
  return (uint32_t)(uintptr_t)(lds_char *)p;
}
__device__ __forceinline__ float2 lds_f2(uint32_t a) {
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  const f32x2 v = *(__attribute__((address_space(3))) const f32x2 *)(uintptr_t)a;
  return make_float2(v.x, v.y);
}

struct BsSide {
  uint32_t tab, lo_off, f, Mm1;  // table and Wlo LDS addresses, lane frequency, M - 1
  int negM;                      // -M
  // log2 of the entry size (3), a run-time value: the lookups then compile to
  // one shift-add (v_lshl_add_u32) per address instead of shift, mask and add
  uint32_t sh;
};

// The two table entries (Whi, Wlo) of the entries of two corners.
struct BsPair {
  float2 a[2], b[2];
};

template <bool NARROW, bool YSIDE>
__device__ __forceinline__ void bs_lookup(BsPair &P, const BsSide &sd,
                                          const uint4 &c0, const uint4 &c1) {
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const uint32_t p = big_word_phase<NARROW, !YSIDE>(sd.f, e ? c1 : c0, sd.Mm1, sd.negM);
    P.a[e] = lds_f2(lshl_add(p >> kBigBits, sd.sh, sd.tab));
    P.b[e] = lds_f2(lshl_add(p & (uint32_t)(kBigLo - 1), sd.sh, sd.lo_off));
  }
}

// Entries of the pair (y side: times the corner's sign, zero for padding),
// rounded into word i of the four operand registers.
template <int PREC, bool YSIDE>
__device__ __forceinline__ void bs_finish(const BsPair &P, const uint4 &c0, const uint4 &c1,
                                          u32x4 &ch, u32x4 &sh, u32x4 &cl, u32x4 &sl, int i) {
  float2 w[2];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    w[e] = cmulf(P.a[e], P.b[e]);
    if (YSIDE) {
      // 0, -1 or +1 from the (uniform) flags
      const uint32_t fl = (e ? c1 : c0).z;
      const uint32_t sb = (fl >> 31) ? 0u : ((fl >> 30) & 1u ? 0xbf800000u : 0x3f800000u);
      const float sgn = __uint_as_float(sb);
      w[e].x *= sgn;
      w[e].y *= sgn;
    }
  }
  float c0r, c1r, s0r, s1r;
  ch[i] = bs_round2<PREC>(w[0].x, w[1].x, c0r, c1r);
  sh[i] = bs_round2<PREC>(w[0].y, w[1].y, s0r, s1r);
  cl[i] = bs_round2<PREC>(w[0].x - c0r, w[1].x - c1r);
  sl[i] = bs_round2<PREC>(w[0].y - s0r, w[1].y - s1r);
}

__device__ __forceinline__ void bs_store(uint4 *op, int h, int fl, const u32x4 &ch,
                                         const u32x4 &sh, const u32x4 &cl, const u32x4 &sl) {
  op[(0 * 2 + h) * 128 + fl] = __builtin_bit_cast(uint4, ch);
  op[(1 * 2 + h) * 128 + fl] = __builtin_bit_cast(uint4, sh);
  op[(2 * 2 + h) * 128 + fl] = __builtin_bit_cast(uint4, cl);
  op[(3 * 2 + h) * 128 + fl] = __builtin_bit_cast(uint4, sl);
}

// MFMA m of a step, in the order term (hi hi', hi lo', lo hi') major, then
// (kb, lb, quadrant): successive MFMAs on one accumulator are 16 apart.
template <int PREC, int M>
__device__ __forceinline__ void bs_mfma(f32x16 (&acc)[2][2][4], const Frag<2, 2> &f) {
  constexpr int term = M / 16, kb = (M >> 3) & 1, lb = (M >> 2) & 1, q = M & 3;
  const u32x4 &a = term == 2 ? (q >> 1 ? f.asl[kb] : f.acl[kb]) : (q >> 1 ? f.ash[kb] : f.ach[kb]);
  const u32x4 &b = term == 1 ? (q & 1 ? f.bsl[lb] : f.bcl[lb]) : (q & 1 ? f.bsh[lb] : f.bch[lb]);
  acc[kb][lb][q] = mfma16<PREC>(a, b, acc[kb][lb][q]);
}

// Unit U of the build of a step (entries of pair U: x side for U < 4, then y
// side) and, with MM, MFMAs 6U .. 6U+5 of the previous step.
template <int PREC, bool NARROW, int U, bool MM>
__device__ __forceinline__ void bs_unit(f32x16 (&acc)[2][2][4], const Frag<2, 2> &f,
                                        BsPair (&P)[2], const uint4 (&cw)[8], const char *lds,
                                        const BsSide &sx, const BsSide &sy, u32x4 (&o)[4],
                                        uint4 *opA, uint4 *opB, int h, int fl) {
  constexpr int N = U + 1;
  if constexpr (N < 8) {
    if constexpr (N < 4)
      bs_lookup<NARROW, false>(P[N & 1], sx, cw[2 * (N & 3)], cw[2 * (N & 3) + 1]);
    else
      bs_lookup<NARROW, true>(P[N & 1], sy, cw[2 * (N & 3)], cw[2 * (N & 3) + 1]);
  }
  bs_finish<PREC, (U >= 4)>(P[U & 1], cw[2 * (U & 3)], cw[2 * (U & 3) + 1], o[0], o[1], o[2],
                            o[3], U & 3);
  if constexpr (U == 3) bs_store(opA, h, fl, o[0], o[1], o[2], o[3]);
  if constexpr (U == 7) bs_store(opB, h, fl, o[0], o[1], o[2], o[3]);
  if constexpr (MM) {
    bs_mfma<PREC, 6 * U + 0>(acc, f);
    bs_mfma<PREC, 6 * U + 1>(acc, f);
    bs_mfma<PREC, 6 * U + 2>(acc, f);
    bs_mfma<PREC, 6 * U + 3>(acc, f);
    bs_mfma<PREC, 6 * U + 4>(acc, f);
    bs_mfma<PREC, 6 * U + 5>(acc, f);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
      __builtin_amdgcn_sched_group_barrier(0x002, 7, 0);  // VALU
      if (k < 4) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // LDS read
    }
  }
  __builtin_amdgcn_sched_barrier(0);
}

// Build of one step (cw: the 8 corner words of the wave's half), with the
// MFMAs of the previous step when MM.
template <int PREC, bool NARROW, bool MM>
__device__ __forceinline__ void bs_step(f32x16 (&acc)[2][2][4], const Frag<2, 2> &f,
                                        const uint4 (&cw)[8], const char *lds, const BsSide &sx,
                                        const BsSide &sy, uint4 *opA, uint4 *opB, int h, int fl) {
  BsPair P[2];
  u32x4 o[4];
  bs_lookup<NARROW, false>(P[0], sx, cw[0], cw[1]);
  bs_unit<PREC, NARROW, 0, MM>(acc, f, P, cw, lds, sx, sy, o, opA, opB, h, fl);
  bs_unit<PREC, NARROW, 1, MM>(acc, f, P, cw, lds, sx, sy, o, opA, opB, h, fl);
  bs_unit<PREC, NARROW, 2, MM>(acc, f, P, cw, lds, sx, sy, o, opA, opB, h, fl);
  bs_unit<PREC, NARROW, 3, MM>(acc, f, P, cw, lds, sx, sy, o, opA, opB, h, fl);
  bs_unit<PREC, NARROW, 4, MM>(acc, f, P, cw, lds, sx, sy, o, opA, opB, h, fl);
  bs_unit<PREC, NARROW, 5, MM>(acc, f, P, cw, lds, sx, sy, o, opA, opB, h, fl);
  bs_unit<PREC, NARROW, 6, MM>(acc, f, P, cw, lds, sx, sy, o, opA, opB, h, fl);
  bs_unit<PREC, NARROW, 7, MM>(acc, f, P, cw, lds, sx, sy, o, opA, opB, h, fl);
}

template <int PREC, bool NARROW>
__device__ __forceinline__ void contract_big_shared_body(
    char *lds, uint32_t ybase, uint32_t opa, const uint4 *__restrict__ words, int Mx, int My,
    int nhx, int nhy, int64_t chunk, int tiles_l, int kp, int lp, float *__restrict__ part,
    int tile, int split, uint32_t sh) {
  const int t = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6), lane = t & 63;
  const int li = lane & 31, lh = lane >> 5;
  const int tk = tile / tiles_l, tl = tile % tiles_l;
  uint4 *opA = (uint4 *)(lds + opa);
  uint4 *opB = (uint4 *)(lds + opa + 16u * kBsOpWords);
  // builder role: half h, local frequency fl of both sides
  const int h = wave >> 1, fl = 64 * (wave & 1) + lane;
  const uint32_t l0 = lds_addr(lds);
  const BsSide sx{l0, l0 + 8u * (uint32_t)nhx, (uint32_t)(tk * 128 + fl), (uint32_t)Mx - 1u, -Mx,
                  sh};
  const BsSide sy{l0 + ybase, l0 + ybase + 8u * (uint32_t)nhy, (uint32_t)(tl * 128 + fl),
                  (uint32_t)My - 1u, -My, sh};
  // MFMA role: block (wk, wl) of 64 x 64
  const int wk = wave >> 1, wl = wave & 1;

  f32x16 acc[2][2][4];
#pragma unroll
  for (int kb = 0; kb < 2; ++kb)
#pragma unroll
    for (int lb = 0; lb < 2; ++lb)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[kb][lb][q][r] = 0.0f;

  const int nsteps = (int)(chunk >> 4);
  const uint4 *cp = words + (size_t)split * chunk + 8 * h;
  Frag<2, 2> f;
  uint4 cw[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) cw[j] = cp[j];
  __syncthreads();  // the tables
  bs_step<PREC, NARROW, false>(acc, f, cw, lds, sx, sy, opA, opB, h, fl);
  __syncthreads();
  for (int s = 0; s < nsteps; ++s) {
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      const int i = lh * 128 + 64 * wk + 32 * kb + li;
      f.ach[kb] = __builtin_bit_cast(u32x4, opA[0 * 256 + i]);
      f.ash[kb] = __builtin_bit_cast(u32x4, opA[1 * 256 + i]);
      f.acl[kb] = __builtin_bit_cast(u32x4, opA[2 * 256 + i]);
      f.asl[kb] = __builtin_bit_cast(u32x4, opA[3 * 256 + i]);
    }
#pragma unroll
    for (int lb = 0; lb < 2; ++lb) {
      const int i = lh * 128 + 64 * wl + 32 * lb + li;
      f.bch[lb] = __builtin_bit_cast(u32x4, opB[0 * 256 + i]);
      f.bsh[lb] = __builtin_bit_cast(u32x4, opB[1 * 256 + i]);
      f.bcl[lb] = __builtin_bit_cast(u32x4, opB[2 * 256 + i]);
      f.bsl[lb] = __builtin_bit_cast(u32x4, opB[3 * 256 + i]);
    }
    // the last step builds its own corners again, into buffers nobody reads
    const int sn = min(s + 1, nsteps - 1);
#pragma unroll
    for (int j = 0; j < 8; ++j) cw[j] = cp[16 * sn + j];
    __syncthreads();  // every wave holds its fragments: the buffers are free
    bs_step<PREC, NARROW, true>(acc, f, cw, lds, sx, sy, opA, opB, h, fl);
    __syncthreads();
  }
  store_part<2, 2>(part, acc, split, kp, lp, tk * 128 + 64 * wk, tl * 128 + 64 * wl, li, lh);
}


template <int PREC>
__global__ __launch_bounds__(256, 1) void k_contract_big_shared(
    const uint4 *__restrict__ words, const float2 *__restrict__ tabx, const float2 *__restrict__ taby, int Mx, int My, int nhx,
    int nhy, int64_t chunk, int tiles_l, int kp, int lp, float *__restrict__ part, double r2,
    RouteArgs ra, uint32_t sh /* 3 */) {
  if (tile_outside(blockIdx.x, tiles_l, 128, 128, r2)) return;
  extern __shared__ __align__(16) char lds_bs[];
  const bool one = tabx == taby;
  const int nx = nhx + kBigLo, ny = nhy + kBigLo;
  float2 *tx = (float2 *)lds_bs;
  float2 *ty = one ? tx : tx + nx;
  stage_entries(tx, tabx, nx);
  if (!one) stage_entries(ty, taby, ny);
  const uint32_t ybase = one ? 0u : 8u * (uint32_t)nx;
  const uint32_t opa = big_shared_tab_bytes(nhx, nhy, one);
  const bool narrow = big_narrow(Mx, My);
  if constexpr (PREC == kBF16) {
    if (block_route_fp16(ra)) {
      if (narrow)
        contract_big_shared_body<kFP16, true>(lds_bs, ybase, opa, words, Mx, My, nhx, nhy,
                                              chunk, tiles_l, kp, lp, part, blockIdx.x,
                                              blockIdx.y, sh);
      else
        contract_big_shared_body<kFP16, false>(lds_bs, ybase, opa, words, Mx, My, nhx, nhy,
                                               chunk, tiles_l, kp, lp, part, blockIdx.x,
                                               blockIdx.y, sh);
      return;
    }
  }
  if (narrow)
    contract_big_shared_body<PREC, true>(lds_bs, ybase, opa, words, Mx, My, nhx, nhy, chunk,
                                         tiles_l, kp, lp, part, blockIdx.x, blockIdx.y, sh);
  else
    contract_big_shared_body<PREC, false>(lds_bs, ybase, opa, words, Mx, My, nhx, nhy, chunk,
                                          tiles_l, kp, lp, part, blockIdx.x, blockIdx.y, sh);
}

// Batch of general tiles: one workgroup per (clip, tile, split) work item.
// A one-level clip stages its split tables and runs the pipelined form; a
// two-level clip stages its FP32 tables and runs the shared-operand form.
// The LDS holds either (kGBatchLds); a split-bf16 clip the rounding model
// routes (block_route_fp16) runs split-fp16.
template <int PREC>
__global__ __launch_bounds__(256, 1) void k_gbatch_contract(const GBatchClip *__restrict__ clips,
                                                            const int4 *__restrict__ items) {
  const int4 d = items[blockIdx.x];
  const GBatchClip &c = clips[d.x];
  __shared__ __align__(16) uint2 lds[kGBatchLds / 8];
  bool fp16 = false;
  if constexpr (PREC == kBF16) {
    RouteArgs ra;
    ra.area_part = c.area_part;
    ra.pre_blocks = c.pre_blocks;
    ra.V = c.V;
    ra.gscale = c.gscale;
    ra.gscale_alt = c.gscale_alt;
    fp16 = block_route_fp16(ra);
  }
  if (c.big) {
    const bool one = c.tx == c.ty;
    const int nx = c.nhx + kBigLo, ny = c.nhy + kBigLo;
    float2 *tx = (float2 *)lds;
    float2 *ty = one ? tx : tx + nx;
    stage_entries(tx, (const float2 *)(const void *)c.tx, nx);
    if (!one) stage_entries(ty, (const float2 *)(const void *)c.ty, ny);
    const uint32_t ybase = one ? 0u : 8u * (uint32_t)nx;
    const uint32_t opa = big_shared_tab_bytes(c.nhx, c.nhy, one);
    char *l = (char *)lds;
    // the body's first barrier completes the tables
    if (big_narrow(c.Mx, c.My)) {
      if (fp16)
        contract_big_shared_body<kFP16, true>(l, ybase, opa, c.words, c.Mx, c.My, c.nhx, c.nhy,
                                              c.chunk, c.tiles_l, c.kp, c.lp, c.part, d.y, d.z,
                                              3u);
      else
        contract_big_shared_body<PREC, true>(l, ybase, opa, c.words, c.Mx, c.My, c.nhx, c.nhy,
                                             c.chunk, c.tiles_l, c.kp, c.lp, c.part, d.y, d.z, 3u);
    } else {
      if (fp16)
        contract_big_shared_body<kFP16, false>(l, ybase, opa, c.words, c.Mx, c.My, c.nhx, c.nhy,
                                               c.chunk, c.tiles_l, c.kp, c.lp, c.part, d.y, d.z,
                                               3u);
      else
        contract_big_shared_body<PREC, false>(l, ybase, opa, c.words, c.Mx, c.My, c.nhx, c.nhy,
                                              c.chunk, c.tiles_l, c.kp, c.lp, c.part, d.y, d.z,
                                              3u);
    }
    return;
  }
  if (fp16) {
    stage_gen_tables<uint2>(lds, c.tx16, c.ty16, c.Mx, c.My);
    contract_gen_pipe_body<kFP16>(lds, c.tx16 == c.ty16, c.packed, c.Mx, c.My, c.chunk,
                                  c.tiles_l, c.kp, c.lp, c.part, d.y, d.z);
  } else {
    stage_gen_tables<uint2>(lds, c.tx, c.ty, c.Mx, c.My);
    contract_gen_pipe_body<PREC>(lds, c.tx == c.ty, c.packed, c.Mx, c.My, c.chunk, c.tiles_l,
                                 c.kp, c.lp, c.part, d.y, d.z);
  }
}

constexpr size_t kMaxLds = 160 * 1024;

template <int PREC>
hipError_t launch_big_t(const FwdPlan &p, const uint4 *packed, const uint4 *phi, const void *tx,
                        const void *ty, float *part, const RouteArgs &ra, hipStream_t st) {
  if constexpr (PREC != kFP32) {
    const size_t lds = big_shared_lds_bytes(p.nhx, p.nhy, tx == ty);
    if (lds <= kMaxLds - 1024 && p.chunk % 16 == 0) {
      // the kernel's static LDS (the routing reduction) comes on top
      static size_t attr = 0;
      if (lds > attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_contract_big_shared<PREC>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e) return e;
        attr = lds;
      }
      hipLaunchKernelGGL(k_contract_big_shared<PREC>, dim3(p.tiles_k * p.tiles_l, p.nsplit),
                         dim3(256), lds, st, phi, (const float2 *)tx, (const float2 *)ty,
                         p.Mx, p.My, p.nhx, p.nhy, p.chunk, p.tiles_l, p.kp, p.lp, part, p.r2, ra,
                         3u);
      return hipGetLastError();
    }
  }
  const size_t lds = sizeof(float2) * ((size_t)p.nhx + kBigLo +
                                       (tx == ty ? 0 : (size_t)p.nhy + kBigLo));
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)k_contract_big<PREC>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(sizeof(float2) * 4 * kBigLo));
    if (e) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(k_contract_big<PREC>, dim3(p.tiles_k * p.tiles_l, p.nsplit),
                     dim3(64 * kGenWaves), lds, st, phi, (const float2 *)tx,
                     (const float2 *)ty, p.Mx, p.My, p.nhx, p.nhy, p.chunk, p.tiles_l, p.kp, p.lp,
                     part, p.r2, ra);
  return hipGetLastError();
}

template <int PREC>
hipError_t launch_gen_pipe_t(const FwdPlan &p, const uint4 *packed, const void *tx,
                             const void *ty, const void *tx16, const void *ty16, float *part,
                             const RouteArgs &ra, hipStream_t st) {
  hipLaunchKernelGGL(k_contract_gen_pipe<PREC>, dim3(p.tiles_k * p.tiles_l, p.nsplit), dim3(256),
                     0, st, packed, (const uint2 *)tx, (const uint2 *)ty, p.Mx, p.My, p.chunk,
                     p.tiles_l, p.kp, p.lp, part, p.r2, ra, (const uint2 *)tx16,
                     (const uint2 *)ty16);
  return hipGetLastError();
}

template <int PREC>
hipError_t launch_gen_t(const FwdPlan &p, const uint4 *packed, const void *tx, const void *ty,
                        const void *tx16, const void *ty16, float *part, const RouteArgs &ra,
                        hipStream_t st) {
  const size_t lds = sizeof(uint2) * ((size_t)p.Mx + 1 + (tx == ty ? 0 : (size_t)p.My));
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)k_contract_gen<PREC>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(sizeof(uint2) * (2 * kTabN + 1)));
    if (e) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(k_contract_gen<PREC>, dim3(p.tiles_k * p.tiles_l, p.nsplit),
                     dim3(64 * kGenWaves), lds, st, packed, tx, ty, p.Mx, p.My, p.chunk, p.tiles_l,
                     p.kp, p.lp, part, p.r2, ra, tx16, ty16);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gbatch_contract(const GBatchLaunch &b, hipStream_t st) {
  if (b.n_items == 0) return hipSuccess;
  if (b.prec == kBF16)
    hipLaunchKernelGGL(k_gbatch_contract<kBF16>, dim3(b.n_items), dim3(256), 0, st, b.clips,
                       b.items);
  else if (b.prec == kFP16)
    hipLaunchKernelGGL(k_gbatch_contract<kFP16>, dim3(b.n_items), dim3(256), 0, st, b.clips,
                       b.items);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_gen_contract(const FwdPlan &p, const uint4 *packed, const void *tx,
                               const void *ty, float *part, hipStream_t st,
                               const unsigned long long *area_part, const void *tx16,
                               const void *ty16, const uint4 *phi) {
  RouteArgs ra = route_args(p, area_part);
  if (!p.big && (!tx16 || !ty16)) ra.gscale_alt = 0.0;
  if (p.big) {
    if (!phi) return hipErrorInvalidValue;
    switch (p.prec) {
      case kFP32: return launch_big_t<kFP32>(p, packed, phi, tx, ty, part, ra, st);
      case kBF16: return launch_big_t<kBF16>(p, packed, phi, tx, ty, part, ra, st);
      default: return launch_big_t<kFP16>(p, packed, phi, tx, ty, part, ra, st);
    }
  }
  if (p.tile == kGenPipeTile) {
    if (p.chunk % 32) return hipErrorInvalidValue;
    return p.prec == kBF16 ? launch_gen_pipe_t<kBF16>(p, packed, tx, ty, tx16, ty16, part, ra, st)
                           : launch_gen_pipe_t<kFP16>(p, packed, tx, ty, tx16, ty16, part, ra, st);
  }
  switch (p.prec) {
    case kFP32: return launch_gen_t<kFP32>(p, packed, tx, ty, tx16, ty16, part, ra, st);
    case kBF16: return launch_gen_t<kBF16>(p, packed, tx, ty, tx16, ty16, part, ra, st);
    default: return launch_gen_t<kFP16>(p, packed, tx, ty, tx16, ty16, part, ra, st);
  }
}

}  // namespace fcfs
