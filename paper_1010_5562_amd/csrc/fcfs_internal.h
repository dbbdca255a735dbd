// Internal declarations shared by the host runtime and the kernel launchers
// of the FCFS library (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <stddef.h>
#include <stdint.h>

namespace fcfs {

// One twiddle table of N = 8192 entries serves every power-of-two period
// T <= 8192: the phase index of period T is scaled by 8192 / T.
constexpr int kTabBits = 13;
constexpr int kTabN = 1 << kTabBits;
// Entry kTabN of every device table is zero: padded corners point there.
constexpr int kTabEntries = kTabN + 1;

// Corner record written by the pre-pass (uint4, 16 bytes), already decoded
// for the inner loops (byte offsets into 8-byte-per-entry tables):
//   .x = xs * 8, .y = ys * 8  with xs = (x mod T) * (8192 / T), ys likewise
//   .z = 4096 * 8 if s = -1 else 0  (half a period: a factor -1 on the y side)
//   .w = kTabN * 8 for padding records (points the y side at the zero entry)
constexpr uint32_t kNegOff = (uint32_t)(kTabN / 2) * 8u;
constexpr uint32_t kPadOff = (uint32_t)kTabN * 8u;

enum Prec { kFP32 = 0, kBF16 = 1, kFP16 = 2 };

// Histogram bins per block of the axis DFTs (partials per frequency: T / kAxisBins).
constexpr int kAxisBins = 128;
// The FP64 guard region.  Blocks of 8 x 8 frequencies whose sums are taken in
// FP64 and replace the MFMA values where the 1/(k l) factor of alpha_{k,l}
// amplifies the contraction's rounding most: the core block k, l = 1..8
// always, and for a span n > 1 the strips k = 1..8, l <= 8 n and l = 1..8,
// k <= 8 n next to the axes, plus the block k, l = 9..16 once n reaches
// kGuardDiagSpan.  Each block holds 16 x 16 sums ([cos; sin] of its 8 k by
// [cos; sin] of its 8 l).  Slot 0 is the core block, slot g (1 <= g < n) the
// strip block l = 8 g + 1..8 g + 8, slot kGuardSpanMax - 1 + h (1 <= h < n)
// the strip block k = 8 h + 1..8 h + 8, slot kGuardSlots - 1 the block 9..16.
constexpr int kGuard = 8;
constexpr int kGuardSpanMax = 16;
constexpr int kGuardDiagSpan = 11;  // 8 n > 81 = 9 x 9
constexpr int kGuardSlots = 2 * kGuardSpanMax;
constexpr int kGuardD = 256;
// The side kernel computes the slots in groups of up to four per corner
// range (guard_group); groups 0..3 walk the l strip, 4..7 the k strip, group
// 8 is the block 9..16.
constexpr int kGuardGroups = 9;
__host__ __device__ inline bool guarded(int k, int l, int n) {
  return (k <= kGuard && l <= kGuard * n) || (l <= kGuard && k <= kGuard * n) ||
         (n >= kGuardDiagSpan && k > kGuard && k <= 2 * kGuard && l > kGuard && l <= 2 * kGuard);
}
// Frequency-block offsets (in units of kGuard) of slot j: k = 8 kb + 1..8,
// l = 8 lb + 1..8.
__host__ __device__ inline void guard_slot_block(int j, int &kb, int &lb) {
  if (j < kGuardSpanMax) {
    kb = 0;
    lb = j;
  } else if (j < kGuardSlots - 1) {
    kb = j - kGuardSpanMax + 1;
    lb = 0;
  } else {
    kb = lb = 1;
  }
}
// Slot j is in use for span n.
__host__ __device__ inline bool guard_slot_used(int j, int n) {
  int kb, lb;
  guard_slot_block(j, kb, lb);
  return j == kGuardSlots - 1 ? n >= kGuardDiagSpan : (kb > lb ? kb : lb) < n;
}
// Slot group g: the first slot's block offsets (kb, lb), whether the group
// steps along l (else along k) and how many of its slots span n uses.
struct GuardGroup {
  int kb, lb, ymove, ns, slot;
};
__host__ __device__ inline GuardGroup guard_group(int g, int n) {
  GuardGroup r;
  if (g < 4) {
    r.kb = 0;
    r.lb = 4 * g;
    r.ymove = 1;
    r.ns = n - r.lb;
    r.slot = r.lb;
  } else if (g < 8) {
    r.kb = 4 * (g - 4) + 1;
    r.lb = 0;
    r.ymove = 0;
    r.ns = (kGuardSpanMax < n ? kGuardSpanMax : n) - r.kb;
    r.slot = kGuardSpanMax - 1 + r.kb;
  } else {
    r.kb = r.lb = 1;
    r.ymove = 1;
    r.ns = n >= kGuardDiagSpan ? 1 : 0;
    r.slot = kGuardSlots - 1;
  }
  r.ns = r.ns < 0 ? 0 : (r.ns > 4 ? 4 : r.ns);
  return r;
}
// Span of the guard region from a rounding model of the contraction.
// Every corner term carries a rounding of about eps (the table entries and, in
// the split forms, the dropped lo x lo product), so the error of S(k, l) grows
// like eps sqrt(V); alpha_{k,l} turns it into an error relative to |F[0,0]|
// of about eps sqrt(V) P / (4 pi^2 |A| k l), P the period area and A the exact
// polygon area in the same units.  gscale = 2 eps P / (4 pi^2 tol) (a factor 2
// of margin, tol the bound of the precision) is fixed by the plan; the guard
// has to cover every k l below reach = gscale sqrt(V) / |A|.  gscale = 0 keeps
// the core block.
__host__ __device__ inline double guard_reach(double gscale, int64_t V, long long A) {
  if (gscale <= 0.0 || V <= 0) return 0.0;
  const double a = A < 0 ? -(double)A : (double)A;
  return a > 0.0 ? gscale * sqrt((double)V) / a : 1e300;
}
// The strips k <= 8, l <= 8 n (and mirrored) plus the block 9..16 cover every
// k l <= 8 n up to the widest span; past it the model asks for more than the
// guard region holds.
__host__ __device__ inline bool guard_exceeded(double gscale, int64_t V, long long A) {
  return guard_reach(gscale, V, A) > (double)(kGuard * kGuardSpanMax);
}
__host__ __device__ inline int guard_span(double gscale, int64_t V, long long A) {
  const double n = ceil(guard_reach(gscale, V, A) / kGuard);
  return n <= 1.0 ? 1 : (n >= (double)kGuardSpanMax ? kGuardSpanMax : (int)n);
}
// Precision routing of split-bf16 plans (gscale_alt > 0, the split-fp16
// factor): a clip whose bf16 reach exceeds the guard region runs its
// contraction in split-fp16 (11 + 11 significant bits, eps 16 times smaller)
// and sizes its guard with the fp16 factor.  Decided on the device from the
// exact area, identically by the contraction and the side kernels.
__host__ __device__ inline bool route_fp16(double gscale, double gscale_alt, int64_t V,
                                           long long A) {
  return gscale_alt > 0.0 && guard_exceeded(gscale, V, A);
}
__host__ __device__ inline int guard_span_routed(double gscale, double gscale_alt, int64_t V,
                                                 long long A) {
  return guard_span(route_fp16(gscale, gscale_alt, V, A) ? gscale_alt : gscale, V, A);
}

// Periods above the LDS table size (general tiles with Nx 2^F or Ny 2^F past
// 8192 grid units): two-level twiddles.  The phase p = (f x) mod M is reduced
// exactly in FP64 and the entry is e(2 pi p / M) = Whi[p >> kBigBits] x
// Wlo[p & (kBigLo - 1)], Whi[j] = e(2 pi j kBigLo / M), Wlo[i] = e(2 pi i / M),
// both tables at most 4096 entries (M <= kBigMaxPeriod).  A two-level table
// of period M stores Whi (big_hi(M) entries) followed by Wlo (kBigLo).
constexpr int kBigBits = 12;
constexpr int kBigLo = 1 << kBigBits;
constexpr int64_t kBigMaxPeriod = (int64_t)1 << 24;
__host__ __device__ inline int big_hi(int64_t M) { return (int)((M + kBigLo - 1) / kBigLo); }
// (f x) mod M for x < M <= 2^24 and f < 2^13: f x < 2^37 is exact in FP64, the
// quotient estimate is off by at most one and the remainder fma is exact.
__device__ __forceinline__ uint32_t big_phase(uint32_t f, uint32_t x, double M, double invM) {
  const double t = (double)f * (double)x;
  const double q = floor(t * invM);
  double r = fma(-q, M, t);
  r = r < 0.0 ? r + M : (r >= M ? r - M : r);
  return (uint32_t)r;
}

// The same phase in 32-bit integer arithmetic, from a per-corner magic
// ph = floor(x 2^38 / M) + 1 (38 bits, big_magic): ph exceeds x 2^38 / M by
// d in (0, 1], so f ph / 2^38 exceeds f x / M by f d / 2^38 < 2^-25 <= 1 / (2 M)
// < 1 / M, and as the
// fractional part of f x / M is at most 1 - 1/M, the floor of f ph / 2^38 is
// the exact quotient q; the remainder f x - q M < 2^24 is exact modulo 2^32.
// With ph = hi 2^32 + lo: floor(f ph / 2^38) = (f hi + floor(f lo / 2^32)) >> 6.
__host__ __device__ inline uint64_t big_magic(uint32_t x, uint32_t M) {
  return ((uint64_t)x << 38) / M + 1u;
}

// x may carry other bits above bit 23 (the 24-bit products ignore them).
__device__ __forceinline__ uint32_t big_phase_int(uint32_t f, uint32_t x, uint32_t ph_lo,
                                                  uint32_t ph_hi, uint32_t Mm1) {
  const uint32_t q = (__umul24(f, ph_hi) + __umulhi(f, ph_lo)) >> 6;
  // q M = q (M - 1) + q keeps both 24-bit product operands below 2^24
  return __umul24(f, x) - (__umul24(q, Mm1) + q);
}

// Periods up to 2^20 (narrow): a 32-bit magic mu = floor(x 2^32 / M) + 1
// suffices, as f mu / 2^32 exceeds f x / M by f d / 2^32 with d in (0, 1] and
// f M < 2^12 2^20 = 2^32 keeps that below 1 / M; then q = floor(f mu / 2^32)
// and r = f x - q M, the product q M taken as the signed 24-bit product of q
// and -M (M <= 2^20 < 2^23).  Frequencies f < 2^12.
constexpr int64_t kBigNarrowMax = (int64_t)1 << 20;
__host__ __device__ inline uint32_t big_magic32(uint32_t x, uint32_t M) {
  return (uint32_t)(((uint64_t)x << 32) / M) + 1u;
}

__device__ __forceinline__ uint32_t big_phase_narrow(uint32_t f, uint32_t x, uint32_t mu,
                                                     int negM) {
  const uint32_t q = __umulhi(f, mu);
  return __umul24(f, x) + (uint32_t)__mul24((int)q, negM);
}

// Corner word of a plan with a period past 8192 (written by the pre-pass):
// {x | ph_x.hi << 24, ph_x.lo, y | ph_y.hi << 24 | sign << 30 | pad << 31,
// ph_y.lo}, x, y the residues, ph the 38-bit magics (hi below 2^6), sign set
// for s = -1 and pad for the padding records (x = y = 0).  When both periods
// are narrow (big_narrow) the magics are the 32-bit mu and the hi fields 0.
__host__ __device__ inline bool big_narrow(int64_t Mx, int64_t My) {
  return Mx <= kBigNarrowMax && My <= kBigNarrowMax;
}

__host__ __device__ inline uint4 big_word(uint32_t x, uint32_t y, uint32_t Mx, uint32_t My,
                                          bool neg, bool pad) {
  const uint32_t fl = (neg ? 1u << 30 : 0u) | (pad ? 1u << 31 : 0u);
  if (big_narrow(Mx, My)) return make_uint4(x, big_magic32(x, Mx), y | fl, big_magic32(y, My));
  const uint64_t px = big_magic(x, Mx), py = big_magic(y, My);
  return make_uint4(x | (uint32_t)(px >> 32) << 24, (uint32_t)px,
                    y | (uint32_t)(py >> 32) << 24 | fl, (uint32_t)py);
}

// Frequencies per block of the direct axis sums of a two-level plan
// (k_gen_axis_big): 128, 256 or 512, the smallest that covers max(K, L).
__host__ __device__ inline int axis_big_freqs(int K, int L) {
  const int m = K > L ? K : L;
  return m <= 128 ? 128 : (m <= 256 ? 256 : 512);
}

// (f x) mod M of the x side (XS) or y side of a corner word.
template <bool NARROW, bool XS>
__device__ __forceinline__ uint32_t big_word_phase(uint32_t f, const uint4 &w, uint32_t Mm1,
                                                   int negM) {
  const uint32_t xw = XS ? w.x : w.z, lo = XS ? w.y : w.w;
  if constexpr (NARROW)
    return big_phase_narrow(f, xw, lo, negM);
  else
    return big_phase_int(f, xw, lo, (xw >> 24) & 63u, Mm1);
}

// Device-resident constant tables owned by a handle.
struct Tables {
  double2 *w64 = nullptr;    // [kTabN]       (cos, sin)(2 pi p / N), FP64
  float2 *w32 = nullptr;     // [kTabEntries] FP32 (cos, sin)
  uint2 *wbf16 = nullptr;    // [kTabEntries] {hi(c)|hi(s)<<16, lo(c)|lo(s)<<16}
  uint2 *wfp16 = nullptr;    // [kTabEntries] same layout, binary16
};

// Launch geometry of one forward (or adjoint) call, fixed by the planner
// from (V, T, K, L, precision) alone.
struct FwdPlan {
  int prec;
  int T, K, L;       // period and computed band |k| <= K, |l| <= L
  int KO, LO;        // output grid (2 KO + 1) x (2 LO + 1), KO >= K, LO >= L
  double r2;         // pupil: entries with k^2 + l^2 > r2 written as zero (< 0: none)
  double eg, eax, eay, edc;  // epilogue factors of alpha (square tile: T, 1, 1, 1/T)
  int Mx, My;        // periods of the phase reduction (square tile: T, T)
  int64_t V;
  int shift;         // log2(8192 / T)
  int tile;          // contraction tile variant id
  int wgk, wgl;      // workgroup tile in k and l (frequencies)
  int kp, lp;        // padded frequency counts (multiples of wgk, wgl)
  int tiles_k, tiles_l;
  int nsplit;        // vertex splits of the contraction
  int64_t chunk;     // corners per split (multiple of 16)
  int64_t vpad;      // nsplit * chunk
  int pre_blocks;    // pre-pass blocks (area partials)
  int hist_blocks;   // histogram blocks of the side kernel
  int ax_fb_k;       // 256-frequency blocks of the x-axis DFT (two-level: axis_big_freqs)
  int ax_fb_l;       // and of the y-axis DFT
  int ax_chunks;     // bin chunks of the axis DFTs (partials per frequency)
  int g_chunks;      // corner chunks (blocks) of the FP64 guard region
  int64_t g_chunk;
  double gscale;     // guard-span model factor (guard_span; 0: core block only)
  double gscale_alt; // split-bf16: the split-fp16 factor of a routed clip (route_fp16), else 0
  int big;           // general tile with a period past 8192: two-level tables
  int nhx, nhy;      // two-level tables: entries of Whi per period (big_hi)
  // workspace offsets (bytes): off_guard holds the guard partials
  // [chunk][slot][16 x 16], off_gspan the span the side kernel chose,
  // off_phi the corner words (big_word) of a two-level plan (vpad x 16 bytes)
  size_t off_packed, off_area, off_hist, off_axis, off_part, off_guard, off_gspan, off_phi, bytes;
  // lattice (FFT) form only: bin counters, corner list, row transforms
  size_t off_fcnt, off_flist, off_fd;
};

// Kernel launchers (fcfs_kernels.hip).  All enqueue on `st` and return the
// launch status; `ws` is the workspace laid out by the plan.  The pre-pass
// also clears the histograms when they are non-NULL.
hipError_t launch_prepass(const FwdPlan &p, const int32_t *x, const int32_t *y, const int8_t *s,
                          uint4 *packed, unsigned long long *area_part,
                          unsigned long long *hist, hipStream_t st);
// histograms + guard region (unless guard is false; with large frequency
// blocks its corner-range partials are then folded into range 0), then the
// axis DFTs
hipError_t launch_side(const FwdPlan &p, const int32_t *x, const int32_t *y, const double2 *w64,
                       void *ws, hipStream_t st, bool guard = true);
// area_part: the pre-pass area partials, which let a split-bf16 plan route a
// clip to split-fp16 (route_fp16); nullptr keeps the plan's precision.
hipError_t launch_contract(const FwdPlan &p, const uint4 *packed, const Tables &t, float *part,
                           hipStream_t st, const unsigned long long *area_part = nullptr);
// after launch_side or launch_gen_side (which fold the guard partials when
// guard_folded(p); the epilogue then reads range 0 only)
bool guard_folded(const FwdPlan &p);
// the band forward's entries outside the computed band (KO > K or LO > L):
// zeroed before the epilogue writes the band, on any stream ordered before it
hipError_t launch_zero_outside(const FwdPlan &p, float *F, hipStream_t st);
hipError_t launch_epilogue(const FwdPlan &p, const void *ws, float *F, int64_t *area,
                           hipStream_t st);
// the axes and DC entries only (lattice form)
hipError_t launch_epilogue_axes(const FwdPlan &p, const void *ws, float *F, int64_t *area,
                                hipStream_t st);
// direct form for small problems: every coefficient in FP64 from the raw
// corner arrays in one launch (uses p.V, T, shift, K, L and the output grid)
hipError_t launch_direct(const FwdPlan &p, const int32_t *x, const int32_t *y, const int8_t *s,
                         const double2 *w64, float *F, int64_t *area, hipStream_t st);
// lattice form of the general term (fcfs_fft.hip): writes F for k, l != 0
// General tile (periods Mx, My in [2, 8192], any integers): pre-pass into
// residue records, side-stream work (histograms, FP64 guard region, axis DFTs
// with the per-period FP64 tables wx, wy) and the MFMA contraction with the
// per-period operand tables tx, ty (split or FP32 entries; tx has Mx + 1
// entries, the last zero).
hipError_t launch_gen_prepass(const FwdPlan &p, const int32_t *x, const int32_t *y,
                              const int8_t *s, uint32_t smask, void *ws, hipStream_t st);
// residue records only (no histograms), for the adjoint of a general tile
hipError_t launch_gen_prepass_records(const int32_t *x, const int32_t *y, const int8_t *s,
                                      int64_t V, int64_t vpad, int Mx, int My, int pre_blocks,
                                      uint4 *packed, unsigned long long *area_part,
                                      hipStream_t st);
// With p.big, wx and wy are two-level FP64 tables, the histograms are not used
// and the axis sums are taken directly over the corners.
hipError_t launch_gen_side(const FwdPlan &p, const int32_t *x, const int32_t *y,
                           const double2 *wx, const double2 *wy, void *ws, hipStream_t st);
// FwdPlan::tile of a general-tile plan: kGenPipeTile selects the pipelined
// split kernel (one wave per SIMD, chunk a multiple of 32), any other value
// the eight-wave kernel.
constexpr int kGenPipeTile = 1;
// With p.big, tx and ty are two-level FP32 tables for every precision (the
// split entries are formed from the FP32 product in the kernel).
// area_part, tx16, ty16: the pre-pass area partials and the split-fp16 tables
// of both periods, which let a split-bf16 plan route a clip to split-fp16
// (route_fp16); nullptr keeps the plan's precision.
hipError_t launch_gen_contract(const FwdPlan &p, const uint4 *packed, const void *tx,
                               const void *ty, float *part, hipStream_t st,
                               const unsigned long long *area_part = nullptr,
                               const void *tx16 = nullptr, const void *ty16 = nullptr,
                               const uint4 *phi = nullptr);
struct RouteArgs;
// routing inputs of a forward plan (fcfs_kernels.hip)
RouteArgs route_args(const FwdPlan &p, const unsigned long long *area_part);
hipError_t launch_fft(const FwdPlan &p, const int32_t *x, const int32_t *y, const int8_t *s,
                      const double2 *w64, void *ws, float *F, hipStream_t st);
hipError_t launch_debug_phases(const FwdPlan &p, const uint4 *packed, int axis, int k0, int nk,
                               int32_t *out, hipStream_t st);

// Geometry of one adjoint call (Hermitian-folded real GEMM, vertices x
// frequencies).  kmax, lmax: the band outside which the cotangent is zero.
struct AdjPlan {
  int prec;
  int T, K, L, kmax, lmax;
  double r2;         // pupil k^2 + l^2 <= r2 (< 0: none)
  int64_t V;
  int shift;
  int kb, lb;        // kmax, lmax padded to multiples of 16 and 32
  int R, NC;         // GEMM inner rows 2*kb and columns 4*lb
  int64_t vpad;      // V padded to the 256-corner block of the split GEMM
  int pre_blocks;
  size_t off_packed, off_area, off_coef, off_wf, off_whi, off_wlo, off_scale, bytes;
  // general tile: periods Mx, My of the phase reduction and the factors of
  // the derivatives (square tile: T, T, 1, 1, 1/T): rx = sqrt(Ny/Nx) and
  // ry = sqrt(Nx/Ny) scale the x- and y-gradient coefficients j/(2 pi f),
  // dcf = 2^-F / sqrt(Nx Ny) replaces 1/T in the axis and DC terms
  bool gen;
  int Mx, My;
  int big, nhx, nhy;  // periods past 8192: two-level tables (nh entries of Whi)
  double rx, ry, dcf;
  // register-resident main term (square tiles, split precisions, kb <= 128):
  // kb / 16 steps (0: the streaming kernel), chunk sets, and its partials
  // [4 chunks per set x sets][vpad]
  int regb_nks, regb_sets;
  size_t off_rpart;
};

// Register-resident adjoint main term (k_adj_gemm_regb): 32-frequency chunks
// per set (one wave per chunk and column type) for kb / 16 = nks steps, and
// the number of chunk sets for lb.
inline int adj_regb_nbw(int nks) { return nks <= 6 ? 3 : 2; }
inline int adj_regb_sets(int nks, int lb) {
  const int nchunk = lb / 32, per = adj_regb_nbw(nks);
  return (nchunk + per - 1) / per;
}
constexpr int kAdjRegbGrid = 256;  // persistent workgroups (one per CU)

// Per-period tables of a general tile for the adjoint: FP64 (cos, sin) for
// the axis terms and the operand entries of the plan's precision (split or
// FP32 pairs) for the GEMM, one set per axis.
struct PeriodTables {
  const double2 *w64x, *w64y;
  const void *opx, *opy;
};

// gtab: non-null for a general tile (a.gen), else the square-tile tables t.
// main_ev: when given, two events recorded on st around the main-term GEMM
// (timing of that kernel alone).
hipError_t launch_adjoint(const AdjPlan &a, const int32_t *x, const int32_t *y, const int8_t *s,
                          const float *gradF, const Tables &t, void *ws, float *gx, float *gy,
                          hipStream_t st, const PeriodTables *gtab = nullptr,
                          hipEvent_t *main_ev = nullptr);
hipError_t launch_edge_grad(const float *gx, const float *gy, const int64_t *hedge,
                            const int64_t *vedge, int64_t V, int64_t E, float *g_edge,
                            hipStream_t st);

// Pupil loss and its cotangent (workspace: pupil_loss_workspace_bytes()).
size_t pupil_loss_workspace_bytes();
hipError_t launch_pupil_loss(const float *F, const float *G, const float *H, int K, int L, double r2,
                             double *loss, float *grad, void *ws, hipStream_t st);
hipError_t launch_apply_offsets(const int32_t *bx, const int32_t *by, const int64_t *hedge,
                                const int64_t *vedge, const float *off, int64_t V, int32_t *x,
                                int32_t *y, hipStream_t st, int frac_bits = 0);

// ---------------------------------------------------------------------------
// Batched form: one descriptor per clip (device copy), work lists.
// ---------------------------------------------------------------------------

// A pointer into device global memory, as a descriptor field.  A plain
// pointer read from memory is generic, so every access through it becomes a
// flat access, which the hardware counts both as a memory and as an LDS
// operation: an LDS wait then also waits for those loads.  The global address
// space in the field's type keeps the accesses global; it converts to and
// from a plain pointer.
template <typename T>
struct gptr {
  __attribute__((address_space(1))) T *p;
  __host__ __device__ operator T *() const { return (T *)p; }
  __host__ __device__ gptr &operator=(T *q) {
    p = (__attribute__((address_space(1))) T *)q;
    return *this;
  }
};

struct BatchClip {
  gptr<const int32_t> x, y;
  gptr<const int8_t> s;
  gptr<float2> F;
  gptr<int64_t> area;
  gptr<uint4> packed;
  gptr<unsigned long long> area_part;
  gptr<double2> axis_part;
  gptr<float> part;
  gptr<double> gpart;        // guard partials [chunk][slot][16 x 16]
  gptr<unsigned int> gspan;  // guard span chosen by the side kernel
  double gscale, gscale_alt;
  gptr<unsigned long long> hist;
  int64_t V, vpad, chunk, g_chunk;
  int T, shift, K, L, kp, lp, tiles_l, nsplit;
  int ax_fb_k, ax_chunks, g_chunks, hist_blocks;
  int direct;  // one split: the contraction writes F itself (no partials)
};

// K bucket of a batch clip, max(K, L) <= 63, 127, 255, 511 or larger: the
// batch takes its contraction tile variant and corners per work item per
// bucket.  Clips whose buckets share a variant share one persistent launch.
constexpr int kBatchKBuckets = 5;
__host__ __device__ inline int batch_kbucket(int K, int L) {
  const int m = K > L ? K : L;
  return m <= 63 ? 0 : (m <= 127 ? 1 : (m <= 255 ? 2 : (m <= 511 ? 3 : 4)));
}
constexpr int kBatchMaxGroups = 8;

struct BatchLaunch {
  int n_clips;
  int prec;
  const BatchClip *clips;   // device
  int pre_blocks;           // pre-pass blocks per clip
  const int4 *side_desc;    // device: (clip, 0 = histogram | 1 = guard, block) per side block
  int n_side;
  const int4 *ax_desc;      // device: (clip, frequency block, bin chunk) per axis block
  int n_ax;
  // device: (clip, tile, split) per work item, grouped by tile variant and in
  // LPT order within a group; group g (variant group_tile[g]) holds the items
  // [group_off[g], group_off[g + 1]) and runs as one persistent launch
  const int4 *items;
  int n_items;
  int n_groups;
  int group_tile[kBatchMaxGroups];
  int group_off[kBatchMaxGroups + 1];
  // device work counters: [g] group g's pass, [n_groups + g] its pass over the
  // routed clips, [2 n_groups] set when some clip is routed to split-fp16
  unsigned int *counter;
  unsigned int *route;      // device: per clip 1 if routed to split-fp16 (split-bf16 plans)
  const int *epi_off;       // device: prefix of epilogue blocks per clip [n+1]
  int n_epi;
};

// Batch of general tiles (split precisions) as one launch per step over all
// clips: the pre-pass (blocks (b, clip)), the side-stream blocks and axis
// blocks (one descriptor each), the contraction (one workgroup per (clip,
// tile, split) work item, longest first; each stages its clip's period tables
// and runs the pipelined form, or for periods past 8192 the shared-operand
// two-level form) and the epilogue (blocks mapped to clips by a prefix).  Each
// clip keeps the workspace layout of a single-clip plan, with the split count
// chosen for the whole batch.
struct GBatchClip {
  gptr<const int32_t> x, y;
  gptr<const int8_t> s;
  gptr<float2> F;
  gptr<int64_t> area;
  gptr<uint4> packed;
  gptr<uint4> words;                // two-level clips: corner words (big_word), else null
  gptr<unsigned long long> area_part, hist;
  gptr<double2> axis_part;
  gptr<float> part;
  gptr<double> gpart;
  gptr<unsigned int> gspan;
  gptr<const void> tx, ty;          // split operand tables (uint2), two-level: FP32 pairs (float2)
  gptr<const void> tx16, ty16;      // split-fp16 tables of a one-level split-bf16 clip (routing)
  gptr<const double2> w64x, w64y;   // FP64 tables, one- or two-level (axis sums and guard region)
  double gscale, gscale_alt;
  double eg, eax, eay, edc;    // alpha factors of the output grid
  int64_t V, vpad, chunk, g_chunk, ax_chunk;
  int Mx, My, K, L, kp, lp, tiles_l, nsplit, pre_blocks, hist_blocks, ax_fb_k, ax_chunks,
      g_chunks, big, nhx, nhy;
  uint32_t smask;
};

struct GBatchLaunch {
  int n_clips, prec;
  const GBatchClip *clips;  // device
  int max_pre_blocks;
  // device: (clip, 0 = histogram | 1 = guard | 2 = two-level guard, block)
  const int4 *side_desc;
  int n_side;
  // device: (clip, 0 = DFT of the histograms | 1 = two-level direct sums,
  // frequency block, chunk); after the side blocks
  const int4 *ax_desc;
  int n_ax;
  const int4 *items;        // device: (clip, tile, split), longest first
  int n_items;
  const int *epi_off;       // device: prefix of epilogue blocks per clip [n + 1]
  int n_epi;
};

// LDS of the shared-operand two-level contraction (tables rounded to 16
// bytes, then the two operand buffers of kBsOpWords 16-byte words each), and
// the static LDS of the batch contraction kernel, which holds either form.
constexpr int kBsOpWords = 4 * 2 * 128;
__host__ __device__ inline uint32_t big_shared_tab_bytes(int nhx, int nhy, bool one_tab) {
  const uint32_t e = (uint32_t)(nhx + kBigLo + (one_tab ? 0 : nhy + kBigLo));
  return (8u * e + 15u) & ~15u;
}
__host__ __device__ inline size_t big_shared_lds_bytes(int nhx, int nhy, bool one_tab) {
  return big_shared_tab_bytes(nhx, nhy, one_tab) + 16 * (size_t)(2 * kBsOpWords);
}
constexpr size_t kGBatchLds = 159 * 1024;

hipError_t launch_gbatch_prepass(const GBatchLaunch &b, hipStream_t st);
hipError_t launch_gbatch_side(const GBatchLaunch &b, hipStream_t st);
hipError_t launch_gbatch_contract(const GBatchLaunch &b, hipStream_t st);
hipError_t launch_gbatch_epilogue(const GBatchLaunch &b, hipStream_t st);

hipError_t launch_batch_prepass(const BatchLaunch &b, hipStream_t st);
hipError_t launch_batch_side(const BatchLaunch &b, const double2 *w64, hipStream_t st);
hipError_t launch_batch_contract(const BatchLaunch &b, const Tables &t, hipStream_t st);
hipError_t launch_batch_epilogue(const BatchLaunch &b, hipStream_t st);
int batch_grid(int tile, int prec);
// blocks of the epilogue launch of one clip
int epilogue_block_count(int K, int L, bool direct = false);

// Contraction tile variants (wave tile in k x l frequencies; 2 x 2 waves).
struct TileVariant {
  int id;
  int prec_mask;   // bit per Prec this variant is built for
  int wk, wl;      // frequencies per wave
  int pipe;        // loop form: 0 lean, 1 double-buffered, 2 interleaved (one wave per SIMD)
  int wg_per_cu;   // resident workgroups per CU the launch is sized for
  int chunk_mult;  // corners per split are a multiple of this
};
int n_tile_variants();
const TileVariant &tile_variant(int i);

// Pruned continuous Haar transform of one tile (Sec. III-B1).
constexpr int kHaarMaxJ = 13;      // deepest pyramid (tiles up to 8192 units)
constexpr int kHaarMaxSide = 8192; // largest Nx, Ny
struct HaarArgs {
  const int32_t *x, *y;  // corners, loop order
  const int8_t *s;       // corner signs
  const int64_t *off;    // polygon offsets [M + 1]
  int64_t M, V;
  int Nx, Ny, J;
  int64_t *U;            // [4^J] integer sums
  double *W;             // [4^J] coefficients, or nullptr
  int64_t *stats;        // [2] cells visited, cell-corner pairs; or nullptr
};
// Workspace of the Haar launches for M polygons (control words, copies of the
// coarse levels' block, task counts and the list of extra tasks of split
// polygons).
size_t haar_workspace_bytes(int64_t M);
// clears U and the control words, plans the split of large polygons
hipError_t launch_haar_prep(const HaarArgs &a, void *ws, hipStream_t st);
// the quadtree walk (coefficients into U)
hipError_t launch_haar_walk(const HaarArgs &a, void *ws, hipStream_t st);
// coarse levels from their copies into U; W from U when W is not null
hipError_t launch_haar_scale(const HaarArgs &a, void *ws, hipStream_t st);

}  // namespace fcfs
