// Pruned continuous Haar transform (PCHT) of rectilinear polygons on gfx950.
//
// Sec. III-B1: the 2-D Haar coefficients of a polygon are intersection areas
// of the polygon with the cells of a quadtree over the tile, scaled by
// 2^j / sqrt(Nx Ny); a cell wholly inside or outside the polygon ends the
// recursion.  Per non-terminating cell (j, kx, ky) the four child areas
// A_nm (n: x half, m: y half) give
//     hg = A00 + A01 - A10 - A11,  gh = A00 + A10 - A01 - A11,
//     hh = A00 - A01 - A10 + A11,
// and the children with 0 < A_nm < |child| are visited next.
//
// Intersection areas (Algorithm 1) are sums over the polygon's horizontal
// edges.  The corner form of the indicator, sum_v s_v [x >= x_v][y >= y_v],
// pairs the two corners of a horizontal edge (xa, y) - (xb, y) into the strip
// s_left [min, max) x [y, inf) with the sign of its left corner, so
//     Area(P inside [a1,a2) x [b1,b2)) = sum_h s_left (clamp(v; a1, a2) - clamp(u; a1, a2))
//                                               * (b2 - clamp(y; b1, b2))
// (u, v the edge's x range): per edge and child two med3 and a subtraction
// per axis, then four multiply-adds for the four children.  This is the
// upward-strip form of Algorithm 1 (which sums downward strips); for a closed
// loop both give the same area, and this one needs no orientation test.
// Coordinates are clamped to the tile first, which changes no area inside it.
// All area arithmetic is 32-bit with wraparound: every true area is below
// 2^26 (Nx, Ny <= 8192), so the wrapped sums are exact.
//
// Mapping: one wave per task (a polygon or, for a large polygon, a share of
// its subtrees), tasks dealt round-robin over the waves.  The polygon's horizontal
// edges are staged in LDS (a negative strip with its ends swapped, so that
// its width is negative and one signed multiply-add loop serves both) and
// read as broadcasts.  All cells of the coarse
// levels that meet the polygon's bounding box go through one batch (cells
// that turn out wholly inside or outside give zero coefficients and no
// children); below that a LIFO stack of cell codes in LDS is popped 64 at a
// time (one cell per lane).  Coefficients go to the caller's int64 pyramid
// with 64-bit atomic adds (integers: the result does not depend on the
// order).  The levels below kHaarCoarse, which nearly every polygon meets, and
// the scaling coefficient would make every wave add into the same few
// entries; their sums go to kHaarReplicas copies of the coarse block instead
// (copy chosen by the workgroup, area summed per wave first), and the last
// pass adds the copies into U beside scaling U to doubles.
#include "fcfs_internal.h"

namespace fcfs {
namespace {

// Stack of cell codes per wave.  LIFO batches of at most 64 cells that push
// at most 4 children each keep at most 64 + 192 (J - 4) entries in the worst
// case (every child active); 3072 covers J <= 13 with room to spare.
constexpr int kHaarStack = 3072;
// Corners whose edges are staged in LDS per pass (a polygon with more
// corners is restaged per batch).  A valid loop has half as many horizontal
// edges as corners; the stage holds one slot per corner so that no input can
// overrun it.
constexpr int kHaarStageCorners = 512;
constexpr int kHaarStage = kHaarStageCorners;
// Workgroups of one wave; at 20 KB of LDS each, eight fit on a CU.  The grid
// holds twice that many: a workgroup takes tasks blockIdx, blockIdx + grid,
// ..., so the larger grid hands the tasks out in finer shares as workgroups
// finish (layout clip, J = 12: 8 per CU 139 us, 16 per CU 129 us, 32 or 64
// per CU no faster).
constexpr int kHaarWgPerCU = 16;
constexpr int kCUs = 256;
// Levels j < kHaarCoarse (the pyramid's top-left kHaarCoarseSide square,
// scaling coefficient included) are summed in kHaarReplicas copies of that
// square in the workspace.
constexpr int kHaarCoarse = 6;
constexpr int kHaarCoarseSide = 1 << kHaarCoarse;
constexpr int kHaarCoarseN = kHaarCoarseSide * kHaarCoarseSide;
constexpr int kHaarReplicas = 64;
constexpr size_t kHaarRepBytes = sizeof(unsigned long long) * kHaarCoarseN * kHaarReplicas;
static_assert(kHaarReplicas == 64, "the fold splits the copies eight ways, eight each");

static_assert(kHaarStack >= 256 + 192 * kHaarMaxJ, "cell stack too small for the deepest pyramid");

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Orders LDS accesses between the lanes of the one wave of a workgroup.  The
// wave's LDS operations complete in program order, so no s_barrier (and no
// wait for outstanding global atomics, which a workgroup barrier's fence
// would add) is needed, only a stop to compiler reordering.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int med3i(int a, int lo, int hi) {
  int r;
  asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(lo), "v"(hi));
  return r;
}

// acc += a * b on 24-bit signed operands, 32-bit wraparound result.
__device__ __forceinline__ void mad24(uint32_t &acc, int a, int b) {
  asm("v_mad_i32_i24 %0, %1, %2, %0" : "+v"(acc) : "v"(a), "v"(b));
}

// Stages the horizontal edges that start at corners [c0, c0 + cn) of the
// polygon (corners o0 .. o0 + K - 1, edge i joins corner i to corner i + 1
// mod K) at stg[0, ne), clamped to the tile.  A strip with a positive left
// corner is stored as {u, v, y} (u < v), a negative one as {v, u, y}: the
// width v - u then carries the sign.
__device__ __forceinline__ void stage(const int32_t *__restrict__ x, const int32_t *__restrict__ y,
                                      const int8_t *__restrict__ s, int64_t o0, int64_t K,
                                      int64_t c0, int cn, int Nx, int Ny, int4 *stg, int &ne) {
  const int lane = threadIdx.x;
  int cnt = 0;
  for (int i0 = 0; i0 < cn; i0 += 64) {
    const int64_t i = c0 + i0 + lane;
    int u = 0, v = 0, yy = 0, sg = 0;
    if (i0 + lane < cn) {
      const int64_t a = o0 + i, b = o0 + (i + 1 == K ? 0 : i + 1);
      const int xa = x[a], xb = x[b], ya = y[a];
      if (ya == y[b] && xa != xb) {
        u = clampi(min(xa, xb), 0, Nx);
        v = clampi(max(xa, xb), 0, Nx);
        yy = clampi(ya, 0, Ny);
        sg = xa < xb ? s[a] : s[b];
        if (u == v) sg = 0;
      }
    }
    const uint64_t bl = __ballot(sg != 0);
    if (sg != 0) stg[cnt + (int)lanes_below(bl)] = sg > 0 ? make_int4(u, v, yy, 0) : make_int4(v, u, yy, 0);
    cnt += __popcll(bl);
  }
  ne = __builtin_amdgcn_readfirstlane(cnt);
  wave_sync();
}

// One strip {u, v, y} (u > v for a negative one) added to the four child
// areas (see the header).
__device__ __forceinline__ void strip(const int4 &e, int a1, int mid, int a2, int b1, int my,
                                      int b2, uint32_t (&acc)[4]) {
  const int w0 = med3i(e.y, a1, mid) - med3i(e.x, a1, mid);
  const int w1 = med3i(e.y, mid, a2) - med3i(e.x, mid, a2);
  const int h0 = my - med3i(e.z, b1, my);
  const int h1 = b2 - med3i(e.z, my, b2);
  mad24(acc[0], w0, h0);
  mad24(acc[1], w0, h1);
  mad24(acc[2], w1, h0);
  mad24(acc[3], w1, h1);
}

// Adds the strips stg[0, ne) to the four child areas of the cell with x
// range [a1, a1 + 2 hx) and y range [my - hy, my + hy).  Strips are read four
// at a time, one group ahead of the arithmetic, so that the LDS latency
// overlaps it.
__device__ __forceinline__ void child_areas(const int4 *stg, int ne, int a1, int hx, int my, int hy,
                                            uint32_t (&acc)[4]) {
  const int mid = a1 + hx, a2 = mid + hx, b1 = my - hy, b2 = my + hy;
  int i = 0;
  if (ne >= 4) {
    int4 n0 = stg[0], n1 = stg[1], n2 = stg[2], n3 = stg[3];
    for (i = 4; i + 4 <= ne; i += 4) {
      const int4 e0 = n0, e1 = n1, e2 = n2, e3 = n3;
      n0 = stg[i];
      n1 = stg[i + 1];
      n2 = stg[i + 2];
      n3 = stg[i + 3];
      strip(e0, a1, mid, a2, b1, my, b2, acc);
      strip(e1, a1, mid, a2, b1, my, b2, acc);
      strip(e2, a1, mid, a2, b1, my, b2, acc);
      strip(e3, a1, mid, a2, b1, my, b2, acc);
    }
    strip(n0, a1, mid, a2, b1, my, b2, acc);
    strip(n1, a1, mid, a2, b1, my, b2, acc);
    strip(n2, a1, mid, a2, b1, my, b2, acc);
    strip(n3, a1, mid, a2, b1, my, b2, acc);
  }
  for (; i < ne; ++i) strip(stg[i], a1, mid, a2, b1, my, b2, acc);
}

// Clears U, the coarse-block copies and the control words.
__global__ void k_haar_reset(unsigned long long *__restrict__ U, int64_t n,
                             unsigned long long *__restrict__ rep,
                             unsigned long long *__restrict__ ctl, unsigned long long *__restrict__ stats) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) U[i] = 0ull;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)kHaarCoarseN * kHaarReplicas;
       i += stride)
    rep[i] = 0ull;
  if (blockIdx.x == 0 && threadIdx.x < 16) {
    ctl[threadIdx.x] = 0ull;
    if (stats && threadIdx.x < 2) stats[threadIdx.x] = 0ull;
  }
}

// Splitting of large polygons.  The cells of a polygon's quadtree below the
// split level L0 (cells of at least kHaarSplitCell units) form independent
// subtrees; a polygon whose estimated work exceeds kHaarTaskPairs cell-corner
// pairs is walked by n tasks: every task refines the cells above L0 (only
// task 0 emits their coefficients), and task t keeps the L0 cells whose hash
// is t mod n.  The integer sums do not depend on the partition.  Split cells
// of 128 units balance the layout clip's walk better than 256 (148 -> 139 us
// at 8 workgroups per CU; 512: 168 us; 64: as 128).
constexpr int kHaarSplitCell = 128;
constexpr int64_t kHaarTaskPairs = 16384;
constexpr int kHaarMaxSplit = 64;

// Task (of nt) that owns the subtree of split-level cell (kx, ky).
__device__ __forceinline__ int cell_owner(uint32_t kx, uint32_t ky, int nt) {
  uint32_t h = kx * 0x9E3779B1u ^ ky * 0x85EBCA77u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  return (int)__umulhi(h, (uint32_t)nt);
}

// One thread per polygon: task count from the estimated work (boundary
// length in finest cells, about twice the cells the walk visits, times the
// corner count); the extra tasks (m, t), t >= 1, are appended to a list of
// `cap` entries (a polygon gets fewer tasks when the list is full).
__global__ void k_haar_plan(const int32_t *__restrict__ x, const int32_t *__restrict__ y,
                            const int64_t *__restrict__ off, int64_t M, int64_t V, int Nx,
                            int Ny, int J, int L0, int *__restrict__ nsplit,
                            int2 *__restrict__ extra, int64_t cap,
                            unsigned long long *__restrict__ ctl) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  int64_t o0 = off[m], o1 = off[m + 1];
  o0 = o0 < 0 ? 0 : (o0 > V ? V : o0);
  o1 = o1 < o0 ? o0 : (o1 > V ? V : o1);
  const int64_t K = o1 - o0;
  int n = 1;
  if (L0 > 0 && K > 1) {
    int64_t per = 0;
    for (int64_t i = 0; i < K; ++i) {
      const int64_t a = o0 + i, b = o0 + (i + 1 == K ? 0 : i + 1);
      per += llabs((int64_t)x[b] - x[a]) + llabs((int64_t)y[b] - y[a]);
    }
    const int64_t wf = max(1, min(Nx, Ny) >> (J - 1));
    const int64_t work = 2 * (per / wf) * K;
    n = (int)min<int64_t>(kHaarMaxSplit, max<int64_t>(1, (work + kHaarTaskPairs - 1) / kHaarTaskPairs));
  }
  if (n > 1) {
    const unsigned long long base = atomicAdd(&ctl[2], (unsigned long long)(n - 1));
    const int64_t room = (int64_t)base < cap ? cap - (int64_t)base : 0;
    n = 1 + (int)min<int64_t>(n - 1, room);
    for (int t = 1; t < n; ++t) extra[base + t - 1] = make_int2((int)m, t);
  }
  nsplit[m] = n;
}

// Task i of the M + extra tasks goes to workgroup i mod gridDim (a static
// order: one shared task counter served past the per-XCD caches costs more
// than the imbalance it removes).  ctl[1]: set when a stack push had to be
// dropped (cannot happen within the bound above; kept so that no push can
// leave LDS); ctl[2]: extra tasks requested by the plan.
__global__ __launch_bounds__(64) void k_haar_walk(const int32_t *__restrict__ x,
                                                  const int32_t *__restrict__ y,
                                                  const int8_t *__restrict__ s,
                                                  const int64_t *__restrict__ off, int64_t M,
                                                  int64_t V, int Nx, int Ny, int J, int L0,
                                                  const int *__restrict__ nsplit,
                                                  const int2 *__restrict__ extra, int64_t cap,
                                                  unsigned long long *__restrict__ U,
                                                  unsigned long long *__restrict__ rep,
                                                  unsigned long long *__restrict__ ctl,
                                                  unsigned long long *__restrict__ stats) {
  __shared__ uint32_t stk[kHaarStack];
  __shared__ int4 stg[kHaarStage];
  const int lane = threadIdx.x;
  const int64_t side = (int64_t)1 << J;
  const int64_t n_extra = min<int64_t>((int64_t)__atomic_load_n(&ctl[2], __ATOMIC_RELAXED), cap);
  const int64_t n_tasks = M + n_extra;
  // this workgroup's copy of the coarse block
  unsigned long long *const crep = rep + (size_t)(blockIdx.x % kHaarReplicas) * kHaarCoarseN;
  unsigned long long n_cells = 0, n_pairs = 0;
  int64_t wave_area = 0;  // scaling-coefficient sum of this wave's polygons
  for (int64_t task = blockIdx.x; task < n_tasks; task += gridDim.x) {
    int64_t m;
    int t;
    if (task < M) {
      m = task;
      t = 0;
    } else {
      const int2 e = extra[task - M];
      m = e.x;
      t = e.y;
    }
    const int nt = nsplit[m];
    int64_t o0 = off[m], o1 = off[m + 1];
    o0 = o0 < 0 ? 0 : (o0 > V ? V : o0);
    o1 = o1 < o0 ? o0 : (o1 > V ? V : o1);
    const int64_t K = o1 - o0;
    // scaling coefficient (the polygon's area inside the tile) and the
    // bounding box of the clamped corners
    uint32_t a = 0;
    int bx0 = Nx, bx1 = 0, by0 = Ny, by1 = 0;
    for (int64_t i = lane; i < K; i += 64) {
      const int xv = clampi(x[o0 + i], 0, Nx), yv = clampi(y[o0 + i], 0, Ny);
      const uint32_t q = (uint32_t)(Nx - xv) * (uint32_t)(Ny - yv);
      const int sv = s[o0 + i];
      a += sv > 0 ? q : (sv < 0 ? 0u - q : 0u);
      bx0 = min(bx0, xv);
      bx1 = max(bx1, xv);
      by0 = min(by0, yv);
      by1 = max(by1, yv);
    }
    a = wave_sum(a);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      bx0 = min(bx0, __shfl_xor(bx0, o, 64));
      bx1 = max(bx1, __shfl_xor(bx1, o, 64));
      by0 = min(by0, __shfl_xor(by0, o, 64));
      by1 = max(by1, __shfl_xor(by1, o, 64));
    }
    const int64_t area = (int32_t)a;
    if (t == 0) wave_area += area;
    if (!(J > 0 && area > 0 && area < (int64_t)Nx * Ny)) continue;
    const bool one_pass = K <= kHaarStageCorners;
    int ne = 0;
    if (one_pass) stage(x, y, s, o0, K, 0, (int)K, Nx, Ny, stg, ne);
    // Coarse batch: every cell of levels 0..j0 that meets the bounding box
    // [bx0, bx1) x [by0, by1), j0 the deepest level with at most 64 such
    // cells in total.  Lane i takes the i-th of them, level by level.
    int j0 = 0, ncoarse = 0;
    int cj = 0, ckx = 0, cky = 0;
    {
      // level-j cell widths are (Nx >> J) 2^(J-j): one division per task,
      // then shifts (floor(floor(a / c) / 2^s) = floor(a / (c 2^s)))
      const int cx = Nx >> J, cy = Ny >> J;
      const int qx0 = bx0 / cx, qx1 = (bx1 - 1) / cx, qy0 = by0 / cy, qy1 = (by1 - 1) / cy;
      int cum = 0;
      for (int j = 0; j < J; ++j) {
        const int sh = J - j;
        const int ix0 = qx0 >> sh, iy0 = qy0 >> sh;
        const int nx = (qx1 >> sh) - ix0 + 1, ny = (qy1 >> sh) - iy0 + 1;
        if (cum + nx * ny > 64) break;
        if (lane >= cum && lane < cum + nx * ny) {
          // r / nx for r < 64: the half offset keeps the quotient away from
          // integers, so an approximate reciprocal floors correctly
          const int r = lane - cum;
          const int q = (int)(((float)r + 0.5f) * __builtin_amdgcn_rcpf((float)nx));
          cj = j;
          ckx = ix0 + (r - q * nx);
          cky = iy0 + q;
        }
        cum += nx * ny;
        j0 = j;
      }
      ncoarse = cum;
    }
    int size = 0;
    bool coarse = true;
    for (;;) {
      int n, top, j, kx, ky;
      bool act;
      if (coarse) {
        n = ncoarse;
        top = 0;
        act = lane < n;
        j = act ? cj : 0;
        kx = act ? ckx : 0;
        ky = act ? cky : 0;
      } else {
        if (size == 0) break;
        n = size < 64 ? size : 64;
        top = size - n;
        act = lane < n;
        const uint32_t code = act ? stk[top + lane] : 0u;
        j = (int)(code >> 26);
        kx = (int)((code >> 13) & 8191u);
        ky = (int)(code & 8191u);
      }
      const int wx = Nx >> j, wy = Ny >> j, hx = wx >> 1, hy = wy >> 1;
      const int a1 = (int)__umul24((uint32_t)kx, (uint32_t)wx);
      const int my = (int)__umul24((uint32_t)ky, (uint32_t)wy) + hy;
      uint32_t pa[4] = {0u, 0u, 0u, 0u};
      if (one_pass) {
        child_areas(stg, ne, a1, hx, my, hy, pa);
      } else {
        for (int64_t c0 = 0; c0 < K; c0 += kHaarStageCorners) {
          const int cn = (int)(K - c0 < kHaarStageCorners ? K - c0 : kHaarStageCorners);
          wave_sync();
          stage(x, y, s, o0, K, c0, cn, Nx, Ny, stg, ne);
          child_areas(stg, ne, a1, hx, my, hy, pa);
        }
      }
      const int A00 = (int)pa[0], A01 = (int)pa[1], A10 = (int)pa[2], A11 = (int)pa[3];
      const int full = hx * hy;
      // Ownership: cells above the split level are refined by every task of
      // the polygon and emitted by task 0; below it, by the task that owns
      // the split-level ancestor.  Popped cells are always this task's.
      bool owned = true;
      if (coarse && nt > 1 && j >= L0)
        owned = cell_owner((uint32_t)(kx >> (j - L0)), (uint32_t)(ky >> (j - L0)), nt) == t;
      const bool emit = act && owned && (j >= L0 || t == 0);
      const int own = A00 + A01 + A10 + A11;
      const bool visited = !coarse || (own > 0 && own < 4 * full);
      if (emit) {
        const int64_t p = (int64_t)1 << j;
        const int hg = A00 + A01 - A10 - A11;
        const int gh = A00 + A10 - A01 - A11;
        const int hh = A00 - A01 - A10 + A11;
        // level j's entries lie in rows and columns below 2p: levels below
        // kHaarCoarse stay inside the coarse block
        unsigned long long *const dst = j < kHaarCoarse ? crep : U;
        const int64_t row = j < kHaarCoarse ? kHaarCoarseSide : side;
        if (hg) atomicAdd(&dst[ky * row + p + kx], (unsigned long long)(int64_t)hg);
        if (gh) atomicAdd(&dst[(p + ky) * row + kx], (unsigned long long)(int64_t)gh);
        if (hh) atomicAdd(&dst[(p + ky) * row + p + kx], (unsigned long long)(int64_t)hh);
      }
      const int n_mine = __popcll(__ballot(emit && visited));
      n_cells += (unsigned long long)n_mine;
      n_pairs += (unsigned long long)n_mine * (unsigned long long)K;
      // children that meet the boundary, pushed in child order 00, 01, 10, 11
      // (from the coarse batch only those of level j0 + 1); at the split
      // level only this task's share
      const bool deeper = act && owned && j + 1 < J && (!coarse || j == j0);
      const int Av[4] = {A00, A01, A10, A11};
      int pos = top;
      uint32_t ccode[4];
      uint64_t bal[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const uint32_t cx = (uint32_t)(2 * kx + (c >> 1)), cy = (uint32_t)(2 * ky + (c & 1));
        bool live = deeper && Av[c] > 0 && Av[c] < full;
        if (nt > 1 && j + 1 == L0) live = live && cell_owner(cx, cy, nt) == t;
        bal[c] = __ballot(live);
        ccode[c] = ((uint32_t)(j + 1) << 26) | (cx << 13) | cy;
      }
      wave_sync();  // every lane has read its cell before the slots are reused
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int slot = pos + (int)lanes_below(bal[c]);
        if (((bal[c] >> lane) & 1ull) != 0ull) {
          if (slot < kHaarStack)
            stk[slot] = ccode[c];
          else
            ctl[1] = 1ull;
        }
        pos += __popcll(bal[c]);
      }
      size = pos < kHaarStack ? pos : kHaarStack;
      coarse = false;
      wave_sync();
    }
    wave_sync();
  }
  if (lane == 0 && wave_area != 0) atomicAdd(&crep[0], (unsigned long long)wave_area);
  if (lane == 0 && stats && n_cells) {
    atomicAdd(&stats[0], n_cells);
    atomicAdd(&stats[1], n_pairs);
  }
}

// Coarse entries per fold block: 256 threads, eight per entry, each summing
// an eighth of the copies (eight loads in flight), partial sums met in LDS.
constexpr int kHaarFoldPerBlock = 32;

// Last pass.  Blocks [0, nfold): the entries of the coarse block (rows and
// columns below cs = min(2^J, kHaarCoarseSide)) summed from the copies into U
// (and W).  The other blocks, when W is wanted, stream the rest of the
// pyramid: W = U * 2^level / sqrt(Nx Ny), the level of entry (row, col)
// being floor(log2(max(row, col))) (0 for the scaling coefficient).
__global__ __launch_bounds__(256) void k_haar_finish(unsigned long long *__restrict__ U,
                                                     double *__restrict__ W,
                                                     const unsigned long long *__restrict__ rep,
                                                     int J, double r, int64_t n, int nfold) {
  __shared__ unsigned long long part[256];
  const uint32_t cs = (uint32_t)min(1 << J, kHaarCoarseSide);
  auto level = [](uint32_t row, uint32_t col) {
    const uint32_t mx = row > col ? row : col;
    return mx ? 31 - __clz(mx) : 0;
  };
  if ((int)blockIdx.x < nfold) {
    const uint32_t k = threadIdx.x % kHaarFoldPerBlock, sub = threadIdx.x / kHaarFoldPerBlock;
    const uint32_t i = blockIdx.x * kHaarFoldPerBlock + k;
    const bool live = i < cs * cs;
    const uint32_t row = live ? i / cs : 0u, col = live ? i - row * cs : 0u;
    const int e = (int)(row * kHaarCoarseSide + col);
    unsigned long long w[8];
    constexpr int per = kHaarReplicas / 8;
#pragma unroll
    for (int u = 0; u < per; ++u) w[u] = live ? rep[(size_t)(sub * per + u) * kHaarCoarseN + e] : 0ull;
    part[threadIdx.x] = ((w[0] + w[1]) + (w[2] + w[3])) + ((w[4] + w[5]) + (w[6] + w[7]));
    __syncthreads();
    if (sub == 0 && live) {
      unsigned long long v = 0ull;
#pragma unroll
      for (int q = 0; q < 8; ++q) v += part[q * kHaarFoldPerBlock + k];
      const int64_t at = ((int64_t)row << J) + col;
      U[at] = v;
      if (W) W[at] = (double)(long long)v * (r * (double)(1u << level(row, col)));
    }
    return;
  }
  const int64_t stride = (int64_t)(gridDim.x - nfold) * blockDim.x;
  const uint32_t mask = (1u << J) - 1u;
  for (int64_t i = (int64_t)(blockIdx.x - nfold) * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint32_t row = (uint32_t)(i >> J), col = (uint32_t)i & mask;
    if (row < cs && col < cs) continue;
    W[i] = (double)(long long)U[i] * (r * (double)(1u << level(row, col)));
  }
}

}  // namespace

int haar_split_level(int Nx, int Ny, int J) {
  int L0 = 0;
  while (L0 + 1 < J && (std::min(Nx, Ny) >> (L0 + 1)) >= kHaarSplitCell) ++L0;
  return L0;
}

size_t haar_workspace_bytes(int64_t M) {
  const int64_t cap = std::max<int64_t>(M, 4096);
  return 256 + kHaarRepBytes + ((sizeof(int) * (size_t)M + 255) & ~(size_t)255) +
         sizeof(int2) * (size_t)cap;
}

namespace {
// Workspace layout: control words (256 bytes), the coarse-block copies, task
// counts per polygon, the extra-task list.
struct HaarWs {
  unsigned long long *ctl;
  unsigned long long *rep;
  int *nsplit;
  int2 *extra;
  int64_t cap;
};
HaarWs haar_ws(const HaarArgs &a, void *ws) {
  HaarWs w;
  char *b = static_cast<char *>(ws);
  w.ctl = reinterpret_cast<unsigned long long *>(b);
  w.rep = reinterpret_cast<unsigned long long *>(b + 256);
  w.nsplit = reinterpret_cast<int *>(b + 256 + kHaarRepBytes);
  w.extra = reinterpret_cast<int2 *>(b + 256 + kHaarRepBytes +
                                     ((sizeof(int) * (size_t)a.M + 255) & ~(size_t)255));
  w.cap = std::max<int64_t>(a.M, 4096);
  return w;
}
int pyramid_blocks(int J) {
  const int64_t n = (int64_t)1 << (2 * J);
  return (int)std::min<int64_t>(4096, std::max<int64_t>(1, (n + 255) / 256));
}
}  // namespace

hipError_t launch_haar_prep(const HaarArgs &a, void *ws, hipStream_t st) {
  const HaarWs w = haar_ws(a, ws);
  const int64_t n = (int64_t)1 << (2 * a.J);
  hipLaunchKernelGGL(k_haar_reset, dim3(std::max(pyramid_blocks(a.J), 64)), dim3(256), 0, st,
                     reinterpret_cast<unsigned long long *>(a.U), n, w.rep, w.ctl,
                     reinterpret_cast<unsigned long long *>(a.stats));
  hipError_t e = hipGetLastError();
  if (e || a.M == 0) return e;
  hipLaunchKernelGGL(k_haar_plan, dim3((unsigned)((a.M + 255) / 256)), dim3(256), 0, st, a.x, a.y,
                     a.off, a.M, a.V, a.Nx, a.Ny, a.J, haar_split_level(a.Nx, a.Ny, a.J), w.nsplit,
                     w.extra, w.cap, w.ctl);
  return hipGetLastError();
}

hipError_t launch_haar_walk(const HaarArgs &a, void *ws, hipStream_t st) {
  if (a.M == 0) return hipSuccess;
  const HaarWs w = haar_ws(a, ws);
  const int64_t g = std::min<int64_t>(a.M + w.cap, (int64_t)kCUs * kHaarWgPerCU);
  hipLaunchKernelGGL(k_haar_walk, dim3((unsigned)g), dim3(64), 0, st, a.x, a.y, a.s, a.off, a.M,
                     a.V, a.Nx, a.Ny, a.J, haar_split_level(a.Nx, a.Ny, a.J), w.nsplit, w.extra,
                     w.cap, reinterpret_cast<unsigned long long *>(a.U), w.rep, w.ctl,
                     reinterpret_cast<unsigned long long *>(a.stats));
  return hipGetLastError();
}

hipError_t launch_haar_scale(const HaarArgs &a, void *ws, hipStream_t st) {
  const HaarWs w = haar_ws(a, ws);
  const int cs = std::min(1 << a.J, kHaarCoarseSide);
  const int nfold = (cs * cs + kHaarFoldPerBlock - 1) / kHaarFoldPerBlock;
  const int64_t n = (int64_t)1 << (2 * a.J);
  const double r = 1.0 / std::sqrt((double)a.Nx * (double)a.Ny);
  const int g = nfold + (a.W ? pyramid_blocks(a.J) : 0);
  hipLaunchKernelGGL(k_haar_finish, dim3(g), dim3(256), 0, st,
                     reinterpret_cast<unsigned long long *>(a.U), a.W, w.rep, a.J, r, n, nfold);
  return hipGetLastError();
}

}  // namespace fcfs
