// Lattice (FFT) form of the forward transform, FP64 (gfx950).
//
// The general term of Prop. 3 (Sec. III-C1) needs
//   S(k, l) = sum_v s_v e(k x_v) e(l y_v),  e(t) = e^{-j 2 pi t / T},
// which, for integer corners, is the 2-D DFT of the corner image
// C[x][y] = sum of s_v over the corners at (x mod T, y mod T): the Step 4
// formulation of the paper.  Here it is taken in two passes that exploit the
// sparsity of C and the band |k| <= K, |l| <= L:
//   rows:    D(x, l) = sum_y C[x][y] e(l y)  for l = 1..L, one x-row at a time
//            from the exact integer row image (O(V L) work);
//   columns: S(k, l) = sum_x D(x, l) e(k x), an FFT of length T per l
//            (O(L T log T)), of which |k| <= K are kept;
// then F[k, l] = alpha_{k,l} S(k, l) and F[-k, -l] = conj F[k, l].  The axes and
// DC come from the same kernels as the contraction form.  All sums are FP64,
// every twiddle an exact entry of the FP64 table: the result is the direct
// evaluation up to FP64 rounding, an independent check of the MFMA path.
#include "fcfs_device.h"

namespace fcfs {

constexpr int kFftChunk = 8;      // nonzeros of a row per twiddle-table chunk
constexpr int kFftMaxA = 128;     // l = 32 a + b: a < 128 (L <= 4095)

// Corners binned by x mod T: counts, exclusive offsets, cursors.
__global__ __launch_bounds__(256) void k_fft_clear(int *__restrict__ p, int n) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = 0;
}

__global__ __launch_bounds__(256) void k_fft_count(const int32_t *__restrict__ x, int64_t V,
                                                   uint32_t tmask, int *__restrict__ cnt) {
  for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < V; v += (int64_t)gridDim.x * 256)
    atomicAdd(&cnt[(uint32_t)x[v] & tmask], 1);
}

// Exclusive prefix of T <= 8192 counts, one block of 1024 threads.
__global__ __launch_bounds__(1024) void k_fft_scan(const int *__restrict__ cnt, int T,
                                                   int *__restrict__ off) {
  __shared__ int part[1024];
  const int per = (T + 1023) / 1024;
  const int b0 = threadIdx.x * per;
  int sum = 0;
  for (int i = 0; i < per; ++i)
    if (b0 + i < T) sum += cnt[b0 + i];
  part[threadIdx.x] = sum;
  __syncthreads();
  // Hillis-Steele inclusive scan over the 1024 partial sums
  for (int o = 1; o < 1024; o <<= 1) {
    const int v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int run = part[threadIdx.x] - sum;
  for (int i = 0; i < per; ++i)
    if (b0 + i < T) {
      off[b0 + i] = run;
      run += cnt[b0 + i];
    }
  if (threadIdx.x == 1023) off[T] = part[1023];
}

// list entry: y mod T in the low 13 bits, bit 31 set for s = -1.  The order
// inside a bin is arbitrary; the row pass only forms integer sums from it.
__global__ __launch_bounds__(256) void k_fft_scatter(const int32_t *__restrict__ x,
                                                     const int32_t *__restrict__ y,
                                                     const int8_t *__restrict__ s, int64_t V,
                                                     uint32_t tmask, const int *__restrict__ off,
                                                     int *__restrict__ cur,
                                                     uint32_t *__restrict__ list) {
  for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < V;
       v += (int64_t)gridDim.x * 256) {
    const uint32_t xb = (uint32_t)x[v] & tmask;
    const int pos = off[xb] + atomicAdd(&cur[xb], 1);
    list[pos] = ((uint32_t)y[v] & tmask) | (s[v] < 0 ? 0x80000000u : 0u);
  }
}

// Rows: D[x][l - 1] = sum_y C[x][y] e(l y), l = 1..L.  The twiddles
// e(l y) = e(b y) e(32 a y) e(1024 c y), l = 1024 c + 32 a + b, are products
// of exact FP64 table entries kept in small per-nonzero tables.  Each row's
// nonzeros are summed in increasing y, so the FP64 sums run in a fixed order
// whatever the order of the bin.
//
// Sparse rows (at most kFftSparse corners): one wave per row.  The row's list
// entries are sorted by y with a bitonic sort in the wave's LDS slice, equal y
// are merged into exact integer weights, then each lane accumulates its l.
// Dense rows go to an overflow list handled by k_fft_rows_dense.
constexpr int kFftSparse = 512;   // corners of a row on the one-wave path
constexpr int kFftRowWaves = 4;

// Accumulates acc[m] += sum_j val_j e(l y_j) for l = l0 + lstride m (m < 16,
// l <= L) over the nonzeros (ys[j], vs[j]), j < nnz, of one row in increasing
// j; ta/tb/tc: this wave's tables, filled by its 64 lanes.
__device__ __forceinline__ void row_accumulate(const uint16_t *ys, const int *vs, int nnz, int L,
                                               int shift, const double2 *__restrict__ w64,
                                               double2 (*ta)[32], double2 (*tb)[32],
                                               double2 (*tc)[4], int lane, int l0, int lstride,
                                               double2 *acc) {
  const uint32_t mask = (uint32_t)(kTabN - 1);
  const int na = min(32, L / 32 + 1), nc = L / 1024 + 1;
  for (int j0 = 0; j0 < nnz; j0 += kFftChunk) {
    const int nj = min(kFftChunk, nnz - j0);
    // ta[j][b] = e^{+j 2 pi b y / T}, tb[j][a] = e^{+j 2 pi 32 a y / T},
    // tc[j][c] = e^{+j 2 pi 1024 c y / T}
    for (int i = lane; i < nj * 32; i += 64) {
      const int j = i >> 5, q = i & 31;
      const uint32_t yy = ys[j0 + j];
      ta[j][q] = w64[((uint32_t)q * yy << shift) & mask];
      if (q < na) tb[j][q] = w64[((uint32_t)(32 * q) * yy << shift) & mask];
      if (q < nc) tc[j][q] = w64[((uint32_t)(1024 * q) * yy << shift) & mask];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int j = 0; j < nj; ++j) {
      const double cv = (double)vs[j0 + j];
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        const int l = l0 + lstride * m;
        if (l > L) break;
        const double2 p = ta[j][l & 31], q = tb[j][(l >> 5) & 31];
        double re = p.x * q.x - p.y * q.y, im = p.x * q.y + p.y * q.x;
        if (l >= 1024) {
          const double2 r = tc[j][l >> 10];
          const double r2 = re * r.x - im * r.y, i2 = re * r.y + im * r.x;
          re = r2;
          im = i2;
        }
        // e(l y) = conj of the product
        acc[m].x = fma(cv, re, acc[m].x);
        acc[m].y = fma(-cv, im, acc[m].y);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(64 * kFftRowWaves) void k_fft_rows(
    const int *__restrict__ off, const uint32_t *__restrict__ list, int T, int shift, int L,
    const double2 *__restrict__ w64, double2 *__restrict__ D, int *__restrict__ overflow) {
  __shared__ uint32_t keys[kFftRowWaves][kFftSparse];
  __shared__ int vals[kFftRowWaves][kFftSparse];
  __shared__ uint16_t ys[kFftRowWaves][kFftSparse];
  __shared__ double2 ta[kFftRowWaves][kFftChunk][32];
  __shared__ double2 tb[kFftRowWaves][kFftChunk][32];
  __shared__ double2 tc[kFftRowWaves][kFftChunk][4];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int x = blockIdx.x * kFftRowWaves + wave;
  if (x >= T) return;
  const int b0 = off[x], n = off[x + 1] - b0;
  if (n > kFftSparse) {  // dense row: handled by k_fft_rows_dense
    if (lane == 0) overflow[1 + atomicAdd(&overflow[0], 1)] = x;
    return;
  }
  uint32_t *kw = keys[wave];
  // keys: y (13 bits) << 1 | sign; padded to a power of two with ~0
  int np = 1;
  while (np < n) np <<= 1;
  for (int i = lane; i < np; i += 64) {
    uint32_t k = 0xFFFFFFFFu;
    if (i < n) {
      const uint32_t e = list[b0 + i];
      k = ((e & 0x1FFFu) << 1) | (e >> 31);
    }
    kw[i] = k;
  }
  wave_sync();
  // bitonic sort ascending
  for (int size = 2; size <= np; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = lane; i < np / 2; i += 64) {
        const int lo = 2 * i - (i & (stride - 1));
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const uint32_t a = kw[lo], b = kw[hi];
        if ((a > b) == up) {
          kw[lo] = b;
          kw[hi] = a;
        }
      }
      wave_sync();
    }
  // merge equal y into integer weights: run starts in order
  int *vw = vals[wave];
  uint16_t *yw = ys[wave];
  int nnz = 0;
  for (int i0 = 0; i0 < n; i0 += 64) {
    const int i = i0 + lane;
    const uint32_t k = i < n ? kw[i] : 0xFFFFFFFFu;
    const bool start = i < n && (i == 0 || (kw[i - 1] >> 1) != (k >> 1));
    const unsigned long long bal = __ballot(start);
    if (start) {
      int sum = 0;
      for (int j = i; j < n && (kw[j] >> 1) == (k >> 1); ++j) sum += (kw[j] & 1u) ? -1 : 1;
      const int pos = nnz + __popcll(bal & ((1ull << lane) - 1ull));
      vw[pos] = sum;
      yw[pos] = (uint16_t)(k >> 1);
    }
    nnz += __popcll(bal);
  }
  wave_sync();
  double2 acc[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) acc[m] = make_double2(0.0, 0.0);
  row_accumulate(yw, vw, nnz, L, shift, w64, ta[wave], tb[wave], tc[wave], lane, 1 + lane, 64,
                 acc);
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int l = 1 + lane + 64 * m;
    if (l <= L) D[(size_t)x * L + (l - 1)] = acc[m];
  }
}

// Dense rows (more than kFftSparse corners), one workgroup each: the exact
// integer row image in LDS, compacted in y order, then the same accumulation
// with the l split over the four waves.
__global__ __launch_bounds__(256) void k_fft_rows_dense(const int *__restrict__ off,
                                                        const uint32_t *__restrict__ list, int T,
                                                        int shift, int L,
                                                        const double2 *__restrict__ w64,
                                                        double2 *__restrict__ D,
                                                        const int *__restrict__ overflow) {
  __shared__ int img[kTabN];       // row image, then the compacted weights
  __shared__ uint16_t ny[kTabN];   // y of the compacted nonzeros
  __shared__ double2 ta[4][kFftChunk][32];
  __shared__ double2 tb[4][kFftChunk][32];
  __shared__ double2 tc[4][kFftChunk][4];
  __shared__ int s_cnt[256];
  const int nrows = overflow[0];
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  for (int r = blockIdx.x; r < nrows; r += gridDim.x) {
    const int x = overflow[1 + r];
    __syncthreads();
    for (int i = t; i < T; i += 256) img[i] = 0;
    __syncthreads();
    const int b0 = off[x], b1 = off[x + 1];
    for (int i = b0 + t; i < b1; i += 256) {
      const uint32_t e = list[i];
      atomicAdd(&img[e & 0x1FFFu], (e >> 31) ? -1 : 1);
    }
    __syncthreads();
    const int per = (T + 255) / 256;
    int v[32];
    int c = 0;
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      v[i] = 0;
      if (i < per && t * per + i < T) {
        v[i] = img[t * per + i];
        c += v[i] != 0;
      }
    }
    s_cnt[t] = c;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
      const int add = t >= o ? s_cnt[t - o] : 0;
      __syncthreads();
      s_cnt[t] += add;
      __syncthreads();
    }
    const int nnz = s_cnt[255];
    int pos = s_cnt[t] - c;
    __syncthreads();  // every thread has read its image bins
#pragma unroll
    for (int i = 0; i < 32; ++i)
      if (i < per && v[i] != 0) {
        img[pos] = v[i];
        ny[pos] = (uint16_t)(t * per + i);
        ++pos;
      }
    __syncthreads();
    // wave w accumulates l = 1 + 64 w + lane + 256 m
    double2 acc[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) acc[m] = make_double2(0.0, 0.0);
    row_accumulate(ny, img, nnz, L, shift, w64, ta[wave], tb[wave], tc[wave], lane,
                   1 + 64 * wave + lane, 256, acc);
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int l = 1 + 64 * wave + lane + 256 * m;
      if (l <= L) D[(size_t)x * L + (l - 1)] = acc[m];
    }
  }
}

// Columns: for l = 1..L, S(k, l) = sum_x D[x][l - 1] e(k x) by a radix-2
// decimation-in-time FFT of length T in LDS (bit-reversed load), then
// F[k, l] = alpha_{k,l} S(k, l), F[-k, -l] = conj F[k, l] for 1 <= |k| <= K.
// Workgroups with consecutive l share their D cache lines: blockIdx is mapped
// so that they land on the same XCD (dispatch is round-robin over 8 XCDs).
__global__ __launch_bounds__(1024) void k_fft_cols(const double2 *__restrict__ D, int T,
                                                   int logT, int K, int L,
                                                   const double2 *__restrict__ w64,
                                                   float2 *__restrict__ F) {
  __shared__ double2 a[kTabN];
  const int per_xcd = gridDim.x / 8;  // the grid is 8 * ceil(L / 8)
  const int li = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (li >= L) return;
  const int l = li + 1;
  const int t = threadIdx.x;
  for (int x = t; x < T; x += 1024) {
    const uint32_t r = __brev((uint32_t)x) >> (32 - logT);
    a[r] = D[(size_t)x * L + li];
  }
  const uint32_t mask = (uint32_t)(kTabN - 1);
  for (int s = 1; s <= logT; ++s) {
    __syncthreads();
    const int half = 1 << (s - 1);
    for (int b = t; b < T / 2; b += 1024) {
      const int grp = b >> (s - 1), r = b & (half - 1);
      const int i0 = (grp << s) + r, i1 = i0 + half;
      // e^{-j 2 pi r / 2^s} = conj(table[r 8192 / 2^s])
      const double2 w = w64[((uint32_t)r << (kTabBits - s)) & mask];
      const double2 u = a[i0], v = a[i1];
      const double tr = v.x * w.x + v.y * w.y, ti = v.y * w.x - v.x * w.y;
      a[i0] = make_double2(u.x + tr, u.y + ti);
      a[i1] = make_double2(u.x - tr, u.y - ti);
    }
  }
  __syncthreads();
  const size_t W = 2 * (size_t)L + 1;
  for (int k = 1 + t; k <= K; k += 1024) {
    for (int sg = 0; sg < 2; ++sg) {
      const int kk = sg ? -k : k;
      const double2 S = a[(uint32_t)kk & (uint32_t)(T - 1)];
      const double al = -(double)T / (4.0 * kPi * kPi * (double)kk * (double)l);
      const float re = (float)(al * S.x), im = (float)(al * S.y);
      F[(size_t)(K + kk) * W + (L + l)] = make_float2(re, im);
      F[(size_t)(K - kk) * W + (L - l)] = make_float2(re, -im);
    }
  }
}

hipError_t launch_fft(const FwdPlan &p, const int32_t *x, const int32_t *y, const int8_t *s,
                      const double2 *w64, void *ws, float *F, hipStream_t st) {
  char *w = (char *)ws;
  int *cnt = (int *)(w + p.off_fcnt), *cur = cnt + p.T, *off = cur + p.T;
  uint32_t *list = (uint32_t *)(w + p.off_flist);
  double2 *D = (double2 *)(w + p.off_fd);
  const uint32_t tmask = (uint32_t)(p.T - 1);
  int logT = 0;
  while ((1 << logT) < p.T) ++logT;
  hipLaunchKernelGGL(k_fft_clear, dim3((2 * p.T + 255) / 256), dim3(256), 0, st, cnt, 2 * p.T);
  const unsigned vb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, (p.V + 255) / 256));
  if (p.V > 0) hipLaunchKernelGGL(k_fft_count, dim3(vb), dim3(256), 0, st, x, p.V, tmask, cnt);
  hipLaunchKernelGGL(k_fft_scan, dim3(1), dim3(1024), 0, st, cnt, p.T, off);
  if (p.V > 0)
    hipLaunchKernelGGL(k_fft_scatter, dim3(vb), dim3(256), 0, st, x, y, s, p.V, tmask, off, cur,
                       list);
  int *overflow = off + p.T + 1;  // [count, rows...]
  hipLaunchKernelGGL(k_fft_clear, dim3(1), dim3(256), 0, st, overflow, 1);
  hipLaunchKernelGGL(k_fft_rows, dim3((p.T + kFftRowWaves - 1) / kFftRowWaves),
                     dim3(64 * kFftRowWaves), 0, st, off, list, p.T, p.shift, p.L, w64, D,
                     overflow);
  hipLaunchKernelGGL(k_fft_rows_dense, dim3(256), dim3(256), 0, st, off, list, p.T, p.shift, p.L,
                     w64, D, overflow);
  // 8 * ceil(L / 8) blocks: every l is reached by the XCD-grouped mapping
  hipLaunchKernelGGL(k_fft_cols, dim3((unsigned)(8 * ((p.L + 7) / 8))), dim3(1024), 0, st, D, p.T,
                     logT, p.K, p.L, w64, (float2 *)F);
  return hipGetLastError();
}

}  // namespace fcfs
