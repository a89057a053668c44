// Step S9: AdamW (Section 5.1: AdamW, learning rate 1e-3) on the packed
// parameter vector, the refresh of the GEMM-layout weight copies, and two
// memory utilities (a fill, and the plain copy that calibrates HBM counters).
#include "common.hpp"

namespace hgnn {

namespace {

inline int cdiv(long long a, int b) { return (int)((a + b - 1) / b); }

// AdamW over the packed vector.  *step counts the completed steps; this one
// is t = *step + 1 (the staging launch that follows advances the counter).
// Each workgroup derives the bias corrections 1/(1-b1^t), 1/(1-b2^t) in
// double from the device-resident counter, so a captured step replays
// correctly.
__global__ void __launch_bounds__(256)
k_adamw(float *__restrict__ theta, const float *__restrict__ g, float *__restrict__ m,
        float *__restrict__ v, long long n, float lr, double b1d, double b2d, float b1,
        float omb1, float b2, float omb2, float eps, float decay,
        const long long *__restrict__ step) {
  __shared__ float corr[2];
  if (threadIdx.x == 0) {
    const double t = (double)(*step + 1);
    corr[0] = (float)(1.0 / (1.0 - pow(b1d, t)));
    corr[1] = (float)(1.0 / (1.0 - pow(b2d, t)));
  }
  __syncthreads();
  const float c1 = corr[0], c2 = corr[1];
  auto one = [&](float th, float gi, float &mi, float &vi) {
    mi = b1 * mi + omb1 * gi;
    vi = b2 * vi + omb2 * gi * gi;
    return th * decay - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  };
  // four elements per thread, 16-byte accesses (the arrays are 16-byte
  // aligned); the last n % 4 elements one by one
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x, i0 = 4 * q;
  if (i0 + 4 <= n) {
    f4 th = *reinterpret_cast<const f4 *>(theta + i0);
    const f4 gi = *reinterpret_cast<const f4 *>(g + i0);
    f4 mi = *reinterpret_cast<const f4 *>(m + i0);
    f4 vi = *reinterpret_cast<const f4 *>(v + i0);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      float me = mi[e], ve = vi[e];
      th[e] = one(th[e], gi[e], me, ve);
      mi[e] = me;
      vi[e] = ve;
    }
    *reinterpret_cast<f4 *>(m + i0) = mi;
    *reinterpret_cast<f4 *>(v + i0) = vi;
    *reinterpret_cast<f4 *>(theta + i0) = th;
  } else {
    for (long long i = i0; i < n; ++i) {
      float mi = m[i], vi = v[i];
      theta[i] = one(theta[i], g[i], mi, vi);
      m[i] = mi;
      v[i] = vi;
    }
  }
}

// FP32 copies store the value; BF16 copies store hi = bf16(v) and, in a
// second array, lo = bf16(v - hi), so that hi + lo carries ~16 mantissa bits.
template <typename T>
__device__ __forceinline__ void put(void *dst, void *dst_lo, size_t i, float v) {
  if constexpr (sizeof(T) == 4) {
    reinterpret_cast<float *>(dst)[i] = v;
  } else {
    const __bf16 hi = (__bf16)v;
    reinterpret_cast<__bf16 *>(dst)[i] = hi;
    reinterpret_cast<__bf16 *>(dst_lo)[i] = (__bf16)(v - (float)hi);
  }
}

// Per layer: the four GEMM-layout copies of W^m and W^p (index 0..3 of o).
//  Wds   [2H, Fp]     rows n < H: W^m[n, 0:F]; n >= H: W^m[n-H, F:2F]; zero pad
//  Wpp   [H, Fp+12H]  W^p with its first block padded from F to Fp columns
//  WpTA  [4H, 3H]     WpTA[c, j H + m] = W^p[m, F + 4 H j + c]
//  WhdsT [Fp, 3H]     [W^p[:, c]; W^m[:, c]; W^m[:, F + c]]^T, zero rows c >= F
//  weT   [Fe, H]      weT[f, c] = W^m[c, 2F + f] (FP32 in both precisions)
// With nb degree buckets the update copies are per bucket q instead:
//  Wpp   [nb][H, Fp+4H]  [W_h padded | W_eff(q)]
//  WpTA  [nb][4H, H]     W_eff(q)^T
// where W_eff(q)[m, c] = W_0 + s+(q) W_+ + s-(q) W_- (blocks of W^p at
// columns F + c, F + 4H + c, F + 8H + c), evaluated in FP32 in that order
// with the FP32 scalers of the table.
__device__ __forceinline__ float w_eff(const float *__restrict__ Wp, int ldp, int F, int H,
                                       const float *__restrict__ table, int q, int m, int c) {
  const float *row = Wp + (size_t)m * ldp + F + c;
  return fmaf(table[2 * q + 1], row[8 * H], fmaf(table[2 * q], row[4 * H], row[0]));
}

// One row of the untransposed copies: rows 0 .. 2H - 1 are Wds's, the next
// nb H (or H) the update copy's, the last Fe weT's; the workgroup's threads
// stride over the row's columns (one division per row, coalesced loads and
// stores along it).
template <typename T>
__device__ __forceinline__ void stage_row(const float *__restrict__ Wm,
                                          const float *__restrict__ Wp, int F, int Fp,
                                          int H, int Fe, int nb,
                                          const float *__restrict__ table,
                                          const StageOut &o, int row) {
  const int ldm = 2 * F + Fe, ldp = F + 12 * H;
  const int wu = nb ? Fp + 4 * H : Fp + 12 * H; // row width of the update copy
  const int r1 = 2 * H, r2 = r1 + (nb ? nb : 1) * H;
  if (row < r1) {
    const float *src = row < H ? Wm + (size_t)row * ldm : Wm + (size_t)(row - H) * ldm + F;
    for (int c = threadIdx.x; c < Fp; c += blockDim.x)
      put<T>(o.hi[0], o.lo[0], (size_t)row * Fp + c, c < F ? src[c] : 0.f);
  } else if (row < r2) {
    const int rr = row - r1, q = rr / H, m = rr - q * H;
    const float *src = Wp + (size_t)m * ldp;
    for (int c = threadIdx.x; c < wu; c += blockDim.x) {
      float v = 0.f;
      if (c < Fp) { if (c < F) v = src[c]; }
      else if (nb) v = w_eff(Wp, ldp, F, H, table, q, m, c - Fp);
      else v = src[F + (c - Fp)];
      put<T>(o.hi[1], o.lo[1], (size_t)rr * wu + c, v);
    }
  } else if (row < r2 + Fe) {
    const int f = row - r2;
    for (int c = threadIdx.x; c < H; c += blockDim.x)
      o.weT[(size_t)f * H + c] = Wm[(size_t)c * ldm + 2 * F + f];
  }
}

// The transposed copies (WpTA and WhdsT of the layout above), through LDS in
// 32 x 32 tiles so that both the reads of W^p / W^m rows and the writes are
// coalesced: dst[c, col0 + m] = sum_s coef_s src_s[m, c] for m < H, c < C
// (zero for c >= cvalid).  Tile jobs per layer:
//  bucketed: nb jobs, job q: C = 4H, dst = WpTA + q 4H H (ld H), sources
//            the W_0, W_+, W_- blocks with 1, s+(q), s-(q);
//  else:     3 jobs, job j: C = 4H, dst = WpTA (ld 3H) at column j H, source
//            the block j of W^p's 12H aggregate columns;
//  then 3 WhdsT jobs, job j: C = Fp (F valid), dst = WhdsT (ld 3H) at column
//  j H, source W^p[:, 0:F], W^m[:, 0:F] or W^m[:, F:2F].
template <typename T>
__device__ void stage_transposed(const float *__restrict__ Wm, const float *__restrict__ Wp,
                                 int F, int Fp, int H, int Fe, int nb,
                                 const float *__restrict__ table, const StageOut &o,
                                 int tile) {
  __shared__ float tl[32][33];
  const int ldm = 2 * F + Fe, ldp = F + 12 * H;
  const int mt = (H + 31) / 32;
  const int ta = ((4 * H + 31) / 32) * mt; // tiles of one WpTA job
  const int tw = ((Fp + 31) / 32) * mt;    // tiles of one WhdsT job
  const int na = nb ? nb : 3;
  int job, jt, C, cvalid, ld_dst, col0, nsrc = 1;
  const float *src[3] = {nullptr, nullptr, nullptr};
  float coef[3] = {1.f, 0.f, 0.f};
  int ld_src;
  void *dhi, *dlo;
  size_t dbase = 0;
  if (tile < na * ta) {
    job = tile / ta;
    jt = tile % ta;
    C = cvalid = 4 * H;
    ld_src = ldp;
    dhi = o.hi[2];
    dlo = o.lo[2];
    if (nb) {
      dbase = (size_t)job * 4 * H * H;
      ld_dst = H;
      col0 = 0;
      src[0] = Wp + F;
      src[1] = Wp + F + 4 * H;
      src[2] = Wp + F + 8 * H;
      coef[1] = table[2 * job];
      coef[2] = table[2 * job + 1];
      nsrc = 3;
    } else {
      ld_dst = 3 * H;
      col0 = job * H;
      src[0] = Wp + F + 4 * H * job;
    }
  } else {
    tile -= na * ta;
    if (tile >= 3 * tw) return;
    job = tile / tw;
    jt = tile % tw;
    C = Fp;
    cvalid = F;
    ld_dst = 3 * H;
    col0 = job * H;
    dhi = o.hi[3];
    dlo = o.lo[3];
    src[0] = job == 0 ? Wp : (job == 1 ? Wm : Wm + F);
    ld_src = job == 0 ? ldp : ldm;
  }
  const int c0 = (jt / mt) * 32, m0 = (jt % mt) * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5; // 32 x 8 threads
  // read rows m (coalesced along c) into the tile
  for (int r = ty; r < 32; r += 8) {
    const int m = m0 + r, c = c0 + tx;
    float v = 0.f;
    if (m < H && c < cvalid) {
      const size_t off = (size_t)m * ld_src + c;
      v = src[0][off];
      if (nsrc == 3) v = fmaf(coef[2], src[2][off], fmaf(coef[1], src[1][off], v));
    }
    tl[r][tx] = v;
  }
  __syncthreads();
  // write rows c (coalesced along m)
  for (int r = ty; r < 32; r += 8) {
    const int c = c0 + r, m = m0 + tx;
    if (c < C && m < H) put<T>(dhi, dlo, dbase + (size_t)c * ld_dst + col0 + m, tl[tx][r]);
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_stage_t_layer(const float *__restrict__ Wm, const float *__restrict__ Wp, int F, int Fp,
                int H, int Fe, int nb, const float *__restrict__ table, StageOut o) {
  stage_transposed<T>(Wm, Wp, F, Fp, H, Fe, nb, table, o, blockIdx.x);
}

template <typename T>
__global__ void __launch_bounds__(256)
k_stage_layer(const float *__restrict__ Wm, const float *__restrict__ Wp, int F, int Fp,
              int H, int Fe, int nb, const float *__restrict__ table, StageOut o) {
  stage_row<T>(Wm, Wp, F, Fp, H, Fe, nb, table, o, blockIdx.x);
}

// Every layer's copies in one launch (blockIdx.y = layer): the first `rows`
// workgroups write the untransposed copies a row each, the rest the
// transposed copies a 32 x 32 tile each (the two sets are independent);
// optionally advances the AdamW step counter once the preceding update has
// been applied.  One launch instead of two: the step's launches cost host
// time that the BF16 step is short enough to feel.
template <typename T>
__global__ void __launch_bounds__(256)
k_stage_all(const StageDesc *__restrict__ tab, int H, int Fe, int nb,
            const float *__restrict__ table, long long *bump, int rows) {
  const StageDesc &d = tab[blockIdx.y];
  if ((int)blockIdx.x < rows)
    stage_row<T>(d.Wm, d.Wp, d.F, d.Fp, H, Fe, nb, table, d.o, blockIdx.x);
  else
    stage_transposed<T>(d.Wm, d.Wp, d.F, d.Fp, H, Fe, nb, table, d.o, blockIdx.x - rows);
  if (bump && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *bump += 1;
}

__global__ void k_fill(float *p, long long n, float v) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}


// Plain float4 copy used to calibrate the HBM byte counters.
__global__ void __launch_bounds__(256) k_calib_copy(const f4 *__restrict__ src,
                                                    f4 *__restrict__ dst, long long n4) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n4) dst[i] = src[i];
}
} // namespace

hipError_t launch_adamw(float *theta, const float *g, float *m, float *v, int64_t n,
                        float lr, double b1, double b2, float eps, float wd,
                        const long long *step, hipStream_t s) {
  if (n > 0)
    k_adamw<<<cdiv((n + 3) / 4, 256), 256, 0, s>>>(theta, g, m, v, n, lr, b1, b2, (float)b1,
                                         (float)(1.0 - b1), (float)b2, (float)(1.0 - b2),
                                         eps, (float)(1.0 - (double)lr * wd), step);
  return hipGetLastError();
}

// rows of the untransposed copies (Wds, Wpp, weT) of one layer
static int stage_rows(int H, int Fe, int nb) { return (2 + (nb ? nb : 1)) * H + Fe; }

// 32 x 32 tiles of the transposed copies of one layer
static int stage_t_tiles(int Fp, int H, int nb) {
  const int mt = (H + 31) / 32;
  return (nb ? nb : 3) * ((4 * H + 31) / 32) * mt + 3 * ((Fp + 31) / 32) * mt;
}

hipError_t launch_stage_all(const StageDesc *tab, int L, int maxFp, int H, int Fe, int nb,
                            const float *table, int to_bf16, long long *bump, hipStream_t s) {
  const int rows = stage_rows(H, Fe, nb);
  const dim3 grid(rows + stage_t_tiles(maxFp, H, nb), L);
  if (to_bf16) k_stage_all<__bf16><<<grid, 256, 0, s>>>(tab, H, Fe, nb, table, bump, rows);
  else k_stage_all<float><<<grid, 256, 0, s>>>(tab, H, Fe, nb, table, bump, rows);
  return hipGetLastError();
}

hipError_t launch_stage_layer(const float *Wm, const float *Wp, int F, int Fp, int H,
                              int Fe, int nb, const float *table, const StageOut &o,
                              int to_bf16, hipStream_t s) {
  const int rows = stage_rows(H, Fe, nb);
  const int tiles = stage_t_tiles(Fp, H, nb);
  if (to_bf16) {
    k_stage_layer<__bf16><<<rows, 256, 0, s>>>(Wm, Wp, F, Fp, H, Fe, nb, table, o);
    k_stage_t_layer<__bf16><<<tiles, 256, 0, s>>>(Wm, Wp, F, Fp, H, Fe, nb, table, o);
  } else {
    k_stage_layer<float><<<rows, 256, 0, s>>>(Wm, Wp, F, Fp, H, Fe, nb, table, o);
    k_stage_t_layer<float><<<tiles, 256, 0, s>>>(Wm, Wp, F, Fp, H, Fe, nb, table, o);
  }
  return hipGetLastError();
}

// Seeded initialisation: element j of the packed vector (global index) is
// bound * k * 2^-23 with k = (z >> 40) - 2^23 in [-2^23, 2^23), where z is
// the j-th output of SplitMix64 started from `seed` (Steele, Lea and Flood,
// OOPSLA 2014): z = mix(seed + (j + 1) * 0x9E3779B97F4A7C15).  A counter
// generator, so every element is computed on its own; k * 2^-23 is exact in
// FP32 and the product with the FP32 bound is rounded once.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t j) {
  uint64_t z = seed + (j + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void __launch_bounds__(256)
k_init_uniform(float *__restrict__ p, long long off, long long n, float bound, uint64_t seed) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const uint64_t z = splitmix64_at(seed, (uint64_t)(off + t));
  const int k = (int)(z >> 40) - (1 << 23);
  p[off + t] = bound * ((float)k * 0x1p-23f);
}

hipError_t launch_init_uniform(float *p, int64_t off, int64_t n, float bound, uint64_t seed,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_init_uniform<<<cdiv(n, 256), 256, 0, s>>>(p, off, n, bound, seed);
  return hipGetLastError();
}

hipError_t launch_fill(float *p, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_fill<<<cdiv(n, 256), 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_calib_copy(const float *src, float *dst, long long n, hipStream_t s) {
  const long long n4 = n / 4;
  if (n4 <= 0) return hipSuccess;
  k_calib_copy<<<cdiv(n4, 256), 256, 0, s>>>(reinterpret_cast<const f4 *>(src),
                                             reinterpret_cast<f4 *>(dst), n4);
  return hipGetLastError();
}

} // namespace hgnn
