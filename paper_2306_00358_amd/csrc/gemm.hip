// Dense contractions of the HOTRG step as MFMA GEMMs for gfx950.
//
// Every contraction of a step (environment halves and combine, the three
// coarse contractions; Sec. 2 of arXiv 2306.00358) is a plain GEMM once its
// operands are laid out with the contracted legs contiguous; the index
// permutation that the next contraction needs is applied in the epilogue
// (OutMap), so no separate transpose pass touches the large intermediates.
//
// FP64: v_mfma_f64_16x16x4f64.  Lane layout of one 16x16x4 product
// (64 lanes): A[i][k] from lane i + 16k, B[k][j] from lane j + 16k, and the
// four accumulator values of lane L hold D[L/16 + 4v][L % 16], v = 0..3.
#include <hip/hip_runtime.h>

#include <cstdlib>

#include <map>
#include <mutex>

#include "internal.h"

namespace hotrg {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ long long map_row(const OutMap& o, int m) {
  int m2 = m % o.r2;
  int q = m / o.r2;
  int m1 = q % o.r1;
  int m0 = q / o.r1;
  return (long long)m0 * o.s0 + (long long)m1 * o.s1 + (long long)m2 * o.s2;
}

__device__ __forceinline__ long long map_col(const OutMap& o, int n) {
  int n2 = n % o.c2;
  int q = n / o.c2;
  int n1 = q % o.c1;
  int n0 = q / o.c1;
  return (long long)n0 * o.t0 + (long long)n1 * o.t1 + (long long)n2 * o.t2;
}

__device__ __forceinline__ void atomic_max_bits(unsigned long long* p, double v) {
  // |v| >= 0: the IEEE bit pattern of a non-negative double orders like
  // the value; NaN patterns compare above +inf and propagate.
  atomicMax(p, (unsigned long long)__double_as_longlong(v));
}

__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Block tile BM x BN, K slab BK; 4 waves in a 2 x 2 arrangement, each wave
// owns a (BM/2) x (BN/2) sub-tile made of 16x16 MFMA tiles.  Operand tiles
// go global -> registers -> LDS; the next slab's global loads are issued
// before the current slab's MFMAs so that they overlap.
template <int BM, int BN, int BK, int BL>
__device__ __forceinline__ void f64_tile(const double* __restrict__ A, long long lda,
                                         const double* __restrict__ B, long long ldb,
                                         double* __restrict__ C, const OutMap& om, int M, int N,
                                         int K, unsigned long long* maxbits, int m0, int n0) {
  constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 16, TN = WN / 16;
  constexpr int A_PER = BM * BK / 256, B_PER = BN * BK / 256;
  static_assert(BM * BK % 256 == 0 && BN * BK % 256 == 0, "tile must split over 256 threads");
  __shared__ double As[BM][BK + 1];
  // B_NCONTIG: Bs[k][n]; B_KCONTIG: Bs[n][k] (padded against bank conflicts)
  __shared__ double Bs[BL == B_NCONTIG ? BK : BN][BL == B_NCONTIG ? BN : BK + 1];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  d4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  double ra[A_PER], rb[B_PER];

  auto load = [&](int k0) {
#pragma unroll
    for (int p = 0; p < A_PER; ++p) {
      int e = tid + 256 * p;
      int r = e / BK, c = e % BK;
      int gm = m0 + r, gk = k0 + c;
      ra[p] = (gm < M && gk < K) ? A[(long long)gm * lda + gk] : 0.0;
    }
#pragma unroll
    for (int p = 0; p < B_PER; ++p) {
      int e = tid + 256 * p;
      if (BL == B_NCONTIG) {
        int r = e / BN, c = e % BN;
        int gk = k0 + r, gn = n0 + c;
        rb[p] = (gk < K && gn < N) ? B[(long long)gk * ldb + gn] : 0.0;
      } else {
        int r = e / BK, c = e % BK;
        int gn = n0 + r, gk = k0 + c;
        rb[p] = (gk < K && gn < N) ? B[(long long)gn * ldb + gk] : 0.0;
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int p = 0; p < A_PER; ++p) {
      int e = tid + 256 * p;
      As[e / BK][e % BK] = ra[p];
    }
#pragma unroll
    for (int p = 0; p < B_PER; ++p) {
      int e = tid + 256 * p;
      if (BL == B_NCONTIG)
        Bs[e / BN][e % BN] = rb[p];
      else
        Bs[e / BK][e % BK] = rb[p];
    }
  };

  const int li = lane & 15, lk = lane >> 4;
  load(0);
  for (int k0 = 0; k0 < K; k0 += BK) {
    __syncthreads();
    store();
    __syncthreads();
    if (k0 + BK < K) load(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = As[wm * WM + i * 16 + li][kk + lk];
#pragma unroll
      for (int j = 0; j < TN; ++j)
        b[j] = (BL == B_NCONTIG) ? Bs[kk + lk][wn * WN + j * 16 + li]
                                 : Bs[wn * WN + j * 16 + li][kk + lk];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }

  // epilogue: scatter through the OutMap, track max |C|
  double mx = 0.0;
  long long coff[TN];
  bool cok[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    int n = n0 + wn * WN + j * 16 + li;
    cok[j] = n < N;
    coff[j] = cok[j] ? map_col(om, n) : 0;
  }
#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int m = m0 + wm * WM + i * 16 + lk + 4 * v;
      if (m >= M) continue;
      long long roff = map_row(om, m);
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        if (!cok[j]) continue;
        double x = acc[i][j][v];
        C[roff + coff[j]] = x;
        mx = fmax(mx, fabs(x));
      }
    }
  }
  if (maxbits) {
    mx = wave_max(mx);
    if (lane == 0) atomic_max_bits(maxbits, mx);
  }
}

template <int BM, int BN, int BK, int BL>
__global__ __launch_bounds__(256) void k_gemm_f64(const double* __restrict__ A, long long lda,
                                                  const double* __restrict__ B, long long ldb,
                                                  double* __restrict__ C, OutMap om, int M, int N,
                                                  int K, unsigned long long* maxbits, int kchunk,
                                                  long long cstride) {
  // split-K: block z sums k in [z*kchunk, min((z+1)*kchunk, K)) into C + z*cstride
  if (kchunk > 0) {
    const int z = blockIdx.z;
    const int kb = z * kchunk;
    A += kb;
    B += BL == B_NCONTIG ? (long long)kb * ldb : kb;
    C += z * cstride;
    K = K - kb < kchunk ? K - kb : kchunk;
  }
  f64_tile<BM, BN, BK, BL>(A, lda, B, ldb, C, om, M, N, K, maxbits, blockIdx.y * BM,
                           blockIdx.x * BN);
}

// Grouped form over a device table of products (the block eigensolver of a
// batch of problems): workgroup b takes tile b - begin[i] of the item i whose
// range holds b; an item whose gate reads 0 skips its tiles.
template <int BM, int BN, int BK, int BL>
__global__ __launch_bounds__(256) void k_gemm_f64_grouped(const F64Item* __restrict__ items,
                                                          const int* __restrict__ begin,
                                                          int count) {
  int lo = 0, hi = count - 1;
  const int b = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (begin[mid] <= b) lo = mid; else hi = mid - 1;
  }
  const F64Item& it = items[lo];
  if (it.gate && *it.gate == 0) return;
  const int local = b - begin[lo];
  const int tn = (it.N + BN - 1) / BN;
  f64_tile<BM, BN, BK, BL>(it.A, it.lda, it.B, it.ldb, it.C, out_rowmajor(it.ldc), it.M, it.N,
                           it.K, nullptr, (local / tn) * BM, (local % tn) * BN);
}

int f64_group_tiles(const F64Item& it) { return ((it.M + 63) / 64) * ((it.N + 63) / 64); }

void gemm_f64_grouped(int blayout, const F64Item* d_items, const int* d_begin, int count,
                      int tiles, hipStream_t s) {
  if (count <= 0 || tiles <= 0) return;
  if (blayout == B_NCONTIG)
    hipLaunchKernelGGL((k_gemm_f64_grouped<64, 64, 16, B_NCONTIG>), dim3(tiles), dim3(256), 0, s,
                       d_items, d_begin, count);
  else
    hipLaunchKernelGGL((k_gemm_f64_grouped<64, 64, 16, B_KCONTIG>), dim3(tiles), dim3(256), 0, s,
                       d_items, d_begin, count);
}

// Large-GEMM variant: 128 x 128 block tile, K slab BK = 32, LDS double
// buffered so that one barrier per slab separates the MFMAs of slab s from
// the LDS stores of slab s+1 (whose global loads were issued before the
// MFMAs of slab s).  TAG only gives each call site its own kernel symbol,
// so per-contraction times can be read from a kernel trace.
template <int BL, int TAG>
__global__ __launch_bounds__(256) void k_gemm_f64_big(const double* __restrict__ A, long long lda,
                                                      const double* __restrict__ B, long long ldb,
                                                      double* __restrict__ C, OutMap om, int M,
                                                      int N, int K, unsigned long long* maxbits) {
  constexpr int BM = 128, BN = 128, BK = 32;
  constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 16, TN = WN / 16;
  constexpr int A_PER = BM * BK / 256, B_PER = BN * BK / 256;
  constexpr int AS = BK + 1;                               // A row pitch (doubles)
  constexpr int BR = BL == B_NCONTIG ? BK : BN;            // B rows in LDS
  constexpr int BP = BL == B_NCONTIG ? BN : BK + 1;        // B row pitch
  __shared__ double As[2][BM * AS];
  __shared__ double Bs[2][BR * BP];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;

  d4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  double ra[A_PER], rb[B_PER];
  auto load = [&](int k0) {
#pragma unroll
    for (int p = 0; p < A_PER; ++p) {
      int e = tid + 256 * p;
      int r = e / BK, c = e % BK;
      int gm = m0 + r, gk = k0 + c;
      ra[p] = (gm < M && gk < K) ? A[(long long)gm * lda + gk] : 0.0;
    }
#pragma unroll
    for (int p = 0; p < B_PER; ++p) {
      int e = tid + 256 * p;
      if (BL == B_NCONTIG) {
        int r = e / BN, c = e % BN;
        int gk = k0 + r, gn = n0 + c;
        rb[p] = (gk < K && gn < N) ? B[(long long)gk * ldb + gn] : 0.0;
      } else {
        int r = e / BK, c = e % BK;
        int gn = n0 + r, gk = k0 + c;
        rb[p] = (gk < K && gn < N) ? B[(long long)gn * ldb + gk] : 0.0;
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int p = 0; p < A_PER; ++p) {
      int e = tid + 256 * p;
      As[buf][(e / BK) * AS + e % BK] = ra[p];
    }
#pragma unroll
    for (int p = 0; p < B_PER; ++p) {
      int e = tid + 256 * p;
      if (BL == B_NCONTIG)
        Bs[buf][(e / BN) * BP + e % BN] = rb[p];
      else
        Bs[buf][(e / BK) * BP + e % BK] = rb[p];
    }
  };

  const int li = lane & 15, lk = lane >> 4;
  const int nslab = (K + BK - 1) / BK;
  load(0);
  store(0);
  __syncthreads();
  for (int s = 0; s < nslab; ++s) {
    const int cur = s & 1;
    if (s + 1 < nslab) load((s + 1) * BK);
    const double* as = As[cur];
    const double* bs = Bs[cur];
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = as[(wm * WM + i * 16 + li) * AS + kk + lk];
#pragma unroll
      for (int j = 0; j < TN; ++j)
        b[j] = (BL == B_NCONTIG) ? bs[(kk + lk) * BP + wn * WN + j * 16 + li]
                                 : bs[(wn * WN + j * 16 + li) * BP + kk + lk];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (s + 1 < nslab) store(cur ^ 1);
    __syncthreads();
  }

  double mx = 0.0;
  long long coff[TN];
  bool cok[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    int n = n0 + wn * WN + j * 16 + li;
    cok[j] = n < N;
    coff[j] = cok[j] ? map_col(om, n) : 0;
  }
#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int m = m0 + wm * WM + i * 16 + lk + 4 * v;
      if (m >= M) continue;
      long long roff = map_row(om, m);
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        if (!cok[j]) continue;
        double x = acc[i][j][v];
        C[roff + coff[j]] = x;
        mx = fmax(mx, fabs(x));
      }
    }
  }
  if (maxbits) {
    mx = wave_max(mx);
    if (lane == 0) atomic_max_bits(maxbits, mx);
  }
}

template <int BM, int BN, int BK>
static void launch_f64(const double* A, long long lda, const double* B, long long ldb, int bl,
                       double* C, const OutMap& om, int M, int N, int K,
                       unsigned long long* maxbits, hipStream_t s, int kchunk = 0,
                       long long cstride = 0) {
  const int nz = kchunk > 0 ? (K + kchunk - 1) / kchunk : 1;
  dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, nz);
  if (bl == B_NCONTIG)
    hipLaunchKernelGGL((k_gemm_f64<BM, BN, BK, B_NCONTIG>), grid, dim3(256), 0, s, A, lda, B, ldb,
                       C, om, M, N, K, maxbits, kchunk, cstride);
  else
    hipLaunchKernelGGL((k_gemm_f64<BM, BN, BK, B_KCONTIG>), grid, dim3(256), 0, s, A, lda, B, ldb,
                       C, om, M, N, K, maxbits, kchunk, cstride);
}

__global__ void k_sum_partials(const double* __restrict__ P, int parts, long long count,
                               long long stride, double* __restrict__ out,
                               const double* __restrict__ sub, double sigma) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < count;
       e += (long long)gridDim.x * blockDim.x) {
    double s = 0.0;
#pragma unroll 8
    for (int z = 0; z < parts; ++z) s += P[z * stride + e];
    if (sub) s -= sigma * sub[e];
    out[e] = s;
  }
}

void gemm_f64_splitk(const double* A, long long lda, const double* B, long long ldb, int blayout,
                     double* C, long long ldc, int M, int N, int K, int kchunk, double* partials,
                     hipStream_t s, const double* sub, double sigma) {
  if (M <= 0 || N <= 0) return;
  const int parts = (K + kchunk - 1) / kchunk;
  const long long cstride = (long long)M * N;
  launch_f64<64, 64, 16>(A, lda, B, ldb, blayout, partials, out_rowmajor(N), M, N, K, nullptr, s,
                         kchunk, cstride);
  long long count = (long long)M * N;
  int blocks = (int)((count + 255) / 256);
  hipLaunchKernelGGL(k_sum_partials, dim3(blocks < 4096 ? blocks : 4096), dim3(256), 0, s,
                     partials, parts, count, cstride, C, sub, sigma);
  (void)ldc;
}

template <int TAG>
static void launch_big(const double* A, long long lda, const double* B, long long ldb, int bl,
                       double* C, const OutMap& om, int M, int N, int K,
                       unsigned long long* maxbits, hipStream_t s) {
  dim3 grid((N + 127) / 128, (M + 127) / 128);
  if (bl == B_NCONTIG)
    hipLaunchKernelGGL((k_gemm_f64_big<B_NCONTIG, TAG>), grid, dim3(256), 0, s, A, lda, B, ldb, C,
                       om, M, N, K, maxbits);
  else
    hipLaunchKernelGGL((k_gemm_f64_big<B_KCONTIG, TAG>), grid, dim3(256), 0, s, A, lda, B, ldb, C,
                       om, M, N, K, maxbits);
}

// ------------------------------------------------------------- autotuner --
// Large products (M * N >= 2^20) pick their kernel by measurement: on the
// first call with a given shape, operand strides, layout, output map and tag,
// every applicable candidate runs three times on the caller's operands and
// stream, timed with HIP events (the faster of the last two counts: the
// first loads code and warms caches; single runs of the largest products
// spread by a few percent, as much as some candidates differ); the fastest
// is kept for the rest of the process and produces the output of that first
// call too.  Candidates differ only in
// tiling (same products, different summation order), so results agree to
// rounding.  HOTRG_AUTOTUNE=0 keeps the fixed rule below; HOTRG_GEMM_VARIANT
// forces one kernel.
namespace {

enum { C_LDS2 = 0, C_LDS3, C_LDS32, C_LDS_HALF, C_LDS_N64, C_BIG, C_G128, C_G64, C_COUNT };

struct TuneKey {
  long long v[16];
  bool operator<(const TuneKey& o) const {
    for (int i = 0; i < 16; ++i)
      if (v[i] != o.v[i]) return v[i] < o.v[i];
    return false;
  }
};

std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;

bool autotune_on() {
  static const bool on = [] {
    const char* e = std::getenv("HOTRG_AUTOTUNE");
    return !(e && e[0] == '0');
  }();
  return on;
}

TuneKey make_key(int prec, long long lda, long long ldb, int bl, const OutMap& om, int M, int N,
                 int K, bool mx, int tag) {
  TuneKey k{};
  const long long v[16] = {prec, lda, ldb, bl, M, N, K, mx, tag, om.r1, om.r2, om.s0,
                           om.c1, om.c2, om.t0, om.s1 * 1000003LL + om.s2 + om.t1 * 7919LL + om.t2};
  for (int i = 0; i < 16; ++i) k.v[i] = v[i];
  return k;
}

// time each applicable candidate (faster of runs two and three); -1 if none
// applies
// The lock is held through a measurement, so each shape is measured once
// per process and every call sees the same choice.
template <class Run>
int tune(const TuneKey& key, int count, Run&& run, hipStream_t s, bool* tuned) {
  *tuned = false;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(key);
  if (it != g_tune.end()) return it->second;
  *tuned = true;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return -1;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return -1;
  }
  int best = -1;
  float best_ms = 0.f;
  for (int c = 0; c < count; ++c) {
    if (!run(c)) continue;  // not applicable to this shape
    float ms = 0.f;
    bool ok = true;
    for (int rep = 0; rep < 2 && ok; ++rep) {
      (void)hipEventRecord(a, s);
      run(c);
      (void)hipEventRecord(b, s);
      float t = 0.f;
      ok = hipEventSynchronize(b) == hipSuccess && hipEventElapsedTime(&t, a, b) == hipSuccess;
      if (ok && (rep == 0 || t < ms)) ms = t;
    }
    if (!ok) continue;
    if (best < 0 || ms < best_ms) {
      best = c;
      best_ms = ms;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (best >= 0) g_tune[key] = best;
  return best;
}

}  // namespace

void gemm_f64(const double* A, long long lda, const double* B, long long ldb, int blayout,
              double* C, const OutMap& om, int M, int N, int K, unsigned long long* maxbits,
              hipStream_t s, int tag) {
  if (M <= 0 || N <= 0) return;
  const bool no_tune = (tag & GEMM_NO_TUNE) != 0;
  tag &= ~GEMM_NO_TUNE;
  static const int forced = [] {
    const char* e = std::getenv("HOTRG_GEMM_VARIANT");
    return e ? std::atoi(e) : -1;
  }();
  auto cand = [&](int c) -> bool {
    switch (c) {
      case C_LDS2:
        return N >= 128 && gemm_f64_lds(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s, tag, 1);
      case C_LDS3:
        return N >= 128 && K >= 64 &&
               gemm_f64_lds(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s, tag, 3);
      case C_LDS32:
        return N >= 128 && gemm_f64_lds(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s, tag, 0);
      case C_LDS_HALF:
        return N >= 128 && gemm_f64_lds(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s, tag, 4);
      case C_LDS_N64:
        return N <= 64 && gemm_f64_lds(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s, tag, 5);
      case C_BIG:
        if (N < 128 || K < 64) return false;
        switch (tag) {
          case GEMM_TAG_C2:
            launch_big<GEMM_TAG_C2>(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s);
            break;
          case GEMM_TAG_ENV:
            launch_big<GEMM_TAG_ENV>(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s);
            break;
          default:
            launch_big<GEMM_TAG_OTHER>(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s);
        }
        return true;
      case C_G128:
        if (N < 128) return false;
        launch_f64<128, 128, 16>(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s);
        return true;
      default:
        launch_f64<64, 64, 16>(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s);
        return true;
    }
  };
  if (!no_tune && forced < 0 && autotune_on() && (long long)M * N >= (1LL << 20)) {
    bool tuned = false;
    const int c = tune(make_key(0, lda, ldb, blayout, om, M, N, K, maxbits != nullptr, tag),
                       C_COUNT, cand, s, &tuned);
    // the candidates' runs all reached the output max: start it again
    if (tuned && maxbits) (void)hipMemsetAsync(maxbits, 0, 8, s);
    if (c >= 0 && cand(c)) return;
  }
  // fixed rule: 256 x 128 tiles, three LDS stages for long K (one barrier per
  // slab, two slabs in flight), two for short K
  const int variant = forced >= 0 ? forced : (K >= 256 ? 3 : 1);
  if ((long long)M * N >= (1LL << 20) && (N >= 128 || (variant == 5 && N <= 64)) &&
      variant != 2 && gemm_f64_lds(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s, tag, variant))
    return;
  if ((long long)M * N >= (1LL << 22) && N >= 128 && K >= 64) {
    cand(C_BIG);
  } else if ((long long)M * N >= (1LL << 22) && N >= 128) {
    launch_f64<128, 128, 16>(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s);
  } else {
    launch_f64<64, 64, 16>(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s);
  }
}

// the autotuner's table, for the reduced-precision launcher
int tune_choice(int prec, long long lda, long long ldb, int bl, const OutMap& om, int M, int N,
                int K, unsigned long long* maxbits, int tag, int count,
                bool (*run)(void*, int), void* ctx, hipStream_t s) {
  if (!autotune_on()) return -1;
  bool tuned = false;
  const int c = tune(make_key(prec, lda, ldb, bl, om, M, N, K, maxbits != nullptr, tag), count,
                     [&](int k) { return run(ctx, k); }, s, &tuned);
  if (tuned && maxbits) (void)hipMemsetAsync(maxbits, 0, 8, s);
  return c;
}

}  // namespace hotrg
