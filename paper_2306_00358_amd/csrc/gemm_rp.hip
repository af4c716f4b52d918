// Reduced-precision contractions of the HOTRG step: FP32 MFMA, or split
// BF16 with three products and FP32 accumulation.
//
//   C[map(m, n)] = sum_k A[m][k] * B[n][k]      (both operands K-contiguous)
//
// Operand formats (rows of ldk elements, ldk a multiple of 32, entries past
// the true K are zero):
//   RP_F32    one float array;
//   RP_BF16X3 two bf16 arrays hi, lo with x = hi + lo + O(2^-16 |x|):
//             hi = bf16(x), lo = bf16(x - hi), both round-to-nearest.
//             a*b is taken as lo_a*hi_b + hi_a*lo_b + hi_a*hi_b (the lo*lo
//             term, O(2^-16), is dropped), products exact, sums in FP32.
// Output: FP32, split BF16 (for a following BF16X3 contraction) or FP64
// (for the FP64 eigensolver).
//
// Tiling: 8 waves, 256 x 256 block tile, each wave 128 x 64 as 8 x 4 MFMA
// tiles (256 x 128 and 64 x 64 per wave when N < 256); K slabs of 32 elements streamed into LDS with
// global_load_lds_dwordx4 (16 bytes per lane), two LDS stages and one
// barrier per slab (a three-stage form software-pipelines the fragment reads
// across slabs).  The split-BF16 products of a slab start after five of its
// 24 fragment reads; the rest are placed among the MFMAs.  An LDS row
// is 128 bytes = 8 chunks of 16 bytes: for RP_F32 the 32 floats of the slab,
// for RP_BF16X3 four hi chunks then four lo chunks (8 bf16 each).  Chunk c
// of row r sits at chunk position c ^ ((r >> 1) & 7), so the 16 rows read by
// one 16-lane group fall into distinct LDS banks.
//
// MFMA lane layouts (gfx950): f32_16x16x4f32 and f32_16x16x32_bf16 both
// take A[i][k] from lane i + 16 g and return D[4 g + v][i] in value v of
// lane i + 16 g; the bf16 form takes 8 consecutive k per lane.  For FP32
// the 32 k of a slab are split by lane group: group g owns k in [8g, 8g+8),
// one k per MFMA; for BF16 group g owns the same 8 k in one MFMA.
#include <hip/hip_runtime.h>

#include <type_traits>

#include <cstdlib>

#include "internal.h"

namespace hotrg {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) void lds_void_rp;

__device__ __forceinline__ long long rmap_row(const OutMap& o, int m) {
  int m2 = m % o.r2;
  int q = m / o.r2;
  int m1 = q % o.r1;
  int m0 = q / o.r1;
  return (long long)m0 * o.s0 + (long long)m1 * o.s1 + (long long)m2 * o.s2;
}

__device__ __forceinline__ long long rmap_col(const OutMap& o, int n) {
  int n2 = n % o.c2;
  int q = n / o.c2;
  int n1 = q % o.c1;
  int n0 = q / o.c1;
  return (long long)n0 * o.t0 + (long long)n1 * o.t1 + (long long)n2 * o.t2;
}

__device__ __forceinline__ int rp_swz(int r) { return (r >> 1) & 7; }

// Stream rows [row0, row0 + R) x slab [k0, k0 + 32) of an operand into LDS.
// One wave instruction moves 8 rows (1 KB).
template <int R, int MODE>
__device__ __forceinline__ void rp_load(const void* __restrict__ hi, const void* __restrict__ lo,
                                        long long ldk, int row0, int rows_valid, int k0, char* lds,
                                        int wave, int lane) {
  constexpr int INSTS = R / 8;
  static_assert(INSTS % 8 == 0, "instructions must split over 8 waves");
#pragma unroll
  for (int q = 0; q < INSTS / 8; ++q) {
    const int inst = wave + q * 8;
    const int r = inst * 8 + lane / 8;
    const int c = lane % 8;
    const int g = c ^ rp_swz(r);  // chunk stored at position c
    int gr = row0 + r;
    gr = gr < rows_valid ? gr : rows_valid - 1;
    const char* src;
    if (MODE == RP_F32)
      src = (const char*)hi + ((long long)gr * ldk + k0 + 4 * g) * 4;
    else
      src = (const char*)(g < 4 ? hi : lo) + ((long long)gr * ldk + k0 + 8 * (g & 3)) * 2;
    __builtin_amdgcn_global_load_lds((const void*)src, (lds_void_rp*)(lds + inst * 1024), 16, 0, 0);
  }
}

// Block tile 256 x BN with 8 waves; each wave owns 16 TM rows x 64 columns
// (TM MFMA tiles of 16 rows): TM = 4 for BN = 128, TM = 8 for BN = 256.
// One output tile at rows m0.., columns n0.. (shared by the single-product
// kernel and the grouped one).
template <int MODE, int OUT, int TM, int BN, int NST, int PRIO = 0>
__device__ __forceinline__ void rp_tile(const void* __restrict__ Ahi, const void* __restrict__ Alo,
                                        long long lda, const void* __restrict__ Bhi,
                                        const void* __restrict__ Blo, long long ldb,
                                        void* __restrict__ C, void* __restrict__ Clo,
                                        const OutMap& om, int M, int N, int K,
                                        unsigned long long* maxbits, int m0, int n0) {
  constexpr int BM = 256, A_BYTES = BM * 128, B_BYTES = BN * 128;
  constexpr int STAGE = A_BYTES + B_BYTES;
  constexpr int WN = BN / 64;               // waves along N
  static_assert((BM / (16 * TM)) * WN == 8, "8 waves per block");
  constexpr int LOADS = BM / 64 + BN / 64;  // per wave per slab
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int li = lane & 15, lg = lane >> 4;

  f4 acc[TM][4];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  auto issue = [&](int k0, int stage) {
    char* base = smem + stage * STAGE;
    rp_load<BM, MODE>(Ahi, Alo, lda, m0, M, k0, base, wave, lane);
    rp_load<BN, MODE>(Bhi, Blo, ldb, n0, N, k0, base + A_BYTES, wave, lane);
  };
  // the two 16-byte chunks a lane group reads from a row
  const int c0 = MODE == RP_F32 ? 2 * lg : lg;
  const int c1 = MODE == RP_F32 ? 2 * lg + 1 : 4 + lg;

  static_assert(NST == 2 || NST == 3, "two or three LDS stages");
  const int nslab = K / 32;
  issue(0, 0);
  if (NST == 3 && nslab > 1) issue(32, 1);
  // a slab's fragments: rows of A (hi/lo or the two f32 halves), columns of B
  struct Frag {
    f4 a0[TM], a1[TM], b0[4], b1[4];
  };
  auto read_frag = [&](int stage, Frag& f) {
    const char* as = smem + stage * STAGE;
    const char* bs = as + A_BYTES;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int r = wm * 16 * TM + i * 16 + li;
      f.a0[i] = *(const f4*)(as + r * 128 + ((c0 ^ rp_swz(r)) << 4));
      f.a1[i] = *(const f4*)(as + r * 128 + ((c1 ^ rp_swz(r)) << 4));
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = wn * 64 + j * 16 + li;
      f.b0[j] = *(const f4*)(bs + r * 128 + ((c0 ^ rp_swz(r)) << 4));
      f.b1[j] = *(const f4*)(bs + r * 128 + ((c1 ^ rp_swz(r)) << 4));
    }
  };
  // the MFMAs of row tile i of a slab
  auto mfma_row = [&](int i, const Frag& f) {
    if (MODE == RP_F32) {
#pragma unroll
      for (int t = 0; t < 8; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float av = t < 4 ? f.a0[i][t] : f.a1[i][t - 4];
          const float bv = t < 4 ? f.b0[j][t] : f.b1[j][t - 4];
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[i][j], 0, 0, 0);
        }
    } else {
      const bf8 ah = __builtin_bit_cast(bf8, f.a0[i]);
      const bf8 al = __builtin_bit_cast(bf8, f.a1[i]);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bf8 bh = __builtin_bit_cast(bf8, f.b0[j]);
        const bf8 bl = __builtin_bit_cast(bf8, f.b1[j]);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[i][j], 0, 0, 0);
      }
    }
  };
  if constexpr (NST == 3) {
    // Software-pipelined across slabs (one barrier per slab): the barrier
    // into slab s+1 and the reads of its fragments come before the MFMAs of
    // the second half of slab s's row tiles.  PRE: copies of slab s+2 go
    // out during slab s; CROSS: slab s+1 follows (compile-time flags, so the
    // main loop body has no branches).
    if (nslab > 1)
      asm volatile("s_waitcnt vmcnt(%0)" ::"n"(LOADS) : "memory");
    else
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    Frag cur;
    read_frag(0, cur);
    auto slab = [&](int s, auto pre_c, auto cross_c) {
      constexpr bool PRE = decltype(pre_c)::value;
      constexpr bool CROSS = decltype(cross_c)::value;
      // slab s+2 goes to the stage slab s-1 held, free since the barrier
      // that opened slab s
      if constexpr (PRE) issue((s + 2) * 32, (s + 2) % 3);
      Frag nxt;
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        if constexpr (CROSS) {
          if (i == TM / 2) {
            // this wave's copies of slab s+1 have landed (those of s+2 may
            // be pending) and its reads of slab s have returned; after the
            // barrier every wave's have
            if constexpr (PRE)
              asm volatile("s_waitcnt vmcnt(%0)" ::"n"(LOADS) : "memory");
            else
              asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
            read_frag((s + 1) % 3, nxt);
          }
        }
        mfma_row(i, cur);
      }
      if constexpr (CROSS) cur = nxt;
    };
    using yes = std::integral_constant<bool, true>;
    using no = std::integral_constant<bool, false>;
    int s = 0;
    for (; s + 2 < nslab; ++s) slab(s, yes{}, yes{});
    if (s + 1 < nslab) slab(s++, no{}, yes{});
    if (s < nslab) slab(s, no{}, no{});
  } else
  for (int s = 0; s < nslab; ++s) {
    // two stages: slab s has landed for every wave, and every wave has read
    // slab s-1 (its reads were waited for at the end of that slab), whose
    // stage then takes slab s+1.  One barrier per slab.
    const int cur = s & 1;
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    if (s + 1 < nslab) issue((s + 1) * 32, cur ^ 1);
    const char* as = smem + cur * STAGE;
    const char* bs = as + A_BYTES;
    if constexpr (MODE == RP_BF16X3) {
      // fragments read as they are needed: the lo half of row tile 0 and the
      // hi half of B first (the first four products use only those), the
      // other five during those products, row tile i+1 of A during the
      // products of row tile i; the order of the products into each
      // accumulator (lo*hi, hi*lo, hi*hi, slab by slab) is unchanged
      f4 fh[TM], fl[TM], gh[4], gl[4];
      auto rd = [&](const char* base, int r, int c) {
        return *(const f4*)(base + r * 128 + ((c ^ rp_swz(r)) << 4));
      };
      const int ra = wm * 16 * TM + li, rb = wn * 64 + li;
      fl[0] = rd(as, ra, c1);
#pragma unroll
      for (int j = 0; j < 4; ++j) gh[j] = rd(bs, rb + 16 * j, c0);
      fh[0] = rd(as, ra, c0);
#pragma unroll
      for (int j = 0; j < 4; ++j) gl[j] = rd(bs, rb + 16 * j, c1);
      __builtin_amdgcn_sched_group_barrier(0x100, 5, 0);  // 5 LDS reads
      // PRIO: the wave in its MFMA sequence takes issue priority over the
      // other wave of its SIMD
      if constexpr (PRIO) __builtin_amdgcn_s_setprio(1);
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        if (i + 1 < TM) {
          fh[i + 1] = rd(as, ra + 16 * (i + 1), c0);
          fl[i + 1] = rd(as, ra + 16 * (i + 1), c1);
        }
        const bf8 ah = __builtin_bit_cast(bf8, fh[i]);
        const bf8 al = __builtin_bit_cast(bf8, fl[i]);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, __builtin_bit_cast(bf8, gh[j]),
                                                              acc[i][j], 0, 0, 0);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, __builtin_bit_cast(bf8, gl[j]),
                                                              acc[i][j], 0, 0, 0);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, __builtin_bit_cast(bf8, gh[j]),
                                                              acc[i][j], 0, 0, 0);
        // placement (0x008 = MFMA, 0x100 = LDS read)
        if (i == 0) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, 5, 0);
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
        } else {
          __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
        }
      }
      if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
    } else {
    f4 a0[TM], a1[TM], b0[4], b1[4];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int r = wm * 16 * TM + i * 16 + li;
      a0[i] = *(const f4*)(as + r * 128 + ((c0 ^ rp_swz(r)) << 4));
      a1[i] = *(const f4*)(as + r * 128 + ((c1 ^ rp_swz(r)) << 4));
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = wn * 64 + j * 16 + li;
      b0[j] = *(const f4*)(bs + r * 128 + ((c0 ^ rp_swz(r)) << 4));
      b1[j] = *(const f4*)(bs + r * 128 + ((c1 ^ rp_swz(r)) << 4));
    }
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float av = t < 4 ? a0[i][t] : a1[i][t - 4];
          const float bv = t < 4 ? b0[j][t] : b1[j][t - 4];
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[i][j], 0, 0, 0);
        }
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  }

  float mx = 0.f;
  long long coff[4];
  bool cok[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int n = n0 + wn * 64 + j * 16 + li;
    cok[j] = n < N;
    coff[j] = cok[j] ? rmap_col(om, n) : 0;
  }
#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int m = m0 + wm * 16 * TM + i * 16 + 4 * lg + v;
      if (m >= M) continue;
      const long long roff = rmap_row(om, m);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (!cok[j]) continue;
        const float x = acc[i][j][v];
        const long long o = roff + coff[j];
        if (OUT == RP_OUT_F32) {
          ((float*)C)[o] = x;
        } else if (OUT == RP_OUT_F64) {
          ((double*)C)[o] = (double)x;
        } else {
          const __bf16 h = (__bf16)x;
          ((__bf16*)C)[o] = h;
          ((__bf16*)Clo)[o] = (__bf16)(x - (float)h);
        }
        mx = fmaxf(mx, fabsf(x));
      }
    }
  }
  if (maxbits) {
    double m = mx;
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if (lane == 0) atomicMax(maxbits, (unsigned long long)__double_as_longlong(m));
  }
}

template <int MODE, int OUT, int TAG, int TM, int BN, int NST, int PRIO = 0>
__global__ __launch_bounds__(512) void k_gemm_rp(const void* __restrict__ Ahi,
                                                 const void* __restrict__ Alo, long long lda,
                                                 const void* __restrict__ Bhi,
                                                 const void* __restrict__ Blo, long long ldb,
                                                 void* __restrict__ C, void* __restrict__ Clo,
                                                 OutMap om, int M, int N, int K,
                                                 unsigned long long* maxbits, int gm) {
  int im, in;
  tile_order((M + 255) / 256, (N + BN - 1) / BN, blockIdx.x, gm, im, in);
  rp_tile<MODE, OUT, TM, BN, NST, PRIO>(Ahi, Alo, lda, Bhi, Blo, ldb, C, Clo, om, M, N, K,
                                        maxbits, im * 256, in * BN);
}

// Grouped form: one launch over the output tiles of every product in the
// table (problems of a batch with uneven shapes); workgroup b takes tile
// b - tile_begin of the item whose range holds b.  Items with a gate that
// reads 0 (a finished problem) skip their tiles.
__device__ __forceinline__ int find_item(const int* __restrict__ begin, int count, int b) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {  // last item with begin <= b
    const int mid = (lo + hi + 1) >> 1;
    if (begin[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int MODE, int OUT, int TM, int BN, int NST>
__global__ __launch_bounds__(512) void k_gemm_rp_grouped(const RpItem* __restrict__ items,
                                                         const int* __restrict__ begin,
                                                         int count) {
  const int g = find_item(begin, count, blockIdx.x);
  const RpItem& it = items[g];
  if (it.gate && *it.gate == 0) return;
  const int local = blockIdx.x - begin[g];
  const int tm = (it.M + 255) / 256, tn = (it.N + BN - 1) / BN;
  if (local >= tm * tn) return;  // padding of the item's range to a multiple of 8
  int im, in;
  tile_order(tm, tn, local, 4, im, in);
  rp_tile<MODE, OUT, TM, BN, NST>(it.A.hi, it.A.lo, it.lda, it.B.hi, it.B.lo, it.ldb, it.C,
                                  it.Clo, it.om, it.M, it.N, it.K, it.maxbits, im * 256, in * BN);
}

// tile configuration: 0 = 256 x 256 blocks, two stages (N >= 256);
// 1 = 256 x 128 blocks, two stages; 2 = 256 x 128 blocks, three stages
static int rp_config(int N) {
  static const int forced = [] {
    const char* e = getenv("HOTRG_RP_CFG");
    return e ? atoi(e) : -1;
  }();
  if (forced == 0 && N >= 256) return 0;
  if (forced == 1 || forced == 2) return forced;
  return N >= 256 ? 0 : 1;
}

template <int MODE, int OUT, int TM, int BN, int NST>
static void launch_rp_shape(int tag, const RpOperand& A, long long lda, const RpOperand& B,
                            long long ldb, void* C, void* Clo, const OutMap& om, int M, int N,
                            int K, unsigned long long* maxbits, hipStream_t s) {
  constexpr int LDS = NST * (256 + BN) * 128;
  dim3 grid(((N + BN - 1) / BN) * ((M + 255) / 256));
  // XCD-grouped tile order, 4 row panels at a time (half the L2 misses of
  // row-major order on the D^7 contraction, 1.5% faster)
  const int gm = 4;
  auto go = [&](auto kern) {
    static const bool ok = hipFuncSetAttribute((const void*)kern,
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               LDS) == hipSuccess;
    (void)ok;
    hipLaunchKernelGGL(kern, grid, dim3(512), LDS, s, A.hi, A.lo, lda, B.hi, B.lo, ldb, C, Clo,
                       om, M, N, K, maxbits, gm);
  };
  if constexpr (MODE == RP_BF16X3 && NST == 2) {
    // the split-BF16 two-stage tile of C2 raises its wave priority over its
    // MFMA sequence (s_setprio): 0.5% faster at D = 64 in alternating runs on
    // one chip, the same results; HOTRG_RP_PRIO=0 turns it off
    static const bool prio = [] {
      const char* e = getenv("HOTRG_RP_PRIO");
      return !(e && atoi(e) == 0);
    }();
    if (prio && tag == GEMM_TAG_C2) {
      go(k_gemm_rp<MODE, OUT, GEMM_TAG_C2, TM, BN, NST, 1>);
      return;
    }
  }
  if (tag == GEMM_TAG_C2)
    go(k_gemm_rp<MODE, OUT, GEMM_TAG_C2, TM, BN, NST>);
  else if (tag == GEMM_TAG_ENV)
    go(k_gemm_rp<MODE, OUT, GEMM_TAG_ENV, TM, BN, NST>);
  else
    go(k_gemm_rp<MODE, OUT, GEMM_TAG_OTHER, TM, BN, NST>);
}

template <int MODE, int OUT>
static void launch_rp_cfg(int cfg, int tag, const RpOperand& A, long long lda,
                          const RpOperand& B, long long ldb, void* C, void* Clo,
                          const OutMap& om, int M, int N, int K, unsigned long long* maxbits,
                          hipStream_t s) {
  if (cfg == 0)
    launch_rp_shape<MODE, OUT, 8, 256, 2>(tag, A, lda, B, ldb, C, Clo, om, M, N, K, maxbits, s);
  else if (cfg == 2)
    launch_rp_shape<MODE, OUT, 4, 128, 3>(tag, A, lda, B, ldb, C, Clo, om, M, N, K, maxbits, s);
  else
    launch_rp_shape<MODE, OUT, 4, 128, 2>(tag, A, lda, B, ldb, C, Clo, om, M, N, K, maxbits, s);
}

template <int MODE, int OUT>
static void launch_rp_tag(int tag, const RpOperand& A, long long lda, const RpOperand& B,
                          long long ldb, void* C, void* Clo, const OutMap& om, int M, int N,
                          int K, unsigned long long* maxbits, hipStream_t s) {
  static const bool forced = getenv("HOTRG_RP_CFG") != nullptr;
  if (!forced && (long long)M * N >= (1LL << 20)) {
    struct Args {
      int tag;
      const RpOperand *A, *B;
      long long lda, ldb;
      void *C, *Clo;
      const OutMap* om;
      int M, N, K;
      unsigned long long* maxbits;
      hipStream_t s;
    } args{tag, &A, &B, lda, ldb, C, Clo, &om, M, N, K, maxbits, s};
    auto run = [](void* p, int cfg) -> bool {
      const Args& a = *(const Args*)p;
      if (cfg == 0 && a.N < 256) return false;
      launch_rp_cfg<MODE, OUT>(cfg, a.tag, *a.A, a.lda, *a.B, a.ldb, a.C, a.Clo, *a.om, a.M,
                               a.N, a.K, a.maxbits, a.s);
      return true;
    };
    const int cfg = tune_choice(10 * MODE + OUT + 1, lda, ldb, 0, om, M, N, K, maxbits, tag, 3,
                                run, &args, s);
    if (cfg >= 0) {
      run(&args, cfg);
      return;
    }
  }
  launch_rp_cfg<MODE, OUT>(rp_config(N), tag, A, lda, B, ldb, C, Clo, om, M, N, K, maxbits, s);
}

// ---- grouped launch ----
int rp_group_tiles(const RpItem& it, int cfg) {
  // rounded up to a multiple of 8, so that every item's range starts on a
  // multiple of 8 and the XCD-grouped tile order sees blockIdx % 8 as the XCD
  // (the workgroups past the item's tiles return at once)
  const int bn = cfg == 0 ? 256 : 128;
  return (((it.M + 255) / 256) * ((it.N + bn - 1) / bn) + 7) / 8 * 8;
}

template <int MODE, int OUT, int TM, int BN, int NST>
static void launch_rp_grouped_shape(const RpItem* d_items, const int* d_begin, int count,
                                    int tiles, hipStream_t s) {
  constexpr int LDS = NST * (256 + BN) * 128;
  auto kern = k_gemm_rp_grouped<MODE, OUT, TM, BN, NST>;
  static const bool ok = hipFuncSetAttribute((const void*)kern,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             LDS) == hipSuccess;
  (void)ok;
  hipLaunchKernelGGL(kern, dim3(tiles), dim3(512), LDS, s, d_items, d_begin, count);
}

template <int MODE, int OUT>
static void launch_rp_grouped_cfg(int cfg, const RpItem* d_items, const int* d_begin, int count,
                                  int tiles, hipStream_t s) {
  if (cfg == 0)
    launch_rp_grouped_shape<MODE, OUT, 8, 256, 2>(d_items, d_begin, count, tiles, s);
  else if (cfg == 2)
    launch_rp_grouped_shape<MODE, OUT, 4, 128, 3>(d_items, d_begin, count, tiles, s);
  else
    launch_rp_grouped_shape<MODE, OUT, 4, 128, 2>(d_items, d_begin, count, tiles, s);
}

void gemm_rp_grouped(int mode, int out, int cfg, const RpItem* d_items, const int* d_begin,
                     int count, int tiles, hipStream_t s) {
  if (count <= 0 || tiles <= 0) return;
  if (mode == RP_F32) {
    if (out == RP_OUT_F32)
      launch_rp_grouped_cfg<RP_F32, RP_OUT_F32>(cfg, d_items, d_begin, count, tiles, s);
    else
      launch_rp_grouped_cfg<RP_F32, RP_OUT_F64>(cfg, d_items, d_begin, count, tiles, s);
  } else {
    if (out == RP_OUT_SPLIT)
      launch_rp_grouped_cfg<RP_BF16X3, RP_OUT_SPLIT>(cfg, d_items, d_begin, count, tiles, s);
    else if (out == RP_OUT_F64)
      launch_rp_grouped_cfg<RP_BF16X3, RP_OUT_F64>(cfg, d_items, d_begin, count, tiles, s);
    else
      launch_rp_grouped_cfg<RP_BF16X3, RP_OUT_F32>(cfg, d_items, d_begin, count, tiles, s);
  }
}

bool gemm_rp(int mode, const RpOperand& A, long long lda, const RpOperand& B, long long ldb,
             int out, void* C, void* Clo, const OutMap& om, int M, int N, int K,
             unsigned long long* maxbits, hipStream_t s, int tag) {
  if (M < 1 || N < 1 || K < 32 || K % 32 != 0) return false;
  if ((lda % 8) || (ldb % 8)) return false;
  const void* ptrs[4] = {A.hi, A.lo, B.hi, B.lo};
  for (int i = 0; i < 4; ++i)
    if (((uintptr_t)ptrs[i] & 15) || (mode == RP_BF16X3 && !ptrs[i] && i % 2 == 1)) return false;
  if (mode == RP_F32) {
    if (out == RP_OUT_F32)
      launch_rp_tag<RP_F32, RP_OUT_F32>(tag, A, lda, B, ldb, C, Clo, om, M, N, K, maxbits, s);
    else if (out == RP_OUT_F64)
      launch_rp_tag<RP_F32, RP_OUT_F64>(tag, A, lda, B, ldb, C, Clo, om, M, N, K, maxbits, s);
    else
      return false;
  } else {
    if (out == RP_OUT_SPLIT)
      launch_rp_tag<RP_BF16X3, RP_OUT_SPLIT>(tag, A, lda, B, ldb, C, Clo, om, M, N, K, maxbits, s);
    else if (out == RP_OUT_F64)
      launch_rp_tag<RP_BF16X3, RP_OUT_F64>(tag, A, lda, B, ldb, C, Clo, om, M, N, K, maxbits, s);
    else if (out == RP_OUT_F32)
      launch_rp_tag<RP_BF16X3, RP_OUT_F32>(tag, A, lda, B, ldb, C, Clo, om, M, N, K, maxbits, s);
    else
      return false;
  }
  return true;
}

}  // namespace hotrg
