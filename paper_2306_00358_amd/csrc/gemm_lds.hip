// FP64 MFMA GEMM with operands streamed straight from global memory into LDS
// (global_load_lds_dwordx4, 16 bytes per lane), for the large contractions of
// the HOTRG step: the O(D^7) contraction and the environment products.
//
//   C[map(m, n)] = sum_k A[m*lda + k] * B(k, n)
//   B(k, n) = B[k*ldb + n] (B_NCONTIG) or B[n*ldb + k] (B_KCONTIG)
//
// Block: WGM x WGN waves, each owning a 64 x 64 output tile of 4 x 4
// v_mfma_f64_16x16x4f64 tiles (accumulators stay in registers for the whole
// K loop).  K advances in slabs of BK through NST LDS stages.  Two stages:
// the slab s+1 copy is in flight while slab s is multiplied, with a barrier
// after the copy lands and one before the stage is refilled.  Three stages:
// slabs s+1 and s+2 are in flight; one barrier per slab both publishes slab
// s and frees the stage of slab s-1 for the copy of slab s+2.  With an
// N-contiguous B the three-stage loop is also software-pipelined across
// slabs (copies issued from inside the MFMA sequence, the barrier into the
// next slab and its first fragment reads among this slab's MFMAs).
//
// Symmetric mode (sym, for Gram matrices C = A A^T): a 1-D grid over the
// tiles that reach the upper triangle; each element m <= n is stored at
// (m, n) and, for m < n, at (n, m) -- the same products summed in the same
// order as the full product's element (n, m), for about half the MFMAs.
//
// LDS layout.  Operand rows that are K-contiguous in global memory (A, and B
// when K-contiguous) are stored as rows of BK doubles cut into 16-byte
// chunks; chunk c of row r is stored at chunk position c ^ swz(r), which
// puts the 16 rows read by one 16-lane group of an MFMA fragment into 16
// different bank groups.  N-contiguous B is stored as plain rows of BN.
//
// K order inside a slab.  Lane group g = lane/16 of the MFMA takes the
// contiguous quarter k in [g*BK/4, (g+1)*BK/4) of the slab, one k per MFMA;
// this lets each lane read its A values with 16-byte LDS loads.  The sum
// over k is unchanged, only its rounding order differs.
//
// Requirements (checked by the launcher): K % BK == 0; lda, ldb even; N even
// for B_NCONTIG; 16-byte aligned base pointers.  Rows m >= M and columns
// n >= N are loaded from clamped (valid) addresses and never stored.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.h"

namespace hotrg {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) void lds_void;

__device__ __forceinline__ long long lmap_row(const OutMap& o, int m) {
  int m2 = m % o.r2;
  int q = m / o.r2;
  int m1 = q % o.r1;
  int m0 = q / o.r1;
  return (long long)m0 * o.s0 + (long long)m1 * o.s1 + (long long)m2 * o.s2;
}

__device__ __forceinline__ long long lmap_col(const OutMap& o, int n) {
  int n2 = n % o.c2;
  int q = n / o.c2;
  int n1 = q % o.c1;
  int n0 = q / o.c1;
  return (long long)n0 * o.t0 + (long long)n1 * o.t1 + (long long)n2 * o.t2;
}

template <int BK>
__device__ __forceinline__ int swz(int r) {
  // rows per 256-byte LDS line: BK=32 -> 1, BK=16 -> 2
  constexpr int L = 256 / (BK * 8);
  constexpr int CH = BK / 2;
  return (r / L) % CH;
}

// Copy rows [0, R) x K-slab of a K-contiguous operand into swizzled LDS.
// One wave instruction moves 1 KB = 1024 / (BK*8) rows.
template <int R, int BK, int NW>
__device__ __forceinline__ void load_kcontig(const double* __restrict__ G, long long ld, int row0,
                                             int rows_valid, int k0, char* lds, int wave,
                                             int lane) {
  constexpr int RPI = 1024 / (BK * 8);
  constexpr int CH = BK / 2;
  constexpr int INSTS = R / RPI;
  static_assert(INSTS % NW == 0, "instructions must split over waves");
#pragma unroll
  for (int q = 0; q < INSTS / NW; ++q) {
    const int inst = wave + q * NW;
    const int r = inst * RPI + lane / CH;
    const int c = lane % CH;
    int gr = row0 + r;
    gr = gr < rows_valid ? gr : rows_valid - 1;
    const double* src = G + (long long)gr * ld + k0 + 2 * (c ^ swz<BK>(r));
    __builtin_amdgcn_global_load_lds((const void*)src, (lds_void*)(lds + inst * 1024), 16, 0, 0);
  }
}

// Copy a BK x BN slab of an N-contiguous operand (BN = 128: one row per instruction).
template <int BK, int BN, int NW>
__device__ __forceinline__ void load_ncontig(const double* __restrict__ G, long long ld, int k0,
                                             int col0, int cols_valid, char* lds, int wave,
                                             int lane) {
  static_assert(BN * 8 == 1024, "one 1 KB row per instruction");
  static_assert(BK % NW == 0, "rows must split over waves");
#pragma unroll
  for (int q = 0; q < BK / NW; ++q) {
    const int r = wave + q * NW;
    int gc = col0 + 2 * lane;
    gc = gc < cols_valid ? gc : cols_valid - 2;
    const double* src = G + (long long)(k0 + r) * ld + gc;
    __builtin_amdgcn_global_load_lds((const void*)src, (lds_void*)(lds + r * 1024), 16, 0, 0);
  }
}

// Copy a BK x 64 slab of an N-contiguous operand: a 64-wide row is 512
// bytes, so one wave instruction moves two rows (lanes 0-31 and 32-63).
template <int BK, int NW>
__device__ __forceinline__ void load_ncontig64(const double* __restrict__ G, long long ld, int k0,
                                               int col0, int cols_valid, char* lds, int wave,
                                               int lane) {
  static_assert((BK / 2) % NW == 0, "row pairs must split over waves");
#pragma unroll
  for (int q = 0; q < BK / 2 / NW; ++q) {
    const int pr = wave + q * NW;
    const int r = 2 * pr + (lane >> 5);
    int gc = col0 + 2 * (lane & 31);
    gc = gc < cols_valid ? gc : cols_valid - 2;
    const double* src = G + (long long)(k0 + r) * ld + gc;
    __builtin_amdgcn_global_load_lds((const void*)src, (lds_void*)(lds + pr * 1024), 16, 0, 0);
  }
}

template <int WGM, int WGN, int BK, int BL, int TAG, int NST>
__global__ __launch_bounds__(64 * WGM * WGN) void k_gemm_f64_lds(
    const double* __restrict__ A, long long lda, const double* __restrict__ B, long long ldb,
    double* __restrict__ C, OutMap om, int M, int N, int K, unsigned long long* maxbits,
    int sym, const double* __restrict__ A_2, double* __restrict__ C_2) {
  constexpr int NW = WGM * WGN;
  constexpr int BM = 64 * WGM, BN = 64 * WGN;
  constexpr int CH = BK / 2;
  constexpr int A_BYTES = BM * BK * 8, B_BYTES = BK * BN * 8;
  constexpr int STAGE = A_BYTES + B_BYTES;
  constexpr int KQ = BK / 4;  // k values per lane group per slab
  constexpr int A_INST = BM / (1024 / (BK * 8)) / NW;
  constexpr int B_INST = BL == B_NCONTIG ? (BN == 64 ? BK / 2 / NW : BK / NW)
                                          : BN / (1024 / (BK * 8)) / NW;
  constexpr int LOADS = A_INST + B_INST;  // global_load_lds per wave per slab
  static_assert(LOADS <= 63, "vmcnt range");
  static_assert(NST == 2 || NST == 3, "two or three LDS stages");
  __shared__ __attribute__((aligned(16))) char smem[NST * STAGE];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  // sym (C = A A^T, M = N, B = A): the 1-D grid enumerates, row tile by row
  // tile, the tiles that reach the upper triangle (n >= m somewhere); row
  // tile bm starts at column tile bm*BM/BN, and every row tile has at least
  // one, so the walk ends inside the grid the host computed the same way
  // With sym == 2 the grid holds two such products of the same shape, the
  // second on A_2 into C_2, one after the other.
  int bm = blockIdx.y, bn = blockIdx.x;
  if (sym) {
    const int nbn = (N + BN - 1) / BN;
    int rem = blockIdx.x;
    if (sym == 2) {
      int tiles = 0;
      for (int r = 0; r * BM < M; ++r) tiles += nbn - r * BM / BN;
      if (rem >= tiles) {
        rem -= tiles;
        A = A_2;
        B = A_2;
        C = C_2;
      }
    }
    bm = 0;
    while (rem >= nbn - bm * BM / BN) {
      rem -= nbn - bm * BM / BN;
      ++bm;
    }
    bn = bm * BM / BN + rem;
  }
  const int m0 = bm * BM, n0 = bn * BN;
  const int li = lane & 15, lg = lane >> 4;

  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  auto issue_a = [&](int k0, int stage) {
    load_kcontig<BM, BK, NW>(A, lda, m0, M, k0, smem + stage * STAGE, wave, lane);
  };
  auto issue_b = [&](int k0, int stage) {
    char* base = smem + stage * STAGE;
    if constexpr (BL == B_NCONTIG && BN == 64)
      load_ncontig64<BK, NW>(B, ldb, k0, n0, N, base + A_BYTES, wave, lane);
    else if constexpr (BL == B_NCONTIG)
      load_ncontig<BK, BN, NW>(B, ldb, k0, n0, N, base + A_BYTES, wave, lane);
    else
      load_kcontig<BN, BK, NW>(B, ldb, n0, N, k0, base + A_BYTES, wave, lane);
  };
  auto issue = [&](int k0, int stage) {
    issue_a(k0, stage);
    issue_b(k0, stage);
  };

  const int nslab = K / BK;
  issue(0, 0);
  if (NST == 3 && nslab > 1) issue(BK, 1);
  if constexpr (NST == 3 && BL == B_NCONTIG) {
    // Software-pipelined across slabs: the barrier into slab s+1 and the
    // reads of its first fragments come before the MFMAs of slab s's last k
    // step, so both waves of a SIMD still have MFMAs to issue while the
    // barrier and the LDS reads complete.
    auto read_a = [&](int stage, double (&a)[4][KQ]) {
      const char* as = smem + stage * STAGE;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = wm * 64 + i * 16 + li;
#pragma unroll
        for (int u = 0; u < KQ / 2; ++u) {
          const int c = lg * (KQ / 2) + u;
          const d2 v = *(const d2*)(as + (r * CH + (c ^ swz<BK>(r))) * 16);
          a[i][2 * u] = v.x;
          a[i][2 * u + 1] = v.y;
        }
      }
    };
    auto read_b = [&](int stage, int t, double (&b)[4]) {
      const char* bs = smem + stage * STAGE + A_BYTES;
      const int k = lg * KQ + t;
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = *(const double*)(bs + (k * BN + wn * 64 + j * 16 + li) * 8);
    };
    // slab 0: this wave's copies (slab 1's may be pending), then everyone's
    if (nslab > 1)
      asm volatile("s_waitcnt vmcnt(%0)" ::"n"(LOADS) : "memory");
    else
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    double a[4][KQ], b[4];
    read_a(0, a);
    read_b(0, 0, b);
    // one slab; PRE: copies of slab s+2 go out during it, CROSS: slab s+1
    // follows (compile-time flags, so the main loop body has no branches
    // and the compiler can interleave the LDS reads with the MFMAs)
    auto slab = [&](int s, auto pre_c, auto cross_c) {
      constexpr bool PRE = decltype(pre_c)::value;
      constexpr bool CROSS = decltype(cross_c)::value;
      const int cur = s % 3;
      double an[4][KQ];
#pragma unroll
      for (int t = 0; t < KQ; ++t) {
        double bn[4];
        if (t + 1 < KQ) {
          read_b(cur, t + 1, bn);
        } else if constexpr (CROSS) {
          // this wave's copies of slab s+1 have landed (those of s+2 may be
          // pending) and its reads of slab s have returned; after the
          // barrier every wave's have, so slab s+1 may be read and, during
          // it, the stage of slab s refilled
          if constexpr (PRE)
            asm volatile("s_waitcnt vmcnt(%0)" ::"n"(LOADS) : "memory");
          else
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
          // lgkmcnt(0) as the builtin (vmcnt and expcnt left at their
          // maximum), which the compiler's own wait insertion accounts for
          __builtin_amdgcn_s_waitcnt(0xC07F);
          __builtin_amdgcn_s_barrier();
          asm volatile("" ::: "memory");
          read_a((s + 1) % 3, an);
          read_b((s + 1) % 3, 0, bn);
        }
        // slab s+2 goes to the stage slab s-1 held, free since the barrier
        // that opened slab s
        if constexpr (PRE) {
          if (t == 0) issue_a((s + 2) * BK, (s + 2) % 3);
          if (t == 1) issue_b((s + 2) * BK, (s + 2) % 3);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i][t], b[j], acc[i][j], 0, 0, 0);
        if (t + 1 < KQ || CROSS) {
#pragma unroll
          for (int j = 0; j < 4; ++j) b[j] = bn[j];
        }
      }
      if constexpr (CROSS) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int u = 0; u < KQ; ++u) a[i][u] = an[i][u];
      }
    };
    using yes = std::integral_constant<bool, true>;
    using no = std::integral_constant<bool, false>;
    int s = 0;
    for (; s + 2 < nslab; ++s) slab(s, yes{}, yes{});
    if (s + 1 < nslab) slab(s++, no{}, yes{});
    if (s < nslab) slab(s, no{}, no{});
  } else
  for (int s = 0; s < nslab; ++s) {
    const int cur = NST == 2 ? (s & 1) : s % 3;
    if (NST == 2) {
      if (s + 1 < nslab) {
        issue((s + 1) * BK, cur ^ 1);
        // this wave's copies of slab s are done; those of slab s+1 may be pending
        asm volatile("s_waitcnt vmcnt(%0)" ::"n"(LOADS) : "memory");
      } else {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      }
    } else {
      // slabs s and s+1 are in flight: wait for s only
      if (s + 1 < nslab)
        asm volatile("s_waitcnt vmcnt(%0)" ::"n"(LOADS) : "memory");
      else
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
    // every wave's copies of slab s have landed (a plain barrier: a fenced
    // one would also wait for the copies still in flight); with three stages
    // every wave has also finished reading slab s-1, whose stage takes s+2
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");  // no LDS access moves above the barrier
    // with three stages the copies of slab s+2 go out from inside the MFMA
    // sequence below (A after the first k step's reads, B after the
    // second's), so that both waves of a SIMD have MFMAs to issue meanwhile
    const bool pre = NST == 3 && s + 2 < nslab;
    const char* as = smem + cur * STAGE;
    const char* bs = as + A_BYTES;
    // A values of this lane for the slab: rows wm*64 + i*16 + li, k in [lg*KQ, lg*KQ + KQ)
    double a[4][KQ];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = wm * 64 + i * 16 + li;
#pragma unroll
      for (int u = 0; u < KQ / 2; ++u) {
        const int c = lg * (KQ / 2) + u;
        const d2 v = *(const d2*)(as + (r * CH + (c ^ swz<BK>(r))) * 16);
        a[i][2 * u] = v.x;
        a[i][2 * u + 1] = v.y;
      }
    }
    if (BL == B_NCONTIG) {
#pragma unroll
      for (int t = 0; t < KQ; ++t) {
        const int k = lg * KQ + t;
        double b[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = *(const double*)(bs + (k * BN + wn * 64 + j * 16 + li) * 8);
        if (pre && t == 0) issue_a((s + 2) * BK, (s + 2) % 3);
        if (pre && t == 1) issue_b((s + 2) * BK, (s + 2) % 3);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i][t], b[j], acc[i][j], 0, 0, 0);
      }
    } else {
      double b[4][KQ];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = wn * 64 + j * 16 + li;
#pragma unroll
        for (int u = 0; u < KQ / 2; ++u) {
          const int c = lg * (KQ / 2) + u;
          const d2 v = *(const d2*)(bs + (r * CH + (c ^ swz<BK>(r))) * 16);
          b[j][2 * u] = v.x;
          b[j][2 * u + 1] = v.y;
        }
      }
#pragma unroll
      for (int t = 0; t < KQ; ++t) {
        if (pre && t == 1) issue_a((s + 2) * BK, (s + 2) % 3);
        if (pre && t == 2) issue_b((s + 2) * BK, (s + 2) % 3);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i][t], b[j][t], acc[i][j], 0, 0, 0);
      }
    }
    // all LDS reads of this stage have returned before any wave refills it
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    if (NST == 2) {
      __builtin_amdgcn_s_barrier();
      asm volatile("" ::: "memory");  // no copy into the stage moves above the barrier
    }
  }

  double mx = 0.0;
  long long coff[4];
  bool cok[4];
  int ncol[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int n = n0 + wn * 64 + j * 16 + li;
    ncol[j] = n;
    cok[j] = n < N;
    coff[j] = cok[j] ? lmap_col(om, n) : 0;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int m = m0 + wm * 64 + i * 16 + lg + 4 * v;
      if (m >= M) continue;
      const long long roff = lmap_row(om, m);
      const long long moff = sym ? lmap_col(om, m) : 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (!cok[j]) continue;
        const double x = acc[i][j][v];
        if (sym) {
          // the upper triangle, and its mirror image (same products, same order)
          if (m > ncol[j]) continue;
          if (m < ncol[j]) C[lmap_row(om, ncol[j]) + moff] = x;
        }
        C[roff + coff[j]] = x;
        mx = fmax(mx, fabs(x));
      }
    }
  }
  if (maxbits) {
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if (lane == 0) atomicMax(maxbits, (unsigned long long)__double_as_longlong(mx));
  }
}

template <int WGM, int WGN, int BK, int TAG, int NST = 2>
static void launch_lds(const double* A, long long lda, const double* B, long long ldb, int bl,
                       double* C, const OutMap& om, int M, int N, int K,
                       unsigned long long* maxbits, hipStream_t s, int sym = 0,
                       const double* A_2 = nullptr, double* C_2 = nullptr) {
  constexpr int BM = 64 * WGM, BN = 64 * WGN;
  dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM);
  if (sym) {
    // tiles reaching the upper triangle: row tile bm from column tile bm*BM/BN on
    const int nbn = (N + BN - 1) / BN;
    int tiles = 0;
    for (int bm = 0; bm * BM < M; ++bm) tiles += nbn - bm * BM / BN;
    grid = dim3(sym == 2 ? 2 * tiles : tiles, 1);
  }
  dim3 block(64 * WGM * WGN);
  if (bl == B_NCONTIG)
    hipLaunchKernelGGL((k_gemm_f64_lds<WGM, WGN, BK, B_NCONTIG, TAG, NST>), grid, block, 0, s, A,
                       lda, B, ldb, C, om, M, N, K, maxbits, sym, A_2, C_2);
  else
    hipLaunchKernelGGL((k_gemm_f64_lds<WGM, WGN, BK, B_KCONTIG, TAG, NST>), grid, block, 0, s, A,
                       lda, B, ldb, C, om, M, N, K, maxbits, sym, A_2, C_2);
}

// Returns false when the operands do not meet the requirements above.
bool gemm_f64_lds(const double* A, long long lda, const double* B, long long ldb, int blayout,
                  double* C, const OutMap& om, int M, int N, int K, unsigned long long* maxbits,
                  hipStream_t s, int tag, int variant) {
  const int BK = variant == 0 ? 32 : 16;
  if (M < 1 || N < 2 || K < BK || K % BK != 0) return false;
  if ((lda & 1) || (ldb & 1)) return false;
  if (blayout == B_NCONTIG && (N & 1)) return false;
  if (((uintptr_t)A & 15) || ((uintptr_t)B & 15)) return false;
  if (blayout == B_KCONTIG && N < 1) return false;
  if (variant == 5) {
    // 512 x 64 tile (8 waves along M), two stages of 72 KB: products with
    // N = 64 (the last coarse contraction), which the 128-wide tiles would pad
    if (tag == GEMM_TAG_C2)
      launch_lds<8, 1, 16, GEMM_TAG_C2>(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s);
    else if (tag == GEMM_TAG_ENV)
      launch_lds<8, 1, 16, GEMM_TAG_ENV>(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s);
    else
      launch_lds<8, 1, 16, GEMM_TAG_OTHER>(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s);
  } else if (variant == 4) {
    // 128 x 128 tile, 4 waves, 64 KB of LDS: two workgroups per CU
    if (tag == GEMM_TAG_C2)
      launch_lds<2, 2, 16, GEMM_TAG_C2>(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s);
    else if (tag == GEMM_TAG_ENV)
      launch_lds<2, 2, 16, GEMM_TAG_ENV>(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s);
    else
      launch_lds<2, 2, 16, GEMM_TAG_OTHER>(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s);
  } else if (variant == 3) {
    if (tag == GEMM_TAG_C2)
      launch_lds<4, 2, 16, GEMM_TAG_C2, 3>(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s);
    else if (tag == GEMM_TAG_ENV)
      launch_lds<4, 2, 16, GEMM_TAG_ENV, 3>(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s);
    else
      launch_lds<4, 2, 16, GEMM_TAG_OTHER, 3>(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s);
  } else if (variant == 1) {
    if (tag == GEMM_TAG_C2)
      launch_lds<4, 2, 16, GEMM_TAG_C2>(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s);
    else if (tag == GEMM_TAG_ENV)
      launch_lds<4, 2, 16, GEMM_TAG_ENV>(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s);
    else
      launch_lds<4, 2, 16, GEMM_TAG_OTHER>(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s);
  } else {
    if (tag == GEMM_TAG_C2)
      launch_lds<2, 2, 32, GEMM_TAG_C2>(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s);
    else if (tag == GEMM_TAG_ENV)
      launch_lds<2, 2, 32, GEMM_TAG_ENV>(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s);
    else
      launch_lds<2, 2, 32, GEMM_TAG_OTHER>(A, lda, B, ldb, blayout, C, om, M, N, K, maxbits, s);
  }
  return true;
}

// C = A A^T for an M x K K-contiguous A (M = N): the tiles that reach the
// upper triangle, each element written also at its mirror position; the
// same products are summed in the same order as the full product.  Returns
// false where the LDS kernel does not apply (the caller then runs the full
// product).
// With A_2 and C_2 given, C_2 = A_2 A_2^T (same shape, strides and map) in
// the same launch: the half-size grids of the two products together balance
// better over the CUs than each alone (at M = 4096 with 256 x 128 tiles, 544
// tiles in three rounds of 256 workgroups instead of two rounds each).
bool gemm_f64_syrk(const double* A, long long lda, double* C, const OutMap& om, int M, int K,
                   hipStream_t s, const double* A_2, double* C_2) {
  if (M < 128 || (long long)M * M < (1LL << 20) || K < 16 || K % 16 != 0) return false;
  if ((lda & 1) || ((uintptr_t)A & 15) || ((uintptr_t)A_2 & 15)) return false;
  // the symmetric grid (256 x 128 tiles reaching the upper triangle) must
  // fill at least half of the 256 compute units: below that (M = 1024: 40
  // workgroups for both products, each with the whole K loop) the two full
  // products with their many smaller tiles take less time despite twice the
  // MFMAs
  const int nbn = (M + 127) / 128;
  int tiles = 0;
  for (int bm = 0; bm * 256 < M; ++bm) tiles += nbn - 2 * bm;
  if ((A_2 ? 2 : 1) * tiles < 128) return false;
  launch_lds<4, 2, 16, GEMM_TAG_ENV, 3>(A, lda, A, lda, B_KCONTIG, C, om, M, M, K, nullptr, s,
                                        A_2 ? 2 : 1, A_2, C_2);
  return true;
}

}  // namespace hotrg
