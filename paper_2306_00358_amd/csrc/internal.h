// Internal declarations of libhotrg: kernel launchers shared by the engine.
// Not part of the C ABI (see include/hotrg.h).
#pragma once

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <stdint.h>

#include <atomic>

#include "../../include/hotrg.h"

namespace hotrg {

// Where a GEMM output element (m, n) is stored.  The row index is read as
// three mixed-radix digits m = (m0 * r1 + m1) * r2 + m2 and the column as
// n = (n0 * c1 + n1) * c2 + n2; the destination offset is
// m0*s0 + m1*s1 + m2*s2 + n0*t0 + n1*t1 + n2*t2.  This is how the index
// permutations between the contractions of one step are fused into the
// GEMM epilogues instead of separate transpose passes.
struct OutMap {
  int r1, r2;
  long long s0, s1, s2;
  int c1, c2;
  long long t0, t1, t2;
};

// Two-level map: m = mh * rr + ml -> mh*sh + ml*sl; n = nh * cr + nl -> nh*th + nl*tl.
__host__ __device__ inline OutMap omap2(int rr, long long sh, long long sl, int cr, long long th,
                                        long long tl) {
  OutMap o;
  o.r1 = 1; o.r2 = rr; o.s0 = sh; o.s1 = 0; o.s2 = sl;
  o.c1 = 1; o.c2 = cr; o.t0 = th; o.t1 = 0; o.t2 = tl;
  return o;
}

// Plain row-major output of an M x N matrix with leading dimension ld.
__host__ __device__ inline OutMap out_rowmajor(long long ld) { return omap2(1, ld, 0, 1, 1, 0); }

enum BLayout { B_NCONTIG = 0, B_KCONTIG = 1 };

// Call-site tags: large GEMMs get a kernel symbol per tag.  GEMM_NO_TUNE, or-ed
// into a tag, keeps the fixed tile rule (no timed candidate runs, no host wait).
enum GemmTag { GEMM_TAG_OTHER = 0, GEMM_TAG_ENV = 1, GEMM_TAG_C2 = 2, GEMM_NO_TUNE = 0x100 };

// C[map(m,n)] = sum_k A[m*lda + k] * B(k, n), FP64 MFMA.
// B(k, n) = B[k*ldb + n] for B_NCONTIG, B[n*ldb + k] for B_KCONTIG.
// maxbits (may be null): atomic max of |C| as the bit pattern of a
// non-negative double.
void gemm_f64(const double* A, long long lda, const double* B, long long ldb, int blayout,
              double* C, const OutMap& om, int M, int N, int K,
              unsigned long long* maxbits, hipStream_t s, int tag = GEMM_TAG_OTHER);

// One product of a grouped FP64 launch (device table): C (row-major, leading
// dimension ldc) = A B with B's layout given per launch; gate as for RpItem.
struct F64Item {
  const double* A;
  long long lda;
  const double* B;
  long long ldb;
  double* C;
  long long ldc;
  int M, N, K;
  const int* gate;
};
int f64_group_tiles(const F64Item& it);  // 64 x 64 output tiles
void gemm_f64_grouped(int blayout, const F64Item* d_items, const int* d_begin, int count,
                      int tiles, hipStream_t s);

// Split-K FP64 GEMM for products with small M x N and long K: partial
// products of K chunks go to `partials` (ceil(K/kchunk) * M * N doubles) and
// are summed in a fixed order into the row-major M x N matrix C.
// C = A B over K chunks of kchunk summed in order; with sub, C -= sigma * sub
// (sub laid out like C)
void gemm_f64_splitk(const double* A, long long lda, const double* B, long long ldb, int blayout,
                     double* C, long long ldc, int M, int N, int K, int kchunk, double* partials,
                     hipStream_t s, const double* sub = nullptr, double sigma = 0.0);

// Direct-to-LDS FP64 GEMM (gemm_lds.hip); returns false if the operands do
// not meet its alignment / K-multiple requirements.  variant 0: 4 waves,
// 128 x 128 tile, K slab 32; variant 1: 8 waves, 256 x 128 tile, K slab 16.
// C = A A^T (M x M, A M x K K-contiguous) from the upper-triangle tiles with
// mirrored stores, and C_2 = A_2 A_2^T in the same launch when A_2 is given;
// false where it does not apply.
bool gemm_f64_syrk(const double* A, long long lda, double* C, const OutMap& om, int M, int K,
                   hipStream_t s, const double* A_2 = nullptr, double* C_2 = nullptr);
bool gemm_f64_lds(const double* A, long long lda, const double* B, long long ldb, int blayout,
                  double* C, const OutMap& om, int M, int N, int K, unsigned long long* maxbits,
                  hipStream_t s, int tag, int variant);

// Tile order of a launch over tm x tn output tiles.  Workgroups are handed
// round-robin to the 8 XCDs, each with its own L2.  With group gm > 0 the
// XCD that receives workgroup b takes a contiguous eighth of the tiles,
// walked gm row panels at a time (all of a group's rows for one column
// panel, then the next column panel), so that the workgroups resident on an
// XCD share a few row panels of A and column panels of B.  gm = 0:
// row-major order.
__device__ __forceinline__ void tile_order(int tm, int tn, int b, int gm, int& im, int& in) {
  if (gm <= 0) {
    im = b / tn;
    in = b - im * tn;
    return;
  }
  const int T = tm * tn;
  const int t = (T & 7) ? b : (b & 7) * (T >> 3) + (b >> 3);
  const int g = t / (gm * tn);
  const int rows = min(gm, tm - g * gm);
  const int r = t - g * gm * tn;
  im = g * gm + r % rows;
  in = r / rows;
}

// ---- reduced-precision contractions (gemm_rp.hip) ----
enum RpMode { RP_F32 = 0, RP_BF16X3 = 1 };
enum RpOut { RP_OUT_F32 = 0, RP_OUT_SPLIT = 1, RP_OUT_F64 = 2 };
// An operand: one float array (RP_F32) or bf16 arrays hi and lo (RP_BF16X3).
struct RpOperand {
  const void* hi;
  const void* lo;
};
// C[map(m,n)] = sum_k A[m][k] B[n][k]; rows of lda / ldb elements (multiples
// of 8, zero past the true K); K a multiple of 32.  Output as float, split
// bf16 (C = hi, Clo = lo) or double.  Returns false if a requirement fails.
// Autotuner table shared by the GEMM launchers: the fastest of `count`
// candidates (run(ctx, c) launches candidate c, false if it does not apply)
// for this shape, measured on first use; -1 if tuning is off.  If it had to
// measure, *maxbits (when given) is zeroed again for the final run.
int tune_choice(int prec, long long lda, long long ldb, int bl, const OutMap& om, int M, int N,
                int K, unsigned long long* maxbits, int tag, int count,
                bool (*run)(void*, int), void* ctx, hipStream_t s);
bool gemm_rp(int mode, const RpOperand& A, long long lda, const RpOperand& B, long long ldb,
             int out, void* C, void* Clo, const OutMap& om, int M, int N, int K,
             unsigned long long* maxbits, hipStream_t s, int tag);
inline long long pad32(long long k) { return (k + 31) / 32 * 32; }

// One product of a grouped launch (device table): the operands and output
// of gemm_rp, and a gate (device int, may be null) that skips the product's
// tiles while it reads 0.
struct RpItem {
  RpOperand A;
  long long lda;
  RpOperand B;
  long long ldb;
  void* C;
  void* Clo;
  OutMap om;
  int M, N, K;
  unsigned long long* maxbits;
  const int* gate;
};
// Workgroups of an item under tile configuration cfg (0: 256 x 256,
// 1: 256 x 128 two stages, 2: 256 x 128 three stages): its output tiles,
// rounded up to a multiple of 8.
int rp_group_tiles(const RpItem& it, int cfg);
// One launch over `tiles` tiles; d_begin[i] is the first tile of item i
// (ascending, d_begin[0] = 0).  Requirements per item as for gemm_rp.
void gemm_rp_grouped(int mode, int out, int cfg, const RpItem* d_items, const int* d_begin,
                     int count, int tiles, hipStream_t s);

// Reduced-precision operands of a step from the coarse tensor `src` (f64 or
// f32, legs optionally transposed, divided by the max read from maxbits).
// Each output is an RpOperand written in `mode`; rows are zero-padded to the
// lengths given (multiples of 32):
//   Tn   natural float tensor (dx,dy,dx,dy)               (also the state)
//   OT   rows (l,u), K (r,d), row length ldP                (environment half)
//   OX   rows (l,d), K (u,r), row length ldP                (environment half)
//   OC1  rows (j,d,c), K b, row length ldx                  (first contraction)
//   OC2  rows (l,e), K (a,c) of T[a,c,e,l], row length ldP  (O(D^7) contraction)
struct RpOps {
  void* hi[4];
  void* lo[4];
};
void launch_prep_rp(const void* src, bool src_f32, bool rotate, int dx, int dy,
                    const unsigned long long* maxbits, float* Tn, int mode, const RpOps& ops,
                    long long ldP, long long ldx, hipStream_t s);
// U1 rows (i,a), K b (row length ldx); U3 rows k, K (d,e) = U[e,d,k] (row length ldn)
void launch_layout_u_rp(const double* Ucan, int dx, int dn, int mode, void* u1hi, void* u1lo,
                        void* u3hi, void* u3lo, long long ldx, long long ldn, hipStream_t s);

// All eigenpairs of the symmetric tridiagonal (d, e), n <= 128, in one
// workgroup (divide and conquer): eigenvalues ascending into W (which may be
// d), eigenvectors as the rows of Zt (n x n); *info = 1 if a result is not
// finite.  False when the launch fails.
bool tridiag_eig_small(const double* d, const double* e, int n, double* W, double* Zt, int* info,
                       hipStream_t s);
// The same with the back-transform: Hb (n x n) holds Q^T of the Householder
// reduction on entry and the eigenvector rows (row c for W[c]) on exit.
bool tridiag_eig_small_back(const double* d, const double* e, int n, double* W, double* Hb,
                            int* info, hipStream_t s);
// All eigenpairs of a small symmetric matrix (3 <= n <= 128, row-major, over
// M): W ascending, M <- eigenvector rows; E (n) scratch; false when not
// applicable or the launch fails.
bool dense_eig_small(double* M, int n, double* W, double* E, int* info, hipStream_t s);

// ---- small kernels (kernels.hip) ----
void launch_maxabs(const void* x, long long n, bool is_f32, unsigned long long* maxbits, hipStream_t s);
void launch_init_acc(const unsigned long long* maxbits, double* acc, hipStream_t s);
// Sticky eigensolver failure: *flag = 1 if *info != 0 or force.
void launch_fold_info(const int* info, int* flag, int force, hipStream_t s);
// Operands of the next step from the coarse tensor `src` (f64 or f32),
// optionally with legs transposed (l,u,r,d) -> (u,l,d,r), scaled by
// 1/max (read from maxbits): Tn natural (dx,dy,dx,dy); Xt [(l,d),(u,r)];
// Tp [(l,u),(d,r)].  Outputs are f64 or f32 per out_f32.
void launch_prep_mirror(const double* T, int dx, int dy, double* Tn, double* Xt, hipStream_t s);
void launch_store(double* p, double v, hipStream_t s);
void launch_prep(const void* src, bool src_f32, bool rotate, int dx, int dy,
                 const unsigned long long* maxbits, void* Tn, void* Xt, void* Tp, bool out_f32,
                 hipStream_t s);
void launch_symmetrize(double* M, int n, hipStream_t s);
// W: the `cnt` leading eigenvalues of M in ascending order (cnt <= n);
// total: trace(M) (device scalar).
void launch_spectrum(const double* W, int cnt, int n, int dn, int trunc, double tau, int spec_len,
                     const double* total, double* spec_out, double* rec, int* kept, hipStream_t s);
// V: `cols` eigenvectors of length n, vector c at V[c*n], ascending order.
void launch_isometry(const double* V, int cols, int n, int dn, const int* kept, double* Ucan,
                     hipStream_t s);
void launch_trace(const double* M, int n, double* out, hipStream_t s);
size_t topk_workspace_doubles(int n, int p);
// Batched shifted Cholesky-QR step of the block eigensolver: per problem,
// Rt = (R^-1)^T with G (+ shift) = R^T R (one workgroup each; p <= 128, a
// multiple of 16).  Pass 0 and 1 factor the diagonally scaled, shifted G,
// pass 2 the plain one; pass 1 between checks (!full) is skipped when G is
// the identity to 1e-2.  A non-positive pivot sets *fail.
struct CholItem {
  const double* G;
  double* Rt;
  int* fail;
  const int* gate;
  int p;
  double shift_rel;
};
void launch_chol_inv_batched(const CholItem* d_items, int count, int pmax, int pass, bool full,
                             hipStream_t s);
bool topk_eigs(const double* M, int n, int p, int need, double tol,
               int q_first, double* shift, int* nocheck, double* ws, double* W, double* Xout,
               int* dinfo, int* iters, int* enough, double* resid, hipStream_t s);
void launch_layout_u(const double* Ucan, int dx, int dn, void* U1, void* U3, bool out_f32,
                     hipStream_t s);
void launch_norm(const unsigned long long* maxbits, const void* Tt, bool f32, int dn, int dy,
                 double weight, double* acc, double* rec, hipStream_t s);
void launch_finish(const void* Tn, bool f32, int dx, int dy, double weight, const double* acc,
                   double* out, hipStream_t s);
void launch_f64_to_f32(const double* x, float* y, long long n, hipStream_t s);
void launch_f32_to_f64(const float* x, double* y, long long n, hipStream_t s);

// ---- lockstep batch engine (group.hip) ----
constexpr int kGroupRec = 6;  // doubles per step record (as the engine's)
// Per-problem control block, updated by the kernels of a sweep.
struct GroupCtl {
  int active;  // the problem has steps left
  int iter;    // its block eigensolver is still iterating in this step
  int fail;    // sticky: eigensolver budget exhausted or a Cholesky pivot <= 0
  int k;       // steps done
};
// Per-problem descriptor of a run (device memory, fixed while it runs).
struct GroupStep {
  GroupCtl* ctl;
  int n, dn, dy, p, need, trunc, spec_len, K;
  double tau, tol;
  const double* M;  // environment (n x n)
  double* trace;
  double* W;
  double* X;
  int* kept;
  double *V, *Y, *T2, *Yx, *G, *Rt, *H, *res;
  double* recs;
  double* spec;
  double* acc;
  const void* Tt;
  int tt_f32;
  unsigned long long* maxbits;
  double* shift;  // sweep shift per step parity (theta_min / 2 of the last Rayleigh-Ritz)
};
void group_begin(const GroupStep* d, int count, hipStream_t s);
void group_seed(const GroupStep* d, int count, long long max_pn, hipStream_t s);
void group_symm_h(const GroupStep* d, int count, hipStream_t s);
// Rayleigh-Ritz matrices H (p x p, p a multiple of 16, <= 128) of the
// iterating problems: Householder reduction (diagonal into W, off-diagonal
// into G, Q^T over H), then divide and conquer with the back-transform:
// W ascending, H <- Z^T (row c = eigenvector c)
void group_sytrd(const GroupStep* d, int count, int pmax, hipStream_t s);
void group_stedc(const GroupStep* d, int count, int pmax, hipStream_t s);
void group_resid(const GroupStep* d, int count, bool last, hipStream_t s);
void group_restart(const GroupStep* d, int count, long long max_pn, hipStream_t s);
void group_shift(const GroupStep* d, int count, long long max_pn, hipStream_t s);
// whole small environments (n <= 128, p = n rounded up to even) by the same two kernels
void group_dense(const GroupStep* d, int count, int pmax, hipStream_t s);
void group_spectrum(const GroupStep* d, int count, hipStream_t s);
void group_norm(const GroupStep* d, int count, hipStream_t s);
void group_zero_max(const GroupStep* d, int count, hipStream_t s);
void group_advance(const GroupStep* d, int count, hipStream_t s);

// ---- engine hooks used by the scheduler (sched.cpp) ----
// C1 -> C2 -> C3 in FP64 on caller buffers (X1, X2: dn*dx*dy*dx*dy doubles;
// Tt: dn*dy*dn*dy); *maxbits is cleared by a kernel and receives max|Tt|.
void coarse_f64_into(hotrg_ctx* c, const double* Tn, const double* Tp, const double* U1,
                     const double* U3, int dx, int dy, int dn, double* X1, double* X2, double* Tt,
                     unsigned long long* maxbits, int tag_flags);
hipStream_t ctx_stream(const hotrg_ctx* c);
// Allocation-free entry point's scratch (noalloc.hip): look up this device's
// copy of the static array once (call with the device current).
void noalloc_init_device(int device);
// hotrg_run with a cancellation flag checked between steps.
hotrg_status run_problem(hotrg_ctx* c, const hotrg_model_params* params, const hotrg_opts* o,
                         hotrg_result* res, const std::atomic<bool>* cancel);
void ctx_trim(hotrg_ctx* c);  // release the step workspace
double ctx_seconds(const hotrg_ctx* c);
int ctx_device(const hotrg_ctx* c);
size_t ctx_budget(const hotrg_ctx* c);
int& ctx_workers(hotrg_ctx* c);
int& ctx_test_fail_step(hotrg_ctx* c);  // failure-injection hook, 0: off
void*& ctx_sched(hotrg_ctx* c);
void sched_shutdown(hotrg_ctx* c);
const char* last_error_text();
void set_last_error(const char* m);

}  // namespace hotrg
