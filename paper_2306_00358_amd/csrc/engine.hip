// Host engine of libhotrg: contexts, device buffers, the directional step
// and the C ABI of include/hotrg.h (arXiv 2306.00358, Sec. 2, Fig. 1).
//
// One step on one HIP stream, no host wait inside:
//   environment halves  A2 = X_b X_b^T, A1 = X_t X_t^T      (MFMA GEMM)
//   environment combine M = A2' A1'^T, symmetrised          (MFMA GEMM)
//   eigendecomposition of M in FP64                          (rocSOLVER dsyevd)
//   spectrum, truncation error, cut gap, projector U          (single-block kernels)
//   C1: X1 = U T,  C2: X2 = X1 T,  C3: T~ = X2 U, max|T~|     (MFMA GEMMs)
//   ln n_k accumulation and torus trace                       (single block)
//   operands of the next step: legs transposed, divided by n_k
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/hotrg.h"
#include "internal.h"
#include "precision.h"

namespace hotrg {
std::vector<double> ising_tensor(double beta, double J);
std::vector<double> xy_tensor(double beta, int n_max);
std::vector<double> potts_tensor(double beta, int q);
std::vector<double> gxy_tensor(double beta, double delta, int n_max);
}  // namespace hotrg

using namespace hotrg;

static thread_local std::string g_err;

namespace {

struct Error {
  hotrg_status st;
  std::string msg;
};

[[noreturn]] void fail(hotrg_status st, const std::string& msg) { throw Error{st, msg}; }

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) fail(HOTRG_ERR_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

// doubles per step record: ln n_k, truncation error, cut gap, torus ln Z/N,
// kept columns, side of the environment the projector came from
constexpr int kRec = 6;

// two-sided choice: the right projector only when its truncation error is
// smaller by more than this (reflection-symmetric tensors keep the left one)
constexpr double kSideMargin = 1e-12;

}  // namespace

struct hotrg_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  size_t budget = 0;
  size_t in_use = 0;
  rocblas_handle blas = nullptr;
  // step workspace, grown on demand
  Buf A1, A2, M, W, E, Ucan, U1, U3, X1, X2, Tt, scal, EW, Xr;
  // two-sided isometry: mirrored operands, right environment and its solve,
  // and its step record / kept count / trace / spectrum (Side)
  Buf Tm, Xm, M2, W2, Xr2, Side;
  // reduced-precision workspace: [0] hi / float, [1] lo (split bf16 only)
  Buf RA1[2], RA2[2], RX1[2], RX2[2], RU1[2], RU3[2];
  // scal layout (bytes): 0 maxbits (u64), 8 info (int), 16 kept (int), 24 finish out (double),
  // 32 primitive max (u64), 40 trace(M) (double), 48 iterative solver info (int)
  int last_eig_iters = 0;      // sweeps of the last iterative solve (0: dense solver)
  double last_eig_resid = 0.0;
  // many-problem scheduler (sched.cpp), created on first use
  void* sched = nullptr;
  int n_workers = 16;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  // test hook (environment HOTRG_TEST_EIG_FAIL_STEP, read at creation): the
  // eigensolve of this step number reports failure, as a non-zero rocSOLVER
  // info would; 0: off
  int test_fail_step = 0;
  // lockstep batches: sweeps run, of them graph replays, graph captures,
  // problems re-run alone after their batched eigensolve failed
  uint64_t g_sweeps = 0, g_replays = 0, g_captures = 0, g_fallbacks = 0;
  // per-phase timing
  bool timing = false;
  struct Mark {
    int step, phase, dx, dy, dn;
    hipEvent_t a, b;
  };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> pool;
  hipEvent_t open_ev = nullptr;
  int open_phase = -1, m_step = 0, m_dx = 0, m_dy = 0, m_dn = 0;
};

// What an iterative eigensolve learnt, for the next solve of the same kind:
// its n, the sweeps it is estimated to have needed, the shift of its sweeps
// and whether its orthogonality checks stopped missing.
struct EigHint {
  int n = 0, sweeps = 0, nocheck = 0;
  double shift = 0.0;
};

struct hotrg_state {
  int prec = HOTRG_FP64;
  int dx = 0, dy = 0, k = 0;
  // current normalised tensor: Tn (FP64) when !cur_f32, Tn32 (FP32) otherwise
  bool cur_f32 = false;
  Buf Tn32;
  // precision the operands below were prepared for
  int ops_prec = HOTRG_FP64;
  Buf Tn, Xt, Tp;      // FP64 operands of the next step (normalised)
  Buf RO[4][2];        // reduced-precision operands OT, OX, OC1, OC2 ([.][0] hi/float, [.][1] lo)
  Buf acc;             // device: double ln n_0 + sum_k 2^-k ln n_k, then an int
                       // sticky flag set when any step's eigensolve failed
  Buf recs;            // device: kRec doubles per step
  Buf spec;            // device spectra, spec_cap doubles per step
  int rec_cap = 0, spec_len = 0;
  // what the last iterative eigensolve of each step parity learnt
  // ([parity + 2 * side])
  EigHint eig[4];
  // precision schedule: first step allowed in reduced precision, and the
  // a-priori error bound of the steps run reduced so far
  int first_reduced = 1;
  double err_bound = 0.0;
};

namespace {

void ctx_free(hotrg_ctx* c, Buf& b) {
  if (b.p) {
    (void)hipFree(b.p);
    c->in_use -= b.bytes;
    b.p = nullptr;
    b.bytes = 0;
  }
}

// Make `b` hold at least `bytes`, keeping the HBM budget.  Growing frees the
// old buffer first (its contents are not kept).
void ensure(hotrg_ctx* c, Buf& b, size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (b.bytes >= bytes) return;
  HIPCHK(hipStreamSynchronize(c->stream));
  ctx_free(c, b);
  if (c->budget && c->in_use + bytes > c->budget)
    fail(HOTRG_ERR_OOM, "device memory budget exceeded: need " + std::to_string(bytes) +
                            " more bytes, " + std::to_string(c->in_use) + " of " +
                            std::to_string(c->budget) + " in use");
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess)
    fail(e == hipErrorOutOfMemory ? HOTRG_ERR_OOM : HOTRG_ERR_DEVICE,
         std::string("hipMalloc(") + std::to_string(bytes) + "): " + hipGetErrorString(e));
  b.p = p;
  b.bytes = bytes;
  c->in_use += bytes;
}

// Grow while keeping the first `keep` bytes.
void ensure_keep(hotrg_ctx* c, Buf& b, size_t bytes, size_t keep) {
  if (b.bytes >= bytes) return;
  Buf old = b;
  b = Buf{};
  try {
    ensure(c, b, bytes);
  } catch (...) {
    b = old;
    throw;
  }
  if (old.p) {
    if (keep) HIPCHK(hipMemcpyAsync(b.p, old.p, keep, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    (void)hipFree(old.p);
    c->in_use -= old.bytes;
  }
}

hipEvent_t get_event(hotrg_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIPCHK(hipEventCreate(&e));
  return e;
}

// Close the open phase (if any) and open `phase` (-1: just close).
void mark(hotrg_ctx* c, int phase) {
  if (!c->timing) return;
  hipEvent_t e = get_event(c);
  HIPCHK(hipEventRecord(e, c->stream));
  if (c->open_phase >= 0)
    c->marks.push_back({c->m_step, c->open_phase, c->m_dx, c->m_dy, c->m_dn, c->open_ev, e});
  if (phase >= 0) {
    // the closing event of one phase opens the next
    c->open_ev = e;
    c->open_phase = phase;
  } else {
    c->open_phase = -1;
    c->open_ev = nullptr;
  }
}


void check_prec(int prec) {
  if (prec != HOTRG_FP64 && prec != HOTRG_FP32 && prec != HOTRG_BF16X3)
    fail(HOTRG_ERR_INVALID, "prec must be HOTRG_FP64, HOTRG_FP32 or HOTRG_BF16X3");
}

void check_opts(const hotrg_opts* o) {
  if (!o) fail(HOTRG_ERR_INVALID, "opts is NULL");
  if (o->d_cut < 1) fail(HOTRG_ERR_INVALID, "d_cut must be >= 1");
  if (o->n_steps < 0) fail(HOTRG_ERR_INVALID, "n_steps must be >= 0");
  if (o->trunc != HOTRG_TRUNC_PLAIN && o->trunc != HOTRG_TRUNC_MULTIPLET)
    fail(HOTRG_ERR_INVALID, "trunc must be HOTRG_TRUNC_PLAIN or HOTRG_TRUNC_MULTIPLET");
  if (o->trunc == HOTRG_TRUNC_MULTIPLET && !(o->degen_tol >= 0.0))
    fail(HOTRG_ERR_INVALID, "degen_tol must be >= 0");
  if (o->spec_len < 0) fail(HOTRG_ERR_INVALID, "spec_len must be >= 0");
  if (o->eig != HOTRG_EIG_AUTO && o->eig != HOTRG_EIG_DENSE)
    fail(HOTRG_ERR_INVALID, "eig must be HOTRG_EIG_AUTO or HOTRG_EIG_DENSE");
  if (o->isometry != HOTRG_ISO_ONE_SIDED && o->isometry != HOTRG_ISO_TWO_SIDED)
    fail(HOTRG_ERR_INVALID, "isometry must be HOTRG_ISO_ONE_SIDED or HOTRG_ISO_TWO_SIDED");
  if (!(o->tol >= 0.0) || !std::isfinite(o->tol)) fail(HOTRG_ERR_INVALID, "tol must be >= 0");
  if (o->prec == HOTRG_PREC_AUTO) {
    if (!(o->tol > 0.0)) fail(HOTRG_ERR_INVALID, "HOTRG_PREC_AUTO needs tol > 0");
    return;  // resolved by the caller (resolve_prec)
  }
  check_prec(o->prec);
  if (o->isometry == HOTRG_ISO_TWO_SIDED && o->prec != HOTRG_FP64)
    fail(HOTRG_ERR_INVALID, "two-sided isometry needs FP64 contractions");
}

// Options with HOTRG_PREC_AUTO resolved for a run from dims (dx, dy): the
// cheapest precision whose a-priori bound meets tol (FP64 with the two-sided
// isometry, which has no reduced-precision path).
hotrg_opts resolve_prec(const hotrg_opts* o, int dx, int dy) {
  hotrg_opts r = *o;
  if (r.prec == HOTRG_PREC_AUTO)
    r.prec = r.isometry == HOTRG_ISO_TWO_SIDED
                 ? HOTRG_FP64
                 : plan_auto(r.tol, dx, dy, r.d_cut, r.n_steps).prec;
  return r;
}

// Largest intermediate of a step with dims (dx, dy) and D' = dn, in elements.
long long x_elems(int dx, int dy, int dn) { return (long long)dn * dx * dy * dx * dy; }

void check_dims(int dx, int dy, int dn) {
  long long n = (long long)dx * dx;
  if (n > 16384) fail(HOTRG_ERR_INVALID, "dx*dx exceeds 16384 (environment matrix too large)");
  if (x_elems(dx, dy, dn) > (1LL << 36)) fail(HOTRG_ERR_INVALID, "intermediate exceeds 2^36 elements");
  if ((long long)dn * dy * dx > 0x7fffffffLL || (long long)dx * dy * dx > 0x7fffffffLL)
    fail(HOTRG_ERR_INVALID, "GEMM dimension exceeds 2^31");
}

// FP64 operands of T (dims dx, dy) in the state: environment halves into M.
void environment_f64(hotrg_ctx* c, const double* Tn, const double* Xt, int dx, int dy,
                     Buf* out = nullptr) {
  Buf& Mb = out ? *out : c->M;
  const long long P = (long long)dx * dy;  // rows / cols of the halves
  const long long n = (long long)dx * dx;
  const long long K2 = (long long)dy * dy;
  ensure(c, c->A1, (size_t)(P * P) * 8);
  ensure(c, c->A2, (size_t)(P * P) * 8);
  ensure(c, Mb, (size_t)(n * n) * 8);
  // A2[(i,e),(k,f)] = sum_{c,d} T[i,e,c,d] T[k,f,c,d], stored as A2'[(i,k),(e,f)]
  // rows (i,e): i -> dx*dy^2, e -> dy; cols (k,f): k -> dy^2, f -> 1
  // A1[(j,e),(l,f)] = sum_{a,b} T[j,a,b,e] T[l,a,b,f] from Xt[(l,d),(u,r)], stored as A1'[(j,l),(e,f)]
  // Both halves are Gram matrices X X^T: where it applies, one launch
  // computes the upper triangles of both and mirrors them (half the MFMAs).
  const OutMap o2 = omap2(dy, dx * K2, dy, dy, K2, 1);
  if (!gemm_f64_syrk(Tn, P, (double*)c->A2.p, o2, (int)P, (int)P, c->stream, Xt,
                     (double*)c->A1.p)) {
    gemm_f64(Tn, P, Tn, P, B_KCONTIG, (double*)c->A2.p, o2, (int)P, (int)P, (int)P, nullptr,
             c->stream, GEMM_TAG_ENV);
    gemm_f64(Xt, P, Xt, P, B_KCONTIG, (double*)c->A1.p, o2, (int)P, (int)P, (int)P, nullptr,
             c->stream, GEMM_TAG_ENV);
  }
  // M[(i,j),(k,l)] = sum_{e,f} A2'[(i,k),(e,f)] A1'[(j,l),(e,f)]: GEMM rows (i,k), cols (j,l)
  // rows (i,k): i -> dx*n, k -> dx; cols (j,l): j -> n, l -> 1
  const OutMap om = omap2(dx, dx * n, dx, dx, n, 1);
  gemm_f64((const double*)c->A2.p, K2, (const double*)c->A1.p, K2, B_KCONTIG, (double*)Mb.p, om,
           (int)n, (int)n, (int)K2, nullptr, c->stream, GEMM_TAG_ENV);
}

}  // namespace

namespace hotrg {

// C1, C2, C3 in FP64 on caller-provided buffers: X1 and X2 hold
// dn*dx*dy*dx*dy doubles each, Tt receives T~[i,j,k,l] (dims dn,dy,dn,dy),
// and *maxbits (cleared here by a kernel) max|T~|.  `tag_flags` is or-ed
// into every GEMM tag (GEMM_NO_TUNE: fixed tile rule, no measurement, and no
// per-phase timing events: the allocation-free entry point's path).
void coarse_f64_into(hotrg_ctx* c, const double* Tn, const double* Tp, const double* U1,
                     const double* U3, int dx, int dy, int dn, double* X1, double* X2, double* Tt,
                     unsigned long long* maxbits, int tag_flags) {
  const bool marks = tag_flags == 0;
  const long long Q = (long long)dx * dy;
  // C1: rows (i,a), cols (j,d,c) = j*(dx*dy) + (d*dy + c); K = b.
  //     X1[(i,j,d),(a,c)] at ((i*dy + j)*dx + d)*Q + a*dy + c
  //     rows (i,a): i -> dy*dx*Q, a -> dy; cols (j,d,c): j -> dx*Q, d -> Q, c -> 1
  OutMap o1 = omap2(dx, (long long)dy * dx * Q, dy, 1, 0, 0);
  o1.c1 = dx; o1.c2 = dy; o1.t0 = (long long)dx * Q; o1.t1 = Q; o1.t2 = 1;
  if (marks) mark(c, HOTRG_PHASE_C1);
  gemm_f64(U1, dx, Tn, (long long)dy * dx * dy, B_NCONTIG, X1, o1, dn * dx, dy * dx * dy, dx,
           nullptr, c->stream, GEMM_TAG_OTHER | tag_flags);
  // C2: rows (i,j,d) = (ij)*dx + d, cols (l,e) = l*dx + e; K = (a,c).
  //     X2[(i,j,l),(d,e)] at ((ij)*dy + l)*dx*dx + d*dx + e
  const long long n = (long long)dx * dx;
  //     rows (ij,d): ij -> dy*n, d -> dx; cols (l,e): l -> n, e -> 1
  const OutMap o2 = omap2(dx, (long long)dy * n, dx, dx, n, 1);
  if (marks) mark(c, HOTRG_PHASE_C2);
  gemm_f64(X1, Q, Tp, Q, B_NCONTIG, X2, o2, dn * dy * dx, (int)Q, (int)Q, nullptr, c->stream,
           GEMM_TAG_C2 | tag_flags);
  // C3: rows (i,j,l) = (ij)*dy + l, cols k; K = (d,e).
  //     T~[i,j,k,l] at ((ij)*dn + k)*dy + l
  if (marks) mark(c, HOTRG_PHASE_C3);
  launch_store((double*)maxbits, 0.0, c->stream);  // a kernel, not a memset
  //     rows (ij,l): ij -> dn*dy, l -> 1; cols k -> dy
  const OutMap o3 = omap2(dy, (long long)dn * dy, 1, 1, dy, 0);
  gemm_f64(X2, n, U3, dn, B_NCONTIG, Tt, o3, dn * dy * dy, dn, (int)n, maxbits, c->stream,
           GEMM_TAG_OTHER | tag_flags);
}

hipStream_t ctx_stream(const hotrg_ctx* c) { return c->stream; }

}  // namespace hotrg

namespace {

// C1, C2, C3 in FP64: T~[i,j,k,l] (dims dn,dy,dn,dy) into c->Tt, max into scal.
void coarse_f64(hotrg_ctx* c, const double* Tn, const double* Tp, const double* U1,
                const double* U3, int dx, int dy, int dn, unsigned long long* maxbits) {
  const long long X = x_elems(dx, dy, dn);
  ensure(c, c->X1, (size_t)X * 8);
  ensure(c, c->X2, (size_t)X * 8);
  ensure(c, c->Tt, (size_t)dn * dy * dn * dy * 8);
  coarse_f64_into(c, Tn, Tp, U1, U3, dx, dy, dn, (double*)c->X1.p, (double*)c->X2.p,
                  (double*)c->Tt.p, maxbits, 0);
}

void prepare_operands(hotrg_ctx* c, hotrg_state* st, int prec, const void* src, bool src_f32,
                      bool rotate, int dx, int dy, const unsigned long long* mb);

hotrg_state* new_state(hotrg_ctx* c, const std::vector<double>& T0, int dx, int dy, int prec) {
  for (double v : T0)
    if (!std::isfinite(v)) fail(HOTRG_ERR_NUMERIC, "initial tensor has a non-finite element");
  auto* st = new hotrg_state();
  try {
    st->prec = prec;
    st->dx = dx;
    st->dy = dy;
    const size_t ne = T0.size();
    ensure(c, st->acc, 16);
    ensure(c, c->scal, 64);
    // upload through the Tt workspace as FP64
    ensure(c, c->Tt, ne * 8);
    HIPCHK(hipMemcpyAsync(c->Tt.p, T0.data(), ne * 8, hipMemcpyHostToDevice, c->stream));
    unsigned long long* mb = (unsigned long long*)c->scal.p;
    HIPCHK(hipMemsetAsync(mb, 0, 8, c->stream));
    launch_maxabs(c->Tt.p, (long long)ne, false, mb, c->stream);
    launch_init_acc(mb, (double*)st->acc.p, c->stream);
    prepare_operands(c, st, HOTRG_FP64, c->Tt.p, false, false, dx, dy, mb);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
  } catch (...) {
    hotrg_state_free(c, st);
    throw;
  }
  return st;
}

// Precision of step k's contractions: reduced (FP32 or split BF16) only in
// the steady state, where both legs already have the kept dimension, and
// from the state's first_reduced step on (precision.h); the warm-up steps
// and the heavily weighted early steps a tolerance asks for stay FP64.
int step_precision(const hotrg_state* st, int k, int dx, int dy, int d_cut) {
  return step_is_reduced(st->prec, k, dx, dy, d_cut, st->first_reduced) ? st->prec : HOTRG_FP64;
}

int rp_mode(int prec) { return prec == HOTRG_FP32 ? RP_F32 : RP_BF16X3; }

// Operands of a step with dims (dx, dy) in precision `prec`, from the tensor
// `src` (FP64 or FP32; legs transposed if `rotate`; divided by the max read
// from `mb`).  Also records the state's natural tensor in matching format.
void prepare_operands(hotrg_ctx* c, hotrg_state* st, int prec, const void* src, bool src_f32,
                      bool rotate, int dx, int dy, const unsigned long long* mb) {
  const size_t ne = (size_t)dx * dy * dx * dy;
  if (prec == HOTRG_FP64) {
    ensure_keep(c, st->Tn, ne * 8, 0);
    ensure_keep(c, st->Xt, ne * 8, 0);
    ensure_keep(c, st->Tp, ne * 8, 0);
    launch_prep(src, src_f32, rotate, dx, dy, mb, st->Tn.p, st->Xt.p, st->Tp.p, false, c->stream);
    st->cur_f32 = false;
  } else {
    const int mode = rp_mode(prec);
    const size_t es = mode == RP_F32 ? 4 : 2;
    const long long P = (long long)dx * dy, ldP = pad32(P), ldx = pad32(dx);
    const size_t rows[4] = {(size_t)P, (size_t)P, (size_t)dy * dx * dy, (size_t)P};
    const size_t ld[4] = {(size_t)ldP, (size_t)ldP, (size_t)ldx, (size_t)ldP};
    const bool padded[4] = {ldP != P, ldP != P, ldx != dx, ldP != P};
    RpOps ops;
    ensure_keep(c, st->Tn32, ne * 4, 0);
    for (int i = 0; i < 4; ++i) {
      for (int h = 0; h < (mode == RP_F32 ? 1 : 2); ++h) {
        ensure_keep(c, st->RO[i][h], rows[i] * ld[i] * es, 0);
        if (padded[i]) HIPCHK(hipMemsetAsync(st->RO[i][h].p, 0, rows[i] * ld[i] * es, c->stream));
      }
      ops.hi[i] = st->RO[i][0].p;
      ops.lo[i] = mode == RP_F32 ? nullptr : st->RO[i][1].p;
    }
    launch_prep_rp(src, src_f32, rotate, dx, dy, mb, (float*)st->Tn32.p, mode, ops, ldP, ldx,
                   c->stream);
    st->cur_f32 = true;
  }
  st->ops_prec = prec;
}

void release_operands(hotrg_ctx* c, hotrg_state* st) {
  Buf* bufs[] = {&st->Tn, &st->Xt, &st->Tp, &st->Tn32};
  for (Buf* b : bufs) ctx_free(c, *b);
  for (auto& o : st->RO)
    for (auto& b : o) ctx_free(c, b);
}

// Environment M (FP64 output) from reduced-precision operands.
void environment_rp(hotrg_ctx* c, hotrg_state* st, int mode, int dx, int dy) {
  const long long P = (long long)dx * dy, n = (long long)dx * dx, K2 = (long long)dy * dy;
  const long long ldP = pad32(P), ldK2 = pad32(K2);
  const size_t es = mode == RP_F32 ? 4 : 2;
  const int fmt = mode == RP_F32 ? RP_OUT_F32 : RP_OUT_SPLIT;
  const int halves = mode == RP_F32 ? 1 : 2;
  for (int h = 0; h < halves; ++h) {
    ensure(c, c->RA1[h], (size_t)n * ldK2 * es);
    ensure(c, c->RA2[h], (size_t)n * ldK2 * es);
    if (ldK2 != K2) {
      HIPCHK(hipMemsetAsync(c->RA1[h].p, 0, (size_t)n * ldK2 * es, c->stream));
      HIPCHK(hipMemsetAsync(c->RA2[h].p, 0, (size_t)n * ldK2 * es, c->stream));
    }
  }
  ensure(c, c->M, (size_t)(n * n) * 8);
  auto op = [&](Buf* b) { return RpOperand{b[0].p, halves == 2 ? b[1].p : nullptr}; };
  const RpOperand OT = op(st->RO[0]), OX = op(st->RO[1]);
  // halves stored as [(i,k),(e,f)]: rows (i,e): i -> dx*ldK2, e -> dy; cols (k,f): k -> ldK2, f -> 1
  const OutMap o2 = omap2(dy, dx * ldK2, dy, dy, ldK2, 1);
  bool ok = gemm_rp(mode, OT, ldP, OT, ldP, fmt, c->RA2[0].p, halves == 2 ? c->RA2[1].p : nullptr,
                    o2, (int)P, (int)P, (int)ldP, nullptr, c->stream, GEMM_TAG_ENV);
  ok = ok && gemm_rp(mode, OX, ldP, OX, ldP, fmt, c->RA1[0].p,
                     halves == 2 ? c->RA1[1].p : nullptr, o2, (int)P, (int)P, (int)ldP, nullptr,
                     c->stream, GEMM_TAG_ENV);
  const OutMap om = omap2(dx, dx * n, dx, dx, n, 1);
  ok = ok && gemm_rp(mode, op(c->RA2), ldK2, op(c->RA1), ldK2, RP_OUT_F64, c->M.p, nullptr, om,
                     (int)n, (int)n, (int)ldK2, nullptr, c->stream, GEMM_TAG_ENV);
  if (!ok) fail(HOTRG_ERR_INVALID, "reduced-precision environment: unsupported operand shape");
}

// C1, C2, C3 from reduced-precision operands; T~ (FP32) into c->Tt.
void coarse_rp(hotrg_ctx* c, hotrg_state* st, int mode, int dx, int dy, int dn,
               unsigned long long* maxbits) {
  const long long P = (long long)dx * dy, n = (long long)dx * dx;
  const long long ldP = pad32(P), ldx = pad32(dx), ldn = pad32(n);
  const size_t es = mode == RP_F32 ? 4 : 2;
  const int fmt = mode == RP_F32 ? RP_OUT_F32 : RP_OUT_SPLIT;
  const int halves = mode == RP_F32 ? 1 : 2;
  const long long x1rows = (long long)dn * dy * dx, x2rows = (long long)dn * dy * dy;
  for (int h = 0; h < halves; ++h) {
    ensure(c, c->RX1[h], (size_t)x1rows * ldP * es);
    ensure(c, c->RX2[h], (size_t)x2rows * ldn * es);
    if (ldP != P) HIPCHK(hipMemsetAsync(c->RX1[h].p, 0, (size_t)x1rows * ldP * es, c->stream));
    if (ldn != n) HIPCHK(hipMemsetAsync(c->RX2[h].p, 0, (size_t)x2rows * ldn * es, c->stream));
  }
  ensure(c, c->Tt, (size_t)dn * dy * dn * dy * 4);
  auto op = [&](Buf* b) { return RpOperand{b[0].p, halves == 2 ? b[1].p : nullptr}; };
  // C1: rows (i,a): i -> dy*dx*ldP, a -> dy; cols (j,d,c): j -> dx*ldP, d -> ldP, c -> 1
  OutMap o1 = omap2(dx, (long long)dy * dx * ldP, dy, 1, 0, 0);
  o1.c1 = dx;
  o1.c2 = dy;
  o1.t0 = (long long)dx * ldP;
  o1.t1 = ldP;
  o1.t2 = 1;
  mark(c, HOTRG_PHASE_C1);
  bool ok = gemm_rp(mode, op(c->RU1), ldx, op(st->RO[2]), ldx, fmt, c->RX1[0].p,
                    halves == 2 ? c->RX1[1].p : nullptr, o1, dn * dx, dy * dx * dy, (int)ldx,
                    nullptr, c->stream, GEMM_TAG_OTHER);
  // C2: rows (ij,d): ij -> dy*ldn, d -> dx; cols (l,e): l -> ldn, e -> 1
  const OutMap o2 = omap2(dx, (long long)dy * ldn, dx, dx, ldn, 1);
  mark(c, HOTRG_PHASE_C2);
  ok = ok && gemm_rp(mode, op(c->RX1), ldP, op(st->RO[3]), ldP, fmt, c->RX2[0].p,
                     halves == 2 ? c->RX2[1].p : nullptr, o2, (int)x1rows, (int)P, (int)ldP,
                     nullptr, c->stream, GEMM_TAG_C2);
  // C3: rows (ij,l): ij -> dn*dy, l -> 1; cols k -> dy
  mark(c, HOTRG_PHASE_C3);
  launch_store((double*)maxbits, 0.0, c->stream);
  const OutMap o3 = omap2(dy, (long long)dn * dy, 1, 1, dy, 0);
  ok = ok && gemm_rp(mode, op(c->RX2), ldn, op(c->RU3), ldn, RP_OUT_F32, c->Tt.p, nullptr, o3,
                     (int)x2rows, dn, (int)ldn, maxbits, c->stream, GEMM_TAG_OTHER);
  if (!ok) fail(HOTRG_ERR_INVALID, "reduced-precision contraction: unsupported operand shape");
}

// Records and spectra of steps 1..k (device), spectra of spec_len values.
void reserve_records(hotrg_ctx* c, hotrg_state* st, int k, int spec_len) {
  if (k > st->rec_cap) {
    int cap = st->rec_cap ? 2 * st->rec_cap : 64;
    while (cap < k) cap *= 2;
    ensure_keep(c, st->recs, (size_t)cap * kRec * 8, (size_t)st->rec_cap * kRec * 8);
    if (st->spec_len)
      ensure_keep(c, st->spec, (size_t)cap * st->spec_len * 8, (size_t)st->rec_cap * st->spec_len * 8);
    st->rec_cap = cap;
  }
  if (spec_len != st->spec_len) {
    if (st->k > 0 && st->spec_len != 0)
      fail(HOTRG_ERR_INVALID, "spec_len must not change between steps of one state");
    st->spec_len = spec_len;
    if (st->spec_len) ensure(c, st->spec, (size_t)st->rec_cap * st->spec_len * 8);
  }
}

// Block size of the iterative eigensolve for d_new leading pairs of an n x n
// environment; whether it applies (else the dense solver runs: the two-launch
// one up to n = 128, rocSOLVER above, where a block of p >= need + 16 vectors
// would exceed half of n).
static bool eig_block(int n, int dn, int spec_len, int eig_mode, int* need_out, int* p_out) {
  const int need = std::max(dn + 1, std::min(spec_len, n));
  int p = std::min(128, std::max(2 * dn, need + 16));
  p = (p + 15) / 16 * 16;
  *need_out = need;
  *p_out = p;
  return eig_mode == HOTRG_EIG_AUTO && n > 128 && need + 16 <= p && p <= 128 && p * 2 <= n;
}

// Leading eigenpairs of the symmetric n x n matrix in Mb: eigenvalues
// (ascending) into Wb, eigenvector rows into Xb (p rows, iterative) or over Mb
// (n rows, dense); returns the rows and their count.  A non-converged dense
// solve is folded into *sticky; an iterative one that does not converge falls
// back to the dense solver.
static const double* leading_eigs(hotrg_ctx* c, Buf& Mb, Buf& Wb, Buf& Xb, int n, int need, int p,
                                  bool sub_ok, EigHint& h, int* inf, int* sticky, int* cols_out,
                                  double tol = 5e-14) {
  ensure(c, Wb, (size_t)n * 8);
  if (sub_ok) {
    ensure(c, c->EW, topk_workspace_doubles(n, p) * 8);
    ensure(c, Xb, (size_t)p * n * 8);
    int iters = 0, enough = 0;
    double resid = 0.0;
    // solves of the same kind: start with one sweep more than the last one
    // is estimated to have needed, at its shift
    const int q_first = h.n == n ? h.sweeps + 1 : 3;
    if (h.n != n) {
      h.shift = 0.0;
      h.nocheck = 0;
    }
    const bool ok = topk_eigs((const double*)Mb.p, n, p, need, tol, q_first, &h.shift,
                              &h.nocheck, (double*)c->EW.p, (double*)Wb.p, (double*)Xb.p,
                              (int*)((char*)c->scal.p + 48), &iters, &enough, &resid, c->stream);
    h.n = ok ? n : 0;
    h.sweeps = enough;
    c->last_eig_iters = ok ? iters : 0;
    c->last_eig_resid = resid;
    if (ok) {
      *cols_out = p;
      return (const double*)Xb.p;
    }
  }
  ensure(c, c->E, (size_t)n * 8);
  c->last_eig_iters = 0;  // dense
  // small environments: two single-workgroup launches (Householder reduction,
  // divide and conquer with the back-transform); larger ones rocSOLVER dsyevd
  if (!dense_eig_small((double*)Mb.p, n, (double*)Wb.p, (double*)c->E.p, inf, c->stream)) {
    rocblas_status rs = rocsolver_dsyevd(c->blas, rocblas_evect_original, rocblas_fill_lower, n,
                                         (double*)Mb.p, n, (double*)Wb.p, (double*)c->E.p, inf);
    if (rs != rocblas_status_success)
      fail(HOTRG_ERR_DEVICE, "rocsolver_dsyevd failed with status " + std::to_string((int)rs));
  }
  // a non-converged solve marks the caller's flag: later solves overwrite `inf`
  launch_fold_info(inf, sticky, 0, c->stream);
  *cols_out = n;
  return (const double*)Mb.p;
}

void do_step(hotrg_ctx* c, hotrg_state* st, const hotrg_opts* o) {
  const int dx = st->dx, dy = st->dy;
  const int n = dx * dx;
  const int dn = o->d_cut < n ? o->d_cut : n;
  check_dims(dx, dy, dn);
  const int k = st->k + 1;
  reserve_records(c, st, k, o->spec_len);
  double* rec = (double*)st->recs.p + kRec * (size_t)(k - 1);
  double* spec = st->spec_len ? (double*)st->spec.p + (size_t)(k - 1) * st->spec_len : nullptr;
  ensure(c, c->scal, 64);
  unsigned long long* mb = (unsigned long long*)c->scal.p;
  int* info = (int*)((char*)c->scal.p + 8);
  int* kept = (int*)((char*)c->scal.p + 16);
  unsigned long long* one = (unsigned long long*)((char*)c->scal.p + 56);
  int* st_fail = (int*)((char*)st->acc.p + 8);

  const int sp = step_precision(st, k, dx, dy, o->d_cut);
  if (sp != st->ops_prec) {
    // operands were prepared for another precision (d_cut changed): rebuild
    const unsigned long long one_bits = 0x3ff0000000000000ULL;
    HIPCHK(hipMemcpyAsync(one, &one_bits, 8, hipMemcpyHostToDevice, c->stream));
    const size_t ne = (size_t)dx * dy * dx * dy;
    Buf tmp;
    ensure(c, tmp, ne * (st->cur_f32 ? 4 : 8));
    HIPCHK(hipMemcpyAsync(tmp.p, st->cur_f32 ? st->Tn32.p : st->Tn.p, ne * (st->cur_f32 ? 4 : 8),
                          hipMemcpyDeviceToDevice, c->stream));
    const bool f32 = st->cur_f32;
    prepare_operands(c, st, sp, tmp.p, f32, false, dx, dy, one);
    HIPCHK(hipStreamSynchronize(c->stream));
    ctx_free(c, tmp);
  }

  c->m_step = k;
  c->m_dx = dx;
  c->m_dy = dy;
  c->m_dn = dn;
  mark(c, HOTRG_PHASE_ENV);
  // environment M (FP64 out)
  if (sp == HOTRG_FP64)
    environment_f64(c, (const double*)st->Tn.p, (const double*)st->Xt.p, dx, dy);
  else
    environment_rp(c, st, rp_mode(sp), dx, dy);
  launch_symmetrize((double*)c->M.p, n, c->stream);
  // FP64 eigendecomposition, spectrum and projector
  ensure(c, c->E, (size_t)n * 8);
  double* trace = (double*)((char*)c->scal.p + 40);
  launch_trace((const double*)c->M.p, n, trace, c->stream);
  mark(c, HOTRG_PHASE_EIGH);
  // leading eigenpairs: block subspace iteration when D' is small against n
  int need = 0, p = 0;
  const bool sub_ok = eig_block(n, dn, o->spec_len, o->eig, &need, &p);
  auto solve = [&](Buf& Mb, Buf& Wb, Buf& Xb, int side, int* inf, int* cols_out) {
    return leading_eigs(c, Mb, Wb, Xb, n, need, p, sub_ok, st->eig[(st->k & 1) + 2 * side], inf,
                        st_fail, cols_out, eig_tolerance(sp));
  };
  int cols = n;
  const double* evec = solve(c->M, c->W, c->Xr, 0, info, &cols);
  if (k == c->test_fail_step) launch_fold_info(info, st_fail, 1, c->stream);
  mark(c, HOTRG_PHASE_PROJ);
  launch_spectrum((const double*)c->W.p, cols, n, dn, o->trunc, o->degen_tol, st->spec_len,
                  trace, spec, rec, kept, c->stream);
  launch_store(rec + 5, 0.0, c->stream);
  if (o->isometry == HOTRG_ISO_TWO_SIDED && dn < n) {
    // the right pair of legs: environment of the reflected tensor (FP64)
    if (sp != HOTRG_FP64) fail(HOTRG_ERR_INVALID, "two-sided isometry needs FP64 contractions");
    const size_t ne = (size_t)dx * dy * dx * dy;
    ensure(c, c->Tm, ne * 8);
    ensure(c, c->Xm, ne * 8);
    ensure(c, c->Side, (size_t)(kRec + 3 + st->spec_len) * 8);
    double* rec2 = (double*)c->Side.p;
    int* kept2 = (int*)(rec2 + kRec);
    double* trace2 = rec2 + kRec + 1;
    int* info2 = (int*)(rec2 + kRec + 2);
    double* spec2 = st->spec_len ? rec2 + kRec + 3 : nullptr;
    mark(c, HOTRG_PHASE_ENV);
    launch_prep_mirror((const double*)st->Tn.p, dx, dy, (double*)c->Tm.p, (double*)c->Xm.p,
                       c->stream);
    environment_f64(c, (const double*)c->Tm.p, (const double*)c->Xm.p, dx, dy, &c->M2);
    launch_symmetrize((double*)c->M2.p, n, c->stream);
    launch_trace((const double*)c->M2.p, n, trace2, c->stream);
    mark(c, HOTRG_PHASE_EIGH);
    int cols2 = n;
    const double* evec2 = solve(c->M2, c->W2, c->Xr2, 1, info2, &cols2);
    mark(c, HOTRG_PHASE_PROJ);
    launch_spectrum((const double*)c->W2.p, cols2, n, dn, o->trunc, o->degen_tol, st->spec_len,
                    trace2, spec2, rec2, kept2, c->stream);
    double errs[2] = {0.0, 0.0};
    int sticky = 0;
    HIPCHK(hipMemcpyAsync(&errs[0], rec + 1, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(&errs[1], rec2 + 1, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(&sticky, st_fail, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    // both solves of this step (and every earlier one) are folded into the flag
    if (sticky != 0) fail(HOTRG_ERR_NUMERIC, "eigensolver did not converge");
    if (errs[1] < errs[0] - kSideMargin) {
      HIPCHK(hipMemcpyAsync(rec, rec2, 5 * 8, hipMemcpyDeviceToDevice, c->stream));
      HIPCHK(hipMemcpyAsync(kept, kept2, sizeof(int), hipMemcpyDeviceToDevice, c->stream));
      if (spec)
        HIPCHK(hipMemcpyAsync(spec, spec2, (size_t)st->spec_len * 8, hipMemcpyDeviceToDevice,
                              c->stream));
      launch_store(rec + 5, 1.0, c->stream);
      evec = evec2;
      cols = cols2;
    }
  }
  ensure(c, c->Ucan, (size_t)n * dn * 8);
  launch_isometry(evec, cols, n, dn, kept, (double*)c->Ucan.p, c->stream);
  if (sp == HOTRG_FP64) {
    ensure(c, c->U1, (size_t)n * dn * 8);
    ensure(c, c->U3, (size_t)n * dn * 8);
    launch_layout_u((const double*)c->Ucan.p, dx, dn, c->U1.p, c->U3.p, false, c->stream);
    // the three contractions, max|T~|
    coarse_f64(c, (const double*)st->Tn.p, (const double*)st->Tp.p, (const double*)c->U1.p,
               (const double*)c->U3.p, dx, dy, dn, mb);
  } else {
    const int mode = rp_mode(sp);
    const size_t es = mode == RP_F32 ? 4 : 2;
    const long long ldx = pad32(dx), ldn = pad32(n);
    for (int h = 0; h < (mode == RP_F32 ? 1 : 2); ++h) {
      ensure(c, c->RU1[h], (size_t)dn * dx * ldx * es);
      ensure(c, c->RU3[h], (size_t)dn * ldn * es);
      if (ldx != dx) HIPCHK(hipMemsetAsync(c->RU1[h].p, 0, (size_t)dn * dx * ldx * es, c->stream));
      if (ldn != n) HIPCHK(hipMemsetAsync(c->RU3[h].p, 0, (size_t)dn * ldn * es, c->stream));
    }
    launch_layout_u_rp((const double*)c->Ucan.p, dx, dn, mode, c->RU1[0].p,
                       mode == RP_F32 ? nullptr : c->RU1[1].p, c->RU3[0].p,
                       mode == RP_F32 ? nullptr : c->RU3[1].p, ldx, ldn, c->stream);
    coarse_rp(c, st, mode, dx, dy, dn, mb);
  }
  // ln n_k, torus estimate; operands of the next step (legs transposed)
  mark(c, HOTRG_PHASE_NORM);
  const bool tt_f32 = sp != HOTRG_FP64;
  launch_norm(mb, c->Tt.p, tt_f32, dn, dy, std::ldexp(1.0, -k), (double*)st->acc.p, rec, c->stream);
  const int ndx = dy, ndy = dn;
  const int nsp = step_precision(st, k + 1, ndx, ndy, o->d_cut);
  prepare_operands(c, st, nsp, c->Tt.p, tt_f32, true, ndx, ndy, mb);
  mark(c, -1);
  HIPCHK(hipGetLastError());
  if (sp != HOTRG_FP64) st->err_bound += kErrPerStep[sp] * std::ldexp(1.0, -k);
  st->dx = ndx;
  st->dy = ndy;
  st->k = k;
}

void fetch_info(hotrg_ctx* c, hotrg_state* st, int first, int count, const int* dims_dx,
                hotrg_step_info* out, double* spectra) {
  // dims are reconstructed by the caller; records come from the device
  std::vector<double> r((size_t)count * kRec);
  if (count == 0) return;
  HIPCHK(hipMemcpyAsync(r.data(), (double*)st->recs.p + kRec * (size_t)first, r.size() * 8,
                        hipMemcpyDeviceToHost, c->stream));
  if (spectra && st->spec_len)
    HIPCHK(hipMemcpyAsync(spectra, (double*)st->spec.p + (size_t)first * st->spec_len,
                          (size_t)count * st->spec_len * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (out)
    for (int i = 0; i < count; ++i) {
      out[i].log_norm = r[kRec * i + 0];
      out[i].trunc_err = r[kRec * i + 1];
      out[i].cut_gap = r[kRec * i + 2];
      out[i].lnz_torus = r[kRec * i + 3];
      out[i].kept = (int)r[kRec * i + 4];
      out[i].side = (int)r[kRec * i + 5];
    }
  (void)dims_dx;
}

// The state's sticky flag: set if the eigensolve of any step so far failed.
void check_info(hotrg_ctx* c, const hotrg_state* st) {
  int flag = 0;
  HIPCHK(hipMemcpyAsync(&flag, (const char*)st->acc.p + 8, sizeof(int), hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (flag != 0) fail(HOTRG_ERR_NUMERIC, "eigensolver did not converge in an earlier step");
}

std::vector<double> build_tensor(const hotrg_model_params* p, int* dx, int* dy) {
  if (!p) fail(HOTRG_ERR_INVALID, "params is NULL");
  try {
    switch (p->model) {
      case HOTRG_ISING:
        *dx = *dy = 2;
        return ising_tensor(p->beta, p->J);
      case HOTRG_XY:
        *dx = *dy = 2 * p->n_max + 1;
        return xy_tensor(p->beta, p->n_max);
      case HOTRG_POTTS:
        *dx = *dy = p->q;
        return potts_tensor(p->beta, p->q);
      case HOTRG_GXY:
        *dx = *dy = 2 * p->n_max + 1;
        return gxy_tensor(p->beta, p->delta, p->n_max);
      case HOTRG_RAW: {
        if (!p->raw || p->raw_dx < 1 || p->raw_dy < 1 || p->raw_dx > 128 || p->raw_dy > 16384)
          fail(HOTRG_ERR_INVALID, "raw tensor: need raw != NULL, 1 <= raw_dx <= 128, raw_dy >= 1");
        *dx = p->raw_dx;
        *dy = p->raw_dy;
        size_t ne = (size_t)p->raw_dx * p->raw_dy * p->raw_dx * p->raw_dy;
        return std::vector<double>(p->raw, p->raw + ne);
      }
      default:
        fail(HOTRG_ERR_INVALID, "unknown model");
    }
  } catch (const std::invalid_argument& e) {
    fail(HOTRG_ERR_INVALID, e.what());
  }
}

template <class F>
hotrg_status guard(F&& f) {
  try {
    f();
    return HOTRG_OK;
  } catch (const Error& e) {
    g_err = e.msg;
    return e.st;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return HOTRG_ERR_OOM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return HOTRG_ERR_DEVICE;
  }
}

}  // namespace

namespace {

// ------------------------------------------------------ lockstep batches --
// hotrg_run_grouped: the problems of a batch take their steady-state steps
// together, each phase one launch over all of them (grouped GEMMs over a
// device table of products, batched eigensolver and bookkeeping kernels), and
// the whole sweep is captured once as a HIP graph and replayed.

constexpr int kGroupRounds = 9;          // Rayleigh-Ritz checks per step
constexpr int kGroupSweepsPerRound = 4;  // subspace sweeps before each check

struct GProb {
  int idx = 0;          // position in the caller's arrays
  hotrg_opts o{};       // options with the precision resolved
  hotrg_state* st = nullptr;
  std::vector<int> dxs, dys, dns;
  int D = 0, n = 0, p = 0, need = 0, sp = HOTRG_FP64;  // steady dims, block size, precision
  bool dense = false;  // environment diagonalised whole (n <= 128) instead of a block
  Buf M, eig, U, scal, Tt, U1, U3;
  Buf RA1[2], RA2[2], RX1[2], RX2[2], RU1[2], RU3[2];
  GroupCtl* ctl = nullptr;  // device
  int k_host = 0;           // steps done, as the host counts them
  double t0 = 0.0;
};

struct GTable {  // a grouped launch's device table
  char* items = nullptr;
  int* begin[3] = {nullptr, nullptr, nullptr};  // per tile configuration (reduced precision)
  int count = 0, tiles[3] = {0, 0, 0};
};

struct GRun {
  std::vector<GProb*> act;
  bool dense = false;  // all problems' environments diagonalised whole
  int sp = HOTRG_FP64, mode = RP_F32, pmax = 16;
  long long max_pn = 1;
  GroupStep* steps = nullptr;
  CholItem* chol = nullptr;
  // eigensolver products
  GTable vm, gramY, gramT2, apYT2, apT2V, apT2Y, apYV, rrH, rrX, rrYx;
  // reduced-precision contractions and their tile configuration
  GTable halves, combine, c1, c2, c3;
  int cfg[5] = {-1, -1, -1, -1, -1};
};

void launch_f64_table(const GTable& t, int bl, hipStream_t s) {
  gemm_f64_grouped(bl, (const F64Item*)t.items, t.begin[0], t.count, t.tiles[0], s);
}

void launch_rp_table(const GTable& t, int mode, int out, int cfg, hipStream_t s) {
  gemm_rp_grouped(mode, out, cfg, (const RpItem*)t.items, t.begin[cfg], t.count, t.tiles[cfg], s);
}

// tile configurations chosen for grouped reduced-precision launches, by the
// shapes of their products (the tuner of the lockstep engine)
std::mutex g_gtune_mu;
std::map<std::vector<long long>, int> g_gtune;

std::vector<long long> table_key(int mode, int op, const std::vector<RpItem>& items) {
  std::vector<long long> k = {mode, op};
  for (const RpItem& it : items) {
    k.push_back(it.M);
    k.push_back(it.N);
    k.push_back(it.K);
  }
  return k;
}

// One steady sweep of every active problem (captured or eager).  With
// `tune`, each grouped reduced-precision launch without a recorded tile
// configuration times the three candidates first (they all write the same
// products; C3's max is idempotent).
void group_sweep(hotrg_ctx* c, GRun& R, bool tune, std::vector<std::vector<long long>>* keys) {
  hipStream_t s = c->stream;
  const int G = (int)R.act.size();
  const bool red = R.sp != HOTRG_FP64;
  const int split = R.mode == RP_BF16X3;
  // environment M of every problem
  if (red) {
    const int outs[2] = {split ? RP_OUT_SPLIT : RP_OUT_F32, RP_OUT_F64};
    GTable* tabs[2] = {&R.halves, &R.combine};
    for (int q = 0; q < 2; ++q) {
      if (tune && R.cfg[q] < 0) {
        hipEvent_t a, b;
        HIPCHK(hipEventCreate(&a));
        HIPCHK(hipEventCreate(&b));
        float best = 0.f;
        for (int cf = 0; cf < 3; ++cf) {
          float ms = 0.f;
          for (int rep = 0; rep < 2; ++rep) {
            HIPCHK(hipEventRecord(a, s));
            launch_rp_table(*tabs[q], R.mode, outs[q], cf, s);
            HIPCHK(hipEventRecord(b, s));
            HIPCHK(hipEventSynchronize(b));
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, a, b));
            ms = rep == 0 ? t : std::min(ms, t);
          }
          if (R.cfg[q] < 0 || ms < best) {
            best = ms;
            R.cfg[q] = cf;
          }
        }
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        std::lock_guard<std::mutex> lk(g_gtune_mu);
        g_gtune[(*keys)[q]] = R.cfg[q];
      }
      launch_rp_table(*tabs[q], R.mode, outs[q], R.cfg[q], s);
    }
  } else {
    for (GProb* g : R.act)
      environment_f64(c, (const double*)g->st->Tn.p, (const double*)g->st->Xt.p, g->D, g->D, &g->M);
  }
  for (GProb* g : R.act) {
    launch_symmetrize((double*)g->M.p, g->n, s);
    launch_trace((const double*)g->M.p, g->n, (double*)((char*)g->scal.p + 8), s);
  }
  // leading eigenpairs: block subspace iteration with a fixed budget (its
  // Rayleigh-Ritz matrices by tridiagonal divide and conquer), or the whole
  // (small) environment by the same divide and conquer
  group_begin(R.steps, G, s);
  if (R.dense) group_dense(R.steps, G, R.pmax, s);
  if (!R.dense) group_seed(R.steps, G, R.max_pn, s);
  auto pass = [&](const GTable& gram, int ps, bool full, const GTable& apply) {
    launch_f64_table(gram, B_KCONTIG, s);
    launch_chol_inv_batched(R.chol, G, R.pmax, ps, full, s);
    launch_f64_table(apply, B_NCONTIG, s);
  };
  for (int round = 0; round < (R.dense ? 0 : kGroupRounds); ++round) {
    for (int sw = 0; sw < kGroupSweepsPerRound; ++sw) {
      const bool full = sw == kGroupSweepsPerRound - 1;
      launch_f64_table(R.vm, B_NCONTIG, s);  // Y = V M
      group_shift(R.steps, G, R.max_pn, s);  // Y -= sigma V
      pass(R.gramY, 0, full, R.apYT2);
      if (full) {
        pass(R.gramT2, 1, full, R.apT2Y);
        pass(R.gramY, 2, full, R.apYV);
      } else {
        pass(R.gramT2, 1, full, R.apT2V);
      }
    }
    launch_f64_table(R.vm, B_NCONTIG, s);    // Y = V M
    launch_f64_table(R.rrH, B_KCONTIG, s);   // H = V Y^T
    group_symm_h(R.steps, G, s);
    group_sytrd(R.steps, G, R.pmax, s);      // H -> Q^T, tridiagonal into W, G
    group_stedc(R.steps, G, R.pmax, s);      // H <- Z^T, W ascending
    launch_f64_table(R.rrX, B_NCONTIG, s);   // X = Z^T V
    launch_f64_table(R.rrYx, B_NCONTIG, s);  // Yx = Z^T Y
    group_resid(R.steps, G, round == kGroupRounds - 1, s);
    if (round + 1 < kGroupRounds) group_restart(R.steps, G, R.max_pn, s);
  }
  // projector
  group_spectrum(R.steps, G, s);
  for (GProb* g : R.act) {
    const int* kept = (const int*)((char*)g->scal.p + 16);
    launch_isometry((const double*)((double*)g->eig.p + 4LL * g->p * g->n), g->p, g->n, g->D, kept,
                    (double*)g->U.p, s);
    if (red) {
      const long long ldx = pad32(g->D), ldn = pad32(g->n);
      launch_layout_u_rp((const double*)g->U.p, g->D, g->D, R.mode, g->RU1[0].p,
                         split ? g->RU1[1].p : nullptr, g->RU3[0].p, split ? g->RU3[1].p : nullptr,
                         ldx, ldn, s);
    } else {
      launch_layout_u((const double*)g->U.p, g->D, g->D, g->U1.p, g->U3.p, false, s);
    }
  }
  // the three contractions, max|T~|
  if (red) {
    group_zero_max(R.steps, G, s);
    GTable* tabs[3] = {&R.c1, &R.c2, &R.c3};
    const int outs[3] = {split ? RP_OUT_SPLIT : RP_OUT_F32, split ? RP_OUT_SPLIT : RP_OUT_F32,
                         RP_OUT_F32};
    for (int q = 0; q < 3; ++q) {
      if (tune && R.cfg[2 + q] < 0) {
        hipEvent_t a, b;
        HIPCHK(hipEventCreate(&a));
        HIPCHK(hipEventCreate(&b));
        float best = 0.f;
        for (int cf = 0; cf < 3; ++cf) {
          float ms = 0.f;
          for (int rep = 0; rep < 2; ++rep) {
            HIPCHK(hipEventRecord(a, s));
            launch_rp_table(*tabs[q], R.mode, outs[q], cf, s);
            HIPCHK(hipEventRecord(b, s));
            HIPCHK(hipEventSynchronize(b));
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, a, b));
            ms = rep == 0 ? t : std::min(ms, t);
          }
          if (R.cfg[2 + q] < 0 || ms < best) {
            best = ms;
            R.cfg[2 + q] = cf;
          }
        }
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        std::lock_guard<std::mutex> lk(g_gtune_mu);
        g_gtune[(*keys)[2 + q]] = R.cfg[2 + q];
      }
      launch_rp_table(*tabs[q], R.mode, outs[q], R.cfg[2 + q], s);
    }
  } else {
    for (GProb* g : R.act)
      coarse_f64_into(c, (const double*)g->st->Tn.p, (const double*)g->st->Tp.p,
                      (const double*)g->U1.p, (const double*)g->U3.p, g->D, g->D, g->D,
                      (double*)c->X1.p, (double*)c->X2.p, (double*)g->Tt.p,
                      (unsigned long long*)g->scal.p, 0);  // shapes tuned by the eager sweep
  }
  // ln n_k, torus estimate; operands of the next step (legs transposed)
  group_norm(R.steps, G, s);
  for (GProb* g : R.act) {
    const unsigned long long* mb = (const unsigned long long*)g->scal.p;
    if (red) {
      RpOps ops;
      for (int i = 0; i < 4; ++i) {
        ops.hi[i] = g->st->RO[i][0].p;
        ops.lo[i] = split ? g->st->RO[i][1].p : nullptr;
      }
      launch_prep_rp(g->Tt.p, true, true, g->D, g->D, mb, (float*)g->st->Tn32.p, R.mode, ops,
                     pad32((long long)g->D * g->D), pad32(g->D), s);
    } else {
      launch_prep(g->Tt.p, false, true, g->D, g->D, mb, g->st->Tn.p, g->st->Xt.p, g->st->Tp.p,
                  false, s);
    }
  }
  group_advance(R.steps, G, s);
}

// Device tables of the active problems (items ordered as R.act).
void group_tables(hotrg_ctx* c, GRun& R, Buf& store, std::vector<std::vector<long long>>* keys) {
  const int G = (int)R.act.size();
  std::vector<char> host;
  auto put = [&](const void* p, size_t bytes) {
    const size_t off = (host.size() + 255) / 256 * 256;
    host.resize(off + bytes);
    std::memcpy(host.data() + off, p, bytes);
    return off;
  };
  struct Pending {
    GTable* t;
    size_t items;
    size_t begin[3];
  };
  std::vector<Pending> pend;
  auto f64tab = [&](GTable& t, auto make) {
    std::vector<F64Item> it;
    std::vector<int> b(1, 0);
    for (GProb* g : R.act) {
      it.push_back(make(g));
      b.push_back(b.back() + f64_group_tiles(it.back()));
    }
    t.count = G;
    t.tiles[0] = b.back();
    b.pop_back();
    pend.push_back({&t, put(it.data(), it.size() * sizeof(F64Item)),
                    {put(b.data(), b.size() * sizeof(int)), 0, 0}});
  };
  auto rptab = [&](GTable& t, const std::vector<RpItem>& it, int op) {
    Pending pe{&t, put(it.data(), it.size() * sizeof(RpItem)), {0, 0, 0}};
    for (int cf = 0; cf < 3; ++cf) {
      std::vector<int> b(1, 0);
      for (const RpItem& x : it) b.push_back(b.back() + rp_group_tiles(x, cf));
      t.tiles[cf] = b.back();
      b.pop_back();
      pe.begin[cf] = put(b.data(), b.size() * sizeof(int));
    }
    t.count = (int)it.size();
    pend.push_back(pe);
    keys->push_back(table_key(R.mode, op, it));
  };
  // descriptors
  std::vector<GroupStep> st;
  std::vector<CholItem> ch;
  for (GProb* g : R.act) {
    const long long pn = (long long)g->p * g->n, pp = (long long)g->p * g->p;
    double* e = (double*)g->eig.p;
    GroupStep d{};
    d.ctl = g->ctl;
    d.n = g->n;
    d.dn = g->D;
    d.dy = g->D;
    d.p = g->p;
    d.need = g->need;
    d.trunc = g->o.trunc;
    d.spec_len = g->st->spec_len;
    d.K = g->o.n_steps;
    d.tau = g->o.degen_tol;
    d.tol = eig_tolerance(R.sp);  // residual tolerance (as do_step's solver)
    d.M = (const double*)g->M.p;
    d.V = e;
    d.Y = e + pn;
    d.T2 = e + 2 * pn;
    d.Yx = e + 3 * pn;
    d.X = e + 4 * pn;
    d.G = e + 5 * pn;
    d.Rt = d.G + pp;
    d.H = d.Rt + pp;
    d.W = d.H + pp;
    d.res = d.W + g->p;
    d.trace = (double*)((char*)g->scal.p + 8);
    d.kept = (int*)((char*)g->scal.p + 16);
    d.maxbits = (unsigned long long*)g->scal.p;
    d.shift = (double*)((char*)g->scal.p + 64);
    d.recs = (double*)g->st->recs.p;
    d.spec = (double*)g->st->spec.p;
    d.acc = (double*)g->st->acc.p;
    d.Tt = g->Tt.p;
    d.tt_f32 = R.sp != HOTRG_FP64;
    st.push_back(d);
    CholItem ci{d.G, d.Rt, &g->ctl->fail, &g->ctl->iter, g->p,
                11.0 * ((double)g->n * g->p + (double)g->p * (g->p + 1)) * std::ldexp(1.0, -53)};
    ch.push_back(ci);
  }
  const size_t o_steps = put(st.data(), st.size() * sizeof(GroupStep));
  const size_t o_chol = put(ch.data(), ch.size() * sizeof(CholItem));
  auto stp = [&](GProb* g) {
    for (size_t i = 0; i < R.act.size(); ++i)
      if (R.act[i] == g) return st[i];
    return st[0];
  };
  auto item = [&](const double* A, long long lda, const double* B, long long ldb, double* C,
                  long long ldc, int M, int N, int K, GProb* g) {
    return F64Item{A, lda, B, ldb, C, ldc, M, N, K, &g->ctl->iter};
  };
  f64tab(R.vm, [&](GProb* g) { auto d = stp(g); return item(d.V, g->n, (const double*)g->M.p, g->n, d.Y, g->n, g->p, g->n, g->n, g); });
  f64tab(R.gramY, [&](GProb* g) { auto d = stp(g); return item(d.Y, g->n, d.Y, g->n, d.G, g->p, g->p, g->p, g->n, g); });
  f64tab(R.gramT2, [&](GProb* g) { auto d = stp(g); return item(d.T2, g->n, d.T2, g->n, d.G, g->p, g->p, g->p, g->n, g); });
  f64tab(R.apYT2, [&](GProb* g) { auto d = stp(g); return item(d.Rt, g->p, d.Y, g->n, d.T2, g->n, g->p, g->n, g->p, g); });
  f64tab(R.apT2V, [&](GProb* g) { auto d = stp(g); return item(d.Rt, g->p, d.T2, g->n, d.V, g->n, g->p, g->n, g->p, g); });
  f64tab(R.apT2Y, [&](GProb* g) { auto d = stp(g); return item(d.Rt, g->p, d.T2, g->n, d.Y, g->n, g->p, g->n, g->p, g); });
  f64tab(R.apYV, [&](GProb* g) { auto d = stp(g); return item(d.Rt, g->p, d.Y, g->n, d.V, g->n, g->p, g->n, g->p, g); });
  f64tab(R.rrH, [&](GProb* g) { auto d = stp(g); return item(d.V, g->n, d.Y, g->n, d.H, g->p, g->p, g->p, g->n, g); });
  f64tab(R.rrX, [&](GProb* g) { auto d = stp(g); return item(d.H, g->p, d.V, g->n, d.X, g->n, g->p, g->n, g->p, g); });
  f64tab(R.rrYx, [&](GProb* g) { auto d = stp(g); return item(d.H, g->p, d.Y, g->n, d.Yx, g->n, g->p, g->n, g->p, g); });
  if (R.sp != HOTRG_FP64) {
    const bool split = R.mode == RP_BF16X3;
    auto op = [&](const Buf* b) { return RpOperand{b[0].p, split ? b[1].p : nullptr}; };
    std::vector<RpItem> hv, cb, i1, i2, i3;
    for (GProb* g : R.act) {
      const long long D = g->D, P = D * D, n = g->n, ldP = pad32(P), ldK2 = pad32(D * D),
                      ldx = pad32(D), ldn = pad32(n);
      const int* gate = &g->ctl->active;
      const OutMap oh = omap2((int)D, D * ldK2, D, (int)D, ldK2, 1);
      hv.push_back(RpItem{op(g->st->RO[0]), ldP, op(g->st->RO[0]), ldP, g->RA2[0].p,
                          split ? g->RA2[1].p : nullptr, oh, (int)P, (int)P, (int)ldP, nullptr,
                          gate});
      hv.push_back(RpItem{op(g->st->RO[1]), ldP, op(g->st->RO[1]), ldP, g->RA1[0].p,
                          split ? g->RA1[1].p : nullptr, oh, (int)P, (int)P, (int)ldP, nullptr,
                          gate});
      const OutMap om = omap2((int)D, D * n, D, (int)D, n, 1);
      cb.push_back(RpItem{op(g->RA2), ldK2, op(g->RA1), ldK2, g->M.p, nullptr, om, (int)n, (int)n,
                          (int)ldK2, nullptr, gate});
      OutMap o1 = omap2((int)D, D * D * ldP, D, 1, 0, 0);
      o1.c1 = (int)D;
      o1.c2 = (int)D;
      o1.t0 = D * ldP;
      o1.t1 = ldP;
      o1.t2 = 1;
      i1.push_back(RpItem{op(g->RU1), ldx, op(g->st->RO[2]), ldx, g->RX1[0].p,
                          split ? g->RX1[1].p : nullptr, o1, (int)(D * D), (int)(D * D * D),
                          (int)ldx, nullptr, gate});
      const OutMap o2 = omap2((int)D, D * ldn, D, (int)D, ldn, 1);
      i2.push_back(RpItem{op(g->RX1), ldP, op(g->st->RO[3]), ldP, g->RX2[0].p,
                          split ? g->RX2[1].p : nullptr, o2, (int)(D * D * D), (int)P, (int)ldP,
                          nullptr, gate});
      const OutMap o3 = omap2((int)D, D * D, 1, 1, D, 0);
      i3.push_back(RpItem{op(g->RX2), ldn, op(g->RU3), ldn, g->Tt.p, nullptr, o3,
                          (int)(D * D * D), (int)D, (int)ldn, (unsigned long long*)g->scal.p,
                          gate});
    }
    rptab(R.halves, hv, 0);
    rptab(R.combine, cb, 1);
    rptab(R.c1, i1, 2);
    rptab(R.c2, i2, 3);
    rptab(R.c3, i3, 4);
  }
  // the tables are rewritten only when nothing on the stream reads them: a
  // replay still in flight would index the new, smaller tables with the old
  // grid sizes
  HIPCHK(hipStreamSynchronize(c->stream));
  ensure(c, store, host.size());
  HIPCHK(hipMemcpyAsync(store.p, host.data(), host.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  char* base = (char*)store.p;
  R.steps = (GroupStep*)(base + o_steps);
  R.chol = (CholItem*)(base + o_chol);
  for (const Pending& pe : pend) {
    pe.t->items = base + pe.items;
    for (int cf = 0; cf < 3; ++cf) pe.t->begin[cf] = (int*)(base + pe.begin[cf]);
  }
  R.pmax = 16;
  R.max_pn = 1;
  for (GProb* g : R.act) {
    R.pmax = std::max(R.pmax, g->p);
    R.max_pn = std::max(R.max_pn, (long long)g->p * g->n);
  }
}

}  // namespace

namespace {

// Step (1-based) from which a problem's steps keep the same dims and the same
// contraction precision, or n_steps + 1 if that never happens within the run.
int steady_step(const hotrg_opts& o, int prec, int dx, int dy, int first_reduced) {
  for (int k = 1; k <= o.n_steps; ++k) {
    const int dn = (int)std::min<long long>(o.d_cut, (long long)dx * dx);
    // dims (D, D, D) repeat from here on; a reduced precision also has to have
    // started (steps before first_reduced are FP64)
    if (dx == dy && dy == dn && (prec == HOTRG_FP64 || k >= first_reduced)) return k;
    const int ndx = dy;
    dy = dn;
    dx = ndx;
  }
  return o.n_steps + 1;
}

void free_group_buffers(hotrg_ctx* c, GProb& g) {
  Buf* bs[] = {&g.M, &g.eig, &g.U, &g.scal, &g.Tt, &g.U1, &g.U3};
  for (Buf* b : bs) ctx_free(c, *b);
  for (Buf* arr : {g.RA1, g.RA2, g.RX1, g.RX2, g.RU1, g.RU3})
    for (int h = 0; h < 2; ++h) ctx_free(c, arr[h]);
}

// ln Z / N and the per-step records of a finished state into res.
void finish_into(hotrg_ctx* c, hotrg_state* st, const GProb& g, hotrg_result* res, double secs) {
  double lnz = 0;
  hotrg_status fs = hotrg_finish(c, st, &lnz);
  if (fs != HOTRG_OK) fail(fs, g_err);
  const int K = g.o.n_steps;
  if (res->steps || res->spectra) {
    fetch_info(c, st, 0, K, nullptr, res->steps, res->spectra);
    if (res->steps)
      for (int k = 0; k < K; ++k) {
        res->steps[k].dx = g.dxs[k];
        res->steps[k].dy = g.dys[k];
        res->steps[k].d_new = g.dns[k];
      }
  }
  res->lnz_per_site = lnz;
  res->n_steps = K;
  res->prec_used = g.o.prec;
  res->err_bound = st->err_bound;
  res->seconds = secs;
}

void run_grouped_impl(hotrg_ctx* c, int N, const hotrg_model_params* params,
                      const hotrg_opts* opts, hotrg_result* results, hotrg_status* statuses) {
  HIPCHK(hipSetDevice(c->device));
  const auto t0 = std::chrono::steady_clock::now();
  auto secs = [&] {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  };
  const bool timing = c->timing;
  c->timing = false;
  std::vector<GProb> P(N);
  std::vector<char> done(N, 0);
  // plan: the steady step of each problem and whether the batch takes it
  int group_sp = -1;
  bool group_dense_kind = false;
  for (int i = 0; i < N; ++i) {
    GProb& g = P[i];
    g.idx = i;
    statuses[i] = guard([&] {
      check_opts(&opts[i]);
      int dx = 0, dy = 0;
      (void)build_tensor(&params[i], &dx, &dy);
      g.o = resolve_prec(&opts[i], dx, dy);
      check_opts(&g.o);
      const int fr = first_reduced_step(g.o.prec, g.o.tol);
      const int ks = steady_step(g.o, g.o.prec, dx, dy, fr);
      // dims of every step
      int x = dx, y = dy;
      for (int k = 1; k <= g.o.n_steps; ++k) {
        const int dn = (int)std::min<long long>(g.o.d_cut, (long long)x * x);
        g.dxs.push_back(x);
        g.dys.push_back(y);
        g.dns.push_back(dn);
        if (k == ks) {
          g.D = x;
          g.sp = step_is_reduced(g.o.prec, k, x, y, g.o.d_cut, fr) ? g.o.prec : HOTRG_FP64;
        }
        const int nx = y;
        y = dn;
        x = nx;
      }
      // (a reduced-precision problem steady from step 1 would start from FP64
      // operands: it runs alone)
      bool ok = ks <= g.o.n_steps && g.o.isometry == HOTRG_ISO_ONE_SIDED &&
                g.o.eig == HOTRG_EIG_AUTO && !(ks == 1 && g.sp != HOTRG_FP64);
      if (ok) {
        g.n = g.D * g.D;
        g.need = std::max(g.D + 1, std::min(g.o.spec_len, g.n));
        g.p = (std::min(128, std::max(2 * g.D, g.need + 16)) + 15) / 16 * 16;
        const bool block = g.need + 16 <= g.p && g.p <= 128 && 4 * g.p <= g.n;
        // small environments: the whole matrix, padded to even size (at least 4)
        g.dense = !block && g.n <= 128;
        if (g.dense) g.p = std::max(4, g.n + (g.n & 1));
        ok = block || g.dense;
      }
      if (ok && group_sp < 0) {
        group_sp = g.sp;
        group_dense_kind = g.dense;
      }
      g.k_host = ok && g.sp == group_sp && g.dense == group_dense_kind ? ks - 1 : -1;  // -1: alone
    });
  }
  // warm-up steps one problem at a time; problems outside the batch run whole
  for (int i = 0; i < N; ++i) {
    GProb& g = P[i];
    if (statuses[i] != HOTRG_OK) {
      done[i] = 1;
      continue;
    }
    statuses[i] = guard([&] {
      int dx = 0, dy = 0;
      std::vector<double> T0 = build_tensor(&params[i], &dx, &dy);
      g.st = new_state(c, T0, dx, dy, g.o.prec);
      g.st->first_reduced = first_reduced_step(g.o.prec, g.o.tol);
      const int upto = g.k_host >= 0 ? g.k_host : g.o.n_steps;
      while (g.st->k < upto) do_step(c, g.st, &g.o);
      if (g.k_host < 0) {
        finish_into(c, g.st, g, &results[i], secs());
        done[i] = 1;
      }
    });
    if (statuses[i] != HOTRG_OK) done[i] = 1;
  }
  // per-problem buffers of the batch
  std::vector<GProb*> grp;
  for (int i = 0; i < N; ++i)
    if (!done[i]) grp.push_back(&P[i]);
  Buf ctlbuf, tables;
  hipGraphExec_t exec = nullptr;
  try {
    if (!grp.empty()) {
      const bool red = group_sp != HOTRG_FP64;
      const int mode = red ? rp_mode(group_sp) : RP_F32;
      const size_t es = mode == RP_F32 ? 4 : 2;
      const int halves = red && mode == RP_BF16X3 ? 2 : 1;
      ensure(c, ctlbuf, grp.size() * sizeof(GroupCtl));
      std::vector<GroupCtl> ctl(grp.size());
      for (size_t j = 0; j < grp.size(); ++j) {
        GProb& g = *grp[j];
        g.ctl = (GroupCtl*)ctlbuf.p + j;
        ctl[j] = GroupCtl{1, 0, 0, g.st->k};
        reserve_records(c, g.st, g.o.n_steps, g.o.spec_len);
        const long long D = g.D, n = g.n, pn = (long long)g.p * n, pp = (long long)g.p * g.p;
        ensure(c, g.M, (size_t)(n * n) * 8);
        ensure(c, g.eig, (size_t)(5 * pn + 3 * pp + 2 * g.p + 16) * 8);
        ensure(c, g.U, (size_t)(n * D) * 8);
        ensure(c, g.scal, 128);
        // sweep shifts of the two step parities (offset 64): none yet
        HIPCHK(hipMemsetAsync((char*)g.scal.p + 64, 0, 16, c->stream));
        if (red) {
          const long long ldP = pad32(D * D), ldx = pad32(D), ldn = pad32(n);
          ensure(c, g.Tt, (size_t)(D * D * D * D) * 4);
          for (int h = 0; h < halves; ++h) {
            ensure(c, g.RA1[h], (size_t)(n * ldP) * es);
            ensure(c, g.RA2[h], (size_t)(n * ldP) * es);
            ensure(c, g.RX1[h], (size_t)(D * D * D * ldP) * es);
            ensure(c, g.RX2[h], (size_t)(D * D * D * ldn) * es);
            ensure(c, g.RU1[h], (size_t)(D * D * ldx) * es);
            ensure(c, g.RU3[h], (size_t)(D * ldn) * es);
            // zero padding past the true K stays zero: the products write
            // only the valid columns
            Buf* pads[] = {&g.RA1[h], &g.RA2[h], &g.RX1[h], &g.RX2[h], &g.RU1[h], &g.RU3[h]};
            for (Buf* b : pads) HIPCHK(hipMemsetAsync(b->p, 0, b->bytes, c->stream));
          }
        } else {
          ensure(c, g.Tt, (size_t)(D * D * D * D) * 8);
          ensure(c, g.U1, (size_t)(n * D) * 8);
          ensure(c, g.U3, (size_t)(n * D) * 8);
        }
      }
      if (!red) {
        // FP64 contractions run problem after problem through the context's
        // intermediates: sized for the largest
        long long xmax = 1;
        for (GProb* g : grp) xmax = std::max(xmax, (long long)g->D * g->D * g->D * g->D * g->D);
        ensure(c, c->X1, (size_t)xmax * 8);
        ensure(c, c->X2, (size_t)xmax * 8);
      }
      HIPCHK(hipMemcpyAsync(ctlbuf.p, ctl.data(), ctl.size() * sizeof(GroupCtl),
                            hipMemcpyHostToDevice, c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
      GRun R;
      R.sp = group_sp;
      R.mode = mode;
      R.dense = group_dense_kind;
      std::vector<GProb*> cur;
      bool eager_done = false;
      for (;;) {
        std::vector<GProb*> act;
        for (GProb* g : grp)
          if (g->k_host < g->o.n_steps) act.push_back(g);
        if (act.empty()) break;
        if (act != cur) {
          // replays of the previous graph finish before its tables change
          HIPCHK(hipStreamSynchronize(c->stream));
          if (exec) {
            (void)hipGraphExecDestroy(exec);
            exec = nullptr;
          }
          std::vector<std::vector<long long>> keys;
          R.act = act;
          R.cfg[0] = R.cfg[1] = R.cfg[2] = R.cfg[3] = R.cfg[4] = -1;
          group_tables(c, R, tables, &keys);
          bool untuned = false;
          {
            std::lock_guard<std::mutex> lk(g_gtune_mu);
            for (size_t q = 0; q < keys.size(); ++q) {
              auto it = g_gtune.find(keys[q]);
              if (it != g_gtune.end()) R.cfg[q] = it->second;
              else untuned = true;
            }
          }
          if (!eager_done || untuned) {
            // an eager sweep: tunes the shapes, allocates what the step needs
            group_sweep(c, R, true, &keys);
            HIPCHK(hipGetLastError());
            HIPCHK(hipStreamSynchronize(c->stream));
            eager_done = true;
            ++c->g_sweeps;
            for (GProb* g : act) ++g->k_host;
            cur.clear();
            continue;
          }
          hipGraph_t graph = nullptr;
          HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
          try {
            group_sweep(c, R, false, &keys);
          } catch (...) {
            (void)hipStreamEndCapture(c->stream, &graph);
            if (graph) (void)hipGraphDestroy(graph);
            throw;
          }
          HIPCHK(hipStreamEndCapture(c->stream, &graph));
          const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
          (void)hipGraphDestroy(graph);
          HIPCHK(ie);
          ++c->g_captures;
          cur = act;
        }
        HIPCHK(hipGraphLaunch(exec, c->stream));
        ++c->g_sweeps;
        ++c->g_replays;
        for (GProb* g : act) ++g->k_host;
      }
      HIPCHK(hipStreamSynchronize(c->stream));
      HIPCHK(hipMemcpy(ctl.data(), ctlbuf.p, ctl.size() * sizeof(GroupCtl), hipMemcpyDeviceToHost));
      for (size_t j = 0; j < grp.size(); ++j) {
        GProb& g = *grp[j];
        const int i = g.idx;
        if (ctl[j].fail || ctl[j].k != g.o.n_steps) {
          // the batched eigensolve did not converge within its budget: this
          // problem is run again alone (with the dense fallback)
          ++c->g_fallbacks;
          hotrg_state_free(c, g.st);
          g.st = nullptr;
          statuses[i] = run_problem(c, &params[i], &g.o, &results[i], nullptr);
          continue;
        }
        statuses[i] = guard([&] {
          for (int k = g.st->k + 1; k <= g.o.n_steps; ++k)
            if (group_sp != HOTRG_FP64) g.st->err_bound += kErrPerStep[group_sp] * std::ldexp(1.0, -k);
          g.st->k = g.o.n_steps;
          finish_into(c, g.st, g, &results[i], secs());
        });
      }
    }
  } catch (...) {
    if (exec) (void)hipGraphExecDestroy(exec);
    for (GProb& g : P) {
      free_group_buffers(c, g);
      if (g.st) hotrg_state_free(c, g.st);
    }
    ctx_free(c, ctlbuf);
    ctx_free(c, tables);
    c->timing = timing;
    throw;
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  for (GProb& g : P) {
    free_group_buffers(c, g);
    if (g.st) hotrg_state_free(c, g.st);
  }
  ctx_free(c, ctlbuf);
  ctx_free(c, tables);
  c->timing = timing;
}

}  // namespace

namespace hotrg {

hotrg_status run_problem(hotrg_ctx* c, const hotrg_model_params* params, const hotrg_opts* o_in,
                         hotrg_result* res, const std::atomic<bool>* cancel) {
  hotrg_state* st = nullptr;
  hotrg_status s = guard([&] {
    if (!c || !res) fail(HOTRG_ERR_INVALID, "ctx/result is NULL");
    check_opts(o_in);
    HIPCHK(hipSetDevice(c->device));
    auto t0 = std::chrono::steady_clock::now();
    int dx = 0, dy = 0;
    std::vector<double> T0 = build_tensor(params, &dx, &dy);
    const hotrg_opts ro = resolve_prec(o_in, dx, dy);
    const hotrg_opts* o = &ro;
    check_opts(o);
    if (cancel && cancel->load()) fail(HOTRG_ERR_CANCELLED, "cancelled");
    st = new_state(c, T0, dx, dy, o->prec);
    st->first_reduced = first_reduced_step(o->prec, o->tol);
    std::vector<int> dxs, dys, dns;
    for (int k = 0; k < o->n_steps; ++k) {
      if (cancel && cancel->load()) fail(HOTRG_ERR_CANCELLED, "cancelled");
      dxs.push_back(st->dx);
      dys.push_back(st->dy);
      do_step(c, st, o);
      dns.push_back(st->dy);
    }
    double lnz = 0;
    hotrg_status fs = hotrg_finish(c, st, &lnz);
    if (fs != HOTRG_OK) fail(fs, g_err);
    if (res->steps || res->spectra) {
      fetch_info(c, st, 0, o->n_steps, nullptr, res->steps, res->spectra);
      if (res->steps)
        for (int k = 0; k < o->n_steps; ++k) {
          res->steps[k].dx = dxs[k];
          res->steps[k].dy = dys[k];
          res->steps[k].d_new = dns[k];
        }
    }
    res->lnz_per_site = lnz;
    res->n_steps = o->n_steps;
    res->prec_used = o->prec;
    res->err_bound = st->err_bound;
    res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  });
  if (st) hotrg_state_free(c, st);
  return s;
}

void ctx_trim(hotrg_ctx* c) {
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  Buf* bufs[] = {&c->A1, &c->A2, &c->M, &c->W, &c->E, &c->Ucan, &c->U1, &c->U3,
                 &c->X1, &c->X2, &c->Tt, &c->EW, &c->Xr, &c->Tm, &c->Xm, &c->M2,
                 &c->W2, &c->Xr2, &c->Side};
  for (Buf* b : bufs) ctx_free(c, *b);
  for (Buf* arr : {c->RA1, c->RA2, c->RX1, c->RX2, c->RU1, c->RU3})
    for (int h = 0; h < 2; ++h) ctx_free(c, arr[h]);
}

double ctx_seconds(const hotrg_ctx* c) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - c->t0).count();
}
int ctx_device(const hotrg_ctx* c) { return c->device; }
size_t ctx_budget(const hotrg_ctx* c) { return c->budget; }
int& ctx_workers(hotrg_ctx* c) { return c->n_workers; }
int& ctx_test_fail_step(hotrg_ctx* c) { return c->test_fail_step; }
void*& ctx_sched(hotrg_ctx* c) { return c->sched; }
const char* last_error_text() { return g_err.c_str(); }
void set_last_error(const char* m) { g_err = m; }

}  // namespace hotrg


extern "C" {

const char* hotrg_last_error(void) { return g_err.c_str(); }

hotrg_status hotrg_ctx_create(int device, void* hip_stream, size_t hbm_budget, hotrg_ctx** out) {
  return guard([&] {
    if (!out) fail(HOTRG_ERR_INVALID, "out is NULL");
    int n = 0;
    HIPCHK(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) fail(HOTRG_ERR_INVALID, "no such device");
    HIPCHK(hipSetDevice(device));
    noalloc_init_device(device);  // this device's address of the no-alloc scratch array
    auto* c = new hotrg_ctx();
    c->device = device;
    if (const char* e = getenv("HOTRG_TEST_EIG_FAIL_STEP")) c->test_fail_step = atoi(e);
    c->budget = hbm_budget;
    if (hip_stream) {
      c->stream = (hipStream_t)hip_stream;
    } else {
      hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
      if (e != hipSuccess) {
        delete c;
        fail(HOTRG_ERR_DEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
      }
      c->own_stream = true;
    }
    if (rocblas_create_handle(&c->blas) != rocblas_status_success) {
      if (c->own_stream) (void)hipStreamDestroy(c->stream);
      delete c;
      fail(HOTRG_ERR_DEVICE, "rocblas_create_handle failed");
    }
    rocblas_set_stream(c->blas, c->stream);
    *out = c;
  });
}

void hotrg_ctx_destroy(hotrg_ctx* c) {
  if (!c) return;
  hotrg::sched_shutdown(c);
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  Buf* bufs[] = {&c->A1, &c->A2, &c->M, &c->W, &c->E, &c->Ucan, &c->U1, &c->U3,
                 &c->X1, &c->X2, &c->Tt, &c->scal, &c->EW, &c->Xr, &c->Tm, &c->Xm,
                 &c->M2, &c->W2, &c->Xr2, &c->Side};
  for (Buf* b : bufs) ctx_free(c, *b);
  for (Buf* arr : {c->RA1, c->RA2, c->RX1, c->RX2, c->RU1, c->RU3})
    for (int h = 0; h < 2; ++h) ctx_free(c, arr[h]);
  for (auto& m : c->marks) {
    c->pool.push_back(m.a);
    c->pool.push_back(m.b);
  }
  std::sort(c->pool.begin(), c->pool.end());
  c->pool.erase(std::unique(c->pool.begin(), c->pool.end()), c->pool.end());
  for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
  if (c->blas) rocblas_destroy_handle(c->blas);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

size_t hotrg_ctx_bytes_in_use(const hotrg_ctx* c) { return c ? c->in_use : 0; }

hotrg_status hotrg_init_tensor(hotrg_ctx* c, const hotrg_model_params* params, int prec,
                               hotrg_state** out) {
  return guard([&] {
    if (!c || !out) fail(HOTRG_ERR_INVALID, "ctx/out is NULL");
    check_prec(prec);
    HIPCHK(hipSetDevice(c->device));
    int dx = 0, dy = 0;
    std::vector<double> T0 = build_tensor(params, &dx, &dy);
    *out = new_state(c, T0, dx, dy, prec);
  });
}

hotrg_status hotrg_step(hotrg_ctx* c, hotrg_state* st, const hotrg_opts* o, hotrg_step_info* info,
                        double* spectrum) {
  return guard([&] {
    if (!c || !st) fail(HOTRG_ERR_INVALID, "ctx/state is NULL");
    check_opts(o);
    if (o->isometry == HOTRG_ISO_TWO_SIDED && st->prec != HOTRG_FP64)
      fail(HOTRG_ERR_INVALID, "two-sided isometry needs FP64 contractions");
    if (o->prec == HOTRG_PREC_AUTO)
      fail(HOTRG_ERR_INVALID, "HOTRG_PREC_AUTO applies to whole runs only");
    HIPCHK(hipSetDevice(c->device));
    const int dx = st->dx, dy = st->dy;
    st->first_reduced = first_reduced_step(st->prec, o->tol);
    do_step(c, st, o);
    if (info || spectrum) {
      check_info(c, st);
      hotrg_step_info tmp;
      double* sp = nullptr;
      std::vector<double> spv;
      if (spectrum && st->spec_len) {
        spv.resize(st->spec_len);
        sp = spv.data();
      }
      fetch_info(c, st, st->k - 1, 1, nullptr, &tmp, sp);
      tmp.dx = dx;
      tmp.dy = dy;
      tmp.d_new = st->dy;
      if (info) *info = tmp;
      if (spectrum && sp) std::memcpy(spectrum, sp, spv.size() * 8);
    }
  });
}

hotrg_status hotrg_finish(hotrg_ctx* c, hotrg_state* st, double* lnz) {
  return guard([&] {
    if (!c || !st || !lnz) fail(HOTRG_ERR_INVALID, "ctx/state/out is NULL");
    HIPCHK(hipSetDevice(c->device));
    ensure(c, c->scal, 64);
    double* outp = (double*)((char*)c->scal.p + 24);
    launch_finish(st->cur_f32 ? st->Tn32.p : st->Tn.p, st->cur_f32, st->dx, st->dy,
                  std::ldexp(1.0, -st->k), (const double*)st->acc.p, outp, c->stream);
    HIPCHK(hipGetLastError());
    double v = 0;
    HIPCHK(hipMemcpyAsync(&v, outp, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (st->k > 0) check_info(c, st);
    if (!std::isfinite(v)) fail(HOTRG_ERR_NUMERIC, "non-finite ln Z (norm or trace <= 0)");
    *lnz = v;
  });
}

hotrg_status hotrg_state_export(hotrg_ctx* c, const hotrg_state* st, double* host, size_t cap,
                                int dims[2], double* acc, int* k) {
  return guard([&] {
    if (!c || !st) fail(HOTRG_ERR_INVALID, "ctx/state is NULL");
    HIPCHK(hipSetDevice(c->device));
    size_t ne = (size_t)st->dx * st->dy * st->dx * st->dy;
    if (host && cap < ne) fail(HOTRG_ERR_INVALID, "host buffer too small");
    if (host) {
      if (!st->cur_f32) {
        HIPCHK(hipMemcpyAsync(host, st->Tn.p, ne * 8, hipMemcpyDeviceToHost, c->stream));
      } else {
        std::vector<float> f(ne);
        HIPCHK(hipMemcpyAsync(f.data(), st->Tn32.p, ne * 4, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        for (size_t i = 0; i < ne; ++i) host[i] = f[i];
      }
    }
    double a = 0;
    HIPCHK(hipMemcpyAsync(&a, st->acc.p, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (dims) {
      dims[0] = st->dx;
      dims[1] = st->dy;
    }
    if (acc) *acc = a;
    if (k) *k = st->k;
  });
}

void hotrg_state_free(hotrg_ctx* c, hotrg_state* st) {
  if (!c || !st) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  Buf* bufs[] = {&st->Tn, &st->Xt, &st->Tp, &st->acc, &st->recs, &st->spec, &st->Tn32};
  for (Buf* b : bufs) ctx_free(c, *b);
  for (auto& o : st->RO)
    for (auto& b : o) ctx_free(c, b);
  delete st;
}

hotrg_status hotrg_run(hotrg_ctx* c, const hotrg_model_params* params, const hotrg_opts* o,
                       hotrg_result* res) {
  return hotrg::run_problem(c, params, o, res, nullptr);
}

hotrg_status hotrg_plan(const hotrg_model_params* params, const hotrg_opts* o, int* prec,
                        int* first_reduced, double* err_bound) {
  return guard([&] {
    check_opts(o);
    int dx = 0, dy = 0;
    (void)build_tensor(params, &dx, &dy);
    const hotrg_opts r = resolve_prec(o, dx, dy);
    check_opts(&r);
    const PrecPlan pl = plan_precision(r.prec, r.tol, dx, dy, r.d_cut, r.n_steps);
    if (prec) *prec = pl.err_bound > 0.0 ? r.prec : HOTRG_FP64;
    if (first_reduced) *first_reduced = pl.first_reduced;
    if (err_bound) *err_bound = pl.err_bound;
  });
}

hotrg_status hotrg_run_grouped(hotrg_ctx* c, int n, const hotrg_model_params* params,
                               const hotrg_opts* opts, hotrg_result* results,
                               hotrg_status* statuses) {
  std::vector<hotrg_status> st(n > 0 ? n : 0, HOTRG_OK);
  hotrg_status s = guard([&] {
    if (!c || n < 0 || (n > 0 && (!params || !opts || !results)))
      fail(HOTRG_ERR_INVALID, "NULL argument");
    run_grouped_impl(c, n, params, opts, results, st.data());
  });
  if (s != HOTRG_OK) {
    for (auto& x : st) x = s;
  }
  hotrg_status first = HOTRG_OK;
  for (int i = 0; i < n; ++i) {
    if (statuses) statuses[i] = st[i];
    if (st[i] != HOTRG_OK && first == HOTRG_OK) first = st[i];
  }
  return s != HOTRG_OK ? s : first;
}

hotrg_status hotrg_ctx_group_stats(hotrg_ctx* c, uint64_t* sweeps, uint64_t* replays,
                                   uint64_t* captures, uint64_t* fallbacks) {
  return guard([&] {
    if (!c) fail(HOTRG_ERR_INVALID, "ctx is NULL");
    if (sweeps) *sweeps = c->g_sweeps;
    if (replays) *replays = c->g_replays;
    if (captures) *captures = c->g_captures;
    if (fallbacks) *fallbacks = c->g_fallbacks;
  });
}

hotrg_status hotrg_ctx_enable_timing(hotrg_ctx* c, int on) {
  return guard([&] {
    if (!c) fail(HOTRG_ERR_INVALID, "ctx is NULL");
    c->timing = on != 0;
  });
}

hotrg_status hotrg_ctx_last_eig(hotrg_ctx* c, int* sweeps, double* resid) {
  return guard([&] {
    if (!c) fail(HOTRG_ERR_INVALID, "ctx is NULL");
    if (sweeps) *sweeps = c->last_eig_iters;
    if (resid) *resid = c->last_eig_resid;
  });
}

int hotrg_ctx_timings(hotrg_ctx* c, hotrg_phase_time* out, int cap) {
  int n = -1;
  hotrg_status s = guard([&] {
    if (!c) fail(HOTRG_ERR_INVALID, "ctx is NULL");
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize(c->stream));
    n = 0;
    for (auto& m : c->marks) {
      if (out && n < cap) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, m.a, m.b));
        out[n++] = hotrg_phase_time{m.step, m.phase, m.dx, m.dy, m.dn, ms};
      }
    }
    // events are shared between consecutive marks: return each once
    std::vector<hipEvent_t> evs;
    for (auto& m : c->marks) {
      evs.push_back(m.a);
      evs.push_back(m.b);
    }
    std::sort(evs.begin(), evs.end());
    evs.erase(std::unique(evs.begin(), evs.end()), evs.end());
    for (hipEvent_t e : evs) c->pool.push_back(e);
    c->marks.clear();
  });
  return s == HOTRG_OK ? n : -1;
}

hotrg_status hotrg_environment(hotrg_ctx* c, int prec, const double* T, int dx, int dy,
                               double* M) {
  return guard([&] {
    if (!c || !T || !M) fail(HOTRG_ERR_INVALID, "NULL argument");
    if (dx < 1 || dy < 1) fail(HOTRG_ERR_INVALID, "dx, dy must be >= 1");
    check_prec(prec);
    check_dims(dx, dy, 1);
    HIPCHK(hipSetDevice(c->device));
    ensure(c, c->scal, 64);
    unsigned long long* one = (unsigned long long*)((char*)c->scal.p + 56);
    const unsigned long long one_bits = 0x3ff0000000000000ULL;
    HIPCHK(hipMemcpyAsync(one, &one_bits, 8, hipMemcpyHostToDevice, c->stream));
    hotrg_state tmp;  // operands only, freed below
    try {
      prepare_operands(c, &tmp, prec, T, false, false, dx, dy, one);
      c->m_step = 0;
      c->m_dx = dx;
      c->m_dy = dy;
      c->m_dn = dx * dx;
      mark(c, HOTRG_PHASE_ENV);
      if (prec == HOTRG_FP64)
        environment_f64(c, (const double*)tmp.Tn.p, (const double*)tmp.Xt.p, dx, dy);
      else
        environment_rp(c, &tmp, rp_mode(prec), dx, dy);
      mark(c, -1);
      const size_t nn = (size_t)dx * dx * dx * dx;
      HIPCHK(hipMemcpyAsync(M, c->M.p, nn * 8, hipMemcpyDeviceToDevice, c->stream));
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(c->stream));
    } catch (...) {
      release_operands(c, &tmp);
      throw;
    }
    release_operands(c, &tmp);
  });
}

hotrg_status hotrg_projector(hotrg_ctx* c, const double* M, int n, int dn, int trunc,
                             double degen_tol, int spec_len, double* U, double* spec, int* kept,
                             double* trunc_err) {
  return guard([&] {
    if (!c || !M || !U || !kept || !trunc_err) fail(HOTRG_ERR_INVALID, "NULL argument");
    if (n < 2 || dn < 1 || dn > n) fail(HOTRG_ERR_INVALID, "need 2 <= n and 1 <= d_new <= n");
    if ((long long)n * n > (1LL << 28)) fail(HOTRG_ERR_INVALID, "n too large");
    if (spec_len < 0 || (spec_len > 0 && !spec))
      fail(HOTRG_ERR_INVALID, "spec_len < 0 or spec NULL with spec_len > 0");
    if (trunc != HOTRG_TRUNC_PLAIN && trunc != HOTRG_TRUNC_MULTIPLET)
      fail(HOTRG_ERR_INVALID, "unknown truncation rule");
    if (!(degen_tol >= 0.0)) fail(HOTRG_ERR_INVALID, "degen_tol must be >= 0");
    HIPCHK(hipSetDevice(c->device));
    ensure(c, c->scal, 64);
    ensure(c, c->M, (size_t)n * n * 8);
    HIPCHK(hipMemcpyAsync(c->M.p, M, (size_t)n * n * 8, hipMemcpyDeviceToDevice, c->stream));
    launch_symmetrize((double*)c->M.p, n, c->stream);
    double* trace = (double*)((char*)c->scal.p + 40);
    int* info = (int*)((char*)c->scal.p + 8);
    launch_trace((const double*)c->M.p, n, trace, c->stream);
    int need = 0, p = 0;
    const bool sub_ok = eig_block(n, dn, spec_len, HOTRG_EIG_AUTO, &need, &p);
    // record (6 doubles), sticky flag, kept count, spectrum
    Buf out;
    ensure(c, out, (size_t)(8 + spec_len) * 8);
    try {
      double* rec = (double*)out.p;
      int* sticky = (int*)(rec + 6);
      int* kept_d = sticky + 1;
      double* spec_d = spec_len ? rec + 8 : nullptr;
      HIPCHK(hipMemsetAsync(sticky, 0, sizeof(int), c->stream));
      EigHint h;  // a solve of its own
      int cols = n;
      const double* evec =
          leading_eigs(c, c->M, c->W, c->Xr, n, need, p, sub_ok, h, info, sticky, &cols);
      launch_spectrum((const double*)c->W.p, cols, n, dn, trunc, degen_tol, spec_len, trace,
                      spec_d, rec, kept_d, c->stream);
      launch_isometry(evec, cols, n, dn, kept_d, U, c->stream);
      int hk[2] = {0, 0};
      HIPCHK(hipMemcpyAsync(hk, sticky, 2 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipMemcpyAsync(trunc_err, rec + 1, 8, hipMemcpyDeviceToHost, c->stream));
      if (spec_len)
        HIPCHK(hipMemcpyAsync(spec, spec_d, (size_t)spec_len * 8, hipMemcpyDeviceToHost,
                              c->stream));
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(c->stream));
      if (hk[0] != 0) fail(HOTRG_ERR_NUMERIC, "eigensolver did not converge");
      *kept = hk[1];
    } catch (...) {
      ctx_free(c, out);
      throw;
    }
    ctx_free(c, out);
  });
}

hotrg_status hotrg_coarse(hotrg_ctx* c, int prec, const double* T, const double* U, int dx,
                          int dy, int dn, double* Tt, double* max_abs) {
  return guard([&] {
    if (!c || !T || !U || !Tt) fail(HOTRG_ERR_INVALID, "NULL argument");
    if (dx < 1 || dy < 1 || dn < 1) fail(HOTRG_ERR_INVALID, "dims must be >= 1");
    check_prec(prec);
    check_dims(dx, dy, dn);
    HIPCHK(hipSetDevice(c->device));
    ensure(c, c->scal, 64);
    unsigned long long* one = (unsigned long long*)((char*)c->scal.p + 56);
    const unsigned long long one_bits = 0x3ff0000000000000ULL;
    HIPCHK(hipMemcpyAsync(one, &one_bits, 8, hipMemcpyHostToDevice, c->stream));
    unsigned long long* mb = (unsigned long long*)c->scal.p + 4;
    hotrg_state tmp;
    try {
      prepare_operands(c, &tmp, prec, T, false, false, dx, dy, one);
      c->m_step = 0;
      c->m_dx = dx;
      c->m_dy = dy;
      c->m_dn = dn;
      const size_t no = (size_t)dn * dy * dn * dy;
      if (prec == HOTRG_FP64) {
        const size_t nu = (size_t)dx * dx * dn;
        ensure(c, c->U1, nu * 8);
        ensure(c, c->U3, nu * 8);
        launch_layout_u(U, dx, dn, c->U1.p, c->U3.p, false, c->stream);
        coarse_f64(c, (const double*)tmp.Tn.p, (const double*)tmp.Tp.p, (const double*)c->U1.p,
                   (const double*)c->U3.p, dx, dy, dn, mb);
        mark(c, -1);
        HIPCHK(hipMemcpyAsync(Tt, c->Tt.p, no * 8, hipMemcpyDeviceToDevice, c->stream));
      } else {
        const int mode = rp_mode(prec);
        const size_t es = mode == RP_F32 ? 4 : 2;
        const long long n = (long long)dx * dx, ldx = pad32(dx), ldn = pad32(n);
        for (int h = 0; h < (mode == RP_F32 ? 1 : 2); ++h) {
          ensure(c, c->RU1[h], (size_t)dn * dx * ldx * es);
          ensure(c, c->RU3[h], (size_t)dn * ldn * es);
          HIPCHK(hipMemsetAsync(c->RU1[h].p, 0, (size_t)dn * dx * ldx * es, c->stream));
          HIPCHK(hipMemsetAsync(c->RU3[h].p, 0, (size_t)dn * ldn * es, c->stream));
        }
        launch_layout_u_rp(U, dx, dn, mode, c->RU1[0].p, mode == RP_F32 ? nullptr : c->RU1[1].p,
                           c->RU3[0].p, mode == RP_F32 ? nullptr : c->RU3[1].p, ldx, ldn,
                           c->stream);
        coarse_rp(c, &tmp, mode, dx, dy, dn, mb);
        mark(c, -1);
        launch_f32_to_f64((const float*)c->Tt.p, Tt, (long long)no, c->stream);
      }
      if (max_abs) HIPCHK(hipMemcpyAsync(max_abs, mb, 8, hipMemcpyDeviceToDevice, c->stream));
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(c->stream));
    } catch (...) {
      release_operands(c, &tmp);
      throw;
    }
    release_operands(c, &tmp);
  });
}

}  // extern "C"
