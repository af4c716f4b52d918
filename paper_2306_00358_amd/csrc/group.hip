// Batched kernels of the lockstep batch engine (hotrg_run_grouped): many
// problems -- temperatures, couplings, uneven D_cut -- take their steady-state
// coarse-graining steps together (arXiv 2306.00358, Sec. 2, one directional
// step per sweep), one launch per phase over all of them, so that a whole
// sweep can be captured as one HIP graph and replayed without host waits.
//
// Each problem has a GroupStep descriptor (device memory, fixed for a run)
// and a GroupCtl block the kernels update: the step counter, whether the
// problem still has steps, whether its block eigensolver is still iterating
// in this step, and a sticky failure flag.  A kernel's grid covers every
// problem; a problem that is finished (or has converged, for the eigensolver)
// returns at once.
//
// Block eigensolver of a batch: the subspace iteration of eigs.hip with a
// fixed budget (rounds of sweeps, each round ending in a Rayleigh-Ritz check
// on the device), so that no host read decides the number of sweeps; the
// p x p Rayleigh-Ritz matrices go through the Householder reduction and the
// tridiagonal divide and conquer of the per-problem path (one workgroup per
// problem, eigs.hip and stedc.hip).  Small environments are diagonalised
// whole by a parallel two-sided Jacobi method (one workgroup per problem,
// below): in each of the p - 1 rounds of a
// sweep the p indices form p/2 disjoint pairs (a round-robin tournament, so
// every pair meets once per sweep); each pair's 2 x 2 rotation annihilates
// its off-diagonal element, and the rotations of one round, acting on
// disjoint index pairs, are applied to the matrix (in LDS) as independent
// 2 x 2 blocks R_a^T H_ab R_b, and to the accumulated eigenvectors.  Sweeps
// stop when no off-diagonal element exceeds 2^-53 sqrt(|h_ii h_jj|).
#include <hip/hip_runtime.h>

#include "internal.h"

namespace hotrg {

// ----------------------------------------------------------- eigensolver --

__global__ void k_group_begin(const GroupStep* __restrict__ d, int count) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < count) d[g].ctl->iter = d[g].ctl->active;
}

// deterministic start block: splitmix64 of the element index -> [-1, 1)
__global__ void k_group_seed(const GroupStep* __restrict__ d) {
  const GroupStep& s = d[blockIdx.y];
  if (!s.ctl->iter) return;
  const long long count = (long long)s.p * s.n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < count;
       e += (long long)gridDim.x * blockDim.x) {
    unsigned long long z = (unsigned long long)e + 12345ULL * 0x9E3779B97F4A7C15ULL;
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    s.V[e] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
}

__global__ void k_group_symm_h(const GroupStep* __restrict__ d) {
  const GroupStep& s = d[blockIdx.y];
  if (!s.ctl->iter) return;
  const int p = s.p;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < p * p; e += gridDim.x * blockDim.x) {
    const int i = e / p, j = e % p;
    if (i < j) {
      const double v = 0.5 * (s.H[i * p + j] + s.H[j * p + i]);
      s.H[i * p + j] = v;
      s.H[j * p + i] = v;
    }
  }
}

constexpr int kJacThreads = 256;
constexpr int kJacMaxSweeps = 40;

// index at tournament position q in round r (position 0 stays)
__device__ __forceinline__ int jac_player(int q, int r, int p) {
  return q == 0 ? 0 : 1 + (q - 1 + r) % (p - 1);
}

// H (p x p, symmetric) -> W (p eigenvalues, ascending) and H overwritten by
// Z^T (row c = eigenvector c, same order).  Z^T is accumulated in LDS next to
// the matrix when both fit (vt_lds: p <= 96), else in T2 (p x p, global).
__global__ __launch_bounds__(kJacThreads) void k_group_jacobi(const GroupStep* __restrict__ d,
                                                              int vt_lds) {
  const GroupStep& s = d[blockIdx.x];
  if (!s.ctl->iter) return;
  extern __shared__ double A[];            // p x p (then Z^T, p x p, with vt_lds)
  __shared__ double cs_c[64], cs_s[64];    // rotation of pair m
  __shared__ int pi[64], pj[64];           // its indices, pi < pj
  __shared__ int rot;
  __shared__ int rank_s[128];
  const int p = s.p, h = p / 2, t = threadIdx.x;
  double* Vt = vt_lds ? A + p * p : s.T2;
  for (int e = t; e < p * p; e += kJacThreads) {
    A[e] = s.H[e];
    Vt[e] = (e / p == e % p) ? 1.0 : 0.0;
  }
  __syncthreads();
  const double eps = 1.1102230246251565e-16;  // 2^-53
  int sweep = 0;
  for (; sweep < kJacMaxSweeps; ++sweep) {
    if (t == 0) rot = 0;
    __syncthreads();
    for (int r = 0; r < p - 1; ++r) {
      if (t < h) {
        int i = jac_player(t, r, p), j = jac_player(p - 1 - t, r, p);
        if (i > j) { const int x = i; i = j; j = x; }
        const double aii = A[i * p + i], ajj = A[j * p + j], aij = A[i * p + j];
        double c = 1.0, sn = 0.0;
        if (aij != 0.0 && fabs(aij) > eps * sqrt(fabs(aii * ajj))) {
          const double tau = (ajj - aii) / (2.0 * aij);
          const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + tt * tt);
          sn = tt * c;
          rot = 1;
        }
        cs_c[t] = c;
        cs_s[t] = sn;
        pi[t] = i;
        pj[t] = j;
      }
      __syncthreads();
      // A <- P^T A P as independent 2 x 2 blocks (pair m1 rows, pair m2 columns)
      for (int b = t; b < h * h; b += kJacThreads) {
        const int m1 = b / h, m2 = b % h;
        const int i1 = pi[m1], j1 = pj[m1], i2 = pi[m2], j2 = pj[m2];
        const double c1 = cs_c[m1], s1 = cs_s[m1], c2 = cs_c[m2], s2 = cs_s[m2];
        const double x11 = A[i1 * p + i2], x12 = A[i1 * p + j2];
        const double x21 = A[j1 * p + i2], x22 = A[j1 * p + j2];
        const double t11 = x11 * c2 - x12 * s2, t12 = x11 * s2 + x12 * c2;
        const double t21 = x21 * c2 - x22 * s2, t22 = x21 * s2 + x22 * c2;
        double a12 = c1 * t12 - s1 * t22, a21 = s1 * t11 + c1 * t21;
        if (m1 == m2) a12 = a21 = 0.0;
        A[i1 * p + i2] = c1 * t11 - s1 * t21;
        A[i1 * p + j2] = a12;
        A[j1 * p + i2] = a21;
        A[j1 * p + j2] = s1 * t12 + c1 * t22;
      }
      // Z <- Z P, i.e. rows i, j of Z^T rotate
      for (int e = t; e < h * p; e += kJacThreads) {
        const int m = e / p, col = e % p;
        const int i = pi[m], j = pj[m];
        const double c = cs_c[m], sn = cs_s[m];
        const double vi = Vt[i * p + col], vj = Vt[j * p + col];
        Vt[i * p + col] = c * vi - sn * vj;
        Vt[j * p + col] = sn * vi + c * vj;
      }
      __syncthreads();
    }
    // every thread reads the flag before thread 0 clears it for the next sweep
    const int any = rot;
    __syncthreads();
    if (!any) break;
  }
  if (sweep == kJacMaxSweeps && t == 0) s.ctl->fail = 1;
  // ascending order: rank of each diagonal value (ties by index)
  if (t < p) {
    const double w = A[t * p + t];
    int rk = 0;
    for (int j = 0; j < p; ++j) {
      const double x = A[j * p + j];
      rk += (x < w || (x == w && j < t)) ? 1 : 0;
    }
    rank_s[t] = rk;
    s.W[rk] = w;
  }
  __syncthreads();
  for (int e = t; e < p * p; e += kJacThreads) {
    const int i = e / p, col = e % p;
    s.H[rank_s[i] * p + col] = Vt[e];
  }
}

// Residuals of the `need` leading Ritz pairs, |Yx_i - theta_i X_i|, against
// tol * theta_1: converged problems stop iterating; in the last round a
// problem that has not converged stops too and is marked failed.
__global__ void k_group_resid(const GroupStep* __restrict__ d, int last) {
  const GroupStep& s = d[blockIdx.x];
  if (!s.ctl->iter) return;
  __shared__ double red[256];
  const int t = threadIdx.x, p = s.p, n = s.n;
  const double th1 = s.W[p - 1];
  double worst = 0.0;
  for (int q = 0; q < s.need; ++q) {
    const int i = p - 1 - q;
    const double th = s.W[i];
    double acc = 0.0;
    for (int j = t; j < n; j += 256) {
      const double r = s.Yx[(long long)i * n + j] - th * s.X[(long long)i * n + j];
      acc += r * r;
    }
    red[t] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (t < o) red[t] += red[t + o];
      __syncthreads();
    }
    worst = fmax(worst, sqrt(red[0]));
    __syncthreads();
  }
  if (t == 0) {
    s.res[0] = th1 > 0.0 ? worst / th1 : 1.0;
    const bool ok = th1 > 0.0 && worst <= s.tol * th1;
    if (ok || last) s.ctl->iter = 0;
    if (!ok && last) s.ctl->fail = 1;
    // the shift of the sweeps to come, and of the next solve of this parity
    s.shift[s.ctl->k & 1] = 0.5 * fmax(s.W[0], 0.0);
  }
}

// Y <- Y - sigma V after a sweep's product Y = V M: the sweeps iterate with
// M - sigma I (M positive semidefinite, unwanted eigenvalues in
// [0, lambda_{p+1}]; sigma = theta_min / 2 <= lambda_p / 2), the
// Rayleigh-Ritz products with M
__global__ void k_group_shift(const GroupStep* __restrict__ d) {
  const GroupStep& s = d[blockIdx.y];
  if (!s.ctl->iter) return;
  const double sg = s.shift[s.ctl->k & 1];
  if (!(sg > 0.0)) return;
  const long long count = (long long)s.p * s.n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < count;
       e += (long long)gridDim.x * blockDim.x)
    s.Y[e] -= sg * s.V[e];
}

// continue from the Ritz vectors: V <- X while still iterating
__global__ void k_group_restart(const GroupStep* __restrict__ d) {
  const GroupStep& s = d[blockIdx.y];
  if (!s.ctl->iter) return;
  const long long count = (long long)s.p * s.n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < count;
       e += (long long)gridDim.x * blockDim.x)
    s.V[e] = s.X[e];
}

// Small environments (n <= 96) are diagonalised whole by the Jacobi kernel:
// H = M padded with zero rows and columns to the even size p (a padded index
// adds an eigenvalue 0 below the spectrum), and the eigenvectors' first n
// components become the rows of X.
__global__ void k_group_dense_in(const GroupStep* __restrict__ d) {
  const GroupStep& s = d[blockIdx.y];
  if (!s.ctl->iter) return;
  const int p = s.p, n = s.n;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < p * p; e += gridDim.x * blockDim.x) {
    const int i = e / p, j = e % p;
    s.H[e] = (i < n && j < n) ? s.M[(long long)i * n + j] : 0.0;
  }
}

__global__ void k_group_dense_out(const GroupStep* __restrict__ d) {
  const GroupStep& s = d[blockIdx.y];
  if (!s.ctl->iter) return;
  const int p = s.p, n = s.n;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < p * n; e += gridDim.x * blockDim.x) {
    const int i = e / n, j = e % n;
    s.X[e] = s.H[(long long)i * p + j];
  }
}

// ------------------------------------------------------------ bookkeeping --

// Spectrum record of step k = ctl.k + 1 (as k_spectrum: lambda / lambda_1,
// truncation error, cut gap, multiplet-safe kept count, side 0).
__global__ void k_group_spectrum(const GroupStep* __restrict__ d) {
  const GroupStep& s = d[blockIdx.x];
  if (!s.ctl->active) return;
  __shared__ double red[256];
  __shared__ int kept_s;
  const int t = threadIdx.x, cnt = s.p, n = s.n, dn = s.dn;
  const int k = s.ctl->k + 1;
  double* rec = s.recs + kGroupRec * (long long)(k - 1);
  double* spec = s.spec_len ? s.spec + (long long)(k - 1) * s.spec_len : nullptr;
  const double* W = s.W;
  const double l1 = W[cnt - 1];
  if (t == 0) {
    int kept = dn;
    if (s.trunc == 1 && dn < n)
      while (kept > 0 && (W[cnt - kept] - W[cnt - 1 - kept]) <= s.tau * l1) --kept;
    kept_s = kept;
    *s.kept = kept;
  }
  __syncthreads();
  const int kept = kept_s;
  double kp = 0.0;
  for (int m = t; m < kept; m += 256) kp += W[cnt - 1 - m];
  red[t] = kp;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  if (t == 0) {
    rec[1] = 1.0 - red[0] / s.trace[0];
    rec[2] = dn < n ? (W[cnt - dn] - W[cnt - 1 - dn]) / l1 : -1.0;
    rec[4] = (double)kept;
    rec[5] = 0.0;
  }
  if (spec)
    for (int m = t; m < s.spec_len; m += 256) spec[m] = m < cnt ? W[cnt - 1 - m] / l1 : 0.0;
}

// ln n_k, acc += 2^-k ln n_k and the torus estimate of step k (as k_norm).
__global__ void k_group_norm(const GroupStep* __restrict__ d) {
  const GroupStep& s = d[blockIdx.x];
  if (!s.ctl->active) return;
  __shared__ double red[256];
  const int t = threadIdx.x, dn = s.dn, dy = s.dy;
  const int k = s.ctl->k + 1;
  double* rec = s.recs + kGroupRec * (long long)(k - 1);
  const double nk = __longlong_as_double((long long)*s.maxbits);
  double sum = 0.0;
  for (int e = t; e < dn * dy; e += 256) {
    const int i = e / dy, j = e % dy;
    const long long o = (((long long)i * dy + j) * dn + i) * dy + j;
    sum += s.tt_f32 ? (double)((const float*)s.Tt)[o] : ((const double*)s.Tt)[o];
  }
  red[t] = sum;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  if (t == 0) {
    const double w = ldexp(1.0, -k);
    const double ln = log(nk);
    const double a = s.acc[0] + w * ln;
    s.acc[0] = a;
    const double tr = red[0] / nk;
    rec[0] = ln;
    rec[3] = tr > 0.0 ? a + w * log(tr) : __longlong_as_double(0x7ff8000000000000LL);
  }
}

// max|T~| slots start at zero (a kernel: no memset node in a captured sweep)
__global__ void k_group_zero_max(const GroupStep* __restrict__ d, int count) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < count && d[g].ctl->active) *d[g].maxbits = 0ULL;
}

// one step done: advance the counter, retire problems that have all their steps
__global__ void k_group_advance(const GroupStep* __restrict__ d, int count) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= count || !d[g].ctl->active) return;
  GroupCtl* c = d[g].ctl;
  c->k += 1;
  if (c->k >= d[g].K) c->active = 0;
}

// ------------------------------------------------------------- launchers --

static inline int gblocks(long long n) {
  long long b = (n + 255) / 256;
  return (int)(b < 1024 ? (b > 0 ? b : 1) : 1024);
}

void group_begin(const GroupStep* d, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_group_begin, dim3((count + 63) / 64), dim3(64), 0, s, d, count);
}
void group_seed(const GroupStep* d, int count, long long max_pn, hipStream_t s) {
  hipLaunchKernelGGL(k_group_seed, dim3(gblocks(max_pn), count), dim3(256), 0, s, d);
}
void group_symm_h(const GroupStep* d, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_group_symm_h, dim3(16, count), dim3(256), 0, s, d);
}
void group_jacobi(const GroupStep* d, int count, int pmax, hipStream_t s) {
  static bool lds_set = [] {
    return hipFuncSetAttribute((const void*)k_group_jacobi,
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               2 * 96 * 96 * (int)sizeof(double)) == hipSuccess;
  }();
  (void)lds_set;
  // the matrix and its eigenvectors both in LDS up to p = 96 (144 KB)
  const int vt_lds = pmax <= 96 ? 1 : 0;
  hipLaunchKernelGGL(k_group_jacobi, dim3(count), dim3(kJacThreads),
                     (size_t)(vt_lds + 1) * pmax * pmax * sizeof(double), s, d, vt_lds);
}
void group_resid(const GroupStep* d, int count, bool last, hipStream_t s) {
  hipLaunchKernelGGL(k_group_resid, dim3(count), dim3(256), 0, s, d, last ? 1 : 0);
}
void group_shift(const GroupStep* d, int count, long long max_pn, hipStream_t s) {
  hipLaunchKernelGGL(k_group_shift, dim3(gblocks(max_pn), count), dim3(256), 0, s, d);
}
void group_restart(const GroupStep* d, int count, long long max_pn, hipStream_t s) {
  hipLaunchKernelGGL(k_group_restart, dim3(gblocks(max_pn), count), dim3(256), 0, s, d);
}
void group_dense(const GroupStep* d, int count, int pmax, hipStream_t s) {
  hipLaunchKernelGGL(k_group_dense_in, dim3(16, count), dim3(256), 0, s, d);
  group_jacobi(d, count, pmax, s);
  hipLaunchKernelGGL(k_group_dense_out, dim3(16, count), dim3(256), 0, s, d);
}
void group_spectrum(const GroupStep* d, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_group_spectrum, dim3(count), dim3(256), 0, s, d);
}
void group_norm(const GroupStep* d, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_group_norm, dim3(count), dim3(256), 0, s, d);
}
void group_zero_max(const GroupStep* d, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_group_zero_max, dim3((count + 63) / 64), dim3(64), 0, s, d, count);
}
void group_advance(const GroupStep* d, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_group_advance, dim3((count + 63) / 64), dim3(64), 0, s, d, count);
}

}  // namespace hotrg
