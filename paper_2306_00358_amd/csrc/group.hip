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
// problem, eigs.hip and stedc.hip); small environments (n <= 128) go through
// the same two kernels whole, copied into H with a zero row and column when
// n is odd (one extra eigenvalue 0 below the spectrum).
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

// Small environments (n <= 128) are diagonalised whole by the Householder
// reduction and the divide and conquer: H = M padded with zero rows and
// columns to the size p (a padded index adds an eigenvalue 0 below the
// spectrum), and the eigenvectors' first n components become the rows of X.
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
  group_sytrd(d, count, pmax, s);
  group_stedc(d, count, pmax, s);
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
