// Leading eigenpairs of the environment matrix M (n x n, symmetric positive
// semi-definite) in FP64 by block subspace iteration with Rayleigh-Ritz.
//
// The projector of one coarse-graining step needs only the D' leading
// eigenvectors of M (plus the next eigenvalue for the cut gap), while a full
// dense eigensolver spends most of its time in a memory-bound
// tridiagonalisation of all n = D^2 rows.  The environment spectrum decays
// fast, so iterating a block of p > D' vectors converges in a few sweeps at
// the rate lambda_{p+1} / lambda_{D'} per sweep.
//
// One sweep:  Y = V M  (rows of V are the p basis vectors)
//             V = orth(Y) by shifted Cholesky-QR three times (Fukaya et al.,
//             "Shifted Cholesky QR for computing the QR factorization of
//             ill-conditioned matrices", SIAM J. Sci. Comput. 42 (2020)):
//             G = Y Y^T + s I, G = R^T R, V = R^-T Y; the first pass uses
//             s = 11 (n p + p(p+1)) u trace(G), the next two s = 0.
// Check:      H = V (V M)^T, H = Z diag(theta) Z^T (rocSOLVER on p x p),
//             Ritz vectors X = Z^T V, residuals |(Z^T Y)_i - theta_i X_i|.
// Converged when the residuals of the `need` leading pairs are below
// tol * theta_1; otherwise the sweeps continue from X.  All products are
// FP64 MFMA GEMMs; the host reads p Ritz values and residuals per check.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <cmath>
#include <vector>

#include "internal.h"

namespace hotrg {

// deterministic start block: splitmix64 of the element index -> [-1, 1)
__global__ void k_seed_block(double* V, long long count, unsigned long long seed) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < count;
       e += (long long)gridDim.x * blockDim.x) {
    unsigned long long z = (unsigned long long)e + seed * 0x9E3779B97F4A7C15ULL;
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    V[e] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
}

// G (p x p, row-major) -> RinvT = (R^-1)^T where G + s I = R^T R, s =
// shift_rel * trace(G).  One workgroup of 1024 threads (32 x 32); G lives
// in LDS (p <= 128).  Right-looking Cholesky: column j updates the trailing
// upper triangle with the unscaled row j divided by its pivot, while row j
// of R is written, scaled, into the strict lower triangle (as R^T) and the
// pivots into rdiag -- one barrier per column.  Then Gauss-Jordan on the
// upper triangle: X = R^-1 from X = I eliminating columns p-1 .. 0, again
// one barrier per column (row k is scaled one column later, when nothing
// reads it any more).  *fail is set if a pivot is not positive.
__global__ __launch_bounds__(1024) void k_chol_inv(const double* __restrict__ G, int p,
                                                   double shift_rel, double* __restrict__ RinvT,
                                                   int* fail) {
  extern __shared__ double A[];  // p * p, then rdiag (p), then 1024 scratch
  double* rdiag = A + p * p;
  double* red = rdiag + p;
  const int t = threadIdx.x;
  const int tx = t & 31, ty = t >> 5;
  double tr = 0.0;
  for (int i = ty; i < p; i += 32)
    for (int j = tx; j < p; j += 32) {
      const double v = i <= j ? G[i * p + j] : G[j * p + i];  // upper part, mirrored
      A[i * p + j] = v;
      if (i == j) tr += v;
    }
  red[t] = tr;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  const double shift = shift_rel * red[0];
  if (t < p) A[t * p + t] += shift;
  __syncthreads();
  for (int j = 0; j < p; ++j) {
    const double d = A[j * p + j];
    if (!(d > 0.0)) {
      if (t == 0) *fail = 1;
      return;  // uniform: every thread reads the same pivot
    }
    const double rd = sqrt(d), inv_d = 1.0 / d, inv_rd = 1.0 / rd;
    // R^T column j (lower triangle) and the pivot
    if (ty == 0) {
      for (int k = j + 1 + tx; k < p; k += 32) A[k * p + j] = A[j * p + k] * inv_rd;
      if (tx == 0) rdiag[j] = rd;
    }
    // trailing update of the upper triangle, rows/cols j+1 .. p-1
    for (int i = j + 1 + ty; i < p; i += 32) {
      const double aji = A[j * p + i] * inv_d;
      for (int k = i + tx; k < p; k += 32) A[i * p + k] -= aji * A[j * p + k];
    }
    __syncthreads();
  }
  // X = R^-1 in the upper triangle; R[i][k] = A[k*p + i] for i < k
  for (int i = ty; i < p; i += 32)
    for (int c = i + tx; c < p; c += 32) A[i * p + c] = i == c ? 1.0 : 0.0;
  __syncthreads();
  for (int k = p - 1; k >= 0; --k) {
    const double inv_rkk = 1.0 / rdiag[k];
    if (k + 1 < p && ty == 31)  // scale row k+1 (final since the last column)
      for (int c = k + 1 + tx; c < p; c += 32) A[(k + 1) * p + c] /= rdiag[k + 1];
    for (int i = ty; i < k; i += 32) {
      const double f = A[k * p + i] * inv_rkk;  // R[i][k] / R[k][k]
      for (int c = k + tx; c < p; c += 32) A[i * p + c] -= f * A[k * p + c];
    }
    __syncthreads();
  }
  if (ty == 0)
    for (int c = tx; c < p; c += 32) A[c] /= rdiag[0];
  __syncthreads();
  // RinvT[i][k] = X[k][i] (lower triangular)
  for (int i = ty; i < p; i += 32)
    for (int k = tx; k < p; k += 32) RinvT[i * p + k] = k <= i ? A[k * p + i] : 0.0;
}

__global__ void k_symmetrize_small(double* H, int p) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < p * p; e += gridDim.x * blockDim.x) {
    const int i = e / p, j = e % p;
    if (i < j) {
      const double v = 0.5 * (H[i * p + j] + H[j * p + i]);
      H[i * p + j] = v;
      H[j * p + i] = v;
    }
  }
}

// res[i] = |Yx[i,:] - theta[i] X[i,:]| (one block per row, fixed-order tree)
__global__ void k_ritz_residual(const double* __restrict__ Yx, const double* __restrict__ X,
                                const double* __restrict__ theta, int n, double* res) {
  __shared__ double red[256];
  const int i = blockIdx.x, t = threadIdx.x;
  const double th = theta[i];
  double s = 0.0;
  for (int j = t; j < n; j += 256) {
    const double d = Yx[(long long)i * n + j] - th * X[(long long)i * n + j];
    s += d * d;
  }
  red[t] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  if (t == 0) res[i] = sqrt(red[0]);
}

// trace of M (n x n) -> *out, fixed-order tree
__global__ void k_trace(const double* __restrict__ M, int n, double* out) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  double s = 0.0;
  for (int i = t; i < n; i += 256) s += M[(long long)i * n + i];
  red[t] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  if (t == 0) *out = red[0];
}

void launch_trace(const double* M, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_trace, dim3(1), dim3(256), 0, s, M, n, out);
}

static inline int splitk_chunk(int K) {
  // about 64 partial products, each K chunk a multiple of 16
  int c = (K + 63) / 64;
  c = (c + 15) / 16 * 16;
  return c < 16 ? 16 : c;
}

size_t topk_workspace_doubles(int n, int p) {
  const size_t pn = (size_t)p * n, pp = (size_t)p * p;
  const int parts = (n + splitk_chunk(n) - 1) / splitk_chunk(n);
  return 4 * pn + (size_t)parts * pp + 4 * pp + 4 * (size_t)p + 16;
}

// Returns true and leaves theta (ascending, p values) in W and the Ritz
// vectors (rows, same order) in Xout (p x n) on convergence.
bool topk_eigs(rocblas_handle blas, const double* M, int n, int p, int need, double tol,
               double* ws, double* W, double* Xout, int* dinfo, int* iters, double* resid,
               hipStream_t s) {
  const size_t pn = (size_t)p * n, pp = (size_t)p * p;
  const int kc = splitk_chunk(n);
  const int parts = (n + kc - 1) / kc;
  double* V = ws;
  double* Y = V + pn;
  double* T2 = Y + pn;
  double* Yx = T2 + pn;
  double* part = Yx + pn;
  double* G = part + (size_t)parts * pp;
  double* Rt = G + pp;
  double* H = Rt + pp;
  double* E = H + pp;          // p (tridiagonal work for dsyevd)
  double* res = E + pp;        // p
  int* fail = (int*)(res + p); // 1 int
  const size_t lds = ((size_t)p * p + p + 1024) * sizeof(double);
  const double u = std::ldexp(1.0, -53);
  const double shift_rel = 11.0 * ((double)n * p + (double)p * (p + 1)) * u;

  static bool lds_set = [] {
    return hipFuncSetAttribute((const void*)k_chol_inv, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(((size_t)128 * 128 + 128 + 1024) * sizeof(double))) ==
           hipSuccess;
  }();
  if (!lds_set || p > 128) return false;
  (void)hipMemsetAsync(fail, 0, sizeof(int), s);
  hipLaunchKernelGGL(k_seed_block, dim3(256), dim3(256), 0, s, V, (long long)pn, 12345ULL);

  // one orthonormalisation of rows of Y into V
  auto orth = [&](const double* Yin, double* Vout) {
    const double* src = Yin;
    for (int pass = 0; pass < 3; ++pass) {
      gemm_f64_splitk(src, n, src, n, B_KCONTIG, G, p, p, p, n, kc, part, s);
      hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(1024), lds, s, G, p,
                         pass == 0 ? shift_rel : 0.0, Rt, fail);
      double* dst = (pass == 2) ? Vout : (src == T2 ? Y : T2);
      if (dst == src) dst = (src == Y) ? T2 : Y;
      gemm_f64(Rt, p, src, n, B_NCONTIG, dst, out_rowmajor(n), p, n, p, nullptr, s);
      src = dst;
    }
  };

  int it = 0, q = 3;
  const int max_it = 80;
  double prev = 1e300;
  std::vector<double> th(p), rs(p);
  while (true) {
    for (int r = 0; r < q; ++r) {
      gemm_f64(V, n, M, n, B_NCONTIG, Y, out_rowmajor(n), p, n, n, nullptr, s);
      orth(Y, V);
      ++it;
    }
    // Rayleigh-Ritz
    gemm_f64(V, n, M, n, B_NCONTIG, Y, out_rowmajor(n), p, n, n, nullptr, s);
    gemm_f64_splitk(V, n, Y, n, B_KCONTIG, H, p, p, p, n, kc, part, s);
    hipLaunchKernelGGL(k_symmetrize_small, dim3(16), dim3(256), 0, s, H, p);
    if (rocsolver_dsyevd(blas, rocblas_evect_original, rocblas_fill_lower, p, H, p, W, E, dinfo) !=
        rocblas_status_success)
      return false;
    // H now holds Z column-major: row i of Z^T is H[i*p .. i*p+p)
    gemm_f64(H, p, V, n, B_NCONTIG, Xout, out_rowmajor(n), p, n, p, nullptr, s);
    gemm_f64(H, p, Y, n, B_NCONTIG, Yx, out_rowmajor(n), p, n, p, nullptr, s);
    hipLaunchKernelGGL(k_ritz_residual, dim3(p), dim3(256), 0, s, Yx, Xout, W, n, res);
    int hinfo[2] = {0, 0};
    (void)hipMemcpyAsync(th.data(), W, p * sizeof(double), hipMemcpyDeviceToHost, s);
    (void)hipMemcpyAsync(rs.data(), res, p * sizeof(double), hipMemcpyDeviceToHost, s);
    (void)hipMemcpyAsync(&hinfo[0], dinfo, sizeof(int), hipMemcpyDeviceToHost, s);
    (void)hipMemcpyAsync(&hinfo[1], fail, sizeof(int), hipMemcpyDeviceToHost, s);
    if (hipStreamSynchronize(s) != hipSuccess) return false;
    if (hinfo[0] != 0 || hinfo[1] != 0) return false;
    const double t1 = th[p - 1];
    if (!(t1 > 0.0)) return false;
    double top = 0.0;
    for (int i = 0; i < need; ++i) top = std::fmax(top, rs[p - 1 - i] / t1);
    if (iters) *iters = it;
    if (resid) *resid = top;
    if (top <= tol) return true;
    if (it >= max_it || !(top < 0.5 * prev)) return false;
    prev = top;
    double rate = th[p - need] > 0.0 ? th[0] / th[p - need] : 0.5;
    rate = std::fmin(std::fmax(rate, 1e-6), 0.95);
    q = (int)std::ceil(std::log(tol / top) / std::log(rate));
    q = q < 1 ? 1 : (q > max_it - it ? max_it - it : q);
    // continue from the Ritz vectors
    (void)hipMemcpyAsync(V, Xout, pn * sizeof(double), hipMemcpyDeviceToDevice, s);
  }
}

}  // namespace hotrg
