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
// One sweep:  Y = V (M - sigma I)  (rows of V are the p basis vectors)
//             V = orth(Y) by shifted Cholesky-QR (Fukaya et al., "Shifted
//             Cholesky QR for computing the QR factorization of
//             ill-conditioned matrices", SIAM J. Sci. Comput. 42 (2020)):
//             G = Y Y^T + s I, G = R^T R, V = R^-T Y; the first two passes
//             factor the diagonally scaled G with s = 11 (n p + p(p+1)) u
//             trace, the third with s = 0.  (When M's spectrum falls to
//             rounding noise within the block -- deep in an ordered phase --
//             one shifted pass leaves a basis too ill-conditioned for an
//             unshifted Cholesky; a second shifted pass brings it within
//             reach, and the third restores orthonormality to rounding.)
//             V = R^-T Y is a blocked triangular solve (k_trsm_rows).
//             Before a check all three passes run.  Between checks V only
//             has to stay a well-conditioned basis of the same span: one
//             pass, then a second that the device reduces to R = I when G is
//             already the identity to 1e-2 -- after the first pass it is
//             typically so to 1e-7..1e-4, except in a solve's first sweep
//             (and once no such check misses, only the first sweep after a
//             check is checked).
// Check:      H = V (V M)^T, H = Z diag(theta) Z^T (Householder reduction to
//             tridiagonal form in one workgroup, k_sytrd_small, then divide
//             and conquer on the tridiagonal in another, k_stedc_small in
//             stedc.hip, and one small GEMM for Z^T = Z_T^T Q^T),
//             Ritz vectors X = Z^T V, residuals |(Z^T Y)_i - theta_i X_i|.
// Converged when the residuals of the `need` leading pairs are below
// tol * theta_1; otherwise the sweeps continue from X.  The first check
// comes after q_first sweeps.  On convergence `enough` estimates the fewest
// sweeps that would have met the tolerance: the residual of the slowest
// needed pair shrinks by about theta_min / theta_need per sweep, so a result
// k such factors below tol was k sweeps more than necessary.  The caller
// starts the next solve of the same kind from that estimate plus one, so most
// solves take a single Rayleigh-Ritz without sweeping far past convergence.
// All products are FP64 MFMA GEMMs; the host reads p Ritz values and
// residuals per check.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace hotrg {

typedef double d4 __attribute__((ext_vector_type(4)));

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
// shift_rel * trace(G).  One workgroup of 256 threads as a 16 x 16 grid;
// thread (ty, tx) keeps the elements (ty + 16a, tx + 16b), a, b < 8, of the
// working matrix in registers (p <= 128, p a multiple of 16; indices past p
// are clamped, and those registers are never published or stored).
//
// Blocked right-looking Cholesky with blocks of 8 columns: the owners of the
// block's 8 rows (final by then) publish them in LDS; thread c < p then
// factors the 8 x 8 diagonal block itself (the same operations on the same
// data in every such thread) and forms column c of the block rows of R by
// forward substitution, straight into R in LDS; after a second barrier every
// thread applies the rank-8 update to its elements.  The inverse X = R^-1 is
// eliminated from X = I block by block from the bottom the same way: thread c
// back-substitutes column c of the block's rows in place, and every row takes
// the rank-8 update with column j0.. of R (zero below the diagonal, so rows
// at and below the block are left alone; the block's rows then take their
// final values).  Two barriers per block of 8 columns.
//
// R starts as zeros in LDS, so every load below is unconditional: rows and
// columns that are already finished take updates nobody reads again, which
// costs less than the waits a load under a branch would.  X^T leaves through
// LDS for coalesced stores.  *fail is set if a pivot is not positive.
constexpr int kCholThreads = 256;

__device__ __forceinline__ void chol_inv_body(const double* __restrict__ G, int p,
                                              double shift_rel, int scale, double identity_tol,
                                              double* __restrict__ RinvT, int* fail) {
  extern __shared__ double lds[];
  double* R = lds;             // p * p: R (upper, zeros below), later X^T
  double* P = R + p * p;       // 2 x 8 x 128 published rows
  __shared__ int bad;
  __shared__ double dev[kCholThreads];
  __shared__ double dsc[128];  // diag(G)^-1/2 when scaling, else 1
  const int t = threadIdx.x;
  const int tx = t & 15, ty = t >> 4;
  const int pm = p - 1;
  double A[8][8];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int i = min(ty + 16 * a, pm), k = min(tx + 16 * b, pm);
      A[a][b] = G[min(i, k) * p + max(i, k)];  // upper part, mirrored
    }
  if (identity_tol > 0.0) {
    // G already the identity to within identity_tol: R^-1 = I
    double d = 0.0;
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const int i = ty + 16 * a, k = tx + 16 * b;
        if (i < p && k < p) d = fmax(d, fabs(A[a][b] - (i == k ? 1.0 : 0.0)));
      }
    dev[t] = d;
    __syncthreads();
    double mx = 0.0;
    for (int i = 0; i < kCholThreads; ++i) mx = fmax(mx, dev[i]);
    if (mx <= identity_tol) {  // uniform: every thread reduced the same values
      for (int e = t; e < p * p; e += kCholThreads) RinvT[e] = (e / p == e % p) ? 1.0 : 0.0;
      return;
    }
  }
  for (int e = t; e < p * p; e += kCholThreads) R[e] = 0.0;
  // diagonal: the owners publish it
  if (tx == ty) {
#pragma unroll
    for (int a = 0; a < 8; ++a)
      if (ty + 16 * a < p) P[ty + 16 * a] = A[a][a];
  }
  if (t == 0) bad = 0;
  __syncthreads();
  // with `scale`, factor D^-1 G D^-1 (D = diag(G)^1/2) instead of G: the
  // columns' lengths drop out of the conditioning, and the scaling is put
  // back into the rows of R^-1 at the end
  if (t < 128) dsc[t] = (scale && t < p) ? 1.0 / sqrt(P[t]) : 1.0;
  __syncthreads();
  if (scale) {
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const double dr = dsc[min(ty + 16 * a, pm)];
#pragma unroll
      for (int b = 0; b < 8; ++b) A[a][b] *= dr * dsc[min(tx + 16 * b, pm)];
    }
  }
  // trace (of the matrix factored), every thread sums in the same order
  double tr = 0.0;
  if (scale)
    tr = (double)p;
  else
    for (int i = 0; i < p; ++i) tr += P[i];
  const double shift = shift_rel * tr;
  if (tx == ty) {
#pragma unroll
    for (int a = 0; a < 8; ++a) A[a][a] += shift;
  }
  __syncthreads();  // everyone has read the trace before P is reused

  const int nblk = p >> 3;
  for (int J = 0; J < nblk; ++J) {
    const int j0 = 8 * J, aj = j0 >> 4, tj = j0 & 15;
    double* Pb = P + (J & 1) * 1024;
    if (ty >= tj && ty < tj + 8) {
#pragma unroll
      for (int a = 0; a < 8; ++a)
        if (a == aj) {
#pragma unroll
          for (int b = 0; b < 8; ++b) Pb[(ty - tj) * 128 + tx + 16 * b] = A[a][b];
        }
    }
    __syncthreads();
    if (t < p && t >= j0) {
      // the 8 x 8 diagonal block: L[r][c] (c >= r) becomes R[j0+r][j0+c]
      double L[8][8], inv[8];
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int c = r; c < 8; ++c) L[r][c] = Pb[r * 128 + j0 + c];
      bool ok = true;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const double d = L[r][r];
        ok = ok && d > 0.0;
        // 1 / sqrt(d) from v_rsq_f64 and two Newton steps; sqrt(d) = d / sqrt(d)
        const double dd = d > 0.0 ? d : 1.0;
        double y = __builtin_amdgcn_rsq(dd);
        y = fma(y, fma(-0.5 * dd * y, y, 0.5), y);
        y = fma(y, fma(-0.5 * dd * y, y, 0.5), y);
        inv[r] = y;
        L[r][r] = dd * y;
#pragma unroll
        for (int c = r + 1; c < 8; ++c) L[r][c] *= inv[r];
#pragma unroll
        for (int r2 = r + 1; r2 < 8; ++r2)
#pragma unroll
          for (int c = r2; c < 8; ++c) L[r2][c] -= L[r][r2] * L[r][c];
      }
      if (!ok) bad = 1;
      if (t >= j0 + 8) {
        double v[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          double w = Pb[r * 128 + t];
#pragma unroll
          for (int m = 0; m < r; ++m) w -= L[m][r] * v[m];
          v[r] = w * inv[r];
          R[(j0 + r) * p + t] = v[r];
        }
      } else {
        const int cc = t - j0;  // column inside the block
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          double v = 0.0;
#pragma unroll
          for (int c = r; c < 8; ++c) v = cc == c ? L[r][c] : v;
          R[(j0 + r) * p + t] = v;
        }
      }
    }
    __syncthreads();
    if (bad) {
      if (t == 0) *fail = 1;
      return;  // uniform: every thread read the same flag after the barrier
    }
    // register rows / columns whose indices all lie before j0 + 8 are
    // finished: skip them (a uniform test)
    double Ri[8][8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      if (16 * a + 15 < j0 + 8) continue;
      const int i = min(ty + 16 * a, pm);
#pragma unroll
      for (int r = 0; r < 8; ++r) Ri[a][r] = R[(j0 + r) * p + i];
    }
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      if (16 * b + 15 < j0 + 8) continue;
      const int k = min(tx + 16 * b, pm);
      double Rk[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) Rk[r] = R[(j0 + r) * p + k];
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        if (16 * a + 15 < j0 + 8) continue;
        double v = A[a][b];
#pragma unroll
        for (int r = 0; r < 8; ++r) v -= Ri[a][r] * Rk[r];
        A[a][b] = v;
      }
    }
  }
  // X = I in registers
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) A[a][b] = (ty + 16 * a == tx + 16 * b) ? 1.0 : 0.0;
  __syncthreads();  // the last reads of P and R rows are done
  for (int J = nblk - 1; J >= 0; --J) {
    const int j0 = 8 * J, aj = j0 >> 4, tj = j0 & 15;
    double* Pb = P + (J & 1) * 1024;
    if (ty >= tj && ty < tj + 8) {
#pragma unroll
      for (int a = 0; a < 8; ++a)
        if (a == aj) {
#pragma unroll
          for (int b = 0; b < 8; ++b) Pb[(ty - tj) * 128 + tx + 16 * b] = A[a][b];
        }
    }
    __syncthreads();
    if (t < p) {  // column t of the block rows, back substitution in place
      double L[8][8], inv[8], x[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
#pragma unroll
        for (int c = r; c < 8; ++c) L[r][c] = R[(j0 + r) * p + j0 + c];
        inv[r] = 1.0 / L[r][r];
        x[r] = Pb[r * 128 + t];
      }
#pragma unroll
      for (int r = 7; r >= 0; --r) {
        double v = x[r];
#pragma unroll
        for (int m = r + 1; m < 8; ++m) v -= L[r][m] * x[m];
        x[r] = v * inv[r];
        Pb[r * 128 + t] = x[r];
      }
    }
    __syncthreads();
    // X is upper triangular: the block's rows vanish before column j0, and
    // rows from j0 + 8 on are final; skip those register groups (uniform)
    double Xb[8][8];  // the block's final rows at the thread's own columns
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      if (16 * b + 15 < j0) continue;
#pragma unroll
      for (int r = 0; r < 8; ++r) Xb[b][r] = Pb[r * 128 + tx + 16 * b];
    }
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      if (16 * a >= j0 + 8) continue;
      const int i = ty + 16 * a;
      const int ic = min(i, pm);
      double Rr[8];  // R[i][j0 + r]: zero for rows at or below the block
#pragma unroll
      for (int r = 0; r < 8; ++r) Rr[r] = R[ic * p + j0 + r];
      const bool in_blk = i >= j0 && i < j0 + 8;
      const int rb = i - j0;
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        if (16 * b + 15 < j0) continue;
        double v = A[a][b];
#pragma unroll
        for (int r = 0; r < 8; ++r) v -= Rr[r] * Xb[b][r];
        double xr = Xb[b][0];
#pragma unroll
        for (int r = 1; r < 8; ++r) xr = rb == r ? Xb[b][r] : xr;
        A[a][b] = in_blk ? xr : v;
      }
    }
  }
  __syncthreads();  // all reads of R are done: reuse it for X^T
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int i = ty + 16 * a, k = tx + 16 * b;
      // with scaling R = R^ D, so row i of R^-1 = D^-1 R^^-1 carries G_ii^-1/2
      if (i < p && k < p) R[k * p + i] = A[a][b] * dsc[i];
    }
  __syncthreads();
  for (int e = t; e < p * p; e += kCholThreads) RinvT[e] = R[e];
}


// Factor-only Cholesky of a sweep's Gram matrix (Q = R^-T D^-1 Y then comes
// from k_trsm_rows): R with R^T R = D^-1 G D^-1 + s I (`scale`; D = diag(G)^1/2) or
// G + s I, s = shift_rel * trace of the matrix factored, into Rout (p x p
// row-major, zeros below the diagonal) and D^-1 (ones without `scale`) into
// Rout + p * p; with identity_tol > 0 and G the identity to within it, R = I.
// One workgroup of GW x GW threads (GW = 32 for p <= 128, 16 for p <= 64:
// the same register tiles, and barriers over 4 waves instead of 16); thread
// (ty, tx) keeps the elements (ty + GW a, tx + GW b), a, b < 4, in registers
// (p a multiple of 16; indices past p are clamped and never published).  Blocks of 8
// columns: the owners of the block's 8 rows publish them in LDS; the first
// wave factors the 8 x 8 diagonal block, one column per lane, the values of
// other columns by readlane (1/sqrt of a pivot from v_rsq_f64 and two Newton
// steps), into LDS; after a second barrier thread c < p forms column c of the
// block's rows of R, into LDS (8 doubles per column) and Rout; after a third
// every thread takes the rank-8 update on its register tiles that still
// matter (not wholly finished, not wholly past p).  Only the current block
// lives in LDS, so four waves per SIMD fit with their register tiles.  *fail
// is set if a pivot is not positive.

// value of v in lane l of the wave (l uniform)
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <int GW>
__global__ __launch_bounds__(GW * GW) void k_chol_factor(const double* __restrict__ G, int p,
                                                               double shift_rel, int scale,
                                                               double identity_tol,
                                                               double* __restrict__ Rout,
                                                               int* fail, int* missed) {
  __shared__ double Pb[8 * 128];                 // the block's rows of the working matrix
  __shared__ __align__(16) double Rb[128 * 8];   // the block's rows of R, by column
  __shared__ __align__(16) double Ls[64];
  __shared__ double dg[128], dsc[128], red[GW * GW / 64], Li[8];
  __shared__ int bad;
  const int t = threadIdx.x, tx = t % GW, ty = t / GW;
  const int pm = p - 1;
  double A[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = min(ty + GW * a, pm), k = min(tx + GW * b, pm);
      A[a][b] = G[min(i, k) * p + max(i, k)];  // upper part, mirrored
    }
  if (identity_tol > 0.0) {
    double d = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int i = ty + GW * a, k = tx + GW * b;
        if (i < p && k < p) d = fmax(d, fabs(A[a][b] - (i == k ? 1.0 : 0.0)));
      }
    for (int o = 32; o > 0; o >>= 1) d = fmax(d, __shfl_xor(d, o, 64));
    if ((t & 63) == 0) red[t >> 6] = d;
    __syncthreads();
    double mx = 0.0;
    for (int w = 0; w < GW * GW / 64; ++w) mx = fmax(mx, red[w]);
    if (mx <= identity_tol) {  // uniform: every thread reduced the same values
      for (int e = t; e < p * p; e += GW * GW) Rout[e] = (e / p == e % p) ? 1.0 : 0.0;
      if (t < p) Rout[p * p + t] = 1.0;
      return;
    }
    if (missed && t == 0) *missed += 1;  // the check found a real factorisation to do
  }
  if (tx == ty) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
      if (ty + GW * a < p) dg[ty + GW * a] = A[a][a];
  }
  if (t == 0) bad = 0;
  __syncthreads();
  if (t < 128) dsc[t] = (scale && t < p) ? 1.0 / sqrt(dg[t]) : 1.0;
  // trace of the matrix factored, every thread summing in the same order
  double tr = 0.0;
  if (scale)
    tr = (double)p;
  else
    for (int i = 0; i < p; ++i) tr += dg[i];
  __syncthreads();
  if (scale) {
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const double dr = dsc[min(ty + GW * a, pm)];
#pragma unroll
      for (int b = 0; b < 4; ++b) A[a][b] *= dr * dsc[min(tx + GW * b, pm)];
    }
  }
  const double shift = shift_rel * tr;
  if (tx == ty) {
#pragma unroll
    for (int a = 0; a < 4; ++a) A[a][a] += shift;
  }

  const int nblk = p >> 3;
  for (int J = 0; J < nblk; ++J) {
    const int j0 = 8 * J, aj = j0 / GW, tj = j0 % GW;
    if (ty >= tj && ty < tj + 8) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
        if (a == aj) {
#pragma unroll
          for (int b = 0; b < 4; ++b) Pb[(ty - tj) * 128 + tx + GW * b] = A[a][b];
        }
    }
    __syncthreads();
    if (t < 64) {
      // the 8 x 8 diagonal block, right-looking, one column per lane (lane
      // c0 < 8 keeps L[r][c0] -> R[j0+r][j0+c0] in x[r], zeros below the
      // diagonal; the other lanes repeat columns and are not used); the
      // pivot and L[r][r2] of another column come from readlane, so no step
      // waits on LDS
      const int c0 = t & 7;
      double x[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) x[r] = r <= c0 ? Pb[r * 128 + j0 + c0] : 0.0;
      bool ok = true;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const double d = readlane_f64(x[r], r);
        ok = ok && d > 0.0;
        const double dd = d > 0.0 ? d : 1.0;
        double y = __builtin_amdgcn_rsq(dd);
        y = fma(y, fma(-0.5 * dd * y, y, 0.5), y);
        y = fma(y, fma(-0.5 * dd * y, y, 0.5), y);
        x[r] = c0 == r ? dd * y : (c0 > r ? x[r] * y : x[r]);
        if (t == r) Li[r] = y;
#pragma unroll
        for (int r2 = r + 1; r2 < 8; ++r2) {
          const double lr = readlane_f64(x[r], r2);  // L[r][r2]
          if (c0 >= r2) x[r2] -= lr * x[r];
        }
      }
      if (t < 8) {
#pragma unroll
        for (int r = 0; r < 8; ++r) Ls[t * 8 + r] = x[r];  // column t: Ls[c * 8 + r] = L[r][c]
      }
      if (t == 0 && !ok) bad = 1;
    }
    __syncthreads();
    if (t < p) {
      // column t of the block's rows of R: forward substitution past the
      // block, the factor itself inside it, zeros before it
      double v[8];
      if (t >= j0 + 8) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          double w = Pb[r * 128 + t];
#pragma unroll
          for (int m = 0; m < r; ++m) w -= Ls[r * 8 + m] * v[m];
          v[r] = w * Li[r];
        }
      } else {
        const int cc = t - j0;
#pragma unroll
        for (int r = 0; r < 8; ++r) v[r] = cc >= 0 ? Ls[min(max(cc, 0), 7) * 8 + r] : 0.0;
      }
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        if (t >= j0) Rb[t * 8 + r] = v[r];
        Rout[(j0 + r) * p + t] = v[r];
      }
    }
    __syncthreads();
    if (bad) {
      if (t == 0) *fail = 1;
      return;  // uniform: every thread read the same flag after the barrier
    }
    // rank-8 update; register rows / columns wholly before j0 + 8 are
    // finished and those wholly past p hold only clamped copies: both are
    // skipped (uniform tests); the others take it even where an element is
    // finished -- nobody reads those again
#pragma unroll
    for (int h = 0; h < 8; h += 4) {  // two rank-4 halves keep the operands few
      double Ri[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        if (GW * a + GW - 1 < j0 + 8 || GW * a >= p) continue;
        const int i = min(ty + GW * a, pm);
#pragma unroll
        for (int r = 0; r < 4; ++r) Ri[a][r] = Rb[i * 8 + h + r];
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        if (GW * b + GW - 1 < j0 + 8 || GW * b >= p) continue;
        const int k = min(tx + GW * b, pm);
        double Rk[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) Rk[r] = Rb[k * 8 + h + r];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          if (GW * a + GW - 1 < j0 + 8 || GW * a >= p) continue;
          double v = A[a][b];
#pragma unroll
          for (int r = 0; r < 4; ++r) v -= Ri[a][r] * Rk[r];
          A[a][b] = v;
        }
      }
    }
  }
  if (t < p) Rout[p * p + t] = dsc[t];
}

// Q = R^-T D^-1 Y for the rows of Y (p x n, row-major): with L = R^T (lower
// triangular), L Q = D^-1 Y is solved by blocks of 16 rows,
//   Q_b = L_bb^-1 (D_b^-1 Y_b - sum_{a<b} L_ba Q_a),
// where R and D^-1 are the output of k_chol_factor (R at Rf, D^-1 at
// Rf + p * p).  One workgroup per 64 columns; each of its 4 waves owns 16
// columns and keeps their Q blocks in registers: in the accumulator layout of
// v_mfma_f64_16x16x4f64 (lane j + 16 l holds rows l + 4 v of column j) value
// v of a lane is exactly the B operand the next products take at k step v,
// so the blocks never leave the registers until the end.  R is staged in LDS
// (the A operands of every wave) and the 16 x 16 inverses of the diagonal
// blocks are formed there by forward substitution, one column per thread.
// p a multiple of 16, at most 128; columns past n are computed but not
// stored.
constexpr int kTrsmCols = 64;
__global__ __launch_bounds__(256) void k_trsm_rows(const double* __restrict__ Rf, int p,
                                                   const double* __restrict__ Y, int n,
                                                   double* __restrict__ Q) {
  extern __shared__ double lds[];
  double* Rs = lds;              // p x p
  double* Li = lds + p * p;      // p / 16 blocks of 16 x 16: Li[b][i][c]
  const double* dinv = Rf + p * p;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int nb = p >> 4;
  const int j = lane & 15, l = lane >> 4;
  const int col = blockIdx.x * kTrsmCols + wave * 16 + j;
  const int cc = col < n ? col : n - 1;
  // this lane's rows of D^-1 Y, loaded before anything waits on them
  d4 y[8];
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    if (b >= nb) break;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * b + l + 4 * v;
      y[b][v] = Y[(long long)r * n + cc];
    }
  }
  {
    // p * p is a multiple of 256 doubles: 16-byte copies, 8 in flight
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2* src = (const d2*)Rf;
    d2* dst = (d2*)Rs;
#pragma unroll 8
    for (int e = t; e < p * p / 2; e += 256) dst[e] = src[e];
  }
  __syncthreads();
  if (t < 16 * nb) {
    // column c of the inverse of L_bb, L_bb[i][j] = R[16b + j][16b + i]
    const int b = t >> 4, c = t & 15, o = 16 * b;
    double x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      double v = i == c ? 1.0 : 0.0;
#pragma unroll
      for (int j = 0; j < i; ++j) v -= Rs[(o + j) * p + o + i] * x[j];
      x[i] = v / Rs[(o + i) * p + o + i];
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) Li[(b * 16 + i) * 16 + c] = x[i];
  }
  __syncthreads();
  d4 q[8];
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    if (b >= nb) break;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      if (a >= b) break;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        // A[i][k] = L[16b + i][16a + 4s + k] = R[16a + 4s + k][16b + i], lane i + 16k
        const double av = Rs[(16 * a + 4 * s + l) * p + 16 * b + j];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, q[a][s], acc, 0, 0, 0);
      }
    }
    d4 x;
#pragma unroll
    for (int v = 0; v < 4; ++v) x[v] = dinv[16 * b + l + 4 * v] * y[b][v] - acc[v];
    d4 qb = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const double av = Li[(b * 16 + j) * 16 + 4 * s + l];
      qb = __builtin_amdgcn_mfma_f64_16x16x4f64(av, x[s], qb, 0, 0, 0);
    }
    q[b] = qb;
  }
  if (col < n) {
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      if (b >= nb) break;
#pragma unroll
      for (int v = 0; v < 4; ++v) Q[(long long)(16 * b + l + 4 * v) * n + col] = q[b][v];
    }
  }
}

// One workgroup per problem of a batch; a problem whose gate reads 0 (its
// eigensolve has converged, or it has no steps left) is skipped.
__global__ __launch_bounds__(kCholThreads) void k_chol_inv_b(const CholItem* __restrict__ items,
                                                             int pass, int full) {
  const CholItem& it = items[blockIdx.x];
  if (it.gate && *it.gate == 0) return;
  chol_inv_body(it.G, it.p, pass < 2 ? it.shift_rel : 0.0, pass < 2 ? 1 : 0,
                (pass == 0 || full) ? 0.0 : 1e-2, it.Rt, it.fail);
}

void launch_chol_inv_batched(const CholItem* d_items, int count, int pmax, int pass, bool full,
                             hipStream_t s) {
  static bool lds_set = [] {
    return hipFuncSetAttribute((const void*)k_chol_inv_b,
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(((size_t)128 * 128 + 2048) * sizeof(double))) == hipSuccess;
  }();
  (void)lds_set;
  const size_t lds = ((size_t)pmax * pmax + 2048) * sizeof(double);
  hipLaunchKernelGGL(k_chol_inv_b, dim3(count), dim3(kCholThreads), lds, s, d_items, pass,
                     full ? 1 : 0);
}

// Householder reduction of a small symmetric matrix to tridiagonal form in
// one workgroup, for the Rayleigh-Ritz step (its tridiagonal eigenproblem
// goes to the divide and conquer of k_stedc_small).  H (p x p, symmetric, 3 <= p <=
// 128) lives in registers: thread t = 8 i + q holds row i's entries in
// columns q, q + 8, ..., so a matrix-vector product is 16 FMAs per thread and
// a reduction over 8 neighbouring lanes.  For k = 0 .. p-3 the entries of row
// k past the diagonal, x (the column, by symmetry), give v (v_0 = 1) and tau
// with (I - tau v v^T) x = beta e_1, and the trailing block takes
// A <- A - v w^T - w v^T, w = tau A v - (tau^2 / 2) (v^T A v) v (the standard
// symmetric two-sided update).  The reflectors are kept in LDS; Q = H_0 H_1
// ... H_{p-3} is then accumulated from the back, as Q^T in the same register
// layout, and written over H column-major as the reduction matrix the
// tridiagonal solver expects; d (p) and e (p - 1) receive the tridiagonal.
// Every loop has a fixed trip count and every sum a fixed order.
constexpr int kTrdThreads = 1024;
// threads of a launch for p rows: the 8 lanes of every row below p, whole
// waves, at least 128 (the threads that clear the 128-entry vectors); fewer
// waves than 1024 threads for small p make every barrier cheaper
static inline int trd_threads(int p) { return std::max(128, (8 * p + 63) / 64 * 64); }

// another lane of the same 8-lane group (DPP: quad_perm [1,0,3,2],
// quad_perm [2,3,0,1], row_half_mirror); every lane of the group is active
template <int kCtrl>
__device__ __forceinline__ double trd_dpp(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, kCtrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), kCtrl, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// sum over the 8-lane group, the same bits in every lane
__device__ __forceinline__ double trd_sum8(double v) {
  v += trd_dpp<0xB1>(v);
  v += trd_dpp<0x4E>(v);
  return v + trd_dpp<0x141>(v);
}

__device__ __forceinline__ void sytrd_body(double* __restrict__ H, int p, double* __restrict__ d,
                                           double* __restrict__ e) {
  // reflector k at Vr[128 k + c], zero outside its columns k+1 .. p-1; the
  // vectors of a step are likewise zero outside the trailing block, so the
  // register loops below need no bounds tests
  extern __shared__ double Vr[];
  __shared__ double vsa[2][128], wsa[128], wvs[128], taus[128];
  const int t = threadIdx.x, i = t >> 3, q = t & 7;
  const bool own = i < p;
  double a[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int c = q + 8 * r;
    a[r] = (own && c < p) ? H[i * p + c] : 0.0;
  }
  if (t < 128) wsa[t] = wvs[t] = 0.0;
  for (int k = 0; k + 2 < p; ++k) {
    const int o = k + 1;
    double* vs = vsa[k & 1];
    if (i == k) {
      // row k's eight owners (eight lanes of one wave) form the reflector
      // from their own entries and publish it with tau, beta and d_k
      double s2 = 0.0, x0 = 0.0, dk = 0.0;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int c = q + 8 * r;
        s2 += (c >= o && c < p) ? a[r] * a[r] : 0.0;
        x0 = c == o ? a[r] : x0;
        dk = c == k ? a[r] : dk;
      }
      const double nrm2 = trd_sum8(s2);
      x0 = trd_sum8(x0);  // one lane holds it, the others add zeros
      dk = trd_sum8(dk);
      double beta, tau, scale;
      if (nrm2 == 0.0) {
        beta = x0;
        tau = 0.0;
        scale = 0.0;
      } else {
        beta = -copysign(sqrt(nrm2), x0);
        tau = (beta - x0) / beta;
        scale = 1.0 / (x0 - beta);
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int c = q + 8 * r;
        const double v = c == o ? 1.0 : ((c > o && c < p) ? a[r] * scale : 0.0);
        vs[c] = v;
        Vr[128 * k + c] = v;
      }
      if (q == 0) {
        taus[k] = tau;
        e[k] = beta;
        d[k] = dk;
      }
    }
    __syncthreads();
    const double tau = taus[k];
    // (tau A v)_i for the rows of the trailing block
    const bool act = own && i >= o;
    double acc = 0.0;
    if (act) {
#pragma unroll
      for (int r = 0; r < 16; ++r) acc += a[r] * vs[q + 8 * r];
    }
    const double wraw = tau * trd_sum8(acc);
    if (own && q == 0) {
      wsa[i] = act ? wraw : 0.0;
      wvs[i] = act ? wraw * vs[i] : 0.0;
    }
    __syncthreads();
    // alpha = -tau/2 v^T w: every 8-lane group sums the rows' products w_i v_i
    // over its rows q + 8 r (together all p) -- the same bits everywhere
    double pv = 0.0;
#pragma unroll
    for (int r = 0; r < 16; ++r) pv += wvs[q + 8 * r];
    const double alpha = -0.5 * tau * trd_sum8(pv);
    if (act) {
      const double vi = vs[i], wi = wraw + alpha * vi;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int c = q + 8 * r;
        a[r] -= vi * (wsa[c] + alpha * vs[c]) + wi * vs[c];
      }
    }
  }
  // the last 2 x 2 block
  if (i == p - 2 || i == p - 1) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int c = q + 8 * r;
      if (c == i) d[i] = a[r];
      if (i == p - 1 && c == p - 2) e[p - 2] = a[r];
    }
  }
  __syncthreads();
  // Q from the back, held as Q^T: rows j >= k+1 of Q^T take
  // -(tau Q^T v)_j v^T (v zero outside columns k+1 ..)
#pragma unroll
  for (int r = 0; r < 16; ++r) a[r] = (own && q + 8 * r == i) ? 1.0 : 0.0;
  for (int k = p - 3; k >= 0; --k) {
    const double* v = Vr + 128 * k;
    const bool act = own && i > k;
    double acc = 0.0;
    if (act) {
#pragma unroll
      for (int r = 0; r < 16; ++r) acc += a[r] * v[q + 8 * r];
    }
    const double y = taus[k] * trd_sum8(acc);
    if (act) {
#pragma unroll
      for (int r = 0; r < 16; ++r) a[r] -= y * v[q + 8 * r];
    }
  }
  // Q column-major: H[c + j p] = Q[c][j] = Q^T[j][c]
  if (own) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int c = q + 8 * r;
      if (c < p) H[c + i * p] = a[r];
    }
  }
}

__global__ __launch_bounds__(kTrdThreads) void k_sytrd_small(double* __restrict__ H, int p,
                                                             double* __restrict__ d,
                                                             double* __restrict__ e) {
  sytrd_body(H, p, d, e);
}

// All eigenpairs of a small symmetric matrix M (n x n, 3 <= n <= 128,
// row-major, overwritten): W ascending, M <- the eigenvector rows (row c for
// W[c]); E (n doubles) is scratch, *info = 1 when a result is not finite.
// Two single-workgroup launches: the Householder reduction and the divide and
// conquer with its back-transform.
bool dense_eig_small(double* M, int n, double* W, double* E, int* info, hipStream_t s) {
  static bool lds_set = hipFuncSetAttribute((const void*)k_sytrd_small,
                                            hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)((size_t)128 * 128 * sizeof(double))) ==
                        hipSuccess;
  if (!lds_set || n < 3 || n > 128) return false;
  hipLaunchKernelGGL(k_sytrd_small, dim3(1), dim3(trd_threads(n)), (size_t)128 * n * sizeof(double),
                     s, M, n, W, E);
  return tridiag_eig_small_back(W, E, n, W, M, info, s);
}

// The same reduction for every problem of a lockstep batch whose block
// eigensolver is still iterating: H (p x p) -> Q^T, diagonal into W, the
// off-diagonal into G (free during the Rayleigh-Ritz step).
__global__ __launch_bounds__(kTrdThreads) void k_group_sytrd(const GroupStep* __restrict__ dsc) {
  const GroupStep& g = dsc[blockIdx.x];
  if (!g.ctl->iter) return;  // uniform
  sytrd_body(g.H, g.p, g.W, g.G);
}

void group_sytrd(const GroupStep* d, int count, int pmax, hipStream_t s) {
  static bool lds_set = hipFuncSetAttribute((const void*)k_group_sytrd,
                                            hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)((size_t)128 * 128 * sizeof(double))) ==
                        hipSuccess;
  (void)lds_set;
  hipLaunchKernelGGL(k_group_sytrd, dim3(count), dim3(trd_threads(pmax)),
                     (size_t)128 * pmax * sizeof(double), s, d);
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
  // about 32 partial products, each K chunk a multiple of 16
  int c = (K + 31) / 32;
  c = (c + 15) / 16 * 16;
  return c < 16 ? 16 : c;
}

// K chunk of the block products V M (p x n times n x n) by 64 x 64 tiles:
// enough partial products for about 1024 workgroups (at least 4, at most
// 16), so that p = 128, n = 4096 takes 8 x 2 x 64 (four workgroups per CU
// hide each other's slab loads: 2% less eigensolver time than 4 x 2 x 64)
// and p = 64, n = 1024 takes 16 x 1 x 16 instead of the 64 workgroups of a
// 4-way split that left most of the chip idle
static inline int vm_chunk(int n, int p) {
  const int tiles = ((p + 63) / 64) * ((n + 63) / 64);
  const int parts = std::min(16, std::max(4, (1024 + tiles - 1) / tiles));
  return ((n + parts - 1) / parts + 15) / 16 * 16;
}

static inline size_t partial_doubles(int n, int p) {
  const size_t pn = (size_t)p * n, pp = (size_t)p * p;
  const size_t gram = (size_t)((n + splitk_chunk(n) - 1) / splitk_chunk(n)) * pp;
  const size_t vm = (size_t)((n + vm_chunk(n, p) - 1) / vm_chunk(n, p)) * pn;
  return gram > vm ? gram : vm;
}

size_t topk_workspace_doubles(int n, int p) {
  const size_t pn = (size_t)p * n, pp = (size_t)p * p;
  return 4 * pn + partial_doubles(n, p) + 4 * pp + 4 * (size_t)p + 16;
}

// Returns true and leaves theta (ascending, p values) in W and the Ritz
// vectors (rows, same order) in Xout (p x n) on convergence.
//
// The sweeps multiply by M - sigma I (the Rayleigh-Ritz products use M
// itself).  M is positive semidefinite and the unwanted eigenvalues lie in
// [0, lambda_{p+1}]; with sigma = lambda_{p+1} / 2 the worst of them shrinks
// by sigma / (lambda_need - sigma) per sweep instead of lambda_{p+1} /
// lambda_need.  *shift holds the sigma to start with (from an earlier solve
// of the same kind; 0 if none) and returns theta_min / 2 of the last
// Rayleigh-Ritz step (theta_min <= lambda_p, so sigma never exceeds half of
// a wanted eigenvalue).
//
// Between Rayleigh-Ritz steps a sweep orthonormalises with one shifted
// Cholesky-QR pass and checks the result with a second Gram matrix (a real
// second pass when it is not the identity to 1e-2).  When no check since the
// last Rayleigh-Ritz step needed that second pass, only the first sweep of
// the next group is checked; *nocheck carries that state to the next solve.
// Every Rayleigh-Ritz step still sees a basis from three passes, and its
// residuals decide convergence.
bool topk_eigs(const double* M, int n, int p, int need, double tol,
               int q_first, double* shift, int* nocheck, double* ws, double* W, double* Xout,
               int* dinfo, int* iters, int* enough, double* resid, hipStream_t s) {
  const size_t pn = (size_t)p * n, pp = (size_t)p * p;
  const int kc = splitk_chunk(n);
  const int kv = vm_chunk(n, p);
  double* V = ws;
  double* Y = V + pn;
  double* T2 = Y + pn;
  double* Yx = T2 + pn;
  double* part = Yx + pn;
  double* G = part + partial_doubles(n, p);
  double* Rt = G + pp;
  double* H = Rt + pp;
  double* E = H + pp;          // off-diagonal of the tridiagonal form (p - 1)
  double* res = E + pp;        // p
  int* fail = (int*)(res + p); // fail flag, then the count of checks that missed
  // a pass's Cholesky factor (p x p) at Rt and its row scaling (p) in the
  // first p entries of H, which only the Rayleigh-Ritz step uses
  double* Rf = Rt;
  const double u = std::ldexp(1.0, -53);
  const double shift_rel = 11.0 * ((double)n * p + (double)p * (p + 1)) * u;

  static bool lds_set = [] {
    return hipFuncSetAttribute((const void*)k_trsm_rows,
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(((size_t)128 * 128 + 128 * 16) * sizeof(double))) ==
               hipSuccess &&
           hipFuncSetAttribute((const void*)k_sytrd_small,
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)((size_t)128 * 128 * sizeof(double))) == hipSuccess;
  }();
  const size_t trsm_lds = ((size_t)p * p + (size_t)p * 16) * sizeof(double);
  if (!lds_set || p > 128 || p % 16 != 0) return false;
  (void)hipMemsetAsync(fail, 0, 2 * sizeof(int), s);
  hipLaunchKernelGGL(k_seed_block, dim3(256), dim3(256), 0, s, V, (long long)pn, 12345ULL);

  // one orthonormalisation of rows of Y into V: shifted Cholesky-QR of the
  // column-scaled Gram matrix twice, then a plain pass -- all three before a
  // Rayleigh-Ritz check (`full`); between checks only the first two, the
  // second skipped on the device (R^-1 = I) when its Gram matrix is the
  // identity to 1e-2.
  auto orth = [&](const double* Yin, double* Vout, bool full, bool check) {
    const double* src = Yin;
    const int last = full ? 2 : (check ? 1 : 0);
    for (int pass = 0; pass <= last; ++pass) {
      gemm_f64_splitk(src, n, src, n, B_KCONTIG, G, p, p, p, n, kc, part, s);
      const double sh = pass < 2 ? shift_rel : 0.0, itol = (pass == 0 || full) ? 0.0 : 1e-2;
      if (p <= 64)
        hipLaunchKernelGGL(k_chol_factor<16>, dim3(1), dim3(256), 0, s, G, p, sh,
                           pass < 2 ? 1 : 0, itol, Rf, fail, fail + 1);
      else
        hipLaunchKernelGGL(k_chol_factor<32>, dim3(1), dim3(1024), 0, s, G, p, sh,
                           pass < 2 ? 1 : 0, itol, Rf, fail, fail + 1);
      double* dst = (pass == last) ? Vout : (src == T2 ? Y : T2);
      if (dst == src) dst = (src == Y) ? T2 : Y;
      hipLaunchKernelGGL(k_trsm_rows, dim3((n + kTrsmCols - 1) / kTrsmCols), dim3(256), trsm_lds,
                         s, (const double*)Rf, p, src, n, dst);
      src = dst;
    }
  };

  // Y = V (M - sigma I)
  double sigma = shift && *shift > 0.0 ? *shift : 0.0;
  auto vm = [&](const double* Vin, double* Yout, double sg) {
    gemm_f64_splitk(Vin, n, M, n, B_NCONTIG, Yout, n, p, n, n, kv, part, s,
                    sg > 0.0 ? Vin : nullptr, sg);
  };

  int it = 0, q = q_first > 0 ? q_first : 3;
  const int max_it = 80;
  double prev = 1e300;
  std::vector<double> th(p), rs(p);
  while (true) {
    const bool skip = nocheck && *nocheck;
    for (int r = 0; r < q; ++r) {
      vm(V, Y, sigma);
      orth(Y, V, r == q - 1, r == 0 || !skip);
      ++it;
    }
    // Rayleigh-Ritz
    vm(V, Y, 0.0);
    gemm_f64_splitk(V, n, Y, n, B_KCONTIG, H, p, p, p, n, kc, part, s);
    hipLaunchKernelGGL(k_symmetrize_small, dim3(16), dim3(256), 0, s, H, p);
    // tridiagonal form and its reduction matrix (H = Q^T, row-major) in one
    // workgroup, then divide and conquer on the tridiagonal in another
    // (Z^T into Rt, eigenvalues over its diagonal in W)
    hipLaunchKernelGGL(k_sytrd_small, dim3(1), dim3(trd_threads(p)),
                       (size_t)128 * p * sizeof(double), s, H, p, W, E);
    if (!tridiag_eig_small(W, E, p, W, Rt, dinfo, s)) return false;
    // Ritz vectors of H as rows: G = Z^T Q^T
    gemm_f64(Rt, p, H, p, B_NCONTIG, G, out_rowmajor(p), p, p, p, nullptr, s);
    gemm_f64(G, p, V, n, B_NCONTIG, Xout, out_rowmajor(n), p, n, p, nullptr, s);
    gemm_f64(G, p, Y, n, B_NCONTIG, Yx, out_rowmajor(n), p, n, p, nullptr, s);
    hipLaunchKernelGGL(k_ritz_residual, dim3(p), dim3(256), 0, s, Yx, Xout, W, n, res);
    int hinfo[3] = {0, 0, 0};
    (void)hipMemcpyAsync(th.data(), W, p * sizeof(double), hipMemcpyDeviceToHost, s);
    (void)hipMemcpyAsync(rs.data(), res, p * sizeof(double), hipMemcpyDeviceToHost, s);
    (void)hipMemcpyAsync(&hinfo[0], dinfo, sizeof(int), hipMemcpyDeviceToHost, s);
    (void)hipMemcpyAsync(&hinfo[1], fail, 2 * sizeof(int), hipMemcpyDeviceToHost, s);
    if (hipStreamSynchronize(s) != hipSuccess) return false;
    if (hinfo[0] != 0 || hinfo[1] != 0) return false;
    if (nocheck) *nocheck = hinfo[2] == 0 ? 1 : 0;
    (void)hipMemsetAsync(fail + 1, 0, sizeof(int), s);
    const double t1 = th[p - 1];
    if (!(t1 > 0.0)) return false;
    double top = 0.0;
    for (int i = 0; i < need; ++i) top = std::fmax(top, rs[p - 1 - i] / t1);
    // the worst unwanted factor per sweep at the shift the sweeps used, and
    // the shift for the next ones
    const double lo = std::fmax(th[0], 0.0);
    double rate = th[p - need] > sigma ? std::fmax(lo - sigma, sigma) / (th[p - need] - sigma)
                                       : 0.5;
    rate = std::fmin(std::fmax(rate, 1e-6), 0.95);
    sigma = 0.5 * lo;
    if (shift) *shift = sigma;
    if (iters) *iters = it;
    if (resid) *resid = top;
    if (top <= tol) {
      // sweeps beyond the first that met tol: top / rate^k <= tol
      int extra = top > 0.0 ? (int)std::floor(std::log(top / tol) / std::log(rate)) : it;
      extra = extra < 0 ? 0 : extra;
      if (enough) *enough = it - extra < 1 ? 1 : it - extra;
      return true;
    }
    if (it >= max_it || !(top < 0.5 * prev)) return false;
    prev = top;
    // the sweeps to come run at the new shift
    rate = th[p - need] > sigma ? std::fmax(lo - sigma, sigma) / (th[p - need] - sigma) : 0.5;
    rate = std::fmin(std::fmax(rate, 1e-6), 0.95);
    q = (int)std::ceil(std::log(tol / top) / std::log(rate));
    q = q < 1 ? 1 : (q > max_it - it ? max_it - it : q);
    // continue from the Ritz vectors
    (void)hipMemcpyAsync(V, Xout, pn * sizeof(double), hipMemcpyDeviceToDevice, s);
  }
}

}  // namespace hotrg
