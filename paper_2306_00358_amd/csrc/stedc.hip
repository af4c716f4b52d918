// Eigenvalues and eigenvectors of a small symmetric tridiagonal matrix (the
// Rayleigh-Ritz matrix of the block eigensolver after Householder reduction,
// n <= 128) by divide and conquer, in one workgroup.
//
// Method (Cuppen's divide and conquer with the deflation and the
// eigenvector formula of Gu and Eisenstat).  Index range [a, b) splits at c
// into [a, c) and [c, b); with beta = e[c-1],
//   T = diag(T1', T2') + |beta| v v^T,  v = e_{c-1} + sign(beta) e_c,
// where T1' and T2' have |beta| taken off their diagonal entries c-1 and c.
// The tree halves every range down to single indices, so every diagonal entry
// loses the moduli of both neighbouring off-diagonal entries up front and the
// leaves are 1 x 1.  A merge, given the children's eigenpairs (Z1, L1), (Z2,
// L2), solves diag(L1, L2) + rho z z^T with z = (last row of Z1,
// sign(beta) first row of Z2) / |.|, rho = |beta| |z|^2:
//   * deflation, scanning the poles in ascending order: a component with
//     rho |z_i| <= tol leaves (d_i, its column) unchanged; two poles closer
//     than tol after the rotation that zeroes one z component are rotated
//     (columns of Z too) and the zeroed one leaves;
//     tol = 8 u max(max |d|, rho);
//   * each remaining root lam_j of 1/rho + sum_i z_i^2 / (d_i - lam) = 0 lies
//     in (d_j, d_{j+1}) (the last in (d_K, d_K + rho |z|^2]) and is stored as
//     lam_j = d_o + tau_j with the nearer pole o as origin, so that every
//     d_i - lam_j = (d_i - d_o) - tau_j is accurate; tau comes from a
//     safeguarded iteration on a two-pole rational model of the secular
//     function (value and slope of the parts left and right of the root);
//   * z is recomputed from the roots (Gu-Eisenstat),
//     z_i^2 = (lam_i - d_i) / rho * prod_{j != i} (d_i - lam_j) / (d_i - d_j),
//     with the sign of the original z_i, so that the vectors
//     u_j = (z_i / (d_i - lam_j))_i / |.| are orthogonal to working accuracy;
//   * the merged block of Z becomes Z [u_1 .. u_K] in the columns of the
//     remaining poles (MFMA, v_mfma_f64_16x16x4f64, the u entries formed as
//     B operands), deflated columns staying where they are.
// All merges of one tree level run together; the scans are sequential per
// merge, the roots, z and norms take 8 lanes per index, the products 16 x 16
// tiles per wave.  Eigenvalues leave ascending (ties by index) in W and the
// eigenvectors as rows of Zt (row c = eigenvector of W[c]); info = 1 when a
// result is not finite.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"

namespace hotrg {

constexpr int kDcThreads = 1024;
constexpr int kDcMax = 128;
constexpr int kDcLd = kDcMax + 1;  // row stride of Z in LDS (padded against bank conflicts)

typedef double dc4 __attribute__((ext_vector_type(4)));

// value of another lane of the same 8-lane group (DPP: quad_perm [1,0,3,2],
// quad_perm [2,3,0,1], row_half_mirror); every lane of the group is active
template <int kCtrl>
__device__ __forceinline__ double dc_dpp(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, kCtrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), kCtrl, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// sum / product over an 8-lane group, the same bits in every lane
__device__ __forceinline__ double dc_sum8(double v) {
  v += dc_dpp<0xB1>(v);
  v += dc_dpp<0x4E>(v);
  return v + dc_dpp<0x141>(v);
}

__device__ __forceinline__ double dc_prod8(double v) {
  v *= dc_dpp<0xB1>(v);
  v *= dc_dpp<0x4E>(v);
  return v * dc_dpp<0x141>(v);
}

// 1 / x: v_rcp_f64 refined by two Newton steps
__device__ __forceinline__ double dc_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

__device__ __forceinline__ double dc_max8(double v) {
  v = fmax(v, dc_dpp<0xB1>(v));
  v = fmax(v, dc_dpp<0x4E>(v));
  return fmax(v, dc_dpp<0x141>(v));
}

// node k of tree level D over n indices: [(k n) >> D, ((k + 1) n) >> D)
struct DcMerge {
  int a, b, c;
  bool real;  // both children non-empty
};

__device__ __forceinline__ DcMerge dc_merge_of(int s, int D, int n) {
  const int k = (((s + 1) << D) + n - 1) / n - 1;
  DcMerge m;
  m.a = (k * n) >> D;
  m.b = ((k + 1) * n) >> D;
  m.c = ((2 * k + 1) * n) >> (D + 1);
  m.real = m.c > m.a && m.c < m.b;
  return m;
}

// din may be W: it is read before the first barrier and W written after the
// last.  With Hb (n x n, row-major, holding Q^T of a Householder reduction
// Q^T A Q = T) the eigenvectors leave as the rows of Z^T Q^T over Hb instead
// of Z^T into Zt: row c of Hb becomes A's eigenvector for W[c].
__device__ __forceinline__ void stedc_body(const double* din, const double* ein, int n, double* W,
                                           double* __restrict__ Zt, double* __restrict__ Hb,
                                           int* __restrict__ info) {
  extern __shared__ double Z[];  // n rows of kDcLd: Z[r * kDcLd + c]
  __shared__ double lam[kDcMax], e[kDcMax], zv[kDcMax];
  __shared__ double sd[kDcMax], sz[kDcMax];
  __shared__ double dh[kDcMax], zh[kDcMax], zt[kDcMax], tau[kDcMax], inrm[kDcMax];
  __shared__ double rc[kDcMax], rs[kDcMax];
  __shared__ double mrho[kDcMax], mtol[kDcMax], msc[kDcMax];
  __shared__ int scol[kDcMax], ndc[kDcMax], og[kDcMax], rp[kDcMax], rq[kDcMax];
  __shared__ int kcnt[kDcMax], rcnt[kDcMax], ord[kDcMax];
  __shared__ int tiles[64];
  __shared__ int ntiles, bad;
  const int t = threadIdx.x;
  const double eps = 1.1102230246251565e-16;  // 2^-53

  for (int x = t; x < n * kDcLd; x += kDcThreads) Z[x] = (x / kDcLd == x % kDcLd) ? 1.0 : 0.0;
  if (t < n) {
    e[t] = t < n - 1 ? ein[t] : 0.0;
    double dv = din[t];
    if (t >= 1) dv -= fabs(ein[t - 1]);
    if (t < n - 1) dv -= fabs(ein[t]);
    lam[t] = dv;
  }
  if (t == 0) bad = 0;
  int L = 0;
  while ((1 << L) < n) ++L;
  __syncthreads();

  for (int D = L - 1; D >= 0; --D) {
    // (A) the coupling vector z of each merge, by column
    if (t < n) {
      const DcMerge g = dc_merge_of(t, D, n);
      if (g.real) {
        const double sg = e[g.c - 1] < 0.0 ? -1.0 : 1.0;
        zv[t] = t < g.c ? Z[(g.c - 1) * kDcLd + t] : sg * Z[g.c * kDcLd + t];
      }
    }
    __syncthreads();
    // poles of each merge in ascending order (ties by column), 8 lanes per
    // index; the first index of a merge also forms |z|, rho and tol
    {
      const int e8 = t >> 3, u = t & 7;
      const DcMerge g = dc_merge_of(e8 < n ? e8 : 0, D, n);
      if (e8 < n && g.real) {
        const double lv = lam[e8];
        double r = 0.0;
        for (int i = g.a + u; i < g.b; i += 8) {
          const double li = lam[i];
          r += (li < lv || (li == lv && i < e8)) ? 1.0 : 0.0;
        }
        const int rk = (int)dc_sum8(r);
        if (u == 0) {
          sd[g.a + rk] = lv;
          sz[g.a + rk] = zv[e8];
          scol[g.a + rk] = e8 - g.a;
        }
        if (e8 == g.a) {
          double s2 = 0.0, dmax = 0.0;
          for (int i = g.a + u; i < g.b; i += 8) {
            s2 += zv[i] * zv[i];
            dmax = fmax(dmax, fabs(lam[i]));
          }
          s2 = dc_sum8(s2);
          dmax = dc_max8(dmax);
          if (u == 0) {
            const double rho = fabs(e[g.c - 1]) * s2;
            mrho[g.a] = rho;
            msc[g.a] = s2 > 0.0 ? 1.0 / sqrt(s2) : 0.0;
            mtol[g.a] = 8.0 * eps * fmax(dmax, rho);
          }
        }
      }
    }
    __syncthreads();
    // (B) deflation scan, one thread per merge
    if (t < n) {
      const DcMerge g = dc_merge_of(t, D, n);
      if (g.real && t == g.a) {
        const int a = g.a, m = g.b - g.a;
        const double rho = mrho[a], tol = mtol[a], sc = msc[a];
        int K = 0, R = 0, pj = -1;
        double pd = 0.0, pz = 0.0;
        for (int s0 = 0; s0 < m; s0 += 8) {
          int cb[8];
          double db[8], zb[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const int sq = a + min(s0 + q, m - 1);
            cb[q] = scol[sq];
            db[q] = sd[sq];
            zb[q] = sz[sq];
          }
#pragma unroll
          for (int q = 0; q < 8; ++q) {
          if (s0 + q >= m) break;
          const int col = cb[q];
          double dv = db[q];
          const double zs = zb[q] * sc;
          if (rho * fabs(zs) <= tol) {
            lam[a + col] = dv;
            continue;
          }
          if (pj < 0) {
            pj = col;
            pd = dv;
            pz = zs;
            continue;
          }
          if (fabs(dv - pd) * fabs(pz * zs) <= tol * (pz * pz + zs * zs)) {
            const double r = sqrt(pz * pz + zs * zs);
            const double cth = zs / r, sth = -pz / r;
            rp[a + R] = pj;
            rq[a + R] = col;
            rc[a + R] = cth;
            rs[a + R] = sth;
            ++R;
            lam[a + pj] = pd * cth * cth + dv * sth * sth;
            dv = pd * sth * sth + dv * cth * cth;
            pj = col;
            pd = dv;
            pz = r;
          } else {
            ndc[a + K] = pj;
            dh[a + K] = pd;
            zh[a + K] = pz;
            ++K;
            pj = col;
            pd = dv;
            pz = zs;
          }
          }
        }
        if (pj >= 0) {
          ndc[a + K] = pj;
          dh[a + K] = pd;
          zh[a + K] = pz;
          ++K;
        }
        kcnt[a] = K;
        rcnt[a] = R;
      }
    }
    __syncthreads();
    // (C) the deflating rotations on the rows of each merged block; one
    // thread lists the product tiles of the level
    if (t < n) {
      const DcMerge g = dc_merge_of(t, D, n);
      if (g.real) {
        const int R = rcnt[g.a];
        double* zr = Z + t * kDcLd + g.a;
        for (int q = 0; q < R; ++q) {
          const int x = rp[g.a + q], y = rq[g.a + q];
          const double cq = rc[g.a + q], sq = rs[g.a + q];
          const double zx = zr[x], zy = zr[y];
          zr[x] = cq * zx + sq * zy;
          zr[y] = -sq * zx + cq * zy;
        }
      }
    } else if (t >= kDcThreads - 64) {
      // lane k lists merge k's tiles (at most 64 merges, 64 tiles a level)
      const int k = t - (kDcThreads - 64);
      int cnt = 0, a = 0, cts = 1;
      if (k < (1 << D)) {
        a = (k * n) >> D;
        const int b = ((k + 1) * n) >> D, c = ((2 * k + 1) * n) >> (D + 1);
        if (c > a && c < b) {
          cts = (kcnt[a] + 15) / 16;
          cnt = ((b - a + 15) / 16) * cts;
        }
      }
      int x = cnt;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (k >= o) x += y;
      }
      for (int q = 0; q < cnt; ++q) tiles[x - cnt + q] = a | ((q / cts) << 8) | ((q % cts) << 12);
      if (k == 63) ntiles = x;
    }
    __syncthreads();
    // (D) secular roots, 8 lanes per root
    const int gs = t >> 3, u = t & 7;
    {
      const DcMerge g = dc_merge_of(gs < n ? gs : 0, D, n);
      const int a = g.a;
      const int K = (gs < n && g.real) ? kcnt[a] : 0;
      const int j = gs - a;
      if (gs < n && g.real && j < K) {
        const double rho = mrho[a], rinv = 1.0 / rho;
        // sums of the secular function and of its slope over the poles left
        // (i <= j) and right of the root at tv, in the frame of origin pole org
        double psi = 0.0, dpsi = 0.0, phi = 0.0, dphi = 0.0;
        auto sums = [&](double org, double tv) {
          psi = dpsi = phi = dphi = 0.0;
          for (int i = u; i < K; i += 8) {
            const double zq = zh[a + i];
            const double r = zq * dc_rcp((dh[a + i] - org) - tv);
            if (i <= j) {
              psi += zq * r;
              dpsi += r * r;
            } else {
              phi += zq * r;
              dphi += r * r;
            }
          }
          psi = dc_sum8(psi);
          dpsi = dc_sum8(dpsi);
          phi = dc_sum8(phi);
          dphi = dc_sum8(dphi);
        };
        int o;
        double lo, hi, tv;
        bool have = false;
        if (j < K - 1) {
          // the sign at the midpoint of (d_j, d_j+1) picks the nearer pole as
          // origin; the sums there start the iteration
          const double gap = dh[a + j + 1] - dh[a + j];
          const double mid = 0.5 * gap;
          sums(dh[a + j], mid);
          have = true;
          if (rinv + psi + phi >= 0.0) {
            o = j;
            lo = 0.0;
            hi = mid;
            tv = mid;
          } else {
            o = j + 1;
            lo = -(gap - mid);
            hi = 0.0;
            tv = lo;
          }
        } else {
          double s2 = 0.0;
          for (int i = u; i < K; i += 8) s2 += zh[a + i] * zh[a + i];
          o = K - 1;
          lo = 0.0;
          hi = rho * dc_sum8(s2);
          tv = 0.5 * hi;
        }
        const double org = dh[a + o];
        for (int it = 0; it < 80; ++it) {
          if (!have) sums(org, tv);
          have = false;
          const double f = rinv + psi + phi;
          if (!(fabs(f) < INFINITY)) {
            if (u == 0) bad = 1;
            break;
          }
          const double err = 8.0 * (fabs(psi) + fabs(phi) + rinv) + fabs(tv) * (dpsi + dphi);
          if (fabs(f) <= 4.0 * eps * err) break;
          if (f > 0.0)
            hi = fmin(hi, tv);
          else
            lo = fmax(lo, tv);
          // two-pole model f(tv + eta) ~ cf + s / (Dj - eta) + S / (Dj1 - eta)
          double eta;
          if (j < K - 1) {
            const double Dj = (dh[a + j] - org) - tv, Dj1 = (dh[a + j + 1] - org) - tv;
            const double s = dpsi * Dj * Dj, S = dphi * Dj1 * Dj1;
            const double cf = f - dpsi * Dj - dphi * Dj1;
            const double qb = -(cf * (Dj + Dj1) + s + S);
            const double qc = cf * Dj * Dj1 + s * Dj1 + S * Dj;
            eta = NAN;
            if (cf == 0.0) {
              eta = -qc / qb;
            } else {
              const double sq = sqrt(fmax(qb * qb - 4.0 * cf * qc, 0.0));
              const double qq = -0.5 * (qb + copysign(sq, qb));
              const double r1 = qq / cf, r2 = qq != 0.0 ? qc / qq : NAN;
              const bool in1 = tv + r1 > lo && tv + r1 < hi;
              const bool in2 = tv + r2 > lo && tv + r2 < hi;
              if (in1 && in2)
                eta = fabs(r1) < fabs(r2) ? r1 : r2;
              else if (in1)
                eta = r1;
              else if (in2)
                eta = r2;
            }
          } else {
            const double Dj = (dh[a + j] - org) - tv;
            const double s = dpsi * Dj * Dj, cf = f - dpsi * Dj;
            eta = cf != 0.0 ? Dj + s / cf : NAN;
          }
          double nt = tv + eta;
          if (!(nt > lo && nt < hi)) nt = 0.5 * (lo + hi);
          if (nt == tv) break;
          tv = nt;
        }
        if (u == 0) {
          og[gs] = a + o;
          tau[gs] = tv;
        }
      }
    }
    __syncthreads();
    // (E) z recomputed from the roots
    {
      const DcMerge g = dc_merge_of(gs < n ? gs : 0, D, n);
      const int a = g.a;
      const int K = (gs < n && g.real) ? kcnt[a] : 0;
      const int i = gs - a;
      if (gs < n && g.real && i < K) {
        const double di = dh[a + i], rho = mrho[a];
        double pr = 1.0;
        for (int j = u; j < K; j += 8) {
          const double dl = (di - dh[og[a + j]]) - tau[a + j];
          pr *= (j == i) ? -dl / rho : dl / (di - dh[a + j]);
        }
        pr = dc_prod8(pr);
        if (u == 0) zt[gs] = copysign(sqrt(fmax(pr, 0.0)), zh[gs]);
      }
    }
    __syncthreads();
    // (F) norms of the vectors (z_i / (d_i - lam_j))_i
    {
      const DcMerge g = dc_merge_of(gs < n ? gs : 0, D, n);
      const int a = g.a;
      const int K = (gs < n && g.real) ? kcnt[a] : 0;
      const int j = gs - a;
      if (gs < n && g.real && j < K) {
        const double dj = dh[og[gs]], tj = tau[gs];
        double s2 = 0.0;
        for (int i = u; i < K; i += 8) {
          const double q = zt[a + i] / ((dh[a + i] - dj) - tj);
          s2 += q * q;
        }
        s2 = dc_sum8(s2);
        if (u == 0) inrm[gs] = 1.0 / sqrt(s2);
      }
    }
    __syncthreads();
    // (G) Z block <- Z block [u_1 .. u_K] in the remaining poles' columns
    {
      const int w = t >> 6, ln = t & 63, li = ln & 15, lk = ln >> 4;
      const int nt = ntiles;
      dc4 acc[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        acc[q] = dc4{0.0, 0.0, 0.0, 0.0};
        const int ti = w + 16 * q;
        if (ti >= nt) continue;
        const int tl = tiles[ti];
        const int a = tl & 255, rt = (tl >> 8) & 15, ct = (tl >> 12) & 15;
        const DcMerge g = dc_merge_of(a, D, n);
        const int K = kcnt[a];
        const int r = a + 16 * rt + li;
        const int j = 16 * ct + li;
        double dj = 0.0, tj = 0.0, nj = 0.0;
        if (j < K) {
          dj = dh[og[a + j]];
          tj = tau[a + j];
          nj = inrm[a + j];
        }
        for (int kk = 0; kk < (K + 3) / 4; ++kk) {
          const int i = 4 * kk + lk;
          const double av = (r < g.b && i < K) ? Z[r * kDcLd + a + ndc[a + i]] : 0.0;
          const double bv = (j < K && i < K) ? zt[a + i] / ((dh[a + i] - dj) - tj) * nj : 0.0;
          acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[q], 0, 0, 0);
        }
      }
      __syncthreads();  // every read of the old block is done
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ti = w + 16 * q;
        if (ti >= nt) continue;
        const int tl = tiles[ti];
        const int a = tl & 255, rt = (tl >> 8) & 15, ct = (tl >> 12) & 15;
        const DcMerge g = dc_merge_of(a, D, n);
        const int K = kcnt[a];
        const int j = 16 * ct + li;
        if (j >= K) continue;
        const int col = a + ndc[a + j];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = a + 16 * rt + lk + 4 * v;
          if (r < g.b) Z[r * kDcLd + col] = acc[q][v];
        }
      }
      if (t < n) {
        const DcMerge g = dc_merge_of(t, D, n);
        if (g.real && t - g.a < kcnt[g.a]) lam[g.a + ndc[t]] = dh[og[t]] + tau[t];
      }
    }
    __syncthreads();
  }

  // ascending order (ties by index)
  if (t < n) {
    const double lv = lam[t];
    int r = 0;
    for (int i = 0; i < n; ++i) {
      const double li = lam[i];
      r += (li < lv || (li == lv && i < t)) ? 1 : 0;
    }
    ord[r] = t;
    W[r] = lv;
    if (!(fabs(lv) < INFINITY)) bad = 1;
  }
  __syncthreads();
  if (Hb) {
    // (Q z_c)_i = sum_k Hb[k][i] Z[k][ord[c]]: thread (i, group cg) forms
    // columns i of rows c = cg, cg + 8, ..; every read of Hb precedes the
    // barrier, every write follows it
    const int i = t & 127, cg = t >> 7;
    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;
    if (i < n) {
#pragma unroll
      for (int half = 0; half < 16; half += 8) {  // eight rows at a time: fewer live indices
        int col[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int c = cg + 8 * (half + q);
          col[q] = ord[c < n ? c : 0];
        }
        for (int k = 0; k < n; ++k) {
          const double h = Hb[(long long)k * n + i];
          const double* zr = Z + k * kDcLd;
#pragma unroll
          for (int q = 0; q < 8; ++q) acc[half + q] += h * zr[col[q]];
        }
      }
    }
    __syncthreads();
    if (i < n) {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int c = cg + 8 * q;
        if (c < n) Hb[(long long)c * n + i] = acc[q];
      }
    }
  } else {
    for (int x = t; x < n * n; x += kDcThreads) {
      const int c = x / n, r = x % n;
      Zt[x] = Z[r * kDcLd + ord[c]];
    }
  }
  if (t == 0) *info = bad;
}

__global__ __launch_bounds__(kDcThreads) void k_stedc_small(const double* din, const double* ein,
                                                            int n, double* W,
                                                            double* __restrict__ Zt,
                                                            int* __restrict__ info) {
  stedc_body(din, ein, n, W, Zt, nullptr, info);
}

// Every problem of a lockstep batch whose block eigensolver is still
// iterating: the tridiagonal (diagonal in W, off-diagonal in G) of its
// Rayleigh-Ritz matrix, whose reduction matrix Q^T is in H, becomes W
// ascending and H = the Ritz coefficient rows; a non-finite result marks
// the problem failed (it is then run again alone).
__global__ __launch_bounds__(kDcThreads) void k_group_stedc(const GroupStep* __restrict__ dsc) {
  const GroupStep& g = dsc[blockIdx.x];
  if (!g.ctl->iter) return;  // uniform
  __shared__ int bad_out;
  stedc_body(g.W, g.G, g.p, g.W, nullptr, g.H, &bad_out);
  if (threadIdx.x == 0 && bad_out) g.ctl->fail = 1;  // thread 0 wrote bad_out itself
}

void group_stedc(const GroupStep* d, int count, int pmax, hipStream_t s) {
  static bool lds_set = hipFuncSetAttribute((const void*)k_group_stedc,
                                            hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)((size_t)kDcMax * kDcLd * sizeof(double))) ==
                        hipSuccess;
  (void)lds_set;
  hipLaunchKernelGGL(k_group_stedc, dim3(count), dim3(kDcThreads),
                     (size_t)pmax * kDcLd * sizeof(double), s, d);
}

// The same with the back-transform: Hb (n x n) holds Q^T on entry and the
// eigenvector rows on exit.
__global__ __launch_bounds__(kDcThreads) void k_stedc_small_back(const double* din,
                                                                 const double* ein, int n,
                                                                 double* W,
                                                                 double* __restrict__ Hb,
                                                                 int* __restrict__ info) {
  stedc_body(din, ein, n, W, nullptr, Hb, info);
}

bool tridiag_eig_small_back(const double* d, const double* e, int n, double* W, double* Hb,
                            int* info, hipStream_t s) {
  static bool lds_set = hipFuncSetAttribute((const void*)k_stedc_small_back,
                                            hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)((size_t)kDcMax * kDcLd * sizeof(double))) ==
                        hipSuccess;
  if (!lds_set || n < 1 || n > kDcMax) return false;
  hipLaunchKernelGGL(k_stedc_small_back, dim3(1), dim3(kDcThreads),
                     (size_t)n * kDcLd * sizeof(double), s, d, e, n, W, Hb, info);
  return hipGetLastError() == hipSuccess;
}

bool tridiag_eig_small(const double* d, const double* e, int n, double* W, double* Zt, int* info,
                       hipStream_t s) {
  static bool lds_set = hipFuncSetAttribute((const void*)k_stedc_small,
                                            hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)((size_t)kDcMax * kDcLd * sizeof(double))) ==
                        hipSuccess;
  if (!lds_set || n < 1 || n > kDcMax) return false;
  hipLaunchKernelGGL(k_stedc_small, dim3(1), dim3(kDcThreads),
                     (size_t)n * kDcLd * sizeof(double), s, d, e, n, W, Zt, info);
  return hipGetLastError() == hipSuccess;
}

}  // namespace hotrg
