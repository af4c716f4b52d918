// Bandwidth-bound and single-block kernels of one HOTRG step:
// operand preparation (leg transposition, normalisation, layouts), the
// environment symmetrisation, spectrum bookkeeping, projector extraction,
// and the FP64 log-norm accumulation (arXiv 2306.00358, Sec. 2).
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.h"

namespace hotrg {

static inline int nblocks(long long n, int t) {
  long long b = (n + t - 1) / t;
  return (int)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

__device__ __forceinline__ double ld_any(const void* p, long long i, bool f32) {
  return f32 ? (double)((const float*)p)[i] : ((const double*)p)[i];
}
__device__ __forceinline__ void st_any(void* p, long long i, double v, bool f32) {
  if (f32)
    ((float*)p)[i] = (float)v;
  else
    ((double*)p)[i] = v;
}

// ---------------------------------------------------------------- max|x| --
__global__ void k_maxabs(const void* x, long long n, bool f32, unsigned long long* maxbits) {
  double m = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    m = fmax(m, fabs(ld_any(x, i, f32)));
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(maxbits, (unsigned long long)__double_as_longlong(m));
}

void launch_maxabs(const void* x, long long n, bool is_f32, unsigned long long* maxbits,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_maxabs, dim3(nblocks(n, 256) < 1024 ? nblocks(n, 256) : 1024), dim3(256),
                     0, s, x, n, is_f32, maxbits);
}

// acc[0] = ln n_0; the state's sticky failure flag (an int in acc[1]) is cleared
__global__ void k_init_acc(const unsigned long long* maxbits, double* acc) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    acc[0] = log(__longlong_as_double((long long)*maxbits));
    *(int*)(acc + 1) = 0;
  }
}

// *flag = 1 when *info != 0 (or `force`): a failed eigensolve of any step stays
// visible until the state is finished
__global__ void k_fold_info(const int* info, int* flag, int force) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && (force || *info != 0)) *flag = 1;
}

void launch_fold_info(const int* info, int* flag, int force, hipStream_t s) {
  hipLaunchKernelGGL(k_fold_info, dim3(1), dim3(64), 0, s, info, flag, force);
}

void launch_init_acc(const unsigned long long* maxbits, double* acc, hipStream_t s) {
  hipLaunchKernelGGL(k_init_acc, dim3(1), dim3(64), 0, s, maxbits, acc);
}

// ------------------------------------------------------------- operands --
// Destination tensor T[l,u,r,d] of dims (dx,dy,dx,dy).  With `rotate`, the
// source has dims (dy,dx,dy,dx) and T[l,u,r,d] = src[u,l,d,r].
// One pass of an operand preparation: element (l, u, r, d) of the tensor
// (dims n = (dx, dy, dx, dy)) is read at sum idx * sst, scaled by 1 / max|T~|
// and written at sum idx * dst (and at sum idx * tst into an FP32 copy when
// one is given).  The dims ta (unit source stride) and tb (unit destination
// stride, or another one when that is ta) are tiled 32 x 32; blockIdx.y / z
// run over the other two.  With different unit-stride dims the tile passes
// through LDS, so reads run along ta and writes along tb, both coalesced;
// otherwise both run along ta directly.
struct PrepPass {
  long long sst[4], dst[4], tst[4];
  int n[4];
  int ta, tb, o0, o1;
};

// the pass geometry: source strides sst, destination strides dst (index
// order l, u, r, d), dims (dx, dy, dx, dy); returns the grid
static dim3 prep_pass(PrepPass& P, const long long* sst, const long long* dst, int dx, int dy) {
  const long long nat[4] = {(long long)dy * dx * dy, (long long)dx * dy, dy, 1};
  for (int i = 0; i < 4; ++i) {
    P.sst[i] = sst[i];
    P.dst[i] = dst[i];
    P.tst[i] = nat[i];
  }
  P.n[0] = dx;
  P.n[1] = dy;
  P.n[2] = dx;
  P.n[3] = dy;
  int ta = 0, tb = -1;
  for (int i = 0; i < 4; ++i)
    if (sst[i] == 1) ta = i;
  for (int i = 0; i < 4; ++i)
    if (dst[i] == 1 && i != ta) tb = i;
  if (tb < 0) tb = ta == 3 ? 2 : 3;  // the same unit-stride dim: any other one
  int rest[2], nr = 0;
  for (int i = 0; i < 4; ++i)
    if (i != ta && i != tb) rest[nr++] = i;
  P.ta = ta;
  P.tb = tb;
  P.o0 = rest[0];
  P.o1 = rest[1];
  return dim3((unsigned)(((P.n[ta] + 31) / 32) * ((P.n[tb] + 31) / 32)), (unsigned)P.n[rest[0]],
              (unsigned)P.n[rest[1]]);
}

// FP64 (or FP32, out_f32) operands of the FP64 path
__global__ __launch_bounds__(256) void k_prep_pass(const void* src, bool src_f32, PrepPass P,
                                                   const unsigned long long* maxbits, void* out,
                                                   bool out_f32) {
  __shared__ double tile[32][33];
  const double inv = 1.0 / __longlong_as_double((long long)*maxbits);
  const int na = P.n[P.ta], nb = P.n[P.tb];
  const int tiles_a = (na + 31) / 32;
  const int a0 = (blockIdx.x % tiles_a) * 32, b0 = (blockIdx.x / tiles_a) * 32;
  const long long sb = blockIdx.y * P.sst[P.o0] + blockIdx.z * P.sst[P.o1];
  const long long db = blockIdx.y * P.dst[P.o0] + blockIdx.z * P.dst[P.o1];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const bool direct = P.dst[P.ta] == 1;
  for (int k = ty; k < 32; k += 8) {
    const int a = a0 + tx, b = b0 + k;
    double v = 0.0;
    if (a < na && b < nb) {
      v = ld_any(src, sb + a * P.sst[P.ta] + b * P.sst[P.tb], src_f32) * inv;
      if (direct) st_any(out, db + a * P.dst[P.ta] + b * P.dst[P.tb], v, out_f32);
    }
    tile[k][tx] = v;
  }
  if (direct) return;  // uniform
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int b = b0 + tx, a = a0 + k;
    if (a < na && b < nb) st_any(out, db + a * P.dst[P.ta] + b * P.dst[P.tb], tile[tx][k], out_f32);
  }
}

void launch_prep(const void* src, bool src_f32, bool rotate, int dx, int dy,
                 const unsigned long long* maxbits, void* Tn, void* Xt, void* Tp, bool out_f32,
                 hipStream_t s) {
  // index order (l, u, r, d); the source is T~ itself or, rotated, T~[u, l, d, r]
  const long long X = dx, Y = dy;
  const long long src_rot[4] = {Y * X, X * Y * X, 1, X};
  const long long src_nat[4] = {Y * X * Y, X * Y, Y, 1};
  // Tn natural; Xt[(l,d),(u,r)]; Tp[(l,u),(d,r)]: T[a,c,e,l] read as rows (a,c), columns (l,e)
  const long long dsts[3][4] = {{Y * X * Y, X * Y, Y, 1},
                                {Y * Y * X, X, 1, Y * X},
                                {Y * Y * X, Y * X, 1, X}};
  void* outs[3] = {Tn, Xt, Tp};
  for (int o = 0; o < 3; ++o) {
    PrepPass P{};
    const dim3 grid = prep_pass(P, rotate ? src_rot : src_nat, dsts[o], dx, dy);
    hipLaunchKernelGGL(k_prep_pass, grid, dim3(256), 0, s, src, src_f32, P, maxbits, outs[o],
                       out_f32);
  }
}

// The reflected tensor T'[l,u,r,d] = T[r,u,l,d] (FP64, dims (dx,dy,dx,dy)) in
// the natural layout and in the Xt layout [(l,d),(u,r)]: the operands whose
// environment is that of the right pair of legs of T.
__global__ void k_prep_mirror(const double* __restrict__ T, int dx, int dy, double* Tn,
                              double* Xt) {
  const long long total = (long long)dx * dy * dx * dy;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    long long q = e;
    int d = (int)(q % dy); q /= dy;
    int r = (int)(q % dx); q /= dx;
    int u = (int)(q % dy); q /= dy;
    int l = (int)q;
    const double v = T[(((long long)r * dy + u) * dx + l) * dy + d];
    Tn[e] = v;
    Xt[(((long long)l * dy + d) * dy + u) * dx + r] = v;
  }
}

void launch_prep_mirror(const double* T, int dx, int dy, double* Tn, double* Xt, hipStream_t s) {
  long long total = (long long)dx * dy * dx * dy;
  hipLaunchKernelGGL(k_prep_mirror, dim3(nblocks(total, 256)), dim3(256), 0, s, T, dx, dy, Tn, Xt);
}

__global__ void k_store(double* p, double v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

void launch_store(double* p, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_store, dim3(1), dim3(64), 0, s, p, v);
}

// ------------------------------------------------------------ environment --
// M <- (M + M^T) / 2 by 32 x 32 tile pairs (I, J), I <= J: both tiles are
// read coalesced into LDS and written back, each entry 0.5 (M_rc + M_cr)
// with r < c the upper one; a diagonal tile is its own partner.
__global__ __launch_bounds__(256) void k_symmetrize(double* M, int n) {
  const int I = blockIdx.y, J = blockIdx.x;
  if (I > J) return;  // uniform
  __shared__ double A[32][33], B[32][33];  // tiles (I, J) and (J, I)
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int r0 = I * 32, c0 = J * 32;
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + k, c = c0 + tx;
    A[k][tx] = (r < n && c < n) ? M[(long long)r * n + c] : 0.0;
    const int r2 = c0 + k, c2 = r0 + tx;
    B[k][tx] = (r2 < n && c2 < n) ? M[(long long)r2 * n + c2] : 0.0;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + k, c = c0 + tx;  // in tile (I, J): M_rc = A[k][tx], M_cr = B[tx][k]
    if (r < n && c < n && r < c) M[(long long)r * n + c] = 0.5 * (A[k][tx] + B[tx][k]);
    const int r2 = c0 + k, c2 = r0 + tx;  // in tile (J, I), lower: upper partner (c2, r2)
    if (r2 < n && c2 < n && c2 < r2) M[(long long)r2 * n + c2] = 0.5 * (A[tx][k] + B[k][tx]);
  }
}

void launch_symmetrize(double* M, int n, hipStream_t s) {
  const int T = (n + 31) / 32;
  hipLaunchKernelGGL(k_symmetrize, dim3(T, T), dim3(256), 0, s, M, n);
}

// --------------------------------------------------------------- spectrum --
// W: the cnt leading eigenvalues of M, ascending; lambda_m = W[cnt-1-m]
// (descending).  total = trace(M).  rec[1] = truncation error, rec[2] = cut
// gap, rec[4] = kept (as double).  Sums use a fixed-order tree.
__global__ void k_spectrum(const double* W, int cnt, int n, int dn, int trunc, double tau,
                           int spec_len, const double* total, double* spec_out, double* rec,
                           int* kept_out) {
  __shared__ double red[256];
  __shared__ int kept_s;
  const int t = threadIdx.x;
  const double l1 = W[cnt - 1];
  if (t == 0) {
    int kept = dn;
    if (trunc == 1 && dn < n)
      while (kept > 0 && (W[cnt - kept] - W[cnt - 1 - kept]) <= tau * l1) --kept;
    kept_s = kept;
    *kept_out = kept;
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
    rec[1] = 1.0 - red[0] / total[0];
    rec[2] = dn < n ? (W[cnt - dn] - W[cnt - 1 - dn]) / l1 : -1.0;
    rec[4] = (double)kept;
  }
  if (spec_out)
    for (int m = t; m < spec_len; m += 256) spec_out[m] = m < cnt ? W[cnt - 1 - m] / l1 : 0.0;
}

void launch_spectrum(const double* W, int cnt, int n, int dn, int trunc, double tau, int spec_len,
                     const double* total, double* spec_out, double* rec, int* kept,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_spectrum, dim3(1), dim3(256), 0, s, W, cnt, n, dn, trunc, tau, spec_len,
                     total, spec_out, rec, kept);
}

// ------------------------------------------------------------- projector --
// V: `cols` eigenvectors of M of length n, vector c at V[c*n .. c*n + n),
// ascending eigenvalue order.
// Ucan[(a*dx + b)*dn + i] = U[a,b,i] = vector cols-1-i (zero for i >= kept).
__global__ void k_isometry(const double* V, int cols, int n, int dn, const int* kept,
                           double* Ucan) {
  const int kp = *kept;
  long long total = (long long)n * dn;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    int i = (int)(e % dn);
    int row = (int)(e / dn);
    Ucan[e] = i < kp ? V[(long long)(cols - 1 - i) * n + row] : 0.0;
  }
}

void launch_isometry(const double* V, int cols, int n, int dn, const int* kept, double* Ucan,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_isometry, dim3(nblocks((long long)n * dn, 256)), dim3(256), 0, s, V, cols,
                     n, dn, kept, Ucan);
}

// U1[(i*dx + a)*dx + b] = U[a,b,i]     (A operand of the first contraction)
// U3[(d*dx + e)*dn + k] = U[e,d,k]     (B operand of the last contraction)
__global__ void k_layout_u(const double* Ucan, int dx, int dn, void* U1, void* U3, bool f32) {
  long long total = (long long)dx * dx * dn;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    int i = (int)(e % dn);
    int ab = (int)(e / dn);
    int a = ab / dx, b = ab % dx;
    double v = Ucan[e];
    st_any(U1, ((long long)i * dx + a) * dx + b, v, f32);
    // e index of U3 is (d,e) with U[e,d,k]: here (a,b) plays (e,d)
    st_any(U3, ((long long)b * dx + a) * dn + i, v, f32);
  }
}

void launch_layout_u(const double* Ucan, int dx, int dn, void* U1, void* U3, bool out_f32,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_layout_u, dim3(nblocks((long long)dx * dx * dn, 256)), dim3(256), 0, s,
                     Ucan, dx, dn, U1, U3, out_f32);
}

// ------------------------------------------------------ log-norm and trace --
// n_k from maxbits; acc += w ln n_k; trace of the normalised coarse tensor
// Tt (dims (dn,dy,dn,dy)) gives the torus estimate.
// rec[0] = ln n_k, rec[3] = acc + w ln trace (NaN if trace <= 0).
__global__ void k_norm(const unsigned long long* maxbits, const void* Tt, bool f32, int dn, int dy,
                       double w, double* acc, double* rec) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  const double nk = __longlong_as_double((long long)*maxbits);
  double s = 0.0;
  const int cnt = dn * dy;
  for (int e = t; e < cnt; e += 256) {
    int i = e / dy, j = e % dy;
    s += ld_any(Tt, (((long long)i * dy + j) * dn + i) * dy + j, f32);
  }
  red[t] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  if (t == 0) {
    double ln = log(nk);
    double a = acc[0] + w * ln;
    acc[0] = a;
    double tr = red[0] / nk;
    rec[0] = ln;
    rec[3] = tr > 0.0 ? a + w * log(tr) : __longlong_as_double(0x7ff8000000000000LL);
  }
}

void launch_norm(const unsigned long long* maxbits, const void* Tt, bool f32, int dn, int dy,
                 double weight, double* acc, double* rec, hipStream_t s) {
  hipLaunchKernelGGL(k_norm, dim3(1), dim3(256), 0, s, maxbits, Tt, f32, dn, dy, weight, acc, rec);
}

// ln Z / N = acc + w ln sum_{i,j} T[i,j,i,j]  (periodic trace, Sec. 2)
__global__ void k_finish(const void* Tn, bool f32, int dx, int dy, double w, const double* acc,
                         double* out) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  double s = 0.0;
  const int cnt = dx * dy;
  for (int e = t; e < cnt; e += 256) {
    int i = e / dy, j = e % dy;
    s += ld_any(Tn, (((long long)i * dy + j) * dx + i) * dy + j, f32);
  }
  red[t] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  if (t == 0)
    out[0] = red[0] > 0.0 ? acc[0] + w * log(red[0]) : __longlong_as_double(0x7ff8000000000000LL);
}

void launch_finish(const void* Tn, bool f32, int dx, int dy, double weight, const double* acc,
                   double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, Tn, f32, dx, dy, weight, acc, out);
}

// ----------------------------------------------- reduced-precision operands --
__device__ __forceinline__ void st_rp(void* hi, void* lo, long long i, float v, int mode) {
  if (mode == RP_F32) {
    ((float*)hi)[i] = v;
  } else {
    const __bf16 h = (__bf16)v;
    ((__bf16*)hi)[i] = h;
    ((__bf16*)lo)[i] = (__bf16)(v - (float)h);
  }
}

// The reduced-precision operands, one PrepPass each (rounded by st_rp).
__global__ __launch_bounds__(256) void k_prep_rp_pass(const void* src, bool src_f32, PrepPass P,
                                                      const unsigned long long* maxbits,
                                                      void* hi, void* lo, int mode, float* Tn) {
  __shared__ float tile[32][33];
  const double inv = 1.0 / __longlong_as_double((long long)*maxbits);
  const int na = P.n[P.ta], nb = P.n[P.tb];
  const int tiles_a = (na + 31) / 32;
  const int a0 = (blockIdx.x % tiles_a) * 32, b0 = (blockIdx.x / tiles_a) * 32;
  const long long sb = blockIdx.y * P.sst[P.o0] + blockIdx.z * P.sst[P.o1];
  const long long db = blockIdx.y * P.dst[P.o0] + blockIdx.z * P.dst[P.o1];
  const long long tb = blockIdx.y * P.tst[P.o0] + blockIdx.z * P.tst[P.o1];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const bool direct = P.dst[P.ta] == 1;
  for (int k = ty; k < 32; k += 8) {
    const int a = a0 + tx, b = b0 + k;
    float v = 0.0f;
    if (a < na && b < nb) {
      v = (float)(ld_any(src, sb + a * P.sst[P.ta] + b * P.sst[P.tb], src_f32) * inv);
      if (direct) {
        st_rp(hi, lo, db + a * P.dst[P.ta] + b * P.dst[P.tb], v, mode);
        if (Tn) Tn[tb + a * P.tst[P.ta] + b * P.tst[P.tb]] = v;
      }
    }
    tile[k][tx] = v;
  }
  if (direct) return;  // uniform
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int b = b0 + tx, a = a0 + k;
    if (a < na && b < nb) {
      const float v = tile[tx][k];
      st_rp(hi, lo, db + a * P.dst[P.ta] + b * P.dst[P.tb], v, mode);
      if (Tn) Tn[tb + a * P.tst[P.ta] + b * P.tst[P.tb]] = v;
    }
  }
}

void launch_prep_rp(const void* src, bool src_f32, bool rotate, int dx, int dy,
                    const unsigned long long* maxbits, float* Tn, int mode, const RpOps& ops,
                    long long ldP, long long ldx, hipStream_t s) {
  // logical index order (l, u, r, d), dims (dx, dy, dx, dy); the source is
  // T~ itself or, rotated, T~[u, l, d, r]
  const long long X = dx, Y = dy;
  const long long src_rot[4] = {Y * X, X * Y * X, 1, X};
  const long long src_nat[4] = {Y * X * Y, X * Y, Y, 1};
  const long long* sst = rotate ? src_rot : src_nat;
  // OT rows (l,u), K (r,d); OX rows (l,d), K (u,r); OC1 rows (u,r,d), K l;
  // OC2 rows (d,r), K (l,u)
  const long long dsts[4][4] = {{Y * ldP, ldP, Y, 1},
                                {Y * ldP, X, 1, ldP},
                                {1, X * Y * ldx, Y * ldx, ldx},
                                {Y, 1, ldP, X * ldP}};
  for (int o = 0; o < 4; ++o) {
    PrepPass P{};
    const dim3 grid = prep_pass(P, sst, dsts[o], dx, dy);
    // the FP32 copy goes with OT, whose order it shares
    hipLaunchKernelGGL(k_prep_rp_pass, grid, dim3(256), 0, s, src, src_f32, P, maxbits,
                       ops.hi[o], ops.lo[o], mode, o == 0 ? Tn : nullptr);
  }
}

__global__ void k_layout_u_rp(const double* Ucan, int dx, int dn, int mode, void* u1hi,
                              void* u1lo, void* u3hi, void* u3lo, long long ldx, long long ldn) {
  const long long total = (long long)dx * dx * dn;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % dn);
    const int ab = (int)(e / dn);
    const int a = ab / dx, b = ab % dx;
    const float v = (float)Ucan[e];
    // U1 rows (i,a), k = b
    st_rp(u1hi, u1lo, ((long long)i * dx + a) * ldx + b, v, mode);
    // U3 rows k = i, K (d,e) with U[e,d,k]: (a,b) plays (e,d) -> column d*dx + e = b*dx + a
    st_rp(u3hi, u3lo, (long long)i * ldn + (long long)b * dx + a, v, mode);
  }
}

void launch_layout_u_rp(const double* Ucan, int dx, int dn, int mode, void* u1hi, void* u1lo,
                        void* u3hi, void* u3lo, long long ldx, long long ldn, hipStream_t s) {
  const long long total = (long long)dx * dx * dn;
  hipLaunchKernelGGL(k_layout_u_rp, dim3(nblocks(total, 256)), dim3(256), 0, s, Ucan, dx, dn, mode,
                     u1hi, u1lo, u3hi, u3lo, ldx, ldn);
}

__global__ void k_f64_to_f32(const double* x, float* y, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}

__global__ void k_f32_to_f64(const float* x, double* y, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = (double)x[i];
}

void launch_f32_to_f64(const float* x, double* y, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_f32_to_f64, dim3(nblocks(n, 256)), dim3(256), 0, s, x, y, n);
}

void launch_f64_to_f32(const double* x, float* y, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_f64_to_f32, dim3(nblocks(n, 256)), dim3(256), 0, s, x, y, n);
}

}  // namespace hotrg
