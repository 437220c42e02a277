// Dense linear algebra of the hot path: Gram / projection products, blocked
// FP64 Cholesky with the inverse of the factor (for CholQR), the triangular
// update X R^{-1}, and the FP64 Lanczos estimate of the extreme eigenvalues of
// H_s.
#include <cmath>

#include "ctx.h"
#include "gemm.h"

namespace dk {

namespace {

constexpr int NB = 32;  // Cholesky block size

// out = scale * sum_s P[s]; symmetric: mirror the upper triangle (the only
// tiles computed); otherwise symmetrise (P + P^T)/2.
__global__ void reduce_square_kernel(const double* __restrict__ part, int splits, int n,
                                     double scale, int mirror_upper, double* __restrict__ out) {
  const long nn = (long)n * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nn;
       e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    const long et = (long)j + (long)i * n;  // transposed position
    double s = 0.0;
    if (mirror_upper) {
      const long src = (i <= j) ? e : et;
      for (int k = 0; k < splits; ++k) s += part[(long)k * nn + src];
    } else {
      double a = 0.0, b = 0.0;
      for (int k = 0; k < splits; ++k) { a += part[(long)k * nn + e]; b += part[(long)k * nn + et]; }
      s = 0.5 * (a + b);
    }
    out[e] = scale * s;
  }
}

// Factor the NB x NB diagonal block at (k0, k0) of the lower-triangular
// working matrix in LDS: A_kk = L L^T, then Linv = L^{-1}.  L goes back into
// the lower triangle of g, Linv into the same block of linv.
// A pivot below 1e-14 of the original diagonal entry (diag) is treated as
// singular: X is then rank-deficient to working precision.
__global__ __launch_bounds__(256) void potrf_diag_kernel(double* g, int n, int k0, double* linv,
                                                         const double* diag, unsigned* err) {
  __shared__ double a[NB][NB + 1];
  __shared__ double z[NB][NB + 1];
  const int tid = threadIdx.x;
  const int nb = min(NB, n - k0);
  for (int e = tid; e < NB * NB; e += 256) {
    const int i = e % NB, j = e / NB;
    double v = 0.0;
    if (i < nb && j < nb) v = g[(k0 + i) + (long)(k0 + j) * n];
    else if (i == j) v = 1.0;
    a[i][j] = v;
    z[i][j] = 0.0;
  }
  __syncthreads();
  // right-looking unblocked Cholesky on the lower triangle
  for (int k = 0; k < NB; ++k) {
    __shared__ double piv;
    if (tid == 0) {
      double d = a[k][k];
      const double ref = (k < nb) ? diag[k0 + k] : 1.0;
      if (!(d > 1e-14 * ref) || !isfinite(d)) { atomicOr(err, kErrNotSpd); d = 1.0; }
      piv = sqrt(d);
      a[k][k] = piv;
    }
    __syncthreads();
    for (int i = k + 1 + tid; i < NB; i += 256) a[i][k] /= piv;
    __syncthreads();
    for (int e = tid; e < NB * NB; e += 256) {
      const int i = e % NB, j = e / NB;
      if (j > k && i >= j) a[i][j] -= a[i][k] * a[j][k];
    }
    __syncthreads();
  }
  // inverse of the lower-triangular factor, one column per thread
  if (tid < NB) {
    const int j = tid;
    z[j][j] = 1.0 / a[j][j];
    for (int i = j + 1; i < NB; ++i) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s += a[i][k] * z[k][j];
      z[i][j] = -s / a[i][i];
    }
  }
  __syncthreads();
  for (int e = tid; e < NB * NB; e += 256) {
    const int i = e % NB, j = e / NB;
    if (i < nb && j < nb) {
      g[(k0 + i) + (long)(k0 + j) * n] = (i >= j) ? a[i][j] : 0.0;
      linv[(k0 + i) + (long)(k0 + j) * n] = (i >= j) ? z[i][j] : 0.0;
    }
  }
}

__global__ void diag_kernel(const double* __restrict__ g, int n, double* __restrict__ d) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    d[i] = g[i + (long)i * n];
}

__global__ void zero_kernel(double* p, long n) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    p[e] = 0.0;
}

template <typename TS, typename TD>
__global__ void copy_block_kernel(const TS* __restrict__ src, TD* __restrict__ dst, long rows,
                                  long ld, int cols) {
  const long tot = rows * cols;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot;
       e += (long)gridDim.x * blockDim.x) {
    const long c = e / rows, r = e - c * rows;
    dst[r + c * ld] = (TD)src[r + c * ld];
  }
}

__global__ void finite_kernel(const double* __restrict__ p, long n, unsigned* err) {
  bool bad = false;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    if (!isfinite(p[e])) bad = true;
  if (bad) atomicOr(err, kErrNonFinite);
}

inline int grid_for(long n) {
  long b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

hipError_t copy_block(dk_ctx* c, const void* src, void* dst, long ld, int n_s) {
  if (c->precision == DK_PREC_FP64)
    hipLaunchKernelGGL((copy_block_kernel<double, double>), dim3(grid_for(c->ngrid * n_s)),
                       dim3(256), 0, c->stream, (const double*)src, (double*)dst, c->ngrid, ld, n_s);
  else
    hipLaunchKernelGGL((copy_block_kernel<float, float>), dim3(grid_for(c->ngrid * n_s)),
                       dim3(256), 0, c->stream, (const float*)src, (float*)dst, c->ngrid, ld, n_s);
  return hipGetLastError();
}

hipError_t check_finite(dk_ctx* c, const double* p, long n) {
  hipLaunchKernelGGL(finite_kernel, dim3(grid_for(n)), dim3(256), 0, c->stream, p, n, c->err_dev);
  return hipGetLastError();
}

// ----------------------------------------------------------------- Gram --

static int gram_splits(const dk_ctx* c, int n_s) {
  GemmArgs g;
  g.M = n_s;
  g.N = n_s;
  g.K = (int)c->ngrid;
  plan_split_k(g, 2048);
  return g.splits;
}

size_t gram_ws_bytes(const dk_ctx* c, int n_s) {
  return ws_slice((size_t)gram_splits(c, n_s) * n_s * n_s * sizeof(double));
}

// out = scale * X^T Y (n_s x n_s FP64).  symmetric_x: Y == X, only the upper
// tiles are computed and mirrored; otherwise the result is symmetrised.
// FP64 context: FP64 MFMA.  Mixed context: FP64 MFMA on the widened FP32
// block (Gram), or split-BF16 MFMA (bf16x3, projection).
hipError_t gram(dk_ctx* c, const void* x, const void* y, long ld, int n_s, bool symmetric_x,
                double scale, double* out, void* ws, bool bf16x3, int kind) {
  KTimer kt(c, kind);
  GemmArgs g;
  g.M = n_s;
  g.N = n_s;
  g.K = (int)c->ngrid;
  g.A = x;
  g.lda = ld;
  g.B = y;
  g.ldb = ld;
  g.C = ws;
  g.tile_sel = symmetric_x ? kUpperTiles : kAllTiles;
  plan_split_k(g, 2048);
  hipError_t e;
  if (c->precision == DK_PREC_FP64)
    e = launch_gemm<kF64, double, double, true, true, kPartial, double>(g, c->stream);
  else if (bf16x3)
    e = launch_gemm<kBF16X3, float, float, true, true, kPartial, double>(g, c->stream);
  else
    e = launch_gemm<kF64, float, float, true, true, kPartial, double>(g, c->stream);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_square_kernel, dim3(grid_for((long)n_s * n_s)), dim3(256), 0,
                     c->stream, (const double*)ws, g.splits, n_s, scale, symmetric_x ? 1 : 0, out);
  return hipGetLastError();
}

// ------------------------------------------------------------ Cholesky --

// Blocked right-looking Cholesky G = L L^T of the symmetric positive definite
// g (n x n, column-major): the lower triangle of g is overwritten by L (the
// strictly upper blocks are left as they were) and linv receives L^{-1}
// (zero above the diagonal).  diag (n doubles) receives the diagonal of G; a
// pivot below 1e-14 of it sets kErrNotSpd.
hipError_t cholesky_inverse(dk_ctx* c, double* g, int n, double* linv, double* diag) {
  hipError_t e;
  hipLaunchKernelGGL(diag_kernel, dim3(grid_for(n)), dim3(256), 0, c->stream, g, n, diag);
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for((long)n * n)), dim3(256), 0, c->stream, linv,
                     (long)n * n);
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int nb = (n - k0 < NB) ? n - k0 : NB;
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(256), 0, c->stream, g, n, k0, linv, diag,
                       c->err_dev);
    const int rest = n - k0 - nb;
    if (rest <= 0) break;
    double* a21 = g + (k0 + nb) + (long)k0 * n;
    const double* li = linv + k0 + (long)k0 * n;
    // panel: L21 = A21 L11^{-T}   (B(k,j) = Linv11(j,k): n-contiguous)
    {
      GemmArgs p;
      p.M = rest; p.N = nb; p.K = nb;
      p.A = a21; p.lda = n;
      p.B = li; p.ldb = n;
      p.C = a21; p.ldc = n;
      e = launch_gemm<kF64, double, double, false, false, kStore, double>(p, c->stream);
      if (e != hipSuccess) return e;
    }
    // trailing update: A22 -= L21 L21^T (lower tiles)
    {
      double* a22 = g + (k0 + nb) + (long)(k0 + nb) * n;
      GemmArgs u;
      u.M = rest; u.N = rest; u.K = nb;
      u.A = a21; u.lda = n;
      u.B = a21; u.ldb = n;
      u.C = a22; u.ldc = n;
      u.Cin = a22; u.ldcin = n;
      u.alpha = -1.0; u.beta = 1.0;
      u.tile_sel = kLowerTiles;
      e = launch_gemm<kF64, double, double, false, false, kStore, double>(u, c->stream);
      if (e != hipSuccess) return e;
    }
  }
  // off-diagonal blocks of L^{-1}, one block row at a time:
  //   W = L[i0:i0+nb, 0:i0] Z[0:i0, 0:i0]        (into Z's block row i0)
  //   Z[i0:i0+nb, 0:i0] = -Linv_ii W             (in place: a workgroup reads
  //                                               its whole column tile of W
  //                                               before writing it)
  for (int i0 = NB; i0 < n; i0 += NB) {
    const int nb = (n - i0 < NB) ? n - i0 : NB;
    GemmArgs w;
    w.M = nb; w.N = i0; w.K = i0;
    w.A = g + i0; w.lda = n;        // L(i0+m, k), m-contiguous
    w.B = linv; w.ldb = n;          // Z(k, j), k-contiguous
    w.C = linv + i0; w.ldc = n;
    w.a_lower_tri = 0;
    e = launch_gemm<kF64, double, double, false, true, kStore, double>(w, c->stream);
    if (e != hipSuccess) return e;
    GemmArgs t;
    t.M = nb; t.N = i0; t.K = nb;
    t.A = linv + i0 + (long)i0 * n; t.lda = n;   // Linv_ii, m-contiguous
    t.B = linv + i0; t.ldb = n;                   // W(k, j) = linv[i0+k + j n]
    t.C = linv + i0; t.ldc = n;
    t.alpha = -1.0;
    e = launch_gemm<kF64, double, double, false, true, kStore, double>(t, c->stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// out = X L^{-T}: B(k,j) = linv(j,k) is upper triangular (zero for k > j).
hipError_t apply_right_upper(dk_ctx* c, const void* x, long ld, int n_s, const double* linv,
                             void* out) {
  GemmArgs g;
  g.M = (int)c->ngrid;
  g.N = n_s;
  g.K = n_s;
  g.A = x;
  g.lda = ld;
  g.B = linv;
  g.ldb = n_s;
  g.C = out;
  g.ldc = ld;
  g.b_upper_tri = 1;
  if (c->precision == DK_PREC_FP64)
    return launch_gemm<kF64, double, double, false, false, kStore, double>(g, c->stream);
  return launch_gemm<kF64, float, double, false, false, kStore, float>(g, c->stream);
}

// -------------------------------------------------------------- Lanczos --

namespace {

constexpr int LZ_THREADS = 1024;

__device__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
  return s;
}

// number of eigenvalues of the tridiagonal (a, b) below x (Sturm sequence)
__device__ int sturm_count(const double* a, const double* b, int m, double x) {
  int cnt = 0;
  double d = 1.0;
  for (int i = 0; i < m; ++i) {
    const double bb = (i > 0) ? b[i - 1] * b[i - 1] : 0.0;
    d = (a[i] - x) - ((i > 0) ? bb / d : 0.0);
    if (d == 0.0) d = -1e-300;
    if (d < 0.0) ++cnt;
  }
  return cnt;
}

// extreme eigenvalue of the m x m tridiagonal by parallel multisection:
// which = 0 -> smallest, 1 -> largest
__device__ double tri_extreme(const double* a, const double* b, int m, double lo, double hi,
                              int which, double* shx, int* shc) {
  for (int round = 0; round < 8; ++round) {
    const int t = threadIdx.x;
    const double x = lo + (hi - lo) * (double)(t + 1) / (double)(LZ_THREADS + 1);
    const int cnt = sturm_count(a, b, m, x);
    __syncthreads();
    shc[t] = cnt;
    shx[t] = x;
    __syncthreads();
    if (t == 0) {
      double nlo = lo, nhi = hi;
      if (which == 0) {  // first x with count >= 1
        for (int i = 0; i < LZ_THREADS; ++i)
          if (shc[i] >= 1) { nhi = shx[i]; nlo = (i > 0) ? shx[i - 1] : lo; break; }
      } else {           // first x with count >= m
        for (int i = 0; i < LZ_THREADS; ++i)
          if (shc[i] >= m) { nhi = shx[i]; nlo = (i > 0) ? shx[i - 1] : lo; break; }
      }
      shx[LZ_THREADS] = nlo;
      shx[LZ_THREADS + 1] = nhi;
    }
    __syncthreads();
    lo = shx[LZ_THREADS];
    hi = shx[LZ_THREADS + 1];
    __syncthreads();
    if (hi - lo <= 1e-17 * fmax(fabs(lo), fabs(hi))) break;
  }
  return 0.5 * (lo + hi);
}

// Single-workgroup Lanczos on the symmetric n x n matrix h (no
// re-orthogonalisation: only the two extreme Ritz values are wanted).
// Start vector 1/sqrt(n) (1, ..., 1) with a deterministic perturbation.
// Stops when both extreme Ritz values change by less than 1e-15 relative
// between checks (every 4 steps), or when the Krylov space is exhausted.
__global__ __launch_bounds__(LZ_THREADS) void lanczos_kernel(const double* __restrict__ h, int n,
                                                             int maxit, double* v, double* vp,
                                                             double* w, double* al, double* be,
                                                             double* result, unsigned* err) {
  __shared__ double sh[LZ_THREADS / 64];
  __shared__ double shx[LZ_THREADS + 2];
  __shared__ int shc[LZ_THREADS];
  const int t = threadIdx.x;
  // start vector
  double nrm = 0.0;
  for (int i = t; i < n; i += LZ_THREADS) {
    const double x = 1.0 + 0.25 * sin(0.7 * (double)i + 0.3);
    v[i] = x;
    vp[i] = 0.0;
    nrm += x * x;
  }
  nrm = sqrt(block_sum(nrm, sh));
  for (int i = t; i < n; i += LZ_THREADS) v[i] /= nrm;
  __syncthreads();
  double beta_prev = 0.0;
  double tmin_old = 0.0, tmax_old = 0.0, tmin = 0.0, tmax = 0.0;
  int m = 0;
  bool done = false;
  const int wave = t >> 6, lane = t & 63, nwaves = LZ_THREADS / 64;
  while (!done) {
    // w = h v   (h symmetric: row r = column r, contiguous)
    for (int r = wave; r < n; r += nwaves) {
      double s = 0.0;
      const double* col = h + (long)r * n;
      for (int k = lane; k < n; k += 64) s += col[k] * v[k];
      for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
      if (lane == 0) w[r] = s;
    }
    __syncthreads();
    double dot = 0.0;
    for (int i = t; i < n; i += LZ_THREADS) dot += w[i] * v[i];
    const double alpha = block_sum(dot, sh);
    double nn = 0.0;
    for (int i = t; i < n; i += LZ_THREADS) {
      const double x = w[i] - alpha * v[i] - beta_prev * vp[i];
      w[i] = x;
      nn += x * x;
    }
    const double beta = sqrt(block_sum(nn, sh));
    if (t == 0) { al[m] = alpha; be[m] = beta; }
    ++m;
    __syncthreads();
    const bool exhausted = (m >= maxit) || (m >= n) || !(beta > 1e-14 * (fabs(alpha) + fabs(beta_prev) + 1e-300));
    if (m % 4 == 0 || exhausted) {
      // Gershgorin interval of the m x m tridiagonal
      double glo = 1e300, ghi = -1e300;
      if (t == 0) {
        for (int i = 0; i < m; ++i) {
          const double r = (i > 0 ? fabs(be[i - 1]) : 0.0) + (i < m - 1 ? fabs(be[i]) : 0.0);
          glo = fmin(glo, al[i] - r);
          ghi = fmax(ghi, al[i] + r);
        }
        shx[0] = glo;
        shx[1] = ghi;
      }
      __syncthreads();
      glo = shx[0];
      ghi = shx[1];
      __syncthreads();
      tmin = tri_extreme(al, be, m, glo, ghi, 0, shx, shc);
      tmax = tri_extreme(al, be, m, glo, ghi, 1, shx, shc);
      const double scale = fmax(fabs(tmin), fabs(tmax)) + 1e-300;
      if (m >= 8 && fabs(tmin - tmin_old) <= 1e-15 * scale && fabs(tmax - tmax_old) <= 1e-15 * scale)
        done = true;
      tmin_old = tmin;
      tmax_old = tmax;
    }
    if (exhausted) {
      if (m >= maxit && !done && m < n && (beta > 1e-14 * (fabs(alpha) + fabs(beta_prev) + 1e-300)))
        if (t == 0) atomicOr(err, kErrConvergence);
      done = true;
    }
    if (!done) {
      for (int i = t; i < n; i += LZ_THREADS) {
        vp[i] = v[i];
        v[i] = w[i] / beta;
      }
      beta_prev = beta;
    }
    __syncthreads();
  }
  if (t == 0) {
    result[0] = tmin;
    result[1] = tmax;
    result[2] = (double)m;
  }
}

}  // namespace

size_t lanczos_ws_bytes(int n) {
  const int maxit = n < 2000 ? n : 2000;
  return 3 * ws_slice((size_t)n * sizeof(double)) +
         2 * ws_slice((size_t)(maxit + 1) * sizeof(double)) + ws_slice(4 * sizeof(double));
}

hipError_t lanczos_bounds(dk_ctx* c, const double* hs, int n, void* ws, double* lo, double* hi,
                          int* iters) {
  const int maxit = n < 2000 ? n : 2000;
  WsCursor cur((char*)ws, lanczos_ws_bytes(n));
  double* v = cur.take<double>(n);
  double* vp = cur.take<double>(n);
  double* w = cur.take<double>(n);
  double* al = cur.take<double>(maxit + 1);
  double* be = cur.take<double>(maxit + 1);
  double* res = cur.take<double>(4);
  if (!cur.ok) return hipErrorInvalidValue;
  hipLaunchKernelGGL(lanczos_kernel, dim3(1), dim3(LZ_THREADS), 0, c->stream, hs, n, maxit, v, vp,
                     w, al, be, res, c->err_dev);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  double host[3];
  e = hipMemcpyAsync(host, res, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return e;
  *lo = host[0];
  *hi = host[1];
  if (iters) *iters = (int)host[2];
  return hipSuccess;
}

}  // namespace dk
