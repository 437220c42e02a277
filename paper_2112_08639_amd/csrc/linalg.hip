// Dense linear algebra of the hot path: Gram / projection products, blocked
// FP64 Cholesky with the inverse of the factor (for CholQR), the triangular
// update X R^{-1}, and the FP64 extreme eigenvalues of H_s by shifted
// repeated squaring.
#include <cmath>

#include "ctx.h"
#include "gemm.h"

namespace dk {

namespace {

constexpr int NB = 32;  // Cholesky block size

// out = scale * sum_s P[s]; mirror_upper: out(i,j) = out(j,i) = the sum at
// (min(i,j), max(i,j)) (the upper tiles are the only ones computed);
// otherwise symmetrise, (P + P^T)/2.  One workgroup per pair of 16 x 16 tiles
// (bi, bj) and (bj, bi) with bi <= bj: both are read along columns and the
// transposes go through LDS, so every global access is coalesced.
constexpr int RT = 16;
template <typename PT>
__global__ __launch_bounds__(256) void reduce_square_kernel(const PT* __restrict__ part,
                                                            int splits, int n, double scale,
                                                            int mirror_upper,
                                                            double* __restrict__ out) {
  const int bi = blockIdx.x, bj = blockIdx.y;
  if (bi > bj) return;
  __shared__ double ta[RT][RT + 1];  // ta[c][r] = P(bi RT + r, bj RT + c)
  __shared__ double tb[RT][RT + 1];  // tb[c][r] = P(bj RT + r, bi RT + c)
  const long nn = (long)n * n;
  const int r = threadIdx.x % RT, c = threadIdx.x / RT;
  auto sum_at = [&](int i, int j) {
    double v = 0.0;
    if (i < n && j < n)
      for (int k = 0; k < splits; ++k) v += (double)part[(long)k * nn + i + (long)j * n];
    return v;
  };
  ta[c][r] = sum_at(bi * RT + r, bj * RT + c);
  if (!mirror_upper && bi != bj) tb[c][r] = sum_at(bj * RT + r, bi * RT + c);
  __syncthreads();
  // tile (bi, bj): element (i, j) = (bi RT + r, bj RT + c)
  {
    const int i = bi * RT + r, j = bj * RT + c;
    double v;
    if (mirror_upper) v = (bi < bj || r <= c) ? ta[c][r] : ta[r][c];
    else v = 0.5 * (ta[c][r] + (bi == bj ? ta[r][c] : tb[r][c]));
    if (i < n && j < n) out[i + (long)j * n] = scale * v;
  }
  // tile (bj, bi): element (bj RT + r, bi RT + c)
  if (bi < bj) {
    const int i = bj * RT + r, j = bi * RT + c;
    const double v = mirror_upper ? ta[r][c] : 0.5 * (tb[c][r] + ta[r][c]);
    if (i < n && j < n) out[i + (long)j * n] = scale * v;
  }
}

// Factor the NB x NB diagonal block at (k0, k0) of the lower-triangular
// working matrix: A_kk = L L^T, then Linv = L^{-1}.  L goes back into the
// lower triangle of g, Linv into the same block of linv.
// A pivot below 1e-14 of the original diagonal entry (diag) is treated as
// singular: X is then rank-deficient to working precision.
// One workgroup of 256 threads with the block in LDS; thread t owns the
// entries e = t + 256 q (q < 4) at row e % NB, column e / NB.  Both sweeps are
// right-looking with one barrier per step:
//   Cholesky step k: with d_k = a_kk, a_ij -= a_ik a_jk / d_k for k < j <= i
//   (the columns are scaled by 1/sqrt(d_k) afterwards);
//   inverse step i: z_jc -= l_ji z_ic / l_ii for j > i, c <= i, starting from
//   Z = I (the rows are scaled by 1/l_ii afterwards).
__global__ __launch_bounds__(256) void potrf_diag_kernel(double* g, int n, int k0, double* linv,
                                                         const double* diag, unsigned* err) {
  static_assert(NB == 32, "four entries of the 32 x 32 block per thread");
  __shared__ double A[NB][NB + 1];
  __shared__ double Z[NB][NB + 1];
  __shared__ double dinv[NB];  // 1 / d_k, then 1 / l_kk
  const int t = threadIdx.x;
  const int nb = min(NB, n - k0);
  int ri[4], cj[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = t + 256 * q;
    ri[q] = e & (NB - 1);
    cj[q] = e >> 5;
    const int i = ri[q], j = cj[q];
    A[i][j] = (i < nb && j < nb) ? g[(k0 + i) + (long)(k0 + j) * n] : (i == j ? 1.0 : 0.0);
    Z[i][j] = (i == j) ? 1.0 : 0.0;
  }
  // lanes 0..31 of every wave hold the original diagonal entries of rows 0..31
  const int lane = t & 63;
  const double dref = (lane < nb) ? diag[k0 + lane] : 1.0;
  __syncthreads();
  for (int k = 0; k < NB; ++k) {
    double d = A[k][k];
    const double ref = __shfl(dref, k);
    if (!(d > 1e-14 * ref) || !isfinite(d)) {
      if (t == 0) atomicOr(err, kErrNotSpd);
      d = 1.0;
    }
    const double id = 1.0 / d;
    if (t == 0) dinv[k] = id;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = ri[q], j = cj[q];
      if (j > k && i >= j) A[i][j] -= A[i][k] * A[j][k] * id;
    }
    __syncthreads();
  }
  // L: column k scaled by 1/sqrt(d_k) below the diagonal, l_kk = sqrt(d_k)
  double lval[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = ri[q], j = cj[q];
    const double s = sqrt(dinv[j]);
    lval[q] = (i > j) ? A[i][j] * s : ((i == j) ? 1.0 / s : 0.0);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) A[ri[q]][cj[q]] = lval[q];
  if (t < NB) dinv[t] = sqrt(dinv[t]);  // 1 / l_tt = 1 / sqrt(d_t)
  __syncthreads();
  for (int i = 0; i < NB; ++i) {
    const double il = dinv[i];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = ri[q], c = cj[q];
      if (j > i && c <= i) Z[j][c] -= A[j][i] * Z[i][c] * il;
    }
    __syncthreads();
  }
  // write L (zeros above the diagonal) and L^{-1} (rows scaled by 1/l_ii)
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = ri[q], j = cj[q];
    if (i < nb && j < nb) {
      g[(k0 + i) + (long)(k0 + j) * n] = (i >= j) ? A[i][j] : 0.0;
      linv[(k0 + i) + (long)(k0 + j) * n] = (i >= j) ? Z[i][j] * dinv[i] : 0.0;
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

// Split-K of the N_grid-long products X^T Y.  Up to 256 output tiles
// (N_s <= 1024): about 4096 workgroups; beyond, about 32768 counting every
// tile (half of them run for a Gram matrix), at most 128 splits.  Measured
// (FP64 MFMA on FP32 X): 884736 x 4096, 617 ms with 1 split against 325 ms
// with 8; 373248 x 2048, 54 ms with 4 against 34 ms with 32; at 110592 x 512
// 128 splits instead of 64 cost more in partial traffic than they gain.
static void plan_gram(GemmArgs& g) {
  const long tiles = (long)ceil_div(g.M, 64) * ceil_div(g.N, 64);
  plan_split_k(g, tiles <= 256 ? 4096 : 32768);
  if (g.splits > 128) {
    const long kblocks = (g.K + 63) / 64;
    const long per = (kblocks + 127) / 128;
    g.k_per_split = (int)(per * 64);
    g.splits = (int)((kblocks + per - 1) / per);
  }
}

// Beyond 256 tiles of 64 (N_s > 1024) the FP64 products X^T Y run 128 x 128
// tiles (each wave 64 x 64: half the LDS reads per MFMA of the 64 x 64 tile,
// which keeps four workgroups per CU LDS-bound).  At 884736 x 4096: the
// projection 545 against 639 ms, split to about 2048 workgroups; the Gram
// (upper tiles) 632 against 686 ms, split to about 8192 so that the last of
// its rounds is short (at about 2048: 991 ms).  On the FP32 block of the mixed
// path the 128 x 128 Gram ran slower (807 against 666 ms): it keeps 64 x 64.
constexpr int kGramWideTile = 128;
static bool gram_wide(int n_s) { return (long)ceil_div(n_s, 64) * ceil_div(n_s, 64) > 256; }
static void plan_gram_wide(GemmArgs& g, bool upper) {
  const long tm = ceil_div(g.M, kGramWideTile), tn = ceil_div(g.N, kGramWideTile);
  const long active = upper ? (tm * (tm + 1)) / 2 : tm * tn;
  const long kblocks = (g.K + 63) / 64;
  // upper tiles: about 16 rounds of two workgroups per CU, so that the last
  // round is a small part of the whole (at 3 rounds the tail cost 2x)
  long want = (upper ? 8192 : 2048) / (active > 0 ? active : 1);
  if (want < 1) want = 1;
  if (want > kblocks) want = kblocks;
  const long per = (kblocks + want - 1) / want;
  g.k_per_split = (int)(per * 64);
  g.splits = (int)((kblocks + per - 1) / per);
}

// The split-BF16 projection runs 128 x 128 tiles (four 64 x 64 sub-tiles per
// wave: enough MFMA work per slab to cover the split of the fragments) over
// about 1024 workgroups, with FP32 partials (its accumulators are FP32).
constexpr int kProjTile = 128;
static void plan_projection(GemmArgs& g) {
  const long tiles = (long)ceil_div(g.M, kProjTile) * ceil_div(g.N, kProjTile);
  long want = 1024 / (tiles > 0 ? tiles : 1);
  const long kblocks = (g.K + 63) / 64;
  if (want > 128) want = 128;
  // FP32 accumulation: at most kF32SplitBlocks blocks per split
  const long least = (kblocks + kF32SplitBlocks - 1) / kF32SplitBlocks;
  if (want < least) want = least;
  if (want > kblocks) want = kblocks;
  if (want < 1) want = 1;
  const long per = (kblocks + want - 1) / want;
  g.k_per_split = (int)(per * 64);
  g.splits = (int)((kblocks + per - 1) / per);
}

size_t gram_ws_bytes(const dk_ctx* c, int n_s) {
  GemmArgs g;
  g.M = n_s;
  g.N = n_s;
  g.K = (int)c->ngrid;
  plan_gram(g);
  size_t bytes = (size_t)g.splits * n_s * n_s * sizeof(double);
  if (c->precision == DK_PREC_FP64 && gram_wide(n_s)) {
    for (int upper = 0; upper < 2; ++upper) {
      GemmArgs w = g;
      plan_gram_wide(w, upper != 0);
      const size_t wb = (size_t)w.splits * n_s * n_s * sizeof(double);
      if (wb > bytes) bytes = wb;
    }
  }
  if (c->precision == DK_PREC_MIXED) {
    GemmArgs p = g;
    plan_projection(p);
    const size_t pb = (size_t)p.splits * n_s * n_s * sizeof(float);
    if (pb > bytes) bytes = pb;
    // the same slice holds the pieces of L^{-T} for X L^{-T}
    if (split_planes_bytes(n_s, n_s, 3) > bytes) bytes = split_planes_bytes(n_s, n_s, 3);
  }
  return ws_slice(bytes);
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
  const dim3 rgrid(ceil_div(n_s, RT), ceil_div(n_s, RT));
  hipError_t e;
  if (c->precision == DK_PREC_MIXED && bf16x3) {
    plan_projection(g);
    e = launch_gemm<kBF16X3S, float, float, true, true, kPartial, float, kProjTile, kProjTile, 32>(
        g, c->stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_square_kernel<float>, rgrid, dim3(256), 0, c->stream,
                       (const float*)ws, g.splits, n_s, scale, symmetric_x ? 1 : 0, out);
    return hipGetLastError();
  }
  if (gram_wide(n_s) && c->precision == DK_PREC_FP64) {
    plan_gram_wide(g, symmetric_x);
    e = launch_gemm<kF64, double, double, true, true, kPartial, double, kGramWideTile,
                    kGramWideTile, 8>(g, c->stream);
  } else {
    plan_gram(g);
    if (c->precision == DK_PREC_FP64)
      e = launch_gemm<kF64, double, double, true, true, kPartial, double>(g, c->stream);
    else
      e = launch_gemm<kF64, float, float, true, true, kPartial, double>(g, c->stream);
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_square_kernel<double>, rgrid, dim3(256), 0, c->stream,
                     (const double*)ws, g.splits, n_s, scale, symmetric_x ? 1 : 0, out);
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
      e = launch_gemm<kF64, double, double, false, false, kStore, double, 32>(p, c->stream);
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
      e = launch_gemm<kF64, double, double, false, false, kStore, double, 32>(u, c->stream);
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
    e = launch_gemm<kF64, double, double, false, true, kStore, double, 32>(w, c->stream);
    if (e != hipSuccess) return e;
    GemmArgs t;
    t.M = nb; t.N = i0; t.K = nb;
    t.A = linv + i0 + (long)i0 * n; t.lda = n;   // Linv_ii, m-contiguous
    t.B = linv + i0; t.ldb = n;                   // W(k, j) = linv[i0+k + j n]
    t.C = linv + i0; t.ldc = n;
    t.alpha = -1.0;
    e = launch_gemm<kF64, double, double, false, true, kStore, double, 32>(t, c->stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ----------------------------------------------------- bf16 piece planes --

// The NP bf16 pieces of an FP64 matrix, as the split-at-store products would
// split it on its way into LDS (rounded to FP32, then x = hi + lo or
// hi + mid + lo): element (k, n) = src[k*s_k + n*s_n], piece p to
// dst[p*plane + n*ldp + k] (k-contiguous), zeros for K <= k < ldp.  32 x 32
// tiles pass through LDS so that both the read (along the source's contiguous
// index) and the write (along k) are coalesced.
template <int NP>
__global__ __launch_bounds__(256) void split_planes_kernel(const double* __restrict__ src,
                                                           long s_k, long s_n, int K, int N,
                                                           __bf16* __restrict__ dst, long ldp,
                                                           long plane) {
  __shared__ float t[32][33];  // t[k][n]
  const int k0 = blockIdx.x * 32, n0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const bool n_contig = (s_n == 1);
  for (int r = ty; r < 32; r += 8) {
    const int kl = n_contig ? r : tx, nl = n_contig ? tx : r;
    const int k = k0 + kl, n = n0 + nl;
    t[kl][nl] = (k < K && n < N) ? (float)src[(long)k * s_k + (long)n * s_n] : 0.f;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int n = n0 + r, k = k0 + tx;
    if (n >= N || k >= ldp) continue;
    const float v = t[tx][r];
    __bf16* o = dst + (long)n * ldp + k;
    if constexpr (NP == 3) {
      __bf16 h, m, l;
      split3_bf16(v, h, m, l);
      o[0] = h; o[plane] = m; o[2 * plane] = l;
    } else {
      __bf16 h, l;
      split_bf16(v, h, l);
      o[0] = h; o[plane] = l;
    }
  }
}

long split_planes_ld(int K) { return ((long)K + 7) / 8 * 8; }

size_t split_planes_bytes(int K, int N, int np) {
  return ws_slice((size_t)np * N * split_planes_ld(K) * sizeof(__bf16));
}

hipError_t split_planes(dk_ctx* c, const double* src, long s_k, long s_n, int K, int N, int np,
                        void* dst) {
  const long ldp = split_planes_ld(K);
  const dim3 grid(ceil_div(ldp, 32), ceil_div(N, 32));
  if (np == 3)
    hipLaunchKernelGGL(split_planes_kernel<3>, grid, dim3(256), 0, c->stream, src, s_k, s_n, K, N,
                       (__bf16*)dst, ldp, (long)N * ldp);
  else
    hipLaunchKernelGGL(split_planes_kernel<2>, grid, dim3(256), 0, c->stream, src, s_k, s_n, K, N,
                       (__bf16*)dst, ldp, (long)N * ldp);
  return hipGetLastError();
}

// out = X L^{-T}: B(k,j) = linv(j,k) is upper triangular (zero for k > j).
// Mixed: ws receives the bf16 pieces of B (split_planes_bytes(n_s, n_s, 3)).
hipError_t apply_right_upper(dk_ctx* c, const void* x, long ld, int n_s, const double* linv,
                             void* out, void* ws) {
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
  g.xcd_groups = 0;  // measured faster in plain round-robin order
  if (c->precision == DK_PREC_FP64)
    return launch_gemm<kF64, double, double, false, false, kStore, double>(g, c->stream);
  // mixed: three-piece split-BF16 (FP32-level products for an FP32 result),
  // 128 x 128 tiles; X split once on its way into LDS, L^{-T} split beforehand
  hipError_t e = split_planes(c, linv, n_s, 1, n_s, n_s, 3, ws);
  if (e != hipSuccess) return e;
  g.B = ws;
  g.ldb = split_planes_ld(n_s);
  g.b_plane = (long)n_s * g.ldb;
  return launch_gemm<kBF16X6S, float, __bf16, false, true, kStore, float, 128, 128, 32>(g, c->stream);
}

// ------------------------------------------------------- spectral bounds --
//
// Extreme eigenvalues of the symmetric n x n H_s by shifted repeated squaring.
// For the largest: M = H - s I with s a Gershgorin lower bound (M positive
// semidefinite), X_0 = M / tr M, Y_k = X_k X_k (FP64 MFMA), X_{k+1} = Y_k / tr Y_k.
// X_k is proportional to M^(2^k), so the Rayleigh-type quotient
//   q_k = <M, Y_k>_F / tr Y_k = sum_i mu_i^(2^(k+1)+1) / sum_i mu_i^(2^(k+1))
// (mu_i the eigenvalues of M) converges to max mu with the error shrinking
// like (mu_2/mu_max)^(2^(k+1)): doubly exponentially once the top separates.
// lambda_max = q + s.  The smallest eigenvalue uses M = s' I - H with s'
// the Gershgorin upper bound, so the two sequences are independent and run
// side by side: a step is one batched GEMM of both, one reduction and one
// scaling; the host stops when both q change by less than 1e-15 relative.

namespace {

constexpr int SB_THREADS = 256;

__device__ double block_sum256(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  const double s = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return s;
}

// per row i of sym(H): lower[i] = H_ii - sum_{j!=i} |H_ij|, upper[i] = H_ii + ...,
// diag[i] = H_ii (one wave per row)
__global__ __launch_bounds__(256) void gersh_rows_kernel(const double* __restrict__ h, int n,
                                                         double* __restrict__ lower,
                                                         double* __restrict__ upper,
                                                         double* __restrict__ diag) {
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (r >= n) return;
  double off = 0.0;
  for (int k = lane; k < n; k += 64)
    if (k != r) off += fabs(0.5 * (h[k + (long)r * n] + h[r + (long)k * n]));
  for (int o = 32; o > 0; o >>= 1) off += __shfl_xor(off, o);
  if (lane == 0) {
    const double d = h[r + (long)r * n];
    lower[r] = d - off;
    upper[r] = d + off;
    diag[r] = d;
  }
}

// scal[0] = min lower, scal[1] = max upper, scal[2] = trace
__global__ __launch_bounds__(256) void gersh_reduce_kernel(const double* lower, const double* upper,
                                                           const double* diag, int n, double* scal) {
  __shared__ double sh[4];
  __shared__ double mn[256], mx[256];
  const int t = threadIdx.x;
  double a = 1e300, b = -1e300, tr = 0.0;
  for (int i = t; i < n; i += 256) { a = fmin(a, lower[i]); b = fmax(b, upper[i]); tr += diag[i]; }
  mn[t] = a;
  mx[t] = b;
  tr = block_sum256(tr, sh);
  __syncthreads();
  if (t == 0) {
    for (int i = 1; i < 256; ++i) { a = fmin(a, mn[i]); b = fmax(b, mx[i]); }
    scal[0] = fmin(a, mn[0]);
    scal[1] = fmax(b, mx[0]);
    scal[2] = tr;
  }
}

// blockIdx.y = mode; mode 0: M = sym(H) - s I, s = scal[0];  mode 1:
// M = s I - sym(H), s = scal[3].  X = M / tr M.  Mode m writes M + m n^2, X + m n^2,
// and sets its sequence's product scale alpha[m] = 1 and reduction counter cnt[m] = 0.
__global__ __launch_bounds__(256) void squaring_init_kernel(const double* __restrict__ h, int n,
                                                            const double* __restrict__ scal,
                                                            double* __restrict__ M,
                                                            double* __restrict__ X,
                                                            double* __restrict__ alpha,
                                                            unsigned* __restrict__ cnt) {
  const long nn = (long)n * n;
  const int mode = blockIdx.y;
  M += mode * nn;
  X += mode * nn;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    alpha[mode] = 1.0;
    cnt[mode] = 0u;
  }
  const double sft = mode == 0 ? scal[0] : scal[3];
  const double trm = mode == 0 ? scal[2] - n * sft : n * sft - scal[2];
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nn;
       e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    double v = 0.5 * (h[e] + h[(long)j + (long)i * n]);
    if (mode == 0) v = v - (i == j ? sft : 0.0);
    else v = (i == j ? sft : 0.0) - v;
    M[e] = v;
    X[e] = v / trm;
  }
}

// Statistics of squaring step `step` of sequence y = m0 + blockIdx.y (the pair
// M + y n^2, Y + y n^2): per-block partial sums of tr Y and <M, Y>_F into
// part + 2 y gridDim.x; the last block of the sequence to finish (an atomic
// count, no waiting) sums the partials in block order and writes
// est[y * est_stride + step] = <M, Y> / tr Y and alpha[y] = 1 / (tr Y)^2, the
// scale of the next product Y' = alpha Y Y (= (Y / tr Y)^2), and rearms the count.
__global__ __launch_bounds__(256) void squaring_stats_kernel(const double* __restrict__ M,
                                                             const double* __restrict__ Y, int n,
                                                             double* __restrict__ part, int m0,
                                                             double* __restrict__ est,
                                                             int est_stride, int step,
                                                             double* __restrict__ alpha,
                                                             unsigned* __restrict__ cnt) {
  __shared__ double sh[4];
  __shared__ bool last;
  const long nn = (long)n * n;
  const long y = m0 + (long)blockIdx.y;
  M += y * nn;
  Y += y * nn;
  part += 2L * y * gridDim.x;
  double my = 0.0, ty = 0.0;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nn;
       e += (long)gridDim.x * blockDim.x) {
    const double v = Y[e];
    my += M[e] * v;
    if (e % (n + 1) == 0) ty += v;
  }
  my = block_sum256(my, sh);
  ty = block_sum256(ty, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = ty;
    part[2 * blockIdx.x + 1] = my;
    __threadfence();  // the partials are visible before the count moves
    last = atomicAdd(cnt + y, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last || threadIdx.x >= 64) return;
  __threadfence();  // every other block's partials are visible
  double t = 0.0, m = 0.0;
  for (int i = threadIdx.x; i < (int)gridDim.x; i += 64) {
    t += part[2 * i];
    m += part[2 * i + 1];
  }
  for (int o = 32; o > 0; o >>= 1) {
    t += __shfl_xor(t, o);
    m += __shfl_xor(m, o);
  }
  if (threadIdx.x == 0) {
    est[y * est_stride + step] = m / t;
    alpha[y] = 1.0 / (t * t);
    cnt[y] = 0u;
  }
}

__global__ void set_scalar_kernel(double* p, double v) { p[0] = v; }

constexpr int SB_MAX_STEPS = 48;
constexpr int SB_PARTS = 128;

}  // namespace

size_t spectral_ws_bytes(int n) {
  const size_t nn = (size_t)n * n;
  return 3 * ws_slice(2 * nn * sizeof(double)) + 3 * ws_slice((size_t)n * sizeof(double)) +
         ws_slice(8 * sizeof(double)) + ws_slice(4 * SB_PARTS * sizeof(double)) +
         ws_slice(2 * SB_MAX_STEPS * sizeof(double)) + ws_slice(2 * sizeof(double)) +
         ws_slice(2 * sizeof(unsigned));
}

// Both squaring sequences side by side (M, X, Y hold the two n x n
// matrices back to back); q[0], q[1] are the converged quotients, *steps the
// squarings taken (both sequences counted).  A sequence that has converged is left where it is and the
// other runs on alone.  X and Y alternate as the input and output of the
// squarings; each product carries the normalisation 1 / (tr)^2 of its input
// (alpha, set by the statistics of the step before), so no pass rescales the
// matrices.
static hipError_t squaring_pair(dk_ctx* c, const double* hs, int n, double* M, double* X,
                                double* Y, double* scal, double* part, double* est, double* alpha,
                                unsigned* cnt, double* q, int* steps) {
  const long nn = (long)n * n;
  const int blocks = (int)((nn + 255) / 256 < SB_PARTS ? (nn + 255) / 256 : SB_PARTS);
  const int eblocks = (int)((nn + 255) / 256 < 4096 ? (nn + 255) / 256 : 4096);
  hipLaunchKernelGGL(squaring_init_kernel, dim3(eblocks, 2), dim3(256), 0, c->stream, hs, n, scal,
                     M, X, alpha, cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  double cur[2] = {0, 0};
  bool done_m[2] = {false, false};
  bool conv = false;
  int k = 0, squarings = 0;
  // For N_s <= 1024 the host checks step k - 1 while step k runs: each step's
  // estimates are copied to one of two pinned buffers and an event marks the
  // copy done, so the GPU does not idle during the check (a converged sequence
  // may run one squaring more, which is discarded): al32 0.86 -> 0.72 ms.
  // Larger matrices check each step as it ends (a squaring outweighs the wait).
  // (Two steps behind, with three buffers, was slower: 0.72 -> 0.77 ms.)
  const int lag = n <= 1024 ? 1 : 0;
  constexpr int kBufs = 2;
  constexpr size_t kEstBytes = 2 * SB_MAX_STEPS * sizeof(double);
  if (!c->sb_host) {
    if ((e = hipHostMalloc((void**)&c->sb_host, kBufs * kEstBytes)) != hipSuccess) return e;
    for (hipEvent_t& ev : c->sb_ev)
      if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return e;
  }
  for (; k < SB_MAX_STEPS; ++k) {
    // the sequences still running: [first, first + active)
    const int first = done_m[0] ? 1 : 0;
    const int active = (done_m[0] ? 0 : 1) + (done_m[1] ? 0 : 1);
    double* P = (k & 1) ? Y : X;  // this step's input
    double* Q = (k & 1) ? X : Y;  // and output
    GemmArgs g;
    g.M = n; g.N = n; g.K = n;
    g.A = P + first * nn; g.lda = n;
    g.B = P + first * nn; g.ldb = n;
    g.C = Q + first * nn; g.ldc = n;
    g.alpha_dev = alpha + first;
    g.batch = active;
    squarings += active;
    g.bs_a = g.bs_b = g.bs_c = nn;
    // X_k is symmetric (a power of M): upper tiles only, mirrored
    g.tile_sel = kUpperTiles;
    g.mirror = 1;
    // 32-deep K slabs: half the slab barriers of the 16-deep default for these
    // small, latency-bound products (al32 bounds 0.73 -> 0.66 ms per step)
    if (n <= 1024)
      e = launch_gemm<kF64, double, double, false, true, kStore, double, 32, 32, 32>(g, c->stream);
    else
      e = launch_gemm<kF64, double, double, false, true, kStore, double, 64>(g, c->stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(squaring_stats_kernel, dim3(blocks, active), dim3(256), 0, c->stream, M,
                       Q, n, part, first, est, SB_MAX_STEPS, k, alpha, cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    double* hb = c->sb_host + (k % kBufs) * 2 * SB_MAX_STEPS;
    if ((e = hipMemcpyAsync(hb, est, kEstBytes, hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
      return e;
    if ((e = hipEventRecord(c->sb_ev[k % kBufs], c->stream)) != hipSuccess) return e;
    const int j = k - lag;  // the step checked now
    if (j >= 5) {
      if ((e = hipEventSynchronize(c->sb_ev[j % kBufs])) != hipSuccess) return e;
      const double* two = c->sb_host + (j % kBufs) * 2 * SB_MAX_STEPS;
      bool finite = true;
      for (int m = 0; m < 2; ++m) {
        if (done_m[m]) continue;
        const double prev = two[m * SB_MAX_STEPS + j - 1];
        cur[m] = two[m * SB_MAX_STEPS + j];
        if (fabs(cur[m] - prev) <= 1e-15 * fabs(cur[m])) done_m[m] = true;
        finite = finite && std::isfinite(cur[m]);
      }
      if ((done_m[0] && done_m[1]) || !finite) { conv = done_m[0] && done_m[1]; ++k; break; }
    }
  }
  if (!conv && k >= SB_MAX_STEPS) {
    unsigned flag = 0;
    hipMemcpy(&flag, c->err_dev, sizeof flag, hipMemcpyDeviceToHost);
    flag |= kErrConvergence;
    hipMemcpy(c->err_dev, &flag, sizeof flag, hipMemcpyHostToDevice);
  }
  if (!std::isfinite(cur[0]) || !std::isfinite(cur[1])) {
    unsigned flag = 0;
    hipMemcpy(&flag, c->err_dev, sizeof flag, hipMemcpyDeviceToHost);
    flag |= kErrNonFinite;
    hipMemcpy(c->err_dev, &flag, sizeof flag, hipMemcpyHostToDevice);
  }
  q[0] = cur[0];
  q[1] = cur[1];
  *steps = squarings;
  return hipSuccess;
}

hipError_t spectral_bounds(dk_ctx* c, const double* hs, int n, void* ws, double* lo, double* hi,
                           int* iters) {
  const size_t nn = (size_t)n * n;
  WsCursor cur((char*)ws, spectral_ws_bytes(n));
  double* M = cur.take<double>(2 * nn);
  double* X = cur.take<double>(2 * nn);
  double* Y = cur.take<double>(2 * nn);
  double* lower = cur.take<double>(n);
  double* upper = cur.take<double>(n);
  double* diag = cur.take<double>(n);
  double* scal = cur.take<double>(8);
  double* part = cur.take<double>(4 * SB_PARTS);
  double* est = cur.take<double>(2 * SB_MAX_STEPS);
  double* alpha = cur.take<double>(2);
  unsigned* cnt = cur.take<unsigned>(2);
  if (!cur.ok) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gersh_rows_kernel, dim3((n + 3) / 4), dim3(256), 0, c->stream, hs, n, lower,
                     upper, diag);
  hipLaunchKernelGGL(gersh_reduce_kernel, dim3(1), dim3(256), 0, c->stream, lower, upper, diag, n,
                     scal);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  double gl[3];
  e = hipMemcpyAsync(gl, scal, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return e;
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return e;
  // a Gershgorin interval of (numerically) zero width pins both eigenvalues
  // (n = 1, or H_s a multiple of the identity): M would vanish
  const double gscale = fmax(1.0, fmax(fabs(gl[0]), fabs(gl[1])));
  if (n == 1 || gl[1] - gl[0] <= 1e-13 * gscale) {
    *lo = gl[0];
    *hi = gl[1];
    if (n == 1) *lo = *hi = gl[2];
    if (iters) *iters = 0;
    return hipSuccess;
  }
  // shift for the smallest: the Gershgorin upper bound, nudged up so that
  // s'I - H stays semidefinite through rounding
  const double sh = gl[1] + 1e-12 * (1.0 + fabs(gl[1])) + 1e-12 * (gl[1] - gl[0]);
  hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(1), 0, c->stream, scal + 3, sh);
  double q[2] = {0, 0};
  int k = 0;
  if ((e = squaring_pair(c, hs, n, M, X, Y, scal, part, est, alpha, cnt, q, &k)) != hipSuccess)
    return e;
  *hi = q[0] + gl[0];
  *lo = sh - q[1];
  if (iters) *iters = k;
  return hipSuccess;
}

}  // namespace dk
