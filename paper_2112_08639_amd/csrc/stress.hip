// Orbital terms of the Hellmann-Feynman stress (Sec. 3, Eqs. stressIRe and
// stressIIIRe, divided by the cell volume as in Eq. Stress:NewForm).
//
// Kinetic: sigma^I_ab = -2 sum_i <d_a x_i, d_b xt_i> / |Omega| with
// xt = X D stored once in the workspace; one kernel forms the nine sums from
// both blocks, taking the twelfth-order first differences on the fly.
//
// Nonlocal: with C = h^3 chi^T X and E = C D (so E_pi = <chi_p, xt_i>),
//   sum_i <m^b_p, d_a xt_i> C_pi = <m^b_p, d_a z_p>,   z = X E^T  (N_grid x n_proj),
// because z_p = sum_i xt_i C_pi.  The moment tables m^b_p are never stored:
// the contraction evaluates them from the projector model at the points each
// atom reaches.  The delta_ab term is -2 sum_p gamma_p sum_i E_pi C_pi.
#include "ctx.h"
#include "gemm.h"

namespace dk {

namespace {

__constant__ double kFdW[7] = {0.0, 6.0 / 7.0, -15.0 / 56.0, 5.0 / 63.0, -1.0 / 56.0, 1.0 / 385.0,
                               -1.0 / 5544.0};

// part[(col * per_col + chunk) * 9 + 3a + b] = sum over the chunk's points of
// (d_a f)(x) (d_b g)(x) for column col of f = X and g = X D (differences
// without the 1/h factors, applied by the caller).  Thread per grid point,
// 32-bit index arithmetic (N_grid < 2^31 since every axis is at most 1024).
template <typename T>
__global__ __launch_bounds__(256) void kinetic_stress_kernel(const T* __restrict__ f, long ldf,
                                                             const T* __restrict__ g, long ldg,
                                                             int nx, int ny, int nz, int per_col,
                                                             double* __restrict__ part) {
  __shared__ double red[4][9];
  const int col = blockIdx.y, chunk = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const T* fc = f + (long)col * ldf;
  const T* gc = g + (long)col * ldg;
  const int ng = nx * ny * nz, plane = nx * ny;
  double acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = 0.0;
  for (int e = chunk * 256 + threadIdx.x; e < ng; e += per_col * 256) {
    const int t = e / nx;
    const int x = e - t * nx;
    const int z = t / ny;
    const int y = t - z * ny;
    const int row = e - x, ycol = e - y * nx, zcol = e - z * plane;
    T df[3] = {0, 0, 0}, dg[3] = {0, 0, 0};
#pragma unroll
    for (int k = 1; k <= 6; ++k) {
      int xp = x + k; if (xp >= nx) xp -= nx;
      int xm = x - k; if (xm < 0) xm += nx;
      int yp = y + k; if (yp >= ny) yp -= ny;
      int ym = y - k; if (ym < 0) ym += ny;
      int zp = z + k; if (zp >= nz) zp -= nz;
      int zm = z - k; if (zm < 0) zm += nz;
      const T w = (T)kFdW[k];
      df[0] += w * (fc[row + xp] - fc[row + xm]);
      dg[0] += w * (gc[row + xp] - gc[row + xm]);
      df[1] += w * (fc[ycol + yp * nx] - fc[ycol + ym * nx]);
      dg[1] += w * (gc[ycol + yp * nx] - gc[ycol + ym * nx]);
      df[2] += w * (fc[zcol + zp * plane] - fc[zcol + zm * plane]);
      dg[2] += w * (gc[zcol + zp * plane] - gc[zcol + zm * plane]);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) acc[3 * a + b] += (double)df[a] * (double)dg[b];
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    double v = acc[k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) red[wave][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < 9)
    part[((long)col * per_col + chunk) * 9 + threadIdx.x] =
        (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

// The same sums with W consecutive x points per thread moved as one 16-byte
// vector (float x 4, double x 2; needs nx % W == 0 and 16-byte aligned
// columns): the x window of W + 12 points is read as whole vectors, periodic
// wrap by whole vectors, and each y or z neighbour row gives W points at once.
template <typename T, int W>
__global__ __launch_bounds__(256) void kinetic_stress_vec_kernel(const T* __restrict__ f, long ldf,
                                                                 const T* __restrict__ g, long ldg,
                                                                 int nx, int ny, int nz,
                                                                 int per_col,
                                                                 double* __restrict__ part) {
  static_assert(W * sizeof(T) == 16, "one 16-byte vector per group");
  constexpr int HV = (6 + W - 1) / W;  // whole vectors of halo on each side
  constexpr int NW = 2 * HV + 1;       // vectors in the x window
  typedef T vt __attribute__((ext_vector_type(W)));
  __shared__ double red[4][9];
  const int col = blockIdx.y, chunk = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const T* fc = f + (long)col * ldf;
  const T* gc = g + (long)col * ldg;
  const int segs = nx / W, plane = nx * ny;
  const int nvec = segs * ny * nz;
  double acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = 0.0;
  for (int e = chunk * 256 + threadIdx.x; e < nvec; e += per_col * 256) {
    const int t = e / segs;
    const int xs = e - t * segs;
    const int z = t / ny;
    const int y = t - z * ny;
    const int row = t * nx, x0 = xs * W;
    T wf[NW * W], wg[NW * W];
#pragma unroll
    for (int d = 0; d < NW; ++d) {
      int v = xs + d - HV;
      if (v < 0) v += segs;
      if (v >= segs) v -= segs;
      const vt a = *reinterpret_cast<const vt*>(fc + row + v * W);
      const vt b = *reinterpret_cast<const vt*>(gc + row + v * W);
#pragma unroll
      for (int j = 0; j < W; ++j) { wf[d * W + j] = a[j]; wg[d * W + j] = b[j]; }
    }
    T df[3][W], dg[3][W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
      df[0][j] = dg[0][j] = df[1][j] = dg[1][j] = df[2][j] = dg[2][j] = (T)0;
#pragma unroll
      for (int k = 1; k <= 6; ++k) {
        const int c = HV * W + j;
        df[0][j] += (T)kFdW[k] * (wf[c + k] - wf[c - k]);
        dg[0][j] += (T)kFdW[k] * (wg[c + k] - wg[c - k]);
      }
    }
    const int ycol = x0 + z * plane, zcol = x0 + y * nx;
#pragma unroll
    for (int k = 1; k <= 6; ++k) {
      int yp = y + k; if (yp >= ny) yp -= ny;
      int ym = y - k; if (ym < 0) ym += ny;
      int zp = z + k; if (zp >= nz) zp -= nz;
      int zm = z - k; if (zm < 0) zm += nz;
      const vt fyp = *reinterpret_cast<const vt*>(fc + ycol + yp * nx);
      const vt fym = *reinterpret_cast<const vt*>(fc + ycol + ym * nx);
      const vt gyp = *reinterpret_cast<const vt*>(gc + ycol + yp * nx);
      const vt gym = *reinterpret_cast<const vt*>(gc + ycol + ym * nx);
      const vt fzp = *reinterpret_cast<const vt*>(fc + zcol + zp * plane);
      const vt fzm = *reinterpret_cast<const vt*>(fc + zcol + zm * plane);
      const vt gzp = *reinterpret_cast<const vt*>(gc + zcol + zp * plane);
      const vt gzm = *reinterpret_cast<const vt*>(gc + zcol + zm * plane);
      const T w = (T)kFdW[k];
#pragma unroll
      for (int j = 0; j < W; ++j) {
        df[1][j] += w * (fyp[j] - fym[j]);
        dg[1][j] += w * (gyp[j] - gym[j]);
        df[2][j] += w * (fzp[j] - fzm[j]);
        dg[2][j] += w * (gzp[j] - gzm[j]);
      }
    }
#pragma unroll
    for (int j = 0; j < W; ++j)
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) acc[3 * a + b] += (double)df[a][j] * (double)dg[b][j];
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    double v = acc[k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) red[wave][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < 9)
    part[((long)col * per_col + chunk) * 9 + threadIdx.x] =
        (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

// part[block] = sum over the block's elements e of gamma[e % np] a[e] b[e]
// (a, b: np x n_s column-major with ld np)
__global__ __launch_bounds__(256) void gamma_dot_kernel(const double* __restrict__ a,
                                                        const double* __restrict__ b,
                                                        const double* __restrict__ gamma, int np,
                                                        long total, double* __restrict__ part) {
  __shared__ double red[4];
  double s = 0.0;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256)
    s += gamma[e % np] * a[e] * b[e];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// out[b * ncomp + k] = sum over j in block b's slice of part[j * ncomp + k],
// k < ncomp <= 9, slices of ceil(n / gridDim.x) consecutive j (fixed order).
// Thread t < span strides through the slice's flat range by span, a multiple
// of ncomp, so it always meets component t % ncomp.
__global__ __launch_bounds__(256) void sum_parts_kernel(const double* __restrict__ part, long n,
                                                        int ncomp, double* __restrict__ out) {
  __shared__ double sh[256];
  const int span = (256 / ncomp) * ncomp;
  const long per = (n + gridDim.x - 1) / gridDim.x;
  const long j0 = (long)blockIdx.x * per;
  const long j1 = j0 + per < n ? j0 + per : n;
  double s = 0.0;
  if ((int)threadIdx.x < span)
    for (long e = j0 * ncomp + threadIdx.x; e < j1 * ncomp; e += span) s += part[e];
  sh[threadIdx.x] = s;
  __syncthreads();
  if ((int)threadIdx.x < ncomp) {
    double t = 0.0;
    for (int j = threadIdx.x; j < span; j += ncomp) t += sh[j];
    out[(long)blockIdx.x * ncomp + threadIdx.x] = t;
  }
}

constexpr int kSumBlocks = 256;

// out[k] = sum_j part[j * ncomp + k]: kSumBlocks partial sums (into mid), then one block
hipError_t sum_parts(const double* part, long n, int ncomp, double* mid, double* out,
                     hipStream_t st) {
  hipLaunchKernelGGL(sum_parts_kernel, dim3(kSumBlocks), dim3(256), 0, st, part, n, ncomp, mid);
  hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(256), 0, st, (const double*)mid,
                     (long)kSumBlocks, ncomp, out);
  return hipGetLastError();
}

// part[block] = sum over the block's elements of (b - rho) v
__global__ __launch_bounds__(256) void diff_dot_kernel(const double* __restrict__ b,
                                                       const double* __restrict__ rho,
                                                       const double* __restrict__ v, long n,
                                                       double* __restrict__ part) {
  __shared__ double red[4];
  double s = 0.0;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < n; e += (long)gridDim.x * 256)
    s += (b[e] - rho[e]) * v[e];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

constexpr int kDotBlocks = 1024;

// blocks per column: about 8 points per thread, at most 65536 blocks in all
int kinetic_per_col(const dk_ctx* c, int n_s) {
  long per = (c->ngrid + 2047) / 2048;
  const long cap = 65536 / (n_s > 0 ? n_s : 1);
  if (per > cap) per = cap;
  if (per < 1) per = 1;
  return (int)per;
}

size_t elem_bytes(const dk_ctx* c) { return c->precision == DK_PREC_FP64 ? 8 : 4; }

long stress_parts(const dk_ctx* c, int n_s) {
  long p = (long)kinetic_per_col(c, n_s) * n_s;
  p = std::max(p, (long)projector_moment_stress_parts(c));
  p = std::max(p, (long)kDotBlocks);
  return p;
}

}  // namespace

// Electrostatic terms (pseudocharge model, atoms of dk_set_atoms):
//   sigma_ab = ( (1/4 pi) <d_a V, d_b V> + sum_I <sum_L d_a b_I (x-R-L)_b, V>
//              + sum_I <rho, sum_L d_a v_core,I (x-R-L)_b> + delta_ab (1/2) <b - rho, V> ) / |Omega|
size_t electrostatic_stress_ws_bytes(const dk_ctx* c) {
  const long parts = std::max<long>(std::max<long>(kinetic_per_col(c, 1), es_moment_parts(c)),
                                    kDotBlocks);
  return ws_slice(es_moment_ws_bytes(c)) + ws_slice(9 * (size_t)parts * sizeof(double)) +
         ws_slice(9 * (size_t)kSumBlocks * sizeof(double)) + ws_slice(32 * sizeof(double));
}

hipError_t electrostatic_stress(dk_ctx* c, const double* rho, const double* vc, double* sigma,
                                void* ws) {
  const long ng = c->ngrid;
  const long parts = std::max<long>(std::max<long>(kinetic_per_col(c, 1), es_moment_parts(c)),
                                    kDotBlocks);
  WsCursor cur((char*)ws, electrostatic_stress_ws_bytes(c));
  void* mws = cur.take<char>(es_moment_ws_bytes(c));
  double* part = cur.take<double>(9 * (size_t)parts);
  double* mid = cur.take<double>(9 * (size_t)kSumBlocks);
  double* out = cur.take<double>(32);
  if (!cur.ok) return hipErrorInvalidValue;
  hipError_t e;
  // (1/4 pi) <d_a V, d_b V>: the kinetic-stress kernel on the one column V
  const int per_col = kinetic_per_col(c, 1);
  if (c->nx % 2 == 0 && ng % 2 == 0)
    hipLaunchKernelGGL((kinetic_stress_vec_kernel<double, 2>), dim3(per_col, 1), dim3(256), 0,
                       c->stream, vc, ng, vc, ng, c->nx, c->ny, c->nz, per_col, part);
  else
    hipLaunchKernelGGL(kinetic_stress_kernel<double>, dim3(per_col, 1), dim3(256), 0, c->stream,
                       vc, ng, vc, ng, c->nx, c->ny, c->nz, per_col, part);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = sum_parts(part, per_col, 9, mid, out, c->stream)) != hipSuccess) return e;
  if ((e = es_moment_stress(c, rho, vc, mws, part)) != hipSuccess) return e;
  if ((e = sum_parts(part, es_moment_parts(c), 9, mid, out + 9, c->stream)) != hipSuccess) return e;
  hipLaunchKernelGGL(diff_dot_kernel, dim3(kDotBlocks), dim3(256), 0, c->stream, c->b_dev, rho, vc,
                     ng, part);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = sum_parts(part, kDotBlocks, 1, mid, out + 18, c->stream)) != hipSuccess) return e;
  double h_out[19];
  if ((e = hipMemcpyAsync(h_out, out, 19 * sizeof(double), hipMemcpyDeviceToHost, c->stream)) !=
      hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return e;
  const double vol = c->lx * c->ly * c->lz;
  const double ih[3] = {1.0 / c->hx, 1.0 / c->hy, 1.0 / c->hz};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      sigma[3 * a + b] = (c->dv * h_out[3 * a + b] * ih[a] * ih[b] / (4.0 * M_PI) +
                          c->dv * h_out[9 + 3 * a + b] + (a == b ? 0.5 * c->dv * h_out[18] : 0.0)) /
                         vol;
  return hipSuccess;
}

size_t stress_ws_bytes(const dk_ctx* c, int n_s) {
  const size_t ng = (size_t)c->ngrid, np = (size_t)c->n_proj;
  const size_t region = std::max(ng * n_s * elem_bytes(c), ng * np * sizeof(double));
  size_t b = ws_slice(region) + 2 * ws_slice(np * n_s * sizeof(double)) +
             ws_slice(9 * (size_t)stress_parts(c, n_s) * sizeof(double)) + ws_slice(32 * sizeof(double)) +
             ws_slice(9 * (size_t)kSumBlocks * sizeof(double));
  if (np > 0) b += ws_slice(projector_integrals_ws_bytes(c, n_s, (int)np));
  if (c->precision == DK_PREC_MIXED) b += split_planes_bytes(n_s, n_s, 3);
  return b;
}

hipError_t stress(dk_ctx* c, const void* x, long ld, int n_s, const double* ds, double* kinetic,
                  double* nonlocal, void* ws) {
  const size_t ng = (size_t)c->ngrid;
  const int np = c->n_proj;
  const size_t pn = (size_t)np * n_s;
  WsCursor cur((char*)ws, stress_ws_bytes(c, n_s));
  char* region = cur.take<char>(std::max(ng * n_s * elem_bytes(c), ng * (size_t)np * sizeof(double)));
  double* Cm = cur.take<double>(pn);
  double* E = cur.take<double>(pn);
  const long max_parts = stress_parts(c, n_s);
  double* part = cur.take<double>(9 * (size_t)max_parts);
  double* out = cur.take<double>(32);
  double* mid = cur.take<double>(9 * (size_t)kSumBlocks);
  void* pws = np > 0 ? cur.take<char>(projector_integrals_ws_bytes(c, n_s, np)) : nullptr;
  const bool f64 = c->precision == DK_PREC_FP64;
  void* planes = f64 ? nullptr : cur.take<char>(split_planes_bytes(n_s, n_s, 3));
  if (!cur.ok) return hipErrorInvalidValue;
  hipError_t e;

  // kinetic: xt = X D into the region, then the nine difference products
  {
    GemmArgs g;
    g.M = (int)ng; g.N = n_s; g.K = n_s;
    g.A = x; g.lda = ld;
    g.B = ds; g.ldb = n_s;
    g.C = region; g.ldc = (long)ng;
    g.n_fastest = 1;  // the n tiles of a row block share its rows of X
    if (f64) {
      e = launch_gemm<kF64, double, double, false, true, kStore, double>(g, c->stream);
    } else {
      // D split beforehand into its bf16 pieces
      e = split_planes(c, ds, 1, n_s, n_s, n_s, 3, planes);
      if (e != hipSuccess) return e;
      g.B = planes;
      g.ldb = split_planes_ld(n_s);
      g.b_plane = (long)n_s * g.ldb;
      e = launch_gemm<kBF16X6S, float, __bf16, false, true, kStore, float, 128, 128, 32>(
          g, c->stream);
    }
    if (e != hipSuccess) return e;
    const int per_col = kinetic_per_col(c, n_s);
    dim3 grid(per_col, n_s);
    const int W = f64 ? 2 : 4;
    const bool vec = c->nx % W == 0 && ld % W == 0 && ng % W == 0 &&
                     reinterpret_cast<uintptr_t>(x) % 16 == 0;
    if (f64 && vec)
      hipLaunchKernelGGL((kinetic_stress_vec_kernel<double, 2>), grid, dim3(256), 0, c->stream,
                         (const double*)x, ld, (const double*)region, (long)ng, c->nx, c->ny, c->nz,
                         per_col, part);
    else if (f64)
      hipLaunchKernelGGL(kinetic_stress_kernel<double>, grid, dim3(256), 0, c->stream,
                         (const double*)x, ld, (const double*)region, (long)ng, c->nx, c->ny, c->nz,
                         per_col, part);
    else if (vec)
      hipLaunchKernelGGL((kinetic_stress_vec_kernel<float, 4>), grid, dim3(256), 0, c->stream,
                         (const float*)x, ld, (const float*)region, (long)ng, c->nx, c->ny, c->nz,
                         per_col, part);
    else
      hipLaunchKernelGGL(kinetic_stress_kernel<float>, grid, dim3(256), 0, c->stream,
                         (const float*)x, ld, (const float*)region, (long)ng, c->nx, c->ny, c->nz,
                         per_col, part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = sum_parts(part, (long)per_col * n_s, 9, mid, out, c->stream)) != hipSuccess) return e;
  }

  // nonlocal
  if (np > 0) {
    e = projector_integrals(c, x, ld, n_s, c->chi64, np, c->dv, Cm, pws);
    if (e != hipSuccess) return e;
    GemmArgs g;  // E = C D
    g.M = np; g.N = n_s; g.K = n_s;
    g.A = Cm; g.lda = np;
    g.B = ds; g.ldb = n_s;
    g.C = E; g.ldc = np;
    e = launch_gemm<kF64, double, double, false, true, kStore, double>(g, c->stream);
    if (e != hipSuccess) return e;
    GemmArgs zg;  // z = X E^T  (N_grid x n_proj FP64)
    zg.M = (int)ng; zg.N = np; zg.K = n_s;
    zg.A = x; zg.lda = ld;
    zg.B = E; zg.ldb = np;
    zg.C = region; zg.ldc = (long)ng;
    e = f64 ? launch_gemm<kF64, double, double, false, false, kStore, double>(zg, c->stream)
            : launch_gemm<kF64, float, double, false, false, kStore, double>(zg, c->stream);
    if (e != hipSuccess) return e;
    int n_part = 0;
    e = projector_moment_stress(c, (const double*)region, part, (int)max_parts, &n_part);
    if (e != hipSuccess) return e;
    if ((e = sum_parts(part, (long)n_part, 9, mid, out + 9, c->stream)) != hipSuccess) return e;
    hipLaunchKernelGGL(gamma_dot_kernel, dim3(kDotBlocks), dim3(256), 0, c->stream, E, Cm,
                       c->gamma_dev, np, (long)pn, part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = sum_parts(part, (long)kDotBlocks, 1, mid, out + 18, c->stream)) != hipSuccess) return e;
  }
  double h_out[19] = {};
  e = hipMemcpyAsync(h_out, out, (np > 0 ? 19 : 9) * sizeof(double), hipMemcpyDeviceToHost,
                     c->stream);
  if (e != hipSuccess) return e;
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return e;
  const double vol = c->lx * c->ly * c->lz;
  const double ih[3] = {1.0 / c->hx, 1.0 / c->hy, 1.0 / c->hz};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      kinetic[3 * a + b] = -2.0 * c->dv * h_out[3 * a + b] * ih[a] * ih[b] / vol;
      nonlocal[3 * a + b] =
          (-4.0 * c->dv * h_out[9 + 3 * a + b] - (a == b ? 2.0 * h_out[18] : 0.0)) / vol;
    }
  return hipSuccess;
}

}  // namespace dk
