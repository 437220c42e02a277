// Local part of the Hamiltonian on a block of grid vectors, fused with the
// Chebyshev-filter update:
//
//   Y_out = alpha * ((-1/2 Lap_h + V_eff - shift) Y_in) + beta * Y_prev
//
// -1/2 Lap_h is the twelfth-order central-difference kinetic operator of the
// paper's real-space discretisation (Sec. 5): a 37-point star of radius 6,
// periodic in x, y, z.  Y_prev may alias Y_out (the recurrence overwrites
// Y_{k-1} with Y_{k+1} point by point).  The nonlocal projector term is added
// by nonlocal_apply.
//
// Kernel layout.  A workgroup owns one column of the block, TY full x-rows of
// an xy-plane, and streams through a chunk of z-planes.  Each thread keeps the
// 13 values of its points' z-columns in registers (a queue shifted once per
// plane), so every value of Y_in is loaded from memory once per chunk plus a
// 12-plane prologue.  The centre plane of the tile, with 6 periodic halo rows
// above and below, is staged in LDS for the x and y neighbours; x wraps within
// the row.
#include "ctx.h"

namespace dk {

struct StencilArgs {
  const void* yin;
  const void* yprev;
  void* yout;
  const void* veff;
  long ld;
  int nx, ny, nz;
  int ty_tile;  // rows per tile
  int zc;       // planes per z-chunk
  double cx[7], cy[7], cz[7];  // -1/2 w_k / h_a^2, k = 1..6 (index 0 unused)
  double diag;                 // -1/2 w_0 (1/hx^2 + 1/hy^2 + 1/hz^2)
  double alpha, beta, shift;
};

template <typename T, int PPT>
__global__ __launch_bounds__(256) void stencil_kernel(StencilArgs a) {
  extern __shared__ unsigned char smem_raw[];
  T* plane = reinterpret_cast<T*>(smem_raw);
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const long pstride = (long)nx * ny;
  const int col = blockIdx.z;
  const int y0 = blockIdx.x * a.ty_tile;
  const int ty = min(a.ty_tile, ny - y0);
  const int z0 = blockIdx.y * a.zc;
  const int z1 = min(nz, z0 + a.zc);
  const int npts = nx * ty;
  const int tid = threadIdx.x;

  const T* __restrict__ yin = reinterpret_cast<const T*>(a.yin) + (long)col * a.ld;
  const T* __restrict__ yprev =
      a.yprev ? reinterpret_cast<const T*>(a.yprev) + (long)col * a.ld : nullptr;
  T* yout = reinterpret_cast<T*>(a.yout) + (long)col * a.ld;
  const T* __restrict__ veff = reinterpret_cast<const T*>(a.veff);

  T cx[7], cy[7], cz[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) { cx[k] = (T)a.cx[k]; cy[k] = (T)a.cy[k]; cz[k] = (T)a.cz[k]; }
  const T alpha = (T)a.alpha, beta = (T)a.beta, dshift = (T)(a.diag - a.shift);

  int px[PPT], prow[PPT];
  long poff[PPT];
  bool pval[PPT];
  T q[PPT][13];
#pragma unroll
  for (int r = 0; r < PPT; ++r) {
    const int p = tid + 256 * r;
    pval[r] = p < npts;
    px[r] = pval[r] ? p % nx : 0;
    prow[r] = pval[r] ? p / nx : 0;
    poff[r] = px[r] + (long)nx * (y0 + prow[r]);
  }
  // prologue: planes z0-6 .. z0+5
#pragma unroll
  for (int d = 0; d < 12; ++d) {
    int zz = z0 - 6 + d;
    zz = ((zz % nz) + nz) % nz;
#pragma unroll
    for (int r = 0; r < PPT; ++r) q[r][d] = pval[r] ? yin[zz * pstride + poff[r]] : (T)0;
  }
  const int halo_n = 12 * nx;

  for (int z = z0; z < z1; ++z) {
    int zn = z + 6;
    if (zn >= nz) zn -= nz;
#pragma unroll
    for (int r = 0; r < PPT; ++r) q[r][12] = pval[r] ? yin[zn * pstride + poff[r]] : (T)0;
    // centre plane of the tile into LDS (row offset 6)
#pragma unroll
    for (int r = 0; r < PPT; ++r)
      if (pval[r]) plane[(prow[r] + 6) * nx + px[r]] = q[r][6];
    for (int e = tid; e < halo_n; e += 256) {
      const int hr = e / nx, hx = e - hr * nx;
      const int row = hr < 6 ? hr - 6 : ty + hr - 6;
      int gy = y0 + row;
      gy = ((gy % ny) + ny) % ny;
      plane[(row + 6) * nx + hx] = yin[(long)z * pstride + hx + (long)nx * gy];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < PPT; ++r) {
      if (!pval[r]) continue;
      const int x = px[r];
      const T* rowp = plane + (prow[r] + 6) * nx;
      const long g = (long)z * pstride + poff[r];
      T acc = (dshift + veff[g]) * q[r][6];
#pragma unroll
      for (int k = 1; k <= kFdRadius; ++k) {
        int xp = x + k; if (xp >= nx) xp -= nx;
        int xm = x - k; if (xm < 0) xm += nx;
        acc += cx[k] * (rowp[xp] + rowp[xm]);
        acc += cy[k] * (rowp[x + k * nx] + rowp[x - k * nx]);
        acc += cz[k] * (q[r][6 + k] + q[r][6 - k]);
      }
      T out = alpha * acc;
      if (yprev) out += beta * yprev[g];
      yout[g] = out;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < PPT; ++r)
#pragma unroll
      for (int d = 0; d < 12; ++d) q[r][d] = q[r][d + 1];
  }
}

static void fill_coeffs(const dk_ctx* c, StencilArgs& a) {
  // twelfth-order central second-derivative weights (closed form of the
  // order-12 Lagrange stencil): w_0 = -5369/1800, w_k = 2(-1)^{k+1}(6!)^2/(k^2(6-k)!(6+k)!)
  static const double w[7] = {-5369.0 / 1800.0, 12.0 / 7.0, -15.0 / 56.0, 10.0 / 189.0,
                              -1.0 / 112.0, 2.0 / 1925.0, -1.0 / 16632.0};
  const double ix = 1.0 / (c->hx * c->hx), iy = 1.0 / (c->hy * c->hy), iz = 1.0 / (c->hz * c->hz);
  for (int k = 0; k < 7; ++k) {
    a.cx[k] = -0.5 * w[k] * ix;
    a.cy[k] = -0.5 * w[k] * iy;
    a.cz[k] = -0.5 * w[k] * iz;
  }
  a.diag = -0.5 * w[0] * (ix + iy + iz);
}

template <typename T, int PPT>
static hipError_t launch_stencil(StencilArgs a, int n_s, int n_ytiles, int n_zch, hipStream_t st) {
  size_t smem = (size_t)(a.ty_tile + 12) * a.nx * sizeof(T);
  dim3 grid(n_ytiles, n_zch, n_s);
  hipLaunchKernelGGL((stencil_kernel<T, PPT>), grid, dim3(256), smem, st, a);
  return hipGetLastError();
}

hipError_t stencil_step(dk_ctx* c, const void* yin, const void* yprev, void* yout, long ld,
                        int n_s, double alpha, double beta, double shift) {
  if (n_s <= 0) return hipSuccess;
  StencilArgs a{};
  a.yin = yin;
  a.yprev = (beta != 0.0) ? yprev : nullptr;
  a.yout = yout;
  a.ld = ld;
  a.nx = c->nx; a.ny = c->ny; a.nz = c->nz;
  a.alpha = alpha; a.beta = beta; a.shift = shift;
  fill_coeffs(c, a);
  // points per thread: enough rows for at least one full plane row per thread group
  int ppt = (int)((long)c->nx * c->ny + 255) / 256;
  if (ppt > 4) ppt = 4;
  if (ppt < 1) ppt = 1;
  int ty = (256 * ppt) / c->nx;
  if (ty > c->ny) ty = c->ny;
  if (ty < 1) return hipErrorInvalidValue;  // nx > 1024 is not supported
  a.ty_tile = ty;
  const int n_ytiles = ceil_div(c->ny, ty);
  int n_zch = ceil_div(2048, (long)n_ytiles * n_s);
  const int max_zch = c->nz / 12 > 0 ? c->nz / 12 : 1;
  if (n_zch > max_zch) n_zch = max_zch;
  if (n_zch < 1) n_zch = 1;
  a.zc = ceil_div(c->nz, n_zch);
  n_zch = ceil_div(c->nz, a.zc);
  const bool f64 = c->precision == DK_PREC_FP64;
  a.veff = f64 ? (const void*)c->veff64 : (const void*)c->veff32;
  KTimer kt(c, DK_K_STENCIL);
  switch (ppt) {
    case 1: return f64 ? launch_stencil<double, 1>(a, n_s, n_ytiles, n_zch, c->stream)
                       : launch_stencil<float, 1>(a, n_s, n_ytiles, n_zch, c->stream);
    case 2: return f64 ? launch_stencil<double, 2>(a, n_s, n_ytiles, n_zch, c->stream)
                       : launch_stencil<float, 2>(a, n_s, n_ytiles, n_zch, c->stream);
    case 3: return f64 ? launch_stencil<double, 3>(a, n_s, n_ytiles, n_zch, c->stream)
                       : launch_stencil<float, 3>(a, n_s, n_ytiles, n_zch, c->stream);
    default: return f64 ? launch_stencil<double, 4>(a, n_s, n_ytiles, n_zch, c->stream)
                        : launch_stencil<float, 4>(a, n_s, n_ytiles, n_zch, c->stream);
  }
}

// grad_h of every projector table along x, y and z (twelfth-order central
// first difference a_k = (-1)^{k+1}(6!)^2/(k(6-k)!(6+k)!)), used by the
// nonlocal force in the transposed form <chi, grad_h f> = -<grad_h chi, f>.
template <typename T>
__global__ void fd_gradient_kernel(const T* __restrict__ chi, T* __restrict__ dchi, long ngrid,
                                   int n_proj, int nx, int ny, int nz, double ihx, double ihy,
                                   double ihz) {
  const double a[7] = {0.0, 6.0 / 7.0, -15.0 / 56.0, 5.0 / 63.0, -1.0 / 56.0, 1.0 / 385.0,
                       -1.0 / 5544.0};
  const long tot = ngrid * n_proj;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot;
       e += (long)gridDim.x * blockDim.x) {
    const int p = (int)(e / ngrid);
    const long g = e - (long)p * ngrid;
    const int x = (int)(g % nx);
    const int y = (int)((g / nx) % ny);
    const int z = (int)(g / ((long)nx * ny));
    const T* col = chi + (long)p * ngrid;
    double gx = 0, gy = 0, gz = 0;
    for (int k = 1; k <= kFdRadius; ++k) {
      int xp = (x + k) % nx, xm = (x - k + nx * 8) % nx;
      int yp = (y + k) % ny, ym = (y - k + ny * 8) % ny;
      int zp = (z + k) % nz, zm = (z - k + nz * 8) % nz;
      gx += a[k] * ((double)col[xp + (long)nx * (y + (long)ny * z)] - (double)col[xm + (long)nx * (y + (long)ny * z)]);
      gy += a[k] * ((double)col[x + (long)nx * (yp + (long)ny * z)] - (double)col[x + (long)nx * (ym + (long)ny * z)]);
      gz += a[k] * ((double)col[x + (long)nx * (y + (long)ny * zp)] - (double)col[x + (long)nx * (y + (long)ny * zm)]);
    }
    dchi[e] = (T)(gx * ihx);
    dchi[tot + e] = (T)(gy * ihy);
    dchi[2 * tot + e] = (T)(gz * ihz);
  }
}

hipError_t fd_gradient_tables(dk_ctx* c) {
  if (c->n_proj == 0) return hipSuccess;
  const long tot = c->ngrid * c->n_proj;
  int blocks = (int)((tot + 255) / 256);
  if (blocks > 65536) blocks = 65536;
  // FP64 tables in both precisions: the forces are accumulated in FP64
  hipLaunchKernelGGL(fd_gradient_kernel<double>, dim3(blocks), dim3(256), 0, c->stream,
                     c->chi64, c->dchi64, c->ngrid, c->n_proj, c->nx, c->ny, c->nz,
                     1.0 / c->hx, 1.0 / c->hy, 1.0 / c->hz);
  return hipGetLastError();
}

}  // namespace dk
