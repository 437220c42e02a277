// Self-consistent-field support: atoms' local fields, the electrostatic
// Poisson solve, LDA exchange-correlation, the effective potential with its
// energy integrals, Pulay mixing and the local forces.  All FP64.
//
// Electrostatics (Sec. 2, pseudocharge form of the real-space method):
//   b(x)      = sum_I -Z (pi rc^2)^(-3/2) sum_L exp(-|x - R_I - L|^2 / rc^2)
//   v_core(x) = sum_I -c sum_L exp(-|x - R_I - L|^2 / w2)
//   -Lap_h V_c = 4 pi (rho + b - mean)      (twelfth-order FD, CG, zero-mean V_c)
// The Gaussians separate per axis: each field is a sum over atoms of products
// of three one-dimensional periodic factors, tabulated once per atom and axis.
//
// Exchange-correlation: Perdew-Wang 1992 LDA (unpolarised), v_xc = d(rho eps)/d rho.
//
// Pulay mixing of the density with the residual-minimising combination of
// the last `history` difference pairs and a linear step of weight beta.
#include <cmath>

#include "ctx.h"

namespace dk {

namespace {

constexpr int TPB = 256;
constexpr int RB = 512;  // blocks of the reduction kernels

__device__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < TPB / 64; ++i) s += sh[i];
  __syncthreads();
  return s;
}

// sum of part[0..n) by one block, in a fixed order
__device__ double reduce_partials(const double* part, int n, double* sh) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += TPB) s += part[i];
  return block_sum(s, sh);
}

struct Dims {
  int nx, ny, nz;
  long ng;
  double hx, hy, hz, lx, ly, lz;
};

Dims dims_of(const dk_ctx* c) {
  return {c->nx, c->ny, c->nz, c->ngrid, c->hx, c->hy, c->hz, c->lx, c->ly, c->lz};
}

// ------------------------------------------------------------ atom fields --

// tab[(a * 4 + f) * L + off_axis + i], L = nx + ny + nz, f = 0: pseudocharge
// factor, 1: its derivative, 2: core factor, 3: its derivative; each the sum
// over periodic images d = x_i - R - n l of d^m exp(-d^2 / w2) (derivative:
// -2 d / w2 exp(...)); images beyond exp(-50) dropped.
__global__ void factor_tables_kernel(const double* __restrict__ pos, int n_atoms, Dims d,
                                     double w2b, double w2c, double* __restrict__ tab) {
  const int L = d.nx + d.ny + d.nz;
  const long total = (long)n_atoms * L;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int a = (int)(e / L);
    int i = (int)(e % L);
    int axis = 0, n = d.nx;
    double h = d.hx, len = d.lx;
    if (i >= d.nx) {
      i -= d.nx;
      axis = 1; n = d.ny; h = d.hy; len = d.ly;
      if (i >= d.ny) { i -= d.ny; axis = 2; n = d.nz; h = d.hz; len = d.lz; }
    }
    (void)n;
    const double r0 = pos[3 * a + axis];
    double d0 = i * h - r0;
    d0 -= len * rint(d0 / len);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int f = 0; f < 2; ++f) {
      const double w2 = f == 0 ? w2b : w2c;
      const double reach = sqrt(50.0 * w2);
      const int m = (int)ceil(reach / len) + 1;
      double g = 0.0, dg = 0.0;
      for (int img = -m; img <= m; ++img) {
        const double x = d0 - img * len;
        const double ex = exp(-x * x / w2);
        g += ex;
        dg += -2.0 * x / w2 * ex;
      }
      acc[2 * f] = g;
      acc[2 * f + 1] = dg;
    }
    const int off = (axis == 0) ? 0 : (axis == 1 ? d.nx : d.nx + d.ny);
    for (int f = 0; f < 4; ++f) tab[((long)a * 4 + f) * L + off + i] = acc[f];
  }
}

// b = pb sum_a Gx Gy Gz (pseudocharge factors), vcore = pc sum_a Cx Cy Cz
__global__ void local_fields_kernel(const double* __restrict__ tab, int n_atoms, Dims d,
                                    double pb, double pc, double* __restrict__ b,
                                    double* __restrict__ vcore) {
  const int L = d.nx + d.ny + d.nz;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < d.ng;
       e += (long)gridDim.x * blockDim.x) {
    const int ix = (int)(e % d.nx);
    const int iy = (int)((e / d.nx) % d.ny);
    const int iz = (int)(e / ((long)d.nx * d.ny));
    double sb = 0.0, sc = 0.0;
    for (int a = 0; a < n_atoms; ++a) {
      const double* t = tab + (long)a * 4 * L;
      sb += t[ix] * t[d.nx + iy] * t[d.nx + d.ny + iz];
      const double* u = t + 2 * L;
      sc += u[ix] * u[d.nx + iy] * u[d.nx + d.ny + iz];
    }
    b[e] = pb * sb;
    vcore[e] = pc * sc;
  }
}

// f[3 a + axis] = h^3 sum_x (pb dG_axis G G) vc + (pc dC_axis C C) rho; one block per (atom, axis)
__global__ __launch_bounds__(TPB) void local_forces_kernel(const double* __restrict__ tab,
                                                           Dims d, double pb, double pc,
                                                           const double* __restrict__ rho,
                                                           const double* __restrict__ vc,
                                                           double dv, double* __restrict__ f) {
  __shared__ double sh[TPB / 64];
  const int a = blockIdx.x / 3, axis = blockIdx.x % 3;
  const int L = d.nx + d.ny + d.nz;
  const double* t = tab + (long)a * 4 * L;
  const int off[3] = {0, d.nx, d.nx + d.ny};
  double s = 0.0;
  for (long e = threadIdx.x; e < d.ng; e += TPB) {
    const int ix = (int)(e % d.nx);
    const int iy = (int)((e / d.nx) % d.ny);
    const int iz = (int)(e / ((long)d.nx * d.ny));
    const int idx[3] = {ix, iy, iz};
    double gb = 1.0, gc = 1.0;
    for (int k = 0; k < 3; ++k) {
      const int fb = (k == axis) ? 1 : 0;
      gb *= t[fb * L + off[k] + idx[k]];
      gc *= t[(2 + fb) * L + off[k] + idx[k]];
    }
    s += pb * gb * vc[e] + pc * gc * rho[e];
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) f[blockIdx.x] = dv * s;
}

// Image moments for the electrostatic stress, same layout as the factor
// tables: mtab[(a * 4 + f) * L + off_axis + i], f = 0: sum d exp(-d^2/w2b),
// 1: -2/w2b sum d^2 exp(-d^2/w2b), 2 and 3 the same with w2c (d = x_i - R -
// n l over the periodic images).
__global__ void moment_tables_kernel(const double* __restrict__ pos, int n_atoms, Dims d,
                                     double w2b, double w2c, double* __restrict__ mtab) {
  const int L = d.nx + d.ny + d.nz;
  const long total = (long)n_atoms * L;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int a = (int)(e / L);
    int i = (int)(e % L);
    int axis = 0;
    double h = d.hx, len = d.lx;
    if (i >= d.nx) {
      i -= d.nx;
      axis = 1; h = d.hy; len = d.ly;
      if (i >= d.ny) { i -= d.ny; axis = 2; h = d.hz; len = d.lz; }
    }
    const double r0 = pos[3 * a + axis];
    double d0 = i * h - r0;
    d0 -= len * rint(d0 / len);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int f = 0; f < 2; ++f) {
      const double w2 = f == 0 ? w2b : w2c;
      const double reach = sqrt(50.0 * w2);
      const int m = (int)ceil(reach / len) + 1;
      double m1 = 0.0, m2 = 0.0;
      for (int img = -m; img <= m; ++img) {
        const double x = d0 - img * len;
        const double ex = exp(-x * x / w2);
        m1 += x * ex;
        m2 += x * x * ex;
      }
      acc[2 * f] = m1;
      acc[2 * f + 1] = -2.0 / w2 * m2;
    }
    const int off = (axis == 0) ? 0 : (axis == 1 ? d.nx : d.nx + d.ny);
    for (int f = 0; f < 4; ++f) mtab[((long)a * 4 + f) * L + off + i] = acc[f];
  }
}

// part[block * 9 + 3 a + b] = sum over the block's points x and the atoms of
//   pb [sum_L d_a b(d) d_b] vc(x) + pc [sum_L d_a c(d) d_b] rho(x)
// with b, c the unit Gaussians of the pseudocharge and core terms, from the
// factor tables (value, derivative) and the moment tables
__global__ __launch_bounds__(TPB) void es_moment_stress_kernel(const double* __restrict__ tab,
                                                               const double* __restrict__ mtab,
                                                               int n_atoms, Dims d, double pb,
                                                               double pc,
                                                               const double* __restrict__ rho,
                                                               const double* __restrict__ vc,
                                                               double* __restrict__ part) {
  __shared__ double sh[TPB / 64];
  const int L = d.nx + d.ny + d.nz;
  const int off[3] = {0, d.nx, d.nx + d.ny};
  double acc[9];
  for (int k = 0; k < 9; ++k) acc[k] = 0.0;
  for (long e = blockIdx.x * (long)TPB + threadIdx.x; e < d.ng; e += (long)gridDim.x * TPB) {
    const int idx[3] = {(int)(e % d.nx), (int)((e / d.nx) % d.ny), (int)(e / ((long)d.nx * d.ny))};
    const double wv = pb * vc[e], wr = pc * rho[e];
    for (int at = 0; at < n_atoms; ++at) {
      const double* t = tab + (long)at * 4 * L;
      const double* u = mtab + (long)at * 4 * L;
      for (int sp = 0; sp < 2; ++sp) {  // 0: pseudocharge, 1: core
        double g[3], dg[3], m1[3], dm[3];
        for (int k = 0; k < 3; ++k) {
          const int j = off[k] + idx[k];
          g[k] = t[(2 * sp) * L + j];
          dg[k] = t[(2 * sp + 1) * L + j];
          m1[k] = u[(2 * sp) * L + j];
          dm[k] = u[(2 * sp + 1) * L + j];
        }
        const double w = sp == 0 ? wv : wr;
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) {
            double v;
            if (a == b) {
              v = dm[a] * g[(a + 1) % 3] * g[(a + 2) % 3];
            } else {
              const int c = 3 - a - b;
              v = dg[a] * m1[b] * g[c];
            }
            acc[3 * a + b] += w * v;
          }
      }
    }
  }
  for (int k = 0; k < 9; ++k) {
    const double v = block_sum(acc[k], sh);
    if (threadIdx.x == 0) part[(long)blockIdx.x * 9 + k] = v;
  }
}

__global__ void add_kernel(const double* __restrict__ a, const double* __restrict__ b,
                           double* __restrict__ o, long n) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    o[e] = a[e] + b[e];
}

__global__ void negate_kernel(const double* __restrict__ s, double* __restrict__ o, long n) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    o[e] = -s[e];
}

// --------------------------------------------------------------- Poisson --

struct LapCoef {
  double cx[7], cy[7], cz[7];  // -w_k / h_a^2 (index 0 unused): -Lap_h weights
  double diag;                 // -w_0 sum_a 1/h_a^2
};

// Second-derivative weights of the twelfth-order central difference.
constexpr double kW[7] = {-5369.0 / 1800.0, 12.0 / 7.0, -15.0 / 56.0, 10.0 / 189.0,
                          -1.0 / 112.0, 2.0 / 1925.0, -1.0 / 16632.0};

LapCoef lap_coef(const Dims& d) {
  LapCoef k;
  for (int i = 0; i < 7; ++i) {
    k.cx[i] = -kW[i] / (d.hx * d.hx);
    k.cy[i] = -kW[i] / (d.hy * d.hy);
    k.cz[i] = -kW[i] / (d.hz * d.hz);
  }
  k.diag = k.cx[0] + k.cy[0] + k.cz[0];
  return k;
}

__device__ __forceinline__ double neg_lap_at(const double* __restrict__ p, long e, const Dims& d,
                                             const LapCoef& k) {
  const int ix = (int)(e % d.nx);
  const int iy = (int)((e / d.nx) % d.ny);
  const int iz = (int)(e / ((long)d.nx * d.ny));
  const long row = e - ix;                       // start of the x-row
  const long plane = (long)d.nx * d.ny;
  const long pz = (long)iz * plane;
  double s = k.diag * p[e];
#pragma unroll
  for (int r = 1; r <= 6; ++r) {
    int xp = ix + r; if (xp >= d.nx) xp -= d.nx;
    int xm = ix - r; if (xm < 0) xm += d.nx;
    int yp = iy + r; if (yp >= d.ny) yp -= d.ny;
    int ym = iy - r; if (ym < 0) ym += d.ny;
    int zp = iz + r; if (zp >= d.nz) zp -= d.nz;
    int zm = iz - r; if (zm < 0) zm += d.nz;
    s += k.cx[r] * (p[row + xp] + p[row + xm]);
    s += k.cy[r] * (p[pz + (long)yp * d.nx + ix] + p[pz + (long)ym * d.nx + ix]);
    s += k.cz[r] * (p[(long)zp * plane + (long)iy * d.nx + ix] +
                    p[(long)zm * plane + (long)iy * d.nx + ix]);
  }
  return s;
}

struct CgState {
  double rr, bb, alpha, beta, mean;
  int done;  // 1 converged, 2 iteration limit
  int iters;
};

__global__ __launch_bounds__(TPB) void sum_kernel(const double* __restrict__ x, long n,
                                                  double* __restrict__ part) {
  __shared__ double sh[TPB / 64];
  double s = 0.0;
  for (long e = blockIdx.x * (long)TPB + threadIdx.x; e < n; e += (long)gridDim.x * TPB) s += x[e];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(TPB) void cg_mean_kernel(const double* part, int nb, long n,
                                                      int center, CgState* st) {
  __shared__ double sh[TPB / 64];
  const double s = center ? reduce_partials(part, nb, sh) : 0.0;
  if (threadIdx.x == 0) {
    st->mean = center ? s / (double)n : 0.0;
    st->done = 0;
    st->iters = 0;
  }
}

// ap = (-Lap_h + shift) p; part = per-block sum of p . ap
__global__ __launch_bounds__(TPB) void cg_apply_kernel(const double* __restrict__ p,
                                                       double* __restrict__ ap, Dims d, LapCoef k,
                                                       double shift, double* __restrict__ part,
                                                       const CgState* st) {
  __shared__ double sh[TPB / 64];
  if (st->done) return;
  double s = 0.0;
  for (long e = blockIdx.x * (long)TPB + threadIdx.x; e < d.ng; e += (long)gridDim.x * TPB) {
    const double v = neg_lap_at(p, e, d, k) + shift * p[e];
    ap[e] = v;
    s += p[e] * v;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// r = scale (src - mean) - ap, p = r; partials of r.r and of |scale (src - mean)|^2
__global__ __launch_bounds__(TPB) void cg_init_kernel(const double* __restrict__ src,
                                                      const double* __restrict__ ap,
                                                      double* __restrict__ r,
                                                      double* __restrict__ p, long n,
                                                      double scale, double* __restrict__ part,
                                                      const CgState* st) {
  __shared__ double sh[TPB / 64];
  const double mean = st->mean;
  double srr = 0.0, sbb = 0.0;
  for (long e = blockIdx.x * (long)TPB + threadIdx.x; e < n; e += (long)gridDim.x * TPB) {
    const double rhs = scale * (src[e] - mean);
    const double v = rhs - ap[e];
    r[e] = v;
    p[e] = v;
    srr += v * v;
    sbb += rhs * rhs;
  }
  srr = block_sum(srr, sh);
  sbb = block_sum(sbb, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = srr;
    part[RB + blockIdx.x] = sbb;
  }
}

__global__ __launch_bounds__(TPB) void cg_start_kernel(const double* part, int nb, double tol2,
                                                       CgState* st) {
  __shared__ double sh[TPB / 64];
  const double rr = reduce_partials(part, nb, sh);
  const double bb = reduce_partials(part + RB, nb, sh);
  if (threadIdx.x == 0) {
    st->rr = rr;
    st->bb = bb;
    st->done = (rr <= tol2 * bb) ? 1 : 0;
  }
}

__global__ __launch_bounds__(TPB) void cg_alpha_kernel(const double* part, int nb, CgState* st) {
  __shared__ double sh[TPB / 64];
  if (st->done) return;
  const double pap = reduce_partials(part, nb, sh);
  if (threadIdx.x == 0) st->alpha = st->rr / pap;
}

// x += alpha p, r -= alpha ap; partials of r.r
__global__ __launch_bounds__(TPB) void cg_update_kernel(double* __restrict__ x,
                                                        double* __restrict__ r,
                                                        const double* __restrict__ p,
                                                        const double* __restrict__ ap, long n,
                                                        double* __restrict__ part,
                                                        const CgState* st) {
  __shared__ double sh[TPB / 64];
  if (st->done) return;
  const double a = st->alpha;
  double s = 0.0;
  for (long e = blockIdx.x * (long)TPB + threadIdx.x; e < n; e += (long)gridDim.x * TPB) {
    x[e] += a * p[e];
    const double v = r[e] - a * ap[e];
    r[e] = v;
    s += v * v;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(TPB) void cg_beta_kernel(const double* part, int nb, double tol2,
                                                      int max_iter, CgState* st) {
  __shared__ double sh[TPB / 64];
  if (st->done) return;
  const double rr = reduce_partials(part, nb, sh);
  if (threadIdx.x == 0) {
    st->iters += 1;
    st->beta = rr / st->rr;
    st->rr = rr;
    if (rr <= tol2 * st->bb) st->done = 1;
    else if (st->iters >= max_iter) st->done = 2;
  }
}

__global__ void cg_direction_kernel(double* __restrict__ p, const double* __restrict__ r, long n,
                                    const CgState* st) {
  if (st->done) return;
  const double b = st->beta;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    p[e] = r[e] + b * p[e];
}

__global__ void subtract_mean_kernel(double* __restrict__ x, long n, const double* part, int nb) {
  __shared__ double sh[TPB / 64];
  const double m = reduce_partials(part, nb, sh) / (double)n;
  for (long e = blockIdx.x * (long)TPB + threadIdx.x; e < n; e += (long)gridDim.x * TPB) x[e] -= m;
}

// ------------------------------------------------------------------- LDA --

constexpr double kPwA = 0.031091, kPwAlpha1 = 0.21370;
constexpr double kPwB1 = 7.5957, kPwB2 = 3.5876, kPwB3 = 1.6382, kPwB4 = 0.49294;
constexpr double kRhoFloor = 1e-20;

// eps_xc and v_xc of the unpolarised gas (Perdew-Wang 1992 correlation, Slater exchange)
__device__ __forceinline__ void pw92(double rho, double& eps, double& v) {
  if (!(rho > kRhoFloor)) { eps = 0.0; v = 0.0; return; }
  const double rs = cbrt(3.0 / (4.0 * M_PI * rho));
  const double cx = (3.0 / (4.0 * M_PI)) * cbrt(9.0 * M_PI / 4.0);
  const double ex = -cx / rs;
  const double srs = sqrt(rs);
  const double q0 = -2.0 * kPwA * (1.0 + kPwAlpha1 * rs);
  const double q1 = 2.0 * kPwA * (kPwB1 * srs + kPwB2 * rs + kPwB3 * rs * srs + kPwB4 * rs * rs);
  const double dq1 = kPwA * (kPwB1 / srs + 2.0 * kPwB2 + 3.0 * kPwB3 * srs + 4.0 * kPwB4 * rs);
  const double lg = log1p(1.0 / q1);
  const double ec = q0 * lg;
  const double dec = -2.0 * kPwA * kPwAlpha1 * lg - q0 * dq1 / (q1 * q1 + q1);
  eps = ex + ec;
  v = (4.0 / 3.0) * ex + ec - (rs / 3.0) * dec;
}

// veff = vc + vcore + vxc (any of vc / vcore / veff may be null: then xc only);
// partials [4][RB]: rho eps, rho vc, rho vxc, (rho + b) vc
__global__ __launch_bounds__(TPB) void potential_kernel(const double* __restrict__ rho,
                                                        const double* __restrict__ b,
                                                        const double* __restrict__ vc,
                                                        const double* __restrict__ vcore,
                                                        double* __restrict__ vxc_out,
                                                        double* __restrict__ veff, long n,
                                                        double* __restrict__ part) {
  __shared__ double sh[TPB / 64];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (long e = blockIdx.x * (long)TPB + threadIdx.x; e < n; e += (long)gridDim.x * TPB) {
    const double r = rho[e];
    double eps, v;
    pw92(r, eps, v);
    if (vxc_out) vxc_out[e] = v;
    s0 += r * eps;
    s2 += r * v;
    if (vc) {
      const double c = vc[e];
      s1 += r * c;
      s3 += (r + b[e]) * c;
      if (veff) veff[e] = c + vcore[e] + v;
    }
  }
  s0 = block_sum(s0, sh);
  s1 = block_sum(s1, sh);
  s2 = block_sum(s2, sh);
  s3 = block_sum(s3, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s0;
    part[RB + blockIdx.x] = s1;
    part[2 * RB + blockIdx.x] = s2;
    part[3 * RB + blockIdx.x] = s3;
  }
}

__global__ __launch_bounds__(TPB) void reduce_rows_small_kernel(const double* part, int nb,
                                                                int rows, double* out) {
  __shared__ double sh[TPB / 64];
  for (int q = 0; q < rows; ++q) {
    const double s = reduce_partials(part + (long)q * RB, nb, sh);
    if (threadIdx.x == 0) out[q] = s;
  }
}

// out = -Lap_h f
__global__ void neg_lap_kernel(const double* __restrict__ f, double* __restrict__ out, Dims d,
                               LapCoef k) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < d.ng; e += (long)gridDim.x * blockDim.x)
    out[e] = neg_lap_at(f, e, d, k);
}

__global__ void fill_kernel(double* __restrict__ x, double v, long n) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    x[e] = v;
}

// y += a x
__global__ void axpy_kernel(double a, const double* __restrict__ x, double* __restrict__ y, long n) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    y[e] += a * x[e];
}

// ----------------------------------------------------------------- Pulay --

// F = out - in; with history: dR[slot] = in - prev_in, dF[slot] = F - prev_F.
// partials: |F|^2, |out|^2
__global__ __launch_bounds__(TPB) void pulay_prepare_kernel(const double* __restrict__ in,
                                                            const double* __restrict__ out,
                                                            const double* __restrict__ prev_in,
                                                            const double* __restrict__ prev_f,
                                                            double* __restrict__ fcur,
                                                            double* __restrict__ dr,
                                                            double* __restrict__ df, long n,
                                                            int have_prev,
                                                            double* __restrict__ part) {
  __shared__ double sh[TPB / 64];
  double sf = 0.0, so = 0.0;
  for (long e = blockIdx.x * (long)TPB + threadIdx.x; e < n; e += (long)gridDim.x * TPB) {
    const double o = out[e], i = in[e];
    const double f = o - i;
    fcur[e] = f;
    if (have_prev) {
      dr[e] = i - prev_in[e];
      df[e] = f - prev_f[e];
    }
    sf += f * f;
    so += o * o;
  }
  sf = block_sum(sf, sh);
  so = block_sum(so, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = sf;
    part[RB + blockIdx.x] = so;
  }
}

// grid (RB, products): product q < m*m is dF_i . dF_j (i = q / m, j = q % m),
// q >= m*m is dF_{q - m*m} . F
__global__ __launch_bounds__(TPB) void pulay_dots_kernel(const double* __restrict__ df,
                                                         const double* __restrict__ fcur,
                                                         long n, int m,
                                                         double* __restrict__ part) {
  __shared__ double sh[TPB / 64];
  const int q = blockIdx.y;
  const double* u;
  const double* v;
  if (q < m * m) { u = df + (long)(q / m) * n; v = df + (long)(q % m) * n; }
  else { u = df + (long)(q - m * m) * n; v = fcur; }
  double s = 0.0;
  for (long e = blockIdx.x * (long)TPB + threadIdx.x; e < n; e += (long)gridDim.x * TPB)
    s += u[e] * v[e];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[(long)(2 + q) * RB + blockIdx.x] = s;
}

// reduce the partials, solve (A + eps tr(A)/m I) gamma = rhs by Cholesky
// (one block; the tiny solve in thread 0); out: gamma[0..m), [8] = |F|/|out|
__global__ __launch_bounds__(TPB) void pulay_solve_kernel(const double* part, int nb, int m,
                                                          double reg, double* out) {
  __shared__ double sh[TPB / 64];
  __shared__ double vals[2 + 8 * 8 + 8];
  const int nq = 2 + m * m + m;
  for (int q = 0; q < nq; ++q) {
    const double s = reduce_partials(part + (long)q * RB, nb, sh);
    if (threadIdx.x == 0) vals[q] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  out[8] = sqrt(vals[0]) / sqrt(vals[1]);
  if (m == 0) return;
  double A[8][8], g[8];
  double tr = 0.0;
  for (int i = 0; i < m; ++i) tr += vals[2 + i * m + i];
  const double shift = reg * tr / m;
  for (int i = 0; i < m; ++i) {
    for (int j = 0; j < m; ++j) A[i][j] = vals[2 + i * m + j];
    A[i][i] += shift;
    g[i] = vals[2 + m * m + i];
  }
  // Cholesky A = L L^T in place (lower)
  for (int j = 0; j < m; ++j) {
    double d = A[j][j];
    for (int k = 0; k < j; ++k) d -= A[j][k] * A[j][k];
    d = sqrt(d > 0.0 ? d : 0.0);
    A[j][j] = d;
    for (int i = j + 1; i < m; ++i) {
      double s = A[i][j];
      for (int k = 0; k < j; ++k) s -= A[i][k] * A[j][k];
      A[i][j] = d > 0.0 ? s / d : 0.0;
    }
  }
  for (int i = 0; i < m; ++i) {  // L y = g
    double s = g[i];
    for (int k = 0; k < i; ++k) s -= A[i][k] * g[k];
    g[i] = A[i][i] > 0.0 ? s / A[i][i] : 0.0;
  }
  for (int i = m - 1; i >= 0; --i) {  // L^T gamma = y
    double s = g[i];
    for (int k = i + 1; k < m; ++k) s -= A[k][i] * g[k];
    g[i] = A[i][i] > 0.0 ? s / A[i][i] : 0.0;
  }
  for (int i = 0; i < m; ++i) out[i] = g[i];
}

// next = in + beta F - sum_j gamma_j (dR_j + beta dF_j); prev_in = in, prev_F = F
__global__ void pulay_combine_kernel(const double* __restrict__ in, const double* __restrict__ fcur,
                                     const double* __restrict__ dr, const double* __restrict__ df,
                                     const double* __restrict__ gamma, int m, double beta, long n,
                                     double* __restrict__ next, double* __restrict__ prev_in,
                                     double* __restrict__ prev_f) {
  double gm[8];
  for (int j = 0; j < 8; ++j) gm[j] = j < m ? gamma[j] : 0.0;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const double i = in[e], f = fcur[e];
    double v = i + beta * f;
    for (int j = 0; j < m; ++j) v -= gm[j] * (dr[(long)j * n + e] + beta * df[(long)j * n + e]);
    next[e] = v;
    prev_in[e] = i;
    prev_f[e] = f;
  }
}

// rho_bar = in - sum_j gamma_j dR_j -> next, F_bar = F - sum_j gamma_j dF_j -> fbar;
// prev_in = in, prev_F = F
__global__ void pulay_bar_kernel(const double* __restrict__ in, const double* __restrict__ fcur,
                                 const double* __restrict__ dr, const double* __restrict__ df,
                                 const double* __restrict__ gamma, int m, long n,
                                 double* __restrict__ next, double* __restrict__ fbar,
                                 double* __restrict__ prev_in, double* __restrict__ prev_f) {
  double gm[8];
  for (int j = 0; j < 8; ++j) gm[j] = j < m ? gamma[j] : 0.0;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const double i = in[e], f = fcur[e];
    double r = i, g = f;
    for (int j = 0; j < m; ++j) {
      r -= gm[j] * dr[(long)j * n + e];
      g -= gm[j] * df[(long)j * n + e];
    }
    next[e] = r;
    fbar[e] = g;
    prev_in[e] = i;
    prev_f[e] = f;
  }
}

inline int grid_for(long n) {
  long b = (n + TPB - 1) / TPB;
  return (int)(b > RB ? RB : (b < 1 ? 1 : b));
}

// ------------------------------------------------------ molecular dynamics --

// v += scale f  (scale = (dt/2) / M)
__global__ void md_kick_kernel(double* __restrict__ v, const double* __restrict__ f, double scale,
                               int n) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x)
    v[e] += scale * f[e];
}

// x += dt v
__global__ void md_drift_kernel(double* __restrict__ x, const double* __restrict__ v, double dt,
                                int n) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x)
    x[e] += dt * v[e];
}

// out[0] = (M/2) sum v^2 (one block)
__global__ __launch_bounds__(TPB) void md_kinetic_kernel(const double* __restrict__ v, int n,
                                                         double mass, double* __restrict__ out) {
  __shared__ double sh[TPB / 64];
  double s = 0.0;
  for (int e = threadIdx.x; e < n; e += TPB) s += v[e] * v[e];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[0] = 0.5 * mass * s;
}

// Isokinetic half kick (one block): the exact flow over tau of
// dv/dt = g - (g.v / v.v) v with g = f / M held fixed,
//   v <- (v + g s) / s',  s = a tau^2 (cosh w - 1)/w^2 + tau sinh(w)/w,
//   s' = a tau sinh(w)/w + cosh w,  w = sqrt(b) tau,
// a = g.v / v.v, b = g.g / v.v; (cosh w - 1)/w^2 = (sinh(w/2)/(w/2))^2 / 2.
__global__ __launch_bounds__(TPB) void md_isokinetic_kernel(double* __restrict__ v,
                                                            const double* __restrict__ f,
                                                            double inv_mass, double tau, int n) {
  __shared__ double sh[TPB / 64];
  double vv = 0.0, gv = 0.0, gg = 0.0;
  for (int e = threadIdx.x; e < n; e += TPB) {
    const double g = f[e] * inv_mass;
    vv += v[e] * v[e];
    gv += g * v[e];
    gg += g * g;
  }
  vv = block_sum(vv, sh);
  gv = block_sum(gv, sh);
  gg = block_sum(gg, sh);
  if (!(vv > 0.0)) return;  // no motion: the friction term is undefined, v stays 0
  const double a = gv / vv, b = gg / vv;
  const double w = sqrt(b) * tau;
  const double sinhc = w > 0.0 ? sinh(w) / w : 1.0;
  const double half = w > 0.0 ? sinh(0.5 * w) / (0.5 * w) : 1.0;
  const double s = a * tau * tau * 0.5 * half * half + tau * sinhc;
  const double sdot = a * tau * sinhc + cosh(w);
  for (int e = threadIdx.x; e < n; e += TPB) v[e] = (v[e] + f[e] * inv_mass * s) / sdot;
}

}  // namespace

hipError_t md_isokinetic_kick(dk_ctx* c, double* v, const double* f, double inv_mass, double tau,
                              int n) {
  hipLaunchKernelGGL(md_isokinetic_kernel, dim3(1), dim3(TPB), 0, c->stream, v, f, inv_mass, tau,
                     n);
  return hipGetLastError();
}

hipError_t md_kick(dk_ctx* c, double* v, const double* f, double scale, int n) {
  hipLaunchKernelGGL(md_kick_kernel, dim3((n + TPB - 1) / TPB), dim3(TPB), 0, c->stream, v, f,
                     scale, n);
  return hipGetLastError();
}

hipError_t md_drift(dk_ctx* c, double* x, const double* v, double dt, int n) {
  hipLaunchKernelGGL(md_drift_kernel, dim3((n + TPB - 1) / TPB), dim3(TPB), 0, c->stream, x, v,
                     dt, n);
  return hipGetLastError();
}

hipError_t md_kinetic(dk_ctx* c, const double* v, int n, double mass, double* out_dev) {
  hipLaunchKernelGGL(md_kinetic_kernel, dim3(1), dim3(TPB), 0, c->stream, v, n, mass, out_dev);
  return hipGetLastError();
}


// ---------------------------------------------------------------- host side --

size_t atom_tables_bytes(const dk_ctx* c, int n_atoms) {
  return (size_t)n_atoms * 4 * (c->nx + c->ny + c->nz) * sizeof(double);
}

hipError_t local_fields(dk_ctx* c, const double* pos_dev, int n_atoms, double z, double rc,
                        double core_amp, double core_w2, double* tab, double* b, double* vcore) {
  const Dims d = dims_of(c);
  const long tn = (long)n_atoms * (d.nx + d.ny + d.nz);
  hipLaunchKernelGGL(factor_tables_kernel, dim3((int)((tn + TPB - 1) / TPB)), dim3(TPB), 0,
                     c->stream, pos_dev, n_atoms, d, rc * rc, core_w2, tab);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const double pb = -z * pow(M_PI * rc * rc, -1.5);
  long blocks = (d.ng + TPB - 1) / TPB;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(local_fields_kernel, dim3((int)blocks), dim3(TPB), 0, c->stream, tab,
                     n_atoms, d, pb, -core_amp, b, vcore);
  return hipGetLastError();
}

hipError_t local_forces(dk_ctx* c, const double* tab, int n_atoms, double z, double rc,
                        double core_amp, const double* rho, const double* vc, double* f_dev) {
  const Dims d = dims_of(c);
  const double pb = -z * pow(M_PI * rc * rc, -1.5);
  hipLaunchKernelGGL(local_forces_kernel, dim3(3 * n_atoms), dim3(TPB), 0, c->stream, tab, d, pb,
                     -core_amp, rho, vc, c->dv, f_dev);
  return hipGetLastError();
}

size_t es_moment_ws_bytes(const dk_ctx* c) {
  const int na = c->n_local_atoms > 0 ? c->n_local_atoms : 1;
  return ws_slice(atom_tables_bytes(c, na));
}

int es_moment_parts(const dk_ctx* c) { return grid_for(c->ngrid); }

hipError_t es_moment_stress(dk_ctx* c, const double* rho, const double* vc, void* ws,
                            double* part) {
  const Dims d = dims_of(c);
  const int na = c->n_local_atoms;
  WsCursor cur((char*)ws, es_moment_ws_bytes(c));
  double* mtab = cur.take<double>(atom_tables_bytes(c, na > 0 ? na : 1) / sizeof(double));
  if (!cur.ok) return hipErrorInvalidValue;
  const long tn = (long)na * (d.nx + d.ny + d.nz);
  hipLaunchKernelGGL(moment_tables_kernel, dim3((int)((tn + TPB - 1) / TPB)), dim3(TPB), 0,
                     c->stream, c->pos_dev, na, d, c->loc_rc * c->loc_rc, c->loc_core_w2, mtab);
  const double pb = -c->loc_z * pow(M_PI * c->loc_rc * c->loc_rc, -1.5);
  hipLaunchKernelGGL(es_moment_stress_kernel, dim3(es_moment_parts(c)), dim3(TPB), 0, c->stream,
                     c->atom_tab, mtab, na, d, pb, -c->loc_core_amp, rho, vc, part);
  return hipGetLastError();
}

hipError_t negate(dk_ctx* c, const double* src, double* dst) {
  hipLaunchKernelGGL(negate_kernel, dim3(grid_for(c->ngrid)), dim3(TPB), 0, c->stream, src, dst,
                     c->ngrid);
  return hipGetLastError();
}

hipError_t add_fields(dk_ctx* c, const double* a, const double* b, double* out) {
  hipLaunchKernelGGL(add_kernel, dim3(grid_for(c->ngrid)), dim3(TPB), 0, c->stream, a, b, out,
                     c->ngrid);
  return hipGetLastError();
}

size_t poisson_ws_bytes(const dk_ctx* c);

// Conjugate gradients for (-Lap_h + shift) x = scale (src - mean), mean the
// average of src when center (the singular Poisson case, shift = 0; the
// solution is then returned with zero mean), else 0.  x holds the start
// vector.  Convergence: |r| <= tol |scale (src - mean)|.
static hipError_t cg_solve(dk_ctx* c, const double* src, double* x, double tol, int max_iter,
                           void* ws, double scale, double shift, bool center, int* iters,
                           double* relres, int* status) {
  const Dims d = dims_of(c);
  const long n = d.ng;
  WsCursor cur((char*)ws, poisson_ws_bytes(c));
  double* r = cur.take<double>(n);
  double* p = cur.take<double>(n);
  double* ap = cur.take<double>(n);
  double* part = cur.take<double>(4 * RB);
  CgState* st = cur.take<CgState>(1);
  if (!cur.ok) return hipErrorInvalidValue;
  const LapCoef k = lap_coef(d);
  const int nb = grid_for(n);
  const double tol2 = tol * tol;
  hipStream_t s = c->stream;
  if (center) hipLaunchKernelGGL(sum_kernel, dim3(nb), dim3(TPB), 0, s, src, n, part);
  hipLaunchKernelGGL(cg_mean_kernel, dim3(1), dim3(TPB), 0, s, part, nb, n, center ? 1 : 0, st);
  hipLaunchKernelGGL(cg_apply_kernel, dim3(nb), dim3(TPB), 0, s, x, ap, d, k, shift, part, st);
  hipLaunchKernelGGL(cg_init_kernel, dim3(nb), dim3(TPB), 0, s, src, ap, r, p, n, scale, part, st);
  hipLaunchKernelGGL(cg_start_kernel, dim3(1), dim3(TPB), 0, s, part, nb, tol2, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  CgState host{};
  constexpr int kBatch = 32;  // iterations queued between host checks
  for (;;) {
    for (int it = 0; it < kBatch; ++it) {
      hipLaunchKernelGGL(cg_apply_kernel, dim3(nb), dim3(TPB), 0, s, p, ap, d, k, shift, part, st);
      hipLaunchKernelGGL(cg_alpha_kernel, dim3(1), dim3(TPB), 0, s, part, nb, st);
      hipLaunchKernelGGL(cg_update_kernel, dim3(nb), dim3(TPB), 0, s, x, r, p, ap, n, part, st);
      hipLaunchKernelGGL(cg_beta_kernel, dim3(1), dim3(TPB), 0, s, part, nb, tol2, max_iter, st);
      hipLaunchKernelGGL(cg_direction_kernel, dim3(nb), dim3(TPB), 0, s, p, r, n, st);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(&host, st, sizeof host, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    if (host.done) break;
  }
  if (center) {
    // the iterates keep the mean of the start vector: return the zero-mean solution
    hipLaunchKernelGGL(sum_kernel, dim3(nb), dim3(TPB), 0, s, x, n, part);
    hipLaunchKernelGGL(subtract_mean_kernel, dim3(nb), dim3(TPB), 0, s, x, n, part, nb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  *iters = host.iters;
  *relres = host.bb > 0 ? sqrt(host.rr / host.bb) : 0.0;
  *status = host.done;
  return hipSuccess;
}

// ------------------------------------------------------------------- AAR --
//
// Alternating Anderson-Richardson for (-Lap_h + shift) x = b (Sec. 5 solves
// the Poisson equation and applies the Kerker preconditioner with AAR): with
// the Jacobi-scaled residual f_k = (b - A x_k) / diag A and the difference
// pairs of the last m iterations,
//   x_{k+1} = x_k + omega f_k                              ((k+1) mod p != 0)
//   x_{k+1} = x_k + beta f_k - (dX + beta dF) gamma_k      ((k+1) mod p == 0)
// gamma_k from the Pulay normal equations (the mixing's kernels).  Every
// kernel of an iteration checks the device-side flag set when
// ||b - A x|| <= tol ||b||, so iterations queued past convergence do nothing.

namespace {

struct AarState {
  double rr, bb, mean;
  int done;  // 1 converged, 2 iteration limit
  int iters;
};

__global__ __launch_bounds__(TPB) void aar_mean_kernel(const double* part, int nb, long n,
                                                       int center, AarState* st) {
  __shared__ double sh[TPB / 64];
  const double s = center ? reduce_partials(part, nb, sh) : 0.0;
  if (threadIdx.x == 0) {
    st->mean = center ? s / (double)n : 0.0;
    st->done = 0;
    st->iters = 0;
  }
}

// b = scale (src - mean); partials |b|^2 into row 1
__global__ __launch_bounds__(TPB) void aar_rhs_kernel(const double* __restrict__ src, double scale,
                                                      long n, double* __restrict__ b,
                                                      double* __restrict__ part,
                                                      const AarState* st) {
  __shared__ double sh[TPB / 64];
  const double mean = st->mean;
  double s = 0.0;
  for (long e = blockIdx.x * (long)TPB + threadIdx.x; e < n; e += (long)gridDim.x * TPB) {
    const double v = scale * (src[e] - mean);
    b[e] = v;
    s += v * v;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[RB + blockIdx.x] = s;
}

__global__ __launch_bounds__(TPB) void aar_bb_kernel(const double* part, int nb, AarState* st) {
  __shared__ double sh[TPB / 64];
  const double s = reduce_partials(part + RB, nb, sh);
  if (threadIdx.x == 0) st->bb = s;
}

// f = (b - (-Lap_h + shift) x) inv_diag; with a previous iterate the pair
// dX = x - x_prev, dF = f - f_prev into its slot; partials |r|^2 into row 0
__global__ __launch_bounds__(TPB) void aar_residual_kernel(
    const double* __restrict__ x, const double* __restrict__ b, double* __restrict__ fcur,
    const double* __restrict__ prev_x, const double* __restrict__ prev_f, double* __restrict__ dx,
    double* __restrict__ df, int have_prev, Dims d, LapCoef k, double shift, double inv_diag,
    double* __restrict__ part, const AarState* st) {
  __shared__ double sh[TPB / 64];
  if (st->done) return;
  double s = 0.0;
  for (long e = blockIdx.x * (long)TPB + threadIdx.x; e < d.ng; e += (long)gridDim.x * TPB) {
    const double xe = x[e];
    const double r = b[e] - (neg_lap_at(x, e, d, k) + shift * xe);
    const double f = r * inv_diag;
    fcur[e] = f;
    if (have_prev) {
      dx[e] = xe - prev_x[e];
      df[e] = f - prev_f[e];
    }
    s += r * r;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// convergence test of iterate k (k updates done)
__global__ __launch_bounds__(TPB) void aar_check_kernel(const double* part, int nb, double tol2,
                                                        int k, int max_iter, AarState* st) {
  __shared__ double sh[TPB / 64];
  if (st->done) return;
  const double rr = reduce_partials(part, nb, sh);
  if (threadIdx.x == 0) {
    st->rr = rr;
    st->iters = k;
    if (rr <= tol2 * st->bb) st->done = 1;
    else if (k >= max_iter) st->done = 2;
  }
}

// prev_x = x, prev_f = f; x += coef f - sum_j gamma_j (dX_j + coef dF_j)
__global__ void aar_update_kernel(double* __restrict__ x, const double* __restrict__ fcur,
                                  const double* __restrict__ dx, const double* __restrict__ df,
                                  const double* __restrict__ gamma, int m, double coef, long n,
                                  double* __restrict__ prev_x, double* __restrict__ prev_f,
                                  const AarState* st) {
  if (st->done) return;
  double gm[8];
  for (int j = 0; j < 8; ++j) gm[j] = j < m ? gamma[j] : 0.0;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const double xe = x[e], f = fcur[e];
    double v = xe + coef * f;
    for (int j = 0; j < m; ++j) v -= gm[j] * (dx[(long)j * n + e] + coef * df[(long)j * n + e]);
    prev_x[e] = xe;
    prev_f[e] = f;
    x[e] = v;
  }
}

size_t aar_ws_bytes(const dk_ctx* c) {
  const size_t n = c->ngrid;
  return 4 * ws_slice(n * sizeof(double)) +
         2 * ws_slice((size_t)kPulayMaxHistory * n * sizeof(double)) +
         ws_slice((size_t)(2 + kPulayMaxHistory * kPulayMaxHistory + kPulayMaxHistory) * RB *
                  sizeof(double)) +
         ws_slice(16 * sizeof(double)) + ws_slice(sizeof(AarState));
}

size_t cg_ws_bytes(const dk_ctx* c) {
  return 3 * ws_slice(c->ngrid * sizeof(double)) + ws_slice(4 * RB * sizeof(double)) +
         ws_slice(sizeof(CgState));
}

}  // namespace

static hipError_t aar_solve(dk_ctx* c, const double* src, double* x, double tol, int max_iter,
                            void* ws, double scale, double shift, bool center, int* iters,
                            double* relres, int* status) {
  const Dims d = dims_of(c);
  const long n = d.ng;
  const int hist = c->aar_history, period = c->aar_period;
  WsCursor cur((char*)ws, aar_ws_bytes(c));
  double* b = cur.take<double>(n);
  double* fcur = cur.take<double>(n);
  double* prev_x = cur.take<double>(n);
  double* prev_f = cur.take<double>(n);
  double* dx = cur.take<double>((size_t)kPulayMaxHistory * n);
  double* df = cur.take<double>((size_t)kPulayMaxHistory * n);
  double* part =
      cur.take<double>((size_t)(2 + kPulayMaxHistory * kPulayMaxHistory + kPulayMaxHistory) * RB);
  double* res = cur.take<double>(16);
  AarState* st = cur.take<AarState>(1);
  if (!cur.ok) return hipErrorInvalidValue;
  const LapCoef k = lap_coef(d);
  const double inv_diag = 1.0 / (k.diag + shift);
  const int nb = grid_for(n);
  hipStream_t s = c->stream;
  if (center) hipLaunchKernelGGL(sum_kernel, dim3(nb), dim3(TPB), 0, s, src, n, part);
  hipLaunchKernelGGL(aar_mean_kernel, dim3(1), dim3(TPB), 0, s, part, nb, n, center ? 1 : 0, st);
  hipLaunchKernelGGL(aar_rhs_kernel, dim3(nb), dim3(TPB), 0, s, src, scale, n, b, part, st);
  hipLaunchKernelGGL(aar_bb_kernel, dim3(1), dim3(TPB), 0, s, part, nb, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  AarState host{};
  constexpr int kBatch = 32;  // iterations queued between host checks
  for (int it = 0; it <= max_iter;) {
    for (int q = 0; q < kBatch && it <= max_iter; ++q, ++it) {
      const int have_prev = it > 0 ? 1 : 0;
      const long slot = have_prev ? (it - 1) % hist : 0;
      hipLaunchKernelGGL(aar_residual_kernel, dim3(nb), dim3(TPB), 0, s, x, b, fcur, prev_x,
                         prev_f, dx + slot * n, df + slot * n, have_prev, d, k, shift, inv_diag,
                         part, st);
      hipLaunchKernelGGL(aar_check_kernel, dim3(1), dim3(TPB), 0, s, part, nb, tol * tol, it,
                         max_iter, st);
      if (it == max_iter) break;
      const int m = ((it + 1) % period == 0) ? (it < hist ? it : hist) : 0;
      if (m > 0) {
        hipLaunchKernelGGL(pulay_dots_kernel, dim3(nb, m * m + m), dim3(TPB), 0, s, df, fcur, n,
                           m, part);
        hipLaunchKernelGGL(pulay_solve_kernel, dim3(1), dim3(TPB), 0, s, part, nb, m, kPulayReg,
                           res);
      }
      hipLaunchKernelGGL(aar_update_kernel, dim3(nb), dim3(TPB), 0, s, x, fcur, dx, df, res, m,
                         m > 0 ? c->aar_beta : c->aar_omega, n, prev_x, prev_f, st);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(&host, st, sizeof host, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    if (host.done) break;
  }
  if (center) {
    hipLaunchKernelGGL(sum_kernel, dim3(nb), dim3(TPB), 0, s, x, n, part);
    hipLaunchKernelGGL(subtract_mean_kernel, dim3(nb), dim3(TPB), 0, s, x, n, part, nb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  *iters = host.iters;
  *relres = host.bb > 0 ? sqrt(host.rr / host.bb) : 0.0;
  *status = host.done ? host.done : 2;
  return hipSuccess;
}

size_t poisson_ws_bytes(const dk_ctx* c) {
  const size_t a = cg_ws_bytes(c), b = aar_ws_bytes(c);
  return a > b ? a : b;
}

// the context's linear solver for (-Lap_h + shift) x = scale (src - mean)
static hipError_t linear_solve(dk_ctx* c, const double* src, double* x, double tol, int max_iter,
                               void* ws, double scale, double shift, bool center, int* iters,
                               double* relres, int* status) {
  if (c->linear_solver == DK_SOLVER_AAR)
    return aar_solve(c, src, x, tol, max_iter, ws, scale, shift, center, iters, relres, status);
  return cg_solve(c, src, x, tol, max_iter, ws, scale, shift, center, iters, relres, status);
}

hipError_t poisson_cg(dk_ctx* c, const double* src, double* x, double tol, int max_iter,
                      void* ws, int* iters, double* relres, int* status) {
  return linear_solve(c, src, x, tol, max_iter, ws, 4.0 * M_PI, 0.0, true, iters, relres, status);
}

size_t potential_ws_bytes() { return ws_slice(4 * RB * sizeof(double)) + ws_slice(8 * sizeof(double)); }

// sums[0..4) = sum rho eps, sum rho vc, sum rho vxc, sum (rho + b) vc (unweighted)
hipError_t effective_potential(dk_ctx* c, const double* rho, const double* b, const double* vc,
                               const double* vcore, double* vxc, double* veff, void* ws,
                               double* sums) {
  WsCursor cur((char*)ws, potential_ws_bytes());
  double* part = cur.take<double>(4 * RB);
  double* out = cur.take<double>(8);
  if (!cur.ok) return hipErrorInvalidValue;
  const int nb = grid_for(c->ngrid);
  hipLaunchKernelGGL(potential_kernel, dim3(nb), dim3(TPB), 0, c->stream, rho, b, vc, vcore, vxc,
                     veff, c->ngrid, part);
  hipLaunchKernelGGL(reduce_rows_small_kernel, dim3(1), dim3(TPB), 0, c->stream, part, nb, 4, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(sums, out, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(c->stream);
}

// Pulay state: dR (history x N), dF (history x N), prev_in, prev_F, F, gamma/out (16), partials
size_t pulay_state_bytes(const dk_ctx* c, int history) {
  const size_t n = c->ngrid;
  return 2 * ws_slice((size_t)history * n * sizeof(double)) + 3 * ws_slice(n * sizeof(double)) +
         ws_slice(16 * sizeof(double)) +
         ws_slice((size_t)(2 + kPulayMaxHistory * kPulayMaxHistory + kPulayMaxHistory) * RB *
                  sizeof(double));
}

hipError_t pulay_mix(dk_ctx* c, void* state, int history, int iter, double beta,
                     const double* in, const double* out, double* next, double* residual) {
  const long n = c->ngrid;
  WsCursor cur((char*)state, pulay_state_bytes(c, history));
  double* dr = cur.take<double>((size_t)history * n);
  double* df = cur.take<double>((size_t)history * n);
  double* prev_in = cur.take<double>(n);
  double* prev_f = cur.take<double>(n);
  double* fcur = cur.take<double>(n);
  double* res = cur.take<double>(16);
  double* part = cur.take<double>((size_t)(2 + kPulayMaxHistory * kPulayMaxHistory + kPulayMaxHistory) * RB);
  if (!cur.ok) return hipErrorInvalidValue;
  const int have_prev = iter > 0 ? 1 : 0;
  const int slot = have_prev ? (iter - 1) % history : 0;
  const int m = iter < history ? iter : history;
  const int nb = grid_for(n);
  hipStream_t s = c->stream;
  hipLaunchKernelGGL(pulay_prepare_kernel, dim3(nb), dim3(TPB), 0, s, in, out, prev_in, prev_f,
                     fcur, dr + (long)slot * n, df + (long)slot * n, n, have_prev, part);
  if (m > 0)
    hipLaunchKernelGGL(pulay_dots_kernel, dim3(nb, m * m + m), dim3(TPB), 0, s, df, fcur, n, m,
                       part);
  hipLaunchKernelGGL(pulay_solve_kernel, dim3(1), dim3(TPB), 0, s, part, nb, m, kPulayReg, res);
  hipLaunchKernelGGL(pulay_combine_kernel, dim3(nb), dim3(TPB), 0, s, in, fcur, dr, df, res, m,
                     beta, n, next, prev_in, prev_f);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(residual, res + 8, sizeof(double), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

// Kerker-preconditioned periodic Pulay state: the Pulay state, then F_bar,
// the right-hand side -Lap_h F_bar and the CG workspace of the Kerker solve
size_t kerker_pulay_state_bytes(const dk_ctx* c, int history) {
  return pulay_state_bytes(c, history) + 2 * ws_slice(c->ngrid * sizeof(double)) +
         ws_slice(c->ngrid * sizeof(double)) + ws_slice(poisson_ws_bytes(c));
}

hipError_t kerker_pulay_mix(dk_ctx* c, void* state, int history, int iter, int period,
                            int restart, double beta, double k0, double tol, int max_iter,
                            const double* in, const double* out, double* next, double* residual,
                            int* cg_iters, int* cg_status) {
  const long n = c->ngrid;
  WsCursor cur((char*)state, kerker_pulay_state_bytes(c, history));
  double* dr = cur.take<double>((size_t)history * n);
  double* df = cur.take<double>((size_t)history * n);
  double* prev_in = cur.take<double>(n);
  double* prev_f = cur.take<double>(n);
  double* fcur = cur.take<double>(n);
  double* res = cur.take<double>(16);
  double* part = cur.take<double>((size_t)(2 + kPulayMaxHistory * kPulayMaxHistory + kPulayMaxHistory) * RB);
  double* fbar = cur.take<double>(n);
  double* z = cur.take<double>(n);
  double* rhs = cur.take<double>(n);
  void* cgws = cur.take<char>(poisson_ws_bytes(c));
  if (!cur.ok) return hipErrorInvalidValue;
  const int have_prev = iter > 0 ? 1 : 0;
  int slot, m;
  if (restart) {
    // the pairs since the last extrapolation (which discarded the others) fill
    // slots 0, 1, ...: the pair of call iter goes to iter - base, base = 1
    // before the first extrapolation, else the first call after the last one
    const int done = iter / period;
    const int base = done == 0 ? 1 : done * period;
    slot = have_prev ? iter - base : 0;
    m = (have_prev && (iter + 1) % period == 0) ? slot + 1 : 0;
  } else {
    slot = have_prev ? (iter - 1) % history : 0;
    const int m_hist = iter < history ? iter : history;
    // the extrapolation runs on every period-th call (calls counted from 1)
    m = ((iter + 1) % period == 0) ? m_hist : 0;
  }
  const int nb = grid_for(n);
  hipStream_t s = c->stream;
  hipLaunchKernelGGL(pulay_prepare_kernel, dim3(nb), dim3(TPB), 0, s, in, out, prev_in, prev_f,
                     fcur, dr + (long)slot * n, df + (long)slot * n, n, have_prev, part);
  if (m > 0)
    hipLaunchKernelGGL(pulay_dots_kernel, dim3(nb, m * m + m), dim3(TPB), 0, s, df, fcur, n, m,
                       part);
  hipLaunchKernelGGL(pulay_solve_kernel, dim3(1), dim3(TPB), 0, s, part, nb, m, kPulayReg, res);
  hipLaunchKernelGGL(pulay_bar_kernel, dim3(nb), dim3(TPB), 0, s, in, fcur, dr, df, res, m, n,
                     next, fbar, prev_in, prev_f);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  *cg_iters = 0;
  *cg_status = 1;
  const double* pz = fbar;
  if (k0 > 0.0) {
    // z = (-Lap_h + k0^2)^{-1} (-Lap_h F_bar), from z = 0
    const Dims d = dims_of(c);
    hipLaunchKernelGGL(neg_lap_kernel, dim3(nb), dim3(TPB), 0, s, fbar, rhs, d, lap_coef(d));
    hipLaunchKernelGGL(fill_kernel, dim3(nb), dim3(TPB), 0, s, z, 0.0, n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    double relres = 0.0;
    e = linear_solve(c, rhs, z, tol, max_iter, cgws, 1.0, k0 * k0, false, cg_iters, &relres,
                     cg_status);
    if (e != hipSuccess) return e;
    pz = z;
  }
  hipLaunchKernelGGL(axpy_kernel, dim3(nb), dim3(TPB), 0, s, beta, pz, next, n);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  e = hipMemcpyAsync(residual, res + 8, sizeof(double), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

}  // namespace dk
