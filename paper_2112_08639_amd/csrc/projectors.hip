// Projector tables built on the device from atom positions (the
// Kleinman-Bylander projectors of Eq. nonlocaloperator, periodically extended),
// so that a molecular-dynamics step re-places them without host work.
//
// Channel c of atom a: radial Gaussian A_l exp(-r^2 / rc^2) times 1 (l = 0)
// or the Cartesian component x, y, z of r (l = 1, three functions), with
// A_0 = (2 / (pi rc^2))^(3/4), A_1 = 2 A_0 / rc (unit continuum norm).  Every
// periodic image whose distance is at most rc sqrt(ln(1 / cutoff_rel)) from
// the point contributes, the candidate images of each axis being the integer
// indices i in [ceil((R - rcut)/h), floor((R + rcut)/h)] that map to the
// point.  Table layout as dk_set_projectors builds it: dense column-major
// N_grid x n_proj, atom-major, channels in order, l = 1 as x, y, z.
#include <algorithm>
#include <cmath>

#include "ctx.h"

namespace dk {

namespace {

struct Channel {
  int l;
  double rc, rc2, rcut, norm;
};

constexpr int kMaxChannels = 4;

struct ChannelSet {
  Channel ch[kMaxChannels];
  int n;
  int per_atom;  // functions per atom
};

// one thread per (grid point, atom)
__global__ void build_tables_kernel(const double* __restrict__ pos, int n_atoms, ChannelSet cs,
                                    int nx, int ny, int nz, double hx, double hy, double hz,
                                    double* __restrict__ chi) {
  const long ng = (long)nx * ny * nz;
  const long total = ng * n_atoms;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const long x = e % ng;
    const int a = (int)(e / ng);
    const int w[3] = {(int)(x % nx), (int)((x / nx) % ny), (int)(x / ((long)nx * ny))};
    const int n[3] = {nx, ny, nz};
    const double h[3] = {hx, hy, hz};
    const double R[3] = {pos[3 * a], pos[3 * a + 1], pos[3 * a + 2]};
    int col = a * cs.per_atom;
    for (int c = 0; c < cs.n; ++c) {
      const Channel C = cs.ch[c];
      // image ranges per axis: i = w + k n within [lo, hi]
      int k0[3], k1[3];
      for (int ax = 0; ax < 3; ++ax) {
        const int lo = (int)ceil((R[ax] - C.rcut) / h[ax]);
        const int hi = (int)floor((R[ax] + C.rcut) / h[ax]);
        k0[ax] = (int)ceil((double)(lo - w[ax]) / n[ax]);
        k1[ax] = (int)floor((double)(hi - w[ax]) / n[ax]);
      }
      double s0 = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
      for (int kz = k0[2]; kz <= k1[2]; ++kz) {
        const double dz = (double)(w[2] + kz * nz) * hz - R[2];
        for (int ky = k0[1]; ky <= k1[1]; ++ky) {
          const double dy = (double)(w[1] + ky * ny) * hy - R[1];
          for (int kx = k0[0]; kx <= k1[0]; ++kx) {
            const double dx = (double)(w[0] + kx * nx) * hx - R[0];
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 > C.rcut * C.rcut) continue;
            const double g = C.norm * exp(-r2 / C.rc2);
            s0 += g;
            sx += g * dx;
            sy += g * dy;
            sz += g * dz;
          }
        }
      }
      if (C.l == 0) {
        chi[x + (long)col * ng] = s0;
        col += 1;
      } else {
        chi[x + (long)col * ng] = sx;
        chi[x + (long)(col + 1) * ng] = sy;
        chi[x + (long)(col + 2) * ng] = sz;
        col += 3;
      }
    }
  }
}

// mask_t[(p/64) gblocks + gb] = 1 if any entry of projector p in the 64-point
// block gb is nonzero (every writer stores 1); one wave per (projector,
// block), lane i reading point 64 gb + i
__global__ __launch_bounds__(256) void table_masks_kernel(const double* __restrict__ chi, long ng,
                                                          int n_proj, long gblocks,
                                                          uint8_t* __restrict__ mask_t) {
  const int lane = threadIdx.x & 63;
  const long total = gblocks * n_proj;
  const long stride = ((long)gridDim.x * blockDim.x) >> 6;
  for (long e = (blockIdx.x * (long)blockDim.x + threadIdx.x) >> 6; e < total; e += stride) {
    const long gb = e % gblocks;
    const int p = (int)(e / gblocks);
    const long x = gb * 64 + lane;
    const bool nz = x < ng && chi[(long)p * ng + x] != 0.0;
    if (__any(nz) && lane == 0) mask_t[(long)(p / 64) * gblocks + gb] = 1;
  }
}

// norms[p] = sum_x chi_p(x)^2, one block per projector
__global__ __launch_bounds__(256) void table_norms_kernel(const double* __restrict__ chi, long ng,
                                                          double* __restrict__ norms) {
  __shared__ double sh[4];
  const double* col = chi + (long)blockIdx.x * ng;
  double s = 0.0;
  for (long x = threadIdx.x; x < ng; x += 256) s += col[x] * col[x];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) norms[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ void table_f32_kernel(const double* __restrict__ s, float* __restrict__ d, long n) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    d[e] = (float)s[e];
}

inline int blocks_for(long n) {
  long b = (n + 255) / 256;
  return (int)(b > 16384 ? 16384 : (b < 1 ? 1 : b));
}

// Grid points an atom's projectors can reach along one axis: indices lo ..
// lo + len - 1 (taken modulo n), the whole axis when the cutoff sphere is as
// wide as the cell.
struct AxisBox {
  int lo, len;
};
__host__ __device__ inline AxisBox axis_box(double r, double rcut, double h, int n) {
  const int lo = (int)ceil((r - rcut) / h), hi = (int)floor((r + rcut) / h);
  AxisBox b{lo, hi - lo + 1};
  if (b.len >= n) b = AxisBox{0, n};
  if (b.len < 0) b.len = 0;
  return b;
}

// Twelfth-order central first-difference weights a_k = (-1)^{k+1}(6!)^2/(k(6-k)!(6+k)!).
__constant__ double kFdA[7] = {0.0, 6.0 / 7.0, -15.0 / 56.0, 5.0 / 63.0, -1.0 / 56.0, 1.0 / 385.0,
                               -1.0 / 5544.0};

// Nonlocal stress contraction of one atom's projectors with a field z_p:
//   part[blockIdx][3a + b] = sum over the block's points x of
//       sum_{p of the atom} gamma_p m^b_p(x) (d_a z_p)(x),
// m^b_p the first moment of projector p (the sum over periodic images of
// chi_p(x - R - L)(x - R - L)_b, evaluated here from the model), d_a the
// twelfth-order first difference without the 1/h factor (applied per axis
// by the caller through ih).  Block b covers chunk b % chunks of the box of
// atom b / chunks; z is N_grid x n_proj FP64 (ld = N_grid).
__global__ __launch_bounds__(256) void moment_stress_kernel(const double* __restrict__ pos,
                                                            ChannelSet cs, double rcut_max,
                                                            const double* __restrict__ gamma,
                                                            const double* __restrict__ z, int nx,
                                                            int ny, int nz, double hx, double hy,
                                                            double hz, int chunks,
                                                            double* __restrict__ part) {
  __shared__ double red[4][9];
  const int atom = blockIdx.x / chunks, chunk = blockIdx.x % chunks;
  const long ng = (long)nx * ny * nz;
  const int n[3] = {nx, ny, nz};
  const double h[3] = {hx, hy, hz};
  const double ih[3] = {1.0 / hx, 1.0 / hy, 1.0 / hz};
  const double R[3] = {pos[3 * atom], pos[3 * atom + 1], pos[3 * atom + 2]};
  AxisBox bx[3];
  for (int ax = 0; ax < 3; ++ax) bx[ax] = axis_box(R[ax], rcut_max, h[ax], n[ax]);
  const long nbox = (long)bx[0].len * bx[1].len * bx[2].len;
  double acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = 0.0;
  for (long t = (long)chunk * 256 + threadIdx.x; t < nbox; t += (long)chunks * 256) {
    const int i[3] = {(int)(t % bx[0].len), (int)((t / bx[0].len) % bx[1].len),
                      (int)(t / ((long)bx[0].len * bx[1].len))};
    int w[3];
    for (int ax = 0; ax < 3; ++ax) w[ax] = ((bx[ax].lo + i[ax]) % n[ax] + n[ax]) % n[ax];
    const long x = w[0] + (long)nx * (w[1] + (long)ny * w[2]);
    int col = atom * cs.per_atom;
    for (int c = 0; c < cs.n; ++c) {
      const Channel C = cs.ch[c];
      const int nf = (C.l == 0) ? 1 : 3;
      int k0[3], k1[3];
      for (int ax = 0; ax < 3; ++ax) {
        const int lo = (int)ceil((R[ax] - C.rcut) / h[ax]);
        const int hi = (int)floor((R[ax] + C.rcut) / h[ax]);
        k0[ax] = (int)ceil((double)(lo - w[ax]) / n[ax]);
        k1[ax] = (int)floor((double)(hi - w[ax]) / n[ax]);
      }
      // s1[b] = sum g d_b (l = 0 moments), s2[m][b] = sum g d_m d_b (l = 1)
      double s1[3] = {0, 0, 0}, s2[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
      bool any = false;
      for (int kz = k0[2]; kz <= k1[2]; ++kz) {
        const double dz = (double)(w[2] + kz * nz) * hz - R[2];
        for (int ky = k0[1]; ky <= k1[1]; ++ky) {
          const double dy = (double)(w[1] + ky * ny) * hy - R[1];
          for (int kx = k0[0]; kx <= k1[0]; ++kx) {
            const double dx = (double)(w[0] + kx * nx) * hx - R[0];
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 > C.rcut * C.rcut) continue;
            any = true;
            const double g = C.norm * exp(-r2 / C.rc2);
            const double d[3] = {dx, dy, dz};
            for (int b = 0; b < 3; ++b) {
              s1[b] += g * d[b];
              for (int m = 0; m < 3; ++m) s2[m][b] += g * d[m] * d[b];
            }
          }
        }
      }
      if (any) {
        for (int f = 0; f < nf; ++f) {
          const int p = col + f;
          const double* zp = z + (long)p * ng;
          double grad[3] = {0, 0, 0};
          for (int k = 1; k <= 6; ++k) {
            const int xp = (w[0] + k) % nx, xm = (w[0] - k + 8 * nx) % nx;
            const int yp = (w[1] + k) % ny, ym = (w[1] - k + 8 * ny) % ny;
            const int zp_ = (w[2] + k) % nz, zm = (w[2] - k + 8 * nz) % nz;
            const long row = (long)nx * (w[1] + (long)ny * w[2]);
            grad[0] += kFdA[k] * (zp[xp + row] - zp[xm + row]);
            grad[1] += kFdA[k] * (zp[w[0] + (long)nx * (yp + (long)ny * w[2])] -
                                  zp[w[0] + (long)nx * (ym + (long)ny * w[2])]);
            grad[2] += kFdA[k] * (zp[w[0] + (long)nx * (w[1] + (long)ny * zp_)] -
                                  zp[w[0] + (long)nx * (w[1] + (long)ny * zm)]);
          }
          const double gp = gamma[p];
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
              const double mb = (C.l == 0) ? s1[b] : s2[f][b];
              acc[3 * a + b] += gp * mb * grad[a] * ih[a];
            }
        }
      }
      col += nf;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    double v = acc[k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) red[wave][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < 9)
    part[(long)blockIdx.x * 9 + threadIdx.x] =
        (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

}  // namespace

int model_functions(int n_channels, const int* l) {
  int f = 0;
  for (int c = 0; c < n_channels; ++c) f += (l[c] == 0) ? 1 : 3;
  return f;
}

// Fills chi64 (and chi32 if present), the masks and the per-projector norms
// (host) for the atoms at pos_dev.  Tables must already be allocated for
// n_atoms * model_functions projectors.
static ChannelSet channel_set(int n_channels, const int* l, const double* rc, double cutoff_rel) {
  ChannelSet cs{};
  cs.n = n_channels;
  cs.per_atom = model_functions(n_channels, l);
  const double cut = std::sqrt(std::log(1.0 / cutoff_rel));
  for (int k = 0; k < n_channels; ++k) {
    Channel& C = cs.ch[k];
    C.l = l[k];
    C.rc = rc[k];
    C.rc2 = rc[k] * rc[k];
    C.rcut = rc[k] * cut;
    const double a0 = std::pow(2.0 / (M_PI * rc[k] * rc[k]), 0.75);
    C.norm = (l[k] == 0) ? a0 : a0 * 2.0 / rc[k];
  }
  return cs;
}

hipError_t build_projector_tables(dk_ctx* c, const double* pos_dev, int n_atoms, int n_channels,
                                  const int* l, const double* rc, double cutoff_rel,
                                  double* norms_dev) {
  const ChannelSet cs = channel_set(n_channels, l, rc, cutoff_rel);
  const long ng = c->ngrid;
  hipLaunchKernelGGL(build_tables_kernel, dim3(blocks_for(ng * n_atoms)), dim3(256), 0, c->stream,
                     pos_dev, n_atoms, cs, c->nx, c->ny, c->nz, c->hx, c->hy, c->hz, c->chi64);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int n_proj = n_atoms * cs.per_atom;
  const long gblocks = (ng + 63) / 64;
  const int ptiles = (n_proj + 63) / 64;
  if ((e = hipMemsetAsync(c->mask_t, 0, (size_t)ptiles * gblocks, c->stream)) != hipSuccess) return e;
  hipLaunchKernelGGL(table_masks_kernel, dim3(blocks_for(gblocks * n_proj * 64)), dim3(256), 0,
                     c->stream, c->chi64, ng, n_proj, gblocks, c->mask_t);
  hipLaunchKernelGGL(table_norms_kernel, dim3(n_proj), dim3(256), 0, c->stream, c->chi64, ng,
                     norms_dev);
  if (c->chi32)
    hipLaunchKernelGGL(table_f32_kernel, dim3(blocks_for(ng * n_proj)), dim3(256), 0, c->stream,
                       c->chi64, c->chi32, ng * n_proj);
  return hipGetLastError();
}

// Work split of projector_moment_stress: chunks per atom box, so that the
// grid has enough blocks and each thread some dozens of points.
static int moment_stress_chunks(const dk_ctx* c, double rcut_max) {
  const double h[3] = {c->hx, c->hy, c->hz};
  const int n[3] = {c->nx, c->ny, c->nz};
  long nbox = 1;
  for (int ax = 0; ax < 3; ++ax) {
    long len = (long)(2.0 * rcut_max / h[ax]) + 2;
    if (len > n[ax]) len = n[ax];
    nbox *= len;
  }
  const int na = c->n_atoms > 0 ? c->n_atoms : 1;
  long chunks = (nbox + 8191) / 8192;
  const long fill = (1024 + na - 1) / na;
  if (chunks < fill) chunks = fill;
  const long most = (nbox + 255) / 256;
  if (chunks > most) chunks = most;
  if (chunks < 1) chunks = 1;
  return (int)chunks;
}

static double model_rcut_max(const dk_ctx* c) {
  const double cut = std::sqrt(std::log(1.0 / c->model_cutoff_rel));
  double r = 0.0;
  for (int k = 0; k < c->model_channels; ++k) r = std::max(r, c->model_rc[k] * cut);
  return r;
}

int projector_moment_stress_parts(const dk_ctx* c) {
  if (c->model_channels == 0 || c->n_atoms == 0) return 0;
  return c->n_atoms * moment_stress_chunks(c, model_rcut_max(c));
}

hipError_t projector_moment_stress(dk_ctx* c, const double* z, double* part, int n_part_max,
                                   int* n_part) {
  *n_part = 0;
  if (c->model_channels == 0 || c->n_atoms == 0 || c->n_proj == 0) return hipSuccess;
  const ChannelSet cs = channel_set(c->model_channels, c->model_l, c->model_rc, c->model_cutoff_rel);
  const double rmax = model_rcut_max(c);
  const int chunks = moment_stress_chunks(c, rmax);
  const long blocks = (long)c->n_atoms * chunks;
  if (blocks > n_part_max) return hipErrorInvalidValue;
  const double* pos_dev = c->proj_aux;  // positions lead the auxiliary buffer
  hipLaunchKernelGGL(moment_stress_kernel, dim3((unsigned)blocks), dim3(256), 0, c->stream, pos_dev,
                     cs, rmax, c->gamma_dev, z, c->nx, c->ny, c->nz, c->hx, c->hy, c->hz, chunks,
                     part);
  *n_part = (int)blocks;
  return hipGetLastError();
}

}  // namespace dk
