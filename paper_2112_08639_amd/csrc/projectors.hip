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

}  // namespace

int model_functions(int n_channels, const int* l) {
  int f = 0;
  for (int c = 0; c < n_channels; ++c) f += (l[c] == 0) ? 1 : 3;
  return f;
}

// Fills chi64 (and chi32 if present), the masks and the per-projector norms
// (host) for the atoms at pos_dev.  Tables must already be allocated for
// n_atoms * model_functions projectors.
hipError_t build_projector_tables(dk_ctx* c, const double* pos_dev, int n_atoms, int n_channels,
                                  const int* l, const double* rc, double cutoff_rel,
                                  double* norms_dev) {
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

}  // namespace dk
