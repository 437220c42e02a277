// Density and Hellmann-Feynman forces from the orbitals and the density kernel.
//
// Density (Eqs. phi_tilde, density:NewForm):  rho(x) = 2 sum_i (X D)_{x i} X_{x i}.
// One MFMA product X D whose epilogue multiplies each output tile by the
// matching tile of X and sums over the tile's columns; Phi~ = X D is never
// stored.  Per-tile partial sums are added in FP64 in a second pass.  The
// mixed path forms X D in the three-piece split-BF16 form (six products,
// ~2^-24 per product): with two pieces (~2^-16) the density carries a noise of
// ~2e-6 relative, above a 1e-6 SCF tolerance on rho; three pieces remove that
// floor at ~10% more time for this product.
//
// Nonlocal force (Eq. force_nl:NewForm):
//   f_I = -4 sum_{p in I} gamma_p sum_i (h^3 chi_p^T x_i)(h^3 chi_p^T grad_h phi~_i).
// With phi~ = X D and grad_h antisymmetric on the periodic grid,
//   h^3 chi_p^T grad_h phi~_i = (G D)_{p i},  G = -h^3 (grad_h chi)^T X,
// so the gradient falls on the (fixed) projector tables, and
//   f_{I,a} = -4 sum_{p in I} gamma_p sum_i C_{p i} (G_a D)_{p i},  C = h^3 chi^T X.
// Local force of the fixed-potential problem: f_I += h^3 sum_x rho(x) grad v_I(x).
#include <mutex>

#include "ctx.h"
#include "gemm.h"

namespace dk {

// Scratch of dk_density_noalloc: what density() takes from a workspace (the
// per-tile row partials of the density product, and in the mixed path the bf16
// pieces of D; density_ws_bytes) for callers that cannot allocate.
// Every GPU the library runs on holds its own copy until the process ends.
// In host code `scratch` names a host-side stand-in: only the device address
// taken by hipGetSymbolAddress (density_scratch_init) may reach a kernel.
static __device__ __align__(256) double scratch[kDensityScratchBytes / sizeof(double)];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

__global__ void rho_reduce_kernel(const double* __restrict__ part, int ntiles, long m,
                                  double* __restrict__ rho) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < m;
       e += (long)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int t = 0; t < ntiles; ++t) s += part[(long)t * m + e];
    rho[e] = 2.0 * s;
  }
}

// per (projector p, direction a): f_pa = -4 gamma_p sum_i E[p, i] G_a[p, i], with
// G_a = -W[np(1+a) + p, i] (W holds h^3 (grad_a chi)^T X); then summed per atom
__global__ void nl_force_kernel(const double* __restrict__ E, const double* __restrict__ W,
                                int n_proj, int n_s, const double* __restrict__ gamma,
                                double* __restrict__ per_proj) {
  __shared__ double sh[4];
  const int p = blockIdx.x, a = blockIdx.y;
  const long ldw = 4L * n_proj;
  const double* g = W + (long)(a + 1) * n_proj;
  double s = 0.0;
  for (int i = threadIdx.x; i < n_s; i += 256) s += E[p + (long)i * n_proj] * g[p + (long)i * ldw];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) per_proj[p + (long)a * n_proj] = 4.0 * gamma[p] * (sh[0] + sh[1] + sh[2] + sh[3]);
}

__global__ void local_force_kernel(const double* __restrict__ rho, const double* __restrict__ gradv,
                                   long ngrid, double dv, double* __restrict__ out) {
  __shared__ double sh[4];
  const long row = blockIdx.x;  // atom*3 + direction
  const double* g = gradv + row * ngrid;
  double s = 0.0;
  for (long x = threadIdx.x; x < ngrid; x += 256) s += rho[x] * g[x];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[row] = dv * (sh[0] + sh[1] + sh[2] + sh[3]);
}

__global__ void gather_atoms_kernel(const double* __restrict__ per_proj, const int* __restrict__ atom,
                                    int n_proj, const double* __restrict__ local, int n_atoms,
                                    double* __restrict__ f) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 3 * n_atoms) return;
  const int i = e / 3, a = e % 3;
  double s = local ? local[e] : 0.0;
  for (int p = 0; p < n_proj; ++p)
    if (atom[p] == i) s += per_proj[p + (long)a * n_proj];
  f[e] = s;
}

inline int grid_for(long n) {
  long b = (n + 255) / 256;
  return (int)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

}  // namespace

hipError_t density_scratch_init(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

void* density_scratch(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

// Row partials of the X D product, one per n tile (64 columns FP64, 128 mixed),
// and in the mixed path the bf16 pieces of D.
size_t density_ws_bytes(const dk_ctx* c, int n_s) {
  if (c->precision == DK_PREC_FP64)
    return ws_slice((size_t)ceil_div(n_s, 64) * c->ngrid * sizeof(double));
  return ws_slice((size_t)ceil_div(n_s, 128) * c->ngrid * sizeof(double)) +
         split_planes_bytes(n_s, n_s, 3);
}

hipError_t density(dk_ctx* c, const void* x, long ld, int n_s, const double* ds, double* rho,
                   void* ws) {
  GemmArgs g;
  g.M = (int)c->ngrid;
  g.N = n_s;
  g.K = n_s;
  g.A = x;
  g.lda = ld;
  g.B = ds;
  g.ldb = n_s;
  g.rowpart = (double*)ws;
  g.R = x;
  g.ldr = ld;
  g.n_fastest = 1;  // a tile's 64 block rows are shared by its n tiles
  hipError_t e;
  // row partials: one per n tile (64 columns FP64, 128 mixed)
  int n_parts;
  if (c->precision == DK_PREC_FP64) {
    e = launch_gemm<kF64, double, double, false, true, kRowSum, double>(g, c->stream);
    n_parts = ceil_div(n_s, 64);
  } else {
    // D split beforehand into its bf16 pieces, after the row partials
    n_parts = ceil_div(n_s, 128);
    void* planes = (char*)ws + ws_slice((size_t)n_parts * c->ngrid * sizeof(double));
    e = split_planes(c, ds, 1, n_s, n_s, n_s, 3, planes);
    if (e != hipSuccess) return e;
    g.B = planes;
    g.ldb = split_planes_ld(n_s);
    g.b_plane = (long)n_s * g.ldb;
    e = launch_gemm<kBF16X6S, float, __bf16, false, true, kRowSum, float, 128, 128, 32>(g, c->stream);
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(rho_reduce_kernel, dim3(grid_for(c->ngrid)), dim3(256), 0, c->stream,
                     (const double*)ws, n_parts, c->ngrid, rho);
  return hipGetLastError();
}

size_t forces_ws_bytes(const dk_ctx* c, int n_s, int n_atoms) {
  const size_t pn = (size_t)c->n_proj * n_s;
  return ws_slice(4 * pn * sizeof(double)) + ws_slice(pn * sizeof(double)) +
         ws_slice(3 * (size_t)(c->n_proj > 0 ? c->n_proj : 1) * sizeof(double)) +
         2 * ws_slice((3 * (size_t)n_atoms + 8) * sizeof(double)) +
         ws_slice(projector_integrals_ws_bytes(c, n_s, 4 * c->n_proj));
}

hipError_t forces(dk_ctx* c, const void* x, long ld, int n_s, const double* ds,
                  const double* rho, const double* gradv, int n_atoms, double* f_host, void* ws) {
  WsCursor cur((char*)ws, forces_ws_bytes(c, n_s, n_atoms));
  const size_t pn = (size_t)c->n_proj * n_s;
  const int np = c->n_proj, m4 = 4 * c->n_proj;
  // W (4 n_proj x n_s) = h^3 [chi | grad_x chi | grad_y chi | grad_z chi]^T X:
  // rows 0..np-1 are C, rows np(1+a).. are -G_a
  double* W = cur.take<double>(4 * pn);
  double* E = cur.take<double>(pn);
  double* per_proj = cur.take<double>(3 * (size_t)(np > 0 ? np : 1));
  double* local = cur.take<double>(3 * (size_t)n_atoms + 8);
  double* fdev = cur.take<double>(3 * (size_t)n_atoms + 8);
  void* pws = cur.take<char>(projector_integrals_ws_bytes(c, n_s, m4));
  if (!cur.ok) return hipErrorInvalidValue;
  hipError_t e;
  if (np > 0) {
    e = projector_integrals(c, x, ld, n_s, c->chi64, m4, c->dv, W, pws);
    if (e != hipSuccess) return e;
    // E = C D  (n_proj x n_s; C = rows 0..np-1 of W, leading dimension 4 np)
    GemmArgs g;
    g.M = np; g.N = n_s; g.K = n_s;
    g.A = W; g.lda = m4;
    g.B = ds; g.ldb = n_s;
    g.C = E; g.ldc = np;
    e = launch_gemm<kF64, double, double, false, true, kStore, double>(g, c->stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(nl_force_kernel, dim3(np, 3), dim3(256), 0, c->stream, E, W, np, n_s,
                       c->gamma_dev, per_proj);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (gradv) {
    hipLaunchKernelGGL(local_force_kernel, dim3(3 * n_atoms), dim3(256), 0, c->stream, rho, gradv,
                       c->ngrid, c->dv, local);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(gather_atoms_kernel, dim3(ceil_div(3 * n_atoms, 256)), dim3(256), 0,
                     c->stream, per_proj, c->atom_dev, c->n_proj, gradv ? local : nullptr, n_atoms,
                     fdev);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  e = hipMemcpyAsync(f_host, fdev, 3 * (size_t)n_atoms * sizeof(double), hipMemcpyDeviceToHost,
                     c->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(c->stream);
}

}  // namespace dk
