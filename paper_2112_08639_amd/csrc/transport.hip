// Green-Kubo transport coefficients from molecular-dynamics series (Sec. 5,
// high-temperature QMD): the self-diffusion coefficient and the shear
// viscosity are time integrals of the velocity and stress autocorrelation
// functions.
//
//   C(k) = sum_c sum_{t0 < T-k} s_c(t0 + k) s_c(t0) / (n_comp (T - k))
//
// over the time origins of one run (the ensemble average of a stationary
// run), averaged over the components; I(k) = scale * trapezoid integral of C
// from 0 to k dt.  For the 3N velocity components C is the VACF / 3 and I with
// scale 1 is D(t); for the five deviatoric stress components C is the SACF and
// I with scale |Omega| / k_B T is eta(t).
#include "ctx.h"

namespace dk {

namespace {

// one workgroup per lag k: the products s[e + k n] s[e] over the flat index
// e = t0 n + c < (T - k) n, coalesced, summed in FP64
__global__ __launch_bounds__(256) void time_corr_kernel(const double* __restrict__ s, long n_steps,
                                                        int n_comp, double* __restrict__ corr) {
  __shared__ double sh[4];
  const long k = blockIdx.x;
  const long m = (n_steps - k) * n_comp;
  const double* __restrict__ sk = s + k * n_comp;
  double a0 = 0.0, a1 = 0.0;
  long e = threadIdx.x;
  for (; e + 256 < m; e += 512) {
    a0 += sk[e] * s[e];
    a1 += sk[e + 256] * s[e + 256];
  }
  if (e < m) a0 += sk[e] * s[e];
  double v = a0 + a1;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0)
    corr[k] = ((sh[0] + sh[1]) + (sh[2] + sh[3])) / ((double)n_comp * (double)(n_steps - k));
}

// I(0) = 0, I(k) = I(k-1) + scale dt (C(k-1) + C(k)) / 2: one lane, in order
__global__ void trapezoid_kernel(const double* __restrict__ corr, int n, double dt, double scale,
                                 double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double acc = 0.0;
  out[0] = 0.0;
  for (int k = 1; k < n; ++k) {
    acc += 0.5 * dt * (corr[k - 1] + corr[k]);
    out[k] = scale * acc;
  }
}

// per step t: sigma_t (row-major 3 x 3) minus the ions' momentum flux
// sum_I M v_Ia v_Ib / |Omega| (if v is given), then the five deviatoric
// components s_12, s_23, s_31, (s_11 - s_22)/2, (s_22 - s_33)/2.  One wave per
// step; lanes split the atoms for the flux.
__global__ __launch_bounds__(256) void deviatoric_kernel(const double* __restrict__ sigma,
                                                         const double* __restrict__ v,
                                                         int n_atoms, double mass_over_vol,
                                                         long n_steps, double* __restrict__ out) {
  const long t = (blockIdx.x * (long)blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (t >= n_steps) return;
  double f[6] = {0, 0, 0, 0, 0, 0};  // xx, yy, zz, xy, yz, zx
  if (v) {
    const double* vt = v + t * 3L * n_atoms;
    for (int i = lane; i < n_atoms; i += 64) {
      const double x = vt[3 * i], y = vt[3 * i + 1], z = vt[3 * i + 2];
      f[0] += x * x; f[1] += y * y; f[2] += z * z;
      f[3] += x * y; f[4] += y * z; f[5] += z * x;
    }
#pragma unroll
    for (int q = 0; q < 6; ++q)
      for (int o = 32; o > 0; o >>= 1) f[q] += __shfl_xor(f[q], o);
  }
  if (lane == 0) {
    const double* s = sigma + 9 * t;
    const double s11 = s[0] - mass_over_vol * f[0], s22 = s[4] - mass_over_vol * f[1];
    const double s33 = s[8] - mass_over_vol * f[2];
    const double s12 = s[1] - mass_over_vol * f[3];
    const double s23 = s[5] - mass_over_vol * f[4];
    const double s31 = s[6] - mass_over_vol * f[5];
    double* o = out + 5 * t;
    o[0] = s12;
    o[1] = s23;
    o[2] = s31;
    o[3] = 0.5 * (s11 - s22);
    o[4] = 0.5 * (s22 - s33);
  }
}

}  // namespace

hipError_t time_correlation(dk_ctx* c, const double* series, long n_steps, int n_comp, int max_lag,
                            double dt, double scale, double* corr, double* integral) {
  hipLaunchKernelGGL(time_corr_kernel, dim3(max_lag), dim3(256), 0, c->stream, series, n_steps,
                     n_comp, corr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !integral) return e;
  hipLaunchKernelGGL(trapezoid_kernel, dim3(1), dim3(64), 0, c->stream, corr, max_lag, dt, scale,
                     integral);
  return hipGetLastError();
}

hipError_t deviatoric_stress(dk_ctx* c, const double* sigma, const double* v, int n_atoms,
                             double mass, long n_steps, double* out) {
  const double vol = c->lx * c->ly * c->lz;
  const long blocks = (n_steps * 64 + 255) / 256;
  hipLaunchKernelGGL(deviatoric_kernel, dim3((unsigned)blocks), dim3(256), 0, c->stream, sigma, v,
                     n_atoms, mass / vol, n_steps, out);
  return hipGetLastError();
}

}  // namespace dk
