// Learned start density: descriptors, the per-point MLP (forward, loss
// gradient by backpropagation), Adam, and the predicted density.
//
//   descriptors  d_k(x) = sum_J sum_L exp(-|x - R_J - L|^2 / (2 w_k^2))  (per-axis
//                factor tables, as for the pseudocharges)
//   network      a_0 = (d - mean) * inv_std, a_l = SiLU(W_l a_{l-1} + b_l),
//                z = W_out a_L + b_out, y = softplus(z)
//   loss         mean_p (y_p - t_p)^2
//   Adam         m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
//                theta <- theta - lr mhat / (sqrt(vhat) + eps)
//
// Layouts: activations are feature-fastest (a[f + p * F]); parameters one FP32
// vector, per layer W (n_out x n_in, row-major) then b.  Every layer product
// is an MFMA GEMM: BF16 operands with FP32 accumulation (the weights are the
// BF16 rounding of the FP32 master copy), or FP32 MFMA for verification.
#include <cmath>

#include "ctx.h"
#include "gemm.h"

namespace dk {

namespace {

constexpr int TPB = 256;
constexpr int RB = 512;
constexpr long kDensityChunk = 65536;

__device__ double block_sum_d(double v, double* sh) {
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

inline int grid_for(long n) {
  long b = (n + TPB - 1) / TPB;
  return (int)(b > RB ? RB : (b < 1 ? 1 : b));
}

__device__ __forceinline__ float sigmoidf_(float z) { return 0.5f * (1.0f + tanhf(0.5f * z)); }
__device__ __forceinline__ float softplusf_(float z) { return fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))); }

// tab[((a * K + k) * 3 + axis) * nmax + i] = sum_L exp(-(x_i - R_a,axis - L)^2 / (2 w_k^2))
__global__ void desc_tables_kernel(const double* __restrict__ pos, int n_atoms, int K,
                                   const double* __restrict__ w, int nx, int ny, int nz,
                                   double hx, double hy, double hz, double lx, double ly,
                                   double lz, int nmax, double* __restrict__ tab) {
  const long total = (long)n_atoms * K * 3 * nmax;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e % nmax);
    const int axis = (int)((e / nmax) % 3);
    const int k = (int)((e / (3L * nmax)) % K);
    const int a = (int)(e / (3L * nmax * K));
    const int n = axis == 0 ? nx : (axis == 1 ? ny : nz);
    if (i >= n) { tab[e] = 0.0; continue; }
    const double h = axis == 0 ? hx : (axis == 1 ? hy : hz);
    const double len = axis == 0 ? lx : (axis == 1 ? ly : lz);
    const double w2 = 2.0 * w[k] * w[k];
    double d0 = i * h - pos[3 * a + axis];
    d0 -= len * rint(d0 / len);
    const int m = (int)ceil(sqrt(50.0 * w2) / len) + 1;
    double g = 0.0;
    for (int img = -m; img <= m; ++img) {
      const double x = d0 - img * len;
      g += exp(-x * x / w2);
    }
    tab[e] = g;
  }
}

// desc[x * K + k] = sum_a Gx Gy Gz
__global__ void descriptors_kernel(const double* __restrict__ tab, int n_atoms, int K, int nx,
                                   int ny, long ng, int nmax, float* __restrict__ desc) {
  const long total = ng * K;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int k = (int)(e % K);
    const long x = e / K;
    const int ix = (int)(x % nx), iy = (int)((x / nx) % ny), iz = (int)(x / ((long)nx * ny));
    double s = 0.0;
    for (int a = 0; a < n_atoms; ++a) {
      const double* t = tab + ((long)a * K + k) * 3 * nmax;
      s += t[ix] * t[nmax + iy] * t[2 * nmax + iz];
    }
    desc[e] = (float)s;
  }
}

// per-channel partial sums: mode 0 sum d, mode 1 sum (d - mean)^2; grid (RB, K)
__global__ __launch_bounds__(TPB) void channel_sums_kernel(const float* __restrict__ d, long n,
                                                           int K, const double* __restrict__ mean,
                                                           int mode, double* __restrict__ part) {
  __shared__ double sh[TPB / 64];
  const int k = blockIdx.y;
  const double mk = mode ? mean[k] : 0.0;
  double s = 0.0;
  for (long p = blockIdx.x * (long)TPB + threadIdx.x; p < n; p += (long)gridDim.x * TPB) {
    const double v = (double)d[p * K + k] - mk;
    s += mode ? v * v : v;
  }
  s = block_sum_d(s, sh);
  if (threadIdx.x == 0) part[(long)k * RB + blockIdx.x] = s;
}

__global__ __launch_bounds__(TPB) void channel_finish_kernel(const double* __restrict__ part,
                                                             int nb, long n, int mode,
                                                             double* __restrict__ out) {
  __shared__ double sh[TPB / 64];
  const int k = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += TPB) s += part[(long)k * RB + i];
  s = block_sum_d(s, sh);
  // mode 1: 1 / standard deviation (a constant channel gets 1)
  if (threadIdx.x == 0) {
    const double sd = sqrt(s / (double)n);
    out[k] = mode ? (sd > 0.0 ? 1.0 / sd : 1.0) : s / (double)n;
  }
}

// u[k + j K] = (desc[q_j K + k] - mean_k) inv_std_k, t[j] = rho[q_j] * scale
// (idx == null: q_j = j; rho == null: no target)
__global__ void gather_kernel(const float* __restrict__ desc, const double* __restrict__ rho,
                              const int64_t* __restrict__ idx, int K, long n_pts,
                              const double* __restrict__ mean, const double* __restrict__ inv_std,
                              double scale, float* __restrict__ u, float* __restrict__ t) {
  const long total = n_pts * K;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int k = (int)(e % K);
    const long j = e / K;
    const long q = idx ? idx[j] : j;
    u[e] = (float)(((double)desc[q * K + k] - mean[k]) * inv_std[k]);
    if (k == 0 && rho) t[j] = (float)(rho[q] * scale);
  }
}

// z += b (per row); hidden: a = SiLU(z)
__global__ void bias_act_kernel(float* __restrict__ z, float* __restrict__ a,
                                const float* __restrict__ b, int F, long n_pts) {
  const long total = (long)F * n_pts;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const float v = z[e] + b[e % F];
    z[e] = v;
    if (a) a[e] = v * sigmoidf_(v);
  }
}

// output layer: z (1 x P, bias added here), y = softplus(z);
// with a target: dz = (2/P)(y - t) sigmoid(z) and loss partials sum (y - t)^2
__global__ __launch_bounds__(TPB) void output_kernel(const float* __restrict__ z,
                                                     const float* __restrict__ bias,
                                                     const float* __restrict__ t, long n_pts,
                                                     float* __restrict__ dz,
                                                     double* __restrict__ y_out,
                                                     double* __restrict__ part) {
  __shared__ double sh[TPB / 64];
  const float b = bias[0];
  double s = 0.0;
  for (long p = blockIdx.x * (long)TPB + threadIdx.x; p < n_pts; p += (long)gridDim.x * TPB) {
    const float v = z[p] + b;
    const float y = softplusf_(v);
    if (y_out) y_out[p] = (double)y;
    if (t) {
      const float r = y - t[p];
      dz[p] = (2.0f / (float)n_pts) * r * sigmoidf_(v);
      s += (double)r * r;
    } else {
      s += (double)y;
    }
  }
  s = block_sum_d(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(TPB) void finish_sum_kernel(const double* __restrict__ part, int nb,
                                                         double* __restrict__ out) {
  __shared__ double sh[TPB / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += TPB) s += part[i];
  s = block_sum_d(s, sh);
  if (threadIdx.x == 0) out[0] = s;
}

// delta *= SiLU'(z)
__global__ void silu_backward_kernel(float* __restrict__ delta, const float* __restrict__ z,
                                     long total) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const float v = z[e];
    const float s = sigmoidf_(v);
    delta[e] *= s * (1.0f + v * (1.0f - s));
  }
}

// grad_W[o * in + i] = sum_s part[s * out * in + o + i * out] (FP64 partials of the
// split-K product), grad_b[o] = sum over the bias partials
__global__ void weight_grad_kernel(const double* __restrict__ part, int splits, int out, int in,
                                   float* __restrict__ gw) {
  const long mn = (long)out * in;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < mn;
       e += (long)gridDim.x * blockDim.x) {
    const int o = (int)(e % out), i = (int)(e / out);
    double s = 0.0;
    for (int k = 0; k < splits; ++k) s += part[(long)k * mn + e];
    gw[(long)o * in + i] = (float)s;
  }
}

// bias gradient partials: grid (RB, F), part[f * RB + block]
__global__ __launch_bounds__(TPB) void row_sums_kernel(const float* __restrict__ delta, int F,
                                                       long n_pts, double* __restrict__ part) {
  __shared__ double sh[TPB / 64];
  const int f = blockIdx.y;
  double s = 0.0;
  for (long p = blockIdx.x * (long)TPB + threadIdx.x; p < n_pts; p += (long)gridDim.x * TPB)
    s += (double)delta[f + p * F];
  s = block_sum_d(s, sh);
  if (threadIdx.x == 0) part[(long)f * RB + blockIdx.x] = s;
}

__global__ __launch_bounds__(TPB) void row_finish_kernel(const double* __restrict__ part, int nb,
                                                         float* __restrict__ gb) {
  __shared__ double sh[TPB / 64];
  const int f = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += TPB) s += part[(long)f * RB + i];
  s = block_sum_d(s, sh);
  if (threadIdx.x == 0) gb[f] = (float)s;
}

__global__ void adam_kernel(long n, float* __restrict__ th, float* __restrict__ m,
                            float* __restrict__ v, const float* __restrict__ g, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n;
       e += (long)gridDim.x * blockDim.x) {
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.0f - b1) * gi;
    const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    th[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

__global__ void scale_kernel(double* __restrict__ y, long n, double s) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n;
       e += (long)gridDim.x * blockDim.x)
    y[e] *= s;
}

// layer product C (out x P) = W (out x in, row-major) . A (in x P)
template <int MODE>
hipError_t layer_forward(const float* W, const float* A, float* C, int out, int in, long P,
                         hipStream_t st) {
  GemmArgs g;
  g.M = out; g.N = (int)P; g.K = in;
  g.A = W; g.lda = in;
  g.B = A; g.ldb = in;
  g.C = C; g.ldc = out;
  return launch_gemm<MODE, float, float, true, true, kStore, float>(g, st);
}

// C (in x P) = W^T (in x out) . delta (out x P)
template <int MODE>
hipError_t layer_backward_data(const float* W, const float* delta, float* C, int out, int in,
                               long P, hipStream_t st) {
  GemmArgs g;
  g.M = in; g.N = (int)P; g.K = out;
  g.A = W; g.lda = in;          // A(m=i, k=o) = W[o * in + i]: m-contiguous
  g.B = delta; g.ldb = out;     // B(k=o, n=p) = delta[o + p * out]: k-contiguous
  g.C = C; g.ldc = in;
  return launch_gemm<MODE, float, float, false, true, kStore, float>(g, st);
}

// FP64 partials of dW (out x in) = sum_p delta[o, p] A[i, p]
template <int MODE>
hipError_t layer_backward_weights(const float* delta, const float* A, double* part, int out,
                                  int in, long P, int* splits, hipStream_t st) {
  GemmArgs g;
  g.M = out; g.N = in; g.K = (int)P;
  g.A = delta; g.lda = out;     // A(m=o, k=p) = delta[o + p * out]: m-contiguous
  g.B = A; g.ldb = in;          // B(k=p, n=i) = A[i + p * in]: n-contiguous
  g.C = part;
  plan_split_k(g, 512);
  *splits = g.splits;
  return launch_gemm<MODE, float, float, false, false, kPartial, double>(g, st);
}

}  // namespace

// ------------------------------------------------------------------ host --

size_t mlp_params(int n_in, int hidden, int layers) {
  size_t n = (size_t)hidden * n_in + hidden;
  for (int l = 1; l < layers; ++l) n += (size_t)hidden * hidden + hidden;
  return n + hidden + 1;
}

size_t desc_tables_bytes(int n_atoms, int K, int nmax) {
  return (size_t)n_atoms * K * 3 * nmax * sizeof(double);
}

hipError_t descriptors(dk_ctx* c, const double* pos_dev, int n_atoms, int K, const double* w_dev,
                       double* tab, float* desc) {
  const int nmax = std::max(c->nx, std::max(c->ny, c->nz));
  const long tn = (long)n_atoms * K * 3 * nmax;
  long b = (tn + TPB - 1) / TPB; if (b > 8192) b = 8192;
  hipLaunchKernelGGL(desc_tables_kernel, dim3((int)b), dim3(TPB), 0, c->stream, pos_dev, n_atoms,
                     K, w_dev, c->nx, c->ny, c->nz, c->hx, c->hy, c->hz, c->lx, c->ly, c->lz,
                     nmax, tab);
  long bd = (c->ngrid * K + TPB - 1) / TPB; if (bd > 8192) bd = 8192;
  hipLaunchKernelGGL(descriptors_kernel, dim3((int)bd), dim3(TPB), 0, c->stream, tab, n_atoms, K,
                     c->nx, c->ny, c->ngrid, nmax, desc);
  return hipGetLastError();
}

size_t channel_stats_ws_bytes(int K) { return ws_slice((size_t)K * RB * sizeof(double)); }

hipError_t channel_stats(dk_ctx* c, const float* d, long n, int K, double* mean, double* inv_std,
                         void* ws) {
  double* part = (double*)ws;
  const int nb = grid_for(n);
  hipLaunchKernelGGL(channel_sums_kernel, dim3(nb, K), dim3(TPB), 0, c->stream, d, n, K, mean, 0, part);
  hipLaunchKernelGGL(channel_finish_kernel, dim3(K), dim3(TPB), 0, c->stream, part, nb, n, 0, mean);
  hipLaunchKernelGGL(channel_sums_kernel, dim3(nb, K), dim3(TPB), 0, c->stream, d, n, K, mean, 1, part);
  hipLaunchKernelGGL(channel_finish_kernel, dim3(K), dim3(TPB), 0, c->stream, part, nb, n, 1, inv_std);
  return hipGetLastError();
}

hipError_t mlp_gather(dk_ctx* c, const float* desc, const double* rho, const int64_t* idx, int K,
                      long n_pts, const double* mean, const double* inv_std, double scale,
                      float* u, float* t) {
  long b = (n_pts * K + TPB - 1) / TPB; if (b > 8192) b = 8192;
  hipLaunchKernelGGL(gather_kernel, dim3((int)b), dim3(TPB), 0, c->stream, desc, rho, idx, K,
                     n_pts, mean, inv_std, scale, u, t);
  return hipGetLastError();
}

// workspace of a forward / loss-gradient pass over n_pts points
size_t mlp_ws_bytes(int n_in, int hidden, int layers, long n_pts) {
  const size_t hp = ws_slice((size_t)hidden * n_pts * sizeof(float));
  const size_t splits_max = 512;  // plan_split_k never exceeds its target
  (void)n_in;
  return (size_t)(2 * layers + 2) * hp + 2 * ws_slice((size_t)n_pts * sizeof(float)) +
         ws_slice(splits_max * (size_t)hidden * std::max(hidden, n_in) * sizeof(double)) +
         ws_slice((size_t)hidden * RB * sizeof(double)) + ws_slice((size_t)RB * sizeof(double)) +
         ws_slice(8 * sizeof(double));
}

struct MlpBuffers {
  float* Z[8];
  float* A[8];
  float* d0;
  float* d1;
  float* zout;
  float* dz;
  double* part;
  double* rpart;
  double* lpart;
  double* res;
};

static bool take_buffers(WsCursor& cur, int hidden, int layers, long P, MlpBuffers& b) {
  for (int l = 0; l < layers; ++l) {
    b.Z[l] = cur.take<float>((size_t)hidden * P);
    b.A[l] = cur.take<float>((size_t)hidden * P);
  }
  b.d0 = cur.take<float>((size_t)hidden * P);
  b.d1 = cur.take<float>((size_t)hidden * P);
  b.zout = cur.take<float>(P);
  b.dz = cur.take<float>(P);
  return cur.ok;
}

template <int MODE>
static hipError_t mlp_pass(dk_ctx* c, int n_in, int hidden, int layers, const float* params,
                           const float* u, const float* t, long P, float* grad, double* y_out,
                           void* ws, double* host_out) {
  if (layers < 1 || layers > 8) return hipErrorInvalidValue;
  WsCursor cur((char*)ws, mlp_ws_bytes(n_in, hidden, layers, P));
  MlpBuffers b;
  if (!take_buffers(cur, hidden, layers, P, b)) return hipErrorInvalidValue;
  b.part = cur.take<double>(512 * (size_t)hidden * std::max(hidden, n_in));
  b.rpart = cur.take<double>((size_t)hidden * RB);
  b.lpart = cur.take<double>(RB);
  b.res = cur.take<double>(8);
  if (!cur.ok) return hipErrorInvalidValue;
  hipStream_t st = c->stream;
  hipError_t e;
  // parameter offsets
  size_t offW[9], offB[9];
  int din[9], dout[9];
  size_t off = 0;
  for (int l = 0; l <= layers; ++l) {
    din[l] = l == 0 ? n_in : hidden;
    dout[l] = l == layers ? 1 : hidden;
    offW[l] = off; off += (size_t)din[l] * dout[l];
    offB[l] = off; off += dout[l];
  }
  const long tot = (long)hidden * P;
  const int gb = grid_for(tot);
  // forward
  const float* a_in = u;
  for (int l = 0; l < layers; ++l) {
    if ((e = layer_forward<MODE>(params + offW[l], a_in, b.Z[l], dout[l], din[l], P, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(bias_act_kernel, dim3(gb), dim3(TPB), 0, st, b.Z[l], b.A[l], params + offB[l], hidden, P);
    a_in = b.A[l];
  }
  if ((e = layer_forward<MODE>(params + offW[layers], a_in, b.zout, 1, hidden, P, st)) != hipSuccess) return e;
  const int gp = grid_for(P);
  hipLaunchKernelGGL(output_kernel, dim3(gp), dim3(TPB), 0, st, b.zout, params + offB[layers], t, P,
                     b.dz, y_out, b.lpart);
  hipLaunchKernelGGL(finish_sum_kernel, dim3(1), dim3(TPB), 0, st, b.lpart, gp, b.res);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (t && grad) {
    // backward: delta of layer l is (dout[l] x P)
    const float* delta = b.dz;
    for (int l = layers; l >= 0; --l) {
      const float* a_prev = l == 0 ? u : b.A[l - 1];
      int splits = 1;
      if ((e = layer_backward_weights<MODE>(delta, a_prev, b.part, dout[l], din[l], P, &splits, st)) != hipSuccess) return e;
      const long mn = (long)dout[l] * din[l];
      hipLaunchKernelGGL(weight_grad_kernel, dim3(grid_for(mn)), dim3(TPB), 0, st, b.part, splits,
                         dout[l], din[l], grad + offW[l]);
      hipLaunchKernelGGL(row_sums_kernel, dim3(gp, dout[l]), dim3(TPB), 0, st, delta, dout[l], P, b.rpart);
      hipLaunchKernelGGL(row_finish_kernel, dim3(dout[l]), dim3(TPB), 0, st, b.rpart, gp, grad + offB[l]);
      if (l > 0) {
        float* dnext = (delta == b.d0) ? b.d1 : b.d0;
        if ((e = layer_backward_data<MODE>(params + offW[l], delta, dnext, dout[l], din[l], P, st)) != hipSuccess) return e;
        hipLaunchKernelGGL(silu_backward_kernel, dim3(gb), dim3(TPB), 0, st, dnext, b.Z[l - 1], tot);
        delta = dnext;
      }
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  if (host_out) {
    e = hipMemcpyAsync(host_out, b.res, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);
  }
  return hipSuccess;
}

hipError_t mlp_run(dk_ctx* c, int precision, int n_in, int hidden, int layers,
                   const float* params, const float* u, const float* t, long P, float* grad,
                   double* y_out, void* ws, double* host_out) {
  if (precision == 1)
    return mlp_pass<kF32>(c, n_in, hidden, layers, params, u, t, P, grad, y_out, ws, host_out);
  return mlp_pass<kBF16>(c, n_in, hidden, layers, params, u, t, P, grad, y_out, ws, host_out);
}

hipError_t adam_update(dk_ctx* c, long n, float* th, float* m, float* v, const float* g, int t,
                       double lr, double b1, double b2, double eps) {
  const float c1 = (float)(1.0 - std::pow(b1, t)), c2 = (float)(1.0 - std::pow(b2, t));
  hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(TPB), 0, c->stream, n, th, m, v, g,
                     (float)lr, (float)b1, (float)b2, (float)eps, c1, c2);
  return hipGetLastError();
}

// Predicted start density on the whole grid, in chunks of kDensityChunk points:
// rho = n_e y / (h^3 sum y), y = softplus(network(standardised descriptors)).
size_t mlp_density_ws_bytes(int n_in, int hidden, int layers) {
  return ws_slice((size_t)n_in * kDensityChunk * sizeof(float)) +
         mlp_ws_bytes(n_in, hidden, layers, kDensityChunk);
}

hipError_t mlp_density(dk_ctx* c, int precision, int n_in, int hidden, int layers,
                       const float* params, const float* desc, const double* mean,
                       const double* inv_std, double n_e, double* rho, void* ws) {
  WsCursor cur((char*)ws, mlp_density_ws_bytes(n_in, hidden, layers));
  float* u = cur.take<float>((size_t)n_in * kDensityChunk);
  void* mws = cur.take<char>(mlp_ws_bytes(n_in, hidden, layers, kDensityChunk));
  if (!cur.ok) return hipErrorInvalidValue;
  double total = 0.0;
  for (long p0 = 0; p0 < c->ngrid; p0 += kDensityChunk) {
    const long np = std::min((long)kDensityChunk, c->ngrid - p0);
    hipError_t e = mlp_gather(c, desc + p0 * n_in, nullptr, nullptr, n_in, np, mean, inv_std, 1.0,
                              u, nullptr);
    if (e != hipSuccess) return e;
    double part = 0.0;
    e = mlp_run(c, precision, n_in, hidden, layers, params, u, nullptr, np, nullptr, rho + p0,
                mws, &part);
    if (e != hipSuccess) return e;
    total += part;
  }
  if (!(total > 0.0)) return hipErrorInvalidValue;
  const double factor = n_e / (c->dv * total);
  hipLaunchKernelGGL(scale_kernel, dim3(grid_for(c->ngrid)), dim3(TPB), 0, c->stream, rho,
                     c->ngrid, factor);
  return hipGetLastError();
}

}  // namespace dk
