// Chebyshev Fermi-operator expansion of the density kernel (Sec. 4):
//
//   Hhat = (H_s - chi I)/xi,  chi, xi from the extreme eigenvalues of H_s
//   T_0 = I, T_1 = Hhat, T_{j+1} = 2 Hhat T_j - T_{j-1}     (Eq. ThreeTermRecurrenceRelation,
//                                                              all columns at once: FP64 MFMA,
//                                                              batched by T_{k+i} = 2T_kT_i - T_{k-i})
//   tau_j = tr T_j = sum_n e_n^T t_n^j
//   mu: 2 sum'_j c_j(mu) tau_j = N_e                         (Eq. FermiLevelCalc)
//   c_j, d_j, e_j: K-node Gauss-Chebyshev quadrature of Eq. ChebyshevCoeff and
//                  of the E_band / E_ent integrands
//   D_s = sum'_j c_j T_j                                     (Eqs. ChebyshevExpansion, DMCFinal)
//
// The electron count is evaluated through quadrature-node weights
//   w_k = sum'_j tau_j cos(j theta_k),  N(mu) = (4/K) sum_k g(E_k; mu) w_k,
// which is the same double sum with the j-sum done once, so each evaluation
// of N costs O(K).  E_band and E_ent use the same weights.
#include <cmath>

#include "ctx.h"
#include "gemm.h"

namespace dk {

namespace {

constexpr int FT = 1024;  // threads of the single-workgroup Fermi kernel

__device__ __forceinline__ double fermi_g(double e, double mu, double sigma) {
  const double s = (e - mu) / sigma;
  const double q = exp(-fabs(s));
  return s > 0.0 ? q / (1.0 + q) : 1.0 / (1.0 + q);
}

// g log g + (1-g) log(1-g) = -(g softplus(s) + (1-g) softplus(-s))
__device__ __forceinline__ double entropy_f(double e, double mu, double sigma) {
  const double s = (e - mu) / sigma;
  const double q = exp(-fabs(s));
  const double g = s > 0.0 ? q / (1.0 + q) : 1.0 / (1.0 + q);
  const double l1 = log1p(q);
  const double sp_pos = fmax(s, 0.0) + l1;   // softplus(s)
  const double sp_neg = fmax(-s, 0.0) + l1;  // softplus(-s)
  return -(g * sp_pos + (1.0 - g) * sp_neg);
}

__device__ double block_sum_ft(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < FT / 64; ++i) s += sh[i];
  __syncthreads();
  return s;
}

__global__ void init_recurrence_kernel(const double* __restrict__ hs, int n, double chi, double xi,
                                       double* __restrict__ t0, double* __restrict__ t1) {
  const long nn = (long)n * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nn;
       e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    const double h = 0.5 * (hs[e] + hs[(long)j + (long)i * n]);
    t0[e] = (i == j) ? 1.0 : 0.0;
    t1[e] = (h - ((i == j) ? chi : 0.0)) / xi;
  }
}

__global__ void traces_kernel(const double* __restrict__ stack, int n, int count,
                              double* __restrict__ tau) {
  __shared__ double sh[4];
  const int j = blockIdx.x;
  if (j >= count) return;
  const double* t = stack + (long)j * n * n;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += t[(long)i * (n + 1)];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) tau[j] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void assemble_kernel(const double* __restrict__ stack, long nn, int n_pl,
                                const double* __restrict__ c, double* __restrict__ ds) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nn;
       e += (long)gridDim.x * blockDim.x) {
    double s = 0.5 * c[0] * stack[e];
    for (int j = 1; j <= n_pl; ++j) s += c[j] * stack[(long)j * nn + e];
    ds[e] = s;
  }
}

// The Fermi-level search and the quadratures run as four kernels: the cosine
// table, the node weights w_k (many workgroups), the search for mu with the
// node occupations and the E_band / E_ent integrals (one workgroup), and the
// coefficients c_j, d_j, e_j (many workgroups, one wave per j).  Tables live in
// LDS when they fit (use_lds), otherwise they are read from global scratch.

// ct[m] = cos(pi m / (2K)), m < 4K; the node angles theta_k = pi (2k+1)/(2K)
// are ct[2k + 1], and cos(j theta_k) = ct[j (2k+1) mod 4K]
__global__ __launch_bounds__(256) void costab_kernel(int K, double* __restrict__ ct) {
  const int K4 = 4 * K;
  for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < K4; m += gridDim.x * blockDim.x)
    ct[m] = cospi((double)m / (2.0 * K));
}

// The tables are read either from LDS or from global scratch, chosen at compile
// time (LDS): a pointer that may address either space makes flat loads, and a
// flat address whose constant offset was folded out of it can fall below the
// LDS aperture (a table index wrapping to 0 faults the access).

// w_k = sum'_j tau_j cos(j theta_k), one thread per node
template <bool LDS>
__global__ __launch_bounds__(256) void fermi_weights_kernel(const double* __restrict__ tau, int n_pl,
                                                            int K, const double* __restrict__ ct_g,
                                                            double* __restrict__ wk) {
  extern __shared__ double fermi_lds[];
  const int K4 = 4 * K;
  if constexpr (LDS) {
    for (int m = threadIdx.x; m < K4; m += blockDim.x) fermi_lds[m] = ct_g[m];
    __syncthreads();
  }
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const long step = 2L * k + 1;
  double s = 0.5 * tau[0];
  int idx = 0;
  for (int j = 1; j <= n_pl; ++j) {
    idx += (int)step;
    if (idx >= K4) idx -= K4;
    s += tau[j] * (LDS ? fermi_lds[idx] : ct_g[idx]);
  }
  wk[k] = s;
}

// sums of a and b over the workgroup, returned to every thread
__device__ void block_sum2_ft(double& a, double& b, double* sha, double* shb) {
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) {
    sha[w] = a;
    shb[w] = b;
  }
  __syncthreads();
  a = 0.0;
  b = 0.0;
  for (int i = 0; i < FT / 64; ++i) {
    a += sha[i];
    b += shb[i];
  }
  __syncthreads();
}

// out[0] = mu, [1] = e_band, [2] = e_ent, [3] = n_count, [4] = search steps.
// fixed_mu: use mu_in.  Otherwise mu solves N(mu) = N_e on the bracket
// [lam_min - 40 sigma - 1, lam_max + 40 sigma + 1] (N increases with mu):
// while the bracket is wider than 16 sigma, each of the 16 waves evaluates N at
// one of 16 interior points and the bracket shrinks to the sub-interval where
// N crosses N_e (divided by 17 per step); then Newton steps on
// N'(mu) = (4/K) sum_k w_k g_k (1 - g_k) / sigma, every one shrinking the
// bracket and falling back to its midpoint when the step leaves it, until the
// step is below 1e-15 |mu| or the bracket below 1e-14 |mu|.
// gk_g (3K): g_k, E_k g_k and the entropy integrand at the nodes.
template <bool LDS>
__global__ __launch_bounds__(FT) void fermi_search_kernel(
    const double* __restrict__ ct, const double* __restrict__ wk_g, int K, double chi, double xi,
    double lam_min, double lam_max, double sigma, double n_e, int fixed_mu, double mu_in,
    double* __restrict__ gk_g, double* out, unsigned* err) {
  extern __shared__ double fermi_lds[];
  __shared__ double sha[FT / 64], shb[FT / 64];
  const int t = threadIdx.x;
  // node energies E_k (LDS [0, K)) and weights w_k (LDS [K, 2K))
  if constexpr (LDS) {
    for (int k = t; k < K; k += FT) {
      fermi_lds[k] = xi * ct[2 * k + 1] + chi;
      fermi_lds[K + k] = wk_g[k];
    }
    __syncthreads();
  }
  auto node_e = [&](int k) { return LDS ? fermi_lds[k] : xi * ct[2 * k + 1] + chi; };
  auto node_w = [&](int k) { return LDS ? fermi_lds[K + k] : wk_g[k]; };
  // N(mu) - N_e and N'(mu) over all nodes, on every thread
  auto count = [&](double mu, double& f, double& df) {
    double s = 0.0, d = 0.0;
    for (int k = t; k < K; k += FT) {
      const double g = fermi_g(node_e(k), mu, sigma);
      const double w = node_w(k);
      s += g * w;
      d += g * (1.0 - g) * w;
    }
    block_sum2_ft(s, d, sha, shb);
    f = (4.0 / K) * s - n_e;
    df = (4.0 / K) * d / sigma;
  };
  double mu;
  int it = 0;
  if (fixed_mu) {
    mu = mu_in;
  } else {
    double lo = lam_min - 40.0 * sigma - 1.0, hi = lam_max + 40.0 * sigma + 1.0;
    double flo, fhi, dummy;
    count(lo, flo, dummy);
    count(hi, fhi, dummy);
    mu = 0.5 * (lo + hi);
    if (!(flo < 0.0 && fhi > 0.0)) {
      if (t == 0) atomicOr(err, kErrFermi);
    } else {
      constexpr int W = FT / 64;
      __shared__ double fw[W];
      const int wv = t >> 6, lane = t & 63;
      auto narrow = [&]() { return hi - lo <= 1e-14 * fmax(1.0, fabs(0.5 * (lo + hi))); };
      while (it < 200 && !narrow() && hi - lo > 16.0 * sigma) {
        const double width = hi - lo;
        const double mw = lo + width * (double)(wv + 1) / (double)(W + 1);
        double sw = 0.0;
        for (int k = lane; k < K; k += 64) sw += fermi_g(node_e(k), mw, sigma) * node_w(k);
        for (int o = 32; o > 0; o >>= 1) sw += __shfl_xor(sw, o);
        if (lane == 0) fw[wv] = (4.0 / K) * sw - n_e;
        __syncthreads();
        int first = W;  // first trial point with count >= N_e
        for (int v = 0; v < W; ++v)
          if (fw[v] >= 0.0) { first = v; break; }
        const double nlo = (first == 0) ? lo : lo + width * (double)first / (double)(W + 1);
        const double nhi = (first == W) ? hi : lo + width * (double)(first + 1) / (double)(W + 1);
        lo = nlo;
        hi = nhi;
        __syncthreads();  // fw is rewritten by the next step
        ++it;
      }
      mu = 0.5 * (lo + hi);
      while (it < 200 && !narrow()) {
        double f, df;
        count(mu, f, df);
        ++it;
        if (f < 0.0) lo = mu;
        else hi = mu;
        double mn = (df > 0.0) ? mu - f / df : 0.5 * (lo + hi);
        if (!(mn > lo && mn < hi)) mn = 0.5 * (lo + hi);
        const bool done = fabs(mn - mu) <= 1e-15 * fmax(1.0, fabs(mu)) || f == 0.0;
        mu = (f == 0.0) ? mu : mn;
        if (done) break;
      }
      if (narrow()) mu = 0.5 * (lo + hi);
    }
  }
  // occupations, band and entropy integrands at the nodes, and their integrals
  double* gk = gk_g;
  double* ek = gk_g + K;
  double* sk = gk_g + 2 * K;
  double sn = 0.0, sb = 0.0, sent = 0.0;
  for (int k = t; k < K; k += FT) {
    const double e = node_e(k);
    const double w = node_w(k);
    const double g = fermi_g(e, mu, sigma);
    const double ent = entropy_f(e, mu, sigma);
    gk[k] = g;
    ek[k] = e * g;
    sk[k] = ent;
    sn += g * w;
    sb += e * g * w;
    sent += ent * w;
  }
  block_sum2_ft(sn, sb, sha, shb);
  double zero = 0.0;
  block_sum2_ft(sent, zero, sha, shb);
  if (t == 0) {
    out[0] = mu;
    out[1] = (4.0 / K) * sb;
    out[2] = sigma * (4.0 / K) * sent;
    out[3] = (4.0 / K) * sn;
    out[4] = (double)it;
  }
}

// c_j, d_j, e_j = (2/K) sum_k f(E_k) cos(j theta_k); one wave per j, lanes over
// the nodes (cos(j theta_k) = ct[j (2k+1) mod 4K], stepped by 64 nodes without
// a division)
template <bool LDS>
__global__ __launch_bounds__(256) void fermi_coef_kernel(const double* __restrict__ ct_g,
                                                         const double* __restrict__ gk_g, int n_pl,
                                                         int K, double* __restrict__ coef) {
  extern __shared__ double fermi_lds[];
  const int K4 = 4 * K;
  if constexpr (LDS) {
    for (int m = threadIdx.x; m < K4; m += blockDim.x) fermi_lds[m] = ct_g[m];
    for (int m = threadIdx.x; m < 3 * K; m += blockDim.x) fermi_lds[K4 + m] = gk_g[m];
    __syncthreads();
  }
  // cos table at [0, 4K), then g_k, E_k g_k, entropy at [4K, 7K) (LDS) or gk_g
  auto cs_at = [&](int i) { return LDS ? fermi_lds[i] : ct_g[i]; };
  auto f_at = [&](int i) { return LDS ? fermi_lds[K4 + i] : gk_g[i]; };
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (j > n_pl) return;
  double sc = 0.0, sd = 0.0, se = 0.0;
  const int inc = (int)((128L * j) % K4);
  int idx = (int)(((long)j * (2L * lane + 1)) % K4);
  for (int k = lane; k < K; k += 64) {
    const double cs = cs_at(idx);
    idx += inc;
    if (idx >= K4) idx -= K4;
    sc += f_at(k) * cs;
    sd += f_at(K + k) * cs;
    se += f_at(2 * K + k) * cs;
  }
  for (int o = 32; o > 0; o >>= 1) {
    sc += __shfl_xor(sc, o);
    sd += __shfl_xor(sd, o);
    se += __shfl_xor(se, o);
  }
  if (lane == 0) {
    coef[j] = (2.0 / K) * sc;
    coef[(n_pl + 1) + j] = (2.0 / K) * sd;
    coef[2 * (n_pl + 1) + j] = (2.0 / K) * se;
  }
}

// out[0] = sum_{n < j <= J} |c_j(mu)| with c_j by K-node Gauss-Chebyshev
// quadrature of the Fermi-Dirac function on [chi - xi, chi + xi]; gk: K scratch.
__global__ __launch_bounds__(FT) void coefficient_tail_kernel(int n, int J, int K, double chi,
                                                              double xi, double mu, double sigma,
                                                              double* __restrict__ gk,
                                                              double* out) {
  __shared__ double sh[FT / 64];
  const int t = threadIdx.x;
  const long K4 = 4L * K;
  for (int k = t; k < K; k += FT)
    gk[k] = fermi_g(xi * cospi((double)(2 * k + 1) / (2.0 * K)) + chi, mu, sigma);
  __syncthreads();
  double tail = 0.0;
  for (int j = n + 1 + t; j <= J; j += FT) {
    double sc = 0.0;
    const long step = (2L * j) % K4;
    long idx = j % K4;
    for (int k = 0; k < K; ++k) {
      sc += gk[k] * cospi((double)idx / (2.0 * K));
      idx += step;
      if (idx >= K4) idx -= K4;
    }
    tail += fabs((2.0 / K) * sc);
  }
  tail = block_sum_ft(tail, sh);
  if (t == 0) out[0] = tail;
}

}  // namespace

static int n_nodes(int n_pl) { return (4 * (n_pl + 1) > 1024) ? 4 * (n_pl + 1) : 1024; }

// n_pl = 0 (tail rule): degrees 32, 64, ... up to kTailCap
static int max_degree(int n_pl) { return n_pl > 0 ? n_pl : kTailCap; }

size_t foe_ws_bytes(int n_s, int n_pl) {
  const size_t nn = (size_t)n_s * n_s;
  const int nmax = max_degree(n_pl);
  const int K = n_nodes(nmax);
  const int Kt = n_nodes(4 * nmax);
  return ws_slice((size_t)(nmax + 1) * nn * sizeof(double))         // T_0 .. T_n_pl
         + ws_slice((size_t)(nmax + 2) * sizeof(double))            // tau
         + ws_slice(3 * (size_t)(nmax + 1) * sizeof(double))        // c, d, e
         + ws_slice(spectral_ws_bytes(n_s))                           // spectral-bound scratch
         + ws_slice((size_t)(4 * K) * sizeof(double))               // cos table
         + ws_slice((size_t)K * sizeof(double))                     // w_k
         + ws_slice((size_t)(3 * K) * sizeof(double))               // g_k, E_k g_k, entropy
         + ws_slice(16 * sizeof(double))                             // results
         + ws_slice((size_t)Kt * sizeof(double));                   // tail-rule nodes
}

struct FermiScratch {
  double* costab;
  double* wk;
  double* gk;
  double* res;
};

static FermiScratch take_fermi_scratch(WsCursor& cur, int nmax) {
  const int K = n_nodes(nmax);
  FermiScratch f;
  f.costab = cur.take<double>(4 * K);
  f.wk = cur.take<double>(K);
  f.gk = cur.take<double>(3 * K);
  f.res = cur.take<double>(16);
  return f;
}

static hipError_t run_fermi(dk_ctx* c, const double* tau, int n_pl, double chi, double xi,
                            double lam_min, double lam_max, double sigma, double n_e,
                            int fixed_mu, double mu_in, const FermiScratch& f, double* coef_out,
                            double* host_out) {
  const int K = n_nodes(n_pl);
  double* res = f.res;
  constexpr size_t kMaxLds = 150 * 1024;
  if (!(c->lds_attr_done & kAttrFermi)) {
    const void* fns[] = {(const void*)fermi_weights_kernel<true>,
                         (const void*)fermi_search_kernel<true>,
                         (const void*)fermi_coef_kernel<true>};
    for (const void* fn : fns) {
      const hipError_t e =
          hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
      if (e != hipSuccess) return e;
    }
    c->lds_attr_done |= kAttrFermi;
  }
  const size_t lds_w = 4 * (size_t)K * sizeof(double);
  const size_t lds_s = 2 * (size_t)K * sizeof(double);
  const size_t lds_c = 7 * (size_t)K * sizeof(double);
  const bool use_w = lds_w <= kMaxLds, use_s = lds_s <= kMaxLds, use_c = lds_c <= kMaxLds;
  hipLaunchKernelGGL(costab_kernel, dim3(ceil_div(4L * K, 256)), dim3(256), 0, c->stream, K,
                     f.costab);
  const dim3 gw(ceil_div(K, 256)), gc(ceil_div(n_pl + 1, 4));
  if (use_w)
    hipLaunchKernelGGL(fermi_weights_kernel<true>, gw, dim3(256), lds_w, c->stream, tau, n_pl, K,
                       f.costab, f.wk);
  else
    hipLaunchKernelGGL(fermi_weights_kernel<false>, gw, dim3(256), 0, c->stream, tau, n_pl, K,
                       f.costab, f.wk);
  if (use_s)
    hipLaunchKernelGGL(fermi_search_kernel<true>, dim3(1), dim3(FT), lds_s, c->stream, f.costab,
                       f.wk, K, chi, xi, lam_min, lam_max, sigma, n_e, fixed_mu, mu_in, f.gk, res,
                       c->err_dev);
  else
    hipLaunchKernelGGL(fermi_search_kernel<false>, dim3(1), dim3(FT), 0, c->stream, f.costab,
                       f.wk, K, chi, xi, lam_min, lam_max, sigma, n_e, fixed_mu, mu_in, f.gk, res,
                       c->err_dev);
  if (use_c)
    hipLaunchKernelGGL(fermi_coef_kernel<true>, gc, dim3(256), lds_c, c->stream, f.costab, f.gk,
                       n_pl, K, coef_out);
  else
    hipLaunchKernelGGL(fermi_coef_kernel<false>, gc, dim3(256), 0, c->stream, f.costab, f.gk, n_pl,
                       K, coef_out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(host_out, res, 5 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(c->stream);
}

static inline int blocks_for(long n) {
  long b = (n + 255) / 256;
  return (int)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

hipError_t foe_run(dk_ctx* c, const double* hs, int n_s, double n_e, double sigma, int n_pl,
                   double* ds, double* tau_out, dk_fermi_info* info, void* ws) {
  const int nmax = max_degree(n_pl);
  WsCursor cur((char*)ws, foe_ws_bytes(n_s, n_pl));
  const long nn = (long)n_s * n_s;
  double* stack = cur.take<double>((size_t)(nmax + 1) * nn);
  double* tau = cur.take<double>(nmax + 2);
  double* coef = cur.take<double>(3 * (nmax + 1));
  void* lz = cur.take<char>(spectral_ws_bytes(n_s));
  const FermiScratch fs = take_fermi_scratch(cur, nmax);
  double* tail_nodes = cur.take<double>(n_nodes(4 * nmax));
  if (!cur.ok) return hipErrorInvalidValue;
  double lo = 0, hi = 0;
  int lz_it = 0;
  hipError_t e;
  {
    KTimer kt(c, DK_K_BOUNDS);
    e = spectral_bounds(c, hs, n_s, lz, &lo, &hi, &lz_it);
  }
  if (e != hipSuccess) return e;
  const double chi = 0.5 * (hi + lo);
  double xi = 0.5 * (hi - lo);
  if (!(xi > 1e-12 * fmax(1.0, fabs(chi)))) xi = 1.0;
  {
    KTimer kt(c, DK_K_FERMI);
    hipLaunchKernelGGL(init_recurrence_kernel, dim3(blocks_for(nn)), dim3(256), 0, c->stream, hs,
                       n_s, chi, xi, stack, stack + nn);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // T_{k+i} = 2 T_k T_i - T_{k-i} (i = 1..k) gives T_{k+1}..T_{2k} from
  // T_0..T_k in one batched product: the three-term recurrence (the case i = 1)
  // applied to all columns, regrouped so that ceil(log2 n_pl) launches cover
  // the degree.  Same products, same rounding growth as the step-by-step form.
  int built = 1;  // T_0, T_1 exist
  auto extend = [&](int target) -> hipError_t {
    while (built < target) {
      const int k = built;
      const int cnt = (2 * k <= target) ? k : target - k;
      KTimer kt(c, DK_K_FOE_GEMM);
      GemmArgs g;
      g.M = n_s; g.N = n_s; g.K = n_s;
      g.A = stack + (long)k * nn; g.lda = n_s;         // T_k, m-contiguous (symmetric)
      g.B = stack + nn; g.ldb = n_s;                    // T_i, i = 1..cnt
      g.C = stack + (long)(k + 1) * nn; g.ldc = n_s;   // T_{k+i}
      g.Cin = stack + (long)(k - 1) * nn; g.ldcin = n_s; // T_{k-i}
      g.alpha = 2.0; g.beta = -1.0;
      // every T_j is symmetric: upper tiles only, each mirrored into the lower
      g.tile_sel = kUpperTiles;
      g.mirror = 1;
      g.batch = cnt;
      g.bs_a = 0; g.bs_b = nn; g.bs_c = nn; g.bs_cin = -nn;
      // 32x32 tiles keep every CU busy for small batches of subspaces up to
      // ~1000 orbitals; 64x64 tiles once the batch alone gives ~1000 of them
      const long tiles64 = (long)ceil_div(n_s, 64) * ceil_div(n_s, 64) * cnt;
      hipError_t r = (n_s <= 1024 && tiles64 < 1024)
          ? launch_gemm<kF64, double, double, false, true, kStore, double, 32>(g, c->stream)
          : launch_gemm<kF64, double, double, false, true, kStore, double, 64>(g, c->stream);
      if (r != hipSuccess) return r;
      built = k + cnt;
    }
    return hipSuccess;
  };
  const bool tail_rule = (n_pl == 0);
  int deg = tail_rule ? kTailStart : n_pl;
  double host[5];
  for (;;) {
    if ((e = extend(deg)) != hipSuccess) return e;
    {
      KTimer kt(c, DK_K_FERMI);
      hipLaunchKernelGGL(traces_kernel, dim3(deg + 1), dim3(256), 0, c->stream, stack, n_s,
                         deg + 1, tau);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    {
      KTimer kt(c, DK_K_FERMI);
      e = run_fermi(c, tau, deg, chi, xi, lo, hi, sigma, n_e, 0, 0.0, fs, coef, host);
    }
    if (e != hipSuccess) return e;
    if (!tail_rule) break;
    // tail rule: accept deg once sum_{deg < j <= 4 deg} |c_j(mu)| <= kTailTol
    double tail = 0.0;
    {
      KTimer kt(c, DK_K_FERMI);
      hipLaunchKernelGGL(coefficient_tail_kernel, dim3(1), dim3(FT), 0, c->stream, deg, 4 * deg,
                         n_nodes(4 * deg), chi, xi, host[0], sigma, tail_nodes, fs.res + 8);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      e = hipMemcpyAsync(&tail, fs.res + 8, sizeof(double), hipMemcpyDeviceToHost, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    if (e != hipSuccess) return e;
    if (tail <= kTailTol) break;
    if (2 * deg > kTailCap) {
      flag_error(c, kErrDegree);
      break;
    }
    deg *= 2;
  }
  {
    KTimer kt(c, DK_K_FERMI);
    hipLaunchKernelGGL(assemble_kernel, dim3(blocks_for(nn)), dim3(256), 0, c->stream, stack, nn,
                       deg, coef, ds);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (tau_out) {
    e = hipMemcpyAsync(tau_out, tau, (deg + 1) * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return e;
  }
  info->mu = host[0];
  info->e_band = host[1];
  info->e_ent = host[2];
  info->n_count = host[3];
  info->bisect_iters = (int)host[4];
  info->lam_min = lo;
  info->lam_max = hi;
  info->chi = chi;
  info->xi = xi;
  info->n_pl = deg;
  info->bound_steps = lz_it;
  info->reserved = 0;
  return hipSuccess;
}

hipError_t energies(dk_ctx* c, const double* tau, int n_pl, double mu, double chi, double xi,
                    double sigma, double* e_band, double* e_ent, void* ws) {
  WsCursor cur((char*)ws, foe_ws_bytes(1, n_pl));
  double* coef = cur.take<double>(3 * (n_pl + 1));
  const FermiScratch fs = take_fermi_scratch(cur, n_pl);
  if (!cur.ok) return hipErrorInvalidValue;
  double host[5];
  hipError_t e = run_fermi(c, tau, n_pl, chi, xi, chi - xi, chi + xi, sigma, 0.0, 1, mu, fs,
                           coef, host);
  if (e != hipSuccess) return e;
  *e_band = host[1];
  *e_ent = host[2];
  return hipSuccess;
}

}  // namespace dk
