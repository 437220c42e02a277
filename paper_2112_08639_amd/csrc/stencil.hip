// Local part of the Hamiltonian on a block of grid vectors, fused with the
// Chebyshev-filter update:
//
//   Y_out = alpha * ((-1/2 Lap_h + V_eff - shift) Y_in) + beta * Y_prev
//
// -1/2 Lap_h is the twelfth-order central-difference kinetic operator of the
// paper's real-space discretisation (Sec. 5): a 37-point star of radius 6,
// periodic in x, y, z.  Y_prev may alias Y_out (the recurrence overwrites
// Y_{k-1} with Y_{k+1} point by point).  The nonlocal projector term is added
// by nonlocal_scatter.
//
// Kernel layout.  A workgroup owns one column of the block, TY full x-rows of
// an xy-plane, and streams through a chunk of z-planes.  Each thread keeps the
// 13 values of its points' z-columns in registers (a queue shifted once per
// plane), so every value of Y_in is loaded from memory once per chunk plus a
// 12-plane prologue.  The centre plane of the tile, with 6 periodic halo rows
// above and below, is staged in LDS for the x and y neighbours; x wraps within
// the row.
#include <utility>

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
  // the same in FP32, converted once on the host (uniform SGPR operands)
  float fcx[7], fcy[7], fcz[7];
  float falpha, fbeta, fdshift, fshift;
};

// (a + b) - 2 c with one rounding of the difference.  The kinetic term is
// accumulated as sum_k c_k ((x_{+k} + x_{-k}) - 2 x_0) per axis rather than
// as diag x_0 + sum_k c_k (x_{+k} + x_{-k}): the running sum then stays at the
// size of the kinetic term instead of cancelling diag x_0 (~45 Ha x_0 at
// h = 0.32 bohr), and a constant is annihilated exactly whatever the rounding
// of the coefficients.  In FP32 the other form shifts smooth states by
// ~3e-6 Ha (the rounded coefficients do not sum to zero) plus a correlated
// rounding bias of the cancelling sums.
template <typename T>
__device__ __forceinline__ T pair_d2(T a, T b, T c) {
  if constexpr (sizeof(T) == 4) return __builtin_fmaf(-2.0f, c, a + b);
  else return __builtin_fma(-2.0, c, a + b);
}

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
  const T alpha = (T)a.alpha, beta = (T)a.beta, vshift = (T)a.shift;

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
      const T x0 = q[r][6];
      T acc = 0;
#pragma unroll
      for (int k = 1; k <= kFdRadius; ++k) {
        int xp = x + k; if (xp >= nx) xp -= nx;
        int xm = x - k; if (xm < 0) xm += nx;
        acc += cx[k] * pair_d2(rowp[xp], rowp[xm], x0);
        acc += cy[k] * pair_d2(rowp[x + k * nx], rowp[x - k * nx], x0);
        acc += cz[k] * pair_d2(q[r][6 + k], q[r][6 - k], x0);
      }
      acc += (veff[g] - vshift) * x0;
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

// Whole-plane variant for planes of at most 4096 points with nx % 4 == 0.
// A workgroup owns one column and a chunk of z-planes; thread t owns the four
// consecutive points x0..x0+3 of row y (x0 = 4 (t % (nx/4)), y = t / (nx/4)),
// moved as one 16-byte (float) or 32-byte (double) vector.  Its 13-plane
// z-queue lives in registers and the load of the plane entering the queue is
// issued one step ahead.  The centre plane goes to one of two LDS buffers whose
// rows carry 8 periodic copies on each side, so the x and y neighbours are
// aligned vector reads with no wrap test; y wraps by row index.  One barrier
// per plane (double buffering).
template <typename T>
struct Vec4 { T v[4]; };

template <typename T>
__device__ __forceinline__ Vec4<T> ld4(const T* p) {
  Vec4<T> r;
  if constexpr (sizeof(T) == 4) {
    const float4 f = *reinterpret_cast<const float4*>(p);
    r.v[0] = f.x; r.v[1] = f.y; r.v[2] = f.z; r.v[3] = f.w;
  } else {
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    r.v[0] = a.x; r.v[1] = a.y; r.v[2] = b.x; r.v[3] = b.y;
  }
  return r;
}

template <typename T>
__device__ __forceinline__ void st4(T* p, const Vec4<T>& r) {
  if constexpr (sizeof(T) == 4) {
    *reinterpret_cast<float4*>(p) = make_float4(r.v[0], r.v[1], r.v[2], r.v[3]);
  } else {
    *reinterpret_cast<double2*>(p) = make_double2(r.v[0], r.v[1]);
    *reinterpret_cast<double2*>(p + 2) = make_double2(r.v[2], r.v[3]);
  }
}

constexpr int kPad = 8;  // periodic copies on each side of an LDS row

// MAXT bounds the workgroup size: a plane of up to 640 threads (10 waves)
// runs one workgroup per CU at 3 waves per SIMD, which leaves up to 168
// VGPRs for the z-queue and the prefetched V_eff and Y_{k-1} vectors.
template <typename T, int MAXT>
__global__ __launch_bounds__(MAXT) void stencil_plane_kernel(StencilArgs a) {
  extern __shared__ unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int pitch = nx + 2 * kPad;
  const int plane_lds = ny * pitch;
  const long pstride = (long)nx * ny;
  const int col = blockIdx.z;
  const int z0 = blockIdx.y * a.zc;
  const int z1 = min(nz, z0 + a.zc);
  const int segs = nx / 4;
  const int t = threadIdx.x;
  const bool active = t < segs * ny;
  const int y = active ? t / segs : 0;
  const int x0 = active ? 4 * (t - y * segs) : 0;
  const long off = x0 + (long)nx * y;

  const T* __restrict__ yin = reinterpret_cast<const T*>(a.yin) + (long)col * a.ld;
  const T* __restrict__ yprev =
      a.yprev ? reinterpret_cast<const T*>(a.yprev) + (long)col * a.ld : nullptr;
  T* yout = reinterpret_cast<T*>(a.yout) + (long)col * a.ld;
  const T* __restrict__ veff = reinterpret_cast<const T*>(a.veff);

  T cx[7], cy[7], cz[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) { cx[k] = (T)a.cx[k]; cy[k] = (T)a.cy[k]; cz[k] = (T)a.cz[k]; }
  const T alpha = (T)a.alpha, beta = (T)a.beta, vshift = (T)a.shift;

  // row offsets of the y neighbours (periodic), k = 1..6
  int yp[7], ym[7];
#pragma unroll
  for (int k = 1; k <= 6; ++k) {
    int u = y + k; if (u >= ny) u -= ny;
    int d = y - k; if (d < 0) d += ny;
    yp[k] = u * pitch + kPad + x0;
    ym[k] = d * pitch + kPad + x0;
  }
  const int own = y * pitch + kPad + x0;
  // periodic copies: the first kPad points of a row also go right of the row,
  // the last kPad points also go left of it
  const int copy_r = (x0 < kPad) ? y * pitch + kPad + nx + x0 : -1;
  const int copy_l = (x0 >= nx - kPad) ? y * pitch + x0 - (nx - kPad) : -1;

  Vec4<T> q[13];
  const Vec4<T> zero4 = {{(T)0, (T)0, (T)0, (T)0}};
#pragma unroll
  for (int d = 0; d < 12; ++d) {
    int zz = z0 - 6 + d;
    zz = ((zz % nz) + nz) % nz;
    q[d] = active ? ld4(yin + zz * pstride + off) : zero4;
  }
  int zn = z0 + 6; if (zn >= nz) zn -= nz;
  Vec4<T> nxt = active ? ld4(yin + zn * pstride + off) : zero4;
  // with registers to spare (MAXT <= 640), V_eff and Y_{k-1} of the next
  // plane are loaded one plane ahead
  constexpr bool PRE = MAXT <= 640;
  Vec4<T> vv_n = zero4, pv_n = zero4;
  if constexpr (PRE) {
    if (active && z0 < z1) {
      vv_n = ld4(veff + (long)z0 * pstride + off);
      if (yprev) pv_n = ld4(yprev + (long)z0 * pstride + off);
    }
  }
  int buf = 0;
  for (int z = z0; z < z1; ++z) {
    q[12] = nxt;
    Vec4<T> vv = vv_n, pv = pv_n;
    int zl = z + 7; if (zl >= nz) zl -= nz;
    if (z + 1 < z1 && active) {
      nxt = ld4(yin + zl * pstride + off);
      if constexpr (PRE) {
        const long gn = (long)(z + 1) * pstride + off;
        vv_n = ld4(veff + gn);
        if (yprev) pv_n = ld4(yprev + gn);
      }
    }
    const long g = (long)z * pstride + off;
    if constexpr (!PRE) {
      if (active) {
        vv = ld4(veff + g);
        if (yprev) pv = ld4(yprev + g);
      }
    }
    T* P = lds + buf * plane_lds;
    if (active) {
      st4(P + own, q[6]);
      if (copy_r >= 0) st4(P + copy_r, q[6]);
      if (copy_l >= 0) st4(P + copy_l, q[6]);
    }
    __syncthreads();
    if (active) {
      // x window: x0-8 .. x0+11
      T w[20];
#pragma unroll
      for (int s = 0; s < 5; ++s) {
        const Vec4<T> r = ld4(P + own - kPad + 4 * s);
        w[4 * s] = r.v[0]; w[4 * s + 1] = r.v[1]; w[4 * s + 2] = r.v[2]; w[4 * s + 3] = r.v[3];
      }
      T acc[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        acc[i] = 0;
#pragma unroll
        for (int k = 1; k <= 6; ++k) acc[i] += cx[k] * pair_d2(w[8 + i + k], w[8 + i - k], q[6].v[i]);
      }
#pragma unroll
      for (int k = 1; k <= 6; ++k) {
        const Vec4<T> up = ld4(P + yp[k]);
        const Vec4<T> dn = ld4(P + ym[k]);
#pragma unroll
        for (int i = 0; i < 4; ++i)
          acc[i] += cy[k] * pair_d2(up.v[i], dn.v[i], q[6].v[i]) +
                    cz[k] * pair_d2(q[6 + k].v[i], q[6 - k].v[i], q[6].v[i]);
      }
      Vec4<T> out;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        out.v[i] = alpha * (acc[i] + (vv.v[i] - vshift) * q[6].v[i]) +
                   (yprev ? beta * pv.v[i] : (T)0);
      st4(yout + g, out);
    }
    buf ^= 1;
#pragma unroll
    for (int d = 0; d < 12; ++d) q[d] = q[d + 1];
  }
}

// FP32 whole-plane variant for planes with 8 <= nx <= 64 and ny >= 6.  Rows
// have a fixed pitch and the plane carries 6 periodic copies of rows above and
// below it, so every LDS read of a thread is one base address plus a constant
// offset, and the FP32 coefficients come converted from the host (scalar
// operands).  That brings the kernel to 90 VGPRs: two plane workgroups share a
// CU.  Per thread and plane the LDS reads are twelve 16-byte vectors for the y
// neighbours and two 16-byte plus two 8-byte ones for x: the x window skips
// the thread's own four values, which it holds in registers.  V_eff and
// Y_{k-1} are loaded after the barrier; their latency is covered by the LDS
// part and by the CU's other workgroup.
constexpr int kPitch2 = 80;
template <int MAXT>
__global__ __launch_bounds__(MAXT) __attribute__((amdgpu_waves_per_eu(5)))
void stencil_plane2_kernel(StencilArgs a) {
  extern __shared__ unsigned char smem_raw[];
  float* lds = reinterpret_cast<float*>(smem_raw);
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int plane_lds = (ny + 12) * kPitch2;
  const int pstride = nx * ny;
  const int col = blockIdx.z;
  const int z0 = blockIdx.y * a.zc;
  const int z1 = min(nz, z0 + a.zc);
  const int segs = nx / 4;
  const int t = threadIdx.x;
  const bool active = t < segs * ny;
  const int y = active ? t / segs : 0;
  const int x0 = active ? 4 * (t - y * segs) : 0;
  const int off = x0 + nx * y;

  const float* __restrict__ yin = reinterpret_cast<const float*>(a.yin) + (long)col * a.ld;
  const float* __restrict__ yprev =
      a.yprev ? reinterpret_cast<const float*>(a.yprev) + (long)col * a.ld : nullptr;
  float* yout = reinterpret_cast<float*>(a.yout) + (long)col * a.ld;
  const float* __restrict__ veff = reinterpret_cast<const float*>(a.veff);

  const float* cx = a.fcx;
  const float* cy = a.fcy;
  const float* cz = a.fcz;
  const float alpha = a.falpha, beta = a.fbeta, vshift = a.fshift;

  // LDS row y + 6 holds plane row y; rows 0..5 and ny+6..ny+11 are periodic
  // copies.  base: row y (six rows above the own row), x0 - kPad.
  const int base = y * kPitch2 + x0;
  const int own = base + 6 * kPitch2 + kPad;
  const int copy_r = (x0 < kPad) ? own + nx : -1;
  const int copy_l = (x0 >= nx - kPad) ? own - nx : -1;
  const int copy_dn = (y < 6) ? own + ny * kPitch2 : -1;
  const int copy_up = (y >= ny - 6) ? own - ny * kPitch2 : -1;

  Vec4<float> q[13];
  const Vec4<float> zero4 = {{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
  for (int d = 0; d < 12; ++d) {
    int zz = z0 - 6 + d;
    zz = ((zz % nz) + nz) % nz;
    q[d] = active ? ld4(yin + zz * pstride + off) : zero4;
  }
  int zn = z0 + 6; if (zn >= nz) zn -= nz;
  Vec4<float> nxt = active ? ld4(yin + zn * pstride + off) : zero4;
  int buf = 0;
  for (int z = z0; z < z1; ++z) {
    q[12] = nxt;
    int zl = z + 7; if (zl >= nz) zl -= nz;
    if (z + 1 < z1 && active) nxt = ld4(yin + zl * pstride + off);
    const int g = z * pstride + off;
    float* P = lds + buf * plane_lds;
    if (active) {
      st4(P + own, q[6]);
      if (copy_r >= 0) st4(P + copy_r, q[6]);
      if (copy_l >= 0) st4(P + copy_l, q[6]);
      if (copy_dn >= 0) st4(P + copy_dn, q[6]);
      if (copy_up >= 0) st4(P + copy_up, q[6]);
    }
    __syncthreads();
    if (active) {
      const Vec4<float> vv = ld4(veff + g);
      const Vec4<float> pv = yprev ? ld4(yprev + g) : zero4;
      const float* B = P + base;
      float acc[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i] = 0.f;
      {
        // x neighbours x0 - 6 .. x0 + 9 of the own row: two 8-byte and two
        // 16-byte reads around the thread's own four values (in registers)
        const float* R = B + 6 * kPitch2 + kPad;
        const float2 l2 = *reinterpret_cast<const float2*>(R - 6);
        const Vec4<float> l4 = ld4(R - 4);
        const Vec4<float> r4 = ld4(R + 4);
        const float2 r2 = *reinterpret_cast<const float2*>(R + 8);
        float w[16];  // w[m]: the value at x0 - 6 + m
        w[0] = l2.x; w[1] = l2.y;
#pragma unroll
        for (int j = 0; j < 4; ++j) { w[2 + j] = l4.v[j]; w[6 + j] = q[6].v[j]; w[10 + j] = r4.v[j]; }
        w[14] = r2.x; w[15] = r2.y;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int k = 1; k <= 6; ++k)
            acc[i] += cx[k] * pair_d2(w[6 + i + k], w[6 + i - k], q[6].v[i]);
      }
#pragma unroll
      for (int k = 1; k <= 6; ++k) {
        const Vec4<float> up = ld4(B + (6 + k) * kPitch2 + kPad);
        const Vec4<float> dn = ld4(B + (6 - k) * kPitch2 + kPad);
#pragma unroll
        for (int i = 0; i < 4; ++i)
          acc[i] += cy[k] * pair_d2(up.v[i], dn.v[i], q[6].v[i]) +
                    cz[k] * pair_d2(q[6 + k].v[i], q[6 - k].v[i], q[6].v[i]);
      }
      Vec4<float> out;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        out.v[i] = alpha * (acc[i] + (vv.v[i] - vshift) * q[6].v[i]) +
                   (yprev ? beta * pv.v[i] : 0.f);
      st4(yout + g, out);
    }
    buf ^= 1;
#pragma unroll
    for (int d = 0; d < 12; ++d) q[d] = q[d + 1];
  }
}

// FP32 whole-plane variant with the x halo taken by DPP row rotations, for
// nx = 16 P (P = 2 or 3), 6 <= ny <= 48 and nz >= 7.  Thread t owns the P
// consecutive points x0 = P (t % 16) .. x0 + P - 1 of row y = t / 16, so the
// 16 lanes of a DPP row hold one whole x-row of the plane: the x neighbours
// x0 - 6 .. x0 + P + 5 are the values of the lanes ceil(6/P) to either side,
// fetched by row_ror (periodic in x by construction: the rotation wraps within
// the row), and only the y neighbours go through LDS (rows of nx floats with 6
// periodic copies of rows above and below the plane).  The 13-plane z-queue of
// P values per thread lives in registers; the load of the plane entering it is
// issued one step ahead; V_eff and Y_{k-1} are loaded after the barrier.  At
// 12 waves per plane and at most 80 VGPRs two plane workgroups share a CU.
template <int D>
__device__ __forceinline__ float row_lane(float v) {
  // value of lane (r + D) mod 16 of this lane's row: row_ror:n moves lane
  // (r - n) mod 16 to lane r
  constexpr int n = ((-D) % 16 + 16) % 16;
  static_assert(n != 0, "a neighbour lane");
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x120 | n, 0xF, 0xF,
                                                    false));
}

// w[m] = value at x0 - 6 + m for the points of lane offset D (m in range)
template <int P, int D>
__device__ __forceinline__ void window_from_lane(const float (&own)[P], float (&w)[P + 12]) {
#pragma unroll
  for (int j = 0; j < P; ++j) {
    constexpr int base = 6 + D * P;
    const int m = base + j;
    if (m >= 0 && m < P + 12) w[m] = row_lane<D>(own[j]);
  }
}

template <int P, int D>
__device__ __forceinline__ void window_lane_dispatch(const float (&own)[P], float (&w)[P + 12]) {
  if constexpr (D != 0) window_from_lane<P, D>(own, w);
}

template <int P, int... I>
__device__ __forceinline__ void x_window_all(const float (&own)[P], float (&w)[P + 12],
                                             std::integer_sequence<int, I...>) {
  constexpr int L = (6 + P - 1) / P;
  (window_lane_dispatch<P, I - L>(own, w), ...);
}

template <int P>
__global__ __launch_bounds__(768) __attribute__((amdgpu_waves_per_eu(6)))
void stencil_dpp_kernel(StencilArgs a) {
  static_assert(P == 2 || P == 3, "16 lanes of P points per row");
  extern __shared__ unsigned char smem_raw[];
  float* lds = reinterpret_cast<float*>(smem_raw);
  const int nx = a.nx, ny = a.ny, nz = a.nz;  // nx = 16 P, blockDim = 16 ny
  const int plane_lds = (ny + 12) * nx;
  const int pstride = nx * ny;
  const int col = blockIdx.z;
  const int z0 = blockIdx.y * a.zc;
  const int z1 = min(nz, z0 + a.zc);
  const int t = threadIdx.x;
  const int y = t >> 4;
  const int x0 = P * (t & 15);
  const int off = x0 + nx * y;

  const float* __restrict__ yin = reinterpret_cast<const float*>(a.yin) + (long)col * a.ld;
  const float* __restrict__ yprev =
      a.yprev ? reinterpret_cast<const float*>(a.yprev) + (long)col * a.ld : nullptr;
  float* yout = reinterpret_cast<float*>(a.yout) + (long)col * a.ld;
  const float* __restrict__ veff = reinterpret_cast<const float*>(a.veff);
  const float* cx = a.fcx;
  const float* cy = a.fcy;
  const float* cz = a.fcz;
  const float alpha = a.falpha, beta = a.fbeta, vshift = a.fshift;

  // LDS row y + 6 holds plane row y; rows 0..5 and ny+6..ny+11 are periodic copies
  const int own = (y + 6) * nx + x0;
  const int copy_dn = (y < 6) ? own + ny * nx : -1;
  const int copy_up = (y >= ny - 6) ? own - ny * nx : -1;

  float q[13][P];
#pragma unroll
  for (int d = 0; d < 12; ++d) {
    int zz = z0 - 6 + d;
    zz = ((zz % nz) + nz) % nz;
#pragma unroll
    for (int j = 0; j < P; ++j) q[d][j] = yin[zz * pstride + off + j];
  }
  float nxt[P];
  {
    int zn = z0 + 6; if (zn >= nz) zn -= nz;
#pragma unroll
    for (int j = 0; j < P; ++j) nxt[j] = yin[zn * pstride + off + j];
  }
  int buf = 0;
  for (int z = z0; z < z1; ++z) {
#pragma unroll
    for (int j = 0; j < P; ++j) q[12][j] = nxt[j];
    int zl = z + 7; if (zl >= nz) zl -= nz;  // nz >= 7: one wrap
    if (z + 1 < z1) {
#pragma unroll
      for (int j = 0; j < P; ++j) nxt[j] = yin[zl * pstride + off + j];
    }
    const int g = z * pstride + off;
    float* B = lds + buf * plane_lds;
#pragma unroll
    for (int j = 0; j < P; ++j) {
      B[own + j] = q[6][j];
      if (copy_dn >= 0) B[copy_dn + j] = q[6][j];
      if (copy_up >= 0) B[copy_up + j] = q[6][j];
    }
    // x window from the row's lanes (every lane of the workgroup is active)
    float w[P + 12];
#pragma unroll
    for (int j = 0; j < P; ++j) w[6 + j] = q[6][j];
    x_window_all<P>(q[6], w, std::make_integer_sequence<int, 2 * ((6 + P - 1) / P) + 1>{});
    __syncthreads();
    float vv[P], pv[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
      vv[j] = veff[g + j];
      pv[j] = yprev ? yprev[g + j] : 0.f;
    }
    float acc[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
      acc[i] = 0.f;
#pragma unroll
      for (int k = 1; k <= 6; ++k) acc[i] += cx[k] * pair_d2(w[6 + i + k], w[6 + i - k], q[6][i]);
    }
#pragma unroll
    for (int k = 1; k <= 6; ++k) {
      const float* up = B + own + k * nx;
      const float* dn = B + own - k * nx;
#pragma unroll
      for (int i = 0; i < P; ++i)
        acc[i] += cy[k] * pair_d2(up[i], dn[i], q[6][i]) +
                  cz[k] * pair_d2(q[6 + k][i], q[6 - k][i], q[6][i]);
    }
#pragma unroll
    for (int i = 0; i < P; ++i)
      yout[g + i] = alpha * (acc[i] + (vv[i] - vshift) * q[6][i]) + (yprev ? beta * pv[i] : 0.f);
    buf ^= 1;
#pragma unroll
    for (int d = 0; d < 12; ++d)
#pragma unroll
      for (int j = 0; j < P; ++j) q[d][j] = q[d + 1][j];
  }
}

// W consecutive points moved as one 16-byte vector (float x 4, double x 2).
template <typename T, int W>
struct VecW { T v[W]; };

template <typename T, int W>
__device__ __forceinline__ VecW<T, W> ldw(const T* p) {
  static_assert(sizeof(T) * W == 16 || sizeof(T) * W == 8, "one 8- or 16-byte vector");
  VecW<T, W> r;
  if constexpr (sizeof(T) == 4 && W == 2) {
    const float2 f = *reinterpret_cast<const float2*>(p);
    r.v[0] = f.x; r.v[1] = f.y;
  } else if constexpr (sizeof(T) == 4) {
    const float4 f = *reinterpret_cast<const float4*>(p);
    r.v[0] = f.x; r.v[1] = f.y; r.v[2] = f.z; r.v[3] = f.w;
  } else {
    const double2 d = *reinterpret_cast<const double2*>(p);
    r.v[0] = d.x; r.v[1] = d.y;
  }
  return r;
}

template <typename T, int W>
__device__ __forceinline__ void stw(T* p, const VecW<T, W>& r) {
  if constexpr (sizeof(T) == 4 && W == 2)
    *reinterpret_cast<float2*>(p) = make_float2(r.v[0], r.v[1]);
  else if constexpr (sizeof(T) == 4)
    *reinterpret_cast<float4*>(p) = make_float4(r.v[0], r.v[1], r.v[2], r.v[3]);
  else
    *reinterpret_cast<double2*>(p) = make_double2(r.v[0], r.v[1]);
}

// Slab variant for planes too large for one workgroup (nx % W == 0): a
// workgroup owns one column, a slab of TY rows and a chunk of z-planes.  As
// in the whole-plane kernel each thread keeps the z-queue of its W points
// in registers; the centre plane of the slab goes to LDS together with 6
// periodic halo rows above and below, which are read from memory for every
// plane (12 / TY extra reads of the input block, mostly served by L2 since
// the neighbouring slabs read them as their own rows).
// With MAXT <= 768 (3 waves per SIMD, up to 168 VGPRs) V_eff, Y_{k-1} and the
// thread's halo vector (when the 12 halo rows need at most one vector per
// thread) are loaded one plane ahead.
template <typename T, int W, int MAXT>
__global__ __launch_bounds__(MAXT) void stencil_slab_kernel(StencilArgs a) {
  extern __shared__ unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int TY = a.ty_tile;
  const int pitch = nx + 2 * kPad;
  const int rows = TY + 12;
  const int plane_lds = rows * pitch;
  const long pstride = (long)nx * ny;
  const int col = blockIdx.z;
  const int y0 = blockIdx.x * TY;
  const int ty = min(TY, ny - y0);
  const int z0 = blockIdx.y * a.zc;
  const int z1 = min(nz, z0 + a.zc);
  const int segs = nx / W;
  const int t = threadIdx.x;
  const bool active = t < segs * ty;
  const int ly = active ? t / segs : 0;       // local row
  const int x0 = active ? W * (t - ly * segs) : 0;
  const long off = x0 + (long)nx * (y0 + ly);

  const T* __restrict__ yin = reinterpret_cast<const T*>(a.yin) + (long)col * a.ld;
  const T* __restrict__ yprev =
      a.yprev ? reinterpret_cast<const T*>(a.yprev) + (long)col * a.ld : nullptr;
  T* yout = reinterpret_cast<T*>(a.yout) + (long)col * a.ld;
  const T* __restrict__ veff = reinterpret_cast<const T*>(a.veff);

  T cx[7], cy[7], cz[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) { cx[k] = (T)a.cx[k]; cy[k] = (T)a.cy[k]; cz[k] = (T)a.cz[k]; }
  const T alpha = (T)a.alpha, beta = (T)a.beta, vshift = (T)a.shift;

  const int own = (ly + 6) * pitch + kPad + x0;
  const int copy_r = (x0 < kPad) ? (ly + 6) * pitch + kPad + nx + x0 : -1;
  const int copy_l = (x0 >= nx - kPad) ? (ly + 6) * pitch + x0 - (nx - kPad) : -1;
  // halo work items: 12 rows x segs segments, spread over the workgroup
  const int halo_items = 12 * segs;

  VecW<T, W> q[13];
  VecW<T, W> zero4;
#pragma unroll
  for (int i = 0; i < W; ++i) zero4.v[i] = (T)0;
#pragma unroll
  for (int d = 0; d < 12; ++d) {
    int zz = z0 - 6 + d;
    zz = ((zz % nz) + nz) % nz;
    q[d] = active ? ldw<T, W>(yin + zz * pstride + off) : zero4;
  }
  int zn = z0 + 6; if (zn >= nz) zn -= nz;
  VecW<T, W> nxt = active ? ldw<T, W>(yin + zn * pstride + off) : zero4;
  constexpr bool PRE = MAXT <= 768;
  // the thread's halo item: row hr of the 12 halo rows, segment h_x0
  const bool one_halo = PRE && halo_items <= (int)blockDim.x;
  const bool has_halo = one_halo && t < halo_items;
  int h_base = 0, h_x0 = 0;
  long h_off = 0;
  if (has_halo) {
    const int hr = t / segs;
    h_x0 = W * (t - hr * segs);
    const int lrow = hr < 6 ? hr - 6 : ty + hr - 6;   // -6..-1, ty..ty+5
    int gy = y0 + lrow;
    gy = ((gy % ny) + ny) % ny;
    h_off = (long)nx * gy + h_x0;
    h_base = (lrow + 6) * pitch;
  }
  VecW<T, W> vv_n = zero4, pv_n = zero4, hv_n = zero4;
  if constexpr (PRE) {
    if (z0 < z1) {
      if (active) {
        vv_n = ldw<T, W>(veff + (long)z0 * pstride + off);
        if (yprev) pv_n = ldw<T, W>(yprev + (long)z0 * pstride + off);
      }
      if (has_halo) hv_n = ldw<T, W>(yin + (long)z0 * pstride + h_off);
    }
  }
  int buf = 0;
  for (int z = z0; z < z1; ++z) {
    q[12] = nxt;
    VecW<T, W> vv = vv_n, pv = pv_n;
    const VecW<T, W> hv = hv_n;
    int zl = z + 7; if (zl >= nz) zl -= nz;
    if (z + 1 < z1) {
      if (active) nxt = ldw<T, W>(yin + zl * pstride + off);
      if constexpr (PRE) {
        const long gn = (long)(z + 1) * pstride + off;
        if (active) {
          vv_n = ldw<T, W>(veff + gn);
          if (yprev) pv_n = ldw<T, W>(yprev + gn);
        }
        if (has_halo) hv_n = ldw<T, W>(yin + (long)(z + 1) * pstride + h_off);
      }
    }
    const long g = (long)z * pstride + off;
    if constexpr (!PRE) {
      if (active) {
        vv = ldw<T, W>(veff + g);
        if (yprev) pv = ldw<T, W>(yprev + g);
      }
    }
    T* P = lds + buf * plane_lds;
    if (active) {
      stw<T, W>(P + own, q[6]);
      if (copy_r >= 0) stw<T, W>(P + copy_r, q[6]);
      if (copy_l >= 0) stw<T, W>(P + copy_l, q[6]);
    }
    // halo rows of this plane: local rows -6..-1 and ty..ty+5 (periodic in y)
    if (one_halo) {
      if (has_halo) {
        stw<T, W>(P + h_base + kPad + h_x0, hv);
        if (h_x0 < kPad) stw<T, W>(P + h_base + kPad + nx + h_x0, hv);
        if (h_x0 >= nx - kPad) stw<T, W>(P + h_base + h_x0 - (nx - kPad), hv);
      }
    } else {
      for (int e = t; e < halo_items; e += blockDim.x) {
        const int hr = e / segs, hx0 = W * (e - hr * segs);
        const int lrow = hr < 6 ? hr - 6 : ty + hr - 6;
        int gy = y0 + lrow;
        gy = ((gy % ny) + ny) % ny;
        const VecW<T, W> hl = ldw<T, W>(yin + (long)z * pstride + (long)nx * gy + hx0);
        const int base = (lrow + 6) * pitch;
        stw<T, W>(P + base + kPad + hx0, hl);
        if (hx0 < kPad) stw<T, W>(P + base + kPad + nx + hx0, hl);
        if (hx0 >= nx - kPad) stw<T, W>(P + base + hx0 - (nx - kPad), hl);
      }
    }
    __syncthreads();
    if (active) {
      // x window x0-6 .. x0+W+5; the thread's own W values come from
      // registers, the six on each side from LDS
      T w[W + 12];
#pragma unroll
      for (int i = 0; i < W; ++i) w[6 + i] = q[6].v[i];
      if constexpr (W == 2) {
#pragma unroll
        for (int s2 = 0; s2 < 3; ++s2) {
          const VecW<T, 2> l = ldw<T, 2>(P + own - 6 + 2 * s2);
          const VecW<T, 2> r = ldw<T, 2>(P + own + 2 + 2 * s2);
          w[2 * s2] = l.v[0]; w[2 * s2 + 1] = l.v[1];
          w[8 + 2 * s2] = r.v[0]; w[8 + 2 * s2 + 1] = r.v[1];
        }
      } else {
        const VecW<T, 2> l2 = ldw<T, 2>(P + own - 6);
        const VecW<T, 4> l4 = ldw<T, 4>(P + own - 4);
        const VecW<T, 4> r4 = ldw<T, 4>(P + own + 4);
        const VecW<T, 2> r2 = ldw<T, 2>(P + own + 8);
        w[0] = l2.v[0]; w[1] = l2.v[1];
#pragma unroll
        for (int j = 0; j < 4; ++j) { w[2 + j] = l4.v[j]; w[10 + j] = r4.v[j]; }
        w[14] = r2.v[0]; w[15] = r2.v[1];
      }
      T acc[W];
#pragma unroll
      for (int i = 0; i < W; ++i) {
        acc[i] = 0;
#pragma unroll
        for (int k = 1; k <= 6; ++k) acc[i] += cx[k] * pair_d2(w[6 + i + k], w[6 + i - k], q[6].v[i]);
      }
#pragma unroll
      for (int k = 1; k <= 6; ++k) {
        const VecW<T, W> up = ldw<T, W>(P + own + k * pitch);
        const VecW<T, W> dn = ldw<T, W>(P + own - k * pitch);
#pragma unroll
        for (int i = 0; i < W; ++i)
          acc[i] += cy[k] * pair_d2(up.v[i], dn.v[i], q[6].v[i]) +
                    cz[k] * pair_d2(q[6 + k].v[i], q[6 - k].v[i], q[6].v[i]);
      }
      VecW<T, W> out;
#pragma unroll
      for (int i = 0; i < W; ++i)
        out.v[i] = alpha * (acc[i] + (vv.v[i] - vshift) * q[6].v[i]) +
                   (yprev ? beta * pv.v[i] : (T)0);
      stw<T, W>(yout + g, out);
    }
    buf ^= 1;
#pragma unroll
    for (int d = 0; d < 12; ++d) q[d] = q[d + 1];
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
  for (int k = 0; k < 7; ++k) {
    a.fcx[k] = (float)a.cx[k];
    a.fcy[k] = (float)a.cy[k];
    a.fcz[k] = (float)a.cz[k];
  }
  a.falpha = (float)a.alpha;
  a.fbeta = (float)a.beta;
  a.fdshift = (float)(a.diag - a.shift);
  a.fshift = (float)a.shift;
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
  const long plane = (long)c->nx * c->ny;
  // whole-plane kernel: FP32 only (the FP64 queue of 4-wide vectors costs
  // ~180 VGPRs and ran slower than the row-tile kernel)
  if (!f64 && c->nx % 4 == 0 && c->nx >= kPad && plane <= 4096 && (ld % 4) == 0) {
    // whole-plane workgroups: one per column and z-chunk
    const int threads = ((int)(plane / 4) + 63) / 64 * 64;
    // z-chunks only when there are too few columns to fill the GPU: every
    // chunk re-reads 12 planes
    int zch = ceil_div(512, (long)n_s);
    const int maxz = c->nz / 12 > 0 ? c->nz / 12 : 1;
    if (zch > maxz) zch = maxz;
    if (zch < 1) zch = 1;
    a.zc = ceil_div(c->nz, zch);
    zch = ceil_div(c->nz, a.zc);
    const size_t smem = 2 * (size_t)c->ny * (c->nx + 2 * kPad) * (f64 ? 8 : 4);
    dim3 grid(1, zch, n_s);
    // nx = 32 or 48: one x-row per DPP row of 16 lanes (P = 4 needs more
    // registers than two workgroups per CU allow)
    const int P = c->nx / 16;
    if (c->nx % 16 == 0 && (P == 2 || P == 3) && c->ny >= 6 && c->ny <= 48 && c->nz >= 7) {
      const size_t smemd = 2 * (size_t)(c->ny + 12) * c->nx * sizeof(float);
      const dim3 blk(16 * c->ny);
      if (P == 2)
        hipLaunchKernelGGL((stencil_dpp_kernel<2>), grid, blk, smemd, c->stream, a);
      else
        hipLaunchKernelGGL((stencil_dpp_kernel<3>), grid, blk, smemd, c->stream, a);
      return hipGetLastError();
    }
    const size_t smem2 = 2 * (size_t)(c->ny + 12) * kPitch2 * sizeof(float);
    if (c->nx >= kPad && c->nx + 2 * kPad <= kPitch2 && c->ny >= 6 && threads <= 640 &&
        smem2 <= 64 * 1024) {
      hipLaunchKernelGGL((stencil_plane2_kernel<640>), grid, dim3(threads), smem2, c->stream, a);
      return hipGetLastError();
    }
    if (smem <= 160 * 1024) {
      if (!(c->lds_attr_done & kAttrPlane)) {
        hipError_t e = hipFuncSetAttribute((const void*)stencil_plane_kernel<float, 640>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e == hipSuccess)
          e = hipFuncSetAttribute((const void*)stencil_plane_kernel<float, 1024>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        c->lds_attr_done |= kAttrPlane;
      }
      if (threads <= 640)
        hipLaunchKernelGGL((stencil_plane_kernel<float, 640>), grid, dim3(threads), smem, c->stream, a);
      else
        hipLaunchKernelGGL((stencil_plane_kernel<float, 1024>), grid, dim3(threads), smem, c->stream, a);
      return hipGetLastError();
    }
  }
  // slab kernel: FP32 planes larger than one workgroup (4-point vectors), and
  // every FP64 plane (2-point vectors: the FP64 whole-plane form needs too many
  // registers)
  {
    const int W = f64 ? 2 : 4;
    if (c->nx % W == 0 && (ld % W) == 0 && (f64 || plane > 4096) && c->nx <= W * 1024 / 7 &&
        c->ny >= 12) {
      const int segs = c->nx / W;
      // slabs of equal height with at most 1024 threads each
      const int max_ty = 1024 / segs;
      const int n_slabs = ceil_div(c->ny, max_ty);
      const int ty = ceil_div(c->ny, n_slabs);
      a.ty_tile = ty;
      const int threads = ((ty * segs) + 63) / 64 * 64;
      int zch = ceil_div(512, (long)n_slabs * n_s);
      const int maxz = c->nz / 12 > 0 ? c->nz / 12 : 1;
      if (zch > maxz) zch = maxz;
      if (zch < 1) zch = 1;
      a.zc = ceil_div(c->nz, zch);
      zch = ceil_div(c->nz, a.zc);
      const size_t smem = 2 * (size_t)(ty + 12) * (c->nx + 2 * kPad) * (f64 ? 8 : 4);
      if (smem <= 160 * 1024) {
        if (!(c->lds_attr_done & kAttrSlab)) {
          const void* fns[4] = {(const void*)stencil_slab_kernel<double, 2, 768>,
                                (const void*)stencil_slab_kernel<double, 2, 1024>,
                                (const void*)stencil_slab_kernel<float, 4, 768>,
                                (const void*)stencil_slab_kernel<float, 4, 1024>};
          for (const void* f : fns) {
            const hipError_t e =
                hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            if (e != hipSuccess) return e;
          }
          c->lds_attr_done |= kAttrSlab;
        }
        dim3 grid(n_slabs, zch, n_s);
        const bool small = threads <= 768;
        if (f64) {
          if (small)
            hipLaunchKernelGGL((stencil_slab_kernel<double, 2, 768>), grid, dim3(threads), smem, c->stream, a);
          else
            hipLaunchKernelGGL((stencil_slab_kernel<double, 2, 1024>), grid, dim3(threads), smem, c->stream, a);
        } else {
          if (small)
            hipLaunchKernelGGL((stencil_slab_kernel<float, 4, 768>), grid, dim3(threads), smem, c->stream, a);
          else
            hipLaunchKernelGGL((stencil_slab_kernel<float, 4, 1024>), grid, dim3(threads), smem, c->stream, a);
        }
        return hipGetLastError();
      }
    }
  }
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
