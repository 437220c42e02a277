// Kleinman-Bylander nonlocal operator on a block (Eq. nonlocaloperator):
//
//   Y += alpha * sum_p gamma_p chi_p (h^3 chi_p^T X)
//
// as two MFMA contractions:
//   1. C = h^3 chi^T X              (N_proj x N_s; split over the grid, partials)
//   2. C <- alpha gamma_p C (row scale, FP64 reduction of the partials)
//   3. Y += chi C                   (accumulated into the block)
// Up to 64 atom groups the integrals run over the dense N_grid x N_proj table
// and skip 64-point grid blocks where a 64-projector tile is zero; beyond, over
// the atoms' compact supports (gather.hip).  The scatter runs each 64-point
// tile over the 4-projector groups that reach it.  Mixed path: FP32 tables and
// scatter; split-BF16 integrals (three pieces, two in the filter steps).
#include <type_traits>

#include "ctx.h"
#include "gemm.h"

namespace dk {

namespace {

// out[e] = scale * rowscale[e % m] * sum_s part[s * mn + e].  A block owns 64
// consecutive entries; its four waves sum interleaved quarters of the splits
// (two independent chains each), then combine in LDS.
template <typename PT>
__global__ __launch_bounds__(256) void reduce_rows_kernel(const PT* __restrict__ part, int splits,
                                                          long mn, int m,
                                                          const double* __restrict__ rowscale,
                                                          double scale, double* out64,
                                                          float* out32) {
  __shared__ double sh[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (long e0 = blockIdx.x * 64L; e0 < mn; e0 += (long)gridDim.x * 64) {
    const long e = e0 + lane;
    double s0 = 0.0, s1 = 0.0;
    if (e < mn) {
      int k = wv;
      for (; k + 4 < splits; k += 8) {
        s0 += (double)part[(long)k * mn + e];
        s1 += (double)part[(long)(k + 4) * mn + e];
      }
      for (; k < splits; k += 4) s0 += (double)part[(long)k * mn + e];
    }
    sh[wv][lane] = s0 + s1;
    __syncthreads();
    if (wv == 0 && e < mn) {
      double s = (sh[0][lane] + sh[1][lane]) + (sh[2][lane] + sh[3][lane]);
      s *= scale * (rowscale ? rowscale[(int)(e % m)] : 1.0);
      if (out64) out64[e] = s;
      if (out32) out32[e] = (float)s;
    }
    __syncthreads();
  }
}

// Split count of the projector-integral product: about 2048 workgroups of
// 128x64 tiles (latency hiding needs many workgroups per CU: measured 0.27 ->
// 0.16 ms at 110592 x 512 x 128 when going from ~40 to ~160 splits).  The
// 128x128 tiles of the three-piece split-BF16 form (wide) take about 2048
// workgroups for the H X integrals, with at least 13 blocks of 64 points per
// split so that the partials stay a small fraction of the block read (per
// application: 135 -> 122 us at 110592 x 512 x 128, 5.4 -> 5.2 ms at
// 373248 x 2048 x 432), and about 1024 for the force integrals (512 rows).
int gather_splits_m(const dk_ctx* c, int m, int n_s, bool wide, bool forces) {
  const long tiles = (long)ceil_div(m, 128) * ceil_div(n_s, wide ? 128 : 64);
  const long kblocks = (c->ngrid + 63) / 64;
  long want = ((wide && forces) ? 1024 : 2048) / (tiles > 0 ? tiles : 1);
  if (wide && !forces && want > kblocks / 13) want = kblocks / 13;
  if (c->precision == DK_PREC_MIXED) {
    // FP32 accumulation: at most kF32SplitBlocks blocks per split
    const long least = (kblocks + kF32SplitBlocks - 1) / kF32SplitBlocks;
    if (want < least) want = least;
  }
  if (want > kblocks) want = kblocks;
  if (want < 1) want = 1;
  const long per = (kblocks + want - 1) / want;
  return (int)((kblocks + per - 1) / per);
}

// The mixed path forms h^3 chi^T X with the three-piece split-BF16 MFMA
// (FP32-level products, ~30% faster than FP32 MFMA at these shapes) once
// there are more than 64 projectors, two pieces in the Chebyshev filter's
// steps; smaller tables keep 64-row FP32 tiles.
bool gather_wide(const dk_ctx* c, int m) { return c->precision == DK_PREC_MIXED && m > 64; }

// out (N_proj x n_s FP64) = scale * rowscale_p * table^T X, with the table an
// N_grid x N_proj column-major array of type TT and X of type TX.
// partials of an FP32-accumulating product are stored in FP32 (lossless)
template <int MODE> using PartialT = typename std::conditional<MODE == kF64, double, float>::type;

// pieces (mixed, wide): the table's bf16 pieces (build_table_pieces), used in
// place of splitting the table in every column tile
// two_piece (with pieces): the first two pieces only, x = hi + lo, and the three
// products of weight >= 2^-8 (relative error ~2^-17 per product)
template <int MODE, typename TT, typename TX>
hipError_t table_transpose_product(dk_ctx* c, const TT* table, const void* x, long ld, int n_s,
                                   double scale, const double* rowscale, double* out64,
                                   float* out32, void* part_raw, bool use_mask, int m_rows = 0,
                                   const void* pieces = nullptr, bool two_piece = false) {
  using PT = PartialT<MODE>;
  PT* part = (PT*)part_raw;
  GemmArgs g;
  g.M = m_rows > 0 ? m_rows : c->n_proj;
  g.N = n_s;
  g.K = (int)c->ngrid;
  g.A = table;
  g.lda = c->ngrid;
  g.B = x;
  g.ldb = ld;
  g.C = part;
  const bool wide = (MODE == kF32) && g.M > 64;
  {
    const int want = gather_splits_m(c, g.M, n_s, wide, m_rows > 0);
    const long kblocks = (g.K + 63) / 64;
    const long per = (kblocks + want - 1) / want;
    g.k_per_split = (int)(per * 64);
    g.splits = (int)((kblocks + per - 1) / per);
  }
  if (use_mask) {
    g.kmask = c->mask_t;
    g.kmask_stride = c->mask_t_stride;
    g.kmask_blk = 64;
    g.kmask_mrows = 64;  // mask rows are 64-projector tiles, whatever the GEMM tile
  }
  // with more than 64 projectors one 128-row tile reads each block slab once;
  // FP32 slabs of 32 give 128-byte row segments
  constexpr int BKG = (MODE == kF32) ? 32 : 0;
  hipError_t e;
  if constexpr (MODE == kF32) {
    if (wide && pieces) {
      g.A = pieces;
      g.lda = split_planes_ld((int)c->ngrid);
      g.a_plane = (long)g.M * g.lda;
      e = two_piece
              ? launch_gemm<kBF16X3S, __bf16, TX, true, true, kPartial, PT, 128, 128, 32>(g, c->stream)
              : launch_gemm<kBF16X6S, __bf16, TX, true, true, kPartial, PT, 128, 128, 32>(g, c->stream);
    } else {
      e = wide ? launch_gemm<kBF16X6S, TT, TX, true, true, kPartial, PT, 128, 128, 32>(g, c->stream)
               : launch_gemm<MODE, TT, TX, true, true, kPartial, PT, 64, 64, BKG>(g, c->stream);
    }
  } else {
    e = (g.M > 64) ? launch_gemm<MODE, TT, TX, true, true, kPartial, PT, 128, 64, BKG>(g, c->stream)
                   : launch_gemm<MODE, TT, TX, true, true, kPartial, PT, 64, 64, BKG>(g, c->stream);
  }
  if (e != hipSuccess) return e;
  const long mn = (long)g.M * g.N;
  int blocks = (int)((mn + 63) / 64);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(reduce_rows_kernel<PT>, dim3(blocks), dim3(256), 0, c->stream, part, g.splits,
                     mn, g.M, rowscale, scale, out64, out32);
  return hipGetLastError();
}

// One wave per 64-point block: lane i looks at point 64 gb + i of the four
// projectors of each group; the groups where any lane sees a nonzero are
// listed in increasing order.
__global__ __launch_bounds__(256) void group_lists_kernel(const double* __restrict__ chi, long ng,
                                                          int n_proj, long gblocks, int n_groups,
                                                          int* __restrict__ list,
                                                          int* __restrict__ count) {
  const int lane = threadIdx.x & 63;
  const long nwaves = ((long)gridDim.x * blockDim.x) >> 6;
  for (long gb = (blockIdx.x * (long)blockDim.x + threadIdx.x) >> 6; gb < gblocks; gb += nwaves) {
    const long x = gb * 64 + lane;
    int cnt = 0;
    for (int gr = 0; gr < n_groups; ++gr) {
      bool nz = false;
      if (x < ng)
        for (int p = 4 * gr; p < 4 * gr + 4 && p < n_proj; ++p)
          nz = nz || chi[(long)p * ng + x] != 0.0;
      if (__any(nz)) {
        if (lane == 0) list[gb * n_groups + cnt] = gr;
        ++cnt;
      }
    }
    if (lane == 0) count[gb] = cnt;
  }
}

}  // namespace

hipError_t projector_group_lists(dk_ctx* c) {
  if (c->n_proj == 0) return hipSuccess;
  const long gblocks = (c->ngrid + 63) / 64;
  const int n_groups = (c->n_proj + 3) / 4;
  if (!c->klist || c->n_groups != n_groups) {
    hipFree(c->klist);
    hipFree(c->kcount);
    c->klist = nullptr;
    c->kcount = nullptr;
    hipError_t e = hipMalloc(&c->klist, (size_t)gblocks * n_groups * sizeof(int));
    if (e != hipSuccess) return e;
    if ((e = hipMalloc(&c->kcount, (size_t)gblocks * sizeof(int))) != hipSuccess) return e;
    c->n_groups = n_groups;
  }
  long blocks = (gblocks * 64 + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(group_lists_kernel, dim3((int)blocks), dim3(256), 0, c->stream, c->chi64,
                     c->ngrid, c->n_proj, gblocks, n_groups, c->klist, c->kcount);
  return hipGetLastError();
}

static size_t gather_partial_bytes(const dk_ctx* c, int n_s) {
  if (use_gather_chunks(c)) return gather_chunks_ws_bytes(c, n_s);
  const int splits = gather_splits_m(c, c->n_proj, n_s, gather_wide(c, c->n_proj), false);
  const size_t elem = c->precision == DK_PREC_FP64 ? sizeof(double) : sizeof(float);
  return ws_slice((size_t)splits * c->n_proj * n_s * elem);
}

size_t nonlocal_ws_bytes(const dk_ctx* c, int n_s) {
  if (c->n_proj == 0) return 0;
  const size_t mn = (size_t)c->n_proj * n_s;
  return gather_partial_bytes(c, n_s) + ws_slice(mn * sizeof(double)) +
         ws_slice(mn * sizeof(float));
}

// Mixed path, dense integrals (at most 64 atom groups) over more than 64
// projectors: the table is split into its three bf16 pieces once per set of
// tables instead of once per column tile and application.
hipError_t build_table_pieces(dk_ctx* c) {
  const bool want = c->precision == DK_PREC_MIXED && c->n_proj > 0 &&
                    gather_wide(c, c->n_proj) && !use_gather_chunks(c);
  const size_t bytes = want ? split_planes_bytes((int)c->ngrid, c->n_proj, 3) : 0;
  if (bytes != c->chi_pieces_bytes) {
    hipFree(c->chi_pieces);
    c->chi_pieces = nullptr;
    c->chi_pieces_bytes = 0;
    if (bytes) {
      const hipError_t e = hipMalloc(&c->chi_pieces, bytes);
      if (e != hipSuccess) return e;
      c->chi_pieces_bytes = bytes;
    }
  }
  if (!want) return hipSuccess;
  return split_planes(c, c->chi64, 1, c->ngrid, (int)c->ngrid, c->n_proj, 3, c->chi_pieces);
}

// The nonlocal term in two calls: the integrals C = alpha gamma h^3 chi^T X into
// the workspace, and the scatter Y += chi C from it (callers run the stencil
// between them).
hipError_t nonlocal_integrals(dk_ctx* c, const void* x, long ld, int n_s, double alpha, void* ws,
                              bool subspace) {
  if (c->n_proj == 0 || n_s <= 0) return hipSuccess;
  const size_t mn = (size_t)c->n_proj * n_s;
  WsCursor cur((char*)ws, nonlocal_ws_bytes(c, n_s));
  char* part = cur.take<char>(gather_partial_bytes(c, n_s));
  double* c64 = cur.take<double>(mn);
  float* c32 = cur.take<float>(mn);
  if (!cur.ok) return hipErrorInvalidValue;
  KTimer kt(c, DK_K_NL_GATHER);
  if (c->precision == DK_PREC_FP64)
    return use_gather_chunks(c)
               ? gather_chunks(c, x, ld, n_s, c->dv * alpha, c->gamma_dev, c64, nullptr, part)
               : table_transpose_product<kF64, double, double>(c, c->chi64, x, ld, n_s,
                                                               c->dv * alpha, c->gamma_dev, c64,
                                                               nullptr, part, true);
  return use_gather_chunks(c)
             ? gather_chunks(c, x, ld, n_s, c->dv * alpha, c->gamma_dev, nullptr, c32, part,
                             subspace)
             : table_transpose_product<kF32, float, float>(c, c->chi32, x, ld, n_s, c->dv * alpha,
                                                           c->gamma_dev, nullptr, c32, part, true,
                                                           0, c->chi_pieces, subspace);
}

hipError_t nonlocal_scatter(dk_ctx* c, void* y, long ld, int n_s, void* ws) {
  if (c->n_proj == 0 || n_s <= 0) return hipSuccess;
  const size_t mn = (size_t)c->n_proj * n_s;
  WsCursor cur((char*)ws, nonlocal_ws_bytes(c, n_s));
  cur.take<char>(gather_partial_bytes(c, n_s));
  double* c64 = cur.take<double>(mn);
  float* c32 = cur.take<float>(mn);
  if (!cur.ok) return hipErrorInvalidValue;
  GemmArgs g;
  g.M = (int)c->ngrid;
  g.N = n_s;
  g.K = c->n_proj;
  g.lda = c->ngrid;
  g.ldb = c->n_proj;
  g.C = y;
  g.ldc = ld;
  g.alpha = 1.0;
  // each 64-point tile runs only over the 4-projector groups that reach it
  g.klist = c->klist;
  g.klist_count = c->kcount;
  g.klist_stride = c->n_groups;
  g.xcd_groups = 0;  // measured faster in plain round-robin order
  KTimer kt(c, DK_K_NL_SCATTER);
  if (c->precision == DK_PREC_FP64) {
    g.A = c->chi64;
    g.B = c64;
    return launch_gemm<kF64, double, double, false, true, kAccumulate, double>(g, c->stream);
  }
  g.A = c->chi32;
  g.B = c32;
  // (64 x 256 tiles, reading each tile's table values once per 256 columns,
  // were slower at 884736 x 4096: 389 against 362 ms per SCF iteration)
  return launch_gemm<kF32, float, float, false, true, kAccumulate, float>(g, c->stream);
}

size_t projector_integrals_ws_bytes(const dk_ctx* c, int n_s, int m_rows) {
  const size_t elem = c->precision == DK_PREC_FP64 ? sizeof(double) : sizeof(float);
  return ws_slice((size_t)gather_splits_m(c, m_rows, n_s, gather_wide(c, m_rows), true) * m_rows *
                  n_s * elem);
}

// out (m_rows x n_s FP64) = scale * table^T X for an FP64 N_grid x m_rows table
// (projector values and/or their finite-difference gradients); X in the
// context precision.  The mixed path forms the products like the projector
// integrals of H X (FP32 table values, FP32-level products, FP32 partials).
hipError_t projector_integrals(dk_ctx* c, const void* x, long ld, int n_s, const void* table,
                               int m_rows, double scale, double* out, void* ws) {
  if (m_rows == 0 || n_s <= 0) return hipSuccess;
  if (c->precision == DK_PREC_FP64) {
    const int splits = gather_splits_m(c, m_rows, n_s, false, true);
    WsCursor cur((char*)ws, projector_integrals_ws_bytes(c, n_s, m_rows));
    double* part = cur.take<double>((size_t)splits * m_rows * n_s);
    if (!cur.ok) return hipErrorInvalidValue;
    return table_transpose_product<kF64, double, double>(c, (const double*)table, x, ld, n_s,
                                                         scale, nullptr, out, nullptr, part,
                                                         false, m_rows);
  }
  const int splits = gather_splits_m(c, m_rows, n_s, gather_wide(c, m_rows), true);
  WsCursor cur((char*)ws, projector_integrals_ws_bytes(c, n_s, m_rows));
  float* part = cur.take<float>((size_t)splits * m_rows * n_s);
  if (!cur.ok) return hipErrorInvalidValue;
  return table_transpose_product<kF32, double, float>(c, (const double*)table, x, ld, n_s, scale,
                                                      nullptr, out, nullptr, part, false, m_rows);
}

}  // namespace dk
