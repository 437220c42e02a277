// Projector integrals C = h^3 chi^T X of the nonlocal operator (Eq.
// nonlocaloperator) over the atoms' compact supports.
//
// The grid is cut into blocks of 64 consecutive points; for every block the
// 4-projector groups (one group = one atom's s and p projectors) with a nonzero
// value there are listed (projector_group_lists).  Runs of consecutive blocks
// form chunks whose union of live groups has at most 64 groups (mixed) or 32
// (FP64).  One workgroup takes one chunk and 64 columns of X: it reads each of
// its blocks of X once, multiplies it with the table values of the block's live
// groups only (MFMA on 16-projector row blocks of the chunk's union; row blocks
// with no live group in the block are skipped) and accumulates the union's rows
// in registers; at the end of the chunk they are written as one partial row
// each.  Within a workgroup the waves share the staged block of X and split
// the union's row blocks between them.  The workgroups of one chunk (one per
// 64 columns) run one after another on one XCD, so the chunk's table entries
// come from HBM once and from that XCD's L2 for the other column tiles.  A
// second kernel sums, for every projector, the partial rows of the
// chunks whose union holds its group (in chunk order: deterministic).
//
// Table values come from a compact copy built once per set of projectors: one
// entry per (block, live group) with the 4 x 64 values, pre-split into three
// bf16 pieces (mixed: x = hi + mid + lo, the six products of weight >= 2^-16
// give FP32-level products) or in FP64.  The block X is split on load.  In the
// steps of the Chebyshev filter the mixed path takes the first two pieces only
// (x = hi + lo, three products).  FP32 accumulation runs over at most 32 blocks
// (2048 points) per chunk.
#include <algorithm>
#include <vector>

#include "ctx.h"
#include "gemm.h"

namespace dk {

namespace {

constexpr int kChunkBlocks = 32;  // blocks of 64 points per chunk at most

// compact table: entry e = (block gb, group g); mixed: [3 pieces][4][64] bf16,
// FP64: [4][64] double.  One workgroup of 256 threads per entry.
template <bool MIXED>
__global__ __launch_bounds__(256) void gather_table_kernel(const double* __restrict__ chi,
                                                           long ngrid, int n_proj,
                                                           const int* __restrict__ entry_gb,
                                                           const int* __restrict__ entry_g,
                                                           void* __restrict__ tab) {
  const long e = blockIdx.x;
  const int t = threadIdx.x, p = t >> 6, pt = t & 63;
  const long x = (long)entry_gb[e] * 64 + pt;
  const int proj = 4 * entry_g[e] + p;
  const double v = (x < ngrid && proj < n_proj) ? chi[(long)proj * ngrid + x] : 0.0;
  if constexpr (MIXED) {
    __bf16 h, m, l;
    split3_bf16((float)v, h, m, l);
    __bf16* o = reinterpret_cast<__bf16*>(tab) + e * 768 + p * 64 + pt;
    o[0] = h;
    o[256] = m;
    o[512] = l;
  } else {
    reinterpret_cast<double*>(tab)[e * 256 + p * 64 + pt] = v;
  }
}

// Workgroup (chunk, 64-column tile).  Per block the 64 x 64 tile of X is
// loaded once (each thread 16 points of one column, issued one live block
// ahead), split (mixed) and staged in LDS as [piece][column][point]; wave w
// owns the union's 16-projector row blocks b = w, w + 4, ... and all four
// 16-column blocks of the tile (acc[mb][cb]), so every table entry is read by
// one wave only.  MFMA 16x16x32 bf16: A = table rows (projectors) x 32 points,
// B = 32 points x 16 columns; lane l holds D[4 (l/16) + i][l % 16].
constexpr int kXPitch = 72;  // bf16 per staged column (64 points + 8, 16-byte rows)

__device__ __forceinline__ int next_live_block(const unsigned* __restrict__ bmask, long q0, int t,
                                               int n) {
  while (t < n && bmask[q0 + t] == 0u) ++t;
  return t;
}

// NP = 3: x = hi + mid + lo, six products (FP32-level); NP = 2: x = hi + lo (the
// table's first two pieces are those of the two-piece split), three products
template <int NP>
__global__ __launch_bounds__(256) void gather_chunk_mixed_kernel(
    const float* __restrict__ X, long ld, int n_s, long ngrid, const int4* __restrict__ chunks,
    const int* __restrict__ qoff, const int* __restrict__ amap, const unsigned* __restrict__ bmask,
    const __bf16* __restrict__ tab, int vec, float* __restrict__ part, int ntiles) {
  __shared__ __attribute__((aligned(16))) __bf16 xs[NP][64][kXPitch];
  // (chunk, column tile) from an XCD-grouped work item: the column tiles of a
  // chunk run on one XCD one after another and share its table entries in L2
  const long w = xcd_work_item(blockIdx.x, (long)gridDim.x);
  const int c = (int)(w / ntiles);
  const int4 ch = chunks[c];
  const long q0 = qoff[c];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n0 = (int)(w % ntiles) * 64;
  // staging role: column n0 + lc, points 16 lp .. 16 lp + 15 of the block
  const int lc = tid >> 2, lp = tid & 3;
  const bool lcok = n0 + lc < n_s;
  const float* __restrict__ xsrc = X + (long)(lcok ? n0 + lc : 0) * ld;
  f32x4 acc[4][4];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[mb][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
  float xr[16];
  auto load_x = [&](int t) {
    const long base = ((long)ch.x + t) * 64 + 16 * lp;
    if (lcok && vec && base + 16 <= ngrid) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float4 v = *reinterpret_cast<const float4*>(xsrc + base + 4 * j);
        xr[4 * j] = v.x; xr[4 * j + 1] = v.y; xr[4 * j + 2] = v.z; xr[4 * j + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 16; ++j) xr[j] = (lcok && base + j < ngrid) ? xsrc[base + j] : 0.f;
    }
  };
  const int rrow = lane & 15;  // A row of this lane: slot 4 b + rrow / 4, projector rrow % 4
  int t = next_live_block(bmask, q0, 0, ch.y);
  if (t < ch.y) load_x(t);
  while (t < ch.y) {
    const long q = q0 + t;
    const unsigned mask = bmask[q];
    __syncthreads();  // the previous block's fragments have been read
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      bf16x8 ph, pm, pl;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        __bf16 a, b2, d;
        if constexpr (NP == 3) {
          split3_bf16(xr[8 * h + j], a, b2, d);
          pl[j] = d;
        } else {
          split_bf16(xr[8 * h + j], a, b2);
        }
        ph[j] = a; pm[j] = b2;
      }
      *reinterpret_cast<bf16x8*>(&xs[0][lc][16 * lp + 8 * h]) = ph;
      *reinterpret_cast<bf16x8*>(&xs[1][lc][16 * lp + 8 * h]) = pm;
      if constexpr (NP == 3) *reinterpret_cast<bf16x8*>(&xs[NP - 1][lc][16 * lp + 8 * h]) = pl;
    }
    __syncthreads();
    const int tn = next_live_block(bmask, q0, t + 1, ch.y);
    if (tn < ch.y) load_x(tn);  // in flight while this block runs
    const int* __restrict__ am = amap + q * 64;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      const int b = wave + 4 * mb;
      if (!((mask >> b) & 1u)) continue;
      const int e = am[4 * b + (rrow >> 2)];
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        bf16x8 ah, amd, al;
        if (e >= 0) {
          const __bf16* tp = tab + (long)e * 768 + (rrow & 3) * 64 + 32 * ks + 8 * (lane >> 4);
          ah = *reinterpret_cast<const bf16x8*>(tp);
          amd = *reinterpret_cast<const bf16x8*>(tp + 256);
          if constexpr (NP == 3) al = *reinterpret_cast<const bf16x8*>(tp + 512);
        } else {
#pragma unroll
          for (int j = 0; j < 8; ++j) { ah[j] = 0; amd[j] = 0; al[j] = 0; }
        }
        const int kp = 32 * ks + 8 * (lane >> 4);
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          const int cc = 16 * cb + (lane & 15);
          const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&xs[0][cc][kp]);
          const bf16x8 bm = *reinterpret_cast<const bf16x8*>(&xs[1][cc][kp]);
          if constexpr (NP == 3) {
            const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&xs[NP - 1][cc][kp]);
            // the six products of weight >= 2^-16, smallest first
            acc[mb][cb] = mfma_bf16(al, bh, acc[mb][cb]);
            acc[mb][cb] = mfma_bf16(amd, bm, acc[mb][cb]);
            acc[mb][cb] = mfma_bf16(ah, bl, acc[mb][cb]);
          }
          // (NP = 2: amd and bm are the lo pieces, the three products of weight >= 2^-8)
          acc[mb][cb] = mfma_bf16(amd, bh, acc[mb][cb]);
          acc[mb][cb] = mfma_bf16(ah, bm, acc[mb][cb]);
          acc[mb][cb] = mfma_bf16(ah, bh, acc[mb][cb]);
        }
      }
    }
    t = tn;
  }
  // partial rows (union offset + slot) * 4 + projector, columns contiguous
  const int rows = 4 * ch.w;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const int col = n0 + 16 * cb + (lane & 15);
      if (col >= n_s) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 16 * (wave + 4 * mb) + 4 * (lane >> 4) + i;
        if (r < rows) part[((long)4 * ch.z + r) * n_s + col] = acc[mb][cb][i];
      }
    }
}

// FP64: the same with MFMA 16x16x4 f64 (lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; register r holds D[l/16 + 4r][l%16]), 8 row blocks (wave w
// owns w and w + 4) and the tile staged as [column][point] doubles.
__global__ __launch_bounds__(256) void gather_chunk_f64_kernel(
    const double* __restrict__ X, long ld, int n_s, long ngrid, const int4* __restrict__ chunks,
    const int* __restrict__ qoff, const int* __restrict__ amap, const unsigned* __restrict__ bmask,
    const double* __restrict__ tab, double* __restrict__ part, int ntiles) {
  __shared__ double xs[64][65];
  const long w = xcd_work_item(blockIdx.x, (long)gridDim.x);
  const int c = (int)(w / ntiles);
  const int4 ch = chunks[c];
  const long q0 = qoff[c];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n0 = (int)(w % ntiles) * 64;
  const int lc = tid >> 2, lp = tid & 3;
  const bool lcok = n0 + lc < n_s;
  const double* __restrict__ xsrc = X + (long)(lcok ? n0 + lc : 0) * ld;
  f64x4 acc[2][4];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[mb][cb] = f64x4{0.0, 0.0, 0.0, 0.0};
  double xr[16];
  auto load_x = [&](int t) {
    const long base = ((long)ch.x + t) * 64 + 16 * lp;
#pragma unroll
    for (int j = 0; j < 16; ++j) xr[j] = (lcok && base + j < ngrid) ? xsrc[base + j] : 0.0;
  };
  const int rrow = lane & 15, kq = lane >> 4;
  int t = next_live_block(bmask, q0, 0, ch.y);
  if (t < ch.y) load_x(t);
  while (t < ch.y) {
    const long q = q0 + t;
    const unsigned mask = bmask[q];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) xs[lc][16 * lp + j] = xr[j];
    __syncthreads();
    const int tn = next_live_block(bmask, q0, t + 1, ch.y);
    if (tn < ch.y) load_x(tn);
    const int* __restrict__ am = amap + q * 64;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
      const int b = wave + 4 * mb;
      if (!((mask >> b) & 1u)) continue;
      const int e = am[4 * b + (rrow >> 2)];
      const double* tp = tab + (long)(e >= 0 ? e : 0) * 256 + (rrow & 3) * 64 + kq;
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        const double a = (e >= 0) ? tp[4 * s] : 0.0;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
          acc[mb][cb] = mfma_f64(a, xs[16 * cb + rrow][4 * s + kq], acc[mb][cb]);
      }
    }
    t = tn;
  }
  const int rows = 4 * ch.w;
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const int col = n0 + 16 * cb + (lane & 15);
      if (col >= n_s) continue;
#pragma unroll
      for (int r4 = 0; r4 < 4; ++r4) {
        const int r = 16 * (wave + 4 * mb) + kq + 4 * r4;
        if (r < rows) part[((long)4 * ch.z + r) * n_s + col] = acc[mb][cb][r4];
      }
    }
}

// out[proj + col n_proj] = scale rowscale[proj] sum over the chunks whose union
// holds proj's group of the partial row (occurrence * 4 + proj % 4).  Thread
// (projector of the group fastest, column); one block row per group.
template <typename PT>
__global__ __launch_bounds__(256) void gather_reduce_kernel(const PT* __restrict__ part, int n_s,
                                                            int n_proj,
                                                            const int* __restrict__ occ_off,
                                                            const int* __restrict__ occ,
                                                            double scale,
                                                            const double* __restrict__ rowscale,
                                                            double* out64, float* out32) {
  const int g = blockIdx.x;
  const int p = threadIdx.x & 3;
  const int proj = 4 * g + p;
  const int o0 = occ_off[g], o1 = occ_off[g + 1];
  const double f = proj < n_proj ? scale * (rowscale ? rowscale[proj] : 1.0) : 0.0;
  for (int col = blockIdx.y * 64 + (threadIdx.x >> 2); col < n_s; col += gridDim.y * 64) {
    double s = 0.0;
    for (int o = o0; o < o1; ++o) s += (double)part[((long)4 * occ[o] + p) * n_s + col];
    if (proj < n_proj) {
      s *= f;
      if (out64) out64[proj + (long)col * n_proj] = s;
      if (out32) out32[proj + (long)col * n_proj] = (float)s;
    }
  }
}

}  // namespace

// The compact-support form pays once most projectors are dead at a point.
// Measured per application of the mixed path: at 256 atoms (1024 projectors,
// 96^3, N_s = 4096) 24 ms against 44 ms for the dense masked product; at 32
// atoms (128 projectors, each 64-point block reaching about half of them)
// 0.31 ms against 0.13 ms.  The form is used from 65 groups (260 projectors) on.
bool use_gather_chunks(const dk_ctx* c) { return c->n_proj > 0 && (c->n_proj + 3) / 4 > 64; }

void free_gather_chunks(dk_ctx* c) {
  hipFree(c->gchunk); c->gchunk = nullptr;
  hipFree(c->gqoff); c->gqoff = nullptr;
  hipFree(c->gamap); c->gamap = nullptr;
  hipFree(c->gbmask); c->gbmask = nullptr;
  hipFree(c->gocc_off); c->gocc_off = nullptr;
  hipFree(c->gocc); c->gocc = nullptr;
  hipFree(c->gtab); c->gtab = nullptr;
  c->n_gchunks = 0;
  c->g_rows = 0;
  c->g_entries = 0;
}

// Chunks, maps and the compact table from the per-block group lists (on the
// device after projector_group_lists).  Host work: one copy of the lists and a
// linear pass over the blocks.
hipError_t build_gather_chunks(dk_ctx* c) {
  free_gather_chunks(c);
  if (!use_gather_chunks(c)) return hipSuccess;
  const bool mixed = c->precision == DK_PREC_MIXED;
  const int umax = mixed ? 64 : 32;  // groups per chunk union (16 / 8 row blocks of 16)
  const long nb = (c->ngrid + 63) / 64;
  const int ng = c->n_groups;
  std::vector<int> kc(nb), kl((size_t)nb * ng);
  hipError_t e;
  if ((e = hipMemcpyAsync(kc.data(), c->kcount, nb * sizeof(int), hipMemcpyDeviceToHost,
                          c->stream)) != hipSuccess)
    return e;
  if ((e = hipMemcpyAsync(kl.data(), c->klist, (size_t)nb * ng * sizeof(int),
                          hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return e;
  // entries (block, live group) in block order
  std::vector<long> eoff(nb + 1, 0);
  for (long b = 0; b < nb; ++b) eoff[b + 1] = eoff[b] + kc[b];
  const long n_entries = eoff[nb];
  std::vector<int> egb(n_entries > 0 ? n_entries : 1), egr(n_entries > 0 ? n_entries : 1);
  for (long b = 0; b < nb; ++b)
    for (int i = 0; i < kc[b]; ++i) {
      egb[eoff[b] + i] = (int)b;
      egr[eoff[b] + i] = kl[(size_t)b * ng + i];
    }
  // chunks: runs of blocks whose union stays within umax groups (a block with
  // more live groups than umax is split into several single-block chunks)
  std::vector<int4> chunks;
  std::vector<int> uni;        // union groups of every chunk, chunk after chunk
  std::vector<int> slot_of(ng, -1);
  int cur_begin = 0, cur_n = 0;
  long uoff = 0;
  auto close = [&]() {
    if (cur_n == 0) return;
    const int len = (int)(uni.size() - uoff);
    chunks.push_back(make_int4(cur_begin, cur_n, (int)uoff, len));
    for (size_t s = uoff; s < uni.size(); ++s) slot_of[uni[s]] = -1;
    uoff = (long)uni.size();
    cur_n = 0;
  };
  for (long b = 0; b < nb; ++b) {
    const int* live = &kl[(size_t)b * ng];
    const int n = kc[b];
    if (n > umax) {
      close();
      for (int s0 = 0; s0 < n; s0 += umax) {
        cur_begin = (int)b;
        cur_n = 1;
        for (int i = s0; i < n && i < s0 + umax; ++i) {
          slot_of[live[i]] = (int)(uni.size() - uoff);
          uni.push_back(live[i]);
        }
        close();
      }
      continue;
    }
    int fresh = 0;
    for (int i = 0; i < n; ++i) fresh += slot_of[live[i]] < 0;
    if (cur_n > 0 && ((long)(uni.size() - uoff) + fresh > umax || cur_n >= kChunkBlocks)) close();
    if (cur_n == 0) cur_begin = (int)b;
    for (int i = 0; i < n; ++i)
      if (slot_of[live[i]] < 0) {
        slot_of[live[i]] = (int)(uni.size() - uoff);
        uni.push_back(live[i]);
      }
    ++cur_n;
  }
  close();
  const int nch = (int)chunks.size();
  // per (chunk, block) row q: slot -> entry (or -1) and the live row-block bits
  std::vector<int> qoff(nch + 1, 0);
  for (int k = 0; k < nch; ++k) qoff[k + 1] = qoff[k] + chunks[k].y;
  const long nq = qoff[nch];
  std::vector<int> amap((size_t)nq * 64, -1);
  std::vector<unsigned> bmask(nq > 0 ? nq : 1, 0u);
  std::vector<int> pos(ng, -1);
  for (int k = 0; k < nch; ++k) {
    const int4 ch = chunks[k];
    for (int t = 0; t < ch.y; ++t) {
      const long b = (long)ch.x + t;
      for (int i = 0; i < kc[b]; ++i) pos[kl[(size_t)b * ng + i]] = i;
      const long q = qoff[k] + t;
      for (int s = 0; s < ch.w; ++s) {
        const int i = pos[uni[(size_t)ch.z + s]];
        if (i >= 0) {
          amap[(size_t)q * 64 + s] = (int)(eoff[b] + i);
          bmask[q] |= 1u << (s / 4);
        }
      }
      for (int i = 0; i < kc[b]; ++i) pos[kl[(size_t)b * ng + i]] = -1;
    }
  }
  // occurrences of every group among the unions, in chunk order
  std::vector<int> occ_off(ng + 1, 0);
  for (size_t s = 0; s < uni.size(); ++s) ++occ_off[uni[s] + 1];
  for (int g = 0; g < ng; ++g) occ_off[g + 1] += occ_off[g];
  std::vector<int> occ(uni.size() > 0 ? uni.size() : 1), fill(occ_off.begin(), occ_off.end() - 1);
  for (size_t s = 0; s < uni.size(); ++s) occ[fill[uni[s]]++] = (int)s;
  // upload
  auto up = [&](void** dst, const void* src, size_t bytes) -> hipError_t {
    hipError_t r = hipMalloc(dst, bytes > 0 ? bytes : 16);
    if (r != hipSuccess) return r;
    if (bytes == 0) return hipSuccess;
    return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
  };
  if ((e = up((void**)&c->gchunk, chunks.data(), chunks.size() * sizeof(int4))) != hipSuccess) return e;
  if ((e = up((void**)&c->gqoff, qoff.data(), qoff.size() * sizeof(int))) != hipSuccess) return e;
  if ((e = up((void**)&c->gamap, amap.data(), amap.size() * sizeof(int))) != hipSuccess) return e;
  if ((e = up((void**)&c->gbmask, bmask.data(), bmask.size() * sizeof(unsigned))) != hipSuccess) return e;
  if ((e = up((void**)&c->gocc_off, occ_off.data(), occ_off.size() * sizeof(int))) != hipSuccess) return e;
  if ((e = up((void**)&c->gocc, occ.data(), occ.size() * sizeof(int))) != hipSuccess) return e;
  int *d_egb = nullptr, *d_egr = nullptr;
  if ((e = up((void**)&d_egb, egb.data(), n_entries * sizeof(int))) != hipSuccess) return e;
  if ((e = up((void**)&d_egr, egr.data(), n_entries * sizeof(int))) != hipSuccess) {
    hipFree(d_egb);
    return e;
  }
  const size_t per = mixed ? 768 * sizeof(__bf16) : 256 * sizeof(double);
  if ((e = hipMalloc(&c->gtab, (n_entries > 0 ? n_entries : 1) * per)) == hipSuccess && n_entries > 0) {
    if (mixed)
      hipLaunchKernelGGL(gather_table_kernel<true>, dim3((unsigned)n_entries), dim3(256), 0,
                         c->stream, c->chi64, c->ngrid, c->n_proj, d_egb, d_egr, c->gtab);
    else
      hipLaunchKernelGGL(gather_table_kernel<false>, dim3((unsigned)n_entries), dim3(256), 0,
                         c->stream, c->chi64, c->ngrid, c->n_proj, d_egb, d_egr, c->gtab);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  }
  hipFree(d_egb);
  hipFree(d_egr);
  if (e != hipSuccess) return e;
  c->n_gchunks = nch;
  c->g_rows = (long)uni.size();
  c->g_entries = n_entries;
  return hipSuccess;
}

size_t gather_chunks_ws_bytes(const dk_ctx* c, int n_s) {
  const size_t elem = c->precision == DK_PREC_MIXED ? sizeof(float) : sizeof(double);
  return ws_slice((size_t)4 * (c->g_rows > 0 ? c->g_rows : 1) * n_s * elem);
}

// out = scale * rowscale_p * h^3-free sum chi_p^T X over the compact supports
// (N_proj x n_s, column-major; FP64 and/or FP32)
hipError_t gather_chunks(dk_ctx* c, const void* x, long ld, int n_s, double scale,
                         const double* rowscale, double* out64, float* out32, void* ws,
                         bool two_piece) {
  if (c->n_gchunks == 0) return hipSuccess;
  const int ntiles = ceil_div(n_s, 64);
  const dim3 grid((unsigned)((long)c->n_gchunks * ntiles));
  const dim3 rgrid(c->n_groups, std::min(ceil_div(n_s, 64), 64));
  if (c->precision == DK_PREC_MIXED) {
    const int vec = ((reinterpret_cast<uintptr_t>(x) % 16) == 0 && ld % 4 == 0) ? 1 : 0;
    if (two_piece)
      hipLaunchKernelGGL(gather_chunk_mixed_kernel<2>, grid, dim3(256), 0, c->stream,
                         (const float*)x, ld, n_s, c->ngrid, (const int4*)c->gchunk, c->gqoff,
                         c->gamap, c->gbmask, (const __bf16*)c->gtab, vec, (float*)ws, ntiles);
    else
      hipLaunchKernelGGL(gather_chunk_mixed_kernel<3>, grid, dim3(256), 0, c->stream,
                         (const float*)x, ld, n_s, c->ngrid, (const int4*)c->gchunk, c->gqoff,
                         c->gamap, c->gbmask, (const __bf16*)c->gtab, vec, (float*)ws, ntiles);
    hipLaunchKernelGGL(gather_reduce_kernel<float>, rgrid, dim3(256), 0, c->stream,
                       (const float*)ws, n_s, c->n_proj, c->gocc_off, c->gocc, scale, rowscale,
                       out64, out32);
  } else {
    hipLaunchKernelGGL(gather_chunk_f64_kernel, grid, dim3(256), 0, c->stream, (const double*)x,
                       ld, n_s, c->ngrid, (const int4*)c->gchunk, c->gqoff, c->gamap, c->gbmask,
                       (const double*)c->gtab, (double*)ws, ntiles);
    hipLaunchKernelGGL(gather_reduce_kernel<double>, rgrid, dim3(256), 0, c->stream,
                       (const double*)ws, n_s, c->n_proj, c->gocc_off, c->gocc, scale, rowscale,
                       out64, out32);
  }
  return hipGetLastError();
}

}  // namespace dk
