// MFMA GEMM template used by every dense contraction in libdk.
//
// One workgroup (256 threads, 4 waves in a 2x2 arrangement) computes a 64x64
// tile of C(M x N) = sum_k A(m,k) B(k,n) over a K range.  Operands are staged
// through LDS one K-slab at a time; each wave owns a 32x32 sub-tile made of
// 2x2 MFMA 16x16 blocks.  The MFMA is issued with the B slab as its row
// operand, so a lane's accumulator column is a run of 16 consecutive m: the
// column-major outputs are written in 128-byte (FP64) runs.
//
// Modes
//   kF64    FP64 MFMA 16x16x4, operands converted to double (FP32 operands are
//           widened exactly).
//   kF32    FP32 MFMA 16x16x4.
//   kBF16X3 split-BF16: every FP32 operand x = hi + lo (bf16 each) and
//           A B ~ A_hi B_hi + A_hi B_lo + A_lo B_hi, FP32 accumulation
//           (MFMA 16x16x32 bf16).  Relative error per product ~ 2^-16.
//   kBF16   plain BF16: FP32 operands rounded to bf16, one MFMA 16x16x32,
//           FP32 accumulation (~2^-8 per product).
//   kBF16X6 three-piece split x = hi + mid + lo (bf16 each); the six products
//           whose exponent sum is at most 2^-16 (lo.hi, mid.mid, hi.lo,
//           mid.hi, hi.mid, hi.hi, smallest first) leave ~2^-24 per product,
//           the FP32 level.
//   kBF16X3S, kBF16X6S  the same products with every operand element split
//           once, on its way into LDS: LDS holds the bf16 pieces (one plane
//           per piece, rows of BK + 8 values), a single slab buffer, and the
//           waves read whole 8-value fragments of each piece.  In kBF16X3 /
//           kBF16X6 LDS holds FP32 and each wave splits the fragments it
//           reads, so an element is split once per wave row or column that
//           uses it and the VALU work rivals the MFMA work.  Operands that are
//           contiguous along m (n) move as 4 x 4 blocks (four k rows of four
//           consecutive m), so that the pieces of four consecutive k are
//           written as one 8-byte LDS store.  Block masks apply; k-lists do not.
//
// Operand layouts (column-major storage, lda/ldb leading dimensions)
//   A k-contiguous: A(m,k) = A[m*lda + k]     (A^T of a column-major K x M array)
//   A m-contiguous: A(m,k) = A[k*lda + m]     (column-major M x K array)
//   B k-contiguous: B(k,n) = B[n*ldb + k]     (column-major K x N array)
//   B n-contiguous: B(k,n) = B[k*ldb + n]     (B^T of a column-major N x K array)
//
// Epilogues
//   kStore      C[m + n*ldc] = alpha*acc + beta*Cin[m + n*ldcin]   (Cin may alias C)
//   kPartial    P[s*M*N + m + n*M] = acc     (split-K partial sums of type TC; FP32
//                                           partials lose nothing for FP32 accumulators)
//   kAccumulate C[m + n*ldc] += alpha*acc
//   kRowSum     rowpart[nt*M + m] = sum_{n in tile} acc * R[m + n*ldr]
#pragma once

#include <type_traits>

#include "common.h"

namespace dk {

enum GemmMode { kF64 = 0, kF32 = 1, kBF16X3 = 2, kBF16X6 = 3, kBF16 = 4, kBF16X3S = 5,
                kBF16X6S = 6 };
constexpr bool split_store_mode(int m) { return m == kBF16X3S || m == kBF16X6S; }
constexpr bool split_bf16_mode(int m) {
  return m == kBF16X3 || m == kBF16X6 || m == kBF16 || split_store_mode(m);
}
// bf16 pieces per operand element in the split-at-store modes
constexpr int split_pieces(int m) { return m == kBF16X6S ? 3 : 2; }
enum GemmEpi { kStore = 0, kPartial = 1, kAccumulate = 2, kRowSum = 3 };
enum TileSel { kAllTiles = 0, kUpperTiles = 1, kLowerTiles = 2 };

struct GemmArgs {
  int M = 0, N = 0, K = 0;
  const void* A = nullptr;
  long lda = 0;
  const void* B = nullptr;
  long ldb = 0;
  void* C = nullptr;          // output (kStore / kAccumulate) or partial buffer (kPartial)
  long ldc = 0;
  const void* Cin = nullptr;  // kStore: source of the beta term
  long ldcin = 0;
  double alpha = 1.0, beta = 0.0;
  int splits = 1;             // split-K count (grid z)
  int k_per_split = 0;        // multiple of 64
  int tile_sel = kAllTiles;
  // block-sparse A: rows [r*kmask_mrows, (r+1)*kmask_mrows) of k-block kb are
  // all zero if kmask[r*kmask_stride + kb] == 0; a tile skips a K slab when
  // every mask row it overlaps is zero there
  const uint8_t* kmask = nullptr;
  long kmask_stride = 0;
  int kmask_blk = 64;         // K elements per mask entry (multiple of the K slab)
  int kmask_mrows = 64;       // M rows per mask row
  // indirect K (no split-K, no mask): m-tile mt runs over the K positions
  // 0 .. 4 klist_count[mt] - 1, position p standing for
  // k = 4 klist[mt * klist_stride + p / 4] + p % 4 (groups of 4 consecutive k;
  // a k >= K reads zero).  The K slab must be a multiple of 4.
  const int* klist = nullptr;
  const int* klist_count = nullptr;
  long klist_stride = 0;
  int b_upper_tri = 0;        // B(k,n) = 0 for k > n: stop the K loop at the tile's last n
  // split-at-store modes with TB = __bf16: B comes pre-split, its NP piece planes
  // b_plane elements apart, each k-contiguous (B(k,n) piece p = B[p*b_plane + n*ldb + k])
  long b_plane = 0;
  long a_plane = 0;           // the same for A (TA = __bf16; A(m,k) piece p = A[p*a_plane + m*lda + k])
  int a_lower_tri = 0;        // A(m,k) = 0 for k > m: stop the K loop at the tile's last m
  double* rowpart = nullptr;  // kRowSum output
  const void* R = nullptr;    // kRowSum elementwise partner (column-major, ldr)
  long ldr = 0;
  // batched products (grid z = batch; no split-K): operand b of the batch is
  // offset by b * stride elements (strides may be negative)
  int batch = 1;
  long bs_a = 0, bs_b = 0, bs_c = 0, bs_cin = 0;
  // tile order: 0 = m fastest (neighbours share B and the K-slab), 1 = n
  // fastest (neighbours share the A rows); xcd_groups = 1 hands each XCD a
  // contiguous range of that order, 0 keeps the hardware's round-robin
  int n_fastest = 0;
  int xcd_groups = 1;
  // symmetric results (kStore, FP64 epilogue, tile_sel = kUpperTiles, square
  // tiles): each off-diagonal tile also stores its transpose, so that only the
  // upper tiles are computed and C comes out whole and exactly symmetric
  int mirror = 0;
  // kStore: alpha is multiplied by alpha_dev[b] (device memory) for operand b of the batch
  const double* alpha_dev = nullptr;
};

// Work-item index of this workgroup.  Workgroups are dispatched round-robin
// over the 8 XCDs (each with its own L2), so linear id b runs on XCD b % 8.
// The remap gives each XCD a contiguous range of work items: tiles that share
// an operand (consecutive items) then share that XCD's L2.
__device__ __forceinline__ long xcd_work_item(long b, long total) {
  constexpr long X = 8;
  const long q = total / X, r = total % X;
  const long x = b % X, i = b / X;
  return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

template <int MODE> struct ModeTraits;
template <> struct ModeTraits<kF64> { using CT = double; using Acc = f64x4; static constexpr int BK = 16; };
template <> struct ModeTraits<kF32> { using CT = float; using Acc = f32x4; static constexpr int BK = 16; };
template <> struct ModeTraits<kBF16X3> { using CT = float; using Acc = f32x4; static constexpr int BK = 32; };
template <> struct ModeTraits<kBF16X6> { using CT = float; using Acc = f32x4; static constexpr int BK = 32; };
template <> struct ModeTraits<kBF16> { using CT = float; using Acc = f32x4; static constexpr int BK = 32; };
template <> struct ModeTraits<kBF16X3S> { using CT = float; using Acc = f32x4; static constexpr int BK = 32; };
template <> struct ModeTraits<kBF16X6S> { using CT = float; using Acc = f32x4; static constexpr int BK = 32; };

// Split-at-store slab movement (kBF16X3S / kBF16X6S).  An operand slab holds R
// rows (m or n) by BK k.  k-contiguous operands: groups of 4 consecutive k of one
// row, R*BK/1024 per thread.  Row-contiguous operands: one 4 x 4 block per
// thread (k 4*(t % (BK/4)) .., rows 4*(t / (BK/4)) ..) while t < R*BK/16, so that
// the eight lanes of a row group write one 64-byte run of each LDS row (with
// lanes walking the rows instead, every 8-byte store of a wave fell on four
// banks: 16-way conflicts, half the kernel's cycles), and the lanes of one k row
// still read whole 128-byte runs of it.
template <typename T, typename CT, int R, int BK, bool KC>
struct SplitSlab {
  static constexpr int G = KC ? (R * BK) / 1024 : 1;  // 4-element groups (KC) or one block
  static constexpr int NV = KC ? 4 * G : 16;          // values held per thread
  CT v[NV];

  // rows r0 .., k0 ..; rows < nrows, k < k_end; element (row, k) = P[row*ld + k] (KC)
  // or P[k*ld + row]
  __device__ __forceinline__ void load(const T* __restrict__ P, long ld, long r0, long nrows,
                                       long k0, long k_end, bool vec, int tid) {
    typedef T vt __attribute__((ext_vector_type(4)));
    if constexpr (KC) {
#pragma unroll
      for (int r = 0; r < G; ++r) {
        const int grp = tid + 256 * r;
        const int kc = (grp % (BK / 4)) * 4, row = grp / (BK / 4);
        const long gr = r0 + row, gk = k0 + kc;
        const T* src = P + gr * ld + gk;
        if (vec && gr < nrows && gk + 4 <= k_end) {
          const vt x = *reinterpret_cast<const vt*>(src);
#pragma unroll
          for (int j = 0; j < 4; ++j) v[4 * r + j] = (CT)x[j];
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            v[4 * r + j] = (gr < nrows && gk + j < k_end) ? (CT)src[j] : (CT)0;
        }
      }
    } else {
      if (tid >= (R * BK) / 16) return;
      const int kg = (tid % (BK / 4)) * 4, rg = (tid / (BK / 4)) * 4;
      const long gr = r0 + rg;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const long gk = k0 + kg + kk;
        const T* src = P + gk * ld + gr;
        if (vec && gk < k_end && gr + 4 <= nrows) {
          const vt x = *reinterpret_cast<const vt*>(src);
#pragma unroll
          for (int j = 0; j < 4; ++j) v[4 * kk + j] = (CT)x[j];
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            v[4 * kk + j] = (gk < k_end && gr + j < nrows) ? (CT)src[j] : (CT)0;
        }
      }
    }
  }

  // pieces of 4 consecutive k of one row -> one 8-byte store per piece plane
  template <int NP>
  __device__ static __forceinline__ void put4(__bf16* planes, int plane_elems, int off,
                                              const CT (&x)[4]) {
    typedef __bf16 b4 __attribute__((ext_vector_type(4)));
    b4 hi, mid, lo;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if constexpr (NP == 3) {
        __bf16 h, m, l;
        split3_bf16(x[j], h, m, l);
        hi[j] = h; mid[j] = m; lo[j] = l;
      } else {
        __bf16 h, l;
        split_bf16(x[j], h, l);
        hi[j] = h; lo[j] = l;
      }
    }
    *reinterpret_cast<b4*>(planes + off) = hi;
    if constexpr (NP == 3) {
      *reinterpret_cast<b4*>(planes + plane_elems + off) = mid;
      *reinterpret_cast<b4*>(planes + 2 * plane_elems + off) = lo;
    } else {
      *reinterpret_cast<b4*>(planes + plane_elems + off) = lo;
    }
  }

  // split and write the slab: piece p of (row, k) at planes[p * R * PK + row * PK + k]
  template <int NP, int PK>
  __device__ __forceinline__ void store(__bf16* planes, int tid) const {
    constexpr int PE = R * PK;
    if constexpr (KC) {
#pragma unroll
      for (int r = 0; r < G; ++r) {
        const int grp = tid + 256 * r;
        const int kc = (grp % (BK / 4)) * 4, row = grp / (BK / 4);
        const CT x[4] = {v[4 * r], v[4 * r + 1], v[4 * r + 2], v[4 * r + 3]};
        put4<NP>(planes, PE, row * PK + kc, x);
      }
    } else {
      if (tid >= (R * BK) / 16) return;
      const int kg = (tid % (BK / 4)) * 4, rg = (tid / (BK / 4)) * 4;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const CT x[4] = {v[j], v[4 + j], v[8 + j], v[12 + j]};
        put4<NP>(planes, PE, (rg + j) * PK + kg, x);
      }
    }
  }
};

// Pre-split B slab (split-at-store modes with TB = __bf16): the NP piece planes
// are copied to LDS as they are, 16-byte chunks of 8 consecutive k, NC per thread.
template <int R, int BK, int NP>
struct PreSlab {
  static constexpr int CPP = R * BK / 8;            // chunks per piece plane
  static constexpr int NC = (NP * CPP + 255) / 256;  // chunks per thread
  typedef __bf16 b8 __attribute__((ext_vector_type(8)));
  b8 v[NC];
  long plane = 0;

  __device__ __forceinline__ void load(const __bf16* __restrict__ P, long ld, long r0,
                                       long nrows, long k0, long k_end, bool vec, int tid) {
#pragma unroll
    for (int r = 0; r < NC; ++r) {
      const int c = tid + 256 * r;
      if (c >= NP * CPP) break;
      const int pc = c / CPP, w = c % CPP;
      const int row = w / (BK / 8), k8 = (w % (BK / 8)) * 8;
      const long gr = r0 + row, gk = k0 + k8;
      const __bf16* src = P + pc * plane + gr * ld + gk;
      if (vec && gr < nrows && gk + 8 <= k_end) {
        v[r] = *reinterpret_cast<const b8*>(src);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j)
          v[r][j] = (gr < nrows && gk + j < k_end) ? src[j] : (__bf16)0.0f;
      }
    }
  }

  template <int NP_, int PK>
  __device__ __forceinline__ void store(__bf16* planes, int tid) const {
    static_assert(NP_ == NP, "piece count");
#pragma unroll
    for (int r = 0; r < NC; ++r) {
      const int c = tid + 256 * r;
      if (c >= NP * CPP) break;
      const int pc = c / CPP, w = c % CPP;
      const int row = w / (BK / 8), k8 = (w % (BK / 8)) * 8;
      *reinterpret_cast<b8*>(planes + pc * R * PK + row * PK + k8) = v[r];
    }
  }
};

template <typename T> __device__ __forceinline__ double to_d(T v) { return (double)v; }

template <int MODE, typename TA, typename TB, bool AKC, bool BKC, int EPI, typename TC, int BM_,
          int BN_, int BK_>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
  using Tr = ModeTraits<MODE>;
  using CT = typename Tr::CT;
  using Acc = typename Tr::Acc;
  constexpr int BK = BK_ > 0 ? BK_ : Tr::BK;  // K-slab (a multiple of the MFMA K)
  constexpr int BM = BM_, BN = BN_;    // tile: 32, 64 or 128 per side
  constexpr int MI = BM / 32;          // 16x16 MFMA blocks per wave along m
  constexpr int NJ = BN / 32;          // ... along n
  static_assert(!split_bf16_mode(MODE) || BK % 32 == 0, "bf16 slab must hold whole 16x16x32 steps");
  // F64/F32: slab stored [k][m] (pitch BM+1); BF16X3: [m][k] (pitch BK+4), so a
  // lane's 8 consecutive k are contiguous for the 16x16x32 operand.
  constexpr bool KMAJOR = split_bf16_mode(MODE);
  constexpr int PA = KMAJOR ? (BK + 4) : (BM + 1);
  constexpr int PB = KMAJOR ? (BK + 4) : (BN + 1);
  constexpr int SLAB_A = KMAJOR ? BM * PA : BK * PA;
  constexpr int SLAB_B = KMAJOR ? BN * PB : BK * PB;
  constexpr int NA = (BM * BK) / 256;  // slab elements per thread
  constexpr int NB = (BN * BK) / 256;
  // split-at-store: NP bf16 planes per operand, rows of PKS values, one buffer
  constexpr bool SSTORE = split_store_mode(MODE);
  constexpr int NP = split_pieces(MODE);
  constexpr int PKS = BK + 8;
  constexpr size_t kLdsBytes =
      SSTORE ? (size_t)NP * (BM + BN) * PKS * 2 : (size_t)(2 * SLAB_A + 2 * SLAB_B) * sizeof(CT);
  static_assert(!SSTORE || (BK == 32 && BM % 64 == 0 && BN % 64 == 0),
                "split-at-store tiles: BK = 32, 64- or 128-row sides");
  // one LDS array for both operands, so that the epilogue may stage a whole
  // half tile through it
  __shared__ __attribute__((aligned(16))) unsigned char lds_raw[kLdsBytes];
  CT* smem_ab = reinterpret_cast<CT*>(lds_raw);
  CT* sA = smem_ab;
  CT* sB = smem_ab + 2 * SLAB_A;
  __shared__ double red[2][BM];

  // decode (m tile, n tile, split or batch) from the XCD-grouped item index
  const long gx = gridDim.x, gy = gridDim.y;
  const long total = gx * gy * (long)gridDim.z;
  const long lin = blockIdx.x + gx * (blockIdx.y + gy * (long)blockIdx.z);
  const long w = g.xcd_groups ? xcd_work_item(lin, total) : lin;
  int mt, nt;
  long zi;
  if (g.n_fastest) { nt = (int)(w % gy); mt = (int)((w / gy) % gx); zi = w / (gx * gy); }
  else { mt = (int)(w % gx); nt = (int)((w / gx) % gy); zi = w / (gx * gy); }
  const int s = (g.batch > 1) ? 0 : (int)zi;
  const long bidx = (g.batch > 1) ? zi : 0;
  if (g.tile_sel == kUpperTiles && mt > nt) return;
  if (g.tile_sel == kLowerTiles && mt < nt) return;
  const int m0 = mt * BM, n0 = nt * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * (BM / 2), wn = (wave >> 1) * (BN / 2);

  long k_begin = (long)s * g.k_per_split;
  long k_end = k_begin + g.k_per_split;
  if (k_end > g.K) k_end = g.K;
  if (g.b_upper_tri) { long lim = (long)n0 + BN; if (k_end > lim) k_end = lim; }
  if (g.a_lower_tri) { long lim = (long)m0 + BM; if (k_end > lim) k_end = lim; }
  static_assert(BK % 4 == 0, "k-list groups of 4 must not straddle a slab");
  const int* __restrict__ krow = nullptr;
  if (g.klist) {
    krow = g.klist + (long)mt * g.klist_stride;
    k_begin = 0;
    k_end = 4L * g.klist_count[mt];
  }
  // K position -> k (identity without a k-list)
  auto kmap = [&](long p) -> long { return krow ? 4L * krow[p >> 2] + (p & 3) : p; };

  const TA* __restrict__ A = (const TA*)g.A + bidx * g.bs_a;
  const TB* __restrict__ B = (const TB*)g.B + bidx * g.bs_b;

  Acc acc[NJ][MI];
#pragma unroll
  for (int j = 0; j < NJ; ++j)
#pragma unroll
    for (int i = 0; i < MI; ++i) acc[j][i] = Acc{0, 0, 0, 0};

  // first slab at or after k that the block mask does not skip
  const int mrow0 = g.kmask ? m0 / g.kmask_mrows : 0;
  const int mrow1 = g.kmask ? (((m0 + BM < g.M) ? m0 + BM : g.M) - 1) / g.kmask_mrows : 0;
  auto live = [&](long k) {
    const long kb = k / g.kmask_blk;
    for (int r = mrow0; r <= mrow1; ++r)
      if (g.kmask[(long)r * g.kmask_stride + kb]) return true;
    return false;
  };
  auto next_live = [&](long k) {
    if (g.kmask)
      while (k < k_end && !live(k)) k += BK;
    return k;
  };
  // Operand slabs move in groups of VA (VB) elements consecutive along the
  // operand's contiguous dimension: one vector load per group when the whole
  // group is in range and aligned, element loads otherwise.
  constexpr int VA = (NA % 4 == 0) ? 4 : ((NA % 2 == 0) ? 2 : 1);
  constexpr int VB = (NB % 4 == 0) ? 4 : ((NB % 2 == 0) ? 2 : 1);
  constexpr int GA = NA / VA, GB = NB / VB;
  constexpr int CA = (AKC ? BK : BM) / VA;  // groups along the contiguous dimension
  constexpr int CB = (BKC ? BK : BN) / VB;
  const bool vec_a = ((reinterpret_cast<uintptr_t>(A) % (VA * sizeof(TA))) == 0) && (g.lda % VA == 0);
  const bool vec_b = ((reinterpret_cast<uintptr_t>(B) % (VB * sizeof(TB))) == 0) && (g.ldb % VB == 0);
  CT ra[NA], rb[NB];
  auto load_slab = [&](long k0) {
#pragma unroll
    for (int r = 0; r < GA; ++r) {
      const int grp = tid + 256 * r;
      const int c = (grp % CA) * VA, o = grp / CA;
      const int m = AKC ? o : c, k = AKC ? c : o;
      const long gm = m0 + m, gk = k0 + k;
      // position gk holds k = ka; a group of VA <= 4 positions stays inside one k-list group
      const long ka = (gk < k_end) ? kmap(gk) : gk;
      const bool full = AKC ? (gm < g.M && gk + VA <= k_end && ka + VA <= g.K)
                            : (gk < k_end && ka < g.K && gm + VA <= g.M);
      const TA* src = AKC ? A + gm * g.lda + ka : A + ka * g.lda + gm;
      if (vec_a && full) {
        typedef TA vt __attribute__((ext_vector_type(VA)));
        const vt v = *reinterpret_cast<const vt*>(src);
#pragma unroll
        for (int j = 0; j < VA; ++j) ra[r * VA + j] = (CT)v[j];
      } else {
#pragma unroll
        for (int j = 0; j < VA; ++j) {
          const bool in = AKC ? (gm < g.M && gk + j < k_end && ka + j < g.K)
                              : (gk < k_end && ka < g.K && gm + j < g.M);
          ra[r * VA + j] = in ? (CT)src[j] : (CT)0;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < GB; ++r) {
      const int grp = tid + 256 * r;
      const int c = (grp % CB) * VB, o = grp / CB;
      const int n = BKC ? o : c, k = BKC ? c : o;
      const long gn = n0 + n, gk = k0 + k;
      const long ka = (gk < k_end) ? kmap(gk) : gk;
      const bool full = BKC ? (gn < g.N && gk + VB <= k_end && ka + VB <= g.K)
                            : (gk < k_end && ka < g.K && gn + VB <= g.N);
      const TB* src = BKC ? B + gn * g.ldb + ka : B + ka * g.ldb + gn;
      if (vec_b && full) {
        typedef TB vt __attribute__((ext_vector_type(VB)));
        const vt v = *reinterpret_cast<const vt*>(src);
#pragma unroll
        for (int j = 0; j < VB; ++j) rb[r * VB + j] = (CT)v[j];
      } else {
#pragma unroll
        for (int j = 0; j < VB; ++j) {
          const bool in = BKC ? (gn < g.N && gk + j < k_end && ka + j < g.K)
                              : (gk < k_end && ka < g.K && gn + j < g.N);
          rb[r * VB + j] = in ? (CT)src[j] : (CT)0;
        }
      }
    }
  };
  auto store_slab = [&](int buf) {
    CT* a = sA + buf * SLAB_A;
    CT* b = sB + buf * SLAB_B;
#pragma unroll
    for (int r = 0; r < GA; ++r) {
      const int grp = tid + 256 * r;
      const int c = (grp % CA) * VA, o = grp / CA;
#pragma unroll
      for (int j = 0; j < VA; ++j) {
        const int m = AKC ? o : c + j, k = AKC ? c + j : o;
        if (KMAJOR) a[m * PA + k] = ra[r * VA + j]; else a[k * PA + m] = ra[r * VA + j];
      }
    }
#pragma unroll
    for (int r = 0; r < GB; ++r) {
      const int grp = tid + 256 * r;
      const int c = (grp % CB) * VB, o = grp / CB;
#pragma unroll
      for (int j = 0; j < VB; ++j) {
        const int n = BKC ? o : c + j, k = BKC ? c + j : o;
        if (KMAJOR) b[n * PB + k] = rb[r * VB + j]; else b[k * PB + n] = rb[r * VB + j];
      }
    }
  };
  auto compute = [&](int buf) {
    const CT* a = sA + buf * SLAB_A;
    const CT* b = sB + buf * SLAB_B;
    if constexpr (MODE == kBF16X3) {
#pragma unroll
      for (int ks = 0; ks < BK / 32; ++ks) {
      const int kq = 32 * ks + 8 * (lane >> 4), rr = lane & 15;
      bf16x8 ah[MI], al[MI], bh[NJ], bl[NJ];
#pragma unroll
      for (int i = 0; i < MI; ++i) {
        const float* pa = &a[(wm + 16 * i + rr) * PA + kq];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          __bf16 h, l;
          split_bf16(pa[v], h, l); ah[i][v] = h; al[i][v] = l;
        }
      }
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const float* pb = &b[(wn + 16 * j + rr) * PB + kq];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          __bf16 h, l;
          split_bf16(pb[v], h, l); bh[j][v] = h; bl[j][v] = l;
        }
      }
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int i = 0; i < MI; ++i) {
          acc[j][i] = mfma_bf16(bl[j], ah[i], acc[j][i]);
          acc[j][i] = mfma_bf16(bh[j], al[i], acc[j][i]);
          acc[j][i] = mfma_bf16(bh[j], ah[i], acc[j][i]);
        }
      }
    } else if constexpr (MODE == kBF16) {
#pragma unroll
      for (int ks = 0; ks < BK / 32; ++ks) {
      const int kq = 32 * ks + 8 * (lane >> 4), rr = lane & 15;
      bf16x8 ah[MI], bh[NJ];
#pragma unroll
      for (int i = 0; i < MI; ++i) {
        const float* pa = &a[(wm + 16 * i + rr) * PA + kq];
#pragma unroll
        for (int v = 0; v < 8; ++v) ah[i][v] = to_bf16(pa[v]);
      }
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const float* pb = &b[(wn + 16 * j + rr) * PB + kq];
#pragma unroll
        for (int v = 0; v < 8; ++v) bh[j][v] = to_bf16(pb[v]);
      }
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int i = 0; i < MI; ++i) acc[j][i] = mfma_bf16(bh[j], ah[i], acc[j][i]);
      }
    } else if constexpr (MODE == kBF16X6) {
#pragma unroll
      for (int ks = 0; ks < BK / 32; ++ks) {
      const int kq = 32 * ks + 8 * (lane >> 4), rr = lane & 15;
      bf16x8 ah[MI], am[MI], al[MI], bh[NJ], bm[NJ], bl[NJ];
#pragma unroll
      for (int i = 0; i < MI; ++i) {
        const float* pa = &a[(wm + 16 * i + rr) * PA + kq];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          __bf16 h, m, l;
          split3_bf16(pa[v], h, m, l); ah[i][v] = h; am[i][v] = m; al[i][v] = l;
        }
      }
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const float* pb = &b[(wn + 16 * j + rr) * PB + kq];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          __bf16 h, m, l;
          split3_bf16(pb[v], h, m, l); bh[j][v] = h; bm[j][v] = m; bl[j][v] = l;
        }
      }
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int i = 0; i < MI; ++i) {
          acc[j][i] = mfma_bf16(bl[j], ah[i], acc[j][i]);
          acc[j][i] = mfma_bf16(bm[j], am[i], acc[j][i]);
          acc[j][i] = mfma_bf16(bh[j], al[i], acc[j][i]);
          acc[j][i] = mfma_bf16(bm[j], ah[i], acc[j][i]);
          acc[j][i] = mfma_bf16(bh[j], am[i], acc[j][i]);
          acc[j][i] = mfma_bf16(bh[j], ah[i], acc[j][i]);
        }
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < BK / 4; ++kk) {
        const int kr = kk * 4 + (lane >> 4), cidx = lane & 15;
        CT av[MI], bv[NJ];
#pragma unroll
        for (int i = 0; i < MI; ++i) av[i] = a[kr * PA + wm + 16 * i + cidx];
#pragma unroll
        for (int j = 0; j < NJ; ++j) bv[j] = b[kr * PB + wn + 16 * j + cidx];
#pragma unroll
        for (int j = 0; j < NJ; ++j)
#pragma unroll
          for (int i = 0; i < MI; ++i) {
            if constexpr (MODE == kF64) acc[j][i] = mfma_f64(bv[j], av[i], acc[j][i]);
            else acc[j][i] = mfma_f32(bv[j], av[i], acc[j][i]);
          }
      }
    }
  };

  if constexpr (SSTORE) {
    // split-at-store: one slab buffer of bf16 pieces; the next slab is loaded
    // into registers while MFMA runs the current one
    __bf16* pA = reinterpret_cast<__bf16*>(lds_raw);
    __bf16* pB = pA + NP * BM * PKS;
    constexpr bool APRE = std::is_same<TA, __bf16>::value;
    static_assert(!APRE || AKC, "pre-split A planes are k-contiguous");
    const bool va = APRE ? ((reinterpret_cast<uintptr_t>(A) % 16) == 0 && g.lda % 8 == 0 &&
                            g.a_plane % 8 == 0)
                         : ((reinterpret_cast<uintptr_t>(A) % (4 * sizeof(TA))) == 0) &&
                               (g.lda % 4 == 0);
    constexpr bool BPRE = std::is_same<TB, __bf16>::value;
    static_assert(!BPRE || BKC, "pre-split B planes are k-contiguous");
    const bool vb = BPRE ? ((reinterpret_cast<uintptr_t>(B) % 16) == 0 && g.ldb % 8 == 0 &&
                            g.b_plane % 8 == 0)
                         : ((reinterpret_cast<uintptr_t>(B) % (4 * sizeof(TB))) == 0) &&
                               (g.ldb % 4 == 0);
    std::conditional_t<APRE, PreSlab<BM, BK, NP>, SplitSlab<TA, CT, BM, BK, AKC>> xa;
    std::conditional_t<BPRE, PreSlab<BN, BK, NP>, SplitSlab<TB, CT, BN, BK, BKC>> xb;
    if constexpr (APRE) xa.plane = g.a_plane;
    if constexpr (BPRE) xb.plane = g.b_plane;
    long k0 = next_live(k_begin);
    if (k0 < k_end) {
      xa.load(A, g.lda, m0, g.M, k0, k_end, va, tid);
      xb.load(B, g.ldb, n0, g.N, k0, k_end, vb, tid);
    }
    const int kq = 8 * (lane >> 4), rr = lane & 15;
    while (k0 < k_end) {
      __syncthreads();
      xa.template store<NP, PKS>(pA, tid);
      xb.template store<NP, PKS>(pB, tid);
      __syncthreads();
      const long kn = next_live(k0 + BK);
      if (kn < k_end) {
        xa.load(A, g.lda, m0, g.M, kn, k_end, va, tid);
        xb.load(B, g.ldb, n0, g.N, kn, k_end, vb, tid);
      }
      bf16x8 af[NP][MI];
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int i = 0; i < MI; ++i)
          af[p][i] = *reinterpret_cast<const bf16x8*>(pA + p * BM * PKS + (wm + 16 * i + rr) * PKS + kq);
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        bf16x8 bf[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p)
          bf[p] = *reinterpret_cast<const bf16x8*>(pB + p * BN * PKS + (wn + 16 * j + rr) * PKS + kq);
#pragma unroll
        for (int i = 0; i < MI; ++i) {
          if constexpr (NP == 3) {
            // pieces 0 hi, 1 mid, 2 lo; smallest products first
            acc[j][i] = mfma_bf16(bf[2], af[0][i], acc[j][i]);
            acc[j][i] = mfma_bf16(bf[1], af[1][i], acc[j][i]);
            acc[j][i] = mfma_bf16(bf[0], af[2][i], acc[j][i]);
            acc[j][i] = mfma_bf16(bf[1], af[0][i], acc[j][i]);
            acc[j][i] = mfma_bf16(bf[0], af[1][i], acc[j][i]);
            acc[j][i] = mfma_bf16(bf[0], af[0][i], acc[j][i]);
          } else {
            // pieces 0 hi, 1 lo
            acc[j][i] = mfma_bf16(bf[1], af[0][i], acc[j][i]);
            acc[j][i] = mfma_bf16(bf[0], af[1][i], acc[j][i]);
            acc[j][i] = mfma_bf16(bf[0], af[0][i], acc[j][i]);
          }
        }
      }
      k0 = kn;
    }
  } else {
  // software pipeline: slab t+1 is loaded into registers while slab t runs
  long k0 = next_live(k_begin);
  if (k0 < k_end) load_slab(k0);
  int buf = 0;
  while (k0 < k_end) {
    store_slab(buf);
    __syncthreads();
    const long kn = next_live(k0 + BK);
    if (kn < k_end) load_slab(kn);
    compute(buf);
    buf ^= 1;
    k0 = kn;
  }
  }

  // ---- epilogue: lane holds m = m0+wm+16i+lane%16 and, for register q,
  // n = n0+wn+16j+4*(lane/16)+q (FP32 accumulators) or n0+wn+16j+lane/16+4q (FP64)
  const int mc = lane & 15;
  const int nq = (MODE == kF64) ? (lane >> 4) : 4 * (lane >> 4);
  constexpr int QS = (MODE == kF64) ? 4 : 1;
  if constexpr (EPI == kRowSum) {
    const TC* __restrict__ R = (const TC*)g.R;
    double part[MI];
#pragma unroll
    for (int i = 0; i < MI; ++i) {
      part[i] = 0.0;
      const long m = m0 + wm + 16 * i + mc;
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const long n = n0 + wn + 16 * j + nq + QS * q;
          if (m < g.M && n < g.N) part[i] += to_d(acc[j][i][q]) * to_d(R[m + n * g.ldr]);
        }
      part[i] += __shfl_xor(part[i], 16);
      part[i] += __shfl_xor(part[i], 32);
    }
    if (lane < 16) {
#pragma unroll
      for (int i = 0; i < MI; ++i) red[wave >> 1][wm + 16 * i + mc] = part[i];
    }
    __syncthreads();
    if (tid < BM) {
      const long m = m0 + tid;
      if (m < g.M) g.rowpart[(long)nt * g.M + m] = red[0][tid] + red[1][tid];
    }
  } else if constexpr (MODE != kF64 && std::is_same<TC, float>::value &&
                       (BN / 2) * (BM + 1) * sizeof(float) <= kLdsBytes &&
                       ((BN / 2) * BM / 4) % 256 == 0) {
    // FP32 results go out through LDS, half the tile's columns at a time, so
    // that every lane moves 4 consecutive m (16-byte accesses covering whole
    // column runs) instead of one value per column
    constexpr int SP = BM + 1, HC = BN / 2;
    float* st = reinterpret_cast<float*>(smem_ab);
    float* C = (EPI == kPartial) ? (float*)g.C + (long)s * g.M * g.N : (float*)g.C + bidx * g.bs_c;
    const long ldc = (EPI == kPartial) ? (long)g.M : g.ldc;
    const float* Cin = (EPI == kStore && g.beta != 0.0) ? (const float*)g.Cin + bidx * g.bs_cin
                                                          : nullptr;
    const bool vec_c = (reinterpret_cast<uintptr_t>(C) % 16 == 0) && (ldc % 4 == 0) &&
                       (!Cin || ((reinterpret_cast<uintptr_t>(Cin) % 16 == 0) && g.ldcin % 4 == 0));
    auto finish = [&](float c_old, float v, long m, long n) -> float {
      if constexpr (EPI == kAccumulate) return (float)((double)c_old + g.alpha * (double)v);
      else if constexpr (EPI == kPartial) return v;
      else {
        double out = g.alpha * (double)v;
        if (Cin) out += g.beta * (double)Cin[m + n * g.ldcin];
        return (float)out;
      }
    };
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      __syncthreads();
      if ((wn == 0) == (half == 0)) {
#pragma unroll
        for (int j = 0; j < NJ; ++j)
#pragma unroll
          for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q)
              st[(16 * j + nq + q) * SP + wm + 16 * i + mc] = acc[j][i][q];
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < (HC * BM / 4) / 256; ++r) {
        const int grp = tid + 256 * r;
        const int col = grp / (BM / 4), row = (grp % (BM / 4)) * 4;
        const long n = n0 + HC * half + col, m = m0 + row;
        if (n >= g.N || m >= g.M) continue;
        float* cp = C + m + n * ldc;
        const float* sp = st + col * SP + row;
        if (vec_c && m + 4 <= g.M) {
          float4 cv = make_float4(0.f, 0.f, 0.f, 0.f);
          if constexpr (EPI == kAccumulate) cv = *reinterpret_cast<const float4*>(cp);
          cv.x = finish(cv.x, sp[0], m, n);
          cv.y = finish(cv.y, sp[1], m + 1, n);
          cv.z = finish(cv.z, sp[2], m + 2, n);
          cv.w = finish(cv.w, sp[3], m + 3, n);
          *reinterpret_cast<float4*>(cp) = cv;
        } else {
          for (int e = 0; e < 4 && m + e < g.M; ++e)
            cp[e] = finish(EPI == kAccumulate ? cp[e] : 0.f, sp[e], m + e, n);
        }
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const long m = m0 + wm + 16 * i + mc;
          const long n = n0 + wn + 16 * j + nq + QS * q;
          if (m >= g.M || n >= g.N) continue;
          const double v = to_d(acc[j][i][q]);
          if constexpr (EPI == kPartial) {
            ((TC*)g.C)[(long)s * g.M * g.N + m + n * g.M] = (TC)v;
          } else if constexpr (EPI == kAccumulate) {
            TC* C = (TC*)g.C + bidx * g.bs_c;
            C[m + n * g.ldc] = (TC)(to_d(C[m + n * g.ldc]) + g.alpha * v);
          } else {
            double out = (g.alpha_dev ? g.alpha * g.alpha_dev[bidx] : g.alpha) * v;
            if (g.beta != 0.0)
              out += g.beta * to_d(((const TC*)g.Cin + bidx * g.bs_cin)[m + n * g.ldcin]);
            ((TC*)g.C + bidx * g.bs_c)[m + n * g.ldc] = (TC)out;
            if (BM == BN && g.mirror && mt != nt)
              ((TC*)g.C + bidx * g.bs_c)[n + m * g.ldc] = (TC)out;
          }
        }
  }
}

template <int MODE, typename TA, typename TB, bool AKC, bool BKC, int EPI, typename TC, int BT = 64,
          int BN_ = 0, int BK_ = 0>
inline hipError_t launch_gemm(GemmArgs g, hipStream_t st) {
  constexpr int BM = BT, BN = BN_ > 0 ? BN_ : BT;
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  // the split-at-store modes take a block mask but no k-list
  if (split_store_mode(MODE) && g.klist) return hipErrorInvalidValue;
  if (g.splits <= 0) g.splits = 1;
  if (g.k_per_split <= 0) g.k_per_split = ((g.K + 63) / 64) * 64;
  if (g.batch > 1) g.splits = 1;
  dim3 grid(ceil_div(g.M, BM), ceil_div(g.N, BN), g.batch > 1 ? g.batch : g.splits);
  hipLaunchKernelGGL((gemm_kernel<MODE, TA, TB, AKC, BKC, EPI, TC, BM, BN, BK_>), grid, dim3(256), 0,
                     st, g);
  return hipGetLastError();
}

// Longest K range (in blocks of 64) that one workgroup of an FP32-accumulating
// product (FP32 MFMA, split-BF16) sums before its partial joins the FP64
// reduction.  Long FP32 sums of terms of one sign drift: over the 884,736
// grid points of a 96^3 cell in one range the projection H_s = h^3 X^T (H X)
// came out ~1e-5 Ha too low on its diagonal, a Fermi-level shift of that size.
constexpr long kF32SplitBlocks = 64;

// Split-K bookkeeping: choose `splits` so that the grid has about `target`
// workgroups, with every split a multiple of 64 in K.
inline void plan_split_k(GemmArgs& g, int target_wgs) {
  const long tiles = (long)ceil_div(g.M, 64) * ceil_div(g.N, 64);
  long want = target_wgs / (tiles > 0 ? tiles : 1);
  if (want < 1) want = 1;
  const long kblocks = (g.K + 63) / 64;
  if (want > kblocks) want = kblocks;
  const long per = (kblocks + want - 1) / want;
  g.k_per_split = (int)(per * 64);
  g.splits = (int)((kblocks + per - 1) / per);
}

}  // namespace dk
