// Complex GEMM on the CDNA matrix cores, used for the trailing update of the
// blocked right-looking LU (arXiv:2505.09545, Sec. "Numerical solution": the
// coupled system is solved by LU decomposition), for the blocked triangular
// solves and for the FP64 residual of iterative refinement.
//
// Storage: column-major, interleaved complex.  Viewed as real matrices, an
// m x k complex A is a 2m x k real matrix whose rows alternate (re, im).  The
// product C = A B is then the real product  C^ = A~ B^  with
//   A~ (2m x 2k):  each complex a becomes the 2x2 block [[a_r, -a_i], [a_i, a_r]]
//   B^ (2k x n) :  the real view of B (rows alternate re, im)
// so one real 16x16x4 MFMA covers 8 complex rows x 16 complex columns x 2
// complex k, and the accumulators already hold interleaved complex C.  The
// expansion of A costs one LDS load per lane (the lane picks re or im and the
// sign from its (row, k) parity); no extra storage and no 3M/4M bookkeeping.
//
// Tiles: 2 x 2 waves per 256-thread workgroup, each wave WM x WN MFMA blocks of
// 16 real rows x 16 columns, BK complex k per stage, double-buffered LDS:
//   64 complex rows x 64 columns (WM 4, WN 2) for launches that fill the chip
//     (the bulk of the trailing update, the FP64 residual), 4 complex k per
//     stage for one system's products, 8 for batched launches;
//   32 x 32 x 8 (WM 2, WN 1) for launches of fewer than two 64 x 64 tiles per
//     CU (look-ahead update, U12 blocks, solve steps): four times the
//     workgroups, for products whose time is set by latency rather than by the
//     matrix cores.  Measured on the 66-RHS solves: 8 complex k per stage
//     11.6 ms, 16: 12.4, 32: 14.7, 64: 17.6 (the smaller stage leaves more
//     workgroups resident per CU); wider tiles over all 66 columns: 16.5.
//     One system's products over 64 <= k <= 128 (16 complex k per stage)
//     load their whole k range into registers before the first stage, so a
//     launch waits for memory once instead of once per stage (FP32+IR step
//     72.6 -> 72.0 ms; FP64 takes it in two halves of 64, whose registers
//     would otherwise spill).
// Per thread and stage the big tile loads one (4 k) or two (8 k) complex
// elements of A and as many of B, the small one one of each.
// Workgroups are remapped so that each of the 8 XCDs works on a contiguous
// range of tiles (their operands then share that XCD's L2), taken in the
// grouped order of grouped_tile.
#include "gdm_common.hpp"
#include "gdm_kernels.hpp"

namespace gdm {

// FP32 trailing updates with the 64 x 64 tile by 3M products (1) or the
// expanded 4M form (0)
#ifndef GEMM_UPDATE_3M
#define GEMM_UPDATE_3M 1
#endif
// small-tile products of one system over 64 <= k <= 128 with the whole k range
// prefetched into registers (1) or the two-buffer k loop (0)
// B tile of the 3M update stored with a column swizzle (1) or plainly (0)
#ifndef GEMM3M_BSWZ
#define GEMM3M_BSWZ 1
#endif
#ifndef GEMM_SMALL_PREFETCH
#define GEMM_SMALL_PREFETCH 1
#endif

template <typename T> struct acc_of;
template <> struct acc_of<double> { using type = v4d; };
template <> struct acc_of<float> { using type = v4f; };

__device__ inline v4d mfma16(double a, double b, v4d c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
__device__ inline v4f mfma16(float a, float b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

// Operand masks (used by the triangular-block solves): an element (r, c) of a
// masked square block is kept iff the relation holds, else read as zero.
__device__ inline bool mask_keep(int kind, int64_t r, int64_t c) {
  switch (kind) {
    case GEMM_MASK_STRICT_LOWER: return r > c;
    case GEMM_MASK_UPPER: return r <= c;
    case GEMM_MASK_LOWER: return r >= c;
    case GEMM_MASK_STRICT_UPPER: return r < c;
    default: return true;
  }
}

// Order of the output tiles: the tile columns are cut into NBLK blocks (8 or
// 16: one or two per XCD range of the remap) and each block is walked by
// groups of GM tile rows, a group covering all of the block's columns before
// the next.  An XCD then keeps one block's B strips and the current group's A
// strips in its L2 together (at k = 128 a 64-wide strip is 64 KB in FP32, 128
// KB in FP64), so an A strip comes from memory about once per block instead of
// once per tile column.  Measured on the n = 12 000 FP32 factorisation: HBM
// fetch of the bulk update 598 -> 267 MiB per launch, factorisation 59.1 ->
// 58.45 ms.
template <int GM, int NBLK>
__device__ inline void grouped_tile(int t, int tiles_m, int tiles, int& tm, int& tn) {
  const int tiles_n = tiles / tiles_m;
  const int cbw = (tiles_n + NBLK - 1) / NBLK;
  const int per_blk = tiles_m * cbw;
  const int blk = t / per_blk;
  const int within = t - blk * per_blk;
  const int cols = min(cbw, tiles_n - blk * cbw);
  const int per_grp = GM * cols;
  const int grp = within / per_grp;
  const int w2 = within - grp * per_grp;
  const int rows = min(GM, tiles_m - grp * GM);
  tm = grp * GM + w2 % rows;
  tn = blk * cbw + w2 / rows;
}

template <typename T, int MODE, int TRANSA, int ROLE, int WM, int WN, int BK, bool CB, int NST = 0>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) cgemm_kernel(int64_t m, int64_t n, int64_t k, const cplx<T>* __restrict__ A,
                                                     int64_t lda, const cplx<T>* __restrict__ B, int64_t ldb,
                                                     cplx<T>* __restrict__ C, int64_t ldc, int tiles_m, int tiles,
                                                     GemmMask mk, int64_t sA, int64_t sB, int64_t sC) {
  using CT = cplx<T>;
  constexpr int BM = 16 * WM;  // complex rows per tile
  constexpr int BN = 32 * WN;  // columns per tile
  constexpr int AL = BM * BK / 256, BL = BK * BN / 256;  // elements per thread and stage
  static_assert(AL * 256 == BM * BK && BL * 256 == BK * BN && BK % 2 == 0, "tile shape");
  // batch of independent products: blockIdx.y selects the item
  A += (int64_t)blockIdx.y * sA;
  B += (int64_t)blockIdx.y * sB;
  C += (int64_t)blockIdx.y * sC;
  using ACC = typename acc_of<T>::type;
  // A: rows padded by 16 elements (the MFMA operand reads of one instruction
  // span 2 rows, which would otherwise fall on the same LDS banks).  B: stored
  // column by column ([nc][kk], real view) with a stride of 2 BK + 4 elements:
  // a thread's (re, im) pair is one 64-bit store, and the 16 columns x 4 k of
  // one MFMA operand read fall on 64 distinct banks ((2 BK + 4) / 4 is odd).
  constexpr int AST = BM * 2 + 16, BSK = 2 * BK + 4;
  __shared__ T As[2][BK * AST];  // [kc][mc] complex
  __shared__ T Bs[2][BN * BSK];  // [nc][kk] real view
  // XCD-aware remap: hardware places workgroup b on XCD b % 8.
  const int bid = blockIdx.x;
  const int xcd = bid & 7, loc = bid >> 3;
  const int per = tiles >> 3, rem = tiles & 7;
  const int tile = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + loc;
  int tm, tn;
  grouped_tile<16, sizeof(T) == 8 ? 16 : 8>(tile, tiles_m, tiles, tm, tn);
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wrow = (wave & 1) * 16 * WM;  // real-row offset of the wave inside the tile
  const int wcol = (wave >> 1) * 16 * WN;

  ACC acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = ACC{0, 0, 0, 0};

  CT ra[AL], rb[BL];
  auto gload_to = [&](int64_t kb, CT(&ra)[AL], CT(&rb)[BL]) {
#pragma unroll
    for (int i = 0; i < AL; ++i) {
      const int idx = tid + 256 * i;
      int mc, kc;
      if (TRANSA == 0) { mc = idx % BM; kc = idx / BM; } else { kc = idx % BK; mc = idx / BK; }
      const int64_t gm = m0 + mc, gk = kb + kc;
      CT v;
      v.x = 0; v.y = 0;
      bool keep = gm < m && gk < k;
      if (mk.akind && gm >= mk.ar0 && gm < mk.ar0 + mk.adw) keep = keep && mask_keep(mk.akind, gm - mk.ar0, gk);
      if (keep) v = TRANSA == 0 ? A[gm + gk * lda] : A[gk + gm * lda];
      ra[i] = v;
    }
#pragma unroll
    for (int i = 0; i < BL; ++i) {
      const int idx = tid + 256 * i;
      const int kc2 = idx % BK, nc = idx / BK;
      const int64_t gn = n0 + nc, gk2 = kb + kc2;
      CT u;
      u.x = 0; u.y = 0;
      bool keepb = gn < n && gk2 < k;
      if (mk.bkind) keepb = keepb && mask_keep(mk.bkind, gk2, gn);
      if (keepb) u = B[gk2 + gn * ldb];
      rb[i] = u;
    }
  };
  auto gload = [&](int64_t kb) { gload_to(kb, ra, rb); };
  auto sstore_from = [&](int buf, const CT(&ra)[AL], const CT(&rb)[BL]) {
#pragma unroll
    for (int i = 0; i < AL; ++i) {
      const int idx = tid + 256 * i;
      int mc, kc;
      if (TRANSA == 0) { mc = idx % BM; kc = idx / BM; } else { kc = idx % BK; mc = idx / BK; }
      As[buf][kc * AST + mc * 2 + 0] = ra[i].x;
      As[buf][kc * AST + mc * 2 + 1] = ra[i].y;
    }
#pragma unroll
    for (int i = 0; i < BL; ++i) {
      const int idx = tid + 256 * i;
      const int kc2 = idx % BK, nc = idx / BK;
      Bs[buf][nc * BSK + 2 * kc2 + 0] = rb[i].x;
      Bs[buf][nc * BSK + 2 * kc2 + 1] = rb[i].y;
    }
  };
  auto sstore = [&](int buf) { sstore_from(buf, ra, rb); };

  const int lr = lane & 15;   // row (A) / column (B) inside a 16-block
  const int lk = lane >> 4;   // k index inside a 4-step
  // Output rows of the 16x16 accumulator held by a lane: f32 MFMA gives rows
  // 4*lk + reg, f64 MFMA gives rows lk + 4*reg.  For f64 the A-fragment rows are
  // loaded through the transpose pi(x) = 4*(x & 3) + (x >> 2) of the 4x4 index
  // grid, so that in both cases the lane ends up with real rows 4*lk .. 4*lk+3,
  // i.e. (re, im) of two consecutive complex rows.
  const int arow = sizeof(T) == 8 ? (4 * (lr & 3) + (lr >> 2)) : lr;
  auto mma = [&](int buf) {
#pragma unroll
    for (int s = 0; s < BK / 2; ++s) {
      const int kk = 4 * s + lk;       // real k inside the stage
      const int kc = kk >> 1, sb = kk & 1;
      T a[WM], b[WN];
#pragma unroll
      for (int bm = 0; bm < WM; ++bm) {
        const int r = wrow + bm * 16 + arow;  // real row inside the tile
        const int t = r & 1;
        T v = As[buf][kc * AST + (r >> 1) * 2 + (sb ^ t)];
        a[bm] = (sb == 1 && t == 0) ? -v : v;
      }
#pragma unroll
      for (int bn = 0; bn < WN; ++bn) b[bn] = Bs[buf][(wcol + bn * 16 + lr) * BSK + kk];
#pragma unroll
      for (int bm = 0; bm < WM; ++bm)
#pragma unroll
        for (int bn = 0; bn < WN; ++bn) acc[bm][bn] = mfma16(a[bm], b[bn], acc[bm][bn]);
    }
  };
  // C of this lane's outputs (MODE 0): loaded before the k loop when the whole
  // k range is prefetched, else after it (batched launches)
  CT cold[WM][WN][2];
  auto load_c = [&]() {
#pragma unroll
    for (int bm = 0; bm < WM; ++bm)
#pragma unroll
      for (int bn = 0; bn < WN; ++bn)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int64_t col = n0 + wcol + bn * 16 + lr;
          const int64_t row = m0 + ((wrow + bm * 16) >> 1) + 2 * lk + h;
          cold[bm][bn][h].x = 0;
          cold[bm][bn][h].y = 0;
          if (col < n && row < m) cold[bm][bn][h] = C[row + col * ldc];
        }
  };
  if constexpr (NST > 0) {
    // k in chunks of NST stages, each chunk's operands in flight at once: all
    // of its stages are loaded into registers up front, then staged through
    // LDS one stage at a time, so a chunk pays one memory latency instead of
    // one per stage (these launches are short products whose time is set by
    // latency).  FP32 takes k <= 128 in one chunk; FP64 (twice the registers
    // per element) in two.
    static_assert(NST % 2 == 0, "stages alternate the two LDS buffers across chunks");
    for (int64_t kc0 = 0; kc0 < k; kc0 += (int64_t)NST * BK) {
      CT pa[NST][AL], pb[NST][BL];
#pragma unroll
      for (int s = 0; s < NST; ++s) gload_to(kc0 + (int64_t)s * BK, pa[s], pb[s]);
      if constexpr (MODE == 0) {
        if (kc0 == 0) load_c();
      }
#pragma unroll
      for (int s = 0; s < NST; ++s) {
        if (kc0 + (int64_t)s * BK < k) {  // uniform over the workgroup
          // buffer s & 1 was last read two stages earlier, which every wave
          // finished before the barrier of the stage in between
          sstore_from(s & 1, pa[s], pb[s]);
          __syncthreads();
          mma(s & 1);
        }
      }
    }
  } else {
    const int64_t ktiles = (k + BK - 1) / BK;
    gload(0);
    sstore(0);
    __syncthreads();
    for (int64_t kt = 0; kt < ktiles; ++kt) {
      const int buf = (int)(kt & 1);
      if (kt + 1 < ktiles) gload((kt + 1) * BK);
      mma(buf);
      if (kt + 1 < ktiles) sstore(buf ^ 1);
      __syncthreads();
    }
  }
  // epilogue: lane holds real rows 4*lk + {0..3} = two complex rows of column lane%16
  // (general products only: rows [ar0, ar0 + adw) optionally written to mk.c2)
  CT* const c2 = ROLE == 0 && mk.c2 ? static_cast<CT*>(mk.c2) + (int64_t)blockIdx.y * mk.sc2 : nullptr;
  auto dest = [&](int64_t row, int64_t col) -> CT* {
    if (ROLE == 0 && c2 && row >= mk.ar0 && row < mk.ar0 + mk.adw) return c2 + (row - mk.ar0) + col * mk.ldc2;
    return C + row + col * ldc;
  };
  if constexpr (MODE == 0 && (CB || NST > 0)) {
    // Every C load issued before the first store (a load after a store to the
    // same array waits for it, since the compiler cannot tell the addresses
    // apart: one memory latency per element otherwise).  Measured: batched
    // spectra 72.5 -> 82 systems/s; the single large products of one system
    // keep the plain loop below (2 % slower this way).
    if constexpr (NST == 0) load_c();
#pragma unroll
    for (int bm = 0; bm < WM; ++bm)
#pragma unroll
      for (int bn = 0; bn < WN; ++bn)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int64_t col = n0 + wcol + bn * 16 + lr;
          const int64_t row = m0 + ((wrow + bm * 16) >> 1) + 2 * lk + h;
          if (col >= n || row >= m) continue;
          CT c = cold[bm][bn][h];
          c.x -= acc[bm][bn][2 * h];
          c.y -= acc[bm][bn][2 * h + 1];
          *dest(row, col) = c;
        }
    return;
  }
#pragma unroll
  for (int bm = 0; bm < WM; ++bm)
#pragma unroll
    for (int bn = 0; bn < WN; ++bn) {
      const int64_t col = n0 + wcol + bn * 16 + lr;
      const int64_t crow = m0 + ((wrow + bm * 16) >> 1) + 2 * lk;
      if (col >= n) continue;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int64_t row = crow + h;
        if (row >= m) continue;
        const T vr = acc[bm][bn][2 * h], vi = acc[bm][bn][2 * h + 1];
        if (MODE == 0) {
          CT c = C[row + col * ldc];
          c.x -= vr;
          c.y -= vi;
          *dest(row, col) = c;
        } else {
          CT c;
          c.x = vr;
          c.y = vi;
          *dest(row, col) = c;
        }
      }
    }
}

// FP32 trailing update C -= A B by the 3M form of the complex product: with
// A = Ar + i Ai, B = Br + i Bi the three real products T1 = Ar Br, T2 = Ai Bi
// and T3 = (Ar + Ai)(Br + Bi) give Re(AB) = T1 - T2 and Im(AB) = T3 - T1 - T2,
// so 3 real MFMAs replace the 4 of the expanded form (12 instead of 16 16x16x4
// MFMAs per wave per 4 complex k).  The staging writes each operand as three
// real planes (re, im, re + im; A as [k][row], B as [k][column], rows padded by
// 16 floats) and every wave of the 2 x 2 grid holds 3 x WMB x WNB accumulators.
// The extra rounding of the sums is that of 3M (its error bound is a small
// multiple of the 4M one); the factorisations that use it are FP32 ones
// refined in FP64.  Tiles: BM = 32 WMB complex rows, BN = 32 WNB columns, BK
// complex k per stage; the XCD remap of cgemm_kernel, then grouped_tile.
template <typename T, int WMB, int WNB, int BK, bool CB, int MODE = 0>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
cgemm3m_update_kernel(int64_t m, int64_t n, int64_t k, const cplx<T>* __restrict__ A, int64_t lda,
                      const cplx<T>* __restrict__ B, int64_t ldb, cplx<T>* __restrict__ C, int64_t ldc, int tiles_m,
                      int tiles, int64_t sA, int64_t sB, int64_t sC) {
  using CT = cplx<T>;
  using ACC = typename acc_of<T>::type;
  const CT czero = CT{0, 0};
  constexpr int BM = 32 * WMB, BN = 32 * WNB;
  constexpr int AL = BM * BK / 256, BL = BK * BN / 256;
  static_assert(AL * 256 == BM * BK && BL * 256 == BK * BN && BK % 4 == 0, "tile shape");
  constexpr int AP = BM + 16, BP = BN + 16;
  A += (int64_t)blockIdx.y * sA;
  B += (int64_t)blockIdx.y * sB;
  C += (int64_t)blockIdx.y * sC;
  __shared__ T As[2][3][BK * AP];  // [plane][k][row]
  __shared__ T Bs[2][3][BK * BP];  // [plane][k][column]
  const int bid = blockIdx.x;
  const int xcd = bid & 7, loc = bid >> 3;
  const int per = tiles >> 3, rem = tiles & 7;
  const int tile = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + loc;
  int tm, tn;
  grouped_tile<16, sizeof(T) == 8 ? 16 : 8>(tile, tiles_m, tiles, tm, tn);
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wrow = (wave & 1) * 16 * WMB;  // complex rows
  const int wcol = (wave >> 1) * 16 * WNB;
  const int lr = lane & 15, lk = lane >> 4;
  // B columns of k rows 4..7 (mod 8; FP64: 2..3 mod 4) stored with column bit 3
  // flipped: a wave stores 8 k x 8 columns (FP64: 4 k x 16), and with the row
  // stride BP (16 banks apart mod 64; FP64: 32) rows kc and kc + 4 (kc + 2)
  // would otherwise put the same column on the same bank; an MFMA operand read
  // covers 4 k rows, so its 16-column groups only permute
  constexpr int SWK = sizeof(T) == 8 ? 2 : 4;
  auto bswz = [](int kc, int nc) { return GEMM3M_BSWZ && (kc & SWK) ? nc ^ 8 : nc; };
  ACC acc[3][WMB][WNB];
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int i = 0; i < WMB; ++i)
#pragma unroll
      for (int j = 0; j < WNB; ++j) acc[q][i][j] = ACC{0, 0, 0, 0};
  CT ra[AL], rb[BL];
  auto gload = [&](int64_t kb) {
#pragma unroll
    for (int i = 0; i < AL; ++i) {
      const int idx = tid + 256 * i;
      const int mc = idx % BM, kc = idx / BM;
      const int64_t gm = m0 + mc, gk = kb + kc;
      ra[i] = (gm < m && gk < k) ? A[gm + gk * lda] : czero;
    }
#pragma unroll
    for (int i = 0; i < BL; ++i) {
      const int idx = tid + 256 * i;
      const int kc = idx % BK, nc = idx / BK;
      const int64_t gn = n0 + nc, gk = kb + kc;
      rb[i] = (gn < n && gk < k) ? B[gk + gn * ldb] : czero;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < AL; ++i) {
      const int idx = tid + 256 * i;
      const int mc = idx % BM, kc = idx / BM;
      As[buf][0][kc * AP + mc] = ra[i].x;
      As[buf][1][kc * AP + mc] = ra[i].y;
      As[buf][2][kc * AP + mc] = ra[i].x + ra[i].y;
    }
#pragma unroll
    for (int i = 0; i < BL; ++i) {
      const int idx = tid + 256 * i;
      const int kc = idx % BK, nc = idx / BK;
      const int o = kc * BP + bswz(kc, nc);
      Bs[buf][0][o] = rb[i].x;
      Bs[buf][1][o] = rb[i].y;
      Bs[buf][2][o] = rb[i].x + rb[i].y;
    }
  };
  const int64_t ktiles = (k + BK - 1) / BK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int64_t kt = 0; kt < ktiles; ++kt) {
    const int buf = (int)(kt & 1);
    if (kt + 1 < ktiles) gload((kt + 1) * BK);
#pragma unroll
    for (int k4 = 0; k4 < BK; k4 += 4) {
      const int kr = k4 + lk;
      T a[3][WMB], b[3][WNB];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
#pragma unroll
        for (int i = 0; i < WMB; ++i) a[q][i] = As[buf][q][kr * AP + wrow + 16 * i + lr];
#pragma unroll
        for (int j = 0; j < WNB; ++j) b[q][j] = Bs[buf][q][kr * BP + bswz(kr, wcol + 16 * j + lr)];
      }
#pragma unroll
      for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int i = 0; i < WMB; ++i)
#pragma unroll
          for (int j = 0; j < WNB; ++j) acc[q][i][j] = mfma16(a[q][i], b[q][j], acc[q][i][j]);
    }
    if (kt + 1 < ktiles) sstore(buf ^ 1);
    __syncthreads();
  }
  // lane holds rows 4 lk + r (r < 4) of column lr of each 16 x 16 block (FP32),
  // rows lk + 4 r (FP64, the other result layout of the FP64 MFMA)
  auto rof = [&](int r) { return sizeof(T) == 8 ? lk + 4 * r : 4 * lk + r; };
  auto out = [&](int i, int j, int r, T& cr, T& ci) {
    const T t1 = acc[0][i][j][r], t2 = acc[1][i][j][r], t3 = acc[2][i][j][r];
    cr = t1 - t2;
    ci = t3 - t1 - t2;
  };
  if constexpr (MODE == 1) {
    // C = A B (no read of C)
#pragma unroll
    for (int i = 0; i < WMB; ++i)
#pragma unroll
      for (int j = 0; j < WNB; ++j) {
        const int64_t col = n0 + wcol + 16 * j + lr;
        if (col >= n) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = m0 + wrow + 16 * i + rof(r);
          if (row >= m) continue;
          T cr, ci;
          out(i, j, r, cr, ci);
          C[row + col * ldc] = CT{cr, ci};
        }
      }
    return;
  }
  if constexpr (CB) {
    // every C load before the first store (the batched products' epilogue)
    CT cold[WMB][WNB][4];
#pragma unroll
    for (int i = 0; i < WMB; ++i)
#pragma unroll
      for (int j = 0; j < WNB; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = m0 + wrow + 16 * i + rof(r), col = n0 + wcol + 16 * j + lr;
          cold[i][j][r] = (row < m && col < n) ? C[row + col * ldc] : czero;
        }
#pragma unroll
    for (int i = 0; i < WMB; ++i)
#pragma unroll
      for (int j = 0; j < WNB; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = m0 + wrow + 16 * i + rof(r), col = n0 + wcol + 16 * j + lr;
          if (row >= m || col >= n) continue;
          T cr, ci;
          out(i, j, r, cr, ci);
          C[row + col * ldc] = CT{cold[i][j][r].x - cr, cold[i][j][r].y - ci};
        }
    return;
  }
#pragma unroll
  for (int i = 0; i < WMB; ++i)
#pragma unroll
    for (int j = 0; j < WNB; ++j) {
      const int64_t col = n0 + wcol + 16 * j + lr;
      if (col >= n) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + wrow + 16 * i + rof(r);
        if (row >= m) continue;
        T cr, ci;
        out(i, j, r, cr, ci);
        CT c = C[row + col * ldc];
        c.x -= cr;
        c.y -= ci;
        C[row + col * ldc] = c;
      }
    }
}

// Compute units of the current device (queried once per device).
static int gemm_num_cu() {
  static int cu[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cu[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    cu[dev] = v;
  }
  return cu[dev];
}

// Launch with the tile shape (WM, WN, BK); tile counts checked by the caller's shape.
template <typename T, int MODE, int TRANSA, int ROLE, int WM, int WN, int BK, int NST = 0>
static hipError_t launch_tiles(int64_t m, int64_t n, int64_t k, const cplx<T>* a, int64_t lda, const cplx<T>* b,
                               int64_t ldb, cplx<T>* c, int64_t ldc, hipStream_t st, GemmMask mk, int nbatch,
                               int64_t sA, int64_t sB, int64_t sC) {
  const int64_t tm = (m + 16 * WM - 1) / (16 * WM), tn = (n + 32 * WN - 1) / (32 * WN);
  if (tm * tn > INT32_MAX) return hipErrorInvalidValue;
  const int tiles = (int)(tm * tn);
  // batched launches (several systems at once) take the epilogue with all C
  // loads in flight
  if (NST == 0 && nbatch > 1)
    hipLaunchKernelGGL((cgemm_kernel<T, MODE, TRANSA, ROLE, WM, WN, BK, true>), dim3(tiles, nbatch), dim3(256), 0, st, m,
                       n, k, a, lda, b, ldb, c, ldc, (int)tm, tiles, mk, sA, sB, sC);
  else
    hipLaunchKernelGGL((cgemm_kernel<T, MODE, TRANSA, ROLE, WM, WN, BK, false, NST>), dim3(tiles, nbatch), dim3(256), 0,
                       st, m, n, k, a, lda, b, ldb, c, ldc, (int)tm, tiles, mk, sA, sB, sC);
  return hipGetLastError();
}

// Small tiles when the 64 x 64 tiling gives fewer than two workgroups per CU.
static bool use_small_tiles(int64_t m, int64_t n, int nbatch) {
  const int64_t big = ((m + 63) / 64) * ((n + 63) / 64) * (int64_t)nbatch;
  return big < 2 * (int64_t)gemm_num_cu();
}

template <typename T, int MODE, int TRANSA, int ROLE>
static hipError_t launch_cfg(int64_t m, int64_t n, int64_t k, const cplx<T>* a, int64_t lda, const cplx<T>* b,
                             int64_t ldb, cplx<T>* c, int64_t ldc, hipStream_t st, GemmMask mk, int nbatch, int64_t sA,
                             int64_t sB, int64_t sC) {
  if (use_small_tiles(m, n, nbatch)) {
    // one system's products over k >= 64 (the solve steps, L21 and U12 blocks,
    // the look-ahead columns) with 16 complex k per stage: half the stages of
    // their latency-bound k loop (FP32+IR step 72.9 -> 72.2 ms; 32 measured
    // the same); the batched launches keep 8
    if (nbatch == 1 && k >= 64 && k <= 128 && GEMM_SMALL_PREFETCH)
      return launch_tiles<T, MODE, TRANSA, ROLE, 2, 1, 16, sizeof(T) == 8 ? 4 : 8>(m, n, k, a, lda, b, ldb, c, ldc, st,
                                                                                mk, nbatch, sA, sB, sC);
    if (nbatch == 1 && k >= 64)
      return launch_tiles<T, MODE, TRANSA, ROLE, 2, 1, 16>(m, n, k, a, lda, b, ldb, c, ldc, st, mk, nbatch, sA, sB, sC);
    return launch_tiles<T, MODE, TRANSA, ROLE, 2, 1, 8>(m, n, k, a, lda, b, ldb, c, ldc, st, mk, nbatch, sA, sB, sC);
  }
  // 4 complex k per stage for the products of one system (update GEMM: FP32
  // 87.5 -> 90, FP64 40 -> 45 TFLOP/s; FP64 step 158.6 -> 148.8 ms), 8 for
  // batched launches (83 vs 78 systems/s on the batched spectra)
  if (nbatch == 1)
    return launch_tiles<T, MODE, TRANSA, ROLE, 4, 2, 4>(m, n, k, a, lda, b, ldb, c, ldc, st, mk, nbatch, sA, sB, sC);
  return launch_tiles<T, MODE, TRANSA, ROLE, 4, 2, 8>(m, n, k, a, lda, b, ldb, c, ldc, st, mk, nbatch, sA, sB, sC);
}

template <typename T>
hipError_t launch_gemm(int mode, int transA, int64_t m, int64_t n, int64_t k, const void* A, int64_t lda,
                       const void* B, int64_t ldb, void* C, int64_t ldc, hipStream_t st, GemmMask mk, int nbatch,
                       int64_t sA, int64_t sB, int64_t sC) {
  if (m <= 0 || n <= 0 || nbatch <= 0) return hipSuccess;
  if (nbatch > 65535) return hipErrorInvalidValue;
  const auto* a = static_cast<const cplx<T>*>(A);
  const auto* b = static_cast<const cplx<T>*>(B);
  auto* c = static_cast<cplx<T>*>(C);
  if (k <= 0 && mode == 0) return hipSuccess;  // C - 0
  if (mode == 0 && transA == 0) return launch_cfg<T, 0, 0, 0>(m, n, k, a, lda, b, ldb, c, ldc, st, mk, nbatch, sA, sB, sC);
  if (mode == 0) return launch_cfg<T, 0, 1, 0>(m, n, k, a, lda, b, ldb, c, ldc, st, mk, nbatch, sA, sB, sC);
  if (transA == 0) return launch_cfg<T, 1, 0, 0>(m, n, k, a, lda, b, ldb, c, ldc, st, mk, nbatch, sA, sB, sC);
  return launch_cfg<T, 1, 1, 0>(m, n, k, a, lda, b, ldb, c, ldc, st, mk, nbatch, sA, sB, sC);
}

// The FP32 update with the 64 x 64 tile: 3M products (cgemm3m_update_kernel).
template <typename T>
static hipError_t launch_update_3m(int64_t m, int64_t n, int64_t k, const cplx<T>* a, int64_t lda, const cplx<T>* b,
                                   int64_t ldb, cplx<T>* c, int64_t ldc, hipStream_t st, int nbatch, int64_t sA,
                                   int64_t sB, int64_t sC) {
  const int64_t tm = (m + 63) / 64, tn = (n + 63) / 64;
  if (tm * tn > INT32_MAX) return hipErrorInvalidValue;
  const int tiles = (int)(tm * tn);
  // 8 complex k per stage in FP32 (4 before the grouped tile order, which made
  // 8 the faster: FP32 factorisation 58.2 -> 57.3 ms at n = 12 000; 128 x 64
  // and 64 x 128 tiles measured 59.4 and 59.9 ms); FP64 keeps 4, since 8 would
  // leave one wave per SIMD
  constexpr int BKS = sizeof(T) == 8 ? 4 : 8;
  if (nbatch > 1)
    hipLaunchKernelGGL((cgemm3m_update_kernel<T, 2, 2, BKS, true>), dim3(tiles, nbatch), dim3(256), 0, st, m, n, k, a,
                       lda, b, ldb, c, ldc, (int)tm, tiles, sA, sB, sC);
  else
    hipLaunchKernelGGL((cgemm3m_update_kernel<T, 2, 2, BKS, false>), dim3(tiles, nbatch), dim3(256), 0, st, m, n, k, a,
                       lda, b, ldb, c, ldc, (int)tm, tiles, sA, sB, sC);
  return hipGetLastError();
}

// C = A B with the 3M kernel (64 x 64 tiles, 4 complex k per stage), nbatch
// independent products (item z at A + z sA, B + z sB, C + z sC): the k-split
// partial products of the FP64 refinement residual.
template <typename T>
hipError_t launch_gemm_product_3m(int64_t m, int64_t n, int64_t k, const void* A, int64_t lda, const void* B,
                                  int64_t ldb, void* C, int64_t ldc, hipStream_t st, int nbatch, int64_t sA, int64_t sB,
                                  int64_t sC) {
  if (m <= 0 || n <= 0 || k <= 0 || nbatch <= 0) return hipSuccess;
  if (nbatch > 65535) return hipErrorInvalidValue;
  const int64_t tm = (m + 63) / 64, tn = (n + 63) / 64;
  if (tm * tn > INT32_MAX) return hipErrorInvalidValue;
  const int tiles = (int)(tm * tn);
  hipLaunchKernelGGL((cgemm3m_update_kernel<T, 2, 2, 4, false, 1>), dim3(tiles, nbatch), dim3(256), 0, st, m, n, k,
                     static_cast<const cplx<T>*>(A), lda, static_cast<const cplx<T>*>(B), ldb, static_cast<cplx<T>*>(C),
                     ldc, (int)tm, tiles, sA, sB, sC);
  return hipGetLastError();
}
template hipError_t launch_gemm_product_3m<double>(int64_t, int64_t, int64_t, const void*, int64_t, const void*,
                                                   int64_t, void*, int64_t, hipStream_t, int, int64_t, int64_t,
                                                   int64_t);

template <typename T>
hipError_t launch_gemm_update(int64_t m, int64_t n, int64_t k, const void* A, int64_t lda, const void* B,
                              int64_t ldb, void* C, int64_t ldc, hipStream_t st, int nbatch, int64_t sA, int64_t sB,
                              int64_t sC) {
  if (m <= 0 || n <= 0 || k <= 0 || nbatch <= 0) return hipSuccess;
  if (nbatch > 65535) return hipErrorInvalidValue;
  if (GEMM_UPDATE_3M && !use_small_tiles(m, n, nbatch))
    return launch_update_3m<T>(m, n, k, static_cast<const cplx<T>*>(A), lda, static_cast<const cplx<T>*>(B), ldb,
                               static_cast<cplx<T>*>(C), ldc, st, nbatch, sA, sB, sC);
  return launch_cfg<T, 0, 0, 1>(m, n, k, static_cast<const cplx<T>*>(A), lda, static_cast<const cplx<T>*>(B), ldb,
                                static_cast<cplx<T>*>(C), ldc, st, GemmMask{}, nbatch, sA, sB, sC);
}
template hipError_t launch_gemm_update<double>(int64_t, int64_t, int64_t, const void*, int64_t, const void*, int64_t,
                                               void*, int64_t, hipStream_t, int, int64_t, int64_t, int64_t);
template hipError_t launch_gemm_update<float>(int64_t, int64_t, int64_t, const void*, int64_t, const void*, int64_t,
                                              void*, int64_t, hipStream_t, int, int64_t, int64_t, int64_t);

template hipError_t launch_gemm<double>(int, int, int64_t, int64_t, int64_t, const void*, int64_t, const void*,
                                        int64_t, void*, int64_t, hipStream_t, GemmMask, int, int64_t, int64_t, int64_t);
template hipError_t launch_gemm<float>(int, int, int64_t, int64_t, int64_t, const void*, int64_t, const void*,
                                       int64_t, void*, int64_t, hipStream_t, GemmMask, int, int64_t, int64_t, int64_t);

}  // namespace gdm
