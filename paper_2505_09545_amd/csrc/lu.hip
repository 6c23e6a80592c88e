// Step (b) of the hot path: dense complex LU with partial pivoting and the
// multi-right-hand-side solve (arXiv:2505.09545, Sec. "Numerical solution": the
// system M F = F0 is solved by LU decomposition; many illuminations are solved
// at once, Sec. "Implementation technical details", batch evaluation).
//
// Algorithm: blocked right-looking getrf.  For each block of w columns at k0
//   1. panel: factor A[k0:n, k0:k0+w] with partial pivoting (pivot = largest
//      |re|+|im| in the column, lowest row on ties).  One cooperative launch of
//      G workgroups; each holds R rows of the panel in LDS and the workgroups
//      agree on every pivot through one device-wide barrier per column.
//   2. the panel also lists the block's net row permutation (<= 2w rows move,
//      read off the row labels), which is applied to the trailing columns and,
//      in the solve, to the right-hand sides.  Interchanges are never applied
//      to the columns left of the block: the factors are kept in the factored
//      form
//          M = P1^T L1 P2^T L2 ... Pk^T Lk U
//      and the solve applies P_b before using L_b, which is equivalent.
//   3. U12 = L11^-1 A12 (by substitution for the next panel's columns, by a
//      product with the inverse of L11 for the rest), 4. A22 -= L21 U12
//      (complex GEMM on MFMA, gemm.hip).  With look-ahead, steps 3-4 for the
//      next panel's columns run on the main stream and the rest of the trailing
//      matrix on a side stream, overlapping the next panel.
//
// Layout: column-major interleaved complex, leading dimension ld.  ipiv holds
// 0-based global row indices (LAPACK semantics otherwise).
#include <algorithm>
#include <climits>
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>
#include <vector>

#include "gdm_common.hpp"
#include "gdm_kernels.hpp"

namespace gdm {

constexpr uint32_t SPIN_LIMIT = 1u << 22;

template <typename CT> __device__ inline CT cmul_t(CT a, CT b) {
  CT r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
// t - l u: one entry of a rank-1 update
template <typename CT> __device__ inline CT r1_upd(CT t, const CT& l, const CT& u) {
  t.x -= l.x * u.x - l.y * u.y;
  t.y -= l.x * u.y + l.y * u.x;
  return t;
}
template <typename CT> __device__ inline CT cinv_t(CT a) {
  // 1/a = conj(a) / |a|^2, with a scaled by the power of two 2^-e of its larger
  // component (exact) so that |a|^2 can neither overflow nor underflow; one
  // division (a = 0 gives NaN, as the quotient form did)
  const auto s = fabs(a.x) > fabs(a.y) ? fabs(a.x) : fabs(a.y);
  int e;
  (void)frexp(s, &e);
  const auto ar = ldexp(a.x, -e), ai = ldexp(a.y, -e);
  const auto id = 1 / (ar * ar + ai * ai);
  CT r;
  r.x = ldexp(ar * id, -e);
  r.y = ldexp(-ai * id, -e);
  return r;
}

__device__ inline unsigned long long shfl_xor_u64(unsigned long long v, int m) {
  const unsigned lo = __shfl_xor((unsigned)(v & 0xffffffffu), m);
  const unsigned hi = __shfl_xor((unsigned)(v >> 32), m);
  return ((unsigned long long)hi << 32) | lo;
}

__global__ void zero_u64_kernel(unsigned long long* a, size_t na, unsigned long long* b, size_t nb,
                                int32_t* c, size_t nc) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < na) a[i] = 0;
  if (i < nb) b[i] = 0;
  if (i < nc) c[i] = 0;
}

__global__ void init_err_kernel(int32_t* err) {
  if (threadIdx.x == 0) {
    err[0] = 0;
    err[1] = INT32_MAX;
  }
}

// ---------------------------------------------------------------------------
// 1. panel factorisation (cooperative, one device-wide exchange per column)
// ---------------------------------------------------------------------------
// Cross-workgroup exchange uses self-validating 64-bit words: the high 32 bits
// hold an epoch (unique per column of the whole factorisation), the low 32 bits
// the payload.  Words are written and read with agent-scope relaxed atomics; a
// reader spins on each word until it carries the epoch it expects, so no
// release/acquire fences (L2 write-back / invalidate) are needed.  Every buffer
// is double-buffered by column parity: a workgroup can only overwrite a slot of
// parity j%2 at column j+2, after every other workgroup has published its
// column j+1 key, i.e. after they all finished reading column j.
typedef unsigned long long u64;
// each workgroup's key words get their own 128-byte line (no false sharing
// between the atomic stores of different workgroups)
constexpr int KEY_STRIDE = 16;

__device__ inline void ll_put(u64* p, uint32_t epoch, uint32_t payload) {
  __hip_atomic_store(p, ((u64)epoch << 32) | payload, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Spin until the word carries `epoch`; returns the payload (0 and sets *bad on timeout).
__device__ inline uint32_t ll_get(const u64* p, uint32_t epoch, int* bad) {
  uint32_t it = 0;
  while (true) {
    const u64 v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((uint32_t)(v >> 32) == epoch) return (uint32_t)v;
    if (++it > SPIN_LIMIT) {
      *bad = 1;
      return 0;
    }
  }
}
// Several words at once: all loads are in flight together (one round trip when
// the data is already there); only words not yet carrying `epoch` are re-read.
template <int K>
__device__ inline void ll_get_n(const u64* const (&p)[K], uint32_t epoch, uint32_t (&out)[K], int* bad) {
  u64 v[K];
#pragma unroll
  for (int i = 0; i < K; ++i) v[i] = __hip_atomic_load(p[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  uint32_t it = 0;
  while (true) {
    bool all = true;
#pragma unroll
    for (int i = 0; i < K; ++i) all = all && (uint32_t)(v[i] >> 32) == epoch;
    if (all) break;
    if (++it > SPIN_LIMIT) {
      *bad = 1;
      break;
    }
#pragma unroll
    for (int i = 0; i < K; ++i)
      if ((uint32_t)(v[i] >> 32) != epoch) v[i] = __hip_atomic_load(p[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
#pragma unroll
  for (int i = 0; i < K; ++i) out[i] = (uint32_t)v[i];
}

// f(0), f(1), ..., f(N - 1) with compile-time indices (expanded whatever the
// unroller decides, so register arrays indexed by them stay in registers)
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// CPT records of KW consecutive words each (record u at base[u]), returned once
// every word carries `epoch`; all loads in flight together.  While some word is
// stale every word is loaded again (a word that already carries the epoch keeps
// it until this reader is done, so reloading it is harmless).
template <int KW, int CPT>
__device__ inline void ll_get_rec(const u64* const (&base)[CPT], uint32_t epoch, uint32_t (&out)[CPT * KW], int* bad) {
  u64 v[CPT * KW];
  auto load_all = [&]() {
    static_for<CPT * KW>([&](auto i) {
      v[i] = __hip_atomic_load(base[i / KW] + i % KW, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    });
  };
  load_all();
  uint32_t it = 0;
  while (true) {
    bool all = true;
    static_for<CPT * KW>([&](auto i) { all = all && (uint32_t)(v[i] >> 32) == epoch; });
    if (all) break;
    if (++it > SPIN_LIMIT) {
      *bad = 1;
      break;
    }
    load_all();
  }
  static_for<CPT * KW>([&](auto i) { out[i] = (uint32_t)v[i]; });
}

// K words at p[i] (any addresses), as ll_get_rec.
template <int K>
__device__ inline void ll_get_sel(const u64* const (&p)[K], uint32_t epoch, uint32_t (&out)[K], int* bad) {
  u64 v[K];
  auto load_all = [&]() {
    static_for<K>([&](auto i) { v[i] = __hip_atomic_load(p[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); });
  };
  load_all();
  uint32_t it = 0;
  while (true) {
    bool all = true;
    static_for<K>([&](auto i) { all = all && (uint32_t)(v[i] >> 32) == epoch; });
    if (all) break;
    if (++it > SPIN_LIMIT) {
      *bad = 1;
      break;
    }
    load_all();
  }
  static_for<K>([&](auto i) { out[i] = (uint32_t)v[i]; });
}

// complex values travel as their 32-bit words (2 for complex float, 4 for
// complex double), little-endian order of the (re, im) storage.
template <typename CT> __device__ inline uint32_t cword(const CT& v, int k) {
  return reinterpret_cast<const uint32_t*>(&v)[k];
}

// Rows never move between workgroups inside the panel: each local row carries a
// label, the position it will be written back to.  The interchange of column j
// (positions gj <-> p) swaps the labels of the two rows involved, which their
// owners do locally; the pivot row's values are the only data exchanged.
template <typename CT>
__device__ inline u64 pivot_key(const CT& v, uint32_t label) {
  const float a = (float)(fabs(v.x) + fabs(v.y));
  return ((u64)__float_as_uint(a) << 32) | (0xffffffffu - label);
}

// Wave-wide max of a 64-bit key with DPP moves: xor-1 and xor-2 within quads,
// then mirrors within 8 and 16 lanes leave every lane with the max of its row
// of 16; the four row maxima are combined with readlane.
template <int CTRL>
__device__ inline u64 dpp_u64(u64 v) {
  const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)v, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(v >> 32), CTRL, 0xf, 0xf, false);
  return ((u64)(uint32_t)hi << 32) | (uint32_t)lo;
}
__device__ inline u64 wave_max_u64(u64 v) {
  u64 o;
  o = dpp_u64<0xb1>(v);  // quad_perm [1,0,3,2]
  v = o > v ? o : v;
  o = dpp_u64<0x4e>(v);  // quad_perm [2,3,0,1]
  v = o > v ? o : v;
  o = dpp_u64<0x141>(v);  // row_half_mirror
  v = o > v ? o : v;
  o = dpp_u64<0x140>(v);  // row_mirror
  v = o > v ? o : v;
  u64 r = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 16 * q);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 16 * q);
    const u64 x = ((u64)hi << 32) | lo;
    r = x > r ? x : r;
  }
  return r;
}

// Workgroup-wide argmax of (key, idx); one barrier.  Keys are unique (they end
// with the row label), so only the key is reduced and the lane holding the
// winning key publishes its idx.  skey/sidx: LDS arrays (4 entries) that the
// caller does not touch again before the next barrier.
__device__ inline void block_argmax(u64& key, int& idx, u64* skey, int* sidx) {
  const u64 k = wave_max_u64(key);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) skey[wv] = k;
  if (key == k && k != 0) sidx[wv] = idx;
  __syncthreads();
  key = skey[0];
  int wbest = 0;
#pragma unroll
  for (int i = 1; i < 4; ++i)
    if (skey[i] > key) {
      key = skey[i];
      wbest = i;
    }
  idx = key ? sidx[wbest] : -1;
}

// The panel also lists the rows it moved, as (final position, original
// position) pairs: a row's label is its final position, so a workgroup knows
// its moved rows without replaying the interchanges.  Slots are claimed with an
// atomic counter (zeroed before the factorisation); the order of the list is
// irrelevant, since the permutation gathers every source before it scatters.
template <typename T>
__global__ void __launch_bounds__(256) panel_kernel(cplx<T>* __restrict__ A, int64_t ld, int64_t n, int64_t k0, int w,
                                                     int R, int G, int32_t* __restrict__ ipiv, LUWork ws,
                                                     uint32_t epoch0, int64_t sA, int64_t sipiv,
                                                     int32_t* __restrict__ mdst, int32_t* __restrict__ msrc,
                                                     int32_t* __restrict__ mcount, int mcap) {
  using CT = cplx<T>;
  // batch item blockIdx.y: its own matrix, pivots and exchange buffers
  A += (int64_t)blockIdx.y * sA;
  ipiv += (int64_t)blockIdx.y * sipiv;
  ws.cand += (int64_t)blockIdx.y * ws.s_cand;
  ws.rows += (int64_t)blockIdx.y * ws.s_rows;
  mdst += (int64_t)blockIdx.y * ws.s_pairs;
  msrc += (int64_t)blockIdx.y * ws.s_pairs;
  mcount += (int64_t)blockIdx.y * ws.s_npairs;
  constexpr int NW = sizeof(CT) / 4;  // payload words per complex
  extern __shared__ unsigned char smem_raw[];
  CT* tile = reinterpret_cast<CT*>(smem_raw);           // [w][R], column c at tile + c*R
  CT* prow = tile + (size_t)w * R;                      // [w] pivot row
  int32_t* lab = reinterpret_cast<int32_t*>(prow + w);  // [R] row labels (final positions)
  int32_t* pl = lab + R;                                // [w] pivot positions of this panel
  __shared__ u64 skey1[4], skey2[4];
  __shared__ int sidx1[4], sidx2[4];
  __shared__ int bad;
  const int g = blockIdx.x, tid = threadIdx.x;
  const int64_t rbase = k0 + (int64_t)g * R;
  const int myR = (int)(n - rbase < (int64_t)R ? (n - rbase > 0 ? n - rbase : 0) : R);
  if (tid == 0) bad = 0;
  // columns in batches of LB loads in flight per thread (a load followed by its
  // LDS store in one loop body would put one memory latency per column on the
  // panel's critical path)
  constexpr int LB = 128 / (int)sizeof(CT);
  const int wfull = w - w % LB;
  for (int lr = tid; lr < myR; lr += 256) {
    const CT* src = A + (rbase + lr) + k0 * ld;
    for (int c0 = 0; c0 < wfull; c0 += LB) {
      CT v[LB];
#pragma unroll
      for (int u = 0; u < LB; ++u) v[u] = src[(c0 + u) * ld];
#pragma unroll
      for (int u = 0; u < LB; ++u) tile[(c0 + u) * R + lr] = v[u];
    }
    for (int c = wfull; c < w; ++c) tile[c * R + lr] = src[c * ld];
  }
  for (int lr = tid; lr < myR; lr += 256) lab[lr] = (int32_t)(rbase + lr);
  // 2D mapping for the rank-1 update: RP rows x CG column groups
  int RP = 1;
  while (RP < myR && RP < 256) RP <<= 1;
  const int CG = 256 / RP;
  const int ulr0 = tid & (RP - 1), ucg = tid / RP;
  __syncthreads();
  // candidate of column 0
  u64 best = 0;
  int brow = -1;
  for (int lr = tid; lr < myR; lr += 256) {
    const u64 kk = pivot_key(tile[lr], (uint32_t)lab[lr]);
    if (kk > best) {
      best = kk;
      brow = lr;
    }
  }
  int zero_col = -1;
  // Column j's rank-1 update is split: column j + 1 right after the pivot is
  // known (it holds the next pivot candidates), the rest of the trailing
  // columns after the next candidate has been published, so that it runs while
  // the other workgroups' keys for column j + 1 are on their way.  Every row
  // receives every update exactly once: the candidate row gets its deferred part
  // when it is published, the other rows in the bulk step.
  for (int j = 0; j < w; ++j) {
    const int64_t gj = k0 + j;
    const uint32_t E = epoch0 + (uint32_t)j;
    const int par = j & 1;
    u64* cand = ws.cand + (size_t)par * ws.gitem * KEY_STRIDE;
    u64* rows = ws.rows + (size_t)par * ws.gitem * ws.wwmax;
    // workgroup candidate over its active rows (labels >= gj); column j is final
    block_argmax(best, brow, skey1, sidx1);
    const u64 mybest = best;
    const int lrow = best ? brow : -1;
    // publish key (value, label) and columns j.. of the candidate row; its
    // columns j + 1.. first receive the deferred update by pivot j - 1 (the
    // multipliers of pivot j - 1 sit in tile column j - 1)
    if (tid == 0) {
      ll_put(&cand[KEY_STRIDE * g + 0], E, mybest ? (uint32_t)(mybest >> 32) : 0u);
      ll_put(&cand[KEY_STRIDE * g + 1], E, mybest ? (0xffffffffu - (uint32_t)(mybest & 0xffffffffu)) : 0xffffffffu);
    }
    const int WC = w - j;  // columns still needed by the others
    if (lrow >= 0)
      for (int tc = tid; tc < WC; tc += 256) {
        const int c = j + tc;
        CT v = tile[c * R + lrow];
        if (j > 0 && tc > 0) {
          v = r1_upd(v, tile[(j - 1) * R + lrow], prow[c]);
          tile[c * R + lrow] = v;
        }
#pragma unroll
        for (int q = 0; q < NW; ++q) ll_put(&rows[(size_t)g * ws.wwmax + (size_t)tc * NW + q], E, cword(v, q));
      }
    // deferred part of pivot j - 1's update: columns j + 1.. of the other active rows
    if (j > 0) {
      for (int lr = ulr0; lr < myR; lr += RP) {
        if (lab[lr] <= (int32_t)(gj - 1) || lr == lrow) continue;
        const CT l = tile[(j - 1) * R + lr];
        int c = j + 1 + ucg;
        // FP32: batches of UB columns, all reads first, then the updates, then
        // all writes (written one column at a time, each read would wait for
        // the previous column's write, since the compiler cannot tell them
        // apart).  The same batching makes the FP64 panel slower, so FP64 keeps
        // the column-at-a-time loop.
        constexpr int UB = 8;
        if constexpr (sizeof(T) == 4) {
          for (; c + (UB - 1) * CG < w; c += UB * CG) {
            CT t[UB], u[UB];
#pragma unroll
            for (int e = 0; e < UB; ++e) {
              u[e] = prow[c + e * CG];
              t[e] = tile[(c + e * CG) * R + lr];
            }
#pragma unroll
            for (int e = 0; e < UB; ++e) t[e] = r1_upd(t[e], l, u[e]);
#pragma unroll
            for (int e = 0; e < UB; ++e) tile[(c + e * CG) * R + lr] = t[e];
          }
          for (; c < w; c += CG) tile[c * R + lr] = r1_upd(tile[c * R + lr], l, prow[c]);
        } else {
#pragma unroll 8
          for (; c < w; c += CG) tile[c * R + lr] = r1_upd(tile[c * R + lr], l, prow[c]);
        }
      }
    }
    // gather all keys; winner = largest |re|+|im|, lowest label on ties (the
    // barrier inside block_argmax also ends every read of prow above)
    u64 k = 0;
    int owner = -1;
    if (tid < G) {
      const u64* const pk[2] = {&cand[KEY_STRIDE * tid + 0], &cand[KEY_STRIDE * tid + 1]};
      uint32_t vk[2];
      ll_get_n<2>(pk, E, vk, &bad);
      k = ((u64)vk[0] << 32) | (0xffffffffu - vk[1]);
      owner = tid;
    }
    block_argmax(k, owner, skey2, sidx2);
    const int gp = owner;
    const uint32_t plabel = 0xffffffffu - (uint32_t)(k & 0xffffffffu);
    // pivot row, columns j..
    if (gp >= 0) {
      const int WW = WC * NW;
      const u64* src = rows + (size_t)gp * ws.wwmax;
      uint32_t* dstw = reinterpret_cast<uint32_t*>(prow + j);
      int t = tid;
      for (; t + 256 < WW; t += 512) {
        const u64* const pw[2] = {src + t, src + t + 256};
        uint32_t vw[2];
        ll_get_n<2>(pw, E, vw, &bad);
        dstw[t] = vw[0];
        dstw[t + 256] = vw[1];
      }
      if (t < WW) dstw[t] = ll_get(src + t, E, &bad);
    }
    // interchange of positions gj <-> plabel: swap labels (each row by one thread)
    if (plabel != (uint32_t)gj) {
      for (int lr = tid; lr < myR; lr += 256) {
        const int32_t lb = lab[lr];
        if (lb == (int32_t)gj) lab[lr] = (int32_t)plabel;
        else if (g == gp && lr == lrow) lab[lr] = (int32_t)gj;
      }
    }
    if (tid == 0) pl[j] = (int32_t)plabel;
    __syncthreads();
    if (bad || gp < 0) {
      if (tid == 0) __hip_atomic_store(&ws.err[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    const CT piv = prow[j];
    const bool zero = piv.x == 0 && piv.y == 0;
    if (zero && zero_col < 0) zero_col = j;
    CT inv;
    if (zero) { inv.x = 0; inv.y = 0; } else inv = cinv_t(piv);
    // multipliers of the rows below (labels > gj) into tile column j, and the
    // update of column j + 1 with the next pivot candidates
    best = 0;
    brow = -1;
    const bool nxt = j + 1 < w;
    const CT u1 = nxt ? prow[j + 1] : piv;
    for (int lr = tid; lr < myR; lr += 256) {
      const int32_t lb = lab[lr];
      if (lb <= (int32_t)gj) continue;
      const CT l = cmul_t(tile[j * R + lr], inv);
      tile[j * R + lr] = l;
      if (nxt) {
        const CT t = r1_upd(tile[(j + 1) * R + lr], l, u1);
        tile[(j + 1) * R + lr] = t;
        const u64 kk = pivot_key(t, (uint32_t)lb);
        if (kk > best) {
          best = kk;
          brow = lr;
        }
      }
    }
    // (the barrier inside the next block_argmax orders these writes before any read)
  }
  __syncthreads();
  if (g == 0) {
    for (int j = tid; j < w; j += 256) ipiv[k0 + j] = pl[j];
    if (tid == 0 && zero_col >= 0) atomicMin(&ws.err[1], (int)(k0 + zero_col));
  }
  for (int lr = tid; lr < myR; lr += 256) {
    const int32_t orig = (int32_t)(rbase + lr);
    if (lab[lr] != orig) {
      const int slot = __hip_atomic_fetch_add(mcount, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (slot < mcap) {
        mdst[slot] = lab[lr];
        msrc[slot] = orig;
      }
    }
  }
  for (int lr = tid; lr < myR; lr += 256) {
    CT* dst = A + lab[lr] + k0 * ld;
    for (int c0 = 0; c0 < wfull; c0 += LB) {
      CT v[LB];
#pragma unroll
      for (int u = 0; u < LB; ++u) v[u] = tile[(c0 + u) * R + lr];
#pragma unroll
      for (int u = 0; u < LB; ++u) dst[(c0 + u) * ld] = v[u];
    }
    for (int c = wfull; c < w; ++c) dst[c * ld] = tile[c * R + lr];
  }
}

// ---------------------------------------------------------------------------
// 1b. panel factorisation with tournament pivoting: one exchange per PB columns
// ---------------------------------------------------------------------------
// The columns of the panel are taken in inner steps of PB.  For the step's
// columns [j0, j0 + pw) the pivots are chosen by a tournament of partial
// pivotings, each on the original values of its candidates:
//   * every row workgroup picks up to PB candidate rows among its active rows
//     (one wave, partial pivoting on the step's columns) and publishes them:
//     their labels and step values, and their remaining columns;
//   * root workgroups (one per TP_ROOT_SPAN row workgroups, launched after
//     them) hold one candidate per thread; each wave picks PB among its 64,
//     then one wave PB among the 4 PB winners, and the root publishes them;
//   * every row workgroup reads the roots' winners (one per lane of one wave)
//     and picks the step's PB pivots among them.  The arithmetic is identical
//     everywhere, so all row workgroups agree on the pivots and on the factored
//     PB x PB pivot block (L11 strictly below the diagonal, U11 on and above).
// Then the U rows of the step (a pivot row's remaining columns, fetched from
// its owner, minus L11 times the earlier U rows) and, for every other active
// row, the multipliers l = a U11^-1 and the rank-pw update of its remaining
// columns: the next step's columns first (they decide its candidates), the
// candidates' remaining columns next (they are published), the rest after the
// publication, while the roots work.
// This is the tree form of communication-avoiding LU (tournament pivoting);
// with PB = 1 it would be plain partial pivoting, which panel_kernel
// implements.  Pivot keys and ties follow panel_kernel (largest |re| + |im| in
// FP32, lowest label); rows never move between workgroups, and interchanges
// swap labels.
//
// Exchange buffers (per batch item, double-buffered by the parity of the inner
// step; every 32-bit payload travels in an epoch-tagged 64-bit word):
//   records ws.cand [2][gitem][PB][K], K = 1 + PB NW: label, PB step values
//     (label 0xffffffff: no candidate);
//   root results after them, [2][ceil(gitem / TP_ROOT_SPAN)][PB][KR],
//     KR = 2 + PB NW: candidate index (workgroup PB + slot, 0xffffffff: none),
//     label, PB step values;
//   rows ws.rows [2][gitem][PB][wwmax]: a candidate's columns after the step.
constexpr int TP_ROOT_SPAN = 32;

template <typename CT>
__device__ inline CT rdlane(CT v, int l) {
  if constexpr (sizeof(CT) == 8) {
    CT r;
    r.x = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.x), l));
    r.y = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.y), l));
    return r;
  } else {
    auto rd = [&](double d) {
      const long long b = __double_as_longlong(d);
      const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
      const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
      return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
    };
    CT r;
    r.x = rd(v.x);
    r.y = rd(v.y);
    return r;
  }
}

// One step of partial pivoting inside a wave over the candidates its lanes hold
// (RL per lane: values v[r][0..PB), labels lab[r], live flags alive[r]): the
// live candidate with the largest |re| + |im| in column c (lowest label on ties)
// is chosen; its values pv (multipliers of the earlier steps before column c,
// its U row from c on) reach every lane; every other live candidate is
// eliminated.  wl / wsl: lane and slot of the chosen one (wave-uniform); inv:
// 1 / pv[c] (0 for a zero pivot).  Returns false if no live candidate is left.
template <typename CT, int PB, int RL>
__device__ __forceinline__ bool wave_pivot_step(int c, int pw, CT (&v)[RL][PB], const uint32_t (&lab)[RL], bool (&alive)[RL],
                                       CT (&pv)[PB], CT& inv, int& wl, int& wsl) {
  const int lane = threadIdx.x & 63;
  u64 best = 0;
  int bs = 0;
#pragma unroll
  for (int r = 0; r < RL; ++r)
    if (alive[r]) {
      const u64 k = pivot_key(v[r][c], lab[r]);
      if (k > best) {
        best = k;
        bs = r;
      }
    }
  const u64 wb = wave_max_u64(best);
  if (wb == 0) return false;
  const unsigned long long m = __ballot(best == wb);  // one lane: keys are unique
  wl = __builtin_amdgcn_readfirstlane(__ffsll((unsigned long long)m) - 1);
  wsl = __builtin_amdgcn_readlane(bs, wl);
  // the lane's chosen slot by register selects (the empty asm keeps the
  // compiler from turning the select chain into an indexed load from a stack
  // copy of v)
  CT mine[PB];
#pragma unroll
  for (int cc = 0; cc < PB; ++cc) {
    mine[cc] = v[0][cc];
#pragma unroll
    for (int r = 1; r < RL; ++r) {
      CT t = v[r][cc];
      asm volatile("" : "+v"(t.x), "+v"(t.y));
      mine[cc].x = bs == r ? t.x : mine[cc].x;
      mine[cc].y = bs == r ? t.y : mine[cc].y;
    }
  }
#pragma unroll
  for (int cc = 0; cc < PB; ++cc) pv[cc] = rdlane(mine[cc], wl);
  if (lane == wl)
#pragma unroll
    for (int r = 0; r < RL; ++r)
      if (r == bs) alive[r] = false;
  if (pv[c].x == 0 && pv[c].y == 0) {
    inv.x = 0;
    inv.y = 0;
  } else {
    inv = cinv_t(pv[c]);
  }
#pragma unroll
  for (int r = 0; r < RL; ++r)
    if (alive[r]) {
      const CT l = cmul_t(v[r][c], inv);
      v[r][c] = l;
#pragma unroll
      for (int cc = 0; cc < PB; ++cc)
        if (cc > c && cc < pw) v[r][cc] = r1_upd(v[r][cc], l, pv[cc]);
    }
  return true;
}

template <typename T, int PB>
__global__ void __launch_bounds__(256) panel_tp_kernel(cplx<T>* __restrict__ A, int64_t ld, int64_t n, int64_t k0,
                                                        int w, int R, int G, int32_t* __restrict__ ipiv, LUWork ws,
                                                        uint32_t epoch0, int64_t sA, int64_t sipiv,
                                                        int32_t* __restrict__ mdst, int32_t* __restrict__ msrc,
                                                        int32_t* __restrict__ mcount, int mcap) {
  using CT = cplx<T>;
  constexpr int NW = sizeof(CT) / 4;
  constexpr int K = 1 + PB * NW;   // words of a candidate record
  constexpr int KR = 2 + PB * NW;  // words of a root's winner
  A += (int64_t)blockIdx.y * sA;
  ipiv += (int64_t)blockIdx.y * sipiv;
  ws.cand += (int64_t)blockIdx.y * ws.s_cand;
  ws.rows += (int64_t)blockIdx.y * ws.s_rows;
  mdst += (int64_t)blockIdx.y * ws.s_pairs;
  msrc += (int64_t)blockIdx.y * ws.s_pairs;
  mcount += (int64_t)blockIdx.y * ws.s_npairs;
  const int g = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // an earlier panel's exchange failed (flag set before this launch): the
  // factorisation is lost, so do not wait out another exchange
  if (__hip_atomic_load(&ws.err[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
  const int NR = (G + TP_ROOT_SPAN - 1) / TP_ROOT_SPAN;
  const int nrmax = (ws.gitem + TP_ROOT_SPAN - 1) / TP_ROOT_SPAN;
  const size_t rec_par = (size_t)ws.gitem * PB * K;
  u64* const res_all = ws.cand + 2 * rec_par;
  const size_t res_par = (size_t)nrmax * PB * KR;
  const int nsteps = (w + PB - 1) / PB;
  __shared__ int bad;
  if (tid == 0) bad = 0;

  // ------------------------------------------------------------------ roots
  if (g >= G) {
    __shared__ uint32_t l1ci[4][PB], l1lab[4][PB];
    __shared__ CT l1v[4][PB][PB];
    const int r = g - G;
    const int cg = r * TP_ROOT_SPAN + tid / PB, cs = tid % PB;
    const bool have = tid < TP_ROOT_SPAN * PB && cg < G;
    __syncthreads();
    for (int s = 0; s < nsteps; ++s) {
      const int j0 = s * PB, pw = w - j0 < PB ? w - j0 : PB;
      const uint32_t E = epoch0 + (uint32_t)s;
      const int par = s & 1;
      const u64* rec = ws.cand + par * rec_par;
      const u64* base[1] = {rec + (size_t)(have ? cg * PB + cs : 0) * K};  // record 0 is always published
      uint32_t wd[K];
      ll_get_rec<K, 1>(base, E, wd, &bad);
      CT v[1][PB], v0[PB];
      uint32_t lb[1] = {wd[0]};
      bool al[1] = {have && wd[0] != 0xffffffffu};
#pragma unroll
      for (int c = 0; c < PB; ++c) {
        uint32_t* d = reinterpret_cast<uint32_t*>(&v0[c]);
#pragma unroll
        for (int q = 0; q < NW; ++q) d[q] = wd[1 + c * NW + q];
        v[0][c] = v0[c];
      }
      // level 1: PB winners of each wave, with their original values
      bool more = true;
#pragma unroll
      for (int c = 0; c < PB; ++c) {
        CT pv[PB], inv;
        int wl = 0, wsl = 0;
        if (c < pw && more) more = wave_pivot_step<CT, PB, 1>(c, pw, v, lb, al, pv, inv, wl, wsl);
        if (c < pw && more) {
          if (lane == wl) {
            l1ci[wv][c] = (uint32_t)(cg * PB + cs);
            l1lab[wv][c] = lb[0];
#pragma unroll
            for (int cc = 0; cc < PB; ++cc) l1v[wv][c][cc] = v0[cc];
          }
        } else if (lane == 0) {
          l1ci[wv][c] = 0xffffffffu;
        }
      }
      __syncthreads();
      // level 2 (wave 0): PB winners among the 4 PB, published with their original values
      if (wv == 0) {
        const int sw = lane / PB, sc = lane % PB;
        const bool in = lane < 4 * PB;
        uint32_t ci2 = in ? l1ci[sw][sc] : 0xffffffffu;
        uint32_t lb2[1] = {in ? l1lab[sw][sc] : 0u};
        bool al2[1] = {ci2 != 0xffffffffu};
        CT u0[PB], u[1][PB];
#pragma unroll
        for (int cc = 0; cc < PB; ++cc) {
          if (in) {
            u0[cc] = l1v[sw][sc][cc];
          } else {
            u0[cc].x = 0;
            u0[cc].y = 0;
          }
          u[0][cc] = u0[cc];
        }
        u64* res = res_all + par * res_par + (size_t)r * PB * KR;
        bool more2 = true;
#pragma unroll
        for (int c = 0; c < PB; ++c) {
          CT pv[PB], inv;
          int wl = 0, wsl = 0;
          if (c < pw && more2) more2 = wave_pivot_step<CT, PB, 1>(c, pw, u, lb2, al2, pv, inv, wl, wsl);
          const bool got = c < pw && more2;
          // the winner's lane (lane 0 for an empty slot) writes the slot's KR words
          if ((got && lane == wl) || (!got && lane == 0)) {
            u64* o = res + (size_t)c * KR;
            ll_put(&o[0], E, got ? ci2 : 0xffffffffu);
            ll_put(&o[1], E, got ? lb2[0] : 0u);
#pragma unroll
            for (int cc = 0; cc < PB; ++cc)
#pragma unroll
              for (int q = 0; q < NW; ++q) ll_put(&o[2 + cc * NW + q], E, got ? cword(u0[cc], q) : 0u);
          }
        }
      }
      __syncthreads();  // the level-1 slots are rewritten next step
      if (bad) break;
    }
    if (bad && tid == 0) __hip_atomic_store(&ws.err[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }

  // ------------------------------------------------------------ row workgroups
  extern __shared__ unsigned char smem_raw[];
  CT* tile = reinterpret_cast<CT*>(smem_raw);                        // [w][R], column c at tile + c R
  CT* prow = tile + (size_t)w * R;                                   // [PB][w] U rows of the step
  CT* sel = prow + (size_t)PB * w;                                   // [PB][R] scratch of the local choice (R > 256)
  int32_t* lab = reinterpret_cast<int32_t*>(sel + (size_t)PB * R);  // [R] row labels (final positions)
  int32_t* pl = lab + R;                                             // [w] pivot positions of this panel
  __shared__ CT blk[PB][PB];  // factored pivot block of the step
  __shared__ CT binv[PB];     // 1 / U11[c][c] (0 for a zero pivot)
  __shared__ int pci[PB];     // candidate index (workgroup PB + slot) of pivot c
  __shared__ int32_t plab[PB];  // label of pivot c's row when the step starts
  __shared__ int chosen[PB];  // local rows offered as candidates
  __shared__ int nch;
  __shared__ int zcol;        // first zero pivot column of this panel (-1: none)
  const int64_t rbase = k0 + (int64_t)g * R;
  const int myR = (int)(n - rbase < (int64_t)R ? (n - rbase > 0 ? n - rbase : 0) : R);
  if (tid == 0) zcol = -1;
  constexpr int LB = 128 / (int)sizeof(CT);
  const int wfull = w - w % LB;
  for (int lr = tid; lr < myR; lr += 256) {
    const CT* src = A + (rbase + lr) + k0 * ld;
    for (int c0 = 0; c0 < wfull; c0 += LB) {
      CT v[LB];
#pragma unroll
      for (int u = 0; u < LB; ++u) v[u] = src[(c0 + u) * ld];
#pragma unroll
      for (int u = 0; u < LB; ++u) tile[(c0 + u) * R + lr] = v[u];
    }
    for (int c = wfull; c < w; ++c) tile[c * R + lr] = src[c * ld];
  }
  for (int lr = tid; lr < myR; lr += 256) lab[lr] = (int32_t)(rbase + lr);
  // 2D mapping of the bulk update: RP rows x CG column groups
  int RP = 1;
  while (RP < myR && RP < 256) RP <<= 1;
  const int CG = 256 / RP;
  const int ulr0 = tid & (RP - 1), ucg = tid / RP;
  __syncthreads();

  // Local choice (wave 0): partial pivoting on columns [j1, j1 + pw1) of the
  // active rows (labels >= k0 + j1).  Up to 128 rows the lanes keep their rows
  // (lane, lane + 64) in registers; beyond that, in the LDS scratch.
  // Writes chosen[] and nch.
  auto local_choice = [&](int j1, int pw1) {
    if (wv != 0) return;
    const int32_t gj1 = (int32_t)(k0 + j1);
    int cnt = 0;
    if (myR <= 128) {
      constexpr int RL = 2;
      CT v[RL][PB];
      uint32_t lb[RL];
      bool al[RL];
#pragma unroll
      for (int i = 0; i < RL; ++i) {
        const int lr = lane + 64 * i;
        al[i] = lr < myR && lab[lr] >= gj1;
        lb[i] = al[i] ? (uint32_t)lab[lr] : 0u;
#pragma unroll
        for (int c = 0; c < PB; ++c) {
          v[i][c].x = 0;
          v[i][c].y = 0;
          if (al[i] && c < pw1) v[i][c] = tile[(j1 + c) * R + lr];
        }
      }
      bool more = true;
#pragma unroll
      for (int c = 0; c < PB; ++c) {
        CT pv[PB], inv;
        int wl = 0, wsl = 0;
        if (c < pw1 && more) more = wave_pivot_step<CT, PB, RL>(c, pw1, v, lb, al, pv, inv, wl, wsl);
        if (c < pw1 && more) {
          if (lane == 0) chosen[c] = wl + 64 * wsl;
          cnt = c + 1;
        }
      }
    } else {
      for (int lr = lane; lr < myR; lr += 64)
#pragma unroll
        for (int c = 0; c < PB; ++c)
          if (c < pw1) sel[c * R + lr] = tile[(j1 + c) * R + lr];
      uint32_t taken = 0;  // bit i: row lane + 64 i already chosen
      bool more = true;
#pragma unroll
      for (int c = 0; c < PB; ++c) {
        if (c < pw1 && more) {
          u64 best = 0;
          int blr = -1;
          for (int lr = lane, i = 0; lr < myR; lr += 64, ++i) {
            if (lab[lr] < gj1 || ((taken >> i) & 1u)) continue;
            const u64 kk = pivot_key(sel[c * R + lr], (uint32_t)lab[lr]);
            if (kk > best) {
              best = kk;
              blr = lr;
            }
          }
          const u64 wbest = wave_max_u64(best);
          if (wbest == 0) {
            more = false;  // no active row left
          } else {
            const int wl = __ffsll((unsigned long long)__ballot(best == wbest)) - 1;
            const int wlr = __shfl(blr, wl);
            if (lane == wl) taken |= 1u << ((wlr - lane) >> 6);
            if (lane == 0) chosen[c] = wlr;
            cnt = c + 1;
            CT pv[PB];
#pragma unroll
            for (int cc = 0; cc < PB; ++cc) {
              CT v = {0, 0};
              if (lane == wl && cc >= c && cc < pw1) v = sel[cc * R + wlr];
              pv[cc].x = __shfl(v.x, wl);
              pv[cc].y = __shfl(v.y, wl);
            }
            CT inv;
            if (pv[c].x == 0 && pv[c].y == 0) {
              inv.x = 0;
              inv.y = 0;
            } else {
              inv = cinv_t(pv[c]);
            }
            for (int lr = lane, i = 0; lr < myR; lr += 64, ++i) {
              if (lab[lr] < gj1 || ((taken >> i) & 1u)) continue;
              const CT l = cmul_t(sel[c * R + lr], inv);
#pragma unroll
              for (int cc = 0; cc < PB; ++cc)
                if (cc > c && cc < pw1) sel[cc * R + lr] = r1_upd(sel[cc * R + lr], l, pv[cc]);
            }
          }
        }
      }
    }
    if (lane == 0) nch = cnt;
  };
  auto is_chosen = [&](int lr) {
    bool r = false;
#pragma unroll
    for (int c = 0; c < PB; ++c) r = r || (c < nch && chosen[c] == lr);
    return r;
  };
  // Publish the candidates of step s (columns [j1, j1 + pw1)): records, then
  // the columns after the step.
  auto publish = [&](int s, int j1, int pw1) {
    const uint32_t E = epoch0 + (uint32_t)s;
    const int par = s & 1;
    u64* rec = ws.cand + par * rec_par + (size_t)g * PB * K;
    u64* rws = ws.rows + (size_t)par * ws.gitem * PB * ws.wwmax + (size_t)g * PB * ws.wwmax;
    for (int t = tid; t < PB * K; t += 256) {
      const int c = t / K, k = t % K;
      uint32_t v;
      if (c >= nch) {
        v = k == 0 ? 0xffffffffu : 0u;
      } else {
        const int lr = chosen[c];
        if (k == 0) {
          v = (uint32_t)lab[lr];
        } else {
          const int cc = (k - 1) / NW;
          v = cc < pw1 ? cword(tile[(j1 + cc) * R + lr], (k - 1) % NW) : 0u;
        }
      }
      ll_put(&rec[t], E, v);
    }
    const int WR = (w - j1 - pw1) * NW;
    for (int t = tid; t < nch * WR; t += 256) {
      const int c = t / WR, k = t % WR;
      ll_put(&rws[(size_t)c * ws.wwmax + k], E, cword(tile[(j1 + pw1 + k / NW) * R + chosen[c]], k % NW));
    }
  };

  local_choice(0, PB < w ? PB : w);
  __syncthreads();
  publish(0, 0, PB < w ? PB : w);
  for (int s = 0; s < nsteps; ++s) {
    const int j0 = s * PB, pw = w - j0 < PB ? w - j0 : PB;
    const int j1 = j0 + pw, pw1 = w - j1 < PB ? w - j1 : PB;
    const int32_t gj0 = (int32_t)(k0 + j0), gj1 = (int32_t)(k0 + j1);
    const uint32_t E = epoch0 + (uint32_t)s;
    const int par = s & 1;
    // --- the step's pivots: wave 0 chooses among the roots' winners ---
    if (wv == 0) {
      const bool in = lane < NR * PB;
      const u64* res = res_all + par * res_par;
      const u64* base[1] = {res + (size_t)(in ? lane : 0) * KR};  // root 0's slot 0 is always published
      uint32_t wd[KR];
      ll_get_rec<KR, 1>(base, E, wd, &bad);
      const uint32_t ci = in ? wd[0] : 0xffffffffu;
      uint32_t lb[1] = {wd[1]};
      bool al[1] = {ci != 0xffffffffu};
      CT v[1][PB];
#pragma unroll
      for (int c = 0; c < PB; ++c) {
        uint32_t* d = reinterpret_cast<uint32_t*>(&v[0][c]);
#pragma unroll
        for (int q = 0; q < NW; ++q) d[q] = wd[2 + c * NW + q];
      }
      bool more = true;
#pragma unroll
      for (int c = 0; c < PB; ++c) {
        CT pv[PB], inv;
        int wl = 0, wsl = 0;
        const uint32_t cic = ci, lbc = lb[0];  // before the step retires the winner
        if (c < pw && more) more = wave_pivot_step<CT, PB, 1>(c, pw, v, lb, al, pv, inv, wl, wsl);
        if (c < pw) {
          if (!more) {
            if (lane == 0) bad = 1;  // fewer candidates than columns: cannot happen
          } else {
            const uint32_t wci = (uint32_t)__builtin_amdgcn_readlane((int)cic, wl);
            const uint32_t wlb = (uint32_t)__builtin_amdgcn_readlane((int)lbc, wl);
            if (lane == 0) {
              pci[c] = (int)wci;
              plab[c] = (int32_t)wlb;
              binv[c] = inv;
#pragma unroll
              for (int cc = 0; cc < PB; ++cc) blk[c][cc] = pv[cc];
              if (pv[c].x == 0 && pv[c].y == 0 && zcol < 0) zcol = j0 + c;
            }
          }
        }
      }
    }
    __syncthreads();
    if (bad) {
      if (tid == 0) __hip_atomic_store(&ws.err[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    // --- positions of the pivots before their interchanges (LAPACK ipiv) ---
    int32_t ppos[PB];
#pragma unroll
    for (int c = 0; c < PB; ++c) {
      int32_t p = plab[c < pw ? c : 0];
#pragma unroll
      for (int cc = 0; cc < PB; ++cc)
        if (cc < c && p == gj0 + cc) p = ppos[cc];
      ppos[c] = p;
    }
    if (tid == 0)
#pragma unroll
      for (int c = 0; c < PB; ++c)
        if (c < pw) pl[j0 + c] = ppos[c];
    // which local row is pivot c (-1 if another workgroup owns it)
    int own[PB];
#pragma unroll
    for (int c = 0; c < PB; ++c) own[c] = (c < pw && pci[c] / PB == g) ? chosen[pci[c] % PB] : -1;
    // --- fetch the pivot rows' columns [j1, w) from their owners (at most 8
    // words per thread, all in flight together) ---
    {
      const int WR = (w - j1) * NW;
      const int tot = pw * WR;
      if (tot > 0) {
        const u64* rws = ws.rows + (size_t)par * ws.gitem * PB * ws.wwmax;
        uint32_t* p32 = reinterpret_cast<uint32_t*>(prow);
        constexpr int FB = 8;  // PB w NW <= 8 x 128 x 2 = 4 x 128 x 4 = 2048 = 8 x 256
        const u64* pp[FB];
#pragma unroll
        for (int i = 0; i < FB; ++i) {
          const int t = tid + 256 * i < tot ? tid + 256 * i : 0;
          const int c = t / WR, k = t % WR;
          const int ci = pci[c];
          pp[i] = rws + (size_t)(ci / PB) * PB * ws.wwmax + (size_t)(ci % PB) * ws.wwmax + k;
        }
        uint32_t wd[FB];
        ll_get_sel<FB>(pp, E, wd, &bad);
#pragma unroll
        for (int i = 0; i < FB; ++i) {
          const int t = tid + 256 * i;
          if (t < tot) p32[((size_t)(t / WR) * w + j1) * NW + t % WR] = wd[i];
        }
      }
    }
    // --- interchanges: labels of the pivot rows and of the rows they displace ---
    for (int lr = tid; lr < myR; lr += 256) {
      int32_t L = lab[lr];
      if (L < gj0) continue;
#pragma unroll
      for (int c = 0; c < PB; ++c) {
        if (c < pw) {
          if (own[c] == lr) L = gj0 + c;
          else if (L == gj0 + c) L = ppos[c];
        }
      }
      lab[lr] = L;
    }
    __syncthreads();
    // --- U rows: columns [j1, w) of pivot c minus L11[c][:c] times the earlier ones ---
    for (int col = j1 + tid; col < w; col += 256)
#pragma unroll
      for (int c = 1; c < PB; ++c) {
        if (c < pw) {
          CT u = prow[c * w + col];
#pragma unroll
          for (int cc = 0; cc < PB; ++cc)
            if (cc < c) u = r1_upd(u, blk[c][cc], prow[cc * w + col]);
          prow[c * w + col] = u;
        }
      }
    __syncthreads();
    // --- the step's rows: pivot rows get their factored values, every other
    // active row its multipliers and the update of the next step's columns ---
    for (int t = tid; t < pw * (w - j0); t += 256) {
      const int c = t / (w - j0), col = j0 + t % (w - j0);
      int lr = -1;
#pragma unroll
      for (int cc = 0; cc < PB; ++cc)
        if (cc == c) lr = own[cc];
      if (lr >= 0) tile[col * R + lr] = col < j1 ? blk[c][col - j0] : prow[c * w + col];
    }
    for (int lr = tid; lr < myR; lr += 256) {
      if (lab[lr] < gj1) continue;
      CT l[PB];
#pragma unroll
      for (int c = 0; c < PB; ++c) {
        l[c].x = 0;
        l[c].y = 0;
        if (c < pw) {
          CT a = tile[(j0 + c) * R + lr];
#pragma unroll
          for (int cc = 0; cc < PB; ++cc)
            if (cc < c) a = r1_upd(a, l[cc], blk[cc][c]);
          l[c] = cmul_t(a, binv[c]);
          tile[(j0 + c) * R + lr] = l[c];
        }
      }
#pragma unroll
      for (int cc = 0; cc < PB; ++cc) {
        if (cc < pw1) {
          CT a = tile[(j1 + cc) * R + lr];
#pragma unroll
          for (int c = 0; c < PB; ++c)
            if (c < pw) a = r1_upd(a, l[c], prow[c * w + j1 + cc]);
          tile[(j1 + cc) * R + lr] = a;
        }
      }
    }
    __syncthreads();
    if (j1 >= w) break;
    // --- candidates of the next step, their remaining columns, publication ---
    local_choice(j1, pw1);
    __syncthreads();
    {
      const int WC = w - j1 - pw1;
      for (int t = tid; t < nch * WC; t += 256) {
        const int c = t / WC, col = j1 + pw1 + t % WC;
        const int lr = chosen[c];
        CT a = tile[col * R + lr];
#pragma unroll
        for (int cc = 0; cc < PB; ++cc)
          if (cc < pw) a = r1_upd(a, tile[(j0 + cc) * R + lr], prow[cc * w + col]);
        tile[col * R + lr] = a;
      }
    }
    __syncthreads();
    publish(s + 1, j1, pw1);
    // --- the rest of the update, while the roots choose ---
    for (int lr = ulr0; lr < myR; lr += RP) {
      if (lab[lr] < gj1 || is_chosen(lr)) continue;
      CT l[PB];
#pragma unroll
      for (int c = 0; c < PB; ++c) {
        if (c < pw) {
          l[c] = tile[(j0 + c) * R + lr];
        } else {
          l[c].x = 0;
          l[c].y = 0;
        }
      }
      for (int col = j1 + pw1 + ucg; col < w; col += CG) {
        CT a = tile[col * R + lr];
#pragma unroll
        for (int c = 0; c < PB; ++c)
          if (c < pw) a = r1_upd(a, l[c], prow[c * w + col]);
        tile[col * R + lr] = a;
      }
    }
  }
  __syncthreads();
  if (bad && tid == 0) __hip_atomic_store(&ws.err[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (g == 0) {
    for (int j = tid; j < w; j += 256) ipiv[k0 + j] = pl[j];
    if (tid == 0 && zcol >= 0) atomicMin(&ws.err[1], (int)(k0 + zcol));
  }
  for (int lr = tid; lr < myR; lr += 256) {
    const int32_t orig = (int32_t)(rbase + lr);
    if (lab[lr] != orig) {
      const int slot = __hip_atomic_fetch_add(mcount, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (slot < mcap) {
        mdst[slot] = lab[lr];
        msrc[slot] = orig;
      }
    }
  }
  for (int lr = tid; lr < myR; lr += 256) {
    CT* dst = A + lab[lr] + k0 * ld;
    for (int c0 = 0; c0 < wfull; c0 += LB) {
      CT v[LB];
#pragma unroll
      for (int u = 0; u < LB; ++u) v[u] = tile[(c0 + u) * R + lr];
#pragma unroll
      for (int u = 0; u < LB; ++u) dst[(c0 + u) * ld] = v[u];
    }
    for (int c = wfull; c < w; ++c) dst[c * ld] = tile[c * R + lr];
  }
}

// ---------------------------------------------------------------------------
// 2. row permutations (a block's moved rows, listed by its panel)
// ---------------------------------------------------------------------------
// X[dst[t], col] = Xold[src[t], col] for the columns [c0, c0 + ncols).
template <typename T>
__global__ void __launch_bounds__(256) row_permute_kernel(cplx<T>* __restrict__ X, int64_t ld, int64_t c0,
                                                          const int32_t* __restrict__ dst, const int32_t* __restrict__ src,
                                                          const int32_t* __restrict__ npairs, int64_t sX, int64_t spairs,
                                                          int64_t snpairs) {
  using CT = cplx<T>;
  X += (int64_t)blockIdx.y * sX;  // batch item blockIdx.y
  dst += (int64_t)blockIdx.y * spairs;
  src += (int64_t)blockIdx.y * spairs;
  npairs += (int64_t)blockIdx.y * snpairs;
  const int np = *npairs;
  const int64_t col = c0 + blockIdx.x;
  CT* x = X + col * ld;
  CT v[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int t = threadIdx.x + 256 * i;
    if (t < np) v[i] = x[src[t]];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int t = threadIdx.x + 256 * i;
    if (t < np) x[dst[t]] = v[i];
  }
}

// inverse: Xnew[src[t]] = Xold[dst[t]] (for the transposed solve)
template <typename T>
__global__ void __launch_bounds__(256) row_permute_inv_kernel(cplx<T>* __restrict__ X, int64_t ld, int64_t c0,
                                                              const int32_t* __restrict__ dst, const int32_t* __restrict__ src,
                                                              const int32_t* __restrict__ npairs, int64_t sX,
                                                              int64_t spairs, int64_t snpairs) {
  using CT = cplx<T>;
  X += (int64_t)blockIdx.y * sX;  // batch item blockIdx.y
  dst += (int64_t)blockIdx.y * spairs;
  src += (int64_t)blockIdx.y * spairs;
  npairs += (int64_t)blockIdx.y * snpairs;
  const int np = *npairs;
  const int64_t col = c0 + blockIdx.x;
  CT* x = X + col * ld;
  CT v[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int t = threadIdx.x + 256 * i;
    if (t < np) v[i] = x[dst[t]];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int t = threadIdx.x + 256 * i;
    if (t < np) x[src[t]] = v[i];
  }
}

// ---------------------------------------------------------------------------
// 3. small triangular solves op(Tri) X = B for a w x ncols block B (in place)
// ---------------------------------------------------------------------------
// KIND 0: L unit lower (forward)        KIND 1: U upper non-unit (backward)
// KIND 2: U^T lower non-unit (forward)  KIND 3: L^T upper unit (backward)
// Wave-synchronous substitution (w <= 128): each wave owns CPW columns of B in
// registers, lane l holding rows l and l + 64; x_j is broadcast from its owner
// lane with readlane, so the w sequential steps need no workgroup barrier.  The
// columns of op(Tri) are staged in LDS, PW at a time, shared by the 4 waves.
constexpr int TRSM_LS_BYTES = 64 * 1024;

__device__ inline float2 readlane_c(float2 v, int l) {
  return make_float2(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.x), l)),
                     __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.y), l)));
}
__device__ inline double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ inline double2 readlane_c(double2 v, int l) { return make_double2(readlane_d(v.x, l), readlane_d(v.y, l)); }

// Substitution sweep on register-resident columns b (lane l holds rows l, l+64).
template <typename T, int KIND, int CPW>
__device__ inline void trsm_sweep(const cplx<T>* __restrict__ Tri, int64_t ldt, int w, cplx<T> (&b)[2][CPW],
                                  cplx<T>* Ls, int PW) {
  using CT = cplx<T>;
  const int tid = threadIdx.x, lane = tid & 63;
  constexpr bool forward = (KIND == 0 || KIND == 2);
  constexpr bool unit = (KIND == 0 || KIND == 3);
  constexpr bool transposed = (KIND >= 2);
  // this lane's two rows, clamped into the staged column (masked below)
  const int i0 = lane < w ? lane : w - 1, i1 = lane + 64 < w ? lane + 64 : w - 1;
  for (int ph = 0; ph < w; ph += PW) {
    const int pw = w - ph < PW ? w - ph : PW;
    // columns of op(Tri) handled in this phase: [jb, jb + pw); rows needed: [lo, hi)
    const int jb = forward ? ph : w - ph - pw;
    const int lo = forward ? jb : 0;
    const int hi = forward ? w : jb + pw;
    const int len = hi - lo;
    __syncthreads();
    // staged in batches of SB loads in flight per thread (then a remainder)
    constexpr int SB = 128 / (int)sizeof(CT);
    const int tot = pw * len, full = tot - tot % (256 * SB);
    auto at = [&](int idx, int& i, int& cc) {
      if (!transposed) { i = lo + idx % len; cc = idx / len; }
      else { cc = idx % pw; i = lo + idx / pw; }
    };
    for (int base = tid; base < full; base += 256 * SB) {
      CT v[SB];
#pragma unroll
      for (int u = 0; u < SB; ++u) {
        int i, cc;
        at(base + 256 * u, i, cc);
        const int j = jb + cc;
        v[u] = transposed ? Tri[j + (int64_t)i * ldt] : Tri[i + (int64_t)j * ldt];
      }
#pragma unroll
      for (int u = 0; u < SB; ++u) {
        int i, cc;
        at(base + 256 * u, i, cc);
        Ls[cc * w + i] = v[u];
      }
    }
    for (int idx = full + tid; idx < tot; idx += 256) {
      int i, cc;
      at(idx, i, cc);
      const int j = jb + cc;
      Ls[cc * w + i] = transposed ? Tri[j + (int64_t)i * ldt] : Tri[i + (int64_t)j * ldt];
    }
    __syncthreads();
    // Columns [jb, jb + pw) in order; x_j sits in lane j & 63 of half j >> 6, so
    // the sweep is split at column 64 to make that half a compile-time choice.
    // The L entries of the next steps do not depend on x: with no branches in
    // the loop their LDS reads can run ahead of the substitution chain.
    auto sweep = [&](auto half, int ja, int jz) __attribute__((always_inline)) {
      constexpr int H = decltype(half)::value;
      const int cnt = jz - ja;
      if (cnt <= 0) return;
      // this lane's entries of the next column, read one step ahead
      const CT* lnext = Ls + ((forward ? ja : jz - 1) - jb) * w;
      CT n0 = lnext[i0], n1 = lnext[i1];
      for (int s = 0; s < cnt; ++s) {
        const int j = forward ? ja + s : jz - 1 - s;
        const CT* lcol = Ls + (j - jb) * w;
        const CT l0 = n0, l1 = n1;
        if (s + 1 < cnt) {
          lnext = lcol + (forward ? w : -w);
          n0 = lnext[i0];
          n1 = lnext[i1];
        }
        const bool a0 = forward ? (lane > j && lane < w) : (lane < j);
        const bool a1 = forward ? (lane + 64 > j && lane + 64 < w) : (lane + 64 < j);
        CT x[CPW];
#pragma unroll
        for (int c = 0; c < CPW; ++c) x[c] = readlane_c(b[H][c], j & 63);
        if (!unit) {
          const CT inv = cinv_t(lcol[j]);
#pragma unroll
          for (int c = 0; c < CPW; ++c) {
            x[c] = cmul_t(x[c], inv);
            if (lane == (j & 63)) b[H][c] = x[c];
          }
        }
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
          CT u0 = b[0][c], u1 = b[1][c];
          u0.x -= l0.x * x[c].x - l0.y * x[c].y;
          u0.y -= l0.x * x[c].y + l0.y * x[c].x;
          u1.x -= l1.x * x[c].x - l1.y * x[c].y;
          u1.y -= l1.x * x[c].y + l1.y * x[c].x;
          b[0][c].x = a0 ? u0.x : b[0][c].x;
          b[0][c].y = a0 ? u0.y : b[0][c].y;
          b[1][c].x = a1 ? u1.x : b[1][c].x;
          b[1][c].y = a1 ? u1.y : b[1][c].y;
        }
      }
    };
    const int je = jb + pw;
    if (forward) {
      if (jb < 64) sweep(std::integral_constant<int, 0>{}, jb, je < 64 ? je : 64);
      if (je > 64) sweep(std::integral_constant<int, 1>{}, jb > 64 ? jb : 64, je);
    } else {
      if (je > 64) sweep(std::integral_constant<int, 1>{}, jb > 64 ? jb : 64, je);
      if (jb < 64) sweep(std::integral_constant<int, 0>{}, jb, je < 64 ? je : 64);
    }
  }
}

// Inverse of the diagonal triangle of blocks b0 + blockIdx.y (UPPER 0: unit lower
// L11, 1: non-unit upper U11) by substitution on identity columns; written to
// Dinv[b] (nb x nb column-major, zeros in the other triangle).
template <typename T, int UPPER, int CPW>
__global__ void __launch_bounds__(256) block_inv_kernel(const cplx<T>* __restrict__ A, int64_t ld, int64_t n, int nb,
                                                        int b0, cplx<T>* __restrict__ Dinv, int PW, int64_t sA,
                                                        int64_t sD) {
  using CT = cplx<T>;
  A += (int64_t)blockIdx.z * sA;  // batch item blockIdx.z
  Dinv += (int64_t)blockIdx.z * sD;
  extern __shared__ unsigned char smem_raw[];
  CT* Ls = reinterpret_cast<CT*>(smem_raw);
  const int bb = b0 + blockIdx.y;
  const int64_t k0 = (int64_t)bb * nb;
  const int w = (int)(n - k0 < nb ? n - k0 : nb);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col0 = blockIdx.x * (4 * CPW) + wave * CPW;
  CT b[2][CPW];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      b[h][c].x = (lane + 64 * h == col0 + c) ? 1 : 0;
      b[h][c].y = 0;
    }
  trsm_sweep<T, UPPER ? 1 : 0, CPW>(A + k0 + k0 * ld, ld, w, b, Ls, PW);
  CT* D = Dinv + (size_t)bb * nb * nb;
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const int i = lane + 64 * h;
      if (i < w && col0 + c < w) D[i + (int64_t)(col0 + c) * nb] = b[h][c];
    }
}

// X <- L11^-1 X in place for ncols columns of X (the rows of block b0, leading
// dimension ldx): the forward substitution of block_inv_kernel applied to the
// columns of X instead of identity columns (the look-ahead U12 block, without
// waiting for the triangle's inverse).
// PERM: first the block's row interchanges on each owned column (rows [k0, n),
// X pointing at row k0; moved rows as listed by the panel), as
// row_permute_kernel does, so that one launch replaces two.
template <typename T, int CPW, bool PERM>
__global__ void __launch_bounds__(256) block_trsm_kernel(const cplx<T>* __restrict__ A, int64_t ld, int64_t n, int nb,
                                                         int b0, cplx<T>* __restrict__ X, int64_t ldx, int ncols,
                                                         int PW, int64_t sA, int64_t sX, const int32_t* __restrict__ dst,
                                                         const int32_t* __restrict__ src,
                                                         const int32_t* __restrict__ npairs, int64_t spairs,
                                                         int64_t snpairs) {
  using CT = cplx<T>;
  A += (int64_t)blockIdx.z * sA;  // batch item blockIdx.z
  X += (int64_t)blockIdx.z * sX;
  extern __shared__ unsigned char smem_raw[];
  CT* Ls = reinterpret_cast<CT*>(smem_raw);
  const int64_t k0 = (int64_t)b0 * nb;
  const int w = (int)(n - k0 < nb ? n - k0 : nb);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col0 = blockIdx.x * (4 * CPW) + wave * CPW;
  if constexpr (PERM) {
    dst += (int64_t)blockIdx.z * spairs;
    src += (int64_t)blockIdx.z * spairs;
    const int np = npairs[(int64_t)blockIdx.z * snpairs];  // <= 2 nb <= 256
    CT v[CPW][4];
#pragma unroll
    for (int c = 0; c < CPW; ++c)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int t = lane + 64 * q;
        if (t < np && col0 + c < ncols) v[c][q] = X[(src[t] - k0) + (int64_t)(col0 + c) * ldx];
      }
    __syncthreads();  // every source read before any destination is written
#pragma unroll
    for (int c = 0; c < CPW; ++c)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int t = lane + 64 * q;
        if (t < np && col0 + c < ncols) X[(dst[t] - k0) + (int64_t)(col0 + c) * ldx] = v[c][q];
      }
    __syncthreads();  // the interchanged rows visible to the whole workgroup
  }
  CT b[2][CPW];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const int i = lane + 64 * h;
      b[h][c].x = 0;
      b[h][c].y = 0;
      if (i < w && col0 + c < ncols) b[h][c] = X[i + (int64_t)(col0 + c) * ldx];
    }
  trsm_sweep<T, 0, CPW>(A + k0 + k0 * ld, ld, w, b, Ls, PW);  // every wave takes part (barriers)
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const int i = lane + 64 * h;
      if (i < w && col0 + c < ncols) X[i + (int64_t)(col0 + c) * ldx] = b[h][c];
    }
}

// Diagonal block of block b0 + blockIdx.y: strict lower <- -Linv (UPPER 0), or
// upper incl. diagonal <- I - Uinv (UPPER 1).  MODE 2: the strict lower part
// of Dinv itself <- -Linv (A untouched); MODE 3: strict lower <- that part of
// Dinv as it stands (after MODE 2).
template <typename T, int UPPER>
__global__ void __launch_bounds__(256) diag_store_kernel(cplx<T>* __restrict__ A, int64_t ld, int64_t n, int nb, int b0,
                                                         cplx<T>* __restrict__ Dinv, int64_t sA, int64_t sD) {
  using CT = cplx<T>;
  A += (int64_t)blockIdx.z * sA;  // batch item blockIdx.z
  Dinv += (int64_t)blockIdx.z * sD;
  const int bb = b0 + blockIdx.y;
  const int64_t k0 = (int64_t)bb * nb;
  const int w = (int)(n - k0 < nb ? n - k0 : nb);
  CT* D = Dinv + (size_t)bb * nb * nb;
  for (int idx = blockIdx.x * 256 + threadIdx.x; idx < w * w; idx += gridDim.x * 256) {
    const int i = idx % w, j = idx / w;
    const CT d = D[i + (int64_t)j * nb];
    CT v;
    if (UPPER != 1) {
      if (i <= j) continue;
      v = d;
      if (UPPER != 3) {
        v.x = -d.x;
        v.y = -d.y;
      }
    } else {
      if (i > j) continue;
      v.x = (i == j ? 1 : 0) - d.x;
      v.y = -d.y;
    }
    if (UPPER == 2) D[i + (int64_t)j * nb] = v;
    else A[(k0 + i) + (k0 + j) * ld] = v;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) copy_block_kernel(const cplx<T>* __restrict__ S, int64_t lds,
                                                         cplx<T>* __restrict__ D, int64_t ldd, int64_t m, int64_t n,
                                                         int64_t sS, int64_t sD) {
  S += (int64_t)blockIdx.z * sS;  // batch item blockIdx.z
  D += (int64_t)blockIdx.z * sD;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  for (int64_t j = blockIdx.y; j < n; j += gridDim.y) D[i + j * ldd] = S[i + j * lds];
}

template <typename T>
static hipError_t launch_copy_block(const cplx<T>* S, int64_t lds, cplx<T>* D, int64_t ldd, int64_t m, int64_t n,
                                    hipStream_t st, int nbatch = 1, int64_t sS = 0, int64_t sD = 0) {
  if (m <= 0 || n <= 0 || nbatch <= 0) return hipSuccess;
  const unsigned gy = (unsigned)(n < 65535 ? n : 65535);
  hipLaunchKernelGGL(copy_block_kernel<T>, dim3((unsigned)((m + 255) / 256), gy, (unsigned)nbatch), dim3(256), 0, st, S,
                     lds, D, ldd, m, n, sS, sD);
  return hipGetLastError();
}

static int trsm_pw(int w, int elem) {
  int PW = TRSM_LS_BYTES / (w * 2 * elem);
  if (PW < 1) PW = 1;
  if (PW > w) PW = w;
  return PW;
}

// One column of the inverse per wave keeps the per-step work of the substitution
// chain minimal (the chain, not the arithmetic, sets the time of one triangle);
// with many triangles at once (more workgroups than CUs) four columns per wave
// stage each triangle into LDS four times less often.
// STORE: diag_store_kernel mode applied after the inverse (UPPER by default).
template <typename T, int UPPER, int STORE = UPPER>
static hipError_t launch_block_inv(const cplx<T>* A, int64_t ld, int64_t n, int nb, int b0, int nblocks, cplx<T>* Dinv,
                                   hipStream_t st, int nbatch, int64_t sA, int64_t sD, int ncu) {
  if (nblocks <= 0 || nbatch <= 0) return hipSuccess;
  const int PW = trsm_pw(nb, (int)sizeof(T));
  const size_t lds = (size_t)PW * nb * sizeof(cplx<T>);
  const dim3 g1((unsigned)((nb + 3) / 4), (unsigned)nblocks, (unsigned)nbatch);
  if ((int64_t)g1.x * nblocks * nbatch <= ncu) {
    hipLaunchKernelGGL((block_inv_kernel<T, UPPER, 1>), g1, dim3(256), lds, st, A, ld, n, nb, b0, Dinv, PW, sA, sD);
  } else {
    const dim3 g4((unsigned)((nb + 15) / 16), (unsigned)nblocks, (unsigned)nbatch);
    hipLaunchKernelGGL((block_inv_kernel<T, UPPER, 4>), g4, dim3(256), lds, st, A, ld, n, nb, b0, Dinv, PW, sA, sD);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((diag_store_kernel<T, STORE>), dim3(16, (unsigned)nblocks, (unsigned)nbatch), dim3(256), 0, st,
                     const_cast<cplx<T>*>(A), ld, n, nb, b0, Dinv, sA, sD);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_block_trsm(const cplx<T>* A, int64_t ld, int64_t n, int nb, int b0, cplx<T>* X, int64_t ldx,
                                   int64_t ncols, hipStream_t st, int nbatch, int64_t sA, int64_t sX,
                                   const int32_t* dst = nullptr, const int32_t* src = nullptr,
                                   const int32_t* npairs = nullptr, int64_t spairs = 0, int64_t snpairs = 0) {
  if (ncols <= 0 || nbatch <= 0) return hipSuccess;
  const int PW = trsm_pw(nb, (int)sizeof(T));
  const size_t lds = (size_t)PW * nb * sizeof(cplx<T>);
  const dim3 g((unsigned)((ncols + 3) / 4), 1, (unsigned)nbatch);
  if (npairs)
    hipLaunchKernelGGL((block_trsm_kernel<T, 1, true>), g, dim3(256), lds, st, A, ld, n, nb, b0, X, ldx, (int)ncols,
                       PW, sA, sX, dst, src, npairs, spairs, snpairs);
  else
    hipLaunchKernelGGL((block_trsm_kernel<T, 1, false>), g, dim3(256), lds, st, A, ld, n, nb, b0, X, ldx, (int)ncols,
                       PW, sA, sX, dst, src, npairs, spairs, snpairs);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 1c. speculative panel: diagonal pivots, checked against partial pivoting
// ---------------------------------------------------------------------------
// Partial pivoting keeps the diagonal entry of column j as its pivot exactly
// when no entry below it is larger in |re| + |im| (compared in FP32, lowest row
// on ties: the rule of panel_kernel).  The coupling matrices of dielectric
// structures are diagonally dominant enough for that to hold in every column,
// and then the panel needs no pivot search at all: one workgroup factors the
// diagonal block, and the rows below follow from L21 = A21 U11^-1, a
// triangular solve per row.  The entries partial pivoting would have compared
// in column j are a_ij = l_ij u_jj (the column after the eliminations of the
// earlier columns), so each kernel checks |a_ij| <= |u_jj| for its rows; a
// failure, a zero pivot or a NaN sets the block's flag, and the caller repeats
// the factorisation with the pivot search (panel_kernel).  When no flag is set
// the factors are those of partial pivoting, up to the rounding order of the
// entries compared (near-ties within FP32 rounding may resolve either way).
template <typename CT>
__device__ inline float cabs1_f(const CT& v) {
  return (float)(fabs(v.x) + fabs(v.y));
}

// Diagonal block (w x w at (k0, k0)) of batch item blockIdx.y, NT threads:
// thread (tx, ty) = (tid % 32, tid / 32) holds rows tx + 32 p (p < 4) and
// columns ty + TY q (q < 128 / TY, TY = NT / 32) in registers.  Per column j
// the pivot row and the pivot column go through LDS (double-buffered by the
// parity of j, one barrier per column); each thread reads all the entries it
// needs at once and forms the multipliers of its rows itself.  Row and column
// groups wholly at or before j are skipped (uniform branches), groups wholly
// after it take a plain update and only the groups holding row or column j a
// masked one, so the work per column follows the shrinking triangle (the VALU
// of one CU sets the time: 64 lanes per cycle).  NT = 512: 32 entries per
// thread, two waves per SIMD.
template <typename T, int NT>
__global__ void __launch_bounds__(NT) spec_diag_kernel(cplx<T>* __restrict__ A, int64_t ld, int64_t k0, int w,
                                                        int32_t* __restrict__ ipiv, int32_t* __restrict__ flag,
                                                        int64_t sA, int64_t sipiv, int64_t sflag) {
  using CT = cplx<T>;
  constexpr int TY = NT / 32, Q = 128 / TY;
  A += (int64_t)blockIdx.y * sA;  // batch item blockIdx.y
  ipiv += (int64_t)blockIdx.y * sipiv;
  flag += (int64_t)blockIdx.y * sflag;
  __shared__ CT rowb[2][128], colb[2][128];
  const int tid = threadIdx.x, tx = tid & 31, ty = tid >> 5;
  CT* D = A + k0 + k0 * ld;
  CT a[4][Q];
  static_for<4>([&](auto p) {
    static_for<Q>([&](auto q) {
      const int r = tx + 32 * p, c = ty + TY * q;
      a[p][q].x = 0;
      a[p][q].y = 0;
      if (r < w && c < w) a[p][q] = D[r + (int64_t)c * ld];
    });
  });
  bool bad = false;
  for (int j = 0; j < w; ++j) {
    const int par = j & 1;
    const int jp = j >> 5, jr = j & 31;  // row group and lane index of row j
    const int jq = j / TY, jc = j % TY;  // column group and index of column j
    if (tx == jr) {
      static_for<4>([&](auto p) {
        if (p == jp) static_for<Q>([&](auto q) { rowb[par][ty + TY * q] = a[p][q]; });
      });
    }
    if (ty == jc) {
      static_for<Q>([&](auto q) {
        if (q == jq) static_for<4>([&](auto p) { colb[par][tx + 32 * p] = a[p][q]; });
      });
    }
    __syncthreads();
    CT u[Q], v[4];
    static_for<Q>([&](auto q) { u[q] = rowb[par][ty + TY * q]; });
    static_for<4>([&](auto p) { v[p] = colb[par][tx + 32 * p]; });
    const CT piv = rowb[par][j];
    const float pk = cabs1_f(piv);
    if (!(pk > 0.f)) bad = true;  // zero or NaN pivot
    const CT inv = cinv_t(piv);
    // groups wholly below / right of j take the plain update; the group holding
    // row j (p == jp) or column j (q == jq) the masked one
    static_for<4>([&](auto p) {
      if (p < jp) return;
      const bool pfull = p > jp;
      const bool below = pfull || tx > jr;
      const CT l = cmul_t(v[p], inv);
      if (below && ty == jc && !(cabs1_f(v[p]) <= pk)) bad = true;
      static_for<Q>([&](auto q) {
        if (q < jq) return;
        if (pfull && q > jq) {
          a[p][q] = r1_upd(a[p][q], l, u[q]);
          return;
        }
        const int c = ty + TY * q;
        const CT t = r1_upd(a[p][q], l, u[q]);
        const bool upd = below && c > j;
        const bool mul = below && c == j;
        a[p][q].x = upd ? t.x : (mul ? l.x : a[p][q].x);
        a[p][q].y = upd ? t.y : (mul ? l.y : a[p][q].y);
      });
    });
  }
  static_for<4>([&](auto p) {
    static_for<Q>([&](auto q) {
      const int r = tx + 32 * p, c = ty + TY * q;
      if (r < w && c < w) D[r + (int64_t)c * ld] = a[p][q];
    });
  });
  if (tid < w) ipiv[k0 + tid] = (int32_t)(k0 + tid);
  if (__syncthreads_or(bad) && tid == 0) atomicOr(flag, 1);
}

// The check of the rows below the diagonal block once L21 is formed:
// |l_ij u_jj| <= |u_jj| in |re| + |im| (FP32): the entry partial pivoting
// would compare with the pivot u_jj at step j is a_ij = l_ij u_jj, and the
// diagonal keeps the pivot only if no such entry is larger (ties to the lower
// row index).  Threads along the rows (coalesced), blockIdx.y over groups of
// 16 columns.
template <typename T>
__global__ void __launch_bounds__(256) spec_check_kernel(const cplx<T>* __restrict__ A, int64_t ld, int64_t n,
                                                          int64_t k0, int w, int32_t* __restrict__ flag, int64_t sA,
                                                          int64_t sflag) {
  using CT = cplx<T>;
  A += (int64_t)blockIdx.z * sA;
  flag += (int64_t)blockIdx.z * sflag;
  constexpr int CG = 16;
  const int j0 = blockIdx.y * CG;
  __shared__ CT dg[CG];
  __shared__ float pk[CG];
  if (threadIdx.x < CG) {
    const int j = j0 + threadIdx.x;
    CT d;
    d.x = 0;
    d.y = 0;
    if (j < w) d = A[(k0 + j) + (k0 + j) * ld];
    dg[threadIdx.x] = d;
    pk[threadIdx.x] = cabs1_f(d);
  }
  __syncthreads();
  const int64_t r = k0 + w + (int64_t)blockIdx.x * 256 + threadIdx.x;
  bool bad = false;
  if (r < n) {
    const int jn = w - j0 < CG ? w - j0 : CG;
    CT x[CG];
#pragma unroll
    for (int c = 0; c < CG; ++c)
      if (c < jn) x[c] = A[r + (k0 + j0 + c) * ld];
#pragma unroll
    for (int c = 0; c < CG; ++c)
      if (c < jn && !(cabs1_f(cmul_t(x[c], dg[c])) <= pk[c])) bad = true;
  }
  if (__ballot(bad) != 0 && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// Speculative panel of block bi (columns [k0, k0 + w)): the diagonal block
// (launch_spec_diag), then (launch_spec_l21) L21 = A21 U11^-1 for the rows below
// as U11^-1 (into the block's inverse slot, which later steps overwrite only
// after this panel) and one GEMM from a copy of A21, then the check.  (A row-parallel substitution x U11 = a on the
// VALUs, with U11 staged in LDS, took 115 us per early FP32 block beside the
// bulk update and 590 us in FP64, where the staged triangle fills 132 KB of a
// CU's LDS; the inverse + GEMM form: FP32 factorisation 59.5 -> 59.2 ms, FP64
// 110.3 -> 108.7 ms at n = 12 000.)
template <typename T>
static hipError_t launch_spec_diag(cplx<T>* A, int64_t ld, int nb, int bi, int64_t k0, int w, int32_t* ipiv,
                                   const LUWork& ws, hipStream_t st, int nbatch, int64_t sA, int64_t sipiv) {
  if (w > 128 || !ws.l21c || k0 != (int64_t)bi * nb) return hipErrorInvalidValue;
  int32_t* flag = ws.spec + bi;
  const int64_t sflag = ws.s_npairs;
  constexpr int NT = 512;
  // One system: the diagonal kernel reserves (without using it) nearly all of
  // its CU's LDS, so that no workgroup of the concurrent bulk update shares
  // that CU's VALUs with its 128-step chain.  It is launched before the
  // step's bulk update, so a free CU is there to take it.  Measured at
  // n = 12 000: FP32+IR step 69.7 -> 69.1 ms, FP64 103.4 -> 103.0 ms, adjoint
  // (n = 6000, FP32+IR) 23.9 -> 23.2 ms.
  size_t reserve = 0;
  if (nbatch == 1) {
    static std::once_flag once;
    static size_t bytes = 0;
    static hipError_t attr = hipSuccess;
    std::call_once(once, [] {
      int dev = 0, cu_lds = 0;
      attr = hipGetDevice(&dev);
      if (attr == hipSuccess)
        attr = hipDeviceGetAttribute(&cu_lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev);
      // the static 4 KB of the kernel and a margin stay free
      if (attr == hipSuccess && cu_lds > 96 * 1024) {
        bytes = (size_t)cu_lds - 12 * 1024;
        attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&spec_diag_kernel<float, NT>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (attr == hipSuccess)
          attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&spec_diag_kernel<double, NT>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
      }
    });
    if (attr != hipSuccess) return attr;
    reserve = bytes;
  }
  hipLaunchKernelGGL((spec_diag_kernel<T, NT>), dim3(1, (unsigned)nbatch), dim3(NT), reserve, st, A, ld, k0, w, ipiv,
                     flag, sA, sipiv, sflag);
  return hipGetLastError();
}

// The rest of the speculative panel of block bi: L21 (w columns below the
// diagonal block) and the check of its entries against the pivots.
template <typename T>
static hipError_t launch_spec_l21(cplx<T>* A, int64_t ld, int64_t n, int nb, int bi, int64_t k0, int w,
                                  const LUWork& ws, hipStream_t st, int nbatch, int64_t sA) {
  using CT = cplx<T>;
  int32_t* flag = ws.spec + bi;
  const int64_t sflag = ws.s_npairs;
  hipError_t e;
  const int64_t nr = n - k0 - w;
  if (nr <= 0) return hipSuccess;
  CT* dinv = static_cast<CT*>(ws.dinv);
  const int PW = trsm_pw(nb, (int)sizeof(T));
  const size_t lds = (size_t)PW * nb * sizeof(CT);
  const dim3 g1((unsigned)((nb + 3) / 4), 1, (unsigned)nbatch);
  if ((int64_t)g1.x * nbatch <= ws.gmax) {
    hipLaunchKernelGGL((block_inv_kernel<T, 1, 1>), g1, dim3(256), lds, st, A, ld, n, nb, bi, dinv, PW, sA, ws.s_dinv);
  } else {
    const dim3 g4((unsigned)((nb + 15) / 16), 1, (unsigned)nbatch);
    hipLaunchKernelGGL((block_inv_kernel<T, 1, 4>), g4, dim3(256), lds, st, A, ld, n, nb, bi, dinv, PW, sA, ws.s_dinv);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  CT* l21 = A + (k0 + w) + k0 * ld;
  CT* cp = static_cast<CT*>(ws.l21c);
  if ((e = launch_copy_block<T>(l21, ld, cp, nr, nr, w, st, nbatch, sA, ws.s_l21c)) != hipSuccess) return e;
  GemmMask mk;
  mk.bkind = GEMM_MASK_UPPER;
  if ((e = launch_gemm<T>(1, 0, nr, w, w, cp, nr, dinv + (size_t)bi * nb * nb, nb, l21, ld, st, mk, nbatch, ws.s_l21c,
                          ws.s_dinv, sA)) != hipSuccess)
    return e;
  const dim3 gc((unsigned)((nr + 255) / 256), (unsigned)((w + 15) / 16), (unsigned)nbatch);
  hipLaunchKernelGGL((spec_check_kernel<T>), gc, dim3(256), 0, st, A, ld, n, k0, w, flag, sA, sflag);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// planning and workspace
// ---------------------------------------------------------------------------
static const int LDS_RESERVE = 2048;
// the tournament panel's static LDS (pivot block, wave slots) is larger
static const int LDS_RESERVE_TP = 4096;
// rows per workgroup of the local choice (a 32-bit mask of each lane's rows)
static const int TP_MAX_ROWS = 2048;

// dynamic LDS of a panel workgroup: tile, pivot row(s), scratch, labels, pivots
static size_t panel_lds_bytes(int w, int R, size_t cbytes, int pb) {
  if (pb <= 1) return ((size_t)w * R + w) * cbytes + (size_t)(R + w) * 4;
  return ((size_t)w * R + (size_t)pb * w + (size_t)pb * R) * cbytes + (size_t)(R + w) * 4;
}
static int lds_reserve(int pb) { return pb <= 1 ? LDS_RESERVE : LDS_RESERVE_TP; }
// most rows of one panel workgroup that fit its LDS
static int64_t panel_rows_max(int w, int64_t lds_bytes, int cbytes, int pb) {
  if (pb <= 1) return (lds_bytes - LDS_RESERVE - (int64_t)w * (cbytes + 4)) / ((int64_t)(w + 1) * cbytes + 4);
  const int64_t r = (lds_bytes - LDS_RESERVE_TP - (int64_t)w * (pb * cbytes + 4)) / ((int64_t)(w + pb) * cbytes + 4);
  return r < TP_MAX_ROWS ? r : TP_MAX_ROWS;
}

// root workgroups of a tournament panel over G row workgroups
static int tp_roots(int G) { return (G + 31) / 32; }

LUPlan lu_plan(int64_t n, int elem_bytes, int num_cu, int lds_bytes, int nbatch, int nb_max, int pb) {
  LUPlan p;
  p.n = n;
  if (nbatch < 1) nbatch = 1;
  p.spec = pb == 0;
  if (pb != 1 && pb != 2 && pb != 4 && pb != 8) pb = 1;
  if (elem_bytes == 8 && pb > 4) pb = 4;  // FP64 candidates of 8 columns would need too many registers
  p.pb = pb;
  // the panels of all items run in one launch and must all be resident
  p.max_wg = num_cu / nbatch > 0 ? num_cu / nbatch : 1;
  // row workgroups of one panel: with tournament pivoting, one root workgroup
  // per 32 of them must be resident too (G + ceil(G / 32) <= max_wg)
  const int avail = pb > 1 ? std::max(1, 32 * p.max_wg / 33) : p.max_wg;
  const int cbytes = 2 * elem_bytes;
  int nb = nb_max >= 16 && nb_max <= 128 ? nb_max : 128;
  // the panel must fit: ceil(n / avail) rows x nb columns in LDS
  while (nb > 16) {
    const int64_t R = (n + avail - 1) / avail;
    if (R <= panel_rows_max(nb, lds_bytes, cbytes, pb)) break;
    nb /= 2;
  }
  p.nb = nb;
  // Workgroups of one panel.  Measured on n = 12 000: an FP32 panel over at most
  // 128 CUs is as fast per column as one over all 256 and leaves the other CUs
  // to the look-ahead update (140 vs 150 ms per factorisation + solve step); an
  // FP64 panel (twice the bytes per row) is fastest spread over every CU.  The
  // cap is raised when the panel's rows would not fit the LDS of fewer
  // workgroups.
  int cap = avail;
  if (elem_bytes == 4 && nbatch == 1) {
    const int64_t rmax = panel_rows_max(nb, lds_bytes, cbytes, pb);
    const int64_t need = rmax > 0 ? (n + rmax - 1) / rmax : avail;
    cap = (int)std::min<int64_t>(avail, std::max<int64_t>(128, need));
  }
  for (int64_t k0 = 0; k0 < n; k0 += nb) {
    LUBlock b;
    b.k0 = k0;
    b.w = (int)(n - k0 < nb ? n - k0 : nb);
    const int64_t m = n - k0;
    int64_t R = (m + cap - 1) / cap;
    if (R < 32) R = 32;
    const int64_t Rmax = panel_rows_max(b.w, lds_bytes, cbytes, pb);
    if (R > Rmax) R = Rmax;
    b.R = (int)R;
    b.G = (int)((m + R - 1) / R);
    p.blocks.push_back(b);
  }
  return p;
}

bool lu_plan_fits(const LUPlan& p) {
  for (const LUBlock& b : p.blocks)
    if (b.G + (p.pb > 1 ? tp_roots(b.G) : 0) > p.max_wg || (int64_t)b.G * b.R < p.n - b.k0) return false;
  return true;
}

// rows of the complex scratch `tmp` (x nb columns): operand copies need n; the
// split-k partial sums of the transposed solve need more than n for small n
static int64_t tmp_rows(const LUPlan& p) { return p.n > 512 ? p.n : 512; }

static size_t al256(size_t b) { return (b + 255) / 256 * 256; }

size_t lu_workspace_bytes(const LUPlan& p, int elem_bytes, int num_cu, int nbatch) {
  LUWork w;
  lu_workspace_carve(nullptr, p, elem_bytes, num_cu, w, nbatch);
  return w.bytes;
}

// Every per-item field is nbatch consecutive copies `s_*` elements apart.
void lu_workspace_carve(void* base, const LUPlan& p, int elem_bytes, int num_cu, LUWork& w, int nbatch) {
  if (nbatch < 1) nbatch = 1;
  const size_t nb = (size_t)p.nb, nblk = p.blocks.size();
  const size_t ww = nb * (2 * (size_t)elem_bytes / 4);
  const size_t cb = 2 * (size_t)elem_bytes;
  char* b = static_cast<char*>(base);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* r = b ? b + off : nullptr;
    off += al256(bytes) + 256;
    return r;
  };
  w.nbatch = nbatch;
  w.gmax = num_cu;
  w.gitem = p.max_wg > 0 ? p.max_wg : num_cu;
  w.pb = p.pb;
  w.wwmax = (int)ww;
  const size_t pbz = (size_t)(p.pb > 1 ? p.pb : 1);
  const size_t nwc = 2 * (size_t)elem_bytes / 4;  // 32-bit words per complex
  // tournament: records [2][gitem][pb][1 + pb nwc], then the roots' winners
  // [2][ceil(gitem / 32)][pb][2 + pb nwc]; partial pivoting: keys [2][gitem][KEY_STRIDE]
  const size_t cand_words = p.pb > 1 ? 2 * (size_t)w.gitem * pbz * (1 + pbz * nwc) +
                                           2 * (size_t)tp_roots(w.gitem) * pbz * (2 + pbz * nwc)
                                     : 2 * (size_t)w.gitem * KEY_STRIDE;
  w.s_cand = (int64_t)(al256(cand_words * 8) / 8);
  w.s_rows = (int64_t)(al256(2 * (size_t)w.gitem * pbz * ww * 8) / 8);
  w.cand = reinterpret_cast<unsigned long long*>(take((size_t)nbatch * w.s_cand * 8));
  w.rows = reinterpret_cast<unsigned long long*>(take((size_t)nbatch * w.s_rows * 8));
  w.err = reinterpret_cast<int32_t*>(take(64));
  w.s_pairs = (int64_t)(al256(nblk * 2 * 2 * nb * 4) / 4);
  w.s_npairs = (int64_t)(al256(2 * nblk * 4) / 4);  // moved-row counts, then the speculative panels' flags
  w.pairs = reinterpret_cast<int32_t*>(take((size_t)nbatch * w.s_pairs * 4));
  w.npairs = reinterpret_cast<int32_t*>(take((size_t)nbatch * w.s_npairs * 4));
  w.spec = w.npairs ? w.npairs + nblk : nullptr;
  w.tmp_elems = tmp_rows(p) * (int64_t)nb;
  w.s_tmp = (int64_t)(al256((size_t)w.tmp_elems * cb) / cb);
  w.tmp = take((size_t)nbatch * w.s_tmp * cb);
  w.s_dinv = (int64_t)(al256(nblk * nb * nb * cb) / cb);
  w.dinv = take((size_t)nbatch * w.s_dinv * cb);
  w.s_l21c = p.spec ? w.s_tmp : 0;
  w.l21c = p.spec ? take((size_t)nbatch * w.s_l21c * cb) : nullptr;
  w.events = nullptr;
  w.bytes = off + 256;
}

// The panel kernel of a plan (pb columns per exchange).
template <typename T>
static const void* panel_fn(int pb) {
  switch (pb) {
    case 2: return reinterpret_cast<const void*>(&panel_tp_kernel<T, 2>);
    case 4: return reinterpret_cast<const void*>(&panel_tp_kernel<T, 4>);
    case 8:
      if constexpr (sizeof(T) == 4) return reinterpret_cast<const void*>(&panel_tp_kernel<T, 8>);
      return nullptr;
    default: return reinterpret_cast<const void*>(&panel_kernel<T>);
  }
}

// One panel launch: G row workgroups (plus the roots of a tournament panel) per item.
template <typename T>
static void launch_panel(int pb, const LUBlock& b, int NB, size_t lds, hipStream_t st, cplx<T>* A, int64_t ld,
                         int64_t n, int32_t* ipiv, const LUWork& ws, uint32_t epoch, int64_t sA, int64_t sipiv,
                         int32_t* dst, int32_t* src, int32_t* npr, int mcap) {
  const dim3 grid(b.G + (pb > 1 ? tp_roots(b.G) : 0), NB);
#define GDM_PANEL_ARGS A, ld, n, b.k0, b.w, b.R, b.G, ipiv, ws, epoch, sA, sipiv, dst, src, npr, mcap
  switch (pb) {
    case 2: hipLaunchKernelGGL((panel_tp_kernel<T, 2>), grid, dim3(256), lds, st, GDM_PANEL_ARGS); break;
    case 4: hipLaunchKernelGGL((panel_tp_kernel<T, 4>), grid, dim3(256), lds, st, GDM_PANEL_ARGS); break;
    case 8:
      if constexpr (sizeof(T) == 4) {
        hipLaunchKernelGGL((panel_tp_kernel<T, 8>), grid, dim3(256), lds, st, GDM_PANEL_ARGS);
        break;
      }
      [[fallthrough]];
    default: hipLaunchKernelGGL(panel_kernel<T>, grid, dim3(256), lds, st, GDM_PANEL_ARGS); break;
  }
#undef GDM_PANEL_ARGS
}

// Panels may need more than the default 64 KB of dynamic LDS: raise each panel
// kernel's limit once (a host-side setting; done before any graph capture).
template <typename T>
hipError_t lu_prepare(const LUPlan& plan) {
  static std::map<const void*, size_t> lds_set;
  static std::mutex mu;
  std::lock_guard<std::mutex> lk(mu);
  for (const LUBlock& b : plan.blocks) {
    const size_t need = panel_lds_bytes(b.w, b.R, sizeof(cplx<T>), plan.pb);
    const void* fn = panel_fn<T>(plan.pb);
    if (!fn) return hipErrorInvalidValue;
    size_t& cur = lds_set[fn];
    if (need > 64 * 1024 && need > cur) {
      hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)need);
      if (e != hipSuccess) return e;
      cur = need;
    }
  }
  return hipSuccess;
}
template hipError_t lu_prepare<double>(const LUPlan&);
template hipError_t lu_prepare<float>(const LUPlan&);

template <typename T>
hipError_t lu_factor(void* Av, int64_t ld, const LUPlan& plan, const LUWork& ws, int32_t* ipiv, hipStream_t st,
                     Prof* prof, hipStream_t side, int64_t sA, int64_t sipiv) {
  Prof noprof;
  Prof& P = prof ? *prof : noprof;
  using CT = cplx<T>;
  CT* A = static_cast<CT*>(Av);
  const int64_t n = plan.n;
  const int nb = plan.nb;
  const int nblk = (int)plan.blocks.size();
  const int NB = ws.nbatch;
  const double fb = (double)NB;
  hipError_t e;
  if (NB < 1 || NB > 65535 || !lu_plan_fits(plan) || plan.max_wg * NB > ws.gmax || plan.max_wg > ws.gitem ||
      plan.pb > ws.pb)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(init_err_kernel, dim3(1), dim3(64), 0, st, ws.err);
  // exchange buffers start from zero (epoch 0 is never used), so epochs 1, 2, ...
  // of this factorisation are unique
  // (and the moved-row counters of every block, which the panels fill)
  {
    const size_t nc = (size_t)NB * ws.s_cand, nr = (size_t)NB * ws.s_rows, np = (size_t)NB * ws.s_npairs;
    const size_t nmax = std::max(std::max(nc, nr), np);
    hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)((nmax + 255) / 256)), dim3(256), 0, st, ws.cand, nc, ws.rows, nr,
                       ws.npairs, np);
  }
  uint32_t epoch = 1;
  if ((e = lu_prepare<T>(plan)) != hipSuccess) return e;
  // Look-ahead: the main stream runs the panels and the update of the next
  // panel's columns; the side stream runs the bulk of each trailing update (and
  // the solve-ready transform of L21), overlapping the next panel.
  const bool la = side != nullptr && side != st && ws.events != nullptr;
  // events come from a pool owned by the caller and reused across calls (the
  // caller synchronises the stream before the next factorisation)
  size_t ev_used = 0;
  auto new_event = [&](hipEvent_t& ev) -> hipError_t {
    if (!ws.events) return hipErrorInvalidValue;
    if (ev_used == ws.events->size()) {
      hipEvent_t x;
      hipError_t r = hipEventCreateWithFlags(&x, hipEventDisableTiming);
      if (r != hipSuccess) return r;
      ws.events->push_back(x);
    }
    ev = (*ws.events)[ev_used++];
    return hipSuccess;
  };
#define LUCHK(x)                   \
  do {                             \
    if ((e = (x)) != hipSuccess) { \
      return e;                    \
    }                              \
  } while (0)
  CT* tmpB = static_cast<CT*>(ws.tmp);   // side-stream operand copies (n x nb per item)
  CT* dinv = static_cast<CT*>(ws.dinv);
  hipEvent_t bulk_done = nullptr;  // side stream finished the previous block's bulk update
  // Upper parts of block b (final once panel b is done): the diagonal block
  // gets I - U11^-1, the block column above it U01 U11^-1.  With look-ahead (one
  // system) they are formed on the side stream after a block's bulk update,
  // in the second half of the factorisation (the panels then set the pace and
  // the side stream has time to spare); the rest at the end.  Measured at
  // n = 12 000: FP32+IR step 93.3 -> 90.9 ms, FP64 146.7 -> 144.3 ms with three
  // per step from half the rows (two per step from 3/4 of the rows: 91.5 and
  // 145.8; the batched factorisations, whose side stream has no time to spare,
  // keep the end).  Later, with the faster update and panels, three per step
  // put the side stream on the panels' path (a kernel trace showed the next
  // panel's substitution waiting for a bulk update held back by them); the
  // graded count below: FP32+IR step 71.7 -> 69.6 ms, FP64 105.5 -> 103.5 ms
  // (two per step from half the rows: 70.5 and 104.2).
  int u_next = 0;  // blocks [0, u_next) have their upper parts formed
  auto upper_parts = [&](hipStream_t s, int bb) -> hipError_t {
    hipError_t r;
    const int64_t kb = plan.blocks[bb].k0;
    const int wb = plan.blocks[bb].w;
    if ((r = P.begin(s, PROF_TRSM, 0.0)) != hipSuccess) return r;
    if ((r = launch_block_inv<T, 1>(A, ld, n, nb, bb, 1, dinv, s, NB, sA, ws.s_dinv, ws.gmax)) != hipSuccess) return r;
    if (kb > 0) {
      if ((r = launch_copy_block<T>(A + kb * ld, ld, tmpB, kb, kb, wb, s, NB, sA, ws.s_tmp)) != hipSuccess) return r;
      GemmMask mu;
      mu.bkind = GEMM_MASK_UPPER;
      if ((r = launch_gemm<T>(0, 0, kb, wb, wb, tmpB, kb, A + kb + kb * ld, ld, A + kb * ld, ld, s, mu, NB, ws.s_tmp,
                              sA, sA)) != hipSuccess)
        return r;
    }
    return P.end(s);
  };
  for (int bi = 0; bi < nblk; ++bi) {
    const LUBlock& b = plan.blocks[bi];
    const int64_t k0 = b.k0;
    const int w = b.w;
    const size_t lds = panel_lds_bytes(w, b.R, sizeof(CT), plan.pb);
    LUCHK(P.begin(st, PROF_PANEL, (double)w * fb));
    int32_t* dst = ws.pairs + bi * 4 * (size_t)nb;  // moved rows: destinations, then sources 2 nb later
    int32_t* src = dst + 2 * nb;
    int32_t* npr = ws.npairs + bi;
    if (plan.spec) {
      LUCHK(launch_spec_diag<T>(A, ld, nb, bi, k0, w, ipiv, ws, st, NB, sA, sipiv));
      LUCHK(P.end(st));
      LUCHK(P.begin(st, PROF_PANEL_L21, 8.0 * (double)(n - k0 - w) * w * w * fb));
      LUCHK(launch_spec_l21<T>(A, ld, n, nb, bi, k0, w, ws, st, NB, sA));
    } else {
      launch_panel<T>(plan.pb, b, NB, lds, st, A, ld, n, ipiv, ws, epoch, sA, sipiv, dst, src, npr, 2 * nb);
      epoch += (uint32_t)w;
      LUCHK(hipGetLastError());
    }
    LUCHK(P.end(st));
    const int64_t c1 = k0 + w;
    const int64_t nr = n - c1;
    CT* diag = A + k0 + k0 * ld;
    // L11^-1 -> strict lower part of the diagonal block holds I - L11^-1.  With
    // look-ahead it is formed on the side stream, once the main stream has
    // solved the next panel's U12 block directly (that solve reads L11).
    auto form_inverse = [&](hipStream_t s) -> hipError_t {
      hipError_t r;
      if ((r = P.begin(s, PROF_TRSM, 0.0)) != hipSuccess) return r;
      if ((r = launch_block_inv<T, 0>(A, ld, n, nb, bi, 1, dinv, s, NB, sA, ws.s_dinv, ws.gmax)) != hipSuccess)
        return r;
      return P.end(s);
    };
    if (!la || nr <= 0) LUCHK(form_inverse(st));
    // columns [c1, c1 + wa) on the main stream, [c1 + wa, n) on the side stream
    const int64_t wa = la ? std::min<int64_t>(nr, nb) : nr;
    // While the trailing matrix is large (one system), the bulk update sets the
    // pace: the side stream then starts its part as soon as the panel is done,
    // beside the main stream's part.  L11^-1 goes to the block's inverse slot in
    // its masked-operand form (-L11^-1 below the diagonal, = I - L11^-1 there),
    // and reaches the diagonal block of A only after the main stream's
    // substitution has read L11.
    // (while more than half the rows remain: measured against three quarters,
    // FP32 factorisation 58.4 -> 58.1 ms, FP64 100.5 -> 99.8 ms at n = 12 000)
    const bool early = la && NB == 1 && nr - wa > 0 && 2 * nr > n;
    hipEvent_t panel_done = nullptr;
    if (early) {
      LUCHK(new_event(panel_done));
      LUCHK(hipEventRecord(panel_done, st));
    }
    if (bulk_done) LUCHK(hipStreamWaitEvent(st, bulk_done, 0));  // columns of this step were in the bulk
    if (nr <= 0) break;
    GemmMask ml;
    ml.akind = GEMM_MASK_STRICT_LOWER;
    ml.ar0 = 0;
    ml.adw = w;
    // lop: I - L11^-1 below its diagonal (leading dimension lld, item stride slop)
    auto update_cols = [&](hipStream_t s, int64_t cb, int64_t ncols, CT* tmp, int64_t stmp, const CT* lop,
                           int64_t lld, int64_t slop) -> hipError_t {
      hipError_t r;
      if (ncols <= 0) return hipSuccess;
      if (!plan.spec) {  // a speculative panel moves no rows
        if ((r = P.begin(s, PROF_PERM, 0.0)) != hipSuccess) return r;
        hipLaunchKernelGGL(row_permute_kernel<T>, dim3((unsigned)ncols, NB), dim3(256), 0, s, A, ld, cb, dst, src, npr,
                           sA, ws.s_pairs, ws.s_npairs);
        if ((r = P.end(s)) != hipSuccess) return r;
      }
      // U12 = L11^-1 A12 = A12 - (I - L11^-1) A12
      if ((r = P.begin(s, PROF_TRSM, 8.0 * w * w * (double)ncols * fb)) != hipSuccess) return r;
      if ((r = launch_copy_block<T>(A + k0 + cb * ld, ld, tmp, w, w, ncols, s, NB, sA, stmp)) != hipSuccess) return r;
      if ((r = launch_gemm<T>(0, 0, w, ncols, w, lop, lld, tmp, w, A + k0 + cb * ld, ld, s, ml, NB, slop, stmp, sA)) !=
          hipSuccess)
        return r;
      if ((r = P.end(s)) != hipSuccess) return r;
      // A22[:, cols] -= L21 U12[:, cols]
      if ((r = P.begin(s, PROF_UPDATE, 8.0 * (double)nr * (double)ncols * w * fb)) != hipSuccess) return r;
      if ((r = launch_gemm_update<T>(nr, ncols, w, A + c1 + k0 * ld, ld, A + k0 + cb * ld, ld, A + c1 + cb * ld, ld,
                                     s, NB, sA, sA, sA)) != hipSuccess)
        return r;
      return P.end(s);
    };
    // This event orders the side stream's writes of L11 (its inverse form; the
    // substitution below reads L11) and of L21 (its transform; the look-ahead
    // product reads it) after the main stream's part.  Each event record or
    // wait costs 6-11 us on the GPU timeline, so outside the early blocks above
    // it is the only one per block (measured: batched spectra 83 -> 98
    // systems/s with one event instead of two, FP32+IR step 95.6 -> 95.2 ms).
    hipEvent_t main_updated = nullptr;
    if (la) {
      // next panel's columns: interchanges and U12 by substitution in one
      // launch (one launch and its gap fewer per block on the panels' path),
      // then the update
      LUCHK(P.begin(st, PROF_TRSM, 8.0 * w * w * (double)wa * fb));
      LUCHK(launch_block_trsm<T>(A, ld, n, nb, bi, A + k0 + c1 * ld, ld, wa, st, NB, sA, sA, dst, src,
                                 plan.spec ? nullptr : npr, ws.s_pairs, ws.s_npairs));
      LUCHK(P.end(st));
      LUCHK(P.begin(st, PROF_LOOKAHEAD, 8.0 * (double)nr * (double)wa * w * fb));
      LUCHK(launch_gemm_update<T>(nr, wa, w, A + c1 + k0 * ld, ld, A + k0 + c1 * ld, ld, A + c1 + c1 * ld, ld, st, NB,
                                  sA, sA, sA));
      LUCHK(P.end(st));
      LUCHK(new_event(main_updated));
      LUCHK(hipEventRecord(main_updated, st));
    } else {
      LUCHK(update_cols(st, c1, wa, tmpB, ws.s_tmp, diag, ld, sA));
    }
    hipStream_t sb = la ? side : st;
    CT* dslot = dinv + (size_t)bi * nb * nb;  // this block's inverse slot
    if (early) {
      LUCHK(hipStreamWaitEvent(sb, panel_done, 0));
      LUCHK(P.begin(sb, PROF_TRSM, 0.0));
      LUCHK((launch_block_inv<T, 0, 2>(A, ld, n, nb, bi, 1, dinv, sb, NB, sA, ws.s_dinv, ws.gmax)));
      LUCHK(P.end(sb));
      LUCHK(update_cols(sb, c1 + wa, nr - wa, tmpB, ws.s_tmp, dslot, nb, ws.s_dinv));
    } else {
      if (la) {
        LUCHK(hipStreamWaitEvent(sb, main_updated, 0));
        LUCHK(form_inverse(sb));
      }
      LUCHK(update_cols(sb, c1 + wa, nr - wa, tmpB, ws.s_tmp, diag, ld, sA));
    }
    // The next step's main stream needs only the update above; the work below
    // touches block column bi alone, which no later step of the factorisation
    // reads, so for one system it runs while the main stream goes on (measured
    // at n = 12 000: FP32+IR 92.4 -> 91.8 ms, FP64 144.9 -> 144.0 ms; batched
    // groups, whose side stream sets the pace, were 1 % slower and keep the
    // record after it).
    auto record_bulk_done = [&]() -> hipError_t {
      hipError_t r = new_event(bulk_done);
      return r != hipSuccess ? r : hipEventRecord(bulk_done, sb);
    };
    if (la && NB == 1) LUCHK(record_bulk_done());
    if (early) {
      LUCHK(hipStreamWaitEvent(sb, main_updated, 0));
      LUCHK(P.begin(sb, PROF_TRSM, 0.0));
      hipLaunchKernelGGL((diag_store_kernel<T, 3>), dim3(16, 1, (unsigned)NB), dim3(256), 0, sb, A, ld, n, nb, bi, dinv,
                         sA, ws.s_dinv);
      LUCHK(hipGetLastError());
      LUCHK(P.end(sb));
    }
    // L21 is read by both parts of this step's update: transform it after both
    // (the side stream already waited for the main stream's part above)
    // solve-ready form: L21 <- L21 L11^-1 = L21 - L21 (I - L11^-1)
    LUCHK(P.begin(sb, PROF_TRSM, 8.0 * w * w * (double)nr * fb));
    LUCHK(launch_copy_block<T>(A + c1 + k0 * ld, ld, tmpB, nr, nr, w, sb, NB, sA, ws.s_tmp));
    GemmMask mb;
    mb.bkind = GEMM_MASK_STRICT_LOWER;
    LUCHK(launch_gemm<T>(0, 0, nr, w, w, tmpB, nr, diag, ld, A + c1 + k0 * ld, ld, sb, mb, NB, ws.s_tmp, sA, sA));
    LUCHK(P.end(sb));
    if (la && NB > 1) LUCHK(record_bulk_done());
    if (la && NB == 1) {
      // as many upper parts per step as the side stream has time for beside
      // the shrinking bulk update: none while more than 55 % of the rows
      // remain, then one, two from 30 % and three from 20 %, which catches up
      // with the panels by about the last block (small systems: three per step
      // throughout)
      const int64_t r100 = 100 * nr;
      int per = r100 <= 55 * n ? 1 : 0;
      if (r100 <= 30 * n) per = 2;
      if (r100 <= 20 * n) per = 3;
      if (n <= 4096) per = 3;
      for (int q = 0; q < per && u_next <= bi; ++q) LUCHK(upper_parts(sb, u_next++));
    }
  }
  if (bulk_done) {
    // everything the side stream ran, upper parts included
    hipEvent_t side_done = nullptr;
    LUCHK(new_event(side_done));
    LUCHK(hipEventRecord(side_done, side));
    LUCHK(hipStreamWaitEvent(st, side_done, 0));
  }
  if (u_next == 0) {
    // every block at the end: the inverses in one launch, then the block columns
    LUCHK(P.begin(st, PROF_TRSM, 0.0));
    LUCHK((launch_block_inv<T, 1>(A, ld, n, nb, 0, nblk, dinv, st, NB, sA, ws.s_dinv, ws.gmax)));
    for (int bi = 1; bi < nblk; ++bi) {
      const LUBlock& b = plan.blocks[bi];
      const int64_t k0 = b.k0;
      LUCHK(launch_copy_block<T>(A + k0 * ld, ld, tmpB, k0, k0, b.w, st, NB, sA, ws.s_tmp));
      GemmMask mu;
      mu.bkind = GEMM_MASK_UPPER;
      LUCHK(launch_gemm<T>(0, 0, k0, b.w, b.w, tmpB, k0, A + k0 + k0 * ld, ld, A + k0 * ld, ld, st, mu, NB, ws.s_tmp,
                           sA, sA));
    }
    LUCHK(P.end(st));
  } else {
    while (u_next < nblk) LUCHK(upper_parts(st, u_next++));
  }
  return hipGetLastError();
#undef LUCHK
}

template <typename T>
hipError_t lu_solve(int trans, const void* Av, int64_t ld, const LUPlan& plan, const LUWork& ws, void* Bv,
                    int64_t ldb, int64_t nrhs, hipStream_t st, int64_t sA, int64_t sB) {
  using CT = cplx<T>;
  const CT* A = static_cast<const CT*>(Av);
  CT* Ball = static_cast<CT*>(Bv);
  const int64_t n = plan.n;
  const int nb = plan.nb;
  const int nblk = (int)plan.blocks.size();
  const int NB = ws.nbatch;
  CT* X = static_cast<CT*>(ws.tmp);
  const int64_t sX = ws.s_tmp;
  hipError_t e;
  if (nrhs <= 0) return hipSuccess;
  // RHS columns per pass: the plain solve keeps n per column in tmp; the
  // transposed steps need (chunks of the longest product) x nb partial sums per column.
  const int64_t chunk = ws.tmp_elems / (trans ? skinny_t_chunks(n, nb) * nb : n);
  if (chunk < 1) return hipErrorInvalidValue;
  const int64_t part_elems = (int64_t)NB * sX;  // the transposed partial sums of all items
  // factors left by a speculative plan have no interchanges (a failed check
  // repeats the factorisation with a pivoting plan), so their lists are empty
  const bool perm = !plan.spec;
  for (int64_t r0 = 0; r0 < nrhs; r0 += chunk) {
    const int64_t nr = nrhs - r0 < chunk ? nrhs - r0 : chunk;
    CT* B = Ball + r0 * ldb;
    const bool small = nr <= SKINNY_MAX_RHS;
    if (trans == 0) {
      // The forward result goes to tmp (Y, n x nr, leading dimension n), so that
      // every block step reads its operand rows in place: the step's product
      // writes those rows to the other buffer (the forward into Y, the backward
      // back into B), and no step needs a copy of them.
      CT* Y = X;
      // forward: P_b, then rows [k0, n) -= [I - L11^-1 ; L21 L11^-1] B_b, rows [k0, k0 + w) into Y
      for (int bi = 0; bi < nblk; ++bi) {
        const LUBlock& b = plan.blocks[bi];
        const int64_t k0 = b.k0;
        const int32_t* dst = ws.pairs + bi * 4 * (size_t)nb;
        const int32_t* src = dst + 2 * nb;
        if (perm) {
          hipLaunchKernelGGL(row_permute_kernel<T>, dim3((unsigned)nr, NB), dim3(256), 0, st, B, ldb, (int64_t)0, dst,
                             src, ws.npairs + bi, sB, ws.s_pairs, ws.s_npairs);
          if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        GemmMask m;
        m.akind = GEMM_MASK_STRICT_LOWER;
        m.ar0 = 0;
        m.adw = b.w;
        m.c2 = Y + k0;
        m.ldc2 = n;
        m.sc2 = sX;
        e = small ? launch_skinny_n<T>(n - k0, b.w, A + k0 + k0 * ld, ld, B + k0, ldb, B + k0, ldb, nr, st, m, NB, sA,
                                       sB, sB)
                  : launch_gemm<T>(0, 0, n - k0, nr, b.w, A + k0 + k0 * ld, ld, B + k0, ldb, B + k0, ldb, st, m, NB,
                                   sA, sB, sB);
        if (e != hipSuccess) return e;
      }
      // backward on Y: rows [0, k0 + w) -= [U01 U11^-1 ; I - U11^-1] Y_b, rows [k0, k0 + w) into B
      for (int bi = nblk - 1; bi >= 0; --bi) {
        const LUBlock& b = plan.blocks[bi];
        const int64_t k0 = b.k0;
        GemmMask m;
        m.akind = GEMM_MASK_UPPER;
        m.ar0 = k0;
        m.adw = b.w;
        m.c2 = B + k0;
        m.ldc2 = ldb;
        m.sc2 = sB;
        e = small ? launch_skinny_n<T>(k0 + b.w, b.w, A + k0 * ld, ld, Y + k0, n, Y, n, nr, st, m, NB, sA, sX, sX)
                  : launch_gemm<T>(0, 0, k0 + b.w, nr, b.w, A + k0 * ld, ld, Y + k0, n, Y, n, st, m, NB, sA, sX, sX);
        if (e != hipSuccess) return e;
      }
    } else {
      // M^T = U^T L_k^T P_k ... L_1^T P_1.  U^T forward, with V = U01 U11^-1 stored above the diagonal:
      //   z_b = U11^-T g_b - V^T z_above = g_b - V^T z_above - (I - U11^-1)^T g_b
      // (both products read the pre-step B; the split-k partials are added afterwards)
      for (int bi = 0; bi < nblk; ++bi) {
        const LUBlock& b = plan.blocks[bi];
        const int64_t k0 = b.k0;
        if ((e = launch_skinny_t<T>(b.w, nr, A + k0 * ld, ld, B, ldb, k0, A + k0 + k0 * ld, ld, B + k0, ldb, b.w,
                                    GEMM_MASK_LOWER, X, part_elems, B + k0, ldb, st, NB, sA, sB, sB)) != hipSuccess)
          return e;
      }
      // then for b = k..1: z_b = L11^-T z_b - (L21 L11^-1)^T z_below, and z = P_b^T z
      for (int bi = nblk - 1; bi >= 0; --bi) {
        const LUBlock& b = plan.blocks[bi];
        const int64_t k0 = b.k0, c1 = k0 + b.w;
        if ((e = launch_skinny_t<T>(b.w, nr, A + c1 + k0 * ld, ld, B + c1, ldb, n - c1, A + k0 + k0 * ld, ld, B + k0,
                                    ldb, b.w, GEMM_MASK_STRICT_UPPER, X, part_elems, B + k0, ldb, st, NB, sA, sB, sB)) !=
            hipSuccess)
          return e;
        const int32_t* dst = ws.pairs + bi * 4 * (size_t)nb;
        const int32_t* src = dst + 2 * nb;
        if (perm)
          hipLaunchKernelGGL(row_permute_inv_kernel<T>, dim3((unsigned)nr, NB), dim3(256), 0, st, B, ldb, (int64_t)0,
                             dst, src, ws.npairs + bi, sB, ws.s_pairs, ws.s_npairs);
      }
    }
  }
  return hipGetLastError();
}

template hipError_t lu_factor<double>(void*, int64_t, const LUPlan&, const LUWork&, int32_t*, hipStream_t, Prof*,
                                      hipStream_t, int64_t, int64_t);
template hipError_t lu_factor<float>(void*, int64_t, const LUPlan&, const LUWork&, int32_t*, hipStream_t, Prof*,
                                     hipStream_t, int64_t, int64_t);
template hipError_t lu_solve<double>(int, const void*, int64_t, const LUPlan&, const LUWork&, void*, int64_t, int64_t,
                                     hipStream_t, int64_t, int64_t);
template hipError_t lu_solve<float>(int, const void*, int64_t, const LUPlan&, const LUWork&, void*, int64_t, int64_t,
                                    hipStream_t, int64_t, int64_t);

}  // namespace gdm
