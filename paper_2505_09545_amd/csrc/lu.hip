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
//   2. the net row permutation of the block's w interchanges is computed once
//      (<= 2w rows move) and applied to the trailing columns and, in the solve,
//      to the right-hand sides.  Interchanges are never applied to the columns
//      left of the block: the factors are kept in the factored form
//          M = P1^T L1 P2^T L2 ... Pk^T Lk U
//      and the solve applies P_b before using L_b, which is equivalent.
//   3. U12 = L11^-1 A12 (triangular solve), 4. A22 -= L21 U12 (complex GEMM on
//      MFMA, gemm.hip).
//
// Layout: column-major interleaved complex, leading dimension ld.  ipiv holds
// 0-based global row indices (LAPACK semantics otherwise).
#include <algorithm>
#include <climits>

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
template <typename CT> __device__ inline CT cinv_t(CT a) {
  // 1/a with scaling against overflow of |a|^2
  const auto s = fabs(a.x) > fabs(a.y) ? fabs(a.x) : fabs(a.y);
  CT r;
  const auto ar = a.x / s, ai = a.y / s;
  const auto d = s * (ar * ar + ai * ai);
  r.x = ar / d;
  r.y = -ai / d;
  return r;
}

__device__ inline unsigned long long shfl_xor_u64(unsigned long long v, int m) {
  const unsigned lo = __shfl_xor((unsigned)(v & 0xffffffffu), m);
  const unsigned hi = __shfl_xor((unsigned)(v >> 32), m);
  return ((unsigned long long)hi << 32) | lo;
}

__global__ void zero_u64_kernel(unsigned long long* a, size_t na, unsigned long long* b, size_t nb,
                                unsigned long long* c, size_t nc) {
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

// complex values travel as their 32-bit words (2 for complex float, 4 for
// complex double), little-endian order of the (re, im) storage.
template <typename CT> __device__ inline uint32_t cword(const CT& v, int k) {
  return reinterpret_cast<const uint32_t*>(&v)[k];
}

template <typename T>
__global__ void __launch_bounds__(256) panel_kernel(cplx<T>* __restrict__ A, int64_t ld, int64_t n, int64_t k0, int w,
                                                     int R, int G, int32_t* __restrict__ ipiv, LUWork ws,
                                                     uint32_t epoch0) {
  using CT = cplx<T>;
  constexpr int NW = sizeof(CT) / 4;  // payload words per complex
  extern __shared__ unsigned char smem_raw[];
  CT* tile = reinterpret_cast<CT*>(smem_raw);  // [w][R], column c at tile + c*R
  CT* prow = tile + (size_t)w * R;             // [w] pivot row
  __shared__ u64 red[4];
  __shared__ int bad;
  const int g = blockIdx.x, tid = threadIdx.x;
  const int64_t rbase = k0 + (int64_t)g * R;
  const int myR = (int)(n - rbase < (int64_t)R ? (n - rbase > 0 ? n - rbase : 0) : R);
  const int WW = w * NW;  // payload words per row
  if (tid == 0) bad = 0;
  for (int c = 0; c < w; ++c)
    for (int lr = tid; lr < myR; lr += 256) tile[c * R + lr] = A[(rbase + lr) + (k0 + c) * ld];
  // 2D mapping for the rank-1 update: RP rows x CG column groups
  int RP = 1;
  while (RP < myR && RP < 256) RP <<= 1;
  const int CG = 256 / RP;
  const int ulr0 = tid & (RP - 1), ucg = tid / RP;
  __syncthreads();

  for (int j = 0; j < w; ++j) {
    const int64_t gj = k0 + j;
    const uint32_t E = epoch0 + (uint32_t)j;
    const int par = j & 1;
    u64* cand = ws.cand + (size_t)par * ws.gmax * 2;
    u64* rows = ws.rows + (size_t)par * ws.gmax * ws.wwmax;
    u64* drow = ws.drow + (size_t)par * ws.wwmax;
    // local pivot candidate: key = (|re|+|im| as float bits) << 32 | ~row
    u64 best = 0;
    for (int lr = tid; lr < myR; lr += 256) {
      const int64_t gr = rbase + lr;
      if (gr >= gj) {
        const CT v = tile[j * R + lr];
        const float a = (float)(fabs(v.x) + fabs(v.y));
        const u64 kk = ((u64)__float_as_uint(a) << 32) | (0xffffffffu - (uint32_t)gr);
        best = kk > best ? kk : best;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const u64 o = shfl_xor_u64(best, off);
      best = o > best ? o : best;
    }
    if ((tid & 63) == 0) red[tid >> 6] = best;
    __syncthreads();
    u64 mybest = red[0];
    for (int i = 1; i < 4; ++i) mybest = red[i] > mybest ? red[i] : mybest;
    __syncthreads();
    const int gd = j / R;  // owner of global row gj
    // publish: candidate key, candidate row, and (owner only) row gj
    if (tid == 0) {
      const uint32_t val = mybest ? (uint32_t)(mybest >> 32) : 0u;
      const uint32_t row = mybest ? (0xffffffffu - (uint32_t)(mybest & 0xffffffffu)) : 0xffffffffu;
      ll_put(&cand[2 * g + 0], E, val);
      ll_put(&cand[2 * g + 1], E, row);
    }
    if (mybest) {
      const int lrow = (int)((int64_t)(0xffffffffu - (uint32_t)(mybest & 0xffffffffu)) - rbase);
      for (int t = tid; t < WW; t += 256) ll_put(&rows[(size_t)g * ws.wwmax + t], E, cword(tile[(t / NW) * R + lrow], t % NW));
    }
    if (g == gd) {
      const int ldr = j - gd * R;
      for (int t = tid; t < WW; t += 256) ll_put(&drow[t], E, cword(tile[(t / NW) * R + ldr], t % NW));
    }
    // gather every workgroup's key; winner = largest |re|+|im|, lowest row on ties
    u64 k = 0;
    if (tid < G) {
      const uint32_t val = ll_get(&cand[2 * tid + 0], E, &bad);
      const uint32_t row = ll_get(&cand[2 * tid + 1], E, &bad);
      k = ((u64)val << 32) | (0xffffffffu - row);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const u64 o = shfl_xor_u64(k, off);
      k = o > k ? o : k;
    }
    if ((tid & 63) == 0) red[tid >> 6] = k;
    __syncthreads();
    u64 win = red[0];
    for (int i = 1; i < 4; ++i) win = red[i] > win ? red[i] : win;
    const int64_t p = (int64_t)(0xffffffffu - (uint32_t)(win & 0xffffffffu));
    const int gp = (int)((p - k0) / R);
    const int lp = (int)((p - k0) - (int64_t)gp * R);
    // pivot row
    for (int t = tid; t < WW; t += 256)
      reinterpret_cast<uint32_t*>(prow)[t] = ll_get(&rows[(size_t)gp * ws.wwmax + t], E, &bad);
    __syncthreads();
    if (bad) {
      if (tid == 0) __hip_atomic_store(&ws.err[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    if (p != gj && (g == gd || g == gp)) {
      const int ldr = j - gd * R;
      for (int c = tid; c < w; c += 256) {
        CT dv;
        if (g == gd) {
          dv = tile[c * R + ldr];
        } else {
          for (int q = 0; q < NW; ++q) reinterpret_cast<uint32_t*>(&dv)[q] = ll_get(&drow[c * NW + q], E, &bad);
        }
        if (g == gp) tile[c * R + lp] = dv;
        if (g == gd) tile[c * R + ldr] = prow[c];
      }
    }
    if (g == 0 && tid == 0) ipiv[gj] = (int32_t)p;
    __syncthreads();
    if (bad) {
      if (tid == 0) __hip_atomic_store(&ws.err[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    const CT piv = prow[j];
    const bool zero = piv.x == 0 && piv.y == 0;
    if (zero && g == 0 && tid == 0) atomicMin(&ws.err[1], (int)gj);
    CT inv;
    if (zero) { inv.x = 0; inv.y = 0; } else inv = cinv_t(piv);
    for (int lr = tid; lr < myR; lr += 256)
      if (rbase + lr > gj) tile[j * R + lr] = cmul_t(tile[j * R + lr], inv);
    __syncthreads();
    for (int lr = ulr0; lr < myR; lr += RP) {
      if (rbase + lr <= gj) continue;
      const CT l = tile[j * R + lr];
      for (int c = j + 1 + ucg; c < w; c += CG) {
        const CT u = prow[c];
        CT& t = tile[c * R + lr];
        t.x -= l.x * u.x - l.y * u.y;
        t.y -= l.x * u.y + l.y * u.x;
      }
    }
    __syncthreads();
  }
  for (int c = 0; c < w; ++c)
    for (int lr = tid; lr < myR; lr += 256) A[(rbase + lr) + (k0 + c) * ld] = tile[c * R + lr];
}

// ---------------------------------------------------------------------------
// 2. net permutation of a block's interchanges (one wave)
// ---------------------------------------------------------------------------
// After the w interchanges (k0+i <-> ipiv[k0+i]), row dst[t] holds the former
// row src[t]; rows outside the list are unchanged.
__global__ void __launch_bounds__(64) block_perm_kernel(const int32_t* __restrict__ ipiv, int64_t k0, int w,
                                                         int32_t* __restrict__ dst, int32_t* __restrict__ src,
                                                         int32_t* __restrict__ npairs) {
  __shared__ int32_t key[512];
  __shared__ int32_t val[512];
  __shared__ int cnt;
  const int lane = threadIdx.x;
  for (int i = lane; i < w; i += 64) {
    key[i] = (int32_t)(k0 + i);
    val[i] = (int32_t)(k0 + i);
  }
  if (lane == 0) cnt = w;
  __syncthreads();
  for (int i = 0; i < w; ++i) {
    const int32_t b = ipiv[k0 + i];
    if (b == (int32_t)(k0 + i)) continue;
    int bi;
    if (b < (int32_t)(k0 + w)) {
      bi = (int)(b - k0);
    } else {
      const int c = cnt;
      int found = -1;
      for (int t = w + lane; t < c; t += 64)
        if (key[t] == b) found = t;
      unsigned long long mask = __ballot(found >= 0);
      if (mask) {
        const int src_lane = __ffsll((long long)mask) - 1;
        bi = __shfl(found, src_lane);
      } else {
        bi = c;
        if (lane == 0) {
          key[c] = b;
          val[c] = b;
          cnt = c + 1;
        }
      }
    }
    __syncthreads();
    if (lane == 0) {
      const int32_t t = val[i];
      val[i] = val[bi];
      val[bi] = t;
    }
    __syncthreads();
  }
  const int c = cnt;
  for (int t = lane; t < c; t += 64) {
    dst[t] = key[t];
    src[t] = val[t];
  }
  if (lane == 0) *npairs = c;
}

// X[dst[t], col] = Xold[src[t], col] for the columns [c0, c0 + ncols).
template <typename T>
__global__ void __launch_bounds__(256) row_permute_kernel(cplx<T>* __restrict__ X, int64_t ld, int64_t c0,
                                                          const int32_t* __restrict__ dst, const int32_t* __restrict__ src,
                                                          const int32_t* __restrict__ npairs) {
  using CT = cplx<T>;
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
                                                              const int32_t* __restrict__ npairs) {
  using CT = cplx<T>;
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
// Each workgroup owns TRSM_CB columns of B (in LDS) and sweeps the w steps of
// the substitution; the needed columns of op(Tri) are staged in LDS, PW
// columns at a time, so a step costs one LDS read per element and one barrier.
constexpr int TRSM_CB = 16;
constexpr int TRSM_LS_BYTES = 48 * 1024;

template <typename T, int KIND>
__global__ void __launch_bounds__(256) trsm_kernel(const cplx<T>* __restrict__ Tri, int64_t ldt, int w,
                                                   cplx<T>* __restrict__ B, int64_t ldb, int64_t ncols, int PW) {
  using CT = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  CT* Bs = reinterpret_cast<CT*>(smem_raw);  // [w][CB] row-major
  CT* Ls = Bs + (size_t)w * TRSM_CB;         // [PW][w]: Ls[c*w + i] = op(Tri)[i][jbase + c]
  const int tid = threadIdx.x;
  const int64_t c0 = (int64_t)blockIdx.x * TRSM_CB;
  const int nc = (int)(ncols - c0 < TRSM_CB ? ncols - c0 : TRSM_CB);
  for (int idx = tid; idx < w * TRSM_CB; idx += 256) {
    const int i = idx % w, c = idx / w;
    CT v;
    v.x = 0;
    v.y = 0;
    if (c < nc) v = B[i + (c0 + c) * ldb];
    Bs[i * TRSM_CB + c] = v;
  }
  constexpr bool forward = (KIND == 0 || KIND == 2);
  constexpr bool unit = (KIND == 0 || KIND == 3);
  constexpr bool transposed = (KIND >= 2);
  const int c = tid % TRSM_CB, i0 = tid / TRSM_CB;
  constexpr int ISTEP = 256 / TRSM_CB;
  for (int ph = 0; ph < w; ph += PW) {
    const int pw = w - ph < PW ? w - ph : PW;
    // columns of op(Tri) handled in this phase: [jb, jb + pw); rows needed: [lo, hi)
    const int jb = forward ? ph : w - ph - pw;
    const int lo = forward ? jb : 0;
    const int hi = forward ? w : jb + pw;
    const int len = hi - lo;
    __syncthreads();
    for (int idx = tid; idx < pw * len; idx += 256) {
      int i, cc;
      if (!transposed) { i = lo + idx % len; cc = idx / len; }
      else { cc = idx % pw; i = lo + idx / pw; }
      const int j = jb + cc;
      Ls[cc * w + i] = transposed ? Tri[j + (int64_t)i * ldt] : Tri[i + (int64_t)j * ldt];
    }
    __syncthreads();
    for (int s = 0; s < pw; ++s) {
      const int j = forward ? jb + s : jb + pw - 1 - s;
      const CT* lcol = Ls + (j - jb) * w;
      if (!unit) {
        if (tid < TRSM_CB) Bs[j * TRSM_CB + tid] = cmul_t(Bs[j * TRSM_CB + tid], cinv_t(lcol[j]));
        __syncthreads();
      }
      const CT xj = Bs[j * TRSM_CB + c];
      if (forward) {
        for (int i = j + 1 + i0; i < w; i += ISTEP) {
          const CT t = lcol[i];
          CT& b = Bs[i * TRSM_CB + c];
          b.x -= t.x * xj.x - t.y * xj.y;
          b.y -= t.x * xj.y + t.y * xj.x;
        }
      } else {
        for (int i = i0; i < j; i += ISTEP) {
          const CT t = lcol[i];
          CT& b = Bs[i * TRSM_CB + c];
          b.x -= t.x * xj.x - t.y * xj.y;
          b.y -= t.x * xj.y + t.y * xj.x;
        }
      }
      __syncthreads();
    }
  }
  for (int idx = tid; idx < w * TRSM_CB; idx += 256) {
    const int i = idx % w, cc = idx / w;
    if (cc < nc) B[i + (c0 + cc) * ldb] = Bs[i * TRSM_CB + cc];
  }
}

template <typename T, int KIND>
static hipError_t launch_trsm(const cplx<T>* Tri, int64_t ldt, int w, cplx<T>* B, int64_t ldb, int64_t ncols,
                              hipStream_t st) {
  if (ncols <= 0 || w <= 0) return hipSuccess;
  int PW = TRSM_LS_BYTES / (w * (int)sizeof(cplx<T>));
  if (PW < 1) PW = 1;
  if (PW > w) PW = w;
  const size_t lds = ((size_t)w * TRSM_CB + (size_t)PW * w) * sizeof(cplx<T>);
  static size_t set = 0;
  if (lds > 64 * 1024 && lds > set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&trsm_kernel<T, KIND>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    set = lds;
  }
  const int64_t nblk = (ncols + TRSM_CB - 1) / TRSM_CB;
  hipLaunchKernelGGL((trsm_kernel<T, KIND>), dim3((unsigned)nblk), dim3(256), lds, st, Tri, ldt, w, B, ldb, ncols, PW);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// planning and workspace
// ---------------------------------------------------------------------------
static const int LDS_RESERVE = 2048;

LUPlan lu_plan(int64_t n, int elem_bytes, int num_cu, int lds_bytes) {
  LUPlan p;
  p.n = n;
  p.max_wg = num_cu;
  const int cbytes = 2 * elem_bytes;
  int nb = 128;
  // the panel must fit: ceil(n / num_cu) rows x nb columns in LDS
  while (nb > 16) {
    const int64_t R = (n + num_cu - 1) / num_cu;
    if ((int64_t)(R + 1) * nb * cbytes + LDS_RESERVE <= lds_bytes) break;
    nb /= 2;
  }
  p.nb = nb;
  for (int64_t k0 = 0; k0 < n; k0 += nb) {
    LUBlock b;
    b.k0 = k0;
    b.w = (int)(n - k0 < nb ? n - k0 : nb);
    const int64_t m = n - k0;
    int64_t R = (m + num_cu - 1) / num_cu;
    if (R < 32) R = 32;
    const int64_t Rmax = (lds_bytes - LDS_RESERVE) / ((int64_t)b.w * cbytes) - 1;
    if (R > Rmax) R = Rmax;
    b.R = (int)R;
    b.G = (int)((m + R - 1) / R);
    p.blocks.push_back(b);
  }
  return p;
}

size_t lu_workspace_bytes(const LUPlan& p, int elem_bytes, int num_cu) {
  const size_t nb = (size_t)p.nb, nblk = p.blocks.size();
  const size_t ww = nb * (2 * (size_t)elem_bytes / 4);
  size_t s = 0;
  s += 2 * (size_t)num_cu * 2 * 8 + 256;
  s += 2 * (size_t)num_cu * ww * 8 + 256;
  s += 2 * ww * 8 + 256;
  s += 64 + 256;
  s += nblk * 2 * 2 * nb * 4 + 256;
  s += nblk * 4 + 256;
  return s + 8 * 256;
}

void lu_workspace_carve(void* base, const LUPlan& p, int elem_bytes, int num_cu, LUWork& w) {
  const size_t nb = (size_t)p.nb, nblk = p.blocks.size();
  const size_t ww = nb * (2 * (size_t)elem_bytes / 4);
  char* b = static_cast<char*>(base);
  auto take = [&](size_t bytes) {
    char* r = b;
    b += (bytes + 255) / 256 * 256 + 256;
    return r;
  };
  w.gmax = num_cu;
  w.wwmax = (int)ww;
  w.cand = reinterpret_cast<unsigned long long*>(take(2 * (size_t)num_cu * 2 * 8));
  w.rows = reinterpret_cast<unsigned long long*>(take(2 * (size_t)num_cu * ww * 8));
  w.drow = reinterpret_cast<unsigned long long*>(take(2 * ww * 8));
  w.err = reinterpret_cast<int32_t*>(take(64));
  w.pairs = reinterpret_cast<int32_t*>(take(nblk * 2 * 2 * nb * 4));
  w.npairs = reinterpret_cast<int32_t*>(take(nblk * 4));
}

// ---------------------------------------------------------------------------
// drivers
// ---------------------------------------------------------------------------
template <typename T>
hipError_t lu_factor(void* Av, int64_t ld, const LUPlan& plan, const LUWork& ws, int32_t* ipiv, hipStream_t st,
                     Prof* prof) {
  Prof noprof;
  Prof& P = prof ? *prof : noprof;
  using CT = cplx<T>;
  CT* A = static_cast<CT*>(Av);
  const int64_t n = plan.n;
  const int nb = plan.nb;
  hipError_t e;
  hipLaunchKernelGGL(init_err_kernel, dim3(1), dim3(64), 0, st, ws.err);
  // exchange buffers start from zero (epoch 0 is never used), so epochs 1, 2, ...
  // of this factorisation are unique
  {
    const size_t nc = (size_t)ws.gmax * 4, nr = (size_t)2 * ws.gmax * ws.wwmax, nd = (size_t)2 * ws.wwmax;
    hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, st, ws.cand, nc, ws.rows, nr,
                       ws.drow, nd);
  }
  uint32_t epoch = 1;
  // panels may need more than the default 64 KB of dynamic LDS
  size_t lds_need = 0;
  for (const LUBlock& b : plan.blocks) lds_need = std::max(lds_need, ((size_t)b.w * b.R + b.w) * sizeof(CT));
  static size_t lds_set[2] = {0, 0};
  size_t& cur = lds_set[sizeof(T) == 8 ? 0 : 1];
  if (lds_need > 64 * 1024 && lds_need > cur) {
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&panel_kernel<T>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_need)) != hipSuccess)
      return e;
    cur = lds_need;
  }
  for (size_t bi = 0; bi < plan.blocks.size(); ++bi) {
    const LUBlock& b = plan.blocks[bi];
    const int64_t k0 = b.k0;
    const int w = b.w;
    // the panel's workgroups must all be resident at once (one per CU at most)
    if (b.G > plan.max_wg || b.G > ws.gmax || b.w > nb || (int64_t)b.G * b.R < n - k0) return hipErrorInvalidValue;
    const size_t lds = ((size_t)w * b.R + w) * sizeof(CT);
    if ((e = P.begin(st, PROF_PANEL, (double)w)) != hipSuccess) return e;
    hipLaunchKernelGGL(panel_kernel<T>, dim3(b.G), dim3(256), lds, st, A, ld, n, k0, w, b.R, b.G, ipiv, ws, epoch);
    epoch += (uint32_t)w;
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = P.end(st)) != hipSuccess) return e;
    int32_t* dst = ws.pairs + bi * 4 * (size_t)nb;
    int32_t* src = dst + 2 * nb;
    hipLaunchKernelGGL(block_perm_kernel, dim3(1), dim3(64), 0, st, ipiv, k0, w, dst, src, ws.npairs + bi);
    const int64_t c1 = k0 + w;
    const int64_t nr = n - c1;
    if (nr > 0) {
      if ((e = P.begin(st, PROF_PERM, 0.0)) != hipSuccess) return e;
      hipLaunchKernelGGL(row_permute_kernel<T>, dim3((unsigned)nr), dim3(256), 0, st, A, ld, c1, dst, src,
                         ws.npairs + bi);
      if ((e = P.end(st)) != hipSuccess) return e;
      if ((e = P.begin(st, PROF_TRSM, 4.0 * w * w * (double)nr)) != hipSuccess) return e;
      if ((e = launch_trsm<T, 0>(A + k0 + k0 * ld, ld, w, A + k0 + c1 * ld, ld, nr, st)) != hipSuccess) return e;
      if ((e = P.end(st)) != hipSuccess) return e;
      // A22 -= L21 U12: 8 nr^2 w real flops
      if ((e = P.begin(st, PROF_UPDATE, 8.0 * (double)nr * (double)nr * w)) != hipSuccess) return e;
      if ((e = launch_gemm_update<T>(nr, nr, w, A + c1 + k0 * ld, ld, A + k0 + c1 * ld, ld, A + c1 + c1 * ld, ld,
                                     st)) != hipSuccess)
        return e;
      if ((e = P.end(st)) != hipSuccess) return e;
    }
  }
  return hipGetLastError();
}

template <typename T>
hipError_t lu_solve(int trans, const void* Av, int64_t ld, const LUPlan& plan, const LUWork& ws, void* Bv,
                    int64_t ldb, int64_t nrhs, hipStream_t st) {
  using CT = cplx<T>;
  const CT* A = static_cast<const CT*>(Av);
  CT* B = static_cast<CT*>(Bv);
  const int64_t n = plan.n;
  const int nb = plan.nb;
  const int nblk = (int)plan.blocks.size();
  hipError_t e;
  if (nrhs <= 0) return hipSuccess;
  if (trans == 0) {
    // forward: for each block apply P_b, then L11^-1, then B_below -= L21 B_b
    for (int bi = 0; bi < nblk; ++bi) {
      const LUBlock& b = plan.blocks[bi];
      const int64_t k0 = b.k0, c1 = k0 + b.w;
      const int32_t* dst = ws.pairs + bi * 4 * (size_t)nb;
      const int32_t* src = dst + 2 * nb;
      hipLaunchKernelGGL(row_permute_kernel<T>, dim3((unsigned)nrhs), dim3(256), 0, st, B, ldb, (int64_t)0, dst, src,
                         ws.npairs + bi);
      if ((e = launch_trsm<T, 0>(A + k0 + k0 * ld, ld, b.w, B + k0, ldb, nrhs, st)) != hipSuccess) return e;
      if (n - c1 > 0)
        if ((e = launch_gemm<T>(0, 0, n - c1, nrhs, b.w, A + c1 + k0 * ld, ld, B + k0, ldb, B + c1, ldb, st)) !=
            hipSuccess)
          return e;
    }
    // backward: U
    for (int bi = nblk - 1; bi >= 0; --bi) {
      const LUBlock& b = plan.blocks[bi];
      const int64_t k0 = b.k0;
      if ((e = launch_trsm<T, 1>(A + k0 + k0 * ld, ld, b.w, B + k0, ldb, nrhs, st)) != hipSuccess) return e;
      if (k0 > 0)
        if ((e = launch_gemm<T>(0, 0, k0, nrhs, b.w, A + k0 * ld, ld, B + k0, ldb, B, ldb, st)) != hipSuccess) return e;
    }
  } else {
    // M^T = U^T L_k^T P_k ... L_1^T P_1: solve U^T z = g, then for b = k..1: z = L_b^-T z, z = P_b^T z
    for (int bi = 0; bi < nblk; ++bi) {
      const LUBlock& b = plan.blocks[bi];
      const int64_t k0 = b.k0, c1 = k0 + b.w;
      // z_b = U11^-T (g_b - U01^T z_above)
      if (k0 > 0)
        if ((e = launch_gemm<T>(0, 1, b.w, nrhs, k0, A + k0 * ld, ld, B, ldb, B + k0, ldb, st)) != hipSuccess) return e;
      if ((e = launch_trsm<T, 2>(A + k0 + k0 * ld, ld, b.w, B + k0, ldb, nrhs, st)) != hipSuccess) return e;
      (void)c1;
    }
    for (int bi = nblk - 1; bi >= 0; --bi) {
      const LUBlock& b = plan.blocks[bi];
      const int64_t k0 = b.k0, c1 = k0 + b.w;
      if (n - c1 > 0)
        if ((e = launch_gemm<T>(0, 1, b.w, nrhs, n - c1, A + c1 + k0 * ld, ld, B + c1, ldb, B + k0, ldb, st)) !=
            hipSuccess)
          return e;
      if ((e = launch_trsm<T, 3>(A + k0 + k0 * ld, ld, b.w, B + k0, ldb, nrhs, st)) != hipSuccess) return e;
      const int32_t* dst = ws.pairs + bi * 4 * (size_t)nb;
      const int32_t* src = dst + 2 * nb;
      hipLaunchKernelGGL(row_permute_inv_kernel<T>, dim3((unsigned)nrhs), dim3(256), 0, st, B, ldb, (int64_t)0, dst,
                         src, ws.npairs + bi);
    }
  }
  return hipGetLastError();
}

template hipError_t lu_factor<double>(void*, int64_t, const LUPlan&, const LUWork&, int32_t*, hipStream_t, Prof*);
template hipError_t lu_factor<float>(void*, int64_t, const LUPlan&, const LUWork&, int32_t*, hipStream_t, Prof*);
template hipError_t lu_solve<double>(int, const void*, int64_t, const LUPlan&, const LUWork&, void*, int64_t, int64_t,
                                     hipStream_t);
template hipError_t lu_solve<float>(int, const void*, int64_t, const LUPlan&, const LUWork&, void*, int64_t, int64_t,
                                    hipStream_t);

}  // namespace gdm
