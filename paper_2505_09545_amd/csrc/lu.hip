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

// ---- coherent (agent-scope, cache-bypassing) element access ----------------
__device__ inline void st_coh(double2* p, double2 v) {
  auto* q = reinterpret_cast<unsigned long long*>(p);
  __hip_atomic_store(q, (unsigned long long)__double_as_longlong(v.x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(q + 1, (unsigned long long)__double_as_longlong(v.y), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double2 ld_coh(const double2* p) {
  auto* q = reinterpret_cast<const unsigned long long*>(p);
  const unsigned long long a = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const unsigned long long b = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return make_double2(__longlong_as_double((long long)a), __longlong_as_double((long long)b));
}
__device__ inline void st_coh(float2* p, float2 v) {
  auto* q = reinterpret_cast<unsigned long long*>(p);
  const unsigned long long bits = (unsigned long long)__float_as_uint(v.x) | ((unsigned long long)__float_as_uint(v.y) << 32);
  __hip_atomic_store(q, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline float2 ld_coh(const float2* p) {
  auto* q = reinterpret_cast<const unsigned long long*>(p);
  const unsigned long long bits = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return make_float2(__uint_as_float((unsigned)(bits & 0xffffffffu)), __uint_as_float((unsigned)(bits >> 32)));
}

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

__global__ void zero_u32_kernel(uint32_t* a, int n, unsigned long long* b, int nb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
  if (i < nb) b[i] = 0;
}

__global__ void init_err_kernel(int32_t* err) {
  if (threadIdx.x == 0) {
    err[0] = 0;
    err[1] = INT32_MAX;
  }
}

// ---------------------------------------------------------------------------
// 1. panel factorisation (cooperative, one device-wide barrier per column)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) panel_kernel(cplx<T>* __restrict__ A, int64_t ld, int64_t n, int64_t k0, int w,
                                                     int R, int G, int32_t* __restrict__ ipiv, LUWork ws) {
  using CT = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  CT* tile = reinterpret_cast<CT*>(smem_raw);  // [w][R], column c at tile + c*R
  CT* prow = tile + (size_t)w * R;             // [w] pivot row
  __shared__ unsigned long long red[4];
  __shared__ int abort_flag;
  const int g = blockIdx.x, tid = threadIdx.x;
  const int64_t rbase = k0 + (int64_t)g * R;
  const int myR = (int)(n - rbase < (int64_t)R ? (n - rbase > 0 ? n - rbase : 0) : R);
  CT* slot = static_cast<CT*>(ws.slot);
  CT* dslot = static_cast<CT*>(ws.dslot);
  if (tid == 0) abort_flag = 0;
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
    // local pivot candidate: key = (|re|+|im| as float bits) << 32 | ~row
    unsigned long long best = 0;
    for (int lr = tid; lr < myR; lr += 256) {
      const int64_t gr = rbase + lr;
      if (gr >= gj) {
        const CT v = tile[j * R + lr];
        const float a = (float)(fabs(v.x) + fabs(v.y));
        const unsigned long long kk = ((unsigned long long)__float_as_uint(a) << 32) | (0xffffffffu - (uint32_t)gr);
        best = kk > best ? kk : best;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const unsigned long long o = shfl_xor_u64(best, off);
      best = o > best ? o : best;
    }
    if ((tid & 63) == 0) red[tid >> 6] = best;
    __syncthreads();
    unsigned long long mybest = red[0];
    for (int i = 1; i < 4; ++i) mybest = red[i] > mybest ? red[i] : mybest;
    const int par = j & 1;
    const int gd = j / R;  // owner of global row gj
    if (tid < 64) {
      // publish this workgroup's candidate row and, for the owner, row gj
      if (mybest != 0) {
        const int lrow = (int)((int64_t)(0xffffffffu - (uint32_t)(mybest & 0xffffffffu)) - rbase);
        for (int c = tid; c < w; c += 64) st_coh(&slot[((size_t)par * G + g) * w + c], tile[c * R + lrow]);
      }
      if (g == gd) {
        const int ldr = j - gd * R;
        for (int c = tid; c < w; c += 64) st_coh(&dslot[(size_t)par * w + c], tile[c * R + ldr]);
      }
      __threadfence();
      if (tid == 0) {
        if (mybest != 0) __hip_atomic_fetch_max(&ws.key[j], mybest, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        __hip_atomic_fetch_add(&ws.cnt[j], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t it = 0;
        while (__hip_atomic_load(&ws.cnt[j], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < (uint32_t)G) {
          if (++it > SPIN_LIMIT) {
            abort_flag = 1;
            __hip_atomic_store(&ws.err[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      __threadfence();
    }
    __syncthreads();
    if (abort_flag) return;
    const unsigned long long win = __hip_atomic_load(&ws.key[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int64_t p = (int64_t)(0xffffffffu - (uint32_t)(win & 0xffffffffu));
    const int gp = (int)((p - k0) / R);
    const int lp = (int)((p - k0) - (int64_t)gp * R);
    for (int c = tid; c < w; c += 256) prow[c] = ld_coh(&slot[((size_t)par * G + gp) * w + c]);
    if (p != gj && (g == gd || g == gp)) {
      const int ldr = j - gd * R;
      for (int c = tid; c < w; c += 256) {
        CT dv;
        if (g == gd) dv = tile[c * R + ldr];
        else dv = ld_coh(&dslot[(size_t)par * w + c]);
        if (g == gp) tile[c * R + lp] = dv;
        if (g == gd) tile[c * R + ldr] = ld_coh(&slot[((size_t)par * G + gp) * w + c]);
      }
    }
    if (g == 0 && tid == 0) ipiv[gj] = (int32_t)p;
    __syncthreads();
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
constexpr int TRSM_CB = 16;
template <typename T, int KIND>
__global__ void __launch_bounds__(256) trsm_kernel(const cplx<T>* __restrict__ Tri, int64_t ldt, int w,
                                                   cplx<T>* __restrict__ B, int64_t ldb, int64_t ncols) {
  using CT = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  CT* Bs = reinterpret_cast<CT*>(smem_raw);  // [w][CB] row-major
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
  __syncthreads();
  constexpr bool forward = (KIND == 0 || KIND == 2);
  constexpr bool unit = (KIND == 0 || KIND == 3);
  constexpr bool transposed = (KIND >= 2);
  const int c = tid % TRSM_CB, i0 = tid / TRSM_CB;
  constexpr int ISTEP = 256 / TRSM_CB;
  for (int s = 0; s < w; ++s) {
    const int j = forward ? s : w - 1 - s;
    if (!unit) {
      if (tid < TRSM_CB) {
        const CT d = Tri[j + (int64_t)j * ldt];
        Bs[j * TRSM_CB + tid] = cmul_t(Bs[j * TRSM_CB + tid], cinv_t(d));
      }
      __syncthreads();
    }
    const CT xj = Bs[j * TRSM_CB + c];
    if (forward) {
      for (int i = j + 1 + i0; i < w; i += ISTEP) {
        const CT t = transposed ? Tri[j + (int64_t)i * ldt] : Tri[i + (int64_t)j * ldt];
        CT& b = Bs[i * TRSM_CB + c];
        b.x -= t.x * xj.x - t.y * xj.y;
        b.y -= t.x * xj.y + t.y * xj.x;
      }
    } else {
      for (int i = i0; i < j; i += ISTEP) {
        const CT t = transposed ? Tri[j + (int64_t)i * ldt] : Tri[i + (int64_t)j * ldt];
        CT& b = Bs[i * TRSM_CB + c];
        b.x -= t.x * xj.x - t.y * xj.y;
        b.y -= t.x * xj.y + t.y * xj.x;
      }
    }
    __syncthreads();
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
  const size_t lds = (size_t)w * TRSM_CB * sizeof(cplx<T>);
  const int64_t nblk = (ncols + TRSM_CB - 1) / TRSM_CB;
  hipLaunchKernelGGL((trsm_kernel<T, KIND>), dim3((unsigned)nblk), dim3(256), lds, st, Tri, ldt, w, B, ldb, ncols);
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
  const size_t nb = (size_t)p.nb, nblk = p.blocks.size(), cb = 2 * (size_t)elem_bytes;
  size_t s = 0;
  s += nb * 4 + 256;
  s += nb * 8 + 256;
  s += 2 * (size_t)num_cu * nb * cb + 256;
  s += 2 * nb * cb + 256;
  s += 64 + 256;
  s += nblk * 2 * 2 * nb * 4 + 256;
  s += nblk * 4 + 256;
  return s;
}

void lu_workspace_carve(void* base, const LUPlan& p, int elem_bytes, int num_cu, LUWork& w) {
  const size_t nb = (size_t)p.nb, nblk = p.blocks.size(), cb = 2 * (size_t)elem_bytes;
  char* b = static_cast<char*>(base);
  auto take = [&](size_t bytes) {
    char* r = b;
    b += (bytes + 255) / 256 * 256 + 256;
    return r;
  };
  w.cnt = reinterpret_cast<uint32_t*>(take(nb * 4));
  w.key = reinterpret_cast<uint64_t*>(take(nb * 8));
  w.slot = take(2 * (size_t)num_cu * nb * cb);
  w.dslot = take(2 * nb * cb);
  w.err = reinterpret_cast<int32_t*>(take(64));
  w.pairs = reinterpret_cast<int32_t*>(take(nblk * 2 * 2 * nb * 4));
  w.npairs = reinterpret_cast<int32_t*>(take(nblk * 4));
}

// ---------------------------------------------------------------------------
// drivers
// ---------------------------------------------------------------------------
template <typename T>
hipError_t lu_factor(void* Av, int64_t ld, const LUPlan& plan, const LUWork& ws, int32_t* ipiv, hipStream_t st) {
  using CT = cplx<T>;
  CT* A = static_cast<CT*>(Av);
  const int64_t n = plan.n;
  const int nb = plan.nb;
  hipError_t e;
  hipLaunchKernelGGL(init_err_kernel, dim3(1), dim3(64), 0, st, ws.err);
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
    if (b.G > plan.max_wg || b.w > nb || (int64_t)b.G * b.R < n - k0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(zero_u32_kernel, dim3((nb + 255) / 256), dim3(256), 0, st, ws.cnt, nb,
                       reinterpret_cast<unsigned long long*>(ws.key), nb);
    const size_t lds = ((size_t)w * b.R + w) * sizeof(CT);
    hipLaunchKernelGGL(panel_kernel<T>, dim3(b.G), dim3(256), lds, st, A, ld, n, k0, w, b.R, b.G, ipiv, ws);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int32_t* dst = ws.pairs + bi * 4 * (size_t)nb;
    int32_t* src = dst + 2 * nb;
    hipLaunchKernelGGL(block_perm_kernel, dim3(1), dim3(64), 0, st, ipiv, k0, w, dst, src, ws.npairs + bi);
    const int64_t c1 = k0 + w;
    const int64_t nr = n - c1;
    if (nr > 0) {
      hipLaunchKernelGGL(row_permute_kernel<T>, dim3((unsigned)nr), dim3(256), 0, st, A, ld, c1, dst, src,
                         ws.npairs + bi);
      if ((e = launch_trsm<T, 0>(A + k0 + k0 * ld, ld, w, A + k0 + c1 * ld, ld, nr, st)) != hipSuccess) return e;
      if ((e = launch_gemm<T>(0, 0, nr, nr, w, A + c1 + k0 * ld, ld, A + k0 + c1 * ld, ld, A + c1 + c1 * ld, ld,
                              st)) != hipSuccess)
        return e;
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

template hipError_t lu_factor<double>(void*, int64_t, const LUPlan&, const LUWork&, int32_t*, hipStream_t);
template hipError_t lu_factor<float>(void*, int64_t, const LUPlan&, const LUWork&, int32_t*, hipStream_t);
template hipError_t lu_solve<double>(int, const void*, int64_t, const LUPlan&, const LUWork&, void*, int64_t, int64_t,
                                     hipStream_t);
template hipError_t lu_solve<float>(int, const void*, int64_t, const LUPlan&, const LUWork&, void*, int64_t, int64_t,
                                    hipStream_t);

}  // namespace gdm
