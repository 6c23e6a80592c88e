// Block steps of the triangular solves for the factors of lu_factor when the
// right-hand sides are few, and for every transposed solve.
//
// The forward/backward steps update many rows from one 128-wide block (an
// m x k product with k <= 256); with 1-8 right-hand sides a 64 x 64 matrix-core
// tile would be almost empty, so a plain VALU kernel streams the block once:
// one row per lane, the k range split over the four waves of a workgroup, the
// right-hand sides staged in LDS, the waves' partial sums combined in LDS.
//
// The steps of a transposed solve produce one 128-row block from a long
// product (k up to n): C[w x nr] -= op(A)^T B, and the transposed refinement
// residual is the same shape with w = n.  Each output is the dot product of a
// stored column of A with B: one wave per column, lanes along k (coalesced
// column reads), the k range split into chunks of KC rows, one partial sum per
// (chunk, column) reduced across the wave; the masked diagonal block is one
// more chunk.  A second kernel adds the partials to C in a fixed order
// (deterministic).  Right-hand sides are processed NR at a time (NR = 1, 2, 4
// or 8 picked from their count; blockIdx.y walks the groups).
#include "gdm_common.hpp"
#include "gdm_kernels.hpp"

namespace gdm {

constexpr int SK_KMAX = 256; // max k of the column-form kernel
constexpr int SK_KC = 256;   // k rows per chunk of the transposed form
constexpr int SK_TCOLS = 16; // output columns per workgroup of the transposed form (4 per wave)

__device__ inline bool sk_keep(int kind, int64_t r, int64_t c) {
  switch (kind) {
    case GEMM_MASK_STRICT_LOWER: return r > c;
    case GEMM_MASK_UPPER: return r <= c;
    case GEMM_MASK_LOWER: return r >= c;
    case GEMM_MASK_STRICT_UPPER: return r < c;
    default: return true;
  }
}

template <typename T>
__device__ inline void cfma_t(cplx<T>& acc, const cplx<T>& a, const cplx<T>& b) {
  acc.x += a.x * b.x - a.y * b.y;
  acc.y += a.x * b.y + a.y * b.x;
}

// C[m x nr] -= A[m x k] X[k x nr]; rows [ar0, ar0 + adw) of A are a square
// block of which only the `akind` triangle is read.  64 rows per workgroup, the
// k range split over its four waves.
// With PART, blockIdx.z selects the k chunk [z SK_KMAX, (z + 1) SK_KMAX) of a
// longer product and the sums go to part[(z * nrhs + r) * m + row] instead.
// Batch: blockIdx.z = item (x nchunk + chunk with PART); item z reads A + z sA,
// X + z sX and writes C + z sC (PART: its own nchunk x nrhs x m partials).
template <typename T, int NR, bool PART>
__global__ void __launch_bounds__(256) skinny_n_kernel(int64_t m, int64_t k, const cplx<T>* __restrict__ A,
                                                        int64_t lda, const cplx<T>* __restrict__ X, int64_t ldx,
                                                        cplx<T>* __restrict__ C, int64_t ldc, int64_t nrhs,
                                                        GemmMask mk, int nchunk, int64_t sA, int64_t sX, int64_t sC) {
  using CT = cplx<T>;
  __shared__ CT xs[SK_KMAX][NR];
  __shared__ CT red[3][64][NR];
  const int64_t item = PART ? blockIdx.z / nchunk : blockIdx.z;
  const int64_t chunk = PART ? blockIdx.z - item * nchunk : 0;
  A += item * sA;
  X += item * sX;
  C += PART ? item * nchunk * nrhs * m : item * sC;
  if (PART) {
    const int64_t kc0 = chunk * SK_KMAX;
    A += kc0 * lda;
    X += kc0;
    k = k - kc0 < SK_KMAX ? k - kc0 : SK_KMAX;
  }
  const int64_t r0 = (int64_t)blockIdx.y * NR;
  const int nr = (int)(nrhs - r0 < NR ? nrhs - r0 : NR);
  for (int t = threadIdx.x; t < k * NR; t += 256) {
    const int kk = t / NR, r = t % NR;
    CT v;
    v.x = 0;
    v.y = 0;
    if (r < nr) v = X[kk + (r0 + r) * ldx];
    xs[kk][r] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t row = (int64_t)blockIdx.x * 64 + lane;
  const int64_t kq = (k + 3) / 4;
  const int64_t ka = wave * kq, kb = ka + kq < k ? ka + kq : k;
  CT acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r].x = acc[r].y = 0;
  if (row < m) {
    const bool masked = mk.akind && row >= mk.ar0 && row < mk.ar0 + mk.adw;
    // KB loads in flight per lane, then their products (a load and its use in
    // one loop body put one memory latency per k on the path); the masked
    // triangle is stored, so it is read and replaced by zero
    constexpr int KB = 16;
    for (int64_t k0 = ka; k0 < kb; k0 += KB) {
      CT a[KB];
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        a[u].x = 0;
        a[u].y = 0;
        if (k0 + u < kb) a[u] = A[row + (k0 + u) * lda];
      }
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        const int64_t kk = k0 + u;
        if (kk < kb) {
          CT v = a[u];
          if (masked && !sk_keep(mk.akind, row - mk.ar0, kk)) v.x = v.y = 0;
#pragma unroll
          for (int r = 0; r < NR; ++r) cfma_t<T>(acc[r], v, xs[kk][r]);
        }
      }
    }
  }
  if (wave > 0)
#pragma unroll
    for (int r = 0; r < NR; ++r) red[wave - 1][lane][r] = acc[r];
  __syncthreads();
  if (wave == 0 && row < m) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (r >= nr) break;  // compile-time indices into acc (no private-memory copy)
      CT s = acc[r];
#pragma unroll
      for (int w = 0; w < 3; ++w) {
        s.x += red[w][lane][r].x;
        s.y += red[w][lane][r].y;
      }
      if (PART) {
        C[(chunk * nrhs + r0 + r) * m + row] = s;
      } else {
        // rows [ar0, ar0 + adw) optionally to the second destination mk.c2
        CT c = C[row + (r0 + r) * ldc];
        c.x -= s.x;
        c.y -= s.y;
        if (mk.c2 && row >= mk.ar0 && row < mk.ar0 + mk.adw)
          static_cast<CT*>(mk.c2)[item * mk.sc2 + (row - mk.ar0) + (r0 + r) * mk.ldc2] = c;
        else
          C[row + (r0 + r) * ldc] = c;
      }
    }
  }
}

struct SkSeg {
  const void* A;  // stored k x mo block (column-major, lda): op(A)[i][kk] = A[kk + i lda]
  int64_t lda;
  const void* B;  // k x nrhs (column-major, ldb)
  int64_t ldb;
  int64_t k;
  int kind;       // triangle kept of the square block (row i, column kk), 0 = all
  int nchunk;
};

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// part[(chunk * nrhs + r) * mo + i] = sum_{kk in chunk} op(A)[i][kk] B[kk][r];
// blockIdx.x = chunk * ngroups + column group (16 columns, 4 per wave).
template <typename T, int NR>
__global__ void __launch_bounds__(256) skinny_t_kernel(SkSeg s0, SkSeg s1, int64_t mo, int64_t nrhs, int ngroups,
                                                        cplx<T>* __restrict__ part, int64_t sA, int64_t sB) {
  using CT = cplx<T>;
  __shared__ CT bs[SK_KC][NR];
  const int64_t item = blockIdx.z;  // batch item: A + item sA, B + item sB, own partials
  part += item * (int64_t)(s0.nchunk + s1.nchunk) * nrhs * mo;
  const int chunk = blockIdx.x / ngroups, grp = blockIdx.x - chunk * ngroups;
  const bool second = chunk >= s0.nchunk;
  const SkSeg& s = second ? s1 : s0;
  const int64_t kc0 = (int64_t)(second ? chunk - s0.nchunk : chunk) * SK_KC;
  const int64_t kc1 = kc0 + SK_KC < s.k ? kc0 + SK_KC : s.k;
  const int64_t r0 = (int64_t)blockIdx.y * NR;
  const int nr = (int)(nrhs - r0 < NR ? nrhs - r0 : NR);
  const CT* A = static_cast<const CT*>(s.A) + item * sA;
  const CT* B = static_cast<const CT*>(s.B) + item * sB;
  for (int t = threadIdx.x; t < (kc1 - kc0) * NR; t += 256) {
    const int kk = t % (int)(kc1 - kc0), r = t / (int)(kc1 - kc0);
    CT v;
    v.x = 0;
    v.y = 0;
    if (r < nr) v = B[kc0 + kk + (r0 + r) * s.ldb];
    bs[kk][r] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // all of this wave's loads (CPW columns x KS steps of 64 rows) in flight at
  // once, then the products column by column; masked entries are stored, so
  // they are read and replaced by zero
  constexpr int CPW = SK_TCOLS / 4, KS = SK_KC / 64;
  const int64_t i0 = (int64_t)grp * SK_TCOLS + wave * CPW;
  CT a[CPW][KS];
#pragma unroll
  for (int c = 0; c < CPW; ++c)
#pragma unroll
    for (int q = 0; q < KS; ++q) {
      const int64_t kk = kc0 + lane + 64 * q;
      a[c][q].x = 0;
      a[c][q].y = 0;
      if (i0 + c < mo && kk < kc1) a[c][q] = A[kk + (i0 + c) * s.lda];
    }
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int64_t i = i0 + c;
    if (i >= mo) break;
    CT acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r].x = acc[r].y = 0;
#pragma unroll
    for (int q = 0; q < KS; ++q) {
      const int64_t kk = kc0 + lane + 64 * q;
      if (kk < kc1) {
        CT v = a[c][q];
        if (s.kind && !sk_keep(s.kind, i, kk)) v.x = v.y = 0;
#pragma unroll
        for (int r = 0; r < NR; ++r) cfma_t<T>(acc[r], v, bs[kk - kc0][r]);
      }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const T re = wave_sum(acc[r].x), im = wave_sum(acc[r].y);
      if (lane == 0 && r < nr) {
        CT v;
        v.x = re;
        v.y = im;
        part[((int64_t)chunk * nrhs + r0 + r) * mo + i] = v;
      }
    }
  }
}

// C[i + r ldc] -= sum_chunk part[(chunk * nrhs + r) * mo + i], chunks in order
template <typename T>
__global__ void skinny_reduce_kernel(const cplx<T>* __restrict__ part, int nchunk, int64_t mo, int64_t nrhs,
                                     cplx<T>* __restrict__ C, int64_t ldc, int64_t sC) {
  using CT = cplx<T>;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= mo * nrhs) return;
  // batch item blockIdx.y: its partials follow those of the previous items
  part += (int64_t)blockIdx.y * nchunk * nrhs * mo;
  C += (int64_t)blockIdx.y * sC;
  const int64_t r = t / mo, i = t - r * mo;
  CT s;
  s.x = 0;
  s.y = 0;
  for (int c = 0; c < nchunk; ++c) {
    const CT v = part[((int64_t)c * nrhs + r) * mo + i];
    s.x += v.x;
    s.y += v.y;
  }
  CT* p = C + i + r * ldc;
  CT c = *p;
  c.x -= s.x;
  c.y -= s.y;
  *p = c;
}

static int pick_nr(int64_t nrhs) { return nrhs <= 1 ? 1 : nrhs <= 2 ? 2 : nrhs <= 4 ? 4 : 8; }

template <typename T>
hipError_t launch_skinny_n(int64_t m, int64_t k, const void* A, int64_t lda, const void* X, int64_t ldx, void* C,
                           int64_t ldc, int64_t nrhs, hipStream_t st, GemmMask mk, int nbatch, int64_t sA, int64_t sX,
                           int64_t sC) {
  if (m <= 0 || nrhs <= 0 || k <= 0 || nbatch <= 0) return hipSuccess;
  if (k > SK_KMAX || nbatch > 65535) return hipErrorInvalidValue;
  const int NRp = pick_nr(nrhs);
  const dim3 grid((unsigned)((m + 63) / 64), (unsigned)((nrhs + NRp - 1) / NRp), (unsigned)nbatch);
  const auto* a = static_cast<const cplx<T>*>(A);
  const auto* x = static_cast<const cplx<T>*>(X);
  auto* c = static_cast<cplx<T>*>(C);
  switch (NRp) {
    case 1: hipLaunchKernelGGL((skinny_n_kernel<T, 1, false>), grid, dim3(256), 0, st, m, k, a, lda, x, ldx, c, ldc, nrhs, mk, 1, sA, sX, sC); break;
    case 2: hipLaunchKernelGGL((skinny_n_kernel<T, 2, false>), grid, dim3(256), 0, st, m, k, a, lda, x, ldx, c, ldc, nrhs, mk, 1, sA, sX, sC); break;
    case 4: hipLaunchKernelGGL((skinny_n_kernel<T, 4, false>), grid, dim3(256), 0, st, m, k, a, lda, x, ldx, c, ldc, nrhs, mk, 1, sA, sX, sC); break;
    default: hipLaunchKernelGGL((skinny_n_kernel<T, 8, false>), grid, dim3(256), 0, st, m, k, a, lda, x, ldx, c, ldc, nrhs, mk, 1, sA, sX, sC); break;
  }
  return hipGetLastError();
}

int64_t skinny_n_long_parts(int64_t m, int64_t k, int64_t nrhs) {
  return (k + SK_KMAX - 1) / SK_KMAX * nrhs * m;
}

template <typename T>
hipError_t launch_skinny_n_long(int64_t m, int64_t k, const void* A, int64_t lda, const void* X, int64_t ldx, void* C,
                                int64_t ldc, int64_t nrhs, void* part, int64_t part_elems, hipStream_t st, int nbatch,
                                int64_t sA, int64_t sX, int64_t sC) {
  if (m <= 0 || nrhs <= 0 || k <= 0 || nbatch <= 0) return hipSuccess;
  const int64_t nchunk = (k + SK_KMAX - 1) / SK_KMAX;
  if (nbatch * skinny_n_long_parts(m, k, nrhs) > part_elems || nchunk * nbatch > 65535 || nbatch > 65535)
    return hipErrorInvalidValue;
  const int NRp = pick_nr(nrhs);
  const dim3 grid((unsigned)((m + 63) / 64), (unsigned)((nrhs + NRp - 1) / NRp), (unsigned)(nchunk * nbatch));
  const auto* a = static_cast<const cplx<T>*>(A);
  const auto* x = static_cast<const cplx<T>*>(X);
  auto* p = static_cast<cplx<T>*>(part);
  const GemmMask mk{};
  const int nc = (int)nchunk;
  switch (NRp) {
    case 1: hipLaunchKernelGGL((skinny_n_kernel<T, 1, true>), grid, dim3(256), 0, st, m, k, a, lda, x, ldx, p, m, nrhs, mk, nc, sA, sX, (int64_t)0); break;
    case 2: hipLaunchKernelGGL((skinny_n_kernel<T, 2, true>), grid, dim3(256), 0, st, m, k, a, lda, x, ldx, p, m, nrhs, mk, nc, sA, sX, (int64_t)0); break;
    case 4: hipLaunchKernelGGL((skinny_n_kernel<T, 4, true>), grid, dim3(256), 0, st, m, k, a, lda, x, ldx, p, m, nrhs, mk, nc, sA, sX, (int64_t)0); break;
    default: hipLaunchKernelGGL((skinny_n_kernel<T, 8, true>), grid, dim3(256), 0, st, m, k, a, lda, x, ldx, p, m, nrhs, mk, nc, sA, sX, (int64_t)0); break;
  }
  const int64_t tot = m * nrhs;
  hipLaunchKernelGGL(skinny_reduce_kernel<T>, dim3((unsigned)((tot + 255) / 256), (unsigned)nbatch), dim3(256), 0, st, p,
                     nc, m, nrhs, static_cast<cplx<T>*>(C), ldc, sC);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_partial_reduce(const void* part, int nchunk, int64_t mo, int64_t nrhs, void* C, int64_t ldc,
                                 hipStream_t st) {
  if (mo <= 0 || nrhs <= 0 || nchunk <= 0) return hipSuccess;
  const int64_t tot = mo * nrhs;
  hipLaunchKernelGGL(skinny_reduce_kernel<T>, dim3((unsigned)((tot + 255) / 256), 1), dim3(256), 0, st,
                     static_cast<const cplx<T>*>(part), nchunk, mo, nrhs, static_cast<cplx<T>*>(C), ldc, (int64_t)0);
  return hipGetLastError();
}
template hipError_t launch_partial_reduce<double>(const void*, int, int64_t, int64_t, void*, int64_t, hipStream_t);
template hipError_t launch_partial_reduce<float>(const void*, int, int64_t, int64_t, void*, int64_t, hipStream_t);

int64_t skinny_t_chunks(int64_t k0, int64_t k1) {
  return (k0 + SK_KC - 1) / SK_KC + (k1 + SK_KC - 1) / SK_KC;
}

template <typename T>
hipError_t launch_skinny_t(int64_t mo, int64_t nrhs, const void* A0, int64_t lda0, const void* B0, int64_t ldb0,
                           int64_t k0, const void* A1, int64_t lda1, const void* B1, int64_t ldb1, int64_t k1,
                           int kind1, void* part, int64_t part_elems, void* C, int64_t ldc, hipStream_t st, int nbatch,
                           int64_t sA, int64_t sB, int64_t sC) {
  if (mo <= 0 || nrhs <= 0 || nbatch <= 0) return hipSuccess;
  SkSeg s0{A0, lda0, B0, ldb0, k0, 0, (int)((k0 + SK_KC - 1) / SK_KC)};
  SkSeg s1{A1, lda1, B1, ldb1, k1, kind1, (int)((k1 + SK_KC - 1) / SK_KC)};
  const int nchunk = s0.nchunk + s1.nchunk;
  if (nchunk == 0) return hipSuccess;
  if ((int64_t)nbatch * nchunk * nrhs * mo > part_elems || nbatch > 65535) return hipErrorInvalidValue;
  const int64_t ngroups = (mo + SK_TCOLS - 1) / SK_TCOLS;
  if ((int64_t)nchunk * ngroups > INT32_MAX) return hipErrorInvalidValue;
  const int NRp = pick_nr(nrhs);
  const dim3 grid((unsigned)(nchunk * ngroups), (unsigned)((nrhs + NRp - 1) / NRp), (unsigned)nbatch);
  auto* p = static_cast<cplx<T>*>(part);
  const int ng = (int)ngroups;
  switch (NRp) {
    case 1: hipLaunchKernelGGL((skinny_t_kernel<T, 1>), grid, dim3(256), 0, st, s0, s1, mo, nrhs, ng, p, sA, sB); break;
    case 2: hipLaunchKernelGGL((skinny_t_kernel<T, 2>), grid, dim3(256), 0, st, s0, s1, mo, nrhs, ng, p, sA, sB); break;
    case 4: hipLaunchKernelGGL((skinny_t_kernel<T, 4>), grid, dim3(256), 0, st, s0, s1, mo, nrhs, ng, p, sA, sB); break;
    default: hipLaunchKernelGGL((skinny_t_kernel<T, 8>), grid, dim3(256), 0, st, s0, s1, mo, nrhs, ng, p, sA, sB); break;
  }
  const int64_t tot = mo * nrhs;
  hipLaunchKernelGGL(skinny_reduce_kernel<T>, dim3((unsigned)((tot + 255) / 256), (unsigned)nbatch), dim3(256), 0, st, p,
                     nchunk, mo, nrhs, static_cast<cplx<T>*>(C), ldc, sC);
  return hipGetLastError();
}

template hipError_t launch_skinny_n<double>(int64_t, int64_t, const void*, int64_t, const void*, int64_t, void*,
                                            int64_t, int64_t, hipStream_t, GemmMask, int, int64_t, int64_t, int64_t);
template hipError_t launch_skinny_n<float>(int64_t, int64_t, const void*, int64_t, const void*, int64_t, void*,
                                           int64_t, int64_t, hipStream_t, GemmMask, int, int64_t, int64_t, int64_t);
template hipError_t launch_skinny_n_long<double>(int64_t, int64_t, const void*, int64_t, const void*, int64_t, void*,
                                                 int64_t, int64_t, void*, int64_t, hipStream_t, int, int64_t, int64_t,
                                                 int64_t);
template hipError_t launch_skinny_n_long<float>(int64_t, int64_t, const void*, int64_t, const void*, int64_t, void*,
                                                int64_t, int64_t, void*, int64_t, hipStream_t, int, int64_t, int64_t,
                                                int64_t);
template hipError_t launch_skinny_t<double>(int64_t, int64_t, const void*, int64_t, const void*, int64_t, int64_t,
                                            const void*, int64_t, const void*, int64_t, int64_t, int, void*, int64_t,
                                            void*, int64_t, hipStream_t, int, int64_t, int64_t, int64_t);
template hipError_t launch_skinny_t<float>(int64_t, int64_t, const void*, int64_t, const void*, int64_t, int64_t,
                                           const void*, int64_t, const void*, int64_t, int64_t, int, void*, int64_t,
                                           void*, int64_t, hipStream_t, int, int64_t, int64_t, int64_t);

}  // namespace gdm
