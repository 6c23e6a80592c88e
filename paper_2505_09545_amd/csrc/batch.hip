// Kernels of the batched spectra driver: many systems of one structure (the
// same cells, one permittivity per wavelength) solved together, as in the
// paper's spectra over wavelengths (Sec. "Implementation technical details";
// its Sec. "Observables" defines the cross sections reduced here).
//
// A group holds B items (wavelengths) of one structure of N cubic cells
// (n = 3N unknowns, electric only).  Item z's data sit at a fixed stride: its
// matrices at M + z n^2, its vectors at [z][n_pw][n].  The per-item physics is
// the same as in the single-system kernels: alpha = (eps - eps_env) d^3/(4 pi),
// S = -4 pi/(3 eps_env d^3) (+ i (2/3) k^3/eps_env for the radiative option),
// M = I - G~ A with the dyad of gdm_common.hpp, plane waves e0 exp(i k khat.r),
// q = alpha F, and the cross sections C Im(F0^* q), C Im(F^* q) (cells carry no
// radiation-reaction term), C = 4 pi k0 / (n_env |e0|^2).
#include "gdm_batch.hpp"

namespace gdm {

// Per-item parameters of one group: items beyond nvalid repeat the last valid
// wavelength (their results are computed and discarded).
__global__ void batch_stage_kernel(const double2* __restrict__ eps, int64_t n_wl, int64_t s, int64_t l0,
                                   int64_t nvalid, int B, const double* __restrict__ wl, double eps_env, double f,
                                   double2* __restrict__ alpha, double* __restrict__ k0) {
  const int z = threadIdx.x;
  if (z >= B) return;
  const int64_t l = l0 + (z < nvalid ? z : nvalid - 1);
  const double2 e = eps[s * n_wl + l];
  alpha[z] = make_double2((e.x - eps_env) * f, e.y * f);
  k0[z] = 2.0 * M_PI / wl[l];
}

// One thread per (row cell s, column cell j) of item blockIdx.y; the 3 x 3 block
// is evaluated once in FP64 and stored as complex double and, with DUAL, as
// complex float too.
template <bool DUAL>
__global__ void __launch_bounds__(256) batch_assemble_kernel(const double* __restrict__ pos, int64_t N,
                                                              const double2* __restrict__ alpha,
                                                              const double* __restrict__ k0s, double n_env, double d3,
                                                              int radiative, double2* __restrict__ M64,
                                                              float2* __restrict__ M32, int64_t ld, int64_t sM,
                                                              int64_t row_blocks) {
  const int64_t item = blockIdx.y;
  const int64_t j = blockIdx.x / row_blocks;
  const int64_t s = (blockIdx.x % row_blocks) * blockDim.x + threadIdx.x;
  if (s >= N) return;
  Wave w;
  w.k0 = k0s[item];
  w.k = n_env * w.k0;
  w.eps_env = n_env * n_env;
  const double2 al = alpha[item];
  double2 v[3][3];
  if (s == j) {
    double2 S = make_double2(-4.0 * M_PI / (3.0 * w.eps_env * d3), 0.0);
    if (radiative) S.y = (2.0 / 3.0) * w.k * w.k * w.k / w.eps_env;
    const double2 dg = csub(make_double2(1.0, 0.0), cmul(S, al));
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int a = 0; a < 3; ++a) v[a][c] = a == c ? dg : make_double2(0.0, 0.0);
  } else {
    Green g;
    green_eh(pos[3 * s] - pos[3 * j], pos[3 * s + 1] - pos[3 * j + 1], pos[3 * s + 2] - pos[3 * j + 2], w, false, g);
    const double2 ma = make_double2(-al.x, -al.y);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int a = 0; a < 3; ++a) v[a][c] = cmul(gep(g, a, c), ma);
  }
  double2* m64 = M64 + item * sM + 3 * s + 3 * j * ld;
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int a = 0; a < 3; ++a) m64[a + c * ld] = v[a][c];
  if (DUAL) {
    float2* m32 = M32 + item * sM + 3 * s + 3 * j * ld;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int a = 0; a < 3; ++a) m32[a + c * ld] = make_float2((float)v[a][c].x, (float)v[a][c].y);
  }
}

// f0[(z n_pw + r) n + u] = e0_r[a] exp(i k_z khat_r . r_cell(u))
__global__ void batch_incident_kernel(const double* __restrict__ pos, int64_t n, const double* __restrict__ k0s,
                                      double n_env, int64_t npw, const double* __restrict__ khat,
                                      const double2* __restrict__ e0, double2* __restrict__ f0) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = blockIdx.y, z = blockIdx.z;
  if (u >= n) return;
  const int64_t c = u / 3;
  const int a = (int)(u % 3);
  const double k = n_env * k0s[z];
  double sn, cs;
  sincos(k * (khat[3 * r] * pos[3 * c] + khat[3 * r + 1] * pos[3 * c + 1] + khat[3 * r + 2] * pos[3 * c + 2]), &sn,
         &cs);
  f0[(z * npw + r) * n + u] = cmul(e0[3 * r + a], make_double2(cs, sn));
}

// q[col n + u] = alpha_z F[col n + u], col = z n_pw + r
__global__ void batch_apply_alpha_kernel(const double2* __restrict__ alpha, const double2* __restrict__ F,
                                         double2* __restrict__ q, int64_t n, int64_t npw) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t col = blockIdx.y;
  if (u >= n) return;
  q[col * n + u] = cmul(alpha[col / npw], F[col * n + u]);
}

// rows[z n + i] = sum_j |M_z[i, j]| (one thread per row, columns in order)
__global__ void batch_rowsum_kernel(const double2* __restrict__ M, int64_t ld, int64_t n, int64_t sM,
                                    double* __restrict__ rows) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t z = blockIdx.y;
  if (i >= n) return;
  const double2* m = M + z * sM + i;
  double s = 0;
  for (int64_t j = 0; j < n; ++j) {
    const double2 v = m[j * ld];
    s += sqrt(v.x * v.x + v.y * v.y);
  }
  rows[z * n + i] = s;
}

// minf[z] = max_i rows[z n + i]
__global__ void __launch_bounds__(256) batch_rowmax_kernel(const double* __restrict__ rows, int64_t n,
                                                           double* __restrict__ minf) {
  __shared__ double red[256];
  const int64_t z = blockIdx.x;
  double m = 0;
  for (int64_t i = threadIdx.x; i < n; i += 256) m = fmax(m, rows[z * n + i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) minf[z] = red[0];
}

// be[z] = max_r |r|_inf / (|M_z|_inf |x|_inf + |f0|_inf) over the item's columns
__global__ void batch_be_kernel(const double* __restrict__ rmax, const double* __restrict__ xmax,
                                const double* __restrict__ bmax, const double* __restrict__ minf, int64_t npw, int B,
                                double* __restrict__ be) {
  const int z = threadIdx.x;
  if (z >= B) return;
  double m = 0;
  for (int64_t r = 0; r < npw; ++r) {
    const int64_t c = z * npw + r;
    const double den = minf[z] * xmax[c] + bmax[c];
    const double v = den > 0 ? rmax[c] / den : 0.0;
    m = v > m ? v : m;
  }
  be[z] = m;
}

// out[(z n_pw + r) 3 + (0, 1, 2)] = (ext, sca, abs) from the FP64 sums of cs_sums
__global__ void batch_cs_kernel(const double* __restrict__ sums5, const double* __restrict__ k0s, double n_env,
                                const double2* __restrict__ e0, int64_t npw, int B, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)B * npw) return;
  const int64_t z = t / npw, r = t - z * npw;
  double e2 = 0;
  for (int a = 0; a < 3; ++a) e2 += e0[3 * r + a].x * e0[3 * r + a].x + e0[3 * r + a].y * e0[3 * r + a].y;
  const double C = 4.0 * M_PI * k0s[z] / (n_env * e2);
  const double ext = C * sums5[5 * t], ab = C * sums5[5 * t + 1];
  out[3 * t] = ext;
  out[3 * t + 1] = ext - ab;
  out[3 * t + 2] = ab;
}

// copy the valid items of a group to the caller's arrays
__global__ void batch_unstage_kernel(const double* __restrict__ cs, const double* __restrict__ be, int64_t nvalid,
                                     int64_t npw, int64_t base, double* __restrict__ cs_out,
                                     double* __restrict__ be_out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nvalid * npw * 3) cs_out[base * npw * 3 + t] = cs[t];
  if (be_out && t < nvalid) be_out[base + t] = be[t];
}

// sticky[0] |= err[0] (exchange timeout), sticky[1] = min(sticky[1], err[1]) (zero pivot)
__global__ void batch_err_kernel(const int32_t* __restrict__ err, int32_t* __restrict__ sticky) {
  if (threadIdx.x == 0) {
    sticky[0] |= err[0];
    sticky[1] = err[1] < sticky[1] ? err[1] : sticky[1];
  }
}

// Speculative panels of a group: failed[z] = OR over the blocks of item z's
// flags (flags of item z at flags + z * sflag, nblk of them).
__global__ void batch_spec_collect_kernel(const int32_t* __restrict__ flags, int64_t sflag, int nblk, int B,
                                          int32_t* __restrict__ failed) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= B) return;
  int32_t f = 0;
  for (int b = 0; b < nblk; ++b) f |= flags[(int64_t)z * sflag + b];
  failed[z] = f;
}

// Append the global indices (base + z) of the group's failed items to list,
// count[0] holding the number of entries (capacity cap).
__global__ void batch_spec_list_kernel(const int32_t* __restrict__ failed, int64_t nvalid, int64_t base,
                                       int64_t* __restrict__ list, int32_t* __restrict__ count, int64_t cap) {
  const int64_t z = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= nvalid || !failed[z]) return;
  const int slot = atomicAdd(count, 1);
  if (slot < cap) list[slot] = base + z;
}

// be_max[0] = max(be_max[0], be[z < nvalid])
__global__ void batch_bemax_kernel(const double* __restrict__ be, int64_t nvalid, double* __restrict__ be_max) {
  if (threadIdx.x == 0) {
    double m = be_max[0];
    for (int64_t z = 0; z < nvalid; ++z) m = be[z] > m ? be[z] : m;
    be_max[0] = m;
  }
}

__global__ void batch_err_init_kernel(int32_t* __restrict__ sticky) {
  if (threadIdx.x == 0) {
    sticky[0] = 0;
    sticky[1] = INT32_MAX;
  }
}

hipError_t launch_batch_stage(const double2* eps, int64_t n_wl, int64_t s, int64_t l0, int64_t nvalid, int B,
                              const double* wl, double eps_env, double step, double2* alpha, double* k0,
                              hipStream_t st) {
  const double f = step * step * step / (4.0 * M_PI);
  hipLaunchKernelGGL(batch_stage_kernel, dim3(1), dim3(64 * ((B + 63) / 64)), 0, st, eps, n_wl, s, l0, nvalid, B, wl,
                     eps_env, f, alpha, k0);
  return hipGetLastError();
}

hipError_t launch_batch_assemble(const double* pos, int64_t N, const double2* alpha, const double* k0s, double n_env,
                                 double step, int radiative, double2* M64, float2* M32, int B, hipStream_t st) {
  if (N <= 0 || B <= 0) return hipSuccess;
  const int64_t n = 3 * N;
  const int64_t row_blocks = (N + 255) / 256;
  const dim3 grid((unsigned)(row_blocks * N), (unsigned)B);
  const double d3 = step * step * step;
  if (M32)
    hipLaunchKernelGGL(batch_assemble_kernel<true>, grid, dim3(256), 0, st, pos, N, alpha, k0s, n_env, d3, radiative,
                       M64, M32, n, n * n, row_blocks);
  else
    hipLaunchKernelGGL(batch_assemble_kernel<false>, grid, dim3(256), 0, st, pos, N, alpha, k0s, n_env, d3, radiative,
                       M64, M32, n, n * n, row_blocks);
  return hipGetLastError();
}

hipError_t launch_batch_incident(const double* pos, int64_t n, const double* k0s, double n_env, int64_t npw,
                                 const double* khat, const double2* e0, double2* f0, int B, hipStream_t st) {
  hipLaunchKernelGGL(batch_incident_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)npw, (unsigned)B), dim3(256), 0,
                     st, pos, n, k0s, n_env, npw, khat, e0, f0);
  return hipGetLastError();
}

hipError_t launch_batch_apply_alpha(const double2* alpha, const double2* F, double2* q, int64_t n, int64_t npw, int B,
                                    hipStream_t st) {
  hipLaunchKernelGGL(batch_apply_alpha_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)(npw * B)), dim3(256), 0, st,
                     alpha, F, q, n, npw);
  return hipGetLastError();
}

hipError_t launch_batch_minf(const double2* M, int64_t n, int B, double* rows, double* minf, hipStream_t st) {
  hipLaunchKernelGGL(batch_rowsum_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)B), dim3(256), 0, st, M, n, n,
                     n * n, rows);
  hipLaunchKernelGGL(batch_rowmax_kernel, dim3((unsigned)B), dim3(256), 0, st, rows, n, minf);
  return hipGetLastError();
}

hipError_t launch_batch_be(const double* rmax, const double* xmax, const double* bmax, const double* minf,
                           int64_t npw, int B, double* be, hipStream_t st) {
  hipLaunchKernelGGL(batch_be_kernel, dim3(1), dim3(64 * ((B + 63) / 64)), 0, st, rmax, xmax, bmax, minf, npw, B, be);
  return hipGetLastError();
}

hipError_t launch_batch_cs(const double* sums5, const double* k0s, double n_env, const double2* e0, int64_t npw, int B,
                           double* out, hipStream_t st) {
  const int64_t t = (int64_t)B * npw;
  hipLaunchKernelGGL(batch_cs_kernel, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, sums5, k0s, n_env, e0, npw,
                     B, out);
  return hipGetLastError();
}

hipError_t launch_batch_unstage(const double* cs, const double* be, int64_t nvalid, int64_t npw, int64_t base,
                                double* cs_out, double* be_out, hipStream_t st) {
  const int64_t t = nvalid * npw * 3;
  hipLaunchKernelGGL(batch_unstage_kernel, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, cs, be, nvalid, npw,
                     base, cs_out, be_out);
  return hipGetLastError();
}

hipError_t launch_batch_err(const int32_t* err, int32_t* sticky, hipStream_t st) {
  hipLaunchKernelGGL(batch_err_kernel, dim3(1), dim3(64), 0, st, err, sticky);
  return hipGetLastError();
}

hipError_t launch_batch_bemax(const double* be, int64_t nvalid, double* be_max, hipStream_t st) {
  hipLaunchKernelGGL(batch_bemax_kernel, dim3(1), dim3(64), 0, st, be, nvalid, be_max);
  return hipGetLastError();
}

hipError_t launch_batch_err_init(int32_t* sticky, hipStream_t st) {
  hipLaunchKernelGGL(batch_err_init_kernel, dim3(1), dim3(64), 0, st, sticky);
  return hipGetLastError();
}

}  // namespace gdm

namespace gdm {

hipError_t launch_batch_spec_collect(const int32_t* flags, int64_t sflag, int nblk, int B, int32_t* failed,
                                     hipStream_t st) {
  hipLaunchKernelGGL(batch_spec_collect_kernel, dim3((unsigned)((B + 63) / 64)), dim3(64), 0, st, flags, sflag, nblk, B,
                     failed);
  return hipGetLastError();
}

hipError_t launch_batch_spec_list(const int32_t* failed, int64_t nvalid, int64_t base, int64_t* list, int32_t* count,
                                  int64_t cap, hipStream_t st) {
  if (nvalid <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_spec_list_kernel, dim3((unsigned)((nvalid + 63) / 64)), dim3(64), 0, st, failed, nvalid,
                     base, list, count, cap);
  return hipGetLastError();
}

}  // namespace gdm
