// Global polarisability matrices (GPM) in the coupled system and their
// extraction (arXiv:2505.09545, Sec. "Extraction of effective models" and Fig.
// reference_system (b): M effective electric-magnetic dipole pairs of one
// particle share a non-local 6M x 6M polarisability alpha_G, the moments of
// all pairs follow from the illumination at all of them, q_g = alpha_G F_g;
// the pairs of one group do not couple through G~ since alpha_G already holds
// their interaction).
//
// In the system M = I - G~ A the group's columns become I - G~ alpha_G: the
// assembly writes I - G~ for those columns (unit alpha, zero intra-group
// blocks) and gpm_columns_kernel multiplies the off-identity part by alpha_G
// in place, 16 rows of one group per workgroup (the rows' 6M entries staged in
// LDS, all arithmetic in FP64).
//
// Absorption of a group: besides the self terms of every member, the power its
// members radiate into each other's fields, Im sum_{i != j} q_i^H G6_ij q_j,
// is removed (gpm_mutual_kernel), so that ext - abs is the power radiated by
// all dipoles (the paper's own code obtains GPM absorption as ext minus the
// far-field integral; the two agree exactly).
//
// Extraction (field matching, then alpha_G = F0^+ P): the scattered (E, H) at
// P probes is fitted by 6M dipole moments through the 6P x 6M matrix of dyads
// G6(r_p - r_j), and the moments of all illuminations by alpha_G applied to the
// illuminations' (E0, H0) at the pairs; both least-squares problems by
// Householder QR, one launch per column (one workgroup per remaining column,
// each recomputing the reflector from the same deterministic reduction).
#include <cmath>

#include "gdm_common.hpp"
#include "gdm_kernels.hpp"
#include "gdm_misc.hpp"

namespace gdm {

// unknown index of component a (p then m) of effective dipole e
__device__ inline int64_t gpm_col(const DipoleView& d, int64_t e, int a) {
  return a < 3 ? 3 * (d.nc + e) + a : 3 * (d.N + e) + (a - 3);
}

constexpr int GPM_RB = 16;  // rows per workgroup of the column transform

template <bool W64, bool W32>
__global__ void __launch_bounds__(256) gpm_columns_kernel(DipoleView d, double2* __restrict__ M64,
                                                          float2* __restrict__ M32, int64_t ld, int64_t n) {
  __shared__ double2 tile[6 * GPM_MAX_PAIRS * GPM_RB];  // [k][row]: delta - M'
  const int64_t g = blockIdx.y;
  const int64_t first = d.gtab[3 * g], M = d.gtab[3 * g + 1];
  const double2* aG = d.galpha + d.gtab[3 * g + 2];
  const int K = (int)(6 * M);
  const int64_t r0 = (int64_t)blockIdx.x * GPM_RB;
  for (int idx = threadIdx.x; idx < K * GPM_RB; idx += 256) {
    const int k = idx / GPM_RB, rr = idx % GPM_RB;
    const int64_t r = r0 + rr;
    double2 v = make_double2(0.0, 0.0);
    if (r < n) {
      const int64_t col = gpm_col(d, first + k / 6, k % 6);
      double2 m;
      if (W64) {
        m = M64[r + col * ld];
      } else {
        const float2 f = M32[r + col * ld];
        m = make_double2((double)f.x, (double)f.y);
      }
      v = make_double2((r == col ? 1.0 : 0.0) - m.x, -m.y);
    }
    tile[idx] = v;
  }
  __syncthreads();
  const int rr = threadIdx.x % GPM_RB;
  const int64_t r = r0 + rr;
  if (r >= n) return;
  for (int c = threadIdx.x / GPM_RB; c < K; c += 256 / GPM_RB) {
    double2 s = make_double2(0.0, 0.0);
    for (int k = 0; k < K; ++k) cfma(s, tile[k * GPM_RB + rr], aG[(int64_t)k * K + c]);
    const int64_t col = gpm_col(d, first + c / 6, c % 6);
    const double2 o = make_double2((r == col ? 1.0 : 0.0) - s.x, -s.y);
    if (W64) M64[r + col * ld] = o;
    if (W32) M32[r + col * ld] = make_float2((float)o.x, (float)o.y);
  }
}

hipError_t launch_gpm_columns(const DipoleView& d, double2* M64, float2* M32, int64_t ld, int64_t n, hipStream_t st) {
  if (d.ngroups <= 0 || n <= 0) return hipSuccess;
  const dim3 grid((unsigned)((n + GPM_RB - 1) / GPM_RB), (unsigned)d.ngroups);
  if (M64 && M32) hipLaunchKernelGGL((gpm_columns_kernel<true, true>), grid, dim3(256), 0, st, d, M64, M32, ld, n);
  else if (M64) hipLaunchKernelGGL((gpm_columns_kernel<true, false>), grid, dim3(256), 0, st, d, M64, M32, ld, n);
  else hipLaunchKernelGGL((gpm_columns_kernel<false, true>), grid, dim3(256), 0, st, d, M64, M32, ld, n);
  return hipGetLastError();
}

// one workgroup per (group, RHS)
__global__ void __launch_bounds__(256) gpm_apply_kernel(DipoleView d, const double2* __restrict__ F, int64_t ldf,
                                                        double2* __restrict__ q, int64_t ldq) {
  __shared__ double2 f[6 * GPM_MAX_PAIRS];
  const int64_t g = blockIdx.x, r = blockIdx.y;
  const int64_t first = d.gtab[3 * g], M = d.gtab[3 * g + 1];
  const double2* aG = d.galpha + d.gtab[3 * g + 2];
  const int K = (int)(6 * M);
  const double2* fr = F + r * ldf;
  double2* qr = q + r * ldq;
  for (int k = threadIdx.x; k < K; k += 256) f[k] = fr[gpm_col(d, first + k / 6, k % 6)];
  __syncthreads();
  for (int row = threadIdx.x; row < K; row += 256) {
    double2 s = make_double2(0.0, 0.0);
    for (int k = 0; k < K; ++k) cfma(s, aG[(int64_t)row * K + k], f[k]);
    qr[gpm_col(d, first + row / 6, row % 6)] = s;
  }
}

hipError_t launch_gpm_apply(const DipoleView& d, const double2* F, int64_t ldf, double2* q, int64_t ldq, int64_t nrhs,
                            hipStream_t st) {
  if (d.ngroups <= 0 || nrhs <= 0) return hipSuccess;
  if (F == q) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gpm_apply_kernel, dim3((unsigned)d.ngroups, (unsigned)nrhs), dim3(256), 0, st, d, F, ldf, q, ldq);
  return hipGetLastError();
}

// one workgroup per (group, RHS): threads over the ordered member pairs
__global__ void __launch_bounds__(256) gpm_mutual_kernel(DipoleView d, Wave w, const double2* __restrict__ q,
                                                         int64_t ldq, double* __restrict__ out) {
  __shared__ double2 sq[6 * GPM_MAX_PAIRS];
  __shared__ double red[256];
  const int64_t g = blockIdx.x, r = blockIdx.y;
  const int64_t first = d.gtab[3 * g], M = d.gtab[3 * g + 1];
  const double2* qr = q + r * ldq;
  for (int k = threadIdx.x; k < 6 * M; k += 256) sq[k] = qr[gpm_col(d, first + k / 6, k % 6)];
  __syncthreads();
  double acc = 0.0;
  for (int64_t p = threadIdx.x; p < M * M; p += 256) {
    const int64_t i = p / M, j = p % M;
    if (i == j) continue;
    const double* ri = d.pos + 3 * (d.nc + first + i);
    const double* rj = d.pos + 3 * (d.nc + first + j);
    Green gr;
    green_eh(ri[0] - rj[0], ri[1] - rj[1], ri[2] - rj[2], w, true, gr);
    double2 s = make_double2(0.0, 0.0);
    for (int a = 0; a < 6; ++a) {
      double2 v = make_double2(0.0, 0.0);
      for (int b = 0; b < 6; ++b) cfma(v, g6(gr, w.eps_env, a, b), sq[6 * j + b]);
      cfma(s, cconj(sq[6 * i + a]), v);
    }
    acc += s.y;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[r * d.ngroups + g] = red[0];
}

hipError_t launch_gpm_mutual(const DipoleView& d, const Wave& w, const double2* q, int64_t ldq, int64_t nrhs,
                             double* out, hipStream_t st) {
  if (d.ngroups <= 0 || nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(gpm_mutual_kernel, dim3((unsigned)d.ngroups, (unsigned)nrhs), dim3(256), 0, st, d, w, q, ldq,
                     out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// extraction
// ---------------------------------------------------------------------------
__global__ void gpm_pack_fields_kernel(const double2* __restrict__ E, const double2* __restrict__ H, int64_t nrhs,
                                       int64_t P, double2* __restrict__ Y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // over nrhs * 6P
  if (t >= nrhs * 6 * P) return;
  const int64_t r = t / (6 * P), u = t % (6 * P), p = u / 6;
  const int a = (int)(u % 6);
  Y[t] = a < 3 ? E[(r * P + p) * 3 + a] : H[(r * P + p) * 3 + (a - 3)];
}

hipError_t launch_gpm_pack_fields(const double2* E, const double2* H, int64_t nrhs, int64_t P, double2* Y,
                                  hipStream_t st) {
  const int64_t tot = nrhs * 6 * P;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(gpm_pack_fields_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, E, H, nrhs, P, Y);
  return hipGetLastError();
}

// one thread per (probe, pair)
__global__ void gpm_fit_matrix_kernel(Wave w, const double* __restrict__ rp, int64_t P, const double* __restrict__ rg,
                                      int64_t M, double2* __restrict__ Gf) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P * M) return;
  const int64_t p = t % P, j = t / P;
  Green g;
  green_eh(rp[3 * p] - rg[3 * j], rp[3 * p + 1] - rg[3 * j + 1], rp[3 * p + 2] - rg[3 * j + 2], w, true, g);
  const int64_t m = 6 * P;
  for (int b = 0; b < 6; ++b)
    for (int a = 0; a < 6; ++a) Gf[(6 * p + a) + (6 * j + b) * m] = g6(g, w.eps_env, a, b);
}

hipError_t launch_gpm_fit_matrix(const Wave& w, const double* rp, int64_t P, const double* rg, int64_t M,
                                 double2* Gf, hipStream_t st) {
  if (P * M <= 0) return hipSuccess;
  hipLaunchKernelGGL(gpm_fit_matrix_kernel, dim3((unsigned)((P * M + 127) / 128)), dim3(128), 0, st, w, rp, P, rg, M,
                     Gf);
  return hipGetLastError();
}

// one thread per (illumination, pair)
__global__ void gpm_illumination_kernel(Wave w, double n_env, const double* __restrict__ rg, int64_t M, int64_t n_pw,
                                        const double* __restrict__ khat, const double2* __restrict__ e0,
                                        int64_t n_src, const double* __restrict__ rs, const double2* __restrict__ ds,
                                        double2* __restrict__ F0g) {
  const int64_t N = n_pw + n_src;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * M) return;
  const int64_t i = t % N, j = t / N;
  double2 o[6];
  illumination_at(w, n_env, rg[3 * j], rg[3 * j + 1], rg[3 * j + 2], i, n_pw, khat, e0, rs, ds, o);
  for (int a = 0; a < 6; ++a) F0g[i + (6 * j + a) * N] = o[a];
}

hipError_t launch_gpm_illumination(const Wave& w, double n_env, const double* rg, int64_t M, int64_t n_pw,
                                   const double* khat, const double2* e0, int64_t n_src, const double* rs,
                                   const double2* ds, double2* F0g, hipStream_t st) {
  const int64_t tot = (n_pw + n_src) * M;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(gpm_illumination_kernel, dim3((unsigned)((tot + 127) / 128)), dim3(128), 0, st, w, n_env, rg, M,
                     n_pw, khat, e0, n_src, rs, ds, F0g);
  return hipGetLastError();
}

__global__ void transpose_kernel(const double2* __restrict__ A, int64_t m, int64_t n, double2* __restrict__ B) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // over B's entries, column-major n x m
  if (t >= m * n) return;
  const int64_t i = t % n, j = t / n;  // B(i, j) = A(j, i)
  B[t] = A[j + i * m];
}

hipError_t launch_transpose(const double2* A, int64_t m, int64_t n, double2* B, hipStream_t st) {
  if (m * n <= 0) return hipSuccess;
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)((m * n + 255) / 256)), dim3(256), 0, st, A, m, n, B);
  return hipGetLastError();
}

// sum over the workgroup (256 threads) in a fixed order
__device__ inline double qr_wg_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return ((red[0] + red[1]) + red[2]) + red[3];
}

// |B_r|^2 over rows [m0, m) of each column r: one workgroup per column
__global__ void __launch_bounds__(256) colnorm2_kernel(const double2* __restrict__ B, int64_t m0, int64_t m,
                                                       double* __restrict__ out) {
  __shared__ double red[4];
  const double2* b = B + (int64_t)blockIdx.x * m;
  double s = 0.0;
  for (int64_t i = m0 + threadIdx.x; i < m; i += 256) s += b[i].x * b[i].x + b[i].y * b[i].y;
  s = qr_wg_sum(s, red);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// Householder step `col`: reflector H = I - 2 v v^H / |v|^2 with v = x + e^{i arg x0}
// |x| e_0 for x = A[col:, col]; workgroup b applies it to column col + 1 + b of A
// (b < K - col - 1) or to column b - (K - col - 1) of B.  Every workgroup derives
// v from the same reduction, so all see the same reflector; column col keeps x
// below the diagonal and R_cc goes to rdiag.
__global__ void __launch_bounds__(256) hh_step_kernel(double2* __restrict__ A, int64_t m, int K,
                                                      double2* __restrict__ B, int col, double2* __restrict__ rdiag) {
  __shared__ double red[4];
  const double2* x = A + (int64_t)col * m;
  double s2 = 0.0;
  for (int64_t i = col + threadIdx.x; i < m; i += 256) s2 += x[i].x * x[i].x + x[i].y * x[i].y;
  const double nx2 = qr_wg_sum(s2, red);
  const double nx = sqrt(nx2);
  const double2 x0 = x[col];
  const double ax0 = sqrt(x0.x * x0.x + x0.y * x0.y);
  const double2 ph = ax0 > 0 ? make_double2(x0.x / ax0, x0.y / ax0) : make_double2(1.0, 0.0);
  const double2 v0 = make_double2(x0.x + ph.x * nx, x0.y + ph.y * nx);
  const double vn2 = nx2 - ax0 * ax0 + (v0.x * v0.x + v0.y * v0.y);
  if (blockIdx.x == 0 && threadIdx.x == 0) rdiag[col] = make_double2(-ph.x * nx, -ph.y * nx);
  if (!(vn2 > 0)) return;  // uniform: a zero column leaves the rest unchanged
  const int na = K - col - 1;
  double2* a = (int)blockIdx.x < na ? A + (int64_t)(col + 1 + blockIdx.x) * m : B + (int64_t)(blockIdx.x - na) * m;
  double sr = 0.0, si = 0.0;
  for (int64_t i = col + threadIdx.x; i < m; i += 256) {
    const double2 vi = i == col ? v0 : x[i];
    const double2 ai = a[i];
    sr += vi.x * ai.x + vi.y * ai.y;  // conj(v_i) a_i
    si += vi.x * ai.y - vi.y * ai.x;
  }
  const double tr = qr_wg_sum(sr, red);
  const double ti = qr_wg_sum(si, red);
  const double f = 2.0 / vn2;
  for (int64_t i = col + threadIdx.x; i < m; i += 256) {
    const double2 vi = i == col ? v0 : x[i];
    const double2 u = make_double2(f * (vi.x * tr - vi.y * ti), f * (vi.x * ti + vi.y * tr));
    a[i] = make_double2(a[i].x - u.x, a[i].y - u.y);
  }
}

// R X = (Q^H B)[0:K] for one column of X per thread; R's strict upper part in
// A, its diagonal in rdiag.
__global__ void qr_backsolve_kernel(const double2* __restrict__ A, int64_t m, int K, const double2* __restrict__ B,
                                    int R, const double2* __restrict__ rdiag, double2* __restrict__ X) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= R) return;
  double dmax = 0.0, dmin = INFINITY;
  for (int a = 0; a < K; ++a) {
    const double v = sqrt(rdiag[a].x * rdiag[a].x + rdiag[a].y * rdiag[a].y);
    dmax = v > dmax ? v : dmax;
    dmin = v < dmin ? v : dmin;
  }
  double2* xc = X + (int64_t)c * K;
  if (!(dmin > 1e-12 * dmax)) {
    for (int a = 0; a < K; ++a) xc[a] = make_double2(NAN, NAN);
    return;
  }
  const double2* bc = B + (int64_t)c * m;
  for (int a = K - 1; a >= 0; --a) {
    double2 s = bc[a];
    for (int b = a + 1; b < K; ++b) {
      const double2 r = A[a + (int64_t)b * m];
      const double2 xb = xc[b];
      s.x -= r.x * xb.x - r.y * xb.y;
      s.y -= r.x * xb.y + r.y * xb.x;
    }
    const double2 dg = rdiag[a];
    const double dn = dg.x * dg.x + dg.y * dg.y;
    xc[a] = make_double2((s.x * dg.x + s.y * dg.y) / dn, (s.y * dg.x - s.x * dg.y) / dn);
  }
}

hipError_t launch_qr_lsq(double2* A, int64_t m, int K, double2* B, int R, double2* X, double2* rdiag, double* norms,
                         hipStream_t st) {
  if (K <= 0 || R <= 0 || m < K) return hipErrorInvalidValue;
  hipLaunchKernelGGL(colnorm2_kernel, dim3((unsigned)R), dim3(256), 0, st, B, (int64_t)0, m, norms);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int col = 0; col < K; ++col) {
    hipLaunchKernelGGL(hh_step_kernel, dim3((unsigned)(K - col - 1 + R)), dim3(256), 0, st, A, m, K, B, col, rdiag);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(colnorm2_kernel, dim3((unsigned)R), dim3(256), 0, st, B, (int64_t)K, m, norms + R);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(qr_backsolve_kernel, dim3((unsigned)((R + 63) / 64)), dim3(64), 0, st, A, m, K, B, R, rdiag, X);
  return hipGetLastError();
}

}  // namespace gdm
