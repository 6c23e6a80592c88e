// Small kernels around the hot path: cubic-cell polarisability, incident plane
// wave, q = A F, the FP64 cross-section reductions, the exact far-field
// scattering double sum, and the helpers of FP64 iterative refinement.
//
// Physics (arXiv:2505.09545):
//  * alpha_pE = chi_ee d^3 / (4 pi), chi_ee = eps - eps_env (Sec. "Volume
//    discretization polarizabilities");
//  * plane-wave illumination (Appendix, 3D illuminations): E0 = e0 exp(i k
//    khat.r), H0 = n_env khat x E0 (Gaussian units, mu = 1);
//  * dipole moments (p, m) = alpha (E, H) (Eq. after LPS_6by6_discrete);
//  * extinction / absorption / scattering cross sections (Sec. "Observables"):
//    the kernels return the raw FP64 sums, the prefactor C = 4 pi k0 /
//    (n_env |E0|^2) is applied on the host.
#include "gdm_common.hpp"
#include "gdm_kernels.hpp"
#include "gdm_misc.hpp"

namespace gdm {

__global__ void cell_alpha_kernel(const double2* eps, int64_t nc, double eps_env, double f, double2* alpha) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nc) alpha[i] = make_double2((eps[i].x - eps_env) * f, eps[i].y * f);
}

hipError_t launch_cell_alpha(const double2* eps, int64_t nc, double eps_env, double step, double2* alpha,
                             hipStream_t st) {
  if (nc <= 0) return hipSuccess;
  const double f = step * step * step / (4.0 * 3.14159265358979323846);
  hipLaunchKernelGGL(cell_alpha_kernel, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, eps, nc, eps_env, f,
                     alpha);
  return hipGetLastError();
}

__device__ inline double2 expi(double ph) {
  double s, c;
  sincos(ph, &s, &c);
  return make_double2(c, s);
}

__global__ void incident_kernel(DipoleView d, Wave w, double n_env, int64_t n_pw, const double* khat,
                                const double2* e0, double2* f0, int64_t n) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = blockIdx.y;
  if (u >= n || r >= n_pw) return;
  const int64_t N = d.N;
  const bool magnetic = u >= 3 * N;
  const int64_t dip = magnetic ? d.nc + (u - 3 * N) / 3 : u / 3;
  const int a = (int)(magnetic ? (u - 3 * N) % 3 : u % 3);
  const double kx = khat[3 * r], ky = khat[3 * r + 1], kz = khat[3 * r + 2];
  const double2 ph = expi(w.k * (kx * d.pos[3 * dip] + ky * d.pos[3 * dip + 1] + kz * d.pos[3 * dip + 2]));
  const double2* e = e0 + 3 * r;
  double2 v;
  if (!magnetic) {
    v = cmul(e[a], ph);
  } else {
    // (khat x e)_a
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    const double kb = b == 0 ? kx : (b == 1 ? ky : kz);
    const double kc = c == 0 ? kx : (c == 1 ? ky : kz);
    const double2 cr = csub(cscale(e[c], kb), cscale(e[b], kc));
    v = cscale(cmul(cr, ph), n_env);
  }
  f0[r * n + u] = v;
}

hipError_t launch_incident(const DipoleView& d, const Wave& w, double n_env, int64_t n_pw, const double* khat,
                           const double2* e0, double2* f0, int64_t n, hipStream_t st) {
  if (n_pw <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(incident_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)n_pw), dim3(256), 0, st, d, w, n_env,
                     n_pw, khat, e0, f0, n);
  return hipGetLastError();
}

// ACC: add the plane wave to E (and H) instead of writing it (total field at
// probes = incident + scattered).
template <bool ACC>
__global__ void planewave_points_kernel(Wave w, double n_env, int64_t n_pw, const double* khat, const double2* e0,
                                        const double* rp, int64_t P, double2* E, double2* H) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = blockIdx.y;
  if (p >= P) return;
  const double kx = khat[3 * r], ky = khat[3 * r + 1], kz = khat[3 * r + 2];
  const double2 ph = expi(w.k * (kx * rp[3 * p] + ky * rp[3 * p + 1] + kz * rp[3 * p + 2]));
  const double2* e = e0 + 3 * r;
  const double2 ex = cmul(e[0], ph), ey = cmul(e[1], ph), ez = cmul(e[2], ph);
  double2* oe = E + (r * P + p) * 3;
  oe[0] = ACC ? cadd(oe[0], ex) : ex;
  oe[1] = ACC ? cadd(oe[1], ey) : ey;
  oe[2] = ACC ? cadd(oe[2], ez) : ez;
  if (H) {
    double2* oh = H + (r * P + p) * 3;
    const double2 hx = cscale(csub(cscale(ez, ky), cscale(ey, kz)), n_env);
    const double2 hy = cscale(csub(cscale(ex, kz), cscale(ez, kx)), n_env);
    const double2 hz = cscale(csub(cscale(ey, kx), cscale(ex, ky)), n_env);
    oh[0] = ACC ? cadd(oh[0], hx) : hx;
    oh[1] = ACC ? cadd(oh[1], hy) : hy;
    oh[2] = ACC ? cadd(oh[2], hz) : hz;
  }
}

hipError_t launch_planewave_points(const Wave& w, double n_env, int64_t n_pw, const double* khat, const double2* e0,
                                   const double* r, int64_t P, double2* E, double2* H, hipStream_t st,
                                   bool accumulate) {
  if (n_pw <= 0 || P <= 0) return hipSuccess;
  const dim3 grid((unsigned)((P + 255) / 256), (unsigned)n_pw);
  if (accumulate)
    hipLaunchKernelGGL(planewave_points_kernel<true>, grid, dim3(256), 0, st, w, n_env, n_pw, khat, e0, r, P, E, H);
  else
    hipLaunchKernelGGL(planewave_points_kernel<false>, grid, dim3(256), 0, st, w, n_env, n_pw, khat, e0, r, P, E, H);
  return hipGetLastError();
}

// |E0|^2 = sum_a |e0[r][a]|^2 per plane wave
__global__ void pw_intensity_kernel(int64_t n_pw, const double2* __restrict__ e0, double* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_pw) return;
  double s = 0;
  for (int a = 0; a < 3; ++a) s += e0[3 * r + a].x * e0[3 * r + a].x + e0[3 * r + a].y * e0[3 * r + a].y;
  out[r] = s;
}

hipError_t launch_pw_intensity(int64_t n_pw, const double2* e0, double* out, hipStream_t st) {
  if (n_pw <= 0) return hipSuccess;
  hipLaunchKernelGGL(pw_intensity_kernel, dim3((unsigned)((n_pw + 255) / 256)), dim3(256), 0, st, n_pw, e0, out);
  return hipGetLastError();
}

// one thread per (dipole, rhs)
__global__ void apply_alpha_kernel(DipoleView d, const double2* F, int64_t ldf, double2* q, int64_t ldq,
                                   int64_t nrhs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = blockIdx.y;
  if (i >= d.N) return;
  const double2* f = F + r * ldf;
  double2* o = q + r * ldq;
  if (i < d.nc) {
    const double2 a = d.alpha_c[i];
    for (int c = 0; c < 3; ++c) o[3 * i + c] = cmul(a, f[3 * i + c]);
  } else {
    const int64_t e = i - d.nc;
    double2 v[6];
    for (int c = 0; c < 3; ++c) {
      v[c] = f[3 * i + c];
      v[3 + c] = f[3 * d.N + 3 * e + c];
    }
    const double2* a = d.alpha6 + e * 36;
    for (int rr = 0; rr < 6; ++rr) {
      double2 s = make_double2(0, 0);
      for (int c = 0; c < 6; ++c) cfma(s, a[rr * 6 + c], v[c]);
      if (rr < 3) o[3 * i + rr] = s;
      else o[3 * d.N + 3 * e + (rr - 3)] = s;
    }
  }
}

hipError_t launch_apply_alpha(const DipoleView& d, const double2* F, int64_t ldf, double2* q, int64_t ldq,
                              int64_t nrhs, hipStream_t st) {
  if (d.N <= 0 || nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(apply_alpha_kernel, dim3((unsigned)((d.N + 255) / 256), (unsigned)nrhs), dim3(256), 0, st, d, F,
                     ldf, q, ldq, nrhs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_gpm_apply(d, F, ldf, q, ldq, nrhs, st);  // members of GPM groups (overwrites their q)
}

// one workgroup (1024 threads) per RHS, FP64 tree reduction in LDS
__global__ void __launch_bounds__(1024) cs_sums_kernel(DipoleView d, const double2* f0, const double2* q,
                                                       const double2* f, int64_t n, double* out) {
  const int64_t r = blockIdx.x;
  const double2* a0 = f0 + r * n;
  const double2* aq = q + r * n;
  const double2* af = f + r * n;
  double s[5] = {0, 0, 0, 0, 0};
  const int64_t ncE = 3 * d.nc, NE = 3 * d.N;
  for (int64_t u = threadIdx.x; u < n; u += blockDim.x) {
    const double2 qq = aq[u];
    const double2 x0 = a0[u], xf = af[u];
    s[0] += x0.x * qq.y - x0.y * qq.x;  // Im(conj(F0) q)
    s[1] += xf.x * qq.y - xf.y * qq.x;  // Im(conj(F) q)
    const double q2 = qq.x * qq.x + qq.y * qq.y;
    if (u < ncE) s[2] += q2;
    else if (u < NE) s[3] += q2;
    else s[4] += q2;
  }
  __shared__ double red[5][1024];
  for (int k = 0; k < 5; ++k) red[k][threadIdx.x] = s[k];
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off)
      for (int k = 0; k < 5; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x < 5) out[r * 5 + threadIdx.x] = red[threadIdx.x][0];
}

hipError_t launch_cs_sums(const DipoleView& d, const double2* f0, const double2* q, const double2* f, int64_t n,
                          int64_t nrhs, double* sums5, hipStream_t st) {
  if (nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(cs_sums_kernel, dim3((unsigned)nrhs), dim3(1024), 0, st, d, f0, q, f, n, sums5);
  return hipGetLastError();
}

// Im sum_{i != j} q_i^H G6(r_i - r_j) q_j for one RHS per blockIdx.y
constexpr int FFT = 128;
__global__ void __launch_bounds__(256) sca_ff_kernel(DipoleView d, Wave w, const double2* q, int64_t ldq,
                                                     double* partial, int64_t nblk) {
  __shared__ double spos[FFT][3];
  __shared__ double2 sq[FFT][6];
  __shared__ double red[256];
  const int64_t r = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const double2* qc = q + r * ldq;
  const int64_t N = d.N, nc = d.nc;
  const bool live = i < N;
  double xi = 0, yi = 0, zi = 0;
  double2 qi[6];
  for (int c = 0; c < 6; ++c) qi[c] = make_double2(0, 0);
  if (live) {
    xi = d.pos[3 * i];
    yi = d.pos[3 * i + 1];
    zi = d.pos[3 * i + 2];
    for (int c = 0; c < 3; ++c) qi[c] = qc[3 * i + c];
    if (i >= nc)
      for (int c = 0; c < 3; ++c) qi[3 + c] = qc[3 * N + 3 * (i - nc) + c];
  }
  double acc = 0;
  for (int64_t t0 = 0; t0 < N; t0 += FFT) {
    const int nt = (int)(N - t0 < FFT ? N - t0 : FFT);
    __syncthreads();
    for (int t = threadIdx.x; t < nt; t += 256) {
      const int64_t j = t0 + t;
      for (int a = 0; a < 3; ++a) spos[t][a] = d.pos[3 * j + a];
      for (int c = 0; c < 3; ++c) sq[t][c] = qc[3 * j + c];
      for (int c = 0; c < 3; ++c) sq[t][3 + c] = j >= nc ? qc[3 * N + 3 * (j - nc) + c] : make_double2(0, 0);
    }
    __syncthreads();
    if (!live) continue;
    for (int t = 0; t < nt; ++t) {
      if (t0 + t == i) continue;
      Green g;
      green_eh(xi - spos[t][0], yi - spos[t][1], zi - spos[t][2], w, true, g);
      double2 s = make_double2(0, 0);
      for (int a = 0; a < 6; ++a) {
        double2 v = make_double2(0, 0);
        for (int b = 0; b < 6; ++b) cfma(v, g6(g, w.eps_env, a, b), sq[t][b]);
        cfma(s, cconj(qi[a]), v);
      }
      acc += s.y;
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[r * nblk + blockIdx.x] = red[0];
}

int64_t sca_ff_blocks(int64_t N) { return (N + 255) / 256; }

hipError_t launch_sca_ff(const DipoleView& d, const Wave& w, const double2* q, int64_t ldq, int64_t nrhs,
                         double* partial, int64_t nblk, hipStream_t st) {
  if (nrhs <= 0 || d.N <= 0) return hipSuccess;
  hipLaunchKernelGGL(sca_ff_kernel, dim3((unsigned)nblk, (unsigned)nrhs), dim3(256), 0, st, d, w, q, ldq, partial,
                     nblk);
  return hipGetLastError();
}

// ---- refinement helpers ------------------------------------------------------
__global__ void convert_d2f_kernel(const double2* a, int64_t lda, float2* b, int64_t ldb, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (i < m) {
    const double2 v = a[i + c * lda];
    b[i + c * ldb] = make_float2((float)v.x, (float)v.y);
  }
}
__global__ void convert_f2d_kernel(const float2* a, int64_t lda, double2* b, int64_t ldb, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (i < m) {
    const float2 v = a[i + c * lda];
    b[i + c * ldb] = make_double2(v.x, v.y);
  }
}
__global__ void copy_d_kernel(const double2* a, int64_t lda, double2* b, int64_t ldb, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (i < m) b[i + c * ldb] = a[i + c * lda];
}

// large 2D grids: columns in blockIdx.y up to 65535, so split very wide matrices
template <typename K, typename... Args>
static hipError_t launch_cols(K kernel, int64_t m, int64_t n, hipStream_t st, Args... args) {
  if (m <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(kernel, dim3((unsigned)((m + 255) / 256), (unsigned)n), dim3(256), 0, st, args..., m);
  return hipGetLastError();
}

hipError_t launch_convert_d2f(const double2* a, int64_t lda, float2* b, int64_t ldb, int64_t m, int64_t n,
                              hipStream_t st) {
  for (int64_t c0 = 0; c0 < n; c0 += 65535) {
    const int64_t nc = n - c0 < 65535 ? n - c0 : 65535;
    hipError_t e = launch_cols(convert_d2f_kernel, m, nc, st, a + c0 * lda, lda, b + c0 * ldb, ldb);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
hipError_t launch_convert_f2d(const float2* a, int64_t lda, double2* b, int64_t ldb, int64_t m, int64_t n,
                              hipStream_t st) {
  for (int64_t c0 = 0; c0 < n; c0 += 65535) {
    const int64_t nc = n - c0 < 65535 ? n - c0 : 65535;
    hipError_t e = launch_cols(convert_f2d_kernel, m, nc, st, a + c0 * lda, lda, b + c0 * ldb, ldb);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
hipError_t launch_copy_d(const double2* a, int64_t lda, double2* b, int64_t ldb, int64_t m, int64_t n,
                         hipStream_t st) {
  for (int64_t c0 = 0; c0 < n; c0 += 65535) {
    const int64_t nc = n - c0 < 65535 ? n - c0 : 65535;
    hipError_t e = launch_cols(copy_d_kernel, m, nc, st, a + c0 * lda, lda, b + c0 * ldb, ldb);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// one workgroup per column: x += c, cmax[col] = max |c|
__global__ void __launch_bounds__(256) axpy_f2d_kernel(const float2* c, int64_t ldc, double2* x, int64_t ldx,
                                                       int64_t m, double* cmax) {
  const int64_t col = blockIdx.x;
  double mx = 0;
  for (int64_t i = threadIdx.x; i < m; i += 256) {
    const float2 v = c[i + col * ldc];
    double2 xv = x[i + col * ldx];
    xv.x += (double)v.x;
    xv.y += (double)v.y;
    x[i + col * ldx] = xv;
    const double a = sqrt((double)v.x * v.x + (double)v.y * v.y);
    mx = a > mx ? a : mx;
  }
  __shared__ double red[256];
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) cmax[col] = red[0];
}

hipError_t launch_axpy_f2d(const float2* c, int64_t ldc, double2* x, int64_t ldx, int64_t m, int64_t n,
                           double* cmax, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(axpy_f2d_kernel, dim3((unsigned)n), dim3(256), 0, st, c, ldc, x, ldx, m, cmax);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) colmax_kernel(const double2* a, int64_t lda, int64_t m, double* out) {
  const int64_t col = blockIdx.x;
  double mx = 0;
  for (int64_t i = threadIdx.x; i < m; i += 256) {
    const double2 v = a[i + col * lda];
    const double t = sqrt(v.x * v.x + v.y * v.y);
    mx = t > mx ? t : mx;
  }
  __shared__ double red[256];
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[col] = red[0];
}

hipError_t launch_colmax(const double2* a, int64_t lda, int64_t m, int64_t n, double* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(colmax_kernel, dim3((unsigned)n), dim3(256), 0, st, a, lda, m, out);
  return hipGetLastError();
}

// cols[j] = sum_i |M_ij| (one workgroup per column, fixed-order reduction)
__global__ void __launch_bounds__(256) colsum_abs_kernel(const double2* M, int64_t ld, int64_t n, double* cols) {
  const int64_t col = blockIdx.x;
  double s = 0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double2 v = M[i + col * ld];
    s += sqrt(v.x * v.x + v.y * v.y);
  }
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) cols[col] = red[0];
}

hipError_t launch_colsum_abs(const double2* M, int64_t ld, int64_t n, double* cols, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(colsum_abs_kernel, dim3((unsigned)n), dim3(256), 0, st, M, ld, n, cols);
  return hipGetLastError();
}

// rows[i] = sum_j |M_ij|: grid (row blocks of 256) x (column chunks), one FP64 atomic per (row, chunk)
constexpr int RS_CHUNK = 512;
__global__ void __launch_bounds__(256) rowsum_abs_kernel(const double2* M, int64_t ld, int64_t n, double* rows) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.y * RS_CHUNK;
  const int64_t j1 = j0 + RS_CHUNK < n ? j0 + RS_CHUNK : n;
  if (i >= n) return;
  double s = 0;
  for (int64_t j = j0; j < j1; ++j) {
    const double2 v = M[i + j * ld];
    s += sqrt(v.x * v.x + v.y * v.y);
  }
  atomicAdd(&rows[i], s);
}
__global__ void zero_d_kernel(double* a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}

hipError_t launch_rowsum_abs(const double2* M, int64_t ld, int64_t n, double* rows, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_d_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, rows, n);
  hipLaunchKernelGGL(rowsum_abs_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)((n + RS_CHUNK - 1) / RS_CHUNK)),
                     dim3(256), 0, st, M, ld, n, rows);
  return hipGetLastError();
}

// ---- per-launch event timing -------------------------------------------------
hipError_t Prof::begin(hipStream_t st, int t, double w) {
  open = ((mask >> t) & 1u) != 0;
  if (!open) return hipSuccess;
  if (2 * used + 2 > ev.size()) {
    for (int i = 0; i < 2; ++i) {
      hipEvent_t e;
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      ev.push_back(e);
    }
    tag.push_back(0);
    work.push_back(0);
  }
  tag[used] = t;
  work[used] = w;
  return hipEventRecord(ev[2 * used], st);
}
hipError_t Prof::end(hipStream_t st) {
  if (!open) return hipSuccess;
  open = false;
  hipError_t r = hipEventRecord(ev[2 * used + 1], st);
  ++used;
  return r;
}
void Prof::collect() {
  for (size_t i = 0; i < used; ++i) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]) == hipSuccess) {
      ms[tag[i]] += t;
      wsum[tag[i]] += work[i];
      cnt[tag[i]] += 1;
    }
  }
  used = 0;
}
void Prof::reset() {
  used = 0;
  for (int i = 0; i < PROF_NTAGS; ++i) ms[i] = wsum[i] = cnt[i] = 0;
}
Prof::~Prof() {
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);
}


}  // namespace gdm
