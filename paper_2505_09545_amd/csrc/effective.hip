// Extraction of an effective electric-magnetic dipole pair from a discretised
// structure (arXiv:2505.09545, Sec. "Extraction of effective models": a set of
// illuminations is simulated, the electric and magnetic dipole moments of each
// response are taken -- for a single pair in 3D by the exact multipole
// decomposition -- and the effective polarisability is the least-squares
// solution alpha_eff = F0^+ P).
//
// Device steps after the solves and the multipoles (multipole.hip):
//   illum_at_point_kernel: row i of F0 [N][6] = (E0, H0) at r0 of illumination
//     i (plane waves first, then point-dipole sources, whose field at r0 is the
//     dyad G6(r0 - r_s) applied to their moments);
//   pair_lsq_kernel: one workgroup solves min ||F0 X - P||_F for X (6 x 6) by
//     Householder QR of F0 (FP64, complex), P [N][6] = (p, m) of each
//     response; alpha_eff = X^T and the relative residual ||F0 X - P|| / ||P||
//     (NaN entries when a diagonal entry of R is below 1e-12 of the largest).
#include <cmath>

#include "gdm_common.hpp"
#include "gdm_kernels.hpp"
#include "gdm_misc.hpp"

namespace gdm {

__global__ void illum_at_point_kernel(Wave w, double n_env, double r0x, double r0y, double r0z, int64_t n_pw,
                                      const double* __restrict__ khat, const double2* __restrict__ e0, int64_t n_src,
                                      const double* __restrict__ rs, const double2* __restrict__ ds,
                                      double2* __restrict__ F0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_pw + n_src) return;
  double2 o[6];
  illumination_at(w, n_env, r0x, r0y, r0z, i, n_pw, khat, e0, rs, ds, o);
  for (int a = 0; a < 6; ++a) F0[6 * i + a] = o[a];
}

// sum over the workgroup (256 threads) in a fixed order
__device__ inline double wg_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return ((red[0] + red[1]) + red[2]) + red[3];
}

// A [N][6] (overwritten), moments [N][24] (p, m in slots 0..5), B [N][6] work
// array; alpha [6][6] complex row-major and resid (device).
__global__ void __launch_bounds__(256) pair_lsq_kernel(double2* __restrict__ A, const double2* __restrict__ moments,
                                                       double2* __restrict__ B, int64_t N, double2* __restrict__ alpha,
                                                       double* __restrict__ resid) {
  __shared__ double red[4];
  __shared__ double2 vdot[12];
  __shared__ double2 R[6][6], Y[6][6];
  const int tid = threadIdx.x;
  double bn = 0.0;
  for (int64_t i = tid; i < N; i += 256)
    for (int c = 0; c < 6; ++c) {
      const double2 v = moments[24 * i + c];
      B[6 * i + c] = v;
      bn += v.x * v.x + v.y * v.y;
    }
  const double bnorm2 = wg_sum(bn, red);
  for (int col = 0; col < 6; ++col) {
    // Householder vector of A[col.., col]: v = x + e^{i arg x0} |x| e0, H = I - 2 v v^H / |v|^2
    double s2 = 0.0;
    for (int64_t i = col + tid; i < N; i += 256) {
      const double2 x = A[6 * i + col];
      s2 += x.x * x.x + x.y * x.y;
    }
    const double nx2 = wg_sum(s2, red);
    const double nx = sqrt(nx2);
    const double2 x0 = A[6 * col + col];
    const double ax0 = sqrt(x0.x * x0.x + x0.y * x0.y);
    const double2 ph = ax0 > 0 ? make_double2(x0.x / ax0, x0.y / ax0) : make_double2(1.0, 0.0);
    const double2 v0 = make_double2(x0.x + ph.x * nx, x0.y + ph.y * nx);
    // |v|^2 = |x|^2 - |x0|^2 + |v0|^2
    const double vn2 = nx2 - ax0 * ax0 + (v0.x * v0.x + v0.y * v0.y);
    __syncthreads();  // every read of x0 done before row col changes
    if (vn2 > 0) {
      // w_j = v^H A[:, j] for j > col and v^H B[:, j]
      for (int j = 0; j < 12; ++j) {
        if (j < 6 && j <= col) continue;
        double sr = 0.0, si = 0.0;
        for (int64_t i = col + tid; i < N; i += 256) {
          const double2 vi = i == col ? v0 : A[6 * i + col];
          const double2 a = j < 6 ? A[6 * i + j] : B[6 * i + (j - 6)];
          sr += vi.x * a.x + vi.y * a.y;  // conj(vi) a
          si += vi.x * a.y - vi.y * a.x;
        }
        const double tr = wg_sum(sr, red), ti = wg_sum(si, red);
        if (tid == 0) vdot[j] = make_double2(tr, ti);
      }
      __syncthreads();
      const double f = 2.0 / vn2;
      for (int64_t i = col + tid; i < N; i += 256) {
        const double2 vi = i == col ? v0 : A[6 * i + col];
        for (int j = 0; j < 12; ++j) {
          if (j < 6 && j <= col) continue;
          const double2 t = vdot[j];
          const double2 u = make_double2(f * (vi.x * t.x - vi.y * t.y), f * (vi.x * t.y + vi.y * t.x));
          double2* dst = j < 6 ? &A[6 * i + j] : &B[6 * i + (j - 6)];
          *dst = make_double2(dst->x - u.x, dst->y - u.y);
        }
      }
      __syncthreads();
      if (tid == 0) A[6 * col + col] = make_double2(-ph.x * nx, -ph.y * nx);  // R_cc
    }
    __syncthreads();
  }
  // residual: rows 6.. of the transformed B
  double rr = 0.0;
  for (int64_t i = 6 + tid; i < N; i += 256)
    for (int c = 0; c < 6; ++c) {
      const double2 v = B[6 * i + c];
      rr += v.x * v.x + v.y * v.y;
    }
  const double rn2 = wg_sum(rr, red);
  if (tid < 36) {
    const int a = tid / 6, b = tid % 6;
    R[a][b] = A[6 * a + b];
    Y[a][b] = B[6 * a + b];
  }
  __syncthreads();
  // rank check: a diagonal entry of R far below the largest one means the
  // illuminations leave alpha undetermined (NaN results, reported by the host)
  double dmax = 0.0, dmin = INFINITY;
  for (int a = 0; a < 6; ++a) {
    const double d = sqrt(R[a][a].x * R[a][a].x + R[a][a].y * R[a][a].y);
    dmax = d > dmax ? d : dmax;
    dmin = d < dmin ? d : dmin;
  }
  const bool rank_ok = dmin > 1e-12 * dmax;
  if (tid < 6) {
    // back substitution R X[:, c] = Y[:, c] for column c = tid
    const int c = tid;
    double2 x[6];
    for (int a = 5; a >= 0; --a) {
      double2 s = Y[a][c];
      for (int b = a + 1; b < 6; ++b) {
        const double2 r = R[a][b];
        s.x -= r.x * x[b].x - r.y * x[b].y;
        s.y -= r.x * x[b].y + r.y * x[b].x;
      }
      const double2 d = R[a][a];
      const double dn = d.x * d.x + d.y * d.y;
      x[a] = make_double2((s.x * d.x + s.y * d.y) / dn, (s.y * d.x - s.x * d.y) / dn);
    }
    // alpha = X^T: alpha[c][a] = X[a][c]
    for (int a = 0; a < 6; ++a) alpha[6 * c + a] = rank_ok ? x[a] : make_double2(NAN, NAN);
  }
  if (tid == 0) *resid = bnorm2 > 0 ? sqrt(rn2 / bnorm2) : 0.0;
}

hipError_t launch_pair_extract(const Wave& w, double n_env, const double r0[3], int64_t n_pw, const double* khat,
                               const double2* e0, int64_t n_src, const double* rs, const double2* ds,
                               const double2* moments, double2* F0, double2* B, double2* alpha, double* resid,
                               hipStream_t st) {
  const int64_t N = n_pw + n_src;
  if (N < 6) return hipErrorInvalidValue;
  hipLaunchKernelGGL(illum_at_point_kernel, dim3((unsigned)((N + 127) / 128)), dim3(128), 0, st, w, n_env, r0[0], r0[1],
                     r0[2], n_pw, khat, e0, n_src, rs, ds, F0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pair_lsq_kernel, dim3(1), dim3(256), 0, st, F0, moments, B, N, alpha, resid);
  return hipGetLastError();
}

}  // namespace gdm
