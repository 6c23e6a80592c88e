// Local dipole sources and the Green's tensor / LDOS of the structured
// environment (arXiv:2505.09545, Sec. "Observables": electric and magnetic LDOS
// and Green's tensors in a nano-structured environment; Appendix, illumination
// classes: electric and magnetic point-dipole sources; Sec. "The tg.Simulation
// class": the Green's tensor and LDOS getters).
//
// A point source d = (p, m) at r_s illuminates the dipoles with its own field,
// F0_i = G(r_i, r_s) d (the 6x6 dyad of Eq. superprop_G).  Solving M F = F0
// with the factors and re-propagating the moments q = A F gives the field the
// structure scatters; for the six unit source components (p_x, p_y, p_z, m_x,
// m_y, m_z) these fields at a point r are the columns of the scattered part of
// the structured environment's 6x6 Green's tensor G_sca(r, r_s).
//
// LDOS: a unit dipole emits (omega / 2) Im(d^* . F(r_s)), where F is its total
// field at itself; in the homogeneous host the radiation-reaction parts are
// Im G^Ep(0) = (2/3) k^3 / eps_env I and Im G^Hm(0) = (2/3) k^3 I, so the
// partial LDOS relative to the host, along axis a, is
//   rho_e,a / rho_0 = 1 + (3/2) (eps_env / k^3) Im G_sca^Ep_aa(r_s, r_s),
//   rho_m,a / rho_0 = 1 + (3/2) (1 / k^3)       Im G_sca^Hm_aa(r_s, r_s).
#include "gdm_common.hpp"
#include "gdm_kernels.hpp"
#include "gdm_misc.hpp"

namespace gdm {

// F0[s][u] of the sources d[s] = (p, m) [n_src][6] at r_src [n_src][3]: one
// thread per dipole i, grid.y = source.  A source closer than sqrt(min_r2) to a
// dipole sets *flag (its field there is left zero).
__global__ void dipole_source_kernel(DipoleView d, Wave w, int64_t n, const double* __restrict__ rs,
                                     const double2* __restrict__ ds, double2* __restrict__ f0, double min_r2,
                                     int* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t s = blockIdx.y;
  if (i >= d.N) return;
  const double Rx = d.pos[3 * i] - rs[3 * s], Ry = d.pos[3 * i + 1] - rs[3 * s + 1], Rz = d.pos[3 * i + 2] - rs[3 * s + 2];
  double2 E[3] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
  double2 H[3] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
  if (Rx * Rx + Ry * Ry + Rz * Rz < min_r2) {
    atomicOr(flag, 1);
  } else {
    Green g;
    green_eh(Rx, Ry, Rz, w, true, g);
    const double2* src = ds + 6 * s;
    const double2 px = src[0], py = src[1], pz = src[2], mx = src[3], my = src[4], mz = src[5];
    // E = G^Ep p + G^Em m, G^Em m = -(h x m)
    cfma(E[0], g.e[0], px); cfma(E[0], g.e[3], py); cfma(E[0], g.e[4], pz);
    cfma(E[1], g.e[3], px); cfma(E[1], g.e[1], py); cfma(E[1], g.e[5], pz);
    cfma(E[2], g.e[4], px); cfma(E[2], g.e[5], py); cfma(E[2], g.e[2], pz);
    cfma(E[0], cscale(g.h[1], -1.0), mz); cfma(E[0], g.h[2], my);
    cfma(E[1], cscale(g.h[2], -1.0), mx); cfma(E[1], g.h[0], mz);
    cfma(E[2], cscale(g.h[0], -1.0), my); cfma(E[2], g.h[1], mx);
    // H = G^Hp p + G^Hm m = h x p + eps G^Ep m
    cfma(H[0], g.h[1], pz); cfma(H[0], cscale(g.h[2], -1.0), py);
    cfma(H[1], g.h[2], px); cfma(H[1], cscale(g.h[0], -1.0), pz);
    cfma(H[2], g.h[0], py); cfma(H[2], cscale(g.h[1], -1.0), px);
    double2 u0 = make_double2(0, 0), u1 = make_double2(0, 0), u2 = make_double2(0, 0);
    cfma(u0, g.e[0], mx); cfma(u0, g.e[3], my); cfma(u0, g.e[4], mz);
    cfma(u1, g.e[3], mx); cfma(u1, g.e[1], my); cfma(u1, g.e[5], mz);
    cfma(u2, g.e[4], mx); cfma(u2, g.e[5], my); cfma(u2, g.e[2], mz);
    H[0] = cadd(H[0], cscale(u0, w.eps_env));
    H[1] = cadd(H[1], cscale(u1, w.eps_env));
    H[2] = cadd(H[2], cscale(u2, w.eps_env));
  }
  double2* o = f0 + s * n;
#pragma unroll
  for (int a = 0; a < 3; ++a) o[3 * i + a] = E[a];
  if (i >= d.nc)
#pragma unroll
    for (int a = 0; a < 3; ++a) o[3 * d.N + 3 * (i - d.nc) + a] = H[a];
}

hipError_t launch_dipole_sources(const DipoleView& d, const Wave& w, int64_t n, int64_t n_src, const double* rs,
                                 const double2* ds, double2* f0, double min_r2, int* flag, hipStream_t st) {
  if (n_src <= 0 || d.N <= 0) return hipSuccess;
  hipLaunchKernelGGL(dipole_source_kernel, dim3((unsigned)((d.N + 255) / 256), (unsigned)n_src), dim3(256), 0, st, d,
                     w, n, rs, ds, f0, min_r2, flag);
  return hipGetLastError();
}

// LDOS from the moments q [6 n_src][n] of the unit sources (RHS 6 s + c):
// component c of the scattered field at r_s, sum_j G(r_s - r_j) q_j, reduced in
// a fixed order by one workgroup per RHS, then out[s][c / 3][c % 3] =
// 1 + (3/2) w_c Im(.) with w = eps_env / k^3 (electric) or 1 / k^3 (magnetic).
__global__ void __launch_bounds__(256) ldos_kernel(DipoleView d, Wave w, const double2* __restrict__ q, int64_t n,
                                                    const double* __restrict__ rs, double* __restrict__ out) {
  __shared__ double red[256];
  const int64_t rr = blockIdx.x;
  const int64_t s = rr / 6;
  const int c = (int)(rr % 6), a = c % 3;
  const bool mag = c >= 3;
  const double2* qr = q + rr * n;
  const double x = rs[3 * s], y = rs[3 * s + 1], z = rs[3 * s + 2];
  double acc = 0;
  for (int64_t j = threadIdx.x; j < d.N; j += 256) {
    Green g;
    green_eh(x - d.pos[3 * j], y - d.pos[3 * j + 1], z - d.pos[3 * j + 2], w, true, g);
    const double2 p[3] = {qr[3 * j], qr[3 * j + 1], qr[3 * j + 2]};
    double2 m[3] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
    if (j >= d.nc)
      for (int b = 0; b < 3; ++b) m[b] = qr[3 * d.N + 3 * (j - d.nc) + b];
    double2 f = make_double2(0, 0);
    if (!mag) {
      // E_a = (G^Ep p)_a - (h x m)_a
      for (int b = 0; b < 3; ++b) cfma(f, gep(g, a, b), p[b]);
      for (int b = 0; b < 3; ++b) cfma(f, cscale(ghp(g, a, b), -1.0), m[b]);
    } else {
      // H_a = (h x p)_a + eps (G^Ep m)_a
      for (int b = 0; b < 3; ++b) cfma(f, ghp(g, a, b), p[b]);
      for (int b = 0; b < 3; ++b) cfma(f, cscale(gep(g, a, b), w.eps_env), m[b]);
    }
    acc += f.y;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double k3 = w.k * w.k * w.k;
    out[rr] = 1.0 + 1.5 * (mag ? 1.0 : w.eps_env) / k3 * red[0];
  }
}

hipError_t launch_ldos(const DipoleView& d, const Wave& w, const double2* q, int64_t n, int64_t n_src,
                       const double* rs, double* out, hipStream_t st) {
  if (n_src <= 0) return hipSuccess;
  hipLaunchKernelGGL(ldos_kernel, dim3((unsigned)(6 * n_src)), dim3(256), 0, st, d, w, q, n, rs, out);
  return hipGetLastError();
}

// G[s][p][row][c] = (row < 3 ? E : H)[6 s + c][p][row % 3] for the fields of the
// unit sources at the points.
__global__ void green_gather_kernel(const double2* __restrict__ E, const double2* __restrict__ H, int64_t n_src,
                                    int64_t P, double2* __restrict__ G) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_src * P * 36) return;
  const int c = (int)(idx % 6), row = (int)((idx / 6) % 6);
  const int64_t p = (idx / 36) % P, s = idx / (36 * P);
  const double2* F = row < 3 ? E : H;
  G[idx] = F[((6 * s + c) * P + p) * 3 + row % 3];
}

hipError_t launch_green_gather(const double2* E, const double2* H, int64_t n_src, int64_t P, double2* G,
                               hipStream_t st) {
  const int64_t count = n_src * P * 36;
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(green_gather_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, E, H, n_src, P, G);
  return hipGetLastError();
}

}  // namespace gdm
