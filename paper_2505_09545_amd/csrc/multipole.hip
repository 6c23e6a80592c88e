// Exact multipole decomposition of the mesh cells' polarisation up to
// quadrupole order, and the scattering and extinction cross sections of each
// multipole (arXiv:2505.09545, Sec. "Observables": exact multipole
// decomposition of the polarisation inside a discretised structure and of the
// scattering and extinction cross sections; Sec. "Implementation technical
// details", which names the exact-moment and extinction formulations by
// reference).
//
// For cells with electric dipoles p_j at r_j, R = r_j - r0, x = k |R|, summed
// over cells (Gaussian units, exp(-i w t), the far-field convention of the
// library's fields):
//   p  = p_j j0 + (k^2/2) [3 (R.p_j) R - R^2 p_j] j2/x^2
//   m  = -i k0 (3/2) (R x p_j) j1/x
//   Qe = 3 { [3 (R p_j^T + p_j R^T) - 2 (R.p_j) I] j1/x
//            + 2 k^2 [5 (R.p_j) R R^T - R^2 (R p_j^T + p_j R^T) - R^2 (R.p_j) I] j3/x^3 }
//   Qm = -i k0 15 [R (R x p_j)^T + (R x p_j) R^T] j2/x^2
// Cross sections (over |E0|^2):
//   scattering  ED (8 pi/3) k^4/eps^2 |p|^2, MD (8 pi/3) k0^2 k^2 |m|^2,
//               EQ (pi/45) k^6/eps^2 |Qe|^2, MQ (pi/45) k0^2 k^4 |Qm|^2;
//   extinction  C Im(E0*(r0).p), C Im(H0*(r0).m), (C/6) Im(dE0*(r0) : Qe),
//               (C/6) Im(dH0*(r0) : Qm), C = 4 pi k0 / (n_env |E0|^2),
//               with d_a E0*_b = -i k khat_a E0*_b for a plane wave.
//
// Layout: stage 1, workgroup (split s, RHS r) sums a contiguous range of cells
// into 36 doubles (18 complex: p, m, Qe and Qm by their 6 distinct entries of
// the symmetric tensors, before the constant factors); a fixed-order reduction
// (wave shuffles, then the four waves in order) makes the result independent
// of timing.  Stage 2, one workgroup per RHS, adds the splits in order and
// forms the moments and the cross sections.  HBM-bound on the moments q
// (16 B per unknown read once per RHS) plus the positions; the Bessel weights
// are FP64 VALU work per cell.
#include <cmath>

#include "gdm_common.hpp"
#include "gdm_kernels.hpp"
#include "gdm_misc.hpp"

namespace gdm {

// j0(x) and j_n(x) / x^n for n = 1, 2, 3.  Below x = 2 the power series
// j_n(x)/x^n = sum_s (-x^2/2)^s / (s! (2n + 2s + 1)!!) (its terms fall faster
// than 2^s / (s! (2s)!), 16 terms leave < 1e-17); from x = 2 on the
// trigonometric closed forms, whose cancellation is at most a factor ~20 there.
__device__ inline void sph_bessel_w(double x, double& j0, double& w1, double& w2, double& w3) {
  if (x < 2.0) {
    const double h = -0.5 * x * x;
    double out[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      double df = 1.0;
      for (int i = 3; i <= 2 * n + 1; i += 2) df *= i;
      double t = 1.0 / df, s = t;
#pragma unroll
      for (int k = 1; k <= 16; ++k) {
        t *= h / (double)(k * (2 * n + 2 * k + 1));
        s += t;
      }
      out[n] = s;
    }
    j0 = out[0];
    w1 = out[1];
    w2 = out[2];
    w3 = out[3];
    return;
  }
  double sn, cs;
  sincos(x, &sn, &cs);
  const double ix = 1.0 / x, ix2 = ix * ix;
  const double j1 = (sn * ix - cs) * ix;
  const double j2 = (3.0 * ix2 - 1.0) * sn * ix - 3.0 * cs * ix2;
  const double j3 = (15.0 * ix2 * ix - 6.0 * ix) * sn * ix - (15.0 * ix2 - 1.0) * cs * ix;
  j0 = sn * ix;
  w1 = j1 * ix;
  w2 = j2 * ix2;
  w3 = j3 * ix2 * ix;
}

constexpr int MP_ACC = 36;   // doubles per partial: 18 complex
constexpr int MP_GRAIN = 512;  // cells per split at least

// symmetric-tensor slot order: xx, yy, zz, xy, xz, yz
__device__ inline int sym_slot(int a, int b) {
  if (a == b) return a;
  const int s = a + b;  // 1: xy, 2: xz, 3: yz
  return 2 + s;
}

__global__ void __launch_bounds__(256) multipole_partial_kernel(const double* __restrict__ pos, int64_t nc,
                                                                 const double2* __restrict__ q, int64_t n, double r0x,
                                                                 double r0y, double r0z, double k, int nsplit,
                                                                 double* __restrict__ part) {
  const int s = blockIdx.x, r = blockIdx.y, tid = threadIdx.x;
  const int64_t per = (nc + nsplit - 1) / nsplit;
  const int64_t j0c = (int64_t)s * per, j1c = j0c + per < nc ? j0c + per : nc;
  const double2* qr = q + (int64_t)r * n;
  double acc[MP_ACC];
#pragma unroll
  for (int i = 0; i < MP_ACC; ++i) acc[i] = 0.0;
  for (int64_t j = j0c + tid; j < j1c; j += 256) {
    const double R[3] = {pos[3 * j] - r0x, pos[3 * j + 1] - r0y, pos[3 * j + 2] - r0z};
    const double2 p[3] = {qr[3 * j], qr[3 * j + 1], qr[3 * j + 2]};
    const double R2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
    double b0, w1, w2, w3;
    sph_bessel_w(k * sqrt(R2), b0, w1, w2, w3);
    double2 Rp;  // R.p
    Rp.x = R[0] * p[0].x + R[1] * p[1].x + R[2] * p[2].x;
    Rp.y = R[0] * p[0].y + R[1] * p[1].y + R[2] * p[2].y;
    double2 rxp[3];  // R x p
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int b = (a + 1) % 3, c = (a + 2) % 3;
      rxp[a].x = R[b] * p[c].x - R[c] * p[b].x;
      rxp[a].y = R[b] * p[c].y - R[c] * p[b].y;
    }
    const double hk2 = 0.5 * k * k;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      // p: j0 p + (k^2/2) w2 (3 (R.p) R - R^2 p)
      acc[2 * a] += b0 * p[a].x + hk2 * w2 * (3.0 * Rp.x * R[a] - R2 * p[a].x);
      acc[2 * a + 1] += b0 * p[a].y + hk2 * w2 * (3.0 * Rp.y * R[a] - R2 * p[a].y);
      // m (before -i k0 3/2): w1 (R x p)
      acc[6 + 2 * a] += w1 * rxp[a].x;
      acc[6 + 2 * a + 1] += w1 * rxp[a].y;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = a; b < 3; ++b) {
        const int sl = sym_slot(a, b);
        const double d = a == b ? 1.0 : 0.0;
        // Qe (before the factor 3)
        const double sx = R[a] * p[b].x + p[a].x * R[b], sy = R[a] * p[b].y + p[a].y * R[b];
        const double e1x = 3.0 * sx - 2.0 * Rp.x * d, e1y = 3.0 * sy - 2.0 * Rp.y * d;
        const double e3x = 5.0 * Rp.x * R[a] * R[b] - R2 * sx - R2 * Rp.x * d;
        const double e3y = 5.0 * Rp.y * R[a] * R[b] - R2 * sy - R2 * Rp.y * d;
        acc[12 + 2 * sl] += w1 * e1x + 2.0 * k * k * w3 * e3x;
        acc[12 + 2 * sl + 1] += w1 * e1y + 2.0 * k * k * w3 * e3y;
        // Qm (before -i k0 15): w2 (R (R x p)^T + (R x p) R^T)
        acc[24 + 2 * sl] += w2 * (R[a] * rxp[b].x + rxp[a].x * R[b]);
        acc[24 + 2 * sl + 1] += w2 * (R[a] * rxp[b].y + rxp[a].y * R[b]);
      }
  }
  // fixed-order reduction: butterfly within each wave, then waves 0..3 in order
  __shared__ double red[4][MP_ACC];
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int i = 0; i < MP_ACC; ++i) {
    double v = acc[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) red[wave][i] = v;
  }
  __syncthreads();
  if (tid < MP_ACC) {
    const double v = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
    part[((int64_t)r * nsplit + s) * MP_ACC + tid] = v;
  }
}

// Stage 2: one workgroup per RHS.
__global__ void __launch_bounds__(64) multipole_final_kernel(const double* __restrict__ part, int nsplit, double k,
                                                              double k0, double n_env, double r0x, double r0y,
                                                              double r0z, const double* __restrict__ khat,
                                                              const double2* __restrict__ e0,
                                                              double2* __restrict__ moments,
                                                              double* __restrict__ sigma) {
  const int r = blockIdx.x, tid = threadIdx.x;
  __shared__ double sums[MP_ACC];
  if (tid < MP_ACC) {
    double v = 0.0;
    for (int s = 0; s < nsplit; ++s) v += part[((int64_t)r * nsplit + s) * MP_ACC + tid];
    sums[tid] = v;
  }
  __syncthreads();
  if (tid != 0) return;
  auto cz = [&](int i) { return make_double2(sums[2 * i], sums[2 * i + 1]); };
  double2 p[3], m[3], Qe[3][3], Qm[3][3];
  for (int a = 0; a < 3; ++a) {
    p[a] = cz(a);
    const double2 u = cz(3 + a);  // m = -i k0 (3/2) u
    m[a] = make_double2(1.5 * k0 * u.y, -1.5 * k0 * u.x);
  }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      const int sl = sym_slot(a, b);
      const double2 e = cz(6 + sl), h = cz(12 + sl);
      Qe[a][b] = make_double2(3.0 * e.x, 3.0 * e.y);
      Qm[a][b] = make_double2(15.0 * k0 * h.y, -15.0 * k0 * h.x);  // -i k0 15 h
    }
  if (moments) {
    double2* o = moments + (int64_t)r * 24;
    for (int a = 0; a < 3; ++a) {
      o[a] = p[a];
      o[3 + a] = m[a];
      for (int b = 0; b < 3; ++b) {
        o[6 + 3 * a + b] = Qe[a][b];
        o[15 + 3 * a + b] = Qm[a][b];
      }
    }
  }
  if (!sigma) return;
  double e2 = 1.0;
  double2 es[3] = {}, hs[3] = {};
  double kh[3] = {0.0, 0.0, 0.0};
  if (khat) {
    for (int a = 0; a < 3; ++a) kh[a] = khat[3 * r + a];
    // E0(r0) = e0 exp(i k khat.r0), H0 = n_env khat x E0; conjugated
    const double ph = k * (kh[0] * r0x + kh[1] * r0y + kh[2] * r0z);
    double sn, cs;
    sincos(ph, &sn, &cs);
    double2 E[3];
    e2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double2 v = e0[3 * r + a];
      e2 += v.x * v.x + v.y * v.y;
      E[a] = make_double2(v.x * cs - v.y * sn, v.x * sn + v.y * cs);
    }
    for (int a = 0; a < 3; ++a) {
      const int b = (a + 1) % 3, c = (a + 2) % 3;
      const double2 H = make_double2(n_env * (kh[b] * E[c].x - kh[c] * E[b].x), n_env * (kh[b] * E[c].y - kh[c] * E[b].y));
      es[a] = make_double2(E[a].x, -E[a].y);
      hs[a] = make_double2(H.x, -H.y);
    }
  }
  const double eps = n_env * n_env, k2 = k * k, k02 = k0 * k0;
  double pp = 0, mm = 0, qe = 0, qm = 0;
  for (int a = 0; a < 3; ++a) {
    pp += p[a].x * p[a].x + p[a].y * p[a].y;
    mm += m[a].x * m[a].x + m[a].y * m[a].y;
    for (int b = 0; b < 3; ++b) {
      qe += Qe[a][b].x * Qe[a][b].x + Qe[a][b].y * Qe[a][b].y;
      qm += Qm[a][b].x * Qm[a][b].x + Qm[a][b].y * Qm[a][b].y;
    }
  }
  const double pi = 3.14159265358979323846;
  double* so = sigma + (int64_t)r * 8;
  so[0] = (8.0 * pi / 3.0) * k2 * k2 / (eps * eps) * pp / e2;
  so[1] = (8.0 * pi / 3.0) * k02 * k2 * mm / e2;
  so[2] = (pi / 45.0) * k2 * k2 * k2 / (eps * eps) * qe / e2;
  so[3] = (pi / 45.0) * k02 * k2 * k2 * qm / e2;
  if (!khat) {
    for (int i = 4; i < 8; ++i) so[i] = __builtin_nan("");
    return;
  }
  const double C = 4.0 * pi * k0 / (n_env * e2);
  // Im(a b) for complex a, b
  auto imab = [](double2 a, double2 b) { return a.x * b.y + a.y * b.x; };
  double ed = 0, md = 0, eq = 0, mq = 0;
  for (int a = 0; a < 3; ++a) {
    ed += imab(es[a], p[a]);
    md += imab(hs[a], m[a]);
    for (int b = 0; b < 3; ++b) {
      // d_a E0*_b = -i k khat_a E0*_b
      const double2 gE = make_double2(k * kh[a] * es[b].y, -k * kh[a] * es[b].x);
      const double2 gH = make_double2(k * kh[a] * hs[b].y, -k * kh[a] * hs[b].x);
      eq += imab(gE, Qe[a][b]);
      mq += imab(gH, Qm[a][b]);
    }
  }
  so[4] = C * ed;
  so[5] = C * md;
  so[6] = C / 6.0 * eq;
  so[7] = C / 6.0 * mq;
}

int multipole_num_splits(int64_t nc, int num_cu, int64_t nrhs) {
  int64_t s = (nc + MP_GRAIN - 1) / MP_GRAIN;
  const int64_t want = (2 * (int64_t)num_cu + nrhs - 1) / (nrhs > 0 ? nrhs : 1);
  if (s > want) s = want;
  if (s < 1) s = 1;
  return (int)s;
}

size_t multipole_scratch_bytes(int64_t nrhs, int nsplit) { return (size_t)nrhs * nsplit * MP_ACC * sizeof(double); }

hipError_t launch_multipoles(const double* pos, int64_t nc, const double2* q, int64_t n, int64_t nrhs,
                             const double r0[3], double k, double k0, double n_env, const double* khat,
                             const double2* e0, int nsplit, double* part, double2* moments, double* sigma,
                             hipStream_t st) {
  if (nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(multipole_partial_kernel, dim3((unsigned)nsplit, (unsigned)nrhs), dim3(256), 0, st, pos, nc, q, n,
                     r0[0], r0[1], r0[2], k, nsplit, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(multipole_final_kernel, dim3((unsigned)nrhs), dim3(64), 0, st, part, nsplit, k, k0, n_env, r0[0],
                     r0[1], r0[2], khat, e0, moments, sigma);
  return hipGetLastError();
}

}  // namespace gdm
