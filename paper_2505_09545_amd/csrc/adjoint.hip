// Hand-written adjoint of the GDM hot path: gradient of a real loss built from
// the cross sections and the total electric field at probe points, with respect
// to every dipole position, the permittivity of every cell and the wavelength.
//
// The paper differentiates its solver with PyTorch's automatic differentiation
// (Sec. "Example: Autograd for resonance search"); here the reverse pass is
// written out.  With M F = F0 (Eq. GDM_system_of_equations, M = I - G~ A),
// q = A F, and Wirtinger partials g_x = dL/dx of the real loss (dL = 2 Re sum
// g_x dx), the adjoint field lam solves
//     M^T lam = g_F + A^T g_qe,     g_qe = g_q + sum_p g_E(p) G_pj     (probes),
// and the total variation is
//     dL = 2 Re[ (lam + g_F0) . dF0 + lam . dG~ q + (G~^T lam + g_qe) . dA F
//                + g_E . (dE_inc + dG_p q) ] + explicit dependence of the
//          cross sections on k0 (the prefactor 4 pi k0 / n_env and the
//          radiation term (2/3) k^3 of effective dipoles).
//
// The dyad of a separation R (Eq. superprop_G) is written with three radial
// functions, G^Ep = phi(R) I + psi(R) R R^T and G^Hp = chi(R) [R]_x, so that for
// complex 3-vectors a, b (unconjugated products)
//     a^T G^Ep b = phi (a.b) + psi (a.R)(R.b),     a^T G^Hp b = chi R.(b x a),
//     d/dR_x [a^T G^Ep b] = (R_x/R)[phi' (a.b) + psi' (a.R)(R.b)] + psi [a_x (R.b) + b_x (a.R)],
//     d/dR_x [a^T G^Hp b] = (R_x/R) chi' R.(b x a) + chi (b x a)_x,
// and d/dk0 acts on phi, psi, chi only.  Every (pair, RHS) term is evaluated in
// registers with one sincos; nothing of size N^2 is stored.  All sums that
// cross threads are written as per-workgroup partials and reduced in a fixed
// order (deterministic results).
#include "gdm_adjoint.hpp"

namespace gdm {

namespace {

struct GreenRad {
  double2 phi, psi, chi;     // dyad radial functions
  double2 dphi, dpsi, dchi;  // d/dR
  double2 kphi, kpsi, kchi;  // d/dk0 at fixed R and n_env
  double iR;
};

__device__ inline void green_rad(double R2, const Wave& w, double n_env, GreenRad& g) {
  const double R = sqrt(R2);
  const double iR = 1.0 / R;
  double s, c;
  sincos(w.k * R, &s, &c);
  const double k = w.k, k2 = k * k, ie = 1.0 / w.eps_env;
  const double iR2 = iR * iR, iR3 = iR2 * iR, iR4 = iR2 * iR2, iR5 = iR4 * iR, iR6 = iR3 * iR3;
  const double2 e = make_double2(c * ie, s * ie);  // e^{ikR} / eps_env
  const double2 e1 = make_double2(c, s);           // e^{ikR}
  // phi = e (k^2/R + ik/R^2 - 1/R^3),  psi = e (-k^2/R^3 - 3ik/R^4 + 3/R^5),  chi = k0 e1 (k/R^2 + i/R^3)
  g.phi = cmul(e, make_double2(k2 * iR - iR3, k * iR2));
  g.psi = cmul(e, make_double2(-k2 * iR3 + 3.0 * iR5, -3.0 * k * iR4));
  g.chi = cmul(e1, make_double2(w.k0 * k * iR2, w.k0 * iR3));
  // radial derivatives
  g.dphi = cmul(e, make_double2(-2.0 * k2 * iR2 + 3.0 * iR4, k2 * k * iR - 3.0 * k * iR3));
  g.dpsi = cmul(e, make_double2(6.0 * k2 * iR4 - 15.0 * iR6, -k2 * k * iR3 + 15.0 * k * iR5));
  g.dchi = cmul(e1, make_double2(-3.0 * w.k0 * k * iR3, w.k0 * (k2 * iR2 - 3.0 * iR4)));
  // derivatives w.r.t. k0 (k = n_env k0)
  g.kphi = cscale(cmul(e, make_double2(k * iR, k2)), n_env);
  g.kpsi = cscale(cmul(e, make_double2(k * iR3, -k2 * iR2)), n_env);
  g.kchi = cmul(e1, make_double2(k * iR2, iR3 + k2 * iR));
  g.iR = iR;
}

__device__ inline double2 dot3(const double2 a[3], const double2 b[3]) {
  double2 s = cmul(a[0], b[0]);
  cfma(s, a[1], b[1]);
  cfma(s, a[2], b[2]);
  return s;
}
__device__ inline double2 rdot(const double R[3], const double2 a[3]) {
  return make_double2(R[0] * a[0].x + R[1] * a[1].x + R[2] * a[2].x, R[0] * a[0].y + R[1] * a[1].y + R[2] * a[2].y);
}
__device__ inline void cross3(const double2 a[3], const double2 b[3], double2 o[3]) {
  o[0] = csub(cmul(a[1], b[2]), cmul(a[2], b[1]));
  o[1] = csub(cmul(a[2], b[0]), cmul(a[0], b[2]));
  o[2] = csub(cmul(a[0], b[1]), cmul(a[1], b[0]));
}

// gx += s * d/dR [a^T G^Ep b],  dk += s * d/dk0 [a^T G^Ep b]   (s real)
__device__ inline void acc_ep(const GreenRad& g, const double R[3], const double2 a[3], const double2 b[3], double s,
                              double2 gx[3], double2& dk, bool want_dk) {
  const double2 ab = dot3(a, b), aR = rdot(R, a), Rb = rdot(R, b);
  const double2 aRRb = cmul(aR, Rb);
  double2 rad = cmul(g.dphi, ab);
  cfma(rad, g.dpsi, aRRb);
  rad = cscale(rad, s * g.iR);
  const double2 pRb = cscale(cmul(g.psi, Rb), s), paR = cscale(cmul(g.psi, aR), s);
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    gx[x] = cadd(gx[x], cscale(rad, R[x]));
    cfma(gx[x], pRb, a[x]);
    cfma(gx[x], paR, b[x]);
  }
  if (want_dk) {
    double2 t = cmul(g.kphi, ab);
    cfma(t, g.kpsi, aRRb);
    dk = cadd(dk, cscale(t, s));
  }
}

// gx += s * d/dR [a^T G^Hp b],  dk += s * d/dk0 [a^T G^Hp b]
__device__ inline void acc_hp(const GreenRad& g, const double R[3], const double2 a[3], const double2 b[3], double s,
                              double2 gx[3], double2& dk, bool want_dk) {
  double2 bxa[3];
  cross3(b, a, bxa);
  const double2 Rba = rdot(R, bxa);
  const double2 rad = cscale(cmul(g.dchi, Rba), s * g.iR);
  const double2 cs = cscale(g.chi, s);
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    gx[x] = cadd(gx[x], cscale(rad, R[x]));
    cfma(gx[x], cs, bxa[x]);
  }
  if (want_dk) dk = cadd(dk, cscale(cmul(g.kchi, Rba), s));
}

// o += G^Ep v = phi v + psi R (R.v)
__device__ inline void add_gep(const GreenRad& g, const double R[3], const double2 v[3], double2 o[3]) {
  const double2 t = cmul(g.psi, rdot(R, v));
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    cfma(o[x], g.phi, v[x]);
    o[x] = cadd(o[x], cscale(t, R[x]));
  }
}
// o += G^Hp v = chi (R x v)
__device__ inline void add_ghp(const GreenRad& g, const double R[3], const double2 v[3], double2 o[3]) {
  const double2 rv0 = make_double2(R[1] * v[2].x - R[2] * v[1].x, R[1] * v[2].y - R[2] * v[1].y);
  const double2 rv1 = make_double2(R[2] * v[0].x - R[0] * v[2].x, R[2] * v[0].y - R[0] * v[2].y);
  const double2 rv2 = make_double2(R[0] * v[1].x - R[1] * v[0].x, R[0] * v[1].y - R[1] * v[0].y);
  cfma(o[0], g.chi, rv0);
  cfma(o[1], g.chi, rv1);
  cfma(o[2], g.chi, rv2);
}

// Block-wide sum of one double per thread in a fixed order (blockDim.x a
// multiple of 64, at most 256); thread 0 receives the result.
__device__ inline double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[0];
}

// Load the 6 unknown components (E/p then H/m) of dipole j for RHS column r;
// cells have no magnetic unknowns (zeros).
__device__ inline void load6(const double2* x, int64_t ld, int64_t r, int64_t j, int64_t N, int64_t nc, double2 o[6]) {
  const double2* c = x + r * ld;
#pragma unroll
  for (int a = 0; a < 3; ++a) o[a] = c[3 * j + a];
  if (j >= nc) {
#pragma unroll
    for (int a = 0; a < 3; ++a) o[3 + a] = c[3 * N + 3 * (j - nc) + a];
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a) o[3 + a] = make_double2(0, 0);
  }
}

constexpr int PT = 256;  // probes per LDS tile (probe kernel)
constexpr int ST = 128;  // source dipoles per LDS tile (pair kernel)

// Probe side, one thread per dipole j and one probe range per blockIdx.y:
//   acc_j  = sum_p G6(r_p - r_j)[E rows]^T g_E(p)   -> pacc[split][r][unknowns of j]
//   grad_j = -2 Re sum_p d/dR [g_E(p)^T G6(R)[E rows] q_j],   R = r_p - r_j
//   dk     = 2 Re sum_p d/dk0 [g_E(p)^T G6(R)[E rows] q_j]     (block partial)
template <int NR>
__global__ void __launch_bounds__(256) adj_probe_kernel(DipoleView d, Wave w, double n_env,
                                                        const double2* __restrict__ q, int64_t n, int64_t nrhs, int r0,
                                                        const double* __restrict__ rp, const double2* __restrict__ gE,
                                                        int64_t P, int64_t p_per_split, double2* __restrict__ pacc,
                                                        double* __restrict__ pgr, double* __restrict__ pdk,
                                                        double min_r2, int* __restrict__ flag) {
  __shared__ double spos[PT][3];
  __shared__ double2 sg[PT][NR][3];
  __shared__ double red[256];
  const int64_t N = d.N, nc = d.nc;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int split = blockIdx.y, nsplit = gridDim.y, z = blockIdx.z;
  const int64_t p0 = split * p_per_split;
  const int64_t p1 = p0 + p_per_split < P ? p0 + p_per_split : P;
  const bool live = j < N;
  const bool jmag = live && j >= nc;
  double rj[3] = {0, 0, 0};
  double2 qj[NR][6];
  double2 accE[NR][3], accH[NR][3];
  double2 gx[3] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
  double2 dk = make_double2(0, 0);
#pragma unroll
  for (int r = 0; r < NR; ++r) {
#pragma unroll
    for (int a = 0; a < 3; ++a) accE[r][a] = accH[r][a] = make_double2(0, 0);
    if (live && r0 + r < nrhs) load6(q, n, r0 + r, j, N, nc, qj[r]);
    else
#pragma unroll
      for (int a = 0; a < 6; ++a) qj[r][a] = make_double2(0, 0);
  }
  if (live)
#pragma unroll
    for (int a = 0; a < 3; ++a) rj[a] = d.pos[3 * j + a];
  for (int64_t t0 = p0; t0 < p1; t0 += PT) {
    const int nt = (int)(p1 - t0 < PT ? p1 - t0 : PT);
    __syncthreads();
    for (int t = threadIdx.x; t < nt; t += blockDim.x) {
      const int64_t p = t0 + t;
#pragma unroll
      for (int a = 0; a < 3; ++a) spos[t][a] = rp[3 * p + a];
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int a = 0; a < 3; ++a)
          sg[t][r][a] = r0 + r < nrhs ? gE[((int64_t)(r0 + r) * P + p) * 3 + a] : make_double2(0, 0);
    }
    __syncthreads();
    if (!live) continue;
    for (int t = 0; t < nt; ++t) {
      const double R[3] = {spos[t][0] - rj[0], spos[t][1] - rj[1], spos[t][2] - rj[2]};
      const double R2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
      if (R2 < min_r2) {
        atomicOr(flag, 1);
        continue;
      }
      GreenRad g;
      green_rad(R2, w, n_env, g);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const double2* gv = sg[t][r];
        add_gep(g, R, gv, accE[r]);
        acc_ep(g, R, gv, qj[r], -1.0, gx, dk, true);
        if (jmag) {
          add_ghp(g, R, gv, accH[r]);
          acc_hp(g, R, gv, qj[r] + 3, 1.0, gx, dk, true);
        }
      }
    }
  }
  // gx holds d/dR of g.E summed with sign -1 (dR/dr_j = -1); dk holds -d/dk0 on
  // the E^Ep part and +d/dk0 on the G^Hp part: flip back to + sum d/dk0 [g.E].
  // (acc_ep/acc_hp apply the same sign to both outputs.)
  double dkr = 0.0;
  if (live) {
    const int64_t slot = (int64_t)(z * nsplit + split) * N + j;
#pragma unroll
    for (int x = 0; x < 3; ++x) pgr[3 * slot + x] = 2.0 * gx[x].x;
    dkr = -2.0 * dk.x;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (r0 + r >= nrhs) break;
      double2* o = pacc + ((int64_t)split * nrhs + r0 + r) * n;
#pragma unroll
      for (int a = 0; a < 3; ++a) o[3 * j + a] = accE[r][a];
      if (jmag)
#pragma unroll
        for (int a = 0; a < 3; ++a) o[3 * N + 3 * (j - nc) + a] = accH[r][a];
    }
  }
  const double s = block_sum(dkr, red);
  if (threadIdx.x == 0) pdk[(int64_t)(z * nsplit + split) * gridDim.x + blockIdx.x] = s;
}

// Seed, one thread per (dipole, RHS): Wirtinger partials of
// L_sigma = sum_r ws_ext ext + ws_sca sca + ws_abs abs (sca = ext - abs), with
// C_r = 4 pi k0 / (n_env |e0_r|^2):
//   g_q  = C [ be conj(F0)/(2i) + bb (conj(F)/(2i) - rho (2/3) k^3 w_c conj(q)) ]
//   g_F  = -C bb conj(q)/(2i),   (g_F0 = -C be conj(q)/(2i), used in the finish)
// be = ws_ext + ws_sca, bb = ws_abs - ws_sca, rho = 1 for effective dipoles,
// w_c = 1/eps_env on electric, 1 on magnetic components.  Writes
// gqe = g_q + sum_split pacc and rhs = g_F + A^T gqe.
__global__ void adj_seed_kernel(DipoleView d, Wave w, const double2* __restrict__ f0, const double2* __restrict__ f,
                                const double2* __restrict__ q, int64_t n, int64_t nrhs, const double* __restrict__ Cr,
                                const double* __restrict__ gsig, const double2* __restrict__ pacc, int nsplit,
                                double2* __restrict__ gqe, double2* __restrict__ rhs) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= d.N * nrhs) return;
  const int64_t r = t / d.N, j = t - r * d.N;
  const int64_t N = d.N, nc = d.nc;
  const bool mag = j >= nc;
  const int nu = mag ? 6 : 3;
  int64_t u[6];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    u[a] = 3 * j + a;
    u[3 + a] = mag ? 3 * N + 3 * (j - nc) + a : 0;
  }
  const double C = Cr[r];
  const double ws_ext = gsig ? gsig[3 * r] : 0.0, ws_sca = gsig ? gsig[3 * r + 1] : 0.0,
               ws_abs = gsig ? gsig[3 * r + 2] : 0.0;
  const double be = C * (ws_ext + ws_sca), bb = C * (ws_abs - ws_sca);
  const double k3 = (2.0 / 3.0) * w.k * w.k * w.k;
  const int64_t o = r * n;
  double2 g[6], gF[6];
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    g[a] = gF[a] = make_double2(0.0, 0.0);
    if (a >= nu) continue;  // compile-time indices (no private-memory arrays)
    const double2 F0 = f0[o + u[a]], F = f[o + u[a]], Q = q[o + u[a]];
    // conj(z)/(2i) = (-Im z, -Re z)/2
    double2 gq = make_double2(-0.5 * (be * F0.y + bb * F.y), -0.5 * (be * F0.x + bb * F.x));
    if (mag) {
      const double wc = a < 3 ? 1.0 / w.eps_env : 1.0;
      gq.x -= bb * k3 * wc * Q.x;
      gq.y += bb * k3 * wc * Q.y;
    }
    for (int s = 0; s < nsplit; ++s) gq = cadd(gq, pacc[((int64_t)s * nrhs + r) * n + u[a]]);
    g[a] = gq;
    // -conj(q)/(2i) = (Im q, Re q)/2
    gF[a] = make_double2(0.5 * bb * Q.y, 0.5 * bb * Q.x);
    gqe[o + u[a]] = gq;
  }
  if (!mag) {
    const double2 al = d.alpha_c[j];
#pragma unroll
    for (int a = 0; a < 3; ++a) rhs[o + u[a]] = cadd(gF[a], cmul(al, g[a]));
  } else {
    const double2* A = d.alpha6 + 36 * (j - nc);  // row-major [6][6]; (A^T g)_a = sum_b A[b][a] g_b
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      double2 s = gF[a];
#pragma unroll
      for (int b = 0; b < 6; ++b) cfma(s, A[6 * b + a], g[b]);
      rhs[o + u[a]] = s;
    }
  }
}

// Pair side, one thread per target dipole m and one source range per blockIdx.y,
// R = r_m - r_j (j != m):
//   grad_m += 2 Re [ d/dR lam_m^T G6(R) q_j  -  (d/dR G6)(-R) contracted with lam_j, q_m ]
//   dk     += 2 Re   d/dk0 lam_m^T G6(R) q_j                      (block partial)
//   v_m    += [G6(-R)^T lam_j]_E = G^Ep(R) lam_jE + G^Hp(R) lam_jH   (cells only)
// with lam^T G6 q = EP(lamE, qp) - HP(lamE, qm) + HP(lamH, qp) + eps EP(lamH, qm),
// EP/HP the G^Ep/G^Hp forms; at -R the G^Ep forms change sign under d/dR and the
// G^Hp forms do not.
template <int NR>
__global__ void __launch_bounds__(128) adj_pair_kernel(DipoleView d, Wave w, double n_env,
                                                       const double2* __restrict__ lam, const double2* __restrict__ q,
                                                       int64_t n, int64_t nrhs, int r0, int64_t j_per_split,
                                                       double* __restrict__ pgr, double2* __restrict__ pv,
                                                       double* __restrict__ pdk) {
  __shared__ double spos[ST][3];
  __shared__ double2 sl[ST][NR][6];
  __shared__ double2 sq[ST][NR][6];
  __shared__ double red[128];
  const int64_t N = d.N, nc = d.nc;
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int split = blockIdx.y, nsplit = gridDim.y, z = blockIdx.z;
  const int64_t j0 = split * j_per_split;
  const int64_t j1 = j0 + j_per_split < N ? j0 + j_per_split : N;
  const bool live = m < N;
  const bool mmag = live && m >= nc;
  const double eps = w.eps_env;
  double rm[3] = {0, 0, 0};
  double2 lm[NR][6], qm[NR][6], v[NR][3];
  double2 gx[3] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
  double2 dk = make_double2(0, 0);
#pragma unroll
  for (int r = 0; r < NR; ++r) {
#pragma unroll
    for (int a = 0; a < 3; ++a) v[r][a] = make_double2(0, 0);
    if (live && r0 + r < nrhs) {
      load6(lam, n, r0 + r, m, N, nc, lm[r]);
      load6(q, n, r0 + r, m, N, nc, qm[r]);
    } else {
#pragma unroll
      for (int a = 0; a < 6; ++a) lm[r][a] = qm[r][a] = make_double2(0, 0);
    }
  }
  if (live)
#pragma unroll
    for (int a = 0; a < 3; ++a) rm[a] = d.pos[3 * m + a];
  for (int64_t t0 = j0; t0 < j1; t0 += ST) {
    const int nt = (int)(j1 - t0 < ST ? j1 - t0 : ST);
    __syncthreads();
    for (int t = threadIdx.x; t < nt; t += blockDim.x) {
      const int64_t j = t0 + t;
#pragma unroll
      for (int a = 0; a < 3; ++a) spos[t][a] = d.pos[3 * j + a];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (r0 + r < nrhs) {
          load6(lam, n, r0 + r, j, N, nc, sl[t][r]);
          load6(q, n, r0 + r, j, N, nc, sq[t][r]);
        } else {
#pragma unroll
          for (int a = 0; a < 6; ++a) sl[t][r][a] = sq[t][r][a] = make_double2(0, 0);
        }
      }
    }
    __syncthreads();
    if (!live) continue;
    for (int t = 0; t < nt; ++t) {
      const int64_t j = t0 + t;
      if (j == m) continue;
      const double R[3] = {rm[0] - spos[t][0], rm[1] - spos[t][1], rm[2] - spos[t][2]};
      const double R2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
      if (R2 == 0.0) continue;
      const bool jmag = j >= nc;
      GreenRad g;
      green_rad(R2, w, n_env, g);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const double2* lj = sl[t][r];
        const double2* qj = sq[t][r];
        // target-side term lam_m^T G6(R) q_j (position and k0 derivatives)
        acc_ep(g, R, lm[r], qj, 1.0, gx, dk, true);
        // source-side term -(dG6)(-R) with lam_j, q_m (position only)
        double2 dummy = make_double2(0, 0);
        acc_ep(g, R, lj, qm[r], 1.0, gx, dummy, false);
        if (jmag) {
          acc_hp(g, R, lm[r], qj + 3, -1.0, gx, dk, true);
          acc_hp(g, R, lj + 3, qm[r], -1.0, gx, dummy, false);
        }
        if (mmag) {
          acc_hp(g, R, lm[r] + 3, qj, 1.0, gx, dk, true);
          acc_hp(g, R, lj, qm[r] + 3, 1.0, gx, dummy, false);
          if (jmag) {
            acc_ep(g, R, lm[r] + 3, qj + 3, eps, gx, dk, true);
            acc_ep(g, R, lj + 3, qm[r] + 3, eps, gx, dummy, false);
          }
        } else {
          add_gep(g, R, lj, v[r]);
          if (jmag) add_ghp(g, R, lj + 3, v[r]);
        }
      }
    }
  }
  double dkr = 0.0;
  if (live) {
    const int64_t slot = (int64_t)(z * nsplit + split) * N + m;
#pragma unroll
    for (int x = 0; x < 3; ++x) pgr[3 * slot + x] = 2.0 * gx[x].x;
    dkr = 2.0 * dk.x;
    if (!mmag)
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (r0 + r >= nrhs) break;
        double2* o = pv + (((int64_t)split * nrhs + r0 + r) * nc + m) * 3;
#pragma unroll
        for (int a = 0; a < 3; ++a) o[a] = v[r][a];
      }
  }
  const double s = block_sum(dkr, red);
  if (threadIdx.x == 0) pdk[(int64_t)(z * nsplit + split) * gridDim.x + blockIdx.x] = s;
}

// Finish, one thread per dipole m:
//   grad_r[m] = sum of the probe and pair partials
//               + 2 Re sum_r (lam + g_F0)_m . (i k khat_r) F0_m          (incident phase)
//   cells:    s_m = d^3/(4 pi) sum_r (v_m + S lam_m + gqe_m) . F_m,
//             grad_eps[m] = (2 Re s_m, -2 Im s_m)
//   dk partial: 2 Re sum_r (lam + g_F0) . (i n_env khat_r . r_m) F0  (+ radiative self-term)
__global__ void adj_finish_kernel(DipoleView d, Wave w, double n_env, double step, int radiative,
                                  const double2* __restrict__ f0, const double2* __restrict__ f,
                                  const double2* __restrict__ q, const double2* __restrict__ lam,
                                  const double2* __restrict__ gqe, int64_t n, int64_t nrhs,
                                  const double* __restrict__ khat, const double* __restrict__ Cr,
                                  const double* __restrict__ gsig, const double* __restrict__ pgr_probe,
                                  int nslot_probe, const double* __restrict__ pgr_pair, int nslot_pair,
                                  const double2* __restrict__ pv, int nsplit_pair, double* __restrict__ grad_r,
                                  double* __restrict__ grad_eps, double* __restrict__ pdk) {
  __shared__ double red[256];
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = d.N, nc = d.nc;
  double dkr = 0.0;
  if (m < N) {
    const bool mag = m >= nc;
    const int nu = mag ? 6 : 3;
    int64_t u[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      u[a] = 3 * m + a;
      u[3 + a] = mag ? 3 * N + 3 * (m - nc) + a : 0;
    }
    double gr[3] = {0, 0, 0};
    for (int s = 0; s < nslot_probe; ++s)
      for (int x = 0; x < 3; ++x) gr[x] += pgr_probe[3 * ((int64_t)s * N + m) + x];
    for (int s = 0; s < nslot_pair; ++s)
      for (int x = 0; x < 3; ++x) gr[x] += pgr_pair[3 * ((int64_t)s * N + m) + x];
    const double rx = d.pos[3 * m], ry = d.pos[3 * m + 1], rz = d.pos[3 * m + 2];
    const double2 S = d.self_c;
    double2 sacc = make_double2(0, 0);
    double2 selfk = make_double2(0, 0);
    for (int64_t r = 0; r < nrhs; ++r) {
      const int64_t o = r * n;
      const double be = gsig ? Cr[r] * (gsig[3 * r] + gsig[3 * r + 1]) : 0.0;
      const double kx = khat[3 * r], ky = khat[3 * r + 1], kz = khat[3 * r + 2];
      const double kr = kx * rx + ky * ry + kz * rz;
      double2 t = make_double2(0, 0);  // sum_c (lam + g_F0)_c F0_c
      for (int a = 0; a < nu; ++a) {
        const double2 Q = q[o + u[a]];
        const double2 L = cadd(lam[o + u[a]], make_double2(0.5 * be * Q.y, 0.5 * be * Q.x));
        cfma(t, L, f0[o + u[a]]);
      }
      // d/dr_a: i k khat_a t ;  d/dk0: i n_env (khat . r) t
      gr[0] += -2.0 * w.k * kx * t.y;
      gr[1] += -2.0 * w.k * ky * t.y;
      gr[2] += -2.0 * w.k * kz * t.y;
      dkr += -2.0 * n_env * kr * t.y;
      if (!mag) {
        for (int a = 0; a < 3; ++a) {
          double2 vv = gqe[o + u[a]];
          cfma(vv, S, lam[o + u[a]]);
          for (int s = 0; s < nsplit_pair; ++s) vv = cadd(vv, pv[(((int64_t)s * nrhs + r) * nc + m) * 3 + a]);
          cfma(sacc, vv, f[o + u[a]]);
          if (radiative) cfma(selfk, lam[o + u[a]], q[o + u[a]]);
        }
      }
    }
    for (int x = 0; x < 3; ++x) grad_r[3 * m + x] = gr[x];
    if (!mag) {
      const double sc = step * step * step / (4.0 * M_PI);
      grad_eps[2 * m] = 2.0 * sc * sacc.x;
      grad_eps[2 * m + 1] = -2.0 * sc * sacc.y;
      if (radiative) {
        // d/dk0 of the radiative self-term i (2/3) k^3 / eps_env: i 2 k^2 n_env / eps_env
        const double2 dS = make_double2(0.0, 2.0 * w.k * w.k * n_env / w.eps_env);
        dkr += 2.0 * cmul(dS, selfk).x;
      }
    }
  }
  const double s = block_sum(dkr, red);
  if (threadIdx.x == 0) pdk[blockIdx.x] = s;
}

// Incident field at the probes: 2 Re sum g_E . dE_inc/dk0 with
// E_inc = e0 exp(i k khat.r_p), dE_inc/dk0 = i n_env (khat.r_p) E_inc.
__global__ void adj_einc_kernel(Wave w, double n_env, const double* __restrict__ khat,
                                const double2* __restrict__ e0, const double* __restrict__ rp,
                                const double2* __restrict__ gE, int64_t P, int64_t nrhs, double* __restrict__ pdk) {
  __shared__ double red[256];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (t < P * nrhs) {
    const int64_t r = t / P, p = t - r * P;
    const double kr = khat[3 * r] * rp[3 * p] + khat[3 * r + 1] * rp[3 * p + 1] + khat[3 * r + 2] * rp[3 * p + 2];
    double s, c;
    sincos(w.k * kr, &s, &c);
    const double2 ph = make_double2(c, s);
    double2 acc = make_double2(0, 0);
    for (int a = 0; a < 3; ++a) cfma(acc, gE[(r * P + p) * 3 + a], cmul(e0[3 * r + a], ph));
    // 2 Re[i n kr acc] = -2 n kr Im acc
    v = -2.0 * n_env * kr * acc.y;
  }
  const double s = block_sum(v, red);
  if (threadIdx.x == 0) pdk[blockIdx.x] = s;
}

// C_r = 4 pi k0 / (n_env |e0_r|^2)
__global__ void adj_cr_kernel(Wave w, double n_env, const double2* __restrict__ e0, int64_t nrhs,
                              double* __restrict__ Cr) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  double e2 = 0.0;
  for (int a = 0; a < 3; ++a) e2 += e0[3 * r + a].x * e0[3 * r + a].x + e0[3 * r + a].y * e0[3 * r + a].y;
  Cr[r] = 4.0 * M_PI * w.k0 / (n_env * e2);
}

// dL/dlambda0 = dL/dk0 * (-k0 / lambda0), with dL/dk0 = all partials + the
// explicit dependence of the cross sections on k0:
//   sum_r [ws_ext ext + ws_sca sca + ws_abs abs] / k0 + (ws_sca - ws_abs) 3 C prad_eff / k0,
// ext = C s0, prad_eff = (2/3) k^3 (s3 / eps_env + s4), abs = C (s1 - prad_eff).
__global__ void adj_wl_kernel(Wave w, double wavelength, const double* __restrict__ parts, int64_t nparts,
                              const double* __restrict__ sums5, const double* __restrict__ Cr,
                              const double* __restrict__ gsig, int64_t nrhs, double* __restrict__ grad_wl) {
  __shared__ double red[256];
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < nparts; i += blockDim.x) v += parts[i];
  if (gsig)
    for (int64_t r = threadIdx.x; r < nrhs; r += blockDim.x) {
      const double C = Cr[r];
      const double* s5 = sums5 + 5 * r;
      const double prad = (2.0 / 3.0) * w.k * w.k * w.k * (s5[3] / w.eps_env + s5[4]);
      const double ext = C * s5[0], ab = C * (s5[1] - prad), sca = ext - ab;
      v += (gsig[3 * r] * ext + gsig[3 * r + 1] * sca + gsig[3 * r + 2] * ab) / w.k0 +
           (gsig[3 * r + 1] - gsig[3 * r + 2]) * 3.0 * C * prad / w.k0;
    }
  const double s = block_sum(v, red);
  if (threadIdx.x == 0) grad_wl[0] = s * (-w.k0 / wavelength);
}

}  // namespace

int adjoint_probe_splits(int64_t P, int64_t N, int num_cu) {
  const int64_t xb = (N + 255) / 256;
  int64_t want = (4 * (int64_t)num_cu + xb - 1) / xb;
  const int64_t maxs = (P + PT - 1) / PT;
  if (want > maxs) want = maxs;
  if (want > 64) want = 64;
  return (int)(want < 1 ? 1 : want);
}
int adjoint_pair_splits(int64_t N, int num_cu) {
  const int64_t xb = (N + 127) / 128;
  int64_t want = (4 * (int64_t)num_cu + xb - 1) / xb;
  const int64_t maxs = (N + ST - 1) / ST;
  if (want > maxs) want = maxs;
  if (want > 64) want = 64;
  return (int)(want < 1 ? 1 : want);
}
int64_t adjoint_probe_blocks(int64_t N) { return (N + 255) / 256; }
int64_t adjoint_pair_blocks(int64_t N) { return (N + 127) / 128; }
int64_t adjoint_finish_blocks(int64_t N) { return (N + 255) / 256; }
int64_t adjoint_einc_blocks(int64_t P, int64_t nrhs) { return (P * nrhs + 255) / 256; }
int adjoint_rhs_chunks(int64_t nrhs) { return (int)((nrhs + 1) / 2); }

hipError_t launch_adjoint_cr(const Wave& w, double n_env, const double2* e0, int64_t nrhs, double* Cr,
                             hipStream_t st) {
  hipLaunchKernelGGL(adj_cr_kernel, dim3((unsigned)((nrhs + 63) / 64)), dim3(64), 0, st, w, n_env, e0, nrhs, Cr);
  return hipGetLastError();
}

hipError_t launch_adjoint_probe(const DipoleView& d, const Wave& w, double n_env, const double2* q, int64_t n,
                                int64_t nrhs, const double* rp, const double2* gE, int64_t P, int nsplit,
                                double2* pacc, double* pgr, double* pdk, double min_r2, int* flag, hipStream_t st) {
  const int64_t pps = ((P + nsplit - 1) / nsplit + PT - 1) / PT * PT;
  const int nz = adjoint_rhs_chunks(nrhs);
  const unsigned xb = (unsigned)adjoint_probe_blocks(d.N);
  for (int z = 0; z < nz; ++z) {
    const int r0 = 2 * z;
    // one launch per RHS chunk; blockIdx.z is the chunk's slot in the partial arrays
    double* pgr_z = pgr + (int64_t)z * nsplit * d.N * 3;
    double* pdk_z = pdk + (int64_t)z * nsplit * xb;
    if (nrhs - r0 >= 2)
      hipLaunchKernelGGL(adj_probe_kernel<2>, dim3(xb, nsplit, 1), dim3(256), 0, st, d, w, n_env, q, n, nrhs, r0, rp,
                         gE, P, pps, pacc, pgr_z, pdk_z, min_r2, flag);
    else
      hipLaunchKernelGGL(adj_probe_kernel<1>, dim3(xb, nsplit, 1), dim3(256), 0, st, d, w, n_env, q, n, nrhs, r0, rp,
                         gE, P, pps, pacc, pgr_z, pdk_z, min_r2, flag);
  }
  return hipGetLastError();
}

hipError_t launch_adjoint_seed(const DipoleView& d, const Wave& w, const double2* f0, const double2* f,
                               const double2* q, int64_t n, int64_t nrhs, const double* Cr, const double* gsig,
                               const double2* pacc, int nsplit, double2* gqe, double2* rhs, hipStream_t st) {
  const int64_t tot = d.N * nrhs;
  hipLaunchKernelGGL(adj_seed_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, d, w, f0, f, q, n, nrhs,
                     Cr, gsig, pacc, nsplit, gqe, rhs);
  return hipGetLastError();
}

hipError_t launch_adjoint_pair(const DipoleView& d, const Wave& w, double n_env, const double2* lam,
                               const double2* q, int64_t n, int64_t nrhs, int nsplit, double* pgr, double2* pv,
                               double* pdk, hipStream_t st) {
  const int64_t jps = ((d.N + nsplit - 1) / nsplit + ST - 1) / ST * ST;
  const int nz = adjoint_rhs_chunks(nrhs);
  const unsigned xb = (unsigned)adjoint_pair_blocks(d.N);
  for (int z = 0; z < nz; ++z) {
    const int r0 = 2 * z;
    double* pgr_z = pgr + (int64_t)z * nsplit * d.N * 3;
    double* pdk_z = pdk + (int64_t)z * nsplit * xb;
    if (nrhs - r0 >= 2)
      hipLaunchKernelGGL(adj_pair_kernel<2>, dim3(xb, nsplit, 1), dim3(128), 0, st, d, w, n_env, lam, q, n, nrhs, r0,
                         jps, pgr_z, pv, pdk_z);
    else
      hipLaunchKernelGGL(adj_pair_kernel<1>, dim3(xb, nsplit, 1), dim3(128), 0, st, d, w, n_env, lam, q, n, nrhs, r0,
                         jps, pgr_z, pv, pdk_z);
  }
  return hipGetLastError();
}

hipError_t launch_adjoint_finish(const DipoleView& d, const Wave& w, double n_env, double step, int radiative,
                                 const double2* f0, const double2* f, const double2* q, const double2* lam,
                                 const double2* gqe, int64_t n, int64_t nrhs, const double* khat, const double* Cr,
                                 const double* gsig, const double* pgr_probe, int nslot_probe, const double* pgr_pair,
                                 int nslot_pair, const double2* pv, int nsplit_pair, double* grad_r,
                                 double* grad_eps, double* pdk, hipStream_t st) {
  hipLaunchKernelGGL(adj_finish_kernel, dim3((unsigned)adjoint_finish_blocks(d.N)), dim3(256), 0, st, d, w, n_env,
                     step, radiative, f0, f, q, lam, gqe, n, nrhs, khat, Cr, gsig, pgr_probe, nslot_probe, pgr_pair,
                     nslot_pair, pv, nsplit_pair, grad_r, grad_eps, pdk);
  return hipGetLastError();
}

hipError_t launch_adjoint_einc(const Wave& w, double n_env, const double* khat, const double2* e0, const double* rp,
                               const double2* gE, int64_t P, int64_t nrhs, double* pdk, hipStream_t st) {
  hipLaunchKernelGGL(adj_einc_kernel, dim3((unsigned)adjoint_einc_blocks(P, nrhs)), dim3(256), 0, st, w, n_env, khat,
                     e0, rp, gE, P, nrhs, pdk);
  return hipGetLastError();
}

hipError_t launch_adjoint_wl(const Wave& w, double wavelength, const double* parts, int64_t nparts,
                             const double* sums5, const double* Cr, const double* gsig, int64_t nrhs, double* grad_wl,
                             hipStream_t st) {
  hipLaunchKernelGGL(adj_wl_kernel, dim3(1), dim3(256), 0, st, w, wavelength, parts, nparts, sums5, Cr, gsig, nrhs,
                     grad_wl);
  return hipGetLastError();
}

}  // namespace gdm
