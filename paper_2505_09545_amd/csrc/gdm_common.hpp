// Shared device helpers of libgdm: complex arithmetic on interleaved (re, im)
// storage, the free-space Green's dyad of a homogeneous lossless medium, and the
// launch/error plumbing used by every kernel file.
//
// Physics (arXiv:2505.09545, Sec. "Formalism and implementation", Eq.
// superprop_G): the 6x6 dyad G = [[G^Ep, G^Em], [G^Hp, G^Hm]] maps the electric
// and magnetic dipole moments (p, m) at r' to the fields (E, H) at r.  Gaussian
// units, time factor exp(-i w t), mu = 1, k = n_env k0, eps_env = n_env^2:
//   G^Ep = e^{ikR}/eps_env [ (k^2/R + ik/R^2 - 1/R^3) I + (-k^2/R - 3ik/R^2 + 3/R^3) Rh Rh ]
//   G^Hp = k0 k e^{ikR} (1/R^2 + i/(k R^3)) [R]_x          ([R]_x v = R x v)
//   G^Em = -G^Hp,  G^Hm = eps_env G^Ep.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace gdm {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// complex of T stored as the HIP vector type (16 B for double, 8 B for float)
template <typename T> struct cvec;
template <> struct cvec<double> { using type = double2; };
template <> struct cvec<float> { using type = float2; };
template <typename T> using cplx = typename cvec<T>::type;

__host__ __device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__host__ __device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
// a += b * c
__host__ __device__ inline void cfma(double2& a, double2 b, double2 c) {
  a.x += b.x * c.x - b.y * c.y;
  a.y += b.x * c.y + b.y * c.x;
}
__host__ __device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <typename T> __device__ inline cplx<T> to_c(double2 v);
template <> __device__ inline double2 to_c<double>(double2 v) { return v; }
template <> __device__ inline float2 to_c<float>(double2 v) { return make_float2((float)v.x, (float)v.y); }

__device__ inline double2 to_d(double2 v) { return v; }
__device__ inline double2 to_d(float2 v) { return make_double2(v.x, v.y); }

// Wave-number bundle passed by value to kernels.
struct Wave {
  double k0;       // vacuum wave number 2 pi / lambda0 [1/nm]
  double k;        // n_env k0
  double eps_env;  // n_env^2 (real, lossless host)
};

// Unique entries of the symmetric G^Ep (xx, yy, zz, xy, xz, yz) and the vector
// h with G^Hp = [h]_x.
struct Green {
  double2 e[6];
  double2 h[3];
};

// Green's dyad blocks for separation R = r - r' (R != 0).  One sincos per call.
__device__ inline void green_eh(double Rx, double Ry, double Rz, const Wave& w, bool want_h, Green& g) {
  const double R2 = Rx * Rx + Ry * Ry + Rz * Rz;
  const double R = sqrt(R2);
  const double iR = 1.0 / R;
  double s, c;
  sincos(w.k * R, &s, &c);
  const double iR2 = iR * iR;
  const double iR3 = iR2 * iR;
  const double k = w.k;
  const double ie = 1.0 / w.eps_env;
  // a = e^{ikR}/eps (k^2/R - 1/R^3 + i k/R^2)
  const double ar = k * k * iR - iR3, ai = k * iR2;
  // b = e^{ikR}/eps (-k^2/R + 3/R^3 - 3i k/R^2) / R^2   (multiplies R_a R_b)
  const double br = (-k * k * iR + 3.0 * iR3) * iR2, bi = (-3.0 * k * iR2) * iR2;
  const double pr = c * ie, pi = s * ie;
  const double2 a = make_double2(pr * ar - pi * ai, pr * ai + pi * ar);
  const double2 b = make_double2(pr * br - pi * bi, pr * bi + pi * br);
  g.e[0] = make_double2(a.x + b.x * Rx * Rx, a.y + b.y * Rx * Rx);
  g.e[1] = make_double2(a.x + b.x * Ry * Ry, a.y + b.y * Ry * Ry);
  g.e[2] = make_double2(a.x + b.x * Rz * Rz, a.y + b.y * Rz * Rz);
  g.e[3] = make_double2(b.x * Rx * Ry, b.y * Rx * Ry);
  g.e[4] = make_double2(b.x * Rx * Rz, b.y * Rx * Rz);
  g.e[5] = make_double2(b.x * Ry * Rz, b.y * Ry * Rz);
  if (want_h) {
    // u = k0 k e^{ikR} (1/R^2 + i/(k R^3)), h = u R
    const double ur = w.k0 * k * iR2, ui = w.k0 * iR3;
    const double2 u = make_double2(c * ur - s * ui, c * ui + s * ur);
    g.h[0] = cscale(u, Rx);
    g.h[1] = cscale(u, Ry);
    g.h[2] = cscale(u, Rz);
  }
}

// G^Ep[a][b] from the unique entries.
__device__ inline double2 gep(const Green& g, int a, int b) {
  const int idx[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
  return g.e[idx[a][b]];
}
// G^Hp[a][b] = ([h]_x)[a][b]
__device__ inline double2 ghp(const Green& g, int a, int b) {
  if (a == b) return make_double2(0.0, 0.0);
  // [h]_x = [[0, -hz, hy], [hz, 0, -hx], [-hy, hx, 0]]
  const int c = 3 - a - b;
  const double sgn = ((a + 1) % 3 == b) ? -1.0 : 1.0;
  return cscale(g.h[c], sgn);
}

// 6x6 block entry of the dyad, rows (E, H) x cols (p, m).
__device__ inline double2 g6(const Green& g, double eps_env, int r, int c) {
  if (r < 3) return c < 3 ? gep(g, r, c) : cscale(ghp(g, r, c - 3), -1.0);
  return c < 3 ? ghp(g, r - 3, c) : cscale(gep(g, r - 3, c - 3), eps_env);
}

}  // namespace gdm
