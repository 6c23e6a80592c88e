// Step (b) without a stored matrix: the linear system M F = F0, M = I - G~ A,
// solved by a Krylov method whose matrix-vector product re-evaluates the
// coupling sum from the dyad on every call (arXiv:2505.09545, Sec. "Discrete
// Dipole Approximation - iterative solver": the DDA route past the size where
// the dense inversion no longer fits, cf. Sec. "Benchmarks", runtime and
// memory; the paper's own solver is the dense LU of Sec. "Numerical solution").
//
// Product: y = M x = x - G~ (A x).  q = A x (the dipole moments of the field
// x), then for every dipole i, as a target, the field of all other dipoles,
// sum_{j != i} G(r_i, r_j) q_j, plus the self-term S_i q_i of a cell; the 6x6
// dyad of every pair is recomputed in registers (one sincos) and never stored.
// Sources are swept in LDS tiles, the sum split over several workgroups when
// there are few targets, the partial sums added in a fixed order by the kernel
// that forms y (deterministic).
//
// Preconditioner: block Jacobi over near-field blocks -- consecutive dipoles in
// groups of PC_DIP (spatial neighbours for the cubic grids and lattices of the
// workloads, which are laid out in grid order).  Each block's rows and columns
// of M (its E unknowns, then the H unknowns of its effective dipoles, at most
// PC_MAXD) are assembled in FP64 with the same block formula as the dense
// assembly and inverted by Gauss-Jordan elimination with partial pivoting.
//
// Krylov method: restarted GMRES with right preconditioning (so the residual
// it minimises is that of the original system), classical Gram-Schmidt with
// one re-orthogonalisation, Givens rotations of the small Hessenberg matrix on
// the host; one small device-to-host copy per iteration.  All arithmetic FP64.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "gdm_common.hpp"
#include "gdm_kernels.hpp"
#include "gdm_misc.hpp"
#include "gdm_iterative.hpp"

namespace gdm {

constexpr int CT = 256;  // source dipoles per LDS tile

// Partial coupling sums of the sources [split * jps, (split + 1) * jps): one
// thread per target dipole i; E_i for every target, H_i for effective targets,
// written to part[split][r][u] in the unknown layout (u = 3i + a for E, 3N +
// 3(i - nc) + a for H).  The pair j == i is skipped.
template <int NR>
__global__ void __launch_bounds__(256) coupling_kernel(DipoleView d, Wave w, const double2* __restrict__ q, int64_t n,
                                                        int64_t nrhs, int r0, int64_t jps,
                                                        double2* __restrict__ part) {
  __shared__ double spos[CT][3];
  __shared__ double2 sp[CT][NR][3];
  __shared__ double2 sm[CT][NR][3];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int split = blockIdx.y;
  const int64_t N = d.N, nc = d.nc;
  const int64_t j0 = split * jps;
  const int64_t j1 = j0 + jps < N ? j0 + jps : N;
  const bool live = i < N;
  const bool eff_t = live && i >= nc;
  double x = 0, y = 0, z = 0;
  if (live) {
    x = d.pos[3 * i];
    y = d.pos[3 * i + 1];
    z = d.pos[3 * i + 2];
  }
  double2 E[NR][3], H[NR][3];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      E[r][a] = make_double2(0, 0);
      H[r][a] = make_double2(0, 0);
    }
  for (int64_t t0 = j0; t0 < j1; t0 += CT) {
    const int nt = (int)(j1 - t0 < CT ? j1 - t0 : CT);
    __syncthreads();
    for (int t = threadIdx.x; t < nt; t += 256) {
      const int64_t j = t0 + t;
      double pv[3];
      double2 qv[NR][3], mv[NR][3];
#pragma unroll
      for (int a = 0; a < 3; ++a) pv[a] = d.pos[3 * j + a];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const bool rv = r0 + r < nrhs;
        const double2* qc = q + (int64_t)(r0 + r) * n;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          qv[r][a] = rv ? qc[3 * j + a] : make_double2(0, 0);
          mv[r][a] = (rv && j >= nc) ? qc[3 * N + 3 * (j - nc) + a] : make_double2(0, 0);
        }
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) spos[t][a] = pv[a];
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          sp[t][r][a] = qv[r][a];
          sm[t][r][a] = mv[r][a];
        }
    }
    __syncthreads();
    if (!live) continue;
    const int ncell_in_tile = (int)(nc - t0 > 0 ? (nc - t0 < nt ? nc - t0 : nt) : 0);
    for (int t = 0; t < nt; ++t) {
      if (t0 + t == i) continue;
      const bool eff_s = t >= ncell_in_tile;
      Green g;
      green_eh(x - spos[t][0], y - spos[t][1], z - spos[t][2], w, eff_t || eff_s, g);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const double2 px = sp[t][r][0], py = sp[t][r][1], pz = sp[t][r][2];
        // E += G^Ep p
        cfma(E[r][0], g.e[0], px); cfma(E[r][0], g.e[3], py); cfma(E[r][0], g.e[4], pz);
        cfma(E[r][1], g.e[3], px); cfma(E[r][1], g.e[1], py); cfma(E[r][1], g.e[5], pz);
        cfma(E[r][2], g.e[4], px); cfma(E[r][2], g.e[5], py); cfma(E[r][2], g.e[2], pz);
        if (eff_t) {
          // H += h x p
          cfma(H[r][0], g.h[1], pz); cfma(H[r][0], cscale(g.h[2], -1.0), py);
          cfma(H[r][1], g.h[2], px); cfma(H[r][1], cscale(g.h[0], -1.0), pz);
          cfma(H[r][2], g.h[0], py); cfma(H[r][2], cscale(g.h[1], -1.0), px);
        }
        if (eff_s) {
          const double2 mx = sm[t][r][0], my = sm[t][r][1], mz = sm[t][r][2];
          // E += G^Em m = -(h x m)
          cfma(E[r][0], cscale(g.h[1], -1.0), mz); cfma(E[r][0], g.h[2], my);
          cfma(E[r][1], cscale(g.h[2], -1.0), mx); cfma(E[r][1], g.h[0], mz);
          cfma(E[r][2], cscale(g.h[0], -1.0), my); cfma(E[r][2], g.h[1], mx);
          if (eff_t) {
            // H += eps G^Ep m
            double2 u0 = make_double2(0, 0), u1 = make_double2(0, 0), u2 = make_double2(0, 0);
            cfma(u0, g.e[0], mx); cfma(u0, g.e[3], my); cfma(u0, g.e[4], mz);
            cfma(u1, g.e[3], mx); cfma(u1, g.e[1], my); cfma(u1, g.e[5], mz);
            cfma(u2, g.e[4], mx); cfma(u2, g.e[5], my); cfma(u2, g.e[2], mz);
            H[r][0] = cadd(H[r][0], cscale(u0, w.eps_env));
            H[r][1] = cadd(H[r][1], cscale(u1, w.eps_env));
            H[r][2] = cadd(H[r][2], cscale(u2, w.eps_env));
          }
        }
      }
    }
  }
  if (!live) return;
  const int64_t stride = nrhs * n;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r0 + r >= nrhs) break;
    double2* o = part + split * stride + (int64_t)(r0 + r) * n;
#pragma unroll
    for (int a = 0; a < 3; ++a) o[3 * i + a] = E[r][a];
    if (eff_t)
#pragma unroll
      for (int a = 0; a < 3; ++a) o[3 * N + 3 * (i - nc) + a] = H[r][a];
  }
}

// y = x - sum_s part[s] - (cell E unknowns) S q, over nrhs * n entries
__global__ void coupling_finish_kernel(const double2* __restrict__ part, int nsplit, int64_t stride,
                                       const double2* __restrict__ x, const double2* __restrict__ q, double2 self_c,
                                       int64_t ncell3, int64_t n, double2* __restrict__ y, int64_t count) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= count) return;
  double2 s = part[idx];
  for (int k = 1; k < nsplit; ++k) s = cadd(s, part[k * stride + idx]);
  double2 v = csub(x[idx], s);
  if (idx % n < ncell3) v = csub(v, cmul(self_c, q[idx]));
  y[idx] = v;
}

// ---------------------------------------------------------------------------
// block Jacobi preconditioner
// ---------------------------------------------------------------------------
// Block b: dipoles [b PC_DIP, min((b + 1) PC_DIP, N)).  Local unknowns: the E
// slots of its dipoles (3 each), then the H slots of its effective dipoles.
struct PcBlock {
  int64_t d0;  // first dipole
  int nd;      // dipoles
  int ne;      // effective dipoles among them (the last ne, since cells come first)
  int D;       // local unknowns 3 (nd + ne)
};
__device__ inline PcBlock pc_block(const DipoleView& d, int64_t b) {
  PcBlock p;
  p.d0 = b * PC_DIP;
  const int64_t d1 = p.d0 + PC_DIP < d.N ? p.d0 + PC_DIP : d.N;
  p.nd = (int)(d1 - p.d0);
  const int64_t e0 = p.d0 > d.nc ? p.d0 : d.nc;
  p.ne = d1 > e0 ? (int)(d1 - e0) : 0;
  p.D = 3 * (p.nd + p.ne);
  return p;
}
// global unknown of local unknown l of block p
__device__ inline int64_t pc_unknown(const DipoleView& d, const PcBlock& p, int l) {
  const int slot = l / 3, a = l % 3;
  if (slot < p.nd) return 3 * (p.d0 + slot) + a;
  const int64_t dip = p.d0 + p.nd - p.ne + (slot - p.nd);  // effective dipole
  return 3 * d.N + 3 * (dip - d.nc) + a;
}

// One workgroup per block: its D x D block of M in LDS next to the identity,
// Gauss-Jordan with partial pivoting (largest modulus in the column), the
// inverse written column-major to inv[b] (leading dimension PC_MAXD).  A zero
// pivot leaves the identity for that block (no preconditioning there).
__global__ void __launch_bounds__(256) precond_build_kernel(DipoleView d, Wave w, double2* __restrict__ inv) {
  __shared__ double2 T[PC_MAXD][2 * PC_MAXD + 1];  // augmented rows [block | identity]
  __shared__ int piv_row;
  __shared__ int singular;
  const int64_t b = blockIdx.x;
  const PcBlock p = pc_block(d, b);
  const int D = p.D, tid = threadIdx.x;
  if (tid == 0) singular = 0;
  for (int idx = tid; idx < PC_MAXD * (2 * PC_MAXD + 1); idx += 256)
    T[idx / (2 * PC_MAXD + 1)][idx % (2 * PC_MAXD + 1)] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int r = tid; r < D; r += 256) T[r][PC_MAXD + r] = make_double2(1.0, 0.0);
  // blocks of M: (row slot, column dipole) pairs
  const int nslots = p.nd + p.ne;
  for (int item = tid; item < nslots * p.nd; item += 256) {
    const int rs = item / p.nd, cj = item % p.nd;
    const int64_t jdip = p.d0 + cj;
    const int f = rs < p.nd ? 0 : 1;
    const int64_t dr = f == 0 ? p.d0 + rs : p.d0 + p.nd - p.ne + (rs - p.nd);
    const int ce = jdip >= d.nc ? (int)(jdip - (p.d0 + p.nd - p.ne)) : -1;  // local effective index of the column dipole
    if (jdip < d.nc) {
      double2 v[3][3];
      m_block<false>(d, w, dr, f, jdip, v);
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int a = 0; a < 3; ++a) T[3 * rs + a][3 * cj + c] = v[c][a];
    } else {
      double2 v[6][3];
      m_block<true>(d, w, dr, f, jdip, v);
#pragma unroll
      for (int c = 0; c < 6; ++c)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int col = c < 3 ? 3 * cj + c : 3 * (p.nd + ce) + (c - 3);
          T[3 * rs + a][col] = v[c][a];
        }
    }
  }
  __syncthreads();
  for (int k = 0; k < D; ++k) {
    if (tid < 64) {
      double best = -1.0;
      int br = k;
      for (int r = k + tid; r < D; r += 64) {
        const double m = fabs(T[r][k].x) + fabs(T[r][k].y);
        if (m > best) {
          best = m;
          br = r;
        }
      }
      // wave argmax (lowest row on ties)
      for (int off = 32; off >= 1; off >>= 1) {
        const double ob = __shfl_xor(best, off);
        const int orow = __shfl_xor(br, off);
        if (ob > best || (ob == best && orow < br)) {
          best = ob;
          br = orow;
        }
      }
      if (tid == 0) {
        piv_row = br;
        if (!(best > 0.0)) singular = 1;
      }
    }
    __syncthreads();
    if (singular) break;
    const int pr = piv_row;
    if (pr != k)
      for (int c = tid; c < 2 * PC_MAXD; c += 256) {
        const double2 t = T[k][c];
        T[k][c] = T[pr][c];
        T[pr][c] = t;
      }
    __syncthreads();
    const double2 pv = T[k][k];
    const double den = pv.x * pv.x + pv.y * pv.y;
    const double2 ip = make_double2(pv.x / den, -pv.y / den);
    __syncthreads();
    for (int c = tid; c < 2 * PC_MAXD; c += 256) T[k][c] = cmul(T[k][c], ip);
    __syncthreads();
    for (int idx = tid; idx < D * 2 * PC_MAXD; idx += 256) {
      const int r = idx / (2 * PC_MAXD), c = idx % (2 * PC_MAXD);
      if (r == k) continue;
      const double2 f = T[r][k];
      if (c == k) continue;  // column k of the other rows is cleared below
      T[r][c] = csub(T[r][c], cmul(f, T[k][c]));
    }
    __syncthreads();
    for (int r = tid; r < D; r += 256)
      if (r != k) T[r][k] = make_double2(0.0, 0.0);
    __syncthreads();
  }
  double2* o = inv + b * (int64_t)PC_MAXD * PC_MAXD;
  for (int idx = tid; idx < D * D; idx += 256) {
    const int r = idx % D, c = idx / D;
    const double2 v = singular ? make_double2(r == c ? 1.0 : 0.0, 0.0) : T[r][PC_MAXD + c];
    o[r + (int64_t)c * PC_MAXD] = v;
  }
}

// z = P v: one workgroup per (block, RHS); the block's unknowns of v gathered
// into LDS, multiplied by the block's inverse, scattered into z.
__global__ void __launch_bounds__(64) precond_apply_kernel(DipoleView d, const double2* __restrict__ inv, int64_t n,
                                                            const double2* __restrict__ v, double2* __restrict__ z) {
  __shared__ double2 vl[PC_MAXD];
  const int64_t b = blockIdx.x;
  const int64_t r = blockIdx.y;
  const PcBlock p = pc_block(d, b);
  const int tid = threadIdx.x;
  if (tid < p.D) vl[tid] = v[r * n + pc_unknown(d, p, tid)];
  __syncthreads();
  if (tid >= p.D) return;
  const double2* A = inv + b * (int64_t)PC_MAXD * PC_MAXD;
  double2 s = make_double2(0, 0);
  for (int c = 0; c < p.D; ++c) cfma(s, A[tid + (int64_t)c * PC_MAXD], vl[c]);
  z[r * n + pc_unknown(d, p, tid)] = s;
}

// ---------------------------------------------------------------------------
// Krylov vector kernels on [nrhs][n] arrays (basis vector i at V + i vs)
// ---------------------------------------------------------------------------
// h[i][r] = sum_k conj(V_i[r][k]) w[r][k]: one workgroup per (i, r), fixed order
__global__ void __launch_bounds__(256) mdot_kernel(const double2* __restrict__ V, int64_t vs,
                                                    const double2* __restrict__ w, int64_t n, int nrhs,
                                                    double2* __restrict__ h) {
  __shared__ double2 red[256];
  const int i = blockIdx.x, r = blockIdx.y;
  const double2* a = V + i * vs + (int64_t)r * n;
  const double2* b = w + (int64_t)r * n;
  double2 s = make_double2(0, 0);
  for (int64_t k = threadIdx.x; k < n; k += 256) {
    const double2 av = a[k], bv = b[k];
    s.x += av.x * bv.x + av.y * bv.y;
    s.y += av.x * bv.y - av.y * bv.x;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) h[(int64_t)i * nrhs + r] = red[0];
}

// out[r][k] = beta out[r][k] + sgn sum_{i < m} c[i][r] V_i[r][k]
__global__ void mcomb_kernel(const double2* __restrict__ V, int64_t vs, const double2* __restrict__ c, int m,
                             double sgn, double beta, double2* __restrict__ out, int64_t n, int nrhs) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nrhs * n) return;
  const int r = (int)(idx / n);
  double2 s = make_double2(0, 0);
  for (int i = 0; i < m; ++i) cfma(s, c[(int64_t)i * nrhs + r], V[i * vs + idx]);
  const double2 o = out[idx];
  out[idx] = make_double2(beta * o.x + sgn * s.x, beta * o.y + sgn * s.y);
}

// out[r] = ||w[r]||_2: one workgroup per r, fixed order
__global__ void __launch_bounds__(256) norm_kernel(const double2* __restrict__ w, int64_t n, double* __restrict__ out) {
  __shared__ double red[256];
  const int r = blockIdx.x;
  const double2* a = w + (int64_t)r * n;
  double s = 0;
  for (int64_t k = threadIdx.x; k < n; k += 256) s += a[k].x * a[k].x + a[k].y * a[k].y;
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[r] = sqrt(red[0]);
}

// v[r][k] = w[r][k] / s[r] (0 where s[r] = 0)
__global__ void scale_kernel(const double2* __restrict__ w, const double* __restrict__ s, double2* __restrict__ v,
                             int64_t n, int nrhs) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nrhs * n) return;
  const double sr = s[idx / n];
  const double f = sr > 0 ? 1.0 / sr : 0.0;
  v[idx] = cscale(w[idx], f);
}

// a[i] += b[i]
__global__ void add_kernel(double2* __restrict__ a, const double2* __restrict__ b, int64_t count) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count) a[idx] = cadd(a[idx], b[idx]);
}

// out[i] = a[i] - b[i]
__global__ void sub_kernel(const double2* __restrict__ a, const double2* __restrict__ b, double2* __restrict__ out,
                           int64_t count) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count) out[idx] = csub(a[idx], b[idx]);
}

__global__ void zero_kernel(double2* __restrict__ a, int64_t count) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count) a[idx] = make_double2(0.0, 0.0);
}

static unsigned nblocks(int64_t count) { return (unsigned)((count + 255) / 256); }

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
int coupling_num_splits(int64_t N, int num_cu) {
  const int64_t tblocks = (N + 255) / 256;
  int64_t want = (4 * (int64_t)num_cu + tblocks - 1) / tblocks;
  const int64_t maxs = (N + 31) / 32;
  want = std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(want, maxs), 64));
  const int64_t len = ((N + want - 1) / want + 31) / 32 * 32;
  return (int)((N + len - 1) / len);
}

size_t iter_workspace_bytes(int64_t N, int64_t n, int64_t nrhs, int restart, int num_cu) {
  IterWork w;
  iter_workspace_carve(nullptr, N, n, nrhs, restart, num_cu, w);
  return w.bytes;
}

void iter_workspace_carve(void* base, int64_t N, int64_t n, int64_t nrhs, int restart, int num_cu, IterWork& w) {
  char* p = static_cast<char*>(base);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* r = p ? p + off : nullptr;
    off += (bytes + 255) / 256 * 256;
    return r;
  };
  const size_t vec = (size_t)nrhs * n * sizeof(double2);
  w.nsplit = coupling_num_splits(N, num_cu);
  w.nblk = (N + PC_DIP - 1) / PC_DIP;
  w.V = reinterpret_cast<double2*>(take((size_t)(restart + 1) * vec));
  w.z = reinterpret_cast<double2*>(take(vec));
  w.q = reinterpret_cast<double2*>(take(vec));
  w.t = reinterpret_cast<double2*>(take(vec));
  w.part = reinterpret_cast<double2*>(take((size_t)w.nsplit * vec));
  w.inv = reinterpret_cast<double2*>(take((size_t)w.nblk * PC_MAXD * PC_MAXD * sizeof(double2)));
  w.h = reinterpret_cast<double2*>(take(2 * (size_t)(restart + 1) * nrhs * sizeof(double2)));
  w.nrm = reinterpret_cast<double*>(take(2 * (size_t)nrhs * sizeof(double)));
  w.y = reinterpret_cast<double2*>(take((size_t)(restart + 1) * nrhs * sizeof(double2)));
  w.bytes = off + 256;
}

hipError_t launch_precond_build(const DipoleView& d, const Wave& w, const IterWork& iw, hipStream_t st) {
  hipLaunchKernelGGL(precond_build_kernel, dim3((unsigned)iw.nblk), dim3(256), 0, st, d, w, iw.inv);
  return hipGetLastError();
}

// y = M x for nrhs vectors (x, y: [nrhs][n]; y may not alias x)
hipError_t launch_matvec(const DipoleView& d, const Wave& w, const IterWork& iw, int64_t n, int64_t nrhs,
                         const double2* x, double2* y, hipStream_t st) {
  hipError_t e = launch_apply_alpha(d, x, n, iw.q, n, nrhs, st);
  if (e != hipSuccess) return e;
  const int64_t jps = ((d.N + iw.nsplit - 1) / iw.nsplit + 31) / 32 * 32;
  const dim3 grid((unsigned)((d.N + 255) / 256), (unsigned)iw.nsplit);
  for (int r0 = 0; r0 < nrhs; r0 += 2) {
    if (nrhs - r0 >= 2)
      hipLaunchKernelGGL(coupling_kernel<2>, grid, dim3(256), 0, st, d, w, iw.q, n, nrhs, r0, jps, iw.part);
    else
      hipLaunchKernelGGL(coupling_kernel<1>, grid, dim3(256), 0, st, d, w, iw.q, n, nrhs, r0, jps, iw.part);
  }
  const int64_t count = nrhs * n;
  hipLaunchKernelGGL(coupling_finish_kernel, dim3(nblocks(count)), dim3(256), 0, st, iw.part, iw.nsplit, count, x,
                     iw.q, d.self_c, 3 * d.nc, n, y, count);
  return hipGetLastError();
}

hipError_t launch_precond_apply(const DipoleView& d, const IterWork& iw, int64_t n, int64_t nrhs, const double2* v,
                                double2* z, hipStream_t st) {
  hipLaunchKernelGGL(precond_apply_kernel, dim3((unsigned)iw.nblk, (unsigned)nrhs), dim3(64), 0, st, d, iw.inv, n, v,
                     z);
  return hipGetLastError();
}

hipError_t gmres_solve(const DipoleView& d, const Wave& w, const IterWork& iw, int64_t n, int64_t nrhs,
                       const double2* B, double2* X, double tol, int max_iter, int restart, hipStream_t st,
                       GmresStats& gs, Prof* prof) {
  typedef std::complex<double> cd;
  hipError_t e;
#define GCHK(x)                        \
  do {                                 \
    if ((e = (x)) != hipSuccess) return e; \
  } while (0)
  const int64_t vs = nrhs * n;
  const int64_t count = vs;
  const int m = restart;
  gs = GmresStats{};
  GCHK(launch_precond_build(d, w, iw, st));
  // ||b|| per column
  std::vector<double> bn(nrhs), rn(nrhs), hbuf;
  hipLaunchKernelGGL(norm_kernel, dim3((unsigned)nrhs), dim3(256), 0, st, B, n, iw.nrm);
  GCHK(hipMemcpyAsync(bn.data(), iw.nrm, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
  GCHK(hipStreamSynchronize(st));
  hipLaunchKernelGGL(zero_kernel, dim3(nblocks(count)), dim3(256), 0, st, X, count);
  std::vector<std::vector<cd>> H(nrhs), G(nrhs);
  std::vector<std::vector<cd>> cs(nrhs), sn(nrhs);
  std::vector<double> relres(nrhs, 1.0);
  bool first = true;
  while (true) {
    // r = b - M x (x = 0 at the start: r = b), V_0 = r / ||r||
    double2* V0 = iw.V;
    if (first) {
      GCHK(hipMemcpyAsync(V0, B, sizeof(double2) * count, hipMemcpyDeviceToDevice, st));
    } else {
      if (prof) GCHK(prof->begin(st, PROF_ITER_MATVEC, (double)d.N * (double)d.N * (double)nrhs));
      GCHK(launch_matvec(d, w, iw, n, nrhs, X, iw.t, st));
      if (prof) GCHK(prof->end(st));
      hipLaunchKernelGGL(sub_kernel, dim3(nblocks(count)), dim3(256), 0, st, B, iw.t, V0, count);  // V0 = b - M x
    }
    first = false;
    hipLaunchKernelGGL(norm_kernel, dim3((unsigned)nrhs), dim3(256), 0, st, V0, n, iw.nrm);
    GCHK(hipMemcpyAsync(rn.data(), iw.nrm, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
    GCHK(hipStreamSynchronize(st));
    bool done = true;
    for (int64_t r = 0; r < nrhs; ++r) {
      relres[r] = bn[r] > 0 ? rn[r] / bn[r] : 0.0;
      done = done && relres[r] <= tol;
    }
    gs.relres = *std::max_element(relres.begin(), relres.end());
    if (done || gs.iters >= max_iter) break;
    hipLaunchKernelGGL(scale_kernel, dim3(nblocks(count)), dim3(256), 0, st, V0, iw.nrm, V0, n, (int)nrhs);
    for (int64_t r = 0; r < nrhs; ++r) {
      H[r].assign((size_t)(m + 1) * m, cd(0, 0));
      G[r].assign(m + 1, cd(0, 0));
      G[r][0] = cd(rn[r], 0);
      cs[r].assign(m, cd(0, 0));
      sn[r].assign(m, cd(0, 0));
    }
    int jdone = 0;
    for (int j = 0; j < m && gs.iters < max_iter; ++j) {
      double2* Vj = iw.V + j * vs;
      double2* W = iw.V + (j + 1) * vs;
      // W = M P V_j
      GCHK(launch_precond_apply(d, iw, n, nrhs, Vj, iw.z, st));
      if (prof) GCHK(prof->begin(st, PROF_ITER_MATVEC, (double)d.N * (double)d.N * (double)nrhs));
      GCHK(launch_matvec(d, w, iw, n, nrhs, iw.z, W, st));
      if (prof) GCHK(prof->end(st));
      // classical Gram-Schmidt, twice: h = V^H W, W -= V h
      for (int pass = 0; pass < 2; ++pass) {
        double2* hp = iw.h + (size_t)pass * (m + 1) * nrhs;
        hipLaunchKernelGGL(mdot_kernel, dim3((unsigned)(j + 1), (unsigned)nrhs), dim3(256), 0, st, iw.V, vs, W, n,
                           (int)nrhs, hp);
        hipLaunchKernelGGL(mcomb_kernel, dim3(nblocks(count)), dim3(256), 0, st, iw.V, vs, hp, j + 1, -1.0, 1.0, W,
                           n, (int)nrhs);
      }
      hipLaunchKernelGGL(norm_kernel, dim3((unsigned)nrhs), dim3(256), 0, st, W, n, iw.nrm);
      hipLaunchKernelGGL(scale_kernel, dim3(nblocks(count)), dim3(256), 0, st, W, iw.nrm, W, n, (int)nrhs);
      hbuf.resize(2 * (size_t)(m + 1) * nrhs * 2 + nrhs);
      GCHK(hipMemcpyAsync(hbuf.data(), iw.h, sizeof(double2) * 2 * (m + 1) * nrhs, hipMemcpyDeviceToHost, st));
      GCHK(hipMemcpyAsync(hbuf.data() + 4 * (size_t)(m + 1) * nrhs, iw.nrm, sizeof(double) * nrhs,
                          hipMemcpyDeviceToHost, st));
      GCHK(hipStreamSynchronize(st));
      ++gs.iters;
      jdone = j + 1;
      bool all = true;
      for (int64_t r = 0; r < nrhs; ++r) {
        // Hessenberg column j: h of both passes, then ||W||
        std::vector<cd> col(j + 2);
        for (int i = 0; i <= j; ++i) {
          const size_t a = 2 * ((size_t)i * nrhs + r), b2 = 2 * ((size_t)(m + 1) * nrhs + (size_t)i * nrhs + r);
          col[i] = cd(hbuf[a] + hbuf[b2], hbuf[a + 1] + hbuf[b2 + 1]);
        }
        col[j + 1] = cd(hbuf[4 * (size_t)(m + 1) * nrhs + r], 0);
        // earlier rotations
        for (int i = 0; i < j; ++i) {
          const cd t0 = cs[r][i] * col[i] + sn[r][i] * col[i + 1];
          const cd t1 = -std::conj(sn[r][i]) * col[i] + std::conj(cs[r][i]) * col[i + 1];
          col[i] = t0;
          col[i + 1] = t1;
        }
        // new rotation zeroing col[j + 1]
        const double a = std::abs(col[j]), bb = std::abs(col[j + 1]);
        if (bb == 0.0) {
          cs[r][j] = cd(1, 0);
          sn[r][j] = cd(0, 0);
        } else {
          const double den = std::hypot(a, bb);
          const cd ph = a > 0 ? col[j] / a : cd(1, 0);
          cs[r][j] = cd(a / den, 0);
          sn[r][j] = ph * std::conj(col[j + 1]) / den;
          col[j] = ph * den;
          col[j + 1] = cd(0, 0);
        }
        for (int i = 0; i <= j; ++i) H[r][(size_t)i * m + j] = col[i];
        const cd g0 = G[r][j];
        G[r][j] = cs[r][j] * g0;
        G[r][j + 1] = -std::conj(sn[r][j]) * g0;
        relres[r] = bn[r] > 0 ? std::abs(G[r][j + 1]) / bn[r] : 0.0;
        all = all && relres[r] <= 0.5 * tol;
      }
      if (all) break;
    }
    // y = H^-1 g (upper triangular, jdone x jdone), then x += P V y
    std::vector<double2> yh((size_t)(m + 1) * nrhs, make_double2(0, 0));
    for (int64_t r = 0; r < nrhs; ++r) {
      std::vector<cd> y(jdone);
      for (int i = jdone - 1; i >= 0; --i) {
        cd s = G[r][i];
        for (int k = i + 1; k < jdone; ++k) s -= H[r][(size_t)i * m + k] * y[k];
        const cd hd = H[r][(size_t)i * m + i];
        y[i] = hd != cd(0, 0) ? s / hd : cd(0, 0);
      }
      for (int i = 0; i < jdone; ++i) yh[(size_t)i * nrhs + r] = make_double2(y[i].real(), y[i].imag());
    }
    GCHK(hipMemcpyAsync(iw.y, yh.data(), sizeof(double2) * (size_t)jdone * nrhs, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(mcomb_kernel, dim3(nblocks(count)), dim3(256), 0, st, iw.V, vs, iw.y, jdone, 1.0, 0.0, iw.t, n,
                       (int)nrhs);
    GCHK(launch_precond_apply(d, iw, n, nrhs, iw.t, iw.z, st));
    hipLaunchKernelGGL(add_kernel, dim3(nblocks(count)), dim3(256), 0, st, X, iw.z, count);
    GCHK(hipGetLastError());
    ++gs.cycles;
  }
  return hipGetLastError();
#undef GCHK
}

}  // namespace gdm
