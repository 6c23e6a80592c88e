// Step (c) of the hot path: scattered fields at probe points by re-propagation
// of the dipole moments,  F_sca(r_p) = sum_j G(r_p, r_j) q_j  (arXiv:2505.09545,
// Sec. "Observables", first item, with the dyad of Eq. superprop_G), evaluated
// matrix-free in FP64: the 6x6 dyad of every (probe, dipole) pair is recomputed
// in registers (one sincos per pair) and never stored.
//
// Work decomposition: one thread per probe and RHS chunk; the dipoles are
// swept in tiles of 256 staged in LDS (position + moments), so each dipole is
// read from HBM once per workgroup.  When there are few probes the dipole sum is
// split over several workgroups (down to 32 dipoles each) that write FP64
// partial sums, reduced in a fixed order by a second kernel (deterministic
// result).
//
// Moment layout q[r][u] (u = unknown index): p of dipole d at u = 3d..3d+2 for
// all N dipoles, m of effective dipole e at u = 3N + 3e.  Output E, H [nrhs][P][3].
#include "gdm_common.hpp"
#include "gdm_kernels.hpp"
#include "gdm_misc.hpp"

namespace gdm {

constexpr int FT = 256;  // dipoles per LDS tile

template <int NR>
__global__ void __launch_bounds__(256) fields_kernel(DipoleView d, Wave w, const double2* __restrict__ q, int64_t ldq,
                                                      int64_t nrhs, int r0, const double* __restrict__ rp, int64_t P,
                                                      int64_t j_per_split, double2* __restrict__ outE,
                                                      double2* __restrict__ outH, int64_t split_stride,
                                                      double min_r2, int* __restrict__ flag) {
  __shared__ double spos[FT][3];
  __shared__ double2 sp[FT][NR][3];
  __shared__ double2 sm[FT][NR][3];
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int split = blockIdx.y;
  const int64_t j0 = split * j_per_split;
  const int64_t j1 = j0 + j_per_split < d.N ? j0 + j_per_split : d.N;
  const bool live = p < P;
  double x = 0, y = 0, z = 0;
  if (live) {
    x = rp[3 * p];
    y = rp[3 * p + 1];
    z = rp[3 * p + 2];
  }
  double2 E[NR][3], H[NR][3];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      E[r][a] = make_double2(0, 0);
      H[r][a] = make_double2(0, 0);
    }
  const int64_t N = d.N, nc = d.nc;
  for (int64_t t0 = j0; t0 < j1; t0 += FT) {
    const int nt = (int)(j1 - t0 < FT ? j1 - t0 : FT);
    __syncthreads();
    // a thread's loads all issued before its LDS stores (the position array is
    // reached through a generic pointer, which the compiler must assume may
    // point into LDS: interleaved, each load would wait before the next store)
    for (int t = threadIdx.x; t < nt; t += 256) {
      const int64_t j = t0 + t;
      double pv[3];
      double2 qv[NR][3], mv[NR][3];
#pragma unroll
      for (int a = 0; a < 3; ++a) pv[a] = d.pos[3 * j + a];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const bool rv = r0 + r < nrhs;
        const double2* qc = q + (int64_t)(r0 + r) * ldq;
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
      const double Rx = x - spos[t][0], Ry = y - spos[t][1], Rz = z - spos[t][2];
      const double R2 = Rx * Rx + Ry * Ry + Rz * Rz;
      if (R2 < min_r2) {
        atomicOr(flag, 1);
        continue;
      }
      Green g;
      green_eh(Rx, Ry, Rz, w, true, g);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const double2 px = sp[t][r][0], py = sp[t][r][1], pz = sp[t][r][2];
        // E += G^Ep p
        cfma(E[r][0], g.e[0], px); cfma(E[r][0], g.e[3], py); cfma(E[r][0], g.e[4], pz);
        cfma(E[r][1], g.e[3], px); cfma(E[r][1], g.e[1], py); cfma(E[r][1], g.e[5], pz);
        cfma(E[r][2], g.e[4], px); cfma(E[r][2], g.e[5], py); cfma(E[r][2], g.e[2], pz);
        // H += h x p
        cfma(H[r][0], g.h[1], pz); cfma(H[r][0], cscale(g.h[2], -1.0), py);
        cfma(H[r][1], g.h[2], px); cfma(H[r][1], cscale(g.h[0], -1.0), pz);
        cfma(H[r][2], g.h[0], py); cfma(H[r][2], cscale(g.h[1], -1.0), px);
      }
      if (t >= ncell_in_tile) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const double2 mx = sm[t][r][0], my = sm[t][r][1], mz = sm[t][r][2];
          // E += G^Em m = -(h x m)
          cfma(E[r][0], cscale(g.h[1], -1.0), mz); cfma(E[r][0], g.h[2], my);
          cfma(E[r][1], cscale(g.h[2], -1.0), mx); cfma(E[r][1], g.h[0], mz);
          cfma(E[r][2], cscale(g.h[0], -1.0), my); cfma(E[r][2], g.h[1], mx);
          // H += eps G^Ep m
          double2 t0v = make_double2(0, 0), t1v = make_double2(0, 0), t2v = make_double2(0, 0);
          cfma(t0v, g.e[0], mx); cfma(t0v, g.e[3], my); cfma(t0v, g.e[4], mz);
          cfma(t1v, g.e[3], mx); cfma(t1v, g.e[1], my); cfma(t1v, g.e[5], mz);
          cfma(t2v, g.e[4], mx); cfma(t2v, g.e[5], my); cfma(t2v, g.e[2], mz);
          H[r][0] = cadd(H[r][0], cscale(t0v, w.eps_env));
          H[r][1] = cadd(H[r][1], cscale(t1v, w.eps_env));
          H[r][2] = cadd(H[r][2], cscale(t2v, w.eps_env));
        }
      }
    }
  }
  if (!live) return;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r0 + r >= nrhs) break;
    double2* oe = outE + split * split_stride + ((int64_t)(r0 + r) * P + p) * 3;
#pragma unroll
    for (int a = 0; a < 3; ++a) oe[a] = E[r][a];
    if (outH) {
      double2* oh = outH + split * split_stride + ((int64_t)(r0 + r) * P + p) * 3;
#pragma unroll
      for (int a = 0; a < 3; ++a) oh[a] = H[r][a];
    }
  }
}

__global__ void reduce_splits_kernel(const double2* __restrict__ part, int nsplit, int64_t stride,
                                     double2* __restrict__ out, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  double2 s = part[i];
  for (int k = 1; k < nsplit; ++k) s = cadd(s, part[k * stride + i]);
  out[i] = s;
}

// Dipoles per split: a multiple of SPLIT_GRAIN (a split may be smaller than one
// LDS tile, so that a launch with few probes still spreads over every CU).
constexpr int SPLIT_GRAIN = 32;

static int64_t fields_split_len(int64_t N, int nsplit) {
  return ((N + nsplit - 1) / nsplit + SPLIT_GRAIN - 1) / SPLIT_GRAIN * SPLIT_GRAIN;
}

// Number of dipole splits of a launch: enough workgroups for four per CU, at
// most 64 partial sums per output, and no empty split.
int fields_num_splits(int64_t P, int64_t N, int num_cu) {
  const int64_t pblocks = (P + 255) / 256;
  int64_t want = (4 * (int64_t)num_cu + pblocks - 1) / pblocks;
  const int64_t maxs = (N + SPLIT_GRAIN - 1) / SPLIT_GRAIN;
  if (want > maxs) want = maxs;
  if (want < 1) want = 1;
  if (want > 64) want = 64;
  const int64_t len = fields_split_len(N, (int)want);
  return (int)((N + len - 1) / len);
}

// Scratch bytes launch_fields needs for nsplit > 1 (partial sums of E, and of H if wanted).
size_t fields_scratch_bytes(int64_t nrhs, int64_t P, int nsplit, bool want_h) {
  if (nsplit <= 1) return 0;
  return sizeof(double2) * (want_h ? 2 : 1) * (size_t)nsplit * (size_t)nrhs * (size_t)P * 3;
}

hipError_t launch_fields(const DipoleView& d, const Wave& w, const double2* q, int64_t ldq, int64_t nrhs,
                         const double* rp, int64_t P, double2* E, double2* H, double2* scratch, int nsplit,
                         double min_r2, int* flag, hipStream_t st) {
  if (P <= 0 || nrhs <= 0) return hipSuccess;
  const int64_t count = nrhs * P * 3;
  const int64_t jps = fields_split_len(d.N, nsplit);
  double2* oE = nsplit > 1 ? scratch : E;
  double2* oH = nsplit > 1 ? (H ? scratch + nsplit * count : nullptr) : H;
  const dim3 grid((unsigned)((P + 255) / 256), (unsigned)nsplit);
  for (int r0 = 0; r0 < nrhs; r0 += 2) {
    if (nrhs - r0 >= 2)
      hipLaunchKernelGGL(fields_kernel<2>, grid, dim3(256), 0, st, d, w, q, ldq, nrhs, r0, rp, P, jps, oE, oH, count,
                         min_r2, flag);
    else
      hipLaunchKernelGGL(fields_kernel<1>, grid, dim3(256), 0, st, d, w, q, ldq, nrhs, r0, rp, P, jps, oE, oH, count,
                         min_r2, flag);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (nsplit > 1) {
    const unsigned nb = (unsigned)((count + 255) / 256);
    hipLaunchKernelGGL(reduce_splits_kernel, dim3(nb), dim3(256), 0, st, oE, nsplit, count, E, count);
    if (H) hipLaunchKernelGGL(reduce_splits_kernel, dim3(nb), dim3(256), 0, st, oH, nsplit, count, H, count);
  }
  return hipGetLastError();
}

}  // namespace gdm
