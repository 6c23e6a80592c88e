// Step (a) of the hot path: assembly of the dense coupling matrix
//   M = I - G~ A
// of the discretised Lippmann-Schwinger system (arXiv:2505.09545, Eq.
// LPS_6by6_discrete written as Eq. GDM_system_of_equations), with electric and
// magnetic unknowns separated and the magnetic unknowns of mesh cells removed
// (Sec. "Hybrid discretization GDM", Fig. coupling_matrix).
//
// Unknown layout: "row slot" s in [0, N + ne) owns rows 3s..3s+2.  Slots
// s < N are the electric field of dipole s (cells first, then effective
// dipoles); slots s >= N are the magnetic field of effective dipole s - N.
// Column dipole j owns columns 3j..3j+2 (its electric field) and, if it is an
// effective dipole, columns 3(N + j - nc).. (its magnetic field).
//
// G~_ij = G(r_i, r_j) for i != j and the self-term S_i on the diagonal: the
// cubic-cell S^Ep = -4 pi / (3 eps_env d^3) I (Eq. selfterm_SEp_cubic), zero
// for effective point dipoles.  All arithmetic in FP64 (one sincos per pair);
// the value is rounded to the storage type only at the store.
//
// Memory layout: column-major, interleaved complex, leading dimension ld.  Each
// thread owns one row slot of one column dipole, so the 3 complex rows it
// writes per column sit next to those of its neighbours (coalesced stream).
#include "gdm_common.hpp"
#include "gdm_kernels.hpp"

namespace gdm {

template <typename T>
__global__ void __launch_bounds__(256) assemble_kernel(DipoleView d, Wave w, cplx<T>* __restrict__ M,
                                                        int64_t ld, int64_t row_blocks) {
  const int64_t j = blockIdx.x / row_blocks;  // column dipole (uniform in the block)
  const int64_t s = (blockIdx.x % row_blocks) * blockDim.x + threadIdx.x;
  const int64_t N = d.N, nc = d.nc;
  if (s >= N + d.ne) return;
  const int f = s < N ? 0 : 1;                 // field type of the row slot: E or H
  const int64_t dr = f == 0 ? s : nc + (s - N);  // row dipole
  const bool col_eff = j >= nc;
  const int64_t row0 = 3 * s;
  cplx<T>* colE = M + row0 + (3 * j) * ld;
  if (dr == j) {
    // diagonal block I - S alpha (cells: scalar S^Ep and alpha; effective: S = 0)
    if (!col_eff) {
      const double2 v = csub(make_double2(1.0, 0.0), cmul(d.self_c, d.alpha_c[j]));
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int a = 0; a < 3; ++a) colE[a + c * ld] = to_c<T>(a == c ? v : make_double2(0.0, 0.0));
    } else {
      cplx<T>* colH = M + row0 + (3 * (N + j - nc)) * ld;
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          colE[a + c * ld] = to_c<T>(make_double2((f == 0 && a == c) ? 1.0 : 0.0, 0.0));
          colH[a + c * ld] = to_c<T>(make_double2((f == 1 && a == c) ? 1.0 : 0.0, 0.0));
        }
    }
    return;
  }
  const double Rx = d.pos[3 * dr + 0] - d.pos[3 * j + 0];
  const double Ry = d.pos[3 * dr + 1] - d.pos[3 * j + 1];
  const double Rz = d.pos[3 * dr + 2] - d.pos[3 * j + 2];
  Green g;
  green_eh(Rx, Ry, Rz, w, f == 1 || col_eff, g);
  if (!col_eff) {
    // -G^{f p} alpha_j : 3 x 3
    const double2 al = d.alpha_c[j];
    const double2 ma = make_double2(-al.x, -al.y);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double2 gv = f == 0 ? gep(g, a, c) : ghp(g, a, c);
        colE[a + c * ld] = to_c<T>(cmul(gv, ma));
      }
  } else {
    // -[G^{f p} G^{f m}] alpha6_j : 3 x 6
    const double2* al = d.alpha6 + (j - nc) * 36;
    cplx<T>* colH = M + row0 + (3 * (N + j - nc)) * ld;
    double2 gr[3][6];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 6; ++b) gr[a][b] = g6(g, w.eps_env, 3 * f + a, b);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      double2 acc[3] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
#pragma unroll
      for (int b = 0; b < 6; ++b) {
        const double2 ab = al[b * 6 + c];
#pragma unroll
        for (int a = 0; a < 3; ++a) cfma(acc[a], gr[a][b], ab);
      }
      cplx<T>* col = c < 3 ? colE + c * ld : colH + (c - 3) * ld;
#pragma unroll
      for (int a = 0; a < 3; ++a) col[a] = to_c<T>(make_double2(-acc[a].x, -acc[a].y));
    }
  }
}

template <typename T>
hipError_t launch_assemble(const DipoleView& d, const Wave& w, void* M, int64_t ld, hipStream_t st) {
  const int64_t slots = d.N + d.ne;
  if (slots == 0) return hipSuccess;
  const int64_t row_blocks = (slots + 255) / 256;
  const int64_t blocks = row_blocks * d.N;
  hipLaunchKernelGGL(assemble_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, st, d, w,
                     static_cast<cplx<T>*>(M), ld, row_blocks);
  return hipGetLastError();
}

template hipError_t launch_assemble<double>(const DipoleView&, const Wave&, void*, int64_t, hipStream_t);
template hipError_t launch_assemble<float>(const DipoleView&, const Wave&, void*, int64_t, hipStream_t);

}  // namespace gdm
