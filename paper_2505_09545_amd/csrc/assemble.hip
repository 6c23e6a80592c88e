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
// Memory layout: column-major, interleaved complex, leading dimension ld.  A
// workgroup owns 256 consecutive row slots (768 consecutive rows) of one column
// dipole; each thread evaluates its 3 x 3 (or 3 x 6) block in FP64 in
// registers, then every column of the workgroup's strip (768 values) is staged
// in LDS and written with consecutive lanes on consecutive elements, so each
// store instruction covers one contiguous span (full cache lines).  With both
// outputs the FP64 evaluation is shared by the complex-double and the
// complex-float matrix.  Columns of GPM group members are finished by
// launch_gpm_columns (gpm.hip).
#include "gdm_common.hpp"
#include "gdm_kernels.hpp"
#include "gdm_misc.hpp"

namespace gdm {

// One strip: column dipole j (an effective dipole iff EFF: 6 columns, else 3)
// and row slots [s0, s0 + 256).  All block indices are compile-time so the
// block stays in registers.
template <bool EFF, bool W64, bool W32>
__device__ inline void assemble_strip(const DipoleView& d, const Wave& w, double2* __restrict__ M64,
                                      float2* __restrict__ M32, int64_t ld, int64_t j, int64_t s0, double2* stage) {
  constexpr int NC = EFF ? 6 : 3;
  const int tid = threadIdx.x;
  const int64_t s = s0 + tid;
  const int64_t N = d.N, nc = d.nc, slots = N + d.ne;
  const bool live = s < slots;
  const int f = s < N ? 0 : 1;                    // field type of the row slot: E or H
  const int64_t dr = f == 0 ? s : nc + (s - N);   // row dipole
  double2 v[NC][3];  // v[column][row a] of this thread's block
  if (live) {
    m_block<EFF>(d, w, dr, f, j, v);
  } else {
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int a = 0; a < 3; ++a) v[c][a] = make_double2(0.0, 0.0);
  }
  // write the strip column by column through LDS (coalesced stores)
  const int64_t row0 = 3 * s0;
  const int nrows = (int)(3 * ((slots - s0) < 256 ? (slots - s0) : 256));
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int64_t col = c < 3 ? 3 * j + c : 3 * (N + j - nc) + (c - 3);
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 3; ++a) stage[3 * tid + a] = v[c][a];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int t = tid + 256 * i;
      if (t < nrows) {
        const double2 x = stage[t];
        if (W64) M64[row0 + t + col * ld] = x;
        if (W32) M32[row0 + t + col * ld] = make_float2((float)x.x, (float)x.y);
      }
    }
  }
}

// Column dipoles j0 + blockIdx.x / row_blocks, all cells (EFF false) or all
// effective dipoles (EFF true): one launch per column type.
template <bool EFF, bool W64, bool W32>
__global__ void __launch_bounds__(256) assemble_kernel(DipoleView d, Wave w, double2* __restrict__ M64,
                                                        float2* __restrict__ M32, int64_t ld, int64_t row_blocks,
                                                        int64_t j0) {
  __shared__ double2 stage[768];
  const int64_t j = j0 + blockIdx.x / row_blocks;  // column dipole (uniform in the block)
  const int64_t s0 = (blockIdx.x % row_blocks) * 256;
  assemble_strip<EFF, W64, W32>(d, w, M64, M32, ld, j, s0, stage);
}

template <bool W64, bool W32>
static void launch_assemble_cols(const DipoleView& d, const Wave& w, double2* M64, float2* M32, int64_t ld,
                                 int64_t row_blocks, hipStream_t st) {
  if (d.nc > 0)
    hipLaunchKernelGGL((assemble_kernel<false, W64, W32>), dim3((unsigned)(row_blocks * d.nc)), dim3(256), 0, st, d, w,
                       M64, M32, ld, row_blocks, (int64_t)0);
  if (d.ne > 0)
    hipLaunchKernelGGL((assemble_kernel<true, W64, W32>), dim3((unsigned)(row_blocks * d.ne)), dim3(256), 0, st, d, w,
                       M64, M32, ld, row_blocks, d.nc);
}

static hipError_t launch_assemble_impl(const DipoleView& d, const Wave& w, double2* M64, float2* M32, int64_t ld,
                                       hipStream_t st) {
  const int64_t slots = d.N + d.ne;
  if (slots == 0) return hipSuccess;
  const int64_t row_blocks = (slots + 255) / 256;
  const int64_t blocks = row_blocks * d.N;
  if (blocks > (int64_t)UINT32_MAX) return hipErrorInvalidValue;
  if (M64 && M32) launch_assemble_cols<true, true>(d, w, M64, M32, ld, row_blocks, st);
  else if (M64) launch_assemble_cols<true, false>(d, w, M64, M32, ld, row_blocks, st);
  else launch_assemble_cols<false, true>(d, w, M64, M32, ld, row_blocks, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_gpm_columns(d, M64, M32, ld, 3 * slots, st);  // no-op without GPM groups
}

template <typename T>
hipError_t launch_assemble(const DipoleView& d, const Wave& w, void* M, int64_t ld, hipStream_t st) {
  if (sizeof(T) == 8) return launch_assemble_impl(d, w, static_cast<double2*>(M), nullptr, ld, st);
  return launch_assemble_impl(d, w, nullptr, static_cast<float2*>(M), ld, st);
}

hipError_t launch_assemble_dual(const DipoleView& d, const Wave& w, double2* M64, float2* M32, int64_t ld,
                                hipStream_t st) {
  return launch_assemble_impl(d, w, M64, M32, ld, st);
}

template hipError_t launch_assemble<double>(const DipoleView&, const Wave&, void*, int64_t, hipStream_t);
template hipError_t launch_assemble<float>(const DipoleView&, const Wave&, void*, int64_t, hipStream_t);

}  // namespace gdm
