// Launch declarations of the small kernels (incident field, polarisation,
// cross sections, refinement helpers, probe fields).
#pragma once
#include "gdm_common.hpp"
#include "gdm_kernels.hpp"

namespace gdm {

// alpha_c[i] = (eps[i] - eps_env) d^3 / (4 pi)
hipError_t launch_cell_alpha(const double2* eps, int64_t nc, double eps_env, double step, double2* alpha,
                             hipStream_t st);

// F0 at the dipoles in the unknown layout, [n_pw][n] (ld n): plane wave
// E0 = e0 exp(i k khat.r), H0 = n_env khat x E0.
hipError_t launch_incident(const DipoleView& d, const Wave& w, double n_env, int64_t n_pw, const double* khat,
                           const double2* e0, double2* f0, int64_t n, hipStream_t st);

// Plane wave at arbitrary points: E, H [n_pw][P][3] (H nullable); accumulate:
// added to E, H instead of written.
hipError_t launch_planewave_points(const Wave& w, double n_env, int64_t n_pw, const double* khat, const double2* e0,
                                   const double* r, int64_t P, double2* E, double2* H, hipStream_t st,
                                   bool accumulate = false);
// out[r] = |e0[r]|^2 for n_pw plane-wave amplitudes e0 [n_pw][3]
hipError_t launch_pw_intensity(int64_t n_pw, const double2* e0, double* out, hipStream_t st);

// q = A F in the unknown layout (cells: alpha F; effective: alpha6 (E, H)).
hipError_t launch_apply_alpha(const DipoleView& d, const double2* F, int64_t ldf, double2* q, int64_t ldq,
                              int64_t nrhs, hipStream_t st);

// Five FP64 sums per RHS: Im(F0^* q), Im(F^* q), sum |q|^2 over cell E,
// effective E and effective H unknowns.
hipError_t launch_cs_sums(const DipoleView& d, const double2* f0, const double2* q, const double2* f, int64_t n,
                          int64_t nrhs, double* sums5, hipStream_t st);

// sum_{i != j} q_i^H G6_ij q_j per RHS (partial sums per workgroup, [nrhs][nblk]).
hipError_t launch_sca_ff(const DipoleView& d, const Wave& w, const double2* q, int64_t ldq, int64_t nrhs,
                         double* partial, int64_t nblk, hipStream_t st);
int64_t sca_ff_blocks(int64_t N);

// conversions and refinement helpers
hipError_t launch_convert_d2f(const double2* a, int64_t lda, float2* b, int64_t ldb, int64_t m, int64_t n,
                              hipStream_t st);
hipError_t launch_convert_f2d(const float2* a, int64_t lda, double2* b, int64_t ldb, int64_t m, int64_t n,
                              hipStream_t st);
hipError_t launch_copy_d(const double2* a, int64_t lda, double2* b, int64_t ldb, int64_t m, int64_t n, hipStream_t st);
// x += c (c in float), and per-column max |c| into cmax[col]
hipError_t launch_axpy_f2d(const float2* c, int64_t ldc, double2* x, int64_t ldx, int64_t m, int64_t n,
                           double* cmax, hipStream_t st);
// per-column max |a| (modulus)
hipError_t launch_colmax(const double2* a, int64_t lda, int64_t m, int64_t n, double* out, hipStream_t st);
// row sums of |M| (infinity norm = max row sum), out[m] (zeroed by the kernel driver)
hipError_t launch_rowsum_abs(const double2* M, int64_t ld, int64_t n, double* rows, hipStream_t st);
// column sums of |M| (1-norm = max column sum), out[n]
hipError_t launch_colsum_abs(const double2* M, int64_t ld, int64_t n, double* cols, hipStream_t st);

// Point dipole sources (sources.hip): F0 [n_src][n] of sources d [n_src][6]
// (p, m) at rs [n_src][3]; a source within sqrt(min_r2) of a dipole sets *flag.
hipError_t launch_dipole_sources(const DipoleView& d, const Wave& w, int64_t n, int64_t n_src, const double* rs,
                                 const double2* ds, double2* f0, double min_r2, int* flag, hipStream_t st);
// LDOS out [n_src][2][3] from the moments q [6 n_src][n] of the unit sources
// (RHS 6 s + c: component c of (p, m) at rs[s]).
hipError_t launch_ldos(const DipoleView& d, const Wave& w, const double2* q, int64_t n, int64_t n_src,
                       const double* rs, double* out, hipStream_t st);
// G [n_src][P][6][6] from the fields E, H [6 n_src][P][3] of the unit sources.
hipError_t launch_green_gather(const double2* E, const double2* H, int64_t n_src, int64_t P, double2* G,
                               hipStream_t st);

// Exact multipoles (multipole.hip): moments [nrhs][24] and cross sections
// [nrhs][8] (either may be null) of the first nc dipoles (the cells) of q.
int multipole_num_splits(int64_t nc, int num_cu, int64_t nrhs);
size_t multipole_scratch_bytes(int64_t nrhs, int nsplit);
hipError_t launch_multipoles(const double* pos, int64_t nc, const double2* q, int64_t n, int64_t nrhs,
                             const double r0[3], double k, double k0, double n_env, const double* khat,
                             const double2* e0, int nsplit, double* part, double2* moments, double* sigma,
                             hipStream_t st);

// Effective dipole pair (effective.hip): F0 [N][6] = (E0, H0) at r0 of n_pw
// plane waves then n_src point sources; least squares alpha [6][6] (row-major,
// (p, m) = alpha (E0, H0)) from the moments [N][24]; B [N][6] work array.
hipError_t launch_pair_extract(const Wave& w, double n_env, const double r0[3], int64_t n_pw, const double* khat,
                               const double2* e0, int64_t n_src, const double* rs, const double2* ds,
                               const double2* moments, double2* F0, double2* B, double2* alpha, double* resid,
                               hipStream_t st);

// (E0, H0) at the point (x, y, z) of illumination i: plane wave i (khat,
// e0 [n_pw][3]) when i < n_pw, else the point source s = i - n_pw, whose field
// there is G6(r - rs[s]) ds[s] (ds [n_src][6] = (p, m)).
__device__ inline void illumination_at(const Wave& w, double n_env, double x, double y, double z, int64_t i,
                                       int64_t n_pw, const double* khat, const double2* e0, const double* rs,
                                       const double2* ds, double2 (&o)[6]) {
  if (i < n_pw) {
    const double kx = khat[3 * i], ky = khat[3 * i + 1], kz = khat[3 * i + 2];
    double sn, cs;
    sincos(w.k * (kx * x + ky * y + kz * z), &sn, &cs);
    double2 E[3];
    for (int a = 0; a < 3; ++a) {
      const double2 v = e0[3 * i + a];
      E[a] = make_double2(v.x * cs - v.y * sn, v.x * sn + v.y * cs);
      o[a] = E[a];
    }
    const double kk[3] = {kx, ky, kz};
    for (int a = 0; a < 3; ++a) {
      const int b = (a + 1) % 3, c = (a + 2) % 3;
      o[3 + a] = make_double2(n_env * (kk[b] * E[c].x - kk[c] * E[b].x), n_env * (kk[b] * E[c].y - kk[c] * E[b].y));
    }
    return;
  }
  const int64_t s = i - n_pw;
  Green g;
  green_eh(x - rs[3 * s], y - rs[3 * s + 1], z - rs[3 * s + 2], w, true, g);
  const double2* d = ds + 6 * s;
  for (int r = 0; r < 6; ++r) {
    double2 acc = make_double2(0.0, 0.0);
    for (int c = 0; c < 6; ++c) cfma(acc, g6(g, w.eps_env, r, c), d[c]);
    o[r] = acc;
  }
}

// Global polarisability matrices (gpm.hip).  All use the groups of the
// DipoleView (gtab, galpha on the device) and do nothing without groups.
// Columns of the group members in M (FP64 and/or FP32 copy, ld): from
// M' = I - G~ (members' alpha taken as I, no intra-group coupling) to
// I - G~ alpha_G, in place; the FP64 copy is the source when both are given.
hipError_t launch_gpm_columns(const DipoleView& d, double2* M64, float2* M32, int64_t ld, int64_t n, hipStream_t st);
// q[members] = alpha_G F[members] for every group (q != F).
hipError_t launch_gpm_apply(const DipoleView& d, const double2* F, int64_t ldf, double2* q, int64_t ldq, int64_t nrhs,
                            hipStream_t st);
// out [nrhs][ngroups] = Im sum_{i != j in g} q_i^H G6(r_i - r_j) q_j
hipError_t launch_gpm_mutual(const DipoleView& d, const Wave& w, const double2* q, int64_t ldq, int64_t nrhs,
                             double* out, hipStream_t st);
// Extraction by scattered-field matching:
// Y [nrhs][6P] (column-major 6P x nrhs) from E, H [nrhs][P][3];
hipError_t launch_gpm_pack_fields(const double2* E, const double2* H, int64_t nrhs, int64_t P, double2* Y,
                                  hipStream_t st);
// Gf (6P x 6M, column-major): rows (probe, E then H component), columns
// (pair, p then m): G6(r_p - r_j);
hipError_t launch_gpm_fit_matrix(const Wave& w, const double* rp, int64_t P, const double* rg, int64_t M,
                                 double2* Gf, hipStream_t st);
// F0g (N x 6M, column-major): (E0, H0) of illumination i at pair j;
hipError_t launch_gpm_illumination(const Wave& w, double n_env, const double* rg, int64_t M, int64_t n_pw,
                                   const double* khat, const double2* e0, int64_t n_src, const double* rs,
                                   const double2* ds, double2* F0g, hipStream_t st);
// B (n x m, column-major) = A^T for A (m x n, column-major);
hipError_t launch_transpose(const double2* A, int64_t m, int64_t n, double2* B, hipStream_t st);
// least squares min ||A X - B|| by Householder QR (A m x K, B m x R, both
// column-major and overwritten; m >= K): X (K x R, column-major, ldx K),
// NaN where the diagonal of R falls below 1e-12 of its largest entry;
// norms [2][R] = (|B_r|^2 before, |residual_r|^2); rdiag [K] work array.
hipError_t launch_qr_lsq(double2* A, int64_t m, int K, double2* B, int R, double2* X, double2* rdiag, double* norms,
                         hipStream_t st);

int fields_num_splits(int64_t P, int64_t N, int num_cu);
size_t fields_scratch_bytes(int64_t nrhs, int64_t P, int nsplit, bool want_h);
hipError_t launch_fields(const DipoleView& d, const Wave& w, const double2* q, int64_t ldq, int64_t nrhs,
                         const double* rp, int64_t P, double2* E, double2* H, double2* scratch, int nsplit,
                         double min_r2, int* flag, hipStream_t st);

}  // namespace gdm
