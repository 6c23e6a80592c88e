// Launch declarations of the adjoint (reverse-mode) kernels.
#pragma once
#include "gdm_common.hpp"
#include "gdm_kernels.hpp"

namespace gdm {

// Work decomposition helpers (the host sizes the partial-sum buffers with them).
int adjoint_probe_splits(int64_t P, int64_t N, int num_cu);
int adjoint_pair_splits(int64_t N, int num_cu);
int64_t adjoint_probe_blocks(int64_t N);
int64_t adjoint_pair_blocks(int64_t N);
int64_t adjoint_finish_blocks(int64_t N);
int64_t adjoint_einc_blocks(int64_t P, int64_t nrhs);
int adjoint_rhs_chunks(int64_t nrhs);

// Cr[r] = 4 pi k0 / (n_env |e0_r|^2)
hipError_t launch_adjoint_cr(const Wave& w, double n_env, const double2* e0, int64_t nrhs, double* Cr,
                             hipStream_t st);
// Probe back-propagation: pacc [nsplit][nrhs][n], pgr [chunks*nsplit][N][3],
// pdk [chunks*nsplit][probe_blocks].
hipError_t launch_adjoint_probe(const DipoleView& d, const Wave& w, double n_env, const double2* q, int64_t n,
                                int64_t nrhs, const double* rp, const double2* gE, int64_t P, int nsplit,
                                double2* pacc, double* pgr, double* pdk, double min_r2, int* flag, hipStream_t st);
// gqe = g_q + sum pacc, rhs = g_F + A^T gqe   ([nrhs][n] each)
hipError_t launch_adjoint_seed(const DipoleView& d, const Wave& w, const double2* f0, const double2* f,
                               const double2* q, int64_t n, int64_t nrhs, const double* Cr, const double* gsig,
                               const double2* pacc, int nsplit, double2* gqe, double2* rhs, hipStream_t st);
// Pair terms: pgr [chunks*nsplit][N][3], pv [nsplit][nrhs][nc][3], pdk [chunks*nsplit][pair_blocks].
hipError_t launch_adjoint_pair(const DipoleView& d, const Wave& w, double n_env, const double2* lam,
                               const double2* q, int64_t n, int64_t nrhs, int nsplit, double* pgr, double2* pv,
                               double* pdk, hipStream_t st);
// Gradients w.r.t. positions and cell permittivities; pdk [finish_blocks].
hipError_t launch_adjoint_finish(const DipoleView& d, const Wave& w, double n_env, double step, int radiative,
                                 const double2* f0, const double2* f, const double2* q, const double2* lam,
                                 const double2* gqe, int64_t n, int64_t nrhs, const double* khat, const double* Cr,
                                 const double* gsig, const double* pgr_probe, int nslot_probe, const double* pgr_pair,
                                 int nslot_pair, const double2* pv, int nsplit_pair, double* grad_r,
                                 double* grad_eps, double* pdk, hipStream_t st);
// Incident field at the probes (wavelength term); pdk [einc_blocks].
hipError_t launch_adjoint_einc(const Wave& w, double n_env, const double* khat, const double2* e0, const double* rp,
                               const double2* gE, int64_t P, int64_t nrhs, double* pdk, hipStream_t st);
// grad_wl[0] from all partials and the explicit k0 dependence of the cross sections.
hipError_t launch_adjoint_wl(const Wave& w, double wavelength, const double* parts, int64_t nparts,
                             const double* sums5, const double* Cr, const double* gsig, int64_t nrhs, double* grad_wl,
                             hipStream_t st);

}  // namespace gdm
