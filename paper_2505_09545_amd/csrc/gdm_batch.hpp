// Launch declarations of the batched spectra kernels (batch.hip).  A group is
// B items (wavelengths) of one structure of N cells, n = 3N; matrices of item z
// at M + z n^2, vectors at [z][n_pw][n], per-item scalars at [z].
#pragma once
#include "gdm_common.hpp"
#include "gdm_kernels.hpp"

namespace gdm {

// alpha[z], k0[z] of the group starting at wavelength l0 of structure s
hipError_t launch_batch_stage(const double2* eps, int64_t n_wl, int64_t s, int64_t l0, int64_t nvalid, int B,
                              const double* wl, double eps_env, double step, double2* alpha, double* k0,
                              hipStream_t st);
// M64 (and M32 if not null) = I - G~ A of every item
hipError_t launch_batch_assemble(const double* pos, int64_t N, const double2* alpha, const double* k0s, double n_env,
                                 double step, int radiative, double2* M64, float2* M32, int B, hipStream_t st);
hipError_t launch_batch_incident(const double* pos, int64_t n, const double* k0s, double n_env, int64_t npw,
                                 const double* khat, const double2* e0, double2* f0, int B, hipStream_t st);
hipError_t launch_batch_apply_alpha(const double2* alpha, const double2* F, double2* q, int64_t n, int64_t npw, int B,
                                    hipStream_t st);
// minf[z] = |M_z|_inf (rows: [B][n] scratch)
hipError_t launch_batch_minf(const double2* M, int64_t n, int B, double* rows, double* minf, hipStream_t st);
hipError_t launch_batch_be(const double* rmax, const double* xmax, const double* bmax, const double* minf,
                           int64_t npw, int B, double* be, hipStream_t st);
hipError_t launch_batch_cs(const double* sums5, const double* k0s, double n_env, const double2* e0, int64_t npw, int B,
                           double* out, hipStream_t st);
hipError_t launch_batch_unstage(const double* cs, const double* be, int64_t nvalid, int64_t npw, int64_t base,
                                double* cs_out, double* be_out, hipStream_t st);
hipError_t launch_batch_err(const int32_t* err, int32_t* sticky, hipStream_t st);
// speculative panels: per-item failure flags of a group, and the list of failed
// global item indices (count[0] entries, at most cap stored)
hipError_t launch_batch_spec_collect(const int32_t* flags, int64_t sflag, int nblk, int B, int32_t* failed,
                                     hipStream_t st);
hipError_t launch_batch_spec_list(const int32_t* failed, int64_t nvalid, int64_t base, int64_t* list, int32_t* count,
                                  int64_t cap, hipStream_t st);
hipError_t launch_batch_err_init(int32_t* sticky, hipStream_t st);
// be_max[0] = max(be_max[0], be[0..nvalid))
hipError_t launch_batch_bemax(const double* be, int64_t nvalid, double* be_max, hipStream_t st);

}  // namespace gdm
