// Launch declarations of the matrix-free iterative solver (iterative.hip).
#pragma once
#include "gdm_common.hpp"
#include "gdm_kernels.hpp"

namespace gdm {

constexpr int PC_DIP = 8;                // dipoles per block of the block-Jacobi preconditioner
constexpr int PC_MAXD = 6 * PC_DIP;      // unknowns of a block (all effective: E and H)

// Device workspace of one solve; sized by iter_workspace_bytes().
struct IterWork {
  double2* V;     // [restart + 1][nrhs][n] Krylov basis
  double2* z;     // [nrhs][n] preconditioned vector
  double2* q;     // [nrhs][n] moments A z of the product
  double2* t;     // [nrhs][n] scratch
  double2* part;  // [nsplit][nrhs][n] partial coupling sums
  double2* inv;   // [nblk][PC_MAXD][PC_MAXD] block inverses (column-major)
  double2* h;     // [2][restart + 1][nrhs] Gram-Schmidt coefficients of the two passes
  double* nrm;    // [2][nrhs] norms
  double2* y;     // [restart + 1][nrhs] least-squares solution of a cycle
  int nsplit = 1;
  int64_t nblk = 0;
  size_t bytes = 0;
};

struct GmresStats {
  int iters = 0;         // Krylov iterations (matrix-vector products with M P)
  int cycles = 0;        // restarts completed
  double relres = 1.0;   // max over RHS of ||b - M x|| / ||b|| at the last true residual
};

int coupling_num_splits(int64_t N, int num_cu);
size_t iter_workspace_bytes(int64_t N, int64_t n, int64_t nrhs, int restart, int num_cu);
void iter_workspace_carve(void* base, int64_t N, int64_t n, int64_t nrhs, int restart, int num_cu, IterWork& w);
hipError_t launch_precond_build(const DipoleView& d, const Wave& w, const IterWork& iw, hipStream_t st);
hipError_t launch_precond_apply(const DipoleView& d, const IterWork& iw, int64_t n, int64_t nrhs, const double2* v,
                                double2* z, hipStream_t st);
// y = M x, matrix-free (x, y [nrhs][n], distinct)
hipError_t launch_matvec(const DipoleView& d, const Wave& w, const IterWork& iw, int64_t n, int64_t nrhs,
                         const double2* x, double2* y, hipStream_t st);
// Restarted GMRES(restart) on M X = B, right block-Jacobi preconditioning, X
// from zero, until ||b - M x|| / ||b|| <= tol for every column (true residual
// at a restart) or max_iter iterations.
hipError_t gmres_solve(const DipoleView& d, const Wave& w, const IterWork& iw, int64_t n, int64_t nrhs,
                       const double2* B, double2* X, double tol, int max_iter, int restart, hipStream_t st,
                       GmresStats& gs, Prof* prof);

}  // namespace gdm
