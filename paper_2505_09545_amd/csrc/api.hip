// C-ABI of libgdm (declared in include/gdm.h): context, device buffers, argument
// validation and the host drivers that chain the kernels of the hot path.
#include <algorithm>
#include <functional>
#include <map>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/gdm.h"
#include "gdm_common.hpp"
#include "gdm_kernels.hpp"
#include "gdm_misc.hpp"
#include "gdm_adjoint.hpp"
#include "gdm_batch.hpp"
#include "gdm_iterative.hpp"

using namespace gdm;

namespace {

// Device bytes held by one context's buffers, and the caller's limit on them
// (gdm_set_memory_limit; 0: none).
struct MemAccount {
  size_t used = 0;
  size_t limit = 0;
};

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  MemAccount* acct = nullptr;  // the owning context's account (null: not counted)
  hipError_t ensure(size_t bytes) {
    if (bytes <= cap && p) return hipSuccess;
    if (bytes == 0) bytes = 256;
    // the limit counts what the context would hold after the call
    if (acct && acct->limit > 0 && acct->used - cap + bytes > acct->limit) return hipErrorOutOfMemory;
    if (p) {
      hipError_t e = hipFree(p);
      if (e != hipSuccess) return e;
      if (acct) acct->used -= cap;
      p = nullptr;
      cap = 0;
    }
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      return e;
    }
    cap = bytes;
    if (acct) acct->used += cap;
    return hipSuccess;
  }
  void release() {
    if (p) (void)hipFree(p);
    if (p && acct) acct->used -= cap;
    p = nullptr;
    cap = 0;
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

__global__ void fill_i32_kernel(int* a, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

}  // namespace

struct gdm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t side = nullptr;  // look-ahead stream of the factorisation (default priority)
  bool own_stream = false;
  int num_cu = 256;
  int lds_bytes = 160 * 1024;
  std::string err = "";
  double n_env = 1.0;
  // structure
  int64_t nc = 0, ne = 0, N = 0, n = 0;
  double step = 0.0;
  gdm_selfterm self_mode = GDM_SELF_STATIC;
  DevBuf pos, eps, alpha_c, alpha6;
  // global polarisability matrices (gdm_set_gpm): group of each effective
  // dipole (-1 local), table (first, size, offset) and the matrices
  DevBuf gpm_gid, gpm_tab, gpm_alpha;
  int64_t n_gpm = 0;
  // factorisation state
  double wavelength = 0.0;
  bool factored = false;
  gdm_precision prec = GDM_PREC_FP64;
  DevBuf M, M64, ipiv, luws, rows;
  LUPlan plan;
  int64_t ld = 0;
  double Minf = 0.0;
  double M1 = -1.0;  // 1-norm of the FP64 matrix, computed on first transposed refinement
  // standalone getrf state
  LUPlan ext_plan;
  int ext_dtype = -1;
  DevBuf ext_ws;
  // solve / fields scratch
  DevBuf X, Rr, C32, small, scratch, flag;
  DevBuf Lam, adj;  // adjoint field and adjoint workspace
  DevBuf part;      // split-k partial sums of the small-RHS refinement residual
  DevBuf iter;      // workspace of gdm_solve_iterative
  DevBuf src;       // unit point sources of gdm_ldos / gdm_green_tensor: positions, moments, F0, q, fields
  // batched spectra: workspaces and the measured batch configuration per size class
  DevBuf bM64, bM32, bipiv, bws, bvec, bpart, bsmall, bpos, bwl;
  std::map<int64_t, std::pair<int, int>> batch_tune;  // n / 256 -> (items per group, nb)
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t sev[2] = {nullptr, nullptr};  // ordering only: the residual's side-stream part
  float ms_assemble = 0, ms_factor = 0;
  Prof prof;
  bool lookahead = true;
  std::vector<hipEvent_t> lu_events;
  int pivot_pb = 0;  // panel columns per pivot exchange (gdm_set_pivoting; 0: the library default)
  int64_t pivot_fallbacks = 0;         // speculative factorisations repeated with the pivot search
  int32_t spec_first_failed_block = -1;  // of the last such repetition
  MemAccount mem;    // device bytes of the buffers below and the caller's limit
  std::vector<DevBuf*> buffers() {
    return {&pos, &eps,  &alpha_c, &alpha6, &M,     &M64,  &ipiv,  &luws, &rows,   &ext_ws, &X,   &Rr,   &C32, &small,
            &scratch, &flag, &Lam,  &adj,   &part, &bM64, &bM32, &bipiv, &bws, &bvec, &bpart, &bsmall, &bpos, &bwl, &iter, &src,
            &gpm_gid, &gpm_tab, &gpm_alpha};
  }
};

#define FAIL(ctx, code, ...)                                     \
  do {                                                           \
    char _b[512];                                                \
    snprintf(_b, sizeof(_b), __VA_ARGS__);                       \
    (ctx)->err = _b;                                             \
    return code;                                                 \
  } while (0)

#define HIPCHK(ctx, expr)                                                                                   \
  do {                                                                                                      \
    hipError_t _e = (expr);                                                                                 \
    if (_e != hipSuccess) {                                                                                 \
      if (_e == hipErrorOutOfMemory || _e == hipErrorMemoryAllocation)                                      \
        FAIL(ctx, GDM_E_OOM, "device allocation failed in %s: %s", #expr, hipGetErrorString(_e));           \
      FAIL(ctx, GDM_E_DEVICE, "HIP error in %s: %s", #expr, hipGetErrorString(_e));                         \
    }                                                                                                       \
  } while (0)

static DipoleView view_of(const gdm_ctx* c, double2 self_c) {
  DipoleView d;
  d.pos = c->pos.as<double>();
  d.alpha_c = c->alpha_c.as<double2>();
  d.alpha6 = c->alpha6.as<double2>();
  d.N = c->N;
  d.nc = c->nc;
  d.ne = c->ne;
  d.self_c = self_c;
  if (c->n_gpm > 0) {
    d.gid = c->gpm_gid.as<int32_t>();
    d.gtab = c->gpm_tab.as<int64_t>();
    d.galpha = c->gpm_alpha.as<double2>();
    d.ngroups = c->n_gpm;
  }
  return d;
}

static Wave wave_of(const gdm_ctx* c, double wl) {
  Wave w;
  w.k0 = 2.0 * M_PI / wl;
  w.k = c->n_env * w.k0;
  w.eps_env = c->n_env * c->n_env;
  return w;
}

static double2 self_term(const gdm_ctx* c, const Wave& w) {
  const double eps = w.eps_env;
  double2 s = make_double2(-4.0 * M_PI / (3.0 * eps * c->step * c->step * c->step), 0.0);
  if (c->self_mode == GDM_SELF_RADIATIVE) s.y = (2.0 / 3.0) * w.k * w.k * w.k / eps;
  return s;
}

static gdm_status prepare_alpha(gdm_ctx* c) {
  HIPCHK(c, launch_cell_alpha(c->eps.as<double2>(), c->nc, c->n_env * c->n_env, c->step, c->alpha_c.as<double2>(),
                              c->stream));
  return GDM_OK;
}

static gdm_status check_wavelength(gdm_ctx* c, double wl) {
  if (!(wl > 0.0) || !std::isfinite(wl)) FAIL(c, GDM_E_ARG, "wavelength must be finite and > 0 (got %g)", wl);
  if (c->N == 0) FAIL(c, GDM_E_STATE, "no structure set");
  return GDM_OK;
}

// Panel columns per pivot exchange of the next factorisations: the caller's
// choice (gdm_set_pivoting), else partial pivoting.  Measured at n = 12 000
// (FP32+IR step, panels beside the look-ahead update): 5.14 us per column with
// partial pivoting, 7.1-7.9 with tournaments over 2, 4 or 8 columns.
// Panel mode of a factorisation (lu_plan's pb): by default speculative panels
// (0) where the caller can rebuild the matrix after a failed check, else the
// pivot search in every column (1); otherwise what gdm_set_pivoting chose.
static int panel_pb(const gdm_ctx* c, bool can_rebuild) {
  return c->pivot_pb > 0 ? c->pivot_pb : (can_rebuild ? 0 : 1);
}

// rebuild (may be null): writes the matrix into A again, so that a speculative
// factorisation whose check failed can be repeated with the pivot search.
template <typename T>
static gdm_status run_lu(gdm_ctx* c, void* A, int64_t n, int64_t ld, LUPlan& plan, DevBuf& ws, DevBuf& ipiv,
                         int32_t* ipiv_out, gdm_info* info, const std::function<hipError_t()>& rebuild = nullptr) {
  plan = lu_plan(n, (int)sizeof(T), c->num_cu, c->lds_bytes, 1, 128, panel_pb(c, (bool)rebuild));
  const size_t wsb = lu_workspace_bytes(plan, (int)sizeof(T), c->num_cu);
  HIPCHK(c, ws.ensure(wsb));
  LUWork w;
  lu_workspace_carve(ws.p, plan, (int)sizeof(T), c->num_cu, w);
  w.events = &c->lu_events;
  int32_t* piv = ipiv_out;
  if (!piv) {
    HIPCHK(c, ipiv.ensure(sizeof(int32_t) * n));
    piv = ipiv.as<int32_t>();
  }
  HIPCHK(c, lu_factor<T>(A, ld, plan, w, piv, c->stream, &c->prof, c->lookahead ? c->side : nullptr));
  int32_t err[2] = {0, 0};
  HIPCHK(c, hipMemcpyAsync(err, w.err, sizeof(err), hipMemcpyDeviceToHost, c->stream));
  std::vector<int32_t> flags;
  if (plan.spec) {
    flags.resize(plan.blocks.size());
    HIPCHK(c, hipMemcpyAsync(flags.data(), w.spec, sizeof(int32_t) * flags.size(), hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->prof.collect();
  const auto failed = std::find_if(flags.begin(), flags.end(), [](int32_t f) { return f != 0; });
  if (failed != flags.end()) {
    // a diagonal pivot is not partial pivoting's: again, with the pivot search
    c->spec_first_failed_block = (int32_t)(failed - flags.begin());
    ++c->pivot_fallbacks;
    HIPCHK(c, rebuild());
    plan.spec = false;
    HIPCHK(c, lu_factor<T>(A, ld, plan, w, piv, c->stream, &c->prof, c->lookahead ? c->side : nullptr));
    HIPCHK(c, hipMemcpyAsync(err, w.err, sizeof(err), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->prof.collect();
  }
  if (info) info->bad_index = -1;
  if (err[0] != 0) FAIL(c, GDM_E_DEVICE, "LU panel barrier timed out (workgroups not co-resident?)");
  if (err[1] != INT32_MAX) {
    if (info) info->bad_index = err[1];
    FAIL(c, GDM_E_SINGULAR, "exactly zero pivot in column %d", err[1]);
  }
  return GDM_OK;
}


struct SolveStats {
  int iters = 0;
  double be = 0.0;
  double tol = 0.0;
  float ms_ir = 0.f;
};

// X = op(M)^{-1} B for nrhs columns (op = M for trans 0, M^T for trans 1) with
// the context's factors.  FP64 factors: one solve.  FP32 factors: FP64
// iterative refinement on the stored FP64 matrix until the normwise backward
// error |r|_inf / (|op(M)|_inf |x|_inf + |b|_inf) of every column is <= tol, or
// stagnation, or max_iter corrections (GDM_E_NOCONV, best iterate kept in X).
static gdm_status solve_core(gdm_ctx* c, int trans, int64_t nrhs, const double2* B, double2* X, double tol,
                             int32_t max_iter, SolveStats& ss) {
  const int64_t n = c->n;
  LUWork w;
  const int eb = c->prec == GDM_PREC_FP64 ? 8 : 4;
  lu_workspace_carve(c->luws.p, c->plan, eb, c->num_cu, w);
  const double solve_flops = 8.0 * (double)n * (double)n * (double)nrhs;
  gdm_status status = GDM_OK;
  if (c->prec == GDM_PREC_FP64) {
    HIPCHK(c, launch_copy_d(B, n, X, n, n, nrhs, c->stream));
    HIPCHK(c, c->prof.begin(c->stream, PROF_SOLVE, solve_flops));
    HIPCHK(c, lu_solve<double>(trans, c->M.p, c->ld, c->plan, w, X, n, nrhs, c->stream));
    HIPCHK(c, c->prof.end(c->stream));
    return GDM_OK;
  }
  if (tol <= 0) tol = 1e-14;
  if (max_iter < 0) max_iter = 10;
  ss.tol = tol;
  double Mnorm = c->Minf;
  if (trans) {
    if (c->M1 < 0) {
      HIPCHK(c, c->rows.ensure(sizeof(double) * n));
      HIPCHK(c, launch_colsum_abs(c->M64.as<double2>(), n, n, c->rows.as<double>(), c->stream));
      std::vector<double> cols(n);
      HIPCHK(c, hipMemcpyAsync(cols.data(), c->rows.p, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      c->M1 = *std::max_element(cols.begin(), cols.end());
    }
    Mnorm = c->M1;
  }
  HIPCHK(c, c->Rr.ensure(sizeof(double2) * n * nrhs));
  HIPCHK(c, c->C32.ensure(sizeof(float2) * n * nrhs));
  HIPCHK(c, c->small.ensure(sizeof(double) * 4 * nrhs));
  double2* Rr = c->Rr.as<double2>();
  float2* C32 = c->C32.as<float2>();
  double* sm = c->small.as<double>();  // [0..nrhs): |r|, [nrhs..2nrhs): |x|, [2nrhs..): |b|, [3nrhs..): |c|
  int64_t part_elems = 0;
  struct {
    int64_t kc = 0, gemm_part = 0;
  } rs;
  if (nrhs <= SKINNY_MAX_RHS) {
    part_elems = std::max(skinny_t_chunks(n, 0) * nrhs * n, skinny_n_long_parts(n, n, nrhs));
  } else if (!trans) {
    // k split of the residual product: about 4 workgroups per CU in total
    const int64_t rem = nrhs % 64 <= SKINNY_MAX_RHS ? nrhs % 64 : 0;
    const int64_t nfull = nrhs - rem;
    const int64_t tiles = ((n + 63) / 64) * ((nfull + 63) / 64);
    int64_t splits = tiles > 0 ? (4 * (int64_t)c->num_cu + tiles - 1) / tiles : 1;
    splits = std::max<int64_t>(1, std::min<int64_t>(splits, 32));
    rs.kc = std::max<int64_t>(64, ((n + splits - 1) / splits + 7) / 8 * 8);
    const int64_t nchunk = n / rs.kc + (n % rs.kc > 0);
    rs.gemm_part = nchunk * n * nfull;
    part_elems = rs.gemm_part + (rem > 0 ? skinny_n_long_parts(n, n, rem) : 0);
  }
  if (part_elems > 0) HIPCHK(c, c->part.ensure(sizeof(double2) * part_elems));
  // first solve from B in FP32
  HIPCHK(c, launch_convert_d2f(B, n, C32, n, n, nrhs, c->stream));
  HIPCHK(c, c->prof.begin(c->stream, PROF_SOLVE, solve_flops));
  HIPCHK(c, lu_solve<float>(trans, c->M.p, c->ld, c->plan, w, C32, n, nrhs, c->stream));
  HIPCHK(c, c->prof.end(c->stream));
  HIPCHK(c, launch_convert_f2d(C32, n, X, n, n, nrhs, c->stream));
  HIPCHK(c, launch_colmax(B, n, n, nrhs, sm + 2 * nrhs, c->stream));
  HIPCHK(c, hipEventRecord(c->ev[1], c->stream));
  std::vector<double> h(4 * nrhs);
  std::vector<double> prev_c(nrhs, INFINITY);
  for (int it = 0;; ++it) {
    // r = b - op(M) x  (FP64, stored FP64 matrix)
    HIPCHK(c, launch_copy_d(B, n, Rr, n, n, nrhs, c->stream));
    HIPCHK(c, c->prof.begin(c->stream, PROF_RESID, solve_flops));
    if (nrhs <= SKINNY_MAX_RHS) {
      // few right-hand sides: a GEMV-shaped residual streams M64 once on the VALUs
      if (trans)
        HIPCHK(c, launch_skinny_t<double>(n, nrhs, c->M64.p, n, X, n, n, nullptr, 0, nullptr, 0, 0, 0, c->part.p,
                                          part_elems, Rr, n, c->stream));
      else
        HIPCHK(c, launch_skinny_n_long<double>(n, n, c->M64.p, n, X, n, Rr, n, nrhs, c->part.p, part_elems,
                                               c->stream));
    } else if (trans) {
      HIPCHK(c, launch_gemm<double>(0, trans, n, nrhs, n, c->M64.p, n, X, n, Rr, n, c->stream));
    } else {
      // Whole 64-column tiles on the matrix cores, split over k into independent
      // products (enough workgroups to fill the chip) whose partial sums are
      // added in order; a remainder of <= 8 columns streams M64 once more on
      // the VALUs instead of occupying a nearly empty tile.
      const int64_t rem = nrhs % 64 <= SKINNY_MAX_RHS ? nrhs % 64 : 0;
      const int64_t nfull = nrhs - rem;
      // The remainder (HBM-bound) runs on the side stream while the matrix
      // cores run the 64-column tiles: the two write disjoint columns of Rr and
      // disjoint parts of the partial-sum buffer.
      const bool rem_side = rem > 0 && nfull > 0 && c->side && c->sev[0] && c->sev[1];
      if (rem_side) {
        HIPCHK(c, hipEventRecord(c->sev[0], c->stream));  // x and the copy of b in Rr are ready
        HIPCHK(c, hipStreamWaitEvent(c->side, c->sev[0], 0));
        HIPCHK(c, launch_skinny_n_long<double>(n, n, c->M64.p, n, X + nfull * n, n, Rr + nfull * n, n, rem,
                                               c->part.as<double2>() + rs.gemm_part, part_elems - rs.gemm_part,
                                               c->side));
        HIPCHK(c, hipEventRecord(c->sev[1], c->side));
      }
      if (nfull > 0) {
        const int64_t kc = rs.kc, nk = n / kc, tail = n - nk * kc;
        double2* part = c->part.as<double2>();
        HIPCHK(c, launch_gemm_product_3m<double>(n, nfull, kc, c->M64.p, n, X, n, part, n, c->stream, (int)nk,
                                                 kc * n, kc, n * nfull));
        if (tail > 0)
          HIPCHK(c, launch_gemm_product_3m<double>(n, nfull, tail, c->M64.as<double2>() + nk * kc * n, n, X + nk * kc,
                                                   n, part + nk * n * nfull, n, c->stream));
        HIPCHK(c, launch_partial_reduce<double>(part, (int)(nk + (tail > 0)), n, nfull, Rr, n, c->stream));
      }
      if (rem > 0 && !rem_side)
        HIPCHK(c, launch_skinny_n_long<double>(n, n, c->M64.p, n, X + nfull * n, n, Rr + nfull * n, n, rem,
                                               c->part.as<double2>() + rs.gemm_part, part_elems - rs.gemm_part,
                                               c->stream));
      if (rem_side) HIPCHK(c, hipStreamWaitEvent(c->stream, c->sev[1], 0));
    }
    HIPCHK(c, c->prof.end(c->stream));
    HIPCHK(c, launch_colmax(Rr, n, n, nrhs, sm, c->stream));
    HIPCHK(c, launch_colmax(X, n, n, nrhs, sm + nrhs, c->stream));
    HIPCHK(c, hipMemcpyAsync(h.data(), sm, sizeof(double) * 4 * nrhs, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double be_max = 0.0;
    for (int64_t r = 0; r < nrhs; ++r) {
      const double den = Mnorm * h[nrhs + r] + h[2 * nrhs + r];
      const double be = den > 0 ? h[r] / den : 0.0;
      be_max = std::max(be_max, be);
    }
    ss.be = be_max;
    if (be_max <= tol) break;
    if (it >= max_iter) {
      status = GDM_E_NOCONV;
      break;
    }
    if (it > 0) {
      bool stagnated = true;
      for (int64_t r = 0; r < nrhs; ++r)
        if (!(h[3 * nrhs + r] > 0.5 * prev_c[r])) stagnated = false;
      if (stagnated) {
        status = GDM_E_NOCONV;
        break;
      }
      for (int64_t r = 0; r < nrhs; ++r) prev_c[r] = h[3 * nrhs + r];
    }
    HIPCHK(c, launch_convert_d2f(Rr, n, C32, n, n, nrhs, c->stream));
    HIPCHK(c, c->prof.begin(c->stream, PROF_SOLVE, solve_flops));
    HIPCHK(c, lu_solve<float>(trans, c->M.p, c->ld, c->plan, w, C32, n, nrhs, c->stream));
    HIPCHK(c, c->prof.end(c->stream));
    HIPCHK(c, launch_axpy_f2d(C32, n, X, n, n, nrhs, sm + 3 * nrhs, c->stream));
    ++ss.iters;
  }
  HIPCHK(c, hipEventRecord(c->ev[2], c->stream));
  HIPCHK(c, hipEventSynchronize(c->ev[2]));
  (void)hipEventElapsedTime(&ss.ms_ir, c->ev[1], c->ev[2]);
  return status;
}


// ---------------------------------------------------------------------------
// batched spectra
// ---------------------------------------------------------------------------
namespace {

struct BatchShape {
  int64_t n = 0;
  int B = 0;
  int nb = 0;
  LUPlan plan;
};

// Device views of the batched workspaces (pointers fixed for the whole call, so
// that a captured group graph can be replayed for every group of the same shape).
struct BatchBufs {
  double2* M64;
  float2* M32;
  int32_t* ipiv;
  void* ws;
  double2 *F0, *X, *R, *Q;
  float2* C32;
  void* part;
  int64_t part_elems;
  double *rmax, *xmax, *bmax, *cmax, *minf, *rows, *sums5, *k0, *cs, *be, *be_max;
  double2* alpha;
  int32_t* sticky;
  int32_t* sfail;   // [B] speculative panels: item failed its pivot checks
  int32_t* scount;  // failed items listed so far
  int64_t* slist;   // their global indices (structure * n_wl + wavelength)
  double* pos;
  double* wl;
};

int64_t batch_part_elems(int64_t n, int B, int64_t npw) {
  return npw <= SKINNY_MAX_RHS ? (int64_t)B * skinny_n_long_parts(n, n, npw) : 0;
}

}  // namespace

static bool batch_shape_for(gdm_ctx* c, int64_t n, int B, int nb_max, bool ir, BatchShape& sh) {
  const int eb = ir ? 4 : 8;
  sh.n = n;
  sh.B = B;
  sh.plan = lu_plan(n, eb, c->num_cu, c->lds_bytes, B, nb_max, panel_pb(c, true));
  sh.nb = sh.plan.nb;
  return sh.plan.nb >= 32 && lu_plan_fits(sh.plan) && sh.plan.max_wg * B <= c->num_cu;
}

static size_t batch_item_bytes(int64_t n, bool ir) { return (size_t)n * n * (ir ? 24 : 16); }

// Enqueue the whole pipeline of one group on c->stream (captured into a graph by
// the caller): assembly, LU, incident field, solve with a fixed number of FP64
// refinement corrections and the backward error, q = alpha F, cross sections.
static gdm_status batch_enqueue_group(gdm_ctx* c, const BatchShape& sh, const BatchBufs& b, int64_t npw,
                                      const double* khat, const double2* e0, bool ir, int ir_iters, int radiative,
                                      double step) {
  const int64_t n = sh.n, N = n / 3, nn = n * n, sv = npw * n;
  const int B = sh.B;
  const int64_t cols = (int64_t)B * npw;
  hipStream_t st = c->stream;
  LUWork w;
  lu_workspace_carve(b.ws, sh.plan, ir ? 4 : 8, c->num_cu, w, B);
  w.events = &c->lu_events;
  HIPCHK(c, launch_batch_assemble(b.pos, N, b.alpha, b.k0, c->n_env, step, radiative, b.M64, ir ? b.M32 : nullptr, B,
                                  st));
  if (ir) HIPCHK(c, launch_batch_minf(b.M64, n, B, b.rows, b.minf, st));
  if (ir)
    HIPCHK(c, lu_factor<float>(b.M32, n, sh.plan, w, b.ipiv, st, nullptr, c->lookahead ? c->side : nullptr, nn, n));
  else
    HIPCHK(c, lu_factor<double>(b.M64, n, sh.plan, w, b.ipiv, st, nullptr, c->lookahead ? c->side : nullptr, nn, n));
  HIPCHK(c, launch_batch_err(w.err, b.sticky, st));
  if (sh.plan.spec)
    HIPCHK(c, launch_batch_spec_collect(w.spec, w.s_npairs, (int)sh.plan.blocks.size(), B, b.sfail, st));
  HIPCHK(c, launch_batch_incident(b.pos, n, b.k0, c->n_env, npw, khat, e0, b.F0, B, st));
  auto residual = [&]() -> hipError_t {
    // R = F0 - M X per item (FP64, stored FP64 matrix)
    hipError_t e = launch_copy_d(b.F0, n, b.R, n, n, cols, st);
    if (e != hipSuccess) return e;
    if (npw <= SKINNY_MAX_RHS)
      return launch_skinny_n_long<double>(n, n, b.M64, n, b.X, n, b.R, n, npw, b.part, b.part_elems, st, B, nn, sv, sv);
    return launch_gemm<double>(0, 0, n, npw, n, b.M64, n, b.X, n, b.R, n, st, GemmMask{}, B, nn, sv, sv);
  };
  if (!ir) {
    HIPCHK(c, launch_copy_d(b.F0, n, b.X, n, n, cols, st));
    HIPCHK(c, lu_solve<double>(0, b.M64, n, sh.plan, w, b.X, n, npw, st, nn, sv));
  } else {
    HIPCHK(c, launch_convert_d2f(b.F0, n, b.C32, n, n, cols, st));
    HIPCHK(c, lu_solve<float>(0, b.M32, n, sh.plan, w, b.C32, n, npw, st, nn, sv));
    HIPCHK(c, launch_convert_f2d(b.C32, n, b.X, n, n, cols, st));
    for (int it = 0; it < ir_iters; ++it) {
      HIPCHK(c, residual());
      HIPCHK(c, launch_convert_d2f(b.R, n, b.C32, n, n, cols, st));
      HIPCHK(c, lu_solve<float>(0, b.M32, n, sh.plan, w, b.C32, n, npw, st, nn, sv));
      HIPCHK(c, launch_axpy_f2d(b.C32, n, b.X, n, n, cols, b.cmax, st));
    }
    HIPCHK(c, residual());
    HIPCHK(c, launch_colmax(b.R, n, n, cols, b.rmax, st));
    HIPCHK(c, launch_colmax(b.X, n, n, cols, b.xmax, st));
    HIPCHK(c, launch_colmax(b.F0, n, n, cols, b.bmax, st));
    HIPCHK(c, launch_batch_be(b.rmax, b.xmax, b.bmax, b.minf, npw, B, b.be, st));
  }
  HIPCHK(c, launch_batch_apply_alpha(b.alpha, b.X, b.Q, n, npw, B, st));
  DipoleView d{};
  d.pos = b.pos;
  d.N = N;
  d.nc = N;
  d.ne = 0;
  HIPCHK(c, launch_cs_sums(d, b.F0, b.Q, b.X, n, cols, b.sums5, st));
  HIPCHK(c, launch_batch_cs(b.sums5, b.k0, c->n_env, e0, npw, B, b.cs, st));
  return GDM_OK;
}

static gdm_status batch_capture(gdm_ctx* c, const BatchShape& sh, const BatchBufs& b, int64_t npw, const double* khat,
                                const double2* e0, bool ir, int ir_iters, int radiative, double step,
                                hipGraphExec_t* exec) {
  // one-time settings and event pool before the capture
  if (ir) HIPCHK(c, lu_prepare<float>(sh.plan));
  else HIPCHK(c, lu_prepare<double>(sh.plan));
  while (c->lu_events.size() < 4 * sh.plan.blocks.size() + 8) {
    hipEvent_t x;
    HIPCHK(c, hipEventCreateWithFlags(&x, hipEventDisableTiming));
    c->lu_events.push_back(x);
  }
  const uint32_t prof_mask = c->prof.mask;
  c->prof.mask = 0;
  HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  gdm_status s = batch_enqueue_group(c, sh, b, npw, khat, e0, ir, ir_iters, radiative, step);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->stream, &g);
  c->prof.mask = prof_mask;
  if (s != GDM_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  HIPCHK(c, e);
  e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIPCHK(c, e);
  return GDM_OK;
}

extern "C" int32_t gdm_batch_tuning(const gdm_ctx* c, int32_t* out, int32_t max_entries) {
  if (!c) return 0;
  int32_t k = 0;
  for (const auto& e : c->batch_tune) {
    if (out && k < max_entries) {
      out[3 * k + 0] = (int32_t)(e.first * 256);
      out[3 * k + 1] = e.second.first;
      out[3 * k + 2] = e.second.second;
    }
    ++k;
  }
  return k;
}

extern "C" gdm_status gdm_batch_spectra(gdm_ctx* c, int64_t n_struct, const int64_t* cell_offset,
                                        const double* r_cell, const double* step_nm, int64_t n_wl,
                                        const double* wavelengths, const double* eps, int64_t n_pw, const double* khat,
                                        const double* e0, gdm_precision prec, int32_t ir_iters, double tol,
                                        gdm_selfterm selfterm, double* cs_out, double* be_out, gdm_info* info) {
  if (!c) return GDM_E_ARG;
  if (n_struct <= 0 || !cell_offset || !r_cell || !step_nm || n_wl <= 0 || !wavelengths || !eps || n_pw <= 0 ||
      !khat || !e0 || !cs_out)
    FAIL(c, GDM_E_ARG, "bad batch arguments");
  if (prec != GDM_PREC_FP64 && prec != GDM_PREC_FP32_IR) FAIL(c, GDM_E_ARG, "unknown precision");
  if (selfterm != GDM_SELF_STATIC && selfterm != GDM_SELF_RADIATIVE) FAIL(c, GDM_E_ARG, "unknown self-term mode");
  if (n_pw > 65535 || n_wl > (int64_t)INT32_MAX) FAIL(c, GDM_E_ARG, "too many plane waves or wavelengths");
  if (cell_offset[0] != 0) FAIL(c, GDM_E_ARG, "cell_offset[0] must be 0");
  int64_t nmax = 0;
  for (int64_t s = 0; s < n_struct; ++s) {
    const int64_t N = cell_offset[s + 1] - cell_offset[s];
    if (N <= 0) FAIL(c, GDM_E_ARG, "structure %lld has no cells", (long long)s);
    if (3 * N > 200000) FAIL(c, GDM_E_ARG, "structure %lld too large for the batched driver", (long long)s);
    if (!(step_nm[s] > 0.0) || !std::isfinite(step_nm[s])) FAIL(c, GDM_E_ARG, "step_nm[%lld] must be > 0", (long long)s);
    nmax = std::max(nmax, 3 * N);
  }
  for (int64_t l = 0; l < n_wl; ++l)
    if (!(wavelengths[l] > 0.0) || !std::isfinite(wavelengths[l])) FAIL(c, GDM_E_ARG, "wavelengths must be > 0");
  if (ir_iters < 0) ir_iters = 2;
  if (ir_iters > 20) FAIL(c, GDM_E_ARG, "at most 20 refinement corrections");
  if (!(tol >= 0.0) || !std::isfinite(tol)) FAIL(c, GDM_E_ARG, "tol must be finite and >= 0");
  const bool ir = prec == GDM_PREC_FP32_IR;
  const int radiative = selfterm == GDM_SELF_RADIATIVE ? 1 : 0;
  HIPCHK(c, hipSetDevice(c->device));
  size_t free_b = 0, total_b = 0;
  HIPCHK(c, hipMemGetInfo(&free_b, &total_b));
  size_t budget = std::min<size_t>(free_b / 2, (size_t)64 << 30);
  if (c->mem.limit > 0) budget = std::min(budget, c->mem.limit > c->mem.used ? (c->mem.limit - c->mem.used) / 2 : 0);

  // largest feasible group per structure size: panels of all items co-resident,
  // matrices within the memory budget, at most 32 items and n_wl
  auto bmax_for = [&](int64_t n) {
    int best = 0;
    for (int B = 1; B <= 32 && B <= n_wl; B *= 2) {
      BatchShape sh;
      if (batch_shape_for(c, n, B, 128, ir, sh) && (size_t)B * batch_item_bytes(n, ir) <= budget) best = B;
    }
    return best;
  };
  // size the workspaces for the largest group any structure may use
  size_t m_elems = 0, ws_bytes = 0, vec_elems = 0, part_elems = 0, pos_elems = 0;
  int Bcap = 0;
  std::vector<int> bmax(n_struct);
  for (int64_t s = 0; s < n_struct; ++s) {
    const int64_t n = 3 * (cell_offset[s + 1] - cell_offset[s]);
    bmax[s] = bmax_for(n);
    if (bmax[s] == 0) FAIL(c, GDM_E_OOM, "structure %lld (n = %lld) does not fit the batched driver", (long long)s, (long long)n);
    for (int B = 1; B <= bmax[s]; B *= 2)
      for (int nbm : {128, 64}) {
        BatchShape sh;
        if (!batch_shape_for(c, n, B, nbm, ir, sh)) continue;
        ws_bytes = std::max(ws_bytes, lu_workspace_bytes(sh.plan, ir ? 4 : 8, c->num_cu, B));
      }
    m_elems = std::max(m_elems, (size_t)bmax[s] * n * n);
    vec_elems = std::max(vec_elems, (size_t)bmax[s] * n_pw * n);
    part_elems = std::max(part_elems, (size_t)batch_part_elems(n, bmax[s], n_pw));
    pos_elems = std::max(pos_elems, (size_t)n);
    Bcap = std::max(Bcap, bmax[s]);
  }
  HIPCHK(c, c->bM64.ensure(sizeof(double2) * m_elems));
  if (ir) HIPCHK(c, c->bM32.ensure(sizeof(float2) * m_elems));
  HIPCHK(c, c->bipiv.ensure(sizeof(int32_t) * (size_t)Bcap * nmax));
  HIPCHK(c, c->bws.ensure(ws_bytes));
  HIPCHK(c, c->bvec.ensure(sizeof(double2) * 4 * vec_elems + sizeof(float2) * vec_elems + 256));
  HIPCHK(c, c->bpart.ensure(sizeof(double2) * std::max<size_t>(part_elems, 1)));
  const size_t ncol = (size_t)Bcap * n_pw;
  const size_t n_items = (size_t)n_struct * n_wl;
  const size_t nsmall = 4 * ncol + 2 * (size_t)Bcap + (size_t)Bcap * nmax + 5 * ncol + (size_t)Bcap + 3 * ncol +
                        (size_t)Bcap + 1 + 2 * (size_t)Bcap + 64 + (size_t)Bcap + 1 + n_items;
  HIPCHK(c, c->bsmall.ensure(sizeof(double) * nsmall));
  HIPCHK(c, c->bpos.ensure(sizeof(double) * pos_elems));
  HIPCHK(c, c->bwl.ensure(sizeof(double) * n_wl));
  HIPCHK(c, hipMemcpyAsync(c->bwl.p, wavelengths, sizeof(double) * n_wl, hipMemcpyHostToDevice, c->stream));
  BatchBufs b{};
  b.M64 = c->bM64.as<double2>();
  b.M32 = ir ? c->bM32.as<float2>() : nullptr;
  b.ipiv = c->bipiv.as<int32_t>();
  b.ws = c->bws.p;
  b.F0 = c->bvec.as<double2>();
  b.X = b.F0 + vec_elems;
  b.R = b.X + vec_elems;
  b.Q = b.R + vec_elems;
  b.C32 = reinterpret_cast<float2*>(b.Q + vec_elems);
  b.part = c->bpart.p;
  b.part_elems = (int64_t)std::max<size_t>(part_elems, 1);
  double* sp = c->bsmall.as<double>();
  b.rmax = sp; sp += ncol;
  b.xmax = sp; sp += ncol;
  b.bmax = sp; sp += ncol;
  b.cmax = sp; sp += ncol;
  b.minf = sp; sp += Bcap;
  b.k0 = sp; sp += Bcap;
  b.rows = sp; sp += (size_t)Bcap * nmax;
  b.sums5 = sp; sp += 5 * ncol;
  b.be = sp; sp += Bcap;
  b.cs = sp; sp += 3 * ncol;
  b.be_max = sp; sp += 1;
  b.alpha = reinterpret_cast<double2*>(sp); sp += 2 * (size_t)Bcap;
  b.sticky = reinterpret_cast<int32_t*>(sp); sp += 64;
  b.sfail = reinterpret_cast<int32_t*>(sp); sp += Bcap;
  b.scount = reinterpret_cast<int32_t*>(sp); sp += 1;
  b.slist = reinterpret_cast<int64_t*>(sp);
  b.pos = c->bpos.as<double>();
  b.wl = c->bwl.as<double>();
  HIPCHK(c, launch_batch_err_init(b.sticky, c->stream));
  hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, c->stream, b.scount, 1, 0);
  hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, c->stream, reinterpret_cast<int*>(b.be_max), 2, 0);
  const double2* E0 = reinterpret_cast<const double2*>(e0);
  const double2* EPS = reinterpret_cast<const double2*>(eps);

  struct Cached {
    int64_t n;
    int B, nb;
    double step;
    hipGraphExec_t exec;
  };
  std::vector<Cached> graphs;
  auto release = [&]() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
  };
  hipEvent_t t0, t1, tstart, tend;
  HIPCHK(c, hipEventCreate(&t0));
  HIPCHK(c, hipEventCreate(&t1));
  HIPCHK(c, hipEventCreate(&tstart));
  HIPCHK(c, hipEventCreate(&tend));
  HIPCHK(c, hipEventRecord(tstart, c->stream));
  gdm_status status = GDM_OK;
  int64_t items_done = 0;
  for (int64_t s = 0; s < n_struct && status == GDM_OK; ++s) {
    const int64_t N = cell_offset[s + 1] - cell_offset[s], n = 3 * N;
    const double step = step_nm[s];
    HIPCHK(c, hipMemcpyAsync(b.pos, r_cell + 3 * cell_offset[s], sizeof(double) * 3 * N, hipMemcpyDeviceToDevice,
                             c->stream));
    // batch configuration: measured for this size class, or measured now on the
    // first groups of this structure (they are real work, not discarded)
    // candidates: (items per group, panel width), distinct actual shapes only
    std::vector<std::pair<int, int>> cand;
    const int64_t key = n / 256;
    auto it = c->batch_tune.find(key);
    auto add_cand = [&](int B, int nbm) {
      BatchShape sh;
      if (!batch_shape_for(c, n, B, nbm, ir, sh)) return;
      for (auto& x : cand)
        if (x.first == B && x.second == sh.nb) return;
      cand.push_back({B, sh.nb});
    };
    if (it != c->batch_tune.end() && it->second.first <= bmax[s]) add_cand(it->second.first, it->second.second);
    if (cand.empty()) {
      for (int B = bmax[s]; B >= 1 && (int)cand.size() < 3; B /= 2) add_cand(B, 128);
      add_cand(bmax[s], 64);
    }
    double best_rate = -1.0;
    std::pair<int, int> best = cand[0];
    size_t ci = 0;
    for (int64_t l0 = 0; l0 < n_wl && status == GDM_OK;) {
      const bool tuning = cand.size() > 1 && ci < cand.size();
      const std::pair<int, int> cfg = tuning ? cand[ci] : best;
      BatchShape sh;
      if (!batch_shape_for(c, n, cfg.first, cfg.second, ir, sh)) {
        status = GDM_E_STATE;
        break;
      }
      hipGraphExec_t ex = nullptr;
      for (auto& g : graphs)
        if (g.n == sh.n && g.B == sh.B && g.nb == sh.nb && g.step == step) ex = g.exec;
      if (!ex) {
        status = batch_capture(c, sh, b, n_pw, khat, E0, ir, ir_iters, radiative, step, &ex);
        if (status != GDM_OK) break;
        graphs.push_back({sh.n, sh.B, sh.nb, step, ex});
      }
      const int64_t nvalid = std::min<int64_t>(sh.B, n_wl - l0);
      HIPCHK(c, launch_batch_stage(EPS, n_wl, s, l0, nvalid, sh.B, b.wl, c->n_env * c->n_env, step, b.alpha, b.k0,
                                   c->stream));
      HIPCHK(c, hipEventRecord(t0, c->stream));
      HIPCHK(c, hipGraphLaunch(ex, c->stream));
      HIPCHK(c, hipEventRecord(t1, c->stream));
      HIPCHK(c, launch_batch_unstage(b.cs, ir ? b.be : nullptr, nvalid, n_pw, s * n_wl + l0, cs_out,
                                     ir ? be_out : nullptr, c->stream));
      if (ir) HIPCHK(c, launch_batch_bemax(b.be, nvalid, b.be_max, c->stream));
      if (sh.plan.spec)
        HIPCHK(c, launch_batch_spec_list(b.sfail, nvalid, s * n_wl + l0, b.slist, b.scount, (int64_t)n_items,
                                         c->stream));
      if (tuning) {
        // the candidates run on real groups (results kept); rate = items per ms
        HIPCHK(c, hipEventSynchronize(t1));
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, t0, t1);
        const double rate = (double)sh.B / std::max(ms, 1e-3f);
        if (rate > best_rate) {
          best_rate = rate;
          best = cfg;
        }
        if (++ci == cand.size()) c->batch_tune[key] = best;
      }
      items_done += nvalid;
      l0 += nvalid;
    }
  }
  (void)items_done;
  HIPCHK(c, hipEventRecord(tend, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  float ms_total = 0.f;
  (void)hipEventElapsedTime(&ms_total, tstart, tend);
  int32_t sticky[2] = {0, 0};
  double be_max = 0.0;
  int32_t nfail = 0;
  HIPCHK(c, hipMemcpy(sticky, b.sticky, sizeof(sticky), hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(&be_max, b.be_max, sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(&nfail, b.scount, sizeof(int32_t), hipMemcpyDeviceToHost));
  std::vector<int64_t> failed((size_t)std::min<int64_t>(nfail, (int64_t)n_items));
  if (!failed.empty())
    HIPCHK(c, hipMemcpy(failed.data(), b.slist, sizeof(int64_t) * failed.size(), hipMemcpyDeviceToHost));
  release();
  for (hipEvent_t ev : {t0, t1, tstart, tend}) (void)hipEventDestroy(ev);
  if (status != GDM_OK) return status;
  // Items whose speculative pivots failed their check: each again on its own
  // with the pivot search, overwriting its outputs (rare for dielectrics; the
  // zero-pivot and refinement reports below then cover these runs too).
  if (!failed.empty()) {
    std::sort(failed.begin(), failed.end());
    const int saved = c->pivot_pb;
    c->pivot_pb = 1;
    for (int64_t item : failed) {
      const int64_t s = item / n_wl, l = item % n_wl;
      const int64_t off[2] = {0, cell_offset[s + 1] - cell_offset[s]};
      gdm_info sub{};
      const gdm_status st2 = gdm_batch_spectra(
          c, 1, off, r_cell + 3 * cell_offset[s], step_nm + s, 1, wavelengths + l, eps + 2 * item, n_pw, khat, e0,
          prec, ir_iters, 0.0, selfterm, cs_out + item * n_pw * 3, be_out ? be_out + item : nullptr, &sub);
      ++c->pivot_fallbacks;
      if (st2 != GDM_OK) {
        c->pivot_pb = saved;
        if (info) info->bad_index = sub.bad_index;
        return st2;
      }
      if (ir) be_max = std::max(be_max, sub.backward_err);
    }
    c->pivot_pb = saved;
  }
  if (info) {
    info->ir_iters = ir ? ir_iters : 0;
    info->backward_err = ir ? be_max : 0.0;
    info->bad_index = -1;
    info->ms_factor = ms_total;
  }
  if (sticky[0]) FAIL(c, GDM_E_DEVICE, "LU panel exchange timed out in the batched driver");
  if (sticky[1] != INT32_MAX) {
    if (info) info->bad_index = sticky[1];
    FAIL(c, GDM_E_SINGULAR, "exactly zero pivot in column %d of a batched system", sticky[1]);
  }
  if (ir && tol > 0.0 && !(be_max <= tol))
    FAIL(c, GDM_E_NOCONV, "a batched system ends at backward error %.3e > tol %.3e after %d corrections", be_max,
         tol, ir_iters);
  return GDM_OK;
}

// Static device scratch of gdm_fields_noalloc: each device that loads the
// library holds its own copy until the process ends.  Host code never uses the
// array's name as a device address: gdm_create looks up the address on its
// device once (hipGetSymbolAddress with that device current) and every use goes
// through that pointer.
constexpr size_t NOALLOC_FLAG_BYTES = 256;  // probe-on-dipole flag, then the partial sums
static __device__ __align__(256) unsigned char scratch[GDM_NOALLOC_SCRATCH_BYTES];
constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex noalloc_mu;
static void* noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// device must be current; returns the status of the lookup
static hipError_t noalloc_register(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(noalloc_mu);
  if (noalloc_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return e != hipSuccess ? e : hipErrorInvalidSymbol;
  }
  noalloc_ptr[device] = ptr;
  return hipSuccess;
}

static void* noalloc_scratch(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(noalloc_mu);
  return noalloc_ptr[device];
}

extern "C" {

gdm_status gdm_create(int device, void* hip_stream, gdm_ctx** out) {
  if (!out) return GDM_E_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return GDM_E_DEVICE;
  if (device < 0 || device >= ndev) return GDM_E_ARG;
  if (hipSetDevice(device) != hipSuccess) return GDM_E_DEVICE;
  gdm_ctx* c = new gdm_ctx();
  c->device = device;
  for (DevBuf* b : c->buffers()) b->acct = &c->mem;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    c->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    size_t lds = prop.maxSharedMemoryPerMultiProcessor;
    if (lds == 0 || lds > 160 * 1024) lds = 160 * 1024;
    c->lds_bytes = (int)lds;
  }
  if (hip_stream) {
    c->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return GDM_E_DEVICE;
    }
    c->own_stream = true;
  }
  for (auto& e : c->ev) (void)hipEventCreate(&e);
  for (auto& e : c->sev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) e = nullptr;
  if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess) c->side = nullptr;
  // the no-alloc entry points' static scratch on this device (a failed lookup
  // only disables them: they report it)
  (void)noalloc_register(device);
  *out = c;
  return GDM_OK;
}

void gdm_destroy(gdm_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (DevBuf* b : c->buffers()) b->release();
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : c->sev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->lu_events) (void)hipEventDestroy(e);
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamDestroy(c->side);
  }
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* gdm_last_error(const gdm_ctx* c) { return c ? c->err.c_str() : "null context"; }

gdm_status gdm_sync(gdm_ctx* c) {
  if (!c) return GDM_E_ARG;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return GDM_OK;
}

gdm_status gdm_set_memory_limit(gdm_ctx* c, int64_t bytes) {
  if (!c) return GDM_E_ARG;
  if (bytes < 0) FAIL(c, GDM_E_ARG, "memory limit must be >= 0 (got %lld)", (long long)bytes);
  c->mem.limit = (size_t)bytes;
  return GDM_OK;
}

int64_t gdm_memory_used(const gdm_ctx* c) { return c ? (int64_t)c->mem.used : 0; }

gdm_status gdm_set_pivoting(gdm_ctx* c, int32_t columns_per_exchange) {
  if (!c) return GDM_E_ARG;
  const int v = columns_per_exchange;
  if (v != 0 && v != 1 && v != 2 && v != 4 && v != 8)
    FAIL(c, GDM_E_ARG, "columns per pivot exchange must be 0, 1, 2, 4 or 8 (got %d)", v);
  c->pivot_pb = v;
  return GDM_OK;
}

int64_t gdm_pivot_fallbacks(const gdm_ctx* c) { return c ? c->pivot_fallbacks : -1; }

gdm_status gdm_set_environment(gdm_ctx* c, double n_env) {
  if (!c) return GDM_E_ARG;
  if (!(n_env > 0.0) || !std::isfinite(n_env)) FAIL(c, GDM_E_ARG, "n_env must be finite and > 0 (got %g)", n_env);
  c->n_env = n_env;
  c->factored = false;
  return GDM_OK;
}

gdm_status gdm_set_structure(gdm_ctx* c, int64_t n_cell, const double* r_cell, double step_nm, const double* eps_cell,
                             int64_t n_eff, const double* r_eff, const double* alpha_eff, gdm_selfterm selfterm) {
  if (!c) return GDM_E_ARG;
  if (n_cell < 0 || n_eff < 0 || n_cell + n_eff == 0)
    FAIL(c, GDM_E_ARG, "need n_cell >= 0, n_eff >= 0 and at least one dipole (got %lld, %lld)", (long long)n_cell,
         (long long)n_eff);
  if (n_cell > 0 && (!r_cell || !eps_cell)) FAIL(c, GDM_E_ARG, "r_cell and eps_cell are required when n_cell > 0");
  if (n_cell > 0 && !(step_nm > 0.0 && std::isfinite(step_nm))) FAIL(c, GDM_E_ARG, "step_nm must be > 0");
  if (n_eff > 0 && (!r_eff || !alpha_eff)) FAIL(c, GDM_E_ARG, "r_eff and alpha_eff are required when n_eff > 0");
  if (selfterm != GDM_SELF_STATIC && selfterm != GDM_SELF_RADIATIVE) FAIL(c, GDM_E_ARG, "unknown self-term mode");
  const int64_t N = n_cell + n_eff;
  if (3 * N + 3 * n_eff > (int64_t)INT32_MAX) FAIL(c, GDM_E_ARG, "too many unknowns");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, c->pos.ensure(sizeof(double) * 3 * N));
  HIPCHK(c, c->eps.ensure(sizeof(double2) * std::max<int64_t>(n_cell, 1)));
  HIPCHK(c, c->alpha_c.ensure(sizeof(double2) * std::max<int64_t>(n_cell, 1)));
  HIPCHK(c, c->alpha6.ensure(sizeof(double2) * 36 * std::max<int64_t>(n_eff, 1)));
  if (n_cell > 0) {
    HIPCHK(c, hipMemcpyAsync(c->pos.p, r_cell, sizeof(double) * 3 * n_cell, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->eps.p, eps_cell, sizeof(double2) * n_cell, hipMemcpyDeviceToDevice, c->stream));
  }
  if (n_eff > 0) {
    HIPCHK(c, hipMemcpyAsync(c->pos.as<double>() + 3 * n_cell, r_eff, sizeof(double) * 3 * n_eff,
                             hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->alpha6.p, alpha_eff, sizeof(double2) * 36 * n_eff, hipMemcpyDeviceToDevice,
                             c->stream));
  }
  c->nc = n_cell;
  c->ne = n_eff;
  c->N = N;
  c->n = 3 * N + 3 * n_eff;
  c->n_gpm = 0;  // groups refer to the previous structure's effective dipoles
  c->step = n_cell > 0 ? step_nm : 1.0;
  c->self_mode = selfterm;
  c->factored = false;
  return GDM_OK;
}

int64_t gdm_num_unknowns(const gdm_ctx* c) { return c ? c->n : 0; }

gdm_status gdm_set_gpm(gdm_ctx* c, int64_t n_groups, const int64_t* first, const int64_t* size, const double* alpha) {
  if (!c) return GDM_E_ARG;
  if (n_groups < 0 || (n_groups > 0 && (!first || !size || !alpha)))
    FAIL(c, GDM_E_ARG, "need n_groups >= 0 and, for groups, first, size and alpha");
  if (n_groups > 0 && c->ne <= 0) FAIL(c, GDM_E_ARG, "the structure has no effective dipoles");
  std::vector<int32_t> gid((size_t)std::max<int64_t>(c->ne, 1), -1);
  std::vector<int64_t> tab((size_t)std::max<int64_t>(3 * n_groups, 1));
  int64_t off = 0;
  for (int64_t g = 0; g < n_groups; ++g) {
    const int64_t f = first[g], m = size[g];
    if (m < 1 || m > GPM_MAX_PAIRS) FAIL(c, GDM_E_ARG, "group %lld: size %lld not in [1, %d]", (long long)g, (long long)m, GPM_MAX_PAIRS);
    if (f < 0 || f + m > c->ne)
      FAIL(c, GDM_E_ARG, "group %lld: effective dipoles [%lld, %lld) outside [0, %lld)", (long long)g, (long long)f,
           (long long)(f + m), (long long)c->ne);
    for (int64_t e = f; e < f + m; ++e) {
      if (gid[e] >= 0) FAIL(c, GDM_E_ARG, "effective dipole %lld is in two groups", (long long)e);
      gid[e] = (int32_t)g;
    }
    tab[3 * g] = f;
    tab[3 * g + 1] = m;
    tab[3 * g + 2] = off;
    off += 36 * m * m;
  }
  HIPCHK(c, hipSetDevice(c->device));
  c->factored = false;
  c->n_gpm = 0;
  if (n_groups == 0) return GDM_OK;
  HIPCHK(c, c->gpm_gid.ensure(sizeof(int32_t) * gid.size()));
  HIPCHK(c, c->gpm_tab.ensure(sizeof(int64_t) * tab.size()));
  HIPCHK(c, c->gpm_alpha.ensure(sizeof(double2) * off));
  HIPCHK(c, hipMemcpyAsync(c->gpm_gid.p, gid.data(), sizeof(int32_t) * gid.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->gpm_tab.p, tab.data(), sizeof(int64_t) * tab.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->gpm_alpha.p, alpha, sizeof(double2) * off, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));  // the host vectors go out of scope
  c->n_gpm = n_groups;
  return GDM_OK;
}

gdm_status gdm_assemble(gdm_ctx* c, double wl, int dtype, void* M_out, int64_t ld) {
  if (!c) return GDM_E_ARG;
  gdm_status s = check_wavelength(c, wl);
  if (s != GDM_OK) return s;
  if (!M_out) FAIL(c, GDM_E_ARG, "M_out is NULL");
  if (dtype != 0 && dtype != 1) FAIL(c, GDM_E_ARG, "dtype must be 0 (complex double) or 1 (complex float)");
  if (ld < c->n) FAIL(c, GDM_E_ARG, "ld (%lld) < n (%lld)", (long long)ld, (long long)c->n);
  HIPCHK(c, hipSetDevice(c->device));
  if ((s = prepare_alpha(c)) != GDM_OK) return s;
  const Wave w = wave_of(c, wl);
  const DipoleView d = view_of(c, self_term(c, w));
  if (dtype == 0) HIPCHK(c, launch_assemble<double>(d, w, M_out, ld, c->stream));
  else HIPCHK(c, launch_assemble<float>(d, w, M_out, ld, c->stream));
  return GDM_OK;
}

gdm_status gdm_factorize(gdm_ctx* c, double wl, gdm_precision prec, gdm_info* info) {
  if (!c) return GDM_E_ARG;
  gdm_status s = check_wavelength(c, wl);
  if (s != GDM_OK) return s;
  if (prec != GDM_PREC_FP64 && prec != GDM_PREC_FP32_IR) FAIL(c, GDM_E_ARG, "unknown precision");
  HIPCHK(c, hipSetDevice(c->device));
  c->factored = false;
  const int64_t n = c->n;
  c->ld = n;
  if ((s = prepare_alpha(c)) != GDM_OK) return s;
  const Wave w = wave_of(c, wl);
  const DipoleView d = view_of(c, self_term(c, w));
  HIPCHK(c, hipEventRecord(c->ev[0], c->stream));
  const double nn = (double)n * (double)n;
  if (prec == GDM_PREC_FP64) {
    HIPCHK(c, c->M.ensure(sizeof(double2) * n * n));
    HIPCHK(c, c->prof.begin(c->stream, PROF_ASSEMBLE, 16.0 * nn));
    HIPCHK(c, launch_assemble<double>(d, w, c->M.p, n, c->stream));
    HIPCHK(c, c->prof.end(c->stream));
  } else {
    HIPCHK(c, c->M64.ensure(sizeof(double2) * n * n));
    HIPCHK(c, c->M.ensure(sizeof(float2) * n * n));
    HIPCHK(c, c->prof.begin(c->stream, PROF_ASSEMBLE, 24.0 * nn));
    HIPCHK(c, launch_assemble_dual(d, w, c->M64.as<double2>(), c->M.as<float2>(), n, c->stream));
    HIPCHK(c, c->prof.end(c->stream));
    HIPCHK(c, c->rows.ensure(sizeof(double) * n));
    HIPCHK(c, launch_rowsum_abs(c->M64.as<double2>(), n, n, c->rows.as<double>(), c->stream));
  }
  HIPCHK(c, hipEventRecord(c->ev[1], c->stream));
  // a failed speculative panel needs the matrix again: assembled anew (FP64), or
  // both copies assembled anew (FP32 + IR; the FP64 copy is unchanged by then,
  // and assembling is as fast as converting it)
  auto rebuild = [&]() -> hipError_t {
    if (prec == GDM_PREC_FP64) return launch_assemble<double>(d, w, c->M.p, n, c->stream);
    return launch_assemble_dual(d, w, c->M64.as<double2>(), c->M.as<float2>(), n, c->stream);
  };
  if (prec == GDM_PREC_FP64) s = run_lu<double>(c, c->M.p, n, n, c->plan, c->luws, c->ipiv, nullptr, info, rebuild);
  else s = run_lu<float>(c, c->M.p, n, n, c->plan, c->luws, c->ipiv, nullptr, info, rebuild);
  if (s != GDM_OK) return s;
  HIPCHK(c, hipEventRecord(c->ev[2], c->stream));
  HIPCHK(c, hipEventSynchronize(c->ev[2]));
  (void)hipEventElapsedTime(&c->ms_assemble, c->ev[0], c->ev[1]);
  (void)hipEventElapsedTime(&c->ms_factor, c->ev[1], c->ev[2]);
  if (prec == GDM_PREC_FP32_IR) {
    std::vector<double> rows(n);
    HIPCHK(c, hipMemcpy(rows.data(), c->rows.p, sizeof(double) * n, hipMemcpyDeviceToHost));
    c->Minf = *std::max_element(rows.begin(), rows.end());
  }
  if (info) {
    info->ms_assemble = c->ms_assemble;
    info->ms_factor = c->ms_factor;
    info->bad_index = -1;
  }
  c->wavelength = wl;
  c->prec = prec;
  c->M1 = -1.0;
  c->factored = true;
  return GDM_OK;
}

gdm_status gdm_set_wavelength(gdm_ctx* c, double wl) {
  if (!c) return GDM_E_ARG;
  gdm_status s = check_wavelength(c, wl);
  if (s != GDM_OK) return s;
  if (wl != c->wavelength) c->factored = false;
  c->wavelength = wl;
  return GDM_OK;
}

gdm_status gdm_solve_iterative(gdm_ctx* c, double wl, int64_t nrhs, const double* f0, double tol, int32_t max_iter,
                               int32_t restart, double* q_out, double* f_out, gdm_info* info) {
  if (!c) return GDM_E_ARG;
  gdm_status s = check_wavelength(c, wl);
  if (s != GDM_OK) return s;
  if (nrhs <= 0 || !f0 || !q_out) FAIL(c, GDM_E_ARG, "need n_rhs > 0, f0 and q_out");
  if (nrhs > 65535) FAIL(c, GDM_E_ARG, "at most 65535 right-hand sides per call");
  if (c->n_gpm > 0) FAIL(c, GDM_E_ARG, "the matrix-free solver does not handle GPM groups (use gdm_factorize)");
  if (restart <= 0) restart = 30;
  if (restart > 1000) FAIL(c, GDM_E_ARG, "restart must be <= 1000");
  if (max_iter <= 0) max_iter = 1000;
  if (!(tol > 0.0)) tol = 1e-13;
  HIPCHK(c, hipSetDevice(c->device));
  if ((s = prepare_alpha(c)) != GDM_OK) return s;
  if (wl != c->wavelength) c->factored = false;
  c->wavelength = wl;
  const int64_t n = c->n;
  const Wave w = wave_of(c, wl);
  const DipoleView d = view_of(c, self_term(c, w));
  HIPCHK(c, c->iter.ensure(iter_workspace_bytes(c->N, n, nrhs, restart, c->num_cu)));
  HIPCHK(c, c->X.ensure(sizeof(double2) * n * nrhs));
  IterWork iw;
  iter_workspace_carve(c->iter.p, c->N, n, nrhs, restart, c->num_cu, iw);
  double2* X = c->X.as<double2>();
  HIPCHK(c, hipEventRecord(c->ev[0], c->stream));
  GmresStats gs;
  HIPCHK(c, gmres_solve(d, w, iw, n, nrhs, reinterpret_cast<const double2*>(f0), X, tol, max_iter, restart, c->stream,
                        gs, &c->prof));
  HIPCHK(c, launch_apply_alpha(view_of(c, make_double2(0, 0)), X, n, reinterpret_cast<double2*>(q_out), n, nrhs,
                               c->stream));
  if (f_out) HIPCHK(c, launch_copy_d(X, n, reinterpret_cast<double2*>(f_out), n, n, nrhs, c->stream));
  HIPCHK(c, hipEventRecord(c->ev[3], c->stream));
  HIPCHK(c, hipEventSynchronize(c->ev[3]));
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, c->ev[0], c->ev[3]);
  c->prof.collect();
  if (info) {
    info->ir_iters = gs.iters;
    info->backward_err = gs.relres;
    info->bad_index = -1;
    info->ms_solve = ms;
    info->ms_ir = 0.f;
  }
  if (!(gs.relres <= tol))
    FAIL(c, GDM_E_NOCONV, "GMRES stopped after %d products at relative residual %.3e > tol %.3e", gs.iters, gs.relres,
         tol);
  return GDM_OK;
}

gdm_status gdm_incident_planewave(gdm_ctx* c, int64_t n_pw, const double* khat, const double* e0, double* f0) {
  if (!c) return GDM_E_ARG;
  if (c->wavelength <= 0) FAIL(c, GDM_E_STATE, "no wavelength set (call gdm_factorize first)");
  if (n_pw < 0 || (n_pw > 0 && (!khat || !e0 || !f0))) FAIL(c, GDM_E_ARG, "bad plane-wave arguments");
  if (n_pw > 65535) FAIL(c, GDM_E_ARG, "at most 65535 plane waves per call");
  HIPCHK(c, hipSetDevice(c->device));
  const Wave w = wave_of(c, c->wavelength);
  const DipoleView d = view_of(c, make_double2(0, 0));
  HIPCHK(c, launch_incident(d, w, c->n_env, n_pw, khat, reinterpret_cast<const double2*>(e0),
                            reinterpret_cast<double2*>(f0), c->n, c->stream));
  return GDM_OK;
}

gdm_status gdm_planewave(gdm_ctx* c, int64_t n_pw, const double* khat, const double* e0, int64_t n_pts,
                         const double* r, double* E, double* H) {
  if (!c) return GDM_E_ARG;
  if (c->wavelength <= 0) FAIL(c, GDM_E_STATE, "no wavelength set (call gdm_factorize first)");
  if (n_pw < 0 || n_pts < 0 || (n_pw > 0 && n_pts > 0 && (!khat || !e0 || !r || !E)))
    FAIL(c, GDM_E_ARG, "bad plane-wave arguments");
  if (n_pw > 65535) FAIL(c, GDM_E_ARG, "at most 65535 plane waves per call");
  HIPCHK(c, hipSetDevice(c->device));
  const Wave w = wave_of(c, c->wavelength);
  HIPCHK(c, launch_planewave_points(w, c->n_env, n_pw, khat, reinterpret_cast<const double2*>(e0), r, n_pts,
                                    reinterpret_cast<double2*>(E), reinterpret_cast<double2*>(H), c->stream));
  return GDM_OK;
}

gdm_status gdm_solve(gdm_ctx* c, int64_t nrhs, const double* f0, double tol, int32_t max_iter, double* q_out,
                     double* f_out, gdm_info* info) {
  if (!c) return GDM_E_ARG;
  if (!c->factored) FAIL(c, GDM_E_STATE, "gdm_solve before gdm_factorize");
  if (nrhs <= 0 || !f0 || !q_out) FAIL(c, GDM_E_ARG, "need n_rhs > 0, f0 and q_out");
  if (nrhs > 65535) FAIL(c, GDM_E_ARG, "at most 65535 right-hand sides per call");
  HIPCHK(c, hipSetDevice(c->device));
  const int64_t n = c->n;
  HIPCHK(c, c->X.ensure(sizeof(double2) * n * nrhs));
  double2* X = c->X.as<double2>();
  const DipoleView d = view_of(c, make_double2(0, 0));
  HIPCHK(c, hipEventRecord(c->ev[0], c->stream));
  SolveStats ss;
  gdm_status status = solve_core(c, 0, nrhs, reinterpret_cast<const double2*>(f0), X, tol, max_iter, ss);
  if (status != GDM_OK && status != GDM_E_NOCONV) return status;
  HIPCHK(c, launch_apply_alpha(d, X, n, reinterpret_cast<double2*>(q_out), n, nrhs, c->stream));
  if (f_out) HIPCHK(c, launch_copy_d(X, n, reinterpret_cast<double2*>(f_out), n, n, nrhs, c->stream));
  HIPCHK(c, hipEventRecord(c->ev[3], c->stream));
  HIPCHK(c, hipEventSynchronize(c->ev[3]));
  float ms_total = 0.f;
  (void)hipEventElapsedTime(&ms_total, c->ev[0], c->ev[3]);
  c->prof.collect();
  if (info) {
    info->ir_iters = ss.iters;
    info->backward_err = ss.be;
    info->bad_index = -1;
    info->ms_assemble = c->ms_assemble;
    info->ms_factor = c->ms_factor;
    info->ms_solve = ms_total - ss.ms_ir;
    info->ms_ir = ss.ms_ir;
  }
  if (status == GDM_E_NOCONV)
    FAIL(c, GDM_E_NOCONV, "refinement stopped at backward error %.3e > tol %.3e", ss.be, ss.tol);
  return GDM_OK;
}

gdm_status gdm_adjoint(gdm_ctx* c, int64_t nrhs, const double* khat, const double* e0, const double* f0,
                       const double* q, const double* f, const double* g_sigma, int64_t P, const double* r_probe,
                       const double* g_e, double tol, int32_t max_iter, double* grad_r, double* grad_eps,
                       double* grad_wl, gdm_info* info) {
  if (!c) return GDM_E_ARG;
  if (!c->factored) FAIL(c, GDM_E_STATE, "gdm_adjoint needs the factors of gdm_factorize");
  if (c->n_gpm > 0) FAIL(c, GDM_E_ARG, "gdm_adjoint is written for local polarisabilities (GPM groups are set)");
  if (nrhs <= 0 || nrhs > 65535) FAIL(c, GDM_E_ARG, "need 0 < n_rhs <= 65535");
  if (!khat || !e0 || !f0 || !q || !f) FAIL(c, GDM_E_ARG, "khat, e0, f0, q and f are required");
  if (!grad_r || !grad_wl || (c->nc > 0 && !grad_eps)) FAIL(c, GDM_E_ARG, "grad_r, grad_eps and grad_wl are required");
  if (P < 0 || (P > 0 && g_e && !r_probe)) FAIL(c, GDM_E_ARG, "bad probe arguments");
  HIPCHK(c, hipSetDevice(c->device));
  const int64_t n = c->n, N = c->N, nc = c->nc;
  const bool probes = P > 0 && g_e;
  const Wave w = wave_of(c, c->wavelength);
  const DipoleView d = view_of(c, self_term(c, w));
  const double2* F0 = reinterpret_cast<const double2*>(f0);
  const double2* Fs = reinterpret_cast<const double2*>(f);
  const double2* Q = reinterpret_cast<const double2*>(q);
  const double2* E0 = reinterpret_cast<const double2*>(e0);
  const double2* gE = reinterpret_cast<const double2*>(g_e);
  // workspace layout (doubles): Cr | sums5 | pdk parts | pgr probe | pgr pair | then complex arrays
  const int nz = adjoint_rhs_chunks(nrhs);
  const int sp = probes ? adjoint_probe_splits(P, N, c->num_cu) : 0;
  const int sq = adjoint_pair_splits(N, c->num_cu);
  const int64_t nb_probe = probes ? (int64_t)nz * sp * adjoint_probe_blocks(N) : 0;
  const int64_t nb_pair = (int64_t)nz * sq * adjoint_pair_blocks(N);
  const int64_t nb_fin = adjoint_finish_blocks(N);
  const int64_t nb_einc = probes ? adjoint_einc_blocks(P, nrhs) : 0;
  const int64_t nparts = nb_probe + nb_pair + nb_fin + nb_einc;
  const int64_t nd = 6 * nrhs + nparts + 3 * N * ((int64_t)nz * sp + (int64_t)nz * sq);
  const int64_t ndp = (nd + 1) / 2;  // in double2 units
  const int64_t nzz = (int64_t)sp * nrhs * n + (int64_t)sq * nrhs * std::max<int64_t>(nc, 1) * 3 + 2 * nrhs * n;
  HIPCHK(c, c->adj.ensure(sizeof(double2) * (ndp + nzz)));
  HIPCHK(c, c->Lam.ensure(sizeof(double2) * n * nrhs));
  HIPCHK(c, c->flag.ensure(sizeof(int) * 4));
  double* Cr = c->adj.as<double>();
  double* sums5 = Cr + nrhs;
  double* parts = sums5 + 5 * nrhs;
  double* pdk_probe = parts;
  double* pdk_pair = pdk_probe + nb_probe;
  double* pdk_fin = pdk_pair + nb_pair;
  double* pdk_einc = pdk_fin + nb_fin;
  double* pgr_probe = parts + nparts;
  double* pgr_pair = pgr_probe + 3 * N * (int64_t)nz * sp;
  double2* zb = c->adj.as<double2>() + ndp;
  double2* pacc = zb;
  double2* pv = pacc + (int64_t)sp * nrhs * n;
  double2* gqe = pv + (int64_t)sq * nrhs * std::max<int64_t>(nc, 1) * 3;
  double2* rhs = gqe + nrhs * n;
  double2* lam = c->Lam.as<double2>();

  HIPCHK(c, launch_adjoint_cr(w, c->n_env, E0, nrhs, Cr, c->stream));
  if (probes) {
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, c->stream, c->flag.as<int>(), 4, 0);
    HIPCHK(c, c->prof.begin(c->stream, PROF_ADJ_PROBE, (double)P * (double)N * (double)nrhs));
    HIPCHK(c, launch_adjoint_probe(d, w, c->n_env, Q, n, nrhs, r_probe, gE, P, sp, pacc, pgr_probe, pdk_probe,
                                   1e-18 * c->step * c->step, c->flag.as<int>(), c->stream));
    HIPCHK(c, c->prof.end(c->stream));
    HIPCHK(c, launch_adjoint_einc(w, c->n_env, khat, E0, r_probe, gE, P, nrhs, pdk_einc, c->stream));
  }
  HIPCHK(c, launch_adjoint_seed(d, w, F0, Fs, Q, n, nrhs, Cr, g_sigma, pacc, sp, gqe, rhs, c->stream));
  SolveStats ss;
  gdm_status status = solve_core(c, 1, nrhs, rhs, lam, tol, max_iter, ss);
  if (status != GDM_OK && status != GDM_E_NOCONV) return status;
  HIPCHK(c, c->prof.begin(c->stream, PROF_ADJ_PAIR, (double)N * (double)(N - 1) * (double)nrhs));
  HIPCHK(c, launch_adjoint_pair(d, w, c->n_env, lam, Q, n, nrhs, sq, pgr_pair, pv, pdk_pair, c->stream));
  HIPCHK(c, c->prof.end(c->stream));
  HIPCHK(c, launch_adjoint_finish(d, w, c->n_env, c->step, c->self_mode == GDM_SELF_RADIATIVE ? 1 : 0, F0, Fs, Q, lam,
                                  gqe, n, nrhs, khat, Cr, g_sigma, pgr_probe, nz * sp, pgr_pair, nz * sq, pv, sq,
                                  grad_r, grad_eps, pdk_fin, c->stream));
  if (g_sigma) HIPCHK(c, launch_cs_sums(d, F0, Q, Fs, n, nrhs, sums5, c->stream));
  HIPCHK(c, launch_adjoint_wl(w, c->wavelength, parts, nparts, sums5, Cr, g_sigma, nrhs, grad_wl, c->stream));
  int flag = 0;
  if (probes) HIPCHK(c, hipMemcpyAsync(&flag, c->flag.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->prof.collect();
  if (info) {
    info->ir_iters = ss.iters;
    info->backward_err = ss.be;
    info->bad_index = -1;
    info->ms_ir = ss.ms_ir;
  }
  if (flag) FAIL(c, GDM_E_PROBE_AT_DIPOLE, "a probe point lies on a dipole (|R| < 1e-9 step)");
  if (status == GDM_E_NOCONV)
    FAIL(c, GDM_E_NOCONV, "adjoint refinement stopped at backward error %.3e > tol %.3e", ss.be, ss.tol);
  return GDM_OK;
}

}  // extern "C"

// Probe fields of gdm_fields and gdm_fields_noalloc: partial sums of the dipole
// splits in `part` (capacity part_cap bytes), the probe-on-dipole flag at `flag`.
static gdm_status fields_core(gdm_ctx* c, int64_t nrhs, const double* q, int64_t P, const double* rp, double* E,
                              double* H, void* part, size_t part_cap, int* flag_dev, int nsplit, bool prof,
                              const double* khat = nullptr, const double* e0 = nullptr) {
  const Wave w = wave_of(c, c->wavelength);
  const DipoleView d = view_of(c, make_double2(0, 0));
  if (fields_scratch_bytes(nrhs, P, nsplit, H != nullptr) > part_cap)
    FAIL(c, GDM_E_ARG, "fields scratch too small");
  hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, c->stream, flag_dev, 1, 0);
  HIPCHK(c, hipGetLastError());
  const double rmin = 1e-9 * c->step;
  if (prof) HIPCHK(c, c->prof.begin(c->stream, PROF_FIELDS, (double)P * (double)c->N * (double)nrhs));
  HIPCHK(c, launch_fields(d, w, reinterpret_cast<const double2*>(q), c->n, nrhs, rp, P, reinterpret_cast<double2*>(E),
                          reinterpret_cast<double2*>(H), static_cast<double2*>(part), nsplit, rmin * rmin, flag_dev,
                          c->stream));
  if (prof) HIPCHK(c, c->prof.end(c->stream));
  if (khat)  // total field: add the incident plane waves
    HIPCHK(c, launch_planewave_points(w, c->n_env, nrhs, khat, reinterpret_cast<const double2*>(e0), rp, P,
                                      reinterpret_cast<double2*>(E), reinterpret_cast<double2*>(H), c->stream, true));
  int flag = 0;
  HIPCHK(c, hipMemcpyAsync(&flag, flag_dev, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (flag) FAIL(c, GDM_E_PROBE_AT_DIPOLE, "a probe point lies on a dipole (|R| < 1e-9 step)");
  return GDM_OK;
}

static gdm_status fields_check(gdm_ctx* c, int64_t nrhs, const double* q, int64_t P, const double* rp,
                               const double* E) {
  if (c->wavelength <= 0) FAIL(c, GDM_E_STATE, "no wavelength set (call gdm_factorize first)");
  if (nrhs <= 0 || P < 0 || !q || (P > 0 && (!rp || !E))) FAIL(c, GDM_E_ARG, "bad field arguments");
  if ((P + 255) / 256 > (int64_t)INT32_MAX) FAIL(c, GDM_E_ARG, "too many probes");
  return GDM_OK;
}

extern "C" {

gdm_status gdm_fields(gdm_ctx* c, int64_t nrhs, const double* q, int64_t P, const double* rp, double* E, double* H) {
  if (!c) return GDM_E_ARG;
  gdm_status s = fields_check(c, nrhs, q, P, rp, E);
  if (s != GDM_OK || P == 0) return s;
  HIPCHK(c, hipSetDevice(c->device));
  const int nsplit = fields_num_splits(P, c->N, c->num_cu);
  const size_t need = fields_scratch_bytes(nrhs, P, nsplit, H != nullptr);
  if (need > 0) HIPCHK(c, c->scratch.ensure(need));
  HIPCHK(c, c->flag.ensure(sizeof(int) * 4));
  return fields_core(c, nrhs, q, P, rp, E, H, c->scratch.p, c->scratch.cap, c->flag.as<int>(), nsplit, true);
}

gdm_status gdm_fields_total(gdm_ctx* c, int64_t nrhs, const double* q, const double* khat, const double* e0,
                            int64_t P, const double* rp, double* E, double* H) {
  if (!c) return GDM_E_ARG;
  gdm_status s = fields_check(c, nrhs, q, P, rp, E);
  if (s != GDM_OK || P == 0) return s;
  if (!khat || !e0) FAIL(c, GDM_E_ARG, "khat and e0 are required");
  HIPCHK(c, hipSetDevice(c->device));
  const int nsplit = fields_num_splits(P, c->N, c->num_cu);
  const size_t need = fields_scratch_bytes(nrhs, P, nsplit, H != nullptr);
  if (need > 0) HIPCHK(c, c->scratch.ensure(need));
  HIPCHK(c, c->flag.ensure(sizeof(int) * 4));
  return fields_core(c, nrhs, q, P, rp, E, H, c->scratch.p, c->scratch.cap, c->flag.as<int>(), nsplit, true, khat,
                     e0);
}

gdm_status gdm_planewave_intensity(gdm_ctx* c, int64_t n_pw, const double* e0, double* out) {
  if (!c) return GDM_E_ARG;
  if (n_pw <= 0 || !e0 || !out) FAIL(c, GDM_E_ARG, "need n_pw > 0, e0 and out");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, launch_pw_intensity(n_pw, reinterpret_cast<const double2*>(e0), out, c->stream));
  return GDM_OK;
}

gdm_status gdm_fields_noalloc(gdm_ctx* c, int64_t nrhs, const double* q, int64_t P, const double* rp, double* E,
                              double* H) {
  if (!c) return GDM_E_ARG;
  gdm_status s = fields_check(c, nrhs, q, P, rp, E);
  if (s != GDM_OK || P == 0) return s;
  void* base = noalloc_scratch(c->device);
  if (!base) FAIL(c, GDM_E_DEVICE, "no address of the static scratch array on device %d", c->device);
  HIPCHK(c, hipSetDevice(c->device));
  const int nsplit = fields_num_splits(P, c->N, c->num_cu);
  const size_t need = fields_scratch_bytes(nrhs, P, nsplit, H != nullptr);
  if (need > GDM_NOALLOC_SCRATCH_BYTES - NOALLOC_FLAG_BYTES)
    FAIL(c, GDM_E_ARG,
         "gdm_fields_noalloc needs %zu bytes of scratch for %lld RHS x %lld probes (%d dipole splits); the static "
         "array holds %zu",
         need, (long long)nrhs, (long long)P, nsplit, (size_t)(GDM_NOALLOC_SCRATCH_BYTES - NOALLOC_FLAG_BYTES));
  char* b = static_cast<char*>(base);
  return fields_core(c, nrhs, q, P, rp, E, H, b + NOALLOC_FLAG_BYTES, GDM_NOALLOC_SCRATCH_BYTES - NOALLOC_FLAG_BYTES,
                     reinterpret_cast<int*>(b), nsplit, false);
}

gdm_status gdm_multipoles(gdm_ctx* c, int64_t n_rhs, const double* q, const double* r0, const double* khat,
                          const double* e0, double* moments, double* sigma) {
  if (!c) return GDM_E_ARG;
  if (c->N <= 0) FAIL(c, GDM_E_STATE, "gdm_multipoles before gdm_set_structure");
  if (c->wavelength <= 0) FAIL(c, GDM_E_STATE, "no wavelength set (gdm_factorize or gdm_set_wavelength first)");
  if (n_rhs <= 0 || !q || (!moments && !sigma)) FAIL(c, GDM_E_ARG, "need n_rhs > 0, q, and moments or sigma");
  if (n_rhs > 65535) FAIL(c, GDM_E_ARG, "at most 65535 right-hand sides per call");
  if ((khat == nullptr) != (e0 == nullptr)) FAIL(c, GDM_E_ARG, "khat and e0 are given together or not at all");
  if (c->nc <= 0) FAIL(c, GDM_E_ARG, "the structure has no mesh cells (multipoles of the discretised part only)");
  HIPCHK(c, hipSetDevice(c->device));
  double rc[3] = {0.0, 0.0, 0.0};
  if (r0) {
    for (int a = 0; a < 3; ++a) rc[a] = r0[a];
    if (!std::isfinite(rc[0]) || !std::isfinite(rc[1]) || !std::isfinite(rc[2])) FAIL(c, GDM_E_ARG, "r0 not finite");
  } else {
    // the mean position of the cells, summed in order on the host
    std::vector<double> hp((size_t)3 * c->nc);
    HIPCHK(c, hipMemcpyAsync(hp.data(), c->pos.p, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int64_t j = 0; j < c->nc; ++j)
      for (int a = 0; a < 3; ++a) rc[a] += hp[3 * j + a];
    for (int a = 0; a < 3; ++a) rc[a] /= (double)c->nc;
  }
  const Wave w = wave_of(c, c->wavelength);
  const int ns = multipole_num_splits(c->nc, c->num_cu, n_rhs);
  HIPCHK(c, c->part.ensure(multipole_scratch_bytes(n_rhs, ns)));
  HIPCHK(c, launch_multipoles(c->pos.as<double>(), c->nc, reinterpret_cast<const double2*>(q), c->n, n_rhs, rc, w.k,
                              w.k0, c->n_env, khat, reinterpret_cast<const double2*>(e0), ns, c->part.as<double>(),
                              reinterpret_cast<double2*>(moments), sigma, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return GDM_OK;
}

gdm_status gdm_cross_sections(gdm_ctx* c, int64_t nrhs, const double* f0, const double* q, const double* f,
                              const double* e0_norm2, int32_t want_ff, double* out) {
  if (!c) return GDM_E_ARG;
  if (c->wavelength <= 0) FAIL(c, GDM_E_STATE, "no wavelength set (call gdm_factorize first)");
  if (nrhs <= 0 || !f0 || !q || !f || !e0_norm2 || !out) FAIL(c, GDM_E_ARG, "bad cross-section arguments");
  if (nrhs > 65535) FAIL(c, GDM_E_ARG, "at most 65535 right-hand sides per call");
  HIPCHK(c, hipSetDevice(c->device));
  const Wave w = wave_of(c, c->wavelength);
  const DipoleView d = view_of(c, make_double2(0, 0));
  const int64_t nblk = sca_ff_blocks(c->N);
  const int64_t ng = c->n_gpm;
  HIPCHK(c, c->small.ensure(sizeof(double) * std::max<int64_t>(5 * nrhs + nrhs * (nblk + ng), 4 * nrhs)));
  double* sums = c->small.as<double>();
  double* mutual = sums + 5 * nrhs;  // [nrhs][ng], GPM groups only
  double* part = mutual + nrhs * ng;
  HIPCHK(c, launch_cs_sums(d, reinterpret_cast<const double2*>(f0), reinterpret_cast<const double2*>(q),
                           reinterpret_cast<const double2*>(f), c->n, nrhs, sums, c->stream));
  HIPCHK(c, launch_gpm_mutual(d, w, reinterpret_cast<const double2*>(q), c->n, nrhs, mutual, c->stream));
  if (want_ff)
    HIPCHK(c, launch_sca_ff(d, w, reinterpret_cast<const double2*>(q), c->n, nrhs, part, nblk, c->stream));
  std::vector<double> h(5 * nrhs + nrhs * ng + (want_ff ? nrhs * nblk : 0)), e2(nrhs);
  HIPCHK(c, hipMemcpyAsync(h.data(), sums, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(e2.data(), e0_norm2, sizeof(double) * nrhs, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::vector<double> o(5 * nrhs);
  const double k3 = (2.0 / 3.0) * w.k * w.k * w.k;
  for (int64_t r = 0; r < nrhs; ++r) {
    if (!(e2[r] > 0)) FAIL(c, GDM_E_ARG, "|E0|^2 of RHS %lld is not > 0", (long long)r);
    const double C = 4.0 * M_PI * w.k0 / (c->n_env * e2[r]);
    const double* s = &h[5 * r];
    double mg = 0.0;  // the GPM groups' mutual radiation
    for (int64_t g = 0; g < ng; ++g) mg += h[5 * nrhs + r * ng + g];
    const double ext = C * s[0];
    const double ab = C * (s[1] - k3 * (s[3] / w.eps_env + s[4]) - mg);
    const double rad = C * k3 * ((s[2] + s[3]) / w.eps_env + s[4]);
    o[5 * r + 0] = ext;
    o[5 * r + 1] = ext - ab;
    o[5 * r + 2] = ab;
    o[5 * r + 3] = rad;
    if (want_ff) {
      double off = 0;
      for (int64_t b = 0; b < nblk; ++b) off += h[5 * nrhs + nrhs * ng + r * nblk + b];
      o[5 * r + 4] = C * off + rad;
    } else {
      o[5 * r + 4] = NAN;
    }
  }
  HIPCHK(c, hipMemcpyAsync(out, o.data(), sizeof(double) * o.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return GDM_OK;
}

gdm_status gdm_dipole_sources(gdm_ctx* c, int64_t n_src, const double* r_src, const double* d_src, double* f0) {
  if (!c) return GDM_E_ARG;
  if (c->wavelength <= 0) FAIL(c, GDM_E_STATE, "no wavelength set (gdm_factorize or gdm_set_wavelength first)");
  if (n_src <= 0 || !r_src || !d_src || !f0) FAIL(c, GDM_E_ARG, "need n_src > 0, r_src, d_src and f0");
  if (n_src > 65535) FAIL(c, GDM_E_ARG, "at most 65535 sources per call");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, c->flag.ensure(sizeof(int) * 4));
  hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, c->stream, c->flag.as<int>(), 1, 0);
  const Wave w = wave_of(c, c->wavelength);
  const double rmin = 1e-9 * c->step;
  HIPCHK(c, launch_dipole_sources(view_of(c, make_double2(0, 0)), w, c->n, n_src, r_src,
                                  reinterpret_cast<const double2*>(d_src), reinterpret_cast<double2*>(f0), rmin * rmin,
                                  c->flag.as<int>(), c->stream));
  int flag = 0;
  HIPCHK(c, hipMemcpyAsync(&flag, c->flag.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (flag) FAIL(c, GDM_E_PROBE_AT_DIPOLE, "a source point lies on a dipole (|R| < 1e-9 step)");
  return GDM_OK;
}

}  // extern "C"

// The six unit sources (p_x, p_y, p_z, m_x, m_y, m_z) at each of n_src points:
// their incident fields, the solve with the context's factors, q = A F.  On
// return *Q points to the moments [6 n_src][n] (inside c->src; *extra bytes
// after them are free for the caller).
static gdm_status unit_source_moments(gdm_ctx* c, int64_t S, const double* r_src, double tol, int32_t max_iter,
                                      size_t extra, double2** Q, char** extra_p, SolveStats& ss) {
  const int64_t n = c->n, nr = 6 * S;
  const size_t b_pos = (size_t)nr * 3 * sizeof(double), b_d = (size_t)nr * 6 * sizeof(double2);
  const size_t b_vec = (size_t)nr * n * sizeof(double2);
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  HIPCHK(c, c->src.ensure(al(b_pos) + al(b_d) + 2 * al(b_vec) + al(extra)));
  char* base = static_cast<char*>(c->src.p);
  double* dpos = reinterpret_cast<double*>(base);
  double2* dvec = reinterpret_cast<double2*>(base + al(b_pos));
  double2* F0 = reinterpret_cast<double2*>(base + al(b_pos) + al(b_d));
  *Q = reinterpret_cast<double2*>(base + al(b_pos) + al(b_d) + al(b_vec));
  *extra_p = base + al(b_pos) + al(b_d) + 2 * al(b_vec);
  // positions repeated six times and unit moments (the identity), set up on the host
  std::vector<double> hpos((size_t)nr * 3);
  std::vector<double2> hd((size_t)nr * 6, make_double2(0, 0));
  std::vector<double> rs((size_t)S * 3);
  HIPCHK(c, hipMemcpyAsync(rs.data(), r_src, sizeof(double) * 3 * S, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int64_t r = 0; r < nr; ++r) {
    for (int a = 0; a < 3; ++a) hpos[3 * r + a] = rs[3 * (r / 6) + a];
    hd[6 * r + r % 6] = make_double2(1.0, 0.0);
  }
  HIPCHK(c, hipMemcpyAsync(dpos, hpos.data(), b_pos, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(dvec, hd.data(), b_d, hipMemcpyHostToDevice, c->stream));
  gdm_status s = gdm_dipole_sources(c, nr, dpos, reinterpret_cast<const double*>(dvec), reinterpret_cast<double*>(F0));
  if (s != GDM_OK) return s;
  HIPCHK(c, c->X.ensure(sizeof(double2) * n * nr));
  double2* X = c->X.as<double2>();
  s = solve_core(c, 0, nr, F0, X, tol, max_iter, ss);
  if (s != GDM_OK && s != GDM_E_NOCONV) return s;
  HIPCHK(c, launch_apply_alpha(view_of(c, make_double2(0, 0)), X, n, *Q, n, nr, c->stream));
  return s;
}

extern "C" {

gdm_status gdm_ldos(gdm_ctx* c, int64_t n_src, const double* r_src, double tol, int32_t max_iter, double* out,
                    gdm_info* info) {
  if (!c) return GDM_E_ARG;
  if (!c->factored) FAIL(c, GDM_E_STATE, "gdm_ldos before gdm_factorize");
  if (n_src <= 0 || !r_src || !out) FAIL(c, GDM_E_ARG, "need n_src > 0, r_src and out");
  if (n_src > 10922) FAIL(c, GDM_E_ARG, "at most 10922 source points per call");
  HIPCHK(c, hipSetDevice(c->device));
  double2* Q = nullptr;
  char* ex = nullptr;
  SolveStats ss;
  const gdm_status s = unit_source_moments(c, n_src, r_src, tol, max_iter, 0, &Q, &ex, ss);
  if (s != GDM_OK && s != GDM_E_NOCONV) return s;
  HIPCHK(c, launch_ldos(view_of(c, make_double2(0, 0)), wave_of(c, c->wavelength), Q, c->n, n_src, r_src, out,
                        c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (info) {
    info->ir_iters = ss.iters;
    info->backward_err = ss.be;
    info->bad_index = -1;
  }
  if (s == GDM_E_NOCONV) FAIL(c, GDM_E_NOCONV, "refinement stopped at backward error %.3e > tol %.3e", ss.be, ss.tol);
  return GDM_OK;
}

gdm_status gdm_green_tensor(gdm_ctx* c, int64_t n_src, const double* r_src, int64_t n_pts, const double* r_pts,
                            double tol, int32_t max_iter, double* G, gdm_info* info) {
  if (!c) return GDM_E_ARG;
  if (!c->factored) FAIL(c, GDM_E_STATE, "gdm_green_tensor before gdm_factorize");
  if (n_src <= 0 || n_pts <= 0 || !r_src || !r_pts || !G) FAIL(c, GDM_E_ARG, "bad Green's tensor arguments");
  if (n_src > 10922) FAIL(c, GDM_E_ARG, "at most 10922 source points per call");
  if ((n_src * n_pts * 36 + 255) / 256 > (int64_t)INT32_MAX) FAIL(c, GDM_E_ARG, "too many source-point pairs");
  HIPCHK(c, hipSetDevice(c->device));
  const int64_t nr = 6 * n_src;
  const int nsplit = fields_num_splits(n_pts, c->N, c->num_cu);
  const size_t b_f = sizeof(double2) * (size_t)nr * n_pts * 3;
  const size_t part = fields_scratch_bytes(nr, n_pts, nsplit, true);
  double2* Q = nullptr;
  char* ex = nullptr;
  SolveStats ss;
  const gdm_status s = unit_source_moments(c, n_src, r_src, tol, max_iter, 2 * b_f + part + 256, &Q, &ex, ss);
  if (s != GDM_OK && s != GDM_E_NOCONV) return s;
  double2* E = reinterpret_cast<double2*>(ex);
  double2* H = E + (size_t)nr * n_pts * 3;
  void* pbuf = reinterpret_cast<char*>(H + (size_t)nr * n_pts * 3);
  HIPCHK(c, c->flag.ensure(sizeof(int) * 4));
  const gdm_status sf = fields_core(c, nr, reinterpret_cast<const double*>(Q), n_pts, r_pts,
                                    reinterpret_cast<double*>(E), reinterpret_cast<double*>(H), pbuf, part + 256,
                                    c->flag.as<int>(), nsplit, true);
  if (sf != GDM_OK) return sf;
  HIPCHK(c, launch_green_gather(E, H, n_src, n_pts, reinterpret_cast<double2*>(G), c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (info) {
    info->ir_iters = ss.iters;
    info->backward_err = ss.be;
    info->bad_index = -1;
  }
  if (s == GDM_E_NOCONV) FAIL(c, GDM_E_NOCONV, "refinement stopped at backward error %.3e > tol %.3e", ss.be, ss.tol);
  return GDM_OK;
}

gdm_status gdm_extract_dipole_pair(gdm_ctx* c, int64_t n_pw, const double* khat, const double* e0, int64_t n_src,
                                   const double* r_src, const double* d_src, const double* r0, double tol,
                                   int32_t max_iter, double* alpha, double* resid, gdm_info* info) {
  if (!c) return GDM_E_ARG;
  if (!c->factored) FAIL(c, GDM_E_STATE, "gdm_extract_dipole_pair before gdm_factorize");
  if (c->nc <= 0) FAIL(c, GDM_E_ARG, "the structure has no mesh cells");
  if (n_pw < 0 || n_src < 0 || (n_pw > 0 && (!khat || !e0)) || (n_src > 0 && (!r_src || !d_src)) || !alpha)
    FAIL(c, GDM_E_ARG, "bad illumination or output arguments");
  const int64_t N = n_pw + n_src;
  if (N < 6 || N > 4096) FAIL(c, GDM_E_ARG, "need 6 to 4096 illuminations (got %lld)", (long long)N);
  HIPCHK(c, hipSetDevice(c->device));
  double rc[3] = {0.0, 0.0, 0.0};
  if (r0) {
    for (int a = 0; a < 3; ++a) rc[a] = r0[a];
  } else {
    std::vector<double> hp((size_t)3 * c->nc);
    HIPCHK(c, hipMemcpyAsync(hp.data(), c->pos.p, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int64_t j = 0; j < c->nc; ++j)
      for (int a = 0; a < 3; ++a) rc[a] += hp[3 * j + a];
    for (int a = 0; a < 3; ++a) rc[a] /= (double)c->nc;
  }
  const int64_t n = c->n;
  // F0 [N][n], Q [N][n], moments [N][24], F0 at r0 [N][6], work [N][6], residual
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t b_vec = sizeof(double2) * (size_t)N * n, b_mom = sizeof(double2) * (size_t)N * 24,
               b_six = sizeof(double2) * (size_t)N * 6;
  HIPCHK(c, c->src.ensure(2 * al(b_vec) + al(b_mom) + 2 * al(b_six) + 256));
  char* base = static_cast<char*>(c->src.p);
  double2* F0 = reinterpret_cast<double2*>(base);
  double2* Q = reinterpret_cast<double2*>(base + al(b_vec));
  double2* mom = reinterpret_cast<double2*>(base + 2 * al(b_vec));
  double2* A6 = reinterpret_cast<double2*>(base + 2 * al(b_vec) + al(b_mom));
  double2* B6 = reinterpret_cast<double2*>(base + 2 * al(b_vec) + al(b_mom) + al(b_six));
  double* dres = reinterpret_cast<double*>(base + 2 * al(b_vec) + al(b_mom) + 2 * al(b_six));
  const Wave w = wave_of(c, c->wavelength);
  const DipoleView d = view_of(c, make_double2(0, 0));
  if (n_pw > 0)
    HIPCHK(c, launch_incident(d, w, c->n_env, n_pw, khat, reinterpret_cast<const double2*>(e0), F0, n, c->stream));
  if (n_src > 0) {
    gdm_status s = gdm_dipole_sources(c, n_src, r_src, d_src, reinterpret_cast<double*>(F0 + (size_t)n_pw * n));
    if (s != GDM_OK) return s;
  }
  HIPCHK(c, c->X.ensure(sizeof(double2) * n * N));
  double2* X = c->X.as<double2>();
  SolveStats ss;
  gdm_status s = solve_core(c, 0, N, F0, X, tol, max_iter, ss);
  if (s != GDM_OK && s != GDM_E_NOCONV) return s;
  HIPCHK(c, launch_apply_alpha(d, X, n, Q, n, N, c->stream));
  const int ns = multipole_num_splits(c->nc, c->num_cu, N);
  HIPCHK(c, c->part.ensure(multipole_scratch_bytes(N, ns)));
  HIPCHK(c, launch_multipoles(c->pos.as<double>(), c->nc, Q, n, N, rc, w.k, w.k0, c->n_env, nullptr, nullptr, ns,
                              c->part.as<double>(), mom, nullptr, c->stream));
  HIPCHK(c, launch_pair_extract(w, c->n_env, rc, n_pw, khat, reinterpret_cast<const double2*>(e0), n_src, r_src,
                                reinterpret_cast<const double2*>(d_src), mom, A6, B6,
                                reinterpret_cast<double2*>(alpha), dres, c->stream));
  double hres = 0.0;
  double2 ha[36];
  HIPCHK(c, hipMemcpyAsync(&hres, dres, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(ha, alpha, sizeof(ha), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (resid) *resid = hres;
  if (info) {
    info->ir_iters = ss.iters;
    info->backward_err = ss.be;
    info->bad_index = -1;
  }
  for (int i = 0; i < 36; ++i)
    if (!std::isfinite(ha[i].x) || !std::isfinite(ha[i].y))
      FAIL(c, GDM_E_ARG, "the illuminations do not determine the model (rank-deficient fields at r0)");
  if (s == GDM_E_NOCONV) FAIL(c, GDM_E_NOCONV, "refinement stopped at backward error %.3e > tol %.3e", ss.be, ss.tol);
  return GDM_OK;
}

gdm_status gdm_extract_gpm(gdm_ctx* c, int64_t n_pw, const double* khat, const double* e0, int64_t n_src,
                           const double* r_src, const double* d_src, int64_t n_pairs, const double* r_gpm,
                           int64_t n_probe, const double* r_probe, double tol, int32_t max_iter, double* alpha,
                           double* resid, gdm_info* info) {
  if (!c) return GDM_E_ARG;
  if (!c->factored) FAIL(c, GDM_E_STATE, "gdm_extract_gpm before gdm_factorize");
  if (n_pw < 0 || n_src < 0 || (n_pw > 0 && (!khat || !e0)) || (n_src > 0 && (!r_src || !d_src)) || !alpha ||
      !r_gpm || !r_probe)
    FAIL(c, GDM_E_ARG, "bad illumination, position or output arguments");
  if (n_pairs < 1 || n_pairs > GPM_MAX_PAIRS) FAIL(c, GDM_E_ARG, "n_pairs must be in [1, %d]", GPM_MAX_PAIRS);
  const int64_t N = n_pw + n_src, K = 6 * n_pairs, P = n_probe;
  if (N < K || N > 4096) FAIL(c, GDM_E_ARG, "need 6 n_pairs (%lld) to 4096 illuminations (got %lld)", (long long)K, (long long)N);
  if (P < n_pairs || P > (1 << 20)) FAIL(c, GDM_E_ARG, "need n_pairs to 2^20 probes (got %lld)", (long long)P);
  HIPCHK(c, hipSetDevice(c->device));
  const int64_t n = c->n, m1 = 6 * P;
  // F0 [N][n], Q [N][n], E, H [N][P][3], Gf (m1 x K), Y (m1 x N), X1 (K x N),
  // F0g (N x K), PB (N x K), rdiag [K], norms [2][N] and [2][K]
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t z = sizeof(double2);
  const size_t sizes[] = {z * N * n, z * N * n, z * N * P * 3, z * N * P * 3, z * m1 * K, z * m1 * N,
                          z * K * N, z * N * K, z * N * K, z * K, sizeof(double) * 2 * N, sizeof(double) * 2 * K};
  size_t offs[12], tot = 0;
  for (int i = 0; i < 12; ++i) {
    offs[i] = tot;
    tot += al(sizes[i]);
  }
  HIPCHK(c, c->src.ensure(tot));
  char* base = static_cast<char*>(c->src.p);
  double2* F0 = reinterpret_cast<double2*>(base + offs[0]);
  double2* Q = reinterpret_cast<double2*>(base + offs[1]);
  double2* E = reinterpret_cast<double2*>(base + offs[2]);
  double2* H = reinterpret_cast<double2*>(base + offs[3]);
  double2* Gf = reinterpret_cast<double2*>(base + offs[4]);
  double2* Y = reinterpret_cast<double2*>(base + offs[5]);
  double2* X1 = reinterpret_cast<double2*>(base + offs[6]);
  double2* F0g = reinterpret_cast<double2*>(base + offs[7]);
  double2* PB = reinterpret_cast<double2*>(base + offs[8]);
  double2* rdiag = reinterpret_cast<double2*>(base + offs[9]);
  double* nrm1 = reinterpret_cast<double*>(base + offs[10]);
  double* nrm2 = reinterpret_cast<double*>(base + offs[11]);
  const Wave w = wave_of(c, c->wavelength);
  const DipoleView d = view_of(c, make_double2(0, 0));
  if (n_pw > 0)
    HIPCHK(c, launch_incident(d, w, c->n_env, n_pw, khat, reinterpret_cast<const double2*>(e0), F0, n, c->stream));
  if (n_src > 0) {
    gdm_status s = gdm_dipole_sources(c, n_src, r_src, d_src, reinterpret_cast<double*>(F0 + (size_t)n_pw * n));
    if (s != GDM_OK) return s;
  }
  HIPCHK(c, c->X.ensure(sizeof(double2) * n * N));
  double2* X = c->X.as<double2>();
  SolveStats ss;
  gdm_status s = solve_core(c, 0, N, F0, X, tol, max_iter, ss);
  if (s != GDM_OK && s != GDM_E_NOCONV) return s;
  HIPCHK(c, launch_apply_alpha(d, X, n, Q, n, N, c->stream));
  gdm_status sf = gdm_fields(c, N, reinterpret_cast<const double*>(Q), P, r_probe, reinterpret_cast<double*>(E),
                             reinterpret_cast<double*>(H));
  if (sf != GDM_OK) return sf;
  // moments of the pairs: min || Gf X1 - Y || over all illuminations at once
  HIPCHK(c, launch_gpm_pack_fields(E, H, N, P, Y, c->stream));
  HIPCHK(c, launch_gpm_fit_matrix(w, r_probe, P, r_gpm, n_pairs, Gf, c->stream));
  HIPCHK(c, launch_qr_lsq(Gf, m1, (int)K, Y, (int)N, X1, rdiag, nrm1, c->stream));
  // alpha_G: min || F0g X2 - PB ||, PB = X1^T; X2 (column-major K x K) is alpha_G row-major
  HIPCHK(c, launch_gpm_illumination(w, c->n_env, r_gpm, n_pairs, n_pw, khat, reinterpret_cast<const double2*>(e0),
                                    n_src, r_src, reinterpret_cast<const double2*>(d_src), F0g, c->stream));
  HIPCHK(c, launch_transpose(X1, K, N, PB, c->stream));
  HIPCHK(c, launch_qr_lsq(F0g, N, (int)K, PB, (int)K, reinterpret_cast<double2*>(alpha), rdiag, nrm2, c->stream));
  std::vector<double> h1(2 * N), h2(2 * K);
  std::vector<double2> ha((size_t)K * K);
  HIPCHK(c, hipMemcpyAsync(h1.data(), nrm1, sizeof(double) * h1.size(), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(h2.data(), nrm2, sizeof(double) * h2.size(), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(ha.data(), alpha, sizeof(double2) * ha.size(), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double b1 = 0, r1 = 0, b2 = 0, r2 = 0;
  for (int64_t i = 0; i < N; ++i) b1 += h1[i], r1 += h1[N + i];
  for (int64_t i = 0; i < K; ++i) b2 += h2[i], r2 += h2[K + i];
  if (resid) {
    resid[0] = b1 > 0 ? std::sqrt(r1 / b1) : 0.0;
    resid[1] = b2 > 0 ? std::sqrt(r2 / b2) : 0.0;
  }
  if (info) {
    info->ir_iters = ss.iters;
    info->backward_err = ss.be;
    info->bad_index = -1;
  }
  for (const double2& v : ha)
    if (!std::isfinite(v.x) || !std::isfinite(v.y))
      FAIL(c, GDM_E_ARG, "the probes or the illuminations do not determine the model (rank-deficient fit)");
  if (s == GDM_E_NOCONV) FAIL(c, GDM_E_NOCONV, "refinement stopped at backward error %.3e > tol %.3e", ss.be, ss.tol);
  return GDM_OK;
}

gdm_status gdm_getrf(gdm_ctx* c, int dtype, int64_t n, void* A, int64_t lda, int32_t* ipiv, gdm_info* info) {
  if (!c) return GDM_E_ARG;
  if (dtype != 0 && dtype != 1) FAIL(c, GDM_E_ARG, "dtype must be 0 or 1");
  if (n <= 0 || n > (int64_t)INT32_MAX / 4 || !A || !ipiv || lda < n) FAIL(c, GDM_E_ARG, "bad getrf arguments");
  HIPCHK(c, hipSetDevice(c->device));
  DevBuf dummy;
  gdm_status s = dtype == 0 ? run_lu<double>(c, A, n, lda, c->ext_plan, c->ext_ws, dummy, ipiv, info)
                            : run_lu<float>(c, A, n, lda, c->ext_plan, c->ext_ws, dummy, ipiv, info);
  c->ext_dtype = (s == GDM_OK || s == GDM_E_SINGULAR) ? dtype : -1;
  return s;
}

gdm_status gdm_getrs(gdm_ctx* c, int dtype, int trans, int64_t n, int64_t nrhs, const void* A, int64_t lda, void* B,
                     int64_t ldb) {
  if (!c) return GDM_E_ARG;
  if (c->ext_dtype != dtype || c->ext_plan.n != n) FAIL(c, GDM_E_STATE, "gdm_getrs without a matching gdm_getrf");
  if (nrhs < 0 || !A || (nrhs > 0 && !B) || lda < n || ldb < n || (trans != 0 && trans != 1))
    FAIL(c, GDM_E_ARG, "bad getrs arguments");
  if (nrhs > 65535) FAIL(c, GDM_E_ARG, "at most 65535 right-hand sides per call");
  HIPCHK(c, hipSetDevice(c->device));
  LUWork w;
  lu_workspace_carve(c->ext_ws.p, c->ext_plan, dtype == 0 ? 8 : 4, c->num_cu, w);
  if (dtype == 0) HIPCHK(c, lu_solve<double>(trans, A, lda, c->ext_plan, w, B, ldb, nrhs, c->stream));
  else HIPCHK(c, lu_solve<float>(trans, A, lda, c->ext_plan, w, B, ldb, nrhs, c->stream));
  return GDM_OK;
}

gdm_status gdm_gemm(gdm_ctx* c, int dtype, int mode, int transA, int64_t m, int64_t n, int64_t k, const void* A,
                    int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc) {
  if (!c) return GDM_E_ARG;
  if ((dtype != 0 && dtype != 1) || (mode != 0 && mode != 1) || (transA != 0 && transA != 1))
    FAIL(c, GDM_E_ARG, "bad gemm mode");
  if (m < 0 || n < 0 || k < 0 || !A || !B || !C) FAIL(c, GDM_E_ARG, "bad gemm arguments");
  if (ldc < m || ldb < k || lda < (transA ? k : m)) FAIL(c, GDM_E_ARG, "bad gemm leading dimensions");
  HIPCHK(c, hipSetDevice(c->device));
  if (dtype == 0) HIPCHK(c, launch_gemm<double>(mode, transA, m, n, k, A, lda, B, ldb, C, ldc, c->stream));
  else HIPCHK(c, launch_gemm<float>(mode, transA, m, n, k, A, lda, B, ldb, C, ldc, c->stream));
  return GDM_OK;
}

gdm_status gdm_profile_mask(gdm_ctx* c, int32_t mask) {
  if (!c) return GDM_E_ARG;
  if (mask < 0 || mask >= (1 << PROF_NTAGS)) FAIL(c, GDM_E_ARG, "tag mask %d outside [0, 2^%d)", mask, PROF_NTAGS);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->prof.collect();
  c->prof.reset();
  c->prof.mask = (uint32_t)mask;
  return GDM_OK;
}

gdm_status gdm_profile(gdm_ctx* c, int enable) { return gdm_profile_mask(c, enable ? (1 << PROF_NTAGS) - 1 : 0); }

gdm_status gdm_profile_read(gdm_ctx* c, double* out, int32_t n_out) {
  if (!c) return GDM_E_ARG;
  if (!out || n_out < 3 * PROF_NTAGS) FAIL(c, GDM_E_ARG, "need a host array of at least %d doubles", 3 * PROF_NTAGS);
  for (int i = 0; i < n_out; ++i) out[i] = 0.0;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->prof.collect();
  for (int t = 0; t < PROF_NTAGS; ++t) {
    out[3 * t + 0] = c->prof.ms[t];
    out[3 * t + 1] = c->prof.wsum[t];
    out[3 * t + 2] = c->prof.cnt[t];
  }
  return GDM_OK;
}

}  // extern "C"
