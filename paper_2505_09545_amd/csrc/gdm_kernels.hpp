// Host-side launch declarations shared by the kernel files and the C-ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include "gdm_common.hpp"
#include <cstdint>
#include <vector>

namespace gdm {

// Dipoles in device memory: N = nc cells followed by ne effective ED+MD dipoles.
struct DipoleView {
  const double* pos;       // [N][3] nm
  const double2* alpha_c;  // [nc] cell polarisability (times I3)
  const double2* alpha6;   // [ne][6][6] row-major effective polarisability
  int64_t N, nc, ne;
  double2 self_c;          // S^Ep of a cell (times I3)
  // Global polarisability matrices over runs of effective dipoles (ngroups 0:
  // none).  gid [ne]: group of each effective dipole, -1 for a local one;
  // gtab [ngroups][3]: (first effective index, size M, offset of the group's
  // matrix in galpha); galpha: row-major 6M x 6M complex matrices, rows and
  // columns ordered (member, then p_x..p_z, m_x..m_z).  A member's own alpha6
  // is not used; members of one group do not couple through G~.
  const int32_t* gid = nullptr;
  const int64_t* gtab = nullptr;
  const double2* galpha = nullptr;
  int64_t ngroups = 0;
};

// largest number of dipole pairs in one GPM group
constexpr int GPM_MAX_PAIRS = 32;

// The 3 x NC block of M = I - G~ A at row dipole dr (field f: 0 electric, 1
// magnetic) and column dipole j (NC = 3 columns for a cell, 6 for an effective
// dipole: its electric then magnetic columns): v[column][row].  Diagonal blocks
// I - S alpha (cells) or the identity rows (effective dipoles, S = 0);
// off-diagonal blocks -G^{f.}(r_dr - r_j) alpha_j.  FP64, one sincos.
// A GPM member column j takes alpha_j = I here (the group's matrix is applied
// to its columns afterwards) and a zero block against the other members.
template <bool EFF>
__device__ inline void m_block(const DipoleView& d, const Wave& w, int64_t dr, int f, int64_t j,
                               double2 (&v)[EFF ? 6 : 3][3]) {
  constexpr int NC = EFF ? 6 : 3;
  const int64_t nc = d.nc;
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int a = 0; a < 3; ++a) v[c][a] = make_double2(0.0, 0.0);
  if (dr == j) {
    // diagonal block I - S alpha (cells: scalar S^Ep and alpha; effective: S = 0)
    if (!EFF) {
      const double2 dg = csub(make_double2(1.0, 0.0), cmul(d.self_c, d.alpha_c[j]));
#pragma unroll
      for (int a = 0; a < 3; ++a) v[a][a] = dg;
    } else {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        v[a][a] = make_double2(f == 0 ? 1.0 : 0.0, 0.0);
        v[(3 + a) % NC][a] = make_double2(f == 1 ? 1.0 : 0.0, 0.0);
      }
    }
    return;
  }
  bool unit_alpha = false;
  if (EFF && d.gid) {
    const int32_t gj = d.gid[j - nc];
    if (gj >= 0) {
      if (dr >= nc && d.gid[dr - nc] == gj) return;  // same group: no coupling
      unit_alpha = true;
    }
  }
  const double Rx = d.pos[3 * dr + 0] - d.pos[3 * j + 0];
  const double Ry = d.pos[3 * dr + 1] - d.pos[3 * j + 1];
  const double Rz = d.pos[3 * dr + 2] - d.pos[3 * j + 2];
  Green g;
  green_eh(Rx, Ry, Rz, w, f == 1 || EFF, g);
  if (!EFF) {
    // -G^{f p} alpha_j : 3 x 3
    const double2 al = d.alpha_c[j];
    const double2 ma = make_double2(-al.x, -al.y);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int a = 0; a < 3; ++a) v[c][a] = cmul(f == 0 ? gep(g, a, c) : ghp(g, a, c), ma);
  } else {
    // -[G^{f p} G^{f m}] alpha6_j : 3 x 6
    const double2* al = d.alpha6 + (j - nc) * 36;
    double2 gr[3][6];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 6; ++b) gr[a][b] = f == 0 ? g6(g, w.eps_env, a, b) : g6(g, w.eps_env, 3 + a, b);
    if (unit_alpha) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int a = 0; a < 3; ++a) v[c][a] = make_double2(-gr[a][c].x, -gr[a][c].y);
      return;
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
#pragma unroll
      for (int b = 0; b < 6; ++b) {
        const double2 ab = al[b * 6 + c];
#pragma unroll
        for (int a = 0; a < 3; ++a) cfma(v[c][a], gr[a][b], ab);
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) v[c][a] = make_double2(-v[c][a].x, -v[c][a].y);
    }
  }
}

template <typename T>
hipError_t launch_assemble(const DipoleView& d, const struct Wave& w, void* M, int64_t ld, hipStream_t st);
// both precisions from one FP64 evaluation of every entry
hipError_t launch_assemble_dual(const DipoleView& d, const struct Wave& w, double2* M64, float2* M32, int64_t ld,
                                hipStream_t st);

// Optional operand masks: rows [ar0, ar0 + adw) of op(A) are a square block
// (row r - ar0, column k) of which only one triangle is read (kind below); a
// B mask keeps the triangle of B (row k, column j).  Masked-out elements read
// as zero.
enum { GEMM_MASK_NONE = 0, GEMM_MASK_STRICT_LOWER = 1, GEMM_MASK_UPPER = 2, GEMM_MASK_LOWER = 3,
       GEMM_MASK_STRICT_UPPER = 4 };
struct GemmMask {
  int akind = 0;
  int64_t ar0 = 0, adw = 0;
  int bkind = 0;
  // Optional second destination (launch_gemm only): rows [ar0, ar0 + adw) of
  // the result go to c2 (row r - ar0, leading dimension ldc2, item stride sc2)
  // instead of C; mode 0 still reads their old values from C.  With it a
  // product may read its B operand from those rows of C in place.
  void* c2 = nullptr;
  int64_t ldc2 = 0, sc2 = 0;
};

// C (m x n) = C - op(A) B   (mode 0)   or   C = op(A) B   (mode 1);
// complex interleaved, column-major; op(A) = A (transA 0) or A^T (transA 1, no conjugation).
// nbatch > 1: independent products, item z at A + z sA, B + z sB, C + z sC.
template <typename T>
hipError_t launch_gemm(int mode, int transA, int64_t m, int64_t n, int64_t k, const void* A, int64_t lda,
                       const void* B, int64_t ldb, void* C, int64_t ldc, hipStream_t st, GemmMask mk = GemmMask{},
                       int nbatch = 1, int64_t sA = 0, int64_t sB = 0, int64_t sC = 0);
// C = A B on the 3M kernel (64 x 64 tiles; no masks, no transpose); nbatch
// independent products, item z at A + z sA, B + z sB, C + z sC.
template <typename T>
hipError_t launch_gemm_product_3m(int64_t m, int64_t n, int64_t k, const void* A, int64_t lda, const void* B,
                                  int64_t ldb, void* C, int64_t ldc, hipStream_t st, int nbatch = 1, int64_t sA = 0,
                                  int64_t sB = 0, int64_t sC = 0);
// The LU trailing update A22 -= L21 U12: same kernel body, separate symbol so
// that profilers report it on its own.
template <typename T>
hipError_t launch_gemm_update(int64_t m, int64_t n, int64_t k, const void* A, int64_t lda, const void* B,
                              int64_t ldb, void* C, int64_t ldc, hipStream_t st, int nbatch = 1, int64_t sA = 0,
                              int64_t sB = 0, int64_t sC = 0);

// Small-RHS block steps of the triangular solves (solve_small.hip).  All take
// an optional batch of nbatch independent items (item z: A + z sA, X/B + z sX/sB,
// C + z sC; partial-sum buffers must hold nbatch times the per-item need).
// C[m x nrhs] -= A[m x k] X[k x nrhs], k <= 256, optional triangle mask on A.
template <typename T>
hipError_t launch_skinny_n(int64_t m, int64_t k, const void* A, int64_t lda, const void* X, int64_t ldx, void* C,
                           int64_t ldc, int64_t nrhs, hipStream_t st, GemmMask mk = GemmMask{}, int nbatch = 1,
                           int64_t sA = 0, int64_t sX = 0, int64_t sC = 0);
// C[mo x nrhs] -= A0^T B0 + mask(A1)^T B1 with A0 (k0 x mo) and A1 (k1 x mo)
// stored column-major; split over k into chunks whose partial sums go to
// `part` (capacity part_elems complex), then added to C in a fixed order.
template <typename T>
hipError_t launch_skinny_t(int64_t mo, int64_t nrhs, const void* A0, int64_t lda0, const void* B0, int64_t ldb0,
                           int64_t k0, const void* A1, int64_t lda1, const void* B1, int64_t ldb1, int64_t k1,
                           int kind1, void* part, int64_t part_elems, void* C, int64_t ldc, hipStream_t st,
                           int nbatch = 1, int64_t sA = 0, int64_t sB = 0, int64_t sC = 0);
int64_t skinny_t_chunks(int64_t k0, int64_t k1);
// C[m x nrhs] -= A[m x k] X[k x nrhs] for any k (split over k; partial sums in
// `part`, capacity part_elems >= nbatch skinny_n_long_parts(m, k, nrhs)).
template <typename T>
hipError_t launch_skinny_n_long(int64_t m, int64_t k, const void* A, int64_t lda, const void* X, int64_t ldx, void* C,
                                int64_t ldc, int64_t nrhs, void* part, int64_t part_elems, hipStream_t st,
                                int nbatch = 1, int64_t sA = 0, int64_t sX = 0, int64_t sC = 0);
int64_t skinny_n_long_parts(int64_t m, int64_t k, int64_t nrhs);
// C[mo x nrhs] -= sum over nchunk partial blocks part[(chunk nrhs + r) mo + i], in order
template <typename T>
hipError_t launch_partial_reduce(const void* part, int nchunk, int64_t mo, int64_t nrhs, void* C, int64_t ldc,
                                 hipStream_t st);
constexpr int SKINNY_MAX_RHS = 8;

// Optional per-launch timing with HIP events on the launch stream.
enum ProfTag {
  PROF_UPDATE = 0,
  PROF_PANEL = 1,
  PROF_ASSEMBLE = 2,
  PROF_TRSM = 3,
  PROF_PERM = 4,
  PROF_SOLVE = 5,
  PROF_RESID = 6,
  PROF_ADJ_PAIR = 7,
  PROF_ADJ_PROBE = 8,
  PROF_FIELDS = 9,
  PROF_LOOKAHEAD = 10,
  PROF_ITER_MATVEC = 11,
  PROF_PANEL_L21 = 12,
  PROF_NTAGS = 13
};
struct Prof {
  uint32_t mask = 0;  // bit t: record launches of tag t
  bool open = false;  // the last begin() recorded (its end() must too)
  std::vector<hipEvent_t> ev;
  std::vector<int> tag;
  std::vector<double> work;
  size_t used = 0;
  double ms[PROF_NTAGS] = {};
  double wsum[PROF_NTAGS] = {};
  double cnt[PROF_NTAGS] = {};
  hipError_t begin(hipStream_t st, int t, double w);
  hipError_t end(hipStream_t st);
  // after the stream is synchronised: fold the recorded pairs into ms/wsum/cnt
  void collect();
  void reset();
  ~Prof();
};

// ---------------------------------------------------------------------------
// blocked LU with partial pivoting
// ---------------------------------------------------------------------------
struct LUBlock {
  int64_t k0;  // first row/column of the block
  int w;       // block width
  int R;       // panel rows per workgroup
  int G;       // panel workgroups
};

struct LUPlan {
  int64_t n = 0;
  int nb = 0;
  int max_wg = 0;  // number of CUs: upper bound on panel workgroups
  int pb = 1;      // panel columns per pivot exchange (1: partial pivoting; 2, 4, 8: tournament)
  bool spec = false;  // speculative panels (diagonal pivots checked against partial pivoting; pb = 1 plan)
  std::vector<LUBlock> blocks;
};

// Device workspace of the factorisation; sized by lu_workspace_bytes().  With a
// batch of nbatch items every per-item field below holds nbatch copies, item z
// at field + z * s_field (elements of the field's type).
struct LUWork {
  unsigned long long* cand;  // [2][gitem][max(KEY_STRIDE, pb (1 + pb words per complex))] epoch-tagged
                             // pivot keys / candidate records
  unsigned long long* rows;  // [2][gitem][pb][wwmax] epoch-tagged candidate rows
  int gmax;                  // number of CUs (max panel workgroups of all items together)
  int gitem;                 // max panel workgroups of one item (the plan's max_wg)
  int pb;                    // panel columns per pivot exchange the buffers are sized for
  int wwmax;                 // payload words per row (nb * words per complex)
  int32_t* err;              // [2] (shared): exchange timeout flag, first zero pivot (INT32_MAX if none)
  int32_t* pairs;            // [nblocks][2][2 nb]: destination rows then source rows
  int32_t* npairs;           // [nblocks]
  int32_t* spec;             // [nblocks] speculative panel failed its check (after npairs, same item stride)
  void* tmp;                 // [tmp_elems] complex scratch (operand copies, split-k partials, solve sweeps)
  void* dinv;                // [nblocks][nb][nb] complex inverses of the diagonal triangles
  void* l21c;                // speculative panels: copy of the rows below the diagonal block (n x nb complex)
  std::vector<hipEvent_t>* events;  // host-side pool of reusable events (look-ahead)
  int64_t tmp_elems;         // capacity of tmp per item in complex elements
  int nbatch = 1;
  int64_t s_cand = 0, s_rows = 0, s_pairs = 0, s_npairs = 0, s_tmp = 0, s_dinv = 0, s_l21c = 0;
  size_t bytes = 0;          // total size (set by lu_workspace_carve)
};

// nbatch: number of same-size items factored together (their panels share one
// launch, so each panel gets at most num_cu / nbatch workgroups).
// pb: panel columns per pivot exchange (1: partial pivoting with LAPACK's
// pivots; 2, 4 or 8: tournament pivoting, reduced when the candidates of the
// widest panel would exceed 1024 or its rows would not fit the LDS; 0:
// speculative panels, a partial-pivoting plan with `spec` set).
LUPlan lu_plan(int64_t n, int elem_bytes, int num_cu, int lds_bytes, int nbatch = 1, int nb_max = 128, int pb = 1);
// one-time host-side kernel settings for a plan (call before graph capture)
template <typename T>
hipError_t lu_prepare(const LUPlan& plan);
bool lu_plan_fits(const LUPlan& p);
size_t lu_workspace_bytes(const LUPlan& p, int elem_bytes, int num_cu, int nbatch = 1);
void lu_workspace_carve(void* base, const LUPlan& p, int elem_bytes, int num_cu, LUWork& w, int nbatch = 1);

// `side` (may be null): second stream for the look-ahead; all work is joined
// back into `st` before return.  Batch (ws.nbatch items): matrix z at A + z sA,
// its pivots at ipiv + z sipiv.
template <typename T>
hipError_t lu_factor(void* A, int64_t ld, const LUPlan& plan, const LUWork& ws, int32_t* ipiv, hipStream_t st,
                     Prof* prof = nullptr, hipStream_t side = nullptr, int64_t sA = 0, int64_t sipiv = 0);

// Factors are left in a solve-ready form: for every block the diagonal block
// holds I - L11^-1 (strict lower part) and I - U11^-1 (upper part), the block
// column below holds L21 L11^-1 and the block column above holds U01 U11^-1, so
// that every step of a (transposed) solve is one GEMM.
// Solve op(M) X = B in place for B (n x nrhs, ld ldb) with the factors of
// lu_factor (batch: item z's factors at A + z sA, its B at B + z sB).
template <typename T>
hipError_t lu_solve(int trans, const void* A, int64_t ld, const LUPlan& plan, const LUWork& ws, void* B,
                    int64_t ldb, int64_t nrhs, hipStream_t st, int64_t sA = 0, int64_t sB = 0);

}  // namespace gdm
