/* libgdm: Green's Dyadic Method hot path on an MI355X (gfx950) GPU.
 *
 * The library solves the coupled electric/magnetic dipole scattering problem of
 * arXiv:2505.09545 (TorchGDM):
 *   (a) assembly of the dense coupling matrix M = I - G~ A of the discretised
 *       Lippmann-Schwinger equation (Sec. "Formalism and implementation", Eq.
 *       LPS_6by6_discrete and Eq. GDM_system_of_equations), with electric and
 *       magnetic unknowns separated and the magnetic unknowns of mesh cells
 *       removed (Sec. "Hybrid discretization GDM");
 *   (b) LU decomposition with partial pivoting and a multi-RHS solve (Sec.
 *       "Numerical solution"), in FP64 or in FP32 with FP64 iterative refinement;
 *   (c) matrix-free re-propagation of the dipole moments to probe points (Sec.
 *       "Observables") and the extinction / absorption / scattering cross
 *       sections.
 *
 * Conventions shared by every call
 *  - Units: nm for lengths and wavelengths, nm^2 for cross sections; Gaussian
 *    units, time factor exp(-i w t), Im(eps) > 0 is absorbing.
 *  - Complex numbers are interleaved (re, im) pairs of double.  Every array
 *    argument is a DEVICE pointer on the context's device (e.g. a torch tensor's
 *    data_ptr()), C order as written in the comments.  Work is enqueued on the
 *    context's HIP stream: buffers must stay alive until that stream reaches the
 *    call; calls that return a status derived from device results (factorize,
 *    solve, fields) synchronise the stream before returning.
 *  - Unknown layout (n = 3 (n_cell + n_eff) + 3 n_eff): the electric field of
 *    every dipole (cells first, then effective dipoles), then the magnetic field
 *    of every effective dipole.  Vectors "in the unknown layout" are [n_rhs][n].
 *  - Ownership: the caller owns every buffer it passes; the context owns copies
 *    of the structure, the factors and all workspaces.  Nothing allocated by the
 *    library is handed to the caller.
 *  - Errors: every call returns a gdm_status; arguments are validated before any
 *    work is enqueued (outputs untouched on GDM_E_ARG); gdm_last_error() gives
 *    a message.  A context is not thread-safe; several contexts may coexist.
 */
#ifndef GDM_H
#define GDM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gdm_ctx gdm_ctx;

typedef enum {
  GDM_OK = 0,
  GDM_E_ARG = 1,             /* invalid argument */
  GDM_E_OOM = 2,             /* device allocation failed */
  GDM_E_DEVICE = 3,          /* HIP runtime / kernel failure */
  GDM_E_SINGULAR = 4,        /* exactly zero pivot; gdm_info.bad_index = its column */
  GDM_E_NOCONV = 5,          /* refinement did not reach tol; best iterate written */
  GDM_E_PROBE_AT_DIPOLE = 6, /* a probe lies on a dipole (|R| < 1e-9 step) */
  GDM_E_STATE = 7            /* call order violated (e.g. solve before factorize) */
} gdm_status;

typedef enum { GDM_PREC_FP64 = 0, GDM_PREC_FP32_IR = 1 } gdm_precision;

/* Self-term of the cubic mesh cells.  STATIC is the paper's
 * S^Ep = -4 pi / (3 eps_env d^3) I (Eq. selfterm_SEp_cubic); RADIATIVE adds the
 * radiation-reaction term i (2/3) k^3 / eps_env (an option, not the paper's).
 * Effective dipoles have zero self-term (Sec. "Self-terms", last paragraph). */
typedef enum { GDM_SELF_STATIC = 0, GDM_SELF_RADIATIVE = 1 } gdm_selfterm;

typedef struct {
  int32_t ir_iters;    /* refinement corrections applied after the first solve */
  double backward_err; /* max over RHS of |r|_inf / (|M|_inf |x|_inf + |F0|_inf) */
  int64_t bad_index;   /* zero-pivot column for GDM_E_SINGULAR, else -1 */
  float ms_assemble, ms_factor, ms_solve, ms_ir; /* stage times of the last calls */
} gdm_info;

/* Create a context on HIP device `device`.  `hip_stream` (a hipStream_t, may be
 * NULL for a context-owned stream) is used for all work of the context. */
gdm_status gdm_create(int device, void* hip_stream, gdm_ctx** out);
void gdm_destroy(gdm_ctx* ctx);
/* Message of the last failing call (never NULL; owned by the context). */
const char* gdm_last_error(const gdm_ctx* ctx);

/* Limit on the device memory this context's buffers may hold (bytes; 0: no
 * limit, the default).  A call that would need more fails with GDM_E_OOM before
 * it allocates, as it would when the device itself is full; the batched
 * spectra size their groups within the limit.  GDM_E_ARG for bytes < 0. */
gdm_status gdm_set_memory_limit(gdm_ctx* ctx, int64_t bytes);
/* Device bytes the context's buffers hold now. */
int64_t gdm_memory_used(const gdm_ctx* ctx);

/* Pivoting of the next LU factorisations of this context (gdm_factorize,
 * gdm_getrf, gdm_batch_spectra); the paper factors by LU with partial
 * pivoting (Sec. "Numerical solution").  Every mode yields P M = L U.
 *   1: partial pivoting, the largest |re| + |im| in each column (compared in
 *      FP32), lowest row on ties -- LAPACK's pivot sequence up to such
 *      near-ties -- searched column by column across the device;
 *   2, 4 or 8: tournament pivoting, where the LU panel's workgroups each pick
 *      that many candidate rows for that many columns by partial pivoting on
 *      their own rows, and the pivots are chosen by partial pivoting among all
 *      candidates (one device-wide exchange per that many columns; FP64
 *      factorisations use at most 4); the row interchanges may differ;
 *   0 (the default): speculative partial pivoting in gdm_factorize -- the
 *      diagonal is taken as the pivot of every column without a search, and
 *      every entry that partial pivoting would compare it with is checked
 *      against it by the same rule; if any check fails (or a pivot is zero or
 *      not finite) the matrix is assembled again and factored with mode 1, so
 *      the pivots are partial pivoting's either way (near-ties aside);
 *      gdm_batch_spectra does the same per system (a system whose check
 *      fails is computed again on its own with mode 1, its outputs
 *      overwritten); gdm_getrf uses mode 1.
 * GDM_E_ARG for other values. */
gdm_status gdm_set_pivoting(gdm_ctx* ctx, int32_t columns_per_exchange);
/* Factorisations of this context (since gdm_create), single systems and
 * batched ones, whose speculative panels failed their check and were repeated
 * with the pivot search; -1 for NULL. */
int64_t gdm_pivot_fallbacks(const gdm_ctx* ctx);

/* Real refractive index of the lossless homogeneous host (Appendix, tg.env
 * EnvHomogeneous3D).  Must be > 0.  Invalidates the factors. */
gdm_status gdm_set_environment(gdm_ctx* ctx, double n_env);

/* Structure: n_cell cubic mesh cells of side step_nm at r_cell [n_cell][3] with
 * complex permittivity eps_cell [n_cell] (polarisability (eps - eps_env) d^3 /
 * (4 pi), Sec. "Volume discretization polarizabilities"), plus n_eff effective
 * electric+magnetic point dipoles at r_eff [n_eff][3] with 6x6 polarisability
 * tensors alpha_eff [n_eff][6][6] (row-major, mapping (E, H) to (p, m); Eq.
 * after LPS_6by6_discrete).  Either count may be 0 (not both).  The arrays are
 * copied; the caller may free them after the stream reaches the call.
 * Invalidates the factors. */
gdm_status gdm_set_structure(gdm_ctx* ctx, int64_t n_cell, const double* r_cell, double step_nm,
                             const double* eps_cell, int64_t n_eff, const double* r_eff,
                             const double* alpha_eff, gdm_selfterm selfterm);

/* Number of unknowns n of the current structure (0 if none). */
int64_t gdm_num_unknowns(const gdm_ctx* ctx);

/* Global polarisability matrices (Sec. "Extraction of effective models"; Fig.
 * reference_system (b)): group g joins the effective dipoles [first[g],
 * first[g] + size[g]) of the current structure (host arrays, 1 <= size <= 32,
 * no dipole in two groups) into one non-local model: their moments are
 * q_g = alpha_G F_g with alpha_G the g-th complex matrix of `alpha` (device,
 * the groups' (6 size)^2 matrices one after another, each row-major with rows
 * and columns ordered (member, then p_x, p_y, p_z, m_x, m_y, m_z)), and they do
 * not couple among themselves through G~ (alpha_G holds that).  The members'
 * own alpha_eff is ignored while the groups are set.  Absorption of a group
 * also removes the power its members radiate into each other's fields, so that
 * sca = ext - abs is the power radiated by all dipoles.  n_groups = 0 removes
 * the groups; gdm_set_structure removes them too.  `alpha` is copied.
 * Invalidates the factors.  With groups set, gdm_solve_iterative and
 * gdm_adjoint return GDM_E_ARG. */
gdm_status gdm_set_gpm(gdm_ctx* ctx, int64_t n_groups, const int64_t* first, const int64_t* size,
                       const double* alpha);

/* Step (a) alone: write M = I - G~ A at `wavelength_nm` into the caller's
 * column-major buffer M_out (n x n, leading dimension ld >= n), as complex
 * double (dtype 0) or complex float (dtype 1; FP64 arithmetic, rounded once). */
gdm_status gdm_assemble(gdm_ctx* ctx, double wavelength_nm, int dtype, void* M_out, int64_t ld);

/* Steps (a) + (b1): assemble M at `wavelength_nm` and LU-factorise it in the
 * context, in FP64 (prec 0) or FP32 (prec 1, keeping an FP64 copy of M for the
 * refinement residual).  Sets the context wavelength.  GDM_E_SINGULAR on an
 * exactly zero pivot (info->bad_index, info may be NULL). */
gdm_status gdm_factorize(gdm_ctx* ctx, double wavelength_nm, gdm_precision prec, gdm_info* info);

/* Set the context wavelength without factorising (for gdm_incident_planewave,
 * gdm_fields and gdm_cross_sections ahead of gdm_solve_iterative); factors of
 * another wavelength are dropped.  GDM_E_STATE without a structure. */
gdm_status gdm_set_wavelength(gdm_ctx* ctx, double wavelength_nm);

/* Step (b) without the matrix: solve M F = F0 at `wavelength_nm` by restarted
 * GMRES (restart >= 1; <= 0 selects 30) whose products with M re-evaluate the
 * dipole couplings from the dyad every time (nothing of size n^2 is stored:
 * the discrete dipole approximation's iterative route, Sec. "Discrete Dipole
 * Approximation - iterative solver", for systems past the dense solver's
 * memory, Sec. "Benchmarks"), right-preconditioned by the inverses of the
 * diagonal blocks of M over groups of 8 consecutive dipoles.  FP64 throughout.
 * f0 [n_rhs][n] as in gdm_solve; writes q = A F [n_rhs][n] and, if f_out is not
 * NULL, F.  Stops when ||F0 - M F||_2 / ||F0||_2 <= tol for every RHS (tol <= 0
 * selects 1e-13; the residual is recomputed at each restart) or after max_iter
 * products (max_iter <= 0 selects 1000): GDM_E_NOCONV, the last iterate
 * written.  info->ir_iters = products with M, info->backward_err = the largest
 * relative residual.  Sets the context wavelength (for gdm_fields and
 * gdm_cross_sections); factors of another wavelength are dropped. */
gdm_status gdm_solve_iterative(gdm_ctx* ctx, double wavelength_nm, int64_t n_rhs, const double* f0, double tol,
                               int32_t max_iter, int32_t restart, double* q_out, double* f_out, gdm_info* info);

/* Incident plane waves at the dipoles in the unknown layout: f0 [n_pw][n] with
 * E0 = e0 exp(i k khat.r), H0 = n_env khat x E0 (Appendix, 3D illuminations);
 * khat [n_pw][3] unit vectors, e0 [n_pw][3] complex.  Uses the context
 * wavelength. */
gdm_status gdm_incident_planewave(gdm_ctx* ctx, int64_t n_pw, const double* khat, const double* e0, double* f0);

/* Step (b2): solve M F = F0 for n_rhs right-hand sides f0 [n_rhs][n]; writes the
 * dipole moments q = A F [n_rhs][n] and, if f_out is not NULL, the field F.
 * FP64 factors: one solve.  FP32 factors: FP64 iterative refinement
 * (residual and update in FP64) until the normwise backward error of every RHS
 * is <= tol (tol <= 0 selects 1e-14) or max_iter corrections (max_iter < 0
 * selects 10); GDM_E_NOCONV if not reached (best iterate written). */
gdm_status gdm_solve(gdm_ctx* ctx, int64_t n_rhs, const double* f0, double tol, int32_t max_iter,
                     double* q_out, double* f_out, gdm_info* info);

/* Plane waves at arbitrary points: E, H [n_pw][n_pts][3] (H may be NULL). */
gdm_status gdm_planewave(gdm_ctx* ctx, int64_t n_pw, const double* khat, const double* e0, int64_t n_pts,
                         const double* r, double* E, double* H);

/* Step (c): scattered fields of the moments q [n_rhs][n] at n_probe points
 * r_probe [n_probe][3]: E_sca, H_sca [n_rhs][n_probe][3] (H_sca may be NULL),
 * FP64, matrix-free.  GDM_E_PROBE_AT_DIPOLE if a probe is within 1e-9 step of
 * a dipole (its contribution is then skipped).  Uses the context wavelength. */
gdm_status gdm_fields(gdm_ctx* ctx, int64_t n_rhs, const double* q, int64_t n_probe, const double* r_probe,
                      double* E_sca, double* H_sca);

/* Step (c), total field: E = E_inc + E_sca and H = H_inc + H_sca at the probes
 * for moments q [n_rhs][n] of plane-wave illuminations khat [n_rhs][3], e0
 * [n_rhs][3] complex (as in gdm_planewave); otherwise as gdm_fields. */
gdm_status gdm_fields_total(gdm_ctx* ctx, int64_t n_rhs, const double* q, const double* khat, const double* e0,
                            int64_t n_probe, const double* r_probe, double* E, double* H);

/* Intensity |E0|^2 = sum_a |e0[r][a]|^2 of plane-wave amplitudes e0 [n_pw][3]
 * complex, into out [n_pw] (device; the normalisation of gdm_cross_sections). */
gdm_status gdm_planewave_intensity(gdm_ctx* ctx, int64_t n_pw, const double* e0, double* out);

/* Step (c) for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation, arguments, layouts and errors as gdm_fields, and the same result
 * bit for bit, but the partial sums of its dipole splits and its probe-on-dipole
 * flag live in a static device array of GDM_NOALLOC_SCRATCH_BYTES instead of
 * context buffers; the call allocates nothing (no hipMalloc, no hipFree, no
 * allocating library routine).  Each device holds its own copy of the array
 * from the first gdm_create on it until the process ends.  The launch needs
 * 48 * nsplit * n_rhs * n_probe bytes (twice that with H_sca), where nsplit <= 64
 * is the number of dipole splits (1 from about 262 000 probes on, and at most
 * ceil(N / 32)); GDM_E_ARG, with nothing written, if that exceeds
 * GDM_NOALLOC_SCRATCH_BYTES - 256.  Every call on a device shares that device's
 * array and leaves its contents behind: calls that overlap on one device (from
 * several contexts or streams) race.  GDM_E_DEVICE if the array's address could
 * not be obtained at gdm_create. */
#define GDM_NOALLOC_SCRATCH_BYTES (32u << 20)
gdm_status gdm_fields_noalloc(gdm_ctx* ctx, int64_t n_rhs, const double* q, int64_t n_probe, const double* r_probe,
                              double* E_sca, double* H_sca);

/* Cross sections per RHS (Sec. "Observables"), FP64: out [n_rhs][5] =
 * (extinction, scattering = ext - abs, absorption, radiated-by-dipoles,
 * far-field scattering by the exact double sum or NaN unless want_ff).
 * f0, q, f: [n_rhs][n] incident field, moments and solved field at the dipoles;
 * e0_norm2: |E0|^2 per RHS [n_rhs] (device). */
gdm_status gdm_cross_sections(gdm_ctx* ctx, int64_t n_rhs, const double* f0, const double* q, const double* f,
                              const double* e0_norm2, int32_t want_ff, double* out);

/* Exact multipole decomposition of the mesh cells' polarisation up to
 * quadrupole order, and the scattering and extinction cross sections of each
 * multipole (Sec. "Observables"; Sec. "Implementation technical details").
 * Moments about r0 (host double[3], or NULL for the mean position of the mesh
 * cells) of the cells' electric dipoles in q [n_rhs][n] (gdm_solve's q_out;
 * effective dipoles are not part of the discretised structure and are left
 * out), with R = r_j - r0, x = k|R| and spherical Bessel functions j_n:
 *   p  = sum p_j j0 + (k^2/2) [3 (R.p_j) R - R^2 p_j] j2/x^2
 *   m  = -i k0 (3/2) sum (R x p_j) j1/x
 *   Qe = 3 sum [3 (R p_j^T + p_j R^T) - 2 (R.p_j) I] j1/x
 *          + 2 k^2 [5 (R.p_j) R R^T - R^2 (R p_j^T + p_j R^T) - R^2 (R.p_j) I] j3/x^3
 *   Qm = -i k0 15 sum [R (R x p_j)^T + (R x p_j) R^T] j2/x^2
 * (Gaussian units, the far-field convention of gdm_fields; at x -> 0 the
 * long-wavelength moments).  moments (device, may be NULL): complex [n_rhs][24]
 * = p (3), m (3), Qe (3x3 row-major), Qm (3x3).  sigma (device, may be NULL):
 * double [n_rhs][8] = scattering of ED, MD, EQ, MQ, then their extinction:
 *   (8 pi/3) k^4/eps^2 |p|^2, (8 pi/3) k0^2 k^2 |m|^2, (pi/45) k^6/eps^2 |Qe|^2,
 *   (pi/45) k0^2 k^4 |Qm|^2 over |E0|^2;  C Im(E0*(r0).p), C Im(H0*(r0).m),
 *   (C/6) Im(sum d_a E0*_b(r0) Qe_ab), (C/6) Im(sum d_a H0*_b(r0) Qm_ab),
 *   C = 4 pi k0 / (n_env |E0|^2),
 * for the plane waves khat [n_rhs][3], e0 [n_rhs][3] complex (device, as in
 * gdm_incident_planewave); with khat = e0 = NULL the scattering terms are for
 * |E0| = 1 and the extinction slots hold NaN.  The extinction terms add up to
 * the total extinction up to the octupole and higher orders (which can make
 * single terms negative for non-spherical shapes).  FP64.  Uses the context
 * wavelength.  GDM_E_ARG without mesh cells. */
gdm_status gdm_multipoles(gdm_ctx* ctx, int64_t n_rhs, const double* q, const double* r0, const double* khat,
                          const double* e0, double* moments, double* sigma);

/* Effective model of the structure as one electric-magnetic dipole pair at r0
 * (Sec. "Extraction of effective models"; the paper's single-pair 3D case):
 * the n_pw plane waves (khat [n_pw][3], e0 [n_pw][3] complex, device) and
 * n_src point-dipole sources (r_src [n_src][3], d_src [n_src][6] complex (p, m),
 * device, as in gdm_dipole_sources) are solved with the context's factors (tol,
 * max_iter as in gdm_solve); the electric and magnetic dipole moments of each
 * response about r0 (host double[3], or NULL for the cells' mean position) are
 * the exact ones of gdm_multipoles (rows of P [N][6]); the rows of F0 [N][6]
 * are each illumination's (E0, H0) at r0 (a source's own field there).
 * alpha (device, complex [6][6] row-major) minimises ||F0 alpha^T - P||_F, so
 * that (p, m) ~ alpha (E0, H0) -- an effective dipole's alpha_eff for
 * gdm_set_structure; *resid (host, may be NULL) = ||F0 alpha^T - P||_F / ||P||_F
 * (large values: the structure is too large for one dipole pair).  Needs 6 <=
 * n_pw + n_src <= 4096 and mesh cells; GDM_E_ARG if the illuminations leave
 * alpha undetermined; GDM_E_STATE without factors; GDM_E_PROBE_AT_DIPOLE for a
 * source on a dipole. */
gdm_status gdm_extract_dipole_pair(gdm_ctx* ctx, int64_t n_pw, const double* khat, const double* e0, int64_t n_src,
                                   const double* r_src, const double* d_src, const double* r0, double tol,
                                   int32_t max_iter, double* alpha, double* resid, gdm_info* info);

/* GPM of the structure for n_pairs (1..32) dipole pairs at r_gpm [n_pairs][3]
 * (device) by scattered-field matching (Sec. "Extraction of effective
 * models"): the illuminations (as in gdm_extract_dipole_pair) are solved with
 * the context's factors; the scattered (E, H) of each response at the probes
 * r_probe [n_probe][3] (device, n_pairs <= n_probe <= 2^20, off the dipoles and
 * the pairs) is fitted in least squares by sum_j G6(r_p - r_j) (p_j, m_j);
 * with F0 [N][6 n_pairs] the illuminations' (E0, H0) at the pairs and P
 * [N][6 n_pairs] the fitted moments, alpha (device, complex (6 n_pairs)^2
 * row-major, ordered as in gdm_set_gpm) minimises ||F0 alpha^T - P||_F.
 * resid (host double[2], may be NULL) = relative residuals of the field fit
 * and of the alpha fit.  Needs 6 n_pairs <= n_pw + n_src <= 4096.  GDM_E_ARG
 * if the fit is rank-deficient (pairs or probes that do not determine the
 * model); GDM_E_STATE without factors; GDM_E_PROBE_AT_DIPOLE for a source or
 * probe on a dipole. */
gdm_status gdm_extract_gpm(gdm_ctx* ctx, int64_t n_pw, const double* khat, const double* e0, int64_t n_src,
                           const double* r_src, const double* d_src, int64_t n_pairs, const double* r_gpm,
                           int64_t n_probe, const double* r_probe, double tol, int32_t max_iter, double* alpha,
                           double* resid, gdm_info* info);

/* Point dipole sources as the illumination (Appendix, illumination classes:
 * electric and magnetic dipole point sources): the incident field of sources
 * d_src [n_src][6] complex (p then m) at r_src [n_src][3] on every dipole, in
 * the unknown layout: f0 [n_src][n], F0_i = G(r_i, r_s) d_s with the dyad of Eq.
 * superprop_G.  Uses the context wavelength.  GDM_E_PROBE_AT_DIPOLE if a
 * source lies within 1e-9 step of a dipole. */
gdm_status gdm_dipole_sources(gdm_ctx* ctx, int64_t n_src, const double* r_src, const double* d_src, double* f0);

/* Partial LDOS of the structured environment (Sec. "Observables": electric and
 * magnetic LDOS in a nano-structured environment) at r_src [n_src][3]
 * (n_src <= 10922), relative to the homogeneous host: out [n_src][2][3] =
 * (electric, magnetic) x (x, y, z),
 *   rho_e,a / rho_0 = 1 + (3/2) (eps_env / k^3) Im G_sca^Ep_aa(r_s, r_s),
 *   rho_m,a / rho_0 = 1 + (3/2) (1 / k^3)       Im G_sca^Hm_aa(r_s, r_s),
 * the power a unit dipole emits there over its power in the host.  Solves the
 * six unit sources of every point with the current factors (FP32 factors: FP64
 * refinement to tol / max_iter as in gdm_solve; GDM_E_NOCONV if not reached,
 * results written).  GDM_E_STATE without factors; GDM_E_PROBE_AT_DIPOLE for a
 * point on a dipole.  info: refinement corrections and backward error. */
gdm_status gdm_ldos(gdm_ctx* ctx, int64_t n_src, const double* r_src, double tol, int32_t max_iter, double* out,
                    gdm_info* info);

/* Scattered part of the structured environment's 6x6 Green's tensor (Sec.
 * "The tg.Simulation class", Green's tensor of the environment defined by the
 * structures): G [n_src][n_pts][6][6] complex, G[s][p][row][c] = field row
 * (E_x, E_y, E_z, H_x, H_y, H_z) at r_pts[p] scattered by the structure under
 * the unit source component c (p_x, p_y, p_z, m_x, m_y, m_z) at r_src[s]; the
 * full tensor is the host's G(r_p, r_s) plus this part.  Solves as gdm_ldos;
 * n_src <= 10922; GDM_E_PROBE_AT_DIPOLE for a source or point on a dipole. */
gdm_status gdm_green_tensor(gdm_ctx* ctx, int64_t n_src, const double* r_src, int64_t n_pts, const double* r_pts,
                            double tol, int32_t max_iter, double* G, gdm_info* info);

/* Reverse mode (the paper differentiates the solver with automatic
 * differentiation, Sec. "Example: Autograd for resonance search"; here the
 * adjoint is written out).  For a real loss L that depends on the cross sections
 * of the last solve and on the TOTAL electric field at probe points, given
 *   g_sigma [n_rhs][3] : dL/d(extinction, scattering, absorption) per RHS (real;
 *                        the cross sections of gdm_cross_sections, columns 0-2),
 *                        may be NULL (no cross-section term);
 *   g_e [n_rhs][n_probe][3] complex : Wirtinger partial dL/dE of the total field
 *                        E = E_inc + E_sca at r_probe [n_probe][3] (so that
 *                        dL = 2 Re sum g_e dE), may be NULL (no field term),
 * writes dL/d(every dipole position) grad_r [N][3] (cells then effective
 * dipoles), dL/d(Re eps, Im eps) of every cell grad_eps [n_cell][2], and
 * dL/d(wavelength) grad_wl [1] (through k0 in the dyad, the plane waves, the
 * radiative self-term if selected and the cross-section prefactors; the cell
 * permittivities and the effective polarisabilities are held fixed).  All
 * arrays are device pointers.  The illumination must be the plane waves khat
 * [n_rhs][3], e0 [n_rhs][3] complex, and f0, q, f [n_rhs][n] the incident field,
 * moments and solved field of the last gdm_solve with the current factors,
 * which are reused for the transposed solve M^T lam = g_F + A^T g_q (FP32
 * factors: FP64 refinement of the transposed system to tol / max_iter as in
 * gdm_solve).  GDM_E_STATE without factors; GDM_E_PROBE_AT_DIPOLE as in
 * gdm_fields; GDM_E_NOCONV if the refinement stalls (gradients still written). */
gdm_status gdm_adjoint(gdm_ctx* ctx, int64_t n_rhs, const double* khat, const double* e0, const double* f0,
                       const double* q, const double* f, const double* g_sigma, int64_t n_probe,
                       const double* r_probe, const double* g_e, double tol, int32_t max_iter, double* grad_r,
                       double* grad_eps, double* grad_wl, gdm_info* info);

/* Batched spectra (the paper's spectra over wavelengths and structures, Sec.
 * "Implementation technical details"): for every structure s and wavelength l
 * solve the system of the structure's cubic cells with one permittivity
 * eps[s][l] for all its cells, and write the extinction, scattering and
 * absorption cross sections of n_pw plane waves.  The systems of one structure
 * are solved in groups that share every launch (assembly, LU, solve,
 * refinement, cross sections); each group shape is captured once into a HIP
 * graph and replayed; the group size and LU panel width are measured on the
 * first groups of each size class (kept in the context for later calls).
 *   cell_offset [n_struct + 1] HOST: structure s owns cells cell_offset[s] ..
 *       cell_offset[s+1] - 1 of r_cell [total][3] (device, nm); step_nm
 *       [n_struct] HOST; wavelengths [n_wl] HOST (nm);
 *   eps [n_struct][n_wl] complex (device); khat [n_pw][3], e0 [n_pw][3] complex
 *       (device) as in gdm_incident_planewave; the environment index is the
 *       context's (gdm_set_environment), `selfterm` as in gdm_set_structure;
 *   prec GDM_PREC_FP32_IR: FP32 LU and exactly ir_iters FP64 refinement
 *       corrections (ir_iters < 0 selects 2), be_out [n_struct][n_wl] (device,
 *       may be NULL) receives each system's normwise backward error after them;
 *       with tol > 0, GDM_E_NOCONV if any of them exceeds tol (every output is
 *       still written; tol = 0: no check); GDM_PREC_FP64: FP64 LU, be_out not
 *       written, tol ignored;
 *   cs_out [n_struct][n_wl][n_pw][3] (device) = (ext, sca = ext - abs, abs) nm^2.
 * info->backward_err = max of be_out, info->ms_factor = GPU time of the whole
 * batch.  GDM_E_OOM if a structure does not fit; GDM_E_SINGULAR on an exactly
 * zero pivot.  Cells only (no effective dipoles); at most 65535 plane waves. */
gdm_status gdm_batch_spectra(gdm_ctx* ctx, int64_t n_struct, const int64_t* cell_offset, const double* r_cell,
                             const double* step_nm, int64_t n_wl, const double* wavelengths, const double* eps,
                             int64_t n_pw, const double* khat, const double* e0, gdm_precision prec, int32_t ir_iters,
                             double tol, gdm_selfterm selfterm, double* cs_out, double* be_out, gdm_info* info);

/* The batch configurations measured so far by gdm_batch_spectra on this context:
 * returns their number; if out is not NULL, writes up to max_entries triples
 * (smallest n of the size class, systems per group, LU panel width) to the HOST
 * array out [max_entries][3]. */
int32_t gdm_batch_tuning(const gdm_ctx* ctx, int32_t* out, int32_t max_entries);

/* Dense LU of a caller matrix (dtype 0: complex double, 1: complex float),
 * column-major n x n, leading dimension lda, factored in place; ipiv [n]
 * receives 0-based pivot rows.  The factors are in the library's factored form
 * (row interchanges applied right of each block only) and are meant for
 * gdm_getrs with the same context, which keeps the block permutations. */
gdm_status gdm_getrf(gdm_ctx* ctx, int dtype, int64_t n, void* A, int64_t lda, int32_t* ipiv, gdm_info* info);
/* Solve op(A) X = B in place with the factors of the last gdm_getrf on this
 * context (trans 0: A, 1: A^T without conjugation); B n x nrhs, ldb >= n. */
gdm_status gdm_getrs(gdm_ctx* ctx, int dtype, int trans, int64_t n, int64_t nrhs, const void* A, int64_t lda,
                     void* B, int64_t ldb);

/* Complex GEMM used by the trailing update: C = C - op(A) B (mode 0) or
 * C = op(A) B (mode 1); dtype 0/1 as above; column-major. */
gdm_status gdm_gemm(gdm_ctx* ctx, int dtype, int mode, int transA, int64_t m, int64_t n, int64_t k,
                    const void* A, int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc);

/* Synchronise the context stream. */
gdm_status gdm_sync(gdm_ctx* ctx);

/* Per-kernel timing with HIP events recorded on the context stream around each
 * launch (for benchmarks; adds a few microseconds per launch).  enable != 0
 * clears the counters and starts recording; 0 stops. */
gdm_status gdm_profile(gdm_ctx* ctx, int enable);
/* The same for a subset of the tags listed under gdm_profile_read: launches of
 * tag t are timed iff bit t of mask is set (mask 0 stops; 8191 = all).  Timing
 * only the kernels one needs keeps the events off the critical path of the
 * rest.  GDM_E_ARG for a mask outside [0, 8192). */
gdm_status gdm_profile_mask(gdm_ctx* ctx, int32_t mask);
/* Counters accumulated since gdm_profile / gdm_profile_mask, written to the HOST array
 * out (n_out >= 39): out[3 t + 0..2] = (milliseconds, work, launches) for
 * t = 0 LU trailing-update GEMM, bulk part (the columns after the next panel's;
 * work = real flops 8 m n k), 1 LU panel: the pivot search, or the diagonal
 * block's kernel of a speculative panel (work = columns), 2 assembly (work = bytes written), 3 block triangular solve of the
 * factorisation (work = real flops), 4 row permutation of the trailing columns,
 * 5 forward + backward substitution of gdm_solve / gdm_adjoint (work =
 * 8 n^2 n_rhs), 6 FP64 refinement residual (work = 8 n^2 n_rhs), 7 adjoint
 * dipole-pair kernel (work = ordered pairs x n_rhs), 8 adjoint probe kernel
 * (work = probe-dipole pairs x n_rhs), 9 probe fields (work = probe-dipole
 * pairs x n_rhs), 10 LU trailing-update GEMM of the next panel's columns (the
 * look-ahead product; work = real flops), 11 matrix-free product of
 * gdm_solve_iterative (work = dipole pairs x n_rhs), 12 the rest of a
 * speculative panel: L21 = A21 U11^-1 (the triangle's inverse and the
 * product) and the pivot check (work = real flops 8 (n - k) w^2 of the
 * product). */
gdm_status gdm_profile_read(gdm_ctx* ctx, double* out, int32_t n_out);

#ifdef __cplusplus
}
#endif
#endif /* GDM_H */
