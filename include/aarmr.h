/*
 * aarmr.h -- C ABI of the MI355X (gfx950) library for the analysis step of
 * adaptive auxiliary reduced-model reanalysis (AARMR) topology optimisation
 * (Yin, Wang, Li, Guo, arXiv 2205.00385).
 *
 * The analysis step solves the SIMP equilibrium K(rho~) u = f on a 3D grid
 * of unit hexahedral (hex8) voxels (eqs. 1, 3, 7), by multigrid-preconditioned
 * CG (Algorithm 2) or by the combined-approximation reduced model built on a
 * projection auxiliary model (eqs. 15-29, Algorithm 1), and returns the
 * compliance and its sensitivity (eqs. 3, 6, 33, 34).  Every computation runs
 * in HIP kernels on the GPU; the host only orchestrates.
 *
 * Conventions shared by every entry point:
 *   - Grid: nx * ny * nz elements, (nx+1)(ny+1)(nz+1) nodes.  Element
 *     (i,j,k) has index e = i + nx*(j + ny*k); node (i,j,k) has index
 *     n = i + (nx+1)*(j + (ny+1)*k) (x fastest).
 *   - DOF vectors are structure-of-arrays: v[c * n_node + n], c in {0:x,1:y,2:z};
 *     a DOF id is c * n_node + n.  Several load cases are stored back to back
 *     (case l starts at l * 3 * n_node).
 *   - Plane stress (the paper's 2D examples, Sections 4.1, 4.2.1, 4.3):
 *     nz = 0 selects a grid of nx * ny unit squares (bilinear Q4 elements,
 *     unit thickness), (nx+1)(ny+1) nodes, element e = i + nx*j, node
 *     n = i + (nx+1)*j, two DOFs per node: every "[3][n_node]" below reads
 *     "[2][n_node]" and every 3 * n_node reads 2 * n_node.
 *   - All array arguments marked "device" are pointers to GPU memory of the
 *     device current for the calling thread; "host" pointers are CPU memory.
 *     The caller owns every buffer it passes; the library keeps no pointer to
 *     caller memory after a call returns, except the workspace bound with
 *     aarmr_bind_workspace, which must stay valid until aarmr_mesh_destroy.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Calls returning
 *     host results synchronise that stream before returning; the others are
 *     stream-ordered and asynchronous.
 *   - Every call returns AARMR_OK (0) or an error code; aarmr_last_error()
 *     then gives a thread-local message.  A mesh may be used by one thread
 *     at a time; distinct meshes are independent.  Calls that overlap on one
 *     mesh (two streams) race on its workspace.
 *   - Operator with boundary conditions: with Df the 0/1 diagonal of free
 *     DOFs, every solve works with A = Df K Df + (I - Df), i.e. K on free DOFs
 *     and identity rows on fixed DOFs; loads on fixed DOFs are ignored and the
 *     solution is zero there.
 */
#ifndef AARMR_H
#define AARMR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define AARMR_OK               0
#define AARMR_E_INVALID        1  /* bad argument: null pointer, size, range */
#define AARMR_E_HIP            2  /* a HIP runtime call or kernel launch failed */
#define AARMR_E_NOT_CONVERGED  3  /* CG hit cg_maxit; outputs are written anyway
                                     (aarmr_last_error names the smoother's omega
                                     condition, a common cause of a stall) */
#define AARMR_E_SINGULAR       4  /* non-positive pivot or p^T A p <= 0 */
#define AARMR_E_NO_WORKSPACE   5  /* no (or too small a) workspace bound */
#define AARMR_E_STATE          6  /* CA called before its PARM is complete */

#define AARMR_MAX_RHS     8
#define AARMR_MAX_LEVELS  8
#define AARMR_MAX_BASIS   10
#define AARMR_MAX_SPRINGS 8

/* ---- precision of the inner solve ------------------------------------ */
#define AARMR_FP64         0  /* everything in FP64 */
#define AARMR_FP32_REFINE  1  /* FP32 operator sweeps, V-cycle and inner CG
                                 vectors inside FP64 iterative refinement (FP64
                                 residuals, dot accumulation, updates of u,
                                 reduced systems and coarsest inverse).  Where
                                 FP32 stops making progress (extreme modulus
                                 contrast) the solve continues with FP64 CG
                                 preconditioned by the FP32 V-cycle.  Results
                                 meet cg_rtol in FP64 either way. */

/* ---- orthogonalisation of the CARM basis (Section 2.2) ---------------- */
#define AARMR_ORTH_GS   0  /* two-pass classical Gram-Schmidt with rank drop (named
                              beside eq. 21 as equally valid) */
#define AARMR_ORTH_SVD  1  /* PCA by the SVD of eq. (21), R = R~ Sigma V^T, on the
                              column-normalised basis: R~ = left singular vectors
                              with sigma > gs_tau sigma_1, computed as R = Q T
                              (Gram-Schmidt without drop) and T = U Sigma V^T
                              (one-sided Jacobi on the device), R~ = Q U */

/* ---- flags for aarmr_solve / aarmr_ca_update -------------------------- */
#define AARMR_FILTER_INPUT  1  /* `rho` is the design density: it is filtered
                                  first (eq. 31) and dc is returned w.r.t. the
                                  design density through eq. (33).  Otherwise
                                  `rho` is the physical density rho~ and dc is
                                  dC/drho~. */
#define AARMR_RECORD_PARM   2  /* after solving, push u/||u|| of each load case
                                  into that case's PARM (eqs. 27-28), dropping
                                  the oldest vector once Ns are held */
#define AARMR_WARM_START    4  /* use the incoming u as the CG initial guess
                                  (otherwise CG starts from zero); a guess
                                  whose residual exceeds ||f|| is replaced by
                                  zero */
#define AARMR_INPUT_MASKED  8  /* aarmr_apply_operator: the caller guarantees
                                  that v is zero on fixed DOFs, so the product
                                  skips masking its input (the form every
                                  solver-internal product uses) */
#define AARMR_MUTUAL_SENS  16  /* the non-self-adjoint objective of Section
                                  4.3: with n_rhs = 2, dc is the sensitivity
                                  of f_1^T u_0 (load case 1 is the unit dummy
                                  load on the output DOF, so this is the
                                  output displacement under load case 0):
                                  -dE_e/drho~_e u1_e^T KE u0_e, load case 1's
                                  solution serving as the adjoint.  In
                                  aarmr_ca_update both come from the reduced
                                  model when accepted: the approximate
                                  sensitivity of eq. (34)'s form.  Plane-stress
                                  grid only. */
#define AARMR_REUSE_COARSEST 32  /* Algorithm 2's coarsest solve may keep the
                                  dense inverse of an earlier design's
                                  coarsest operator (same fixed DOFs) instead
                                  of inverting the current one: it stays
                                  symmetric positive definite, so CG still
                                  converges to this design's solution, in a
                                  few more iterations.  The inverse is
                                  rebuilt when a solve with it needed
                                  max(3, n0/8) or more iterations beyond the
                                  n0 of the first solve after the inversion;
                                  a solve that has not converged after
                                  2 n0 + 20 iterations inverts the current
                                  operator and continues from its iterate.
                                  aarmr_setup always inverts. */

/* ---- parameters -------------------------------------------------------- */
typedef struct aarmr_params {
  int32_t nx, ny, nz;        /* elements per axis; each divisible by
                                2^(mg_levels-1); nz = 0: plane stress */
  double E0, Emin, nu, penal;/* SIMP, eq. (1): E = Emin + (E0-Emin) rho~^p */
  double rmin;               /* filter radius in element lengths, eq. (32);
                                <= 0 disables aarmr_filter */
  int32_t mg_levels;         /* grid levels including the finest (>= 2) */
  int32_t nu_pre, nu_post;   /* damped-Jacobi sweeps (Algorithm 2) */
  double omega;              /* Jacobi damping */
  double cg_rtol;            /* stop when ||f - A u|| <= cg_rtol ||f|| */
  int32_t cg_maxit;
  int32_t precision;         /* AARMR_FP64 or AARMR_FP32_REFINE */
  int32_t Ns;                /* PARM size s (eq. 27), <= AARMR_MAX_BASIS */
  int32_t Nm;                /* CARM size m (eq. 20), <= AARMR_MAX_BASIS */
  double ca_tol;             /* eps_tol of eq. (29): accept iff eps < ca_tol */
  double gs_tau;             /* Gram-Schmidt drops a column whose remaining
                                norm is below gs_tau times its initial norm;
                                with AARMR_ORTH_SVD, singular values below
                                gs_tau times the largest are dropped */
  int32_t n_rhs_max;         /* load cases per call, <= AARMR_MAX_RHS */
  int32_t orth;              /* CARM orthogonalisation: AARMR_ORTH_GS or
                                AARMR_ORTH_SVD */
  double oc_eta;             /* OC damping exponent in (0, 1]: 0.5 for
                                compliance, 0.3 for the mechanism of Section
                                4.3 */
} aarmr_params;

/* Statistics of one aarmr_solve call (host struct written by the call). */
typedef struct aarmr_stats {
  int32_t iterations[AARMR_MAX_RHS];   /* CG iterations per load case */
  double rel_residual[AARMR_MAX_RHS];  /* final ||f - A u|| / ||f|| */
  int64_t fine_sweeps;                 /* fine-grid operator applications */
  double setup_ms, solve_ms;           /* host wall time of the phases */
  int32_t coarsest_inversions;         /* dense inversions of the coarsest
                                          operator this call made (0 when an
                                          earlier inverse was kept) */
} aarmr_stats;

/* Statistics of one aarmr_ca_update call. */
typedef struct aarmr_ca_stats {
  double eps[AARMR_MAX_RHS];           /* eq. (29) of the reduced solution */
  int32_t accepted[AARMR_MAX_RHS];     /* 1 if eps < ca_tol */
  int32_t rank[AARMR_MAX_RHS];         /* columns kept by Gram-Schmidt */
  int32_t mgcg_iterations[AARMR_MAX_RHS]; /* fallback CG iterations (0 if accepted) */
  double rel_residual[AARMR_MAX_RHS];  /* final residual of the returned u */
  int64_t fine_sweeps;
  int32_t coarsest_inversions;         /* as in aarmr_stats */
} aarmr_ca_stats;

typedef struct aarmr_mesh aarmr_mesh;

/* Fill *p with the paper's defaults (E0=1, Emin=1e-9, nu=0.3, p=3, Section
 * 4; rmin 2.5, Section 3.2; Ns=Nm=2, Section 4.1.1; 3 grid levels, Section
 * 4.1.2) and solver defaults (omega 0.6, one pre- and post-sweep, rtol 1e-8,
 * 2000 iterations, eps_tol 1e-3, tau 1e-10, one load case). */
void aarmr_default_params(aarmr_params* p);

/* Create a mesh object (host memory only; no device allocation).  Computes
 * the hex8 element stiffness of the unit cube for nu by 2x2x2 Gauss
 * quadrature (nz = 0: the plane-stress Q4 stiffness of the unit square,
 * 2x2 Gauss) and the filter stencil.  *out receives the handle.  The
 * plane-stress grid supports precision AARMR_FP64 only.
 * Errors: AARMR_E_INVALID for non-positive sizes, sizes not divisible by
 * 2^(mg_levels-1), mg_levels outside [2, AARMR_MAX_LEVELS], Ns or Nm outside
 * [1, AARMR_MAX_BASIS], n_rhs_max outside [1, AARMR_MAX_RHS], nu outside
 * (-1, 0.5), a coarsest grid above 8192 DOFs, the DOF count >= 2^31, a
 * 3D grid whose FP64 DOF vector (3 * n_node * 8 bytes) or modulus array
 * (n_elem * 8 bytes) reaches 2^31 bytes (the fine-grid product addresses
 * them with 32-bit offsets; 446^3 elements is the largest cube), or
 * AARMR_FP32_REFINE with nz = 0. */
int aarmr_mesh_create(const aarmr_params* p, aarmr_mesh** out);

/* Release the mesh (host memory and its pinned staging buffer).  The bound
 * workspace belongs to the caller and is not freed. */
void aarmr_mesh_destroy(aarmr_mesh* m);

/* Exact number of device bytes the mesh needs: MG hierarchy, CG and
 * reduced-model vectors, PARM vectors of n_rhs_max load cases, reduction
 * scratch.  Negative on error. */
int64_t aarmr_workspace_bytes(const aarmr_mesh* m);

/* Bind caller-allocated device memory (at least aarmr_workspace_bytes,
 * 256-byte aligned) as the mesh workspace and initialise it on `stream`
 * (element stiffness, filter row sums); on the first bind also allocates a
 * 32 KiB pinned host staging buffer for scalar read-backs.  Clears the PARM
 * and the reference design.  Synchronises `stream`.  Errors:
 * AARMR_E_NO_WORKSPACE if too small, AARMR_E_INVALID if misaligned,
 * AARMR_E_HIP. */
int aarmr_bind_workspace(aarmr_mesh* m, void* dev_ptr, int64_t bytes, void* stream);

/* The analysis step by MGCG (Algorithm 2 as preconditioner of CG).
 *   rho        device [n_elem]     physical density rho~ in [0,1] (design
 *                                  density with AARMR_FILTER_INPUT)
 *   f          device [n_rhs][3][n_node] loads (not modified)
 *   n_rhs      1..n_rhs_max
 *   fixed_dofs device [n_fixed]    DOF ids (c*n_node + n) held at zero
 *   u          device [n_rhs][3][n_node] in/out: initial guess with
 *                                  AARMR_WARM_START, solution on return
 *   compliance host [n_rhs]        C_l = f_l^T u_l (eq. 3) or NULL
 *   dc         device [n_elem]     sum over load cases of dC_l/drho~ (eq. 6),
 *                                  or dC/drho (eq. 33) with
 *                                  AARMR_FILTER_INPUT; or NULL
 *   st         host                statistics, or NULL
 * Also records the physical density as the reference design K0 of the next
 * aarmr_ca_update.  Synchronises `stream`.
 * Errors: AARMR_E_INVALID (null pointers, n_rhs, a fixed DOF id out of
 * range, rho~ outside [0,1]), AARMR_E_NOT_CONVERGED (outputs written),
 * AARMR_E_SINGULAR, AARMR_E_NO_WORKSPACE, AARMR_E_HIP. */
int aarmr_solve(aarmr_mesh* m, const double* rho, const double* f, int32_t n_rhs,
                const int64_t* fixed_dofs, int64_t n_fixed, double* u,
                double* compliance, double* dc, int32_t flags, aarmr_stats* st,
                void* stream);

/* One reanalysis cycle of Algorithm 1 (lines 4-10) for every load case:
 *   K0 = K(reference design of the previous aarmr_solve / aarmr_ca_update),
 *   K_Phi = Phi^T K0 Phi (eq. 15), r_1 = u (the last solution, eq. 26),
 *   r_i = -Phi K_Phi^-1 Phi^T (K - K0) r_(i-1) (eq. 20),
 *   Gram-Schmidt orthonormalisation (named as an alternative to eq. 21),
 *   (R~^T K R~) y = R~^T f, u~ = R~ y (eqs. 22-25) and
 *   eps = ||K R~ y - f|| / ||f|| (eq. 29).
 * If eps < ca_tol, u~ is returned; otherwise MGCG runs warm-started from u~
 * and its normalised solution enters the PARM (Algorithm 1 lines 9-10).
 * Arguments as for aarmr_solve; `u` must hold each case's last solution on
 * entry.  Compliance and dc use the returned u (eq. 34 when accepted).
 * Records the new reference design.  When the previous call on this mesh
 * rejected the reduced model, the MG hierarchy of the new design is built on
 * a second stream the mesh owns (default priority, non-blocking) while the
 * reduced model runs on `stream`; it is joined into `stream` before the
 * fallback and before the call returns.  Synchronises `stream`.
 * Errors: as aarmr_solve, plus AARMR_E_STATE if a case holds fewer than Ns
 * PARM vectors or no reference design exists. */
int aarmr_ca_update(aarmr_mesh* m, const double* rho, const double* f, int32_t n_rhs,
                    const int64_t* fixed_dofs, int64_t n_fixed, double* u,
                    double* compliance, double* dc, int32_t flags,
                    aarmr_ca_stats* st, void* stream);

/* Density filter (eqs. 31-32) with cone weights max(0, rmin - |x_i - x_j|)
 * over element centres, truncated at the domain boundary and normalised by
 * the in-domain weight sums Hs.  mode 0: out = H in / Hs (eq. 31);
 * mode 1: out = H^T (in / Hs), the chain rule of eq. (33).
 * in, out: device [n_elem], distinct.  Stream-ordered, asynchronous.
 * Errors: AARMR_E_INVALID (mode, null, in == out, rmin <= 0). */
int aarmr_filter(aarmr_mesh* m, int32_t mode, const double* in, double* out, void* stream);

/* ---- building blocks (the same kernels the solvers use) --------------- */

/* Set the design state used by aarmr_apply_operator and aarmr_vcycle:
 * SIMP moduli from rho~ (device [n_elem]), the fixed-DOF mask, and the
 * multigrid hierarchy (Jacobi diagonals, Galerkin coarse operators
 * P^T A P per level, inverse of the coarsest operator).  Stream-ordered;
 * rho~ is range-checked on the next synchronising call. */
int aarmr_setup(aarmr_mesh* m, const double* rho_phys, const int64_t* fixed_dofs,
                int64_t n_fixed, void* stream);

/* y = A v on grid level `level` (0 = finest, matrix-free element-by-element
 * product of eq. (7)'s stiffness; coarser levels use the Galerkin operators
 * of aarmr_setup).  v, y: device [3][n_node(level)], distinct.  flags:
 * AARMR_INPUT_MASKED (level 0 only) promises v is zero on fixed DOFs; the
 * result is then the same and cheaper to compute.  Stream-ordered. */
int aarmr_apply_operator(aarmr_mesh* m, int32_t level, const double* v, double* y,
                         int32_t flags, void* stream);

/* z = M^-1 r: one V-cycle of Algorithm 2 from a zero initial guess on the
 * finest level.  r, z: device [3][n_node], distinct.  Stream-ordered. */
int aarmr_vcycle(aarmr_mesh* m, const double* r, double* z, void* stream);

/* Element energies e_e = u_e^T KE u_e of the unit-modulus element stiffness
 * for one displacement u (device [3][n_node]) into energy (device [n_elem]).
 * Fixed DOFs of u are treated as zero. */
int aarmr_element_energy(aarmr_mesh* m, const double* u, double* energy, void* stream);

/* Linear springs to ground on single DOFs (Section 4.3's k_in at the input
 * and k_out at the output of the displacement inverter): the stiffness is
 * K(rho~) + sum_s k_s e_s e_s^T in every solve, V-cycle and operator product
 * after the call (the hierarchy includes them from the next aarmr_setup,
 * aarmr_solve or aarmr_ca_update), and the change K - K0 of the CA step
 * (eqs. 20, 26) does not contain them.  dofs: host [n] DOF ids
 * (c * n_node + n), repeated ids add up; k: host [n], >= 0; 0 <= n <=
 * AARMR_MAX_SPRINGS; n = 0 removes all springs.  Springs on fixed DOFs have
 * no effect.  Plane-stress grid only.  The arrays are copied.
 * Errors: AARMR_E_INVALID (3D mesh, n or an id out of range, k < 0). */
int aarmr_set_springs(aarmr_mesh* m, const int64_t* dofs, const double* k, int32_t n);

/* Optimality-criteria update of the design density (the textbook OC rule
 * for eq. (3)): x_new = clamp(x * (max(0,-dc)/(lambda dv))^eta, x-move,
 * x+move, 0, 1) with lambda found by bisection in [0, 1e9] until
 * (l2-l1)/(l1+l2) <= 1e-3, the volume sum(rho~) of the filtered x_new
 * compared with volfrac * n_elem; eta = params.oc_eta.  x, dc, dv: device [n_elem]; x_new,
 * rho_phys_new: device [n_elem].  Stream-ordered. */
int aarmr_oc_update(aarmr_mesh* m, const double* x, const double* dc, const double* dv,
                    double volfrac, double move, double* x_new, double* rho_phys_new,
                    void* stream);

/* The same OC update for callers that cannot allocate device memory or
 * synchronise (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): it calls no hipMalloc, hipFree or allocating
 * library routine and reads nothing back, so the whole update is
 * stream-ordered.  Its scratch (bisection state and the volume partials of
 * the trial multipliers, 28,736 bytes) lives in a static device array that
 * each GPU holds until the process ends; the call clears what must start at
 * zero.  Every call on one GPU shares that array, so calls that overlap on
 * one GPU (other streams, other threads) race: serialise them.  The
 * partials are per reduction block, not per element, so every grid fits.
 * It issues all 67 launch pairs of the at most 200 bisection steps (pairs
 * after convergence return at once) instead of stopping at the first one
 * after convergence.  Needs the mesh's bound workspace for the filter
 * tables, as aarmr_oc_update does.  Outputs are bitwise those of
 * aarmr_oc_update.  Errors: AARMR_E_NO_WORKSPACE, AARMR_E_INVALID (null
 * argument, rmin <= 0), AARMR_E_HIP (symbol lookup or launch). */
int aarmr_oc_update_noalloc(aarmr_mesh* m, const double* x, const double* dc, const double* dv,
                            double volfrac, double move, double* x_new, double* rho_phys_new,
                            void* stream);

/* Autotuner of the fine-grid operator's launch shape.  The z-marching
 * kernel runs tiles of 30 node columns by ROWS - 1 node rows of the x-y
 * plane (ROWS in {8, 12, 16}; 16 by default), each marching over a
 * chunk of node planes.
 * The autotuner times every tile height (16 being the default) with the
 * residency-sized default chunk length and candidate lengths 2..n_z+1 on this
 * mesh's grid (scratch operands: the solver state is untouched), the best of
 * 3 rounds of 5 launches each after a warm-up, and keeps the fastest for the
 * mesh's later products (FP64 and, in the refinement form, FP32).
 * tz_out: host [2] or NULL, receives the chosen shape words (chunk length in
 * the low 16 bits, 0 = the default; tile rows above them, 0 = the
 * default).  Every product gives the same bits for every shape; CG's dot
 * products are summed per workgroup of that product, so a solve's last bits
 * may change with it.  On the plane-stress grid there is nothing to tune:
 * tz_out receives 0, 0.  Synchronises `stream`.  Errors:
 * AARMR_E_NO_WORKSPACE, AARMR_E_HIP. */
int aarmr_autotune(aarmr_mesh* m, int32_t* tz_out, void* stream);

/* Set the fine-grid operator's launch shapes without timing (for instance
 * the words an earlier aarmr_autotune returned for the same grid): tz64 for
 * FP64 products, tz32 for the refinement form's FP32 products.  A shape word
 * is chunk_length | (tile_rows << 16): chunk length 0 (default) or >= 2
 * (lengths above n_z + 1 are clamped to it), tile rows 0 (default, 16),
 * 8, 12 or 16.  0 restores both defaults.  Host-only, takes effect at the
 * next product.  Errors: AARMR_E_INVALID (null mesh, a negative word, a
 * chunk length of 1, other tile rows). */
int aarmr_set_chunk(aarmr_mesh* m, int32_t tz64, int32_t tz32);

/* ---- batched form ------------------------------------------------------
 * Many independent analyses (meshes of uneven size, each with its own load
 * cases) run concurrently.  Each item is one aarmr_solve call on its own mesh
 * (and therefore its own workspace); the items are spread over `n_streams`
 * caller-owned streams, each driven by one host worker thread of the
 * library, largest items first.  The GPU overlaps the items in flight on
 * different streams.  An item's result does not depend on the batch it runs
 * in (every kernel of an item reads and writes only that item's memory in a
 * fixed order), so it equals the item solved alone, bit for bit. */
typedef struct aarmr_batch_item {
  aarmr_mesh* mesh;             /* distinct meshes per item (workspace bound) */
  const double* rho;            /* as aarmr_solve */
  const double* f;
  int32_t n_rhs;
  const int64_t* fixed_dofs;
  int64_t n_fixed;
  double* u;
  double* compliance;           /* host [n_rhs] or NULL */
  double* dc;                   /* device [n_elem] or NULL */
  int32_t flags;
  int32_t status;               /* out: the item's aarmr_solve return code */
  aarmr_stats stats;            /* out */
  int32_t done;                 /* out: set to 1 (release store) once status,
                                   stats and the item's outputs are final */
} aarmr_batch_item;

/* Solve every item (see above).  streams: host array of n_streams hipStream_t
 * handles (1 <= n_streams <= 64).  Returns AARMR_OK if every item returned
 * AARMR_OK, else the first non-OK item status in item order (each item's own
 * code is in its `status`).  All streams are synchronised on return.
 * Errors: AARMR_E_INVALID for a null or repeated mesh, n_items < 0 or a bad
 * n_streams; item errors as aarmr_solve. */
int aarmr_batch_solve(aarmr_batch_item* items, int32_t n_items, void* const* streams,
                      int32_t n_streams);

/* Asynchronous form of aarmr_batch_solve, for callers that keep submitting
 * work while a batch runs (the serving loop).  aarmr_batch_submit validates
 * the items like aarmr_batch_solve, clears every item's `done`, starts the
 * worker threads and returns at once; *out receives a handle.  The items
 * array, the streams array and all memory the items name must stay valid
 * until aarmr_batch_wait returns.  Errors: as aarmr_batch_solve's argument
 * errors (nothing is started then, *out is NULL). */
typedef struct aarmr_batch aarmr_batch;
int aarmr_batch_submit(aarmr_batch_item* items, int32_t n_items, void* const* streams,
                       int32_t n_streams, aarmr_batch** out);

/* Non-blocking progress: *n_done receives the number of items finished so
 * far (those whose `done` is 1).  Returns AARMR_OK, or AARMR_E_INVALID for a
 * null argument. */
int aarmr_batch_poll(aarmr_batch* b, int32_t* n_done);

/* Block until every item is finished, synchronise the streams and release
 * the handle.  Returns AARMR_OK or the first non-OK item status in item
 * order, like aarmr_batch_solve. */
int aarmr_batch_wait(aarmr_batch* b);

/* Thread-local description of the last error on this thread ("" if none). */
const char* aarmr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* AARMR_H */
