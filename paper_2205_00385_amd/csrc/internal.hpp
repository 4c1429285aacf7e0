// Internal declarations of the AARMR HIP library (gfx950).
//
// Layout: DOF vectors are SoA [3][n_node] in FP64 (or FP32 inside the
// refinement form); elements and nodes are x-fastest.  The fixed-DOF mask is
// one byte per node with bit c set when component c is fixed.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "aarmr.h"
#include "walsh.hpp"

namespace aarmr {

constexpr int kRedBlocks = 512;    // partial-sum blocks of one reduction
constexpr int kFusedBlocks = 2048; // block limit of the CG updates with folded reductions
constexpr int kRedSlots = 24;      // dot products one reduction launch can hold
constexpr int kMaxIt = 4096;       // bound of cg_maxit (scalar history length)
constexpr int kGJBlock = 64;       // block size of the coarsest inversion

// nz == 0 is the plane-stress grid: nx * ny unit squares, (nx+1)(ny+1)
// nodes with 2 DOFs each.
struct Grid {
  int nx, ny, nz;          // elements
  int64_t ne, nn;          // elements, nodes
};

inline Grid make_grid(int nx, int ny, int nz) {
  Grid g;
  g.nx = nx; g.ny = ny; g.nz = nz;
  g.ne = (int64_t)nx * ny * (nz > 0 ? nz : 1);
  g.nn = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  return g;
}

// Reduction scratch: per-slot block partials.
struct RedScratch {
  double* partial;     // [kRedSlots][kRedBlocks]
};

// k dot products a_i . b_i (b_i == nullptr: plain sum of a_i) of vectors of
// element type T, accumulated and returned in FP64.
// Load cases solved in lock step by one set of launches: case l's vectors
// start at l * vs, its CG scalars at l * ss, its workgroup partials at l * ps
// and its host-visible partials at l * hs; active (device, n entries): 0 for
// a case that has finished, whose updates are then skipped.  n = 1 with zero
// strides is the single-case solve.
struct MultiRhs {
  int n = 1;
  int64_t vs = 0;
  int ss = 0, ps = 0, hs = 0;
  const int* active = nullptr;
};

template <typename T>
struct DotSetT {
  const T* a[kRedSlots];
  const T* b[kRedSlots];
  double* out[kRedSlots];
  int k;               // number of products
  int64_t n;           // length
};
using DotSet = DotSetT<double>;

// ---- fine-level operator (element-by-element, reflection-blocked) --------
// mode 0: y = A v = Df K Df v + (I - Df) v for any v; mode 1: y = Df K Df v;
// mode 2: y = Df K v for a v that is zero on fixed DOFs (then equal to both
// A v and Df K Df v), the form every solver-internal product uses.
// tz: z-chunk length (node planes per workgroup); <= 0 takes the default
// sized from the kernel's residency (one round of workgroups fills the GPU).
void launch_ebe(const Grid& g, const WalshConsts& K, const double* E, const uint8_t* mask,
                const double* v, double* y, int mode, hipStream_t s, int tz = 0);
void launch_ebe_f32(const Grid& g, const WalshConsts& K, const float* E, const uint8_t* mask,
                    const float* v, float* y, int mode, hipStream_t s, int tz = 0,
                    int nr = 1);
// The mode-2 product feeding a damped-Jacobi sweep: out = v + omega dinv
// (b - A v), out distinct from v.
void launch_ebe_jacobi(const Grid& g, const WalshConsts& K, const double* E, const uint8_t* mask,
                       const double* v, const double* b, const double* dinv, double omega,
                       double* out, hipStream_t s, int tz = 0);
// The same two products with CG's dot product folded in: each workgroup w
// writes part[w], the sum over the nodes it owns of v . y (launch_ebe_dot,
// mode 2: p^T A p) or b . out (launch_ebe_jacobi_dot: r^T z); the return
// value is the number of partials.  part holds ebe_partials_max(g) entries.
int ebe_partials_max(const Grid& g);
int launch_ebe_dot(const Grid& g, const WalshConsts& K, const double* E, const uint8_t* mask,
                   const double* v, double* y, double* part, hipStream_t s, int tz = 0);
int launch_ebe_jacobi_dot(const Grid& g, const WalshConsts& K, const double* E,
                          const uint8_t* mask, const double* v, const double* b,
                          const double* dinv, double omega, double* out, double* part,
                          hipStream_t s, int tz = 0);
// FP32 forms of the two (vectors FP32, partials summed in FP64).
int launch_ebe_f32_dot(const Grid& g, const WalshConsts& K, const float* E, const uint8_t* mask,
                       const float* v, float* y, double* part, hipStream_t s, int tz = 0,
                       int nr = 1, int pst = 0);
int launch_ebe_jacobi_f32_dot(const Grid& g, const WalshConsts& K, const float* E,
                              const uint8_t* mask, const float* v, const float* b,
                              const float* dinv, float omega, float* out, double* part,
                              hipStream_t s, int tz = 0, int nr = 1, int pst = 0);
void launch_energy_walsh(const Grid& g, const WalshConsts& K, const uint8_t* mask,
                         const double* u, double* energy, hipStream_t s);
void launch_simp(int64_t ne, const double* rho, double E0, double Emin, double p, double* E,
                 float* E32, unsigned* bad, hipStream_t s);
void launch_diff(int64_t n, const double* a, const double* b, double* out, hipStream_t s);
// ncomp: DOFs per node (3, or 2 on the plane-stress grid)
void launch_build_mask(int64_t nn, const int64_t* fixed, int64_t nfixed, uint8_t* mask,
                       unsigned* bad, hipStream_t s, int ncomp = 3);
void launch_mask_diff(int64_t nn, const uint8_t* a, const uint8_t* b, unsigned* flags,
                      hipStream_t s);
void launch_diag_fine(const Grid& g, const double* KE, const double* E, const uint8_t* mask,
                      double* dinv, float* dinv32, hipStream_t s);
void launch_dc_accum(int64_t ne, const double* rho, const double* energy, double E0, double Emin,
                     double p, double* dc, int first, hipStream_t s);

// ---- multigrid ------------------------------------------------------------
// Coarse element matrices are symmetric 24x24 and stored packed (upper
// triangle, row-major: 300 entries) and entry-major, Ke[sym_index(r,c) *
// n_elem + e], so that threads on consecutive elements read consecutive
// addresses.
constexpr int kSymEntries = 300;
__host__ __device__ constexpr int sym_index(int r, int c) {
  return r <= c ? r * 24 - (r * (r - 1)) / 2 + (c - r) : c * 24 - (c * (c - 1)) / 2 + (r - c);
}
// Level-1 operators from the fine moduli: fast path for every parent, exact
// masked product for the parents flagged in eflag (1 = touches a fixed DOF),
// whose indices are listed in list[0..*count); list entries w < cap are also
// stored compactly, Kcomp[entry][w].
// all: also the fast-path matrices of the unflagged parents (needed only when
// level 1 is the coarsest; otherwise nothing reads them).
void launch_galerkin_from_fine(const Grid& coarse, const double* KE, const double* Mc,
                               const double* E, const uint8_t* mask, uint8_t* eflag, int* list,
                               int* count, double* Kc, double* Kcomp, int cap, hipStream_t s,
                               bool all);
// Level-2 Galerkin matrices from the fine moduli (N2: [64][300] descendant
// matrices) for parents without a flagged level-1 child; the others from the
// stored flagged level-1 matrices K1 and the moduli.  list2/count2: scratch.
void launch_galerkin_l2_from_fine(const Grid& l2, const double* N2, const double* Mc,
                                  const double* E, const uint8_t* eflag1, int* list2, int* count2,
                                  const double* K1, double* K2, hipStream_t s);
// Level-1 inverse Jacobi diagonal from the moduli (unflagged parents) and the
// stored matrices (flagged ones).
void launch_diag_l1(const Grid& g, const double* Ke, const double* Mc, const double* E,
                    const uint8_t* eflag, double* dinv, float* dinv32, hipStream_t s);
void launch_galerkin_from_coarse(const Grid& coarse, const double* Kf, double* Kc, hipStream_t s);
void launch_apply_elemmat(const Grid& g, const double* Ke, const double* v, double* y,
                          hipStream_t s);
// Level-1 product through the Walsh form of the child matrices:
// Bw = W M_0 W / 64 (24 x 24, Walsh x component basis, index 3k + s), Y a
// [24][ne] element-product buffer.  Flagged parents (eflag 1, indices in
// list[0..*count), nflag = *count as read back by the host) use their stored Ke.
void launch_apply_l1(const Grid& g, const double* Ke, const double* Kcomp, int cap,
                     const double* Bw, const double* Ef, const uint8_t* eflag, const int* list,
                     const int* count, int nflag, const double* v, double* Y, double* y,
                     hipStream_t s);
// FP32 forms of the Jacobi-fused products and restriction (as the FP64 ones).
void launch_apply_l1_jacobi_f32(const Grid& g, const double* Ke, const double* Kcomp, int cap,
                                const float* Bw, const float* Ef, const uint8_t* eflag,
                                const int* list, const int* count, int nflag, float* x, float* Y,
                                const float* b, const float* dinv, float omega, hipStream_t s, int nr = 1);
void launch_apply_elemmat_jacobi_f32(const Grid& g, const float* Ke, const float* v,
                                     const float* b, const float* dinv, float omega, float* out,
                                     hipStream_t s, int nr = 1);
void launch_restrict_jacobi_f32(const Grid& coarse, const float* bf, const float* tf,
                                const uint8_t* mask, float* bc, const float* dinv_c, float omega,
                                float* xc, hipStream_t s, int nr = 1);
void launch_apply_l1_f32(const Grid& g, const double* Ke, const double* Kcomp, int cap,
                         const float* Bw, const float* Ef, const uint8_t* eflag, const int* list,
                         const int* count, int nflag, const float* v, float* Y, float* y,
                         hipStream_t s, int nr = 1);
void launch_diag_elemmat(const Grid& g, const double* Ke, double* dinv, float* dinv32,
                         hipStream_t s);
// Transfers act per component; ncomp = 2 on the plane-stress grid (nz = 0).
void launch_restrict(const Grid& coarse, const double* bf, const double* tf, const uint8_t* mask,
                     double* bc, hipStream_t s, int ncomp = 3);
void launch_prolong_add(const Grid& fine, const double* xc, const uint8_t* mask, double* xf,
                        hipStream_t s, int ncomp = 3);
void launch_jacobi_first(int64_t n3, const double* b, const double* dinv, double omega, double* x,
                         hipStream_t s);
// Fused damped-Jacobi sweeps (3D hierarchy): restriction that also forms the
// coarse level's first sweep xc = omega dinv_c bc; the level-1 product that
// ends in x += omega dinv (b - A x) in place; the stored-matrix product that
// writes out = v + omega dinv (b - A v) (out distinct from v).
void launch_restrict_jacobi(const Grid& coarse, const double* bf, const double* tf,
                            const uint8_t* mask, double* bc, const double* dinv_c, double omega,
                            double* xc, hipStream_t s);
void launch_apply_l1_jacobi(const Grid& g, const double* Ke, const double* Kcomp, int cap,
                            const double* Bw, const double* Ef, const uint8_t* eflag,
                            const int* list, const int* count, int nflag, double* x, double* Y,
                            const double* b, const double* dinv, double omega, hipStream_t s);
void launch_apply_elemmat_jacobi(const Grid& g, const double* Ke, const double* v, const double* b,
                                 const double* dinv, double omega, double* out, hipStream_t s);
void launch_jacobi_update(int64_t n3, const double* b, const double* t, const double* dinv,
                          double omega, double* x, hipStream_t s);
void launch_assemble_dense(const Grid& g, const double* Ke, double* A, hipStream_t s);
// In-place inverse of the SPD n x n matrix A (blocked symmetric Gauss-Jordan).
// Scratch: P holds two 64 x 64 pivot inverses, T, C and Tb one 64 x n panel
// each.
void launch_gj_invert(int n, double* A, double* P, double* T, double* C, double* Tb,
                      hipStream_t s);
void launch_gemv(int n, const double* A, const double* x, double* y, hipStream_t s);
// FP32 V-cycle pieces (vectors FP32; element matrices and the coarsest
// inverse stay FP64 and are applied with FP32 vectors).
void launch_apply_elemmat_f32(const Grid& g, const float* Ke, const float* v, float* y,
                              hipStream_t s, int nr = 1);
void launch_restrict_f32(const Grid& coarse, const float* bf, const float* tf,
                         const uint8_t* mask, float* bc, hipStream_t s, int nr = 1);
void launch_prolong_add_f32(const Grid& fine, const float* xc, const uint8_t* mask, float* xf,
                            hipStream_t s, int nr = 1);
void launch_jacobi_first_f32(int64_t n3, const float* b, const float* dinv, float omega, float* x,
                             hipStream_t s, int nr = 1);
void launch_jacobi_update_f32(int64_t n3, const float* b, const float* t, const float* dinv,
                              float omega, float* x, hipStream_t s, int nr = 1);
void launch_gemv_f32(int n, const double* A, const float* x, float* y, hipStream_t s, int nr = 1);

// ---- vector kernels and reductions ----------------------------------------
void launch_multidot(const DotSet& d, const RedScratch& rs, hipStream_t s);
void launch_multidot_f32(const DotSetT<float>& d, const RedScratch& rs, hipStream_t s);
// FP32 direction update after a separate r^T z; the scalars stay FP64 in
// device memory and the update is formed in FP64 before rounding to FP32.
void launch_cg_p_f32(int64_t n, const double* rz_new, const double* rz_old, const float* z,
                     float* p, hipStream_t s);
// Refinement transfers: dst32 = src64 / sqrt(*nrm2);  x64 += sqrt(*nrm2) d32.
// dst = (float)src, elementwise.
void launch_to_f32(int64_t n, const double* src, float* dst, hipStream_t s);
void launch_to_f32_scaled(int64_t n, const double* src, const double* nrm2, float* dst,
                          hipStream_t s);
void launch_add_scaled_f32(int64_t n, const float* d, const double* nrm2, double* x,
                           hipStream_t s);
void launch_copy_f32(int64_t n, const float* src, float* dst, hipStream_t s);
void launch_copy_masked(const Grid& g, const double* src, const uint8_t* mask, double* dst,
                        hipStream_t s, int ncomp = 3);
void launch_sub(int64_t n, const double* a, const double* b, double* out, hipStream_t s);
// CG with folded reductions.  dot_blocks(n): the block count of one dot's
// partials; fused_blocks(n): that of the fused updates (each finishes the
// dot partials it needs); launch_dot_partials writes a^T b's partials to
// part[0..dot_blocks(n)).
int dot_blocks(int64_t n);
int fused_blocks(int64_t n);
void launch_dot_partials(int64_t n, const double* a, const double* b, double* part,
                         hipStream_t s);
// pq finished from the n_part entries of pq_part (n_part <= 0: dot_blocks(n)),
// stored to *pq and rr_part[fused_blocks(n)]; x += alpha p, r -= alpha q with
// alpha = *rz / pq; rr_part[0..fused_blocks(n)) = partials of r^T r;
// z0 = omega dinv r unless z0 is null.
void launch_cg_xr_fused(int64_t n, const double* rz, const double* pq_part, int n_part,
                        double* pq, double* x, double* r, const double* p, const double* q,
                        double* rr_part, const double* dinv, double omega, double* z0,
                        hipStream_t s);
// rz_new finished from the n_part entries of rz_part (n_part <= 0:
// dot_blocks(n)), stored to *rz_new; p = z + (rz_new / *rz_old) p.
void launch_cg_p_fused(int64_t n, const double* rz_part, int n_part, double* rz_new,
                       const double* rz_old, const double* z, double* p, hipStream_t s);
// The FP32 forms (FP32 vectors, FP64 scalars and partials); the x/r update
// also stores *rz at rr_part[fused_blocks(n) + 1] and always writes z0.
void launch_cg_xr_fused_f32(int64_t n, const double* rz, const double* pq_part, int n_part,
                            double* pq, float* x, float* r, const float* p, const float* q,
                            double* rr_part, const float* dinv, float omega, float* z0,
                            hipStream_t s,
                            const MultiRhs& mr = MultiRhs());
void launch_cg_p_fused_f32(int64_t n, const double* rz_part, int n_part, double* rz_new,
                           const double* rz_old, const float* z, float* p, hipStream_t s,
                            const MultiRhs& mr = MultiRhs());
void launch_scale_by_inv_sqrt(int64_t n, const double* src, const double* nrm2, double* dst,
                              hipStream_t s);
// out = sum_j coef[j] * V_j (+ add) with coefficients read from device memory
void launch_lincomb(int64_t n, int k, const double* const* V, const double* coef, double sign,
                    const double* add, double* out, hipStream_t s);
// Cholesky solve of A x = b (n x n, row stride lda, entries averaged with
// their transpose); not positive definite: bit 4 of *bad and x = 0.
void launch_small_spd_solve(int n, int lda, const double* A, const double* b, double* x,
                            unsigned* bad, hipStream_t s);
// Gram-Schmidt keep test on a projected column (n0, n1: squared norms before
// and after the projections): dst = src / sqrt(n1) and *keep = 1 when
// sqrt(n1) > tau sqrt(n0), else dst = 0 and *keep = 0.
void launch_gs_keep(int64_t n, const double* src, const double* n0, const double* n1, double tau,
                    double* dst, double* keep, hipStream_t s);
// Thin SVD of the small n x n matrix T (row-major): left singular vectors of
// sigma > tau sigma_1, decreasing, column by column into coef[j * n + i];
// their count (as a double) into *kept.
void launch_small_svd(int n, const double* T, double tau, double* coef, double* kept,
                      hipStream_t s);

// ---- plane stress (bilinear quadrilaterals, grids with nz = 0) -------------
// Coarse element matrices are symmetric 8x8, packed (upper triangle,
// row-major: 36 entries) and entry-major like the 3D ones.  KE: the 8x8
// unit-modulus element stiffness, row-major, DOF 2a + c of corner a = dx + 2dy.
constexpr int kSymEntries2 = 36;
__host__ __device__ constexpr int sym_index2(int r, int c) {
  return r <= c ? r * 8 - (r * (r - 1)) / 2 + (c - r) : c * 8 - (c * (c - 1)) / 2 + (r - c);
}
// mode as for launch_ebe
void launch_q4_apply(const Grid& g, const double* KE, const double* E, const uint8_t* mask,
                     const double* v, double* y, int mode, hipStream_t s);
// energy_e = u_e^T KE w_e (w = u: strain energy)
void launch_q4_energy(const Grid& g, const double* KE, const uint8_t* mask, const double* u,
                      const double* w, double* energy, hipStream_t s);
// Grounded springs on single DOFs (passed by value to the kernels).
struct SpringSet {
  int n;
  int64_t dof[AARMR_MAX_SPRINGS];
  double k[AARMR_MAX_SPRINGS];
};
void launch_springs_add(const SpringSet& S, const Grid& g, const uint8_t* mask, const double* v,
                        double* y, hipStream_t s);
void launch_springs_diag(const SpringSet& S, const Grid& g, const uint8_t* mask, double* dinv,
                         hipStream_t s);
// level-1 contribution (Df P)^T S (Df P); coarse = the level-1 grid
void launch_springs_galerkin(const SpringSet& S, const Grid& coarse, const uint8_t* mask,
                             double* Kc, hipStream_t s);
void launch_q4_diag(const Grid& g, const double* KE, const double* E, const uint8_t* mask,
                    double* dinv, hipStream_t s);
// Level 1: (Df P)^T K (Df P) per parent from the fine moduli and mask.
void launch_q4_galerkin_from_fine(const Grid& coarse, const double* KE, const double* E,
                                  const uint8_t* mask, double* Kc, hipStream_t s);
void launch_q4_galerkin_from_coarse(const Grid& coarse, const double* Kf, double* Kc,
                                    hipStream_t s);
void launch_q4_apply_elemmat(const Grid& g, const double* Ke, const double* v, double* y,
                             hipStream_t s);
void launch_q4_diag_elemmat(const Grid& g, const double* Ke, double* dinv, hipStream_t s);
void launch_q4_assemble_dense(const Grid& g, const double* Ke, double* A, hipStream_t s);

// ---- filter, OC --------------------------------------------------------------
// Cone weights max(0, r - |d|) of the filter offsets, (2R+1)^3 with
// R = ceil(r) - 1, offset (dk, dj, di) at ((dk + R)(2R+1) + dj + R)(2R+1) + di + R.
void filter_weights(double r, double* W);
int filter_taps(double r);
void launch_filter_rowsum(const Grid& g, double r, double* Hs, hipStream_t s);
void launch_filter(const Grid& g, double r, const double* W, int mode, const double* Hs,
                   const double* in, double* out, hipStream_t s);
void launch_fill(int64_t n, double v, double* out, hipStream_t s);
void launch_fill_f32(int64_t n, float v, float* out, hipStream_t s);
// OC bisection, three levels per launch pair: block partials of the volume
// sum_j cw_j x_new_j for the seven multipliers three levels can visit
// (nparts blocks), then the bisection steps on lam; x_new at the last
// multiplier evaluated.
void launch_oc_step3(int64_t ne, const double* x, const double* dc, const double* dv,
                     const double* cw, double move, double eta, const double* lam,
                     double* partial, int nparts, hipStream_t s);
void launch_oc_bisect3(double* lam, const double* partial, int nparts, double target,
                       hipStream_t s);
void launch_oc_final(int64_t ne, const double* x, const double* dc, const double* dv, double move,
                     double eta, const double* lam, double* xnew, hipStream_t s);
void launch_oc_init(double* lam, hipStream_t s);

}  // namespace aarmr
