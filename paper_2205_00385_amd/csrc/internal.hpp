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

namespace aarmr {

constexpr int kRedBlocks = 512;    // partial-sum blocks of one reduction
constexpr int kRedSlots = 24;      // dot products one reduction launch can hold
constexpr int kMaxIt = 4096;       // bound of cg_maxit (scalar history length)
constexpr int kGJBlock = 64;       // block size of the coarsest inversion

struct Grid {
  int nx, ny, nz;          // elements
  int64_t ne, nn;          // elements, nodes
};

inline Grid make_grid(int nx, int ny, int nz) {
  Grid g;
  g.nx = nx; g.ny = ny; g.nz = nz;
  g.ne = (int64_t)nx * ny * nz;
  g.nn = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  return g;
}

// Reduction scratch: per-slot partials, a ticket counter for the
// last-block-finishes pattern, and the output scalars.
struct RedScratch {
  double* partial;     // [kRedSlots][kRedBlocks]
  unsigned* ticket;    // [1]
};

struct DotSet {
  const double* a[kRedSlots];
  const double* b[kRedSlots];
  double* out[kRedSlots];
  int k;               // number of products
  int64_t n;           // length
};

// ---- fine-level operator (element-by-element) ---------------------------
// mode 0: y = A v with identity rows on fixed DOFs; mode 1: y = Df K Df v.
void launch_ebe_fine(const Grid& g, const double* KE, const double* E, const uint8_t* mask,
                     const double* v, double* y, int mode, hipStream_t s);
void launch_ebe_fine_f32(const Grid& g, const float* ke32, const float* E, const uint8_t* mask,
                         const float* v, float* y, hipStream_t s);
void launch_simp(int64_t ne, const double* rho, double E0, double Emin, double p, double* E,
                 float* E32, unsigned* bad, hipStream_t s);
void launch_diff(int64_t n, const double* a, const double* b, double* out, hipStream_t s);
void launch_build_mask(int64_t nn, const int64_t* fixed, int64_t nfixed, uint8_t* mask,
                       unsigned* bad, hipStream_t s);
void launch_diag_fine(const Grid& g, const double* KE, const double* E, const uint8_t* mask,
                      double* dinv, float* dinv32, hipStream_t s);
void launch_energy(const Grid& g, const double* KE, const uint8_t* mask, const double* u,
                   double* energy, hipStream_t s);
void launch_dc_accum(int64_t ne, const double* rho, const double* energy, double E0, double Emin,
                     double p, double* dc, int first, hipStream_t s);

// ---- multigrid ------------------------------------------------------------
void launch_galerkin_from_fine(const Grid& coarse, const double* KE, const double* E,
                               const uint8_t* mask, double* Kc, hipStream_t s);
void launch_galerkin_from_coarse(const Grid& coarse, const double* Kf, double* Kc, hipStream_t s);
void launch_apply_elemmat(const Grid& g, const double* Ke, const double* v, double* y,
                          hipStream_t s);
void launch_diag_elemmat(const Grid& g, const double* Ke, double* dinv, float* dinv32,
                         hipStream_t s);
void launch_restrict(const Grid& coarse, const double* bf, const double* tf, const uint8_t* mask,
                     double* bc, hipStream_t s);
void launch_prolong_add(const Grid& fine, const double* xc, const uint8_t* mask, double* xf,
                        hipStream_t s);
void launch_jacobi_first(int64_t n3, const double* b, const double* dinv, double omega, double* x,
                         hipStream_t s);
void launch_jacobi_update(int64_t n3, const double* b, const double* t, const double* dinv,
                          double omega, double* x, hipStream_t s);
void launch_assemble_dense(const Grid& g, const double* Ke, double* A, hipStream_t s);
void launch_gj_invert(int n, double* A, double* P, double* T, double* Rw, hipStream_t s);
void launch_gemv(int n, const double* A, const double* x, double* y, hipStream_t s);

// ---- vector kernels and reductions ----------------------------------------
void launch_multidot(const DotSet& d, const RedScratch& rs, hipStream_t s);
void launch_copy_masked(const Grid& g, const double* src, const uint8_t* mask, double* dst,
                        hipStream_t s);
void launch_sub(int64_t n, const double* a, const double* b, double* out, hipStream_t s);
void launch_cg_xr(int64_t n, const double* rz, const double* pq, double* x, double* r,
                  const double* p, const double* q, hipStream_t s);
void launch_cg_p(int64_t n, const double* rz_new, const double* rz_old, const double* z,
                 double* p, hipStream_t s);
void launch_scale_by_inv_sqrt(int64_t n, const double* src, const double* nrm2, double* dst,
                              hipStream_t s);
// out = sum_j coef[j] * V_j (+ add) with coefficients read from device memory
void launch_lincomb(int64_t n, int k, const double* const* V, const double* coef, double sign,
                    const double* add, double* out, hipStream_t s);
void launch_small_spd_solve(int n, int lda, const double* A, const double* b, double* x,
                            unsigned* bad, hipStream_t s);
void launch_gs_step(int64_t n, int j, double* const* Q, const double* h, double* v, hipStream_t s);

// ---- filter, OC --------------------------------------------------------------
void launch_filter_rowsum(const Grid& g, double r, double* Hs, hipStream_t s);
void launch_filter(const Grid& g, double r, int mode, const double* Hs, const double* in,
                   double* out, hipStream_t s);
void launch_oc_step(int64_t ne, const double* x, const double* dc, const double* dv,
                    double move, double* lam, double* xnew, hipStream_t s);
void launch_oc_bisect(double* lam, const double* vol, double target, hipStream_t s);
void launch_oc_init(double* lam, hipStream_t s);

// ---- FP32 refinement form -----------------------------------------------------
void launch_to_f32(int64_t n, const double* a, float* b, hipStream_t s);
void launch_add_f32_to_f64(int64_t n, const float* a, double* b, hipStream_t s);
void launch_jacobi_first_f32(int64_t n3, const float* b, const float* dinv, float omega, float* x,
                             hipStream_t s);
void launch_jacobi_update_f32(int64_t n3, const float* b, const float* t, const float* dinv,
                              float omega, float* x, hipStream_t s);
void launch_restrict_f32(const Grid& coarse, const float* bf, const float* tf,
                         const uint8_t* mask, float* bc, hipStream_t s);
void launch_prolong_add_f32(const Grid& fine, const float* xc, const uint8_t* mask, float* xf,
                            hipStream_t s);
void launch_apply_elemmat_f32(const Grid& g, const float* Ke, const float* v, float* y,
                              hipStream_t s);
void launch_convert_f32(int64_t n, const double* a, float* b, hipStream_t s);
void launch_gemv_f32in(int n, const double* A, const float* x, float* y, hipStream_t s);

}  // namespace aarmr
