// Plane-stress path (the paper's 2D examples, Sections 4.1, 4.2.1, 4.3): the
// bilinear quadrilateral (Q4) operator, its element energies and Jacobi
// diagonal, and the 2D Galerkin hierarchy (Algorithm 2) with 8x8 coarse
// element matrices.  Grids are nx x ny unit squares, nodes x-fastest
// (i + (nx+1) j), local corner a = dx + 2 dy, DOF vectors SoA [2][n_node].
#include "internal.hpp"

namespace aarmr {

namespace {

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

__host__ __device__ constexpr int s2(int r, int c) { return sym_index2(r, c); }

// Weight of parent corner A (0/1) at refined position pos (0, 1, 2) along an axis.
__device__ inline double phi1q(int pos, int A) {
  return pos == 1 ? 0.5 : ((pos >> 1) == A ? 1.0 : 0.0);
}

// y = A v (mode 0), Df K Df v (mode 1) or Df K v for a v zero on fixed DOFs
// (mode 2): thread per node, the (up to) 4 adjacent elements in corner order.
__global__ void __launch_bounds__(256) k_q4_apply(int nx, int ny, const double* __restrict__ KE,
                                                  const double* __restrict__ E,
                                                  const uint8_t* __restrict__ mask,
                                                  const double* __restrict__ v,
                                                  double* __restrict__ y, int mode) {
  const int64_t nn = (int64_t)(nx + 1) * (ny + 1);
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const int i = (int)(n % (nx + 1)), j = (int)(n / (nx + 1));
  double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int ex = i - (a & 1), ey = j - (a >> 1);
    if (ex < 0 || ex >= nx || ey < 0 || ey >= ny) continue;
    const double w = E[(int64_t)ex + (int64_t)nx * ey];
    double t0 = 0.0, t1 = 0.0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t nb = (int64_t)(ex + (b & 1)) + (int64_t)(nx + 1) * (ey + (b >> 1));
      const uint8_t mb = (mode != 2) ? mask[nb] : 0;
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        const double vb = ((mb >> d) & 1) ? 0.0 : v[d * nn + nb];
        t0 = fma(KE[(2 * a) * 8 + 2 * b + d], vb, t0);
        t1 = fma(KE[(2 * a + 1) * 8 + 2 * b + d], vb, t1);
      }
    }
    acc0 = fma(w, t0, acc0);
    acc1 = fma(w, t1, acc1);
  }
  const uint8_t m = mask[n];
  const double r[2] = {acc0, acc1};
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const bool fx = (m >> c) & 1;
    y[c * nn + n] = fx ? (mode == 0 ? v[c * nn + n] : 0.0) : r[c];
  }
}

// energy_e = u_e^T KE w_e (unit modulus; w = u: the strain energy), fixed
// DOFs read as zero.
__global__ void k_q4_energy(int nx, int ny, const double* __restrict__ KE,
                            const uint8_t* __restrict__ mask, const double* __restrict__ u,
                            const double* __restrict__ w, double* __restrict__ energy) {
  const int64_t nn = (int64_t)(nx + 1) * (ny + 1);
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)nx * ny) return;
  const int ex = (int)(e % nx), ey = (int)(e / nx);
  double ue[8], we[8];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int64_t nb = (int64_t)(ex + (b & 1)) + (int64_t)(nx + 1) * (ey + (b >> 1));
    const uint8_t mb = mask[nb];
    ue[2 * b] = (mb & 1) ? 0.0 : u[nb];
    ue[2 * b + 1] = (mb & 2) ? 0.0 : u[nn + nb];
    we[2 * b] = (mb & 1) ? 0.0 : w[nb];
    we[2 * b + 1] = (mb & 2) ? 0.0 : w[nn + nb];
  }
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) t = fma(KE[r * 8 + q], we[q], t);
    s = fma(ue[r], t, s);
  }
  energy[e] = s;
}

// Inverse Jacobi diagonal of the fine operator (identity on fixed DOFs).
__global__ void k_q4_diag(int nx, int ny, const double* __restrict__ KE,
                          const double* __restrict__ E, const uint8_t* __restrict__ mask,
                          double* __restrict__ dinv) {
  const int64_t nn = (int64_t)(nx + 1) * (ny + 1);
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const int i = (int)(n % (nx + 1)), j = (int)(n / (nx + 1));
  double d[2] = {0.0, 0.0};
  for (int a = 0; a < 4; ++a) {
    const int ex = i - (a & 1), ey = j - (a >> 1);
    if (ex < 0 || ex >= nx || ey < 0 || ey >= ny) continue;
    const double w = E[(int64_t)ex + (int64_t)nx * ey];
    for (int c = 0; c < 2; ++c) d[c] += w * KE[(2 * a + c) * 9];
  }
  const uint8_t m = mask[n];
  for (int c = 0; c < 2; ++c) dinv[c * nn + n] = (((m >> c) & 1) || d[c] == 0.0) ? 1.0 : 1.0 / d[c];
}

// Galerkin matrix of every parent of the coarse grid (cnx x cny), one thread
// per parent: Kc[I][J] = sum over children c and their corners a, b of
// P_c[a][I/2] P_c[b][J/2] K_c[2a + I%2][2b + J%2].  FROM_FINE: K_c = E_c KE
// with the rows and columns of fixed fine DOFs removed (masked P);
// otherwise K_c is the previous level's packed matrix.
template <bool FROM_FINE>
__global__ void __launch_bounds__(256) k_q4_galerkin(int cnx, int cny, const double* __restrict__ KE,
                                                     const double* __restrict__ E,
                                                     const uint8_t* __restrict__ mask,
                                                     const double* __restrict__ Kf,
                                                     double* __restrict__ Kc) {
  const int64_t cne = (int64_t)cnx * cny;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cne) return;
  const int cx = (int)(e % cnx), cy = (int)(e / cnx);
  const int fnx = 2 * cnx;
  const int64_t fne = cne * 4;
  double w[4];
  int64_t fe[4];
  uint8_t fm[9];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    fe[c] = (int64_t)(2 * cx + (c & 1)) + (int64_t)fnx * (2 * cy + (c >> 1));
    w[c] = FROM_FINE ? E[fe[c]] : 0.0;
  }
  if (FROM_FINE)
    for (int t = 0; t < 9; ++t)
      fm[t] = mask[(int64_t)(2 * cx + t % 3) + (int64_t)(fnx + 1) * (2 * cy + t / 3)];
  for (int I = 0; I < 8; ++I)
    for (int J = I; J < 8; ++J) {
      const int A = I >> 1, ci = I & 1, B = J >> 1, cj = J & 1;
      double acc = 0.0;
      for (int c = 0; c < 4; ++c) {
        const int dx = c & 1, dy = c >> 1;
        for (int a = 0; a < 4; ++a) {
          const double pa = phi1q(dx + (a & 1), A & 1) * phi1q(dy + (a >> 1), A >> 1);
          if (pa == 0.0) continue;
          if (FROM_FINE && ((fm[(dx + (a & 1)) + 3 * (dy + (a >> 1))] >> ci) & 1)) continue;
          for (int b = 0; b < 4; ++b) {
            const double pb = phi1q(dx + (b & 1), B & 1) * phi1q(dy + (b >> 1), B >> 1);
            if (pb == 0.0) continue;
            if (FROM_FINE && ((fm[(dx + (b & 1)) + 3 * (dy + (b >> 1))] >> cj) & 1)) continue;
            const int r = 2 * a + ci, q = 2 * b + cj;
            const double k = FROM_FINE ? w[c] * KE[r * 8 + q] : Kf[(int64_t)s2(r, q) * fne + fe[c]];
            acc = fma(pa * pb, k, acc);
          }
        }
      }
      Kc[(int64_t)s2(I, J) * cne + e] = acc;
    }
}

// y = sum_e L_e^T Ke_e L_e v for packed 8x8 element matrices; thread per node.
template <typename T>
__global__ void __launch_bounds__(256) k_q4_apply_elemmat(int nx, int ny, const double* __restrict__ Ke,
                                                          const T* __restrict__ v, T* __restrict__ y) {
  const int64_t nn = (int64_t)(nx + 1) * (ny + 1);
  const int64_t ne = (int64_t)nx * ny;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const int i = (int)(n % (nx + 1)), j = (int)(n / (nx + 1));
  T acc0 = 0, acc1 = 0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int ex = i - (a & 1), ey = j - (a >> 1);
    if (ex < 0 || ex >= nx || ey < 0 || ey >= ny) continue;
    const int64_t e = (int64_t)ex + (int64_t)nx * ey;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t nb = (int64_t)(ex + (b & 1)) + (int64_t)(nx + 1) * (ey + (b >> 1));
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        const T vb = v[d * nn + nb];
        acc0 = fma((T)Ke[(int64_t)s2(2 * a, 2 * b + d) * ne + e], vb, acc0);
        acc1 = fma((T)Ke[(int64_t)s2(2 * a + 1, 2 * b + d) * ne + e], vb, acc1);
      }
    }
  }
  y[n] = acc0;
  y[nn + n] = acc1;
}

__global__ void k_q4_diag_elemmat(int nx, int ny, const double* __restrict__ Ke,
                                  double* __restrict__ dinv) {
  const int64_t nn = (int64_t)(nx + 1) * (ny + 1);
  const int64_t ne = (int64_t)nx * ny;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const int i = (int)(n % (nx + 1)), j = (int)(n / (nx + 1));
  double d[2] = {0.0, 0.0};
  for (int a = 0; a < 4; ++a) {
    const int ex = i - (a & 1), ey = j - (a >> 1);
    if (ex < 0 || ex >= nx || ey < 0 || ey >= ny) continue;
    const int64_t e = (int64_t)ex + (int64_t)nx * ey;
    for (int c = 0; c < 2; ++c) d[c] += Ke[(int64_t)s2(2 * a + c, 2 * a + c) * ne + e];
  }
  for (int c = 0; c < 2; ++c) dinv[c * nn + n] = d[c] == 0.0 ? 1.0 : 1.0 / d[c];
}

// Grounded springs (one thread each; the host merges repeated DOFs, so no
// two threads touch one DOF).  y += k v on free spring DOFs.
__global__ void k_springs_add(SpringSet S, int64_t nn, const uint8_t* __restrict__ mask,
                              const double* __restrict__ v, double* __restrict__ y) {
  const int t = threadIdx.x;
  if (t >= S.n) return;
  const int64_t d = S.dof[t];
  const int64_t node = d % nn;
  if ((mask[node] >> (int)(d / nn)) & 1) return;
  y[d] = fma(S.k[t], v[d], y[d]);
}

// The inverse Jacobi diagonal with the spring stiffness added.
__global__ void k_springs_diag(SpringSet S, int64_t nn, const uint8_t* __restrict__ mask,
                               double* __restrict__ dinv) {
  const int t = threadIdx.x;
  if (t >= S.n) return;
  const int64_t d = S.dof[t];
  const int64_t node = d % nn;
  if ((mask[node] >> (int)(d / nn)) & 1) return;
  dinv[d] = 1.0 / (1.0 / dinv[d] + S.k[t]);
}

// (Df P)^T S (Df P) for the springs S of the fine grid, added to the level-1
// matrices: the fine DOF of a spring interpolates from the corners of one
// parent (any parent containing it), so k w w^T lands in that parent's
// matrix.  One thread walks the springs in order (two may share a parent).
__global__ void k_springs_galerkin(SpringSet S, int cnx, int cny, const uint8_t* __restrict__ mask,
                                   double* __restrict__ Kc) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int fnx = 2 * cnx;
  const int64_t fnn = (int64_t)(fnx + 1) * (2 * cny + 1);
  const int64_t cne = (int64_t)cnx * cny;
  for (int t = 0; t < S.n; ++t) {
    const int64_t d = S.dof[t];
    const int64_t node = d % fnn;
    const int c = (int)(d / fnn);
    if ((mask[node] >> c) & 1) continue;
    const int fi = (int)(node % (fnx + 1)), fj = (int)(node / (fnx + 1));
    const int px = min(fi >> 1, cnx - 1), py = min(fj >> 1, cny - 1);
    const int lx = fi - 2 * px, ly = fj - 2 * py;
    const int64_t e = (int64_t)px + (int64_t)cnx * py;
    for (int A = 0; A < 4; ++A) {
      const double wa = phi1q(lx, A & 1) * phi1q(ly, A >> 1);
      if (wa == 0.0) continue;
      for (int B = A; B < 4; ++B) {
        const double wb = phi1q(lx, B & 1) * phi1q(ly, B >> 1);
        if (wb == 0.0) continue;
        double& k = Kc[(int64_t)s2(2 * A + c, 2 * B + c) * cne + e];
        k = fma(S.k[t] * wa, wb, k);
      }
    }
  }
}

// Dense coarsest operator in SoA DOF order (c * nn + node); one wavefront
// per row, lanes over the columns: an entry sums, over the elements around
// the row's node in corner order a = 0..3, the entries coupling the two nodes.
__global__ void __launch_bounds__(256) k_q4_assemble_dense(int nx, int ny,
                                                           const double* __restrict__ Ke,
                                                           double* __restrict__ A) {
  const int64_t nn = (int64_t)(nx + 1) * (ny + 1);
  const int64_t ne = (int64_t)nx * ny;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= 2 * nn) return;  // wave-uniform
  const int c = (int)(row / nn);
  const int64_t n = row % nn;
  const int i = (int)(n % (nx + 1)), j = (int)(n / (nx + 1));
  double* Ar = A + row * 2 * nn;
  for (int64_t q = lane; q < 2 * nn; q += 64) {
    const int d = (int)(q / nn);
    const int64_t nb = q % nn;
    const int bi = (int)(nb % (nx + 1)), bj = (int)(nb / (nx + 1));
    double acc = 0.0;
    if (abs(bi - i) <= 1 && abs(bj - j) <= 1) {
      for (int a = 0; a < 4; ++a) {
        const int ex = i - (a & 1), ey = j - (a >> 1);
        if (ex < 0 || ex >= nx || ey < 0 || ey >= ny) continue;
        const int dx = bi - ex, dy = bj - ey;
        if (dx < 0 || dx > 1 || dy < 0 || dy > 1) continue;
        const int64_t e = (int64_t)ex + (int64_t)nx * ey;
        acc += Ke[(int64_t)s2(2 * a + c, 2 * (dx + 2 * dy) + d) * ne + e];
      }
    }
    if (q == row && acc == 0.0) acc = 1.0;  // dead coarse DOF: identity row
    Ar[q] = acc;
  }
}

}  // namespace

void launch_q4_apply(const Grid& g, const double* KE, const double* E, const uint8_t* mask,
                     const double* v, double* y, int mode, hipStream_t s) {
  k_q4_apply<<<nblk(g.nn, 256), 256, 0, s>>>(g.nx, g.ny, KE, E, mask, v, y, mode);
}

void launch_q4_energy(const Grid& g, const double* KE, const uint8_t* mask, const double* u,
                      const double* w, double* energy, hipStream_t s) {
  k_q4_energy<<<nblk(g.ne, 256), 256, 0, s>>>(g.nx, g.ny, KE, mask, u, w, energy);
}

void launch_springs_add(const SpringSet& S, const Grid& g, const uint8_t* mask, const double* v,
                        double* y, hipStream_t s) {
  if (S.n > 0) k_springs_add<<<1, 64, 0, s>>>(S, g.nn, mask, v, y);
}

void launch_springs_diag(const SpringSet& S, const Grid& g, const uint8_t* mask, double* dinv,
                         hipStream_t s) {
  if (S.n > 0) k_springs_diag<<<1, 64, 0, s>>>(S, g.nn, mask, dinv);
}

void launch_springs_galerkin(const SpringSet& S, const Grid& coarse, const uint8_t* mask,
                             double* Kc, hipStream_t s) {
  if (S.n > 0) k_springs_galerkin<<<1, 64, 0, s>>>(S, coarse.nx, coarse.ny, mask, Kc);
}

void launch_q4_diag(const Grid& g, const double* KE, const double* E, const uint8_t* mask,
                    double* dinv, hipStream_t s) {
  k_q4_diag<<<nblk(g.nn, 256), 256, 0, s>>>(g.nx, g.ny, KE, E, mask, dinv);
}

void launch_q4_galerkin_from_fine(const Grid& coarse, const double* KE, const double* E,
                                  const uint8_t* mask, double* Kc, hipStream_t s) {
  k_q4_galerkin<true><<<nblk(coarse.ne, 256), 256, 0, s>>>(coarse.nx, coarse.ny, KE, E, mask,
                                                           nullptr, Kc);
}

void launch_q4_galerkin_from_coarse(const Grid& coarse, const double* Kf, double* Kc,
                                    hipStream_t s) {
  k_q4_galerkin<false><<<nblk(coarse.ne, 256), 256, 0, s>>>(coarse.nx, coarse.ny, nullptr,
                                                            nullptr, nullptr, Kf, Kc);
}

void launch_q4_apply_elemmat(const Grid& g, const double* Ke, const double* v, double* y,
                             hipStream_t s) {
  k_q4_apply_elemmat<double><<<nblk(g.nn, 256), 256, 0, s>>>(g.nx, g.ny, Ke, v, y);
}

void launch_q4_diag_elemmat(const Grid& g, const double* Ke, double* dinv, hipStream_t s) {
  k_q4_diag_elemmat<<<nblk(g.nn, 256), 256, 0, s>>>(g.nx, g.ny, Ke, dinv);
}

void launch_q4_assemble_dense(const Grid& g, const double* Ke, double* A, hipStream_t s) {
  k_q4_assemble_dense<<<(unsigned)((2 * g.nn + 3) / 4), 256, 0, s>>>(g.nx, g.ny, Ke, A);
}

}  // namespace aarmr
