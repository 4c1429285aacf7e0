// Multigrid kernels of the V-cycle (Algorithm 2): Galerkin coarse operators
// P^T A P stored as one 24x24 matrix per coarse element, their products and
// diagonals, restriction P^T and interpolation P (trilinear, 2:1 per axis),
// damped-Jacobi smoothing, and the exact coarsest solve through an explicit
// inverse computed by blocked Gauss-Jordan elimination.
#include "internal.hpp"

namespace aarmr {

namespace {

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

__device__ inline int64_t node_of(int nx, int ny, int i, int j, int k) {
  return (int64_t)i + (int64_t)(nx + 1) * ((int64_t)j + (int64_t)(ny + 1) * k);
}

// Weight of parent corner A (0/1) at position pos (0,1,2) inside the parent
// along one axis: trilinear interpolation at the 2:1 refined nodes.
__device__ inline double phi1(int pos, int A) {
  return pos == 1 ? 0.5 : ((pos >> 1) == A ? 1.0 : 0.0);
}

// Kc(E) = sum over the 8 children c of P_c^T Kchild_c P_c, where P_c maps the
// parent's 8 corners to child c's 8 corners.  Children are fine elements
// (from_fine: Kchild = E_c Df KE Df with the fine fixed-DOF mask) or coarse
// element matrices of the previous level.  One block per coarse element.
template <bool FROM_FINE>
__global__ void __launch_bounds__(256) k_galerkin(int cnx, int cny, int cnz,
                                                  const double* __restrict__ KE,
                                                  const double* __restrict__ E,
                                                  const uint8_t* __restrict__ mask,
                                                  const double* __restrict__ Kf,
                                                  double* __restrict__ Kc) {
  __shared__ double sK[FROM_FINE ? 576 : 8 * 576];
  __shared__ double sw[8];
  __shared__ uint8_t sm[27];
  const int64_t E_id = blockIdx.x;
  const int cx = (int)(E_id % cnx);
  const int64_t rest = E_id / cnx;
  const int cy = (int)(rest % cny);
  const int cz = (int)(rest / cny);
  const int fnx = 2 * cnx, fny = 2 * cny;
  const int tid = threadIdx.x;
  if (FROM_FINE) {
    for (int t = tid; t < 576; t += 256) sK[t] = KE[t];
    if (tid < 8) {
      int dx = tid & 1, dy = (tid >> 1) & 1, dz = tid >> 2;
      int64_t fe = (int64_t)(2 * cx + dx) + (int64_t)fnx * ((2 * cy + dy) + (int64_t)fny * (2 * cz + dz));
      sw[tid] = E[fe];
    }
    if (tid < 27) {
      int px = tid % 3, py = (tid / 3) % 3, pz = tid / 9;
      sm[tid] = mask[node_of(fnx, fny, 2 * cx + px, 2 * cy + py, 2 * cz + pz)];
    }
  } else {
    for (int t = tid; t < 8 * 576; t += 256) {
      int c = t / 576, o = t % 576;
      int dx = c & 1, dy = (c >> 1) & 1, dz = c >> 2;
      int64_t fe = (int64_t)(2 * cx + dx) + (int64_t)fnx * ((2 * cy + dy) + (int64_t)fny * (2 * cz + dz));
      sK[t] = Kf[fe * 576 + o];
    }
  }
  __syncthreads();
  for (int idx = tid; idx < 576; idx += 256) {
    const int I = idx / 24, J = idx % 24;
    const int A = I / 3, i = I % 3, B = J / 3, j = J % 3;
    const int Ax = A & 1, Ay = (A >> 1) & 1, Az = A >> 2;
    const int Bx = B & 1, By = (B >> 1) & 1, Bz = B >> 2;
    double acc = 0.0;
    for (int c = 0; c < 8; ++c) {
      const int dx = c & 1, dy = (c >> 1) & 1, dz = c >> 2;
      for (int b = 0; b < 8; ++b) {
        const int px = dx + (b & 1), py = dy + ((b >> 1) & 1), pz = dz + (b >> 2);
        const double pa = phi1(px, Ax) * phi1(py, Ay) * phi1(pz, Az);
        if (pa == 0.0) continue;
        if (FROM_FINE && ((sm[px + 3 * py + 9 * pz] >> i) & 1)) continue;
        double inner = 0.0;
        for (int b2 = 0; b2 < 8; ++b2) {
          const int qx = dx + (b2 & 1), qy = dy + ((b2 >> 1) & 1), qz = dz + (b2 >> 2);
          const double pb = phi1(qx, Bx) * phi1(qy, By) * phi1(qz, Bz);
          if (pb == 0.0) continue;
          if (FROM_FINE && ((sm[qx + 3 * qy + 9 * qz] >> j) & 1)) continue;
          const double kv = FROM_FINE ? sK[(3 * b + i) * 24 + 3 * b2 + j]
                                      : sK[c * 576 + (3 * b + i) * 24 + 3 * b2 + j];
          inner = fma(pb, kv, inner);
        }
        acc = fma(pa * (FROM_FINE ? sw[c] : 1.0), inner, acc);
      }
    }
    Kc[E_id * 576 + idx] = acc;
  }
}

// y = sum_e L_e^T Ke_e L_e v for per-element matrices; thread per node.
__global__ void __launch_bounds__(256) k_apply_elemmat(int nx, int ny, int nz,
                                                       const double* __restrict__ Ke,
                                                       const double* __restrict__ v,
                                                       double* __restrict__ y) {
  const int64_t nn = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  int i = (int)(n % (nx + 1));
  int64_t rest = n / (nx + 1);
  int j = (int)(rest % (ny + 1));
  int k = (int)(rest / (ny + 1));
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
  for (int ez = k - 1; ez <= k; ++ez) {
    if (ez < 0 || ez >= nz) continue;
    for (int ey = j - 1; ey <= j; ++ey) {
      if (ey < 0 || ey >= ny) continue;
      for (int ex = i - 1; ex <= i; ++ex) {
        if (ex < 0 || ex >= nx) continue;
        const int a = (i - ex) + 2 * (j - ey) + 4 * (k - ez);
        const int64_t e = (int64_t)ex + (int64_t)nx * ((int64_t)ey + (int64_t)ny * ez);
        const double* row = Ke + e * 576 + (3 * a) * 24;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          const int64_t nb = node_of(nx, ny, ex + (b & 1), ey + ((b >> 1) & 1), ez + (b >> 2));
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const double vb = v[c * nn + nb];
            acc0 = fma(row[3 * b + c], vb, acc0);
            acc1 = fma(row[24 + 3 * b + c], vb, acc1);
            acc2 = fma(row[48 + 3 * b + c], vb, acc2);
          }
        }
      }
    }
  }
  y[n] = acc0;
  y[nn + n] = acc1;
  y[2 * nn + n] = acc2;
}

__global__ void k_diag_elemmat(int nx, int ny, int nz, const double* __restrict__ Ke,
                               double* __restrict__ dinv, float* __restrict__ dinv32) {
  const int64_t nn = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  int i = (int)(n % (nx + 1));
  int64_t rest = n / (nx + 1);
  int j = (int)(rest % (ny + 1));
  int k = (int)(rest / (ny + 1));
  double d[3] = {0.0, 0.0, 0.0};
  for (int ez = k - 1; ez <= k; ++ez) {
    if (ez < 0 || ez >= nz) continue;
    for (int ey = j - 1; ey <= j; ++ey) {
      if (ey < 0 || ey >= ny) continue;
      for (int ex = i - 1; ex <= i; ++ex) {
        if (ex < 0 || ex >= nx) continue;
        const int a = (i - ex) + 2 * (j - ey) + 4 * (k - ez);
        const int64_t e = (int64_t)ex + (int64_t)nx * ((int64_t)ey + (int64_t)ny * ez);
        for (int c = 0; c < 3; ++c) d[c] += Ke[e * 576 + (3 * a + c) * 25];
      }
    }
  }
  for (int c = 0; c < 3; ++c) {
    double di = d[c] == 0.0 ? 1.0 : 1.0 / d[c];  // dead coarse DOF: identity row
    dinv[c * nn + n] = di;
    if (dinv32) dinv32[c * nn + n] = (float)di;
  }
}

// bc = P^T Df (bf - tf): thread per coarse node, 27-point gather with
// weights (1/2, 1, 1/2) per axis.  mask == nullptr: no fine fixed DOFs.
template <typename T>
__global__ void k_restrict(int cnx, int cny, int cnz, const T* __restrict__ bf,
                           const T* __restrict__ tf, const uint8_t* __restrict__ mask,
                           T* __restrict__ bc) {
  const int64_t cnn = (int64_t)(cnx + 1) * (cny + 1) * (cnz + 1);
  int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= cnn) return;
  const int fnx = 2 * cnx, fny = 2 * cny, fnz = 2 * cnz;
  const int64_t fnn = (int64_t)(fnx + 1) * (fny + 1) * (fnz + 1);
  int I = (int)(n % (cnx + 1));
  int64_t rest = n / (cnx + 1);
  int J = (int)(rest % (cny + 1));
  int K = (int)(rest / (cny + 1));
  T acc[3] = {0, 0, 0};
  for (int dz = -1; dz <= 1; ++dz) {
    int fk = 2 * K + dz;
    if (fk < 0 || fk > fnz) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      int fj = 2 * J + dy;
      if (fj < 0 || fj > fny) continue;
      for (int dx = -1; dx <= 1; ++dx) {
        int fi = 2 * I + dx;
        if (fi < 0 || fi > fnx) continue;
        const T w = (dx ? T(0.5) : T(1)) * (dy ? T(0.5) : T(1)) * (dz ? T(0.5) : T(1));
        const int64_t fnode = node_of(fnx, fny, fi, fj, fk);
        const uint8_t m = mask ? mask[fnode] : 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if ((m >> c) & 1) continue;
          acc[c] += w * (bf[c * fnn + fnode] - tf[c * fnn + fnode]);
        }
      }
    }
  }
  bc[n] = acc[0];
  bc[cnn + n] = acc[1];
  bc[2 * cnn + n] = acc[2];
}

// xf += Df P xc: thread per fine node.
template <typename T>
__global__ void k_prolong_add(int fnx, int fny, int fnz, const T* __restrict__ xc,
                              const uint8_t* __restrict__ mask, T* __restrict__ xf) {
  const int64_t fnn = (int64_t)(fnx + 1) * (fny + 1) * (fnz + 1);
  int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= fnn) return;
  const int cnx = fnx / 2, cny = fny / 2, cnz = fnz / 2;
  const int64_t cnn = (int64_t)(cnx + 1) * (cny + 1) * (cnz + 1);
  int fi = (int)(n % (fnx + 1));
  int64_t rest = n / (fnx + 1);
  int fj = (int)(rest % (fny + 1));
  int fk = (int)(rest / (fny + 1));
  const uint8_t m = mask ? mask[n] : 0;
  int ix0 = fi >> 1, ix1 = (fi + 1) >> 1;
  int iy0 = fj >> 1, iy1 = (fj + 1) >> 1;
  int iz0 = fk >> 1, iz1 = (fk + 1) >> 1;
  const T wx = (fi & 1) ? T(0.5) : T(1), wy = (fj & 1) ? T(0.5) : T(1), wz = (fk & 1) ? T(0.5) : T(1);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if ((m >> c) & 1) continue;
    const T* x = xc + c * cnn;
    T s;
    if (!(fi & 1) && !(fj & 1) && !(fk & 1)) {
      s = x[node_of(cnx, cny, ix0, iy0, iz0)];
    } else {
      s = 0;
      for (int z = 0; z < ((fk & 1) ? 2 : 1); ++z)
        for (int y = 0; y < ((fj & 1) ? 2 : 1); ++y)
          for (int xx = 0; xx < ((fi & 1) ? 2 : 1); ++xx)
            s += x[node_of(cnx, cny, xx ? ix1 : ix0, y ? iy1 : iy0, z ? iz1 : iz0)];
      s *= wx * wy * wz;
    }
    xf[c * fnn + n] += s;
  }
}

template <typename T>
__global__ void k_jacobi_first(int64_t n3, const T* __restrict__ b, const T* __restrict__ dinv,
                               T omega, T* __restrict__ x) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n3) x[i] = omega * dinv[i] * b[i];
}

template <typename T>
__global__ void k_jacobi_update(int64_t n3, const T* __restrict__ b, const T* __restrict__ t,
                                const T* __restrict__ dinv, T omega, T* __restrict__ x) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n3) x[i] += omega * dinv[i] * (b[i] - t[i]);
}

// Dense coarsest operator in SoA DOF order (c * nn + node); thread per row.
__global__ void k_assemble_dense(int nx, int ny, int nz, const double* __restrict__ Ke,
                                 double* __restrict__ A) {
  const int64_t nn = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  const int64_t nd = 3 * nn;
  int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= nd) return;
  const int c = (int)(row / nn);
  const int64_t n = row % nn;
  double* Ar = A + row * nd;
  for (int64_t t = 0; t < nd; ++t) Ar[t] = 0.0;
  int i = (int)(n % (nx + 1));
  int64_t rest = n / (nx + 1);
  int j = (int)(rest % (ny + 1));
  int k = (int)(rest / (ny + 1));
  for (int ez = k - 1; ez <= k; ++ez) {
    if (ez < 0 || ez >= nz) continue;
    for (int ey = j - 1; ey <= j; ++ey) {
      if (ey < 0 || ey >= ny) continue;
      for (int ex = i - 1; ex <= i; ++ex) {
        if (ex < 0 || ex >= nx) continue;
        const int a = (i - ex) + 2 * (j - ey) + 4 * (k - ez);
        const int64_t e = (int64_t)ex + (int64_t)nx * ((int64_t)ey + (int64_t)ny * ez);
        const double* r = Ke + e * 576 + (3 * a + c) * 24;
        for (int b = 0; b < 8; ++b) {
          const int64_t nb = node_of(nx, ny, ex + (b & 1), ey + ((b >> 1) & 1), ez + (b >> 2));
          for (int cc = 0; cc < 3; ++cc) Ar[cc * nn + nb] += r[3 * b + cc];
        }
      }
    }
  }
  if (Ar[row] == 0.0) Ar[row] = 1.0;  // dead coarse DOF: identity row
}

// ---- blocked Gauss-Jordan inversion of an SPD matrix (sweep operator) -----
// One block step with pivot block K = [k0, k0+kb):
//   P = A_KK^-1, T = A_:K P, A_IJ -= T_I A_KJ (I, J outside K),
//   A_KJ = P A_KJ, A_IK = -T_I, A_KK = P.

// Invert the kb x kb pivot block in LDS (unblocked Gauss-Jordan).
__global__ void __launch_bounds__(256) k_gj_pivot(int n, int k0, int kb,
                                                  const double* __restrict__ A,
                                                  double* __restrict__ P) {
  __shared__ double s[kGJBlock * kGJBlock];
  __shared__ double rowk[kGJBlock], colk[kGJBlock];
  const int tid = threadIdx.x;
  for (int t = tid; t < kb * kb; t += 256) {
    int r = t / kb, c = t % kb;
    s[t] = A[(int64_t)(k0 + r) * n + (k0 + c)];
  }
  __syncthreads();
  for (int k = 0; k < kb; ++k) {
    if (tid < kb) {
      rowk[tid] = s[k * kb + tid];
      colk[tid] = s[tid * kb + k];
    }
    __syncthreads();
    const double piv = 1.0 / colk[k];
    for (int t = tid; t < kb * kb; t += 256) {
      int r = t / kb, c = t % kb;
      if (r == k && c == k) s[t] = piv;
      else if (r == k) s[t] = rowk[c] * piv;
      else if (c == k) s[t] = -colk[r] * piv;
      else s[t] -= colk[r] * rowk[c] * piv;
    }
    __syncthreads();
  }
  for (int t = tid; t < kb * kb; t += 256) P[t] = s[t];
}

// T[i][p] = sum_q A[i][k0+q] P[q][p] (all rows i); Rw[p][j] = A[k0+p][j].
__global__ void k_gj_panels(int n, int k0, int kb, const double* __restrict__ A,
                            const double* __restrict__ P, double* __restrict__ T,
                            double* __restrict__ Rw) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * kb) return;
  const int i = (int)(t / kb), p = (int)(t % kb);
  double acc = 0.0;
  for (int q = 0; q < kb; ++q) acc = fma(A[(int64_t)i * n + k0 + q], P[q * kb + p], acc);
  T[t] = acc;
  const int pr = (int)(t / n), j = (int)(t % n);
  Rw[t] = A[(int64_t)(k0 + pr) * n + j];
}

// A_IJ -= T_I Rw_J for I, J outside the pivot block (32x64 LDS tiles; each
// of the 256 threads computes 2 rows x 4 columns).
__global__ void __launch_bounds__(256) k_gj_update(int n, int k0, int kb,
                                                   double* __restrict__ A,
                                                   const double* __restrict__ T,
                                                   const double* __restrict__ Rw) {
  __shared__ double sT[32][kGJBlock + 1];
  __shared__ double sR[kGJBlock][64 + 1];
  const int bi = blockIdx.y * 32, bj = blockIdx.x * 64;
  const int tid = threadIdx.x;
  for (int t = tid; t < 32 * kb; t += 256) {
    int r = t / kb, p = t % kb;
    int i = bi + r;
    sT[r][p] = (i < n) ? T[(int64_t)i * kb + p] : 0.0;
  }
  for (int t = tid; t < kb * 64; t += 256) {
    int p = t / 64, c = t % 64;
    int j = bj + c;
    sR[p][c] = (j < n) ? Rw[(int64_t)p * n + j] : 0.0;
  }
  __syncthreads();
  const int tr = tid / 16, tc = tid % 16;
  double acc[2][4] = {};
  for (int p = 0; p < kb; ++p) {
    double a[2], b[4];
    for (int u = 0; u < 2; ++u) a[u] = sT[tr * 2 + u][p];
    for (int w = 0; w < 4; ++w) b[w] = sR[p][tc + 16 * w];
    for (int u = 0; u < 2; ++u)
      for (int w = 0; w < 4; ++w) acc[u][w] = fma(a[u], b[w], acc[u][w]);
  }
  for (int u = 0; u < 2; ++u) {
    const int i = bi + tr * 2 + u;
    if (i >= n || (i >= k0 && i < k0 + kb)) continue;
    for (int w = 0; w < 4; ++w) {
      const int j = bj + tc + 16 * w;
      if (j >= n || (j >= k0 && j < k0 + kb)) continue;
      A[(int64_t)i * n + j] -= acc[u][w];
    }
  }
}

// A_KJ = P Rw_J, A_IK = -T_I, A_KK = P.
__global__ void k_gj_finish(int n, int k0, int kb, double* __restrict__ A,
                            const double* __restrict__ P, const double* __restrict__ T,
                            const double* __restrict__ Rw) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * kb) return;
  {  // row panel entry (p, j)
    const int p = (int)(t / n), j = (int)(t % n);
    if (j >= k0 && j < k0 + kb) {
      A[(int64_t)(k0 + p) * n + j] = P[p * kb + (j - k0)];
    } else {
      double acc = 0.0;
      for (int q = 0; q < kb; ++q) acc = fma(P[p * kb + q], Rw[(int64_t)q * n + j], acc);
      A[(int64_t)(k0 + p) * n + j] = acc;
    }
  }
  {  // column panel entry (i, p)
    const int i = (int)(t / kb), p = (int)(t % kb);
    if (!(i >= k0 && i < k0 + kb)) A[(int64_t)i * n + k0 + p] = -T[t];
  }
}

// y = A x for the dense (symmetric) inverse; one wavefront per row.
template <typename TX, typename TY>
__global__ void __launch_bounds__(256) k_gemv(int n, const double* __restrict__ A,
                                              const TX* __restrict__ x, TY* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const double* a = A + (int64_t)row * n;
  double acc = 0.0;
  for (int j = lane; j < n; j += 64) acc = fma(a[j], (double)x[j], acc);
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) y[row] = (TY)acc;
}

}  // namespace

void launch_galerkin_from_fine(const Grid& coarse, const double* KE, const double* E,
                               const uint8_t* mask, double* Kc, hipStream_t s) {
  k_galerkin<true><<<(unsigned)coarse.ne, 256, 0, s>>>(coarse.nx, coarse.ny, coarse.nz, KE, E,
                                                       mask, nullptr, Kc);
}

void launch_galerkin_from_coarse(const Grid& coarse, const double* Kf, double* Kc, hipStream_t s) {
  k_galerkin<false><<<(unsigned)coarse.ne, 256, 0, s>>>(coarse.nx, coarse.ny, coarse.nz, nullptr,
                                                        nullptr, nullptr, Kf, Kc);
}

void launch_apply_elemmat(const Grid& g, const double* Ke, const double* v, double* y,
                          hipStream_t s) {
  k_apply_elemmat<<<nblk(g.nn, 256), 256, 0, s>>>(g.nx, g.ny, g.nz, Ke, v, y);
}

void launch_diag_elemmat(const Grid& g, const double* Ke, double* dinv, float* dinv32,
                         hipStream_t s) {
  k_diag_elemmat<<<nblk(g.nn, 256), 256, 0, s>>>(g.nx, g.ny, g.nz, Ke, dinv, dinv32);
}

void launch_restrict(const Grid& coarse, const double* bf, const double* tf, const uint8_t* mask,
                     double* bc, hipStream_t s) {
  k_restrict<double><<<nblk(coarse.nn, 256), 256, 0, s>>>(coarse.nx, coarse.ny, coarse.nz, bf, tf,
                                                          mask, bc);
}

void launch_prolong_add(const Grid& fine, const double* xc, const uint8_t* mask, double* xf,
                        hipStream_t s) {
  k_prolong_add<double><<<nblk(fine.nn, 256), 256, 0, s>>>(fine.nx, fine.ny, fine.nz, xc, mask,
                                                           xf);
}

void launch_jacobi_first(int64_t n3, const double* b, const double* dinv, double omega, double* x,
                         hipStream_t s) {
  k_jacobi_first<double><<<nblk(n3, 256), 256, 0, s>>>(n3, b, dinv, omega, x);
}

void launch_jacobi_update(int64_t n3, const double* b, const double* t, const double* dinv,
                          double omega, double* x, hipStream_t s) {
  k_jacobi_update<double><<<nblk(n3, 256), 256, 0, s>>>(n3, b, t, dinv, omega, x);
}

void launch_assemble_dense(const Grid& g, const double* Ke, double* A, hipStream_t s) {
  k_assemble_dense<<<nblk(3 * g.nn, 64), 64, 0, s>>>(g.nx, g.ny, g.nz, Ke, A);
}

void launch_gj_invert(int n, double* A, double* P, double* T, double* Rw, hipStream_t s) {
  for (int k0 = 0; k0 < n; k0 += kGJBlock) {
    const int kb = (n - k0 < kGJBlock) ? (n - k0) : kGJBlock;
    k_gj_pivot<<<1, 256, 0, s>>>(n, k0, kb, A, P);
    const int64_t nk = (int64_t)n * kb;
    k_gj_panels<<<nblk(nk, 256), 256, 0, s>>>(n, k0, kb, A, P, T, Rw);
    dim3 grid((n + 63) / 64, (n + 31) / 32);
    k_gj_update<<<grid, 256, 0, s>>>(n, k0, kb, A, T, Rw);
    k_gj_finish<<<nblk(nk, 256), 256, 0, s>>>(n, k0, kb, A, P, T, Rw);
  }
}

void launch_gemv(int n, const double* A, const double* x, double* y, hipStream_t s) {
  k_gemv<double, double><<<nblk(n, 4), 256, 0, s>>>(n, A, x, y);
}

}  // namespace aarmr
