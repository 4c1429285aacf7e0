// Multigrid kernels of the V-cycle (Algorithm 2): Galerkin coarse operators
// P^T A P stored as one packed symmetric 24x24 matrix per coarse element, their products and
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

constexpr int kSym = kSymEntries;
__host__ __device__ constexpr int sidx(int r, int c) { return sym_index(r, c); }

// Level-1 Galerkin matrices, fast path: Kc = sum_c E_c M_c with
// M_c = P_c^T KE P_c precomputed (P_c the trilinear map from the parent's
// corners to child c's corners).  Exact for parents whose 27 fine nodes are
// all free; k_galerkin_lds then overwrites the parents that touch a fixed
// DOF.  Block: 64 parents (lanes) x 4 waves; wave w writes the packed
// entries w, w+4, ...
__global__ void __launch_bounds__(256) k_galerkin_fast(int cnx, int cny, int cnz,
                                                       const double* __restrict__ Mc,
                                                       const double* __restrict__ E,
                                                       double* __restrict__ Kc) {
  const int64_t cne = (int64_t)cnx * cny * cnz;
  const int64_t eid = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  const int wave = threadIdx.x >> 6;
  if (eid >= cne) return;
  const int cx = (int)(eid % cnx);
  const int64_t rest = eid / cnx;
  const int cy = (int)(rest % cny), cz = (int)(rest / cny);
  const int fnx = 2 * cnx, fny = 2 * cny;
  double w[8];
#pragma unroll
  for (int c = 0; c < 8; ++c)
    w[c] = E[(int64_t)(2 * cx + (c & 1)) +
             (int64_t)fnx * ((2 * cy + ((c >> 1) & 1)) + (int64_t)fny * (2 * cz + (c >> 2)))];
  for (int sx = wave; sx < kSym; sx += 4) {
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) acc = fma(w[c], Mc[c * kSym + sx], acc);
    Kc[(int64_t)sx * cne + eid] = acc;
  }
}

// Galerkin matrix of one parent per block: the 8 child matrices are staged
// in LDS, T_c = K_c P_c is formed by a column pass and sum_c P_c^T T_c by a
// row pass.  FROM_FINE: children are E_c Df KE Df with the fine fixed-DOF
// mask, and only parents touching a fixed DOF are written.  Otherwise the
// children are the previous level's packed matrices.
template <bool FROM_FINE>
__global__ void __launch_bounds__(256) k_galerkin_lds(int cnx, int cny, int cnz,
                                                      const double* __restrict__ KE,
                                                      const double* __restrict__ E,
                                                      const uint8_t* __restrict__ mask,
                                                      const double* __restrict__ Kf,
                                                      double* __restrict__ Kc) {
  __shared__ double sK[8][24][25];
  __shared__ uint8_t sm[27];
  __shared__ double sw[8];
  __shared__ int any_fixed;
  const int64_t cne = (int64_t)cnx * cny * cnz;
  const int64_t eid = blockIdx.x;
  const int cx = (int)(eid % cnx);
  const int64_t rest = eid / cnx;
  const int cy = (int)(rest % cny), cz = (int)(rest / cny);
  const int fnx = 2 * cnx, fny = 2 * cny;
  const int64_t fne = cne * 8;
  const int tid = threadIdx.x;
  if (FROM_FINE) {
    if (tid == 0) any_fixed = 0;
    __syncthreads();
    if (tid < 27) {
      const int px = tid % 3, py = (tid / 3) % 3, pz = tid / 9;
      sm[tid] = mask[node_of(fnx, fny, 2 * cx + px, 2 * cy + py, 2 * cz + pz)];
      if (sm[tid]) atomicOr(&any_fixed, 1);
    }
    if (tid < 8)
      sw[tid] = E[(int64_t)(2 * cx + (tid & 1)) +
                  (int64_t)fnx * ((2 * cy + ((tid >> 1) & 1)) + (int64_t)fny * (2 * cz + (tid >> 2)))];
    __syncthreads();
    if (!any_fixed) return;  // block-uniform: the fast path already wrote it
  }
  for (int t = tid; t < 8 * 576; t += 256) {
    const int c = t / 576, r = (t % 576) / 24, q = t % 24;
    const int dx = c & 1, dy = (c >> 1) & 1, dz = c >> 2;
    double v;
    if (FROM_FINE) {
      const int br = r / 3, bq = q / 3;
      const int pr = (dx + (br & 1)) + 3 * (dy + ((br >> 1) & 1)) + 9 * (dz + (br >> 2));
      const int pq = (dx + (bq & 1)) + 3 * (dy + ((bq >> 1) & 1)) + 9 * (dz + (bq >> 2));
      const bool fx = ((sm[pr] >> (r % 3)) & 1) || ((sm[pq] >> (q % 3)) & 1);
      v = fx ? 0.0 : sw[c] * KE[r * 24 + q];
    } else {
      const int64_t fe = (int64_t)(2 * cx + dx) + (int64_t)fnx * ((2 * cy + dy) + (int64_t)fny * (2 * cz + dz));
      v = Kf[(int64_t)sidx(r, q) * fne + fe];
    }
    sK[c][r][q] = v;
  }
  __syncthreads();
  // column pass: T_c[r][3B+j] = sum_b P_c[b][B] K_c[r][3b+j]
  double tv[18];
#pragma unroll
  for (int u = 0; u < 18; ++u) {
    const int t = tid + 256 * u;
    const int c = t / 576, r = (t % 576) / 24, J = t % 24;
    const int B = J / 3, j = J % 3;
    const int dx = c & 1, dy = (c >> 1) & 1, dz = c >> 2;
    double acc = 0.0;
    for (int b = 0; b < 8; ++b) {
      const double pb = phi1(dx + (b & 1), B & 1) * phi1(dy + ((b >> 1) & 1), (B >> 1) & 1) *
                        phi1(dz + (b >> 2), B >> 2);
      acc = fma(pb, sK[c][r][3 * b + j], acc);
    }
    tv[u] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 18; ++u) {
    const int t = tid + 256 * u;
    sK[t / 576][(t % 576) / 24][t % 24] = tv[u];
  }
  __syncthreads();
  // row pass over packed entries (I <= J): sum_c sum_b P_c[b][A] T_c[3b+i][J]
  for (int sx = tid; sx < kSym; sx += 256) {
    int I = 0;
    while (sidx(I, 23) < sx) ++I;  // row of packed entry sx
    const int J = I + (sx - sidx(I, I));
    const int A = I / 3, i = I % 3;
    double acc = 0.0;
    for (int c = 0; c < 8; ++c) {
      const int dx = c & 1, dy = (c >> 1) & 1, dz = c >> 2;
      for (int b = 0; b < 8; ++b) {
        const double pa = phi1(dx + (b & 1), A & 1) * phi1(dy + ((b >> 1) & 1), (A >> 1) & 1) *
                          phi1(dz + (b >> 2), A >> 2);
        acc = fma(pa, sK[c][3 * b + i][J], acc);
      }
    }
    Kc[(int64_t)sx * cne + eid] = acc;
  }
}

// y = sum_e L_e^T Ke_e L_e v for packed element matrices; thread per node.
template <typename T>
__global__ void __launch_bounds__(256) k_apply_elemmat(int nx, int ny, int nz,
                                                       const T* __restrict__ Ke,
                                                       const T* __restrict__ v,
                                                       T* __restrict__ y) {
  const int64_t nn = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  const int64_t ne = (int64_t)nx * ny * nz;
  int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const int i = (int)(n % (nx + 1));
  const int64_t rest = n / (nx + 1);
  const int j = (int)(rest % (ny + 1));
  const int k = (int)(rest / (ny + 1));
  T acc0 = 0, acc1 = 0, acc2 = 0;
#pragma unroll
  for (int a = 0; a < 8; ++a) {  // the node is local corner a of element (i,j,k) - offset(a)
    const int ex = i - (a & 1), ey = j - ((a >> 1) & 1), ez = k - (a >> 2);
    if (ex < 0 || ex >= nx || ey < 0 || ey >= ny || ez < 0 || ez >= nz) continue;
    const int64_t e = (int64_t)ex + (int64_t)nx * ((int64_t)ey + (int64_t)ny * ez);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int64_t nb = node_of(nx, ny, ex + (b & 1), ey + ((b >> 1) & 1), ez + (b >> 2));
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T vb = v[c * nn + nb];
        acc0 = fma(Ke[(int64_t)sidx(3 * a + 0, 3 * b + c) * ne + e], vb, acc0);
        acc1 = fma(Ke[(int64_t)sidx(3 * a + 1, 3 * b + c) * ne + e], vb, acc1);
        acc2 = fma(Ke[(int64_t)sidx(3 * a + 2, 3 * b + c) * ne + e], vb, acc2);
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
  const int64_t ne = (int64_t)nx * ny * nz;
  int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const int i = (int)(n % (nx + 1));
  const int64_t rest = n / (nx + 1);
  const int j = (int)(rest % (ny + 1));
  const int k = (int)(rest / (ny + 1));
  double d[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int ex = i - (a & 1), ey = j - ((a >> 1) & 1), ez = k - (a >> 2);
    if (ex < 0 || ex >= nx || ey < 0 || ey >= ny || ez < 0 || ez >= nz) continue;
    const int64_t e = (int64_t)ex + (int64_t)nx * ((int64_t)ey + (int64_t)ny * ez);
#pragma unroll
    for (int c = 0; c < 3; ++c) d[c] += Ke[(int64_t)sidx(3 * a + c, 3 * a + c) * ne + e];
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
  const int64_t ne = (int64_t)nx * ny * nz;
  const int64_t nd = 3 * nn;
  int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= nd) return;
  const int c = (int)(row / nn);
  const int64_t n = row % nn;
  double* Ar = A + row * nd;
  for (int64_t t = 0; t < nd; ++t) Ar[t] = 0.0;
  const int i = (int)(n % (nx + 1));
  const int64_t rest = n / (nx + 1);
  const int j = (int)(rest % (ny + 1));
  const int k = (int)(rest / (ny + 1));
  for (int a = 0; a < 8; ++a) {
    const int ex = i - (a & 1), ey = j - ((a >> 1) & 1), ez = k - (a >> 2);
    if (ex < 0 || ex >= nx || ey < 0 || ey >= ny || ez < 0 || ez >= nz) continue;
    const int64_t e = (int64_t)ex + (int64_t)nx * ((int64_t)ey + (int64_t)ny * ez);
    for (int b = 0; b < 8; ++b) {
      const int64_t nb = node_of(nx, ny, ex + (b & 1), ey + ((b >> 1) & 1), ez + (b >> 2));
      for (int cc = 0; cc < 3; ++cc) Ar[cc * nn + nb] += Ke[(int64_t)sidx(3 * a + c, 3 * b + cc) * ne + e];
    }
  }
  if (Ar[row] == 0.0) Ar[row] = 1.0;  // dead coarse DOF: identity row
}

// ---- blocked Gauss-Jordan inversion of an SPD matrix (sweep operator) -----
// One block step with pivot block K = [k0, k0+kb):
//   P = A_KK^-1, T = A_:K P, A_IJ -= T_I A_KJ (I, J outside K),
//   A_KJ = P A_KJ, A_IK = -T_I, A_KK = P.

// Invert the kb x kb pivot block (unblocked Gauss-Jordan) in one wavefront:
// lane c holds column c in registers; the pivot column is broadcast with
// readlane.  Rows/columns beyond kb are padded with the identity.
__device__ inline double lane_bcast(double x, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}

__global__ void __launch_bounds__(64) k_gj_pivot(int n, int k0, int kb,
                                                 const double* __restrict__ A,
                                                 double* __restrict__ P) {
  const int c = threadIdx.x;
  double col[kGJBlock];
#pragma unroll
  for (int r = 0; r < kGJBlock; ++r)
    col[r] = (r < kb && c < kb) ? A[(int64_t)(k0 + r) * n + (k0 + c)] : (r == c ? 1.0 : 0.0);
  // the step index k is a runtime value; col[] is only ever indexed by the
  // unrolled r, so it stays in registers (row k is picked out by selects)
  for (int k = 0; k < kGJBlock; ++k) {
    double rk = 0.0;
#pragma unroll
    for (int r = 0; r < kGJBlock; ++r) rk = (r == k) ? col[r] : rk;
    const double piv = 1.0 / lane_bcast(rk, k);
    const bool pc = (c == k);
#pragma unroll
    for (int r = 0; r < kGJBlock; ++r) {
      const double crk = lane_bcast(col[r], k);
      const double upd = pc ? -crk * piv : fma(-crk * piv, rk, col[r]);
      const double kr = pc ? piv : rk * piv;
      col[r] = (r == k) ? kr : upd;
    }
  }
#pragma unroll
  for (int r = 0; r < kGJBlock; ++r)
    if (r < kb && c < kb) P[r * kb + c] = col[r];
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

// A_IJ -= T_I Rw_J for I, J outside the pivot block: 64x64 output tiles, each
// of the 256 threads accumulates a 4x4 sub-tile; the rank-kb product is
// staged through LDS in chunks of 16.
__global__ void __launch_bounds__(256) k_gj_update(int n, int k0, int kb,
                                                   double* __restrict__ A,
                                                   const double* __restrict__ T,
                                                   const double* __restrict__ Rw) {
  __shared__ double sT[16][64 + 1];
  __shared__ double sR[16][64 + 1];
  const int bi = blockIdx.y * 64, bj = blockIdx.x * 64;
  const int tid = threadIdx.x;
  const int tr = tid / 16, tc = tid % 16;
  double acc[4][4] = {};
  for (int p0 = 0; p0 < kb; p0 += 16) {
    for (int t = tid; t < 16 * 64; t += 256) {
      const int q = t / 64, rr = t % 64;
      const int p = p0 + q;
      const int i = bi + rr, j = bj + rr;
      sT[q][rr] = (p < kb && i < n) ? T[(int64_t)i * kb + p] : 0.0;
      sR[q][rr] = (p < kb && j < n) ? Rw[(int64_t)p * n + j] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = sT[q][tr + 16 * u];
#pragma unroll
      for (int w = 0; w < 4; ++w) b[w] = sR[q][tc + 16 * w];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int w = 0; w < 4; ++w) acc[u][w] = fma(a[u], b[w], acc[u][w]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = bi + tr + 16 * u;
    if (i >= n || (i >= k0 && i < k0 + kb)) continue;
#pragma unroll
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

void launch_galerkin_from_fine(const Grid& coarse, const double* KE, const double* Mc,
                               const double* E, const uint8_t* mask, double* Kc, hipStream_t s) {
  k_galerkin_fast<<<nblk(coarse.ne, 64), 256, 0, s>>>(coarse.nx, coarse.ny, coarse.nz, Mc, E, Kc);
  k_galerkin_lds<true><<<(unsigned)coarse.ne, 256, 0, s>>>(coarse.nx, coarse.ny, coarse.nz, KE, E,
                                                          mask, nullptr, Kc);
}

void launch_galerkin_from_coarse(const Grid& coarse, const double* Kf, double* Kc, hipStream_t s) {
  k_galerkin_lds<false><<<(unsigned)coarse.ne, 256, 0, s>>>(coarse.nx, coarse.ny, coarse.nz,
                                                           nullptr, nullptr, nullptr, Kf, Kc);
}

void launch_apply_elemmat(const Grid& g, const double* Ke, const double* v, double* y,
                          hipStream_t s) {
  k_apply_elemmat<double><<<nblk(g.nn, 256), 256, 0, s>>>(g.nx, g.ny, g.nz, Ke, v, y);
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
    k_gj_pivot<<<1, 64, 0, s>>>(n, k0, kb, A, P);
    const int64_t nk = (int64_t)n * kb;
    k_gj_panels<<<nblk(nk, 256), 256, 0, s>>>(n, k0, kb, A, P, T, Rw);
    dim3 grid((n + 63) / 64, (n + 63) / 64);
    k_gj_update<<<grid, 256, 0, s>>>(n, k0, kb, A, T, Rw);
    k_gj_finish<<<nblk(nk, 256), 256, 0, s>>>(n, k0, kb, A, P, T, Rw);
  }
}

void launch_gemv(int n, const double* A, const double* x, double* y, hipStream_t s) {
  k_gemv<double, double><<<nblk(n, 4), 256, 0, s>>>(n, A, x, y);
}

}  // namespace aarmr
