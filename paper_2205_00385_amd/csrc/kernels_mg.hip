// Multigrid kernels of the V-cycle (Algorithm 2): Galerkin coarse operators
// P^T A P stored as one packed symmetric 24x24 matrix per coarse element, their products and
// diagonals, restriction P^T and interpolation P (trilinear, 2:1 per axis),
// damped-Jacobi smoothing, and the exact coarsest solve through an explicit
// inverse computed by blocked Gauss-Jordan elimination.
#include <algorithm>

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
typedef double f64x4 __attribute__((ext_vector_type(4)));
__host__ __device__ constexpr int sidx(int r, int c) { return sym_index(r, c); }

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Workgroup w of `total` is given slot (w % 8) * (total / 8) + w / 8
// (the remainder spread over the first XCDs), so every XCD walks one
// contiguous range of slots and data shared by neighbouring slots meets in
// one L2.
__device__ __forceinline__ int xcd_slot(int w, int total) {
  const int xcd = w & 7, pos = w >> 3, q = total >> 3, r = total & 7;
  return (xcd < r) ? xcd * (q + 1) + pos : r * (q + 1) + (xcd - r) * q + pos;
}

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

// Level-1 parents touching a fixed DOF: eflag[e] = 1 (else 0) and the
// indices of the flagged parents appended to list (in no particular order;
// every entry is processed independently).  *count must be zero on entry.
__global__ void k_parent_flags(int cnx, int cny, int cnz, const uint8_t* __restrict__ mask,
                               uint8_t* __restrict__ eflag, int* __restrict__ list,
                               int* __restrict__ count) {
  const int64_t cne = (int64_t)cnx * cny * cnz;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cne) return;
  const int cx = (int)(e % cnx);
  const int64_t rest = e / cnx;
  const int cy = (int)(rest % cny), cz = (int)(rest / cny);
  const int fnx = 2 * cnx, fny = 2 * cny;
  unsigned any = 0;
  for (int t = 0; t < 27; ++t)
    any |= mask[node_of(fnx, fny, 2 * cx + t % 3, 2 * cy + (t / 3) % 3, 2 * cz + t / 9)];
  eflag[e] = any ? 1 : 0;
  if (any) list[atomicAdd(count, 1)] = (int)e;
}

__global__ void k_zero_int(int* p) { *p = 0; }

// Level-2 parents with a level-1 child flagged in eflag1: indices appended to
// list (in no particular order).  *count must be zero on entry.
__global__ void k_parent_flags2(int cnx, int cny, int cnz, const uint8_t* __restrict__ eflag1,
                                int* __restrict__ list, int* __restrict__ count) {
  const int64_t cne = (int64_t)cnx * cny * cnz;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cne) return;
  const int cx = (int)(e % cnx);
  const int64_t rest = e / cnx;
  const int cy = (int)(rest % cny), cz = (int)(rest / cny);
  const int nx1 = 2 * cnx, ny1 = 2 * cny;
  unsigned any = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c)
    any |= eflag1[(int64_t)(2 * cx + (c & 1)) +
                  (int64_t)nx1 * ((2 * cy + ((c >> 1) & 1)) + (int64_t)ny1 * (2 * cz + (c >> 2)))];
  if (any) list[atomicAdd(count, 1)] = (int)e;
}

// Level-2 Galerkin matrices from the fine moduli: Kc = sum_d E_d N_d over the
// 64 fine descendants d = 8 c1 + c0 (level-1 child c1, its fine child c0),
// N_d = P_c1^T M_c0 P_c1 precomputed and stored transposed, Nt[entry][d].
// Exact for parents whose level-1 children touch no fixed DOF (the level-1
// matrix of such a child is sum_c0 E M_c0); k_galerkin_lds<2> then
// overwrites the others.  The level-1 matrices are never formed for it.
// As a product [300 x 64] x [64 x parents] on FP64 MFMA: each wavefront
// takes 16 parents (their 64 moduli as the B operand, in registers) and
// walks the 19 tiles of 16 entries, 16 MFMA steps of k = 4 each; a lane
// holds result rows g + 4v (g = lane / 16) of column lane % 16, so each
// store writes 16 consecutive parents of one entry.
__global__ void __launch_bounds__(256) k_galerkin_fast2(int cnx, int cny, int cnz,
                                                        const double* __restrict__ Nt,
                                                        const double* __restrict__ E,
                                                        double* __restrict__ Kc) {
  const int64_t cne = (int64_t)cnx * cny * cnz;
  const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15;
  const int64_t p0 = (int64_t)blockIdx.x * 64 + 16 * (threadIdx.x >> 6);
  const int64_t par = p0 + j;
  const bool live = par < cne;
  double bop[16];  // B[k = g][col = j] of step s: modulus of descendant 4 s + g of parent par
  {
    const int64_t e = live ? par : 0;
    const int cx = (int)(e % cnx);
    const int64_t rest = e / cnx;
    const int cy = (int)(rest % cny), cz = (int)(rest / cny);
    const int fnx = 4 * cnx, fny = 4 * cny;
#pragma unroll
    for (int st = 0; st < 16; ++st) {
      const int d = 4 * st + g, c1 = d >> 3, c0 = d & 7;
      const int gx = 4 * cx + 2 * (c1 & 1) + (c0 & 1);
      const int gy = 4 * cy + 2 * ((c1 >> 1) & 1) + ((c0 >> 1) & 1);
      const int gz = 4 * cz + 2 * (c1 >> 2) + (c0 >> 2);
      bop[st] = live ? E[(int64_t)gx + (int64_t)fnx * (gy + (int64_t)fny * gz)] : 0.0;
    }
  }
  if (p0 >= cne) return;  // a whole wavefront past the end (no LDS, no barriers)
  for (int e0 = 0; e0 < kSym; e0 += 16) {
    const int ea = e0 + j;  // A[row = j][k = g] = Nt[e0 + j][4 s + g]
    double aop[16];
#pragma unroll
    for (int st = 0; st < 16; ++st) aop[st] = ea < kSym ? Nt[(int64_t)ea * 64 + 4 * st + g] : 0.0;
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int st = 0; st < 16; ++st)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(aop[st], bop[st], acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ent = e0 + g + 4 * v;
      if (live && ent < kSym) Kc[(int64_t)ent * cne + par] = acc[v];
    }
  }
}

// Level-1 inverse Jacobi diagonal without the stored matrices of unflagged
// parents: their diagonal entries are sum_c0 E_c0 M_c0, formed in the order
// of the level-1 fast path, so the result is the one k_diag_elemmat gives on
// fully stored matrices.
__global__ void k_diag_l1(int nx, int ny, int nz, const double* __restrict__ Ke,
                          const double* __restrict__ Mc, const double* __restrict__ E,
                          const uint8_t* __restrict__ eflag, double* __restrict__ dinv,
                          float* __restrict__ dinv32) {
  const int64_t nn = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  const int64_t ne = (int64_t)nx * ny * nz;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const int i = (int)(n % (nx + 1));
  const int64_t rest = n / (nx + 1);
  const int j = (int)(rest % (ny + 1));
  const int k = (int)(rest / (ny + 1));
  const int fnx = 2 * nx, fny = 2 * ny;
  double d[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int ex = i - (a & 1), ey = j - ((a >> 1) & 1), ez = k - (a >> 2);
    if (ex < 0 || ex >= nx || ey < 0 || ey >= ny || ez < 0 || ez >= nz) continue;
    const int64_t e = (int64_t)ex + (int64_t)nx * ((int64_t)ey + (int64_t)ny * ez);
    if (eflag[e]) {
#pragma unroll
      for (int c = 0; c < 3; ++c) d[c] += Ke[(int64_t)sidx(3 * a + c, 3 * a + c) * ne + e];
    } else {
      double w[8];
#pragma unroll
      for (int c0 = 0; c0 < 8; ++c0)
        w[c0] = E[(int64_t)(2 * ex + (c0 & 1)) +
                  (int64_t)fnx * ((2 * ey + ((c0 >> 1) & 1)) + (int64_t)fny * (2 * ez + (c0 >> 2)))];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int c0 = 0; c0 < 8; ++c0) acc = fma(w[c0], Mc[c0 * kSym + sidx(3 * a + c, 3 * a + c)], acc);
        d[c] += acc;
      }
    }
  }
  for (int c = 0; c < 3; ++c) {
    const double di = d[c] == 0.0 ? 1.0 : 1.0 / d[c];  // dead coarse DOF: identity row
    dinv[c * nn + n] = di;
    if (dinv32) dinv32[c * nn + n] = (float)di;
  }
}

// Galerkin matrix of one parent per block iteration: the 8 child matrices
// are staged in LDS, then child by child T_c = K_c P_c is formed by a column
// pass and P_c^T T_c added by a row pass (registers stay few, so several
// workgroups share a CU).  MODE 1 (from the fine grid): children are
// E_c Df KE Df with the fine fixed-DOF mask, for the parents listed by
// k_parent_flags (the others are exact from the fast path); list entry
// w < cap is also written to the compact copy Kcomp[entry][w].  MODE 0: every
// parent, with the previous level's packed matrices as children.  MODE 2
// (level 2): the parents listed by k_parent_flags2; a child flagged in
// `mask` (the level-1 flags) is read from Kf, the others are formed from
// their fine moduli as sum_c0 E_c0 M_c0 (KE holds the 8 M_c0), the value
// the level-1 fast path would have stored.
template <int MODE>
__global__ void __launch_bounds__(256) k_galerkin_lds(int cnx, int cny, int cnz,
                                                      const double* __restrict__ KE,
                                                      const double* __restrict__ E,
                                                      const uint8_t* __restrict__ mask,
                                                      const int* __restrict__ list,
                                                      const int* __restrict__ count,
                                                      const double* __restrict__ Kf,
                                                      double* __restrict__ Kc,
                                                      double* __restrict__ Kcomp, int cap) {
  __shared__ double sK[8][24][25];
  __shared__ double sT[24][25];
  __shared__ uint8_t sm[27];
  __shared__ double sw[64];
  constexpr bool FROM_FINE = MODE == 1;
  const int64_t cne = (int64_t)cnx * cny * cnz;
  const int fnx = 2 * cnx, fny = 2 * cny;
  const int64_t fne = cne * 8;
  const int tid = threadIdx.x;
  const int64_t nwork = MODE != 0 ? (int64_t)*count : cne;
  // XCD-aware order (every parent): workgroups are dispatched round-robin
  // over the 8 XCDs, so XCD x takes a contiguous range of parents and its
  // workgroups walk it together.  Neighbouring parents read their children
  // from the same cache lines (the children of 8 parents along x share one
  // 128-byte line of each packed entry), which then meet in one L2.
  int64_t w0 = blockIdx.x, w1 = nwork, ws = gridDim.x;
  if (MODE == 0 && gridDim.x >= 8) {
    const int x = blockIdx.x & 7, nbx = (int)(gridDim.x >> 3) + (x < (int)(gridDim.x & 7) ? 1 : 0);
    w0 = nwork * x / 8 + (blockIdx.x >> 3);
    w1 = nwork * (x + 1) / 8;
    ws = nbx;
  }
  for (int64_t w = w0; w < w1; w += ws) {
  const int64_t eid = MODE != 0 ? (int64_t)list[w] : w;
  const int cx = (int)(eid % cnx);
  const int64_t rest = eid / cnx;
  const int cy = (int)(rest % cny), cz = (int)(rest / cny);
  if (FROM_FINE) {
    if (tid < 27) {
      const int px = tid % 3, py = (tid / 3) % 3, pz = tid / 9;
      sm[tid] = mask[node_of(fnx, fny, 2 * cx + px, 2 * cy + py, 2 * cz + pz)];
    }
    if (tid < 8)
      sw[tid] = E[(int64_t)(2 * cx + (tid & 1)) +
                  (int64_t)fnx * ((2 * cy + ((tid >> 1) & 1)) + (int64_t)fny * (2 * cz + (tid >> 2)))];
    __syncthreads();
  }
  if (MODE == 2) {  // child flags, and the moduli of the 64 fine descendants
    if (tid < 8) {
      const int64_t ce = (int64_t)(2 * cx + (tid & 1)) +
                         (int64_t)fnx * ((2 * cy + ((tid >> 1) & 1)) + (int64_t)fny * (2 * cz + (tid >> 2)));
      sm[tid] = mask[ce];
    }
    if (tid < 64) {
      const int c1 = tid >> 3, c0 = tid & 7;
      const int gx = 4 * cx + 2 * (c1 & 1) + (c0 & 1);
      const int gy = 4 * cy + 2 * ((c1 >> 1) & 1) + ((c0 >> 1) & 1);
      const int gz = 4 * cz + 2 * (c1 >> 2) + (c0 >> 2);
      sw[tid] = E[(int64_t)gx + (int64_t)(2 * fnx) * (gy + (int64_t)(2 * fny) * gz)];
    }
    __syncthreads();
  }
  // the 8 x 576 child entries, 18 per thread, all loads in flight before
  // the first LDS store
  double lv[18];
#pragma unroll
  for (int u = 0; u < 18; ++u) {
    const int t = tid + 256 * u;
    const int c = t / 576, r = (t % 576) / 24, q = t % 24;
    const int dx = c & 1, dy = (c >> 1) & 1, dz = c >> 2;
    if (FROM_FINE) {
      const int br = r / 3, bq = q / 3;
      const int pr = (dx + (br & 1)) + 3 * (dy + ((br >> 1) & 1)) + 9 * (dz + (br >> 2));
      const int pq = (dx + (bq & 1)) + 3 * (dy + ((bq >> 1) & 1)) + 9 * (dz + (bq >> 2));
      const bool fx = ((sm[pr] >> (r % 3)) & 1) || ((sm[pq] >> (q % 3)) & 1);
      lv[u] = fx ? 0.0 : sw[c] * KE[r * 24 + q];
    } else if (MODE == 2 && !sm[c]) {
      double acc = 0.0;  // the level-1 fast path's sum, in its order
#pragma unroll
      for (int c0 = 0; c0 < 8; ++c0) acc = fma(sw[8 * c + c0], KE[c0 * kSym + sidx(r, q)], acc);
      lv[u] = acc;
    } else {
      const int64_t fe = (int64_t)(2 * cx + dx) + (int64_t)fnx * ((2 * cy + dy) + (int64_t)fny * (2 * cz + dz));
      lv[u] = Kf[(int64_t)sidx(r, q) * fne + fe];
    }
  }
#pragma unroll
  for (int u = 0; u < 18; ++u) {
    const int t = tid + 256 * u;
    sK[t / 576][(t % 576) / 24][t % 24] = lv[u];
  }
  __syncthreads();
  // child by child: column pass T[r][3B+j] = sum_b P_c[b][B] K_c[r][3b+j]
  // into sT, then the row pass adds sum_b P_c[b][A] T[3b+i][J] to the packed
  // entries (I <= J) this thread owns (sx = tid and tid + 256)
  int Iown[2], Jown[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int sx = tid + 256 * h;
    int I = 0;
    if (sx < kSym)
      while (sidx(I, 23) < sx) ++I;  // row of packed entry sx
    Iown[h] = I;
    Jown[h] = sx < kSym ? I + (sx - sidx(I, I)) : 0;
  }
  double racc[2] = {0.0, 0.0};
  for (int c = 0; c < 8; ++c) {
    const int dx = c & 1, dy = (c >> 1) & 1, dz = c >> 2;
    for (int t = tid; t < 576; t += 256) {
      const int r = t / 24, J = t % 24, B = J / 3, j = J % 3;
      double acc = 0.0;
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const double pb = phi1(dx + (b & 1), B & 1) * phi1(dy + ((b >> 1) & 1), (B >> 1) & 1) *
                          phi1(dz + (b >> 2), B >> 2);
        acc = fma(pb, sK[c][r][3 * b + j], acc);
      }
      sT[r][J] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int A = Iown[h] / 3, i = Iown[h] % 3, J = Jown[h];
      double acc = racc[h];
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const double pa = phi1(dx + (b & 1), A & 1) * phi1(dy + ((b >> 1) & 1), (A >> 1) & 1) *
                          phi1(dz + (b >> 2), A >> 2);
        acc = fma(pa, sT[3 * b + i][J], acc);
      }
      racc[h] = acc;
    }
    __syncthreads();  // sT is rewritten for the next child
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int sx = tid + 256 * h;
    if (sx < kSym) {
      Kc[(int64_t)sx * cne + eid] = racc[h];
      if (FROM_FINE && w < cap) Kcomp[(int64_t)sx * cap + w] = racc[h];
    }
  }
  __syncthreads();  // sK, sm, sw are reused by the next parent
  }
}

// Row and column of packed entry s (upper triangle, row-major, 24 x 24).
__device__ inline void sym_unpack(int s, int& r, int& q) {
  int a = (int)((49.0f - sqrtf((float)(2401 - 8 * s))) * 0.5f);
  if (a < 23 && sidx(a + 1, a + 1) <= s) ++a;
  if (sidx(a, a) > s) --a;
  r = a;
  q = a + (s - sidx(a, a));
}

// Levels >= 2: Kc = sum_c P_c^T Kf_c P_c from the stored matrices of the
// level below, for 8 parents along x per workgroup.  The children of 8
// consecutive parents at one child position lie at every other element of a
// 16-element x-run of the level below, so one load instruction takes 8 whole
// entries from 8 cache lines (a parent alone used 16 bytes of each of its
// 1200 lines).  Per child position: the 8 children are unpacked into LDS,
// then column passes T = K_c P_c for 4 parents at a time and row passes
// add P_c^T T to the packed entries each thread owns (as k_galerkin_lds);
// 5 barriers per child position and 8 parents.
__global__ void __launch_bounds__(256) k_galerkin_row8(int cnx, int cny, int cnz,
                                                       const double* __restrict__ Kf,
                                                       double* __restrict__ Kc) {
  __shared__ double sK[8][24][25];
  __shared__ double sT[4][24][25];
  const int64_t cne = (int64_t)cnx * cny * cnz;
  const int fnx = 2 * cnx, fny = 2 * cny;
  const int64_t fne = cne * 8;
  const int gxr = (cnx + 7) / 8;
  const int64_t nwork = (int64_t)gxr * cny * cnz;
  const int tid = threadIdx.x;
  // XCD-aware order, as in k_galerkin_lds: each XCD walks a contiguous range
  // of groups, so y/z-neighbouring groups are close in time on one L2
  int64_t w0 = blockIdx.x, w1 = nwork, ws = gridDim.x;
  if (gridDim.x >= 8) {
    const int x = blockIdx.x & 7, nbx = (int)(gridDim.x >> 3) + (x < (int)(gridDim.x & 7) ? 1 : 0);
    w0 = nwork * x / 8 + (blockIdx.x >> 3);
    w1 = nwork * (x + 1) / 8;
    ws = nbx;
  }
  int Iown[2], Jown[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int sx = tid + 256 * h;
    int I = 0;
    if (sx < kSym)
      while (sidx(I, 23) < sx) ++I;
    Iown[h] = I;
    Jown[h] = sx < kSym ? I + (sx - sidx(I, I)) : 0;
  }
  for (int64_t w = w0; w < w1; w += ws) {
    const int gx = (int)(w % gxr);
    const int64_t rest = w / gxr;
    const int cy = (int)(rest % cny), cz = (int)(rest / cny);
    const int cx0 = 8 * gx;
    const int np = min(8, cnx - cx0);
    double racc[8][2];
#pragma unroll
    for (int p = 0; p < 8; ++p) racc[p][0] = racc[p][1] = 0.0;
    for (int c = 0; c < 8; ++c) {
      const int dx = c & 1, dy = (c >> 1) & 1, dz = c >> 2;
      const int64_t fe0 = (int64_t)(2 * cx0 + dx) + (int64_t)fnx * ((2 * cy + dy) + (int64_t)fny * (2 * cz + dz));
      // lane t: entry t / 8 of parent t % 8; all loads in flight first
      double lv[10];
#pragma unroll
      for (int u = 0; u < 10; ++u) {
        const int t = tid + 256 * u;
        const int p = t & 7;
        lv[u] = (t < 8 * kSym && p < np) ? Kf[(int64_t)(t >> 3) * fne + fe0 + 2 * p] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 10; ++u) {
        const int t = tid + 256 * u;
        if (t < 8 * kSym) {
          int r, q;
          sym_unpack(t >> 3, r, q);
          sK[t & 7][r][q] = lv[u];
          sK[t & 7][q][r] = lv[u];
        }
      }
      __syncthreads();
#pragma unroll
      for (int pg = 0; pg < 8; pg += 4) {
        for (int t = tid; t < 4 * 576; t += 256) {
          const int pp = t / 576, r = (t % 576) / 24, J = t % 24, B = J / 3, j = J % 3;
          double acc = 0.0;
#pragma unroll
          for (int b = 0; b < 8; ++b) {
            const double pb = phi1(dx + (b & 1), B & 1) * phi1(dy + ((b >> 1) & 1), (B >> 1) & 1) *
                              phi1(dz + (b >> 2), B >> 2);
            acc = fma(pb, sK[pg + pp][r][3 * b + j], acc);
          }
          sT[pp][r][J] = acc;
        }
        __syncthreads();
#pragma unroll
        for (int pp = 0; pp < 4; ++pp)
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int A = Iown[h] / 3, i = Iown[h] % 3, J = Jown[h];
            double acc = racc[pg + pp][h];
#pragma unroll
            for (int b = 0; b < 8; ++b) {
              const double pa = phi1(dx + (b & 1), A & 1) * phi1(dy + ((b >> 1) & 1), (A >> 1) & 1) *
                                phi1(dz + (b >> 2), A >> 2);
              acc = fma(pa, sT[pp][3 * b + i][J], acc);
            }
            racc[pg + pp][h] = acc;
          }
        __syncthreads();  // sT (next round) and sK (next child) are rewritten
      }
    }
    // outputs through LDS, then 8 consecutive parents per entry in one run
    double* sO = &sK[0][0][0];  // [entry][parent], 2400 doubles
#pragma unroll
    for (int p = 0; p < 8; ++p)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int sx = tid + 256 * h;
        if (sx < kSym) sO[sx * 8 + p] = racc[p][h];
      }
    __syncthreads();
    const int64_t e0 = (int64_t)cx0 + (int64_t)cnx * (cy + (int64_t)cny * cz);
    for (int t = tid; t < 8 * kSym; t += 256) {
      const int p = t & 7;
      if (p < np) Kc[(int64_t)(t >> 3) * cne + e0 + p] = sO[t];
    }
    __syncthreads();  // sK is reused by the next group
  }
}

// y = sum_e L_e^T Ke_e L_e v on a coarse level (levels >= 2) from the stored
// packed element matrices.  Block: 64 consecutive nodes x 8 waves; wave a
// takes each node as local corner a of the element e = node - offset(a) and
// forms rows 3a..3a+2 of Ke_e v_e; the 8 partial rows are summed in LDS in a
// fixed order.  Vectors of type T, matrices of type KT (FP64, or the FP32
// copy the refinement form keeps, which holds the values the FP32 product
// would round them to anyway).  Blocks in XCD-contiguous order: the two
// copies of a symmetric entry are read by the waves of two corners, for
// nodes up to a plane apart, and are then fetched into one L2 only.
// With jb non-null the product feeds a damped-Jacobi sweep instead:
// y = v + omega jd (jb - A v) (y distinct from v).
template <typename T, typename KT = double>
__global__ void __launch_bounds__(512) k_apply_elemmat(int nx, int ny, int nz,
                                                       const KT* __restrict__ Ke,
                                                       const T* __restrict__ v,
                                                       T* __restrict__ y,
                                                       const T* __restrict__ jb,
                                                       const T* __restrict__ jd, T omega,
                                                       int64_t rs = 0) {
  __shared__ T red[8][3][64];
  {  // load case blockIdx.z of a lock-step multi-vector (rs: vector stride)
    const int64_t ro = (int64_t)blockIdx.z * rs;
    v += ro;
    y += ro;
    if (jb) jb += ro;
  }
  const int a = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int64_t nn = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  const int64_t ne = (int64_t)nx * ny * nz;
  const int64_t n = (int64_t)xcd_slot(blockIdx.x, gridDim.x) * 64 + lane;
  T acc0 = 0, acc1 = 0, acc2 = 0;
  if (n < nn) {
    const int i = (int)(n % (nx + 1));
    const int64_t rest = n / (nx + 1);
    const int j = (int)(rest % (ny + 1));
    const int k = (int)(rest / (ny + 1));
    const int ex = i - (a & 1), ey = j - ((a >> 1) & 1), ez = k - (a >> 2);
    if (ex >= 0 && ex < nx && ey >= 0 && ey < ny && ez >= 0 && ez < nz) {
      const int64_t e = (int64_t)ex + (int64_t)nx * ((int64_t)ey + (int64_t)ny * ez);
      T ve[24];
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const int64_t nb = node_of(nx, ny, ex + (b & 1), ey + ((b >> 1) & 1), ez + (b >> 2));
#pragma unroll
        for (int c = 0; c < 3; ++c) ve[3 * b + c] = v[c * nn + nb];
      }
#pragma unroll
      for (int q = 0; q < 24; ++q) {
        acc0 = fma((T)Ke[(int64_t)sidx(3 * a + 0, q) * ne + e], ve[q], acc0);
        acc1 = fma((T)Ke[(int64_t)sidx(3 * a + 1, q) * ne + e], ve[q], acc1);
        acc2 = fma((T)Ke[(int64_t)sidx(3 * a + 2, q) * ne + e], ve[q], acc2);
      }
    }
  }
  red[a][0][lane] = acc0;
  red[a][1][lane] = acc1;
  red[a][2][lane] = acc2;
  __syncthreads();
  if (a < 3 && n < nn) {
    T sum = red[0][a][lane];
#pragma unroll
    for (int q = 1; q < 8; ++q) sum += red[q][a][lane];
    const int64_t d = a * nn + n;
    y[d] = jb ? v[d] + omega * jd[d] * (jb[d] - sum) : sum;
  }
}

// 8-point Walsh-Hadamard transform x[k] <- sum_a (-1)^popcount(k & a) x[a]
// of the entries 3a + s (one component s) of a 24-vector.
template <typename T>
__device__ __forceinline__ void wht8(T* x, int s) {
#pragma unroll
  for (int bit = 1; bit < 8; bit <<= 1)
#pragma unroll
    for (int a = 0; a < 8; ++a)
      if (!(a & bit)) {
        const T p = x[3 * a + s], q = x[3 * (a | bit) + s];
        x[3 * a + s] = p + q;
        x[3 * (a | bit) + s] = p - q;
      }
}

// Level-1 element products, pass 1: Y[q][e] = (Ke_e v_e)[q].  SO = 0..2: one
// thread per parent element e and output component SO, which writes the
// entries q = 3a + SO; SO = 3: one thread per parent, all 24 entries (the
// inputs, their transforms and the moduli's are then formed once, not three
// times; on large levels that is faster, on small ones three times the
// threads fill the chip better).  Parents without a fixed DOF among their fine nodes have
// Ke_e = sum_c E_c M_c with M_c = R_c M_0 R_c (R_c the mirror map of child c).
// In the Walsh basis over the 8 corners (index 3k + s), R_c is the diagonal
// sign (-1)^popcount(c & mu), mu(k, s) = k ^ (1 << s), so
//   W Ke_e W / 64 = B'[kappa][lambda] * Ehat[mu(kappa) ^ mu(lambda)]
// with B' = W M_0 W / 64 and Ehat the Walsh transform of the 8 child moduli:
// y = W ((B' o Ehat) (W v)), about 256 FMA per thread.  Parents with eflag 1
// are left to l1_masked_rows, so no wave carries both paths.
template <typename T, int SO>
__device__ __forceinline__ void l1_elem(int nx, int ny, int nz, const double* __restrict__ Ke,
                                        const T* __restrict__ Bw, const T* __restrict__ Ef,
                                        const uint8_t* __restrict__ eflag,
                                        const T* __restrict__ v, T* __restrict__ Y, int nbe) {
  const int64_t nn = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  const int64_t ne = (int64_t)nx * ny * nz;
  const int64_t e = SO == 3 ? ((int64_t)blockIdx.y * nbe + blockIdx.x) * blockDim.x + threadIdx.x
                            : (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne || eflag[e]) return;  // flagged parents: l1_masked_rows
  const int ex = (int)(e % nx);
  const int64_t rest = e / nx;
  const int ey = (int)(rest % ny), ez = (int)(rest / ny);
  T x[24];
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const int64_t nb = node_of(nx, ny, ex + (b & 1), ey + ((b >> 1) & 1), ez + (b >> 2));
#pragma unroll
    for (int c = 0; c < 3; ++c) x[3 * b + c] = v[c * nn + nb];
  }
  {
    T Eh[8];
    const int fnx = 2 * nx, fny = 2 * ny;
#pragma unroll
    for (int c = 0; c < 8; ++c)
      Eh[c] = Ef[(int64_t)(2 * ex + (c & 1)) +
                 (int64_t)fnx * ((2 * ey + ((c >> 1) & 1)) + (int64_t)fny * (2 * ez + (c >> 2)))];
#pragma unroll
    for (int bit = 1; bit < 8; bit <<= 1)
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (!(c & bit)) {
          const T p = Eh[c], q = Eh[c | bit];
          Eh[c] = p + q;
          Eh[c | bit] = p - q;
        }
#pragma unroll
    for (int s = 0; s < 3; ++s) wht8(x, s);
#pragma unroll
    for (int so = 0; so < 3; ++so) {  // output component: entries 3a + so
      if (SO != 3 && so != SO) continue;
      const T* B = Bw + so * 24;       // row kappa = 3k + so starts at B + 72k
      T y[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int muk = k ^ (1 << so);
        T acc = 0;
#pragma unroll
        for (int mm = 0; mm < 8; ++mm) {
          T t = 0;
#pragma unroll
          for (int s2 = 0; s2 < 3; ++s2) {
            const int la = 3 * (muk ^ mm ^ (1 << s2)) + s2;
            t = fma(B[72 * k + la], x[la], t);
          }
          acc = fma(Eh[mm], t, acc);
        }
        y[k] = acc;
      }
#pragma unroll
      for (int bit = 1; bit < 8; bit <<= 1)
#pragma unroll
        for (int a = 0; a < 8; ++a)
          if (!(a & bit)) {
            const T p = y[a], q = y[a | bit];
            y[a] = p + q;
            y[a | bit] = p - q;
          }
#pragma unroll
      for (int a = 0; a < 8; ++a) Y[(int64_t)(3 * a + so) * ne + e] = y[a];
    }
  }
}

// Level-1 element products of the flagged parents (list[0..cnt)) from their
// stored Galerkin matrices.  Row r is uniform per wavefront; its lanes take
// 16 list entries w (from chunk * 16 in steps of nchunk * 16), four lanes per
// entry, each lane two corners (six columns q = 3b + c), so that all of a
// lane's loads are in flight at once; the four sums are then added in a
// fixed order.  Rows come from the compact copy Kcomp[entry][w] (coalesced
// over w) while the list fits its capacity, else from Ke.
template <typename T>
__device__ __forceinline__ void l1_masked_rows(int nx, int ny, int nz,
                                               const double* __restrict__ Ke,
                                               const double* __restrict__ Kcomp, int cap,
                                               const int* __restrict__ list, int cnt,
                                               const T* __restrict__ v, T* __restrict__ Y,
                                               int chunk, int nchunk, int r) {
  const int64_t nn = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  const int64_t ne = (int64_t)nx * ny * nz;
  const bool compact = cnt <= cap;
  const int lane = threadIdx.x & 63, quarter = lane >> 4;
  const int64_t stride = (int64_t)nchunk * 16;
  // the loop bound is uniform per wavefront, so every lane reaches the shuffles
  for (int64_t base = (int64_t)chunk * 16; base < cnt; base += stride) {
    const int64_t w = base + (lane & 15);
    T acc = 0;
    int64_t e = 0;
    if (w < cnt) {
      e = list[w];
      const int ex = (int)(e % nx);
      const int64_t rest = e / nx;
      const int ey = (int)(rest % ny), ez = (int)(rest / ny);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int b = 2 * quarter + h;
        const int64_t nb = node_of(nx, ny, ex + (b & 1), ey + ((b >> 1) & 1), ez + (b >> 2));
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const int q = 3 * b + c;
          const double k =
              compact ? Kcomp[(int64_t)sidx(r, q) * cap + w] : Ke[(int64_t)sidx(r, q) * ne + e];
          acc = fma((T)k, v[c * nn + nb], acc);
        }
      }
    }
    acc += __shfl_down(acc, 32, 64);  // corners 0-3 + 4-7
    acc += __shfl_down(acc, 16, 64);
    if (quarter == 0 && w < cnt) Y[(int64_t)r * ne + e] = acc;
  }
}

// Pass 1 in one launch: workgroups x < nbe run the element path (grid.y:
// output component, or with all3 a third of the elements each); the rest
// run the flagged parents, two per grid.y, each with four rows (one per
// wavefront) of a 16-entry chunk of the list.
template <typename T>
__global__ void __launch_bounds__(256) k_l1_elem(int nx, int ny, int nz,
                                                 const double* __restrict__ Ke,
                                                 const T* __restrict__ Bw,
                                                 const T* __restrict__ Ef,
                                                 const uint8_t* __restrict__ eflag,
                                                 const T* __restrict__ v, T* __restrict__ Y,
                                                 int nbe, const double* __restrict__ Kcomp,
                                                 int cap, const int* __restrict__ list, int cnt,
                                                 int all3, int64_t rs = 0, int64_t Ys = 0) {
  v += (int64_t)blockIdx.z * rs;  // load case blockIdx.z
  Y += (int64_t)blockIdx.z * Ys;
  if ((int)blockIdx.x >= nbe) {  // workgroup-uniform
    const int mb = (int)blockIdx.x - nbe;
    const int r = (int)(blockIdx.y * 2 + (mb & 1)) * 4 + (int)(threadIdx.x >> 6);
    l1_masked_rows<T>(nx, ny, nz, Ke, Kcomp, cap, list, cnt, v, Y, mb >> 1,
                      ((int)gridDim.x - nbe) >> 1, r);
    return;
  }
  if (all3) {
    l1_elem<T, 3>(nx, ny, nz, Ke, Bw, Ef, eflag, v, Y, nbe);
    return;
  }
  switch (blockIdx.y) {  // output component
    case 0: l1_elem<T, 0>(nx, ny, nz, Ke, Bw, Ef, eflag, v, Y, nbe); break;
    case 1: l1_elem<T, 1>(nx, ny, nz, Ke, Bw, Ef, eflag, v, Y, nbe); break;
    default: l1_elem<T, 2>(nx, ny, nz, Ke, Bw, Ef, eflag, v, Y, nbe); break;
  }
}

// Pass 2: y[c][n] = sum over the (up to 8) elements around node n, taken in
// corner order a = 0..7, of Y[3a + c][e(n, a)].
// With jb non-null: y += omega jd (jb - (A v)) in place (y is the product's
// input v, read only here), the damped-Jacobi sweep on the product.
template <typename T>
__global__ void __launch_bounds__(256) k_l1_gather(int nx, int ny, int nz,
                                                   const T* __restrict__ Y, T* __restrict__ y,
                                                   const T* __restrict__ jb,
                                                   const T* __restrict__ jd, T omega,
                                                   int64_t rs = 0, int64_t Ys = 0) {
  const int64_t nn = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  const int64_t ne = (int64_t)nx * ny * nz;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  Y += (int64_t)blockIdx.z * Ys;  // load case blockIdx.z
  y += (int64_t)blockIdx.z * rs;
  if (jb) jb += (int64_t)blockIdx.z * rs;
  if (n >= nn) return;
  const int i = (int)(n % (nx + 1));
  const int64_t rest = n / (nx + 1);
  const int j = (int)(rest % (ny + 1)), k = (int)(rest / (ny + 1));
  T acc[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int ex = i - (a & 1), ey = j - ((a >> 1) & 1), ez = k - (a >> 2);
    if (ex < 0 || ex >= nx || ey < 0 || ey >= ny || ez < 0 || ez >= nz) continue;
    const int64_t e = (int64_t)ex + (int64_t)nx * ((int64_t)ey + (int64_t)ny * ez);
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] += Y[(int64_t)(3 * a + c) * ne + e];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int64_t d = c * nn + n;
    if (jb) y[d] = y[d] + omega * jd[d] * (jb[d] - acc[c]);
    else y[d] = acc[c];
  }
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

// bc = P^T Df (bf - tf) (tf == nullptr: bf alone), weights (1/2, 1, 1/2)
// per axis.  One thread per (coarse node, fine z-offset) and component
// (grid.y); the three z-planes of a coarse node are summed in LDS.  On the
// plane grid (cnz = 0) only the middle offset lies in the grid.
// mask == nullptr: no fine fixed DOFs.
// With xc non-null also the coarse level's first Jacobi sweep from zero,
// xc = omega dc bc.
template <typename T>
__global__ void __launch_bounds__(192) k_restrict(int cnx, int cny, int cnz,
                                                  const T* __restrict__ bf,
                                                  const T* __restrict__ tf,
                                                  const uint8_t* __restrict__ mask,
                                                  T* __restrict__ bc,
                                                  const T* __restrict__ dc, T omega,
                                                  T* __restrict__ xc, int64_t fs = 0,
                                                  int64_t cs = 0) {
  __shared__ T part[3][64];
  {  // load case blockIdx.z (fs, cs: fine and coarse vector strides)
    const int64_t fo = (int64_t)blockIdx.z * fs, co = (int64_t)blockIdx.z * cs;
    bf += fo;
    if (tf) tf += fo;
    bc += co;
    if (xc) xc += co;
  }
  const int lane = threadIdx.x & 63, dzi = threadIdx.x >> 6;
  const int c = blockIdx.y;
  const int64_t cnn = (int64_t)(cnx + 1) * (cny + 1) * (cnz + 1);
  const int64_t n = (int64_t)blockIdx.x * 64 + lane;
  const int fnx = 2 * cnx, fny = 2 * cny, fnz = 2 * cnz;
  const int64_t fnn = (int64_t)(fnx + 1) * (fny + 1) * (fnz + 1);
  T acc = 0;
  if (n < cnn) {
    const int I = (int)(n % (cnx + 1));
    const int64_t rest = n / (cnx + 1);
    const int J = (int)(rest % (cny + 1));
    const int K = (int)(rest / (cny + 1));
    const int fk = 2 * K + dzi - 1;
    if (fk >= 0 && fk <= fnz) {
      const T wz = dzi == 1 ? T(1) : T(0.5);
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
        const int fj = 2 * J + dy;
        if (fj < 0 || fj > fny) continue;
        const T wyz = (dy ? T(0.5) : T(1)) * wz;
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const int fi = 2 * I + dx;
          if (fi < 0 || fi > fnx) continue;
          const T w = (dx ? T(0.5) : T(1)) * wyz;
          const int64_t f = node_of(fnx, fny, fi, fj, fk);
          const bool fixed = mask && ((mask[f] >> c) & 1);
          const T val = tf ? bf[c * fnn + f] - tf[c * fnn + f] : bf[c * fnn + f];
          if (!fixed) acc = fma(w, val, acc);
        }
      }
    }
  }
  part[dzi][lane] = acc;
  __syncthreads();
  if (dzi == 0 && n < cnn) {
    const T v = part[0][lane] + part[1][lane] + part[2][lane];
    bc[c * cnn + n] = v;
    if (xc) xc[c * cnn + n] = omega * dc[c * cnn + n] * v;
  }
}

// Lane i of a wavefront takes lane i-1's (wave_shr:1) or lane i+1's
// (wave_shl:1) value through DPP; the end lanes read 0.
template <int CTRL>
__device__ inline double wave_shift(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ inline float wave_shift(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, true));
}

// The same restriction on large 3D grids, separably and as a z-march: a
// workgroup takes a tile of kRsCI x kRsCJ coarse columns and a chunk of
// coarse planes [K0, K1), and reads each fine plane of the chunk once (the
// tile's 2 kRsCJ + 1 fine rows, one fine node per lane, 63 nodes of a row on
// lanes 0..62: whole rows, coalesced).  A fine plane is restricted along x in
// registers (DPP neighbours) and along y through LDS; every coarse node
// keeps the xy sum of the last odd fine plane and forms plane K along z as
// sy(2K) + (sy(2K-1) + sy(2K+1)) / 2.  Per coarse node the sum is thus
// m + (l + r) / 2 along x, then y, then z: a fixed order, so results are
// deterministic, and equal to the per-node sum of the small-grid kernel up
// to rounding.  All three components in one workgroup (one mask load per
// fine node).  Eight wavefronts take three of the 17 fine rows each.  Two
// raw-plane buffers: a buffer is reloaded with the plane two ahead as soon
// as its values are read, so each plane's loads have two planes of work to
// arrive in.  blockIdx.x: (tile, chunk) with tiles fastest, in XCD-contiguous
// order; blockIdx.z: load case.
constexpr int kRsCI = 31;
constexpr int kRsCJ = 8;
constexpr int kRsRows = 2 * kRsCJ + 1;
constexpr int kRmWaves = 8;
constexpr int kRmRowsPerWave = (kRsRows + kRmWaves - 1) / kRmWaves;
template <typename T>
struct RmRaw {
  T b[3][kRmRowsPerWave], t[3][kRmRowsPerWave];
  uint32_t m[kRmRowsPerWave];
};
template <typename T>
__global__ void __launch_bounds__(64 * kRmWaves) k_restrict_zm(
    int cnx, int cny, int cnz, int gx, int gy, int TK, const T* __restrict__ bf,
    const T* __restrict__ tf, const uint8_t* __restrict__ mask, T* __restrict__ bc,
    const T* __restrict__ dc, T omega, T* __restrict__ xc, int64_t fs, int64_t cs) {
  __shared__ T xr[2][3][kRsRows][32];  // [buffer][component][row][coarse column]
  {  // load case blockIdx.z
    const int64_t fo = (int64_t)blockIdx.z * fs, co = (int64_t)blockIdx.z * cs;
    bf += fo;
    if (tf) tf += fo;
    bc += co;
    if (xc) xc += co;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int bx, by, K0;
  {
    const int t = xcd_slot(blockIdx.x, gridDim.x);
    bx = t % gx;
    by = (t / gx) % gy;
    K0 = (t / (gx * gy)) * TK;
  }
  const int K1 = min(K0 + TK, cnz + 1);
  const int I0 = bx * kRsCI, J0 = by * kRsCJ;
  const int fnx = 2 * cnx, fny = 2 * cny, fnz = 2 * cnz;
  const int64_t fnn = (int64_t)(fnx + 1) * (fny + 1) * (fnz + 1);
  const int64_t cnn = (int64_t)(cnx + 1) * (cny + 1) * (cnz + 1);
  const int64_t fplane = (int64_t)(fnx + 1) * (fny + 1);
  const int fx = 2 * I0 - 1 + lane;
  const bool xok = lane < 2 * kRsCI + 1 && fx >= 0 && fx <= fnx;
  // raw values of this lane's nodes of rows w + 8 q of fine plane fz; 0 outside
  auto load = [&](int fz, RmRaw<T>& R) {
#pragma unroll
    for (int q = 0; q < kRmRowsPerWave; ++q) {
      const int r = w + kRmWaves * q, fy = 2 * J0 - 1 + r;
      const bool ok = r < kRsRows && xok && fy >= 0 && fy <= fny && fz >= 0 && fz <= fnz;
      const int64_t f = (int64_t)fz * fplane + (int64_t)fy * (fnx + 1) + fx;
      R.m[q] = (mask && ok) ? mask[f] : 0u;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        R.b[c][q] = ok ? bf[c * fnn + f] : T(0);
        R.t[c][q] = (tf && ok) ? tf[c * fnn + f] : T(0);
      }
    }
  };
  const int ci = threadIdx.x & 31, cj = threadIdx.x >> 5;  // output thread's coarse node
  const bool out = threadIdx.x < 32 * kRsCJ && ci < kRsCI && I0 + ci <= cnx && J0 + cj <= cny;
  int buf = 0;
  // Df (b - t) of a loaded plane, then its x sums into LDS; after the
  // barrier the output threads form the y sums sy
  auto values = [&](const RmRaw<T>& R, T (&v)[3][kRmRowsPerWave]) {
#pragma unroll
    for (int q = 0; q < kRmRowsPerWave; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        T val = R.b[c][q];
        if (tf) val -= R.t[c][q];
        v[c][q] = ((R.m[q] >> c) & 1u) ? T(0) : val;
      }
  };
  auto xy = [&](const T (&v)[3][kRmRowsPerWave], T (&sy)[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int q = 0; q < kRmRowsPerWave; ++q) {
        const int r = w + kRmWaves * q;
        const T l = wave_shift<0x138>(v[c][q]), rr = wave_shift<0x130>(v[c][q]);
        const T sx = v[c][q] + T(0.5) * (l + rr);
        if (r < kRsRows && (lane & 1) && lane < 2 * kRsCI) xr[buf][c][r][lane >> 1] = sx;
      }
    __syncthreads();
    if (out) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
        sy[c] = xr[buf][c][2 * cj + 1][ci] +
                T(0.5) * (xr[buf][c][2 * cj][ci] + xr[buf][c][2 * cj + 2][ci]);
    }
    buf ^= 1;
  };
  RmRaw<T> RA, RB;
  T carry[3] = {T(0), T(0), T(0)}, s0[3] = {T(0), T(0), T(0)}, s1[3] = {T(0), T(0), T(0)};
  {
    RmRaw<T> R0;
    load(2 * K0 - 1, R0);
    load(2 * K0, RA);
    load(2 * K0 + 1, RB);
    T v[3][kRmRowsPerWave];
    values(R0, v);
    xy(v, carry);
  }
  for (int K = K0; K < K1; ++K) {
    T v[3][kRmRowsPerWave];
    values(RA, v);
    load(K + 1 < K1 ? 2 * K + 2 : -1, RA);
    xy(v, s0);
    values(RB, v);
    load(K + 1 < K1 ? 2 * K + 3 : -1, RB);
    xy(v, s1);
    if (out) {
      const int64_t n =
          (int64_t)K * (cnx + 1) * (cny + 1) + (int64_t)(J0 + cj) * (cnx + 1) + I0 + ci;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T acc = s0[c] + T(0.5) * (carry[c] + s1[c]);
        bc[c * cnn + n] = acc;
        if (xc) xc[c * cnn + n] = omega * dc[c * cnn + n] * acc;
        carry[c] = s1[c];
      }
    }
  }
}

// xf += Df P xc: thread per fine node, branch-free over the (up to) 8
// parent nodes: along an axis an even fine index takes its parent with
// weight 1, an odd one both neighbours with weight 1/2.  On the plane grid
// (fnz = 0) the z pair is (0, 0) with weights (1, 0) and ncomp = 2.
template <typename T>
__global__ void __launch_bounds__(256) k_prolong_add(int fnx, int fny, int fnz,
                                                     const T* __restrict__ xc,
                                                     const uint8_t* __restrict__ mask,
                                                     T* __restrict__ xf, int ncomp,
                                                     int64_t cs = 0, int64_t fs = 0) {
  xc += (int64_t)blockIdx.z * cs;  // load case blockIdx.z
  xf += (int64_t)blockIdx.z * fs;
  const int64_t fnn = (int64_t)(fnx + 1) * (fny + 1) * (fnz + 1);
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= fnn) return;
  const int cnx = fnx / 2, cny = fny / 2, cnz = fnz / 2;
  const int64_t cnn = (int64_t)(cnx + 1) * (cny + 1) * (cnz + 1);
  const int fi = (int)(n % (fnx + 1));
  const int64_t rest = n / (fnx + 1);
  const int fj = (int)(rest % (fny + 1));
  const int fk = (int)(rest / (fny + 1));
  const int ix[2] = {fi >> 1, (fi + 1) >> 1};
  const int iy[2] = {fj >> 1, (fj + 1) >> 1};
  const int iz[2] = {fk >> 1, (fk + 1) >> 1};
  const T wx[2] = {(fi & 1) ? T(0.5) : T(1), (fi & 1) ? T(0.5) : T(0)};
  const T wy[2] = {(fj & 1) ? T(0.5) : T(1), (fj & 1) ? T(0.5) : T(0)};
  const T wz[2] = {(fk & 1) ? T(0.5) : T(1), (fk & 1) ? T(0.5) : T(0)};
  int64_t id[8];
  T w[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    id[q] = node_of(cnx, cny, ix[q & 1], iy[(q >> 1) & 1], iz[q >> 2]);
    w[q] = wx[q & 1] * wy[(q >> 1) & 1] * wz[q >> 2];
  }
  const uint8_t m = mask ? mask[n] : 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (c >= ncomp) break;
    const T* x = xc + c * cnn;
    T s = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) s = fma(w[q], x[id[q]], s);
    if (!((m >> c) & 1)) xf[c * fnn + n] += s;
  }
}

// The same interpolation on large 3D grids with the coarse values staged in
// LDS: a workgroup takes a 64 x 16 tile of the fine planes 2K and 2K+1 (one
// fine node per lane and row, rows w, w+4, w+8, w+12 on wavefront w, whole
// rows per load), which interpolate from the coarse planes K and K+1 only.
// It issues its fine loads, stages the 33 x 9 coarse nodes of both planes
// in LDS, and forms each node's sum with the weights and order of
// k_prolong_add, so the results are the same bits.  blockIdx.x: (tile, K)
// with K fastest, in XCD-contiguous order; blockIdx.z: load case.
constexpr int kPzX = 64, kPzY = 16;
constexpr int kPzCX = kPzX / 2 + 1, kPzCY = kPzY / 2 + 1;
constexpr int kPzRows = kPzY / 4;  // rows per wavefront
template <typename T>
__global__ void __launch_bounds__(256) k_prolong_z(int fnx, int fny, int fnz, int gx,
                                                   const T* __restrict__ xc,
                                                   const uint8_t* __restrict__ mask,
                                                   T* __restrict__ xf, int64_t cs, int64_t fs) {
  __shared__ T sx[3][2][kPzCY][kPzCX];
  xc += (int64_t)blockIdx.z * cs;  // load case blockIdx.z
  xf += (int64_t)blockIdx.z * fs;
  const int cnx = fnx / 2, cny = fny / 2, cnz = fnz / 2;
  const int64_t fnn = (int64_t)(fnx + 1) * (fny + 1) * (fnz + 1);
  const int64_t cnn = (int64_t)(cnx + 1) * (cny + 1) * (cnz + 1);
  int bx, by, K;
  {
    const int total = gridDim.x, wg = blockIdx.x;
    const int xcd = wg & 7, pos = wg >> 3, q = total >> 3, r = total & 7;
    const int t = (xcd < r) ? xcd * (q + 1) + pos : r * (q + 1) + (xcd - r) * q + pos;
    K = t % (cnz + 1);
    const int tile = t / (cnz + 1);
    bx = tile % gx;
    by = tile / gx;
  }
  const int cx0 = bx * (kPzX / 2), cy0 = by * (kPzY / 2);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int fi = bx * kPzX + lane;
  // this thread's fine values first: planes 2K + dz, rows w + 4 q4
  T old[2][kPzRows][3];
  uint8_t msk[2][kPzRows];
#pragma unroll
  for (int dz = 0; dz < 2; ++dz)
#pragma unroll
    for (int q4 = 0; q4 < kPzRows; ++q4) {
      const int fj = by * kPzY + w + 4 * q4, fz = 2 * K + dz;
      const bool ok = fi <= fnx && fj <= fny && fz <= fnz;
      const int64_t n = ok ? node_of(fnx, fny, fi, fj, fz) : 0;
      msk[dz][q4] = (ok && mask) ? mask[n] : 0;
#pragma unroll
      for (int c = 0; c < 3; ++c) old[dz][q4][c] = ok ? xf[c * fnn + n] : T(0);
    }
  for (int x = threadIdx.x; x < 3 * 2 * kPzCY * kPzCX; x += 256) {
    const int ci = x % kPzCX, cj = (x / kPzCX) % kPzCY, pz = (x / (kPzCX * kPzCY)) % 2,
              c = x / (2 * kPzCX * kPzCY);
    const int I = cx0 + ci, J = cy0 + cj, Kz = K + pz;
    T val = T(0);
    if (I <= cnx && J <= cny && Kz <= cnz) val = xc[c * cnn + node_of(cnx, cny, I, J, Kz)];
    sx[c][pz][cj][ci] = val;
  }
  __syncthreads();
  if (fi > fnx) return;  // no barrier below
  const int ixl[2] = {(fi >> 1) - cx0, ((fi + 1) >> 1) - cx0};
  const T wx[2] = {(fi & 1) ? T(0.5) : T(1), (fi & 1) ? T(0.5) : T(0)};
#pragma unroll
  for (int dz = 0; dz < 2; ++dz) {
    const int fz = 2 * K + dz;
    if (fz > fnz) break;
    // local coarse planes of fz: {fz >> 1, (fz + 1) >> 1} - K
    const int izl[2] = {(fz >> 1) - K, ((fz + 1) >> 1) - K};
    const T wz[2] = {(fz & 1) ? T(0.5) : T(1), (fz & 1) ? T(0.5) : T(0)};
#pragma unroll
    for (int q4 = 0; q4 < kPzRows; ++q4) {
      const int fj = by * kPzY + w + 4 * q4;
      if (fj > fny) break;
      const int iyl[2] = {(fj >> 1) - cy0, ((fj + 1) >> 1) - cy0};
      const T wy[2] = {(fj & 1) ? T(0.5) : T(1), (fj & 1) ? T(0.5) : T(0)};
      const int64_t n = node_of(fnx, fny, fi, fj, fz);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        T sum = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q)
          sum = fma(wx[q & 1] * wy[(q >> 1) & 1] * wz[q >> 2],
                    sx[c][izl[q >> 2]][iyl[(q >> 1) & 1]][ixl[q & 1]], sum);
        if (!((msk[dz][q4] >> c) & 1)) xf[c * fnn + n] = old[dz][q4][c] + sum;
      }
    }
  }
}

template <typename T>
__global__ void k_jacobi_first(int64_t n3, const T* __restrict__ b, const T* __restrict__ dinv,
                               T omega, T* __restrict__ x, int64_t rs = 0) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ro = (int64_t)blockIdx.z * rs;  // load case blockIdx.z
  if (i < n3) x[ro + i] = omega * dinv[i] * b[ro + i];
}

template <typename T>
__global__ void k_jacobi_update(int64_t n3, const T* __restrict__ b, const T* __restrict__ t,
                                const T* __restrict__ dinv, T omega, T* __restrict__ x,
                                int64_t rs = 0) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ro = (int64_t)blockIdx.z * rs;  // load case blockIdx.z
  if (i < n3) x[ro + i] += omega * dinv[i] * (b[ro + i] - t[ro + i]);
}

// Dense coarsest operator in SoA DOF order (c * nn + node); thread per row.
// One wavefront per row: the row is zeroed (coalesced stores), then lanes
// take the 81 columns of the 27-node neighbourhood (3 components each); an
// entry is the sum, over the elements around the row's node in corner order
// a = 0..7, of the element matrices' entries coupling the two nodes.  A row
// with zero diagonal (a coarse DOF no free fine DOF interpolates from)
// becomes an identity row.  32-bit indices: the coarsest order is at most
// 8192.
__global__ void __launch_bounds__(256) k_assemble_dense(int nx, int ny, int nz,
                                                        const double* __restrict__ Ke,
                                                        double* __restrict__ A) {
  const int nxp = nx + 1, nyp = ny + 1;
  const int nn = nxp * nyp * (nz + 1), ne = nx * ny * nz, nd = 3 * nn;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const bool active = row < nd;  // wave-uniform; every wave reaches the barrier
  double* Ar = A + (int64_t)(active ? row : 0) * nd;
  if (active)
    for (int t = lane; t < nd; t += 64) Ar[t] = 0.0;
  __syncthreads();  // the zeros are stored before the same addresses are rewritten
  if (!active) return;
  const int c = row / nn, n = row % nn;
  const int i = n % nxp, j = (n / nxp) % nyp, k = n / (nxp * nyp);
  for (int l = lane; l < 81; l += 64) {
    const int cc = l / 27, d = l % 27;
    const int bi = i + d % 3 - 1, bj = j + (d / 3) % 3 - 1, bk = k + d / 9 - 1;
    if (bi < 0 || bi > nx || bj < 0 || bj > ny || bk < 0 || bk > nz) continue;
    double acc = 0.0;
    for (int a = 0; a < 8; ++a) {
      const int ex = i - (a & 1), ey = j - ((a >> 1) & 1), ez = k - (a >> 2);
      if (ex < 0 || ex >= nx || ey < 0 || ey >= ny || ez < 0 || ez >= nz) continue;
      const int dx = bi - ex, dy = bj - ey, dz = bk - ez;  // corner of the column node
      if (dx < 0 || dx > 1 || dy < 0 || dy > 1 || dz < 0 || dz > 1) continue;
      const int b = dx + 2 * dy + 4 * dz;
      const int e = ex + nx * (ey + ny * ez);
      acc += Ke[(int64_t)sidx(3 * a + c, 3 * b + cc) * ne + e];
    }
    const int col = cc * nn + bi + nxp * (bj + nyp * bk);
    Ar[col] = (col == row && acc == 0.0) ? 1.0 : acc;
  }
}

// ---- blocked Gauss-Jordan inversion of an SPD matrix (sweep operator) -----
// One block step with pivot block K = [k0, k0+kb) maps
//   A_KK -> P = A_KK^-1,  A_IK -> -A_IK P,  A_KJ -> P A_KJ,
//   A_IJ -> A_IJ - A_IK P A_KJ            (I, J outside K).
// For symmetric A the matrix stays symmetric up to sign: after the blocks
// before k0 are done, A_ij = A_ji when i and j are both below k0 or both at
// or above it, and A_ij = -A_ji otherwise.  Only tiles on or above the
// diagonal are therefore kept: with c_i = A_iK (read from the stored upper
// triangle as A_iK for i < k0, as A_Ki for i beyond K) and T_i = P c_i,
//   A_ij -= s_j T_i . c_j  (s_j = -1 for j < k0, +1 beyond K),
//   A_iK  = -T_i (i < k0),  A_Kj = T_j (j beyond K).
// After the last block the stored upper triangle is A^-1 and the lower
// triangle is filled by transposition.

// 1/x from the hardware reciprocal estimate and two Newton steps.
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

// 16x16 FP64 MFMA tiles over LDS (row stride ld).  Operand lane layout of
// v_mfma_f64_16x16x4f64: A[l%16][l/16], B[l/16][l%16]; accumulator element
// v of lane l is row l/16 + 4v, column l%16.
__device__ __forceinline__ f64x4 mma16(const double* A, int lda, const double* B, int ldb,
                                       f64x4 acc, double sgn_a) {
  const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const double a = sgn_a * A[li * lda + 4 * kk + lk];
    const double b = B[(4 * kk + lk) * ldb + li];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  return acc;
}

__device__ __forceinline__ f64x4 ld16(const double* C, int ldc) {
  const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
  f64x4 x;
#pragma unroll
  for (int v = 0; v < 4; ++v) x[v] = C[(lk + 4 * v) * ldc + li];
  return x;
}

__device__ __forceinline__ void st16(double* C, int ldc, f64x4 x, double sgn) {
  const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
#pragma unroll
  for (int v = 0; v < 4; ++v) C[(lk + 4 * v) * ldc + li] = sgn * x[v];
}

// Lane (16 r + k)'s value of v for every lane of the 16-lane row r (DPP
// row_newbcast).
template <int K>
__device__ __forceinline__ double row_bcast(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x150 + K, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x150 + K, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// One pivot step k of gj16_wave.  The pivot S[k][k] is wave-uniform (lane
// reads), the pivot column S[4 r4 + q][k] comes from lane k of the lane's own
// 16-lane row (row_newbcast), and the pivot row S[k][c] from lane 16 (k/4) + c.
template <int K>
struct Gj16Step {
  static __device__ __forceinline__ void run(double (&x)[4], int c, int r4) {
    constexpr int kq = K & 3, kr = K >> 2;
    const double rk = __shfl(x[kq], kr * 16 + c, 64);  // S[k][c]
    const int plo = __builtin_amdgcn_readlane(__double2loint(x[kq]), kr * 16 + K);
    const int phi = __builtin_amdgcn_readlane(__double2hiint(x[kq]), kr * 16 + K);
    const double piv = recip(__hiloint2double(phi, plo));
    const bool pc = (c == K);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double ck = row_bcast<K>(x[q]);  // S[4 r4 + q][k]
      const double upd = pc ? -ck * piv : fma(-ck * piv, rk, x[q]);
      x[q] = (4 * r4 + q == K) ? (pc ? piv : rk * piv) : upd;
    }
    Gj16Step<K + 1>::run(x, c, r4);
  }
};
template <>
struct Gj16Step<16> {
  static __device__ __forceinline__ void run(double (&)[4], int, int) {}
};

// In-place Gauss-Jordan inversion of a 16x16 block of LDS (row stride ld) by
// one wavefront in registers: lane l holds rows 4(l/16)..4(l/16)+3 of column
// l%16.
__device__ __forceinline__ void gj16_wave(double* S, int ld) {
  const int l = threadIdx.x & 63, c = l & 15, r4 = l >> 4;
  double x[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) x[q] = S[(4 * r4 + q) * ld + c];
  Gj16Step<0>::run(x, c, r4);
#pragma unroll
  for (int q = 0; q < 4; ++q) S[(4 * r4 + q) * ld + c] = x[q];
}

// In-place Gauss-Jordan inversion of the 64x64 block sS (padded with the
// identity beyond the pivot block size) by 256 threads, in four 16-wide
// sub-steps J over the 4 x 4 grid of 16x16 blocks: Q = S_JJ^-1 (one
// wavefront), then for the other blocks o, o': R_o = Q S_Jo, T_o = S_oJ Q,
// S_oo' -= S_oJ R_o', S_Jo = R_o, S_oJ = -T_o, all on FP64 MFMA.
__device__ __forceinline__ void gj64_block(double (*sS)[kGJBlock + 1]) {
  constexpr int ld = kGJBlock + 1;
  const int w = threadIdx.x >> 6;
  const f64x4 zero = {0.0, 0.0, 0.0, 0.0};
  for (int j = 0; j < 4; ++j) {
    const int J0 = 16 * j;
    if (w == 0) gj16_wave(&sS[J0][J0], ld);
    __syncthreads();
    const int ob = 16 * (w < j ? w : w + 1);  // wave w < 3: the w-th other block
    f64x4 T = zero, R = zero;
    if (w < 3) {
      T = mma16(&sS[ob][J0], ld, &sS[J0][J0], ld, zero, 1.0);
      R = mma16(&sS[J0][J0], ld, &sS[J0][ob], ld, zero, 1.0);
      // no barrier before this store: S_J,ob is read only by this wave
      st16(&sS[J0][ob], ld, R, 1.0);
    }
    __syncthreads();
    for (int t = w; t < 9; t += 4) {
      const int q1 = t / 3, q2 = t % 3;
      const int o1 = 16 * (q1 < j ? q1 : q1 + 1), o2 = 16 * (q2 < j ? q2 : q2 + 1);
      f64x4 c = ld16(&sS[o1][o2], ld);
      c = mma16(&sS[o1][J0], ld, &sS[J0][o2], ld, c, -1.0);
      st16(&sS[o1][o2], ld, c, 1.0);
    }
    __syncthreads();
    if (w < 3) st16(&sS[ob][J0], ld, T, -1.0);
    __syncthreads();
  }
}

// Workgroup 0: pivot inverse of the first block, Pb = A_00^-1 (kb x kb).
// The others copy the first step's panel Cb[p][i] = A[p][i] (p < kb: the
// stored first block row), 2048 entries each.
__global__ void __launch_bounds__(256) k_gj_pivot_first(int n, int kb,
                                                        const double* __restrict__ A,
                                                        double* __restrict__ Pb,
                                                        double* __restrict__ Cb) {
  __shared__ double sS[kGJBlock][kGJBlock + 1];
  if (blockIdx.x > 0) {
    const int64_t base = (int64_t)(blockIdx.x - 1) * 2048, total = (int64_t)kb * n;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int64_t x = base + threadIdx.x + 256 * r;
      if (x < total) Cb[x] = A[x];
    }
    return;
  }
  for (int x = threadIdx.x; x < kGJBlock * kGJBlock; x += 256) {
    const int r = x / 64, c = x % 64;
    sS[r][c] = (r < kb && c < kb) ? A[(int64_t)r * n + c] : (r == c ? 1.0 : 0.0);
  }
  __syncthreads();
  gj64_block(sS);
  for (int x = threadIdx.x; x < kb * kb; x += 256) Pb[x] = sS[x / kb][x % kb];
}

// 64x64 FP64 tile in LDS, row p, column i at p * 64 + (i ^ 8 (p & 3)).  An
// MFMA operand read (lanes l: row 4kk + l/16, 16 consecutive columns) then
// spreads its four 16-lane groups over both bank halves, two groups each:
// two passes, the minimum for 64 doubles, without padding (two tiles fill
// the 64 KB a workgroup may hold).
__device__ __forceinline__ int swz(int p, int i) { return p * 64 + (i ^ ((p & 3) << 3)); }

// The cross part of a block step for large orders, one workgroup per block
// row O: A_KK = Pc for O = K; otherwise T_O = c_O Pc into Tb[q][O0 + i], the
// new cross entries A_OK = -T_O (O < K) or A_KO = T_O (O > K), and for
// O = K+1 the next panel's rows of K.  k_gj_step<true> then forms the tiles.
__global__ void __launch_bounds__(256) k_gj_cross(int n, int k0, int kb, double* __restrict__ A,
                                                  const double* __restrict__ Pc,
                                                  const double* __restrict__ Cc,
                                                  double* __restrict__ Cn,
                                                  double* __restrict__ Tb) {
  __shared__ double sm[2 * kGJBlock * kGJBlock];
  double* sP = sm;
  double* sX = sm + kGJBlock * kGJBlock;
  const int K = k0 / kGJBlock, O = blockIdx.x;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  if (O == K) {
    for (int x = tid; x < kb * kb; x += 256)
      A[(int64_t)(k0 + x / kb) * n + k0 + x % kb] = Pc[x];
    return;
  }
  const int O0 = O * kGJBlock;
  const int orows = (n - O0 < kGJBlock) ? (n - O0) : kGJBlock;
  double pv[16], xv[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int x = tid + 256 * r, a = x >> 6, b = x & 63;
    pv[r] = (a < kb && b < kb) ? Pc[a * kb + b] : 0.0;
    xv[r] = (a < kb && b < orows) ? Cc[(int64_t)a * n + O0 + b] : 0.0;
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int x = tid + 256 * r, a = x >> 6, b = x & 63;
    sP[swz(a, b)] = pv[r];
    sX[swz(a, b)] = xv[r];
  }
  __syncthreads();
  f64x4 tacc[4];
#pragma unroll
  for (int jb = 0; jb < 4; ++jb) tacc[jb] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
    const int p = 4 * kk + lk;
    const double a = sX[swz(p, 16 * w + li)];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
      tacc[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, sP[swz(p, 16 * jb + li)], tacc[jb], 0, 0, 0);
  }
  __syncthreads();
#pragma unroll
  for (int jb = 0; jb < 4; ++jb)
#pragma unroll
    for (int v = 0; v < 4; ++v) sX[swz(16 * jb + li, 16 * w + lk + 4 * v)] = tacc[jb][v];
  if (O < K) {
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * w + lk + 4 * v, q = 16 * jb + li;
        if (i < orows && q < kb) A[(int64_t)(O0 + i) * n + k0 + q] = -tacc[jb][v];
      }
  } else if (O == K + 1) {
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * w + lk + 4 * v, q = 16 * jb + li;
        if (i < orows && q < kb) Cn[(int64_t)i * n + k0 + q] = tacc[jb][v];
      }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 16; ++r) {  // Tb[q][O0 + i] and, beyond K, A[k0 + q][O0 + i]
    const int x = tid + 256 * r, q = x >> 6, i = x & 63;
    if (q < kb && i < orows) {
      const double t = sX[swz(q, i)];
      Tb[(int64_t)q * n + O0 + i] = t;
      if (O > K) A[(int64_t)(k0 + q) * n + O0 + i] = t;
    }
  }
}

// One block step in one launch, one workgroup per upper tile (bi <= bj).
// The step reads the pivot inverse Pc = A_KK^-1 and the panel Cc[p][i] =
// c_i[p] (c_i = A_iK before the step, taken from the stored upper triangle)
// and writes the next step's Pn and Cn, so no workgroup reads what another
// writes:
//   tile (K, K):        A_KK = Pc;
//   tile in row/col K:  T_O = c_O Pc for the other block O, and the new cross
//                       entries A_OK = -T_O (O < K) or A_KO = T_O (O > K);
//   other tiles (I, J): T_I = c_I Pc, A_IJ -= s_J T_I c_J^T (s_J = -1 for
//                       J < K, +1 beyond), all on FP64 MFMA.
// Entries that become the next panel (block column K+1 above the diagonal,
// block row K+1 right of it, and A_{K,K+1}) are also written to Cn.
// Workgroup 0 takes tile (K+1, K+1) and inverts the updated tile into Pn.
// PRE_T: k_gj_cross has already formed T_O (into Tb[q][i]) and the row/col K
// entries for this step; the tiles read T_I instead of forming it, and the
// row/col K workgroups have nothing to do (large orders, where the repeated
// T products cost more than the second launch).
template <bool PRE_T>
__global__ void __launch_bounds__(256) k_gj_step(int n, int k0, int kb, int nb,
                                                 double* __restrict__ A,
                                                 const double* __restrict__ Pc,
                                                 double* __restrict__ Pn,
                                                 const double* __restrict__ Cc,
                                                 double* __restrict__ Cn,
                                                 const double* __restrict__ Tb) {
  __shared__ double sm[2 * kGJBlock * kGJBlock];
  double* sP = sm;                        // Pc [p][q], later c_J [p][j]
  double* sX = sm + kGJBlock * kGJBlock;  // c_O [p][i], later T [q][i]
  const int K = k0 / kGJBlock;
  const bool has_next = K + 1 < nb;
  int bi, bj;
  {
    int t = blockIdx.x;
    if (has_next) {  // workgroup 0: (K+1, K+1); the rest row-major, skipping it
      if (t == 0) {
        t = (K + 1) * nb - ((K + 1) * K) / 2;
      } else {
        --t;
        const int nxt = (K + 1) * nb - ((K + 1) * K) / 2;
        if (t >= nxt) ++t;
      }
    }
    bi = 0;
    while (t >= nb - bi) { t -= nb - bi; ++bi; }
    bj = bi + t;
  }
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const bool cross = bi == K || bj == K;
  if (PRE_T && cross) return;
  if (bi == K && bj == K) {
    for (int x = tid; x < kb * kb; x += 256)
      A[(int64_t)(k0 + x / kb) * n + k0 + x % kb] = Pc[x];
    return;
  }
  const int O = cross ? (bi == K ? bj : bi) : bi;  // the block whose T is formed
  const int O0 = O * kGJBlock, J0 = bj * kGJBlock, I0 = bi * kGJBlock;
  const int orows = (n - O0 < kGJBlock) ? (n - O0) : kGJBlock;
  // every global load in flight before the first LDS store
  double pv[16], xv[16], cj[16];
  f64x4 acc[4];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int x = tid + 256 * r, a = x >> 6, b = x & 63;
    // PRE_T: xv holds T_I as [q][i] instead of c_O as [p][i]
    pv[r] = (!PRE_T && a < kb && b < kb) ? Pc[a * kb + b] : 0.0;
    xv[r] = (a < kb && b < orows) ? (PRE_T ? Tb : Cc)[(int64_t)a * n + O0 + b] : 0.0;
    cj[r] = (!cross && a < kb && J0 + b < n) ? Cc[(int64_t)a * n + J0 + b] : 0.0;
  }
#pragma unroll
  for (int jb = 0; jb < 4; ++jb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = I0 + 16 * w + lk + 4 * v, j = J0 + 16 * jb + li;
      acc[jb][v] = (!cross && i < n && j < n) ? A[(int64_t)i * n + j] : 0.0;
    }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int x = tid + 256 * r, a = x >> 6, b = x & 63;
    if (!PRE_T) sP[swz(a, b)] = pv[r];
    sX[swz(a, b)] = xv[r];
  }
  if (!PRE_T) {
  __syncthreads();
  // T[16w + i][16jb + j] = sum_p c[16w + i][p] P[p][16jb + j]
  f64x4 tacc[4];
#pragma unroll
  for (int jb = 0; jb < 4; ++jb) tacc[jb] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
    const int p = 4 * kk + lk;
    const double a = sX[swz(p, 16 * w + li)];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
      tacc[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, sP[swz(p, 16 * jb + li)], tacc[jb], 0, 0, 0);
  }
  __syncthreads();
  // tacc[jb][v] = T[16w + lk + 4v][16jb + li]; stage T as [q][i]
#pragma unroll
  for (int jb = 0; jb < 4; ++jb)
#pragma unroll
    for (int v = 0; v < 4; ++v) sX[swz(16 * jb + li, 16 * w + lk + 4 * v)] = tacc[jb][v];
  if (cross) {  // only without PRE_T
    if (O < K) {  // A[O0 + i][k0 + q] = -T[i][q], coalesced along q
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * w + lk + 4 * v, q = 16 * jb + li;
          if (i < orows && q < kb) A[(int64_t)(O0 + i) * n + k0 + q] = -tacc[jb][v];
        }
      return;
    }
    if (O == K + 1) {  // next panel, rows of K: Cn[i][k0 + q] = T[i][q]
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * w + lk + 4 * v, q = 16 * jb + li;
          if (i < orows && q < kb) Cn[(int64_t)i * n + k0 + q] = tacc[jb][v];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) {  // A[k0 + q][O0 + i] = T[i][q], coalesced along i
      const int x = tid + 256 * r, q = x >> 6, i = x & 63;
      if (q < kb && i < orows) A[(int64_t)(k0 + q) * n + O0 + i] = sX[swz(q, i)];
    }
    return;
  }
  }  // !PRE_T: T formed and staged as [q][i] in sX
  // tile: c_J as [p][j] replaces P
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int x = tid + 256 * r, a = x >> 6, b = x & 63;
    sP[swz(a, b)] = cj[r];
  }
  __syncthreads();
  const double ns = (J0 < k0) ? 1.0 : -1.0;  // -s_J
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
    const int p = 4 * kk + lk;
    const double a = ns * sX[swz(p, 16 * w + li)];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
      acc[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, sP[swz(p, 16 * jb + li)], acc[jb], 0, 0, 0);
  }
  const bool next_col = bj == K + 1 && bi != K + 1, next_row = bi == K + 1 && bj != K + 1;
#pragma unroll
  for (int jb = 0; jb < 4; ++jb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = I0 + 16 * w + lk + 4 * v, j = J0 + 16 * jb + li;
      if (i < n && j < n) {
        A[(int64_t)i * n + j] = acc[jb][v];
        // row K+1 of the next panel: Cn[p][j] = A[(K+1)0 + p][j]
        if (next_row) Cn[(int64_t)(i - I0) * n + j] = acc[jb][v];
      }
    }
  if (next_col) {  // column K+1: Cn[p][i] = A[i][J0 + p], staged to be coalesced along i
    __syncthreads();
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int v = 0; v < 4; ++v) sX[swz(16 * jb + li, 16 * w + lk + 4 * v)] = acc[jb][v];
    __syncthreads();
    const int ncol = (n - J0 < kGJBlock) ? (n - J0) : kGJBlock;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int x = tid + 256 * r, p = x >> 6, i = x & 63;
      if (p < ncol && I0 + i < n) Cn[(int64_t)p * n + I0 + i] = sX[swz(p, i)];
    }
    return;
  }
  if (blockIdx.x != 0 || !has_next) return;
  // next pivot block: the tile just updated, identity beyond the matrix
  double (*sS)[kGJBlock + 1] = reinterpret_cast<double (*)[kGJBlock + 1]>(sm);
  const int kbn = (n - I0 < kGJBlock) ? (n - I0) : kGJBlock;
  __syncthreads();
#pragma unroll
  for (int jb = 0; jb < 4; ++jb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ti = 16 * w + lk + 4 * v, tj = 16 * jb + li;
      sS[ti][tj] = (ti < kbn && tj < kbn) ? acc[jb][v] : (ti == tj ? 1.0 : 0.0);
    }
  __syncthreads();
  gj64_block(sS);
  for (int x = threadIdx.x; x < kbn * kbn; x += 256) Pn[x] = sS[x / kbn][x % kbn];
}

// Lower tiles (bi > bj) <- transpose of the upper tiles.
__global__ void __launch_bounds__(256) k_gj_mirror(int n, double* __restrict__ A) {
  __shared__ double sX[kGJBlock][kGJBlock + 1];
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bi <= bj) return;
  const int I0 = bi * kGJBlock, J0 = bj * kGJBlock, tid = threadIdx.x;
  for (int x = tid; x < kGJBlock * kGJBlock; x += 256) {  // read A[J0 + r][I0 + c]
    const int r = x / 64, c = x % 64;
    if (J0 + r < n && I0 + c < n) sX[r][c] = A[(int64_t)(J0 + r) * n + I0 + c];
  }
  __syncthreads();
  for (int x = tid; x < kGJBlock * kGJBlock; x += 256) {  // write A[I0 + r][J0 + c]
    const int r = x / 64, c = x % 64;
    if (I0 + r < n && J0 + c < n) A[(int64_t)(I0 + r) * n + J0 + c] = sX[c][r];
  }
}

// y = A x for the dense (symmetric) inverse; one wavefront per row.
template <typename TX, typename TY>
__global__ void __launch_bounds__(256) k_gemv(int n, const double* __restrict__ A,
                                              const TX* __restrict__ x, TY* __restrict__ y,
                                              int64_t rs = 0) {
  x += (int64_t)blockIdx.z * rs;  // load case blockIdx.z
  y += (int64_t)blockIdx.z * rs;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const double* a = A + (int64_t)row * n;
  // four independent accumulators: eight loads in flight per lane
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
  int j = lane;
  for (; j + 192 < n; j += 256) {
    acc0 = fma(a[j], (double)x[j], acc0);
    acc1 = fma(a[j + 64], (double)x[j + 64], acc1);
    acc2 = fma(a[j + 128], (double)x[j + 128], acc2);
    acc3 = fma(a[j + 192], (double)x[j + 192], acc3);
  }
  for (; j < n; j += 64) acc0 = fma(a[j], (double)x[j], acc0);
  double acc = (acc0 + acc1) + (acc2 + acc3);
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) y[row] = (TY)acc;
}

}  // namespace

void launch_galerkin_from_fine(const Grid& coarse, const double* KE, const double* Mc,
                               const double* E, const uint8_t* mask, uint8_t* eflag, int* list,
                               int* count, double* Kc, double* Kcomp, int cap, hipStream_t s,
                               bool all) {
  if (all)
    k_galerkin_fast<<<nblk(coarse.ne, 64), 256, 0, s>>>(coarse.nx, coarse.ny, coarse.nz, Mc, E,
                                                        Kc);
  k_zero_int<<<1, 1, 0, s>>>(count);
  k_parent_flags<<<nblk(coarse.ne, 256), 256, 0, s>>>(coarse.nx, coarse.ny, coarse.nz, mask, eflag,
                                                       list, count);
  const unsigned grid = (unsigned)std::min<int64_t>(coarse.ne, 2048);
  k_galerkin_lds<1><<<grid, 256, 0, s>>>(coarse.nx, coarse.ny, coarse.nz, KE, E, mask, list,
                                            count, nullptr, Kc, Kcomp, cap);
}

void launch_galerkin_l2_from_fine(const Grid& l2, const double* N2, const double* Mc,
                                  const double* E, const uint8_t* eflag1, int* list2, int* count2,
                                  const double* K1, double* K2, hipStream_t s) {
  k_galerkin_fast2<<<nblk(l2.ne, 64), 256, 0, s>>>(l2.nx, l2.ny, l2.nz, N2, E, K2);
  k_zero_int<<<1, 1, 0, s>>>(count2);
  k_parent_flags2<<<nblk(l2.ne, 256), 256, 0, s>>>(l2.nx, l2.ny, l2.nz, eflag1, list2, count2);
  const unsigned grid = (unsigned)std::min<int64_t>(l2.ne, 2048);
  k_galerkin_lds<2><<<grid, 256, 0, s>>>(l2.nx, l2.ny, l2.nz, Mc, E, eflag1, list2, count2, K1,
                                         K2, nullptr, 0);
}

void launch_diag_l1(const Grid& g, const double* Ke, const double* Mc, const double* E,
                    const uint8_t* eflag, double* dinv, float* dinv32, hipStream_t s) {
  k_diag_l1<<<nblk(g.nn, 256), 256, 0, s>>>(g.nx, g.ny, g.nz, Ke, Mc, E, eflag, dinv, dinv32);
}

void launch_galerkin_from_coarse(const Grid& coarse, const double* Kf, double* Kc, hipStream_t s) {
  const int64_t groups = (int64_t)((coarse.nx + 7) / 8) * coarse.ny * coarse.nz;
  if (groups >= 256) {
    // 57.6 KB of LDS per workgroup: two per CU, 512 resident
    const unsigned grid = (unsigned)std::min<int64_t>(groups, 512);
    k_galerkin_row8<<<grid, 256, 0, s>>>(coarse.nx, coarse.ny, coarse.nz, Kf, Kc);
    return;
  }
  // fewer groups than CUs: one parent per workgroup keeps more of the chip busy
  const unsigned grid = (unsigned)std::min<int64_t>(coarse.ne, 4096);
  k_galerkin_lds<0><<<grid, 256, 0, s>>>(coarse.nx, coarse.ny, coarse.nz, nullptr, nullptr,
                                             nullptr, nullptr, nullptr, Kf, Kc, nullptr, 0);
}

void launch_apply_elemmat(const Grid& g, const double* Ke, const double* v, double* y,
                          hipStream_t s) {
  k_apply_elemmat<double><<<nblk(g.nn, 64), 512, 0, s>>>(g.nx, g.ny, g.nz, Ke, v, y, nullptr,
                                                         nullptr, 0.0);
}

void launch_apply_elemmat_jacobi(const Grid& g, const double* Ke, const double* v, const double* b,
                                 const double* dinv, double omega, double* out, hipStream_t s) {
  k_apply_elemmat<double><<<nblk(g.nn, 64), 512, 0, s>>>(g.nx, g.ny, g.nz, Ke, v, out, b, dinv,
                                                         omega);
}

void launch_apply_elemmat_f32(const Grid& g, const float* Ke, const float* v, float* y,
                              hipStream_t s, int nr) {
  k_apply_elemmat<float, float><<<dim3(nblk(g.nn, 64), 1, nr), 512, 0, s>>>(
      g.nx, g.ny, g.nz, Ke, v, y, nullptr, nullptr, 0.0f, 3 * g.nn);
}

// nr load cases in lock step: vectors [nr][3 nn], element products [nr][24][ne]
constexpr int64_t kL1All3 = 200000;
template <typename T>
void l1_apply(const Grid& g, const double* Ke, const double* Kcomp, int cap, const T* Bw,
              const T* Ef, const uint8_t* eflag, const int* list, const int* count, int nflag,
              const T* v, T* Y, T* y, hipStream_t s, const T* jb = nullptr,
              const T* jd = nullptr, T omega = 0, int nr = 1) {
  // nflag: the flagged-parent count, known to the host after setup
  // one thread per element from kL1All3 elements up (256x128x128, level 1:
  // 41.6 -> 33.2 us per call in FP32, 60 -> 49.5 us in FP64); per (element,
  // component) below, where the 96x48x48 loop's level 1 measured faster
  const int all3 = g.ne >= kL1All3 ? 1 : 0;
  const int nbe = (int)nblk(g.ne, all3 ? 3 * 256 : 256);
  const int nbm = nflag > 0 ? 2 * (int)std::min<int64_t>(nblk(nflag, 16), 1024) : 0;
  const int64_t rs = 3 * g.nn, Ys = 24 * g.ne;
  k_l1_elem<T><<<dim3(nbe + nbm, 3, nr), 256, 0, s>>>(g.nx, g.ny, g.nz, Ke, Bw, Ef, eflag, v, Y,
                                                      nbe, Kcomp, cap, list, nflag, all3, rs,
                                                      Ys);
  k_l1_gather<T><<<dim3(nblk(g.nn, 256), 1, nr), 256, 0, s>>>(g.nx, g.ny, g.nz, Y, y, jb, jd,
                                                              omega, rs, Ys);
}

void launch_apply_l1_jacobi(const Grid& g, const double* Ke, const double* Kcomp, int cap,
                            const double* Bw, const double* Ef, const uint8_t* eflag,
                            const int* list, const int* count, int nflag, double* x, double* Y,
                            const double* b, const double* dinv, double omega, hipStream_t s) {
  l1_apply<double>(g, Ke, Kcomp, cap, Bw, Ef, eflag, list, count, nflag, x, Y, x, s, b, dinv,
                   omega);
}

void launch_apply_l1(const Grid& g, const double* Ke, const double* Kcomp, int cap,
                     const double* Bw, const double* Ef, const uint8_t* eflag, const int* list,
                     const int* count, int nflag, const double* v, double* Y, double* y,
                     hipStream_t s) {
  l1_apply<double>(g, Ke, Kcomp, cap, Bw, Ef, eflag, list, count, nflag, v, Y, y, s);
}

void launch_apply_l1_jacobi_f32(const Grid& g, const double* Ke, const double* Kcomp, int cap,
                                const float* Bw, const float* Ef, const uint8_t* eflag,
                                const int* list, const int* count, int nflag, float* x, float* Y,
                                const float* b, const float* dinv, float omega, hipStream_t s,
                                int nr) {
  l1_apply<float>(g, Ke, Kcomp, cap, Bw, Ef, eflag, list, count, nflag, x, Y, x, s, b, dinv,
                  omega, nr);
}

// 3D restriction launch: one workgroup per (tile, chunk of coarse planes,
// case).  Used from kRsMinNodes coarse nodes up; on smaller grids, where a
// launch is a few microseconds either way, the per-node kernel measured
// faster than the separable form (256x128x128, FP32, as one workgroup per
// coarse plane: fine level 90 -> 68 us, second level 13.1 -> 11.0 us, third
// to fifth level 6.1/5.2/4.7 -> 8.2/6.9/5.2).  As a z-march the fine level
// takes 79.5 us (FP64) and 39.1 us (FP32).
constexpr int64_t kRsMinNodes = 100000;
template <typename T>
static void restrict_z(const Grid& coarse, const T* bf, const T* tf, const uint8_t* mask, T* bc,
                       const T* dc, T omega, T* xc, hipStream_t s, int nr, int64_t fs,
                       int64_t cs) {
  const int gx = (coarse.nx + 1 + kRsCI - 1) / kRsCI;
  const int gy = (coarse.ny + 1 + kRsCJ - 1) / kRsCJ;
  // z-march in chunks sized by the device's resident workgroups (one per CU
  // in FP64, two in FP32; 256x128x128 fine level: 79.5 and 39.1 us, three
  // per CU in FP32 46.3 us).  A chunk of t coarse planes reads 2 t + 1 fine
  // planes, and the launch takes about ceil(workgroups / slots) rounds of
  // them: the chunk length with the fewest fine-plane reads in sequence is
  // taken (one round where the tiles fit; results do not depend on it)
  static const int slots = [] {
    int dev = 0, n = 0, per_cu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_restrict_zm<T>,
                                                        64 * kRmWaves, 0);
    return (n > 0 && per_cu > 0) ? n * per_cu : 256;
  }();
  const int planes = coarse.nz + 1, tiles = gx * gy;
  int tk = planes;
  int64_t best = -1;
  for (int n = 1; n <= planes; ++n) {
    const int t = (planes + n - 1) / n;
    const int64_t chunks = (planes + t - 1) / t;
    const int64_t cost = ((int64_t)tiles * chunks + slots - 1) / slots * (2 * t + 1);
    if (best < 0 || cost < best) {
      best = cost;
      tk = t;
    }
  }
  const int gz = (planes + tk - 1) / tk;
  k_restrict_zm<T><<<dim3((unsigned)(tiles * gz), 1, (unsigned)nr), 64 * kRmWaves, 0, s>>>(
      coarse.nx, coarse.ny, coarse.nz, gx, gy, tk, bf, tf, mask, bc, dc, omega, xc, fs, cs);
}

void launch_apply_l1_f32(const Grid& g, const double* Ke, const double* Kcomp, int cap,
                         const float* Bw, const float* Ef, const uint8_t* eflag, const int* list,
                         const int* count, int nflag, const float* v, float* Y, float* y,
                         hipStream_t s, int nr) {
  l1_apply<float>(g, Ke, Kcomp, cap, Bw, Ef, eflag, list, count, nflag, v, Y, y, s, nullptr,
                  nullptr, 0.0f, nr);
}

void launch_apply_elemmat_jacobi_f32(const Grid& g, const float* Ke, const float* v,
                                     const float* b, const float* dinv, float omega, float* out,
                                     hipStream_t s, int nr) {
  k_apply_elemmat<float, float><<<dim3(nblk(g.nn, 64), 1, nr), 512, 0, s>>>(
      g.nx, g.ny, g.nz, Ke, v, out, b, dinv, omega, 3 * g.nn);
}

void launch_restrict_jacobi_f32(const Grid& coarse, const float* bf, const float* tf,
                                const uint8_t* mask, float* bc, const float* dinv_c, float omega,
                                float* xc, hipStream_t s, int nr) {
  const int64_t fnn = (int64_t)(2 * coarse.nx + 1) * (2 * coarse.ny + 1) * (2 * coarse.nz + 1);
  if (coarse.nz > 0 && coarse.nn >= kRsMinNodes) {
    restrict_z<float>(coarse, bf, tf, mask, bc, dinv_c, omega, xc, s, nr, 3 * fnn, 3 * coarse.nn);
    return;
  }
  k_restrict<float><<<dim3(nblk(coarse.nn, 64), 3, nr), 192, 0, s>>>(
      coarse.nx, coarse.ny, coarse.nz, bf, tf, mask, bc, dinv_c, omega, xc, 3 * fnn,
      3 * coarse.nn);
}

void launch_restrict_f32(const Grid& coarse, const float* bf, const float* tf,
                         const uint8_t* mask, float* bc, hipStream_t s, int nr) {
  const int64_t fnn = (int64_t)(2 * coarse.nx + 1) * (2 * coarse.ny + 1) * (2 * coarse.nz + 1);
  if (coarse.nz > 0 && coarse.nn >= kRsMinNodes) {
    restrict_z<float>(coarse, bf, tf, mask, bc, nullptr, 0.0f, nullptr, s, nr, 3 * fnn,
                      3 * coarse.nn);
    return;
  }
  k_restrict<float><<<dim3(nblk(coarse.nn, 64), 3, nr), 192, 0, s>>>(
      coarse.nx, coarse.ny, coarse.nz, bf, tf, mask, bc, nullptr, 0.0f, nullptr, 3 * fnn,
      3 * coarse.nn);
}

// Interpolation with the coarse values in LDS on 3D grids from kPzMinNodes
// fine nodes up (256x128x128 fine level: 87.5 -> 61 us FP64, 39 -> 36 us
// FP32; on the smaller levels the per-node kernel's few microseconds stand).
constexpr int64_t kPzMinNodes = 1000000;
template <typename T>
static void prolong_z(const Grid& fine, const T* xc, const uint8_t* mask, T* xf, hipStream_t s,
                      int nr, int64_t cs, int64_t fs) {
  const int gx = (fine.nx + 1 + kPzX - 1) / kPzX, gy = (fine.ny + 1 + kPzY - 1) / kPzY;
  k_prolong_z<T><<<dim3((unsigned)(gx * gy * (fine.nz / 2 + 1)), 1, (unsigned)nr), 256, 0, s>>>(
      fine.nx, fine.ny, fine.nz, gx, xc, mask, xf, cs, fs);
}

void launch_prolong_add_f32(const Grid& fine, const float* xc, const uint8_t* mask, float* xf,
                            hipStream_t s, int nr) {
  const int64_t cnn = (int64_t)(fine.nx / 2 + 1) * (fine.ny / 2 + 1) * (fine.nz / 2 + 1);
  if (fine.nz > 0 && fine.nn >= kPzMinNodes) {
    prolong_z<float>(fine, xc, mask, xf, s, nr, 3 * cnn, 3 * fine.nn);
    return;
  }
  k_prolong_add<float><<<dim3(nblk(fine.nn, 256), 1, nr), 256, 0, s>>>(
      fine.nx, fine.ny, fine.nz, xc, mask, xf, 3, 3 * cnn, 3 * fine.nn);
}

void launch_jacobi_first_f32(int64_t n3, const float* b, const float* dinv, float omega, float* x,
                             hipStream_t s, int nr) {
  k_jacobi_first<float><<<dim3(nblk(n3, 256), 1, nr), 256, 0, s>>>(n3, b, dinv, omega, x, n3);
}

void launch_jacobi_update_f32(int64_t n3, const float* b, const float* t, const float* dinv,
                              float omega, float* x, hipStream_t s, int nr) {
  k_jacobi_update<float><<<dim3(nblk(n3, 256), 1, nr), 256, 0, s>>>(n3, b, t, dinv, omega, x, n3);
}

void launch_gemv_f32(int n, const double* A, const float* x, float* y, hipStream_t s, int nr) {
  k_gemv<float, float><<<dim3(nblk(n, 4), 1, nr), 256, 0, s>>>(n, A, x, y, n);
}

void launch_diag_elemmat(const Grid& g, const double* Ke, double* dinv, float* dinv32,
                         hipStream_t s) {
  k_diag_elemmat<<<nblk(g.nn, 256), 256, 0, s>>>(g.nx, g.ny, g.nz, Ke, dinv, dinv32);
}

void launch_restrict(const Grid& coarse, const double* bf, const double* tf, const uint8_t* mask,
                     double* bc, hipStream_t s, int ncomp) {
  if (coarse.nz > 0 && ncomp == 3 && coarse.nn >= kRsMinNodes) {
    restrict_z<double>(coarse, bf, tf, mask, bc, nullptr, 0.0, nullptr, s, 1, 0, 0);
    return;
  }
  k_restrict<double><<<dim3(nblk(coarse.nn, 64), ncomp), 192, 0, s>>>(coarse.nx, coarse.ny, coarse.nz,
                                                                  bf, tf, mask, bc, nullptr, 0.0,
                                                                  nullptr);
}

void launch_restrict_jacobi(const Grid& coarse, const double* bf, const double* tf,
                            const uint8_t* mask, double* bc, const double* dinv_c, double omega,
                            double* xc, hipStream_t s) {
  if (coarse.nz > 0 && coarse.nn >= kRsMinNodes) {
    restrict_z<double>(coarse, bf, tf, mask, bc, dinv_c, omega, xc, s, 1, 0, 0);
    return;
  }
  k_restrict<double><<<dim3(nblk(coarse.nn, 64), 3), 192, 0, s>>>(coarse.nx, coarse.ny, coarse.nz,
                                                                  bf, tf, mask, bc, dinv_c, omega,
                                                                  xc);
}

void launch_prolong_add(const Grid& fine, const double* xc, const uint8_t* mask, double* xf,
                        hipStream_t s, int ncomp) {
  if (fine.nz > 0 && ncomp == 3 && fine.nn >= kPzMinNodes) {
    prolong_z<double>(fine, xc, mask, xf, s, 1, 0, 0);
    return;
  }
  k_prolong_add<double><<<nblk(fine.nn, 256), 256, 0, s>>>(fine.nx, fine.ny, fine.nz, xc, mask,
                                                           xf, ncomp);
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
  k_assemble_dense<<<(unsigned)((3 * g.nn + 3) / 4), 256, 0, s>>>(g.nx, g.ny, g.nz, Ke, A);
}

void launch_gj_invert(int n, double* A, double* P, double* T, double* C, double* Tb,
                      hipStream_t s) {
  const int nb = (n + kGJBlock - 1) / kGJBlock;
  const unsigned n_upper = (unsigned)(nb * (nb + 1) / 2);
  // pivot inverses and panels alternate between two buffers each
  double* Pb[2] = {P, P + kGJBlock * kGJBlock};
  double* Cb[2] = {C, T};
  // beyond 40 block rows the repeated T products of the one-launch step cost
  // more than a separate cross launch (measured: 32 us per step at 30 block
  // rows in one launch; 73 vs 61 us per step at 65)
  const bool split = nb > 40;
  const int kb0 = std::min(n, kGJBlock);
  k_gj_pivot_first<<<(unsigned)(1 + ((int64_t)kb0 * n + 2047) / 2048), 256, 0, s>>>(n, kb0, A,
                                                                                  Pb[0], Cb[0]);
  int step = 0;
  for (int k0 = 0; k0 < n; k0 += kGJBlock, ++step) {
    const int kb = std::min(kGJBlock, n - k0);
    if (split) {
      k_gj_cross<<<nb, 256, 0, s>>>(n, k0, kb, A, Pb[step & 1], Cb[step & 1],
                                    Cb[(step + 1) & 1], Tb);
      k_gj_step<true><<<n_upper, 256, 0, s>>>(n, k0, kb, nb, A, Pb[step & 1],
                                              Pb[(step + 1) & 1], Cb[step & 1],
                                              Cb[(step + 1) & 1], Tb);
    } else {
      k_gj_step<false><<<n_upper, 256, 0, s>>>(n, k0, kb, nb, A, Pb[step & 1],
                                               Pb[(step + 1) & 1], Cb[step & 1],
                                               Cb[(step + 1) & 1], nullptr);
    }
  }
  k_gj_mirror<<<dim3(nb, nb), 256, 0, s>>>(n, A);
}

void launch_gemv(int n, const double* A, const double* x, double* y, hipStream_t s) {
  k_gemv<double, double><<<nblk(n, 4), 256, 0, s>>>(n, A, x, y);
}

}  // namespace aarmr
