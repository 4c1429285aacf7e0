// Fine-grid stiffness product y = A v (the eq. 7 operator) as a z-marching,
// reflection-blocked element-by-element kernel for gfx950.
//
// Element stiffness in the Walsh basis.  Number the 8 corners of a unit
// hexahedron a = dx + 2 dy + 4 dz and let W be the 8x8 Walsh matrix
// W[k][a] = (-1)^popcount(k & a).  The reflection symmetries of the
// isotropic unit cube make W KE W^T / 8 (per displacement component) sparse:
// index 0 (translations) is null and the rest splits into blocks of at most
// three entries with eight distinct constants (checked on the host when a
// mesh is created).  So KE v = W^T B (W v) / 8 costs two 8-point Walsh
// transforms per component plus ~40 multiply-adds instead of 576.
//
// Data flow.  A workgroup of 32 x ROWS threads (two 32-lane x-rows per
// wavefront; ROWS = 16 unless a tuned shape says otherwise) owns
// 30 x (ROWS - 1) node columns; thread (tx, ty) handles the element column
// (i, j) = (30 bx - 1 + tx, (ROWS - 1) by - 1 + ty) (the last lane of a row
// only supplies node values) and marches along z over a chunk of node
// planes.  The x-y
// Walsh transform of a node plane is computed once and reused by the two
// element layers that share the plane; the dz = 1 outputs of layer k-1 stay
// in registers and are added to the dz = 0 outputs of layer k.  The four
// element columns around a node are combined in a fixed order: x neighbours
// through DPP wavefront shifts, y neighbours through one
// double-buffered LDS exchange per layer.  The next node plane is loaded
// while the current one is processed.  No atomics: every node is
// written once by its owner, so results are deterministic.
#include "internal.hpp"
#include "walsh.hpp"

namespace aarmr {

namespace {

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Lane i of a wavefront takes the value of lane i+1 (wave_shl:1) or lane
// i-1 (wave_shr:1) through DPP; the end lanes read 0 (bound_ctrl), so the
// destination needs no copy of the source first.  Across the boundary of
// two 32-lane x-rows this moves a value between the last lane of a row
// (which only supplies node values) and the first lane of the next (a halo
// lane that owns nothing); lanes 0 and 63 are such lanes too, so none of
// these results is used.
template <int CTRL>
__device__ inline double dpp(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ inline float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, true));
}
constexpr int kWaveShl1 = 0x130;  // lane i <- lane i+1 across the wavefront
constexpr int kWaveShr1 = 0x138;  // lane i <- lane i-1
template <typename T>
__device__ inline T from_next_lane(T v) { return dpp<kWaveShl1>(v); }
template <typename T>
__device__ inline T from_prev_lane(T v) { return dpp<kWaveShr1>(v); }

// 2D Walsh transform of a 2x2 quad q[cxy] (cxy = dx + 2 dy), in place.
template <typename T>
__device__ inline void walsh4(T& q0, T& q1, T& q2, T& q3) {
  const T s0 = q0 + q1, d0 = q0 - q1, s1 = q2 + q3, d1 = q2 - q3;
  q0 = s0 + s1;
  q1 = d0 + d1;
  q2 = s0 - s1;
  q3 = d0 - d1;
}

// Raw buffer access.  A buffer resource carries the array's size in bytes;
// the hardware returns 0 for loads at or beyond it and drops such stores.
// The kernel uses this documented range check instead of branches: a lane
// whose node lies outside the grid, or that owns no output, uses the offset
// kOutside.  Loads and stores then are unconditional instructions, so the
// compiler can count outstanding memory operations statically and never has
// to drain the prefetched plane.
constexpr uint32_t kOutside = 0x80000000u;
// 32-lane rows: a row segment of y is 30 nodes, so per owned node half as
// many cache lines are shared with the neighbouring tile as with 16 lanes.
// A workgroup has ROWS x-rows (2 per wavefront) and owns ROWS - 1 node rows;
// ROWS is one of {8, 12, 16} (ebe_rows below).
constexpr int kLanes = 32;           // element columns per x-row
constexpr int kTileX = kLanes - 2;   // node columns owned per row
constexpr int kBufferWord3 = 0x00020000;  // raw buffer, 32-bit dwords (gfx9)

__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                           kBufferWord3);
}
// `soff` is a wave-uniform byte offset carried in the scalar operand (the
// component stride), so it costs no vector instruction.  An out-of-range
// lane stays out of range with it: kOutside + soff is below 2^32 and above
// every buffer size.
__device__ inline double ld(__amdgpu_buffer_rsrc_t r, uint32_t off, double, uint32_t soff = 0) {
  return __builtin_bit_cast(double,
                            __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, (int)soff, 0));
}
__device__ inline float ld(__amdgpu_buffer_rsrc_t r, uint32_t off, float, uint32_t soff = 0) {
  return __builtin_bit_cast(float,
                            __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, (int)soff, 0));
}
__device__ inline void st(__amdgpu_buffer_rsrc_t r, uint32_t off, double x, uint32_t soff = 0) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(decltype(
      __builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)), x), r, (int)off, (int)soff, 0);
}
__device__ inline void st(__amdgpu_buffer_rsrc_t r, uint32_t off, float x, uint32_t soff = 0) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(decltype(
      __builtin_amdgcn_raw_buffer_load_b32(r, 0, 0, 0)), x), r, (int)off, (int)soff, 0);
}
__device__ inline uint32_t ld_u8(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(r, (int)off, 0, 0);
}

// Raw node values and fixed-DOF masks of one plane as seen by a thread: its
// nodes (i, j) and (i, j+1); the (i+1) corners come from the next lane.
template <typename T>
struct PlaneRaw {
  T q0[3], q2[3];
  uint32_t m0, m2;
};

// y = Df K Df v (zero on fixed DOFs).  MASK_IN: zero the fixed DOFs of v on
// load; without it the caller guarantees that v is already zero there (true
// of every vector inside the solvers), which saves the loads and selects.
// PF: prefetch distance in node planes (1 or 2).  JAC: the product feeds a
// damped-Jacobi sweep, y = v + omega jd (jb - A v) (y distinct from v); the
// node's own v, jb and jd are fetched one plane ahead like the moduli.
// DOT: the workgroup also writes part[blockIdx.x], the sum over the nodes it
// owns of d . y with d = jb (JAC) or d = v: the partials of CG's r^T z or
// p^T A p, summed in a fixed order by the kernel that consumes them.
#ifndef AARMR_EBE_MINB
#define AARMR_EBE_MINB 1  // workgroups per CU the register budget is sized for
#endif
template <typename T, int ROWS, bool MASK_IN, int PF, bool JAC, bool DOT>
__global__ void __launch_bounds__(kLanes * ROWS, AARMR_EBE_MINB) k_ebe_z(int nx, int ny, int nz, int gx, int gy, int TZ,
                                                    WalshConsts K, const T* __restrict__ E,
                                                    const uint8_t* __restrict__ mask,
                                                    const T* __restrict__ v, T* __restrict__ y,
                                                    const T* __restrict__ jb,
                                                    const T* __restrict__ jd, T omega,
                                                    double* __restrict__ part, int64_t rs,
                                                    int pst) {
  constexpr bool OWNV = JAC || DOT;  // keep the node's own v of the plane written next
  {  // load case blockIdx.z of a lock-step multi-vector (the moduli, mask and
     // Jacobi diagonal are shared)
    const int64_t ro = (int64_t)blockIdx.z * rs;
    v += ro;
    y += ro;
    if (JAC) jb += ro;
    if (DOT) part += (int64_t)blockIdx.z * pst;
  }
  constexpr int kTileY = ROWS - 1;   // node rows owned per workgroup
  __shared__ T xs[2][3][ROWS][kLanes];
  const int tx = threadIdx.x & (kLanes - 1), ty = threadIdx.x / kLanes;
  // XCD-aware tile order: workgroups are dispatched round-robin over the 8
  // XCDs, so workgroup w is given tile (w % 8) * (count / 8) + w / 8 and
  // every XCD walks a contiguous range of tiles.  Tiles that share cache
  // lines (x neighbours) or halo rows (y neighbours) then meet in one L2.
  int bx, by, bz;
  {
    const int total = gridDim.x;
    const int w = blockIdx.x;
    const int xcd = w & 7, pos = w >> 3, q = total >> 3, r = total & 7;
    const int t = (xcd < r) ? xcd * (q + 1) + pos : r * (q + 1) + (xcd - r) * q + pos;
    bx = t % gx;
    by = (t / gx) % gy;
    bz = t / (gx * gy);
  }
  const int i = bx * kTileX - 1 + tx;
  const int j = by * kTileY - 1 + ty;
  const int kz0 = bz * TZ;
  const int kz1 = min(kz0 + TZ, nz + 1);
  // 32-bit offsets: the host guarantees 3 * n_node * 8 < 2^31
  const int nxp = nx + 1, nyp = ny + 1;
  const int plane = nxp * nyp, nn = plane * (nz + 1), eplane = nx * ny;
  const uint32_t TS = (uint32_t)sizeof(T);
  const auto rv = make_rsrc(v, 3u * nn * TS);
  const auto ry = make_rsrc(y, 3u * nn * TS);
  const auto rE = make_rsrc(E, (uint32_t)eplane * nz * TS);
  const auto rm = make_rsrc(mask, (uint32_t)nn);
  const auto rjb = make_rsrc(jb, JAC ? 3u * nn * TS : 0u);
  const auto rjd = make_rsrc(jd, JAC ? 3u * nn * TS : 0u);
  // the last lane of a row only supplies node values to its left neighbour:
  // it computes no element and owns no node
  const bool col_ok = tx < kLanes - 1 && i >= 0 && i < nx && j >= 0 && j < ny;
  const bool xi_ok = i >= 0 && i <= nx;
  const bool yj_ok = j >= 0 && j <= ny, yj1_ok = j + 1 >= 0 && j + 1 <= ny;
  const bool own = tx >= 1 && tx < kLanes - 1 && ty >= 1 && i <= nx && j <= ny;
  const int off00 = i + nxp * j;

  // One select per node: kOutside + c * 3 n_node * sizeof(T) stays out of
  // range (below 2^32, above every buffer size), so components need none.
  const uint32_t cstride = (uint32_t)nn * TS;
  auto load_node = [&](bool ok, int node, T (&q)[3], uint32_t& m, bool want_mask) {
    const uint32_t o = ok ? (uint32_t)node * TS : kOutside;
    m = want_mask ? ld_u8(rm, ok ? (uint32_t)node : kOutside) : 0u;
#pragma unroll
    for (int c = 0; c < 3; ++c) q[c] = ld(rv, o, T(), (uint32_t)c * cstride);
  };
  auto load_plane = [&](int k, PlaneRaw<T>& R) {
    const bool kin = k >= 0 && k <= nz;
    const int base = k * plane + off00;
    load_node(kin && xi_ok && yj_ok, base, R.q0, R.m0, true);  // m0 also masks the output
    load_node(kin && xi_ok && yj1_ok, base + nxp, R.q2, R.m2, MASK_IN);
  };
  auto masked = [](T x, uint32_t m, int c) { return (MASK_IN && ((m >> c) & 1u)) ? (T)0 : x; };
  // x-y Walsh transform of the element's four plane corners: the y
  // butterfly of the lane's own two nodes first, then the x butterfly with
  // the next lane's (6 additions and 2 lane moves per component)
  auto transform = [&](const PlaneRaw<T>& R, T (&P)[4][3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T a0 = masked(R.q0[c], R.m0, c), a2 = masked(R.q2[c], R.m2, c);
      const T ye = a0 + a2, yo = a0 - a2;
      const T ye1 = from_next_lane(ye), yo1 = from_next_lane(yo);
      P[0][c] = ye + ye1;
      P[1][c] = ye - ye1;
      P[2][c] = yo + yo1;
      P[3][c] = yo - yo1;
    }
  };
  auto load_w = [&](int k) -> T {
    const bool ok = col_ok && k >= 0 && k < nz;
    return ld(rE, ok ? (uint32_t)(i + nx * j + eplane * k) * TS : kOutside, T());
  };

  T P0[4][3], P1[4][3], carry[4][3];
  {
    PlaneRaw<T> r0;
    load_plane(kz0 - 1, r0);
    transform(r0, P0);
  }
  // PF planes in flight: a plane's loads have PF element layers of work to
  // arrive in.  The loop is unrolled by two: the two plane transforms swap
  // the roles of bottom and top instead of being copied, and with PF = 2 the
  // two raw-plane buffers alternate.
  PlaneRaw<T> RA, RB;
  load_plane(kz0, RA);
  T WA = load_w(kz0 - 1), WB = (T)0;
  if (PF == 2) {
    load_plane(kz0 + 1 <= kz1 ? kz0 + 1 : -2, RB);
    WB = load_w(kz0 < kz1 ? kz0 : -1);
  }
  uint32_t own_m = 7u;  // fixed-DOF mask of node (i, j) on the plane written next
  T own_v[3] = {}, own_b[3] = {}, own_d[3] = {};  // JAC: that node's v, jb, jd
  double dacc = 0.0;                               // DOT: this thread's share, FP64
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int c = 0; c < 3; ++c) carry[q][c] = (T)0;
  int buf = 0;

  // Element layer k: node planes k (Pb) and k+1 (R, transformed into Pt);
  // writes plane k and refills R with plane k+1+PF.  The first layer of a
  // chunk only primes the carry (its stores go outside).
  auto step = [&](int k, PlaneRaw<T>& R, T& W, const T (&Pb)[4][3], T (&Pt)[4][3]) {
    transform(R, Pt);
    const T w = W;
    const uint32_t m_next = R.m0;
    T v_next[3], b_next[3], d_next[3];
    if (OWNV) {  // node (i, j) of plane k + 1, written by the next step
#pragma unroll
      for (int c = 0; c < 3; ++c) v_next[c] = R.q0[c];
    }
    if (JAC) {
      const uint32_t on = (own && k + 1 <= nz) ? (uint32_t)((k + 1) * plane + off00) * TS : kOutside;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        b_next[c] = ld(rjb, on, T(), (uint32_t)c * cstride);
        d_next[c] = ld(rjd, on, T(), (uint32_t)c * cstride);
      }
    }
    load_plane(k + 1 + PF <= kz1 ? k + 1 + PF : -2, R);
    W = load_w(k + PF < kz1 ? k + PF : -1);
    T h[8][3], z[8][3];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        h[q][c] = Pb[q][c] + Pt[q][c];
        h[q + 4][c] = Pb[q][c] - Pt[q][c];
      }
    walsh_blocks<T>(K, w, h, z);
    // plane k: carry (dz=1 of layer k-1) + dz=0 of layer k, then back to
    // corners and summed with the previous lane's element.  With the x
    // butterfly s = a0 + a1, d = a0 - a1 (y index 0) and t = a2 + a3,
    // e = a2 - a3 (y index 1), node (i, j) of row j is s + t + prev(d + e)
    // and node (i, j+1) is s - t + prev(d - e), so u = s + prev(d) and
    // w = t + prev(e) give both as u + w and u - w.  The carry is then
    // replaced by the dz=1 part of layer k.
    T X0[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T a0 = carry[0][c] + (z[0][c] + z[4][c]);
      const T a1 = carry[1][c] + (z[1][c] + z[5][c]);
      const T a2 = carry[2][c] + (z[2][c] + z[6][c]);
      const T a3 = carry[3][c] + (z[3][c] + z[7][c]);
      carry[0][c] = z[0][c] - z[4][c];
      carry[1][c] = z[1][c] - z[5][c];
      carry[2][c] = z[2][c] - z[6][c];
      carry[3][c] = z[3][c] - z[7][c];
      const T u = (a0 + a1) + from_prev_lane(a0 - a1);
      const T w = (a2 + a3) + from_prev_lane(a2 - a3);
      X0[c] = u + w;                 // node (i, j), row j
      xs[buf][c][ty][tx] = u - w;    // node (i, j+1), row j
    }
    __syncthreads();
    const bool wr = own && k >= kz0;
    const uint32_t oy = wr ? (uint32_t)(k * plane + off00) * TS : kOutside;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T out = X0[c] + xs[buf][c][ty > 0 ? ty - 1 : 0][tx];
      if (JAC) out = own_v[c] + omega * own_d[c] * (own_b[c] - out);
      if ((own_m >> c) & 1u) out = (T)0;
      st(ry, oy, out, (uint32_t)c * cstride);
      if (DOT) dacc += wr ? (double)(JAC ? own_b[c] : own_v[c]) * (double)out : 0.0;
    }
    buf ^= 1;
    own_m = m_next;
    if (OWNV) {
#pragma unroll
      for (int c = 0; c < 3; ++c) own_v[c] = v_next[c];
    }
    if (JAC) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        own_b[c] = b_next[c];
        own_d[c] = d_next[c];
      }
    }
  };
  for (int k = kz0 - 1; k < kz1; k += 2) {
    step(k, RA, WA, P0, P1);
    if (k + 1 < kz1) {
      if (PF == 2) step(k + 1, RB, WB, P1, P0);
      else step(k + 1, RA, WA, P1, P0);
    }
  }
  if (DOT) {  // wavefront sums, then the four in wave order
    __shared__ double wsum[ROWS / 2];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) dacc += __shfl_down(dacc, off, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = dacc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
#pragma unroll
      for (int q = 4; q < ROWS / 2; q += 2) t += wsum[q] + wsum[q + 1];
      part[blockIdx.x] = t;
    }
  }
}

// e_e = u_e^T KE u_e = (W u)^T B (W u) / 8 per element; fixed DOFs read as zero.
__global__ void __launch_bounds__(256) k_energy_walsh(int nx, int ny, int nz, WalshConsts K,
                                                      const uint8_t* __restrict__ mask,
                                                      const double* __restrict__ u,
                                                      double* __restrict__ energy) {
  const int64_t ne = (int64_t)nx * ny * nz;
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int ex = (int)(e % nx);
  const int64_t rest = e / nx;
  const int ey = (int)(rest % ny), ez = (int)(rest / ny);
  const int64_t nxp = nx + 1, plane = nxp * (ny + 1), nn = plane * (nz + 1);
  double P[2][4][3];
#pragma unroll
  for (int dz = 0; dz < 2; ++dz) {
    double q[4][3];
#pragma unroll
    for (int cxy = 0; cxy < 4; ++cxy) {
      const int64_t node = (int64_t)(ex + (cxy & 1)) + nxp * (ey + (cxy >> 1)) + plane * (ez + dz);
      const uint8_t m = mask[node];
#pragma unroll
      for (int c = 0; c < 3; ++c) q[cxy][c] = ((m >> c) & 1) ? 0.0 : u[c * nn + node];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      walsh4(q[0][c], q[1][c], q[2][c], q[3][c]);
#pragma unroll
      for (int cxy = 0; cxy < 4; ++cxy) P[dz][cxy][c] = q[cxy][c];
    }
  }
  double h[8][3], z[8][3];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      h[q][c] = P[0][q][c] + P[1][q][c];
      h[q + 4][c] = P[0][q][c] - P[1][q][c];
    }
  walsh_blocks<double>(K, 1.0, h, z);
  double s = 0.0;
#pragma unroll
  for (int q = 1; q < 8; ++q)
#pragma unroll
    for (int c = 0; c < 3; ++c) s = fma(h[q][c], z[q][c], s);
  energy[e] = s;
}

}  // namespace

// y[fixed] = v[fixed]: the identity rows of A on fixed DOFs.
template <typename T>
__global__ void k_identity_rows(int64_t nn, const uint8_t* __restrict__ mask,
                                const T* __restrict__ v, T* __restrict__ y) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const uint32_t m = mask[n];
  if (!m) return;
#pragma unroll
  for (int c = 0; c < 3; ++c)
    if ((m >> c) & 1u) y[c * nn + n] = v[c * nn + n];
}

// z-chunk of node planes per workgroup.  A chunk costs one extra element
// layer (the carry is primed from the layer below it); the length is chosen
// by the number of rounds over the device's resident workgroup slots times
// the plane steps per chunk (see launch_ebe_r), at least 4 planes per chunk
// unless a tuned length (2 or more) is given.
// Prefetch distance: two node planes in flight for the 16-row tile (a
// 512-thread workgroup leaves registers to spare at its occupancy of two
// wavefronts per SIMD; 256x128x128: 70 -> 67 us), one for the smaller tiles,
// whose occupancy the extra registers would cut.
#ifndef AARMR_EBE_PF
#define AARMR_EBE_PF(ROWS) ((ROWS) == 16 ? 2 : 1)
#endif

// Tile rows.  The launch shape word `shape` carries a tuned z-chunk length
// in its low 16 bits (0: residency-sized) and a tuned ROWS in the bits above
// (0: the default, 16 rows).  Sixteen rows measured fastest on both the
// 96x48x48 and the 256x128x128 grid: 8.8 and 66.7 us against 9.2 and 76 us
// with 8 rows and 14 and 83 us with 12, although a 512-thread workgroup of
// this kernel leaves a third of the wavefront slots of a compute unit empty.
#ifndef AARMR_EBE_ROWS
#define AARMR_EBE_ROWS 16
#endif

int ebe_rows(int shape) {
  const int tuned = shape >> 16;
  if (tuned == 8 || tuned == 12 || tuned == 16) return tuned;
  return AARMR_EBE_ROWS;
}

template <typename T, int ROWS, bool MASK_IN, bool JAC, bool DOT>
static int launch_ebe_r(const Grid& g, const WalshConsts& K, const T* E, const uint8_t* mask,
                        const T* v, T* y, int tz_req, hipStream_t s, const T* jb, const T* jd,
                        T omega, double* part, int nr, int pst) {
  constexpr int kThreads = kLanes * ROWS;
  constexpr int kTileY = ROWS - 1;
  // resident workgroups of this kernel on the device (thread-safe one-time init)
  static const int slots = [] {
    int dev = 0, cus = 0, per_cu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, k_ebe_z<T, ROWS, MASK_IN, AARMR_EBE_PF(ROWS), JAC, DOT>, kThreads, 0);
    return (cus > 0 && per_cu > 0) ? cus * per_cu : 512;
  }();
  const int gx = (g.nx + 1 + kTileX - 1) / kTileX;
  const int gy = (g.ny + 1 + kTileY - 1) / kTileY;
  const int planes = g.nz + 1;
  int tz = planes;
  if (tz_req > 0) {
    tz = tz_req < planes ? tz_req : planes;  // tuned z-chunk length
  } else {
    // Chunks of t planes take about ceil(workgroups / slots) rounds of t + 1
    // plane steps (a chunk also primes its carry with one layer), so take
    // the length with the fewest steps, at least 4 planes a chunk.  Grids
    // with fewer tiles than slots get one round of the shortest chunks that
    // fit; larger ones get a split whose last round is well filled.
    const int64_t tiles = (int64_t)gx * gy;
    int64_t best = -1;
    for (int n = 1; n <= planes; ++n) {
      const int t = (planes + n - 1) / n;
      if (t < 4 && n > 1) break;
      const int64_t chunks = (planes + t - 1) / t;
      const int64_t cost = (tiles * chunks + slots - 1) / slots * (t + 1);
      if (best < 0 || cost < best) {
        best = cost;
        tz = t;
      }
    }
  }
  if (tz < 2) tz = 2;
  const int gz = (planes + tz - 1) / tz;
  k_ebe_z<T, ROWS, MASK_IN, AARMR_EBE_PF(ROWS), JAC, DOT>
      <<<dim3((unsigned)(gx * gy * gz), 1, (unsigned)nr), kThreads, 0, s>>>(
          g.nx, g.ny, g.nz, gx, gy, tz, K, E, mask, v, y, jb, jd, omega, part, 3 * g.nn, pst);
  return gx * gy * gz;
}

template <typename T, bool MASK_IN, bool JAC = false, bool DOT = false>
static int launch_ebe_t(const Grid& g, const WalshConsts& K, const T* E, const uint8_t* mask,
                        const T* v, T* y, int shape, hipStream_t s, const T* jb = nullptr,
                        const T* jd = nullptr, T omega = 0, double* part = nullptr, int nr = 1,
                        int pst = 0) {
  const int tz = shape & 0xFFFF;
  switch (ebe_rows(shape)) {
    case 8:
      return launch_ebe_r<T, 8, MASK_IN, JAC, DOT>(g, K, E, mask, v, y, tz, s, jb, jd, omega, part,
                                                   nr, pst);
    case 12:
      return launch_ebe_r<T, 12, MASK_IN, JAC, DOT>(g, K, E, mask, v, y, tz, s, jb, jd, omega,
                                                    part, nr, pst);
    default:
      return launch_ebe_r<T, 16, MASK_IN, JAC, DOT>(g, K, E, mask, v, y, tz, s, jb, jd, omega,
                                                    part, nr, pst);
  }
}

int ebe_partials_max(const Grid& g) {
  // the most workgroups of any tile height (8 rows) and chunk length (2)
  const int gx = (g.nx + 1 + kTileX - 1) / kTileX;
  const int gy = (g.ny + 1 + 7 - 1) / 7;
  return gx * gy * ((g.nz + 1 + 1) / 2);
}

int launch_ebe_dot(const Grid& g, const WalshConsts& K, const double* E, const uint8_t* mask,
                   const double* v, double* y, double* part, hipStream_t s, int tz) {
  return launch_ebe_t<double, false, false, true>(g, K, E, mask, v, y, tz, s, nullptr, nullptr,
                                                  0.0, part);
}

int launch_ebe_jacobi_dot(const Grid& g, const WalshConsts& K, const double* E,
                          const uint8_t* mask, const double* v, const double* b,
                          const double* dinv, double omega, double* out, double* part,
                          hipStream_t s, int tz) {
  return launch_ebe_t<double, false, true, true>(g, K, E, mask, v, out, tz, s, b, dinv, omega,
                                                 part);
}

int launch_ebe_f32_dot(const Grid& g, const WalshConsts& K, const float* E, const uint8_t* mask,
                       const float* v, float* y, double* part, hipStream_t s, int tz, int nr,
                       int pst) {
  return launch_ebe_t<float, false, false, true>(g, K, E, mask, v, y, tz, s, nullptr, nullptr,
                                                 0.0f, part, nr, pst);
}

int launch_ebe_jacobi_f32_dot(const Grid& g, const WalshConsts& K, const float* E,
                              const uint8_t* mask, const float* v, const float* b,
                              const float* dinv, float omega, float* out, double* part,
                              hipStream_t s, int tz, int nr, int pst) {
  return launch_ebe_t<float, false, true, true>(g, K, E, mask, v, out, tz, s, b, dinv, omega,
                                                part, nr, pst);
}

void launch_ebe(const Grid& g, const WalshConsts& K, const double* E, const uint8_t* mask,
                const double* v, double* y, int mode, hipStream_t s, int tz) {
  if (mode == 2) {
    launch_ebe_t<double, false>(g, K, E, mask, v, y, tz, s);
    return;
  }
  launch_ebe_t<double, true>(g, K, E, mask, v, y, tz, s);
  if (mode == 0) k_identity_rows<double><<<nblk(g.nn, 256), 256, 0, s>>>(g.nn, mask, v, y);
}

void launch_ebe_jacobi(const Grid& g, const WalshConsts& K, const double* E, const uint8_t* mask,
                       const double* v, const double* b, const double* dinv, double omega,
                       double* out, hipStream_t s, int tz) {
  launch_ebe_t<double, false, true>(g, K, E, mask, v, out, tz, s, b, dinv, omega);
}

void launch_ebe_f32(const Grid& g, const WalshConsts& K, const float* E, const uint8_t* mask,
                    const float* v, float* y, int mode, hipStream_t s, int tz, int nr) {
  if (mode == 2) {
    launch_ebe_t<float, false>(g, K, E, mask, v, y, tz, s, nullptr, nullptr, 0.0f, nullptr, nr);
    return;
  }
  launch_ebe_t<float, true>(g, K, E, mask, v, y, tz, s);
  if (mode == 0) k_identity_rows<float><<<nblk(g.nn, 256), 256, 0, s>>>(g.nn, mask, v, y);
}

void launch_energy_walsh(const Grid& g, const WalshConsts& K, const uint8_t* mask,
                         const double* u, double* energy, hipStream_t s) {
  k_energy_walsh<<<nblk(g.ne, 256), 256, 0, s>>>(g.nx, g.ny, g.nz, K, mask, u, energy);
}

}  // namespace aarmr
