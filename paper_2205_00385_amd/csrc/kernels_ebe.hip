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
// Data flow.  A workgroup of 16 x 16 threads owns 15 x 15 node columns;
// thread (tx, ty) owns the element column (i, j) = (15 bx - 1 + tx,
// 15 by - 1 + ty) and marches along z over a chunk of node planes.  The x-y
// Walsh transform of a node plane is computed once and reused by the two
// element layers that share the plane; the dz = 1 outputs of layer k-1 stay
// in registers and are added to the dz = 0 outputs of layer k.  The four
// element columns around a node are combined in a fixed order: x neighbours
// through DPP row shifts inside 16-lane rows, y neighbours through one
// double-buffered LDS exchange per layer.  The next node plane is loaded
// while the current one is processed.  No atomics: every node is
// written once by its owner, so results are deterministic.
#include "internal.hpp"
#include "walsh.hpp"

namespace aarmr {

namespace {

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Lane i of each 16-lane row takes the value of lane i+1 (row_shl:1) or
// lane i-1 (row_shr:1) through DPP; lanes whose source lies outside the row
// keep their own value.
template <int CTRL>
__device__ inline double dpp(double x) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(x), __double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(x), __double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ inline float dpp(float x) {
  const int v = __float_as_int(x);
  return __int_as_float(__builtin_amdgcn_update_dpp(v, v, CTRL, 0xF, 0xF, false));
}
constexpr int kRowShl1 = 0x101;
constexpr int kRowShr1 = 0x111;
template <typename T>
__device__ inline T from_next_lane(T v) { return dpp<kRowShl1>(v); }
template <typename T>
__device__ inline T from_prev_lane(T v) { return dpp<kRowShr1>(v); }

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
constexpr int kBufferWord3 = 0x00020000;  // raw buffer, 32-bit dwords (gfx9)

__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                           kBufferWord3);
}
__device__ inline double ld(__amdgpu_buffer_rsrc_t r, uint32_t off, double) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
__device__ inline float ld(__amdgpu_buffer_rsrc_t r, uint32_t off, float) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
__device__ inline void st(__amdgpu_buffer_rsrc_t r, uint32_t off, double x) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(decltype(
      __builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)), x), r, (int)off, 0, 0);
}
__device__ inline void st(__amdgpu_buffer_rsrc_t r, uint32_t off, float x) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(decltype(
      __builtin_amdgcn_raw_buffer_load_b32(r, 0, 0, 0)), x), r, (int)off, 0, 0);
}
__device__ inline uint32_t ld_u8(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(r, (int)off, 0, 0);
}

// Raw node values and fixed-DOF masks of one plane as seen by a thread: its
// own nodes (i, j) and (i, j+1), and for the last lane of a row also
// (i+1, j), (i+1, j+1) (the other lanes get those from the next lane).
template <typename T>
struct PlaneRaw {
  T q0[3], q2[3], q1[3], q3[3];
  uint32_t m0, m2, m1, m3;
};

template <typename T, int TZ>
__global__ void __launch_bounds__(256) k_ebe_z(int nx, int ny, int nz, WalshConsts K,
                                               const T* __restrict__ E,
                                               const uint8_t* __restrict__ mask,
                                               const T* __restrict__ v, T* __restrict__ y,
                                               int mode) {
  __shared__ T xs[2][3][16][16];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i = (int)blockIdx.x * 15 - 1 + tx;
  const int j = (int)blockIdx.y * 15 - 1 + ty;
  const int kz0 = (int)blockIdx.z * TZ;
  const int kz1 = min(kz0 + TZ, nz + 1);
  // 32-bit offsets: the host guarantees 3 * n_node * 8 < 2^31
  const int nxp = nx + 1, nyp = ny + 1;
  const int plane = nxp * nyp, nn = plane * (nz + 1), eplane = nx * ny;
  const uint32_t TS = (uint32_t)sizeof(T);
  const auto rv = make_rsrc(v, 3u * nn * TS);
  const auto ry = make_rsrc(y, 3u * nn * TS);
  const auto rE = make_rsrc(E, (uint32_t)eplane * nz * TS);
  const auto rm = make_rsrc(mask, (uint32_t)nn);
  const bool col_ok = i >= 0 && i < nx && j >= 0 && j < ny;
  const bool xi_ok = i >= 0 && i <= nx, xi1_ok = i + 1 >= 0 && i + 1 <= nx;
  const bool yj_ok = j >= 0 && j <= ny, yj1_ok = j + 1 >= 0 && j + 1 <= ny;
  const bool own = tx >= 1 && ty >= 1 && i <= nx && j <= ny;
  const bool last = tx == 15;
  const int off00 = i + nxp * j;

  // One select per node: kOutside + c * 3 n_node * sizeof(T) stays out of
  // range (below 2^32, above every buffer size), so components need none.
  const uint32_t cstride = (uint32_t)nn * TS;
  auto load_node = [&](bool ok, int node, T (&q)[3], uint32_t& m) {
    const uint32_t o = ok ? (uint32_t)node * TS : kOutside;
    m = ld_u8(rm, ok ? (uint32_t)node : kOutside);
#pragma unroll
    for (int c = 0; c < 3; ++c) q[c] = ld(rv, o + (uint32_t)c * cstride, T());
  };
  auto load_plane = [&](int k, PlaneRaw<T>& R) {
    const bool kin = k >= 0 && k <= nz;
    const int base = k * plane + off00;
    load_node(kin && xi_ok && yj_ok, base, R.q0, R.m0);
    load_node(kin && xi_ok && yj1_ok, base + nxp, R.q2, R.m2);
    load_node(last && kin && xi1_ok && yj_ok, base + 1, R.q1, R.m1);
    load_node(last && kin && xi1_ok && yj1_ok, base + nxp + 1, R.q3, R.m3);
  };
  auto masked = [](T x, uint32_t m, int c) { return ((m >> c) & 1u) ? (T)0 : x; };
  auto transform = [&](const PlaneRaw<T>& R, T (&P)[4][3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T a0 = masked(R.q0[c], R.m0, c), a2 = masked(R.q2[c], R.m2, c);
      T a1 = from_next_lane(a0), a3 = from_next_lane(a2);
      if (last) {
        a1 = masked(R.q1[c], R.m1, c);
        a3 = masked(R.q3[c], R.m3, c);
      }
      walsh4(a0, a1, a2, a3);
      P[0][c] = a0;
      P[1][c] = a1;
      P[2][c] = a2;
      P[3][c] = a3;
    }
  };
  auto load_w = [&](int k) -> T {
    const bool ok = col_ok && k >= 0 && k < nz;
    return ld(rE, ok ? (uint32_t)(i + nx * j + eplane * k) * TS : kOutside, T());
  };

  T Pb[4][3], carry[4][3];
  {
    PlaneRaw<T> r0;
    load_plane(kz0 - 1, r0);
    transform(r0, Pb);
  }
  PlaneRaw<T> R;
  load_plane(kz0, R);
  T W = load_w(kz0 - 1);
  T own_v[3] = {(T)0, (T)0, (T)0};  // raw v and mask of node (i, j) on the plane written next
  uint32_t own_m = 7u;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int c = 0; c < 3; ++c) carry[q][c] = (T)0;
  int buf = 0;

  // Element layer k: node planes k (Pb) and k+1 (R); writes plane k.  The
  // first layer of a chunk only primes the carry (its stores go outside).
  for (int k = kz0 - 1; k < kz1; ++k) {
    T Pt[4][3];
    transform(R, Pt);
    const T w = W;
    T v_next[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) v_next[c] = R.q0[c];
    const uint32_t m_next = R.m0;
    load_plane(k + 2 <= kz1 ? k + 2 : -2, R);  // prefetch plane k+2
    W = load_w(k + 1 < kz1 ? k + 1 : -1);
    T h[8][3], z[8][3];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        h[q][c] = Pb[q][c] + Pt[q][c];
        h[q + 4][c] = Pb[q][c] - Pt[q][c];
      }
    walsh_blocks<T>(K, w, h, z);
    // plane k: carry (dz=1 of layer k-1) + dz=0 of layer k, back to corners
    T cor[4][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T a0 = carry[0][c] + (z[0][c] + z[4][c]);
      T a1 = carry[1][c] + (z[1][c] + z[5][c]);
      T a2 = carry[2][c] + (z[2][c] + z[6][c]);
      T a3 = carry[3][c] + (z[3][c] + z[7][c]);
      walsh4(a0, a1, a2, a3);
      cor[0][c] = a0;
      cor[1][c] = a1;
      cor[2][c] = a2;
      cor[3][c] = a3;
    }
    T X0[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      X0[c] = cor[0][c] + from_prev_lane(cor[1][c]);                 // node (i, j), row j
      xs[buf][c][ty][tx] = cor[2][c] + from_prev_lane(cor[3][c]);  // node (i, j+1), row j
    }
    __syncthreads();
    const bool wr = own && k >= kz0;
    const uint32_t oy = wr ? (uint32_t)(k * plane + off00) * TS : kOutside;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T out = X0[c] + xs[buf][c][ty > 0 ? ty - 1 : 0][tx];
      if ((own_m >> c) & 1u) out = mode == 0 ? own_v[c] : (T)0;
      st(ry, oy + (uint32_t)c * cstride, out);
    }
    buf ^= 1;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      carry[0][c] = z[0][c] - z[4][c];
      carry[1][c] = z[1][c] - z[5][c];
      carry[2][c] = z[2][c] - z[6][c];
      carry[3][c] = z[3][c] - z[7][c];
      own_v[c] = v_next[c];
    }
    own_m = m_next;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) Pb[q][c] = Pt[q][c];
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

// z-chunk of node planes per workgroup: the longest chunk that still gives
// at least four workgroups per compute unit (256 CUs), 4 at the least.
template <typename T>
static void launch_ebe_t(const Grid& g, const WalshConsts& K, const T* E, const uint8_t* mask,
                         const T* v, T* y, int mode, hipStream_t s) {
  const unsigned gx = (unsigned)((g.nx + 1 + 14) / 15), gy = (unsigned)((g.ny + 1 + 14) / 15);
  const int planes = g.nz + 1;
  auto gz = [&](int tz) { return (unsigned)((planes + tz - 1) / tz); };
  if ((int64_t)gx * gy * gz(16) >= 1024)
    k_ebe_z<T, 16><<<dim3(gx, gy, gz(16)), 256, 0, s>>>(g.nx, g.ny, g.nz, K, E, mask, v, y, mode);
  else if ((int64_t)gx * gy * gz(8) >= 1024)
    k_ebe_z<T, 8><<<dim3(gx, gy, gz(8)), 256, 0, s>>>(g.nx, g.ny, g.nz, K, E, mask, v, y, mode);
  else
    k_ebe_z<T, 4><<<dim3(gx, gy, gz(4)), 256, 0, s>>>(g.nx, g.ny, g.nz, K, E, mask, v, y, mode);
}

void launch_ebe(const Grid& g, const WalshConsts& K, const double* E, const uint8_t* mask,
                const double* v, double* y, int mode, hipStream_t s) {
  launch_ebe_t<double>(g, K, E, mask, v, y, mode, s);
}

void launch_ebe_f32(const Grid& g, const WalshConsts& K, const float* E, const uint8_t* mask,
                    const float* v, float* y, int mode, hipStream_t s) {
  launch_ebe_t<float>(g, K, E, mask, v, y, mode, s);
}

void launch_energy_walsh(const Grid& g, const WalshConsts& K, const uint8_t* mask,
                         const double* u, double* energy, hipStream_t s) {
  k_energy_walsh<<<nblk(g.ne, 256), 256, 0, s>>>(g.nx, g.ny, g.nz, K, mask, u, energy);
}

}  // namespace aarmr
