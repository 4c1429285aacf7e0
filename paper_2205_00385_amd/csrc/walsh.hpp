// Reflection-blocked form of the unit-cube hex8 stiffness (shared by the
// kernels and by the host check that validates it for a given nu).
//
// With corners a = dx + 2 dy + 4 dz and the Walsh matrix
// W[k][a] = (-1)^popcount(k & a), applied per displacement component,
// B = W KE W^T / 64 satisfies KE = W^T B W.  For an isotropic material the
// reflection symmetries of the cube leave B with the block pattern coded in
// walsh_blocks(): index 0 (translations) is null; {(1,x),(2,y),(4,z)} and
// {(3,z),(5,y),(6,x)} are 3x3 blocks a I + b (J - I); {(1,y),(2,x)},
// {(1,z),(4,x)}, {(2,z),(4,y)} are [[g,g],[g,g]]; {(3,x),(6,z)},
// {(3,y),(5,z)}, {(5,x),(6,y)} are [[d,e],[e,d]]; (7,c) is h.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace aarmr {

struct WalshConsts {
  double a1mb1, b1;  // 3x3 block at Walsh indices 1,2,4: diagonal - off, off
  double g;          // rotation-type pairs
  double d, e;       // [[d, e], [e, d]] pairs
  double a4mb4, b4;  // 3x3 block at Walsh indices 3,5,6
  double h;          // Walsh index 7
};

// z = w * B * what for the block structure of the unit-cube stiffness.
// what/z are indexed [k][c], k = Walsh index (kx + 2 ky + 4 kz), c = component.
template <typename T>
__host__ __device__ inline void walsh_blocks(const WalshConsts& K, T w, const T (&h)[8][3], T (&z)[8][3]) {
  using std::fma;
  const T a1 = w * (T)K.a1mb1, b1 = w * (T)K.b1, g = w * (T)K.g, d = w * (T)K.d,
          e = w * (T)K.e, a4 = w * (T)K.a4mb4, b4 = w * (T)K.b4, eta = w * (T)K.h;
  z[0][0] = z[0][1] = z[0][2] = (T)0;
  {  // {(1,x), (2,y), (4,z)}
    const T s = b1 * (h[1][0] + h[2][1] + h[4][2]);
    z[1][0] = fma(a1, h[1][0], s);
    z[2][1] = fma(a1, h[2][1], s);
    z[4][2] = fma(a1, h[4][2], s);
  }
  {  // rotation-type pairs [[g, g], [g, g]]
    const T t0 = g * (h[1][1] + h[2][0]);
    z[1][1] = t0;
    z[2][0] = t0;
    const T t1 = g * (h[1][2] + h[4][0]);
    z[1][2] = t1;
    z[4][0] = t1;
    const T t2 = g * (h[2][2] + h[4][1]);
    z[2][2] = t2;
    z[4][1] = t2;
  }
  {  // pairs [[d, e], [e, d]]
    z[3][0] = fma(d, h[3][0], e * h[6][2]);
    z[6][2] = fma(d, h[6][2], e * h[3][0]);
    z[3][1] = fma(d, h[3][1], e * h[5][2]);
    z[5][2] = fma(d, h[5][2], e * h[3][1]);
    z[5][0] = fma(d, h[5][0], e * h[6][1]);
    z[6][1] = fma(d, h[6][1], e * h[5][0]);
  }
  {  // {(3,z), (5,y), (6,x)}
    const T s = b4 * (h[3][2] + h[5][1] + h[6][0]);
    z[3][2] = fma(a4, h[3][2], s);
    z[5][1] = fma(a4, h[5][1], s);
    z[6][0] = fma(a4, h[6][0], s);
  }
  z[7][0] = eta * h[7][0];
  z[7][1] = eta * h[7][1];
  z[7][2] = eta * h[7][2];
}


}  // namespace aarmr
