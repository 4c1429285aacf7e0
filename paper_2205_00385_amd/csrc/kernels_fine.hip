// Fine-grid kernels: SIMP moduli (eq. 1), fixed-DOF mask, the diagonal of
// the stiffness operator (Jacobi smoother of Algorithm 2) and the
// sensitivity of eq. (6) from element energies.
#include "internal.hpp"

namespace aarmr {

namespace {

__device__ inline int64_t node_of(int nx, int ny, int i, int j, int k) {
  return (int64_t)i + (int64_t)(nx + 1) * ((int64_t)j + (int64_t)(ny + 1) * k);
}

// eq. (1): E = Emin + (E0 - Emin) rho~^p; flags rho~ outside [0, 1].
__global__ void k_simp(int64_t ne, const double* __restrict__ rho, double E0, double Emin,
                       double p, double* __restrict__ E, float* __restrict__ E32,
                       unsigned* __restrict__ bad) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  double r = rho[e];
  if (!(r >= 0.0 && r <= 1.0)) {  // also catches NaN
    atomicOr(bad, 1u);
    r = fmin(fmax(r, 0.0), 1.0);
    if (r != r) r = 0.0;
  }
  double v = Emin + (E0 - Emin) * pow(r, p);
  E[e] = v;
  if (E32) E32[e] = (float)v;
}

__global__ void k_diff(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                       double* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] - b[i];
}

__global__ void k_mask_clear(int64_t nn, uint32_t* mask_words) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (nn + 3) / 4) mask_words[i] = 0u;
}

__global__ void k_mask_set(int64_t nn, int ncomp, const int64_t* __restrict__ fixed, int64_t nf,
                           uint32_t* mask_words, unsigned* bad) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nf) return;
  int64_t d = fixed[t];
  if (d < 0 || d >= ncomp * nn) {
    atomicOr(bad, 2u);
    return;
  }
  int64_t node = d % nn;
  int c = (int)(d / nn);
  uint32_t bit = (1u << c) << (8 * (node & 3));
  atomicOr(&mask_words[node >> 2], bit);
}

// flags |= 4 if the two masks differ in any word (padding bytes are zero in
// both: the mask is cleared word-wise before its bits are set).
__global__ void k_mask_diff(int64_t nw, const uint32_t* __restrict__ a,
                            const uint32_t* __restrict__ b, unsigned* flags) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nw && a[t] != b[t]) atomicOr(flags, 4u);
}

// Jacobi diagonal of A: sum over adjacent elements of E_e * KE_(aa) per
// component; identity on fixed DOFs.  Stores the inverse.
__global__ void k_diag_fine(int nx, int ny, int nz, const double* __restrict__ KE,
                            const double* __restrict__ E, const uint8_t* __restrict__ mask,
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
        const double w = E[(int64_t)ex + (int64_t)nx * ((int64_t)ey + (int64_t)ny * ez)];
        for (int c = 0; c < 3; ++c) d[c] += w * KE[(3 * a + c) * 25];
      }
    }
  }
  const uint8_t m = mask[n];
  for (int c = 0; c < 3; ++c) {
    double di = (((m >> c) & 1) || d[c] == 0.0) ? 1.0 : 1.0 / d[c];
    dinv[c * nn + n] = di;
    if (dinv32) dinv32[c * nn + n] = (float)di;
  }
}

// dc (+)= -p rho~^(p-1) (E0 - Emin) e_e  (eq. 6 with eq. 1).
__global__ void k_dc_accum(int64_t ne, const double* __restrict__ rho,
                           const double* __restrict__ energy, double E0, double Emin, double p,
                           double* __restrict__ dc, int first) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  double r = fmin(fmax(rho[e], 0.0), 1.0);
  double v = -p * pow(r, p - 1.0) * (E0 - Emin) * energy[e];
  dc[e] = first ? v : dc[e] + v;
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

void launch_simp(int64_t ne, const double* rho, double E0, double Emin, double p, double* E,
                 float* E32, unsigned* bad, hipStream_t s) {
  k_simp<<<nblk(ne, 256), 256, 0, s>>>(ne, rho, E0, Emin, p, E, E32, bad);
}

void launch_diff(int64_t n, const double* a, const double* b, double* out, hipStream_t s) {
  k_diff<<<nblk(n, 256), 256, 0, s>>>(n, a, b, out);
}

void launch_build_mask(int64_t nn, const int64_t* fixed, int64_t nfixed, uint8_t* mask,
                       unsigned* bad, hipStream_t s, int ncomp) {
  uint32_t* w = reinterpret_cast<uint32_t*>(mask);
  k_mask_clear<<<nblk((nn + 3) / 4, 256), 256, 0, s>>>(nn, w);
  if (nfixed > 0) k_mask_set<<<nblk(nfixed, 256), 256, 0, s>>>(nn, ncomp, fixed, nfixed, w, bad);
}

void launch_mask_diff(int64_t nn, const uint8_t* a, const uint8_t* b, unsigned* flags,
                      hipStream_t s) {
  const int64_t nw = (nn + 3) / 4;
  k_mask_diff<<<nblk(nw, 256), 256, 0, s>>>(nw, reinterpret_cast<const uint32_t*>(a),
                                            reinterpret_cast<const uint32_t*>(b), flags);
}

void launch_diag_fine(const Grid& g, const double* KE, const double* E, const uint8_t* mask,
                      double* dinv, float* dinv32, hipStream_t s) {
  k_diag_fine<<<nblk(g.nn, 256), 256, 0, s>>>(g.nx, g.ny, g.nz, KE, E, mask, dinv, dinv32);
}

void launch_dc_accum(int64_t ne, const double* rho, const double* energy, double E0, double Emin,
                     double p, double* dc, int first, hipStream_t s) {
  k_dc_accum<<<nblk(ne, 256), 256, 0, s>>>(ne, rho, energy, E0, Emin, p, dc, first);
}

}  // namespace aarmr
