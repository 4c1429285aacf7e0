// Density filter (eqs. 31-32), its adjoint (eq. 33) and the device-side
// bisection of the optimality-criteria update.
#include <cmath>

#include "internal.hpp"

namespace aarmr {

namespace {

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Hs_e = sum of in-domain cone weights max(0, r - |d|) around element e.
__global__ void k_filter_rowsum(int nx, int ny, int nz, double r, int R, double* __restrict__ Hs) {
  const int64_t ne = (int64_t)nx * ny * nz;
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int i = (int)(e % nx);
  const int64_t rest = e / nx;
  const int j = (int)(rest % ny), k = (int)(rest / ny);
  double s = 0.0;
  for (int dk = -R; dk <= R; ++dk) {
    if (k + dk < 0 || k + dk >= nz) continue;
    for (int dj = -R; dj <= R; ++dj) {
      if (j + dj < 0 || j + dj >= ny) continue;
      for (int di = -R; di <= R; ++di) {
        if (i + di < 0 || i + di >= nx) continue;
        const double w = r - sqrt((double)(di * di + dj * dj + dk * dk));
        if (w > 0.0) s += w;
      }
    }
  }
  Hs[e] = s;
}

// mode 0: out_e = sum_j w_ej in_j / Hs_e;  mode 1: out_e = sum_i w_ie in_i / Hs_i.
// W holds the cone weights max(0, r - |d|) of the (2R+1)^3 offsets
// (dk, dj, di), di fastest; zero weights are summed too (adding +0 changes
// nothing).  RC > 0 fixes R at compile time; elements whose neighbourhood
// lies inside the grid take an unrolled path without bounds checks.
template <int RC>
__global__ void __launch_bounds__(256) k_filter(int nx, int ny, int nz, int Rrt, int mode,
                                                const double* __restrict__ W,
                                                const double* __restrict__ Hs,
                                                const double* __restrict__ in,
                                                double* __restrict__ out) {
  const int R = RC > 0 ? RC : Rrt;
  const int D = 2 * R + 1;
  const int64_t ne = (int64_t)nx * ny * nz;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int i = (int)(e % nx);
  const int64_t rest = e / nx;
  const int j = (int)(rest % ny), k = (int)(rest / ny);
  const int64_t sy = nx, sz = (int64_t)nx * ny;
  double s = 0.0;
  const bool inside = i >= R && i < nx - R && j >= R && j < ny - R && k >= R && k < nz - R;
  if (RC > 0 && inside && mode == 0) {
#pragma unroll
    for (int dk = -RC; dk <= RC; ++dk)
#pragma unroll
      for (int dj = -RC; dj <= RC; ++dj)
#pragma unroll
        for (int di = -RC; di <= RC; ++di)
          s = fma(W[((dk + RC) * D + (dj + RC)) * D + (di + RC)], in[e + di + sy * dj + sz * dk], s);
  } else {
    for (int dk = -R; dk <= R; ++dk) {
      const int kk = k + dk;
      if (kk < 0 || kk >= nz) continue;
      for (int dj = -R; dj <= R; ++dj) {
        const int jj = j + dj;
        if (jj < 0 || jj >= ny) continue;
        for (int di = -R; di <= R; ++di) {
          const int ii = i + di;
          if (ii < 0 || ii >= nx) continue;
          const double w = W[((dk + R) * D + (dj + R)) * D + (di + R)];
          const int64_t nb = e + di + sy * dj + sz * dk;
          s = mode == 0 ? fma(w, in[nb], s) : fma(w, in[nb] / Hs[nb], s);
        }
      }
    }
  }
  out[e] = mode == 0 ? s / Hs[e] : s;
}

// lam[0] = l1, lam[1] = l2, lam[2] = current midpoint, lam[3] = done flag,
// lam[4] = bisection steps taken (at most 200).
__global__ void k_oc_init(double* lam) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    lam[0] = 0.0;
    lam[1] = 1e9;
    lam[2] = 0.5e9;
    lam[3] = 0.0;
    lam[4] = 0.0;
  }
}

// The OC update of one element at multiplier lmid.
__device__ inline double oc_x(double xe, double B, double lmid, double move, double eta) {
  double v = xe * (eta == 0.5 ? sqrt(B / lmid) : pow(B / lmid, eta));
  v = fmin(v, fmin(1.0, xe + move));
  return fmax(v, fmax(0.0, xe - move));
}

// Three bisection levels per launch.  The seven multipliers a three-level
// bisection of [lam[0], lam[1]] can visit, in heap order (t: midpoint;
// 2t + 1: its left half's midpoint, 2t + 2: its right half's), computed with
// the same expressions the one-level steps would use; for each, block
// partials of sum_j c_j x_new_j, the volume of the filtered x_new (c =
// H^T (1 / Hs), the column weights of the normalised filter), in the
// summation order of a one-level step, so every decision is bitwise the one
// the one-level bisection takes.
__global__ void __launch_bounds__(256) k_oc_step3(int64_t ne, const double* __restrict__ x,
                                                  const double* __restrict__ dc,
                                                  const double* __restrict__ dv,
                                                  const double* __restrict__ cw, double move,
                                                  double eta, const double* __restrict__ lam,
                                                  double* __restrict__ partial) {
  __shared__ double red[7][4];
  if (lam[3] != 0.0) return;  // block-uniform
  const double l1 = lam[0], l2 = lam[1];
  double lm[7];
  lm[0] = 0.5 * (l1 + l2);
  lm[1] = 0.5 * (l1 + lm[0]);
  lm[2] = 0.5 * (lm[0] + l2);
  lm[3] = 0.5 * (l1 + lm[1]);
  lm[4] = 0.5 * (lm[1] + lm[0]);
  lm[5] = 0.5 * (lm[0] + lm[2]);
  lm[6] = 0.5 * (lm[2] + l2);
  double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double B = fmax(0.0, -dc[e]) / dv[e];
    const double xe = x[e], c = cw[e];
#pragma unroll
    for (int t = 0; t < 7; ++t) acc[t] = fma(c, oc_x(xe, B, lm[t], move, eta), acc[t]);
  }
#pragma unroll
  for (int t = 0; t < 7; ++t) {
    double a = acc[t];
    for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
    if ((threadIdx.x & 63) == 0) red[t][threadIdx.x >> 6] = a;
  }
  __syncthreads();
  if (threadIdx.x < 7) {
    const int t = threadIdx.x;
    partial[t * kRedBlocks + blockIdx.x] = (red[t][0] + red[t][1]) + (red[t][2] + red[t][3]);
  }
}

// The volumes of the seven multipliers (partials summed in a fixed order),
// then up to three bisection steps along the path the decisions take; lam[2]
// records the last multiplier evaluated, lam[3] = 1 once (l2-l1)/(l1+l2) <= 1e-3
// or after the 200th step.
__global__ void __launch_bounds__(512) k_oc_bisect3(double* lam, const double* __restrict__ partial,
                                                    int nparts, double target) {
  __shared__ double vol[7];
  if (lam[3] != 0.0) return;
  const int t = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (t < 7) {  // wave t sums trial t's partials
    double acc = 0.0;
    for (int b = lane; b < nparts; b += 64) acc += partial[t * kRedBlocks + b];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) vol[t] = acc;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  int h = 0;  // heap index of the multiplier evaluated next
  for (int level = 0; level < 3 && lam[3] == 0.0; ++level) {
    const double lmid = 0.5 * (lam[0] + lam[1]);
    lam[2] = lmid;
    if (vol[h] > target) {
      lam[0] = lmid;
      h = 2 * h + 2;
    } else {
      lam[1] = lmid;
      h = 2 * h + 1;
    }
    lam[4] += 1.0;
    if ((lam[1] - lam[0]) / (lam[0] + lam[1]) <= 1e-3 || lam[4] >= 200.0) lam[3] = 1.0;
  }
}

// x_new at the last multiplier the bisection evaluated.
__global__ void k_oc_final(int64_t ne, const double* __restrict__ x, const double* __restrict__ dc,
                           const double* __restrict__ dv, double move, double eta,
                           const double* __restrict__ lam, double* __restrict__ xnew) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  xnew[e] = oc_x(x[e], fmax(0.0, -dc[e]) / dv[e], lam[2], move, eta);
}

template <typename T>
__global__ void k_fill(int64_t n, T v, T* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = v;
}

}  // namespace

static int filter_reach(double r) { return (int)ceil(r) - 1; }

void filter_weights(double r, double* W) {
  const int R = filter_reach(r), D = 2 * R + 1;
  for (int dk = -R; dk <= R; ++dk)
    for (int dj = -R; dj <= R; ++dj)
      for (int di = -R; di <= R; ++di) {
        const double w = r - std::sqrt((double)(di * di + dj * dj + dk * dk));
        W[((dk + R) * D + (dj + R)) * D + (di + R)] = w > 0.0 ? w : 0.0;
      }
}

int filter_taps(double r) {
  const int D = 2 * filter_reach(r) + 1;
  return D * D * D;
}

void launch_filter_rowsum(const Grid& g, double r, double* Hs, hipStream_t s) {
  k_filter_rowsum<<<nblk(g.ne, 256), 256, 0, s>>>(g.nx, g.ny, g.nz, r, filter_reach(r), Hs);
}

void launch_filter(const Grid& g, double r, const double* W, int mode, const double* Hs,
                   const double* in, double* out, hipStream_t s) {
  const int R = filter_reach(r);
  const unsigned nb = nblk(g.ne, 256);
  switch (R) {
    case 1: k_filter<1><<<nb, 256, 0, s>>>(g.nx, g.ny, g.nz, R, mode, W, Hs, in, out); break;
    case 2: k_filter<2><<<nb, 256, 0, s>>>(g.nx, g.ny, g.nz, R, mode, W, Hs, in, out); break;
    default: k_filter<0><<<nb, 256, 0, s>>>(g.nx, g.ny, g.nz, R, mode, W, Hs, in, out); break;
  }
}

void launch_fill(int64_t n, double v, double* out, hipStream_t s) {
  k_fill<double><<<nblk(n, 256), 256, 0, s>>>(n, v, out);
}

void launch_fill_f32(int64_t n, float v, float* out, hipStream_t s) {
  k_fill<float><<<nblk(n, 256), 256, 0, s>>>(n, v, out);
}

void launch_oc_init(double* lam, hipStream_t s) { k_oc_init<<<1, 64, 0, s>>>(lam); }

void launch_oc_step3(int64_t ne, const double* x, const double* dc, const double* dv,
                     const double* cw, double move, double eta, const double* lam,
                     double* partial, int nparts, hipStream_t s) {
  k_oc_step3<<<nparts, 256, 0, s>>>(ne, x, dc, dv, cw, move, eta, lam, partial);
}

void launch_oc_bisect3(double* lam, const double* partial, int nparts, double target,
                       hipStream_t s) {
  k_oc_bisect3<<<1, 512, 0, s>>>(lam, partial, nparts, target);
}

void launch_oc_final(int64_t ne, const double* x, const double* dc, const double* dv, double move,
                     double eta, const double* lam, double* xnew, hipStream_t s) {
  k_oc_final<<<nblk(ne, 256), 256, 0, s>>>(ne, x, dc, dv, move, eta, lam, xnew);
}

}  // namespace aarmr
