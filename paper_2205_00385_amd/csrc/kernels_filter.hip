// Density filter (eqs. 31-32), its adjoint (eq. 33) and the device-side
// bisection of the optimality-criteria update.
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
__global__ void __launch_bounds__(256) k_filter(int nx, int ny, int nz, double r, int R, int mode,
                                                const double* __restrict__ Hs,
                                                const double* __restrict__ in,
                                                double* __restrict__ out) {
  const int64_t ne = (int64_t)nx * ny * nz;
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int i = (int)(e % nx);
  const int64_t rest = e / nx;
  const int j = (int)(rest % ny), k = (int)(rest / ny);
  double s = 0.0;
  for (int dk = -R; dk <= R; ++dk) {
    const int kk = k + dk;
    if (kk < 0 || kk >= nz) continue;
    for (int dj = -R; dj <= R; ++dj) {
      const int jj = j + dj;
      if (jj < 0 || jj >= ny) continue;
      for (int di = -R; di <= R; ++di) {
        const int ii = i + di;
        if (ii < 0 || ii >= nx) continue;
        const double w = r - sqrt((double)(di * di + dj * dj + dk * dk));
        if (!(w > 0.0)) continue;
        const int64_t nb = (int64_t)ii + (int64_t)nx * ((int64_t)jj + (int64_t)ny * kk);
        s += mode == 0 ? w * in[nb] : w * in[nb] / Hs[nb];
      }
    }
  }
  out[e] = mode == 0 ? s / Hs[e] : s;
}

// lam[0] = l1, lam[1] = l2, lam[2] = current midpoint, lam[3] = done flag.
__global__ void k_oc_init(double* lam) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    lam[0] = 0.0;
    lam[1] = 1e9;
    lam[2] = 0.5e9;
    lam[3] = 0.0;
  }
}

__global__ void k_oc_step(int64_t ne, const double* __restrict__ x, const double* __restrict__ dc,
                          const double* __restrict__ dv, double move,
                          const double* __restrict__ lam, double* __restrict__ xnew) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne || lam[3] != 0.0) return;
  const double lmid = 0.5 * (lam[0] + lam[1]);
  const double B = fmax(0.0, -dc[e]) / dv[e];
  const double xe = x[e];
  double v = xe * sqrt(B / lmid);
  v = fmin(v, fmin(1.0, xe + move));
  v = fmax(v, fmax(0.0, xe - move));
  xnew[e] = v;
}

__global__ void k_oc_bisect(double* lam, const double* __restrict__ vol, double target) {
  if (threadIdx.x != 0 || blockIdx.x != 0 || lam[3] != 0.0) return;
  const double lmid = 0.5 * (lam[0] + lam[1]);
  lam[2] = lmid;
  if (*vol > target) lam[0] = lmid;
  else lam[1] = lmid;
  if ((lam[1] - lam[0]) / (lam[0] + lam[1]) <= 1e-3) lam[3] = 1.0;
}

}  // namespace

static int filter_reach(double r) { return (int)ceil(r) - 1; }

void launch_filter_rowsum(const Grid& g, double r, double* Hs, hipStream_t s) {
  k_filter_rowsum<<<nblk(g.ne, 256), 256, 0, s>>>(g.nx, g.ny, g.nz, r, filter_reach(r), Hs);
}

void launch_filter(const Grid& g, double r, int mode, const double* Hs, const double* in,
                   double* out, hipStream_t s) {
  k_filter<<<nblk(g.ne, 256), 256, 0, s>>>(g.nx, g.ny, g.nz, r, filter_reach(r), mode, Hs, in,
                                           out);
}

void launch_oc_init(double* lam, hipStream_t s) { k_oc_init<<<1, 64, 0, s>>>(lam); }

void launch_oc_step(int64_t ne, const double* x, const double* dc, const double* dv, double move,
                    double* lam, double* xnew, hipStream_t s) {
  k_oc_step<<<nblk(ne, 256), 256, 0, s>>>(ne, x, dc, dv, move, lam, xnew);
}

void launch_oc_bisect(double* lam, const double* vol, double target, hipStream_t s) {
  k_oc_bisect<<<1, 64, 0, s>>>(lam, vol, target);
}

}  // namespace aarmr
