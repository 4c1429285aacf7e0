// Vector kernels of CG and of the reduced model: deterministic FP64 dot
// products (wavefront shuffles, fixed-order block partials, a one-block
// finishing pass), CG updates whose scalars stay in device memory, linear
// combinations with device coefficients and small dense SPD solves.
#include "internal.hpp"

namespace aarmr {

namespace {

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Block (256 threads) sum in a fixed order; result valid in thread 0.
__device__ inline double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

// k dot products over n entries.  Pass 1: a grid of nb <= kRedBlocks blocks,
// each striding over the vectors in a fixed pattern, writes one partial per
// product.  Pass 2 (one block) sums the partials in index order.  Both
// passes have a fixed summation order, so results are bitwise reproducible;
// the kernel boundary orders the partial stores before their reads without
// any device-scope fence (each of which would write back an XCD's L2).
template <typename T>
__global__ void __launch_bounds__(256) k_multidot(DotSetT<T> d, double* __restrict__ partial) {
  __shared__ double sh[4];
  const int nb = gridDim.x;
  const int64_t stride = (int64_t)nb * 256;
  for (int k = 0; k < d.k; ++k) {
    const T* a = d.a[k];
    const T* b = d.b[k];
    double s = 0.0;
    if (b) {
      for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < d.n; i += stride)
        s = fma((double)a[i], (double)b[i], s);
    } else {  // plain sum
      for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < d.n; i += stride)
        s += (double)a[i];
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) partial[k * kRedBlocks + blockIdx.x] = s;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_multidot_finish(DotSetT<T> d, int nb,
                                                         const double* __restrict__ partial) {
  __shared__ double sh[4];
  for (int k = 0; k < d.k; ++k) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) s += partial[k * kRedBlocks + i];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) *d.out[k] = s;
  }
}

// The finished sum of nb block partials, in the order of k_multidot_finish
// (so bitwise the value that kernel writes); returned to every thread.
__device__ inline double finish_partials(const double* __restrict__ part, int nb, double* sh) {
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) s += part[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) sh[4] = s;
  __syncthreads();
  s = sh[4];
  __syncthreads();
  return s;
}

// CG step with its reductions folded in (grid-stride over gridDim.x blocks):
// p^T q is finished from the nb partials of k_multidot (block 0 stores it in
// *pq and in rr_part[gridDim.x], so one copy brings it to the host with the
// r^T r partials), alpha = *rz / p^T q, x += alpha p, r -= alpha q; the
// block partials of r^T r go to rr_part[blockIdx]; z0 = omega dinv r is the
// first Jacobi sweep of the next V-cycle (skipped when z0 is null).
__global__ void __launch_bounds__(256) k_cg_xr_fused(int64_t n, const double* __restrict__ rz,
                                                     const double* __restrict__ pq_part, int nb,
                                                     double* __restrict__ pq,
                                                     double* __restrict__ x,
                                                     double* __restrict__ r,
                                                     const double* __restrict__ p,
                                                     const double* __restrict__ q,
                                                     double* __restrict__ rr_part,
                                                     const double* __restrict__ dinv, double omega,
                                                     double* __restrict__ z0) {
  __shared__ double sh[5];
  const double pqv = finish_partials(pq_part, nb, sh);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *pq = pqv;
    rr_part[gridDim.x] = pqv;
  }
  const double alpha = *rz / pqv;
  const int64_t stride = (int64_t)gridDim.x * 256;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    x[i] = fma(alpha, p[i], x[i]);
    const double ri = fma(-alpha, q[i], r[i]);
    r[i] = ri;
    acc = fma(ri, ri, acc);
    if (z0) z0[i] = omega * dinv[i] * ri;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) rr_part[blockIdx.x] = acc;
}

// beta = rz_new / *rz_old with rz_new finished from the nb partials of
// k_multidot (block 0 stores it in *rz_new); p = z + beta p.
__global__ void __launch_bounds__(256) k_cg_p_fused(int64_t n, const double* __restrict__ rz_part,
                                                    int nb, double* __restrict__ rz_new,
                                                    const double* __restrict__ rz_old,
                                                    const double* __restrict__ z,
                                                    double* __restrict__ p) {
  __shared__ double sh[5];
  const double rzv = finish_partials(rz_part, nb, sh);
  if (blockIdx.x == 0 && threadIdx.x == 0) *rz_new = rzv;
  const double beta = rzv / *rz_old;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride)
    p[i] = fma(beta, p[i], z[i]);
}

// The FP32 CG step with its reductions folded in, as k_cg_xr_fused: FP32
// vectors, FP64 scalars and partials.  Block 0 also stores *rz beside p^T q
// (rr_part[gridDim.x + 1]) so that the host sees both signs the stall test
// needs.  z0 = omega dinv r in FP32, the V-cycle's first sweep.
__global__ void __launch_bounds__(256) k_cg_xr_fused_f32(int64_t n, const double* __restrict__ rz,
                                                         const double* __restrict__ pq_part,
                                                         int nb, double* __restrict__ pq,
                                                         float* __restrict__ x,
                                                         float* __restrict__ r,
                                                         const float* __restrict__ p,
                                                         const float* __restrict__ q,
                                                         double* __restrict__ rr_part,
                                                         const float* __restrict__ dinv,
                                                         float omega, float* __restrict__ z0,
                                                         int64_t vs = 0, int ss = 0, int ps = 0,
                                                         int hs = 0,
                                                         const int* __restrict__ active = nullptr) {
  __shared__ double sh[5];
  {  // load case blockIdx.z of a lock-step solve; a finished case is left as it is
    const int l = blockIdx.z;
    if (active && !active[l]) return;  // workgroup-uniform
    rz += l * ss;
    pq += l * ss;
    pq_part += l * ps;
    rr_part += l * hs;
    x += l * vs;
    r += l * vs;
    p += l * vs;
    q += l * vs;
    z0 += l * vs;
  }
  const double pqv = finish_partials(pq_part, nb, sh);
  const double rzv = *rz;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *pq = pqv;
    rr_part[gridDim.x] = pqv;
    rr_part[gridDim.x + 1] = rzv;
  }
  const double alpha = rzv / pqv;
  const int64_t stride = (int64_t)gridDim.x * 256;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    x[i] = (float)fma(alpha, (double)p[i], (double)x[i]);
    const float ri = (float)fma(-alpha, (double)q[i], (double)r[i]);
    r[i] = ri;
    acc = fma((double)ri, (double)ri, acc);
    z0[i] = omega * dinv[i] * ri;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) rr_part[blockIdx.x] = acc;
}

// beta = rz_new / *rz_old, rz_new finished from nb FP64 partials (block 0
// stores it); p = z + beta p in FP32 vectors.
__global__ void __launch_bounds__(256) k_cg_p_fused_f32(int64_t n, const double* __restrict__ rz_part,
                                                        int nb, double* __restrict__ rz_new,
                                                        const double* __restrict__ rz_old,
                                                        const float* __restrict__ z,
                                                        float* __restrict__ p, int64_t vs = 0,
                                                        int ss = 0, int ps = 0,
                                                        const int* __restrict__ active = nullptr) {
  __shared__ double sh[5];
  {  // load case blockIdx.z of a lock-step solve
    const int l = blockIdx.z;
    if (active && !active[l]) return;  // workgroup-uniform
    rz_part += l * ps;
    rz_new += l * ss;
    rz_old += l * ss;
    z += l * vs;
    p += l * vs;
  }
  const double rzv = finish_partials(rz_part, nb, sh);
  if (blockIdx.x == 0 && threadIdx.x == 0) *rz_new = rzv;
  const double beta = rzv / *rz_old;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride)
    p[i] = (float)fma(beta, (double)p[i], (double)z[i]);
}

__global__ void k_copy_masked(int64_t nn, int ncomp, const double* __restrict__ src,
                              const uint8_t* __restrict__ mask, double* __restrict__ dst) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncomp * nn) return;
  const int c = (int)(i / nn);
  const int64_t n = i - c * nn;
  dst[i] = ((mask[n] >> c) & 1) ? 0.0 : src[i];
}

__global__ void k_sub(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                      double* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] - b[i];
}

__global__ void k_scale_inv_sqrt(int64_t n, const double* __restrict__ src,
                                 const double* __restrict__ nrm2, double* __restrict__ dst) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double s = *nrm2 > 0.0 ? 1.0 / sqrt(*nrm2) : 0.0;  // a zero vector stays zero
  dst[i] = src[i] * s;
}

__global__ void k_cg_p_f32(int64_t n, const double* __restrict__ rz_new,
                           const double* __restrict__ rz_old, const float* __restrict__ z,
                           float* __restrict__ p) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double beta = *rz_new / *rz_old;
  p[i] = (float)fma(beta, (double)p[i], (double)z[i]);
}

__global__ void k_to_f32(int64_t n, const double* __restrict__ src, float* __restrict__ dst) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

__global__ void k_to_f32_scaled(int64_t n, const double* __restrict__ src,
                                const double* __restrict__ nrm2, float* __restrict__ dst) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  dst[i] = (float)(src[i] / sqrt(*nrm2));
}

__global__ void k_add_scaled_f32(int64_t n, const float* __restrict__ d,
                                 const double* __restrict__ nrm2, double* __restrict__ x) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  x[i] = fma(sqrt(*nrm2), (double)d[i], x[i]);
}

__global__ void k_copy_f32(int64_t n, const float* __restrict__ src, float* __restrict__ dst) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// Thin SVD T = U Sigma V^T of a small n x n matrix (row-major T[i * n + j],
// n <= 2 * AARMR_MAX_BASIS) by one-sided Jacobi in one thread: rotate column
// pairs of A = T (and V) until their inner products vanish, then
// sigma_j = |A_j|, U_j = A_j / sigma_j, sorted by decreasing sigma.
// Writes U_j for sigma_j > tau sigma_1 column by column (coef[j * n + i] =
// U[i][j]) and their count (as a double) to *kept.
__global__ void k_small_svd(int n, const double* __restrict__ T, double tau,
                            double* __restrict__ coef, double* __restrict__ kept) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  constexpr int N = 2 * AARMR_MAX_BASIS;
  double A[N][N];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) A[i][j] = T[i * n + j];
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double a = 0.0, b = 0.0, g = 0.0;
        for (int i = 0; i < n; ++i) {
          a += A[i][p] * A[i][p];
          b += A[i][q] * A[i][q];
          g += A[i][p] * A[i][q];
        }
        if (!(fabs(g) > 1e-15 * sqrt(a * b)) || g == 0.0) continue;
        rotated = true;
        const double zeta = (b - a) / (2.0 * g);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
        for (int i = 0; i < n; ++i) {
          const double x = A[i][p], y = A[i][q];
          A[i][p] = c * x - sn * y;
          A[i][q] = sn * x + c * y;
        }
      }
    if (!rotated) break;
  }
  double sig[N];
  int ord[N];
  for (int j = 0; j < n; ++j) {
    double s2 = 0.0;
    for (int i = 0; i < n; ++i) s2 += A[i][j] * A[i][j];
    sig[j] = sqrt(s2);
    ord[j] = j;
  }
  for (int a = 0; a < n; ++a)  // selection sort, decreasing sigma
    for (int b = a + 1; b < n; ++b)
      if (sig[ord[b]] > sig[ord[a]]) {
        const int t = ord[a];
        ord[a] = ord[b];
        ord[b] = t;
      }
  int k = 0;
  const double s1 = n > 0 ? sig[ord[0]] : 0.0;
  for (int j = 0; j < n; ++j) {
    const int c = ord[j];
    if (!(sig[c] > tau * s1) || sig[c] == 0.0) break;
    for (int i = 0; i < n; ++i) coef[k * n + i] = A[i][c] / sig[c];
    ++k;
  }
  *kept = (double)k;
}

struct VecList {
  const double* v[2 * AARMR_MAX_BASIS];
};

// out = add + sign * sum_j coef[j] V_j   (add may be null)
__global__ void k_lincomb(int64_t n, int k, VecList V, const double* __restrict__ coef,
                          double sign, const double* __restrict__ add, double* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int j = 0; j < k; ++j) s = fma(coef[j], V.v[j][i], s);
  out[i] = add ? fma(sign, s, add[i]) : sign * s;
}

// Solve A x = b for a small SPD matrix (row-major, leading dimension lda) by
// Cholesky in one thread; flags a non-positive pivot.
// Cholesky solve of the small SPD system A x = b (entries averaged with
// their transpose); one that is not positive definite sets bit 4 of *bad
// and gives x = 0.  One thread.
__global__ void k_small_spd_solve(int n, int lda, const double* __restrict__ A,
                                  const double* __restrict__ b, double* __restrict__ x,
                                  unsigned* bad) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double L[2 * AARMR_MAX_BASIS][2 * AARMR_MAX_BASIS];
  double y[2 * AARMR_MAX_BASIS];
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j <= i; ++j) {
      double s = 0.5 * (A[i * lda + j] + A[j * lda + i]);
      for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
      if (i == j) {
        if (!(s > 0.0)) {
          atomicOr(bad, 4u);
          for (int t = 0; t < n; ++t) x[t] = 0.0;
          return;
        }
        L[i][i] = sqrt(s);
      } else {
        L[i][j] = s / L[j][j];
      }
    }
  }
  for (int i = 0; i < n; ++i) {
    double s = b[i];
    for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
    y[i] = s / L[i][i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = y[i];
    for (int k = i + 1; k < n; ++k) s -= L[k][i] * x[k];
    x[i] = s / L[i][i];
  }
}

// Gram-Schmidt keep test: with n0 = ||v||^2 before and n1 after the
// projections, a column with sqrt(n1) > tau sqrt(n0) is scaled to unit norm
// (dst = src / sqrt(n1)) and *keep = 1; any other becomes zero, *keep = 0.
__global__ void k_gs_keep(int64_t n, const double* __restrict__ src,
                          const double* __restrict__ n0, const double* __restrict__ n1,
                          double tau, double* __restrict__ dst, double* __restrict__ keep) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double a = *n0, b = *n1;
  const bool k = sqrt(b) > tau * sqrt(a);
  const double sc = 1.0 / sqrt(b);
  if (i < n) dst[i] = k ? src[i] * sc : 0.0;  // exact zeros, also for a non-finite column
  if (i == 0) *keep = k ? 1.0 : 0.0;
}

}  // namespace

template <typename T>
void multidot_t(const DotSetT<T>& d, const RedScratch& rs, hipStream_t s) {
  int64_t want = (d.n + 255) / 256;
  int nb = (int)(want < kRedBlocks ? (want < 1 ? 1 : want) : kRedBlocks);
  k_multidot<T><<<nb, 256, 0, s>>>(d, rs.partial);
  k_multidot_finish<T><<<1, 256, 0, s>>>(d, nb, rs.partial);
}

void launch_multidot(const DotSet& d, const RedScratch& rs, hipStream_t s) {
  multidot_t<double>(d, rs, s);
}

int dot_blocks(int64_t n) {
  const int64_t want = (n + 255) / 256;
  return (int)(want < kRedBlocks ? (want < 1 ? 1 : want) : kRedBlocks);
}

int fused_blocks(int64_t n) {
  const int64_t want = (n + 1023) / 1024;  // about four entries per thread
  return (int)(want < kFusedBlocks ? (want < 1 ? 1 : want) : kFusedBlocks);
}

void launch_dot_partials(int64_t n, const double* a, const double* b, double* part,
                         hipStream_t s) {
  DotSet d{};
  d.k = 1;
  d.n = n;
  d.a[0] = a;
  d.b[0] = b;
  k_multidot<double><<<dot_blocks(n), 256, 0, s>>>(d, part);
}

void launch_cg_xr_fused(int64_t n, const double* rz, const double* pq_part, int n_part,
                        double* pq, double* x, double* r, const double* p, const double* q,
                        double* rr_part, const double* dinv, double omega, double* z0,
                        hipStream_t s) {
  k_cg_xr_fused<<<fused_blocks(n), 256, 0, s>>>(n, rz, pq_part, n_part > 0 ? n_part : dot_blocks(n),
                                                pq, x, r, p, q, rr_part, dinv, omega, z0);
}

void launch_cg_p_fused(int64_t n, const double* rz_part, int n_part, double* rz_new,
                       const double* rz_old, const double* z, double* p, hipStream_t s) {
  k_cg_p_fused<<<fused_blocks(n), 256, 0, s>>>(n, rz_part, n_part > 0 ? n_part : dot_blocks(n),
                                               rz_new, rz_old, z, p);
}

void launch_multidot_f32(const DotSetT<float>& d, const RedScratch& rs, hipStream_t s) {
  multidot_t<float>(d, rs, s);
}

void launch_cg_xr_fused_f32(int64_t n, const double* rz, const double* pq_part, int n_part,
                            double* pq, float* x, float* r, const float* p, const float* q,
                            double* rr_part, const float* dinv, float omega, float* z0,
                            hipStream_t s, const MultiRhs& mr) {
  k_cg_xr_fused_f32<<<dim3(fused_blocks(n), 1, mr.n), 256, 0, s>>>(
      n, rz, pq_part, n_part, pq, x, r, p, q, rr_part, dinv, omega, z0, mr.vs, mr.ss, mr.ps,
      mr.hs, mr.active);
}

void launch_cg_p_fused_f32(int64_t n, const double* rz_part, int n_part, double* rz_new,
                           const double* rz_old, const float* z, float* p, hipStream_t s,
                           const MultiRhs& mr) {
  k_cg_p_fused_f32<<<dim3(fused_blocks(n), 1, mr.n), 256, 0, s>>>(
      n, rz_part, n_part, rz_new, rz_old, z, p, mr.vs, mr.ss, mr.ps, mr.active);
}

void launch_cg_p_f32(int64_t n, const double* rz_new, const double* rz_old, const float* z,
                     float* p, hipStream_t s) {
  k_cg_p_f32<<<nblk(n, 256), 256, 0, s>>>(n, rz_new, rz_old, z, p);
}

void launch_to_f32(int64_t n, const double* src, float* dst, hipStream_t s) {
  k_to_f32<<<nblk(n, 256), 256, 0, s>>>(n, src, dst);
}

void launch_to_f32_scaled(int64_t n, const double* src, const double* nrm2, float* dst,
                          hipStream_t s) {
  k_to_f32_scaled<<<nblk(n, 256), 256, 0, s>>>(n, src, nrm2, dst);
}

void launch_add_scaled_f32(int64_t n, const float* d, const double* nrm2, double* x,
                           hipStream_t s) {
  k_add_scaled_f32<<<nblk(n, 256), 256, 0, s>>>(n, d, nrm2, x);
}

void launch_copy_f32(int64_t n, const float* src, float* dst, hipStream_t s) {
  k_copy_f32<<<nblk(n, 256), 256, 0, s>>>(n, src, dst);
}

void launch_copy_masked(const Grid& g, const double* src, const uint8_t* mask, double* dst,
                        hipStream_t s, int ncomp) {
  k_copy_masked<<<nblk(ncomp * g.nn, 256), 256, 0, s>>>(g.nn, ncomp, src, mask, dst);
}

void launch_sub(int64_t n, const double* a, const double* b, double* out, hipStream_t s) {
  k_sub<<<nblk(n, 256), 256, 0, s>>>(n, a, b, out);
}


void launch_scale_by_inv_sqrt(int64_t n, const double* src, const double* nrm2, double* dst,
                              hipStream_t s) {
  k_scale_inv_sqrt<<<nblk(n, 256), 256, 0, s>>>(n, src, nrm2, dst);
}

void launch_lincomb(int64_t n, int k, const double* const* V, const double* coef, double sign,
                    const double* add, double* out, hipStream_t s) {
  VecList L;
  for (int j = 0; j < 2 * AARMR_MAX_BASIS; ++j) L.v[j] = j < k ? V[j] : nullptr;
  k_lincomb<<<nblk(n, 256), 256, 0, s>>>(n, k, L, coef, sign, add, out);
}

void launch_small_svd(int n, const double* T, double tau, double* coef, double* kept,
                      hipStream_t s) {
  k_small_svd<<<1, 64, 0, s>>>(n, T, tau, coef, kept);
}

void launch_small_spd_solve(int n, int lda, const double* A, const double* b, double* x,
                            unsigned* bad, hipStream_t s) {
  k_small_spd_solve<<<1, 64, 0, s>>>(n, lda, A, b, x, bad);
}

void launch_gs_keep(int64_t n, const double* src, const double* n0, const double* n1, double tau,
                    double* dst, double* keep, hipStream_t s) {
  k_gs_keep<<<nblk(n, 256), 256, 0, s>>>(n, src, n0, n1, tau, dst, keep);
}

}  // namespace aarmr
