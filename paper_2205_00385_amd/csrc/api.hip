// C ABI of the AARMR analysis step: host orchestration of the HIP kernels.
//
// The host validates arguments, binds workspace views, issues kernels on the
// caller's stream and reads back the few scalars that steer control flow
// (CG convergence, Gram-Schmidt rank decisions, the eq. (29) accept/reject
// branch).  Every arithmetic step of the method runs on the GPU.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "internal.hpp"

using namespace aarmr;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

// Static scratch of the allocation-free OC update: the bisection state
// (5 doubles, padded to 8) and the volume partials of the seven trial
// multipliers, [7][kRedBlocks].  Each GPU holds its own copy until the
// process ends; host code must use the address hipGetSymbolAddress returns
// for the current device, never the array's name.
constexpr int kOcScratchLam = 8;
constexpr int kOcScratchDoubles = kOcScratchLam + 7 * kRedBlocks;
static __device__ __align__(256) double oc_scratch[kOcScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

int oc_scratch_ptr(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(AARMR_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(AARMR_E_INVALID, "device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(oc_scratch));
    if (e != hipSuccess || !ptr)
      return fail(AARMR_E_HIP, std::string("hipGetSymbolAddress(oc_scratch): ") +
                                   hipGetErrorString(e));
    g_scratch_dev[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_dev[dev];
  return AARMR_OK;
}

#define HIP_TRY(x)                                                               \
  do {                                                                           \
    hipError_t e_ = (x);                                                         \
    if (e_ != hipSuccess)                                                        \
      return fail(AARMR_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)
#define KCHECK() HIP_TRY(hipGetLastError())
#define TRY(x)                 \
  do {                         \
    int rc_ = (x);             \
    if (rc_ != AARMR_OK) return rc_; \
  } while (0)

struct LevelBuf {
  double* Ke = nullptr;    // levels >= 1: packed Galerkin element matrices [300][ne]
  double* dinv = nullptr;  // [3][nn] inverse Jacobi diagonal
  double* b = nullptr;     // levels >= 1: right-hand side
  double* x = nullptr;     // levels >= 1: correction
  double* t = nullptr;     // [3][nn] operator output
  // FP32 copies for the refinement form's V-cycle (same roles)
  float* dinv32 = nullptr;
  float* b32 = nullptr;
  float* x32 = nullptr;
  float* t32 = nullptr;
  float* Ke32 = nullptr;  // 3D levels >= 2: FP32 copy of Ke for the FP32 V-cycle
};

// Scalar history in device memory (indices into m->scal).
constexpr int SC_RZ = 0;
constexpr int SC_PQ = SC_RZ + kMaxIt + 2;
constexpr int SC_RR = SC_PQ + kMaxIt + 2;
constexpr int SC_MISC = SC_RR + kMaxIt + 2;  // 512 misc scalars
constexpr int SC_TOTAL = SC_MISC + 512;
// misc slots
constexpr int M_FF = 0, M_RR0 = 1, M_NRM = 2, M_C = 3, M_EPS = 4, M_VOL = 5;
constexpr int M_RR64 = 6;      // FP64 residual norm^2 of a refinement step
constexpr int M_OC = 8;        // 5 slots: l1, l2, lmid, done, steps
constexpr int M_KPHI = 16;     // Ns*Ns
constexpr int M_G = 120;       // Ns  (Phi^T dK r)
constexpr int M_C2 = 132;      // Ns  (K_Phi^-1 g)
constexpr int M_H = 144;       // up to 10 GS coefficients
constexpr int M_FR = 156;      // reduced rhs
constexpr int M_Y = 168;       // reduced solution
constexpr int M_KR = 180;      // reduced matrix (up to 10x10, slots 180..279)
constexpr int M_SVC = 300;     // SVD basis coefficients (up to 10x10, slots 300..399)
constexpr int M_SVK = 400;     // SVD: number of kept singular vectors
constexpr int M_N0 = 410;      // GS: squared column norms before the projections (Nm)
constexpr int M_N1 = 420;      // GS: and after them (Nm)
constexpr int M_KEEP = 430;    // GS: 1 for a kept column, 0 for a dropped one (Nm)

constexpr int64_t kAlign = 256;

inline int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

}  // namespace

struct aarmr_mesh {
  aarmr_params p;
  Grid lg[AARMR_MAX_LEVELS];  // lg[0] = fine grid
  Grid fg;                    // element grid of the filter (nz >= 1)
  int dim = 3;                // 3: hex8 solid; 2: plane-stress Q4 (nz == 0)
  int nlev = 0;
  int nc = 0;                 // coarsest dense order
  double KE[576];             // 24x24 (3D) or 8x8 (2D) row-major
  WalshConsts wk;             // reflection-blocked form of KE (3D)
  double Mc[8 * kSymEntries]; // P_c^T KE P_c per child position, packed
  std::vector<double> N2;     // [300][64]: P_c1^T M_c0 P_c1 per fine descendant d = 8 c1 + c0 of a level-2 parent
  double Bw[576];             // W M_0 W / 64 in the Walsh x component basis
  float Bw32[576];
  bool fp32 = false;          // precision == AARMR_FP32_REFINE
  int tz64 = 0, tz32 = 0;     // tuned EbE z-chunk lengths (0: default)
  SpringSet springs{};        // grounded springs (plane stress)
  // workspace views
  char* ws = nullptr;
  int64_t ws_bytes = 0;
  double* KEd = nullptr;
  double* Mcd = nullptr;      // P_c^T KE P_c of the 8 children, packed
  double* N2d = nullptr;      // N2 on the device
  int* list2 = nullptr;       // level-2 parents with a flagged level-1 child
  int* count2 = nullptr;
  double* Bwd = nullptr;      // Bw on the device
  float* Bw32d = nullptr;
  double* Y1 = nullptr;       // level-1 element products [24][ne1]
  double* Kcomp1 = nullptr;   // compact copy of the flagged parents' matrices
  int cap1 = 0;               // its capacity (parents)
  int nflag1 = 0;             // flagged level-1 parents of the current hierarchy
  float* Y1f = nullptr;
  float* E32 = nullptr;       // FP32 moduli (refinement form)
  float *r32 = nullptr, *z32 = nullptr, *p32 = nullptr, *q32 = nullptr, *d32 = nullptr;
  uint8_t* eflag1 = nullptr;  // level-1 parents touching a fixed DOF
  int* list1 = nullptr;       // their indices
  int* count1 = nullptr;
  double* E = nullptr;
  double* E_prev = nullptr;
  double* dE = nullptr;
  double* rho_f = nullptr;
  double* Hs = nullptr;
  double* ework = nullptr;
  double* dc_tmp = nullptr;
  double* ones_dv = nullptr;  // all ones [ne]
  double* Wf = nullptr;       // filter weights of the offsets
  double* cw = nullptr;       // H^T (1 / Hs): volume weights of a filtered field
  std::vector<double> Wh;     // host copy of the filter weights
  uint8_t* mask = nullptr;
  double *r = nullptr, *z = nullptr, *pv = nullptr, *q = nullptr, *t0 = nullptr, *fm = nullptr;
  LevelBuf lv[AARMR_MAX_LEVELS];
  double* Ainv = nullptr;
  double *gjP = nullptr, *gjT = nullptr, *gjC = nullptr, *gjTb = nullptr;
  double* Phi = nullptr;   // [n_rhs_max][Ns][3nn]
  double* R = nullptr;     // [Nm][3nn]
  double* KR = nullptr;    // [Nm][3nn]
  double* scal = nullptr;
  double* partial = nullptr;
  double *part_pq = nullptr, *part_rz = nullptr;  // per-workgroup partials of the fine products
  int part_cap = 0;                               // their length per load case
  int* act = nullptr;      // lock-step solve: 1 for a load case still iterating [n_rhs_max]
  int* hact = nullptr;     // pinned host staging of act
  bool want_rz = false;  // the V-cycle's last fine sweep also forms r^T z partials
  int rz_nb = 0;         // how many it wrote (0: none)
  unsigned* flags = nullptr;
  // host state
  int phi_count[AARMR_MAX_RHS] = {};
  int phi_head[AARMR_MAX_RHS] = {};
  bool have_prev = false;
  bool mg_ready = false;
  double* hpin = nullptr;  // pinned host staging
  // CG's r^T r partials: coherent host memory the x/r update stores into
  // directly (host and device addresses), read by the host after an event
  double* hrr = nullptr;
  double* hrr_dev = nullptr;
  hipEvent_t ev_cg = nullptr;  // marks a CG iteration's scalar read-back
  // speculative hierarchy build beside the reduced-model step
  hipStream_t side = nullptr;
  hipEvent_t ev_fine = nullptr, ev_mg = nullptr;
  bool mg_pending = false;     // a build on `side` not yet joined into the caller's stream
  bool spec_mg = false;        // the last reduced-model attempt was rejected
  int oc_pairs = 0;            // OC launch pairs the last update needed
  int64_t sweeps = 0;
  // Reuse of the coarsest inverse across designs (AARMR_REUSE_COARSEST):
  // Ainv may stay the inverse of an earlier design's coarsest operator for
  // the same fixed DOFs while solves with it need few more iterations than
  // the first solve after the inversion did.
  uint8_t* mask_prev = nullptr;  // the mask Ainv was built for
  bool reuse_req = false;        // the running call allows reuse
  bool mask_changed = true;      // the last setup's mask differs from mask_prev
  bool ainv_valid = false;       // Ainv inverts some design's operator for mask_prev
  bool ainv_stale = false;       // the current hierarchy uses such an older inverse
  bool ainv_fresh = false;       // inverted for the current design; no solve yet
  bool ainv_rebuild = false;     // invert again at the next hierarchy build
  int ainv_base_its = 0;         // iterations of the first solve after the inversion
  int ainv_builds = 0, ainv_reuses = 0;
};

// A running batch: worker threads, each with its stream and queue of items.
struct aarmr_batch {
  aarmr_batch_item* items = nullptr;
  int n_items = 0;
  std::vector<void*> streams;
  std::vector<std::vector<int>> queue;
  std::vector<std::thread> pool;
  std::atomic<int> n_done{0};
};

namespace {

// ---- element stiffness of the unit cube (2x2x2 Gauss) ---------------------
void hex8_stiffness(double nu, double* KE) {
  const double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const double mu = 1.0 / (2.0 * (1.0 + nu));
  double D[6][6] = {};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) D[a][b] = lam;
  for (int a = 0; a < 3; ++a) D[a][a] = lam + 2.0 * mu;
  for (int a = 3; a < 6; ++a) D[a][a] = mu;
  const double g[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  std::memset(KE, 0, sizeof(double) * 576);
  for (double x : g)
    for (double y : g)
      for (double z : g) {
        double B[6][24] = {};
        for (int a = 0; a < 8; ++a) {
          const int i = a & 1, j = (a >> 1) & 1, k = a >> 2;
          const double fx = i ? x : 1 - x, fy = j ? y : 1 - y, fz = k ? z : 1 - z;
          const double sx = i ? 1 : -1, sy = j ? 1 : -1, sz = k ? 1 : -1;
          const double dx = sx * fy * fz, dy = fx * sy * fz, dz = fx * fy * sz;
          B[0][3 * a] = dx;
          B[1][3 * a + 1] = dy;
          B[2][3 * a + 2] = dz;
          B[3][3 * a] = dy;
          B[3][3 * a + 1] = dx;
          B[4][3 * a + 1] = dz;
          B[4][3 * a + 2] = dy;
          B[5][3 * a] = dz;
          B[5][3 * a + 2] = dx;
        }
        for (int r = 0; r < 24; ++r)
          for (int c = 0; c < 24; ++c) {
            double s = 0.0;
            for (int u = 0; u < 6; ++u)
              for (int v = 0; v < 6; ++v) s += B[u][r] * D[u][v] * B[v][c];
            KE[r * 24 + c] += 0.125 * s;
          }
      }
}

// Plane-stress element stiffness of the unit square (unit thickness and
// modulus), 2x2 Gauss; DOF 2a + c of corner a = dx + 2 dy.
void q4_stiffness(double nu, double* KE) {
  const double c0 = 1.0 / (1.0 - nu * nu);
  const double D[3][3] = {{c0, c0 * nu, 0.0}, {c0 * nu, c0, 0.0}, {0.0, 0.0, c0 * 0.5 * (1.0 - nu)}};
  const double g[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  std::memset(KE, 0, sizeof(double) * 64);
  for (double x : g)
    for (double y : g) {
      double B[3][8] = {};
      for (int a = 0; a < 4; ++a) {
        const int i = a & 1, j = a >> 1;
        const double dx = (i ? 1.0 : -1.0) * (j ? y : 1 - y);
        const double dy = (i ? x : 1 - x) * (j ? 1.0 : -1.0);
        B[0][2 * a] = dx;
        B[1][2 * a + 1] = dy;
        B[2][2 * a] = dy;
        B[2][2 * a + 1] = dx;
      }
      for (int r = 0; r < 8; ++r)
        for (int c = 0; c < 8; ++c) {
          double s = 0.0;
          for (int u = 0; u < 3; ++u)
            for (int v = 0; v < 3; ++v) s += B[u][r] * D[u][v] * B[v][c];
          KE[r * 8 + c] += 0.25 * s;
        }
    }
}

// Constants of the reflection-blocked form B = W KE W^T / 64 and a check
// that walsh_blocks() (the exact formula the kernels evaluate) reproduces
// every column of B.  Returns false if KE lacks that structure.
bool walsh_form(const double* KE, WalshConsts* K) {
  auto chi = [](int k, int a) { return (__builtin_popcount(k & a) & 1) ? -1.0 : 1.0; };
  double B[24][24];
  double bmax = 0.0;
  for (int k = 0; k < 8; ++k)
    for (int c = 0; c < 3; ++c)
      for (int k2 = 0; k2 < 8; ++k2)
        for (int c2 = 0; c2 < 3; ++c2) {
          double s = 0.0;
          for (int a = 0; a < 8; ++a)
            for (int b = 0; b < 8; ++b) s += chi(k, a) * KE[(3 * a + c) * 24 + 3 * b + c2] * chi(k2, b);
          B[3 * k + c][3 * k2 + c2] = s / 64.0;
          bmax = std::max(bmax, std::fabs(s / 64.0));
        }
  auto at = [&](int k, int c, int k2, int c2) { return B[3 * k + c][3 * k2 + c2]; };
  K->a1mb1 = at(1, 0, 1, 0) - at(1, 0, 2, 1);
  K->b1 = at(1, 0, 2, 1);
  K->g = at(1, 1, 2, 0);
  K->d = at(3, 0, 3, 0);
  K->e = at(3, 0, 6, 2);
  K->a4mb4 = at(3, 2, 3, 2) - at(3, 2, 5, 1);
  K->b4 = at(3, 2, 5, 1);
  K->h = at(7, 0, 7, 0);
  double err = 0.0;
  for (int col = 0; col < 24; ++col) {
    double hv[8][3] = {}, z[8][3];
    hv[col / 3][col % 3] = 1.0;
    walsh_blocks<double>(*K, 1.0, hv, z);
    for (int row = 0; row < 24; ++row)
      err = std::max(err, std::fabs(z[row / 3][row % 3] - B[row][col]));
  }
  return err <= 1e-12 * bmax;
}

// M_c = P_c^T KE P_c for the 8 child positions c of a 2:1 refined parent,
// P_c the trilinear map from the parent's corners to child c's corners
// (per component), packed with sym_index.
void child_galerkin(const double* KE, double* Mc) {
  auto phi = [](int pos, int A) { return pos == 1 ? 0.5 : ((pos >> 1) == A ? 1.0 : 0.0); };
  for (int c = 0; c < 8; ++c) {
    const int dx = c & 1, dy = (c >> 1) & 1, dz = c >> 2;
    double P[8][8];  // P[b][A]
    for (int b = 0; b < 8; ++b)
      for (int A = 0; A < 8; ++A)
        P[b][A] = phi(dx + (b & 1), A & 1) * phi(dy + ((b >> 1) & 1), (A >> 1) & 1) *
                  phi(dz + (b >> 2), A >> 2);
    for (int I = 0; I < 24; ++I)
      for (int J = I; J < 24; ++J) {
        double acc = 0.0;
        for (int b = 0; b < 8; ++b)
          for (int b2 = 0; b2 < 8; ++b2)
            acc += P[b][I / 3] * KE[(3 * b + I % 3) * 24 + 3 * b2 + J % 3] * P[b2][J / 3];
        Mc[c * kSymEntries + sym_index(I, J)] = acc;
      }
  }
}

// Nt[entry][8 c1 + c0] = (P_c1^T M_c0 P_c1)[entry]: the contribution of fine
// descendant c0 of level-1 child c1 to a level-2 parent's Galerkin matrix,
// per unit modulus (packed entries, stored transposed).  So a parent whose level-1 children touch no fixed DOF has the
// matrix sum_d E_d N_d over its 64 fine descendants.
void grandchild_galerkin(const double* Mc, double* N) {
  auto phi = [](int pos, int A) { return pos == 1 ? 0.5 : ((pos >> 1) == A ? 1.0 : 0.0); };
  for (int c1 = 0; c1 < 8; ++c1) {
    const int dx = c1 & 1, dy = (c1 >> 1) & 1, dz = c1 >> 2;
    double P[8][8];  // P[b][A]: child corner b from parent corner A
    for (int b = 0; b < 8; ++b)
      for (int A = 0; A < 8; ++A)
        P[b][A] = phi(dx + (b & 1), A & 1) * phi(dy + ((b >> 1) & 1), (A >> 1) & 1) *
                  phi(dz + (b >> 2), A >> 2);
    for (int c0 = 0; c0 < 8; ++c0) {
      const double* M = Mc + c0 * kSymEntries;
      for (int I = 0; I < 24; ++I)
        for (int J = I; J < 24; ++J) {
          double acc = 0.0;
          for (int b = 0; b < 8; ++b)
            for (int b2 = 0; b2 < 8; ++b2)
              acc += P[b][I / 3] * M[sym_index(3 * b + I % 3, 3 * b2 + J % 3)] * P[b2][J / 3];
          N[(int64_t)sym_index(I, J) * 64 + 8 * c1 + c0] = acc;
        }
    }
  }
}

// Check M_c = R_c M_0 R_c for every child c, where R_c mirrors the parent in
// the axes set in c: (R_c v)[3b + s] = (-1)^(bit s of c) v[3(b ^ c) + s].
bool mirror_children(const double* Mc) {
  double scale = 0.0;
  for (int x = 0; x < kSymEntries; ++x) scale = std::max(scale, std::fabs(Mc[x]));
  for (int c = 1; c < 8; ++c)
    for (int I = 0; I < 24; ++I)
      for (int J = I; J < 24; ++J) {
        const int a = I / 3, r = I % 3, b = J / 3, q = J % 3;
        const double sg = (((c >> r) ^ (c >> q)) & 1) ? -1.0 : 1.0;
        const double ref = sg * Mc[sym_index(3 * (a ^ c) + r, 3 * (b ^ c) + q)];
        if (std::fabs(Mc[c * kSymEntries + sym_index(I, J)] - ref) > 1e-12 * scale) return false;
      }
  return true;
}

// Bw = W M_0 W / 64: child 0's Galerkin matrix in the Walsh x component
// basis, W[3k + s][3a + s] = (-1)^popcount(k & a).
void walsh_child(const double* Mc, double* Bw) {
  auto pc = [](int x) { return __builtin_popcount((unsigned)x); };
  for (int ka = 0; ka < 24; ++ka)
    for (int la = 0; la < 24; ++la) {
      const int k = ka / 3, sk = ka % 3, l = la / 3, sl = la % 3;
      double acc = 0.0;
      for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b) {
          const double sg = ((pc(k & a) + pc(l & b)) & 1) ? -1.0 : 1.0;
          acc += sg * Mc[sym_index(3 * a + sk, 3 * b + sl)];
        }
      Bw[ka * 24 + la] = acc / 64.0;
    }
}

// For moduli E_c = 1 + c / 8: W (B' o Ehat(mu ^ mu)) W == sum_c E_c M_c, the
// identity the level-1 kernel evaluates.
bool walsh_parent_check(const double* Mc, const double* Bw) {
  auto pc = [](int x) { return __builtin_popcount((unsigned)x); };
  double E[8], Eh[8], G[576], scale = 0.0;
  for (int c = 0; c < 8; ++c) E[c] = 1.0 + c / 8.0;
  for (int k = 0; k < 8; ++k) {
    Eh[k] = 0.0;
    for (int c = 0; c < 8; ++c) Eh[k] += (pc(k & c) & 1) ? -E[c] : E[c];
  }
  for (int ka = 0; ka < 24; ++ka)
    for (int la = 0; la < 24; ++la) {
      const int mk = (ka / 3) ^ (1 << (ka % 3)), ml = (la / 3) ^ (1 << (la % 3));
      G[ka * 24 + la] = Bw[ka * 24 + la] * Eh[mk ^ ml];
    }
  for (int x = 0; x < 8 * kSymEntries; ++x) scale = std::max(scale, std::fabs(Mc[x]));
  for (int I = 0; I < 24; ++I)
    for (int J = 0; J < 24; ++J) {
      double want = 0.0, got = 0.0;
      for (int c = 0; c < 8; ++c) want += E[c] * Mc[c * kSymEntries + sym_index(I, J)];
      const int a = I / 3, s = I % 3, b = J / 3, t = J % 3;
      for (int k = 0; k < 8; ++k)
        for (int l = 0; l < 8; ++l) {
          const double sg = ((pc(k & a) + pc(l & b)) & 1) ? -1.0 : 1.0;
          got += sg * G[(3 * k + s) * 24 + 3 * l + t];
        }
      if (std::fabs(got - want) > 1e-11 * scale) return false;
    }
  return true;
}

// DOFs of level l (dim per node).
inline int64_t ndof(const aarmr_mesh* m, int l) { return m->dim * m->lg[l].nn; }

// Assign workspace views; with base == nullptr only computes the size.
int64_t layout(aarmr_mesh* m, char* base) {
  int64_t off = 0;
  auto take = [&](int64_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += align_up(bytes);
    return p;
  };
  const Grid& g = m->lg[0];
  const int64_t n3 = ndof(m, 0);
  const int64_t d8 = sizeof(double);
  const bool solid = m->dim == 3;
  const int64_t nsym = solid ? kSymEntries : kSymEntries2;
  m->KEd = (double*)take(576 * d8);
  if (solid) {  // level-1 Walsh product (3D only)
    m->Mcd = (double*)take(8 * kSymEntries * d8);
    m->N2d = (double*)take(64 * kSymEntries * d8);
    if (m->nlev > 2) {
      m->list2 = (int*)take(m->lg[2].ne * 4);
      m->count2 = (int*)take(4);
    }
    m->eflag1 = (uint8_t*)take(m->lg[1].ne);
    m->list1 = (int*)take(m->lg[1].ne * 4);
    m->count1 = (int*)take(4);
    m->Bwd = (double*)take(576 * d8);
    m->Y1 = (double*)take(24 * m->lg[1].ne * d8);
    m->cap1 = (int)std::min<int64_t>(m->lg[1].ne, std::max<int64_t>(m->lg[1].ne / 8, 1024));
    m->Kcomp1 = (double*)take((int64_t)kSymEntries * m->cap1 * d8);
  }
  m->E = (double*)take(g.ne * d8);
  m->E_prev = (double*)take(g.ne * d8);
  m->dE = (double*)take(g.ne * d8);
  m->rho_f = (double*)take(g.ne * d8);
  m->Hs = (double*)take(g.ne * d8);
  m->ework = (double*)take(g.ne * d8);
  m->dc_tmp = (double*)take(g.ne * d8);
  m->ones_dv = (double*)take(g.ne * d8);
  m->Wf = (double*)take((m->p.rmin > 0.0 ? filter_taps(m->p.rmin) : 1) * d8);
  m->cw = (double*)take(g.ne * d8);
  m->mask = (uint8_t*)take((g.nn + 3) / 4 * 4);
  m->mask_prev = (uint8_t*)take((g.nn + 3) / 4 * 4);
  m->r = (double*)take(n3 * d8);
  m->z = (double*)take(n3 * d8);
  m->pv = (double*)take(n3 * d8);
  m->q = (double*)take(n3 * d8);
  m->t0 = (double*)take(n3 * d8);
  m->fm = (double*)take(n3 * d8);
  m->lv[0] = LevelBuf();
  m->lv[0].dinv = (double*)take(n3 * d8);
  m->lv[0].t = m->t0;
  for (int l = 1; l < m->nlev; ++l) {
    const Grid& G = m->lg[l];
    LevelBuf& L = m->lv[l];
    const int64_t nl = ndof(m, l);
    L.Ke = (double*)take(G.ne * nsym * d8);
    L.dinv = (double*)take(nl * d8);
    L.b = (double*)take(nl * d8);
    L.x = (double*)take(nl * d8);
    L.t = (double*)take(nl * d8);
  }
  // the refinement form's FP32 vectors hold every load case (lock-step solve)
  const int64_t R = m->fp32 ? m->p.n_rhs_max : 1;
  if (m->fp32) {
    const int64_t f4 = sizeof(float);
    m->Bw32d = (float*)take(576 * f4);
    m->Y1f = (float*)take(R * 24 * m->lg[1].ne * f4);
    m->E32 = (float*)take(g.ne * f4);
    m->r32 = (float*)take(R * n3 * f4);
    m->z32 = (float*)take(R * n3 * f4);
    m->p32 = (float*)take(R * n3 * f4);
    m->q32 = (float*)take(R * n3 * f4);
    m->d32 = (float*)take(R * n3 * f4);
    for (int l = 0; l < m->nlev; ++l) {
      const int64_t m3 = ndof(m, l);
      LevelBuf& L = m->lv[l];
      L.dinv32 = (float*)take(m3 * f4);
      L.t32 = (float*)take(R * m3 * f4);
      if (l >= 1) {
        L.b32 = (float*)take(R * m3 * f4);
        L.x32 = (float*)take(R * m3 * f4);
      }
      if (solid && l >= 2 && l < m->nlev - 1) L.Ke32 = (float*)take(m->lg[l].ne * nsym * f4);
    }
    m->act = (int*)take(R * 4);
  }
  m->Ainv = (double*)take((int64_t)m->nc * m->nc * d8);
  m->gjP = (double*)take(2 * kGJBlock * kGJBlock * d8);  // two pivot inverses
  m->gjT = (double*)take((int64_t)m->nc * kGJBlock * d8);
  m->gjC = (double*)take((int64_t)m->nc * kGJBlock * d8);
  m->gjTb = (double*)take((int64_t)m->nc * kGJBlock * d8);
  m->Phi = (double*)take((int64_t)m->p.n_rhs_max * m->p.Ns * n3 * d8);
  m->R = (double*)take((int64_t)m->p.Nm * n3 * d8);
  m->KR = (double*)take((int64_t)m->p.Nm * n3 * d8);
  m->scal = (double*)take(R * SC_TOTAL * d8);  // one block of scalars per load case
  m->partial = (double*)take((int64_t)kRedSlots * kRedBlocks * d8);
  if (m->dim == 3) {  // CG's p^T A p and r^T z partials from the fine-grid products
    const int64_t cap = ebe_partials_max(m->lg[0]);
    m->part_cap = (int)cap;
    m->part_pq = (double*)take(R * cap * d8);
    m->part_rz = (double*)take(R * cap * d8);
  }
  m->flags = (unsigned*)take(64);
  return off;
}

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

int need_ws(const aarmr_mesh* m) {
  if (!m) return fail(AARMR_E_INVALID, "null mesh");
  if (!m->ws) return fail(AARMR_E_NO_WORKSPACE, "no workspace bound (aarmr_bind_workspace)");
  return AARMR_OK;
}

RedScratch red(aarmr_mesh* m) { return RedScratch{m->partial}; }

// Launch one multi-dot with up to kRedSlots products.
int dots(aarmr_mesh* m, int k, const double* const* a, const double* const* b, double* const* out,
         int64_t n, hipStream_t s) {
  for (int base = 0; base < k; base += kRedSlots) {
    DotSet d{};
    d.k = std::min(kRedSlots, k - base);
    d.n = n;
    for (int i = 0; i < d.k; ++i) {
      d.a[i] = a[base + i];
      d.b[i] = b ? b[base + i] : nullptr;
      d.out[i] = out[base + i];
    }
    launch_multidot(d, red(m), s);
    KCHECK();
  }
  return AARMR_OK;
}

int dot1(aarmr_mesh* m, const double* a, const double* b, double* out, int64_t n, hipStream_t s) {
  return dots(m, 1, &a, &b, &out, n, s);
}

// Copy `cnt` device scalars to the pinned staging buffer and synchronise.
int read_scalars(aarmr_mesh* m, const double* const* src, int cnt, double* dst, hipStream_t s) {
  bool contiguous = true;  // then one copy brings them all
  for (int i = 1; i < cnt; ++i) contiguous = contiguous && src[i] == src[0] + i;
  if (contiguous && cnt > 1)
    HIP_TRY(hipMemcpyAsync(m->hpin, src[0], cnt * sizeof(double), hipMemcpyDeviceToHost, s));
  else
    for (int i = 0; i < cnt; ++i)
      HIP_TRY(hipMemcpyAsync(m->hpin + i, src[i], sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int i = 0; i < cnt; ++i) dst[i] = m->hpin[i];
  return AARMR_OK;
}

int read_flags(aarmr_mesh* m, unsigned* out, hipStream_t s) {
  unsigned* h = reinterpret_cast<unsigned*>(m->hpin + 64);
  HIP_TRY(hipMemcpyAsync(h, m->flags, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemsetAsync(m->flags, 0, sizeof(unsigned), s));
  HIP_TRY(hipStreamSynchronize(s));
  *out = *h;
  return AARMR_OK;
}

// eq. (21): R = R~ Sigma V^T on the column-normalised CARM basis in m->R
// (Nm columns).  R = Q T by two-pass Gram-Schmidt without drop (Q in place,
// the normalised columns kept in m->KR), T = Q^T R by dot products, the thin
// SVD of the small T on the device (left singular vectors U of sigma >
// gs_tau sigma_1) and R~ = Q U written back into m->R.  *kept: number of
// basis vectors.
int orth_svd(aarmr_mesh* m, int Nm, int* kept, hipStream_t s) {
  const int64_t n3 = ndof(m, 0);
  double* misc = m->scal + SC_MISC;
  double* R = m->R;
  double* KR = m->KR;
  for (int i = 0; i < Nm; ++i) {
    TRY(dot1(m, R + i * n3, R + i * n3, misc + M_H + i, n3, s));
    launch_scale_by_inv_sqrt(n3, R + i * n3, misc + M_H + i, R + i * n3, s);
    KCHECK();
    HIP_TRY(hipMemcpyAsync(KR + i * n3, R + i * n3, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  for (int i = 0; i < Nm; ++i) {
    double* v = R + i * n3;
    for (int pass = 0; pass < 2 && i > 0; ++pass) {
      std::vector<const double*> a(i), b(i);
      std::vector<double*> o(i);
      for (int j = 0; j < i; ++j) {
        a[j] = R + j * n3;
        b[j] = v;
        o[j] = misc + M_H + j;
      }
      TRY(dots(m, i, a.data(), b.data(), o.data(), n3, s));
      launch_lincomb(n3, i, a.data(), misc + M_H, -1.0, v, v, s);
      KCHECK();
    }
    TRY(dot1(m, v, v, misc + M_NRM, n3, s));
    launch_scale_by_inv_sqrt(n3, v, misc + M_NRM, v, s);
    KCHECK();
  }
  {
    std::vector<const double*> a, b;
    std::vector<double*> o;
    for (int j = 0; j < Nm; ++j)
      for (int i = 0; i < Nm; ++i) {
        a.push_back(R + j * n3);
        b.push_back(KR + i * n3);
        o.push_back(misc + M_KR + j * Nm + i);
      }
    TRY(dots(m, (int)a.size(), a.data(), b.data(), o.data(), n3, s));
  }
  launch_small_svd(Nm, misc + M_KR, m->p.gs_tau, misc + M_SVC, misc + M_SVK, s);
  KCHECK();
  double hk = 0.0;
  const double* src = misc + M_SVK;
  TRY(read_scalars(m, &src, 1, &hk, s));
  *kept = (int)hk;
  std::vector<const double*> Q(Nm);
  for (int i = 0; i < Nm; ++i) Q[i] = R + i * n3;
  for (int j = 0; j < *kept; ++j) {
    launch_lincomb(n3, Nm, Q.data(), misc + M_SVC + j * Nm, 1.0, nullptr, KR + j * n3, s);
    KCHECK();
  }
  for (int j = 0; j < *kept; ++j)
    HIP_TRY(hipMemcpyAsync(R + j * n3, KR + j * n3, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
  return AARMR_OK;
}

// The flagged level-1 parent count of the current hierarchy, copied by setup
// into the pinned staging area (doubles 72.., after the scalar read-backs at
// 0..3 and the flag word at 64); the first call after a setup synchronises.
int flagged_count(aarmr_mesh* m, hipStream_t s) {
  if (m->nflag1 >= 0) return AARMR_OK;
  HIP_TRY(hipStreamSynchronize(s));
  m->nflag1 = *reinterpret_cast<const int*>(m->hpin + 72);
  return AARMR_OK;
}

// y = A v on level l.  Inside the solvers every vector is zero on fixed
// DOFs (loads and initial guesses are masked, and A, the smoother and the
// masked transfer operators preserve that), so the fine product skips input
// masking (mode 2); `any_input` selects the general form.
// Fine product with moduli E (the current design's, the reference design's
// or their difference): y = Df K(E) v for a v zero on fixed DOFs, plus the
// springs unless the product is the change K - K0 (with_springs false).
int fine_product(aarmr_mesh* m, const double* E, const double* v, double* y, hipStream_t s,
                 bool with_springs = true) {
  if (m->dim == 2) {
    launch_q4_apply(m->lg[0], m->KEd, E, m->mask, v, y, 2, s);
    if (with_springs) launch_springs_add(m->springs, m->lg[0], m->mask, v, y, s);
  } else
    launch_ebe(m->lg[0], m->wk, E, m->mask, v, y, 2, s);
  ++m->sweeps;
  KCHECK();
  return AARMR_OK;
}

int apply(aarmr_mesh* m, int l, const double* v, double* y, hipStream_t s,
          bool any_input = false) {
  if (m->dim == 2) {
    if (l == 0) {
      launch_q4_apply(m->lg[0], m->KEd, m->E, m->mask, v, y, any_input ? 0 : 2, s);
      launch_springs_add(m->springs, m->lg[0], m->mask, v, y, s);
      ++m->sweeps;
    } else {
      launch_q4_apply_elemmat(m->lg[l], m->lv[l].Ke, v, y, s);
    }
    KCHECK();
    return AARMR_OK;
  }
  if (l == 0) {
    launch_ebe(m->lg[0], m->wk, m->E, m->mask, v, y, any_input ? 0 : 2, s, m->tz64);
    ++m->sweeps;
  } else if (l == 1) {
    TRY(flagged_count(m, s));
    launch_apply_l1(m->lg[1], m->lv[1].Ke, m->Kcomp1, m->cap1, m->Bwd, m->E, m->eflag1,
                    m->list1, m->count1, m->nflag1, v, m->Y1, y, s);
  } else {
    launch_apply_elemmat(m->lg[l], m->lv[l].Ke, v, y, s);
  }
  KCHECK();
  return AARMR_OK;
}

// One V-cycle (Algorithm 2) on level l from a zero initial guess: x = M_l^-1 b.
// x_init: x already holds the first pre-smoothing sweep omega D^-1 b (formed
// by the kernel that produced b).  On the 3D hierarchy the sweeps are fused
// into neighbouring kernels: the restriction forms the coarse level's first
// sweep, and below the finest level the last post-smoothing sweep is the
// epilogue of its operator product.  On levels >= 2 that product writes into
// L.t and the level's x and t buffers swap roles, so there x must be L.x; on
// the finest level this is done only for the solver's own z (m->z, which
// swaps with t0), a caller's buffer gets the separate sweep.
int vcycle(aarmr_mesh* m, int l, const double* b, double* x, hipStream_t s,
           bool x_init = false) {
  if (l == m->nlev - 1) {
    launch_gemv(m->nc, m->Ainv, b, x, s);
    KCHECK();
    return AARMR_OK;
  }
  const Grid& G = m->lg[l];
  const int64_t n3 = ndof(m, l);
  LevelBuf& L = m->lv[l];
  LevelBuf& C = m->lv[l + 1];
  const uint8_t* mask = (l == 0) ? m->mask : nullptr;
  const double om = m->p.omega;
  const bool fuse = m->dim == 3;
  const bool child_first = fuse && m->p.nu_pre >= 1 && l + 1 < m->nlev - 1;
  if (m->p.nu_pre >= 1) {
    if (!x_init) {
      launch_jacobi_first(n3, b, L.dinv, om, x, s);  // line 1, first sweep from zero
      KCHECK();
    }
    for (int it = 1; it < m->p.nu_pre; ++it) {
      TRY(apply(m, l, x, L.t, s));
      launch_jacobi_update(n3, b, L.t, L.dinv, om, x, s);
      KCHECK();
    }
    TRY(apply(m, l, x, L.t, s));  // line 2: residual, restricted
    if (child_first)
      launch_restrict_jacobi(m->lg[l + 1], b, L.t, mask, C.b, C.dinv, om, C.x, s);
    else
      launch_restrict(m->lg[l + 1], b, L.t, mask, C.b, s, m->dim);
  } else {
    HIP_TRY(hipMemsetAsync(x, 0, n3 * sizeof(double), s));
    HIP_TRY(hipMemsetAsync(L.t, 0, n3 * sizeof(double), s));
    launch_restrict(m->lg[l + 1], b, L.t, mask, C.b, s, m->dim);
  }
  KCHECK();
  TRY(vcycle(m, l + 1, C.b, C.x, s, child_first));  // line 3
  launch_prolong_add(G, C.x, mask, x, s, m->dim);    // line 4
  KCHECK();
  for (int it = 0; it < m->p.nu_post; ++it) {        // line 5
    if (fuse && l == 0 && x == m->z && it == m->p.nu_post - 1) {
      // the solver's own z: the sweep writes into t0 and the two swap roles
      if (m->want_rz)
        m->rz_nb = launch_ebe_jacobi_dot(G, m->wk, m->E, m->mask, x, b, L.dinv, om, m->t0,
                                         m->part_rz, s, m->tz64);
      else
        launch_ebe_jacobi(G, m->wk, m->E, m->mask, x, b, L.dinv, om, m->t0, s, m->tz64);
      ++m->sweeps;
      KCHECK();
      std::swap(m->z, m->t0);
      L.t = m->t0;
      continue;
    }
    if (fuse && l >= 1 && it == m->p.nu_post - 1) {
      if (l == 1) {
        TRY(flagged_count(m, s));
        launch_apply_l1_jacobi(m->lg[1], L.Ke, m->Kcomp1, m->cap1, m->Bwd, m->E, m->eflag1,
                               m->list1, m->count1, m->nflag1, x, m->Y1, b, L.dinv, om, s);
      } else {
        if (x != L.x) return fail(AARMR_E_STATE, "V-cycle iterate is not the level's buffer");
        launch_apply_elemmat_jacobi(G, L.Ke, x, b, L.dinv, om, L.t, s);
        std::swap(L.x, L.t);
      }
      KCHECK();
      continue;
    }
    TRY(apply(m, l, x, L.t, s));
    launch_jacobi_update(n3, b, L.t, L.dinv, om, x, s);
    KCHECK();
  }
  return AARMR_OK;
}

// Algorithm 2's coarsest solve: the dense inverse of the coarsest Galerkin
// operator, by Gauss-Jordan.
int invert_coarsest(aarmr_mesh* m, hipStream_t s) {
  const Grid& G = m->lg[m->nlev - 1];
  if (m->dim == 2)
    launch_q4_assemble_dense(G, m->lv[m->nlev - 1].Ke, m->Ainv, s);
  else
    launch_assemble_dense(G, m->lv[m->nlev - 1].Ke, m->Ainv, s);
  KCHECK();
  launch_gj_invert(m->nc, m->Ainv, m->gjP, m->gjT, m->gjC, m->gjTb, s);
  KCHECK();
  HIP_TRY(hipMemcpyAsync(m->mask_prev, m->mask, (m->lg[0].nn + 3) / 4 * 4,
                         hipMemcpyDeviceToDevice, s));
  m->ainv_valid = true;
  m->ainv_stale = false;
  m->ainv_fresh = true;
  m->ainv_rebuild = false;
  ++m->ainv_builds;
  return AARMR_OK;
}

// The coarsest solve of a new hierarchy: keep the inverse of an earlier
// design when the call allows it, the fixed DOFs are the same and the last
// solve with it did not need markedly more iterations than the first;
// otherwise invert the current coarsest operator.  An older inverse is still
// symmetric positive definite, so the V-cycle stays a symmetric positive
// definite preconditioner and CG still converges to the current design's
// solution; only the iteration count changes.
int coarsest_inverse(aarmr_mesh* m, hipStream_t s) {
  if (m->reuse_req && m->ainv_valid && !m->mask_changed && !m->ainv_rebuild) {
    m->ainv_stale = true;
    m->ainv_fresh = false;
    ++m->ainv_reuses;
    return AARMR_OK;
  }
  return invert_coarsest(m, s);
}

// The MG hierarchy of the current moduli and mask (Algorithm 2's operators):
// Jacobi diagonals, Galerkin operators of the coarse levels, the coarsest
// dense inverse.  Reads E, mask and the element matrices only.
int build_mg(aarmr_mesh* m, hipStream_t s) {
  const Grid& g = m->lg[0];
  if (m->dim == 2) {
    launch_q4_diag(g, m->KEd, m->E, m->mask, m->lv[0].dinv, s);
    launch_springs_diag(m->springs, g, m->mask, m->lv[0].dinv, s);
    KCHECK();
    for (int l = 1; l < m->nlev; ++l) {
      if (l == 1) {
        launch_q4_galerkin_from_fine(m->lg[1], m->KEd, m->E, m->mask, m->lv[1].Ke, s);
        launch_springs_galerkin(m->springs, m->lg[1], m->mask, m->lv[1].Ke, s);
      } else
        launch_q4_galerkin_from_coarse(m->lg[l], m->lv[l - 1].Ke, m->lv[l].Ke, s);
      KCHECK();
      if (l < m->nlev - 1) {
        launch_q4_diag_elemmat(m->lg[l], m->lv[l].Ke, m->lv[l].dinv, s);
        KCHECK();
      }
    }
    TRY(coarsest_inverse(m, s));
    m->mg_ready = true;
    return AARMR_OK;
  }
  launch_diag_fine(g, m->KEd, m->E, m->mask, m->lv[0].dinv, m->lv[0].dinv32, s);
  KCHECK();
  // Below a coarser level, the level-1 matrices of parents without a fixed
  // fine DOF are never stored: the level-1 product forms them from the moduli,
  // the level-1 diagonal and the level-2 Galerkin matrices come from the
  // moduli too.  Only as the coarsest level are they assembled.
  const bool l1_all = m->nlev == 2;
  for (int l = 1; l < m->nlev; ++l) {
    if (l == 1) {
      launch_galerkin_from_fine(m->lg[1], m->KEd, m->Mcd, m->E, m->mask, m->eflag1, m->list1,
                                m->count1, m->lv[1].Ke, m->Kcomp1, m->cap1, s, l1_all);
      KCHECK();
      // the flagged count sizes the level-1 launches: fetched without a
      // stall, read at the first level-1 product (nflag1 < 0 until then)
      HIP_TRY(hipMemcpyAsync(m->hpin + 72, m->count1, sizeof(int), hipMemcpyDeviceToHost, s));
      m->nflag1 = -1;
    } else {
      if (l == 2)
        launch_galerkin_l2_from_fine(m->lg[2], m->N2d, m->Mcd, m->E, m->eflag1, m->list2,
                                     m->count2, m->lv[1].Ke, m->lv[2].Ke, s);
      else
        launch_galerkin_from_coarse(m->lg[l], m->lv[l - 1].Ke, m->lv[l].Ke, s);
      if (m->fp32 && l < m->nlev - 1)  // the FP32 V-cycle's copy (the coarsest uses its inverse)
        launch_to_f32(m->lg[l].ne * kSymEntries, m->lv[l].Ke, m->lv[l].Ke32, s);
    }
    KCHECK();
    if (l < m->nlev - 1) {
      if (l == 1)
        launch_diag_l1(m->lg[1], m->lv[1].Ke, m->Mcd, m->E, m->eflag1, m->lv[1].dinv,
                       m->lv[1].dinv32, s);
      else
        launch_diag_elemmat(m->lg[l], m->lv[l].Ke, m->lv[l].dinv, m->lv[l].dinv32, s);
      KCHECK();
    }
  }
  TRY(coarsest_inverse(m, s));
  m->mg_ready = true;
  return AARMR_OK;
}

// Make stream s wait for a speculative hierarchy build, if one is in flight.
int join_mg(aarmr_mesh* m, hipStream_t s) {
  if (!m->mg_pending) return AARMR_OK;
  m->mg_pending = false;
  HIP_TRY(hipStreamWaitEvent(s, m->ev_mg, 0));
  return AARMR_OK;
}

// Fixed-DOF mask and SIMP moduli of the density rho~; with_mg: also the hierarchy.
int setup(aarmr_mesh* m, const double* rho, const int64_t* fixed, int64_t nfixed, bool with_mg,
          hipStream_t s) {
  TRY(join_mg(m, s));
  const Grid& g = m->lg[0];
  launch_build_mask(g.nn, fixed, nfixed, m->mask, m->flags, s, m->dim);
  KCHECK();
  if (m->reuse_req && m->ainv_valid) {
    launch_mask_diff(g.nn, m->mask, m->mask_prev, m->flags, s);
    KCHECK();
  }
  launch_simp(g.ne, rho, m->p.E0, m->p.Emin, m->p.penal, m->E, m->fp32 ? m->E32 : nullptr,
              m->flags, s);
  KCHECK();
  m->mg_ready = false;
  if (!with_mg) return AARMR_OK;
  return build_mg(m, s);
}

// Appended to the non-convergence messages: a V-cycle whose damped-Jacobi
// sweep is no contraction (omega lambda_max(D^-1 A) >= 2, e.g. on moduli that
// vary from element to element without a filter) is indefinite, and CG then
// stalls instead of failing outright.
#define AARMR_OMEGA_HINT \
  " (if it stalls, the moduli may be too rough for omega: the damped-Jacobi sweep needs " \
  "omega * lambda_max(D^-1 A) < 2, about 0.5 for unfiltered element-wise moduli)"

// ---- refinement form: FP32 inner solve ------------------------------------
// y = A v on level l with FP32 vectors (v zero on fixed DOFs).
int apply32(aarmr_mesh* m, int l, const float* v, float* y, hipStream_t s, int nr = 1) {
  if (l == 0) {
    launch_ebe_f32(m->lg[0], m->wk, m->E32, m->mask, v, y, 2, s, m->tz32, nr);
    ++m->sweeps;
  } else if (l == 1) {
    TRY(flagged_count(m, s));
    launch_apply_l1_f32(m->lg[1], m->lv[1].Ke, m->Kcomp1, m->cap1, m->Bw32d, m->E32,
                        m->eflag1, m->list1, m->count1, m->nflag1, v, m->Y1f, y, s, nr);
  } else {
    launch_apply_elemmat_f32(m->lg[l], m->lv[l].Ke32, v, y, s, nr);
  }
  KCHECK();
  return AARMR_OK;
}

// The V-cycle of vcycle() with FP32 vectors and smoothing, and the same
// fused sweeps; the coarsest inverse is the FP64 one.  x_init: x already
// holds the level's first Jacobi sweep.
// nr load cases in lock step: b and x (and the level buffers) hold nr
// vectors each, one after another.
int vcycle32(aarmr_mesh* m, int l, const float* b, float* x, hipStream_t s,
             bool x_init = false, int nr = 1) {
  if (l == m->nlev - 1) {
    launch_gemv_f32(m->nc, m->Ainv, b, x, s, nr);
    KCHECK();
    return AARMR_OK;
  }
  const Grid& G = m->lg[l];
  const int64_t n3 = ndof(m, l);
  LevelBuf& L = m->lv[l];
  LevelBuf& C = m->lv[l + 1];
  const uint8_t* mask = (l == 0) ? m->mask : nullptr;
  const float om = (float)m->p.omega;
  const bool child_first = m->p.nu_pre >= 1 && l + 1 < m->nlev - 1;
  if (m->p.nu_pre >= 1) {
    if (!x_init) {
      launch_jacobi_first_f32(n3, b, L.dinv32, om, x, s, nr);
      KCHECK();
    }
    for (int it = 1; it < m->p.nu_pre; ++it) {
      TRY(apply32(m, l, x, L.t32, s, nr));
      launch_jacobi_update_f32(n3, b, L.t32, L.dinv32, om, x, s, nr);
      KCHECK();
    }
    TRY(apply32(m, l, x, L.t32, s, nr));
    if (child_first)
      launch_restrict_jacobi_f32(m->lg[l + 1], b, L.t32, mask, C.b32, C.dinv32, om, C.x32, s,
                                 nr);
    else
      launch_restrict_f32(m->lg[l + 1], b, L.t32, mask, C.b32, s, nr);
  } else {
    HIP_TRY(hipMemsetAsync(x, 0, nr * n3 * sizeof(float), s));
    launch_restrict_f32(m->lg[l + 1], b, nullptr, mask, C.b32, s, nr);
  }
  KCHECK();
  TRY(vcycle32(m, l + 1, C.b32, C.x32, s, child_first, nr));
  launch_prolong_add_f32(G, C.x32, mask, x, s, nr);
  KCHECK();
  for (int it = 0; it < m->p.nu_post; ++it) {
    const bool last = it == m->p.nu_post - 1;
    if (l == 0 && x == m->z32 && last) {
      // the solver's own z: the sweep (with r^T z partials) writes into t32,
      // and the two swap roles
      m->rz_nb = launch_ebe_jacobi_f32_dot(G, m->wk, m->E32, m->mask, x, b, L.dinv32, om, L.t32,
                                           m->part_rz, s, m->tz32, nr, m->part_cap);
      ++m->sweeps;
      KCHECK();
      std::swap(m->z32, L.t32);
      continue;
    }
    if (l >= 1 && last) {
      if (l == 1) {
        TRY(flagged_count(m, s));
        launch_apply_l1_jacobi_f32(m->lg[1], L.Ke, m->Kcomp1, m->cap1, m->Bw32d, m->E32,
                                   m->eflag1, m->list1, m->count1, m->nflag1, x, m->Y1f, b,
                                   L.dinv32, om, s, nr);
      } else {
        if (x != L.x32) return fail(AARMR_E_STATE, "V-cycle iterate is not the level's buffer");
        launch_apply_elemmat_jacobi_f32(G, L.Ke32, x, b, L.dinv32, om, L.t32, s, nr);
        std::swap(L.x32, L.t32);
      }
      KCHECK();
      continue;
    }
    TRY(apply32(m, l, x, L.t32, s, nr));
    launch_jacobi_update_f32(n3, b, L.t32, L.dinv32, om, x, s, nr);
    KCHECK();
  }
  return AARMR_OK;
}

int dot32(aarmr_mesh* m, const float* a, const float* b, double* out, int64_t n, hipStream_t s) {
  DotSetT<float> d{};
  d.k = 1;
  d.n = n;
  d.a[0] = a;
  d.b[0] = b;
  d.out[0] = out;
  launch_multidot_f32(d, red(m), s);
  KCHECK();
  return AARMR_OK;
}

// FP32 PCG on A d = r32 (r32 of unit norm, zero on fixed DOFs) from d = 0,
// until ||r|| <= rtol (recurrence residual, FP64 dots) or maxit iterations.
// r32 is overwritten.  *stalled is set when r^T z or p^T A p stops being
// positive, the sign that FP32 can make no further progress.
int pcg32(aarmr_mesh* m, double rtol, int maxit, int* iters, double* relres, bool* stalled,
          hipStream_t s) {
  const Grid& g = m->lg[0];
  const int64_t n3 = ndof(m, 0);
  double* sc = m->scal;
  HIP_TRY(hipMemsetAsync(m->d32, 0, n3 * sizeof(float), s));
  *iters = 0;
  *relres = 1.0;
  *stalled = false;
  const double tol2 = rtol * rtol;
  m->rz_nb = 0;
  TRY(vcycle32(m, 0, m->r32, m->z32, s));
  TRY(dot32(m, m->r32, m->z32, sc + SC_RZ, n3, s));
  launch_copy_f32(n3, m->z32, m->p32, s);
  KCHECK();
  // as pcg64: p^T A p from the product's workgroups, r^T z from the V-cycle's
  // last fine sweep, the x/r update storing the r^T r partials, p^T q and r^T z
  // into host memory, and the next V-cycle and direction update queued before
  // the host waits for them
  const int nb = fused_blocks(n3);
  const double* hrr = m->hrr;
  const float om = (float)m->p.omega;
  for (int it = 0; it < maxit; ++it) {
    const int n_pq = launch_ebe_f32_dot(g, m->wk, m->E32, m->mask, m->p32, m->q32, m->part_pq,
                                        s, m->tz32);
    ++m->sweeps;
    launch_cg_xr_fused_f32(n3, sc + SC_RZ + it, m->part_pq, n_pq, sc + SC_PQ + it, m->d32,
                           m->r32, m->p32, m->q32, m->hrr_dev, m->lv[0].dinv32, om, m->z32, s);
    KCHECK();
    HIP_TRY(hipEventRecord(m->ev_cg, s));
    if (it + 1 < maxit) {
      m->rz_nb = 0;
      TRY(vcycle32(m, 0, m->r32, m->z32, s, m->p.nu_pre >= 1));
      if (m->rz_nb > 0) {
        launch_cg_p_fused_f32(n3, m->part_rz, m->rz_nb, sc + SC_RZ + it + 1, sc + SC_RZ + it,
                              m->z32, m->p32, s);
      } else {
        TRY(dot32(m, m->r32, m->z32, sc + SC_RZ + it + 1, n3, s));
        launch_cg_p_f32(n3, sc + SC_RZ + it + 1, sc + SC_RZ + it, m->z32, m->p32, s);
      }
      KCHECK();
    }
    HIP_TRY(hipEventSynchronize(m->ev_cg));
    double rr = 0.0;
    for (int b = 0; b < nb; ++b) rr += hrr[b];
    *iters = it + 1;
    *relres = std::sqrt(rr);
    if (!(hrr[nb] > 0.0) || !(hrr[nb + 1] > 0.0)) {
      *stalled = true;
      return AARMR_OK;
    }
    if (rr <= tol2) return AARMR_OK;
  }
  return AARMR_OK;
}

// Iterative refinement: r = fm - A x in FP64, the FP32 PCG solves A d = r/||r||
// to a relative accuracy chosen so that the next FP64 residual lands near
// cg_rtol, and x += ||r|| d in FP64; repeated until the FP64 residual meets
// cg_rtol.  *iters counts the inner iterations.  When FP32 stops making
// progress (a non-positive p^T A p or r^T z in the inner CG, or an outer step
// that reduces the FP64 residual less than 5x) *fallback is set and x holds the latest
// iterate: the caller continues from it with FP64 CG and the FP64 V-cycle.
#ifndef AARMR_INNER_FLOOR
#define AARMR_INNER_FLOOR 5e-6
#endif
int refine(aarmr_mesh* m, double* x, int* iters, double* relres, bool* fallback,
           hipStream_t s) {
  const Grid& g = m->lg[0];
  const int64_t n3 = ndof(m, 0);
  double* misc = m->scal + SC_MISC;
  const double rtol = m->p.cg_rtol;
  const int budget = std::min(m->p.cg_maxit, kMaxIt);
  constexpr double kInnerFloor = AARMR_INNER_FLOOR;  // attainable FP32 reduction per step
  *iters = 0;
  *fallback = false;
  double ff = -1.0, prev_rel = 0.0;
  for (int outer = 0; outer < 64; ++outer) {
    TRY(apply(m, 0, x, m->q, s));
    launch_sub(n3, m->fm, m->q, m->r, s);
    KCHECK();
    double h[2];
    if (ff < 0.0) {
      const double* a[2] = {m->fm, m->r};
      double* o[2] = {misc + M_FF, misc + M_RR64};
      TRY(dots(m, 2, a, a, o, n3, s));
      const double* src[2] = {misc + M_FF, misc + M_RR64};
      TRY(read_scalars(m, src, 2, h, s));
      ff = h[0];
      if (ff == 0.0) {
        HIP_TRY(hipMemsetAsync(x, 0, n3 * sizeof(double), s));
        *relres = 0.0;
        return AARMR_OK;
      }
      if (h[1] > ff) {  // the initial guess is worse than zero: start from zero
        HIP_TRY(hipMemsetAsync(x, 0, n3 * sizeof(double), s));
        HIP_TRY(hipMemcpyAsync(m->r, m->fm, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(misc + M_RR64, misc + M_FF, sizeof(double),
                               hipMemcpyDeviceToDevice, s));
        h[1] = ff;
      }
    } else {
      TRY(dot1(m, m->r, m->r, misc + M_RR64, n3, s));
      const double* src = misc + M_RR64;
      TRY(read_scalars(m, &src, 1, h + 1, s));
    }
    const double rel = std::sqrt(h[1] / ff);
    *relres = rel;
    if (rel <= rtol) return AARMR_OK;
    if (*iters >= budget) break;
    const double inner = std::min(0.1, std::max(kInnerFloor, 0.5 * rtol / rel));
    launch_to_f32_scaled(n3, m->r, misc + M_RR64, m->r32, s);
    KCHECK();
    // every step targets a reduction of at least 10x; one that delivers less
    // than 5x shows that FP32 cannot resolve this operator well enough
    if (outer > 0 && rel > 0.2 * prev_rel) {
      *fallback = true;
      return AARMR_OK;
    }
    prev_rel = rel;
    int its = 0;
    double rin = 1.0;
    bool stalled = false;
    TRY(pcg32(m, inner, budget - *iters, &its, &rin, &stalled, s));
    *iters += its;
    if (stalled) {  // FP32 cannot resolve p^T A p here (e.g. extreme contrast)
      *fallback = true;
      return AARMR_OK;
    }
    launch_add_scaled_f32(n3, m->d32, misc + M_RR64, x, s);
    KCHECK();
  }
  return fail(AARMR_E_NOT_CONVERGED, "refinement reached cg_maxit before cg_rtol" AARMR_OMEGA_HINT);
}

// ---- refinement form, load cases in lock step ----------------------------
// The nr load cases of one mesh share every launch of the FP32 inner solve:
// the fine product, the V-cycle and the CG updates run over nr vectors
// stored one after another (a grid dimension per load case), so the
// launches per iteration do not depend on nr.  Each case keeps its own CG
// scalars, partials and stopping test; a finished case is flagged inactive
// and its updates are skipped.  Every case follows exactly the arithmetic
// of its own single-case solve.

// Upload the activity flags act[0..nr) to the device (stream-ordered; the
// host writes the pinned staging only after the stream has passed the
// previous copy, which every caller ensures by synchronising in between).
int upload_act(aarmr_mesh* m, int nr, const bool* act, hipStream_t s) {
  for (int l = 0; l < nr; ++l) m->hact[l] = act[l] ? 1 : 0;
  HIP_TRY(hipMemcpyAsync(m->act, m->hact, nr * sizeof(int), hipMemcpyHostToDevice, s));
  return AARMR_OK;
}

// Lock-step pcg32: case l (act[l] set on entry) solves A d_l = r32_l from
// d_l = 0 until ||r_l|| <= rtol[l] or maxit iterations.  On return act[l] is
// cleared for every case; iters, relres and stalled are per case.
int pcg32_multi(aarmr_mesh* m, int nr, const double* rtol, int maxit, bool* act, int* iters,
                double* relres, bool* stalled, hipStream_t s) {
  const Grid& g = m->lg[0];
  const int64_t n3 = ndof(m, 0);
  double* sc = m->scal;
  const int hs = kFusedBlocks + 8;
  MultiRhs mr;
  mr.n = nr;
  mr.vs = n3;
  mr.ss = SC_TOTAL;
  mr.ps = m->part_cap;
  mr.hs = hs;
  mr.active = m->act;
  TRY(upload_act(m, nr, act, s));
  HIP_TRY(hipMemsetAsync(m->d32, 0, nr * n3 * sizeof(float), s));
  for (int l = 0; l < nr; ++l) {
    iters[l] = 0;
    relres[l] = 1.0;
    stalled[l] = false;
  }
  m->rz_nb = 0;
  TRY(vcycle32(m, 0, m->r32, m->z32, s, false, nr));
  {
    DotSetT<float> d{};
    d.k = nr;
    d.n = n3;
    for (int l = 0; l < nr; ++l) {
      d.a[l] = m->r32 + l * n3;
      d.b[l] = m->z32 + l * n3;
      d.out[l] = sc + l * SC_TOTAL + SC_RZ;
    }
    launch_multidot_f32(d, red(m), s);
    KCHECK();
  }
  launch_copy_f32(nr * n3, m->z32, m->p32, s);
  KCHECK();
  const int nb = fused_blocks(n3);
  const double* hrr = m->hrr;
  const float om = (float)m->p.omega;
  for (int it = 0; it < maxit; ++it) {
    const int n_pq = launch_ebe_f32_dot(g, m->wk, m->E32, m->mask, m->p32, m->q32, m->part_pq,
                                        s, m->tz32, nr, m->part_cap);
    ++m->sweeps;
    launch_cg_xr_fused_f32(n3, sc + SC_RZ + it, m->part_pq, n_pq, sc + SC_PQ + it, m->d32,
                           m->r32, m->p32, m->q32, m->hrr_dev, m->lv[0].dinv32, om, m->z32, s,
                           mr);
    KCHECK();
    HIP_TRY(hipEventRecord(m->ev_cg, s));
    if (it + 1 < maxit) {
      m->rz_nb = 0;
      TRY(vcycle32(m, 0, m->r32, m->z32, s, m->p.nu_pre >= 1, nr));
      if (m->rz_nb <= 0) return fail(AARMR_E_STATE, "lock-step solve needs the fused fine sweep");
      launch_cg_p_fused_f32(n3, m->part_rz, m->rz_nb, sc + SC_RZ + it + 1, sc + SC_RZ + it,
                            m->z32, m->p32, s, mr);
      KCHECK();
    }
    HIP_TRY(hipEventSynchronize(m->ev_cg));
    bool any = false, changed = false;
    for (int l = 0; l < nr; ++l) {
      if (!act[l]) continue;
      const double* h = hrr + (int64_t)l * hs;
      double rr = 0.0;
      for (int b = 0; b < nb; ++b) rr += h[b];
      iters[l] = it + 1;
      relres[l] = std::sqrt(rr);
      if (!(h[nb] > 0.0) || !(h[nb + 1] > 0.0)) {
        stalled[l] = true;
        act[l] = false;
        changed = true;
      } else if (rr <= rtol[l] * rtol[l]) {
        act[l] = false;
        changed = true;
      }
      any = any || act[l];
    }
    if (!any) return AARMR_OK;
    if (changed) TRY(upload_act(m, nr, act, s));
  }
  for (int l = 0; l < nr; ++l) act[l] = false;
  return AARMR_OK;
}

// Lock-step refinement of nr load cases, as refine() per case: the FP64
// residual r_l = f_l - A u_l (f_l masked into fm, case by case), the FP32
// solve of all unfinished cases together on r_l / ||r_l||, u_l += ||r_l||
// d_l.  fallback[l]: FP32 could not resolve case l (the caller continues it
// with FP64 CG).  status[l]: AARMR_OK or AARMR_E_NOT_CONVERGED.
int refine_multi(aarmr_mesh* m, int nr, const double* f, double* u, int* iters, double* relres,
                 bool* fallback, int* status, hipStream_t s) {
  const Grid& g = m->lg[0];
  const int64_t n3 = ndof(m, 0);
  const double rtol = m->p.cg_rtol;
  const int budget = std::min(m->p.cg_maxit, kMaxIt);
  constexpr double kInnerFloor = AARMR_INNER_FLOOR;
  double ff[AARMR_MAX_RHS] = {}, prev_rel[AARMR_MAX_RHS] = {}, inner[AARMR_MAX_RHS] = {};
  double rin[AARMR_MAX_RHS] = {};
  bool done[AARMR_MAX_RHS] = {}, act[AARMR_MAX_RHS] = {}, stalled[AARMR_MAX_RHS] = {};
  int its[AARMR_MAX_RHS] = {};
  for (int l = 0; l < nr; ++l) {
    ff[l] = -1.0;
    prev_rel[l] = 0.0;
    done[l] = false;
    fallback[l] = false;
    status[l] = AARMR_OK;
    iters[l] = 0;
    relres[l] = 1.0;
  }
  // cases that take no part in a round keep a zero FP32 right-hand side
  HIP_TRY(hipMemsetAsync(m->r32, 0, nr * n3 * sizeof(float), s));
  for (int outer = 0; outer < 64; ++outer) {
    bool any = false;
    for (int l = 0; l < nr; ++l) {
      act[l] = false;
      if (done[l] || fallback[l]) continue;
      double* ul = u + l * n3;
      double* misc = m->scal + l * SC_TOTAL + SC_MISC;
      launch_copy_masked(g, f + l * n3, m->mask, m->fm, s, m->dim);
      KCHECK();
      TRY(apply(m, 0, ul, m->q, s));
      launch_sub(n3, m->fm, m->q, m->r, s);
      KCHECK();
      double h[2];
      if (ff[l] < 0.0) {
        const double* a[2] = {m->fm, m->r};
        double* o[2] = {misc + M_FF, misc + M_RR64};
        TRY(dots(m, 2, a, a, o, n3, s));
        const double* src[2] = {misc + M_FF, misc + M_RR64};
        TRY(read_scalars(m, src, 2, h, s));
        ff[l] = h[0];
        if (ff[l] == 0.0) {
          HIP_TRY(hipMemsetAsync(ul, 0, n3 * sizeof(double), s));
          relres[l] = 0.0;
          done[l] = true;
          continue;
        }
        if (h[1] > ff[l]) {  // the initial guess is worse than zero: start from zero
          HIP_TRY(hipMemsetAsync(ul, 0, n3 * sizeof(double), s));
          HIP_TRY(hipMemcpyAsync(m->r, m->fm, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
          HIP_TRY(hipMemcpyAsync(misc + M_RR64, misc + M_FF, sizeof(double),
                                 hipMemcpyDeviceToDevice, s));
          h[1] = ff[l];
        }
      } else {
        TRY(dot1(m, m->r, m->r, misc + M_RR64, n3, s));
        const double* src = misc + M_RR64;
        TRY(read_scalars(m, &src, 1, h + 1, s));
      }
      const double rel = std::sqrt(h[1] / ff[l]);
      relres[l] = rel;
      if (rel <= rtol) {
        done[l] = true;
        continue;
      }
      if (iters[l] >= budget) {
        done[l] = true;
        status[l] = AARMR_E_NOT_CONVERGED;
        continue;
      }
      if (outer > 0 && rel > 0.2 * prev_rel[l]) {
        fallback[l] = true;
        continue;
      }
      prev_rel[l] = rel;
      inner[l] = std::min(0.1, std::max(kInnerFloor, 0.5 * rtol / rel));
      launch_to_f32_scaled(n3, m->r, misc + M_RR64, m->r32 + l * n3, s);
      KCHECK();
      act[l] = true;
      any = true;
    }
    if (!any) return AARMR_OK;
    int maxit = 0;
    for (int l = 0; l < nr; ++l)
      if (act[l]) maxit = std::max(maxit, budget - iters[l]);
    bool was[AARMR_MAX_RHS] = {};
    for (int l = 0; l < nr; ++l) was[l] = act[l];
    TRY(pcg32_multi(m, nr, inner, maxit, act, its, rin, stalled, s));
    for (int l = 0; l < nr; ++l) {
      if (!was[l]) continue;
      iters[l] += its[l];
      if (stalled[l]) {
        fallback[l] = true;
        continue;
      }
      launch_add_scaled_f32(n3, m->d32 + l * n3, m->scal + l * SC_TOTAL + SC_MISC + M_RR64,
                            u + l * n3, s);
      KCHECK();
    }
  }
  for (int l = 0; l < nr; ++l)
    if (!done[l] && !fallback[l]) status[l] = AARMR_E_NOT_CONVERGED;
  return AARMR_OK;
}

int pcg64(aarmr_mesh* m, double* x, int* iters, double* relres, int maxit_in, hipStream_t s);

// Preconditioned CG on A x = fm (fm already masked), x in/out (masked).  In
// the refinement form the FP32 refinement runs first; if it hands over, FP64
// CG with the FP64 V-cycle continues from its iterate.
int pcg(aarmr_mesh* m, double* x, int* iters, double* relres, hipStream_t s) {
  int it0 = 0;
  if (m->fp32) {
    bool fallback = false;
    const int rc = refine(m, x, &it0, relres, &fallback, s);
    if (rc != AARMR_OK || !fallback) {
      *iters = it0;
      return rc;
    }
  }
  const int rc = pcg64(m, x, iters, relres, std::min(m->p.cg_maxit, kMaxIt) - it0, s);
  *iters += it0;
  return rc;
}

// pcg() with the bookkeeping of a reused coarsest inverse.  A solve with an
// older inverse gets at most 2 n0 + 20 iterations (n0: the first solve after
// the inversion); if it has not converged by then the current coarsest
// operator is inverted and CG continues from its iterate.  A solve that
// needs max(3, n0 / 8) or more iterations beyond n0 asks for a new inversion
// at the next hierarchy build.
int pcg_reuse(aarmr_mesh* m, double* x, int* iters, double* relres, hipStream_t s) {
  if (!m->ainv_stale) {
    const int rc = pcg(m, x, iters, relres, s);
    if (m->ainv_fresh && rc == AARMR_OK) {
      m->ainv_base_its = *iters;
      m->ainv_fresh = false;
    }
    return rc;
  }
  const int maxit = m->p.cg_maxit;
  const int cap = std::min(maxit, 2 * m->ainv_base_its + 20);
  m->p.cg_maxit = cap;
  int rc = pcg(m, x, iters, relres, s);
  m->p.cg_maxit = maxit;
  if (rc == AARMR_OK) {
    if (*iters >= m->ainv_base_its + std::max(3, m->ainv_base_its / 8)) m->ainv_rebuild = true;
    return rc;
  }
  if (rc != AARMR_E_NOT_CONVERGED || cap >= maxit) return rc;
  TRY(invert_coarsest(m, s));
  int more = 0;
  m->p.cg_maxit = maxit - *iters;
  rc = pcg(m, x, &more, relres, s);
  m->p.cg_maxit = maxit;
  *iters += more;
  m->ainv_fresh = false;
  m->ainv_base_its = more;
  return rc;
}

// CG with the FP64 V-cycle preconditioner for at most maxit iterations.
int pcg64(aarmr_mesh* m, double* x, int* iters, double* relres, int maxit_in, hipStream_t s) {
  const Grid& g = m->lg[0];
  const int64_t n3 = ndof(m, 0);
  double* sc = m->scal;
  double* misc = sc + SC_MISC;
  TRY(apply(m, 0, x, m->q, s));
  launch_sub(n3, m->fm, m->q, m->r, s);
  KCHECK();
  {
    const double* a[2] = {m->fm, m->r};
    const double* b[2] = {m->fm, m->r};
    double* o[2] = {misc + M_FF, sc + SC_RR};
    TRY(dots(m, 2, a, b, o, n3, s));
  }
  double h[2];
  {
    const double* src[2] = {misc + M_FF, sc + SC_RR};
    TRY(read_scalars(m, src, 2, h, s));
  }
  const double ff = h[0];
  *iters = 0;
  if (ff == 0.0) {
    HIP_TRY(hipMemsetAsync(x, 0, n3 * sizeof(double), s));
    *relres = 0.0;
    return AARMR_OK;
  }
  const double tol2 = m->p.cg_rtol * m->p.cg_rtol * ff;
  double rr = h[1];
  if (rr > ff) {  // the initial guess is worse than zero: start from zero
    HIP_TRY(hipMemsetAsync(x, 0, n3 * sizeof(double), s));
    HIP_TRY(hipMemcpyAsync(m->r, m->fm, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(sc + SC_RR, misc + M_FF, sizeof(double), hipMemcpyDeviceToDevice, s));
    rr = ff;
  }
  *relres = std::sqrt(rr / ff);
  if (rr <= tol2) return AARMR_OK;
  TRY(vcycle(m, 0, m->r, m->z, s));
  TRY(dot1(m, m->r, m->z, sc + SC_RZ, n3, s));
  HIP_TRY(hipMemcpyAsync(m->pv, m->z, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
  const int maxit = std::max(0, maxit_in);
  {
    // reductions folded into the updates: p^T q finished by the x/r update,
    // r^T r summed on the host from its block partials, r^T z finished by the
    // p update; the update also forms the V-cycle's first sweep.  While the
    // host waits for r^T r, the GPU already runs the next preconditioner and
    // direction update: they read r and write only z and p, so when the
    // iteration turns out to be the last, x and r are final and that work is
    // simply unused.
    double* part_pq = m->partial;
    double* part_rz = m->partial + kRedBlocks;
    double* part_rr = m->hrr_dev;  // fused_blocks(n3) + 1 entries, in host memory
    const int nb = fused_blocks(n3);
    const bool z0 = m->p.nu_pre >= 1;
    const double* hrr = m->hrr;
    // 3D: p^T A p comes with the product and r^T z with the V-cycle's last
    // fine sweep (workgroup partials of the EbE kernel)
    const bool ebe_dots = m->dim == 3;
    for (int it = 0; it < maxit; ++it) {
      int n_pq = 0;
      if (ebe_dots) {
        n_pq = launch_ebe_dot(g, m->wk, m->E, m->mask, m->pv, m->q, m->part_pq, s, m->tz64);
        ++m->sweeps;
        KCHECK();
      } else {
        TRY(apply(m, 0, m->pv, m->q, s));
        launch_dot_partials(n3, m->pv, m->q, part_pq, s);
      }
      launch_cg_xr_fused(n3, sc + SC_RZ + it, ebe_dots ? m->part_pq : part_pq, n_pq,
                         sc + SC_PQ + it, x, m->r, m->pv, m->q, part_rr, m->lv[0].dinv,
                         m->p.omega, z0 ? m->z : nullptr, s);
      KCHECK();
      // the update stored the r^T r partials and the finished p^T q (after
      // them) into host memory: the event marks them complete
      HIP_TRY(hipEventRecord(m->ev_cg, s));
      if (it + 1 < maxit) {
        m->want_rz = ebe_dots;
        m->rz_nb = 0;
        const int rc = vcycle(m, 0, m->r, m->z, s, z0);
        m->want_rz = false;
        TRY(rc);
        if (m->rz_nb > 0) {
          launch_cg_p_fused(n3, m->part_rz, m->rz_nb, sc + SC_RZ + it + 1, sc + SC_RZ + it,
                            m->z, m->pv, s);
        } else {
          launch_dot_partials(n3, m->r, m->z, part_rz, s);
          launch_cg_p_fused(n3, part_rz, 0, sc + SC_RZ + it + 1, sc + SC_RZ + it, m->z, m->pv,
                            s);
        }
        KCHECK();
      }
      HIP_TRY(hipEventSynchronize(m->ev_cg));
      rr = 0.0;
      for (int b = 0; b < nb; ++b) rr += hrr[b];
      *iters = it + 1;
      *relres = std::sqrt(rr / ff);
      if (!(hrr[nb] > 0.0)) return fail(AARMR_E_SINGULAR, "CG: p^T A p <= 0");
      if (rr <= tol2) return AARMR_OK;
    }
  }
  return fail(AARMR_E_NOT_CONVERGED, "CG reached cg_maxit before cg_rtol" AARMR_OMEGA_HINT);
}

// phi = u / ||u|| into case l's PARM ring (eqs. 27-28, oldest dropped).
int push_parm(aarmr_mesh* m, int l, const double* u, hipStream_t s) {
  const int64_t n3 = ndof(m, 0);
  double* nrm = m->scal + SC_MISC + M_NRM;
  TRY(dot1(m, u, u, nrm, n3, s));
  const int slot = m->phi_head[l];
  double* dst = m->Phi + ((int64_t)l * m->p.Ns + slot) * n3;
  launch_scale_by_inv_sqrt(n3, u, nrm, dst, s);
  KCHECK();
  m->phi_head[l] = (slot + 1) % m->p.Ns;
  m->phi_count[l] = std::min(m->phi_count[l] + 1, m->p.Ns);
  return AARMR_OK;
}

int check_common(aarmr_mesh* m, const double* rho, const double* f, int32_t n_rhs,
                 const int64_t* fixed, int64_t n_fixed, double* u) {
  TRY(need_ws(m));
  if (!rho || !f || !u) return fail(AARMR_E_INVALID, "null rho, f or u");
  if (n_rhs < 1 || n_rhs > m->p.n_rhs_max) return fail(AARMR_E_INVALID, "n_rhs out of range");
  if (n_fixed < 0 || (n_fixed > 0 && !fixed)) return fail(AARMR_E_INVALID, "bad fixed DOF list");
  return AARMR_OK;
}

int finish_flags(aarmr_mesh* m, hipStream_t s) {
  unsigned fl = 0;
  TRY(read_flags(m, &fl, s));
  m->mask_changed = (fl & 4u) != 0 || !m->ainv_valid;
  if (fl & 1u) return fail(AARMR_E_INVALID, "density outside [0, 1]");
  if (fl & 2u) return fail(AARMR_E_INVALID, "fixed DOF id out of range");
  return AARMR_OK;
}

// compliance, energy and dc contribution of case l.
int post_case(aarmr_mesh* m, int l, const double* rho_phys, const double* ul, double* compliance,
              bool want_dc, hipStream_t s) {
  const Grid& g = m->lg[0];
  const int64_t n3 = ndof(m, 0);
  if (compliance) {
    double* c = m->scal + SC_MISC + M_C;
    TRY(dot1(m, m->fm, ul, c, n3, s));
    double h;
    TRY(read_scalars(m, (const double* const*)&c, 1, &h, s));
    compliance[l] = h;
  }
  if (want_dc) {
    if (m->dim == 2)
      launch_q4_energy(g, m->KEd, m->mask, ul, ul, m->ework, s);
    else
      launch_energy_walsh(g, m->wk, m->mask, ul, m->ework, s);
    KCHECK();
    launch_dc_accum(g.ne, rho_phys, m->ework, m->p.E0, m->p.Emin, m->p.penal, m->dc_tmp, l == 0,
                    s);
    KCHECK();
  }
  return AARMR_OK;
}

// AARMR_MUTUAL_SENS: dc = -dE/drho~ u1_e^T KE u0_e (the sensitivity of
// f_1^T u_0 with case 1's solution as the adjoint).
int mutual_dc(aarmr_mesh* m, const double* rho_phys, const double* u, hipStream_t s) {
  const Grid& g = m->lg[0];
  const int64_t n3 = ndof(m, 0);
  launch_q4_energy(g, m->KEd, m->mask, u + n3, u, m->ework, s);
  KCHECK();
  launch_dc_accum(g.ne, rho_phys, m->ework, m->p.E0, m->p.Emin, m->p.penal, m->dc_tmp, 1, s);
  KCHECK();
  return AARMR_OK;
}

int check_mutual(const aarmr_mesh* m, int32_t n_rhs, int32_t flags) {
  if (!(flags & AARMR_MUTUAL_SENS)) return AARMR_OK;
  if (m->dim != 2) return fail(AARMR_E_INVALID, "AARMR_MUTUAL_SENS needs the plane-stress grid");
  if (n_rhs != 2) return fail(AARMR_E_INVALID, "AARMR_MUTUAL_SENS needs n_rhs = 2");
  return AARMR_OK;
}

int finish_dc(aarmr_mesh* m, double* dc, int32_t flags, hipStream_t s) {
  const Grid& g = m->lg[0];
  if (!dc) return AARMR_OK;
  if (flags & AARMR_FILTER_INPUT) {
    launch_filter(m->fg, m->p.rmin, m->Wf, 1, m->Hs, m->dc_tmp, dc, s);
  } else {
    HIP_TRY(hipMemcpyAsync(dc, m->dc_tmp, g.ne * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  KCHECK();
  return AARMR_OK;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

extern "C" {

void aarmr_default_params(aarmr_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->nx = p->ny = p->nz = 8;
  p->E0 = 1.0;
  p->Emin = 1e-9;
  p->nu = 0.3;
  p->penal = 3.0;
  p->rmin = 2.5;
  p->mg_levels = 3;
  p->nu_pre = 1;
  p->nu_post = 1;
  p->omega = 0.6;
  p->cg_rtol = 1e-8;
  p->cg_maxit = 2000;
  p->precision = AARMR_FP64;
  p->Ns = 2;
  p->Nm = 2;
  p->ca_tol = 1e-3;
  p->gs_tau = 1e-10;
  p->n_rhs_max = 1;
  p->orth = AARMR_ORTH_GS;
  p->oc_eta = 0.5;
}

int aarmr_mesh_create(const aarmr_params* p, aarmr_mesh** out) {
  if (!p || !out) return fail(AARMR_E_INVALID, "null argument");
  *out = nullptr;
  if (p->nx < 1 || p->ny < 1 || p->nz < 0)
    return fail(AARMR_E_INVALID, "grid sizes must be >= 1 (nz = 0: plane stress)");
  const int dim = p->nz == 0 ? 2 : 3;
  if (dim == 2 && p->precision != AARMR_FP64)
    return fail(AARMR_E_INVALID, "the plane-stress grid supports AARMR_FP64 only");
  if (p->mg_levels < 2 || p->mg_levels > AARMR_MAX_LEVELS)
    return fail(AARMR_E_INVALID, "mg_levels outside [2, 8]");
  const int f = 1 << (p->mg_levels - 1);
  if (p->nx % f || p->ny % f || p->nz % f)
    return fail(AARMR_E_INVALID, "grid sizes not divisible by 2^(mg_levels-1)");
  if (p->Ns < 1 || p->Ns > AARMR_MAX_BASIS || p->Nm < 1 || p->Nm > AARMR_MAX_BASIS)
    return fail(AARMR_E_INVALID, "Ns/Nm outside [1, 10]");
  if (p->n_rhs_max < 1 || p->n_rhs_max > AARMR_MAX_RHS)
    return fail(AARMR_E_INVALID, "n_rhs_max outside [1, 8]");
  if (p->orth != AARMR_ORTH_GS && p->orth != AARMR_ORTH_SVD)
    return fail(AARMR_E_INVALID, "unknown orthogonalisation");
  if (!(p->oc_eta > 0.0 && p->oc_eta <= 1.0)) return fail(AARMR_E_INVALID, "oc_eta outside (0, 1]");
  if (!(p->nu > -1.0 && p->nu < 0.5)) return fail(AARMR_E_INVALID, "nu outside (-1, 0.5)");
  if (!(p->E0 > p->Emin && p->Emin > 0.0)) return fail(AARMR_E_INVALID, "need E0 > Emin > 0");
  if (p->cg_maxit < 1 || p->cg_maxit > kMaxIt) return fail(AARMR_E_INVALID, "cg_maxit outside [1, 4096]");
  if (p->precision != AARMR_FP64 && p->precision != AARMR_FP32_REFINE)
    return fail(AARMR_E_INVALID, "unknown precision");
  if (p->nu_pre < 0 || p->nu_post < 0 || !(p->omega > 0.0))
    return fail(AARMR_E_INVALID, "bad smoother parameters");
  if (dim * (int64_t)(p->nx + 1) * (p->ny + 1) * (p->nz + 1) >= (int64_t(1) << 31))
    return fail(AARMR_E_INVALID, "grid too large: DOF count must stay below 2^31");
  // The fine-grid hex8 product addresses its vectors and moduli with 32-bit
  // byte offsets and parks idle lanes at offset 2^31, so every FP64 array it
  // reads or writes must stay below 2^31 bytes.
  if (dim == 3) {
    const int64_t nn3 = (int64_t)(p->nx + 1) * (p->ny + 1) * (p->nz + 1);
    const int64_t ne3 = (int64_t)p->nx * p->ny * p->nz;
    if (3 * nn3 * 8 >= (int64_t(1) << 31) || ne3 * 8 >= (int64_t(1) << 31))
      return fail(AARMR_E_INVALID,
                  "grid too large: 3 * n_node * 8 and n_elem * 8 bytes must stay below 2^31");
  }
  aarmr_mesh* m = new aarmr_mesh();
  m->p = *p;
  m->dim = dim;
  m->nlev = p->mg_levels;
  for (int l = 0; l < m->nlev; ++l) m->lg[l] = make_grid(p->nx >> l, p->ny >> l, p->nz >> l);
  m->fg = make_grid(p->nx, p->ny, std::max(p->nz, 1));
  m->nc = (int)(dim * m->lg[m->nlev - 1].nn);
  if (m->nc > 8192) {
    delete m;
    return fail(AARMR_E_INVALID, "coarsest grid above 8192 DOFs: use more levels");
  }
  if (dim == 2) {
    q4_stiffness(p->nu, m->KE);  // unit modulus and thickness
    *out = m;
    return AARMR_OK;
  }
  hex8_stiffness(p->nu, m->KE);  // unit modulus; E0 enters through SIMP
  child_galerkin(m->KE, m->Mc);
  m->N2.resize(64 * kSymEntries);
  grandchild_galerkin(m->Mc, m->N2.data());
  walsh_child(m->Mc, m->Bw);
  for (int x = 0; x < 576; ++x) m->Bw32[x] = (float)m->Bw[x];
  if (!walsh_parent_check(m->Mc, m->Bw)) {
    delete m;
    return fail(AARMR_E_INVALID, "Walsh form of the level-1 operator does not reproduce it");
  }
  m->fp32 = (p->precision == AARMR_FP32_REFINE);
  if (!mirror_children(m->Mc)) {
    delete m;
    return fail(AARMR_E_INVALID, "child Galerkin matrices are not mirror images of child 0's");
  }
  if (!walsh_form(m->KE, &m->wk)) {
    delete m;
    return fail(AARMR_E_INVALID, "element stiffness lacks the reflection-blocked structure");
  }
  *out = m;
  return AARMR_OK;
}

void aarmr_mesh_destroy(aarmr_mesh* m) {
  if (!m) return;
  if (m->hpin) (void)hipHostFree(m->hpin);
  if (m->hrr) (void)hipHostFree(m->hrr);
  if (m->ev_cg) (void)hipEventDestroy(m->ev_cg);
  if (m->ev_fine) (void)hipEventDestroy(m->ev_fine);
  if (m->ev_mg) (void)hipEventDestroy(m->ev_mg);
  if (m->side) (void)hipStreamDestroy(m->side);
  delete m;
}

int64_t aarmr_workspace_bytes(const aarmr_mesh* m) {
  if (!m) return -1;
  aarmr_mesh tmp = *m;
  tmp.hpin = nullptr;
  tmp.hrr = tmp.hrr_dev = nullptr;
  tmp.ev_cg = nullptr;
  tmp.ev_fine = tmp.ev_mg = nullptr;
  tmp.side = nullptr;
  return layout(&tmp, nullptr);
}

int aarmr_bind_workspace(aarmr_mesh* m, void* dev_ptr, int64_t bytes, void* stream) {
  if (!m || !dev_ptr) return fail(AARMR_E_INVALID, "null argument");
  if (reinterpret_cast<uintptr_t>(dev_ptr) % kAlign) return fail(AARMR_E_INVALID, "workspace not 256-byte aligned");
  const int64_t need = layout(m, nullptr);
  if (bytes < need) return fail(AARMR_E_NO_WORKSPACE, "workspace too small");
  m->ainv_valid = false;  // a new workspace holds no inverse
  if (!m->hpin) HIP_TRY(hipHostMalloc((void**)&m->hpin, 4096 * sizeof(double), hipHostMallocDefault));
  if (!m->hrr) {
    HIP_TRY(hipHostMalloc((void**)&m->hrr,
                          (int64_t)m->p.n_rhs_max * (kFusedBlocks + 8) * sizeof(double),
                          hipHostMallocMapped | hipHostMallocCoherent));
    HIP_TRY(hipHostGetDevicePointer((void**)&m->hrr_dev, m->hrr, 0));
  }
  m->hact = reinterpret_cast<int*>(m->hpin + 3072);  // lock-step flags (n_rhs_max ints)
  if (!m->ev_cg) HIP_TRY(hipEventCreateWithFlags(&m->ev_cg, hipEventDisableTiming));
  if (!m->ev_fine) HIP_TRY(hipEventCreateWithFlags(&m->ev_fine, hipEventDisableTiming));
  if (!m->ev_mg) HIP_TRY(hipEventCreateWithFlags(&m->ev_mg, hipEventDisableTiming));
  // default priority; non-blocking so that it does not serialise with the null stream
  if (!m->side) HIP_TRY(hipStreamCreateWithFlags(&m->side, hipStreamNonBlocking));
  m->ws = static_cast<char*>(dev_ptr);
  m->ws_bytes = bytes;
  layout(m, m->ws);
  hipStream_t s = S(stream);
  HIP_TRY(hipMemcpyAsync(m->KEd, m->KE, 576 * sizeof(double), hipMemcpyHostToDevice, s));
  if (m->dim == 3) {
    HIP_TRY(hipMemcpyAsync(m->Mcd, m->Mc, 8 * kSymEntries * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(m->N2d, m->N2.data(), 64 * kSymEntries * sizeof(double),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(m->Bwd, m->Bw, 576 * sizeof(double), hipMemcpyHostToDevice, s));
  }
  if (m->fp32) {
    HIP_TRY(hipMemcpyAsync(m->Bw32d, m->Bw32, 576 * sizeof(float), hipMemcpyHostToDevice, s));
  }
  HIP_TRY(hipMemsetAsync(m->flags, 0, 64, s));
  HIP_TRY(hipMemsetAsync(m->mask, 0, (m->lg[0].nn + 3) / 4 * 4, s));
  launch_fill(m->lg[0].ne, 1.0, m->ones_dv, s);
  KCHECK();
  if (m->p.rmin > 0.0) {
    m->Wh.assign(filter_taps(m->p.rmin), 0.0);
    filter_weights(m->p.rmin, m->Wh.data());
    HIP_TRY(hipMemcpyAsync(m->Wf, m->Wh.data(), m->Wh.size() * sizeof(double),
                           hipMemcpyHostToDevice, s));
    launch_filter_rowsum(m->fg, m->p.rmin, m->Hs, s);
    KCHECK();
    launch_filter(m->fg, m->p.rmin, m->Wf, 1, m->Hs, m->ones_dv, m->cw, s);
    KCHECK();
  }
  HIP_TRY(hipStreamSynchronize(s));
  for (int l = 0; l < AARMR_MAX_RHS; ++l) m->phi_count[l] = m->phi_head[l] = 0;
  m->have_prev = false;
  m->mg_ready = false;
  return AARMR_OK;
}

int aarmr_setup(aarmr_mesh* m, const double* rho_phys, const int64_t* fixed_dofs, int64_t n_fixed,
                void* stream) {
  TRY(need_ws(m));
  if (!rho_phys) return fail(AARMR_E_INVALID, "null rho");
  if (n_fixed < 0 || (n_fixed > 0 && !fixed_dofs)) return fail(AARMR_E_INVALID, "bad fixed DOF list");
  m->reuse_req = false;
  return setup(m, rho_phys, fixed_dofs, n_fixed, true, S(stream));
}

int aarmr_apply_operator(aarmr_mesh* m, int32_t level, const double* v, double* y, int32_t flags,
                         void* stream) {
  TRY(need_ws(m));
  if (!v || !y || v == y) return fail(AARMR_E_INVALID, "v, y must be distinct non-null");
  if (level < 0 || level >= m->nlev) return fail(AARMR_E_INVALID, "level out of range");
  if (level > 0 && !m->mg_ready) return fail(AARMR_E_STATE, "no hierarchy: call aarmr_setup");
  return apply(m, level, v, y, S(stream), !(flags & AARMR_INPUT_MASKED));
}

int aarmr_vcycle(aarmr_mesh* m, const double* r, double* z, void* stream) {
  TRY(need_ws(m));
  if (!r || !z || r == z) return fail(AARMR_E_INVALID, "r, z must be distinct non-null");
  if (!m->mg_ready) return fail(AARMR_E_STATE, "no hierarchy: call aarmr_setup");
  return vcycle(m, 0, r, z, S(stream));
}

int aarmr_element_energy(aarmr_mesh* m, const double* u, double* energy, void* stream) {
  TRY(need_ws(m));
  if (!u || !energy) return fail(AARMR_E_INVALID, "null argument");
  if (m->dim == 2)
    launch_q4_energy(m->lg[0], m->KEd, m->mask, u, u, energy, S(stream));
  else
    launch_energy_walsh(m->lg[0], m->wk, m->mask, u, energy, S(stream));
  KCHECK();
  return AARMR_OK;
}

int aarmr_filter(aarmr_mesh* m, int32_t mode, const double* in, double* out, void* stream) {
  TRY(need_ws(m));
  if (!in || !out || in == out) return fail(AARMR_E_INVALID, "in, out must be distinct non-null");
  if (mode != 0 && mode != 1) return fail(AARMR_E_INVALID, "mode must be 0 or 1");
  if (!(m->p.rmin > 0.0)) return fail(AARMR_E_INVALID, "filter disabled (rmin <= 0)");
  launch_filter(m->fg, m->p.rmin, m->Wf, mode, m->Hs, in, out, S(stream));
  KCHECK();
  return AARMR_OK;
}

int aarmr_solve(aarmr_mesh* m, const double* rho, const double* f, int32_t n_rhs,
                const int64_t* fixed_dofs, int64_t n_fixed, double* u, double* compliance,
                double* dc, int32_t flags, aarmr_stats* st, void* stream) {
  TRY(check_common(m, rho, f, n_rhs, fixed_dofs, n_fixed, u));
  if ((flags & AARMR_FILTER_INPUT) && !(m->p.rmin > 0.0))
    return fail(AARMR_E_INVALID, "AARMR_FILTER_INPUT needs rmin > 0");
  TRY(check_mutual(m, n_rhs, flags));
  const bool mutual = (flags & AARMR_MUTUAL_SENS) != 0;
  hipStream_t s = S(stream);
  const Grid& g = m->lg[0];
  const int64_t n3 = ndof(m, 0);
  auto t0 = std::chrono::steady_clock::now();
  const int64_t sw0 = m->sweeps;
  const double* rho_phys = rho;
  if (flags & AARMR_FILTER_INPUT) {
    launch_filter(m->fg, m->p.rmin, m->Wf, 0, m->Hs, rho, m->rho_f, s);
    KCHECK();
    rho_phys = m->rho_f;
  }
  m->reuse_req = (flags & AARMR_REUSE_COARSEST) != 0;
  const int inv0 = m->ainv_builds;
  TRY(setup(m, rho_phys, fixed_dofs, n_fixed, false, s));
  TRY(finish_flags(m, s));  // also tells whether the fixed DOFs changed
  TRY(build_mg(m, s));
  if (st) {
    std::memset(st, 0, sizeof(*st));
    st->setup_ms = ms_since(t0);
  }
  auto t1 = std::chrono::steady_clock::now();
  int status = AARMR_OK;
  // Several load cases of the refinement form run their FP32 solves in lock
  // step (one set of launches per iteration for all of them); each case
  // gets the iterates of its own single-case solve.
  const bool lockstep = m->fp32 && m->dim == 3 && n_rhs > 1 && m->p.nu_post >= 1 &&
                        !m->ainv_stale;
  if (lockstep) {
    for (int l = 0; l < n_rhs; ++l) {
      double* ul = u + l * n3;
      if (flags & AARMR_WARM_START) {
        launch_copy_masked(g, ul, m->mask, ul, s, m->dim);
        KCHECK();
      } else {
        HIP_TRY(hipMemsetAsync(ul, 0, n3 * sizeof(double), s));
      }
    }
    int its[AARMR_MAX_RHS] = {}, stl[AARMR_MAX_RHS] = {};
    double rel[AARMR_MAX_RHS] = {};
    bool fb[AARMR_MAX_RHS] = {};
    TRY(refine_multi(m, n_rhs, f, u, its, rel, fb, stl, s));
    int its_max = 0;
    for (int l = 0; l < n_rhs; ++l) {
      double* ul = u + l * n3;
      if (fb[l]) {  // FP32 could not resolve this case: FP64 CG from its iterate
        launch_copy_masked(g, f + l * n3, m->mask, m->fm, s, m->dim);
        KCHECK();
        int more = 0;
        const int rc = pcg64(m, ul, &more, &rel[l], std::min(m->p.cg_maxit, kMaxIt) - its[l], s);
        its[l] += more;
        if (rc != AARMR_OK && rc != AARMR_E_NOT_CONVERGED) return rc;
        if (rc == AARMR_E_NOT_CONVERGED) status = rc;
      } else if (stl[l] != AARMR_OK) {
        status = stl[l];
      }
      if (!fb[l]) {  // C = f^T u below reads this case's masked load
        launch_copy_masked(g, f + l * n3, m->mask, m->fm, s, m->dim);
        KCHECK();
      }
      its_max = std::max(its_max, its[l]);
      if (st) {
        st->iterations[l] = its[l];
        st->rel_residual[l] = rel[l];
      }
      TRY(post_case(m, l, rho_phys, ul, compliance, dc != nullptr && !mutual, s));
      if (flags & AARMR_RECORD_PARM) TRY(push_parm(m, l, ul, s));
    }
    if (m->ainv_fresh) {
      m->ainv_base_its = its_max;
      m->ainv_fresh = false;
    }
  }
  for (int l = 0; l < n_rhs && !lockstep; ++l) {
    double* ul = u + l * n3;
    launch_copy_masked(g, f + l * n3, m->mask, m->fm, s, m->dim);
    KCHECK();
    if (flags & AARMR_WARM_START) {
      launch_copy_masked(g, ul, m->mask, ul, s, m->dim);
      KCHECK();
    } else {
      HIP_TRY(hipMemsetAsync(ul, 0, n3 * sizeof(double), s));
    }
    int its = 0;
    double rel = 0.0;
    int rc = pcg_reuse(m, ul, &its, &rel, s);
    if (rc != AARMR_OK && rc != AARMR_E_NOT_CONVERGED) return rc;
    if (rc == AARMR_E_NOT_CONVERGED) status = rc;
    if (st) {
      st->iterations[l] = its;
      st->rel_residual[l] = rel;
    }
    TRY(post_case(m, l, rho_phys, ul, compliance, dc != nullptr && !mutual, s));
    if (flags & AARMR_RECORD_PARM) TRY(push_parm(m, l, ul, s));
  }
  if (dc && mutual) TRY(mutual_dc(m, rho_phys, u, s));
  TRY(finish_dc(m, dc, flags, s));
  HIP_TRY(hipMemcpyAsync(m->E_prev, m->E, g.ne * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  m->have_prev = true;
  if (st) {
    st->solve_ms = ms_since(t1);
    st->fine_sweeps = m->sweeps - sw0;
    st->coarsest_inversions = m->ainv_builds - inv0;
  }
  if (status != AARMR_OK) return fail(status, "CG reached cg_maxit before cg_rtol" AARMR_OMEGA_HINT);
  return AARMR_OK;
}

int aarmr_ca_update(aarmr_mesh* m, const double* rho, const double* f, int32_t n_rhs,
                    const int64_t* fixed_dofs, int64_t n_fixed, double* u, double* compliance,
                    double* dc, int32_t flags, aarmr_ca_stats* st, void* stream) {
  TRY(check_common(m, rho, f, n_rhs, fixed_dofs, n_fixed, u));
  if ((flags & AARMR_FILTER_INPUT) && !(m->p.rmin > 0.0))
    return fail(AARMR_E_INVALID, "AARMR_FILTER_INPUT needs rmin > 0");
  TRY(check_mutual(m, n_rhs, flags));
  const bool mutual = (flags & AARMR_MUTUAL_SENS) != 0;
  if (!m->have_prev) return fail(AARMR_E_STATE, "no reference design: run aarmr_solve first");
  for (int l = 0; l < n_rhs; ++l)
    if (m->phi_count[l] < m->p.Ns) return fail(AARMR_E_STATE, "PARM of a load case is not complete");
  hipStream_t s = S(stream);
  const Grid& g = m->lg[0];
  const int64_t n3 = ndof(m, 0);
  const int Ns = m->p.Ns, Nm = m->p.Nm;
  const int64_t sw0 = m->sweeps;
  if (st) std::memset(st, 0, sizeof(*st));
  const double* rho_phys = rho;
  if (flags & AARMR_FILTER_INPUT) {
    launch_filter(m->fg, m->p.rmin, m->Wf, 0, m->Hs, rho, m->rho_f, s);
    KCHECK();
    rho_phys = m->rho_f;
  }
  m->reuse_req = (flags & AARMR_REUSE_COARSEST) != 0;
  const int inv0 = m->ainv_builds;
  TRY(setup(m, rho_phys, fixed_dofs, n_fixed, false, s));
  TRY(finish_flags(m, s));
  // Algorithm 1 needs the MG hierarchy only when the reduced model is
  // rejected.  After a rejection, the next attempt builds it on a second
  // stream while the reduced model runs (both read the new moduli; neither
  // writes what the other reads); the fallback and the return wait for it.
  struct JoinOnExit {
    aarmr_mesh* m;
    hipStream_t s;
    ~JoinOnExit() { (void)join_mg(m, s); }
  } join_guard{m, s};
  if (m->spec_mg) {
    HIP_TRY(hipEventRecord(m->ev_fine, s));
    HIP_TRY(hipStreamWaitEvent(m->side, m->ev_fine, 0));
    TRY(build_mg(m, m->side));
    HIP_TRY(hipEventRecord(m->ev_mg, m->side));
    m->mg_pending = true;
  }
  bool any_rejected = false;
  launch_diff(g.ne, m->E, m->E_prev, m->dE, s);  // weights of dK = K - K0
  KCHECK();
  double* misc = m->scal + SC_MISC;
  int status = AARMR_OK;
  for (int l = 0; l < n_rhs; ++l) {
    double* ul = u + l * n3;
    const double* PhiL = m->Phi + (int64_t)l * Ns * n3;
    launch_copy_masked(g, f + l * n3, m->mask, m->fm, s, m->dim);
    KCHECK();
    launch_copy_masked(g, ul, m->mask, ul, s, m->dim);
    KCHECK();
    // eq. (15): K_Phi = Phi^T K0 Phi, K0 = K(previous design)
    for (int j = 0; j < Ns; ++j) {
      TRY(fine_product(m, m->E_prev, PhiL + j * n3, m->t0, s));
      std::vector<const double*> a(Ns), b(Ns);
      std::vector<double*> o(Ns);
      for (int i = 0; i < Ns; ++i) {
        a[i] = PhiL + i * n3;
        b[i] = m->t0;
        o[i] = misc + M_KPHI + i * Ns + j;
      }
      TRY(dots(m, Ns, a.data(), b.data(), o.data(), n3, s));
    }
    // eq. (20)/(26): r_1 = u_last, r_i = -Phi K_Phi^-1 Phi^T dK r_(i-1)
    HIP_TRY(hipMemcpyAsync(m->R, ul, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
    bool ca_ok = true;
    for (int i = 1; i < Nm; ++i) {
      TRY(fine_product(m, m->dE, m->R + (i - 1) * n3, m->t0, s, false));
      std::vector<const double*> a(Ns), b(Ns);
      std::vector<double*> o(Ns);
      for (int j = 0; j < Ns; ++j) {
        a[j] = PhiL + j * n3;
        b[j] = m->t0;
        o[j] = misc + M_G + j;
      }
      TRY(dots(m, Ns, a.data(), b.data(), o.data(), n3, s));
      launch_small_spd_solve(Ns, Ns, misc + M_KPHI, misc + M_G, misc + M_C2, m->flags, s);
      KCHECK();
      std::vector<const double*> V(Ns);
      for (int j = 0; j < Ns; ++j) V[j] = PhiL + j * n3;
      launch_lincomb(n3, Ns, V.data(), misc + M_C2, -1.0, nullptr, m->R + i * n3, s);
      KCHECK();
    }
    // Gram-Schmidt (two passes, classical) with rank drop, or the SVD of
    // eq. 21.  Gram-Schmidt runs on the device: every column stays in its
    // slot, a dropped one becomes zero (its projections onto later columns
    // are then exact zeros) with keep flag 0.  One read-back then brings the
    // keep flags and the flags word (bit 4: K_Phi not positive definite,
    // which rejects the step), and the reduced system uses the kept slots.
    std::vector<int> slot;  // kept columns, in order
    if (m->p.orth == AARMR_ORTH_SVD) {
      unsigned fl = 0;
      TRY(read_flags(m, &fl, s));
      if (fl & 4u) ca_ok = false;  // K_Phi not positive definite: reject CA
      int kept_svd = 0;
      if (ca_ok) TRY(orth_svd(m, Nm, &kept_svd, s));
      for (int j = 0; j < kept_svd; ++j) slot.push_back(j);
    } else {
      for (int i = 0; i < Nm; ++i) {
        double* v = m->R + i * n3;
        TRY(dot1(m, v, v, misc + M_N0 + i, n3, s));
        for (int pass = 0; pass < 2 && i > 0; ++pass) {
          std::vector<const double*> a(i), b(i);
          std::vector<double*> o(i);
          for (int j = 0; j < i; ++j) {
            a[j] = m->R + j * n3;
            b[j] = v;
            o[j] = misc + M_H + j;
          }
          TRY(dots(m, i, a.data(), b.data(), o.data(), n3, s));
          launch_lincomb(n3, i, a.data(), misc + M_H, -1.0, v, v, s);
          KCHECK();
        }
        TRY(dot1(m, v, v, misc + M_N1 + i, n3, s));
        launch_gs_keep(n3, v, misc + M_N0 + i, misc + M_N1 + i, m->p.gs_tau, v,
                       misc + M_KEEP + i, s);
        KCHECK();
      }
      unsigned* hfl = reinterpret_cast<unsigned*>(m->hpin + 64);
      HIP_TRY(hipMemcpyAsync(hfl, m->flags, sizeof(unsigned), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipMemsetAsync(m->flags, 0, sizeof(unsigned), s));
      std::vector<const double*> src(Nm);
      std::vector<double> keep(Nm);
      for (int i = 0; i < Nm; ++i) src[i] = misc + M_KEEP + i;
      TRY(read_scalars(m, src.data(), Nm, keep.data(), s));
      if (*hfl & 4u) ca_ok = false;  // K_Phi not positive definite: reject CA
      for (int i = 0; ca_ok && i < Nm; ++i)
        if (keep[i] != 0.0) slot.push_back(i);
    }
    const int kept = (int)slot.size();
    double eps = 1.0;
    if (kept > 0) {
      // eqs. (22)-(25): K_R~ = R~^T K R~, f_R~ = R~^T f, y, u~ = R~ y
      std::vector<const double*> Q(kept), KQ(kept);
      for (int j = 0; j < kept; ++j) {
        Q[j] = m->R + slot[j] * n3;
        KQ[j] = m->KR + slot[j] * n3;
        TRY(fine_product(m, m->E, Q[j], m->KR + slot[j] * n3, s));
      }
      std::vector<const double*> a, b;
      std::vector<double*> o;
      for (int i = 0; i < kept; ++i)
        for (int j = 0; j < kept; ++j) {
          a.push_back(Q[i]);
          b.push_back(KQ[j]);
          o.push_back(misc + M_KR + i * kept + j);
        }
      for (int i = 0; i < kept; ++i) {
        a.push_back(Q[i]);
        b.push_back(m->fm);
        o.push_back(misc + M_FR + i);
      }
      a.push_back(m->fm);
      b.push_back(m->fm);
      o.push_back(misc + M_FF);
      TRY(dots(m, (int)a.size(), a.data(), b.data(), o.data(), n3, s));
      launch_small_spd_solve(kept, kept, misc + M_KR, misc + M_FR, misc + M_Y, m->flags, s);
      KCHECK();
      launch_lincomb(n3, kept, Q.data(), misc + M_Y, 1.0, nullptr, ul, s);
      KCHECK();
      // eq. (29) from the stored K R~ columns: f - sum_j y_j K r~_j
      launch_lincomb(n3, kept, KQ.data(), misc + M_Y, -1.0, m->fm, m->t0, s);
      KCHECK();
      TRY(dot1(m, m->t0, m->t0, misc + M_EPS, n3, s));
      // one read-back: eps^2, f^T f and the flags (bit 4: K_R~ not positive definite)
      unsigned* hfl = reinterpret_cast<unsigned*>(m->hpin + 64);
      HIP_TRY(hipMemcpyAsync(hfl, m->flags, sizeof(unsigned), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipMemsetAsync(m->flags, 0, sizeof(unsigned), s));
      double h[2];
      const double* src[2] = {misc + M_EPS, misc + M_FF};
      TRY(read_scalars(m, src, 2, h, s));
      eps = (h[1] > 0.0 && !(*hfl & 4u)) ? std::sqrt(h[0] / h[1]) : 1.0;
      if (h[1] == 0.0) eps = 0.0;
    }
    const bool accept = kept > 0 && eps < m->p.ca_tol;
    if (st) {
      st->eps[l] = eps;
      st->accepted[l] = accept ? 1 : 0;
      st->rank[l] = kept;
      st->rel_residual[l] = eps;
    }
    if (!accept) {
      // Algorithm 1 lines 9-10: MGCG warm-started from u~, then PARM update
      any_rejected = true;
      if (kept == 0) HIP_TRY(hipMemsetAsync(ul, 0, n3 * sizeof(double), s));
      TRY(join_mg(m, s));
      if (!m->mg_ready) TRY(build_mg(m, s));
      int its = 0;
      double rel = 0.0;
      int rc = pcg_reuse(m, ul, &its, &rel, s);
      if (rc != AARMR_OK && rc != AARMR_E_NOT_CONVERGED) return rc;
      if (rc == AARMR_E_NOT_CONVERGED) status = rc;
      if (st) {
        st->mgcg_iterations[l] = its;
        st->rel_residual[l] = rel;
      }
      TRY(push_parm(m, l, ul, s));
    }
    TRY(post_case(m, l, rho_phys, ul, compliance, dc != nullptr && !mutual, s));
  }
  if (dc && mutual) TRY(mutual_dc(m, rho_phys, u, s));
  TRY(finish_dc(m, dc, flags, s));
  TRY(join_mg(m, s));
  m->spec_mg = any_rejected;
  HIP_TRY(hipMemcpyAsync(m->E_prev, m->E, g.ne * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (st) {
    st->fine_sweeps = m->sweeps - sw0;
    st->coarsest_inversions = m->ainv_builds - inv0;
  }
  if (status != AARMR_OK)
    return fail(status, "fallback CG reached cg_maxit before cg_rtol" AARMR_OMEGA_HINT);
  return AARMR_OK;
}

int aarmr_set_springs(aarmr_mesh* m, const int64_t* dofs, const double* k, int32_t n) {
  if (!m) return fail(AARMR_E_INVALID, "null mesh");
  if (m->dim != 2) return fail(AARMR_E_INVALID, "springs need the plane-stress grid");
  if (n < 0 || n > AARMR_MAX_SPRINGS) return fail(AARMR_E_INVALID, "spring count outside [0, 8]");
  if (n > 0 && (!dofs || !k)) return fail(AARMR_E_INVALID, "null spring arrays");
  SpringSet S{};
  const int64_t nd = ndof(m, 0);
  for (int i = 0; i < n; ++i) {
    if (dofs[i] < 0 || dofs[i] >= nd) return fail(AARMR_E_INVALID, "spring DOF id out of range");
    if (!(k[i] >= 0.0)) return fail(AARMR_E_INVALID, "spring stiffness must be >= 0");
    int j = 0;
    while (j < S.n && S.dof[j] != dofs[i]) ++j;  // repeated ids add up
    if (j == S.n) {
      S.dof[S.n] = dofs[i];
      S.k[S.n++] = 0.0;
    }
    S.k[j] += k[i];
  }
  m->springs = S;
  m->mg_ready = false;
  m->ainv_valid = false;
  return AARMR_OK;
}

int aarmr_oc_update(aarmr_mesh* m, const double* x, const double* dc, const double* dv,
                    double volfrac, double move, double* x_new, double* rho_phys_new,
                    void* stream) {
  TRY(need_ws(m));
  if (!x || !dc || !dv || !x_new || !rho_phys_new) return fail(AARMR_E_INVALID, "null argument");
  if (!(m->p.rmin > 0.0)) return fail(AARMR_E_INVALID, "OC needs the filter (rmin > 0)");
  hipStream_t s = S(stream);
  const Grid& g = m->lg[0];
  double* lam = m->scal + SC_MISC + M_OC;
  // the volume of the filtered trial density, sum_e (H x / Hs)_e, is the
  // weighted sum sum_j cw_j x_j: no filter inside the bisection
  const double target = volfrac * (double)g.ne;
  const int nparts = kRedBlocks;
  launch_oc_init(lam, s);
  KCHECK();
  // three bisection steps per launch pair, 200 at most (the kernels count
  // them; pairs after the end return at once).  The done flag is first read
  // after one pair more than the previous call needed, then every 4 pairs.
  const int first = std::min(67, std::max(4, m->oc_pairs + 1));
  for (int it = 0; it < 67; ++it) {
    launch_oc_step3(g.ne, x, dc, dv, m->cw, move, m->p.oc_eta, lam, m->partial, nparts, s);
    launch_oc_bisect3(lam, m->partial, nparts, target, s);
    KCHECK();
    if (it + 1 >= first && (it + 1 - first) % 4 == 0) {
      double h[2];
      const double* src[2] = {lam + 3, lam + 4};
      TRY(read_scalars(m, src, 2, h, s));
      if (h[0] != 0.0) {
        m->oc_pairs = ((int)h[1] + 2) / 3;
        break;
      }
    }
  }
  launch_oc_final(g.ne, x, dc, dv, move, m->p.oc_eta, lam, x_new, s);
  KCHECK();
  launch_filter(m->fg, m->p.rmin, m->Wf, 0, m->Hs, x_new, rho_phys_new, s);
  KCHECK();
  return AARMR_OK;
}

int aarmr_oc_update_noalloc(aarmr_mesh* m, const double* x, const double* dc, const double* dv,
                            double volfrac, double move, double* x_new, double* rho_phys_new,
                            void* stream) {
  TRY(need_ws(m));
  if (!x || !dc || !dv || !x_new || !rho_phys_new) return fail(AARMR_E_INVALID, "null argument");
  if (!(m->p.rmin > 0.0)) return fail(AARMR_E_INVALID, "OC needs the filter (rmin > 0)");
  const Grid& g = m->lg[0];
  // the partials are per reduction block, not per element: any grid fits
  const int nparts = kRedBlocks;
  if (kOcScratchLam + 7 * nparts > kOcScratchDoubles)
    return fail(AARMR_E_INVALID, "OC scratch above its static maximum");
  double* base = nullptr;
  TRY(oc_scratch_ptr(&base));
  hipStream_t s = S(stream);
  double* lam = base;
  double* partial = base + kOcScratchLam;
  const double target = volfrac * (double)g.ne;
  // the bisection state starts from the kernel's fill, never from what the
  // array held after an earlier call
  launch_oc_init(lam, s);
  KCHECK();
  // no read-back: every pair is issued (at most 200 bisection steps in 67
  // pairs; pairs after convergence return at once)
  for (int it = 0; it < 67; ++it) {
    launch_oc_step3(g.ne, x, dc, dv, m->cw, move, m->p.oc_eta, lam, partial, nparts, s);
    launch_oc_bisect3(lam, partial, nparts, target, s);
    KCHECK();
  }
  launch_oc_final(g.ne, x, dc, dv, move, m->p.oc_eta, lam, x_new, s);
  KCHECK();
  launch_filter(m->fg, m->p.rmin, m->Wf, 0, m->Hs, x_new, rho_phys_new, s);
  KCHECK();
  return AARMR_OK;
}

int aarmr_set_chunk(aarmr_mesh* m, int32_t tz64, int32_t tz32) {
  if (!m) return fail(AARMR_E_INVALID, "null mesh");
  for (int sh : {tz64, tz32}) {
    const int tz = sh & 0xFFFF, rows = sh >> 16;
    if (sh < 0 || tz == 1 || (rows != 0 && rows != 8 && rows != 12 && rows != 16))
      return fail(AARMR_E_INVALID,
                  "launch shape: chunk length 0 (default) or >= 2, tile rows 0, 8, 12 or 16");
  }
  m->tz64 = tz64;
  m->tz32 = tz32;
  return AARMR_OK;
}

int aarmr_autotune(aarmr_mesh* m, int32_t* tz_out, void* stream) {
  TRY(need_ws(m));
  if (m->dim == 2) {  // the plane-stress product has no tunable chunk
    if (tz_out) tz_out[0] = tz_out[1] = 0;
    return AARMR_OK;
  }
  hipStream_t s = S(stream);
  const Grid& g = m->lg[0];
  const int planes = g.nz + 1;
  const int64_t n3 = ndof(m, 0);
  std::vector<int> cand{0};  // 0: the residency-sized default
  for (int t : {2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512})
    if (t <= planes) cand.push_back(t);
  if (planes > 4) cand.push_back(planes);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  auto time_one = [&](auto launch) -> float {  // best of 3 rounds of 5 launches
    launch();  // warm-up
    float best_ms = 1e30f;
    for (int round = 0; round < 3; ++round) {
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < 5; ++r) launch();
      (void)hipEventRecord(e1, s);
      (void)hipEventSynchronize(e1);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      best_ms = std::min(best_ms, ms);
    }
    return best_ms;
  };
  // scratch operands: moduli 1, input 1 (the timing does not depend on values)
  launch_fill(g.ne, 1.0, m->ework, s);
  launch_fill(n3, 1.0, m->q, s);
  KCHECK();
  // launch shapes: tile rows (0 = the per-grid choice, 8, 12, 16) x chunk length
  std::vector<int> shapes;
  for (int rows : {0, 8, 12})
    for (int tz : cand) shapes.push_back(tz | (rows << 16));
  float best = 1e30f;
  int best_tz = 0;
  for (int sh : shapes) {
    const float ms = time_one([&] {
      launch_ebe(g, m->wk, m->ework, m->mask, m->q, m->t0, 2, s, sh);
    });
    if (ms < best) { best = ms; best_tz = sh; }
  }
  m->tz64 = best_tz;
  if (m->fp32) {
    // FP32 scratch: moduli in d32 (3 n_node >= n_elem floats), input in q32
    launch_fill_f32(g.ne, 1.0f, m->d32, s);
    launch_fill_f32(n3, 1.0f, m->q32, s);
    KCHECK();
    best = 1e30f;
    best_tz = 0;
    for (int sh : shapes) {
      const float ms = time_one([&] {
        launch_ebe_f32(g, m->wk, m->d32, m->mask, m->q32, m->p32, 2, s, sh);
      });
      if (ms < best) { best = ms; best_tz = sh; }
    }
    m->tz32 = best_tz;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  KCHECK();
  HIP_TRY(hipStreamSynchronize(s));
  if (tz_out) {
    tz_out[0] = m->tz64;
    tz_out[1] = m->tz32;
  }
  return AARMR_OK;
}

int aarmr_batch_submit(aarmr_batch_item* items, int32_t n_items, void* const* streams,
                       int32_t n_streams, aarmr_batch** out) {
  if (!out) return fail(AARMR_E_INVALID, "null handle pointer");
  *out = nullptr;
  if (n_items < 0 || (n_items > 0 && !items)) return fail(AARMR_E_INVALID, "bad item array");
  if (!streams || n_streams < 1 || n_streams > 64) return fail(AARMR_E_INVALID, "bad stream array");
  std::vector<int> order(n_items);
  for (int i = 0; i < n_items; ++i) {
    if (!items[i].mesh) return fail(AARMR_E_INVALID, "null mesh in batch");
    order[i] = i;
  }
  {
    std::vector<const aarmr_mesh*> seen;
    for (int i = 0; i < n_items; ++i) seen.push_back(items[i].mesh);
    std::sort(seen.begin(), seen.end());
    if (std::adjacent_find(seen.begin(), seen.end()) != seen.end())
      return fail(AARMR_E_INVALID, "a mesh appears twice in the batch");
  }
  for (int i = 0; i < n_items; ++i) __atomic_store_n(&items[i].done, 0, __ATOMIC_RELAXED);
  aarmr_batch* b = new aarmr_batch();
  b->items = items;
  b->n_items = n_items;
  b->streams.assign(streams, streams + n_streams);
  // largest first, then greedy: next item to the least-loaded worker (work ~
  // nodes x load cases)
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return items[x].mesh->lg[0].nn * items[x].n_rhs > items[y].mesh->lg[0].nn * items[y].n_rhs;
  });
  const int nw = std::max(1, std::min<int>(n_streams, n_items));
  b->queue.assign(nw, {});
  std::vector<int64_t> load(nw, 0);
  for (int i : order) {
    const int w = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    b->queue[w].push_back(i);
    load[w] += items[i].mesh->lg[0].nn * std::max(1, items[i].n_rhs);
  }
  for (int w = 0; w < nw; ++w)
    b->pool.emplace_back([b, w] {
      for (int i : b->queue[w]) {
        aarmr_batch_item& it = b->items[i];
        it.status = aarmr_solve(it.mesh, it.rho, it.f, it.n_rhs, it.fixed_dofs, it.n_fixed, it.u,
                                it.compliance, it.dc, it.flags, &it.stats, b->streams[w]);
        __atomic_store_n(&it.done, 1, __ATOMIC_RELEASE);  // aarmr_solve synchronised the stream
        b->n_done.fetch_add(1, std::memory_order_release);
      }
    });
  *out = b;
  return AARMR_OK;
}

int aarmr_batch_poll(aarmr_batch* b, int32_t* n_done) {
  if (!b || !n_done) return fail(AARMR_E_INVALID, "null argument");
  *n_done = b->n_done.load(std::memory_order_acquire);
  return AARMR_OK;
}

int aarmr_batch_wait(aarmr_batch* b) {
  if (!b) return fail(AARMR_E_INVALID, "null handle");
  for (auto& t : b->pool) t.join();
  int rc = AARMR_OK;
  for (void* st : b->streams)
    if (hipStreamSynchronize(S(st)) != hipSuccess && rc == AARMR_OK) rc = AARMR_E_HIP;
  for (int i = 0; i < b->n_items && rc == AARMR_OK; ++i)
    if (b->items[i].status != AARMR_OK) rc = b->items[i].status;
  delete b;
  if (rc != AARMR_OK) return fail(rc, "a batch item failed (see its status)");
  return AARMR_OK;
}

int aarmr_batch_solve(aarmr_batch_item* items, int32_t n_items, void* const* streams,
                      int32_t n_streams) {
  aarmr_batch* b = nullptr;
  TRY(aarmr_batch_submit(items, n_items, streams, n_streams, &b));
  return aarmr_batch_wait(b);
}

const char* aarmr_last_error(void) { return g_err.c_str(); }

}  // extern "C"
