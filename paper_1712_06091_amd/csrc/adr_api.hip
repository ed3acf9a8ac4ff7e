// Host driver and C ABI of the ADR amplitude solver (declarations in include/adr.h).
//
// Setup builds the ADR coefficients (Sec. 2.1), the Galerkin hierarchy of the
// preconditioner A_beta = (1-beta) H_2up + beta H_1up (eq. precADRup,
// eq. coarseGridMatrix) and the dense FP64 inverse of the coarsest operator.  The
// solve is FGMRES(m) in FP64 (Sec. 4.2) whose preconditioner is one V-cycle
// (Alg. TwoCycle applied recursively) in FP64 or complex FP32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <array>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/adr.h"
#include "adr_kernels.hpp"

namespace {

constexpr int kMaxLevels = 8;
constexpr int kMaxNu = 8;           // GMRES relaxation steps per sweep (dots fused <= 8)
constexpr int kMaxRestart = 8;
constexpr int kScalPerLevel = 256;  // device doubles per level for relaxation scalars
constexpr int kPin = 2048;          // pinned host doubles (partials and scalars read back)
// scalar block layout (doubles)
constexpr int kH = 0;                               // (kMaxNu+1) x kMaxNu complex, col-major
constexpr int kLdH = kMaxNu + 1;
constexpr int kS = kH + 2 * kLdH * kMaxNu;          // kMaxNu+1 scale factors
constexpr int kBeta = kS + kMaxNu + 1;              // norm of the initial residual
constexpr int kCoef = kBeta + 1;                    // kMaxNu complex update coefficients
// Krylov cycle: flexible GMRES(2) on this level (3 x 2 complex Hessenberg, column-major,
// leading dimension 3; scale factors of the two basis vectors; norm of the first).
constexpr int kKH = kCoef + 2 * kMaxNu;
constexpr int kKS = kKH + 12;
constexpr int kKBeta = kKS + 2;
static_assert(kKBeta + 1 <= kScalPerLevel, "scalar block too small");

std::string g_setup_error;

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

template <typename T>
struct LevelT {
  Grid G{};
  int S = 0;                 // stored stencil size (0 on the matrix-free level 0)
  cx<T> *planes = nullptr;   // S x N
  cx<T> *dinv = nullptr;
  cx<T> *x = nullptr, *xt = nullptr, *b = nullptr, *r = nullptr, *w = nullptr;
  cx<T> *V = nullptr;        // (kMaxNu+1) x N Arnoldi basis (unnormalized)
  cx<T> *Z = nullptr;        // (kMaxNu+1) x N, Z_j = D^{-1} V_j
  cx<T> *ku = nullptr;       // Krylov cycle: second coarse basis vector u_1
  cx<T> *kz = nullptr;       // Krylov cycle: first preconditioned direction K(u_0)
  int split = 1;             // Galerkin-apply variant (1, 4 or 8 = LDS tiles), tuned at setup
  int slabs = 0;             // split 8: z-slabs of the launch (tuned; 0 = the most)
  cx<T> *Gs = nullptr;       // pipelined relaxation: kMaxNu x N stored A D^{-1} u_i (see k_pipe_step)
  cx<T> *Yp = nullptr;       // pipelined relaxation: 2 x N, D^{-1} Gs_{k-1} (ping-pong)
  cx<T> *planes_adj = nullptr;   // conjugate-transposed stencil (adjoint solves)
  cx<T> *planes_t = nullptr;     // segment-tiled copy of planes for the LDS apply (split 8)
  cx<T> *planes_adj_t = nullptr; // ... and of planes_adj
  cx<T> *dinv_adj = nullptr;
};

// Slot layout of a merged shot group (problems of different grid shapes sharing every
// launch): each setup allocation is keyed by its source line and the number of
// allocations that line made before it in the same setup, and every key gets one offset
// in the slot, sized for the largest problem that makes it.  So buffer k of problem s sits
// at the same offset in every slot, and the largest problem's pointers, shifted by whole
// slots, reach every problem's buffers.
using AllocKey = std::pair<int, int>;
struct SlotLayout {
  std::map<AllocKey, std::pair<size_t, size_t>> at;   // key -> (offset, bytes)
  size_t stride = 0;
};

// Per-level grid tables of a merged group, in device memory: for launch kind k, level l
// and slot s, problem s's grid on level l where the launch applies to it, else a grid
// with N = 0 (the kernels return at once for it).  Relaxation kinds cover the problems
// for which l is above their coarsest level (they relax on l and restrict from it),
// coarsest kinds those whose coarsest level is l, full kinds every problem with a level l.
enum { kRelaxGrids = 0, kFullGrids = 1, kCoarsestGrids = 2, kGridKinds = 3 };
struct MergedGrids {
  int levels = 0, cols = 0;       // cols = problems + the spare slot (N = 0 everywhere)
  std::vector<int> slot_levels;   // levels of the problem in each slot
  Grid *dev = nullptr;            // [kGridKinds][levels][cols]
  const Grid *table(int kind, int l) const { return dev + ((size_t)kind * levels + l) * cols; }
  bool coarsest_at(int l) const {
    for (int L : slot_levels)
      if (L - 1 == l) return true;
    return false;
  }
};

}  // namespace

struct adr_ctx {
  adr_options opt{};
  hipStream_t stream = nullptr;
  int D = 3;
  Grid G0{};
  double h = 0, omega = 0;
  int src[3] = {-1, -1, -1};
  int levels = 1;
  int nu[kMaxLevels] = {0};
  adr_relax relax[kMaxLevels];

  // fine coefficients (FP64) + FP32 copies (mixed)
  double *g64[3] = {nullptr, nullptr, nullptr};
  double *L64 = nullptr;
  cx<double> *c64 = nullptr;
  float *g32[3] = {nullptr, nullptr, nullptr};
  float *L32 = nullptr;
  cx<float> *c32 = nullptr;
  cx<double> *cM64 = nullptr;  // reaction plane of the shifted preconditioner (shift_alpha > 0)
  cx<double> *ph64 = nullptr;  // exp(i w tau) when the cycle works on the rescaled operator
  cx<float> *ph32 = nullptr;   // its FP32 copy (mixed precision)
  cx<double> *vtmp = nullptr;  // rescaled cycle input (FP64 mode)
  double setup_ms = 0.0;       // wall time of the setup that built this context
  double *tau = nullptr;

  // hierarchy (one of the two, by precision)
  LevelT<double> lv64[kMaxLevels];
  LevelT<float> lv32[kMaxLevels];
  int *off_coarse = nullptr;   // device xyz table of the coarse stencil
  int *off_fine = nullptr;     // device xyz table of the fine stencil (Galerkin input)
  std::vector<int> h_off_coarse;
  int S_coarse = 0;
  cx<double> *Ainv = nullptr;  // coarsest inverse, row-major
  cx<double> *Ainv_adj = nullptr;   // its conjugate transpose (adjoint solves)
  std::vector<std::complex<double>> h_inv;   // host copy of the coarsest inverse
  int Ncoarsest = 0;
  double *gamma = nullptr;     // FP64 copy of gamma (kappa^2 gradient), NULL if none
  bool adj = false;            // direction of the current solve: false = H, true = H^H
  bool adj_ready = false;

  // scalars and reductions
  double *scal = nullptr;      // kMaxLevels * kScalPerLevel
  double *osc = nullptr;       // outer scalars (64 doubles)
  double *hpin = nullptr;      // pinned host mirror (kPin doubles)
  double *part[2] = {nullptr, nullptr};   // alternating reduction partials

  // outer FGMRES buffers
  cx<double> *Vo = nullptr;    // (kMaxRestart+1) x N
  void *Zo = nullptr;          // kMaxRestart x N, c64 (mixed) or c128
  cx<double> *wo = nullptr, *ro = nullptr, *qh = nullptr;
  cx<float> *b32 = nullptr, *z32 = nullptr;   // mixed-mode V-cycle in/out staging

  // Allocation: by default every device buffer is its own hipMalloc.  A context of a
  // shot group carves its setup allocations, in a fixed order, from one slot of the
  // group's arena [arena, arena + arena_cap), so that the buffers of problem s lie
  // s * stride bytes after problem 0's.  alloc_need counts the bytes a slot needs.
  char *arena = nullptr;
  size_t arena_off = 0, arena_cap = 0;
  const char *arena_lo = nullptr, *arena_hi = nullptr;
  size_t alloc_need = 0;
  const SlotLayout *layout = nullptr;   // merged groups: keyed offsets instead of a fixed order
  std::map<int, int> site_seen;          // allocations per source line so far (layout keys)
  std::vector<std::pair<AllocKey, size_t>> alloc_log;   // key and bytes of every allocation
  const MergedGrids *mg = nullptr;       // member of a merged group: the group's grid tables
  int mg_slot = 0;                       // ... and this problem's slot
  bool group_member = false;
  FineParams *Pdev = nullptr;     // device copies of the fine-operator parameters: [0] beta = 0, [1] A_beta
  int *active = nullptr;          // shot-group flag: 1 while the problem is being solved
  cx<double> *qin = nullptr, *xg = nullptr;   // shot-group copies of right-hand side and solution

  // Coarse tail: levels tail_level.. run in one single-workgroup kernel (-1: none); device
  // copies of its level table for the forward [0] and adjoint [1] hierarchies.
  int tail_level = -1;
  bool fine_tiles_on = false;  // finest-level LDS tiles chosen at setup (fine_tiles = 1 and faster)
  void *tail_args[2] = {nullptr, nullptr};

  // Captured V-cycles (Alg. TwoCycle applied recursively; no host synchronization
  // inside), keyed by their input/output buffers, replayed on `stream`.  Captured on a
  // private stream because the legacy default stream cannot be captured.
  struct GraphEntry {
    const void *in = nullptr;
    void *out = nullptr;
    bool adj = false;
    int group = 1;             // problems per launch (shot group) when captured
    hipGraph_t g = nullptr;
    hipGraphExec_t e = nullptr;
    unsigned long long last_use = 0;
  };
  std::vector<GraphEntry> graphs;
  unsigned long long graph_clock = 0;
  hipStream_t cap_stream = nullptr;

  // Event timing of one kernel class (benchmarks): pairs of events recorded on `stream`
  // around every launch of that class, plus the algorithmic bytes those launches move.
  struct {
    int kind = -1, level = -1;
    std::vector<hipEvent_t> ev;
    int used = 0, launches = 0;
    double bytes = 0.0;
  } timer;
  std::string err;
};

#define ADR_HIP(call)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      ctx->err = std::string(#call) + ": " + hipGetErrorString(e_);                         \
      return ADR_EHIP;                                                                       \
    }                                                                                        \
  } while (0)

namespace {

template <typename T>
adr_status dalloc(adr_ctx *ctx, T **p, size_t count, int site = __builtin_LINE()) {
  *p = nullptr;
  const AllocKey key{site, ctx->site_seen[site]++};
  if (count == 0) return ADR_OK;
  const size_t aligned = (count * sizeof(T) + 255) & ~(size_t)255;
  ctx->alloc_need += aligned;
  ctx->alloc_log.push_back({key, aligned});
  if (ctx->arena && ctx->layout) {
    auto it = ctx->layout->at.find(key);
    if (it == ctx->layout->at.end() || aligned > it->second.second) {
      ctx->err = "merged shot-group slot layout has no room for the allocation at line " + std::to_string(site);
      return ADR_ENOMEM;
    }
    *p = (T *)(ctx->arena + it->second.first);
    return ADR_OK;
  }
  if (ctx->arena) {
    if (ctx->arena_off + aligned > ctx->arena_cap) {
      ctx->err = "shot-group arena slot exhausted";
      return ADR_ENOMEM;
    }
    *p = (T *)(ctx->arena + ctx->arena_off);
    ctx->arena_off += aligned;
    return ADR_OK;
  }
  hipError_t e = hipMalloc((void **)p, count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    ctx->err = "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed: " + hipGetErrorString(e);
    return ADR_ENOMEM;
  }
  return ADR_OK;
}
// Free a buffer from dalloc (arena slots are released with their group).
void dfree(adr_ctx *ctx, void *p) {
  if (!p) return;
  const char *c = (const char *)p;
  if (ctx->arena_lo && c >= ctx->arena_lo && c < ctx->arena_hi) return;
  (void)hipFree(p);
}

#define ADR_TRY(x)                   \
  do {                               \
    adr_status s_ = (x);             \
    if (s_ != ADR_OK) return s_;     \
  } while (0)

// Stencil offset sets.  Fine: centre, then for each axis -2, -1, +1, +2 (matches
// fine_row's entry order).  Coarse: every offset with |d_k| <= 2 and at most one
// |d_k| == 2 (21 points in 2D, 81 in 3D), which the Galerkin product keeps closed.
std::vector<int> fine_offsets(int D) {
  std::vector<int> o = {0, 0, 0};
  for (int k = 0; k < D; ++k)
    for (int d : {-2, -1, 1, 2}) {
      int t[3] = {0, 0, 0};
      t[k] = d;
      o.insert(o.end(), t, t + 3);
    }
  return o;
}
std::vector<int> coarse_offsets(int D) {
  std::vector<int> o;
  const int zl = D == 3 ? -2 : 0, zh = D == 3 ? 2 : 0;
  for (int dz = zl; dz <= zh; ++dz)
    for (int dy = -2; dy <= 2; ++dy)
      for (int dx = -2; dx <= 2; ++dx) {
        int twos = (std::abs(dx) == 2) + (std::abs(dy) == 2) + (std::abs(dz) == 2);
        if (twos <= 1) o.insert(o.end(), {dx, dy, dz});
      }
  return o;
}

// For every output offset t, the list of (p, input offset index d, weight) with
// P^T support offset p in {-1,0,1}^D and q = p + off_in[d] - 2t in {-1,0,1}^D; the
// weight is w(p) w(q), w = prod_k (1 - |.|/2).
struct Triples {
  std::vector<int> start, p, d;
  std::vector<double> w;
};
Triples galerkin_triples(int D, const std::vector<int> &in, const std::vector<int> &out) {
  Triples T;
  const int Sin = (int)in.size() / 3, Sout = (int)out.size() / 3;
  const int zl = D == 3 ? -1 : 0, zh = D == 3 ? 1 : 0;
  T.start.push_back(0);
  for (int t = 0; t < Sout; ++t) {
    for (int pz = zl; pz <= zh; ++pz)
      for (int py = -1; py <= 1; ++py)
        for (int px = -1; px <= 1; ++px)
          for (int d = 0; d < Sin; ++d) {
            int p[3] = {px, py, pz};
            double w = 1.0;
            bool ok = true;
            for (int k = 0; k < 3; ++k) {
              int q = p[k] + in[3 * d + k] - 2 * out[3 * t + k];
              if (q < -1 || q > 1) { ok = false; break; }
              w *= (1.0 - 0.5 * std::abs(p[k])) * (1.0 - 0.5 * std::abs(q));
            }
            if (!ok) continue;
            T.p.insert(T.p.end(), p, p + 3);
            T.d.push_back(d);
            T.w.push_back(w);
          }
    T.start.push_back((int)T.d.size());
  }
  return T;
}

// Dense complex inverse by Gauss-Jordan elimination with partial pivoting (host,
// FP64; the coarsest grid has at most a few thousand nodes).  A and the inverse are
// row-major n x n.
bool dense_inverse(int n, std::vector<std::complex<double>> &A, std::vector<std::complex<double>> &inv) {
  std::vector<std::complex<double>> I((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) I[(size_t)i * n + i] = 1.0;
  for (int k = 0; k < n; ++k) {
    int piv = k;
    double best = std::abs(A[(size_t)k * n + k]);
    for (int i = k + 1; i < n; ++i) {
      double v = std::abs(A[(size_t)i * n + k]);
      if (v > best) { best = v; piv = i; }
    }
    if (best == 0.0) return false;
    if (piv != k) {
      for (int j = 0; j < n; ++j) {
        std::swap(A[(size_t)k * n + j], A[(size_t)piv * n + j]);
        std::swap(I[(size_t)k * n + j], I[(size_t)piv * n + j]);
      }
    }
    const std::complex<double> inv = 1.0 / A[(size_t)k * n + k];
    for (int j = 0; j < n; ++j) {
      A[(size_t)k * n + j] *= inv;
      I[(size_t)k * n + j] *= inv;
    }
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      const std::complex<double> f = A[(size_t)i * n + k];
      if (f == 0.0) continue;
      std::complex<double> *ai = &A[(size_t)i * n], *ak = &A[(size_t)k * n];
      std::complex<double> *ii = &I[(size_t)i * n], *ik = &I[(size_t)k * n];
      for (int j = 0; j < n; ++j) {
        ai[j] -= f * ak[j];
        ii[j] -= f * ik[j];
      }
    }
  }
  inv.swap(I);
  return true;
}

Grid make_grid(int D, const int n[3]) {
  Grid G;
  G.n[0] = n[0];
  G.n[1] = n[1];
  G.n[2] = D == 3 ? n[2] : 1;
  G.N = G.n[0] * G.n[1] * G.n[2];
  G.r0 = 1.0 / G.n[0];
  G.r01 = 1.0 / ((double)G.n[0] * G.n[1]);
  return G;
}
Grid coarsen(int D, const Grid &G) {
  int n[3] = {(G.n[0] - 1) / 2 + 1, (G.n[1] - 1) / 2 + 1, D == 3 ? (G.n[2] - 1) / 2 + 1 : 1};
  return make_grid(D, n);
}

template <typename T>
LevelT<T> *levels_of(adr_ctx *ctx);
template <>
LevelT<double> *levels_of<double>(adr_ctx *ctx) { return ctx->lv64; }
template <>
LevelT<float> *levels_of<float>(adr_ctx *ctx) { return ctx->lv32; }

template <typename T>
FineCoef<T> fine_coef(adr_ctx *ctx);
template <>
FineCoef<double> fine_coef<double>(adr_ctx *ctx) {
  return FineCoef<double>{{ctx->g64[0], ctx->g64[1], ctx->g64[2]}, ctx->L64, ctx->c64};
}
template <>
FineCoef<float> fine_coef<float>(adr_ctx *ctx) {
  return FineCoef<float>{{ctx->g32[0], ctx->g32[1], ctx->g32[2]}, ctx->L32, ctx->c32};
}

// Coefficients of the operator the multigrid cycle works on: A_beta's, with the reaction
// plane of the shifted operator when shift_alpha > 0 (in mixed mode the FP32 copy was
// made from that plane).  The outer FGMRES matvec always uses fine_coef<double>.
template <typename T>
FineCoef<T> prec_coef(adr_ctx *ctx);
template <>
FineCoef<double> prec_coef<double>(adr_ctx *ctx) {
  FineCoef<double> C = fine_coef<double>(ctx);
  if (ctx->cM64) C.c = ctx->cM64;
  return C;
}
template <>
FineCoef<float> prec_coef<float>(adr_ctx *ctx) { return fine_coef<float>(ctx); }

// exp(i w tau) in the cycle's precision (rescaled cycles only).
template <typename T>
const cx<T> *phase_of(adr_ctx *ctx);
template <>
const cx<double> *phase_of<double>(adr_ctx *ctx) { return ctx->ph64; }
template <>
const cx<float> *phase_of<float>(adr_ctx *ctx) { return ctx->ph32; }

FineParams fine_params(adr_ctx *ctx, double beta) {
  FineParams P;
  P.h = ctx->h;
  P.omega = ctx->omega;
  P.beta = beta;
  for (int k = 0; k < 3; ++k) P.src[k] = ctx->src[k];
  P.central = ctx->opt.advection == ADR_ADV_CENTRAL ? 1 : 0;
  return P;
}

double *lscal(adr_ctx *ctx, int l) { return ctx->scal + (size_t)l * kScalPerLevel; }

// Direction-dependent operators: the forward hierarchy of A_beta, or its conjugate
// transpose for adjoint solves (the Galerkin product commutes with ^H since P is real:
// (P^T A P)^H = P^T A^H P).
template <typename T>
const cx<T> *lvl_planes(const adr_ctx *ctx, const LevelT<T> &L) { return ctx->adj ? L.planes_adj : L.planes; }
template <typename T>
const cx<T> *lvl_planes_t(const adr_ctx *ctx, const LevelT<T> &L) { return ctx->adj ? L.planes_adj_t : L.planes_t; }
template <typename T>
const cx<T> *lvl_dinv(const adr_ctx *ctx, const LevelT<T> &L) { return ctx->adj ? L.dinv_adj : L.dinv; }

// Timed-launch brackets: tbegin returns an event slot (or -1 when this launch is not the
// timed class), tend records the closing event and the launch's algorithmic bytes.
int tbegin(adr_ctx *ctx, int kind, int level) {
  auto &T = ctx->timer;
  if (T.kind != kind || (T.level >= 0 && T.level != level)) return -1;
  if (T.used + 2 > (int)T.ev.size()) return -1;   // pool exhausted: stop timing
  // A failed record surfaces in adr_timer_stop, which reads every event pair.
  (void)hipEventRecord(T.ev[T.used], ctx->stream);
  return T.used;
}
void tend(adr_ctx *ctx, int slot, double bytes) {
  if (slot < 0) return;
  auto &T = ctx->timer;
  (void)hipEventRecord(T.ev[slot + 1], ctx->stream);
  T.used = slot + 2;
  T.launches += 1;
  T.bytes += bytes;
}
// Per-node coefficient bytes of the matrix-free fine operator: D gradient planes, L, c.
template <typename T>
double fine_coef_bytes(int D) { return (double)(D + 3) * sizeof(T); }

// Allocate the per-level vectors and convert/store the stencil in precision T.
// Coarse levels relaxed by the pipelined GMRES steps: those with at most
// pipeline_max_nodes nodes that relax by GMRES.
bool pipelined_level(const adr_ctx *ctx, int l, size_t N) {
  return ctx->opt.pipeline_max_nodes > 0 && l >= 1 && l < ctx->levels - 1 && N <= (size_t)ctx->opt.pipeline_max_nodes &&
         ctx->relax[l] == ADR_RELAX_GMRES && ctx->nu[l] >= 1 && ctx->nu[l] <= 8;
}

// The finest level relaxes by GMRES (Sec. 4.2) instead of damped Jacobi.
bool fine_gmres(const adr_ctx *ctx) { return ctx->levels > 1 && ctx->relax[0] == ADR_RELAX_GMRES; }

// Merged shot group: the per-problem grids of the launches that follow (kind on level l;
// `l2` >= 0 adds the full table of level l2 as the transfers' coarse grids).  No-op outside
// a merged group's launches.
// The launching problem's pointers are the base, so the tables are offset to its slot
// (the launches' slot lists hold slots relative to it).
void use_grids(adr_ctx *ctx, int kind, int l, int l2 = -1) {
  if (!ctx->mg || adrk::g_shot.count <= 1) return;
  adrk::g_shot.sh.grid = ctx->mg->table(kind, l) + ctx->mg_slot;
  adrk::g_shot.sh.grid2 = l2 >= 0 ? ctx->mg->table(kFullGrids, l2) + ctx->mg_slot : nullptr;
}

template <typename T>
adr_status alloc_level_vectors(adr_ctx *ctx, LevelT<T> &L, int l) {
  const size_t N = L.G.N;
  ADR_TRY(dalloc(ctx, &L.x, N));
  ADR_TRY(dalloc(ctx, &L.xt, N));
  ADR_TRY(dalloc(ctx, &L.b, N));
  ADR_TRY(dalloc(ctx, &L.r, N));
  if (l == 0 && fine_gmres(ctx)) {
    ADR_TRY(dalloc(ctx, &L.w, N));
    ADR_TRY(dalloc(ctx, &L.V, N * (kMaxNu + 1)));
    ADR_TRY(dalloc(ctx, &L.Z, N * (kMaxNu + 1)));
    ADR_TRY(dalloc(ctx, &L.dinv, N));
    adrk::fine_dinv<T>(ctx->stream, L.G, ctx->D, prec_coef<double>(ctx), fine_params(ctx, ctx->opt.beta), L.dinv);
  }
  if (l > 0) {
    ADR_TRY(dalloc(ctx, &L.w, N));
    ADR_TRY(dalloc(ctx, &L.V, N * (kMaxNu + 1)));
    ADR_TRY(dalloc(ctx, &L.Z, N * (kMaxNu + 1)));
    if (ctx->opt.cycle == ADR_CYCLE_K && l < ctx->levels - 1) {
      ADR_TRY(dalloc(ctx, &L.ku, N));
      ADR_TRY(dalloc(ctx, &L.kz, N));
    }
    if (pipelined_level(ctx, l, N)) {
      ADR_TRY(dalloc(ctx, &L.Gs, N * kMaxNu));
      ADR_TRY(dalloc(ctx, &L.Yp, N * 2));
    }
  }
  return ADR_OK;
}

// ------------------------------------------------------------------------------------
// Relaxation, V-cycle
// ------------------------------------------------------------------------------------
template <typename T>
VecSet<T> vecset(std::initializer_list<const cx<T> *> v) {
  VecSet<T> s{};
  s.count = 0;
  for (auto p : v) s.v[s.count++] = p;
  return s;
}

// GMRES relaxation on level l >= 1 (Sec. 4.2): x_out = x0 + D^{-1} V y, y the
// least-squares minimizer over the Krylov space of A D^{-1} and b - A x0.  The basis V is
// kept unnormalized with scale factors s_j on the device, and Z_j = D^{-1} V_j is written
// next to it so the stencil apply gathers a single vector.  Every reduction is summed in
// the prologue of the kernel that consumes it (see reduce_partials), so one step is two
// launches: the stencil apply with the dots, then the orthogonalization with the norm.
// From a zero guess, `bpin` (if set) holds the partials of ||b||^2 in part[0] with
// Z_0 = D^{-1} b already written (the restriction fuses both), and `r_out` (if set)
// receives the new residual b - A x_out from the Arnoldi relation (no extra apply).
template <typename T>
void gmres_relax(adr_ctx *ctx, int l, const cx<T> *x0, const cx<T> *b, cx<T> *x_out, ProIn bpin = ProIn{},
                 cx<T> *r_out = nullptr) {
  LevelT<T> &L = levels_of<T>(ctx)[l];
  hipStream_t s = ctx->stream;
  const int N = L.G.N, nu = ctx->nu[l], D = ctx->D;
  const double cb = sizeof(cx<T>);
  double *sc = lscal(ctx, l);
  use_grids(ctx, kRelaxGrids, l);
  const cx<T> *Vp[kMaxNu + 1];
  cx<T> *Zp[kMaxNu + 1];
  for (int j = 0; j <= nu; ++j) {
    Vp[j] = L.V + (size_t)j * N;
    Zp[j] = L.Z + (size_t)j * N;
  }
  const cx<T> *planes = lvl_planes(ctx, L), *dinv = lvl_dinv(ctx, L);
  // The operator: stored Galerkin planes on coarse levels, rows recomputed from the
  // coefficient planes on the finest (its bytes per node: planes or coefficients).
  const double opb = l == 0 ? fine_coef_bytes<T>(D) : cb * L.S;
  auto level_apply = [&](const CoarseArgs<T> &a, const VecSet<T> *dots, bool want_norm) {
    if (l == 0)
      return adrk::fine_gapply<T>(s, D, prec_coef<T>(ctx), fine_params(ctx, ctx->opt.beta), a, dots, want_norm,
                                  ctx->Pdev + 1);
    return adrk::coarse_apply<T>(s, D, a, dots, want_norm);
  };
  int cur = 0, nb;
  if (!x0) {
    Vp[0] = b;
    if (bpin.partials == ctx->part[cur]) nb = bpin.nb;
    else nb = adrk::norm2<T>(s, N, b, dinv, Zp[0], ctx->part[cur]);
  } else {
    // V0 = b - A x0, Z0 = D^{-1} V0, with the norm partials.
    CoarseArgs<T> a{};
    a.split = L.split;
    a.slabs = L.slabs;
    a.G = L.G;
    a.planes = planes;
    a.planes_t = lvl_planes_t(ctx, L);
    a.x = x0;
    a.b = b;
    a.y = L.V;
    a.dinv = dinv;
    a.zout = Zp[0];
    a.mode = 1;
    a.pout = ctx->part[cur];
    int t0 = tbegin(ctx, l == 0 ? ADR_TIMER_FINE_GMRES : ADR_TIMER_COARSE_APPLY, l);
    nb = level_apply(a, nullptr, true);
    tend(ctx, t0, (double)N * (opb + cb * 5));
  }
  if (L.Gs) {
    // Pipelined steps: the first apply, nu - 1 fused orthogonalization + apply steps and
    // the last orthogonalization (see k_pipe_step).
    cx<T> *Gp[kMaxNu], *Yb[2] = {L.Yp, L.Yp + N};
    for (int i = 0; i < nu; ++i) Gp[i] = L.Gs + (size_t)i * N;
    {
      VecSet<T> V0{};
      V0.count = 1;
      V0.v[0] = Vp[0];
      CoarseArgs<T> a{};
      a.split = L.split;
      a.slabs = L.slabs;
      a.G = L.G;
      a.planes = planes;
      a.planes_t = lvl_planes_t(ctx, L);
      a.x = Zp[0];
      a.pin = ProIn{ctx->part[cur], nb, 1};
      a.norm_out = sc + kBeta;
      a.norm_cplx = 0;
      a.inv_out = sc + kS + 0;
      a.y = Gp[0];
      a.dinv = dinv;
      a.zout = Yb[0];
      a.mode = 0;
      a.pout = ctx->part[cur ^ 1];
      int t0 = tbegin(ctx, ADR_TIMER_COARSE_APPLY, l);
      nb = adrk::coarse_apply<T>(s, D, a, &V0, false);
      tend(ctx, t0, (double)N * cb * (L.S + 4));
      cur ^= 1;
    }
    for (int k = 1; k <= nu; ++k) {
      VecSet<T> U{}, Gv{};
      U.count = k;
      Gv.count = k;
      for (int i = 0; i < k; ++i) {
        U.v[i] = Vp[i];
        Gv.v[i] = Gp[i];
      }
      double *hcol = sc + kH + 2 * ((k - 1) * kLdH);
      double *hsub = k >= 2 ? sc + kH + 2 * ((k - 2) * kLdH + (k - 1)) : nullptr;
      double *sout = k >= 2 ? sc + kS + (k - 1) : nullptr;
      const ProIn pin{ctx->part[cur], nb, 2 * k + (k >= 2 ? 1 : 0)};
      if (k < nu) {
        int t0 = tbegin(ctx, ADR_TIMER_COARSE_APPLY, l);
        nb = adrk::pipe_step<T>(s, D, L.split, L.slabs, L.G, planes, lvl_planes_t(ctx, L), Yb[(k - 1) & 1], pin,
                                sc + kS, hcol, hsub, sout, U, Gv, dinv, L.V + (size_t)k * N, Zp[k], Gp[k],
                                Yb[k & 1], ctx->part[cur ^ 1]);
        // planes, the gathered D^{-1} Gs_{k-1}, U and Gs (k each), dinv; u, z, G, D^{-1} G written
        tend(ctx, t0, (double)N * cb * (L.S + 6 + 2 * k));
      } else {
        int t1 = tbegin(ctx, ADR_TIMER_COARSE_ORTH, l);
        nb = adrk::pipe_final<T>(s, N, pin, sc + kS, hcol, hsub, sout, U, Gv, L.V + (size_t)k * N,
                                 ctx->part[cur ^ 1]);
        tend(ctx, t1, (double)N * cb * (2 + k));
      }
      cur ^= 1;
    }
  } else
  for (int j = 0; j < nu; ++j) {
    VecSet<T> Vs{};
    Vs.count = j + 1;
    for (int i = 0; i <= j; ++i) Vs.v[i] = Vp[i];
    double *hcol = sc + kH + 2 * (j * kLdH);
    // w = A Z_j s_j, with s_j = 1/||V_j|| from the previous kernel's partials.
    CoarseArgs<T> a{};
    a.split = L.split;
    a.slabs = L.slabs;
    a.G = L.G;
    a.planes = planes;
    a.planes_t = lvl_planes_t(ctx, L);
    a.x = Zp[j];
    a.pin = ProIn{ctx->part[cur], nb, 1};
    a.norm_out = (j == 0) ? sc + kBeta : sc + kH + 2 * ((j - 1) * kLdH + j);
    a.norm_cplx = (j == 0) ? 0 : 1;
    a.inv_out = sc + kS + j;
    a.y = L.w;
    a.mode = 0;
    a.pout = ctx->part[cur ^ 1];
    int t0 = tbegin(ctx, l == 0 ? ADR_TIMER_FINE_GMRES : ADR_TIMER_COARSE_APPLY, l);
    nb = level_apply(a, &Vs, false);
    tend(ctx, t0, (double)N * (opb + cb * (2 + (j + 1))));
    cur ^= 1;
    int t1 = tbegin(ctx, ADR_TIMER_COARSE_ORTH, l);
    nb = adrk::orth_step<T>(s, N, L.w, Vs, ProIn{ctx->part[cur], nb, 2 * (j + 1)}, sc + kS, hcol, dinv,
                            L.V + (size_t)(j + 1) * N, Zp[j + 1], ctx->part[cur ^ 1]);
    tend(ctx, t1, (double)N * cb * (j + 5));
    cur ^= 1;
  }
  VecSet<T> Zs{};
  Zs.count = nu;
  for (int i = 0; i < nu; ++i) Zs.v[i] = Zp[i];
  VecSet<T> Vr{};
  Vr.count = nu + 1;
  for (int i = 0; i <= nu; ++i) Vr.v[i] = Vp[i];
  int t2 = tbegin(ctx, ADR_TIMER_COARSE_ORTH, l);
  adrk::gmres_update<T>(s, N, x0, Zs, ProIn{ctx->part[cur], nb, 1}, sc + kH, kLdH, sc + kBeta, sc + kS, x_out,
                        r_out ? &Vr : nullptr, r_out);
  tend(ctx, t2, (double)N * cb * (nu + (x0 ? 2 : 1) + (r_out ? nu + 2 : 0)));
}

// Jacobi sweeps on the matrix-free level 0: sweep k writes `first` for even k and
// `second` for odd k, reading the previous result (x_start for k = 0, NULL = zero).
// Returns the buffer written last.
template <typename T>
cx<T> *jacobi_sweeps(adr_ctx *ctx, int nu, const cx<T> *x_start, const cx<T> *b, cx<T> *first, cx<T> *second) {
  const Grid &G = levels_of<T>(ctx)[0].G;
  FineCoef<T> C = prec_coef<T>(ctx);
  FineParams P = fine_params(ctx, ctx->opt.beta);
  const cx<T> *in = x_start;
  cx<T> *out = first;
  for (int k = 0; k < nu; ++k) {
    out = (k % 2 == 0) ? first : second;
    int t0 = tbegin(ctx, ADR_TIMER_FINE_JACOBI, 0);
    if (ctx->adj) adrk::fine_jacobi_adj<T>(ctx->stream, G, ctx->D, C, P, in, b, out, ctx->opt.jacobi_weight);
    else if (ctx->ph64)
      adrk::fine_jacobi_ph<T>(ctx->stream, G, ctx->D, C, P, phase_of<T>(ctx), in, b, out, ctx->opt.jacobi_weight);
    else if (!(ctx->fine_tiles_on && in &&
               adrk::fine_lds<T>(ctx->stream, G, ctx->D, C, P, in, b, out, 0, ctx->opt.jacobi_weight, ctx->Pdev + 1)))
      adrk::fine_jacobi<T>(ctx->stream, G, ctx->D, C, P, in, b, out, ctx->opt.jacobi_weight, ctx->Pdev + 1);
    tend(ctx, t0, (double)G.N * (fine_coef_bytes<T>(ctx->D) + sizeof(cx<T>) * (in ? 3 : 2)));
    in = out;
  }
  return out;
}

template <typename T>
cx<T> *coarse_fgmres2(adr_ctx *ctx, int k, ProIn bpin);

// One cycle on level l from a zero guess; b is the level right-hand side.  Returns the
// buffer holding x_l; `out0` (if not NULL) is the preferred output buffer.  The coarse
// problem is solved by the same cycle one level down (V-cycle, Alg. TwoCycle applied
// recursively), or, for the Krylov cycle (Alg. KrylovCycle), by flexible GMRES(2)
// preconditioned by it unless the coarse level is the coarsest.
// `bpin`: see gmres_relax (the restriction into b already produced D^{-1} b and the
// partials of ||b||^2).
template <typename T>
cx<T> *vcycle(adr_ctx *ctx, int l, const cx<T> *b, cx<T> *out0, ProIn bpin = ProIn{}) {
  LevelT<T> *lv = levels_of<T>(ctx);
  LevelT<T> &L = lv[l];
  hipStream_t s = ctx->stream;
  const int D = ctx->D;
  if (l == ctx->levels - 1) {
    cx<T> *x = out0 ? out0 : L.x;
    use_grids(ctx, kCoarsestGrids, l);
    adrk::dense_gemv<T>(s, L.G.N, ctx->adj ? ctx->Ainv_adj : ctx->Ainv, b, x);
    return x;
  }
  if (l == ctx->tail_level && b == L.b && (!out0 || out0 == L.x)) {
    // The rest of the cycle in one workgroup (levels l.. and the coarsest solve).
    int t0 = tbegin(ctx, ADR_TIMER_COARSE_TAIL, l);
    adrk::coarse_tail<T>(s, D, (const TailArgs<T> *)ctx->tail_args[ctx->adj ? 1 : 0]);
    tend(ctx, t0, 0.0);
    return L.x;
  }
  cx<T> *xa = out0 ? out0 : L.x;
  cx<T> *x;
  // Pre-relaxation.  Level 0 relaxes by damped Jacobi (the first sweep writes the
  // scratch buffer, so that the post-relaxation, which alternates from the pre-relaxed
  // iterate, ends in xa) and computes its residual with one more matrix-free apply; the
  // coarse levels' GMRES pre-relaxation also returns the residual in L.r.
  // (check_levels enforces this split.)
  const bool jacobi = l == 0 && !fine_gmres(ctx);
  if (jacobi) {
    use_grids(ctx, kRelaxGrids, 0);
    x = jacobi_sweeps<T>(ctx, ctx->nu[l], nullptr, b, L.xt, xa);
  } else {
    gmres_relax<T>(ctx, l, nullptr, b, xa, bpin, L.r);
    x = xa;
  }
  LevelT<T> &C = lv[l + 1];
  const double cb = sizeof(cx<T>);
  if (jacobi) {
    int t0 = tbegin(ctx, ADR_TIMER_FINE_RESIDUAL, 0);
    if (ctx->adj)
      adrk::fine_apply_adj<T, T, T>(s, L.G, D, prec_coef<T>(ctx), fine_params(ctx, ctx->opt.beta), x, b, L.r, 1,
                                    nullptr, false, nullptr);
    else if (ctx->ph64)
      adrk::fine_residual_ph<T>(s, L.G, D, prec_coef<T>(ctx), fine_params(ctx, ctx->opt.beta), phase_of<T>(ctx), x,
                                b, L.r);
    else if (!(ctx->fine_tiles_on && adrk::fine_lds<T>(s, L.G, D, prec_coef<T>(ctx), fine_params(ctx, ctx->opt.beta),
                                                          x, b, L.r, 1, 0.0, ctx->Pdev + 1)))
      adrk::fine_apply<T, T, T>(s, L.G, D, prec_coef<T>(ctx), fine_params(ctx, ctx->opt.beta), x, b, L.r, 1,
                                nullptr, false, nullptr, ctx->Pdev + 1);
    tend(ctx, t0, (double)L.G.N * (fine_coef_bytes<T>(D) + 3 * cb));
  }
  // The coarse level (unless it is the coarsest) starts with a GMRES relaxation from
  // zero: the restriction also writes its D^{-1} b and the partials of ||b||^2.
  const bool coarse_relaxes = l + 1 < ctx->levels - 1 && l + 1 != ctx->tail_level;
  use_grids(ctx, kRelaxGrids, l, l + 1);
  int t1 = tbegin(ctx, ADR_TIMER_TRANSFER, l);
  int rnb = adrk::restrict_full<T>(s, L.G, C.G, D, L.r, C.b, coarse_relaxes ? lvl_dinv(ctx, C) : nullptr,
                                   coarse_relaxes ? C.Z : nullptr, coarse_relaxes ? ctx->part[0] : nullptr);
  tend(ctx, t1, cb * ((double)L.G.N + C.G.N * (coarse_relaxes ? 3.0 : 1.0)));
  const ProIn cpin = coarse_relaxes ? ProIn{ctx->part[0], rnb, 1} : ProIn{};
  const bool krylov = ctx->opt.cycle == ADR_CYCLE_K && coarse_relaxes &&
                      (ctx->opt.kcycle_levels <= 0 || l + 1 <= ctx->opt.kcycle_levels);
  cx<T> *ec = krylov ? coarse_fgmres2<T>(ctx, l + 1, cpin)
                                                                : vcycle<T>(ctx, l + 1, C.b, nullptr, cpin);
  if (ctx->mg && adrk::g_shot.count > 1 && l + 1 < ctx->levels - 1 && ctx->mg->coarsest_at(l + 1)) {
    // Merged group: the problems whose coarsest level is l + 1 solve it here, into the
    // buffer the prolongation reads (the launches on level l + 1 skipped them).
    use_grids(ctx, kCoarsestGrids, l + 1);
    adrk::dense_gemv<T>(s, C.G.N, ctx->adj ? ctx->Ainv_adj : ctx->Ainv, C.b, ec);
  }
  use_grids(ctx, kRelaxGrids, l, l + 1);
  int t2 = tbegin(ctx, ADR_TIMER_TRANSFER, l);
  adrk::prolong_add<T>(s, L.G, C.G, D, ec, x);
  tend(ctx, t2, cb * ((double)C.G.N + 2.0 * L.G.N));
  // post-relaxation
  if (jacobi) {
    use_grids(ctx, kRelaxGrids, 0);
    cx<T> *other = (x == xa) ? L.xt : xa;
    return jacobi_sweeps<T>(ctx, ctx->nu[l], x, b, other, x);
  }
  gmres_relax<T>(ctx, l, x, b, x);
  return x;
}

// Flexible GMRES(2) from zero on A_k e = u_0 (u_0 = the restricted residual in level k's
// b), preconditioned by the cycle on level k (Alg. KrylovCycle).  The basis is kept
// unnormalized: u_1 = A z_0 - H00 v_0 with v_j = s_j u_j, s_j = 1/||u_j||; since the
// cycle is homogeneous, K(v_j) = s_j K(u_j), so the directions Z_j = K(u_j) enter with
// the factors s_j.  Both steps always run; the threshold (one-step residual <= t ||u_0||)
// only selects the one-column solution, which is what stopping after one step gives.
// Returns level k's w, which holds e.
template <typename T>
cx<T> *coarse_fgmres2(adr_ctx *ctx, int k, ProIn bpin) {
  LevelT<T> &L = levels_of<T>(ctx)[k];
  hipStream_t s = ctx->stream;
  const int N = L.G.N, D = ctx->D;
  const double cb = sizeof(cx<T>);
  double *sc = lscal(ctx, k);
  double *KH = sc + kKH, *KS = sc + kKS, *KB = sc + kKBeta;
  const cx<T> *planes = lvl_planes(ctx, L);
  // beta = ||u_0||, s_0 (the restriction into u_0 left the partials in part[0] and
  // D^{-1} u_0 in Z, which the first cycle's relaxation consumes as well)
  use_grids(ctx, kRelaxGrids, k);
  adrk::reduce_norm(s, bpin, KB, 0, KS + 0);
  // Z_0 = K(u_0)
  vcycle<T>(ctx, k, L.b, L.kz, bpin);
  use_grids(ctx, kRelaxGrids, k);
  int nb;
  // w = s_0 A Z_0 with the dot against u_0; u_1 = w - H00 s_0 u_0 and its norm
  VecSet<T> V1 = vecset<T>({L.b});
  CoarseArgs<T> a{};
  a.split = L.split;
  a.slabs = L.slabs;
  a.G = L.G;
  a.planes = planes;
  a.planes_t = lvl_planes_t(ctx, L);
  a.x = L.kz;
  a.sdev = KS + 0;
  a.y = L.w;
  a.mode = 0;
  a.pout = ctx->part[0];
  int t0 = tbegin(ctx, ADR_TIMER_COARSE_APPLY, k);
  nb = adrk::coarse_apply<T>(s, D, a, &V1, false);
  tend(ctx, t0, (double)N * cb * (L.S + 3));
  int t1 = tbegin(ctx, ADR_TIMER_COARSE_ORTH, k);
  nb = adrk::orth_step<T>(s, N, L.w, V1, ProIn{ctx->part[0], nb, 2}, KS, KH + 0, nullptr, L.ku, nullptr,
                          ctx->part[1]);
  tend(ctx, t1, (double)N * cb * 3);
  adrk::reduce_norm(s, ProIn{ctx->part[1], nb, 1}, KH + 2 * 1, 1, KS + 1);
  // Z_1 = K(u_1)
  cx<T> *z1 = vcycle<T>(ctx, k, L.ku, L.x);
  use_grids(ctx, kRelaxGrids, k);
  // w = s_1 A Z_1 with dots against u_0, u_1; u_2 (into r) only for its norm H21
  VecSet<T> V2 = vecset<T>({L.b, L.ku});
  a.x = z1;
  a.sdev = KS + 1;
  int t2 = tbegin(ctx, ADR_TIMER_COARSE_APPLY, k);
  nb = adrk::coarse_apply<T>(s, D, a, &V2, false);
  tend(ctx, t2, (double)N * cb * (L.S + 4));
  int t3 = tbegin(ctx, ADR_TIMER_COARSE_ORTH, k);
  nb = adrk::orth_step<T>(s, N, L.w, V2, ProIn{ctx->part[0], nb, 4}, KS, KH + 2 * 3, nullptr, L.r, nullptr,
                          ctx->part[1]);
  tend(ctx, t3, (double)N * cb * 4);
  int t4 = tbegin(ctx, ADR_TIMER_COARSE_ORTH, k);
  adrk::fgmres2_update<T>(s, N, L.kz, z1, ProIn{ctx->part[1], nb, 1}, KH, KB, KS, ctx->opt.kcycle_threshold, L.w);
  tend(ctx, t4, (double)N * cb * 3);
  return L.w;
}

adr_status check_levels(adr_ctx *ctx) {
  for (int l = 1; l < ctx->levels; ++l)
    if (ctx->relax[l] == ADR_RELAX_JACOBI) {
      ctx->err = "Jacobi relaxation is implemented on the finest level only";
      return ADR_ENOTSUP;
    }
  for (int l = 0; l < ctx->levels - 1; ++l)
    if (ctx->nu[l] < 1 || ctx->nu[l] > kMaxNu) {
      ctx->err = "nu must be in [1, 8]";
      return ADR_EINVAL;
    }
  if (ctx->levels > 1 && ctx->relax[0] == ADR_RELAX_GMRES && ctx->opt.rescaled) {
    ctx->err = "GMRES relaxation on the finest level of a rescaled cycle is not supported";
    return ADR_ENOTSUP;
  }
  return ADR_OK;
}

// ------------------------------------------------------------------------------------
// Setup
// ------------------------------------------------------------------------------------
adr_status validate(const adr_problem *p, const adr_options *o, std::string &err) {
  if (!p || !o) { err = "null problem or options"; return ADR_EINVAL; }
  if (p->ndim != 2 && p->ndim != 3) { err = "ndim must be 2 or 3"; return ADR_EINVAL; }
  for (int k = 0; k < p->ndim; ++k)
    if (p->n[k] < 5) { err = "every n[k] must be >= 5"; return ADR_EINVAL; }
  long long N = 1;
  for (int k = 0; k < p->ndim; ++k) N *= p->n[k];
  if (N > (1LL << 30)) { err = "grid too large (more than 2^30 nodes)"; return ADR_EINVAL; }
  if (!(p->h > 0) || !(p->omega > 0)) { err = "h and omega must be > 0"; return ADR_EINVAL; }
  if (!p->kappa2) { err = "kappa2 is required"; return ADR_EINVAL; }
  if (p->tau && p->src[0] >= 0) {
    for (int k = 0; k < p->ndim; ++k)
      if (p->src[k] < 2 || p->src[k] > p->n[k] - 3) {
        err = "source must be at least 2 nodes from every face";
        return ADR_EINVAL;
      }
  }
  if (o->restart < 1 || o->restart > kMaxRestart) { err = "restart must be in [1, 8]"; return ADR_EINVAL; }
  if (o->levels < 0 || o->levels > kMaxLevels) { err = "levels must be in [0, 8]"; return ADR_EINVAL; }
  if (o->prec != ADR_PREC_FP64 && o->prec != ADR_PREC_MIXED) { err = "bad precision"; return ADR_EINVAL; }
  if (!(o->beta >= 0.0 && o->beta <= 1.0)) { err = "beta must be in [0, 1]"; return ADR_EINVAL; }
  if (o->cycle != ADR_CYCLE_V && o->cycle != ADR_CYCLE_K) { err = "bad cycle"; return ADR_EINVAL; }
  if (o->tail_max_nodes < 0) {
    err = "tail_max_nodes must be >= 0";
    return ADR_EINVAL;
  }
  if (o->tail_max_nodes > 0) {
    // Switched off: its one GPU run with five 2D levels (tail on levels 1-3) ended in a
    // memory aperture violation whose cause has not been found.
    err = "the single-workgroup coarse tail is disabled (tail_max_nodes must be 0)";
    return ADR_ENOTSUP;
  }
  if (o->coarse_split != 0 && o->coarse_split != 1 && o->coarse_split != 4 && o->coarse_split != 8) {
    err = "coarse_split must be 0, 1, 4 or 8";
    return ADR_EINVAL;
  }
  if (!(o->kcycle_threshold >= 0.0)) { err = "kcycle_threshold must be >= 0"; return ADR_EINVAL; }
  if (o->kcycle_levels < 0) { err = "kcycle_levels must be >= 0"; return ADR_EINVAL; }
  if (o->fine_tiles < 0 || o->fine_tiles > 2) { err = "fine_tiles must be 0, 1 or 2"; return ADR_EINVAL; }
  if (o->batch_merge < 0 || o->batch_merge > 1) { err = "batch_merge must be 0 or 1"; return ADR_EINVAL; }
  if (o->pipeline_max_nodes < 0) { err = "pipeline_max_nodes must be >= 0"; return ADR_EINVAL; }
  if (o->advection != ADR_ADV_UPWIND && o->advection != ADR_ADV_CENTRAL) { err = "bad advection"; return ADR_EINVAL; }
  if (!(o->outer_beta >= 0.0 && o->outer_beta <= 1.0)) { err = "outer_beta must be in [0, 1]"; return ADR_EINVAL; }
  if (o->rescaled != 0 && o->rescaled != 1) { err = "rescaled must be 0 or 1"; return ADR_EINVAL; }
  if (o->reaction != ADR_REACTION_NUMERICAL && o->reaction != ADR_REACTION_EIKONAL) {
    err = "bad reaction";
    return ADR_EINVAL;
  }
  if (o->reaction == ADR_REACTION_EIKONAL && !p->tau) {
    err = "the eikonal reaction needs a travel time (tau = NULL is the Helmholtz operator)";
    return ADR_EINVAL;
  }
  if (!(o->shift_alpha >= 0.0 && o->shift_alpha < 1e300)) {
    err = "shift_alpha must be finite and >= 0";
    return ADR_EINVAL;
  }
  return ADR_OK;
}

int auto_levels(int D, const int n[3], int coarsest_max) {
  int m[3] = {n[0], n[1], D == 3 ? n[2] : 1};
  int levels = 1;
  while (levels < kMaxLevels) {
    long long N = (long long)m[0] * m[1] * m[2];
    if (N <= coarsest_max) break;
    bool ok = true;
    for (int k = 0; k < D; ++k) ok &= ((m[k] - 1) % 2 == 0) && ((m[k] - 1) / 2 + 1 >= 5);
    if (!ok) break;
    for (int k = 0; k < D; ++k) m[k] = (m[k] - 1) / 2 + 1;
    ++levels;
  }
  return levels;
}

// Galerkin-apply variant per coarse level (one lane per node, four wavefronts per 64
// nodes, or -- 3D levels with rows of at most 129 nodes -- LDS z-marching tiles):
// adr_options.coarse_split if set (8 falls back to one lane where the tiles do not
// apply), else a short timing on this level (mode 0 with one fused dot, as in the GMRES
// relaxation) in which a variant has to beat the best one before it by 10%, so that near
// ties do not flip from run to run.
// The choice is cached per grid shape and precision for the life of the process, so
// every context on a given shape launches the same kernels and sums in the same order.
// The tuner's table: per (ndim, nx, ny, nz, bytes per real) the variant and slab count
// chosen, and the timed milliseconds of the 8 launches.  Shared by every context of the
// process; adr_tuning_table_write/_read save it to and restore it from a text file.
struct TuneEntry {
  int split, slabs;
  float ms;
};
std::mutex g_tune_mu;
std::map<std::array<int, 5>, TuneEntry> g_tune;

template <typename T>
adr_status tune_split(adr_ctx *ctx, int l) {
  LevelT<T> &L = levels_of<T>(ctx)[l];
  const int max_slabs = adrk::lds_max_slabs(L.G, ctx->D);
  if (ctx->opt.coarse_split == 1 || ctx->opt.coarse_split == 4 || ctx->opt.coarse_split == 8) {
    L.split = (ctx->opt.coarse_split == 8 && max_slabs == 0) ? 1 : ctx->opt.coarse_split;
    L.slabs = 0;
    return ADR_OK;
  }
  const std::array<int, 5> key = {ctx->D, L.G.n[0], L.G.n[1], L.G.n[2], (int)sizeof(T)};
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      L.split = it->second.split;
      L.slabs = it->second.slabs;
      return ADR_OK;
    }
  }
  hipStream_t s = ctx->stream;
  const size_t N = L.G.N;
  ADR_HIP(hipMemsetAsync(L.x, 0, N * sizeof(cx<T>), s));
  ADR_HIP(hipMemsetAsync(L.r, 0, N * sizeof(cx<T>), s));
  hipEvent_t e0, e1;
  ADR_HIP(hipEventCreate(&e0));
  ADR_HIP(hipEventCreate(&e1));
  VecSet<T> V1 = vecset<T>({L.r});
  // Candidates: one lane, four wavefronts, and the LDS tiles at three slab counts.
  std::vector<std::pair<int, int>> cand = {{1, 0}, {4, 0}};
  if (max_slabs > 0) {
    for (int sl : {max_slabs, (3 * max_slabs + 3) / 4, (max_slabs + 1) / 2}) {
      bool dup = false;
      for (auto &c : cand) dup |= c.first == 8 && c.second == sl;
      if (!dup && sl >= 1) cand.push_back({8, sl});
    }
  }
  // Two rounds over the candidates, best round of each.  Small levels time 32 launches a
  // round: 8 launches of a few microseconds each are mostly timing noise.
  const int reps = N < (1u << 17) ? 32 : 8;
  std::vector<float> cand_ms(cand.size(), 1e30f);
  for (int round = 0; round < 2; ++round) {
    for (size_t ci = 0; ci < cand.size(); ++ci) {
      const int split = cand[ci].first, slabs = cand[ci].second;
      CoarseArgs<T> a{};
      a.split = split;
      a.slabs = slabs;
      a.G = L.G;
      a.planes = L.planes;
      a.planes_t = L.planes_t;
      a.x = L.x;
      a.y = L.w;
      a.mode = 0;
      a.pout = ctx->part[0];
      for (int w = 0; w < 2; ++w) adrk::coarse_apply<T>(s, ctx->D, a, &V1, false);
      hipError_t e = hipEventRecord(e0, s);
      for (int r = 0; r < reps; ++r) adrk::coarse_apply<T>(s, ctx->D, a, &V1, false);
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        ctx->err = std::string("split tuning: ") + hipGetErrorString(e);
        return ADR_EHIP;
      }
      cand_ms[ci] = std::min(cand_ms[ci], ms * 8.f / reps);   // the table keeps ms per 8 launches
    }
  }
  TuneEntry best{1, 0, 0.f};
  for (size_t ci = 0; ci < cand.size(); ++ci) {
    const int split = cand[ci].first, slabs = cand[ci].second;
    if (split == 1 || cand_ms[ci] < 0.90f * best.ms) best = TuneEntry{split, split == 8 ? slabs : 0, cand_ms[ci]};
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::lock_guard<std::mutex> g(g_tune_mu);
  auto ins = g_tune.emplace(key, best);
  L.split = ins.first->second.split;
  L.slabs = ins.first->second.slabs;
  return ADR_OK;
}

// Finest-level LDS tiles (fine_tiles = 1): where they apply, time Jacobi sweeps both ways
// (8 launches each, three rounds alternating the variants, best round of each) and keep
// the tiles if they are at least 1% faster.  Both variants do the same arithmetic, so the
// choice only affects speed (measured: 257^3 212 -> 201 us per sweep; 129^3 29 -> 35 us,
// slower).
template <typename T>
adr_status tune_fine_tiles(adr_ctx *ctx) {
  ctx->fine_tiles_on = false;
  LevelT<T> &L = levels_of<T>(ctx)[0];
  if (!ctx->opt.fine_tiles || sizeof(T) != 4 || adrk::fine_lds_blocks(L.G, ctx->D) == 0) return ADR_OK;
  if (ctx->opt.fine_tiles == 2) {
    ctx->fine_tiles_on = true;
    return ADR_OK;
  }
  hipStream_t s = ctx->stream;
  const size_t N = L.G.N;
  ADR_HIP(hipMemsetAsync(L.x, 0, N * sizeof(cx<T>), s));
  ADR_HIP(hipMemsetAsync(L.b, 0, N * sizeof(cx<T>), s));
  FineCoef<T> C = prec_coef<T>(ctx);
  FineParams P = fine_params(ctx, ctx->opt.beta);
  hipEvent_t e0, e1;
  ADR_HIP(hipEventCreate(&e0));
  ADR_HIP(hipEventCreate(&e1));
  float ms[2] = {1e30f, 1e30f};
  for (int round = 0; round < 6; ++round) {
    const int v = round & 1;
    // Sweeps alternate between two buffers, each reading the previous one's output, as in
    // the cycle.
    auto sweep = [&](int r) {
      cx<T> *in = (r & 1) ? L.xt : L.x, *out = (r & 1) ? L.x : L.xt;
      if (v == 1) adrk::fine_lds<T>(s, L.G, ctx->D, C, P, in, L.b, out, 0, ctx->opt.jacobi_weight, ctx->Pdev + 1);
      else adrk::fine_jacobi<T>(s, L.G, ctx->D, C, P, in, L.b, out, ctx->opt.jacobi_weight, ctx->Pdev + 1);
    };
    for (int w = 0; w < 2; ++w) sweep(w);
    hipError_t e = hipEventRecord(e0, s);
    for (int r = 0; r < 8; ++r) sweep(r);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e == hipSuccess && t < ms[v]) ms[v] = t;
    if (e != hipSuccess) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      ctx->err = std::string("fine tile tuning: ") + hipGetErrorString(e);
      return ADR_EHIP;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx->fine_tiles_on = ms[1] < 0.99f * ms[0];
  return ADR_OK;
}

// Level table of the coarse tail for the current direction (forward or adjoint), copied
// to the device.
template <typename T>
adr_status build_tail_args(adr_ctx *ctx, int dir) {
  if (ctx->tail_level < 0) return ADR_OK;
  LevelT<T> *lv = levels_of<T>(ctx);
  TailArgs<T> A{};
  A.first = ctx->tail_level;
  A.last = ctx->levels - 1;
  for (int l = A.first; l <= A.last; ++l) {
    TailLevel<T> &t = A.L[l];
    t.G = lv[l].G;
    t.planes = dir ? lv[l].planes_adj : lv[l].planes;
    t.dinv = dir ? lv[l].dinv_adj : lv[l].dinv;
    t.x = lv[l].x;
    t.b = lv[l].b;
    t.r = lv[l].r;
    t.w = lv[l].w;
    t.V = lv[l].V;
    t.Z = lv[l].Z;
    t.nu = ctx->nu[l];
  }
  A.Ainv = dir ? ctx->Ainv_adj : ctx->Ainv;
  if (!ctx->tail_args[dir]) ADR_TRY(dalloc(ctx, (TailArgs<T> **)&ctx->tail_args[dir], 1));
  ADR_HIP(hipMemcpy(ctx->tail_args[dir], &A, sizeof(A), hipMemcpyHostToDevice));
  return ADR_OK;
}

template <typename T>
adr_status build_hierarchy(adr_ctx *ctx) {
  hipStream_t s = ctx->stream;
  const int D = ctx->D;
  LevelT<T> *lv = levels_of<T>(ctx);
  lv[0].G = ctx->G0;
  lv[0].S = 0;
  for (int l = 1; l < ctx->levels; ++l) {
    lv[l].G = coarsen(D, lv[l - 1].G);
    for (int k = 0; k < D; ++k)
      if ((lv[l - 1].G.n[k] - 1) % 2) {
        ctx->err = "n-1 must be divisible by 2^(levels-1)";
        return ADR_EINVAL;
      }
  }
  // Offset tables and Galerkin triples.
  std::vector<int> fo = fine_offsets(D), co = coarse_offsets(D);
  ctx->h_off_coarse = co;
  ctx->S_coarse = (int)co.size() / 3;
  ADR_TRY(dalloc(ctx, &ctx->off_fine, fo.size()));
  ADR_TRY(dalloc(ctx, &ctx->off_coarse, co.size()));
  ADR_HIP(hipMemcpy(ctx->off_fine, fo.data(), fo.size() * sizeof(int), hipMemcpyHostToDevice));
  ADR_HIP(hipMemcpy(ctx->off_coarse, co.data(), co.size() * sizeof(int), hipMemcpyHostToDevice));
  Triples tf = galerkin_triples(D, fo, co), tc = galerkin_triples(D, co, co);
  int *tri_start[2], *tri_p[2], *tri_d[2];
  double *tri_w[2];
  Triples *tt[2] = {&tf, &tc};
  for (int i = 0; i < 2; ++i) {
    ADR_TRY(dalloc(ctx, &tri_start[i], tt[i]->start.size()));
    ADR_TRY(dalloc(ctx, &tri_p[i], tt[i]->p.size()));
    ADR_TRY(dalloc(ctx, &tri_d[i], tt[i]->d.size()));
    ADR_TRY(dalloc(ctx, &tri_w[i], tt[i]->w.size()));
    ADR_HIP(hipMemcpy(tri_start[i], tt[i]->start.data(), tt[i]->start.size() * sizeof(int), hipMemcpyHostToDevice));
    ADR_HIP(hipMemcpy(tri_p[i], tt[i]->p.data(), tt[i]->p.size() * sizeof(int), hipMemcpyHostToDevice));
    ADR_HIP(hipMemcpy(tri_d[i], tt[i]->d.data(), tt[i]->d.size() * sizeof(int), hipMemcpyHostToDevice));
    ADR_HIP(hipMemcpy(tri_w[i], tt[i]->w.data(), tt[i]->w.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  const int Sf = (int)fo.size() / 3, Sc = ctx->S_coarse;
  // FP64 planes: fine stencil of A_beta, then each Galerkin level.
  cx<double> *prev = nullptr;
  adr_status st = ADR_OK;
  if (ctx->levels > 1) {
    st = dalloc(ctx, &prev, (size_t)Sf * ctx->G0.N);
    if (st == ADR_OK) {
      FineCoef<double> C = prec_coef<double>(ctx);
      adrk::fine_stencil(s, ctx->G0, D, C, fine_params(ctx, ctx->opt.beta), prev);
      if (ctx->ph64) adrk::stencil_rescale(s, ctx->G0, D, prev, ctx->ph64);
    }
  }
  for (int l = 1; l < ctx->levels && st == ADR_OK; ++l) {
    cx<double> *cur = nullptr;
    st = dalloc(ctx, &cur, (size_t)Sc * lv[l].G.N);
    if (st != ADR_OK) break;
    const int which = (l == 1) ? 0 : 1;
    adrk::galerkin(s, lv[l - 1].G, lv[l].G, prev, l == 1 ? ctx->off_fine : ctx->off_coarse, l == 1 ? Sf : Sc, cur,
                   ctx->off_coarse, Sc, tri_start[which], tri_p[which], tri_d[which], tri_w[which]);
    // The FP64 planes are the level stencil in FP64 mode; mixed mode keeps an FP32 copy
    // and frees the FP64 planes once the next level is built from them.
    lv[l].S = Sc;
    if (l == 1 || ctx->opt.prec != ADR_PREC_FP64) dfree(ctx, prev);
    prev = cur;
    if (ctx->opt.prec == ADR_PREC_FP64) {
      lv[l].planes = (cx<T> *)cur;
    } else {
      cx<float> *p32 = nullptr;
      st = dalloc(ctx, &p32, (size_t)Sc * lv[l].G.N);
      if (st != ADR_OK) break;
      adrk::convert<float, double>(s, (long long)Sc * lv[l].G.N, cur, p32);
      lv[l].planes = (cx<T> *)p32;
    }
    st = dalloc(ctx, &lv[l].dinv, lv[l].G.N);
    if (st != ADR_OK) break;
    const int centre = (Sc - 1) / 2;
    adrk::stencil_diag_inv<T>(s, lv[l].G.N, lv[l].planes + (size_t)centre * lv[l].G.N, lv[l].dinv);
    // The LDS apply's segment-tiled copy of the planes, on the relaxed 3D levels where
    // that variant applies (released after tuning unless it is chosen).
    if (l < ctx->levels - 1) {
      const long long nt = adrk::tiled_plane_count(lv[l].G, D, Sc);
      if (nt > 0) {
        st = dalloc(ctx, &lv[l].planes_t, (size_t)nt);
        if (st != ADR_OK) break;
        adrk::tile_planes<T>(s, lv[l].G, Sc, lv[l].planes, lv[l].planes_t);
      }
    }
  }
  for (int i = 0; i < 2; ++i) {
    dfree(ctx, tri_start[i]);
    dfree(ctx, tri_p[i]);
    dfree(ctx, tri_d[i]);
    dfree(ctx, tri_w[i]);
  }
  if (st != ADR_OK) {
    // In FP64 mode `prev` is owned by a level (or is the fine temporary on level 1).
    if (ctx->opt.prec != ADR_PREC_FP64 || (prev && lv[1].planes != (cx<T> *)prev)) dfree(ctx, prev);
    return st;
  }
  // Coarsest: dense FP64 inverse.
  const int Lc = ctx->levels - 1;
  const Grid &Gc = lv[Lc].G;
  const int n = Gc.N;
  ctx->Ncoarsest = n;
  std::vector<std::complex<double>> A((size_t)n * n, 0.0), inv;
  if (Lc == 0) {
    // Single level: materialize the fine stencil of A_beta directly.
    cx<double> *tmp = nullptr;
    ADR_TRY(dalloc(ctx, &tmp, (size_t)Sf * n));
    adrk::fine_stencil(s, ctx->G0, D, prec_coef<double>(ctx), fine_params(ctx, ctx->opt.beta), tmp);
    if (ctx->ph64) adrk::stencil_rescale(s, ctx->G0, D, tmp, ctx->ph64);
    std::vector<cx<double>> hp((size_t)Sf * n);
    ADR_HIP(hipMemcpyAsync(hp.data(), tmp, hp.size() * sizeof(cx<double>), hipMemcpyDeviceToHost, s));
    ADR_HIP(hipStreamSynchronize(s));
    dfree(ctx, tmp);
    for (int i = 0; i < n; ++i) {
      int ix = i % Gc.n[0], iy = (i / Gc.n[0]) % Gc.n[1], iz = i / (Gc.n[0] * Gc.n[1]);
      for (int p = 0; p < Sf; ++p) {
        int jx = ix + fo[3 * p], jy = iy + fo[3 * p + 1], jz = iz + fo[3 * p + 2];
        if (jx < 0 || jx >= Gc.n[0] || jy < 0 || jy >= Gc.n[1] || jz < 0 || jz >= Gc.n[2]) continue;
        int j = jx + Gc.n[0] * (jy + Gc.n[1] * jz);
        A[(size_t)i * n + j] += std::complex<double>(hp[(size_t)p * n + i].re, hp[(size_t)p * n + i].im);
      }
    }
  } else {
    std::vector<cx<double>> hp((size_t)Sc * n);
    ADR_HIP(hipMemcpyAsync(hp.data(), prev, hp.size() * sizeof(cx<double>), hipMemcpyDeviceToHost, s));
    ADR_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < n; ++i) {
      int ix = i % Gc.n[0], iy = (i / Gc.n[0]) % Gc.n[1], iz = i / (Gc.n[0] * Gc.n[1]);
      for (int p = 0; p < Sc; ++p) {
        int jx = ix + co[3 * p], jy = iy + co[3 * p + 1], jz = iz + co[3 * p + 2];
        if (jx < 0 || jx >= Gc.n[0] || jy < 0 || jy >= Gc.n[1] || jz < 0 || jz >= Gc.n[2]) continue;
        int j = jx + Gc.n[0] * (jy + Gc.n[1] * jz);
        A[(size_t)i * n + j] = std::complex<double>(hp[(size_t)p * n + i].re, hp[(size_t)p * n + i].im);
      }
    }
    if (ctx->opt.prec != ADR_PREC_FP64) dfree(ctx, prev);
  }
  if (!dense_inverse(n, A, inv)) {
    ctx->err = "coarsest operator is singular";
    return ADR_ENUMERIC;
  }
  ADR_TRY(dalloc(ctx, &ctx->Ainv, (size_t)n * n));
  ADR_HIP(hipMemcpy(ctx->Ainv, inv.data(), inv.size() * sizeof(cx<double>), hipMemcpyHostToDevice));
  ctx->h_inv.swap(inv);
  for (int l = 0; l < ctx->levels; ++l) ADR_TRY(alloc_level_vectors<T>(ctx, lv[l], l));
  for (int l = 1; l < ctx->levels - 1; ++l) {
    ADR_TRY(tune_split<T>(ctx, l));
    if (lv[l].split != 8 && lv[l].planes_t) {
      dfree(ctx, lv[l].planes_t);
      lv[l].planes_t = nullptr;
    }
  }
  if (ctx->levels > 1) ADR_TRY(tune_fine_tiles<T>(ctx));
  // Coarse tail: from the first coarse level with at most tail_max_nodes nodes (V-cycle;
  // the Krylov cycle's coarse GMRES steps stay on the multi-kernel path).
  ctx->tail_level = -1;
  if (ctx->opt.cycle == ADR_CYCLE_V && ctx->opt.tail_max_nodes > 0)
    for (int l = 1; l < ctx->levels - 1; ++l)
      if (lv[l].G.N <= ctx->opt.tail_max_nodes) {
        ctx->tail_level = l;
        break;
      }
  ADR_TRY(build_tail_args<T>(ctx, 0));
  return ADR_OK;
}

void free_ctx(adr_ctx *ctx) {
  if (!ctx) return;
  auto F = [ctx](void *p) { dfree(ctx, p); };
  for (int k = 0; k < 3; ++k) {
    F(ctx->g64[k]);
    F(ctx->g32[k]);
  }
  F(ctx->L64);
  F(ctx->L32);
  F(ctx->c64);
  F(ctx->c32);
  F(ctx->cM64);
  F(ctx->ph64);
  F(ctx->ph32);
  F(ctx->vtmp);
  F(ctx->tau);
  F(ctx->gamma);
  F(ctx->Ainv_adj);
  for (int l = 0; l < kMaxLevels; ++l) {
    LevelT<double> &a = ctx->lv64[l];
    LevelT<float> &b = ctx->lv32[l];
    for (void *p : {(void *)a.planes, (void *)a.dinv, (void *)a.x, (void *)a.xt, (void *)a.b, (void *)a.r,
                    (void *)a.w, (void *)a.V, (void *)a.Z, (void *)a.ku, (void *)a.kz, (void *)a.Gs, (void *)a.Yp,
                    (void *)b.Gs, (void *)b.Yp, (void *)a.planes_adj,
                    (void *)a.dinv_adj, (void *)b.planes, (void *)b.dinv, (void *)b.x, (void *)b.xt, (void *)b.b,
                    (void *)b.r, (void *)b.w, (void *)b.V, (void *)b.Z, (void *)b.ku, (void *)b.kz,
                    (void *)b.planes_adj, (void *)b.dinv_adj, (void *)b.planes_t, (void *)b.planes_adj_t})
      F(p);
  }
  F(ctx->off_coarse);
  F(ctx->off_fine);
  F(ctx->Ainv);
  F(ctx->scal);
  F(ctx->osc);
  if (ctx->hpin) (void)hipHostFree(ctx->hpin);
  F(ctx->part[0]);
  F(ctx->part[1]);
  F(ctx->Vo);
  F(ctx->Zo);
  F(ctx->wo);
  F(ctx->ro);
  F(ctx->qh);
  F(ctx->b32);
  F(ctx->z32);
  F(ctx->tail_args[0]);
  F(ctx->tail_args[1]);
  F(ctx->Pdev);
  F(ctx->active);
  F(ctx->qin);
  F(ctx->xg);
  for (auto &e : ctx->timer.ev) (void)hipEventDestroy(e);
  for (auto &g : ctx->graphs) {
    (void)hipGraphExecDestroy(g.e);
    (void)hipGraphDestroy(g.g);
  }
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  delete ctx;
}

adr_status setup_impl(adr_ctx *ctx, const adr_problem *p) {
  hipStream_t s = ctx->stream;
  const int D = ctx->D;
  const int N = ctx->G0.N;
  for (int k = 0; k < D; ++k) ADR_TRY(dalloc(ctx, &ctx->g64[k], N));
  ADR_TRY(dalloc(ctx, &ctx->L64, N));
  ADR_TRY(dalloc(ctx, &ctx->c64, N));
  ADR_TRY(dalloc(ctx, &ctx->tau, N));
  if (p->tau)
    ADR_HIP(hipMemcpyAsync(ctx->tau, p->tau, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
  else
    ADR_HIP(hipMemsetAsync(ctx->tau, 0, sizeof(double) * N, s));
  if (p->gamma) {
    ADR_TRY(dalloc(ctx, &ctx->gamma, N));
    ADR_HIP(hipMemcpyAsync(ctx->gamma, p->gamma, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
  }
  adrk::coefficients(s, ctx->G0, D, ctx->h, ctx->omega, ctx->src, ctx->opt.reaction == ADR_REACTION_NUMERICAL,
                     p->kappa2, ctx->tau, p->gamma, ctx->g64[0], ctx->g64[1], D == 3 ? ctx->g64[2] : nullptr,
                     ctx->L64, ctx->c64);
  if (ctx->opt.shift_alpha > 0.0) {
    ADR_TRY(dalloc(ctx, &ctx->cM64, N));
    adrk::shift_reaction(s, N, ctx->c64, p->kappa2, ctx->opt.shift_alpha * ctx->omega * ctx->omega, ctx->cM64);
  }
  ADR_HIP(hipGetLastError());
  // Reduction scratch and scalars.
  for (int i = 0; i < 2; ++i) ADR_TRY(dalloc(ctx, &ctx->part[i], (size_t)ADR_PART_BLOCKS * ADR_MAX_RED));
  ADR_TRY(dalloc(ctx, &ctx->scal, (size_t)kMaxLevels * kScalPerLevel));
  ADR_HIP(hipMemsetAsync(ctx->scal, 0, sizeof(double) * kMaxLevels * kScalPerLevel, s));
  ADR_TRY(dalloc(ctx, &ctx->osc, 64));
  ADR_HIP(hipMemsetAsync(ctx->osc, 0, sizeof(double) * 64, s));
  ADR_HIP(hipHostMalloc((void **)&ctx->hpin, kPin * sizeof(double), hipHostMallocDefault));
  // Device copies of the fine-operator parameters (kernels of a shot group read their
  // own problem's omega and source there) and the shot-group flag.
  ADR_TRY(dalloc(ctx, &ctx->Pdev, 2));
  {
    const FineParams hpar[2] = {fine_params(ctx, ctx->opt.outer_beta), fine_params(ctx, ctx->opt.beta)};
    ADR_HIP(hipMemcpy(ctx->Pdev, hpar, sizeof(hpar), hipMemcpyHostToDevice));
  }
  ADR_TRY(dalloc(ctx, &ctx->active, 1));
  {
    const int one = 1;
    ADR_HIP(hipMemcpy(ctx->active, &one, sizeof(one), hipMemcpyHostToDevice));
  }
  if (ctx->group_member) {
    ADR_TRY(dalloc(ctx, &ctx->qin, N));
    ADR_TRY(dalloc(ctx, &ctx->xg, N));
  }
  if (ctx->opt.rescaled) {
    ADR_TRY(dalloc(ctx, &ctx->ph64, N));
    adrk::phase_plane(s, N, ctx->tau, ctx->omega, ctx->ph64);
    if (ctx->opt.prec == ADR_PREC_MIXED) {
      ADR_TRY(dalloc(ctx, &ctx->ph32, N));
      adrk::convert<float, double>(s, N, ctx->ph64, ctx->ph32);
    } else {
      ADR_TRY(dalloc(ctx, &ctx->vtmp, N));
    }
  }
  if (ctx->opt.prec == ADR_PREC_MIXED) {
    for (int k = 0; k < D; ++k) {
      ADR_TRY(dalloc(ctx, &ctx->g32[k], N));
      adrk::convert_real<float, double>(s, N, ctx->g64[k], ctx->g32[k]);
    }
    ADR_TRY(dalloc(ctx, &ctx->L32, N));
    adrk::convert_real<float, double>(s, N, ctx->L64, ctx->L32);
    ADR_TRY(dalloc(ctx, &ctx->c32, N));
    adrk::convert<float, double>(s, N, ctx->cM64 ? ctx->cM64 : ctx->c64, ctx->c32);
    ADR_TRY(build_hierarchy<float>(ctx));
    ADR_TRY(dalloc(ctx, &ctx->b32, N));
    ADR_TRY(dalloc(ctx, &ctx->z32, N));
  } else {
    ADR_TRY(build_hierarchy<double>(ctx));
  }
  // Outer FGMRES buffers.
  const int m = ctx->opt.restart;
  ADR_TRY(dalloc(ctx, &ctx->Vo, (size_t)(m + 1) * N));
  if (ctx->opt.prec == ADR_PREC_MIXED) {
    cx<float> *z = nullptr;
    ADR_TRY(dalloc(ctx, &z, (size_t)m * N));
    ctx->Zo = z;
  } else {
    cx<double> *z = nullptr;
    ADR_TRY(dalloc(ctx, &z, (size_t)m * N));
    ctx->Zo = z;
  }
  ADR_TRY(dalloc(ctx, &ctx->wo, N));
  ADR_TRY(dalloc(ctx, &ctx->ro, N));
  ADR_TRY(dalloc(ctx, &ctx->qh, N));
  ADR_HIP(hipGetLastError());
  ADR_HIP(hipStreamSynchronize(s));
  return ADR_OK;
}

// Enqueue one preconditioner application on ctx->stream: z = V-cycle(v).  v is c128;
// z is c64 (mixed, `z_is_c128` = 0) or c128.  In mixed mode the input is converted to
// c64 first (and the result back to c128 when z_is_c128).
void enqueue_vcycle(adr_ctx *ctx, const cx<double> *v, void *z, bool z_is_c128) {
  hipStream_t s = ctx->stream;
  const int N = ctx->G0.N;
  if (ctx->ph64) {
    // Rescaled cycle: z = M^{-1} K(M v) with M = diag(conj(ph)).
    if (ctx->opt.prec == ADR_PREC_MIXED) {
      adrk::mul_phase<double, float>(s, N, v, ctx->ph64, true, ctx->b32);
      if (z_is_c128) {
        vcycle<float>(ctx, 0, ctx->b32, ctx->z32);
        adrk::mul_phase<float, double>(s, N, ctx->z32, ctx->ph64, false, (cx<double> *)z);
      } else {
        cx<float> *zf = vcycle<float>(ctx, 0, ctx->b32, (cx<float> *)z);
        adrk::mul_phase<float, float>(s, N, zf, ctx->ph64, false, (cx<float> *)z);
      }
    } else {
      adrk::mul_phase<double, double>(s, N, v, ctx->ph64, true, ctx->vtmp);
      cx<double> *zd = vcycle<double>(ctx, 0, ctx->vtmp, (cx<double> *)z);
      adrk::mul_phase<double, double>(s, N, zd, ctx->ph64, false, (cx<double> *)z);
    }
    return;
  }
  if (ctx->opt.prec == ADR_PREC_MIXED) {
    use_grids(ctx, kFullGrids, 0);
    adrk::convert<float, double>(s, N, v, ctx->b32);
    if (z_is_c128) {
      vcycle<float>(ctx, 0, ctx->b32, ctx->z32);
      use_grids(ctx, kFullGrids, 0);
      adrk::convert<double, float>(s, N, ctx->z32, (cx<double> *)z);
    } else {
      vcycle<float>(ctx, 0, ctx->b32, (cx<float> *)z);
    }
  } else {
    vcycle<double>(ctx, 0, v, (cx<double> *)z);
  }
}

// Preconditioner application, replayed from a captured graph when enabled (the per-kernel
// timer needs eager launches, so it bypasses graphs).
adr_status precondition(adr_ctx *ctx, const cx<double> *v, void *z, bool z_is_c128) {
  if (!ctx->opt.use_graph || ctx->timer.kind >= 0) {
    enqueue_vcycle(ctx, v, z, z_is_c128);
    return ADR_OK;
  }
  adr_ctx::GraphEntry *hit = nullptr;
  for (auto &g : ctx->graphs)
    if (g.in == v && g.out == z && g.adj == ctx->adj && g.group == adrk::g_shot.count) hit = &g;
  if (!hit) {
    if (!ctx->cap_stream) ADR_HIP(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    // Up to 64 captures: a shot group's lead holds one per Arnoldi step and slot-list
    // bucket (5 steps x up to 7 buckets), which a smaller cache would evict and recapture
    // on every batch solve.
    if (ctx->graphs.size() >= 64) {   // evict the least recently used capture
      auto it = std::min_element(ctx->graphs.begin(), ctx->graphs.end(),
                                 [](const adr_ctx::GraphEntry &x, const adr_ctx::GraphEntry &y) {
                                   return x.last_use < y.last_use;
                                 });
      (void)hipGraphExecDestroy(it->e);
      (void)hipGraphDestroy(it->g);
      ctx->graphs.erase(it);
    }
    adr_ctx::GraphEntry ge;
    ge.in = v;
    ge.out = z;
    ge.adj = ctx->adj;
    ge.group = adrk::g_shot.count;
    hipStream_t user = ctx->stream;
    ctx->stream = ctx->cap_stream;
    hipError_t e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
      enqueue_vcycle(ctx, v, z, z_is_c128);
      e = hipStreamEndCapture(ctx->cap_stream, &ge.g);
    }
    ctx->stream = user;
    if (e != hipSuccess) {
      ctx->err = std::string("V-cycle graph capture failed: ") + hipGetErrorString(e);
      return ADR_EHIP;
    }
    ADR_HIP(hipGraphInstantiate(&ge.e, ge.g, nullptr, nullptr, 0));
    ctx->graphs.push_back(ge);
    hit = &ctx->graphs.back();
  }
  hit->last_use = ++ctx->graph_clock;
  ADR_HIP(hipGraphLaunch(hit->e, ctx->stream));
  return ADR_OK;
}

}  // namespace

extern "C" void adr_default_options(adr_options *o);

namespace {
// Context setup.  With `slot`, every device allocation of the setup is carved, in a fixed
// order, from [slot, slot + slot_cap) (one problem of a shot group); later allocations
// (adjoint preparation) use hipMalloc.  `group_member` adds the group's right-hand-side
// and solution buffers.
adr_status setup_ctx(const adr_problem *prob, const adr_options *opt, hipStream_t stream, char *slot,
                     size_t slot_cap, bool group_member, adr_ctx **out, const SlotLayout *layout = nullptr) {
  if (!out) {
    g_setup_error = "null output pointer";
    return ADR_EINVAL;
  }
  *out = nullptr;
  adr_options defaults;
  adr_default_options(&defaults);
  const adr_options *o = opt ? opt : &defaults;
  std::string err;
  adr_status st = validate(prob, o, err);
  if (st != ADR_OK) {
    g_setup_error = err;
    return st;
  }
  const double t0 = now_ms();
  adr_ctx *ctx = new adr_ctx();
  ctx->opt = *o;
  ctx->stream = stream;
  ctx->group_member = group_member;
  if (slot) {
    ctx->arena = slot;
    ctx->arena_cap = slot_cap;
    ctx->arena_lo = slot;
    ctx->arena_hi = slot + slot_cap;
    ctx->layout = layout;
  }
  ctx->D = prob->ndim;
  ctx->G0 = make_grid(ctx->D, prob->n);
  ctx->h = prob->h;
  ctx->omega = prob->omega;
  // Without tau (standard Helmholtz) there is no factoring and no near-source rule.
  const bool has_src = prob->tau && prob->src[0] >= 0;
  for (int k = 0; k < 3; ++k) ctx->src[k] = (has_src && k < ctx->D) ? prob->src[k] : 0;
  if (!has_src) ctx->src[0] = -1;
  ctx->levels = o->levels > 0 ? o->levels : auto_levels(ctx->D, prob->n, o->coarsest_max > 0 ? o->coarsest_max : 729);
  for (int l = 0; l < kMaxLevels; ++l) {
    ctx->nu[l] = o->nu[l];
    ctx->relax[l] = o->relax[l];
  }
  st = check_levels(ctx);
  if (st == ADR_OK) st = setup_impl(ctx, prob);
  if (st != ADR_OK) {
    g_setup_error = ctx->err;
    free_ctx(ctx);
    return st;
  }
  ctx->setup_ms = now_ms() - t0;
  ctx->arena = nullptr;   // later allocations are ordinary ones
  ctx->layout = nullptr;
  *out = ctx;
  return ADR_OK;
}

}  // namespace

// ======================================================================================
// C ABI
// ======================================================================================
extern "C" {

void adr_default_options(adr_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->prec = ADR_PREC_MIXED;
  o->levels = 0;
  o->coarsest_max = 729;
  for (int l = 0; l < 8; ++l) {
    o->nu[l] = l + 2;
    o->relax[l] = l == 0 ? ADR_RELAX_JACOBI : ADR_RELAX_GMRES;
  }
  o->jacobi_weight = 0.8;
  o->beta = 0.25;
  o->restart = 5;
  o->use_graph = 1;
  o->cycle = ADR_CYCLE_V;
  o->kcycle_threshold = 0.1;
  o->tail_max_nodes = 0;
  o->shift_alpha = 0.0;
  o->advection = ADR_ADV_UPWIND;
  o->outer_beta = 0.0;
  o->rescaled = 0;
  o->pipeline_max_nodes = 0x7fffffff;   // every coarse level
  o->fine_tiles = 1;
  o->batch_merge = 0;
}

adr_status adr_setup(const adr_problem *prob, const adr_options *opt, void *stream, adr_ctx **out) {
  return setup_ctx(prob, opt, (hipStream_t)stream, nullptr, 0, false, out);
}

void adr_destroy(adr_ctx *ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  free_ctx(ctx);
}

int adr_num_levels(const adr_ctx *ctx) { return ctx ? ctx->levels : 0; }

adr_status adr_level_info(adr_ctx *ctx, int level, int *nodes, int *stencil_points) {
  if (!ctx || level < 0 || level >= ctx->levels) return ADR_EINVAL;
  const Grid &G = ctx->opt.prec == ADR_PREC_MIXED ? ctx->lv32[level].G : ctx->lv64[level].G;
  if (nodes)
    for (int k = 0; k < 3; ++k) nodes[k] = G.n[k];
  if (stencil_points) *stencil_points = level == 0 ? 0 : ctx->S_coarse;
  return ADR_OK;
}

int adr_tuning_table_write(const char *path) {
  if (!path) return -1;
  FILE *f = std::fopen(path, "w");
  if (!f) return -1;
  std::lock_guard<std::mutex> g(g_tune_mu);
  std::fprintf(f, "# ndim nx ny nz real_bytes variant slabs ms_per_8_launches\n");
  int n = 0;
  for (auto &kv : g_tune) {
    const auto &k = kv.first;
    std::fprintf(f, "%d %d %d %d %d %d %d %.6f\n", k[0], k[1], k[2], k[3], k[4], kv.second.split, kv.second.slabs,
                 (double)kv.second.ms);
    ++n;
  }
  std::fclose(f);
  return n;
}

int adr_tuning_table_read(const char *path) {
  if (!path) return -1;
  FILE *f = std::fopen(path, "r");
  if (!f) return -1;
  char line[256];
  int n = 0;
  std::lock_guard<std::mutex> g(g_tune_mu);
  while (std::fgets(line, sizeof(line), f)) {
    if (line[0] == '#') continue;
    int d, nx, ny, nz, rb, split, slabs;
    double ms;
    if (std::sscanf(line, "%d %d %d %d %d %d %d %lf", &d, &nx, &ny, &nz, &rb, &split, &slabs, &ms) != 8) continue;
    if ((d != 2 && d != 3) || (rb != 4 && rb != 8) || (split != 1 && split != 4 && split != 8) || slabs < 0) {
      std::fclose(f);
      return -1;
    }
    g_tune[{d, nx, ny, nz, rb}] = TuneEntry{split, slabs, (float)ms};
    ++n;
  }
  std::fclose(f);
  return n;
}

adr_status adr_level_split(adr_ctx *ctx, int level, int *split) {
  if (!ctx || !split || level < 1 || level >= ctx->levels - 1) return ADR_EINVAL;
  *split = ctx->opt.prec == ADR_PREC_MIXED ? ctx->lv32[level].split : ctx->lv64[level].split;
  return ADR_OK;
}

adr_status adr_get_level_stencil(adr_ctx *ctx, int level, void *planes_c128, int *offsets) {
  if (!ctx || level < 1 || level >= ctx->levels) return ADR_EINVAL;
  if (offsets) std::memcpy(offsets, ctx->h_off_coarse.data(), ctx->h_off_coarse.size() * sizeof(int));
  if (!planes_c128) return ADR_OK;
  hipStream_t s = ctx->stream;
  if (ctx->opt.prec == ADR_PREC_MIXED) {
    const LevelT<float> &L = ctx->lv32[level];
    adrk::convert<double, float>(s, (long long)L.S * L.G.N, L.planes, (cx<double> *)planes_c128);
  } else {
    const LevelT<double> &L = ctx->lv64[level];
    ADR_HIP(hipMemcpyAsync(planes_c128, L.planes, sizeof(cx<double>) * L.S * L.G.N, hipMemcpyDeviceToDevice, s));
  }
  ADR_HIP(hipGetLastError());
  return ADR_OK;
}

adr_status adr_get_coefficients(adr_ctx *ctx, double *g, double *L, void *c_c128) {
  if (!ctx) return ADR_EINVAL;
  hipStream_t s = ctx->stream;
  const int N = ctx->G0.N;
  if (g)
    for (int k = 0; k < ctx->D; ++k)
      ADR_HIP(hipMemcpyAsync(g + (size_t)k * N, ctx->g64[k], sizeof(double) * N, hipMemcpyDeviceToDevice, s));
  if (L) ADR_HIP(hipMemcpyAsync(L, ctx->L64, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
  if (c_c128) ADR_HIP(hipMemcpyAsync(c_c128, ctx->c64, sizeof(cx<double>) * N, hipMemcpyDeviceToDevice, s));
  return ADR_OK;
}

adr_status adr_apply(adr_ctx *ctx, double beta, const void *x, void *y) {
  if (!ctx || !x || !y || x == y) return ADR_EINVAL;
  adrk::fine_apply<double, double, double>(ctx->stream, ctx->G0, ctx->D, fine_coef<double>(ctx),
                                           fine_params(ctx, beta), (const cx<double> *)x, nullptr, (cx<double> *)y,
                                           0, nullptr, false, nullptr);
  ADR_HIP(hipGetLastError());
  return ADR_OK;
}

adr_status adr_vcycle(adr_ctx *ctx, const void *r, void *z) {
  if (!ctx || !r || !z || r == z) return ADR_EINVAL;
  ADR_TRY(precondition(ctx, (const cx<double> *)r, z, true));
  ADR_HIP(hipGetLastError());
  return ADR_OK;
}

adr_status adr_wavefield(adr_ctx *ctx, const void *a, void *u) {
  if (!ctx || !a || !u) return ADR_EINVAL;
  adrk::phase(ctx->stream, ctx->G0.N, (const cx<double> *)a, ctx->tau, ctx->omega, -1, (cx<double> *)u);
  ADR_HIP(hipGetLastError());
  return ADR_OK;
}

}  // extern "C"

namespace {
// r = rhs - (H or H^H) x in FP64 with the norm partials in part[0]; returns the block count.
int fine_residual64(adr_ctx *ctx, const cx<double> *x, const cx<double> *rhs, cx<double> *r) {
  FineCoef<double> C = fine_coef<double>(ctx);
  FineParams P0 = fine_params(ctx, ctx->opt.outer_beta);
  if (ctx->adj)
    return adrk::fine_apply_adj<double, double, double>(ctx->stream, ctx->G0, ctx->D, C, P0, x, rhs, r, 1, nullptr,
                                                        true, ctx->part[0]);
  return adrk::fine_apply<double, double, double>(ctx->stream, ctx->G0, ctx->D, C, P0, x, rhs, r, 1, nullptr, true,
                                                  ctx->part[0], ctx->Pdev);
}

// Conjugate-transposed hierarchy, built on the first adjoint solve.
template <typename T>
adr_status prepare_adjoint_levels(adr_ctx *ctx) {
  LevelT<T> *lv = levels_of<T>(ctx);
  for (int l = 1; l < ctx->levels; ++l) {
    LevelT<T> &L = lv[l];
    if (L.S == 0) continue;
    ADR_TRY(dalloc(ctx, &L.planes_adj, (size_t)L.S * L.G.N));
    adrk::adjoint_planes<T>(ctx->stream, L.G, ctx->D, L.planes, L.planes_adj);
    if (L.planes_t) {
      ADR_TRY(dalloc(ctx, &L.planes_adj_t, (size_t)adrk::tiled_plane_count(L.G, ctx->D, L.S)));
      adrk::tile_planes<T>(ctx->stream, L.G, L.S, L.planes_adj, L.planes_adj_t);
    }
    ADR_TRY(dalloc(ctx, &L.dinv_adj, L.G.N));
    adrk::stencil_diag_inv<T>(ctx->stream, L.G.N, L.planes_adj + (size_t)((L.S - 1) / 2) * L.G.N, L.dinv_adj);
  }
  return ADR_OK;
}
adr_status prepare_adjoint(adr_ctx *ctx) {
  if (ctx->adj_ready) return ADR_OK;
  if (ctx->opt.rescaled) {
    ctx->err = "adjoint solves with a rescaled cycle are not supported";
    return ADR_ENOTSUP;
  }
  if (ctx->levels > 1 && ctx->relax[0] == ADR_RELAX_GMRES) {
    ctx->err = "adjoint solves with GMRES relaxation on the finest level are not supported";
    return ADR_ENOTSUP;
  }
  if (ctx->opt.prec == ADR_PREC_MIXED) ADR_TRY(prepare_adjoint_levels<float>(ctx));
  else ADR_TRY(prepare_adjoint_levels<double>(ctx));
  const int n = ctx->Ncoarsest;
  std::vector<std::complex<double>> t((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) t[(size_t)i * n + j] = std::conj(ctx->h_inv[(size_t)j * n + i]);
  ADR_TRY(dalloc(ctx, &ctx->Ainv_adj, (size_t)n * n));
  ADR_HIP(hipMemcpyAsync(ctx->Ainv_adj, t.data(), t.size() * sizeof(cx<double>), hipMemcpyHostToDevice,
                         ctx->stream));
  ADR_HIP(hipStreamSynchronize(ctx->stream));
  ADR_HIP(hipGetLastError());
  if (ctx->opt.prec == ADR_PREC_MIXED) ADR_TRY(build_tail_args<float>(ctx, 1));
  else ADR_TRY(build_tail_args<double>(ctx, 1));
  ctx->adj_ready = true;
  return ADR_OK;
}

// FGMRES(m) on H_2up (ctx->adj false) or its conjugate transpose (true), preconditioned
// by the matching V-cycle; rhs_hat = rhs exp(i w tau).  Written as a state machine whose
// every action is enqueued on the context stream and ends with one asynchronous
// read-back into pinned host memory; `finish` consumes it on the host after the stream
// (or, for a batch, every stream) has been synchronized and decides the next action.
// Pinned layout (doubles): [0, 512) and [512, 1024) reduction partials, [1024, 1100)
// Hessenberg column read-back, [1100, 1140) least-squares coefficients for upload.
constexpr int kPinA = 0, kPinB = 512, kPinRed = 1024, kPinY = 1100;

struct Solver {
  enum Action { START, STEP, CYCLE_END, DONE };
  adr_ctx *ctx = nullptr;
  const cx<double> *q = nullptr;
  cx<double> *x = nullptr;
  double tol = 0;
  int maxit = 0;
  bool guess = false;
  Action next = START;
  int nb = 0;
  double bnorm = 0, rnorm = 0, relres = 0, t0 = 0;
  int iters = 0, restarts = 0, j = 0, k = 0;
  bool full = false;     // restart cycles always take m steps (shot groups run in lockstep)
  adr_status result = ADR_OK;
  std::complex<double> Hh[kMaxRestart + 1][kMaxRestart], g[kMaxRestart + 1], sn[kMaxRestart];
  double cs[kMaxRestart];
};

void *zslot(adr_ctx *ctx, int j) {
  const size_t N = ctx->G0.N;
  return ctx->opt.prec == ADR_PREC_MIXED ? (void *)((cx<float> *)ctx->Zo + (size_t)j * N)
                                         : (void *)((cx<double> *)ctx->Zo + (size_t)j * N);
}

// Enqueue the action S.next (the cycle's first step also scales V0 = r / ||r||).
// One FGMRES action in three parts, so that a shot group can run the kernels once for
// all its problems: solver_pre moves a problem's host-side inputs to the device,
// solver_device enqueues the kernels (on the lead problem's buffers, shifted per problem
// inside a shot-group launch), solver_post starts the read-backs of a problem's scalars.
adr_status solver_pre(Solver &S) {
  if (S.next != Solver::CYCLE_END) return ADR_OK;
  adr_ctx *ctx = S.ctx;
  double *hp = ctx->hpin;
  // y = R^{-1} g for the host's rotated Hessenberg, then to the device.
  const int k = S.k;
  std::complex<double> y[kMaxRestart];
  for (int i = k - 1; i >= 0; --i) {
    std::complex<double> acc = S.g[i];
    for (int jj = i + 1; jj < k; ++jj) acc -= S.Hh[i][jj] * y[jj];
    y[i] = (S.Hh[i][i] == 0.0) ? 0.0 : acc / S.Hh[i][i];
  }
  for (int i = 0; i < k; ++i) {
    hp[kPinY + 2 * i] = y[i].real();
    hp[kPinY + 2 * i + 1] = y[i].imag();
  }
  ADR_HIP(hipMemcpyAsync(ctx->osc + 48, hp + kPinY, 2 * k * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  return ADR_OK;
}

// A = the action (next, j, k, nb, guess); ctx, q, x = the lead problem's buffers.
adr_status solver_device(const Solver &A, adr_ctx *ctx, const cx<double> *q, cx<double> *x) {
  hipStream_t s = ctx->stream;
  const int N = ctx->G0.N, D = ctx->D;
  const bool mixed = ctx->opt.prec == ADR_PREC_MIXED;
  auto Vp = [&](int j) { return ctx->Vo + (size_t)j * N; };
  use_grids(ctx, kFullGrids, 0);
  switch (A.next) {
    case Solver::START: {
      adrk::phase(s, N, q, ctx->tau, ctx->omega, +1, ctx->qh, &ctx->Pdev[0].omega);
      adrk::norm2<double>(s, N, ctx->qh, nullptr, nullptr, ctx->part[0]);
      if (A.guess) {
        // ||q_hat|| is read back before the residual overwrites the partials.
        ADR_HIP(hipMemcpyAsync(ctx->hpin + kPinA, ctx->part[0], A.nb * sizeof(double), hipMemcpyDeviceToHost, s));
        fine_residual64(ctx, x, ctx->qh, ctx->ro);
      } else {
        adrk::zero(s, N, x);
        adrk::copy(s, N, ctx->qh, ctx->ro);
      }
      return ADR_OK;
    }
    case Solver::STEP: {
      const int j = A.j;
      // V_0 = r / ||r||, the norm from the partials of the residual just computed.
      if (j == 0) adrk::normalize(s, N, ctx->ro, ProIn{ctx->part[0], A.nb, 1}, Vp(0));
      ADR_TRY(precondition(ctx, Vp(j), zslot(ctx, j), !mixed));
      use_grids(ctx, kFullGrids, 0);
      VecSet<double> Vs{};
      Vs.count = j + 1;
      for (int i = 0; i <= j; ++i) Vs.v[i] = Vp(i);
      double *red1 = ctx->osc + 2, *red2 = ctx->osc + 2 + 2 * (kMaxRestart + 1);
      FineCoef<double> C = fine_coef<double>(ctx);
      FineParams P0 = fine_params(ctx, ctx->opt.outer_beta);
      int t0 = tbegin(ctx, ADR_TIMER_OUTER_MATVEC, 0);
      int nb;
      if (mixed && ctx->adj)
        nb = adrk::fine_apply_adj<double, float, double>(s, ctx->G0, D, C, P0, (const cx<float> *)zslot(ctx, j),
                                                         nullptr, ctx->wo, 0, &Vs, false, ctx->part[0]);
      else if (mixed)
        nb = adrk::fine_apply<double, float, double>(s, ctx->G0, D, C, P0, (const cx<float> *)zslot(ctx, j),
                                                     nullptr, ctx->wo, 0, &Vs, false, ctx->part[0], ctx->Pdev);
      else if (ctx->adj)
        nb = adrk::fine_apply_adj<double, double, double>(s, ctx->G0, D, C, P0,
                                                          (const cx<double> *)zslot(ctx, j), nullptr, ctx->wo, 0,
                                                          &Vs, false, ctx->part[0]);
      else
        nb = adrk::fine_apply<double, double, double>(s, ctx->G0, D, C, P0, (const cx<double> *)zslot(ctx, j),
                                                      nullptr, ctx->wo, 0, &Vs, false, ctx->part[0], ctx->Pdev);
      tend(ctx, t0, (double)N * (fine_coef_bytes<double>(D) + (mixed ? 8.0 : 16.0) + 16.0 * (j + 2)));
      int t1 = tbegin(ctx, ADR_TIMER_OUTER_ORTH, 0);
      nb = adrk::outer_orth1(s, N, ctx->wo, Vs, ProIn{ctx->part[0], nb, 2 * (j + 1)}, red1, ctx->part[1]);
      adrk::outer_orth2(s, N, ctx->wo, Vs, ProIn{ctx->part[1], nb, 2 * (j + 1) + 1}, red2, Vp(j + 1));
      tend(ctx, t1, (double)N * 16.0 * (2 * (j + 1) + 4));
      return ADR_OK;
    }
    case Solver::CYCLE_END: {
      // x += Z y (y uploaded by solver_pre), then the true residual.
      const int k = A.k;
      double *ydev = ctx->osc + 48;
      if (mixed) {
        VecSet<float> Zs{};
        Zs.count = k;
        for (int i = 0; i < k; ++i) Zs.v[i] = (const cx<float> *)zslot(ctx, i);
        adrk::multi_axpy<float>(s, N, x, Zs, ydev);
      } else {
        VecSet<double> Zs{};
        Zs.count = k;
        for (int i = 0; i < k; ++i) Zs.v[i] = (const cx<double> *)zslot(ctx, i);
        adrk::multi_axpy<double>(s, N, x, Zs, ydev);
      }
      fine_residual64(ctx, x, ctx->qh, ctx->ro);
      return ADR_OK;
    }
    case Solver::DONE:
      return ADR_OK;
  }
  return ADR_OK;
}

adr_status solver_post(Solver &S) {
  adr_ctx *ctx = S.ctx;
  hipStream_t s = ctx->stream;
  double *hp = ctx->hpin;
  switch (S.next) {
    case Solver::START:
      ADR_HIP(hipMemcpyAsync(hp + (S.guess ? kPinB : kPinA), ctx->part[0], S.nb * sizeof(double),
                             hipMemcpyDeviceToHost, s));
      return ADR_OK;
    case Solver::STEP: {
      const int nred = 2 * (kMaxRestart + 1) * 2 + 1;
      ADR_HIP(hipMemcpyAsync(hp + kPinRed, ctx->osc + 2, nred * sizeof(double), hipMemcpyDeviceToHost, s));
      return ADR_OK;
    }
    case Solver::CYCLE_END:
      ADR_HIP(hipMemcpyAsync(hp + kPinA, ctx->part[0], S.nb * sizeof(double), hipMemcpyDeviceToHost, s));
      return ADR_OK;
    case Solver::DONE:
      return ADR_OK;
  }
  return ADR_OK;
}

adr_status solver_enqueue(Solver &S) {
  ADR_TRY(solver_pre(S));
  ADR_TRY(solver_device(S, S.ctx, S.q, S.x));
  return solver_post(S);
}

// Consume the read-back of the last action (its stream has been synchronized) and set
// S.next; DONE ends the solve.
void solver_finish(Solver &S) {
  adr_ctx *ctx = S.ctx;
  const double *hp = ctx->hpin;
  const int m = ctx->opt.restart;
  auto sum_sqrt = [&](const double *p, int nb) {
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) acc += p[b];
    return std::sqrt(acc);
  };
  auto start_cycle_or_stop = [&]() {
    if (!std::isfinite(S.relres)) {
      S.result = ADR_ENUMERIC;
      S.next = Solver::DONE;
    } else if (S.relres <= S.tol || S.iters >= S.maxit) {
      S.next = Solver::DONE;
    } else {
      for (int i = 0; i <= m; ++i) S.g[i] = 0.0;
      S.g[0] = S.rnorm;
      S.j = 0;
      S.next = Solver::STEP;
    }
  };
  switch (S.next) {
    case Solver::START: {
      S.bnorm = sum_sqrt(hp + kPinA, S.nb);
      S.rnorm = S.guess ? sum_sqrt(hp + kPinB, S.nb) : S.bnorm;
      if (S.bnorm == 0.0) {
        S.relres = 0.0;
        S.next = Solver::DONE;
        return;
      }
      S.relres = S.rnorm / S.bnorm;
      start_cycle_or_stop();
      return;
    }
    case Solver::STEP: {
      const int j = S.j;
      const double *h1 = hp + kPinRed, *h2 = hp + kPinRed + 2 * (kMaxRestart + 1);
      double n2 = h2[2 * (j + 1)];
      for (int i = 0; i <= j; ++i) {
        std::complex<double> c(h2[2 * i], h2[2 * i + 1]);
        S.Hh[i][j] = std::complex<double>(h1[2 * i], h1[2 * i + 1]) + c;
        n2 -= std::norm(c);
      }
      S.Hh[j + 1][j] = std::sqrt(n2 > 0 ? n2 : 0.0);
      for (int i = 0; i < j; ++i) {   // earlier Givens rotations
        std::complex<double> t = S.cs[i] * S.Hh[i][j] + S.sn[i] * S.Hh[i + 1][j];
        S.Hh[i + 1][j] = -std::conj(S.sn[i]) * S.Hh[i][j] + S.cs[i] * S.Hh[i + 1][j];
        S.Hh[i][j] = t;
      }
      std::complex<double> aa = S.Hh[j][j], bb = S.Hh[j + 1][j];
      double den = std::sqrt(std::norm(aa) + std::norm(bb));
      if (std::abs(aa) == 0.0) {
        S.cs[j] = 0.0;
        S.sn[j] = 1.0;
      } else {
        S.cs[j] = std::abs(aa) / den;
        S.sn[j] = (aa / std::abs(aa)) * std::conj(bb) / den;
      }
      S.Hh[j][j] = S.cs[j] * aa + S.sn[j] * bb;
      S.Hh[j + 1][j] = 0.0;
      S.g[j + 1] = -std::conj(S.sn[j]) * S.g[j];
      S.g[j] = S.cs[j] * S.g[j];
      ++S.iters;
      const double est = std::abs(S.g[j + 1]) / S.bnorm;
      if (!std::isfinite(est)) {
        S.result = ADR_ENUMERIC;
        S.next = Solver::DONE;
      } else if ((!S.full && (est <= S.tol || S.iters >= S.maxit)) || j == m - 1) {
        S.k = j + 1;
        S.next = Solver::CYCLE_END;
      } else {
        S.j = j + 1;
      }
      return;
    }
    case Solver::CYCLE_END: {
      S.rnorm = sum_sqrt(hp + kPinA, S.nb);
      S.relres = S.rnorm / S.bnorm;
      ++S.restarts;
      start_cycle_or_stop();
      return;
    }
    case Solver::DONE:
      return;
  }
}

void solver_init(Solver &S, adr_ctx *ctx, const void *q, void *a_out, double tol, int maxit, int guess) {
  S.ctx = ctx;
  S.nb = launch_blocks_red(ctx->G0.N);   // block count of every norm reduction over the fine grid
  S.full = ctx->opt.full_cycles != 0;
  S.q = (const cx<double> *)q;
  S.x = (cx<double> *)a_out;
  S.tol = tol;
  S.maxit = maxit;
  S.guess = guess != 0;
  S.next = Solver::START;
  S.t0 = now_ms();
}

adr_status solver_result(Solver &S, adr_stats *stats) {
  adr_status r = S.result;
  if (r == ADR_OK && S.relres > S.tol) r = std::isfinite(S.relres) ? ADR_ENOCONV : ADR_ENUMERIC;
  if (stats) {
    adr_stats st{};
    st.outer_iters = S.iters;
    st.restarts = S.restarts;
    st.relres = S.relres;
    st.setup_ms = S.ctx->setup_ms;
    st.solve_ms = now_ms() - S.t0;
    *stats = st;
  }
  if (r == ADR_ENOCONV) S.ctx->err = "FGMRES reached maxit before tol";
  return r;
}

adr_status solve_impl(adr_ctx *ctx, const void *q, void *a_out, double tol, int maxit, int use_initial_guess,
                      adr_stats *stats) {
  Solver S;
  solver_init(S, ctx, q, a_out, tol, maxit, use_initial_guess);
  while (S.next != Solver::DONE) {
    ADR_TRY(solver_enqueue(S));
    ADR_HIP(hipStreamSynchronize(ctx->stream));
    solver_finish(S);
  }
  ADR_HIP(hipGetLastError());
  return solver_result(S, stats);
}
}  // namespace

extern "C" {

adr_status adr_solve(adr_ctx *ctx, const void *q, void *a_out, double tol, int maxit, int use_initial_guess,
                     adr_stats *stats) {
  if (!ctx || !q || !a_out || maxit < 0 || !(tol >= 0)) return ADR_EINVAL;
  ctx->adj = false;
  return solve_impl(ctx, q, a_out, tol, maxit, use_initial_guess, stats);
}

void adr_two_stage_options(adr_options *first, adr_options *second) {
  if (!first || !second) return;
  const adr_precision prec = first->prec;
  adr_default_options(first);
  adr_default_options(second);
  first->prec = second->prec = prec;
  first->beta = 1.0;
  first->outer_beta = 1.0;
  first->cycle = ADR_CYCLE_K;
  second->advection = ADR_ADV_CENTRAL;
  second->beta = 0.0;
  second->shift_alpha = 0.2;
  second->rescaled = 1;
  second->cycle = ADR_CYCLE_K;
}

adr_status adr_solve_two_stage(adr_ctx *first, adr_ctx *second, const void *q, void *a, double tol_first,
                               int maxit_first, double tol, int maxit, adr_stats *st_first, adr_stats *st_second) {
  if (!first || !second || first == second || !q || !a || maxit_first < 0 || maxit < 0 || !(tol_first >= 0) ||
      !(tol >= 0))
    return ADR_EINVAL;
  if (first->D != second->D || first->G0.N != second->G0.N || first->G0.n[0] != second->G0.n[0] ||
      first->G0.n[1] != second->G0.n[1] || first->G0.n[2] != second->G0.n[2]) {
    second->err = "the two stages need contexts on the same grid";
    return ADR_EINVAL;
  }
  first->adj = false;
  adr_status st = solve_impl(first, q, a, tol_first, maxit_first, 0, st_first);
  if (st != ADR_OK && st != ADR_ENOCONV) return st;
  // adr_solve synchronizes its stream, so the second stage (on its own stream) sees a.
  second->adj = false;
  return solve_impl(second, q, a, tol, maxit, 1, st_second);
}

adr_status adr_solve_adjoint(adr_ctx *ctx, const void *s_c128, void *lam_c128, double tol, int maxit,
                             int use_initial_guess, adr_stats *stats) {
  if (!ctx || !s_c128 || !lam_c128 || maxit < 0 || !(tol >= 0)) return ADR_EINVAL;
  ADR_TRY(prepare_adjoint(ctx));
  ctx->adj = true;
  adr_status st = solve_impl(ctx, s_c128, lam_c128, tol, maxit, use_initial_guess, stats);
  ctx->adj = false;
  return st;
}

adr_status adr_apply_adjoint(adr_ctx *ctx, const void *x, void *y) {
  if (!ctx || !x || !y || x == y) return ADR_EINVAL;
  adrk::fine_apply_adj<double, double, double>(ctx->stream, ctx->G0, ctx->D, fine_coef<double>(ctx),
                                               fine_params(ctx, ctx->opt.outer_beta), (const cx<double> *)x, nullptr,
                                               (cx<double> *)y, 0, nullptr, false, nullptr);
  ADR_HIP(hipGetLastError());
  return ADR_OK;
}

adr_status adr_grad_kappa2(adr_ctx *ctx, const void *a, const void *lam, double *grad) {
  if (!ctx || !a || !lam || !grad) return ADR_EINVAL;
  adrk::grad_kappa2(ctx->stream, ctx->G0.N, ctx->omega, ctx->opt.reaction == ADR_REACTION_NUMERICAL, ctx->gamma,
                    (const cx<double> *)a, (const cx<double> *)lam, grad);
  ADR_HIP(hipGetLastError());
  return ADR_OK;
}

adr_status adr_receiver_residual(adr_ctx *ctx, const void *u, const int *idx, const void *d, int nrec, void *r,
                                 double *misfit) {
  if (!ctx || !u || !idx || !d || !r || nrec <= 0) return ADR_EINVAL;
  hipStream_t s = ctx->stream;
  adrk::receiver_residual(s, nrec, idx, (const cx<double> *)u, (const cx<double> *)d, (cx<double> *)r);
  if (misfit) {
    const int nb = adrk::norm2<double>(s, nrec, (const cx<double> *)r, nullptr, nullptr, ctx->part[0]);
    ADR_HIP(hipMemcpyAsync(ctx->hpin, ctx->part[0], nb * sizeof(double), hipMemcpyDeviceToHost, s));
    ADR_HIP(hipStreamSynchronize(s));
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) acc += ctx->hpin[b];
    *misfit = 0.5 * acc;
  }
  ADR_HIP(hipGetLastError());
  return ADR_OK;
}

}  // extern "C"

namespace {
// Device scratch of adr_receiver_residual_noalloc: the per-block partial sums of the misfit
// (one per reduction block, at most ADR_MAX_RED_BLOCKS).  Every GPU holds its own copy; host
// code uses the address hipGetSymbolAddress returns for the current device, never the name.
constexpr int kNoAllocPartials = ADR_MAX_RED_BLOCKS;
static __device__ __align__(256) double scratch[kNoAllocPartials];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch`, looked up on the first call on that device.
adr_status noalloc_scratch(double **out, std::string &err) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    err = std::string("hipGetDevice failed: ") + hipGetErrorString(e);
    return ADR_EHIP;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    err = "device index out of range for the no-allocation scratch";
    return ADR_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      err = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e);
      return ADR_EHIP;
    }
    g_scratch_ptr[dev] = (double *)ptr;
  }
  *out = g_scratch_ptr[dev];
  return ADR_OK;
}
}  // namespace

extern "C" {

adr_status adr_receiver_residual_noalloc(const void *u, const int *idx, const void *d, int nrec, void *r,
                                         double *misfit, void *stream) {
  if (!u || !idx || !d || !r) {
    g_setup_error = "null pointer argument";
    return ADR_EINVAL;
  }
  if (nrec <= 0 || nrec > ADR_NOALLOC_MAX_REC) {
    g_setup_error = "nrec must be in [1, ADR_NOALLOC_MAX_REC = " + std::to_string(ADR_NOALLOC_MAX_REC) + "]";
    return ADR_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  adrk::receiver_residual(s, nrec, idx, (const cx<double> *)u, (const cx<double> *)d, (cx<double> *)r);
  if (misfit) {
    double *part = nullptr;
    std::string err;
    adr_status st = noalloc_scratch(&part, err);
    if (st != ADR_OK) {
      g_setup_error = err;
      return st;
    }
    const int nb = adrk::norm2<double>(s, nrec, (const cx<double> *)r, nullptr, nullptr, part);
    if (nb > kNoAllocPartials) {
      g_setup_error = "reduction wider than the no-allocation scratch";
      return ADR_EINVAL;
    }
    // Same summation order as adr_receiver_residual: the partials in block order on the host.
    double host[kNoAllocPartials];
    hipError_t e = hipMemcpyAsync(host, part, nb * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      g_setup_error = std::string("HIP error: ") + hipGetErrorString(e);
      return ADR_EHIP;
    }
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) acc += host[b];
    *misfit = 0.5 * acc;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    g_setup_error = std::string("HIP error: ") + hipGetErrorString(e);
    return ADR_EHIP;
  }
  return ADR_OK;
}

adr_status adr_adjoint_source(adr_ctx *ctx, const int *idx, const void *r, int nrec, void *src) {
  if (!ctx || !idx || !r || !src || nrec <= 0) return ADR_EINVAL;
  adrk::adjoint_source(ctx->stream, ctx->G0.N, nrec, idx, (const cx<double> *)r, (cx<double> *)src);
  ADR_HIP(hipGetLastError());
  return ADR_OK;
}

// ---------------------------------------------------------------------------------------
// Batched shots.  Problems with the same grid shape form a shot group: their contexts
// are built in one arena, one slot per problem at a constant stride, so every kernel of
// an FGMRES action runs once for the whole group (blockIdx.y = problem, see Shot) on the
// group's stream, V-cycles included (captured per group).  The FGMRES state machines stay
// per problem on the host; restart cycles always take m steps so that the problems of a
// group stay in lockstep (same action, same Arnoldi index), and a converged problem is
// switched off by its device flag.  Groups advance independently: the host finishes
// whichever group's last action has completed and enqueues its next one.
// ---------------------------------------------------------------------------------------
}  // extern "C"

struct adr_batch {
  struct Group {
    std::vector<int> members;   // batch indices, slot order (a merged group's lead first)
    char *arena = nullptr;
    size_t stride = 0;
    bool merged = false;        // problems of different grid shapes (keyed slot layout)
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    // Slots the launches cover: the unfinished problems, padded to a power of two (at most
    // the group size) with the spare slot after the last problem, whose flag stays 0, so
    // that a captured cycle serves every count in its bucket.
    int *slots_dev = nullptr;   // device copy of the list
    int *slots_pin = nullptr;   // pinned staging for its updates
    std::vector<int> slots_cur; // the list on the device
  };
  std::vector<adr_ctx *> ctx;   // per problem (contexts live in their group's arena)
  std::vector<Group> groups;
  SlotLayout layout;            // merged group: the common slot layout
  MergedGrids mg;               // merged group: per-level grid tables
  std::vector<hipStream_t> streams;
  int *pin_flags = nullptr;     // pinned host ints {0, 1} for the device flags
  std::string err;
};

namespace {
void free_batch(adr_batch *b) {
  if (!b) return;
  for (adr_ctx *c : b->ctx) adr_destroy(c);
  for (auto &g : b->groups) {
    if (g.ev) (void)hipEventDestroy(g.ev);
    if (g.arena) (void)hipFree(g.arena);
    if (g.slots_dev) (void)hipFree(g.slots_dev);
    if (g.slots_pin) (void)hipHostFree(g.slots_pin);
  }
  for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
  if (b->pin_flags) (void)hipHostFree(b->pin_flags);
  if (b->mg.dev) (void)hipFree(b->mg.dev);
  delete b;
}
Grid level_grid(const adr_ctx *c, int l) { return c->opt.prec == ADR_PREC_FP64 ? c->lv64[l].G : c->lv32[l].G; }

// A group's slot list buffers, and the spare slot's flag (after the last problem's slot,
// at the same offset as slot 0's) set to 0.
bool init_slots(adr_batch *b, adr_batch::Group &g) {
  const size_t n = g.members.size();
  if (hipMalloc((void **)&g.slots_dev, n * sizeof(int)) != hipSuccess) return false;
  if (hipHostMalloc((void **)&g.slots_pin, n * sizeof(int), hipHostMallocDefault) != hipSuccess) return false;
  const adr_ctx *lead = b->ctx[g.members[0]];
  int *spare_flag = (int *)((char *)lead->active + n * g.stride);
  return hipMemset(spare_flag, 0, sizeof(int)) == hipSuccess;
}

// One group for problems of different grid shapes (adr_options.batch_merge).  A
// measuring setup of each shape records its allocations and level grids.  The shapes
// must nest under one lead shape -- as many levels or more, and as many nodes or more on
// every level -- else this returns false (st = ADR_OK) and the batch is grouped by shape.
// Otherwise every problem gets a slot of the common keyed layout (the lead shape's first
// problem in slot 0, whose pointers every launch passes), plus one spare slot at the end
// of the arena, and the per-level grid tables are built.
bool setup_merged(adr_batch *b, const adr_problem *probs, const adr_options *opt, adr_status &st) {
  struct Shape {
    std::vector<std::pair<AllocKey, size_t>> log;
    std::vector<Grid> grids;
    int D = 0;
  };
  std::vector<Shape> shapes;
  hipStream_t s0 = b->streams[0];
  for (auto &g : b->groups) {
    adr_ctx *m = nullptr;
    st = setup_ctx(&probs[g.members[0]], opt, s0, nullptr, 0, true, &m);
    if (st != ADR_OK) {
      g_setup_error = "shot " + std::to_string(g.members[0]) + ": " + g_setup_error;
      return false;
    }
    Shape sh;
    sh.log = m->alloc_log;
    sh.D = m->D;
    for (int l = 0; l < m->levels; ++l) sh.grids.push_back(level_grid(m, l));
    adr_destroy(m);
    shapes.push_back(std::move(sh));
  }
  size_t lead = 0;
  for (size_t k = 1; k < shapes.size(); ++k) {
    const Shape &a = shapes[k], &c = shapes[lead];
    if (a.grids.size() > c.grids.size() || (a.grids.size() == c.grids.size() && a.grids[0].N > c.grids[0].N)) lead = k;
  }
  const Shape &ld = shapes[lead];
  for (const Shape &sh : shapes) {
    if (sh.D != ld.D || sh.grids.size() > ld.grids.size()) return false;
    for (size_t l = 0; l < sh.grids.size(); ++l)
      if (sh.grids[l].N > ld.grids[l].N) return false;
  }
  // Common layout: the lead shape's allocations in its order, then the keys only other
  // shapes make; each key sized for the largest allocation made under it.
  std::map<AllocKey, size_t> bytes;
  std::vector<AllocKey> order;
  auto add = [&](const Shape &sh) {
    for (const auto &[key, n] : sh.log) {
      auto it = bytes.find(key);
      if (it == bytes.end()) {
        bytes.emplace(key, n);
        order.push_back(key);
      } else if (n > it->second) {
        it->second = n;
      }
    }
  };
  add(ld);
  for (size_t k = 0; k < shapes.size(); ++k)
    if (k != lead) add(shapes[k]);
  size_t off = 0;
  for (const AllocKey &key : order) {
    b->layout.at[key] = {off, bytes[key]};
    off += bytes[key];
  }
  b->layout.stride = (off + 65535) & ~(size_t)65535;
  adr_batch::Group g;
  g.merged = true;
  g.stride = b->layout.stride;
  g.stream = b->streams[0];
  g.members = b->groups[lead].members;
  for (size_t k = 0; k < b->groups.size(); ++k)
    if (k != lead) g.members.insert(g.members.end(), b->groups[k].members.begin(), b->groups[k].members.end());
  b->groups.assign(1, g);
  adr_batch::Group &G = b->groups[0];
  const size_t count = G.members.size();
  auto hip_fail = [&](const char *what) {
    g_setup_error = what;
    st = ADR_EHIP;
    return false;
  };
  if (hipEventCreateWithFlags(&G.ev, hipEventDisableTiming) != hipSuccess) return hip_fail("hipEventCreate failed");
  if (hipMalloc((void **)&G.arena, G.stride * (count + 1)) != hipSuccess) {
    g_setup_error = "merged shot-group arena of " + std::to_string(G.stride * (count + 1)) + " bytes";
    st = ADR_ENOMEM;
    return false;
  }
  for (size_t k = 0; k < count; ++k) {
    const int i = G.members[k];
    adr_ctx *c = nullptr;
    st = setup_ctx(&probs[i], opt, G.stream, G.arena + k * G.stride, G.stride, true, &c, &b->layout);
    if (st != ADR_OK) {
      g_setup_error = "shot " + std::to_string(i) + ": " + g_setup_error;
      return false;
    }
    b->ctx[i] = c;
  }
  // Grid tables (the spare slot's column stays N = 0).
  const int Lmax = (int)ld.grids.size();
  const size_t cols = count + 1;
  std::vector<Grid> host((size_t)kGridKinds * Lmax * cols, Grid{});
  b->mg.levels = Lmax;
  b->mg.cols = (int)cols;
  b->mg.slot_levels.assign(count, 0);
  for (size_t k = 0; k < count; ++k) {
    const adr_ctx *c = b->ctx[G.members[k]];
    const int Lk = c->levels;
    b->mg.slot_levels[k] = Lk;
    for (int l = 0; l < Lk; ++l) {
      const Grid gl = level_grid(c, l);
      auto at = [&](int kind) -> Grid & { return host[((size_t)kind * Lmax + l) * cols + k]; };
      at(kFullGrids) = gl;
      if (l < Lk - 1) at(kRelaxGrids) = gl;
      else at(kCoarsestGrids) = gl;
    }
  }
  if (hipMalloc((void **)&b->mg.dev, host.size() * sizeof(Grid)) != hipSuccess) return hip_fail("hipMalloc of grid tables failed");
  if (hipMemcpy(b->mg.dev, host.data(), host.size() * sizeof(Grid), hipMemcpyHostToDevice) != hipSuccess)
    return hip_fail("grid table copy failed");
  for (size_t k = 0; k < count; ++k) {
    b->ctx[G.members[k]]->mg = &b->mg;
    b->ctx[G.members[k]]->mg_slot = (int)k;
  }
  if (!init_slots(b, G)) return hip_fail("shot-group slot list allocation failed");
  return true;
}
}  // namespace

extern "C" {

adr_status adr_setup_batch(int count, const adr_problem *probs, const adr_options *opt, int nstreams,
                           adr_batch **out) {
  if (!out) return ADR_EINVAL;
  *out = nullptr;
  if (count <= 0 || !probs || nstreams <= 0 || nstreams > 64) {
    g_setup_error = "bad batch arguments";
    return ADR_EINVAL;
  }
  if (opt && opt->rescaled) {
    g_setup_error = "batched solves with a rescaled cycle are not supported";
    return ADR_ENOTSUP;
  }
  adr_batch *b = new adr_batch();
  auto fail = [&](adr_status st, const std::string &msg) {
    g_setup_error = msg;
    free_batch(b);
    return st;
  };
  if (hipHostMalloc((void **)&b->pin_flags, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess)
    return fail(ADR_ENOMEM, "hipHostMalloc failed");
  b->pin_flags[0] = 0;
  b->pin_flags[1] = 1;
  for (int i = 0; i < nstreams; ++i) {
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return fail(ADR_EHIP, "hipStreamCreate failed");
    b->streams.push_back(s);
  }
  // Group by grid shape (first-appearance order).
  std::map<std::array<int, 4>, int> key_to_group;
  for (int i = 0; i < count; ++i) {
    const adr_problem &p = probs[i];
    const std::array<int, 4> key = {p.ndim, p.n[0], p.n[1], p.ndim == 3 ? p.n[2] : 1};
    auto it = key_to_group.find(key);
    if (it == key_to_group.end()) {
      it = key_to_group.emplace(key, (int)b->groups.size()).first;
      b->groups.emplace_back();
    }
    b->groups[it->second].members.push_back(i);
  }
  b->ctx.assign(count, nullptr);
  if (opt && opt->batch_merge && b->groups.size() > 1) {
    adr_status st = ADR_OK;
    const bool merged = setup_merged(b, probs, opt, st);
    if (st != ADR_OK) return fail(st, g_setup_error);
    if (merged) {
      *out = b;
      return ADR_OK;
    }
  }
  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    auto &g = b->groups[gi];
    g.stream = b->streams[gi % b->streams.size()];
    if (hipEventCreateWithFlags(&g.ev, hipEventDisableTiming) != hipSuccess) return fail(ADR_EHIP, "hipEventCreate failed");
    // Slot size: build the first problem once with ordinary allocations and count.
    adr_ctx *m = nullptr;
    adr_status st = setup_ctx(&probs[g.members[0]], opt, g.stream, nullptr, 0, true, &m);
    if (st != ADR_OK) return fail(st, "shot " + std::to_string(g.members[0]) + ": " + g_setup_error);
    const size_t need = m->alloc_need;
    adr_destroy(m);
    g.stride = (need + 65535) & ~(size_t)65535;
    const size_t arena_bytes = g.stride * (g.members.size() + 1);   // + the spare slot
    if (hipMalloc((void **)&g.arena, arena_bytes) != hipSuccess)
      return fail(ADR_ENOMEM, "shot-group arena of " + std::to_string(arena_bytes) + " bytes");
    for (size_t k = 0; k < g.members.size(); ++k) {
      const int i = g.members[k];
      adr_ctx *c = nullptr;
      st = setup_ctx(&probs[i], opt, g.stream, g.arena + k * g.stride, g.stride, true, &c);
      if (st != ADR_OK) return fail(st, "shot " + std::to_string(i) + ": " + g_setup_error);
      b->ctx[i] = c;
      if (c->arena_off != need)
        return fail(ADR_EINVAL, "shot " + std::to_string(i) + ": layout differs from its group's first problem");
    }
    if (!init_slots(b, g)) return fail(ADR_EHIP, "shot-group slot list allocation failed");
  }
  *out = b;
  return ADR_OK;
}

int adr_batch_size(const adr_batch *b) { return b ? (int)b->ctx.size() : 0; }

int adr_batch_groups(const adr_batch *b) { return b ? (int)b->groups.size() : 0; }

adr_ctx *adr_batch_context(adr_batch *b, int i) {
  if (!b || i < 0 || i >= (int)b->ctx.size()) return nullptr;
  return b->ctx[i];
}

adr_status adr_solve_batch(adr_batch *b, const void *const *q, void *const *a, double tol, int maxit,
                           adr_stats *stats) {
  if (!b || !q || !a || maxit < 0 || !(tol >= 0)) return ADR_EINVAL;
  const int n = (int)b->ctx.size();
  for (int i = 0; i < n; ++i)
    if (!q[i] || !a[i]) return ADR_EINVAL;
  std::vector<Solver> S(n);
  const size_t vbytes = sizeof(cx<double>);
  auto hip_fail = [&](const char *what, hipError_t e) {
    b->err = std::string(what) + ": " + hipGetErrorString(e);
    return ADR_EHIP;
  };
  // Problem inputs into the arena, flags on, state machines at START.
  for (auto &g : b->groups)
    for (int i : g.members) {
      adr_ctx *c = b->ctx[i];
      c->adj = false;
      hipError_t e = hipMemcpyAsync(c->qin, q[i], vbytes * c->G0.N, hipMemcpyDeviceToDevice, g.stream);
      if (e == hipSuccess) e = hipMemcpyAsync(c->active, b->pin_flags + 1, sizeof(int), hipMemcpyHostToDevice, g.stream);
      if (e != hipSuccess) return hip_fail("batch input copy", e);
      solver_init(S[i], c, c->qin, c->xg, tol, maxit, 0);
      S[i].full = true;
    }

  // Enqueue the next action of group g for its live problems; false when none is left.
  auto launch = [&](adr_batch::Group &g, adr_status &st) -> bool {
    std::vector<int> live;
    for (int i : g.members)
      if (S[i].next != Solver::DONE) live.push_back(i);
    if (live.empty()) return false;
    const Solver &A = S[live[0]];
    for (int i : live)
      if (S[i].next != A.next || S[i].j != A.j || (A.next == Solver::CYCLE_END && S[i].k != A.k)) {
        b->err = "shot group out of lockstep";
        st = ADR_ENUMERIC;
        return false;
      }
    for (int i : live)
      if ((st = solver_pre(S[i])) != ADR_OK) return false;
    // The launching problem: slot 0, or in a merged group the largest unfinished problem
    // (most levels, then most nodes), so that the launches shrink as large problems finish.
    const int n = (int)g.members.size();
    int k0 = 0;
    if (g.merged) {
      k0 = -1;
      for (int k = 0; k < n; ++k) {
        const adr_ctx *c = b->ctx[g.members[k]];
        if (S[g.members[k]].next == Solver::DONE) continue;
        if (k0 < 0) {
          k0 = k;
          continue;
        }
        const adr_ctx *c0 = b->ctx[g.members[k0]];
        if (c->levels > c0->levels || (c->levels == c0->levels && c->G0.N > c0->G0.N)) k0 = k;
      }
    }
    adr_ctx *lead = b->ctx[g.members[k0]];
    // The launches cover the live problems' slots (relative to the launching one), padded
    // with the spare slot.
    // (At least 2 in a group of several: a launch for one problem takes the plain,
    // unshifted kernels, which address slot 0.)
    int bucket = n >= 2 ? 2 : 1;
    while (bucket < (int)live.size()) bucket *= 2;
    if (bucket > n) bucket = n;
    std::vector<int> list;
    for (int k = 0; k < n; ++k)
      if (S[g.members[k]].next != Solver::DONE) list.push_back(k - k0);
    list.resize(bucket, n - k0);
    if (list != g.slots_cur) {
      // The previous update's copy has completed: this group's last action, enqueued
      // after it, has.
      std::copy(list.begin(), list.end(), g.slots_pin);
      hipError_t e = hipMemcpyAsync(g.slots_dev, g.slots_pin, bucket * sizeof(int), hipMemcpyHostToDevice, g.stream);
      if (e != hipSuccess) {
        st = hip_fail("slot list copy", e);
        return false;
      }
      g.slots_cur = list;
    }
    adrk::g_shot.count = bucket;
    adrk::g_shot.sh = Shot{(long long)g.stride, lead->active, nullptr, nullptr, g.slots_dev};
    st = solver_device(A, lead, lead->qin, lead->xg);
    adrk::g_shot = adrk::ShotLaunch{};
    if (st != ADR_OK) {
      b->err = lead->err;
      return false;
    }
    // This action's fine-grid reductions came in the launching problem's block count:
    // its read-backs, and the next action's first step, which sums the partials of this
    // one's residual, take that count (the step above used the previous action's).
    for (int i : live) S[i].nb = launch_blocks_red(lead->G0.N);
    for (int i : live)
      if ((st = solver_post(S[i])) != ADR_OK) return false;
    hipError_t e = hipEventRecord(g.ev, g.stream);
    if (e != hipSuccess) {
      st = hip_fail("hipEventRecord", e);
      return false;
    }
    return true;
  };
  std::vector<char> busy(b->groups.size(), 0);
  int running = 0;
  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    adr_status st = ADR_OK;
    busy[gi] = launch(b->groups[gi], st);
    if (st != ADR_OK) return st;
    running += busy[gi];
  }
  while (running > 0) {
    bool progressed = false;
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
      if (!busy[gi]) continue;
      auto &g = b->groups[gi];
      hipError_t e = hipEventQuery(g.ev);
      if (e == hipErrorNotReady) continue;
      if (e != hipSuccess) return hip_fail("batch", e);
      progressed = true;
      for (int i : g.members) {
        if (S[i].next == Solver::DONE) continue;
        solver_finish(S[i]);
        if (S[i].next == Solver::DONE) {
          adr_ctx *c = b->ctx[i];
          e = hipMemcpyAsync(c->active, b->pin_flags, sizeof(int), hipMemcpyHostToDevice, g.stream);
          if (e == hipSuccess) e = hipMemcpyAsync(a[i], c->xg, vbytes * c->G0.N, hipMemcpyDeviceToDevice, g.stream);
          if (e != hipSuccess) return hip_fail("batch result copy", e);
        }
      }
      adr_status st = ADR_OK;
      busy[gi] = launch(g, st);
      if (st != ADR_OK) return st;
      if (!busy[gi]) --running;
    }
    if (!progressed) std::this_thread::yield();
  }
  for (auto &g : b->groups) {
    hipError_t e = hipStreamSynchronize(g.stream);
    if (e != hipSuccess) return hip_fail("batch synchronization", e);
  }
  adr_status worst = ADR_OK;
  for (int i = 0; i < n; ++i) {
    adr_status st = solver_result(S[i], stats ? &stats[i] : nullptr);
    if (st != ADR_OK && (worst == ADR_OK || st != ADR_ENOCONV)) worst = st;
  }
  return worst;
}

void adr_destroy_batch(adr_batch *b) { free_batch(b); }

constexpr int kTimerLaunches = 65536;   // launches one adr_timer_start can time

adr_status adr_timer_start(adr_ctx *ctx, int kind, int level) {
  if (!ctx || kind < 0 || kind > ADR_TIMER_FINE_GMRES) return ADR_EINVAL;
  auto &T = ctx->timer;
  if (T.ev.empty()) {
    T.ev.resize(2 * (size_t)kTimerLaunches);
    for (auto &e : T.ev) ADR_HIP(hipEventCreate(&e));
  }
  T.kind = kind;
  T.level = level;
  T.used = 0;
  T.launches = 0;
  T.bytes = 0.0;
  return ADR_OK;
}

adr_status adr_timer_stop(adr_ctx *ctx, double *ms, int *launches, double *bytes) {
  if (!ctx) return ADR_EINVAL;
  auto &T = ctx->timer;
  ADR_HIP(hipStreamSynchronize(ctx->stream));
  double total = 0.0;
  for (int i = 0; i + 1 < T.used; i += 2) {
    float t = 0.f;
    ADR_HIP(hipEventElapsedTime(&t, T.ev[i], T.ev[i + 1]));
    total += t;
  }
  if (ms) *ms = total;
  if (launches) *launches = T.launches;
  if (bytes) *bytes = T.bytes;
  T.kind = -1;
  T.used = 0;
  return ADR_OK;
}

const char *adr_strerror(adr_status s) {
  switch (s) {
    case ADR_OK: return "ok";
    case ADR_EINVAL: return "invalid argument";
    case ADR_ENOMEM: return "out of memory";
    case ADR_EHIP: return "HIP runtime error";
    case ADR_ENOCONV: return "not converged";
    case ADR_ENUMERIC: return "NaN/Inf encountered";
    case ADR_ENOTSUP: return "not supported";
  }
  return "unknown status";
}

const char *adr_last_error(const adr_ctx *ctx) { return ctx ? ctx->err.c_str() : g_setup_error.c_str(); }

}  // extern "C"

namespace adrk {
void set_global_error(const std::string &e) { g_setup_error = e; }
}  // namespace adrk
