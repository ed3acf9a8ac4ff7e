// Common device/host helpers for the ADR solver kernels (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define ADR_BLOCK 256
#define ADR_MAX_BLOCKS 8192
#define ADR_NUM_XCD 8
#define ADR_MAX_RED 40      // max reduced doubles per kernel (dots are 2 doubles each)
#define ADR_MAXV 17         // max basis vectors held by one kernel (restart <= 16)

// ------------------------------------------------------------------------------------
// Complex numbers (interleaved storage, 8 or 16 bytes).
// ------------------------------------------------------------------------------------
template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T re, T im) { cx<T> r; r.re = re; r.im = im; return r; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mk<T>(a.re + b.re, a.im + b.im); }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mk<T>(a.re - b.re, a.im - b.im); }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return mk<T>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return mk<T>(s * a.re, s * a.im); }
// a + b*c
template <typename T>
__host__ __device__ __forceinline__ cx<T> cfma(cx<T> b, cx<T> c, cx<T> a) {
  a.re = fma(b.re, c.re, a.re);
  a.re = fma(-b.im, c.im, a.re);
  a.im = fma(b.re, c.im, a.im);
  a.im = fma(b.im, c.re, a.im);
  return a;
}
// conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ cx<T> cdotc(cx<T> a, cx<T> b) {
  return mk<T>(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> cinv(cx<T> a) {
  T d = a.re * a.re + a.im * a.im;
  return mk<T>(a.re / d, -a.im / d);
}
template <typename To, typename Ti>
__host__ __device__ __forceinline__ cx<To> cvt(cx<Ti> a) { return mk<To>((To)a.re, (To)a.im); }

// ------------------------------------------------------------------------------------
// Grid: nx fastest, 2D grids have nz == 1.
// ------------------------------------------------------------------------------------
struct Grid {
  int n[3];        // nodes along x, y, z
  int N;           // total nodes
  double r0, r01;  // 1 / n[0] and 1 / (n[0] n[1]) (index decoding without integer division)
};

// Node index -> (x, y, z).  The quotients come from a double-precision multiply by the
// reciprocal, then one exact correction step: for i < 2^30 the product is within 2^-22 of
// the true quotient, so the truncated value is off by at most one.
__device__ __forceinline__ void decode(const Grid &g, int i, int &x, int &y, int &z) {
  const int nxy = g.n[0] * g.n[1];
  int q = (int)((double)i * g.r01);
  int rem = i - q * nxy;
  if (rem < 0) {
    --q;
    rem += nxy;
  } else if (rem >= nxy) {
    ++q;
    rem -= nxy;
  }
  int q2 = (int)((double)rem * g.r0);
  int r2 = rem - q2 * g.n[0];
  if (r2 < 0) {
    --q2;
    r2 += g.n[0];
  } else if (r2 >= g.n[0]) {
    ++q2;
    r2 -= g.n[0];
  }
  z = q;
  y = q2;
  x = r2;
}

// ------------------------------------------------------------------------------------
// Launch shape: at most ADR_MAX_BLOCKS blocks, each owning one contiguous chunk of the
// index range.  Blocks are dispatched round-robin over the 8 XCDs; the remap below gives
// each XCD a contiguous run of chunks, so stencil neighbours in other rows and planes
// are mostly in that XCD's own L2.
// ------------------------------------------------------------------------------------
inline int launch_blocks(long long N) {
  long long b = (N + ADR_BLOCK - 1) / ADR_BLOCK;
  if (b > ADR_MAX_BLOCKS) b = ADR_MAX_BLOCKS;
  if (b < 1) b = 1;
  return (int)b;
}

// Gather-heavy kernels without reductions or per-block prologues (the matrix-free fine
// rows, prolongation): about one node per thread, up to ADR_MAX_WIDE_BLOCKS blocks.  A
// thread that loops over a chunk waits on each node's gathers in turn; many resident waves
// with one node each keep more of them in flight.
#define ADR_MAX_WIDE_BLOCKS (1 << 17)
inline int launch_blocks_wide(long long N) {
  long long b = (N + ADR_BLOCK - 1) / ADR_BLOCK;
  if (b > ADR_MAX_WIDE_BLOCKS) b = ADR_MAX_WIDE_BLOCKS;
  if (b < 1) b = 1;
  return (int)b;
}

__device__ __forceinline__ int logical_block() {
  int nb = gridDim.x, bid = blockIdx.x;
  int q = nb / ADR_NUM_XCD, r = nb % ADR_NUM_XCD;
  int xcd = bid % ADR_NUM_XCD, local = bid / ADR_NUM_XCD;
  return xcd * q + (xcd < r ? xcd : r) + local;
}

__device__ __forceinline__ void chunk_range(int N, int &beg, int &end) {
  int nb = gridDim.x;
  int lb = logical_block();
  long long chunk = ((long long)N + nb - 1) / nb;
  long long b = lb * chunk, e = b + chunk;
  if (b > N) b = N;
  if (e > N) e = N;
  beg = (int)b;
  end = (int)e;
}

// ------------------------------------------------------------------------------------
// Deterministic reductions without inter-block synchronization: every block reduces its
// K doubles in a fixed tree and writes partials[block*K + k] (plain stores).  The next
// kernel on the stream -- which needs the totals anyway -- sums those partials in block
// order in a short prologue in every block (block 0 also stores the resulting scalars
// for later kernels), or the host sums them when it reads them back.  Two partials
// buffers alternate so a kernel can read its predecessor's partials while writing its
// own.  (Device-scope fences and atomics would serialize through memory across the 8
// XCDs; a separate one-block finish kernel costs a launch per reduction.)
// ------------------------------------------------------------------------------------
// Reduction partial buffers hold ADR_PART_BLOCKS blocks; most reducing kernels launch at
// most ADR_MAX_RED_BLOCKS, the LDS-tiled Galerkin apply up to ADR_PART_BLOCKS.
#define ADR_PART_BLOCKS 1024
#ifndef ADR_MAX_RED_BLOCKS
#define ADR_MAX_RED_BLOCKS 512
#endif

inline int launch_blocks_red(long long N) {
  long long b = (N + ADR_BLOCK - 1) / ADR_BLOCK;
  if (b > ADR_MAX_RED_BLOCKS) b = ADR_MAX_RED_BLOCKS;
  if (b < 1) b = 1;
  return (int)b;
}

// ------------------------------------------------------------------------------------
// Shot groups.  One launch can serve `count` problems whose device data are laid out at a
// constant byte stride (one arena slot per problem): blockIdx.y selects the problem's
// slot (through `slots` when set), every pointer argument refers to slot 0 and is shifted
// by slot * stride, and a problem whose flag (an int at `active` + slot * stride) is 0
// exits at once.
// stride = 0, active = NULL is an ordinary single-problem launch.
// ------------------------------------------------------------------------------------
struct Shot {
  long long stride;
  const int *active;
  const Grid *grid;    // merged shapes: each problem's grid on the launch's level (else NULL)
  const Grid *grid2;   // merged shapes, transfers: each problem's coarse grid
  const int *slots;    // slot of blockIdx.y (the problems still being solved, padded with a
                       // spare slot whose flag is 0); NULL: slot = blockIdx.y
};
template <typename P>
__device__ __forceinline__ P *shot_ptr(P *p, long long off) {
  return p ? (P *)((char *)p + off) : p;
}
// Group-capable kernels carry a template flag GRP: the GRP = false instance (ordinary
// launches) compiles to the plain kernel, the GRP = true instance (shot-group launches)
// shifts its pointers and skips inactive problems.  ADR_SHOT_ENTER declares shot_off_;
// ADR_SHOT_LIVE returns from an inactive problem (uniform per block).
#define ADR_SHOT_ENTER(sh)                                                                     \
  [[maybe_unused]] const int shot_slot_ = GRP ? ((sh).slots ? (sh).slots[blockIdx.y] : (int)blockIdx.y) : 0; \
  const long long shot_off_ = GRP ? (long long)shot_slot_ * (sh).stride : 0LL
#define ADR_SHOT_LIVE(sh)                                                                    \
  do {                                                                                       \
    if constexpr (GRP) {                                                                     \
      if ((sh).active && !*(const int *)((const char *)(sh).active + shot_off_)) return;    \
    }                                                                                        \
  } while (0)
// Groups that merge problems of different grid shapes (one slot layout for all, sized
// for the largest) take each problem's own grid (and coarse grid, for the transfers) from
// the launch's per-problem table instead of the argument, which is the largest problem's;
// a problem without that level (N = 0 in the table) exits.  Block counts stay those of
// the largest problem, so a smaller problem's blocks own shorter chunks.
#define ADR_SHOT_GRID(sh, G)                               \
  do {                                                     \
    if constexpr (GRP) {                                   \
      if ((sh).grid) {                                     \
        (G) = (sh).grid[shot_slot_];                       \
        if ((G).N == 0) return;                            \
      }                                                    \
    }                                                      \
  } while (0)
#define ADR_SHOT_GRID2(sh, G)                              \
  do {                                                     \
    if constexpr (GRP) {                                   \
      if ((sh).grid2) (G) = (sh).grid2[shot_slot_];        \
    }                                                      \
  } while (0)
#define ADR_SHOT_N(sh, n)                                  \
  do {                                                     \
    if constexpr (GRP) {                                   \
      if ((sh).grid) {                                     \
        (n) = (sh).grid[shot_slot_].N;                     \
        if ((n) == 0) return;                              \
      }                                                    \
    }                                                      \
  } while (0)
#define ADR_SHOT_SKIP(sh)                                  \
  do {                                                     \
    if constexpr (GRP) {                                   \
      if ((sh).grid && (sh).grid[shot_slot_].N == 0) return; \
    }                                                      \
  } while (0)
#define ADR_SHIFT(p)                        \
  do {                                      \
    if constexpr (GRP) {                    \
      (p) = shot_ptr((p), shot_off_);       \
    }                                       \
  } while (0)

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Reduce acc[0..K) over the block; thread 0 ends with the block totals.
template <int KMAX>
__device__ __forceinline__ void block_sum(double (&acc)[KMAX], int K, double *lds /*[KMAX*4]*/) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int k = 0; k < K; ++k) {
    double v = wave_sum(acc[k]);
    if (lane == 0) lds[k * 4 + wid] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < K; ++k) acc[k] = (lds[k * 4 + 0] + lds[k * 4 + 1]) + (lds[k * 4 + 2] + lds[k * 4 + 3]);
  }
  __syncthreads();
}

template <int KMAX>
__device__ __forceinline__ void block_partials(double (&acc)[KMAX], int K, double *partials) {
  __shared__ double lds[KMAX * 4];
  block_sum<KMAX>(acc, K, lds);
  if (threadIdx.x == 0)
    for (int k = 0; k < K; ++k) partials[(size_t)blockIdx.x * K + k] = acc[k];
}

// Prologue: tot[k] = sum_b partials[b*K + k] for k < K, the same fixed order in every
// block (wave w owns k = w, w+4, ...).  tot is shared memory; ends with a barrier.
__device__ __forceinline__ void reduce_partials(const double *__restrict__ partials, int nb, int K, double *tot) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int k = wid; k < K; k += 4) {
    double acc = 0.0;
    for (int b = lane; b < nb; b += 64) acc += partials[(size_t)b * K + k];
    acc = wave_sum(acc);
    if (lane == 0) tot[k] = acc;
  }
  __syncthreads();
}
