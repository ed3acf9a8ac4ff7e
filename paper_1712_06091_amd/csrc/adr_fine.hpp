// Fine-level ADR operator row, computed on the fly from per-node coefficients.
//
// Row j of A_beta (Sec. 2.2-2.3; eq. precADRup):
//   sum_k (a_{j-e_k} - 2 a_j + a_{j+e_k}) / h^2          Laplacian (ghost-node rows on
//                                                         faces, eq. BCADR)
//   - 2 i w sum_k g_k (D_k^beta a)_j                      advection, eq. londUpwindDiff
//   - i w L_j avg(a)_j                                    averaging mass of Sec. 2.3
//   + c_j a_j                                             reaction
// D_k^beta = (1-beta) D^{2up} + beta D^{1up}; backward formulas where g_k >= 0, forward
// where g_k < 0; central differences (eq. londDiff) within one node (Chebyshev distance)
// of the source.  Where an upwind stencil would leave the grid: one node short -> both
// orders use the first-order formula; two short (face node, g pointing inwards) -> the
// inward one-sided formulas of the same orders.  avg(a) is the mean of the 2d axis
// neighbours inside and a_j on the faces.  Ghost node on the low face of axis k:
// a_{-1} = a_1 - 2 h i w g_k a_0; on the high face a_n = a_{n-2} + 2 h i w g_k a_{n-1}.
//
// Entries: e[0] = centre; for axis k, e[1+4k+{0,1,2,3}] = offsets -2, -1, +1, +2.
// An entry whose neighbour lies outside the grid is exactly zero.
#pragma once
#include "adr_common.hpp"

template <typename T>
struct FineCoef {
  const T *g[3];   // d tau / d x_k, one plane per axis
  const T *L;      // Lap tau
  const cx<T> *c;  // reaction
};

struct FineParams {
  double h, omega, beta;
  int src[3];      // source node; src[0] < 0: no near-source rule
  int central;     // 1: central advection (eq. londDiff) off the faces of each axis
};

// Shift the coefficient planes to the launch's problem of a shot group (see Shot).
template <typename T>
__device__ __forceinline__ void shift_fine_coef(FineCoef<T> &C, long long off) {
#pragma unroll
  for (int k = 0; k < 3; ++k) C.g[k] = shot_ptr(C.g[k], off);
  C.L = shot_ptr(C.L, off);
  C.c = shot_ptr(C.c, off);
}

template <typename T, int D>
__device__ __forceinline__ void fine_row(const Grid &G, const FineParams &P, int idx[3], const T gk[3],
                                         T L, cx<T> c, cx<T> (&e)[1 + 4 * D]) {
  const T h = (T)P.h, w = (T)P.omega, beta = (T)P.beta;
  const T ih = T(1) / h, ih2 = ih * ih;
  bool on_face = false;
  bool near = P.src[0] >= 0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    on_face |= (idx[k] == 0) | (idx[k] == G.n[k] - 1);
    int dk = idx[k] - P.src[k];
    near &= (dk >= -1) & (dk <= 1);
  }
  T cre = c.re, cim = c.im;
  // Mass term: on faces it multiplies a_j, inside the neighbours' mean.
  const T mass_nb = on_face ? T(0) : -w * L * (T(1) / T(2 * D));
  if (on_face) cim += -w * L;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const int i = idx[k], n = G.n[k];
    const T g = gk[k];
    const bool low = (i == 0), high = (i == n - 1);
    // Laplacian
    T lm1 = (low ? T(0) : (high ? T(2) * ih2 : ih2));
    T lp1 = (high ? T(0) : (low ? T(2) * ih2 : ih2));
    cre += T(-2) * ih2;
    if (low) cim += T(-2) * w * g * ih;
    if (high) cim += T(2) * w * g * ih;
    // Advection weights for offsets -2..+2 (real), scaled by -2 w g into the imaginary part.
    T d_m2 = 0, d_m1 = 0, d_0 = 0, d_p1 = 0, d_p2 = 0;
    if (near || (P.central && !low && !high)) {
      d_m1 = T(-0.5) * ih;
      d_p1 = T(0.5) * ih;
    } else {
      const bool backward = (g >= T(0));
      // mode: 0 = second-order backward, 1 = first-order backward,
      //       2 = second-order forward,  3 = first-order forward
      int mode;
      if (backward) mode = (i >= 2) ? 0 : ((i == 1) ? 1 : 2);
      else mode = (i <= n - 3) ? 2 : ((i == n - 2) ? 3 : 0);
      const T a2 = T(1) - beta;
      if (mode == 0) {
        d_0 = a2 * T(1.5) * ih + beta * ih;
        d_m1 = a2 * T(-2) * ih - beta * ih;
        d_m2 = a2 * T(0.5) * ih;
      } else if (mode == 1) {
        d_0 = ih;
        d_m1 = -ih;
      } else if (mode == 2) {
        d_0 = a2 * T(-1.5) * ih - beta * ih;
        d_p1 = a2 * T(2) * ih + beta * ih;
        d_p2 = a2 * T(-0.5) * ih;
      } else {
        d_0 = -ih;
        d_p1 = ih;
      }
    }
    const T s = T(-2) * w * g;
    cim += s * d_0;
    e[1 + 4 * k + 0] = mk<T>(T(0), s * d_m2);
    e[1 + 4 * k + 1] = mk<T>(lm1, s * d_m1 + (i > 0 ? mass_nb : T(0)));
    e[1 + 4 * k + 2] = mk<T>(lp1, s * d_p1 + (i < n - 1 ? mass_nb : T(0)));
    e[1 + 4 * k + 3] = mk<T>(T(0), s * d_p2);
  }
  e[0] = mk<T>(cre, cim);
}

// Neighbour linear offsets for the fine row (clamped to the centre where the neighbour
// is outside the grid; the matching entry is zero there).
template <int D>
__device__ __forceinline__ void fine_neighbours(const Grid &G, int i, int idx[3], int (&nb)[1 + 4 * D]) {
  nb[0] = i;
  int stride = 1;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const int p = idx[k], n = G.n[k];
    nb[1 + 4 * k + 0] = (p >= 2) ? i - 2 * stride : i;
    nb[1 + 4 * k + 1] = (p >= 1) ? i - stride : i;
    nb[1 + 4 * k + 2] = (p <= n - 2) ? i + stride : i;
    nb[1 + 4 * k + 3] = (p <= n - 3) ? i + 2 * stride : i;
    stride *= n;
  }
}

template <typename T, int D>
__device__ __forceinline__ void load_fine_coef(const FineCoef<T> &C, int i, T (&gk)[3], T &L, cx<T> &c) {
#pragma unroll
  for (int k = 0; k < 3; ++k) gk[k] = (k < D) ? C.g[k][i] : T(0);
  L = C.L[i];
  c = C.c[i];
}

// Off-diagonal entry of the fine row of node j (index idx, coefficients gk, L) towards its
// neighbour at offset o in {-2, -1, +1, +2} along axis k -- the same value fine_row puts
// in e[1 + 4k + {0,1,2,3}].  Used by the conjugate-transposed (adjoint) operator, which
// gathers, for each node i, the entries of the neighbours' rows that point back to i.
template <typename T, int D>
__device__ __forceinline__ cx<T> fine_offdiag(const Grid &G, const FineParams &P, const int idx[3], const T gk[3],
                                              T L, int k, int o) {
  const T h = (T)P.h, w = (T)P.omega, beta = (T)P.beta;
  const T ih = T(1) / h, ih2 = ih * ih;
  bool on_face = false;
  bool near = P.src[0] >= 0;
#pragma unroll
  for (int m = 0; m < D; ++m) {
    on_face |= (idx[m] == 0) | (idx[m] == G.n[m] - 1);
    const int dm = idx[m] - P.src[m];
    near &= (dm >= -1) & (dm <= 1);
  }
  const int i = idx[k], n = G.n[k];
  const T g = gk[k];
  const bool low = (i == 0), high = (i == n - 1);
  T lap = 0;
  if (o == -1) lap = low ? T(0) : (high ? T(2) * ih2 : ih2);
  if (o == 1) lap = high ? T(0) : (low ? T(2) * ih2 : ih2);
  T d = 0;
  if (near || (P.central && !low && !high)) {
    if (o == -1) d = T(-0.5) * ih;
    if (o == 1) d = T(0.5) * ih;
  } else {
    const bool backward = (g >= T(0));
    int mode;
    if (backward) mode = (i >= 2) ? 0 : ((i == 1) ? 1 : 2);
    else mode = (i <= n - 3) ? 2 : ((i == n - 2) ? 3 : 0);
    const T a2 = T(1) - beta;
    if (mode == 0) {
      if (o == -1) d = a2 * T(-2) * ih - beta * ih;
      if (o == -2) d = a2 * T(0.5) * ih;
    } else if (mode == 1) {
      if (o == -1) d = -ih;
    } else if (mode == 2) {
      if (o == 1) d = a2 * T(2) * ih + beta * ih;
      if (o == 2) d = a2 * T(-0.5) * ih;
    } else {
      if (o == 1) d = ih;
    }
  }
  T im = T(-2) * w * g * d;
  if (!on_face && (o == -1 || o == 1)) im += -w * L * (T(1) / T(2 * D));
  return mk<T>(lap, im);
}
