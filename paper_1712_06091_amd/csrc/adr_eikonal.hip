// First-arrival travel time on the GPU: the factored eikonal equation (Sec. 1,
// eq. factoredEikonal), |tau0 grad tau1 + tau1 grad tau0|^2 = kappa^2 with tau0 = |x - x0|,
// solved by fixed-point sweeps.  Every sweep recomputes each node's value from its
// neighbours' values of the previous sweep (ping-pong buffers, so the result does not
// depend on the order in which nodes are visited) and keeps the smaller of the old and
// the new value; sweeps continue until one changes nothing.  The paper uses factored
// fast marching, which is sequential; sweeps of a local update are the parallel form.
//
// Local update of node i (r = tau0(x_i), p = grad tau0 at x_i):
//  * per axis k the neighbour j with the smaller tau (the minus side on ties) is upwind
//    unless its tau is still infinite; s_k = +1 for the neighbour at x - h e_k, else -1;
//    the first-order one-sided difference of tau1 towards it makes the k-th component of
//    grad tau A_k T + B_k, A_k = r s_k / h + p_k, B_k = -r s_k tau1_j / h (T = tau1_i);
//  * for a subset S of those axes (components p_k T on the others) the larger root T of
//    sum_S (A_k T + B_k)^2 + sum_{not S} (p_k T)^2 = kappa_i^2 is admissible if T > 0 and on
//    every axis of S the component points away from the neighbour and r T >= tau_j;
//  * the candidate comes from the largest admissible S (smallest T among equal sizes);
//  * it may not exceed min_j (tau_j + 1.1 h max(kappa_i, kappa_j)) over the 2d neighbours
//    (a first arrival is Lipschitz with the local slowness); if it does, or nothing is
//    admissible, the node takes the first-order Godunov update of the unfactored
//    equation, sum over the u smallest upwind values t_k of (T - t_k)^2 = (h kappa_i)^2.
//
// Sums over axes run from the slowest axis (z) to x, and floating-point contraction is
// off in the update, so the arithmetic is exactly that of a plain evaluation of these
// formulas in that order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "../../include/adr.h"
#include "adr_common.hpp"

namespace {

constexpr double kCausalEps = 1e-12;
constexpr double kLipschitz = 1.1;
constexpr int kSweepsPerCheck = 32;

struct EikArgs {
  Grid G;
  double h;
  int src[3];
};

// Value of `a` at the neighbour of node (idx) offset by o along axis k, `fill` outside.
__device__ __forceinline__ double nb_val(const double *a, const Grid &G, int i, const int idx[3], int k, int o,
                                         double fill) {
  const int q = idx[k] + o;
  if (q < 0 || q >= G.n[k]) return fill;
  const int stride = k == 0 ? 1 : (k == 1 ? G.n[0] : G.n[0] * G.n[1]);
  return a[i + o * stride];
}

template <int D>
__device__ double eik_update(const EikArgs &E, const double *__restrict__ kappa2, const double *__restrict__ tin,
                             int i, const int idx[3]) {
#pragma clang fp contract(off)
  const double h = E.h;
  double dx[3];
  double r2 = 0.0;
  for (int k = D - 1; k >= 0; --k) {
    dx[k] = (double)(idx[k] - E.src[k]) * h;
    r2 = r2 + dx[k] * dx[k];
  }
  const double r = sqrt(r2);
  const bool at_src = r == 0.0;
  const double r_safe = at_src ? 1.0 : r;
  const double kap = sqrt(kappa2[i]);
  double p[3];
  for (int k = 0; k < D; ++k) p[k] = at_src ? 0.0 : dx[k] / r_safe;
  // tau1 at a neighbour: tau / tau0 there (kappa at the source).
  auto tau1_of = [&](int k, int o, double tj) -> double {
    double rj2 = 0.0;
    for (int m = D - 1; m >= 0; --m) {
      const double d = (double)(idx[m] + (m == k ? o : 0) - E.src[m]) * h;
      rj2 = rj2 + d * d;
    }
    const double rj = sqrt(rj2);
    if (rj == 0.0) return sqrt(kappa2[i + o * (k == 0 ? 1 : (k == 1 ? E.G.n[0] : E.G.n[0] * E.G.n[1]))]);
    return tj / rj;
  };
  double A[3], B[3], tn[3], sd[3];
  for (int k = 0; k < D; ++k) {
    const double tm = nb_val(tin, E.G, i, idx, k, -1, INFINITY);
    const double tp = nb_val(tin, E.G, i, idx, k, +1, INFINITY);
    const bool minus = tm <= tp;
    const double s = minus ? 1.0 : -1.0;
    const double t = minus ? tm : tp;
    tn[k] = t;
    sd[k] = s;
    A[k] = r * s / h + p[k];
    if (isfinite(t)) {
      const double t1n = tau1_of(k, minus ? -1 : 1, t);
      B[k] = -r * s * t1n / h;
    } else {
      B[k] = 0.0;
    }
  }
  double best = INFINITY;
  int best_size = 0;
  for (int mask = 1; mask < (1 << D); ++mask) {
    int size = 0;
    double qa = 0.0, qb = 0.0, qc = 0.0;
    for (int k = D - 1; k >= 0; --k) {
      if (mask >> k & 1) {
        ++size;
        qa = qa + A[k] * A[k];
        qb = qb + 2.0 * A[k] * B[k];
        qc = qc + B[k] * B[k];
      } else {
        qa = qa + p[k] * p[k];
      }
    }
    qc = qc - kappa2[i];
    const double disc = qb * qb - 4.0 * qa * qc;
    bool ok = disc >= 0.0 && qa > 0.0;
    const double T = (-qb + sqrt(ok ? disc : 0.0)) / (2.0 * qa);
    ok = ok && T > 0.0;
    for (int k = 0; k < D; ++k)
      if (mask >> k & 1) {
        ok = ok && isfinite(tn[k]);
        ok = ok && sd[k] * (A[k] * T + B[k]) >= -kCausalEps * fabs(T);
        ok = ok && r * T >= tn[k];
      }
    if (ok && (size > best_size || (size == best_size && T < best))) {
      best = T;
      best_size = size;
    }
  }
  double cand = isfinite(best) ? r * best : INFINITY;
  // Lipschitz bound over the 2d neighbours; unfactored Godunov fallback.
  double bound = INFINITY;
  for (int k = D - 1; k >= 0; --k)
    for (int o = -1; o <= 1; o += 2) {
      const double tj = nb_val(tin, E.G, i, idx, k, o, INFINITY);
      const double kj = sqrt(nb_val(kappa2, E.G, i, idx, k, o, 0.0));
      bound = fmin(bound, tj + kLipschitz * h * fmax(kap, kj));
    }
  double ts[3];
  for (int k = 0; k < D; ++k) ts[k] = tn[k];
  for (int a = 0; a < D; ++a)
    for (int b = a + 1; b < D; ++b)
      if (ts[b] < ts[a]) {
        const double t = ts[a];
        ts[a] = ts[b];
        ts[b] = t;
      }
  const double f = h * kap;
  double tg = ts[0] + f;
  bool grow = true;
  for (int u = 2; u <= D; ++u) {
    grow = grow && tg > ts[u - 1];
    const double qa = (double)u;
    double sum = 0.0, sq = 0.0;
    for (int k = 0; k < u; ++k) {
      sum = sum + ts[k];
      sq = sq + ts[k] * ts[k];
    }
    const double qb = -2.0 * sum;
    const double qc = sq - f * f;
    const double disc = qb * qb - 4.0 * qa * qc;
    grow = grow && disc >= 0.0;
    const double root = (-qb + sqrt(grow ? disc : 0.0)) / (2.0 * qa);
    if (grow) tg = root;
  }
  if (!isfinite(cand) || cand > bound) cand = tg;
  return cand;
}

template <int D>
__global__ __launch_bounds__(ADR_BLOCK) void k_eikonal_sweep(EikArgs E, const double *__restrict__ kappa2,
                                                             const double *__restrict__ tin,
                                                             double *__restrict__ tout, int *changed, int sweep) {
  const int sidx = E.src[0] + E.G.n[0] * (E.src[1] + E.G.n[1] * E.src[2]);
  int beg, end;
  chunk_range(E.G.N, beg, end);
  bool any = false;
  for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
    const double old = tin[i];
    double v = 0.0;
    if (i != sidx) {
      int idx[3];
      decode(E.G, i, idx[0], idx[1], idx[2]);
      v = fmin(old, eik_update<D>(E, kappa2, tin, i, idx));
    }
    tout[i] = v;
    any |= v != old;
  }
  // Every writer of a sweep stores the same value, sweep + 1.
  if (any) *changed = sweep + 1;
}

__global__ __launch_bounds__(ADR_BLOCK) void k_eikonal_init(int N, int sidx, double *tau, int *changed) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x)
    tau[i] = i == sidx ? 0.0 : INFINITY;
  if (blockIdx.x == 0 && threadIdx.x == 0) *changed = 0;
}

}  // namespace

namespace adrk {
void set_global_error(const std::string &e);   // adr_last_error(NULL) reports it
}

extern "C" {

adr_status adr_eikonal(int ndim, const int *n, double h, const double *kappa2, const int *src, double *tau,
                       double *work, int max_sweeps, int *sweeps, void *stream) {
  if (!n || !kappa2 || !src || !tau || !work || (ndim != 2 && ndim != 3) || !(h > 0) || max_sweeps < 1) {
    adrk::set_global_error("bad argument");
    return ADR_EINVAL;
  }
  EikArgs E{};
  long long N = 1;
  for (int k = 0; k < 3; ++k) {
    E.G.n[k] = k < ndim ? n[k] : 1;
    if (k < ndim && n[k] < 2) {
      adrk::set_global_error("every n[k] must be >= 2");
      return ADR_EINVAL;
    }
    N *= E.G.n[k];
    E.src[k] = k < ndim ? src[k] : 0;
    if (E.src[k] < 0 || E.src[k] >= E.G.n[k]) {
      adrk::set_global_error("source outside the grid");
      return ADR_EINVAL;
    }
  }
  if (N > (1LL << 30)) {
    adrk::set_global_error("grid too large");
    return ADR_EINVAL;
  }
  E.G.N = (int)N;
  E.G.r0 = 1.0 / E.G.n[0];
  E.G.r01 = 1.0 / ((double)E.G.n[0] * E.G.n[1]);
  E.h = h;
  hipStream_t s = (hipStream_t)stream;
  int *changed = (int *)(work + N);
  const int sidx = E.src[0] + E.G.n[0] * (E.src[1] + E.G.n[1] * E.src[2]);
  const int nb = launch_blocks(N);
  hipLaunchKernelGGL(k_eikonal_init, dim3(nb), dim3(ADR_BLOCK), 0, s, (int)N, sidx, tau, changed);
  double *buf[2] = {tau, work};
  int done = 0, last = 0;
  while (done < max_sweeps) {
    const int batch = std::min(kSweepsPerCheck, max_sweeps - done);
    for (int b = 0; b < batch; ++b, ++done) {
      const double *in = buf[done & 1];
      double *out = buf[(done + 1) & 1];
      if (ndim == 2)
        hipLaunchKernelGGL(k_eikonal_sweep<2>, dim3(nb), dim3(ADR_BLOCK), 0, s, E, kappa2, in, out, changed, done);
      else
        hipLaunchKernelGGL(k_eikonal_sweep<3>, dim3(nb), dim3(ADR_BLOCK), 0, s, E, kappa2, in, out, changed, done);
    }
    hipError_t e = hipMemcpyAsync(&last, changed, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      adrk::set_global_error(std::string("HIP error: ") + hipGetErrorString(e));
      return ADR_EHIP;
    }
    if (last < done) break;   // the latest sweep changed nothing
  }
  // The fixed point is in the buffer the last sweep wrote (and, once a sweep has changed
  // nothing, in both); make sure the caller's tau holds it.
  if (done & 1) {
    hipError_t e = hipMemcpyAsync(tau, work, sizeof(double) * N, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      adrk::set_global_error(std::string("HIP error: ") + hipGetErrorString(e));
      return ADR_EHIP;
    }
  }
  if (sweeps) *sweeps = last;
  if (last >= done) {
    adrk::set_global_error("eikonal sweeps reached max_sweeps before a fixed point");
    return ADR_ENOCONV;
  }
  return ADR_OK;
}

}  // extern "C"
