// Factored fast marching for the eikonal equation |grad tau| = kappa on a nodal grid
// (CPU; an input generator for the ADR solver, which takes tau as given).
//
// tau = tau0 * tau1 with tau0 = |x - x0| (Sec. 1, eq. factoredEikonal):
//   |tau0 grad tau1 + tau1 grad tau0|^2 = kappa^2.
// Nodes are accepted in increasing tau from a binary heap.  The update of a node uses,
// per axis, the accepted neighbour with the smaller tau; the one-sided difference of tau1
// towards it is first order, or second order when the next node along that direction is
// accepted too and not later (order = 2).  An axis without an accepted neighbour
// contributes only tau1 * d tau0/dx_k.  The update uses as many axes as give a causal
// root (each used axis' derivative points away from its neighbour and tau does not
// decrease), the smallest such root among sets of that size; a trial value computed
// from more axes replaces one from fewer.  The source node has tau1 = kappa(x0).
//
// Safeguard: a first arrival is Lipschitz, tau_i <= tau_j + h max(kappa_i, kappa_j) for
// every grid neighbour j.  Where the factored update has no causal root, or its root
// exceeds that bound by more than 10% for an accepted neighbour (near caustics, where the
// factored one-sided differences straddle a kink), the node takes the first-order
// Godunov update of the unfactored equation, sum_k (tau - t_k)^2 = (h kappa_i)^2 over
// the smallest accepted neighbour values t_k for which the root stays above them.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <queue>
#include <vector>

namespace {

struct Item {
  double t;
  int64_t i;
  bool operator<(const Item &o) const { return t > o.t; }   // min-heap
};

}  // namespace

extern "C" int fm_factored(int ndim, const int *n /* n[0] = x fastest */, double h, const double *kappa2,
                           const int *src /* per axis, x first */, int order, double *tau_out) {
  if (ndim < 2 || ndim > 3 || h <= 0) return 1;
  const int D = ndim;
  int64_t stride[3] = {1, n[0], (int64_t)n[0] * n[1]};
  int64_t N = 1;
  for (int k = 0; k < D; ++k) N *= n[k];
  std::vector<double> t1(N, INFINITY);      // tau1
  std::vector<uint8_t> state(N, 0);         // 0 far, 1 trial, 2 accepted
  std::vector<uint8_t> axes(N, 0);          // number of axes behind the current trial value
  int64_t s = 0;
  for (int k = 0; k < D; ++k) {
    if (src[k] < 0 || src[k] >= n[k]) return 2;
    s += src[k] * stride[k];
  }
  auto coords = [&](int64_t i, int c[3]) {
    int64_t r = i;
    for (int k = D - 1; k >= 0; --k) {
      c[k] = (int)(r / stride[k]);
      r -= (int64_t)c[k] * stride[k];
    }
  };
  auto tau0 = [&](const int c[3]) {
    double r2 = 0;
    for (int k = 0; k < D; ++k) {
      double d = (c[k] - src[k]) * h;
      r2 += d * d;
    }
    return std::sqrt(r2);
  };
  std::priority_queue<Item> heap;
  t1[s] = std::sqrt(kappa2[s]);
  state[s] = 2;

  // Local update of node i: returns the new tau1 (INFINITY if none) and the number of
  // axes it used.
  int used_axes = 0;
  auto update = [&](int64_t i) -> double {
    used_axes = 0;
    int c[3];
    coords(i, c);
    const double r = tau0(c);
    double p[3];
    for (int k = 0; k < D; ++k) p[k] = (c[k] - src[k]) * h / r;
    const double k2 = kappa2[i];
    // Per axis candidate: coefficients of the axis term A T + B and its side sign.
    double A[3], B[3], side[3], tn[3];
    bool has[3];
    for (int k = 0; k < D; ++k) {
      has[k] = false;
      double best = INFINITY;
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        const int q = c[k] + sgn;
        if (q < 0 || q >= n[k]) continue;
        const int64_t j = i + sgn * stride[k];
        if (state[j] != 2) continue;
        int cj[3] = {c[0], c[1], c[2]};
        cj[k] = q;
        const double tj = tau0(cj) * t1[j];
        if (tj < best) {
          best = tj;
          has[k] = true;
          // neighbour at x - h (sgn = -1): backward difference, s = +1
          const double sd = (sgn < 0) ? 1.0 : -1.0;
          side[k] = sd;
          tn[k] = tj;
          const int q2 = c[k] + 2 * sgn;
          bool second = false;
          if (order >= 2 && q2 >= 0 && q2 < n[k]) {
            const int64_t j2 = i + 2 * sgn * stride[k];
            if (state[j2] == 2) {
              int c2[3] = {c[0], c[1], c[2]};
              c2[k] = q2;
              second = tau0(c2) * t1[j2] <= tj;
              if (second) {
                A[k] = r * sd * 1.5 / h + p[k];
                B[k] = -r * sd * (4.0 * t1[j] - t1[j2]) / (2.0 * h);
              }
            }
          }
          if (!second) {
            A[k] = r * sd / h + p[k];
            B[k] = -r * sd * t1[j] / h;
          }
        }
      }
    }
    // Prefer the largest set of axes with a causal root (dropping an axis assumes
    // d tau1/dx_k = 0 there, which is only a fallback); smallest root within a size.
    double bestT = INFINITY;
    for (int size = D; size >= 1 && !(bestT < INFINITY); --size) {
      for (int mask = 1; mask < (1 << D); ++mask) {
        if (__builtin_popcount(mask) != size) continue;
        bool ok = true;
        for (int k = 0; k < D; ++k)
          if ((mask >> k & 1) && !has[k]) ok = false;
        if (!ok) continue;
        double a = 0, b = 0, cc = -k2;
        for (int k = 0; k < D; ++k) {
          const double Ak = (mask >> k & 1) ? A[k] : p[k];
          const double Bk = (mask >> k & 1) ? B[k] : 0.0;
          a += Ak * Ak;
          b += 2 * Ak * Bk;
          cc += Bk * Bk;
        }
        const double disc = b * b - 4 * a * cc;
        if (disc < 0 || a <= 0) continue;
        const double T = (-b + std::sqrt(disc)) / (2 * a);
        if (!(T > 0)) continue;
        bool causal = true;
        for (int k = 0; k < D; ++k)
          if (mask >> k & 1) {
            const double deriv = A[k] * T + B[k];   // d tau / d x_k
            if (deriv * side[k] < -1e-12 * std::fabs(T)) causal = false;
            if (r * T < tn[k]) causal = false;
          }
        if (causal && T < bestT) {
          bestT = T;
          used_axes = size;
        }
      }
    }
    return bestT;
  };

  // Unfactored first-order Godunov update of node i from its accepted neighbours, and the
  // Lipschitz bound min_j (tau_j + 1.1 h max(kappa_i, kappa_j)) over them.
  auto godunov = [&](int64_t i, double &bound) -> double {
    int c[3];
    coords(i, c);
    double tk[3];
    int m = 0;
    bound = INFINITY;
    const double ki = std::sqrt(kappa2[i]);
    for (int k = 0; k < D; ++k) {
      double best = INFINITY;
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        const int q = c[k] + sgn;
        if (q < 0 || q >= n[k]) continue;
        const int64_t j = i + sgn * stride[k];
        if (state[j] != 2) continue;
        int cj[3] = {c[0], c[1], c[2]};
        cj[k] = q;
        const double tj = (j == s) ? 0.0 : tau0(cj) * t1[j];
        best = std::fmin(best, tj);
        bound = std::fmin(bound, tj + 1.1 * h * std::fmax(ki, std::sqrt(kappa2[j])));
      }
      if (best < INFINITY) tk[m++] = best;
    }
    if (m == 0) return INFINITY;
    std::sort(tk, tk + m);
    const double f = h * ki;
    double T = tk[0] + f;
    for (int u = 2; u <= m; ++u) {
      if (T <= tk[u - 1]) break;
      // sum_{k<u} (T - t_k)^2 = f^2
      double a = u, b = 0, cc = -f * f;
      for (int k = 0; k < u; ++k) {
        b -= 2 * tk[k];
        cc += tk[k] * tk[k];
      }
      const double disc = b * b - 4 * a * cc;
      if (disc < 0) break;
      T = (-b + std::sqrt(disc)) / (2 * a);
    }
    return T;
  };

  auto push_neighbours = [&](int64_t i) {
    int c[3];
    coords(i, c);
    for (int k = 0; k < D; ++k)
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        const int q = c[k] + sgn;
        if (q < 0 || q >= n[k]) continue;
        const int64_t j = i + sgn * stride[k];
        if (state[j] == 2) continue;
        int cj[3] = {c[0], c[1], c[2]};
        cj[k] = q;
        const double rj = tau0(cj);
        double T = update(j);
        double bound;
        const double tg = godunov(j, bound);
        if (!(T < INFINITY) || rj * T > bound) {
          T = tg / rj;
          used_axes = D;
        }
        // A value from more axes replaces one from fewer (a one-axis factored update can
        // under-estimate); among equal axis counts the smaller value wins.  Whatever stays
        // must respect the bound from the neighbours accepted so far, so every node
        // ends within it of each neighbour accepted before it.
        bool changed = false;
        if (T < INFINITY && (used_axes > axes[j] || (used_axes == axes[j] && T < t1[j]))) {
          t1[j] = T;
          axes[j] = (uint8_t)used_axes;
          changed = true;
        }
        if (rj * t1[j] > bound) {
          t1[j] = tg / rj;
          axes[j] = (uint8_t)D;
          changed = true;
        }
        if (changed) {
          state[j] = 1;
          heap.push(Item{rj * t1[j], j});
        }
      }
  };
  push_neighbours(s);
  while (!heap.empty()) {
    Item it = heap.top();
    heap.pop();
    if (state[it.i] == 2) continue;
    int c[3];
    coords(it.i, c);
    if (std::fabs(it.t - tau0(c) * t1[it.i]) > 1e-15 * (1 + it.t)) continue;   // stale entry
    state[it.i] = 2;
    push_neighbours(it.i);
  }
  for (int64_t i = 0; i < N; ++i) {
    int c[3];
    coords(i, c);
    tau_out[i] = (i == s) ? 0.0 : tau0(c) * t1[i];
  }
  return 0;
}
