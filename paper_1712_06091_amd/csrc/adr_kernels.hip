// HIP kernels of the ADR amplitude solver for gfx950 (MI355X).
//
// Everything here is bandwidth-bound stencil or vector work: coalesced SoA planes,
// one node per lane, contiguous per-block chunks remapped per XCD, and deterministic
// fused reductions (no MFMA: there is no dense contraction on this path).
#include "adr_kernels.hpp"

#include <cmath>
#include <cstdio>

namespace adrk {

thread_local ShotLaunch g_shot;

// Launch of a group-capable kernel: the GRP = true instance with one y-slice of blocks per
// problem of the current shot group, else the plain instance.
template <typename F, typename... Args>
inline void launch_g(F k_single, F k_group, int nblocks, hipStream_t s, Args... args) {
  if (g_shot.count > 1)
    hipLaunchKernelGGL(k_group, dim3(nblocks, g_shot.count), dim3(ADR_BLOCK), 0, s, args..., g_shot.sh);
  else
    hipLaunchKernelGGL(k_single, dim3(nblocks), dim3(ADR_BLOCK), 0, s, args..., Shot{0, nullptr});
}

#define ADR_LAUNCH(kernel, nblocks, stream, ...) \
  hipLaunchKernelGGL(kernel, dim3(nblocks), dim3(ADR_BLOCK), 0, stream, __VA_ARGS__)

// =====================================================================================
// Setup: coefficients from tau (Sec. 2.1, eq. travel_time_coeff)
// =====================================================================================
template <int D>
__global__ __launch_bounds__(ADR_BLOCK) void k_coefficients(Grid G, double h, double omega, int sx, int sy, int sz,
                                                            double w2r, const double *__restrict__ kappa2,
                                                            const double *__restrict__ tau,
                                                            const double *__restrict__ gamma, double *g0,
                                                            double *g1, double *g2, double *Lout,
                                                            cx<double> *cout) {
  int beg, end;
  chunk_range(G.N, beg, end);
  const int src[3] = {sx, sy, sz};
  const bool fact = sx >= 0;
  const int stride[3] = {1, G.n[0], G.n[0] * G.n[1]};
  const int srcidx = fact ? sx + G.n[0] * (sy + G.n[1] * sz) : -1;
  // tau1 at the source (0/0 there): the mean of tau / h over its 2D axis neighbours, a
  // function of tau alone, so kappa2 enters the operator only through the reaction.
  double ksrc = 0.0;
  if (fact) {
    for (int k = 0; k < D; ++k) ksrc += tau[srcidx - stride[k]] / h + tau[srcidx + stride[k]] / h;
    ksrc /= (double)(2 * D);
  }
  for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
    int idx[3];
    decode(G, i, idx[0], idx[1], idx[2]);
    // f(k, o): tau1 (factored) or tau at the node shifted by o along axis k.
    auto f = [&](int k, int o) -> double {
      const int j = i + o * stride[k];
      if (!fact) return tau[j];
      if (j == srcidx) return ksrc;
      double r2 = 0.0;
#pragma unroll
      for (int m = 0; m < D; ++m) {
        double dm = (double)(idx[m] + (m == k ? o : 0) - src[m]) * h;
        r2 += dm * dm;
      }
      return tau[j] / sqrt(r2);
    };
    double d1[3] = {0, 0, 0}, d2sum = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const int p = idx[k], n = G.n[k];
      double a, b2;
      if (p == 0) {
        const double f0 = f(k, 0), f1 = f(k, 1), f2 = f(k, 2), f3 = f(k, 3);
        a = (f1 - f0) / h;
        b2 = (2.0 * f0 - 5.0 * f1 + 4.0 * f2 - f3) / (h * h);
      } else if (p == n - 1) {
        const double f0 = f(k, 0), f1 = f(k, -1), f2 = f(k, -2), f3 = f(k, -3);
        a = (f0 - f1) / h;
        b2 = (2.0 * f0 - 5.0 * f1 + 4.0 * f2 - f3) / (h * h);
      } else {
        const double fm = f(k, -1), f0 = f(k, 0), fp = f(k, 1);
        a = (fp - fm) / (2.0 * h);
        b2 = (fp - 2.0 * f0 + fm) / (h * h);
      }
      d1[k] = a;
      d2sum += b2;
    }
    double g[3] = {0, 0, 0}, L;
    if (!fact) {
      for (int k = 0; k < D; ++k) g[k] = d1[k];
      L = d2sum;
    } else if (i == srcidx) {
      L = 0.0;
      for (int k = 0; k < D; ++k)
        L += (tau[i + stride[k]] - 2.0 * tau[i] + tau[i - stride[k]]) / (h * h);
    } else {
      double r2 = 0.0, dt0[3] = {0, 0, 0};
      for (int k = 0; k < D; ++k) {
        double dk = (double)(idx[k] - src[k]) * h;
        dt0[k] = dk;
        r2 += dk * dk;
      }
      const double r = sqrt(r2);
      const double t1 = tau[i] / r;
      double dot = 0.0;
      for (int k = 0; k < D; ++k) {
        dt0[k] /= r;
        g[k] = r * d1[k] + t1 * dt0[k];
        dot += dt0[k] * d1[k];
      }
      L = t1 * (double)(D - 1) / r + 2.0 * dot + r * d2sum;
    }
    double gg = 0.0;
    for (int k = 0; k < D; ++k) gg += g[k] * g[k];
    const double k2 = kappa2[i];
    const double gam = gamma ? gamma[i] : 0.0;
    g0[i] = g[0];
    g1[i] = g[1];
    if (D == 3) g2[i] = g[2];
    Lout[i] = L;
    cout[i] = mk<double>(w2r * (k2 - gg), -omega * gam * k2);
  }
}

void coefficients(hipStream_t s, const Grid &G, int D, double h, double omega, const int src[3],
                  bool numerical_reaction, const double *kappa2, const double *tau, const double *gamma, double *g0,
                  double *g1, double *g2, double *L, cx<double> *c) {
  int nb = launch_blocks(G.N);
  const double w2r = numerical_reaction ? omega * omega : 0.0;
  if (D == 2)
    ADR_LAUNCH(k_coefficients<2>, nb, s, G, h, omega, src[0], src[1], src[2], w2r, kappa2, tau, gamma, g0, g1, g2, L,
               c);
  else
    ADR_LAUNCH(k_coefficients<3>, nb, s, G, h, omega, src[0], src[1], src[2], w2r, kappa2, tau, gamma, g0, g1, g2, L,
               c);
}

// =====================================================================================
// Setup: materialize the fine stencil (for the Galerkin product) and Galerkin A_c
// =====================================================================================
template <int D>
__global__ __launch_bounds__(ADR_BLOCK) void k_fine_stencil(Grid G, FineCoef<double> C, FineParams P,
                                                            cx<double> *planes) {
  int beg, end;
  chunk_range(G.N, beg, end);
  for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
    int idx[3];
    decode(G, i, idx[0], idx[1], idx[2]);
    double gk[3], L;
    cx<double> c;
    load_fine_coef<double, D>(C, i, gk, L, c);
    cx<double> e[1 + 4 * D];
    fine_row<double, D>(G, P, idx, gk, L, c, e);
#pragma unroll
    for (int p = 0; p < 1 + 4 * D; ++p) planes[(size_t)p * G.N + i] = e[p];
  }
}

void fine_stencil(hipStream_t s, const Grid &G, int D, const FineCoef<double> &C, const FineParams &P,
                  cx<double> *planes) {
  int nb = launch_blocks(G.N);
  if (D == 2) ADR_LAUNCH(k_fine_stencil<2>, nb, s, G, C, P, planes);
  else ADR_LAUNCH(k_fine_stencil<3>, nb, s, G, C, P, planes);
}

// A_c[t][J] = sum over (p, d, w) in the triple list of t of
//             w * A_f[d][2J + p]        (fine node 2J+p and its neighbour in the grid)
// where the list pairs each P^T support offset p with each input stencil offset d that
// lands on the P support of coarse node J + t, w = w(p) w(q) (eq. coarseGridMatrix).
__global__ __launch_bounds__(ADR_BLOCK) void k_galerkin(Grid Gf, Grid Gc, const cx<double> *__restrict__ in,
                                                        const int *__restrict__ in_off, cx<double> *out, const int *__restrict__ out_off, int S_out,
                                                        const int *__restrict__ tri_start,
                                                        const int *__restrict__ tri_p,
                                                        const int *__restrict__ tri_d,
                                                        const double *__restrict__ tri_w) {
  const long long total = (long long)S_out * Gc.N;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (long long)gridDim.x * blockDim.x) {
    const int t = (int)(q / Gc.N);
    const int J = (int)(q - (long long)t * Gc.N);
    int jc[3];
    decode(Gc, J, jc[0], jc[1], jc[2]);
    const int tx = out_off[3 * t], ty = out_off[3 * t + 1], tz = out_off[3 * t + 2];
    const int Ix = jc[0] + tx, Iy = jc[1] + ty, Iz = jc[2] + tz;
    cx<double> acc = mk<double>(0.0, 0.0);
    if (Ix >= 0 && Ix < Gc.n[0] && Iy >= 0 && Iy < Gc.n[1] && Iz >= 0 && Iz < Gc.n[2]) {
      for (int e = tri_start[t]; e < tri_start[t + 1]; ++e) {
        const int fx = 2 * jc[0] + tri_p[3 * e], fy = 2 * jc[1] + tri_p[3 * e + 1], fz = 2 * jc[2] + tri_p[3 * e + 2];
        if (fx < 0 || fx >= Gf.n[0] || fy < 0 || fy >= Gf.n[1] || fz < 0 || fz >= Gf.n[2]) continue;
        const int d = tri_d[e];
        const int gx = fx + in_off[3 * d], gy = fy + in_off[3 * d + 1], gz = fz + in_off[3 * d + 2];
        if (gx < 0 || gx >= Gf.n[0] || gy < 0 || gy >= Gf.n[1] || gz < 0 || gz >= Gf.n[2]) continue;
        const int f = fx + Gf.n[0] * (fy + Gf.n[1] * fz);
        const cx<double> a = in[(size_t)d * Gf.N + f];
        acc.re += tri_w[e] * a.re;
        acc.im += tri_w[e] * a.im;
      }
    }
    out[(size_t)t * Gc.N + J] = acc;
  }
}

void galerkin(hipStream_t s, const Grid &Gf, const Grid &Gc, const cx<double> *in_planes, const int *in_off_xyz,
              int S_in, cx<double> *out_planes, const int *out_off_xyz, int S_out, const int *tri_start,
              const int *tri_p, const int *tri_d, const double *tri_w) {
  (void)S_in;
  long long total = (long long)S_out * Gc.N;
  long long nb = (total + ADR_BLOCK - 1) / ADR_BLOCK;
  if (nb > 65536) nb = 65536;
  ADR_LAUNCH(k_galerkin, (int)nb, s, Gf, Gc, in_planes, in_off_xyz, out_planes,
             out_off_xyz, S_out, tri_start, tri_p, tri_d, tri_w);
}

template <typename T>
__global__ __launch_bounds__(ADR_BLOCK) void k_diag_inv(int N, const cx<T> *c, cx<T> *d) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) d[i] = cinv(c[i]);
}
template <typename T>
void stencil_diag_inv(hipStream_t s, int N, const cx<T> *centre_plane, cx<T> *dinv) {
  ADR_LAUNCH(k_diag_inv<T>, launch_blocks(N), s, N, centre_plane, dinv);
}
template void stencil_diag_inv<double>(hipStream_t, int, const cx<double> *, cx<double> *);
template void stencil_diag_inv<float>(hipStream_t, int, const cx<float> *, cx<float> *);

template <typename To, typename Ti, bool GRP>
__global__ __launch_bounds__(ADR_BLOCK) void k_convert(long long n, const cx<Ti> *in, cx<To> *out, Shot sh) {
  ADR_SHOT_ENTER(sh);
  ADR_SHOT_N(sh, n);
  ADR_SHIFT(in);
  ADR_SHIFT(out);
  ADR_SHOT_LIVE(sh);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = cvt<To, Ti>(in[i]);
}
template <typename To, typename Ti>
void convert(hipStream_t s, long long n, const cx<Ti> *in, cx<To> *out) {
  launch_g(k_convert<To, Ti, false>, k_convert<To, Ti, true>, launch_blocks(n), s, n, in, out);
}
template void convert<float, double>(hipStream_t, long long, const cx<double> *, cx<float> *);
template void convert<double, float>(hipStream_t, long long, const cx<float> *, cx<double> *);
template void convert<double, double>(hipStream_t, long long, const cx<double> *, cx<double> *);

template <typename To, typename Ti>
__global__ __launch_bounds__(ADR_BLOCK) void k_convert_real(long long n, const Ti *in, To *out) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = (To)in[i];
}
template <typename To, typename Ti>
void convert_real(hipStream_t s, long long n, const Ti *in, To *out) {
  ADR_LAUNCH((k_convert_real<To, Ti>), launch_blocks(n), s, n, in, out);
}
template void convert_real<float, double>(hipStream_t, long long, const double *, float *);

// =====================================================================================
// Fine level: matrix-free apply / residual with fused reductions, Jacobi sweep
// =====================================================================================
template <typename T, typename Tin, typename To, int D, int NV, bool NORM, bool GRP>
__global__ __launch_bounds__(ADR_BLOCK) void k_fine_apply(Grid G, FineCoef<T> C, FineParams P,
                                                          const cx<Tin> *__restrict__ x,
                                                          const cx<To> *__restrict__ b, cx<To> *__restrict__ y,
                                                          int mode, VecSet<To> V, double *pout,
                                                          const FineParams *Pd, Shot sh) {
  ADR_SHOT_ENTER(sh);
  ADR_SHOT_GRID(sh, G);
  if constexpr (GRP) shift_fine_coef(C, shot_off_);
  if constexpr (GRP) {
    if (Pd) P = *shot_ptr(Pd, shot_off_);
  }
  ADR_SHIFT(x);
  ADR_SHIFT(b);
  ADR_SHIFT(y);
  if constexpr (GRP) shift_set<NV>(V, shot_off_);
  ADR_SHIFT(pout);
  ADR_SHOT_LIVE(sh);
  constexpr int K = 2 * NV + (NORM ? 1 : 0);
  constexpr int KA = K > 0 ? K : 1;
  double red[KA];
#pragma unroll
  for (int k = 0; k < KA; ++k) red[k] = 0.0;
  int beg, end;
  chunk_range(G.N, beg, end);
  for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
    int idx[3];
    decode(G, i, idx[0], idx[1], idx[2]);
    // Gathers first, so that their latency overlaps the row computation.
    int nb[1 + 4 * D];
    fine_neighbours<D>(G, i, idx, nb);
    cx<Tin> xv[1 + 4 * D];
#pragma unroll
    for (int p = 0; p < 1 + 4 * D; ++p) xv[p] = x[nb[p]];
    T gk[3], L;
    cx<T> c;
    load_fine_coef<T, D>(C, i, gk, L, c);
    cx<T> e[1 + 4 * D];
    fine_row<T, D>(G, P, idx, gk, L, c, e);
    cx<T> acc = mk<T>(T(0), T(0));
#pragma unroll
    for (int p = 0; p < 1 + 4 * D; ++p) acc = cfma(e[p], cvt<T, Tin>(xv[p]), acc);
    cx<To> o = cvt<To, T>(acc);
    if (mode == 1) o = b[i] - o;
    y[i] = o;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const cx<To> vv = V.v[v][i];
      const cx<double> d = cdotc(cvt<double, To>(vv), cvt<double, To>(o));
      red[2 * v] += d.re;
      red[2 * v + 1] += d.im;
    }
    if (NORM) red[K - 1] += (double)o.re * o.re + (double)o.im * o.im;
  }
  if (K > 0) block_partials<KA>(red, K, pout);
}

template <typename T, typename Tin, typename To, int D, int NV, bool NORM>
static void launch_fine_apply(hipStream_t s, int nb, const Grid &G, const FineCoef<T> &C, const FineParams &P,
                              const cx<Tin> *x, const cx<To> *b, cx<To> *y, int mode, const VecSet<To> &V,
                              double *pout, const FineParams *Pd) {
  launch_g(k_fine_apply<T, Tin, To, D, NV, NORM, false>, k_fine_apply<T, Tin, To, D, NV, NORM, true>, nb, s, G, C, P, x, b, y, mode, V, pout, Pd);
}

template <typename T, typename Tin, typename To, int D, bool NORM>
static void dispatch_fine_apply_nv(hipStream_t s, int nb, const Grid &G, const FineCoef<T> &C,
                                   const FineParams &P, const cx<Tin> *x, const cx<To> *b, cx<To> *y, int mode,
                                   const VecSet<To> &V, double *pout, const FineParams *Pd) {
  switch (V.count) {
#define ADR_NV_CASE(n) \
  case n: launch_fine_apply<T, Tin, To, D, n, NORM>(s, nb, G, C, P, x, b, y, mode, V, pout, Pd); break;
    ADR_NV_CASE(0) ADR_NV_CASE(1) ADR_NV_CASE(2) ADR_NV_CASE(3) ADR_NV_CASE(4) ADR_NV_CASE(5) ADR_NV_CASE(6)
    ADR_NV_CASE(7) ADR_NV_CASE(8)
#undef ADR_NV_CASE
    default: break;
  }
}

template <typename T, typename Tin, typename To>
int fine_apply(hipStream_t s, const Grid &G, int D, const FineCoef<T> &C, const FineParams &P, const cx<Tin> *x,
               const cx<To> *b, cx<To> *y, int mode, const VecSet<To> *dots, bool want_norm, double *pout,
               const FineParams *Pd) {
  VecSet<To> V{};
  if (dots) V = *dots;
  const bool red = want_norm || V.count > 0;
  const int nb = red ? launch_blocks_red(G.N) : launch_blocks_wide(G.N);
  if (D == 2) {
    if (want_norm) dispatch_fine_apply_nv<T, Tin, To, 2, true>(s, nb, G, C, P, x, b, y, mode, V, pout, Pd);
    else dispatch_fine_apply_nv<T, Tin, To, 2, false>(s, nb, G, C, P, x, b, y, mode, V, pout, Pd);
  } else {
    if (want_norm) dispatch_fine_apply_nv<T, Tin, To, 3, true>(s, nb, G, C, P, x, b, y, mode, V, pout, Pd);
    else dispatch_fine_apply_nv<T, Tin, To, 3, false>(s, nb, G, C, P, x, b, y, mode, V, pout, Pd);
  }
  return nb;
}
template int fine_apply<double, double, double>(hipStream_t, const Grid &, int, const FineCoef<double> &,
                                                const FineParams &, const cx<double> *, const cx<double> *,
                                                cx<double> *, int, const VecSet<double> *, bool, double *,
                                                const FineParams *);
template int fine_apply<double, float, double>(hipStream_t, const Grid &, int, const FineCoef<double> &,
                                               const FineParams &, const cx<float> *, const cx<double> *,
                                               cx<double> *, int, const VecSet<double> *, bool, double *,
                                               const FineParams *);
template int fine_apply<float, float, float>(hipStream_t, const Grid &, int, const FineCoef<float> &,
                                             const FineParams &, const cx<float> *, const cx<float> *,
                                             cx<float> *, int, const VecSet<float> *, bool, double *,
                                             const FineParams *);

// HASX = false: the sweep starts from x = 0 (no gathers).  A compile-time flag, because a
// run-time test around the gathers makes the compiler wait for all of them at the join
// before it issues the coefficient loads.
template <typename T, int D, bool HASX, bool GRP>
__global__ __launch_bounds__(ADR_BLOCK) void k_fine_jacobi(Grid G, FineCoef<T> C, FineParams P,
                                                           const cx<T> *__restrict__ xin,
                                                           const cx<T> *__restrict__ b, cx<T> *__restrict__ xout,
                                                           T weight, const FineParams *Pd, Shot sh) {
  ADR_SHOT_ENTER(sh);
  ADR_SHOT_GRID(sh, G);
  if constexpr (GRP) shift_fine_coef(C, shot_off_);
  if constexpr (GRP) {
    if (Pd) P = *shot_ptr(Pd, shot_off_);
  }
  ADR_SHIFT(xin);
  ADR_SHIFT(b);
  ADR_SHIFT(xout);
  ADR_SHOT_LIVE(sh);
  int beg, end;
  chunk_range(G.N, beg, end);
  for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
    T gk[3], L;
    cx<T> c;
    load_fine_coef<T, D>(C, i, gk, L, c);
    const cx<T> bi = b[i];
    int idx[3];
    decode(G, i, idx[0], idx[1], idx[2]);
    cx<T> xv[1 + 4 * D];
    if constexpr (HASX) {
      int nb[1 + 4 * D];
      fine_neighbours<D>(G, i, idx, nb);
#pragma unroll
      for (int p = 0; p < 1 + 4 * D; ++p) xv[p] = xin[nb[p]];
    }
    cx<T> e[1 + 4 * D];
    fine_row<T, D>(G, P, idx, gk, L, c, e);
    cx<T> r = bi;
    cx<T> x0 = mk<T>(T(0), T(0));
    if constexpr (HASX) {
      cx<T> acc = mk<T>(T(0), T(0));
#pragma unroll
      for (int p = 0; p < 1 + 4 * D; ++p) acc = cfma(e[p], xv[p], acc);
      r = r - acc;
      x0 = xv[0];
    }
    xout[i] = cfma(weight * cinv(e[0]), r, x0);
  }
}

template <typename T>
void fine_jacobi(hipStream_t s, const Grid &G, int D, const FineCoef<T> &C, const FineParams &P, const cx<T> *x_in,
                 const cx<T> *b, cx<T> *x_out, double weight, const FineParams *Pd) {
  int nb = launch_blocks_wide(G.N);
  if (x_in) {
    if (D == 2)
      launch_g(k_fine_jacobi<T, 2, true, false>, k_fine_jacobi<T, 2, true, true>, nb, s, G, C, P, x_in, b, x_out,
               (T)weight, Pd);
    else
      launch_g(k_fine_jacobi<T, 3, true, false>, k_fine_jacobi<T, 3, true, true>, nb, s, G, C, P, x_in, b, x_out,
               (T)weight, Pd);
  } else {
    if (D == 2)
      launch_g(k_fine_jacobi<T, 2, false, false>, k_fine_jacobi<T, 2, false, true>, nb, s, G, C, P, x_in, b, x_out,
               (T)weight, Pd);
    else
      launch_g(k_fine_jacobi<T, 3, false, false>, k_fine_jacobi<T, 3, false, true>, nb, s, G, C, P, x_in, b, x_out,
               (T)weight, Pd);
  }
}
// -------------------------------------------------------------------------------------
// LDS z-marching on the matrix-free finest level (3D, FP32): Jacobi sweeps from a given
// iterate and the V-cycle residual.  A block owns a segment of kFineSeg consecutive
// in-plane nodes and a slab of z-planes.  The 13-point row reads x at the node, at +-1 and
// +-2 along x and y (all inside the plane window: the segment and 2 rows either side) and
// at +-1, +-2 along z (only the segment of those planes).  So LDS holds the plane window of
// the current plane (double-buffered: the next plane's is loaded during this one) and a
// ring of six plane segments (z-2..z+3); the node's coefficients and right-hand side are
// also loaded a plane ahead.  One barrier per plane.  The row arithmetic is fine_row's, in
// the same order as the one-lane kernels, so the results are the same.
// -------------------------------------------------------------------------------------
constexpr int kFineSeg = ADR_BLOCK;
constexpr int kFineMaxN0 = 257;
constexpr int kFineWin = kFineSeg + 4 * kFineMaxN0;
constexpr int kFineMinPlanes = 16;

int fine_lds_blocks(const Grid &G, int D) {
  if (D != 3 || G.n[0] > kFineMaxN0 || G.n[2] < kFineMinPlanes) return 0;
  const int nseg = (G.n[0] * G.n[1] + kFineSeg - 1) / kFineSeg;
  int nslab = G.n[2] / kFineMinPlanes;
  const int cap = 4096 / nseg;
  if (nslab > cap) nslab = cap;
  if (nslab < 1) nslab = 1;
  return nseg * nslab;
}

// MODE 0: Jacobi sweep out = x + w D^{-1} (b - A x); MODE 1: residual out = b - A x.
template <typename T, int MODE, bool GRP>
__global__ __launch_bounds__(ADR_BLOCK) void k_fine_lds(Grid G, FineCoef<T> C, FineParams P,
                                                        const cx<T> *__restrict__ xin, const cx<T> *__restrict__ b,
                                                        cx<T> *__restrict__ out, T weight, const FineParams *Pd,
                                                        Shot sh) {
  ADR_SHOT_ENTER(sh);
  if constexpr (GRP) shift_fine_coef(C, shot_off_);
  if constexpr (GRP) {
    if (Pd) P = *shot_ptr(Pd, shot_off_);
  }
  ADR_SHIFT(xin);
  ADR_SHIFT(b);
  ADR_SHIFT(out);
  ADR_SHOT_LIVE(sh);
  constexpr int D = 3;
  __shared__ cx<T> ring[6][kFineSeg];
  __shared__ cx<T> cwin[2][kFineWin];
  const int n0 = G.n[0], nxy = G.n[0] * G.n[1], n2 = G.n[2];
  const int nseg = (nxy + kFineSeg - 1) / kFineSeg;
  const int nslab = gridDim.x / nseg;
  const int lb = logical_block();
  const int seg = lb % nseg, slab = lb / nseg;
  const int z0 = (int)((long long)n2 * slab / nslab), z1 = (int)((long long)n2 * (slab + 1) / nslab);
  const int s0 = seg * kFineSeg;
  const int halo = 2 * n0;
  const int W = kFineSeg + 2 * halo;
  const int tid = threadIdx.x;
  constexpr int RW = (kFineWin + ADR_BLOCK - 1) / ADR_BLOCK;
  auto xval = [&](int zp, int q) -> cx<T> {
    return (zp >= 0 && zp < n2 && q >= 0 && q < nxy) ? xin[(size_t)zp * nxy + q] : mk<T>(T(0), T(0));
  };
  auto load_win = [&](int zp, cx<T> (&reg)[RW]) {
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int w = tid + r * ADR_BLOCK;
      reg[r] = w < W ? xval(zp, s0 - halo + w) : mk<T>(T(0), T(0));
    }
  };
  auto store_win = [&](int buf, const cx<T> (&reg)[RW]) {
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int w = tid + r * ADR_BLOCK;
      if (w < W) cwin[buf][w] = reg[r];
    }
  };
  // Preload: segments of planes z0-2 .. z0+2 and the window of plane z0.
  for (int zp = z0 - 2; zp <= z0 + 2; ++zp) ring[(zp + 6) % 6][tid] = xval(zp, s0 + tid);
  {
    cx<T> reg[RW];
    load_win(z0, reg);
    store_win(z0 & 1, reg);
  }
  __syncthreads();
  const int ip = s0 + tid;
  const bool act = ip < nxy;
  const int base = tid + halo;
  // The node's coefficients and right-hand side are loaded one plane ahead too, so that a
  // plane's arithmetic waits on LDS only and every global load of the step overlaps it.
  auto load_cb = [&](int zp, T (&g)[3], T &l, cx<T> &cc, cx<T> &bb) {
    if (act && zp < z1) {
      const int i = zp * nxy + ip;
      load_fine_coef<T, D>(C, i, g, l, cc);
      bb = b[i];
    }
  };
  T gk[3] = {T(0), T(0), T(0)}, L = T(0);
  cx<T> c = mk<T>(T(0), T(0)), bi = c;
  load_cb(z0, gk, L, c, bi);
  for (int z = z0; z < z1; ++z) {
    // Next plane's window, coefficients and right-hand side and the segment of plane
    // z + 3, in flight during this plane.
    cx<T> reg[RW];
    load_win(z + 1, reg);
    const cx<T> seg3 = xval(z + 3, s0 + tid);
    T gn[3] = {T(0), T(0), T(0)}, Ln = T(0);
    cx<T> cn = mk<T>(T(0), T(0)), bn = cn;
    load_cb(z + 1, gn, Ln, cn, bn);
    if (act) {
      const int i = z * nxy + ip;
      int idx[3];
      idx[0] = ip % n0;
      idx[1] = ip / n0;
      idx[2] = z;
      // x at the 13 stencil nodes in fine_neighbours' order: centre, then per axis
      // offsets -2, -1, +1, +2.
      const cx<T> *cw = cwin[z & 1];
      cx<T> xv[1 + 4 * D];
      xv[0] = cw[base];
      xv[1] = cw[base - 2];
      xv[2] = cw[base - 1];
      xv[3] = cw[base + 1];
      xv[4] = cw[base + 2];
      xv[5] = cw[base - 2 * n0];
      xv[6] = cw[base - n0];
      xv[7] = cw[base + n0];
      xv[8] = cw[base + 2 * n0];
      xv[9] = ring[(z - 2 + 6) % 6][tid];
      xv[10] = ring[(z - 1 + 6) % 6][tid];
      xv[11] = ring[(z + 1) % 6][tid];
      xv[12] = ring[(z + 2) % 6][tid];
      cx<T> e[1 + 4 * D];
      fine_row<T, D>(G, P, idx, gk, L, c, e);
      cx<T> acc = mk<T>(T(0), T(0));
#pragma unroll
      for (int p = 0; p < 1 + 4 * D; ++p) acc = cfma(e[p], xv[p], acc);
      const cx<T> r = bi - acc;
      if constexpr (MODE == 0) out[i] = cfma(weight * cinv(e[0]), r, xv[0]);
      else out[i] = r;
    }
    store_win((z + 1) & 1, reg);
    ring[(z + 3) % 6][tid] = seg3;
#pragma unroll
    for (int k = 0; k < 3; ++k) gk[k] = gn[k];
    L = Ln;
    c = cn;
    bi = bn;
    __syncthreads();
  }
}

template <typename T>
bool fine_lds(hipStream_t s, const Grid &G, int D, const FineCoef<T> &C, const FineParams &P, const cx<T> *x,
              const cx<T> *b, cx<T> *out, int mode, double weight, const FineParams *Pd) {
  if constexpr (sizeof(T) != 4) {
    return false;
  } else {
    // The tiles' geometry follows the launch's own grid: not in merged-shape groups.
    const int nb = g_shot.sh.grid ? 0 : fine_lds_blocks(G, D);
    if (nb == 0 || !x) return false;
    if (mode == 0)
      launch_g(k_fine_lds<T, 0, false>, k_fine_lds<T, 0, true>, nb, s, G, C, P, x, b, out, (T)weight, Pd);
    else
      launch_g(k_fine_lds<T, 1, false>, k_fine_lds<T, 1, true>, nb, s, G, C, P, x, b, out, (T)weight, Pd);
    return true;
  }
}
template bool fine_lds<float>(hipStream_t, const Grid &, int, const FineCoef<float> &, const FineParams &,
                              const cx<float> *, const cx<float> *, cx<float> *, int, double, const FineParams *);
template bool fine_lds<double>(hipStream_t, const Grid &, int, const FineCoef<double> &, const FineParams &,
                               const cx<double> *, const cx<double> *, cx<double> *, int, double,
                               const FineParams *);

template void fine_jacobi<double>(hipStream_t, const Grid &, int, const FineCoef<double> &, const FineParams &,
                                  const cx<double> *, const cx<double> *, cx<double> *, double, const FineParams *);
template void fine_jacobi<float>(hipStream_t, const Grid &, int, const FineCoef<float> &, const FineParams &,
                                 const cx<float> *, const cx<float> *, cx<float> *, double, const FineParams *);

// The coarse stencil set: offsets with |d_k| <= 2 and at most one |d_k| == 2, ordered
// dz-major then dy then dx (81 points in 3D, 21 in 2D).  Compile-time table so that the
// fully unrolled apply has constant offsets.
template <int D>
struct OffTable {
  int dx[81], dy[81], dz[81];
};
template <int D>
__host__ __device__ constexpr OffTable<D> make_off_table() {
  OffTable<D> t{};
  int c = 0;
  for (int z = (D == 3 ? -2 : 0); z <= (D == 3 ? 2 : 0); ++z)
    for (int y = -2; y <= 2; ++y)
      for (int x = -2; x <= 2; ++x) {
        const int twos = (x == 2 || x == -2) + (y == 2 || y == -2) + (z == 2 || z == -2);
        if (twos > 1) continue;
        t.dx[c] = x;
        t.dy[c] = y;
        t.dz[c] = z;
        ++c;
      }
  return t;
}

// =====================================================================================
// Fine level, conjugate-transposed operator A^H (adjoint solves)
// =====================================================================================
// (A^H x)_i = conj(A_ii) x_i + sum over neighbours j = i - o e_k of conj(A_{j, j + o e_k}) x_j:
// the entries of the neighbours' rows that point back to node i.  Returns the sum and
// conj(A_ii) (the adjoint diagonal).
template <typename T, typename Tin, int D>
__device__ __forceinline__ cx<T> fine_adjoint_row(const Grid &G, const FineCoef<T> &C, const FineParams &P, int i,
                                                  const int idx[3], const cx<Tin> *__restrict__ x, cx<T> &dconj) {
  T gk[3], L;
  cx<T> c;
  load_fine_coef<T, D>(C, i, gk, L, c);
  cx<T> e[1 + 4 * D];
  int id[3] = {idx[0], idx[1], idx[2]};
  fine_row<T, D>(G, P, id, gk, L, c, e);
  dconj = mk<T>(e[0].re, -e[0].im);
  cx<T> acc = dconj * cvt<T, Tin>(x[i]);
  int stride = 1;
#pragma unroll
  for (int k = 0; k < D; ++k) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int o = (q < 2) ? q - 2 : q - 1;   // -2, -1, +1, +2
      const int pj = idx[k] - o;
      if (pj < 0 || pj >= G.n[k]) continue;
      const int j = i - o * stride;
      int jdx[3] = {idx[0], idx[1], idx[2]};
      jdx[k] = pj;
      T gj[3];
#pragma unroll
      for (int m = 0; m < 3; ++m) gj[m] = (m == k) ? C.g[k][j] : T(0);
      const cx<T> a = fine_offdiag<T, D>(G, P, jdx, gj, C.L[j], k, o);
      acc = cfma(mk<T>(a.re, -a.im), cvt<T, Tin>(x[j]), acc);
    }
    stride *= G.n[k];
  }
  return acc;
}

template <typename T, typename Tin, typename To, int D, int NV, bool NORM>
__global__ __launch_bounds__(ADR_BLOCK) void k_fine_apply_adj(Grid G, FineCoef<T> C, FineParams P,
                                                              const cx<Tin> *__restrict__ x,
                                                              const cx<To> *__restrict__ b, cx<To> *__restrict__ y,
                                                              int mode, VecSet<To> V, double *pout) {
  constexpr int K = 2 * NV + (NORM ? 1 : 0);
  constexpr int KA = K > 0 ? K : 1;
  double red[KA];
#pragma unroll
  for (int k = 0; k < KA; ++k) red[k] = 0.0;
  int beg, end;
  chunk_range(G.N, beg, end);
  for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
    int idx[3];
    decode(G, i, idx[0], idx[1], idx[2]);
    cx<T> dc;
    const cx<T> acc = fine_adjoint_row<T, Tin, D>(G, C, P, i, idx, x, dc);
    cx<To> o = cvt<To, T>(acc);
    if (mode == 1) o = b[i] - o;
    y[i] = o;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const cx<double> d = cdotc(cvt<double, To>(V.v[v][i]), cvt<double, To>(o));
      red[2 * v] += d.re;
      red[2 * v + 1] += d.im;
    }
    if (NORM) red[K - 1] += (double)o.re * o.re + (double)o.im * o.im;
  }
  if (K > 0) block_partials<KA>(red, K, pout);
}

template <typename T, typename Tin, typename To, int D, bool NORM>
static void dispatch_fine_adj_nv(hipStream_t s, int nb, const Grid &G, const FineCoef<T> &C, const FineParams &P,
                                 const cx<Tin> *x, const cx<To> *b, cx<To> *y, int mode, const VecSet<To> &V,
                                 double *pout) {
  switch (V.count) {
#define ADR_NV_CASE(n) \
  case n: ADR_LAUNCH((k_fine_apply_adj<T, Tin, To, D, n, NORM>), nb, s, G, C, P, x, b, y, mode, V, pout); break;
    ADR_NV_CASE(0) ADR_NV_CASE(1) ADR_NV_CASE(2) ADR_NV_CASE(3) ADR_NV_CASE(4) ADR_NV_CASE(5) ADR_NV_CASE(6)
    ADR_NV_CASE(7) ADR_NV_CASE(8)
#undef ADR_NV_CASE
    default: break;
  }
}

template <typename T, typename Tin, typename To>
int fine_apply_adj(hipStream_t s, const Grid &G, int D, const FineCoef<T> &C, const FineParams &P, const cx<Tin> *x,
                   const cx<To> *b, cx<To> *y, int mode, const VecSet<To> *dots, bool want_norm, double *pout) {
  VecSet<To> V{};
  if (dots) V = *dots;
  const bool red = want_norm || V.count > 0;
  const int nb = red ? launch_blocks_red(G.N) : launch_blocks_wide(G.N);
  if (D == 2) {
    if (want_norm) dispatch_fine_adj_nv<T, Tin, To, 2, true>(s, nb, G, C, P, x, b, y, mode, V, pout);
    else dispatch_fine_adj_nv<T, Tin, To, 2, false>(s, nb, G, C, P, x, b, y, mode, V, pout);
  } else {
    if (want_norm) dispatch_fine_adj_nv<T, Tin, To, 3, true>(s, nb, G, C, P, x, b, y, mode, V, pout);
    else dispatch_fine_adj_nv<T, Tin, To, 3, false>(s, nb, G, C, P, x, b, y, mode, V, pout);
  }
  return nb;
}
template int fine_apply_adj<double, double, double>(hipStream_t, const Grid &, int, const FineCoef<double> &,
                                                    const FineParams &, const cx<double> *, const cx<double> *,
                                                    cx<double> *, int, const VecSet<double> *, bool, double *);
template int fine_apply_adj<double, float, double>(hipStream_t, const Grid &, int, const FineCoef<double> &,
                                                   const FineParams &, const cx<float> *, const cx<double> *,
                                                   cx<double> *, int, const VecSet<double> *, bool, double *);
template int fine_apply_adj<float, float, float>(hipStream_t, const Grid &, int, const FineCoef<float> &,
                                                 const FineParams &, const cx<float> *, const cx<float> *,
                                                 cx<float> *, int, const VecSet<float> *, bool, double *);

// x_out = x_in + w conj(A_ii)^{-1} (b - A^H x_in); x_in NULL means zero.
template <typename T, int D>
__global__ __launch_bounds__(ADR_BLOCK) void k_fine_jacobi_adj(Grid G, FineCoef<T> C, FineParams P,
                                                               const cx<T> *__restrict__ xin,
                                                               const cx<T> *__restrict__ b, cx<T> *__restrict__ xout,
                                                               T weight) {
  int beg, end;
  chunk_range(G.N, beg, end);
  for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
    int idx[3];
    decode(G, i, idx[0], idx[1], idx[2]);
    cx<T> r = b[i], x0 = mk<T>(T(0), T(0)), dc;
    if (xin) {
      const cx<T> acc = fine_adjoint_row<T, T, D>(G, C, P, i, idx, xin, dc);
      r = r - acc;
      x0 = xin[i];
    } else {
      T gk[3], L;
      cx<T> c;
      load_fine_coef<T, D>(C, i, gk, L, c);
      cx<T> e[1 + 4 * D];
      fine_row<T, D>(G, P, idx, gk, L, c, e);
      dc = mk<T>(e[0].re, -e[0].im);
    }
    xout[i] = cfma(weight * cinv(dc), r, x0);
  }
}
template <typename T>
void fine_jacobi_adj(hipStream_t s, const Grid &G, int D, const FineCoef<T> &C, const FineParams &P,
                     const cx<T> *x_in, const cx<T> *b, cx<T> *x_out, double weight) {
  int nb = launch_blocks_wide(G.N);
  if (D == 2) ADR_LAUNCH((k_fine_jacobi_adj<T, 2>), nb, s, G, C, P, x_in, b, x_out, (T)weight);
  else ADR_LAUNCH((k_fine_jacobi_adj<T, 3>), nb, s, G, C, P, x_in, b, x_out, (T)weight);
}
template void fine_jacobi_adj<double>(hipStream_t, const Grid &, int, const FineCoef<double> &, const FineParams &,
                                      const cx<double> *, const cx<double> *, cx<double> *, double);
template void fine_jacobi_adj<float>(hipStream_t, const Grid &, int, const FineCoef<float> &, const FineParams &,
                                     const cx<float> *, const cx<float> *, cx<float> *, double);

// Conjugate transpose of a Galerkin level: AH[t][i] = conj(A[-t][i + t]) (zero when i + t
// is outside the grid).  The offset set is symmetric and ordered so that -t is plane
// S-1-t.
template <typename T, int D>
__global__ __launch_bounds__(ADR_BLOCK) void k_adjoint_planes(Grid G, const cx<T> *__restrict__ A,
                                                              cx<T> *__restrict__ AH) {
  constexpr int S = D == 3 ? 81 : 21;
  constexpr OffTable<D> OT = make_off_table<D>();
  const long long total = (long long)S * G.N;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (long long)gridDim.x * blockDim.x) {
    const int t = (int)(q / G.N), i = (int)(q - (long long)t * G.N);
    int ix, iy, iz;
    decode(G, i, ix, iy, iz);
    int dx = 0, dy = 0, dz = 0;
#pragma unroll
    for (int p = 0; p < S; ++p)
      if (p == t) {
        dx = OT.dx[p];
        dy = OT.dy[p];
        dz = OT.dz[p];
      }
    const int jx = ix + dx, jy = iy + dy, jz = iz + dz;
    cx<T> v = mk<T>(T(0), T(0));
    if (jx >= 0 && jx < G.n[0] && jy >= 0 && jy < G.n[1] && jz >= 0 && jz < G.n[2]) {
      const cx<T> a = A[(size_t)(S - 1 - t) * G.N + jx + G.n[0] * (jy + G.n[1] * jz)];
      v = mk<T>(a.re, -a.im);
    }
    AH[(size_t)t * G.N + i] = v;
  }
}
template <typename T>
void adjoint_planes(hipStream_t s, const Grid &G, int D, const cx<T> *A, cx<T> *AH) {
  long long total = (long long)(D == 3 ? 81 : 21) * G.N;
  long long nb = (total + ADR_BLOCK - 1) / ADR_BLOCK;
  if (nb > 65536) nb = 65536;
  if (D == 2) ADR_LAUNCH((k_adjoint_planes<T, 2>), (int)nb, s, G, A, AH);
  else ADR_LAUNCH((k_adjoint_planes<T, 3>), (int)nb, s, G, A, AH);
}
template void adjoint_planes<double>(hipStream_t, const Grid &, int, const cx<double> *, cx<double> *);
template void adjoint_planes<float>(hipStream_t, const Grid &, int, const cx<float> *, cx<float> *);

// grad[i] += -Re(conj(lam_i) c'_i a_i): the derivative of a receiver misfit with respect to
// kappa^2_i at fixed travel time, given the forward amplitude a and the adjoint state lam
// (dH_2up / dkappa2_i = c'_i e_i e_i^T, c'_i = w2r - i w gamma_i with w2r = w^2 when the
// reaction keeps w^2 kappa^2, 0 when the eikonal equation removed it).
__global__ __launch_bounds__(ADR_BLOCK) void k_grad_kappa2(int N, double omega, double w2r,
                                                           const double *__restrict__ gamma,
                                                           const cx<double> *__restrict__ a,
                                                           const cx<double> *__restrict__ lam, double *grad) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    const double gm = gamma ? gamma[i] : 0.0;
    const cx<double> t = cdotc(lam[i], mk<double>(w2r, -omega * gm) * a[i]);
    grad[i] -= t.re;
  }
}
void grad_kappa2(hipStream_t s, int N, double omega, bool numerical_reaction, const double *gamma,
                 const cx<double> *a, const cx<double> *lam, double *grad) {
  const double w2r = numerical_reaction ? omega * omega : 0.0;
  ADR_LAUNCH(k_grad_kappa2, launch_blocks(N), s, N, omega, w2r, gamma, a, lam, grad);
}

// Receivers: r_k = u[idx_k] - d_k; adjoint source s = sum_k e_{idx_k} r_k (s is zeroed
// first; one lane adds the receivers in order, so repeated indices accumulate
// deterministically).
__global__ __launch_bounds__(ADR_BLOCK) void k_receiver_residual(int nrec, const int *__restrict__ idx,
                                                                 const cx<double> *__restrict__ u,
                                                                 const cx<double> *__restrict__ d,
                                                                 cx<double> *__restrict__ r) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nrec; k += gridDim.x * blockDim.x)
    r[k] = u[idx[k]] - d[k];
}
void receiver_residual(hipStream_t s, int nrec, const int *idx, const cx<double> *u, const cx<double> *d,
                       cx<double> *r) {
  hipLaunchKernelGGL(k_receiver_residual, dim3((nrec + ADR_BLOCK - 1) / ADR_BLOCK), dim3(ADR_BLOCK), 0, s, nrec, idx,
                     u, d, r);
}
template <bool GRP>
__global__ __launch_bounds__(ADR_BLOCK) void k_zero(long long n, cx<double> *x, Shot sh) {
  ADR_SHOT_ENTER(sh);
  ADR_SHOT_N(sh, n);
  ADR_SHIFT(x);
  ADR_SHOT_LIVE(sh);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    x[i] = mk<double>(0.0, 0.0);
}
__global__ void k_scatter_add(int nrec, const int *__restrict__ idx, const cx<double> *__restrict__ r,
                              cx<double> *__restrict__ s) {
  // One lane walks the receivers in order so repeated indices add deterministically.
  if (blockIdx.x == 0 && threadIdx.x == 0)
    for (int k = 0; k < nrec; ++k) s[idx[k]] = s[idx[k]] + r[k];
}
void adjoint_source(hipStream_t s, int N, int nrec, const int *idx, const cx<double> *r, cx<double> *src) {
  launch_g(k_zero<false>, k_zero<true>, launch_blocks(N), s, (long long)N, src);
  hipLaunchKernelGGL(k_scatter_add, dim3(1), dim3(64), 0, s, nrec, idx, r, src);
}
void zero(hipStream_t s, long long n, cx<double> *x) { launch_g(k_zero<false>, k_zero<true>, launch_blocks(n), s, n, x); }
template <bool GRP>
__global__ __launch_bounds__(ADR_BLOCK) void k_copy(long long n, const cx<double> *in, cx<double> *out, Shot sh) {
  ADR_SHOT_ENTER(sh);
  ADR_SHOT_N(sh, n);
  ADR_SHIFT(in);
  ADR_SHIFT(out);
  ADR_SHOT_LIVE(sh);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = in[i];
}
void copy(hipStream_t s, long long n, const cx<double> *in, cx<double> *out) {
  launch_g(k_copy<false>, k_copy<true>, launch_blocks(n), s, n, in, out);
}

// =====================================================================================
// Rescaled fine operator B = M A M^{-1} with M = diag(exp(-i w tau)) (Sec. 3.2,
// eq. ADRcenRescaled): with ph = exp(i w tau), row j of B is
// conj(ph_j) sum_k A_jk ph_k x_k, and its diagonal is A's.  The multigrid cycle of the
// second stage of Alg. ADRlong works on B (shifted), so that its coarse levels are
// Galerkin products of B.
// =====================================================================================
__global__ __launch_bounds__(ADR_BLOCK) void k_phase_plane(long long n, const double *__restrict__ tau, double omega,
                                                           cx<double> *__restrict__ ph) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    double sn, cs;
    sincos(omega * tau[i], &sn, &cs);
    ph[i] = mk<double>(cs, sn);
  }
}
void phase_plane(hipStream_t s, long long n, const double *tau, double omega, cx<double> *ph) {
  ADR_LAUNCH(k_phase_plane, launch_blocks(n), s, n, tau, omega, ph);
}

// out = conj(ph) in (conj != 0) or ph in; in and out may alias.
template <typename Ti, typename To>
__global__ __launch_bounds__(ADR_BLOCK) void k_mul_phase(long long n, const cx<Ti> *in, const cx<double> *__restrict__ ph,
                                                         int conj, cx<To> *out) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const cx<double> p = ph[i];
    const cx<double> v = cvt<double, Ti>(in[i]);
    out[i] = cvt<To, double>(conj ? cdotc(p, v) : p * v);
  }
}
template <typename Ti, typename To>
void mul_phase(hipStream_t s, long long n, const cx<Ti> *in, const cx<double> *ph, bool conj, cx<To> *out) {
  ADR_LAUNCH((k_mul_phase<Ti, To>), launch_blocks(n), s, n, in, ph, conj ? 1 : 0, out);
}
template void mul_phase<double, double>(hipStream_t, long long, const cx<double> *, const cx<double> *, bool,
                                        cx<double> *);
template void mul_phase<double, float>(hipStream_t, long long, const cx<double> *, const cx<double> *, bool,
                                       cx<float> *);
template void mul_phase<float, double>(hipStream_t, long long, const cx<float> *, const cx<double> *, bool,
                                       cx<double> *);
template void mul_phase<float, float>(hipStream_t, long long, const cx<float> *, const cx<double> *, bool,
                                      cx<float> *);

// planes[p][j] *= conj(ph_j) ph_{nb_p(j)} for the 1 + 4D planes of the fine stencil (the
// entries towards neighbours outside the grid are zero and stay zero).
template <int D>
__global__ __launch_bounds__(ADR_BLOCK) void k_stencil_rescale(Grid G, cx<double> *planes,
                                                               const cx<double> *__restrict__ ph) {
  int beg, end;
  chunk_range(G.N, beg, end);
  for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
    int idx[3];
    decode(G, i, idx[0], idx[1], idx[2]);
    int nb[1 + 4 * D];
    fine_neighbours<D>(G, i, idx, nb);
    const cx<double> pj = ph[i];
#pragma unroll
    for (int p = 1; p < 1 + 4 * D; ++p) {
      cx<double> &e = planes[(size_t)p * G.N + i];
      e = cdotc(pj, ph[nb[p]] * e);
    }
  }
}
void stencil_rescale(hipStream_t s, const Grid &G, int D, cx<double> *planes, const cx<double> *ph) {
  int nb = launch_blocks(G.N);
  if (D == 2) ADR_LAUNCH(k_stencil_rescale<2>, nb, s, G, planes, ph);
  else ADR_LAUNCH(k_stencil_rescale<3>, nb, s, G, planes, ph);
}

// Damped Jacobi on B (x_in NULL: from zero), and the residual r = b - B x.
template <typename T, int D, bool HASX>
__global__ __launch_bounds__(ADR_BLOCK) void k_fine_jacobi_ph(Grid G, FineCoef<T> C, FineParams P,
                                                              const cx<T> *__restrict__ ph,
                                                              const cx<T> *__restrict__ xin,
                                                              const cx<T> *__restrict__ b, cx<T> *__restrict__ xout,
                                                              T weight) {
  int beg, end;
  chunk_range(G.N, beg, end);
  for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
    T gk[3], L;
    cx<T> c;
    load_fine_coef<T, D>(C, i, gk, L, c);
    const cx<T> bi = b[i];
    const cx<T> pi = ph[i];
    int idx[3];
    decode(G, i, idx[0], idx[1], idx[2]);
    cx<T> xv[1 + 4 * D], pv[1 + 4 * D];
    if constexpr (HASX) {
      int nb[1 + 4 * D];
      fine_neighbours<D>(G, i, idx, nb);
#pragma unroll
      for (int p = 0; p < 1 + 4 * D; ++p) {
        xv[p] = xin[nb[p]];
        pv[p] = ph[nb[p]];
      }
    }
    cx<T> e[1 + 4 * D];
    fine_row<T, D>(G, P, idx, gk, L, c, e);
    cx<T> r = bi;
    cx<T> x0 = mk<T>(T(0), T(0));
    if constexpr (HASX) {
      cx<T> acc = mk<T>(T(0), T(0));
#pragma unroll
      for (int p = 0; p < 1 + 4 * D; ++p) acc = cfma(e[p], pv[p] * xv[p], acc);
      r = r - cdotc(pi, acc);
      x0 = xv[0];
    }
    xout[i] = cfma(weight * cinv(e[0]), r, x0);
  }
}
template <typename T, int D>
__global__ __launch_bounds__(ADR_BLOCK) void k_fine_residual_ph(Grid G, FineCoef<T> C, FineParams P,
                                                                const cx<T> *__restrict__ ph,
                                                                const cx<T> *__restrict__ x,
                                                                const cx<T> *__restrict__ b, cx<T> *__restrict__ r) {
  int beg, end;
  chunk_range(G.N, beg, end);
  for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
    T gk[3], L;
    cx<T> c;
    load_fine_coef<T, D>(C, i, gk, L, c);
    const cx<T> bi = b[i];
    const cx<T> pi = ph[i];
    int idx[3];
    decode(G, i, idx[0], idx[1], idx[2]);
    int nb[1 + 4 * D];
    fine_neighbours<D>(G, i, idx, nb);
    cx<T> xv[1 + 4 * D], pv[1 + 4 * D];
#pragma unroll
    for (int p = 0; p < 1 + 4 * D; ++p) {
      xv[p] = x[nb[p]];
      pv[p] = ph[nb[p]];
    }
    cx<T> e[1 + 4 * D];
    fine_row<T, D>(G, P, idx, gk, L, c, e);
    cx<T> acc = mk<T>(T(0), T(0));
#pragma unroll
    for (int p = 0; p < 1 + 4 * D; ++p) acc = cfma(e[p], pv[p] * xv[p], acc);
    r[i] = bi - cdotc(pi, acc);
  }
}
template <typename T>
void fine_jacobi_ph(hipStream_t s, const Grid &G, int D, const FineCoef<T> &C, const FineParams &P, const cx<T> *ph,
                    const cx<T> *x_in, const cx<T> *b, cx<T> *x_out, double weight) {
  int nb = launch_blocks(G.N);
  if (x_in) {
    if (D == 2) ADR_LAUNCH((k_fine_jacobi_ph<T, 2, true>), nb, s, G, C, P, ph, x_in, b, x_out, (T)weight);
    else ADR_LAUNCH((k_fine_jacobi_ph<T, 3, true>), nb, s, G, C, P, ph, x_in, b, x_out, (T)weight);
  } else {
    if (D == 2) ADR_LAUNCH((k_fine_jacobi_ph<T, 2, false>), nb, s, G, C, P, ph, x_in, b, x_out, (T)weight);
    else ADR_LAUNCH((k_fine_jacobi_ph<T, 3, false>), nb, s, G, C, P, ph, x_in, b, x_out, (T)weight);
  }
}
template <typename T>
void fine_residual_ph(hipStream_t s, const Grid &G, int D, const FineCoef<T> &C, const FineParams &P,
                      const cx<T> *ph, const cx<T> *x, const cx<T> *b, cx<T> *r) {
  int nb = launch_blocks(G.N);
  if (D == 2) ADR_LAUNCH((k_fine_residual_ph<T, 2>), nb, s, G, C, P, ph, x, b, r);
  else ADR_LAUNCH((k_fine_residual_ph<T, 3>), nb, s, G, C, P, ph, x, b, r);
}
template void fine_jacobi_ph<double>(hipStream_t, const Grid &, int, const FineCoef<double> &, const FineParams &,
                                     const cx<double> *, const cx<double> *, const cx<double> *, cx<double> *,
                                     double);
template void fine_jacobi_ph<float>(hipStream_t, const Grid &, int, const FineCoef<float> &, const FineParams &,
                                    const cx<float> *, const cx<float> *, const cx<float> *, cx<float> *, double);
template void fine_residual_ph<double>(hipStream_t, const Grid &, int, const FineCoef<double> &,
                                       const FineParams &, const cx<double> *, const cx<double> *,
                                       const cx<double> *, cx<double> *);
template void fine_residual_ph<float>(hipStream_t, const Grid &, int, const FineCoef<float> &, const FineParams &,
                                      const cx<float> *, const cx<float> *, const cx<float> *, cx<float> *);

// =====================================================================================
// Coarse levels: stored Galerkin stencils (SoA planes)
// =====================================================================================
// Clamped neighbour index tables of node i along each axis (offsets -2..2), as linear
// index contributions.
template <int D>
__device__ __forceinline__ void coarse_neighbours(const Grid &G, int i, int (&X)[5], int (&Y)[5], int (&Z)[5]) {
  int ix, iy, iz;
  decode(G, i, ix, iy, iz);
  const int sy = G.n[0], sz = G.n[0] * G.n[1];
#pragma unroll
  for (int d = -2; d <= 2; ++d) {
    X[d + 2] = min(max(ix + d, 0), G.n[0] - 1);
    Y[d + 2] = sy * min(max(iy + d, 0), G.n[1] - 1);
    Z[d + 2] = (D == 3) ? sz * min(max(iz + d, 0), G.n[2] - 1) : 0;
  }
}

// Sum of the stencil entries p = W, W + SPLIT, W + 2 SPLIT, ... of one node (every entry
// for SPLIT = 1), in batches of up to CHMAX loads in flight per lane; `pl` points at the
// node's entry in plane 0.  Neighbour indices are clamped per axis (the matching stencil
// entries are exactly zero outside the grid).
template <typename T, int D, int W, int SPLIT, int CHMAX = 27>
__device__ __forceinline__ cx<T> stencil_part(const cx<T> *__restrict__ pl, int N, const cx<T> *__restrict__ x,
                                              const int (&X)[5], const int (&Y)[5], const int (&Z)[5]) {
  constexpr int S = D == 3 ? 81 : 21;
  constexpr OffTable<D> OT = make_off_table<D>();
  constexpr int CNT = (S - W + SPLIT - 1) / SPLIT;
  constexpr int CH = CNT < CHMAX ? CNT : CHMAX;
  cx<T> acc[2] = {mk<T>(T(0), T(0)), mk<T>(T(0), T(0))};
#pragma unroll
  for (int c = 0; c < CNT; c += CH) {
    cx<T> pv[CH], xv[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int k = c + q;
      if (k < CNT) {
        const int p = W + SPLIT * k;
        pv[q] = pl[(size_t)p * N];
        xv[q] = x[X[OT.dx[p] + 2] + Y[OT.dy[p] + 2] + Z[OT.dz[p] + 2]];
      }
    }
#pragma unroll
    for (int q = 0; q < CH; ++q)
      if (c + q < CNT) acc[q & 1] = cfma(pv[q], xv[q], acc[q & 1]);
  }
  return acc[0] + acc[1];
}

template <typename T, int D, int SPLIT>
__device__ __forceinline__ cx<T> stencil_part_of(int w, const cx<T> *__restrict__ pl, int N,
                                                 const cx<T> *__restrict__ x, const int (&X)[5], const int (&Y)[5],
                                                 const int (&Z)[5]) {
  // w is uniform across a wavefront, so each wave takes one branch.
  if constexpr (SPLIT == 1) {
    return stencil_part<T, D, 0, 1>(pl, N, x, X, Y, Z);
  } else if constexpr (SPLIT == 2) {
    return w == 0 ? stencil_part<T, D, 0, 2>(pl, N, x, X, Y, Z) : stencil_part<T, D, 1, 2>(pl, N, x, X, Y, Z);
  } else {
    switch (w) {
      case 0: return stencil_part<T, D, 0, 4>(pl, N, x, X, Y, Z);
      case 1: return stencil_part<T, D, 1, 4>(pl, N, x, X, Y, Z);
      case 2: return stencil_part<T, D, 2, 4>(pl, N, x, X, Y, Z);
      default: return stencil_part<T, D, 3, 4>(pl, N, x, X, Y, Z);
    }
  }
}

// LDS z-marching of the 81-point apply (3D, complex float or double; "split" 8; the
// complex-double window ring takes 74.5 KB of LDS, two blocks per CU).  A block owns a segment of
// kLdsSeg consecutive in-plane nodes and a slab of z-planes.  The gathered vector's window
// of a plane (the segment and 2 rows + 2 nodes either side, so every in-plane offset
// (dx, dy) of the stencil lands in it) sits in a ring of kLdsSlots plane windows in LDS;
// while plane z is computed from windows z-2..z+2, the window of plane z+3 is loaded into
// registers and stored afterwards, one barrier per plane.  The stencil planes stream
// from the segment-tiled copy (tile_planes): per block and z-plane one contiguous run of
// 81 x kLdsSeg entries, where the SoA planes would be 81 separate streams (a plane-read
// probe of 129^3 measured 200 us tiled against 385 us SoA).  Window entries outside the
// grid are zero; in-plane offsets that wrap to the next row meet zero stencil entries.
// The sums run in the order of stencil_part, so the result equals the one-lane variant.
constexpr int kLdsSeg = ADR_BLOCK;
constexpr int kLdsMaxN0 = 129;
constexpr int kLdsWin = kLdsSeg + 4 * kLdsMaxN0 + 4;
constexpr int kLdsSlots = 6;
constexpr int kLdsMinPlanes = 8;   // planes per slab below which the window preload dominates

// Stencil-plane load of the LDS variant: each plane entry is read once per apply and the
// gathered vector is in LDS, so the planes are loaded non-temporally (measured at 257^3:
// 324.5 -> 321.3 us per level-1 apply).
template <typename T>
__device__ __forceinline__ cx<T> lds_plane_load(const cx<T> *p) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2 *>(p));
  return mk<T>(v.x, v.y);
}

template <typename T, typename F>
__device__ __forceinline__ void lds_march3(const Grid &G, const cx<T> *__restrict__ planes,
                                           const cx<T> *__restrict__ x, F &&finish) {
  __shared__ cx<T> win[kLdsSlots][kLdsWin];
  constexpr OffTable<3> OT = make_off_table<3>();
  const int n0 = G.n[0], nxy = G.n[0] * G.n[1], n2 = G.n[2];
  const int nseg = (nxy + kLdsSeg - 1) / kLdsSeg;
  const int nslab = gridDim.x / nseg;
  const int lb = logical_block();
  const int seg = lb % nseg, slab = lb / nseg;
  const int z0 = (int)((long long)n2 * slab / nslab), z1 = (int)((long long)n2 * (slab + 1) / nslab);
  const int s0 = seg * kLdsSeg;
  const int halo = 2 * n0 + 2;
  const int W = kLdsSeg + 2 * halo;
  const int tid = threadIdx.x;
  constexpr int R = (kLdsWin + ADR_BLOCK - 1) / ADR_BLOCK;
  auto load_plane = [&](int zp, cx<T> (&reg)[R]) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int w = tid + r * ADR_BLOCK;
      const int q = s0 - halo + w;
      const bool in = w < W && zp >= 0 && zp < n2 && q >= 0 && q < nxy;
      reg[r] = in ? x[(size_t)zp * nxy + q] : mk<T>(T(0), T(0));
    }
  };
  auto store_plane = [&](int zp, const cx<T> (&reg)[R]) {
    const int sl = (zp + kLdsSlots) % kLdsSlots;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int w = tid + r * ADR_BLOCK;
      if (w < W) win[sl][w] = reg[r];
    }
  };
  for (int zp = z0 - 2; zp <= z0 + 2; ++zp) {
    cx<T> reg[R];
    load_plane(zp, reg);
    store_plane(zp, reg);
  }
  __syncthreads();
  const int ip = s0 + tid;
  const bool act = ip < nxy;
  const int base = tid + halo;
  for (int z = z0; z < z1; ++z) {
    cx<T> reg[R];
    load_plane(z + 3, reg);
    if (act) {
      const int i = z * nxy + ip;
      int sl[5];
#pragma unroll
      for (int d = -2; d <= 2; ++d) sl[d + 2] = (z + d + kLdsSlots) % kLdsSlots;
      // This segment's 81 entries of plane z are one contiguous run (tiled layout).
      const cx<T> *pl = planes + ((size_t)z * nseg + seg) * (81 * kLdsSeg) + tid;
      constexpr int CH = 27;
      cx<T> acc[2] = {mk<T>(T(0), T(0)), mk<T>(T(0), T(0))};
#pragma unroll
      for (int c = 0; c < 81; c += CH) {
        // A batch of plane loads in flight; the LDS operands are read as they are used.
        cx<T> pv[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q) pv[q] = lds_plane_load(pl + (size_t)(c + q) * kLdsSeg);
#pragma unroll
        for (int q = 0; q < CH; ++q) {
          const int p = c + q;
          acc[q & 1] = cfma(pv[q], win[sl[OT.dz[p] + 2]][base + OT.dy[p] * n0 + OT.dx[p]], acc[q & 1]);
        }
      }
      finish(i, acc[0] + acc[1]);
    }
    store_plane(z + 3, reg);
    __syncthreads();
  }
}

// The LDS variant's launch on grid G: segments x slabs blocks, at most ADR_PART_BLOCKS so
// the partials fit and slabs of at least kLdsMinPlanes planes.  lds_max_slabs is 0 where
// it does not apply (2D, rows longer than kLdsMaxN0); lds_blocks takes `slabs` (the tuned
// tile depth; 0 or out of range = the most slabs) and returns the block count.
int lds_max_slabs(const Grid &G, int D) {
  if (D != 3 || G.n[0] > kLdsMaxN0) return 0;
  const int nseg = (G.n[0] * G.n[1] + kLdsSeg - 1) / kLdsSeg;
  int nslab = ADR_PART_BLOCKS / nseg;
  if (nslab > G.n[2] / kLdsMinPlanes) nslab = G.n[2] / kLdsMinPlanes;
  return nslab >= 1 ? nslab : 0;
}
long long tiled_plane_count(const Grid &G, int D, int S) {
  if (lds_max_slabs(G, D) == 0) return 0;
  const long long nseg = (G.n[0] * G.n[1] + kLdsSeg - 1) / kLdsSeg;
  return (long long)G.n[2] * nseg * S * kLdsSeg;
}

// tiled[((z nseg + seg) S + p) kLdsSeg + k] = planes[p N + z nxy + seg kLdsSeg + k], zero
// past the end of a plane.
template <typename T>
__global__ __launch_bounds__(ADR_BLOCK) void k_tile_planes(Grid G, int S, const cx<T> *__restrict__ planes,
                                                           cx<T> *__restrict__ tiled, long long total) {
  const int nxy = G.n[0] * G.n[1];
  const int nseg = (nxy + kLdsSeg - 1) / kLdsSeg;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(t % kLdsSeg);
    const long long r = t / kLdsSeg;
    const int p = (int)(r % S);
    const long long zs = r / S;
    const int seg = (int)(zs % nseg), z = (int)(zs / nseg);
    const int ip = seg * kLdsSeg + k;
    tiled[t] = ip < nxy ? planes[(size_t)p * G.N + (size_t)z * nxy + ip] : mk<T>(T(0), T(0));
  }
}
template <typename T>
void tile_planes(hipStream_t s, const Grid &G, int S, const cx<T> *planes, cx<T> *tiled) {
  const long long total = tiled_plane_count(G, 3, S);
  if (total == 0) return;
  ADR_LAUNCH(k_tile_planes<T>, launch_blocks(total), s, G, S, planes, tiled, total);
}
template void tile_planes<float>(hipStream_t, const Grid &, int, const cx<float> *, cx<float> *);
template void tile_planes<double>(hipStream_t, const Grid &, int, const cx<double> *, cx<double> *);

int lds_blocks(const Grid &G, int D, int slabs) {
  const int mx = lds_max_slabs(G, D);
  if (mx == 0) return 0;
  const int nslab = (slabs >= 1 && slabs < mx) ? slabs : mx;
  return ((G.n[0] * G.n[1] + kLdsSeg - 1) / kLdsSeg) * nslab;
}

// mode 0: y = s * (A x), where s = 1/||.|| of the predecessor's partials (prologue
//         `pin`, K = 1; block 0 stores the norm in norm_out[0] (and 0 in norm_out[1]
//         when norm_cplx) and s in inv_out), or s = *sdev, or s = 1;
// mode 1: y = b - A x, and z = dinv o y when zout is given.
// SPLIT = 1: one lane per node.  SPLIT = 2 or 4: SPLIT wavefronts share 64 nodes, each
// summing every SPLIT-th stencil entry; the parts are added in LDS in wave order (fewer
// loads in flight per lane and SPLIT times more blocks, for the small coarse levels).
// Partials: NV dots conj(V_v).y, then ||y||^2 if NORM.
template <typename T, int D, int NV, bool NORM, int SPLIT, bool GRP>
__device__ __forceinline__ void coarse_apply_body(Grid G, const cx<T> *__restrict__ planes,
                                                  const cx<T> *__restrict__ x, ProIn pin, const double *sdev,
                                                  double *norm_out, int norm_cplx, double *inv_out,
                                                  const cx<T> *__restrict__ b, cx<T> *__restrict__ y,
                                                  const cx<T> *__restrict__ dinv, cx<T> *__restrict__ zout, int mode,
                                                  VecSet<T> V, double *pout, Shot sh) {
  ADR_SHOT_ENTER(sh);
  ADR_SHOT_GRID(sh, G);
  ADR_SHIFT(planes);
  ADR_SHIFT(x);
  ADR_SHIFT(pin.partials);
  ADR_SHIFT(sdev);
  ADR_SHIFT(norm_out);
  ADR_SHIFT(inv_out);
  ADR_SHIFT(b);
  ADR_SHIFT(y);
  ADR_SHIFT(dinv);
  ADR_SHIFT(zout);
  if constexpr (GRP) shift_set<NV>(V, shot_off_);
  ADR_SHIFT(pout);
  ADR_SHOT_LIVE(sh);
  constexpr int K = 2 * NV + (NORM ? 1 : 0);
  constexpr int KA = K > 0 ? K : 1;
  __shared__ double tot[1];
  T xs = T(1);
  if (pin.partials) {
    reduce_partials(pin.partials, pin.nb, 1, tot);
    const double nrm = sqrt(tot[0]);
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    xs = (T)inv;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      norm_out[0] = nrm;
      if (norm_cplx) norm_out[1] = 0.0;
      *inv_out = inv;
    }
  } else if (sdev) {
    xs = (T)*sdev;
  }
  double red[KA];
#pragma unroll
  for (int k = 0; k < KA; ++k) red[k] = 0.0;
  int beg, end;
  chunk_range(G.N, beg, end);
  const int N = G.N;
  auto neighbours = [&](int i, int (&X)[5], int (&Y)[5], int (&Z)[5]) { coarse_neighbours<D>(G, i, X, Y, Z); };
  auto finish = [&](int i, const cx<T> &sum) {
    cx<T> o;
    if (mode == 0) {
      o = xs * sum;
      if (zout) zout[i] = o * dinv[i];
    } else {
      o = b[i] - sum;
      if (zout) zout[i] = o * dinv[i];
    }
    y[i] = o;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const cx<double> d = cdotc(cvt<double, T>(V.v[v][i]), cvt<double, T>(o));
      red[2 * v] += d.re;
      red[2 * v + 1] += d.im;
    }
    if (NORM) red[K - 1] += (double)o.re * o.re + (double)o.im * o.im;
  };
  if constexpr (SPLIT == 8) {
    lds_march3<T>(G, planes, x, finish);
  } else if constexpr (SPLIT == 1) {
    for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
      int X[5], Y[5], Z[5];
      neighbours(i, X, Y, Z);
      finish(i, stencil_part<T, D, 0, 1>(planes + i, N, x, X, Y, Z));
    }
  } else {
    constexpr int GROUPS = ADR_BLOCK / 64 / SPLIT;   // node groups of 64 per block
    __shared__ cx<T> part[GROUPS][SPLIT - 1][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int grp = wave / SPLIT, sub = wave % SPLIT;
    // Every wave runs the same trip count, so the barriers are uniform.
    for (int base = beg; base < end; base += GROUPS * 64) {
      const int i = base + grp * 64 + lane;
      const bool act = i < end;
      cx<T> sum = mk<T>(T(0), T(0));
      if (act) {
        int X[5], Y[5], Z[5];
        neighbours(i, X, Y, Z);
        sum = stencil_part_of<T, D, SPLIT>(sub, planes + i, N, x, X, Y, Z);
        if (sub > 0) part[grp][sub - 1][lane] = sum;
      }
      __syncthreads();
      if (act && sub == 0) {
#pragma unroll
        for (int w = 1; w < SPLIT; ++w) sum = sum + part[grp][w - 1][lane];
        finish(i, sum);
      }
      __syncthreads();
    }
  }
  if (K > 0) block_partials<KA>(red, K, pout);
}

// The kernel, in two register budgets: the FP32 instances fit 4 waves per SIMD; the FP64
// ones (twice the registers for a batch of 27 plane loads and gathers) are given room
// for 2, which measured faster for them.
template <typename T, int D, int NV, bool NORM, int SPLIT, bool GRP>
__global__ __launch_bounds__(ADR_BLOCK) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_coarse_apply(
    Grid G, const cx<T> *__restrict__ planes, const cx<T> *__restrict__ x, ProIn pin, const double *sdev,
    double *norm_out, int norm_cplx, double *inv_out, const cx<T> *__restrict__ b, cx<T> *__restrict__ y,
    const cx<T> *__restrict__ dinv, cx<T> *__restrict__ zout, int mode, VecSet<T> V, double *pout, Shot sh) {
  coarse_apply_body<T, D, NV, NORM, SPLIT, GRP>(G, planes, x, pin, sdev, norm_out, norm_cplx, inv_out, b, y, dinv,
                                                zout, mode, V, pout, sh);
}
template <typename T, int D, int NV, bool NORM, int SPLIT, bool GRP>
__global__ __launch_bounds__(ADR_BLOCK) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_coarse_apply_w2(
    Grid G, const cx<T> *__restrict__ planes, const cx<T> *__restrict__ x, ProIn pin, const double *sdev,
    double *norm_out, int norm_cplx, double *inv_out, const cx<T> *__restrict__ b, cx<T> *__restrict__ y,
    const cx<T> *__restrict__ dinv, cx<T> *__restrict__ zout, int mode, VecSet<T> V, double *pout, Shot sh) {
  coarse_apply_body<T, D, NV, NORM, SPLIT, GRP>(G, planes, x, pin, sdev, norm_out, norm_cplx, inv_out, b, y, dinv,
                                                zout, mode, V, pout, sh);
}

// =====================================================================================
// Pipelined GMRES relaxation (one launch per Arnoldi step).  With the unnormalized
// basis u_i (v_i = s_i u_i, s_i = 1/||u_i||) and G_i = A D^{-1} u_i, the step that forms
// u_k = w_{k-1} - sum_i H[i][k-1] v_i (w_{k-1} = A D^{-1} v_{k-1}) also forms, by
// linearity, G_k = A D^{-1} w_{k-1} - sum_i H[i][k-1] A D^{-1} v_i, the first term a
// stencil apply to D^{-1} w_{k-1}, the others the stored G_i.  So the orthogonalization
// of step k-1 and the operator apply of step k share one launch.
// Storage: Gs_0 = w_0 (normalized by the first apply), Gs_i = G_i (i >= 1, unnormalized),
// so w_i = phi_i Gs_i and A D^{-1} u_i = psi_i Gs_i with phi_0 = 1, psi_0 = 1/s_0 and
// phi_i = s_i, psi_i = 1 for i >= 1.  Y = D^{-1} Gs_{k-1}.
// Prologue: the predecessor's partials hold conj(u_i).Gs_{k-1} for i < NK (= k) and,
// when NK >= 2, ||u_{k-1}||^2 (then s_{k-1} and H[k-1][k-2] are stored here).
// =====================================================================================
template <typename T, int NK>
struct PipeCoef {
  cx<T> cu[NK];   // coefficients of u_i in u_k
  cx<T> cg[NK];   // coefficients of Gs_i in G_k
  T phi;          // w_{k-1} = phi Gs_{k-1}
};
template <typename T, int NK>
__device__ __forceinline__ PipeCoef<T, NK> pipe_prologue(ProIn pin, const double *scales, double *hcol, double *hsub,
                                                         double *sout) {
  constexpr int KP = 2 * NK + (NK >= 2 ? 1 : 0);
  __shared__ double tot[KP];
  reduce_partials(pin.partials, pin.nb, KP, tot);
  double slast;
  if constexpr (NK >= 2) {
    const double n = sqrt(tot[2 * NK]);
    slast = n > 0.0 ? 1.0 / n : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      *sout = slast;
      hsub[0] = n;
      hsub[1] = 0.0;
    }
  } else {
    slast = scales[0];
  }
  const double phi = NK == 1 ? 1.0 : slast;
  PipeCoef<T, NK> pc;
  pc.phi = (T)phi;
#pragma unroll
  for (int i = 0; i < NK; ++i) {
    const double si = (i == NK - 1) ? slast : scales[i];
    const double hre = si * phi * tot[2 * i], him = si * phi * tot[2 * i + 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      hcol[2 * i] = hre;
      hcol[2 * i + 1] = him;
    }
    pc.cu[i] = mk<T>((T)(hre * si), (T)(him * si));
    const double psi = (i == 0) ? (scales[0] > 0.0 ? 1.0 / scales[0] : 0.0) : 1.0;
    pc.cg[i] = mk<T>((T)(hre * si * psi), (T)(him * si * psi));
  }
  return pc;
}

template <typename T, int D, int NK, int SPLIT, bool GRP>
__global__ __launch_bounds__(ADR_BLOCK) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_pipe_step(
    Grid G, const cx<T> *__restrict__ planes, const cx<T> *__restrict__ yin, ProIn pin, const double *scales,
    double *hcol, double *hsub, double *sout, VecSet<T> U, VecSet<T> Gs, const cx<T> *__restrict__ dinv,
    cx<T> *__restrict__ uo, cx<T> *__restrict__ zo, cx<T> *__restrict__ go, cx<T> *__restrict__ yo, double *pout,
    Shot sh) {
  ADR_SHOT_ENTER(sh);
  ADR_SHOT_GRID(sh, G);
  ADR_SHIFT(planes);
  ADR_SHIFT(yin);
  ADR_SHIFT(pin.partials);
  ADR_SHIFT(scales);
  ADR_SHIFT(hcol);
  ADR_SHIFT(hsub);
  ADR_SHIFT(sout);
  if constexpr (GRP) {
    shift_set<NK>(U, shot_off_);
    shift_set<NK>(Gs, shot_off_);
  }
  ADR_SHIFT(dinv);
  ADR_SHIFT(uo);
  ADR_SHIFT(zo);
  ADR_SHIFT(go);
  ADR_SHIFT(yo);
  ADR_SHIFT(pout);
  ADR_SHOT_LIVE(sh);
  const PipeCoef<T, NK> pc = pipe_prologue<T, NK>(pin, scales, hcol, hsub, sout);
  constexpr int K = 2 * (NK + 1) + 1;
  double red[K];
#pragma unroll
  for (int k = 0; k < K; ++k) red[k] = 0.0;
  int beg, end;
  chunk_range(G.N, beg, end);
  const int N = G.N;
  auto finish = [&](int i, const cx<T> &t) {
    cx<T> u = pc.phi * Gs.v[NK - 1][i];
    cx<T> g = pc.phi * t;
#pragma unroll
    for (int v = 0; v < NK; ++v) {
      const cx<T> ui = U.v[v][i];
      u = u - pc.cu[v] * ui;
      g = g - pc.cg[v] * Gs.v[v][i];
    }
    const cx<T> di = dinv[i];
    uo[i] = u;
    zo[i] = u * di;
    go[i] = g;
    yo[i] = g * di;
    const cx<double> gd = cvt<double, T>(g);
#pragma unroll
    for (int v = 0; v < NK; ++v) {
      const cx<double> d = cdotc(cvt<double, T>(U.v[v][i]), gd);
      red[2 * v] += d.re;
      red[2 * v + 1] += d.im;
    }
    const cx<double> ud = cvt<double, T>(u);
    const cx<double> d = cdotc(ud, gd);
    red[2 * NK] += d.re;
    red[2 * NK + 1] += d.im;
    red[K - 1] += ud.re * ud.re + ud.im * ud.im;
  };
  if constexpr (SPLIT == 8) {
    lds_march3<T>(G, planes, yin, finish);
  } else if constexpr (SPLIT == 1) {
    for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
      int X[5], Y[5], Z[5];
      coarse_neighbours<D>(G, i, X, Y, Z);
      finish(i, stencil_part<T, D, 0, 1>(planes + i, N, yin, X, Y, Z));
    }
  } else {
    constexpr int GROUPS = ADR_BLOCK / 64 / SPLIT;
    __shared__ cx<T> part[GROUPS][SPLIT - 1][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int grp = wave / SPLIT, sub = wave % SPLIT;
    for (int base = beg; base < end; base += GROUPS * 64) {
      const int i = base + grp * 64 + lane;
      const bool act = i < end;
      cx<T> sum = mk<T>(T(0), T(0));
      if (act) {
        int X[5], Y[5], Z[5];
        coarse_neighbours<D>(G, i, X, Y, Z);
        sum = stencil_part_of<T, D, SPLIT>(sub, planes + i, N, yin, X, Y, Z);
        if (sub > 0) part[grp][sub - 1][lane] = sum;
      }
      __syncthreads();
      if (act && sub == 0) {
#pragma unroll
        for (int w = 1; w < SPLIT; ++w) sum = sum + part[grp][w - 1][lane];
        finish(i, sum);
      }
      __syncthreads();
    }
  }
  block_partials<K>(red, K, pout);
}

// Last step: u_nu only (no operator apply), and the partials of ||u_nu||^2.
template <typename T, int NK, bool GRP>
__global__ __launch_bounds__(ADR_BLOCK) void k_pipe_final(int N, ProIn pin, const double *scales, double *hcol,
                                                          double *hsub, double *sout, VecSet<T> U, VecSet<T> Gs,
                                                          cx<T> *__restrict__ uo, double *pout, Shot sh) {
  ADR_SHOT_ENTER(sh);
  ADR_SHOT_N(sh, N);
  ADR_SHIFT(pin.partials);
  ADR_SHIFT(scales);
  ADR_SHIFT(hcol);
  ADR_SHIFT(hsub);
  ADR_SHIFT(sout);
  if constexpr (GRP) {
    shift_set<NK>(U, shot_off_);
    shift_set<NK>(Gs, shot_off_);
  }
  ADR_SHIFT(uo);
  ADR_SHIFT(pout);
  ADR_SHOT_LIVE(sh);
  const PipeCoef<T, NK> pc = pipe_prologue<T, NK>(pin, scales, hcol, hsub, sout);
  double red[1] = {0.0};
  int beg, end;
  chunk_range(N, beg, end);
  for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
    cx<T> u = pc.phi * Gs.v[NK - 1][i];
#pragma unroll
    for (int v = 0; v < NK; ++v) u = u - pc.cu[v] * U.v[v][i];
    uo[i] = u;
    red[0] += (double)u.re * u.re + (double)u.im * u.im;
  }
  block_partials<1>(red, 1, pout);
}

template <typename T>
int pipe_step(hipStream_t s, int D, int split, int slabs, const Grid &G, const cx<T> *planes, const cx<T> *planes_t,
              const cx<T> *yin, ProIn pin, const double *scales, double *hcol, double *hsub, double *sout,
              const VecSet<T> &U, const VecSet<T> &Gs, const cx<T> *dinv, cx<T> *uo, cx<T> *zo, cx<T> *go, cx<T> *yo,
              double *pout) {
  const int nlds = (split == 8 && planes_t && !g_shot.sh.grid) ? lds_blocks(G, D, slabs) : 0;
  if (split == 8 && nlds == 0) split = 1;
  const int nb = split == 8 ? nlds : (split == 4 ? launch_blocks_red(4LL * G.N) : launch_blocks_red(G.N));
#define ADR_PIPE_CASE(n)                                                                                        \
  case n:                                                                                                       \
    if (split == 8) {                                                                                           \
      launch_g(k_pipe_step<T, 3, n, 8, false>, k_pipe_step<T, 3, n, 8, true>, nb, s, G, planes_t, yin, pin, scales,   \
               hcol, hsub, sout, U, Gs, dinv, uo, zo, go, yo, pout);                                             \
    } else if (D == 2) {                                                                                        \
      if (split == 4)                                                                                           \
        launch_g(k_pipe_step<T, 2, n, 4, false>, k_pipe_step<T, 2, n, 4, true>, nb, s, G, planes, yin, pin, scales, \
                 hcol, hsub, sout, U, Gs, dinv, uo, zo, go, yo, pout);                                           \
      else                                                                                                      \
        launch_g(k_pipe_step<T, 2, n, 1, false>, k_pipe_step<T, 2, n, 1, true>, nb, s, G, planes, yin, pin, scales, \
                 hcol, hsub, sout, U, Gs, dinv, uo, zo, go, yo, pout);                                           \
    } else {                                                                                                    \
      if (split == 4)                                                                                           \
        launch_g(k_pipe_step<T, 3, n, 4, false>, k_pipe_step<T, 3, n, 4, true>, nb, s, G, planes, yin, pin, scales, \
                 hcol, hsub, sout, U, Gs, dinv, uo, zo, go, yo, pout);                                           \
      else                                                                                                      \
        launch_g(k_pipe_step<T, 3, n, 1, false>, k_pipe_step<T, 3, n, 1, true>, nb, s, G, planes, yin, pin, scales, \
                 hcol, hsub, sout, U, Gs, dinv, uo, zo, go, yo, pout);                                           \
    }                                                                                                           \
    break;
  switch (U.count) {
    ADR_PIPE_CASE(1) ADR_PIPE_CASE(2) ADR_PIPE_CASE(3) ADR_PIPE_CASE(4) ADR_PIPE_CASE(5) ADR_PIPE_CASE(6)
    ADR_PIPE_CASE(7)
    default: break;
  }
#undef ADR_PIPE_CASE
  return nb;
}
template <typename T>
int pipe_final(hipStream_t s, int N, ProIn pin, const double *scales, double *hcol, double *hsub, double *sout,
               const VecSet<T> &U, const VecSet<T> &Gs, cx<T> *uo, double *pout) {
  const int nb = launch_blocks_red(N);
  switch (U.count) {
#define ADR_PF_CASE(n) \
  case n: launch_g(k_pipe_final<T, n, false>, k_pipe_final<T, n, true>, nb, s, N, pin, scales, hcol, hsub, sout, U, Gs, uo, pout); break;
    ADR_PF_CASE(1) ADR_PF_CASE(2) ADR_PF_CASE(3) ADR_PF_CASE(4) ADR_PF_CASE(5) ADR_PF_CASE(6) ADR_PF_CASE(7)
    ADR_PF_CASE(8)
#undef ADR_PF_CASE
    default: break;
  }
  return nb;
}
template int pipe_step<float>(hipStream_t, int, int, int, const Grid &, const cx<float> *, const cx<float> *,
                              const cx<float> *, ProIn,
                              const double *, double *, double *, double *, const VecSet<float> &,
                              const VecSet<float> &, const cx<float> *, cx<float> *, cx<float> *, cx<float> *,
                              cx<float> *, double *);
template int pipe_step<double>(hipStream_t, int, int, int, const Grid &, const cx<double> *, const cx<double> *,
                              const cx<double> *, ProIn,
                               const double *, double *, double *, double *, const VecSet<double> &,
                               const VecSet<double> &, const cx<double> *, cx<double> *, cx<double> *,
                               cx<double> *, cx<double> *, double *);
template int pipe_final<float>(hipStream_t, int, ProIn, const double *, double *, double *, double *,
                               const VecSet<float> &, const VecSet<float> &, cx<float> *, double *);
template int pipe_final<double>(hipStream_t, int, ProIn, const double *, double *, double *, double *,
                                const VecSet<double> &, const VecSet<double> &, cx<double> *, double *);

template <typename T, int D, bool NORM, int SPLIT>
static void dispatch_coarse_nv(hipStream_t s, int nb, const CoarseArgs<T> &a, const VecSet<T> &V) {
  switch (V.count) {
#define ADR_NV_CASE(n)                                                                                              \
  case n:                                                                                                           \
    if constexpr (sizeof(T) == 8)                                                                                   \
      launch_g(k_coarse_apply_w2<T, D, n, NORM, SPLIT, false>, k_coarse_apply_w2<T, D, n, NORM, SPLIT, true>, nb, s, \
               a.G, a.planes, a.x, a.pin, a.sdev, a.norm_out, a.norm_cplx, a.inv_out, a.b, a.y, a.dinv, a.zout,     \
               a.mode, V, a.pout);                                                                                   \
    else                                                                                                            \
      launch_g(k_coarse_apply<T, D, n, NORM, SPLIT, false>, k_coarse_apply<T, D, n, NORM, SPLIT, true>, nb, s, a.G,  \
               a.planes, a.x, a.pin, a.sdev, a.norm_out, a.norm_cplx, a.inv_out, a.b, a.y, a.dinv, a.zout, a.mode,   \
               V, a.pout);                                                                                           \
    break;
    ADR_NV_CASE(0) ADR_NV_CASE(1) ADR_NV_CASE(2) ADR_NV_CASE(3) ADR_NV_CASE(4) ADR_NV_CASE(5) ADR_NV_CASE(6)
    ADR_NV_CASE(7) ADR_NV_CASE(8)
#undef ADR_NV_CASE
    default: break;
  }
}

template <typename T, int D, bool NORM>
static void dispatch_coarse_split(hipStream_t s, int nb, const CoarseArgs<T> &a, const VecSet<T> &V) {
  if constexpr (D == 3) {
    if (a.split == 8) {
      dispatch_coarse_nv<T, D, NORM, 8>(s, nb, a, V);
      return;
    }
  }
  if (a.split == 4) dispatch_coarse_nv<T, D, NORM, 4>(s, nb, a, V);
  else dispatch_coarse_nv<T, D, NORM, 1>(s, nb, a, V);
}

template <typename T>
static int coarse_apply_lanes(hipStream_t s, int D, const CoarseArgs<T> &a, const VecSet<T> &V, bool red,
                              bool want_norm) {
  const long long lanes = (long long)a.G.N * (a.split == 4 ? 4 : 1);
  const int nb = red ? launch_blocks_red(lanes) : launch_blocks(lanes);
  if (D == 2) {
    if (want_norm) dispatch_coarse_split<T, 2, true>(s, nb, a, V);
    else dispatch_coarse_split<T, 2, false>(s, nb, a, V);
  } else {
    if (want_norm) dispatch_coarse_split<T, 3, true>(s, nb, a, V);
    else dispatch_coarse_split<T, 3, false>(s, nb, a, V);
  }
  return nb;
}

// split 8 (LDS z-marching) where lds_blocks allows it, else the one-lane variant.
template <typename T>
int coarse_apply(hipStream_t s, int D, const CoarseArgs<T> &a, const VecSet<T> *dots, bool want_norm) {
  VecSet<T> V{};
  if (dots) V = *dots;
  const bool red = want_norm || V.count > 0;
  if (a.split == 8) {
    const int nb = (a.planes_t && !g_shot.sh.grid) ? lds_blocks(a.G, D, a.slabs) : 0;
    if (nb > 0) {
      // The LDS variant streams the segment-tiled copy of the planes.
      CoarseArgs<T> at = a;
      at.planes = a.planes_t;
      if (want_norm) dispatch_coarse_split<T, 3, true>(s, nb, at, V);
      else dispatch_coarse_split<T, 3, false>(s, nb, at, V);
      return nb;
    }
    CoarseArgs<T> a1 = a;
    a1.split = 1;
    return coarse_apply_lanes<T>(s, D, a1, V, red, want_norm);
  }
  return coarse_apply_lanes<T>(s, D, a, V, red, want_norm);
}
template int coarse_apply<double>(hipStream_t, int, const CoarseArgs<double> &, const VecSet<double> *, bool);
template int coarse_apply<float>(hipStream_t, int, const CoarseArgs<float> &, const VecSet<float> *, bool);

// =====================================================================================
// GMRES relaxation on the matrix-free finest level (Sec. 4.2: Jacobi-preconditioned GMRES
// on every level).  The same contract as coarse_apply with the row recomputed from the
// coefficient planes instead of read from stored Galerkin planes:
// mode 0: y = s * (A x), s = 1/||.|| of the predecessor's partials (`pin`; block 0 stores
//         the norm and the scale), or s = 1 without them;
// mode 1: y = b - A x;
// z = dinv o y when zout is given; partials: NV dots conj(V_v).y, then ||y||^2 if NORM.
// =====================================================================================
template <typename T, int D, int NV, bool NORM, bool GRP>
__global__ __launch_bounds__(ADR_BLOCK) void k_fine_gapply(Grid G, FineCoef<T> C, FineParams P,
                                                           const cx<T> *__restrict__ x, ProIn pin, double *norm_out,
                                                           int norm_cplx, double *inv_out,
                                                           const cx<T> *__restrict__ b, cx<T> *__restrict__ y,
                                                           const cx<T> *__restrict__ dinv, cx<T> *__restrict__ zout,
                                                           int mode, VecSet<T> V, double *pout, const FineParams *Pd,
                                                           Shot sh) {
  ADR_SHOT_ENTER(sh);
  ADR_SHOT_GRID(sh, G);
  if constexpr (GRP) shift_fine_coef(C, shot_off_);
  if constexpr (GRP) {
    if (Pd) P = *shot_ptr(Pd, shot_off_);
  }
  ADR_SHIFT(x);
  ADR_SHIFT(pin.partials);
  ADR_SHIFT(norm_out);
  ADR_SHIFT(inv_out);
  ADR_SHIFT(b);
  ADR_SHIFT(y);
  ADR_SHIFT(dinv);
  ADR_SHIFT(zout);
  if constexpr (GRP) shift_set<NV>(V, shot_off_);
  ADR_SHIFT(pout);
  ADR_SHOT_LIVE(sh);
  constexpr int K = 2 * NV + (NORM ? 1 : 0);
  constexpr int KA = K > 0 ? K : 1;
  __shared__ double tot[1];
  T xs = T(1);
  if (pin.partials) {
    reduce_partials(pin.partials, pin.nb, 1, tot);
    const double nrm = sqrt(tot[0]);
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    xs = (T)inv;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      norm_out[0] = nrm;
      if (norm_cplx) norm_out[1] = 0.0;
      *inv_out = inv;
    }
  }
  double red[KA];
#pragma unroll
  for (int k = 0; k < KA; ++k) red[k] = 0.0;
  int beg, end;
  chunk_range(G.N, beg, end);
  for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
    int idx[3];
    decode(G, i, idx[0], idx[1], idx[2]);
    int nb[1 + 4 * D];
    fine_neighbours<D>(G, i, idx, nb);
    cx<T> xv[1 + 4 * D];
#pragma unroll
    for (int p = 0; p < 1 + 4 * D; ++p) xv[p] = x[nb[p]];
    T gk[3], L;
    cx<T> c;
    load_fine_coef<T, D>(C, i, gk, L, c);
    cx<T> e[1 + 4 * D];
    fine_row<T, D>(G, P, idx, gk, L, c, e);
    cx<T> acc = mk<T>(T(0), T(0));
#pragma unroll
    for (int p = 0; p < 1 + 4 * D; ++p) acc = cfma(e[p], xv[p], acc);
    const cx<T> o = (mode == 0) ? xs * acc : b[i] - acc;
    if (zout) zout[i] = o * dinv[i];
    y[i] = o;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const cx<double> d = cdotc(cvt<double, T>(V.v[v][i]), cvt<double, T>(o));
      red[2 * v] += d.re;
      red[2 * v + 1] += d.im;
    }
    if (NORM) red[K - 1] += (double)o.re * o.re + (double)o.im * o.im;
  }
  if (K > 0) block_partials<KA>(red, K, pout);
}

template <typename T, int D, bool NORM>
static void dispatch_fine_gapply(hipStream_t s, int nb, const FineCoef<T> &C, const FineParams &P,
                                 const CoarseArgs<T> &a, const VecSet<T> &V, const FineParams *Pd) {
  switch (V.count) {
#define ADR_NV_CASE(n)                                                                                          \
  case n:                                                                                                       \
    launch_g(k_fine_gapply<T, D, n, NORM, false>, k_fine_gapply<T, D, n, NORM, true>, nb, s, a.G, C, P, a.x,    \
             a.pin, a.norm_out, a.norm_cplx, a.inv_out, a.b, a.y, a.dinv, a.zout, a.mode, V, a.pout, Pd);       \
    break;
    ADR_NV_CASE(0) ADR_NV_CASE(1) ADR_NV_CASE(2) ADR_NV_CASE(3) ADR_NV_CASE(4) ADR_NV_CASE(5) ADR_NV_CASE(6)
    ADR_NV_CASE(7) ADR_NV_CASE(8)
#undef ADR_NV_CASE
    default: break;
  }
}

template <typename T>
int fine_gapply(hipStream_t s, int D, const FineCoef<T> &C, const FineParams &P, const CoarseArgs<T> &a,
                const VecSet<T> *dots, bool want_norm, const FineParams *Pd) {
  VecSet<T> V{};
  if (dots) V = *dots;
  const bool red = want_norm || V.count > 0;
  const int nb = red ? launch_blocks_red(a.G.N) : launch_blocks(a.G.N);
  if (D == 2) {
    if (want_norm) dispatch_fine_gapply<T, 2, true>(s, nb, C, P, a, V, Pd);
    else dispatch_fine_gapply<T, 2, false>(s, nb, C, P, a, V, Pd);
  } else {
    if (want_norm) dispatch_fine_gapply<T, 3, true>(s, nb, C, P, a, V, Pd);
    else dispatch_fine_gapply<T, 3, false>(s, nb, C, P, a, V, Pd);
  }
  return nb;
}
template int fine_gapply<double>(hipStream_t, int, const FineCoef<double> &, const FineParams &,
                                 const CoarseArgs<double> &, const VecSet<double> *, bool, const FineParams *);
template int fine_gapply<float>(hipStream_t, int, const FineCoef<float> &, const FineParams &,
                                const CoarseArgs<float> &, const VecSet<float> *, bool, const FineParams *);

// dinv = 1 / (diagonal entry of the fine row), from the FP64 coefficients (setup).
template <typename T, int D>
__global__ __launch_bounds__(ADR_BLOCK) void k_fine_dinv(Grid G, FineCoef<double> C, FineParams P,
                                                         cx<T> *__restrict__ dinv) {
  int beg, end;
  chunk_range(G.N, beg, end);
  for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
    int idx[3];
    decode(G, i, idx[0], idx[1], idx[2]);
    double gk[3], L;
    cx<double> c;
    load_fine_coef<double, D>(C, i, gk, L, c);
    cx<double> e[1 + 4 * D];
    fine_row<double, D>(G, P, idx, gk, L, c, e);
    const double den = e[0].re * e[0].re + e[0].im * e[0].im;
    dinv[i] = cvt<T, double>(mk<double>(e[0].re / den, -e[0].im / den));
  }
}
template <typename T>
void fine_dinv(hipStream_t s, const Grid &G, int D, const FineCoef<double> &C, const FineParams &P, cx<T> *dinv) {
  if (D == 2) ADR_LAUNCH((k_fine_dinv<T, 2>), launch_blocks(G.N), s, G, C, P, dinv);
  else ADR_LAUNCH((k_fine_dinv<T, 3>), launch_blocks(G.N), s, G, C, P, dinv);
}
template void fine_dinv<double>(hipStream_t, const Grid &, int, const FineCoef<double> &, const FineParams &,
                                cx<double> *);
template void fine_dinv<float>(hipStream_t, const Grid &, int, const FineCoef<double> &, const FineParams &,
                               cx<float> *);

// =====================================================================================
// Transfers: r_c = P^T r_f (nodal full weighting x 2^d), x_f += P e_c (bi/trilinear)
// =====================================================================================
// With pout: also z_c = dinv_c o r_c and the partials of ||r_c||^2 (the coarse
// relaxation's first Krylov vector and its norm).
// Full weighting with fixed trip counts: neighbours outside the fine grid are clamped to
// it and weighted 0, so all loads of a node can be issued together (the sum is the same
// as skipping them).
template <typename T, int D>
__device__ __forceinline__ cx<T> restrict_value(const Grid &Gf, const Grid &Gc, const cx<T> *__restrict__ rf, int J) {
  int jx, jy, jz;
  decode(Gc, J, jx, jy, jz);
  const int fx = 2 * jx, fy = 2 * jy, fz = 2 * jz;
  constexpr int NZ = (D == 3) ? 3 : 1;
  int xo[3], yo[3], zo[3];
  T wx[3], wy[3], wz[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int x = fx + q - 1, y = fy + q - 1, z = fz + q - 1;
    xo[q] = min(max(x, 0), Gf.n[0] - 1);
    yo[q] = Gf.n[0] * min(max(y, 0), Gf.n[1] - 1);
    zo[q] = (D == 3) ? Gf.n[0] * Gf.n[1] * min(max(z, 0), Gf.n[2] - 1) : 0;
    const T w = q == 1 ? T(1) : T(0.5);
    wx[q] = (x >= 0 && x < Gf.n[0]) ? w : T(0);
    wy[q] = (y >= 0 && y < Gf.n[1]) ? w : T(0);
    wz[q] = (D == 2) ? T(1) : ((z >= 0 && z < Gf.n[2]) ? w : T(0));
  }
  cx<T> v[NZ][3][3];
#pragma unroll
  for (int c = 0; c < NZ; ++c)
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int a = 0; a < 3; ++a) v[c][b][a] = rf[xo[a] + yo[b] + zo[D == 3 ? c : 1]];
  cx<T> acc = mk<T>(T(0), T(0));
#pragma unroll
  for (int c = 0; c < NZ; ++c) {
    const T w2 = (D == 3) ? wz[c] : T(1);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const T w1 = w2 * wy[b];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const T w = w1 * wx[a];
        acc.re += w * v[c][b][a].re;
        acc.im += w * v[c][b][a].im;
      }
    }
  }
  return acc;
}

template <typename T, int D, bool GRP>
__global__ __launch_bounds__(ADR_BLOCK) void k_restrict(Grid Gf, Grid Gc, const cx<T> *__restrict__ rf,
                                                        cx<T> *__restrict__ rc, const cx<T> *__restrict__ dinv_c,
                                                        cx<T> *__restrict__ z_c, double *pout, Shot sh) {
  ADR_SHOT_ENTER(sh);
  ADR_SHOT_GRID(sh, Gf);
  ADR_SHOT_GRID2(sh, Gc);
  ADR_SHIFT(rf);
  ADR_SHIFT(rc);
  ADR_SHIFT(dinv_c);
  ADR_SHIFT(z_c);
  ADR_SHIFT(pout);
  ADR_SHOT_LIVE(sh);
  double red[1] = {0.0};
  int beg, end;
  chunk_range(Gc.N, beg, end);
  for (int J = beg + threadIdx.x; J < end; J += blockDim.x) {
    const cx<T> acc = restrict_value<T, D>(Gf, Gc, rf, J);
    rc[J] = acc;
    if (pout) {
      z_c[J] = acc * dinv_c[J];
      red[0] += (double)acc.re * acc.re + (double)acc.im * acc.im;
    }
  }
  if (pout) block_partials<1>(red, 1, pout);
}

constexpr int kRestrictMaxBlocks = 4096;
static_assert(kRestrictMaxBlocks <= ADR_MAX_RED_BLOCKS * ADR_MAX_RED, "restriction partials must fit");
template <typename T>
int restrict_full(hipStream_t s, const Grid &Gf, const Grid &Gc, int D, const cx<T> *rf, cx<T> *rc,
                  const cx<T> *dinv_c, cx<T> *z_c, double *pout) {
  // One partial per block: more blocks than the usual reduction cap cost the consumer
  // little (its prologue sums nb doubles) and give the gathers more parallelism.
  int nb = launch_blocks(Gc.N);
  if (pout && nb > kRestrictMaxBlocks) nb = kRestrictMaxBlocks;
  if (D == 2) launch_g(k_restrict<T, 2, false>, k_restrict<T, 2, true>, nb, s, Gf, Gc, rf, rc, dinv_c, z_c, pout);
  else launch_g(k_restrict<T, 3, false>, k_restrict<T, 3, true>, nb, s, Gf, Gc, rf, rc, dinv_c, z_c, pout);
  return nb;
}
template int restrict_full<double>(hipStream_t, const Grid &, const Grid &, int, const cx<double> *, cx<double> *,
                                   const cx<double> *, cx<double> *, double *);
template int restrict_full<float>(hipStream_t, const Grid &, const Grid &, int, const cx<float> *, cx<float> *,
                                  const cx<float> *, cx<float> *, double *);

// Multilinear interpolation with fixed trip counts: the second coarse node along an axis
// gets weight 0 when the fine node sits on a coarse node (clamped into the grid).
template <typename T, int D>
__device__ __forceinline__ cx<T> prolong_value(const Grid &Gf, const Grid &Gc, const cx<T> *__restrict__ ec, int f) {
  int fx, fy, fz;
  decode(Gf, f, fx, fy, fz);
  const int x0 = fx >> 1, y0 = fy >> 1, z0 = fz >> 1;
  constexpr int NZ = (D == 3) ? 2 : 1;
  const int xs[2] = {x0, min(x0 + 1, Gc.n[0] - 1)};
  const int ys[2] = {Gc.n[0] * y0, Gc.n[0] * min(y0 + 1, Gc.n[1] - 1)};
  const int zs[2] = {Gc.n[0] * Gc.n[1] * z0, (D == 3) ? Gc.n[0] * Gc.n[1] * min(z0 + 1, Gc.n[2] - 1) : 0};
  const T wx[2] = {(fx & 1) ? T(0.5) : T(1), (fx & 1) ? T(0.5) : T(0)};
  const T wy[2] = {(fy & 1) ? T(0.5) : T(1), (fy & 1) ? T(0.5) : T(0)};
  const T wz[2] = {(D == 3 && (fz & 1)) ? T(0.5) : T(1), (D == 3 && (fz & 1)) ? T(0.5) : T(0)};
  cx<T> v[NZ][2][2];
#pragma unroll
  for (int c = 0; c < NZ; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) v[c][b][a] = ec[xs[a] + ys[b] + zs[c]];
  cx<T> acc = mk<T>(T(0), T(0));
#pragma unroll
  for (int c = 0; c < NZ; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const T w = wx[a] * wy[b] * wz[c];
        acc.re += w * v[c][b][a].re;
        acc.im += w * v[c][b][a].im;
      }
  return acc;
}

template <typename T, int D, bool GRP>
__global__ __launch_bounds__(ADR_BLOCK) void k_prolong_add(Grid Gf, Grid Gc, const cx<T> *__restrict__ ec,
                                                           cx<T> *__restrict__ xf, Shot sh) {
  ADR_SHOT_ENTER(sh);
  ADR_SHOT_GRID(sh, Gf);
  ADR_SHOT_GRID2(sh, Gc);
  ADR_SHIFT(ec);
  ADR_SHIFT(xf);
  ADR_SHOT_LIVE(sh);
  int beg, end;
  chunk_range(Gf.N, beg, end);
  for (int f = beg + threadIdx.x; f < end; f += blockDim.x) xf[f] = xf[f] + prolong_value<T, D>(Gf, Gc, ec, f);
}

template <typename T>
void prolong_add(hipStream_t s, const Grid &Gf, const Grid &Gc, int D, const cx<T> *ec, cx<T> *xf) {
  int nb = launch_blocks_wide(Gf.N);
  if (D == 2) launch_g(k_prolong_add<T, 2, false>, k_prolong_add<T, 2, true>, nb, s, Gf, Gc, ec, xf);
  else launch_g(k_prolong_add<T, 3, false>, k_prolong_add<T, 3, true>, nb, s, Gf, Gc, ec, xf);
}
template void prolong_add<double>(hipStream_t, const Grid &, const Grid &, int, const cx<double> *, cx<double> *);
template void prolong_add<float>(hipStream_t, const Grid &, const Grid &, int, const cx<float> *, cx<float> *);

// =====================================================================================
// GMRES relaxation pieces
// =====================================================================================
// Prologue: H[i][j] = s_i * (sum of the predecessor's dot partials), i < NV (block 0
// stores them in hcol).  Then v_new = w - sum_i H[i][j] s_i V_i (the basis is kept
// unnormalized, v_i = s_i V_i), z_new = dinv o v_new, partial ||v_new||^2.
template <typename T, int NV, bool GRP>
__global__ __launch_bounds__(ADR_BLOCK) void k_orth_step(int N, const cx<T> *__restrict__ w, VecSet<T> V, ProIn pin,
                                                         const double *scales, double *hcol,
                                                         const cx<T> *__restrict__ dinv, cx<T> *__restrict__ vnew,
                                                         cx<T> *__restrict__ znew, double *pout, Shot sh) {
  ADR_SHOT_ENTER(sh);
  ADR_SHOT_N(sh, N);
  ADR_SHIFT(w);
  if constexpr (GRP) shift_set<NV>(V, shot_off_);
  ADR_SHIFT(pin.partials);
  ADR_SHIFT(scales);
  ADR_SHIFT(hcol);
  ADR_SHIFT(dinv);
  ADR_SHIFT(vnew);
  ADR_SHIFT(znew);
  ADR_SHIFT(pout);
  ADR_SHOT_LIVE(sh);
  __shared__ double tot[2 * NV];
  reduce_partials(pin.partials, pin.nb, 2 * NV, tot);
  cx<T> coef[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double sc = scales[v];
    const double hre = sc * tot[2 * v], him = sc * tot[2 * v + 1];
    coef[v] = mk<T>((T)(hre * sc), (T)(him * sc));
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      hcol[2 * v] = hre;
      hcol[2 * v + 1] = him;
    }
  }
  double red[1] = {0.0};
  int beg, end;
  chunk_range(N, beg, end);
  for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
    cx<T> o = w[i];
#pragma unroll
    for (int v = 0; v < NV; ++v) o = o - coef[v] * V.v[v][i];
    vnew[i] = o;
    if (znew) znew[i] = o * dinv[i];
    red[0] += (double)o.re * o.re + (double)o.im * o.im;
  }
  block_partials<1>(red, 1, pout);
}

template <typename T>
int orth_step(hipStream_t s, int N, const cx<T> *w, const VecSet<T> &V, ProIn pin, const double *scales,
              double *hcol, const cx<T> *dinv, cx<T> *vnew, cx<T> *znew, double *pout) {
  const int nb = launch_blocks_red(N);
  switch (V.count) {
#define ADR_NV_CASE(n) \
  case n: launch_g(k_orth_step<T, n, false>, k_orth_step<T, n, true>, nb, s, N, w, V, pin, scales, hcol, dinv, vnew, znew, pout); break;
    ADR_NV_CASE(1) ADR_NV_CASE(2) ADR_NV_CASE(3) ADR_NV_CASE(4) ADR_NV_CASE(5) ADR_NV_CASE(6) ADR_NV_CASE(7)
    ADR_NV_CASE(8)
#undef ADR_NV_CASE
    default: break;
  }
  return nb;
}
template int orth_step<double>(hipStream_t, int, const cx<double> *, const VecSet<double> &, ProIn, const double *,
                               double *, const cx<double> *, cx<double> *, cx<double> *, double *);
template int orth_step<float>(hipStream_t, int, const cx<float> *, const VecSet<float> &, ProIn, const double *,
                              double *, const cx<float> *, cx<float> *, cx<float> *, double *);

// partial ||x||^2; z = dinv o x if z is given.
template <typename T, bool GRP>
__global__ __launch_bounds__(ADR_BLOCK) void k_norm2(int N, const cx<T> *__restrict__ x, const cx<T> *__restrict__ dinv,
                                                     cx<T> *__restrict__ z, double *pout, Shot sh) {
  ADR_SHOT_ENTER(sh);
  ADR_SHOT_N(sh, N);
  ADR_SHIFT(x);
  ADR_SHIFT(dinv);
  ADR_SHIFT(z);
  ADR_SHIFT(pout);
  ADR_SHOT_LIVE(sh);
  double red[1] = {0.0};
  int beg, end;
  chunk_range(N, beg, end);
  for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
    const cx<T> o = x[i];
    if (z) z[i] = o * dinv[i];
    red[0] += (double)o.re * o.re + (double)o.im * o.im;
  }
  block_partials<1>(red, 1, pout);
}
template <typename T>
int norm2(hipStream_t s, int N, const cx<T> *x, const cx<T> *dinv, cx<T> *z, double *pout) {
  const int nb = launch_blocks_red(N);
  launch_g(k_norm2<T, false>, k_norm2<T, true>, nb, s, N, x, dinv, z, pout);
  return nb;
}
template int norm2<double>(hipStream_t, int, const cx<double> *, const cx<double> *, cx<double> *, double *);
template int norm2<float>(hipStream_t, int, const cx<float> *, const cx<float> *, cx<float> *, double *);

// Least squares min || beta e1 - H y || for the (K+1) x K upper Hessenberg H by Givens
// rotations G = [[c, s], [-conj(s), c]]; R and g are rotated in place, then y = R^{-1} g.
template <int K>
__device__ void gmres_lsq(cx<double> (&R)[K + 1][K], double beta, cx<double> (&y)[K]) {
  cx<double> g[K + 1];
#pragma unroll
  for (int i = 0; i <= K; ++i) g[i] = mk<double>(0.0, 0.0);
  g[0] = mk<double>(beta, 0.0);
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const cx<double> a = R[j][j], b = R[j + 1][j];
    const double aa = sqrt(a.re * a.re + a.im * a.im), bb = sqrt(b.re * b.re + b.im * b.im);
    const double den = sqrt(aa * aa + bb * bb);
    double c;
    cx<double> sn;
    if (den == 0.0) {
      c = 1.0;
      sn = mk<double>(0.0, 0.0);
    } else if (aa == 0.0) {
      c = 0.0;
      sn = mk<double>(b.re / bb, -b.im / bb);
    } else {
      c = aa / den;
      sn = mk<double>(a.re / aa, a.im / aa) * mk<double>(b.re / den, -b.im / den);
    }
#pragma unroll
    for (int jj = j; jj < K; ++jj) {
      const cx<double> x1 = R[j][jj], x2 = R[j + 1][jj];
      R[j][jj] = c * x1 + sn * x2;
      R[j + 1][jj] = mk<double>(-sn.re, sn.im) * x1 + c * x2;
    }
    const cx<double> g1 = g[j], g2 = g[j + 1];
    g[j] = c * g1 + sn * g2;
    g[j + 1] = mk<double>(-sn.re, sn.im) * g1 + c * g2;
  }
#pragma unroll
  for (int j = K - 1; j >= 0; --j) {
    cx<double> acc = g[j];
#pragma unroll
    for (int jj = j + 1; jj < K; ++jj) acc = acc - R[j][jj] * y[jj];
    const cx<double> d = R[j][j];
    y[j] = (d.re == 0.0 && d.im == 0.0) ? mk<double>(0.0, 0.0) : acc * cinv(d);
  }
}

// Prologue: H[NV][NV-1] = sqrt(sum of the last orthogonalization's partials); thread 0
// solves the least squares with the Hessenberg H (column-major, leading dimension ldh,
// complex) and beta; coef_j = y_j s_j goes through shared memory.  Then
// x_out = x0 + sum_j coef_j Z_j  (Z_j = D^{-1} V_j, so this is x0 + D^{-1} V y).
// With rout, also the new residual from the Arnoldi relation A Z = V Hbar:
// b - A x_out = (b - A x0) - V Hbar y = sum_{i <= NV} (beta e_1 - Hbar y)_i s_i V_i, where
// V_NV is the last (unnormalized) Arnoldi vector, s_NV = 1/H[NV][NV-1].
template <typename T, int NV, bool GRP>
__global__ __launch_bounds__(ADR_BLOCK) void k_gmres_update(int N, const cx<T> *__restrict__ x0, VecSet<T> Z,
                                                            ProIn pin, const double *H, int ldh, const double *beta,
                                                            const double *scales, cx<T> *__restrict__ xout,
                                                            VecSet<T> Vr, cx<T> *__restrict__ rout, Shot sh) {
  ADR_SHOT_ENTER(sh);
  ADR_SHOT_N(sh, N);
  ADR_SHIFT(x0);
  if constexpr (GRP) shift_set<NV>(Z, shot_off_);
  ADR_SHIFT(pin.partials);
  ADR_SHIFT(H);
  ADR_SHIFT(beta);
  ADR_SHIFT(scales);
  ADR_SHIFT(xout);
  if constexpr (GRP) shift_set<NV + 1>(Vr, shot_off_);
  ADR_SHIFT(rout);
  ADR_SHOT_LIVE(sh);
  __shared__ double tot[1];
  __shared__ double cs[2 * NV];
  __shared__ double rs[2 * (NV + 1)];
  reduce_partials(pin.partials, pin.nb, 1, tot);
  if (threadIdx.x == 0) {
    cx<double> R[NV + 1][NV], Hb[NV + 1][NV];
#pragma unroll
    for (int j = 0; j < NV; ++j)
#pragma unroll
      for (int i = 0; i <= NV; ++i)
        R[i][j] = (i <= j + 1) ? mk<double>(H[2 * (j * ldh + i)], H[2 * (j * ldh + i) + 1]) : mk<double>(0.0, 0.0);
    const double hlast = sqrt(tot[0]);
    R[NV][NV - 1] = mk<double>(hlast, 0.0);
#pragma unroll
    for (int j = 0; j < NV; ++j)
#pragma unroll
      for (int i = 0; i <= NV; ++i) Hb[i][j] = R[i][j];
    cx<double> y[NV];
    gmres_lsq<NV>(R, *beta, y);
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      cs[2 * j] = y[j].re * scales[j];
      cs[2 * j + 1] = y[j].im * scales[j];
    }
    if (rout) {
#pragma unroll
      for (int i = 0; i <= NV; ++i) {
        cx<double> c = mk<double>(i == 0 ? *beta : 0.0, 0.0);
#pragma unroll
        for (int j = 0; j < NV; ++j) c = c - Hb[i][j] * y[j];
        const double si = (i < NV) ? scales[i] : (hlast > 0.0 ? 1.0 / hlast : 0.0);
        rs[2 * i] = c.re * si;
        rs[2 * i + 1] = c.im * si;
      }
    }
  }
  __syncthreads();
  cx<T> c[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) c[v] = mk<T>((T)cs[2 * v], (T)cs[2 * v + 1]);
  int beg, end;
  chunk_range(N, beg, end);
  for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
    cx<T> acc = x0 ? x0[i] : mk<T>(T(0), T(0));
#pragma unroll
    for (int v = 0; v < NV; ++v) acc = cfma(c[v], Z.v[v][i], acc);
    xout[i] = acc;
  }
  if (rout) {
    cx<T> cr[NV + 1];
#pragma unroll
    for (int v = 0; v <= NV; ++v) cr[v] = mk<T>((T)rs[2 * v], (T)rs[2 * v + 1]);
    for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
      cx<T> acc = cr[0] * Vr.v[0][i];
#pragma unroll
      for (int v = 1; v <= NV; ++v) acc = cfma(cr[v], Vr.v[v][i], acc);
      rout[i] = acc;
    }
  }
}
template <typename T>
void gmres_update(hipStream_t s, int N, const cx<T> *x0, const VecSet<T> &Z, ProIn pin, const double *H, int ldh,
                  const double *beta, const double *scales, cx<T> *x_out, const VecSet<T> *Vr, cx<T> *r_out) {
  int nb = launch_blocks(N);
  VecSet<T> V{};
  if (Vr) V = *Vr;
  if (r_out && V.count != Z.count + 1) return;
  switch (Z.count) {
#define ADR_NV_CASE(n) \
  case n: launch_g(k_gmres_update<T, n, false>, k_gmres_update<T, n, true>, nb, s, N, x0, Z, pin, H, ldh, beta, scales, x_out, V, r_out); break;
    ADR_NV_CASE(1) ADR_NV_CASE(2) ADR_NV_CASE(3) ADR_NV_CASE(4) ADR_NV_CASE(5) ADR_NV_CASE(6) ADR_NV_CASE(7)
    ADR_NV_CASE(8)
#undef ADR_NV_CASE
    default: break;
  }
}
template void gmres_update<double>(hipStream_t, int, const cx<double> *, const VecSet<double> &, ProIn,
                                   const double *, int, const double *, const double *, cx<double> *,
                                   const VecSet<double> *, cx<double> *);
template void gmres_update<float>(hipStream_t, int, const cx<float> *, const VecSet<float> &, ProIn, const double *,
                                  int, const double *, const double *, cx<float> *, const VecSet<float> *,
                                  cx<float> *);

// =====================================================================================
// Krylov cycle: flexible GMRES(2) on a coarse level
// =====================================================================================
template <bool GRP>
__global__ __launch_bounds__(ADR_BLOCK) void k_reduce_norm(ProIn pin, double *norm_out, int norm_cplx,
                                                           double *inv_out, Shot sh) {
  ADR_SHOT_ENTER(sh);
  ADR_SHOT_SKIP(sh);
  ADR_SHIFT(pin.partials);
  ADR_SHIFT(norm_out);
  ADR_SHIFT(inv_out);
  ADR_SHOT_LIVE(sh);
  __shared__ double tot[1];
  reduce_partials(pin.partials, pin.nb, 1, tot);
  if (threadIdx.x == 0) {
    const double nrm = sqrt(tot[0]);
    norm_out[0] = nrm;
    if (norm_cplx) norm_out[1] = 0.0;
    inv_out[0] = nrm > 0.0 ? 1.0 / nrm : 0.0;
  }
}
void reduce_norm(hipStream_t s, ProIn pin, double *norm_out, int norm_cplx, double *inv_out) {
  launch_g(k_reduce_norm<false>, k_reduce_norm<true>, 1, s, pin, norm_out, norm_cplx, inv_out);
}

// Thread 0 of every block solves the 1- or 2-column least squares (the same in every
// block, from the same device scalars and partials), then e = c_0 Z0 + c_1 Z1.
template <typename T, bool GRP>
__global__ __launch_bounds__(ADR_BLOCK) void k_fgmres2_update(int N, const cx<T> *__restrict__ Z0,
                                                              const cx<T> *__restrict__ Z1, ProIn pin,
                                                              const double *H, const double *beta,
                                                              const double *scales, double threshold,
                                                              cx<T> *__restrict__ e, Shot sh) {
  ADR_SHOT_ENTER(sh);
  ADR_SHOT_N(sh, N);
  ADR_SHIFT(Z0);
  ADR_SHIFT(Z1);
  ADR_SHIFT(pin.partials);
  ADR_SHIFT(H);
  ADR_SHIFT(beta);
  ADR_SHIFT(scales);
  ADR_SHIFT(e);
  ADR_SHOT_LIVE(sh);
  __shared__ double tot[1];
  __shared__ double cs[4];
  reduce_partials(pin.partials, pin.nb, 1, tot);
  if (threadIdx.x == 0) {
    auto at = [&](int i, int j) { return mk<double>(H[2 * (j * 3 + i)], H[2 * (j * 3 + i) + 1]); };
    const double b = *beta;
    const cx<double> h00 = at(0, 0), h10 = at(1, 0);
    const double a0 = h00.re * h00.re + h00.im * h00.im, a1 = h10.re * h10.re + h10.im * h10.im;
    // residual of the one-step least squares: beta |h10| / sqrt(|h00|^2 + |h10|^2)
    const double res1 = (a0 + a1) > 0.0 ? b * sqrt(a1 / (a0 + a1)) : b;
    if (res1 <= threshold * b || a1 == 0.0) {
      cx<double> R[2][1] = {{h00}, {h10}};
      cx<double> y[1];
      gmres_lsq<1>(R, b, y);
      cs[0] = y[0].re * scales[0];
      cs[1] = y[0].im * scales[0];
      cs[2] = 0.0;
      cs[3] = 0.0;
    } else {
      cx<double> R[3][2] = {{h00, at(0, 1)}, {h10, at(1, 1)}, {mk<double>(0.0, 0.0), mk<double>(sqrt(tot[0]), 0.0)}};
      cx<double> y[2];
      gmres_lsq<2>(R, b, y);
      cs[0] = y[0].re * scales[0];
      cs[1] = y[0].im * scales[0];
      cs[2] = y[1].re * scales[1];
      cs[3] = y[1].im * scales[1];
    }
  }
  __syncthreads();
  const cx<T> c0 = mk<T>((T)cs[0], (T)cs[1]), c1 = mk<T>((T)cs[2], (T)cs[3]);
  const bool two = cs[2] != 0.0 || cs[3] != 0.0;
  int beg, end;
  chunk_range(N, beg, end);
  for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
    cx<T> acc = c0 * Z0[i];
    if (two) acc = cfma(c1, Z1[i], acc);
    e[i] = acc;
  }
}
template <typename T>
void fgmres2_update(hipStream_t s, int N, const cx<T> *Z0, const cx<T> *Z1, ProIn pin, const double *H,
                    const double *beta, const double *scales, double threshold, cx<T> *e) {
  launch_g(k_fgmres2_update<T, false>, k_fgmres2_update<T, true>, launch_blocks(N), s, N, Z0, Z1, pin, H, beta, scales, threshold, e);
}
template void fgmres2_update<double>(hipStream_t, int, const cx<double> *, const cx<double> *, ProIn,
                                     const double *, const double *, const double *, double, cx<double> *);
template void fgmres2_update<float>(hipStream_t, int, const cx<float> *, const cx<float> *, ProIn, const double *,
                                    const double *, const double *, double, cx<float> *);

// =====================================================================================
// Outer FGMRES (FP64) Arnoldi: classical Gram-Schmidt with one re-orthogonalization
// =====================================================================================
// Prologue: h = sums of the matvec's dot partials (block 0 stores them in h_out).
template <int NV, bool GRP>
__global__ __launch_bounds__(ADR_BLOCK) void k_outer_orth1(int N, cx<double> *__restrict__ w, VecSet<double> V,
                                                           ProIn pin, double *h_out, double *pout, Shot sh) {
  ADR_SHOT_ENTER(sh);
  ADR_SHOT_N(sh, N);
  ADR_SHIFT(w);
  if constexpr (GRP) shift_set<NV>(V, shot_off_);
  ADR_SHIFT(pin.partials);
  ADR_SHIFT(h_out);
  ADR_SHIFT(pout);
  ADR_SHOT_LIVE(sh);
  constexpr int K = 2 * NV + 1;
  __shared__ double tot[2 * NV];
  reduce_partials(pin.partials, pin.nb, 2 * NV, tot);
  cx<double> h[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    h[v] = mk<double>(tot[2 * v], tot[2 * v + 1]);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      h_out[2 * v] = tot[2 * v];
      h_out[2 * v + 1] = tot[2 * v + 1];
    }
  }
  double red[K];
#pragma unroll
  for (int k = 0; k < K; ++k) red[k] = 0.0;
  int beg, end;
  chunk_range(N, beg, end);
  for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
    cx<double> vv[NV];
    cx<double> o = w[i];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      vv[v] = V.v[v][i];
      o = o - h[v] * vv[v];
    }
    w[i] = o;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const cx<double> d = cdotc(vv[v], o);
      red[2 * v] += d.re;
      red[2 * v + 1] += d.im;
    }
    red[K - 1] += o.re * o.re + o.im * o.im;
  }
  block_partials<K>(red, K, pout);
}
int outer_orth1(hipStream_t s, int N, cx<double> *w, const VecSet<double> &V, ProIn pin, double *h_out,
                double *pout) {
  const int nb = launch_blocks_red(N);
  switch (V.count) {
#define ADR_NV_CASE(n) \
  case n: launch_g(k_outer_orth1<n, false>, k_outer_orth1<n, true>, nb, s, N, w, V, pin, h_out, pout); break;
    ADR_NV_CASE(1) ADR_NV_CASE(2) ADR_NV_CASE(3) ADR_NV_CASE(4) ADR_NV_CASE(5) ADR_NV_CASE(6) ADR_NV_CASE(7)
    ADR_NV_CASE(8)
#undef ADR_NV_CASE
    default: break;
  }
  return nb;
}

// Prologue: c_i and ||w||^2 from the first pass's partials (block 0 stores them in
// red_out for the host).  V_new = (w - sum_i c_i V_i) / sqrt(||w||^2 - sum |c_i|^2).
template <int NV, bool GRP>
__global__ __launch_bounds__(ADR_BLOCK) void k_outer_orth2(int N, const cx<double> *__restrict__ w, VecSet<double> V,
                                                           ProIn pin, double *red_out, cx<double> *__restrict__ vnew,
                                                           Shot sh) {
  ADR_SHOT_ENTER(sh);
  ADR_SHOT_N(sh, N);
  ADR_SHIFT(w);
  if constexpr (GRP) shift_set<NV>(V, shot_off_);
  ADR_SHIFT(pin.partials);
  ADR_SHIFT(red_out);
  ADR_SHIFT(vnew);
  ADR_SHOT_LIVE(sh);
  __shared__ double red[2 * NV + 1];
  reduce_partials(pin.partials, pin.nb, 2 * NV + 1, red);
  if (blockIdx.x == 0 && threadIdx.x == 0)
    for (int k = 0; k < 2 * NV + 1; ++k) red_out[k] = red[k];
  cx<double> c[NV];
  double n2 = red[2 * NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    c[v] = mk<double>(red[2 * v], red[2 * v + 1]);
    n2 -= c[v].re * c[v].re + c[v].im * c[v].im;
  }
  const double nrm = sqrt(n2 > 0.0 ? n2 : 0.0);
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  int beg, end;
  chunk_range(N, beg, end);
  for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
    cx<double> o = w[i];
#pragma unroll
    for (int v = 0; v < NV; ++v) o = o - c[v] * V.v[v][i];
    vnew[i] = inv * o;
  }
}
void outer_orth2(hipStream_t s, int N, const cx<double> *w, const VecSet<double> &V, ProIn pin, double *red_out,
                 cx<double> *vnew) {
  int nb = launch_blocks(N);
  switch (V.count) {
#define ADR_NV_CASE(n) \
  case n: launch_g(k_outer_orth2<n, false>, k_outer_orth2<n, true>, nb, s, N, w, V, pin, red_out, vnew); break;
    ADR_NV_CASE(1) ADR_NV_CASE(2) ADR_NV_CASE(3) ADR_NV_CASE(4) ADR_NV_CASE(5) ADR_NV_CASE(6) ADR_NV_CASE(7)
    ADR_NV_CASE(8)
#undef ADR_NV_CASE
    default: break;
  }
}

template <typename Tz, int NV, bool GRP>
__global__ __launch_bounds__(ADR_BLOCK) void k_multi_axpy(int N, cx<double> *__restrict__ x, VecSet<Tz> Z,
                                                          const double *y, Shot sh) {
  ADR_SHOT_ENTER(sh);
  ADR_SHOT_N(sh, N);
  ADR_SHIFT(x);
  if constexpr (GRP) shift_set<NV>(Z, shot_off_);
  ADR_SHIFT(y);
  ADR_SHOT_LIVE(sh);
  cx<double> c[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) c[v] = mk<double>(y[2 * v], y[2 * v + 1]);
  int beg, end;
  chunk_range(N, beg, end);
  for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
    cx<double> acc = x[i];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc = cfma(c[v], cvt<double, Tz>(Z.v[v][i]), acc);
    x[i] = acc;
  }
}
template <typename Tz>
void multi_axpy(hipStream_t s, int N, cx<double> *x, const VecSet<Tz> &Z, const double *y) {
  int nb = launch_blocks(N);
  switch (Z.count) {
#define ADR_NV_CASE(n) \
  case n: launch_g(k_multi_axpy<Tz, n, false>, k_multi_axpy<Tz, n, true>, nb, s, N, x, Z, y); break;
    ADR_NV_CASE(1) ADR_NV_CASE(2) ADR_NV_CASE(3) ADR_NV_CASE(4) ADR_NV_CASE(5) ADR_NV_CASE(6) ADR_NV_CASE(7)
    ADR_NV_CASE(8)
#undef ADR_NV_CASE
    default: break;
  }
}
template void multi_axpy<double>(hipStream_t, int, cx<double> *, const VecSet<double> &, const double *);
template void multi_axpy<float>(hipStream_t, int, cx<double> *, const VecSet<float> &, const double *);

// y = x / ||x||, the norm from the predecessor's partials of ||x||^2 (K = 1); y = 0 for a
// zero norm.
template <bool GRP>
__global__ __launch_bounds__(ADR_BLOCK) void k_normalize(int N, const cx<double> *__restrict__ x, ProIn pin,
                                                         cx<double> *__restrict__ y, Shot sh) {
  ADR_SHOT_ENTER(sh);
  ADR_SHOT_N(sh, N);
  ADR_SHIFT(x);
  ADR_SHIFT(pin.partials);
  ADR_SHIFT(y);
  ADR_SHOT_LIVE(sh);
  __shared__ double tot[1];
  reduce_partials(pin.partials, pin.nb, 1, tot);
  const double nrm = sqrt(tot[0]);
  const double a = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) y[i] = a * x[i];
}
void normalize(hipStream_t s, int N, const cx<double> *x, ProIn pin, cx<double> *y) {
  launch_g(k_normalize<false>, k_normalize<true>, launch_blocks(N), s, N, x, pin, y);
}

template <bool GRP>
__global__ __launch_bounds__(ADR_BLOCK) void k_phase(int N, const cx<double> *__restrict__ in,
                                                     const double *__restrict__ tau, double omega, int sign,
                                                     cx<double> *out, const double *omega_dev, Shot sh) {
  ADR_SHOT_ENTER(sh);
  ADR_SHOT_N(sh, N);
  ADR_SHIFT(in);
  ADR_SHIFT(tau);
  ADR_SHIFT(out);
  if constexpr (GRP) {
    if (omega_dev) omega = *shot_ptr(omega_dev, shot_off_);
  }
  ADR_SHOT_LIVE(sh);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    double sn, cs;
    sincos(omega * tau[i], &sn, &cs);
    out[i] = in[i] * mk<double>(cs, sign * sn);
  }
}
void phase(hipStream_t s, int N, const cx<double> *in, const double *tau, double omega, int sign, cx<double> *out,
           const double *omega_dev) {
  launch_g(k_phase<false>, k_phase<true>, launch_blocks(N), s, N, in, tau, omega, sign, out, omega_dev);
}

// Reaction plane of the shifted operator H_s = H - i alpha w^2 diag(kappa^2) (Sec. 3.1,
// eq. shift): out = c - i s kappa2 with s = alpha w^2.  Setup only.
__global__ __launch_bounds__(ADR_BLOCK) void k_shift_reaction(long long n, const cx<double> *__restrict__ c,
                                                              const double *__restrict__ kappa2, double s,
                                                              cx<double> *__restrict__ out) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = mk<double>(c[i].re, c[i].im - s * kappa2[i]);
}
void shift_reaction(hipStream_t s, long long n, const cx<double> *c, const double *kappa2, double shift,
                    cx<double> *out) {
  hipLaunchKernelGGL(k_shift_reaction, dim3(launch_blocks(n)), dim3(ADR_BLOCK), 0, s, n, c, kappa2, shift, out);
}

// =====================================================================================
// Coarsest level: x = A_L^{-1} b with the dense FP64 inverse (row-major), one
// wavefront per row, lanes striding over the columns.
// =====================================================================================
template <typename T, bool GRP>
__global__ __launch_bounds__(ADR_BLOCK) void k_dense_gemv(int N, const cx<double> *__restrict__ Ainv,
                                                          const cx<T> *__restrict__ b, cx<T> *__restrict__ x,
                                                          Shot sh) {
  ADR_SHOT_ENTER(sh);
  ADR_SHOT_N(sh, N);
  ADR_SHIFT(Ainv);
  ADR_SHIFT(b);
  ADR_SHIFT(x);
  ADR_SHOT_LIVE(sh);
  const int row = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (row >= N) return;
  const cx<double> *a = Ainv + (size_t)row * N;
  double re = 0.0, im = 0.0;
  for (int j = lane; j < N; j += 64) {
    const cx<double> v = cfma(a[j], cvt<double, T>(b[j]), mk<double>(0.0, 0.0));
    re += v.re;
    im += v.im;
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if (lane == 0) x[row] = cvt<T, double>(mk<double>(re, im));
}
template <typename T>
void dense_gemv(hipStream_t s, int N, const cx<double> *Ainv, const cx<T> *b, cx<T> *x) {
  const int rows_per_block = ADR_BLOCK / 64;
  launch_g(k_dense_gemv<T, false>, k_dense_gemv<T, true>, (N + rows_per_block - 1) / rows_per_block, s, N, Ainv, b, x);
}
template void dense_gemv<double>(hipStream_t, int, const cx<double> *, const cx<double> *, cx<double> *);
template void dense_gemv<float>(hipStream_t, int, const cx<double> *, const cx<float> *, cx<float> *);


// =====================================================================================
// Coarse tail: the V-cycle below a given level in one workgroup
// =====================================================================================
// On grids small enough that a launch costs more than the work, levels first..last-1 and
// the coarsest solve run inside one kernel of ADR_TAIL_BLOCK threads, separated by
// workgroup barriers: GMRES pre-relaxation from zero (residual from the Arnoldi
// relation), restriction, ... , dense coarsest solve, ..., prolongation and GMRES
// post-relaxation.  The arithmetic per node is the multi-kernel path's (same helpers and
// scalar formulas); only the order of the reductions differs.
template <int K>
__device__ __forceinline__ void tail_reduce(double (&v)[K], int k_used, double *lds /*[16 * K]*/, double *out /*[K]*/) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int k = 0; k < k_used; ++k) {
    const double t = wave_sum(v[k]);
    if (lane == 0) lds[wid * K + k] = t;
  }
  __syncthreads();
  if (threadIdx.x < k_used) {
    double a = 0.0;
    for (int w = 0; w < ADR_TAIL_BLOCK / 64; ++w) a += lds[w * K + threadIdx.x];
    out[threadIdx.x] = a;
  }
  __syncthreads();
}

template <typename T, int D>
__device__ __forceinline__ cx<T> tail_stencil(const TailLevel<T> &L, const cx<T> *__restrict__ x, int i) {
  int X[5], Y[5], Z[5];
  coarse_neighbours<D>(L.G, i, X, Y, Z);
  // Small load batches: the 1024-thread workgroup leaves 128 VGPRs per lane.
  return stencil_part<T, D, 0, 1, 6>(L.planes + i, L.G.N, x, X, Y, Z);
}

// Shared state of one GMRES relaxation (thread 0 owns the Hessenberg matrix).
struct TailScratch {
  double red[16 * (2 * ADR_MAXNU + 2)];
  double tot[2 * ADR_MAXNU + 2];
  double H[2 * (ADR_MAXNU + 1) * ADR_MAXNU];   // complex, column-major, ld ADR_MAXNU + 1
  double R[2 * (ADR_MAXNU + 1) * ADR_MAXNU];   // rotated copy (least squares)
  double s[ADR_MAXNU + 1];                     // scale of each unnormalized basis vector
  double beta;
  double cx_[2 * ADR_MAXNU];                   // update coefficients y_j s_j
  double cr[2 * (ADR_MAXNU + 1)];              // residual coefficients (beta e1 - Hbar y)_i s_i
};

// Thread 0: least squares min ||beta e1 - Hbar y|| by Givens rotations on an LDS copy of
// Hbar (the rotations of gmres_lsq, G = [[c, s], [-conj(s), c]]), then the update and
// residual coefficients.  Only the right-hand side and y live in registers.
template <int NV>
__device__ void tail_lsq(TailScratch &S, bool want_r) {
  constexpr int LD = ADR_MAXNU + 1;
  auto H = [&](int i, int j) { return mk<double>(S.H[2 * (j * LD + i)], S.H[2 * (j * LD + i) + 1]); };
  auto R = [&](int i, int j) { return mk<double>(S.R[2 * (j * LD + i)], S.R[2 * (j * LD + i) + 1]); };
  auto setR = [&](int i, int j, cx<double> v) {
    S.R[2 * (j * LD + i)] = v.re;
    S.R[2 * (j * LD + i) + 1] = v.im;
  };
#pragma unroll
  for (int j = 0; j < NV; ++j)
#pragma unroll
    for (int i = 0; i <= j + 1; ++i) setR(i, j, H(i, j));
  cx<double> g[NV + 1];
#pragma unroll
  for (int i = 0; i <= NV; ++i) g[i] = mk<double>(i == 0 ? S.beta : 0.0, 0.0);
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const cx<double> a = R(j, j), b = R(j + 1, j);
    const double aa = sqrt(a.re * a.re + a.im * a.im), bb = sqrt(b.re * b.re + b.im * b.im);
    const double den = sqrt(aa * aa + bb * bb);
    double c;
    cx<double> sn;
    if (den == 0.0) {
      c = 1.0;
      sn = mk<double>(0.0, 0.0);
    } else if (aa == 0.0) {
      c = 0.0;
      sn = mk<double>(b.re / bb, -b.im / bb);
    } else {
      c = aa / den;
      sn = mk<double>(a.re / aa, a.im / aa) * mk<double>(b.re / den, -b.im / den);
    }
#pragma unroll
    for (int jj = j; jj < NV; ++jj) {
      const cx<double> x1 = R(j, jj), x2 = R(j + 1, jj);
      setR(j, jj, c * x1 + sn * x2);
      setR(j + 1, jj, mk<double>(-sn.re, sn.im) * x1 + c * x2);
    }
    const cx<double> g1 = g[j], g2 = g[j + 1];
    g[j] = c * g1 + sn * g2;
    g[j + 1] = mk<double>(-sn.re, sn.im) * g1 + c * g2;
  }
  cx<double> y[NV];
#pragma unroll
  for (int j = NV - 1; j >= 0; --j) {
    cx<double> acc = g[j];
#pragma unroll
    for (int jj = j + 1; jj < NV; ++jj) acc = acc - R(j, jj) * y[jj];
    const cx<double> d = R(j, j);
    y[j] = (d.re == 0.0 && d.im == 0.0) ? mk<double>(0.0, 0.0) : acc * cinv(d);
  }
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    S.cx_[2 * j] = y[j].re * S.s[j];
    S.cx_[2 * j + 1] = y[j].im * S.s[j];
  }
  if (want_r) {
#pragma unroll
    for (int i = 0; i <= NV; ++i) {
      cx<double> c = mk<double>(i == 0 ? S.beta : 0.0, 0.0);
#pragma unroll
      for (int j = (i > 0 ? i - 1 : 0); j < NV; ++j) c = c - H(i, j) * y[j];
      S.cr[2 * i] = c.re * S.s[i];
      S.cr[2 * i + 1] = c.im * S.s[i];
    }
  }
}

// GMRES relaxation on level L (see gmres_relax): x_out = x0 + D^{-1} V y; with r_out
// also b - A x_out.  x_out may alias x0.
template <typename T, int D>
__device__ void tail_gmres(const TailLevel<T> &L, const cx<T> *x0, const cx<T> *b, cx<T> *x_out, cx<T> *r_out,
                           TailScratch &S) {
  constexpr int KR = 2 * ADR_MAXNU + 2;
  const int N = L.G.N, nu = L.nu;
  const int tid = threadIdx.x;
  double acc[KR];
  // V_0 = b - A x0 (or b), Z_0 = D^{-1} V_0, ||V_0||^2
  acc[0] = 0.0;
  for (int i = tid; i < N; i += ADR_TAIL_BLOCK) {
    const cx<T> v = x0 ? b[i] - tail_stencil<T, D>(L, x0, i) : b[i];
    L.V[i] = v;
    L.Z[i] = v * L.dinv[i];
    acc[0] += (double)v.re * v.re + (double)v.im * v.im;
  }
  tail_reduce<KR>(acc, 1, S.red, S.tot);
  if (tid == 0) {
    S.beta = sqrt(S.tot[0]);
    S.s[0] = S.beta > 0.0 ? 1.0 / S.beta : 0.0;
  }
  __syncthreads();
  constexpr int LD = ADR_MAXNU + 1;
  // Unrolled to the maximum step count so that every per-basis index is static.
#pragma unroll
  for (int j = 0; j < ADR_MAXNU; ++j) {
    if (j >= nu) break;
    const cx<T> *Zj = L.Z + (size_t)j * N;
    const T sj = (T)S.s[j];
    // w = s_j A Z_j, dots conj(V_k) . w for k <= j
#pragma unroll
    for (int k = 0; k < 2 * (j + 1); ++k) acc[k] = 0.0;
    for (int i = tid; i < N; i += ADR_TAIL_BLOCK) {
      const cx<T> w = sj * tail_stencil<T, D>(L, Zj, i);
      L.w[i] = w;
#pragma unroll
      for (int k = 0; k <= j; ++k) {
        const cx<double> d = cdotc(cvt<double, T>(L.V[(size_t)k * N + i]), cvt<double, T>(w));
        acc[2 * k] += d.re;
        acc[2 * k + 1] += d.im;
      }
    }
    tail_reduce<KR>(acc, 2 * (j + 1), S.red, S.tot);
    if (tid <= j) {
      S.H[2 * (j * LD + tid)] = S.s[tid] * S.tot[2 * tid];
      S.H[2 * (j * LD + tid) + 1] = S.s[tid] * S.tot[2 * tid + 1];
    }
    __syncthreads();
    // v_{j+1} = w - sum_k H[k][j] s_k V_k, Z_{j+1} = D^{-1} v_{j+1}, its norm
    cx<T> coef[ADR_MAXNU];   // fixed size: device code must not allocate a variable-length stack array
#pragma unroll
    for (int k = 0; k <= j; ++k)
      coef[k] = mk<T>((T)(S.H[2 * (j * LD + k)] * S.s[k]), (T)(S.H[2 * (j * LD + k) + 1] * S.s[k]));
    acc[0] = 0.0;
    cx<T> *Vn = L.V + (size_t)(j + 1) * N, *Zn = L.Z + (size_t)(j + 1) * N;
    for (int i = tid; i < N; i += ADR_TAIL_BLOCK) {
      cx<T> o = L.w[i];
#pragma unroll
      for (int k = 0; k <= j; ++k) o = o - coef[k] * L.V[(size_t)k * N + i];
      Vn[i] = o;
      Zn[i] = o * L.dinv[i];
      acc[0] += (double)o.re * o.re + (double)o.im * o.im;
    }
    tail_reduce<KR>(acc, 1, S.red, S.tot);
    if (tid == 0) {
      const double nrm = sqrt(S.tot[0]);
      S.H[2 * (j * LD + j + 1)] = nrm;
      S.H[2 * (j * LD + j + 1) + 1] = 0.0;
      S.s[j + 1] = nrm > 0.0 ? 1.0 / nrm : 0.0;
    }
    __syncthreads();
  }
  if (tid == 0) {
    switch (nu) {
#define ADR_TAIL_LSQ(n) \
  case n: tail_lsq<n>(S, r_out != nullptr); break;
      ADR_TAIL_LSQ(1) ADR_TAIL_LSQ(2) ADR_TAIL_LSQ(3) ADR_TAIL_LSQ(4) ADR_TAIL_LSQ(5) ADR_TAIL_LSQ(6) ADR_TAIL_LSQ(7)
      ADR_TAIL_LSQ(8)
#undef ADR_TAIL_LSQ
      default: break;
    }
  }
  __syncthreads();
  cx<T> c[ADR_MAXNU], cr[ADR_MAXNU + 1];
#pragma unroll
  for (int k = 0; k < ADR_MAXNU; ++k)
    c[k] = k < nu ? mk<T>((T)S.cx_[2 * k], (T)S.cx_[2 * k + 1]) : mk<T>(T(0), T(0));
#pragma unroll
  for (int k = 0; k <= ADR_MAXNU; ++k)
    cr[k] = (r_out && k <= nu) ? mk<T>((T)S.cr[2 * k], (T)S.cr[2 * k + 1]) : mk<T>(T(0), T(0));
  for (int i = tid; i < N; i += ADR_TAIL_BLOCK) {
    cx<T> a = x0 ? x0[i] : mk<T>(T(0), T(0));
#pragma unroll
    for (int k = 0; k < ADR_MAXNU; ++k)
      if (k < nu) a = cfma(c[k], L.Z[(size_t)k * N + i], a);
    x_out[i] = a;
    if (r_out) {
      cx<T> r = cr[0] * L.V[i];
#pragma unroll
      for (int k = 1; k <= ADR_MAXNU; ++k)
        if (k <= nu) r = cfma(cr[k], L.V[(size_t)k * N + i], r);
      r_out[i] = r;
    }
  }
  __syncthreads();
}

template <typename T, int D>
__global__ __launch_bounds__(ADR_TAIL_BLOCK) void k_coarse_tail(const TailArgs<T> *__restrict__ Ap) {
  __shared__ TailScratch S;
  const TailArgs<T> &A = *Ap;
  const int tid = threadIdx.x;
  for (int l = A.first; l < A.last; ++l) {
    const TailLevel<T> &L = A.L[l];
    tail_gmres<T, D>(L, nullptr, L.b, L.x, L.r, S);
    const TailLevel<T> &C = A.L[l + 1];
    for (int J = tid; J < C.G.N; J += ADR_TAIL_BLOCK) C.b[J] = restrict_value<T, D>(L.G, C.G, L.r, J);
    __syncthreads();
  }
  {
    // coarsest: x = A^{-1} b, one wavefront per row (as dense_gemv)
    const TailLevel<T> &C = A.L[A.last];
    const int n = C.G.N, lane = tid & 63;
    for (int row = tid >> 6; row < n; row += ADR_TAIL_BLOCK / 64) {
      const cx<double> *a = A.Ainv + (size_t)row * n;
      double re = 0.0, im = 0.0;
      for (int j = lane; j < n; j += 64) {
        const cx<double> v = cfma(a[j], cvt<double, T>(C.b[j]), mk<double>(0.0, 0.0));
        re += v.re;
        im += v.im;
      }
      re = wave_sum(re);
      im = wave_sum(im);
      if (lane == 0) C.x[row] = cvt<T, double>(mk<double>(re, im));
    }
    __syncthreads();
  }
  for (int l = A.last - 1; l >= A.first; --l) {
    const TailLevel<T> &L = A.L[l];
    const TailLevel<T> &C = A.L[l + 1];
    for (int f = tid; f < L.G.N; f += ADR_TAIL_BLOCK) L.x[f] = L.x[f] + prolong_value<T, D>(L.G, C.G, C.x, f);
    __syncthreads();
    tail_gmres<T, D>(L, L.x, L.b, L.x, nullptr, S);
  }
}

template <typename T>
void coarse_tail(hipStream_t s, int D, const TailArgs<T> *a_dev) {
  if (D == 2) hipLaunchKernelGGL((k_coarse_tail<T, 2>), dim3(1), dim3(ADR_TAIL_BLOCK), 0, s, a_dev);
  else hipLaunchKernelGGL((k_coarse_tail<T, 3>), dim3(1), dim3(ADR_TAIL_BLOCK), 0, s, a_dev);
}
template void coarse_tail<double>(hipStream_t, int, const TailArgs<double> *);
template void coarse_tail<float>(hipStream_t, int, const TailArgs<float> *);

}  // namespace adrk
