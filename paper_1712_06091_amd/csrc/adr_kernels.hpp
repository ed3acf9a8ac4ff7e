// Host-side launchers for the ADR kernels (definitions in adr_kernels.hip).
#pragma once
#include "adr_common.hpp"
#include "adr_fine.hpp"

// Pointers to up to ADR_MAXV basis vectors plus their scale factors (device scalars,
// NULL = 1).
template <typename T>
struct VecSet {
  const cx<T> *v[ADR_MAXV];
  const double *scale[ADR_MAXV];
  int count;
};

#define ADR_MAXNU 8   // GMRES relaxation steps per sweep

// One-block finishing step of a two-launch reduction (see RedScratch).
enum FinishAction { FIN_RAW = 0, FIN_NORM_INV = 1, FIN_DOTS = 2, FIN_ORTH = 3 };
struct FinishArgs {
  int nb, K, action;
  int nv;                          // FIN_DOTS: number of complex dots
  const double *scale[ADR_MAXV];   // FIN_DOTS: per-dot scale (NULL = 1)
  double *out;                     // RAW: K values; NORM_INV: norm; DOTS: 2*nv (+norm);
                                   // ORTH: complex slot H[j+1][j]
  double *out_inv;                 // NORM_INV/DOTS: 1/norm; ORTH: new scale factor
  int lsq_k;                       // ORTH: > 0 -> also solve the k-step least squares
  const double *H;
  int ldh;
  const double *beta;
  const double *s;
  double *coef;
};

namespace adrk {

// ---- setup (FP64) ----------------------------------------------------------------
void coefficients(hipStream_t s, const Grid &G, int D, double h, double omega, const int src[3],
                  const double *kappa2, const double *tau, const double *gamma, double *g0, double *g1,
                  double *g2, double *L, cx<double> *c);
void fine_stencil(hipStream_t s, const Grid &G, int D, const FineCoef<double> &C, const FineParams &P,
                  cx<double> *planes /* (1+4D) x N */);
void galerkin(hipStream_t s, const Grid &Gf, const Grid &Gc, const cx<double> *in_planes, const int *in_off_xyz,
              int S_in, cx<double> *out_planes, const int *out_off_xyz, int S_out, const int *tri_start,
              const int *tri_p, const int *tri_d, const double *tri_w);
template <typename T>
void stencil_diag_inv(hipStream_t s, int N, const cx<T> *centre_plane, cx<T> *dinv);
template <typename To, typename Ti>
void convert(hipStream_t s, long long n, const cx<Ti> *in, cx<To> *out);
template <typename To, typename Ti>
void convert_real(hipStream_t s, long long n, const Ti *in, To *out);

// ---- fine level (matrix-free) ------------------------------------------------------
// y = A x (mode 0), r = b - A x (mode 1); optional fused reductions into `out`:
// dots scale_i * conj(V_i) . y for the basis in `dots` (2 doubles each, first), then
// ||y|| (the norm, not its square) if want_norm.  Output precision To, compute T, input Tin.
// Returns the number of blocks launched (the partial count for the finish kernel).
template <typename T, typename Tin, typename To>
int fine_apply(hipStream_t s, const Grid &G, int D, const FineCoef<T> &C, const FineParams &P, const cx<Tin> *x,
               const cx<To> *b, cx<To> *y, int mode, const VecSet<To> *dots, bool want_norm, RedScratch rs);
// x_out = x_in + w D^{-1} (b - A x_in); x_in NULL means zero.
template <typename T>
void fine_jacobi(hipStream_t s, const Grid &G, int D, const FineCoef<T> &C, const FineParams &P, const cx<T> *x_in,
                 const cx<T> *b, cx<T> *x_out, double weight);

// ---- coarse levels (stored stencils) ----------------------------------------------
// Stencil planes: 81 (3D) / 21 (2D) planes of N entries in the fixed offset order.
// mode 0: y = (A x) * xscale   (xscale device scalar, NULL = 1)
// mode 1: y = b - A x
// Fused reductions as for fine_apply; returns the block count.
template <typename T>
int coarse_apply(hipStream_t s, const Grid &G, int D, const cx<T> *planes, const cx<T> *x, const double *xscale,
                 const cx<T> *b, cx<T> *y, int mode, const VecSet<T> *dots, bool want_norm, RedScratch rs);

// ---- transfers ---------------------------------------------------------------------
template <typename T>
void restrict_full(hipStream_t s, const Grid &Gf, const Grid &Gc, int D, const cx<T> *rf, cx<T> *rc);
template <typename T>
void prolong_add(hipStream_t s, const Grid &Gf, const Grid &Gc, int D, const cx<T> *ec, cx<T> *xf);

// ---- GMRES relaxation / Arnoldi helpers --------------------------------------------
// v_new = w - sum_i h_i * scale_i * V_i (h_i = hcol[2i..2i+1]); z_new = dinv o v_new if
// z_new; partial ||v_new||^2.  Returns the block count.
template <typename T>
int orth_step(hipStream_t s, int N, const cx<T> *w, const VecSet<T> &V, const double *hcol, const cx<T> *dinv,
              cx<T> *vnew, cx<T> *znew, RedScratch rs);
// partial ||x||^2, and z = dinv o x when z != NULL.  Returns the block count.
template <typename T>
int norm2(hipStream_t s, int N, const cx<T> *x, const cx<T> *dinv, cx<T> *z, RedScratch rs);
// Finishing step of a reduction (one block).
void finish(hipStream_t s, const FinishArgs &A, RedScratch rs);
// x_out = x0 + sum_j coef_j Z_j  (x0 may be NULL; x_out may alias x0)
template <typename T>
void gmres_update(hipStream_t s, int N, const cx<T> *x0, const VecSet<T> &Z, const double *coef, cx<T> *x_out);

// ---- outer FGMRES (FP64) -----------------------------------------------------------
// Pass 1 of CGS2: w -= sum_i h_i V_i (h from `hcol`), with partial conj(V_i).w (2 each)
// and ||w||^2 (finish with FIN_RAW).  Returns the block count.
int outer_orth1(hipStream_t s, int N, cx<double> *w, const VecSet<double> &V, const double *hcol, RedScratch rs);
// Pass 2: V_new = (w - sum_i c_i V_i) / nrm where c = out[0..2k) and
// nrm = sqrt(||w||^2 - sum |c_i|^2) computed from `red` on the device.
void outer_orth2(hipStream_t s, int N, const cx<double> *w, const VecSet<double> &V, const double *red,
                 cx<double> *vnew);
// x += sum_j y_j Z_j (y host-provided via device array of complex doubles)
template <typename Tz>
void multi_axpy(hipStream_t s, int N, cx<double> *x, const VecSet<Tz> &Z, const double *y);
// y = x * (1/scale), scale = device scalar (real)
void scale_by_inv(hipStream_t s, int N, const cx<double> *x, const double *scale, cx<double> *y);
// q_hat = q exp(+i w tau)  (sign = +1) or u = a exp(-i w tau) (sign = -1)
void phase(hipStream_t s, int N, const cx<double> *in, const double *tau, double omega, int sign, cx<double> *out);

// ---- coarsest level ------------------------------------------------------------------
template <typename T>
void dense_gemv(hipStream_t s, int N, const cx<double> *Ainv_rowmajor, const cx<T> *b, cx<T> *x);

}  // namespace adrk
