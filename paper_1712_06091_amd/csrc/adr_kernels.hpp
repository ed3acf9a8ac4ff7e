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

// Coarse (Galerkin) stencil: S planes of N entries, plane p = neighbour offset
// (off[p][0..2]) in x, y, z.
template <typename T>
struct Stencil {
  const cx<T> *planes;
  int S;
  int centre;            // index of the (0,0,0) plane
  const int *off_lin;    // device: linear offset of each plane
  const int *off_xyz;    // device: 3 ints per plane
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
template <typename T, typename Tin, typename To>
void fine_apply(hipStream_t s, const Grid &G, int D, const FineCoef<T> &C, const FineParams &P, const cx<Tin> *x,
                const cx<To> *b, cx<To> *y, int mode, const VecSet<To> *dots, bool want_norm, double *out,
                RedScratch rs);
// x_out = x_in + w D^{-1} (b - A x_in); x_in NULL means zero.
template <typename T>
void fine_jacobi(hipStream_t s, const Grid &G, int D, const FineCoef<T> &C, const FineParams &P, const cx<T> *x_in,
                 const cx<T> *b, cx<T> *x_out, double weight);

// ---- coarse levels (stored stencils) ----------------------------------------------
// mode 0: y = A (dinv o x) * xscale   (xscale device scalar, NULL = 1; dinv NULL = 1)
// mode 1: y = b - A x
// Fused reductions as for fine_apply.
template <typename T>
void coarse_apply(hipStream_t s, const Grid &G, int D, const Stencil<T> &A, const cx<T> *x, const double *xscale,
                  const cx<T> *dinv, const cx<T> *b, cx<T> *y, int mode, const VecSet<T> *dots, bool want_norm,
                  double *out, RedScratch rs);

// ---- transfers ---------------------------------------------------------------------
template <typename T>
void restrict_full(hipStream_t s, const Grid &Gf, const Grid &Gc, int D, const cx<T> *rf, cx<T> *rc);
template <typename T>
void prolong_add(hipStream_t s, const Grid &Gf, const Grid &Gc, int D, const cx<T> *ec, cx<T> *xf);

// ---- GMRES relaxation / Arnoldi helpers --------------------------------------------
// v_new = w - sum_i h_i * scale_i * V_i, with h_i = H[hcol + i] (complex, device);
// reduces ||v_new||^2; the last block stores norm = sqrt into *hsub (complex slot, real
// part) and 1/norm (0 if norm == 0) into *snew.
template <typename T>
void orth_step(hipStream_t s, int N, const cx<T> *w, const VecSet<T> &V, const double *hcol, cx<T> *vnew,
               double *hsub, double *snew, RedScratch rs);
// ||x||^2 -> *out_norm = sqrt, *out_inv = 1/sqrt (0 if zero)
template <typename T>
void norm_inv(hipStream_t s, int N, const cx<T> *x, double *out_norm, double *out_inv, RedScratch rs);
// Givens least squares on the (k+1) x k Hessenberg H (column-major, ld = ldh complex),
// rhs beta e1: coef[j] = y_j * scale_j (complex).
void gmres_lsq(hipStream_t s, const double *H, int ldh, int k, const double *beta, const double *scales,
               double *coef);
// x_out = x0 + dinv o sum_j coef_j V_j  (x0 may be NULL, dinv may be NULL)
template <typename T>
void gmres_update(hipStream_t s, int N, const cx<T> *x0, const cx<T> *dinv, const VecSet<T> &V,
                  const double *coef, cx<T> *x_out);

// ---- outer FGMRES (FP64) -----------------------------------------------------------
// Pass 1 of CGS2: w -= sum_i h_i V_i (h from `hcol`), then reduce conj(V_i).w (2 each) and
// ||w||^2 into out[0 .. 2k], all in one pass.
void outer_orth1(hipStream_t s, int N, cx<double> *w, const VecSet<double> &V, const double *hcol, double *out,
                 RedScratch rs);
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
void dense_gemv(hipStream_t s, int N, const cx<double> *Ainv_colmajor, const cx<T> *b, cx<T> *x);

}  // namespace adrk
