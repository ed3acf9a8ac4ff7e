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

// Prologue input: the predecessor kernel's per-block partials (see reduce_partials).
struct ProIn {
  const double *partials;
  int nb, K;
};

// Shift the first NV pointers of a set to the launch's problem of a shot group.
template <int NV, typename T>
__device__ __forceinline__ void shift_set(VecSet<T> &V, long long off) {
#pragma unroll
  for (int i = 0; i < NV; ++i) V.v[i] = shot_ptr(V.v[i], off);
}

// Arguments of the Galerkin-stencil apply (see k_coarse_apply).
template <typename T>
struct CoarseArgs {
  Grid G;
  const cx<T> *planes;   // 81 (3D) / 21 (2D) planes of N entries, fixed offset order
  const cx<T> *x;
  ProIn pin;             // mode 0: scale = 1/||.|| of these partials (K = 1); none if NULL
  const double *sdev;    // mode 0 without pin: scale = *sdev when not NULL
  double *norm_out;      // mode 0 with pin: block 0 stores the norm here ...
  int norm_cplx;         // ... and 0 in norm_out[1] if set (complex Hessenberg slot)
  double *inv_out;       // ... and the scale here
  const cx<T> *b;        // mode 1
  cx<T> *y;
  const cx<T> *dinv;     // mode 1: z = dinv o y when zout != NULL
  cx<T> *zout;
  int mode;
  double *pout;          // partials (when reducing)
  int split;             // 4: four wavefronts share each node's stencil sum; 8: LDS z-marching
                         // tiles (3D, see lds_blocks); else one lane
  int slabs;             // split 8: z-slabs per launch (0 = the most)
  const cx<T> *planes_t; // split 8: the same planes tiled by segment (see tile_planes); the
                         // apply falls back to one lane when NULL
};

// Coarse tail (one workgroup): per-level data and the level range.
#define ADR_TAIL_BLOCK 1024
#define ADR_TAIL_MAXL 8
template <typename T>
struct TailLevel {
  Grid G;
  const cx<T> *planes;   // Galerkin stencil (direction of the solve)
  const cx<T> *dinv;
  cx<T> *x, *b, *r, *w;
  cx<T> *V, *Z;          // nu + 1 planes each
  int nu;
};
template <typename T>
struct TailArgs {
  int first, last;               // relaxed levels first..last-1; `last` is the coarsest
  TailLevel<T> L[ADR_TAIL_MAXL];
  const cx<double> *Ainv;        // coarsest inverse, row-major (direction of the solve)
};

namespace adrk {

// Launch configuration of the group-capable kernels: problems per launch and their
// layout (see Shot).  Set by the batch driver while it enqueues a group's work on the
// calling thread; {1, {0, NULL}} otherwise.
struct ShotLaunch {
  int count = 1;
  Shot sh{0, nullptr};
};
extern thread_local ShotLaunch g_shot;

// ---- setup (FP64) ----------------------------------------------------------------
// numerical_reaction: c = w^2 (kappa2 - |g|^2) - i w gamma kappa2, else c = -i w gamma kappa2
void coefficients(hipStream_t s, const Grid &G, int D, double h, double omega, const int src[3],
                  bool numerical_reaction, const double *kappa2, const double *tau, const double *gamma, double *g0,
                  double *g1, double *g2, double *L, cx<double> *c);
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
// y = A x (mode 0), r = b - A x (mode 1); optional fused reductions: dots conj(V_i) . y
// for the basis in `dots` (2 doubles each, first), then ||y||^2 if want_norm, as
// per-block partials in pout.  Output precision To, compute T, input Tin.  The operator
// parameters are P, or *Pd when Pd is given (a device copy, per problem in a shot
// group).  Returns the number of blocks launched.
template <typename T, typename Tin, typename To>
int fine_apply(hipStream_t s, const Grid &G, int D, const FineCoef<T> &C, const FineParams &P, const cx<Tin> *x,
               const cx<To> *b, cx<To> *y, int mode, const VecSet<To> *dots, bool want_norm, double *pout,
               const FineParams *Pd = nullptr);
// x_out = x_in + w D^{-1} (b - A x_in); x_in NULL means zero.  Parameters as fine_apply.
template <typename T>
void fine_jacobi(hipStream_t s, const Grid &G, int D, const FineCoef<T> &C, const FineParams &P, const cx<T> *x_in,
                 const cx<T> *b, cx<T> *x_out, double weight, const FineParams *Pd = nullptr);

// Pipelined GMRES relaxation steps (see k_pipe_step): one fused orthogonalization and
// apply, and the last orthogonalization; return the block count of their partials.
template <typename T>
int pipe_step(hipStream_t s, int D, int split, int slabs, const Grid &G, const cx<T> *planes, const cx<T> *planes_t,
              const cx<T> *yin, ProIn pin,
              const double *scales, double *hcol, double *hsub, double *sout, const VecSet<T> &U,
              const VecSet<T> &Gs, const cx<T> *dinv, cx<T> *uo, cx<T> *zo, cx<T> *go, cx<T> *yo, double *pout);
template <typename T>
int pipe_final(hipStream_t s, int N, ProIn pin, const double *scales, double *hcol, double *hsub, double *sout,
               const VecSet<T> &U, const VecSet<T> &Gs, cx<T> *uo, double *pout);

// Rescaled fine operator B = M A M^{-1}, M = diag(conj(ph)), ph = exp(i w tau):
// ph = exp(i w tau); out = conj(ph) in or ph in (in, out may alias); the fine stencil
// planes of A turned into B's; Jacobi on B and r = b - B x.
void phase_plane(hipStream_t s, long long n, const double *tau, double omega, cx<double> *ph);
template <typename Ti, typename To>
void mul_phase(hipStream_t s, long long n, const cx<Ti> *in, const cx<double> *ph, bool conj, cx<To> *out);
void stencil_rescale(hipStream_t s, const Grid &G, int D, cx<double> *planes, const cx<double> *ph);
template <typename T>
void fine_jacobi_ph(hipStream_t s, const Grid &G, int D, const FineCoef<T> &C, const FineParams &P, const cx<T> *ph,
                    const cx<T> *x_in, const cx<T> *b, cx<T> *x_out, double weight);
template <typename T>
void fine_residual_ph(hipStream_t s, const Grid &G, int D, const FineCoef<T> &C, const FineParams &P,
                      const cx<T> *ph, const cx<T> *x, const cx<T> *b, cx<T> *r);

// A^H x on the fine level (conjugate transpose, matrix-free), same conventions.
template <typename T, typename Tin, typename To>
int fine_apply_adj(hipStream_t s, const Grid &G, int D, const FineCoef<T> &C, const FineParams &P, const cx<Tin> *x,
                   const cx<To> *b, cx<To> *y, int mode, const VecSet<To> *dots, bool want_norm, double *pout);
// x_out = x_in + w conj(diag)^{-1} (b - A^H x_in); x_in NULL means zero.
template <typename T>
void fine_jacobi_adj(hipStream_t s, const Grid &G, int D, const FineCoef<T> &C, const FineParams &P,
                     const cx<T> *x_in, const cx<T> *b, cx<T> *x_out, double weight);
// AH[t][i] = conj(A[-t][i+t]) for a Galerkin level (zero outside the grid).
template <typename T>
void adjoint_planes(hipStream_t s, const Grid &G, int D, const cx<T> *A, cx<T> *AH);
// grad[i] += -Re(conj(lam_i) (w^2 - i w gamma_i) a_i)  (gamma may be NULL)
void grad_kappa2(hipStream_t s, int N, double omega, bool numerical_reaction, const double *gamma,
                 const cx<double> *a, const cx<double> *lam, double *grad);
// r_k = u[idx_k] - d_k
void receiver_residual(hipStream_t s, int nrec, const int *idx, const cx<double> *u, const cx<double> *d,
                       cx<double> *r);
// src = 0, then src[idx_k] += r_k in receiver order
void adjoint_source(hipStream_t s, int N, int nrec, const int *idx, const cx<double> *r, cx<double> *src);
void zero(hipStream_t s, long long n, cx<double> *x);
// out = in
void copy(hipStream_t s, long long n, const cx<double> *in, cx<double> *out);

// ---- coarse levels (stored stencils) ----------------------------------------------
// Galerkin-stencil apply (see CoarseArgs); fused dot/norm partials; returns the block
// count.
template <typename T>
int coarse_apply(hipStream_t s, int D, const CoarseArgs<T> &a, const VecSet<T> *dots, bool want_norm);
// LDS z-marching Galerkin apply (split 8) on grid G: the most z-slabs (0 where it does not
// apply) and the block count for a slab count (0 = the most).
int lds_max_slabs(const Grid &G, int D);
int lds_blocks(const Grid &G, int D, int slabs);
// The planes as the LDS apply streams them: for each z-plane and each xy-segment of
// kLdsSeg nodes, the S planes' entries of that segment, contiguous ([z][segment][plane]
// [node], the last segment of a plane zero-padded), so that one block reads one
// contiguous run per z-plane.  tiled_plane_count is the entry count (0 where the LDS
// apply does not apply); tile_planes fills it from the SoA planes.
long long tiled_plane_count(const Grid &G, int D, int S);
template <typename T>
void tile_planes(hipStream_t s, const Grid &G, int S, const cx<T> *planes, cx<T> *tiled);
// LDS z-marching on the matrix-free finest level (3D FP32, rows of at most 257 nodes and
// at least 16 planes): mode 0 = Jacobi sweep from x, mode 1 = residual b - A x.  Returns
// false (nothing launched) where it does not apply.
template <typename T>
bool fine_lds(hipStream_t s, const Grid &G, int D, const FineCoef<T> &C, const FineParams &P, const cx<T> *x,
              const cx<T> *b, cx<T> *out, int mode, double weight, const FineParams *Pd);
int fine_lds_blocks(const Grid &G, int D);
// The coarse_apply contract on the matrix-free finest level (a.planes and a.split unused):
// GMRES relaxation there.  Pd: per-problem fine parameters of a shot group.
template <typename T>
int fine_gapply(hipStream_t s, int D, const FineCoef<T> &C, const FineParams &P, const CoarseArgs<T> &a,
                const VecSet<T> *dots, bool want_norm, const FineParams *Pd);
// dinv = 1 / diag(A_beta) of the fine operator, from the FP64 coefficients.
template <typename T>
void fine_dinv(hipStream_t s, const Grid &G, int D, const FineCoef<double> &C, const FineParams &P, cx<T> *dinv);

// ---- transfers ---------------------------------------------------------------------
// With pout (else NULL): also z_c = dinv_c o r_c and the partials of ||r_c||^2; returns
// the block count.
template <typename T>
int restrict_full(hipStream_t s, const Grid &Gf, const Grid &Gc, int D, const cx<T> *rf, cx<T> *rc,
                  const cx<T> *dinv_c, cx<T> *z_c, double *pout);
template <typename T>
void prolong_add(hipStream_t s, const Grid &Gf, const Grid &Gc, int D, const cx<T> *ec, cx<T> *xf);

// ---- GMRES relaxation / Arnoldi helpers --------------------------------------------
// Prologue H[i][j] = scales_i * (dot partials), stored by block 0 in hcol; then
// v_new = w - sum_i H[i][j] scales_i V_i, z_new = dinv o v_new (skipped when z_new is
// NULL), norm partials to pout.
template <typename T>
int orth_step(hipStream_t s, int N, const cx<T> *w, const VecSet<T> &V, ProIn pin, const double *scales,
              double *hcol, const cx<T> *dinv, cx<T> *vnew, cx<T> *znew, double *pout);
// partial ||x||^2 to pout, and z = dinv o x when z != NULL.  Returns the block count.
template <typename T>
int norm2(hipStream_t s, int N, const cx<T> *x, const cx<T> *dinv, cx<T> *z, double *pout);
// Prologue: last subdiagonal from pin, least squares with H/beta, coef_j = y_j scales_j;
// x_out = x0 + sum_j coef_j Z_j  (x0 may be NULL; x_out may alias x0).  With r_out (and
// Vr = the NV + 1 Arnoldi vectors), also r_out = b - A x_out by the Arnoldi relation.
template <typename T>
void gmres_update(hipStream_t s, int N, const cx<T> *x0, const VecSet<T> &Z, ProIn pin, const double *H, int ldh,
                  const double *beta, const double *scales, cx<T> *x_out, const VecSet<T> *Vr, cx<T> *r_out);

// One block: tot = sum of the partials (K = 1); norm_out[0] = sqrt(tot) (and
// norm_out[1] = 0 when norm_cplx), inv_out[0] = 1/sqrt(tot) (0 for a zero norm).
void reduce_norm(hipStream_t s, ProIn pin, double *norm_out, int norm_cplx, double *inv_out);
// Flexible GMRES(2) update of the Krylov cycle.  H (3 x 2 complex, column-major,
// leading dimension 3) holds columns 0 and 1 except H[2][1] = sqrt(partials of pin);
// beta = ||u_0||; scales s_j = 1/||u_j||.  If the one-step residual is <= threshold *
// beta (or H[1][0] = 0) e = y_0 s_0 Z0 with the one-column least squares, else
// e = y_0 s_0 Z0 + y_1 s_1 Z1 with the two-column one.
template <typename T>
void fgmres2_update(hipStream_t s, int N, const cx<T> *Z0, const cx<T> *Z1, ProIn pin, const double *H,
                    const double *beta, const double *scales, double threshold, cx<T> *e);

// ---- outer FGMRES (FP64) -----------------------------------------------------------
// Pass 1 of CGS2: h = dot partials of the matvec (prologue; block 0 stores them in
// h_out), w -= sum_i h_i V_i, partial conj(V_i).w (2 each) and ||w||^2 to pout.
int outer_orth1(hipStream_t s, int N, cx<double> *w, const VecSet<double> &V, ProIn pin, double *h_out,
                double *pout);
// Pass 2: c and ||w||^2 from pass 1's partials (block 0 stores them in red_out);
// V_new = (w - sum_i c_i V_i) / sqrt(||w||^2 - sum |c_i|^2).
void outer_orth2(hipStream_t s, int N, const cx<double> *w, const VecSet<double> &V, ProIn pin, double *red_out,
                 cx<double> *vnew);
// x += sum_j y_j Z_j (y host-provided via device array of complex doubles)
template <typename Tz>
void multi_axpy(hipStream_t s, int N, cx<double> *x, const VecSet<Tz> &Z, const double *y);
// y = x / ||x|| with ||x||^2 from the predecessor's partials (pin, K = 1)
void normalize(hipStream_t s, int N, const cx<double> *x, ProIn pin, cx<double> *y);
// q_hat = q exp(+i w tau)  (sign = +1) or u = a exp(-i w tau) (sign = -1); w = *omega_dev
// when given (device copy, per problem in a shot group), else omega.
void phase(hipStream_t s, int N, const cx<double> *in, const double *tau, double omega, int sign, cx<double> *out,
           const double *omega_dev = nullptr);
// out = c - i shift kappa2 (reaction plane of the shifted preconditioner).
void shift_reaction(hipStream_t s, long long n, const cx<double> *c, const double *kappa2, double shift,
                    cx<double> *out);

// ---- coarse tail ---------------------------------------------------------------------
// The V-cycle on levels first..last (coarsest) from a zero guess on level `first` with
// right-hand side L[first].b, in one workgroup; the result is L[first].x.  a_dev is a
// device copy of the level table.
template <typename T>
void coarse_tail(hipStream_t s, int D, const TailArgs<T> *a_dev);

// ---- coarsest level ------------------------------------------------------------------
template <typename T>
void dense_gemv(hipStream_t s, int N, const cx<double> *Ainv_rowmajor, const cx<T> *b, cx<T> *x);

}  // namespace adrk
