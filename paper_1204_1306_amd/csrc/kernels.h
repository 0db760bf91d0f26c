// Host-side launchers of the HIP kernels (internal to libpsms; not the C-ABI).
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.h"

namespace psms {

constexpr int MAXPROP = 16;  // proposals (gauge fields) addressed by one launch

// Kernel-bracketing timer. While armed (t_kernel_timer set), launches made through
// launch_timed take `start` at the first kernel's start and `stop` at the end of
// the latest kernel (hipExtLaunchKernelGGL), so the measured span is the kernels'
// own duration without the dispatch gaps that separate event records add.
struct KernelTimer {
  hipEvent_t start, stop;
  bool used;
};
extern thread_local KernelTimer* t_kernel_timer;

template <typename F, typename... Args>
inline void launch_timed(F kernel, dim3 grid, dim3 block, uint32_t shm, hipStream_t st, Args... args) {
  KernelTimer* t = t_kernel_timer;
  if (!t) {
    hipLaunchKernelGGL(kernel, grid, block, shm, st, args...);
    return;
  }
  hipExtLaunchKernelGGL(kernel, grid, block, shm, st, t->used ? nullptr : t->start, t->stop, 0u, args...);
  t->used = true;
}

enum HopSel : int { HOP_ALL = 0, HOP_INTRA = 1, HOP_CROSS = 2 };
enum LinkFmt : int { LK_F64 = 0, LK_F32C12 = 1, LK_F32F18 = 2 };

// A batch of spinor fields: nprop groups of nrhs fields, [prop][rhs][p][unit][Vh].
struct FieldBatch {
  void* p;
  Prec prec;
  int nprop, nrhs;
};

size_t units_per_field(Prec prec, int Vh);        // storage units of one full-lattice field
size_t bytes_per_field(Prec prec, int Vh);

struct DslashParams {
  int sel;                 // HopSel
  int p0, np;              // output parities [p0, p0 + np)
  int blk0, nb;            // output blocks [blk0, blk0 + nb)
  double cdiag, chop;      // out = cdiag * in(x) + chop * (H_sel in)(x) [+ out if accumulate]
  int accumulate;
  int variant = 0;         // full-lattice stencil form (HOP_ALL only), see dslash_variant
  int xcd_map = 1;         // remap workgroups to per-XCD contiguous tile ranges
};

// out = cdiag * in + chop * H_sel in (+ out), on the selected parities/blocks.
// Scratch bytes per lane (register spills) of the kernel that stencil form v runs for
// input storage `in` and output storage `out` (F64 and F32 forms map to themselves;
// BF16 input to BF16 or F32 output); 0 when the runtime does not say.
constexpr int NVAR = 9;  // full-lattice stencil forms 0 .. NVAR - 1
size_t dslash_variant_scratch(Prec in, Prec out, int v);
void launch_dslash(hipStream_t st, const Geo& g, const void* const* links, int linkfmt, const FieldBatch& in,
                   const FieldBatch& out, const DslashParams& dp, int nr_pref);

// the same fields in another block layout (a lattice with two block sizes)
void launch_permute(hipStream_t st, const Geo& from, const Geo& to, const FieldBatch& in, const FieldBatch& out);

// boundary layout [rhs][V][4][3] complex double  <->  internal batch
void launch_pack(hipStream_t st, const Geo& g, const double* src, const FieldBatch& dst);
void launch_unpack(hipStream_t st, const Geo& g, const FieldBatch& src, double* dst);
// links [V][4][3][3] complex double -> internal F64 or F32C12
void launch_pack_links(hipStream_t st, const Geo& g, const double* U, void* dst, int linkfmt);
// zero the links that leave their outer block (g.ob), in the internal format given
void launch_cut_links(hipStream_t st, const Geo& g, void* links, int linkfmt);
// FP32 18-real links from the internal FP64 links of the same layout (any field, SU(3) or not)
void launch_links_f64_to_f18(hipStream_t st, const Geo& g, const void* f64, void* f18);
// max over links of |U U^+ - 1| (per-workgroup maxima in partial, host reduces)
void launch_unitarity(hipStream_t st, const Geo& g, const double* U, double* partial, int nwg);

// out = P in (projector of the Schur complement, black block boundaries)
void launch_project(hipStream_t st, const Geo& g, const FieldBatch& in, const FieldBatch& out);

// --- BLAS-1 on batches (per-RHS complex coefficients read from device arrays)
// y = a[r] * x + b[r] * y   (a, b: complex per rhs; nullptr a -> 0, nullptr b -> 1)
void launch_axpby(hipStream_t st, const Geo& g, const double2* a, const FieldBatch& x, const double2* b,
                  const FieldBatch& y, int coef_sign);
// y = x (precision conversion allowed), optionally scaled by real s[r]
void launch_copy(hipStream_t st, const Geo& g, const FieldBatch& x, const FieldBatch& y, const double* s);
void launch_zero(hipStream_t st, const FieldBatch& y, int Vh);
// zero the sites of one parity in every field of the batch
void launch_zero_parity(hipStream_t st, const FieldBatch& y, int Vh, int parity);
// zero every site whose block colour differs from keep_colour
void launch_keep_colour(hipStream_t st, const Geo& g, const FieldBatch& y, int keep_colour);
// y -= sum_{j<m} c[r][j] * X_j, X_j = basis + j * vstride units; c laid out [rhs][cstride]
void launch_lincomb(hipStream_t st, const Geo& g, const FieldBatch& basis, size_t vstride, int m, const double2* c,
                    int cstride, const FieldBatch& y, int sign);

// Deterministic two-pass reductions. out[r*k + j] (double2) or out[r] (double).
struct Reducer {
  double* partial;   // scratch, >= nrhs_total * nwg * 2 * kmax doubles
  int nwg;           // workgroups per rhs in pass one
};
void reduce_norm2(hipStream_t st, const Geo& g, const FieldBatch& x, const Reducer& R, double* out);
// Scalar steps of flexible GCR for basis vector k (capacity m, nrhs right-hand sides)
// that the last pass of a reduction can take over; the reduced values then go only
// into these arrays (out is not written).
struct GcrStep {
  int k, m, nrhs;
  const int* active;   // right-hand sides still iterating
  double* nw;          // [r*m + j] |w_j|^2
  double2* a;          // [r*m + j] projection coefficients (w_j, w_k) / |w_j|^2
  double2* T;          // [(r*m + j)*m + k] the same, kept for the back substitution
  double2* alpha;      // [k*nrhs + r] step length (w_k, r) / |w_k|^2
  double2* neg_alpha;  // [r] -alpha
};
// out[r*m + j] = (X_j, y)_r for j < m, X_j = basis + j*vstride. With gs (m = gs->k):
// gs->a[r*m' + j] = out / gs->nw[r*m' + j] (0 when that norm is 0; m' = gs->m) and
// gs->T[(r*m' + j)*m' + k] = gs->a[r*m' + j].
void reduce_multidot(hipStream_t st, const Geo& g, const FieldBatch& basis, size_t vstride, int m,
                     const FieldBatch& y, const Reducer& R, double2* out, const GcrStep* gs = nullptr);
// out3[r*3] = {|x|^2, Re (x, y), Im (x, y)} in one pass (x, y of one storage). With gs
// (x = w_k, y = r): gs->nw[r*m + k] = |x|^2, gs->alpha[k*nrhs + r] = (x, y) / |x|^2 for
// active right-hand sides with a nonzero norm (else 0), gs->neg_alpha[r] = -alpha.
void reduce_norm_dot(hipStream_t st, const Geo& g, const FieldBatch& x, const FieldBatch& y, const Reducer& R, double* out3,
                     const GcrStep* gs = nullptr);
// y -= sum_{j<m} c[r*cstride + j] X_j, then gs->nw, gs->alpha and gs->neg_alpha from |y|^2
// and (y, z) as reduce_norm_dot with gs makes them (x = y, y = z there); y, z and the
// basis of one storage. The reduction order is that of launch_lincomb followed by
// reduce_norm_dot.
void lincomb_norm_dot(hipStream_t st, const Geo& g, const FieldBatch& basis, size_t vstride, int m, const double2* c, int cstride,
                      const FieldBatch& y, const FieldBatch& z, const Reducer& R, const GcrStep& gs);
// out[r * nblk + blk] = |x_r|^2 over block blk (FP64 fields, deterministic)
void launch_block_norm2(hipStream_t st, const Geo& g, const FieldBatch& x, double* out);
// y += a[r] x and out[r] = |y|^2 in one pass (x, y of one storage)
void axpy_norm2(hipStream_t st, const Geo& g, const double2* a, const FieldBatch& x, const FieldBatch& y, const Reducer& R,
                double* out);

// out = wx x + wy y over n doubles (intermediate link fields of the interpolation)
void launch_lerp(hipStream_t st, const double* x, const double* y, double wx, double wy, double* out, size_t n);

// --- block solver (Schwarz / Dirichlet block inverses, minimal residual)
struct BlockMRParams {
  int colour;
  int niter;
  double tol;     // >0: stop a block when |r_b| <= tol |rho_b(initial)|
  double kappa;
  int face = 0;   // 1: first rho_b -= D_{b,other} delta_other across the block faces
  int lanes = 0;  // LDS-resident 256-site blocks: lanes per site (1, 2; 0 = by grid size)
  int eo = 0;     // even-odd preconditioned minimal residual
  const void* rho_in = nullptr;  // non-null: initial rho read from here (rho is still written)
  int x_assign = 0;              // 1: x = delta instead of x += delta
  int eo_lanes = 0;              // even-odd form on 256-site FP32 blocks: lanes per site (2, 4; 0 = by grid)
  int xcd_map = 0;               // 1: the right-hand sides of one block run back to back on one XCD
  int rho_in_f32 = 0;            // 1: rho_in is FP32 (the kernel's storage otherwise)
  int link16 = 0;                // fixed-iteration Schwarz sweeps only: 1 staged 12-real links in FP16,
                                 // 2 whole FP16 links and FP16 exchange fields
};
// For every block of the colour: (optionally) the face update of rho_b from the
// other colour's delta, then delta = MR approximation of D_b^-1 rho_b, x += delta,
// rho_b <- rho_b - D_b delta. pbuf is scratch of the same shape.
void launch_block_mr(hipStream_t st, const Geo& g, const void* const* links, int linkfmt, const FieldBatch& rho,
                     const FieldBatch& x, const FieldBatch& delta, const FieldBatch& pbuf, const BlockMRParams& bp,
                     int* iters_out);

// --- flexible GCR scalar kernels and mixed-storage site-level ops
void gcr_alpha(hipStream_t st, const double2* d, const double* nw, int k, int m, int nrhs, const int* active, double2* alpha,
               double2* neg_alpha);
void gcr_backsub(hipStream_t st, const double2* T, const double2* alpha, int n, int m, int nrhs, double2* beta);
void scatter_col(hipStream_t st, const double* src, int k, int m, int nrhs, double* dst);
void defect_scales(hipStream_t st, const double* v, const int* active, int nrhs, double* inv, double2* sq);
void launch_axpy_mixed(hipStream_t st, const Geo& g, const double2* a, const FieldBatch& x, const FieldBatch& y, int sgn);
// y += sgn * sum_j c[r * cstride + j] X_j with the basis X in another storage than y
// (BF16 -> F32, F32 -> F64, BF16 -> F64); false for any other pair (nothing launched)
bool launch_lincomb_mixed(hipStream_t st, const Geo& g, const FieldBatch& basis, size_t vstride, int m, const double2* c,
                          int cstride, const FieldBatch& y, int sgn);
void reduce_dot_mixed(hipStream_t st, const Geo& g, const FieldBatch& x, const FieldBatch& y, const Reducer& R, double2* out);
// fused passes for a BF16 basis vector x and an FP32 residual y (fused_mixed_ok)
bool fused_mixed_ok(const FieldBatch& x, const FieldBatch& y);
void reduce_norm_dot_mixed(hipStream_t st, const Geo& g, const FieldBatch& x, const FieldBatch& y, const Reducer& R,
                           double* out3, const GcrStep* gs = nullptr);
void axpy_norm2_mixed(hipStream_t st, const Geo& g, const double2* a, const FieldBatch& x, const FieldBatch& y, const Reducer& R,
                      double* out);

// --- exact block determinants (kernels_lu.hip)
// unit-vector columns k0 .. k0 + nr - 1 of the even-odd reduced block operator, in every
// block at once (fields zeroed by the caller)
void launch_lu_units(hipStream_t st, const Geo& g, double2* e, int k0, int nr, int n);
// column k0 + r of each matrix of blocks [b0, b0 + nb) from y (= -kappa^2 H_eo H_oe e), plus 1
void launch_lu_scatter(hipStream_t st, const Geo& g, const double2* y, double* M, int k0, int nr, int n, int npad, int b0,
                       int nb);
// zero nmat matrices (npad x npad complex, planar), ones on the padded diagonal
void launch_lu_init(hipStream_t st, double* M, int n, int npad, int nmat);
// blocked LU of nmat matrices in place; logdet[mat] += (sum ln|u_cc|, sum arg u_cc),
// minpiv[mat] = min(minpiv[mat], |u_cc|); inv: scratch of 4 * 64 * 64 doubles per matrix
void launch_lu_factor(hipStream_t st, double* M, int npad, int nmat, double2* logdet, double* minpiv, double* inv);

// --- relative gauge fixing (kernels_gf.hip): links in the boundary layout [V][4][3][3]
int gf_partials(const Geo& g);  // workgroups (partial sums) of the per-site kernels
void launch_gf_unpack(hipStream_t st, const Geo& g, const void* links_f64, double* U);
void launch_gf_eye(hipStream_t st, const Geo& g, double* G);
// K = exp(half_alpha C) on the block-interior sites (1 elsewhere); theta partial sums
void launch_gf_step(hipStream_t st, const Geo& g, const double* U, const double* Upc, double* K, double half_alpha,
                    double* theta_part);
// Upt(x,mu) = K(x)^+ Upc(x,mu) K(x+mu); partial sums of Re Tr(U^+ Upt)
void launch_gf_trial(hipStream_t st, const Geo& g, const double* U, const double* Upc, const double* K, double* Upt,
                     double* f_part);
void launch_gf_overlap(hipStream_t st, const Geo& g, const double* U, const double* Up, double* f_part);
void launch_gf_accept(hipStream_t st, const Geo& g, double* G, const double* K);
// g = G^(1/2) on the domain; Ug = U^g, Upg = U'^(g^-1)
void launch_gf_finish(hipStream_t st, const Geo& g, const double* G, double* gout, const double* U, const double* Up,
                      double* Ug, double* Upg);

// out = U' on the links inside the blocks x // b whose accept flag (lexicographic block
// index) is set, U elsewhere (boundary layout)
void launch_merge_links(hipStream_t st, const Geo& g, const int* b, const int* accept, const double* U, const double* Up,
                        double* out);
// per-workgroup max |U' - U| over the links that leave their block x // b
void launch_change_across(hipStream_t st, const Geo& g, const int* b, const double* U, const double* Up, double* part);

// --- gauge-covariant network
// one layer (forward, or adjoint with adj = 1) on F32 activations [batch][channel][field]
void launch_net_layer(hipStream_t st, const Geo& g, const void* links, const void* in, void* out, const float2* W, int cin_f,
                      int cout_f, int adj, int batch);
// matrix-core form of the layer: weights packed into bf16 MFMA fragments first
size_t net_pack_units(int cin_f, int cout_f, int adj);
void launch_net_pack(hipStream_t st, const float2* W, int cin_f, int cout_f, int adj, uint2* Apack);
void launch_net_layer_mfma(hipStream_t st, const Geo& g, const void* links, const void* in, void* out, const uint2* Apack,
                           int cin_f, int cout_f, int adj, int batch);
// number of float2 partial blocks (each 9*cout*cin*16) the gradient kernel writes
int net_wgrad_partials(const Geo& g, int batch);
// grad_out[t][co][ci][s1][s2] = sum_x G_co(x)[s1,.] conj((T_t Phi_ci)(x)[s2,.]), summed over the batch
void launch_net_wgrad(hipStream_t st, const Geo& g, const void* links, const void* phi, const void* G, int cin, int cout,
                      int batch, float2* partial, double2* grad_out);
void launch_adam(hipStream_t st, float* w, const double* grad, float* m, float* v, int n, float lr, float b1, float b2,
                 float eps, int step);
// complex Gaussian boundary-layout fields (density exp(-|z|^2)), counter-based
void launch_gaussian(hipStream_t st, double* out, size_t ncomplex, int nfield, uint64_t seed, uint32_t stream);

}  // namespace psms
