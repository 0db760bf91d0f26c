/* libpsms: Wilson-Dirac / domain-decomposition hot path of the stochastic
 * fermion-determinant-ratio estimator (Finkenrath, Knechtli, Leder, "Fermions
 * as Global Correction: the QCD Case"), for AMD MI355X (gfx950).
 *
 * Conventions for every call
 * --------------------------
 * Operator. D = 2 kappa (D_w + m_0) = 1 - kappa H, the Wilson-Dirac operator of
 *   eq. Dw (Sec. 5) with kappa = 1/(2 m_0 + 8); periodic in space, antiperiodic
 *   in time when geom.antiperiodic_t is set (Sec. 6). Gamma matrices in the
 *   chiral basis gamma_0 = [[0,-1],[-1,0]], gamma_k = [[0,-i s_k],[i s_k,0]].
 * Sites. Direction 0 is time; site index ((x0*L1 + x1)*L2 + x2)*L3 + x3.
 * Spinor fields (every "in", "out", "b", "x", "noise"): nrhs consecutive fields,
 *   each [V][4 spin][3 colour] complex FP64 stored as interleaved (re, im):
 *   24*V doubles per field. FP64 at the boundary for every precision.
 * Gauge fields: [V][4 mu][3][3] complex FP64 (row-major 3x3), U[x][mu] is the link
 *   from x to x + mu.
 * Blocks (Sec. 3, eq. domdec): non-overlapping boxes of size b[mu]; the block
 *   containing the origin is black, colours alternate like a checker board.
 *   Requirements: L[mu] % b[mu] == 0, L[mu]/b[mu] even, b[mu] even, L[mu] <= 255.
 * Pointers. Any pointer may be host memory or device memory of the context's
 *   device (e.g. a PyTorch tensor's data_ptr). Device pointers are used in place;
 *   host buffers are staged. Work runs on the stream given to psms_create; calls
 *   return after the results are in the caller's buffers (host outputs) or
 *   enqueued (device outputs). The caller owns every buffer; nothing is freed
 *   across the ABI. One context per stream and thread.
 * Errors. Every call returns a psms_status; no exception crosses the ABI.
 *   psms_last_error() gives a message for the last failure on the context.
 */
#ifndef PSMS_H
#define PSMS_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PSMS_OK = 0,
  PSMS_EINVAL = -1,    /* bad argument or geometry */
  PSMS_ENOMEM = -2,    /* device allocation failed */
  PSMS_EHIP = -3,      /* HIP runtime error */
  PSMS_ENOTCONV = -4,  /* solver hit max_iter or stagnated; outputs hold the last iterate */
  PSMS_ENOTSU3 = -5,   /* a link is not SU(3) (12-real compression needs it) */
  PSMS_ENAN = -6       /* NaN or Inf met in a residual */
} psms_status;

typedef enum { PSMS_F64 = 0, PSMS_MIXED = 1 } psms_prec;  /* MIXED: FP32 12-real links, FP32/BF16 spinors inside, FP64 outside */
typedef enum { PSMS_OP_FULL = 0, PSMS_OP_SCHUR = 1 } psms_op;
typedef enum { PSMS_PC_NONE = 0, PSMS_PC_SAP = 1, PSMS_PC_NET = 2 } psms_pc;
typedef enum { PSMS_SPINOR_F32 = 0, PSMS_SPINOR_BF16 = 1 } psms_inner_storage;

typedef struct {
  int L[4];            /* lattice extent, mu = 0 is time */
  int b[4];            /* block extent of the domain decomposition (Schur complement) */
  int antiperiodic_t;  /* 1: fermions antiperiodic in time */
  double kappa;        /* hopping parameter */
  int sap_b[4];        /* block extent of the Schwarz preconditioner of the full-lattice
                          solves; all zero: the same as b. Must divide b, be even, with
                          L[mu]/sap_b[mu] even. The solver then works in a second block
                          layout (fields permuted in and out, links held twice). */
  int outer_b[4];      /* recursive domain decomposition (Sec. 3, eq. ddrec): all zero for
                          none; else every operator of the context is the Dirichlet operator
                          of the outer blocks of this extent (the direct sum of their block
                          operators D_B: hops across outer faces are dropped), whose Schur
                          complement is taken over the sub-blocks b. Must be a multiple of
                          b[mu] with outer_b[mu]/b[mu] even, and divide L[mu]. */
} psms_geom;

typedef struct {
  double tol;          /* stop when the FP64 true residual |b - D x| / |b| <= tol, per right-hand side */
  int max_iter;        /* outer iterations (FP64 path: GCR iterations; mixed: total inner iterations) */
  int restart;         /* GCR restart length (Krylov basis size), <= 64 */
  psms_prec prec;
  psms_pc pc;          /* right preconditioner of the flexible GCR */
  int sap_cycles;      /* Schwarz cycles per preconditioner application */
  int block_iters;     /* minimal-residual iterations per block solve inside the Schwarz cycle */
  double inner_tol;    /* mixed: relative residual reduction asked of each inner solve; a
                          later pass asks only half the reduction still needed to reach
                          tol, when that is looser */
  psms_inner_storage inner_storage;
  int net_fallback;    /* PC_NET: fall back to SAP when the residual stalls */
  int rhs_chunk;       /* psms_logdet_ratio: right-hand sides solved together (0: all) */
} psms_solve_params;

typedef struct {
  int converged;
  int outer_iters;        /* defect-correction steps (mixed) or restarts (FP64) */
  int inner_iters;        /* total GCR iterations */
  int used_fallback;
  double true_rel_residual; /* max over right-hand sides */
  double seconds;
} psms_solve_stats;

typedef struct psms_ctx psms_ctx;

/* Fills params with defaults: tol 1e-10, max_iter 2000, restart 16, F64, SAP,
 * 4 cycles, 6 block iterations, inner_tol 1e-2 (BF16 inner storage clamps it to
 * >= 5e-3), F32 inner storage, fallback on, rhs_chunk 0. */
void psms_default_params(psms_solve_params* params);

/* Creates a context for the geometry on HIP device `device`, enqueueing work on
 * `hip_stream` (hipStream_t, may be NULL for the default stream). */
psms_status psms_create(const psms_geom* geom, int device, void* hip_stream, psms_ctx** out);
void psms_destroy(psms_ctx* ctx);
const char* psms_last_error(const psms_ctx* ctx);
const char* psms_status_string(psms_status s);
/* Device bytes held by the context (gauge copies and workspaces). */
unsigned long long psms_device_bytes(const psms_ctx* ctx);

/* Uploads gauge field U into slot (0 <= slot < 64), converting it to the internal
 * layouts (FP64 and FP32 12-real). Returns PSMS_ENOTSU3 if some link deviates from
 * SU(3) by more than 1e-6: the FP64 copy is still loaded, mixed-precision operators
 * and solves then use FP32 copies of all 18 reals of each link (made on first use),
 * and the network and psms_apply_dw_noalloc in MIXED refuse the slot (PSMS_ENOTSU3).
 * PSMS_EINVAL if an entry is NaN or Inf (the slot is then left unloaded). */
psms_status psms_gauge_load(psms_ctx* ctx, int slot, const double* U);

/* out = D in (eq. Dw, rescaled), full lattice. prec MIXED applies the FP32 12-real
 * link, FP32 spinor kernel (input rounded to FP32); for a slot that is not SU(3), FP32
 * 18-real links. */
psms_status psms_apply_dw(psms_ctx* ctx, int slot, const double* in, double* out, int nrhs, psms_prec prec);

/* out = D in (eq. Dw, rescaled) with the operands of the mixed-precision inner solves:
 * FP32 12-real links, the input rounded to in_storage (FP32, or BF16 round-to-nearest-
 * even), arithmetic in FP32, the result stored in out_storage and returned as FP64.
 * Pairs: F32 -> F32, BF16 -> BF16, BF16 -> F32 (an FP32 input with a BF16 output is
 * PSMS_EINVAL). The stencil form is that of the context's tuning for the input
 * storage ("dslash_variant_f32" / "dslash_variant_bf16"); for a slot that is not
 * SU(3), FP32 18-real links and the one-lane form. */
psms_status psms_apply_dw_lowp(psms_ctx* ctx, int slot, const double* in, double* out, int nrhs,
                               psms_inner_storage in_storage, psms_inner_storage out_storage);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): psms_apply_dw without any
 * allocation and without synchronising. `in` and `out` must be device memory of the
 * context's device (PSMS_EINVAL otherwise); the work is only enqueued on the
 * context's stream. The two internal-layout fields live in a fixed device array of
 * 64 MiB that the library holds on every device it runs on until the process ends:
 * nrhs fields need 2 x nrhs x V x 192 bytes (F64) or 96 bytes (MIXED), and a larger
 * request is PSMS_EINVAL. All calls on one device share that array: calls that overlap
 * on one device (other streams, other threads, other contexts) race and must be
 * serialised by the caller. Results equal those of psms_apply_dw. MIXED needs a slot
 * holding SU(3) links (PSMS_ENOTSU3 otherwise: the FP32 18-real copies that other
 * calls make for such a slot would need an allocation). */
psms_status psms_apply_dw_noalloc(psms_ctx* ctx, int slot, const double* in, double* out, int nrhs, psms_prec prec);

/* Even-odd preconditioned operator on even sites: out_e = in_e - kappa^2 H_eo H_oe in_e
 * (the block-size-one case of eq. ddfactor). Odd sites of `in` are ignored, odd sites
 * of `out` are set to zero. */
psms_status psms_apply_dhat_ee(psms_ctx* ctx, int slot, const double* in, double* out, int nrhs);

/* out = D_bb in (colour 0) or D_ww in (colour 1): the block-diagonal part of D on the
 * blocks of that colour with Dirichlet block boundaries (eq. domdec). Sites of the
 * other colour are ignored in `in` and zero in `out`. */
psms_status psms_apply_block(psms_ctx* ctx, int slot, int colour, const double* in, double* out, int nrhs);

/* Inter-block hops (eq. domdec): from_colour 0 gives out = D_wb in (input on black
 * sites, output on white sites), from_colour 1 gives out = D_bw in. */
psms_status psms_apply_hop_bw(psms_ctx* ctx, int slot, int from_colour, const double* in, double* out, int nrhs);

/* out = P in: the orthogonal projector of Sec. 4.4 onto the boundary sites of the
 * black blocks ((1 + gamma_mu)/2 or (1 - gamma_mu)/2 where a site has a single
 * neighbour in another block, at +mu or -mu; identity with two or more; zero elsewhere). */
psms_status psms_apply_proj(psms_ctx* ctx, const double* in, double* out, int nrhs);

/* Solves D x = b (flexible GCR with the chosen right preconditioner; mixed precision
 * wraps FP32/BF16 inner solves in FP64 defect correction). x is an output only. */
psms_status psms_solve(psms_ctx* ctx, int slot, const double* b, double* x, int nrhs, const psms_solve_params* params,
                       psms_solve_stats* stats);

/* Solves D_bb x = b (colour 0) or D_ww x = b (colour 1) block by block to params->tol
 * relative residual per block (at most params->max_iter iterations). */
psms_status psms_solve_block(psms_ctx* ctx, int slot, int colour, const double* b, double* x, int nrhs,
                             const psms_solve_params* params, psms_solve_stats* stats);

/* out = (1 - P Q) in with Q = D_bb^-1 D_bw D_ww^-1 D_wb (eq. detschur); `in` must lie in
 * the range of P. Block inverses to params->tol. */
psms_status psms_apply_schur(psms_ctx* ctx, int slot, const double* in, double* out, int nrhs,
                             const psms_solve_params* params, psms_solve_stats* stats);

/* out = (1 - P Q)^-1 in = in - P [D^-1 (0 + D_wb in)]_black (eq. inverseschur): one
 * full-lattice solve per right-hand side. */
psms_status psms_apply_schur_inv(psms_ctx* ctx, int slot, const double* in, double* out, int nrhs,
                                 const psms_solve_params* params, psms_solve_stats* stats);

/* Stochastic estimator (eq. stacc, eq. Deltaistoch). For every proposal slot_Up[p] and
 * noise field eta_j: delta[p*nnoise + j] = |M xi_j|^2 - |xi_j|^2 with
 *   op FULL : M = D(U')^-1 D(U),                 xi_j = eta_j;
 *   op SCHUR: M = (1 - PQ(U'))^-1 (1 - PQ(U)),   xi_j = P eta_j.
 * noise holds nnoise fields with density exp(-|eta|^2).
 * n_interp = N > 1: gauge-field interpolation (Sec. 4.3) with the intermediate fields
 * U_i = ((N - i) U + i U') / N of eq. gfparam (no relative gauge fixing, g = 1) and
 * delta[p*nnoise + j] = sum_i (|M_i xi_ij|^2 - |xi_ij|^2), M_i = D(U_{i+1})^-1 D(U_i)
 * (eq. Mparam; the Schur complements for SCHUR), eq. staccN. noise then holds N groups
 * of nnoise fields, group i (fields i*nnoise .. i*nnoise + nnoise - 1) for factor i.
 * The intermediate fields are not SU(3): in MIXED their inner solves use FP32 18-real
 * links (FP64 outside, as always). They use two free gauge slots (PSMS_EINVAL when
 * fewer are free), which are free again on return.
 * SCHUR: the full solve inside (1 - PQ(U'))^-1 starts from the exact solution of the
 * same system with U, a by-product of applying (1 - PQ(U)); tol still refers to |b|.
 * delta may be host or device memory (nprop*nnoise doubles). */
psms_status psms_logdet_ratio(psms_ctx* ctx, psms_op op, int slot_U, const int* slot_Up, int nprop, const double* noise,
                              int nnoise, int n_interp, const psms_solve_params* params, double* delta,
                              psms_solve_stats* stats);

/* Relative gauge fixing of a field pair (Sec. 4.2, eqs. relgf, choiceg, matrixMgf;
 * App. B): the gauge transformation g, defined on the block-interior sites of the
 * context's blocks (no nearest neighbour in another block) and 1 elsewhere, that
 * minimises eq. relgf with g1 = g2^-1 = g, i.e. the distance (eq. sprodgf) between
 * U^g(x,mu) = g(x) U(x,mu) g(x+mu)^+ and U'^(g^-1)(x,mu) = g(x)^+ U'(x,mu) g(x+mu).
 * Since the link term depends on G = g^2 only, the steepest descent of App. B (eq. ming)
 * runs on G, fixing U' to U, with Delta of eq. GF:Delta on the current pair and the step
 * exp(alpha/2 C), C the traceless anti-Hermitian part of Delta - Delta^+ (the sign that
 * lowers eq. relgf); a step that raises eq. relgf is rejected and alpha lowered by 0.01
 * down to alpha_min, after which a rejected step ends the descent; the descent stops when
 * the mean of theta (eq. GF:theta, -Tr C^2) over the domain is below theta_tol, or after
 * max_iter steps. Then g = G^(1/2) (principal root), and U^g goes into slot_gU, U'^(g^-1)
 * into slot_gUp (both SU(3); usable as the end points of the interpolation of
 * psms_logdet_ratio, eq. gfparam). g_out (may be NULL, host or device): [V][3][3]
 * complex FP64. FP64 throughout. PSMS_EINVAL on a context with outer blocks. */
typedef struct {
  double alpha;      /* step scale (App. B: 0.15) */
  double alpha_min;  /* smallest step scale after rejections (0.10) */
  double theta_tol;  /* stop when the mean theta over the domain is below it (1e-3) */
  int max_iter;      /* steps tried at most (1000) */
} psms_gf_params;
typedef struct {
  int iterations;          /* steps tried */
  double functional_start; /* eq. sprodgf of (U, U') */
  double functional_end;   /* eq. sprodgf of (U^g, U'^(g^-1)) */
  double theta_end;        /* mean theta over the domain at the last check */
  double alpha_end;
} psms_gf_stats;
void psms_default_gf_params(psms_gf_params* p);
psms_status psms_relative_gauge_fix(psms_ctx* ctx, int slot_U, int slot_Up, const psms_gf_params* params, int slot_gU,
                                    int slot_gUp, double* g_out, psms_gf_stats* stats);

/* The block-Schur filter of the recursive decomposition (Sec. 3, eq. ddrec; the second
 * acceptance step of eq. 4step), on a context with outer blocks (geom.outer_b): for every
 * proposal p, noise field j and outer block B (lexicographic order of x // outer_b),
 *   delta[(p * nnoise + j) * nouter + B] = |(M xi_j)_B|^2 - |(xi_j)_B|^2,
 *   M = (1 - PQ(U'))^-1 (1 - PQ(U)),   xi_j = P eta_j,
 * with Q and P those of the outer blocks' Dirichlet operators over their sub-blocks b: the
 * stochastic estimator of det(Dhat_B(U')^+ Dhat_B(U')) / det(Dhat_B(U)^+ Dhat_B(U)) for each
 * outer block B at once (eq. Deltaistoch per block), since the operators are block-diagonal
 * over the outer blocks and each block sees its own part of the noise. Summed over B it is
 * what psms_logdet_ratio (SCHUR) gives on the same context. The full solve inside is judged
 * on the whole lattice: params->tol bounds |b - D x| / |b| over all outer blocks together.
 * delta: host or device memory, nprop * nnoise * nouter doubles. */
psms_status psms_logdet_ratio_blocks(psms_ctx* ctx, int slot_U, const int* slot_Up, int nprop, const double* noise,
                                     int nnoise, const psms_solve_params* params, double* delta, psms_solve_stats* stats);

/* The hierarchy of acceptance steps of one recursion level (Sec. 2, eq. hierarchy;
 * Sec. 3, eq. 4step; App. A.2, eq. paccstoch; App. C, eq. Si) for a proposal U -> U'
 * (slots slot_U, slot_Up, loaded in both contexts) that changes links inside the
 * smallest blocks only (PSMS_EINVAL otherwise). `in` has the smallest blocks b' as its
 * blocks and the blocks B as outer_b; `out` has B as its blocks (same lattice, kappa,
 * device and stream). Each step accepts when its uniform u in [0, 1) is below
 * exp(-Delta), i.e. with probability min{1, e^-Delta}, one Delta per decision:
 *  1) every b' separately: Delta1 = beta[0] dS1_b', dS1_b' = -2 (ln|det D_b'(U')| -
 *     ln|det D_b'(U)|) exactly (psms_block_logdet); U1 = U' in the accepted b', U elsewhere;
 *  2) every B separately: Delta2 = dS2_B + beta[1] sum_{b' in B, accepted} dS1_b', dS2_B the
 *     block-Schur estimator of U1 against U with noise field 0 (psms_logdet_ratio_blocks);
 *     U2 = U1 in the accepted B, U elsewhere;
 *  3) Delta3 = dS3 + beta[2] sum_{b' kept in U2} dS1_b', dS3 the Schur estimator of the
 *     blocks B (psms_logdet_ratio, SCHUR) of U2 against U with noise field 1;
 *     the new state is U2 when accepted, else U.
 * beta are the coefficients of the exactly computed block-determinant action at the three
 * steps (App. C); they must sum to 1. uniforms: nsmall + nouter + 1 values (steps 1, 2, 3;
 * blocks in lexicographic order); noise: 2 fields, density exp(-|eta|^2). The two work
 * slots are overwritten in both contexts; with slot_out >= 0 the new state is loaded there
 * in both contexts. The proposal step itself and any gauge-action terms are the caller's. */
typedef struct {
  double beta[3];              /* coefficients of the block-determinant action per step (1, 0, 0) */
  psms_solve_params solve;     /* the solves of steps 2 and 3 */
  int work_slot[2];            /* slots overwritten in both contexts (62, 63) */
  int slot_out;                /* -1: not loaded */
} psms_filter_params;
typedef struct {
  double* delta1;   /* [nsmall] or NULL */
  int* accept1;     /* [nsmall] or NULL */
  double* delta2;   /* [nouter] or NULL */
  int* accept2;     /* [nouter] or NULL */
  double delta3;
  int accept3;
  int inner_iters;  /* Krylov iterations of steps 2 and 3 */
} psms_filter_result;
void psms_default_filter_params(psms_filter_params* p);
psms_status psms_filter_step(psms_ctx* in, psms_ctx* out, int slot_U, int slot_Up, const psms_filter_params* params,
                             const double* uniforms, const double* noise, psms_filter_result* result);

/* Exact block determinants: the first acceptance step of eq. 4step (the block filter,
 * Sec. 3), whose determinants the paper computes exactly by LU for blocks of up to about
 * 6^4 points. For every gauge slot slots[s] and every block of the context's block
 * decomposition (blocks in lexicographic order of their coordinates x // b, direction 3
 * fastest):
 *   out[(s * nblk + k) * 2 + 0] = ln |det D_b|,  out[(s * nblk + k) * 2 + 1] = arg det D_b
 * (in [-pi, pi]; det D_b is real, so 0 or pi up to rounding), D_b the Dirichlet block
 * operator of eq. domdec. Computed as det(1 - kappa^2 H_eo H_oe) on the block's even sites
 * (D_b has unit even-even and odd-odd blocks), by a dense LU in FP64 without row exchanges.
 * The block filter's exponent is Delta_b = -2 (ln|det D_b(U')| - ln|det D_b(U)|).
 * Blocks of more than 1024 sites: PSMS_EINVAL. A pivot of modulus below 1e-8: PSMS_ENOTCONV
 * (the result is refused). out: host or device memory, nslot * nblk * 2 doubles. */
psms_status psms_block_logdet(psms_ctx* ctx, const int* slots, int nslot, double* out);

/* The estimate of the log-determinant ratio from the Deltas of psms_logdet_ratio
 * (Sec. 4.1, eq. stacc: the mean of e^-Delta over Gaussian noise is det(M^+ M)^-1):
 *   out[p] = ln( (1/nnoise) sum_j exp(-delta[p*nnoise + j]) ),   p < nprop.
 * Host arrays, FP64; the largest -delta of each row is factored out first, so large
 * |delta| neither overflow nor underflow. Needs no context. PSMS_EINVAL for null
 * pointers, nprop or nnoise < 1, or a non-finite delta. */
psms_status psms_log_ratio_estimate(const double* delta, int nprop, int nnoise, double* out);

/* ---- Learned preconditioner (not from the paper; wraps its solves) ----------------
 * A gauge-covariant linear network N with layers
 *   Psi_c(x) = sum_{t=0..8} sum_c' W[t][c][c'] (T_t Phi_c')(x),
 * T_0 = 1, T_{1+2mu} Phi(x) = U(x,mu) Phi(x+mu), T_{2+2mu} Phi(x) = U(x-mu,mu)^+ Phi(x-mu)
 * (with the boundary sign of the Dirac operator), W[t][c][c'] a complex 4x4 spin
 * matrix. Used as the right preconditioner of flexible GCR (params.pc = PSMS_PC_NET);
 * the true FP64 residual still decides convergence, so the results stay exact.
 * Weights: complex, layer by layer, each [9][c_out][c_in][4][4] (row-major spin
 * matrix), as interleaved (re, im) doubles at the boundary; FP32 on the device.
 * Links in the network are the 12-real FP32 copies, so the slot must hold SU(3) links. */
typedef struct {
  int npairs;            /* residual/correction pairs generated in total */
  int batch;             /* pairs per optimisation step */
  int epochs;            /* passes over each generated chunk */
  int chunk;             /* pairs generated (and held on the GPU) at a time */
  double lr;             /* Adam learning rate */
  double solve_tol;      /* relative residual of the solves that produce e = D^-1 r */
  unsigned long long seed;
  const char* ckpt_path; /* checkpoint file (weights + Adam state), may be NULL */
  int ckpt_every;        /* steps between checkpoints (0: only at the end) */
} psms_train_params;

typedef struct {
  double first_loss, final_loss; /* mean relative loss |N(r) - e|^2 / |e|^2 of the first and last step */
  int steps;
  double seconds_data, seconds_train;
} psms_train_stats;

/* Creates a network with channels[0..nlayers] (channels[0] = channels[nlayers] = 1,
 * every entry <= 8): weights N(0, scale^2 / (36 c_in)) plus the identity on the
 * channel-0, t = 0 path, so that the untrained network is close to N(r) = r. */
psms_status psms_net_init(psms_ctx* ctx, const int* channels, int nlayers, unsigned long long seed, double scale);
long long psms_net_num_weights(const psms_ctx* ctx); /* complex weights, 0 without a network */
psms_status psms_net_set_weights(psms_ctx* ctx, const double* w, long long n);
psms_status psms_net_get_weights(psms_ctx* ctx, double* w, long long n);
/* out = N(in) with the links of `slot`. */
psms_status psms_net_apply(psms_ctx* ctx, int slot, const double* in, double* out, int nrhs);
/* loss = sum_b |N(r_b) - e_b|^2 / |e_b|^2 and grad = dloss / dconj(W) (Wirtinger
 * convention, same layout as the weights); grad may be NULL. */
psms_status psms_net_loss_grad(psms_ctx* ctx, int slot, const double* r, const double* e, int npairs, double* loss,
                               double* grad);
void psms_default_train_params(psms_train_params* p);
/* Trains on pairs (r, e = D^-1 r): r Gaussian (counter-based generator), e from the
 * mixed-precision Schwarz-GCR solver, cycling over the gauge slots; Adam on the mean
 * relative loss; all on the GPU. */
psms_status psms_net_train(psms_ctx* ctx, const int* slots, int nconf, const psms_train_params* params,
                           psms_train_stats* stats);
psms_status psms_net_save(psms_ctx* ctx, const char* path);
psms_status psms_net_load(psms_ctx* ctx, const char* path);

/* Launch tuning of the context. Keys: "dslash_variant_f64", "dslash_variant_f32",
 * "dslash_variant_bf16" (full-lattice stencil form, 0..5: one lane or two wave groups
 * per site, times three register budgets; 6: four lanes per site; 7: one workgroup per
 * block of at most 256 sites with the block's input spinor in LDS; 8: as 7, with every
 * link read once per block and the backward hops passed between sites in LDS; 7 and 8
 * run other block sizes as 0),
 * "nr_f64", "nr_low" (right-hand sides per
 * stencil thread: 1, 2 or 4), "xcd_map" (1: each XCD sweeps a contiguous range of
 * tiles), "net_mfma" (1: network channel mixing on the matrix cores in bf16, 0: FP32 on
 * the vector units), "block_solver" (block inverses to tolerance: 0 minimal residual
 * per block, 1 flexible GCR on the block-diagonal operator) and "block_lanes" (block
 * solver for 256-site blocks with 12-real links: 1 or 2 lanes per site, 0 = two lanes
 * when the launch has fewer than two workgroups per compute unit) and "block_eo" (block
 * solver: 0 plain minimal residual; 1 minimal residual on the even-odd Schur complement of
 * each block, where an iteration counts as about two plain ones, 12-real links staged in
 * LDS; 3 the same with links read from L2 and Schwarz sweeps with block_iters/2 iterations
 * rounded up; 2, the default, as 3 with the links staged in LDS) and "block_eo_lanes" (even-odd block
 * solver on 256-site blocks in FP32 or BF16 storage: 2 or 4 lanes per site; 0, the
 * default, 4 when the launch has fewer workgroups than the GPU has compute units, else
 * 2; FP64 block solves always use 2) and "block_tol_prec" (block inverses to tolerance in
 * a mixed-precision solve with SU(3) links: 1 FP32 block passes inside FP64 defect
 * correction, 2 FP64 block solves, 0, the default, FP32 passes for blocks of more than
 * 256 sites and FP64 for smaller ones) and "sap_bf16" (mixed precision with a BF16 Krylov
 * basis: 1, the default, keeps the Schwarz preconditioner's residual, iterate and
 * corrections in BF16, 0 in FP32) and "block_xcd" (block-solver launches: 1 runs the
 * right-hand sides of one block back to back on one XCD, which then serves their link
 * reads from its L2, and gives each XCD a contiguous range of blocks; 0 the launch order;
 * 2, the default, 1 when the links the launch reads exceed the 256 MB Infinity Cache) and
 * "sap_link16" (mixed-precision Schwarz sweeps on 256-site blocks: 2, the default, stage
 * kappa times the whole links in LDS as FP16 and exchange the block's fields between
 * lanes in FP16, scaled to unit RMS per block, with the face update of 4^4 blocks spread
 * over all lanes; 1 stages the 12-real links in FP16 and exchanges FP32 fields; 0 stages
 * FP32 links; block inverses to a tolerance always use FP32 links).
 * Unknown keys or values give
 * PSMS_EINVAL. Results do not depend on the tuning beyond rounding; only speed does. */
psms_status psms_set_tuning(psms_ctx* ctx, const char* key, int value);
psms_status psms_get_tuning(psms_ctx* ctx, const char* key, int* value);

/* Autotuner: times every stencil form and right-hand-side blocking on this context's
 * geometry (in the solvers' layout when the Schwarz blocks differ from the domain blocks) (HIP events; the mean of repeated launches, best of three interleaved rounds
 * after a warm-up round). Stencil forms are timed on two launch shapes: gauge slot `slot`
 * with 16 right-hand sides (1 from 2^20 sites up), and every other loaded gauge slot as
 * the proposals of one launch (up to the proposals one launch addresses, SU(3) slots only
 * for the reduced-precision forms; `slot` itself when there is no other) with 128
 * right-hand sides in all (from 2^20 sites up 8 per proposal), on Gaussian inputs; BF16 forms also
 * into FP32 outputs at the second shape. Forms whose kernels spill registers to scratch
 * are skipped while any form does not. The
 * form kept is the one whose worst slowdown against the fastest form of either shape is
 * smallest. For the right-hand-side blocking the fastest is kept. If cache_path names a
 * JSON-lines file holding an entry for this GPU architecture and geometry, that entry is
 * used instead and nothing is timed; a fresh result is appended to the file. cache_path
 * may be NULL. Load the gauge fields before tuning. */
psms_status psms_autotune(psms_ctx* ctx, int slot, const char* cache_path);

/* Kernel timing with HIP events on the context's stream. enable=1 starts recording
 * the launches of the named kernel families ("dslash", "dslash_part", "block_mr" (Schwarz sweeps),
 * "block_solve" (block inverses to a tolerance), "blas", "net"),
 * 0 stops. psms_profile_read gives the total milliseconds, launch count and
 * algorithmic bytes moved since the last enable. */
psms_status psms_profile(psms_ctx* ctx, int enable);
psms_status psms_profile_read(psms_ctx* ctx, const char* family, double* total_ms, long long* launches,
                              double* algorithmic_bytes);

#ifdef __cplusplus
}
#endif
#endif /* PSMS_H */
